// HIP kernels (gfx950) of the thin-disk force pipeline.
//
//  k_ktable      exact cell-integrated kernels at every source offset (FP64)
//  k_row_fwd     real-to-complex row transforms of zero-padded fields,
//                written transposed (column-major spectra)
//  k_col         per spectral column: forward column transforms of the input
//                fields, products with the kernel spectra, inverse column
//                transforms of the force components
//  k_row_inv     complex-to-real row transforms of the force components
//  k_col_extract table spectra: forward column transform + quadrant store
//  k_inject      AMR: composite leaves -> finest lattice (linear density)
//  k_gather      AMR: finest-lattice forces -> composite leaf outputs
#include "kernels.hpp"

#include <cmath>

namespace grav {

// ---------------------------------------------------------------------------
// launch configurations
// ---------------------------------------------------------------------------

constexpr int cmin(int a, int b) { return a < b ? a : b; }
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int floor_pow2(int v) { return v < 2 ? 1 : 2 * floor_pow2(v / 2); }

// Row transforms: length L = M/2 complex (two real samples packed per
// element), E elements per thread, RPB rows per block.  Lanes are
// interleaved with the row index fastest, so one store instruction writes
// RPB consecutive rows of a spectral column (transposed, coalesced output).
template <typename T, int M> struct RowCfg {
    static constexpr int L = M / 2;
    static constexpr int E = (sizeof(T) == 4 && L >= 1024) ? 16 : 8;
    static constexpr int NTR = L / E;
    static constexpr int RMAX = sizeof(T) == 4 ? 8 : 4;
    static constexpr int REG = lds_region<L>();
    static constexpr int BYTES = REG * (int)sizeof(C<T>);
    // a power of two (rows per solve are powers of two), LDS kept <= 80 KB
    static constexpr int RPB = floor_pow2(cmax(1, cmin(RMAX, cmin(1024 / NTR, 81920 / BYTES))));
    static_assert((RPB & (RPB - 1)) == 0, "rows per block must be a power of two");
    static constexpr int NTH = RPB * NTR;
};

// Column transforms: length M, E elements per thread, one column per block.
template <typename T, int M> struct ColCfg {
    static constexpr int E = (sizeof(T) == 4 && M >= 2048) ? 16 : 8;
    static constexpr int NT = M / E;
};

// ---------------------------------------------------------------------------
// row forward: z[m] = x[2m] + i x[2m+1] -> Z = FFT_L(z) -> X[k], k in [0, L]
// ---------------------------------------------------------------------------
template <typename T, int M, bool PRUNED>
__global__ void __launch_bounds__((RowCfg<T, M>::NTH))
    k_row_fwd(RowFwdArgs<T> a, const C<T> *__restrict__ tw) {
    using CF = RowCfg<T, M>;
    constexpr int L = CF::L, E = CF::E, NTR = CF::NTR, RPB = CF::RPB;
    __shared__ C<T> lds[RPB * CF::REG];
    const int t = threadIdx.x;
    const int r = t % RPB, tr = t / RPB;
    const int f = blockIdx.y;
    const int64_t j = (int64_t)blockIdx.x * RPB + r;
    C<T> *my = lds + r * CF::REG;

    const C<T> *row = reinterpret_cast<const C<T> *>(a.in[f] + j * a.in_pitch);
    const T sc = a.scale[f];
    C<T> reg[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if (PRUNED && e >= E / 2) {
            reg[e] = mk<T>(0, 0);
        } else {
            C<T> v = row[tr + NTR * e];
            reg[e] = mk<T>(v.x * sc, v.y * sc);
        }
    }
    fft<T, L, NTR, -1>(reg, my, tw, 2, tr);

#pragma unroll
    for (int e = 0; e < E; ++e) my[pidx(tr + NTR * e)] = reg[e];
    __syncthreads();
    C<T> *dst = a.out + f * a.out_fstride + j;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = tr + NTR * e;
        const C<T> zk = reg[e];
        const C<T> zn = my[pidx((L - k) & (L - 1))];
        const C<T> w = tw[k];
        const T px = zk.x + zn.x, py = zk.y - zn.y;
        const T qx = zk.x - zn.x, qy = zk.y + zn.y;
        dst[(int64_t)k * a.out_pitch] =
            mk<T>((T)0.5 * (px + w.x * qy + w.y * qx), (T)0.5 * (py - w.x * qx + w.y * qy));
    }
    if (tr == 0) dst[(int64_t)L * a.out_pitch] = mk<T>(reg[0].x - reg[0].y, (T)0);
}

// ---------------------------------------------------------------------------
// column: for each input field, forward transform of the (zero-padded)
// column, product with the kernel spectra of both force components, then
// inverse transforms of the accumulated force spectra.
//
// Kernel spectra are stored as one real quadrant per kind (ky in [0, M/2]):
// kinds {x0, y0} are purely imaginary, the others real; a negative ky takes
// the kind's parity in y.  Corner-family spectra carry the phase
// exp(-i pi (kx + ky)/M) (targets half a cell from the source lattice),
// applied once to the accumulated sums.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int parity_y(int kind) {
    // x0 even, xx even, xy odd, y0 odd, yx odd, yy even (in y)
    return (kind == 2 || kind == 3 || kind == 4) ? -1 : 1;
}

template <typename T, int M, int NF, int NFAM>
__global__ void __launch_bounds__((ColCfg<T, M>::NT))
    k_col(ColArgs<T> a, const C<T> *__restrict__ tw, const C<T> *__restrict__ ph) {
    constexpr int E = ColCfg<T, M>::E, NT = ColCfg<T, M>::NT, H = M / 2;
    __shared__ C<T> lds[lds_region<M>()];
    const int t = threadIdx.x;
    const int kx = blockIdx.x;

    C<T> acc[2 * NFAM][E];
#pragma unroll
    for (int g = 0; g < 2 * NFAM; ++g)
#pragma unroll
        for (int e = 0; e < E; ++e) acc[g][e] = mk<T>(0, 0);

#pragma unroll
    for (int f = 0; f < NF; ++f) {
        C<T> reg[E];
        const C<T> *src = a.in + f * a.in_fstride + (int64_t)kx * a.in_pitch;
#pragma unroll
        for (int e = 0; e < E; ++e) reg[e] = (e < E / 2) ? src[t + NT * e] : mk<T>(0, 0);
        fft<T, M, NT, -1>(reg, lds, tw, 1, t);
#pragma unroll
        for (int fam = 0; fam < NFAM; ++fam) {
            const T *qx = a.q[fam] + f * a.q_kstride + (int64_t)kx * a.q_pitch;
            const T *qy = a.q[fam] + (3 + f) * a.q_kstride + (int64_t)kx * a.q_pitch;
            const T sx = (T)parity_y(f), sy = (T)parity_y(3 + f);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int ky = t + NT * e;
                const bool neg = ky > H;
                const int kq = neg ? M - ky : ky;
                T vx = qx[kq], vy = qy[kq];
                if (neg) {
                    vx *= sx;
                    vy *= sy;
                }
                const C<T> X = reg[e];
                if (f == 0) {  // imaginary spectra: X * (i v)
                    acc[2 * fam][e].x -= X.y * vx;
                    acc[2 * fam][e].y += X.x * vx;
                    acc[2 * fam + 1][e].x -= X.y * vy;
                    acc[2 * fam + 1][e].y += X.x * vy;
                } else {
                    acc[2 * fam][e].x += X.x * vx;
                    acc[2 * fam][e].y += X.y * vx;
                    acc[2 * fam + 1][e].x += X.x * vy;
                    acc[2 * fam + 1][e].y += X.y * vy;
                }
            }
        }
    }
    if constexpr (NFAM == 2) {
        const C<T> px = ph[kx];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int ky = t + NT * e;
            const C<T> py = ky <= H ? ph[ky] : cconj<T>(ph[M - ky]);
            const C<T> p = cmul<T>(px, py);
            acc[2][e] = cmul<T>(acc[2][e], p);
            acc[3][e] = cmul<T>(acc[3][e], p);
        }
    }
#pragma unroll
    for (int g = 0; g < 2 * NFAM; ++g) {
        fft<T, M, NT, +1>(acc[g], lds, tw, 1, t);
        C<T> *dst = a.out + g * a.out_gstride + (int64_t)kx * a.out_pitch;
#pragma unroll
        for (int e = 0; e < E / 2; ++e) dst[t + NT * e] = acc[g][e];
    }
}

// ---------------------------------------------------------------------------
// row inverse: Y[k], k in [0, L] (Hermitian half) -> y[n], n < M/2, scaled
// ---------------------------------------------------------------------------
template <typename T, int M>
__global__ void __launch_bounds__((RowCfg<T, M>::NTH))
    k_row_inv(RowInvArgs<T> a, const C<T> *__restrict__ tw) {
    using CF = RowCfg<T, M>;
    constexpr int L = CF::L, E = CF::E, NTR = CF::NTR, RPB = CF::RPB;
    __shared__ C<T> lds[RPB * CF::REG];
    const int t = threadIdx.x;
    const int r = t % RPB, tr = t / RPB;
    const int g = blockIdx.y;
    const int64_t j = (int64_t)blockIdx.x * RPB + r;
    C<T> *my = lds + r * CF::REG;

    const C<T> *src = a.in + g * a.in_gstride + j;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = tr + NTR * e;
        my[pidx(k)] = src[(int64_t)k * a.in_pitch];
    }
    if (tr == 0) my[pidx(L)] = src[(int64_t)L * a.in_pitch];
    __syncthreads();
    C<T> reg[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = tr + NTR * e;
        C<T> yk = my[pidx(k)];
        C<T> yn = my[pidx(L - k)];
        if (k == 0) {  // Y[0] and Y[L] of a real signal are real
            yk.y = 0;
            yn.y = 0;
        }
        const C<T> ze = mk<T>(yk.x + yn.x, yk.y - yn.y);
        const C<T> zo = cmulc<T>(mk<T>(yk.x - yn.x, yk.y + yn.y), tw[k]);
        reg[e] = mk<T>(ze.x - zo.y, ze.y + zo.x);
    }
    __syncthreads();
    fft<T, L, NTR, +1>(reg, my, tw, 2, tr);
    C<T> *dst = reinterpret_cast<C<T> *>(a.out[g] + j * a.out_pitch);
    const T sc = a.scale;
#pragma unroll
    for (int e = 0; e < E / 2; ++e) dst[tr + NTR * e] = mk<T>(reg[e].x * sc, reg[e].y * sc);
}

// ---------------------------------------------------------------------------
// kernel tables (double precision, cell units)
// ---------------------------------------------------------------------------

// ln(a + sqrt(a^2 + b^2)); b == 0 uses the x-bar = x convention sgn(a) ln|a|;
// a < 0 uses ln(b^2 / (R - a)) (no cancellation).
__device__ double lam(double a, double b) {
    if (b == 0.0) return a > 0.0 ? log(a) : -log(-a);
    const double R = sqrt(a * a + b * b);
    if (a >= 0.0) return log(a + R);
    return log((b * b) / (R - a));
}
__device__ double vlam(double v, double u) { return v == 0.0 ? 0.0 : v * lam(u, v); }
__device__ double rad(double u, double v) { return sqrt(u * u + v * v); }

// Exact kernel `kind` of the unit source cell [u1,u2] x [v1,v2] (offsets
// from the target) whose centre is (uc, vc); t0zero: the target touches the
// cell at a corner, where K^{x,0} and K^{y,0} are replaced by 0 (their
// divergent parts cancel against the adjacent cells of the same zone).
__device__ double closed_kernel(int kind, double uc, double vc, bool t0zero) {
    const double u1 = uc - 0.5, u2 = uc + 0.5, v1 = vc - 0.5, v2 = vc + 0.5;
    const double dxc = -uc, dyc = -vc;  // x_t - x_c, y_t - y_c
    if (kind < 3) {
        double k0 = 0.0;
        if (!t0zero) k0 = -((lam(v2, u2) - lam(v2, u1)) - (lam(v1, u2) - lam(v1, u1)));
        if (kind == 0) return k0;
        if (kind == 1) return dxc * k0 + ((vlam(v2, u2) - vlam(v2, u1)) - (vlam(v1, u2) - vlam(v1, u1)));
        return dyc * k0 - ((rad(u2, v2) - rad(u1, v2)) - (rad(u2, v1) - rad(u1, v1)));
    } else {
        double k0 = 0.0;
        if (!t0zero) k0 = -((lam(u2, v2) - lam(u2, v1)) - (lam(u1, v2) - lam(u1, v1)));
        if (kind == 3) return k0;
        if (kind == 4) return dxc * k0 - ((rad(v2, u2) - rad(v1, u2)) - (rad(v2, u1) - rad(v1, u1)));
        return dyc * k0 + ((vlam(u2, v2) - vlam(u2, v1)) - (vlam(u1, v2) - vlam(u1, v1)));
    }
}

// The same integral by a 10 x 10 Gauss-Legendre rule, used for cells at
// least 3.5 cells from the target: there the integrand is analytic in a
// Bernstein ellipse of parameter >= 15 about the cell, so the rule's error
// is below 1e-23 relative, while the closed form's double difference would
// cancel ~2 log10(distance) digits.
__device__ double quad_kernel(int kind, double uc, double vc, const TableArgs &a) {
    double sum = 0.0;
    for (int i = 0; i < 10; ++i) {
        const double du = 0.5 * a.glx[i];
        const double u = uc + du;
        double si = 0.0;
        for (int jj = 0; jj < 10; ++jj) {
            const double dv = 0.5 * a.glx[jj];
            const double v = vc + dv;
            const double r2 = u * u + v * v;
            const double ir = 1.0 / sqrt(r2);
            const double ir3 = ir * ir * ir;
            double f;
            switch (kind) {
                case 0: f = u; break;
                case 1: f = du * u; break;
                case 2: f = dv * u; break;
                case 3: f = v; break;
                case 4: f = du * v; break;
                default: f = dv * v; break;
            }
            si += a.glw[jj] * f * ir3;
        }
        sum += a.glw[i] * si;
    }
    return 0.25 * sum;
}

// Circulant table c[m] = K(-m): entry (my, mx) holds the kernel of the source
// cell at offset d = -(signed m) from the target.  Family 0 (cell-centre
// targets): cell [d - 1/2, d + 1/2], |d| <= M/2 - 1, the rest zero.
// Family 1 (targets on lattice corners): cell [d, d + 1], d in [-M/2, M/2 - 1].
__global__ void __launch_bounds__(256) k_ktable(TableArgs a) {
    const int64_t total = (int64_t)a.M * a.M;
    const int H = a.M / 2;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int mx = (int)(q % a.M), my = (int)(q / a.M);
        double val = 0.0;
        int sx, sy;
        if (a.family == 0) {
            sx = mx < H ? mx : mx - a.M;
            sy = my < H ? my : my - a.M;
        } else {
            sx = mx <= H ? mx : mx - a.M;
            sy = my <= H ? my : my - a.M;
        }
        const int dx = -sx, dy = -sy;
        bool valid = true;
        if (a.family == 0) valid = (mx != H) && (my != H);
        if (valid) {
            const double off = a.family == 0 ? 0.0 : 0.5;
            const double uc = dx + off, vc = dy + off;
            const double distx = fmax(fabs(uc) - 0.5, 0.0), disty = fmax(fabs(vc) - 0.5, 0.0);
            if (fmax(distx, disty) >= 3.5) {
                val = quad_kernel(a.kind, uc, vc, a);
            } else {
                const bool t0zero = a.family == 1 && (dx == 0 || dx == -1) && (dy == 0 || dy == -1);
                val = closed_kernel(a.kind, uc, vc, t0zero);
            }
        }
        a.out[q] = val;
    }
}

template <typename TQ, int M>
__global__ void __launch_bounds__((ColCfg<double, M>::NT))
    k_col_extract(const C<double> *__restrict__ in, TQ *__restrict__ q, int64_t q_pitch, int imag,
                  int corner, const C<double> *__restrict__ tw, const C<double> *__restrict__ ph) {
    constexpr int E = ColCfg<double, M>::E, NT = ColCfg<double, M>::NT, H = M / 2;
    __shared__ C<double> lds[lds_region<M>()];
    const int t = threadIdx.x;
    const int kx = blockIdx.x;
    const C<double> *src = in + (int64_t)kx * M;
    C<double> reg[E];
#pragma unroll
    for (int e = 0; e < E; ++e) reg[e] = src[t + NT * e];
    fft<double, M, NT, -1>(reg, lds, tw, 1, t);
    TQ *dst = q + (int64_t)kx * q_pitch;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int ky = t + NT * e;
        if (ky <= H) {
            C<double> v = reg[e];
            if (corner) v = cmulc<double>(v, cmul<double>(ph[kx], ph[ky]));
            dst[ky] = (TQ)(imag ? v.y : v.x);
        }
    }
}

// ---------------------------------------------------------------------------
// AMR injection and gather
// ---------------------------------------------------------------------------
template <typename T> __global__ void __launch_bounds__(256) k_inject(InjectArgs<T> a) {
    const int64_t n2 = (int64_t)a.nf * a.nf;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n2) return;
    const int I = (int)(idx % a.nf), J = (int)(idx / a.nf);
    const int32_t o = a.owner[idx];
    const int32_t c = o & 0x0FFFFFFF;
    const int kb = (o >> 28) & 0xF;
    const int B = 1 << kb;
    T s = a.s[c];
    T dx = 0, dy = 0;
    if (a.slopes) {
        dx = a.dx[c];
        dy = a.dy[c];
        // offset of this finest cell's centre from the leaf centre
        const T ox = (T)(2 * (I & (B - 1)) + 1 - B) * (T)0.5 * a.hf;
        const T oy = (T)(2 * (J & (B - 1)) + 1 - B) * (T)0.5 * a.hf;
        s = s + dx * ox + dy * oy;
    }
    a.w0[idx] = s;
    if (a.slopes) {
        a.w1[idx] = dx;
        a.w2[idx] = dy;
    }
}

template <typename T> __global__ void __launch_bounds__(256) k_gather(GatherArgs<T> a) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n) return;
    const int32_t m = a.gmap[c];
    if (m < 0) {
        a.fx[c] = 0;
        a.fy[c] = 0;
        return;
    }
    const int fam = (m >> 30) & 1;
    const int32_t pos = m & 0x3FFFFFFF;
    a.fx[c] = a.o[2 * fam][pos];
    a.fy[c] = a.o[2 * fam + 1][pos];
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

template <typename T, int M> struct Dispatch {
    static hipError_t row_fwd(const RowFwdArgs<T> &a, bool pruned, int nrows, int nfields,
                              const C<T> *tw, hipStream_t s) {
        using CF = RowCfg<T, M>;
        if (nrows % CF::RPB) return hipErrorInvalidValue;
        dim3 grid(nrows / CF::RPB, nfields);
        if (pruned)
            hipLaunchKernelGGL((k_row_fwd<T, M, true>), grid, dim3(CF::NTH), 0, s, a, tw);
        else
            hipLaunchKernelGGL((k_row_fwd<T, M, false>), grid, dim3(CF::NTH), 0, s, a, tw);
        return hipGetLastError();
    }
    static hipError_t col(const ColArgs<T> &a, int nfields, int nfam, const C<T> *tw,
                          const C<T> *ph, hipStream_t s) {
        dim3 grid(M / 2 + 1);
        dim3 block(ColCfg<T, M>::NT);
        if (nfields == 3 && nfam == 1)
            hipLaunchKernelGGL((k_col<T, M, 3, 1>), grid, block, 0, s, a, tw, ph);
        else if (nfields == 3 && nfam == 2)
            hipLaunchKernelGGL((k_col<T, M, 3, 2>), grid, block, 0, s, a, tw, ph);
        else if (nfields == 1 && nfam == 1)
            hipLaunchKernelGGL((k_col<T, M, 1, 1>), grid, block, 0, s, a, tw, ph);
        else if (nfields == 1 && nfam == 2)
            hipLaunchKernelGGL((k_col<T, M, 1, 2>), grid, block, 0, s, a, tw, ph);
        else
            return hipErrorInvalidValue;
        return hipGetLastError();
    }
    static hipError_t row_inv(const RowInvArgs<T> &a, int nrows, int nout, const C<T> *tw,
                              hipStream_t s) {
        using CF = RowCfg<T, M>;
        if (nrows % CF::RPB) return hipErrorInvalidValue;
        dim3 grid(nrows / CF::RPB, nout);
        hipLaunchKernelGGL((k_row_inv<T, M>), grid, dim3(CF::NTH), 0, s, a, tw);
        return hipGetLastError();
    }
};

template <typename TQ, int M>
static hipError_t col_extract_m(const C<double> *in, TQ *q, int64_t q_pitch, int imag, int corner,
                                const C<double> *tw, const C<double> *ph, hipStream_t s) {
    hipLaunchKernelGGL((k_col_extract<TQ, M>), dim3(M / 2 + 1), dim3(ColCfg<double, M>::NT), 0, s,
                       in, q, q_pitch, imag, corner, tw, ph);
    return hipGetLastError();
}

#define GRAV_SWITCH_M(M, ...)                             \
    switch (M) {                                          \
        case 32: { constexpr int MM = 32; __VA_ARGS__; }         \
        case 64: { constexpr int MM = 64; __VA_ARGS__; }         \
        case 128: { constexpr int MM = 128; __VA_ARGS__; }       \
        case 256: { constexpr int MM = 256; __VA_ARGS__; }       \
        case 512: { constexpr int MM = 512; __VA_ARGS__; }       \
        case 1024: { constexpr int MM = 1024; __VA_ARGS__; }     \
        case 2048: { constexpr int MM = 2048; __VA_ARGS__; }     \
        case 4096: { constexpr int MM = 4096; __VA_ARGS__; }     \
        case 8192: { constexpr int MM = 8192; __VA_ARGS__; }     \
        default: return hipErrorInvalidValue;             \
    }

template <typename T> static int row_threads_t(int M) {
    GRAV_SWITCH_M(M, return RowCfg<T, MM>::NTH)
}
template <typename T> static int row_rpb_t(int M) { GRAV_SWITCH_M(M, return RowCfg<T, MM>::RPB) }
template <typename T> static int col_threads_t(int M) { GRAV_SWITCH_M(M, return ColCfg<T, MM>::NT) }

int row_threads(int prec, int M) { return prec ? row_threads_t<double>(M) : row_threads_t<float>(M); }
int row_rows_per_block(int prec, int M) { return prec ? row_rpb_t<double>(M) : row_rpb_t<float>(M); }
int col_threads(int prec, int M) { return prec ? col_threads_t<double>(M) : col_threads_t<float>(M); }

template <typename T>
hipError_t launch_row_fwd(const RowFwdArgs<T> &a, int M, bool pruned, int nrows, int nfields,
                          const C<T> *tw, hipStream_t s) {
    GRAV_SWITCH_M(M, return (Dispatch<T, MM>::row_fwd(a, pruned, nrows, nfields, tw, s)))
}
template <typename T>
hipError_t launch_col(const ColArgs<T> &a, int M, int nfields, int nfam, const C<T> *tw,
                      const C<T> *ph, hipStream_t s) {
    GRAV_SWITCH_M(M, return (Dispatch<T, MM>::col(a, nfields, nfam, tw, ph, s)))
}
template <typename T>
hipError_t launch_row_inv(const RowInvArgs<T> &a, int M, int nrows, int nout, const C<T> *tw,
                          hipStream_t s) {
    GRAV_SWITCH_M(M, return (Dispatch<T, MM>::row_inv(a, nrows, nout, tw, s)))
}
template <typename T> hipError_t launch_inject(const InjectArgs<T> &a, hipStream_t s) {
    const int64_t n2 = (int64_t)a.nf * a.nf;
    hipLaunchKernelGGL((k_inject<T>), dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}
template <typename T> hipError_t launch_gather(const GatherArgs<T> &a, hipStream_t s) {
    hipLaunchKernelGGL((k_gather<T>), dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_ktable(const TableArgs &a, hipStream_t s) {
    const int64_t total = (int64_t)a.M * a.M;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_ktable, dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}
template <typename TQ>
hipError_t launch_col_extract(const C<double> *in, int M, TQ *q, int64_t q_pitch, int imag,
                              int corner, const C<double> *tw, const C<double> *ph,
                              hipStream_t s) {
    GRAV_SWITCH_M(M, return (col_extract_m<TQ, MM>(in, q, q_pitch, imag, corner, tw, ph, s)))
}

template hipError_t launch_row_fwd<float>(const RowFwdArgs<float> &, int, bool, int, int,
                                          const C<float> *, hipStream_t);
template hipError_t launch_row_fwd<double>(const RowFwdArgs<double> &, int, bool, int, int,
                                           const C<double> *, hipStream_t);
template hipError_t launch_col<float>(const ColArgs<float> &, int, int, int, const C<float> *,
                                      const C<float> *, hipStream_t);
template hipError_t launch_col<double>(const ColArgs<double> &, int, int, int, const C<double> *,
                                       const C<double> *, hipStream_t);
template hipError_t launch_row_inv<float>(const RowInvArgs<float> &, int, int, int,
                                          const C<float> *, hipStream_t);
template hipError_t launch_row_inv<double>(const RowInvArgs<double> &, int, int, int,
                                           const C<double> *, hipStream_t);
template hipError_t launch_inject<float>(const InjectArgs<float> &, hipStream_t);
template hipError_t launch_inject<double>(const InjectArgs<double> &, hipStream_t);
template hipError_t launch_gather<float>(const GatherArgs<float> &, hipStream_t);
template hipError_t launch_gather<double>(const GatherArgs<double> &, hipStream_t);
template hipError_t launch_col_extract<float>(const C<double> *, int, float *, int64_t, int, int,
                                              const C<double> *, const C<double> *, hipStream_t);
template hipError_t launch_col_extract<double>(const C<double> *, int, double *, int64_t, int, int,
                                               const C<double> *, const C<double> *, hipStream_t);

}  // namespace grav
