// Auxiliary kernels: kernel tables and their spectra (plan time) and the AMR
// gather (the AMR injection is fused into the row transform's load).
//
//  k_ktable      exact cell-integrated kernels at every source offset (FP64)
//  k_col_extract forward column transform of a table's row spectra and
//                storage of one real half plane (ky in [0, M/2])
//  k_gather      AMR: finest-lattice forces -> composite leaf outputs
#include "kernels_impl.hpp"

#include <cmath>

namespace grav {

// Column transforms of the table spectra: length M, 8 elements per thread.
template <int M> struct ExtractCfg {
    static constexpr int E = 8;
    static constexpr int NT = M / E;
};

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

// Off-plane targets (height zc != 0 above the disk, in cells): the nine
// kernels from the defining integrals with R = sqrt(u^2 + v^2 + zc^2),
// a = |zc|:  K^{x,0} = -DD[ln(v + R)], I_uu = DD[v ln(u + R) - a atan(uv/(aR))],
// I_uv = -DD[R], J = DD[atan(uv/(aR))]/a, K^{z,0} = -zc J, and
// K^{.,x} = (x_t - x_c) K^{.,0} + ..., K^{z,x} = (x_t - x_c) K^{z,0} - zc K^{x,0}
// (y family by symmetry).  ln(b + R) for b < 0 uses ln((R^2 - b^2)/(R - b)).
__device__ double lnz(double b, double c, double a2) {
    const double R = sqrt(b * b + c * c + a2);
    return b >= 0.0 ? log(b + R) : log((c * c + a2) / (R - b));
}
__device__ double closed_kernel_z(int kind, double uc, double vc, double zc) {
    const double us[2] = {uc - 0.5, uc + 0.5}, vs[2] = {vc - 0.5, vc + 0.5};
    const double a = fabs(zc), a2 = a * a;
    const double dxc = -uc, dyc = -vc;  // x_t - x_c, y_t - y_c
    double kx0 = 0, ky0 = 0, iuu = 0, ivv = 0, iuv = 0, jj = 0;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            const double sg = ((i + j) & 1) ? -1.0 : 1.0;
            const double u = us[i], v = vs[j];
            const double R = sqrt(u * u + v * v + a2);
            const double at = atan(u * v / (a * R));
            kx0 -= sg * lnz(v, u, a2);
            ky0 -= sg * lnz(u, v, a2);
            iuu += sg * (v * lnz(u, v, a2) - a * at);
            ivv += sg * (u * lnz(v, u, a2) - a * at);
            iuv -= sg * R;
            jj += sg * at;
        }
    const double kz0 = -zc * jj / a;
    switch (kind) {
        case 0: return kx0;
        case 1: return dxc * kx0 + iuu;
        case 2: return dyc * kx0 + iuv;
        case 3: return ky0;
        case 4: return dxc * ky0 + iuv;
        case 5: return dyc * ky0 + ivv;
        case 6: return kz0;
        case 7: return dxc * kz0 - zc * kx0;
        default: return dyc * kz0 - zc * ky0;
    }
}

// The same integral by an N x N Gauss-Legendre rule, used for cells at
// least 3.5 cells from the target, where the closed form's double difference
// would cancel ~2 log10(distance) digits.  At distance D (cells, from the
// cell's nearest edge) the integrand is analytic in a Bernstein ellipse of
// parameter rho ~ 4 D about the cell, and the rule's relative error is about
// rho^(-2N): the order falls with distance, 10 points below 8 cells, 8 below
// 24, 6 below 128 and 4 beyond, each below 1e-22 relative (1e-19 for the
// first-moment kinds, whose integral is ~1/D smaller than their integrand).
template <int N>
__device__ double quad_kernel(int kind, double uc, double vc, double zc, const double *gx,
                              const double *gw) {
    double sum = 0.0;
    for (int i = 0; i < N; ++i) {
        const double du = 0.5 * gx[i];
        const double u = uc + du;
        double si = 0.0;
        for (int jj = 0; jj < N; ++jj) {
            const double dv = 0.5 * gx[jj];
            const double v = vc + dv;
            const double r2 = u * u + v * v + zc * zc;
            const double ir = 1.0 / sqrt(r2);
            const double ir3 = ir * ir * ir;
            double f;
            switch (kind) {
                case 0: f = u; break;
                case 1: f = du * u; break;
                case 2: f = dv * u; break;
                case 3: f = v; break;
                case 4: f = du * v; break;
                case 5: f = dv * v; break;
                case 6: f = -zc; break;
                case 7: f = -zc * du; break;
                default: f = -zc * dv; break;
            }
            si += gw[jj] * f * ir3;
        }
        sum += gw[i] * si;
    }
    return 0.25 * sum;
}

// Table c[m] = K(-m): entry (my, mx) holds the kernel of the source cell at
// offset d = -(signed m) from the target.  Family 0 (cell-centre targets):
// cell [d - 1/2, d + 1/2], |d| <= M/2 - 1, the rest zero.  Family 1 (targets
// on lattice corners): cell [d, d + 1], d in [-M/2, M/2 - 1].  Circulant in
// y; negacyclic in x (entries of negative signed mx, mx > M/2, negated), the
// embedding whose odd-frequency transform turns the product of spectra into
// the same linear convolution.
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
            const double dist = fmax(distx, disty);
            if (dist >= 128.0) {
                val = quad_kernel<4>(a.kind, uc, vc, a.zc, a.glx4, a.glw4);
            } else if (dist >= 24.0) {
                val = quad_kernel<6>(a.kind, uc, vc, a.zc, a.glx6, a.glw6);
            } else if (dist >= 8.0) {
                val = quad_kernel<8>(a.kind, uc, vc, a.zc, a.glx8, a.glw8);
            } else if (dist >= 3.5) {
                val = quad_kernel<10>(a.kind, uc, vc, a.zc, a.glx, a.glw);
            } else if (a.zc != 0.0) {
                val = closed_kernel_z(a.kind, uc, vc, a.zc);
            } else {
                const bool t0zero = a.family == 1 && (dx == 0 || dx == -1) && (dy == 0 || dy == -1);
                val = closed_kernel(a.kind, uc, vc, t0zero);
            }
        }
        a.out[q] = mx > H ? -val : val;
    }
}

template <typename TQ, int M>
__global__ void __launch_bounds__((ExtractCfg<M>::NT))
    k_col_extract(const C<double> *__restrict__ in, TQ *__restrict__ q, int64_t q_pitch, int imag,
                  int corner, const C<double> *__restrict__ tw, const C<double> *__restrict__ ph) {
    constexpr int E = ExtractCfg<M>::E, NT = ExtractCfg<M>::NT, H = M / 2;
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
            if (corner) v = cmulc<double>(v, cmul<double>(ph[H + 1 + kx], ph[ky]));
            dst[ky] = (TQ)(imag ? v.y : v.x);
        }
    }
}

// ---------------------------------------------------------------------------
// AMR gather
// ---------------------------------------------------------------------------
template <typename T> __global__ void __launch_bounds__(256) k_gather(Pack<GatherArgs<T>> pk) {
    const GatherArgs<T> &a = pk.a[blockIdx.z];
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n) return;
    const int32_t m = a.gmap[c];
    if (m < 0) {
        a.fx[c] = 0;
        a.fy[c] = 0;
        if (a.ncomp == 3) a.fz[c] = 0;
        return;
    }
    const int fam = (m >> 30) & 1;
    const int32_t pos = m & 0x3FFFFFFF;
    a.fx[c] = a.o[a.ncomp * fam][pos];
    a.fy[c] = a.o[a.ncomp * fam + 1][pos];
    if (a.ncomp == 3) a.fz[c] = a.o[3 * fam + 2][pos];
}

// ---------------------------------------------------------------------------
// nested-correction AMR
// ---------------------------------------------------------------------------
// composite inputs -> working copy (absent slopes read as 0), plus one zero
// cell at index n that region cells outside the domain point to
template <typename T>
__global__ void __launch_bounds__(256) k_nest_copy_in(const T *s, const T *dx, const T *dy, T *rs, T *rdx,
                                                      T *rdy, int64_t n) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c > n) return;
    if (c == n) {
        rs[c] = 0;
        rdx[c] = 0;
        rdy[c] = 0;
        return;
    }
    rs[c] = s[c];
    rdx[c] = dx ? dx[c] : (T)0;
    rdy[c] = dy ? dy[c] : (T)0;
}

// The linear density of least-squares distance to four children's linear
// pieces: mean value, and slopes 3/(4h) (right - left children sum) plus the
// mean child slope / 4; conserves mass and both first moments (Section 2's
// zone integrals of a first-order Taylor density).
template <typename T> __global__ void __launch_bounds__(256) k_nest_restrict(RestrictArgs<T> a) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.n) return;
    const int32_t *q = a.ent + 5 * e;
    const int32_t p = q[0], c00 = q[1], c10 = q[2], c01 = q[3], c11 = q[4];
    const double s00 = a.s[c00], s10 = a.s[c10], s01 = a.s[c01], s11 = a.s[c11];
    const double k = 3.0 / (4.0 * a.h);
    const double gx = (double)a.dx[c00] + (double)a.dx[c01] + (double)a.dx[c10] + (double)a.dx[c11];
    const double gy = (double)a.dy[c00] + (double)a.dy[c01] + (double)a.dy[c10] + (double)a.dy[c11];
    a.s[p] = (T)((s00 + s10 + s01 + s11) / 4.0);
    a.dx[p] = (T)(k * ((s10 + s11) - (s00 + s01)) + gx / 16.0);
    a.dy[p] = (T)(k * ((s01 + s11) - (s00 + s10)) + gy / 16.0);
}

template <typename T>
__global__ void __launch_bounds__(256) k_nest_lift(const T *fx, const T *fy, double *accx, double *accy,
                                                   int64_t n) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    accx[c] = (double)fx[c];
    accy[c] = (double)fy[c];
}

// Interpolation of a parent-level field to a child centre a quarter parent
// cell from parent (I, J) towards (sx, sy), from the available parent-level
// cells: biquadratic on the 3 x 3 block if all of it exists; else bilinear,
// planar, linear in x, linear in y, or the parent's own value, each tried
// with the neighbour directions (sx, sy), (-sx, sy), (sx, -sy), (-sx, -sy)
// in that order.  av(a, b) tells whether parent (I + a, J + b) exists.
// Writes up to 9 (a, b, weight) and returns the count.
// The far-field stencil of a cell, in coordinates turned by its parity: the
// parent's neighbour (p sx, q sy), p, q in {-1, 0, 1}, lies towards the cell
// for p = 1 (q = 1).  The first form whose points are all available wins:
// biquadratic over the 3x3 block, else bilinear over a quadrant (ex, ey),
// planar over (ex, 0) and (0, ey), linear along x or y, the parent alone.
// Only scalars (kind, ex, ey) are kept: weights are formed per point.
struct NestStencil {
    int kind;  // 0 biquadratic, 1 bilinear, 2 planar, 3 linear in x, 4 linear in y, 5 parent
    int ex, ey;
    // weight of point (p, q), or false if the stencil does not use it
    __device__ __forceinline__ bool weight(int p, int q, double &w) const {
        const double al = ex / 4.0, be = ey / 4.0;
        switch (kind) {
            case 0: {
                const double wx = p == 0 ? 15.0 / 16.0 : (p == 1 ? 5.0 / 32.0 : -3.0 / 32.0);
                const double wy = q == 0 ? 15.0 / 16.0 : (q == 1 ? 5.0 / 32.0 : -3.0 / 32.0);
                w = wx * wy;
                return true;
            }
            case 1:
                if ((p != 0 && p != ex) || (q != 0 && q != ey)) return false;
                w = (p == 0 ? 1 - al : al) * (q == 0 ? 1 - be : be);
                return true;
            case 2:
                if (p == 0 && q == 0) w = 1 - al - be;
                else if (p == ex && q == 0) w = al;
                else if (p == 0 && q == ey) w = be;
                else return false;
                return true;
            case 3:
                if (q != 0 || (p != 0 && p != ex)) return false;
                w = p == 0 ? 1 - al : al;
                return true;
            case 4:
                if (p != 0 || (q != 0 && q != ey)) return false;
                w = q == 0 ? 1 - be : be;
                return true;
            default:
                if (p != 0 || q != 0) return false;
                w = 1.0;
                return true;
        }
    }
};
template <class AV> __device__ __forceinline__ NestStencil nest_stencil(const AV &av, int sx, int sy) {
    auto avn = [&](int p, int q) { return av(p * sx, q * sy); };
    bool all = true;
#pragma unroll
    for (int q = -1; q <= 1; ++q)
#pragma unroll
        for (int p = -1; p <= 1; ++p) all = all && avn(p, q);
    if (all) return NestStencil{0, 0, 0};
    // quadrants (ex, ey) = (1, 1), (-1, 1), (1, -1), (-1, -1) in turn
    for (int d = 0; d < 4; ++d) {
        const int ex = (d & 1) ? -1 : 1, ey = (d & 2) ? -1 : 1;
        if (avn(ex, 0) && avn(0, ey) && avn(ex, ey)) return NestStencil{1, ex, ey};
    }
    for (int d = 0; d < 4; ++d) {
        const int ex = (d & 1) ? -1 : 1, ey = (d & 2) ? -1 : 1;
        if (avn(ex, 0) && avn(0, ey)) return NestStencil{2, ex, ey};
    }
    if (avn(1, 0)) return NestStencil{3, 1, 0};
    if (avn(-1, 0)) return NestStencil{3, -1, 0};
    if (avn(0, 1)) return NestStencil{4, 0, 1};
    if (avn(0, -1)) return NestStencil{4, 0, -1};
    return NestStencil{5, 0, 0};
}

// One thread per cell of a box: level-l cells of the box get
// F^l = F_fine + sum_k w_k (F^{l-1}(p_k) - F_coarse(p_k)) in FP64.
template <typename T> __global__ void __launch_bounds__(256) k_nest_combine(CombineArgs<T> a) {
    const int b = blockIdx.y;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.nbox || idx >= kNestBox * kNestBox) return;
    const int tx = idx % kNestBox, ty = idx / kNestBox;
    const int fxl = tx + kNestExt, fyl = ty + kNestExt;  // position in the fine region
    const int64_t fo = (int64_t)b * kNestFine * kNestFine + (int64_t)fyl * kNestFine + fxl;
    const int32_t o = a.fown[fo];
    const int32_t c = o & 0x0FFFFFFF;
    if (c == a.sentinel || (o >> 28) != 0) return;  // no level-l cell here
    // box origins are multiples of kNestBox, so cell parity and the parent's
    // place in the coarse region follow from the position in the box
    const int sx = (tx & 1) ? 1 : -1, sy = (ty & 1) ? 1 : -1;
    const int ci = (tx >> 1) + kNestExt / 2, cj = (ty >> 1) + kNestExt / 2;
    const int32_t *cown = a.cown + (int64_t)b * kNestCoarse * kNestCoarse;
    auto av = [&](int da, int db) {
        const int32_t q = cown[(cj + db) * kNestCoarse + ci + da];
        return (q & 0x0FFFFFFF) != a.sentinel && (q >> 28) == 0;
    };
    const NestStencil st = nest_stencil(av, sx, sy);
    const T *cfx = a.cfx + (int64_t)b * kNestCoarse * kNestCoarse;
    const T *cfy = a.cfy + (int64_t)b * kNestCoarse * kNestCoarse;
    double ex = 0.0, ey = 0.0;
#pragma unroll
    for (int q = -1; q <= 1; ++q)
#pragma unroll
        for (int p = -1; p <= 1; ++p) {
            double w;
            if (!st.weight(p, q, w)) continue;
            const int pos = (cj + q * sy) * kNestCoarse + ci + p * sx;
            const int32_t pc = cown[pos] & 0x0FFFFFFF;
            ex += w * (a.accx[pc] - (double)cfx[pos]);
            ey += w * (a.accy[pc] - (double)cfy[pos]);
        }
    a.accx[c] = (double)a.ffx[fo] + ex;
    a.accy[c] = (double)a.ffy[fo] + ey;
}

template <typename T>
__global__ void __launch_bounds__(256) k_nest_finalize(const double *accx, const double *accy,
                                                       const uint8_t *leaf, T *fx, T *fy, int64_t n) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const bool l = leaf[c] != 0;
    fx[c] = l ? (T)accx[c] : (T)0;
    fy[c] = l ? (T)accy[c] : (T)0;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

template <typename TQ, int M>
static hipError_t col_extract_m(const C<double> *in, TQ *q, int64_t q_pitch, int imag, int corner,
                                const C<double> *tw, const C<double> *ph, hipStream_t s) {
    hipLaunchKernelGGL((k_col_extract<TQ, M>), dim3(M / 2), dim3(ExtractCfg<M>::NT), 0, s, in, q,
                       q_pitch, imag, corner, tw, ph);
    return hipGetLastError();
}

template <typename T, int M> static bool row_ok_t(int var) {
    switch (var) {
        case 0: return row_var_ok<T, M, 0>();
        case 1: return row_var_ok<T, M, 1>();
        case 2: return row_var_ok<T, M, 2>();
        case 3: return row_var_ok<T, M, 3>();
        case 4: return row_var_ok<T, M, 4>();
        case 5: return row_var_ok<T, M, 5>();
        case 6: return row_var_ok<T, M, 6>();
        case 7: return row_var_ok<T, M, 7>();
        case 8: return row_var_ok<T, M, 8>();
        case 9: return row_var_ok<T, M, 9>();
        case 10: return row_var_ok<T, M, 10>();
        case 11: return row_var_ok<T, M, 11>();
    }
    return false;
}
template <int M> static bool row_ok(int prec, int var) {
    return prec ? row_ok_t<double, M>(var) : row_ok_t<float, M>(var);
}
template <typename T, int M, int NF, int NFAM, int NC> static bool col_ok(int var) {
    switch (var) {
        case 0: return col_var_ok<T, M, 0, NF, NFAM, NC>();
        case 1: return col_var_ok<T, M, 1, NF, NFAM, NC>();
        case 2: return col_var_ok<T, M, 2, NF, NFAM, NC>();
        case 3: return col_var_ok<T, M, 3, NF, NFAM, NC>();
        case 4: return col_var_ok<T, M, 4, NF, NFAM, NC>();
        case 6: return col_var_ok<T, M, 6, NF, NFAM, NC>();
        case 8: return col_var_ok<T, M, 8, NF, NFAM, NC>();
        case 9: return col_var_ok<T, M, 9, NF, NFAM, NC>();
        case 10: return col_var_ok<T, M, 10, NF, NFAM, NC>();
        case 11: return col_var_ok<T, M, 11, NF, NFAM, NC>();
        case 12: return col_var_ok<T, M, 12, NF, NFAM, NC>();
        case 13: return col_var_ok<T, M, 13, NF, NFAM, NC>();
        case 14: return col_var_ok<T, M, 14, NF, NFAM, NC>();
        case 15: return col_var_ok<T, M, 15, NF, NFAM, NC>();
        case 16: return col_var_ok<T, M, 16, NF, NFAM, NC>();
    }
    return false;
}
template <typename T, int M, int NC> static bool col_ok_k(int var, int nf, int nfam) {
    if (nf == 3 && nfam == 1) return col_ok<T, M, 3, 1, NC>(var);
    if (nf == 3 && nfam == 2) return col_ok<T, M, 3, 2, NC>(var);
    if (nf == 1 && nfam == 1) return col_ok<T, M, 1, 1, NC>(var);
    if (nf == 1 && nfam == 2) return col_ok<T, M, 1, 2, NC>(var);
    return false;
}
template <int M> static bool col_ok_p(int prec, int var, int nf, int nfam, int nc) {
    if (nc == 2) return prec ? col_ok_k<double, M, 2>(var, nf, nfam) : col_ok_k<float, M, 2>(var, nf, nfam);
    if (nc == 3) return prec ? col_ok_k<double, M, 3>(var, nf, nfam) : col_ok_k<float, M, 3>(var, nf, nfam);
    return false;
}
bool row_variant_valid(int prec, int M, int var) {
    switch (M) {
        case 32: return row_ok<32>(prec, var);
        case 64: return row_ok<64>(prec, var);
        case 128: return row_ok<128>(prec, var);
        case 256: return row_ok<256>(prec, var);
        case 512: return row_ok<512>(prec, var);
        case 1024: return row_ok<1024>(prec, var);
        case 2048: return row_ok<2048>(prec, var);
        case 4096: return row_ok<4096>(prec, var);
        case 8192: return row_ok<8192>(prec, var);
    }
    return false;
}
bool col_variant_valid(int prec, int M, int var, int nf, int nfam, int nc) {
    switch (M) {
        case 32: return col_ok_p<32>(prec, var, nf, nfam, nc);
        case 64: return col_ok_p<64>(prec, var, nf, nfam, nc);
        case 128: return col_ok_p<128>(prec, var, nf, nfam, nc);
        case 256: return col_ok_p<256>(prec, var, nf, nfam, nc);
        case 512: return col_ok_p<512>(prec, var, nf, nfam, nc);
        case 1024: return col_ok_p<1024>(prec, var, nf, nfam, nc);
        case 2048: return col_ok_p<2048>(prec, var, nf, nfam, nc);
        case 4096: return col_ok_p<4096>(prec, var, nf, nfam, nc);
        case 8192: return col_ok_p<8192>(prec, var, nf, nfam, nc);
    }
    return false;
}

template <typename T>
hipError_t launch_gather(const Pack<GatherArgs<T>> &a, int n, int64_t maxcells, hipStream_t s) {
    if (n < 1 || n > kPack) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_gather<T>), dim3((unsigned)((maxcells + 255) / 256), 1, n), dim3(256), 0, s,
                       a);
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

static unsigned nblocks(int64_t n) { return (unsigned)((n + 255) / 256); }

template <typename T>
hipError_t launch_nest_copy_in(const T *s, const T *dx, const T *dy, T *rs, T *rdx, T *rdy, int64_t n,
                               hipStream_t st) {
    hipLaunchKernelGGL((k_nest_copy_in<T>), dim3(nblocks(n + 1)), dim3(256), 0, st, s, dx, dy, rs, rdx, rdy, n);
    return hipGetLastError();
}
template <typename T> hipError_t launch_nest_restrict(const RestrictArgs<T> &a, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_nest_restrict<T>), dim3(nblocks(a.n)), dim3(256), 0, st, a);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_nest_lift(const T *fx, const T *fy, double *accx, double *accy, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL((k_nest_lift<T>), dim3(nblocks(n)), dim3(256), 0, st, fx, fy, accx, accy, n);
    return hipGetLastError();
}
template <typename T> hipError_t launch_nest_combine(const CombineArgs<T> &a, hipStream_t st) {
    if (a.nbox <= 0) return hipSuccess;
    if (a.nbox > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_nest_combine<T>), dim3(kNestBox * kNestBox / 256, a.nbox), dim3(256), 0, st, a);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_nest_finalize(const double *accx, const double *accy, const uint8_t *leaf, T *fx, T *fy,
                                int64_t n, hipStream_t st) {
    hipLaunchKernelGGL((k_nest_finalize<T>), dim3(nblocks(n)), dim3(256), 0, st, accx, accy, leaf, fx, fy, n);
    return hipGetLastError();
}
#define GRAV_NEST_INST(T)                                                                                   \
    template hipError_t launch_nest_copy_in<T>(const T *, const T *, const T *, T *, T *, T *, int64_t,     \
                                               hipStream_t);                                                \
    template hipError_t launch_nest_restrict<T>(const RestrictArgs<T> &, hipStream_t);                      \
    template hipError_t launch_nest_lift<T>(const T *, const T *, double *, double *, int64_t, hipStream_t); \
    template hipError_t launch_nest_combine<T>(const CombineArgs<T> &, hipStream_t);                        \
    template hipError_t launch_nest_finalize<T>(const double *, const double *, const uint8_t *, T *, T *,   \
                                                int64_t, hipStream_t);
GRAV_NEST_INST(float)
GRAV_NEST_INST(double)
#undef GRAV_NEST_INST

template hipError_t launch_gather<float>(const Pack<GatherArgs<float>> &, int, int64_t, hipStream_t);
template hipError_t launch_gather<double>(const Pack<GatherArgs<double>> &, int, int64_t, hipStream_t);
template hipError_t launch_col_extract<float>(const C<double> *, int, float *, int64_t, int, int,
                                              const C<double> *, const C<double> *, hipStream_t);
template hipError_t launch_col_extract<double>(const C<double> *, int, double *, int64_t, int, int,
                                               const C<double> *, const C<double> *, hipStream_t);

}  // namespace grav
