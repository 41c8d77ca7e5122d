// Solve-path kernels (templates) and their launch dispatch.  Instantiated per
// precision and kernel in kernels_{f32,f64}_{row,col}.hip.
//
//  k_row_fwd   real-to-complex row transforms of zero-padded fields at the
//              odd frequencies k + 1/2, written transposed (column-major)
//  k_col       per spectral column: forward column transforms of the input
//              fields, products with the kernel spectra, inverse column
//              transforms of the force components
//  k_row_inv   complex-to-real row transforms of the force components
//
// Each kernel has variants (elements per thread E, and how many transforms a
// thread carries: one field per block row, or all fields in sequence or in
// lockstep); the plan's autotuner times them and keeps the fastest.
#pragma once

#include <type_traits>

#include "kernels.hpp"

namespace grav {

constexpr int cmin(int a, int b) { return a < b ? a : b; }
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int floor_pow2(int v) { return v < 2 ? 1 : 2 * floor_pow2(v / 2); }

// Row transforms: length L = M/2 complex (two real samples packed per
// element), E elements per thread, RPB rows per block.  Lanes are
// interleaved with the row index fastest, so one store instruction writes
// RPB consecutive rows of a spectral column (transposed, coalesced output).
// SC scales the rows per block: 0 the default (at most 8 FP32 / 4 FP64 rows
// in 80 KB of LDS), 1 doubled (up to 160 KB), -1 halved (more, smaller
// blocks for small sizes).
template <typename T, int M, int E, int SC = 0> struct RowCfg {
    static constexpr int L = M / 2;
    static constexpr int NTR = L / E;
    static constexpr int RMAX = (sizeof(T) == 4 ? 8 : 4) * (SC == 1 ? 2 : 1);
    static constexpr int SLOTS = aos_slots<L>();  // LDS elements per row (AoS)
    static constexpr int BYTES = SLOTS * (int)sizeof(C<T>);
    static constexpr int LMAX = SC == 1 ? 163840 : 81920;
    // a power of two (rows per solve are powers of two)
    static constexpr int RPB0 = floor_pow2(cmax(1, cmin(RMAX, cmin(1024 / NTR, LMAX / BYTES))));
    static constexpr int RPB = SC == -1 ? cmax(1, RPB0 / 2) : RPB0;
    static constexpr int NTH = RPB * NTR;
    static_assert((RPB & (RPB - 1)) == 0, "rows per block must be a power of two");
};

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  The row kernels write (forward) or read (inverse) spectral columns in
// segments of RPB consecutive rows, so adjacent row groups share cache lines;
// this remap gives every XCD a contiguous range of row groups, so that the
// partial lines of neighbouring groups meet in one L2.  Needs gridDim.x to be
// a multiple of 8 (then blockIdx.x % 8 is the XCD); otherwise the identity.
__device__ __forceinline__ int xcd_row_group(int b, int nb) {
    return (nb & 7) ? b : (b & 7) * (nb >> 3) + (b >> 3);
}

// variant ids: bit 1 selects E = 16 (else 8); bit 0 selects all fields per
// thread (rows: in sequence; columns: in lockstep) instead of one.  Row
// kernels: bits 2-3 scale the rows per block (0 default, 1 doubled, 2
// halved; ids 0..11).  Column kernel: bit 2 selects two columns per block
// (ids 0..7).
constexpr int var_e(int v) { return (v & 2) ? 16 : 8; }
constexpr bool var_all(int v) { return (v & 1) != 0; }
constexpr bool var_dbl(int v) { return (v & 4) != 0; }
constexpr int row_scale(int v) { return (v >> 2) == 1 ? 1 : ((v >> 2) == 2 ? -1 : 0); }
// column kernel: ids 8 and 9 are ids 0 and 1 with 4 elements per thread
// (twice the threads, fewer registers per thread: for FP64); ids 10 and 11
// are ids 0 and 1 held to 128 registers per lane (4 waves per SIMD), 12 and
// 13 to 102 (5 waves per SIMD): the compiler otherwise spends registers
// freely and these latency-bound kernels run at 2-3 waves per SIMD.  Ids 14
// and 15 are ids 0 and 2 for two kernel families (AMR) with the families
// split over blocks: each block transforms its column's fields and
// accumulates one family, so half the accumulator planes are live (the
// two-family kernels at 4096 and 8192 points otherwise spill to scratch
// memory), at the price of transforming every field twice.  Id 16 is id 10
// with two exchange buffers (one barrier per exchange).
constexpr bool col_split(int v) { return v == 14 || v == 15; }
constexpr bool col_pp(int v) { return v == 16; }
constexpr int col_base(int v) { return v == 15 ? 2 : ((v == 14 || v == 16) ? 0 : (v >= 10 ? (v & 1) : v)); }
constexpr int col_e(int v) { return (v == 8 || v == 9) ? 4 : var_e(col_base(v)); }
constexpr bool col_all(int v) { return var_all(col_base(v)); }
constexpr bool col_dbl(int v) { return v < 8 && var_dbl(v); }
constexpr int col_waves(int v) {
    return (v == 12 || v == 13) ? 5 : ((v == 10 || v == 11 || v == 16) ? 4 : 1);
}
// a row variant exists if each row has at least 2 threads; the doubled and
// halved ones only where they really change the rows per block
template <typename T, int M, int V> constexpr bool row_var_ok() {
    if constexpr (V >= 12 || M / 2 < 2 * var_e(V)) return false;
    else if constexpr (row_scale(V) == 1)
        return RowCfg<T, M, var_e(V), 1>::RPB > RowCfg<T, M, var_e(V), 0>::RPB;
    else if constexpr (row_scale(V) == -1)
        return RowCfg<T, M, var_e(V), -1>::RPB < RowCfg<T, M, var_e(V), 0>::RPB;
    else return true;
}
template <typename T, int M, int V, int NF, int NFAM, int NC> constexpr bool col_var_ok();

// ---------------------------------------------------------------------------
// row forward, odd frequencies: X(k + 1/2) = sum_n x[n] exp(-2 pi i n (k+1/2)/M)
// for k in [0, M/2).  z[m] = (x[2m] + i x[2m+1]) exp(-2 pi i m/M) -> Z =
// FFT_L(z); with Zn = Z[L-1-k]: X(k+1/2) = (Z[k] + conj Zn)/2
// + exp(-i pi (2k+1)/M) (Z[k] - conj Zn)/(2i).  A real row has exactly M/2
// independent odd-frequency bins (X(M-1-k+1/2) = conj X(k+1/2)), all
// complex, so there is no separate real Nyquist bin.
// ---------------------------------------------------------------------------
// AMR inject, fused into the row load: the value of field f at finest cell
// (x, j) from the leaf covering it (Section 2: each leaf's density is linear,
// and the integral is additive over the finest cells it covers).
template <typename T>
__device__ __forceinline__ T inject_value(const RowFwdArgs<T> &a, int f, int64_t j, int x) {
    const int32_t o = a.owner[j * a.in_pitch + x];
    const int32_t c = o & 0x0FFFFFFF;
    if (f != 0) return a.in[f][c];
    T s = a.in[0][c];
    if (a.slopes) {
        const int B = 1 << ((o >> 28) & 0xF);
        const T ox = (T)(2 * (x & (B - 1)) + 1 - B) * (T)0.5 * a.hf;
        const T oy = (T)(2 * ((int)j & (B - 1)) + 1 - B) * (T)0.5 * a.hf;
        s = s + a.in[1][c] * ox + a.in[2][c] * oy;
    }
    return s;
}

// Fields [f0, f1) of row j, transformed by the NTR lanes tr of that row; the
// block's rows are interleaved lane by lane (map); every thread of the block
// must call it (it contains block-wide barriers).
template <typename T, int M, int E, bool PRUNED, bool INJ, class TW>
__device__ __forceinline__ void row_fwd_rows(const RowFwdArgs<T> &a, int64_t j, int tr, int f0, int f1,
                                             C<T> *lds, const LdsAoS &map, const C<T> *__restrict__ tw,
                                             const TW &twr) {
    constexpr int L = M / 2, NTR = L / E;
    const C<T> *__restrict__ hw = tw + M;  // exp(-i pi (2k+1)/M)
    for (int f = f0; f < f1; ++f) {
        const C<T> *row = INJ ? nullptr : reinterpret_cast<const C<T> *>(a.in[f] + j * a.in_pitch);
        const T sc = a.scale[f];
        C<T> reg[1][E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (PRUNED && e >= E / 2) {
                reg[0][e] = mk<T>(0, 0);
            } else {
                const int m = tr + NTR * e;
                const C<T> v = INJ ? mk<T>(inject_value<T>(a, f, j, 2 * m), inject_value<T>(a, f, j, 2 * m + 1))
                                   : row[m];
                reg[0][e] = cmul<T>(mk<T>(v.x * sc, v.y * sc), tw[m]);
            }
        }
        fft_multi<T, L, NTR, -1, 1>(reg, lds, map, twr, tr);
#pragma unroll
        for (int e = 0; e < E; ++e) lds[map.at(0, tr + NTR * e)] = reg[0][e];
        block_sync();
        C<T> *dst = a.out + f * a.out_fstride + j;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = tr + NTR * e;
            const C<T> zk = reg[0][e];
            const C<T> zn = lds[map.at(0, L - 1 - k)];
            const C<T> w = hw[k];
            const T px = zk.x + zn.x, py = zk.y - zn.y;
            const T qx = zk.x - zn.x, qy = zk.y + zn.y;
            dst[(int64_t)k * a.out_pitch] =
                mk<T>((T)0.5 * (px + w.x * qy + w.y * qx), (T)0.5 * (py - w.x * qx + w.y * qy));
        }
        block_sync();  // the next field's first pass reuses this row's LDS
    }
}

template <typename T, int M, int V, bool PRUNED, bool INJ>
__global__ void __launch_bounds__((RowCfg<T, M, var_e(V), row_scale(V)>::NTH))
    k_row_fwd(Pack<RowFwdArgs<T>> pk, int nfields, const C<T> *__restrict__ tw) {
    const RowFwdArgs<T> &a = pk.a[blockIdx.z];
    constexpr int E = var_e(V);
    using CF = RowCfg<T, M, E, row_scale(V)>;
    constexpr int L = CF::L, NTR = CF::NTR, RPB = CF::RPB;
    __shared__ C<T> lds[RPB * CF::SLOTS];
    const int t = threadIdx.x;
    const int r = t % RPB, tr = t / RPB;
    const int64_t grp = xcd_row_group(blockIdx.x, gridDim.x);
    if (grp * RPB >= a.nrows) return;  // whole block: beyond this item's rows
    const int64_t j = grp * RPB + r;
    const LdsAoS map{RPB, r};
    TwReg<T, L, NTR> twr;
    twr.load(tw, 2, tr);
    const int f0 = var_all(V) ? 0 : (int)blockIdx.y;
    const int f1 = var_all(V) ? nfields : f0 + 1;
    row_fwd_rows<T, M, E, PRUNED, INJ>(a, j, tr, f0, f1, lds, map, tw, twr);
}

// ---------------------------------------------------------------------------
// column: for each input field, forward transform of the (zero-padded)
// column, product with the kernel spectra of both force components, then
// inverse transforms of the accumulated force spectra.
//
// Column kx holds the odd x frequency kx + 1/2, kx in [0, M/2).  Kernel
// spectra are stored as one real half plane per kind (all M/2 columns, ky in
// [0, M/2]): kinds {x0, y0} are purely imaginary, the others real; a negative
// ky takes the kind's parity in y.  Corner-family spectra carry the phase
// exp(-i pi (kx + 1/2 + ky)/M) (targets half a cell from the source
// lattice), applied once to the accumulated sums.
// ---------------------------------------------------------------------------


// NC force components (2 in the disk plane, 3 above it): output plane
// NC fam + c accumulates component c of family fam; kind 3 c + f multiplies
// field f.
template <typename T, int M, int E, int NFAM, int NC>
__device__ __forceinline__ void col_mac(C<T> (*acc)[E], const C<T> *x, int f, const ColArgs<T> &a,
                                        int kx, int t, int fam0 = 0) {
    constexpr int NT = M / E, H = M / 2;
#pragma unroll
    for (int fam = 0; fam < NFAM; ++fam) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int kind = 3 * c + f;
            // a select, not an index: a runtime index into the argument
            // copy would place it in scratch memory
            const T *q = (fam0 + fam ? a.q[1] : a.q[0]) + kind * a.q_kstride + (int64_t)kx * a.q_pitch;
            const T sg = (T)parity_y(kind);
            C<T>(&o)[E] = acc[NC * fam + c];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int ky = t + NT * e;
                const bool neg = ky > H;
                T vq = q[neg ? M - ky : ky];
                if (neg) vq *= sg;
                const C<T> X = x[e];
                if (imag_kind(kind)) {  // X * (i v)
                    o[e].x -= X.y * vq;
                    o[e].y += X.x * vq;
                } else {
                    o[e].x += X.x * vq;
                    o[e].y += X.y * vq;
                }
            }
        }
    }
}

// Column exchanges use the padded map, whose additive addresses cost one
// lane address per butterfly group instead of address arithmetic per element.
template <int M> using ColMap = LdsSoA;
template <int M> constexpr int col_region() { return ColMap<M>::template region<M>(); }

template <typename T, int M, int V, int NF, int NFAM, int NC> struct ColLds {
    static constexpr int NB = col_all(V) ? cmax(NF, NC * NFAM) : 1;
    static constexpr int PPO = col_pp(V) ? NB * col_region<M>() : 0;  // second exchange buffer
    static constexpr int N = NB * col_region<M>() * (col_pp(V) ? 2 : 1);
};
// a column variant exists if its transform has at least 2 threads and its
// LDS fits the 160 KB of a gfx950 CU; plans without slopes (one field) and
// small sizes keep only the variants that can differ in speed there
template <typename T, int M, int V, int NF, int NFAM, int NC> constexpr bool col_var_ok() {
    constexpr int B = col_base(V);
    if constexpr (V >= 17 || (V >= 4 && V < 8 && (V == 5 || V == 7 || M < 512))) return false;
    else if constexpr (col_split(V) && (NFAM != 2 || M < 2048)) return false;  // large AMR columns
    else if constexpr (col_pp(V) && (NFAM != 1 || NC != 2 || NF != 3 || M < 1024 || M > 4096)) return false;
    else if constexpr (((V >= 10 && V < 14) || V == 16) && (M < 1024 || M > 4096 || NC == 3))
        return false;  // capped: large midplane columns
    else if constexpr (M / col_e(V) > 1024) return false;  // threads per block
    else if constexpr (NC == 3 && B > 1 && B < 8) return false;  // off-plane: one column, E <= 8
    else if constexpr (V >= 4 && V < 8) return M >= 2 * col_e(V) && 2 * col_region<M>() * (int)sizeof(C<T>) <= 163840;
    else if constexpr (NF == 1 && (B & 1)) return false;
    else if constexpr (M <= 256 && V > 1) return false;
    else return M >= 2 * col_e(V) && ColLds<T, M, V, NF, NFAM, NC>::N * (int)sizeof(C<T>) <= 163840;
}

// Column kx by the NT = M/E threads t of one group; lds: the group's
// exchange regions (ColLds elements); every thread of the block must call it.
// Family-split variants accumulate family fam0 only (output planes
// NC fam0 + c).
template <typename T, int M, int V, int NF, int NFAM, int NC>
__device__ __forceinline__ void col_body(const ColArgs<T> &a, const C<T> *__restrict__ tw,
                                         const C<T> *__restrict__ ph, C<T> *lds, int t, int kx,
                                         int fam0 = 0) {
    constexpr int E = col_e(V), NT = M / E, H = M / 2;
    constexpr int NA = col_split(V) ? 1 : NFAM;  // families accumulated by this block
    constexpr int PPO = ColLds<T, M, V, NF, NFAM, NC>::PPO;
    const ColMap<M> map{col_region<M>()};
    TwReg<T, M, NT> twr;
    twr.load(tw, 1, t);

    C<T> acc[NC * NA][E];
#pragma unroll
    for (int g = 0; g < NC * NA; ++g)
#pragma unroll
        for (int e = 0; e < E; ++e) acc[g][e] = mk<T>(0, 0);

    if constexpr (col_all(V)) {
        C<T> x[NF][E];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const C<T> *src = a.in + f * a.in_fstride + (int64_t)kx * a.in_pitch;
#pragma unroll
            for (int e = 0; e < E; ++e) x[f][e] = (e < E / 2) ? src[t + NT * e] : mk<T>(0, 0);
        }
        fft_multi<T, M, NT, -1, NF, ColMap<M>, PPO>(x, lds, map, twr, t);
#pragma unroll
        for (int f = 0; f < NF; ++f) col_mac<T, M, E, NA, NC>(acc, x[f], f, a, kx, t, fam0);
    } else {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            C<T> x[1][E];
            const C<T> *src = a.in + f * a.in_fstride + (int64_t)kx * a.in_pitch;
#pragma unroll
            for (int e = 0; e < E; ++e) x[0][e] = (e < E / 2) ? src[t + NT * e] : mk<T>(0, 0);
            fft_multi<T, M, NT, -1, 1, ColMap<M>, PPO>(x, lds, map, twr, t);
            col_mac<T, M, E, NA, NC>(acc, x[0], f, a, kx, t, fam0);
        }
    }
    if (NFAM == 2 && (NA == 2 || fam0 == 1)) {  // the corner family's planes
        constexpr int G0 = NA == 2 ? NC : 0;
        const C<T> px = ph[H + 1 + kx];  // exp(-i pi (kx + 1/2)/M)
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int ky = t + NT * e;
            const C<T> py = ky <= H ? ph[ky] : cconj<T>(ph[M - ky]);
            const C<T> p = cmul<T>(px, py);
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[G0 + c][e] = cmul<T>(acc[G0 + c][e], p);
        }
    }
    if constexpr (col_all(V)) {
        fft_multi<T, M, NT, +1, NC * NA, ColMap<M>, PPO>(acc, lds, map, twr, t);
    } else {
#pragma unroll
        for (int g = 0; g < NC * NA; ++g) fft_multi<T, M, NT, +1, 1, ColMap<M>, PPO>(&acc[g], lds, map, twr, t);
    }
#pragma unroll
    for (int g = 0; g < NC * NA; ++g) {
        C<T> *dst = a.out + (NC * fam0 + g) * a.out_gstride + (int64_t)kx * a.out_pitch;
#pragma unroll
        for (int e = 0; e < E / 2; ++e) dst[t + NT * e] = acc[g][e];
    }
}

// Two adjacent columns per block (variants 4, 6): the fields are taken one
// after the other, but each transform runs for both columns in lockstep, so
// the twiddle registers serve two columns and M/4 blocks (512 blocks of 32 KB
// LDS at M = 2048 FP32: two per CU) run in a single dispatch round.
template <typename T, int M, int V, int NF, int NFAM, int NC>
__device__ __forceinline__ void col2_body(const ColArgs<T> &a, const C<T> *__restrict__ tw,
                                          const C<T> *__restrict__ ph) {
    constexpr int E = col_e(V), NT = M / E, H = M / 2;
    const ColMap<M> map{col_region<M>()};
    __shared__ C<T> lds[2 * col_region<M>()];
    const int t = threadIdx.x;
    const int kx0 = 2 * blockIdx.x;
    TwReg<T, M, NT> twr;
    twr.load(tw, 1, t);

    C<T> acc[2][NC * NFAM][E];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int g = 0; g < NC * NFAM; ++g)
#pragma unroll
            for (int e = 0; e < E; ++e) acc[c][g][e] = mk<T>(0, 0);

#pragma unroll
    for (int f = 0; f < NF; ++f) {
        C<T> x[2][E];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const C<T> *src = a.in + f * a.in_fstride + (int64_t)(kx0 + c) * a.in_pitch;
#pragma unroll
            for (int e = 0; e < E; ++e) x[c][e] = (e < E / 2) ? src[t + NT * e] : mk<T>(0, 0);
        }
        fft_multi<T, M, NT, -1, 2>(x, lds, map, twr, t);
        col_mac<T, M, E, NFAM, NC>(acc[0], x[0], f, a, kx0, t);
        col_mac<T, M, E, NFAM, NC>(acc[1], x[1], f, a, kx0 + 1, t);
    }
    if constexpr (NFAM == 2) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const C<T> px = ph[H + 1 + kx0 + c];  // exp(-i pi (kx + 1/2)/M)
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int ky = t + NT * e;
                const C<T> py = ky <= H ? ph[ky] : cconj<T>(ph[M - ky]);
                const C<T> p = cmul<T>(px, py);
#pragma unroll
                for (int g = NC; g < 2 * NC; ++g) acc[c][g][e] = cmul<T>(acc[c][g][e], p);
            }
        }
    }
#pragma unroll
    for (int g = 0; g < NC * NFAM; ++g) {
        C<T> y[2][E];
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int e = 0; e < E; ++e) y[c][e] = acc[c][g][e];
        fft_multi<T, M, NT, +1, 2>(y, lds, map, twr, t);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            C<T> *dst = a.out + g * a.out_gstride + (int64_t)(kx0 + c) * a.out_pitch;
#pragma unroll
            for (int e = 0; e < E / 2; ++e) dst[t + NT * e] = y[c][e];
        }
    }
}

template <typename T, int M, int V, int NF, int NFAM, int NC>
__global__ void __launch_bounds__((M / col_e(V))) __attribute__((amdgpu_waves_per_eu(col_waves(V))))
    k_col(Pack<ColArgs<T>> pk, const C<T> *__restrict__ tw, const C<T> *__restrict__ ph) {
    ColArgs<T> a = pk.a[blockIdx.z];
    if ((int)blockIdx.y >= a.nsub) return;  // whole block: beyond this item's sub-items
    a.in += (int64_t)blockIdx.y * a.sub_off;
    a.out += (int64_t)blockIdx.y * a.sub_off;
    if constexpr (col_dbl(V)) {
        col2_body<T, M, V, NF, NFAM, NC>(a, tw, ph);
    } else if constexpr (col_split(V)) {
        // blocks b and b + 8 (same XCD, dispatched together) take the two
        // families of one column, so the second read of its spectra is
        // likely served from that XCD's L2
        __shared__ C<T> lds[ColLds<T, M, V, NF, NFAM, NC>::N];
        const int b = (int)blockIdx.x;
        col_body<T, M, V, NF, NFAM, NC>(a, tw, ph, lds, (int)threadIdx.x, (b >> 4) * 8 + (b & 7), (b >> 3) & 1);
    } else {
        __shared__ C<T> lds[ColLds<T, M, V, NF, NFAM, NC>::N];
        col_body<T, M, V, NF, NFAM, NC>(a, tw, ph, lds, (int)threadIdx.x, (int)blockIdx.x);
    }
}

// ---------------------------------------------------------------------------
// row inverse, odd frequencies: Y(k + 1/2), k in [0, L) (the independent
// half of a real row's spectrum) -> y[n] = sum over all M odd frequencies of
// Y exp(+2 pi i n (k+1/2)/M), n < M/2, scaled.  With Yn = Y[L-1-k]:
// Z[k] = (Y[k] + conj Yn) + i exp(+i pi (2k+1)/M) (Y[k] - conj Yn),
// z = IFFT_L(Z) (unnormalised), y[2m] + i y[2m+1] = z[m] exp(+2 pi i m/M).
// ---------------------------------------------------------------------------
// Outputs [g0, g1) of row j (see row_fwd_rows).
template <typename T, int M, int E, class TW>
__device__ __forceinline__ void row_inv_rows(const RowInvArgs<T> &a, int64_t j, int tr, int g0, int g1,
                                             C<T> *lds, const LdsAoS &map, const C<T> *__restrict__ tw,
                                             const TW &twr) {
    constexpr int L = M / 2, NTR = L / E;
    const C<T> *__restrict__ hw = tw + M;  // exp(-i pi (2k+1)/M)
    for (int g = g0; g < g1; ++g) {
        const C<T> *src = a.in + g * a.in_gstride + j;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = tr + NTR * e;
            lds[map.at(0, k)] = src[(int64_t)k * a.in_pitch];
        }
        block_sync();
        C<T> reg[1][E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = tr + NTR * e;
            const C<T> yk = lds[map.at(0, k)];
            const C<T> yn = lds[map.at(0, L - 1 - k)];
            const C<T> ze = mk<T>(yk.x + yn.x, yk.y - yn.y);
            const C<T> zo = cmulc<T>(mk<T>(yk.x - yn.x, yk.y + yn.y), hw[k]);
            reg[0][e] = mk<T>(ze.x - zo.y, ze.y + zo.x);
        }
        block_sync();
        fft_multi<T, L, NTR, +1, 1>(reg, lds, map, twr, tr);
        C<T> *dst = reinterpret_cast<C<T> *>(a.out[g] + j * a.out_pitch);
        const T sc = a.scale;
#pragma unroll
        for (int e = 0; e < E / 2; ++e) {
            const int m = tr + NTR * e;
            const C<T> z = cmulc<T>(reg[0][e], tw[m]);
            dst[m] = mk<T>(z.x * sc, z.y * sc);
        }
        block_sync();  // the next output's staging reuses this row's LDS
    }
}

template <typename T, int M, int V>
__global__ void __launch_bounds__((RowCfg<T, M, var_e(V), row_scale(V)>::NTH))
    k_row_inv(Pack<RowInvArgs<T>> pk, int nout, const C<T> *__restrict__ tw) {
    const RowInvArgs<T> &a = pk.a[blockIdx.z];
    constexpr int E = var_e(V);
    using CF = RowCfg<T, M, E, row_scale(V)>;
    constexpr int L = CF::L, NTR = CF::NTR, RPB = CF::RPB;
    __shared__ C<T> lds[RPB * CF::SLOTS];
    const int t = threadIdx.x;
    const int r = t % RPB, tr = t / RPB;
    const int64_t grp = xcd_row_group(blockIdx.x, gridDim.x);
    if (grp * RPB >= a.nrows) return;  // whole block: beyond this item's rows
    const int64_t j = grp * RPB + r;
    const LdsAoS map{RPB, r};
    TwReg<T, L, NTR> twr;
    twr.load(tw, 2, tr);
    const int g0 = var_all(V) ? 0 : (int)blockIdx.y;
    const int g1 = var_all(V) ? nout : g0 + 1;
    row_inv_rows<T, M, E>(a, j, tr, g0, g1, lds, map, tw, twr);
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
#define GRAV_SWITCH_M(M, ...)                               \
    switch (M) {                                            \
        case 32: { constexpr int MM = 32; __VA_ARGS__; }    \
        case 64: { constexpr int MM = 64; __VA_ARGS__; }    \
        case 128: { constexpr int MM = 128; __VA_ARGS__; }  \
        case 256: { constexpr int MM = 256; __VA_ARGS__; }  \
        case 512: { constexpr int MM = 512; __VA_ARGS__; }  \
        case 1024: { constexpr int MM = 1024; __VA_ARGS__; } \
        case 2048: { constexpr int MM = 2048; __VA_ARGS__; } \
        case 4096: { constexpr int MM = 4096; __VA_ARGS__; } \
        case 8192: { constexpr int MM = 8192; __VA_ARGS__; } \
        default: return hipErrorInvalidValue;               \
    }

template <typename T, int M> struct Dispatch {
    template <int V>
    static hipError_t row_fwd_v(const Pack<RowFwdArgs<T>> &a, int n, bool pruned, int64_t nrows,
                                int nfields, const C<T> *tw, hipStream_t s) {
        if constexpr (!row_var_ok<T, M, V>()) {
            return hipErrorInvalidValue;
        } else {
            using CF = RowCfg<T, M, var_e(V), row_scale(V)>;
            if (nrows % CF::RPB || nrows / CF::RPB > 0x7FFFFFFF) return hipErrorInvalidValue;
            for (int i = 0; i < n; ++i)
                if (a.a[i].nrows % CF::RPB || a.a[i].nrows > nrows) return hipErrorInvalidValue;
            dim3 grid((unsigned)(nrows / CF::RPB), var_all(V) ? 1 : nfields, n);
            if (pruned && a.a[0].owner)  // AMR: every item of a pack shares the layout kind
                hipLaunchKernelGGL((k_row_fwd<T, M, V, true, true>), grid, dim3(CF::NTH), 0, s, a, nfields, tw);
            else if (pruned)
                hipLaunchKernelGGL((k_row_fwd<T, M, V, true, false>), grid, dim3(CF::NTH), 0, s, a, nfields,
                                   tw);
            else
                hipLaunchKernelGGL((k_row_fwd<T, M, V, false, false>), grid, dim3(CF::NTH), 0, s, a, nfields,
                                   tw);
            return hipGetLastError();
        }
    }
    static hipError_t row_fwd(const Pack<RowFwdArgs<T>> &a, int n, int var, bool pruned, int64_t nrows,
                              int nfields, const C<T> *tw, hipStream_t s) {
        switch (var) {
            case 0: return row_fwd_v<0>(a, n, pruned, nrows, nfields, tw, s);
            case 1: return row_fwd_v<1>(a, n, pruned, nrows, nfields, tw, s);
            case 2: return row_fwd_v<2>(a, n, pruned, nrows, nfields, tw, s);
            case 3: return row_fwd_v<3>(a, n, pruned, nrows, nfields, tw, s);
            case 4: return row_fwd_v<4>(a, n, pruned, nrows, nfields, tw, s);
            case 5: return row_fwd_v<5>(a, n, pruned, nrows, nfields, tw, s);
            case 6: return row_fwd_v<6>(a, n, pruned, nrows, nfields, tw, s);
            case 7: return row_fwd_v<7>(a, n, pruned, nrows, nfields, tw, s);
            case 8: return row_fwd_v<8>(a, n, pruned, nrows, nfields, tw, s);
            case 9: return row_fwd_v<9>(a, n, pruned, nrows, nfields, tw, s);
            case 10: return row_fwd_v<10>(a, n, pruned, nrows, nfields, tw, s);
            case 11: return row_fwd_v<11>(a, n, pruned, nrows, nfields, tw, s);
        }
        return hipErrorInvalidValue;
    }
    template <int V, int NF, int NFAM, int NC>
    static hipError_t col_v(const Pack<ColArgs<T>> &a, int n, const C<T> *tw, const C<T> *ph,
                            hipStream_t s, int nsub) {
        if constexpr (!col_var_ok<T, M, V, NF, NFAM, NC>()) {
            return hipErrorInvalidValue;
        } else {
            if (nsub < 1 || nsub > 65535) return hipErrorInvalidValue;
            for (int i = 0; i < n; ++i)
                if (a.a[i].nsub < 1 || a.a[i].nsub > nsub) return hipErrorInvalidValue;
            const unsigned nblk = col_dbl(V) ? M / 4 : (col_split(V) ? M : M / 2);
            hipLaunchKernelGGL((k_col<T, M, V, NF, NFAM, NC>), dim3(nblk, nsub, n), dim3(M / col_e(V)), 0, s,
                               a, tw, ph);
            return hipGetLastError();
        }
    }
    template <int V, int NC>
    static hipError_t col_nc(const Pack<ColArgs<T>> &a, int n, int nfields, int nfam, const C<T> *tw,
                             const C<T> *ph, hipStream_t s, int nsub) {
        if (nfields == 3 && nfam == 1) return col_v<V, 3, 1, NC>(a, n, tw, ph, s, nsub);
        if (nfields == 3 && nfam == 2) return col_v<V, 3, 2, NC>(a, n, tw, ph, s, nsub);
        if (nfields == 1 && nfam == 1) return col_v<V, 1, 1, NC>(a, n, tw, ph, s, nsub);
        if (nfields == 1 && nfam == 2) return col_v<V, 1, 2, NC>(a, n, tw, ph, s, nsub);
        return hipErrorInvalidValue;
    }
    template <int V>
    static hipError_t col_nf(const Pack<ColArgs<T>> &a, int n, int nfields, int nfam, int ncomp,
                             const C<T> *tw, const C<T> *ph, hipStream_t s, int nsub) {
        if (ncomp == 2) return col_nc<V, 2>(a, n, nfields, nfam, tw, ph, s, nsub);
        if (ncomp == 3) return col_nc<V, 3>(a, n, nfields, nfam, tw, ph, s, nsub);
        return hipErrorInvalidValue;
    }
    static hipError_t col(const Pack<ColArgs<T>> &a, int n, int var, int nfields, int nfam, int ncomp,
                          const C<T> *tw, const C<T> *ph, hipStream_t s, int nsub) {
        switch (var) {
            case 0: return col_nf<0>(a, n, nfields, nfam, ncomp, tw, ph, s, nsub);
            case 1: return col_nf<1>(a, n, nfields, nfam, ncomp, tw, ph, s, nsub);
            case 2: return col_nf<2>(a, n, nfields, nfam, ncomp, tw, ph, s, nsub);
            case 3: return col_nf<3>(a, n, nfields, nfam, ncomp, tw, ph, s, nsub);
            case 4: return col_nf<4>(a, n, nfields, nfam, ncomp, tw, ph, s, nsub);
            case 6: return col_nf<6>(a, n, nfields, nfam, ncomp, tw, ph, s, nsub);
            case 8: return col_nf<8>(a, n, nfields, nfam, ncomp, tw, ph, s, nsub);
            case 9: return col_nf<9>(a, n, nfields, nfam, ncomp, tw, ph, s, nsub);
            case 10: return col_nf<10>(a, n, nfields, nfam, ncomp, tw, ph, s, nsub);
            case 11: return col_nf<11>(a, n, nfields, nfam, ncomp, tw, ph, s, nsub);
            case 12: return col_nf<12>(a, n, nfields, nfam, ncomp, tw, ph, s, nsub);
            case 13: return col_nf<13>(a, n, nfields, nfam, ncomp, tw, ph, s, nsub);
            case 14: return col_nf<14>(a, n, nfields, nfam, ncomp, tw, ph, s, nsub);
            case 15: return col_nf<15>(a, n, nfields, nfam, ncomp, tw, ph, s, nsub);
            case 16: return col_nf<16>(a, n, nfields, nfam, ncomp, tw, ph, s, nsub);
        }
        return hipErrorInvalidValue;
    }
    template <int V>
    static hipError_t row_inv_v(const Pack<RowInvArgs<T>> &a, int n, int64_t nrows, int nout,
                                const C<T> *tw, hipStream_t s) {
        if constexpr (!row_var_ok<T, M, V>()) {
            return hipErrorInvalidValue;
        } else {
            using CF = RowCfg<T, M, var_e(V), row_scale(V)>;
            if (nrows % CF::RPB || nrows / CF::RPB > 0x7FFFFFFF) return hipErrorInvalidValue;
            for (int i = 0; i < n; ++i)
                if (a.a[i].nrows % CF::RPB || a.a[i].nrows > nrows) return hipErrorInvalidValue;
            dim3 grid((unsigned)(nrows / CF::RPB), var_all(V) ? 1 : nout, n);
            hipLaunchKernelGGL((k_row_inv<T, M, V>), grid, dim3(CF::NTH), 0, s, a, nout, tw);
            return hipGetLastError();
        }
    }
    static hipError_t row_inv(const Pack<RowInvArgs<T>> &a, int n, int var, int64_t nrows, int nout,
                              const C<T> *tw, hipStream_t s) {
        switch (var) {
            case 0: return row_inv_v<0>(a, n, nrows, nout, tw, s);
            case 1: return row_inv_v<1>(a, n, nrows, nout, tw, s);
            case 2: return row_inv_v<2>(a, n, nrows, nout, tw, s);
            case 3: return row_inv_v<3>(a, n, nrows, nout, tw, s);
            case 4: return row_inv_v<4>(a, n, nrows, nout, tw, s);
            case 5: return row_inv_v<5>(a, n, nrows, nout, tw, s);
            case 6: return row_inv_v<6>(a, n, nrows, nout, tw, s);
            case 7: return row_inv_v<7>(a, n, nrows, nout, tw, s);
            case 8: return row_inv_v<8>(a, n, nrows, nout, tw, s);
            case 9: return row_inv_v<9>(a, n, nrows, nout, tw, s);
            case 10: return row_inv_v<10>(a, n, nrows, nout, tw, s);
            case 11: return row_inv_v<11>(a, n, nrows, nout, tw, s);
        }
        return hipErrorInvalidValue;
    }
};

template <typename T>
hipError_t launch_row_fwd(const Pack<RowFwdArgs<T>> &a, int n, int M, int var, bool pruned,
                          int64_t nrows, int nfields, const C<T> *tw, hipStream_t s) {
    if (n < 1 || n > kPack) return hipErrorInvalidValue;
    GRAV_SWITCH_M(M, return (Dispatch<T, MM>::row_fwd(a, n, var, pruned, nrows, nfields, tw, s)))
}
template <typename T>
hipError_t launch_col(const Pack<ColArgs<T>> &a, int n, int M, int var, int nfields, int nfam,
                      int ncomp, const C<T> *tw, const C<T> *ph, hipStream_t s, int nsub) {
    if (n < 1 || n > kPack) return hipErrorInvalidValue;
    GRAV_SWITCH_M(M, return (Dispatch<T, MM>::col(a, n, var, nfields, nfam, ncomp, tw, ph, s, nsub)))
}
template <typename T>
hipError_t launch_row_inv(const Pack<RowInvArgs<T>> &a, int n, int M, int var, int64_t nrows, int nout,
                          const C<T> *tw, hipStream_t s) {
    if (n < 1 || n > kPack) return hipErrorInvalidValue;
    GRAV_SWITCH_M(M, return (Dispatch<T, MM>::row_inv(a, n, var, nrows, nout, tw, s)))
}

}  // namespace grav
