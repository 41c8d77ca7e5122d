// Register/LDS Stockham FFT engine for gfx950 (wave64, 160 KB LDS per CU).
//
// A length-L complex transform is computed by NT cooperating threads, each
// holding E = L / NT elements in registers.  On entry and on exit thread t
// holds the elements of index t + NT*e (e = 0..E-1), natural order.  Each
// radix-R pass is the Stockham autosort step: butterfly j reads x[j + r L/R],
// applies the twiddles W_{Ns R}^{r (j mod Ns)}, transforms, and writes to
// index (j / Ns) Ns R + (j mod Ns) + r Ns.  Intermediate passes exchange
// through LDS; the last pass lands every output in the register of the
// thread that owns it, so the forward output distribution equals the input
// distribution of the next transform and of pointwise products (no exchange
// between a forward transform, a spectral multiply and an inverse transform).
//
// Twiddles are read from a device table tw[k] = exp(-2 pi i k / M) built in
// double precision; a length-L transform uses stride M / L.  DIR = -1 is the
// forward transform, DIR = +1 the unnormalised inverse.
#pragma once

#include <hip/hip_runtime.h>

namespace grav {

// Block barrier for the LDS exchanges.  The compiler does not treat the
// barrier instruction as a memory write, so it may sink LDS loads that precede
// it into a later, conditionally executed block, where they would read LDS that
// other waves have already overwritten.  The empty asm statements with a
// memory clobber on both sides keep every LDS access on its own side.
__device__ __forceinline__ void block_sync() {
    asm volatile("" ::: "memory");
    __syncthreads();
    asm volatile("" ::: "memory");
}


template <typename T> struct vec2;
template <> struct vec2<float> { typedef float2 type; };
template <> struct vec2<double> { typedef double2 type; };
template <typename T> using C = typename vec2<T>::type;

template <typename T> __device__ __forceinline__ C<T> mk(T x, T y) { C<T> r; r.x = x; r.y = y; return r; }
template <typename T> __device__ __forceinline__ C<T> cadd(C<T> a, C<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ C<T> csub(C<T> a, C<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T> __device__ __forceinline__ C<T> cmul(C<T> a, C<T> b) {
    return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename T> __device__ __forceinline__ C<T> cmulc(C<T> a, C<T> b) {
    return mk<T>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename T> __device__ __forceinline__ C<T> cconj(C<T> a) { return mk<T>(a.x, -a.y); }
template <typename T> __device__ __forceinline__ C<T> cscale(C<T> a, T s) { return mk<T>(a.x * s, a.y * s); }

// multiply by DIR * i  (forward: -i)
template <int DIR, typename T> __device__ __forceinline__ C<T> rot(C<T> a) {
    return DIR < 0 ? mk<T>(a.y, -a.x) : mk<T>(-a.y, a.x);
}
// multiply by w (forward) or conj(w) (inverse)
template <int DIR, typename T> __device__ __forceinline__ C<T> twm(C<T> a, C<T> w) {
    return DIR < 0 ? cmul<T>(a, w) : cmulc<T>(a, w);
}

// cos and sin of 2 pi m / 16
__host__ __device__ constexpr double cos16(int m) {
    constexpr double t[16] = {
        1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
        0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
        -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
        0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
    return t[m & 15];
}
__host__ __device__ constexpr double sin16(int m) { return cos16(m + 12); }

template <int DIR, typename T> __device__ __forceinline__ void dft2(C<T> &a, C<T> &b) {
    C<T> t = a;
    a = cadd<T>(t, b);
    b = csub<T>(t, b);
}

template <int DIR, typename T>
__device__ __forceinline__ void dft4(C<T> &x0, C<T> &x1, C<T> &x2, C<T> &x3) {
    C<T> a = cadd<T>(x0, x2), b = csub<T>(x0, x2);
    C<T> c = cadd<T>(x1, x3), d = rot<DIR, T>(csub<T>(x1, x3));
    x0 = cadd<T>(a, c);
    x2 = csub<T>(a, c);
    x1 = cadd<T>(b, d);
    x3 = csub<T>(b, d);
}

// multiply by W_16^m in direction DIR, m a compile-time constant
template <int DIR, int m, typename T> __device__ __forceinline__ C<T> w16(C<T> a) {
    constexpr int mm = m & 15;
    if constexpr (mm == 0) return a;
    else if constexpr (mm == 4) return rot<DIR, T>(a);
    else if constexpr (mm == 8) return mk<T>(-a.x, -a.y);
    else if constexpr (mm == 12) return rot<-DIR, T>(a);
    else {
        constexpr double cd = cos16(mm), sd = DIR * sin16(mm);
        const T c = (T)cd;
        const T s = (T)sd;
        return mk<T>(a.x * c - a.y * s, a.x * s + a.y * c);
    }
}

template <int DIR, typename T> __device__ __forceinline__ void dft8(C<T> *v) {
    C<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    C<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<DIR, T>(e0, e1, e2, e3);
    dft4<DIR, T>(o0, o1, o2, o3);
    o1 = w16<DIR, 2, T>(o1);
    o2 = w16<DIR, 4, T>(o2);
    o3 = w16<DIR, 6, T>(o3);
    v[0] = cadd<T>(e0, o0); v[4] = csub<T>(e0, o0);
    v[1] = cadd<T>(e1, o1); v[5] = csub<T>(e1, o1);
    v[2] = cadd<T>(e2, o2); v[6] = csub<T>(e2, o2);
    v[3] = cadd<T>(e3, o3); v[7] = csub<T>(e3, o3);
}

// 16 = 4 x 4: inner DFT-4 over n1 of x[4 n1 + n2], twiddle W16^{n2 k1},
// outer DFT-4 over n2 giving X[k1 + 4 k2].
template <int DIR, typename T> __device__ __forceinline__ void dft16(C<T> *v) {
    C<T> a[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
        a[n2][0] = v[n2]; a[n2][1] = v[n2 + 4]; a[n2][2] = v[n2 + 8]; a[n2][3] = v[n2 + 12];
        dft4<DIR, T>(a[n2][0], a[n2][1], a[n2][2], a[n2][3]);
    }
    a[1][1] = w16<DIR, 1, T>(a[1][1]); a[1][2] = w16<DIR, 2, T>(a[1][2]); a[1][3] = w16<DIR, 3, T>(a[1][3]);
    a[2][1] = w16<DIR, 2, T>(a[2][1]); a[2][2] = w16<DIR, 4, T>(a[2][2]); a[2][3] = w16<DIR, 6, T>(a[2][3]);
    a[3][1] = w16<DIR, 3, T>(a[3][1]); a[3][2] = w16<DIR, 6, T>(a[3][2]); a[3][3] = w16<DIR, 9, T>(a[3][3]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        C<T> b0 = a[0][k1], b1 = a[1][k1], b2 = a[2][k1], b3 = a[3][k1];
        dft4<DIR, T>(b0, b1, b2, b3);
        v[k1] = b0; v[k1 + 4] = b1; v[k1 + 8] = b2; v[k1 + 12] = b3;
    }
}

template <int R, int DIR, typename T> __device__ __forceinline__ void dft(C<T> *v) {
    if constexpr (R == 2) dft2<DIR, T>(v[0], v[1]);
    else if constexpr (R == 4) dft4<DIR, T>(v[0], v[1], v[2], v[3]);
    else if constexpr (R == 8) dft8<DIR, T>(v);
    else if constexpr (R == 16) dft16<DIR, T>(v);
    else static_assert(R == 2, "unsupported radix");
}

// LDS index with one pad element every 16 (breaks power-of-two strides)
__device__ __forceinline__ int pidx(int i) { return i + (i >> 4); }
// LDS elements needed for a length-L exchange region
template <int L> constexpr int lds_region() { return L + (L >> 4) + 1; }

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v >> 1); }

// radix of pass p for a length-L transform on NT threads: radix E, then a
// final pass of the leftover radix if log2 L is not a multiple of log2 E
// (leftover last measured faster than leftover first on gfx950: the 1024^2
// FP64 column kernel 52.3 -> 51.5 us, the FP32 row kernels equal or faster)
template <int L, int NT> struct Plan {
    static constexpr int E = L / NT;
    static constexpr int l = ilog2(L), e = ilog2(E);
    static constexpr int rem = l % e;
    static constexpr int npass = l / e + (rem ? 1 : 0);
    static constexpr int radix(int p) { return (p == npass - 1 && rem) ? (1 << rem) : E; }
    static_assert(E >= 2 && E <= 16 && (E & (E - 1)) == 0, "E must be 2..16, power of two");
    static_assert(NT * E == L, "NT * E must equal L");
};

template <typename T, int L, int NT, int DIR, int NS, int R, bool LAST>
__device__ __forceinline__ void st_pass(C<T> *reg, C<T> *lds, const C<T> *__restrict__ tw,
                                        int tws, int t) {
    constexpr int E = L / NT;
    constexpr int B = E / R;
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int j = t + NT * b;
        const int k = j & (NS - 1);
        C<T> v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = reg[b + r * B];
        if constexpr (NS > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const C<T> w = tw[(r * k * (L / (NS * R))) * tws];
                v[r] = twm<DIR, T>(v[r], w);
            }
        }
        dft<R, DIR, T>(v);
        if constexpr (LAST) {
#pragma unroll
            for (int r = 0; r < R; ++r) reg[b + r * B] = v[r];
        } else {
            const int base = (j / NS) * NS * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) lds[pidx(base + r * NS)] = v[r];
        }
    }
    if constexpr (!LAST) {
        block_sync();
#pragma unroll
        for (int e = 0; e < E; ++e) reg[e] = lds[pidx(t + NT * e)];
        block_sync();
    }
}

template <typename T, int L, int NT, int DIR, int P, int NS>
__device__ __forceinline__ void st_passes(C<T> *reg, C<T> *lds, const C<T> *__restrict__ tw,
                                          int tws, int t) {
    using PL = Plan<L, NT>;
    constexpr int R = PL::radix(P);
    constexpr bool LAST = (P == PL::npass - 1);
    st_pass<T, L, NT, DIR, NS, R, LAST>(reg, lds, tw, tws, t);
    if constexpr (!LAST) st_passes<T, L, NT, DIR, P + 1, NS * R>(reg, lds, tw, tws, t);
}

// Length-L transform by NT threads; t in [0, NT); lds: this transform's
// region (lds_region<L>() elements); every thread of the block must call it
// (it contains block-wide barriers).
template <typename T, int L, int NT, int DIR>
__device__ __forceinline__ void fft(C<T> *reg, C<T> *lds, const C<T> *__restrict__ tw, int tws,
                                    int t) {
    st_passes<T, L, NT, DIR, 0, 1>(reg, lds, tw, tws, t);
}

}  // namespace grav

namespace grav {

// ---------------------------------------------------------------------------
// Register-twiddle variant.  A thread's twiddles depend only on its index and
// the pass, not on the data, so a kernel that runs several transforms of the
// same length (the column kernel runs five) loads them once into registers
// (TwReg) and every pass of every transform, forward or inverse, reuses them.
// fft_multi runs NB independent transforms in lockstep (shared twiddles, NB
// LDS regions lds + i * ldss).
// ---------------------------------------------------------------------------

template <int L, int NT, int P> struct PassInfo {
    using PL = Plan<L, NT>;
    using PREV = PassInfo<L, NT, P - 1>;
    static constexpr int R = PL::radix(P);
    static constexpr int E = PL::E;
    static constexpr int B = E / R;
    static constexpr int NS = PREV::NS * PREV::R;
};
template <int L, int NT> struct PassInfo<L, NT, 0> {
    using PL = Plan<L, NT>;
    static constexpr int R = PL::radix(0);
    static constexpr int E = PL::E;
    static constexpr int B = E / R;
    static constexpr int NS = 1;
};

// Compact twiddles: transforms of length 1024 and more keep only the base
// twiddle w = e^{-2 pi i k / (NS R)} of each butterfly group and form its
// powers w^r by products at use (w^r = w^{r/2} w^{r - r/2}, at most log2 R
// products deep).  The base twiddle passes through an empty volatile asm at
// each use, so that the compiler cannot keep the products of one transform
// alive for the next.  Holding all R - 1 powers in registers made the column
// kernels from 4096 points on (blocks of M/E threads leave at most 256, at
// 1024 threads 128, registers per lane) spill to scratch memory; at 1024 and
// 2048 points the smaller register footprint alone measured 10-15% faster
// (column and row kernels of the 1024^2 solve), below 1024 it is neutral.
template <int L> constexpr bool tw_compact() { return L >= 1024; }
// FP64 transforms of 8192 points (1024-thread blocks: at most 128 registers
// per lane) read each base twiddle from the table at its pass instead: even
// the compact bases (28 registers) tipped those column kernels into
// scratch memory.
template <typename T, int L> constexpr bool tw_mem() { return sizeof(T) == 8 && L >= 8192; }

// twiddle registers (complex) of one pass: R - 1 powers per butterfly
// group, or the base twiddle only (compact); none for the first pass
template <int L, int NT, int P> constexpr int tw_pass_count() {
    using PI = PassInfo<L, NT, P>;
    return PI::NS > 1 ? PI::B * (tw_compact<L>() ? 1 : PI::R - 1) : 0;
}

// number of complex twiddle registers needed by passes [P, npass)
template <int L, int NT, int P> constexpr int tw_count() {
    if constexpr (P >= Plan<L, NT>::npass) return 0;
    else return tw_pass_count<L, NT, P>() + tw_count<L, NT, P + 1>();
}

// p[r] = w^r for r in [1, R), from p[1] = w
template <typename T, int R> __device__ __forceinline__ void tw_powers(C<T> *p) {
#pragma unroll
    for (int r = 2; r < R; ++r) p[r] = cmul<T>(p[r >> 1], p[r - (r >> 1)]);
}

template <typename T, int L, int NT> struct TwReg {
    static constexpr int N = (tw_count<L, NT, 0>() > 0 && !tw_mem<T, L>()) ? tw_count<L, NT, 0>() : 1;
    C<T> w[N];
    const C<T> *tab;  // the table and its stride (tw_mem)
    int tws;

    template <int P, int OFF>
    __device__ __forceinline__ void load_pass(const C<T> *__restrict__ tw, int tws, int t) {
        if constexpr (P < Plan<L, NT>::npass) {
            using PI = PassInfo<L, NT, P>;
            constexpr int NS = PI::NS, R = PI::R, B = PI::B;
            constexpr int CNT = tw_pass_count<L, NT, P>();
            if constexpr (NS > 1) {
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const int k = (t + NT * b) & (NS - 1);
                    if constexpr (tw_compact<L>()) {
                        w[OFF + b] = tw[(k * (L / (NS * R))) * tws];
                    } else {
#pragma unroll
                        for (int r = 1; r < R; ++r)
                            w[OFF + b * (R - 1) + (r - 1)] = tw[(r * k * (L / (NS * R))) * tws];
                    }
                }
            }
            load_pass<P + 1, OFF + CNT>(tw, tws, t);
        }
    }
    __device__ __forceinline__ void load(const C<T> *__restrict__ tw, int stride, int t) {
        tab = tw;
        tws = stride;
        if constexpr (!tw_mem<T, L>()) load_pass<0, 0>(tw, stride, t);
    }
};

// LDS address maps for the exchanges of fft_multi: element x of transform i.
// LdsSoA: one contiguous region per transform (column kernels), one pad slot
// per 32 elements; LdsAoS: the RPB rows of a block interleaved element by
// element, row fastest (row kernels, whose lanes are interleaved the same
// way), one pad slot per 8.  Both are additive: at(i, b + c) = at(i, b) +
// off(c) when b mod BLK + c mod BLK < BLK (no carry into a pad), so an
// exchange forms one lane address per butterfly group and reaches its
// elements with constant offsets (an XOR swizzle spreads the banks better
// but costs address arithmetic per element, which measured slower).
struct LdsSoA {
    static constexpr bool kSoA = true;
    static constexpr int BLK = 32;
    int reg;
    __device__ __forceinline__ int at(int i, int x) const { return i * reg + x + (x >> 5); }
    __device__ __forceinline__ int off(int c) const { return c + (c >> 5); }
    __device__ __forceinline__ int ioff(int i) const { return i * reg; }
    template <int L> static constexpr int region() { return L + (L >> 5) + 1; }
};
struct LdsAoS {
    static constexpr bool kSoA = false;
    static constexpr int BLK = 8;
    int stride, lane;
    __device__ __forceinline__ int at(int, int x) const { return (x + (x >> 3)) * stride + lane; }
    __device__ __forceinline__ int off(int c) const { return (c + (c >> 3)) * stride; }
    __device__ __forceinline__ int ioff(int) const { return 0; }
};
template <int L> constexpr int aos_slots() { return L + 1 + ((L + 1) >> 3) + 1; }

// PPO > 0: two exchange buffers (the second PPO elements on), taken in turn
// by successive exchanges.  A buffer is written again only two exchanges
// later, after the barrier of the exchange in between, which every thread
// reaches only once it has read its elements, so the barrier after the reads
// is not needed: one barrier per exchange instead of two.
template <typename T, int L, int NT, int DIR, int NB, int P, int OFF, class MAP, int PPO, class TWR>
__device__ __forceinline__ void mpass(C<T> (*reg)[L / NT], C<T> *lds0, const MAP &map, const TWR &tr,
                                      int t_in) {
    using PI = PassInfo<L, NT, P>;
    constexpr int E = L / NT, R = PI::R, B = PI::B, NS = PI::NS;
    constexpr bool LAST = (P == Plan<L, NT>::npass - 1);
    constexpr int CNT = tw_pass_count<L, NT, P>();
    // The lane index passes through an empty asm at every pass, so that the
    // pass's LDS addresses are formed where they are used: otherwise the
    // compiler computes the addresses of every pass of every transform of
    // the kernel up front and keeps them all live (tens of registers, and
    // spills in the largest transforms).
    int t = t_in;
    asm volatile("" : "+v"(t));
    C<T> *lds = (PPO > 0 && (P & 1)) ? lds0 + PPO : lds0;
    // FP64 column exchanges: real and imaginary parts in separate planes of
    // the region (8-byte accesses, as in FP32, instead of 16-byte ones)
    constexpr bool PLANAR = sizeof(T) == 8 && MAP::kSoA;
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int j = t + NT * b;
        const int k = j & (NS - 1);
        C<T> pw[R];  // compact twiddles: the powers of this group's base twiddle
        if constexpr (NS > 1 && tw_compact<L>()) {
            if constexpr (tw_mem<T, L>())
                pw[1] = tr.tab[(k * (L / (NS * R))) * tr.tws];
            else
                pw[1] = tr.w[OFF + b];
            asm volatile("" : "+v"(pw[1].x), "+v"(pw[1].y));
            tw_powers<T, R>(pw);
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            C<T> v[R];
#pragma unroll
            for (int r = 0; r < R; ++r) v[r] = reg[i][b + r * B];
            if constexpr (NS > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r)
                    v[r] = twm<DIR, T>(v[r], tw_compact<L>() ? pw[r] : tr.w[OFF + b * (R - 1) + (r - 1)]);
            }
            dft<R, DIR, T>(v);
            if constexpr (LAST) {
#pragma unroll
                for (int r = 0; r < R; ++r) reg[i][b + r * B] = v[r];
            } else if constexpr (PLANAR) {
                const int base = (j / NS) * NS * R + k;
                T *pr = reinterpret_cast<T *>(lds) + map.ioff(i);
                if constexpr (NS * R >= MAP::BLK) {
                    pr += map.at(i, base);
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        pr[map.off(r * NS)] = v[r].x;
                        pr[map.reg + map.off(r * NS)] = v[r].y;
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        pr[map.at(i, base + r * NS)] = v[r].x;
                        pr[map.reg + map.at(i, base + r * NS)] = v[r].y;
                    }
                }
            } else {
                const int base = (j / NS) * NS * R + k;
                if constexpr (NS * R >= MAP::BLK) {
                    // base mod BLK = k < NS and (r NS) mod BLK <= BLK - NS
                    C<T> *p = lds + map.at(i, base);
#pragma unroll
                    for (int r = 0; r < R; ++r) p[map.off(r * NS)] = v[r];
                } else {
#pragma unroll
                    for (int r = 0; r < R; ++r) lds[map.at(i, base + r * NS)] = v[r];
                }
            }
        }
    }
    if constexpr (!LAST) {
        block_sync();
        if constexpr (PLANAR) {
            const T *pr = reinterpret_cast<const T *>(lds) + map.at(0, t);
#pragma unroll
            for (int i = 0; i < NB; ++i)
#pragma unroll
                for (int e = 0; e < E; ++e)
                    reg[i][e] = mk<T>(pr[2 * map.ioff(i) + map.off(NT * e)],
                                      pr[2 * map.ioff(i) + map.reg + map.off(NT * e)]);
        } else {
            // NT and BLK are powers of two: t mod BLK + (NT e) mod BLK < BLK
            const C<T> *p = lds + map.at(0, t);
#pragma unroll
            for (int i = 0; i < NB; ++i)
#pragma unroll
                for (int e = 0; e < E; ++e) reg[i][e] = p[map.ioff(i) + map.off(NT * e)];
        }
        if constexpr (PPO == 0) block_sync();
        mpass<T, L, NT, DIR, NB, P + 1, OFF + CNT, MAP, PPO, TWR>(reg, lds0, map, tr, t);
    }
}

// NB length-L transforms in lockstep; reg[i][e] holds element t + NT e of
// transform i on entry and exit.  With two buffers (PPO > 0) successive
// transforms continue the alternation when a transform has an even number
// of exchanges; with an odd number a barrier on entry separates the last
// reads of one transform from the first writes of the next.
template <typename T, int L, int NT, int DIR, int NB, class MAP, int PPO = 0, class TWR>
__device__ __forceinline__ void fft_multi(C<T> (*reg)[L / NT], C<T> *lds, const MAP &map, const TWR &tr,
                                          int t) {
    if constexpr (PPO > 0 && (Plan<L, NT>::npass - 1) % 2 == 1) block_sync();
    mpass<T, L, NT, DIR, NB, 0, 0, MAP, PPO, TWR>(reg, lds, map, tr, t);
}

}  // namespace grav
