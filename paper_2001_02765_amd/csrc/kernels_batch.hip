// One persistent launch over a batch of independent uniform solves of mixed
// sizes.  The work is a queue of units in pass order: every row-forward unit
// of every solve, then every column unit, then every row-inverse unit.  A
// block takes the next unit from an atomic counter (one unit ahead of the
// one it works on); a unit of a later pass waits (bounded) until its own
// solve's previous pass has completed all its units.  Every unit a block can
// wait for was taken earlier by a running block, and the smallest unfinished
// unit is always one that a block works on with all of its earlier passes
// complete, so the waits end.
//
// Shapes (256 threads per block; 4 elements per thread, 8 in the 2048-point
// columns):
//   row pass    L = M/2 points per row, NTR = L/4 threads per row, 256/NTR
//               rows per step (rows interleaved lane by lane)
//   column pass NT = M/E threads per column, 256/NT columns per step (one
//               exchange region per column)
// and up to 8 steps per unit (about 8K points), so that taking a unit (an
// atomic and a search over the solves) stays small beside its work;
// for 128 <= M <= 2048.
#include <algorithm>

#include "kernels_impl.hpp"

namespace grav {

namespace {

constexpr int kBT = 256;  // threads per block

// elements per thread: 4 (fewer registers per thread, so that every size
// fits one kernel at a useful occupancy), 8 for the 2048-point columns
template <typename T, int M> struct BShape {
    static constexpr int L = M / 2;
    static constexpr int RE = 4, CE = M > 1024 ? 8 : 4;
    static constexpr int NTR = L / RE;
    static constexpr int RPU = kBT / NTR;  // rows per step
    static constexpr int NT = M / CE;
    static constexpr int CPU = kBT / NT;   // columns per step
    // steps per unit (up to 8 row groups / column groups: about 8K points)
    static constexpr int KR = cmin(8, L / RPU);
    static constexpr int KC = cmin(CE == 8 ? 4 : 8, L / CPU);
    static constexpr int ROW_LDS = RPU * aos_slots<L>();
    static constexpr int COL_LDS = CPU * col_region<M>();
    static constexpr int LDS = ROW_LDS > COL_LDS ? ROW_LDS : COL_LDS;
};
template <typename T> constexpr int batch_lds() {
    constexpr int a = BShape<T, 128>::LDS, b = BShape<T, 256>::LDS, c = BShape<T, 512>::LDS;
    constexpr int d = BShape<T, 1024>::LDS, e = BShape<T, 2048>::LDS;
    return cmax(cmax(cmax(a, b), cmax(c, d)), e);
}

// The lane index passes through an empty asm at every unit: otherwise the
// compiler hoists the lane-dependent addressing of every size and pass out of
// the unit loop, and keeps all of it live (hundreds of registers).
__device__ __forceinline__ int lane_id() {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

template <typename T, int M>
__device__ void unit_row_fwd(const BatchItem<T> &it, int u, C<T> *lds) {
    using S = BShape<T, M>;
    const int t = lane_id(), r = t % S::RPU, tr = t / S::RPU;
    const LdsAoS map{S::RPU, r};
    TwReg<T, S::L, S::NTR> twr;
    twr.load(it.tw, 2, tr);
    for (int k = 0; k < S::KR; ++k) {
        const int64_t j = ((int64_t)u * S::KR + k) * S::RPU + r;
        row_fwd_rows<T, M, S::RE, true, false>(it.rf, j, tr, 0, 3, lds, map, it.tw, twr);
    }
}

template <typename T, int M>
__device__ void unit_col(const BatchItem<T> &it, int u, C<T> *lds) {
    using S = BShape<T, M>;
    const int t = lane_id(), g = t / S::NT, tl = t % S::NT;
    // variants 8 (4 elements per thread) and 0 (8): fields one after the other
    for (int k = 0; k < S::KC; ++k)
        col_body<T, M, S::CE == 4 ? 8 : 0, 3, 1, 2>(it.col, it.tw, it.ph, lds + g * col_region<M>(), tl,
                                                      (u * S::KC + k) * S::CPU + g);
}

template <typename T, int M>
__device__ void unit_row_inv(const BatchItem<T> &it, int u, C<T> *lds) {
    using S = BShape<T, M>;
    const int t = lane_id(), r = t % S::RPU, tr = t / S::RPU;
    const LdsAoS map{S::RPU, r};
    TwReg<T, S::L, S::NTR> twr;
    twr.load(it.tw, 2, tr);
    for (int k = 0; k < S::KR; ++k) {
        const int64_t j = ((int64_t)u * S::KR + k) * S::RPU + r;
        row_inv_rows<T, M, S::RE>(it.ri, j, tr, 0, 2, lds, map, it.tw, twr);
    }
}

template <typename T, int M> __device__ void run_unit(const BatchItem<T> &it, int pass, int u, C<T> *lds) {
    if (pass == 0)
        unit_row_fwd<T, M>(it, u, lds);
    else if (pass == 1)
        unit_col<T, M>(it, u, lds);
    else
        unit_row_inv<T, M>(it, u, lds);
}

// 3 waves per SIMD for FP32 (168 registers: the 2048-point column fits), 2
// for FP64
constexpr int kFirstLds = 1024;  // pass offsets cached in LDS up to this many entries

template <typename T>
__global__ void __launch_bounds__(kBT) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 3 : 2))) k_batch(
    BatchCtl *ctl, const uint32_t *first, uint32_t *done, const BatchItem<T> *items, int n, uint32_t spin_limit) {
    __shared__ C<T> lds[batch_lds<T>()];
    __shared__ uint32_t s_first[kFirstLds];
    __shared__ uint32_t s_u;
    const uint32_t e0 = ctl->end[0], e1 = ctl->end[1], total = ctl->end[2];
    const int nf = 3 * (n + 1);
    const bool cached = nf <= kFirstLds;
    if (cached)
        for (int k = threadIdx.x; k < nf; k += kBT) s_first[k] = first[k];
    // Control flow stays uniform across the block: lane 0 only takes units
    // (a branch with no loop inside), every other decision is made by all
    // lanes on values made uniform with readfirstlane.  A loop or exit taken
    // by one lane alone around the barriers lets the compiler keep the other
    // lanes cycling over the barriers without it (a hang).
    if (threadIdx.x == 0) s_u = __hip_atomic_fetch_add(&ctl->head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    block_sync();
    for (;;) {
        const uint32_t u = __builtin_amdgcn_readfirstlane(s_u);
        block_sync();  // s_u is rewritten below
        if (u >= total) break;
        // take the next unit now, so that the atomic's latency hides behind
        // this unit's work (units are still worked in the order taken)
        if (threadIdx.x == 0) s_u = __hip_atomic_fetch_add(&ctl->head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int pass = u < e0 ? 0 : (u < e1 ? 1 : 2);
        auto fget = [&](int k) -> uint32_t {
            return __builtin_amdgcn_readfirstlane(cached ? s_first[k] : first[k]);
        };
        const int fb = pass * (n + 1);
        int lo = 0, hi = n - 1;  // last solve whose first unit of this pass is <= u
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (fget(fb + mid) <= u) lo = mid; else hi = mid - 1;
        }
        const int r = __builtin_amdgcn_readfirstlane(lo);
        const int unit = (int)(u - fget(fb + r));
        if (pass > 0) {
            // the solve's previous pass: all of its units complete
            const int pb = (pass - 1) * (n + 1);
            const uint32_t need = fget(pb + r + 1) - fget(pb + r);
            uint32_t *cnt = done + 3 * r + (pass - 1);
            uint32_t spins = 0;
            bool ok = true;
            while (__builtin_amdgcn_readfirstlane(
                       __hip_atomic_load(cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)) < need) {
                if (++spins > spin_limit) {
                    ok = false;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            if (!ok) {
                if (threadIdx.x == 0)
                    __hip_atomic_fetch_add(&ctl->timeouts, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
        const BatchItem<T> &it = items[r];
        switch (it.M) {
            case 128: run_unit<T, 128>(it, pass, unit, lds); break;
            case 256: run_unit<T, 256>(it, pass, unit, lds); break;
            case 512: run_unit<T, 512>(it, pass, unit, lds); break;
            case 1024: run_unit<T, 1024>(it, pass, unit, lds); break;
            case 2048: run_unit<T, 2048>(it, pass, unit, lds); break;
            default: break;
        }
        block_sync();  // every thread's writes of this unit are issued and complete
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(done + 3 * r + pass, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

}  // namespace

bool batch_size_ok(int M) { return M >= 128 && M <= 2048 && (M & (M - 1)) == 0; }

template <int M> static void units_of(uint32_t units[3]) {
    using S = BShape<float, M>;  // the shapes do not depend on the precision
    units[0] = units[2] = (uint32_t)(S::L / (S::RPU * S::KR));  // rows: n = M/2 = L
    units[1] = (uint32_t)(S::L / (S::CPU * S::KC));
}
void batch_units(int M, uint32_t units[3]) {
    units[0] = units[1] = units[2] = 0;
    switch (M) {
        case 128: units_of<128>(units); break;
        case 256: units_of<256>(units); break;
        case 512: units_of<512>(units); break;
        case 1024: units_of<1024>(units); break;
        case 2048: units_of<2048>(units); break;
    }
}

template <typename T>
hipError_t launch_batch(BatchCtl *ctl, const uint32_t *first, uint32_t *done, const BatchItem<T> *items, int n,
                        uint32_t total_units, hipStream_t s) {
    if (n < 1 || total_units == 0) return hipSuccess;
    int dev = 0, cus = 0, per = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batch<T>, kBT, 0);
    if (e != hipSuccess) return e;
    const uint32_t resident = (uint32_t)std::max(1, per) * (uint32_t)std::max(1, cus);
    const uint32_t grid = std::min(total_units, resident);
    // about a second of waiting at most per unit (s_sleep 2 is ~128 cycles)
    const uint32_t spin_limit = 1u << 24;
    hipLaunchKernelGGL(k_batch<T>, dim3(grid), dim3(kBT), 0, s, ctl, first, done, items, n, spin_limit);
    return hipGetLastError();
}

template hipError_t launch_batch<float>(BatchCtl *, const uint32_t *, uint32_t *, const BatchItem<float> *, int,
                                        uint32_t, hipStream_t);
template hipError_t launch_batch<double>(BatchCtl *, const uint32_t *, uint32_t *, const BatchItem<double> *,
                                         int, uint32_t, hipStream_t);

}  // namespace grav
