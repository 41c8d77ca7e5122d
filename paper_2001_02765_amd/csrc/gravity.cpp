// Host runtime of the thin-disk gravity library: plans, the resident kernel
// spectrum cache, AMR lattice maps, workspace layout and the C ABI.
#include "../../include/gravity.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <thread>
#include <unordered_map>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <tuple>
#include <vector>

#include "arena.hpp"
#include "kernels.hpp"

namespace {

using namespace grav;

thread_local std::string g_err;

struct Failure {
    gravity_status_t st;
    std::string msg;
};

[[noreturn]] void fail(gravity_status_t st, const std::string &msg) { throw Failure{st, msg}; }

void hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return;
    if (e == hipErrorOutOfMemory) fail(GRAVITY_ENOMEM, std::string(what) + ": out of device memory");
    fail(GRAVITY_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Optional failure injection: GRAVITY_FAIL_ALLOC_AFTER=n makes every device
// allocation after the first n fail with GRAVITY_ENOMEM.
std::mutex g_alloc_mu;
long g_alloc_count = 0;

void *dev_alloc(size_t bytes, const char *what) {
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        const char *env = std::getenv("GRAVITY_FAIL_ALLOC_AFTER");
        if (env && *env) {
            long lim = std::atol(env);
            if (g_alloc_count >= lim) fail(GRAVITY_ENOMEM, std::string(what) + ": injected allocation failure");
        }
        ++g_alloc_count;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes ? bytes : 1);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(GRAVITY_ENOMEM, std::string(what) + ": hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    return p;
}

// Teardown (frees, the server's streams and events) can run while the
// caller captures a stream into a graph: a plan dropped by a garbage
// collector in the middle of a capture, for instance.  Under the default
// (global) capture mode such calls are prohibited during any capture and
// would invalidate it; they touch no captured work, so they run with this
// thread's capture mode relaxed.
struct RelaxedCapture {
    hipStreamCaptureMode prev = hipStreamCaptureModeRelaxed;
    RelaxedCapture() { (void)hipThreadExchangeStreamCaptureMode(&prev); }
    ~RelaxedCapture() { (void)hipThreadExchangeStreamCaptureMode(&prev); }
    RelaxedCapture(const RelaxedCapture &) = delete;
    RelaxedCapture &operator=(const RelaxedCapture &) = delete;
};

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(size_t b, const char *what) : p(dev_alloc(b, what)), bytes(b) {}
    ~DevBuf() { release(); }
    void release() {
        if (p) {
            RelaxedCapture relaxed;
            (void)hipFree(p);
        }
        p = nullptr;
        bytes = 0;
    }
    void alloc(size_t b, const char *what) {
        release();
        p = dev_alloc(b, what);
        bytes = b;
    }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
};

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_n, long double)
void gauss_legendre(int n, double *x, double *w) {
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < n; ++i) {
        long double z = cosl(pi * (i + 0.75L) / (n + 0.5L)), dp = 0;
        for (int it = 0; it < 100; ++it) {
            long double p0 = 1, p1 = z;
            for (int k = 2; k <= n; ++k) {
                long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1);
            long double dz = p1 / dp;
            z -= dz;
            if (fabsl(dz) < 1e-19L) break;
        }
        x[i] = (double)z;
        w[i] = (double)(2.0L / ((1 - z * z) * dp * dp));
    }
}

// ---------------------------------------------------------------------------
// resident device tables
// ---------------------------------------------------------------------------

// twiddles exp(-2 pi i k / M), k < M, and half-angle phases exp(-i pi k / M),
// k <= M/2, in the plan precision (computed in long double, rounded)
struct Twiddles {
    int device, M, prec;
    DevBuf tw, ph;
};

// tw: exp(-2 pi i k / M) for k in [0, M), then the half-bin factors
//     exp(-i pi (2k + 1) / M) for k in [0, M/2) of the odd-frequency row
//     transforms.
// ph: exp(-i pi k / M) for k in [0, M/2] (corner phase of a y frequency),
//     then exp(-i pi (k + 1/2) / M) for k in [0, M/2) (corner phase of the
//     odd x frequency k + 1/2).
template <typename T> void fill_twiddles(int M, std::vector<T> &tw, std::vector<T> &ph) {
    const long double pi = 3.141592653589793238462643383279502884L;
    const int H = M / 2;
    tw.resize(2 * (size_t)(M + H));
    ph.resize(2 * (size_t)(H + 1 + H));
    auto put = [](std::vector<T> &v, size_t i, long double a) {
        v[2 * i] = (T)cosl(a);
        v[2 * i + 1] = (T)(-sinl(a));
    };
    for (int k = 0; k < M; ++k) put(tw, k, 2 * pi * k / M);
    for (int k = 0; k < H; ++k) put(tw, M + k, pi * (2 * k + 1) / M);
    for (int k = 0; k <= H; ++k) put(ph, k, pi * k / M);
    for (int k = 0; k < H; ++k) put(ph, H + 1 + k, pi * (k + 0.5L) / M);
}

std::shared_ptr<Twiddles> make_twiddles(int device, int M, int prec) {
    auto t = std::make_shared<Twiddles>();
    t->device = device;
    t->M = M;
    t->prec = prec;
    size_t esz = prec ? sizeof(double) : sizeof(float);
    t->tw.alloc(2 * esz * (M + M / 2), "twiddle table");
    t->ph.alloc(2 * esz * (M + 1), "phase table");
    if (prec) {
        std::vector<double> tw, ph;
        fill_twiddles<double>(M, tw, ph);
        hip_check(hipMemcpy(t->tw.p, tw.data(), tw.size() * sizeof(double), hipMemcpyHostToDevice), "twiddle upload");
        hip_check(hipMemcpy(t->ph.p, ph.data(), ph.size() * sizeof(double), hipMemcpyHostToDevice), "phase upload");
    } else {
        std::vector<float> tw, ph;
        fill_twiddles<float>(M, tw, ph);
        hip_check(hipMemcpy(t->tw.p, tw.data(), tw.size() * sizeof(float), hipMemcpyHostToDevice), "twiddle upload");
        hip_check(hipMemcpy(t->ph.p, ph.data(), ph.size() * sizeof(float), hipMemcpyHostToDevice), "phase upload");
    }
    return t;
}

// the kernel spectra of one family at one size, precision and target height
// (6 kinds in the midplane, 9 above it): per kind the odd x frequencies
// kx + 1/2, kx in [0, M/2), by the y frequencies ky in [0, M/2] (a half
// plane; negative ky follow from the kind's parity in y)
struct KernelSet {
    int device, M, prec, family;
    double zc;  // target height in finest cells
    DevBuf q;
    int64_t q_pitch, q_kstride;
};

std::mutex g_cache_mu;
std::map<std::tuple<int, int, int>, std::weak_ptr<Twiddles>> g_tw_cache;
std::map<std::tuple<int, int, int, int, double>, std::weak_ptr<KernelSet>> g_ks_cache;

std::shared_ptr<Twiddles> get_twiddles(int device, int M, int prec) {
    auto key = std::make_tuple(device, M, prec);
    auto it = g_tw_cache.find(key);
    if (it != g_tw_cache.end()) {
        if (auto sp = it->second.lock()) return sp;
    }
    auto sp = make_twiddles(device, M, prec);
    g_tw_cache[key] = sp;
    return sp;
}

std::shared_ptr<KernelSet> build_kernel_set(int device, int M, int prec, int family, double zc) {
    auto ks = std::make_shared<KernelSet>();
    ks->device = device;
    ks->M = M;
    ks->prec = prec;
    ks->family = family;
    ks->zc = zc;
    const int nkinds = zc != 0.0 ? 9 : 6;
    const int H = M / 2;
    ks->q_pitch = ((H + 1) + 63) / 64 * 64;
    ks->q_kstride = ks->q_pitch * H;
    const size_t esz = prec ? sizeof(double) : sizeof(float);
    ks->q.alloc(nkinds * esz * ks->q_kstride, "kernel spectra");
    // transient double-precision buffers
    DevBuf table(sizeof(double) * (size_t)M * M, "kernel table");
    DevBuf rows(sizeof(double) * 2 * (size_t)H * M, "kernel table row spectra");
    auto tw64 = get_twiddles(device, M, 1);
    TableArgs ta{};
    ta.out = (double *)table.p;
    ta.M = M;
    ta.family = family;
    ta.zc = zc;
    gauss_legendre(10, ta.glx, ta.glw);
    gauss_legendre(8, ta.glx8, ta.glw8);
    gauss_legendre(6, ta.glx6, ta.glw6);
    gauss_legendre(4, ta.glx4, ta.glw4);
    hipStream_t s = nullptr;
    for (int kind = 0; kind < nkinds; ++kind) {
        ta.kind = kind;
        hip_check(launch_ktable(ta, s), "kernel table build");
        Pack<RowFwdArgs<double>> rp{};
        RowFwdArgs<double> &ra = rp.a[0];
        ra.in[0] = (const double *)table.p;
        ra.scale[0] = 1.0;
        ra.in_pitch = M;
        ra.out = (C<double> *)rows.p;
        ra.out_pitch = M;
        ra.out_fstride = 0;
        ra.nrows = M;
        hip_check(launch_row_fwd<double>(rp, 1, M, 0, false, M, 1, (const C<double> *)tw64->tw.p, s),
                  "kernel table row transform");
        const int imag = imag_kind(kind) ? 1 : 0;
        if (prec) {
            hip_check(launch_col_extract<double>((const C<double> *)rows.p, M,
                                                 (double *)ks->q.p + kind * ks->q_kstride, ks->q_pitch,
                                                 imag, family, (const C<double> *)tw64->tw.p,
                                                 (const C<double> *)tw64->ph.p, s),
                      "kernel spectrum");
        } else {
            hip_check(launch_col_extract<float>((const C<double> *)rows.p, M,
                                                (float *)ks->q.p + kind * ks->q_kstride, ks->q_pitch,
                                                imag, family, (const C<double> *)tw64->tw.p,
                                                (const C<double> *)tw64->ph.p, s),
                      "kernel spectrum");
        }
    }
    hip_check(hipStreamSynchronize(s), "kernel spectra build");
    return ks;
}

std::shared_ptr<KernelSet> get_kernel_set(int device, int M, int prec, int family, double zc) {
    auto key = std::make_tuple(device, M, prec, family, zc);
    auto it = g_ks_cache.find(key);
    if (it != g_ks_cache.end()) {
        if (auto sp = it->second.lock()) return sp;
    }
    auto sp = build_kernel_set(device, M, prec, family, zc);
    g_ks_cache[key] = sp;
    return sp;
}

}  // namespace

// ---------------------------------------------------------------------------
// plans
// ---------------------------------------------------------------------------

struct gravity_plan_s {
    int device = 0;
    int prec = 0;
    int slopes = 1;
    double G = 1.0;
    int n0 = 0, nlevels = 1;
    double x0 = 0, y0 = 0, h0 = 0;
    std::vector<gravity_patch_t> patches;
    int nf = 0;  // finest lattice cells per side
    int M = 0;
    bool amr = false;
    int nfields = 3;
    double z = 0.0;  // target height (domain units); 0: midplane
    int ncomp = 2;   // force components: 2 in the midplane, 3 above it
    int64_t ncells = 0, nleaves = 0;
    std::shared_ptr<Twiddles> tw;
    std::shared_ptr<KernelSet> centre, corner;
    DevBuf owner, gmap;
    // kernel variants (row forward, column, row inverse), chosen at plan time
    int var_rf = 0, var_col = 0, var_ri = 0;
    // workspace layout (byte offsets)
    size_t off_a = 0, off_b = 0, off_o = 0, ws_bytes = 0;
    // GRAVITY_AMR_NESTED plans: sub-plans, box maps and workspace layout
    std::shared_ptr<struct NestedPlan> nest;
};

// Nested-correction plan data (see GRAVITY_AMR_NESTED in gravity.h).
struct NestedPlan {
    // uniform sub-plans: the base grid, the fine (kNestFine^2) and coarse
    // (kNestCoarse^2) region solves; they own twiddles, spectra and variants
    std::unique_ptr<gravity_plan_s> base, fine, coarse;
    int nbox = 0;                        // boxes over all refined levels
    std::vector<int> box0, nboxl;        // per level l (index l): first box, count
    std::vector<int64_t> r_off, r_cnt;   // per level l: restriction entries l -> l-1
    DevBuf fown, cown;                   // region owner maps [box][R][R]
    DevBuf rent;                         // restriction entries, 5 int32 each
    DevBuf leaf;                         // uint8 per composite cell
    // workspace byte offsets
    int64_t rstride = 0;  // elements per restricted composite array (cells + zero cell, padded)
    size_t off_r = 0, off_acc = 0, off_bws = 0, off_bout = 0;
    size_t off_fa = 0, off_fb = 0, off_fo = 0, off_ca = 0, off_cb = 0, off_co = 0;
};

namespace {

void validate_and_build_maps(gravity_plan_s &p, std::vector<int32_t> &owner, std::vector<int32_t> &gmap) {
    const int L = p.nlevels;
    // blocks: base then patches, composite offsets
    struct Blk {
        int level, i0, j0, nx, ny;
        int64_t off;
    };
    std::vector<Blk> blks;
    blks.push_back({0, 0, 0, p.n0, p.n0, 0});
    int64_t off = (int64_t)p.n0 * p.n0;
    for (auto &q : p.patches) {
        if (q.level < 1 || q.level >= L) fail(GRAVITY_EINVAL, "patch level out of range");
        if (q.nx <= 0 || q.ny <= 0) fail(GRAVITY_EINVAL, "empty patch");
        if ((q.i0 | q.j0 | q.nx | q.ny) & 1) fail(GRAVITY_EINVAL, "patch corners and sizes must be even");
        const int64_t nl = (int64_t)p.n0 << q.level;
        if (q.i0 < 0 || q.j0 < 0 || q.i0 + (int64_t)q.nx > nl || q.j0 + (int64_t)q.ny > nl)
            fail(GRAVITY_EINVAL, "patch outside the domain");
        blks.push_back({q.level, q.i0, q.j0, q.nx, q.ny, off});
        off += (int64_t)q.nx * q.ny;
    }
    p.ncells = off;
    if (off >= (1 << 28)) fail(GRAVITY_EUNSUPPORTED, "too many composite cells");
    const int nf = p.nf;
    // coverage per level: which block (index) covers each cell of that level
    // (as a map on that level's lattice), to find leaves and check nesting
    std::vector<std::vector<int32_t>> cover(L);
    for (int l = 0; l < L; ++l) {
        const int64_t n = (int64_t)p.n0 << l;
        cover[l].assign((size_t)(n * n), -1);
    }
    for (size_t b = 0; b < blks.size(); ++b) {
        const Blk &k = blks[b];
        const int64_t n = (int64_t)p.n0 << k.level;
        for (int j = 0; j < k.ny; ++j)
            for (int i = 0; i < k.nx; ++i) {
                int32_t &c = cover[k.level][(size_t)((k.j0 + j) * n + k.i0 + i)];
                if (c >= 0) fail(GRAVITY_EINVAL, "overlapping patches on one level");
                c = (int32_t)b;
            }
    }
    // nesting: every level-l cell covered by a patch must have a covered parent
    for (int l = 1; l < L; ++l) {
        const int64_t n = (int64_t)p.n0 << l;
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < n; ++i)
                if (cover[l][(size_t)(j * n + i)] >= 0 && cover[l - 1][(size_t)((j / 2) * (n / 2) + i / 2)] < 0)
                    fail(GRAVITY_EINVAL, "patch not nested inside the level below");
    }
    owner.assign((size_t)nf * nf, -1);
    gmap.assign((size_t)p.ncells, -1);
    int64_t leaves = 0;
    for (size_t b = 0; b < blks.size(); ++b) {
        const Blk &k = blks[b];
        const int l = k.level;
        const int64_t n = (int64_t)p.n0 << l;
        const int kb = L - 1 - l;  // log2 of finest cells per side of this level's cell
        const int B = 1 << kb;
        for (int j = 0; j < k.ny; ++j)
            for (int i = 0; i < k.nx; ++i) {
                const int64_t gi = k.i0 + i, gj = k.j0 + j;
                bool leaf = true;
                if (l + 1 < L) {
                    const int64_t nc = n * 2;
                    if (cover[l + 1][(size_t)((2 * gj) * nc + 2 * gi)] >= 0) leaf = false;
                }
                (void)n;
                if (!leaf) continue;
                ++leaves;
                const int64_t c = k.off + (int64_t)j * k.nx + i;
                for (int jj = 0; jj < B; ++jj)
                    for (int ii = 0; ii < B; ++ii) {
                        int32_t &o = owner[(size_t)((gj * B + jj) * nf + gi * B + ii)];
                        if (o >= 0) fail(GRAVITY_EINVAL, "leaves overlap");
                        o = (int32_t)c | (kb << 28);
                    }
                if (kb == 0) {
                    gmap[(size_t)c] = (int32_t)(gj * nf + gi);  // centre family, its own cell
                } else {
                    const int64_t I = gi * B + B / 2, J = gj * B + B / 2;  // centre vertex
                    gmap[(size_t)c] = (int32_t)(J * nf + I) | (1 << 30);
                }
            }
    }
    for (auto o : owner)
        if (o < 0) fail(GRAVITY_EINVAL, "leaves do not tile the domain");
    p.nleaves = leaves;
}

gravity_status_t finish(gravity_status_t st, const std::string &msg) {
    g_err = msg;
    return st;
}

template <typename F> gravity_status_t guarded(F &&fn) {
    try {
        fn();
        return GRAVITY_OK;
    } catch (const Failure &f) {
        return finish(f.st, f.msg);
    } catch (const std::bad_alloc &) {
        return finish(GRAVITY_ENOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return finish(GRAVITY_EDEVICE, e.what());
    } catch (...) {
        return finish(GRAVITY_EDEVICE, "unknown error");
    }
}

const char *const kStagesUniform[] = {"row_fwd", "col", "row_inv"};
const char *const kStagesAmr[] = {"row_fwd", "col", "row_inv", "gather"};

int n_stages(const gravity_plan_s &p) { return p.amr ? 4 : 3; }

// One solve's arguments (device pointers) and workspace.
struct Item {
    const gravity_plan_s *p;
    const void *s, *dx, *dy;
    void *fx, *fy;
    char *ws;
    void *fz = nullptr;  // off-plane plans only
};

// Solves that can share every launch: same precision, size, fields, layout
// kind and kernel variants.
bool same_group(const gravity_plan_s &a, const gravity_plan_s &b) {
    if (a.nest || b.nest) return &a == &b;  // nested solves run one by one (run_items)
    return a.prec == b.prec && a.M == b.M && a.nfields == b.nfields && a.amr == b.amr &&
           a.ncomp == b.ncomp &&
           a.var_rf == b.var_rf && a.var_col == b.var_col && a.var_ri == b.var_ri &&
           a.device == b.device;
}

// Queue n (1..kPack) solves of one group; ev: optional n_stages + 1 events
// recorded between the stages.  srep > 1 (timing only) launches every stage
// srep times back to back between its two events; each stage rewrites its
// whole output from its input, so the repeats leave the result unchanged.
template <typename T>
void run_group(const Item *it, int n, hipStream_t s, hipEvent_t *ev = nullptr, int srep = 1) {
    const gravity_plan_s &p0 = *it[0].p;
    const int nf = p0.nf, M = p0.M, H = M / 2;
    const int NF = p0.nfields;
    const int nfam = p0.amr ? 2 : 1;
    const int NC = p0.ncomp;
    const C<T> *tw = (const C<T> *)p0.tw->tw.p;
    const C<T> *ph = (const C<T> *)p0.tw->ph.p;
    const int64_t colsz = (int64_t)H * nf;  // M/2 spectral columns of nf rows
    const int64_t n2 = (int64_t)nf * nf;
    int stage = 0;
    auto mark = [&]() {
        if (ev) hip_check(hipEventRecord(ev[stage++], s), "hipEventRecord");
    };

    Pack<RowFwdArgs<T>> rf{};
    for (int i = 0; i < n; ++i) {
        const gravity_plan_s &p = *it[i].p;
        const T h = (T)(p.h0 / (double)(1 << (p.nlevels - 1)));
        RowFwdArgs<T> &ra = rf.a[i];
        // uniform: the caller's fields; AMR: the leaf arrays, injected onto
        // the finest lattice by the row kernel's load through the owner map
        ra.in[0] = (const T *)it[i].s;
        ra.in[1] = (const T *)it[i].dx;
        ra.in[2] = (const T *)it[i].dy;
        ra.owner = p.amr ? (const int32_t *)p.owner.p : nullptr;
        ra.hf = h;
        ra.slopes = NF == 3;
        ra.scale[0] = (T)1;
        ra.scale[1] = h;
        ra.scale[2] = h;
        ra.in_pitch = nf;
        ra.out = (C<T> *)(it[i].ws + p.off_a);
        ra.out_pitch = nf;
        ra.out_fstride = colsz;
        ra.nrows = nf;
    }
    mark();
    for (int r = 0; r < srep; ++r)
        hip_check(launch_row_fwd<T>(rf, n, M, p0.var_rf, true, nf, NF, tw, s), "row transform");

    Pack<ColArgs<T>> cp{};
    for (int i = 0; i < n; ++i) {
        const gravity_plan_s &p = *it[i].p;
        ColArgs<T> &ca = cp.a[i];
        ca.in = rf.a[i].out;
        ca.in_pitch = nf;
        ca.in_fstride = colsz;
        ca.q[0] = (const T *)p.centre->q.p;
        ca.q[1] = p.amr ? (const T *)p.corner->q.p : (const T *)p.centre->q.p;
        ca.q_pitch = p.centre->q_pitch;
        ca.q_kstride = p.centre->q_kstride;
        ca.out = (C<T> *)(it[i].ws + p.off_b);
        ca.out_pitch = nf;
        ca.out_gstride = colsz;
        ca.nsub = 1;
        ca.sub_off = 0;
    }
    mark();
    for (int r = 0; r < srep; ++r)
        hip_check(launch_col<T>(cp, n, M, p0.var_col, NF, nfam, NC, tw, ph, s), "column transform");

    Pack<RowInvArgs<T>> ip{};
    for (int i = 0; i < n; ++i) {
        const gravity_plan_s &p = *it[i].p;
        RowInvArgs<T> &ia = ip.a[i];
        ia.in = cp.a[i].out;
        ia.in_pitch = nf;
        ia.in_gstride = colsz;
        ia.out_pitch = nf;
        ia.scale = (T)(p.G / ((double)M * (double)M));
        ia.nrows = nf;
        if (!p.amr) {
            ia.out[0] = (T *)it[i].fx;
            ia.out[1] = (T *)it[i].fy;
            ia.out[2] = (T *)it[i].fz;  // used when NC == 3
        } else {
            T *O = (T *)(it[i].ws + p.off_o);
            for (int g = 0; g < NC * nfam; ++g) ia.out[g] = O + g * n2;
        }
    }
    mark();
    for (int r = 0; r < srep; ++r)
        hip_check(launch_row_inv<T>(ip, n, M, p0.var_ri, nf, NC * nfam, tw, s), "inverse row transform");

    if (p0.amr) {
        Pack<GatherArgs<T>> gp{};
        int64_t maxc = 0;
        for (int i = 0; i < n; ++i) {
            const gravity_plan_s &p = *it[i].p;
            GatherArgs<T> &ga = gp.a[i];
            ga.gmap = (const int32_t *)p.gmap.p;
            for (int g = 0; g < NC * nfam; ++g) ga.o[g] = ip.a[i].out[g];
            ga.fx = (T *)it[i].fx;
            ga.fy = (T *)it[i].fy;
            ga.fz = (T *)it[i].fz;
            ga.n = p.ncells;
            ga.ncomp = NC;
            maxc = std::max<int64_t>(maxc, p.ncells);
        }
        mark();
        for (int r = 0; r < srep; ++r) hip_check(launch_gather<T>(gp, n, maxc, s), "gather");
    }
    mark();
}

// One batched pass of region solves (all boxes of all refined levels, one
// launch per kernel): level l is item l - 1 of each pack, its boxes' rows
// stacked (the row kernels see nbox_l * R rows, the column kernel one
// sub-item per box).  Inputs are the restricted composite arrays, injected
// on load through the boxes' region owner maps.
template <typename T>
void run_regions(const gravity_plan_s &p, const gravity_plan_s &sp, int R, int coarse, const int32_t *own,
                 const T *const *in, char *A, char *B, char *O, hipStream_t s) {
    const NestedPlan &N = *p.nest;
    const int M = 2 * R, H = M / 2;
    const int64_t TR = (int64_t)N.nbox * R;  // stacked rows of all boxes
    const C<T> *tw = (const C<T> *)sp.tw->tw.p;
    const C<T> *ph = (const C<T> *)sp.tw->ph.p;
    Pack<RowFwdArgs<T>> rf{};
    Pack<ColArgs<T>> cp{};
    Pack<RowInvArgs<T>> ip{};
    int n = 0, maxsub = 1;
    int64_t maxrows = 0;
    for (int l = 1; l < p.nlevels; ++l) {
        const int nb = N.nboxl[l];
        if (nb == 0) continue;
        const int64_t b0 = N.box0[l];
        const int m = coarse ? l - 1 : l;  // level of the region lattice
        const T h = (T)(p.h0 / (double)(1 << m));
        RowFwdArgs<T> &ra = rf.a[n];
        for (int f = 0; f < 3; ++f) ra.in[f] = in[f];
        ra.scale[0] = (T)1;
        ra.scale[1] = h;
        ra.scale[2] = h;
        ra.in_pitch = R;
        ra.owner = own + b0 * R * R;
        ra.hf = h;
        ra.slopes = 1;
        ra.out = (C<T> *)A + b0 * R;
        ra.out_pitch = TR;
        ra.out_fstride = H * TR;
        ra.nrows = (int64_t)nb * R;
        ColArgs<T> &ca = cp.a[n];
        ca.in = ra.out;
        ca.in_pitch = TR;
        ca.in_fstride = H * TR;
        ca.q[0] = ca.q[1] = (const T *)sp.centre->q.p;
        ca.q_pitch = sp.centre->q_pitch;
        ca.q_kstride = sp.centre->q_kstride;
        ca.out = (C<T> *)B + b0 * R;
        ca.out_pitch = TR;
        ca.out_gstride = H * TR;
        ca.nsub = nb;
        ca.sub_off = R;
        RowInvArgs<T> &ia = ip.a[n];
        ia.in = ca.out;
        ia.in_pitch = TR;
        ia.in_gstride = H * TR;
        ia.out[0] = (T *)O + b0 * R * R;
        ia.out[1] = (T *)O + TR * R + b0 * R * R;
        ia.out_pitch = R;
        ia.scale = (T)(p.G / ((double)M * (double)M));
        ia.nrows = (int64_t)nb * R;
        maxrows = std::max(maxrows, ra.nrows);
        maxsub = std::max(maxsub, nb);
        ++n;
    }
    if (n == 0) return;
    hip_check(launch_row_fwd<T>(rf, n, M, sp.var_rf, true, maxrows, 3, tw, s), "region row transform");
    hip_check(launch_col<T>(cp, n, M, sp.var_col, 3, 1, 2, tw, ph, s, maxsub), "region column transform");
    hip_check(launch_row_inv<T>(ip, n, M, sp.var_ri, maxrows, 2, tw, s), "region inverse row transform");
}

template <typename T> void run_nested(const Item &it, hipStream_t s) {
    const gravity_plan_s &p = *it.p;
    const NestedPlan &N = *p.nest;
    const int64_t nc = p.ncells;
    char *ws = it.ws;
    T *rs = (T *)(ws + N.off_r), *rdx = rs + N.rstride, *rdy = rdx + N.rstride;
    double *accx = (double *)(ws + N.off_acc), *accy = accx + nc;
    hip_check(launch_nest_copy_in<T>((const T *)it.s, p.nfields == 3 ? (const T *)it.dx : nullptr,
                                     p.nfields == 3 ? (const T *)it.dy : nullptr, rs, rdx, rdy, nc, s),
              "nested copy-in");
    for (int l = p.nlevels - 1; l >= 1; --l) {
        RestrictArgs<T> ra{rs, rdx, rdy, (const int32_t *)N.rent.p + 5 * N.r_off[l], N.r_cnt[l],
                           p.h0 / (double)(1 << (l - 1))};
        hip_check(launch_nest_restrict<T>(ra, s), "nested restriction");
    }
    // level 0: the base grid with restricted data, solved exactly
    const int64_t n0sq = (int64_t)p.n0 * p.n0;
    T *bfx = (T *)(ws + N.off_bout), *bfy = bfx + n0sq;
    Item bi{N.base.get(), rs, rdx, rdy, bfx, bfy, ws + N.off_bws};
    run_group<T>(&bi, 1, s);
    hip_check(launch_nest_lift<T>(bfx, bfy, accx, accy, n0sq, s), "nested lift");
    const T *in[3] = {rs, rdx, rdy};
    run_regions<T>(p, *N.fine, kNestFine, 0, (const int32_t *)N.fown.p, in, ws + N.off_fa, ws + N.off_fb,
                   ws + N.off_fo, s);
    run_regions<T>(p, *N.coarse, kNestCoarse, 1, (const int32_t *)N.cown.p, in, ws + N.off_ca,
                   ws + N.off_cb, ws + N.off_co, s);
    const int64_t fplane = (int64_t)N.nbox * kNestFine * kNestFine;
    const int64_t cplane = (int64_t)N.nbox * kNestCoarse * kNestCoarse;
    const T *ffo = (const T *)(ws + N.off_fo), *cfo = (const T *)(ws + N.off_co);
    for (int l = 1; l < p.nlevels; ++l) {
        const int64_t b0 = N.box0[l];
        CombineArgs<T> ca{(const int32_t *)N.fown.p + b0 * kNestFine * kNestFine,
                          (const int32_t *)N.cown.p + b0 * kNestCoarse * kNestCoarse,
                          ffo + b0 * kNestFine * kNestFine,
                          ffo + fplane + b0 * kNestFine * kNestFine,
                          cfo + b0 * kNestCoarse * kNestCoarse,
                          cfo + cplane + b0 * kNestCoarse * kNestCoarse,
                          accx, accy, (int32_t)nc, N.nboxl[l]};
        hip_check(launch_nest_combine<T>(ca, s), "nested level combine");
    }
    hip_check(launch_nest_finalize<T>(accx, accy, (const uint8_t *)N.leaf.p, (T *)it.fx, (T *)it.fy, nc, s),
              "nested finalize");
}

void run_items(const Item *it, int n, hipStream_t s, hipEvent_t *ev = nullptr) {
    if (it[0].p->nest) {  // never grouped: one at a time
        for (int i = 0; i < n; ++i) {
            if (it[i].p->prec)
                run_nested<double>(it[i], s);
            else
                run_nested<float>(it[i], s);
        }
        return;
    }
    if (it[0].p->prec)
        run_group<double>(it, n, s, ev);
    else
        run_group<float>(it, n, s, ev);
}

// single solve entry used by the autotuner and the profiling call
template <typename T>
void solve_t(const gravity_plan_s &p, const void *sigma, const void *dsx, const void *dsy, void *fx,
             void *fy, char *ws, hipStream_t s, hipEvent_t *ev = nullptr, int srep = 1,
             void *fz = nullptr) {
    Item it{&p, sigma, dsx, dsy, fx, fy, ws, fz};
    run_group<T>(&it, 1, s, ev, srep);
}

// ---------------------------------------------------------------------------
// autotuner: per (device, M, precision, fields, families) pick the fastest
// variant of each solve kernel by timing all of them on scratch buffers.
// GRAVITY_AUTOTUNE=0 keeps the defaults; GRAVITY_VARIANTS="rf,col,ri" forces
// a choice; GRAVITY_TUNE_FILE names a text file that persists choices.
// ---------------------------------------------------------------------------
struct Variants {
    int rf, col, ri;
};
// key: device, M, precision, fields, families, components
std::map<std::tuple<std::string, int, int, int, int, int>, Variants> g_tuned;
bool g_tune_file_loaded = false;

std::string device_key(int device) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
    std::string s = prop.gcnArchName;
    for (auto &c : s)
        if (c == ' ') c = '_';
    return s + "/" + std::to_string(prop.multiProcessorCount);
}

void load_tune_file() {
    if (g_tune_file_loaded) return;
    g_tune_file_loaded = true;
    const char *path = std::getenv("GRAVITY_TUNE_FILE");
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char dev[256];
    int M, prec, nf, nfam, nc, rf, col, ri;
    while (std::fscanf(f, "%255s %d %d %d %d %d %d %d %d", dev, &M, &prec, &nf, &nfam, &nc, &rf, &col,
                       &ri) == 9)
        g_tuned[std::make_tuple(std::string(dev), M, prec, nf, nfam, nc)] = Variants{rf, col, ri};
    std::fclose(f);
}

void save_tune_entry(const std::string &dev, int M, int prec, int nf, int nfam, int nc, const Variants &v) {
    const char *path = std::getenv("GRAVITY_TUNE_FILE");
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d %d %d %d %d %d %d\n", dev.c_str(), M, prec, nf, nfam, nc, v.rf, v.col, v.ri);
    std::fclose(f);
}

bool col_ok(const gravity_plan_s &p, int v) {
    return col_variant_valid(p.prec, p.M, v, p.nfields, p.amr ? 2 : 1, p.ncomp);
}

Variants default_variants(const gravity_plan_s &p) {
    Variants v{1, 0, 1};
    if (!row_variant_valid(p.prec, p.M, v.rf)) v.rf = 0;
    if (!row_variant_valid(p.prec, p.M, v.ri)) v.ri = 0;
    if (!col_ok(p, v.col)) v.col = 0;
    return v;
}

template <typename T> Variants autotune(gravity_plan_s &p) {
    const int M = p.M;
    const int ns = n_stages(p);
    const int s_rf = 0, s_col = 1, s_ri = 2;  // stage indices (AMR adds the gather last)
    DevBuf ws(p.ws_bytes, "autotune workspace");
    DevBuf in(3 * sizeof(T) * (size_t)p.ncells, "autotune inputs");
    DevBuf out(3 * sizeof(T) * (size_t)p.ncells, "autotune outputs");
    hip_check(hipMemset(in.p, 0, in.bytes), "autotune memset");
    const T *sg = (const T *)in.p;
    std::vector<hipEvent_t> ev(ns + 1, nullptr);
    Variants best = default_variants(p);
    struct EvGuard {
        std::vector<hipEvent_t> &e;
        ~EvGuard() {
            for (auto x : e)
                if (x) (void)hipEventDestroy(x);
        }
    } guard{ev};
    for (auto &e : ev) hip_check(hipEventCreate(&e), "hipEventCreate");
    double tb[3] = {1e300, 1e300, 1e300};
    const int reps = M >= 4096 ? 3 : 8;
    for (int v = 0; v < kNumVariants; ++v) {
        const bool okr = row_variant_valid(p.prec, M, v), okc = col_ok(p, v);
        if (!okr && !okc) continue;
        p.var_rf = okr ? v : best.rf;
        p.var_ri = okr ? v : best.ri;
        p.var_col = okc ? v : best.col;
        double acc[8] = {0};
        for (int r = 0; r < 2; ++r) {  // warm-up, then every stage reps times back to back
            solve_t<T>(p, sg, sg + p.ncells, sg + 2 * p.ncells, out.p, (T *)out.p + p.ncells,
                       (char *)ws.p, nullptr, ev.data(), r == 0 ? 1 : reps, (T *)out.p + 2 * p.ncells);
            hip_check(hipEventSynchronize(ev[ns]), "hipEventSynchronize");
            if (r == 0) continue;
            for (int k = 0; k < ns; ++k) {
                float ms = 0;
                hip_check(hipEventElapsedTime(&ms, ev[k], ev[k + 1]), "hipEventElapsedTime");
                acc[k] += ms;
            }
        }
        if (okr && acc[s_rf] < tb[0]) { tb[0] = acc[s_rf]; best.rf = v; }
        if (okc && acc[s_col] < tb[1]) { tb[1] = acc[s_col]; best.col = v; }
        if (okr && acc[s_ri] < tb[2]) { tb[2] = acc[s_ri]; best.ri = v; }
    }
    return best;
}

void choose_variants(gravity_plan_s &p) {
    const char *force = std::getenv("GRAVITY_VARIANTS");
    if (force && *force) {
        int a = 0, b = 0, c = 0;
        if (std::sscanf(force, "%d,%d,%d", &a, &b, &c) != 3 || !row_variant_valid(p.prec, p.M, a) ||
            !col_ok(p, b) || !row_variant_valid(p.prec, p.M, c))
            fail(GRAVITY_EINVAL, "GRAVITY_VARIANTS must be three valid variant ids 'rf,col,ri'");
        p.var_rf = a;
        p.var_col = b;
        p.var_ri = c;
        return;
    }
    Variants v = default_variants(p);
    const char *at = std::getenv("GRAVITY_AUTOTUNE");
    if (!(at && std::string(at) == "0")) {
        load_tune_file();
        const std::string dev = device_key(p.device);
        auto key = std::make_tuple(dev, p.M, p.prec, p.nfields, p.amr ? 2 : 1, p.ncomp);
        auto it = g_tuned.find(key);
        // an entry of a tune file written by another build may name a
        // variant this build does not have: tune again then
        if (it != g_tuned.end() && row_variant_valid(p.prec, p.M, it->second.rf) &&
            col_ok(p, it->second.col) && row_variant_valid(p.prec, p.M, it->second.ri)) {
            v = it->second;
        } else {
            v = p.prec ? autotune<double>(p) : autotune<float>(p);
            g_tuned[key] = v;
            save_tune_entry(dev, p.M, p.prec, p.nfields, p.amr ? 2 : 1, p.ncomp, v);
        }
    }
    p.var_rf = v.rf;
    p.var_col = v.col;
    p.var_ri = v.ri;
}

}  // namespace

// ---------------------------------------------------------------------------
// nested-correction plans: layout validation and maps without any lattice
// finer than a box region (the finest lattice may reach 2^30 cells per side)
// ---------------------------------------------------------------------------
struct PatchRec {
    int level, i0, j0, nx, ny;
    int64_t off;  // composite offset of the patch's first cell
};

// patches of one level binned by kNestBox x kNestBox cell tiles, for lookups
struct LevelBins {
    int64_t n = 0;  // lattice cells per side at this level
    int64_t nb = 0;
    std::unordered_map<int64_t, std::vector<int>> bins;
    void add(const PatchRec &q, int id) {
        for (int64_t by = q.j0 / kNestBox; by <= (q.j0 + q.ny - 1) / kNestBox; ++by)
            for (int64_t bx = q.i0 / kNestBox; bx <= (q.i0 + q.nx - 1) / kNestBox; ++bx)
                bins[by * nb + bx].push_back(id);
    }
    const std::vector<int> *at(int64_t gi, int64_t gj) const {
        auto it = bins.find((gj / kNestBox) * nb + gi / kNestBox);
        return it == bins.end() ? nullptr : &it->second;
    }
};

int64_t rect_overlap(int64_t ax0, int64_t ax1, int64_t ay0, int64_t ay1, int64_t bx0, int64_t bx1,
                     int64_t by0, int64_t by1) {
    const int64_t w = std::min(ax1, bx1) - std::max(ax0, bx0);
    const int64_t h = std::min(ay1, by1) - std::max(ay0, by0);
    return (w > 0 && h > 0) ? w * h : 0;
}

// owner map of a region of the level-m lattice, R x R cells from (RX, RY):
// the composite index of the finest cell of level <= m covering each region
// cell | log2(its size in level-m cells) << 28; `sentinel` outside the domain
void region_owner(const gravity_plan_s &p, const std::vector<PatchRec> &pr, int m, int64_t RX, int64_t RY,
                  int R, int32_t sentinel, int32_t *out) {
    const int64_t nm = (int64_t)p.n0 << m;
    for (int y = 0; y < R; ++y)
        for (int x = 0; x < R; ++x) {
            const int64_t gx = RX + x, gy = RY + y;
            int32_t v = sentinel;
            if (gx >= 0 && gy >= 0 && gx < nm && gy < nm)
                v = (int32_t)((gy >> m) * p.n0 + (gx >> m)) | (m << 28);
            out[(size_t)y * R + x] = v;
        }
    for (int k = 1; k <= m; ++k) {
        const int sh = m - k;
        for (const PatchRec &q : pr) {
            if (q.level != k) continue;
            const int64_t x0 = std::max<int64_t>(RX, (int64_t)q.i0 << sh);
            const int64_t x1 = std::min<int64_t>(RX + R, (int64_t)(q.i0 + q.nx) << sh);
            const int64_t y0 = std::max<int64_t>(RY, (int64_t)q.j0 << sh);
            const int64_t y1 = std::min<int64_t>(RY + R, (int64_t)(q.j0 + q.ny) << sh);
            for (int64_t gy = y0; gy < y1; ++gy)
                for (int64_t gx = x0; gx < x1; ++gx) {
                    const int64_t c = q.off + ((gy >> sh) - q.j0) * q.nx + ((gx >> sh) - q.i0);
                    out[(size_t)(gy - RY) * R + (gx - RX)] = (int32_t)c | (sh << 28);
                }
        }
    }
}

std::unique_ptr<gravity_plan_s> sub_plan(const gravity_plan_s &p, int n, double h0) {
    gravity_desc_t d{};
    d.n0x = d.n0y = n;
    d.x0 = p.x0;
    d.y0 = p.y0;
    d.h0 = h0;
    d.nlevels = 1;
    d.prec = (gravity_prec_t)p.prec;
    d.slopes = GRAVITY_SLOPES_GIVEN;
    d.G = p.G;
    gravity_plan_t sp = nullptr;
    const gravity_status_t st = gravity_plan(&d, &sp);
    if (st != GRAVITY_OK) fail(st, std::string("nested sub-plan: ") + gravity_last_error());
    return std::unique_ptr<gravity_plan_s>(sp);
}

void build_nested(gravity_plan_s &p) {
    const int L = p.nlevels;
    auto N = std::make_shared<NestedPlan>();
    // patches, composite offsets, validity
    std::vector<PatchRec> pr;
    int64_t off = (int64_t)p.n0 * p.n0;
    std::vector<LevelBins> lb(L);
    for (int l = 0; l < L; ++l) {
        lb[l].n = (int64_t)p.n0 << l;
        lb[l].nb = (lb[l].n + kNestBox - 1) / kNestBox;
    }
    for (auto &q : p.patches) {
        if (q.level < 1 || q.level >= L) fail(GRAVITY_EINVAL, "patch level out of range");
        if (q.nx <= 0 || q.ny <= 0) fail(GRAVITY_EINVAL, "empty patch");
        if ((q.i0 | q.j0 | q.nx | q.ny) & 1) fail(GRAVITY_EINVAL, "patch corners and sizes must be even");
        const int64_t nl = (int64_t)p.n0 << q.level;
        if (q.i0 < 0 || q.j0 < 0 || q.i0 + (int64_t)q.nx > nl || q.j0 + (int64_t)q.ny > nl)
            fail(GRAVITY_EINVAL, "patch outside the domain");
        pr.push_back(PatchRec{q.level, q.i0, q.j0, q.nx, q.ny, off});
        off += (int64_t)q.nx * q.ny;
        if (off >= (1 << 28) - 1) fail(GRAVITY_EUNSUPPORTED, "too many composite cells");
    }
    p.ncells = off;
    for (size_t k = 0; k < pr.size(); ++k) lb[pr[k].level].add(pr[k], (int)k);
    // no overlap within a level
    for (int l = 1; l < L; ++l)
        for (auto &kv : lb[l].bins) {
            const auto &v = kv.second;
            for (size_t a = 0; a < v.size(); ++a)
                for (size_t b = a + 1; b < v.size(); ++b) {
                    const PatchRec &A = pr[v[a]], &Bq = pr[v[b]];
                    if (rect_overlap(A.i0, A.i0 + A.nx, A.j0, A.j0 + A.ny, Bq.i0, Bq.i0 + Bq.nx, Bq.j0,
                                     Bq.j0 + Bq.ny))
                        fail(GRAVITY_EINVAL, "overlapping patches on one level");
                }
        }
    // composite index of the level-k cell (gi, gj), -1 if level k has none
    auto lookup = [&](int k, int64_t gi, int64_t gj) -> int64_t {
        if (k == 0) return gj * p.n0 + gi;
        const std::vector<int> *v = lb[k].at(gi, gj);
        if (!v) return -1;
        for (int id : *v) {
            const PatchRec &q = pr[id];
            if (gi >= q.i0 && gi < q.i0 + q.nx && gj >= q.j0 && gj < q.j0 + q.ny)
                return q.off + (gj - q.j0) * q.nx + (gi - q.i0);
        }
        return -1;
    };
    // nesting, leaves and the restriction entries (children level l -> l-1)
    std::vector<uint8_t> leaf((size_t)p.ncells, 1);
    std::vector<std::vector<int32_t>> ent(L);
    for (const PatchRec &q : pr) {
        const int l = q.level;
        for (int64_t J = q.j0 / 2; J < (q.j0 + q.ny) / 2; ++J)
            for (int64_t I = q.i0 / 2; I < (q.i0 + q.nx) / 2; ++I) {
                const int64_t c = lookup(l - 1, I, J);
                if (c < 0) fail(GRAVITY_EINVAL, "patch not nested inside the level below");
                leaf[(size_t)c] = 0;
                const int64_t ci = 2 * I - q.i0, cj = 2 * J - q.j0;
                auto child = [&](int a, int b) { return (int32_t)(q.off + (cj + b) * q.nx + ci + a); };
                ent[l].insert(ent[l].end(), {(int32_t)c, child(0, 0), child(1, 0), child(0, 1), child(1, 1)});
            }
    }
    int64_t leaves = 0;
    for (auto v : leaf) leaves += v;
    p.nleaves = leaves;
    N->r_off.assign(L, 0);
    N->r_cnt.assign(L, 0);
    std::vector<int32_t> rent;
    for (int l = 1; l < L; ++l) {
        N->r_off[l] = (int64_t)rent.size() / 5;
        N->r_cnt[l] = (int64_t)ent[l].size() / 5;
        rent.insert(rent.end(), ent[l].begin(), ent[l].end());
    }
    // boxes of every refined level, ordered by level then (by, bx)
    N->box0.assign(L, 0);
    N->nboxl.assign(L, 0);
    std::vector<std::pair<int, std::pair<int64_t, int64_t>>> boxes;  // (level, (by, bx))
    for (int l = 1; l < L; ++l) {
        std::vector<std::pair<int64_t, int64_t>> bl;
        for (const PatchRec &q : pr) {
            if (q.level != l) continue;
            for (int64_t by = q.j0 / kNestBox; by <= (q.j0 + q.ny - 1) / kNestBox; ++by)
                for (int64_t bx = q.i0 / kNestBox; bx <= (q.i0 + q.nx - 1) / kNestBox; ++bx)
                    bl.push_back({by, bx});
        }
        std::sort(bl.begin(), bl.end());
        bl.erase(std::unique(bl.begin(), bl.end()), bl.end());
        N->box0[l] = (int)boxes.size();
        N->nboxl[l] = (int)bl.size();
        if (bl.size() > 65535) fail(GRAVITY_EUNSUPPORTED, "more than 65535 boxes on one level");
        for (auto &b : bl) boxes.push_back({l, b});
    }
    N->nbox = (int)boxes.size();
    const int32_t sentinel = (int32_t)p.ncells;
    std::vector<int32_t> fown((size_t)N->nbox * kNestFine * kNestFine);
    std::vector<int32_t> cown((size_t)N->nbox * kNestCoarse * kNestCoarse);
    for (int b = 0; b < N->nbox; ++b) {
        const int l = boxes[b].first;
        const int64_t X0 = boxes[b].second.second * kNestBox, Y0 = boxes[b].second.first * kNestBox;
        region_owner(p, pr, l, X0 - kNestExt, Y0 - kNestExt, kNestFine, sentinel,
                     fown.data() + (size_t)b * kNestFine * kNestFine);
        region_owner(p, pr, l - 1, X0 / 2 - kNestExt / 2, Y0 / 2 - kNestExt / 2, kNestCoarse, sentinel,
                     cown.data() + (size_t)b * kNestCoarse * kNestCoarse);
    }
    // every index the kernels will follow stays inside its array
    for (auto *v : {&fown, &cown})
        for (int32_t o : *v)
            if ((o & 0x0FFFFFFF) > sentinel || ((o >> 28) & 0xF) > kNestMaxLevels)
                fail(GRAVITY_EDEVICE, "internal error: nested region map out of range");
    for (int32_t c : rent)
        if (c < 0 || c >= sentinel) fail(GRAVITY_EDEVICE, "internal error: restriction entry out of range");
    // sub-plans (kernel spectra and variants of the three uniform sizes)
    N->base = sub_plan(p, p.n0, p.h0);
    N->fine = sub_plan(p, kNestFine, 2.0 / kNestFine);
    N->coarse = sub_plan(p, kNestCoarse, 2.0 / kNestCoarse);
    // device maps
    auto upload = [](DevBuf &d, const void *src, size_t bytes, const char *what) {
        d.alloc(bytes, what);
        if (bytes) hip_check(hipMemcpy(d.p, src, bytes, hipMemcpyHostToDevice), what);
    };
    upload(N->fown, fown.data(), fown.size() * sizeof(int32_t), "nested fine region maps");
    upload(N->cown, cown.data(), cown.size() * sizeof(int32_t), "nested coarse region maps");
    upload(N->rent, rent.data(), rent.size() * sizeof(int32_t), "nested restriction entries");
    upload(N->leaf, leaf.data(), leaf.size(), "nested leaf flags");
    // workspace layout
    const size_t esz = p.prec ? sizeof(double) : sizeof(float);
    const int64_t nc = p.ncells, n0sq = (int64_t)p.n0 * p.n0, nb = N->nbox;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align256(bytes);
        return at;
    };
    N->rstride = (nc + 1 + 63) / 64 * 64;  // keeps every array two-element aligned
    N->off_r = take(3 * esz * (size_t)N->rstride);
    N->off_acc = take(2 * sizeof(double) * (size_t)nc);
    N->off_bws = take(N->base->ws_bytes);
    N->off_bout = take(2 * esz * (size_t)n0sq);
    const size_t fcols = (size_t)kNestFine * nb * kNestFine, ccols = (size_t)kNestCoarse * nb * kNestCoarse;
    N->off_fa = take(3 * 2 * esz * fcols);   // M/2 = kNestFine columns of nb * kNestFine rows
    N->off_fb = take(2 * 2 * esz * fcols);
    N->off_fo = take(2 * esz * fcols);
    N->off_ca = take(3 * 2 * esz * ccols);
    N->off_cb = take(2 * 2 * esz * ccols);
    N->off_co = take(2 * esz * ccols);
    p.ws_bytes = o;
    p.nest = N;
    p.var_rf = N->base->var_rf;
    p.var_col = N->base->var_col;
    p.var_ri = N->base->var_ri;
}

extern "C" {

gravity_status_t gravity_plan(const gravity_desc_t *d, gravity_plan_t *out) {
    if (out) *out = nullptr;
    return guarded([&] {
        if (!d || !out) fail(GRAVITY_EINVAL, "NULL descriptor or output");
        if (d->n0x != d->n0y) fail(GRAVITY_EUNSUPPORTED, "only square base grids are supported");
        if (!is_pow2(d->n0x)) fail(GRAVITY_EUNSUPPORTED, "base size must be a power of two");
        if (d->nlevels < 1 || d->nlevels > 8) fail(GRAVITY_EINVAL, "nlevels must be 1..8");
        if (!(d->h0 > 0) || !std::isfinite(d->h0) || !std::isfinite(d->x0) || !std::isfinite(d->y0) ||
            !std::isfinite(d->z))
            fail(GRAVITY_EINVAL, "bad geometry");
        if (d->prec != GRAVITY_F32 && d->prec != GRAVITY_F64) fail(GRAVITY_EINVAL, "bad precision");
        if (d->slopes != GRAVITY_SLOPES_NONE && d->slopes != GRAVITY_SLOPES_GIVEN)
            fail(GRAVITY_EINVAL, "bad slope mode");
        if (d->npatches < 0 || (d->npatches > 0 && !d->patches)) fail(GRAVITY_EINVAL, "bad patch list");
        if (d->nlevels == 1 && d->npatches > 0) fail(GRAVITY_EINVAL, "patches need nlevels > 1");
        if (d->amr_method != GRAVITY_AMR_EXACT && d->amr_method != GRAVITY_AMR_NESTED)
            fail(GRAVITY_EINVAL, "bad AMR method");
        const bool nested = d->amr_method == GRAVITY_AMR_NESTED && d->nlevels > 1;
        const int64_t nf = (int64_t)d->n0x << (d->nlevels - 1);
        if (nested) {
            if (d->n0x < 16 || d->n0x > kMaxM / 2)
                fail(GRAVITY_EUNSUPPORTED, "nested AMR: base grid must have 16..4096 cells per side");
            if (d->nlevels > kNestMaxLevels) fail(GRAVITY_EUNSUPPORTED, "nested AMR: at most 6 levels");
            if (d->z != 0.0) fail(GRAVITY_EUNSUPPORTED, "nested AMR: midplane targets only");
        } else if (nf < 16 || nf > kMaxM / 2) {
            fail(GRAVITY_EUNSUPPORTED, "finest lattice must have 16..4096 cells per side");
        }
        auto p = std::make_unique<gravity_plan_s>();
        p->prec = d->prec;
        p->slopes = d->slopes;
        p->G = d->G;
        p->z = d->z;
        p->ncomp = d->z != 0.0 ? 3 : 2;
        p->n0 = d->n0x;
        p->nlevels = d->nlevels;
        p->x0 = d->x0;
        p->y0 = d->y0;
        p->h0 = d->h0;
        p->patches.assign(d->patches, d->patches + d->npatches);
        p->nfields = d->slopes == GRAVITY_SLOPES_GIVEN ? 3 : 1;
        if (nested) {
            hip_check(hipGetDevice(&p->device), "hipGetDevice");
            p->nf = (int)std::min<int64_t>(nf, 1 << 30);
            p->M = 2 * p->n0;
            build_nested(*p);
            *out = p.release();
            return;
        }
        p->nf = (int)nf;
        p->M = 2 * p->nf;
        p->amr = d->nlevels > 1;
        std::vector<int32_t> owner, gmap;
        if (p->amr) {
            validate_and_build_maps(*p, owner, gmap);
        } else {
            p->ncells = p->nleaves = (int64_t)p->n0 * p->n0;
        }
        hip_check(hipGetDevice(&p->device), "hipGetDevice");
        {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            p->tw = get_twiddles(p->device, p->M, p->prec);
            // target height in finest cells (the kernel tables are in cell units)
            const double zc = p->z / (p->h0 / (double)(1 << (p->nlevels - 1)));
            p->centre = get_kernel_set(p->device, p->M, p->prec, 0, zc);
            if (p->amr) p->corner = get_kernel_set(p->device, p->M, p->prec, 1, zc);
        }
        if (p->amr) {
            p->owner.alloc(owner.size() * sizeof(int32_t), "AMR owner map");
            p->gmap.alloc(gmap.size() * sizeof(int32_t), "AMR gather map");
            hip_check(hipMemcpy(p->owner.p, owner.data(), owner.size() * sizeof(int32_t), hipMemcpyHostToDevice),
                      "owner map upload");
            hip_check(hipMemcpy(p->gmap.p, gmap.data(), gmap.size() * sizeof(int32_t), hipMemcpyHostToDevice),
                      "gather map upload");
        }
        const size_t esz = p->prec ? sizeof(double) : sizeof(float);
        const int64_t n = p->nf, H = p->M / 2;
        const size_t colsz = 2 * esz * (size_t)(H * n);
        size_t off = 0;
        p->off_a = off;
        off += align256(colsz * p->nfields);
        p->off_b = off;
        off += align256(colsz * p->ncomp * (p->amr ? 2 : 1));
        if (p->amr) {
            p->off_o = off;
            off += align256(esz * 2 * p->ncomp * (size_t)(n * n));
        }
        p->ws_bytes = off;
        {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            choose_variants(*p);
        }
        *out = p.release();
    });
}

gravity_status_t gravity_plan_workspace_bytes(gravity_plan_t p, size_t *bytes) {
    return guarded([&] {
        if (!p || !bytes) fail(GRAVITY_EINVAL, "NULL argument");
        *bytes = p->ws_bytes;
    });
}

gravity_status_t gravity_plan_get_info(gravity_plan_t p, gravity_plan_info_t *info) {
    return guarded([&] {
        if (!p || !info) fail(GRAVITY_EINVAL, "NULL argument");
        info->n_finest = p->nf;
        info->fft_size = p->M;
        info->n_cells = p->ncells;
        info->n_leaves = p->nleaves;
        info->workspace_bytes = p->ws_bytes;
        size_t r = p->owner.bytes + p->gmap.bytes;
        if (p->centre) r += p->centre->q.bytes;
        if (p->corner) r += p->corner->q.bytes;
        if (p->tw) r += p->tw->tw.bytes + p->tw->ph.bytes;
        if (p->nest) {
            const NestedPlan &N = *p->nest;
            r += N.fown.bytes + N.cown.bytes + N.rent.bytes + N.leaf.bytes;
            for (const gravity_plan_s *sp : {N.base.get(), N.fine.get(), N.coarse.get()})
                r += sp->centre->q.bytes + sp->tw->tw.bytes + sp->tw->ph.bytes;
        }
        info->resident_bytes = r;
        info->ncomp = p->ncomp;
        info->variants[0] = p->var_rf;
        info->variants[1] = p->var_col;
        info->variants[2] = p->var_ri;
    });
}

static void check_solve_args(gravity_plan_t p, const void *sigma, const void *dsx, const void *dsy,
                             void *fx, void *fy, void *ws) {
    if (!p) fail(GRAVITY_EINVAL, "NULL plan");
    if (!sigma || !fx || !fy || !ws) fail(GRAVITY_EINVAL, "NULL array argument");
    if (p->nfields == 3 && (!dsx || !dsy)) fail(GRAVITY_EINVAL, "slopes required by this plan");
    if (((uintptr_t)ws) & 255) fail(GRAVITY_EINVAL, "workspace must be 256-byte aligned");
    const size_t al = p->prec ? 16 : 8;
    if ((((uintptr_t)sigma) | ((uintptr_t)fx) | ((uintptr_t)fy)) & (al - 1))
        fail(GRAVITY_EINVAL, "arrays must be aligned to two elements");
    if (p->nfields == 3 && ((((uintptr_t)dsx) | ((uintptr_t)dsy)) & (al - 1)))
        fail(GRAVITY_EINVAL, "arrays must be aligned to two elements");
    int dev = -1;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (dev != p->device) fail(GRAVITY_EINVAL, "plan was created on another device");
}

gravity_status_t gravity_solve(gravity_plan_t p, const void *sigma, const void *dsx, const void *dsy,
                               void *fx, void *fy, void *workspace, void *stream) {
    return guarded([&] {
        check_solve_args(p, sigma, dsx, dsy, fx, fy, workspace);
        if (p->ncomp == 3) fail(GRAVITY_EINVAL, "off-plane plan: use gravity_solve_xyz");
        Item it{p, sigma, dsx, dsy, fx, fy, (char *)workspace};
        run_items(&it, 1, (hipStream_t)stream);
    });
}

gravity_status_t gravity_solve_xyz(gravity_plan_t p, const void *sigma, const void *dsx, const void *dsy,
                                   void *fx, void *fy, void *fz, void *workspace, void *stream) {
    return guarded([&] {
        check_solve_args(p, sigma, dsx, dsy, fx, fy, workspace);
        if (p->ncomp != 3) fail(GRAVITY_EINVAL, "midplane plan: use gravity_solve");
        if (!fz) fail(GRAVITY_EINVAL, "NULL array argument");
        if (((uintptr_t)fz) & ((p->prec ? 16 : 8) - 1)) fail(GRAVITY_EINVAL, "arrays must be aligned to two elements");
        Item it{p, sigma, dsx, dsy, fx, fy, (char *)workspace, fz};
        run_items(&it, 1, (hipStream_t)stream);
    });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// allocation-free solves: the workspace is a static device array
// ---------------------------------------------------------------------------
// Every device the library runs on holds its own copy of this array from the
// first allocation-free solve on that device until the process ends.  In
// host code `scratch` names a host-side stand-in, not device memory: only the
// address hipGetSymbolAddress returns for the current device is passed to
// kernels.
static __device__ __align__(256) unsigned char scratch[GRAVITY_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::vector<void *> g_scratch_ptr;  // per device: device address of `scratch`

void *scratch_address(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize(device + 1, nullptr);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!ptr || ((uintptr_t)ptr & 255)) fail(GRAVITY_EDEVICE, "scratch array has no aligned device address");
        g_scratch_ptr[device] = ptr;
    }
    return g_scratch_ptr[device];
}

}  // namespace

extern "C" {

gravity_status_t gravity_solve_noalloc(gravity_plan_t p, const void *sigma, const void *dsx,
                                       const void *dsy, void *fx, void *fy, void *stream) {
    return guarded([&] {
        if (!p) fail(GRAVITY_EINVAL, "NULL plan");
        if (p->ncomp == 3) fail(GRAVITY_EINVAL, "off-plane plan: use gravity_solve_xyz");
        if (p->ws_bytes > (size_t)GRAVITY_NOALLOC_SCRATCH_BYTES)
            fail(GRAVITY_EUNSUPPORTED, "plan needs " + std::to_string(p->ws_bytes) +
                                           " workspace bytes; the allocation-free solve has " +
                                           std::to_string((size_t)GRAVITY_NOALLOC_SCRATCH_BYTES));
        int dev = -1;
        hip_check(hipGetDevice(&dev), "hipGetDevice");
        if (dev != p->device) fail(GRAVITY_EINVAL, "plan was created on another device");
        char *ws = (char *)scratch_address(dev);
        check_solve_args(p, sigma, dsx, dsy, fx, fy, ws);
        Item it{p, sigma, dsx, dsy, fx, fy, ws};
        run_items(&it, 1, (hipStream_t)stream);
    });
}

}  // extern "C"

namespace {

// Persistent-batch tables: control block, pass-major unit offsets, per-solve
// pass counters, argument blocks.  One table per precision follows the
// solves' workspaces in the batch workspace.
size_t batch_table_bytes(int n) {
    const size_t head = (sizeof(BatchCtl) + 4 * 3 * ((size_t)n + 1) + 4 * 3 * (size_t)n + 15) / 16 * 16;
    return align256(head + (size_t)n * sizeof(BatchItem<double>));
}

// Host staging of the tables: a ring of pinned buffers, each reused only
// once the copy last queued from it has completed (its event).
struct Staging {
    std::mutex mu;
    struct Slot {
        void *buf = nullptr;
        size_t bytes = 0;
        hipEvent_t ev = nullptr;
    };
    Slot slot[16];
    int next = 0;
};
// held until the process ends (no release at exit, when the runtime may be
// gone already)
Staging &g_staging = *new Staging;

void stage_and_copy(const std::vector<char> &host, void *dev, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_staging.mu);
    Staging::Slot &sl = g_staging.slot[g_staging.next];
    g_staging.next = (g_staging.next + 1) % 16;
    if (sl.ev) hip_check(hipEventSynchronize(sl.ev), "hipEventSynchronize (staging)");
    else hip_check(hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming), "hipEventCreate");
    if (sl.bytes < host.size()) {
        if (sl.buf) (void)hipHostFree(sl.buf);
        sl.buf = nullptr;
        sl.bytes = 0;
        hip_check(hipHostMalloc(&sl.buf, host.size(), hipHostMallocDefault), "hipHostMalloc (staging)");
        sl.bytes = host.size();
    }
    std::memcpy(sl.buf, host.data(), host.size());
    hip_check(hipMemcpyAsync(dev, sl.buf, host.size(), hipMemcpyHostToDevice, s), "batch table upload");
    hip_check(hipEventRecord(sl.ev, s), "hipEventRecord (staging)");
}

bool persistent_ok(const gravity_plan_s &p) {
    return !p.amr && !p.nest && p.ncomp == 2 && p.nfields == 3 && batch_size_ok(p.M);
}

// One persistent launch over the uniform solves `it` of one precision.
template <typename T> void run_persistent(const std::vector<Item> &it, char *table, hipStream_t s) {
    const int n = (int)it.size();
    std::vector<uint32_t> first(3 * ((size_t)n + 1));
    uint32_t acc = 0, ends[3];
    for (int pass = 0; pass < 3; ++pass) {
        for (int r = 0; r < n; ++r) {
            uint32_t u[3];
            batch_units(it[r].p->M, u);
            first[(size_t)pass * (n + 1) + r] = acc;
            acc += u[pass];
        }
        first[(size_t)pass * (n + 1) + n] = acc;
        ends[pass] = acc;
    }
    std::vector<BatchItem<T>> items(n);
    for (int r = 0; r < n; ++r) {
        const gravity_plan_s &p = *it[r].p;
        const int nf = p.nf, H = p.M / 2;
        const int64_t colsz = (int64_t)H * nf;
        const T h = (T)p.h0;
        BatchItem<T> &b = items[r];
        std::memset((void *)&b, 0, sizeof(b));
        b.rf.in[0] = (const T *)it[r].s;
        b.rf.in[1] = (const T *)it[r].dx;
        b.rf.in[2] = (const T *)it[r].dy;
        b.rf.scale[0] = (T)1;
        b.rf.scale[1] = h;
        b.rf.scale[2] = h;
        b.rf.in_pitch = nf;
        b.rf.out = (C<T> *)(it[r].ws + p.off_a);
        b.rf.out_pitch = nf;
        b.rf.out_fstride = colsz;
        b.rf.hf = h;
        b.rf.slopes = 1;
        b.rf.nrows = nf;
        b.col.in = b.rf.out;
        b.col.in_pitch = nf;
        b.col.in_fstride = colsz;
        b.col.q[0] = b.col.q[1] = (const T *)p.centre->q.p;
        b.col.q_pitch = p.centre->q_pitch;
        b.col.q_kstride = p.centre->q_kstride;
        b.col.out = (C<T> *)(it[r].ws + p.off_b);
        b.col.out_pitch = nf;
        b.col.out_gstride = colsz;
        b.col.nsub = 1;
        b.ri.in = b.col.out;
        b.ri.in_pitch = nf;
        b.ri.in_gstride = colsz;
        b.ri.out[0] = (T *)it[r].fx;
        b.ri.out[1] = (T *)it[r].fy;
        b.ri.out_pitch = nf;
        b.ri.scale = (T)(p.G / ((double)p.M * (double)p.M));
        b.ri.nrows = nf;
        b.tw = (const C<T> *)p.tw->tw.p;
        b.ph = (const C<T> *)p.tw->ph.p;
        b.M = p.M;
    }
    const size_t o_first = sizeof(BatchCtl);
    const size_t o_done = o_first + 4 * first.size();
    const size_t o_items = (o_done + 4 * 3 * (size_t)n + 15) / 16 * 16;
    std::vector<char> host(o_items + (size_t)n * sizeof(BatchItem<T>), 0);
    BatchCtl ctl{};
    for (int k = 0; k < 3; ++k) ctl.end[k] = ends[k];
    std::memcpy(host.data(), &ctl, sizeof(ctl));
    std::memcpy(host.data() + o_first, first.data(), 4 * first.size());
    std::memcpy(host.data() + o_items, items.data(), (size_t)n * sizeof(BatchItem<T>));
    stage_and_copy(host, table, s);
    hip_check(launch_batch<T>((BatchCtl *)table, (const uint32_t *)(table + o_first), (uint32_t *)(table + o_done),
                              (const BatchItem<T> *)(table + o_items), n, ends[2], s),
              "persistent batch");
}

}  // namespace

extern "C" {

gravity_status_t gravity_batch_workspace_bytes(int32_t n, const gravity_plan_t *plans, size_t *bytes) {
    return guarded([&] {
        if (n < 0 || (n > 0 && !plans) || !bytes) fail(GRAVITY_EINVAL, "bad batch arguments");
        size_t tot = 0;
        for (int i = 0; i < n; ++i) {
            if (!plans[i]) fail(GRAVITY_EINVAL, "NULL plan in batch");
            tot += align256(plans[i]->ws_bytes);
        }
        *bytes = tot + 2 * batch_table_bytes(n);  // room for the persistent launch's tables
    });
}

// fz: NULL, or n pointers (entries of midplane plans ignored); off-plane
// plans need theirs
static gravity_status_t solve_batch(int32_t n, const gravity_plan_t *plans, const void *const *sigma,
                             const void *const *dsx, const void *const *dsy, void *const *fx,
                             void *const *fy, void *const *fz, void *workspace, void *stream,
                             bool persistent = false) {
    return guarded([&] {
        if (n < 0 || (n > 0 && (!plans || !sigma || !fx || !fy))) fail(GRAVITY_EINVAL, "bad batch arguments");
        std::vector<Item> items;
        items.reserve(n);
        size_t off = 0;
        for (int i = 0; i < n; ++i) {
            const void *dx = dsx ? dsx[i] : nullptr;
            const void *dy = dsy ? dsy[i] : nullptr;
            char *ws = workspace ? (char *)workspace + off : nullptr;
            check_solve_args(plans[i], sigma[i], dx, dy, fx[i], fy[i], ws);
            void *z = nullptr;
            if (plans[i]->ncomp == 3) {
                if (!fz) fail(GRAVITY_EUNSUPPORTED, "off-plane plans need gravity_solve_batch_xyz");
                z = fz[i];
                if (!z || (((uintptr_t)z) & ((plans[i]->prec ? 16 : 8) - 1)))
                    fail(GRAVITY_EINVAL, "off-plane solve needs an aligned fz");
            }
            items.push_back(Item{plans[i], sigma[i], dx, dy, fx[i], fy[i], ws, z});
            off += align256(plans[i]->ws_bytes);
        }
        std::vector<bool> done(n, false);
        hipStream_t s = (hipStream_t)stream;
        if (persistent) {
            // uniform solves of the supported sizes: one launch per precision
            char *table = (char *)workspace + off;
            for (int prec = 0; prec < 2; ++prec) {
                std::vector<Item> sel;
                for (int i = 0; i < n; ++i)
                    if (!done[i] && items[i].p->prec == prec && persistent_ok(*items[i].p)) {
                        sel.push_back(items[i]);
                        done[i] = true;
                    }
                if (sel.empty()) continue;
                if (prec)
                    run_persistent<double>(sel, table, s);
                else
                    run_persistent<float>(sel, table, s);
                table += batch_table_bytes(n);
            }
        }
        // group the other solves that can share launches (stable order within a group)
        std::vector<Item> grp;
        for (int i = 0; i < n; ++i) {
            if (done[i]) continue;
            grp.assign(1, items[i]);
            done[i] = true;
            for (int j = i + 1; j < n; ++j) {
                if (!done[j] && same_group(*items[i].p, *items[j].p)) {
                    grp.push_back(items[j]);
                    done[j] = true;
                }
            }
            for (size_t k = 0; k < grp.size(); k += kPack)
                run_items(grp.data() + k, (int)std::min<size_t>(kPack, grp.size() - k), s);
        }
    });
}

gravity_status_t gravity_solve_batch(int32_t n, const gravity_plan_t *plans, const void *const *sigma,
                                     const void *const *dsx, const void *const *dsy, void *const *fx,
                                     void *const *fy, void *workspace, void *stream) {
    return solve_batch(n, plans, sigma, dsx, dsy, fx, fy, nullptr, workspace, stream);
}

gravity_status_t gravity_solve_batch_persistent(int32_t n, const gravity_plan_t *plans, const void *const *sigma,
                                                const void *const *dsx, const void *const *dsy, void *const *fx,
                                                void *const *fy, void *workspace, void *stream) {
    if (!workspace && n > 0) {
        g_err = "persistent batch needs its workspace";
        return GRAVITY_EINVAL;
    }
    return solve_batch(n, plans, sigma, dsx, dsy, fx, fy, nullptr, workspace, stream, true);
}

gravity_status_t gravity_batch_persistent_abandoned(int32_t n, const gravity_plan_t *plans, const void *workspace,
                                                   void *stream, uint32_t *abandoned) {
    return guarded([&] {
        if (n < 0 || (n > 0 && (!plans || !workspace)) || !abandoned) fail(GRAVITY_EINVAL, "bad arguments");
        size_t off = 0;
        bool has[2] = {false, false};
        for (int i = 0; i < n; ++i) {
            if (!plans[i]) fail(GRAVITY_EINVAL, "NULL plan");
            off += align256(plans[i]->ws_bytes);
            if (persistent_ok(*plans[i])) has[plans[i]->prec] = true;
        }
        // the tables sit after the solves' workspaces, one per precision
        // present, in the order the launches took them (FP32 first)
        const char *table = (const char *)workspace + off;
        uint32_t tot = 0;
        hipStream_t s = (hipStream_t)stream;
        for (int prec = 0; prec < 2; ++prec) {
            if (!has[prec]) continue;
            BatchCtl ctl{};
            hip_check(hipMemcpyAsync(&ctl, table, sizeof(ctl), hipMemcpyDeviceToHost, s), "control block copy");
            hip_check(hipStreamSynchronize(s), "control block copy");
            tot += ctl.timeouts;
            table += batch_table_bytes(n);
        }
        *abandoned = tot;
    });
}

gravity_status_t gravity_solve_batch_xyz(int32_t n, const gravity_plan_t *plans, const void *const *sigma,
                                         const void *const *dsx, const void *const *dsy, void *const *fx,
                                         void *const *fy, void *const *fz, void *workspace, void *stream) {
    return solve_batch(n, plans, sigma, dsx, dsy, fx, fy, fz, workspace, stream);
}

gravity_status_t gravity_solve_profiled(gravity_plan_t p, const void *sigma, const void *dsx,
                                        const void *dsy, void *fx, void *fy, void *workspace,
                                        void *stream, int32_t reps, double *stage_ms, int32_t *nstages) {
    std::vector<hipEvent_t> ev;
    gravity_status_t st = guarded([&] {
        check_solve_args(p, sigma, dsx, dsy, fx, fy, workspace);
        if (reps < 1 || !stage_ms || !nstages) fail(GRAVITY_EINVAL, "bad profiling arguments");
        if (p->ncomp == 3) fail(GRAVITY_EUNSUPPORTED, "off-plane plans are solved with gravity_solve_xyz");
        if (p->nest) fail(GRAVITY_EUNSUPPORTED, "nested AMR plans are not profiled by stage");
        const int ns = n_stages(*p);
        ev.resize(ns + 1);
        for (auto &e : ev) {
            e = nullptr;
            hip_check(hipEventCreate(&e), "hipEventCreate");
        }
        hipStream_t s = (hipStream_t)stream;
        // every stage launched reps times back to back between its two events
        if (p->prec)
            solve_t<double>(*p, sigma, dsx, dsy, fx, fy, (char *)workspace, s, ev.data(), reps);
        else
            solve_t<float>(*p, sigma, dsx, dsy, fx, fy, (char *)workspace, s, ev.data(), reps);
        hip_check(hipEventSynchronize(ev[ns]), "hipEventSynchronize");
        for (int k = 0; k < ns; ++k) {
            float ms = 0;
            hip_check(hipEventElapsedTime(&ms, ev[k], ev[k + 1]), "hipEventElapsedTime");
            stage_ms[k] = (double)ms / reps;
        }
        *nstages = ns;
    });
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    return st;
}

const char *gravity_stage_name(gravity_plan_t p, int32_t stage) {
    if (!p || stage < 0 || stage >= n_stages(*p)) return "";
    return p->amr ? kStagesAmr[stage] : kStagesUniform[stage];
}

void gravity_plan_destroy(gravity_plan_t p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    delete p;
}

size_t gravity_cache_bytes(void) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    size_t tot = 0;
    for (auto &kv : g_ks_cache)
        if (auto sp = kv.second.lock()) tot += sp->q.bytes;
    for (auto &kv : g_tw_cache)
        if (auto sp = kv.second.lock()) tot += sp->tw.bytes + sp->ph.bytes;
    return tot;
}

const char *gravity_last_error(void) { return g_err.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------
// request server (continuous batching)
// ---------------------------------------------------------------------------
namespace {

using Clock = std::chrono::steady_clock;

struct SrvRequest {
    int64_t ticket;
    Item item;  // ws filled at admission
    size_t ws_bytes, off = 0;
    Clock::time_point t_submit;
    hipEvent_t ready = nullptr;  // recorded on the caller's stream at submit
};

struct SrvTicket {
    int done = 0;
    gravity_status_t status = GRAVITY_OK;
    double latency_ms = 0;
};

struct SrvBatch {
    std::vector<SrvRequest> reqs;
    int stream = 0;
    hipEvent_t ev = nullptr;
};

}  // namespace

struct gravity_server_s {
    int device = 0;
    int max_batch = kPack;
    DevBuf arena_mem;
    std::unique_ptr<grav::Arena> arena;
    std::vector<hipStream_t> streams;
    std::vector<int> load;
    std::vector<hipEvent_t> event_pool;  // completion and input-ready events
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<SrvRequest> pending;
    std::vector<SrvBatch> inflight;
    std::unordered_map<int64_t, SrvTicket> tickets;
    int64_t next_ticket = 1;
    std::vector<double> latencies;
    int64_t submitted = 0, completed = 0, batches = 0, leaves = 0;
    size_t peak = 0;
    bool stop = false;
    std::thread th;

    void loop();
    void complete(SrvBatch &b, gravity_status_t st);
    hipEvent_t take_event();  // with mu held; nullptr if creation fails
};

hipEvent_t gravity_server_s::take_event() {
    if (event_pool.empty()) {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return e;
    }
    hipEvent_t e = event_pool.back();
    event_pool.pop_back();
    return e;
}

void gravity_server_s::complete(SrvBatch &b, gravity_status_t st) {
    // called with mu held
    const auto now = Clock::now();
    for (auto &r : b.reqs) {
        SrvTicket &tk = tickets[r.ticket];
        tk.done = 1;
        tk.status = st;
        tk.latency_ms = std::chrono::duration<double, std::milli>(now - r.t_submit).count();
        if (st == GRAVITY_OK) {
            latencies.push_back(tk.latency_ms);
            leaves += r.item.p->nleaves;
        }
        arena->release(r.off, r.ws_bytes);
        if (r.ready) event_pool.push_back(r.ready);
        ++completed;
    }
    --load[b.stream];
    if (b.ev) event_pool.push_back(b.ev);
}

void gravity_server_s::loop() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        // admission: arrival order, first fit; later requests may pass one that waits
        std::vector<SrvRequest> admitted;
        for (auto it = pending.begin(); it != pending.end();) {
            size_t off;
            if (arena->alloc(it->ws_bytes, &off)) {
                it->off = off;
                it->item.ws = (char *)arena_mem.p + off;
                admitted.push_back(*it);
                it = pending.erase(it);
            } else {
                ++it;
            }
        }
        peak = std::max(peak, arena->used());
        // continuous batching: group admitted requests that can share launches
        std::vector<SrvBatch> ready;
        std::vector<bool> used(admitted.size(), false);
        for (size_t i = 0; i < admitted.size(); ++i) {
            if (used[i]) continue;
            SrvBatch b;
            b.reqs.push_back(admitted[i]);
            used[i] = true;
            for (size_t j = i + 1; j < admitted.size() && (int)b.reqs.size() < max_batch; ++j) {
                if (!used[j] && same_group(*admitted[i].item.p, *admitted[j].item.p)) {
                    b.reqs.push_back(admitted[j]);
                    used[j] = true;
                }
            }
            b.stream = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            ++load[b.stream];
            b.ev = take_event();
            ready.push_back(std::move(b));
        }
        // launch without holding the lock
        lk.unlock();
        std::vector<gravity_status_t> st(ready.size(), GRAVITY_OK);
        for (size_t k = 0; k < ready.size(); ++k) {
            SrvBatch &b = ready[k];
            hipStream_t sb = streams[b.stream];
            bool queued = false;  // kernels of this batch may be on the stream
            try {
                if (!b.ev) fail(GRAVITY_EDEVICE, "hipEventCreate failed");
                std::vector<Item> items;
                for (auto &r : b.reqs) {
                    items.push_back(r.item);
                    // the request's inputs: ready once the caller's stream reached submit
                    hip_check(hipStreamWaitEvent(sb, r.ready, 0), "hipStreamWaitEvent");
                }
                queued = true;
                run_items(items.data(), (int)items.size(), sb);
                hip_check(hipEventRecord(b.ev, sb), "hipEventRecord");
            } catch (const Failure &f) {
                st[k] = f.st;
            } catch (const std::bad_alloc &) {
                st[k] = GRAVITY_ENOMEM;
            } catch (...) {
                st[k] = GRAVITY_EDEVICE;
            }
            // a failed batch releases its arena range at once: first let
            // whatever it queued finish
            if (st[k] != GRAVITY_OK && queued) (void)hipStreamSynchronize(sb);
        }
        lk.lock();
        for (size_t k = 0; k < ready.size(); ++k) {
            ++batches;
            if (st[k] != GRAVITY_OK) {
                complete(ready[k], st[k]);
            } else {
                inflight.push_back(std::move(ready[k]));
            }
        }
        if (!ready.empty()) cv_done.notify_all();
        // completion polling
        bool progressed = false;
        for (size_t k = 0; k < inflight.size();) {
            hipError_t q = hipEventQuery(inflight[k].ev);
            if (q == hipErrorNotReady) {
                ++k;
                continue;
            }
            complete(inflight[k], q == hipSuccess ? GRAVITY_OK : GRAVITY_EDEVICE);
            inflight.erase(inflight.begin() + k);
            progressed = true;
        }
        if (progressed) cv_done.notify_all();
        if (stop && pending.empty() && inflight.empty()) break;
        if (progressed || !ready.empty()) continue;
        if (!inflight.empty())
            cv_work.wait_for(lk, std::chrono::microseconds(20));
        else
            cv_work.wait(lk, [&] { return stop || !pending.empty(); });
    }
}

extern "C" {

gravity_status_t gravity_server_create(size_t budget, int32_t nstreams, int32_t max_batch,
                                       gravity_server_t *out) {
    if (out) *out = nullptr;
    return guarded([&] {
        if (!out || nstreams < 1 || nstreams > 16 || max_batch < 1) fail(GRAVITY_EINVAL, "bad server arguments");
        auto srv = std::make_unique<gravity_server_s>();
        hip_check(hipGetDevice(&srv->device), "hipGetDevice");
        srv->max_batch = std::min<int>(max_batch, kPack);
        srv->arena_mem.alloc(budget, "server arena");
        srv->arena = std::make_unique<grav::Arena>(budget);
        for (int i = 0; i < nstreams; ++i) {
            hipStream_t s = nullptr;
            hip_check(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreate");
            srv->streams.push_back(s);
            srv->load.push_back(0);
        }
        gravity_server_s *raw = srv.get();
        srv->th = std::thread([raw] { raw->loop(); });
        *out = srv.release();
    });
}

static gravity_status_t server_submit(gravity_server_t srv, gravity_plan_t p, const void *sigma, const void *dsx,
                               const void *dsy, void *fx, void *fy, void *fz, void *stream, int64_t *ticket) {
    return guarded([&] {
        if (!srv || !ticket) fail(GRAVITY_EINVAL, "NULL argument");
        alignas(256) static char aligned_dummy;
        check_solve_args(p, sigma, dsx, dsy, fx, fy, &aligned_dummy);
        if (p->ncomp == 3 && !fz) fail(GRAVITY_EUNSUPPORTED, "off-plane plans need gravity_server_submit_xyz");
        if (p->ncomp == 3 && (((uintptr_t)fz) & ((p->prec ? 16 : 8) - 1)))
            fail(GRAVITY_EINVAL, "arrays must be aligned to two elements");
        if (p->device != srv->device) fail(GRAVITY_EINVAL, "plan and server are on different devices");
        const size_t ws = align256(p->ws_bytes);
        if (ws > srv->arena->size()) fail(GRAVITY_ENOMEM, "request workspace exceeds the server budget");
        SrvRequest r;
        r.item = Item{p, sigma, dsx, dsy, fx, fy, nullptr, p->ncomp == 3 ? fz : nullptr};
        r.ws_bytes = ws;
        r.t_submit = Clock::now();
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            if (srv->stop) fail(GRAVITY_EBUSY, "server is shutting down");
            r.ready = srv->take_event();
            if (!r.ready) fail(GRAVITY_EDEVICE, "hipEventCreate failed");
            const hipError_t e = hipEventRecord(r.ready, (hipStream_t)stream);
            if (e != hipSuccess) {
                srv->event_pool.push_back(r.ready);
                hip_check(e, "hipEventRecord on the caller's stream");
            }
            r.ticket = srv->next_ticket++;
            srv->tickets[r.ticket] = SrvTicket{};
            srv->pending.push_back(r);
            ++srv->submitted;
            *ticket = r.ticket;
        }
        srv->cv_work.notify_one();
    });
}

gravity_status_t gravity_server_submit(gravity_server_t srv, gravity_plan_t p, const void *sigma,
                                       const void *dsx, const void *dsy, void *fx, void *fy, void *stream,
                                       int64_t *ticket) {
    return server_submit(srv, p, sigma, dsx, dsy, fx, fy, nullptr, stream, ticket);
}

gravity_status_t gravity_server_submit_xyz(gravity_server_t srv, gravity_plan_t p, const void *sigma,
                                           const void *dsx, const void *dsy, void *fx, void *fy, void *fz,
                                           void *stream, int64_t *ticket) {
    return server_submit(srv, p, sigma, dsx, dsy, fx, fy, fz, stream, ticket);
}

gravity_status_t gravity_server_poll(gravity_server_t srv, int64_t ticket, int32_t *done) {
    return guarded([&] {
        if (!srv || !done) fail(GRAVITY_EINVAL, "NULL argument");
        std::lock_guard<std::mutex> lk(srv->mu);
        auto it = srv->tickets.find(ticket);
        if (it == srv->tickets.end()) fail(GRAVITY_EINVAL, "unknown ticket");
        *done = it->second.done;
        if (it->second.done && it->second.status != GRAVITY_OK) fail(it->second.status, "request failed");
    });
}

gravity_status_t gravity_server_wait(gravity_server_t srv, int64_t ticket, double *latency_ms) {
    return guarded([&] {
        if (!srv) fail(GRAVITY_EINVAL, "NULL server");
        std::unique_lock<std::mutex> lk(srv->mu);
        auto it = srv->tickets.find(ticket);
        if (it == srv->tickets.end()) fail(GRAVITY_EINVAL, "unknown ticket");
        srv->cv_done.wait(lk, [&] { return srv->tickets[ticket].done != 0; });
        SrvTicket tk = srv->tickets[ticket];
        srv->tickets.erase(ticket);
        if (latency_ms) *latency_ms = tk.latency_ms;
        if (tk.status != GRAVITY_OK) fail(tk.status, "request failed on the device");
    });
}

gravity_status_t gravity_server_drain(gravity_server_t srv) {
    return guarded([&] {
        if (!srv) fail(GRAVITY_EINVAL, "NULL server");
        std::unique_lock<std::mutex> lk(srv->mu);
        srv->cv_done.wait(lk, [&] { return srv->completed == srv->submitted; });
    });
}

gravity_status_t gravity_server_get_stats(gravity_server_t srv, gravity_server_stats_t *st) {
    return guarded([&] {
        if (!srv || !st) fail(GRAVITY_EINVAL, "NULL argument");
        std::lock_guard<std::mutex> lk(srv->mu);
        st->submitted = srv->submitted;
        st->completed = srv->completed;
        int64_t infl = 0;
        for (auto &b : srv->inflight) infl += (int64_t)b.reqs.size();
        st->in_flight = infl;
        st->pending = (int64_t)srv->pending.size();
        std::vector<double> l = srv->latencies;
        auto pct = [&](double q) {
            if (l.empty()) return 0.0;
            size_t k = (size_t)std::min<double>((double)l.size() - 1, std::floor(q * (double)(l.size() - 1) + 0.5));
            std::nth_element(l.begin(), l.begin() + k, l.end());
            return l[k];
        };
        st->latency_p50_ms = pct(0.50);
        st->latency_p99_ms = pct(0.99);
        st->latency_max_ms = l.empty() ? 0.0 : *std::max_element(l.begin(), l.end());
        st->budget_bytes = srv->arena->size();
        st->bytes_in_use = srv->arena->used();
        st->peak_bytes_in_use = srv->peak;
        st->batches = srv->batches;
        st->leaves_completed = srv->leaves;
    });
}

gravity_status_t gravity_server_reset_stats(gravity_server_t srv) {
    return guarded([&] {
        if (!srv) fail(GRAVITY_EINVAL, "NULL server");
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->latencies.clear();
        srv->batches = 0;
        srv->leaves = 0;
        srv->submitted -= srv->completed;
        srv->completed = 0;
        srv->peak = srv->arena->used();
    });
}

void gravity_server_destroy(gravity_server_t srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv_work.notify_all();
    if (srv->th.joinable()) srv->th.join();
    RelaxedCapture relaxed;
    for (auto s : srv->streams) (void)hipStreamDestroy(s);
    for (auto e : srv->event_pool)
        if (e) (void)hipEventDestroy(e);
    delete srv;
}

}  // extern "C"
