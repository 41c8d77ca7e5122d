// Kernel argument blocks and host launchers shared by the HIP kernels and
// the host runtime.  Layouts (all device memory):
//   fields   : n x n row-major real arrays (row = y index, x fastest)
//   A        : forward row spectra at the odd x frequencies kx + 1/2,
//              A[f][kx][j], kx in [0, M/2), j in [0, rows)
//   Q        : kernel spectra, Q[kind][kx][ky], kx in [0, M/2), ky in [0, M/2]
//   B        : column-inverted spectra, B[g][kx][j]
// M is the zero-padded transform size (2 n), n the lattice cells per side.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fft_core.hpp"

namespace grav {

constexpr int kMinM = 32;
constexpr int kMaxM = 8192;

template <typename T> struct RowFwdArgs {
    const T *in[3];     // up to three real fields (AMR: composite-packed leaf arrays)
    T scale[3];         // per-field multiplier applied on load
    int64_t in_pitch;   // elements between input rows (AMR: finest lattice side)
    C<T> *out;          // A
    int64_t out_pitch;  // elements between kx columns of A (= rows)
    int64_t out_fstride;
    // AMR: each finest cell's value is injected on load from the leaf that
    // covers it (owner: leaf index | log2(leaf size in finest cells) << 28),
    // the leaf's linear density taken at the cell centre; hf = finest cell size
    const int32_t *owner;
    T hf;
    int slopes;
    int64_t nrows;      // rows of this item (items of one launch may differ)
};

template <typename T> struct ColArgs {
    const C<T> *in;  // A
    int64_t in_pitch, in_fstride;
    const T *q[2];   // spectra of the centre / corner family: kind k at q[f] + k q_kstride
    int64_t q_pitch, q_kstride;
    C<T> *out;       // B
    int64_t out_pitch, out_gstride;
    // sub-items (blockIdx.y < nsub): independent column sets of one size
    // whose input and output columns start sub_off elements further on
    int nsub;
    int64_t sub_off;
};

template <typename T> struct RowInvArgs {
    const C<T> *in;  // B
    int64_t in_pitch, in_gstride;
    T *out[6];       // one real plane per output (component x family)
    int64_t out_pitch;
    T scale;
    int64_t nrows;   // rows of this item (items of one launch may differ)
};

template <typename T> struct GatherArgs {
    const int32_t *gmap;  // per composite cell: -1, or lattice index | family << 30
    const T *o[6];        // finest-lattice outputs: component c of family f at o[ncomp f + c]
    T *fx, *fy, *fz;      // fz only when ncomp == 3
    int64_t n;
    int ncomp;
};

// Up to kPack independent solves of one size share a launch: the kernels
// take their argument blocks by value in a Pack and pick item blockIdx.z.
constexpr int kPack = 8;
template <typename A> struct Pack {
    A a[kPack];
};

// Kernel kinds: 3 c + f is force component c (x, y, z) times input field f
// (sigma, dsx, dsy): x0, xx, xy, y0, yx, yy, z0, zx, zy.
// Parity in y: x0 even, xx even, xy odd, y0 odd, yx odd, yy even, z0 even,
// zx even, zy odd.
__host__ __device__ constexpr int parity_y(int kind) {
    return (kind == 2 || kind == 3 || kind == 4 || kind == 8) ? -1 : 1;
}
// kinds whose spectrum is purely imaginary (odd in exactly one of x, y)
__host__ __device__ constexpr bool imag_kind(int kind) {
    return kind == 0 || kind == 3 || kind == 7 || kind == 8;
}

struct TableArgs {
    double *out;  // M x M table, row-major [my][mx]
    int M;
    int family;   // 0: cell-centre targets, 1: lattice-corner targets
    int kind;     // 0..8: x0, xx, xy, y0, yx, yy, z0, zx, zy (z kinds need zc != 0)
    double zc;    // height of the target plane above the disk, in cells (0: midplane)
    double glx[10], glw[10];  // Gauss-Legendre nodes and weights on [-1, 1]: 10 points
    double glx8[8], glw8[8], glx6[6], glw6[6], glx4[4], glw4[4];  // 8, 6 and 4 points
};

// Kernel variants of the three solve kernels (see kernels_impl.hpp): bit 1
// selects 16 elements per thread (else 8), bit 0 all fields per thread; bits
// 2-3 scale the rows per block of the row kernels (doubled, halved), bit 2
// selects two columns per block in the column kernel (ids below 8; ids 8-9
// take 4 elements per thread, 10-13 cap the registers per lane, 14-15 split
// two kernel families over blocks, 16 uses two exchange buffers).
// Validity depends on size, precision and fields.
constexpr int kNumVariants = 17;
bool row_variant_valid(int prec, int M, int var);
bool col_variant_valid(int prec, int M, int var, int nfields, int nfam, int ncomp);

// Launchers: n (1..kPack) items of the same size and kind in one launch.
// nrows / nsub: the largest item's rows / sub-items (the grid is sized for
// it; the blocks beyond a smaller item's own count exit at once).
template <typename T>
hipError_t launch_row_fwd(const Pack<RowFwdArgs<T>> &a, int n, int M, int var, bool pruned,
                          int64_t nrows, int nfields, const C<T> *tw, hipStream_t s);
template <typename T>
hipError_t launch_col(const Pack<ColArgs<T>> &a, int n, int M, int var, int nfields, int nfam,
                      int ncomp, const C<T> *tw, const C<T> *ph, hipStream_t s, int nsub = 1);
template <typename T>
hipError_t launch_row_inv(const Pack<RowInvArgs<T>> &a, int n, int M, int var, int64_t nrows, int nout,
                          const C<T> *tw, hipStream_t s);
template <typename T>
hipError_t launch_gather(const Pack<GatherArgs<T>> &a, int n, int64_t maxcells, hipStream_t s);

// ---------------------------------------------------------------------------
// nested-correction AMR (approximate; cost follows the refined area)
// ---------------------------------------------------------------------------
// Each refined level l >= 1 is tiled by kNestBox x kNestBox boxes of level-l
// cells; a box is solved on its region grown by kNestExt cells on every side
// (fine region: kNestFine^2 level-l cells, coarse region: kNestCoarse^2
// level-(l-1) cells).
constexpr int kNestBox = 64, kNestExt = 32;
constexpr int kNestFine = kNestBox + 2 * kNestExt, kNestCoarse = kNestFine / 2;
constexpr int kNestMaxLevels = 6;  // region origins stay aligned to every leaf size

// restriction of four children into their parent (per entry: parent and
// children (x, y) = (0,0), (1,0), (0,1), (1,1), composite indices)
template <typename T> struct RestrictArgs {
    T *s, *dx, *dy;          // composite arrays, updated in place
    const int32_t *ent;      // 5 indices per entry
    int64_t n;               // entries
    double h;                // parent cell size
};
// combine of one refined level: F^l = F_fine + sum_k w_k (F^{l-1}(p_k) - F_coarse(p_k))
template <typename T> struct CombineArgs {
    const int32_t *fown, *cown;  // region owner maps of this level's boxes
    const T *ffx, *ffy;          // fine-region forces [box][kNestFine^2]
    const T *cfx, *cfy;          // coarse-region forces [box][kNestCoarse^2]
    double *accx, *accy;         // per composite cell: F^l of its level (FP64)
    int32_t sentinel;            // owner index of cells outside the domain
    int nbox;
};
template <typename T>
hipError_t launch_nest_copy_in(const T *s, const T *dx, const T *dy, T *rs, T *rdx, T *rdy, int64_t n,
                               hipStream_t st);
template <typename T> hipError_t launch_nest_restrict(const RestrictArgs<T> &a, hipStream_t st);
template <typename T>
hipError_t launch_nest_lift(const T *fx, const T *fy, double *accx, double *accy, int64_t n, hipStream_t st);
template <typename T> hipError_t launch_nest_combine(const CombineArgs<T> &a, hipStream_t st);
template <typename T>
hipError_t launch_nest_finalize(const double *accx, const double *accy, const uint8_t *leaf, T *fx, T *fy,
                                int64_t n, hipStream_t st);

// ---------------------------------------------------------------------------
// one persistent launch over a batch of uniform solves of mixed sizes
// ---------------------------------------------------------------------------
struct BatchCtl {
    uint32_t head;      // next unit to take (zero at launch)
    uint32_t timeouts;  // units abandoned after a wait reached its bound
    uint32_t end[3];    // pass boundaries: units of passes < p end at end[p]
    uint32_t pad[3];
};
template <typename T> struct BatchItem {
    RowFwdArgs<T> rf;
    ColArgs<T> col;
    RowInvArgs<T> ri;
    const C<T> *tw, *ph;
    int M;
};
bool batch_size_ok(int M);                 // transform sizes the persistent launch takes
void batch_units(int M, uint32_t units[3]);  // units of each pass for one solve of size M
// ctl, first (3 x (n+1) global unit offsets, pass-major), done (3 n counters,
// zero at launch) and items: device memory, written before the launch
template <typename T>
hipError_t launch_batch(BatchCtl *ctl, const uint32_t *first, uint32_t *done, const BatchItem<T> *items, int n,
                        uint32_t total_units, hipStream_t s);

hipError_t launch_ktable(const TableArgs &a, hipStream_t s);
// forward FFT of the columns of a table's row spectra (odd x frequencies)
// and extraction of one real half plane, kx in [0, M/2), ky in [0, M/2]:
// Q[kx][ky] = part(e^{i pi corner (kx + 1/2 + ky)/M} S[ky][kx])
template <typename TQ>
hipError_t launch_col_extract(const C<double> *in, int M, TQ *q, int64_t q_pitch, int imag,
                              int corner, const C<double> *tw, const C<double> *ph,
                              hipStream_t s);

}  // namespace grav
