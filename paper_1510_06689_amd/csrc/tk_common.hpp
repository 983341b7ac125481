// Internal helpers shared by the library's translation units: error
// plumbing, the block-column view of a mode-n unfolding, and the column-tile
// map that every streaming kernel (Gram, TTM) walks.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "tucker.h"

namespace tk {

// ------------------------------------------------------------- errors

void set_error(const char* fmt, ...);  // thread-local message for tk_last_error()
int fail(int status, const char* fmt, ...);

#define TK_HIP(call)                                                                 \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess)                                                        \
            return ::tk::fail(TK_ERR_HIP, "%s failed: %s (%s:%d)", #call,            \
                              hipGetErrorString(e_), __FILE__, __LINE__);            \
    } while (0)

#define TK_TRY(expr)                 \
    do {                             \
        int rc_ = (expr);            \
        if (rc_ != TK_OK) return rc_; \
    } while (0)

// ------------------------------------------------------------- shapes

inline size_t dtype_size(int dt) { return dt == TK_F64 ? 8 : 4; }

inline int64_t numel(const tk_shape& s) {
    int64_t p = 1;
    for (int k = 0; k < s.ndim; ++k) p *= s.dims[k];
    return p;
}

// Validates ndim, dims and dtype.  Never touches the device.
int check_shape(const tk_shape* s, const char* what);

// Block-column view of the mode-n unfolding (Sec. IV-C): the tensor read as
// Y[B][J][L] with L = prod_{m<n} dims[m], J = dims[n], B = prod_{m>n} dims[m].
// Column kk of the unfolding is (b, l) with kk = b * L + l; the element
// (i, b, l) sits at offset l + L * (i + J * b).
struct ModeView {
    int64_t L, B;
    int J;
};

__host__ __device__ inline ModeView mode_view(const int64_t* dims, int ndim, int n) {
    ModeView v{1, 1, (int)dims[n]};
    for (int k = 0; k < n; ++k) v.L *= dims[k];
    for (int k = n + 1; k < ndim; ++k) v.B *= dims[k];
    return v;
}

// Column tiles of KT columns over a ModeView.  Two regimes:
//  packed  (L <= KT): a tile is nbb = floor(KT / L) consecutive b-blocks, one
//          contiguous memory range of nbb * J * L elements; column
//          kk = bb * L + l, and columns nbb * L .. KT - 1 are padding (zero).
//  strided (L > KT):  a tile is a segment [l0, l0 + KT) of one b-block, J
//          rows of up to KT contiguous elements with row stride L.
struct TileMap {
    int64_t L, B;
    int J, KT;
    int packed;     // 1 = packed regime
    int nbb;        // packed: b-blocks per tile
    int64_t lsegs;  // strided: ceil(L / KT) segments per b-block
    int64_t ntiles;
};

__host__ __device__ inline TileMap make_tiles(const ModeView& v, int KT) {
    TileMap t{};
    t.L = v.L;
    t.B = v.B;
    t.J = v.J;
    t.KT = KT;
    t.packed = v.L <= KT ? 1 : 0;
    if (t.packed) {
        t.nbb = (int)(KT / v.L);
        t.lsegs = 1;
        t.ntiles = (v.B + t.nbb - 1) / t.nbb;
    } else {
        t.nbb = 1;
        t.lsegs = (v.L + KT - 1) / KT;
        t.ntiles = v.B * t.lsegs;
    }
    return t;
}

// Per-tile geometry, computed on the device.
struct Tile {
    int64_t base;  // offset of the tile's first element (packed) or of (b, i=0, l0) (strided)
    int ncols;     // valid columns in the tile
    int64_t nvalid;  // packed: valid contiguous elements
};

__device__ __forceinline__ Tile tile_at(const TileMap& m, int64_t t, int64_t rows) {
    Tile r;
    if (m.packed) {
        int64_t b0 = t * m.nbb;
        int64_t nb = m.B - b0 < m.nbb ? m.B - b0 : m.nbb;
        r.base = b0 * rows * m.L;
        r.ncols = (int)(nb * m.L);
        r.nvalid = nb * rows * m.L;
    } else {
        int64_t b = t / m.lsegs;
        int64_t l0 = (t - b * m.lsegs) * m.KT;
        int64_t w = m.L - l0 < m.KT ? m.L - l0 : m.KT;
        r.base = b * rows * m.L + l0;
        r.ncols = (int)w;
        r.nvalid = 0;
    }
    return r;
}

// ------------------------------------------------------------- launch

// Compute units the launch grids are sized for: MI355X's 256, a constant on
// purpose.  Workspace-size queries are host-only (no HIP call, the same
// answer with or without a device), and the partial-sum buffers they size
// follow these grids.  On a part with fewer CUs the grids stay correct, only
// less evenly spread.
int device_cu_count();

// Workspace carving: bump allocator over the caller's buffer, 256-B aligned.
struct Carver {
    char* base;
    size_t size, used;
    explicit Carver(void* p, size_t n) : base((char*)p), size(n), used(0) {}
    void* take(size_t bytes) {
        size_t off = (used + 255) & ~size_t(255);
        used = off + bytes;
        return base ? base + off : nullptr;
    }
    bool ok() const { return used <= size; }
};

// ------------------------------------------------------------- kernels API
// (host-side launchers implemented in the .hip files; arguments already
// validated by the C-ABI layer)

struct GramPlan {
    int KT, P, G, npairs, pairs_per_group, nb;
    int narrow;            // 16 or 32: the FP64 narrow-mode kernel's row extent; 0: tiled
    size_t partial_bytes;  // this shape's partials
    size_t partial_bound;  // partials of any shape with this mode extent (grid cap)
};
// FP64 Gram without an LDS tile: J <= 32 where the unfolding rows are made
// of long contiguous runs (L a multiple of 8, at least kNarrowMinRun).
constexpr int64_t kNarrowMinRun = 64;
inline bool gram_narrow_view(const ModeView& v) {
    return v.J <= 32 && v.L % 8 == 0 && v.L >= kNarrowMinRun;
}
GramPlan plan_gram(const ModeView& v, int precision, int elem_bytes);
GramPlan plan_gram_mixed(const ModeView& v);
int launch_gram_mixed(const float* y, const ModeView& v, const GramPlan& pl, double* partial,
                      hipStream_t st);
// split_stats (may be NULL; split-bf16 Grams only): receives {sum of d^2,
// largest row exponent} of the split representation (see EigArgs).
// ev: NULL, or two events recorded on st just before and just after the
// partial-Gram kernel (not the reduction).
int launch_gram(const void* y, int dtype, const ModeView& v, int precision, double* s,
                double* sumsq, void* ws, size_t ws_bytes, hipStream_t st,
                double* split_stats = nullptr, const hipEvent_t* ev = nullptr);

int launch_ttm(const void* y, int dtype, const ModeView& v, const double* m, int64_t K,
               int64_t ldm, int transpose, int precision, void* z, hipStream_t st);

// Eigendecomposition + truncation of one J x J FP64 Gram matrix (Alg. 1).
// rank_mode: 0 = eps rule with tau = eps2_over_n * (*nu), 1 = fixed rank.
// Writes lambda (J, descending), U (J x R column-major, ld J) into u_out,
// R to *rank_out and the discarded tail sum to *disc_out (device).
struct EigArgs {
    const double* s;
    int J;
    const double* nu;      // device scalar ||X||^2
    double eps2_over_n;    // eps^2 / N
    int fixed_rank;        // > 0: fixed
    int max_rank;          // capacity bound; larger R sets the capacity flag
    double* lambda;        // J
    double* u;             // J x R (capacity J * J)
    int64_t* rank_out;     // device
    double* disc_out;      // device
    int* flags;            // device status flags (bit 0: no convergence, bit 1: capacity,
                           // bit 2: rank within the guard margin)
    double* scratch;       // eig_scratch_doubles(J)
    // Guard of a rank found from a split-bf16 Gram.  With Y the unfolding
    // (K columns), Y~ its split representation and D = Y - Y~, the Gram
    // formed is Y~ Y~^T - diag(D D^T) (the diagonal of D D^T is subtracted
    // exactly, per row), so the computed tail sum t~_R and the exact t_R
    // differ by tr((I-Q) F) with F = offdiag(D D^T) - Y D^T - D Y^T, Q the
    // projector onto the kept space.  The products are exact (the split's
    // halves are 8-bit integers), so D is the whole error; modelling its
    // entries d as quantization noise independent of the data and of each
    // other, mean 0, |d| <= 2^(E_max - 16) (uniform: variance at most
    // delta^2 = 4^(E_max - 16) / 3), tr((I-Q) F) has mean 0 and variance at
    // most 4 delta^2 t + 2 K delta^4 (J - R).  The subtracted diagonal rests
    // on the same model (independent noise adds exactly its energy), so it is
    // trusted only to kSplitModelError of its size, ||D||_F^2.  The bound is
    // `guard` standard deviations of the first part plus
    // kSplitModelError ||D||_F^2 (at t~_R); under the eps rule the rank is
    // certified when tau - t~_R and t~_{R-1} - tau both exceed that bound at
    // their own t and rank; otherwise flag bit 2.
    double guard = 0.0;
    const double* split_stats = nullptr;  // device {sum of d^2, E_max} of the Gram
    double ncols = 0.0;                   // K, the unfolding's columns (an upper bound)
    double* tail_bound = nullptr;         // device out (may be NULL): the bound on
                                          // |t_R - t~_R|; 0 without the guard
    int aug = 0;           // 1: s is [[0, R^T], [R, 0]] (J = 2 J_R): its leading J_R
                           // eigenvalues are sigma_i(R); lambda (J_R values) and the
                           // rank rule use sigma_i^2, u receives 2 J_R x R vectors
};

// Householder QR (R factor only) of A = Y_(n)^T through a reduction tree.
struct QrPlan {
    int JC, BR, levels;           // column class (32/64/128), tile rows, tree levels
    int P[16];                    // workgroups per level
    int64_t rows_per_wg[16];
    size_t part_doubles[2];       // ping-pong partial factors
    size_t ss_doubles;            // first-level sums of squares
};
QrPlan plan_qr(const ModeView& v);
size_t qr_workspace_doubles(const QrPlan& pl);
size_t qr_workspace_bound_doubles(int J);
int launch_tsqr(const void* y, int dtype, const ModeView& v, const QrPlan& pl, double* ws,
                double* r_out, double* sumsq, hipStream_t st);
int launch_jw(const double* r, int J, double* m, hipStream_t st);
int launch_jw_extract(const double* z, int J, int max_rank, const int64_t* rank, double* u,
                      hipStream_t st);

// Standard deviations of the model's error terms the split-Gram guard
// allows for (EigArgs::guard), and the share of ||D||_F^2 it allows for the
// subtracted diagonal (an emulation of this split on combustion-like data
// found the corrected tail sums off by up to about 3% of ||D||_F^2 when
// ||D||_F^2 is a hundred times the threshold, and by 0.04% near it).
constexpr double kSplitGramGuard = 6.0;
constexpr double kSplitModelError = 0.125;

// The split-bf16 TTM leaves a relative error of about 2^-17 in every output,
// which adds about 2^-34 ||X||^2 to later modes' tail sums; below
// eps^2 / N = 8 * 2^-34 the threshold would feel it, so the TTMs run in FP64.
constexpr double kSplitTtmFloor = 8.0 / 17179869184.0;
// The plain bf16 TTM (both operands rounded to bf16) leaves about 2^-8, i.e.
// about 2^-16 ||X||^2 in later tail sums: under the eps rule it keeps the
// same factor 8 only for eps^2 / N >= 8 * 2^-16.
constexpr double kBf16TtmFloor = 8.0 / 65536.0;
// TTM arithmetic under the eps rule: a requested precision whose error would
// reach the rank threshold is raised to the next more accurate one.
inline int ttm_precision_for_eps(int requested, double eps2_over_n) {
    int p = requested;
    if (p == TK_TTM_BF16 && eps2_over_n < kBf16TtmFloor) p = TK_TTM_BF16X3;
    if (p == TK_TTM_BF16X3 && eps2_over_n < kSplitTtmFloor) p = TK_TTM_FP64;
    return p;
}
// Mixed path: modes with J <= 32 and at most this many unfolding elements
// use the FP64 Gram (2^26: 256 MB of FP32), and so does any mode the FP64
// narrow-mode kernel takes.
constexpr double kSmallFp64GramElems = 67108864.0;
inline bool mixed_takes_fp64_gram(const ModeView& v) {
    return v.J <= 32 && ((double)v.L * (double)v.J * (double)v.B <= kSmallFp64GramElems ||
                         gram_narrow_view(v));
}
size_t eig_scratch_doubles(int J);
int launch_eig(const EigArgs& a, hipStream_t st);
size_t eig_lds_bytes(int J);
int launch_eig_batched(const EigArgs* args_dev, int count, int jmax, int conditional,
                       int mode_bit, hipStream_t st);

// ------------------------------------------------------------- batches
// Device-resident task tables of a batch (one entry per problem and mode
// step).  The shapes of later modes depend on ranks found on the device, so
// every workgroup derives its problem's current view from `ranks`: modes in
// `done` have extent ranks[m], the others their original extent.
struct BatchView {
    int64_t dims[TK_MAX_NDIM];
    const int64_t* ranks;  // device, ndim entries
    int ndim, n, done;
    int wg_begin, nwg;     // this problem's workgroups in the launch
};

// Unrolled over the maximal order with constant indices, so that a kernel
// keeps the problem's extents in registers (no private stack array).
__host__ __device__ inline ModeView batch_mode_view(const BatchView& b) {
    ModeView v{1, 1, 1};
#pragma unroll
    for (int m = 0; m < TK_MAX_NDIM; ++m) {
        if (m < b.ndim) {
            const int64_t d = ((b.done >> m) & 1) ? b.ranks[m] : b.dims[m];
            if (m < b.n) v.L *= d;
            else if (m == b.n) v.J = (int)d;
            else v.B *= d;
        }
    }
    return v;
}

// MI355X has 8 XCDs, each with its own L2, and deals consecutive workgroup
// ids to them round-robin.  A Gram whose block pairs are split into G > 1
// groups reads every tile range G times; placing the G workgroups of one
// range on one XCD in consecutive slots lets them stream the same tiles
// through that XCD's L2.  The launch has P * G workgroups, P a multiple of
// kXcds (any mapping would be correct; this one is about locality).
constexpr int kXcds = 8;

__device__ __forceinline__ void xcd_range_group(int b, int G, int& p, int& g) {
    if (G == 1) {
        p = b;
        g = 0;
        return;
    }
    const int x = b % kXcds, s = b / kXcds;
    g = s % G;
    p = x + kXcds * (s / G);
}

// Tile ranges for a G-group Gram: min(ntiles, want), and for G > 1 a multiple
// of kXcds (ranges beyond the tiles are empty and write zero partials).
// `want` is rounded the same way by the caller's workspace bound.
inline int64_t xcd_round_want(int64_t want, int G) {
    if (G == 1) return want < 1 ? 1 : want;
    want = want / kXcds * kXcds;
    return want < kXcds ? kXcds : want;
}
inline int xcd_ranges(int64_t ntiles, int64_t want, int G) {
    int64_t p = ntiles < want ? ntiles : want;
    if (p < 1) p = 1;
    if (G > 1) p = (p + kXcds - 1) / kXcds * kXcds;  // <= want: want is a multiple of kXcds
    return (int)p;
}

// Values the compiler cannot prove wave-uniform (a task table entry found by
// a search, extents read from device memory) but that are: moved to scalar
// registers, so that everything derived from them stays there too.
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t uni(int64_t x) {
    const int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const int hi = __builtin_amdgcn_readfirstlane((int)(x >> 32));
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
template <typename T>
__device__ __forceinline__ T* uni(T* p) {
    return (T*)(uintptr_t)uni((int64_t)(uintptr_t)p);
}
// A wave-uniform pointer to device global memory, typed so: it passes
// through an empty asm as an integer, so the compiler cannot fold the casts
// away, and every access derived from it becomes a global (not flat) load or
// store.  A flat access also counts against the LDS counter, so that LDS
// reads issued behind it would wait for it as well.
template <typename T>
__device__ __forceinline__ T* uni_global(T* p) {
    uint64_t a = (uint64_t)(uintptr_t)uni(p);
    asm volatile("" : "+s"(a));
    return (T*)(__attribute__((address_space(1))) T*)a;
}
__device__ __forceinline__ ModeView uni(const ModeView& v) {
    ModeView u;
    u.L = uni(v.L);
    u.J = uni(v.J);
    u.B = uni(v.B);
    return u;
}

// Task of workgroup `wg` in a launch whose tasks (stride bytes apart, each
// starting with a BatchView) own consecutive workgroup ranges.
__device__ __forceinline__ int find_task_wg(const BatchView* v0, size_t stride, int ntasks,
                                            int wg) {
    int lo = 0, hi = ntasks - 1;  // last task with wg_begin <= wg
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const BatchView* vm = (const BatchView*)((const char*)v0 + (size_t)mid * stride);
        if (vm->wg_begin <= wg) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// A Gram task owns nwg workgroups (sized for the capacity shape); at run time
// only as many take part as the actual tiles need (tpw tiles each for the
// split Gram, at least one tile each for the FP64 Gram), and workgroup 0
// records that count in *nparts for the reduction.
struct BatchGramTask {
    BatchView v;
    const float* y;
    double* partial;     // nwg partial slots
    double* aux;         // nwg x 2 split statistics (split-bf16 Gram)
    const int* status;   // the problem's status word (bit 4: rank not certified,
                         // bit 8: FP64 Gram only)
    int* nparts;         // partial slots written by the last Gram launch
    int tpw;             // split-Gram tiles per workgroup
};
struct BatchTtmTask {
    BatchView v;
    const float* y;
    const double* u;  // factor, I_n x R_n column-major (ld I_n)
    float* z;
};
struct BatchReduceTask {
    const double* partial;
    double* s;
    double* nu;  // trace target or nullptr
    const double* aux;  // split statistics per partial slot, or nullptr
    double* stats;      // {sum of d^2, E_max} over the slots written (with aux)
    int P, npairs, nb, J;  // P: partial slots reserved (the sum runs over *nparts)
    int wg_begin, nwg;
    const int* status;
    const int* nparts;
};

// loaders: bit 0 launches the L == 1 variant, bit 1 the L % 4 == 0 one,
// bit 2 the strided one (7: all three, when the strides are decided on the
// device); a task whose variant is not launched gets no Gram.
int launch_gram_split_batched(const BatchGramTask* tasks_dev, int ntasks, int total_wg, int jb,
                              unsigned loaders, hipStream_t st);
// Sets status bit 8 of every task's problem whose FP64 Gram (2 K J^2 flops at
// the actual shape) is at most max_flops: the split Gram skips it, the FP64
// Gram launched with conditional = 2 takes it, and the reduction and the
// eigensolver treat it as an FP64 Gram (the eigensolver clears the bit).
int launch_batch_mark_fp64(const BatchGramTask* tasks_dev, int ntasks, double max_flops,
                           hipStream_t st);
// J: the largest extent among the tasks (it sets the 32-row k-steps);
// kmax: the largest rank capacity (it sets the 16-row blocks and groups).
int launch_ttm_bf16_batched(const BatchTtmTask* tasks_dev, int ntasks, int total_wg, int J,
                            int kmax, int precision, hipStream_t st);
// conditional = 1: only problems whose status has bit 4 set take part (the
// guard's FP64 recomputation), = 2: only those with bit 8 (FP64-only); the
// others' workgroups return at once.
int launch_gram_f64_batched(const BatchGramTask* tasks_dev, int ntasks, int total_wg, int jb,
                            int conditional, hipStream_t st);
int launch_gram_reduce_batched(const BatchReduceTask* tasks_dev, int ntasks, int total_wg,
                               int conditional, hipStream_t st);
int mx_gram_kt(int jb);   // tile width of the split Gram for a padded extent
int launch_fill_i32(int* p, int n, int v, hipStream_t st);
int check_ws(void* ws, size_t ws_bytes, size_t need, const char* what);

int launch_error_metrics(const void* x, const void* xh, int dtype, int64_t n, double* partial,
                         int nblocks, double* out3, hipStream_t st);
int error_metrics_blocks(int64_t n);

}  // namespace tk
