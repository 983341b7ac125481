// C-ABI entry points: host-side validation (no HIP call before it), workspace
// planning, and the mode loop of Alg. 1 (ST-HOSVD) and of the Tucker
// reconstruction (Sec. II-C).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <mutex>
#include <vector>

#include "tk_common.hpp"

namespace tk {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

int fail(int status, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return status;
}

int device_cu_count() { return 256; }  // MI355X; see tk_common.hpp

int check_shape(const tk_shape* s, const char* what) {
    if (!s) return fail(TK_ERR_INVALID_ARG, "%s: shape is NULL", what);
    if (s->ndim < 1 || s->ndim > TK_MAX_NDIM)
        return fail(TK_ERR_INVALID_ARG, "%s: ndim %d outside [1, %d]", what, s->ndim, TK_MAX_NDIM);
    if (s->dtype != TK_F64 && s->dtype != TK_F32)
        return fail(TK_ERR_INVALID_ARG, "%s: unknown dtype %d", what, s->dtype);
    double total = 1.0;
    for (int k = 0; k < s->ndim; ++k) {
        if (s->dims[k] < 1)
            return fail(TK_ERR_INVALID_ARG, "%s: dims[%d] = %lld < 1", what, k,
                        (long long)s->dims[k]);
        total *= (double)s->dims[k];
    }
    if (total > 9.0e15) return fail(TK_ERR_INVALID_ARG, "%s: tensor too large", what);
    return TK_OK;
}

int check_ws(void* ws, size_t ws_bytes, size_t need, const char* what) {
    if (ws_bytes < need)
        return fail(TK_ERR_WORKSPACE, "%s: workspace %zu bytes < required %zu", what, ws_bytes,
                    need);
    if (need > 0 && (!ws || ((uintptr_t)ws & 255)))
        return fail(TK_ERR_WORKSPACE, "%s: workspace NULL or not 256-byte aligned", what);
    return TK_OK;
}

static bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb) {
    uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b;
    return pa < pb + nb && pb < pa + na;
}

}  // namespace tk

using namespace tk;

// Scalar block of one compression (device): [0] ||X||^2, [1..8] discarded
// sums, [16..23] ranks, [32] status flags, [40..41] split statistics of the
// last split-bf16 Gram, [48..55] tail-sum error bounds.  The per-mode readback copies
// its first 33 doubles in one transfer into pinned host memory allocated
// once per thread (kept for the thread's lifetime: 512 bytes); pageable
// stack memory is the fallback if that allocation fails.
static double* pinned_scalars() {
    static thread_local double* p = nullptr;
    static thread_local bool tried = false;
    if (!tried) {
        tried = true;
        if (hipHostMalloc((void**)&p, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
        }
    }
    return p;
}

static int read_scalars(const double* scal_dev, hipStream_t st, int n, int64_t* rank, double* nu,
                        int* flags) {
    double local[33];
    double* h = pinned_scalars();
    if (!h) h = local;
    TK_HIP(hipMemcpyAsync(h, scal_dev, 33 * sizeof(double), hipMemcpyDeviceToHost, st));
    TK_HIP(hipStreamSynchronize(st));
    int64_t r;
    int f;
    memcpy(&r, h + 16 + n, sizeof r);
    memcpy(&f, h + 32, sizeof f);
    *rank = r;
    *nu = h[0];
    *flags = f;
    return TK_OK;
}

extern "C" {

const char* tk_status_string(int status) {
    switch (status) {
        case TK_OK: return "ok";
        case TK_ERR_INVALID_ARG: return "invalid argument";
        case TK_ERR_UNSUPPORTED: return "unsupported dtype/precision combination";
        case TK_ERR_WORKSPACE: return "workspace too small or misaligned";
        case TK_ERR_HIP: return "HIP runtime error";
        case TK_ERR_NONFINITE: return "input holds Inf or NaN";
        case TK_ERR_EIG_NO_CONVERGENCE: return "eigensolver did not converge";
        case TK_ERR_CAPACITY: return "output capacity exceeded";
        default: return "unknown status";
    }
}

const char* tk_last_error(void) { return g_err; }

// ------------------------------------------------------------------ Gram

static int check_gram_args(const tk_shape* y, int mode, int precision) {
    TK_TRY(check_shape(y, "gram_mode_n"));
    if (mode < 0 || mode >= y->ndim)
        return fail(TK_ERR_INVALID_ARG, "gram_mode_n: mode %d outside [0, %d)", mode, y->ndim);
    if (y->dims[mode] > TK_MAX_MODE_DIM)
        return fail(TK_ERR_UNSUPPORTED, "gram_mode_n: dims[%d] = %lld exceeds %d", mode,
                    (long long)y->dims[mode], TK_MAX_MODE_DIM);
    if (precision != TK_GRAM_FP64 && precision != TK_GRAM_SPLIT_BF16)
        return fail(TK_ERR_INVALID_ARG, "gram_mode_n: unknown precision %d", precision);
    if (precision == TK_GRAM_SPLIT_BF16 && y->dtype != TK_F32)
        return fail(TK_ERR_UNSUPPORTED, "gram_mode_n: split-bf16 Gram needs FP32 input");
    return TK_OK;
}

size_t gram_workspace_bytes(const tk_shape* y, int mode, int precision) {
    if (check_gram_args(y, mode, precision) != TK_OK) return 0;
    ModeView v = mode_view(y->dims, y->ndim, mode);
    GramPlan pl = plan_gram(v, precision, (int)dtype_size(y->dtype));
    return pl.partial_bytes + 256;
}

int gram_mode_n(const tk_shape* y, const void* y_dev, int mode, int precision, double* s_dev,
                double* sumsq_dev, void* ws, size_t ws_bytes, void* stream) {
    TK_TRY(check_gram_args(y, mode, precision));
    if (!y_dev || !s_dev) return fail(TK_ERR_INVALID_ARG, "gram_mode_n: NULL device pointer");
    size_t need = gram_workspace_bytes(y, mode, precision);
    TK_TRY(check_ws(ws, ws_bytes, need, "gram_mode_n"));
    ModeView v = mode_view(y->dims, y->ndim, mode);
    return launch_gram(y_dev, y->dtype, v, precision, s_dev, sumsq_dev, ws, ws_bytes,
                       (hipStream_t)stream);
}

// -------------------------------------------------- Gram without allocation
//
// The scratch of gram_mode_n_noalloc: a file-scope device array, one copy on
// each device the library runs on, held until the process ends.  Host code
// never uses the array's name as an address: each device's copy is looked up
// once (hipGetSymbolAddress with that device current) and that pointer is what
// the kernels receive.
constexpr size_t kNoAllocScratchBytes = (size_t)72 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {nullptr};

int scratch_for_current_device(void** out) {
    int dev = 0;
    TK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(TK_ERR_UNSUPPORTED, "gram_mode_n_noalloc: device %d beyond %d", dev,
                    kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        TK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return TK_OK;
}
}  // namespace

size_t gram_noalloc_scratch_bytes(void) { return kNoAllocScratchBytes; }

int gram_mode_n_noalloc(const tk_shape* y, const void* y_dev, int mode, int precision,
                        double* s_dev, double* sumsq_dev, void* stream) {
    TK_TRY(check_gram_args(y, mode, precision));
    if (!y_dev || !s_dev)
        return fail(TK_ERR_INVALID_ARG, "gram_mode_n_noalloc: NULL device pointer");
    const size_t need = gram_workspace_bytes(y, mode, precision);
    if (need > kNoAllocScratchBytes)
        return fail(TK_ERR_WORKSPACE, "gram_mode_n_noalloc: this shape needs %zu bytes of scratch, "
                    "more than the static %zu", need, kNoAllocScratchBytes);
    void* ws = nullptr;
    TK_TRY(scratch_for_current_device(&ws));
    ModeView v = mode_view(y->dims, y->ndim, mode);
    // every partial slot the kernels read is written by them first: nothing
    // in the scratch has to start at zero
    return launch_gram(y_dev, y->dtype, v, precision, s_dev, sumsq_dev, ws, kNoAllocScratchBytes,
                       (hipStream_t)stream);
}

// -------------------------------------------------------------------- QR

static int check_qr_args(const tk_shape* y, int mode) {
    TK_TRY(check_shape(y, "qr_r_mode_n"));
    if (mode < 0 || mode >= y->ndim)
        return fail(TK_ERR_INVALID_ARG, "qr_r_mode_n: mode %d outside [0, %d)", mode, y->ndim);
    if (y->dims[mode] > TK_QR_MAX_MODE_DIM)
        return fail(TK_ERR_UNSUPPORTED, "qr_r_mode_n: dims[%d] = %lld exceeds %d", mode,
                    (long long)y->dims[mode], TK_QR_MAX_MODE_DIM);
    return TK_OK;
}

size_t qr_workspace_bytes(const tk_shape* y, int mode) {
    if (check_qr_args(y, mode) != TK_OK) return 0;
    ModeView v = mode_view(y->dims, y->ndim, mode);
    return qr_workspace_doubles(plan_qr(v)) * sizeof(double) + 256;
}

int qr_r_mode_n(const tk_shape* y, const void* y_dev, int mode, double* r_dev,
                double* sumsq_dev, void* ws, size_t ws_bytes, void* stream) {
    TK_TRY(check_qr_args(y, mode));
    if (!y_dev || !r_dev) return fail(TK_ERR_INVALID_ARG, "qr_r_mode_n: NULL device pointer");
    TK_TRY(check_ws(ws, ws_bytes, qr_workspace_bytes(y, mode), "qr_r_mode_n"));
    ModeView v = mode_view(y->dims, y->ndim, mode);
    return launch_tsqr(y_dev, y->dtype, v, plan_qr(v), (double*)ws, r_dev, sumsq_dev,
                       (hipStream_t)stream);
}

// ------------------------------------------------------------------- TTM

static int check_ttm_args(const tk_shape* y, int mode, int64_t m_rows, int64_t m_cols,
                          int transpose, int precision, int64_t* K) {
    TK_TRY(check_shape(y, "ttm_mode_n"));
    if (mode < 0 || mode >= y->ndim)
        return fail(TK_ERR_INVALID_ARG, "ttm_mode_n: mode %d outside [0, %d)", mode, y->ndim);
    if (y->dims[mode] > TK_MAX_MODE_DIM)
        return fail(TK_ERR_UNSUPPORTED, "ttm_mode_n: dims[%d] = %lld exceeds %d", mode,
                    (long long)y->dims[mode], TK_MAX_MODE_DIM);
    if (transpose != 0 && transpose != 1)
        return fail(TK_ERR_INVALID_ARG, "ttm_mode_n: transpose must be 0 or 1");
    int64_t jn = transpose ? m_rows : m_cols;
    *K = transpose ? m_cols : m_rows;
    if (m_rows < 1 || m_cols < 1 || jn != y->dims[mode])
        return fail(TK_ERR_INVALID_ARG,
                    "ttm_mode_n: op(M) must be K x dims[mode] (m_rows=%lld m_cols=%lld "
                    "transpose=%d dims[mode]=%lld)",
                    (long long)m_rows, (long long)m_cols, transpose, (long long)y->dims[mode]);
    if (*K > (1 << 20)) return fail(TK_ERR_UNSUPPORTED, "ttm_mode_n: K too large");
    if (precision != TK_TTM_FP64 && precision != TK_TTM_BF16 && precision != TK_TTM_BF16X3)
        return fail(TK_ERR_INVALID_ARG, "ttm_mode_n: unknown precision %d", precision);
    if (precision != TK_TTM_FP64 && y->dtype != TK_F32)
        return fail(TK_ERR_UNSUPPORTED, "ttm_mode_n: bf16 TTM variants need FP32 storage");
    return TK_OK;
}

int ttm_mode_n(const tk_shape* y, const void* y_dev, int mode, const double* m_dev,
               int64_t m_rows, int64_t m_cols, int transpose, int precision, void* z_dev,
               void* stream) {
    int64_t K;
    TK_TRY(check_ttm_args(y, mode, m_rows, m_cols, transpose, precision, &K));
    if (!y_dev || !m_dev || !z_dev) return fail(TK_ERR_INVALID_ARG, "ttm_mode_n: NULL pointer");
    size_t b = dtype_size(y->dtype);
    int64_t ny = numel(*y), nz = ny / y->dims[mode] * K;
    if (ranges_overlap(y_dev, ny * b, z_dev, nz * b))
        return fail(TK_ERR_INVALID_ARG, "ttm_mode_n: output overlaps input");
    ModeView v = mode_view(y->dims, y->ndim, mode);
    return launch_ttm(y_dev, y->dtype, v, m_dev, K, m_rows, transpose, precision, z_dev,
                      (hipStream_t)stream);
}

// -------------------------------------------------------------- ST-HOSVD

struct SthosvdPlan {
    int N;
    int order[TK_MAX_NDIM];
    int64_t cap[TK_MAX_NDIM];   // rank capacity per mode
    size_t y_bytes[2];          // ping-pong buffers
    size_t gram_bytes, s_bytes, eig_bytes, lam_bytes;
    size_t qr_bytes, r_bytes, z_bytes;  // TK_SVD_QR only
    size_t total;
};

static int check_options(const tk_shape* x, const tk_options* opt, SthosvdPlan* pl) {
    TK_TRY(check_shape(x, "sthosvd_compress"));
    if (!opt) return fail(TK_ERR_INVALID_ARG, "sthosvd_compress: options NULL");
    if (!(opt->eps >= 0.0) || !std::isfinite(opt->eps))
        return fail(TK_ERR_INVALID_ARG, "sthosvd_compress: eps must be finite and >= 0");
    const int N = x->ndim;
    pl->N = N;
    bool seen[TK_MAX_NDIM] = {false};
    for (int k = 0; k < N; ++k) {
        int n = opt->mode_order ? opt->mode_order[k] : k;
        if (n < 0 || n >= N || seen[n])
            return fail(TK_ERR_INVALID_ARG, "sthosvd_compress: mode_order is not a permutation");
        seen[n] = true;
        pl->order[k] = n;
        if (x->dims[n] > TK_MAX_MODE_DIM)
            return fail(TK_ERR_UNSUPPORTED, "sthosvd_compress: dims[%d] = %lld exceeds %d", n,
                        (long long)x->dims[n], TK_MAX_MODE_DIM);
    }
    for (int n = 0; n < N; ++n) {
        int64_t c = x->dims[n];
        if (opt->max_ranks) {
            if (opt->max_ranks[n] < 1)
                return fail(TK_ERR_INVALID_ARG, "sthosvd_compress: max_ranks[%d] < 1", n);
            if (opt->max_ranks[n] < c) c = opt->max_ranks[n];
        }
        if (opt->fixed_ranks) {
            int64_t r = opt->fixed_ranks[n];
            if (r < 1 || r > x->dims[n])
                return fail(TK_ERR_INVALID_ARG, "sthosvd_compress: fixed_ranks[%d] = %lld not in "
                            "[1, %lld]", n, (long long)r, (long long)x->dims[n]);
            if (r > c)
                return fail(TK_ERR_CAPACITY, "sthosvd_compress: fixed_ranks[%d] exceeds max_ranks",
                            n);
            c = r;
        }
        pl->cap[n] = c;
    }
    const bool qr = opt->gram_precision == TK_SVD_QR;
    if (opt->gram_precision != TK_GRAM_FP64 && opt->gram_precision != TK_GRAM_SPLIT_BF16 && !qr)
        return fail(TK_ERR_INVALID_ARG, "sthosvd_compress: unknown gram precision");
    if (qr)
        for (int n = 0; n < N; ++n)
            if (x->dims[n] > TK_QR_MAX_MODE_DIM)
                return fail(TK_ERR_UNSUPPORTED, "sthosvd_compress: the QR path needs dims[%d] "
                            "<= %d", n, TK_QR_MAX_MODE_DIM);
    if (opt->ttm_precision != TK_TTM_FP64 && opt->ttm_precision != TK_TTM_BF16 &&
        opt->ttm_precision != TK_TTM_BF16X3)
        return fail(TK_ERR_INVALID_ARG, "sthosvd_compress: unknown ttm precision");
    if (x->dtype != TK_F32 &&
        (opt->gram_precision == TK_GRAM_SPLIT_BF16 || opt->ttm_precision != TK_TTM_FP64))
        return fail(TK_ERR_UNSUPPORTED, "sthosvd_compress: bf16 paths need FP32 storage");

    // workspace plan: sizes at the rank capacities
    const size_t b = dtype_size(x->dtype);
    int64_t cur[TK_MAX_NDIM];
    for (int k = 0; k < N; ++k) cur[k] = x->dims[k];
    pl->y_bytes[0] = pl->y_bytes[1] = 0;
    pl->gram_bytes = 0;
    int jmax = 1;
    for (int s = 0; s < N; ++s) {
        int n = pl->order[s];
        ModeView v = mode_view(cur, N, n);
        // the tile count (hence the partial count) depends on the ranks found
        // at run time, so size for the grid cap of this mode's extent
        GramPlan gp = plan_gram(v, qr ? TK_GRAM_FP64 : opt->gram_precision, (int)b);
        size_t gb = qr ? 0 : gp.partial_bound;
        if (gb > pl->gram_bytes) pl->gram_bytes = gb;
        if (opt->gram_precision == TK_GRAM_SPLIT_BF16) {  // room for the guard's FP64 Gram
            GramPlan g64 = plan_gram(v, TK_GRAM_FP64, (int)b);
            if (g64.partial_bound > pl->gram_bytes) pl->gram_bytes = g64.partial_bound;
        }
        if (v.J > jmax) jmax = v.J;
        cur[n] = pl->cap[n];
        if (s + 1 < N) {
            int64_t ne = 1;
            for (int k = 0; k < N; ++k) ne *= cur[k];
            size_t by = (size_t)ne * b;
            if (by > pl->y_bytes[s & 1]) pl->y_bytes[s & 1] = by;
        }
    }
    // the QR path hands the eigensolver 2J x 2J matrices
    const int jeig = qr ? 2 * jmax : jmax;
    pl->s_bytes = (size_t)jeig * jeig * sizeof(double);
    pl->eig_bytes = eig_scratch_doubles(jeig) * sizeof(double);
    pl->qr_bytes = qr ? qr_workspace_bound_doubles(jmax) * sizeof(double) : 0;
    pl->r_bytes = qr ? (size_t)jmax * jmax * sizeof(double) : 0;
    pl->z_bytes = qr ? (size_t)2 * jmax * jmax * sizeof(double) : 0;
    int64_t sumdims = 0;
    for (int k = 0; k < N; ++k) sumdims += x->dims[k];
    pl->lam_bytes = (size_t)sumdims * sizeof(double);
    Carver c(nullptr, 0);
    c.take(pl->y_bytes[0]);
    c.take(pl->y_bytes[1]);
    c.take(pl->gram_bytes);
    c.take(pl->s_bytes);
    c.take(pl->eig_bytes);
    c.take(pl->lam_bytes);
    c.take(64 * sizeof(double));  // scalars
    c.take(pl->qr_bytes);
    c.take(pl->r_bytes);
    c.take(pl->z_bytes);
    pl->total = c.used + 256;
    return TK_OK;
}

size_t sthosvd_workspace_bytes(const tk_shape* x, const tk_options* opt) {
    SthosvdPlan pl;
    if (check_options(x, opt, &pl) != TK_OK) return 0;
    return pl.total;
}

int sthosvd_compress(const tk_shape* x, const void* x_dev, const tk_options* opt,
                     tk_tucker* out, void* ws, size_t ws_bytes, void* stream) {
    SthosvdPlan pl;
    TK_TRY(check_options(x, opt, &pl));
    if (!x_dev) return fail(TK_ERR_INVALID_ARG, "sthosvd_compress: x_dev NULL");
    if (!out || !out->core_dev || out->core_capacity < 1)
        return fail(TK_ERR_INVALID_ARG, "sthosvd_compress: output core missing");
    const int N = pl.N;
    for (int n = 0; n < N; ++n)
        if (!out->factors_dev[n])
            return fail(TK_ERR_INVALID_ARG, "sthosvd_compress: factors_dev[%d] NULL", n);
    TK_TRY(check_ws(ws, ws_bytes, pl.total, "sthosvd_compress"));
    hipStream_t st = (hipStream_t)stream;

    Carver c(ws, ws_bytes);
    void* ybuf[2] = {c.take(pl.y_bytes[0]), c.take(pl.y_bytes[1])};
    void* gram_ws = c.take(pl.gram_bytes);
    double* S = (double*)c.take(pl.s_bytes);
    double* eig_ws = (double*)c.take(pl.eig_bytes);
    double* lam_ws = (double*)c.take(pl.lam_bytes);
    double* scal = (double*)c.take(64 * sizeof(double));
    double* qr_ws = (double*)c.take(pl.qr_bytes);
    double* r_ws = (double*)c.take(pl.r_bytes);
    double* z_ws = (double*)c.take(pl.z_bytes);
    const bool qr = opt->gram_precision == TK_SVD_QR;
    double* nu_dev = scal;                       // [0]
    double* disc_dev = scal + 1;                 // [1..8]
    int64_t* rank_dev = (int64_t*)(scal + 16);   // [16..23]
    int* flags_dev = (int*)(scal + 32);          // [32]
    double* stats_dev = scal + 40;               // [40..41]
    double* bound_dev = scal + 48;               // [48..55]
    double* lam_all = out->eigvals_dev ? out->eigvals_dev : lam_ws;

    TK_HIP(hipMemsetAsync(scal, 0, 64 * sizeof(double), st));
    // events around the first mode's partial Gram, destroyed on every return
    struct GramEvents {
        hipEvent_t e[2] = {nullptr, nullptr};
        ~GramEvents() {
            for (hipEvent_t x : e)
                if (x) (void)hipEventDestroy(x);
        }
    } gev;
    out->first_gram_ms = 0.0;
    if (opt->time_first_gram && !qr) {
        TK_HIP(hipEventCreate(&gev.e[0]));
        TK_HIP(hipEventCreate(&gev.e[1]));
    }

    int64_t lam_off[TK_MAX_NDIM];
    {
        int64_t o = 0;
        for (int n = 0; n < N; ++n) {
            lam_off[n] = o;
            o += x->dims[n];
        }
    }
    int64_t cur[TK_MAX_NDIM];
    for (int k = 0; k < N; ++k) cur[k] = x->dims[k];
    const void* ycur = x_dev;
    const double eps2n = opt->eps * opt->eps / (double)N;
    uint32_t fp64_modes = 0;
    const int ttm_prec = opt->fixed_ranks ? opt->ttm_precision
                                          : ttm_precision_for_eps(opt->ttm_precision, eps2n);
    double nu_host = 0.0;

    for (int s = 0; s < N; ++s) {
        const int n = pl.order[s];
        ModeView v = mode_view(cur, N, n);
        // A narrow mode (J <= 32) over a small unfolding, or one the narrow
        // FP64 kernel streams, takes the FP64 Gram even on the mixed path: at
        // J <= 32 its arithmetic intensity on FP32 data, (J + 1) / 4 flop/B,
        // is below the FP64 MFMA ridge, so it costs no more than the split
        // one, and it needs no guard recomputation.
        int gprec = opt->gram_precision;
        if (gprec == TK_GRAM_SPLIT_BF16 && mixed_takes_fp64_gram(v)) gprec = TK_GRAM_FP64;
        if (qr) {
            // R of Y_(n)^T, then the Jordan-Wielandt matrix [[0, R^T], [R, 0]]
            TK_TRY(launch_tsqr(ycur, x->dtype, v, plan_qr(v), qr_ws, r_ws,
                               s == 0 ? nu_dev : nullptr, st));
            TK_TRY(launch_jw(r_ws, v.J, S, st));
        } else {
            TK_TRY(launch_gram(ycur, x->dtype, v, gprec, S, s == 0 ? nu_dev : nullptr, gram_ws,
                               pl.gram_bytes, st,
                               gprec == TK_GRAM_SPLIT_BF16 ? stats_dev : nullptr,
                               s == 0 && gev.e[0] ? gev.e : nullptr));
        }
        EigArgs ea;
        ea.s = S;
        ea.J = qr ? 2 * v.J : v.J;
        ea.aug = qr ? 1 : 0;
        ea.nu = nu_dev;
        ea.eps2_over_n = eps2n;
        ea.fixed_rank = opt->fixed_ranks ? (int)opt->fixed_ranks[n] : 0;
        ea.max_rank = (int)pl.cap[n];
        ea.lambda = lam_all + lam_off[n];
        ea.u = qr ? z_ws : out->factors_dev[n];
        ea.rank_out = rank_dev + n;
        ea.disc_out = disc_dev + n;
        ea.flags = flags_dev;
        ea.scratch = eig_ws;
        const bool mixed = gprec == TK_GRAM_SPLIT_BF16;
        // split Gram: bound the tail-sum error (and, under the eps rule,
        // certify the rank) from its measured representation error
        ea.guard = mixed ? kSplitGramGuard : 0.0;
        ea.split_stats = mixed ? stats_dev : nullptr;
        ea.ncols = (double)v.L * (double)v.B;
        ea.tail_bound = bound_dev + n;
        TK_TRY(launch_eig(ea, st));
        if (qr) TK_TRY(launch_jw_extract(z_ws, v.J, (int)pl.cap[n], rank_dev + n,
                                         out->factors_dev[n], st));

        int64_t R;
        if (opt->fixed_ranks && s > 0) {
            R = opt->fixed_ranks[n];
        } else {
            // the rank (and, after the first Gram, ||X||^2) must reach the host:
            // one copy of the scalar block into pinned memory, then a sync
            int64_t rk;
            int flags;
            double nu_read;
            TK_TRY(read_scalars(scal, st, n, &rk, &nu_read, &flags));
            if (flags & 4) {
                // the mixed Gram cannot certify this rank: redo the mode in FP64
                TK_HIP(hipMemsetAsync(flags_dev, 0, sizeof(int), st));
                TK_TRY(launch_gram(ycur, x->dtype, v, TK_GRAM_FP64, S, s == 0 ? nu_dev : nullptr,
                                   gram_ws, pl.gram_bytes, st));
                ea.guard = 0.0;  // an FP64 Gram: plain rank rule
                ea.split_stats = nullptr;
                TK_TRY(launch_eig(ea, st));
                TK_TRY(read_scalars(scal, st, n, &rk, &nu_read, &flags));
                fp64_modes |= 1u << n;
            }
            nu_host = nu_read;
            if (!std::isfinite(nu_host))
                return fail(TK_ERR_NONFINITE, "sthosvd_compress: input holds Inf or NaN");
            if (flags & 2)
                return fail(TK_ERR_CAPACITY, "sthosvd_compress: rank of mode %d exceeds max_ranks",
                            n);
            R = rk;
        }
        int64_t nxt[TK_MAX_NDIM];
        memcpy(nxt, cur, sizeof cur);
        nxt[n] = R;
        void* dst;
        if (s + 1 == N) {
            int64_t ncore = 1;
            for (int k = 0; k < N; ++k) ncore *= nxt[k];
            if (ncore > out->core_capacity)
                return fail(TK_ERR_CAPACITY, "sthosvd_compress: core has %lld elements, capacity "
                            "%lld", (long long)ncore, (long long)out->core_capacity);
            dst = out->core_dev;
        } else {
            dst = ybuf[s & 1];
        }
        TK_TRY(launch_ttm(ycur, x->dtype, v, out->factors_dev[n], R, v.J, 1, ttm_prec, dst, st));
        memcpy(cur, nxt, sizeof cur);
        ycur = dst;
    }
    double disc[TK_MAX_NDIM], bounds[TK_MAX_NDIM];
    int flags = 0;
    TK_HIP(hipMemcpyAsync(disc, disc_dev, N * sizeof(double), hipMemcpyDeviceToHost, st));
    TK_HIP(hipMemcpyAsync(bounds, bound_dev, N * sizeof(double), hipMemcpyDeviceToHost, st));
    TK_HIP(hipMemcpyAsync(&nu_host, nu_dev, sizeof(double), hipMemcpyDeviceToHost, st));
    TK_HIP(hipMemcpyAsync(&flags, flags_dev, sizeof(int), hipMemcpyDeviceToHost, st));
    TK_HIP(hipStreamSynchronize(st));
    if (!std::isfinite(nu_host))
        return fail(TK_ERR_NONFINITE, "sthosvd_compress: input holds Inf or NaN");
    if (flags & 2) return fail(TK_ERR_CAPACITY, "sthosvd_compress: a rank exceeds max_ranks");
    for (int n = 0; n < N; ++n) {
        out->ranks[n] = cur[n];
        out->discarded[n] = disc[n];
        out->tail_error_bound[n] = bounds[n];
    }
    out->norm2 = nu_host;
    out->fp64_modes = fp64_modes;
    out->ttm_precision_used = ttm_prec;
    if (gev.e[0]) {  // both recorded before the synchronisation above
        float ms = 0.0f;
        TK_HIP(hipEventElapsedTime(&ms, gev.e[0], gev.e[1]));
        out->first_gram_ms = ms;
    }
    return TK_OK;
}

// --------------------------------------------------------- reconstruction

// Products are applied in increasing order of growth full/rank so the
// intermediate tensors stay as small as possible.
static void recon_order(const tk_shape* core, const int64_t* full, int* order) {
    int N = core->ndim;
    for (int k = 0; k < N; ++k) order[k] = k;
    for (int a = 1; a < N; ++a) {
        int cur = order[a], b2 = a - 1;
        double gc = (double)full[cur] / (double)core->dims[cur];
        while (b2 >= 0 && (double)full[order[b2]] / (double)core->dims[order[b2]] > gc) {
            order[b2 + 1] = order[b2];
            --b2;
        }
        order[b2 + 1] = cur;
    }
}

static int check_recon(const tk_shape* core, const int64_t* full_dims, size_t* bufs) {
    TK_TRY(check_shape(core, "tucker_reconstruct"));
    if (!full_dims) return fail(TK_ERR_INVALID_ARG, "tucker_reconstruct: full_dims NULL");
    const int N = core->ndim;
    double tot = 1.0;
    for (int n = 0; n < N; ++n) {
        if (full_dims[n] < 1 || full_dims[n] > (1 << 20))
            return fail(TK_ERR_INVALID_ARG, "tucker_reconstruct: full_dims[%d] invalid", n);
        if (core->dims[n] > TK_MAX_MODE_DIM)
            return fail(TK_ERR_UNSUPPORTED, "tucker_reconstruct: rank %lld exceeds %d",
                        (long long)core->dims[n], TK_MAX_MODE_DIM);
        tot *= (double)full_dims[n];
    }
    if (tot > 9.0e15) return fail(TK_ERR_INVALID_ARG, "tucker_reconstruct: output too large");
    int order[TK_MAX_NDIM];
    recon_order(core, full_dims, order);
    int64_t cur[TK_MAX_NDIM];
    for (int k = 0; k < N; ++k) cur[k] = core->dims[k];
    size_t b = dtype_size(core->dtype);
    bufs[0] = bufs[1] = 0;
    for (int s = 0; s + 1 < N; ++s) {
        cur[order[s]] = full_dims[order[s]];
        int64_t ne = 1;
        for (int k = 0; k < N; ++k) ne *= cur[k];
        size_t by = (size_t)ne * b;
        if (by > bufs[s & 1]) bufs[s & 1] = by;
    }
    return TK_OK;
}

size_t reconstruct_workspace_bytes(const tk_shape* core, const int64_t* full_dims) {
    size_t bufs[2];
    if (check_recon(core, full_dims, bufs) != TK_OK) return 0;
    Carver c(nullptr, 0);
    c.take(bufs[0]);
    c.take(bufs[1]);
    return c.used + 256;
}

int tucker_reconstruct(const tk_shape* core, const void* core_dev,
                       const double* const* factors_dev, const int64_t* factor_ld,
                       const int64_t* full_dims, int precision, void* xhat_dev, void* ws,
                       size_t ws_bytes, void* stream) {
    size_t bufs[2];
    TK_TRY(check_recon(core, full_dims, bufs));
    if (!core_dev || !factors_dev || !xhat_dev)
        return fail(TK_ERR_INVALID_ARG, "tucker_reconstruct: NULL pointer");
    const int N = core->ndim;
    for (int n = 0; n < N; ++n) {
        if (!factors_dev[n])
            return fail(TK_ERR_INVALID_ARG, "tucker_reconstruct: factors_dev[%d] NULL", n);
        if (factor_ld && factor_ld[n] < full_dims[n])
            return fail(TK_ERR_INVALID_ARG, "tucker_reconstruct: factor_ld[%d] < full_dims", n);
    }
    if (precision != TK_TTM_FP64 && precision != TK_TTM_BF16 && precision != TK_TTM_BF16X3)
        return fail(TK_ERR_INVALID_ARG, "tucker_reconstruct: unknown precision %d", precision);
    if (precision != TK_TTM_FP64 && core->dtype != TK_F32)
        return fail(TK_ERR_UNSUPPORTED, "tucker_reconstruct: bf16 variants need FP32 storage");
    size_t need = reconstruct_workspace_bytes(core, full_dims);
    TK_TRY(check_ws(ws, ws_bytes, need, "tucker_reconstruct"));
    hipStream_t st = (hipStream_t)stream;
    Carver c(ws, ws_bytes);
    void* buf[2] = {c.take(bufs[0]), c.take(bufs[1])};
    int order[TK_MAX_NDIM];
    recon_order(core, full_dims, order);
    int64_t cur[TK_MAX_NDIM];
    for (int k = 0; k < N; ++k) cur[k] = core->dims[k];
    const void* src = core_dev;
    for (int s = 0; s < N; ++s) {
        int n = order[s];
        ModeView v = mode_view(cur, N, n);
        void* dst = (s + 1 == N) ? xhat_dev : buf[s & 1];
        int64_t ld = factor_ld ? factor_ld[n] : full_dims[n];
        TK_TRY(launch_ttm(src, core->dtype, v, factors_dev[n], full_dims[n], ld, 0, precision,
                          dst, st));
        cur[n] = full_dims[n];
        src = dst;
    }
    return TK_OK;
}

// ---------------------------------------------------------------- metrics

size_t error_metrics_workspace_bytes(const tk_shape* x) {
    if (check_shape(x, "tucker_error_metrics") != TK_OK) return 0;
    int nb = error_metrics_blocks(numel(*x));
    return (size_t)(3 * nb + 3) * sizeof(double) + 512;
}

int tucker_error_metrics(const tk_shape* x, const void* x_dev, const void* xhat_dev,
                         double* out_host, void* ws, size_t ws_bytes, void* stream) {
    TK_TRY(check_shape(x, "tucker_error_metrics"));
    if (!x_dev || !xhat_dev || !out_host)
        return fail(TK_ERR_INVALID_ARG, "tucker_error_metrics: NULL pointer");
    TK_TRY(check_ws(ws, ws_bytes, error_metrics_workspace_bytes(x), "tucker_error_metrics"));
    hipStream_t st = (hipStream_t)stream;
    int64_t n = numel(*x);
    int nb = error_metrics_blocks(n);
    Carver c(ws, ws_bytes);
    double* part = (double*)c.take((size_t)3 * nb * sizeof(double));
    double* out3 = (double*)c.take(3 * sizeof(double));
    TK_TRY(launch_error_metrics(x_dev, xhat_dev, x->dtype, n, part, nb, out3, st));
    TK_HIP(hipMemcpyAsync(out_host, out3, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
    TK_HIP(hipStreamSynchronize(st));
    return TK_OK;
}

int sthosvd_mode_order(int ndim, const int64_t* dims, const int64_t* ranks, int rule,
                       int elem_bytes, int* order_out) {
    if (ndim < 1 || ndim > TK_MAX_NDIM)
        return fail(TK_ERR_INVALID_ARG, "sthosvd_mode_order: ndim %d outside [1, %d]", ndim,
                    TK_MAX_NDIM);
    if (!dims || !ranks || !order_out)
        return fail(TK_ERR_INVALID_ARG, "sthosvd_mode_order: NULL pointer");
    for (int k = 0; k < ndim; ++k)
        if (dims[k] < 1 || ranks[k] < 1 || ranks[k] > dims[k])
            return fail(TK_ERR_INVALID_ARG, "sthosvd_mode_order: mode %d has extent %lld, rank %lld",
                        k, (long long)dims[k], (long long)ranks[k]);
    if (rule == TK_ORDER_GREEDY_FLOPS || rule == TK_ORDER_GREEDY_RATIO) {
        bool used[TK_MAX_NDIM] = {false};
        for (int s = 0; s < ndim; ++s) {
            int best = -1;
            for (int k = 0; k < ndim; ++k) {
                if (used[k]) continue;
                if (best < 0) {
                    best = k;
                    continue;
                }
                bool better;
                if (rule == TK_ORDER_GREEDY_FLOPS)  // least I + R (#Y is common to all choices)
                    better = dims[k] + ranks[k] < dims[best] + ranks[best];
                else  // largest I / R, compared exactly as I_k R_best > I_best R_k
                    better = (double)dims[k] * (double)ranks[best] >
                             (double)dims[best] * (double)ranks[k];
                if (better) best = k;
            }
            used[best] = true;
            order_out[s] = best;
        }
        return TK_OK;
    }
    if (rule != TK_ORDER_MIN_BYTES)
        return fail(TK_ERR_INVALID_ARG, "sthosvd_mode_order: unknown rule %d", rule);
    if (elem_bytes < 1) return fail(TK_ERR_INVALID_ARG, "sthosvd_mode_order: elem_bytes < 1");
    int perm[TK_MAX_NDIM];
    for (int k = 0; k < ndim; ++k) perm[k] = k;
    double best_cost = -1.0;
    do {  // permutations in lexicographic order: the first minimum wins ties
        double cur[TK_MAX_NDIM], cost = 0.0;
        for (int k = 0; k < ndim; ++k) cur[k] = (double)dims[k];
        for (int s = 0; s < ndim; ++s) {
            double ny = 1.0;
            for (int k = 0; k < ndim; ++k) ny *= cur[k];
            const int n = perm[s];
            cur[n] = (double)ranks[n];
            cost += 2.0 * ny + ny / (double)dims[n] * (double)ranks[n];
        }
        cost *= (double)elem_bytes;
        if (best_cost < 0.0 || cost < best_cost) {
            best_cost = cost;
            for (int k = 0; k < ndim; ++k) order_out[k] = perm[k];
        }
    } while (std::next_permutation(perm, perm + ndim));
    return TK_OK;
}

}  // extern "C"
