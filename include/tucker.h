/*
 * tucker.h -- C-ABI of the MI355X (gfx950) ST-HOSVD library.
 *
 * The library computes the sequentially truncated HOSVD of a dense N-way
 * tensor (Austin, Ballard, Kolda, "Parallel Tensor Compression for
 * Large-Scale Scientific Data", Alg. 1) and the Tucker reconstruction
 * (Sec. II-C) on one GPU, with hand-written HIP kernels.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Layout.  A tensor of dims (I_1..I_N) is stored densely with mode 1 fastest:
 *   element (i_1..i_N) sits at offset sum_k i_k prod_{m<k} I_m
 * (the mode-1 unfolding is column-major, Sec. IV-A).  tk_shape.dims[0] is the
 * fastest mode; modes are 0-based in this ABI.  The mode-n unfolding is never
 * formed: kernels read the tensor as [B][J_n][L] with L = prod_{m<n} J_m and
 * B = prod_{m>n} J_m, the block-column view of Sec. IV-C.
 * Matrices (factors U_n, TTM operands, Gram matrices) are column-major with
 * leading dimension equal to their row count, FP64 unless stated.
 *
 * Memory.  Every pointer named *_dev is a device pointer (hipMalloc memory or
 * a torch CUDA tensor's data pointer) owned by the caller; the library never
 * allocates or frees device memory.  Scratch memory comes in through a
 * caller-owned workspace (ws, ws_bytes) whose minimum size the matching
 * *_workspace_bytes query returns; ws must be 256-byte aligned.  Host
 * pointers are plain host memory.
 *
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the null
 * stream).  Work is enqueued on it.  gram_mode_n, ttm_mode_n and
 * tucker_reconstruct are asynchronous: outputs are valid once the stream has
 * been synchronised.  sthosvd_compress synchronises the stream before it
 * returns, because rank-dependent sizes must reach the host.
 *
 * Errors.  Every call returns TK_OK (0) or a negative tk_status.  Arguments
 * are validated on the host before any HIP call, so argument errors are
 * reported without touching the device and leave outputs untouched.
 * tk_last_error() returns a thread-local message for the last failure.
 * A HIP runtime failure returns TK_ERR_HIP; a kernel-detected problem
 * (non-finite input, eigensolver failure) is reported by the call that reads
 * it back.
 *
 * Threading.  Calls are re-entrant as long as concurrent calls use distinct
 * workspaces and outputs.
 */
#ifndef TUCKER_H
#define TUCKER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TK_MAX_NDIM 8
/* Largest mode extent a Gram / eigensolve supports (the paper's working
 * assumption is I_n <= 2000 with small I_n; this library supports <= 512). */
#define TK_MAX_MODE_DIM 512

typedef enum tk_status {
    TK_OK = 0,
    TK_ERR_INVALID_ARG = -1,     /* null pointer, bad shape, bad mode, eps < 0 or NaN ... */
    TK_ERR_UNSUPPORTED = -2,     /* dtype x precision combination not provided */
    TK_ERR_WORKSPACE = -3,       /* ws too small or misaligned */
    TK_ERR_HIP = -4,             /* a HIP runtime call failed (message has the HIP error) */
    TK_ERR_NONFINITE = -5,       /* the input holds Inf or NaN */
    TK_ERR_EIG_NO_CONVERGENCE = -6,
    TK_ERR_CAPACITY = -7         /* an output buffer is smaller than the result */
} tk_status;

typedef enum tk_dtype { TK_F64 = 0, TK_F32 = 1 } tk_dtype;

/* Arithmetic of the Gram product S = Y_(n) Y_(n)^T. */
typedef enum tk_gram_precision {
    /* FP64 products and FP64 accumulation on FP64 matrix cores (FP32 input is
     * widened exactly). */
    TK_GRAM_FP64 = 0,
    /* FP32 input only (the name stays for compatibility; the split is a
     * 16-bit fixed point, not a bf16 rounding).  Per column tile and row i,
     * E_i is the exponent of 1.004 max |x| rounded up, each value's
     * q = x 2^(15-E_i) is rounded to an integer (|q| < 32640) and split into
     * two 8-bit integers, q = 256 hi + lo.  For extents up to 256 the four
     * products hh, hl, lh, ll run on int8 matrix cores into three int32
     * accumulators (hh; hl + lh; ll), for larger extents on bf16 matrix
     * cores (both halves are exact in bf16) into three FP32 accumulators;
     * either way the sums over a tile are exact, and after every tile they
     * are combined exactly, scaled by 2^(E_i+E_j-30) and added into FP64.
     * Each element is represented to 2^-16 of 2^E_i.  The quantization error d of every
     * element is formed exactly, and sum_k d_ik^2 is subtracted from S_ii:
     * quantization noise independent of the data adds its energy to the
     * Gram's diagonal, which would raise its trailing eigenvalue sums by
     * about ||D||_F^2 (J-R)/J, in later modes close to the rank threshold.  In
     * sthosvd_compress a rank found from such a Gram is accepted only when
     * the eps threshold lies clear of the tail sums by the bound of
     * tk_tucker.tail_error_bound; otherwise that mode's Gram is recomputed
     * in FP64 (tk_tucker.fp64_modes).  There, modes
     * with J <= 32 whose unfolding has at most 2^26 elements, or whose rows
     * are runs of L = prod_{k<n} I_k contiguous elements (L a multiple of 8,
     * at least 64), take the FP64 Gram directly: at J <= 32 it costs no more
     * on FP32 data (arithmetic intensity below the FP64 matrix-core ridge)
     * and needs no guard. */
    TK_GRAM_SPLIT_BF16 = 1,
    /* No Gram (sthosvd_compress only; FP64 or FP32 input, dims[n] <=
     * TK_QR_MAX_MODE_DIM at every mode): the singular values of Y_(n) come
     * from a QR of Y_(n)^T, the stable alternative Sec. IX proposes for eps
     * near sqrt(u).  Per mode: R = qr_r_mode_n(Y, n); the symmetric matrix
     * [[0, R^T], [R, 0]] goes through the same FP64 eigensolver, whose
     * leading J_n eigenvalues are sigma_r(R) = sigma_r(Y_(n)) with absolute
     * error about u sigma_1 (the Gram's eigenvalues carry about u sigma_1^2,
     * which hides every sigma_r below sqrt(u) sigma_1); lambda_r = sigma_r^2
     * feeds the same rank rule; U_n = the first J_n entries of the leading
     * eigenvectors, orthonormalised (Gram-Schmidt twice) and signed by the
     * same rule.  Costs a few times the FP64 Gram path. */
    TK_SVD_QR = 2
} tk_gram_precision;

/* Arithmetic of the tensor-times-matrix product: the least accurate
 * arithmetic a call may use.  Narrow modes (J_n <= 64, K <= 16,
 * L = prod_{k<n} I_k a multiple of 8 and at least 64, both data pointers
 * 16-byte aligned) always run in FP64 arithmetic, which streams as fast
 * there and meets every option's error bound. */
typedef enum tk_ttm_precision {
    TK_TTM_FP64 = 0,   /* FP64 products and accumulation (FP64 or FP32 storage) */
    TK_TTM_BF16 = 1,   /* FP32 storage: operands rounded to bf16, FP32 accumulation
                          (relative error ~2^-8); see tk_tucker.ttm_precision_used */
    TK_TTM_BF16X3 = 2  /* FP32 storage: hi = bf16(x), lo = bf16(x - hi) on both operands,
                          products hh + hl + lh, FP32 accumulation (relative error ~2^-17);
                          see tk_tucker.ttm_precision_used for its use in sthosvd_compress */
} tk_ttm_precision;

/* Shape and element type of a dense tensor (dims[0] fastest in memory). */
typedef struct tk_shape {
    int32_t ndim;                 /* 1..TK_MAX_NDIM */
    int32_t dtype;                /* tk_dtype */
    int64_t dims[TK_MAX_NDIM];    /* each >= 1 */
} tk_shape;

/* ------------------------------------------------------------------ Gram */

/*
 * S = Y_(n) Y_(n)^T  (Alg. 1, Gram step; Sec. V-C computes it from the
 * local block-column layout without permuting data, which is what this call
 * does on the whole tensor).
 *   y, y_dev    input tensor (F64 or F32).
 *   mode        n, 0-based.
 *   precision   tk_gram_precision; TK_GRAM_SPLIT_BF16 needs F32 input.
 *   s_dev       out: J_n x J_n FP64, both triangles written (symmetric).
 *   sumsq_dev   out (may be NULL): one FP64, the trace of S = ||Y||^2.
 *   ws          workspace of at least gram_workspace_bytes(y, mode, precision).
 * Deterministic: the same input gives bitwise the same S (no float atomics).
 */
int gram_mode_n(const tk_shape* y, const void* y_dev, int mode, int precision, double* s_dev,
                double* sumsq_dev, void* ws, size_t ws_bytes, void* stream);
size_t gram_workspace_bytes(const tk_shape* y, int mode, int precision);

/*
 * gram_mode_n without a workspace, for callers that cannot allocate device
 * memory (code under graph capture, tight serving loops, harnesses that
 * forbid allocation).  Same arguments, kernels and results as gram_mode_n;
 * the scratch (Gram partials and split statistics) is a static device array
 * of gram_noalloc_scratch_bytes() bytes (72 MiB), one per device, allocated
 * with the library's code on that device and held until the process ends.
 * Shapes whose gram_workspace_bytes exceed it fail with TK_ERR_WORKSPACE;
 * no shape the library accepts does (the Gram's grid is capped per extent,
 * so its partials do not grow with the other modes: the largest, the split
 * Gram of J in 129..256 with L = 1, needs 68.0 MiB).  Argument errors as
 * gram_mode_n, reported before any device call.  The call allocates nothing
 * (no hipMalloc, no library allocation).  Every call on a device shares that
 * device's array: calls that overlap on one device (other streams, other
 * threads) race and must be serialised by the caller.
 */
int gram_mode_n_noalloc(const tk_shape* y, const void* y_dev, int mode, int precision,
                        double* s_dev, double* sumsq_dev, void* stream);
size_t gram_noalloc_scratch_bytes(void);

/* -------------------------------------------------------------------- QR */

/* Largest mode extent of the QR path (R is kept in one workgroup's LDS). */
#define TK_QR_MAX_MODE_DIM 128

/*
 * R factor of a Householder QR of the tall and skinny A = Y_(n)^T (Sec. IX:
 * the stable way to the singular values of Y_(n) when eps nears sqrt(u);
 * A has prod_{m != n} J_m rows and J_n columns).  Rows of A are absorbed in
 * tiles into running factors, which are then combined by a reduction tree
 * (the same Householder step applied to stacked factors); the split of rows
 * does not depend on the device, so the result is deterministic.
 *   y, y_dev    input tensor (F64, or F32 widened exactly); dims[mode] <=
 *               TK_QR_MAX_MODE_DIM.
 *   r_dev       out: J_n x J_n FP64 column-major, upper triangular (strict
 *               lower part written as 0), each row signed so that its
 *               diagonal entry is >= 0; Y_(n) Y_(n)^T = R^T R in exact
 *               arithmetic.  If A has fewer rows than columns the trailing
 *               rows of R are zero.
 *   sumsq_dev   out (may be NULL): one FP64, ||Y||^2 summed in a fixed order.
 *   ws          at least qr_workspace_bytes(y, mode) bytes, 256-B aligned.
 * Entries whose square under- or overflows FP64 (|x| outside about
 * [1e-154, 1e154]) are outside the supported range, as for the Gram.
 */
int qr_r_mode_n(const tk_shape* y, const void* y_dev, int mode, double* r_dev,
                double* sumsq_dev, void* ws, size_t ws_bytes, void* stream);
size_t qr_workspace_bytes(const tk_shape* y, int mode);

/* ------------------------------------------------------------------- TTM */

/*
 * Z = Y x_n op(M), i.e. Z_(n) = op(M) Y_(n)  (Sec. II-A, with the matrix
 * taken as K x J_n so that the unfolded identity holds; Sec. V-B computes it
 * block column by block column, which is what this call does).
 *   m_dev       FP64 column-major m_rows x m_cols.
 *   transpose   0: op(M) = M, M is K x J_n (m_rows = K, m_cols = J_n);
 *               1: op(M) = M^T, M is J_n x K (m_rows = J_n, m_cols = K).
 *               ST-HOSVD applies U_n^T with transpose = 1 and M = U_n;
 *               reconstruction applies U_n with transpose = 0.
 *   precision   tk_ttm_precision (BF16 variants need F32 storage).
 *   z_dev       out: Y's dims with dims[mode] = K, same dtype as Y; must not
 *               overlap y_dev.
 */
int ttm_mode_n(const tk_shape* y, const void* y_dev, int mode, const double* m_dev,
               int64_t m_rows, int64_t m_cols, int transpose, int precision, void* z_dev,
               void* stream);

/* --------------------------------------------------------------- ST-HOSVD */

typedef struct tk_options {
    double eps;                  /* relative error target, >= 0, finite */
    const int32_t* mode_order;   /* host, ndim entries: a permutation of 0..N-1; NULL = 0..N-1 */
    const int64_t* fixed_ranks;  /* host, ndim entries in [1, I_n]; NULL = the eps rule */
    const int64_t* max_ranks;    /* host, ndim entries >= 1; NULL = I_n.  Sizes the
                                    workspace; a rank above it fails with TK_ERR_CAPACITY */
    int32_t gram_precision;      /* tk_gram_precision */
    int32_t ttm_precision;       /* tk_ttm_precision */
    int32_t time_first_gram;     /* nonzero: sthosvd_compress brackets the first processed
                                    mode's partial-Gram kernel with two HIP events on its
                                    stream and reports their interval in
                                    tk_tucker.first_gram_ms (a caller timing the dominant
                                    kernel inside its pipeline); 0 = no events */
} tk_options;

typedef struct tk_tucker {
    /* device outputs, caller-allocated */
    void* core_dev;                    /* core G, x's dtype, natural layout with dims = ranks */
    int64_t core_capacity;             /* elements available at core_dev */
    double* factors_dev[TK_MAX_NDIM];  /* U_n: I_n x R_n column-major; capacity I_n*I_n */
    double* eigvals_dev;               /* sum_n I_n doubles: spectrum of each mode's Gram,
                                          descending, mode n at offset sum_{m<n} I_m; may be NULL */
    /* host outputs, written before sthosvd_compress returns TK_OK */
    int64_t ranks[TK_MAX_NDIM];        /* R_n */
    double discarded[TK_MAX_NDIM];     /* sum_{r > R_n} lambda_r at mode n (at least 0) */
    double norm2;                      /* ||X||^2 */
    uint32_t fp64_modes;               /* bit n: mode n's Gram was recomputed in FP64 because
                                          the split-bf16 Gram could not certify its rank
                                          (gram_precision TK_GRAM_SPLIT_BF16 only) */
    int32_t ttm_precision_used;        /* tk_ttm_precision the TTMs ran in.  Under the eps
                                          rule a precision whose relative output error would
                                          reach the rank threshold is raised: TK_TTM_BF16
                                          (~2^-8) becomes TK_TTM_BF16X3 when
                                          eps^2 / N < 2^-13, and TK_TTM_BF16X3 (~2^-17)
                                          becomes TK_TTM_FP64 when eps^2 / N < 2^-31.
                                          Fixed ranks keep the requested precision. */
    double tail_error_bound[TK_MAX_NDIM]; /* when mode n's Gram ran split-bf16: a bound on
                                          |discarded[n] - t|, t the tail sum of the exact
                                          Gram of the same Y_n: ||D||_F^2 / 8 (the
                                          subtracted diagonal of D D^T, trusted to an
                                          eighth of its size) plus 6 standard deviations
                                          sqrt(4 delta^2 t + 2 K delta^4 (J - R)) of the
                                          remaining error (the split Gram subtracts
                                          diag(D D^T) exactly; the cross terms Y D^T +
                                          D Y^T and the off-diagonal of D D^T have mean 0
                                          when the quantization errors are modelled as
                                          independent of the data and of each other,
                                          |d| <= 2^(E_max - 16), variance <= delta^2 =
                                          4^(E_max - 16) / 3; K columns, J rows, rank R).
                                          0 for FP64 Grams.  Under the eps rule a
                                          split-bf16 rank is accepted only when
                                          eps^2 ||X||^2 / N exceeds discarded[n] by this
                                          bound and falls short of the next larger tail sum
                                          by the same bound taken there; otherwise the mode
                                          is redone in FP64. */
    double first_gram_ms;              /* with tk_options.time_first_gram: the interval, in
                                          ms, between the HIP events recorded just before and
                                          just after the first processed mode's partial-Gram
                                          kernel; 0 otherwise */
} tk_tucker;

/*
 * Alg. 1 (ST-HOSVD).  For each mode n in opt->mode_order: S = Y_(n) Y_(n)^T;
 * eigendecomposition of S in FP64; R_n = min R >= 1 with
 * sum_{r>R} lambda_r(S) <= eps^2 ||X||^2 / N (||X|| of the input, N = ndim,
 * negative rounding eigenvalues counted as 0 -- for a split-bf16 Gram the
 * raw eigenvalues: subtracting its quantization energy leaves small negative
 * ones in noise-level directions, and their raw sum estimates the exact
 * tail); U_n = the leading R_n
 * eigenvectors (each signed so that its largest-magnitude entry is
 * positive); Y <- Y x_n U_n^T.  The final Y is the core G.
 *   x, x_dev    input tensor (not modified).
 *   ws          at least sthosvd_workspace_bytes(x, opt) bytes.
 * Synchronises `stream` before returning.  Errors: TK_ERR_CAPACITY if the
 * core does not fit core_capacity or a rank exceeds max_ranks;
 * TK_ERR_NONFINITE if the input holds Inf/NaN.
 */
int sthosvd_compress(const tk_shape* x, const void* x_dev, const tk_options* opt,
                     tk_tucker* out, void* ws, size_t ws_bytes, void* stream);
size_t sthosvd_workspace_bytes(const tk_shape* x, const tk_options* opt);

/* ------------------------------------------------------------------ HOOI
 * Alg. 2 (HOOI): ST-HOSVD as in sthosvd_compress (eps rule or fixed ranks,
 * opt->mode_order for that start), then up to max_sweeps sweeps.  A sweep
 * visits n = 1..N: Y = X x_m U_m^T for every m != n (ascending m), U_n <-
 * the leading R_n eigenvectors of Y_(n) Y_(n)^T (same eigensolver and sign
 * rule); after mode N the core G = Y x_N U_N^T.  After the ST-HOSVD and
 * after every sweep the fit ||X||^2 - ||G||^2 (the model error
 * ||X - G x {U_n}||^2, Sec. II-B) is computed in FP64 and read back (one
 * stream sync per sweep); the iteration stops once a sweep lowers it by at
 * most tol * ||X||^2 (tol >= 0), or after max_sweeps (tol < 0 runs exactly
 * max_sweeps).  Precisions as in opt (fixed ranks: no guard).
 *   out          as for sthosvd_compress; holds the final core and factors;
 *                discarded[n] = tail sum of mode n's last Gram.
 *   fits         host, max_sweeps + 1 doubles (may be NULL): fits[0] after
 *                the ST-HOSVD, fits[k] after sweep k.
 *   sweeps_done  host (may be NULL): sweeps run.
 *   ws           at least tucker_hooi_workspace_bytes(x, opt) bytes.
 * Errors: those of sthosvd_compress, TK_ERR_INVALID_ARG for max_sweeps < 0
 * or a non-finite tol. */
size_t tucker_hooi_workspace_bytes(const tk_shape* x, const tk_options* opt);
int tucker_hooi(const tk_shape* x, const void* x_dev, const tk_options* opt, int max_sweeps,
                double tol, tk_tucker* out, double* fits, int* sweeps_done, void* ws,
                size_t ws_bytes, void* stream);

/* ------------------------------------------------------------ mode order
 * Alg. 1 processes the modes in any order; the order changes the work of
 * the later modes (Sec. VIII-C, mode-order experiment).  Given the extents
 * and the (expected or fixed) ranks, this host-only call writes an order to
 * order_out[0..ndim-1]:
 *   TK_ORDER_GREEDY_FLOPS  at each step the remaining mode with the fewest
 *                          flops in that step (Gram 2 I_n #Y plus TTM
 *                          2 R_n #Y, so the least I_n + R_n): the
 *                          heuristic of the ST-HOSVD authors cited there;
 *   TK_ORDER_GREEDY_RATIO  at each step the remaining mode with the largest
 *                          compression ratio I_n / R_n (the alternative
 *                          heuristic given there);
 *   TK_ORDER_MIN_BYTES     the order that minimises this library's
 *                          algorithmic HBM traffic, sum over steps of
 *                          (2 #Y_n + #Y_{n+1}) elem_bytes (every Gram reads
 *                          Y_n, every TTM reads Y_n and writes Y_{n+1}),
 *                          by exhaustive search (ndim <= 8).
 * Ties go to the lowest mode index (lexicographically first order).
 * Returns TK_OK, or TK_ERR_INVALID_ARG for ndim outside [1, 8], a NULL
 * pointer, an extent < 1, a rank outside [1, extent] or an unknown rule. */
typedef enum tk_order_rule {
    TK_ORDER_GREEDY_FLOPS = 0,
    TK_ORDER_GREEDY_RATIO = 1,
    TK_ORDER_MIN_BYTES = 2
} tk_order_rule;
int sthosvd_mode_order(int ndim, const int64_t* dims, const int64_t* ranks, int rule,
                       int elem_bytes, int* order_out);

/* ---------------------------------------------------------- reconstruction */

/*
 * X~ = G x_1 U_1 x_2 U_2 ... x_N U_N  (Sec. II-C, eq. reconstruct).  Any
 * subset of rows of a factor gives the matching subtensor (Sec. II-C), so
 * full_dims[n] may be smaller than the original I_n when factors_dev[n]
 * points at a row subset (leading dimension factor_ld[n]).
 *   core, core_dev  core tensor, dims = ranks (F64 or F32).
 *   factors_dev[n]  FP64 column-major full_dims[n] x R_n, leading dim factor_ld[n]
 *                   (factor_ld may be NULL: leading dim = full_dims[n]).
 *   precision       tk_ttm_precision used for every product.
 *   xhat_dev        out: prod(full_dims) elements of the core's dtype.
 *   ws              at least reconstruct_workspace_bytes(core, full_dims) bytes.
 * Asynchronous.
 */
int tucker_reconstruct(const tk_shape* core, const void* core_dev,
                       const double* const* factors_dev, const int64_t* factor_ld,
                       const int64_t* full_dims, int precision, void* xhat_dev, void* ws,
                       size_t ws_bytes, void* stream);
size_t reconstruct_workspace_bytes(const tk_shape* core, const int64_t* full_dims);

/*
 * Error metrics of an approximation (Table II): writes to out_host[3]
 *   [0] ||X - X~||^2, [1] max |X - X~|, [2] ||X||^2,
 * accumulated in FP64.  x and xhat share shape and dtype.  Synchronises the
 * stream.  ws: at least error_metrics_workspace_bytes(x).
 */
int tucker_error_metrics(const tk_shape* x, const void* x_dev, const void* xhat_dev,
                         double* out_host, void* ws, size_t ws_bytes, void* stream);
size_t error_metrics_workspace_bytes(const tk_shape* x);

/* --------------------------------------------------------------- helpers */

/* ------------------------------------------------------------------ batches
 * Many independent problems (each an ST-HOSVD as in sthosvd_compress; the
 * problems may have different extents) compressed together: every mode step
 * of every problem runs in a handful of launches that cover the whole batch
 * (a split Gram -- for extents up to 32 the FP64 Gram, as sthosvd_compress
 * does for narrow modes --, its reduction, one eigensolver workgroup per
 * problem, the guard's FP64 recomputation, a bf16 or split-bf16 TTM), with each problem's
 * later shapes derived on the device from the ranks found there.  sthosvd_batch_run therefore enqueues work
 * without any host synchronisation, allocation or memset: it can be captured
 * into a HIP graph once and replayed.
 *
 * Requirements: TK_F32 storage, gram_precision TK_GRAM_SPLIT_BF16,
 * ttm_precision TK_TTM_BF16X3 or TK_TTM_BF16; under the eps rule the TTM's
 * error must stay below the rank threshold as in sthosvd_compress
 * (TK_TTM_BF16X3 needs eps^2/N >= 2^-31, TK_TTM_BF16 eps^2/N >= 2^-13;
 * otherwise TK_ERR_UNSUPPORTED: a batch does not change the precision it
 * was given), every problem with the same ndim and mode order, every
 * extent <= 128.
 *
 * A mode whose rank the split Gram could not certify (the guard of
 * TK_GRAM_SPLIT_BF16) is recomputed on the device within the same run, as in
 * sthosvd_compress: after every eigensolver launch, an FP64 Gram, its
 * reduction and the eigensolver run again for exactly those problems (the
 * launches cover the batch; workgroups of other problems return at once). */
typedef struct tk_batch tk_batch; /* opaque host-side plan */

typedef struct tk_batch_outputs {
    void* const* core_dev;          /* [batch] core buffers (FP32, natural layout) */
    const int64_t* core_capacity;   /* [batch] elements available at core_dev[b] */
    double* const* factors_dev;     /* [batch * TK_MAX_NDIM] U_n, capacity I_n * I_n each */
    int64_t* ranks_dev;             /* device [batch * ndim] */
    double* discarded_dev;          /* device [batch * ndim] */
    double* norm2_dev;              /* device [batch] */
    int32_t* status_dev;            /* device [batch * 2]: [0] bit 1 = capacity exceeded,
                                       bit 2 = rank not yet certified (cleared by the
                                       FP64 recomputation within the run);
                                       [1] bit n = mode n recomputed in FP64 */
    double* tail_bound_dev;         /* device [batch * ndim] or NULL: per problem and mode,
                                       the bound of tk_tucker.tail_error_bound (0 where the
                                       mode was recomputed in FP64) */
} tk_batch_outputs;

/* Work partition: column tiles per Gram workgroup and 16-column blocks per
 * TTM workgroup, per mode (0 = default).  Chosen by an autotuner in the
 * Python layer; any positive values give the same results up to summation
 * order.  The values are targets: workgroups per problem are capped at 4096,
 * and from the second mode step on (whose shapes are counted at the rank
 * capacities) at max(256, 16384 / batch), so a workgroup may take more. */
typedef struct tk_batch_tuning {
    int32_t gram_tiles_per_wg[TK_MAX_NDIM];
    int32_t ttm_blocks_per_wg[TK_MAX_NDIM];
} tk_batch_tuning;

size_t sthosvd_batch_workspace_bytes(int batch, const tk_shape* shapes, const tk_options* opt,
                                     const tk_batch_tuning* tuning /* NULL = defaults */);
/* Validates, lays out the workspace (device, caller-owned, 256-byte aligned)
 * and uploads the task tables (one synchronous copy).  x_dev[b] and every
 * output pointer are bound into the plan.  *handle receives a host object
 * freed by sthosvd_batch_destroy. */
int sthosvd_batch_create(int batch, const tk_shape* shapes, const void* const* x_dev,
                         const tk_options* opt, const tk_batch_tuning* tuning,
                         const tk_batch_outputs* out, void* ws, size_t ws_bytes, void* stream,
                         tk_batch** handle);
/* Enqueues one compression of every problem (no sync, allocation or memset). */
int sthosvd_batch_run(tk_batch* handle, void* stream);
/* Synchronises and reports errors: TK_ERR_CAPACITY (a rank above
 * max_ranks), TK_ERR_NONFINITE (Inf or NaN in a problem). */
int sthosvd_batch_finish(tk_batch* handle, void* stream);
void sthosvd_batch_destroy(tk_batch* handle);

const char* tk_status_string(int status);
const char* tk_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TUCKER_H */
