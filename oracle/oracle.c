/*
 * oracle.c -- plain, slow, FP64 CPU reference for sequentially truncated
 * HOSVD (ST-HOSVD) and Tucker reconstruction.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the package smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no code, header, table or
 * helper with the GPU library.
 *
 * Every routine follows the paper's definitions literally, in its notation,
 * with no blocking or fusion:
 *
 *   - tensor layout: element (i_1..i_N) sits at offset sum_k i_k prod_{m<k} I_m,
 *     i.e. the mode-1 unfolding is column-major (Sec. IV-A);
 *   - mode-n unfolding X_(n): element (i_1..i_N) -> (i_n, j) with
 *     j = sum_{k != n} i_k prod_{m<k, m != n} I_m  (Sec. II-A; the printed
 *     formula has a garbled hat/bar, the prefix-product reading is the one the
 *     unfolding figure of Sec. IV-C shows);
 *   - TTM Y = X x_n V  <=>  Y_(n) = V X_(n), with V of size K x I_n (Sec. II-A);
 *   - Gram S = Y_(n) Y_(n)^T (Alg. 1, Gram step);
 *   - symmetric eigendecomposition by cyclic two-sided Jacobi rotations
 *     (textbook method; the paper uses a LAPACK subset solver, Sec. V-D);
 *   - rank rule: smallest R with sum_{r>R} lambda_r <= eps^2 ||X||^2 / N
 *     (Alg. 1, rank step), with ||X|| the norm of the ORIGINAL tensor;
 *   - factor U_n = leading R_n eigenvectors; Y <- Y x_n U_n^T (Alg. 1);
 *   - reconstruction X~ = G x {U_n} (Sec. II-C, eq. reconstruct);
 *   - the QR-preprocessed alternative of Sec. IX for eps near sqrt(u): the R
 *     factor of a Householder QR of Y_(n)^T, then an SVD of R by one-sided
 *     Jacobi; the left singular vectors of Y_(n) are R's right singular
 *     vectors and lambda_r = sigma_r^2.
 *
 * Matrices in this file are dense row-major arrays (A[r*cols + c]).
 * All sums of long products use pairwise (recursive halving) summation.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2
#define ORC_ENOCONV -3

#define ORC_MAX_NDIM 16

/* ------------------------------------------------------------------ sums */

/* Pairwise sum of a[k]*b[k*stride_b] products, k < n. */
static double pw_dot(const double* a, const double* b, int64_t n) {
    if (n <= 16) {
        double s = 0.0;
        for (int64_t k = 0; k < n; ++k) s += a[k] * b[k];
        return s;
    }
    int64_t h = n / 2;
    return pw_dot(a, b, h) + pw_dot(a + h, b + h, n - h);
}

static double pw_sumsq(const double* a, int64_t n) {
    if (n <= 16) {
        double s = 0.0;
        for (int64_t k = 0; k < n; ++k) s += a[k] * a[k];
        return s;
    }
    int64_t h = n / 2;
    return pw_sumsq(a, h) + pw_sumsq(a + h, n - h);
}

static int64_t prod_dims(int ndim, const int64_t* dims) {
    int64_t p = 1;
    for (int k = 0; k < ndim; ++k) p *= dims[k];
    return p;
}

static int check_shape(int ndim, const int64_t* dims) {
    if (ndim < 1 || ndim > ORC_MAX_NDIM || !dims) return ORC_EINVAL;
    for (int k = 0; k < ndim; ++k)
        if (dims[k] < 1) return ORC_EINVAL;
    return ORC_OK;
}

/* Norm squared of the tensor: sum of squares of all entries (Sec. II-A). */
double orc_norm2(const double* x, int64_t count) { return pw_sumsq(x, count); }

/* ------------------------------------------------------------- unfolding */

/*
 * Mode-n unfolding (Sec. II-A, n is 0-based here): visit every multi-index
 * with an odometer, compute its memory offset from the layout definition
 * and its unfolded column j from the prefix-product formula.
 * m is J_n x (J/J_n), row-major.
 */
int orc_unfold(const double* x, int ndim, const int64_t* dims, int n, double* m) {
    if (check_shape(ndim, dims) || n < 0 || n >= ndim || !x || !m) return ORC_EINVAL;
    int64_t total = prod_dims(ndim, dims);
    int64_t cols = total / dims[n];
    int64_t idx[ORC_MAX_NDIM] = {0};
    for (int64_t off = 0; off < total; ++off) {
        /* off enumerates elements in memory order, so idx is its multi-index */
        int64_t j = 0, mult = 1;
        for (int k = 0; k < ndim; ++k) {
            if (k == n) continue;
            j += idx[k] * mult;
            mult *= dims[k];
        }
        m[idx[n] * cols + j] = x[off];
        for (int k = 0; k < ndim; ++k) { /* advance odometer, mode 1 fastest */
            if (++idx[k] < dims[k]) break;
            idx[k] = 0;
        }
    }
    return ORC_OK;
}

/* Inverse of orc_unfold: write the J_n x (J/J_n) matrix back into a tensor. */
int orc_fold(const double* m, int ndim, const int64_t* dims, int n, double* x) {
    if (check_shape(ndim, dims) || n < 0 || n >= ndim || !x || !m) return ORC_EINVAL;
    int64_t total = prod_dims(ndim, dims);
    int64_t cols = total / dims[n];
    int64_t idx[ORC_MAX_NDIM] = {0};
    for (int64_t off = 0; off < total; ++off) {
        int64_t j = 0, mult = 1;
        for (int k = 0; k < ndim; ++k) {
            if (k == n) continue;
            j += idx[k] * mult;
            mult *= dims[k];
        }
        x[off] = m[idx[n] * cols + j];
        for (int k = 0; k < ndim; ++k) {
            if (++idx[k] < dims[k]) break;
            idx[k] = 0;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------- TTM */

/*
 * Z = Y x_n V with V of size K x J_n (row-major), via the unfolded identity
 * Z_(n) = V Y_(n) (Sec. II-A).  Z has Y's dims with dims[n] replaced by K.
 */
int orc_ttm(const double* y, int ndim, const int64_t* dims, int n, const double* v,
            int64_t k_rows, double* z) {
    if (check_shape(ndim, dims) || n < 0 || n >= ndim || k_rows < 1 || !y || !v || !z)
        return ORC_EINVAL;
    int64_t jn = dims[n];
    int64_t cols = prod_dims(ndim, dims) / jn;
    double* my = (double*)malloc(sizeof(double) * jn * cols);
    double* mz = (double*)malloc(sizeof(double) * k_rows * cols);
    double* col = (double*)malloc(sizeof(double) * jn);
    if (!my || !mz || !col) { free(my); free(mz); free(col); return ORC_ENOMEM; }
    orc_unfold(y, ndim, dims, n, my);
    for (int64_t c = 0; c < cols; ++c) {
        for (int64_t i = 0; i < jn; ++i) col[i] = my[i * cols + c];
        for (int64_t r = 0; r < k_rows; ++r) mz[r * cols + c] = pw_dot(v + r * jn, col, jn);
    }
    int64_t zdims[ORC_MAX_NDIM];
    memcpy(zdims, dims, sizeof(int64_t) * ndim);
    zdims[n] = k_rows;
    orc_fold(mz, ndim, zdims, n, z);
    free(my); free(mz); free(col);
    return ORC_OK;
}

/* ------------------------------------------------------------------ Gram */

/* S = M M^T for a row-major J x K matrix M; S is J x J row-major, symmetric. */
int orc_gram_matrix(const double* m, int64_t j, int64_t k, double* s) {
    if (!m || !s || j < 1 || k < 1) return ORC_EINVAL;
    for (int64_t a = 0; a < j; ++a)
        for (int64_t b = a; b < j; ++b) {
            double v = pw_dot(m + a * k, m + b * k, k);
            s[a * j + b] = v;
            s[b * j + a] = v;
        }
    return ORC_OK;
}

/* S = Y_(n) Y_(n)^T (Alg. 1, Gram step) from an explicit unfolding. */
int orc_gram(const double* y, int ndim, const int64_t* dims, int n, double* s) {
    if (check_shape(ndim, dims) || n < 0 || n >= ndim || !y || !s) return ORC_EINVAL;
    int64_t jn = dims[n];
    int64_t cols = prod_dims(ndim, dims) / jn;
    double* m = (double*)malloc(sizeof(double) * jn * cols);
    if (!m) return ORC_ENOMEM;
    orc_unfold(y, ndim, dims, n, m);
    int rc = orc_gram_matrix(m, jn, cols, s);
    free(m);
    return rc;
}

/*
 * One Gram entry S[a][b] = sum over all multi-indices with i_n free of
 * y(..a..) * y(..b..), visiting the multi-indices directly (for spot checks
 * on tensors too large to unfold).  Sequential summation in FP64.
 */
double orc_gram_entry(const double* y, int ndim, const int64_t* dims, int n, int64_t a,
                      int64_t b) {
    int64_t stride_n = 1;
    for (int k = 0; k < n; ++k) stride_n *= dims[k];
    int64_t total = prod_dims(ndim, dims);
    double s = 0.0;
    int64_t idx[ORC_MAX_NDIM] = {0};
    for (int64_t off = 0; off < total; ++off) {
        if (idx[n] == 0) {
            s += y[off + a * stride_n] * y[off + b * stride_n];
        }
        for (int k = 0; k < ndim; ++k) {
            if (++idx[k] < dims[k]) break;
            idx[k] = 0;
        }
    }
    return s;
}

/* One TTM output entry: (Y x_n V)(i_1..K_r..i_N) = sum_i V[r][i] Y(..i..). */
double orc_ttm_entry(const double* y, int ndim, const int64_t* dims, int n, const double* v,
                     const int64_t* out_idx) {
    int64_t off = 0, mult = 1, stride_n = 1;
    for (int k = 0; k < ndim; ++k) {
        if (k == n) stride_n = mult;
        else off += out_idx[k] * mult;
        mult *= dims[k];
    }
    int64_t r = out_idx[n];
    double s = 0.0;
    for (int64_t i = 0; i < dims[n]; ++i) s += v[r * dims[n] + i] * y[off + i * stride_n];
    return s;
}

/* ------------------------------------------------------- Jacobi eigensolver */

/*
 * Cyclic-by-row two-sided Jacobi for a symmetric J x J matrix (textbook
 * method, e.g. Golub & Van Loan, "symmetric Schur decomposition").  On exit
 * lam holds the eigenvalues sorted descending (ties kept in index order) and
 * vecs (row-major, J x J) the matching eigenvectors in its columns.  Each
 * eigenvector is signed so that its largest-magnitude entry (lowest index on
 * ties) is positive.  The matrix s is overwritten.  Returns the number of
 * sweeps used, or ORC_ENOCONV after max_sweeps.
 *
 * Rotation rule: annihilate s[p][q] when |s[p][q]| > tol * sqrt(|s[p][p] s[q][q]|)
 * (relative threshold) and |s[p][q]| > 1e-17 ||S||_F; stop after a sweep that
 * applies no rotation.
 */
int orc_sym_eig(double* s, int64_t j, double* lam, double* vecs, int max_sweeps) {
    if (!s || !lam || !vecs || j < 1) return ORC_EINVAL;
    const double tol = 1e-15;
    /* absolute floor: entries below 1e-17 ||S||_F change no eigenvalue by more
       than FP64 rounding already does, so they are left alone */
    double frob2 = 0.0;
    for (int64_t a = 0; a < j * j; ++a) frob2 += s[a] * s[a];
    const double floor_abs = 1e-17 * sqrt(frob2);
    for (int64_t a = 0; a < j; ++a)
        for (int64_t b = 0; b < j; ++b) vecs[a * j + b] = (a == b) ? 1.0 : 0.0;
    int sweep = 0, converged = 0;
    for (sweep = 1; sweep <= max_sweeps; ++sweep) {
        int rotated = 0;
        for (int64_t p = 0; p < j - 1; ++p) {
            for (int64_t q = p + 1; q < j; ++q) {
                double apq = s[p * j + q];
                double app = s[p * j + p], aqq = s[q * j + q];
                if (fabs(apq) <= floor_abs) continue;
                if (fabs(apq) <= tol * sqrt(fabs(app * aqq))) continue;
                rotated = 1;
                /* choose t = tan(theta) of smaller magnitude root of
                   t^2 + 2 t zeta - 1 = 0, zeta = (aqq - app) / (2 apq) */
                double zeta = (aqq - app) / (2.0 * apq);
                double t;
                if (fabs(zeta) > 1e150) t = 0.5 / zeta;
                else t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double c = 1.0 / sqrt(1.0 + t * t);
                double sn = t * c;
                /* S <- G^T S G with G the rotation in plane (p, q) */
                for (int64_t r = 0; r < j; ++r) { /* columns p, q */
                    double srp = s[r * j + p], srq = s[r * j + q];
                    s[r * j + p] = c * srp - sn * srq;
                    s[r * j + q] = sn * srp + c * srq;
                }
                for (int64_t r = 0; r < j; ++r) { /* rows p, q */
                    double spr = s[p * j + r], sqr = s[q * j + r];
                    s[p * j + r] = c * spr - sn * sqr;
                    s[q * j + r] = sn * spr + c * sqr;
                }
                s[p * j + q] = 0.0;
                s[q * j + p] = 0.0;
                for (int64_t r = 0; r < j; ++r) { /* V <- V G */
                    double vrp = vecs[r * j + p], vrq = vecs[r * j + q];
                    vecs[r * j + p] = c * vrp - sn * vrq;
                    vecs[r * j + q] = sn * vrp + c * vrq;
                }
            }
        }
        if (!rotated) { converged = 1; break; }
    }
    /* sort descending, stable on index (insertion sort over a permutation) */
    int64_t* perm = (int64_t*)malloc(sizeof(int64_t) * j);
    double* tmp = (double*)malloc(sizeof(double) * j * j);
    if (!perm || !tmp) { free(perm); free(tmp); return ORC_ENOMEM; }
    for (int64_t a = 0; a < j; ++a) perm[a] = a;
    for (int64_t a = 1; a < j; ++a) {
        int64_t cur = perm[a];
        int64_t b = a - 1;
        while (b >= 0 && s[perm[b] * j + perm[b]] < s[cur * j + cur]) {
            perm[b + 1] = perm[b];
            --b;
        }
        perm[b + 1] = cur;
    }
    for (int64_t a = 0; a < j; ++a) lam[a] = s[perm[a] * j + perm[a]];
    for (int64_t r = 0; r < j; ++r)
        for (int64_t a = 0; a < j; ++a) tmp[r * j + a] = vecs[r * j + perm[a]];
    /* sign rule: largest |entry| positive, lowest index on ties */
    for (int64_t a = 0; a < j; ++a) {
        int64_t best = 0;
        for (int64_t r = 1; r < j; ++r)
            if (fabs(tmp[r * j + a]) > fabs(tmp[best * j + a])) best = r;
        if (tmp[best * j + a] < 0)
            for (int64_t r = 0; r < j; ++r) tmp[r * j + a] = -tmp[r * j + a];
    }
    memcpy(vecs, tmp, sizeof(double) * j * j);
    free(perm); free(tmp);
    return converged ? sweep : ORC_ENOCONV;
}

/* ------------------------------------------------------------ truncation */

/*
 * Rank rule of Alg. 1: R = min R in [1, J] with sum_{r>R} max(lambda_r, 0) <= tau.
 * lam is sorted descending.  Tail sums accumulate from the smallest
 * eigenvalue upward.  fixed_rank > 0 overrides the rule.  Writes the tail sum
 * t_R (the discarded eigenvalue mass) to *discarded.
 */
int orc_truncate(const double* lam, int64_t j, double tau, int64_t fixed_rank,
                 int64_t* rank, double* discarded) {
    if (!lam || !rank || !discarded || j < 1 || fixed_rank > j) return ORC_EINVAL;
    double* tail = (double*)malloc(sizeof(double) * (j + 1)); /* tail[R] = sum_{r>R} */
    if (!tail) return ORC_ENOMEM;
    tail[j] = 0.0;
    for (int64_t r = j - 1; r >= 0; --r) tail[r] = tail[r + 1] + (lam[r] > 0 ? lam[r] : 0.0);
    int64_t R = j;
    if (fixed_rank > 0) {
        R = fixed_rank;
    } else {
        for (int64_t c = 1; c <= j; ++c)
            if (tail[c] <= tau) { R = c; break; }
    }
    *rank = R;
    *discarded = tail[R];
    free(tail);
    return ORC_OK;
}

/* --------------------------------------------------------------- ST-HOSVD */

/*
 * Alg. 1 (ST-HOSVD).  Inputs: tensor x (ndim, dims), eps, optional mode
 * order (0-based permutation; NULL = 0..N-1), optional fixed ranks (NULL =
 * rank rule).  Outputs (caller-allocated):
 *   core      capacity prod(dims) doubles; holds G in the same layout;
 *   ranks     ndim;
 *   factors   ndim blocks of dims[n]*dims[n] doubles; block n holds U_n as a
 *             row-major dims[n] x ranks[n] matrix;
 *   eigvals   sum(dims) doubles; the spectrum of mode n starts at
 *             sum_{m<n} dims[m] and is sorted descending;
 *   discarded ndim; the tail sum dropped at each mode;
 *   norm2     ||X||^2;
 *   sweeps    ndim; Jacobi sweeps per mode.
 */
int orc_sthosvd(const double* x, int ndim, const int64_t* dims, double eps, const int* order,
                const int64_t* fixed_ranks, double* core, int64_t* ranks, double* factors,
                double* eigvals, double* discarded, double* norm2, int* sweeps) {
    if (check_shape(ndim, dims) || !x || !core || !ranks || !factors || !eigvals ||
        !discarded || !norm2 || !sweeps || !(eps >= 0))
        return ORC_EINVAL;
    int ord[ORC_MAX_NDIM];
    int seen[ORC_MAX_NDIM] = {0};
    for (int k = 0; k < ndim; ++k) {
        ord[k] = order ? order[k] : k;
        if (ord[k] < 0 || ord[k] >= ndim || seen[ord[k]]) return ORC_EINVAL;
        seen[ord[k]] = 1;
    }
    int64_t total = prod_dims(ndim, dims);
    double nrm2 = orc_norm2(x, total);
    *norm2 = nrm2;
    double tau = eps * eps * nrm2 / (double)ndim;

    int64_t jd[ORC_MAX_NDIM];
    memcpy(jd, dims, sizeof(int64_t) * ndim);
    double* y = (double*)malloc(sizeof(double) * total);
    double* ynext = (double*)malloc(sizeof(double) * total);
    if (!y || !ynext) { free(y); free(ynext); return ORC_ENOMEM; }
    memcpy(y, x, sizeof(double) * total);

    int64_t fac_off[ORC_MAX_NDIM], eig_off[ORC_MAX_NDIM];
    int64_t fo = 0, eo = 0;
    for (int k = 0; k < ndim; ++k) {
        fac_off[k] = fo; fo += dims[k] * dims[k];
        eig_off[k] = eo; eo += dims[k];
    }
    int rc = ORC_OK;
    for (int step = 0; step < ndim; ++step) {
        int n = ord[step];
        int64_t jn = jd[n];
        double* s = (double*)malloc(sizeof(double) * jn * jn);
        double* v = (double*)malloc(sizeof(double) * jn * jn);
        double* ut = NULL;
        if (!s || !v) { free(s); free(v); rc = ORC_ENOMEM; break; }
        orc_gram(y, ndim, jd, n, s);
        int sw = orc_sym_eig(s, jn, eigvals + eig_off[n], v, 50);
        sweeps[n] = sw;
        if (sw < 0) { free(s); free(v); rc = sw; break; }
        int64_t R;
        rc = orc_truncate(eigvals + eig_off[n], jn, tau, fixed_ranks ? fixed_ranks[n] : 0, &R,
                          &discarded[n]);
        if (rc) { free(s); free(v); break; }
        ranks[n] = R;
        double* u = factors + fac_off[n];
        for (int64_t i = 0; i < jn; ++i)
            for (int64_t r = 0; r < R; ++r) u[i * R + r] = v[i * jn + r];
        /* Y <- Y x_n U_n^T, with U_n^T (R x J_n) row-major */
        ut = (double*)malloc(sizeof(double) * R * jn);
        if (!ut) { free(s); free(v); rc = ORC_ENOMEM; break; }
        for (int64_t r = 0; r < R; ++r)
            for (int64_t i = 0; i < jn; ++i) ut[r * jn + i] = u[i * R + r];
        orc_ttm(y, ndim, jd, n, ut, R, ynext);
        jd[n] = R;
        double* t = y; y = ynext; ynext = t;
        free(s); free(v); free(ut);
    }
    if (rc == ORC_OK) memcpy(core, y, sizeof(double) * prod_dims(ndim, jd));
    free(y); free(ynext);
    return rc;
}

/*
 * Reconstruction X~ = G x_1 U_1 ... x_N U_N (Sec. II-C).  core has dims
 * ranks[]; factors holds N row-major matrices, U_n of size full[n] x ranks[n],
 * packed back to back.  out has prod(full) doubles.
 */
int orc_reconstruct(const double* core, int ndim, const int64_t* ranks,
                    const double* factors, const int64_t* full, double* out) {
    if (check_shape(ndim, ranks) || check_shape(ndim, full) || !core || !factors || !out)
        return ORC_EINVAL;
    int64_t cap = prod_dims(ndim, full);
    int64_t cur[ORC_MAX_NDIM];
    memcpy(cur, ranks, sizeof(int64_t) * ndim);
    int64_t peak = prod_dims(ndim, ranks);
    /* the working tensor only grows from ranks to full dims */
    if (cap > peak) peak = cap;
    for (int k = 0; k < ndim; ++k) {
        int64_t t = 1;
        for (int m = 0; m < ndim; ++m) t *= (m <= k) ? full[m] : ranks[m];
        if (t > peak) peak = t;
    }
    double* a = (double*)malloc(sizeof(double) * peak);
    double* b = (double*)malloc(sizeof(double) * peak);
    if (!a || !b) { free(a); free(b); return ORC_ENOMEM; }
    memcpy(a, core, sizeof(double) * prod_dims(ndim, ranks));
    const double* u = factors;
    for (int n = 0; n < ndim; ++n) {
        orc_ttm(a, ndim, cur, n, u, full[n], b); /* U_n is full[n] x ranks[n] */
        cur[n] = full[n];
        u += full[n] * ranks[n];
        double* t = a; a = b; b = t;
    }
    memcpy(out, a, sizeof(double) * cap);
    free(a); free(b);
    return ORC_OK;
}

/*
 * Error metrics against the original tensor: out[0] = ||X - X~||^2,
 * out[1] = max |X - X~|, out[2] = ||X||^2 (pairwise sums).
 */
int orc_error_metrics(const double* x, const double* xh, int64_t count, double* out) {
    if (!x || !xh || !out || count < 1) return ORC_EINVAL;
    double* d = (double*)malloc(sizeof(double) * count);
    if (!d) return ORC_ENOMEM;
    double mx = 0.0;
    for (int64_t i = 0; i < count; ++i) {
        d[i] = x[i] - xh[i];
        if (fabs(d[i]) > mx) mx = fabs(d[i]);
    }
    out[0] = pw_sumsq(d, count);
    out[1] = mx;
    out[2] = pw_sumsq(x, count);
    free(d);
    return ORC_OK;
}

/* --------------------------------------------- QR-preprocessed SVD (Sec. IX) */

/*
 * R factor of a Householder QR of the row-major m x j matrix a (the paper's
 * stable alternative to the Gram for eps near sqrt(u), Sec. IX: Y_(n)^T is
 * tall and skinny, so its SVD goes through a QR factorisation first).
 * Textbook column-by-column reduction (Golub & Van Loan, "Householder QR"):
 * for k = 0 .. min(m, j) - 1 the reflector I - tau v v^T with v_k = 1 maps
 * a[k:m, k] to beta e_k, beta = -sign(a_kk) ||a[k:m, k]|| (sign(0) = +),
 * tau = (beta - a_kk) / beta, v_i = a_ik / (a_kk - beta) for i > k; no
 * reflection (tau = 0) when a[k+1:m, k] is zero.  It is applied to columns
 * k+1 .. j-1.  On exit r (row-major j x j) holds R with its strict lower part
 * zero and each row signed so that its diagonal entry is >= 0 (R is unique
 * when a has full column rank); rows >= m of R are zero.  a is overwritten.
 */
int orc_qr_r(double* a, int64_t m, int64_t j, double* r) {
    if (!a || !r || m < 1 || j < 1) return ORC_EINVAL;
    double* col = (double*)malloc(sizeof(double) * m);
    double* vcol = (double*)malloc(sizeof(double) * m);
    if (!col || !vcol) { free(col); free(vcol); return ORC_ENOMEM; }
    const int64_t kmax = m < j ? m : j;
    for (int64_t k = 0; k < kmax; ++k) {
        const int64_t len = m - k - 1; /* entries below the diagonal */
        for (int64_t i = 0; i < len; ++i) col[i] = a[(k + 1 + i) * j + k];
        const double xnorm = sqrt(pw_sumsq(col, len));
        if (xnorm == 0.0) continue; /* H_k = I */
        const double alpha = a[k * j + k];
        const double nrm = hypot(alpha, xnorm);
        const double beta = alpha >= 0.0 ? -nrm : nrm;
        const double tau = (beta - alpha) / beta;
        const double scal = 1.0 / (alpha - beta);
        for (int64_t i = 0; i < len; ++i) vcol[i] = col[i] * scal;
        a[k * j + k] = beta;
        for (int64_t i = 0; i < len; ++i) a[(k + 1 + i) * j + k] = 0.0;
        for (int64_t c = k + 1; c < j; ++c) {
            for (int64_t i = 0; i < len; ++i) col[i] = a[(k + 1 + i) * j + c];
            const double w = tau * (a[k * j + c] + pw_dot(vcol, col, len));
            a[k * j + c] -= w;
            for (int64_t i = 0; i < len; ++i) a[(k + 1 + i) * j + c] -= vcol[i] * w;
        }
    }
    for (int64_t i = 0; i < j; ++i) {
        const double sg = (i < m && a[i * j + i] < 0.0) ? -1.0 : 1.0;
        for (int64_t c = 0; c < j; ++c)
            r[i * j + c] = (i < m && c >= i) ? sg * a[i * j + c] : 0.0;
    }
    free(col); free(vcol);
    return ORC_OK;
}

/*
 * One-sided (Hestenes) Jacobi SVD of a square j x j matrix b (row-major;
 * textbook method, e.g. Golub & Van Loan, "one-sided Jacobi"): cyclic
 * sweeps over column pairs (p, q) rotate columns p and q of b so that they
 * become orthogonal, and accumulate the same rotations in v, so that on
 * convergence b_in v = W diag(sigma) with orthonormal W.  A pair is skipped
 * when |b_p . b_q| <= tol ||b_p|| ||b_q|| (tol = 4 j DBL_EPSILON) or one of
 * the columns is zero; iteration stops after a sweep with no rotation.
 * On exit sigma holds the column norms sorted descending (ties in index
 * order) -- the singular values -- and the columns of v (row-major j x j)
 * the matching right singular vectors, each signed so that its
 * largest-magnitude entry (lowest index on ties) is positive.  b is
 * overwritten.  Returns the sweeps used, or ORC_ENOCONV after max_sweeps.
 */
int orc_svd_jacobi(double* b, int64_t j, double* sigma, double* v, int max_sweeps) {
    if (!b || !sigma || !v || j < 1) return ORC_EINVAL;
    const double tol = 4.0 * (double)j * 2.220446049250313e-16;
    double* cp = (double*)malloc(sizeof(double) * j);
    double* cq = (double*)malloc(sizeof(double) * j);
    double* nrm = (double*)malloc(sizeof(double) * j);
    int64_t* perm = (int64_t*)malloc(sizeof(int64_t) * j);
    double* tmp = (double*)malloc(sizeof(double) * j * j);
    if (!cp || !cq || !nrm || !perm || !tmp) {
        free(cp); free(cq); free(nrm); free(perm); free(tmp);
        return ORC_ENOMEM;
    }
    for (int64_t a = 0; a < j; ++a)
        for (int64_t c = 0; c < j; ++c) v[a * j + c] = (a == c) ? 1.0 : 0.0;
    int sweep = 0, converged = 0;
    for (sweep = 1; sweep <= max_sweeps; ++sweep) {
        int rotated = 0;
        for (int64_t p = 0; p < j - 1; ++p) {
            for (int64_t q = p + 1; q < j; ++q) {
                for (int64_t i = 0; i < j; ++i) { cp[i] = b[i * j + p]; cq[i] = b[i * j + q]; }
                const double alpha = pw_sumsq(cp, j), beta = pw_sumsq(cq, j);
                const double gamma = pw_dot(cp, cq, j);
                if (alpha == 0.0 || beta == 0.0) continue;
                if (fabs(gamma) <= tol * sqrt(alpha) * sqrt(beta)) continue;
                rotated = 1;
                /* rotation zeroing the (p, q) entry of the 2 x 2 Gram
                   [[alpha, gamma], [gamma, beta]] (same root choice as the
                   two-sided Jacobi above) */
                const double zeta = (beta - alpha) / (2.0 * gamma);
                double t;
                if (fabs(zeta) > 1e150) t = 0.5 / zeta;
                else t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / sqrt(1.0 + t * t);
                const double s = t * c;
                for (int64_t i = 0; i < j; ++i) {
                    b[i * j + p] = c * cp[i] - s * cq[i];
                    b[i * j + q] = s * cp[i] + c * cq[i];
                }
                for (int64_t i = 0; i < j; ++i) {
                    const double vp = v[i * j + p], vq = v[i * j + q];
                    v[i * j + p] = c * vp - s * vq;
                    v[i * j + q] = s * vp + c * vq;
                }
            }
        }
        if (!rotated) { converged = 1; break; }
    }
    for (int64_t p = 0; p < j; ++p) {
        for (int64_t i = 0; i < j; ++i) cp[i] = b[i * j + p];
        nrm[p] = sqrt(pw_sumsq(cp, j));
    }
    for (int64_t a = 0; a < j; ++a) perm[a] = a;
    for (int64_t a = 1; a < j; ++a) { /* stable insertion sort, descending */
        int64_t cur = perm[a];
        int64_t c = a - 1;
        while (c >= 0 && nrm[perm[c]] < nrm[cur]) { perm[c + 1] = perm[c]; --c; }
        perm[c + 1] = cur;
    }
    for (int64_t a = 0; a < j; ++a) sigma[a] = nrm[perm[a]];
    for (int64_t i = 0; i < j; ++i)
        for (int64_t a = 0; a < j; ++a) tmp[i * j + a] = v[i * j + perm[a]];
    for (int64_t a = 0; a < j; ++a) { /* sign rule */
        int64_t best = 0;
        for (int64_t i = 1; i < j; ++i)
            if (fabs(tmp[i * j + a]) > fabs(tmp[best * j + a])) best = i;
        if (tmp[best * j + a] < 0)
            for (int64_t i = 0; i < j; ++i) tmp[i * j + a] = -tmp[i * j + a];
    }
    memcpy(v, tmp, sizeof(double) * j * j);
    free(cp); free(cq); free(nrm); free(perm); free(tmp);
    return converged ? sweep : ORC_ENOCONV;
}
