// HOOI (Alg. 2) of one tensor on the device: ST-HOSVD (Alg. 1) for the
// starting factors and ranks, then sweeps.  In a sweep, for n = 1..N the
// tensor is multiplied by U_m^T in every mode m != n (ascending m, TTMs on
// the ping-pong buffers), the Gram of the result in mode n is formed and its
// leading R_n eigenvectors replace U_n; after mode N the core is
// G = Y x_N U_N^T.  The fit ||X||^2 - ||G||^2 (equal to the model error for
// orthonormal factors and this core) is read back once per sweep and decides
// whether to continue.
#include <cmath>
#include <cstring>

#include "tk_common.hpp"

using namespace tk;

namespace {

int64_t cap_rank(const tk_shape* x, const tk_options* opt, int n) {
    int64_t c = x->dims[n];
    if (opt->max_ranks && opt->max_ranks[n] < c) c = opt->max_ranks[n];
    if (opt->fixed_ranks && opt->fixed_ranks[n] < c) c = opt->fixed_ranks[n];
    return c;
}

// Gram precision of mode n in a sweep: as sthosvd_compress, narrow small
// modes take the FP64 Gram on the mixed path.
int gram_prec(const tk_options* opt, const ModeView& v) {
    int g = opt->gram_precision;
    if (g == TK_GRAM_SPLIT_BF16 && mixed_takes_fp64_gram(v)) g = TK_GRAM_FP64;
    return g;
}

struct HooiPlan {
    size_t ybytes = 0, gram_bytes = 0, s_bytes = 0, eig_bytes = 0, lam_bytes = 0;
    size_t sweep_total = 0, total = 0;
};

// Sizes at the rank capacities (the ranks are found by the ST-HOSVD).
HooiPlan plan_hooi(const tk_shape* x, const tk_options* opt) {
    HooiPlan pl;
    const int N = x->ndim;
    const size_t b = x->dtype == TK_F64 ? 8 : 4;
    int64_t cap[TK_MAX_NDIM];
    int jmax = 1;
    int64_t sumd = 0;
    for (int k = 0; k < N; ++k) {
        cap[k] = cap_rank(x, opt, k);
        if (x->dims[k] > jmax) jmax = (int)x->dims[k];
        sumd += x->dims[k];
    }
    for (int n = 0; n < N; ++n) {
        int64_t cur[TK_MAX_NDIM];
        for (int k = 0; k < N; ++k) cur[k] = x->dims[k];
        for (int m = 0; m < N; ++m) {
            if (m == n) continue;
            cur[m] = cap[m];
            int64_t ne = 1;
            for (int k = 0; k < N; ++k) ne *= cur[k];
            if ((size_t)ne * b > pl.ybytes) pl.ybytes = (size_t)ne * b;
        }
        const ModeView v = mode_view(cur, N, n);
        const GramPlan gp = plan_gram(v, gram_prec(opt, v), (int)b);
        if (gp.partial_bound > pl.gram_bytes) pl.gram_bytes = gp.partial_bound;
    }
    {   // ||G||^2: the core's mode-1 Gram in FP64
        const ModeView v = mode_view(cap, N, 0);
        const GramPlan gp = plan_gram(v, TK_GRAM_FP64, (int)b);
        if (gp.partial_bound > pl.gram_bytes) pl.gram_bytes = gp.partial_bound;
        if (cap[0] > jmax) jmax = (int)cap[0];
    }
    pl.s_bytes = (size_t)jmax * jmax * sizeof(double);
    pl.eig_bytes = eig_scratch_doubles(jmax) * sizeof(double);
    pl.lam_bytes = (size_t)sumd * sizeof(double);
    Carver c(nullptr, 0);
    c.take(pl.ybytes);
    c.take(pl.ybytes);
    c.take(pl.gram_bytes);
    c.take(pl.s_bytes);
    c.take(pl.eig_bytes);
    c.take(pl.lam_bytes);
    c.take(64 * sizeof(double));
    pl.sweep_total = c.used + 256;
    const size_t sth = sthosvd_workspace_bytes(x, opt);
    pl.total = sth > pl.sweep_total ? sth : pl.sweep_total;
    return pl;
}

int read_back(const double* dev, size_t n, double* host, hipStream_t st) {
    TK_HIP(hipMemcpyAsync(host, dev, n * sizeof(double), hipMemcpyDeviceToHost, st));
    TK_HIP(hipStreamSynchronize(st));
    return TK_OK;
}

}  // namespace

extern "C" {

size_t tucker_hooi_workspace_bytes(const tk_shape* x, const tk_options* opt) {
    if (!x || !opt || opt->gram_precision == TK_SVD_QR || sthosvd_workspace_bytes(x, opt) == 0)
        return 0;
    return plan_hooi(x, opt).total;
}

int tucker_hooi(const tk_shape* x, const void* x_dev, const tk_options* opt, int max_sweeps,
                double tol, tk_tucker* out, double* fits, int* sweeps_done, void* ws,
                size_t ws_bytes, void* stream) {
    if (max_sweeps < 0) return fail(TK_ERR_INVALID_ARG, "tucker_hooi: max_sweeps %d < 0", max_sweeps);
    if (!std::isfinite(tol)) return fail(TK_ERR_INVALID_ARG, "tucker_hooi: tol is not finite");
    if (!x || !opt || !out) return fail(TK_ERR_INVALID_ARG, "tucker_hooi: NULL argument");
    if (opt->gram_precision == TK_SVD_QR)
        return fail(TK_ERR_UNSUPPORTED, "tucker_hooi: the QR path is provided by "
                    "sthosvd_compress only");
    if (sthosvd_workspace_bytes(x, opt) == 0)  // invalid shape or options: let compress report
        return sthosvd_compress(x, x_dev, opt, out, ws, ws_bytes, stream);
    const HooiPlan pl = plan_hooi(x, opt);
    TK_TRY(check_ws(ws, ws_bytes, pl.total, "tucker_hooi"));
    // Alg. 2, first line: ST-HOSVD
    TK_TRY(sthosvd_compress(x, x_dev, opt, out, ws, ws_bytes, stream));
    hipStream_t st = (hipStream_t)stream;
    const int N = x->ndim;
    const size_t b = x->dtype == TK_F64 ? 8 : 4;
    const int ttm_prec = out->ttm_precision_used;
    int64_t R[TK_MAX_NDIM];
    for (int k = 0; k < N; ++k) R[k] = out->ranks[k];
    if ((double)out->core_capacity < 1.0)
        return fail(TK_ERR_CAPACITY, "tucker_hooi: no core capacity");

    Carver c(ws, ws_bytes);
    void* ybuf[2] = {c.take(pl.ybytes), c.take(pl.ybytes)};
    void* gram_ws = c.take(pl.gram_bytes);
    double* S = (double*)c.take(pl.s_bytes);
    double* eig_ws = (double*)c.take(pl.eig_bytes);
    double* lam_ws = (double*)c.take(pl.lam_bytes);
    double* scal = (double*)c.take(64 * sizeof(double));
    double* g2_dev = scal;                      // [0]
    double* disc_dev = scal + 1;                // [1..8]
    int64_t* rank_dev = (int64_t*)(scal + 16);  // [16..23]
    int* flags_dev = (int*)(scal + 32);         // [32]
    double* lam_all = out->eigvals_dev ? out->eigvals_dev : lam_ws;
    int64_t lam_off[TK_MAX_NDIM];
    {
        int64_t o = 0;
        for (int k = 0; k < N; ++k) {
            lam_off[k] = o;
            o += x->dims[k];
        }
    }
    TK_HIP(hipMemsetAsync(scal, 0, 64 * sizeof(double), st));

    auto core_norm2 = [&](double* g2) -> int {
        const ModeView v = mode_view(R, N, 0);
        TK_TRY(launch_gram(out->core_dev, x->dtype, v, TK_GRAM_FP64, S, g2_dev, gram_ws,
                           pl.gram_bytes, st));
        return read_back(g2_dev, 1, g2, st);
    };
    const double nu = out->norm2;
    double g2 = 0.0;
    TK_TRY(core_norm2(&g2));
    double fit_prev = nu - g2;
    if (fits) fits[0] = fit_prev;
    int done = 0;
    for (int it = 0; it < max_sweeps; ++it) {
        const void* y = x_dev;
        int64_t cur[TK_MAX_NDIM];
        for (int n = 0; n < N; ++n) {
            // Y = X x_m U_m^T for every m != n
            for (int k = 0; k < N; ++k) cur[k] = x->dims[k];
            y = x_dev;
            int pp = 0;
            for (int m = 0; m < N; ++m) {
                if (m == n) continue;
                const ModeView v = mode_view(cur, N, m);
                TK_TRY(launch_ttm(y, x->dtype, v, out->factors_dev[m], R[m], x->dims[m], 1,
                                  ttm_prec, ybuf[pp], st));
                cur[m] = R[m];
                y = ybuf[pp];
                pp ^= 1;
            }
            const ModeView v = mode_view(cur, N, n);
            TK_TRY(launch_gram(y, x->dtype, v, gram_prec(opt, v), S, nullptr, gram_ws,
                               pl.gram_bytes, st));
            EigArgs ea;
            ea.s = S;
            ea.J = v.J;
            ea.nu = g2_dev;           // unused with a fixed rank
            ea.eps2_over_n = 0.0;
            ea.fixed_rank = (int)R[n];
            ea.max_rank = (int)R[n];
            ea.lambda = lam_all + lam_off[n];
            ea.u = out->factors_dev[n];
            ea.rank_out = rank_dev + n;
            ea.disc_out = disc_dev + n;
            ea.flags = flags_dev;
            ea.scratch = eig_ws;
            ea.guard = 0.0;
            TK_TRY(launch_eig(ea, st));
        }
        // core from the last mode's Y (every mode but N already applied)
        {
            const ModeView v = mode_view(cur, N, N - 1);
            int64_t ncore = 1;
            for (int k = 0; k < N; ++k) ncore *= R[k];
            if (ncore > out->core_capacity)
                return fail(TK_ERR_CAPACITY, "tucker_hooi: core has %lld elements, capacity %lld",
                            (long long)ncore, (long long)out->core_capacity);
            TK_TRY(launch_ttm(y, x->dtype, v, out->factors_dev[N - 1], R[N - 1], x->dims[N - 1],
                              1, ttm_prec, out->core_dev, st));
        }
        TK_TRY(core_norm2(&g2));
        const double fit = nu - g2;
        ++done;
        if (fits) fits[done] = fit;
        const bool stop = tol >= 0.0 && fit_prev - fit <= tol * nu;
        fit_prev = fit;
        if (stop) break;
    }
    if (done > 0) {
        double sc[9];
        TK_TRY(read_back(scal, 9, sc, st));
        for (int k = 0; k < N; ++k) out->discarded[k] = sc[1 + k];
    }
    if (sweeps_done) *sweeps_done = done;
    (void)b;
    return TK_OK;
}

}  // extern "C"
