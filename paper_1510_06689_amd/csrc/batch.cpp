// Batches of independent ST-HOSVD problems (Alg. 1 per problem): host-side
// planning, the enqueue-only run (graph-capturable) and the finishing step.
//
// Every mode step s of the common mode order runs, for the whole batch, as
//   split Gram       (one launch per padded-extent class, workgroups dealt
//                     to problems in proportion to their capacity-size tiles;
//                     the class of extents up to 32 takes the FP64 Gram
//                     instead, which costs no more there and needs no guard)
//   reduction        (one launch; step 0 also forms ||X||^2 per problem)
//   eigensolver      (one workgroup per problem, rank rule and guard on the
//                     device)
//   guard redo       (FP64 Gram, reduction and eigensolver again, each
//                     launch doing work only for the problems whose rank the
//                     split Gram could not certify)
//   split-bf16 TTM   (one launch per extent class; each problem's rank read
//                     from device memory)
// with each problem's shapes at later steps derived on the device from its
// ranks.  Buffers are laid out at the rank capacities, so the plan -- the
// device task tables -- is fixed and uploaded once.
#include <cmath>
#include <cstring>
#include <algorithm>
#include <array>
#include <map>
#include <vector>

#include "tk_common.hpp"

using namespace tk;

namespace {

struct GramLaunch {
    int jb, ntasks, total_wg;
    size_t off;  // byte offset of its tasks in the table area
    bool f64;    // FP64 Gram (extents up to 32), else the split Gram
    // split Gram loader variants to launch (launch_gram_split_batched): at the
    // first step the strides are the input's, so L == 1 (bit 0) or not (bits
    // 1 and 2, both, the alignment rule being the device's) is known; later
    // strides come from ranks found on the device, and all three run
    unsigned loaders = 7;
};

// Extent classes whose Gram runs in FP64 arithmetic: at J <= 32 the FP64
// Gram's intensity on FP32 data is below the FP64 matrix-core ridge, so it
// costs no more than the split Gram, and its rank needs no guard.
bool f64_class(int jb) { return jb <= 32; }

// Workgroups of one problem's Gram: its tiles over tiles-per-workgroup.  An
// FP64 class's problems are small and its kernel walks finer tiles, so it
// takes a quarter of the tiles per workgroup (more workgroups in flight).
int gram_wgs(int64_t ntiles, int tpw, int jb, int cap) {
    const int t = f64_class(jb) ? std::max(1, tpw / 4) : tpw;
    return std::max(1, std::min(cap, (int)((ntiles + t - 1) / t)));
}

// Workgroups per task and launch at step s of a batch of B problems.  From
// the second step on a task's shape is known only on the device, so its
// workgroups are counted at the capacity shape, most of which truncation
// usually removes (the surplus exits at once, at a few microseconds per
// thousand workgroups).  The cap, 16384 over the batch and at least 256 per
// task, binds where that count runs far past what fills the GPU (the last
// modes of many small problems); should the ranks come out at capacity, the
// workgroups walk more tiles or column blocks each.  A cap of 4096 over the
// batch also bound the middle modes' split Grams, whose truncated shapes
// still hold real work, and slowed them.
int batch_wg_cap(int s, int B) {
    return s == 0 ? 4096 : std::min(4096, std::max(256, 16384 / std::max(1, B)));
}

// From the second step on, a problem of a split class whose FP64 Gram takes
// at most this many flops (2 K J^2 at its actual shape, known on the device
// only) is marked before the Grams (status bit 8) and takes the FP64 Gram
// instead of the split one.  A truncated unfolding's rows span a wide range
// of magnitudes, so the 16-bit split's error bound often cannot certify its
// rank, and for a small problem the split Gram plus an FP64 redo costs more
// than the FP64 Gram alone.  Marked problems take the same reduction and
// eigensolver launches as the others, so the step keeps one eigensolver pass.
constexpr double kBatchF64Flops = 6e7;
struct TtmLaunch {
    int J, kmax, ntasks, total_wg;  // J: the largest extent of the launch's tasks
    size_t off;
};
struct StepPlan {
    std::vector<GramLaunch> grams;
    size_t red_off = 0;
    int red_ntasks = 0, red_wg = 0;
    size_t eig_off = 0;
    int jmax = 0;
    std::vector<TtmLaunch> ttms;
};

constexpr int kDefaultGramTilesPerWg = 16;
constexpr int kDefaultTtmBlocksPerWg = 64;

int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

int round_pow2_32(int J) {
    int jb = 32;
    while (jb < J) jb *= 2;
    return jb;
}

}  // namespace

struct tk_batch {
    int B = 0, N = 0;
    int order[TK_MAX_NDIM];
    std::vector<tk_shape> shapes;
    std::vector<const void*> x;
    tk_options opt{};
    std::vector<int32_t> mode_order;
    std::vector<int64_t> fixed, maxr;
    std::vector<void*> cores;
    std::vector<int64_t> core_cap;
    std::vector<double*> factors;  // B * TK_MAX_NDIM
    int64_t* ranks_dev = nullptr;
    double* disc_dev = nullptr;
    double* norm2_dev = nullptr;
    int32_t* status_dev = nullptr;
    double* tail_bound_dev = nullptr;  // optional output
    std::vector<StepPlan> steps;
    char* tables_dev = nullptr;
    std::vector<double*> lam;  // per problem, sum of extents
    bool guarded = false;      // rank rule with the split Gram's guard
};

namespace {

// Validation shared by the size query and create.
int check_batch(int batch, const tk_shape* shapes, const tk_options* opt) {
    if (batch < 1) return fail(TK_ERR_INVALID_ARG, "sthosvd_batch: batch %d < 1", batch);
    if (!shapes || !opt) return fail(TK_ERR_INVALID_ARG, "sthosvd_batch: NULL shapes or options");
    const int N = shapes[0].ndim;
    for (int b = 0; b < batch; ++b) {
        TK_TRY(check_shape(&shapes[b], "sthosvd_batch"));
        if (shapes[b].ndim != N)
            return fail(TK_ERR_INVALID_ARG, "sthosvd_batch: problem %d has ndim %d != %d", b,
                        shapes[b].ndim, N);
        if (shapes[b].dtype != TK_F32)
            return fail(TK_ERR_UNSUPPORTED, "sthosvd_batch: problems must be stored FP32");
        for (int k = 0; k < N; ++k)
            if (shapes[b].dims[k] > 128)
                return fail(TK_ERR_UNSUPPORTED, "sthosvd_batch: extent %lld > 128",
                            (long long)shapes[b].dims[k]);
    }
    if (!(opt->eps >= 0.0) || !std::isfinite(opt->eps))
        return fail(TK_ERR_INVALID_ARG, "sthosvd_batch: eps must be finite and >= 0");
    if (opt->gram_precision != TK_GRAM_SPLIT_BF16)
        return fail(TK_ERR_UNSUPPORTED, "sthosvd_batch: needs gram_precision TK_GRAM_SPLIT_BF16");
    if (opt->ttm_precision != TK_TTM_BF16X3 && opt->ttm_precision != TK_TTM_BF16)
        return fail(TK_ERR_UNSUPPORTED, "sthosvd_batch: needs a bf16 TTM precision");
    if (!opt->fixed_ranks &&
        ttm_precision_for_eps(opt->ttm_precision, opt->eps * opt->eps / N) != opt->ttm_precision)
        return fail(TK_ERR_UNSUPPORTED, "sthosvd_batch: eps^2/N below the %s TTM's accuracy "
                    "floor (%s)", opt->ttm_precision == TK_TTM_BF16 ? "bf16" : "split-bf16",
                    opt->ttm_precision == TK_TTM_BF16 ? "2^-13; use TK_TTM_BF16X3"
                                                      : "2^-31");
    bool seen[TK_MAX_NDIM] = {false};
    for (int k = 0; k < N; ++k) {
        const int n = opt->mode_order ? opt->mode_order[k] : k;
        if (n < 0 || n >= N || seen[n])
            return fail(TK_ERR_INVALID_ARG, "sthosvd_batch: mode_order is not a permutation");
        seen[n] = true;
    }
    for (int b = 0; b < batch; ++b)
        for (int n = 0; n < N; ++n) {
            if (opt->fixed_ranks && (opt->fixed_ranks[n] < 1 || opt->fixed_ranks[n] > shapes[b].dims[n]))
                return fail(TK_ERR_INVALID_ARG, "sthosvd_batch: fixed_ranks[%d] out of range", n);
            if (opt->max_ranks && opt->max_ranks[n] < 1)
                return fail(TK_ERR_INVALID_ARG, "sthosvd_batch: max_ranks[%d] < 1", n);
        }
    return TK_OK;
}

int64_t cap_of(const tk_shape& sh, const tk_options* opt, int n) {
    int64_t c = sh.dims[n];
    if (opt->max_ranks && opt->max_ranks[n] < c) c = opt->max_ranks[n];
    if (opt->fixed_ranks && opt->fixed_ranks[n] < c) c = opt->fixed_ranks[n];
    return c;
}

// Lays out the workspace and, when h is non-null, fills the host-side plan
// and the task tables (returned in `tables`, copied to the device by create).
// Returns the workspace bytes.
size_t plan_batch(int B, const tk_shape* shapes, const tk_options* opt, const tk_batch_tuning* tn,
                  void* ws, tk_batch* h, std::vector<char>* tables) {
    const int N = shapes[0].ndim;
    int order[TK_MAX_NDIM];
    for (int k = 0; k < N; ++k) order[k] = opt->mode_order ? opt->mode_order[k] : k;
    Carver c(ws, ~size_t(0) >> 1);
    // per-problem buffers
    struct Bufs {
        void* y[2];
        double *partial, *aux, *stats, *S, *scratch, *lam;
        int* nparts;
    };
    std::vector<Bufs> bufs(B);
    for (int b = 0; b < B; ++b) {
        const tk_shape& sh = shapes[b];
        int64_t capcur[TK_MAX_NDIM];
        for (int k = 0; k < N; ++k) capcur[k] = sh.dims[k];
        size_t yb[2] = {0, 0}, pb = 0, ab = 0;
        int jmax = 1;
        for (int s = 0; s < N; ++s) {
            const int n = order[s];
            const ModeView v = mode_view(capcur, N, n);
            const int jb = round_pow2_32(v.J);
            const int nb16 = 2 * (jb / 32), np16 = nb16 * (nb16 + 1) / 2;
            const int tpw = tn && tn->gram_tiles_per_wg[s] > 0 ? tn->gram_tiles_per_wg[s]
                                                               : kDefaultGramTilesPerWg;
            const int nwg = gram_wgs(make_tiles(v, mx_gram_kt(jb)).ntiles, tpw, jb,
                                     batch_wg_cap(s, B));
            pb = std::max(pb, (size_t)nwg * np16 * 256 * sizeof(double));
            ab = std::max(ab, (size_t)nwg * 2 * sizeof(double));
            jmax = std::max(jmax, v.J);
            capcur[n] = cap_of(sh, opt, n);
            if (s + 1 < N) {
                int64_t ne = 1;
                for (int k = 0; k < N; ++k) ne *= capcur[k];
                yb[s & 1] = std::max(yb[s & 1], (size_t)ne * sizeof(float));
            }
        }
        int64_t sumd = 0;
        for (int k = 0; k < N; ++k) sumd += sh.dims[k];
        bufs[b].y[0] = c.take(yb[0]);
        bufs[b].y[1] = c.take(yb[1]);
        bufs[b].partial = (double*)c.take(pb);
        bufs[b].aux = (double*)c.take(ab);
        bufs[b].stats = (double*)c.take(2 * sizeof(double));
        bufs[b].S = (double*)c.take((size_t)jmax * jmax * sizeof(double));
        bufs[b].scratch = (double*)c.take(eig_scratch_doubles(jmax) * sizeof(double));
        bufs[b].lam = (double*)c.take((size_t)sumd * sizeof(double));
        bufs[b].nparts = (int*)c.take(sizeof(int));
    }

    // task tables: build on the host in one byte array
    std::vector<char> tab;
    auto put = [&](const void* p, size_t n) {
        size_t o = (tab.size() + 15) & ~size_t(15);
        tab.resize(o + n);
        memcpy(tab.data() + o, p, n);
        return o;
    };
    std::vector<StepPlan> steps(N);
    int done = 0;
    std::vector<std::array<int64_t, TK_MAX_NDIM>> capcur(B);
    for (int b = 0; b < B; ++b)
        for (int k = 0; k < N; ++k) capcur[b][k] = shapes[b].dims[k];
    for (int s = 0; s < N; ++s) {
        const int n = order[s];
        StepPlan& sp = steps[s];
        // Gram tasks, grouped by padded-extent class
        std::map<int, std::vector<BatchGramTask>> gclass;
        std::map<int, unsigned> gloaders;
        std::map<int, std::vector<BatchTtmTask>> tclass;
        std::map<int, int> tkmax, tjmax;
        std::vector<BatchReduceTask> red;
        std::vector<EigArgs> eig(B);
        int red_wg = 0;
        for (int b = 0; b < B; ++b) {
            const tk_shape& sh = shapes[b];
            const ModeView v = mode_view(capcur[b].data(), N, n);
            const int jb = round_pow2_32(v.J);
            const int nb16 = 2 * (jb / 32), np16 = nb16 * (nb16 + 1) / 2;
            const int tpw = tn && tn->gram_tiles_per_wg[s] > 0 ? tn->gram_tiles_per_wg[s]
                                                               : kDefaultGramTilesPerWg;
            const int64_t ntiles = make_tiles(v, mx_gram_kt(jb)).ntiles;
            const int nwg = gram_wgs(ntiles, tpw, jb, batch_wg_cap(s, B));
            BatchView bv{};
            for (int k = 0; k < N; ++k) bv.dims[k] = sh.dims[k];
            bv.ranks = h ? h->ranks_dev + (size_t)b * N : nullptr;
            bv.ndim = N;
            bv.n = n;
            bv.done = done;
            const void* yin = s == 0 ? (h ? h->x[b] : nullptr) : bufs[b].y[(s - 1) & 1];
            const int* status = h ? h->status_dev + 2 * b : nullptr;
            BatchGramTask gt{bv, (const float*)yin, bufs[b].partial, bufs[b].aux, status,
                             bufs[b].nparts, ceil_div(ntiles, nwg)};
            gt.v.nwg = nwg;
            gclass[jb].push_back(gt);
            // the first step's view is the input's (capacities start at the
            // extents), so its stride is exact here
            gloaders[jb] |= s > 0 ? 7u : v.L == 1 ? 1u : 6u;
            const bool f64 = f64_class(jb);
            BatchReduceTask rt{bufs[b].partial, bufs[b].S,
                               s == 0 && h ? h->norm2_dev + b : nullptr,
                               f64 ? nullptr : bufs[b].aux, f64 ? nullptr : bufs[b].stats, nwg,
                               np16, nb16, v.J, 0, 0, status, bufs[b].nparts};
            // one more workgroup: split statistics, and at step 0 the trace
            rt.nwg = ceil_div((int64_t)np16 * 256, 64) + 1;
            rt.wg_begin = red_wg;
            red_wg += rt.nwg;
            red.push_back(rt);
            int64_t lam_off = 0;
            for (int k = 0; k < n; ++k) lam_off += sh.dims[k];
            EigArgs& ea = eig[b];
            ea.s = bufs[b].S;
            ea.J = v.J;
            ea.nu = h ? h->norm2_dev + b : nullptr;
            ea.eps2_over_n = opt->eps * opt->eps / (double)N;
            ea.fixed_rank = opt->fixed_ranks ? (int)opt->fixed_ranks[n] : 0;
            ea.max_rank = (int)cap_of(sh, opt, n);
            ea.lambda = bufs[b].lam + lam_off;
            ea.u = h ? h->factors[(size_t)b * TK_MAX_NDIM + n] : nullptr;
            ea.rank_out = h ? h->ranks_dev + (size_t)b * N + n : nullptr;
            ea.disc_out = h ? h->disc_dev + (size_t)b * N + n : nullptr;
            ea.flags = h ? h->status_dev + 2 * b : nullptr;
            ea.scratch = bufs[b].scratch;
            // the rank rule flags only under the eps rule, and only split Grams
            ea.guard = f64 ? 0.0 : kSplitGramGuard;
            ea.split_stats = f64 ? nullptr : bufs[b].stats;
            ea.ncols = (double)v.L * (double)v.B;  // at the capacity shape: an upper bound
            ea.tail_bound = h && h->tail_bound_dev ? h->tail_bound_dev + (size_t)b * N + n
                                                    : nullptr;
            sp.jmax = std::max(sp.jmax, v.J);
            // TTM into the other buffer (the core at the last step)
            void* yout = s + 1 == N ? (h ? h->cores[b] : nullptr) : bufs[b].y[s & 1];
            const int bpw = tn && tn->ttm_blocks_per_wg[s] > 0 ? tn->ttm_blocks_per_wg[s]
                                                               : kDefaultTtmBlocksPerWg;
            BatchTtmTask tt{bv, (const float*)yin, ea.u, (float*)yout};
            tt.v.nwg = std::max(1, std::min(batch_wg_cap(s, B),
                                            ceil_div(ceil_div(v.L * v.B, 16), bpw)));
            const int jcls = v.J <= 32 ? 32 : v.J <= 64 ? 64 : 128;
            tclass[jcls].push_back(tt);
            tkmax[jcls] = std::max(tkmax[jcls], ea.max_rank);
            tjmax[jcls] = std::max(tjmax[jcls], v.J);  // a mode's extent is not truncated before it
            capcur[b][n] = cap_of(sh, opt, n);
        }
        for (auto& kv : gclass) {
            int wg = 0;
            for (auto& t : kv.second) {
                t.v.wg_begin = wg;
                wg += t.v.nwg;
            }
            sp.grams.push_back({kv.first, (int)kv.second.size(), wg,
                                put(kv.second.data(), kv.second.size() * sizeof(BatchGramTask)),
                                f64_class(kv.first), gloaders[kv.first]});
        }
        sp.red_off = put(red.data(), red.size() * sizeof(BatchReduceTask));
        sp.red_ntasks = (int)red.size();
        sp.red_wg = red_wg;
        sp.eig_off = put(eig.data(), eig.size() * sizeof(EigArgs));
        for (auto& kv : tclass) {
            int wg = 0;
            for (auto& t : kv.second) {
                t.v.wg_begin = wg;
                wg += t.v.nwg;
            }
            sp.ttms.push_back({tjmax[kv.first], tkmax[kv.first], (int)kv.second.size(), wg,
                               put(kv.second.data(), kv.second.size() * sizeof(BatchTtmTask))});
        }
        done |= 1 << n;
    }
    char* tables_dev = (char*)c.take(tab.size());
    if (h) {
        h->steps = steps;
        h->tables_dev = tables_dev;
        h->guarded = !opt->fixed_ranks;
        h->lam.resize(B);
        for (int b = 0; b < B; ++b) h->lam[b] = bufs[b].lam;
        *tables = tab;
    }
    return c.used + 256;
}

}  // namespace

extern "C" {

size_t sthosvd_batch_workspace_bytes(int batch, const tk_shape* shapes, const tk_options* opt,
                                     const tk_batch_tuning* tuning) {
    if (check_batch(batch, shapes, opt) != TK_OK) return 0;
    return plan_batch(batch, shapes, opt, tuning, nullptr, nullptr, nullptr);
}

int sthosvd_batch_create(int batch, const tk_shape* shapes, const void* const* x_dev,
                         const tk_options* opt, const tk_batch_tuning* tuning,
                         const tk_batch_outputs* out, void* ws, size_t ws_bytes, void* stream,
                         tk_batch** handle) {
    if (!handle) return fail(TK_ERR_INVALID_ARG, "sthosvd_batch_create: handle NULL");
    *handle = nullptr;
    TK_TRY(check_batch(batch, shapes, opt));
    if (!x_dev || !out || !out->core_dev || !out->core_capacity || !out->factors_dev ||
        !out->ranks_dev || !out->discarded_dev || !out->norm2_dev || !out->status_dev)
        return fail(TK_ERR_INVALID_ARG, "sthosvd_batch_create: NULL input or output pointer");
    const int N = shapes[0].ndim;
    for (int b = 0; b < batch; ++b) {
        if (!x_dev[b] || !out->core_dev[b])
            return fail(TK_ERR_INVALID_ARG, "sthosvd_batch_create: problem %d has a NULL buffer", b);
        int64_t ncore = 1;
        for (int n = 0; n < N; ++n) {
            if (!out->factors_dev[(size_t)b * TK_MAX_NDIM + n])
                return fail(TK_ERR_INVALID_ARG, "sthosvd_batch_create: factor %d of problem %d NULL",
                            n, b);
            ncore *= cap_of(shapes[b], opt, n);
        }
        if (out->core_capacity[b] < ncore)
            return fail(TK_ERR_CAPACITY, "sthosvd_batch_create: core capacity of problem %d < %lld",
                        b, (long long)ncore);
    }
    const size_t need = plan_batch(batch, shapes, opt, tuning, nullptr, nullptr, nullptr);
    TK_TRY(check_ws(ws, ws_bytes, need, "sthosvd_batch_create"));

    tk_batch* h = new tk_batch();
    h->B = batch;
    h->N = N;
    h->shapes.assign(shapes, shapes + batch);
    h->x.assign(x_dev, x_dev + batch);
    h->opt = *opt;
    for (int k = 0; k < N; ++k) h->order[k] = opt->mode_order ? opt->mode_order[k] : k;
    if (opt->mode_order) {
        h->mode_order.assign(opt->mode_order, opt->mode_order + N);
        h->opt.mode_order = h->mode_order.data();
    }
    if (opt->fixed_ranks) {
        h->fixed.assign(opt->fixed_ranks, opt->fixed_ranks + N);
        h->opt.fixed_ranks = h->fixed.data();
    }
    if (opt->max_ranks) {
        h->maxr.assign(opt->max_ranks, opt->max_ranks + N);
        h->opt.max_ranks = h->maxr.data();
    }
    h->cores.assign(out->core_dev, out->core_dev + batch);
    h->core_cap.assign(out->core_capacity, out->core_capacity + batch);
    h->factors.assign(out->factors_dev, out->factors_dev + (size_t)batch * TK_MAX_NDIM);
    h->ranks_dev = out->ranks_dev;
    h->disc_dev = out->discarded_dev;
    h->norm2_dev = out->norm2_dev;
    h->status_dev = out->status_dev;
    h->tail_bound_dev = out->tail_bound_dev;
    std::vector<char> tables;
    plan_batch(batch, shapes, &h->opt, tuning, ws, h, &tables);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(h->tables_dev, tables.data(), tables.size(),
                                  hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        delete h;
        return fail(TK_ERR_HIP, "sthosvd_batch_create: table upload failed: %s",
                    hipGetErrorString(e));
    }
    *handle = h;
    return TK_OK;
}

int sthosvd_batch_run(tk_batch* h, void* stream) {
    if (!h) return fail(TK_ERR_INVALID_ARG, "sthosvd_batch_run: handle NULL");
    hipStream_t st = (hipStream_t)stream;
    TK_TRY(launch_fill_i32((int*)h->status_dev, 2 * h->B, 0, st));
    for (int s = 0; s < h->N; ++s) {
        const StepPlan& sp = h->steps[s];
        bool split = false;
        if (h->guarded && s > 0)
            for (const GramLaunch& g : sp.grams)
                if (!g.f64)
                    TK_TRY(launch_batch_mark_fp64((const BatchGramTask*)(h->tables_dev + g.off),
                                                  g.ntasks, kBatchF64Flops, st));
        for (const GramLaunch& g : sp.grams) {
            const BatchGramTask* tasks = (const BatchGramTask*)(h->tables_dev + g.off);
            if (g.f64) {
                TK_TRY(launch_gram_f64_batched(tasks, g.ntasks, g.total_wg, g.jb, 0, st));
            } else {
                TK_TRY(launch_gram_split_batched(tasks, g.ntasks, g.total_wg, g.jb, g.loaders,
                                                 st));
                if (h->guarded && s > 0)
                    TK_TRY(launch_gram_f64_batched(tasks, g.ntasks, g.total_wg, g.jb, 2, st));
                split = true;
            }
        }
        TK_TRY(launch_gram_reduce_batched((const BatchReduceTask*)(h->tables_dev + sp.red_off),
                                          sp.red_ntasks, sp.red_wg, 0, st));
        TK_TRY(launch_eig_batched((const EigArgs*)(h->tables_dev + sp.eig_off), h->B, sp.jmax,
                                  0, 0, st));
        if (h->guarded && split) {
            // ranks the split Gram could not certify: FP64 Gram and eigensolver
            // again for those problems (the others' workgroups exit at once)
            for (const GramLaunch& g : sp.grams)
                if (!g.f64)
                    TK_TRY(launch_gram_f64_batched((const BatchGramTask*)(h->tables_dev + g.off),
                                                   g.ntasks, g.total_wg, g.jb, 1, st));
            TK_TRY(launch_gram_reduce_batched(
                (const BatchReduceTask*)(h->tables_dev + sp.red_off), sp.red_ntasks, sp.red_wg,
                1, st));
            TK_TRY(launch_eig_batched((const EigArgs*)(h->tables_dev + sp.eig_off), h->B,
                                      sp.jmax, 1, 1 << h->order[s], st));
        }
        for (const TtmLaunch& t : sp.ttms)
            TK_TRY(launch_ttm_bf16_batched((const BatchTtmTask*)(h->tables_dev + t.off),
                                           t.ntasks, t.total_wg, t.J, t.kmax,
                                           h->opt.ttm_precision, st));
    }
    return TK_OK;
}

int sthosvd_batch_finish(tk_batch* h, void* stream) {
    if (!h) return fail(TK_ERR_INVALID_ARG, "sthosvd_batch_finish: handle NULL");
    hipStream_t st = (hipStream_t)stream;
    const int B = h->B;
    std::vector<int32_t> status(2 * (size_t)B);
    TK_HIP(hipMemcpyAsync(status.data(), h->status_dev, status.size() * sizeof(int32_t),
                          hipMemcpyDeviceToHost, st));
    TK_HIP(hipStreamSynchronize(st));
    std::vector<double> norm2(B);
    TK_HIP(hipMemcpy(norm2.data(), h->norm2_dev, B * sizeof(double), hipMemcpyDeviceToHost));
    for (int b = 0; b < B; ++b) {
        if (!std::isfinite(norm2[b]))
            return fail(TK_ERR_NONFINITE, "sthosvd_batch: problem %d holds Inf or NaN", b);
        if (status[2 * b] & 2)
            return fail(TK_ERR_CAPACITY, "sthosvd_batch: a rank of problem %d exceeds max_ranks", b);
    }
    return TK_OK;
}

void sthosvd_batch_destroy(tk_batch* h) { delete h; }

}  // extern "C"
