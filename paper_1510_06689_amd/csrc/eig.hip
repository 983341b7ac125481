// FP64 symmetric eigensolver + rank truncation for one J x J Gram matrix
// (Alg. 1, eigenvector and rank steps; Sec. V-D uses a LAPACK subset solver,
// this is the same family of method on one workgroup):
//
//   1. Householder reduction to tridiagonal form T = Q^T S Q.  Each step
//      derives the reflector from the pivot row, forms p = tau A22 v, then
//      applies the rank-2 update A22 -= v w^T + w v^T.  For J <= 128 the
//      matrix lives in registers; otherwise it lives in global scratch and
//      the first J - 128 columns are reduced in panels of eight (the rank-2
//      updates of a panel are kept as vectors in LDS, applied to the pivot
//      rows and to A22 x on the fly and to the trailing block once per
//      panel, as in LAPACK's latrd) before the last 128 x 128 block moves to
//      registers; reflector k is kept in column k below the diagonal and
//      copied to global scratch at the end;
//   2. all eigenvalues of T by multisection: groups of threads per
//      eigenvalue evaluate Sturm counts with the three-term determinant
//      recurrence of T scaled by a power of two (exact), rescaled by 2^+-300
//      every four steps; a ballot picks the sub-interval;
//   3. rank rule R = min R >= 1 with sum_{r>R} max(lambda_r,0) <= eps^2 nu / N
//      (tail sums accumulated smallest first), or a fixed rank;
//   4. the R leading eigenvectors of T by inverse iteration (tridiagonal LU
//      with partial pivoting kept in LDS, reciprocal pivots, two sweeps),
//      in batches that fit in LDS, then modified Gram-Schmidt (twice) inside
//      eigenvalue clusters by one wave;
//   5. back-transformation X <- Q X, one wave per eigenvector with the
//      vector in registers (no barriers), and a sign rule (largest |entry|
//      positive, lowest index on ties), written to the factor output.
// Barriers never wait on global stores inside loops: global memory is only
// written between phases.  One workgroup of 1024 threads, except that from
// J = 64 on step 2 runs in a launch of its own (eig_multisect, one wave per
// eigenvalue) between two launches of the solver; no host sync.
#include <cfloat>
#include <type_traits>

#include "tk_common.hpp"

namespace tk {

constexpr int kEigThreads = 1024;
constexpr int kEigWaves = kEigThreads / 64;
constexpr int kInvIters = 2;
constexpr int kPanel = 8;  // columns per panel of the global-memory reduction
constexpr int kLuArrays = 6;  // u0 (reciprocal), u1, u2, multiplier, pivot flag, x
constexpr int kMaxVecSlots = TK_MAX_MODE_DIM / 64;  // per-lane elements of one vector
constexpr int kSweepRows = 4;  // rows per block of the inverse-iteration sweeps

// Rows of the inverse-iteration arrays: J padded to whole sweep blocks.
__host__ __device__ constexpr int eig_sweep_rows(int J) {
    return (J + kSweepRows - 1) / kSweepRows * kSweepRows;
}

// Moves a double across lanes with one DPP pattern (applied to both 32-bit
// halves); lanes the pattern does not write receive 0.
template <int CTRL, int ROW_MASK, bool BOUND_CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const long long bits = __double_as_longlong(v);
    int lo = (int)(bits & 0xffffffffll), hi = (int)(bits >> 32);
    lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROW_MASK, 0xf, BOUND_CTRL);
    hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROW_MASK, 0xf, BOUND_CTRL);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Calls f(std::integral_constant<int, I>) for I = B .. E - 1 in order.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

__device__ __forceinline__ double read_lane(double v, int lane) {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes of a wave, in a fixed order, returned to every lane.
// Row prefix sums by row_shr 1, 2, 4, 8 leave each 16-lane row's total in its
// lane 15; row_bcast 15 and 31 then carry the row totals into lane 63.  Must
// be called with all lanes active.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_move<0x111, 0xf, true>(v);   // row_shr:1
    v += dpp_move<0x112, 0xf, true>(v);   // row_shr:2
    v += dpp_move<0x114, 0xf, true>(v);   // row_shr:4
    v += dpp_move<0x118, 0xf, true>(v);   // row_shr:8
    v += dpp_move<0x142, 0xa, false>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_move<0x143, 0xc, false>(v);  // row_bcast:31 into rows 2 and 3
    return read_lane(v, 63);
}

// 1/q from the hardware reciprocal refined by one Newton step.
__device__ __forceinline__ double recip(double q) {
    double r = __builtin_amdgcn_rcp(q);
    double err = fma(-q, r, 1.0);
    return fma(r, err, r);
}

// 1/sqrt(s) (s > 0 finite) from the hardware estimate refined by two Newton
// steps r <- r + r (1 - s r^2) / 2.
__device__ __forceinline__ double rsq(double s) {
    double r = __builtin_amdgcn_rsq(s);
    double err = fma(-(s * r), r, 1.0);
    r = fma(0.5 * r, err, r);
    err = fma(-(s * r), r, 1.0);
    return fma(0.5 * r, err, r);
}

// Deterministic start vector entry in [-1, 1) for inverse iteration: the
// pair (a, b) goes through SplitMix64's golden-ratio increment and its
// published 64-bit finaliser (Steele, Lea and Flood, 2014).
__device__ __forceinline__ double hash_unit(uint32_t a, uint32_t b) {
    uint64_t z = ((uint64_t)a << 32) ^ (uint64_t)b ^ 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;  // [-1, 1)
}

size_t eig_scratch_doubles(int J) {
    // A (J*J, used when J > 128) + reflectors H (J*J)
    return (size_t)2 * J * J + 64;
}

// small per-matrix arrays + the [C][rb] partial sums of the tridiagonal step
static size_t eig_small_doubles(int J) { return (size_t)10 * J + 64 + 8 + (size_t)kEigThreads; }

// LDS doubles for the matrix (J <= 128) and later the inverse-iteration
// batch; region + small arrays stay within the 160 KB of LDS.
static size_t eig_region_doubles(int J) {
    const size_t lds_doubles = 160 * 1024 / sizeof(double);
    size_t cap = lds_doubles - eig_small_doubles(J) - 128;
    if (cap > 16384) cap = 16384;                 // J <= 128 also holds A here (J*J <= 16384)
    // room for every vector in one batch: a record of kLuArrays values per
    // padded row plus one, and two scale factors, per vector
    const size_t want = ((size_t)kLuArrays * eig_sweep_rows(J) + 3) * J;
    return want < cap ? want : cap;
}

// Number of eigenvalues of the (scaled) tridiagonal matrix below x: sign
// changes along the leading principal minors
//   p_0 = 1,  p_i = (d_i - x) p_{i-1} - e_{i-1}^2 p_{i-2}.
// An exactly zero minor is replaced by +2^-600: over that step and the next
// one the number of sign changes is the same whichever sign a zero takes (it
// is one), a zero last minor (x an eigenvalue) is correctly not counted, and
// a zero followed by e_i = 0 restarts the next block from a tiny value.  The
// pair (p_{i-1}, p_i) is rescaled by 2^+-300 every four steps (exact).
__device__ __forceinline__ int sturm_count(const double* __restrict__ ds,
                                           const double* __restrict__ e2s, int J, double x) {
    constexpr double kUp = 0x1p300, kDown = 0x1p-300, kZero = 0x1p-600;
    double p0 = 1.0, p1 = ds[0] - x;
    p1 = p1 == 0.0 ? kZero : p1;
    bool neg = p1 < 0.0;
    int c = (int)neg;
    auto step = [&](double di, double ei2) {
        double p2 = fma(di - x, p1, -ei2 * p0);
        p2 = p2 == 0.0 ? kZero : p2;
        const bool n2 = p2 < 0.0;
        c += (int)(n2 != neg);
        neg = n2;
        p0 = p1;
        p1 = p2;
    };
    int i = 1;
    for (; i + 3 < J; i += 4) {  // four steps per trip: the eight loads go out together
        const double d0 = ds[i], d1 = ds[i + 1], d2 = ds[i + 2], d3 = ds[i + 3];
        const double f0 = e2s[i - 1], f1 = e2s[i], f2 = e2s[i + 1], f3 = e2s[i + 2];
        step(d0, f0);
        step(d1, f1);
        step(d2, f2);
        step(d3, f3);
        const double mg = fmax(fabs(p0), fabs(p1));
        const double f = mg > kUp ? kDown : (mg < kDown ? kUp : 1.0);
        p0 *= f;
        p1 *= f;
    }
    for (; i < J; ++i) step(ds[i], e2s[i - 1]);
    return c;
}

// Sum over the 8 consecutive lanes of a row group (every lane gets the same
// bits: each step adds the same two values in either order).
__device__ __forceinline__ double row8_sum(double v) {
    v += dpp_move<0xb1, 0xf, false>(v);   // quad_perm [1,0,3,2]
    v += dpp_move<0x4e, 0xf, false>(v);   // quad_perm [2,3,0,1]
    v += dpp_move<0x141, 0xf, false>(v);  // row_half_mirror
    return v;
}

// Sum over the 16 lanes of a row (every lane gets the same bits).
__device__ __forceinline__ double row16_sum(double v) {
    v = row8_sum(v);
    v += dpp_move<0x140, 0xf, false>(v);  // row_mirror
    return v;
}

// Householder tridiagonalisation of a symmetric Jr x Jr block held in
// registers (Jr <= JP): element (i, j) of the block is src[i + ld j].  Its
// diagonal, off-diagonal and reflector scalars go to d, e, beta at offset
// koff, and reflector koff + k (length Jr - k - 1) to H[(koff + k) J ..].
// With koff = 0, Jr = J this is the whole reduction; with koff > 0 it
// finishes one whose first koff steps ran on the matrix in global memory.
template <int JP>
__device__ __forceinline__ void tridiag_regs(const double* __restrict__ src, int ld, int Jr,
                                             int koff, int J, double* reg, double* red,
                                             double* d, double* e, double* beta, double* H) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // ---- 1. Householder tridiagonalisation, A in registers ---------------
    // Thread t owns row i = t / 8 and the columns j = t % 8 + 8 q.  Per column
    // k: the owners of row k form the reflector and publish v; (A22 v)_i is a
    // sum over the row's 8 lanes and p = tau A22 v is published; each thread
    // then updates its own elements.  Vectors alternate between two LDS
    // buffers so that two barriers per column suffice; reflectors collect in
    // LDS and go to the global scratch once at the end.
    constexpr int NQ = JP / 8;
    const int ri = tid >> 3, rc = tid & 7;
    const bool rowok = ri < Jr;
    double av[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int j = rc + 8 * q;
        av[q] = (rowok && j < Jr) ? src[ri + (size_t)ld * j] : 0.0;
    }
    double* Hs = reg;
    constexpr int NS = (JP + 63) / 64;  // per-lane slots of a wave-wide reduction
    // Every load below stays inside the reflector store (zeroed first, so
    // that entries no step writes are exact zeros: reflector k is written
    // from column k + 1 on) and four JP-long vector buffers in the
    // 1024-double area after misc (zeroed too; the global-A path alone uses
    // it otherwise).  Finished rows and columns see v = p = 0, so the
    // register loops need no masks.  Each column reads v and p from LDS by
    // every row, which bounds the step: from block KEEP on v, and from KEEP2
    // on p, stay in registers between the matrix-vector product and the
    // update (the live chunks shrink with the block index).
    static_assert(4 * JP <= kEigThreads, "vector buffers must fit the partial-sum area");
    double* vbuf = red + 64 + 8;
    for (int i = tid; i < 4 * JP; i += kEigThreads) vbuf[i] = 0.0;
    for (int i = tid; i < (Jr > 2 ? Jr - 2 : 0) * JP; i += kEigThreads) Hs[i] = 0.0;
    __syncthreads();
    // Columns run in blocks of eight, the block index KB a compile-time
    // constant: chunks below KB are finished for every column of the block
    // (their v and p are zero), so each loop starts at chunk KB with no test,
    // and only chunks KB and KB + 1 can hold the pivot column k + 1.
    static_for<0, NQ>([&](auto kbc) {
        constexpr int KB = decltype(kbc)::value;
        const int kend = min(8 * KB + 8, Jr - 2);
        for (int k = 8 * KB; k < kend; ++k) {
            double* vs = Hs + (size_t)k * JP;        // v = reflector k: v_{k+1} = 1, zero outside k < j < Jr
            double* ps = vbuf + (2 + (k & 1)) * JP;  // p = tau A22 v, zero outside k < i < Jr
            double* sg = red + 40 + (k & 1);         // tau of column k
            // The row index goes through an empty asm so that the compiler
            // cannot use ri == k to replace the uniform k by the per-lane ri
            // inside the owner branch (that turns every column test below
            // into a per-lane mask held across the loop).
            int ri_k = ri;
            asm volatile("" : "+v"(ri_k));
            if (ri_k == k) {
                // The owners of row k (= column k, x = its part beyond the
                // diagonal) form the reflector alone, in the form of LAPACK's
                // dlarfg: alpha = -sign(x_0) |x|, tau = 1 + |x_0| / |x|,
                // v = x / (x_0 - alpha) (one reciprocal square root and one
                // reciprocal), and publish v.
                double sq[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int q = KB; q < NQ; ++q) {
                    const double m = (q > KB + 1 || rc + 8 * q >= k + 2) ? av[q] : 0.0;
                    sq[q & 3] = fma(m, m, sq[q & 3]);
                }
                const double sigma = row8_sum((sq[0] + sq[1]) + (sq[2] + sq[3]));
                // a_kk and a_k,k+1 from the lanes of row k that hold them:
                // column k lies in chunk KB, column k + 1 in KB or KB + 1
                const int l0 = 8 * (k & 7);
                const double akk = read_lane(av[KB], l0 + (k & 7));
                const double x0 = read_lane(((k + 1) >> 3) == KB ? av[KB] : av[KB + 1 < NQ ? KB + 1 : KB],
                                            l0 + ((k + 1) & 7));
                double tau = 0.0, alpha = x0, inv_v0 = 0.0;
                if (sigma != 0.0) {
                    const double ss = fma(x0, x0, sigma);
                    const double r = rsq(ss);  // 1 / |x|
                    const double mu = ss * r;
                    const double sgn = x0 < 0.0 ? -1.0 : 1.0;
                    alpha = -sgn * mu;
                    tau = fma(fabs(x0), r, 1.0);
                    inv_v0 = sgn * recip(fabs(x0) + mu);
                }
#pragma unroll
                for (int q = KB; q < NQ; ++q) {
                    const int j = rc + 8 * q;
                    const double vj = av[q] * inv_v0;  // av is 0 beyond Jr
                    vs[j] = q > KB + 1 ? vj : (j == k + 1 ? 1.0 : (j > k + 1 ? vj : 0.0));
                }
                if (rc == 0) {
                    *sg = tau;
                    d[koff + k] = akk;
                    e[koff + k] = alpha;
                    beta[koff + k] = tau;
                }
            }
            __syncthreads();
            const double tau = *sg;
            // A wave whose 8 rows are all <= k has nothing to form or update (uniform).
            const bool wact = 8 * wave + 7 > k;
            double part = 0.0;
            constexpr int KEEP = 2, KEEP2 = 4;
            double vq[NQ];
            if (wact) {  // formed before tau is tested, so that v's loads do not wait for it
                double pr[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int q = KB; q < NQ; ++q) {
                    vq[q] = vs[rc + 8 * q];
                    pr[q & 3] = fma(av[q], vq[q], pr[q & 3]);
                }
                part = row8_sum((pr[0] + pr[1]) + (pr[2] + pr[3]));  // (A22 v)_i
            }
            if (tau == 0.0) continue;  // uniform: the reflector is the identity
            if (rc == 0 && ri < JP) ps[ri] = (wact && ri > k && rowok) ? tau * part : 0.0;
            __syncthreads();
            if (!wact) continue;  // uniform over the wave; it still meets every barrier
            // A22 -= v w^T + w v^T with w = p - (tau/2)(p.v) v, two fused
            // multiply-adds per element; entries outside the trailing block
            // see v = w = 0.  Every lane forms p.v with the same bits (from
            // KEEP2 on as a sum over its row's 8 lanes, all rows holding the
            // same values).  The update rounds a_ij and a_ji differently, so
            // A is symmetric up to rounding; only each row's own elements are
            // ever read, so the reduction is that of a matrix within rounding
            // of the exact iterate.
            double pq[NQ];
            double half;
            if constexpr (KB >= KEEP2) {
                double pr2[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int q = KB; q < NQ; ++q) {
                    pq[q] = ps[rc + 8 * q];
                    pr2[q & 3] = fma(pq[q], vq[q], pr2[q & 3]);
                }
                half = 0.5 * tau * row8_sum((pr2[0] + pr2[1]) + (pr2[2] + pr2[3]));
            } else {
                double pv = 0.0;
#pragma unroll
                for (int r = 0; r < NS; ++r) {
                    const int j = lane + 64 * r;
                    if (j < JP) pv = fma(ps[j], vs[j], pv);
                }
                half = 0.5 * tau * wave_sum(pv);
            }
            const int ric = ri < JP ? ri : 0;
            const double vi = vs[ric], wi = fma(-half, vi, ps[ric]);
#pragma unroll
            for (int q = KB; q < NQ; ++q) {
                double vj;
                if constexpr (KB >= KEEP) vj = vq[q];
                else vj = vs[rc + 8 * q];
                double pj;
                if constexpr (KB >= KEEP2) pj = pq[q];
                else pj = ps[rc + 8 * q];
                const double wj = fma(-half, vj, pj);
                av[q] = fma(-wi, vj, fma(-vi, wj, av[q]));
            }
        }
    });
    // the trailing 2 x 2 block (or 1 x 1)
    if (ri >= Jr - 2 && rowok) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int j = rc + 8 * q;
            if (j == ri) d[koff + ri] = av[q];
            if (ri == Jr - 2 && j == Jr - 1) e[koff + Jr - 2] = av[q];
        }
    }
    if (tid == 0) {
        if (Jr >= 2) beta[koff + Jr - 2] = 0.0;
        e[koff + Jr - 1] = 0.0;
        beta[koff + Jr - 1] = 0.0;
    }
    __syncthreads();
    // reflector koff + k has length J - (koff + k) - 1 = Jr - k - 1
    for (int idx = tid; idx < (Jr - 2) * Jr; idx += kEigThreads) {
        const int k = idx / Jr, i = idx - k * Jr;
        if (i < Jr - k - 1) H[(size_t)(koff + k) * J + i] = Hs[(size_t)k * JP + k + 1 + i];
    }
    __syncthreads();
}

// Hand-off area of a split solve (6 J + 4 doubles): the start of the
// scratch (A's area, J x J, unused or dead once step 1 is done) when it fits,
// else the 64 spare doubles behind the reflectors (J <= 6).
__host__ __device__ inline double* eig_handoff(double* scratch, int J) {
    return 6 * J + 4 <= J * J ? scratch : scratch + (size_t)2 * J * J;
}

// JP = 32, 64, 128: A lives in registers during the tridiagonalisation
// (J <= JP); JP = 0: A lives in the global scratch (J > 128).
// PH = 0: the whole solver in one launch.  PH = 1: steps 1 and the scaling of
// T, then T, beta and the bounds go to the hand-off area (the first 6 J + 4
// doubles of the scratch, A's area, unused or free by then) and the launch
// ends; eig_multisect then finds the eigenvalues with one workgroup each and
// PH = 3 picks everything up for steps 3 to 5.
template <int JP, int PH>
__device__ __forceinline__ void eig_body(const EigArgs& a, int region) {
    extern __shared__ double smem[];
    const int J = a.J;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double* reg = smem;                        // A (J <= 128) then the LU batch
    double* sv = smem + region;
    double* d = sv;              // J
    double* e = d + J;           // J
    double* e2 = e + J;          // J (scaled)
    double* beta = e2 + J;       // J
    double* pw = beta + J;       // J: A22 x
    double* lam = pw + J;        // J (descending)
    double* shift = lam + J;     // J
    double* dots = shift + J;    // J: v during step 1, scaled d during step 2
    double* colv = dots + J;     // J: w during step 1
    double* red = colv + J;      // 64
    int* misc = (int*)(red + 64);  // [0] = R
    double* H = a.scratch + (size_t)J * J;    // reflector k at H[k * J], length J - k - 1
    double* X = a.u;                          // column-major J x R
    double* ho = eig_handoff(a.scratch, J);   // hand-off between split launches
    double sc, tnorm;
    // the rank rule's global inputs, loaded now so that their latency
    // overlaps the earlier phases
    double nu_in = 0.0, stat_d2 = 0.0, stat_e = 0.0;
    if constexpr (PH != 1) {
        if (tid == 0) {
            if (a.fixed_rank <= 0) nu_in = *a.nu;
            if (a.guard > 0.0 && a.split_stats) {
                stat_d2 = a.split_stats[0];
                stat_e = a.split_stats[1];
            }
        }
    }

    if constexpr (PH != 3) {
    if constexpr (JP > 0) {
    // ---- 1. Householder tridiagonalisation, A in registers ---------------
    tridiag_regs<JP>(a.s, J, J, 0, J, reg, red, d, e, beta, H);
    } else {
    double* A = a.scratch;  // row-major J x J

    // ---- load S (symmetric) -------------------------------------------
    for (int idx = tid; idx < J * J; idx += kEigThreads) A[idx] = a.s[idx];
    __syncthreads();

    // ---- 1. Householder tridiagonalisation ------------------------------
    // Column-chunked matrix-vector product: thread t owns row i = t % RB of
    // A22 and the columns j = c, c + C, ... with c = t / RB; the C partials
    // of each row are added in a fixed order by whoever needs them.
    int rb = 32;
    while (rb < J) rb *= 2;
    const int C = kEigThreads / rb;  // chunks per row
    const int mi = tid % rb, mc = tid / rb;
    double* part = red + 64 + 8;  // [C][rb] = kEigThreads partial sums, after misc
    double* pp = colv;                                    // p
    double* vv = dots;                                    // v
    // Once the trailing block is 128 x 128 it moves to registers and the
    // register path finishes the reduction (when the LDS region can hold
    // its 126 reflectors at pitch 128).
    const bool hybrid = J > 128 && region >= 126 * 128;
    const int kend = hybrid ? J - 128 : J - 2;
    // Panels of kPanel columns (LAPACK's latrd scheme): inside a panel A keeps
    // its values from the panel start, and column q of the panel leaves
    // v_q and w_q = p_q - (kc_q) v_q in LDS (Vs, Ws), so that the matrix the
    // reduction has reached is A - sum_q (v_q w_q^T + w_q v_q^T).  Row k and
    // row k + 1 are corrected by those terms, A22 x is formed from the panel
    // start's A22 and corrected by V (W^T x) + W (V^T x); after the panel the
    // trailing block takes all of its rank-2 updates in one pass, in a
    // commutative form so that A stays exactly symmetric.  A22 is read once
    // per column and written once per panel.
    double* Vs = reg;              // [kPanel][J], indexed by row of A
    double* Ws = reg + kPanel * J;
    double* xs = lam;              // corrected row k (columns k + 1 ..)
    double* a0s = shift;           // corrected row k + 1 (columns k + 1 ..)
    for (int k0 = 0; k0 < kend; k0 += kPanel) {
        const int nq = min(kPanel, kend - k0);
        for (int c = 0; c < nq; ++c) {
            const int k = k0 + c, m = J - k - 1;
            for (int j = tid; j < m; j += kEigThreads) {
                const int g = k + 1 + j;
                double xv = A[(size_t)k * J + g], av = A[(size_t)(k + 1) * J + g];
                for (int q = 0; q < c; ++q) {
                    const double vg = Vs[q * J + g], wg = Ws[q * J + g];
                    xv -= Vs[q * J + k] * wg + Ws[q * J + k] * vg;
                    av -= Vs[q * J + k + 1] * wg + Ws[q * J + k + 1] * vg;
                }
                xs[j] = xv;
                a0s[j] = av;
            }
            __syncthreads();
            // A22 x with the panel start's A22 (read column i so that a
            // wave's loads are contiguous)
            {
                double acc = 0.0;
                if (mi < m) {
#pragma unroll 8
                    for (int j = mc; j < m; j += C)
                        acc += A[(size_t)(k + 1 + j) * J + (k + 1 + mi)] * xs[j];
                }
                part[mc * rb + mi] = acc;
            }
            // red[q] = v_q . x, red[c + q] = w_q . x (one wave each)
            if (wave < 2 * c) {
                const double* vec = wave < c ? Vs + wave * J : Ws + (wave - c) * J;
                double sdot = 0.0;
                for (int j = lane; j < m; j += 64) sdot += vec[k + 1 + j] * xs[j];
                sdot = wave_sum(sdot);
                if (lane == 0) red[wave] = sdot;
            }
            double sq = 0.0;
            for (int j = 1 + lane; j < m; j += 64) sq += xs[j] * xs[j];
            const double sigma = wave_sum(sq);  // same bits in every wave
            const double x0 = xs[0];
            double b, mu, v0;
            if (sigma == 0.0) {
                b = 0.0;
                mu = x0;
                v0 = 1.0;
            } else {
                mu = sqrt(x0 * x0 + sigma);
                v0 = (x0 <= 0.0) ? x0 - mu : -sigma / (x0 + mu);
                b = 2.0 * v0 * v0 / (sigma + v0 * v0);
            }
            const double inv_v0 = 1.0 / v0;
            if (tid == 0) {
                double dk = A[(size_t)k * J + k];
                for (int q = 0; q < c; ++q) {
                    const double vk = Vs[q * J + k], wk = Ws[q * J + k];
                    dk -= vk * wk + wk * vk;
                }
                d[k] = dk;
                e[k] = mu;
                beta[k] = b;
            }
            __syncthreads();
            // v = (x - mu e_1) / v0, so p = b A22 v = b (A22 x - mu A22 e_1) / v0
            // with A22 e_1 = row k + 1.  Every wave forms kc2 = b p.v from the
            // partials itself (same order, same bits); wave 0 keeps p, v.
            double pv = 0.0;
            for (int j = lane; j < m; j += 64) {
                double wj = 0.0;
#pragma unroll 8
                for (int cc = 0; cc < C; ++cc) wj += part[cc * rb + j];
                for (int q = 0; q < c; ++q)
                    wj -= Vs[q * J + k + 1 + j] * red[c + q] + Ws[q * J + k + 1 + j] * red[q];
                const double pj = b * (wj - mu * a0s[j]) * inv_v0;
                const double vj = j == 0 ? 1.0 : xs[j] * inv_v0;
                pv += pj * vj;
                if (wave == 0) {
                    pp[j] = pj;
                    vv[j] = vj;
                }
            }
            const double kc2 = b * wave_sum(pv);  // 2 kc
            if (wave == 0) {
                // v p^T + p v^T - 2 kc v v^T = v w^T + w v^T with w = p - kc v;
                // b = 0 leaves v = w = 0 (no reflection).  Lane j reads the
                // pp, vv entries it wrote itself.
                for (int j = lane; j < m; j += 64) {
                    const double vj = b != 0.0 ? vv[j] : 0.0;
                    const double wj = b != 0.0 ? pp[j] - 0.5 * kc2 * vv[j] : 0.0;
                    Vs[c * J + k + 1 + j] = vj;
                    Ws[c * J + k + 1 + j] = wj;
                    // the reflector goes below the diagonal of column k
                    if (b != 0.0) A[(size_t)(k + 1 + j) * J + k] = vj;
                }
            }
            __syncthreads();
        }
        // trailing block (rows and columns from k0 + nq) takes the panel's
        // updates: thread t owns columns t % 256 (+ 256) and rows t / 256 + 4 i
        const int t0 = k0 + nq, mt = J - t0;
        const int jc = tid & 255, ir = tid >> 8;
        for (int jb = jc; jb < mt; jb += 256) {
            double vj[kPanel], wj[kPanel];
#pragma unroll
            for (int q = 0; q < kPanel; ++q) {
                vj[q] = q < nq ? Vs[q * J + t0 + jb] : 0.0;
                wj[q] = q < nq ? Ws[q * J + t0 + jb] : 0.0;
            }
            // rows in batches of UR whose loads go out together (a row's
            // store would otherwise hold back the next row's load: the
            // compiler cannot tell the addresses apart); each element has
            // one owner, so the values are those of a row-by-row pass
            constexpr int UR = 4;
            for (int i0 = ir; i0 < mt; i0 += 4 * UR) {  // uniform over the wave
                double av[UR];
#pragma unroll
                for (int u = 0; u < UR; ++u) {
                    const int i = min(i0 + 4 * u, mt - 1);  // in bounds; unused past mt
                    av[u] = A[(size_t)(t0 + i) * J + t0 + jb];
                }
#pragma unroll
                for (int u = 0; u < UR; ++u) {
                    const int i = i0 + 4 * u;
                    if (i >= mt) break;  // uniform over the wave
                    double t = 0.0;
#pragma unroll
                    for (int q = 0; q < kPanel; ++q) {
                        if (q < nq) {
                            const double vi = Vs[q * J + t0 + i], wi = Ws[q * J + t0 + i];
                            t = __dadd_rn(t, __dadd_rn(__dmul_rn(vi, wj[q]), __dmul_rn(wi, vj[q])));
                        }
                    }
                    A[(size_t)(t0 + i) * J + t0 + jb] = av[u] - t;
                }
            }
        }
        __syncthreads();
    }
    if (tid == 0 && !hybrid) {
        if (J >= 2) {
            d[J - 2] = A[(size_t)(J - 2) * J + (J - 2)];
            e[J - 2] = A[(size_t)(J - 2) * J + (J - 1)];
            beta[J - 2] = 0.0;
        }
        d[J - 1] = A[(size_t)(J - 1) * J + (J - 1)];
        e[J - 1] = 0.0;
        beta[J - 1] = 0.0;
    }
    // reflectors to global scratch: the LDS region is reused from step 4 on
    for (int idx = tid; idx < kend * J; idx += kEigThreads) {
        const int k = idx / J, i = idx - k * J;
        if (i < J - k - 1) H[idx] = A[(size_t)(k + 1 + i) * J + k];
    }
    __syncthreads();
    if (hybrid) tridiag_regs<128>(A + (size_t)kend * J + kend, J, 128, kend, J, reg, red, d, e,
                                  beta, H);
    }
    if (tid == 0) {
        double gl = DBL_MAX, gu = -DBL_MAX;
        for (int i = 0; i < J; ++i) {
            double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < J ? fabs(e[i]) : 0.0);
            gl = fmin(gl, d[i] - r);
            gu = fmax(gu, d[i] + r);
        }
        const double tnorm = fmax(fabs(gl), fabs(gu));
        // scale T by a power of two so that |entries| <= 1 (exact)
        int ex = 0;
        frexp(tnorm > 0.0 ? tnorm : 1.0, &ex);
        const double sc = ldexp(1.0, -ex);
        // widen slightly so that count(gl) = 0 and count(gu) = J hold exactly
        red[32] = (gl - 2.0 * DBL_EPSILON * tnorm * J) * sc - 0x1p-900;
        red[33] = (gu + 2.0 * DBL_EPSILON * tnorm * J) * sc + 0x1p-900;
        red[34] = sc;
        red[35] = tnorm;
    }
    __syncthreads();
    sc = red[34];
    tnorm = red[35];
    double* ds = dots;  // scaled diagonal
    for (int i = tid; i < J; i += kEigThreads) {
        ds[i] = d[i] * sc;
        e2[i] = (e[i] * sc) * (e[i] * sc);
    }
    __syncthreads();
    if constexpr (PH == 1) {
        for (int i = tid; i < J; i += kEigThreads) {
            ho[i] = d[i];
            ho[J + i] = e[i];
            ho[2 * J + i] = beta[i];
            ho[3 * J + i] = ds[i];
            ho[4 * J + i] = e2[i];
        }
        if (tid < 4) ho[5 * J + tid] = red[32 + tid];  // gl, gu, sc, tnorm
        return;
    }

    // ---- 2. eigenvalues by multisection ---------------------------------
    {
        const double gl = red[32], gu = red[33];
        int jp = 32;
        while (jp < J) jp *= 2;
        // about 512 active lanes (two waves per SIMD): more sample points per
        // eigenvalue add work faster than they remove iterations
        const int tpe = jp >= 512 ? 1 : 512 / jp;  // threads (sample points) per eigenvalue
        const int k = tid / tpe, s = tid - (tid / tpe) * tpe;
        const int gofs = (lane / tpe) * tpe;
        const uint64_t gmask = (((1ull << tpe) - 1ull) << gofs);
        (void)wave;
        const double atol = 2.0 * DBL_EPSILON;  // T is scaled to norm <= 1
        double lo = gl, hi = gu;
        if (k < J) {
            for (int it = 0; it < 160; ++it) {
                const double tol = fmax(atol, 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)));
                if (hi - lo <= tol) break;
                const double h = (hi - lo) / (double)(tpe + 1);
                const int c = sturm_count(ds, e2, J, lo + h * (double)(s + 1));
                const uint64_t bal = __ballot(c > k) & gmask;
                const int sstar = bal ? (__ffsll((long long)bal) - gofs) : tpe + 1;  // 1-based point
                const double nlo = sstar == 1 ? lo : lo + h * (double)(sstar - 1);
                const double nhi = sstar == tpe + 1 ? hi : lo + h * (double)sstar;
                lo = nlo;
                hi = nhi;
            }
            if (s == 0) lam[J - 1 - k] = 0.5 * (lo + hi) / sc;
        }
    }
    __syncthreads();
    } else {
        for (int i = tid; i < J; i += kEigThreads) {
            d[i] = ho[i];
            e[i] = ho[J + i];
            beta[i] = ho[2 * J + i];
            lam[i] = ho[5 * J + 4 + i];
        }
        sc = ho[5 * J + 2];
        tnorm = ho[5 * J + 3];
        __syncthreads();
    }
    (void)sc;
    // Jordan-Wielandt input: the leading half of the spectrum is sigma(R)
    const int Jv = a.aug ? J / 2 : J;
    // Tail sums: negative rounding eigenvalues count as 0 -- except for a
    // split Gram, whose subtracted quantization energy leaves small negative
    // eigenvalues in noise-level directions; there the raw sum is the
    // estimate of the exact tail (clamping would raise it).
    const bool raw = a.guard > 0.0 && a.split_stats != nullptr && !a.aug;
    auto val = [&](int r) {
        const double l = raw ? lam[r] : fmax(lam[r], 0.0);
        return a.aug ? l * l : l;
    };
    // the values of the tail sums, formed in parallel (pw is free after step 1)
    double* vals = pw;
    for (int i = tid; i < Jv; i += kEigThreads) {
        const double v = val(i);
        vals[i] = v;
        a.lambda[i] = a.aug ? v : lam[i];
    }
    __syncthreads();

    // ---- 3. rank rule ---------------------------------------------------
    if (tid == 0) {
        int R;
        double tail = 0.0;
        const bool eps_rule = a.fixed_rank <= 0;
        const double tau = eps_rule ? a.eps2_over_n * nu_in : 0.0;
        if (!eps_rule) {
            R = a.fixed_rank < Jv ? a.fixed_rank : Jv;
            for (int r = Jv - 1; r >= R; --r) tail += vals[r];
        } else {
            // R = Jv; while (R > 1 && tail + val(R - 1) <= tau) tail += val(--R),
            // with the values loaded eight at a time ahead of the running sum
            R = Jv;
            bool more = true;
            double vb[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) vb[u] = vals[max(R - 1 - u, 0)];  // unused past r = 1
            while (more) {
                double nb8[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) nb8[u] = vals[max(R - 9 - u, 0)];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const double t = tail + vb[u];
                    more = more && R > 1 && t <= tau;
                    tail = more ? t : tail;
                    R -= more ? 1 : 0;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) vb[u] = nb8[u];
            }
        }
        double bound = 0.0;
        if (a.guard > 0.0 && a.split_stats) {
            // The cut must survive the split representation's error in the
            // tail sums (EigArgs::guard): a model standard deviation at each
            // side, sqrt(4 delta^2 t + 2 K delta^4 (J - r)) for the tail t
            // beyond rank r.  R = J discards nothing and is exact.
            const double d2 = stat_d2;
            const double dl2 = ldexp(1.0, 2 * ((int)stat_e - 16)) / 3.0;
            auto margin = [&](double t, int r) {
                return a.guard * sqrt(4.0 * dl2 * t + 2.0 * a.ncols * dl2 * dl2 * (double)(Jv - r)) +
                       kSplitModelError * d2;
            };
            const double next = tail + val(R - 1);
            bound = R == Jv ? 0.0 : margin(fmax(tail, 0.0), R);
            if (eps_rule) {
                const bool below = tau - tail >= bound;
                const bool above = R == 1 || next - tau >= margin(fmax(next, 0.0), R - 1);
                if (!(below && above)) a.flags[0] |= 4;
            }
        }
        if (a.tail_bound) *a.tail_bound = bound;
        int flag = 0;
        if (R > a.max_rank) {
            flag |= 2;
            R = a.max_rank;
        }
        *a.rank_out = R;
        *a.disc_out = fmax(tail, 0.0);
        if (flag) a.flags[0] |= flag;  // single writer: thread 0 of the only workgroup
        misc[0] = R;
        // shifts for inverse iteration: separate (near-)equal eigenvalues
        const double pert = 10.0 * DBL_EPSILON * tnorm;
        double prev = 0.0;
        for (int j0 = 0; j0 < R; j0 += 8) {
            double lb[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) lb[u] = lam[min(j0 + u, R - 1)];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int j = j0 + u;
                if (j < R) {
                    double sj = lb[u];
                    if (j > 0 && prev - sj < pert) sj = prev - pert;
                    shift[j] = sj;
                    prev = sj;
                }
            }
        }
    }
    __syncthreads();
    const int R = misc[0];


    // ---- 4. inverse iteration, batches of vectors held in LDS -----------
    // One thread per vector runs the recurrences on a record of its own in
    // LDS: row i holds (x, reciprocal pivot, u1, u2, multiplier, pivot flag)
    // at rec[kLuArrays i ..], so every access is the thread's base plus an
    // immediate offset; the record's last double is x of row Jb (zero), and
    // records are an odd number of doubles apart, which keeps the lanes of a
    // wave in distinct banks.  Loads are never conditional (a guarded load
    // waits for its value inside the guard).  Operands are read a block
    // of kSweepRows rows ahead of the recurrence (a load that follows a store
    // to the same record waits for it), and rows are padded to whole blocks
    // with exact zeros, which every sweep maps to zeros.  A sweep's
    // normalisation is applied when the next sweep (or the copy-out) reads
    // its result, with the same two roundings as an in-place pass.
    const double tiny = DBL_EPSILON * tnorm + DBL_MIN;
    const int Jb = eig_sweep_rows(J);
    const int recd = kLuArrays * Jb + 1;  // doubles per record
    const int batch = (int)((size_t)region / ((size_t)recd + 2));
    constexpr int oX = 0, oRP = 1, oU1 = 2, oU2 = 3, oLM = 4, oPV = 5;
    for (int j0 = 0; j0 < R; j0 += batch) {
        const int nb = min(batch, R - j0);
        double* SC1 = reg + (size_t)recd * nb;  // nb: pending scale factors of x
        double* SC2 = SC1 + nb;
        __syncthreads();  // the region is free (A or the previous batch)
        // deterministic start vectors, zero in the padding rows and row Jb
        for (int idx = tid; idx < (Jb + 1) * nb; idx += kEigThreads) {
            const int jj = idx / (Jb + 1), i = idx - jj * (Jb + 1);
            reg[(size_t)jj * recd + kLuArrays * i + oX] =
                i < J ? hash_unit((uint32_t)(j0 + jj), (uint32_t)i) : 0.0;
        }
        __syncthreads();
        if (tid < nb) {
            constexpr int IB = kSweepRows;
            constexpr int W = kLuArrays;
            const int jj = tid, j = j0 + tid;
            double* rec = reg + (size_t)jj * recd;
            // Row i0 of the record.  The offset goes through an empty asm so
            // that each block forms one address and reaches its rows by
            // immediate offsets (the compiler otherwise keeps one address per
            // row and field across the sweep loops).
            auto row = [&](int i0) {
                int o = W * i0;
                asm volatile("" : "+s"(o));
                return rec + o;
            };
            const double sg = shift[j];
            const double rtiny = recip(tiny);  // recip(-tiny) = -recip(tiny) exactly
            // LU factorisation of T - sg I with partial pivoting
            double ai = d[0] - sg, bi = (J > 1) ? e[0] : 0.0;
            for (int i0 = 0; i0 + 1 < J; i0 += IB) {
                double cb[IB], anb[IB], bnb[IB];
#pragma unroll
                for (int u = 0; u < IB; ++u) {
                    const int i = min(i0 + u, J - 2);
                    cb[u] = e[i];
                    anb[u] = d[i + 1] - sg;
                    const double en = e[i + 1];
                    bnb[u] = (i + 2 < J) ? en : 0.0;
                }
                double* rr = row(i0);
#pragma unroll
                for (int u = 0; u < IB; ++u) {
                    if (i0 + u + 1 < J) {  // uniform
                        // Without interchange (|a_i| >= |c_i|) the pivot is a_i,
                        // raised to +-tiny if smaller; with it the pivot is c_i
                        // (|c_i| > |a_i|), the multiplier uses c_i itself and only
                        // the stored reciprocal is that of +-tiny.  Selects, not
                        // branches: lanes of a wave take either case.
                        const double ci = cb[u], an = anb[u], bn = bnb[u];
                        const bool keep = fabs(ai) >= fabs(ci);
                        const double pa = fabs(ai) < tiny ? (ai < 0.0 ? -tiny : tiny) : ai;
                        const double rl = recip(keep ? pa : ci);
                        const double l = (keep ? ci : ai) * rl;
                        const double rp = (!keep && fabs(ci) < tiny) ? (ci < 0.0 ? -rtiny : rtiny) : rl;
                        const double u1 = keep ? bi : an;
                        const double u2 = keep ? 0.0 : bn;
                        const double pf = keep ? 0.0 : 1.0;
                        const double ain = keep ? an - l * bi : bi - l * an;
                        bi = keep ? bn : -l * bn;
                        ai = ain;
                        rr[W * u + oRP] = rp;
                        rr[W * u + oU1] = u1;
                        rr[W * u + oU2] = u2;
                        rr[W * u + oLM] = l;
                        rr[W * u + oPV] = pf;
                    }
                }
            }
            if (fabs(ai) < tiny) ai = (ai < 0.0 ? -tiny : tiny);
            // The last row has no superdiagonal terms and no multiplier; the
            // padding rows are all zero (their pivot reciprocal included).
            for (int i = J - 1; i < Jb; ++i) {
                rec[W * i + oRP] = i == J - 1 ? recip(ai) : 0.0;
                rec[W * i + oU1] = 0.0;
                rec[W * i + oU2] = 0.0;
                rec[W * i + oLM] = 0.0;
                rec[W * i + oPV] = 0.0;
            }
            double f1 = 1.0, f2 = 1.0;  // x = (stored x f1) f2
            // Both sweeps alternate two register sets: the next block's loads
            // are issued before this block's arithmetic and stores.  Rows past
            // J (all in the last block) carry zeros: the forward sweep maps a
            // zero row to zero, the backward one forces them.
            for (int it = 0; it < kInvIters; ++it) {
                // forward: row interchanges and multipliers, running value in xc
                double xA[IB], pA[IB], lA[IB], xB[IB], pB[IB], lB[IB];
                auto fload = [&](int i0, double (&xb)[IB], double (&pb)[IB], double (&lb)[IB]) {
                    const double* rr = row(i0);
#pragma unroll
                    for (int u = 0; u < IB; ++u) {
                        xb[u] = (rr[W * (u + 1) + oX] * f1) * f2;  // row Jb: zero
                        pb[u] = rr[W * u + oPV];
                        lb[u] = rr[W * u + oLM];
                    }
                };
                double xc = (rec[oX] * f1) * f2;
                auto fstep = [&](int i0, const double (&xb)[IB], const double (&pb)[IB],
                                 const double (&lb)[IB]) {
                    double ob[IB];
#pragma unroll
                    for (int u = 0; u < IB; ++u) {
                        double xn = xb[u];
                        if (pb[u] != 0.0) {
                            const double t = xc;
                            xc = xn;
                            xn = t;
                        }
                        ob[u] = xc;
                        xc = xn - lb[u] * xc;
                    }
                    double* rw = row(i0);
#pragma unroll
                    for (int u = 0; u < IB; ++u) rw[W * u + oX] = ob[u];
                };
                fload(0, xA, pA, lA);
                for (int i0 = 0;; i0 += 2 * IB) {
                    fload(min(i0 + IB, Jb - IB), xB, pB, lB);
                    fstep(i0, xA, pA, lA);
                    if (i0 + IB >= Jb) break;
                    fload(min(i0 + 2 * IB, Jb - IB), xA, pA, lA);
                    fstep(i0 + IB, xB, pB, lB);
                    if (i0 + 2 * IB >= Jb) break;
                }
                // backward substitution
                double u1A[IB], u2A[IB], rA[IB], u1B[IB], u2B[IB], rB[IB];
                auto bload = [&](int i0, double (&xb)[IB], double (&u1b)[IB], double (&u2b)[IB],
                                 double (&rb)[IB]) {
                    const double* rr = row(i0);
#pragma unroll
                    for (int u = 0; u < IB; ++u) {
                        xb[u] = rr[W * u + oX];
                        u1b[u] = rr[W * u + oU1];
                        u2b[u] = rr[W * u + oU2];
                        rb[u] = rr[W * u + oRP];
                    }
                };
                double x1 = 0.0, x2 = 0.0, amax = 0.0;
                auto bstep = [&](auto top, int i0, const double (&xb)[IB], const double (&u1b)[IB],
                                 const double (&u2b)[IB], const double (&rb)[IB]) {
                    double ob[IB];
#pragma unroll
                    for (int u = IB - 1; u >= 0; --u) {
                        double v = xb[u];
                        v = fma(-u1b[u], x1, v);
                        v = fma(-u2b[u], x2, v);
                        v *= rb[u];
                        if constexpr (decltype(top)::value) v = i0 + u < J ? v : 0.0;
                        ob[u] = v;
                        x2 = x1;
                        x1 = v;
                        amax = fmax(amax, fabs(v));
                    }
                    double* rw = row(i0);
#pragma unroll
                    for (int u = 0; u < IB; ++u) rw[W * u + oX] = ob[u];
                };
                bload(Jb - IB, xA, u1A, u2A, rA);
                for (int i0 = Jb - IB;; i0 -= 2 * IB) {
                    bload(max(i0 - IB, 0), xB, u1B, u2B, rB);
                    if (i0 == Jb - IB)
                        bstep(std::true_type{}, i0, xA, u1A, u2A, rA);
                    else
                        bstep(std::false_type{}, i0, xA, u1A, u2A, rA);
                    if (i0 == 0) break;
                    bload(max(i0 - 2 * IB, 0), xA, u1A, u2A, rA);
                    bstep(std::false_type{}, i0 - IB, xB, u1B, u2B, rB);
                    if (i0 == IB) break;
                }
                double nrm2 = 0.0;
                const double scl = amax > 0.0 ? 1.0 / amax : 1.0;
#pragma unroll 8
                for (int i = 0; i < J; ++i) {
                    const double v = rec[W * i + oX] * scl;
                    nrm2 += v * v;
                }
                f1 = scl;
                f2 = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 0.0;
            }
            SC1[jj] = f1;
            SC2[jj] = f2;
        }
        __syncthreads();
        for (int idx = tid; idx < J * nb; idx += kEigThreads) {
            const int jj = idx / J, i = idx - jj * J;
            X[(size_t)(j0 + jj) * J + i] =
                (reg[(size_t)jj * recd + kLuArrays * i + oX] * SC1[jj]) * SC2[jj];
        }
    }
    __syncthreads();

    // Modified Gram-Schmidt, twice, inside clusters (descending order), by
    // wave 0 with the working vector in registers and the others in LDS;
    // cluster starts are found in one pass over the eigenvalues.
    const int nslot = (J + 63) / 64;
    // per-lane slots of a vector: JP / 64 rounded up on the register path
    constexpr int kGsSlots = JP > 0 ? (JP + 63) / 64 : kMaxVecSlots;
    const double ortol = 1e-3 * tnorm;
    const bool clustered =
        __syncthreads_or(tid >= 1 && tid < R && lam[tid - 1] - lam[tid] <= ortol);
    if (clustered) {
        // vector j at XL[j J ..]: a copy in LDS when the region holds all R
        const bool in_lds = (size_t)R * J <= (size_t)region;
        double* XL = in_lds ? reg : X;
        if (in_lds)
            for (int idx = tid; idx < R * J; idx += kEigThreads) XL[idx] = X[idx];
        __syncthreads();
        if (wave == 0) {
            int c0 = 0;
            for (int j = 1; j < R; ++j) {
                c0 = lam[j - 1] - lam[j] <= ortol ? c0 : j;
                if (c0 == j) continue;
                // slot q holds element lane + 64 q (zero past J; the load
                // itself is clamped to the vector)
                auto ld = [&](int v, int q) {
                    const int t = lane + 64 * q;
                    const double x = XL[(size_t)v * J + min(t, J - 1)];
                    return t < J ? x : 0.0;
                };
                double xj[kGsSlots];
#pragma unroll
                for (int q = 0; q < kGsSlots; ++q) xj[q] = q < nslot ? ld(j, q) : 0.0;
                for (int pass = 0; pass < 2; ++pass) {
                    for (int i = c0; i < j; ++i) {
                        double xi[kGsSlots];
                        double s = 0.0;
#pragma unroll
                        for (int q = 0; q < kGsSlots; ++q) {
                            xi[q] = q < nslot ? ld(i, q) : 0.0;
                            s += xi[q] * xj[q];
                        }
                        s = wave_sum(s);
#pragma unroll
                        for (int q = 0; q < kGsSlots; ++q) xj[q] -= s * xi[q];
                    }
                }
                double n2 = 0.0;
#pragma unroll
                for (int q = 0; q < kGsSlots; ++q) n2 += xj[q] * xj[q];
                n2 = wave_sum(n2);
                const double inv = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
#pragma unroll
                for (int q = 0; q < kGsSlots; ++q) {
                    const int t = lane + 64 * q;
                    if (q < nslot && t < J) XL[(size_t)j * J + t] = xj[q] * inv;
                }
                if (!in_lds) __threadfence_block();  // later iterations read column j
            }
        }
        __syncthreads();
        if (in_lds)
            for (int idx = tid; idx < R * J; idx += kEigThreads) X[idx] = XL[idx];
    }
    __syncthreads();

    // ---- 5. back-transformation X <- Q X, Q = H_0 H_1 ... H_{J-3} -------
    // Sign rule for every vector: the largest |entry| (lowest index on ties)
    // is positive.
    if constexpr (JP > 0) {
        // A in registers (J <= JP): the LDS region, free again, takes the
        // reflectors in one coalesced pass at pitch JP with zeros outside
        // k < t < J (Hz[k JP + t] = v_t of reflector k).  Each vector is held
        // by 16 lanes, element t = 32 p + 2 l + h at lane l, pair p, half h,
        // so that a dot product ends in four row-local lane exchanges; a wave
        // carries four vectors through the J - 2 reflectors without barriers.
        constexpr int NP = JP / 32;
        double* Hz = reg;
        for (int idx = tid; idx < (J - 2) * JP; idx += kEigThreads) {
            const int k = idx / JP, t = idx - k * JP;
            Hz[idx] = (t > k && t < J) ? H[(size_t)k * J + (t - k - 1)] : 0.0;
        }
        __syncthreads();
        const int g = lane >> 4, l16 = lane & 15;
        for (int jw = 4 * wave; jw < R; jw += 4 * kEigWaves) {  // uniform over the wave
            const int j = jw + g;
            const bool jok = j < R;
            double2 xr[NP];
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const int t = 32 * p + 2 * l16;
                xr[p].x = (jok && t < J) ? X[(size_t)j * J + t] : 0.0;
                xr[p].y = (jok && t + 1 < J) ? X[(size_t)j * J + t + 1] : 0.0;
            }
            // reflector k and beta_k are loaded one reflector ahead of their use
            auto hload = [&](int k, double2 (&h)[NP], double& b) {
                b = beta[k];
                const double2* hk = reinterpret_cast<const double2*>(Hz + (size_t)k * JP);
#pragma unroll
                for (int p = 0; p < NP; ++p) h[p] = hk[16 * p + l16];
            };
            auto apply = [&](const double2 (&h)[NP], double b) {
                if (b == 0.0) return;  // uniform: the identity
                double s0 = 0.0, s1 = 0.0;
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    s0 = fma(h[p].x, xr[p].x, s0);
                    s1 = fma(h[p].y, xr[p].y, s1);
                }
                const double sk = b * row16_sum(s0 + s1);
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    xr[p].x -= sk * h[p].x;
                    xr[p].y -= sk * h[p].y;
                }
            };
            if (J >= 3) {
                double2 hA[NP], hB[NP];
                double bA, bB;
                hload(J - 3, hA, bA);
                for (int k = J - 3;; k -= 2) {
                    hload(max(k - 1, 0), hB, bB);
                    apply(hA, bA);
                    if (k == 0) break;
                    hload(max(k - 2, 0), hA, bA);
                    apply(hB, bB);
                    if (k == 1) break;
                }
            }
            double bv = -1.0;
            int bi = J;
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const int t = 32 * p + 2 * l16;
                if (t < J && fabs(xr[p].x) > bv) {
                    bv = fabs(xr[p].x);
                    bi = t;
                }
                if (t + 1 < J && fabs(xr[p].y) > bv) {
                    bv = fabs(xr[p].y);
                    bi = t + 1;
                }
            }
#pragma unroll
            for (int off = 8; off > 0; off >>= 1) {  // within the 16-lane group
                const double ov = __shfl_xor(bv, off, 64);
                const int oi = __shfl_xor(bi, off, 64);
                if (ov > bv || (ov == bv && oi < bi)) {
                    bv = ov;
                    bi = oi;
                }
            }
            double at = 0.0;
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const int t = 32 * p + 2 * l16;
                if (t == bi) at = xr[p].x;
                if (t + 1 == bi) at = xr[p].y;
            }
            const double sgn = row16_sum(at) < 0.0 ? -1.0 : 1.0;
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const int t = 32 * p + 2 * l16;
                if (jok && t < J) X[(size_t)j * J + t] = sgn * xr[p].x;
                if (jok && t + 1 < J) X[(size_t)j * J + t + 1] = sgn * xr[p].y;
            }
        }
    } else {
    // reflectors from global scratch; one wave per vector
    for (int j = wave; j < R; j += kEigWaves) {
        double xr[kMaxVecSlots];
#pragma unroll
        for (int q = 0; q < kMaxVecSlots; ++q) {
            const int t = lane + 64 * q;
            xr[q] = (q < nslot && t < J) ? X[(size_t)j * J + t] : 0.0;
        }
        for (int k = J - 3; k >= 0; --k) {
            const double b = beta[k];
            if (b == 0.0) continue;  // uniform
            double hv[kMaxVecSlots];
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < kMaxVecSlots; ++q) {
                const int t = lane + 64 * q;
                hv[q] = (q < nslot && t > k && t < J) ? H[(size_t)k * J + (t - k - 1)] : 0.0;
                s += hv[q] * xr[q];
            }
            s = b * wave_sum(s);
#pragma unroll
            for (int q = 0; q < kMaxVecSlots; ++q) xr[q] -= s * hv[q];
        }
        double bv = -1.0;
        int bi = J;
#pragma unroll
        for (int q = 0; q < kMaxVecSlots; ++q) {
            const int t = lane + 64 * q;
            if (q < nslot && t < J && fabs(xr[q]) > bv) {
                bv = fabs(xr[q]);
                bi = t;
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double ov = __shfl_xor(bv, off, 64);
            const int oi = __shfl_xor(bi, off, 64);
            if (ov > bv || (ov == bv && oi < bi)) {
                bv = ov;
                bi = oi;
            }
        }
        double at = 0.0;
#pragma unroll
        for (int q = 0; q < kMaxVecSlots; ++q)
            if (lane + 64 * q == bi) at = xr[q];
        const double sgn = wave_sum(at) < 0.0 ? -1.0 : 1.0;
#pragma unroll
        for (int q = 0; q < kMaxVecSlots; ++q) {
            const int t = lane + 64 * q;
            if (q < nslot && t < J) X[(size_t)j * J + t] = sgn * xr[q];
        }
    }
    }
}

template <int JP, int PH>
__global__ __launch_bounds__(kEigThreads) void eig_kernel(EigArgs a, int region) {
    eig_body<JP, PH>(a, region);
}

// Step 2 of a split solve by multisection on the scaled T in the hand-off
// area: each group of TPE lanes of a wave finds one eigenvalue k (k-th
// smallest) with TPE sample points per round (TPE + 1 sub-intervals), the
// same Sturm counts and stopping rule as the one-launch solver, and stores
// it, unscaled, at position J - 1 - k of the descending list.  TPE = 64 (one
// eigenvalue per wave, six bits per round) suits a single solve, whose few
// waves are latency-bound; a batch fills the GPU and is issue-bound, so
// TPE = 16 (four eigenvalues per wave) does less work in all.
template <int TPE>
__device__ __forceinline__ void multisect_group(double* __restrict__ ho, int J, int k,
                                                bool active, double* sm) {
    double* ds = sm;
    double* e2 = sm + J;
    const int lane = threadIdx.x;
    for (int i = lane; i < J; i += 64) {
        ds[i] = ho[3 * J + i];
        e2[i] = ho[4 * J + i];
    }
    __syncthreads();
    if (!active) return;  // the whole group (k is the same in its lanes)
    const int s = lane % TPE, gofs = lane - s;
    const uint64_t gmask = TPE == 64 ? ~0ull : (((1ull << TPE) - 1ull) << gofs);
    double lo = ho[5 * J], hi = ho[5 * J + 1];
    const double sc = ho[5 * J + 2];
    const double atol = 2.0 * DBL_EPSILON;  // T is scaled to norm <= 1
    for (int it = 0; it < 160; ++it) {
        const double tol = fmax(atol, 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)));
        if (hi - lo <= tol) break;  // lo, hi are the same in every lane of the group
        const double h = (hi - lo) / (double)(TPE + 1);
        const int c = sturm_count(ds, e2, J, lo + h * (double)(s + 1));
        const uint64_t bal = __ballot(c > k) & gmask;
        const int sstar = bal ? (__ffsll((long long)bal) - gofs) : TPE + 1;  // 1-based point
        const double nlo = sstar == 1 ? lo : lo + h * (double)(sstar - 1);
        const double nhi = sstar == TPE + 1 ? hi : lo + h * (double)sstar;
        lo = nlo;
        hi = nhi;
    }
    if (s == 0) ho[5 * J + 4 + (J - 1 - k)] = 0.5 * (lo + hi) / sc;
}

__global__ __launch_bounds__(64) void eig_multisect(double* __restrict__ scratch, int J) {
    extern __shared__ double sm[];
    multisect_group<64>(eig_handoff(scratch, J), J, blockIdx.x, true, sm);
}

// The same for a batch, four eigenvalues per workgroup: workgroup w takes
// eigenvalues 4 q .. 4 q + 3 of problem w / nq, q = w % nq, nq = ceil(jmax / 4)
// (groups beyond that problem's J do nothing).
constexpr int kBatchTpe = 16;
constexpr int kBatchGroups = 64 / kBatchTpe;

__global__ __launch_bounds__(64) void eig_multisect_batched(const EigArgs* __restrict__ args,
                                                            int nq, int conditional) {
    extern __shared__ double sm[];
    const int p = blockIdx.x / nq, q = blockIdx.x - p * nq;
    const int J = args[p].J;
    if (kBatchGroups * q >= J) return;  // uniform over the workgroup
    if (conditional && !(args[p].flags[0] & 4)) return;  // the redo pass: bit 4 only
    const int k = kBatchGroups * q + (int)threadIdx.x / kBatchTpe;
    multisect_group<kBatchTpe>(eig_handoff(uni_global(args[p].scratch), J), J, k, k < J, sm);
}

// One workgroup per problem of a batch, as PH = 1, eig_multisect_batched,
// PH = 3.  A problem whose status word has the FP64-only mark (8) took the
// FP64 Gram: the plain rank rule applies, and the pass's last launch clears
// the mark.  conditional != 0: only problems whose status word has the guard
// bit (4) run, on their FP64 Gram and without the guard; afterwards the bit is
// cleared and `mode_bit` is recorded in the problem's second status word.
template <int JP, int PH>
__global__ __launch_bounds__(kEigThreads) void eig_batched(const EigArgs* __restrict__ args,
                                                           int region, int conditional,
                                                           int mode_bit) {
    EigArgs a = args[blockIdx.x];
    // table pointers as global ones (global, not flat, accesses)
    a.s = uni_global(a.s);
    a.nu = uni_global(a.nu);
    a.lambda = uni_global(a.lambda);
    a.u = uni_global(a.u);
    a.rank_out = uni_global(a.rank_out);
    a.disc_out = uni_global(a.disc_out);
    a.flags = uni_global(a.flags);
    a.scratch = uni_global(a.scratch);
    a.split_stats = uni_global(a.split_stats);
    a.tail_bound = uni_global(a.tail_bound);
    const int f0 = a.flags ? a.flags[0] : 0;
    if (conditional && !(f0 & 4)) return;  // uniform over the workgroup
    if (conditional || (f0 & 8)) {
        a.guard = 0.0;  // an FP64 Gram: plain rank rule
        a.split_stats = nullptr;
    }
    eig_body<JP, PH>(a, region);
    if (PH != 1 && (conditional || (f0 & 8))) {  // the pass's last launch
        __syncthreads();
        if (threadIdx.x == 0) {
            if (conditional) {
                a.flags[0] &= ~4;
                a.flags[1] |= mode_bit;
            } else {
                a.flags[0] &= ~8;
            }
        }
    }
}

// The register path (J <= JP) keeps reflector k at row k, pitch JP, of the
// region: at least JP * J doubles (<= 16384 for JP <= 128).
static size_t eig_region_doubles_jp(int J, int JP) {
    const size_t r = eig_region_doubles(J), hs = (size_t)JP * J;
    return r < hs ? hs : r;
}

// Register layouts: 32, 64, 96 and 128 rows (8 lanes per row, 8 columns
// per register block); larger extents take the global-memory path (0).
static int eig_jp(int J) { return J <= 32 ? 32 : J <= 64 ? 64 : J <= 96 ? 96 : J <= 128 ? 128 : 0; }

size_t eig_lds_bytes(int J) {
    const int JP = eig_jp(J);
    return ((size_t)eig_region_doubles_jp(J, JP) + eig_small_doubles(J)) * sizeof(double);
}

int launch_eig_batched(const EigArgs* args_dev, int count, int jmax, int conditional,
                       int mode_bit, hipStream_t st) {
    if (jmax > 128) return fail(TK_ERR_UNSUPPORTED, "batched eigensolver: extent %d > 128", jmax);
    // every problem uses the register layout of the largest extent (96 rows
    // up to 96, else 128); the LDS partition follows each problem's own J
    // (region computed per J <= jmax)
    const int jp = jmax <= 96 ? 96 : 128;
    const int region = (int)eig_region_doubles_jp(jmax, jp);
    const size_t lds = ((size_t)region + eig_small_doubles(jmax)) * sizeof(double);
    auto launch = [&](auto fn) -> int {
        TK_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds));
        hipLaunchKernelGGL(fn, dim3(count), dim3(kEigThreads), lds, st, args_dev, region,
                           conditional, mode_bit);
        TK_HIP(hipGetLastError());
        return TK_OK;
    };
    TK_TRY(jp == 96 ? launch(eig_batched<96, 1>) : launch(eig_batched<128, 1>));
    const int nq = (jmax + kBatchGroups - 1) / kBatchGroups;
    hipLaunchKernelGGL(eig_multisect_batched, dim3(count * nq), dim3(64),
                       (size_t)2 * jmax * sizeof(double), st, args_dev, nq, conditional);
    TK_HIP(hipGetLastError());
    return jp == 96 ? launch(eig_batched<96, 3>) : launch(eig_batched<128, 3>);
}

// Extents of at least kSplitEig take three launches (reduction, multisection
// over J workgroups, vectors): the multisection then runs on the whole GPU.
constexpr int kSplitEig = 64;

template <int JP, int PH>
static int launch_eig_phase(const EigArgs& a, int region, size_t lds, hipStream_t st) {
    auto fn = eig_kernel<JP, PH>;
    TK_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
    hipLaunchKernelGGL(fn, dim3(1), dim3(kEigThreads), lds, st, a, region);
    TK_HIP(hipGetLastError());
    return TK_OK;
}

template <int JP>
static int launch_eig_jp(const EigArgs& a, int region, size_t lds, hipStream_t st) {
    if (a.J < kSplitEig) return launch_eig_phase<JP, 0>(a, region, lds, st);
    TK_TRY((launch_eig_phase<JP, 1>(a, region, lds, st)));
    hipLaunchKernelGGL(eig_multisect, dim3(a.J), dim3(64), (size_t)2 * a.J * sizeof(double), st,
                       a.scratch, a.J);
    TK_HIP(hipGetLastError());
    return launch_eig_phase<JP, 3>(a, region, lds, st);
}

int launch_eig(const EigArgs& a, hipStream_t st) {
    const int JP = eig_jp(a.J);
    const int region = (int)eig_region_doubles_jp(a.J, JP);
    const size_t lds = ((size_t)region + eig_small_doubles(a.J)) * sizeof(double);
    switch (JP) {
        case 32: return launch_eig_jp<32>(a, region, lds, st);
        case 64: return launch_eig_jp<64>(a, region, lds, st);
        case 96: return launch_eig_jp<96>(a, region, lds, st);
        case 128: return launch_eig_jp<128>(a, region, lds, st);
        default: return launch_eig_jp<0>(a, region, lds, st);
    }
}

}  // namespace tk
