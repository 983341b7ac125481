// Gram matrix S = Y_(n) Y_(n)^T of a mode-n unfolding (Alg. 1, Gram step),
// computed in the natural layout without permuting data (Sec. V-C, local
// part), exploiting symmetry: only 16x16 blocks (bi <= bj) are formed.
//
// Stage 1 (gram_partial_f64): workgroup (p, g) streams its contiguous range
// of column tiles (TileMap) through a double-buffered LDS tile and
// accumulates the block pairs of pair group g in registers.  Each wave owns
// NPW block pairs (a compile-time count, so the MFMA loop is branch-free)
// and a k-slice of each tile.  One barrier per tile: while the MFMAs read
// buffer t % 2 the registers holding tile t + 1 are written to the other
// buffer.  It writes one partial per pair to the workspace.
// Stage 2 (gram_reduce): sums the partials over p in a fixed order (so S is
// bitwise reproducible) and mirrors the upper blocks into both triangles.
//
// FP64 path: v_mfma_f64_16x16x4f64 on FP64 data (FP32 input is widened
// exactly while staging).  Narrow modes (J <= 32 over long contiguous runs)
// replace stage 1 by gram_narrow_f64, which needs no LDS tile.
#include "tile_io.hpp"
#include "tk_common.hpp"

namespace tk {

typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int kGramThreads = 512;
constexpr int kGramWaves = kGramThreads / 64;

// Pair index p -> (bi, bj), upper-triangle blocks in row-major order.
__device__ __forceinline__ void pair_of(int p, int nb, int& bi, int& bj) {
    int row = 0;
    int start = 0;
    while (p >= start + (nb - row)) {
        start += nb - row;
        ++row;
    }
    bi = row;
    bj = row + (p - start);
}

// LDS doubles: two [JB][KT + 1] tile buffers (at least the area used to fold
// k-slices at the end).
template <int JB, int KT, int NPW>
constexpr int kGramLdsDoubles = 2 * JB * (KT + 1) > kGramWaves * NPW * 256
                                    ? 2 * JB * (KT + 1)
                                    : kGramWaves * NPW * 256;

// NPW: block pairs per wave; KS: waves sharing one pair set, each taking
// every KS-th k-step.  The waves form kGramWaves / KS groups of NPW pairs.
// One workgroup's share: tiles [t0, t1) of pair group g0 .. g0 + npg - 1;
// writes npairs * 256 partial sums at `out` (those of its own pairs).
template <typename T, int JB, int KT, int NPW, int KS, bool SKIP = false>
__device__ __forceinline__ void gram_f64_body(const T* __restrict__ y, const TileMap& tm, int nb,
                                              int g0, int npg, int64_t t0, int64_t t1,
                                              double* __restrict__ out, double* lds) {
    constexpr int P = KT + 1;
    constexpr int NG = kGramWaves / KS;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r16 = lane & 15, k4 = lane >> 4;

    for (int e = tid; e < 2 * JB * P; e += kGramThreads) lds[e] = 0.0;

    const int grp = wave % NG, slice = wave / NG;
    // SKIP (batches, J below the extent class): pairs with a block at or past
    // ceil(J / 16) sum zeros only and skip their products (partials stay 0)
    const int nbv = SKIP ? __builtin_amdgcn_readfirstlane((tm.J + 15) >> 4) : nb;
    int aoff[NPW], boff[NPW];
    bool live[NPW];
#pragma unroll
    for (int q = 0; q < NPW; ++q) {
        int p = g0 + min(grp * NPW + q, npg - 1);  // spare slots repeat the last pair
        int bi, bj;
        pair_of(p, nb, bi, bj);
        live[q] = !SKIP || max(bi, bj) < nbv;
        aoff[q] = (bi * 16 + r16) * P + k4;
        boff[q] = (bj * 16 + r16) * P + k4;
    }
    d4_t acc[NPW];
#pragma unroll
    for (int q = 0; q < NPW; ++q) acc[q] = d4_t{0.0, 0.0, 0.0, 0.0};

    ColumnTile<T, double, JB, KT, kGramThreads> ld;
    ld.setup(tm, tid);
    if (t0 < t1) ld.load(y, tm, tile_at(tm, t0, tm.J));
    __syncthreads();  // zeroing done before the first store
    if (t0 < t1) ld.store(lds);
    __syncthreads();
    for (int64_t t = t0; t < t1; ++t) {
        const double* cur = lds + ((t - t0) & 1) * (JB * P);
        double* nxt = lds + (((t - t0) + 1) & 1) * (JB * P);
        const bool more = t + 1 < t1;
        if (more) ld.load(y, tm, tile_at(tm, t + 1, tm.J));  // in flight during the MFMAs
#pragma unroll
        for (int kq = 0; kq < KT / 4 / KS; ++kq) {
            const int ks = kq * KS + slice;
            double a[NPW], b[NPW];
#pragma unroll
            for (int q = 0; q < NPW; ++q) {
                a[q] = cur[aoff[q] + ks * 4];
                b[q] = cur[boff[q] + ks * 4];
            }
#pragma unroll
            for (int q = 0; q < NPW; ++q) {
                if (SKIP && !live[q]) continue;  // uniform
                acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], b[q], acc[q], 0, 0, 0);
            }
        }
        if (more) ld.store(nxt);
        __syncthreads();
    }

    // v_mfma_f64_16x16x4f64 leaves D[row][col] in lane col + 16 * (row % 4),
    // register row / 4, i.e. row = 4 * v + lane / 16, col = lane % 16.
    if constexpr (KS > 1) {
        double* red = lds;  // [wave][NPW][256]
#pragma unroll
        for (int q = 0; q < NPW; ++q)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                red[(wave * NPW + q) * 256 + (4 * v + k4) * 16 + r16] = acc[q][v];
        __syncthreads();
        if (slice == 0) {
#pragma unroll
            for (int q = 0; q < NPW; ++q) {
                int pl = grp * NPW + q;
                if (pl < npg) {
                    for (int e = lane; e < 256; e += 64) {
                        double s = 0.0;
#pragma unroll
                        for (int sl = 0; sl < KS; ++sl)
                            s += red[((sl * NG + grp) * NPW + q) * 256 + e];
                        out[(int64_t)(g0 + pl) * 256 + e] = s;
                    }
                }
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < NPW; ++q) {
            int pl = grp * NPW + q;
            if (pl < npg) {
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    out[(int64_t)(g0 + pl) * 256 + (4 * v + k4) * 16 + r16] = acc[q][v];
            }
        }
    }
}

// P tile ranges x G pair groups, one workgroup each (xcd_range_group).
template <typename T, int JB, int KT, int NPW, int KS>
__global__ __launch_bounds__(kGramThreads) void gram_partial_f64(
    const T* __restrict__ y, TileMap tm, int nb, int npairs, int pairs_per_group, int P, int G,
    double* __restrict__ partial) {
    extern __shared__ double lds[];
    int p, g;
    xcd_range_group(blockIdx.x, G, p, g);
    const int g0 = g * pairs_per_group;
    const int npg = min(npairs - g0, pairs_per_group);
    const int64_t t0 = tm.ntiles * (int64_t)p / P;
    const int64_t t1 = tm.ntiles * (int64_t)(p + 1) / P;
    gram_f64_body<T, JB, KT, NPW, KS>(y, tm, nb, g0, npg, t0, t1,
                                      partial + (int64_t)p * npairs * 256, lds);
}

// acc + partial[q n + idx] over q = g, g + 4, ... < P, added in that order;
// eight loads go out per trip so that they overlap.
__device__ __forceinline__ double sum_partials(const double* __restrict__ partial, int P,
                                               int n, int idx, int g) {
    double acc = 0.0;
    int q = g;
    for (; q + 28 < P; q += 32) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = partial[(int64_t)(q + 4 * u) * n + idx];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; q < P; q += 4) acc += partial[(int64_t)q * n + idx];
    return acc;
}

// {sum over p of aux[2 p], max over p of aux[2 p + 1]} -> out[0..1], summed
// by the first wave of a workgroup in a fixed order (lane-strided partial
// sums, then lane by lane).
__device__ __forceinline__ void reduce_split_stats(const double* __restrict__ aux, int P,
                                                   double* __restrict__ out, double* part) {
    const int lane = threadIdx.x;
    if (lane < 64) {
        double d = 0.0, e = -125.0;
        for (int q = lane; q < P; q += 64) {
            d += aux[2 * q];
            e = fmax(e, aux[2 * q + 1]);
        }
        part[lane] = d;
        part[64 + lane] = e;
    }
    __syncthreads();
    if (lane == 0) {
        double d = 0.0, e = -125.0;
        for (int k = 0; k < 64; ++k) {
            d += part[k];
            e = fmax(e, part[64 + k]);
        }
        out[0] = d;
        out[1] = e;
    }
}

// S[r + J c] for the upper block pairs.  Each workgroup reduces 64 outputs;
// its 4 wave-sized groups sum the partials p = g, g + 4, ... and the four
// group sums are added in a fixed order.  With aux, one more workgroup
// reduces the split statistics into stats.
__global__ __launch_bounds__(256) void gram_reduce(const double* __restrict__ partial, int P,
                                                   int npairs, int nb, int J,
                                                   double* __restrict__ s,
                                                   const double* __restrict__ aux,
                                                   double* __restrict__ stats) {
    __shared__ double part[4][64];
    if (aux && blockIdx.x == gridDim.x - 1) {  // uniform over the workgroup
        reduce_split_stats(aux, P, stats, &part[0][0]);
        return;
    }
    const int o = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int idx = blockIdx.x * 64 + o;
    const int n = npairs * 256;
    const double acc = idx < n ? sum_partials(partial, P, n, idx, g) : 0.0;
    part[g][o] = acc;
    __syncthreads();
    if (g != 0 || idx >= n) return;
    const double tot = ((part[0][o] + part[1][o]) + part[2][o]) + part[3][o];
    int p = idx >> 8, e = idx & 255;
    int bi, bj;
    pair_of(p, nb, bi, bj);
    int r = bi * 16 + (e >> 4), c = bj * 16 + (e & 15);
    if (r >= J || c >= J) return;
    if (bi == bj && r > c) return;  // diagonal blocks: upper triangle only, then mirror
    s[r + (int64_t)J * c] = tot;
    s[c + (int64_t)J * r] = tot;
}

// trace(S) = ||Y||^2, summed in a fixed order by one wave.
__global__ void gram_trace(const double* __restrict__ s, int J, double* __restrict__ out) {
    __shared__ double part[64];
    int lane = threadIdx.x;
    double acc = 0.0;
    for (int i = lane; i < J; i += 64) acc += s[i + (int64_t)J * i];
    part[lane] = acc;
    __syncthreads();
    if (lane == 0) {
        double t = 0.0;
        for (int k = 0; k < 64; ++k) t += part[k];
        *out = t;
    }
}

// ------------------------------------------------------------ narrow modes
//
// J <= 32 where every unfolding row is made of long contiguous runs (L a
// multiple of 8): no LDS tile.  A step is 32 consecutive l of one slab b.
// Lane t of a wave owns unfolding row t % 16 (and 16 + t % 16 when J > 16)
// and the eight columns l0 + 8 (t / 16) + e of a step, read with one vector
// load per row straight from HBM.  For MFMA call e each lane's element is
// both A[t % 16][t / 16] and B[t / 16][t % 16], so the eight calls sum
// y_i y_j over the step's 32 columns.  A wave takes U consecutive steps at a
// time (one contiguous run of 32 U elements per row); its accumulators stay
// in registers until the end, where the 8 waves of a workgroup fold them
// through LDS, in a fixed order, into one partial per workgroup.
constexpr int kNarrowThreads = 512;
constexpr int kNarrowWaves = kNarrowThreads / 64;

template <typename T>
struct Run8;
template <>
struct Run8<float> {
    typedef float type __attribute__((ext_vector_type(8)));
};
template <>
struct Run8<double> {
    typedef double type __attribute__((ext_vector_type(8)));
};

// Block pairs of the narrow kernel: (0,0) for J <= 16; (0,0), (0,1), (1,1)
// (pair_of order with nb = 2) for 16 < J <= 32.
template <int JN>
constexpr int kNarrowPairs = JN == 16 ? 1 : 3;

template <typename T, int JN, int U>
__global__ __launch_bounds__(kNarrowThreads) void gram_narrow_f64(
    const T* __restrict__ y, int64_t L, int J, int64_t nsteps, int P,
    double* __restrict__ partial) {
    constexpr int NR = JN / 16;  // row blocks per lane
    constexpr int NP = kNarrowPairs<JN>;
    constexpr int NA = JN == 16 ? 2 : 3;  // J <= 16: two accumulator chains
    typedef typename Run8<T>::type run_t;
    __shared__ double red[kNarrowWaves * NP * 256];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r16 = lane & 15, k4 = lane >> 4;
    const int p = blockIdx.x;
    const int64_t s0 = nsteps * p / P, s1 = nsteps * (p + 1) / P;
    const int64_t sb = (L + 31) >> 5;  // steps per slab
    const int64_t slab = (int64_t)J * L;
    int64_t roff[NR];
    bool rok[NR];
#pragma unroll
    for (int h = 0; h < NR; ++h) {
        const int r = 16 * h + r16;
        rok[h] = r < J;
        roff[h] = (int64_t)(rok[h] ? r : 0) * L + 8 * k4;
    }
    d4_t acc[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) acc[a] = d4_t{0.0, 0.0, 0.0, 0.0};

    for (int64_t q = s0 + (int64_t)wave * U; q < s1; q += (int64_t)kNarrowWaves * U) {
        int64_t b = q / sb;
        int64_t l0 = (q - b * sb) << 5;
        run_t v[U][NR];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool ok = q + u < s1 && l0 + 8 * k4 < L;
            const T* base = y + b * slab + l0;
#pragma unroll
            for (int h = 0; h < NR; ++h) {
                if (ok && rok[h])
                    v[u][h] = *reinterpret_cast<const run_t*>(base + roff[h]);
                else
                    v[u][h] = run_t(0);
            }
            l0 += 32;
            if (l0 >= L) {
                l0 = 0;
                ++b;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const double a0 = (double)v[u][0][e];
                if constexpr (JN == 16) {
                    acc[e & 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, a0, acc[e & 1], 0, 0, 0);
                } else {
                    const double a1 = (double)v[u][1][e];
                    acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, a0, acc[0], 0, 0, 0);
                    acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, a1, acc[1], 0, 0, 0);
                    acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, a1, acc[2], 0, 0, 0);
                }
            }
    }
    if constexpr (JN == 16) acc[0] += acc[1];

    // D[row][col] of pair c sits in lane col + 16 (row % 4), register row / 4
#pragma unroll
    for (int c = 0; c < NP; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            red[(wave * NP + c) * 256 + (4 * r + k4) * 16 + r16] = acc[c][r];
    __syncthreads();
    for (int e = threadIdx.x; e < NP * 256; e += kNarrowThreads) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kNarrowWaves; ++w) s += red[w * NP * 256 + e];
        partial[(int64_t)p * NP * 256 + e] = s;
    }
}

// ------------------------------------------------------------------ host

static int round_jb(int J) {
    int jb = 32;
    while (jb < J) jb *= 2;
    return jb;
}

// Static schedule per padded extent: tile width, pairs per wave, k-slices
// per pair set, and pairs per workgroup group.
struct GramShape {
    int KT, NPW, KS, per_group;
};

template <int JB>
constexpr GramShape gram_shape() {
    return JB == 32    ? GramShape{32, 1, 2, 4}    //   3 pairs: 4 groups x 1, 2 k-slices
           : JB == 64  ? GramShape{32, 3, 2, 12}   //  10 pairs: 4 groups x 3, 2 k-slices
           : JB == 128 ? GramShape{32, 5, 1, 40}   //  36 pairs: 8 waves x 5
           : JB == 256 ? GramShape{32, 6, 1, 48}   // 136 pairs: 3 groups of <= 48
                       : GramShape{16, 8, 1, 64};  // 528 pairs: 9 groups of <= 64
}

static GramShape gram_shape_rt(int jb) {
    switch (jb) {
        case 32: return gram_shape<32>();
        case 64: return gram_shape<64>();
        case 128: return gram_shape<128>();
        case 256: return gram_shape<256>();
        default: return gram_shape<512>();
    }
}

// Narrow-mode plan: one partial per workgroup, at most 2 per CU, each
// workgroup holding at least one batch of steps per wave.
constexpr int kNarrowStepsF32 = 4, kNarrowStepsF64 = 2;  // U: steps per batch

static int64_t narrow_steps(const ModeView& v) { return v.B * ((v.L + 31) / 32); }

static GramPlan plan_narrow(const ModeView& v, int elem_bytes) {
    GramPlan pl{};
    pl.narrow = v.J <= 16 ? 16 : 32;
    pl.nb = pl.narrow / 16;
    pl.npairs = pl.nb * (pl.nb + 1) / 2;
    pl.G = 1;
    pl.pairs_per_group = pl.npairs;
    const int U = elem_bytes == 8 ? kNarrowStepsF64 : kNarrowStepsF32;
    const int64_t per_wg = (int64_t)kNarrowWaves * U;
    const int64_t cap = 2 * (int64_t)device_cu_count();
    int64_t P = (narrow_steps(v) + per_wg - 1) / per_wg;
    pl.P = (int)(P < 1 ? 1 : P > cap ? cap : P);
    pl.partial_bytes = (size_t)pl.P * pl.npairs * 256 * sizeof(double);
    pl.partial_bound = (size_t)cap * pl.npairs * 256 * sizeof(double);
    return pl;
}

static GramPlan plan_tiled(const ModeView& v) {
    GramPlan pl{};
    GramShape gs = gram_shape_rt(round_jb(v.J));
    pl.KT = gs.KT;
    pl.nb = (v.J + 15) / 16;
    pl.npairs = pl.nb * (pl.nb + 1) / 2;
    pl.G = (pl.npairs + gs.per_group - 1) / gs.per_group;
    pl.pairs_per_group = (pl.npairs + pl.G - 1) / pl.G;
    TileMap tm = make_tiles(v, pl.KT);
    const int64_t want = xcd_round_want((int64_t)2 * device_cu_count() / pl.G, pl.G);
    pl.P = xcd_ranges(tm.ntiles, want, pl.G);
    pl.partial_bytes = (size_t)pl.P * pl.npairs * 256 * sizeof(double);
    pl.partial_bound = (size_t)want * pl.npairs * 256 * sizeof(double);
    return pl;
}

// The narrow kernel's plan where the view qualifies; its workspace bounds
// also cover the tiled plan, which runs instead when the data pointer is not
// aligned for the kernel's vector loads.
GramPlan plan_gram(const ModeView& v, int precision, int elem_bytes) {
    if (precision == TK_GRAM_SPLIT_BF16) return plan_gram_mixed(v);
    GramPlan tiled = plan_tiled(v);
    if (!gram_narrow_view(v)) return tiled;
    GramPlan pl = plan_narrow(v, elem_bytes);
    if (tiled.partial_bytes > pl.partial_bytes) pl.partial_bytes = tiled.partial_bytes;
    if (tiled.partial_bound > pl.partial_bound) pl.partial_bound = tiled.partial_bound;
    return pl;
}

template <typename T, int JN>
static int launch_narrow(const T* y, const ModeView& v, const GramPlan& pl, double* partial,
                         hipStream_t st) {
    constexpr int U = sizeof(T) == 8 ? kNarrowStepsF64 : kNarrowStepsF32;
    hipLaunchKernelGGL((gram_narrow_f64<T, JN, U>), dim3(pl.P), dim3(kNarrowThreads), 0, st, y,
                       v.L, v.J, narrow_steps(v), pl.P, partial);
    TK_HIP(hipGetLastError());
    return TK_OK;
}

template <typename T>
static int dispatch_narrow(const T* y, const ModeView& v, const GramPlan& pl, double* partial,
                           hipStream_t st) {
    return pl.narrow == 16 ? launch_narrow<T, 16>(y, v, pl, partial, st)
                           : launch_narrow<T, 32>(y, v, pl, partial, st);
}

template <typename T, int JB>
static int launch_partial(const T* y, const TileMap& tm, const GramPlan& pl, double* partial,
                          hipStream_t st) {
    constexpr GramShape gs = gram_shape<JB>();
    size_t lds = (size_t)kGramLdsDoubles<JB, gs.KT, gs.NPW> * sizeof(double);
    auto fn = gram_partial_f64<T, JB, gs.KT, gs.NPW, gs.KS>;
    TK_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
    hipLaunchKernelGGL(fn, dim3(pl.P * pl.G), dim3(kGramThreads), lds, st, y, tm, pl.nb,
                       pl.npairs, pl.pairs_per_group, pl.P, pl.G, partial);
    TK_HIP(hipGetLastError());
    return TK_OK;
}

template <typename T>
static int dispatch_partial(const T* y, const ModeView& v, const GramPlan& pl, double* partial,
                            hipStream_t st) {
    TileMap tm = make_tiles(v, pl.KT);
    switch (round_jb(v.J)) {
        case 32: return launch_partial<T, 32>(y, tm, pl, partial, st);
        case 64: return launch_partial<T, 64>(y, tm, pl, partial, st);
        case 128: return launch_partial<T, 128>(y, tm, pl, partial, st);
        case 256: return launch_partial<T, 256>(y, tm, pl, partial, st);
        case 512: return launch_partial<T, 512>(y, tm, pl, partial, st);
        default: return fail(TK_ERR_UNSUPPORTED, "mode extent %d exceeds %d", v.J, TK_MAX_MODE_DIM);
    }
}

int launch_gram_reduce(const double* partial, const GramPlan& pl, int J, double* s,
                       const double* aux, double* stats, hipStream_t st) {
    int n = pl.npairs * 256;
    const int nblk = (n + 63) / 64 + (aux ? 1 : 0);
    hipLaunchKernelGGL(gram_reduce, dim3(nblk), dim3(256), 0, st, partial, pl.P, pl.npairs,
                       pl.nb, J, s, aux, stats);
    TK_HIP(hipGetLastError());
    return TK_OK;
}

// One launch reduces the partials of every problem of a batch (and forms the
// trace of those that need ||X||^2), in the same fixed order as gram_reduce.
__global__ __launch_bounds__(256) void gram_reduce_batched(const BatchReduceTask* __restrict__ tasks,
                                                           int ntasks, int conditional) {
    __shared__ double part[4][64];
    int lo = 0, hi = ntasks - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tasks[mid].wg_begin <= (int)blockIdx.x) lo = mid; else hi = mid - 1;
    }
    BatchReduceTask tk = tasks[lo];
    tk.partial = uni_global(tk.partial);  // global, not flat, accesses
    tk.s = uni_global(tk.s);
    if (conditional && !(*tk.status & 4)) return;  // uniform over the workgroup
    const int w = blockIdx.x - tk.wg_begin;
    const int o = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int n = tk.npairs * 256;
    const int P = *tk.nparts;  // slots the Gram launch wrote (<= tk.P)
    // split statistics: a split Gram's, not a redo's nor an FP64-only problem's
    const bool split = tk.aux != nullptr && !conditional && !(tk.status && (*tk.status & 8));
    const bool extra = tk.nu != nullptr || split;
    if (w < tk.nwg - 1 || !extra) {
        const int idx = w * 64 + o;
        const double acc = idx < n ? sum_partials(tk.partial, P, n, idx, g) : 0.0;
        part[g][o] = acc;
        __syncthreads();
        if (g != 0 || idx >= n) return;
        const double tot = ((part[0][o] + part[1][o]) + part[2][o]) + part[3][o];
        const int p = idx >> 8, e = idx & 255;
        int bi, bj;
        pair_of(p, tk.nb, bi, bj);
        const int r = bi * 16 + (e >> 4), c = bj * 16 + (e & 15);
        if (r >= tk.J || c >= tk.J) return;
        if (bi == bj && r > c) return;
        tk.s[r + (int64_t)tk.J * c] = tot;
        tk.s[c + (int64_t)tk.J * r] = tot;
    } else {
        // the problem's last workgroup: split statistics of the unconditional
        // (split) pass, and the trace of its diagonal from the partials
        // (diagonal 16-blocks p = bi nb - bi (bi - 1) / 2), fixed order
        if (split) {
            reduce_split_stats(tk.aux, P, tk.stats, &part[0][0]);
            __syncthreads();
        }
        if (tk.nu == nullptr) return;
        // each diagonal entry summed as the other workgroups sum S's entries
        // (four slot groups, eight loads in flight each, then added in a
        // fixed order), the entries then lane by lane
        double acc = 0.0;
        for (int i0 = 0; i0 < tk.J; i0 += 64) {  // uniform
            const int i = i0 + o;
            const int bi = i >> 4, p = bi * tk.nb - bi * (bi - 1) / 2;
            const int idx = p * 256 + (i & 15) * 17;
            part[g][o] = i < tk.J ? sum_partials(tk.partial, P, n, idx, g) : 0.0;
            __syncthreads();
            if (g == 0) acc += ((part[0][o] + part[1][o]) + part[2][o]) + part[3][o];
            __syncthreads();
        }
        if (g == 0) part[0][o] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int k = 0; k < 64; ++k) t += part[0][k];
            *tk.nu = t;
        }
    }
}

// Clears status words with a kernel (no memset node in a captured graph).
__global__ void fill_i32(int* __restrict__ p, int n, int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

int launch_fill_i32(int* p, int n, int v, hipStream_t st) {
    if (n <= 0) return TK_OK;
    hipLaunchKernelGGL(fill_i32, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
    TK_HIP(hipGetLastError());
    return TK_OK;
}

int launch_gram_reduce_batched(const BatchReduceTask* tasks_dev, int ntasks, int total_wg,
                               int conditional, hipStream_t st) {
    hipLaunchKernelGGL(gram_reduce_batched, dim3(total_wg), dim3(256), 0, st, tasks_dev, ntasks,
                       conditional);
    TK_HIP(hipGetLastError());
    return TK_OK;
}

// FP64 Gram of every problem of a batch (the guard's recomputation when
// `conditional`).  The partials use the split kernel's layout -- 16-blocks of
// the padded extent JB, pairs in pair_of order -- so the same reduction
// tasks apply; pairs in the padding come out zero.
template <int JB>
__global__ __launch_bounds__(kGramThreads) void gram_f64_batched(
    const BatchGramTask* __restrict__ tasks, int ntasks, int conditional) {
    extern __shared__ double lds[];
    constexpr GramShape gs = gram_shape<JB>();
    constexpr int nb = JB / 16, npairs = nb * (nb + 1) / 2;
    static_assert(gs.per_group >= npairs, "batches need a single pair group");
    const int ti = find_task_wg(&tasks[0].v, sizeof(BatchGramTask), ntasks, blockIdx.x);
    BatchGramTask tk = tasks[ti];
    tk.y = uni_global(tk.y);  // global, not flat, accesses
    tk.partial = uni_global(tk.partial);
    // uniform over the workgroup: 1 = the redo of uncertain ranks (bit 4),
    // 2 = the problems marked FP64-only (bit 8)
    if (conditional && !(*tk.status & (conditional == 2 ? 8 : 4))) return;
    const int w = blockIdx.x - tk.v.wg_begin;
    const TileMap tm = make_tiles(batch_mode_view(tk.v), gs.KT);
    const int active = (int)(tm.ntiles < tk.v.nwg ? tm.ntiles : tk.v.nwg);
    if (w == 0 && threadIdx.x == 0) *tk.nparts = active;
    if (w >= active) return;  // uniform over the workgroup
    const int64_t t0 = tm.ntiles * (int64_t)w / active;
    const int64_t t1 = tm.ntiles * (int64_t)(w + 1) / active;
    gram_f64_body<float, JB, gs.KT, gs.NPW, gs.KS, true>(
        tk.y, tm, nb, 0, npairs, t0, t1, tk.partial + (int64_t)w * npairs * 256, lds);
}

template <int JB>
static int launch_f64_batched_t(const BatchGramTask* tasks, int ntasks, int total_wg,
                                int conditional, hipStream_t st) {
    constexpr GramShape gs = gram_shape<JB>();
    const size_t lds = (size_t)kGramLdsDoubles<JB, gs.KT, gs.NPW> * sizeof(double);
    auto fn = gram_f64_batched<JB>;
    TK_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
    hipLaunchKernelGGL(fn, dim3(total_wg), dim3(kGramThreads), lds, st, tasks, ntasks,
                       conditional);
    TK_HIP(hipGetLastError());
    return TK_OK;
}

// One thread per task: the problem's FP64 Gram work at its actual shape
// (the truncated extents come from the device ranks) decides bit 8.
__global__ __launch_bounds__(64) void batch_mark_fp64(const BatchGramTask* __restrict__ tasks,
                                                      int ntasks, double max_flops) {
    const int t = blockIdx.x * 64 + threadIdx.x;
    if (t >= ntasks) return;
    const BatchGramTask tk = tasks[t];
    const ModeView v = batch_mode_view(tk.v);
    const double flops = 2.0 * (double)v.J * (double)v.J * (double)v.L * (double)v.B;
    if (flops <= max_flops) *const_cast<int*>(tk.status) |= 8;  // the task is the word's only writer here
}

int launch_batch_mark_fp64(const BatchGramTask* tasks_dev, int ntasks, double max_flops,
                           hipStream_t st) {
    if (ntasks <= 0) return TK_OK;
    hipLaunchKernelGGL(batch_mark_fp64, dim3((ntasks + 63) / 64), dim3(64), 0, st, tasks_dev,
                       ntasks, max_flops);
    TK_HIP(hipGetLastError());
    return TK_OK;
}

int launch_gram_f64_batched(const BatchGramTask* tasks_dev, int ntasks, int total_wg, int jb,
                            int conditional, hipStream_t st) {
    switch (jb) {
        case 32: return launch_f64_batched_t<32>(tasks_dev, ntasks, total_wg, conditional, st);
        case 64: return launch_f64_batched_t<64>(tasks_dev, ntasks, total_wg, conditional, st);
        case 128: return launch_f64_batched_t<128>(tasks_dev, ntasks, total_wg, conditional, st);
        default: return fail(TK_ERR_UNSUPPORTED, "batched FP64 Gram: extent class %d", jb);
    }
}

int launch_gram(const void* y, int dtype, const ModeView& v, int precision, double* s,
                double* sumsq, void* ws, size_t ws_bytes, hipStream_t st,
                double* split_stats, const hipEvent_t* ev) {
    GramPlan pl = plan_gram(v, precision, (int)dtype_size(dtype));
    if (ws_bytes < pl.partial_bytes)
        return fail(TK_ERR_WORKSPACE, "gram workspace %zu < %zu", ws_bytes, pl.partial_bytes);
    double* partial = (double*)ws;
    // the narrow kernel's 8-element vector loads need the run's own alignment
    if (pl.narrow && (uintptr_t)y % (8 * dtype_size(dtype)) != 0) pl = plan_tiled(v);
    if (ev) TK_HIP(hipEventRecord(ev[0], st));
    if (precision == TK_GRAM_SPLIT_BF16) {
        TK_TRY(launch_gram_mixed((const float*)y, v, pl, partial, st));
    } else if (pl.narrow) {
        if (dtype == TK_F64)
            TK_TRY(dispatch_narrow((const double*)y, v, pl, partial, st));
        else
            TK_TRY(dispatch_narrow((const float*)y, v, pl, partial, st));
    } else if (dtype == TK_F64) {
        TK_TRY(dispatch_partial((const double*)y, v, pl, partial, st));
    } else {
        TK_TRY(dispatch_partial((const float*)y, v, pl, partial, st));
    }
    if (ev) TK_HIP(hipEventRecord(ev[1], st));
    const bool split = precision == TK_GRAM_SPLIT_BF16;
    const double* aux = split && split_stats ? partial + (size_t)pl.P * pl.npairs * 256 : nullptr;
    TK_TRY(launch_gram_reduce(partial, pl, v.J, s, aux, split_stats, st));
    if (sumsq) {
        hipLaunchKernelGGL(gram_trace, dim3(1), dim3(64), 0, st, s, v.J, sumsq);
        TK_HIP(hipGetLastError());
    }
    return TK_OK;
}

}  // namespace tk
