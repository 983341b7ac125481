// Tensor-times-matrix Z = Y x_n op(M), i.e. Z_(n) = op(M) Y_(n)
// (Sec. II-A; Alg. 1 TTM step; Sec. V-B local product), in the natural
// layout: for every column tile of the block-column view Y[B][J][L] the
// kernel forms the K x KT output tile A * Y_tile with A = op(M) (K x J).
//
// Workgroup (p, g) streams its contiguous range of column tiles through LDS
// (the next tile is prefetched into registers while the current one is
// multiplied) and produces output rows [g*KB, g*KB + KB); A's rows for the
// group are staged in LDS once.  The 16x16 output blocks of a tile are
// dealt to waves at compile time (NBW per wave); when a tile has fewer
// blocks than waves, the spare waves only load.  The FP64 TTM needs far
// less matrix throughput than HBM delivers, so idle MFMA slots cost nothing.
// The MFMA operand order is chosen so that the lanes of a quarter-wave
// write consecutive output addresses: when the output's rows are contiguous
// (L >= 16) the kernel forms Z blocks, otherwise Z^T blocks.  Narrow modes
// (J <= 64, K <= 16 over long contiguous runs) take ttm_narrow_f64 instead,
// whatever precision is asked for.
#include "tile_io.hpp"
#include "tk_common.hpp"

namespace tk {

typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int kTtmThreads = 512;
constexpr int kTtmWaves = kTtmThreads / 64;

template <typename T, int JB, int KB, int KT, bool ZT>
__global__ __launch_bounds__(kTtmThreads) void ttm_f64_kernel(
    const T* __restrict__ y, TileMap tm, const double* __restrict__ m, int64_t ldm, int K,
    int transpose, T* __restrict__ z) {
    extern __shared__ double lds[];
    constexpr int PY = KT + 1;
    constexpr int PA = KB + 1;
    constexpr int nrb = KB / 16, ncb = KT / 16, nblk = nrb * ncb;
    constexpr int NBW = nblk >= kTtmWaves ? nblk / kTtmWaves : 1;
    static_assert(nblk < kTtmWaves || nblk % kTtmWaves == 0, "blocks must split over waves");
    double* ly = lds;              // [JB][PY]
    double* la = lds + JB * PY;    // [JB][PA]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int c16 = lane & 15, q4 = lane >> 4;
    const int J = tm.J;
    const int r_g0 = blockIdx.y * KB;

    // stage A[r][i] = op(M)[r_g0 + r][i] as la[i][r]
    for (int e = tid; e < JB * KB; e += kTtmThreads) {
        int i = e / KB, r = e - (e / KB) * KB;
        int rg = r_g0 + r;
        double v = 0.0;
        if (i < J && rg < K) v = transpose ? m[i + ldm * rg] : m[rg + ldm * i];
        la[i * PA + r] = v;
    }

    const bool busy = wave < nblk;  // waves beyond the block count only load
    int aoff[NBW], yoff[NBW], rbk[NBW], cbk[NBW];
#pragma unroll
    for (int b = 0; b < NBW; ++b) {
        int blk = busy ? wave + b * kTtmWaves : 0;
        rbk[b] = blk / ncb;
        cbk[b] = blk - (blk / ncb) * ncb;
        aoff[b] = q4 * PA + rbk[b] * 16 + c16;
        yoff[b] = q4 * PY + cbk[b] * 16 + c16;
    }
    const int nks = (J + 3) / 4;

    const int64_t t0 = tm.ntiles * (int64_t)blockIdx.x / gridDim.x;
    const int64_t t1 = tm.ntiles * (int64_t)(blockIdx.x + 1) / gridDim.x;

    ColumnTile<T, double, JB, KT, kTtmThreads> ld;
    ld.setup(tm, tid);
    if (t0 < t1) ld.load(y, tm, tile_at(tm, t0, J));
    for (int64_t t = t0; t < t1; ++t) {
        __syncthreads();  // previous tile consumed (and A staged)
        ld.store(ly);
        __syncthreads();
        const int ncols = tile_at(tm, t, J).ncols;
        const int64_t out_base = tile_at(tm, t, K).base;
        if (t + 1 < t1) ld.load(y, tm, tile_at(tm, t + 1, J));  // in flight during the MFMAs
        if (!busy) continue;
        d4_t acc[NBW];
#pragma unroll
        for (int b = 0; b < NBW; ++b) acc[b] = d4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
        for (int ks = 0; ks < nks; ++ks) {
#pragma unroll
            for (int b = 0; b < NBW; ++b) {
                const double av = la[aoff[b] + ks * 4 * PA];
                const double yv = ly[yoff[b] + ks * 4 * PY];
                acc[b] = ZT ? __builtin_amdgcn_mfma_f64_16x16x4f64(yv, av, acc[b], 0, 0, 0)
                            : __builtin_amdgcn_mfma_f64_16x16x4f64(av, yv, acc[b], 0, 0, 0);
            }
        }
#pragma unroll
        for (int b = 0; b < NBW; ++b) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                // f64 MFMA output: row 4 * v + lane / 16, column lane % 16
                int r, kk;
                if (ZT) {
                    kk = cbk[b] * 16 + 4 * v + q4;
                    r = rbk[b] * 16 + c16;
                } else {
                    r = rbk[b] * 16 + 4 * v + q4;
                    kk = cbk[b] * 16 + c16;
                }
                const int rg = r_g0 + r;
                if (rg < K && kk < ncols)
                    z[out_base + tile_col_offset(kk, tm.L, K) + (int64_t)rg * tm.L] = (T)acc[b][v];
            }
        }
    }
}

// ------------------------------------------------------------ narrow modes
//
// J <= 64 and K <= 16 where the rows of Y_(n) and Z_(n) are made of runs of
// L contiguous elements (L a multiple of 8): no LDS.  A step is 16 E
// consecutive l of one slab b (E = 16 bytes / element size).  In k-step s
// lane t holds A[t % 16][4 s + t / 16] (op(M), FP64, loaded once) and reads
// Y[4 s + t / 16][l0 + E (t % 16) + e], e < E, with one 16-byte load.  MFMA
// call (s, e) takes that element as B[t / 16][t % 16], so accumulator e
// gathers Z[r][l0 + E c + e] for output row r and column block c: each lane
// ends up with E consecutive l of four output rows and stores them with one
// 16-byte store per row.  Arithmetic is FP64 (exact products of the stored
// values), rounded once to the storage type.
constexpr int kNarrowTtmThreads = 512;
constexpr int kNarrowTtmWaves = kNarrowTtmThreads / 64;

template <typename T, int JN, int U>
__global__ __launch_bounds__(kNarrowTtmThreads) void ttm_narrow_f64(
    const T* __restrict__ y, int64_t L, int J, const double* __restrict__ m, int64_t ldm, int K,
    int transpose, int64_t nsteps, int P, T* __restrict__ z) {
    constexpr int E = 16 / (int)sizeof(T);  // columns per lane per load
    constexpr int SC = 16 * E;              // columns per step
    constexpr int NS = JN / 4;              // k-steps
    typedef T vec_t __attribute__((ext_vector_type(E)));
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c16 = lane & 15, q4 = lane >> 4;

    double a[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int i = 4 * s + q4;
        a[s] = (c16 < K && i < J) ? (transpose ? m[i + ldm * c16] : m[c16 + ldm * i]) : 0.0;
    }
    bool iok[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) iok[s] = 4 * s + q4 < J;
    bool rok[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) rok[v] = 4 * v + q4 < K;

    const int p = blockIdx.x;
    const int64_t s0 = nsteps * p / P, s1 = nsteps * (p + 1) / P;
    const int64_t sb = (L + SC - 1) / SC;  // steps per slab
    const int64_t yslab = (int64_t)J * L, zslab = (int64_t)K * L;
    for (int64_t q = s0 + (int64_t)wave * U; q < s1; q += (int64_t)kNarrowTtmWaves * U) {
        int64_t b = q / sb;
        int64_t l0 = (q - b * sb) * SC;
        vec_t v[U][NS];
        int64_t lo[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            lo[u] = b * zslab + l0 + E * c16;
            ok[u] = q + u < s1 && l0 + E * c16 < L;
            const T* src = y + b * yslab + l0 + E * c16;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                if (ok[u] && iok[s])
                    v[u][s] = *reinterpret_cast<const vec_t*>(src + (int64_t)(4 * s + q4) * L);
                else
                    v[u][s] = vec_t(0);
            }
            l0 += SC;
            if (l0 >= L) {
                l0 = 0;
                ++b;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            d4_t acc[E];
#pragma unroll
            for (int e = 0; e < E; ++e) acc[e] = d4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < NS; ++s)
#pragma unroll
                for (int e = 0; e < E; ++e)
                    acc[e] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], (double)v[u][s][e],
                                                                  acc[e], 0, 0, 0);
            // D[row][col] sits in lane col + 16 (row % 4), register row / 4:
            // this lane holds rows 4 w + q4, columns l0 + E c16 + e
            if (ok[u]) {
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    if (!rok[w]) continue;
                    vec_t out;
#pragma unroll
                    for (int e = 0; e < E; ++e) out[e] = (T)acc[e][w];
                    *reinterpret_cast<vec_t*>(z + lo[u] + (int64_t)(4 * w + q4) * L) = out;
                }
            }
        }
    }
}

// U: steps per batch (one at J <= 64, where a step already holds 16 loads)
template <int JN>
constexpr int kNarrowTtmSteps = JN == 64 ? 1 : 2;

// Views the narrow TTM takes (the data pointers are checked at launch).
static bool ttm_narrow_view(const ModeView& v, int64_t K) {
    return v.J <= 64 && K >= 1 && K <= 16 && v.L % 8 == 0 && v.L >= 64;
}

template <typename T, int JN>
static int launch_ttm_narrow(const T* y, const ModeView& v, const double* m, int64_t K,
                             int64_t ldm, int transpose, T* z, hipStream_t st) {
    constexpr int U = kNarrowTtmSteps<JN>;
    constexpr int SC = 16 * (16 / (int)sizeof(T));
    const int64_t nsteps = v.B * ((v.L + SC - 1) / SC);
    const int64_t per_wg = (int64_t)kNarrowTtmWaves * U;
    const int64_t cap = 2 * (int64_t)device_cu_count();
    int64_t P = (nsteps + per_wg - 1) / per_wg;
    P = P < 1 ? 1 : P > cap ? cap : P;
    hipLaunchKernelGGL((ttm_narrow_f64<T, JN, U>), dim3((int)P), dim3(kNarrowTtmThreads), 0, st,
                       y, v.L, v.J, m, ldm, (int)K, transpose, nsteps, (int)P, z);
    TK_HIP(hipGetLastError());
    return TK_OK;
}

template <typename T>
static int dispatch_ttm_narrow(const T* y, const ModeView& v, const double* m, int64_t K,
                               int64_t ldm, int transpose, T* z, hipStream_t st) {
    if (v.J <= 16) return launch_ttm_narrow<T, 16>(y, v, m, K, ldm, transpose, z, st);
    if (v.J <= 32) return launch_ttm_narrow<T, 32>(y, v, m, K, ldm, transpose, z, st);
    return launch_ttm_narrow<T, 64>(y, v, m, K, ldm, transpose, z, st);
}

// ------------------------------------------------------------------ host

static int round_pow2(int v, int lo) {
    int r = lo;
    while (r < v) r *= 2;
    return r;
}

// Tile shapes per padded extent JB: tile width KT and the largest number of
// output rows KB per workgroup, sized so the Y tile and A fit in LDS.
template <int JB>
constexpr int ttm_kt() { return JB <= 64 ? 128 : JB == 128 ? 64 : JB == 256 ? 32 : 16; }
template <int JB>
constexpr int ttm_kbmax() { return JB <= 32 ? 256 : JB == 64 ? 128 : JB == 128 ? 64 : JB == 256 ? 32 : 16; }

template <typename T, int JB, int KB>
static int launch_ttm_t(const T* y, const ModeView& v, const double* m, int64_t ldm, int K,
                        int transpose, T* z, hipStream_t st) {
    constexpr int KT = ttm_kt<JB>();
    TileMap tm = make_tiles(v, KT);
    size_t lds = (size_t)JB * ((KT + 1) + (KB + 1)) * sizeof(double);
    int G = (K + KB - 1) / KB;
    auto fn = v.L < 16 ? ttm_f64_kernel<T, JB, KB, KT, true> : ttm_f64_kernel<T, JB, KB, KT, false>;
    TK_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
    // One wave of resident workgroups: as many per CU as registers and LDS
    // allow, each streaming a contiguous range of tiles.
    int per_cu = 1;
    TK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)fn, kTtmThreads,
                                                        lds));
    per_cu = per_cu < 1 ? 1 : (per_cu > 4 ? 4 : per_cu);
    int64_t want = (int64_t)per_cu * device_cu_count() / G;
    if (want < 1) want = 1;
    int P = (int)(tm.ntiles < want ? tm.ntiles : want);
    if (P < 1) return TK_OK;
    hipLaunchKernelGGL(fn, dim3(P, G), dim3(kTtmThreads), lds, st, y, tm, m, ldm, K, transpose,
                       z);
    TK_HIP(hipGetLastError());
    return TK_OK;
}

// KB (output rows per workgroup group): the smallest power of two >= K,
// capped so that A fits in LDS; larger K uses several row groups.
template <typename T, int JB>
static int pick_kb(const T* y, const ModeView& v, const double* m, int64_t ldm, int K,
                   int transpose, T* z, hipStream_t st) {
    constexpr int kbmax = ttm_kbmax<JB>();
    if (K <= 16 || kbmax == 16) return launch_ttm_t<T, JB, 16>(y, v, m, ldm, K, transpose, z, st);
    if constexpr (kbmax >= 32) {
        if (K <= 32 || kbmax == 32)
            return launch_ttm_t<T, JB, 32>(y, v, m, ldm, K, transpose, z, st);
    }
    if constexpr (kbmax >= 64) {
        if (K <= 64 || kbmax == 64)
            return launch_ttm_t<T, JB, 64>(y, v, m, ldm, K, transpose, z, st);
    }
    if constexpr (kbmax >= 128) {
        if (K <= 128 || kbmax == 128)
            return launch_ttm_t<T, JB, 128>(y, v, m, ldm, K, transpose, z, st);
    }
    if constexpr (kbmax >= 256) return launch_ttm_t<T, JB, 256>(y, v, m, ldm, K, transpose, z, st);
    return fail(TK_ERR_UNSUPPORTED, "ttm: no tile for K=%d", K);
}

template <typename T>
static int dispatch_ttm(const T* y, const ModeView& v, const double* m, int64_t K, int64_t ldm,
                        int transpose, T* z, hipStream_t st) {
    switch (round_pow2(v.J, 32)) {
        case 32: return pick_kb<T, 32>(y, v, m, ldm, (int)K, transpose, z, st);
        case 64: return pick_kb<T, 64>(y, v, m, ldm, (int)K, transpose, z, st);
        case 128: return pick_kb<T, 128>(y, v, m, ldm, (int)K, transpose, z, st);
        case 256: return pick_kb<T, 256>(y, v, m, ldm, (int)K, transpose, z, st);
        case 512: return pick_kb<T, 512>(y, v, m, ldm, (int)K, transpose, z, st);
        default: return fail(TK_ERR_UNSUPPORTED, "mode extent %d exceeds %d", v.J, TK_MAX_MODE_DIM);
    }
}

int launch_ttm_mixed(const float* y, const ModeView& v, const double* m, int64_t K, int64_t ldm,
                     int transpose, int precision, float* z, hipStream_t st);

int launch_ttm(const void* y, int dtype, const ModeView& v, const double* m, int64_t K,
               int64_t ldm, int transpose, int precision, void* z, hipStream_t st) {
    // Narrow modes: FP64 arithmetic at streaming speed, which meets the error
    // bound of every precision option (16-byte vector loads and stores need
    // both data pointers aligned to 16 bytes).
    if (ttm_narrow_view(v, K) && (uintptr_t)y % 16 == 0 && (uintptr_t)z % 16 == 0) {
        if (dtype == TK_F64)
            return dispatch_ttm_narrow((const double*)y, v, m, K, ldm, transpose, (double*)z, st);
        return dispatch_ttm_narrow((const float*)y, v, m, K, ldm, transpose, (float*)z, st);
    }
    if (precision == TK_TTM_FP64) {
        if (dtype == TK_F64)
            return dispatch_ttm((const double*)y, v, m, K, ldm, transpose, (double*)z, st);
        return dispatch_ttm((const float*)y, v, m, K, ldm, transpose, (float*)z, st);
    }
    return launch_ttm_mixed((const float*)y, v, m, K, ldm, transpose, precision, (float*)z, st);
}

}  // namespace tk
