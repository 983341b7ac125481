// Tensor-times-matrix Z = Y x_n op(M), i.e. Z_(n) = op(M) Y_(n)
// (Sec. II-A; Alg. 1 TTM step; Sec. V-B local product), in the natural
// layout: for every column tile of the block-column view Y[B][J][L] the
// kernel forms the K x KT output tile A * Y_tile with A = op(M) (K x J).
//
// Workgroup (p, g) streams its contiguous range of column tiles through LDS
// (register prefetch of the next tile while the current one is multiplied)
// and produces output rows [g*KB, g*KB + KB).  A is staged once per
// workgroup.  The MFMA operand order is chosen so that the lanes of a
// quarter-wave write consecutive output addresses: when the output's rows
// are contiguous (L >= 16) the kernel forms Z blocks, otherwise Z^T blocks.
#include "tk_common.hpp"

namespace tk {

typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int kTtmThreads = 512;
constexpr int kTtmWaves = kTtmThreads / 64;
constexpr int kTtmMaxBlocks = 8;

template <typename T>
__device__ __forceinline__ double ld_widen(const T* p) { return (double)*p; }

template <typename T>
__device__ __forceinline__ T narrow(double v) { return (T)v; }

// LDS: the Y tile [JB][KT + 1] (at least the [waves][256] area that folds
// k-slices), then A as [JB][KB + 1].
template <int JB, int KT>
constexpr int kTtmYDoubles = JB * (KT + 1) > kTtmWaves * 256 ? JB * (KT + 1) : kTtmWaves * 256;

template <typename T, int JB, int KB, int KT, bool ZT>
__global__ __launch_bounds__(kTtmThreads) void ttm_f64_kernel(
    const T* __restrict__ y, TileMap tm, const double* __restrict__ m, int64_t ldm, int K,
    int transpose, T* __restrict__ z) {
    extern __shared__ double lds[];
    constexpr int PY = KT + 1;
    constexpr int PA = KB + 1;
    double* ly = lds;                          // [JB][PY]
    double* la = lds + kTtmYDoubles<JB, KT>;   // [JB][PA]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
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
    for (int e = tid; e < JB * PY; e += kTtmThreads) ly[e] = 0.0;

    // output blocks of this tile: (KB/16) x (KT/16); waves take them
    // round-robin, and idle waves split the J reduction of a block.
    constexpr int nrb = KB / 16, ncb = KT / 16, nblk = nrb * ncb;
    int kslices = 1, slice = 0, first = wave, stride = kTtmWaves, mine;
    if (nblk < kTtmWaves) {
        kslices = kTtmWaves / nblk;
        slice = wave / nblk;
        first = wave % nblk;
        stride = nblk;
        mine = (wave < nblk * kslices) ? 1 : 0;
    } else {
        mine = (nblk - wave + kTtmWaves - 1) / kTtmWaves;
    }
    const int nks = (J + 3) / 4;

    const int64_t t0 = tm.ntiles * (int64_t)blockIdx.x / gridDim.x;
    const int64_t t1 = tm.ntiles * (int64_t)(blockIdx.x + 1) / gridDim.x;

    constexpr int kPer = (JB * KT + kTtmThreads - 1) / kTtmThreads;
    double pf[kPer];
    Tile cur{};
    auto load = [&](const Tile& t) {
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            int e = tid + kTtmThreads * q;
            double v = 0.0;
            if (tm.packed) {
                if (e < t.nvalid) v = ld_widen(y + t.base + e);
            } else {
                int i = e / KT, kk = e - (e / KT) * KT;
                if (i < J && kk < t.ncols) v = ld_widen(y + t.base + (int64_t)i * tm.L + kk);
            }
            pf[q] = v;
        }
    };
    auto store = [&](const Tile& t) {
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            int e = tid + kTtmThreads * q;
            if (tm.packed) {
                int L = (int)tm.L, JL = J * L;
                int bb = e / JL, rem = e - bb * JL, i = rem / L, l = rem - i * L;
                if (bb < tm.nbb) ly[i * PY + bb * L + l] = pf[q];
            } else {
                int i = e / KT, kk = e - (e / KT) * KT;
                if (i < JB) ly[i * PY + kk] = pf[q];
            }
        }
    };
    if (t0 < t1) {
        cur = tile_at(tm, t0, J);
        load(cur);
    }
    const int c16 = lane & 15, q4 = lane >> 4;
    for (int64_t t = t0; t < t1; ++t) {
        __syncthreads();
        store(cur);
        __syncthreads();
        const Tile here = cur;
        const int64_t out_base = tile_at(tm, t, K).base;
        if (t + 1 < t1) {
            cur = tile_at(tm, t + 1, J);
            load(cur);
        }
        d4_t acc[kTtmMaxBlocks];
#pragma unroll
        for (int b = 0; b < kTtmMaxBlocks; ++b) acc[b] = d4_t{0.0, 0.0, 0.0, 0.0};
        for (int ks = slice; ks < nks; ks += kslices) {
            const int i = ks * 4 + q4;
#pragma unroll
            for (int b = 0; b < kTtmMaxBlocks; ++b) {
                if (b < mine) {
                    int blk = first + b * stride;
                    int rb = blk / ncb, cb = blk - (blk / ncb) * ncb;
                    double av = la[i * PA + rb * 16 + c16];
                    double yv = ly[i * PY + cb * 16 + c16];
                    acc[b] = ZT ? __builtin_amdgcn_mfma_f64_16x16x4f64(yv, av, acc[b], 0, 0, 0)
                                : __builtin_amdgcn_mfma_f64_16x16x4f64(av, yv, acc[b], 0, 0, 0);
                }
            }
        }
        if (kslices > 1) {
            // fold the k-slices of each block through LDS in a fixed order
            __syncthreads();
            double* red = ly;  // reuse the Y tile area: [wave][256]
            if (mine) {
#pragma unroll
                for (int v = 0; v < 4; ++v) red[wave * 256 + (4 * v + q4) * 16 + c16] = acc[0][v];
            }
            __syncthreads();
            if (mine && slice == 0) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    double s = 0.0;
                    for (int sl = 0; sl < kslices; ++sl)
                        s += red[(sl * nblk + first) * 256 + (4 * v + q4) * 16 + c16];
                    acc[0][v] = s;
                }
            }
            __syncthreads();  // red (= ly) is rewritten by the next tile's store
            if (slice != 0) continue;
        }
#pragma unroll
        for (int b = 0; b < kTtmMaxBlocks; ++b) {
            if (b < mine) {
                int blk = first + b * stride;
                int rb = blk / ncb, cb = blk - (blk / ncb) * ncb;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    // f64 MFMA output: row 4 * v + lane / 16, column lane % 16
                    int r, kk;
                    if (ZT) {
                        kk = cb * 16 + 4 * v + q4;
                        r = rb * 16 + c16;
                    } else {
                        r = rb * 16 + 4 * v + q4;
                        kk = cb * 16 + c16;
                    }
                    int rg = r_g0 + r;
                    if (rg < K && kk < here.ncols) {
                        int64_t off;
                        if (tm.packed) {
                            int L = (int)tm.L;
                            int bb = kk / L, l = kk - bb * L;
                            off = out_base + ((int64_t)bb * K + rg) * L + l;
                        } else {
                            off = out_base + (int64_t)rg * tm.L + kk;
                        }
                        z[off] = narrow<T>(acc[b][v]);
                    }
                }
            }
        }
    }
}

// ------------------------------------------------------------------ host

static int round_pow2(int v, int lo) {
    int r = lo;
    while (r < v) r *= 2;
    return r;
}

template <typename T, int JB, int KB, int KT>
static int launch_ttm_t(const T* y, const TileMap& tm, const double* m, int64_t ldm, int K,
                        int transpose, T* z, bool zt, hipStream_t st) {
    size_t lds = (size_t)(kTtmYDoubles<JB, KT> + JB * (KB + 1)) * sizeof(double);
    int cus = device_cu_count();
    int G = (K + KB - 1) / KB;
    int64_t want = (int64_t)2 * cus / G;
    if (want < 1) want = 1;
    int P = (int)(tm.ntiles < want ? tm.ntiles : want);
    if (P < 1) return TK_OK;
    if (zt) {
        auto fn = ttm_f64_kernel<T, JB, KB, KT, true>;
        TK_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds));
        hipLaunchKernelGGL(fn, dim3(P, G), dim3(kTtmThreads), lds, st, y, tm, m, ldm, K,
                           transpose, z);
    } else {
        auto fn = ttm_f64_kernel<T, JB, KB, KT, false>;
        TK_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds));
        hipLaunchKernelGGL(fn, dim3(P, G), dim3(kTtmThreads), lds, st, y, tm, m, ldm, K,
                           transpose, z);
    }
    TK_HIP(hipGetLastError());
    return TK_OK;
}

// KB (output rows per workgroup) shrinks as J grows so that A fits in LDS.
template <typename T, int JB, int KT>
static int pick_kb(const T* y, const TileMap& tm, const double* m, int64_t ldm, int K,
                   int transpose, T* z, bool zt, hipStream_t st) {
    constexpr int kbmax = (JB <= 32) ? 256 : (JB == 64) ? 128 : (JB == 128) ? 64 : (JB == 256) ? 32 : 16;
    if (K <= 16 || kbmax == 16)
        return launch_ttm_t<T, JB, 16, KT>(y, tm, m, ldm, K, transpose, z, zt, st);
    if constexpr (kbmax >= 32) {
        if (K <= 32 || kbmax == 32)
            return launch_ttm_t<T, JB, 32, KT>(y, tm, m, ldm, K, transpose, z, zt, st);
    }
    if constexpr (kbmax >= 64) {
        if (K <= 64 || kbmax == 64)
            return launch_ttm_t<T, JB, 64, KT>(y, tm, m, ldm, K, transpose, z, zt, st);
    }
    if constexpr (kbmax >= 128) {
        if (K <= 128 || kbmax == 128)
            return launch_ttm_t<T, JB, 128, KT>(y, tm, m, ldm, K, transpose, z, zt, st);
    }
    if constexpr (kbmax >= 256) return launch_ttm_t<T, JB, 256, KT>(y, tm, m, ldm, K, transpose, z, zt, st);
    return fail(TK_ERR_UNSUPPORTED, "ttm: no tile for K=%d", K);
}

template <typename T>
static int dispatch_ttm(const T* y, const ModeView& v, const double* m, int64_t K, int64_t ldm,
                        int transpose, T* z, hipStream_t st) {
    int jb = round_pow2(v.J, 32);
    const int KT = jb >= 512 ? 16 : 32;
    TileMap tm = make_tiles(v, KT);
    bool zt = v.L < 16;
    switch (jb) {
        case 32: return pick_kb<T, 32, 32>(y, tm, m, ldm, (int)K, transpose, z, zt, st);
        case 64: return pick_kb<T, 64, 32>(y, tm, m, ldm, (int)K, transpose, z, zt, st);
        case 128: return pick_kb<T, 128, 32>(y, tm, m, ldm, (int)K, transpose, z, zt, st);
        case 256: return pick_kb<T, 256, 32>(y, tm, m, ldm, (int)K, transpose, z, zt, st);
        case 512: return pick_kb<T, 512, 16>(y, tm, m, ldm, (int)K, transpose, z, zt, st);
        default: return fail(TK_ERR_UNSUPPORTED, "mode extent %d exceeds %d", v.J, TK_MAX_MODE_DIM);
    }
}

int launch_ttm_mixed(const float* y, const ModeView& v, const double* m, int64_t K, int64_t ldm,
                     int transpose, int precision, float* z, hipStream_t st);

int launch_ttm(const void* y, int dtype, const ModeView& v, const double* m, int64_t K,
               int64_t ldm, int transpose, int precision, void* z, hipStream_t st) {
    if (precision == TK_TTM_FP64) {
        if (dtype == TK_F64)
            return dispatch_ttm((const double*)y, v, m, K, ldm, transpose, (double*)z, st);
        return dispatch_ttm((const float*)y, v, m, K, ldm, transpose, (float*)z, st);
    }
    return launch_ttm_mixed((const float*)y, v, m, K, ldm, transpose, precision, (float*)z, st);
}

}  // namespace tk
