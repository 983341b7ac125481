// Gram matrix S = Y_(n) Y_(n)^T of a mode-n unfolding (Alg. 1, Gram step),
// computed in the natural layout without permuting data (Sec. V-C, local
// part), exploiting symmetry: only 16x16 blocks (bi <= bj) are formed.
//
// Stage 1 (gram_partial_*): workgroup (p, g) streams its contiguous range of
// column tiles (TileMap) through LDS and accumulates the block pairs of pair
// group g in registers; it writes one partial per pair to the workspace.
// Stage 2 (gram_reduce): sums the partials over p in a fixed order (so S is
// bitwise reproducible) and mirrors the upper blocks into both triangles.
//
// FP64 path: v_mfma_f64_16x16x4f64 on FP64 data (FP32 input is widened
// exactly while staging).
#include "tk_common.hpp"

namespace tk {

typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int kGramThreads = 512;
constexpr int kGramWaves = kGramThreads / 64;
constexpr int kGramMaxPairs = 8;  // 16x16 block pairs held per wave (FP64)

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

template <typename T>
__device__ __forceinline__ double widen(T v) { return (double)v; }

// Loads this thread's share of one column tile into registers.  The tile is
// J x KT (rows padded to JB); element e = tid + kGramThreads * q is mapped so
// that consecutive threads read consecutive memory.  Masked elements are 0.
template <typename T, int JB, int KT>
struct TileLoader {
    static constexpr int kElems = JB * KT;
    static constexpr int kPer = (kElems + kGramThreads - 1) / kGramThreads;
    double v[kPer];

    __device__ __forceinline__ void load(const T* __restrict__ y, const TileMap& tm,
                                         const Tile& t, int tid) {
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            int e = tid + kGramThreads * q;
            double val = 0.0;
            if (tm.packed) {
                if (e < t.nvalid) val = widen(y[t.base + e]);
            } else {
                int i = e / KT, kk = e - (e / KT) * KT;
                if (i < tm.J && kk < t.ncols) val = widen(y[t.base + (int64_t)i * tm.L + kk]);
            }
            v[q] = val;
        }
    }

    // LDS layout: [row i][column kk] with pitch KT + 1 doubles.
    __device__ __forceinline__ void store(double* lds, const TileMap& tm, const Tile& t,
                                          int tid) const {
        constexpr int P = KT + 1;
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            int e = tid + kGramThreads * q;
            if (tm.packed) {
                // memory order [bb][i][l]; column kk = bb * L + l
                int L = (int)tm.L;
                int JL = tm.J * L;
                int bb = e / JL;
                int rem = e - bb * JL;
                int i = rem / L;
                int l = rem - i * L;
                if (bb < tm.nbb) lds[i * P + bb * L + l] = v[q];
            } else {
                int i = e / KT, kk = e - (e / KT) * KT;
                if (i < JB) lds[i * P + kk] = v[q];
            }
        }
    }
};

// LDS doubles: the [JB][KT + 1] tile, at least the [waves][256] area used to
// fold k-slices at the end.
template <int JB, int KT>
constexpr int kGramLdsDoubles =
    JB * (KT + 1) > kGramWaves * 256 ? JB * (KT + 1) : kGramWaves * 256;

template <typename T, int JB, int KT>
__global__ __launch_bounds__(kGramThreads) void gram_partial_f64(
    const T* __restrict__ y, TileMap tm, int nb, int npairs, int pairs_per_group,
    double* __restrict__ partial) {
    extern __shared__ double lds[];
    constexpr int P = KT + 1;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;

    // zero the whole tile area once; padded rows J..JB-1 stay zero
    for (int e = tid; e < kGramLdsDoubles<JB, KT>; e += kGramThreads) lds[e] = 0.0;

    // this group's pairs and this wave's assignment
    const int g0 = blockIdx.y * pairs_per_group;
    const int npg = min(npairs - g0, pairs_per_group);
    int kslices = 1, slice = 0, first = wave, stride = kGramWaves, mine = 0;
    if (npg < kGramWaves) {
        kslices = kGramWaves / npg;
        slice = wave / npg;
        first = wave % npg;
        stride = npg;
        mine = (wave < npg * kslices) ? 1 : 0;
    } else {
        mine = (npg - wave + kGramWaves - 1) / kGramWaves;
    }
    int bi[kGramMaxPairs], bj[kGramMaxPairs];
#pragma unroll
    for (int q = 0; q < kGramMaxPairs; ++q) {
        bi[q] = 0;
        bj[q] = 0;
        if (q < mine) pair_of(g0 + first + q * stride, nb, bi[q], bj[q]);
    }
    d4_t acc[kGramMaxPairs];
#pragma unroll
    for (int q = 0; q < kGramMaxPairs; ++q) acc[q] = d4_t{0.0, 0.0, 0.0, 0.0};

    const int64_t t0 = tm.ntiles * (int64_t)blockIdx.x / gridDim.x;
    const int64_t t1 = tm.ntiles * (int64_t)(blockIdx.x + 1) / gridDim.x;

    TileLoader<T, JB, KT> ld;
    Tile cur{};
    if (t0 < t1) {
        cur = tile_at(tm, t0, tm.J);
        ld.load(y, tm, cur, tid);
    }
    const int r16 = lane & 15;
    const int k4 = lane >> 4;
    for (int64_t t = t0; t < t1; ++t) {
        __syncthreads();  // previous tile fully consumed
        ld.store(lds, tm, cur, tid);
        __syncthreads();
        if (t + 1 < t1) {
            cur = tile_at(tm, t + 1, tm.J);
            ld.load(y, tm, cur, tid);  // in flight while the MFMAs run
        }
#pragma unroll 2
        for (int ks = slice; ks < KT / 4; ks += kslices) {
            const int col = ks * 4 + k4;
#pragma unroll
            for (int q = 0; q < kGramMaxPairs; ++q) {
                if (q < mine) {
                    double a = lds[(bi[q] * 16 + r16) * P + col];
                    double b = lds[(bj[q] * 16 + r16) * P + col];
                    acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[q], 0, 0, 0);
                }
            }
        }
    }

    // combine k-slices (fixed order), then write one partial per pair.
    // v_mfma_f64_16x16x4f64 leaves D[row][col] in lane col + 16 * (row % 4),
    // register row / 4, i.e. row = 4 * v + lane / 16, col = lane % 16.
    double* out = partial + (int64_t)blockIdx.x * npairs * 256;
    if (kslices > 1) {
        __syncthreads();
        double* red = lds;  // [wave][256]
        if (mine) {
#pragma unroll
            for (int v = 0; v < 4; ++v) red[wave * 256 + (4 * v + k4) * 16 + r16] = acc[0][v];
        }
        __syncthreads();
        if (mine && slice == 0) {
            for (int e = lane; e < 256; e += 64) {
                double s = 0.0;
                for (int sl = 0; sl < kslices; ++sl) s += red[(sl * npg + first) * 256 + e];
                out[(int64_t)(g0 + first) * 256 + e] = s;
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < kGramMaxPairs; ++q) {
            if (q < mine) {
                int p = g0 + first + q * stride;
#pragma unroll
                for (int v = 0; v < 4; ++v) out[(int64_t)p * 256 + (4 * v + k4) * 16 + r16] = acc[q][v];
            }
        }
    }
}

// S[r + J c] for the upper block pairs, summed over the P partials in order.
__global__ void gram_reduce(const double* __restrict__ partial, int P, int npairs, int nb, int J,
                            double* __restrict__ s) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= npairs * 256) return;
    int p = idx >> 8, e = idx & 255;
    int bi, bj;
    pair_of(p, nb, bi, bj);
    int r = bi * 16 + (e >> 4), c = bj * 16 + (e & 15);
    if (r >= J || c >= J) return;
    if (bi == bj && r > c) return;  // diagonal blocks: upper triangle only, then mirror
    double acc = 0.0;
    for (int q = 0; q < P; ++q) acc += partial[(int64_t)q * npairs * 256 + idx];
    s[r + (int64_t)J * c] = acc;
    s[c + (int64_t)J * r] = acc;
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

// ------------------------------------------------------------------ host

static int round_jb(int J) {
    int jb = 32;
    while (jb < J) jb *= 2;
    return jb;
}

GramPlan plan_gram(const ModeView& v, int precision, int elem_bytes) {
    (void)precision;
    (void)elem_bytes;
    GramPlan pl{};
    int jb = round_jb(v.J);
    pl.KT = jb >= 512 ? 16 : 32;
    pl.nb = (v.J + 15) / 16;
    pl.npairs = pl.nb * (pl.nb + 1) / 2;
    int per_group = kGramWaves * kGramMaxPairs;
    pl.G = (pl.npairs + per_group - 1) / per_group;
    pl.pairs_per_group = (pl.npairs + pl.G - 1) / pl.G;
    TileMap tm = make_tiles(v, pl.KT);
    int cus = device_cu_count();
    int64_t want = (int64_t)2 * cus / pl.G;
    if (want < 1) want = 1;
    pl.P = (int)(tm.ntiles < want ? tm.ntiles : want);
    if (pl.P < 1) pl.P = 1;
    pl.partial_bytes = (size_t)pl.P * pl.npairs * 256 * sizeof(double);
    return pl;
}

template <typename T, int JB, int KT>
static int launch_partial(const T* y, const TileMap& tm, const GramPlan& pl, double* partial,
                          hipStream_t st) {
    size_t lds = (size_t)kGramLdsDoubles<JB, KT> * sizeof(double);
    auto fn = gram_partial_f64<T, JB, KT>;
    TK_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
    hipLaunchKernelGGL(fn, dim3(pl.P, pl.G), dim3(kGramThreads), lds, st, y, tm, pl.nb, pl.npairs,
                       pl.pairs_per_group, partial);
    TK_HIP(hipGetLastError());
    return TK_OK;
}

template <typename T>
static int dispatch_partial(const T* y, const ModeView& v, const GramPlan& pl, double* partial,
                            hipStream_t st) {
    TileMap tm = make_tiles(v, pl.KT);
    int jb = round_jb(v.J);
    switch (jb) {
        case 32: return launch_partial<T, 32, 32>(y, tm, pl, partial, st);
        case 64: return launch_partial<T, 64, 32>(y, tm, pl, partial, st);
        case 128: return launch_partial<T, 128, 32>(y, tm, pl, partial, st);
        case 256: return launch_partial<T, 256, 32>(y, tm, pl, partial, st);
        case 512: return launch_partial<T, 512, 16>(y, tm, pl, partial, st);
        default: return fail(TK_ERR_UNSUPPORTED, "mode extent %d exceeds %d", v.J, TK_MAX_MODE_DIM);
    }
}

int launch_gram_mixed(const float* y, const ModeView& v, double* s, void* ws, size_t ws_bytes,
                      hipStream_t st);

int launch_gram(const void* y, int dtype, const ModeView& v, int precision, double* s,
                double* sumsq, void* ws, size_t ws_bytes, hipStream_t st) {
    if (precision == TK_GRAM_SPLIT_BF16) {
        TK_TRY(launch_gram_mixed((const float*)y, v, s, ws, ws_bytes, st));
    } else {
        GramPlan pl = plan_gram(v, precision, (int)dtype_size(dtype));
        if (ws_bytes < pl.partial_bytes)
            return fail(TK_ERR_WORKSPACE, "gram workspace %zu < %zu", ws_bytes, pl.partial_bytes);
        double* partial = (double*)ws;
        if (dtype == TK_F64) {
            TK_TRY(dispatch_partial((const double*)y, v, pl, partial, st));
        } else {
            TK_TRY(dispatch_partial((const float*)y, v, pl, partial, st));
        }
        int n = pl.npairs * 256;
        hipLaunchKernelGGL(gram_reduce, dim3((n + 255) / 256), dim3(256), 0, st, partial, pl.P,
                           pl.npairs, pl.nb, v.J, s);
        TK_HIP(hipGetLastError());
    }
    if (sumsq) {
        hipLaunchKernelGGL(gram_trace, dim3(1), dim3(64), 0, st, s, v.J, sumsq);
        TK_HIP(hipGetLastError());
    }
    return TK_OK;
}

}  // namespace tk
