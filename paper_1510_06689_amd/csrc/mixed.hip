// Mixed-precision kernels for FP32-stored tensors: the split-bf16 Gram and
// the bf16 / split-bf16 TTM.  Neither changes what Alg. 1 computes; they
// change the arithmetic of its two bulk steps (Gram, TTM) while the
// eigendecomposition and the rank rule stay in FP64.
//
// Split-bf16 Gram.  The rank rule compares tail sums of eigenvalues with
// eps^2 ||X||^2 / N, so the Gram's error in the trailing eigenvalues must
// stay far below that threshold.  Rounding inside the products would not
// (dropping lo*lo, or rounding FP32 partial sums, leaves errors that do not
// average out of the trailing eigenvalues).  Hence every product and sum on
// the matrix cores is exact: per tile of KT columns and per row i with
// max |x| < 2^E_i, s = x 2^(7 - E_i) is rounded to the grid 2^-8 (16-bit
// fixed point) and split into two 8-bit halves
//     hi = round(s)                        an integer in [-128, 128]
//     lo = round(256 (s - hi)) / 256       256 lo an integer in [-128, 128]
// both exact in bf16, and a 32x32 block of S = Y_(n) Y_(n)^T is
//     2^(E_i + E_j - 14) (H_i H_j^T + [H_i L_j^T + L_i H_j^T] + L_i L_j^T)
// on v_mfma_f32_32x32x16_bf16, the three terms in three FP32 accumulators:
// over at most 128 columns each sum is an integer multiple of its quantum
// (1, 2^-8, 2^-16) below 2^22 of it, so exact.  They are scaled and added
// into FP64 registers after every tile.  What remains is the quantization
// error d = s - hi - lo, |d| <= 2^-9, of every element: the split Gram is
// exactly Y~ Y~^T with Y~ = Y - D.  Quantization noise independent of the
// data adds its energy to the diagonal, so sum_k d_ik^2 (formed exactly
// per element) is subtracted from S_ii; the rest of D's contribution has
// mean zero (see EigArgs::guard for the model and the bound it gives).
// Partials use the FP64 Gram's 16x16 pair layout and its fixed-order
// reduction.
//
// bf16 TTM.  Z = op(M) Y with op(M) (K x J) split into bf16 hi/lo fragments
// once per workgroup (in LDS) and Y split per element as it is loaded:
// BF16 forms A_hi Y_hi; BF16X3 adds A_hi Y_lo + A_lo Y_hi
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation, FP32 output).  When the
// columns are contiguous (mode 1) every lane loads its eight consecutive
// rows straight from HBM, no LDS staging needed.
#include <algorithm>

#include "tk_common.hpp"

namespace tk {

typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef float f16_t __attribute__((ext_vector_type(16)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef int i4_t __attribute__((ext_vector_type(4)));

// ================================================================== Gram

constexpr int kMxThreads = 512;
constexpr int kMxWaves = kMxThreads / 64;

// Loader modes.
enum { kUnit = 0, kContig = 1, kStrided = 2 };

template <int CTRL>
__device__ __forceinline__ unsigned dpp_max(unsigned v) {
    const unsigned o = (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xf, 0xf, false);
    return o > v ? o : v;
}

// One J x KT tile of FP32 columns, held by the workgroup in registers as
// groups of eight consecutive columns of one row, split as described above
// and stored to LDS as two [JB][KT + 8] bf16 planes (a 16-byte row pad keeps
// the 16-byte fragment reads and writes free of bank conflicts) plus the
// JB row exponents.  Every row's groups sit in one wave, so the row maximum
// is a reduction among a few lanes, with no barrier:
//   kUnit    (L == 1): wave w owns rows [w RW, w RW + RW); lane l holds row
//            l % RW, groups l / RW + m (64 / RW).  A load instruction reads
//            RW consecutive rows (contiguous) of 64 / RW columns.
//   kContig  (L % 8 == 0, 16-byte aligned): lane group of KT / 8 consecutive
//            threads owns one row, thread t the column group t % (KT / 8);
//            each group is two 16-byte loads.
//   kStrided (otherwise): as kContig, one element per load.
template <int JB, int KT, int MODE>
struct SplitTile {
    static constexpr int PK = KT + 8;
    static constexpr int NCG = KT / 8;                              // groups per row
    static constexpr int RW = JB / kMxWaves > 16 ? JB / kMxWaves : 16;  // kUnit rows per wave
    static constexpr int LPR = 64 / RW;                             // kUnit lanes per row
    static constexpr int ROWSTEP = kMxThreads / NCG;                // strided rows per pass
    static constexpr int NGRP = MODE == kUnit ? NCG / LPR : JB * NCG / kMxThreads;
    static_assert(RW <= 64 && NCG % LPR == 0, "unit mapping");
    static_assert(MODE == kUnit || (NGRP >= 1 && JB * NCG % kMxThreads == 0 && NCG <= 16),
                  "strided mapping");

    float v[NGRP][8];
    int i0, cg0;
    bool owner;      // kUnit: this wave holds rows
    int coff[8];     // strided: offsets of the thread's 8 columns inside a tile
    // Representation error of the split: per row of the thread, the sum of
    // d^2 over its elements, d = x - 2^(E-7) (hi + lo) exactly, and the
    // largest row exponent E it used.
    static constexpr int NROW = MODE == kUnit ? 1 : NGRP;
    double rd[NROW];
    int emax;

    __device__ static __forceinline__ int64_t col_offset(int kk, int64_t L, int J) {
        const int64_t bb = kk / L;
        return bb * J * L + (kk - bb * L);
    }

    __device__ __forceinline__ void setup(const TileMap& tm, int tid) {
#pragma unroll
        for (int m = 0; m < NROW; ++m) rd[m] = 0.0;
        emax = -125;
        if (MODE == kUnit) {
            const int w = tid >> 6, l = tid & 63;
            owner = w * RW < JB;
            i0 = w * RW + l % RW;
            cg0 = l / RW;
        } else {
            owner = true;
            cg0 = tid % NCG;
            i0 = tid / NCG;
#pragma unroll
            for (int e = 0; e < 8; ++e) coff[e] = (int)col_offset(8 * cg0 + e, tm.L, tm.J);
        }
    }
    __device__ __forceinline__ int row_of(int m) const {
        return MODE == kUnit ? i0 : i0 + m * ROWSTEP;
    }
    __device__ __forceinline__ int cg_of(int m) const {
        return MODE == kUnit ? cg0 + m * LPR : cg0;
    }

    __device__ __forceinline__ void load(const float* __restrict__ y, const TileMap& tm,
                                         const Tile& t) {
        const int J = tm.J;
        if (MODE == kUnit) {
            // element (i0, kk) with kk = 8 cg0 + [8 m LPR + e]: a wave-uniform
            // column part plus a fixed per-lane 32-bit offset
            const bool ok = owner && i0 < J;
            const int loff = i0 + 8 * cg0 * J;
#pragma unroll
            for (int m = 0; m < NGRP; ++m) {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int ku = 8 * m * LPR + e;
                    const float* ub = y + t.base + (int64_t)ku * J;
                    v[m][e] = (ok && 8 * cg0 + ku < t.ncols) ? ub[loff] : 0.f;
                }
            }
        } else {
#pragma unroll
            for (int m = 0; m < NGRP; ++m) {
                const int i = row_of(m);
                const int64_t rowbase = t.base + (int64_t)i * tm.L;
                if (MODE == kContig && i < J && 8 * cg0 + 8 <= t.ncols) {
                    const f4_t* p = (const f4_t*)(y + rowbase + coff[0]);
                    const f4_t a = p[0], b = p[1];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        v[m][e] = a[e];
                        v[m][4 + e] = b[e];
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int kk = 8 * cg0 + e;
                        v[m][e] = (i < J && kk < t.ncols) ? y[rowbase + coff[e]] : 0.f;
                    }
                }
            }
        }
    }

    // Largest |x| of the row of group m over the whole tile (as float bits).
    __device__ __forceinline__ unsigned row_max_bits(int m) const {
        unsigned b = 0;
        if (MODE == kUnit) {
#pragma unroll
            for (int q = 0; q < NGRP; ++q)
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const unsigned u = __float_as_uint(v[q][e]) & 0x7fffffffu;
                    b = u > b ? u : b;
                }
#pragma unroll
            for (int d = RW; d < 64; d *= 2) {
                const unsigned o = (unsigned)__shfl_xor((int)b, d);
                b = o > b ? o : b;
            }
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const unsigned u = __float_as_uint(v[m][e]) & 0x7fffffffu;
                b = u > b ? u : b;
            }
            // max over the NCG (aligned, consecutive) lanes of the row
            if (NCG >= 2) b = dpp_max<0xb1>(b);    // quad_perm [1,0,3,2]
            if (NCG >= 4) b = dpp_max<0x4e>(b);    // quad_perm [2,3,0,1]
            if (NCG >= 8) b = dpp_max<0x141>(b);   // row_half_mirror
            if (NCG >= 16) b = dpp_max<0x140>(b);  // row_mirror
        }
        return b;
    }

    // Split and store the tile; the row exponents go next to the planes.
    // The residual x 2^(7-E) - hi - lo of every element is formed exactly in
    // FP32 (the bf16 rounding error of lo) and its square summed, rescaled
    // by 2^(2 (E-7)) per row.
    __device__ __forceinline__ void store(__bf16* hi, __bf16* lo, int* ex) {
        unsigned mb = 0;
        if (MODE == kUnit) mb = row_max_bits(0);  // every group of the thread is one row
        float rs = 0.f;                            // kUnit: the row's scaled sum of d^2
        int sh = 0;
#pragma unroll
        for (int m = 0; m < NGRP; ++m) {
            if (MODE != kUnit || m == 0) {
                if (MODE != kUnit) mb = row_max_bits(m);
                // max |x| < 2^E; zero rows get the smallest normal exponent
                const int E = (int)(mb >> 23) - 126;
                sh = 7 - (E < -125 ? -125 : E);
            }
            bf8_t h, l;
            float gs = 0.f;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                // s = x 2^(7-E) rounded to the grid 2^-8: h + l, h and 256 l
                // integers in [-128, 128] (exact in bf16); d = s - h - l exactly
                const float sx = __builtin_ldexpf(v[m][e], sh);
                const float hv = __builtin_rintf(sx);
                const float r = sx - hv;
                const float lv = __builtin_rintf(r * 256.f) * 0.00390625f;
                h[e] = (__bf16)hv;
                l[e] = (__bf16)lv;
                const float dd = r - lv;
                gs = __builtin_fmaf(dd, dd, gs);
            }
            const int r = row_of(m);
            const bool mine = MODE != kUnit || owner;
            if (mine) {
                const int off = r * PK + 8 * cg_of(m);
                *(bf8_t*)(hi + off) = h;
                *(bf8_t*)(lo + off) = l;
                if (cg_of(m) == 0) ex[r] = 7 - sh;
            }
            if (MODE == kUnit) {
                rs += gs;
            } else if (r < JB) {
                rd[m] += __builtin_ldexp((double)gs, -2 * sh);
                emax = max(emax, 7 - sh);
            }
        }
        if (MODE == kUnit && owner) {
            rd[0] += __builtin_ldexp((double)rs, -2 * sh);
            emax = max(emax, 7 - sh);
        }
    }

    // Per-row sums of d^2 over the workgroup into rowd[0..JB) (each row's
    // holders form a fixed xor-butterfly; rows nobody holds stay as set).
    __device__ __forceinline__ void row_sums(double* rowd, int lane) const {
        if (MODE == kUnit) {
            double v = rd[0];
#pragma unroll
            for (int d = RW; d < 64; d *= 2) v += __shfl_xor(v, d);
            if (owner && lane < RW) rowd[i0] = v;
        } else {
#pragma unroll
            for (int m = 0; m < NROW; ++m) {
                double v = rd[m];
#pragma unroll
                for (int d = 1; d < NCG; d *= 2) v += __shfl_xor(v, d);
                if (cg0 == 0) rowd[row_of(m)] = v;
            }
        }
    }
    __device__ __forceinline__ double total() const {
        double t = 0.0;
#pragma unroll
        for (int m = 0; m < NROW; ++m) t += rd[m];
        return t;
    }
};

// Pair index p -> (bi, bj), upper-triangle 32-blocks in row-major order.
__device__ __forceinline__ void pair32_of(int p, int nb, int& bi, int& bj) {
    int row = 0, start = 0;
    while (p >= start + (nb - row)) {
        start += nb - row;
        ++row;
    }
    bi = row;
    bj = row + (p - start);
}

// One LDS tile buffer: hi plane, lo plane (bf16 [JB][KT + 8]) and JB row
// exponents; two buffers alternate.
template <int JB, int KT>
constexpr size_t mx_buf_bytes() {
    return ((size_t)2 * JB * (KT + 8) * sizeof(__bf16) + (size_t)JB * sizeof(int) + 15) / 16 * 16;
}

// Every 32-block pair of the workgroup's pair group has one owner wave
// (pair g0 + wave + 8 q, q < NPW), which sees every column of every tile, so
// each output lives in exactly one wave's registers.
//
// The body processes tiles [t0, t1) of pair group `group` and writes its
// partial (npairs16 x 256 doubles) to `out`; the single-tensor kernel and the
// batched kernel differ only in how they find those.
// Sum of d over the workgroup (fixed order: lanes by xor butterfly, then
// waves by index) and max of e; thread 0 writes {sum, max} to aux.
__device__ __forceinline__ void split_stats_out(double d, int e, double* aux, double* lds) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        d += __shfl_xor(d, o);
        e = max(e, __shfl_xor(e, o));
    }
    int* le = (int*)(lds + kMxWaves);
    if (lane == 0) {
        lds[wave] = d;
        le[wave] = e;
    }
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        int m = -125;
        const int nw = (int)(blockDim.x >> 6);  // at most kMxWaves
        for (int w = 0; w < nw; ++w) {
            t += lds[w];
            m = max(m, le[w]);
        }
        aux[0] = t;
        aux[1] = (double)m;
    }
}

// aux (may be NULL): receives {sum of d^2, largest row exponent} of the split
// representation of the tiles this workgroup processed.
template <int JB, int KT, int NPW, int MODE>
__device__ __forceinline__ void gram_bf16s_body(
    const float* __restrict__ y, const TileMap& tm, int npairs32, int pairs_per_group,
    int npairs16, int group, int64_t t0, int64_t t1, double* __restrict__ out,
    double* aux, double* lds_raw) {
    using Ld = SplitTile<JB, KT, MODE>;
    constexpr int PK = Ld::PK;
    constexpr int PLANE = JB * PK;
    constexpr size_t BUF = mx_buf_bytes<JB, KT>();
    constexpr int NKS = KT / 16;
    constexpr int NB = JB / 32;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r32 = lane & 31, kh = lane >> 5;
    const int g0 = group * pairs_per_group;

    int bi[NPW], bj[NPW], aoff[NPW], boff[NPW];
    bool act[NPW];
#pragma unroll
    for (int q = 0; q < NPW; ++q) {
        const int pl = wave + q * kMxWaves;
        const int p = g0 + pl;
        act[q] = pl < pairs_per_group && p < npairs32;
        pair32_of(act[q] ? p : 0, NB, bi[q], bj[q]);
        aoff[q] = (32 * bi[q] + r32) * PK + 8 * kh;
        boff[q] = (32 * bj[q] + r32) * PK + 8 * kh;
    }

    f16_t acch[NPW], accm[NPW], accl[NPW];
    double accd[NPW][16];
#pragma unroll
    for (int q = 0; q < NPW; ++q) {
#pragma unroll
        for (int v = 0; v < 16; ++v) accd[q][v] = 0.0;
    }

    char* base = (char*)lds_raw;
    auto hi_of = [&](int b) { return (__bf16*)(base + b * BUF); };
    auto ex_of = [&](int b) { return (int*)(base + b * BUF + 2 * PLANE * sizeof(__bf16)); };

    Ld ld;
    ld.setup(tm, tid);
    if (t0 < t1) {
        ld.load(y, tm, tile_at(tm, t0, tm.J));
        ld.store(hi_of(0), hi_of(0) + PLANE, ex_of(0));
    }
    __syncthreads();
    for (int64_t t = t0; t < t1; ++t) {
        const int cur = (int)((t - t0) & 1);
        const bool more = t + 1 < t1;
        if (more) ld.load(y, tm, tile_at(tm, t + 1, tm.J));  // in flight during the MFMAs
        const __bf16* hb = hi_of(cur);
        const __bf16* lb = hb + PLANE;
        const int* ex = ex_of(cur);
#pragma unroll
        for (int q = 0; q < NPW; ++q) {
            if (!act[q]) continue;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                acch[q][v] = 0.f;
                accm[q][v] = 0.f;
                accl[q][v] = 0.f;
            }
#pragma unroll 2
            for (int ks = 0; ks < NKS; ++ks) {
                const bf8_t ah = *(const bf8_t*)(hb + aoff[q] + 16 * ks);
                const bf8_t al = *(const bf8_t*)(lb + aoff[q] + 16 * ks);
                const bf8_t bh = *(const bf8_t*)(hb + boff[q] + 16 * ks);
                const bf8_t bl = *(const bf8_t*)(lb + boff[q] + 16 * ks);
                acch[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acch[q], 0, 0, 0);
                accm[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, accm[q], 0, 0, 0);
                accm[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, accm[q], 0, 0, 0);
                accl[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bl, accl[q], 0, 0, 0);
            }
            // v_mfma_f32_32x32x16: row (v / 4) * 8 + (lane / 32) * 4 + v % 4, column lane % 32
            const int ej = ex[32 * bj[q] + r32] - 14;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const i4_t ei = *(const i4_t*)(ex + 32 * bi[q] + 8 * g + 4 * kh);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int v = 4 * g + c;
                    const double sv = (double)acch[q][v] + ((double)accm[q][v] + (double)accl[q][v]);
                    accd[q][v] += __builtin_ldexp(sv, ei[c] + ej);
                }
            }
        }
        if (more) {
            const int nb2 = cur ^ 1;
            ld.store(hi_of(nb2), hi_of(nb2) + PLANE, ex_of(nb2));
        }
        __syncthreads();
    }

    // With D = Y - Y~ (Y~ the split representation) the products form
    // Y~ Y~^T = Y Y^T - Y D^T - D Y^T + D D^T: rounding errors independent of
    // the data add their energy, diag(D D^T), to the diagonal, which would
    // raise every tail sum by about ||D||_F^2 (J - R) / J.  That diagonal,
    // sum_k d_ik^2, is known exactly per row and is subtracted here; what
    // remains (Y D^T + D Y^T and the off-diagonal of D D^T) has mean 0.
    double* rowd = lds_raw + 64;  // past split_stats_out's slots
    for (int i = tid; i < JB; i += kMxThreads) rowd[i] = 0.0;
    __syncthreads();
    ld.row_sums(rowd, lane);
    __syncthreads();
    constexpr int NB16 = 2 * NB;
#pragma unroll
    for (int q = 0; q < NPW; ++q) {
        if (!act[q]) continue;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int row = (v >> 2) * 8 + kh * 4 + (v & 3);
            const int gi = 32 * bi[q] + row, gj = 32 * bj[q] + r32;
            const int BI = gi >> 4, BJ = gj >> 4;
            if (BI > BJ) continue;  // lower half of a diagonal 32-block
            const int p16 = BI * NB16 - BI * (BI - 1) / 2 + (BJ - BI);
            out[(int64_t)p16 * 256 + (gi & 15) * 16 + (gj & 15)] =
                gi == gj ? accd[q][v] - rowd[gi] : accd[q][v];
        }
    }
    if (aux) split_stats_out(ld.total(), ld.emax, aux, lds_raw);  // uniform branch
}

// P tile ranges x G pair groups, one workgroup each (xcd_range_group).  The
// P x 2 split statistics follow the P partials; pair group 0 writes them.
template <int JB, int KT, int NPW, int MODE>
__global__ __launch_bounds__(kMxThreads) void gram_partial_bf16s(
    const float* __restrict__ y, TileMap tm, int npairs32, int pairs_per_group, int npairs16,
    int P, int G, double* __restrict__ partial) {
    extern __shared__ double lds_raw[];
    int p, g;
    xcd_range_group(blockIdx.x, G, p, g);
    const int64_t t0 = tm.ntiles * (int64_t)p / P;
    const int64_t t1 = tm.ntiles * (int64_t)(p + 1) / P;
    double* aux = g == 0 ? partial + (int64_t)P * npairs16 * 256 + 2 * p : nullptr;
    gram_bf16s_body<JB, KT, NPW, MODE>(y, tm, npairs32, pairs_per_group, npairs16, g, t0, t1,
                                      partial + (int64_t)p * npairs16 * 256, aux, lds_raw);
}

// Static schedule per padded extent: tile width, pairs per wave, pair groups
// (each re-reads the tensor), workgroups per CU.
struct MxGramShape {
    int KT, NPW, G, per_cu;
};
template <int JB>
constexpr MxGramShape mx_gram_shape() {
    return JB == 32    ? MxGramShape{128, 1, 1, 2}   //   1 pair
           : JB == 64  ? MxGramShape{128, 1, 1, 2}   //   3 pairs
           : JB == 128 ? MxGramShape{128, 2, 1, 1}   //  10 pairs over 8 waves
           : JB == 256 ? MxGramShape{64, 2, 3, 1}    //  36 pairs: 3 groups of 12
                       : MxGramShape{16, 2, 9, 1};   // 136 pairs: 9 groups of 16
}

static int mx_round_jb(int J) {
    int jb = 32;
    while (jb < J) jb *= 2;
    return jb;
}

template <int JB>
static GramPlan mx_plan(const ModeView& v) {
    constexpr MxGramShape gs = mx_gram_shape<JB>();
    static_assert(kMxWaves * gs.NPW * gs.G >= JB / 32 * (JB / 32 + 1) / 2 &&
                      kMxWaves * gs.NPW >= (JB / 32 * (JB / 32 + 1) / 2 + gs.G - 1) / gs.G,
                  "every pair of a group needs an owner wave");
    GramPlan pl{};
    TileMap tm = make_tiles(v, gs.KT);
    const int nb32 = JB / 32;
    const int npairs32 = nb32 * (nb32 + 1) / 2;
    pl.KT = gs.KT;
    pl.G = gs.G;
    pl.pairs_per_group = (npairs32 + gs.G - 1) / gs.G;
    pl.nb = 2 * nb32;  // 16-blocks, for the shared reduction
    pl.npairs = pl.nb * (pl.nb + 1) / 2;
    const int64_t want = xcd_round_want((int64_t)gs.per_cu * device_cu_count() / pl.G, pl.G);
    pl.P = xcd_ranges(tm.ntiles, want, pl.G);
    // partials, then 2 doubles of split statistics per tile range
    pl.partial_bytes = (size_t)pl.P * (pl.npairs * 256 + 2) * sizeof(double);
    pl.partial_bound = (size_t)want * (pl.npairs * 256 + 2) * sizeof(double);
    return pl;
}

GramPlan plan_gram_mixed(const ModeView& v) {
    switch (mx_round_jb(v.J)) {
        case 32: return mx_plan<32>(v);
        case 64: return mx_plan<64>(v);
        case 128: return mx_plan<128>(v);
        case 256: return mx_plan<256>(v);
        default: return mx_plan<512>(v);
    }
}

template <int JB, int MODE>
static int mx_launch(const float* y, const TileMap& tm, const GramPlan& pl, double* partial,
                     hipStream_t st) {
    constexpr MxGramShape gs = mx_gram_shape<JB>();
    auto fn = gram_partial_bf16s<JB, gs.KT, gs.NPW, MODE>;
    const size_t lds = 2 * mx_buf_bytes<JB, gs.KT>();
    TK_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
    const int nb32 = JB / 32;
    hipLaunchKernelGGL(fn, dim3(pl.P * pl.G), dim3(kMxThreads), lds, st, y, tm,
                       nb32 * (nb32 + 1) / 2, pl.pairs_per_group, pl.npairs, pl.P, pl.G, partial);
    TK_HIP(hipGetLastError());
    return TK_OK;
}

template <int JB>
static int mx_dispatch_mode(const float* y, const ModeView& v, const GramPlan& pl,
                            double* partial, hipStream_t st) {
    TileMap tm = make_tiles(v, pl.KT);
    if (v.L == 1) return mx_launch<JB, kUnit>(y, tm, pl, partial, st);
    const bool contig = v.L % 8 == 0 && ((uintptr_t)y & 15) == 0;
    if (contig) return mx_launch<JB, kContig>(y, tm, pl, partial, st);
    return mx_launch<JB, kStrided>(y, tm, pl, partial, st);
}

// ---- batches: one launch covers every problem of a batch ----------------
template <int JB>
__global__ __launch_bounds__(kMxThreads) void gram_bf16s_batched(
    const BatchGramTask* __restrict__ tasks, int ntasks) {
    extern __shared__ double lds_raw[];
    constexpr MxGramShape gs = mx_gram_shape<JB>();
    const int ti = find_task_wg(&tasks[0].v, sizeof(BatchGramTask), ntasks, blockIdx.x);
    const BatchGramTask tk = tasks[ti];
    const int w = blockIdx.x - tk.v.wg_begin;
    const ModeView mv = batch_mode_view(tk.v);
    const TileMap tm = make_tiles(mv, gs.KT);
    // workgroups needed at the actual shape (>= 1: a shape has >= 1 tile)
    const int64_t need = (tm.ntiles + tk.tpw - 1) / tk.tpw;
    const int active = (int)(need < tk.v.nwg ? need : tk.v.nwg);
    if (w == 0 && threadIdx.x == 0) *tk.nparts = active;
    if (w >= active) return;  // uniform over the workgroup
    const int64_t t0 = tm.ntiles * (int64_t)w / active;
    const int64_t t1 = tm.ntiles * (int64_t)(w + 1) / active;
    constexpr int nb32 = JB / 32, np32 = nb32 * (nb32 + 1) / 2, np16 = 2 * nb32 * (2 * nb32 + 1) / 2;
    double* out = tk.partial + (int64_t)w * np16 * 256;
    double* aux = tk.aux + 2 * w;
    if (mv.L == 1)
        gram_bf16s_body<JB, gs.KT, gs.NPW, kUnit>(tk.y, tm, np32, np32, np16, 0, t0, t1, out,
                                                  aux, lds_raw);
    else if (mv.L % 8 == 0 && ((uintptr_t)tk.y & 15) == 0)
        gram_bf16s_body<JB, gs.KT, gs.NPW, kContig>(tk.y, tm, np32, np32, np16, 0, t0, t1, out,
                                                    aux, lds_raw);
    else
        gram_bf16s_body<JB, gs.KT, gs.NPW, kStrided>(tk.y, tm, np32, np32, np16, 0, t0, t1, out,
                                                     aux, lds_raw);
}

int mx_gram_kt(int jb) {
    switch (jb) {
        case 32: return mx_gram_shape<32>().KT;
        case 64: return mx_gram_shape<64>().KT;
        case 128: return mx_gram_shape<128>().KT;
        case 256: return mx_gram_shape<256>().KT;
        default: return mx_gram_shape<512>().KT;
    }
}

template <int JB>
static int launch_bf16s_batched_t(const BatchGramTask* tasks, int ntasks, int total_wg,
                                  hipStream_t st) {
    static_assert(mx_gram_shape<JB>().G == 1, "batches need a single pair group");
    auto fn = gram_bf16s_batched<JB>;
    const size_t lds = 2 * mx_buf_bytes<JB, mx_gram_shape<JB>().KT>();
    TK_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
    hipLaunchKernelGGL(fn, dim3(total_wg), dim3(kMxThreads), lds, st, tasks, ntasks);
    TK_HIP(hipGetLastError());
    return TK_OK;
}

int launch_gram_bf16s_batched(const BatchGramTask* tasks_dev, int ntasks, int total_wg, int jb,
                              hipStream_t st) {
    switch (jb) {
        case 32: return launch_bf16s_batched_t<32>(tasks_dev, ntasks, total_wg, st);
        case 64: return launch_bf16s_batched_t<64>(tasks_dev, ntasks, total_wg, st);
        case 128: return launch_bf16s_batched_t<128>(tasks_dev, ntasks, total_wg, st);
        default: return fail(TK_ERR_UNSUPPORTED, "batched split Gram: extent class %d", jb);
    }
}

int launch_gram_mixed(const float* y, const ModeView& v, const GramPlan& pl, double* partial,
                      hipStream_t st) {
    switch (mx_round_jb(v.J)) {
        case 32: return mx_dispatch_mode<32>(y, v, pl, partial, st);
        case 64: return mx_dispatch_mode<64>(y, v, pl, partial, st);
        case 128: return mx_dispatch_mode<128>(y, v, pl, partial, st);
        case 256: return mx_dispatch_mode<256>(y, v, pl, partial, st);
        case 512: return mx_dispatch_mode<512>(y, v, pl, partial, st);
        default: return fail(TK_ERR_UNSUPPORTED, "mode extent %d exceeds %d", v.J, TK_MAX_MODE_DIM);
    }
}

// ================================================================== TTM

constexpr int kMtThreads = 256;
constexpr int kMtWaves = kMtThreads / 64;

// NKB: 16-row blocks of op(M) per workgroup; NKS: 32-wide k-steps over J;
// X3: split both operands (three products) instead of one bf16 product.
// UNIT: columns contiguous (L == 1, J % 8 == 0), loaded as 16-byte vectors.
// SKIP: row blocks at or beyond K skip their products (a batch sizes NKB for
// the rank capacity, the rank comes later from the device).
// The body stages rows [r0, r0 + 16 NKB) of op(M) and walks column blocks
// wg, wg + nwg, ... (one block of 16 columns per wave at a time).
template <int NKB, int NKS, bool X3, bool UNIT, bool SKIP = false>
__device__ __forceinline__ void ttm_bf16_body(
    const float* __restrict__ y, int64_t L, int64_t ncols, int J, const double* __restrict__ m,
    int64_t ldm, int K, int transpose, float* __restrict__ z, int r0, int64_t wg, int64_t nwg,
    bf8_t (*afr)[64]) {
    const int tid = threadIdx.x, lane = tid & 63;

    // A fragments: lane l holds op(M)[r0 + 16 kb + l % 16][32 ks + 8 (l / 16) + e].
    for (int f = tid; f < NKB * NKS * 64; f += kMtThreads) {
        const int l = f & 63, kbks = f >> 6;
        const int kb = kbks / NKS, ks = kbks - (kbks / NKS) * NKS;
        const int r = r0 + 16 * kb + (l & 15);
        bf8_t h, lo;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int j = 32 * ks + 8 * (l >> 4) + e;
            double a = 0.0;
            if (r < K && j < J) a = transpose ? m[j + ldm * r] : m[r + ldm * j];
            const float af = (float)a;
            const __bf16 ah = (__bf16)af;
            h[e] = ah;
            lo[e] = (__bf16)(af - (float)ah);
        }
        afr[kbks * 2][l] = h;
        afr[kbks * 2 + 1][l] = lo;
    }
    __syncthreads();

    const int c16 = lane & 15, g4 = lane >> 4;
    // row blocks that hold rows < K: the others' products are never stored
    const int nkb = min(NKB, (K - r0 + 15) / 16);
    const int64_t nblk = (ncols + 15) / 16;
    const int64_t wstride = nwg * kMtWaves;
    const int64_t JL = (int64_t)J * L, KL = (int64_t)K * L;
    for (int64_t cb = wg * kMtWaves + (tid >> 6); cb < nblk; cb += wstride) {
        const int64_t col = cb * 16 + c16;
        const bool cv = col < ncols;
        int64_t b = 0, l = 0;
        if (!UNIT) {
            b = col / L;
            l = col - b * L;
        }
        const float* ycol = UNIT ? y + col * J : y + b * JL + l;
        f4_t acc[NKB];
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb) acc[kb] = f4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) {
            const int j0 = 32 * ks + 8 * g4;
            float x[8];
            if (UNIT) {
                if (cv && j0 < J) {
                    const f4_t* p = (const f4_t*)(ycol + j0);
                    const f4_t a = p[0], c = p[1];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        x[e] = a[e];
                        x[4 + e] = c[e];
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < 8; ++e) x[e] = 0.f;
                }
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    x[e] = (cv && j0 + e < J) ? ycol[(int64_t)(j0 + e) * L] : 0.f;
            }
            bf8_t yh, yl;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const __bf16 h = (__bf16)x[e];
                yh[e] = h;
                if (X3) yl[e] = (__bf16)(x[e] - (float)h);
            }
#pragma unroll
            for (int kb = 0; kb < NKB; ++kb) {
                if constexpr (SKIP && NKB > 1) {
                    if (kb >= nkb) break;  // uniform over the workgroup
                }
                const bf8_t ah = afr[(kb * NKS + ks) * 2][lane];
                acc[kb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, yh, acc[kb], 0, 0, 0);
                if (X3) {
                    const bf8_t al = afr[(kb * NKS + ks) * 2 + 1][lane];
                    acc[kb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, yl, acc[kb], 0, 0, 0);
                    acc[kb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, yh, acc[kb], 0, 0, 0);
                }
            }
        }
        if (!cv) continue;
        // v_mfma_f32_16x16x32: row 4 * (lane / 16) + v, column lane % 16
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb) {
            const int rb = r0 + 16 * kb + 4 * g4;
            if (UNIT) {
                float* zc = z + col * K;
                if (rb + 4 <= K && (K & 3) == 0) {
                    *(f4_t*)(zc + rb) = acc[kb];
                } else {
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        if (rb + v < K) zc[rb + v] = acc[kb][v];
                }
            } else {
                float* zc = z + b * KL + l;
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (rb + v < K) zc[(int64_t)(rb + v) * L] = acc[kb][v];
            }
        }
    }
}

template <int NKB, int NKS, bool X3, bool UNIT>
__global__ __launch_bounds__(kMtThreads) void ttm_bf16_kernel(
    const float* __restrict__ y, int64_t L, int64_t ncols, int J, const double* __restrict__ m,
    int64_t ldm, int K, int transpose, float* __restrict__ z) {
    __shared__ bf8_t afr[NKB * NKS * 2][64];  // [(kb * NKS + ks) * 2 + hi/lo][lane]
    ttm_bf16_body<NKB, NKS, X3, UNIT>(y, L, ncols, J, m, ldm, K, transpose, z,
                                      blockIdx.y * NKB * 16, blockIdx.x, gridDim.x, afr);
}

template <int NKB, int NKS, bool X3>
static int mt_launch(const float* y, const ModeView& v, const double* m, int64_t ldm, int K,
                     int transpose, float* z, hipStream_t st) {
    const int64_t ncols = v.L * v.B;
    const bool unit = v.L == 1 && v.J % 8 == 0 && ((uintptr_t)y & 15) == 0 &&
                      ((uintptr_t)z & 15) == 0;
    const int G = (K + NKB * 16 - 1) / (NKB * 16);
    auto fn = unit ? ttm_bf16_kernel<NKB, NKS, X3, true> : ttm_bf16_kernel<NKB, NKS, X3, false>;
    int per_cu = 1;
    TK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)fn, kMtThreads, 0));
    if (per_cu < 1) per_cu = 1;
    const int64_t nblk = (ncols + 15) / 16;
    int64_t want = ((int64_t)per_cu * device_cu_count() + G - 1) / G;
    int64_t P = (nblk + kMtWaves - 1) / kMtWaves;
    if (P > want) P = want;
    if (P < 1) return TK_OK;
    hipLaunchKernelGGL(fn, dim3((unsigned)P, G), dim3(kMtThreads), 0, st, y, v.L, ncols, v.J, m,
                       ldm, K, transpose, z);
    TK_HIP(hipGetLastError());
    return TK_OK;
}

// NKB * NKS <= 16 keeps the fragment table at 32 KB of LDS.
template <int NKS, bool X3>
static int mt_pick_kb(const float* y, const ModeView& v, const double* m, int64_t ldm, int K,
                      int transpose, float* z, hipStream_t st) {
    constexpr int kbmax = 16 / NKS < 4 ? 16 / NKS : 4;
    const int need = (K + 15) / 16;
    if (need <= 1 || kbmax == 1) return mt_launch<1, NKS, X3>(y, v, m, ldm, K, transpose, z, st);
    if constexpr (kbmax >= 2) {
        if (need <= 2 || kbmax == 2)
            return mt_launch<2, NKS, X3>(y, v, m, ldm, K, transpose, z, st);
    }
    if constexpr (kbmax >= 4) return mt_launch<4, NKS, X3>(y, v, m, ldm, K, transpose, z, st);
    return fail(TK_ERR_UNSUPPORTED, "bf16 ttm: no tile for K=%d", K);
}

template <bool X3>
static int mt_dispatch(const float* y, const ModeView& v, const double* m, int64_t ldm, int K,
                       int transpose, float* z, hipStream_t st) {
    const int nks = (v.J + 31) / 32;
    if (nks <= 1) return mt_pick_kb<1, X3>(y, v, m, ldm, K, transpose, z, st);
    if (nks <= 2) return mt_pick_kb<2, X3>(y, v, m, ldm, K, transpose, z, st);
    if (nks <= 4) return mt_pick_kb<4, X3>(y, v, m, ldm, K, transpose, z, st);
    if (nks <= 8) return mt_pick_kb<8, X3>(y, v, m, ldm, K, transpose, z, st);
    if (nks <= 16) return mt_pick_kb<16, X3>(y, v, m, ldm, K, transpose, z, st);
    return fail(TK_ERR_UNSUPPORTED, "mode extent %d exceeds %d", v.J, TK_MAX_MODE_DIM);
}

template <int NKB, int NKS, bool X3>
__global__ __launch_bounds__(kMtThreads) void ttm_bf16_batched(const BatchTtmTask* __restrict__ tasks,
                                                             int ntasks) {
    __shared__ bf8_t afr[NKB * NKS * 2][64];
    const int ti = find_task_wg(&tasks[0].v, sizeof(BatchTtmTask), ntasks, blockIdx.x);
    const BatchTtmTask tk = tasks[ti];
    const int w = blockIdx.x - tk.v.wg_begin;
    const ModeView mv = batch_mode_view(tk.v);
    const int K = (int)tk.v.ranks[tk.v.n];  // this mode's rank, decided on the device
    const int r0 = blockIdx.y * NKB * 16;
    if (r0 >= K) return;                     // row groups beyond the rank: nothing to do
    const int64_t ncols = mv.L * mv.B;
    const bool unit = mv.L == 1 && mv.J % 8 == 0 && ((uintptr_t)tk.y & 15) == 0 &&
                      ((uintptr_t)tk.z & 15) == 0;
    if (unit)
        ttm_bf16_body<NKB, NKS, X3, true, true>(tk.y, mv.L, ncols, mv.J, tk.u, mv.J, K, 1, tk.z,
                                                r0, w, tk.v.nwg, afr);
    else
        ttm_bf16_body<NKB, NKS, X3, false, true>(tk.y, mv.L, ncols, mv.J, tk.u, mv.J, K, 1, tk.z,
                                                 r0, w, tk.v.nwg, afr);
}

template <int NKB, int NKS, bool X3>
static int launch_ttm_batched_t(const BatchTtmTask* tasks, int ntasks, int total_wg, int kmax,
                                hipStream_t st) {
    const int G = (kmax + NKB * 16 - 1) / (NKB * 16);  // row groups up to the rank capacity
    hipLaunchKernelGGL((ttm_bf16_batched<NKB, NKS, X3>), dim3(total_wg, G), dim3(kMtThreads), 0,
                       st, tasks, ntasks);
    TK_HIP(hipGetLastError());
    return TK_OK;
}

template <bool X3>
static int ttm_batched_nks(const BatchTtmTask* tasks, int ntasks, int total_wg, int J, int kmax,
                           hipStream_t st) {
    const int nks = (J + 31) / 32, nkb = std::min(4, (kmax + 15) / 16);
    if (nks > 4) return fail(TK_ERR_UNSUPPORTED, "batched TTM: extent %d too large", J);
#define TK_TTM_B(KB, KS)                                                            \
    if (nkb <= KB && nks <= KS)                                                     \
        return launch_ttm_batched_t<KB, KS, X3>(tasks, ntasks, total_wg, kmax, st)
    TK_TTM_B(1, 1); TK_TTM_B(1, 2); TK_TTM_B(1, 4);
    TK_TTM_B(2, 1); TK_TTM_B(2, 2); TK_TTM_B(2, 4);
    TK_TTM_B(4, 1); TK_TTM_B(4, 2); TK_TTM_B(4, 4);
#undef TK_TTM_B
    return fail(TK_ERR_UNSUPPORTED, "batched TTM: no tile");
}

int launch_ttm_bf16_batched(const BatchTtmTask* tasks_dev, int ntasks, int total_wg, int J,
                            int kmax, int precision, hipStream_t st) {
    if (precision == TK_TTM_BF16X3) return ttm_batched_nks<true>(tasks_dev, ntasks, total_wg, J, kmax, st);
    return ttm_batched_nks<false>(tasks_dev, ntasks, total_wg, J, kmax, st);
}

int launch_ttm_mixed(const float* y, const ModeView& v, const double* m, int64_t K, int64_t ldm,
                     int transpose, int precision, float* z, hipStream_t st) {
    if (precision == TK_TTM_BF16X3) return mt_dispatch<true>(y, v, m, ldm, (int)K, transpose, z, st);
    return mt_dispatch<false>(y, v, m, ldm, (int)K, transpose, z, st);
}

}  // namespace tk
