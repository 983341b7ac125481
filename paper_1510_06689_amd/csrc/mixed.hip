// Mixed-precision kernels for FP32-stored tensors: the split Gram and the
// bf16 / split-bf16 TTM.  Neither changes what Alg. 1 computes; they change
// the arithmetic of its two bulk steps (Gram, TTM) while the
// eigendecomposition and the rank rule stay in FP64.
//
// Split Gram.  The rank rule compares tail sums of eigenvalues with
// eps^2 ||X||^2 / N, so the Gram's error in the trailing eigenvalues must
// stay far below that threshold.  Rounding inside the products would not
// (dropping lo*lo, or rounding FP32 partial sums, leaves errors that do not
// average out of the trailing eigenvalues).  Hence every product and sum on
// the matrix cores is exact: per tile of KT columns and per row i, every
// element is rounded to 16-bit fixed point relative to 2^E_i (E_i from the
// row's largest magnitude) and split into two 8-bit integer halves.  For
// extents up to 256 (gram_s16_body) the halves are int8 operands of
// v_mfma_i32_16x16x64_i8 with exact int32 sums; for 512 (gram_bf16s_body)
// they are exact bf16 operands of v_mfma_f32_32x32x16_bf16, whose FP32 sums
// over at most 128 columns are integer multiples of their quantum below 2^22
// of it, so exact as well.  Either way the three sums (hi hi, hi lo + lo hi,
// lo lo) are combined exactly, scaled and added into FP64 registers after
// every tile.  What remains is the quantization error d, |d| <= 2^(E_i-16),
// of every element: the split Gram is exactly Y~ Y~^T with Y~ = Y - D.
// Quantization noise independent of the data adds its energy to the
// diagonal, so sum_k d_ik^2 (formed exactly per element) is subtracted from
// S_ii; the rest of D's contribution has mean zero (see EigArgs::guard for
// the model and the bound it gives).  Partials use the FP64 Gram's 16x16
// pair layout and its fixed-order reduction.
//
// bf16 TTM.  Z = op(M) Y with op(M) (K x J) split into bf16 hi/lo fragments
// once per workgroup (in LDS) and Y split per element as it is loaded:
// BF16 forms A_hi Y_hi; BF16X3 adds A_hi Y_lo + A_lo Y_hi
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation, FP32 output).  When the
// columns are contiguous (mode 1) every lane loads its eight consecutive
// rows straight from HBM, no LDS staging needed.
#include <algorithm>
#include <type_traits>

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
enum { kUnit = 0, kContig = 1, kStrided = 2, kUnit4 = 3 };

// max of v over lanes l and l ^ OFF (OFF = 16, 32: permlane swaps; 4, 8:
// rotation inside a 16-lane row, which after offsets 4 then 8 leaves every
// lane the max of its residue class mod 4 in that row)
template <int OFF>
__device__ __forceinline__ float lane_fmax(float v) {
    if constexpr (OFF == 32 || OFF == 16) {
        const int b = __float_as_int(v);
        const auto r = OFF == 32 ? __builtin_amdgcn_permlane32_swap(b, b, false, false)
                                 : __builtin_amdgcn_permlane16_swap(b, b, false, false);
        return __builtin_fmaxf(__int_as_float(r[0]), __int_as_float(r[1]));
    } else {
        static_assert(OFF == 4 || OFF == 8, "row rotations by 4 or 8");
        const int o = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x120 + OFF, 0xf, 0xf,
                                                  false);  // row_ror:OFF
        return __builtin_fmaxf(v, __int_as_float(o));
    }
}

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
//   kContig  (L % 4 == 0, 16-byte aligned): lane group of KT / 8 consecutive
//            threads owns one row, thread t the column group t % (KT / 8);
//            each group is two 16-byte loads, one per 4-column half (each
//            half lies in one run of L).
//   kStrided (otherwise): as kContig, one element per load.
//   kUnit4   (L == 1, J % 4 == 0, 16-byte aligned; JB >= 128): wave w owns
//            rows [w JB/NW, (w+1) JB/NW); lane l holds the four consecutive
//            rows 4 (l % QPW) of them for the eight columns 8 (l / QPW +
//            s CGW) + e of each of its NSET column sets s, one 16-byte load
//            per column (groups m = 4 s + the row).
// NW is the number of waves of the workgroup.
template <int JB, int KT, int MODE, int NBUF = 1, int NW = kMxWaves>
struct SplitTile {
    static constexpr int NT = 64 * NW;                              // threads
    static constexpr int PK = KT + 8;
    static constexpr int NCG = KT / 8;                              // groups per row
    static constexpr int RW = JB / NW > 16 ? JB / NW : 16;          // kUnit rows per wave
    static constexpr int LPR = 64 / RW;                             // kUnit lanes per row
    static constexpr int ROWSTEP = NT / NCG;                        // strided rows per pass
    static constexpr int QPW = JB / NW / 4;                         // kUnit4 row quads per wave
    static constexpr int CGW = QPW >= 1 ? 64 / QPW : 1;             // kUnit4 column groups per set
    static constexpr int NSET = MODE == kUnit4 ? KT / (8 * CGW) : 1;  // kUnit4 sets per lane
    static constexpr int NGRP = MODE == kUnit4  ? 4 * NSET
                                : MODE == kUnit ? NCG / LPR
                                                : JB * NCG / NT;
    static_assert(RW <= 64 && NCG % LPR == 0, "unit mapping");
    static_assert(MODE == kUnit || MODE == kUnit4 ||
                      (NGRP >= 1 && JB * NCG % NT == 0 && NCG <= 16),
                  "strided mapping");
    static_assert(MODE != kUnit4 ||
                      (QPW >= 1 && 64 % QPW == 0 && NSET >= 1 && KT == 8 * CGW * NSET &&
                       NSET * 8 <= 32),
                  "kUnit4 mapping: the wave's lanes cover its rows and the tile's columns");

    float vb[NBUF][NGRP][8];  // NBUF register tiles (loads of one in flight while another is split)
    unsigned okm[NBUF];       // kUnit4: bit 8 s + e set if set s, element e is inside the tile
    int i0, cg0;
    bool owner;      // kUnit: this wave holds rows
    // Offsets of the thread's 8 columns inside a tile.  kContig (L % 4 == 0)
    // keeps coff[0] and coff[4] only: each 4-column half lies in one run of
    // L, at coff[0] + e and coff[4] + e - 4.  With two register tiles
    // (L % 8 == 0 only) the second half is at coff[0] + 4 and coff[4] is not
    // kept.
    int coff[8];
    __device__ __forceinline__ int coff4() const { return NBUF == 2 ? coff[0] + 4 : coff[4]; }
    // Representation error of the split: per row of the thread, the sum of
    // d^2 over its elements, d = x - 2^(E-7) (hi + lo) exactly, and the
    // largest row exponent E it used.
    static constexpr int NROW = MODE == kUnit ? 1 : MODE == kUnit4 ? 4 : NGRP;
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
        if (MODE == kUnit4) {
            const int w = tid >> 6, l = tid & 63;
            owner = true;
            i0 = w * (JB / NW) + 4 * (l % QPW);
            cg0 = l / QPW;
        } else if (MODE == kUnit) {
            const int w = tid >> 6, l = tid & 63;
            owner = w * RW < JB;
            i0 = w * RW + l % RW;
            cg0 = l / RW;
        } else {
            owner = true;
            cg0 = tid % NCG;
            i0 = tid / NCG;
#pragma unroll
            for (int e = 0; e < (MODE == kContig && NBUF == 2 ? 1 : 8);
                 e += MODE == kContig ? 4 : 1)
                coff[e] = (int)col_offset(8 * cg0 + e, tm.L, tm.J);
        }
    }
    __device__ __forceinline__ int row_of(int m) const {
        return MODE == kUnit ? i0 : MODE == kUnit4 ? i0 + (m & 3) : i0 + m * ROWSTEP;
    }
    __device__ __forceinline__ int cg_of(int m) const {
        return MODE == kUnit ? cg0 + m * LPR : MODE == kUnit4 ? cg0 + CGW * (m >> 2) : cg0;
    }

    // kUnit4, full tile t with J == JB (L == 1: the tile is the KT JB floats
    // from t KT JB on).  Raw buffer loads: the tile's base goes into a scalar
    // descriptor whose range is the tile, the lane's offset is fixed and the
    // column step is a scalar offset, so no vector register is written to
    // address the loads (a register written while an older load into it may
    // be in flight would make the compiler wait for every load).
    template <int B>
    __device__ __forceinline__ void load_full(const float* __restrict__ y, int64_t t) {
        static_assert(MODE == kUnit4, "full-tile loads: kUnit4 only");
        float(&v)[NGRP][8] = vb[B];
        okm[B] = (1u << (8 * NSET)) - 1u;
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void*)uni(y + t * (int64_t)(KT * JB)), (short)0, KT * JB * (int)sizeof(float),
            0x00020000);  // gfx9 word 3: 32-bit data format, untyped access
        const int voff = (8 * cg0 * JB + i0) * (int)sizeof(float);
#pragma unroll
        for (int st = 0; st < NSET; ++st)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const f4_t x = __builtin_amdgcn_raw_buffer_load_b128(
                    rs, voff, (8 * CGW * st + e) * JB * (int)sizeof(float), 0);
#pragma unroll
                for (int j = 0; j < 4; ++j) v[4 * st + j][e] = x[j];
            }
    }

    // kContig with L % 8 == 0 (the group's 8 columns in one run: its second
    // half at coff[0] + 4), full tile (KT columns, J == JB): the elements
    // load() reads, as raw buffer loads with no test around them.  The tile's base goes into
    // a scalar descriptor whose range is the tile, the lane's offset (row i0,
    // column 8 cg0) is fixed and the row step is a scalar offset, so no vector
    // register is written to address the loads.  The caller guarantees that
    // a tile spans fewer than 2^31 bytes.
    template <int B>
    __device__ __forceinline__ void load_full_contig(const float* __restrict__ y,
                                                     const TileMap& tm, const Tile& t) {
        static_assert(MODE == kContig, "contiguous full-tile loads");
        float(&v)[NGRP][8] = vb[B];
        const int L4 = (int)tm.L * (int)sizeof(float);
        const int range =
            (JB - 1) * L4 + ((int)col_offset(KT - 1, tm.L, JB) + 1) * (int)sizeof(float);
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void*)uni(y + t.base), (short)0, range, 0x00020000);  // as in load_full
        const int voff = (i0 * (int)tm.L + coff[0]) * (int)sizeof(float);
#pragma unroll
        for (int m = 0; m < NGRP; ++m) {
            const int so = m * ROWSTEP * L4;
            const f4_t a = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, so, 0);
            const f4_t b = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, so + 16, 0);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                v[m][e] = a[e];
                v[m][4 + e] = b[e];
            }
        }
    }

    template <int B = 0>
    __device__ __forceinline__ void load(const float* __restrict__ y, const TileMap& tm,
                                         const Tile& t) {
        float(&v)[NGRP][8] = vb[B];
        const int J = tm.J;
        if (MODE == kUnit4) {
            // column kk = 8 cg0 + e holds rows i0..i0+3 at base + kk J + i0.
            // Elements outside the tile come from clamped addresses and are
            // zeroed when the tile is split, so no load result is used here.
            if (t.ncols == KT && J == JB) {
                okm[B] = (1u << (8 * NSET)) - 1u;
#pragma unroll
                for (int st = 0; st < NSET; ++st)
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const f4_t x = *(const f4_t*)(y + t.base +
                                                      (int64_t)(8 * (cg0 + CGW * st) + e) * JB + i0);
#pragma unroll
                        for (int j = 0; j < 4; ++j) v[4 * st + j][e] = x[j];
                    }
            } else {
                // J % 4 == 0: a row quad is wholly in or out
                const bool rok = i0 < J;
                const int ic = rok ? i0 : J - 4;
                unsigned mk = 0;
                // opaque here, so that the column indices below are formed
                // per call rather than held across the tile loop
                int c0 = cg0;
                asm volatile("" : "+v"(c0));
#pragma unroll
                for (int st = 0; st < NSET; ++st)
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int kk = 8 * (c0 + CGW * st) + e;
                        mk |= (rok && kk < t.ncols) ? 1u << (8 * st + e) : 0u;
                        const int kc = kk < t.ncols ? kk : t.ncols - 1;
                        const f4_t x = *(const f4_t*)(y + t.base + (int64_t)kc * J + ic);
#pragma unroll
                        for (int j = 0; j < 4; ++j) v[4 * st + j][e] = x[j];
                    }
                okm[B] = mk;
            }
        } else if (MODE == kUnit) {
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
                    const f4_t a = *(const f4_t*)(y + rowbase + coff[0]);
                    const f4_t b = *(const f4_t*)(y + rowbase + coff4());
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        v[m][e] = a[e];
                        v[m][4 + e] = b[e];
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int kk = 8 * cg0 + e;
                        const int ce = MODE != kContig ? coff[e]
                                       : e < 4          ? coff[0] + e
                                                        : coff4() + e - 4;
                        v[m][e] = (i < J && kk < t.ncols) ? y[rowbase + ce] : 0.f;
                    }
                }
            }
        }
    }

    // Largest |x| of the row of group m over the whole tile (as float bits).
    template <int B = 0>
    __device__ __forceinline__ unsigned row_max_bits(int m) const {
        const float(&v)[NGRP][8] = vb[B];
        unsigned b = 0;
        if (MODE == kUnit4) {
            // |x| maxima as floats (abs is a free operand modifier); NaN and
            // Inf still reach the Gram through d = x 2^(15-E) - q.  Row m & 3
            // over all of the lane's column sets.
            const int j = m & 3;
            float f = __builtin_fmaxf(__builtin_fabsf(v[j][0]), __builtin_fabsf(v[j][1]));
#pragma unroll
            for (int st = 0; st < NSET; ++st)
#pragma unroll
                for (int e = st == 0 ? 2 : 0; e < 8; e += 2)
                    f = __builtin_fmaxf(f, __builtin_fmaxf(__builtin_fabsf(v[4 * st + j][e]),
                                                           __builtin_fabsf(v[4 * st + j][e + 1])));
            if constexpr (QPW <= 4) f = lane_fmax<4>(f);
            if constexpr (QPW <= 8) f = lane_fmax<8>(f);
            if constexpr (QPW <= 16) f = lane_fmax<16>(f);
            f = lane_fmax<32>(f);
            b = __float_as_uint(f);
        } else if (MODE == kUnit) {
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
        const float(&v)[NGRP][8] = vb[0];
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

    // The int8 form of the same 16-bit fixed point: per row, E is chosen with
    // max |x| 2^(15-E) < 32640, so q = round(x 2^(15-E)) lies in
    // [-32639, 32639] and splits as q = 256 hi + lo with
    //     hi = (q + 128) >> 8 in [-128, 127],  lo = q - 256 hi in [-128, 127].
    // Adding 1.5 2^23 + 128 to x 2^(15-E) rounds it to an integer (to
    // nearest, ties to even) whose float bits end in the 16-bit two's
    // complement of q + 128: byte 1 is hi, byte 0 xor 0x80 is lo.  The two
    // int8 planes are [JB][KT + 16] bytes; each row's scale 2^(E-15) goes to
    // sc[row] as a double.  d = x 2^(15-E) - q is formed exactly.
    template <int B = 0>
    __device__ __forceinline__ void store16(unsigned char* hi, unsigned char* lo, double* sc,
                                            bool count = true) {
        float(&v)[NGRP][8] = vb[B];
        if (MODE == kUnit4 && okm[B] != (1u << (8 * NSET)) - 1u) {  // a partial tile:
#pragma unroll                                                     // zero what lies outside
            for (int st = 0; st < NSET; ++st)
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const bool ok = (okm[B] >> (8 * st + e)) & 1u;
#pragma unroll
                    for (int j = 0; j < 4; ++j) v[4 * st + j][e] = ok ? v[4 * st + j][e] : 0.f;
                }
        }
        constexpr int PKB = KT + 16;
        constexpr float kMagic = 12583040.0f;  // 1.5 2^23 + 128
        unsigned mb = 0;
        if (MODE == kUnit) mb = row_max_bits<B>(0);
        float rs = 0.f;
        int sh = 0;
        int shr[4] = {0, 0, 0, 0};  // kUnit4: the row's shift, from its first set
#pragma unroll
        for (int m = 0; m < NGRP; ++m) {
            if (MODE == kUnit4 ? m < 4 : (MODE != kUnit || m == 0)) {
                if (MODE != kUnit) mb = row_max_bits<B>(m);
                // E: the exponent of max |x| (1 + 2^-8) rounded up, so that
                // max |x| 2^(15-E) < 32768 / 1.004 < 32639.5; zero rows get
                // the smallest normal exponent
                const unsigned bb = __float_as_uint(__uint_as_float(mb) * 1.004f);
                const int E = (int)(bb >> 23) - 126;
                sh = 15 - (E < -125 ? -125 : E);
                if (MODE == kUnit4) shr[m & 3] = sh;
            } else if (MODE == kUnit4) {
                sh = shr[m & 3];
            }
            unsigned b[8];
            float gs = 0.f;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const float sx = __builtin_ldexpf(v[m][e], sh);
                const float f = sx + kMagic;
                const float qf = f - kMagic;
                const float dd = sx - qf;
                gs = __builtin_fmaf(dd, dd, gs);
                b[e] = __float_as_uint(f);
            }
            unsigned hw[2], lw[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                // [lo'0, hi0, lo'1, hi1] and [lo'2, hi2, lo'3, hi3], lo' = lo ^ 0x80
                const unsigned p01 = __builtin_amdgcn_perm(b[4 * h + 1], b[4 * h], 0x05040100u);
                const unsigned p23 = __builtin_amdgcn_perm(b[4 * h + 3], b[4 * h + 2], 0x05040100u);
                hw[h] = __builtin_amdgcn_perm(p23, p01, 0x07050301u);
                lw[h] = __builtin_amdgcn_perm(p23, p01, 0x06040200u) ^ 0x80808080u;
            }
            const int r = row_of(m);
            const bool mine = MODE != kUnit || owner;
            if (mine) {
                const int off = r * PKB + 8 * cg_of(m);
                *(uint2*)(hi + off) = make_uint2(hw[0], hw[1]);
                *(uint2*)(lo + off) = make_uint2(lw[0], lw[1]);
                if (cg_of(m) == 0) sc[r] = __builtin_ldexp(1.0, -sh);
            }
            if (MODE == kUnit) {
                rs += gs;
            } else if (r < JB && count) {
                rd[MODE == kUnit4 ? (m & 3) : m] += __builtin_ldexp((double)gs, -2 * sh);
                emax = max(emax, 15 - sh);
            }
        }
        if (MODE == kUnit && owner && count) {
            rd[0] += __builtin_ldexp((double)rs, -2 * sh);
            emax = max(emax, 15 - sh);
        }
    }

    // Per-row sums of d^2 over the workgroup into rowd[0..JB) (each row's
    // holders form a fixed xor-butterfly; rows nobody holds stay as set).
    __device__ __forceinline__ void row_sums(double* rowd, int lane) const {
        if (MODE == kUnit4) {
#pragma unroll
            for (int m = 0; m < NROW; ++m) {
                double v = rd[m];
#pragma unroll
                for (int d = QPW; d < 64; d *= 2) v += __shfl_xor(v, d);
                if (cg0 == 0 && i0 + m < JB) rowd[i0 + m] = v;
            }
        } else if (MODE == kUnit) {
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

// ---- the same split on int8 matrix cores (extents up to 256) ----------
//
// A 16x16 block of S is
//     sum_k q_ik q_jk 2^(E_i + E_j - 30)
//       = 2^(E_i + E_j - 30) (65536 HH + 256 [HL + LH] + LL)
// with HH = sum hi_i hi_j etc.: v_mfma_i32_16x16x64_i8 forms the three sums
// exactly in int32 (|HH| <= 2^14 KT, |HL + LH| <= 2^15 KT, KT <= 256), and
// after every tile 256 HH + (HL + LH) (below 2^31) and LL are converted and
// combined exactly in FP64, scaled by the two row scales and added.  The
// 16-block pairs (bi <= bj) of the workgroup's pair group are dealt to the
// waves in a snake order (q even: wave w, q odd: wave 7 - w), which balances
// the SIMDs (waves w and w + 4 share one) when a group has 36 pairs.
typedef int i4v_t __attribute__((ext_vector_type(4)));

// Extent 128 (8 blocks of 16, 36 pairs): a fixed schedule per wave whose
// pairs share blocks, so that each wave reads every block's fragments once
// per k-step (at most 5 blocks, 140 KB of fragment reads per tile instead of
// 288 KB with 4 per pair).  Waves w < 4 take row w's pairs (w, w..w+4);
// wave w + 4 the rest of row w and all of row 7 - w.  Waves w and w + 4 share
// a SIMD and hold 9 pairs between them.
struct WaveSched {
    int nblk, blk[5];         // blocks whose fragments the wave reads
    int npair, pa[5], pb[5];  // pair q = (blk[pa[q]], blk[pb[q]])
};
constexpr WaveSched kSched128[8] = {
    {5, {0, 1, 2, 3, 4}, 5, {0, 0, 0, 0, 0}, {0, 1, 2, 3, 4}},
    {5, {1, 2, 3, 4, 5}, 5, {0, 0, 0, 0, 0}, {0, 1, 2, 3, 4}},
    {5, {2, 3, 4, 5, 6}, 5, {0, 0, 0, 0, 0}, {0, 1, 2, 3, 4}},
    {5, {3, 4, 5, 6, 7}, 5, {0, 0, 0, 0, 0}, {0, 1, 2, 3, 4}},
    {4, {0, 5, 6, 7, 0}, 4, {0, 0, 0, 3, 0}, {1, 2, 3, 3, 0}},  // (0,5) (0,6) (0,7) (7,7)
    {3, {1, 6, 7, 0, 0}, 4, {0, 0, 1, 1, 0}, {1, 2, 1, 2, 0}},  // (1,6) (1,7) (6,6) (6,7)
    {4, {2, 5, 6, 7, 0}, 4, {0, 1, 1, 1, 0}, {3, 1, 2, 3, 0}},  // (2,7) (5,5) (5,6) (5,7)
    {4, {4, 5, 6, 7, 0}, 4, {0, 0, 0, 0, 0}, {0, 1, 2, 3, 0}},  // (4,4) (4,5) (4,6) (4,7)
};

template <int JB, int KT>
constexpr size_t s16_buf_bytes() {
    return ((size_t)2 * JB * (KT + 16) + (size_t)JB * sizeof(double) + 15) / 16 * 16;
}

// NBUF = 2 keeps two register tiles: tile t + 2 loads while tile t is on
// the matrix cores and tile t + 1 is split, so every load has about two
// iterations to arrive.  Its loads are unconditional (past the range end the
// last tile is loaded again and split without counting its statistics).
template <int JB, int KT, int NPW, int MODE, int NBUF = 1, int NW = kMxWaves>
__device__ __forceinline__ void gram_s16_body(
    const float* __restrict__ y, const TileMap& tm, int npairs16, int pairs_per_group, int group,
    int64_t t0, int64_t t1, double* __restrict__ out, double* aux, double* lds_raw) {
    using Ld = SplitTile<JB, KT, MODE, NBUF, NW>;
    constexpr int PKB = KT + 16;
    constexpr int PLANE = JB * PKB;
    constexpr size_t BUF = s16_buf_bytes<JB, KT>();
    constexpr int NKS = KT / 64;
    constexpr int NB = JB / 16;
    static_assert(KT % 64 == 0 && KT <= 256, "k-steps of 64; int32 sums exact for KT <= 256");

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // pair choices stay scalar
    const int r16 = lane & 15, kq = lane >> 4;
    const int g0 = group * pairs_per_group;
    // row blocks holding rows < J: a pair with a block past them sums zeros
    // only, so it skips its products and flushes (its partial stays zero).
    // Extents up to 128 (the batches' classes) with one register tile only:
    // two register tiles run with J == JB, where no pair is skipped.
    constexpr bool kSkip = NBUF == 1 && JB <= 128;
    const int nbv = kSkip ? uni((tm.J + 15) >> 4) : NB;

    constexpr bool kSched = JB == 128 && NW == 8;  // the fixed per-wave schedule above
    static_assert(!kSched || NPW == 5, "the extent-128 schedule has up to 5 pairs per wave");
    int bi[NPW], bj[NPW], aoff[NPW], boff[NPW];
    bool act[NPW];
#pragma unroll
    for (int q = 0; q < NPW; ++q) {
        if constexpr (kSched) {
            const WaveSched& ws = kSched128[wave];
            act[q] = q < ws.npair;
            bi[q] = ws.blk[ws.pa[q]];
            bj[q] = ws.blk[ws.pb[q]];
        } else {
            const int pl = q * NW + ((q & 1) ? NW - 1 - wave : wave);
            const int p = g0 + pl;
            act[q] = pl < pairs_per_group && p < npairs16;
            pair32_of(act[q] ? p : 0, NB, bi[q], bj[q]);  // the upper-triangle order, NB blocks
        }
        // block parts only (wave-uniform); the lane part is added per tile
        aoff[q] = 16 * bi[q] * PKB;
        boff[q] = 16 * bj[q] * PKB;
    }

    double accd[NPW][4];
#pragma unroll
    for (int q = 0; q < NPW; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) accd[q][v] = 0.0;

    char* base = (char*)lds_raw;
    auto hi_of = [&](int b) { return (unsigned char*)(base + b * BUF); };
    auto sc_of = [&](int b) { return (double*)(base + b * BUF + 2 * PLANE); };

    // flush of pair q's exact int32 sums into its FP64 accumulators
    // (v_mfma_i32_16x16x64 output: row 4 (lane / 16) + v, column lane % 16)
    auto flush = [&](int q, const i4v_t& hh, const i4v_t& mm, const i4v_t& ll, const double* sc) {
        const double sj = sc[16 * bj[q] + r16];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const double si = sc[16 * bi[q] + 4 * kq + v];
            const double c1 = (double)(hh[v] * 256 + mm[v]);
            const double tv = __builtin_fma(c1, 256.0, (double)ll[v]);
            accd[q][v] = __builtin_fma(tv * si, sj, accd[q][v]);
        }
    };
    // the scheduled waves: fragments of each block read once per k-step
    auto mfma_sched = [&](auto wc, const unsigned char* hb, const unsigned char* lb,
                          const double* sc) {
        constexpr WaveSched ws = kSched128[decltype(wc)::value];
        i4v_t acc[5][3];
#pragma unroll
        for (int q = 0; q < ws.npair; ++q)
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[q][c] = i4v_t{0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) {
            i4v_t fh[5], fl[5];
#pragma unroll
            for (int b = 0; b < ws.nblk; ++b) {
                const int off = (16 * ws.blk[b] + r16) * PKB + 16 * kq + 64 * ks;
                fh[b] = *(const i4v_t*)(hb + off);
                fl[b] = *(const i4v_t*)(lb + off);
            }
#pragma unroll
            for (int q = 0; q < ws.npair; ++q) {
                const int a = ws.pa[q], c = ws.pb[q];
                if (kSkip && max(ws.blk[a], ws.blk[c]) >= nbv) continue;  // uniform
                acc[q][0] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fh[a], fh[c], acc[q][0], 0, 0, 0);
                acc[q][1] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fh[a], fl[c], acc[q][1], 0, 0, 0);
                acc[q][1] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fl[a], fh[c], acc[q][1], 0, 0, 0);
                acc[q][2] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fl[a], fl[c], acc[q][2], 0, 0, 0);
            }
            // one k-step's fragments live at a time
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int q = 0; q < ws.npair; ++q) {
            if (kSkip && max(ws.blk[ws.pa[q]], ws.blk[ws.pb[q]]) >= nbv) continue;  // uniform
            flush(q, acc[q][0], acc[q][1], acc[q][2], sc);
        }
    };
    // all block pairs of the wave on the tile in LDS buffer b
    auto mfma_tile = [&](int b) {
        const unsigned char* hb = hi_of(b);
        const unsigned char* lb = hb + PLANE;
        const double* sc = sc_of(b);
        if constexpr (kSched) {
            switch (wave) {  // uniform
                case 0: mfma_sched(std::integral_constant<int, 0>{}, hb, lb, sc); break;
                case 1: mfma_sched(std::integral_constant<int, 1>{}, hb, lb, sc); break;
                case 2: mfma_sched(std::integral_constant<int, 2>{}, hb, lb, sc); break;
                case 3: mfma_sched(std::integral_constant<int, 3>{}, hb, lb, sc); break;
                case 4: mfma_sched(std::integral_constant<int, 4>{}, hb, lb, sc); break;
                case 5: mfma_sched(std::integral_constant<int, 5>{}, hb, lb, sc); break;
                case 6: mfma_sched(std::integral_constant<int, 6>{}, hb, lb, sc); break;
                default: mfma_sched(std::integral_constant<int, 7>{}, hb, lb, sc); break;
            }
            return;
        }
        // lane part of the fragment offsets, opaque here so that its sums
        // with the pairs' block parts are formed per tile, not held across
        // the loop in a register per pair
        int lo = r16 * PKB + 16 * kq;
        asm volatile("" : "+v"(lo));
#pragma unroll
        for (int q = 0; q < NPW; ++q) {
            if (!act[q] || (kSkip && max(bi[q], bj[q]) >= nbv)) continue;  // uniform
            i4v_t hh = {0, 0, 0, 0}, mm = {0, 0, 0, 0}, ll = {0, 0, 0, 0};
#pragma unroll
            for (int ks = 0; ks < NKS; ++ks) {
                const i4v_t ah = *(const i4v_t*)(hb + lo + aoff[q] + 64 * ks);
                const i4v_t al = *(const i4v_t*)(lb + lo + aoff[q] + 64 * ks);
                const i4v_t bh = *(const i4v_t*)(hb + lo + boff[q] + 64 * ks);
                const i4v_t bl = *(const i4v_t*)(lb + lo + boff[q] + 64 * ks);
                hh = __builtin_amdgcn_mfma_i32_16x16x64_i8(ah, bh, hh, 0, 0, 0);
                mm = __builtin_amdgcn_mfma_i32_16x16x64_i8(ah, bl, mm, 0, 0, 0);
                mm = __builtin_amdgcn_mfma_i32_16x16x64_i8(al, bh, mm, 0, 0, 0);
                ll = __builtin_amdgcn_mfma_i32_16x16x64_i8(al, bl, ll, 0, 0, 0);
            }
            flush(q, hh, mm, ll, sc);
        }
    };

    Ld ld;
    ld.setup(tm, tid);
    if constexpr (NBUF == 1) {
        if (t0 < t1) {
            ld.load(y, tm, tile_at(tm, t0, tm.J));
            ld.store16(hi_of(0), hi_of(0) + PLANE, sc_of(0));
        }
        __syncthreads();
        for (int64_t t = t0; t < t1; ++t) {
            const int cur = (int)((t - t0) & 1);
            const bool more = t + 1 < t1;
            if (more) ld.load(y, tm, tile_at(tm, t + 1, tm.J));  // in flight during the MFMAs
            mfma_tile(cur);
            if (more) {
                const int nb2 = cur ^ 1;
                ld.store16(hi_of(nb2), hi_of(nb2) + PLANE, sc_of(nb2));
            }
            __syncthreads();
        }
    } else {
        // Two register tiles; only for kUnit4 or kContig with J == JB, where
        // every tile but the tensor's last is full.  The loop runs over the
        // full tiles [t0, tf) with loads clamped to tf - 1 and no branch around
        // them; a ragged last tile follows on its own.
        static_assert(NBUF == 2 && (MODE == kUnit4 || MODE == kContig),
                      "two register tiles: kUnit4 or kContig");
        auto load_full = [&](auto bc, int64_t tt) {
            constexpr int BB = decltype(bc)::value;
            if constexpr (MODE == kUnit4)
                ld.template load_full<BB>(y, tt);
            else
                ld.template load_full_contig<BB>(y, tm, tile_at(tm, tt, tm.J));
        };
        // tile counters relative to t0 in 32 bits (a workgroup's range is far
        // below 2^31 tiles), so that every comparison stays scalar
        int nf = (int)(t1 - t0);
        if (nf > 0 && tile_at(tm, t1 - 1, tm.J).ncols < KT) --nf;
        auto tile = [&](int r) { return t0 + (r < nf ? r : nf - 1); };
        if (nf > 0) {  // uniform
            load_full(std::integral_constant<int, 0>{}, tile(0));
            ld.template store16<0>(hi_of(0), hi_of(0) + PLANE, sc_of(0));
            load_full(std::integral_constant<int, 1>{}, tile(1));
            __syncthreads();
            int r = 0;
            for (;;) {
                // LDS buffer 0: tile r; registers 1: tile r + 1 (loaded)
                load_full(std::integral_constant<int, 0>{}, tile(r + 2));
                mfma_tile(0);
                ld.template store16<1>(hi_of(1), hi_of(1) + PLANE, sc_of(1), r + 1 < nf);
                __syncthreads();
                if (++r >= nf) break;
                load_full(std::integral_constant<int, 1>{}, tile(r + 2));
                mfma_tile(1);
                ld.template store16<0>(hi_of(0), hi_of(0) + PLANE, sc_of(0), r + 1 < nf);
                __syncthreads();
                if (++r >= nf) break;
            }
        }
        if (t0 + nf < t1) {  // the ragged last tile
            ld.template load<0>(y, tm, tile_at(tm, t1 - 1, tm.J));
            ld.template store16<0>(hi_of(0), hi_of(0) + PLANE, sc_of(0));
            __syncthreads();
            mfma_tile(0);
        }
        __syncthreads();
    }

    // subtract each row's sum of d^2 from its diagonal entry (as the bf16 body)
    double* rowd = lds_raw + 64;
    for (int i = tid; i < JB; i += 64 * NW) rowd[i] = 0.0;
    __syncthreads();
    ld.row_sums(rowd, lane);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NPW; ++q) {
        if (!act[q]) continue;
        const int p16 = bi[q] * NB - bi[q] * (bi[q] - 1) / 2 + (bj[q] - bi[q]);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int il = 4 * kq + v;
            const bool dg = bi[q] == bj[q] && il == r16;
            out[(int64_t)p16 * 256 + il * 16 + r16] =
                dg ? accd[q][v] - rowd[16 * bi[q] + il] : accd[q][v];
        }
    }
    if (aux) split_stats_out(ld.total(), ld.emax, aux, lds_raw);  // uniform branch
}

template <int JB, int KT, int NPW, int MODE, int NBUF, int NW>
__global__ __launch_bounds__(64 * NW) void gram_partial_s16(
    const float* __restrict__ y, TileMap tm, int npairs16, int pairs_per_group, int P, int G,
    double* __restrict__ partial) {
    extern __shared__ double lds_raw[];
    int p, g;
    xcd_range_group(blockIdx.x, G, p, g);
    const int64_t t0 = tm.ntiles * (int64_t)p / P;
    const int64_t t1 = tm.ntiles * (int64_t)(p + 1) / P;
    double* aux = g == 0 ? partial + (int64_t)P * npairs16 * 256 + 2 * p : nullptr;
    gram_s16_body<JB, KT, NPW, MODE, NBUF, NW>(y, tm, npairs16, pairs_per_group, g, t0, t1,
                                           partial + (int64_t)p * npairs16 * 256, aux, lds_raw);
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
// (each streams and splits every tile again), workgroups per CU.  Extents up to 256 run the
// int8 kernel on 16-block pairs, 512 the bf16 kernel on 32-block pairs.
struct MxGramShape {
    int KT, NPW, G, per_cu, NW;  // NW: waves per workgroup
};
template <int JB>
constexpr bool mx_int8() {
    return JB <= 256;
}
// UNIT: the view has L == 1.  At extent 256 its loaders (one register tile)
// leave room for 17 pairs per wave: one pair group of 136 on tiles of 128
// columns, so every tile is split once and the FP64 flushes come once per
// 128 columns; the strided loaders leave room for 9 (two groups of 68 on
// tiles of 64: three groups of 46 took a quarter longer).  A pair's int32 sums live only
// from its first MFMA to its flush; the FP64 accumulators of all the wave's
// pairs (8 registers each) are what limits the count.
template <int JB, bool UNIT = false>
constexpr MxGramShape mx_gram_shape() {
    return JB == 32    ? MxGramShape{128, 1, 1, 2, 8}    //   3 16-pairs
           : JB == 64  ? MxGramShape{128, 2, 1, 2, 8}    //  10 16-pairs
           : JB == 128 ? MxGramShape{128, 5, 1, 1, 8}    //  36 16-pairs, 9 per SIMD
           : JB == 256 ? (UNIT ? MxGramShape{128, 17, 1, 1, 8}   // 136 16-pairs: 1 x 136
                               : MxGramShape{64, 9, 2, 1, 8})    //               2 x 68
                       : MxGramShape{16, 2, 9, 1, 8};    // 136 32-pairs: 9 groups of 16
}
template <int JB>
constexpr int mx_owned_pairs() {  // pairs the kernel's owner waves are dealt
    return mx_int8<JB>() ? (JB / 16) * (JB / 16 + 1) / 2 : (JB / 32) * (JB / 32 + 1) / 2;
}

static int mx_round_jb(int J) {
    int jb = 32;
    while (jb < J) jb *= 2;
    return jb;
}

template <int JB, bool UNIT>
static GramPlan mx_plan(const ModeView& v) {
    constexpr MxGramShape gs = mx_gram_shape<JB, UNIT>();
    constexpr int owned = mx_owned_pairs<JB>();
    static_assert(gs.NW * gs.NPW >= (owned + gs.G - 1) / gs.G,
                  "every pair of a group needs an owner wave");
    GramPlan pl{};
    TileMap tm = make_tiles(v, gs.KT);
    pl.KT = gs.KT;
    pl.G = gs.G;
    pl.pairs_per_group = (owned + gs.G - 1) / gs.G;
    pl.nb = JB / 16;  // 16-blocks, for the shared reduction
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
        case 32: return mx_plan<32, false>(v);
        case 64: return mx_plan<64, false>(v);
        case 128: return mx_plan<128, false>(v);
        case 256: return v.L == 1 ? mx_plan<256, true>(v) : mx_plan<256, false>(v);
        default: return mx_plan<512, false>(v);
    }
}

template <int JB, int MODE, int NBUF = 1>
static int mx_launch(const float* y, const TileMap& tm, const GramPlan& pl, double* partial,
                     hipStream_t st) {
    // the shape the plan chose (L == 1 exactly for the unit loaders)
    constexpr MxGramShape gs = mx_gram_shape<JB, MODE == kUnit || MODE == kUnit4>();
    if constexpr (mx_int8<JB>()) {
        auto fn = gram_partial_s16<JB, gs.KT, gs.NPW, MODE, NBUF, gs.NW>;
        const size_t lds = 2 * s16_buf_bytes<JB, gs.KT>();
        TK_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds));
        hipLaunchKernelGGL(fn, dim3(pl.P * pl.G), dim3(64 * gs.NW), lds, st, y, tm, pl.npairs,
                           pl.pairs_per_group, pl.P, pl.G, partial);
    } else {
        auto fn = gram_partial_bf16s<JB, gs.KT, gs.NPW, MODE>;
        const size_t lds = 2 * mx_buf_bytes<JB, gs.KT>();
        TK_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds));
        const int nb32 = JB / 32;
        hipLaunchKernelGGL(fn, dim3(pl.P * pl.G), dim3(kMxThreads), lds, st, y, tm,
                           nb32 * (nb32 + 1) / 2, pl.pairs_per_group, pl.npairs, pl.P, pl.G,
                           partial);
    }
    TK_HIP(hipGetLastError());
    return TK_OK;
}

template <int JB>
static int mx_dispatch_mode(const float* y, const ModeView& v, const GramPlan& pl,
                            double* partial, hipStream_t st) {
    TileMap tm = make_tiles(v, pl.KT);
    if constexpr (JB == 128 || JB == 256) {
        if (v.L == 1 && v.J % 4 == 0 && ((uintptr_t)y & 15) == 0) {
            // two register tiles at extent 128 with J == JB; extent 256 keeps
            // one (its 17 pairs per wave take the registers of the second)
            if constexpr (JB == 128) {
                if (v.J == JB) return mx_launch<JB, kUnit4, 2>(y, tm, pl, partial, st);
            }
            return mx_launch<JB, kUnit4, 1>(y, tm, pl, partial, st);
        }
    }
    if (v.L == 1) return mx_launch<JB, kUnit>(y, tm, pl, partial, st);
    const bool contig = v.L % 4 == 0 && ((uintptr_t)y & 15) == 0;
    if constexpr (JB == 128) {
        // two register tiles: L % 8 == 0, J == JB, every tile but the tensor's last full
        // (KT a multiple of L when tiles pack whole b-blocks, L a multiple of
        // KT when they cut one), and a full tile spans < 2^31 bytes
        const int64_t kl = pl.KT - 1;
        const int64_t span = (int64_t)(v.J - 1) * v.L + (kl / v.L) * v.J * v.L + kl % v.L + 1;
        const bool even = tm.packed ? pl.KT % v.L == 0 : v.L % pl.KT == 0;
        if (contig && v.L % 8 == 0 && v.J == JB && even &&
            span * (int64_t)sizeof(float) < (int64_t(1) << 31))
            return mx_launch<JB, kContig, 2>(y, tm, pl, partial, st);
    }
    if (contig) return mx_launch<JB, kContig>(y, tm, pl, partial, st);
    return mx_launch<JB, kStrided>(y, tm, pl, partial, st);
}

// ---- batches: three launches cover every problem of a batch -------------
// A problem's unfolding stride L depends on ranks found on the device, so
// the three loader variants (L == 1; L % 4 == 0 with 16-byte alignment; any
// other) run over the same task table, each returning at once for the tasks
// of the others (one variant per kernel keeps each kernel's registers those
// of its own loader).
__device__ __forceinline__ int batch_loader(const ModeView& mv, const float* y) {
    return mv.L == 1 ? kUnit : (mv.L % 4 == 0 && ((uintptr_t)y & 15) == 0) ? kContig : kStrided;
}

template <int JB, int MODE>
__global__ __launch_bounds__(kMxThreads) void gram_s16_batched(
    const BatchGramTask* __restrict__ tasks, int ntasks) {
    extern __shared__ double lds_raw[];
    constexpr MxGramShape gs = mx_gram_shape<JB>();
    const int ti = uni(find_task_wg(&tasks[0].v, sizeof(BatchGramTask), ntasks, blockIdx.x));
    BatchGramTask tk = tasks[ti];
    tk.y = uni_global(tk.y);
    tk.partial = uni_global(tk.partial);
    tk.aux = uni_global(tk.aux);
    tk.tpw = uni(tk.tpw);
    if (tk.status && (uni(*tk.status) & 8)) return;  // uniform: marked for the FP64 pass
    const int w = blockIdx.x - uni(tk.v.wg_begin);
    const ModeView mv = uni(batch_mode_view(tk.v));
    if (batch_loader(mv, tk.y) != MODE) return;  // uniform: another launch's task
    const TileMap tm = make_tiles(mv, gs.KT);
    // workgroups needed at the actual shape (>= 1: a shape has >= 1 tile)
    const int64_t need = (tm.ntiles + tk.tpw - 1) / tk.tpw;
    const int active = (int)(need < tk.v.nwg ? need : tk.v.nwg);
    if (w == 0 && threadIdx.x == 0) *tk.nparts = active;
    if (w >= active) return;  // uniform over the workgroup
    const int64_t t0 = tm.ntiles * (int64_t)w / active;
    const int64_t t1 = tm.ntiles * (int64_t)(w + 1) / active;
    constexpr int np16 = (JB / 16) * (JB / 16 + 1) / 2;
    static_assert(mx_int8<JB>(), "batches run the int8 kernel");
    double* out = tk.partial + (int64_t)w * np16 * 256;
    double* aux = tk.aux + 2 * w;
    gram_s16_body<JB, gs.KT, gs.NPW, MODE>(tk.y, tm, np16, np16, 0, t0, t1, out, aux, lds_raw);
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
static int launch_split_batched_t(const BatchGramTask* tasks, int ntasks, int total_wg,
                                  unsigned loaders, hipStream_t st) {
    static_assert(mx_gram_shape<JB>().G == 1, "batches need a single pair group");
    static_assert(kUnit == 0 && kContig == 1 && kStrided == 2, "bit i of loaders is variant i");
    const size_t lds = 2 * s16_buf_bytes<JB, mx_gram_shape<JB>().KT>();
    const decltype(&gram_s16_batched<JB, kUnit>) fns[3] = {
        gram_s16_batched<JB, kUnit>, gram_s16_batched<JB, kContig>,
        gram_s16_batched<JB, kStrided>};
    for (int i = 0; i < 3; ++i) {
        if (!((loaders >> i) & 1u)) continue;
        const auto fn = fns[i];
        TK_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds));
        hipLaunchKernelGGL(fn, dim3(total_wg), dim3(kMxThreads), lds, st, tasks, ntasks);
        TK_HIP(hipGetLastError());
    }
    return TK_OK;
}

int launch_gram_split_batched(const BatchGramTask* tasks_dev, int ntasks, int total_wg, int jb,
                              unsigned loaders, hipStream_t st) {
    switch (jb) {
        case 32: return launch_split_batched_t<32>(tasks_dev, ntasks, total_wg, loaders, st);
        case 64: return launch_split_batched_t<64>(tasks_dev, ntasks, total_wg, loaders, st);
        case 128: return launch_split_batched_t<128>(tasks_dev, ntasks, total_wg, loaders, st);
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
// UNIT: L == 1, each column's J floats contiguous: a lane's 8 rows of a
// column come in two 16-byte loads, and its 4 outputs go out in one 16-byte
// store.  With J (or K) not a multiple of 4 these addresses are only 4-byte
// aligned; the target runs in unaligned-access mode, where wide accesses at
// any dword address are legal (memcpy lets the compiler emit them).
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
                if (cv && j0 + 8 <= J) {
                    __builtin_memcpy(x, ycol + j0, sizeof(x));
                } else {  // the column's last rows (J % 8 != 0), or no column
#pragma unroll
                    for (int e = 0; e < 8; ++e) x[e] = (cv && j0 + e < J) ? ycol[j0 + e] : 0.f;
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
                if (rb + 4 <= K) {
                    __builtin_memcpy(zc + rb, &acc[kb], sizeof(f4_t));
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
    const bool unit = v.L == 1;
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
    if (nks <= 3) return mt_pick_kb<3, X3>(y, v, m, ldm, K, transpose, z, st);
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
    BatchTtmTask tk = tasks[ti];
    tk.y = uni_global(tk.y);
    tk.u = uni_global(tk.u);
    tk.z = uni_global(tk.z);
    const int w = blockIdx.x - tk.v.wg_begin;
    const ModeView mv = batch_mode_view(tk.v);
    const int K = (int)tk.v.ranks[tk.v.n];  // this mode's rank, decided on the device
    const int r0 = blockIdx.y * NKB * 16;
    if (r0 >= K) return;                     // row groups beyond the rank: nothing to do
    const int64_t ncols = mv.L * mv.B;
    const bool unit = mv.L == 1;
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
    TK_TTM_B(1, 1); TK_TTM_B(1, 2); TK_TTM_B(1, 3); TK_TTM_B(1, 4);
    TK_TTM_B(2, 1); TK_TTM_B(2, 2); TK_TTM_B(2, 3); TK_TTM_B(2, 4);
    TK_TTM_B(4, 1); TK_TTM_B(4, 2); TK_TTM_B(4, 3); TK_TTM_B(4, 4);
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
