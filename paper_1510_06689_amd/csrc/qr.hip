// R factor of a Householder QR of the tall and skinny matrix A = Y_(n)^T
// (Sec. IX: the singular values of Y_(n) taken from a QR of Y_(n)^T instead
// of from the Gram, the stable choice when eps approaches sqrt(u)), and the
// pieces that turn R into U_n:
//
//   tsqr_kernel   one 512-thread workgroup keeps a running R (JC x JC, FP64)
//                 in LDS and absorbs tiles of BR rows of A held in registers:
//                 the stacked matrix [R; tile] is reduced column by column
//                 with Householder reflectors (LAPACK's dlarfg convention,
//                 beta = -sign(alpha) ||x||).  Wave w of 8 owns the columns
//                 c = w + 8 q, lane l the tile rows l + 64 p (64 values per
//                 lane, up to 256 VGPRs at two waves per SIMD); the owner wave
//                 of column k forms the reflector alone (wave sums, no
//                 barrier), publishes v in LDS (double buffered, so one
//                 barrier per column), and every wave forms its columns' dot
//                 products with one butterfly reduce-scatter across lanes.
//                 Only rows of R that the step touches are read: row k at
//                 step k, by the waves owning its columns.
//                 A first level gives each workgroup a contiguous slice of
//                 rows; further levels absorb the partial R factors the same
//                 way (a reduction tree) until one workgroup writes the final
//                 R with a non-negative diagonal.
//   jw_kernel     the symmetric 2J x 2J matrix [[0, R^T], [R, 0]] whose
//                 eigenvalues are +-sigma_i(R) (= +-sigma_i(Y_(n))).
//   jw_extract    U = leading right singular vectors of R from the leading
//                 eigenvectors [x; y] of that matrix: x, orthonormalised by
//                 classical Gram-Schmidt applied twice, sign rule.
#include "tk_common.hpp"

namespace tk {
namespace {

constexpr int kQrThreads = 512;
constexpr int kQrWaves = kQrThreads / 64;

__device__ __forceinline__ double qr_wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Cross-lane exchanges on VALU (no LDS round trip):
//   offset 32: v_permlane32_swap(a, b) -> ([a 0-31, b 0-31], [a 32-63, b 32-63]),
//   offset 16: v_permlane16_swap(a, b) -> (even rows of a, b; odd rows of a, b),
// so first + second adds a value to its partner's (l ^ 32, resp. the other
// row of the pair) with lanes below the offset holding a's pair sum and lanes
// above it holding b's; offsets 8, 4, 2, 1 pair lanes inside a 16-lane row
// with the DPP patterns row_ror:8, row_half_mirror, quad_perm [2,3,0,1] and
// [1,0,3,2] (each an involution across that offset's bit).
template <int OFF>
__device__ __forceinline__ void pair_swap(double a, double b, double& x, double& y) {
    const int al = __double2loint(a), ah = __double2hiint(a);
    const int bl = __double2loint(b), bh = __double2hiint(b);
    if constexpr (OFF == 32) {
        const auto lo = __builtin_amdgcn_permlane32_swap(al, bl, false, false);
        const auto hi = __builtin_amdgcn_permlane32_swap(ah, bh, false, false);
        x = __hiloint2double(hi[0], lo[0]);
        y = __hiloint2double(hi[1], lo[1]);
    } else {
        const auto lo = __builtin_amdgcn_permlane16_swap(al, bl, false, false);
        const auto hi = __builtin_amdgcn_permlane16_swap(ah, bh, false, false);
        x = __hiloint2double(hi[0], lo[0]);
        y = __hiloint2double(hi[1], lo[1]);
    }
}

template <int OFF>
__device__ __forceinline__ double dpp_partner(double v) {
    constexpr int ctrl = OFF == 8 ? 0x128 : OFF == 4 ? 0x141 : OFF == 2 ? 0x4e : 0xb1;
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), ctrl, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), ctrl, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// One reduce-scatter stage at offset OFF: the lane keeps value a (its offset
// bit clear) or b (set) and adds its partner's copy of the same one.
template <int OFF>
__device__ __forceinline__ double rs_stage(double a, double b, bool up) {
    if constexpr (OFF >= 16) {
        double x, y;
        pair_swap<OFF>(a, b, x, y);
        return x + y;
    } else {
        const double keep = up ? b : a, send = up ? a : b;
        return keep + dpp_partner<OFF>(send);
    }
}

// Full sum stage at offset OFF (every lane of the pair gets the same bits).
template <int OFF>
__device__ __forceinline__ double sum_stage(double v) {
    if constexpr (OFF >= 16) {
        double x, y;
        pair_swap<OFF>(v, v, x, y);
        return x + y;
    } else {
        return v + dpp_partner<OFF>(v);
    }
}

__device__ __forceinline__ double wave_total(double v) {
    v = sum_stage<32>(v);
    v = sum_stage<16>(v);
    v = sum_stage<8>(v);
    v = sum_stage<4>(v);
    v = sum_stage<2>(v);
    return sum_stage<1>(v);
}

// Sum over the 64 lanes of NS per-lane values at once (the slots OFFS ..
// OFFS + NS - 1 of d): at offsets 32, 16, ... each lane keeps half of its
// values (the upper half where its offset bit is set) and adds its partner's
// copy of that half; after log2(NS) stages the remaining value is summed over
// the lanes that share those bits.  Lane l returns the total for slot
// OFFS + slot_of_lane<NS>(l) (offset bit 32 >> s stands for NS >> (s + 1));
// all lanes of a group hold bitwise the same total (every stage adds the
// same two operands).
template <int NS, int CPW, int OFFS>
__device__ __forceinline__ double reduce_window(double (&d)[CPW], int lane) {
    constexpr int lg = NS >= 16 ? 4 : NS >= 8 ? 3 : NS >= 4 ? 2 : NS >= 2 ? 1 : 0;
    static_assert((1 << lg) == NS && OFFS + NS <= CPW, "window of a power-of-two width");
    if constexpr (lg >= 1) {
#pragma unroll
        for (int i = 0; i < NS / 2; ++i)
            d[OFFS + i] = rs_stage<32>(d[OFFS + i], d[OFFS + NS / 2 + i], lane & 32);
    }
    if constexpr (lg >= 2) {
#pragma unroll
        for (int i = 0; i < NS / 4; ++i)
            d[OFFS + i] = rs_stage<16>(d[OFFS + i], d[OFFS + NS / 4 + i], lane & 16);
    }
    if constexpr (lg >= 3) {
#pragma unroll
        for (int i = 0; i < NS / 8; ++i)
            d[OFFS + i] = rs_stage<8>(d[OFFS + i], d[OFFS + NS / 8 + i], lane & 8);
    }
    if constexpr (lg >= 4) d[OFFS] = rs_stage<4>(d[OFFS], d[OFFS + 1], lane & 4);
    double t = d[OFFS];
    if constexpr (lg < 1) t = sum_stage<32>(t);
    if constexpr (lg < 2) t = sum_stage<16>(t);
    if constexpr (lg < 3) t = sum_stage<8>(t);
    if constexpr (lg < 4) t = sum_stage<4>(t);
    t = sum_stage<2>(t);
    return sum_stage<1>(t);
}

// Window slot whose total lane l holds after reduce_window<CPW, ...>.
template <int CPW>
__device__ __forceinline__ int slot_of_lane(int l) {
    int q = 0;
#pragma unroll
    for (int s = 0; (CPW >> s) > 1; ++s)
        if (l & (32 >> s)) q += CPW >> (s + 1);
    return q;
}

}  // namespace

// Householder reflector of the stacked column [R_kk; col] (dlarfg convention:
// beta = -sign(alpha) ||.||, tau = (beta - alpha) / beta, v = col / (alpha -
// beta), no reflection when col is zero).  Called by the one wave owning
// column k; writes v (BR values) and tau to vbuf and beta to R_kk.
template <int RPL, int BR, int JC>
__device__ __forceinline__ void make_reflector(const double (&col)[RPL], int k, double* Rs,
                                               double* vbuf, int lane) {
    double s = 0.0;
#pragma unroll
    for (int p = 0; p < RPL; ++p) s = fma(col[p], col[p], s);
    const double xn2 = wave_total(s);
    const double alpha = Rs[k * JC + k];
    double tau = 0.0, scal = 0.0;
    if (xn2 > 0.0) {
        const double nrm = sqrt(fma(alpha, alpha, xn2));
        const double beta = alpha >= 0.0 ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
        if (lane == 0) Rs[k * JC + k] = beta;
    }
#pragma unroll
    for (int p = 0; p < RPL; ++p) vbuf[lane + 64 * p] = col[p] * scal;
    if (lane == 0) vbuf[BR] = tau;
}

// Rows of A: row r = b * L + l holds the elements (r, j) at b * sB + j * sJ + l.
struct QrSrc {
    const void* y;
    int f32;       // 1: FP32 elements (widened exactly), 0: FP64
    int64_t rows;  // rows of A
    int64_t L, sB, sJ;
};

template <int JC>
struct QrGeom {
    static constexpr int CPW = JC / kQrWaves;  // columns per wave
    static constexpr int RPL = 64 / CPW;       // tile rows per lane (64 doubles per lane)
    static constexpr int BR = 64 * RPL;   // tile rows
    static constexpr int VB = BR + 2;     // v buffer pitch (v, then tau)
    static constexpr size_t lds_bytes =
        ((size_t)JC * JC + 2 * VB + kQrWaves + kQrWaves * CPW) * sizeof(double);
};

// Steps k = 8 KB .. 8 KB + 7 of the reduction of [R; tile] (kQrWaves = 8
// columns, one per wave, all in slot KB).  Slots q < KB hold finished
// columns, slots q > KB only columns c > k, and slot KB column k itself in
// wave kk = k - 8 KB (the owner, which forms reflector k) and live columns in
// waves above it; the live slots lie in the window of the last NS slots,
// whose width shrinks block by block.  Reflector k is published in
// vb[k & 1] behind one barrier per column: that buffer is rewritten two
// columns later, after every wave has passed the next barrier (and so
// finished this step).  R row k, column c is read and written only by the
// wave owning c.
template <int JC, int KB>
__device__ __forceinline__ void absorb_block(double (&a)[QrGeom<JC>::RPL][QrGeom<JC>::CPW],
                                             int J, int wave, int lane, double* Rs,
                                             double* vb, double* wb) {
    using G = QrGeom<JC>;
    constexpr int CPW = G::CPW, RPL = G::RPL, BR = G::BR, VB = G::VB;
    constexpr int LIVE = CPW - KB;
    constexpr int NS = LIVE > 8 ? 16 : LIVE > 4 ? 8 : LIVE > 2 ? 4 : LIVE > 1 ? 2 : 1;
    constexpr int OFFS = CPW - NS;
    for (int kk = 0; kk < kQrWaves; ++kk) {
        const int k = KB * kQrWaves + kk;
        if (k >= J) return;  // uniform
        double* vk = vb + (k & 1) * VB;
        if (wave == kk) {
            double col[RPL];
#pragma unroll
            for (int p = 0; p < RPL; ++p) col[p] = a[p][KB];
            make_reflector<RPL, BR, JC>(col, k, Rs, vk, lane);
        }
        __syncthreads();
        // tau = 0 (identity reflector) leaves v = 0 and w = 0: the update
        // below is then exact no-op arithmetic, so the step needs no branch
        const double tau = vk[BR];
        double v[RPL];
#pragma unroll
        for (int p = 0; p < RPL; ++p) v[p] = vk[lane + 64 * p];
        // this lane's window slot after the reduction, and its R_kc (read
        // now, used after the reduction)
        const int ql = OFFS + slot_of_lane<NS>(lane);
        const int cl = wave + kQrWaves * ql;
        const bool act = cl > k && cl < J;
        const double rk = act ? Rs[k * JC + cl] : 0.0;
        double d[CPW];
#pragma unroll
        for (int q = OFFS; q < CPW; ++q) {
            double s = 0.0;
            const int c = wave + kQrWaves * q;
            if (q >= KB && (q > KB || wave > kk) && c < J) {  // uniform
#pragma unroll
                for (int p = 0; p < RPL; ++p) s = fma(v[p], a[p][q], s);
            }
            d[q] = s;
        }
        const double tot = reduce_window<NS, CPW, OFFS>(d, lane);
        {
            const double w = act ? tau * (rk + tot) : 0.0;
            if (act) Rs[k * JC + cl] = rk - w;  // all lanes of the slot: same value
            wb[ql] = w;
        }
        // LDS operations of one wave complete in order: the reads below see
        // this wave's writes above (the wave barrier keeps the compiler from
        // moving them across)
        __builtin_amdgcn_wave_barrier();
        double wq[CPW];
        if constexpr (NS >= 2) {
#pragma unroll
            for (int q = OFFS; q < CPW; q += 2) {
                const double2 t = *reinterpret_cast<const double2*>(wb + q);
                wq[q] = t.x;
                wq[q + 1] = t.y;
            }
        } else {
            wq[OFFS] = wb[OFFS];
        }
#pragma unroll
        for (int q = KB; q < CPW; ++q) {
            const int c = wave + kQrWaves * q;
            if ((q > KB || wave > kk) && c < J) {  // uniform
#pragma unroll
                for (int p = 0; p < RPL; ++p) a[p][q] = fma(-v[p], wq[q], a[p][q]);
            }
        }
    }
}

template <int JC, int KB>
__device__ __forceinline__ void absorb_from(double (&a)[QrGeom<JC>::RPL][QrGeom<JC>::CPW], int J,
                                            int wave, int lane, double* Rs, double* vb,
                                            double* wb) {
    absorb_block<JC, KB>(a, J, wave, lane, Rs, vb, wb);
    if constexpr (KB + 1 < QrGeom<JC>::CPW) absorb_from<JC, KB + 1>(a, J, wave, lane, Rs, vb, wb);
}

// One level of the reduction.  Workgroup g absorbs rows
// [g * rows_per_wg, min(rows, (g + 1) * rows_per_wg)) of src.  Unless r_final
// is set it writes its R (column-major JC x JC, zero below the diagonal) to
// r_part + g JC^2 and, when ss_part is set, the sum of squares of its rows to
// ss_part[g].  With r_final (one workgroup) it writes R as column-major J x J
// with each row signed so that the diagonal is >= 0, and *ss_final = the sum
// of ss_in[0 .. n_ss_in) in index order (or of its own rows if ss_in is NULL).
template <int JC>
__global__ __launch_bounds__(kQrThreads) void tsqr_kernel(QrSrc src, int J, int64_t rows_per_wg,
                                                          double* __restrict__ r_part,
                                                          double* __restrict__ ss_part,
                                                          double* __restrict__ r_final,
                                                          double* __restrict__ ss_final,
                                                          const double* __restrict__ ss_in,
                                                          int n_ss_in) {
    using G = QrGeom<JC>;
    constexpr int CPW = G::CPW, RPL = G::RPL, BR = G::BR, VB = G::VB;
    extern __shared__ double smem[];
    double* Rs = smem;              // JC x JC, row-major
    double* vb = Rs + JC * JC;      // 2 x VB
    double* red = vb + 2 * VB;      // kQrWaves
    double* wbuf = red + kQrWaves;  // kQrWaves x CPW: one wave's w values per step
    // wave index made visibly uniform: column offsets and tests stay scalar
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    double* wb = wbuf + wave * CPW;

    for (int i = tid; i < JC * JC; i += kQrThreads) Rs[i] = 0.0;
    const int64_t r_begin = (int64_t)blockIdx.x * rows_per_wg;
    const int64_t r_end = min(r_begin + rows_per_wg, src.rows);
    double ss = 0.0;
    double a[RPL][CPW];
    __syncthreads();

    for (int64_t r0 = r_begin; r0 < r_end; r0 += BR) {
        // ---- tile: rows r0 + lane + 64 p, columns wave + kQrWaves q; zero padding
#pragma unroll
        for (int p = 0; p < RPL; ++p) {
            const int64_t r = r0 + lane + 64 * p;
            const bool rv = r < r_end;
            int64_t off = 0;
            if (rv) {
                const int64_t b = r / src.L;
                off = b * src.sB + (r - b * src.L);
            }
#pragma unroll
            for (int q = 0; q < CPW; ++q) {
                const int c = wave + kQrWaves * q;
                double x = 0.0;
                if (rv && c < J) {
                    const int64_t o = off + (int64_t)c * src.sJ;
                    x = src.f32 ? (double)((const float*)src.y)[o] : ((const double*)src.y)[o];
                }
                a[p][q] = x;
                ss = fma(x, x, ss);
            }
        }
        // ---- reduce [R; tile] column by column.  Every wave has finished the
        // previous tile's last step (which may read vb[0]) before reflector 0
        // of this tile is written there.
        __syncthreads();
        absorb_from<JC, 0>(a, J, wave, lane, Rs, vb, wb);
    }
    ss = wave_total(ss);
    if (lane == 0) red[wave] = ss;
    __syncthreads();
    if (!r_final) {
        double* out = r_part + (size_t)blockIdx.x * JC * JC;
        for (int idx = tid; idx < JC * JC; idx += kQrThreads) {
            const int j = idx / JC, i = idx - j * JC;
            out[idx] = j >= i ? Rs[i * JC + j] : 0.0;
        }
        if (ss_part && tid == 0) {
            double t = 0.0;
            for (int w = 0; w < kQrThreads / 64; ++w) t += red[w];
            ss_part[blockIdx.x] = t;
        }
    } else {
        for (int idx = tid; idx < J * J; idx += kQrThreads) {
            const int j = idx / J, i = idx - j * J;
            const double sg = Rs[i * JC + i] < 0.0 ? -1.0 : 1.0;
            r_final[idx] = j >= i ? sg * Rs[i * JC + j] : 0.0;
        }
        if (ss_final && tid == 0) {
            double t = 0.0;
            if (ss_in) {
                for (int g = 0; g < n_ss_in; ++g) t += ss_in[g];
            } else {
                for (int w = 0; w < kQrThreads / 64; ++w) t += red[w];
            }
            *ss_final = t;
        }
    }
}

// M = [[0, R^T], [R, 0]] (2J x 2J, symmetric) from R (J x J column-major).
__global__ void jw_kernel(const double* __restrict__ r, int J, double* __restrict__ m) {
    const int n = 2 * J;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * n) return;
    const int j = (int)(idx / n), i = (int)(idx - (int64_t)j * n);
    double v = 0.0;
    if (i < J && j >= J) v = r[(size_t)i * J + (j - J)];       // R^T(i, j - J) = R(j - J, i)
    else if (i >= J && j < J) v = r[(size_t)j * J + (i - J)];  // R(i - J, j)
    m[idx] = v;
}

// U (J x R column-major) from the leading R eigenvectors Z (2J x R, ld 2J) of
// the matrix above: u_r = the first J entries of z_r, then classical
// Gram-Schmidt against u_0 .. u_{r-1} applied twice and normalisation.  A
// column left with a squared norm below 2^-20 after the projections (z is a
// unit vector, so it came from a numerically zero singular value, where z
// may lie in the lower half) is replaced by the first unit vector e_t that keeps at least half
// its norm after the same projections.  Sign rule: the largest |entry|
// (lowest index on ties) is positive.  One workgroup; J <= 128.
__global__ __launch_bounds__(kQrThreads) void jw_extract(const double* __restrict__ z, int J,
                                                          const int64_t* __restrict__ rank,
                                                          double* __restrict__ u) {
    extern __shared__ double smem[];
    const int R = (int)*rank;
    double* X = smem;                  // J x R, column-major
    double* dots = X + (size_t)J * R;  // R
    double* red = dots + R;            // 32
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int idx = tid; idx < J * R; idx += kQrThreads) {
        const int r = idx / J, i = idx - r * J;
        X[idx] = z[(size_t)r * 2 * J + i];
    }
    __syncthreads();
    for (int r = 0; r < R; ++r) {
        double* xr = X + (size_t)r * J;
        for (int attempt = -1; attempt < J; ++attempt) {
            if (attempt >= 0) {  // candidate e_attempt
                for (int i = tid; i < J; i += kQrThreads) xr[i] = i == attempt ? 1.0 : 0.0;
                __syncthreads();
            }
            // norm before the projections
            double s = 0.0;
            for (int i = tid; i < J; i += kQrThreads) s = fma(xr[i], xr[i], s);
            s = qr_wave_sum(s);
            if (lane == 0) red[wave] = s;
            __syncthreads();
            double n0 = 0.0;
            for (int w = 0; w < kQrThreads / 64; ++w) n0 += red[w];
            __syncthreads();
            for (int pass = 0; pass < 2 && r > 0; ++pass) {
                // dots[i] = u_i . x_r, 8 lanes per i
                for (int i = tid >> 3; i < r; i += kQrThreads / 8) {
                    const double* xi = X + (size_t)i * J;
                    double t = 0.0;
                    for (int e = tid & 7; e < J; e += 8) t = fma(xi[e], xr[e], t);
                    t += __shfl_xor(t, 1, 64);
                    t += __shfl_xor(t, 2, 64);
                    t += __shfl_xor(t, 4, 64);
                    if ((tid & 7) == 0) dots[i] = t;
                }
                __syncthreads();
                for (int e = tid; e < J; e += kQrThreads) {
                    double t = xr[e];
                    for (int i = 0; i < r; ++i) t = fma(-dots[i], X[(size_t)i * J + e], t);
                    xr[e] = t;
                }
                __syncthreads();
            }
            s = 0.0;
            for (int i = tid; i < J; i += kQrThreads) s = fma(xr[i], xr[i], s);
            s = qr_wave_sum(s);
            if (lane == 0) red[16 + wave] = s;
            __syncthreads();
            double n1 = 0.0;
            for (int w = 0; w < kQrThreads / 64; ++w) n1 += red[16 + w];
            // z is a unit vector: a healthy top half keeps about half of it
            const bool ok = attempt < 0 ? n1 > 0x1p-20 : n1 >= 0.25 * n0;
            if (ok) {
                const double inv = 1.0 / sqrt(n1);
                for (int i = tid; i < J; i += kQrThreads) xr[i] *= inv;
                __syncthreads();
                break;
            }
            __syncthreads();
        }
    }
    // sign rule and store, one wave per column
    for (int r = wave; r < R; r += kQrThreads / 64) {
        const double* xr = X + (size_t)r * J;
        double bv = -1.0;
        int bi = J;
        for (int i = lane; i < J; i += 64)
            if (fabs(xr[i]) > bv) {
                bv = fabs(xr[i]);
                bi = i;
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
        const double sg = xr[bi] < 0.0 ? -1.0 : 1.0;
        for (int i = lane; i < J; i += 64) u[(size_t)r * J + i] = sg * xr[i];
    }
}

// ------------------------------------------------------------------ host

namespace {

constexpr int kQrMaxWg = 256;  // first-level workgroups (independent of the device)

int qr_class(int J) { return J <= 32 ? 32 : J <= 64 ? 64 : 128; }

int qr_tile_rows(int JC) { return 64 * (64 / (JC / kQrWaves)); }

}  // namespace

QrPlan plan_qr(const ModeView& v) {
    QrPlan pl{};
    pl.JC = qr_class(v.J);
    pl.BR = qr_tile_rows(pl.JC);
    const int64_t rows = v.L * v.B;
    const int64_t T = (rows + pl.BR - 1) / pl.BR;
    int64_t P = T < kQrMaxWg ? T : kQrMaxWg;
    const int64_t tiles_per = (T + P - 1) / P;
    pl.rows_per_wg[0] = tiles_per * pl.BR;
    pl.P[0] = (int)((rows + pl.rows_per_wg[0] - 1) / pl.rows_per_wg[0]);
    pl.levels = 1;
    // later levels: each workgroup absorbs F partial factors (about four tiles of rows)
    int F = 4 * pl.BR / v.J;
    if (F < 2) F = 2;
    while (pl.P[pl.levels - 1] > 1) {
        const int prev = pl.P[pl.levels - 1];
        pl.rows_per_wg[pl.levels] = (int64_t)F * v.J;
        pl.P[pl.levels] = (prev + F - 1) / F;
        ++pl.levels;
    }
    pl.part_doubles[0] = (size_t)pl.P[0] * pl.JC * pl.JC;
    pl.part_doubles[1] = pl.levels > 2 ? (size_t)pl.P[1] * pl.JC * pl.JC : 0;
    pl.ss_doubles = (size_t)pl.P[0];
    return pl;
}

size_t qr_workspace_doubles(const QrPlan& pl) {
    return pl.part_doubles[0] + pl.part_doubles[1] + pl.ss_doubles + 64;
}

// Upper bound of qr_workspace_doubles over every row count for extent J
// (first level <= 256 workgroups, second level <= 128).
size_t qr_workspace_bound_doubles(int J) {
    const size_t jc = (size_t)qr_class(J);
    return (size_t)(kQrMaxWg + kQrMaxWg / 2) * jc * jc + kQrMaxWg + 64;
}

template <int JC>
static int launch_tsqr_t(const void* y, int dtype, const ModeView& v, const QrPlan& pl,
                         double* ws, double* r_out, double* sumsq, hipStream_t st) {
    auto fn = tsqr_kernel<JC>;
    const size_t lds = QrGeom<JC>::lds_bytes;
    TK_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
    double* part[2] = {ws, ws + pl.part_doubles[0]};
    double* ssp = ws + pl.part_doubles[0] + pl.part_doubles[1];
    QrSrc src{y, dtype == TK_F32 ? 1 : 0, v.L * v.B, v.L, (int64_t)v.J * v.L, v.L};
    for (int lv = 0; lv < pl.levels; ++lv) {
        const bool last = lv + 1 == pl.levels;
        double* dst = part[lv & 1];
        if (lv > 0) {  // the previous level's partial factors, J meaningful rows each
            const double* prev = part[(lv - 1) & 1];
            src = QrSrc{prev, 0, (int64_t)pl.P[lv - 1] * v.J, v.J, (int64_t)JC * JC, JC};
        }
        hipLaunchKernelGGL(fn, dim3(pl.P[lv]), dim3(kQrThreads), lds, st, src, v.J,
                           pl.rows_per_wg[lv], last ? nullptr : dst,
                           lv == 0 && !last ? ssp : nullptr, last ? r_out : nullptr,
                           last ? sumsq : nullptr, lv > 0 ? ssp : nullptr,
                           lv > 0 ? pl.P[0] : 0);
        TK_HIP(hipGetLastError());
    }
    return TK_OK;
}

int launch_tsqr(const void* y, int dtype, const ModeView& v, const QrPlan& pl, double* ws,
                double* r_out, double* sumsq, hipStream_t st) {
    if (v.J > 128) return fail(TK_ERR_UNSUPPORTED, "QR path: mode extent %d exceeds 128", v.J);
    switch (pl.JC) {
        case 32: return launch_tsqr_t<32>(y, dtype, v, pl, ws, r_out, sumsq, st);
        case 64: return launch_tsqr_t<64>(y, dtype, v, pl, ws, r_out, sumsq, st);
        default: return launch_tsqr_t<128>(y, dtype, v, pl, ws, r_out, sumsq, st);
    }
}

int launch_jw(const double* r, int J, double* m, hipStream_t st) {
    const int64_t n = (int64_t)4 * J * J;
    hipLaunchKernelGGL(jw_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, r, J, m);
    TK_HIP(hipGetLastError());
    return TK_OK;
}

int launch_jw_extract(const double* z, int J, int max_rank, const int64_t* rank, double* u,
                      hipStream_t st) {
    if (J > 128) return fail(TK_ERR_UNSUPPORTED, "QR path: mode extent %d exceeds 128", J);
    const size_t lds = ((size_t)J * max_rank + max_rank + 32) * sizeof(double);
    TK_HIP(hipFuncSetAttribute((const void*)jw_extract, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
    hipLaunchKernelGGL(jw_extract, dim3(1), dim3(kQrThreads), lds, st, z, J, rank, u);
    TK_HIP(hipGetLastError());
    return TK_OK;
}

}  // namespace tk
