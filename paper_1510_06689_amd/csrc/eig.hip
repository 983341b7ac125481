// FP64 symmetric eigensolver + rank truncation for one J x J Gram matrix
// (Alg. 1, eigenvector and rank steps; Sec. V-D uses a LAPACK subset solver,
// this is the same family of method on one workgroup):
//
//   1. Householder reduction to tridiagonal form T = Q^T S Q (matrix in LDS
//      for J <= 128, otherwise in global scratch), reflectors kept below the
//      diagonal;
//   2. all eigenvalues of T by multisection of Sturm counts (groups of
//      threads per eigenvalue, ballots combine the sub-interval tests);
//   3. rank rule R = min R >= 1 with sum_{r>R} max(lambda_r,0) <= eps^2 nu / N
//      (tail sums accumulated smallest first), or a fixed rank;
//   4. the R leading eigenvectors of T by inverse iteration with partial-
//      pivoting tridiagonal LU, re-orthogonalised inside eigenvalue clusters
//      after every sweep;
//   5. back-transformation by Q, and a sign rule (largest |entry| positive,
//      lowest index on ties).
// A single workgroup of 1024 threads; no host synchronisation.
#include <cfloat>

#include "tk_common.hpp"

namespace tk {

constexpr int kEigThreads = 1024;
constexpr int kEigWaves = kEigThreads / 64;
constexpr int kInvIters = 3;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Block-wide sum in a fixed order; every thread gets the result.
__device__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kEigWaves; ++w) t += red[w];
    return t;
}

__device__ __forceinline__ double hash_unit(uint32_t a, uint32_t b) {
    uint64_t z = ((uint64_t)a << 32) ^ (uint64_t)b ^ 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;  // [-1, 1)
}

size_t eig_scratch_doubles(int J) {
    // A (J*J) + X (J*J) + LU arrays l, u0, u1, u2, piv (5 * J*J)
    return (size_t)7 * J * J + 64;
}

template <bool A_IN_LDS>
__global__ __launch_bounds__(kEigThreads) void eig_kernel(EigArgs a) {
    extern __shared__ double smem[];
    const int J = a.J;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double* A = A_IN_LDS ? smem : a.scratch;  // row-major J x J
    double* sv = A_IN_LDS ? smem + (size_t)J * J : smem;
    double* d = sv;              // J
    double* e = d + J;           // J
    double* e2 = e + J;          // J
    double* beta = e2 + J;       // J
    double* vb = beta + J;       // J
    double* pw = vb + J;         // J
    double* lam = pw + J;        // J (descending)
    double* shift = lam + J;     // J
    double* dots = shift + J;    // J
    double* red = dots + J;      // 64
    int* misc = (int*)(red + 64);  // [0] = R
    double* X = a.scratch + (size_t)J * J;  // [t][j], column j is vector j
    double* Lm = X + (size_t)J * J;
    double* U0 = Lm + (size_t)J * J;
    double* U1 = U0 + (size_t)J * J;
    double* U2 = U1 + (size_t)J * J;
    double* PV = U2 + (size_t)J * J;

    // ---- load S (symmetric) -------------------------------------------
    for (int idx = tid; idx < J * J; idx += kEigThreads) A[idx] = a.s[idx];
    __syncthreads();

    // ---- 1. Householder tridiagonalisation ------------------------------
    for (int k = 0; k + 2 < J; ++k) {
        const int m = J - k - 1;
        double part = 0.0;
        for (int i = 1 + tid; i < m; i += kEigThreads) {
            double xi = A[(size_t)(k + 1 + i) * J + k];
            part += xi * xi;
        }
        const double sigma = block_sum(part, red);
        const double x0 = A[(size_t)(k + 1) * J + k];
        const double dk = A[(size_t)k * J + k];
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
        if (tid == 0) {
            d[k] = dk;
            e[k] = mu;
            beta[k] = b;
        }
        for (int i = tid; i < m; i += kEigThreads)
            vb[i] = (i == 0) ? 1.0 : A[(size_t)(k + 1 + i) * J + k] / v0;
        __syncthreads();
        if (b != 0.0) {
            // p = b * A22 v, one wave per row
            for (int i = wave; i < m; i += kEigWaves) {
                const double* row = A + (size_t)(k + 1 + i) * J + (k + 1);
                double s = 0.0;
                for (int j = lane; j < m; j += 64) s += row[j] * vb[j];
                s = wave_sum(s);
                if (lane == 0) pw[i] = b * s;
            }
            __syncthreads();
            part = 0.0;
            for (int i = tid; i < m; i += kEigThreads) part += pw[i] * vb[i];
            const double kc = 0.5 * b * block_sum(part, red);
            // A22 -= v w^T + w v^T with w = p - kc v
            for (int i = wave; i < m; i += kEigWaves) {
                const double vi = vb[i], wi = pw[i] - kc * vb[i];
                double* row = A + (size_t)(k + 1 + i) * J + (k + 1);
                for (int j = lane; j < m; j += 64) {
                    const double wj = pw[j] - kc * vb[j];
                    row[j] -= vi * wj + wi * vb[j];
                }
            }
        }
        __syncthreads();
        for (int i = tid; i < m; i += kEigThreads) A[(size_t)(k + 1 + i) * J + k] = vb[i];
        __syncthreads();
    }
    if (tid == 0) {
        if (J >= 2) {
            d[J - 2] = A[(size_t)(J - 2) * J + (J - 2)];
            e[J - 2] = A[(size_t)(J - 1) * J + (J - 2)];
            beta[J - 2] = 0.0;
        }
        d[J - 1] = A[(size_t)(J - 1) * J + (J - 1)];
        e[J - 1] = 0.0;
        beta[J - 1] = 0.0;
    }
    __syncthreads();
    for (int i = tid; i < J; i += kEigThreads) e2[i] = e[i] * e[i];
    // Gershgorin interval and pivot floor
    if (tid == 0) {
        double gl = DBL_MAX, gu = -DBL_MAX, emax2 = 0.0;
        for (int i = 0; i < J; ++i) {
            double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < J ? fabs(e[i]) : 0.0);
            gl = fmin(gl, d[i] - r);
            gu = fmax(gu, d[i] + r);
            if (i + 1 < J) emax2 = fmax(emax2, e[i] * e[i]);
        }
        double tnorm = fmax(fabs(gl), fabs(gu));
        // widen slightly so that count(gl) = 0 and count(gu) = J hold exactly
        gl -= 2.0 * DBL_EPSILON * tnorm * J + 2.0 * DBL_MIN;
        gu += 2.0 * DBL_EPSILON * tnorm * J + 2.0 * DBL_MIN;
        red[32] = gl;
        red[33] = gu;
        red[34] = DBL_MIN * fmax(1.0, emax2);  // pivmin
        red[35] = tnorm;
    }
    __syncthreads();
    const double gl = red[32], gu = red[33], pivmin = red[34], tnorm = red[35];

    // ---- 2. eigenvalues by multisection ---------------------------------
    {
        int jp = 32;
        while (jp < J) jp *= 2;
        const int tpe = kEigThreads / jp;  // threads per eigenvalue, <= 32
        const int k = tid / tpe, s = tid - (tid / tpe) * tpe;
        const int gofs = (lane / tpe) * tpe;  // group's first lane within the wave
        const uint64_t gmask = (tpe == 64) ? ~0ull : (((1ull << tpe) - 1ull) << gofs);
        const double atol = 2.0 * DBL_EPSILON * tnorm + 4.0 * pivmin;
        double lo = gl, hi = gu;
        if (k < J) {
            for (int it = 0; it < 128; ++it) {
                const double tol = fmax(atol, 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)));
                if (hi - lo <= tol) break;
                const double x = lo + (hi - lo) * (double)(s + 1) / (double)(tpe + 1);
                int c = 0;
                double q = d[0] - x;
                if (fabs(q) < pivmin) q = -pivmin;
                c += q < 0.0;
                for (int i = 1; i < J; ++i) {
                    q = (d[i] - x) - e2[i - 1] / q;
                    if (fabs(q) < pivmin) q = -pivmin;
                    c += q < 0.0;
                }
                const uint64_t bal = __ballot(c > k) & gmask;
                const int sstar = bal ? (__ffsll((long long)bal) - 1 - gofs) : tpe;
                const double nlo =
                    sstar == 0 ? lo : lo + (hi - lo) * (double)sstar / (double)(tpe + 1);
                const double nhi =
                    sstar == tpe ? hi : lo + (hi - lo) * (double)(sstar + 1) / (double)(tpe + 1);
                lo = nlo;
                hi = nhi;
            }
            if (s == 0) lam[J - 1 - k] = 0.5 * (lo + hi);
        }
    }
    __syncthreads();
    for (int i = tid; i < J; i += kEigThreads) a.lambda[i] = lam[i];

    // ---- 3. rank rule ---------------------------------------------------
    if (tid == 0) {
        int R;
        double tail = 0.0;
        if (a.fixed_rank > 0) {
            R = a.fixed_rank < J ? a.fixed_rank : J;
            for (int r = J - 1; r >= R; --r) tail += fmax(lam[r], 0.0);
        } else {
            const double tau = a.eps2_over_n * (*a.nu);
            R = J;
            while (R > 1 && tail + fmax(lam[R - 1], 0.0) <= tau) {
                tail += fmax(lam[R - 1], 0.0);
                --R;
            }
        }
        int flag = 0;
        if (R > a.max_rank) {
            flag |= 2;
            R = a.max_rank;
        }
        *a.rank_out = R;
        *a.disc_out = tail;
        if (flag) a.flags[0] |= flag;  // single writer: thread 0 of the only workgroup
        misc[0] = R;
        // shifts for inverse iteration: separate (near-)equal eigenvalues
        const double pert = 10.0 * DBL_EPSILON * tnorm;
        for (int j = 0; j < R; ++j) {
            double sj = lam[j];
            if (j > 0 && shift[j - 1] - sj < pert) sj = shift[j - 1] - pert;
            shift[j] = sj;
        }
    }
    __syncthreads();
    const int R = misc[0];
    const double ortol = 1e-3 * tnorm;

    // ---- 4. inverse iteration for the R leading eigenvectors -------------
    const double tiny = DBL_EPSILON * tnorm + DBL_MIN;
    if (tid < R) {
        const int j = tid;
        const double sg = shift[j];
        // LU with partial pivoting of T - sg I; arrays strided by J per row
        double ai = d[0] - sg, bi = (J > 1) ? e[0] : 0.0;
        for (int i = 0; i + 1 < J; ++i) {
            const double ci = e[i];                 // sub-diagonal below row i
            const double an = d[i + 1] - sg;        // next diagonal
            const double bn = (i + 2 < J) ? e[i + 1] : 0.0;
            if (fabs(ai) >= fabs(ci)) {
                double piv = ai;
                if (fabs(piv) < tiny) piv = (piv < 0.0 ? -tiny : tiny);
                const double l = ci / piv;
                U0[(size_t)i * J + j] = piv;
                U1[(size_t)i * J + j] = bi;
                U2[(size_t)i * J + j] = 0.0;
                Lm[(size_t)i * J + j] = l;
                PV[(size_t)i * J + j] = 0.0;
                ai = an - l * bi;
                bi = bn;
            } else {
                const double l = ai / ci;
                U0[(size_t)i * J + j] = ci;
                U1[(size_t)i * J + j] = an;
                U2[(size_t)i * J + j] = bn;
                Lm[(size_t)i * J + j] = l;
                PV[(size_t)i * J + j] = 1.0;
                ai = bi - l * an;
                bi = -l * bn;
            }
        }
        if (fabs(ai) < tiny) ai = (ai < 0.0 ? -tiny : tiny);
        U0[(size_t)(J - 1) * J + j] = ai;
        for (int i = 0; i < J; ++i) X[(size_t)i * J + j] = hash_unit((uint32_t)j, (uint32_t)i);
    }
    for (int it = 0; it < kInvIters; ++it) {
        if (tid < R) {
            const int j = tid;
            // forward: apply the row interchanges and multipliers
            for (int i = 0; i + 1 < J; ++i) {
                double xi = X[(size_t)i * J + j], xn = X[(size_t)(i + 1) * J + j];
                if (PV[(size_t)i * J + j] != 0.0) {
                    double t = xi;
                    xi = xn;
                    xn = t;
                }
                X[(size_t)i * J + j] = xi;
                X[(size_t)(i + 1) * J + j] = xn - Lm[(size_t)i * J + j] * xi;
            }
            // backward substitution with the three upper diagonals
            double x1 = 0.0, x2 = 0.0, amax = 0.0;
            for (int i = J - 1; i >= 0; --i) {
                double v = X[(size_t)i * J + j];
                if (i + 1 < J) v -= U1[(size_t)i * J + j] * x1;
                if (i + 2 < J) v -= U2[(size_t)i * J + j] * x2;
                v /= U0[(size_t)i * J + j];
                X[(size_t)i * J + j] = v;
                x2 = x1;
                x1 = v;
                amax = fmax(amax, fabs(v));
            }
            // normalise (scale by the max first to avoid overflow)
            double nrm2 = 0.0;
            const double sc = amax > 0.0 ? 1.0 / amax : 1.0;
            for (int i = 0; i < J; ++i) {
                double v = X[(size_t)i * J + j] * sc;
                X[(size_t)i * J + j] = v;
                nrm2 += v * v;
            }
            const double inv = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 0.0;
            for (int i = 0; i < J; ++i) X[(size_t)i * J + j] *= inv;
        }
        __syncthreads();
        // modified Gram-Schmidt inside clusters, in descending order
        for (int j = 1; j < R; ++j) {
            int c0 = j;
            while (c0 > 0 && lam[c0 - 1] - lam[c0] <= ortol) --c0;
            if (c0 == j) continue;  // uniform: every thread reads the same lam
            for (int pass = 0; pass < 2; ++pass) {
                for (int i = c0 + wave; i < j; i += kEigWaves) {
                    double s = 0.0;
                    for (int t = lane; t < J; t += 64) s += X[(size_t)t * J + i] * X[(size_t)t * J + j];
                    s = wave_sum(s);
                    if (lane == 0) dots[i] = s;
                }
                __syncthreads();
                for (int t = tid; t < J; t += kEigThreads) {
                    double v = X[(size_t)t * J + j];
                    for (int i = c0; i < j; ++i) v -= dots[i] * X[(size_t)t * J + i];
                    X[(size_t)t * J + j] = v;
                }
                __syncthreads();
            }
            double part = 0.0;
            for (int t = tid; t < J; t += kEigThreads) {
                double v = X[(size_t)t * J + j];
                part += v * v;
            }
            const double n2 = block_sum(part, red);
            const double inv = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
            for (int t = tid; t < J; t += kEigThreads) X[(size_t)t * J + j] *= inv;
            __syncthreads();
        }
    }

    // ---- 5. back-transformation X <- Q X and the sign rule ---------------
    if (tid < R) {
        const int j = tid;
        for (int k = J - 3; k >= 0; --k) {
            const double b = beta[k];
            if (b == 0.0) continue;
            const int m = J - k - 1;
            double s = 0.0;
            for (int i = 0; i < m; ++i) s += A[(size_t)(k + 1 + i) * J + k] * X[(size_t)(k + 1 + i) * J + j];
            s *= b;
            for (int i = 0; i < m; ++i)
                X[(size_t)(k + 1 + i) * J + j] -= s * A[(size_t)(k + 1 + i) * J + k];
        }
        int best = 0;
        double bv = fabs(X[j]);
        for (int i = 1; i < J; ++i) {
            double v = fabs(X[(size_t)i * J + j]);
            if (v > bv) {
                bv = v;
                best = i;
            }
        }
        const double sgn = X[(size_t)best * J + j] < 0.0 ? -1.0 : 1.0;
        for (int i = 0; i < J; ++i) a.u[i + (size_t)J * j] = sgn * X[(size_t)i * J + j];
    }
}

int launch_eig(const EigArgs& a, hipStream_t st) {
    const size_t small = (size_t)(10 * a.J + 64) * sizeof(double) + 64;
    if (a.J <= 128) {
        size_t lds = (size_t)a.J * a.J * sizeof(double) + small;
        auto fn = eig_kernel<true>;
        TK_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds));
        hipLaunchKernelGGL(fn, dim3(1), dim3(kEigThreads), lds, st, a);
    } else {
        auto fn = eig_kernel<false>;
        TK_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)small));
        hipLaunchKernelGGL(fn, dim3(1), dim3(kEigThreads), small, st, a);
    }
    TK_HIP(hipGetLastError());
    return TK_OK;
}

}  // namespace tk
