// Error metrics of a reconstruction (Table II: normalized RMS and maximum
// absolute element error): ||X - X~||^2, max |X - X~| and ||X||^2, in FP64,
// reduced in two fixed-order stages so the result is reproducible.
#include "tk_common.hpp"

namespace tk {

constexpr int kMetThreads = 256;

template <typename T>
__global__ __launch_bounds__(kMetThreads) void metrics_partial(const T* __restrict__ x,
                                                               const T* __restrict__ xh,
                                                               int64_t n,
                                                               double* __restrict__ part) {
    __shared__ double s0[kMetThreads], s1[kMetThreads], s2[kMetThreads];
    double e2 = 0.0, mx = 0.0, n2 = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kMetThreads;
    for (int64_t i = (int64_t)blockIdx.x * kMetThreads + threadIdx.x; i < n; i += stride) {
        double a = (double)x[i], b = (double)xh[i];
        double dlt = a - b;
        e2 += dlt * dlt;
        mx = fmax(mx, fabs(dlt));
        n2 += a * a;
    }
    s0[threadIdx.x] = e2;
    s1[threadIdx.x] = mx;
    s2[threadIdx.x] = n2;
    __syncthreads();
    for (int w = kMetThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            s0[threadIdx.x] += s0[threadIdx.x + w];
            s1[threadIdx.x] = fmax(s1[threadIdx.x], s1[threadIdx.x + w]);
            s2[threadIdx.x] += s2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x + 0] = s0[0];
        part[3 * blockIdx.x + 1] = s1[0];
        part[3 * blockIdx.x + 2] = s2[0];
    }
}

__global__ void metrics_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
    if (threadIdx.x != 0) return;
    double e2 = 0.0, mx = 0.0, n2 = 0.0;
    for (int b = 0; b < nb; ++b) {
        e2 += part[3 * b];
        mx = fmax(mx, part[3 * b + 1]);
        n2 += part[3 * b + 2];
    }
    out[0] = e2;
    out[1] = mx;
    out[2] = n2;
}

int error_metrics_blocks(int64_t n) {
    int64_t b = (n + kMetThreads * 16 - 1) / (kMetThreads * 16);
    int cap = 4 * device_cu_count();
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return (int)b;
}

int launch_error_metrics(const void* x, const void* xh, int dtype, int64_t n, double* partial,
                         int nblocks, double* out3, hipStream_t st) {
    if (dtype == TK_F64)
        hipLaunchKernelGGL(metrics_partial<double>, dim3(nblocks), dim3(kMetThreads), 0, st,
                           (const double*)x, (const double*)xh, n, partial);
    else
        hipLaunchKernelGGL(metrics_partial<float>, dim3(nblocks), dim3(kMetThreads), 0, st,
                           (const float*)x, (const float*)xh, n, partial);
    TK_HIP(hipGetLastError());
    hipLaunchKernelGGL(metrics_final, dim3(1), dim3(64), 0, st, partial, nblocks, out3);
    TK_HIP(hipGetLastError());
    return TK_OK;
}

}  // namespace tk
