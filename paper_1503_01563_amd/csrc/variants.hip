// variants.hip -- elementwise steps of the other outer iterations over the
// chain proxes (Sec. 4.1-4.2 of the paper), in this package's sign: u = -w,
// primal x = u - sum_j y_j, dual blocks y_j in K_j, Pi_{K_j}(v) = v - prox_j(v).
//
//   cyclic projections / BCD:  v = x + y_i;  x <- prox_i(v);  y_i <- v - x
//   alternating projections:   y_j = l_j - prox_j(l_j);  x = u - sum_j y_j;
//                              l_j <- y_j + x / r
//   FISTA on the dual:         yt = y + beta (y - y_prev);  xt = u - sum_j yt_j;
//                              v_j = yt_j + xt / r;  y_j <- v_j - prox_j(v_j)
// The proxes are the chain sweeps (mode ModeProx); these kernels are the
// elementwise glue between them.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch.hpp"

namespace mc {

namespace {

constexpr int kThreads = 256;

inline int blocks_for(size_t n)
{
    const size_t b = (n + kThreads - 1) / kThreads;
    return (int)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

#define GRID_STRIDE(i, n) \
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < (n); i += (size_t)gridDim.x * blockDim.x)

__global__ void k_neg(size_t n, const float* __restrict__ w, float* __restrict__ x)
{
    GRID_STRIDE(i, n) x[i] = -w[i];
}

__global__ void k_add(size_t n, const float* __restrict__ x, const float* __restrict__ y, float* __restrict__ v)
{
    GRID_STRIDE(i, n) v[i] = x[i] + y[i];
}

// d <- a - d
__global__ void k_rsub(size_t n, const float* __restrict__ a, float* __restrict__ d)
{
    GRID_STRIDE(i, n) d[i] = a[i] - d[i];
}

// d <- d - a
__global__ void k_sub(size_t n, const float* __restrict__ a, float* __restrict__ d)
{
    GRID_STRIDE(i, n) d[i] = d[i] - a[i];
}

// d <- a - b
__global__ void k_diff(size_t n, const float* __restrict__ a, const float* __restrict__ b, float* __restrict__ d)
{
    GRID_STRIDE(i, n) d[i] = a[i] - b[i];
}

// d <- f * a
__global__ void k_scale(size_t n, float f, const float* __restrict__ a, float* __restrict__ d)
{
    GRID_STRIDE(i, n) d[i] = f * a[i];
}

template <int R>
__global__ void k_ap_update(size_t n, float* __restrict__ lam, const float* __restrict__ q,
                            const float* __restrict__ w)
{
    GRID_STRIDE(i, n)
    {
        float y[R], s = 0.f;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            y[j] = lam[j * n + i] - q[j * n + i];
            s += y[j];
        }
        const float x = -w[i] - s;
        const float xr = x * (1.f / (float)R);
#pragma unroll
        for (int j = 0; j < R; ++j) lam[j * n + i] = y[j] + xr;
    }
}

// first AP step from l = 0: every projection of 0 is 0, so l_j = u / r
template <int R>
__global__ void k_ap_cold(size_t n, float* __restrict__ lam, const float* __restrict__ w)
{
    GRID_STRIDE(i, n)
    {
        const float xr = -w[i] * (1.f / (float)R);
#pragma unroll
        for (int j = 0; j < R; ++j) lam[j * n + i] = xr;
    }
}

template <int R>
__global__ void k_fista_pre(size_t n, const float* __restrict__ y, const float* __restrict__ yp, float beta,
                            const float* __restrict__ w, float* __restrict__ v)
{
    GRID_STRIDE(i, n)
    {
        float yt[R], s = 0.f;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const float a = y[j * n + i];
            yt[j] = a + beta * (a - yp[j * n + i]);
            s += yt[j];
        }
        const float xr = (-w[i] - s) * (1.f / (float)R);
#pragma unroll
        for (int j = 0; j < R; ++j) v[j * n + i] = yt[j] + xr;
    }
}

}  // namespace

hipError_t launch_neg(size_t n, const float* w, float* x, hipStream_t s)
{
    hipLaunchKernelGGL(k_neg, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, w, x);
    return hipGetLastError();
}

hipError_t launch_add(size_t n, const float* x, const float* y, float* v, hipStream_t s)
{
    hipLaunchKernelGGL(k_add, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, x, y, v);
    return hipGetLastError();
}

hipError_t launch_rsub(size_t n, const float* a, float* d, hipStream_t s)
{
    hipLaunchKernelGGL(k_rsub, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, a, d);
    return hipGetLastError();
}

hipError_t launch_sub(size_t n, const float* a, float* d, hipStream_t s)
{
    hipLaunchKernelGGL(k_sub, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, a, d);
    return hipGetLastError();
}

hipError_t launch_diff(size_t n, const float* a, const float* b, float* d, hipStream_t s)
{
    hipLaunchKernelGGL(k_diff, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, a, b, d);
    return hipGetLastError();
}

hipError_t launch_scale(size_t n, float f, const float* a, float* d, hipStream_t s)
{
    hipLaunchKernelGGL(k_scale, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, f, a, d);
    return hipGetLastError();
}

hipError_t launch_ap_update(size_t n, int r, float* lam, const float* q, const float* w, bool cold, hipStream_t s)
{
    if (r == 2) {
        if (cold) hipLaunchKernelGGL(k_ap_cold<2>, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, lam, w);
        else hipLaunchKernelGGL(k_ap_update<2>, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, lam, q, w);
    } else if (r == 3) {
        if (cold) hipLaunchKernelGGL(k_ap_cold<3>, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, lam, w);
        else hipLaunchKernelGGL(k_ap_update<3>, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, lam, q, w);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fista_pre(size_t n, int r, const float* y, const float* yp, float beta, const float* w, float* v,
                            hipStream_t s)
{
    if (r == 2) hipLaunchKernelGGL(k_fista_pre<2>, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, y, yp, beta, w, v);
    else if (r == 3) hipLaunchKernelGGL(k_fista_pre<3>, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, y, yp, beta, w, v);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace mc
