// grid8.hip -- 8-connected 2D grids: the zig-zag chain families (Sec. 3.1 and
// Fig. 1 of the paper) and the averaging step of the product-space splitting
// over four families (rows, columns, two zig-zag families).
//
// Strip r (rows r and r+1, r = 0..H-2) holds two zig-zag paths over the
// columns q = 0..W-1: path 0 visits row r + (q & 1), path 1 row r + 1 - (q & 1).
// Edge q of a path joins its positions q and q+1: the diagonal of cell (r, q),
// (r,q)-(r+1,q+1), when q + path is even, else its anti-diagonal
// (r+1,q)-(r,q+1).  The two paths share no vertex and hold every diagonal edge
// of the strip once; strips with even r form family 2, odd r family 3.
//
// The chain prox runs on a straightened copy: chain c = 2r + path is row c of
// a [2(H-1)][W] array (gathered, swept by the row prox kernel, scattered
// back).  Vertices on no path of a family are left alone by its prox.
// Duals of the diagonal edges are kept per cell: pdd[r][q] for the diagonal,
// pad[r][q] for the anti-diagonal (chain difference x_v - x_u along the path,
// u its position q), zero where the edge does not exist.
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

__global__ void k_zz_gather(int H, int W, const float* __restrict__ z2, const float* __restrict__ z3,
                            const float* __restrict__ add, const float* __restrict__ aad, float* __restrict__ zv,
                            float* __restrict__ za)
{
    const size_t nz = (size_t)2 * (H - 1) * W;
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < nz; k += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(k / W), q = (int)(k - (size_t)c * W);
        const int r = c >> 1, path = c & 1;
        const int row = r + ((q + path) & 1);
        const float* z = (r & 1) ? z3 : z2;
        zv[k] = z[(size_t)row * W + q];
        float a = 0.f;
        if (q + 1 < W) a = ((q + path) & 1) == 0 ? add[(size_t)r * W + q] : aad[(size_t)r * W + q];
        za[k] = a;
    }
}

__global__ void k_zz_scatter(int H, int W, const float* __restrict__ z2, const float* __restrict__ z3,
                             const float* __restrict__ zx, const float* __restrict__ zp, float* __restrict__ q2,
                             float* __restrict__ q3, float* __restrict__ pdd, float* __restrict__ pad)
{
    const size_t n = (size_t)H * W;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int rho = (int)(i / W), q = (int)(i - (size_t)rho * W);
#pragma unroll
        for (int pi = 0; pi < 2; ++pi) {
            float v = pi ? z3[i] : z2[i];  // identity off the family's paths
            if (rho >= pi) {
                const int r = pi + ((rho - pi) & ~1);  // the family's strip holding row rho
                if (r <= H - 2) {
                    const int path = rho == r ? (q & 1) : 1 - (q & 1);
                    v = zx[(size_t)(2 * r + path) * W + q];
                }
            }
            (pi ? q3 : q2)[i] = v;
        }
        if (zp) {
            float dd = 0.f, ad = 0.f;
            if (rho + 1 < H && q + 1 < W) {
                dd = zp[(size_t)(2 * rho + (q & 1)) * W + q];
                ad = zp[(size_t)(2 * rho + 1 - (q & 1)) * W + q];
            }
            pdd[i] = dd;
            pad[i] = ad;
        }
    }
}

// z_j' = y_j - (2Y - Z + w) / R with y_j = z_j - q_j, Y = sum y_j, Z = sum z_j
// Inputs are read once, with non-temporal loads: they then do not push out
// of L2 the lines the next sweep comes back to (volume solve -1 %).
template <int R>
__global__ void k_combine(size_t n, const float* __restrict__ z, const float* __restrict__ q,
                          const float* __restrict__ w, float* __restrict__ zn)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        float y[R], Y = 0.f, Z = 0.f;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const float zj = __builtin_nontemporal_load(z + j * n + i);
            y[j] = zj - __builtin_nontemporal_load(q + j * n + i);
            Y += y[j];
            Z += zj;
        }
        const float corr = (2.f * Y - Z + __builtin_nontemporal_load(w + i)) * (1.f / (float)R);
#pragma unroll
        for (int j = 0; j < R; ++j) zn[j * n + i] = y[j] - corr;
    }
}

}  // namespace

hipError_t launch_zz_gather(int H, int W, const float* z2, const float* z3, const float* add, const float* aad,
                            float* zv, float* za, hipStream_t s)
{
    if (H < 2) return hipSuccess;
    hipLaunchKernelGGL(k_zz_gather, dim3(blocks_for((size_t)2 * (H - 1) * W)), dim3(kThreads), 0, s, H, W, z2, z3,
                       add, aad, zv, za);
    return hipGetLastError();
}

hipError_t launch_zz_scatter(int H, int W, const float* z2, const float* z3, const float* zx, const float* zp,
                             float* q2, float* q3, float* pdd, float* pad, hipStream_t s)
{
    hipLaunchKernelGGL(k_zz_scatter, dim3(blocks_for((size_t)H * W)), dim3(kThreads), 0, s, H, W, z2, z3, zx, zp,
                       q2, q3, pdd, pad);
    return hipGetLastError();
}

hipError_t launch_combine3(size_t n, const float* z, const float* q, const float* w, float* zn, hipStream_t s)
{
    hipLaunchKernelGGL(k_combine<3>, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, z, q, w, zn);
    return hipGetLastError();
}

hipError_t launch_combine4(size_t n, const float* z, const float* q, const float* w, float* zn, hipStream_t s)
{
    hipLaunchKernelGGL(k_combine<4>, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, z, q, w, zn);
    return hipGetLastError();
}

}  // namespace mc
