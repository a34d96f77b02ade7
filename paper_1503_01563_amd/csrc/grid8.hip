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
// a [2(H-1)][W] array (gathered once, swept by the row prox kernel; the
// averaging step reads the prox from there and writes the next state back in
// both layouts).  Vertices on no path of a family are left alone by its prox.
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

// The averaging step over the four families, z_j' = y_j - (2Y - Z + w)/4 with
// y_j = z_j - q_j, taking the zig-zag families' prox q_2, q_3 straight from the
// straightened chains zx: at the vertex's position on its path of the family,
// or q_j = z_j (identity) on no path.  Besides zn per vertex it writes zn of
// families 2 and 3 straightened into zv, the next sweep's input, and, when zp
// is not null, the diagonal and anti-diagonal duals per cell.  (One pass in
// place of a scatter of q_2, q_3, the averaging and a gather of the next state:
// 15 floats per vertex moved instead of 27.)  A block takes a tile of 8 rows
// by 32 columns, so that a wave holds two whole rows of a strip: the two paths
// alternate between the strip's rows column by column, and the halves of each
// straightened line are then read and written by the same wave.
constexpr int kTileW = 32, kTileH = kThreads / kTileW;

__global__ void __launch_bounds__(kThreads) k_combine8(int H, int W, const float* __restrict__ z, const float* __restrict__ q01,
                           const float* __restrict__ zx, const float* __restrict__ zp, const float* __restrict__ w,
                           float* __restrict__ zn, float* __restrict__ zv, float* __restrict__ pdd,
                           float* __restrict__ pad)
{
    const int n = H * W;
    const int tw = (W + kTileW - 1) / kTileW, ntiles = tw * ((H + kTileH - 1) / kTileH);
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int rho = (t / tw) * kTileH + (int)threadIdx.x / kTileW;
        const int q = (t % tw) * kTileW + (int)threadIdx.x % kTileW;
        if (rho >= H || q >= W) continue;
        const int i = rho * W + q;
        int k[2];  // position in zx / zv on family 2 + pi's path through the vertex, or -1
#pragma unroll
        for (int pi = 0; pi < 2; ++pi) {
            k[pi] = -1;
            const int r = pi + ((rho - pi) & ~1);  // the family's strip holding row rho
            if (rho >= pi && r <= H - 2) k[pi] = (2 * r + (rho == r ? (q & 1) : 1 - (q & 1))) * W + q;
        }
        float y[4], Y = 0.f, Z = 0.f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float zj = __builtin_nontemporal_load(z + (size_t)j * n + i);
            float qj;
            if (j < 2) qj = __builtin_nontemporal_load(q01 + (size_t)j * n + i);
            else qj = k[j - 2] >= 0 ? __builtin_nontemporal_load(zx + k[j - 2]) : zj;
            y[j] = zj - qj;
            Y += y[j];
            Z += zj;
        }
        const float corr = (2.f * Y - Z + __builtin_nontemporal_load(w + i)) * 0.25f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float v = y[j] - corr;
            zn[(size_t)j * n + i] = v;
            if (j >= 2 && k[j - 2] >= 0) zv[k[j - 2]] = v;
        }
        if (zp) {
            float dd = 0.f, ad = 0.f;
            if (rho + 1 < H && q + 1 < W) {
                dd = zp[(2 * rho + (q & 1)) * W + q];
                ad = zp[(2 * rho + 1 - (q & 1)) * W + q];
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

hipError_t launch_combine8(int H, int W, const float* z, const float* q01, const float* zx, const float* zp,
                           const float* w, float* zn, float* zv, float* pdd, float* pad, hipStream_t s)
{
    const size_t tiles = (size_t)((W + kTileW - 1) / kTileW) * ((H + kTileH - 1) / kTileH);
    hipLaunchKernelGGL(k_combine8, dim3(blocks_for(tiles * kThreads)), dim3(kThreads), 0, s, H, W, z, q01, zx, zp,
                       w, zn, zv, pdd, pad);
    return hipGetLastError();
}

hipError_t launch_combine3(size_t n, const float* z, const float* q, const float* w, float* zn, hipStream_t s)
{
    hipLaunchKernelGGL(k_combine<3>, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, z, q, w, zn);
    return hipGetLastError();
}

}  // namespace mc
