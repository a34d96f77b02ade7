// reduce.hip -- certificate, cut energy, input validation and label kernels
// for gfx950.
//
// Grid-stride kernels over voxels; reductions accumulate in FP64, reduce each
// wave with xor-shuffles, then across the block in LDS, then across blocks in
// a single fixed-order block: results do not depend on timing.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "chain.hpp"
#include "launch.hpp"
#include "mc.h"

namespace mc {

namespace {

// ---- reductions ---------------------------------------------------------------

template <int NV>
__device__ __forceinline__ void block_reduce_store(double (&v)[NV], double* __restrict__ out)
{
    constexpr int kWaves = kReduceThreads / 64;
    __shared__ double sm[NV][kWaves];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_xor(v[q], off, 64);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) sm[q][wv] = v[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double s = 0.0;
            for (int k = 0; k < kWaves; ++k) s += sm[q][k];
            out[q] = s;
        }
    }
}

// sum of nblk rows of NV partials, fixed order
template <int NV>
__global__ void __launch_bounds__(kReduceThreads)
k_finalize(const double* __restrict__ partials, int nblk, double* __restrict__ out)
{
    double v[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = 0.0;
    // nblk <= kReduceBlocks: a fixed number of rounds, loads of all rounds in flight together
#pragma unroll
    for (int k = 0; k < kReduceBlocks / kReduceThreads; ++k) {
        const int b = threadIdx.x + k * kReduceThreads;
        if (b < nblk) {
#pragma unroll
            for (int q = 0; q < NV; ++q) v[q] += partials[b * NV + q];
        }
    }
    block_reduce_store<NV>(v, out);
}

// both reductions of the certificate in one block: out[0..kNumTau] from the
// ladder partials (kNumTau + 1 per block), out[kNumTau + 1] from the
// lower-bound partials (one per block)
__global__ void __launch_bounds__(kReduceThreads)
k_finalize_cert(const double* __restrict__ part_cut, const double* __restrict__ part_lb, int nblk,
                double* __restrict__ out)
{
    double v[kNumTau + 2];
#pragma unroll
    for (int q = 0; q < kNumTau + 2; ++q) v[q] = 0.0;
#pragma unroll
    for (int k = 0; k < kReduceBlocks / kReduceThreads; ++k) {
        const int b = threadIdx.x + k * kReduceThreads;
        if (b < nblk) {
#pragma unroll
            for (int q = 0; q <= kNumTau; ++q) v[q] += part_cut[b * (kNumTau + 1) + q];
            v[kNumTau + 1] += part_lb[b];
        }
    }
    block_reduce_store<kNumTau + 2>(v, out);
}

struct Coords {
    int x, y, d;
};

__device__ __forceinline__ Coords coords_of(const Geo& g, int i)
{
    Coords c;
    const int hw = g.H * g.W;
    c.d = i / hw;
    const int r = i - c.d * hw;
    c.y = r / g.W;
    c.x = r - c.y * g.W;
    return c;
}

struct Ptr3 {
    const float* p[3];
};

// Grid-stride walk over the voxels that carries the coordinates along: one
// division per thread at the start, then at most one carry per axis per step
// (x + sx < 2W and y + sy + 1 < 2H since both parts of the stride are reduced).
struct Walk {
    int i, stride, end;
    Coords c;
    int sx, sy, sd;

    __device__ __forceinline__ Walk(const Geo& g)
        : Walk(g, blockIdx.x * kReduceThreads + threadIdx.x, gridDim.x * kReduceThreads)
    {
    }
    __device__ __forceinline__ Walk(const Geo& g, int start, int step)
    {
        stride = step;
        end = g.n;
        i = start;
        c = coords_of(g, i < g.n ? i : 0);
        const Coords s = coords_of(g, stride);
        sx = s.x;
        sy = s.y;
        sd = s.d;
    }
    __device__ __forceinline__ void next(const Geo& g)
    {
        i += stride;
        c.x += sx;
        const int cx = c.x >= g.W ? 1 : 0;
        c.x -= cx ? g.W : 0;
        c.y += sy + cx;
        const int cy = c.y >= g.H ? 1 : 0;
        c.y -= cy ? g.H : 0;
        c.d += sd + cy;
    }
};

// Workgroups are dealt to the eight XCDs in turn (workgroup b runs on XCD
// b mod 8), each with its own L2.  With one walk over the whole grid the
// voxels one row away belong to workgroups on other XCDs, and a kernel that
// reads them fetches those lines from memory again (the certificate kernels:
// 1.2-1.3x their algorithmic bytes).  Here XCD x's workgroups walk together
// through their own contiguous eighth of the grid, so a round of them covers
// consecutive rows and the rows and slices next to it are in the same L2.
// The launch takes a multiple of 8 workgroups.
constexpr int kXcds = 8;

__device__ __forceinline__ Walk xcd_walk(const Geo& g)
{
    const int x = (int)blockIdx.x % kXcds;
    const int n8 = (g.n + kXcds - 1) / kXcds;
    Walk k(g, x * n8 + ((int)blockIdx.x / kXcds) * kReduceThreads + (int)threadIdx.x,
           ((int)gridDim.x / kXcds) * kReduceThreads);
    k.end = (x + 1) * n8 < g.n ? (x + 1) * n8 : g.n;
    return k;
}

// Primal estimate and lower bound from the edge duals (Sec. 2.2, 2.3):
// y = sum_j D_j^T p_j with p clipped to its box (so y lies in K exactly),
// x = -w - y (the TV primal x = w - y in the paper's sign), and
// LB(y) = sum_i min(y_i + w_i, 0).  Both are formed in FP64 from the FP32
// duals, which stay bounded by the weights, unlike the diverging state.
// Returns the voxel's LB term and writes its primal.
template <int ND>
__device__ __forceinline__ double primal_voxel(const Geo& g, const float* __restrict__ w,
                                               const Ptr3& p, float* __restrict__ xc, int i, const Coords& c)
{
    const int st[3] = {1, g.W, g.W * g.H};
    const int cc[3] = {c.x, c.y, c.d};
    double y = 0.0;
#pragma unroll
    for (int j = 0; j < ND; ++j) {
        y -= (double)p.p[j][i];  // zero on the last slice
        if (cc[j] > 0) y += (double)p.p[j][i - st[j]];
    }
    const double s = y + (double)w[i];
    xc[i] = (float)(-s);
    return s < 0.0 ? s : 0.0;
}

// The walk in groups of kGroup voxels: the loads of a whole group are issued
// before any of its stores (the arrays are not known not to alias, so a store
// would otherwise hold back the next voxel's loads), then the voxels are
// finished in walk order, so the sums are the same as voxel by voxel.
constexpr int kGroup = 4;
// The ladder holds eleven FP64 sums per lane: groups of two voxels keep it at
// 64 VGPRs, eight waves per SIMD, so that all kReduceBlocks blocks of a
// full-chip launch are resident at once (with groups of four, 86 VGPRs, five
// waves: the launch ran in two rounds; 256x256x128 volume 74.6 -> 71.0 us).
constexpr int kLadderGroup = 2;

template <int ND>
__global__ void __launch_bounds__(kReduceThreads)
k_primal(Geo g, const float* __restrict__ w, Ptr3 p, float* __restrict__ xc,
         double* __restrict__ partials)
{
    const int st[3] = {1, g.W, g.W * g.H};
    double lb = 0.0;
    Walk k = xcd_walk(g);
    while (k.i < k.end) {
        int idx[kGroup];
        bool ok[kGroup];
        float pc[kGroup][ND], pb[kGroup][ND], wv[kGroup];
        bool hb[kGroup][ND];
#pragma unroll
        for (int u = 0; u < kGroup; ++u) {
            ok[u] = k.i < k.end;
            idx[u] = ok[u] ? k.i : 0;
            const int cc[3] = {k.c.x, k.c.y, k.c.d};
#pragma unroll
            for (int j = 0; j < ND; ++j) hb[u][j] = ok[u] & (cc[j] > 0);
            k.next(g);
        }
#pragma unroll
        for (int u = 0; u < kGroup; ++u) {
            const int i = idx[u];
            wv[u] = w[i];
#pragma unroll
            for (int j = 0; j < ND; ++j) {
                pc[u][j] = p.p[j][i];  // zero on the last slice
                pb[u][j] = p.p[j][hb[u][j] ? i - st[j] : i];
            }
        }
#pragma unroll
        for (int u = 0; u < kGroup; ++u) {
            double y = 0.0;
#pragma unroll
            for (int j = 0; j < ND; ++j) {
                y -= (double)pc[u][j];
                if (hb[u][j]) y += (double)pb[u][j];
            }
            const double sv = y + (double)wv[u];
            if (ok[u]) {
                xc[idx[u]] = (float)(-sv);
                lb += sv < 0.0 ? sv : 0.0;
            }
        }
    }
    double v[1] = {lb};
    block_reduce_store<1>(v, partials + blockIdx.x);
}

// Energies of S_t = {x > tau_t} over the threshold ladder (eq. (4)) and the
// TV duality gap sum_e (a_e |Dx_e| - p_e Dx_e) at the rounded x (diagnostic).
// The ladder is decreasing, so x > tau_t holds exactly for t >= cnt(x) with
// cnt(x) = #{t : x <= tau_t}; a node enters S_t for t >= cnt and an edge is
// cut for t in [min(cnt_i, cnt_j), max(cnt_i, cnt_j)).
struct Taus {
    float t[kNumTau];
};

// Number of thresholds at or above x.  The ladder is descending and spans
// [-tau0, tau0]; most values lie outside it, and a wave counts the thresholds
// one by one only when one of its lanes holds a value inside (256x256x128
// volume: ladder kernel 69.2 -> 56.2 us).
__device__ __forceinline__ int ladder_count(float x, const Taus& tz)
{
    if (x > tz.t[0]) return 0;
    if (x <= tz.t[kNumTau - 1]) return kNumTau;
    int c = 0;
#pragma unroll
    for (int t = 0; t < kNumTau; ++t) c += (x <= tz.t[t]) ? 1 : 0;
    return c;
}

// Ladder accumulators: e[t] for the thresholds, e[kNumTau] the TV-gap term.
// Most nodes lie below or above every threshold (count 0 or kNumTau) and most
// edges join nodes of the same count: a node of count 0 adds to `all`, which
// store() folds into every e[t], an edge of equal counts adds nothing, and
// only the rest take the per-threshold adds, written without branches inside
// a region a wave skips when none of its lanes needs it.
struct Ladder {
    double e[kNumTau + 1];
    double all;

    __device__ __forceinline__ Ladder()
    {
#pragma unroll
        for (int t = 0; t <= kNumTau; ++t) e[t] = 0.0;
        all = 0.0;
    }
    // a node with cnt = c is in S_t for t >= c
    __device__ __forceinline__ void node(int c, double wv)
    {
        all += c == 0 ? wv : 0.0;
        if (c > 0 && c < kNumTau) {
#pragma unroll
            for (int t = 1; t < kNumTau; ++t)
                if (t >= c) e[t] += wv;
        }
    }
    // an edge between nodes of cnt cu and cv is cut for t in [min, max)
    __device__ __forceinline__ void edge(int cu, int cv, double av)
    {
        const int lo = cu < cv ? cu : cv, hi = cu < cv ? cv : cu;
        if (lo < hi) {
#pragma unroll
            for (int t = 0; t < kNumTau; ++t)
                if (t >= lo && t < hi) e[t] += av;
        }
    }
    // the block's sums (threshold energies, then the TV-gap term) to out
    __device__ __forceinline__ void store(double* out)
    {
#pragma unroll
        for (int t = 0; t < kNumTau; ++t) e[t] += all;
        block_reduce_store<kNumTau + 1>(e, out);
    }
};

template <int ND>
__device__ __forceinline__ void cut_voxel(const Geo& g, const float* __restrict__ xc,
                                          const float* __restrict__ w, const Ptr3& a,
                                          const Ptr3& p, const Taus& tz, int i, const Coords& c,
                                          Ladder& L)
{
    const int st[3] = {1, g.W, g.W * g.H};
    const int cc[3] = {c.x, c.y, c.d};
    const int ext[3] = {g.W, g.H, g.D};
    const float xi = xc[i];
    const int ci = ladder_count(xi, tz);
    L.node(ci, (double)w[i]);
#pragma unroll
    for (int j = 0; j < ND; ++j) {
        if (cc[j] + 1 < ext[j]) {
            const float xn = xc[i + st[j]];
            const double aj = (double)a.p[j][i];
            L.edge(ci, ladder_count(xn, tz), aj);
            const double dx = (double)xn - (double)xi;
            L.e[kNumTau] += aj * fabs(dx) - (double)p.p[j][i] * dx;
        }
    }
}

template <int ND>
__global__ void __launch_bounds__(kReduceThreads)
k_cut_ladder(Geo g, const float* __restrict__ xc, const float* __restrict__ w, Ptr3 a, Ptr3 p,
             Taus tz, double* __restrict__ partials)
{
    const int st[3] = {1, g.W, g.W * g.H};
    const int ext[3] = {g.W, g.H, g.D};
    Ladder L;
    Walk k = xcd_walk(g);
    while (k.i < k.end) {
        // loads of a group first (see kLadderGroup), then the voxels in walk order
        bool ok[kLadderGroup], he[kLadderGroup][ND];
        float xi[kLadderGroup], wv[kLadderGroup], xn[kLadderGroup][ND], av[kLadderGroup][ND], pv[kLadderGroup][ND];
#pragma unroll
        for (int u = 0; u < kLadderGroup; ++u) {
            ok[u] = k.i < k.end;
            const int i = ok[u] ? k.i : 0;
            const int cc[3] = {k.c.x, k.c.y, k.c.d};
            xi[u] = xc[i];
            wv[u] = w[i];
#pragma unroll
            for (int j = 0; j < ND; ++j) {
                he[u][j] = cc[j] + 1 < ext[j];
                xn[u][j] = xc[he[u][j] ? i + st[j] : i];
                av[u][j] = a.p[j][i];
                pv[u][j] = p.p[j][i];
            }
            k.next(g);
        }
#pragma unroll
        for (int u = 0; u < kLadderGroup; ++u) {
            if (!ok[u]) continue;
            const int ci = ladder_count(xi[u], tz);
            L.node(ci, (double)wv[u]);
#pragma unroll
            for (int j = 0; j < ND; ++j) {
                if (!he[u][j]) continue;  // no edge beyond the last slice
                const double aj = (double)av[u][j];
                L.edge(ci, ladder_count(xn[u][j], tz), aj);
                const double dx = (double)xn[u][j] - (double)xi[u];
                L.e[kNumTau] += aj * fabs(dx) - (double)pv[u][j] * dx;
            }
        }
    }
    L.store(partials + (size_t)blockIdx.x * (kNumTau + 1));
}

// ---- 8-connected 2D grids -------------------------------------------------------
//
// a[0..3] weigh the edges (r,c)-(r,c+1), (r,c)-(r+1,c), the diagonal
// (r,c)-(r+1,c+1) and the anti-diagonal (r+1,c)-(r,c+1), stored at vertex /
// cell (r,c) and zero where the edge does not exist; p[0..3] are the clipped
// duals of the same edges (p_e for the chain difference x_v - x_u, u the
// edge's left end).

struct Ptr4 {
    const float* p[4];
};

__device__ __forceinline__ double primal8_voxel(const Geo& g, const float* __restrict__ w, const Ptr4& p,
                                                float* __restrict__ xc, int i, int r, int c)
{
    const int W = g.W;
    // left end of its own row, column and diagonal edges
    double y = -(double)p.p[0][i] - (double)p.p[1][i] - (double)p.p[2][i];
    if (c > 0) y += (double)p.p[0][i - 1];
    if (r > 0) y += (double)p.p[1][i - W];
    if (r > 0 && c > 0) y += (double)p.p[2][i - W - 1];  // right end of the diagonal of cell (r-1, c-1)
    if (r > 0) y -= (double)p.p[3][i - W];               // left end (r'+1, c') of cell (r-1, c)
    if (c > 0) y += (double)p.p[3][i - 1];               // right end (r', c'+1) of cell (r, c-1)
    const double s = y + (double)w[i];
    xc[i] = (float)(-s);
    return s < 0.0 ? s : 0.0;
}

__global__ void __launch_bounds__(kReduceThreads)
k_primal8(Geo g, const float* __restrict__ w, Ptr4 p, float* __restrict__ xc, double* __restrict__ partials)
{
    double lb = 0.0;
    for (Walk k(g); k.i < g.n; k.next(g)) lb += primal8_voxel(g, w, p, xc, k.i, k.c.y, k.c.x);
    double v[1] = {lb};
    block_reduce_store<1>(v, partials + blockIdx.x);
}

// one edge u-v of weight ae and dual pe: ladder energies and TV-gap term
__device__ __forceinline__ void cut_edge(float xu, int cu, double ae, double pe, const Taus& tz,
                                         const float* __restrict__ xc, int v, Ladder& L)
{
    const float xn = xc[v];
    L.edge(cu, ladder_count(xn, tz), ae);
    const double dx = (double)xn - (double)xu;
    L.e[kNumTau] += ae * fabs(dx) - pe * dx;
}

__global__ void __launch_bounds__(kReduceThreads)
k_cut_ladder8(Geo g, const float* __restrict__ xc, const float* __restrict__ w, Ptr4 a, Ptr4 p, Taus tz,
              double* __restrict__ partials)
{
    Ladder L;
    const int W = g.W, H = g.H;
    for (Walk k(g); k.i < g.n; k.next(g)) {
        const int i = k.i, r = k.c.y, c = k.c.x;
        const float xi = xc[i];
        const int ci = ladder_count(xi, tz);
        L.node(ci, (double)w[i]);
        if (c + 1 < W) cut_edge(xi, ci, (double)a.p[0][i], (double)p.p[0][i], tz, xc, i + 1, L);
        if (r + 1 < H) cut_edge(xi, ci, (double)a.p[1][i], (double)p.p[1][i], tz, xc, i + W, L);
        if (r + 1 < H && c + 1 < W) {
            cut_edge(xi, ci, (double)a.p[2][i], (double)p.p[2][i], tz, xc, i + W + 1, L);
            // anti-diagonal of cell (r, c): from (r+1, c) to (r, c+1)
            const float xu = xc[i + W];
            cut_edge(xu, ladder_count(xu, tz), (double)a.p[3][i], (double)p.p[3][i], tz, xc, i + 1, L);
        }
    }
    L.store(partials + (size_t)blockIdx.x * (kNumTau + 1));
}

__global__ void __launch_bounds__(kReduceThreads)
k_energy8(Geo g, const float* __restrict__ w, Ptr4 a, const uint8_t* __restrict__ lab, double* __restrict__ partials)
{
    double e = 0.0;
    const int stride = gridDim.x * kReduceThreads;
    const int W = g.W, H = g.H;
    for (int i = blockIdx.x * kReduceThreads + threadIdx.x; i < g.n; i += stride) {
        const int r = i / W, c = i - r * W;
        const bool b = lab[i] != 0;
        if (b) e += (double)w[i];
        if (c + 1 < W && b != (lab[i + 1] != 0)) e += (double)a.p[0][i];
        if (r + 1 < H && b != (lab[i + W] != 0)) e += (double)a.p[1][i];
        if (r + 1 < H && c + 1 < W) {
            if (b != (lab[i + W + 1] != 0)) e += (double)a.p[2][i];
            if ((lab[i + W] != 0) != (lab[i + 1] != 0)) e += (double)a.p[3][i];
        }
    }
    double v[1] = {e};
    block_reduce_store<1>(v, partials + blockIdx.x);
}

// out[0]: negative weights or non-zero weights of missing edges, out[1]: non-finite values
__global__ void __launch_bounds__(kReduceThreads)
k_validate8(Geo g, const float* __restrict__ w, Ptr4 a, double* __restrict__ partials)
{
    double bad = 0.0, nonfinite = 0.0;
    const int stride = gridDim.x * kReduceThreads;
    const int W = g.W, H = g.H;
    for (int i = blockIdx.x * kReduceThreads + threadIdx.x; i < g.n; i += stride) {
        const int r = i / W, c = i - r * W;
        if (!isfinite(w[i])) nonfinite += 1.0;
        const bool exists[4] = {c + 1 < W, r + 1 < H, r + 1 < H && c + 1 < W, r + 1 < H && c + 1 < W};
        for (int j = 0; j < 4; ++j) {
            const float v = a.p[j][i];
            if (!isfinite(v)) nonfinite += 1.0;
            else if (v < 0.f || (!exists[j] && v != 0.f)) bad += 1.0;
        }
    }
    double v[2] = {bad, nonfinite};
    block_reduce_store<2>(v, partials + 2 * blockIdx.x);
}

// ---- batched: every reduction block belongs to one grid ------------------------

__device__ __forceinline__ Ptr3 batch_duals(const BatchGrid& t)
{
    Ptr3 p;
    p.p[0] = t.p;
    p.p[1] = t.p + t.g.n;
    p.p[2] = nullptr;
    return p;
}

__global__ void __launch_bounds__(kReduceThreads)
k_batch_primal(BatchLaunch b, double* __restrict__ partials)
{
    const BatchGrid& t = b.tab[b.blk_grid[blockIdx.x]];
    if (t.done) return;
    const Ptr3 p = batch_duals(t);
    double lb = 0.0;
    for (Walk k(t.g, ((int)blockIdx.x - t.blk0) * kReduceThreads + threadIdx.x, t.nblk * kReduceThreads); k.i < t.g.n;
         k.next(t.g))
        lb += primal_voxel<2>(t.g, t.w, p, t.xc, k.i, k.c);
    double v[1] = {lb};
    block_reduce_store<1>(v, partials + (size_t)blockIdx.x * kCertValues + kNumTau + 1);
}

__global__ void __launch_bounds__(kReduceThreads)
k_batch_cut(BatchLaunch b, Taus tz, double* __restrict__ partials)
{
    const BatchGrid& t = b.tab[b.blk_grid[blockIdx.x]];
    if (t.done) return;
    Ptr3 a;
    a.p[0] = t.ax;
    a.p[1] = t.ay;
    a.p[2] = nullptr;
    const Ptr3 p = batch_duals(t);
    Ladder L;
    for (Walk k(t.g, ((int)blockIdx.x - t.blk0) * kReduceThreads + threadIdx.x, t.nblk * kReduceThreads); k.i < t.g.n;
         k.next(t.g))
        cut_voxel<2>(t.g, t.xc, t.w, a, p, tz, k.i, k.c, L);
    L.store(partials + (size_t)blockIdx.x * kCertValues);
}

// one block per grid: fixed-order sum of the grid's block partials, then the
// certificate and the decision
__global__ void __launch_bounds__(kReduceThreads)
k_batch_finalize(BatchLaunch b, const double* __restrict__ partials, double gap_tol,
                 const int* __restrict__ iter_dev)
{
    BatchGrid& t = b.tab[blockIdx.x];
    if (t.done) return;
    double v[kCertValues];
#pragma unroll
    for (int q = 0; q < kCertValues; ++q) v[q] = 0.0;
    for (int k = threadIdx.x; k < t.nblk; k += kReduceThreads) {
#pragma unroll
        for (int q = 0; q < kCertValues; ++q) v[q] += partials[(size_t)(t.blk0 + k) * kCertValues + q];
    }
    __shared__ double tot[kCertValues];
    block_reduce_store<kCertValues>(v, tot);
    __syncthreads();
    if (threadIdx.x != 0) return;
    double best = tot[0];
    int bi = 0;
    for (int q = 1; q < kNumTau; ++q) {
        if (tot[q] < best) {
            best = tot[q];
            bi = q;
        }
    }
    for (int q = 0; q < kNumTau; ++q) t.e[q] = tot[q];
    t.tvgap = tot[kNumTau];
    t.lb = tot[kNumTau + 1];
    t.cert = best - t.lb;
    t.tau_idx = bi;
    t.iters = *iter_dev;
    t.checks += 1;
    if (t.cert < gap_tol) {
        t.done = 1;
        t.t_done = wall_clock64();
    }
}

// number of grids of a batch not finished yet (one wave)
__global__ void __launch_bounds__(64) k_batch_undone(BatchLaunch b, int* __restrict__ out)
{
    int c = 0;
    for (int g = threadIdx.x; g < b.n_grids; g += 64) c += b.tab[g].done ? 0 : 1;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if (threadIdx.x == 0) *out = c;
}

__global__ void __launch_bounds__(kReduceThreads) k_batch_labels(BatchLaunch b, Taus tz)
{
    const BatchGrid& t = b.tab[b.blk_grid[blockIdx.x]];
    const float tau = tz.t[t.tau_idx];
    const int stride = t.nblk * kReduceThreads;
    for (int i = ((int)blockIdx.x - t.blk0) * kReduceThreads + threadIdx.x; i < t.g.n; i += stride) {
        const float x = t.xc[i];
        t.labels[i] = x > tau ? 1 : 0;
        if (t.x_out) t.x_out[i] = x;
    }
}

__global__ void k_set_int(int* dst, int v) { *dst = v; }

// First product-space iteration from z = 0: every prox of 0 is 0, so
// z_j' = y_j - (2Y - Z - u)/r = -(w * (1/r)) for every family j (the same FP32
// expression the fused final sweep evaluates).
__global__ void k_cold_product(const float* __restrict__ w, int n, int r, float* __restrict__ zn)
{
    const float inv = 1.f / (float)r;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float v = -(w[i] * inv);
        for (int j = 0; j < r; ++j) zn[(size_t)j * n + i] = v;
    }
}

__global__ void k_stamp(unsigned long long* dst) { *dst = wall_clock64(); }

__global__ void __launch_bounds__(kReduceThreads)
k_energy(Geo g, const float* __restrict__ w, Ptr3 a, const uint8_t* __restrict__ lab,
         double* __restrict__ partials)
{
    double e = 0.0;
    const int st[3] = {1, g.W, g.W * g.H};
    for (Walk k(g); k.i < g.n; k.next(g)) {
        const int i = k.i;
        const int cc[3] = {k.c.x, k.c.y, k.c.d};
        const int ext[3] = {g.W, g.H, g.D};
        const bool b = lab[i] != 0;
        if (b) e += (double)w[i];
        for (int j = 0; j < g.ndim; ++j) {
            if (cc[j] + 1 < ext[j]) {
                if (b != (lab[i + st[j]] != 0)) e += (double)a.p[j][i];
            }
        }
    }
    double v[1] = {e};
    block_reduce_store<1>(v, partials + blockIdx.x);
}

__global__ void __launch_bounds__(kReduceThreads)
k_validate(Geo g, const float* __restrict__ w, Ptr3 a, double* __restrict__ partials)
{
    double bad_w = 0.0, nonfin = 0.0;
    for (Walk k(g); k.i < g.n; k.next(g)) {
        const int i = k.i;
        const int cc[3] = {k.c.x, k.c.y, k.c.d};
        const int ext[3] = {g.W, g.H, g.D};
        if (!isfinite(w[i])) nonfin += 1.0;
        for (int j = 0; j < g.ndim; ++j) {
            const float aj = a.p[j][i];
            if (!isfinite(aj)) nonfin += 1.0;
            else if (aj < 0.f || (cc[j] + 1 == ext[j] && aj != 0.f)) bad_w += 1.0;
        }
    }
    double v[2] = {bad_w, nonfin};
    block_reduce_store<2>(v, partials + (size_t)blockIdx.x * 2);
}

// Debug checks of the edge duals of a check iteration: out[0] = duals
// outside their box |p_j| <= a_j (or not finite), out[1] = non-zero duals on
// a family's last slice, where no edge exists.
__global__ void __launch_bounds__(kReduceThreads)
k_debug_duals(Geo g, Ptr3 a, Ptr3 p, double* __restrict__ partials)
{
    double out_box = 0.0, on_last = 0.0;
    for (Walk k(g); k.i < g.n; k.next(g)) {
        const int i = k.i;
        const int cc[3] = {k.c.x, k.c.y, k.c.d};
        const int ext[3] = {g.W, g.H, g.D};
        for (int j = 0; j < g.ndim; ++j) {
            const float pj = p.p[j][i], aj = a.p[j][i];
            if (!(fabsf(pj) <= aj)) out_box += 1.0;
            if (cc[j] + 1 == ext[j] && pj != 0.f) on_last += 1.0;
        }
    }
    double v[2] = {out_box, on_last};
    block_reduce_store<2>(v, partials + (size_t)blockIdx.x * 2);
}

__global__ void __launch_bounds__(kReduceThreads)
k_count_nonfinite(const float* __restrict__ x, int n, double* __restrict__ partials)
{
    double c = 0.0;
    const int stride = gridDim.x * kReduceThreads;
    for (int i = blockIdx.x * kReduceThreads + threadIdx.x; i < n; i += stride)
        if (!isfinite(x[i])) c += 1.0;
    double v[1] = {c};
    block_reduce_store<1>(v, partials + blockIdx.x);
}

// ---- multi-label energies (alpha-expansion) -------------------------------------

// number of labels outside [0, L)
__global__ void __launch_bounds__(kReduceThreads)
k_check_labels(int n, int L, const int32_t* __restrict__ f, double* __restrict__ partials)
{
    double bad = 0.0;
    const int stride = gridDim.x * kReduceThreads;
    for (int i = blockIdx.x * kReduceThreads + threadIdx.x; i < n; i += stride)
        if (f[i] < 0 || f[i] >= L) bad += 1.0;
    double v[1] = {bad};
    block_reduce_store<1>(v, partials + blockIdx.x);
}

// the pairwise metric: Potts [a != b] or truncated linear min(|a - b|, T)
__device__ __forceinline__ float ml_v(int kind, float trunc, int a, int b)
{
    if (kind == MC_V_POTTS) return a != b ? 1.f : 0.f;
    const float d = (float)(a > b ? a - b : b - a);
    return d < trunc ? d : trunc;
}

// E(f) = sum_i data[f_i][i] + sum_e lam_e V(f_u, f_v): FP64 sums of FP32 terms
// (each lam_e V a product of two exact FP32 values, formed in FP64)
__global__ void __launch_bounds__(kReduceThreads)
k_ml_energy(Geo g, const float* __restrict__ data, const float* __restrict__ lx, const float* __restrict__ ly,
            int kind, float trunc, const int32_t* __restrict__ f, double* __restrict__ partials)
{
    double e = 0.0;
    for (Walk k(g); k.i < g.n; k.next(g)) {
        const int i = k.i, fi = f[i];
        e += (double)data[(size_t)fi * g.n + i];
        if (k.c.x + 1 < g.W) e += (double)lx[i] * (double)ml_v(kind, trunc, fi, f[i + 1]);
        if (k.c.y + 1 < g.H) e += (double)ly[i] * (double)ml_v(kind, trunc, fi, f[i + g.W]);
    }
    double v[1] = {e};
    block_reduce_store<1>(v, partials + blockIdx.x);
}

__global__ void __launch_bounds__(kReduceThreads)
k_labels(int n, const float* __restrict__ xc, float tau, uint8_t* __restrict__ lab)
{
    const int stride = gridDim.x * kReduceThreads;
    for (int i = blockIdx.x * kReduceThreads + threadIdx.x; i < n; i += stride)
        lab[i] = xc[i] > tau ? 1 : 0;
}

inline int reduce_blocks(int n)
{
    int b = (n + kReduceThreads - 1) / kReduceThreads;
    return b < 1 ? 1 : (b > kReduceBlocks ? kReduceBlocks : b);
}

}  // namespace

// ---- launchers ----------------------------------------------------------------

hipError_t launch_cert(const Geo& g, const float* w, const float* const* a,
                       const float* const* p, float tau0, float* xc, double* partials,
                       double* out, hipStream_t s)
{
    Ptr3 pa, pp;
    for (int j = 0; j < 3; ++j) {
        pa.p[j] = j < g.ndim ? a[j] : nullptr;
        pp.p[j] = j < g.ndim ? p[j] : nullptr;
    }
    Taus tz;
    tau_ladder(tau0, tz.t);
    const int nb = (reduce_blocks(g.n) + kXcds - 1) / kXcds * kXcds;  // <= kReduceBlocks
    double* part_lb = partials;
    double* part_cut = partials + kReduceBlocks;
    if (g.ndim == 3) {
        hipLaunchKernelGGL(k_primal<3>, dim3(nb), dim3(kReduceThreads), 0, s, g, w, pp, xc, part_lb);
        hipLaunchKernelGGL(k_cut_ladder<3>, dim3(nb), dim3(kReduceThreads), 0, s, g, xc, w, pa, pp, tz, part_cut);
    } else {
        hipLaunchKernelGGL(k_primal<2>, dim3(nb), dim3(kReduceThreads), 0, s, g, w, pp, xc, part_lb);
        hipLaunchKernelGGL(k_cut_ladder<2>, dim3(nb), dim3(kReduceThreads), 0, s, g, xc, w, pa, pp, tz, part_cut);
    }
    hipLaunchKernelGGL(k_finalize_cert, dim3(1), dim3(kReduceThreads), 0, s, part_cut, part_lb, nb, out);
    return hipGetLastError();
}

hipError_t launch_cert8(const Geo& g, const float* w, const float* const* a, const float* const* p, float tau0,
                        float* xc, double* partials, double* out, hipStream_t s)
{
    Ptr4 pa, pp;
    for (int j = 0; j < 4; ++j) {
        pa.p[j] = a[j];
        pp.p[j] = p[j];
    }
    Taus tz;
    tau_ladder(tau0, tz.t);
    const int nb = reduce_blocks(g.n);
    double* part_cut = partials;
    double* part_lb = partials + (size_t)nb * (kNumTau + 1);
    hipLaunchKernelGGL(k_primal8, dim3(nb), dim3(kReduceThreads), 0, s, g, w, pp, xc, part_lb);
    hipLaunchKernelGGL(k_cut_ladder8, dim3(nb), dim3(kReduceThreads), 0, s, g, xc, w, pa, pp, tz, part_cut);
    hipLaunchKernelGGL(k_finalize_cert, dim3(1), dim3(kReduceThreads), 0, s, part_cut, part_lb, nb, out);
    return hipGetLastError();
}

hipError_t launch_energy8(const Geo& g, const float* w, const float* const* a, const uint8_t* labels,
                          double* partials, double* out, hipStream_t s)
{
    Ptr4 pa;
    for (int j = 0; j < 4; ++j) pa.p[j] = a[j];
    const int nb = reduce_blocks(g.n);
    hipLaunchKernelGGL(k_energy8, dim3(nb), dim3(kReduceThreads), 0, s, g, w, pa, labels, partials);
    hipLaunchKernelGGL(k_finalize<1>, dim3(1), dim3(kReduceThreads), 0, s, partials, nb, out);
    return hipGetLastError();
}

hipError_t launch_validate8(const Geo& g, const float* w, const float* const* a, double* partials, double* out,
                            hipStream_t s)
{
    Ptr4 pa;
    for (int j = 0; j < 4; ++j) pa.p[j] = a[j];
    const int nb = reduce_blocks(g.n);
    hipLaunchKernelGGL(k_validate8, dim3(nb), dim3(kReduceThreads), 0, s, g, w, pa, partials);
    hipLaunchKernelGGL(k_finalize<2>, dim3(1), dim3(kReduceThreads), 0, s, partials, nb, out);
    return hipGetLastError();
}

hipError_t launch_batch_check(const BatchLaunch& b, float tau0, double gap_tol, const int* iter_dev,
                              double* partials, hipStream_t s)
{
    Taus tz;
    tau_ladder(tau0, tz.t);
    hipLaunchKernelGGL(k_batch_primal, dim3(b.blocks), dim3(kReduceThreads), 0, s, b, partials);
    hipLaunchKernelGGL(k_batch_cut, dim3(b.blocks), dim3(kReduceThreads), 0, s, b, tz, partials);
    hipLaunchKernelGGL(k_batch_finalize, dim3(b.n_grids), dim3(kReduceThreads), 0, s, b, partials,
                       gap_tol, iter_dev);
    return hipGetLastError();
}

hipError_t launch_batch_undone(const BatchLaunch& b, int* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_undone, dim3(1), dim3(64), 0, s, b, out);
    return hipGetLastError();
}

hipError_t launch_batch_labels(const BatchLaunch& b, float tau0, hipStream_t s)
{
    Taus tz;
    tau_ladder(tau0, tz.t);
    hipLaunchKernelGGL(k_batch_labels, dim3(b.blocks), dim3(kReduceThreads), 0, s, b, tz);
    return hipGetLastError();
}

hipError_t launch_cold_product(const Geo& g, int r, const float* w, float* zn, hipStream_t s)
{
    const int blocks = (g.n + 255) / 256 < 2048 ? (g.n + 255) / 256 : 2048;
    hipLaunchKernelGGL(k_cold_product, dim3(blocks), dim3(256), 0, s, w, g.n, r, zn);
    return hipGetLastError();
}

hipError_t launch_set_int(int* dst, int value, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, dst, value);
    return hipGetLastError();
}

hipError_t launch_stamp(unsigned long long* dst, hipStream_t s)
{
    hipLaunchKernelGGL(k_stamp, dim3(1), dim3(1), 0, s, dst);
    return hipGetLastError();
}

hipError_t launch_labels(const Geo& g, const float* xc, float tau, uint8_t* labels, hipStream_t s)
{
    hipLaunchKernelGGL(k_labels, dim3(reduce_blocks(g.n)), dim3(kReduceThreads), 0, s, g.n, xc,
                       tau, labels);
    return hipGetLastError();
}

hipError_t launch_energy(const Geo& g, const float* w, const float* const* a,
                         const uint8_t* labels, double* partials, double* out, hipStream_t s)
{
    Ptr3 pa;
    for (int j = 0; j < 3; ++j) pa.p[j] = j < g.ndim ? a[j] : nullptr;
    const int nb = reduce_blocks(g.n);
    hipLaunchKernelGGL(k_energy, dim3(nb), dim3(kReduceThreads), 0, s, g, w, pa, labels, partials);
    hipLaunchKernelGGL(k_finalize<1>, dim3(1), dim3(kReduceThreads), 0, s, partials, nb, out);
    return hipGetLastError();
}

hipError_t launch_validate(const Geo& g, const float* w, const float* const* a,
                           double* partials, double* out, hipStream_t s)
{
    Ptr3 pa;
    for (int j = 0; j < 3; ++j) pa.p[j] = j < g.ndim ? a[j] : nullptr;
    const int nb = reduce_blocks(g.n);
    hipLaunchKernelGGL(k_validate, dim3(nb), dim3(kReduceThreads), 0, s, g, w, pa, partials);
    hipLaunchKernelGGL(k_finalize<2>, dim3(1), dim3(kReduceThreads), 0, s, partials, nb, out);
    return hipGetLastError();
}

hipError_t launch_check_labels(int n, int L, const int32_t* f, double* partials, double* out, hipStream_t s)
{
    const int nb = reduce_blocks(n);
    hipLaunchKernelGGL(k_check_labels, dim3(nb), dim3(kReduceThreads), 0, s, n, L, f, partials);
    hipLaunchKernelGGL(k_finalize<1>, dim3(1), dim3(kReduceThreads), 0, s, partials, nb, out);
    return hipGetLastError();
}

hipError_t launch_ml_energy(const Geo& g, const float* data, const float* const* lam, int kind, float trunc,
                            const int32_t* f, double* partials, double* out, hipStream_t s)
{
    const int nb = reduce_blocks(g.n);
    hipLaunchKernelGGL(k_ml_energy, dim3(nb), dim3(kReduceThreads), 0, s, g, data, lam[0], lam[1], kind, trunc, f,
                       partials);
    hipLaunchKernelGGL(k_finalize<1>, dim3(1), dim3(kReduceThreads), 0, s, partials, nb, out);
    return hipGetLastError();
}

hipError_t launch_debug_duals(const Geo& g, const float* const* a, const float* const* p, double* partials,
                             double* out, hipStream_t s)
{
    const int nb = reduce_blocks(g.n);
    Ptr3 pa, pp;
    for (int j = 0; j < 3; ++j) {
        pa.p[j] = j < g.ndim ? a[j] : nullptr;
        pp.p[j] = j < g.ndim ? p[j] : nullptr;
    }
    hipLaunchKernelGGL(k_debug_duals, dim3(nb), dim3(kReduceThreads), 0, s, g, pa, pp, partials);
    hipLaunchKernelGGL(k_finalize<2>, dim3(1), dim3(kReduceThreads), 0, s, partials, nb, out);
    return hipGetLastError();
}

hipError_t launch_count_nonfinite(const float* x, int n, double* partials, double* out,
                                  hipStream_t s)
{
    const int nb = reduce_blocks(n);
    hipLaunchKernelGGL(k_count_nonfinite, dim3(nb), dim3(kReduceThreads), 0, s, x, n, partials);
    hipLaunchKernelGGL(k_finalize<1>, dim3(1), dim3(kReduceThreads), 0, s, partials, nb, out);
    return hipGetLastError();
}

}  // namespace mc
