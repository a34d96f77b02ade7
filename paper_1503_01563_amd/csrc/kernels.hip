// kernels.hip -- chain-prox sweeps, splitting steps, certificate and energy
// reductions for gfx950.
//
// Sweeps map one chain to one lane (wave64).  Chains along H and D are
// indexed so that neighbouring lanes hold neighbouring W positions: their
// loads and stores coalesce.  Chains along W are read through the caches.
// Reductions accumulate in FP64, reduce each wave with xor-shuffles, then
// across the block in LDS, then across blocks in a single fixed-order block:
// results do not depend on timing.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "chain.hpp"
#include "launch.hpp"

namespace mc {

namespace {

constexpr int kSweepThreads = 64;

struct Chain {
    int base, stride, m;
};

__device__ __forceinline__ Chain chain_of(const Geo g, int axis, int c)
{
    Chain ch;
    if (axis == 0) {
        ch.base = c * g.W;
        ch.stride = 1;
        ch.m = g.W;
    } else if (axis == 1) {
        const int d = c / g.W;
        const int x = c - d * g.W;
        ch.base = d * g.H * g.W + x;
        ch.stride = g.W;
        ch.m = g.H;
    } else {
        ch.base = c;
        ch.stride = g.H * g.W;
        ch.m = g.D;
    }
    return ch;
}

// ---- chain functors -------------------------------------------------------

struct ChainBase {
    int base, stride;
    SegRec* rec;
    __device__ __forceinline__ int idx(int k) const { return base + k * stride; }
    __device__ __forceinline__ void put(int k, double val, uint32_t info) const
    {
        SegRec r;
        r.val = val;
        r.info = info;
        r.pad = 0u;
        rec[idx(k)] = r;
    }
    __device__ __forceinline__ SegRec get(int k) const { return rec[idx(k)]; }
};

// plain prox: x = c, optional clipped duals
struct ProxF : ChainBase {
    const float* vin;
    const float* aa;
    float* x;
    float* p;
    __device__ __forceinline__ float v(int k) const { return vin[idx(k)]; }
    __device__ __forceinline__ float a(int k) const { return aa[idx(k)]; }
    __device__ __forceinline__ double emit(int j, double c64, double pj, bool last)
    {
        const int i = idx(j);
        x[i] = (float)c64;
        if (p) {
            p[i] = last ? 0.f : clip_dual(pj, aa[i]);
            return pj - c64 + (double)vin[i];
        }
        return 0.0;
    }
};

// two-set rows: v = z; t = u + q1 - y1, y1 = z - q1
struct Dr2RowF : ChainBase {
    const float* z;
    const float* ax;
    const float* w;
    float* t;
    float* y1;
    float* p1;
    __device__ __forceinline__ float v(int k) const { return z[idx(k)]; }
    __device__ __forceinline__ float a(int k) const { return ax[idx(k)]; }
    __device__ __forceinline__ double emit(int j, double c64, double pj, bool last)
    {
        const int i = idx(j);
        const float c = (float)c64;
        const float zi = z[i];
        const float yi = zi - c;
        y1[i] = yi;
        t[i] = (c - yi) - w[i];
        if (p1) {
            p1[i] = last ? 0.f : clip_dual(pj, ax[i]);
            return pj - c64 + (double)zi;
        }
        return 0.0;
    }
};

// two-set columns: v = t; z <- y1 + q2; checks: p2
struct Dr2ColF : ChainBase {
    const float* t;
    const float* ay;
    const float* y1;
    float* z;
    float* p2;
    __device__ __forceinline__ float v(int k) const { return t[idx(k)]; }
    __device__ __forceinline__ float a(int k) const { return ay[idx(k)]; }
    __device__ __forceinline__ double emit(int j, double c64, double pj, bool last)
    {
        const int i = idx(j);
        const float c = (float)c64;
        const float yi = y1[i];
        z[i] = yi + c;
        if (p2) {
            p2[i] = last ? 0.f : clip_dual(pj, ay[i]);
            return pj - c64 + (double)t[i];
        }
        return 0.0;
    }
};

// product space, non-final family: y_j = z_j - q_j
struct DrpSweepF : ChainBase {
    const float* zj;
    const float* aj;
    float* yj;
    float* pj_out;
    __device__ __forceinline__ float v(int k) const { return zj[idx(k)]; }
    __device__ __forceinline__ float a(int k) const { return aj[idx(k)]; }
    __device__ __forceinline__ double emit(int j, double c64, double pj, bool last)
    {
        const int i = idx(j);
        const float c = (float)c64;
        const float zi = zj[i];
        yj[i] = zi - c;
        if (pj_out) {
            pj_out[i] = last ? 0.f : clip_dual(pj, aj[i]);
            return pj - c64 + (double)zi;
        }
        return 0.0;
    }
};

// product space, final family fused with the average step
template <int R>
struct DrpFinalF : ChainBase {
    float* z;        // R*n, family j at j*n
    const float* y;  // (R-1)*n
    const float* al;
    const float* w;
    float* pl;
    int n;
    __device__ __forceinline__ float v(int k) const { return z[(R - 1) * n + idx(k)]; }
    __device__ __forceinline__ float a(int k) const { return al[idx(k)]; }
    __device__ __forceinline__ double emit(int j, double c64, double pj, bool last)
    {
        const int i = idx(j);
        const float c = (float)c64;
        const float zl = z[(R - 1) * n + i];
        const float yl = zl - c;
        float yv[R];
        float Y = yl, Z = zl;
#pragma unroll
        for (int q = 0; q < R - 1; ++q) {
            yv[q] = y[q * n + i];
            Y += yv[q];
            Z += z[q * n + i];
        }
        const float u = -w[i];
        const float corr = (2.f * Y - Z - u) * (1.f / (float)R);
#pragma unroll
        for (int q = 0; q < R - 1; ++q) z[q * n + i] = yv[q] - corr;
        z[(R - 1) * n + i] = yl - corr;
        if (pl) {
            pl[i] = last ? 0.f : clip_dual(pj, al[i]);
            return pj - c64 + (double)zl;
        }
        return 0.0;
    }
};

template <class F>
__device__ __forceinline__ void run_chain(F& f, int m)
{
    chain_scan(f, m);
    chain_fill(f, m);
}

// ---- sweep kernels ----------------------------------------------------------

__global__ void __launch_bounds__(kSweepThreads)
k_prox(Geo g, int axis, const float* __restrict__ v, const float* __restrict__ a,
       float* __restrict__ x, float* __restrict__ p, SegRec* __restrict__ rec)
{
    const int c = blockIdx.x * kSweepThreads + threadIdx.x;
    if (c >= geo_nchains(g, axis)) return;
    const Chain ch = chain_of(g, axis, c);
    ProxF f;
    f.base = ch.base; f.stride = ch.stride; f.rec = rec;
    f.vin = v; f.aa = a; f.x = x; f.p = p;
    run_chain(f, ch.m);
}

__global__ void __launch_bounds__(kSweepThreads)
k_dr2_rows(Geo g, const float* __restrict__ z, const float* __restrict__ ax,
           const float* __restrict__ w, float* __restrict__ t, float* __restrict__ y1,
           float* __restrict__ p1, SegRec* __restrict__ rec)
{
    const int c = blockIdx.x * kSweepThreads + threadIdx.x;
    if (c >= geo_nchains(g, 0)) return;
    const Chain ch = chain_of(g, 0, c);
    Dr2RowF f;
    f.base = ch.base; f.stride = ch.stride; f.rec = rec;
    f.z = z; f.ax = ax; f.w = w; f.t = t; f.y1 = y1; f.p1 = p1;
    run_chain(f, ch.m);
}

__global__ void __launch_bounds__(kSweepThreads)
k_dr2_cols(Geo g, const float* __restrict__ t, const float* __restrict__ ay,
           const float* __restrict__ y1, float* __restrict__ z, float* __restrict__ p2,
           SegRec* __restrict__ rec)
{
    const int c = blockIdx.x * kSweepThreads + threadIdx.x;
    if (c >= geo_nchains(g, 1)) return;
    const Chain ch = chain_of(g, 1, c);
    Dr2ColF f;
    f.base = ch.base; f.stride = ch.stride; f.rec = rec;
    f.t = t; f.ay = ay; f.y1 = y1; f.z = z; f.p2 = p2;
    run_chain(f, ch.m);
}

struct SweepSet {
    const float* a[3];
};

// all non-final families of the product space in one launch: blocks
// [off[j], off[j+1]) handle family j
__global__ void __launch_bounds__(kSweepThreads)
k_drp_sweeps(Geo g, int nfam, int off1, int off2, const float* __restrict__ z, SweepSet as,
             float* __restrict__ y, float* __restrict__ p, SegRec* __restrict__ rec)
{
    int fam = 0, blk = blockIdx.x;
    if (nfam > 1 && blk >= off1) { fam = 1; blk -= off1; }
    if (nfam > 2 && fam == 1 && blk >= off2 - off1) { fam = 2; blk -= off2 - off1; }
    const int c = blk * kSweepThreads + threadIdx.x;
    if (c >= geo_nchains(g, fam)) return;
    const Chain ch = chain_of(g, fam, c);
    DrpSweepF f;
    f.base = ch.base; f.stride = ch.stride; f.rec = rec + (size_t)fam * g.n;
    f.zj = z + (size_t)fam * g.n;
    f.aj = as.a[fam];
    f.yj = y + (size_t)fam * g.n;
    f.pj_out = p ? p + (size_t)fam * g.n : nullptr;
    run_chain(f, ch.m);
}

template <int R>
__global__ void __launch_bounds__(kSweepThreads)
k_drp_final(Geo g, float* __restrict__ z, const float* __restrict__ y,
            const float* __restrict__ al, const float* __restrict__ w, float* __restrict__ pl,
            SegRec* __restrict__ rec)
{
    const int c = blockIdx.x * kSweepThreads + threadIdx.x;
    if (c >= geo_nchains(g, R - 1)) return;
    const Chain ch = chain_of(g, R - 1, c);
    DrpFinalF<R> f;
    f.base = ch.base; f.stride = ch.stride; f.rec = rec;
    f.z = z; f.y = y; f.al = al; f.w = w; f.pl = pl; f.n = g.n;
    run_chain(f, ch.m);
}

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
    for (int b = threadIdx.x; b < nblk; b += kReduceThreads) {
#pragma unroll
        for (int q = 0; q < NV; ++q) v[q] += partials[b * NV + q];
    }
    block_reduce_store<NV>(v, out);
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

// Primal estimate and lower bound from the edge duals (Sec. 2.2, 2.3):
// y = sum_j D_j^T p_j with p clipped to its box (so y lies in K exactly),
// x = -w - y (the TV primal x = w - y in the paper's sign), and
// LB(y) = sum_i min(y_i + w_i, 0).  Both are formed in FP64 from the FP32
// duals, which stay bounded by the weights, unlike the diverging state.
__global__ void __launch_bounds__(kReduceThreads)
k_primal(Geo g, const float* __restrict__ w, Ptr3 p, float* __restrict__ xc,
         double* __restrict__ partials)
{
    double lb = 0.0;
    const int stride = gridDim.x * kReduceThreads;
    const int st[3] = {1, g.W, g.W * g.H};
    for (int i = blockIdx.x * kReduceThreads + threadIdx.x; i < g.n; i += stride) {
        const Coords c = coords_of(g, i);
        const int cc[3] = {c.x, c.y, c.d};
        double y = 0.0;
        for (int j = 0; j < g.ndim; ++j) {
            y -= (double)p.p[j][i];  // zero on the last slice
            if (cc[j] > 0) y += (double)p.p[j][i - st[j]];
        }
        const double s = y + (double)w[i];
        if (s < 0.0) lb += s;
        xc[i] = (float)(-s);
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

__device__ __forceinline__ int ladder_count(float x, const Taus& tz)
{
    int c = 0;
#pragma unroll
    for (int t = 0; t < kNumTau; ++t) c += (x <= tz.t[t]) ? 1 : 0;
    return c;
}

__global__ void __launch_bounds__(kReduceThreads)
k_cut_ladder(Geo g, const float* __restrict__ xc, const float* __restrict__ w, Ptr3 a, Ptr3 p,
             Taus tz, double* __restrict__ partials)
{
    double e[kNumTau + 1];
#pragma unroll
    for (int t = 0; t <= kNumTau; ++t) e[t] = 0.0;
    const int stride = gridDim.x * kReduceThreads;
    const int st[3] = {1, g.W, g.W * g.H};
    for (int i = blockIdx.x * kReduceThreads + threadIdx.x; i < g.n; i += stride) {
        const Coords c = coords_of(g, i);
        const int cc[3] = {c.x, c.y, c.d};
        const int ext[3] = {g.W, g.H, g.D};
        const float xi = xc[i];
        const int ci = ladder_count(xi, tz);
        const double wi = (double)w[i];
#pragma unroll
        for (int t = 0; t < kNumTau; ++t)
            if (t >= ci) e[t] += wi;
        for (int j = 0; j < g.ndim; ++j) {
            if (cc[j] + 1 < ext[j]) {
                const float xn = xc[i + st[j]];
                const int cn = ladder_count(xn, tz);
                const double aj = (double)a.p[j][i];
                const int lo = ci < cn ? ci : cn, hi = ci < cn ? cn : ci;
#pragma unroll
                for (int t = 0; t < kNumTau; ++t)
                    if (t >= lo && t < hi) e[t] += aj;
                const double dx = (double)xn - (double)xi;
                e[kNumTau] += aj * fabs(dx) - (double)p.p[j][i] * dx;
            }
        }
    }
    block_reduce_store<kNumTau + 1>(e, partials + (size_t)blockIdx.x * (kNumTau + 1));
}

__global__ void __launch_bounds__(kReduceThreads)
k_energy(Geo g, const float* __restrict__ w, Ptr3 a, const uint8_t* __restrict__ lab,
         double* __restrict__ partials)
{
    double e = 0.0;
    const int stride = gridDim.x * kReduceThreads;
    const int st[3] = {1, g.W, g.W * g.H};
    for (int i = blockIdx.x * kReduceThreads + threadIdx.x; i < g.n; i += stride) {
        const Coords c = coords_of(g, i);
        const int cc[3] = {c.x, c.y, c.d};
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
    const int stride = gridDim.x * kReduceThreads;
    for (int i = blockIdx.x * kReduceThreads + threadIdx.x; i < g.n; i += stride) {
        const Coords c = coords_of(g, i);
        const int cc[3] = {c.x, c.y, c.d};
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

__global__ void __launch_bounds__(kReduceThreads)
k_labels(int n, const float* __restrict__ xc, float tau, uint8_t* __restrict__ lab)
{
    const int stride = gridDim.x * kReduceThreads;
    for (int i = blockIdx.x * kReduceThreads + threadIdx.x; i < n; i += stride)
        lab[i] = xc[i] > tau ? 1 : 0;
}

inline int sweep_blocks(int nchains) { return (nchains + kSweepThreads - 1) / kSweepThreads; }

inline int reduce_blocks(int n)
{
    int b = (n + kReduceThreads - 1) / kReduceThreads;
    return b < 1 ? 1 : (b > kReduceBlocks ? kReduceBlocks : b);
}

}  // namespace

// ---- launchers ----------------------------------------------------------------

hipError_t launch_prox(const Geo& g, int axis, const float* v, const float* a, float* x,
                       float* p, SegRec* rec, hipStream_t s)
{
    hipLaunchKernelGGL(k_prox, dim3(sweep_blocks(geo_nchains(g, axis))), dim3(kSweepThreads), 0, s,
                       g, axis, v, a, x, p, rec);
    return hipGetLastError();
}

hipError_t launch_dr2_rows(const Geo& g, const float* z, const float* a_x, const float* w,
                           float* t, float* y1, float* p1, SegRec* rec, hipStream_t s)
{
    hipLaunchKernelGGL(k_dr2_rows, dim3(sweep_blocks(geo_nchains(g, 0))), dim3(kSweepThreads), 0, s,
                       g, z, a_x, w, t, y1, p1, rec);
    return hipGetLastError();
}

hipError_t launch_dr2_cols(const Geo& g, const float* t, const float* a_y, const float* y1,
                           float* z, float* p2, SegRec* rec, hipStream_t s)
{
    hipLaunchKernelGGL(k_dr2_cols, dim3(sweep_blocks(geo_nchains(g, 1))), dim3(kSweepThreads), 0, s,
                       g, t, a_y, y1, z, p2, rec);
    return hipGetLastError();
}

hipError_t launch_drp_sweeps(const Geo& g, int nfam, const float* z, const float* const* a,
                             float* y, float* p, SegRec* rec, hipStream_t s)
{
    SweepSet as;
    for (int j = 0; j < 3; ++j) as.a[j] = j < nfam ? a[j] : nullptr;
    const int b0 = sweep_blocks(geo_nchains(g, 0));
    const int b1 = nfam > 1 ? sweep_blocks(geo_nchains(g, 1)) : 0;
    const int b2 = nfam > 2 ? sweep_blocks(geo_nchains(g, 2)) : 0;
    hipLaunchKernelGGL(k_drp_sweeps, dim3(b0 + b1 + b2), dim3(kSweepThreads), 0, s,
                       g, nfam, b0, b0 + b1, z, as, y, p, rec);
    return hipGetLastError();
}

hipError_t launch_drp_final(const Geo& g, int r, float* z, const float* y, const float* a_last,
                            const float* w, float* p_last, SegRec* rec, hipStream_t s)
{
    const dim3 grid(sweep_blocks(geo_nchains(g, r - 1)));
    if (r == 2)
        hipLaunchKernelGGL(k_drp_final<2>, grid, dim3(kSweepThreads), 0, s, g, z, y, a_last, w,
                           p_last, rec);
    else if (r == 3)
        hipLaunchKernelGGL(k_drp_final<3>, grid, dim3(kSweepThreads), 0, s, g, z, y, a_last, w,
                           p_last, rec);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

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
    const int nb = reduce_blocks(g.n);
    double* part_lb = partials;
    double* part_cut = partials + kReduceBlocks;
    hipLaunchKernelGGL(k_primal, dim3(nb), dim3(kReduceThreads), 0, s, g, w, pp, xc, part_lb);
    hipLaunchKernelGGL(k_cut_ladder, dim3(nb), dim3(kReduceThreads), 0, s, g, xc, w, pa, pp, tz,
                       part_cut);
    hipLaunchKernelGGL(k_finalize<kNumTau + 1>, dim3(1), dim3(kReduceThreads), 0, s, part_cut, nb,
                       out);
    hipLaunchKernelGGL(k_finalize<1>, dim3(1), dim3(kReduceThreads), 0, s, part_lb, nb,
                       out + kNumTau + 1);
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

hipError_t launch_count_nonfinite(const float* x, int n, double* partials, double* out,
                                  hipStream_t s)
{
    const int nb = reduce_blocks(n);
    hipLaunchKernelGGL(k_count_nonfinite, dim3(nb), dim3(kReduceThreads), 0, s, x, n, partials);
    hipLaunchKernelGGL(k_finalize<1>, dim3(1), dim3(kReduceThreads), 0, s, partials, nb, out);
    return hipGetLastError();
}

}  // namespace mc
