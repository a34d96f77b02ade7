// fp64.hip -- the splitting with its state in FP64 (MC_FP64_STATE, a debug
// option of mc_tv_solve): the same iteration as the FP32 path -- two-set form
// in 2D, product space (Sec. 3.3, eq. (dualA)) -- with every chain prox,
// state update and averaging step in FP64, so that a solve can be checked
// against rounding in the FP32 state.  Speed does not matter here: one lane
// scans one whole chain from global memory.
//
// Chain prox (Sec. 3.2).  The direct scan of the weighted 1D-TV prox: the open
// segment [k0, k] is entered with dual A = -nA (the dual of edge k0 - 1); the
// dual of edge e inside it, P_e(c) = A + sum_{i=k0..e} (c - v_i), stays in
// [-a_e, a_e] for c in [lo_e, hi_e] = vref + (S'_e + nA -+ a_e) / (e - k0 + 1)
// with S'_e the sum of v_i - vref.  The feasible values of the segment are
// [vmin, vmax] (max of the lo, min of the hi); when a new position empties
// the interval the segment ends at the last position where the violated
// bound was attained, with that bound as its value and the knot's dual +-a
// there, and the scan starts the next segment after the knot.  The chain end
// is an edge of weight 0.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch.hpp"

namespace mc {

namespace {

constexpr int kLanes64 = 64;

struct Line {
    int base, stride;
};

__device__ __forceinline__ Line line_of(const Geo& g, int axis, int c)
{
    if (axis == 0) return {c * g.W, 1};                                       // c = d*H + h
    if (axis == 1) return {(c / g.W) * g.H * g.W + c % g.W, g.W};             // c = d*W + x
    return {c, g.H * g.W};                                                    // c = h*W + x
}

// One whole chain of length m.  v(k), a(k): scan input and weight of edge k
// at position k; seg(k0, kend, c, A, pend) receives each finished segment:
// positions k0..kend take the value c, the dual in front of k0 is A and the
// dual at kend is pend (exact: +-a at a knot, 0 at the chain end).
template <class V, class Wt, class Seg>
__device__ void prox64_chain(int m, const V& v, const Wt& a, const Seg& seg)
{
    const double inf = __builtin_huge_val();
    int k0 = 0, k = 0;
    double nA = 0.0, vref = 0.0, S = 0.0;
    double vmin = -inf, vmax = inf, amin = 0.0, amax = 0.0;
    int kmin = 0, kmax = 0;
    for (;;) {
        const double vk = v(k);
        const double ak = k + 1 < m ? a(k) : 0.0;
        if (k == k0) {
            vref = vk;
            S = 0.0;
        }
        const double s1 = S + (vk - vref);
        const double len = (double)(k - k0 + 1);
        const double lo = (s1 + (nA - ak)) / len, hi = (s1 + (nA + ak)) / len;
        if (vmin > hi || vmax < lo) {
            const bool down = vmin > hi;
            const int kend = down ? kmin : kmax;
            const double pend = down ? -amin : amax;
            seg(k0, kend, vref + (down ? vmin : vmax), -nA, pend);
            nA = -pend;
            k0 = k = kend + 1;
            vmin = -inf;
            vmax = inf;
            continue;
        }
        if (lo >= vmin) {
            vmin = lo;
            kmin = k;
            amin = ak;
        }
        if (hi <= vmax) {
            vmax = hi;
            kmax = k;
            amax = ak;
        }
        S = s1;
        if (k == m - 1) {
            seg(k0, m - 1, vref + lo, -nA, 0.0);
            return;
        }
        ++k;
    }
}

// modes: scan input at voxel i, and what a finished position i writes
struct Rows64 {  // two-set rows: q1 = prox(z)
    const double* z;
    double* q1;
    __device__ double v(int i) const { return z[i]; }
    __device__ void out(int i, double c) const { q1[i] = c; }
};
struct Cols64 {  // two-set columns: t = q1 - (z - q1) - w, z' = (z - q1) + prox(t)
    const double* q1;
    const double* z;
    const float* w;
    double* znew;
    __device__ double v(int i) const { return q1[i] - (z[i] - q1[i]) - (double)w[i]; }
    __device__ void out(int i, double c) const { znew[i] = (z[i] - q1[i]) + c; }
};
struct Fam64 {  // product space family j: q_j = prox(z_j)
    const double* z;
    double* q;
    __device__ double v(int i) const { return z[i]; }
    __device__ void out(int i, double c) const { q[i] = c; }
};

// one lane per chain along `axis`; p (nullable) gets the FP32 duals clipped to
// their boxes (0 on the last position)
template <class M>
__global__ void __launch_bounds__(kLanes64) k_prox64(Geo g, int axis, M mode, const float* __restrict__ a,
                                                      float* __restrict__ p)
{
    const int m = geo_extent(g, axis);
    const int c = blockIdx.x * kLanes64 + threadIdx.x;
    if (c >= geo_nchains(g, axis)) return;
    const Line ln = line_of(g, axis, c);
    auto vk = [&](int k) { return mode.v(ln.base + k * ln.stride); };
    auto ak = [&](int k) { return (double)a[ln.base + k * ln.stride]; };
    auto seg = [&](int k0, int kend, double cv, double A, double pend) {
        double P = A;
        for (int e = k0; e <= kend; ++e) {
            const int i = ln.base + e * ln.stride;
            P += cv - mode.v(i);
            mode.out(i, cv);
            if (p) {
                const float ae = a[i];
                const double pe = e == kend ? pend : P;
                p[i] = e == m - 1 ? 0.f : fminf(fmaxf((float)pe, -ae), ae);
            }
        }
    };
    prox64_chain(m, vk, ak, seg);
}

// z_j' = y_j - (2 Y - Z + w) / R, y_j = z_j - q_j (the averaging step)
template <int R>
__global__ void k_combine64(size_t n, const double* __restrict__ z, const double* __restrict__ q,
                            const float* __restrict__ w, double* __restrict__ zn)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        double y[R], Y = 0.0, Z = 0.0;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            y[j] = z[j * n + i] - q[j * n + i];
            Y += y[j];
            Z += z[j * n + i];
        }
        const double corr = (2.0 * Y - Z + (double)w[i]) / (double)R;
#pragma unroll
        for (int j = 0; j < R; ++j) zn[j * n + i] = y[j] - corr;
    }
}

__global__ void k_f32_to_f64(size_t n, const float* __restrict__ x, double* __restrict__ y)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        y[i] = (double)x[i];
}

__global__ void k_f64_to_f32(size_t n, const double* __restrict__ x, float* __restrict__ y)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        y[i] = (float)x[i];
}

inline dim3 grid_for(size_t n)
{
    const size_t b = (n + 255) / 256;
    return dim3((unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096));
}

template <class M>
hipError_t launch_prox64(const Geo& g, int axis, const M& mode, const float* a, float* p, hipStream_t s)
{
    const int nch = geo_nchains(g, axis);
    hipLaunchKernelGGL((k_prox64<M>), dim3((nch + kLanes64 - 1) / kLanes64), dim3(kLanes64), 0, s, g, axis, mode,
                       a, p);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_dr2_rows64(const Geo& g, const double* z, const float* a_x, double* q1, float* p1, hipStream_t s)
{
    return launch_prox64(g, 0, Rows64{z, q1}, a_x, p1, s);
}

hipError_t launch_dr2_cols64(const Geo& g, const double* q1, const double* z, double* znew, const float* w,
                             const float* a_y, float* p2, hipStream_t s)
{
    return launch_prox64(g, 1, Cols64{q1, z, w, znew}, a_y, p2, s);
}

hipError_t launch_family64(const Geo& g, int axis, const double* z, const float* a, double* q, float* p,
                           hipStream_t s)
{
    return launch_prox64(g, axis, Fam64{z, q}, a, p, s);
}

hipError_t launch_combine64(size_t n, int r, const double* z, const double* q, const float* w, double* zn,
                            hipStream_t s)
{
    if (r == 2) hipLaunchKernelGGL(k_combine64<2>, grid_for(n), dim3(256), 0, s, n, z, q, w, zn);
    else if (r == 3) hipLaunchKernelGGL(k_combine64<3>, grid_for(n), dim3(256), 0, s, n, z, q, w, zn);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_f32_to_f64(size_t n, const float* x, double* y, hipStream_t s)
{
    hipLaunchKernelGGL(k_f32_to_f64, grid_for(n), dim3(256), 0, s, n, x, y);
    return hipGetLastError();
}

hipError_t launch_f64_to_f32(size_t n, const double* x, float* y, hipStream_t s)
{
    hipLaunchKernelGGL(k_f64_to_f32, grid_for(n), dim3(256), 0, s, n, x, y);
    return hipGetLastError();
}

}  // namespace mc
