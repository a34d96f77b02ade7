// chain.hpp -- exact weighted 1D total-variation prox of chain pieces, run by
// one GPU lane each (Sec. 3.2 of the paper: the chain subproblem
//     x = argmin_x 1/2 |x - v|^2 + sum_e a_e |x_{e+1} - x_e| ).
//
// Direct scan.  A segment [k0, k] of constant value c is feasible while every
// edge dual inside it stays in its box: with P_e(c) = A + sum_{i=k0..e}
// (c - v_i) the dual of edge e (A the dual of the edge left of k0),
// |P_e(c)| <= a_e.  Each P_e increases with c, so the feasible values form an
// interval [vmin, vmax]; umin / umax hold the dual of the newest edge at
// c = vmin / vmax and kmin / kmax the last edge where the lower / upper bound
// was tight.  A new element k either tightens the interval or empties it: if
// even c = vmin pushes the dual above +a_k, the segment ends at kmin with a
// downward jump (dual -a there); symmetrically for vmax.  The scan restarts
// after the knot with that dual as its anchor.  The chain end is an edge of
// weight 0 (the taut string is pinned there).  This is the direct method of
// Condat with per-edge weights, i.e. the taut string of the paper's weighted
// solver seen through its dual offsets.  Every restart moves k0 forward, so a
// piece of L elements takes at most L(L+1)/2 steps.
//
// Segment values come from a running sum taken in FP64 relative to the first
// element, c = vref + (S' - A -+ a_knot) / L: accurate for large offsets,
// huge weights and long segments.  When edge duals are wanted the value is
// kept in FP64 and the fill carries p_j = p_{j-1} + c - v_j in FP64 from the
// segment's exact left anchor.
//
// Pieces of one chain in parallel.  Shortest paths through the tube from two
// different start heights to the same end never cross, and once they share a
// tube vertex they coincide.  A lane that starts inside a chain does not know
// the dual at its start, but the dual lies in [-a, +a]: it scans twice, from
// the lowest (L) and the highest (U) start.  The true string lies between the
// two, so the first knot both scans emit (same position, same side) is a knot
// of the true string, and everything after it is exact.  The lane starts an
// overlap W before its piece; if the two scans have not met before the piece
// begins, it moves the start further back (at the chain start the dual is 0
// and one scan suffices).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace mc {

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// num / den for a positive integer-valued den, to FP64 accuracy: hardware
// reciprocal refined by two Newton steps, then one residual correction.
__device__ __forceinline__ double div_by_len(double num, double den)
{
    double r = __builtin_amdgcn_rcp(den);
    r = __builtin_fma(__builtin_fma(-den, r, 1.0), r, r);
    r = __builtin_fma(__builtin_fma(-den, r, 1.0), r, r);
    const double q = num * r;
    return __builtin_fma(__builtin_fma(-den, q, num), r, q);
}

// dual clipped to its box and rounded to FP32 (|result| <= a exactly)
__device__ __forceinline__ float clip_dual(double p, float a)
{
    return fminf(fmaxf((float)p, -a), a);
}

// Segment values are FP64 when edge duals are wanted (the duals are carried
// from them), FP32 otherwise (only FP32 values are emitted).
template <bool kExact>
using SegVal = std::conditional_t<kExact, double, float>;

// A finished segment ending at kend, of value c, entered with dual A.
template <bool kExact>
struct Seg {
    SegVal<kExact> c;
    float A;
    int kend;
};

// State of one direct scan.
struct Scan {
    int k0, k;       // open segment start, next position to read
    float A;         // dual of the edge left of k0 (exactly +-a or 0)
    bool on;         // still scanning
    float vmin, vmax, umin, umax, len;
    int kmin, kmax;
    float amin, amax;  // weights of the edges kmin and kmax
    float vref;
    double s, smin, smax;
};

__device__ __forceinline__ void scan_start(Scan& s, int k0, float A, bool on)
{
    s.k0 = k0;
    s.k = k0;
    s.A = A;
    s.on = on;
    s.vmin = s.vmax = s.umin = s.umax = s.vref = s.amin = s.amax = 0.f;
    s.len = 1.f;
    s.kmin = s.kmax = k0;
    s.s = s.smin = s.smax = 0.0;
}

__device__ __forceinline__ void scan_open(Scan& s, float vk, float ak)
{
    s.vref = vk;
    const float v0 = vk - s.A;
    s.vmin = v0 - ak;
    s.vmax = v0 + ak;
    s.umin = -ak;
    s.umax = ak;
    s.kmin = s.kmax = s.k0;
    s.amin = s.amax = ak;
    s.s = s.smin = s.smax = 0.0;
    s.len = 1.f;
}

template <bool kExact>
__device__ __forceinline__ SegVal<kExact> seg_value(float vref, double num, int len)
{
    if constexpr (kExact)
        return (double)vref + div_by_len(num, (double)len);
    else
        return vref + (float)num * fast_rcp((float)len);
}

// One step at position s.k with vk = v(s.k), ak = weight of edge s.k (0 for
// the chain's last element m-1).  Returns true and fills `out` when a segment
// is finished.  kExact selects an FP64 segment value (needed for edge duals).
// Written with selects rather than branches: under SIMT every branch that any
// lane takes costs all lanes, and the state updates of the three cases (open,
// extend, knot) are cheap next to the exec-mask bookkeeping of branches.
template <bool kExact>
__device__ __forceinline__ bool scan_step(Scan& s, int m, float vk, float ak, Seg<kExact>& out)
{
    const bool opening = s.k == s.k0;
    const bool last = s.k == m - 1;
    const float pmin = s.umin + (s.vmin - vk);
    const float pmax = s.umax + (s.vmax - vk);
    const bool down = !opening && pmin > ak;  // even the smallest value overflows edge k
    const bool up = !opening && !down && pmax < -ak;  // even the largest underflows it
    const bool knot = down || up;
    const bool extend = !opening && !knot;

    // the segment finished by this step: [k0, kn] at a knot, [k0, m-1] at the
    // chain end (kn = m-1, dual 0 there)
    const int kn = down ? s.kmin : (up ? s.kmax : m - 1);
    const float an = down ? -s.amin : (up ? s.amax : 0.f);
    const double s_ext = s.s + ((double)vk - (double)s.vref);
    const double sn = down ? s.smin : (up ? s.smax : (opening ? 0.0 : s_ext));
    const float vr = opening ? vk : s.vref;
    out.c = seg_value<kExact>(vr, sn - (double)s.A + (double)an, kn - s.k0 + 1);
    out.A = s.A;
    out.kend = kn;
    const bool finished = knot || last;

    // after a knot at kn the next segment starts at kn + 1: at once if that is
    // the current element (and not the last), else by rescanning from there
    const bool reopen = knot && kn + 1 == s.k && !last;
    const bool rescan = knot && !reopen;
    const bool open_now = opening || reopen;
    const float A1 = knot ? an : s.A;
    const int k01 = knot ? kn + 1 : s.k0;

    const float len1 = s.len + 1.f;
    const float inv = fast_rcp(len1);
    const bool tl = extend && pmin <= -ak, tu = extend && pmax >= ak;
    const float v0 = vk - A1;
    s.vmin = open_now ? v0 - ak : (tl ? s.vmin + (-ak - pmin) * inv : s.vmin);
    s.vmax = open_now ? v0 + ak : (tu ? s.vmax - (pmax - ak) * inv : s.vmax);
    s.umin = open_now ? -ak : (tl ? -ak : pmin);
    s.umax = open_now ? ak : (tu ? ak : pmax);
    s.kmin = open_now ? s.k : (tl ? s.k : s.kmin);
    s.kmax = open_now ? s.k : (tu ? s.k : s.kmax);
    s.amin = open_now || tl ? ak : s.amin;
    s.amax = open_now || tu ? ak : s.amax;
    s.smin = open_now ? 0.0 : (tl ? s_ext : s.smin);
    s.smax = open_now ? 0.0 : (tu ? s_ext : s.smax);
    s.s = open_now ? 0.0 : (extend ? s_ext : s.s);
    s.len = open_now ? 1.f : (extend ? len1 : s.len);
    s.vref = open_now ? vk : s.vref;
    s.A = A1;
    s.k0 = k01;
    s.on = s.on && !(last && !rescan);
    s.k = rescan ? k01 : s.k + 1;
    // at the last element after a knot the one-element final segment is
    // finished by the next step (rescan from k01 = m - 1)
    return finished;
}

}  // namespace mc
