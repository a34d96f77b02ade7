// chain.hpp -- exact weighted 1D total-variation prox of one chain, run by one
// GPU lane (Sec. 3.2 of the paper: the chain subproblem
//     x = argmin_x 1/2 |x - v|^2 + sum_e a_e |x_{e+1} - x_e| ).
//
// Two passes over the chain.
//
// Scan (forward, direct method with restarts).  A segment [k0, k] of constant
// value c is feasible while every edge dual inside it stays in its box:
// with P_e(c) = A + sum_{i=k0..e} (c - v_i) the dual of edge e (A the dual of
// the edge left of k0), |P_e(c)| <= a_e.  Each P_e is increasing in c, so the
// feasible c form an interval [vmin, vmax]; umin / umax hold the dual of the
// newest edge at c = vmin / vmax and kmin / kmax the last edge where the lower
// / upper bound was tight.  A new element k either tightens the interval
// (one division by the segment length) or empties it: if even c = vmin
// pushes the dual above +a_k, the segment must end at kmin with value vmin and
// a downward jump (dual -a there); symmetrically for vmax.  The scan then
// restarts after the knot with that dual as the new anchor.  The chain end is
// an edge of weight 0 (the taut string is pinned there).  This is the direct
// method of Condat generalised to per-edge weights, equivalently the taut
// string of the paper's weighted solver seen through its dual offsets.  Every
// restart moves k0 forward, so the scan ends after at most m(m+1)/2 steps.
//
// Each finished segment leaves one record at its last position: the segment
// value and its first index, plus how the segment was entered (anchor code
// 0 = chain start, 1 = dual +a, 2 = dual -a).
//
// Fill (backward, one step per element in lock-step across lanes).  Walks
// j = m-1 .. 0, fetching a record whenever it enters a new segment, hands
// (j, c, p_j) to the caller's emitter (p_j = dual of edge (j, j+1)), and
// carries the dual leftwards by p_{j-1} = p_j - c + v_j inside a segment (in
// FP64), snapping to the exact anchor +-a at each knot.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mc {

struct alignas(16) SegRec {
    double val;     // segment value (FP64, see chain_scan)
    uint32_t info;  // first index (bits 0..29) | anchor code << 30
    uint32_t pad;
};

static_assert(sizeof(SegRec) == 16, "SegRec must be 16 bytes");

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// F provides: float v(int k); float a(int k) (edge k, k < m-1);
//             void put(int k, double val, uint32_t info); SegRec get(int k);
//             double emit(int j, double c, double pj, bool last) -> p_{j-1}.
template <class F>
__device__ __forceinline__ void chain_scan(const F& f, int m)
{
    int k0 = 0;
    float A = 0.f;
    uint32_t anc = 0u;
    while (k0 < m) {
        const float ak0 = (k0 + 1 < m) ? f.a(k0) : 0.f;
        // Values are emitted from an FP64 running sum taken relative to the
        // first element, c = vref + (S' - A -+ a_knot) / L.  It stays accurate
        // for large offsets (S' small), for huge weights (where the FP32
        // interval bounds lose the data's low bits) and over long segments;
        // the duals rebuilt from c in the fill then drift by FP64 rounding only.
        const float vref = f.v(k0);
        const double vref64 = (double)vref;
        const float v0 = vref - A;
        float vmin = v0 - ak0, vmax = v0 + ak0;
        float umin = -ak0, umax = ak0;
        int kmin = k0, kmax = k0;
        double s = 0.0, smin = 0.0, smax = 0.0;
        int next = m;  // m: the segment runs to the chain end
        float len = 1.f;
        for (int k = k0 + 1; k < m; ++k) {
            const float vk = f.v(k);
            const float ak = (k + 1 < m) ? f.a(k) : 0.f;
            const float pmin = umin + (vmin - vk);
            const float pmax = umax + (vmax - vk);
            if (pmin > ak) {
                // even the smallest feasible value overflows edge k: knot at kmin, jump down
                const float akn = f.a(kmin);
                const double c = vref64 + (smin - (double)A - (double)akn) / (double)(kmin - k0 + 1);
                f.put(kmin, c, (uint32_t)k0 | (anc << 30));
                A = -akn;
                anc = 2u;
                next = kmin + 1;
                break;
            }
            if (pmax < -ak) {
                // even the largest feasible value underflows edge k: knot at kmax, jump up
                const float akn = f.a(kmax);
                const double c = vref64 + (smax - (double)A + (double)akn) / (double)(kmax - k0 + 1);
                f.put(kmax, c, (uint32_t)k0 | (anc << 30));
                A = akn;
                anc = 1u;
                next = kmax + 1;
                break;
            }
            s += (double)vk - vref64;
            len += 1.f;
            const float inv = fast_rcp(len);
            if (pmin <= -ak) {
                vmin += (-ak - pmin) * inv;
                umin = -ak;
                kmin = k;
                smin = s;
            } else {
                umin = pmin;
            }
            if (pmax >= ak) {
                vmax -= (pmax - ak) * inv;
                umax = ak;
                kmax = k;
                smax = s;
            } else {
                umax = pmax;
            }
        }
        if (next == m) f.put(m - 1, vref64 + (s - (double)A) / (double)(m - k0), (uint32_t)k0 | (anc << 30));
        k0 = next;
    }
}

template <class F>
__device__ __forceinline__ void chain_fill(F& f, int m)
{
    double c = 0.0;
    int seg0 = m;
    uint32_t anc_right = 0u;
    double pj = 0.0;
    for (int j = m - 1; j >= 0; --j) {
        if (j < seg0) {
            if (j < m - 1) {
                const double aj = (double)f.a(j);
                pj = anc_right == 1u ? aj : (anc_right == 2u ? -aj : 0.0);
            } else {
                pj = 0.0;
            }
            const SegRec r = f.get(j);
            c = r.val;
            seg0 = (int)(r.info & 0x3fffffffu);
            anc_right = r.info >> 30;
        }
        pj = f.emit(j, c, pj, j == m - 1);
    }
}

// dual clipped to its box and rounded to FP32 (|result| <= a exactly)
__device__ __forceinline__ float clip_dual(double p, float a)
{
    return fminf(fmaxf((float)p, -a), a);
}

}  // namespace mc
