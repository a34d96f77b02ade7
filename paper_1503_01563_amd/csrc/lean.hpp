// lean.hpp -- the chain prox scan of the sweeps that only need prox values
// (every splitting iteration that does not evaluate the certificate), in
// FP32, with the per-step work cut to the funnel test (Sec. 3.2 of the paper:
// exact weighted 1D-TV prox of each chain).
//
// Slope form of the direct scan.  The open segment [k0, k] (value c) is
// entered with dual A (edge k0 - 1).  The dual of edge e inside it is
// P_e(c) = A + sum_{i=k0..e} (c - v_i), so |P_e(c)| <= a_e holds for
//     c >= lo_e = vref + (S'_e - A - a_e) / (e - k0 + 1)   and
//     c <= hi_e = vref + (S'_e - A + a_e) / (e - k0 + 1),
// S'_e = sum_{i=k0..e} (v_i - vref), vref = v_k0.  The feasible values of the
// open segment are [vmin, vmax] = [max lo_e, min hi_e]; kmin / kmax are the
// last positions where the bounds were attained and amin / amax the weights
// there.  A new element k with vmin > hi_k ends the segment at kmin with the
// value vmin and a downward jump (dual -a_kmin); vmax < lo_k ends it at kmax
// with vmax (dual +a_kmax); the scan then restarts after the knot.  The chain
// end is an edge of weight 0 (the taut string is pinned there), where
// lo = hi is the value of the last segment.  This is the same funnel as the
// taut string and as Condat's direct algorithm, evaluated from the running
// sum at every step instead of by increments, so no rounding accumulates in
// the bounds beyond the running sum itself.
//
// Precision.  Every bound is formed as (S' + (nA -+ a)) / len relative to
// vref, with nA = -A: the two weights are combined first, so large weights
// that cancel (a knot dual of a segment against the next edge) cancel
// exactly, and the bounds are compared as offsets from a reference value of
// the segment itself (data far from 0 keep the precision of their spread).
// The reciprocal of len is the hardware one (1 ulp).
//
// Knots of the scan that finishes a piece go to LDS.  Value sweeps store the
// segment value at the knot's slot and a negative weight as its mark (weights
// are >= 0, staged as a + 0 so that a -0 weight does not look like a mark);
// after the scan a backward pass over the piece gives every position the
// value of the next mark at or after it; the segment covering the piece's last
// position comes from registers.  Sweeps that also write edge duals keep the
// scan's running sums in FP64 as well, store each knot's FP64 segment value
// (as a pair of floats) and mark the knot in a bit mask with its side; their
// backward pass carries the duals from each knot's exact dual +-a (Sec. 3.2:
// the dual of edge e inside a segment is P_e = P_{e+1} - (c - v_{e+1})).
#pragma once

#include <hip/hip_runtime.h>

namespace mc {

#if defined(__HIP_DEVICE_COMPILE__)
__device__ __forceinline__ float lean_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
// num / den for a positive integer-valued den, to FP64 accuracy: hardware
// reciprocal refined by two Newton steps, then one residual correction
__device__ __forceinline__ double lean_div(double num, double den)
{
    double r = __builtin_amdgcn_rcp(den);
    r = __builtin_fma(__builtin_fma(-den, r, 1.0), r, r);
    r = __builtin_fma(__builtin_fma(-den, r, 1.0), r, r);
    const double q = num * r;
    return __builtin_fma(__builtin_fma(-den, q, num), r, q);
}
#else
__host__ __device__ inline float lean_rcp(float x) { return 1.f / x; }
__host__ __device__ inline double lean_div(double num, double den) { return num / den; }
#endif

// State of one scan (FP32).  len = elements in the open segment (0: the next
// step opens one at k).  The bounds vmin / vmax are kept relative to vref, so
// that they are compared to the precision of the offsets, not of vref.
struct LeanScan {
    int k;
    bool on;
    float nA;  // minus the dual of the edge in front of the open segment
    float vref, s, len;
    float vmin, vmax, amin, amax;  // vmin, vmax: minus vref
    int kmin, kmax;
};

// FP64 part of a scan whose segment values must be exact to FP64 (the sweeps
// that also write edge duals: the duals are carried from the segment values,
// and the certificate needs them to the FP32 rounding of the exact value).
// Running sums of v - vref over the open segment, and at kmin / kmax.
struct LeanExact {
    double s, smin, smax;
};

// What an exact step reports about the segment it finished.
struct LeanSeg {
    double c;     // segment value, FP64: vref + (S' + nA + an) / len
    float nA;     // minus the dual in front of the segment
    float vref;   // its reference value
    float an;     // dual of the edge at its end (the knot dual; 0 at the chain end)
};

__host__ __device__ inline void lean_start(LeanScan& S, int k0, float A, bool on)
{
    S.k = k0;
    S.on = on;
    S.nA = -A;
    S.vref = 0.f;
    S.s = 0.f;
    S.len = 0.f;
    S.vmin = -__builtin_huge_valf();
    S.vmax = __builtin_huge_valf();
    S.amin = S.amax = 0.f;
    S.kmin = S.kmax = k0;
}

// One step at position S.k: vk = v(k), ak = weight of edge k (0 for the
// chain's last element m - 1).  Returns true when a segment is finished: it
// ends at kend with value c.  After a knot the scan continues at kend + 1
// with S.nA the negated knot dual; after the chain's last segment S.on is
// false.
template <bool kExact>
__host__ __device__ inline bool lean_step_t(LeanScan& S, LeanExact& X, int m, float vk, float ak, int& kend,
                                            float& c, LeanSeg& sg)
{
    const bool opening = S.len == 0.f;
    const float vr = opening ? vk : S.vref;
    const float s1 = S.s + (vk - vr);
    const float len1 = S.len + 1.f;
    const float inv = lean_rcp(len1);
    const float lo = (s1 + (S.nA - ak)) * inv;  // bounds relative to vr
    const float hi = (s1 + (S.nA + ak)) * inv;
    const bool down = S.vmin > hi;  // even the smallest value overflows edge k
    const bool up = S.vmax < lo;    // even the largest underflows it
    const bool knot = down | up;
    const bool tl = lo >= S.vmin, tu = hi <= S.vmax;
    const bool last = S.k == m - 1;

    // the finished segment: at a knot the old bound, at the chain end the
    // common value of both bounds
    kend = down ? S.kmin : (up ? S.kmax : m - 1);
    c = vr + (down ? S.vmin : (up ? S.vmax : lo));
    const float nA_knot = down ? S.amin : -S.amax;
    double s1x = 0.0;
    if constexpr (kExact) {
        // FP64 running sum (v - vref is exact in FP64) and the finished
        // segment's value to FP64: length kend - k0 + 1 at a knot, len1 at
        // the chain end; k0 = k - len
        s1x = X.s + ((double)vk - (double)vr);
        const double sn = down ? X.smin : (up ? X.smax : s1x);
        const float an = knot ? -nA_knot : 0.f;
        const float ln = knot ? (float)(kend - S.k) + S.len + 1.f : len1;
        sg.c = (double)vr + lean_div(sn + ((double)S.nA + (double)an), (double)ln);
        sg.nA = S.nA;
        sg.vref = vr;
        sg.an = an;
    }

    // After a knot at k - 1 the next segment starts at k itself: open it with
    // this element at once (its bounds are the one-element ones, from the
    // knot's dual).  After a knot further back the scan resumes at kend + 1
    // (the next step opens there); at the chain's last element a knot always
    // resumes, so that the last one-element segment is finished by a step.
    const float nA_next = knot ? nA_knot : S.nA;
    const bool reopen = knot & (kend + 1 == S.k) & !last;
    const bool rescan = knot & !reopen;
    const float lo1 = nA_next - ak, hi1 = nA_next + ak;  // relative to vk
    S.kmin = reopen | tl ? S.k : S.kmin;
    S.amin = reopen | tl ? ak : S.amin;
    S.kmax = reopen | tu ? S.k : S.kmax;
    S.amax = reopen | tu ? ak : S.amax;
    S.vref = reopen ? vk : vr;
    const float inf = __builtin_huge_valf();
    S.vmin = reopen ? lo1 : (rescan ? -inf : (tl ? lo : S.vmin));
    S.vmax = reopen ? hi1 : (rescan ? inf : (tu ? hi : S.vmax));
    S.s = knot ? 0.f : s1;
    S.len = reopen ? 1.f : (rescan ? 0.f : len1);
    if constexpr (kExact) {
        X.smin = reopen ? 0.0 : (tl ? s1x : X.smin);
        X.smax = reopen ? 0.0 : (tu ? s1x : X.smax);
        X.s = knot ? 0.0 : s1x;
    }
    S.nA = nA_next;
    S.k = rescan ? kend + 1 : S.k + 1;
    S.on = S.on & (knot | !last);
    return knot | last;
}

__host__ __device__ inline bool lean_step(LeanScan& S, int m, float vk, float ak, int& kend, float& c)
{
    LeanExact X;
    LeanSeg sg;
    return lean_step_t<false>(S, X, m, vk, ak, kend, c, sg);
}

// One lane's piece [b0, b1) of a chain of length m.  Two scans bracket the
// unknown dual at the start p0 = b0 - W (start duals -a and +a, see
// chain.hpp); each only advances while its last knot is not ahead of the
// other's, and the first knot both emit (same position, same side) is a knot
// of the true solution.  If that knot lies before b0, U stops and L goes on
// alone, exact from there; otherwise the lane restarts with a twice longer
// overlap (from the chain start the dual is 0 and L alone is exact).
template <bool kExact>
struct LeanLaneT {
    int m, b0, b1, W;
    bool bracket;   // L and U both running
    bool scanning;  // the segment covering b1 - 1 is not finished yet
    LeanScan L, U;
    LeanExact X;         // L's FP64 sums (exact sweeps)
    int lastL, lastU;    // position of each scan's last knot (-1: none)
    float ancL, ancU;    // its negated dual
    float c_last;        // value of the segment covering b1 - 1
    // exact sweeps: knots inside the piece (bit q - b0 of kmask; umask: the
    // knot dual is +a), the covering segment's FP64 value and the dual of
    // edge b1 - 1, and L's running sum and length at b1 - 1
    unsigned long long kmask, umask;
    double c_last64, p_b1, s_b1;
    float l_b1;

    template <class AAt>
    __host__ __device__ inline void restart(const AAt& a_before)
    {
        const int p0 = b0 - W > 0 ? b0 - W : 0;
        lastL = lastU = -1;
        ancL = ancU = 0.f;
        X.s = X.smin = X.smax = 0.0;
        if (p0 == 0) {
            bracket = false;
            lean_start(L, 0, 0.f, true);
            lean_start(U, 0, 0.f, false);
        } else {
            const float ab = a_before(p0 - 1);
            bracket = true;
            lean_start(L, p0, -ab, true);
            lean_start(U, p0, ab, true);
        }
    }

    template <class AAt>
    __host__ __device__ inline void begin(bool active, int m_, int b0_, int b1_, int W0, const AAt& a_before)
    {
        m = m_;
        b0 = b0_;
        b1 = b1_;
        W = W0;
        scanning = active;
        c_last = 0.f;
        kmask = umask = 0ull;
        c_last64 = p_b1 = s_b1 = 0.0;
        l_b1 = 0.f;
        restart(a_before);
        if (!active) L.on = U.on = false;
    }

    // Whether each scan takes a step this iteration: both decided from the
    // knots at the start of the iteration (a scan whose last knot is ahead of
    // the other's waits; deciding before either steps only makes a scan wait
    // one iteration longer, and keeps the two steps independent of each other).
    __host__ __device__ inline bool steps_l() const { return scanning && !(bracket && lastL > lastU); }
    __host__ __device__ inline bool needs_u() const { return scanning && bracket && lastU <= lastL; }

    // L's step and what follows from it; br: the lane still brackets.
    // mark(kend, c, seg, on, k0, out) records a knot inside the piece (on:
    // kend in [b0, b1 - 1), once the bracket is resolved); out: a segment
    // [k0, kend] of the result was finished (the streamed sweeps write every
    // such segment).
    template <class Mark>
    __host__ __device__ inline void advance_l(bool br, float vk, float ak, const Mark& mark)
    {
        const int kp = L.k;
        const int k0 = kp - (int)L.len;  // start of the open segment
        int kend;
        float c;
        LeanSeg sg;
        const bool fin = lean_step_t<kExact>(L, X, m, vk, ak, kend, c, sg);
        if constexpr (kExact) {
            // the running sum at b1 - 1 of the segment that covers it (the
            // last pass over b1 - 1 that kept the element is that segment's)
            const bool rec = (kp == b1 - 1) & (L.k == kp + 1);
            s_b1 = rec ? X.s : s_b1;
            l_b1 = rec ? L.len : l_b1;
        }
        lastL = fin & br ? kend : lastL;
        ancL = fin & br ? L.nA : ancL;
        const bool out = fin & !br;
        const bool inside = out & (kend >= b0) & (kend < b1 - 1);
        mark(kend, c, sg, inside, k0, out);
        if constexpr (kExact) {
            const unsigned long long bit = inside & (kend - b0 < 64) ? 1ull << (kend - b0) : 0ull;
            kmask |= bit;
            umask |= sg.an > 0.f ? bit : 0ull;
        }
        const bool covers = out & (kend >= b1 - 1);
        c_last = covers ? c : c_last;
        if constexpr (kExact) {
            // dual of edge b1 - 1: the knot's own when the segment ends
            // there, else carried from the segment's left dual in FP64
            const double pc = kend == b1 - 1 ? (double)sg.an
                                             : -(double)sg.nA + (double)l_b1 * (sg.c - (double)sg.vref) - s_b1;
            c_last64 = covers ? sg.c : c_last64;
            p_b1 = covers ? pc : p_b1;
        }
        scanning = scanning & !covers;
    }

    // Advance L when go (= steps_l() at the start of the iteration); vk, ak at L.k.
    template <class Mark>
    __host__ __device__ inline void step_l(bool go, float vk, float ak, const Mark& mark)
    {
        if (!go) return;
        advance_l(bracket, vk, ak, mark);
    }

    // Advance L once no lane brackets any more (every lane is exact from its
    // merge knot or from the chain start); vk, ak at L.k.
    template <class Mark>
    __host__ __device__ inline void step_plain(float vk, float ak, const Mark& mark)
    {
        advance_l(false, vk, ak, mark);
    }

    // advance U when go (= needs_u() at the start of the iteration); vk, ak at U.k
    __host__ __device__ inline void step_u(bool go, float vk, float ak)
    {
        if (!go) return;
        int kend;
        float c;
        const bool fin = lean_step(U, m, vk, ak, kend, c);
        lastU = fin ? kend : lastU;
        ancU = fin ? U.nA : ancU;
    }

    // after both scans stepped: merged, failed, or keep going
    template <class AAt>
    __host__ __device__ inline void resolve(const AAt& a_before)
    {
        if (!scanning || !bracket) return;
        if (lastL == lastU && lastL >= 0 && ancL == ancU && lastL < b0 && L.on) {
            bracket = false;  // merged at a knot before the piece: L is exact from here
            U.on = false;
        } else if ((lastL >= b0 - 1 && lastU >= b0 - 1) || !L.on || !U.on) {
            W *= 2;  // no shared knot before the piece: start further back
            restart(a_before);
        }
    }
};

using LeanLane = LeanLaneT<false>;

}  // namespace mc
