// piece.hpp -- one lane's share of a chain sweep: the chain prox restricted to
// the piece [b0, b1) of one chain (see chain.hpp for the scan and for why a
// piece that starts inside a chain can be solved exactly on its own).
//
// The lane brackets the unknown dual at its start with two scans L (start dual
// -a) and U (start dual +a) from p0 = b0 - W.  Each scan only advances while
// its last knot is not ahead of the other's, so the first knot they share is
// seen when the second of them emits it.  A shared knot K < b0 makes
// everything from K+1 on exact: U is dropped and L continues alone.  If the
// scans pass b0 without sharing a knot, the lane restarts with a four times
// longer overlap; from the chain start (dual 0) one scan is exact at once.
//
// Finished segments go to a two-entry queue; a fill trails the scan and
// writes the outputs of positions in [b0, b1) (the dual of each edge is carried
// in FP64 from the segment's exact left anchor when kExact).  The scan stops
// once the segment covering b1 - 1 is finished.
//
// The caller reads the values of the positions the three steps work on --
// fill_pos(), l_pos(), u_pos() -- before the steps (all three reads can then
// be in flight together): RingVals r[0] is the scan input, r[1] the weight of
// the edge to the next position.  The fill only writes positions the scans
// have finished with, so its writes never touch a value read for L or U.
// Emit(q, c, p, last, on) records the result of position q when `on`: segment
// value c and dual p of edge (q, q+1) (meaningful when kExact and not last);
// it is called on every fill step and must discard the write when !on.
#pragma once

#include "chain.hpp"

namespace mc {

template <int NR>
struct RingVals {
    float r[NR];
};

template <int NR, bool kExact>
struct PieceLane {
    int m, b0, b1, W;
    bool bracket;    // L and U both running
    bool scanning;   // the piece is not determined yet
    Scan L, U;
    int lastL, lastU;  // position of the last knot of each scan (-1: none)
    float ancL, ancU;  // dual of the edge at that knot
    // fill
    int fj, fend;  // next position to write, end of the segment being written
    using V = SegVal<kExact>;
    V fc, fp;                // its value, dual of the edge left of fj
    Seg<kExact> q0, q1;      // queued finished segments
    int qn;

    // (Re)start the scans from p0 = max(0, b0 - W); a_before(q) is the weight
    // of edge q (only read when p0 > 0).
    template <class AAt>
    __device__ __forceinline__ void restart(const AAt& a_before)
    {
        const int p0 = b0 - W > 0 ? b0 - W : 0;
        qn = 0;
        fend = -1;
        fc = V(0);
        fp = V(0);
        lastL = lastU = -1;
        ancL = ancU = 0.f;
        if (p0 == 0) {
            bracket = false;
            scan_start(L, 0, 0.f, true);
            scan_start(U, 0, 0.f, false);
            fj = 0;
        } else {
            const float ab = a_before(p0 - 1);
            bracket = true;
            scan_start(L, p0, -ab, true);
            scan_start(U, p0, ab, true);
            fj = m;  // no fill before the scans merge
        }
    }

    template <class AAt>
    __device__ __forceinline__ void begin(bool active, int m_, int b0_, int b1_, int W0,
                                          const AAt& a_before)
    {
        m = m_;
        b0 = b0_;
        b1 = b1_;
        W = W0;
        scanning = active;
        restart(a_before);
        if (!active) {
            L.on = U.on = false;
            fj = m;
        }
    }

    __device__ __forceinline__ bool fill_ready() const { return fj < b1 && (fend >= fj || qn > 0); }
    __device__ __forceinline__ bool busy() const { return scanning || fill_ready(); }

    // positions whose values the next fill / step_l / step_u read (`idle`
    // when the step will not read)
    __device__ __forceinline__ int fill_pos(int idle) const { return fill_ready() ? fj : idle; }
    __device__ __forceinline__ int l_pos(int idle) const { return scanning && L.k < m ? L.k : idle; }
    __device__ __forceinline__ int u_pos(int idle) const { return scanning && bracket && U.k < m ? U.k : idle; }

    __device__ __forceinline__ void push(bool on, const Seg<kExact>& s)
    {
        const bool to0 = on && qn == 0, to1 = on && qn == 1;
        q0.c = to0 ? s.c : q0.c;
        q0.A = to0 ? s.A : q0.A;
        q0.kend = to0 ? s.kend : q0.kend;
        q1.c = to1 ? s.c : q1.c;
        q1.A = to1 ? s.A : q1.A;
        q1.kend = to1 ? s.kend : q1.kend;
        qn += on ? 1 : 0;
    }

    // One iteration is fill(), step_l(), then -- only while some lane of the
    // wave brackets -- step_u() and resolve().  Keeping the scans in separate
    // calls lets a wave skip U once all its lanes have merged.

    // write one position of the finished segments; rv = values at fill_pos()
    template <class Emit>
    __device__ __forceinline__ void fill(const RingVals<NR>& rv, const Emit& emit)
    {
        // branch-free, so that its instructions can fill the stalls of the
        // scan's dependency chain; Emit gets whether the write is real
        const bool go = fill_ready();
        const bool pop = go && fend < fj;
        fc = pop ? q0.c : fc;
        fp = pop ? (V)q0.A : fp;
        fend = pop ? q0.kend : fend;
        q0.c = pop ? q1.c : q0.c;
        q0.A = pop ? q1.A : q0.A;
        q0.kend = pop ? q1.kend : q0.kend;
        qn -= pop ? 1 : 0;
        const V pr = kExact ? fp + (fc - (V)rv.r[0]) : V(0);
        emit(fj, fc, pr, fj == m - 1, go && fj >= b0);
        fp = go ? pr : fp;
        fj += go ? 1 : 0;
    }

    // advance L (the only scan once the bracket is resolved); rv = values at l_pos()
    __device__ __forceinline__ void step_l(const RingVals<NR>& rv)
    {
        if (!scanning || qn == 2 || (bracket && lastL > lastU)) return;
        const int k = L.k;
        Seg<kExact> sg;
        const bool fin = scan_step<kExact>(L, m, rv.r[0], k + 1 < m ? rv.r[1] : 0.f, sg);
        const bool br = bracket;
        lastL = fin && br ? sg.kend : lastL;
        ancL = fin && br ? L.A : ancL;
        push(fin && !br, sg);
        scanning = scanning && !(fin && !br && sg.kend >= b1 - 1);
    }

    __device__ __forceinline__ bool needs_u() const { return scanning && bracket && lastU <= lastL; }


    // advance U when go (= needs_u() before step_l ran: deciding after L's
    // step would let U pass a knot that L has just reached, so the shared
    // knot would be missed and the lane restart); rv = values at u_pos()
    __device__ __forceinline__ void step_u(bool go, const RingVals<NR>& rv)
    {
        if (!go) return;
        const int k = U.k;
        Seg<false> sg;
        const bool fin = scan_step<false>(U, m, rv.r[0], k + 1 < m ? rv.r[1] : 0.f, sg);
        lastU = fin ? sg.kend : lastU;
        ancU = fin ? U.A : ancU;
    }

    // after both scans stepped: merged, failed, or keep going
    template <class AAt>
    __device__ __forceinline__ void resolve(const AAt& a_before)
    {
        if (!scanning || !bracket) return;
        if (lastL == lastU && lastL >= 0 && ancL == ancU && lastL < b0 && L.on) {
            // merged at a knot before the piece: L is exact from here
            bracket = false;
            U.on = false;
            fj = lastL + 1;
            fend = lastL;
        } else if ((lastL >= b0 - 1 && lastU >= b0 - 1) || !L.on || !U.on) {
            // no shared knot before the piece: start further back
            W *= 4;
            restart(a_before);
        }
    }
};

}  // namespace mc
