// sweeps.hip -- chain-prox sweeps (Sec. 3.2) and the splitting steps built on
// them (Sec. 3.3, 4.3), for gfx950.
//
// Work item = one wave64 = 64 chains of one family x one piece [b0, b1) of
// those chains (see piece.hpp).  Cutting chains into pieces multiplies the
// lanes available to a sweep (a 1024 x 1024 grid has only 1024 chains per
// family, 16 waves for a 256-CU GPU) at the price of an overlap W scanned
// twice in front of each piece.
//
// A work item runs in three phases, with global memory touched only in the
// first and the last:
//   load    the window [b0 - W - 1, b1 + T) of the 64 chains goes to LDS with
//           coalesced loads (chains along W are loaded transposed: lanes walk
//           (row, position) pairs, consecutive lanes on consecutive
//           positions); per position the scan input v (formed on the fly by
//           the mode, e.g. 2 q1 - z - w) and the weight a of the edge to the
//           next position;
//   solve   every lane runs its piece from LDS and overwrites each slot it has
//           finished with (segment value, edge dual).  When some lane's last
//           segment runs past the tail, the whole wave stages the next block
//           at once into LDS reserved for it; positions beyond that reserve
//           (a longer tail, or the deeper overlap after a failed bracket) are
//           read from global memory one by one;
//   store   the piece's results go back with coalesced accesses, combined
//           with the mode's other arrays (e.g. z <- (z - q1) + q2).
// No global store is in flight during the solve phase, so its loads never
// wait for stores (on gfx9 the vector memory counter covers both).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "chain.hpp"
#include "launch.hpp"
#include "lean.hpp"
#include "piece.hpp"

namespace mc {

namespace {

constexpr int kLanes = 64;        // chains per work item; one wave per workgroup
constexpr int kPad = kLanes + 1;  // LDS row stride: spreads the transposed accesses over banks

// workgroups hold exactly one wave: ordering LDS traffic among its lanes needs
// no barrier, only a fence that keeps the compiler from moving accesses
__device__ __forceinline__ void wave_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct Chain {
    int base, stride;
};

__device__ __forceinline__ Chain chain_of(const Geo& g, int axis, int c)
{
    Chain ch;
    if (axis == 0) {  // c = d*H + h
        ch.base = c * g.W;
        ch.stride = 1;
    } else if (axis == 1) {  // c = d*W + x
        const int d = c / g.W;
        ch.base = d * g.H * g.W + (c - d * g.W);
        ch.stride = g.W;
    } else {  // c = h*W + x
        ch.base = c;
        ch.stride = g.H * g.W;
    }
    return ch;
}

// ---- modes ---------------------------------------------------------------------
//
// v_at(i), a_at(i)       scan input and weight of the edge (i, i+stride) at voxel i
// pre(i) -> Pre          other inputs the results of voxel i are combined with
// store(i, pre, c, p)    write the results of voxel i (segment value c, dual p
//                        of its edge; p only when duals were requested)

// plain prox: x = c, optional clipped duals
struct ModeProx {
    const float* v;
    const float* a;
    float* x;
    float* p;
    __device__ __forceinline__ float v_at(int i) const { return v[i]; }
    __device__ __forceinline__ float a_at(int i) const { return a[i]; }
    struct Pre {};
    __device__ __forceinline__ Pre pre(int) const { return {}; }
    __device__ __forceinline__ void store(int i, float c, float pd) const
    {
        x[i] = c;
        if (p) p[i] = pd;
    }
    __device__ __forceinline__ void store(int i, const Pre&, float c, float pd) const { store(i, c, pd); }
};

// two-set form, rows: q1 = prox_rows(z)  (y1 = z - q1 is formed by the columns)
struct ModeRows2 {
    const float* z;
    const float* a;
    float* q1;
    float* p1;
    __device__ __forceinline__ float v_at(int i) const { return z[i]; }
    __device__ __forceinline__ float a_at(int i) const { return a[i]; }
    struct Pre {};
    __device__ __forceinline__ Pre pre(int) const { return {}; }
    __device__ __forceinline__ void store(int i, float c, float pd) const
    {
        q1[i] = c;
        if (p1) p1[i] = pd;
    }
    __device__ __forceinline__ void store(int i, const Pre&, float c, float pd) const { store(i, c, pd); }
};

// two-set form, columns: t = u - 2 y1 + z = q1 - y1 - w with y1 = z - q1;
// q2 = prox_cols(t); z' = y1 + q2 (Sec. 3.3 special case r = 2, reflected
// through rows first).  z' goes to a second buffer: pieces re-read the
// overlap and tail of their neighbours, so the state is never updated in place.
struct ModeCols2 {
    const float* q1;
    const float* z;
    float* znew;
    const float* w;
    const float* a;
    float* p2;
    __device__ __forceinline__ float v_at(int i) const
    {
        const float q = q1[i];
        const float y = z[i] - q;
        return (q - y) - w[i];
    }
    __device__ __forceinline__ float a_at(int i) const { return a[i]; }
    struct Pre {
        float y;
    };
    __device__ __forceinline__ Pre pre(int i) const { return {z[i] - q1[i]}; }
    __device__ __forceinline__ void store(int i, const Pre& pr, float c, float pd) const
    {
        znew[i] = pr.y + c;
        if (p2) p2[i] = pd;
    }
    __device__ __forceinline__ void store(int i, float c, float pd) const { store(i, pre(i), c, pd); }
};

// product space, non-final family j: q_j = prox_j(z_j)
struct ModeSweepP {
    const float* z;
    const float* a;
    float* q;
    float* p;
    __device__ __forceinline__ float v_at(int i) const { return z[i]; }
    __device__ __forceinline__ float a_at(int i) const { return a[i]; }
    struct Pre {};
    __device__ __forceinline__ Pre pre(int) const { return {}; }
    __device__ __forceinline__ void store(int i, float c, float pd) const
    {
        q[i] = c;
        if (p) p[i] = pd;
    }
    __device__ __forceinline__ void store(int i, const Pre&, float c, float pd) const { store(i, c, pd); }
    // non-temporal (streaming) accesses: data that one wave reads or writes
    // once, kept from crowding the L2 lines other waves still come back to
    __device__ __forceinline__ float v_nt(int i) const { return __builtin_nontemporal_load(z + i); }
    __device__ __forceinline__ float a_nt(int i) const { return __builtin_nontemporal_load(a + i); }
    __device__ __forceinline__ void store_nt(int i, float c, float pd) const
    {
        __builtin_nontemporal_store(c, q + i);
        if (p) __builtin_nontemporal_store(pd, p + i);
    }
};

// product space, final family R-1 fused with the average step (Pi_L of
// eq. (dualA) inside the reflection R_L): with y_j = z_j - q_j,
// z_j' = y_j - (2 Y - Z - u) / R, Y = sum y_j, Z = sum z_j; z' goes to a
// second buffer (see ModeCols2).
template <int R>
struct ModeFinalP {
    const float* z;  // R*n, family j at j*n
    float* znew;     // R*n
    const float* q;  // (R-1)*n
    const float* a;
    const float* w;
    float* p;
    int n;
    __device__ __forceinline__ float v_at(int i) const { return z[(R - 1) * n + i]; }
    __device__ __forceinline__ float a_at(int i) const { return a[i]; }
    struct Pre {
        float zl, y[R - 1], sz, w;
    };
    __device__ __forceinline__ Pre pre(int i) const
    {
        Pre pr;
        pr.zl = z[(R - 1) * n + i];
        pr.sz = 0.f;
#pragma unroll
        for (int f = 0; f < R - 1; ++f) {
            const float zf = z[f * n + i];
            pr.y[f] = zf - q[f * n + i];
            pr.sz += zf;
        }
        pr.w = w[i];
        return pr;
    }
    __device__ __forceinline__ void store(int i, const Pre& pr, float c, float pd) const
    {
        const float yl = pr.zl - c;
        float Y = yl;
#pragma unroll
        for (int f = 0; f < R - 1; ++f) Y += pr.y[f];
        const float Z = pr.sz + pr.zl;
        const float corr = (2.f * Y - Z + pr.w) * (1.f / (float)R);
#pragma unroll
        for (int f = 0; f < R - 1; ++f) znew[f * n + i] = pr.y[f] - corr;
        znew[(R - 1) * n + i] = yl - corr;
        if (p) p[i] = pd;
    }
    __device__ __forceinline__ void store(int i, float c, float pd) const { store(i, pre(i), c, pd); }
};

// ---- one work item -----------------------------------------------------------------

template <class M, bool kRows, bool kExact>
__device__ __forceinline__ void sweep_piece(const Geo& g, int axis, int item, const M& mode,
                                            const PieceCfg& cfg, float* lds)
{
    const int lane = threadIdx.x;
    const int nch = geo_nchains(g, axis);
    const int m = geo_extent(g, axis);
    const int cg = item / cfg.pieces, s = item - cg * cfg.pieces;
    const int c0 = cg * kLanes;
    const int c = c0 + lane;
    const bool valid = c < nch;
    const int nrows = nch - c0 < kLanes ? nch - c0 : kLanes;
    const Chain ch = chain_of(g, axis, valid ? c : c0);
    const int b0 = s * cfg.len;
    const int b1 = b0 + cfg.len < m ? b0 + cfg.len : m;
    // LDS slot k holds position base + k.  The staged window [lo, hi) starts
    // one position before the overlap (the weight of the edge in front of the
    // scans' start) and grows at its end on demand up to hi_cap.
    const int base = b0 - cfg.reach_lo > 0 ? b0 - cfg.reach_lo : 0;
    const int hi_cap = b1 + cfg.reach_hi < m ? b1 + cfg.reach_hi : m;
    const int lo = base;
    int hi = b1 + cfg.tail < m ? b1 + cfg.tail : m;
    const int slots = cfg.reach_lo + cfg.len + cfg.reach_hi;
    // [slot][lane] pairs (v, a), later (segment value, edge dual): one LDS
    // access moves both.  Two spare rows: writes of lanes with nothing to
    // emit, and values fetched from outside the window (row slots for L,
    // slots + 1 for U).  Position q of this lane is at q * kPad + lb.
    float2* lw = reinterpret_cast<float2*>(lds);
    const int lb = lane - base * kPad;
    const int spare = slots * kPad + lane;

    // Stage positions [qa, qb) of the 64 chains: B independent loads per lane
    // in flight before any LDS write (more for the initial window, when the
    // scan state is not live yet, 8 for growth inside the solve loop).  Rows are walked (row, position)
    // flattened over the lanes, so consecutive lanes read consecutive positions.
    // The loads are unconditional (elements past the end re-read a valid one)
    // so that they are all issued before the first wait; only the LDS writes
    // are predicated.  Weights are staged as a + 0: a -0 weight must not look
    // like a knot mark of the value sweeps.
    constexpr int kBatch = 16;
    auto stage = [&](int qa, int qb, auto batch) {
        constexpr int B = decltype(batch)::value;
        const int len_r = qb - qa;
        if (len_r <= 0) return;
        if (kRows) {
            const int total = nrows * len_r;
            const int drr = kLanes / len_r, dq = kLanes - drr * len_r;
            int rr = lane / len_r, q = lane - rr * len_r;  // element lane + kLanes * t
            for (int t0 = 0; t0 * kLanes < total; t0 += B) {
                float vv[B], aa[B];
                int r2 = rr, q2 = q;
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    const int i = (c0 + (rr < nrows ? rr : nrows - 1)) * g.W + qa + q;
                    vv[u] = mode.v_at(i);
                    aa[u] = mode.a_at(i);
                    rr += drr;
                    q += dq;
                    if (q >= len_r) {
                        q -= len_r;
                        ++rr;
                    }
                }
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    if (r2 < nrows) lw[(qa + q2 - base) * kPad + r2] = make_float2(vv[u], aa[u] + 0.f);
                    r2 += drr;
                    q2 += dq;
                    if (q2 >= len_r) {
                        q2 -= len_r;
                        ++r2;
                    }
                }
            }
        } else if (valid) {
            for (int qb0 = qa; qb0 < qb; qb0 += B) {
                float vv[B], aa[B];
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    const int q = qb0 + u < qb ? qb0 + u : qb - 1;
                    const int i = ch.base + q * ch.stride;
                    vv[u] = mode.v_at(i);
                    aa[u] = mode.a_at(i);
                }
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    const int q = qb0 + u;
                    if (q < qb) lw[__mul24(q, kPad) + lb] = make_float2(vv[u], aa[u] + 0.f);
                }
            }
        }
        wave_fence();
    };
    // rows load two arrays per element, the column modes up to four
    using Big = std::integral_constant<int, kRows ? 2 * kBatch : kBatch>;
    using Small = std::integral_constant<int, 8>;
    stage(lo, hi, Big{});

    // solve: the lean scan of each lane (see lean.hpp).  Knots inside the
    // piece are recorded in LDS at their slot: value sweeps store the segment
    // value and a negative weight as the mark; sweeps with duals store the
    // FP64 segment value as a float pair (the knot's v and a are read again
    // from global memory by the backward pass) and mark the knot in the
    // lane's bit masks.
    auto a_before = [&](int q) -> float {
        return (q >= lo && q < hi) ? lw[__mul24(q, kPad) + lb].y : mode.a_at(ch.base + q * ch.stride);
    };
    constexpr int kGrow = 8;
    const int W0 = cfg.overlap > 0 ? cfg.overlap : 1;
    LeanLaneT<kExact> pl;
    pl.begin(valid, m, b0, b1, W0, a_before);
    auto mark = [&](int q, float cv, const LeanSeg& sg, bool on, int, bool) {
        const int sl = on ? __mul24(q, kPad) + lb : spare;
        if constexpr (kExact) {
            const float chi = (float)sg.c;
            lw[sl] = make_float2(chi, (float)(sg.c - (double)chi));
        } else {
            lw[sl] = make_float2(cv, -1.f);
        }
    };
    auto grow = [&]() {
        if (hi < hi_cap && __any(pl.scanning && pl.L.k >= hi)) {
            const int nh = hi + kGrow < hi_cap ? hi + kGrow : hi_cap;
            stage(hi, nh, Small{});
            hi = nh;
        }
    };
    // Slot of position q for a scan read.  A position outside the window
    // (rare: the deeper overlap after a failed bracket, a tail beyond the
    // reserve) is fetched from global memory into the lane's slot of the
    // spare row first, so that the read itself is always an LDS read.
    auto slot_of = [&](int q) {
        const bool in = (q >= lo) & (q < hi);
        if (__any(!in)) {
            if (!in) {
                const int i = ch.base + q * ch.stride;
                lw[spare] = make_float2(mode.v_at(i), mode.a_at(i));
            }
            wave_fence();
        }
        return in ? __mul24(q, kPad) + lb : spare;
    };
    // While some lane brackets: both scans, U only where it brackets.
    // Positions outside the window go through the spare rows (L's in
    // row `slots`, U's in row `slots + 1`), one check for both.
    auto in_window = [&](int q) { return (q >= lo) & (q < hi); };
    const int spare_u = spare + kPad;
    while (__any(pl.bracket && pl.scanning)) {
        grow();
        const bool gl = pl.steps_l(), gu = pl.needs_u();
        const int ql = gl ? pl.L.k : lo, qu = gu ? pl.U.k : lo;
        const bool inl = in_window(ql), inu = in_window(qu);
        if (__any(!inl || !inu)) {
            if (!inl) {
                const int i = ch.base + ql * ch.stride;
                lw[spare] = make_float2(mode.v_at(i), mode.a_at(i));
            }
            if (!inu) {
                const int i = ch.base + qu * ch.stride;
                lw[spare_u] = make_float2(mode.v_at(i), mode.a_at(i));
            }
            wave_fence();
        }
        const float2 xl = lw[inl ? __mul24(ql, kPad) + lb : spare], xu = lw[inu ? __mul24(qu, kPad) + lb : spare_u];
        pl.step_l(gl, xl.x, ql != m - 1 ? xl.y : 0.f, mark);
        pl.step_u(gu, xu.x, qu != m - 1 ? xu.y : 0.f);
        pl.resolve(a_before);
    }
    // then L alone in every lane until its piece is covered
    while (__any(pl.scanning)) {
        grow();
        const int ql = pl.scanning ? pl.L.k : lo;
        const float2 x = lw[slot_of(ql)];
        if (pl.scanning) pl.step_plain(x.x, ql != m - 1 ? x.y : 0.f, mark);
    }
    wave_fence();
    if (g.restarts) {
        // lanes whose bracket did not close (they restarted further back); one
        // vector atomic per counter from lane 0
        const int nr = __popcll(__ballot(valid && pl.W != W0));
        const int nv = __popcll(__ballot(valid));
        if (lane == 0) {
            atomicAdd(g.restarts, nr);
            atomicAdd(g.restarts + 1, nv);
        }
    }
    if constexpr (!kExact) {
        // every position takes the value of the first knot at or after it;
        // the segment covering b1 - 1 is in registers
        float cur = pl.c_last;
        for (int q = b1 - 1; q >= b0; --q) {
            const int sl = __mul24(q, kPad) + lb;
            const float2 x = lw[sl];
            cur = x.y < 0.f ? x.x : cur;
            lw[sl].x = cur;
        }
    } else if (valid) {
        // Backward from b1 - 1, where the covering segment's value and the
        // dual of edge b1 - 1 are in registers: at a knot the value becomes
        // the knot's segment value and the dual its exact +-a; inside a
        // segment P_{q-1} = P_q + v_q - c, in FP64.  v and a of the knots
        // come from global memory, 8 positions' loads issued together.
        constexpr int kB = 8;
        double cur = pl.c_last64, p = pl.p_b1;
        for (int qt = b1 - 1; qt >= b0; qt -= kB) {
            float gv[kB], ga[kB];
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                const int q = qt - u;
                const bool kn = q >= b0 && ((pl.kmask >> (q - b0)) & 1ull);
                gv[u] = ga[u] = 0.f;
                if (kn) {
                    const int i = ch.base + q * ch.stride;
                    gv[u] = mode.v_at(i);
                    ga[u] = mode.a_at(i);
                }
            }
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                const int q = qt - u;
                if (q >= b0) {
                    const int sl = __mul24(q, kPad) + lb;
                    const float2 x = lw[sl];
                    const float x0 = x.x, x1 = x.y;
                    const bool kn = (pl.kmask >> (q - b0)) & 1ull;
                    const bool up = (pl.umask >> (q - b0)) & 1ull;
                    const float vq = kn ? gv[u] : x0, aq = kn ? ga[u] : x1;
                    cur = kn ? (double)x0 + (double)x1 : cur;
                    p = kn ? (double)(up ? aq : -aq) : p;
                    lw[sl] = make_float2((float)cur, q == m - 1 ? 0.f : clip_dual(p, aq));
                    p += (double)vq - cur;
                }
            }
        }
    }
    wave_fence();

    // store
    if (kRows) {
        const int len_r = b1 - b0;
        const int total = nrows * len_r;
        const int drr = kLanes / len_r, dq = kLanes - drr * len_r;
        int rr = lane / len_r, q = lane - rr * len_r;
        for (int t = 0; t * kLanes < total; ++t) {
            if (rr < nrows) {
                const float2 x = lw[(b0 + q - base) * kPad + rr];
                mode.store((c0 + rr) * g.W + b0 + q, x.x, kExact ? x.y : 0.f);
            }
            rr += drr;
            q += dq;
            if (q >= len_r) {
                q -= len_r;
                ++rr;
            }
        }
    } else if (valid) {
        for (int qb = b0; qb < b1; qb += kBatch) {
            float cv[kBatch], pv[kBatch];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int q = qb + u;
                const float2 x = q < b1 ? lw[__mul24(q, kPad) + lb] : make_float2(0.f, 0.f);
                cv[u] = x.x;
                pv[u] = kExact ? x.y : 0.f;
            }
            typename M::Pre pre[kBatch];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int q = qb + u;
                if (q < b1) pre[u] = mode.pre(ch.base + q * ch.stride);
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int q = qb + u;
                if (q < b1) mode.store(ch.base + q * ch.stride, pre[u], cv[u], pv[u]);
            }
        }
    }
}

// Workgroups of a launch are dealt to the chip's eight XCDs in turn
// (workgroup b runs on XCD b mod 8), and each XCD has its own L2.  Neighbouring
// pieces of a chain group stage overlapping windows, so they should share an
// L2; the work of a launch (grids of a batch that finish at different times)
// should still spread over all XCDs.  xcd_item gives each XCD runs of kXcdRun
// consecutive work items, the runs dealt to the XCDs in turn: workgroup b,
// the j-th on its XCD x = b mod 8, takes item ((j / kXcdRun) * 8 + x) * kXcdRun
// + j mod kXcdRun.  Items past the last whole round of runs keep their index.
// A bijection of [0, n).
constexpr int kXcds = 8;
constexpr int kXcdRun = 16;

__device__ __forceinline__ int xcd_item(int b, int n)
{
    const int round = kXcds * kXcdRun;
    if (b >= n / round * round) return b;
    const int x = b % kXcds, j = b / kXcds;
    return ((j / kXcdRun) * kXcds + x) * kXcdRun + j % kXcdRun;
}

// Whole chains: one lane per chain runs a single exact scan from the chain
// start, where the dual is 0, so there is no bracket and no restart; the fill
// trails the scan and writes each output through the mode.  Values come from
// global memory (a lane walks its own chain: rows share cache lines, columns
// are coalesced across lanes).  When the chain proxes have long constant
// segments, the brackets of the piece scheme do not close and its lanes scan
// back to the chain start anyway, many lanes per chain; here each chain is
// scanned once.
template <class M, bool kExact>
__global__ void __launch_bounds__(kLanes) k_sweep_whole(Geo g, int axis, M mode)
{
    const int c = blockIdx.x * kLanes + threadIdx.x;
    const int m = geo_extent(g, axis);
    const bool valid = c < geo_nchains(g, axis);
    const Chain ch = chain_of(g, axis, valid ? c : 0);
    auto at = [&](int q) -> RingVals<2> {
        const int i = ch.base + q * ch.stride;
        return {{mode.v_at(i), mode.a_at(i)}};
    };
    auto emit = [&](int q, auto cv, auto pr, bool last, bool on) {
        if (!on) return;
        const int i = ch.base + q * ch.stride;
        float pd = 0.f;
        if constexpr (kExact) pd = last ? 0.f : clip_dual(pr, mode.a_at(i));
        mode.store(i, mode.pre(i), (float)cv, pd);
    };
    auto no_weight_before = [](int) { return 0.f; };  // never read: the scan starts at the chain start
    PieceLane<2, kExact> pl;
    pl.begin(valid, m, 0, m, 1, no_weight_before);
    while (__any(pl.busy())) {
        const RingVals<2> rf = at(pl.fill_pos(0)), rl = at(pl.l_pos(0));
        pl.fill(rf, emit);
        pl.step_l(rl);
    }
}

// Whole chains staged in LDS: cpi chains per work item (lanes cpi..63 idle)
// with all m positions of their scan input and weights in LDS, so the scan
// never waits on global memory.  A scan position is known only after the
// previous step (a rescan jumps back), so read from global memory every loop
// iteration waits one round trip; when only a few waves run (whole chains are
// chosen for flat data, one lane per chain) nothing hides that latency.
// LDS [position][chain] with pitch cpi + 1: column cpi takes the reads of idle
// lanes, row m the writes of lanes with nothing to emit.  Loads and stores
// walk (chain, position) flattened over the lanes, the contiguous index
// fastest (positions for rows, chains for columns and depth).
constexpr size_t kWholeLdsBytes = 48 * 1024;
// With many chains the global-memory sweep keeps all 64 lanes of every wave
// busy and enough waves resident to hide its latency, while the LDS version
// (fewer chains per wave, LDS-limited residency) issues more instructions per
// chain: measured on the 256x256x128 volume, 1053 against 687 us for the
// three families of an iteration.  Staging pays while the global sweep would
// launch fewer than one wave per CU.
constexpr int kWholeLdsMaxWaves = 256;

__host__ __device__ inline int whole_lds_cpi(int m)
{
    const int pad = (int)(kWholeLdsBytes / (2 * sizeof(float) * ((size_t)m + 1)));
    return pad - 1 < kLanes ? pad - 1 : kLanes;
}

template <class M, bool kRows, bool kExact>
__global__ void __launch_bounds__(kLanes) k_sweep_whole_lds(Geo g, int axis, M mode, int cpi)
{
    extern __shared__ __attribute__((aligned(16))) float lds[];
    const int lane = threadIdx.x;
    const int m = geo_extent(g, axis);
    const int nch = geo_nchains(g, axis);
    const int c0 = blockIdx.x * cpi;
    const int nrows = nch - c0 < cpi ? nch - c0 : cpi;
    const bool valid = lane < nrows;
    const int pad = cpi + 1;
    const int col = valid ? lane : cpi;
    float* lv = lds;                          // [position][chain]: v, later segment value
    float* la = lds + (size_t)(m + 1) * pad;  // [position][chain]: a, later edge dual
    const int total = nrows * m;
    // element e of the work item -> chain r and position q
    auto elem = [&](int e, int& r, int& q) {
        if (kRows) {
            r = e / m;
            q = e - r * m;
        } else {
            q = e / nrows;
            r = e - q * nrows;
        }
    };
    constexpr int B = 16;
    for (int e0 = 0; e0 < total; e0 += kLanes * B) {
        float vv[B], aa[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int e = e0 + u * kLanes + lane;
            if (e < total) {
                int r, q;
                elem(e, r, q);
                const Chain ch = chain_of(g, axis, c0 + r);
                const int i = ch.base + q * ch.stride;
                vv[u] = mode.v_at(i);
                aa[u] = mode.a_at(i);
            }
        }
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int e = e0 + u * kLanes + lane;
            if (e < total) {
                int r, q;
                elem(e, r, q);
                lv[q * pad + r] = vv[u];
                la[q * pad + r] = aa[u];
            }
        }
    }
    wave_fence();

    auto at = [&](int q) -> RingVals<2> {
        const int sl = q * pad + col;
        return {{lv[sl], la[sl]}};
    };
    auto emit = [&](int q, auto cv, auto pr, bool last, bool on) {
        const int sl = (on ? q : m) * pad + col;
        lv[sl] = (float)cv;
        if constexpr (kExact) la[sl] = last ? 0.f : clip_dual(pr, la[sl]);
    };
    auto no_weight_before = [](int) { return 0.f; };  // never read: the scan starts at the chain start
    PieceLane<2, kExact> pl;
    pl.begin(valid, m, 0, m, 1, no_weight_before);
    while (__any(pl.busy())) {
        const RingVals<2> rf = at(pl.fill_pos(0)), rl = at(pl.l_pos(0));
        pl.fill(rf, emit);
        pl.step_l(rl);
    }
    wave_fence();

    constexpr int S = 8;
    for (int e0 = 0; e0 < total; e0 += kLanes * S) {
        int idx[S];
        float cv[S], pv[S];
        typename M::Pre pre[S];
#pragma unroll
        for (int u = 0; u < S; ++u) {
            const int e = e0 + u * kLanes + lane;
            idx[u] = -1;
            if (e < total) {
                int r, q;
                elem(e, r, q);
                const Chain ch = chain_of(g, axis, c0 + r);
                idx[u] = ch.base + q * ch.stride;
                cv[u] = lv[q * pad + r];
                pv[u] = kExact ? la[q * pad + r] : 0.f;
                pre[u] = mode.pre(idx[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < S; ++u)
            if (idx[u] >= 0) mode.store(idx[u], pre[u], cv[u], pv[u]);
    }
}

template <class M, bool kRows, bool kExact>
__global__ void __launch_bounds__(kLanes) k_sweep(Geo g, int axis, M mode, PieceCfg cfg)
{
    extern __shared__ __attribute__((aligned(16))) float lds[];
    sweep_piece<M, kRows, kExact>(g, axis, xcd_item(blockIdx.x, gridDim.x), mode, cfg, lds);
}

// the two non-final families of the 3D product space in one launch:
// items [0, n0) sweep the rows (axis 0), the rest the columns (axis 1)
template <bool kExact>
__global__ void __launch_bounds__(kLanes)
k_sweep_pair(Geo g, ModeSweepP m0, ModeSweepP m1, PieceCfg c0, PieceCfg c1, int n0)
{
    extern __shared__ __attribute__((aligned(16))) float lds[];
    const int item = xcd_item(blockIdx.x, gridDim.x);
    if (item < n0)
        sweep_piece<ModeSweepP, true, kExact>(g, 0, item, m0, c0, lds);
    else
        sweep_piece<ModeSweepP, false, kExact>(g, 1, item - n0, m1, c1, lds);
}

// Three independent families in one launch: items [0, n0) the rows and
// [n0, n0 + n1) the columns of g (product-space sweeps), the rest family 3:
// the straightened zig-zag chains of an 8-connected grid (rows of gz), or
// the depth chains of a volume (axis 2 of g)
template <class M2, bool kRows2, bool kExact>
__global__ void __launch_bounds__(kLanes)
k_sweep_triple(Geo g, ModeSweepP m0, ModeSweepP m1, Geo g2, int axis2, M2 m2, PieceCfg c0, PieceCfg c1,
               PieceCfg c2, int n0, int n1)
{
    extern __shared__ __attribute__((aligned(16))) float lds[];
    const int item = xcd_item(blockIdx.x, gridDim.x);
    if (item < n0)
        sweep_piece<ModeSweepP, true, kExact>(g, 0, item, m0, c0, lds);
    else if (item < n0 + n1)
        sweep_piece<ModeSweepP, false, kExact>(g, 1, item - n0, m1, c1, lds);
    else
        sweep_piece<M2, kRows2, kExact>(g2, axis2, item - n0 - n1, m2, c2, lds);
}


inline int items_of(const Geo& g, int axis, const PieceCfg& cfg)
{
    return (geo_nchains(g, axis) + kLanes - 1) / kLanes * cfg.pieces;
}

inline size_t lds_bytes(const PieceCfg& cfg)
{
    return sizeof(float) * 2 * (size_t)(cfg.reach_lo + cfg.len + cfg.reach_hi + 2) * kPad;
}

// Volumes in throughput mode: 16-position pieces (about 8192 work items per
// family), overlap 4 and no staged tail.  The window is then 23 LDS rows
// (12 KB per wave), and residency is set by the registers (12 waves per CU)
// instead of by LDS (6 with the default 32-position pieces, overlap and tail
// 8): the scans hide their stalls behind the extra waves more than the extra
// restarts, overlap and tail reads from global memory cost.  Volume solve:
// 75.8 ms with the defaults; 68.8 ms with 32-position pieces, overlap 4 and no
// tail (8 waves); 67.6 ms with 24-position pieces (10 waves); 67.2 ms with
// 16 (overlap 5 or 8 at 7 waves: 71.0, 71.6 ms).  On the 64-grid batch
// overlap 4 and no tail were slower, so the other launches keep 8 and 8.  The sweeps that count restarts (the solve's
// first, which choose between pieces and whole chains) keep the default
// overlap: early iterations have long constant segments, and with overlap 4
// about 1 lane in 10 restarts there (the threshold of that choice) against
// 0.4 % later on (simulated on the volume's states).
constexpr int kVolOverlap = 4, kVolTail = 0, kVolItems = 8192;

// ---- long pieces streamed through an LDS ring (sweeps of volumes) -------------------
//
// The sweeps of a volume after the first iteration: pieces of about
// kStreamLen positions (a 256 x 256 x 128 volume: rows and columns in two
// pieces, depth chains whole -- 3072 waves, 3 per SIMD, every wave about
// 128 positions long), each scanned as the short pieces are (the lean scan,
// bracketed from kVolOverlap positions before the piece unless it starts the
// chain), but with the window streamed through a ring of kRing LDS rows
// instead of staged whole: the overlap and the bracket are then paid once
// per 128 positions instead of once per 16.  The ring holds positions
// [lo, hi) of the 64 chains (row q mod kRing), staged kStage positions at a
// time with coalesced loads issued one batch ahead.  A finished segment of
// the result marks its last position with (value, -1); positions leave the
// ring oldest first when the next batch needs the room: a backward pass gives
// every position of the piece up to the lane's last finished one the value
// of the next mark at or after it, and the batch goes to global memory with
// coalesced stores, issued after the next batch is in.  The columns and depth
// families read and write whole rows of 64 chains (256 bytes) once, with
// non-temporal accesses; the rows family reads 32 bytes of each row per
// batch and comes back for the rest of the line, so it keeps its lines in L2
// (FETCH_SIZE per value launch -33 %).  Sweeps that also
// write edge duals fill every finished segment at once instead: its
// positions in order, the dual carried forward in FP64 from the one in front
// of the segment (P_e = P_{e-1} + c - v_e, Sec. 3.2), exactly +-a at its
// knot; the ring slots then hold (value, dual) and leave as they are.  A
// lane still reads from the start of its open segment(s) on; while that is
// below the room needed and some lane can still step, the lanes that reached
// hi wait.  Only when every lane waits (a segment longer than kRing - kStage
// positions) the oldest positions go anyway; a lane behind them reads them
// from global memory through its spare slot, and writes the values (and
// duals) of its finished segments there directly.  Same values as the short
// pieces (every piece is exact from a knot of the true solution or the chain
// start); the duals agree to the FP64 rounding of the carried sums.
constexpr int kRing = 16;      // positions per chain in the ring (a power of 2)
constexpr int kStage = 8;      // positions staged at a time (4 with duals: fewer registers, 3 waves per SIMD)
constexpr int kStreamLen = 128;
// launches with fewer 64-chain waves keep the short pieces (too few lanes otherwise)
constexpr int kStreamMinWaves = 2048;

inline size_t stream_lds_bytes() { return sizeof(float2) * (kRing + 2) * kPad + sizeof(int) * kLanes; }

struct StreamCfg {
    int len, pieces;
};

inline StreamCfg stream_config(const Geo& g, int axis)
{
    const int m = geo_extent(g, axis);
    int pieces = (m + kStreamLen / 2) / kStreamLen;
    pieces = pieces < 1 ? 1 : pieces;
    StreamCfg c;
    c.len = (m + pieces - 1) / pieces;
    c.pieces = (m + c.len - 1) / c.len;
    return c;
}

template <bool kRows, bool kExact>
__device__ __forceinline__ void stream_piece(const Geo& g, int axis, int grp, int s, int len, const ModeSweepP& mode,
                                             float2* ring, int* lastk_sh)
{
    constexpr int kSt = kExact ? 4 : kStage;  // positions staged at a time
    const int lane = threadIdx.x;
    const int nch = geo_nchains(g, axis);
    const int m = geo_extent(g, axis);
    const int c0 = grp * kLanes;
    const bool valid = c0 + lane < nch;
    const int nrows = nch - c0 < kLanes ? nch - c0 : kLanes;
    const Chain ch = chain_of(g, axis, valid ? c0 + lane : c0);
    const int b0 = s * len;
    const int b1 = b0 + len < m ? b0 + len : m;
    const int spare = kRing * kPad + lane, spare_u = spare + kPad;
    auto slot = [&](int q, int r) { return __mul24(q & (kRing - 1), kPad) + r; };

    // Prefetch registers: one batch of kSt positions of the 64 chains.
    // Rows (chains along W, contiguous): element lane + 64 u of the
    // 64 x kSt block is chain (lane + 64 u) / kSt, position
    // (lane + 64 u) mod kSt, so that kSt consecutive lanes read one
    // row's consecutive positions; otherwise position qa + u of the lane's
    // chain.  Elements past the chain's end re-read its last position.
    constexpr int kRowsPer = kLanes / kSt;
    auto e_row = [&](int u) { return kRows ? lane / kSt + kRowsPer * u : lane; };
    auto e_pos = [&](int qa, int u) { return kRows ? qa + lane % kSt : qa + u; };
    auto gidx = [&](int r, int q) { return kRows ? (c0 + r) * g.W + q : ch.base + q * ch.stride; };
    float pv[kSt], pa[kSt], ov[kSt], op[kExact ? kSt : 1];
    auto issue = [&](int qa) {
#pragma unroll
        for (int u = 0; u < kSt; ++u) {
            const int r = e_row(u), q = e_pos(qa, u);
            const int i = gidx(r < nrows ? r : nrows - 1, q < m ? q : m - 1);
            pv[u] = kRows ? mode.v_at(i) : mode.v_nt(i);
            pa[u] = kRows ? mode.a_at(i) : mode.a_nt(i);
        }
    };
    auto commit = [&](int qa, int qb) {
#pragma unroll
        for (int u = 0; u < kSt; ++u) {
            const int r = e_row(u), q = e_pos(qa, u);
            if (r < nrows && q < qb) ring[slot(q, r)] = make_float2(pv[u], pa[u] + 0.f);
        }
    };

    // the window starts at the weight in front of the bracket's start
    int lo = b0 - kVolOverlap - 1 > 0 ? b0 - kVolOverlap - 1 : 0;
    int hi = lo + kSt < m ? lo + kSt : m;
    issue(lo);
    commit(lo, hi);
    if (hi < m) issue(hi);
    wave_fence();

    int lastk = -1;        // last position of the lane's last finished segment
    int fq = 1, fe = 0;    // positions of a finished segment to write directly (values) or to fill (duals)
    float fc = 0.f;
    double fc64 = 0.0, fA = 0.0;  // duals: the segment's FP64 value and the dual in front of it
    int fend = 0;
    float fan = 0.f;
    auto a_before = [&](int q) -> float {
        return (q >= lo && q < hi) ? ring[slot(q, lane)].y : mode.a_at(ch.base + q * ch.stride);
    };
    auto mark = [&](int q, float cv, const LeanSeg& sg, bool, int k0, bool out) {
        lastk = out ? q : lastk;
        if constexpr (kExact) {
            // the whole segment [k0, q] is filled forward after the step
            fq = out ? k0 : 1;
            fe = out ? (q < b1 - 1 ? q : b1 - 1) : 0;
            fend = q;
            fc64 = sg.c;
            fA = -(double)sg.nA;
            fan = sg.an;
        } else {
            ring[out && q >= lo ? slot(q, lane) : spare] = make_float2(cv, -1.f);
            const int e0 = q < lo - 1 ? q : lo - 1;
            fq = out ? (k0 > b0 ? k0 : b0) : 1;
            fe = out ? (e0 < b1 - 1 ? e0 : b1 - 1) : 0;
            fc = cv;
        }
    };
    // Values: the finished segment's positions that left the ring already.
    // Duals: every position of the finished segment [k0, kend] in order, the
    // dual carried forward in FP64 from the one in front of it
    // (P_e = P_{e-1} + c - v_e, Sec. 3.2), exactly +-a at the knot and 0 at
    // the chain's end; positions of the piece take (value, clipped dual) in
    // their ring slot, or in global memory when they left the ring already.
    auto fill_direct = [&]() {
        if constexpr (kExact) {
            double P = fA;
            const float cf = (float)fc64;
            while (__any(fq <= fe)) {
                if (fq <= fe) {
                    const bool in = fq >= lo;
                    const int i = ch.base + fq * ch.stride;
                    const float2 x = in ? ring[slot(fq, lane)] : make_float2(mode.v_at(i), mode.a_at(i));
                    P += fc64 - (double)x.x;
                    if (fq >= b0) {
                        const float pd = fq == m - 1 ? 0.f : clip_dual(fq == fend ? (double)fan : P, x.y);
                        if (in) ring[slot(fq, lane)] = make_float2(cf, pd);
                        else mode.store(i, cf, pd);
                    }
                    ++fq;
                }
            }
        } else {
            while (__any(fq <= fe)) {
                if (fq <= fe) {
                    mode.store(ch.base + fq * ch.stride, fc, 0.f);
                    ++fq;
                }
            }
        }
        fq = 1;
        fe = 0;
    };
    LeanLaneT<kExact> pl;
    pl.begin(valid, m, b0, b1, kVolOverlap, a_before);

    // Positions [qa, qb) of the piece leave the ring or are final: each
    // lane's positions up to lastk take the value of the next mark at or
    // after them (searched from top - 1 down), written over v in the ring.
    auto fill_back = [&](int qa, int qb, int top) {
        wave_fence();
        float cur = 0.f;
        for (int q = top - 1; q >= qa; --q) {
            const int sl = slot(q, lane);
            const float2 x = ring[sl];
            cur = x.y < 0.f ? x.x : cur;
            if (q < qb) ring[sl].x = cur;
        }
        lastk_sh[lane] = lastk;
        wave_fence();
    };
    // oldest position a lane may still read: the start of its open segment
    // (of both scans while it brackets)
    auto need_of = [&]() {
        int nd = pl.scanning ? pl.L.k - (int)pl.L.len : m;
        const int nu = pl.U.k - (int)pl.U.len;
        nd = pl.scanning && pl.bracket && nu < nd ? nu : nd;
#pragma unroll
        for (int o = kLanes / 2; o > 0; o >>= 1) {
            const int t = __shfl_xor(nd, o);
            nd = t < nd ? t : nd;
        }
        return nd;
    };
    // Stage the next batch when some lane needs position hi; evictions
    // (at most kSt positions) read their values into registers before the
    // batch overwrites their slots and store them after it is in.
    auto stage = [&](bool want, bool can_step) {
        if (hi >= m || !want) return;
        const int nh = hi + kSt < m ? hi + kSt : m;
        const int nl = nh - kRing > lo ? nh - kRing : lo;
        if (nl > lo && nl > need_of() && can_step) return;  // the lanes at hi wait
        const int ol = lo;
        if (nl > ol) {
            if constexpr (kExact) {
                wave_fence();
                lastk_sh[lane] = lastk;
                wave_fence();
            } else {
                fill_back(ol, nl, hi);
            }
#pragma unroll
            for (int u = 0; u < kSt; ++u) {
                const float2 x = ring[slot(e_pos(ol, u), e_row(u))];
                ov[u] = x.x;
                if constexpr (kExact) op[u] = x.y;
            }
            wave_fence();
        }
        commit(hi, nh);
        if (nl > ol) {
#pragma unroll
            for (int u = 0; u < kSt; ++u) {
                const int r = e_row(u), q = e_pos(ol, u);
                if (r < nrows && q < nl && q >= b0 && q < b1 && q <= lastk_sh[r]) {
                    if (kRows) mode.store(gidx(r, q), ov[u], kExact ? op[u] : 0.f);
                    else mode.store_nt(gidx(r, q), ov[u], kExact ? op[u] : 0.f);
                }
            }
        }
        lo = nl;
        hi = nh;
        if (hi < m) issue(hi);
        wave_fence();
    };

    // both scans while some lane brackets (positions below lo through the
    // spare slots: L's in row kRing, U's in row kRing + 1)
    while (__any(pl.bracket && pl.scanning)) {
        const bool gl0 = pl.steps_l(), gu0 = pl.needs_u();
        stage(__any((gl0 && pl.L.k >= hi) || (gu0 && pl.U.k >= hi)),
              __any((gl0 && pl.L.k < hi) || (gu0 && pl.U.k < hi)));
        const bool gl = gl0 && pl.L.k < hi, gu = gu0 && pl.U.k < hi;
        const int ql = gl ? pl.L.k : lo, qu = gu ? pl.U.k : lo;
        const bool inl = ql >= lo, inu = qu >= lo;
        if (__any(!inl || !inu)) {
            if (!inl) {
                const int i = ch.base + ql * ch.stride;
                ring[spare] = make_float2(mode.v_at(i), mode.a_at(i));
            }
            if (!inu) {
                const int i = ch.base + qu * ch.stride;
                ring[spare_u] = make_float2(mode.v_at(i), mode.a_at(i));
            }
            wave_fence();
        }
        const float2 xl = ring[inl ? slot(ql, lane) : spare], xu = ring[inu ? slot(qu, lane) : spare_u];
        pl.step_l(gl, xl.x, ql != m - 1 ? xl.y : 0.f, mark);
        pl.step_u(gu, xu.x, qu != m - 1 ? xu.y : 0.f);
        pl.resolve(a_before);
        fill_direct();
    }
    // then L alone in every lane until its piece is covered
    while (__any(pl.scanning)) {
        stage(__any(pl.scanning && pl.L.k >= hi), __any(pl.scanning && pl.L.k < hi));
        const bool go = pl.scanning && pl.L.k < hi;
        const int ql = go ? pl.L.k : lo;
        const bool in = ql >= lo;
        if (__any(!in)) {
            if (!in) {
                const int i = ch.base + ql * ch.stride;
                ring[spare] = make_float2(mode.v_at(i), mode.a_at(i));
            }
            wave_fence();
        }
        const float2 x = ring[in ? slot(ql, lane) : spare];
        if (go) pl.step_plain(x.x, ql != m - 1 ? x.y : 0.f, mark);
        fill_direct();
    }
    // the rest of the piece: every lane is final up to b1 - 1
    const int qa = lo > b0 ? lo : b0;
    if (qa < b1) {
        if constexpr (kExact) wave_fence();
        else fill_back(qa, b1, hi);
        const int len_r = b1 - qa;
        if (kRows) {
            const int total = nrows * len_r;
            const int drr = kLanes / len_r, dq = kLanes - drr * len_r;
            int rr = lane / len_r, q = lane - rr * len_r;
            for (int t = 0; t * kLanes < total; ++t) {
                if (rr < nrows) {
                    const float2 x = ring[slot(qa + q, rr)];
                    mode.store(gidx(rr, qa + q), x.x, kExact ? x.y : 0.f);
                }
                rr += drr;
                q += dq;
                if (q >= len_r) {
                    q -= len_r;
                    ++rr;
                }
            }
        } else if (valid) {
            for (int q = qa; q < b1; ++q) {
                const float2 x = ring[slot(q, lane)];
                mode.store(gidx(lane, q), x.x, kExact ? x.y : 0.f);
            }
        }
    }
}

// the value sweep of the three families of a volume in streamed pieces (mode j
// sweeps axis j): waves [0, w1) the columns, [w1, w1 + w0) the rows, the rest
// the depth chains; wave -> (chain group, piece) with the piece fastest
template <bool kExact>
__global__ void __launch_bounds__(kLanes) __attribute__((amdgpu_waves_per_eu(3, 3)))
k_stream3(Geo g, ModeSweepP m0, ModeSweepP m1, ModeSweepP m2, StreamCfg s0, StreamCfg s1, StreamCfg s2, int w1,
          int w0)
{
    extern __shared__ __attribute__((aligned(16))) float lds[];
    float2* ring = reinterpret_cast<float2*>(lds);
    int* lastk_sh = reinterpret_cast<int*>(ring + (kRing + 2) * kPad);
    const int b = blockIdx.x;
    if (b < w1)
        stream_piece<false, kExact>(g, 1, b / s1.pieces, b % s1.pieces, s1.len, m1, ring, lastk_sh);
    else if (b < w1 + w0)
        stream_piece<true, kExact>(g, 0, (b - w1) / s0.pieces, (b - w1) % s0.pieces, s0.len, m0, ring, lastk_sh);
    else
        stream_piece<false, kExact>(g, 2, (b - w1 - w0) / s2.pieces, (b - w1 - w0) % s2.pieces, s2.len, m2, ring,
                                    lastk_sh);
}


// the launch of k_sweep_triple with the latency / throughput mode decided on
// its total number of work items; in throughput mode, want > 0 (work items
// per family) and overlap / tail >= 0 replace the defaults
template <class M2, bool kRows2>
hipError_t launch_triple(const Geo& g, const ModeSweepP& m0, const ModeSweepP& m1, const Geo& g2, int axis2,
                         const M2& m2, bool duals, hipStream_t s, int want = 0, int overlap = 0, int tail = -1)
{
    PieceCfg c0 = piece_config(g, 0, kDefaultItems, 0), c1 = piece_config(g, 1, kDefaultItems, 0),
             c2 = piece_config(g2, axis2, kDefaultItems, 0);
    int tot = items_of(g, 0, c0) + items_of(g, 1, c1) + items_of(g2, axis2, c2);
    const bool thr = tot > kLatencyItems;
    const int wi = thr && want > 0 ? want : kDefaultItems;
    if (wi != kDefaultItems) {
        c0 = piece_config(g, 0, wi, 0), c1 = piece_config(g, 1, wi, 0), c2 = piece_config(g2, axis2, wi, 0);
        tot = items_of(g, 0, c0) + items_of(g, 1, c1) + items_of(g2, axis2, c2);
    }
    c0 = piece_config(g, 0, wi, tot, thr ? overlap : 0, thr ? tail : -1);
    c1 = piece_config(g, 1, wi, tot, thr ? overlap : 0, thr ? tail : -1);
    c2 = piece_config(g2, axis2, wi, tot, thr ? overlap : 0, thr ? tail : -1);
    const int n0 = items_of(g, 0, c0), n1 = items_of(g, 1, c1), n2 = items_of(g2, axis2, c2);
    size_t shm = lds_bytes(c0);
    if (lds_bytes(c1) > shm) shm = lds_bytes(c1);
    if (lds_bytes(c2) > shm) shm = lds_bytes(c2);
    if (duals)
        hipLaunchKernelGGL((k_sweep_triple<M2, kRows2, true>), dim3(n0 + n1 + n2), dim3(kLanes), shm, s, g, m0, m1,
                           g2, axis2, m2, c0, c1, c2, n0, n1);
    else
        hipLaunchKernelGGL((k_sweep_triple<M2, kRows2, false>), dim3(n0 + n1 + n2), dim3(kLanes), shm, s, g, m0,
                           m1, g2, axis2, m2, c0, c1, c2, n0, n1);
    return hipGetLastError();
}

template <class M, bool kExact>
hipError_t launch_mode_x(const Geo& g, int axis, const M& mode, const PieceCfg& cfg, hipStream_t s)
{
    const dim3 grid(items_of(g, axis, cfg)), block(kLanes);
    if (axis == 0)
        hipLaunchKernelGGL((k_sweep<M, true, kExact>), grid, block, lds_bytes(cfg), s, g, axis, mode, cfg);
    else
        hipLaunchKernelGGL((k_sweep<M, false, kExact>), grid, block, lds_bytes(cfg), s, g, axis, mode, cfg);
    return hipGetLastError();
}

template <class M>
hipError_t launch_mode(const Geo& g, int axis, const M& mode, bool duals, hipStream_t s)
{
    if (g.whole) {
        const int m = geo_extent(g, axis);
        const int cpi = whole_lds_cpi(m);
        if (cpi >= 1 && (geo_nchains(g, axis) + kLanes - 1) / kLanes < kWholeLdsMaxWaves) {  // staged in LDS
            const dim3 grid((geo_nchains(g, axis) + cpi - 1) / cpi), block(kLanes);
            const size_t shm = 2 * sizeof(float) * ((size_t)m + 1) * (size_t)(cpi + 1);
            if (axis == 0) {
                if (duals) hipLaunchKernelGGL((k_sweep_whole_lds<M, true, true>), grid, block, shm, s, g, axis, mode, cpi);
                else hipLaunchKernelGGL((k_sweep_whole_lds<M, true, false>), grid, block, shm, s, g, axis, mode, cpi);
            } else {
                if (duals) hipLaunchKernelGGL((k_sweep_whole_lds<M, false, true>), grid, block, shm, s, g, axis, mode, cpi);
                else hipLaunchKernelGGL((k_sweep_whole_lds<M, false, false>), grid, block, shm, s, g, axis, mode, cpi);
            }
            return hipGetLastError();
        }
        // chains too long for LDS, or many of them: every position from global memory
        const dim3 grid((geo_nchains(g, axis) + kLanes - 1) / kLanes), block(kLanes);
        if (duals) hipLaunchKernelGGL((k_sweep_whole<M, true>), grid, block, 0, s, g, axis, mode);
        else hipLaunchKernelGGL((k_sweep_whole<M, false>), grid, block, 0, s, g, axis, mode);
        return hipGetLastError();
    }
    // A grid with few chains (a 1024^2 image: 16 groups of 64 per family)
    // gets 8-position pieces while that keeps the launch latency-bound (at
    // most kLatencyItems work items, about two waves per SIMD): its waves then
    // scan half as many positions each.  1024^2 image: 12.8 -> 12.5 ms to the
    // exact cut.  (Batches keep 16: their waves overlap, and shorter pieces
    // only add overlap work -- 69.7 -> 75.3 ms p50 on the 64-grid batch.)
    PieceCfg cfg = piece_config(g, axis, kDefaultItems, 0, 0, -1, 8);
    if (items_of(g, axis, cfg) > kLatencyItems) cfg = piece_config(g, axis, kDefaultItems, 0);
    return duals ? launch_mode_x<M, true>(g, axis, mode, cfg, s)
                 : launch_mode_x<M, false>(g, axis, mode, cfg, s);
}

// ---- batched two-set iteration ----------------------------------------------------

template <bool kExact>
__global__ void __launch_bounds__(kLanes) k_batch_rows(BatchLaunch b, int parity)
{
    extern __shared__ __attribute__((aligned(16))) float lds[];
    const int item = xcd_item(blockIdx.x, gridDim.x);
    const int gi = b.item_grid_r[item];
    const BatchGrid& t = b.tab[gi];
    if (t.done) return;
    ModeRows2 m{t.z[parity], t.ax, t.q1, kExact ? t.p : nullptr};
    sweep_piece<ModeRows2, true, kExact>(t.g, 0, item - t.item0_r, m, t.cr, lds);
}

template <bool kExact>
__global__ void __launch_bounds__(kLanes) k_batch_cols(BatchLaunch b, int parity)
{
    extern __shared__ __attribute__((aligned(16))) float lds[];
    const int item = xcd_item(blockIdx.x, gridDim.x);
    const int gi = b.item_grid_c[item];
    const BatchGrid& t = b.tab[gi];
    if (t.done) return;
    ModeCols2 m{t.q1, t.z[parity], t.z[parity ^ 1], t.w, t.ay, kExact ? t.p + t.g.n : nullptr};
    sweep_piece<ModeCols2, false, kExact>(t.g, 1, item - t.item0_c, m, t.cc, lds);
}

// cold start: the row prox of z = 0 is 0 for every grid, with zero duals
// (blockIdx.y = grid)
__global__ void k_batch_zero_rows(BatchLaunch b, int duals)
{
    const BatchGrid& t = b.tab[blockIdx.y];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < t.g.n; i += gridDim.x * blockDim.x) {
        t.q1[i] = 0.f;
        if (duals) t.p[i] = 0.f;
    }
}

// ---- batched iterations as one persistent launch ------------------------------------
//
// Resident waves (one per workgroup, co-resident by a cooperative launch) run
// K two-set iterations over every unfinished grid: per phase (the row sweeps,
// then the column sweeps, of one iteration) the waves take the phase's work
// items in the order the hardware deals workgroups (wave b takes virtual
// workgroups b, b + waves, ..., each mapped by xcd_item), then all waves meet
// at a device-wide barrier before the next phase reads what this one wrote.
// (Claiming items from a device counter instead balances uneven items
// dynamically but serialises on the counter: slower on the 64-grid batch.)
// ctl: the barrier's arrival count and generation, an error flag and what
// the first wave that gave up saw.  The spin at a barrier is bounded: past
// kSpinLimit polls the wave sets the flag and returns, and every wave that
// sees the flag returns too, so the launch always ends.
constexpr int kCtlArrive = 2, kCtlGen = 3, kCtlErr = 4, kCtlDiag = 5;
constexpr long kSpinLimit = 1L << 22;
constexpr long kStartSpinLimit = 1L << 16;

// ctl lives in fine-grained memory and its atomics are system scope, so that
// every XCD sees one copy (ordinary device memory is kept coherent across the
// XCDs' L2 caches only at kernel boundaries)
__device__ __forceinline__ int ctl_load(int* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM); }
__device__ __forceinline__ int ctl_add(int* p, int v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void ctl_store(int* p, int v)
{
    __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// all waves of the launch past phase `phase` (-1: the start); false on a
// barrier failure
__device__ bool batch_barrier(int* ctl, int phase, long spin_limit)
{
    __threadfence();  // this wave's results before the arrival
    int ok = 1;
    if (threadIdx.x == 0) {
        const int g0 = ctl_load(ctl + kCtlGen);
        if (ctl_add(ctl + kCtlArrive, 1) == (int)gridDim.x - 1) {
            ctl_store(ctl + kCtlArrive, 0);
            __threadfence();
            ctl_add(ctl + kCtlGen, 1);
        } else {
            long spins = 0;
            while (ctl_load(ctl + kCtlGen) == g0) {
                if (ctl_load(ctl + kCtlErr) != 0 || ++spins > spin_limit) {
                    if (ctl_add(ctl + kCtlErr, 1) == 0) {
                        // the first wave to give up records where: arrivals, phase, waves
                        ctl_store(ctl + kCtlDiag, ctl_load(ctl + kCtlArrive));
                        ctl_store(ctl + kCtlDiag + 1, phase);
                        ctl_store(ctl + kCtlDiag + 2, (int)gridDim.x);
                    }
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
    }
    ok = __shfl(ok, 0);
    __threadfence();  // the other waves' results after the departure
    return ok != 0;
}

__global__ void __launch_bounds__(kLanes) k_batch_persistent(BatchLaunch b, int* ctl, int p0, int K)
{
    extern __shared__ __attribute__((aligned(16))) float lds[];
    // Every workgroup must be resident for the barriers to complete; a first
    // barrier (phase -1, short spin) checks that before any work is done.  If
    // it gives up, its arrival count is the number that were resident.
    if (!batch_barrier(ctl, -1, kStartSpinLimit)) return;
    for (int j = 0; j < K; ++j) {
        const int parity = (p0 + j) & 1;
        const bool duals = j == K - 1;
        for (int fam = 0; fam < 2; ++fam) {
            const int phase = 2 * j + fam;
            const int n_items = fam ? b.items_c : b.items_r;
            for (int v = blockIdx.x; v < n_items; v += gridDim.x) {
                const int idx = xcd_item(v, n_items);
                if (fam == 0) {
                    const int gi = b.item_grid_r[idx];
                    const BatchGrid& t = b.tab[gi];
                    if (t.done) continue;
                    if (duals) {
                        ModeRows2 m{t.z[parity], t.ax, t.q1, t.p};
                        sweep_piece<ModeRows2, true, true>(t.g, 0, idx - t.item0_r, m, t.cr, lds);
                    } else {
                        ModeRows2 m{t.z[parity], t.ax, t.q1, nullptr};
                        sweep_piece<ModeRows2, true, false>(t.g, 0, idx - t.item0_r, m, t.cr, lds);
                    }
                } else {
                    const int gi = b.item_grid_c[idx];
                    const BatchGrid& t = b.tab[gi];
                    if (t.done) continue;
                    if (duals) {
                        ModeCols2 m{t.q1, t.z[parity], t.z[parity ^ 1], t.w, t.ay, t.p + t.g.n};
                        sweep_piece<ModeCols2, false, true>(t.g, 1, idx - t.item0_c, m, t.cc, lds);
                    } else {
                        ModeCols2 m{t.q1, t.z[parity], t.z[parity ^ 1], t.w, t.ay, nullptr};
                        sweep_piece<ModeCols2, false, false>(t.g, 1, idx - t.item0_c, m, t.cc, lds);
                    }
                }
                wave_fence();  // the next item's staging overwrites this one's LDS
            }
            if (!batch_barrier(ctl, phase, kSpinLimit)) return;
        }
    }
}

}  // namespace

// Workgroups of k_batch_persistent that are resident at once (0 on error).
int batch_persistent_blocks(size_t lds)
{
    int dev = 0, per_cu = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_batch_persistent, kLanes, lds) !=
            hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return per_cu * cus / kXcds * kXcds;
}

hipError_t launch_batch_persistent(const BatchLaunch& b, int* ctl, int p0, int K, int blocks, hipStream_t s)
{
    const size_t lds = b.lds_r > b.lds_c ? b.lds_r : b.lds_c;
    BatchLaunch bb = b;
    void* args[] = {&bb, &ctl, &p0, &K};
    return hipLaunchCooperativeKernel((const void*)k_batch_persistent, dim3(blocks), dim3(kLanes), args,
                                      (unsigned)lds, s);
}

hipError_t launch_batch_iteration(const BatchLaunch& b, int parity, bool duals, hipStream_t s, bool cold)
{
    if (cold)
        hipLaunchKernelGGL(k_batch_zero_rows, dim3(64, b.n_grids), dim3(256), 0, s, b, duals ? 1 : 0);
    if (duals) {
        if (!cold) hipLaunchKernelGGL(k_batch_rows<true>, dim3(b.items_r), dim3(kLanes), b.lds_r, s, b, parity);
        hipLaunchKernelGGL(k_batch_cols<true>, dim3(b.items_c), dim3(kLanes), b.lds_c, s, b, parity);
    } else {
        if (!cold) hipLaunchKernelGGL(k_batch_rows<false>, dim3(b.items_r), dim3(kLanes), b.lds_r, s, b, parity);
        hipLaunchKernelGGL(k_batch_cols<false>, dim3(b.items_c), dim3(kLanes), b.lds_c, s, b, parity);
    }
    return hipGetLastError();
}

size_t piece_lds_bytes(const PieceCfg& cfg) { return lds_bytes(cfg); }


PieceCfg piece_config(const Geo& g, int axis, int want, int launch_items, int overlap, int tail, int min_len)
{
    // about `want` work items, pieces of min_len (8 or 16) to kMaxLen positions
    // (a work item's LDS, 2 x (reach_lo + len + reach_hi) x 65 floats, stays
    // below 64 KiB)
    constexpr int kMaxLen = 64;
    const int m = geo_extent(g, axis);
    const int groups = (geo_nchains(g, axis) + kLanes - 1) / kLanes;
    if (want < 1) want = 1;
    int pieces = (want + groups - 1) / groups;
    int len = (m + pieces - 1) / pieces;
    len = len < min_len ? min_len : ((len + min_len - 1) / min_len) * min_len;
    len = len < kMaxLen ? len : kMaxLen;
    PieceCfg cfg;
    cfg.len = len < m ? len : m;
    cfg.pieces = (m + cfg.len - 1) / cfg.len;
    const bool cut = cfg.pieces > 1;
    // With few work items (about one wave per SIMD) the slowest wave sets the
    // launch time, and one lane whose bracket fails doubles its wave's work:
    // scan from further back so that almost no piece restarts.  With many
    // work items waves overlap and the total work counts: keep the overlap
    // short and LDS small (more waves resident).
    const long items = launch_items > 0 ? launch_items : (long)groups * cfg.pieces;
    const bool latency_bound = items <= kLatencyItems;
    cfg.overlap = cut ? (overlap > 0 ? overlap : (latency_bound ? 12 : 8)) : 0;
    cfg.tail = cut ? (tail >= 0 ? tail : 8) : 0;
    // LDS: the overlap plus the weight of the edge in front of it, the piece,
    // and the tail -- plus one block of tail growth when latency bound (with
    // many work items, LDS per wave sets how many waves are resident)
    cfg.reach_lo = cut ? cfg.overlap + 1 : 0;
    cfg.reach_hi = cut ? cfg.tail + (latency_bound ? 8 : 0) : 0;
    return cfg;
}

hipError_t launch_prox(const Geo& g, int axis, const float* v, const float* a, float* x, float* p,
                       hipStream_t s)
{
    ModeProx m{v, a, x, p};
    return launch_mode(g, axis, m, p != nullptr, s);
}

hipError_t launch_dr2_rows(const Geo& g, const float* z, const float* a_x, float* q1, float* p1,
                           hipStream_t s)
{
    ModeRows2 m{z, a_x, q1, p1};
    return launch_mode(g, 0, m, p1 != nullptr, s);
}

hipError_t launch_dr2_cols(const Geo& g, const float* q1, const float* z, float* znew,
                           const float* w, const float* a_y, float* p2, hipStream_t s)
{
    ModeCols2 m{q1, z, znew, w, a_y, p2};
    return launch_mode(g, 1, m, p2 != nullptr, s);
}

hipError_t launch_drp_sweeps(const Geo& g, int nfam, const float* z, const float* const* a,
                             float* q, float* p, hipStream_t s)
{
    const size_t n = (size_t)g.n;
    ModeSweepP m0{z, a[0], q, p};
    if (nfam == 1) return launch_mode(g, 0, m0, p != nullptr, s);
    if (nfam != 2) return hipErrorInvalidValue;
    ModeSweepP m1{z + n, a[1], q + n, p ? p + n : nullptr};
    if (g.whole) {
        const hipError_t e = launch_mode(g, 0, m0, p != nullptr, s);
        return e != hipSuccess ? e : launch_mode(g, 1, m1, p != nullptr, s);
    }
    PieceCfg c0 = piece_config(g, 0, kDefaultItems, 0), c1 = piece_config(g, 1, kDefaultItems, 0);
    {
        // one launch holds both families: decide latency mode on its total
        const int tot = items_of(g, 0, c0) + items_of(g, 1, c1);
        c0 = piece_config(g, 0, kDefaultItems, tot);
        c1 = piece_config(g, 1, kDefaultItems, tot);
    }
    const int n0 = items_of(g, 0, c0), n1 = items_of(g, 1, c1);
    const size_t shm = lds_bytes(c0) > lds_bytes(c1) ? lds_bytes(c0) : lds_bytes(c1);
    if (p)
        hipLaunchKernelGGL(k_sweep_pair<true>, dim3(n0 + n1), dim3(kLanes), shm, s, g, m0, m1, c0, c1, n0);
    else
        hipLaunchKernelGGL(k_sweep_pair<false>, dim3(n0 + n1), dim3(kLanes), shm, s, g, m0, m1, c0, c1, n0);
    return hipGetLastError();
}

hipError_t launch_sweeps8(const Geo& g, const float* z, const float* const* a, float* q, float* p, const Geo& gz,
                          const float* zzv, const float* zza, float* zzx, float* zzp, hipStream_t s)
{
    if (g.whole || gz.n == 0) {
        const hipError_t e = launch_drp_sweeps(g, 2, z, a, q, p, s);
        if (e != hipSuccess || gz.n == 0) return e;
        return launch_prox(gz, 0, zzv, zza, zzx, zzp, s);
    }
    const size_t n = (size_t)g.n;
    ModeSweepP m0{z, a[0], q, p};
    ModeSweepP m1{z + n, a[1], q + n, p ? p + n : nullptr};
    ModeProx mz{zzv, zza, zzx, zzp};
    return launch_triple<ModeProx, true>(g, m0, m1, gz, 0, mz, p != nullptr, s);
}

hipError_t launch_sweeps3(const Geo& g, const float* z, const float* const* a, float* q, float* p, hipStream_t s)
{
    const size_t n = (size_t)g.n;
    ModeSweepP m2{z + 2 * n, a[2], q + 2 * n, p ? p + 2 * n : nullptr};
    if (g.whole) {
        const hipError_t e = launch_drp_sweeps(g, 2, z, a, q, p, s);
        return e != hipSuccess ? e : launch_mode(g, 2, m2, p != nullptr, s);
    }
    ModeSweepP m0{z, a[0], q, p};
    ModeSweepP m1{z + n, a[1], q + n, p ? p + n : nullptr};
    const bool probe = g.restarts != nullptr;
    if (!probe && g.stream) {  // sweeps in streamed pieces when there are enough
        const StreamCfg s0 = stream_config(g, 0), s1 = stream_config(g, 1), s2 = stream_config(g, 2);
        auto waves = [&](int axis, const StreamCfg& c) { return (geo_nchains(g, axis) + kLanes - 1) / kLanes * c.pieces; };
        const int w0 = waves(0, s0), w1 = waves(1, s1), w2 = waves(2, s2);
        if (w0 + w1 + w2 >= kStreamMinWaves) {
            if (p)
                hipLaunchKernelGGL(k_stream3<true>, dim3(w0 + w1 + w2), dim3(kLanes), stream_lds_bytes(), s, g, m0, m1,
                                   m2, s0, s1, s2, w1, w0);
            else
                hipLaunchKernelGGL(k_stream3<false>, dim3(w0 + w1 + w2), dim3(kLanes), stream_lds_bytes(), s, g, m0, m1,
                                   m2, s0, s1, s2, w1, w0);
            return hipGetLastError();
        }
    }
    return launch_triple<ModeSweepP, false>(g, m0, m1, g, 2, m2, p != nullptr, s, probe ? 0 : kVolItems,
                                            probe ? 0 : kVolOverlap, probe ? -1 : kVolTail);
}

hipError_t launch_drp_final(const Geo& g, int r, const float* z, float* znew, const float* q,
                            const float* a_last, const float* w, float* p_last, hipStream_t s)
{
    if (r == 2) {
        ModeFinalP<2> m{z, znew, q, a_last, w, p_last, g.n};
        return launch_mode(g, 1, m, p_last != nullptr, s);
    }
    if (r == 3) {
        ModeFinalP<3> m{z, znew, q, a_last, w, p_last, g.n};
        return launch_mode(g, 2, m, p_last != nullptr, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace mc
