// batch.hip -- mc_tv_solve_batched: minimum cuts of many 2D grids of uneven
// sizes at once (two-set form of the splitting, Sec. 3.3).
//
// All grids share each launch: a sweep launch covers the row (or column)
// pieces of every unfinished grid, a reduction launch the certificate terms of
// every unfinished grid, and a per-grid finalize marks a grid done on the
// device once its certificate is below the tolerance (with the iteration and
// a wall-clock stamp), after which its work items return at once.  One check
// period (an even number of iterations, the last one writing duals, then the
// certificate) is captured in a hipGraph and replayed; the host looks at the
// done flags once per replay.  With MC_BATCH_PERSISTENT a period's iterations
// run instead as one cooperative launch of resident waves with device-wide
// barriers between phases (same iterates; slower, kept as an option).
//
// The split of chains into pieces (work items per launch) is chosen on the
// first solve of a batch shape: the first iterations run with each candidate
// and the fastest is kept for this shape.  The iterates do not depend on the
// split (every piece is solved exactly), so tuning costs no extra work.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "ctx.hpp"
#include "launch.hpp"
#include "mc.h"

using namespace mc;

namespace {

constexpr size_t kAlignFloats = 64;
constexpr int kVoxelsPerRedBlock = kReduceThreads * 8;
constexpr int kMaxRedBlocksPerGrid = 256;
// Autotune candidates: work items per sweep launch (which sets the piece
// length of each grid), and the overlap the pieces scan in front of them
// (0: by launch size, 8 or 12; a short overlap saves scan work where brackets
// close early, a long one saves restarts where they close late).
struct Cand {
    int items, overlap;
};
const Cand kCandidates[] = {{2048, 0}, {4096, 0}, {8192, 0}, {16384, 0}, {2048, 4}, {4096, 4},
                            {8192, 4}, {16384, 4}, {2048, 16}, {4096, 16}, {8192, 16}, {16384, 16}};
constexpr int kNumCandidates = sizeof(kCandidates) / sizeof(kCandidates[0]);

size_t align_floats(size_t x) { return (x + kAlignFloats - 1) / kAlignFloats * kAlignFloats; }
size_t align_bytes(size_t x) { return (x + 255) / 256 * 256; }

struct Plan {
    std::vector<BatchGrid> tab;
    std::vector<int> item_r, item_c, blk;
    size_t lds_r = 0, lds_c = 0;
};

void plan_pieces(Plan& pl, const std::vector<Geo>& geos, size_t n_total, int want_total, int overlap = 0)
{
    pl.item_r.clear();
    pl.item_c.clear();
    pl.lds_r = pl.lds_c = 0;
    auto want_of = [&](const Geo& g) {
        const int w = (int)((double)want_total * (double)g.n / (double)n_total + 0.5);
        return w < 1 ? 1 : w;
    };
    // work items of each sweep launch over the whole batch (latency mode is
    // decided on those totals, not per grid)
    long tot_r = 0, tot_c = 0;
    for (const Geo& g : geos) {
        const int want = want_of(g);
        tot_r += (long)((geo_nchains(g, 0) + 63) / 64) * piece_config(g, 0, want, INT32_MAX, overlap).pieces;
        tot_c += (long)((geo_nchains(g, 1) + 63) / 64) * piece_config(g, 1, want, INT32_MAX, overlap).pieces;
    }
    const int lr = (int)std::min<long>(tot_r, INT32_MAX), lc = (int)std::min<long>(tot_c, INT32_MAX);
    for (size_t gi = 0; gi < geos.size(); ++gi) {
        const Geo& g = geos[gi];
        const int want = want_of(g);
        BatchGrid& t = pl.tab[gi];
        t.cr = piece_config(g, 0, want, lr, overlap);
        t.cc = piece_config(g, 1, want, lc, overlap);
        const int groups_r = (geo_nchains(g, 0) + 63) / 64, groups_c = (geo_nchains(g, 1) + 63) / 64;
        t.item0_r = (int)pl.item_r.size();
        pl.item_r.insert(pl.item_r.end(), (size_t)groups_r * t.cr.pieces, (int)gi);
        t.item0_c = (int)pl.item_c.size();
        pl.item_c.insert(pl.item_c.end(), (size_t)groups_c * t.cc.pieces, (int)gi);
        pl.lds_r = std::max(pl.lds_r, piece_lds_bytes(t.cr));
        pl.lds_c = std::max(pl.lds_c, piece_lds_bytes(t.cc));
    }
}

// Device metadata: a fixed header (start stamp at 0, iteration counter at 64),
// then the table, the item and block maps and the reduction partials of a plan.
constexpr size_t kHeader = 256;

size_t plan_bytes(const Plan& pl, size_t* o_ir, size_t* o_ic, size_t* o_bk, size_t* o_pa)
{
    const size_t o_tab = kHeader;
    *o_ir = align_bytes(o_tab + pl.tab.size() * sizeof(BatchGrid));
    *o_ic = align_bytes(*o_ir + pl.item_r.size() * sizeof(int));
    *o_bk = align_bytes(*o_ic + pl.item_c.size() * sizeof(int));
    *o_pa = align_bytes(*o_bk + pl.blk.size() * sizeof(int));
    return align_bytes(*o_pa + pl.blk.size() * kCertValues * sizeof(double));
}

int reserve_meta(mc_ctx* c, size_t total, hipStream_t s)
{
    if (total <= c->bmeta_cap) return MC_OK;
    MC_HIP(hipStreamSynchronize(s));
    (void)hipFree(c->bmeta);  // the old buffer is dropped either way
    c->bmeta = nullptr;
    c->bmeta_cap = 0;
    if (hipMalloc(&c->bmeta, total) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(MC_ERR_NOMEM, "batch table allocation failed");
    }
    c->bmeta_cap = total;
    return MC_OK;
}

// device copy of a plan (metadata already reserved); fills the launch descriptor
int upload(mc_ctx* c, const Plan& pl, hipStream_t s, BatchLaunch* bl, double** partials)
{
    size_t o_ir, o_ic, o_bk, o_pa;
    const size_t total = plan_bytes(pl, &o_ir, &o_ic, &o_bk, &o_pa);
    if (total > c->bmeta_cap) return set_error(MC_ERR_DEVICE, "batch metadata not reserved");
    char* b = c->bmeta;
    MC_HIP(hipMemcpyAsync(b + kHeader, pl.tab.data(), pl.tab.size() * sizeof(BatchGrid), hipMemcpyHostToDevice, s));
    MC_HIP(hipMemcpyAsync(b + o_ir, pl.item_r.data(), pl.item_r.size() * sizeof(int), hipMemcpyHostToDevice, s));
    MC_HIP(hipMemcpyAsync(b + o_ic, pl.item_c.data(), pl.item_c.size() * sizeof(int), hipMemcpyHostToDevice, s));
    MC_HIP(hipMemcpyAsync(b + o_bk, pl.blk.data(), pl.blk.size() * sizeof(int), hipMemcpyHostToDevice, s));
    // the host vectors are pageable and change with the next plan
    MC_HIP(hipStreamSynchronize(s));
    bl->tab = reinterpret_cast<BatchGrid*>(b + kHeader);
    bl->item_grid_r = reinterpret_cast<const int*>(b + o_ir);
    bl->item_grid_c = reinterpret_cast<const int*>(b + o_ic);
    bl->blk_grid = reinterpret_cast<const int*>(b + o_bk);
    bl->n_grids = (int)pl.tab.size();
    bl->items_r = (int)pl.item_r.size();
    bl->items_c = (int)pl.item_c.size();
    bl->blocks = (int)pl.blk.size();
    bl->lds_r = pl.lds_r;
    bl->lds_c = pl.lds_c;
    *partials = reinterpret_cast<double*>(b + o_pa);
    return MC_OK;
}

unsigned long long signature(const std::vector<Geo>& geos)
{
    unsigned long long h = 1469598103934665603ull;
    auto mix = [&](unsigned long long v) {
        h ^= v;
        h *= 1099511628211ull;
    };
    mix(geos.size());
    for (const Geo& g : geos) {
        mix((unsigned long long)g.H);
        mix((unsigned long long)g.W);
    }
    return h;
}

}  // namespace

extern "C" int mc_tv_solve_batched(mc_ctx* c, int n_grids, const mc_grid* grids,
                                   const float* const* w, const float* const* a,
                                   uint8_t* const* labels, float* const* x_out, float* const* z_out,
                                   mc_stats* stats, const mc_opts* opts_in, void* stream)
{
    if (!c) return set_error(MC_ERR_INVALID_ARG, "ctx is null");
    MC_HIP(hipSetDevice(c->device));
    if (n_grids < 1 || !grids || !w || !a || !labels || !stats)
        return set_error(MC_ERR_INVALID_ARG, "null argument or n_grids < 1");
    mc_opts o;
    if (opts_in) o = *opts_in; else mc_opts_default(&o);
    if (o.max_iters < 1 || o.check_every < 1) return set_error(MC_ERR_INVALID_ARG, "max_iters and check_every must be >= 1");
    if (o.variant == MC_VARIANT_PRODUCT) return set_error(MC_ERR_INVALID_ARG, "batched solves use the two-set form");
    const int K = (o.check_every + 1) / 2 * 2;  // iterations per replay, even: the state parity repeats
    // (the state after it iterations is z[it & 1]; iteration it + 1 reads it)

    std::vector<Geo> geos((size_t)n_grids);
    size_t n_total = 0, floats = 0;
    for (int gi = 0; gi < n_grids; ++gi) {
        const mc_grid& gr = grids[gi];
        if (gr.conn != 0 && gr.conn != 4)
            return set_error(MC_ERR_INVALID_ARG, "batched grids are 4-connected");
        if (gr.ndim != 2 || gr.dims[0] <= 0 || gr.dims[1] <= 0)
            return set_error(MC_ERR_INVALID_ARG, "batched grids must be 2D with positive dims");
        if (gr.dims[0] * gr.dims[1] > kMaxNodes || gr.dims[0] >= (1 << 30) || gr.dims[1] >= (1 << 30))
            return set_error(MC_ERR_INVALID_ARG, "grid too large");
        if (!w[gi] || !a[2 * gi] || !a[2 * gi + 1] || !labels[gi])
            return set_error(MC_ERR_INVALID_ARG, "null array for a grid");
        Geo& g = geos[gi];
        g.D = 1;
        g.H = (int)gr.dims[0];
        g.W = (int)gr.dims[1];
        g.n = g.H * g.W;
        g.ndim = 2;
        n_total += (size_t)g.n;
        floats += 6 * align_floats((size_t)g.n);
    }
    hipStream_t us = (hipStream_t)stream;
    hipStream_t s = c->bstream;
    if (floats > c->bcap) {
        MC_HIP(hipDeviceSynchronize());
        (void)hipFree(c->bbuf);  // the old buffer is dropped either way
        c->bbuf = nullptr;
        c->bcap = 0;
        if (hipMalloc(&c->bbuf, floats * sizeof(float)) != hipSuccess) {
            (void)hipGetLastError();
            return set_error(MC_ERR_NOMEM, "batch workspace allocation failed");
        }
        c->bcap = floats;
    }

    // per-grid table, reduction blocks
    Plan pl;
    pl.tab.resize((size_t)n_grids);
    size_t off = 0;
    for (int gi = 0; gi < n_grids; ++gi) {
        BatchGrid& t = pl.tab[gi];
        memset(&t, 0, sizeof(t));
        const Geo& g = geos[gi];
        const size_t na = align_floats((size_t)g.n);
        t.g = g;
        t.w = w[gi];
        t.ax = a[2 * gi];
        t.ay = a[2 * gi + 1];
        t.z[0] = c->bbuf + off;
        t.z[1] = c->bbuf + off + na;
        t.q1 = c->bbuf + off + 2 * na;
        t.p = c->bbuf + off + 3 * na;  // 2 * na: row duals at p, column duals at p + n
        t.xc = c->bbuf + off + 5 * na;
        off += 6 * na;
        t.labels = labels[gi];
        t.x_out = x_out ? x_out[gi] : nullptr;
        int nb = (g.n + kVoxelsPerRedBlock - 1) / kVoxelsPerRedBlock;
        nb = std::max(1, std::min(nb, kMaxRedBlocksPerGrid));
        t.blk0 = (int)pl.blk.size();
        t.nblk = nb;
        pl.blk.insert(pl.blk.end(), (size_t)nb, gi);
    }

    // start after the caller's pending work
    hipEvent_t ev_in = c->ev0, ev_out = c->ev1;
    MC_HIP(hipEventRecord(ev_in, us));
    MC_HIP(hipStreamWaitEvent(s, ev_in, 0));
    for (int gi = 0; gi < n_grids; ++gi)
        MC_HIP(hipMemsetAsync(pl.tab[gi].z[0], 0, sizeof(float) * (size_t)geos[gi].n, s));

    const unsigned long long sig = signature(geos);
    int items = o.batch_items > 0 ? o.batch_items : 0, overlap = 0;
    auto it_tuned = c->tuned_items.find(sig);
    if (items == 0 && it_tuned != c->tuned_items.end()) {
        items = it_tuned->second.first;
        overlap = it_tuned->second.second;
    }

    // metadata for the largest plan that may be used, header first
    std::vector<Cand> cands;
    if (items == 0) cands.assign(kCandidates, kCandidates + kNumCandidates);
    else cands.push_back({items, overlap});
    size_t need = 0;
    for (const Cand& cand : cands) {
        plan_pieces(pl, geos, n_total, cand.items, cand.overlap);
        size_t a1, a2, a3, a4;
        need = std::max(need, plan_bytes(pl, &a1, &a2, &a3, &a4));
    }
    int rc;
    if ((rc = reserve_meta(c, need, s))) return rc;
    unsigned long long* t0_dev = reinterpret_cast<unsigned long long*>(c->bmeta);
    int* iter_dev = reinterpret_cast<int*>(c->bmeta + 64);
    MC_HIP(launch_stamp(t0_dev, s));

    BatchLaunch bl;
    double* partials = nullptr;
    int it = 0;  // iterations done
    // The first iteration from z = 0 (row proxes 0), on the plan of the first
    // candidate; it is not timed by the autotuner (it sweeps only the
    // columns).  The iterations before the replays leave at least one for
    // the last check.
    if (o.max_iters > 1) {
        if (items > 0) plan_pieces(pl, geos, n_total, items, overlap);
        else plan_pieces(pl, geos, n_total, kCandidates[0].items, kCandidates[0].overlap);
        if ((rc = upload(c, pl, s, &bl, &partials))) return rc;
        MC_HIP(launch_batch_iteration(bl, 0, false, s, true));
        ++it;
    }
    if (items == 0) {
        // autotune on the first iterations of the solve itself
        float best_ms = INFINITY;
        Cand best = kCandidates[0];
        for (int k = 0; k < kNumCandidates && it + 1 < o.max_iters; ++k) {
            plan_pieces(pl, geos, n_total, kCandidates[k].items, kCandidates[k].overlap);
            if ((rc = upload(c, pl, s, &bl, &partials))) return rc;
            MC_HIP(hipEventRecord(c->ev0, s));
            MC_HIP(launch_batch_iteration(bl, it & 1, false, s));
            MC_HIP(hipEventRecord(c->ev1, s));
            MC_HIP(hipEventSynchronize(c->ev1));
            float ms = 0.f;
            MC_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
            if (ms < best_ms) {
                best_ms = ms;
                best = kCandidates[k];
            }
            ++it;
        }
        items = best.items;
        overlap = best.overlap;
        if (best_ms < INFINITY) c->tuned_items[sig] = {items, overlap};  // (no candidate timed: nothing learnt)
    } else {
        // as many iterations as the autotuner runs, so that every call checks
        // at the same iterations (and reports the same results) whether it
        // tuned or not
        for (int k = 0; k < kNumCandidates && it + 1 < o.max_iters; ++k) {
            MC_HIP(launch_batch_iteration(bl, it & 1, false, s));
            ++it;
        }
    }
    plan_pieces(pl, geos, n_total, items, overlap);
    if ((rc = upload(c, pl, s, &bl, &partials))) return rc;
    // checks at multiples of K, as mc_tv_solve checks at multiples of check_every
    for (; it % K != 0 && it + 1 < o.max_iters; ++it) MC_HIP(launch_batch_iteration(bl, it & 1, false, s));

    // One check period: K iterations from the current state parity, the last
    // with duals, then the certificate -- a captured graph of per-phase
    // launches, or (MC_BATCH_PERSISTENT) one persistent launch for the
    // iterations and the certificate launches after it.
    const int p0 = it & 1;
    const bool persistent = (o.flags & MC_BATCH_PERSISTENT) != 0;
    int* ctl = c->bctl;
    int blocks = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    if (persistent) {
        // The control words are shared by waves on every XCD: in fine-grained
        // memory, whose atomics are coherent across the XCDs' L2 caches (the
        // default coarse-grained memory is coherent across XCDs only at
        // kernel boundaries).
        if (!c->bctl) {
            MC_HIP(hipStreamSynchronize(s));
            if (hipExtMallocWithFlags((void**)&c->bctl, 64, hipDeviceMallocFinegrained) != hipSuccess) {
                (void)hipGetLastError();
                c->bctl = nullptr;
                return set_error(MC_ERR_NOMEM, "persistent batch control allocation failed");
            }
        }
        ctl = c->bctl;
        const size_t lds = std::max(bl.lds_r, bl.lds_c);
        const auto f = c->persist_blocks.find(lds);
        blocks = f != c->persist_blocks.end() ? f->second : batch_persistent_blocks(lds);  // (verified below)
        if (blocks < 1) return set_error(MC_ERR_DEVICE, "no resident workgroups for the persistent batch launch");
    } else {
        MC_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        hipError_t cap = hipSuccess;
        for (int j = 0; j < K && cap == hipSuccess; ++j)
            cap = launch_batch_iteration(bl, (p0 + j) & 1, j == K - 1, s);
        if (cap == hipSuccess) cap = launch_batch_check(bl, o.tau0, o.gap_tol, iter_dev, partials, s);
        hipError_t endc = hipStreamEndCapture(s, &graph);
        if (cap != hipSuccess) return hip_error(cap, "batch graph capture");
        if (endc != hipSuccess) return hip_error(endc, "hipStreamEndCapture");
        MC_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    }
    int ctl_h[8] = {0};
    const size_t lds_p = std::max(bl.lds_r, bl.lds_c);
    auto period = [&]() -> hipError_t {
        hipError_t e = launch_set_int(iter_dev, it + K, s);
        if (e != hipSuccess) return e;
        if (!persistent) return hipGraphLaunch(exec, s);
        // The occupancy query can promise more resident workgroups than run
        // at once; the kernel's first barrier finds out before any work.  The
        // first launch with a workgroup count waits for its verdict, and a
        // launch whose workgroups were not all resident is repeated with as
        // many as were (the count that works is remembered).
        for (;;) {
            const auto f = c->persist_blocks.find(lds_p);
            const bool verified = f != c->persist_blocks.end() && f->second == blocks;
            if ((e = hipMemsetAsync(ctl, 0, 8 * sizeof(int), s)) != hipSuccess) return e;
            if ((e = launch_batch_persistent(bl, ctl, p0, K, blocks, s)) != hipSuccess) return e;
            if (verified) break;
            if ((e = hipMemcpyAsync(ctl_h, ctl, sizeof(ctl_h), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
            if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
            if (ctl_h[4] && ctl_h[6] == -1 && ctl_h[5] >= 8 && ctl_h[5] < blocks) {
                blocks = ctl_h[5] / 8 * 8;
                continue;
            }
            if (!ctl_h[4]) c->persist_blocks[lds_p] = blocks;
            break;
        }
        if ((e = launch_batch_check(bl, o.tau0, o.gap_tol, iter_dev, partials, s)) != hipSuccess) return e;
        return hipMemcpyAsync(ctl_h, ctl, sizeof(ctl_h), hipMemcpyDeviceToHost, s);  // read by read_done
    };
    std::vector<BatchGrid> host_tab((size_t)n_grids);
    bool all_done = false;
    int graph_err = MC_OK;
    auto read_done = [&]() -> int {
        if (hipMemcpyAsync(host_tab.data(), bl.tab, host_tab.size() * sizeof(BatchGrid), hipMemcpyDeviceToHost,
                           s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return hip_error(hipGetLastError(), "batch status read");
        if (ctl_h[4])
            return set_error(MC_ERR_DEVICE, "persistent batch launch: a device-wide barrier timed out (" +
                                                std::to_string(ctl_h[5]) + " of " + std::to_string(ctl_h[7]) +
                                                " workgroups arrived, phase " + std::to_string(ctl_h[6]) + ")");
        all_done = true;
        for (const BatchGrid& t : host_tab) all_done = all_done && t.done;
        return MC_OK;
    };
    if (persistent) {
        while (it + K <= o.max_iters && !all_done) {
            const hipError_t e = period();
            if (e != hipSuccess) {
                graph_err = hip_error(e, "persistent batch launch");
                break;
            }
            it += K;
            if ((graph_err = read_done())) break;
        }
    } else {
        // Graph replays: each is followed by a count of the grids not done,
        // copied to pinned memory behind an event of its own, and the host
        // waits for a count only once the next replay is queued, so that the
        // device does not idle while it reads.  Queuing never passes
        // max_iters; behind the replay that finishes the last grid at most
        // one more runs, in which the finished grids exit at once.
        int* undone_dev = reinterpret_cast<int*>(c->bmeta + 128);
        int* undone_h = reinterpret_cast<int*>(c->hout);
        hipEvent_t ev[2] = {nullptr, nullptr};
        for (int k = 0; k < 2 && !graph_err; ++k) {
            const hipError_t e = hipEventCreateWithFlags(&ev[k], hipEventDisableTiming);
            if (e != hipSuccess) graph_err = hip_error(e, "hipEventCreateWithFlags");
        }
        int queued = 0, wr = 0, rd = 0;
        while (!graph_err && !all_done) {
            while (queued < 2 && it + K <= o.max_iters) {
                hipError_t e = period();
                if (e == hipSuccess) e = launch_batch_undone(bl, undone_dev + wr, s);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(undone_h + wr, undone_dev + wr, sizeof(int), hipMemcpyDeviceToHost, s);
                if (e == hipSuccess) e = hipEventRecord(ev[wr], s);
                if (e != hipSuccess) {
                    graph_err = hip_error(e, "batch graph replay");
                    break;
                }
                it += K;
                wr ^= 1;
                ++queued;
            }
            if (graph_err || queued == 0) break;
            const hipError_t e = hipEventSynchronize(ev[rd]);
            if (e != hipSuccess) {
                graph_err = hip_error(e, "batch status wait");
                break;
            }
            all_done = undone_h[rd] == 0;
            rd ^= 1;
            --queued;
        }
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        if (!graph_err) graph_err = read_done();  // the table after the last replay
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (graph_err) return graph_err;
    // the iterations left below a whole period, the last with duals, then the
    // last check (every solve ends on a check: each grid gets a certificate
    // and a primal to label)
    if (!all_done && it < o.max_iters) {
        for (; it < o.max_iters; ++it)
            MC_HIP(launch_batch_iteration(bl, it & 1, it + 1 == o.max_iters, s, it == 0));
        MC_HIP(launch_set_int(iter_dev, it, s));
        MC_HIP(launch_batch_check(bl, o.tau0, o.gap_tol, iter_dev, partials, s));
        if ((rc = read_done())) return rc;
    }

    MC_HIP(launch_batch_labels(bl, o.tau0, s));
    if (z_out) {
        // each grid's state after its last check (a certified grid stops iterating)
        for (int gi = 0; gi < n_grids; ++gi) {
            if (!z_out[gi]) continue;
            const BatchGrid& t = host_tab[gi];
            MC_HIP(hipMemcpyAsync(z_out[gi], t.z[t.iters & 1], sizeof(float) * (size_t)t.g.n,
                                  hipMemcpyDeviceToDevice, s));
        }
    }
    unsigned long long t0 = 0;
    MC_HIP(hipMemcpyAsync(host_tab.data(), bl.tab, host_tab.size() * sizeof(BatchGrid), hipMemcpyDeviceToHost, s));
    MC_HIP(hipMemcpyAsync(&t0, t0_dev, sizeof(t0), hipMemcpyDeviceToHost, s));
    unsigned long long t_end = 0;
    MC_HIP(hipStreamSynchronize(s));
    {
        // end stamp for grids that did not converge
        MC_HIP(launch_stamp(t0_dev, s));
        MC_HIP(hipMemcpyAsync(&t_end, t0_dev, sizeof(t_end), hipMemcpyDeviceToHost, s));
        MC_HIP(hipStreamSynchronize(s));
    }
    int rate_khz = 0;
    MC_HIP(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, c->device));
    float taus[kNumTau];
    tau_ladder(o.tau0, taus);
    bool ok = true;
    for (int gi = 0; gi < n_grids; ++gi) {
        const BatchGrid& t = host_tab[gi];
        mc_stats& st = stats[gi];
        memset(&st, 0, sizeof(st));
        st.status = t.done ? MC_OK : MC_NOT_CONVERGED;
        ok = ok && t.done;
        st.iters = t.iters;
        st.cert_gap = t.checks ? t.cert : INFINITY;
        st.energy = t.checks ? t.e[t.tau_idx] : INFINITY;
        st.lower_bound = t.lb;
        st.tv_gap = t.tvgap;
        st.tau_used = taus[t.tau_idx];
        const unsigned long long tend = t.done ? t.t_done : t_end;
        st.ms = rate_khz > 0 ? (float)((double)(tend - t0) / (double)rate_khz) : 0.f;
        st.checks = t.checks;
        st.items = items;
        if (t.checks && !isfinite(t.cert)) return set_error(MC_ERR_NUMERIC, "non-finite certificate in a batched grid");
    }
    MC_HIP(hipEventRecord(ev_out, s));
    MC_HIP(hipStreamWaitEvent(us, ev_out, 0));
    return ok ? MC_OK : MC_NOT_CONVERGED;
}
