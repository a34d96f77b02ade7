// api.hip -- the C ABI declared in include/mc.h: contexts, workspace,
// argument checks and the host loop of the splitting method.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "ctx.hpp"
#include "launch.hpp"
#include "mc.h"

using namespace mc;

namespace mc {

thread_local std::string g_last_error;

int set_error(int code, const std::string& msg)
{
    g_last_error = msg;
    return code;
}

int make_geo(const mc_grid* grid, Geo* g)
{
    if (!grid) return set_error(MC_ERR_INVALID_ARG, "grid is null");
    int64_t D, H, W;
    if (grid->ndim == 2) {
        D = 1; H = grid->dims[0]; W = grid->dims[1];
    } else if (grid->ndim == 3) {
        D = grid->dims[0]; H = grid->dims[1]; W = grid->dims[2];
    } else {
        return set_error(MC_ERR_INVALID_ARG, "ndim must be 2 or 3");
    }
    if (D <= 0 || H <= 0 || W <= 0) return set_error(MC_ERR_INVALID_ARG, "dims must be positive");
    const int64_t n = D * H * W;
    if (n > kMaxNodes || D > INT32_MAX || H > INT32_MAX || W > INT32_MAX)
        return set_error(MC_ERR_INVALID_ARG, "grid has more than 2^31 - 2^24 nodes");
    if (W >= (1 << 30) || H >= (1 << 30) || D >= (1 << 30))
        return set_error(MC_ERR_INVALID_ARG, "chain length must be below 2^30");
    g->D = (int)D; g->H = (int)H; g->W = (int)W;
    g->n = (int)n;
    g->ndim = grid->ndim;
    if (grid->conn != 0 && grid->conn != 4 && grid->conn != 6 && grid->conn != 8)
        return set_error(MC_ERR_INVALID_ARG, "conn must be 0, 4, 6 or 8");
    if (grid->conn == 8 && grid->ndim != 2) return set_error(MC_ERR_INVALID_ARG, "8-connected grids are 2D");
    return MC_OK;
}

int check_ctx(mc_ctx* c)
{
    if (!c) return set_error(MC_ERR_INVALID_ARG, "ctx is null");
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_error(e, "hipSetDevice");
    return MC_OK;
}

}  // namespace mc

namespace {

int fail(int code, const std::string& msg) { return set_error(code, msg); }

int hip_fail(hipError_t e, const char* where) { return hip_error(e, where); }

void free_ws(mc_ctx* c)
{
    // release errors are not actionable here; the pointers are dropped either way
    for (float* q : {c->z, c->z2, c->y, c->p, c->xt}) (void)hipFree(q);
    c->z = c->z2 = c->y = c->p = c->xt = nullptr;
    c->cap_n = 0;
    c->cap_r = 0;
}

int ensure_ws(mc_ctx* c, size_t n, int r)
{
    if (c->cap_n >= n && c->cap_r >= r && c->z) return MC_OK;
    size_t nn = n > c->cap_n ? n : c->cap_n;
    int rr = r > c->cap_r ? r : c->cap_r;
    free_ws(c);
    const size_t fb = sizeof(float);
    const int ry = rr;  // prox outputs q_j of every family (product space)
    if (hipMalloc(&c->z, fb * nn * rr) != hipSuccess || hipMalloc(&c->z2, fb * nn * rr) != hipSuccess ||
        hipMalloc(&c->y, fb * nn * ry) != hipSuccess || hipMalloc(&c->p, fb * nn * rr) != hipSuccess ||
        hipMalloc(&c->xt, fb * nn) != hipSuccess) {
        free_ws(c);
        (void)hipGetLastError();
        return fail(MC_ERR_NOMEM, "workspace allocation failed");
    }
    c->cap_n = nn;
    c->cap_r = rr;
    return MC_OK;
}

// Device buffers of one single-grid solve: the context's workspace, or the
// static scratch array of mc_tv_solve_noalloc.
struct SolveWs {
    float* z;          // splitting state (n two-set, r*n product space)
    float* z2;         // next state
    float* y;          // prox outputs: q1 (two-set) or q_j (r*n)
    float* p;          // r*n edge duals of check iterations
    float* xt;         // n primal estimate
    double* partials;  // kReduceBlocks * kCertValues
    double* dout;      // kCertValues
    int* scnt;         // 2 counters of the sweep-kind probe
};

SolveWs ctx_ws(mc_ctx* c) { return {c->z, c->z2, c->y, c->p, c->xt, c->partials, c->dout, c->scnt}; }

// Counts the chain-sweep launches; with MC_PROFILE also brackets each with a
// pair of events from a pool, drained at every synchronisation point of the
// solve.  (An event record costs a few microseconds of stream time.)
struct SweepTimer {
    mc_ctx* c;
    bool on;
    size_t used = 0;
    double ms = 0.0, dual_ms = 0.0;
    int launches = 0, dual_launches = 0;
    bool cur_dual = false;
    std::vector<uint8_t> tags;  // per timed launch: 1 when it also wrote edge duals
    // dual: the launch also writes the edge duals (a certificate iteration)
    hipError_t begin(hipStream_t s, bool dual = false)
    {
        cur_dual = dual;
        if (!on) return hipSuccess;
        if (used + 2 > c->prof_ev.size()) {
            for (int k = 0; k < 2; ++k) {
                hipEvent_t e;
                hipError_t r = hipEventCreate(&e);
                if (r != hipSuccess) return r;
                c->prof_ev.push_back(e);
            }
        }
        return hipEventRecord(c->prof_ev[used], s);
    }
    hipError_t end(hipStream_t s)
    {
        ++launches;
        if (cur_dual) ++dual_launches;
        if (!on) return hipSuccess;
        hipError_t r = hipEventRecord(c->prof_ev[used + 1], s);
        used += 2;
        tags.push_back(cur_dual ? 1 : 0);
        return r;
    }
    // call after the stream has been synchronised
    hipError_t drain()
    {
        for (size_t k = 0; k < used; k += 2) {
            float t = 0.f;
            hipError_t r = hipEventElapsedTime(&t, c->prof_ev[k], c->prof_ev[k + 1]);
            if (r != hipSuccess) return r;
            ms += t;
            if (tags[k / 2]) dual_ms += t;
        }
        used = 0;
        tags.clear();
        return hipSuccess;
    }
};


// ---- shared by the solve loops ----------------------------------------------------

// Choice of the sweep kind when neither MC_WHOLE_CHAINS nor MC_PIECE_CHAINS is
// set: the first sweeps of the solve run as pieces and count their lanes and
// the lanes whose bracket did not close (they restarted further back).  When
// that is 1 in 10 or more, the chain proxes have long constant segments and
// the rest of the solve sweeps whole chains.  One extra synchronisation.
struct SweepProbe {
    mc_ctx* c;
    int* cnt;
    Geo& g;
    hipStream_t s;
    bool on;
    SweepProbe(mc_ctx* c_, const SolveWs& ws, Geo& g_, const mc_opts& o, hipStream_t s_)
        : c(c_), cnt(ws.scnt), g(g_), s(s_), on(!(o.flags & (MC_WHOLE_CHAINS | MC_PIECE_CHAINS)))
    {
    }
    int start()
    {
        if (!on) return MC_OK;
        MC_HIP(hipMemsetAsync(cnt, 0, 2 * sizeof(int), s));
        g.restarts = cnt;
        return MC_OK;
    }
    // after each iteration: decide once the first sweeps have run
    int after_iteration(int launches)
    {
        if (!on || launches == 0) return MC_OK;
        MC_HIP(hipMemcpyAsync(c->scnt_h, cnt, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
        MC_HIP(hipStreamSynchronize(s));
        on = false;
        g.restarts = nullptr;
        if (c->scnt_h[0] > 0 && 10ll * c->scnt_h[0] >= (long long)c->scnt_h[1]) g.whole = 1;
        return MC_OK;
    }
};

struct CheckState {
    double cert = INFINITY, energy = INFINITY, lb = -INFINITY, tvgap = NAN;
    float tau_used = 0.f;
    int checks = 0;
    bool ev1_recorded = false;  // ev1 marks the end of the last check
};

// Certificate from the edge duals pj (Sec. 2.2): energies of the threshold
// ladder, LB, TV gap, copied to the host; ev1 is recorded behind the copy.
int enqueue_check(mc_ctx* c, const SolveWs& ws, const Geo& g, bool conn8, const float* w, const float* const* a,
                  const float* const* pj, const mc_opts& o, hipStream_t s, CheckState& st)
{
    ++st.checks;
    if (conn8) MC_HIP(launch_cert8(g, w, a, pj, o.tau0, ws.xt, ws.partials, ws.dout, s));
    else MC_HIP(launch_cert(g, w, a, pj, o.tau0, ws.xt, ws.partials, ws.dout, s));
    MC_HIP(hipMemcpyAsync(c->hout, ws.dout, kCertValues * sizeof(double), hipMemcpyDeviceToHost, s));
    MC_HIP(hipEventRecord(c->ev1, s));
    st.ev1_recorded = true;
    return MC_OK;
}

// Waits for the last enqueued check and reads it; `done` when cert < gap_tol.
int read_check(mc_ctx* c, const mc_opts& o, const float* taus, SweepTimer& tm, CheckState& st, bool& done)
{
    MC_HIP(hipEventSynchronize(c->ev1));
    MC_HIP(tm.drain());
    st.energy = INFINITY;
    for (int k = 0; k < kNumTau; ++k) {
        if (c->hout[k] < st.energy) {
            st.energy = c->hout[k];
            st.tau_used = taus[k];
        }
    }
    st.tvgap = c->hout[kNumTau];
    st.lb = c->hout[kNumTau + 1];
    st.cert = st.energy - st.lb;
    if (!isfinite(st.cert)) return fail(MC_ERR_NUMERIC, "non-finite certificate (NaN/Inf in the state)");
    done = st.cert < o.gap_tol;
    return MC_OK;
}

// A check read at once.
int run_check(mc_ctx* c, const SolveWs& ws, const Geo& g, bool conn8, const float* w, const float* const* a,
              const float* const* pj, const mc_opts& o, const float* taus, SweepTimer& tm, hipStream_t s,
              CheckState& st, bool& done)
{
    int rc;
    if ((rc = enqueue_check(c, ws, g, conn8, w, a, pj, o, s, st))) return rc;
    return read_check(c, o, taus, tm, st, done);
}

// MC_DEBUG: the state after iteration `it` holds no NaN/Inf.
int debug_state(mc_ctx* c, const SolveWs& ws, const float* z, size_t nz, int it, hipStream_t s)
{
    MC_HIP(launch_count_nonfinite(z, (int)nz, ws.partials, ws.dout, s));
    MC_HIP(hipMemcpyAsync(c->hout, ws.dout, sizeof(double), hipMemcpyDeviceToHost, s));
    MC_HIP(hipStreamSynchronize(s));
    if (c->hout[0] > 0)
        return fail(MC_ERR_NUMERIC, "MC_DEBUG: " + std::to_string((long long)c->hout[0]) +
                                        " non-finite state values after iteration " + std::to_string(it));
    return MC_OK;
}

// MC_DEBUG: the edge duals of check iteration `it` lie in their boxes and
// vanish where no edge exists.
int debug_duals(mc_ctx* c, const SolveWs& ws, const Geo& g, const float* const* a, const float* const* pj, int it,
                hipStream_t s)
{
    MC_HIP(launch_debug_duals(g, a, pj, ws.partials, ws.dout, s));
    MC_HIP(hipMemcpyAsync(c->hout, ws.dout, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    MC_HIP(hipStreamSynchronize(s));
    if (c->hout[0] > 0 || c->hout[1] > 0)
        return fail(MC_ERR_NUMERIC, "MC_DEBUG: iteration " + std::to_string(it) + ": " +
                                        std::to_string((long long)c->hout[0]) + " edge duals outside |p| <= a, " +
                                        std::to_string((long long)c->hout[1]) + " non-zero on a last slice");
    return MC_OK;
}

// Labels of the last certificate's primal, optional outputs, stats.
int finish_solve(mc_ctx* c, const SolveWs& ws, const Geo& g, const float* state, size_t nstate, float* x_out,
                 uint8_t* labels_out, float* z_out, mc_stats* stats, int it, bool converged, const CheckState& st,
                 SweepTimer& tm, hipStream_t s)
{
    const size_t n = (size_t)g.n;
    if (!st.ev1_recorded) MC_HIP(hipEventRecord(c->ev1, s));
    MC_HIP(launch_labels(g, ws.xt, st.tau_used, labels_out, s));
    if (x_out) MC_HIP(hipMemcpyAsync(x_out, ws.xt, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
    if (z_out) MC_HIP(hipMemcpyAsync(z_out, state, sizeof(float) * nstate, hipMemcpyDeviceToDevice, s));
    MC_HIP(hipStreamSynchronize(s));
    float ms = 0.f;
    MC_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    stats->status = converged ? MC_OK : MC_NOT_CONVERGED;
    stats->iters = it;
    stats->cert_gap = st.cert;
    stats->energy = st.energy;
    stats->lower_bound = st.lb;
    stats->tv_gap = st.tvgap;
    stats->tau_used = st.tau_used;
    stats->ms = ms;
    MC_HIP(tm.drain());
    stats->sweep_ms = tm.ms;
    stats->sweep_launches = tm.launches;
    stats->dual_sweep_ms = tm.dual_ms;
    stats->dual_sweep_launches = tm.dual_launches;
    stats->checks = st.checks;
    stats->items = 0;
    stats->whole_chains = g.whole;
    return stats->status;
}

// Cyclic projections (BCD), alternating projections in the product space and
// FISTA on the dual (Sec. 4.1-4.2) over the same chain proxes; 4- and
// 6-connected grids.  State (z0 / z_out): the dual blocks y (BCD, FISTA) or
// the point l projected onto K (AP), r*n floats.
int solve_variant(mc_ctx* c, const Geo& g0, const float* w, const float* const* a, const float* z0, float* x_out,
                  uint8_t* labels_out, float* z_out, mc_stats* stats, const mc_opts& o, hipStream_t s)
{
    Geo g = g0;  // the sweep kind may change after the first sweeps
    const int r = g.ndim;
    const size_t n = (size_t)g.n;
    int rc;
    if ((rc = ensure_ws(c, n, r))) return rc;
    // buffers: A (r n), B (r n), V (r n), X (n)
    const size_t need = 3 * (size_t)r * n + n;
    if (need > c->vcap) {
        (void)hipFree(c->vbuf);
        c->vbuf = nullptr;
        c->vcap = 0;
        if (hipMalloc(&c->vbuf, sizeof(float) * need) != hipSuccess) {
            (void)hipGetLastError();
            return fail(MC_ERR_NOMEM, "variant workspace allocation failed");
        }
        c->vcap = need;
    }
    float* A = c->vbuf;
    float* B = A + r * n;
    float* V = B + r * n;
    float* X = V + r * n;
    if (o.flags & MC_VALIDATE) {
        MC_HIP(launch_validate(g, w, a, c->partials, c->dout, s));
        MC_HIP(hipMemcpyAsync(c->hout, c->dout, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        MC_HIP(hipStreamSynchronize(s));
        if (c->hout[1] > 0) return fail(MC_ERR_NONFINITE, "non-finite value in w or a");
        if (c->hout[0] > 0) return fail(MC_ERR_NEGATIVE_WEIGHT, "negative weight or non-zero weight on a last slice");
    }
    if (z0) MC_HIP(hipMemcpyAsync(A, z0, sizeof(float) * r * n, hipMemcpyDeviceToDevice, s));
    else MC_HIP(hipMemsetAsync(A, 0, sizeof(float) * r * n, s));
    if (o.variant == MC_VARIANT_FISTA) MC_HIP(hipMemcpyAsync(B, A, sizeof(float) * r * n, hipMemcpyDeviceToDevice, s));
    if (o.variant == MC_VARIANT_BCD) {
        // x = u - sum_j y_j
        MC_HIP(launch_neg(n, w, X, s));
        for (int j = 0; j < r; ++j) MC_HIP(launch_sub(n, A + (size_t)j * n, X, s));
    }
    MC_HIP(hipEventRecord(c->ev0, s));

    const float* pj[3] = {c->p, c->p + n, c->p + 2 * n};
    SweepTimer tm{c, (o.flags & MC_PROFILE) != 0};
    float taus[kNumTau];
    tau_ladder(o.tau0, taus);
    CheckState st;
    int it = 0;
    bool converged = false;
    double t = 1.0;
    float* y = A;   // FISTA: current y, B: previous
    float* yp = B;
    const SolveWs ws = ctx_ws(c);
    SweepProbe probe(c, ws, g, o, s);
    if ((rc = probe.start())) return rc;
    while (it < o.max_iters) {
        ++it;
        const bool check = (it % o.check_every == 0) || it == o.max_iters;
        if (o.variant == MC_VARIANT_BCD) {
            for (int i = 0; i < r; ++i) {
                float* yi = A + (size_t)i * n;
                MC_HIP(launch_add(n, X, yi, V, s));
                MC_HIP(tm.begin(s));
                MC_HIP(launch_prox(g, i, V, a[i], X, check ? c->p + (size_t)i * n : nullptr, s));
                MC_HIP(tm.end(s));
                MC_HIP(launch_diff(n, V, X, yi, s));
            }
        } else if (o.variant == MC_VARIANT_AP) {
            const bool cold = it == 1 && !z0;
            if (cold) {
                if (check) MC_HIP(hipMemsetAsync(c->p, 0, sizeof(float) * r * n, s));
            } else {
                for (int j = 0; j < r; ++j) {
                    MC_HIP(tm.begin(s));
                    MC_HIP(launch_prox(g, j, A + (size_t)j * n, a[j], V + (size_t)j * n,
                                       check ? c->p + (size_t)j * n : nullptr, s));
                    MC_HIP(tm.end(s));
                }
            }
            MC_HIP(launch_ap_update(n, r, A, V, w, cold, s));
        } else {  // FISTA
            const double t_next = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
            const float beta = (float)((t - 1.0) / t_next);
            t = t_next;
            MC_HIP(launch_fista_pre(n, r, y, yp, beta, w, V, s));
            for (int j = 0; j < r; ++j) {
                MC_HIP(tm.begin(s));
                MC_HIP(launch_prox(g, j, V + (size_t)j * n, a[j], yp + (size_t)j * n,
                                   check ? c->p + (size_t)j * n : nullptr, s));
                MC_HIP(tm.end(s));
            }
            MC_HIP(launch_rsub((size_t)r * n, V, yp, s));  // new y = v - prox(v), into the old buffer
            float* tmp = y;
            y = yp;
            yp = tmp;
        }
        if ((rc = probe.after_iteration(tm.launches))) return rc;
        if (!check) continue;
        bool done = false;
        if ((rc = run_check(c, ws, g, false, w, a, pj, o, taus, tm, s, st, done))) return rc;
        if (done) {
            converged = true;
            break;
        }
    }
    const float* state = o.variant == MC_VARIANT_FISTA ? y : A;
    return finish_solve(c, ws, g, state, (size_t)r * n, x_out, labels_out, z_out, stats, it, converged, st, tm, s);
}

// 8-connected 2D grids: product-space splitting over rows, columns and the
// two zig-zag families (Sec. 3.1, 4.3), certified like the other grids.
int solve8(mc_ctx* c, const Geo& g, const float* w, const float* const* a, const float* z0, float* x_out,
           uint8_t* labels_out, float* z_out, mc_stats* stats, const mc_opts& o, hipStream_t s)
{
    constexpr int R = 4;
    const size_t n = (size_t)g.n;
    const int H = g.H, W = g.W;
    const size_t nz = (size_t)2 * (H > 1 ? H - 1 : 0) * W;
    if (nz > (size_t)kMaxNodes) return fail(MC_ERR_INVALID_ARG, "8-connected grid too large (2(H-1)W > 2^31 - 2^24)");
    int rc;
    if ((rc = ensure_ws(c, n, R))) return rc;
    const size_t need = 2 * n + 4 * nz;
    if (need > c->g8cap) {
        (void)hipFree(c->g8buf);
        c->g8buf = nullptr;
        c->g8cap = 0;
        if (hipMalloc(&c->g8buf, sizeof(float) * need) != hipSuccess) {
            (void)hipGetLastError();
            return fail(MC_ERR_NOMEM, "8-connected workspace allocation failed");
        }
        c->g8cap = need;
    }
    float* q = c->g8buf;  // prox of rows and columns (2n)
    float* zzv = q + 2 * n;
    float* zza = zzv + nz;
    float* zzx = zza + nz;
    float* zzp = zzx + nz;
    Geo gz;
    gz.D = 1;
    gz.H = 2 * (H - 1);
    gz.W = W;
    gz.n = (int)nz;
    gz.ndim = 2;

    if (o.flags & MC_VALIDATE) {
        MC_HIP(launch_validate8(g, w, a, c->partials, c->dout, s));
        MC_HIP(hipMemcpyAsync(c->hout, c->dout, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        MC_HIP(hipStreamSynchronize(s));
        if (c->hout[1] > 0) return fail(MC_ERR_NONFINITE, "non-finite value in w or a");
        if (c->hout[0] > 0) return fail(MC_ERR_NEGATIVE_WEIGHT, "negative weight or non-zero weight of a missing edge");
    }
    if (z0) MC_HIP(hipMemcpyAsync(c->z, z0, sizeof(float) * R * n, hipMemcpyDeviceToDevice, s));
    else MC_HIP(hipMemsetAsync(c->z, 0, sizeof(float) * R * n, s));
    MC_HIP(hipEventRecord(c->ev0, s));

    const float* pj[R] = {c->p, c->p + n, c->p + 2 * n, c->p + 3 * n};
    SweepTimer tm{c, (o.flags & MC_PROFILE) != 0};
    float taus[kNumTau];
    tau_ladder(o.tau0, taus);
    CheckState st;
    int it = 0;
    bool converged = false;
    float* zc = c->z;
    float* zn = c->z2;
    bool zz_current = false;  // zzv holds the zig-zag families of zc
    // checks are read behind the next iteration, as in solve_split
    const bool overlap_checks = !(o.flags & MC_PROFILE);
    bool pending = false;
    auto is_check = [&](int i) { return (i % o.check_every == 0) || i == o.max_iters; };
    auto overlap = [&](int i) {
        return overlap_checks && !g.whole && st.checks >= 3 && i < o.max_iters && !is_check(i + 1);
    };
    while (it < o.max_iters) {
        ++it;
        const bool check = is_check(it);
        if (it == 1 && !z0) {
            // every prox of the zero state is zero (see mc_tv_solve)
            if (check) MC_HIP(hipMemsetAsync(c->p, 0, sizeof(float) * R * n, s));
            MC_HIP(launch_cold_product(g, R, w, zn, s));
        } else {
            // the zig-zag chains are gathered once (with their weights); from
            // then on the averaging step writes them
            if (!zz_current) MC_HIP(launch_zz_gather(H, W, zc + 2 * n, zc + 3 * n, a[2], a[3], zzv, zza, s));
            MC_HIP(tm.begin(s));
            MC_HIP(launch_sweeps8(g, zc, a, q, check ? c->p : nullptr, gz, zzv, zza, zzx, check ? zzp : nullptr,
                                  s));
            MC_HIP(tm.end(s));
            MC_HIP(launch_combine8(H, W, zc, q, zzx, check ? zzp : nullptr, w, zn, zzv, c->p + 2 * n,
                                   c->p + 3 * n, s));
            zz_current = true;
        }
        float* zt = zc;
        zc = zn;
        zn = zt;
        if (pending) {
            pending = false;
            bool done = false;
            if ((rc = read_check(c, o, taus, tm, st, done))) return rc;
            if (done) {  // certified at the previous iteration, whose state is in zn
                converged = true;
                --it;
                zc = zn;
                break;
            }
        }
        if (!check) continue;
        if ((rc = enqueue_check(c, ctx_ws(c), g, true, w, a, pj, o, s, st))) return rc;
        if (overlap(it)) {
            pending = true;
            continue;
        }
        bool done = false;
        if ((rc = read_check(c, o, taus, tm, st, done))) return rc;
        if (done) {
            converged = true;
            break;
        }
    }
    return finish_solve(c, ctx_ws(c), g, zc, R * n, x_out, labels_out, z_out, stats, it, converged, st, tm, s);
}

// opts (nullable: defaults) with the checks every single-grid solve shares
int read_opts(const mc_opts* in, mc_opts& o)
{
    if (in) o = *in; else mc_opts_default(&o);
    if (o.max_iters < 1 || o.check_every < 1) return fail(MC_ERR_INVALID_ARG, "max_iters and check_every must be >= 1");
    if (!(o.tau0 >= 0.f)) return fail(MC_ERR_INVALID_ARG, "tau0 must be >= 0");
    if ((o.flags & MC_WHOLE_CHAINS) && (o.flags & MC_PIECE_CHAINS))
        return fail(MC_ERR_INVALID_ARG, "MC_WHOLE_CHAINS and MC_PIECE_CHAINS exclude each other");
    return MC_OK;
}

// ---- scratch of mc_tv_solve_noalloc -----------------------------------------------
//
// One static device array per GPU, reserved when the code object loads and held
// until the process ends: the reduction partials, the certificate values and the
// probe counters, then up to kNoAllocFloats floats of solver state (five arrays,
// each starting on a 256-byte boundary).  In host code `scratch` only names the
// symbol; its device address comes from hipGetSymbolAddress, taken once per
// device by mc_ctx_create with that device current, and only that address is
// passed to kernels and copies.
constexpr size_t kNoAllocFloats = size_t(1) << 23;  // 32 MiB of state
constexpr size_t kScratchAlign = 256;
constexpr size_t scratch_round(size_t bytes) { return (bytes + kScratchAlign - 1) / kScratchAlign * kScratchAlign; }
constexpr size_t kScratchPartials = scratch_round(sizeof(double) * kReduceBlocks * kCertValues);
constexpr size_t kScratchDout = scratch_round(sizeof(double) * kCertValues);
constexpr size_t kScratchCnt = scratch_round(2 * sizeof(int));
constexpr size_t kScratchHeader = kScratchPartials + kScratchDout + kScratchCnt;
constexpr size_t kScratchState = sizeof(float) * kNoAllocFloats + 5 * kScratchAlign;
constexpr int kScratchDevices = 64;

std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kScratchDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchHeader + kScratchState];

namespace {

// with `device` current: its address of the scratch array (once per device)
int scratch_setup(int device)
{
    if (device >= kScratchDevices) return MC_OK;  // mc_tv_solve_noalloc refuses such devices
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return MC_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_error(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[device] = static_cast<unsigned char*>(ptr);
    return MC_OK;
}

// MC_FP64_STATE: the splitting of solve_split with its state, chain proxes
// and averaging in FP64 (fp64.hip); the duals of check iterations are
// written as clipped FP32 into ws.p and certified as usual.
int solve_fp64(mc_ctx* c, const SolveWs& ws, Geo g, bool two_set, const float* w, const float* const* a,
               const float* z0, float* x_out, uint8_t* labels_out, float* z_out, mc_stats* stats, const mc_opts& o,
               hipStream_t s)
{
    int rc;
    const int r = g.ndim;
    const size_t n = (size_t)g.n;
    const size_t nz = two_set ? n : (size_t)r * n;
    const size_t need = 3 * nz;  // state, next state, prox outputs (n for the rows or r n)
    if (need > c->d64cap) {
        MC_HIP(hipStreamSynchronize(s));
        (void)hipFree(c->d64buf);
        c->d64buf = nullptr;
        c->d64cap = 0;
        if (hipMalloc(&c->d64buf, sizeof(double) * need) != hipSuccess) {
            (void)hipGetLastError();
            return fail(MC_ERR_NOMEM, "FP64 state allocation failed");
        }
        c->d64cap = need;
    }
    double* zc = c->d64buf;
    double* zn = zc + nz;
    double* q = zn + nz;
    if (o.flags & MC_VALIDATE) {
        MC_HIP(launch_validate(g, w, a, ws.partials, ws.dout, s));
        MC_HIP(hipMemcpyAsync(c->hout, ws.dout, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        MC_HIP(hipStreamSynchronize(s));
        if (c->hout[1] > 0) return fail(MC_ERR_NONFINITE, "non-finite value in w or a");
        if (c->hout[0] > 0) return fail(MC_ERR_NEGATIVE_WEIGHT, "negative weight or non-zero weight on a last slice");
    }
    if (z0) MC_HIP(launch_f32_to_f64(nz, z0, zc, s));
    else MC_HIP(hipMemsetAsync(zc, 0, sizeof(double) * nz, s));
    MC_HIP(hipEventRecord(c->ev0, s));
    const float* pj[3] = {ws.p, ws.p + n, ws.p + 2 * n};
    SweepTimer tm{c, false};
    float taus[kNumTau];
    tau_ladder(o.tau0, taus);
    CheckState st;
    int it = 0;
    bool converged = false;
    while (it < o.max_iters) {
        ++it;
        const bool check = (it % o.check_every == 0) || it == o.max_iters;
        if (two_set) {
            MC_HIP(launch_dr2_rows64(g, zc, a[0], q, check ? ws.p : nullptr, s));
            MC_HIP(launch_dr2_cols64(g, q, zc, zn, w, a[1], check ? ws.p + n : nullptr, s));
        } else {
            for (int j = 0; j < r; ++j)
                MC_HIP(launch_family64(g, j, zc + (size_t)j * n, a[j], q + (size_t)j * n,
                                       check ? ws.p + (size_t)j * n : nullptr, s));
            MC_HIP(launch_combine64(n, r, zc, q, w, zn, s));
        }
        double* zt = zc;
        zc = zn;
        zn = zt;
        tm.launches += two_set ? 2 : r;
        if (!check) continue;
        bool done = false;
        if ((rc = run_check(c, ws, g, false, w, a, pj, o, taus, tm, s, st, done))) return rc;
        if (done) {
            converged = true;
            break;
        }
    }
    MC_HIP(launch_f64_to_f32(nz, zc, ws.z, s));  // the state, rounded, for z_out
    g.whole = 1;
    return finish_solve(c, ws, g, ws.z, nz, x_out, labels_out, z_out, stats, it, converged, st, tm, s);
}

// The splitting method on a 4- or 6-connected grid (two-set form or product
// space) with the device buffers of ws; arguments already checked.
int solve_split(mc_ctx* c, const SolveWs& ws, Geo g, bool two_set, const float* w, const float* const* a,
                const float* z0, float* x_out, uint8_t* labels_out, float* z_out, mc_stats* stats, const mc_opts& o,
                hipStream_t s)
{
    int rc;
    const int r = g.ndim;
    const size_t n = (size_t)g.n;
    const size_t nz = two_set ? n : (size_t)r * n;

    if (o.flags & MC_VALIDATE) {
        MC_HIP(launch_validate(g, w, a, ws.partials, ws.dout, s));
        MC_HIP(hipMemcpyAsync(c->hout, ws.dout, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        MC_HIP(hipStreamSynchronize(s));
        if (c->hout[1] > 0) return fail(MC_ERR_NONFINITE, "non-finite value in w or a");
        if (c->hout[0] > 0) return fail(MC_ERR_NEGATIVE_WEIGHT, "negative weight or non-zero weight on a last slice");
    }

    if (z0) MC_HIP(hipMemcpyAsync(ws.z, z0, sizeof(float) * nz, hipMemcpyDeviceToDevice, s));
    else MC_HIP(hipMemsetAsync(ws.z, 0, sizeof(float) * nz, s));
    MC_HIP(hipEventRecord(c->ev0, s));

    const float* pj[3] = {ws.p, ws.p + n, ws.p + 2 * n};
    SweepTimer tm{c, (o.flags & MC_PROFILE) != 0};
    float taus[kNumTau];
    tau_ladder(o.tau0, taus);
    CheckState st;
    int it = 0;
    bool converged = false;
    SweepProbe probe(c, ws, g, o, s);
    if ((rc = probe.start())) return rc;
    float* zc = ws.z;   // current state
    float* zn = ws.z2;  // next state
    // A check is read only once the next iteration is queued behind it (when
    // that one is no check), so that the device does not idle while the host
    // reads the result.  The extra iteration writes neither the duals nor the
    // primal, and the state it leaves in the other buffer is that of the
    // check, so a certified check still ends the solve with its own state.
    // The iteration queued behind the certified check is lost time, so the
    // first two checks of a solve are read at once (short solves, such as
    // the moves of alpha-expansion, pay nothing), and whole-chain sweeps,
    // whose iterations are long against the wait, never overlap.
    auto is_check = [&](int i) { return (i % o.check_every == 0) || i == o.max_iters; };
    const bool overlap_checks = !(o.flags & (MC_PROFILE | MC_DEBUG));
    auto overlap = [&](int i) {
        return overlap_checks && !g.whole && st.checks >= 3 && i < o.max_iters && !is_check(i + 1);
    };
    bool pending = false;
    while (it < o.max_iters) {
        ++it;
        const bool check = is_check(it);
        // A cold start begins at z = 0, whose chain proxes are 0 with zero
        // duals (the prox of a constant chain is the chain itself).  Sweeping
        // that is slow -- every chain is one segment, so no bracket closes
        // before the chain start -- and unnecessary: set the results instead.
        const bool cold_first = it == 1 && !z0;
        if (two_set && cold_first) {
            MC_HIP(hipMemsetAsync(ws.y, 0, sizeof(float) * n, s));
            if (check) MC_HIP(hipMemsetAsync(ws.p, 0, sizeof(float) * n, s));
            MC_HIP(tm.begin(s, check));
            MC_HIP(launch_dr2_cols(g, ws.y, zc, zn, w, a[1], check ? ws.p + n : nullptr, s));
            MC_HIP(tm.end(s));
        } else if (cold_first) {
            if (check) MC_HIP(hipMemsetAsync(ws.p, 0, sizeof(float) * (size_t)r * n, s));
            MC_HIP(launch_cold_product(g, r, w, zn, s));
        } else if (two_set) {
            MC_HIP(tm.begin(s, check));
            MC_HIP(launch_dr2_rows(g, zc, a[0], ws.y, check ? ws.p : nullptr, s));
            MC_HIP(tm.end(s));
            MC_HIP(tm.begin(s, check));
            MC_HIP(launch_dr2_cols(g, ws.y, zc, zn, w, a[1], check ? ws.p + n : nullptr, s));
            MC_HIP(tm.end(s));
        } else if (r == 3) {
            // all three families in one launch, then the averaging step
            MC_HIP(tm.begin(s, check));
            MC_HIP(launch_sweeps3(g, zc, a, ws.y, check ? ws.p : nullptr, s));
            MC_HIP(tm.end(s));
            MC_HIP(launch_combine3(n, zc, ws.y, w, zn, s));
        } else {
            MC_HIP(tm.begin(s, check));
            MC_HIP(launch_drp_sweeps(g, r - 1, zc, a, ws.y, check ? ws.p : nullptr, s));
            MC_HIP(tm.end(s));
            MC_HIP(tm.begin(s, check));
            MC_HIP(launch_drp_final(g, r, zc, zn, ws.y, a[r - 1], w,
                                    check ? ws.p + (size_t)(r - 1) * n : nullptr, s));
            MC_HIP(tm.end(s));
        }
        float* zt = zc;
        zc = zn;
        zn = zt;
        if ((rc = probe.after_iteration(tm.launches))) return rc;
        if ((o.flags & MC_DEBUG) && (rc = debug_state(c, ws, zc, nz, it, s))) return rc;
        if (pending) {
            pending = false;
            bool done = false;
            if ((rc = read_check(c, o, taus, tm, st, done))) return rc;
            if (done) {  // certified at the previous iteration, whose state is in zn
                converged = true;
                --it;
                zc = zn;
                break;
            }
        }
        if (!check) continue;
        if ((o.flags & MC_DEBUG) && (rc = debug_duals(c, ws, g, a, pj, it, s))) return rc;
        if ((rc = enqueue_check(c, ws, g, false, w, a, pj, o, s, st))) return rc;
        if (overlap(it)) {
            pending = true;
            continue;
        }
        bool done = false;
        if ((rc = read_check(c, o, taus, tm, st, done))) return rc;
        if (done) {
            converged = true;
            break;
        }
    }
    return finish_solve(c, ws, g, zc, nz, x_out, labels_out, z_out, stats, it, converged, st, tm, s);
}

}  // namespace

extern "C" {

void mc_opts_default(mc_opts* o)
{
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->max_iters = 500;
    o->check_every = 1;
    o->gap_tol = 1e-3;
    o->variant = MC_VARIANT_AUTO;
    o->tau0 = 1e-3f;
    o->flags = 0;
}

const char* mc_status_string(int code)
{
    switch (code) {
    case MC_OK: return "ok";
    case MC_NOT_CONVERGED: return "not converged (max_iters reached)";
    case MC_ERR_INVALID_ARG: return "invalid argument";
    case MC_ERR_NEGATIVE_WEIGHT: return "negative edge weight (or non-zero weight on a last slice)";
    case MC_ERR_NONFINITE: return "non-finite input";
    case MC_ERR_NOMEM: return "out of device memory";
    case MC_ERR_DEVICE: return "HIP runtime error";
    case MC_ERR_NUMERIC: return "non-finite solver state";
    default: return "unknown status";
    }
}

const char* mc_last_error(void) { return g_last_error.c_str(); }

int mc_ctx_create(mc_ctx** out, int device)
{
    if (!out) return fail(MC_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= ndev) return fail(MC_ERR_INVALID_ARG, "no such device");
    MC_HIP(hipSetDevice(device));
    mc_ctx* c = new mc_ctx();
    c->device = device;
    if (hipMalloc(&c->partials, sizeof(double) * kReduceBlocks * kCertValues) != hipSuccess ||
        hipMalloc(&c->dout, sizeof(double) * kCertValues) != hipSuccess ||
        hipHostMalloc(&c->hout, sizeof(double) * kCertValues, hipHostMallocDefault) != hipSuccess ||
        hipMalloc(&c->scnt, 2 * sizeof(int)) != hipSuccess ||
        hipHostMalloc(&c->scnt_h, 2 * sizeof(int), hipHostMallocDefault) != hipSuccess ||
        hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
        hipStreamCreateWithFlags(&c->bstream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        mc_ctx_destroy(c);
        return fail(MC_ERR_NOMEM, "context allocation failed");
    }
    int rc = scratch_setup(device);
    if (rc) {
        mc_ctx_destroy(c);
        return rc;
    }
    *out = c;
    return MC_OK;
}

int mc_ctx_destroy(mc_ctx* c)
{
    if (!c) return MC_OK;
    // teardown: errors are not actionable, every resource is released regardless
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    free_ws(c);
    (void)hipFree(c->partials);
    (void)hipFree(c->dout);
    if (c->hout) (void)hipHostFree(c->hout);
    (void)hipFree(c->scnt);
    if (c->scnt_h) (void)hipHostFree(c->scnt_h);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    for (hipEvent_t e : c->prof_ev) (void)hipEventDestroy(e);
    (void)hipFree(c->bbuf);
    (void)hipFree(c->bmeta);
    (void)hipFree(c->bctl);
    (void)hipFree(c->nbuf);
    (void)hipFree(c->g8buf);
    (void)hipFree(c->vbuf);
    (void)hipFree(c->d64buf);
    (void)hipFree(c->mlbuf);
    (void)hipFree(c->mlsel);
    if (c->bstream) (void)hipStreamDestroy(c->bstream);
    delete c;
    return MC_OK;
}

int mc_tv_prox_chains(mc_ctx* c, const mc_grid* grid, int axis, const float* v,
                      const float* a_axis, float* x_out, float* p_out, void* stream)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    Geo g;
    if ((rc = make_geo(grid, &g))) return rc;
    if (axis < 0 || axis >= g.ndim) return fail(MC_ERR_INVALID_ARG, "axis out of range");
    if (!v || !a_axis || !x_out) return fail(MC_ERR_INVALID_ARG, "null array");
    if ((rc = ensure_ws(c, (size_t)g.n, 1))) return rc;
    hipStream_t s = (hipStream_t)stream;
    MC_HIP(launch_prox(g, axis, v, a_axis, x_out, p_out, s));
    return MC_OK;
}

int mc_cut_energy(mc_ctx* c, const mc_grid* grid, const float* w, const float* const* a,
                  const uint8_t* labels, double* energy_out, void* stream)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    Geo g;
    if ((rc = make_geo(grid, &g))) return rc;
    if (!w || !a || !labels || !energy_out) return fail(MC_ERR_INVALID_ARG, "null argument");
    const int na = grid->conn == 8 ? 4 : g.ndim;
    for (int j = 0; j < na; ++j)
        if (!a[j]) return fail(MC_ERR_INVALID_ARG, "null weight array");
    hipStream_t s = (hipStream_t)stream;
    if (grid->conn == 8) MC_HIP(launch_energy8(g, w, a, labels, c->partials, c->dout, s));
    else MC_HIP(launch_energy(g, w, a, labels, c->partials, c->dout, s));
    MC_HIP(hipMemcpyAsync(c->hout, c->dout, sizeof(double), hipMemcpyDeviceToHost, s));
    MC_HIP(hipStreamSynchronize(s));
    *energy_out = c->hout[0];
    return MC_OK;
}

int mc_tv_solve(mc_ctx* c, const mc_grid* grid, const float* w, const float* const* a,
                const float* z0, float* x_out, uint8_t* labels_out, float* z_out,
                mc_stats* stats, const mc_opts* opts_in, void* stream)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    Geo g;
    if ((rc = make_geo(grid, &g))) return rc;
    if (!w || !a || !labels_out || !stats) return fail(MC_ERR_INVALID_ARG, "null argument");
    for (int j = 0; j < g.ndim; ++j)
        if (!a[j]) return fail(MC_ERR_INVALID_ARG, "null weight array");
    mc_opts o;
    if ((rc = read_opts(opts_in, o))) return rc;
    g.whole = (o.flags & MC_WHOLE_CHAINS) ? 1 : 0;
    g.stream = (o.flags & MC_PIECE_CHAINS) ? 0 : 1;
    if ((o.flags & MC_FP64_STATE) &&
        (grid->conn == 8 || (o.variant != MC_VARIANT_AUTO && o.variant != MC_VARIANT_TWO_SET &&
                             o.variant != MC_VARIANT_PRODUCT)))
        return fail(MC_ERR_INVALID_ARG, "MC_FP64_STATE: 4- and 6-connected grids, variants AUTO, TWO_SET, PRODUCT");
    if (grid->conn == 8) {
        if (g.ndim != 2) return fail(MC_ERR_INVALID_ARG, "8-connected grids are 2D");
        if (o.variant == MC_VARIANT_TWO_SET) return fail(MC_ERR_INVALID_ARG, "8-connected grids use the product space");
        if (o.variant != MC_VARIANT_AUTO && o.variant != MC_VARIANT_PRODUCT)
            return fail(MC_ERR_INVALID_ARG, "unknown variant");
        for (int j = 2; j < 4; ++j)
            if (!a[j]) return fail(MC_ERR_INVALID_ARG, "null weight array");
        return solve8(c, g, w, a, z0, x_out, labels_out, z_out, stats, o, (hipStream_t)stream);
    }
    if (o.variant == MC_VARIANT_BCD || o.variant == MC_VARIANT_AP || o.variant == MC_VARIANT_FISTA)
        return solve_variant(c, g, w, a, z0, x_out, labels_out, z_out, stats, o, (hipStream_t)stream);
    if (o.variant == MC_VARIANT_BCD_DR) {
        if (z0 || z_out) return fail(MC_ERR_INVALID_ARG, "MC_VARIANT_BCD_DR takes no z0 / z_out");
        const int k = o.bcd_iters > 0 ? o.bcd_iters : 16;
        hipStream_t s = (hipStream_t)stream;
        mc_opts ob = o;
        ob.variant = MC_VARIANT_BCD;
        ob.max_iters = k < o.max_iters ? k : o.max_iters;
        mc_stats s1;
        rc = solve_variant(c, g, w, a, nullptr, x_out, labels_out, nullptr, &s1, ob, s);
        if (rc < 0 || rc == MC_OK || ob.max_iters == o.max_iters) {
            *stats = s1;
            return rc;
        }
        // the BCD blocks y (r n) and the primal x (n) stay in the variant
        // workspace, which the splitting does not use; the start state goes
        // to its third block
        const int r = g.ndim;
        const size_t n = (size_t)g.n;
        float* Y = c->vbuf;
        float* Z0 = c->vbuf + 2 * (size_t)r * n;
        float* X = c->vbuf + 3 * (size_t)r * n;
        if (r == 2) {
            MC_HIP(launch_add(n, X, Y, Z0, s));  // z0 = x + y_rows
        } else {
            for (int j = 0; j < r; ++j) {        // z0_j = y_j + x / r
                MC_HIP(launch_scale(n, 1.f / (float)r, X, Z0 + (size_t)j * n, s));
                MC_HIP(launch_add(n, Z0 + (size_t)j * n, Y + (size_t)j * n, Z0 + (size_t)j * n, s));
            }
        }
        mc_opts od = o;
        od.variant = MC_VARIANT_AUTO;
        od.max_iters = o.max_iters - ob.max_iters;
        od.flags &= ~(uint32_t)MC_VALIDATE;  // checked by the first phase
        rc = mc_tv_solve(c, grid, w, a, Z0, x_out, labels_out, nullptr, stats, &od, stream);
        if (rc < 0) return rc;
        stats->iters += s1.iters;
        stats->ms += s1.ms;
        stats->sweep_ms += s1.sweep_ms;
        stats->sweep_launches += s1.sweep_launches;
        stats->dual_sweep_ms += s1.dual_sweep_ms;
        stats->dual_sweep_launches += s1.dual_sweep_launches;
        stats->checks += s1.checks;
        return rc;
    }
    bool two_set;
    if (o.variant == MC_VARIANT_AUTO) two_set = g.ndim == 2;
    else if (o.variant == MC_VARIANT_TWO_SET) two_set = true;
    else if (o.variant == MC_VARIANT_PRODUCT) two_set = false;
    else return fail(MC_ERR_INVALID_ARG, "unknown variant");
    if (two_set && g.ndim != 2) return fail(MC_ERR_INVALID_ARG, "two-set form needs a 2D grid");
    const int r = g.ndim;
    const size_t n = (size_t)g.n;
    if ((rc = ensure_ws(c, n, r))) return rc;
    if (o.flags & MC_FP64_STATE)
        return solve_fp64(c, ctx_ws(c), g, two_set, w, a, z0, x_out, labels_out, z_out, stats, o,
                          (hipStream_t)stream);
    return solve_split(c, ctx_ws(c), g, two_set, w, a, z0, x_out, labels_out, z_out, stats, o,
                       (hipStream_t)stream);
}

int mc_tv_solve_noalloc(mc_ctx* c, const mc_grid* grid, const float* w, const float* const* a, const float* z0,
                        float* x_out, uint8_t* labels_out, float* z_out, mc_stats* stats, const mc_opts* opts_in,
                        void* stream)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    Geo g;
    if ((rc = make_geo(grid, &g))) return rc;
    if (!w || !a || !labels_out || !stats) return fail(MC_ERR_INVALID_ARG, "null argument");
    for (int j = 0; j < g.ndim; ++j)
        if (!a[j]) return fail(MC_ERR_INVALID_ARG, "null weight array");
    mc_opts o;
    if ((rc = read_opts(opts_in, o))) return rc;
    if (grid->conn == 8) return fail(MC_ERR_INVALID_ARG, "mc_tv_solve_noalloc: 4- and 6-connected grids only");
    if (o.flags & MC_PROFILE) return fail(MC_ERR_INVALID_ARG, "mc_tv_solve_noalloc: MC_PROFILE needs timing events");
    if (o.flags & MC_FP64_STATE)
        return fail(MC_ERR_INVALID_ARG, "mc_tv_solve_noalloc: MC_FP64_STATE allocates its FP64 state");
    bool two_set;
    if (o.variant == MC_VARIANT_AUTO) two_set = g.ndim == 2;
    else if (o.variant == MC_VARIANT_TWO_SET) two_set = true;
    else if (o.variant == MC_VARIANT_PRODUCT) two_set = false;
    else return fail(MC_ERR_INVALID_ARG, "mc_tv_solve_noalloc: variant must be AUTO, TWO_SET or PRODUCT");
    if (two_set && g.ndim != 2) return fail(MC_ERR_INVALID_ARG, "two-set form needs a 2D grid");
    g.whole = (o.flags & MC_WHOLE_CHAINS) ? 1 : 0;
    g.stream = (o.flags & MC_PIECE_CHAINS) ? 0 : 1;
    const size_t n = (size_t)g.n, r = (size_t)g.ndim;
    const size_t nz = two_set ? n : r * n;
    const size_t counts[5] = {nz, nz, two_set ? n : r * n, two_set ? 2 * n : r * n, n};  // z, z2, y, p, xt
    size_t need = 0;
    for (size_t k : counts) need += scratch_round(sizeof(float) * k);
    if (need > kScratchState)
        return fail(MC_ERR_INVALID_ARG, "mc_tv_solve_noalloc: the grid needs " + std::to_string(need) +
                                            " bytes of state, the static scratch holds " +
                                            std::to_string(kScratchState));
    unsigned char* base = c->device < kScratchDevices ? g_scratch_ptr[c->device] : nullptr;
    if (!base) return fail(MC_ERR_DEVICE, "mc_tv_solve_noalloc: no scratch address for this device");
    SolveWs ws;
    ws.partials = reinterpret_cast<double*>(base);
    ws.dout = reinterpret_cast<double*>(base + kScratchPartials);
    ws.scnt = reinterpret_cast<int*>(base + kScratchPartials + kScratchDout);
    unsigned char* f = base + kScratchHeader;
    float* arr[5];
    for (int k = 0; k < 5; ++k) {
        arr[k] = reinterpret_cast<float*>(f);
        f += scratch_round(sizeof(float) * counts[k]);
    }
    ws.z = arr[0];
    ws.z2 = arr[1];
    ws.y = arr[2];
    ws.p = arr[3];
    ws.xt = arr[4];
    return solve_split(c, ws, g, two_set, w, a, z0, x_out, labels_out, z_out, stats, o, (hipStream_t)stream);
}

}  // extern "C"
