// multilabel.hip -- multi-label energies on 2D 4-connected grids by
// alpha-expansion (Sec. 4.4 of the paper: move-making reduces a multi-label
// problem to a series of binary cuts; Sec. 6.1 solves a stereo task so).
//
// E(f) = sum_i data[f_i][i] + sum_{e = (u, v)} lam_e V(f_u, f_v) with a metric V
// (Potts or truncated linear).  The move of label alpha lets every pixel keep
// f_i or take alpha; with A = V(f_u, f_v), B = V(f_u, alpha), C = V(alpha, f_v)
// and V(alpha, alpha) = 0 the edge term of the move is
//     lam (A + (C - A) x_u - C x_v + k (1 - x_u) x_v),   k = B + C - A >= 0,
// and k (1 - x_u) x_v = k/2 |x_u - x_v| + k/2 (x_v - x_u): the move is the cut
// problem of mc_tv_solve with a_e = lam k / 2 and the unary terms
// lam (C - A - B) / 2 at u and lam (B - A - C) / 2 at v, besides the data
// difference data[alpha][i] - data[f_i][i].  Each move is solved exactly
// (certified) and applied when its energy is negative.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <chrono>
#include <vector>

#include "ctx.hpp"
#include "launch.hpp"
#include "mc.h"

namespace mc {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ float vdist(int kind, float trunc, int a, int b)
{
    if (kind == MC_V_POTTS) return a != b ? 1.f : 0.f;
    const float d = (float)(a > b ? a - b : b - a);
    return d < trunc ? d : trunc;
}

// One thread per pixel (r, c).  Its unary gathers the terms of its four edges
// in the order right (as u), left (as v), down (as u), up (as v); it writes the
// weights of its right and down edges (0 on the last column / row).
__global__ void __launch_bounds__(kThreads)
k_expand_build(int H, int W, const float* __restrict__ data, const float* __restrict__ lx,
               const float* __restrict__ ly, int kind, float trunc, const int32_t* __restrict__ f, int alpha,
               float* __restrict__ w, float* __restrict__ ax, float* __restrict__ ay)
{
    const size_t n = (size_t)H * W;
    for (int r = blockIdx.y; r < H; r += gridDim.y) {
        for (int c = blockIdx.x * kThreads + threadIdx.x; c < W; c += gridDim.x * kThreads) {
            const size_t i = (size_t)r * W + c;
            const int fi = f[i];
            float wi = data[(size_t)alpha * n + i] - data[(size_t)fi * n + i];
            float axi = 0.f, ayi = 0.f;
            if (c + 1 < W) {
                const float lam = lx[i];
                const int fv = f[i + 1];
                const float A = vdist(kind, trunc, fi, fv), B = vdist(kind, trunc, fi, alpha),
                            C = vdist(kind, trunc, alpha, fv);
                axi = lam * (B + C - A) * 0.5f;
                wi += lam * (C - A - B) * 0.5f;
            }
            if (c > 0) {
                const float lam = lx[i - 1];
                const int fu = f[i - 1];
                const float A = vdist(kind, trunc, fu, fi), B = vdist(kind, trunc, fu, alpha),
                            C = vdist(kind, trunc, alpha, fi);
                wi += lam * (B - A - C) * 0.5f;
            }
            if (r + 1 < H) {
                const float lam = ly[i];
                const int fv = f[i + W];
                const float A = vdist(kind, trunc, fi, fv), B = vdist(kind, trunc, fi, alpha),
                            C = vdist(kind, trunc, alpha, fv);
                ayi = lam * (B + C - A) * 0.5f;
                wi += lam * (C - A - B) * 0.5f;
            }
            if (r > 0) {
                const float lam = ly[i - W];
                const int fu = f[i - W];
                const float A = vdist(kind, trunc, fu, fi), B = vdist(kind, trunc, fu, alpha),
                            C = vdist(kind, trunc, alpha, fi);
                wi += lam * (B - A - C) * 0.5f;
            }
            w[i] = wi;
            ax[i] = axi;
            ay[i] = ayi;
        }
    }
}

__global__ void __launch_bounds__(kThreads)
k_expand_apply(int n, int alpha, const uint8_t* __restrict__ sel, int32_t* __restrict__ f)
{
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads)
        if (sel[i]) f[i] = alpha;
}

}  // namespace

hipError_t launch_expand_build(const Geo& g, const float* data, const float* const* lam, int kind, float trunc,
                               const int32_t* f, int alpha, float* w, float* ax, float* ay, hipStream_t s)
{
    const int bx = (g.W + kThreads - 1) / kThreads;
    const int by = g.H < 65535 ? g.H : 65535;
    hipLaunchKernelGGL(k_expand_build, dim3(bx, by), dim3(kThreads), 0, s, g.H, g.W, data, lam[0], lam[1], kind,
                       trunc, f, alpha, w, ax, ay);
    return hipGetLastError();
}

hipError_t launch_expand_apply(int n, int alpha, const uint8_t* sel, int32_t* f, hipStream_t s)
{
    const int b = (n + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(k_expand_apply, dim3(b < 4096 ? b : 4096), dim3(kThreads), 0, s, n, alpha, sel, f);
    return hipGetLastError();
}

namespace {

// shared argument checks; the labels are checked on the device (they index data)
int check_ml(mc_ctx* c, const mc_grid* grid, int L, const float* data, const float* const* lam, int kind,
             float trunc, const int32_t* labels, Geo* g, hipStream_t s)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if ((rc = make_geo(grid, g))) return rc;
    if (g->ndim != 2 || (grid->conn != 0 && grid->conn != 4))
        return set_error(MC_ERR_INVALID_ARG, "alpha-expansion needs a 2D 4-connected grid");
    if (L < 1) return set_error(MC_ERR_INVALID_ARG, "n_labels must be >= 1");
    if ((int64_t)L * g->n > kMaxNodes) return set_error(MC_ERR_INVALID_ARG, "n_labels * H * W above 2^31 - 2^24");
    if (!data || !lam || !lam[0] || !lam[1] || !labels) return set_error(MC_ERR_INVALID_ARG, "null argument");
    if (kind != MC_V_POTTS && kind != MC_V_TRUNC_LINEAR) return set_error(MC_ERR_INVALID_ARG, "unknown v_kind");
    if (kind == MC_V_TRUNC_LINEAR && !(trunc >= 0.f && isfinite(trunc)))
        return set_error(MC_ERR_INVALID_ARG, "v_trunc must be finite and >= 0");
    MC_HIP(launch_check_labels(g->n, L, labels, c->partials, c->dout, s));
    MC_HIP(hipMemcpyAsync(c->hout, c->dout, sizeof(double), hipMemcpyDeviceToHost, s));
    MC_HIP(hipStreamSynchronize(s));
    if (c->hout[0] > 0) return set_error(MC_ERR_INVALID_ARG, "label outside [0, n_labels)");
    return MC_OK;
}

// per pixel: w, a_x, a_y, and (warm moves) z0 plus [x; p1] of every label's last move
int ensure_ml_ws(mc_ctx* c, size_t n, size_t per_pixel)
{
    if (c->mlcap >= n && c->mlper >= per_pixel) return MC_OK;
    (void)hipFree(c->mlbuf);
    (void)hipFree(c->mlsel);
    c->mlbuf = nullptr;
    c->mlsel = nullptr;
    c->mlcap = 0;
    c->mlper = 0;
    if (hipMalloc(&c->mlbuf, sizeof(float) * per_pixel * n) != hipSuccess ||
        hipMalloc(&c->mlsel, n) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(c->mlbuf);
        (void)hipFree(c->mlsel);
        c->mlbuf = nullptr;
        c->mlsel = nullptr;
        return set_error(MC_ERR_NOMEM, "alpha-expansion workspace allocation failed");
    }
    c->mlcap = n;
    c->mlper = per_pixel;
    return MC_OK;
}

int read_energy(mc_ctx* c, const Geo& g, const float* data, const float* const* lam, int kind, float trunc,
                const int32_t* labels, double* e, hipStream_t s)
{
    MC_HIP(launch_ml_energy(g, data, lam, kind, trunc, labels, c->partials, c->dout, s));
    MC_HIP(hipMemcpyAsync(c->hout, c->dout, sizeof(double), hipMemcpyDeviceToHost, s));
    MC_HIP(hipStreamSynchronize(s));
    *e = c->hout[0];
    return MC_OK;
}

}  // namespace

}  // namespace mc

using namespace mc;

extern "C" {

int mc_expansion_problem(mc_ctx* c, const mc_grid* grid, int n_labels, const float* data, const float* const* lam,
                         int v_kind, float v_trunc, const int32_t* labels, int alpha, float* w_out,
                         float* const* a_out, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    Geo g;
    int rc = check_ml(c, grid, n_labels, data, lam, v_kind, v_trunc, labels, &g, s);
    if (rc) return rc;
    if (alpha < 0 || alpha >= n_labels) return set_error(MC_ERR_INVALID_ARG, "alpha outside [0, n_labels)");
    if (!w_out || !a_out || !a_out[0] || !a_out[1]) return set_error(MC_ERR_INVALID_ARG, "null output");
    MC_HIP(launch_expand_build(g, data, lam, v_kind, v_trunc, labels, alpha, w_out, a_out[0], a_out[1], s));
    return MC_OK;
}

int mc_ml_energy(mc_ctx* c, const mc_grid* grid, int n_labels, const float* data, const float* const* lam,
                 int v_kind, float v_trunc, const int32_t* labels, double* energy_out, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    Geo g;
    int rc = check_ml(c, grid, n_labels, data, lam, v_kind, v_trunc, labels, &g, s);
    if (rc) return rc;
    if (!energy_out) return set_error(MC_ERR_INVALID_ARG, "energy_out is null");
    return read_energy(c, g, data, lam, v_kind, v_trunc, labels, energy_out, s);
}

int mc_alpha_expansion(mc_ctx* c, const mc_grid* grid, int n_labels, const float* data, const float* const* lam,
                       int v_kind, float v_trunc, int32_t* labels, int max_cycles, mc_ml_stats* stats,
                       const mc_opts* opts, void* stream)
{
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)stream;
    Geo g;
    int rc = check_ml(c, grid, n_labels, data, lam, v_kind, v_trunc, labels, &g, s);
    if (rc) return rc;
    if (!stats) return set_error(MC_ERR_INVALID_ARG, "stats is null");
    if (max_cycles < 1) return set_error(MC_ERR_INVALID_ARG, "max_cycles must be >= 1");
    mc_opts o;
    if (opts) o = *opts;
    else mc_opts_default(&o);
    const size_t n = (size_t)g.n;
    if (o.flags & MC_VALIDATE) {
        // weights: finite, >= 0, zero on the last column / row (the checks of
        // mc_tv_solve, with the first label's costs standing in for w); costs: finite
        MC_HIP(launch_validate(g, data, lam, c->partials, c->dout, s));
        MC_HIP(hipMemcpyAsync(c->hout, c->dout, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        MC_HIP(hipStreamSynchronize(s));
        if (c->hout[1] > 0) return set_error(MC_ERR_NONFINITE, "non-finite value in data or lam");
        if (c->hout[0] > 0) return set_error(MC_ERR_NEGATIVE_WEIGHT, "negative weight or non-zero weight on a last slice");
        MC_HIP(launch_count_nonfinite(data, n_labels * g.n, c->partials, c->dout, s));
        MC_HIP(hipMemcpyAsync(c->hout, c->dout, sizeof(double), hipMemcpyDeviceToHost, s));
        MC_HIP(hipStreamSynchronize(s));
        if (c->hout[0] > 0) return set_error(MC_ERR_NONFINITE, "non-finite value in data");
    }
    const bool warm = (o.flags & MC_WARM_MOVES) != 0;
    // the warm state is a point of the two-set splitting (n values)
    if (warm && o.variant != MC_VARIANT_AUTO && o.variant != MC_VARIANT_TWO_SET)
        return set_error(MC_ERR_INVALID_ARG, "MC_WARM_MOVES needs the two-set splitting (variant AUTO or TWO_SET)");
    if ((rc = ensure_ml_ws(c, n, warm ? 4 + 2 * (size_t)n_labels : 3))) return rc;
    float* w = c->mlbuf;
    float* ax = c->mlbuf + n;
    float* ay = c->mlbuf + 2 * n;
    float* z0 = c->mlbuf + 3 * n;    // warm moves: start state
    float* hist = c->mlbuf + 4 * n;  // warm moves: [label][x; p1]
    std::vector<char> have(warm ? n_labels : 0, 0);
    // applied-move count when each label's move was last solved: while no
    // move has been applied since, the labels are those of that move, which
    // was rejected (an exact move finds nothing again) or applied (expansions
    // of alpha from its result are expansions from the labels before it), so
    // the move is skipped without changing the applied moves or the result
    std::vector<int> seen(n_labels, -1);
    const float* a[2] = {ax, ay};
    mc_grid g2 = *grid;
    g2.conn = 4;
    mc_opts so = o;
    so.flags &= ~(uint32_t)MC_VALIDATE;  // move problems are valid by construction

    *stats = mc_ml_stats{};
    double e = 0.0;
    if ((rc = read_energy(c, g, data, lam, v_kind, v_trunc, labels, &e, s))) return rc;
    stats->energy0 = e;
    bool settled = false;
    for (int cycle = 0; cycle < max_cycles && !settled; ++cycle) {
        ++stats->cycles;
        bool improved = false;
        for (int alpha = 0; alpha < n_labels; ++alpha) {
            if (seen[alpha] == stats->accepted) {
                ++stats->skipped;
                continue;
            }
            MC_HIP(launch_expand_build(g, data, lam, v_kind, v_trunc, labels, alpha, w, ax, ay, s));
            const float* start = nullptr;
            if (warm && have[alpha]) {
                float* h = hist + (size_t)alpha * 2 * n;
                if ((rc = mc_ws_warm_state(c, &g2, h, ax, 1.f, z0, stream))) return rc;
                start = z0;
            }
            mc_stats st;
            rc = mc_tv_solve(c, &g2, w, a, start, nullptr, c->mlsel, nullptr, &st, &so, stream);
            if (rc < 0) return rc;
            if (warm) {
                // every solve ends with a certificate: the context then holds its
                // primal estimate (xt) and the row duals of that iteration (p)
                float* h = hist + (size_t)alpha * 2 * n;
                MC_HIP(hipMemcpyAsync(h, c->xt, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
                MC_HIP(hipMemcpyAsync(h + n, c->p, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
                have[alpha] = 1;
            }
            ++stats->moves;
            stats->dr_iters += st.iters;
            if (rc == MC_NOT_CONVERGED) ++stats->uncertified;
            if (st.energy < 0.0) {  // E(f with the move) = E(f) + st.energy
                MC_HIP(launch_expand_apply(g.n, alpha, c->mlsel, labels, s));
                ++stats->accepted;
                improved = true;
            }
            seen[alpha] = stats->accepted;
        }
        settled = !improved;
    }
    if ((rc = read_energy(c, g, data, lam, v_kind, v_trunc, labels, &e, s))) return rc;
    stats->energy = e;
    stats->status = settled && stats->uncertified == 0 ? MC_OK : MC_NOT_CONVERGED;
    stats->ms = (float)std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return stats->status;
}

}  // extern "C"
