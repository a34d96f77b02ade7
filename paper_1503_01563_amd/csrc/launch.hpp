// launch.hpp -- host-side launchers of the libmc kernels (sweeps.hip, reduce.hip,
// batch.hip, grid8.hip, variants.hip, multilabel.hip) and the structs they share.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "chain.hpp"

namespace mc {

// Grid geometry: [D][H][W], W contiguous; 2D grids have D = 1.
struct Geo {
    int D, H, W;
    int n;
    int ndim;
    int whole = 0;  // sweeps: every chain in one piece, one lane per chain (no overlap, no restarts)
    int stream = 1;  // value sweeps of volumes may take streamed long pieces (0: short pieces only)
    int* restarts = nullptr;  // piece sweeps add {lanes that restarted, lanes run} here (null: no count)
};

__host__ __device__ inline int geo_extent(const Geo& g, int axis)
{
    return axis == 0 ? g.W : (axis == 1 ? g.H : g.D);
}
__host__ __device__ inline int geo_stride(const Geo& g, int axis)
{
    return axis == 0 ? 1 : (axis == 1 ? g.W : g.W * g.H);
}
__host__ __device__ inline int geo_nchains(const Geo& g, int axis) { return g.n / geo_extent(g, axis); }

// How a family's chains are cut into pieces for the sweep kernels: pieces of
// `len` positions (the last may be shorter), each scanned from `overlap`
// positions earlier and past its end by up to `tail` positions from LDS.
struct PieceCfg {
    int len, pieces, overlap, tail;
    int reach_lo, reach_hi;  // LDS reserve in front of / behind the piece
};

// Pieces for a family: about `want` work items (16 to 64 positions per piece).
// launch_items is the number of work items of the whole launch the family is
// part of (0: this family alone); launches of at most kLatencyItems items run
// about one wave per SIMD and get a longer overlap (12 instead of 8), so that
// almost no piece has to restart its scans.  overlap > 0 sets the overlap
// instead (the batched autotuner's candidates), tail >= 0 the tail.
PieceCfg piece_config(const Geo& g, int axis, int want, int launch_items, int overlap = 0, int tail = -1,
                      int min_len = 16);
constexpr int kDefaultItems = 4096;
constexpr int kLatencyItems = 2048;
// dynamic LDS bytes of a sweep launch with these pieces
size_t piece_lds_bytes(const PieceCfg& cfg);

constexpr int kReduceBlocks = 2048;  // blocks of the reduction kernels (fixed: deterministic)
constexpr int kReduceThreads = 256;
static_assert(kReduceBlocks % kReduceThreads == 0, "the finalize kernels read whole rounds of partials");
// Rounding readout: S_t = {x > tau_t} for the decreasing threshold ladder
// tau0 * (1, 1e-1, 1e-2, 1e-3, 0, -1e-3, -1e-2, -1e-1, -1).
constexpr int kNumTau = 9;
constexpr int kCertValues = kNumTau + 2;  // E(S_t) for every t, TV gap, LB

inline void tau_ladder(float tau0, float* taus)
{
    const float f[kNumTau] = {1.f, 1e-1f, 1e-2f, 1e-3f, 0.f, -1e-3f, -1e-2f, -1e-1f, -1.f};
    for (int t = 0; t < kNumTau; ++t) taus[t] = tau0 * f[t];
}

// Standalone prox of every chain along `axis` (x = prox(v), p = clipped duals).
hipError_t launch_prox(const Geo& g, int axis, const float* v, const float* a, float* x,
                       float* p, hipStream_t s);

// Two-set splitting, rows: q1 = prox_rows(z); p1 (clipped duals) when non-null.
hipError_t launch_dr2_rows(const Geo& g, const float* z, const float* a_x, float* q1, float* p1,
                           hipStream_t s);

// Two-set splitting, columns: t = q1 - (z - q1) - w, q2 = prox_cols(t),
// znew = (z - q1) + q2; p2 when non-null.
hipError_t launch_dr2_cols(const Geo& g, const float* q1, const float* z, float* znew,
                           const float* w, const float* a_y, float* p2, hipStream_t s);

// Product space, non-final families 0..nfam-1 (nfam <= 2, one launch):
// q_j = prox_j(z_j) at q + j*n; p_j at p + j*n when p != nullptr.
hipError_t launch_drp_sweeps(const Geo& g, int nfam, const float* z, const float* const* a,
                             float* q, float* p, hipStream_t s);

// Product space, final family (axis r-1) fused with the average over L:
// y_j = z_j - q_j, znew_j = y_j - (2Y - Z - u)/r; p_{r-1} when non-null.
// 8-connected grids: the product-space sweeps of rows and columns and the
// row prox of the straightened zig-zag chains (geometry gz) in one launch
hipError_t launch_sweeps8(const Geo& g, const float* z, const float* const* a, float* q, float* p, const Geo& gz,
                          const float* zzv, const float* zza, float* zzx, float* zzp, hipStream_t s);
// volumes: the product-space sweeps of all three families in one launch,
// q_j and p_j (nullable) at offsets j*n; the averaging step is launch_combine
hipError_t launch_sweeps3(const Geo& g, const float* z, const float* const* a, float* q, float* p, hipStream_t s);
hipError_t launch_drp_final(const Geo& g, int r, const float* z, float* znew, const float* q,
                            const float* a_last, const float* w, float* p_last, hipStream_t s);

// Product space, first iteration from z = 0 (all proxes vanish):
// zn_j = -(w * (1/r)) for j < r.
hipError_t launch_cold_product(const Geo& g, int r, const float* w, float* zn, hipStream_t s);

// ---- 8-connected 2D grids (a[0..3]: along W, along H, diagonal, anti-diagonal) ----

// Zig-zag families 2 and 3 straightened into chains [2(H-1)][W] (values from
// z2 / z3, edge weights from the diagonal / anti-diagonal arrays).
hipError_t launch_zz_gather(int H, int W, const float* z2, const float* z3, const float* add, const float* aad,
                            float* zv, float* za, hipStream_t s);
// Averaging step over the four families, zn_j = y_j - (2Y - Z + w)/4: z holds
// the four families per vertex, q01 the row and column prox, zx the zig-zag
// prox as straightened chains (q_2, q_3 = z off the families' paths).  Writes
// zn per vertex, zn of families 2 and 3 straightened into zv, and, when zp is
// not null, the diagonal and anti-diagonal duals per cell into pdd / pad.
hipError_t launch_combine8(int H, int W, const float* z, const float* q01, const float* zx, const float* zp,
                           const float* w, float* zn, float* zv, float* pdd, float* pad, hipStream_t s);
// ---- FP64 state (MC_FP64_STATE, fp64.hip): one lane per whole chain ----------
// Duals (nullable) are written as FP32 clipped to their boxes.
hipError_t launch_dr2_rows64(const Geo& g, const double* z, const float* a_x, double* q1, float* p1, hipStream_t s);
hipError_t launch_dr2_cols64(const Geo& g, const double* q1, const double* z, double* znew, const float* w,
                             const float* a_y, float* p2, hipStream_t s);
hipError_t launch_family64(const Geo& g, int axis, const double* z, const float* a, double* q, float* p,
                           hipStream_t s);
// z_j' = y_j - (2Y - Z + w) / r for r = 2 or 3 families
hipError_t launch_combine64(size_t n, int r, const double* z, const double* q, const float* w, double* zn,
                            hipStream_t s);
hipError_t launch_f32_to_f64(size_t n, const float* x, double* y, hipStream_t s);
hipError_t launch_f64_to_f32(size_t n, const double* x, float* y, hipStream_t s);

// z_j' = y_j - (2Y - Z + w) / 3 for a volume's three families
hipError_t launch_combine3(size_t n, const float* z, const float* q, const float* w, float* zn, hipStream_t s);
// Certificate, energy and input checks with the diagonal edges.
hipError_t launch_cert8(const Geo& g, const float* w, const float* const* a, const float* const* p, float tau0,
                        float* xc, double* partials, double* out, hipStream_t s);
hipError_t launch_energy8(const Geo& g, const float* w, const float* const* a, const uint8_t* labels,
                          double* partials, double* out, hipStream_t s);
hipError_t launch_validate8(const Geo& g, const float* w, const float* const* a, double* partials, double* out,
                            hipStream_t s);

// ---- elementwise steps of the other outer iterations (BCD, AP, FISTA) ----------
hipError_t launch_neg(size_t n, const float* w, float* x, hipStream_t s);                     // x = -w
hipError_t launch_add(size_t n, const float* x, const float* y, float* v, hipStream_t s);     // v = x + y
hipError_t launch_rsub(size_t n, const float* a, float* d, hipStream_t s);                   // d = a - d
hipError_t launch_sub(size_t n, const float* a, float* d, hipStream_t s);                    // d = d - a
hipError_t launch_diff(size_t n, const float* a, const float* b, float* d, hipStream_t s);    // d = a - b
hipError_t launch_scale(size_t n, float f, const float* a, float* d, hipStream_t s);     // d = f a
// AP: y_j = l_j - q_j, x = -w - sum y_j, l_j = y_j + x / r (cold: l_j = -w / r)
hipError_t launch_ap_update(size_t n, int r, float* lam, const float* q, const float* w, bool cold, hipStream_t s);
// FISTA: yt = y + beta (y - yp), xt = -w - sum yt_j, v_j = yt_j + xt / r
hipError_t launch_fista_pre(size_t n, int r, const float* y, const float* yp, float beta, const float* w, float* v,
                            hipStream_t s);

// Certificate from the edge duals p: primal xc = -w - sum_j D_j^T p_j (FP32
// out), then out[kCertValues] = {E(S_t) for the ladder, TV gap, LB} in FP64.
// partials needs kCertValues * kReduceBlocks doubles.
hipError_t launch_cert(const Geo& g, const float* w, const float* const* a,
                       const float* const* p, float tau0, float* xc, double* partials,
                       double* out, hipStream_t s);

hipError_t launch_labels(const Geo& g, const float* xc, float tau, uint8_t* labels, hipStream_t s);

// ---- batched two-set solves -------------------------------------------------

// One 2D grid of a batch (device table entry).  Results are written on the
// device: `done` once the certificate is below the tolerance, with the
// iteration and a wall-clock stamp.
struct BatchGrid {
    Geo g;
    const float* w;
    const float* ax;
    const float* ay;
    float* z[2];     // state, ping-pong by iteration parity
    float* q1;
    float* p;        // 2n: row duals then column duals
    float* xc;       // primal estimate
    uint8_t* labels;
    float* x_out;    // nullable
    PieceCfg cr, cc;     // pieces of the row and column sweeps
    int item0_r, item0_c;  // first work item of this grid in each sweep launch
    int blk0, nblk;      // reduction blocks of this grid
    int done, iters, checks, tau_idx;
    double e[kNumTau], tvgap, lb, cert;
    unsigned long long t_done;
};

struct BatchLaunch {
    BatchGrid* tab;
    const int* item_grid_r;  // sweep work item -> grid (rows)
    const int* item_grid_c;  // sweep work item -> grid (columns)
    const int* blk_grid;     // reduction block -> grid
    int n_grids, items_r, items_c, blocks;
    size_t lds_r, lds_c;     // dynamic LDS of the sweep launches
};

// One two-set iteration over every unfinished grid; parity selects the state
// buffer read.  With duals, the row/column duals are written for the check.
// cold: the first iteration from z = 0, whose row proxes are 0 (q1, and the
// row duals when asked for, are zeroed instead of swept).
hipError_t launch_batch_iteration(const BatchLaunch& b, int parity, bool duals, hipStream_t s,
                                  bool cold = false);
// K iterations (from state parity p0, the last with duals) over every
// unfinished grid as one cooperative launch of `blocks` resident waves (a
// multiple of 8) that share out each phase's work items and meet at a
// device-wide barrier between phases.  ctl: 8 ints, zero before the launch; ctl[4] != 0 after it
// means a barrier gave up (the results are then invalid; ctl[5..7]: arrivals
// seen, phase, workgroups).  Phase -1 is a barrier before any work: when it
// gives up, fewer workgroups than launched were resident (ctl[5] of them)
// and the launch changed nothing.
int batch_persistent_blocks(size_t lds);
hipError_t launch_batch_persistent(const BatchLaunch& b, int* ctl, int p0, int K, int blocks, hipStream_t s);
// Certificate of every unfinished grid: grids whose certificate is below
// gap_tol are marked done at iteration *iter_dev.
hipError_t launch_batch_check(const BatchLaunch& b, float tau0, double gap_tol, const int* iter_dev,
                              double* partials, hipStream_t s);
hipError_t launch_batch_labels(const BatchLaunch& b, float tau0, hipStream_t s);
// The number of grids whose done flag is not set, to *out (device).
hipError_t launch_batch_undone(const BatchLaunch& b, int* out, hipStream_t s);
hipError_t launch_set_int(int* dst, int value, hipStream_t s);
hipError_t launch_stamp(unsigned long long* dst, hipStream_t s);

hipError_t launch_energy(const Geo& g, const float* w, const float* const* a,
                         const uint8_t* labels, double* partials, double* out, hipStream_t s);

// Input checks: out[0] = #negative weights or non-zero weights on a last slice,
// out[1] = #non-finite values in w and a.
hipError_t launch_validate(const Geo& g, const float* w, const float* const* a,
                           double* partials, double* out, hipStream_t s);

// MC_DEBUG: out[0] = duals outside |p_j| <= a_j (or not finite), out[1] =
// non-zero duals on a family's last slice.
hipError_t launch_debug_duals(const Geo& g, const float* const* a, const float* const* p, double* partials,
                              double* out, hipStream_t s);

// Non-finite entries in an array (out[0]).
hipError_t launch_count_nonfinite(const float* x, int n, double* partials, double* out,
                                  hipStream_t s);

// ---- alpha-expansion (multilabel.hip; checks and energy in reduce.hip) ----
// out[0] = number of labels outside [0, L)
hipError_t launch_check_labels(int n, int L, const int32_t* f, double* partials, double* out, hipStream_t s);
// out[0] = E(f) of the multi-label energy (2D grid, lam[0] along W, lam[1] along H)
hipError_t launch_ml_energy(const Geo& g, const float* data, const float* const* lam, int kind, float trunc,
                            const int32_t* f, double* partials, double* out, hipStream_t s);
// binary problem of the expansion move of `alpha` from f: w, a_x, a_y
hipError_t launch_expand_build(const Geo& g, const float* data, const float* const* lam, int kind, float trunc,
                               const int32_t* f, int alpha, float* w, float* ax, float* ay, hipStream_t s);
// f_i = alpha where sel_i != 0
hipError_t launch_expand_apply(int n, int alpha, const uint8_t* sel, int32_t* f, hipStream_t s);

}  // namespace mc
