// ctx.hpp -- the library context and error helpers shared by the C-ABI files.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "launch.hpp"
#include "mc.h"

struct mc_ctx {
    int device = 0;
    size_t cap_n = 0;   // voxels the single-grid workspace was sized for
    int cap_r = 0;      // families the single-grid workspace was sized for
    float* z = nullptr;      // r*n splitting state
    float* z2 = nullptr;     // r*n second state buffer (the sweeps never update in place)
    float* y = nullptr;      // r*n: row prox q1 (two-set) or the prox outputs q_j (product space)
    float* p = nullptr;      // r*n edge duals (check iterations)
    float* xt = nullptr;     // n   primal estimate -w - sum_j D_j^T p_j (check iterations)
    double* partials = nullptr;  // kReduceBlocks * kCertValues
    double* dout = nullptr;      // kCertValues doubles
    double* hout = nullptr;      // kCertValues doubles, pinned host
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int* scnt = nullptr;     // 2 ints: restarted / run lanes of the probe sweep
    int* scnt_h = nullptr;   // 2 ints, pinned host
    std::vector<hipEvent_t> prof_ev;  // MC_PROFILE: start/stop pairs of sweep launches

    // batched solves
    hipStream_t bstream = nullptr;   // capture / replay stream (default priority)
    size_t bcap = 0;                 // floats in bbuf
    float* bbuf = nullptr;           // per-grid state buffers, packed
    size_t bmeta_cap = 0;            // bytes in bmeta
    char* bmeta = nullptr;           // table, maps, partials, counters
    int* bctl = nullptr;             // persistent batch launch control words (fine-grained memory)
    std::map<size_t, int> persist_blocks;  // LDS bytes -> workgroups found resident at once
    std::map<unsigned long long, std::pair<int, int>> tuned_items;  // batch signature -> work items per
                                                                    // launch, piece overlap (0: by mode)

    // 8-connected grids: prox outputs of the four families, straightened zig-zag chains
    size_t g8cap = 0;       // floats in g8buf
    float* g8buf = nullptr;

    // MC_FP64_STATE: z, z2, q of the FP64 iteration (3 * r * n doubles)
    size_t d64cap = 0;      // doubles in d64buf
    double* d64buf = nullptr;

    // other outer iterations (BCD, AP, FISTA)
    size_t vcap = 0;        // floats in vbuf
    float* vbuf = nullptr;

    // alpha-expansion: move problem (w, a_x, a_y), move labels
    size_t mlcap = 0;       // pixels the buffers hold
    size_t mlper = 0;       // floats per pixel in mlbuf
    float* mlbuf = nullptr; // mlper * mlcap floats
    uint8_t* mlsel = nullptr;  // mlcap bytes

    // warm-start network
    size_t ncap = 0;        // bytes in nbuf
    char* nbuf = nullptr;   // packed weights, activations, gradients, partials
};

namespace mc {

// Largest node count (and n_labels * nodes) accepted: the kernels index with
// int and step grid-stride loops by at most 2^20, so 2^24 of headroom below
// 2^31 keeps every index and step in range.
constexpr int64_t kMaxNodes = (int64_t(1) << 31) - (int64_t(1) << 24);

int set_error(int code, const std::string& msg);

// grid -> Geo with the checks every entry point shares (dims, size limits, conn)
int make_geo(const mc_grid* grid, Geo* g);

// non-null context, its device made current
int check_ctx(mc_ctx* c);

inline int hip_error(hipError_t e, const char* where)
{
    return set_error(MC_ERR_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

}  // namespace mc

#define MC_HIP(call)                                         \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return mc::hip_error(e_, #call); \
    } while (0)
