// convnet.hip -- the warm-start network: a 4-layer 3x3 convolutional net that
// maps a 2D cut problem (w, a_x, a_y) to a guess of the TV solution x0 and of
// the row-family edge duals p1, from which the two-set splitting starts
// (z0 = c x0 + D_rows^T clip(p1); reusing a good splitting state is the warm
// start of Sec. 4.4 and 6.1 of the paper).
//
//   features  f = (w / 20, a_x / 10, a_y / 10)
//   h_l = relu(conv3x3(h_{l-1}, W_l) + b_l), l = 1..3, 32 channels
//   o   = conv3x3(h_3, W_4) + b_4, 2 channels (x0, p1)
//
// conv3x3 is a zero-padded cross-correlation,
//   out[y, x, co] = b[co] + sum_{ky,kx,ci} W[co, ky, kx, ci] in[y+ky-1, x+kx-1, ci].
//
// Every convolution is a contraction over k = (tap, ci), run as BF16 MFMA
// (v_mfma_f32_16x16x32_bf16, FP32 accumulate).  Forward and input gradient:
// D[row][pixel] = sum_k A[row][k] B[k][pixel] with A the packed weights (kept
// in registers) and B gathered from an LDS halo tile of the input; 16 pixels
// of one image row per MFMA.  Weight gradient: D[co][k] = sum_pixel
// g[co][pixel] in[pixel + tap][ci], 32 pixels per MFMA, the bias gradient an
// extra column of ones; partial sums per workgroup, reduced in a fixed order.
//
// Operand layout of the MFMA (one wave): lane l holds A[l % 16][8 (l / 16) + e]
// and B[8 (l / 16) + e][l % 16] for e = 0..7, and receives D[4 (l / 16) + r][l % 16]
// for r = 0..3.
//
// Storage: activations and their gradients are [b][y][x][32] BF16 (pixel-major,
// 64 B per pixel); the output and its gradient are [b][2][H][W] FP32 planes.
// Parameters are one FP32 vector, per layer W (co, ky, kx, ci) then b.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <string>

#include "ctx.hpp"
#include "mc.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kC = 32;          // hidden channels
constexpr int kT = 16;          // output tile edge in pixels
constexpr int kTH = kT + 2;     // with halo
constexpr int kThreads = 256;   // four waves, four tile rows each
constexpr int kLayers = 4;
constexpr int kCin[kLayers] = {3, 32, 32, 32};
constexpr int kCout[kLayers] = {32, 32, 32, 2};
constexpr int kWgradBlocks = 512;   // weight-gradient partial sums
constexpr int kLossBlocks = 256;

constexpr int kdim(int cin) { return 9 * cin; }
constexpr int kpad32(int k) { return (k + 31) / 32 * 32; }
constexpr int npad16(int k) { return (k + 15) / 16 * 16; }

constexpr int param_w_off(int l)
{
    int off = 0;
    for (int i = 0; i < l; ++i) off += kCout[i] * kdim(kCin[i]) + kCout[i];
    return off;
}
constexpr int param_b_off(int l) { return param_w_off(l) + kCout[l] * kdim(kCin[l]); }
constexpr int kParams = param_w_off(kLayers);
static_assert(kParams == 19970, "parameter count");

// packed BF16 weights: forward [rows = 16 * ceil(cout / 16)][kpad32(9 cin)],
// input gradient [rows = cin][kpad32(9 cout)] with tap flipped
constexpr int fwd_rows(int l) { return (kCout[l] + 15) / 16 * 16; }
constexpr size_t fwd_elems(int l) { return (size_t)fwd_rows(l) * kpad32(kdim(kCin[l])); }
constexpr size_t bwd_elems(int l) { return (size_t)kCin[l] * kpad32(9 * kCout[l]); }

__device__ __forceinline__ __bf16 bf(float f) { return static_cast<__bf16>(f); }

__device__ __forceinline__ floatx4 mfma(const bf16x8& a, const bf16x8& b, const floatx4& c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// ---- layer input sources (value of channel c at pixel (y, x) of image b) --------

struct SrcFeat {  // network input features from the three FP32 planes
    const float *w, *ax, *ay;
    int H, W;
    __device__ float get(int b, int y, int x, int c) const
    {
        const size_t i = ((size_t)b * H + y) * W + x;
        return c == 0 ? w[i] * (1.f / 20.f) : (c == 1 ? ax[i] : ay[i]) * (1.f / 10.f);
    }
};

struct SrcPlanes2 {  // two FP32 planes per image ([b][2][H][W])
    const float* p;
    int H, W;
    __device__ float get(int b, int y, int x, int c) const
    {
        return p[(((size_t)b * 2 + c) * H + y) * W + x];
    }
};

struct SrcAct {  // BF16 [b][y][x][32]
    const __bf16* p;
    int H, W;
};

// Stage the (kTH x kTH) halo tile with top-left input pixel (y0 - 1, x0 - 1);
// zero outside the image.
template <int CIN, class Src>
__device__ __forceinline__ void fill_halo(const Src& src, __bf16* tile, int b, int y0, int x0, int H, int W)
{
    for (int i = threadIdx.x; i < kTH * kTH * CIN; i += kThreads) {
        const int pix = i / CIN, c = i % CIN;
        const int gy = y0 - 1 + pix / kTH, gx = x0 - 1 + pix % kTH;
        const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
        tile[i] = bf(in ? src.get(b, gy, gx, c) : 0.f);
    }
}

template <int CIN>
__device__ __forceinline__ void fill_halo(const SrcAct& src, __bf16* tile, int b, int y0, int x0, int H, int W)
{
    static_assert(CIN == kC, "activation tiles have 32 channels");
    // 16-byte chunks: 4 per pixel
    for (int i = threadIdx.x; i < kTH * kTH * 4; i += kThreads) {
        const int pix = i >> 2, q = i & 3;
        const int gy = y0 - 1 + pix / kTH, gx = x0 - 1 + pix % kTH;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (gy >= 0 && gy < H && gx >= 0 && gx < W)
            v = *reinterpret_cast<const uint4*>(src.p + (((size_t)b * H + gy) * W + gx) * kC + 8 * q);
        *reinterpret_cast<uint4*>(tile + pix * kC + 8 * q) = v;
    }
}

// Stage the (kT x kT) tile without halo, [y][x][CIN]; zero outside the image.
template <int CIN, class Src>
__device__ __forceinline__ void fill_plain(const Src& src, __bf16* tile, int b, int y0, int x0, int H, int W)
{
    for (int i = threadIdx.x; i < kT * kT * CIN; i += kThreads) {
        const int pix = i / CIN, c = i % CIN;
        const int gy = y0 + pix / kT, gx = x0 + pix % kT;
        const bool in = gy < H && gx < W;
        tile[i] = bf(in ? src.get(b, gy, gx, c) : 0.f);
    }
}

template <int CIN>
__device__ __forceinline__ void fill_plain(const SrcAct& src, __bf16* tile, int b, int y0, int x0, int H, int W)
{
    static_assert(CIN == kC, "activation tiles have 32 channels");
    for (int i = threadIdx.x; i < kT * kT * 4; i += kThreads) {
        const int pix = i >> 2, q = i & 3;
        const int gy = y0 + pix / kT, gx = x0 + pix % kT;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (gy < H && gx < W)
            v = *reinterpret_cast<const uint4*>(src.p + (((size_t)b * H + gy) * W + gx) * kC + 8 * q);
        *reinterpret_cast<uint4*>(tile + pix * kC + 8 * q) = v;
    }
}

// B operand of k-step s for output pixel column li of tile row ty: the eight
// k = 32 s + 8 lg + e values in[ty + ky, li + kx, ci] with k = (3 ky + kx) CIN + ci.
template <int CIN>
__device__ __forceinline__ bf16x8 gather_k(const __bf16* tile, int ty, int li, int lg, int s)
{
    bf16x8 v;
    if constexpr (CIN == kC) {
        const int ky = s / 3, kx = s % 3;
        v = *reinterpret_cast<const bf16x8*>(tile + ((ty + ky) * kTH + li + kx) * kC + 8 * lg);
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = 32 * s + 8 * lg + e;
            const int kk = k < 9 * CIN ? k : 0;  // padding columns read a valid slot
            const int tap = kk / CIN, c = kk % CIN;
            const __bf16 t = tile[((ty + tap / 3) * kTH + li + tap % 3) * CIN + c];
            v[e] = k < 9 * CIN ? t : bf(0.f);
        }
    }
    return v;
}

// ---- epilogues of the convolution kernel ------------------------------------------
// acc[mt][r] is output row 16 mt + 4 lg + r at pixel (y, x).

struct EpiReluAct {  // hidden layer: + bias, ReLU, BF16 activation
    const float* bias;
    __bf16* out;
    int H, W;
    template <int MT>
    __device__ void store(int b, int y, int x, int lg, const floatx4 (&acc)[MT]) const
    {
        __bf16* o = out + (((size_t)b * H + y) * W + x) * kC;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            bf16x4 v;
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] = bf(fmaxf(acc[mt][r] + bias[16 * mt + 4 * lg + r], 0.f));
            *reinterpret_cast<bf16x4*>(o + 16 * mt + 4 * lg) = v;
        }
    }
};

struct EpiOutput {  // last layer: + bias, two FP32 planes
    const float* bias;
    float* out;
    int H, W;
    template <int MT>
    __device__ void store(int b, int y, int x, int lg, const floatx4 (&acc)[MT]) const
    {
        if (lg != 0) return;
        out[(((size_t)b * 2 + 0) * H + y) * W + x] = acc[0][0] + bias[0];
        out[(((size_t)b * 2 + 1) * H + y) * W + x] = acc[0][1] + bias[1];
    }
};

struct EpiGradMask {  // input gradient: zero where the layer input (a ReLU output) is 0
    const __bf16* act;
    __bf16* out;
    int H, W;
    template <int MT>
    __device__ void store(int b, int y, int x, int lg, const floatx4 (&acc)[MT]) const
    {
        const size_t base = (((size_t)b * H + y) * W + x) * kC;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const bf16x4 a = *reinterpret_cast<const bf16x4*>(act + base + 16 * mt + 4 * lg);
            bf16x4 v;
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] = bf((float)a[r] > 0.f ? acc[mt][r] : 0.f);
            *reinterpret_cast<bf16x4*>(out + base + 16 * mt + 4 * lg) = v;
        }
    }
};

// One 16 x 16 pixel tile per workgroup (grid: tiles_x, tiles_y, batch); wave w
// computes tile rows 4w .. 4w+3.  wpk: packed weights [16 MT][kpad32(9 CIN)].
template <int CIN, int MT, class Src, class Epi>
__global__ void __launch_bounds__(kThreads) k_conv(Src src, const __bf16* __restrict__ wpk, Epi epi, int H, int W)
{
    constexpr int KP = kpad32(kdim(CIN)), S = KP / 32;
    __shared__ __attribute__((aligned(16))) __bf16 tile[kTH * kTH * CIN];
    const int b = blockIdx.z, y0 = blockIdx.y * kT, x0 = blockIdx.x * kT;
    fill_halo<CIN>(src, tile, b, y0, x0, H, W);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    bf16x8 A[MT][S];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int s = 0; s < S; ++s)
            A[mt][s] = *reinterpret_cast<const bf16x8*>(wpk + (size_t)(16 * mt + li) * KP + 32 * s + 8 * lg);
    __syncthreads();
#pragma unroll 1
    for (int r = 0; r < 4; ++r) {
        const int ty = 4 * wave + r;
        floatx4 acc[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[mt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const bf16x8 Bv = gather_k<CIN>(tile, ty, li, lg, s);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[mt] = mfma(A[mt][s], Bv, acc[mt]);
        }
        const int y = y0 + ty, x = x0 + li;
        if (y < H && x < W) epi.template store<MT>(b, y, x, lg, acc);
    }
}

// Weight (and bias) gradient partial sums.  Output matrix D[co][k], k < 9 CIN
// the weight column (tap, ci), k == 9 CIN the bias column; wave w owns output
// tiles w, w + 4, ...  Workgroup g handles pixel tiles g, g + grid, ... and
// writes its partial [16 MT][NP] to partial + g * 16 MT * NP.
template <int CIN, int COUT, class SrcIn, class SrcG>
__global__ void __launch_bounds__(kThreads) k_wgrad(SrcIn in, SrcG gsrc, float* __restrict__ partial, int H, int W,
                                                     int tiles_x, int tiles_y, int batch)
{
    constexpr int K = kdim(CIN), NP = npad16(K + 1), NT = NP / 16, MT = (COUT + 15) / 16;
    constexpr int TILES = MT * NT, PER = (TILES + 3) / 4;
    __shared__ __attribute__((aligned(16))) __bf16 tin[kTH * kTH * CIN];
    __shared__ __attribute__((aligned(16))) __bf16 tg[kT * kT * COUT];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;

    // the B column of each owned output tile: kind 0 weight (tap, ci), 1 bias, 2 padding
    int col_off[PER], col_kind[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int t = wave + 4 * i, nt = t % NT;
        const int k = 16 * nt + li;
        const int kk = k < K ? k : 0;  // bias and padding columns read a valid slot
        const int tap = kk / CIN, c = kk % CIN;
        col_kind[i] = k < K ? 0 : (k == K ? 1 : 2);
        col_off[i] = ((tap / 3) * kTH + tap % 3) * CIN + c;
    }
    floatx4 acc[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) acc[i] = floatx4{0.f, 0.f, 0.f, 0.f};

    const int total = tiles_x * tiles_y * batch;
#pragma unroll 1
    for (int tid = blockIdx.x; tid < total; tid += gridDim.x) {
        const int tx = tid % tiles_x, ty = (tid / tiles_x) % tiles_y, b = tid / (tiles_x * tiles_y);
        const int y0 = ty * kT, x0 = tx * kT;
        fill_halo<CIN>(in, tin, b, y0, x0, H, W);
        fill_plain<COUT>(gsrc, tg, b, y0, x0, H, W);
        __syncthreads();
#pragma unroll 1
        for (int ks = 0; ks < kT * kT / 32; ++ks) {
            // pixels of this k-step for lane group lg: row 2 ks + lg / 2, columns 8 (lg & 1) + e
            const int row = 2 * ks + (lg >> 1), xb = 8 * (lg & 1);
            bf16x8 A[MT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const int co = 16 * mt + li, cc = co < COUT ? co : 0;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const __bf16 t = tg[(row * kT + xb + e) * COUT + cc];
                    A[mt][e] = co < COUT ? t : bf(0.f);
                }
            }
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const int t = wave + 4 * i;
                if (t >= TILES) continue;
                const int mt = t / NT;
                bf16x8 Bv;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const __bf16 v = tin[(row * kTH + xb + e) * CIN + col_off[i]];
                    Bv[e] = col_kind[i] == 0 ? v : bf(col_kind[i] == 1 ? 1.f : 0.f);
                }
                acc[i] = mfma(A[mt], Bv, acc[i]);
            }
        }
        __syncthreads();
    }
    float* out = partial + (size_t)blockIdx.x * (16 * MT) * NP;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int t = wave + 4 * i;
        if (t >= TILES) continue;
        const int mt = t / NT, nt = t % NT;
#pragma unroll
        for (int r = 0; r < 4; ++r) out[(size_t)(16 * mt + 4 * lg + r) * NP + 16 * nt + li] = acc[i][r];
    }
}

// grad_W[co][k] and grad_b[co] as fixed-order sums of the partials: one wave
// per entry, lane l sums partials l, l + 64, ..., then a fixed shuffle tree.
template <int CIN, int COUT>
__global__ void __launch_bounds__(kThreads) k_wgrad_reduce(const float* __restrict__ partial, int nblocks,
                                                           float* __restrict__ gw, float* __restrict__ gb)
{
    constexpr int K = kdim(CIN), NP = npad16(K + 1), MT = (COUT + 15) / 16;
    const int i = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= COUT * (K + 1)) return;  // whole waves leave together
    const int co = i / (K + 1), k = i % (K + 1);
    float s = 0.f;
    for (int g = lane; g < nblocks; g += 64) s += partial[((size_t)g * 16 * MT + co) * NP + k];
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) s += __shfl_xor(s, d, 64);
    if (lane != 0) return;
    if (k < K) gw[(size_t)co * K + k] = s;
    else gb[co] = s;
}

// FP32 master parameters -> packed BF16 weights of every layer (forward and
// flipped input-gradient layouts).
struct Packed {
    __bf16* fwd[kLayers];
    __bf16* bwd[kLayers];  // [0] unused
};

// Layer weights Wl [cout][9 cin] -> fwd [rows][kpad32(9 cin)] and, when bwd is
// not null, the input-gradient form bwd[ci][k'] = W[co][8 - tap][ci] with
// k' = tap cout + co (the taps flipped, channels swapped).
__global__ void k_pack(const float* __restrict__ Wl, int cin, int cout, __bf16* __restrict__ fwd,
                       __bf16* __restrict__ bwd)
{
    const int K = 9 * cin;
    const int kp = kpad32(K), rows = (cout + 15) / 16 * 16;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < rows * kp; i += gridDim.x * blockDim.x) {
        const int row = i / kp, k = i % kp;
        fwd[i] = bf(row < cout && k < K ? Wl[(size_t)row * K + k] : 0.f);
    }
    if (!bwd) return;
    const int kb = 9 * cout, kbp = kpad32(kb);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < cin * kbp; i += gridDim.x * blockDim.x) {
        const int ci = i / kbp, k = i % kbp;
        float v = 0.f;
        if (k < kb) {
            const int tap = k / cout, co = k % cout;
            v = Wl[(size_t)co * K + (8 - tap) * cin + ci];
        }
        bwd[i] = bf(v);
    }
}

// d(loss)/d(out) = 2 (out - target) / count and the FP64 sum of squares.
__global__ void k_loss(const float* __restrict__ out, const float* __restrict__ target, size_t count,
                       float* __restrict__ dout, double* __restrict__ partial)
{
    __shared__ double red[kThreads];
    double s = 0.0;
    const float scale = (float)(2.0 / (double)count);
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
        const float d = out[i] - target[i];
        dout[i] = scale * d;
        s += (double)d * (double)d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_loss_final(const double* __restrict__ partial, int n, size_t count, double* __restrict__ loss)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += partial[i];
    *loss = s / (double)count;
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// z0 = c x0 + D_rows^T clip(p1, -a_x, a_x) with (D^T p)_x = p_{x-1} - p_x.
__global__ void k_warm_state(const float* __restrict__ out, const float* __restrict__ ax, float c, int H, int W,
                             float* __restrict__ z0)
{
    const size_t n = (size_t)H * W;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % W);
        const float* p = out + n;
        const float a0 = ax[i];
        float y = -fminf(fmaxf(p[i], -a0), a0);
        if (x > 0) {
            const float a1 = ax[i - 1];
            y += fminf(fmaxf(p[i - 1], -a1), a1);
        }
        z0[i] = c * out[i] + y;
    }
}

// ---- workspace ------------------------------------------------------------------

struct NetWs {
    Packed pk;
    __bf16* act[3];     // h_1, h_2, h_3
    __bf16* dact[2];    // gradients w.r.t. the pre-activations of layers 3..1 (ping-pong)
    float* out;         // [b][2][H][W]
    float* dout;
    float* partial;     // weight-gradient partials
    double* lpart;      // loss partials (kLossBlocks) + result
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int ensure_net_ws(mc_ctx* c, int batch, int H, int W, bool train, NetWs* ws)
{
    const size_t pix = (size_t)batch * H * W;
    size_t off = 0;
    size_t o_fwd[kLayers], o_bwd[kLayers];
    for (int l = 0; l < kLayers; ++l) { o_fwd[l] = off; off = align256(off + 2 * fwd_elems(l)); }
    for (int l = 1; l < kLayers; ++l) { o_bwd[l] = off; off = align256(off + 2 * bwd_elems(l)); }
    size_t o_act[3];
    for (int i = 0; i < 3; ++i) { o_act[i] = off; off = align256(off + 2 * pix * kC); }
    const size_t o_out = off; off = align256(off + 4 * pix * 2);
    size_t o_dact[2] = {0, 0}, o_dout = 0, o_part = 0, o_lp = 0;
    if (train) {
        for (int i = 0; i < 2; ++i) { o_dact[i] = off; off = align256(off + 2 * pix * kC); }
        o_dout = off; off = align256(off + 4 * pix * 2);
        o_part = off; off = align256(off + 4 * (size_t)kWgradBlocks * 32 * npad16(9 * kC + 1));
        o_lp = off; off = align256(off + 8 * (kLossBlocks + 1));
    }
    if (off > c->ncap) {
        (void)hipFree(c->nbuf);
        c->nbuf = nullptr;
        c->ncap = 0;
        if (hipMalloc(&c->nbuf, off) != hipSuccess)
            return mc::set_error(MC_ERR_NOMEM, "network workspace allocation failed");
        c->ncap = off;
    }
    char* base = c->nbuf;
    for (int l = 0; l < kLayers; ++l) ws->pk.fwd[l] = reinterpret_cast<__bf16*>(base + o_fwd[l]);
    ws->pk.bwd[0] = nullptr;
    for (int l = 1; l < kLayers; ++l) ws->pk.bwd[l] = reinterpret_cast<__bf16*>(base + o_bwd[l]);
    for (int i = 0; i < 3; ++i) ws->act[i] = reinterpret_cast<__bf16*>(base + o_act[i]);
    ws->out = reinterpret_cast<float*>(base + o_out);
    for (int i = 0; i < 2; ++i) ws->dact[i] = train ? reinterpret_cast<__bf16*>(base + o_dact[i]) : nullptr;
    ws->dout = train ? reinterpret_cast<float*>(base + o_dout) : nullptr;
    ws->partial = train ? reinterpret_cast<float*>(base + o_part) : nullptr;
    ws->lpart = train ? reinterpret_cast<double*>(base + o_lp) : nullptr;
    return MC_OK;
}

int check_net_args(mc_ctx* c, const float* params, int batch, int H, int W, const float* w, const float* ax,
                   const float* ay)
{
    if (!c) return mc::set_error(MC_ERR_INVALID_ARG, "ctx is null");
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return mc::hip_error(e, "hipSetDevice");
    if (!params || !w || !ax || !ay) return mc::set_error(MC_ERR_INVALID_ARG, "null array");
    if (batch < 1 || H < 1 || W < 1) return mc::set_error(MC_ERR_INVALID_ARG, "batch, H and W must be positive");
    if (batch > 65535) return mc::set_error(MC_ERR_INVALID_ARG, "batch above 65535");
    if ((double)batch * H * W * kC > 4.0e9)
        return mc::set_error(MC_ERR_INVALID_ARG, "batch * H * W too large for the network workspace");
    return MC_OK;
}

hipError_t launch_forward(const NetWs& ws, const float* params, int batch, int H, int W, const float* w,
                          const float* ax, const float* ay, float* out, hipStream_t s)
{
    for (int l = 0; l < kLayers; ++l)
        hipLaunchKernelGGL(k_pack, dim3(16), dim3(256), 0, s, params + param_w_off(l), kCin[l], kCout[l],
                           ws.pk.fwd[l], ws.pk.bwd[l]);
    const dim3 grid((W + kT - 1) / kT, (H + kT - 1) / kT, batch), blk(kThreads);
    SrcFeat f{w, ax, ay, H, W};
    hipLaunchKernelGGL((k_conv<3, 2, SrcFeat, EpiReluAct>), grid, blk, 0, s, f, ws.pk.fwd[0],
                       EpiReluAct{params + param_b_off(0), ws.act[0], H, W}, H, W);
    for (int l = 1; l < 3; ++l)
        hipLaunchKernelGGL((k_conv<kC, 2, SrcAct, EpiReluAct>), grid, blk, 0, s, SrcAct{ws.act[l - 1], H, W},
                           ws.pk.fwd[l], EpiReluAct{params + param_b_off(l), ws.act[l], H, W}, H, W);
    hipLaunchKernelGGL((k_conv<kC, 1, SrcAct, EpiOutput>), grid, blk, 0, s, SrcAct{ws.act[2], H, W}, ws.pk.fwd[3],
                       EpiOutput{params + param_b_off(3), out, H, W}, H, W);
    return hipGetLastError();
}

template <int CIN, int COUT, class SrcIn, class SrcG>
void launch_wgrad(const NetWs& ws, const SrcIn& in, const SrcG& g, int l, int batch, int H, int W, float* grad,
                  hipStream_t s)
{
    const int tx = (W + kT - 1) / kT, ty = (H + kT - 1) / kT;
    const int total = tx * ty * batch;
    const int nb = total < kWgradBlocks ? total : kWgradBlocks;
    hipLaunchKernelGGL((k_wgrad<CIN, COUT, SrcIn, SrcG>), dim3(nb), dim3(kThreads), 0, s, in, g, ws.partial, H, W,
                       tx, ty, batch);
    const int nred = COUT * (kdim(CIN) + 1);
    constexpr int per_block = kThreads / 64;
    hipLaunchKernelGGL((k_wgrad_reduce<CIN, COUT>), dim3((nred + per_block - 1) / per_block), dim3(kThreads), 0, s,
                       ws.partial, nb, grad + param_w_off(l), grad + param_b_off(l));
}

hipError_t launch_backward(const NetWs& ws, const float* params, int batch, int H, int W, const float* w,
                           const float* ax, const float* ay, const float* target, float* grad, hipStream_t s)
{
    hipError_t e = launch_forward(ws, params, batch, H, W, w, ax, ay, ws.out, s);
    if (e != hipSuccess) return e;
    const size_t count = (size_t)batch * 2 * H * W;
    hipLaunchKernelGGL(k_loss, dim3(kLossBlocks), dim3(kThreads), 0, s, ws.out, target, count, ws.dout, ws.lpart);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, s, ws.lpart, kLossBlocks, count, ws.lpart + kLossBlocks);
    const dim3 grid((W + kT - 1) / kT, (H + kT - 1) / kT, batch), blk(kThreads);
    // layer 4: weights from (h_3, d out); d h_3 masked by h_3 > 0
    launch_wgrad<kC, 2>(ws, SrcAct{ws.act[2], H, W}, SrcPlanes2{ws.dout, H, W}, 3, batch, H, W, grad, s);
    hipLaunchKernelGGL((k_conv<2, 2, SrcPlanes2, EpiGradMask>), grid, blk, 0, s, SrcPlanes2{ws.dout, H, W},
                       ws.pk.bwd[3], EpiGradMask{ws.act[2], ws.dact[0], H, W}, H, W);
    // layer 3
    launch_wgrad<kC, kC>(ws, SrcAct{ws.act[1], H, W}, SrcAct{ws.dact[0], H, W}, 2, batch, H, W, grad, s);
    hipLaunchKernelGGL((k_conv<kC, 2, SrcAct, EpiGradMask>), grid, blk, 0, s, SrcAct{ws.dact[0], H, W},
                       ws.pk.bwd[2], EpiGradMask{ws.act[1], ws.dact[1], H, W}, H, W);
    // layer 2
    launch_wgrad<kC, kC>(ws, SrcAct{ws.act[0], H, W}, SrcAct{ws.dact[1], H, W}, 1, batch, H, W, grad, s);
    hipLaunchKernelGGL((k_conv<kC, 2, SrcAct, EpiGradMask>), grid, blk, 0, s, SrcAct{ws.dact[1], H, W},
                       ws.pk.bwd[1], EpiGradMask{ws.act[0], ws.dact[0], H, W}, H, W);
    // layer 1: weights from (features, d h_1 pre-activation)
    launch_wgrad<3, kC>(ws, SrcFeat{w, ax, ay, H, W}, SrcAct{ws.dact[0], H, W}, 0, batch, H, W, grad, s);
    return hipGetLastError();
}

}  // namespace

extern "C" {

int mc_ws_param_count(void) { return kParams; }

int mc_ws_forward(mc_ctx* c, const float* params, int batch, int H, int W, const float* w, const float* a_x,
                  const float* a_y, float* out, void* stream)
{
    int rc = check_net_args(c, params, batch, H, W, w, a_x, a_y);
    if (rc) return rc;
    if (!out) return mc::set_error(MC_ERR_INVALID_ARG, "out is null");
    NetWs ws;
    if ((rc = ensure_net_ws(c, batch, H, W, false, &ws))) return rc;
    MC_HIP(launch_forward(ws, params, batch, H, W, w, a_x, a_y, out, (hipStream_t)stream));
    return MC_OK;
}

int mc_ws_backward(mc_ctx* c, const float* params, int batch, int H, int W, const float* w, const float* a_x,
                   const float* a_y, const float* target, float* grad, double* loss, void* stream)
{
    int rc = check_net_args(c, params, batch, H, W, w, a_x, a_y);
    if (rc) return rc;
    if (!target || !grad) return mc::set_error(MC_ERR_INVALID_ARG, "null target or gradient");
    NetWs ws;
    if ((rc = ensure_net_ws(c, batch, H, W, true, &ws))) return rc;
    hipStream_t s = (hipStream_t)stream;
    MC_HIP(launch_backward(ws, params, batch, H, W, w, a_x, a_y, target, grad, s));
    if (loss) {
        MC_HIP(hipMemcpyAsync(c->hout, ws.lpart + kLossBlocks, sizeof(double), hipMemcpyDeviceToHost, s));
        MC_HIP(hipStreamSynchronize(s));
        *loss = c->hout[0];
    }
    return MC_OK;
}

int mc_ws_adam_step(mc_ctx* c, float* params, const float* grad, float* m, float* v, int step, float lr,
                    float beta1, float beta2, float eps, void* stream)
{
    if (!c) return mc::set_error(MC_ERR_INVALID_ARG, "ctx is null");
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return mc::hip_error(e, "hipSetDevice");
    if (!params || !grad || !m || !v) return mc::set_error(MC_ERR_INVALID_ARG, "null array");
    if (step < 1) return mc::set_error(MC_ERR_INVALID_ARG, "step counts from 1");
    if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f && lr >= 0.f))
        return mc::set_error(MC_ERR_INVALID_ARG, "Adam hyper-parameters out of range");
    const float c1 = (float)(1.0 / (1.0 - pow((double)beta1, step)));
    const float c2 = (float)(1.0 / (1.0 - pow((double)beta2, step)));
    hipLaunchKernelGGL(k_adam, dim3((kParams + 255) / 256), dim3(256), 0, (hipStream_t)stream, params, grad, m, v,
                       kParams, lr, beta1, beta2, eps, c1, c2);
    MC_HIP(hipGetLastError());
    return MC_OK;
}

int mc_ws_warm_state(mc_ctx* c, const mc_grid* grid, const float* out, const float* a_x, float coef, float* z0,
                     void* stream)
{
    if (!c) return mc::set_error(MC_ERR_INVALID_ARG, "ctx is null");
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return mc::hip_error(e, "hipSetDevice");
    if (!grid || grid->ndim != 2) return mc::set_error(MC_ERR_INVALID_ARG, "warm state needs a 2D grid");
    if (grid->dims[0] < 1 || grid->dims[1] < 1 || (double)grid->dims[0] * grid->dims[1] > (double)mc::kMaxNodes)
        return mc::set_error(MC_ERR_INVALID_ARG, "bad grid dims");
    if (!out || !a_x || !z0) return mc::set_error(MC_ERR_INVALID_ARG, "null array");
    const int H = (int)grid->dims[0], W = (int)grid->dims[1];
    const size_t n = (size_t)H * W;
    const int blocks = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
    hipLaunchKernelGGL(k_warm_state, dim3(blocks), dim3(256), 0, (hipStream_t)stream, out, a_x, coef, H, W, z0);
    MC_HIP(hipGetLastError());
    return MC_OK;
}

}  // extern "C"
