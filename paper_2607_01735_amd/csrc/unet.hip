// Learned initial guess: a small U-Net, trained and run by hand-written
// kernels (BF16 activations and weights, FP32 accumulation on MFMA, FP32
// master weights and Adam).
//
// Network: input x0 = f / rms(f) on the N x N interior; four levels on
// grids N_l = (N_{l-1} + 1)/F - 1 (coarsening factor F = 2 or 4) with
// 16/32/64/128 channels; each encoder level is conv3x3+ReLU twice, levels
// are linked by the averaging restriction R; each decoder level
// concatenates the bilinear prolongation P = F^2 R^T of the level below with
// the encoder's output of its own level and applies conv3x3+ReLU twice; a
// 1x1 head gives y, and u0 = y * rms(f).  With F = 4 the coarsest level's
// 3x3 convolutions span the whole grid (N = 511: levels 511, 127, 31, 7).
// The restriction/prolongation pair is the multigrid transfer pair, fixed
// (no weights).  Loss: mean squared error against u*/rms(f).
//
// Tensors are NHWC (batch, row, column, channel) in bfloat16; a tensor view
// has a pixel stride (channels per pixel of its buffer), so an encoder
// output is written straight into the channel slice of the decoder's
// concatenation buffer.  Convolutions are implicit GEMMs on the 16x16x16
// BF16 MFMA: pixels x output channels, K = 9 taps x input channels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "rbgs.h"
#include "rbgs_internal.h"

namespace rbgs {
namespace nn {

typedef uint16_t bf16;
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(bf16 v) { return __uint_as_float(uint32_t(v) << 16); }

__device__ __forceinline__ bf16 f2bf(float x) {
    // round to nearest, ties to even (NaN kept quiet)
    uint32_t b = __float_as_uint(x);
    if ((b & 0x7f800000u) == 0x7f800000u && (b & 0x007fffffu) != 0u) return bf16((b | 0x00400000u) >> 16);
    b += 0x7fffu + ((b >> 16) & 1u);
    return bf16(b >> 16);
}

// ---------------------------------------------------------------------------
// 3x3 convolution, stride 1, zero padding 1, as an implicit GEMM.
// One wave computes kConvGroups x 16 consecutive pixels of one row for all
// output channels (NT tiles of 16), as D[co][pixel] = sum_k W[co][k]
// X[k][pixel], K = 9 taps x input channels.  MFMA 16x16x16 lane layout
// (checked on the device):
//   A[m][k]: lane l holds m = l%16, k = 4(l/16)+j;  B[k][n]: n = l%16,
//   k = 4(l/16)+j;  D[m][n]: lane l holds m = 4(l/16)+i, n = l%16.
// So a lane loads four consecutive input channels of one pixel (B) and of
// one output channel's weights (A), 8 bytes each, and stores four
// consecutive output channels of one pixel, 8 bytes.  Each weight operand
// is loaded once per wave and used for every pixel group.
// X may be masked: an input element counts as 0 where mask <= 0 (this is
// how the backward pass applies the ReLU derivative of the layer output).
// ---------------------------------------------------------------------------
struct ConvArgs {
    const bf16* x;
    int64_t xs;        // pixel stride of x (channels of its buffer)
    const bf16* mask;  // optional, same geometry as x, stride ms
    int64_t ms;
    const bf16* w;     // [cout][9][cin]
    const float* bias; // optional
    bf16* y;
    int64_t ys;
    int batch, h, wd, cin, cout, relu;
};

constexpr int kConvGroups = 2;  // 16-pixel groups per wave

__device__ __forceinline__ bf16x4 load4(const bf16* p) {
    // four consecutive channels: 8 bytes, 8-byte aligned (channel strides
    // and offsets are multiples of 4)
    return *reinterpret_cast<const bf16x4*>(p);
}

template <int NT, bool MASK>
__global__ __launch_bounds__(256) void k_conv3x3(ConvArgs a) {
    constexpr int PG = kConvGroups;
    const int lane = threadIdx.x & 63;
    const int wave = int(blockIdx.x) * 4 + int(threadIdx.x >> 6);
    const int segs = (a.wd + 16 * PG - 1) / (16 * PG);
    if (wave >= a.batch * a.h * segs) return;
    const int seg = wave % segs;
    const int rowb = wave / segs;  // sample * h + row
    const int row = rowb % a.h;
    const int b = rowb / a.h;
    const int x0 = seg * 16 * PG;
    f32x4 acc[PG][NT];
#pragma unroll
    for (int g = 0; g < PG; ++g)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[g][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int n = lane & 15, kq = (lane >> 4) * 4;
    // Per 16-channel chunk and kernel row: the three taps' input operands
    // are loaded first (pixels outside the grid read a pixel inside and are
    // zeroed after the load, so no load sits behind a branch and they are in
    // flight together), then each output tile's three weight operands and
    // MFMAs.
    for (int c0 = 0; c0 < a.cin; c0 += 16) {
#pragma unroll 1
        for (int d = 0; d < 3; ++d) {
            const int yy = row + d - 1;
            const bool rowok = yy >= 0 && yy < a.h;
            const int64_t rbase = int64_t(b * a.h + (rowok ? yy : row)) * a.wd;
            bf16x4 xv[3][PG];
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
#pragma unroll
                for (int g = 0; g < PG; ++g) {
                    const int xx = x0 + g * 16 + n + dx - 1;
                    const bool ok = rowok && xx >= 0 && xx < a.wd;
                    const int64_t pix = rbase + (ok ? xx : 0);
                    bf16x4 v = load4(a.x + pix * a.xs + c0 + kq);
                    if (MASK) {
                        const bf16x4 mv = load4(a.mask + pix * a.ms + c0 + kq);
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            if (!(bf2f(bf16(mv[j])) > 0.f)) v[j] = 0;
                    }
#pragma unroll
                    for (int j = 0; j < 4; ++j) xv[dx][g][j] = ok ? v[j] : short(0);
                }
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const bf16* pw = a.w + (int64_t(t * 16 + n) * 9 + d * 3) * a.cin + c0 + kq;
                bf16x4 wv[3];
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) wv[dx] = load4(pw + dx * a.cin);
#pragma unroll
                for (int dx = 0; dx < 3; ++dx)
#pragma unroll
                    for (int g = 0; g < PG; ++g)
                        acc[g][t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wv[dx], xv[dx][g], acc[g][t], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int g = 0; g < PG; ++g) {
        const int xx = x0 + g * 16 + n;
        if (xx >= a.wd) continue;
        bf16* py = a.y + (int64_t(b * a.h + row) * a.wd + xx) * a.ys + kq;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            bf16x4 out;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float v = acc[g][t][i] + (a.bias ? a.bias[t * 16 + kq + i] : 0.f);
                if (a.relu) v = v > 0.f ? v : 0.f;
                out[i] = short(f2bf(v));
            }
            *reinterpret_cast<bf16x4*>(py + t * 16) = out;
        }
    }
}

// Weight gradient dW[co][ci][tap] = sum_p dZ[p][co] * X[p + off(tap)][ci],
// dZ = dY masked by (Y > 0).  MFMA with M = 16 output channels, N = 16
// input channels, K = 16 pixels of a row.  A workgroup of four waves takes
// four consecutive rows of one sample (one row per wave) for one (ci tile,
// co tile) pair and all nine taps: per 16-pixel chunk a wave loads its dZ
// operand once and, for each of the three X rows, the six pixels its lane
// group spans once, and issues the nine taps' MFMAs from them.  The four
// waves' sums meet in LDS and are added in a fixed order ((w0 + w1) + (w2 +
// w3)) into the workgroup's slot (part[sample * row quads + quad][co][ci]
// [tap]); k_reduce_parts adds the slots in a fixed order, so the gradient
// has the same bits on every run.
struct WGradArgs {
    const bf16* x;
    int64_t xs;
    const bf16* dy;
    int64_t dys;
    const bf16* y;  // layer output (mask), stride ys
    int64_t ys;
    float* part;    // [batch * row quads][cout][cin_w][9] partial sums
    int batch, h, wd, cin, cout;
    int cin_w;      // input channels of the weight tensor (cin is padded to 16)
};

constexpr int kWgradRows = 4;  // rows per workgroup (one per wave)

__global__ __launch_bounds__(256) void k_conv3x3_wgrad(WGradArgs a) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int cit = a.cin / 16, cot = a.cout / 16;
    const int quads = (a.h + kWgradRows - 1) / kWgradRows;
    int64_t r = blockIdx.x;  // the grid is exactly batch x quads x cit x cot
    const int co_t = int(r % cot);
    r /= cot;
    const int ci_t = int(r % cit);
    r /= cit;
    const int qd = int(r % quads);
    const int b = int(r / quads);
    const int row = qd * kWgradRows + wv;
    const int l16 = lane & 15, kq = (lane >> 4) * 4;
    f32x4 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (row < a.h) {
        const int64_t prow = (int64_t(b) * a.h + row) * a.wd;  // first pixel of the row
        const bf16* ym = a.y + prow * a.ys + co_t * 16 + l16;
        const bf16* dym = a.dy + prow * a.dys + co_t * 16 + l16;
        const bf16* xr[3];
        bool rok[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int yy = row + d - 1;
            rok[d] = yy >= 0 && yy < a.h;
            xr[d] = a.x + ((int64_t(b) * a.h + (rok[d] ? yy : row)) * a.wd) * a.xs + ci_t * 16 + l16;
        }
        for (int x0 = 0; x0 < a.wd; x0 += 16) {
            const int xb = x0 + kq;  // this lane group's first pixel
            bf16x4 av;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int xx = xb + j;
                bf16 g = 0;
                if (xx < a.wd && bf2f(ym[int64_t(xx) * a.ys]) > 0.f) g = dym[int64_t(xx) * a.dys];
                av[j] = short(g);
            }
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                // X at pixels xb - 1 .. xb + 4 of row `row + d - 1` (0 outside)
                bf16 xv[6];
#pragma unroll
                for (int m = 0; m < 6; ++m) {
                    const int xs2 = xb - 1 + m;
                    xv[m] = (rok[d] && xs2 >= 0 && xs2 < a.wd) ? xr[d][int64_t(xs2) * a.xs] : bf16(0);
                }
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    bf16x4 bv;
#pragma unroll
                    for (int j = 0; j < 4; ++j) bv[j] = xb + j < a.wd ? short(xv[j + dx]) : short(0);
                    acc[d * 3 + dx] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[d * 3 + dx], 0, 0, 0);
                }
            }
        }
    }
    // [wave][tap][co][ci] in LDS, then the fixed-order sum over the waves
    __shared__ float sh[kWgradRows][9][16][16];
    const int n = lane & 15, mq = (lane >> 4) * 4;
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) sh[wv][t][mq + i][n] = acc[t][i];
    __syncthreads();
    const int64_t slot = int64_t(b) * quads + qd;
    for (int e = threadIdx.x; e < 16 * 16 * 9; e += 256) {
        const int tap = e % 9, ci = (e / 9) % 16, co = e / 144;
        const float v = (sh[0][tap][co][ci] + sh[1][tap][co][ci]) + (sh[2][tap][co][ci] + sh[3][tap][co][ci]);
        const int ci_g = ci_t * 16 + ci, co_g = co_t * 16 + co;
        if (ci_g < a.cin_w) a.part[((slot * a.cout + co_g) * a.cin_w + ci_g) * 9 + tap] = v;
    }
}

// Bias gradient: per row (one block each) part[row][ch] = sum over the row
// of dY[p][ch] where Y[p][ch] > 0, in a fixed order: thread t takes channel
// t % c of the pixels x = t / c, t / c + g, ... (g = 256 / c pixel groups;
// c is a power of two up to 256), then a fixed tree over the groups;
// k_reduce_parts adds the rows in order.
__global__ __launch_bounds__(256) void k_bias_grad(const bf16* dy, int64_t dys, const bf16* y,
                                                   int64_t ys, float* part, int wd, int c) {
    const int64_t row = blockIdx.x;
    const int t = threadIdx.x;
    const int g = 256 / c;
    const int ch = t % c, x0 = t / c;
    float s = 0.f;
    for (int x = x0; x < wd; x += g) {
        const int64_t p = row * wd + x;
        if (bf2f(y[p * ys + ch]) > 0.f) s += bf2f(dy[p * dys + ch]);
    }
    __shared__ float sh[256];
    sh[t] = s;
    __syncthreads();
    for (int st = g / 2; st > 0; st >>= 1) {
        if (x0 < st) sh[t] += sh[t + st * c];
        __syncthreads();
    }
    if (x0 == 0) part[row * c + ch] = sh[t];
}

// out[e] = sum over slots k = 0 .. nparts-1 of part[k * count + e], in a
// fixed order: one block per element, thread t adds slots t, t + 256, ...
// in turn, then a fixed tree over the block (no atomics: the same bits on
// every run).
__global__ __launch_bounds__(256) void k_reduce_parts(const float* __restrict__ part,
                                                      int64_t nparts, int64_t count,
                                                      float* __restrict__ out) {
    const int64_t e = blockIdx.x;
    float s = 0.f;
    for (int64_t k = threadIdx.x; k < nparts; k += 256) s += part[k * count + e];
    __shared__ float sh[256];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (int(threadIdx.x) < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[e] = sh[0];
}

// The same sums for many slots, in two coalesced passes: pass 1 splits the
// slots into kReduceChunks contiguous chunks; a block takes 64 consecutive
// elements and one chunk, its four waves add slots g, g + 4, ... of the
// chunk (each wave reading 64 consecutive floats of a slot), and the four
// wave sums are added as (w0 + w1) + (w2 + w3) into stage[chunk][e];
// pass 2 adds the chunks in order.  A fixed order again.
constexpr int kReduceChunks = 16;

__global__ __launch_bounds__(256) void k_reduce_chunks(const float* __restrict__ part,
                                                       int64_t nparts, int64_t count,
                                                       float* __restrict__ stage) {
    const int l = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int64_t e = int64_t(blockIdx.x) * 64 + l;
    const int64_t per = (nparts + kReduceChunks - 1) / kReduceChunks;
    const int64_t k0 = int64_t(blockIdx.y) * per;
    const int64_t k1 = k0 + per < nparts ? k0 + per : nparts;
    float acc = 0.f;
    if (e < count)
        for (int64_t k = k0 + g; k < k1; k += 4) acc += part[k * count + e];
    __shared__ float sh[4][64];
    sh[g][l] = acc;
    __syncthreads();
    if (g == 0 && e < count)
        stage[int64_t(blockIdx.y) * count + e] = (sh[0][l] + sh[1][l]) + (sh[2][l] + sh[3][l]);
}

__global__ __launch_bounds__(256) void k_reduce_stage(const float* __restrict__ stage,
                                                      int64_t count, float* __restrict__ out) {
    const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (e >= count) return;
    float s = 0.f;
    for (int c = 0; c < kReduceChunks; ++c) s += stage[int64_t(c) * count + e];
    out[e] = s;
}

// Grid transfers between levels coarsened by a factor F (2 or 4): fine
// n_f = F n_c + F - 1, and coarse interior point (I, J) (0-based) sits on
// fine interior point (F I + F - 1, F J + F - 1).  Restriction averages the
// fine points within F - 1 of that point with the separable weights
// (F - |d|) / F^2 per axis (full weighting for F = 2: (1, 2, 1) / 4);
// prolongation is bilinear interpolation, P = F^2 R^T (1-D weights
// (F - |d|) / F).  Per channel, scaled by `scale`; accumulate != 0 adds into
// the output instead of overwriting.
// One thread per (pixel, group of 8 channels): 16-byte loads and stores,
// the index split and the weights formed once per 8 channels.  The host
// keeps batch x pixels x c / 8 (and the grid) below 2^32 (32-bit indexing)
// and c, the pixel strides and the base addresses in whole groups of 8.
struct bf16x8 {
    uint4 v;
    __device__ float get(int k) const {
        const uint32_t w = (&v.x)[k >> 1];
        return __uint_as_float((k & 1) ? (w & 0xffff0000u) : (w << 16));
    }
    __device__ void set(int k, bf16 h) {
        uint32_t& w = (&v.x)[k >> 1];
        w = (k & 1) ? ((w & 0x0000ffffu) | (uint32_t(h) << 16)) : ((w & 0xffff0000u) | h);
    }
};

__device__ __forceinline__ bf16x8 load8(const bf16* p) {
    return bf16x8{*reinterpret_cast<const uint4*>(p)};
}

// k_bias_grad with 16-byte loads (c a multiple of 8, 16-byte aligned rows):
// thread t takes channels 8 (t % c8) .. 8 (t % c8) + 7 of pixels t / c8,
// t / c8 + g, ... (c8 = c / 8, g = 256 / c8), then a fixed tree over the g
// pixel groups; one partial per (row, channel) as there.
__global__ __launch_bounds__(256) void k_bias_grad8(const bf16* dy, int64_t dys, const bf16* y,
                                                    int64_t ys, float* part, int wd, int c) {
    const int64_t row = blockIdx.x;
    const int t = threadIdx.x;
    const int c8 = c / 8;
    const int g = 256 / c8;
    const int grp = t / c8, ch = (t % c8) * 8;
    float s[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) s[k] = 0.f;
    for (int x = grp; x < wd; x += g) {
        const int64_t p = row * wd + x;
        const bf16x8 yv = load8(y + p * ys + ch);
        const bf16x8 dv = load8(dy + p * dys + ch);
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (yv.get(k) > 0.f) s[k] += dv.get(k);
    }
    __shared__ float sh[8][256];
#pragma unroll
    for (int k = 0; k < 8; ++k) sh[k][t] = s[k];
    __syncthreads();
    for (int st = g / 2; st > 0; st >>= 1) {
        if (grp < st) {
#pragma unroll
            for (int k = 0; k < 8; ++k) sh[k][t] += sh[k][t + st * c8];
        }
        __syncthreads();
    }
    if (grp == 0) {
#pragma unroll
        for (int k = 0; k < 8; ++k) part[row * c + ch + k] = sh[k][t];
    }
}

// F (the coarsening factor, 2 or 4) is a template parameter so that the
// window loops unroll and their loads are in flight together.
template <int F>
__global__ __launch_bounds__(256) void k_restrict(const bf16* in, int64_t is, bf16* out, int64_t os,
                                                  int batch, int nc, int c, float scale,
                                                  int accumulate) {
    const int c8 = c / 8;
    const uint32_t idx = blockIdx.x * 256u + threadIdx.x;
    const uint32_t total = uint32_t(batch) * uint32_t(nc) * uint32_t(nc) * uint32_t(c8);
    if (idx >= total) return;
    const int ch = int(idx % uint32_t(c8)) * 8;
    uint32_t r = idx / uint32_t(c8);
    const int J = int(r % uint32_t(nc));
    r /= uint32_t(nc);
    const int I = int(r % uint32_t(nc));
    const int b = int(r / uint32_t(nc));
    const int nf = F * nc + F - 1;
    const int ci = F * I + F - 1, cj = F * J + F - 1;
    float s[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) s[k] = 0.f;
#pragma unroll
    for (int di = 1 - F; di < F; ++di) {
        const float wi = float(F - (di < 0 ? -di : di));
        const bf16* row = in + ((int64_t(b) * nf + ci + di) * nf + cj) * is + ch;
        float t[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) t[k] = 0.f;
#pragma unroll
        for (int dj = 1 - F; dj < F; ++dj) {
            const float wj = float(F - (dj < 0 ? -dj : dj));
            const bf16x8 x = load8(row + dj * is);
#pragma unroll
            for (int k = 0; k < 8; ++k) t[k] += wj * x.get(k);
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) s[k] += wi * t[k];
    }
    bf16* o = out + ((int64_t(b) * nc + I) * nc + J) * os + ch;
    bf16x8 prev = accumulate ? load8(o) : bf16x8{make_uint4(0, 0, 0, 0)};
    bf16x8 res;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        float v = s[k] * (scale / float(F * F * F * F));
        if (accumulate) v += prev.get(k);
        res.set(k, f2bf(v));
    }
    *reinterpret_cast<uint4*>(o) = res.v;
}

template <int F>
__global__ __launch_bounds__(256) void k_prolong(const bf16* in, int64_t is, bf16* out, int64_t os,
                                                 int batch, int nc, int c, float scale,
                                                 int accumulate) {
    const int nf = F * nc + F - 1;
    const int c8 = c / 8;
    const uint32_t idx = blockIdx.x * 256u + threadIdx.x;
    const uint32_t total = uint32_t(batch) * uint32_t(nf) * uint32_t(nf) * uint32_t(c8);
    if (idx >= total) return;
    const int ch = int(idx % uint32_t(c8)) * 8;
    uint32_t r = idx / uint32_t(c8);
    const int j = int(r % uint32_t(nf));
    r /= uint32_t(nf);
    const int i = int(r % uint32_t(nf));
    const int b = int(r / uint32_t(nf));
    // the coarse points within F - 1 of fine i are I = (i + 1) / F - 1 and
    // the next one; weight (F - |d|) / F with d = i - (F I + F - 1)
    const float invF = 1.f / float(F);
    float s[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) s[k] = 0.f;
#pragma unroll
    for (int I = (i + 1) / F - 1; I <= (i + 1) / F; ++I) {
        const int di = i - (F * I + F - 1);
        if (I < 0 || I >= nc || di <= -F || di >= F) continue;
        const float wi = float(F - (di < 0 ? -di : di)) * invF;
#pragma unroll
        for (int J = (j + 1) / F - 1; J <= (j + 1) / F; ++J) {
            const int dj = j - (F * J + F - 1);
            if (J < 0 || J >= nc || dj <= -F || dj >= F) continue;
            const float wj = float(F - (dj < 0 ? -dj : dj)) * invF;
            const bf16x8 x = load8(in + ((int64_t(b) * nc + I) * nc + J) * is + ch);
#pragma unroll
            for (int k = 0; k < 8; ++k) s[k] += wi * wj * x.get(k);
        }
    }
    bf16* o = out + ((int64_t(b) * nf + i) * nf + j) * os + ch;
    bf16x8 prev = accumulate ? load8(o) : bf16x8{make_uint4(0, 0, 0, 0)};
    bf16x8 res;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        float v = s[k] * scale;
        if (accumulate) v += prev.get(k);
        res.set(k, f2bf(v));
    }
    *reinterpret_cast<uint4*>(o) = res.v;
}

// Sum of one double per thread over a block of 256, by a fixed tree; every
// thread gets the total.
__device__ __forceinline__ double block_sum_f64(double v) {
    __shared__ double sh[256];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (int(threadIdx.x) < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    const double total = sh[0];
    __syncthreads();
    return total;
}

// Per-sample rms of f over the interior, FP64 sums in a fixed order: one
// block per (sample, interior row) adds the row's squares (thread t takes
// columns t, t + 256, ..., then a tree), then one block per sample adds its
// rows' sums the same way.
__global__ __launch_bounds__(256) void k_rms_rows(const double* f, int n, int64_t ld,
                                                  int64_t gstride, double* part) {
    const int b = int(blockIdx.x) / n, row = int(blockIdx.x) % n;
    const double* fr = f + int64_t(b) * gstride + int64_t(row + 1) * ld + 1;
    double s = 0.0;
    for (int j = threadIdx.x; j < n; j += 256) {
        const double v = fr[j];
        s += v * v;
    }
    s = block_sum_f64(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_rms_final(const double* part, int n, float* rms) {
    const int b = blockIdx.x;
    double s = 0.0;
    for (int r = threadIdx.x; r < n; r += 256) s += part[int64_t(b) * n + r];
    s = block_sum_f64(s);
    if (threadIdx.x == 0) {
        const double r = sqrt(s / (double(n) * n));
        rms[b] = r > 0.0 ? float(r) : 1.f;
    }
}

// Network input: channel 0 = f / rms, channels 1..15 = 0 (the first conv's
// K is padded to one 16-wide MFMA chunk per tap).
__global__ __launch_bounds__(256) void k_input(const double* f, int n, int64_t ld, int64_t gstride,
                                               const float* rms, bf16* x, int batch) {
    const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
    const int64_t total = int64_t(batch) * n * n;
    if (idx >= total) return;
    const int b = int(idx / (int64_t(n) * n));
    const int64_t k = idx % (int64_t(n) * n);
    const int64_t i = k / n + 1, j = k % n + 1;
    const float v = float(f[int64_t(b) * gstride + i * ld + j] / double(rms[b]));
    bf16* px = x + idx * 16;
    px[0] = f2bf(v);
#pragma unroll
    for (int c = 1; c < 16; ++c) px[c] = 0;
}

// Head: y[p] = sum_c w[c] d[p][c] + b (FP32 out).  c = 16 channels at
// pixel stride ds (a multiple of 8, 16-byte aligned rows): two 16-byte
// loads per pixel.
__global__ __launch_bounds__(256) void k_head(const bf16* d, int64_t ds, const float* w,
                                              const float* bias, float* y, int64_t npix, int c) {
    const int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (p >= npix) return;
    const bf16x8 lo = load8(d + p * ds), hi = load8(d + p * ds + 8);
    float s = bias[0];
    for (int ch = 0; ch < c; ++ch) s += w[ch] * (ch < 8 ? lo.get(ch) : hi.get(ch - 8));
    y[p] = s;
}

// u0 = y * rms on the interior of the natural-layout output.
__global__ __launch_bounds__(256) void k_output(const float* y, const float* rms, double* u, int n,
                                                int64_t ld, int64_t gstride, int batch) {
    const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (idx >= int64_t(batch) * n * n) return;
    const int b = int(idx / (int64_t(n) * n));
    const int64_t k = idx % (int64_t(n) * n);
    const int64_t i = k / n + 1, j = k % n + 1;
    u[int64_t(b) * gstride + i * ld + j] = double(y[idx]) * double(rms[b]);
}

// MSE against u*/rms: dy = 2 (y - t) / count, loss accumulated in FP32.
__global__ __launch_bounds__(256) void k_mse(const float* y, const double* u, const float* rms,
                                             int n, int64_t ld, int64_t gstride, int batch,
                                             float* dy, float* loss_part) {
    const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
    const int64_t count = int64_t(batch) * n * n;
    float d = 0.f;
    if (idx < count) {
        const int b = int(idx / (int64_t(n) * n));
        const int64_t k = idx % (int64_t(n) * n);
        const int64_t i = k / n + 1, j = k % n + 1;
        const float t = float(u[int64_t(b) * gstride + i * ld + j] / double(rms[b]));
        d = y[idx] - t;
        dy[idx] = 2.f * d / float(count);
    }
    __shared__ float sh[256];
    sh[threadIdx.x] = d * d;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = sh[0] / float(count);
}

// Head backward: dd[p][c] = w[c] dy[p] (BF16); per block, the partial sums
// of dy d[c] (c < 16) and of dy go to part[block][0..16] (k_reduce_parts
// adds the blocks in order into dw[0..15], db = dw[16]).  Within a block:
// a fixed butterfly over each wave's 64 lanes, then the four waves in
// order.  d and dd: 16 channels at pixel strides that are multiples of 8,
// moved as two 16-byte accesses per pixel.
__global__ __launch_bounds__(256) void k_head_grad(const bf16* d, int64_t ds, const float* w,
                                                   const float* dy, bf16* dd, int64_t dds,
                                                   float* part, int64_t npix, int c) {
    const int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x;
    const bool ok = p < npix;
    const float g = ok ? dy[p] : 0.f;
    float v[17];
    if (ok) {
        const bf16x8 lo = load8(d + p * ds), hi = load8(d + p * ds + 8);
        bf16x8 olo{make_uint4(0, 0, 0, 0)}, ohi{make_uint4(0, 0, 0, 0)};
#pragma unroll
        for (int ch = 0; ch < 16; ++ch) {
            const float dv = ch < 8 ? lo.get(ch) : hi.get(ch - 8);
            const bf16 o = ch < c ? f2bf(w[ch] * g) : bf16(0);
            if (ch < 8) olo.set(ch, o); else ohi.set(ch - 8, o);
            v[ch] = ch < c ? g * dv : 0.f;
        }
        *reinterpret_cast<uint4*>(dd + p * dds) = olo.v;
        *reinterpret_cast<uint4*>(dd + p * dds + 8) = ohi.v;
    } else {
#pragma unroll
        for (int ch = 0; ch < 16; ++ch) v[ch] = 0.f;
    }
    v[16] = g;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int k = 0; k < 17; ++k) v[k] += __shfl_xor(v[k], off, 64);
    __shared__ float sw[4][17];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < 17; ++k) sw[wv][k] = v[k];
    __syncthreads();
    if (threadIdx.x < 17)
        part[int64_t(blockIdx.x) * 17 + threadIdx.x] =
            ((sw[0][threadIdx.x] + sw[1][threadIdx.x]) + sw[2][threadIdx.x]) + sw[3][threadIdx.x];
}

// Master FP32 weights [co][ci][9] -> forward BF16 [co][9][cin_p] (zero-padded
// input channels) and backward-data BF16 [ci][9][co] with the taps flipped.
__global__ __launch_bounds__(256) void k_prep_weights(const float* w, int cout, int cin, int cin_p,
                                                      bf16* wf, bf16* wb) {
    const int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x;
    const int64_t total = int64_t(cout) * cin_p * 9;
    if (idx >= total) return;
    const int ci = int(idx % cin_p);
    const int tap = int((idx / cin_p) % 9);
    const int co = int(idx / (int64_t(cin_p) * 9));
    const float v = ci < cin ? w[(int64_t(co) * cin + ci) * 9 + tap] : 0.f;
    wf[(int64_t(co) * 9 + tap) * cin_p + ci] = f2bf(v);
    if (wb && ci < cin) wb[(int64_t(ci) * 9 + (8 - tap)) * cout + co] = f2bf(v);
}

// Adam: b1, b2 and their complements 1 - b1, 1 - b2 and the bias corrections
// c1 = 1 - b1^t, c2 = 1 - b2^t are formed in FP64 on the host and rounded
// once (1 - b2^t in binary32 loses four digits to cancellation at small t).
__global__ __launch_bounds__(256) void k_adam(float* p, const float* g, float* m, float* v,
                                              int64_t count, float lr, float b1, float omb1,
                                              float b2, float omb2, float eps, float c1, float c2) {
    const int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (k >= count) return;
    const float gk = g[k];
    const float mk = b1 * m[k] + omb1 * gk;
    const float vk = b2 * v[k] + omb2 * gk * gk;
    m[k] = mk;
    v[k] = vk;
    p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

__global__ __launch_bounds__(256) void k_fill(uint32_t* p, int64_t words) {
    const int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (k < words) p[k] = 0u;
}

}  // namespace nn
}  // namespace rbgs

// ===========================================================================
// Host side: the network object and the C ABI.
// ===========================================================================
namespace rbgs {
namespace nn {
namespace {

constexpr int kLevels = 4;
constexpr int kC[kLevels] = {16, 32, 64, 128};

struct Layer {
    const char* name;
    int cin, cin_p, cout, level;
    size_t w_off, b_off;  // float offsets in the master parameter vector
    bf16* wf = nullptr;   // [cout][9][cin_p]
    bf16* wb = nullptr;   // [cin][9][cout] (flipped taps) for the input gradient
};

// Parameter order and shapes: each conv's weight (cout, cin, 3, 3) then its
// bias (cout), in the order enc0.0 ... enc3.1, dec2.0 ... dec0.1, head.
std::vector<Layer> make_layers(size_t* count) {
    std::vector<Layer> L;
    auto add = [&](const char* name, int cin, int cout, int level) {
        Layer l;
        l.name = name;
        l.cin = cin;
        l.cin_p = cin < 16 ? 16 : cin;
        l.cout = cout;
        l.level = level;
        L.push_back(l);
    };
    add("enc0.0", 1, 16, 0);
    add("enc0.1", 16, 16, 0);
    add("enc1.0", 16, 32, 1);
    add("enc1.1", 32, 32, 1);
    add("enc2.0", 32, 64, 2);
    add("enc2.1", 64, 64, 2);
    add("enc3.0", 64, 128, 3);
    add("enc3.1", 128, 128, 3);
    add("dec2.0", 192, 64, 2);
    add("dec2.1", 64, 64, 2);
    add("dec1.0", 96, 32, 1);
    add("dec1.1", 32, 32, 1);
    add("dec0.0", 48, 16, 0);
    add("dec0.1", 16, 16, 0);
    size_t off = 0;
    for (auto& l : L) {
        l.w_off = off;
        off += size_t(l.cout) * l.cin * 9;
        l.b_off = off;
        off += l.cout;
    }
    *count = off + 16 + 1;  // head weight (1, 16, 1, 1) and bias
    return L;
}

}  // namespace

struct Net {
    int n[kLevels];
    int factor = 2;  // coarsening factor between levels (2 or 4)
    int batch;
    std::vector<Layer> layers;
    size_t nparam;
    float *param, *grad, *m, *v, *rms, *loss, *y, *dy;
    float* parts = nullptr;  // partial sums of the fixed-order gradient reductions
    size_t parts_floats = 0;
    float* stage = nullptr;  // per-chunk sums of the two-pass reduction
    size_t stage_floats = 0;
    double* guess;  // natural-layout scratch grid for the learned solve
    int adam_t = 0;
    // activations (level-indexed) and their gradients
    bf16 *in[kLevels], *aenc[kLevels], *cat[kLevels - 1], *e3, *adec[kLevels - 1], *d[kLevels - 1];
    bf16 *gd[kLevels - 1], *ge3, *gadec[kLevels - 1], *gcat[kLevels - 1], *gaenc[kLevels],
        *gin[kLevels];
    size_t total = 0;
};

namespace {

int cat_channels(int l) { return kC[l + 1] + kC[l]; }
int in_channels(int l) { return l == 0 ? 16 : kC[l - 1]; }

int wgrad_quads(int h) { return (h + kWgradRows - 1) / kWgradRows; }

// Floats of partial sums the largest fixed-order reduction needs: weight
// gradients (batch x row blocks slots of cout x cin x 9), bias gradients
// (batch x rows slots of cout), the head (blocks of 17), the loss and the
// rms row sums.
size_t parts_floats(const Net& net) {
    size_t most = 0;
    const size_t B = size_t(net.batch);
    for (const auto& l : net.layers) {
        const int h = net.n[l.level];
        const size_t rb = size_t(wgrad_quads(h));
        most = std::max(most, B * rb * size_t(l.cout) * size_t(l.cin) * 9);
        most = std::max(most, B * size_t(h) * size_t(l.cout));
    }
    const size_t px0 = B * size_t(net.n[0]) * size_t(net.n[0]);
    most = std::max(most, (px0 + 255) / 256 * 17);
    most = std::max(most, 2 * B * size_t(net.n[0]));  // the rms row sums (doubles)
    return most;
}

// Carves every buffer; with base == nullptr only computes the size.
size_t carve(Net& net, char* base) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    const int64_t B = net.batch;
    net.param = reinterpret_cast<float*>(take(net.nparam * 4));
    net.grad = reinterpret_cast<float*>(take(net.nparam * 4));
    net.m = reinterpret_cast<float*>(take(net.nparam * 4));
    net.v = reinterpret_cast<float*>(take(net.nparam * 4));
    for (auto& l : net.layers) {
        l.wf = reinterpret_cast<bf16*>(take(size_t(l.cout) * 9 * l.cin_p * 2));
        l.wb = reinterpret_cast<bf16*>(take(size_t(l.cin) * 9 * l.cout * 2));
    }
    net.rms = reinterpret_cast<float*>(take(B * 4));
    net.loss = reinterpret_cast<float*>(take(4));
    const int64_t px0 = int64_t(net.n[0]) * net.n[0];
    net.y = reinterpret_cast<float*>(take(B * px0 * 4));
    net.dy = reinterpret_cast<float*>(take(B * px0 * 4));
    net.parts_floats = parts_floats(net);
    net.parts = reinterpret_cast<float*>(take(net.parts_floats * 4));
    size_t most = 0;
    for (const auto& l : net.layers) most = std::max(most, size_t(l.cout) * size_t(l.cin) * 9);
    net.stage_floats = size_t(kReduceChunks) * most;
    net.stage = reinterpret_cast<float*>(take(net.stage_floats * 4));
    net.guess = reinterpret_cast<double*>(take(size_t(net.n[0] + 2) * (net.n[0] + 2) * 8));
    for (int l = 0; l < kLevels; ++l) {
        const int64_t px = B * net.n[l] * net.n[l];
        auto act = [&](int ch) { return reinterpret_cast<bf16*>(take(size_t(px) * ch * 2)); };
        net.in[l] = act(in_channels(l));
        net.aenc[l] = act(kC[l]);
        net.gaenc[l] = act(kC[l]);
        net.gin[l] = act(in_channels(l));
        if (l < kLevels - 1) {
            net.cat[l] = act(cat_channels(l));
            net.gcat[l] = act(cat_channels(l));
            net.adec[l] = act(kC[l]);
            net.gadec[l] = act(kC[l]);
            net.d[l] = act(kC[l]);
            net.gd[l] = act(kC[l]);
        } else {
            net.e3 = act(kC[l]);
            net.ge3 = act(kC[l]);
        }
    }
    return off;
}

unsigned blocks_for(int64_t items, int per_block = 256) {
    return unsigned((items + per_block - 1) / per_block);
}

template <bool MASK>
hipError_t launch_conv(const ConvArgs& a, dim3 grid, dim3 block, hipStream_t s) {
    switch (a.cout / 16) {
        case 1: hipLaunchKernelGGL((k_conv3x3<1, MASK>), grid, block, 0, s, a); break;
        case 2: hipLaunchKernelGGL((k_conv3x3<2, MASK>), grid, block, 0, s, a); break;
        case 3: hipLaunchKernelGGL((k_conv3x3<3, MASK>), grid, block, 0, s, a); break;
        case 4: hipLaunchKernelGGL((k_conv3x3<4, MASK>), grid, block, 0, s, a); break;
        case 6: hipLaunchKernelGGL((k_conv3x3<6, MASK>), grid, block, 0, s, a); break;
        case 8: hipLaunchKernelGGL((k_conv3x3<8, MASK>), grid, block, 0, s, a); break;
        case 12: hipLaunchKernelGGL((k_conv3x3<12, MASK>), grid, block, 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t conv(const Net& net, const Layer& L, const bf16* x, int64_t xs, const bf16* mask,
                int64_t ms, bool forward, bf16* y, int64_t ys, int batch, hipStream_t s) {
    ConvArgs a;
    a.x = x;
    a.xs = xs;
    a.mask = mask;
    a.ms = ms;
    a.batch = batch;
    a.h = a.wd = net.n[L.level];
    if (forward) {
        a.w = L.wf;
        a.bias = net.param + L.b_off;
        a.cin = L.cin_p;
        a.cout = L.cout;
        a.relu = 1;
    } else {  // input gradient: K runs over the layer's outputs
        a.w = L.wb;
        a.bias = nullptr;
        a.cin = L.cout;
        a.cout = L.cin;
        a.relu = 0;
    }
    a.y = y;
    a.ys = ys;
    const int64_t waves = int64_t(batch) * a.h * ((a.wd + 16 * kConvGroups - 1) / (16 * kConvGroups));
    if (waves > (int64_t(1) << 31) - 4 || int64_t(batch) * a.h * a.wd >= (int64_t(1) << 31))
        return hipErrorInvalidValue;
    // 8-byte operand loads and stores: channel strides, counts and base
    // addresses in whole groups of four channels
    if ((a.xs | a.ys | a.cin | (a.mask ? a.ms : 0)) % 4 != 0 || a.cout % 16 != 0 ||
        (reinterpret_cast<uintptr_t>(a.x) | reinterpret_cast<uintptr_t>(a.y) |
         reinterpret_cast<uintptr_t>(a.w) | reinterpret_cast<uintptr_t>(a.mask)) % 8 != 0)
        return hipErrorInvalidValue;
    const dim3 grid(blocks_for(waves, 4)), block(256);
    return a.mask ? launch_conv<true>(a, grid, block, s) : launch_conv<false>(a, grid, block, s);
}

// out[e] = sum over the nparts slots of net.parts[k * count + e] (two passes).
hipError_t reduce_slots(const Net& net, int64_t nparts, int64_t count, float* out, hipStream_t s) {
    if (size_t(count) * kReduceChunks > net.stage_floats) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_reduce_chunks, dim3(unsigned((count + 63) / 64), kReduceChunks), dim3(256), 0,
                       s, net.parts, nparts, count, net.stage);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_stage, dim3(blocks_for(count)), dim3(256), 0, s, net.stage, count, out);
    return hipGetLastError();
}

hipError_t wgrad(const Net& net, const Layer& L, const bf16* x, int64_t xs, const bf16* dy,
                 int64_t dys, const bf16* y, int64_t ys, int batch, hipStream_t s) {
    WGradArgs a;
    a.x = x;
    a.xs = xs;
    a.dy = dy;
    a.dys = dys;
    a.y = y;
    a.ys = ys;
    a.batch = batch;
    a.h = a.wd = net.n[L.level];
    a.cin = L.cin_p;
    a.cout = L.cout;
    a.cin_w = L.cin;  // the first layer's padded input channels feed no weight
    a.part = net.parts;
    const int rb = wgrad_quads(a.h);
    const int64_t blocks = int64_t(batch) * rb * (a.cin / 16) * (a.cout / 16);
    hipLaunchKernelGGL(k_conv3x3_wgrad, dim3(unsigned(blocks)), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t wcount = int64_t(L.cout) * L.cin * 9;
    if ((e = reduce_slots(net, int64_t(batch) * rb, wcount, net.grad + L.w_off, s)) != hipSuccess)
        return e;
    if (L.cout > 256 || (256 % L.cout) != 0) return hipErrorInvalidValue;
    const bool wide = L.cout % 8 == 0 && dys % 8 == 0 && ys % 8 == 0 &&
                      (reinterpret_cast<uintptr_t>(dy) | reinterpret_cast<uintptr_t>(y)) % 16 == 0;
    if (wide)
        hipLaunchKernelGGL(k_bias_grad8, dim3(unsigned(int64_t(batch) * a.h)), dim3(256), 0, s, dy,
                           dys, y, ys, net.parts, a.wd, L.cout);
    else
        hipLaunchKernelGGL(k_bias_grad, dim3(unsigned(int64_t(batch) * a.h)), dim3(256), 0, s, dy,
                           dys, y, ys, net.parts, a.wd, L.cout);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return reduce_slots(net, int64_t(batch) * a.h, int64_t(L.cout), net.grad + L.b_off, s);
}

}  // namespace
}  // namespace nn
}  // namespace rbgs

namespace rbgs {
namespace nn {
namespace {

#define NN_TRY(expr)                         \
    do {                                     \
        hipError_t _e = (expr);              \
        if (_e != hipSuccess) return _e;     \
    } while (0)

// The transfers move whole groups of 8 channels with 16-byte accesses.
bool transfer_ok(const bf16* in, int64_t is, const bf16* out, int64_t os, int c) {
    return c > 0 && c % 8 == 0 && is % 8 == 0 && os % 8 == 0 &&
           (reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) % 16 == 0;
}

hipError_t restrict_op(const Net& net, const bf16* in, int64_t is, bf16* out, int64_t os, int batch,
                       int nc, int c, float scale, int acc, hipStream_t s) {
    if (!transfer_ok(in, is, out, os, c) || int64_t(batch) * nc * nc * (c / 8) > (int64_t(1) << 32) - 256)
        return hipErrorInvalidValue;
    const dim3 grid(blocks_for(int64_t(batch) * nc * nc * (c / 8)));
    if (net.factor == 2)
        hipLaunchKernelGGL(k_restrict<2>, grid, dim3(256), 0, s, in, is, out, os, batch, nc, c,
                           scale, acc);
    else if (net.factor == 4)
        hipLaunchKernelGGL(k_restrict<4>, grid, dim3(256), 0, s, in, is, out, os, batch, nc, c,
                           scale, acc);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t prolong_op(const Net& net, const bf16* in, int64_t is, bf16* out, int64_t os, int batch,
                      int nc, int c, float scale, int acc, hipStream_t s) {
    const int nf = net.factor * nc + net.factor - 1;
    if (!transfer_ok(in, is, out, os, c) || int64_t(batch) * nf * nf * (c / 8) > (int64_t(1) << 32) - 256)
        return hipErrorInvalidValue;
    const dim3 grid(blocks_for(int64_t(batch) * nf * nf * (c / 8)));
    if (net.factor == 2)
        hipLaunchKernelGGL(k_prolong<2>, grid, dim3(256), 0, s, in, is, out, os, batch, nc, c, scale,
                           acc);
    else if (net.factor == 4)
        hipLaunchKernelGGL(k_prolong<4>, grid, dim3(256), 0, s, in, is, out, os, batch, nc, c, scale,
                           acc);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t prep_weights(Net& net, hipStream_t s) {
    for (auto& l : net.layers) {
        hipLaunchKernelGGL(k_prep_weights, dim3(blocks_for(int64_t(l.cout) * l.cin_p * 9)), dim3(256),
                           0, s, net.param + l.w_off, l.cout, l.cin, l.cin_p, l.wf, l.wb);
        NN_TRY(hipGetLastError());
    }
    return hipSuccess;
}

const Layer& layer(const Net& net, const char* name) {
    for (const auto& l : net.layers)
        if (std::strcmp(l.name, name) == 0) return l;
    return net.layers[0];
}

// Forward pass of `batch` samples; f: batch grids back to back (natural
// layout, gstride elements apart).  Leaves y (FP32, normalised) and rms.
hipError_t forward(Net& net, int batch, const double* f, int64_t ld, int64_t gstride,
                   hipStream_t s) {
    const int n0 = net.n[0];
    // the row sums sit in the gradient partials, which are free during a forward pass
    double* rows = reinterpret_cast<double*>(net.parts);
    hipLaunchKernelGGL(k_rms_rows, dim3(unsigned(batch * n0)), dim3(256), 0, s, f, n0, ld, gstride,
                       rows);
    NN_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_rms_final, dim3(batch), dim3(256), 0, s, rows, n0, net.rms);
    NN_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_input, dim3(blocks_for(int64_t(batch) * n0 * n0)), dim3(256), 0, s, f, n0,
                       ld, gstride, net.rms, net.in[0], batch);
    NN_TRY(hipGetLastError());
    // encoder
    for (int l = 0; l < kLevels; ++l) {
        char n0name[8] = "enc0.0", n1name[8] = "enc0.1";
        n0name[3] = n1name[3] = char('0' + l);
        const Layer& c0 = layer(net, n0name);
        const Layer& c1 = layer(net, n1name);
        NN_TRY(conv(net, c0, net.in[l], in_channels(l), nullptr, 0, true, net.aenc[l], kC[l], batch, s));
        bf16* e = l < kLevels - 1 ? net.cat[l] + kC[l + 1] : net.e3;
        const int64_t es = l < kLevels - 1 ? cat_channels(l) : kC[l];
        NN_TRY(conv(net, c1, net.aenc[l], kC[l], nullptr, 0, true, e, es, batch, s));
        if (l + 1 < kLevels)
            NN_TRY(restrict_op(net, e, es, net.in[l + 1], in_channels(l + 1), batch, net.n[l + 1],
                               kC[l], 1.f, 0, s));
    }
    // decoder
    for (int l = kLevels - 2; l >= 0; --l) {
        const bf16* below = l == kLevels - 2 ? net.e3 : net.d[l + 1];
        NN_TRY(prolong_op(net, below, kC[l + 1], net.cat[l], cat_channels(l), batch, net.n[l + 1],
                          kC[l + 1], 1.f, 0, s));
        char n0name[8] = "dec0.0", n1name[8] = "dec0.1";
        n0name[3] = n1name[3] = char('0' + l);
        NN_TRY(conv(net, layer(net, n0name), net.cat[l], cat_channels(l), nullptr, 0, true,
                    net.adec[l], kC[l], batch, s));
        NN_TRY(conv(net, layer(net, n1name), net.adec[l], kC[l], nullptr, 0, true, net.d[l], kC[l],
                    batch, s));
    }
    const size_t hw = net.nparam - 17;
    hipLaunchKernelGGL(k_head, dim3(blocks_for(int64_t(batch) * n0 * n0)), dim3(256), 0, s, net.d[0],
                       kC[0], net.param + hw, net.param + hw + 16, net.y, int64_t(batch) * n0 * n0,
                       kC[0]);
    return hipGetLastError();
}

// Backward pass from dy (FP32, normalised output gradient) into net.grad.
hipError_t backward(Net& net, int batch, hipStream_t s) {
    const int n0 = net.n[0];
    const size_t hw = net.nparam - 17;
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(int64_t(net.nparam))), dim3(256), 0, s,
                       reinterpret_cast<uint32_t*>(net.grad), int64_t(net.nparam));
    NN_TRY(hipGetLastError());
    const unsigned hblocks = blocks_for(int64_t(batch) * n0 * n0);
    hipLaunchKernelGGL(k_head_grad, dim3(hblocks), dim3(256), 0, s, net.d[0], kC[0],
                       net.param + hw, net.dy, net.gd[0], kC[0], net.parts,
                       int64_t(batch) * n0 * n0, kC[0]);
    NN_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_reduce_parts, dim3(17), dim3(256), 0, s, net.parts, int64_t(hblocks),
                       int64_t(17), net.grad + hw);
    NN_TRY(hipGetLastError());
    // decoder, from level 0 (computed last) up
    for (int l = 0; l < kLevels - 1; ++l) {
        char n0name[8] = "dec0.0", n1name[8] = "dec0.1";
        n0name[3] = n1name[3] = char('0' + l);
        const Layer& c0 = layer(net, n0name);
        const Layer& c1 = layer(net, n1name);
        const int C = kC[l], CC = cat_channels(l);
        NN_TRY(wgrad(net, c1, net.adec[l], C, net.gd[l], C, net.d[l], C, batch, s));
        NN_TRY(conv(net, c1, net.gd[l], C, net.d[l], C, false, net.gadec[l], C, batch, s));
        NN_TRY(wgrad(net, c0, net.cat[l], CC, net.gadec[l], C, net.adec[l], C, batch, s));
        NN_TRY(conv(net, c0, net.gadec[l], C, net.adec[l], C, false, net.gcat[l], CC, batch, s));
        // up = P(d_{l+1}) with P = F^2 R^T: the gradient reaching d_{l+1} is F^2 R(dup)
        bf16* gbelow = l == kLevels - 2 ? net.ge3 : net.gd[l + 1];
        NN_TRY(restrict_op(net, net.gcat[l], CC, gbelow, kC[l + 1], batch, net.n[l + 1], kC[l + 1],
                           float(net.factor * net.factor), 0, s));
    }
    // encoder, from the bottom level up
    for (int l = kLevels - 1; l >= 0; --l) {
        char n0name[8] = "enc0.0", n1name[8] = "enc0.1";
        n0name[3] = n1name[3] = char('0' + l);
        const Layer& c0 = layer(net, n0name);
        const Layer& c1 = layer(net, n1name);
        const int C = kC[l];
        const bf16* e = l < kLevels - 1 ? net.cat[l] + kC[l + 1] : net.e3;
        bf16* ge = l < kLevels - 1 ? net.gcat[l] + kC[l + 1] : net.ge3;
        const int64_t es = l < kLevels - 1 ? cat_channels(l) : C;
        NN_TRY(wgrad(net, c1, net.aenc[l], C, ge, es, e, es, batch, s));
        NN_TRY(conv(net, c1, ge, es, e, es, false, net.gaenc[l], C, batch, s));
        NN_TRY(wgrad(net, c0, net.in[l], in_channels(l), net.gaenc[l], C, net.aenc[l], C, batch, s));
        if (l > 0) {
            NN_TRY(conv(net, c0, net.gaenc[l], C, net.aenc[l], C, false, net.gin[l], in_channels(l),
                        batch, s));
            // in_l = R(e_{l-1}): add R^T(g_in) = P(g_in)/F^2 to e_{l-1}'s gradient
            // (which already holds its skip-connection part)
            bf16* gprev = net.gcat[l - 1] + kC[l];
            NN_TRY(prolong_op(net, net.gin[l], in_channels(l), gprev, cat_channels(l - 1), batch,
                              net.n[l], in_channels(l), 1.f / float(net.factor * net.factor), 1, s));
        }
    }
    return hipSuccess;
}

hipError_t adam(Net& net, float lr, hipStream_t s) {
    net.adam_t += 1;
    const double b1 = 0.9, b2 = 0.999, t = double(net.adam_t);
    const double c1 = -std::expm1(t * std::log(b1)), c2 = -std::expm1(t * std::log(b2));
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(int64_t(net.nparam))), dim3(256), 0, s, net.param,
                       net.grad, net.m, net.v, int64_t(net.nparam), lr, float(b1), float(1.0 - b1),
                       float(b2), float(1.0 - b2), 1e-8f, float(c1), float(c2));
    NN_TRY(hipGetLastError());
    return prep_weights(net, s);
}

thread_local std::string g_nn_error = "no error";

int nnfail(int status, const std::string& msg) {
    g_nn_error = msg;
    return status;
}

int nn_hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return RBGS_OK;
    return nnfail(RBGS_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Four levels n_l = (n_{l-1} + 1) / F - 1 with at least one point on the
// coarsest: F = 2 takes n = 2^k - 1 in [63, 8191] (coarsest >= 7 points),
// F = 4 takes n + 1 divisible by 64 in [127, 8191].
bool valid_size(int n, int factor) {
    if (n > 8191) return false;
    if (factor == 2) return n >= 63 && ((n + 1) & n) == 0;
    if (factor == 4) return n >= 127 && (n + 1) % 64 == 0;
    return false;
}

void set_levels(Net& net, int n, int factor) {
    net.factor = factor;
    net.n[0] = n;
    for (int l = 1; l < kLevels; ++l) net.n[l] = (net.n[l - 1] + 1) / factor - 1;
}

}  // namespace
}  // namespace nn
}  // namespace rbgs

using namespace rbgs;

struct rbgs_unet {
    nn::Net net;
};

extern "C" {

size_t rbgs_unet_param_count(void) {
    size_t c = 0;
    (void)nn::make_layers(&c);
    return c;
}

size_t rbgs_unet_workspace_size(int32_t n, int32_t batch, int32_t factor) {
    if (!nn::valid_size(n, factor) || batch < 1 || batch > 4096) return 0;
    nn::Net net;
    net.layers = nn::make_layers(&net.nparam);
    net.batch = batch;
    nn::set_levels(net, n, factor);
    return nn::carve(net, nullptr);
}

const char* rbgs_unet_last_error(void) { return nn::g_nn_error.c_str(); }

int rbgs_unet_create(rbgs_unet** out, int32_t n, int32_t batch, int32_t factor, void* workspace,
                     size_t workspace_bytes) {
    if (!out) return nn::nnfail(RBGS_EINVAL, "net is NULL");
    *out = nullptr;
    if (factor != 2 && factor != 4) return nn::nnfail(RBGS_EINVAL, "factor must be 2 or 4");
    if (!nn::valid_size(n, factor))
        return nn::nnfail(RBGS_EINVAL, factor == 2 ? "n must be 2^k - 1 in [63, 8191] for factor 2"
                                                   : "n + 1 must be a multiple of 64 in "
                                                     "[128, 8192] for factor 4");
    if (batch < 1 || batch > 4096) return nn::nnfail(RBGS_EINVAL, "batch must be in [1, 4096]");
    const size_t need = rbgs_unet_workspace_size(n, batch, factor);
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256 || workspace_bytes < need)
        return nn::nnfail(RBGS_EWORKSPACE, "workspace missing, misaligned or smaller than " +
                                               std::to_string(need) + " bytes");
    rbgs_unet* u = new rbgs_unet;
    u->net.layers = nn::make_layers(&u->net.nparam);
    u->net.batch = batch;
    nn::set_levels(u->net, n, factor);
    u->net.total = nn::carve(u->net, static_cast<char*>(workspace));
    *out = u;
    return RBGS_OK;
}

int rbgs_unet_destroy(rbgs_unet* u) {
    delete u;
    return RBGS_OK;
}

int rbgs_unet_set_params(rbgs_unet* u, const float* host, size_t count, void* stream) {
    if (!u || !host || count != u->net.nparam) return nn::nnfail(RBGS_EINVAL, "bad parameter vector");
    hipStream_t s = static_cast<hipStream_t>(stream);
    nn::Net& net = u->net;
    int rc = nn::nn_hip(hipMemcpyAsync(net.param, host, count * 4, hipMemcpyHostToDevice, s), "upload");
    if (rc) return rc;
    // a fresh parameter vector restarts Adam
    for (float* p : {net.m, net.v}) {
        hipLaunchKernelGGL(nn::k_fill, dim3(nn::blocks_for(int64_t(count))), dim3(256), 0, s,
                           reinterpret_cast<uint32_t*>(p), int64_t(count));
        if ((rc = nn::nn_hip(hipGetLastError(), "fill"))) return rc;
    }
    net.adam_t = 0;
    if ((rc = nn::nn_hip(nn::prep_weights(net, s), "weights"))) return rc;
    return nn::nn_hip(hipStreamSynchronize(s), "synchronise");
}

static int copy_out(float* host, const float* dev, size_t count, hipStream_t s) {
    int rc = nn::nn_hip(hipMemcpyAsync(host, dev, count * 4, hipMemcpyDeviceToHost, s), "download");
    if (rc) return rc;
    return nn::nn_hip(hipStreamSynchronize(s), "synchronise");
}

int rbgs_unet_get_params(rbgs_unet* u, float* host, size_t count, void* stream) {
    if (!u || !host || count != u->net.nparam) return nn::nnfail(RBGS_EINVAL, "bad parameter vector");
    return copy_out(host, u->net.param, count, static_cast<hipStream_t>(stream));
}

int rbgs_unet_get_grads(rbgs_unet* u, float* host, size_t count, void* stream) {
    if (!u || !host || count != u->net.nparam) return nn::nnfail(RBGS_EINVAL, "bad gradient vector");
    return copy_out(host, u->net.grad, count, static_cast<hipStream_t>(stream));
}

int rbgs_unet_get_adam(rbgs_unet* u, float* m, float* v, size_t count, int32_t* step,
                       void* stream) {
    if (!u || !m || !v || !step || count != u->net.nparam)
        return nn::nnfail(RBGS_EINVAL, "bad Adam state arrays");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = copy_out(m, u->net.m, count, s);
    if (rc) return rc;
    if ((rc = copy_out(v, u->net.v, count, s))) return rc;
    *step = int32_t(u->net.adam_t);
    return RBGS_OK;
}

int rbgs_unet_set_adam(rbgs_unet* u, const float* m, const float* v, size_t count, int32_t step,
                       void* stream) {
    if (!u || !m || !v || count != u->net.nparam || step < 0)
        return nn::nnfail(RBGS_EINVAL, "bad Adam state arrays or step");
    hipStream_t s = static_cast<hipStream_t>(stream);
    nn::Net& net = u->net;
    int rc = nn::nn_hip(hipMemcpyAsync(net.m, m, count * 4, hipMemcpyHostToDevice, s), "upload");
    if (rc) return rc;
    if ((rc = nn::nn_hip(hipMemcpyAsync(net.v, v, count * 4, hipMemcpyHostToDevice, s), "upload")))
        return rc;
    net.adam_t = step;
    return nn::nn_hip(hipStreamSynchronize(s), "synchronise");
}

int rbgs_unet_forward(rbgs_unet* u, int32_t batch, const double* f, int64_t ld, double* u0,
                      void* stream) {
    if (!u || !f || !u0) return nn::nnfail(RBGS_EINVAL, "NULL argument");
    nn::Net& net = u->net;
    if (batch < 1 || batch > net.batch) return nn::nnfail(RBGS_EINVAL, "batch out of range");
    if (ld < int64_t(net.n[0]) + 2) return nn::nnfail(RBGS_EINVAL, "ld must be >= n + 2");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t gs = int64_t(net.n[0] + 2) * ld;
    int rc = nn::nn_hip(nn::forward(net, batch, f, ld, gs, s), "forward");
    if (rc) return rc;
    const int n0 = net.n[0];
    hipLaunchKernelGGL(nn::k_output, dim3(nn::blocks_for(int64_t(batch) * n0 * n0)), dim3(256), 0, s,
                       net.y, net.rms, u0, n0, ld, gs, batch);
    return nn::nn_hip(hipGetLastError(), "output");
}

int rbgs_unet_train_step(rbgs_unet* u, int32_t batch, const double* f, const double* target,
                         int64_t ld, float lr, int32_t update, float* loss, void* stream) {
    if (!u || !f || !target) return nn::nnfail(RBGS_EINVAL, "NULL argument");
    nn::Net& net = u->net;
    if (batch < 1 || batch > net.batch) return nn::nnfail(RBGS_EINVAL, "batch out of range");
    if (ld < int64_t(net.n[0]) + 2) return nn::nnfail(RBGS_EINVAL, "ld must be >= n + 2");
    if (!(lr >= 0.f)) return nn::nnfail(RBGS_EINVAL, "lr must be >= 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t gs = int64_t(net.n[0] + 2) * ld;
    const int n0 = net.n[0];
    int rc = nn::nn_hip(nn::forward(net, batch, f, ld, gs, s), "forward");
    if (rc) return rc;
    const unsigned mblocks = nn::blocks_for(int64_t(batch) * n0 * n0);
    hipLaunchKernelGGL(nn::k_mse, dim3(mblocks), dim3(256), 0, s, net.y, target, net.rms, n0, ld,
                       gs, batch, net.dy, net.parts);
    if ((rc = nn::nn_hip(hipGetLastError(), "loss"))) return rc;
    hipLaunchKernelGGL(nn::k_reduce_parts, dim3(1), dim3(256), 0, s, net.parts, int64_t(mblocks),
                       int64_t(1), net.loss);
    if ((rc = nn::nn_hip(hipGetLastError(), "loss"))) return rc;
    if ((rc = nn::nn_hip(nn::backward(net, batch, s), "backward"))) return rc;
    if (update && (rc = nn::nn_hip(nn::adam(net, lr, s), "adam"))) return rc;
    if (loss) {
        if ((rc = copy_out(loss, net.loss, 1, s))) return rc;
    }
    return RBGS_OK;
}

int rbgs_solve_learned(rbgs_unet* u, const rbgs_grid* g, double* uu, const double* f,
                       const rbgs_solve_opts* o, int32_t compare_after, rbgs_solve_info* info,
                       int32_t* used_guess, double* rel_start, void* workspace,
                       size_t workspace_bytes, void* stream) {
    if (!u || !g || !uu || !f || !o) return nn::nnfail(RBGS_EINVAL, "NULL argument");
    nn::Net& net = u->net;
    if (g->n != net.n[0]) return nn::nnfail(RBGS_EINVAL, "grid size differs from the network's");
    if (g->ld != int64_t(g->n) + 2)
        return nn::nnfail(RBGS_EINVAL, "the learned solve needs a dense grid (ld = n + 2)");
    if (compare_after < 0 || compare_after > o->max_sweeps)
        return nn::nnfail(RBGS_EINVAL, "compare_after must be in [0, max_sweeps]");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int n = g->n;
    const size_t bytes = size_t(n + 2) * size_t(n + 2) * 8;
    // The caller's start (normally zero inside the Dirichlet ring) and the
    // network's guess on the same ring; after compare_after sweeps of both
    // (0: as they are), keep whichever has the lower relative residual.  The
    // plain start is both fallback and judge.
    int rc = nn::nn_hip(hipMemcpyAsync(net.guess, uu, bytes, hipMemcpyDeviceToDevice, s), "copy");
    if (rc) return rc;
    if ((rc = rbgs_unet_forward(u, 1, f, g->ld, net.guess, stream))) return rc;
    if (compare_after > 0) {
        rbgs_sweep_opts so = o->sweep;
        so.timing = nullptr;
        if ((rc = rbgs_sweep(g, RBGS_F64, uu, f, compare_after, &so, workspace, workspace_bytes, stream)) ||
            (rc = rbgs_sweep(g, RBGS_F64, net.guess, f, compare_after, &so, workspace,
                             workspace_bytes, stream)))
            return nn::nnfail(rc, rbgs_last_error());
    }
    double rel0 = 0.0, reln = 0.0;
    rc = rbgs_residual(g, RBGS_F64, uu, f, nullptr, &rel0, workspace, workspace_bytes, stream);
    if (rc) return nn::nnfail(rc, rbgs_last_error());
    rc = rbgs_residual(g, RBGS_F64, net.guess, f, nullptr, &reln, workspace, workspace_bytes, stream);
    if (rc) return nn::nnfail(rc, rbgs_last_error());
    const bool use = reln < rel0;
    if (use) {
        rc = nn::nn_hip(hipMemcpyAsync(uu, net.guess, bytes, hipMemcpyDeviceToDevice, s), "copy");
        if (rc) return rc;
    }
    if (used_guess) *used_guess = use ? 1 : 0;
    if (rel_start) *rel_start = use ? reln : rel0;
    rbgs_solve_opts rest = *o;
    rest.max_sweeps = o->max_sweeps - compare_after;
    rbgs_solve_info inner{0, 0, 0.0, 0.0, RBGS_OK};
    rc = rbgs_solve(g, RBGS_F64, uu, f, &rest, &inner, workspace, workspace_bytes, stream);
    // the work done: the comparison sweeps of both starts, then the solve
    inner.sweeps += 2 * compare_after;
    if (info) *info = inner;
    return rc;
}

}  // extern "C"
