// k_unet.hip -- the learned part of the Poisson solve: a small U-Net whose
// convolutions run on the gfx950 BF16 matrix cores (v_mfma_f32_32x32x16_bf16,
// FP32 accumulation), its backward pass and Adam training on the GPU, the
// training set dumped from the method's own (charge, potential) pairs, and its
// use as the preconditioner of flexible CG (k_mgpcg.hip).
//
// Network (levels L, base width C; 3x3 convolutions bias-free + ReLU; 2x2
// average pooling; nearest 2x upsampling; decoder input = [skip, upsampled]):
//   enc_0 = conv(conv(x)), enc_l = conv(conv(pool(enc_{l-1}))), dec_{L-1} = enc_{L-1},
//   dec_l = conv(conv(cat(enc_l, up(dec_{l+1})))), out = conv1x1(dec_0).
// Input channels: b / rms(b) (the volume-weighted right-hand side of the node
// equations, interior rows) and r / R; output: the potential over its RMS.
// A bias-free ReLU network is positively homogeneous, so it can be applied to
// any positive multiple of a residual.
//
// Layouts: activations NHWC in BF16 with channels padded to multiples of 16;
// gradients of activations NHWC in FP32; 3x3 weights packed as
// [c_out (rows padded to tiles of 32)][tap][c_in padded] in BF16 with
// tap = 3 (dy + 1) + (dx + 1); the master weights FP32 in layer order, each
// layer [c_out][tap][c_in] unpadded.
//
// Convolution = implicit GEMM per wave: D[32 pixels of one row][32 c_out] =
// sum over (tap, 16-channel chunks) of A[pixel][channels at the tapped
// pixel] x B[channels][c_out] (the MFMA's A operand: lane l holds row l%32,
// k = 8 (l/32) .. +7; B: column l%32, same k; D: lane l, register i holds
// row 8 (i/4) + 4 (l/32) + i%4, column l%32).  The decoder's concatenation
// and upsampling are read in place (channels past the skip's come from the
// half-resolution tensor at (y/2, x/2)).  The data gradient is the same
// kernel on the output gradient with the weights transposed and the taps
// mirrored; the weight gradient is an MFMA product over pixels, split into
// partial sums that a second kernel adds in a fixed order.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "pd_internal.h"

namespace pd {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

inline int up16(int c) { return (c + 15) / 16 * 16; }
inline int tiles32(int c) { return (c + 31) / 32; }
inline int gridn(int64_t n, int b = 256) {
  int64_t g = (n + b - 1) / b;
  return (int)(g < 1 ? 1 : (g > 65535 ? 65535 : g));
}

// ---- convolution (forward, and data gradient with mirrored weights) ----------
struct ConvArgs {
  const __bf16* in0;  // [N][H][W][c0]
  const __bf16* in1;  // [N][H/2][W/2][c1] or NULL
  const __bf16* w;    // [rows][9][c0 + c1], rows = cog * NT * 32
  int c0, c1, N, H, W;
  int cot;            // c_out tiles of 32 holding real outputs
  int cstore;         // channels of the output tensor
  __bf16* out_bf;     // BF16 output (ReLU if relu), or
  float* out_f;       // FP32 output
  int relu;
  const int* done;    // skip the launch when *done (solver use), or NULL
};

// Block = 4 waves over 4 MT image rows x 32 columns and NT x 32 output
// channels; wave w takes rows w MT .. w MT + MT - 1 (MT x NT accumulator
// tiles).  Per 16-channel chunk the input patch (rows and columns with a
// one-pixel halo, zero outside the image) and the weights [tap][c_out][16]
// are staged in LDS; the MFMA operands are then 16-byte LDS reads (A: 32
// consecutive pixels of one patch row, B: 32 consecutive output channels),
// both conflict-free.
template <int MT, int NT>
__global__ void __launch_bounds__(256) k_conv3x3(ConvArgs a) {
  constexpr int PR = 4 * MT + 2, PW = 34, NC = NT * 32;
  __shared__ bf16x8 ps[PR * PW * 2];
  __shared__ bf16x8 wl[9 * NC * 2];
  if (a.done && *a.done) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, h = lane >> 5, l32 = lane & 31;
  const int cog = (a.cot + NT - 1) / NT;
  const int n = blockIdx.z / cog, cob = (blockIdx.z % cog) * NC;
  const int y0 = blockIdx.y * 4 * MT, x0 = blockIdx.x * 32;
  const int cin = a.c0 + a.c1;
  const int Hh = a.H >> 1, Wh = a.W >> 1;
  f32x16 acc[MT][NT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int q = 0; q < NT; ++q)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[mt][q][i] = 0.f;
  bf16x8 zero;
#pragma unroll
  for (int i = 0; i < 8; ++i) zero[i] = (__bf16)0.f;
  for (int c = 0; c < cin; c += 16) {
    __syncthreads();
    // input patch: unit u = (pixel, half)
    for (int u = t; u < PR * PW * 2; u += 256) {
      const int pp = u >> 1, half = u & 1, r = pp / PW, cx = pp - r * PW;
      const int y = y0 - 1 + r, x = x0 - 1 + cx;
      bf16x8 v = zero;
      if (y >= 0 && y < a.H && x >= 0 && x < a.W) {
        if (c < a.c0)
          v = *(const bf16x8*)(a.in0 + (((size_t)n * a.H + y) * a.W + x) * a.c0 + c + 8 * half);
        else
          v = *(const bf16x8*)(a.in1 + (((size_t)n * Hh + (y >> 1)) * Wh + (x >> 1)) * a.c1 +
                               (c - a.c0) + 8 * half);
      }
      ps[u] = v;
    }
    // weights: unit u = ((tap, co), half)
    for (int u = t; u < 9 * NC * 2; u += 256) {
      const int half = u & 1, tc = u >> 1, tap = tc / NC, co = tc - tap * NC;
      wl[u] = *(const bf16x8*)(a.w + ((size_t)(cob + co) * 9 + tap) * cin + c + 8 * half);
    }
    __syncthreads();
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int dy = tap / 3, dx = tap % 3;
      bf16x8 bv[NT];
#pragma unroll
      for (int q = 0; q < NT; ++q) bv[q] = wl[(tap * NC + q * 32 + l32) * 2 + h];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const bf16x8 av = ps[((w * MT + mt + dy) * PW + l32 + dx) * 2 + h];
#pragma unroll
        for (int q = 0; q < NT; ++q)
          acc[mt][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv[q], acc[mt][q], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    const int co = cob + q * 32 + l32;
    if (co >= a.cstore) continue;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int y = y0 + w * MT + mt;
      if (y >= a.H) continue;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int x = x0 + 8 * (i / 4) + 4 * h + (i % 4);
        if (x >= a.W) continue;
        const size_t o = (((size_t)n * a.H + y) * a.W + x) * a.cstore + co;
        const float v = acc[mt][q][i];
        if (a.out_bf) a.out_bf[o] = (__bf16)(a.relu ? (v > 0.f ? v : 0.f) : v);
        else a.out_f[o] = v;
      }
    }
  }
}

// ---- weight gradient: part[s][co][tap][ci] = sum over the split's pixels ----
struct WgradArgs {
  const __bf16* dP;   // [N][H][W][cop]
  const __bf16* in0;  // forward input sources, as in ConvArgs
  const __bf16* in1;
  int cop, c0, c1, N, H, W;
  int cit;            // c_in tiles of 32
  int nsplit;
  float* part;        // [nsplit][cot*32][9][cit*32]
};

__global__ void __launch_bounds__(64) k_wgrad(WgradArgs a) {
  const int lane = threadIdx.x, h = lane >> 5, l32 = lane & 31;
  const int co0 = (blockIdx.x / a.cit) * 32, ci0 = (blockIdx.x % a.cit) * 32;
  const int tap = blockIdx.y, dy = tap / 3 - 1, dx = tap % 3 - 1;
  const int s = blockIdx.z;
  const int cin = a.c0 + a.c1, co = co0 + l32, ci = ci0 + l32;
  const int Hh = a.H >> 1, Wh = a.W >> 1;
  // pixels in chunks of 16 along image rows: chunk = (row, 16-pixel segment)
  const int xc = (a.W + 15) / 16;
  const int total = a.N * a.H * xc;
  const bool coin = co < a.cop, ciin = ci < cin, from0 = ci < a.c0;
  f32x16 acc;
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.f;
  for (int ch = s; ch < total; ch += a.nsplit) {
    const int row = ch / xc, x0 = (ch - row * xc) * 16 + 8 * h;
    const int n = row / a.H, y = row - n * a.H, yy = y + dy;
    const bool rowin = yy >= 0 && yy < a.H && ciin;
    const __bf16* pa = a.dP + ((size_t)row * a.W) * a.cop + co;
    const __bf16* pb = from0 ? a.in0 + (((size_t)n * a.H + yy) * a.W) * a.c0 + ci
                             : a.in1 + (((size_t)n * Hh + (yy >> 1)) * Wh) * a.c1 + (ci - a.c0);
    bf16x8 av, bv;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int x = x0 + i, xx = x + dx;
      av[i] = (coin && x < a.W) ? pa[(size_t)x * a.cop] : (__bf16)0.f;
      const bool ok = rowin && x < a.W && xx >= 0 && xx < a.W;
      bv[i] = ok ? (from0 ? pb[(size_t)xx * a.c0] : pb[(size_t)(xx >> 1) * a.c1]) : (__bf16)0.f;
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
  }
  const int CoT = gridDim.x / a.cit * 32, CiT = a.cit * 32;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int r = co0 + 8 * (i / 4) + 4 * h + (i % 4);
    a.part[(((size_t)s * CoT + r) * 9 + tap) * CiT + ci] = acc[i];
  }
}

// grad[off + (co 9 + tap) cin + ci] = sum_s part (real channels only; the
// padded channel of real input channel ci is pmap(ci))
__global__ void k_wgrad_reduce(const float* part, int nsplit, int CoT, int CiT, int cout, int cin,
                               int cskip, int c0p, float* grad) {
  const int n = cout * 9 * cin;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    const int ci = t % cin, tap = (t / cin) % 9, co = t / (9 * cin);
    const int cp = ci < cskip ? ci : c0p + (ci - cskip);
    float s = 0.f;
    for (int k = 0; k < nsplit; ++k) s += part[(((size_t)k * CoT + co) * 9 + tap) * CiT + cp];
    grad[t] = s;
  }
}

// ---- elementwise pieces ------------------------------------------------------
__global__ void k_avgpool(const __bf16* in, __bf16* out, int N, int H, int W, int C,
                          const int* done) {
  if (done && *done) return;
  const int64_t n = (int64_t)N * H * W * C;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(t % C);
    const int64_t p = t / C;
    const int x = (int)(p % W), y = (int)((p / W) % H), b = (int)(p / ((int64_t)W * H));
    const size_t i0 = (((size_t)b * 2 * H + 2 * y) * 2 * W + 2 * x) * C + c;
    const size_t rs = (size_t)2 * W * C;
    const float s = ((float)in[i0] + (float)in[i0 + C]) + ((float)in[i0 + rs] + (float)in[i0 + rs + C]);
    out[t] = (__bf16)(0.25f * s);
  }
}

// out[p] = sum_c w[c] in[p][c] (FP32)
__global__ void k_conv1x1(const __bf16* in, const float* w, int C, int64_t P, float* out,
                          const int* done) {
  if (done && *done) return;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P;
       p += (int64_t)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int c = 0; c < C; ++c) s += w[c] * (float)in[p * C + c];
    out[p] = s;
  }
}

// loss: mean over the real interior nodes of (out - y)^2; dout = d loss / d out;
// per-block partial sums of the squared error
__global__ void __launch_bounds__(256) k_loss(const float* out, const float* y, int N, int H, int W,
                                              int nr, int nz, float* dout, double* part) {
  const int64_t P = (int64_t)N * H * W;
  const double cnt = (double)N * (nz - 1) * (nr + 1);
  double acc = 0.0;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(p % W), j = (int)((p / W) % H);
    float d = 0.f;
    if (j >= 1 && j < nz && x <= nr) {
      const float e = out[p] - y[p];
      acc += (double)e * e;
      d = (float)(2.0 * e / cnt);
    }
    dout[p] = d;
  }
  __shared__ double sh[256];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0] / cnt;
}

// 1x1 layer backward: g[p][c] = w[c] dout[p]; partials of sum_p dout[p] in[p][c]
template <int C>
__global__ void __launch_bounds__(256) k_conv1x1_bwd(const __bf16* in, const float* w, int64_t P,
                                                     const float* dout, float* g, float* part) {
  float acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = 0.f;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P;
       p += (int64_t)gridDim.x * blockDim.x) {
    const float d = dout[p];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      g[p * C + c] = w[c] * d;
      acc[c] += d * (float)in[p * C + c];
    }
  }
  __shared__ float sh[256];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    sh[threadIdx.x] = acc[c];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x * C + c] = sh[0];
    __syncthreads();
  }
}

// out[c] = sum_b part[b][c]: one block per column, fixed order
__global__ void __launch_bounds__(256) k_reduce_cols(const float* part, int nb, int C, float* out) {
  const int c = blockIdx.x;
  float s = 0.f;
  for (int b = threadIdx.x; b < nb; b += 256) s += part[b * C + c];
  __shared__ float sh[256];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = sh[0];
}

// dP = bf16(g * (y > 0))
__global__ void k_relu_mask(const float* g, const __bf16* y, int64_t n, __bf16* dP) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    dP[t] = (__bf16)((float)y[t] > 0.f ? g[t] : 0.f);
}

// dst[p][c] += src[p][c_off + c], c < Cd (src has Cs channels)
__global__ void k_add_into(float* dst, const float* src, int64_t P, int Cd, int Cs, int c_off) {
  const int64_t n = P * Cd;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = t / Cd;
    dst[t] += src[p * Cs + c_off + (t % Cd)];
  }
}

// dst (half resolution, Cd channels) += sum over each 2x2 block of src[..][c_off + c]
__global__ void k_sumpool_into(float* dst, const float* src, int N, int Hh, int Wh, int Cd, int Cs,
                               int c_off) {
  const int64_t n = (int64_t)N * Hh * Wh * Cd;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(t % Cd);
    const int64_t p = t / Cd;
    const int x = (int)(p % Wh), y = (int)((p / Wh) % Hh), b = (int)(p / ((int64_t)Wh * Hh));
    const size_t W = 2 * (size_t)Wh;
    const size_t i0 = (((size_t)b * 2 * Hh + 2 * y) * W + 2 * x) * Cs + c_off + c;
    const size_t rs = W * Cs;
    dst[t] += (src[i0] + src[i0 + Cs]) + (src[i0 + rs] + src[i0 + rs + Cs]);
  }
}

// average-pooling backward: dst (full resolution) += src (half) / 4
__global__ void k_unpool_into(float* dst, const float* src, int N, int H, int W, int C) {
  const int64_t n = (int64_t)N * H * W * C;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(t % C);
    const int64_t p = t / C;
    const int x = (int)(p % W), y = (int)((p / W) % H), b = (int)(p / ((int64_t)W * H));
    dst[t] += 0.25f * src[((((size_t)b * (H / 2) + y / 2) * (W / 2)) + x / 2) * C + c];
  }
}

__global__ void k_zero_f(float* p, int64_t n) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    p[t] = 0.f;
}

// master FP32 layer [cout][9][cin] -> forward [rows][9][cin_p] and mirrored
// backward [rows_b][9][cout_p] BF16 (zero padding); pmap as in k_wgrad_reduce
__global__ void k_pack(const float* w, int cout, int cin, int cskip, int c0p, int cinp, int rows,
                       int coutp, int rows_b, __bf16* wf, __bf16* wb) {
  const int nf = rows * 9 * cinp, nb = rows_b * 9 * coutp;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nf + nb; t += gridDim.x * blockDim.x) {
    if (t < nf) {
      const int cp = t % cinp, tap = (t / cinp) % 9, co = t / (9 * cinp);
      int ci = -1;
      if (cp < c0p) ci = cp < cskip ? cp : -1;
      else ci = (cp - c0p) < (cin - cskip) ? cskip + (cp - c0p) : -1;
      const float v = (co < cout && ci >= 0) ? w[(co * 9 + tap) * cin + ci] : 0.f;
      wf[t] = (__bf16)v;
    } else {
      const int u = t - nf;
      const int co = u % coutp, tap = (u / coutp) % 9, cp = u / (9 * coutp);
      int ci = -1;
      if (cp < c0p) ci = cp < cskip ? cp : -1;
      else ci = (cp - c0p) < (cin - cskip) ? cskip + (cp - c0p) : -1;
      const float v = (co < cout && ci >= 0 && cp < cinp) ? w[(co * 9 + (8 - tap)) * cin + ci] : 0.f;
      wb[u] = (__bf16)v;
    }
  }
}

__global__ void k_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const float gt = g[t];
    const float mt = b1 * m[t] + (1.f - b1) * gt;
    const float vt = b2 * v[t] + (1.f - b2) * gt * gt;
    m[t] = mt;
    v[t] = vt;
    w[t] -= lr * (mt / c1) / (sqrtf(vt / c2) + eps);
  }
}

// host input [n][2][H][W] FP32 -> [n][H][W][16] BF16
__global__ void k_input_from_nchw(const float* x, int N, int H, int W, __bf16* out) {
  const int64_t n = (int64_t)N * H * W * 16;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(t % 16);
    const int64_t p = t / 16;
    const int64_t HW = (int64_t)H * W;
    out[t] = (__bf16)(c < 2 ? x[(p / HW) * 2 * HW + c * HW + p % HW] : 0.f);
  }
}

// training batch: ch0 from the stored normalised b, ch1 = r/R on the real
// nodes, target from the stored normalised potential
__global__ void k_batch(const __bf16* dsx, const __bf16* dsy, const int* idx, int N, int H, int W,
                        int nr, int nz, __bf16* xin, float* y) {
  const int64_t HW = (int64_t)H * W, n = (int64_t)N * HW;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = t % HW;
    const int b = (int)(t / HW);
    const int x = (int)(p % W), j = (int)(p / W);
    const size_t src = (size_t)idx[b] * HW + p;
    __bf16* o = xin + t * 16;
    o[0] = dsx[src];
    o[1] = (__bf16)((x <= nr && j <= nz) ? (float)x / (float)nr : 0.f);
    for (int c = 2; c < 16; ++c) o[c] = (__bf16)0.f;
    y[t] = (float)dsy[src];
  }
}

// ---- dataset: one (b, phi_p) pair from the method's current state ------------
__global__ void __launch_bounds__(256) k_sample_stats(MGOp64 o, const double* phi, const int64_t* Q,
                                                      double V, double* part) {
  const int Wn = o.nr + 1, n = Wn * (o.nz - 1);
  double sb = 0.0, sp = 0.0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    const int i = t % Wn, j = 1 + t / Wn, q = j * Wn + i;
    const double b = o.w[i] * ((((double)Q[q] * o.qunit) / o.Vnode[i]) / kEPS0);
    const double pp = phi[q] - ((-V) + (V * ((double)j / (double)o.nz)));
    sb += b * b;
    sp += pp * pp;
  }
  __shared__ double s0[256], s1[256];
  s0[threadIdx.x] = sb;
  s1[threadIdx.x] = sp;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) {
      s0[threadIdx.x] += s0[threadIdx.x + k];
      s1[threadIdx.x] += s1[threadIdx.x + k];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s0[0];
    part[2 * blockIdx.x + 1] = s1[0];
  }
}

__global__ void __launch_bounds__(256) k_sample_write(MGOp64 o, const double* phi, const int64_t* Q,
                                                      double V, const double* part, int nb, int H,
                                                      int W, __bf16* dx, __bf16* dy) {
  __shared__ double scale[2];
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int k = 0; k < nb; ++k) {
      a += part[2 * k];
      b += part[2 * k + 1];
    }
    const double cnt = (double)(o.nr + 1) * (o.nz - 1);
    scale[0] = a > 0 ? 1.0 / sqrt(a / cnt) : 0.0;
    scale[1] = b > 0 ? 1.0 / sqrt(b / cnt) : 0.0;
  }
  __syncthreads();
  const int n = H * W;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    const int i = t % W, j = t / W;
    float vx = 0.f, vy = 0.f;
    if (j >= 1 && j < o.nz && i <= o.nr) {
      const int q = j * (o.nr + 1) + i;
      const double b = o.w[i] * ((((double)Q[q] * o.qunit) / o.Vnode[i]) / kEPS0);
      const double pp = phi[q] - ((-V) + (V * ((double)j / (double)o.nz)));
      vx = (float)(b * scale[0]);
      vy = (float)(pp * scale[1]);
    }
    dx[t] = (__bf16)vx;
    dy[t] = (__bf16)vy;
  }
}

// ---- preconditioner glue -------------------------------------------------------
// iteration gate (as in the V-cycle's first kernel) + network input from the
// CG residual r (level-0 layout, interior rows), scaled to unit RMS
__global__ void __launch_bounds__(256) k_pack_residual(MGLevel m, MGScal* sc, const float* part_rr,
                                                       int nb, int it, int H, int W, __bf16* xin) {
  __shared__ int go;
  __shared__ float scale;
  if (threadIdx.x == 0) {
    int g = sc->done ? 0 : 1;
    float rr = 1.f;  // the first iteration's residual has unit norm
    if (g && it > 0) {
      rr = 0.f;
      for (int b = 0; b < nb; ++b) rr += part_rr[b];
      if (!(rr > sc->tol2)) g = 0;
    }
    go = g;
    scale = sqrtf((float)((m.nr + 1) * (m.nz - 1)) / rr);
    if (blockIdx.x == 0) {
      if (!g) sc->done = 1;
      else {
        sc->iters += 1;
        sc->it_last = it + 1;
      }
    }
  }
  __syncthreads();
  if (!go) return;
  const int Wn = m.nr + 1;
  const int n = H * W;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    const int i = t % W, j = t / W;
    const bool real = j <= m.nz && i <= m.nr;
    const bool inner = real && j >= 1 && j < m.nz;
    __bf16* o = xin + (size_t)t * 16;
    o[0] = (__bf16)(inner ? m.b[j * Wn + i] * scale : 0.f);
    o[1] = (__bf16)(real ? (float)i / (float)m.nr : 0.f);
    for (int c = 2; c < 16; ++c) o[c] = (__bf16)0.f;
  }
}

// z (level-0 layout) = network output on the interior rows
__global__ void k_unpack_z(const float* out, int W, MGLevel m, const MGScal* sc) {
  if (sc->done) return;
  const int Wn = m.nr + 1, n = Wn * (m.nz - 1);
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    const int i = t % Wn, j = 1 + t / Wn;
    m.x[j * Wn + i] = out[(size_t)j * W + i];
  }
}

}  // namespace

// ---------------------------------------------------------------------------
struct Unet {
  struct Layer {
    int cout, cin, k;  // oracle shape
    int level, cskip;  // cskip < cin: concat (skip channels first)
    int c0p, c1p;      // padded channels of the two input sources
    int coutp;         // padded output channels (multiple of 16)
    int rows, rows_b;  // packed weight rows (multiples of NT * 32)
    int64_t off;       // offset in the flat weights
    __bf16 *wf = nullptr, *wb = nullptr;
  };
  int nr = 0, nz = 0, L = 0, C = 0, H = 0, W = 0, nbmax = 0;
  std::vector<Layer> layers;
  int64_t np = 0;
  float *master = nullptr, *grad = nullptr, *am = nullptr, *av = nullptr;
  int64_t adam_t = 0;
  std::vector<void*> allocs;
  // activations (BF16) per name and their FP32 gradients
  __bf16* xin = nullptr;
  std::vector<__bf16*> act;   // index = layer (3x3 layers), output of that conv
  std::vector<__bf16*> pooled;  // pooled[l] = pool(enc_{l-1} b), l >= 1
  std::vector<float*> gact;   // gradient of act
  float *out = nullptr, *gout = nullptr, *target = nullptr, *tmp = nullptr, *wpart = nullptr;
  float* opart = nullptr;
  double* lpart = nullptr;
  __bf16* dP = nullptr;
  size_t wpart_n = 0, tmp_n = 0;
  // dataset
  __bf16 *dsx = nullptr, *dsy = nullptr;
  int64_t ds_cap = 0, ds_n = 0;
  double* spart = nullptr;
  int* idx = nullptr;
  std::string err;

  int lh(int l) const { return H >> l; }
  int lw(int l) const { return W >> l; }
};

namespace {

template <class T>
bool ualloc(Unet* u, T** p, size_t n) {
  void* q = nullptr;
  if (hipMalloc(&q, (n ? n : 1) * sizeof(T)) != hipSuccess) return false;
  u->allocs.push_back(q);
  *p = (T*)q;
  return true;
}

constexpr int kNT = 2;

// pixel splits of a weight-gradient launch: about 4096 waves in all, at
// most one split per 16-pixel chunk
int wgrad_splits(int cot, int cit, int chunks) {
  int ns = 4096 / (cot * cit * 9);
  ns = std::max(1, std::min(512, ns));
  return std::min(ns, std::max(1, chunks));
}

int nt_for(int cot) { return cot >= 2 ? kNT : 1; }

void conv(const Unet& u, int N, int level, const __bf16* in0, int c0, const __bf16* in1, int c1,
          const __bf16* w, int cot, int cstore, __bf16* out_bf, float* out_f, int relu,
          const int* done, hipStream_t s) {
  ConvArgs a{in0, in1, w, c0, c1, N, u.lh(level), u.lw(level), cot, cstore, out_bf, out_f, relu,
             done};
  const int NT = nt_for(cot);
  if (NT == 1) {  // 4 rows x 32 channels per wave
    dim3 grid((a.W + 31) / 32, (a.H + 15) / 16, N * cot);
    k_conv3x3<4, 1><<<grid, 256, 0, s>>>(a);
  } else {        // 2 rows x 64 channels per wave
    dim3 grid((a.W + 31) / 32, (a.H + 7) / 8, N * ((cot + kNT - 1) / kNT));
    k_conv3x3<2, kNT><<<grid, 256, 0, s>>>(a);
  }
}

// input sources of 3x3 layer k in the forward pass
void sources(const Unet& u, int k, const __bf16** in0, const __bf16** in1) {
  const int L = u.L;
  *in1 = nullptr;
  if (k == 0) *in0 = u.xin;
  else if (k < 2 * L) *in0 = (k % 2 == 1) ? u.act[k - 1] : u.pooled[k / 2];
  else {
    const int d = k - 2 * L;  // decoder index: level l = L - 2 - d / 2
    const int l = L - 2 - d / 2;
    if (d % 2 == 1) *in0 = u.act[k - 1];
    else {
      *in0 = u.act[2 * l + 1];                           // enc_l
      *in1 = (d == 0) ? u.act[2 * L - 1] : u.act[k - 1];  // dec_{l+1}
    }
  }
}

}  // namespace

Unet* unet_create(int nr, int nz, int levels, int base, int nbmax, int64_t ds_cap, std::string& err) {
  if (levels < 1 || levels > 6 || base < 16 || base > 64 || base % 16 || (base << (levels - 1)) > 512 ||
      nbmax < 1 || ds_cap < 0 || nr < 2 || nz < 2) {
    err = "invalid network size";
    return nullptr;
  }
  Unet* u = new Unet();
  u->nr = nr;
  u->nz = nz;
  u->L = levels;
  u->C = base;
  u->nbmax = nbmax;
  const int m = 1 << (levels - 1);
  u->H = (nz + 1 + m - 1) / m * m;
  u->W = (nr + 1 + m - 1) / m * m;
  // layers in the oracle order
  auto add = [&](int cout, int cin, int level, int cskip, int c0p, int c1p) {
    Unet::Layer ly;
    ly.cout = cout;
    ly.cin = cin;
    ly.k = 3;
    ly.level = level;
    ly.cskip = cskip;
    ly.c0p = c0p;
    ly.c1p = c1p;
    ly.coutp = up16(cout);
    const int cot = tiles32(cout), NT = nt_for(cot);
    ly.rows = (cot + NT - 1) / NT * NT * 32;
    const int cotb = tiles32(c0p + c1p), NTb = nt_for(cotb);
    ly.rows_b = (cotb + NTb - 1) / NTb * NTb * 32;
    ly.off = u->np;
    u->np += (int64_t)cout * 9 * cin;
    u->layers.push_back(ly);
  };
  int cprev = 2, cprevp = 16;
  for (int l = 0; l < levels; ++l) {
    const int c = base << l;
    add(c, cprev, l, cprev, cprevp, 0);
    add(c, c, l, c, up16(c), 0);
    cprev = c;
    cprevp = up16(c);
  }
  for (int l = levels - 2; l >= 0; --l) {
    const int c = base << l, cu = base << (l + 1);
    add(c, c + cu, l, c, up16(c), up16(cu));
    add(c, c, l, c, up16(c), 0);
  }
  const int64_t off1 = u->np;
  u->np += base;  // 1x1 output layer
  (void)off1;
  bool ok = ualloc(u, &u->master, u->np) && ualloc(u, &u->grad, u->np) && ualloc(u, &u->am, u->np) &&
            ualloc(u, &u->av, u->np);
  const int N = nbmax;
  ok = ok && ualloc(u, &u->xin, (size_t)N * u->H * u->W * 16);
  u->act.assign(u->layers.size(), nullptr);
  u->gact.assign(u->layers.size(), nullptr);
  u->pooled.assign(levels, nullptr);
  size_t maxact = 0;
  for (size_t k = 0; k < u->layers.size() && ok; ++k) {
    Unet::Layer& ly = u->layers[k];
    const size_t n = (size_t)N * u->lh(ly.level) * u->lw(ly.level) * ly.coutp;
    ok = ualloc(u, &u->act[k], n) && ualloc(u, &u->gact[k], n) &&
         ualloc(u, &ly.wf, (size_t)ly.rows * 9 * (ly.c0p + ly.c1p)) &&
         ualloc(u, &ly.wb, (size_t)ly.rows_b * 9 * ly.coutp);
    maxact = std::max(maxact, (size_t)N * u->lh(ly.level) * u->lw(ly.level) * (ly.c0p + ly.c1p));
    maxact = std::max(maxact, n);
    const int cot = ly.rows / 32, cit = tiles32(ly.c0p + ly.c1p);
    const int ns = wgrad_splits(cot, cit, N * u->lh(ly.level) * ((u->lw(ly.level) + 15) / 16));
    u->wpart_n = std::max(u->wpart_n, (size_t)ns * cot * 32 * 9 * cit * 32);
  }
  for (int l = 1; l < levels && ok; ++l)
    ok = ualloc(u, &u->pooled[l], (size_t)N * u->lh(l) * u->lw(l) * up16(base << (l - 1)));
  const size_t P0 = (size_t)N * u->H * u->W;
  u->tmp_n = maxact;
  ok = ok && ualloc(u, &u->out, P0) && ualloc(u, &u->gout, P0) && ualloc(u, &u->target, P0) &&
       ualloc(u, &u->tmp, maxact) && ualloc(u, &u->dP, maxact) && ualloc(u, &u->wpart, u->wpart_n) &&
       ualloc(u, &u->opart, (size_t)1024 * 64) && ualloc(u, &u->lpart, 1024) &&
       ualloc(u, &u->spart, 2 * 1024) && ualloc(u, &u->idx, nbmax);
  u->ds_cap = ds_cap;
  ok = ok && ualloc(u, &u->dsx, (size_t)std::max<int64_t>(ds_cap, 1) * u->H * u->W) &&
       ualloc(u, &u->dsy, (size_t)std::max<int64_t>(ds_cap, 1) * u->H * u->W);
  if (!ok) {
    err = "device allocation failed";
    unet_destroy(u);
    return nullptr;
  }
  return u;
}

void unet_destroy(Unet* u) {
  if (!u) return;
  (void)hipDeviceSynchronize();
  for (void* p : u->allocs) (void)hipFree(p);
  delete u;
}

int64_t unet_nparams(const Unet* u) { return u->np; }
int unet_height(const Unet* u) { return u->H; }
int unet_width(const Unet* u) { return u->W; }
int64_t unet_samples(const Unet* u) { return u->ds_n; }

static void pack_all(Unet* u, hipStream_t s) {
  for (auto& ly : u->layers)
    k_pack<<<256, 256, 0, s>>>(u->master + ly.off, ly.cout, ly.cin, ly.cskip, ly.c0p, ly.c0p + ly.c1p,
                               ly.rows, ly.coutp, ly.rows_b, ly.wf, ly.wb);
}

int unet_set_weights(Unet* u, const float* h, hipStream_t s) {
  if (hipMemcpy(u->master, h, 4 * u->np, hipMemcpyHostToDevice) != hipSuccess) return -1;
  pack_all(u, s);
  k_zero_f<<<gridn(u->np), 256, 0, s>>>(u->am, u->np);
  k_zero_f<<<gridn(u->np), 256, 0, s>>>(u->av, u->np);
  u->adam_t = 0;
  return hipStreamSynchronize(s) == hipSuccess ? 0 : -1;
}

int unet_get_weights(const Unet* u, float* h) {
  return hipMemcpy(h, u->master, 4 * u->np, hipMemcpyDeviceToHost) == hipSuccess ? 0 : -1;
}

// forward of N images already in xin; output FP32 in out [N][H][W]
void unet_forward_dev(Unet* u, int N, const int* done, hipStream_t s) {
  const int L = u->L;
  for (size_t k = 0; k < u->layers.size(); ++k) {
    const Unet::Layer& ly = u->layers[k];
    if (k >= 2 && k < (size_t)2 * L && k % 2 == 0) {
      // pool the previous level's output into this level's input
      const int l = (int)k / 2;
      const int C = u->layers[k - 1].coutp;
      k_avgpool<<<gridn((int64_t)N * u->lh(l) * u->lw(l) * C), 256, 0, s>>>(
          u->act[k - 1], u->pooled[l], N, u->lh(l), u->lw(l), C, done);
    }
    const __bf16 *in0, *in1;
    sources(*u, (int)k, &in0, &in1);
    conv(*u, N, ly.level, in0, ly.c0p, in1, ly.c1p, ly.wf, tiles32(ly.cout), ly.coutp, u->act[k],
         nullptr, 1, done, s);
  }
  const int64_t P = (int64_t)N * u->H * u->W;
  k_conv1x1<<<gridn(P), 256, 0, s>>>(u->act.back(), u->master + (u->np - u->C), u->layers.back().coutp,
                                     P, u->out, done);
}

// gradient of the weights (into grad) for the output gradient in gout
void unet_backward_dev(Unet* u, int N, hipStream_t s) {
  const int L = u->L;
  const int nl = (int)u->layers.size();
  for (int k = 0; k < nl; ++k) {
    const Unet::Layer& ly = u->layers[k];
    k_zero_f<<<gridn((int64_t)N * u->lh(ly.level) * u->lw(ly.level) * ly.coutp), 256, 0, s>>>(
        u->gact[k], (int64_t)N * u->lh(ly.level) * u->lw(ly.level) * ly.coutp);
  }
  const int64_t P0 = (int64_t)N * u->H * u->W;
  {
    const int nb = std::min<int64_t>(1024, (P0 + 255) / 256);
    const __bf16* a0 = u->act.back();
    const float* w1 = u->master + (u->np - u->C);
    switch (u->C) {
      case 16: k_conv1x1_bwd<16><<<nb, 256, 0, s>>>(a0, w1, P0, u->gout, u->gact.back(), u->opart); break;
      case 32: k_conv1x1_bwd<32><<<nb, 256, 0, s>>>(a0, w1, P0, u->gout, u->gact.back(), u->opart); break;
      case 48: k_conv1x1_bwd<48><<<nb, 256, 0, s>>>(a0, w1, P0, u->gout, u->gact.back(), u->opart); break;
      default: k_conv1x1_bwd<64><<<nb, 256, 0, s>>>(a0, w1, P0, u->gout, u->gact.back(), u->opart); break;
    }
    k_reduce_cols<<<u->layers.back().coutp, 256, 0, s>>>(u->opart, nb, u->layers.back().coutp,
                                                        u->grad + (u->np - u->C));
  }
  for (int k = nl - 1; k >= 0; --k) {
    const Unet::Layer& ly = u->layers[k];
    const int l = ly.level, Hl = u->lh(l), Wl = u->lw(l);
    const int64_t Pl = (int64_t)N * Hl * Wl;
    k_relu_mask<<<gridn(Pl * ly.coutp), 256, 0, s>>>(u->gact[k], u->act[k], Pl * ly.coutp, u->dP);
    const __bf16 *in0, *in1;
    sources(*u, k, &in0, &in1);
    // weight gradient
    {
      const int cot = ly.rows / 32, cit = tiles32(ly.c0p + ly.c1p);
      const int nsplit = wgrad_splits(cot, cit, N * Hl * ((Wl + 15) / 16));
      WgradArgs a{u->dP, in0, in1, ly.coutp, ly.c0p, ly.c1p, N, Hl, Wl, cit, nsplit, u->wpart};
      k_wgrad<<<dim3(cot * cit, 9, nsplit), 64, 0, s>>>(a);
      k_wgrad_reduce<<<gridn((int64_t)ly.cout * 9 * ly.cin), 256, 0, s>>>(
          u->wpart, nsplit, cot * 32, cit * 32, ly.cout, ly.cin, ly.cskip, ly.c0p, u->grad + ly.off);
    }
    if (k == 0) continue;  // no gradient for the network input
    // data gradient at full resolution into tmp [Pl][c0p + c1p]
    const int cin_p = ly.c0p + ly.c1p;
    conv(*u, N, l, u->dP, ly.coutp, nullptr, 0, ly.wb, tiles32(cin_p), cin_p, nullptr, u->tmp, 0,
         nullptr, s);
    if (k < 2 * L) {
      if (k % 2 == 1) {
        k_add_into<<<gridn(Pl * cin_p), 256, 0, s>>>(u->gact[k - 1], u->tmp, Pl, cin_p, cin_p, 0);
      } else {
        // input = pool(act[k-1]) at level l: average-pooling backward
        k_unpool_into<<<gridn((int64_t)N * u->lh(l - 1) * u->lw(l - 1) * cin_p), 256, 0, s>>>(
            u->gact[k - 1], u->tmp, N, u->lh(l - 1), u->lw(l - 1), cin_p);
      }
    } else {
      const int d = k - 2 * L;
      if (d % 2 == 1) {
        k_add_into<<<gridn(Pl * cin_p), 256, 0, s>>>(u->gact[k - 1], u->tmp, Pl, cin_p, cin_p, 0);
      } else {
        const int ks = 2 * l + 1;                      // enc_l
        const int kc = (d == 0) ? 2 * L - 1 : k - 1;   // dec_{l+1}
        k_add_into<<<gridn(Pl * ly.c0p), 256, 0, s>>>(u->gact[ks], u->tmp, Pl, ly.c0p, cin_p, 0);
        k_sumpool_into<<<gridn((int64_t)N * (Hl / 2) * (Wl / 2) * ly.c1p), 256, 0, s>>>(
            u->gact[kc], u->tmp, N, Hl / 2, Wl / 2, ly.c1p, cin_p, ly.c0p);
      }
    }
  }
}

int unet_forward_host(Unet* u, int N, const float* x, float* out, hipStream_t s) {
  if (N < 1 || N > u->nbmax) return -1;
  const size_t P = (size_t)N * u->H * u->W;
  float* dx = u->tmp;  // staging: [N][2][H][W] FP32 fits in tmp
  if (hipMemcpy(dx, x, 4 * 2 * P, hipMemcpyHostToDevice) != hipSuccess) return -1;
  k_input_from_nchw<<<gridn((int64_t)P * 16), 256, 0, s>>>(dx, N, u->H, u->W, u->xin);
  unet_forward_dev(u, N, nullptr, s);
  if (hipStreamSynchronize(s) != hipSuccess) return -1;
  return hipMemcpy(out, u->out, 4 * P, hipMemcpyDeviceToHost) == hipSuccess ? 0 : -1;
}

int unet_gradient_host(Unet* u, int N, const float* x, const float* dout, float* dw, hipStream_t s) {
  if (N < 1 || N > u->nbmax) return -1;
  const size_t P = (size_t)N * u->H * u->W;
  if (hipMemcpy(u->tmp, x, 4 * 2 * P, hipMemcpyHostToDevice) != hipSuccess) return -1;
  k_input_from_nchw<<<gridn((int64_t)P * 16), 256, 0, s>>>(u->tmp, N, u->H, u->W, u->xin);
  unet_forward_dev(u, N, nullptr, s);
  if (hipMemcpyAsync(u->gout, dout, 4 * P, hipMemcpyHostToDevice, s) != hipSuccess) return -1;
  unet_backward_dev(u, N, s);
  if (hipStreamSynchronize(s) != hipSuccess) return -1;
  return hipMemcpy(dw, u->grad, 4 * u->np, hipMemcpyDeviceToHost) == hipSuccess ? 0 : -1;
}

int unet_add_sample(Unet* u, const MGOp64& op, const double* phi, const int64_t* Q, double V,
                    hipStream_t s) {
  if (u->ds_n >= u->ds_cap) return -1;
  if (op.nr != u->nr || op.nz != u->nz) return -2;
  const int nb = 256;
  k_sample_stats<<<nb, 256, 0, s>>>(op, phi, Q, V, u->spart);
  const size_t HW = (size_t)u->H * u->W;
  k_sample_write<<<gridn((int64_t)HW), 256, 0, s>>>(op, phi, Q, V, u->spart, nb, u->H, u->W,
                                                     u->dsx + u->ds_n * HW, u->dsy + u->ds_n * HW);
  u->ds_n += 1;
  return 0;
}

// minibatch Adam over the stored pairs; loss = mean squared error of the
// normalised potential over the real interior nodes; returns the mean loss of
// the last epoch
int unet_train(Unet* u, int epochs, int batch, double lr, uint64_t seed, double* loss,
               hipStream_t s) {
  if (batch < 1 || batch > u->nbmax || u->ds_n < 1 || epochs < 1) return -1;
  std::vector<int> perm(u->ds_n);
  uint64_t st = seed ? seed : 1;
  auto rnd = [&]() {  // splitmix64
    uint64_t z = (st += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  const int64_t P = (int64_t)batch * u->H * u->W;
  const int lb = (int)std::min<int64_t>(1024, (P + 255) / 256);
  double last = 0.0;
  std::vector<double> hp(lb);
  for (int e = 0; e < epochs; ++e) {
    for (int64_t k = 0; k < u->ds_n; ++k) perm[k] = (int)k;
    for (int64_t k = u->ds_n - 1; k > 0; --k) std::swap(perm[k], perm[rnd() % (uint64_t)(k + 1)]);
    double tot = 0.0;
    int nbat = 0;
    for (int64_t b0 = 0; b0 + batch <= u->ds_n; b0 += batch) {
      if (hipMemcpyAsync(u->idx, perm.data() + b0, 4 * batch, hipMemcpyHostToDevice, s) != hipSuccess)
        return -1;
      k_batch<<<gridn(P), 256, 0, s>>>(u->dsx, u->dsy, u->idx, batch, u->H, u->W, u->nr, u->nz,
                                       u->xin, u->target);
      unet_forward_dev(u, batch, nullptr, s);
      k_loss<<<lb, 256, 0, s>>>(u->out, u->target, batch, u->H, u->W, u->nr, u->nz, u->gout, u->lpart);
      unet_backward_dev(u, batch, s);
      u->adam_t += 1;
      const float b1 = 0.9f, b2 = 0.999f;
      const float c1 = 1.f - (float)std::pow(b1, (double)u->adam_t);
      const float c2 = 1.f - (float)std::pow(b2, (double)u->adam_t);
      k_adam<<<gridn(u->np), 256, 0, s>>>(u->master, u->grad, u->am, u->av, u->np, (float)lr, b1, b2,
                                          1e-8f, c1, c2);
      pack_all(u, s);
      if (hipMemcpyAsync(hp.data(), u->lpart, 8 * lb, hipMemcpyDeviceToHost, s) != hipSuccess) return -1;
      if (hipStreamSynchronize(s) != hipSuccess) return -1;
      double l = 0.0;
      for (int k = 0; k < lb; ++k) l += hp[k];
      tot += l;
      nbat += 1;
    }
    last = nbat ? tot / nbat : 0.0;
  }
  if (loss) *loss = last;
  return 0;
}

// z = net(r) for the CG residual of level 0 (gated like a V-cycle)
void unet_apply(Unet* u, const MGLevel& m, MGScal* sc, const float* part_rr, int nb, int it,
                hipStream_t s) {
  k_pack_residual<<<gridn((int64_t)u->H * u->W), 256, 0, s>>>(m, sc, part_rr, nb, it, u->H, u->W,
                                                               u->xin);
  unet_forward_dev(u, 1, &sc->done, s);
  k_unpack_z<<<gridn((int64_t)(m.nr + 1) * (m.nz - 1)), 256, 0, s>>>(u->out, u->W, m, sc);
}

}  // namespace pd
