// The warm-start network on gfx950: 3x3 'same' convolutions as implicit GEMMs on the BF16 matrix
// cores (v_mfma_f32_32x32x16_bf16, FP32 accumulation), with the bias, the exact GELU and the
// BF16 rounding fused into the epilogue; the backward pass (data gradient with the GELU
// derivative fused, weight gradient as a pixel-reduction GEMM) on the same instruction; the
// loss, Adam and the parameter packing as plain vector kernels.
//
// Layout: images are NHWC BF16 with 32 channels (8 for the input features and for the output
// gradient, of which 5 and 1 are used); row y, column x of image b at ((b H + y) W + x) C.
// Parameters are FP32 in the layout W[dy][dx][c_in][c_out] then b[c_out] per layer; the kernels
// read BF16 copies packed per use (forward: [tap][c_out][c_in]; data gradient: the taps mirrored
// and the channel roles swapped).
//
// MFMA 32x32x16 lane layout (checked on the device): lane l supplies A[row l%32][k 8(l/32)+j]
// and B[k 8(l/32)+j][col l%32] (j = 0..7) and receives D[8(r/4) + 4(l/32) + r%4][l%32] in
// accumulator r = 0..15.  Here rows are 32 pixels of one image row, columns the 32 output
// channels, and k runs over (tap, input channel).
#include <hip/hip_runtime.h>

#include "cnn_internal.h"

namespace fdd {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
         z * 0.39894228040143268f * expf(-0.5f * z * z);
}

__device__ __forceinline__ bf16x8 zero8() {
  bf16x8 v;
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = (__bf16)0.0f;
  return v;
}

// ---- input features ---------------------------------------------------------------------
// One image per trace: channel 0 the trace value of the column, 1 the height y = j / n, 2 their
// product, 3 log10 K, 4 log10 mu, 5..7 zero.  The trace is scaled to unit root-mean-square
// first (every block recomputes the scale; block 0 of each image stores it).
__global__ __launch_bounds__(256) void k_cnn_features(const double* __restrict__ traces, int ld,
                                                       int n, const double* __restrict__ lk,
                                                       const double* __restrict__ lmu,
                                                       __bf16* __restrict__ X,
                                                       double* __restrict__ scale) {
  const int b = blockIdx.y;
  const int m = n - 1;
  const double* t = traces + (size_t)b * ld;
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < m; i += 256) s += t[i] * t[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const double rms = sqrt(red[0] / m);
  const double inv = rms > 0.0 ? 1.0 / rms : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) scale[b] = rms;
  const float k3 = (float)lk[b], k4 = (float)lmu[b];
  const int64_t npix = (int64_t)m * m;
  for (int64_t p = blockIdx.x * 256 + threadIdx.x; p < npix; p += (int64_t)gridDim.x * 256) {
    const int y = (int)(p / m), x = (int)(p % m);
    const float tv = (float)(t[x] * inv);
    const float yv = (float)(y + 1) / (float)n;
    bf16x8 v = zero8();
    v[0] = (__bf16)tv;
    v[1] = (__bf16)yv;
    v[2] = (__bf16)(yv * tv);
    v[3] = (__bf16)k3;
    v[4] = (__bf16)k4;
    *reinterpret_cast<bf16x8*>(X + ((size_t)b * npix + p) * 8) = v;
  }
}

// ---- convolution (forward, or data gradient) -------------------------------------------------
// Block: 4 waves, an output tile of 4 rows x 32 columns (one row per wave), all 32 output
// channels.  The input tile (6 rows x 34 columns, CIN channels) is staged in LDS with a padded
// pixel stride (bank-conflict-free 16-byte reads); the packed weights of the whole layer live in
// registers as MFMA B fragments.
//   MODE kConvHidden: z = acc + bias; store z (if zout) and gelu(z) as BF16.
//   MODE kConvOut:    out = acc + bias[0] (channel 0), FP32.
//   MODE kConvGrad:   dz_prev = acc * gelu'(z_prev), BF16 (no bias).
template <int CIN, int MODE>
__global__ __launch_bounds__(256) void k_conv(const __bf16* __restrict__ in, int H, int W,
                                              const __bf16* __restrict__ wp,
                                              const float* __restrict__ bias,
                                              __bf16* __restrict__ zout, __bf16* __restrict__ aout,
                                              float* __restrict__ fout,
                                              const __bf16* __restrict__ zprev,
                                              const double* __restrict__ oscale) {
  constexpr int S = CIN == 32 ? 40 : 24;  // LDS pixel stride (elements)
  constexpr int NQ = CIN == 32 ? 18 : 5;  // k chunks of 16
  constexpr int TR = 6, TC = 34;
  __shared__ __attribute__((aligned(16))) __bf16 tile[TR * TC * S];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 4, b = blockIdx.z;
  const size_t img = (size_t)b * H * W;
  // weights -> B fragments (L2-resident; issued first)
  bf16x8 wf[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int tap = CIN == 32 ? (q >> 1) : (2 * q + (lane >> 5));
    const int choff = CIN == 32 ? ((q & 1) * 16 + (lane >> 5) * 8) : 0;
    wf[q] = *reinterpret_cast<const bf16x8*>(wp + ((size_t)tap * 32 + (lane & 31)) * CIN + choff);
  }
  // stage the input tile (zero outside the image)
  constexpr int CH = CIN / 8;  // 16-byte chunks per pixel
  for (int c = threadIdx.x; c < TR * TC * CH; c += 256) {
    const int pix = c / CH, ch = c % CH;
    const int ty = pix / TC, tx = pix % TC;
    const int y = y0 - 1 + ty, x = x0 - 1 + tx;
    bf16x8 v = zero8();
    if (y >= 0 && y < H && x >= 0 && x < W)
      v = *reinterpret_cast<const bf16x8*>(in + (img + (size_t)y * W + x) * CIN + ch * 8);
    *reinterpret_cast<bf16x8*>(tile + pix * S + ch * 8) = v;
  }
  __syncthreads();
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int tap = CIN == 32 ? (q >> 1) : (2 * q + (lane >> 5));
    const int choff = CIN == 32 ? ((q & 1) * 16 + (lane >> 5) * 8) : 0;
    bf16x8 a = zero8();
    if (tap < 9) {
      const int dy = tap / 3, dx = tap % 3;
      a = *reinterpret_cast<const bf16x8*>(tile + ((wave + dy) * TC + (lane & 31) + dx) * S + choff);
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, wf[q], acc, 0, 0, 0);
  }
  const int y = y0 + wave;
  if (y >= H) return;
  const int co = lane & 31;
  const float bco = (MODE == kConvGrad) ? 0.0f : bias[co];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int x = x0 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
    if (x >= W) continue;
    const size_t pix = img + (size_t)y * W + x;
    const float z = acc[r] + bco;
    if (MODE == kConvHidden) {
      if (zout) zout[pix * 32 + co] = (__bf16)z;
      aout[pix * 32 + co] = (__bf16)gelu_f(z);
    } else if (MODE == kConvOut) {
      if (co == 0) fout[pix] = oscale ? (float)(z * oscale[b]) : z;
    } else {
      aout[pix * 32 + co] = (__bf16)(z * gelu_grad_f((float)zprev[pix * 32 + co]));
    }
  }
}

// ---- weight gradient -------------------------------------------------------------------------
// dW[tap][co][ci] = sum over pixels p of dz[p][co] a[p + tap][ci]: a GEMM whose reduction runs
// over pixels.  A block walks a contiguous range of 32-pixel row segments; per segment it stages
// dz (channel-major, 32 x 32) and the three input rows as three column-shifted channel-major
// copies (so every MFMA operand is one aligned 16-byte LDS read), then wave w accumulates taps
// w, w + 4, w + 8.  Each block writes its partial sums; k_cnn_grad_reduce adds them in a fixed
// order (deterministic).  DZC: channels of the dz image (32, or 8 for the output layer);
// CINA: channels of the input image (32, or 8 for the first layer).
template <int DZC, int CINA>
__global__ __launch_bounds__(256) void k_conv_dw(const __bf16* __restrict__ dz,
                                                 const __bf16* __restrict__ a, int B, int H,
                                                 int W, int seg_per_block,
                                                 float* __restrict__ part,
                                                 float* __restrict__ dbpart) {
  constexpr int P = 40;  // LDS row pitch (elements), 16-byte aligned rows
  __shared__ __attribute__((aligned(16))) __bf16 sdz[32 * P];
  __shared__ __attribute__((aligned(16))) __bf16 sa[9 * 32 * P];  // [dy][dx][ci][px]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nsx = (W + 31) / 32;
  const int64_t nseg = (int64_t)B * H * nsx;
  const int64_t s0 = (int64_t)blockIdx.x * seg_per_block;
  const int64_t s1 = s0 + seg_per_block < nseg ? s0 + seg_per_block : nseg;
  // channels beyond the images' own stay zero for the whole block
  for (int k = threadIdx.x; k < 32 * P; k += 256) sdz[k] = (__bf16)0.0f;
  for (int k = threadIdx.x; k < 9 * 32 * P; k += 256) sa[k] = (__bf16)0.0f;
  f32x16 acc[3];
#pragma unroll
  for (int t = 0; t < 3; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[t][r] = 0.0f;
  float dbacc = 0.0f;
  for (int64_t s = s0; s < s1; ++s) {
    const int xs = (int)(s % nsx);
    const int64_t row = s / nsx;  // b * H + y
    const int y = (int)(row % H);
    const int b = (int)(row / H);
    const int x0 = xs * 32;
    __syncthreads();  // the previous segment's reads are done
    // dz: 32 pixels x DZC channels, transposed to [c][px]
    for (int c = threadIdx.x; c < 32 * (DZC / 8); c += 256) {
      const int px = c / (DZC / 8), ch = c % (DZC / 8);
      const int x = x0 + px;
      bf16x8 v = zero8();
      if (x < W) v = *reinterpret_cast<const bf16x8*>(dz + (((size_t)b * H + y) * W + x) * DZC + ch * 8);
#pragma unroll
      for (int j = 0; j < 8; ++j) sdz[(ch * 8 + j) * P + px] = v[j];
    }
    // input rows y-1..y+1, columns x0-1..x0+32, as three shifted copies: sa[dy][dx][ci][px]
    // holds a[y + dy - 1][x0 + px + dx - 1][ci]
    for (int c = threadIdx.x; c < 3 * 34 * (CINA / 8); c += 256) {
      const int ch = c % (CINA / 8);
      const int rest = c / (CINA / 8);
      const int k = rest % 34, dy = rest / 34;
      const int yy = y + dy - 1, xx = x0 - 1 + k;
      bf16x8 v = zero8();
      if (yy >= 0 && yy < H && xx >= 0 && xx < W)
        v = *reinterpret_cast<const bf16x8*>(a + (((size_t)b * H + yy) * W + xx) * CINA + ch * 8);
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const int px = k - dx;
        if (px < 0 || px > 31) continue;
#pragma unroll
        for (int j = 0; j < 8; ++j) sa[((dy * 3 + dx) * 32 + ch * 8 + j) * P + px] = v[j];
      }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const int tap = wave + 4 * t;
      if (tap > 8) continue;
#pragma unroll
      for (int kc = 0; kc < 2; ++kc) {
        const int off = kc * 16 + (lane >> 5) * 8;
        const bf16x8 fa = *reinterpret_cast<const bf16x8*>(sdz + (lane & 31) * P + off);
        const bf16x8 fb = *reinterpret_cast<const bf16x8*>(sa + (tap * 32 + (lane & 31)) * P + off);
        acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa, fb, acc[t], 0, 0, 0);
      }
    }
    if (wave == 0 && lane < 32)
      for (int px = 0; px < 32; ++px) dbacc += (float)sdz[lane * P + px];
  }
  // partial sums of this block: part[block][tap][co][ci], dbpart[block][co]
  float* pb = part + (size_t)blockIdx.x * 9 * 1024;
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    const int tap = wave + 4 * t;
    if (tap > 8) continue;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int co = (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3), ci = lane & 31;
      pb[(size_t)tap * 1024 + co * 32 + ci] = acc[t][r];
    }
  }
  if (wave == 0 && lane < 32) dbpart[(size_t)blockIdx.x * 32 + lane] = dbacc;
}

// Sums the block partials of one layer in a fixed order (deterministic), in two passes: pass 1
// (grid: 37 column blocks x kRedSplit row groups) adds the partials of a contiguous range of
// blocks, with consecutive threads on consecutive partial entries (coalesced); pass 2 adds the
// kRedSplit group sums in order and writes the gradient of W (layout [dy][dx][ci][co]) and b.
constexpr int kRedSplit = 16;
constexpr int kRedLen = 9 * 1024 + 32;  // weight entries, then the bias entries

__global__ __launch_bounds__(256) void k_cnn_grad_sum(const float* __restrict__ part,
                                                      const float* __restrict__ dbpart,
                                                      int nblocks, float* __restrict__ stage) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= kRedLen) return;
  const int g = blockIdx.y;
  const int k0 = (int)((int64_t)nblocks * g / kRedSplit);
  const int k1 = (int)((int64_t)nblocks * (g + 1) / kRedSplit);
  float s = 0.0f;
  if (e < 9 * 1024) {
    for (int k = k0; k < k1; ++k) s += part[(size_t)k * 9 * 1024 + e];
  } else {
    for (int k = k0; k < k1; ++k) s += dbpart[(size_t)k * 32 + (e - 9 * 1024)];
  }
  stage[(size_t)g * kRedLen + e] = s;
}

__global__ __launch_bounds__(256) void k_cnn_grad_scatter(const float* __restrict__ stage,
                                                          int cin, int cout,
                                                          float* __restrict__ gW,
                                                          float* __restrict__ gb) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= kRedLen) return;
  float s = 0.0f;
  for (int g = 0; g < kRedSplit; ++g) s += stage[(size_t)g * kRedLen + e];
  if (e < 9 * 1024) {
    const int tap = e / 1024, co = (e / 32) % 32, ci = e % 32;
    if (co < cout && ci < cin) gW[(tap * cin + ci) * cout + co] = s;
  } else {
    const int co = e - 9 * 1024;
    if (co < cout) gb[co] = s;
  }
}

// ---- loss ------------------------------------------------------------------------------------
// d = out - target over npix pixels; dz image (8 channels, channel 0 = 2 d / npix); per-block
// partial sums of d^2 (summed in order by k_cnn_loss_reduce).
__global__ __launch_bounds__(256) void k_cnn_mse(const float* __restrict__ out,
                                                 const float* __restrict__ target, int64_t npix,
                                                 __bf16* __restrict__ dz,
                                                 double* __restrict__ lpart) {
  __shared__ double red[256];
  double s = 0.0;
  const float g = 2.0f / (float)npix;
  for (int64_t p = blockIdx.x * 256 + threadIdx.x; p < npix; p += (int64_t)gridDim.x * 256) {
    const float d = out[p] - target[p];
    s += (double)d * d;
    bf16x8 v = zero8();
    v[0] = (__bf16)(g * d);
    *reinterpret_cast<bf16x8*>(dz + p * 8) = v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) lpart[blockIdx.x] = red[0];
}

__global__ void k_cnn_loss_reduce(const double* __restrict__ lpart, int nb, int64_t npix,
                                  double* __restrict__ loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int k = 0; k < nb; ++k) s += lpart[k];
  *loss = s / (double)npix;
}

// ---- optimizer and packing -------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_cnn_adam(float* __restrict__ theta,
                                                  const float* __restrict__ g,
                                                  float* __restrict__ m, float* __restrict__ v,
                                                  int n, float lr, float b1, float b2, float eps,
                                                  float c1, float c2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// BF16 copies of one layer's weights: forward [tap][co][ci] with CINK input and 32 output
// channels (taps padded to 10 for CINK = 8), and, for the data gradient, the mirrored taps with
// the roles of the channels swapped: [tap'][ci][co] = W[8 - tap'][ci][co] with CINB channels in.
__global__ __launch_bounds__(256) void k_cnn_pack(const float* __restrict__ W,
                                                  const float* __restrict__ b, int cin, int cout,
                                                  int cink, __bf16* __restrict__ wf,
                                                  float* __restrict__ bias, int cinb,
                                                  __bf16* __restrict__ wb) {
  const int ntf = cink == 8 ? 10 : 9;
  const int nf = ntf * 32 * cink;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e < nf) {
    const int ci = e % cink, co = (e / cink) % 32, tap = e / (cink * 32);
    const float w = (tap < 9 && ci < cin && co < cout) ? W[(tap * cin + ci) * cout + co] : 0.0f;
    wf[e] = (__bf16)w;
  }
  if (e < 32) bias[e] = e < cout ? b[e] : 0.0f;
  if (wb) {
    const int ntb = cinb == 8 ? 10 : 9;
    const int nb = ntb * 32 * cinb;
    if (e < nb) {
      const int co = e % cinb, ci = (e / cinb) % 32, tp = e / (cinb * 32);
      const float w = (tp < 9 && ci < cin && co < cout) ? W[((8 - tp) * cin + ci) * cout + co] : 0.0f;
      wb[e] = (__bf16)w;
    }
  }
}

// ---- launchers -------------------------------------------------------------------------------

void launch_cnn_features(hipStream_t s, const double* traces, int ld, int B, int n,
                         const double* lk, const double* lmu, __bf16* X, double* scale) {
  const int64_t npix = (int64_t)(n - 1) * (n - 1);
  const int gx = (int)((npix + 255) / 256 < 256 ? (npix + 255) / 256 : 256);
  hipLaunchKernelGGL(k_cnn_features, dim3(gx, B), dim3(256), 0, s, traces, ld, n, lk, lmu, X,
                     scale);
}

void launch_conv(hipStream_t s, int cin, int mode, const __bf16* in, int B, int H, int W,
                 const __bf16* wp, const float* bias, __bf16* zout, __bf16* aout, float* fout,
                 const __bf16* zprev, const double* oscale) {
  const dim3 grid((W + 31) / 32, (H + 3) / 4, B);
#define FDD_CONV(C, M)                                                                         \
  hipLaunchKernelGGL((k_conv<C, M>), grid, dim3(256), 0, s, in, H, W, wp, bias, zout, aout, \
                     fout, zprev, oscale)
  if (cin == 32) {
    if (mode == kConvHidden) FDD_CONV(32, kConvHidden);
    else if (mode == kConvOut) FDD_CONV(32, kConvOut);
    else FDD_CONV(32, kConvGrad);
  } else {
    if (mode == kConvHidden) FDD_CONV(8, kConvHidden);
    else if (mode == kConvOut) FDD_CONV(8, kConvOut);
    else FDD_CONV(8, kConvGrad);
  }
#undef FDD_CONV
}

int conv_dw_blocks(int B, int H, int W, int seg_per_block) {
  const int64_t nseg = (int64_t)B * H * ((W + 31) / 32);
  return (int)((nseg + seg_per_block - 1) / seg_per_block);
}

void launch_conv_dw(hipStream_t s, int dzc, int cina, const __bf16* dz, const __bf16* a, int B,
                    int H, int W, int seg_per_block, float* part, float* dbpart) {
  const int nb = conv_dw_blocks(B, H, W, seg_per_block);
  if (dzc == 32 && cina == 32)
    hipLaunchKernelGGL((k_conv_dw<32, 32>), dim3(nb), dim3(256), 0, s, dz, a, B, H, W,
                       seg_per_block, part, dbpart);
  else if (dzc == 32 && cina == 8)
    hipLaunchKernelGGL((k_conv_dw<32, 8>), dim3(nb), dim3(256), 0, s, dz, a, B, H, W,
                       seg_per_block, part, dbpart);
  else
    hipLaunchKernelGGL((k_conv_dw<8, 32>), dim3(nb), dim3(256), 0, s, dz, a, B, H, W,
                       seg_per_block, part, dbpart);
}

void launch_cnn_grad_reduce(hipStream_t s, const float* part, const float* dbpart, int nblocks,
                            int cin, int cout, float* gW, float* gb, float* stage) {
  const int gx = (kRedLen + 255) / 256;
  hipLaunchKernelGGL(k_cnn_grad_sum, dim3(gx, kRedSplit), dim3(256), 0, s, part, dbpart, nblocks,
                     stage);
  hipLaunchKernelGGL(k_cnn_grad_scatter, dim3(gx), dim3(256), 0, s, stage, cin, cout, gW, gb);
}

void launch_cnn_mse(hipStream_t s, const float* out, const float* target, int64_t npix, __bf16* dz,
                    double* lpart, int nb, double* loss) {
  hipLaunchKernelGGL(k_cnn_mse, dim3(nb), dim3(256), 0, s, out, target, npix, dz, lpart);
  hipLaunchKernelGGL(k_cnn_loss_reduce, dim3(1), dim3(64), 0, s, lpart, nb, npix, loss);
}

void launch_cnn_adam(hipStream_t s, float* theta, const float* g, float* m, float* v, int n,
                     float lr, float b1, float b2, float eps, int step) {
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_cnn_adam, dim3((n + 255) / 256), dim3(256), 0, s, theta, g, m, v, n, lr, b1,
                     b2, eps, c1, c2);
}

void launch_cnn_pack(hipStream_t s, const float* W, const float* b, int cin, int cout, int cink,
                     __bf16* wf, float* bias, int cinb, __bf16* wb) {
  const int n = 10 * 32 * 32;
  hipLaunchKernelGGL(k_cnn_pack, dim3((n + 255) / 256), dim3(256), 0, s, W, b, cin, cout, cink, wf,
                     bias, cinb, wb);
}

}  // namespace fdd
