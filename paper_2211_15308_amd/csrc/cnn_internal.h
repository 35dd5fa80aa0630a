// Launchers of the warm-start network kernels (kernels_cnn.hip) and the network's fixed shape.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace fdd {

constexpr int kCnnLayers = 6;
constexpr int kCnnWidths[kCnnLayers + 1] = {5, 32, 32, 32, 32, 32, 1};
constexpr int kCnnHidden = 32;
constexpr int kCnnInCh = 8;      // input image channels (5 used)
constexpr int kCnnSegPerBlock = 64;  // 32-pixel row segments per weight-gradient block

enum ConvMode { kConvHidden = 0, kConvOut = 1, kConvGrad = 2 };

void launch_cnn_features(hipStream_t s, const double* traces, int ld, int B, int n,
                         const double* lk, const double* lmu, __bf16* X, double* scale);
void launch_conv(hipStream_t s, int cin, int mode, const __bf16* in, int B, int H, int W,
                 const __bf16* wp, const float* bias, __bf16* zout, __bf16* aout, float* fout,
                 const __bf16* zprev, const double* oscale = nullptr);
int conv_dw_blocks(int B, int H, int W, int seg_per_block);
void launch_conv_dw(hipStream_t s, int dzc, int cina, const __bf16* dz, const __bf16* a, int B,
                    int H, int W, int seg_per_block, float* part, float* dbpart);
// stage: kCnnGradStage floats of scratch
constexpr int kCnnGradStage = 16 * (9 * 1024 + 32);
void launch_cnn_grad_reduce(hipStream_t s, const float* part, const float* dbpart, int nblocks,
                            int cin, int cout, float* gW, float* gb, float* stage);
void launch_cnn_mse(hipStream_t s, const float* out, const float* target, int64_t npix, __bf16* dz,
                    double* lpart, int nb, double* loss);
void launch_cnn_adam(hipStream_t s, float* theta, const float* g, float* m, float* v, int n,
                     float lr, float b1, float b2, float eps, int step);
void launch_cnn_pack(hipStream_t s, const float* W, const float* b, int cin, int cout, int cink,
                     __bf16* wf, float* bias, int cinb, __bf16* wb);

}  // namespace fdd
