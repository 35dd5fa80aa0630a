// C ABI of the warm-start network (declared in include/fdd.h): set-up, parameters, forward,
// loss, backward and Adam, each a short sequence of the kernels in kernels_cnn.hip.  The
// solver uses a network handle given in fdd_opts.warmstart through cnn_warm_guess().
#include <algorithm>
#include <cstring>
#include <new>

#include "api_internal.h"
#include "cnn_internal.h"

using namespace fdd;

struct fdd_cnn_s {
  int batch_max = 0, n_max = 0, train = 0, device = 0;
  int64_t nparam = 0;
  int64_t offW[kCnnLayers] = {}, offb[kCnnLayers] = {};
  int dw_blocks_max = 0;
  // workspace views
  char* ws = nullptr;
  size_t ws_bytes = 0;
  __bf16* X0 = nullptr;
  __bf16* Z[kCnnLayers] = {};   // pre-activations of layers 1..5 (training)
  __bf16* A[kCnnLayers] = {};   // activations of layers 1..5 (training), or 2 ping-pong buffers
  __bf16* dz6 = nullptr;        // output gradient image (8 channels)
  __bf16* dZ[2] = {};           // data-gradient ping-pong
  float* part = nullptr;        // weight-gradient block partials
  float* dbpart = nullptr;
  float* stage = nullptr;       // two-pass gradient reduction
  double* lpart = nullptr;
  double* loss = nullptr;
  double* scale = nullptr;
  float* wout = nullptr;        // network output image for the solver's warm start
  __bf16* wf[kCnnLayers] = {};
  __bf16* wb[kCnnLayers] = {};
  float* bias[kCnnLayers] = {};
  bool params_set = false;
};

namespace {

constexpr int kLossBlocks = 512;

size_t plan_cnn(fdd_cnn_s* C, char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    off = align_up(off, 256);
    char* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  };
  const size_t P = (size_t)(C->n_max - 1) * (C->n_max - 1);
  const size_t BP = P * C->batch_max;
  C->X0 = (__bf16*)take(2 * BP * kCnnInCh);
  if (C->train) {
    for (int l = 0; l < kCnnLayers - 1; ++l) {
      C->Z[l] = (__bf16*)take(2 * BP * kCnnHidden);
      C->A[l] = (__bf16*)take(2 * BP * kCnnHidden);
    }
    C->dz6 = (__bf16*)take(2 * BP * kCnnInCh);
    C->dZ[0] = (__bf16*)take(2 * BP * kCnnHidden);
    C->dZ[1] = (__bf16*)take(2 * BP * kCnnHidden);
    C->part = (float*)take(sizeof(float) * (size_t)C->dw_blocks_max * 9 * 1024);
    C->dbpart = (float*)take(sizeof(float) * (size_t)C->dw_blocks_max * 32);
    C->stage = (float*)take(sizeof(float) * kCnnGradStage);
    C->lpart = (double*)take(sizeof(double) * kLossBlocks);
    C->loss = (double*)take(sizeof(double));
  } else {
    C->A[0] = (__bf16*)take(2 * BP * kCnnHidden);
    C->A[1] = (__bf16*)take(2 * BP * kCnnHidden);
  }
  C->scale = (double*)take(sizeof(double) * C->batch_max);
  C->wout = (float*)take(sizeof(float) * BP);
  for (int l = 0; l < kCnnLayers; ++l) {
    C->wf[l] = (__bf16*)take(2 * 10 * 32 * 32);
    C->wb[l] = (__bf16*)take(2 * 10 * 32 * 32);
    C->bias[l] = (float*)take(sizeof(float) * 32);
  }
  return align_up(off, 256);
}

int check_shape(const fdd_cnn_s* C, int B, int n) {
  if (B < 1 || B > C->batch_max) return fail(FDD_E_ARG, "batch %d outside [1, %d]", B, C->batch_max);
  if (n < 4 || n > C->n_max) return fail(FDD_E_ARG, "n = %d outside [4, %d]", n, C->n_max);
  if (!C->ws) return fail(FDD_E_WORKSPACE, "no network workspace bound");
  if (!C->params_set) return fail(FDD_E_STATE, "network parameters not set");
  return FDD_OK;
}

// Forward pass into out (FP32, B x (n-1)^2); oscale multiplies image b by oscale[b].
void enqueue_forward(fdd_cnn_s* C, hipStream_t s, const double* traces, int ld, int B, int n,
                     const double* lk, const double* lmu, float* out, const double* oscale) {
  const int H = n - 1, W = n - 1;
  launch_cnn_features(s, traces, ld, B, n, lk, lmu, C->X0, C->scale);
  const __bf16* in = C->X0;
  for (int l = 0; l < kCnnLayers; ++l) {
    const int cin = l == 0 ? kCnnInCh : kCnnHidden;
    if (l < kCnnLayers - 1) {
      __bf16* z = C->train ? C->Z[l] : nullptr;
      __bf16* a = C->train ? C->A[l] : C->A[l & 1];
      launch_conv(s, cin, kConvHidden, in, B, H, W, C->wf[l], C->bias[l], z, a, nullptr, nullptr);
      in = a;
    } else {
      launch_conv(s, cin, kConvOut, in, B, H, W, C->wf[l], C->bias[l], nullptr, nullptr, out,
                  nullptr, oscale);
    }
  }
}

}  // namespace

namespace fdd {

// The solver's warm start: the guess for the trace (length n - 1, device) lands in C->wout with
// its scale in C->scale[0] (the interior solve multiplies them).  lk_lmu: device {log10 K,
// log10 mu}.
int cnn_warm_guess(fdd_cnn_s* C, hipStream_t s, const double* trace, int n, const double* lk_lmu,
                   const float** guess, const double** scale) {
  int rc = check_shape(C, 1, n);
  if (rc) return rc;
  enqueue_forward(C, s, trace, n - 1, 1, n, lk_lmu, lk_lmu + 1, C->wout, nullptr);
  *guess = C->wout;
  *scale = C->scale;
  return FDD_OK;
}

// Guesses for B traces of one size n (rows of `traces`, stride ld, device) into `out` (image b at
// out + b (n-1)^2); out must lie in the network's output buffer (cnn_output).
int cnn_warm_guess_batch(fdd_cnn_s* C, hipStream_t s, const double* traces, int ld, int B, int n,
                         const double* lk, const double* lmu, float* out) {
  int rc = check_shape(C, B, n);
  if (rc) return rc;
  enqueue_forward(C, s, traces, ld, B, n, lk, lmu, out, nullptr);
  return FDD_OK;
}

float* cnn_output(fdd_cnn_s* C, int64_t* capacity) {
  if (capacity) *capacity = (int64_t)(C->n_max - 1) * (C->n_max - 1) * C->batch_max;
  return C->wout;
}

int cnn_batch_max(const fdd_cnn_s* C) { return C->batch_max; }

uint64_t cnn_binding_id(const fdd_cnn_s* C) { return (uint64_t)(uintptr_t)C->ws; }

int cnn_check_for(const fdd_cnn_s* C, int n) {
  if (!C) return fail(FDD_E_ARG, "null network");
  if (n > C->n_max) return fail(FDD_E_ARG, "network sized for n <= %d, problem has n = %d", C->n_max, n);
  if (!C->ws) return fail(FDD_E_WORKSPACE, "no network workspace bound");
  if (!C->params_set) return fail(FDD_E_STATE, "network parameters not set");
  return FDD_OK;
}

}  // namespace fdd

extern "C" {

int fdd_cnn_create(int batch_max, int n_max, int train, int hip_device, fdd_cnn* out) {
  if (!out) return fail(FDD_E_ARG, "null argument");
  *out = nullptr;
  if (batch_max < 1 || batch_max > 4096) return fail(FDD_E_ARG, "batch_max must be in [1, 4096]");
  if (n_max < 4 || n_max > 4096) return fail(FDD_E_ARG, "n_max must be in [4, 4096]");
  if ((int64_t)batch_max * (n_max - 1) * (n_max - 1) * kCnnHidden * 2 > (int64_t(1) << 31))
    return fail(FDD_E_ARG, "one activation tensor would exceed 2 GiB");
  fdd_cnn_s* C = new (std::nothrow) fdd_cnn_s();
  if (!C) return fail(FDD_E_NOMEM, "out of host memory");
  C->batch_max = batch_max;
  C->n_max = n_max;
  C->train = train ? 1 : 0;
  C->device = hip_device;
  int64_t o = 0;
  for (int l = 0; l < kCnnLayers; ++l) {
    C->offW[l] = o;
    o += 9 * kCnnWidths[l] * kCnnWidths[l + 1];
    C->offb[l] = o;
    o += kCnnWidths[l + 1];
  }
  C->nparam = o;
  C->dw_blocks_max = conv_dw_blocks(batch_max, n_max - 1, n_max - 1, kCnnSegPerBlock);
  *out = C;
  return FDD_OK;
}

int fdd_cnn_param_count(fdd_cnn C, int64_t* count) {
  if (!C || !count) return fail(FDD_E_ARG, "null argument");
  *count = C->nparam;
  return FDD_OK;
}

int fdd_cnn_workspace_bytes(fdd_cnn C, size_t* bytes) {
  if (!C || !bytes) return fail(FDD_E_ARG, "null argument");
  fdd_cnn_s tmp = *C;
  *bytes = plan_cnn(&tmp, nullptr);
  return FDD_OK;
}

int fdd_cnn_bind_workspace(fdd_cnn C, void* dev, size_t bytes, void* stream) {
  if (!C || !dev) return fail(FDD_E_ARG, "null argument");
  if (((uintptr_t)dev) & 255) return fail(FDD_E_WORKSPACE, "workspace must be 256-byte aligned");
  fdd_cnn_s tmp = *C;
  const size_t need = plan_cnn(&tmp, nullptr);
  if (bytes < need) return fail(FDD_E_WORKSPACE, "workspace %zu bytes < %zu needed", bytes, need);
  HIPCHK(hipSetDevice(C->device));
  C->ws = (char*)dev;
  C->ws_bytes = bytes;
  plan_cnn(C, C->ws);
  C->params_set = false;
  (void)stream;
  return FDD_OK;
}

int fdd_cnn_set_params(fdd_cnn C, const float* theta, void* stream) {
  if (!C || !theta) return fail(FDD_E_ARG, "null argument");
  if (!C->ws) return fail(FDD_E_WORKSPACE, "no network workspace bound");
  HIPCHK(hipSetDevice(C->device));
  hipStream_t s = (hipStream_t)stream;
  for (int l = 0; l < kCnnLayers; ++l) {
    const int cin = kCnnWidths[l], cout = kCnnWidths[l + 1];
    const int cink = l == 0 ? kCnnInCh : kCnnHidden;
    const int cinb = cout == 1 ? kCnnInCh : kCnnHidden;
    launch_cnn_pack(s, theta + C->offW[l], theta + C->offb[l], cin, cout, cink, C->wf[l],
                    C->bias[l], cinb, l > 0 ? C->wb[l] : nullptr);
  }
  HIPCHK(hipGetLastError());
  C->params_set = true;
  return FDD_OK;
}

int fdd_cnn_forward(fdd_cnn C, const double* traces, int ld, int batch, int n,
                    const double* log10K, const double* log10mu, float* out, int rescale,
                    void* stream) {
  if (!C || !traces || !log10K || !log10mu || !out) return fail(FDD_E_ARG, "null argument");
  int rc = check_shape(C, batch, n);
  if (rc) return rc;
  if (ld < n - 1) return fail(FDD_E_ARG, "trace stride %d < n - 1", ld);
  HIPCHK(hipSetDevice(C->device));
  enqueue_forward(C, (hipStream_t)stream, traces, ld, batch, n, log10K, log10mu, out,
                  rescale ? C->scale : nullptr);
  HIPCHK(hipGetLastError());
  return FDD_OK;
}

int fdd_cnn_loss(fdd_cnn C, const float* out, const float* target, int batch, int n,
                 double* loss, void* stream) {
  if (!C || !out || !target) return fail(FDD_E_ARG, "null argument");
  int rc = check_shape(C, batch, n);
  if (rc) return rc;
  if (!C->train) return fail(FDD_E_STATE, "network created without training buffers");
  HIPCHK(hipSetDevice(C->device));
  const int64_t npix = (int64_t)batch * (n - 1) * (n - 1);
  launch_cnn_mse((hipStream_t)stream, out, target, npix, C->dz6, C->lpart, kLossBlocks,
                 loss ? loss : C->loss);
  HIPCHK(hipGetLastError());
  return FDD_OK;
}

int fdd_cnn_backward(fdd_cnn C, int batch, int n, float* grad, void* stream) {
  if (!C || !grad) return fail(FDD_E_ARG, "null argument");
  int rc = check_shape(C, batch, n);
  if (rc) return rc;
  if (!C->train) return fail(FDD_E_STATE, "network created without training buffers");
  HIPCHK(hipSetDevice(C->device));
  hipStream_t s = (hipStream_t)stream;
  const int H = n - 1, W = n - 1;
  const int nb = conv_dw_blocks(batch, H, W, kCnnSegPerBlock);
  const __bf16* dz = C->dz6;
  int dzc = kCnnInCh;
  int cur = 0;
  for (int l = kCnnLayers - 1; l >= 0; --l) {
    const int cin = kCnnWidths[l], cout = kCnnWidths[l + 1];
    const __bf16* a = l == 0 ? C->X0 : C->A[l - 1];
    launch_conv_dw(s, dzc, l == 0 ? kCnnInCh : kCnnHidden, dz, a, batch, H, W, kCnnSegPerBlock,
                   C->part, C->dbpart);
    launch_cnn_grad_reduce(s, C->part, C->dbpart, nb, cin, cout, grad + C->offW[l],
                           grad + C->offb[l], C->stage);
    if (l > 0) {
      launch_conv(s, dzc, kConvGrad, dz, batch, H, W, C->wb[l], nullptr, nullptr, C->dZ[cur],
                  nullptr, C->Z[l - 1]);
      dz = C->dZ[cur];
      dzc = kCnnHidden;
      cur ^= 1;
    }
  }
  HIPCHK(hipGetLastError());
  return FDD_OK;
}

int fdd_cnn_adam_step(fdd_cnn C, float* theta, const float* grad, float* m, float* v, float lr,
                      float b1, float b2, float eps, int step, void* stream) {
  if (!C || !theta || !grad || !m || !v) return fail(FDD_E_ARG, "null argument");
  if (step < 1 || !(lr > 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps > 0))
    return fail(FDD_E_ARG, "invalid Adam hyper-parameters");
  HIPCHK(hipSetDevice(C->device));
  launch_cnn_adam((hipStream_t)stream, theta, grad, m, v, (int)C->nparam, lr, b1, b2, eps, step);
  HIPCHK(hipGetLastError());
  return FDD_OK;
}

void fdd_cnn_destroy(fdd_cnn C) { delete C; }

}  // extern "C"
