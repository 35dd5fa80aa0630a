// Kernels of the flexible GMRES iteration on the coupled Darcy-Stokes system (Sec. 4; Saad's
// FGMRES with right preconditioning).
//
// * Arnoldi orthogonalization by classical Gram-Schmidt applied twice (CGS2): each pass is one
//   launch for all inner products V_i . w (a 2D grid: chunk x basis vector, per-block partials),
//   one launch summing them in fixed order, and one launch subtracting sum_i h_i V_i (every thread
//   walks the basis for its entries).  Two passes keep the basis orthogonal to working precision,
//   as modified Gram-Schmidt does, with a launch count independent of the iteration.
// * The Givens rotations, the residual estimate and the stop test run in one single-block kernel
//   on the Hessenberg column (a few hundred flops); the final triangular solve likewise.
// * Reductions: per-block partials, summed in fixed order (bitwise reproducible).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ds_internal.h"

namespace fdd {

namespace {

constexpr int kT = 256;

inline int chunks_for(int64_t n) {
  return (int)std::min<int64_t>((n + kT - 1) / kT, kDsChunks);
}
inline int full_grid(int64_t n) { return (int)((n + kT - 1) / kT); }

__device__ double block_sum(double v) {
  __shared__ double sh[kT / 64 + 1];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) s += sh[w];
    sh[kT / 64] = s;
  }
  __syncthreads();
  return sh[kT / 64];
}

__device__ double sum_partials(const double* p, int nb) {
  double v = 0.0;
  for (int k = threadIdx.x; k < nb; k += blockDim.x) v += p[k];
  return block_sum(v);
}

// partials[blockIdx.x] = sum over the block's grid-stride share of a . b
__device__ void dot_chunk(int n, const double* __restrict__ a, const double* __restrict__ b,
                          double* partials) {
  double s = 0.0;
  for (int i = blockIdx.x * kT + threadIdx.x; i < n; i += gridDim.x * kT) s += a[i] * b[i];
  s = block_sum(s);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(kT) void k_ds_dot(int n, const double* __restrict__ a,
                                               const double* __restrict__ b,
                                               double* __restrict__ partials) {
  dot_chunk(n, a, b, partials);
}

__global__ __launch_bounds__(kT) void k_ds_start(const double* partials, int nb, DsState* st,
                                                 double* g) {
  const double bb = sum_partials(partials, nb);
  if (threadIdx.x == 0) {
    const double beta = sqrt(bb);
    st->beta = beta;
    st->res = beta;
    st->hnext = 0.0;
    st->its = 0;
    st->breakdown = isfinite(bb) ? 0 : 4;
    st->done = (bb == 0.0 || !isfinite(bb)) ? 1 : 0;
    g[0] = beta;
  }
}

__global__ __launch_bounds__(kT) void k_ds_scale_by_beta(int n, const double* __restrict__ b,
                                                         double* __restrict__ v, const DsState* st) {
  const double beta = st->beta;
  const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
  for (int i = blockIdx.x * kT + threadIdx.x; i < n; i += gridDim.x * kT) v[i] = b[i] * inv;
}

// partials[i * gridDim.x + chunk] = V_i . w over the chunk, i = blockIdx.y
__global__ __launch_bounds__(kT) void k_ds_mdot(int n, const double* __restrict__ V,
                                                const double* __restrict__ w,
                                                double* __restrict__ partials, const DsState* st) {
  if (st->done) return;
  const int i = blockIdx.y;
  dot_chunk(n, V + (size_t)i * n, w, partials + (size_t)i * gridDim.x);
}

// hpass[i] = sum of the partials of V_i . w; Hcol[i] = hpass[i] (first pass) or += (second)
// (one block per i)
__global__ __launch_bounds__(kT) void k_ds_mdot_finish(const double* partials, int nb,
                                                       double* __restrict__ Hcol,
                                                       double* __restrict__ hpass, int add,
                                                       const DsState* st) {
  if (st->done) return;
  const int i = blockIdx.x;
  const double h = sum_partials(partials + (size_t)i * nb, nb);
  if (threadIdx.x == 0) {
    hpass[i] = h;
    Hcol[i] = add ? Hcol[i] + h : h;
  }
}

// w -= sum_{i <= k} hpass_i V_i: one entry per thread (a full grid: the kernel streams k + 2
// vectors), the coefficients staged in LDS, four independent partial sums
__global__ __launch_bounds__(kT) void k_ds_subtract(int n, int k, const double* __restrict__ V,
                                                    const double* __restrict__ hpass,
                                                    double* __restrict__ w, const DsState* st) {
  if (st->done) return;
  __shared__ double h[kDsMaxKrylov + 1];
  for (int i = threadIdx.x; i <= k; i += kT) h[i] = hpass[i];
  __syncthreads();
  const int j = blockIdx.x * kT + threadIdx.x;
  if (j >= n) return;
  double s0 = w[j], s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int i = 0;
  for (; i + 3 <= k; i += 4) {
    s0 -= h[i] * V[(size_t)i * n + j];
    s1 -= h[i + 1] * V[(size_t)(i + 1) * n + j];
    s2 -= h[i + 2] * V[(size_t)(i + 2) * n + j];
    s3 -= h[i + 3] * V[(size_t)(i + 3) * n + j];
  }
  for (; i <= k; ++i) s0 -= h[i] * V[(size_t)i * n + j];
  w[j] = (s0 + s1) + (s2 + s3);
}

__global__ __launch_bounds__(kT) void k_ds_norm(int n, const double* __restrict__ w,
                                                double* __restrict__ partials, const DsState* st) {
  if (st->done) return;
  dot_chunk(n, w, w, partials);
}

// h_{k+1,k} = ||w||; rotations of column k; residual estimate; stop test
__global__ __launch_bounds__(kT) void k_ds_givens(const double* partials, int nb, int k, int ldh,
                                                  double* __restrict__ Hm, double* __restrict__ cs,
                                                  double* __restrict__ sn, double* __restrict__ g,
                                                  DsState* st, double rtol) {
  if (st->done) return;
  const double ww = sum_partials(partials, nb);
  if (threadIdx.x != 0) return;
  double* h = Hm + (size_t)k * ldh;
  const double hn = sqrt(ww);
  for (int i = 0; i < k; ++i) {
    const double t = cs[i] * h[i] + sn[i] * h[i + 1];
    h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
    h[i] = t;
  }
  const double r = hypot(h[k], hn);
  const double c = r > 0.0 ? h[k] / r : 1.0, s = r > 0.0 ? hn / r : 0.0;
  cs[k] = c;
  sn[k] = s;
  h[k] = r;
  h[k + 1] = 0.0;
  g[k + 1] = -s * g[k];
  g[k] = c * g[k];
  st->hnext = hn;
  st->res = fabs(g[k + 1]);
  st->its = k + 1;
  if (!isfinite(ww) || !isfinite(r)) {
    st->breakdown |= 4;
    st->done = 1;
  } else if (st->res <= rtol * st->beta || hn == 0.0) {
    st->done = 1;   // converged, or the Krylov space is invariant (x_k exact)
  }
}

// w /= h_{k+1,k} (skipped when the norm vanished: the iteration has stopped)
__global__ __launch_bounds__(kT) void k_ds_normalize(int n, double* __restrict__ w,
                                                     const DsState* st) {
  const double hn = st->hnext;
  if (!(hn > 0.0)) return;
  const double inv = 1.0 / hn;
  for (int j = blockIdx.x * kT + threadIdx.x; j < n; j += gridDim.x * kT) w[j] *= inv;
}

// y = R^{-1} g[0..k) by back substitution (R: the rotated upper triangle)
__global__ __launch_bounds__(64) void k_ds_backsolve(int k, int ldh, const double* __restrict__ Hm,
                                                     const double* __restrict__ g,
                                                     double* __restrict__ y) {
  if (threadIdx.x != 0) return;
  for (int i = k - 1; i >= 0; --i) {
    double s = g[i];
    for (int j = i + 1; j < k; ++j) s -= Hm[(size_t)j * ldh + i] * y[j];
    y[i] = s / Hm[(size_t)i * ldh + i];
  }
}

// x = sum_{i < k} y_i Z_i (one entry per thread, y staged in LDS)
__global__ __launch_bounds__(kT) void k_ds_combine(int n, int k, const double* __restrict__ y,
                                                   const double* __restrict__ Z,
                                                   double* __restrict__ x) {
  __shared__ double ys[kDsMaxKrylov];
  for (int i = threadIdx.x; i < k; i += kT) ys[i] = y[i];
  __syncthreads();
  const int j = blockIdx.x * kT + threadIdx.x;
  if (j >= n) return;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int i = 0;
  for (; i + 4 <= k; i += 4) {
    s0 += ys[i] * Z[(size_t)i * n + j];
    s1 += ys[i + 1] * Z[(size_t)(i + 1) * n + j];
    s2 += ys[i + 2] * Z[(size_t)(i + 2) * n + j];
    s3 += ys[i + 3] * Z[(size_t)(i + 3) * n + j];
  }
  for (; i < k; ++i) s0 += ys[i] * Z[(size_t)i * n + j];
  x[j] = (s0 + s1) + (s2 + s3);
}

__global__ __launch_bounds__(kT) void k_ds_scale(int n, double a, const double* __restrict__ x,
                                                 double* __restrict__ y) {
  for (int j = blockIdx.x * kT + threadIdx.x; j < n; j += gridDim.x * kT) y[j] = a * x[j];
}

__device__ __forceinline__ double ell_row(const HdView& A, int i, const double* __restrict__ x) {
  const int t = A.rtype[i];
  const double* v = A.tval + (size_t)t * A.width;
  double s = 0.0;
  for (int k = 0; k < A.width; ++k) {
    const int c = A.toff ? i + A.toff[t * A.width + k] : A.col[(size_t)k * A.rows + i];
    s += v[k] * x[c];
  }
  return s;
}

// partials of ||b - A x||^2 (first half) and ||b||^2 (second half of the grid's partials)
__global__ __launch_bounds__(kT) void k_ds_true_res(HdView Au, HdView Bp, HdView Dd,
                                                    const double* __restrict__ b,
                                                    const double* __restrict__ x,
                                                    double* __restrict__ partials) {
  const int n = Au.rows + Bp.rows + Dd.rows;
  double rr = 0.0, bb = 0.0;
  for (int i = blockIdx.x * kT + threadIdx.x; i < n; i += gridDim.x * kT) {
    double ax;
    if (i < Au.rows) ax = ell_row(Au, i, x);
    else if (i < Au.rows + Bp.rows) ax = ell_row(Bp, i - Au.rows, x);
    else ax = ell_row(Dd, i - Au.rows - Bp.rows, x);
    const double r = b[i] - ax;
    rr += r * r;
    bb += b[i] * b[i];
  }
  rr = block_sum(rr);
  bb = block_sum(bb);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = rr;
    partials[gridDim.x + blockIdx.x] = bb;
  }
}

__global__ __launch_bounds__(kT) void k_ds_true_res_finish(const double* partials, int nb,
                                                           DsState* st) {
  const double rr = sum_partials(partials, nb);
  const double bb = sum_partials(partials + nb, nb);
  if (threadIdx.x == 0) {
    st->t_res[0] = rr;
    st->t_res[1] = bb;
  }
}

}  // namespace

void launch_ds_start(hipStream_t s, int n, const double* b, double* V0, double* g, double* partials,
                     DsState* st) {
  const int nb = chunks_for(n);
  hipLaunchKernelGGL(k_ds_dot, dim3(nb), dim3(kT), 0, s, n, b, b, partials);
  hipLaunchKernelGGL(k_ds_start, dim3(1), dim3(kT), 0, s, partials, nb, st, g);
  hipLaunchKernelGGL(k_ds_scale_by_beta, dim3(nb), dim3(kT), 0, s, n, b, V0, st);
}

void launch_ds_orthogonalize(hipStream_t s, int n, int k, const double* V, double* w, double* Hcol,
                             double* hpass, double* partials, const DsState* st) {
  const int nb = chunks_for(n);
  for (int pass = 0; pass < 2; ++pass) {
    hipLaunchKernelGGL(k_ds_mdot, dim3(nb, k + 1), dim3(kT), 0, s, n, V, w, partials, st);
    hipLaunchKernelGGL(k_ds_mdot_finish, dim3(k + 1), dim3(kT), 0, s, partials, nb, Hcol, hpass,
                       pass, st);
    hipLaunchKernelGGL(k_ds_subtract, dim3(full_grid(n)), dim3(kT), 0, s, n, k, V, hpass, w, st);
  }
}

void launch_ds_normalize_givens(hipStream_t s, int n, int k, int ldh, double* w, double* Hm,
                                double* cs, double* sn, double* g, double* partials, DsState* st,
                                double rtol) {
  const int nb = chunks_for(n);
  hipLaunchKernelGGL(k_ds_norm, dim3(nb), dim3(kT), 0, s, n, w, partials, st);
  hipLaunchKernelGGL(k_ds_givens, dim3(1), dim3(kT), 0, s, partials, nb, k, ldh, Hm, cs, sn, g, st,
                     rtol);
  hipLaunchKernelGGL(k_ds_normalize, dim3(full_grid(n)), dim3(kT), 0, s, n, w, st);
}

void launch_ds_solution(hipStream_t s, int n, int k, int ldh, const double* Hm, const double* g,
                        double* y, const double* Z, double* x) {
  const int nb = chunks_for(n);
  if (k > 0) hipLaunchKernelGGL(k_ds_backsolve, dim3(1), dim3(64), 0, s, k, ldh, Hm, g, y);
  hipLaunchKernelGGL(k_ds_combine, dim3(full_grid(n)), dim3(kT), 0, s, n, k, y, Z, x);
}

void launch_ds_scale(hipStream_t s, int n, double a, const double* x, double* y) {
  hipLaunchKernelGGL(k_ds_scale, dim3(chunks_for(n)), dim3(kT), 0, s, n, a, x, y);
}

void launch_ds_true_residual(hipStream_t s, HdView Au, HdView Bp, HdView Dd, const double* b,
                             const double* x, double* partials, DsState* st) {
  const int nb = chunks_for((int64_t)Au.rows + Bp.rows + Dd.rows);
  hipLaunchKernelGGL(k_ds_true_res, dim3(nb), dim3(kT), 0, s, Au, Bp, Dd, b, x, partials);
  hipLaunchKernelGGL(k_ds_true_res_finish, dim3(1), dim3(kT), 0, s, partials, nb, st);
}

}  // namespace fdd
