// Interface (Gamma) kernels of the 2D solver, FP64, for gfx950.
//
// On the 1D P1 interface with n-1 free nodes, L_h = A_G = (1/h) tridiag(-1, 2, -1) and
// M_h = M_G = (h/6) tridiag(1, 4, 1) (Dirichlet at the ends of Gamma).  The rational
// approximation of the paper's eq. (RA) needs the shifted solves (A_G + p_k M_G)^{-1} r for all
// poles plus M_G^{-1} r; each is a symmetric diagonally dominant tridiagonal system.  One
// workgroup per system solves it by parallel cyclic reduction in LDS (rows normalized so the
// diagonal is 1; ceil(log2(n-1)) elimination steps, each a neighbour exchange at distance 2^s).
// A single-workgroup kernel then forms the weighted sum over systems in a fixed order, fused with
// the epilogue (outer-PCG update, or the mass products of the operator H).
#include "iface_device.h"

#include <mutex>

namespace fdd {

__global__ __launch_bounds__(kIfaceThreads) void k_iface_solve(int n, double h, ShiftTable tab,
                                                               int mode,
                                                               const double* __restrict__ in,
                                                               double* __restrict__ scratch) {
  const int k = blockIdx.x;
  d_iface_solve(n, h, tab.alpha[k], tab.beta[k], tab.coef[k], mode, in, scratch + (size_t)k * n);
}

__global__ __launch_bounds__(kIfaceThreads) void k_iface_combine(
    int n, double h, int m, double d0, int mode, const double* __restrict__ in,
    double* __restrict__ out, const double* __restrict__ scratch, DevState* st,
    const double* __restrict__ p_prev, double* __restrict__ p_next, int ver, int first) {
  d_iface_combine(n, h, m, d0, mode, in, out, scratch, st, p_prev, p_next, ver, first, -1.0);
}

__global__ __launch_bounds__(kIfaceThreads) void k_schur_gather(
    int n, int nf, int pitch, double K, double gamma, const double* __restrict__ p,
    const double* __restrict__ u0, const double* __restrict__ u1, const int* __restrict__ sel,
    const double* __restrict__ Hp, double* __restrict__ y, const double* __restrict__ x,
    double* __restrict__ xn, const double* __restrict__ r, double* __restrict__ rn, DevState* st,
    int mode, int ver) {
  const double* u = (sel && (*sel & 1)) ? u1 : u0;
  d_schur_gather(n, nf, pitch, K, gamma, p, u, Hp, y, x, xn, r, rn, st, mode, ver);
}

// g = b_G - A_GI w = b_G + w|row nf  (right-hand side of the interface problem); x_G = 0.
__global__ void k_rhs_reduce(int n, int pitch, const double* __restrict__ bG,
                             const double* __restrict__ u0, const double* __restrict__ u1,
                             const int* __restrict__ sel, double* __restrict__ g,
                             double* __restrict__ x) {
  const double* u = (sel && (*sel & 1)) ? u1 : u0;
  const size_t row = (size_t)(n - 1) * pitch;
  for (int i = threadIdx.x + blockIdx.x * blockDim.x; i < n; i += blockDim.x * gridDim.x) {
    g[i] = bG[i] + u[row + i];
    x[i] = 0.0;
  }
}

// Copy the interior solution (padded, pitch) into the caller's vector (pitch n-1), and the
// interface part.
__global__ void k_scatter(int nf, int pitch, const double* __restrict__ u0,
                          const double* __restrict__ u1, const int* __restrict__ sel,
                          const double* __restrict__ xG, double* __restrict__ x) {
  const double* u = (sel && (*sel & 1)) ? u1 : u0;
  const int64_t NI = (int64_t)nf * nf;
  for (int64_t k = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; k < NI + nf;
       k += (int64_t)blockDim.x * gridDim.x) {
    if (k < NI) {
      const int i = (int)(k % nf), j = (int)(k / nf);
      x[k] = u[(size_t)j * pitch + i];
    } else if (xG) {
      x[k] = xG[k - NI];
    }
  }
}

// Copy a compact (pitch nf) FP64 interior vector out of a padded one, or into one.
__global__ void k_copy_rows(const double* __restrict__ src, int sp, double* __restrict__ dst,
                            int dp, int width, int rows) {
  const int64_t tot = (int64_t)width * rows;
  for (int64_t k = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; k < tot;
       k += (int64_t)blockDim.x * gridDim.x) {
    const int i = (int)(k % width), j = (int)(k / width);
    dst[(size_t)j * dp + i] = src[(size_t)j * sp + i];
  }
}

// out = a + c u over the nf x nf interior grid (padded rows; the padding is not touched).
__global__ __launch_bounds__(256) void k_interior_axpy(int nf, int pitch, const double* __restrict__ a,
                                                       const double* __restrict__ u,
                                                       const double* __restrict__ coef,
                                                       double scale, double* __restrict__ out) {
  const double c = coef ? *coef : scale;
  const int tot = nf * pitch;  // below 2^23 (nf <= 2047)
  for (int k = threadIdx.x + blockIdx.x * blockDim.x; k < tot; k += blockDim.x * gridDim.x) {
    if (k % pitch >= nf) continue;
    out[k] = (a ? a[k] : 0.0) + c * u[k];
  }
}

// y = A x on all free dofs: K times the P1 stiffness (5-point inside, the natural-boundary row
// (2, -1/2, -1/2, -1 below) on Gamma) plus gamma Hx on the Gamma row.  Optionally the block
// partials of ||b - y||^2 and ||b||^2 (summed by k_full_operator_sum).
__global__ __launch_bounds__(256) void k_full_operator(int n, double K, double gamma,
                                                       const double* __restrict__ x,
                                                       const double* __restrict__ Hx,
                                                       double* __restrict__ y,
                                                       const double* __restrict__ b,
                                                       double* __restrict__ partials) {
  const int m = n - 1;
  const int64_t N = (int64_t)n * m;
  double e2 = 0.0, b2 = 0.0;
  for (int64_t k = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; k < N;
       k += (int64_t)blockDim.x * gridDim.x) {
    const int i = (int)(k % m), j = (int)(k / m);  // 0-based: node (i+1, j+1)
    const double c = x[k];
    const double w = i > 0 ? x[k - 1] : 0.0, e = i < m - 1 ? x[k + 1] : 0.0;
    const double s = j > 0 ? x[k - m] : 0.0;
    double v;
    if (j < n - 1) {
      const double no = x[k + m];
      v = K * (4.0 * c - w - e - s - no);
    } else {
      v = K * (2.0 * c - 0.5 * (w + e) - s) + gamma * Hx[i];
    }
    if (y) y[k] = v;
    if (b) {
      const double d = b[k] - v;
      e2 += d * d;
      b2 += b[k] * b[k];
    }
  }
  if (!b) return;
  __shared__ double s2[2][4];
  for (int o = 32; o > 0; o >>= 1) {
    e2 += __shfl_down(e2, o, 64);
    b2 += __shfl_down(b2, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    s2[0][threadIdx.x >> 6] = e2;
    s2[1][threadIdx.x >> 6] = b2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, bb = 0.0;
    for (int w = 0; w < 4; ++w) {
      a += s2[0][w];
      bb += s2[1][w];
    }
    partials[2 * blockIdx.x] = a;
    partials[2 * blockIdx.x + 1] = bb;
  }
}

// res = the sums of k_full_operator's partials (one block, fixed order).
__global__ __launch_bounds__(256) void k_full_operator_sum(const double* __restrict__ partials,
                                                           int nb, double* res) {
  const double ta = block_sum_partials(partials, nb, 2);
  const double tb = block_sum_partials(partials + 1, nb, 2);
  if (threadIdx.x == 0) {
    res[0] = ta;
    res[1] = tb;
  }
}

// ---- device-resident scratch for callers that cannot allocate --------------------------------
// Room for kStaticPrecondSystems shifted systems of up to kStaticPrecondN unknowns (1.02 MiB).
// Each device holds its own copy at its own address; host code uses the address returned by
// hipGetSymbolAddress on that device, never the array's name.
static_assert(kStaticPrecondN <= kIfaceMaxN, "static scratch rows exceed the interface kernels");
static __device__ __align__(256) double precond_scratch[(size_t)kStaticPrecondSystems * kStaticPrecondN];

int static_precond_scratch(int device, double** out) {
  static std::mutex mu;
  static double* addr[kMaxStaticDevices] = {};
  if (device < 0 || device >= kMaxStaticDevices) return -1;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(precond_scratch)) != hipSuccess || !p) return -2;
    addr[device] = (double*)p;
  }
  *out = addr[device];
  return 0;
}

// ---- launchers ----------------------------------------------------------------------------

// Hands the device state to the host without a stream synchronization: copies it into pinned
// host memory, makes the stores visible system-wide, then writes the sequence word the host is
// waiting for (release order: the state before the word).
__global__ __launch_bounds__(64) void k_publish_state(const DevState* __restrict__ st,
                                                      DevState* __restrict__ host,
                                                      unsigned* __restrict__ seq_word,
                                                      unsigned seq) {
  constexpr int kWords = (int)(sizeof(DevState) / sizeof(unsigned));
  const unsigned* src = reinterpret_cast<const unsigned*>(st);
  unsigned* dst = reinterpret_cast<unsigned*>(host);
  for (int w = threadIdx.x; w < kWords; w += 64) dst[w] = src[w];
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) __atomic_store_n(seq_word, seq, __ATOMIC_RELEASE);
}

void launch_publish_state(hipStream_t s, const DevState* st, DevState* host, unsigned* seq_word,
                          unsigned seq) {
  hipLaunchKernelGGL(k_publish_state, dim3(1), dim3(64), 0, s, st, host, seq_word, seq);
}

void launch_iface_batch(hipStream_t s, int ng, double h, const ShiftTable& tab, int mode,
                        const double* in, double* out, double* scratch, DevState* st,
                        const double* p_prev, double* p_next, int ver, int first) {
  hipLaunchKernelGGL(k_iface_solve, dim3(tab.m), dim3(kIfaceThreads), 0, s, ng, h, tab, mode, in,
                     scratch);
  hipLaunchKernelGGL(k_iface_combine, dim3(1), dim3(kIfaceThreads), 0, s, ng, h, tab.m, tab.d0,
                     mode, in, out, scratch, st, p_prev, p_next, ver, first);
}

void launch_schur_gather(hipStream_t s, int ng, int nf, int pitch, double K, double gamma,
                         const double* p, const double* u0, const double* u1, const int* sel,
                         const double* Hp, double* y, const double* x, double* xn,
                         const double* r, double* rn, DevState* st, int mode, int ver) {
  hipLaunchKernelGGL(k_schur_gather, dim3(1), dim3(kIfaceThreads), 0, s, ng, nf, pitch, K, gamma,
                     p, u0, u1, sel, Hp, y, x, xn, r, rn, st, mode, ver);
}

void launch_rhs_reduce(hipStream_t s, int n, int pitch, const double* bG, const double* u0,
                       const double* u1, const int* sel, double* g, double* x) {
  hipLaunchKernelGGL(k_rhs_reduce, dim3(1), dim3(1024), 0, s, n, pitch, bG, u0, u1, sel, g, x);
}

void launch_scatter(hipStream_t s, int nf, int pitch, const double* u0, const double* u1,
                    const int* sel, const double* xG, double* x) {
  const int64_t tot = (int64_t)nf * nf + nf;
  int blocks = (int)std::min<int64_t>((tot + 255) / 256, 4096);
  hipLaunchKernelGGL(k_scatter, dim3(blocks), dim3(256), 0, s, nf, pitch, u0, u1, sel, xG, x);
}

void launch_copy_rows(hipStream_t s, const double* src, int sp, double* dst, int dp, int width,
                      int rows) {
  const int64_t tot = (int64_t)width * rows;
  int blocks = (int)std::min<int64_t>((tot + 255) / 256, 4096);
  hipLaunchKernelGGL(k_copy_rows, dim3(blocks), dim3(256), 0, s, src, sp, dst, dp, width, rows);
}

void launch_interior_axpy(hipStream_t s, int nf, int pitch, const double* a, const double* u,
                          const double* coef, double scale, double* out) {
  const int64_t tot = (int64_t)nf * pitch;
  int blocks = (int)std::min<int64_t>((tot + 255) / 256, 8192);
  hipLaunchKernelGGL(k_interior_axpy, dim3(blocks), dim3(256), 0, s, nf, pitch, a, u, coef, scale,
                     out);
}

void launch_full_operator(hipStream_t s, int n, double K, double gamma, const double* x,
                          const double* Hx, double* y, const double* b, double* partials,
                          double* res) {
  const int64_t N = (int64_t)n * (n - 1);
  int blocks = (int)std::min<int64_t>((N + 255) / 256, 2048);
  hipLaunchKernelGGL(k_full_operator, dim3(blocks), dim3(256), 0, s, n, K, gamma, x, Hx, y, b,
                     partials);
  if (b) hipLaunchKernelGGL(k_full_operator_sum, dim3(1), dim3(256), 0, s, partials, blocks, res);
}

}  // namespace fdd
