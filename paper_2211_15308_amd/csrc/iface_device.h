// Device-side building blocks of the interface (Gamma) kernels, shared by the single-instance
// kernels (kernels_iface.hip) and the batched kernels (kernels_batch.hip).
#pragma once
#include "fdd_internal.h"

namespace fdd {

constexpr int kIfaceThreads = 1024;
constexpr int kIfaceMaxN = 2048;

__device__ __forceinline__ double bsum(double v) {
  __shared__ double sh[kIfaceThreads / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  __shared__ double tot;
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
    tot = s;
  }
  __syncthreads();
  return tot;  // broadcast to every thread
}

// Sum of count partials p[q * stride] (q = 0 .. count - 1) by every thread of the calling block
// (blockDim.x a multiple of 64, at most 1024), read at agent scope (written by other blocks of the
// same kernel), in a fixed order: thread t adds q = t, t + blockDim.x, ..., then a fixed tree over
// the block.  Every thread receives the total.
__device__ __forceinline__ double block_sum_partials(const double* p, int count, int stride) {
  __shared__ double sw[16];
  // a thread's partials q = tid, tid + B, ... are added in that order, eight loads in flight at
  // a time (a loop adding each value as it arrives waits once per partial)
  constexpr int U = 8;
  double v = 0.0;
  for (int q0 = threadIdx.x; q0 < count; q0 += U * (int)blockDim.x) {
    double a[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = q0 + u * (int)blockDim.x;
      a[u] = q < count ? __hip_atomic_load(&p[(size_t)q * stride], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT)
                       : 0.0;
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (q0 + u * (int)blockDim.x < count) v += a[u];
  }
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sw[w];
  return t;
}

__device__ __forceinline__ double mass_apply(const double* v, int n, double h, int i) {
  const double l = i > 0 ? v[i - 1] : 0.0;
  const double r = i < n - 1 ? v[i + 1] : 0.0;
  return (h / 6.0) * (4.0 * v[i] + l + r);
}

// One batch of shifted systems: block k solves (alpha_k A_G + beta_k M_G) y_k = rhs and stores
// coef_k y_k in scratch[k].  mode kIfaceOperator takes rhs = M p (p = in), otherwise rhs = in.
__device__ __forceinline__ void d_iface_solve(int n, double h, double al, double be, double ck,
                                              int mode, const double* __restrict__ in,
                                              double* __restrict__ out) {
  __shared__ double sa[kIfaceMaxN], sc[kIfaceMaxN], sd[kIfaceMaxN];
  const double off = -al / h + be * h / 6.0;
  const double dia = 2.0 * al / h + 4.0 * be * h / 6.0;
  const double inv = 1.0 / dia;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double rhs = (mode == kIfaceOperator) ? mass_apply(in, n, h, i) : in[i];
    sa[i] = i > 0 ? off * inv : 0.0;
    sc[i] = i < n - 1 ? off * inv : 0.0;
    sd[i] = rhs * inv;
  }
  __syncthreads();
  // parallel cyclic reduction; each thread owns rows threadIdx.x + t * blockDim.x
  constexpr int R = kIfaceMaxN / kIfaceThreads;
  for (int s = 1; s < n; s <<= 1) {
    double na[R], nc[R], nd[R];
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int i = threadIdx.x + t * kIfaceThreads;
      if (i >= n) continue;
      const double ai = sa[i], ci = sc[i], di = sd[i];
      const double am = i - s >= 0 ? sa[i - s] : 0.0, cm = i - s >= 0 ? sc[i - s] : 0.0,
                   dm = i - s >= 0 ? sd[i - s] : 0.0;
      const double ap = i + s < n ? sa[i + s] : 0.0, cp = i + s < n ? sc[i + s] : 0.0,
                   dp = i + s < n ? sd[i + s] : 0.0;
      const double den = 1.0 / (1.0 - ai * cm - ci * ap);
      na[t] = -ai * am * den;
      nc[t] = -ci * cp * den;
      nd[t] = (di - ai * dm - ci * dp) * den;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int i = threadIdx.x + t * kIfaceThreads;
      if (i >= n) continue;
      sa[i] = na[t];
      sc[i] = nc[t];
      sd[i] = nd[t];
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) out[i] = ck * sd[i];
}

// One block: sum of the m weighted solutions (k ascending) and the epilogue.
//   mode kIfacePrecond:      out = sum
//   mode kIfaceOperator:     out = d0 M p + M sum   (= H_RA p, p = in)
//   mode kIfacePrecondOuter: out = z = sum; rho_new = r.z (r = in); p_next = z + beta p_prev
// rtol2 >= 0 (batched solves): the outer PCG of this instance is declared converged on the
// device once rho_new <= rtol2 rho_0, recording the version that holds the final iterate.
__device__ __forceinline__ void d_iface_combine(
    int n, double h, int m, double d0, int mode, const double* __restrict__ in,
    double* __restrict__ out, const double* __restrict__ scratch, DevState* st,
    const double* __restrict__ p_prev, double* __restrict__ p_next, int ver, int first,
    double rtol2) {
  __shared__ double sd[kIfaceMaxN];
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    // the systems' terms are summed in system order; their loads are issued eight at a time
    double v = 0.0;
    int kk = 0;
    for (; kk + 8 <= m; kk += 8) {
      double t[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) t[q] = scratch[(size_t)(kk + q) * n + i];
#pragma unroll
      for (int q = 0; q < 8; ++q) v += t[q];
    }
    for (; kk < m; ++kk) v += scratch[(size_t)kk * n + i];
    sd[i] = v;
  }
  __syncthreads();
  if (mode == kIfacePrecond) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) out[i] = sd[i];
  } else if (mode == kIfaceOperator) {
    for (int i = threadIdx.x; i < n; i += blockDim.x)
      out[i] = d0 * mass_apply(in, n, h, i) + mass_apply(sd, n, h, i);
  } else {
    double rz = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      out[i] = sd[i];
      rz += in[i] * sd[i];
    }
    rz = bsum(rz);
    const double rho_prev = st->o_rho[ver & 1];
    const double beta = first ? 0.0 : rz / rho_prev;
    for (int i = threadIdx.x; i < n; i += blockDim.x)
      p_next[i] = first ? sd[i] : sd[i] + beta * p_prev[i];
    if (threadIdx.x == 0) {
      const int nv = first ? (ver & 1) : ((ver + 1) & 1);
      st->o_rho[nv] = rz;
      if (first) st->o_rho0 = rz;
      st->o_beta = beta;
      if (!(rz > 0.0) || !isfinite(rz)) {
        if (rz != 0.0) st->breakdown |= isfinite(rz) ? 2 : 4;
      }
      if (rtol2 >= 0.0) {
        // every quantity here is a function of version-ver data only, so a repeated call
        // (after the interior solve of this iteration was completed) gives the same state
        const double rho0 = first ? rz : st->o_rho0;
        st->o_its = first ? 0 : ver + 1;
        if (!(rz > rtol2 * rho0) || !isfinite(rz) || st->breakdown) {
          st->outer_done = 1;
          st->o_ver = first ? 0 : ((ver + 1) & 1);
        }
      }
    }
  }
}

// y = K (A_GG p - u|row nf) + gamma H p, with A_GG = tridiag(-1/2, 2, -1/2) on Gamma and u the
// interior solution for the lifted p (the interior neighbours of Gamma couple with -1).
// mode 0: write y.  mode 1 (outer PCG): alpha = rho / p.y, x_next = x + alpha p,
// r_next = r - alpha y.
__device__ __forceinline__ void d_schur_gather(
    int n, int nf, int pitch, double K, double gamma, const double* __restrict__ p,
    const double* __restrict__ u, const double* __restrict__ Hp, double* __restrict__ y,
    const double* __restrict__ x, double* __restrict__ xn, const double* __restrict__ r,
    double* __restrict__ rn, DevState* st, int mode, int ver) {
  const size_t row = (size_t)(nf - 1) * pitch;
  double pq = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double pl = i > 0 ? p[i - 1] : 0.0, pr = i < n - 1 ? p[i + 1] : 0.0;
    const double v = K * (2.0 * p[i] - 0.5 * (pl + pr) - u[row + i]) + gamma * Hp[i];
    y[i] = v;
    pq += p[i] * v;
  }
  if (mode == 0) return;
  pq = bsum(pq);
  const double rho = st->o_rho[ver & 1];
  const bool ok = (pq > 0.0) && isfinite(pq);
  const double alpha = ok ? rho / pq : 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    xn[i] = x[i] + alpha * p[i];
    rn[i] = r[i] - alpha * y[i];
  }
  if (threadIdx.x == 0) {
    st->o_pq = pq;
    st->o_alpha = alpha;
    if (!ok) st->breakdown |= isfinite(pq) ? 2 : 4;
  }
}

}  // namespace fdd
