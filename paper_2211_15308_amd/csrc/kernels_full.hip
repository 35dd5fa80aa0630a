// Full-system PCG of the 2D problem with the block preconditioner of eq. (dd_preconditioner),
// in the cheap form of the paper's remark on evaluating the operator (Sec. 3, Fig. 4-left): the
// operator A = K A_Omega + gamma T^T H_RA T is applied with H by its rational table, and the
// preconditioner's leading block (A^00)^{-1} = (K A_II)^{-1} by one multigrid V-cycle V / K.
//
// Vectors live in the solver's own layout: the interior part on the padded (n-1) x pitch grid
// (FP64), the Gamma part as a separate n-1 vector.  One preconditioner application
//   lower:     t_G = r_G + (V r_I)|row n-1          (A^{i0} (V r_I) / K, A_GI couples with -1)
//   diagonal:  z_G = S_Gamma^{-1} t_G               (rational table, eq. (RA))
//   upper:     z_I = V (r_I + K lift(z_G)) / K      (r_I - A^{0i} z_G)
// takes two V-cycles and one batch of shifted interface solves; one PCG iteration adds one
// operator application (one batch of shifted solves for H_RA p_G and a stencil pass).
//
// Iterations can be enqueued ahead of the host's read-back: once the stop test has passed (or
// a breakdown was flagged) every kernel of a later iteration returns at once, the V-cycles too
// (the stop test marks the multigrid solve stopped; the solve's end clears the mark).
//
// Scalars stay on the device: each reduction stores per-block partials and a one-block kernel
// sums them in a fixed order (no atomics: a ticket counter that every block of a 2048-block grid
// increments costs more than the launch), so every result is deterministic.
#include "iface_device.h"

namespace fdd {

namespace {

constexpr int kFullThreads = 256;
constexpr int kFullMaxBlocks = 2048;

// Block sum of one value per thread, stored by thread 0 as this block's partial.
__device__ __forceinline__ void block_partial(double v, double* __restrict__ partials) {
  __shared__ double sw[kFullThreads / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0;
    for (int w = 0; w < kFullThreads / 64; ++w) a += sw[w];
    partials[blockIdx.x] = a;
  }
}

inline int grid_blocks(int64_t tot) {
  return (int)std::min<int64_t>((tot + kFullThreads - 1) / kFullThreads, kFullMaxBlocks);
}

}  // namespace

// r = b, x = 0 (both parts), and the V-cycle inputs r_I (in the V-cycle's precision VT) and
// f' = r_I (whose top row receives K z_G later).  b: caller layout (compact interior, Gamma last).
template <typename VT>
__global__ __launch_bounds__(kFullThreads) void kf_init(int nf, int pitch, const double* __restrict__ b,
                                                        double* __restrict__ xI, double* __restrict__ rI,
                                                        double* __restrict__ xG, double* __restrict__ rG,
                                                        VT* __restrict__ vr, VT* __restrict__ vf,
                                                        DevState* st) {
  const int64_t NI = (int64_t)nf * nf;
  for (int64_t k = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; k < NI + nf;
       k += (int64_t)blockDim.x * gridDim.x) {
    if (k < NI) {
      const int i = (int)(k % nf), j = (int)(k / nf);
      const size_t o = (size_t)j * pitch + i;
      const double v = b[k];
      rI[o] = v;
      xI[o] = 0.0;
      vr[o] = (VT)v;
      vf[o] = (VT)v;
    } else {
      const int i = (int)(k - NI);
      rG[i] = b[k];
      xG[i] = 0.0;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->inner_done = 0;
    st->solve_done = 0;
    st->outer_done = 0;
    st->breakdown = 0;
    st->o_its = 0;
  }
}

// t_G = r_G + W|row nf (W = V r_I, the first V-cycle's result).  One block.
template <typename VT>
__global__ __launch_bounds__(kIfaceThreads) void kf_gamma_rhs(int nf, int pitch, const VT* __restrict__ W,
                                                              const double* __restrict__ rG,
                                                              double* __restrict__ tG,
                                                              const DevState* st) {
  if (st->outer_done) return;
  const size_t row = (size_t)(nf - 1) * pitch;
  for (int i = threadIdx.x; i < nf; i += blockDim.x) tG[i] = rG[i] + (double)W[row + i];
}

// f' top row += K z_G (so f' = r_I - A^{0i} z_G), before the second V-cycle.  One block.
template <typename VT>
__global__ __launch_bounds__(kIfaceThreads) void kf_lift(int nf, int pitch, double K,
                                                         const double* __restrict__ rI,
                                                         const double* __restrict__ zG,
                                                         VT* __restrict__ vf, const DevState* st) {
  if (st->outer_done) return;
  const size_t row = (size_t)(nf - 1) * pitch;
  for (int i = threadIdx.x; i < nf; i += blockDim.x) vf[row + i] = (VT)(rI[row + i] + K * zG[i]);
}

// rz = r . z with z_I = Z / K (Z the second V-cycle's result) and z_G; the last block derives
// beta = rz / rz_prev, stores rz by iteration parity (cur = the parity of this rz), and takes
// the stop test (rz <= rtol2 rz_0).  first: this rz is rz_0.
template <typename VT>
__global__ __launch_bounds__(kFullThreads) void kf_rz(int nf, int pitch, double invK,
                                                      const VT* __restrict__ Z,
                                                      const double* __restrict__ rI,
                                                      const double* __restrict__ zG,
                                                      const double* __restrict__ rG, DevState* st,
                                                      double* __restrict__ partials, int cur,
                                                      int first, double rtol2) {
  if (st->outer_done) return;
  const int64_t NI = (int64_t)nf * nf;
  double acc = 0.0;
  for (int64_t k = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; k < NI + nf;
       k += (int64_t)blockDim.x * gridDim.x) {
    if (k < NI) {
      const size_t o = (size_t)(k / nf) * pitch + (size_t)(k % nf);
      acc += rI[o] * ((double)Z[o] * invK);
    } else {
      const int i = (int)(k - NI);
      acc += rG[i] * zG[i];
    }
  }
  block_partial(acc, partials);
}

// beta, rz and the stop test from kf_rz's partials (one block).
__global__ __launch_bounds__(kFullThreads) void kf_rz_finish(DevState* st, const double* __restrict__ partials,
                                                             int nb, int cur, int first, double rtol2,
                                                             int it) {
  if (st->outer_done) return;
  const double rz = block_sum_partials(partials, nb, 1);
  if (threadIdx.x != 0) return;
  if (first) st->o_rho0 = rz;
  const double rho0 = first ? rz : st->o_rho0;
  const double prev = st->o_rho[cur ^ 1];
  st->o_rho[cur] = rz;
  st->o_beta = first ? 0.0 : rz / prev;
  if (!isfinite(rz)) st->breakdown |= 4;
  else if (rz < 0.0) st->breakdown |= 2;
  if (!(rz > rtol2 * rho0) || st->breakdown) {
    st->outer_done = 1;
    st->o_its = it;
    st->inner_done = 1;  // the V-cycles of iterations enqueued beyond this one return at once
  }
}

// p_G = z_G + beta p_G' (first: p_G = z_G).  One block.
__global__ __launch_bounds__(kIfaceThreads) void kf_gamma_p(int ng, const double* __restrict__ zG,
                                                            const double* __restrict__ pGo,
                                                            double* __restrict__ pGn,
                                                            const DevState* st, int first) {
  if (st->outer_done) return;
  const double beta = first ? 0.0 : st->o_beta;
  for (int i = threadIdx.x; i < ng; i += blockDim.x) pGn[i] = first ? zG[i] : zG[i] + beta * pGo[i];
}

// p_I = Z / K + beta p_I' (formed where read), q = A p on every dof (K times the P1 stiffness,
// natural-boundary row on Gamma, plus gamma H_RA p_G there), and p . q; the last block sets
// alpha = rz / p.q.  Writes p_I and q.
template <typename VT>
__global__ __launch_bounds__(kFullThreads) void kf_apply(int nf, int pitch, double K, double gamma,
                                                         double invK, const VT* __restrict__ Z,
                                                         const double* __restrict__ pIo,
                                                         double* __restrict__ pIn,
                                                         const double* __restrict__ pG,
                                                         const double* __restrict__ Hp,
                                                         double* __restrict__ qI,
                                                         double* __restrict__ qG, DevState* st,
                                                         double* __restrict__ partials, int cur,
                                                         int first) {
  if (st->outer_done) return;
  const double beta = first ? 0.0 : st->o_beta;
  auto pI = [&](int i, int j) -> double {  // p at interior node (i, j), 0-based, 0 outside
    if (i < 0 || i >= nf || j < 0) return 0.0;
    if (j >= nf) return pG[i];
    const size_t o = (size_t)j * pitch + i;
    const double z = (double)Z[o] * invK;
    return first ? z : z + beta * pIo[o];
  };
  const int64_t NI = (int64_t)nf * nf;
  double acc = 0.0;
  for (int64_t k = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; k < NI + nf;
       k += (int64_t)blockDim.x * gridDim.x) {
    if (k < NI) {
      const int i = (int)(k % nf), j = (int)(k / nf);
      const size_t o = (size_t)j * pitch + i;
      // p at the node and its w, e, s, n neighbours as pI gives it, with every load issued before
      // the first use: an interior point reads Z and p', the north point above the top row reads
      // p_G, and a point outside reads the node's own entries and is zeroed
      constexpr int kDi[5] = {0, -1, 1, 0, 0}, kDj[5] = {0, 0, 0, -1, 1};
      bool in[5];
      size_t oo[5];
      VT zr[5];
      double pr[5];
#pragma unroll
      for (int a = 0; a < 5; ++a) {
        const int ii = i + kDi[a], jj = j + kDj[a];
        in[a] = ii >= 0 && ii < nf && jj >= 0 && jj < nf;
        oo[a] = in[a] ? (size_t)jj * pitch + ii : o;
      }
      const bool top = j == nf - 1;  // the north point is the interface node i
#pragma unroll
      for (int a = 0; a < 5; ++a) {
        zr[a] = Z[oo[a]];
        pr[a] = first ? 0.0 : pIo[oo[a]];
      }
      const double gn = pG[top ? i : 0];
      __builtin_amdgcn_sched_barrier(0);
      double P[5];
#pragma unroll
      for (int a = 0; a < 5; ++a) {
        const double z = (double)zr[a] * invK;
        P[a] = in[a] ? (first ? z : z + beta * pr[a]) : 0.0;
      }
      if (top) P[4] = gn;
      const double c = P[0];
      const double q = K * (4.0 * c - P[1] - P[2] - P[3] - P[4]);
      pIn[o] = c;
      qI[o] = q;
      acc += c * q;
    } else {
      const int i = (int)(k - NI);
      const double c = pG[i];
      const double l = i > 0 ? pG[i - 1] : 0.0, r = i < nf - 1 ? pG[i + 1] : 0.0;
      const double q = K * (2.0 * c - 0.5 * (l + r) - pI(i, nf - 1)) + gamma * Hp[i];
      qG[i] = q;
      acc += c * q;
    }
  }
  block_partial(acc, partials);
}

// alpha = rz / p.q from kf_apply's partials (one block).
__global__ __launch_bounds__(kFullThreads) void kf_pq_finish(DevState* st, const double* __restrict__ partials,
                                                             int nb, int cur, int it) {
  if (st->outer_done) return;
  const double pq = block_sum_partials(partials, nb, 1);
  if (threadIdx.x != 0) return;
  const double rz = st->o_rho[cur];
  const bool ok = pq > 0.0 && isfinite(pq);
  st->o_pq = pq;
  st->o_alpha = ok ? rz / pq : 0.0;
  if (!ok) {
    st->breakdown |= isfinite(pq) ? 2 : 4;
    st->outer_done = 1;
    st->o_its = it;
    st->inner_done = 1;
  }
}

// x += alpha p, r -= alpha q on every dof; the new r_I also goes to the V-cycle inputs.
template <typename VT>
__global__ __launch_bounds__(kFullThreads) void kf_update(int nf, int pitch, double* __restrict__ xI,
                                                          double* __restrict__ rI,
                                                          const double* __restrict__ pI,
                                                          const double* __restrict__ qI,
                                                          double* __restrict__ xG,
                                                          double* __restrict__ rG,
                                                          const double* __restrict__ pG,
                                                          const double* __restrict__ qG,
                                                          VT* __restrict__ vr, VT* __restrict__ vf,
                                                          DevState* st) {
  if (st->outer_done) return;
  const double alpha = st->o_alpha;
  const int64_t NI = (int64_t)nf * nf;
  for (int64_t k = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; k < NI + nf;
       k += (int64_t)blockDim.x * gridDim.x) {
    if (k < NI) {
      const size_t o = (size_t)(k / nf) * pitch + (size_t)(k % nf);
      xI[o] += alpha * pI[o];
      const double r = rI[o] - alpha * qI[o];
      rI[o] = r;
      vr[o] = (VT)r;
      vf[o] = (VT)r;
    } else {
      const int i = (int)(k - NI);
      xG[i] += alpha * pG[i];
      rG[i] -= alpha * qG[i];
    }
  }
}

// out (caller layout) = (a_I * sI, a_G): the iterate (sI = 1) or the preconditioned vector
// (a_I = Z, sI = 1 / K).
template <typename VT>
__global__ __launch_bounds__(kFullThreads) void kf_scatter(int nf, int pitch, const VT* __restrict__ aI,
                                                           double sI, const double* __restrict__ aG,
                                                           double* __restrict__ out) {
  const int64_t NI = (int64_t)nf * nf;
  for (int64_t k = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; k < NI + nf;
       k += (int64_t)blockDim.x * gridDim.x) {
    if (k < NI) out[k] = (double)aI[(size_t)(k / nf) * pitch + (size_t)(k % nf)] * sI;
    else out[k] = aG[k - NI];
  }
}

// The solve's end: the multigrid solve is no longer marked stopped.
__global__ void kf_clear_stop(DevState* st) {
  if (threadIdx.x == 0) st->inner_done = 0;
}

// ---- launchers ----------------------------------------------------------------------------

template <typename VT>
void launch_full_init(const FullCtx& c, const double* b, VT* vr, VT* vf) {
  const int64_t tot = (int64_t)c.nf * c.nf + c.nf;
  hipLaunchKernelGGL(kf_init<VT>, dim3(grid_blocks(tot)), dim3(kFullThreads), 0, c.stream, c.nf,
                     c.pitch, b, c.xI, c.rI, c.xG, c.rG, vr, vf, c.st);
}

template <typename VT>
void launch_full_precond_tail(const FullCtx& c, const ShiftTable& tabP, const VT* W, VT* vf) {
  // lower factor and the interface block, then the upper factor's right-hand side
  hipLaunchKernelGGL(kf_gamma_rhs<VT>, dim3(1), dim3(kIfaceThreads), 0, c.stream, c.nf, c.pitch,
                     W, c.rG, c.tG, (const DevState*)c.st);
  launch_iface_batch(c.stream, c.nf, c.h, tabP, kIfacePrecond, c.tG, c.zG, c.scratchP, c.st,
                     nullptr, nullptr, 0, 0);
  hipLaunchKernelGGL(kf_lift<VT>, dim3(1), dim3(kIfaceThreads), 0, c.stream, c.nf, c.pitch, c.K,
                     c.rI, c.zG, vf, (const DevState*)c.st);
}

template <typename VT>
void launch_full_rz(const FullCtx& c, const VT* Z, int cur, int first, double rtol2, int it) {
  const int64_t tot = (int64_t)c.nf * c.nf + c.nf;
  const int nb = grid_blocks(tot);
  hipLaunchKernelGGL(kf_rz<VT>, dim3(nb), dim3(kFullThreads), 0, c.stream, c.nf, c.pitch,
                     1.0 / c.K, Z, c.rI, c.zG, c.rG, c.st, c.partials, cur, first, rtol2);
  hipLaunchKernelGGL(kf_rz_finish, dim3(1), dim3(kFullThreads), 0, c.stream, c.st,
                     (const double*)c.partials, nb, cur, first, rtol2, it);
}

template <typename VT>
void launch_full_step(const FullCtx& c, const ShiftTable& tabH, const VT* Z, int a, int cur,
                      int first, VT* vr, VT* vf, int it) {
  const int64_t tot = (int64_t)c.nf * c.nf + c.nf;
  const int b = a ^ 1;  // p version written now
  hipLaunchKernelGGL(kf_gamma_p, dim3(1), dim3(kIfaceThreads), 0, c.stream, c.nf, c.zG, c.pG[a],
                     c.pG[b], (const DevState*)c.st, first);
  launch_iface_batch(c.stream, c.nf, c.h, tabH, kIfaceOperator, c.pG[b], c.Hp, c.scratchH, c.st,
                     nullptr, nullptr, 0, 0);
  const int nb = grid_blocks(tot);
  hipLaunchKernelGGL(kf_apply<VT>, dim3(nb), dim3(kFullThreads), 0, c.stream, c.nf, c.pitch, c.K,
                     c.gamma, 1.0 / c.K, Z, c.pI[a], c.pI[b], c.pG[b], c.Hp, c.qI, c.qG, c.st,
                     c.partials, cur, first);
  hipLaunchKernelGGL(kf_pq_finish, dim3(1), dim3(kFullThreads), 0, c.stream, c.st,
                     (const double*)c.partials, nb, cur, it);
  hipLaunchKernelGGL(kf_update<VT>, dim3(grid_blocks(tot)), dim3(kFullThreads), 0, c.stream,
                     c.nf, c.pitch, c.xI, c.rI, c.pI[b], c.qI, c.xG, c.rG, c.pG[b], c.qG, vr, vf,
                     c.st);
}

void launch_full_clear_stop(const FullCtx& c) {
  hipLaunchKernelGGL(kf_clear_stop, dim3(1), dim3(64), 0, c.stream, c.st);
}

template <typename VT>
void launch_full_scatter(const FullCtx& c, const VT* aI, double sI, const double* aG, double* out) {
  const int64_t tot = (int64_t)c.nf * c.nf + c.nf;
  hipLaunchKernelGGL(kf_scatter<VT>, dim3(grid_blocks(tot)), dim3(kFullThreads), 0, c.stream,
                     c.nf, c.pitch, aI, sI, aG, out);
}

#define FDD_FULL_INST(VT)                                                                          \
  template void launch_full_init<VT>(const FullCtx&, const double*, VT*, VT*);                    \
  template void launch_full_precond_tail<VT>(const FullCtx&, const ShiftTable&, const VT*, VT*);  \
  template void launch_full_rz<VT>(const FullCtx&, const VT*, int, int, double, int);             \
  template void launch_full_step<VT>(const FullCtx&, const ShiftTable&, const VT*, int, int, int, \
                                     VT*, VT*, int);                                              \
  template void launch_full_scatter<VT>(const FullCtx&, const VT*, double, const double*, double*);
FDD_FULL_INST(float)
FDD_FULL_INST(double)
#undef FDD_FULL_INST

}  // namespace fdd
