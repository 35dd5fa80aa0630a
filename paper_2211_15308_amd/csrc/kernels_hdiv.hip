// Kernels of the H(div) problem (Sec. 3, remark on H(div)-elliptic problems, eq. (graddiv)).
//
// * Sparse products in typed ELL form (slot k of row i at k * rows + i: a wave reads consecutive
//   rows, so its column loads coalesce; values come from a small per-row-type table, the gathered
//   x entries from L2).
// * The multigrid smoother for A^00 = K(I - grad div) on V_0 is additive Schwarz over vertex
//   patches (the dofs on the edges at a vertex; the patches hold the curls of the P2 vertex and
//   edge functions, which span the kernel of div): one thread per vertex multiplies the patch's
//   residual by the inverse patch matrix (one of a few matrices: congruent patches share it), and
//   one thread per dof sums the two patches holding it.  Both steps are gathers, so no atomics and
//   the sums are in fixed order.
// * Reductions: per-block partials, summed in fixed order by one block (bitwise reproducible).
// * The trace preconditioner: the shifted systems (L + q M) y = r on the loop are block circulant
//   (2 x 2 blocks, one per segment), solved by cyclic reduction in LDS: every row of a step has
//   the same blocks, so only right-hand sides are stored (2 x 4n x 2 doubles <= 128 KB).
#include <hip/hip_runtime.h>

#include "hdiv_internal.h"

namespace fdd {

namespace {

constexpr int kT = 256;            // threads of the vector kernels
constexpr int kOneBlock = 1024;    // threads of the one-block kernels
constexpr int kLoopSeg = 4 * kHdMaxN;

inline int blocks_for(int64_t n) { return (int)((n + kT - 1) / kT); }
inline int red_blocks(int64_t n) { return (int)std::min<int64_t>(blocks_for(n), kHdPartials); }

__device__ __forceinline__ bool stopped(const HdState* s) { return s && s->done; }

// Sum over the block of up to 1024 threads, fixed order; the result is valid in every thread.
__device__ double block_sum(double v) {
  __shared__ double sh[kOneBlock / 64 + 1];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) s += sh[w];
    sh[kOneBlock / 64] = s;
  }
  __syncthreads();
  return sh[kOneBlock / 64];
}

// Fixed-order sum of nb partials by one block.
__device__ double sum_partials(const double* p, int nb) {
  double v = 0.0;
  for (int k = threadIdx.x; k < nb; k += blockDim.x) v += p[k];
  return block_sum(v);
}

// row i of A times x; the two column forms in separate loops (the choice is uniform per launch)
__device__ __forceinline__ double ell_row(const HdView& A, int i, const double* __restrict__ x) {
  const int t = A.rtype[i];
  const double* v = A.tval + (size_t)t * A.width;
  double s = 0.0;
  if (A.toff) {
    const int* o = A.toff + t * A.width;
    for (int k = 0; k < A.width; ++k) s += v[k] * x[i + o[k]];
  } else {
    for (int k = 0; k < A.width; ++k) s += v[k] * x[A.col[(size_t)k * A.rows + i]];
  }
  return s;
}

// The type table of a product (values, and offsets in the relative form) staged in LDS when it
// has at most kTabLds entries: every slot of every row reads it, and LDS serves a wave's reads of
// one entry in one access where the cache would take a vector load per slot.
constexpr int kTabLds = 1024;
struct TabLds {
  double v[kTabLds];
  int o[kTabLds];
};

// every thread of the block (kT threads) calls it; true when the table is in LDS.  A thread
// issues all its loads before its first LDS store, so the block waits for one load latency
// (a loop that stores each entry as it arrives waits once per entry).
__device__ bool stage_table(const HdView& A, TabLds& T) {
  const int nt = A.ntypes * A.width;
  if (nt > kTabLds) return false;
  constexpr int R = kTabLds / kT;
  static_assert(R * kT == kTabLds, "the table is a whole number of block-wide rows");
  double v[R];
  int o[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int k = threadIdx.x + q * kT;
    v[q] = k < nt ? A.tval[k] : 0.0;
    o[q] = (A.toff && k < nt) ? A.toff[k] : 0;
  }
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int k = threadIdx.x + q * kT;
    if (k < nt) {
      T.v[k] = v[q];
      T.o[k] = o[q];
    }
  }
  __syncthreads();
  return true;
}

// row i (of type t) of A times x with the table in LDS (kLds) or in global memory
template <bool kLds>
__device__ __forceinline__ double ell_row_tab(const HdView& A, const TabLds& T, int i, int t,
                                              const double* __restrict__ x) {
  const int base = t * A.width;
  double s = 0.0;
  if (A.toff) {
    for (int k = 0; k < A.width; ++k) {
      const double v = kLds ? T.v[base + k] : A.tval[base + k];
      const int o = kLds ? T.o[base + k] : A.toff[base + k];
      s += v * x[i + o];
    }
  } else {
    for (int k = 0; k < A.width; ++k) {
      const double v = kLds ? T.v[base + k] : A.tval[base + k];
      s += v * x[A.col[(size_t)k * A.rows + i]];
    }
  }
  return s;
}

// grid of the row kernels: a grid-stride loop over at most kRowBlocks blocks, so that each block
// stages the table once for several chunks of rows
constexpr int kRowBlocks = 2048;
inline int row_blocks(int64_t n) { return (int)std::min<int64_t>(blocks_for(n), kRowBlocks); }

// ---- sparse products, smoother, coarse solve ------------------------------------------------

template <int PW>
__device__ __forceinline__ void patch_solve_vertex(const int* __restrict__ patch,
                                                   const int* __restrict__ ptype,
                                                   const double* pinv, int v,
                                                   const double* __restrict__ r,
                                                   double* __restrict__ Y) {
  // no branches between the loads, so the vertex's type, dof indices and residual values are in
  // flight together: indices of empty slots (-1) read r[0] and are zeroed, and a vertex without a
  // patch (type -1, every slot empty) stores zeros into slots that are never read back
  const int t = ptype[v];
  int d[PW];
#pragma unroll
  for (int k = 0; k < PW; ++k) d[k] = patch[(size_t)v * PW + k];
  __builtin_amdgcn_sched_barrier(0);  // every index load issued before the gathers
  double rl[PW];
#pragma unroll
  for (int k = 0; k < PW; ++k) rl[k] = r[d[k] < 0 ? 0 : d[k]];
  __builtin_amdgcn_sched_barrier(0);  // every gather issued before the first product
#pragma unroll
  for (int k = 0; k < PW; ++k) rl[k] = d[k] >= 0 ? rl[k] : 0.0;
  const double* Pi = pinv + (size_t)(t < 0 ? 0 : t) * PW * PW;
  // every slot is written (a lane's PW values are contiguous, so the stores combine)
#pragma unroll
  for (int a = 0; a < PW; ++a) {
    double y = 0.0;
#pragma unroll
    for (int b = 0; b < PW; ++b) y += Pi[a * PW + b] * rl[b];
    Y[(size_t)v * PW + a] = y;
  }
}

__global__ __launch_bounds__(kT) void k_hd_spmv(HdView A, const double* __restrict__ x,
                                                double* __restrict__ y, double alpha, double beta,
                                                const HdState* stop) {
  if (stopped(stop)) return;
  __shared__ TabLds T;
  // a row's type is loaded one step ahead: the first row's before the table is staged (the
  // staging barrier waits for both), the next row's before the current row's gathers
  const int stride = gridDim.x * kT;
  int i = blockIdx.x * kT + threadIdx.x;
  int t = i < A.rows ? A.rtype[i] : 0;
  const bool lds = stage_table(A, T);
  for (; i < A.rows; i += stride) {
    const int tn = i + stride < A.rows ? A.rtype[i + stride] : 0;
    const double s = lds ? ell_row_tab<true>(A, T, i, t, x) : ell_row_tab<false>(A, T, i, t, x);
    y[i] = (beta == 0.0 ? 0.0 : beta * y[i]) + alpha * s;
    t = tn;
  }
}

__global__ __launch_bounds__(kT) void k_hd_residual(HdView A, const double* __restrict__ b,
                                                    const double* __restrict__ x,
                                                    double* __restrict__ r, const HdState* stop) {
  if (stopped(stop)) return;
  __shared__ TabLds T;
  // a row's type and b entry are loaded one step ahead, as in k_hd_spmv
  const int stride = gridDim.x * kT;
  int i = blockIdx.x * kT + threadIdx.x;
  int t = i < A.rows ? A.rtype[i] : 0;
  double bi = i < A.rows ? b[i] : 0.0;
  const bool lds = stage_table(A, T);
  for (; i < A.rows; i += stride) {
    const bool more = i + stride < A.rows;
    const int tn = more ? A.rtype[i + stride] : 0;
    const double bn = more ? b[i + stride] : 0.0;
    r[i] = bi - (lds ? ell_row_tab<true>(A, T, i, t, x) : ell_row_tab<false>(A, T, i, t, x));
    t = tn;
    bi = bn;
  }
}

// (the few inverse patch matrices are staged in LDS: every lane reads a row of its vertex's)
template <int PW>
__global__ __launch_bounds__(kT) void k_hd_patch_solve(const int* __restrict__ patch,
                                                       const int* __restrict__ ptype,
                                                       const double* __restrict__ pinv, int ntypes,
                                                       int nvert, const double* __restrict__ r,
                                                       double* __restrict__ Y, const HdState* stop) {
  if (stopped(stop)) return;
  __shared__ double sp[kHdMaxTypes * PW * PW];
  {
    // all of a thread's loads before its LDS stores (one load latency per block)
    constexpr int R = (kHdMaxTypes * PW * PW + kT - 1) / kT;
    const int nt = ntypes * PW * PW;
    double w[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int k = threadIdx.x + q * kT;
      w[q] = k < nt ? pinv[k] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int k = threadIdx.x + q * kT;
      if (k < nt) sp[k] = w[q];
    }
  }
  __syncthreads();
  const int v = blockIdx.x * kT + threadIdx.x;
  if (v >= nvert) return;
  patch_solve_vertex<PW>(patch, ptype, sp, v, r, Y);
}

__global__ __launch_bounds__(kT) void k_hd_patch_sum(const int* __restrict__ slot, int n0,
                                                     const double* __restrict__ Y, double theta,
                                                     double* __restrict__ x, int add,
                                                     const HdState* stop) {
  if (stopped(stop)) return;
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i >= n0) return;
  // the slots and the old x first, then both patch values (clamped indices, no branch), so the
  // dof waits for two load latencies rather than three
  const int s0 = slot[2 * (size_t)i], s1 = slot[2 * (size_t)i + 1];
  const double xo = add ? x[i] : 0.0;
  __builtin_amdgcn_sched_barrier(0);
  const double y0 = Y[s0 < 0 ? 0 : s0], y1 = Y[s1 < 0 ? 0 : s1];
  double v = 0.0;
  if (s0 >= 0) v += y0;
  if (s1 >= 0) v += y1;
  x[i] = xo + theta * v;
}

// One step of the Jacobi-preconditioned Chebyshev iteration for A x = b (x_0 = 0), the diagonal
// inverse from one-dof patches (Dinv_i = pinv[ptype[i]]):
//   first: d = c_res Dinv b, x_out = d;
//   else:  r = b - A x_in (formed here), d = c_prev d + c_res Dinv r, x_out = x_in + d.
// One launch per step, no inner products (the step count follows from the spectral bounds).
__global__ __launch_bounds__(kT) void k_hd_cheb_step(HdView A, const int* __restrict__ ptype,
                                                     const double* __restrict__ pinv,
                                                     const double* __restrict__ b,
                                                     const double* __restrict__ x_in,
                                                     double* __restrict__ x_out,
                                                     double* __restrict__ d, double c_prev,
                                                     double c_res, int first) {
  __shared__ TabLds T;
  // the first row's type and diagonal-patch type are loaded before the table is staged
  int i = blockIdx.x * kT + threadIdx.x;
  int t = i < A.rows ? A.rtype[i] : 0;
  int pt = i < A.rows ? ptype[i] : 0;
  const bool lds = stage_table(A, T);
  for (; i < A.rows; i += gridDim.x * kT, t = i < A.rows ? A.rtype[i] : 0,
                                         pt = i < A.rows ? ptype[i] : 0) {
    const double dinv = pinv[pt];
    if (first) {
      const double di = c_res * dinv * b[i];
      d[i] = di;
      x_out[i] = di;
    } else {
      const double r = b[i] - (lds ? ell_row_tab<true>(A, T, i, t, x_in)
                                   : ell_row_tab<false>(A, T, i, t, x_in));
      const double di = c_prev * d[i] + c_res * dinv * r;
      d[i] = di;
      x_out[i] = x_in[i] + di;
    }
  }
}

__device__ __forceinline__ double dense_row(const double* __restrict__ C, int n0, int row, int lane,
                                            const double* __restrict__ b) {
  const double* c = C + (size_t)row * n0;
  double s = 0.0;
  for (int j = lane; j < n0; j += 64) s += c[j] * b[j];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  return s;
}

// x = C b, one wave per row (C row-major): the lanes read consecutive entries of the row and
// the wave sums them in fixed order
__global__ __launch_bounds__(kT) void k_hd_coarse(const double* __restrict__ C, int n0,
                                                  const double* __restrict__ b,
                                                  double* __restrict__ x, const HdState* stop) {
  if (stopped(stop)) return;
  const int row = blockIdx.x * (kT / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= n0) return;
  const double s = dense_row(C, n0, row, lane, b);
  if (lane == 0) x[row] = s;
}

// ---- interior PCG ------------------------------------------------------------------------------

__global__ __launch_bounds__(kT) void k_hd_pcg_start(int n0, const double* __restrict__ f,
                                                     double* __restrict__ u, double* __restrict__ r,
                                                     double* __restrict__ partials) {
  double s = 0.0;
  for (int i = blockIdx.x * kT + threadIdx.x; i < n0; i += gridDim.x * kT) {
    const double v = f[i];
    u[i] = 0.0;
    r[i] = v;
    s += v * v;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(kOneBlock) void k_hd_start_finish(const double* partials, int nb,
                                                               HdState* st, double tol2) {
  const double ff = sum_partials(partials, nb);
  if (threadIdx.x == 0) {
    st->ff = ff;
    st->rr = ff;
    st->tol2 = tol2;
    st->its = 0;
    st->breakdown = (st->breakdown & 2) | (isfinite(ff) ? 0 : 4);
    st->done = (ff == 0.0 || !isfinite(ff)) ? 1 : 0;
    st->rz = st->rz_old = st->alpha = st->beta = 0.0;
  }
}

__global__ __launch_bounds__(kT) void k_hd_dot(int n, const double* __restrict__ a,
                                               const double* __restrict__ b,
                                               double* __restrict__ partials, const HdState* stop) {
  if (stopped(stop)) return;
  double s = 0.0;
  for (int i = blockIdx.x * kT + threadIdx.x; i < n; i += gridDim.x * kT) s += a[i] * b[i];
  s = block_sum(s);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(kOneBlock) void k_hd_rz_finish(const double* partials, int nb,
                                                            HdState* st, int first) {
  if (st->done) return;
  const double rz = sum_partials(partials, nb);
  if (threadIdx.x == 0) {
    if (!(rz > 0.0) || !isfinite(rz)) {
      // r.z = 0 with r = 0 is convergence; otherwise the preconditioner is not positive
      if (rz != 0.0) st->breakdown |= isfinite(rz) ? 1 : 4;
      st->done = 1;
      return;
    }
    st->beta = first ? 0.0 : rz / st->rz;
    st->rz_old = st->rz;
    st->rz = rz;
  }
}

template <bool kLds>
__device__ __forceinline__ double pq_row(const HdView& A, const TabLds& T, int i, int t,
                                         const double* __restrict__ z,
                                         const double* __restrict__ p_old, double beta, int first) {
  const int base = t * A.width;
  double qi = 0.0;
  for (int k = 0; k < A.width; ++k) {
    const double v = kLds ? T.v[base + k] : A.tval[base + k];
    const int c = A.toff ? i + (kLds ? T.o[base + k] : A.toff[base + k])
                         : A.col[(size_t)k * A.rows + i];
    qi += v * (first ? z[c] : z[c] + beta * p_old[c]);
  }
  return qi;
}

__global__ __launch_bounds__(kT) void k_hd_pq(HdView A, const double* __restrict__ z,
                                              const double* __restrict__ p_old,
                                              double* __restrict__ p_new, double* __restrict__ q,
                                              double* __restrict__ partials, const HdState* st,
                                              int first) {
  if (st->done) return;
  __shared__ TabLds T;
  // a row's type is loaded one step ahead, as in k_hd_spmv
  const int stride = gridDim.x * kT;
  int i = blockIdx.x * kT + threadIdx.x;
  int t = i < A.rows ? A.rtype[i] : 0;
  const bool lds = stage_table(A, T);
  const double beta = st->beta;
  double s = 0.0;
  for (; i < A.rows; i += stride) {
    const int tn = i + stride < A.rows ? A.rtype[i + stride] : 0;
    // q = A (z + beta p_old), with the direction formed where the product reads it
    const double qi = lds ? pq_row<true>(A, T, i, t, z, p_old, beta, first)
                          : pq_row<false>(A, T, i, t, z, p_old, beta, first);
    t = tn;
    const double pi = first ? z[i] : z[i] + beta * p_old[i];
    p_new[i] = pi;
    q[i] = qi;
    s += pi * qi;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(kOneBlock) void k_hd_pq_finish(const double* partials, int nb,
                                                            HdState* st) {
  if (st->done) return;
  const double pq = sum_partials(partials, nb);
  if (threadIdx.x == 0) {
    if (!(pq > 0.0) || !isfinite(pq)) {
      st->breakdown |= isfinite(pq) ? 1 : 4;
      st->done = 1;
      return;
    }
    st->alpha = st->rz / pq;
  }
}

__global__ __launch_bounds__(kT) void k_hd_update(int n0, const double* __restrict__ p,
                                                  const double* __restrict__ q,
                                                  double* __restrict__ u, double* __restrict__ r,
                                                  double* __restrict__ partials, const HdState* st) {
  if (st->done) return;
  const double a = st->alpha;
  double s = 0.0;
  for (int i = blockIdx.x * kT + threadIdx.x; i < n0; i += gridDim.x * kT) {
    u[i] += a * p[i];
    const double ri = r[i] - a * q[i];
    r[i] = ri;
    s += ri * ri;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(kOneBlock) void k_hd_update_finish(const double* partials, int nb,
                                                                HdState* st) {
  if (st->done) return;
  const double rr = sum_partials(partials, nb);
  if (threadIdx.x == 0) {
    st->rr = rr;
    st->its += 1;
    if (!isfinite(rr)) {
      st->breakdown |= 4;
      st->done = 1;
    } else if (rr <= st->tol2 * st->ff) {
      st->done = 1;
    }
  }
}

// ---- the trace preconditioner -------------------------------------------------------------------

struct M2 {
  double a, b, c, d;  // [[a, b], [c, d]]
};
__device__ __forceinline__ M2 mk(const double* v) { return M2{v[0], v[1], v[2], v[3]}; }
__device__ __forceinline__ M2 mul(M2 x, M2 y) {
  return M2{x.a * y.a + x.b * y.c, x.a * y.b + x.b * y.d, x.c * y.a + x.d * y.c,
            x.c * y.b + x.d * y.d};
}
__device__ __forceinline__ M2 add(M2 x, M2 y) { return M2{x.a + y.a, x.b + y.b, x.c + y.c, x.d + y.d}; }
__device__ __forceinline__ M2 sub(M2 x, M2 y) { return M2{x.a - y.a, x.b - y.b, x.c - y.c, x.d - y.d}; }
__device__ __forceinline__ M2 neg(M2 x) { return M2{-x.a, -x.b, -x.c, -x.d}; }
__device__ __forceinline__ M2 tr(M2 x) { return M2{x.a, x.c, x.b, x.d}; }
__device__ __forceinline__ M2 inv(M2 x) {
  const double det = x.a * x.d - x.b * x.c;
  return M2{x.d / det, -x.b / det, -x.c / det, x.a / det};
}
__device__ __forceinline__ double2 mv(M2 x, double2 v) {
  return make_double2(x.a * v.x + x.b * v.y, x.c * v.x + x.d * v.y);
}
__device__ __forceinline__ double2 sub2(double2 u, double2 v) { return make_double2(u.x - v.x, u.y - v.y); }
__device__ __forceinline__ double2 add2(double2 u, double2 v) { return make_double2(u.x + v.x, u.y + v.y); }

// Blocks < m: y_k = (L + q_k M)^{-1} r by cyclic reduction; block m: the M^-1 terms
// d0 M^-1 L M^-1 r + dsum M^-1 r.  Outputs to scratch rows of 8n.
__global__ __launch_bounds__(kOneBlock) void k_hd_loop_solve(int nseg, HdLoopBlocks blk, HdTable T,
                                                             const double* __restrict__ r,
                                                             double* __restrict__ scratch) {
  __shared__ double2 buf[2][kLoopSeg];
  const int k = blockIdx.x, m = T.m;
  const int N = nseg;
  double2* cur = buf[0];
  double2* nxt = buf[1];
  for (int i = threadIdx.x; i < N; i += blockDim.x) cur[i] = make_double2(r[2 * i], r[2 * i + 1]);
  __syncthreads();
  const M2 Ms = mk(blk.mass), P = mk(blk.prev), O = mk(blk.own);
  double* out = scratch + (size_t)k * 2 * N;
  if (k == m) {
    const M2 Mi = inv(Ms);
    for (int i = threadIdx.x; i < N; i += blockDim.x) nxt[i] = mv(Mi, cur[i]);   // w1 = M^-1 r
    __syncthreads();
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
      const double2 wl = nxt[(i + N - 1) % N], wc = nxt[i], wr = nxt[(i + 1) % N];
      const double2 t = add2(add2(mv(P, wl), mv(O, wc)), mv(tr(P), wr));   // L w1
      const double2 w2 = mv(Mi, t);
      out[2 * i] = T.d0 * w2.x + T.dsum * wc.x;
      out[2 * i + 1] = T.d0 * w2.y + T.dsum * wc.y;
    }
    return;
  }
  // row i: A x_{i-s} + D x_i + C x_{i+s} = r_i (indices mod N); every row has the same blocks
  const double q = T.q[k];
  M2 D = add(O, M2{q * Ms.a, q * Ms.b, q * Ms.c, q * Ms.d});
  M2 A = P, C = tr(P);
  for (int s = 1; 4 * s <= N; s *= 2) {
    const M2 Di = inv(D);
    const M2 AD = mul(A, Di), CD = mul(C, Di);
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
      const double2 rl = cur[(i - s + N) % N], rr = cur[(i + s) % N];
      nxt[i] = sub2(sub2(cur[i], mv(AD, rl)), mv(CD, rr));
    }
    __syncthreads();
    double2* t = cur;
    cur = nxt;
    nxt = t;
    const M2 An = neg(mul(AD, A)), Cn = neg(mul(CD, C));
    D = sub(sub(D, mul(AD, C)), mul(CD, A));
    A = An;
    C = Cn;
  }
  // stride N/2: rows i and i + N/2 couple through E = A + C both ways
  const M2 E = add(A, C);
  const M2 Sp = inv(add(D, E)), Sm = inv(sub(D, E));
  const int H = N / 2;
  for (int i = threadIdx.x; i < H; i += blockDim.x) {
    const double2 s = mv(Sp, add2(cur[i], cur[i + H]));
    const double2 t = mv(Sm, sub2(cur[i], cur[i + H]));
    out[2 * i] = 0.5 * (s.x + t.x);
    out[2 * i + 1] = 0.5 * (s.y + t.y);
    out[2 * (i + H)] = 0.5 * (s.x - t.x);
    out[2 * (i + H) + 1] = 0.5 * (s.y - t.y);
  }
}

__global__ __launch_bounds__(kT) void k_hd_loop_combine(int ng, HdTable T,
                                                        const double* __restrict__ scratch,
                                                        double* __restrict__ z) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i >= ng) return;
  double v = scratch[(size_t)T.m * ng + i];
  for (int k = 0; k < T.m; ++k) v -= T.d[k] * T.q[k] * scratch[(size_t)k * ng + i];
  z[i] = v;
}

// ---- outer PCG on the trace (one block each) -------------------------------------------------

__global__ __launch_bounds__(kOneBlock) void k_hd_outer_alpha(int m, const double* __restrict__ p,
                                                              const double* __restrict__ y,
                                                              HdState* st) {
  if (st->o_done) return;
  double s = 0.0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) s += p[i] * y[i];
  s = block_sum(s);
  if (threadIdx.x == 0) {
    if (!(s > 0.0) || !isfinite(s)) {
      st->breakdown |= isfinite(s) ? 2 : 4;
      st->o_done = 1;
      st->o_alpha = 0.0;
    } else {
      st->o_alpha = st->o_rz / s;
    }
  }
}

__global__ __launch_bounds__(kOneBlock) void k_hd_outer_update(int m, const double* __restrict__ p,
                                                               const double* __restrict__ y,
                                                               double* __restrict__ x,
                                                               double* __restrict__ r,
                                                               HdState* st) {
  if (st->o_done) return;
  const double a = st->o_alpha;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    x[i] += a * p[i];
    r[i] -= a * y[i];
  }
}

__global__ __launch_bounds__(kOneBlock) void k_hd_outer_direction(int m, const double* __restrict__ r,
                                                                  const double* __restrict__ z,
                                                                  double* __restrict__ p,
                                                                  HdState* st, int first,
                                                                  double rtol2) {
  __shared__ double beta_s;
  __shared__ int skip;
  if (threadIdx.x == 0) skip = (!first && st->o_done) ? 1 : 0;
  __syncthreads();
  if (skip) return;
  double s = 0.0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) s += r[i] * z[i];
  const double rz = block_sum(s);
  if (threadIdx.x == 0) {
    double beta = 0.0;
    if (first) {
      st->o_rz0 = rz;
      st->o_its = 0;
      st->o_done = 0;
    } else {
      beta = rz / st->o_rz;
      st->o_its += 1;
    }
    if (!isfinite(rz) || rz < 0.0) {
      st->breakdown |= isfinite(rz) ? 2 : 4;
      st->o_done = 1;
    } else if (rz <= rtol2 * st->o_rz0) {
      st->o_done = 1;
    }
    st->o_rz = rz;
    beta_s = beta;
  }
  __syncthreads();
  const double beta = beta_s;
  for (int i = threadIdx.x; i < m; i += blockDim.x) p[i] = first ? z[i] : z[i] + beta * p[i];
}

// ---- true residual, copies --------------------------------------------------------------------

__global__ __launch_bounds__(kT) void k_hd_true_res(HdView A, const double* __restrict__ b,
                                                    const double* __restrict__ x,
                                                    double* __restrict__ partials) {
  double s = 0.0, t = 0.0;
  for (int i = blockIdx.x * kT + threadIdx.x; i < A.rows; i += gridDim.x * kT) {
    const double e = b[i] - ell_row(A, i, x);
    s += e * e;
    t += b[i] * b[i];
  }
  s = block_sum(s);
  t = block_sum(t);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = s;
    partials[kHdPartials + blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(kOneBlock) void k_hd_true_res_finish(const double* partials, int nb,
                                                                  HdState* st) {
  const double s = sum_partials(partials, nb);
  const double t = sum_partials(partials + kHdPartials, nb);
  if (threadIdx.x == 0) {
    st->t_res[0] = s;
    st->t_res[1] = t;
  }
}

__global__ __launch_bounds__(kT) void k_hd_scale(const double* __restrict__ a, double* __restrict__ b,
                                                 int n, double scale) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i < n) b[i] = scale * a[i];
}

}  // namespace

// ---- launchers -----------------------------------------------------------------------------------

void launch_hd_spmv(hipStream_t s, HdView A, const double* x, double* y, double alpha, double beta,
                    const HdState* stop) {
  if (A.rows == 0) return;
  hipLaunchKernelGGL(k_hd_spmv, dim3(row_blocks(A.rows)), dim3(kT), 0, s, A, x, y, alpha, beta,
                     stop);
}

void launch_hd_residual(hipStream_t s, HdView A, const double* b, const double* x, double* r,
                        const HdState* stop) {
  hipLaunchKernelGGL(k_hd_residual, dim3(row_blocks(A.rows)), dim3(kT), 0, s, A, b, x, r, stop);
}

void launch_hd_patch_solve(hipStream_t s, const HdLevel& L, const double* r, const HdState* stop) {
  // the patch stride is a template argument (12: H(div), 8: P2 velocity, 1: one-dof patches)
  auto go = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, dim3(blocks_for(L.nvert)), dim3(kT), 0, s, (const int*)L.dpatch,
                       (const int*)L.dptype, (const double*)L.dpinv, L.ntypes, L.nvert, r, L.Y,
                       stop);
  };
  if (L.pw == 1) go(k_hd_patch_solve<1>);
  else if (L.pw == 8) go(k_hd_patch_solve<8>);
  else go(k_hd_patch_solve<kHdPatch>);
}

void launch_hd_patch_sum(hipStream_t s, const HdLevel& L, double theta, double* x, int add,
                         const HdState* stop) {
  hipLaunchKernelGGL(k_hd_patch_sum, dim3(blocks_for(L.n0)), dim3(kT), 0, s, (const int*)L.dslot,
                     L.n0, (const double*)L.Y, theta, x, add, stop);
}

void launch_hd_cheb_step(hipStream_t s, const HdLevel& L, const double* b, const double* x_in,
                         double* x_out, double* d, double c_prev, double c_res, int first) {
  hipLaunchKernelGGL(k_hd_cheb_step, dim3(row_blocks(L.A.rows)), dim3(kT), 0, s, view(L.A),
                     (const int*)L.dptype, (const double*)L.dpinv, b, x_in, x_out, d, c_prev,
                     c_res, first);
}

void launch_hd_coarse(hipStream_t s, const double* C, int n0, const double* b, double* x,
                      const HdState* stop) {
  hipLaunchKernelGGL(k_hd_coarse, dim3((n0 + kT / 64 - 1) / (kT / 64)), dim3(kT), 0, s, C, n0, b, x,
                     stop);
}

void launch_hd_pcg_start(hipStream_t s, int n0, const double* f, double* u, double* r,
                         double* partials, HdState* st, double tol2) {
  const int nb = red_blocks(n0);
  hipLaunchKernelGGL(k_hd_pcg_start, dim3(nb), dim3(kT), 0, s, n0, f, u, r, partials);
  hipLaunchKernelGGL(k_hd_start_finish, dim3(1), dim3(kOneBlock), 0, s, (const double*)partials,
                     nb, st, tol2);
}

void launch_hd_pcg_rz(hipStream_t s, int n0, const double* r, const double* z, double* partials,
                      HdState* st, int first) {
  const int nb = red_blocks(n0);
  hipLaunchKernelGGL(k_hd_dot, dim3(nb), dim3(kT), 0, s, n0, r, z, partials, (const HdState*)st);
  hipLaunchKernelGGL(k_hd_rz_finish, dim3(1), dim3(kOneBlock), 0, s, (const double*)partials, nb,
                     st, first);
}

void launch_hd_pcg_pq(hipStream_t s, HdView A, const double* z, const double* p_old, double* p_new,
                      double* q, double* partials, HdState* st, int first) {
  const int nb = red_blocks(A.rows);
  hipLaunchKernelGGL(k_hd_pq, dim3(nb), dim3(kT), 0, s, A, z, p_old, p_new, q, partials,
                     (const HdState*)st, first);
  hipLaunchKernelGGL(k_hd_pq_finish, dim3(1), dim3(kOneBlock), 0, s, (const double*)partials, nb,
                     st);
}

void launch_hd_pcg_update(hipStream_t s, int n0, const double* p, const double* q, double* u,
                          double* r, double* partials, HdState* st) {
  const int nb = red_blocks(n0);
  hipLaunchKernelGGL(k_hd_update, dim3(nb), dim3(kT), 0, s, n0, p, q, u, r, partials,
                     (const HdState*)st);
  hipLaunchKernelGGL(k_hd_update_finish, dim3(1), dim3(kOneBlock), 0, s, (const double*)partials,
                     nb, st);
}

void launch_hd_loop_precond(hipStream_t s, int n, const HdLoopBlocks& blk, const HdTable& T,
                            const double* r, double* z, double* scratch) {
  hipLaunchKernelGGL(k_hd_loop_solve, dim3(T.m + 1), dim3(kOneBlock), 0, s, 4 * n, blk, T, r,
                     scratch);
  hipLaunchKernelGGL(k_hd_loop_combine, dim3(blocks_for(8 * n)), dim3(kT), 0, s, 8 * n, T,
                     (const double*)scratch, z);
}

void launch_hd_outer_alpha(hipStream_t s, int m, const double* p, const double* y, HdState* st) {
  hipLaunchKernelGGL(k_hd_outer_alpha, dim3(1), dim3(kOneBlock), 0, s, m, p, y, st);
}

void launch_hd_outer_update(hipStream_t s, int m, const double* p, const double* y, double* x,
                            double* r, HdState* st) {
  hipLaunchKernelGGL(k_hd_outer_update, dim3(1), dim3(kOneBlock), 0, s, m, p, y, x, r, st);
}

void launch_hd_outer_direction(hipStream_t s, int m, const double* r, const double* z, double* p,
                               HdState* st, int first, double rtol2) {
  hipLaunchKernelGGL(k_hd_outer_direction, dim3(1), dim3(kOneBlock), 0, s, m, r, z, p, st, first,
                     rtol2);
}

void launch_hd_true_residual(hipStream_t s, HdView A, const double* b, const double* x,
                             double* partials, HdState* st) {
  const int nb = red_blocks(A.rows);
  hipLaunchKernelGGL(k_hd_true_res, dim3(nb), dim3(kT), 0, s, A, b, x, partials);
  hipLaunchKernelGGL(k_hd_true_res_finish, dim3(1), dim3(kOneBlock), 0, s, (const double*)partials,
                     nb, st);
}

void launch_hd_scale(hipStream_t s, const double* a, double* b, int n, double scale) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_hd_scale, dim3(blocks_for(n)), dim3(kT), 0, s, a, b, n, scale);
}

}  // namespace fdd
