// Interior Dirichlet solve A_II u = f on the 2D P1 grid (5-point stencil 4, -1, -1, -1, -1),
// by multigrid-preconditioned CG, for gfx950.
//
// The interior block A_II is the leading block A^00 of the domain-decomposition operator
// (paper, Sec. 2, eq. (block_op)) divided by K.  The paper inverts it by LU (Sec. 3); here it is
// inverted iteratively:
//   - V-cycle: red-black Gauss-Seidel (red then black before the coarse correction, black then
//     red after, so the cycle is a symmetric operator), P1 interpolation on nested
//     diagonal-split meshes as prolongation, restriction = its transpose, and the same 5-point
//     stencil on every level (the Galerkin product of P1 interpolation reproduces it).
//   - The finest levels run as fused LDS-tiled kernels: one kernel per level going down
//     (pre-smooth from zero, residual, restriction) and one going up (prolongation + correction,
//     post-smooth).  Halo cells are recomputed redundantly so that a tile never waits on a
//     neighbour.  Levels with at most 63 x 63 points run in one workgroup entirely in LDS.
//   - The PCG vector updates are fused into the level-0 kernels; dot products are reduced
//     deterministically (per-block partials, the last block to arrive sums them in order).
//   - Scalars and convergence flags stay on the device; every kernel returns at once when its
//     solve has converged, so the host can enqueue a schedule without reading anything back.
#include "fdd_internal.h"

namespace fdd {

// --------------------------------------------------------------------------------------------
// helpers
// --------------------------------------------------------------------------------------------

__device__ __forceinline__ bool is_red(int i, int j) { return ((i + j) & 1) == 0; }

// Sum over the block (kBlock threads); result valid in thread 0.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double sh[kCoarseThreads / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (int)(blockDim.x >> 6);
    for (int w = 0; w < nw; ++w) s += sh[w];
  }
  return s;
}

// Stores this block's partial and reports whether the block is the last one to arrive.  In
// the last block, partials of all blocks are visible after the call.
__device__ __forceinline__ bool arrive(double partial, double* partials, unsigned* counter,
                                       unsigned nblocks, unsigned bid) {
  __shared__ int s_last;
  if (threadIdx.x == 0) {
    partials[bid] = partial;
    __threadfence();
    unsigned t = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    int last = (t == nblocks - 1);
    if (last) {
      __threadfence();
      __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    s_last = last;
  }
  __syncthreads();
  return s_last != 0;
}

// Fixed-order sum of the partials (call from every thread of the last block).
__device__ __forceinline__ double gather_partials(const double* partials, unsigned nblocks) {
  double v = 0.0;
  for (unsigned k = threadIdx.x; k < nblocks; k += blockDim.x)
    v += __builtin_nontemporal_load(partials + k);
  return block_sum(v);
}

__device__ __forceinline__ bool stopped(const DevState* st) {
  return (st->inner_done | st->solve_done) != 0;
}

template <typename T>
__device__ __forceinline__ T gload(const T* a, int pitch, int nf, int i, int j) {
  return (i >= 1 && i <= nf && j >= 1 && j <= nf) ? a[(size_t)(j - 1) * pitch + (i - 1)] : T(0);
}

// P1 interpolation from the coarse grid (nc points per side) to fine point (i, j).
template <typename T>
__device__ __forceinline__ T prolong(const T* ec, int pc, int nc, int i, int j) {
  const int I = i >> 1, J = j >> 1;
  if (!(i & 1) && !(j & 1)) return gload(ec, pc, nc, I, J);
  if ((i & 1) && !(j & 1)) return T(0.5) * (gload(ec, pc, nc, I, J) + gload(ec, pc, nc, I + 1, J));
  if (!(i & 1) && (j & 1)) return T(0.5) * (gload(ec, pc, nc, I, J) + gload(ec, pc, nc, I, J + 1));
  return T(0.5) * (gload(ec, pc, nc, I, J) + gload(ec, pc, nc, I + 1, J + 1));
}

// --------------------------------------------------------------------------------------------
// fused level kernels
// --------------------------------------------------------------------------------------------

// Going down one level: u = S^nu(0; f) (red first), r = f - A u, f_c = P^T r.
// CG = true (level 0 inside PCG): f is r_new = r_old - alpha q, computed on the window; the
// tile also updates x += alpha p on its own points, stores r_new, and reduces ||r_new||^2.
template <typename T, int NU, bool CG>
__global__ __launch_bounds__(kBlock) void k_mg_down(
    const T* __restrict__ fin, T* __restrict__ uout, T* __restrict__ fc, int nf, int pitch,
    int pc, const T* __restrict__ q, T* __restrict__ x, const T* __restrict__ p,
    T* __restrict__ rout, DevState* st, double* partials) {
  constexpr int H = 2 * NU + 1;
  constexpr int W = kTile + 2 * H;
  __shared__ T sf[W][W + 1];
  __shared__ T su[W][W + 1];
  if (stopped(st)) return;
  const int i0 = blockIdx.x * kTile, j0 = blockIdx.y * kTile;
  const int ib = i0 + 1 - H, jb = j0 + 1 - H;  // global index of window cell (0, 0)
  const int tid = threadIdx.x;
  T alpha = T(0);
  bool first = false;
  if (CG) {
    const double pq = st->pq, rho = st->rho;
    first = (st->pcg_k == 0);
    alpha = (pq > 0.0 && isfinite(pq)) ? (T)(rho / pq) : T(0);
  }
  double rr = 0.0;
  for (int idx = tid; idx < W * W; idx += kBlock) {
    const int li = idx % W, lj = idx / W;
    const int i = ib + li, j = jb + lj;
    T f = T(0);
    if (i >= 1 && i <= nf && j >= 1 && j <= nf) {
      const size_t o = (size_t)(j - 1) * pitch + (i - 1);
      if (CG) {
        f = fin[o] - alpha * q[o];
        if (li >= H && li < H + kTile && lj >= H && lj < H + kTile) {
          rout[o] = f;
          x[o] = first ? alpha * p[o] : x[o] + alpha * p[o];
          rr += (double)f * (double)f;
        }
      } else {
        f = fin[o];
      }
    }
    sf[lj][li] = f;
    // first red half-sweep from a zero iterate: u = f / 4 on red points, 0 on black points
    su[lj][li] = is_red(i, j) ? T(0.25) * f : T(0);
  }
  __syncthreads();
  // remaining half-sweeps: black, red, black, ...
  for (int s = 1; s < 2 * NU; ++s) {
    const bool red = !(s & 1);
    for (int idx = tid; idx < W * W; idx += kBlock) {
      const int li = idx % W, lj = idx / W;
      const int i = ib + li, j = jb + lj;
      if (li < 1 || li > W - 2 || lj < 1 || lj > W - 2) continue;
      if (is_red(i, j) != red || i < 1 || i > nf || j < 1 || j > nf) continue;
      su[lj][li] = T(0.25) * (sf[lj][li] + su[lj][li - 1] + su[lj][li + 1] + su[lj - 1][li] +
                              su[lj + 1][li]);
    }
    __syncthreads();
  }
  // residual, in place of f (each point reads its own f and the neighbours' u)
  for (int idx = tid; idx < W * W; idx += kBlock) {
    const int li = idx % W, lj = idx / W;
    if (li < 1 || li > W - 2 || lj < 1 || lj > W - 2) continue;
    sf[lj][li] = sf[lj][li] - (T(4) * su[lj][li] - su[lj][li - 1] - su[lj][li + 1] -
                               su[lj - 1][li] - su[lj + 1][li]);
  }
  __syncthreads();
  // restriction to the coarse points whose fine index 2I lies in this tile
  const int nc = (nf - 1) >> 1;
  constexpr int TC = kTile / 2;
  for (int idx = tid; idx < TC * TC; idx += kBlock) {
    const int a = idx % TC, b = idx / TC;
    const int I = (i0 >> 1) + 1 + a, J = (j0 >> 1) + 1 + b;
    if (I > nc || J > nc) continue;
    const int li = 2 * I - ib, lj = 2 * J - jb;
    const T v = sf[lj][li] + T(0.5) * (sf[lj][li - 1] + sf[lj][li + 1] + sf[lj - 1][li] +
                                       sf[lj + 1][li] + sf[lj - 1][li - 1] + sf[lj + 1][li + 1]);
    fc[(size_t)(J - 1) * pc + (I - 1)] = v;
  }
  // store the pre-smoothed iterate on own points
  for (int idx = tid; idx < kTile * kTile; idx += kBlock) {
    const int a = idx % kTile, b = idx / kTile;
    const int i = i0 + 1 + a, j = j0 + 1 + b;
    if (i > nf || j > nf) continue;
    uout[(size_t)(j - 1) * pitch + (i - 1)] = su[b + H][a + H];
  }
  if (CG) {
    const double tot = block_sum(rr);
    const unsigned nb = gridDim.x * gridDim.y, bid = blockIdx.y * gridDim.x + blockIdx.x;
    if (arrive(tot, partials, &st->counters[1], nb, bid)) {
      const double rr_all = gather_partials(partials, nb);
      if (threadIdx.x == 0) {
        st->rr = rr_all;
        st->inner_its += 1;
        st->pcg_k += 1;
        const double pq = st->pq;
        if (!(pq > 0.0) || !isfinite(pq) || !isfinite(rr_all)) {
          st->breakdown |= isfinite(rr_all) ? 1 : 4;
          st->inner_done = 1;
        } else if (rr_all <= st->tau2 * st->rr0) {
          st->inner_done = 1;
          if (st->pcg_is_final) st->solve_done = 1;  // FP64 mode: the PCG residual is the solve's residual
        }
      }
    }
  }
}

// Going up one level: u = u_pre + P e_c, then nu (black, red) pairs; result to eout.
// CG = true (level 0): also reduces r . z over own points (f is r, the result is z).
template <typename T, int NU, bool CG>
__global__ __launch_bounds__(kBlock) void k_mg_up(
    const T* __restrict__ fin, const T* __restrict__ upre, const T* __restrict__ ec,
    T* __restrict__ eout, int nf, int pitch, int pc, DevState* st, double* partials) {
  constexpr int H = 2 * NU;
  constexpr int W = kTile + 2 * H;
  __shared__ T sf[W][W + 1];
  __shared__ T su[W][W + 1];
  if (stopped(st)) return;
  const int i0 = blockIdx.x * kTile, j0 = blockIdx.y * kTile;
  const int ib = i0 + 1 - H, jb = j0 + 1 - H;
  const int nc = (nf - 1) >> 1;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < W * W; idx += kBlock) {
    const int li = idx % W, lj = idx / W;
    const int i = ib + li, j = jb + lj;
    T f = T(0), u = T(0);
    if (i >= 1 && i <= nf && j >= 1 && j <= nf) {
      const size_t o = (size_t)(j - 1) * pitch + (i - 1);
      f = fin[o];
      u = upre[o] + prolong(ec, pc, nc, i, j);
    }
    sf[lj][li] = f;
    su[lj][li] = u;
  }
  __syncthreads();
  for (int s = 0; s < 2 * NU; ++s) {
    const bool red = (s & 1);  // black first
    for (int idx = tid; idx < W * W; idx += kBlock) {
      const int li = idx % W, lj = idx / W;
      const int i = ib + li, j = jb + lj;
      if (li < 1 || li > W - 2 || lj < 1 || lj > W - 2) continue;
      if (is_red(i, j) != red || i < 1 || i > nf || j < 1 || j > nf) continue;
      su[lj][li] = T(0.25) * (sf[lj][li] + su[lj][li - 1] + su[lj][li + 1] + su[lj - 1][li] +
                              su[lj + 1][li]);
    }
    __syncthreads();
  }
  double rz = 0.0;
  for (int idx = tid; idx < kTile * kTile; idx += kBlock) {
    const int a = idx % kTile, b = idx / kTile;
    const int i = i0 + 1 + a, j = j0 + 1 + b;
    if (i > nf || j > nf) continue;
    const T z = su[b + H][a + H];
    eout[(size_t)(j - 1) * pitch + (i - 1)] = z;
    if (CG) rz += (double)sf[b + H][a + H] * (double)z;
  }
  if (CG) {
    const double tot = block_sum(rz);
    const unsigned nb = gridDim.x * gridDim.y, bid = blockIdx.y * gridDim.x + blockIdx.x;
    if (arrive(tot, partials, &st->counters[2], nb, bid)) {
      const double rz_all = gather_partials(partials, nb);
      if (threadIdx.x == 0) {
        st->rho_old = st->rho;
        st->rho = rz_all;
        if (!(rz_all > 0.0) || !isfinite(rz_all)) {
          // r = 0 exactly gives rho = 0: nothing left to do; otherwise an indefinite V-cycle
          if (rz_all != 0.0) st->breakdown |= isfinite(rz_all) ? 1 : 4;
          st->inner_done = 1;
        }
      }
    }
  }
}

// p_new = z + beta p_old (beta = rho / rho_old, 0 on the first iteration), q = A p_new, p.q.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pcg_spmv(const T* __restrict__ z,
                                                     const T* __restrict__ pold,
                                                     T* __restrict__ pnew, T* __restrict__ q,
                                                     int nf, int pitch, DevState* st,
                                                     double* partials) {
  constexpr int W = kTile + 2;
  __shared__ T sp[W][W + 1];
  if (stopped(st)) return;
  const bool first = (st->pcg_k == 0);
  const T beta = first ? T(0) : (T)(st->rho / st->rho_old);
  const int i0 = blockIdx.x * kTile, j0 = blockIdx.y * kTile;
  const int ib = i0, jb = j0;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < W * W; idx += kBlock) {
    const int li = idx % W, lj = idx / W;
    const int i = ib + li, j = jb + lj;
    T v = T(0);
    if (i >= 1 && i <= nf && j >= 1 && j <= nf) {
      const size_t o = (size_t)(j - 1) * pitch + (i - 1);
      v = first ? z[o] : z[o] + beta * pold[o];
    }
    sp[lj][li] = v;
  }
  __syncthreads();
  double pq = 0.0;
  for (int idx = tid; idx < kTile * kTile; idx += kBlock) {
    const int a = idx % kTile, b = idx / kTile;
    const int i = i0 + 1 + a, j = j0 + 1 + b;
    if (i > nf || j > nf) continue;
    const int li = a + 1, lj = b + 1;
    const T pv = sp[lj][li];
    const T qv = T(4) * pv - sp[lj][li - 1] - sp[lj][li + 1] - sp[lj - 1][li] - sp[lj + 1][li];
    const size_t o = (size_t)(j - 1) * pitch + (i - 1);
    pnew[o] = pv;
    q[o] = qv;
    pq += (double)pv * (double)qv;
  }
  const double tot = block_sum(pq);
  const unsigned nb = gridDim.x * gridDim.y, bid = blockIdx.y * gridDim.x + blockIdx.x;
  if (arrive(tot, partials, &st->counters[3], nb, bid)) {
    const double pq_all = gather_partials(partials, nb);
    if (threadIdx.x == 0) st->pq = pq_all;
  }
}

// --------------------------------------------------------------------------------------------
// coarse levels in one workgroup
// --------------------------------------------------------------------------------------------

template <typename T>
struct CoarseLds;  // sizes of the in-LDS hierarchy
template <>
struct CoarseLds<float> {
  static constexpr int kMaxNf = 63;
  static constexpr int kElems = 63 * 63 + 31 * 31 + 15 * 15 + 7 * 7 + 3 * 3 + 1 + 64;
};
template <>
struct CoarseLds<double> {
  static constexpr int kMaxNf = 31;
  static constexpr int kElems = 31 * 31 + 15 * 15 + 7 * 7 + 3 * 3 + 1 + 64;
};

template <typename T>
__device__ __forceinline__ T lds_at(const T* a, int nf, int i, int j) {
  return (i >= 1 && i <= nf && j >= 1 && j <= nf) ? a[(j - 1) * nf + (i - 1)] : T(0);
}

template <typename T>
__device__ void lds_halfsweep(T* u, const T* f, int nf, bool red) {
  const int npts = nf * nf;
  for (int k = threadIdx.x; k < npts; k += blockDim.x) {
    const int i = k % nf + 1, j = k / nf + 1;
    if (is_red(i, j) != red) continue;
    u[k] = T(0.25) * (f[k] + lds_at(u, nf, i - 1, j) + lds_at(u, nf, i + 1, j) +
                      lds_at(u, nf, i, j - 1) + lds_at(u, nf, i, j + 1));
  }
  __syncthreads();
}

// Levels first..nlev-1 entirely in LDS: V-cycle from the right-hand side fin (level `first`,
// global memory) to the result eout (global).  The coarsest level is solved exactly with the
// dense inverse cinv (nfc^2 x nfc^2, row-major).
template <typename T, int NU>
__global__ __launch_bounds__(kCoarseThreads) void k_coarse_vcycle(
    const T* __restrict__ fin, int pin, T* __restrict__ eout, LaunchLevels lv,
    const T* __restrict__ cinv, DevState* st) {
  __shared__ T buf[2 * CoarseLds<T>::kElems];
  if (stopped(st)) return;
  const int first = lv.first, last = lv.nlev - 1;
  T* uL[kMaxLevels];
  T* fL[kMaxLevels];
  {
    int off = 0;
    for (int l = first; l <= last; ++l) {
      const int np = lv.nf[l] * lv.nf[l];
      uL[l] = buf + off;
      off += np;
      fL[l] = buf + off;
      off += np;
    }
  }
  // load the right-hand side of the first in-LDS level
  {
    const int nf = lv.nf[first];
    for (int k = threadIdx.x; k < nf * nf; k += blockDim.x) {
      const int i = k % nf, j = k / nf;
      fL[first][k] = fin[(size_t)j * pin + i];
    }
  }
  __syncthreads();
  // down
  for (int l = first; l < last; ++l) {
    const int nf = lv.nf[l], nc = lv.nf[l + 1];
    T* u = uL[l];
    T* f = fL[l];
    for (int k = threadIdx.x; k < nf * nf; k += blockDim.x) {
      const int i = k % nf + 1, j = k / nf + 1;
      u[k] = is_red(i, j) ? T(0.25) * f[k] : T(0);
    }
    __syncthreads();
    for (int s = 1; s < 2 * NU; ++s) lds_halfsweep(u, f, nf, !(s & 1));
    // residual into the coarse right-hand side buffer's neighbour: compute on the fly
    T* fcb = fL[l + 1];
    for (int k = threadIdx.x; k < nc * nc; k += blockDim.x) {
      const int I = k % nc + 1, J = k / nc + 1;
      T acc = T(0);
      const int di[7] = {0, -1, 1, 0, 0, -1, 1};
      const int dj[7] = {0, 0, 0, -1, 1, -1, 1};
#pragma unroll
      for (int t = 0; t < 7; ++t) {
        const int i = 2 * I + di[t], j = 2 * J + dj[t];
        const T r = lds_at(f, nf, i, j) -
                    (T(4) * lds_at(u, nf, i, j) - lds_at(u, nf, i - 1, j) -
                     lds_at(u, nf, i + 1, j) - lds_at(u, nf, i, j - 1) - lds_at(u, nf, i, j + 1));
        acc += (t == 0 ? T(1) : T(0.5)) * r;
      }
      fcb[k] = acc;
    }
    __syncthreads();
  }
  // coarsest: exact solve with the dense inverse
  {
    const int nf = lv.nf[last];
    const int np = nf * nf;
    for (int k = threadIdx.x; k < np; k += blockDim.x) {
      T acc = T(0);
      for (int m = 0; m < np; ++m) acc += cinv[(size_t)k * np + m] * fL[last][m];
      uL[last][k] = acc;
    }
    __syncthreads();
  }
  // up
  for (int l = last - 1; l >= first; --l) {
    const int nf = lv.nf[l], nc = lv.nf[l + 1];
    T* u = uL[l];
    const T* ec = uL[l + 1];
    for (int k = threadIdx.x; k < nf * nf; k += blockDim.x) {
      const int i = k % nf + 1, j = k / nf + 1;
      const int I = i >> 1, J = j >> 1;
      T e;
      if (!(i & 1) && !(j & 1)) e = lds_at(ec, nc, I, J);
      else if ((i & 1) && !(j & 1)) e = T(0.5) * (lds_at(ec, nc, I, J) + lds_at(ec, nc, I + 1, J));
      else if (!(i & 1) && (j & 1)) e = T(0.5) * (lds_at(ec, nc, I, J) + lds_at(ec, nc, I, J + 1));
      else e = T(0.5) * (lds_at(ec, nc, I, J) + lds_at(ec, nc, I + 1, J + 1));
      u[k] += e;
    }
    __syncthreads();
    for (int s = 0; s < 2 * NU; ++s) lds_halfsweep(u, fL[l], nf, (s & 1));
  }
  {
    const int nf = lv.nf[first];
    for (int k = threadIdx.x; k < nf * nf; k += blockDim.x) {
      const int i = k % nf, j = k / nf;
      eout[(size_t)j * pin + i] = uL[first][k];
    }
  }
}

// --------------------------------------------------------------------------------------------
// FP64 residual of the interior solve (iterative refinement) and right-hand side set-up
// --------------------------------------------------------------------------------------------

__device__ __forceinline__ double rhs_at(const RhsDesc& f, int nf, int i, int j) {
  double v = 0.0;
  if (f.b) v = f.sb * f.b[(size_t)(j - 1) * nf + (i - 1)];
  if (f.g && j == nf) v += f.sg * f.g[i - 1];
  return v;
}

// u_out = u_in + e (u_in = 0 on the first call), r = f - A u_out (written as FP32 or FP64),
// ||r||^2 reduced in FP64; the last block updates the refinement state.
template <typename E>
__global__ __launch_bounds__(kBlock) void k_ir_residual(RhsDesc f, const double* __restrict__ u0,
                                                        const double* __restrict__ u1,
                                                        const E* __restrict__ e,
                                                        double* __restrict__ w0,
                                                        double* __restrict__ w1,
                                                        float* __restrict__ r32,
                                                        double* __restrict__ r64, int nf,
                                                        int pitch, int first, double tol2,
                                                        double tau2, int pcg_is_final,
                                                        DevState* st, double* partials) {
  constexpr int W = kTile + 2;
  __shared__ double su[W][W + 1];
  if (!first && st->solve_done) return;
  const int cur = st->refine_steps & 1;  // parity selects the current buffer
  const double* uin = first ? nullptr : (cur ? u1 : u0);
  double* uout = first ? w0 : (cur ? w0 : w1);
  const int i0 = blockIdx.x * kTile, j0 = blockIdx.y * kTile;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < W * W; idx += kBlock) {
    const int li = idx % W, lj = idx / W;
    const int i = i0 + li, j = j0 + lj;
    double v = 0.0;
    if (i >= 1 && i <= nf && j >= 1 && j <= nf && !first) {
      const size_t o = (size_t)(j - 1) * pitch + (i - 1);
      v = uin[o] + (e ? (double)e[o] : 0.0);
    }
    su[lj][li] = v;
  }
  __syncthreads();
  double rr = 0.0;
  for (int idx = tid; idx < kTile * kTile; idx += kBlock) {
    const int a = idx % kTile, b = idx / kTile;
    const int i = i0 + 1 + a, j = j0 + 1 + b;
    if (i > nf || j > nf) continue;
    const int li = a + 1, lj = b + 1;
    const double u = su[lj][li];
    const double r = rhs_at(f, nf, i, j) -
                     (4.0 * u - su[lj][li - 1] - su[lj][li + 1] - su[lj - 1][li] - su[lj + 1][li]);
    const size_t o = (size_t)(j - 1) * pitch + (i - 1);
    uout[o] = u;
    if (r32) r32[o] = (float)r;
    if (r64) r64[o] = r;
    rr += r * r;
  }
  const double tot = block_sum(rr);
  const unsigned nb = gridDim.x * gridDim.y, bid = blockIdx.y * gridDim.x + blockIdx.x;
  if (arrive(tot, partials, &st->counters[4], nb, bid)) {
    const double res = gather_partials(partials, nb);
    if (threadIdx.x == 0) {
      if (first) {
        st->tol2 = tol2;
        st->tau2 = tau2;
        st->pcg_is_final = pcg_is_final;
        st->breakdown = 0;
        st->ff = res;
        st->refine_steps = 0;
        st->inner_its = 0;
        st->solve_done = (res == 0.0) ? 1 : 0;
      } else {
        st->refine_steps += 1;
      }
      st->res2 = res;
      st->rr0 = res;
      st->pcg_k = 0;
      st->inner_done = 0;
      if (!isfinite(res)) {
        st->breakdown |= 4;
        st->solve_done = 1;
      } else if (res <= st->tol2 * st->ff) {
        st->solve_done = 1;
      }
    }
  }
}

// --------------------------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------------------------

static inline dim3 tiles(int nf) {
  const int t = (nf + kTile - 1) / kTile;
  return dim3(t, t);
}

template <typename T, int NU>
static void vcycle_tail_nu(const LaunchCtx& c, const MGBuffers<T>& mg) {
  // levels 1 .. first_coarse-1 go down, the coarse kernel, then back up to level 1
  const int fc = c.first_coarse;
  for (int l = 1; l < fc; ++l) {
    const Level& L = c.lev[l];
    hipLaunchKernelGGL((k_mg_down<T, NU, false>), tiles(L.nf), dim3(kBlock), 0, c.stream,
                       mg.f[l], mg.u[l], mg.f[l + 1], L.nf, L.pitch, c.lev[l + 1].pitch,
                       (const T*)nullptr, (T*)nullptr, (const T*)nullptr, (T*)nullptr, c.st,
                       c.partials);
  }
  LaunchLevels lv;
  lv.first = fc;
  lv.nlev = c.nlev;
  for (int l = 0; l < c.nlev; ++l) lv.nf[l] = c.lev[l].nf;
  const T* cinv = nullptr;
  if constexpr (sizeof(T) == 4) cinv = (const T*)c.coarse_inv;
  else cinv = (const T*)c.coarse_inv64;
  hipLaunchKernelGGL((k_coarse_vcycle<T, NU>), dim3(1), dim3(kCoarseThreads), 0, c.stream,
                     mg.f[fc], c.lev[fc].pitch, mg.e[fc], lv, cinv, c.st);
  for (int l = fc - 1; l >= 1; --l) {
    const Level& L = c.lev[l];
    hipLaunchKernelGGL((k_mg_up<T, NU, false>), tiles(L.nf), dim3(kBlock), 0, c.stream, mg.f[l],
                       mg.u[l], mg.e[l + 1], mg.e[l], L.nf, L.pitch, c.lev[l + 1].pitch, c.st,
                       c.partials);
  }
}

template <typename T>
void launch_vcycle_tail(const LaunchCtx& c, const MGBuffers<T>& mg) {
  if (c.nu == 2) vcycle_tail_nu<T, 2>(c, mg);
  else vcycle_tail_nu<T, 1>(c, mg);
}

template <typename T, int NU>
static void pcg_init_nu(const LaunchCtx& c, const MGBuffers<T>& mg, const T* r, T* z) {
  const Level& L = c.lev[0];
  hipLaunchKernelGGL((k_mg_down<T, NU, false>), tiles(L.nf), dim3(kBlock), 0, c.stream, r,
                     mg.u[0], mg.f[1], L.nf, L.pitch, c.lev[1].pitch, (const T*)nullptr,
                     (T*)nullptr, (const T*)nullptr, (T*)nullptr, c.st, c.partials);
  launch_vcycle_tail<T>(c, mg);
  hipLaunchKernelGGL((k_mg_up<T, NU, true>), tiles(L.nf), dim3(kBlock), 0, c.stream, r, mg.u[0],
                     mg.e[1], z, L.nf, L.pitch, c.lev[1].pitch, c.st, c.partials);
}

template <typename T>
void launch_pcg_init(const LaunchCtx& c, const MGBuffers<T>& mg, const T* r, T* z) {
  if (c.nu == 2) pcg_init_nu<T, 2>(c, mg, r, z);
  else pcg_init_nu<T, 1>(c, mg, r, z);
}

template <typename T, int NU>
static void pcg_iter_nu(const LaunchCtx& c, const MGBuffers<T>& mg, T* x, T* r_old, T* r_new,
                        T* z, T* p_old, T* p_new, T* q) {
  const Level& L = c.lev[0];
  hipLaunchKernelGGL((k_pcg_spmv<T>), tiles(L.nf), dim3(kBlock), 0, c.stream, z, p_old, p_new, q,
                     L.nf, L.pitch, c.st, c.partials);
  hipLaunchKernelGGL((k_mg_down<T, NU, true>), tiles(L.nf), dim3(kBlock), 0, c.stream, r_old,
                     mg.u[0], mg.f[1], L.nf, L.pitch, c.lev[1].pitch, (const T*)q, x,
                     (const T*)p_new, r_new, c.st, c.partials);
  launch_vcycle_tail<T>(c, mg);
  hipLaunchKernelGGL((k_mg_up<T, NU, true>), tiles(L.nf), dim3(kBlock), 0, c.stream, r_new,
                     mg.u[0], mg.e[1], z, L.nf, L.pitch, c.lev[1].pitch, c.st, c.partials);
}

template <typename T>
void launch_pcg_iteration(const LaunchCtx& c, const MGBuffers<T>& mg, T* x, T* r_old, T* r_new,
                          T* z, T* p_old, T* p_new, T* q) {
  if (c.nu == 2) pcg_iter_nu<T, 2>(c, mg, x, r_old, r_new, z, p_old, p_new, q);
  else pcg_iter_nu<T, 1>(c, mg, x, r_old, r_new, z, p_old, p_new, q);
}

void launch_ir_residual(const LaunchCtx& c, const RhsDesc& f, const double* u0, const double* u1,
                        const float* e32, const double* e64, double* w0, double* w1, float* r32,
                        double* r64, int first, double tol2, double tau2, int pcg_is_final) {
  const Level& L = c.lev[0];
  if (e64 || !e32)
    hipLaunchKernelGGL((k_ir_residual<double>), tiles(L.nf), dim3(kBlock), 0, c.stream, f, u0,
                       u1, e64, w0, w1, r32, r64, L.nf, L.pitch, first, tol2, tau2, pcg_is_final,
                       c.st, c.partials);
  else
    hipLaunchKernelGGL((k_ir_residual<float>), tiles(L.nf), dim3(kBlock), 0, c.stream, f, u0, u1,
                       e32, w0, w1, r32, r64, L.nf, L.pitch, first, tol2, tau2, pcg_is_final,
                       c.st, c.partials);
}

template void launch_pcg_init<float>(const LaunchCtx&, const MGBuffers<float>&, const float*,
                                     float*);
template void launch_pcg_init<double>(const LaunchCtx&, const MGBuffers<double>&, const double*,
                                      double*);
template void launch_pcg_iteration<float>(const LaunchCtx&, const MGBuffers<float>&, float*,
                                          float*, float*, float*, float*, float*, float*);
template void launch_pcg_iteration<double>(const LaunchCtx&, const MGBuffers<double>&, double*,
                                           double*, double*, double*, double*, double*, double*);

}  // namespace fdd
