// The 3D solver's kernels (unit cube, Kuhn tetrahedra, Gamma the face z = 1) for gfx950: interface
// work in FP64, the interior multigrid-PCG in FP32 (inside FP64 refinement) or FP64.
//
// Interior block: on the uniform Kuhn mesh the P1 stiffness of an interior node is h times the
// 7-point stencil (6, -1 x 6), so A_II = h L7 and every interior solve is a solve with L7.  It
// runs by multigrid-preconditioned CG: red-black Gauss-Seidel (red then black before the coarse
// correction, black then red after), P1 interpolation between nested Kuhn meshes (a fine node at
// 2I + d, d in {0,1}^3, takes the mean of the coarse nodes I and I + d: every such d is an edge
// direction of the Kuhn mesh), restriction = its transpose times 1/2 (the Galerkin coarse
// operator P^T L7 P is 2 L7), and a dense inverse on the coarsest grid.  Grids are stored with a
// one-cell zero border, (nf + 2)^3 cells, x fastest, so stencils need no bounds tests.  The
// passes are fused so that one PCG iteration takes few launches: the PCG update with the first
// two half-sweeps, the residual with the restriction, the prolongation with the first sweep
// after it, and every level of at most 15^3 points inside one workgroup.
//
// Interface: A_G is the 2D 5-point stencil on the (n-1)^2 face nodes and M_G the consistent P1
// mass of the face triangles, (h^2 / 12) (6, 1 on the x, y and (1,1) diagonal neighbours).  The
// shifted systems (alpha A_G + beta M_G) y = r of the rational approximation (eq. (RA)) are
// solved all at once (one grid dimension per system) by CG preconditioned with the operator in
// which M_G is replaced by its part diagonal in the sine basis; that preconditioner is applied
// as S D S with S the orthonormal DST-I matrix (batched dense FP64 GEMMs), or, when
// nf = 2^K - 1, as a transform along x, tridiagonal solves along y and the inverse transform.
//
// Scalars of the Krylov methods live on the device; dot products are summed from per-block
// partials in a fixed order (deterministic).
#include <hip/hip_runtime.h>

#include "k3_internal.h"

namespace fdd {

constexpr int kB3 = 256;

__device__ __forceinline__ double block_sum3(double v) {
  __shared__ double sh[kB3 / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kB3 / 64; ++w) s += sh[w];
  return s;  // valid in thread 0
}

// interior point q (0-based, x fastest) of an nf^3 grid -> padded index
__device__ __forceinline__ size_t pidx(int64_t q, int nf, int* i, int* j, int* k) {
  *i = (int)(q % nf) + 1;
  const int64_t r = q / nf;
  *j = (int)(r % nf) + 1;
  *k = (int)(r / nf) + 1;
  const size_t P = (size_t)nf + 2;
  return ((size_t)(*k) * P + (size_t)(*j)) * P + (size_t)(*i);
}

// ---- multigrid -------------------------------------------------------------------------------
// The level kernels run 64 x 4 threads (one wavefront per row of the block); block (bx, by)
// covers plane k = by + 1, rows bx * rows + 1 .. (bx + 1) * rows and every column, so the
// points need no index division and the partials of a reduction kernel number
// ceil(nf / rows) * nf.

constexpr int kX3 = 64, kY3 = 4;

template <typename Fn>
__device__ __forceinline__ void for_points(int nf, int rows, Fn&& fn) {
  const int k = blockIdx.y + 1;
  const int jb = blockIdx.x * rows;
  const int je = min(jb + rows, nf);
  for (int j = jb + 1 + (int)threadIdx.y; j <= je; j += kY3)
    for (int i = 1 + (int)threadIdx.x; i <= nf; i += kX3) fn(i, j, k);
}

__device__ __forceinline__ int tid3() { return (int)(threadIdx.y * kX3 + threadIdx.x); }
__device__ __forceinline__ bool lead3() {
  return blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0 && threadIdx.y == 0;
}

// Sum over the block in a fixed order, broadcast to every thread.
__device__ __forceinline__ double bsum3(double v) {
  __shared__ double sh[kY3 + 1];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  __syncthreads();
  if (threadIdx.x == 0) sh[threadIdx.y] = v;
  __syncthreads();
  if (tid3() == 0) {
    double s = 0.0;
    for (int w = 0; w < kY3; ++w) s += sh[w];
    sh[kY3] = s;
  }
  __syncthreads();
  return sh[kY3];
}

// Sum of np block partials (written by an earlier kernel), the same in every block.
// (a thread's partials q = tid, tid + B, ... are added in that order, eight loads in flight at a
// time: a loop adding each value as it arrives waits once per partial)
template <int B>
__device__ __forceinline__ double thread_partials(const double* __restrict__ part, int np, int t,
                                                  int stride) {
  constexpr int U = 8;
  double a = 0.0;
  for (int q0 = t; q0 < np; q0 += U * B) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = q0 + u * B;
      v[u] = q < np ? part[(size_t)q * stride] : 0.0;
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (q0 + u * B < np) a += v[u];
  }
  return a;
}

__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int np) {
  return bsum3(thread_partials<kX3 * kY3>(part, np, tid3(), 1));
}

__device__ __forceinline__ void put_partial(double* part, double v) {
  v = bsum3(v);
  if (tid3() == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = v;
}

__device__ __forceinline__ bool is_red3(int i, int j, int k) { return ((i + j + k) & 1) == 0; }

// Convergence bookkeeping of the interior solve, done by the first kernel after the residual
// update (every block sums the same partials and takes the same decision; the lead block
// records it).  mode 1: start of a run, the partials are |r_0|^2 of its right-hand side (on the
// first run |F|^2, recorded as F2; on later runs the FP64 refinement residual, which ends the
// solve once |r_0|^2 <= tol2s F2; r_0 = 0 ends it too); mode 2: the partials are |r_{k+1}|^2
// (its += 1; the run stops at |r|^2 <= max(tol2 ff, tol2s F2)).
__device__ __forceinline__ bool k3_check(State3* st, int* stop, const double* part, int np,
                                         int mode) {
  const double a = sum_partials(part, np);
  const bool bad = !isfinite(a);
  bool halt;
  if (mode == 1) {
    const bool first = st->run == 0;
    const bool solved = a == 0.0 || (!first && a <= st->tol2s * st->F2);
    halt = bad || solved;
    if (lead3()) {
      if (first) st->F2 = a;
      st->ff = a;
      st->rr = a;
      st->its = 0;
      if (bad) st->breakdown |= 4;
      if (solved) st->done = 1;
      if (halt) *stop = 1;
    }
  } else {
    halt = bad || a <= fmax(st->tol2 * st->ff, st->tol2s * st->F2);
    if (lead3()) {
      st->rr = a;
      st->its += 1;
      st->its_total += 1;
      if (bad) st->breakdown |= 4;
      if (halt) *stop = 1;
    }
  }
  return halt;
}

// Going down, first two half-sweeps from u = 0 (red, then black) in one pass: u = f / 6 on red
// points and, on black points, (f + sum of the six red neighbours' f / 6) / 6.
// MODE 0: f given.  MODE 1 (level 0, start of a run): also partials of |f|^2.
// MODE 2 (level 0, PCG iteration k): alpha_k = rho_k / (p_k . A p_k) from the partials of the
// previous kernel, f = r_{k+1} = r_k - alpha_k q formed on the fly (q = A p_k), r_{k+1} stored,
// x += alpha_k p_k, partials of |r_{k+1}|^2.  R: the working precision (partials in FP64).
template <typename R, int MODE>
__global__ __launch_bounds__(kX3* kY3) void k3_zp(const R* __restrict__ f, R* __restrict__ u,
                                                   int nf, int rows, const R* __restrict__ qv,
                                                   R* __restrict__ rnew, R* __restrict__ x,
                                                   const R* __restrict__ p, State3* st,
                                                   const double* __restrict__ pin, int np,
                                                   double* __restrict__ part, int* stop) {
  if (*stop) return;
  R al = R(0);
  if constexpr (MODE == 2) {
    const double pq = sum_partials(pin, np);
    if (!(pq > 0.0) || !isfinite(pq)) {
      if (lead3()) {
        st->breakdown |= isfinite(pq) ? 1 : 4;
        *stop = 1;
      }
      return;
    }
    al = R(st->rho[st->its & 1] / pq);
  }
  const int P = nf + 2, PP = P * P;
  const R sixth = R(1) / R(6);
  auto F = [&](int o) -> R {
    if constexpr (MODE == 2) return f[o] - al * qv[o];
    else return f[o];
  };
  double acc = 0.0;
  for_points(nf, rows, [&](int i, int j, int k) {
    const int o = (k * P + j) * P + i;
    const R fo = F(o);
    R v;
    if (is_red3(i, j, k)) {
      v = fo * sixth;
    } else {
      const R s = F(o - 1) + F(o + 1) + F(o - P) + F(o + P) + F(o - PP) + F(o + PP);
      v = (fo + s * sixth) * sixth;
    }
    u[o] = v;
    if constexpr (MODE == 2) {
      rnew[o] = fo;
      x[o] += al * p[o];
    }
    acc += (double)fo * (double)fo;
  });
  if constexpr (MODE != 0) put_partial(part, acc);
}

// Half-sweep of one colour (red: i + j + k even) of L7 u = f, in place; check != 0: first the
// convergence bookkeeping of k3_check.
template <typename R>
__global__ __launch_bounds__(kX3* kY3) void k3_hs(R* __restrict__ u, const R* __restrict__ f,
                                                   int nf, int rows, int red, int check,
                                                   State3* st, const double* __restrict__ pin,
                                                   int np, int* stop) {
  if (*stop) return;
  if (check && k3_check(st, stop, pin, np, check)) return;
  const int P = nf + 2, PP = P * P;
  const int want = red ? 0 : 1;
  const R sixth = R(1) / R(6);
  for_points(nf, rows, [&](int i, int j, int k) {
    if (((i + j + k) & 1) != want) return;
    const int o = (k * P + j) * P + i;
    u[o] = (f[o] + u[o - 1] + u[o + 1] + u[o - P] + u[o + P] + u[o - PP] + u[o + PP]) * sixth;
  });
}

// Residual and restriction in one pass: f_c(I) = 1/2 [t(2I) + 1/2 sum over the 14 Kuhn-edge
// neighbours 2I +- d of t], t = f - L7 u formed where it is read (every such fine point is
// interior).  Grid over the coarse points; check as in k3_hs.
template <typename R>
__global__ __launch_bounds__(kX3* kY3) void k3_rr(const R* __restrict__ u, const R* __restrict__ f,
                                                   R* __restrict__ fc, int nf, int nc, int rows,
                                                   int check, State3* st,
                                                   const double* __restrict__ pin, int np,
                                                   int* stop) {
  if (*stop) return;
  if (check && k3_check(st, stop, pin, np, check)) return;
  const int P = nf + 2, PP = P * P, Pc = nc + 2;
  auto res = [&](int o) {
    return f[o] - (R(6) * u[o] - u[o - 1] - u[o + 1] - u[o - P] - u[o + P] - u[o - PP] -
                   u[o + PP]);
  };
  for_points(nc, rows, [&](int I, int J, int K) {
    const int o = ((2 * K) * P + 2 * J) * P + 2 * I;
    // Kuhn edge directions: e1, e2, e3, e1+e2, e1+e3, e2+e3, e1+e2+e3
    const int d1 = 1, d2 = P, d3 = PP;
    const R s = res(o + d1) + res(o - d1) + res(o + d2) + res(o - d2) + res(o + d3) +
                res(o - d3) + res(o + d1 + d2) + res(o - d1 - d2) + res(o + d1 + d3) +
                res(o - d1 - d3) + res(o + d2 + d3) + res(o - d2 - d3) + res(o + d1 + d2 + d3) +
                res(o - d1 - d2 - d3);
    fc[(K * Pc + J) * Pc + I] = R(0.5) * (res(o) + R(0.5) * s);
  });
}

// Going up: v = u + P e_c (a fine node at 2I + d, d in {0,1}^3, takes the mean of the coarse
// nodes I and I + d), then the first black half-sweep on v, in one pass into uo (uo != u:
// the black points read their red neighbours' v, formed where they are read).
template <typename R>
__global__ __launch_bounds__(kX3* kY3) void k3_pr(const R* __restrict__ u,
                                                   const R* __restrict__ ec,
                                                   const R* __restrict__ f, R* __restrict__ uo,
                                                   int nf, int nc, int rows, int* stop) {
  if (*stop) return;
  const int P = nf + 2, Pc = nc + 2;
  const R sixth = R(1) / R(6);
  // valid on the zero border too: the coarse nodes read there lie on the coarse border
  auto V = [&](int i, int j, int k) {
    const int I = i >> 1, J = j >> 1, K = k >> 1;
    const int oc = (K * Pc + J) * Pc + I;
    const int od = ((k & 1) * Pc + (j & 1)) * Pc + (i & 1);
    const R e = od ? R(0.5) * (ec[oc] + ec[oc + od]) : ec[oc];
    return u[(k * P + j) * P + i] + e;
  };
  for_points(nf, rows, [&](int i, int j, int k) {
    const int o = (k * P + j) * P + i;
    R v;
    if (is_red3(i, j, k)) {
      v = V(i, j, k);
    } else {
      v = (f[o] + V(i - 1, j, k) + V(i + 1, j, k) + V(i, j - 1, k) + V(i, j + 1, k) +
           V(i, j, k - 1) + V(i, j, k + 1)) *
          sixth;
    }
    uo[o] = v;
  });
}

// Last half-sweep of the V-cycle on level 0 (red) with the partials of r . z (f = r, z = u).
template <typename R>
__global__ __launch_bounds__(kX3* kY3) void k3_hsz(R* __restrict__ u, const R* __restrict__ f,
                                                    int nf, int rows, double* __restrict__ part,
                                                    int* stop) {
  if (*stop) return;
  const int P = nf + 2, PP = P * P;
  const R sixth = R(1) / R(6);
  double acc = 0.0;
  for_points(nf, rows, [&](int i, int j, int k) {
    const int o = (k * P + j) * P + i;
    R z = u[o];
    if (is_red3(i, j, k)) {
      z = (f[o] + u[o - 1] + u[o + 1] + u[o - P] + u[o + P] + u[o - PP] + u[o + PP]) * sixth;
      u[o] = z;
    }
    acc += (double)f[o] * (double)z;
  });
  put_partial(part, acc);
}

// PCG iteration k, first pass: rho_k = r_k . z_k from the partials of the V-cycle,
// beta_k = rho_k / rho_{k-1} (beta_0 = 0), p_k = z_k + beta_k p_{k-1} (stored; also formed at
// the neighbours), q = L7 p_k, partials of p_k . q.  rho_k is recorded in st->rho[k & 1].
template <typename R>
__global__ __launch_bounds__(kX3* kY3) void k3_apply1(const R* __restrict__ z,
                                                       const R* __restrict__ pold,
                                                       R* __restrict__ pnew, R* __restrict__ qv,
                                                       int nf, int rows, State3* st,
                                                       const double* __restrict__ pin, int np,
                                                       double* __restrict__ part, int* stop) {
  if (*stop) return;
  const double rz = sum_partials(pin, np);
  const int it = st->its;
  if (!(rz > 0.0) || !isfinite(rz)) {
    if (lead3()) {
      st->breakdown |= isfinite(rz) ? 1 : 4;
      *stop = 1;
    }
    return;
  }
  const R beta = it ? R(rz / st->rho[(it - 1) & 1]) : R(0);
  if (lead3()) st->rho[it & 1] = rz;
  const int P = nf + 2, PP = P * P;
  auto PV = [&](int o) { return it ? z[o] + beta * pold[o] : z[o]; };
  double acc = 0.0;
  for_points(nf, rows, [&](int i, int j, int k) {
    const int o = (k * P + j) * P + i;
    const R pv = PV(o);
    const R q = R(6) * pv - PV(o - 1) - PV(o + 1) - PV(o - P) - PV(o + P) - PV(o - PP) -
                PV(o + PP);
    pnew[o] = pv;
    qv[o] = q;
    acc += (double)pv * (double)q;
  });
  put_partial(part, acc);
}

// FP64 iterative refinement around the working-precision PCG (level 0, padded grids):
// FIRST: r = F (x = 0); otherwise x' = x + e (formed at the neighbours too) is stored,
// r = F - L7 x' (FP64) and the refinement step count st->run is advanced.  r is stored in the
// working precision as the next run's right-hand side and the partials of |r|^2 (FP64) go to
// part.
template <bool FIRST>
__global__ __launch_bounds__(kX3* kY3) void k3_ir(const double* __restrict__ F,
                                                   const double* __restrict__ xin,
                                                   const float* __restrict__ e,
                                                   double* __restrict__ xout,
                                                   float* __restrict__ r32, int nf, int rows,
                                                   State3* st, double* __restrict__ part) {
  if (!FIRST && lead3()) {
    if (st->run < kRuns3) st->run_its[st->run] = st->its;
    st->run += 1;
  }
  const int P = nf + 2, PP = P * P;
  auto X = [&](int o) { return xin[o] + (double)e[o]; };
  double acc = 0.0;
  for_points(nf, rows, [&](int i, int j, int k) {
    const int o = (k * P + j) * P + i;
    double r;
    if constexpr (FIRST) {
      r = F[o];
    } else {
      const double xo = X(o);
      xout[o] = xo;
      r = F[o] - (6.0 * xo - X(o - 1) - X(o + 1) - X(o - P) - X(o + P) - X(o - PP) - X(o + PP));
    }
    r32[o] = (float)r;
    acc += r * r;
  });
  put_partial(part, acc);
}

// Coarse part of the V-cycle in one workgroup: the levels lev[0] > lev[1] > ... > lev[nl - 1]
// (lev[0] <= kCvcMax) held in LDS, the same smoothing, transfers and dense inverse on the
// coarsest grid as the level kernels; f of the first level from fin, its result to uout.
constexpr int kCvcThreads = 1024;
constexpr int kCvcLds = 11600;  // elements: u and f of 15, 7, 3 and 1 (padded)
constexpr int kCvcDense = 729;  // dense coarsest inverses up to 3^3 unknowns are staged in LDS

// Thread t of the workgroup takes the points (i, j, k) = (t % 16, (t / 16) % 16, t / 256 + 4 m)
// + 1 of a level (every level it holds has at most 15 points a side).
template <typename Fn>
__device__ __forceinline__ void cvc_points(int nf, Fn&& fn) {
  const int t = threadIdx.x;
  const int i = (t & 15) + 1, j = ((t >> 4) & 15) + 1;
  if (i > nf || j > nf) return;
  for (int k = (t >> 8) + 1; k <= nf; k += kCvcThreads / 256) fn(i, j, k);
}

template <typename R>
__global__ __launch_bounds__(kCvcThreads) void k3_cvc(const R* __restrict__ fin,
                                                       R* __restrict__ uout, Cvc3 L,
                                                       const double* __restrict__ cinv, int nu,
                                                       const int* __restrict__ stop) {
  if (*stop) return;
  __shared__ R lds[kCvcLds];
  __shared__ R tr[(kCvcMax + 2) * (kCvcMax + 2) * (kCvcMax + 2)];  // residual of a level
  const R sixth = R(1) / R(6);
  const int t = threadIdx.x;
  // level l: u at U[l], f at Fv[l] (the loops over levels are unrolled: static indices)
  R* U[kCvcLevels];
  R* Fv[kCvcLevels];
  int ed[kCvcLevels];
  int tot = 0;
#pragma unroll
  for (int l = 0; l < kCvcLevels; ++l) {
    ed[l] = l < L.nl ? L.lev[l] : 0;
    const int v = (ed[l] + 2) * (ed[l] + 2) * (ed[l] + 2);
    U[l] = lds + tot;
    Fv[l] = lds + tot + v;
    tot += l < L.nl ? 2 * v : 0;
  }
  for (int q = t; q < tot; q += kCvcThreads) lds[q] = R(0);
  // the dense inverse of the coarsest grid, staged in LDS when it is small (<= 27^2 entries)
  __shared__ double sC[kCvcDense];
  const int npc = ed[L.nl - 1] * ed[L.nl - 1] * ed[L.nl - 1];
  const bool staged = npc * npc <= kCvcDense;
  if (staged)
    for (int q = t; q < npc * npc; q += kCvcThreads) sC[q] = cinv[q];
  const double* C = staged ? sC : cinv;
  __syncthreads();
  {
    const int P = ed[0] + 2;
    cvc_points(ed[0], [&](int i, int j, int k) {
      const int o = (k * P + j) * P + i;
      Fv[0][o] = fin[o];
    });
  }
  __syncthreads();
  auto half = [&](R* u, const R* f, int nf, int want) {
    const int P = nf + 2, PP = P * P;
    cvc_points(nf, [&](int i, int j, int k) {
      if (((i + j + k) & 1) != want) return;
      const int o = (k * P + j) * P + i;
      u[o] = (f[o] + u[o - 1] + u[o + 1] + u[o - P] + u[o + P] + u[o - PP] + u[o + PP]) * sixth;
    });
    __syncthreads();
  };
#pragma unroll
  for (int l = 0; l + 1 < kCvcLevels; ++l) {
    if (l + 1 >= L.nl) break;
    const int nf = ed[l], P = nf + 2, PP = P * P;
    R* u = U[l];
    const R* f = Fv[l];
    cvc_points(nf, [&](int i, int j, int k) {
      const int o = (k * P + j) * P + i;
      if (((i + j + k) & 1) == 0) {
        u[o] = f[o] * sixth;
      } else {
        const R s = f[o - 1] + f[o + 1] + f[o - P] + f[o + P] + f[o - PP] + f[o + PP];
        u[o] = (f[o] + s * sixth) * sixth;
      }
    });
    __syncthreads();
    for (int sw = 2; sw < 2 * nu; ++sw) half(u, f, nf, (sw & 1) ? 1 : 0);
    // residual t = f - L7 u once per point, then the restriction from t
    cvc_points(nf, [&](int i, int j, int k) {
      const int o = (k * P + j) * P + i;
      tr[o] = f[o] - (R(6) * u[o] - u[o - 1] - u[o + 1] - u[o - P] - u[o + P] - u[o - PP] -
                      u[o + PP]);
    });
    __syncthreads();
    const int nc = ed[l + 1], Pc = nc + 2;
    R* fc = Fv[l + 1];
    cvc_points(nc, [&](int I, int J, int K) {
      const int o = ((2 * K) * P + 2 * J) * P + 2 * I;
      const int d1 = 1, d2 = P, d3 = PP;
      const R s = tr[o + d1] + tr[o - d1] + tr[o + d2] + tr[o - d2] + tr[o + d3] + tr[o - d3] +
                  tr[o + d1 + d2] + tr[o - d1 - d2] + tr[o + d1 + d3] + tr[o - d1 - d3] +
                  tr[o + d2 + d3] + tr[o - d2 - d3] + tr[o + d1 + d2 + d3] + tr[o - d1 - d2 - d3];
      fc[(K * Pc + J) * Pc + I] = R(0.5) * (tr[o] + R(0.5) * s);
    });
    __syncthreads();
  }
  // coarsest grid: dense inverse of L7 (unknowns in the order (k * nc + j) * nc + i, 0-based);
  // up to 32 unknowns, row r is a dot product over the lanes of a half wavefront
#pragma unroll
  for (int l = 0; l < kCvcLevels; ++l) {
    if (l != L.nl - 1) continue;
    const int nc = ed[l], np = nc * nc * nc, Pc = nc + 2;
    auto pad = [&](int q) {
      return (((q / (nc * nc)) + 1) * Pc + (q / nc) % nc + 1) * Pc + q % nc + 1;
    };
    if (np <= 32) {
      const int r = 2 * (t >> 6) + ((t >> 5) & 1), c = t & 31;
      double v = (r < np && c < np) ? C[r * np + c] * (double)Fv[l][pad(c)] : 0.0;
      for (int o = 16; o > 0; o >>= 1) v += __shfl_down(v, o, 32);
      if (r < np && c == 0) U[l][pad(r)] = (R)v;
    } else {
      cvc_points(nc, [&](int i, int j, int k) {
        const int row = ((k - 1) * nc + (j - 1)) * nc + (i - 1);
        double a = 0.0;
        for (int q = 0; q < np; ++q) a += C[row * np + q] * (double)Fv[l][pad(q)];
        U[l][(k * Pc + j) * Pc + i] = (R)a;
      });
    }
  }
  __syncthreads();
#pragma unroll
  for (int l = kCvcLevels - 2; l >= 0; --l) {
    if (l + 1 >= L.nl) continue;
    const int nf = ed[l], P = nf + 2;
    const int nc = ed[l + 1], Pc = nc + 2;
    R* u = U[l];
    const R* ec = U[l + 1];
    cvc_points(nf, [&](int i, int j, int k) {
      const int I = i >> 1, J = j >> 1, K = k >> 1;
      const int oc = (K * Pc + J) * Pc + I;
      const int od = ((k & 1) * Pc + (j & 1)) * Pc + (i & 1);
      u[(k * P + j) * P + i] += od ? R(0.5) * (ec[oc] + ec[oc + od]) : ec[oc];
    });
    __syncthreads();
    for (int sw = 0; sw < 2 * nu; ++sw) half(u, Fv[l], nf, (sw & 1) ? 0 : 1);
  }
  {
    const int P = ed[0] + 2;
    cvc_points(ed[0], [&](int i, int j, int k) {
      const int o = (k * P + j) * P + i;
      uout[o] = U[0][o];
    });
  }
}

// ---- interior PCG (level 0) -----------------------------------------------------------------

// f (padded) = sb b (compact interior order) + sg g on the plane k = nf (face order)
__global__ __launch_bounds__(kB3) void k3_rhs(Rhs3 rhs, double* __restrict__ f, int nf) {
  const int64_t N = (int64_t)nf * nf * nf;
  for (int64_t q = blockIdx.x * (int64_t)kB3 + threadIdx.x; q < N; q += (int64_t)gridDim.x * kB3) {
    int i, j, k;
    const size_t o = pidx(q, nf, &i, &j, &k);
    double v = rhs.b ? rhs.sb * rhs.b[q] : 0.0;
    if (rhs.g && k == nf) v += rhs.sg * rhs.g[(size_t)(j - 1) * nf + (i - 1)];
    f[o] = v;
  }
}

// interior solution (padded) -> caller's compact vector (interior then, optionally, Gamma)
__global__ __launch_bounds__(kB3) void k3_gather(const double* __restrict__ u, int nf,
                                                double* __restrict__ out,
                                                const double* __restrict__ xg) {
  const int64_t N = (int64_t)nf * nf * nf;
  const int64_t NG = (int64_t)nf * nf;
  for (int64_t q = blockIdx.x * (int64_t)kB3 + threadIdx.x; q < N + (xg ? NG : 0);
       q += (int64_t)gridDim.x * kB3) {
    if (q < N) {
      int i, j, k;
      out[q] = u[pidx(q, nf, &i, &j, &k)];
    } else {
      out[q] = xg[q - N];
    }
  }
}

// ---- interface (face) operators -------------------------------------------------------------
// Face vectors are compact (nf x nf, x fastest); system s of a batch at offset s * nf^2.

// ---- batched face CG ------------------------------------------------------------------------
// System s of a batch solves (alpha_s A_G + beta_s M_G) y_s = r_s by PCG with the preconditioner
// S D_s^{-1} S (S the orthonormal DST-I matrix, D_s the part of the operator diagonal in the
// sine basis).  An iteration is kf_apply1 (p, q = B_s p), the update y += alpha p,
// r' = r - alpha q (r in two buffers by the parity of the iteration), the convergence test and
// the preconditioner, whose last pass leaves the partials of r' . z.  When nf = 2^K - 1 that is
// three passes (kf_dst2u: update and transform along x; kf_cr: test and tridiagonal solves
// along y; kf_dst2: inverse transform), else kf_axpy1 and four DST passes (the first takes the
// test).  The scalars are summed by the pass that uses them (every block of a system sums the
// same partials; block 0 records them), and a system whose test is met is skipped by every
// later pass.  Partials of system s are at part[s * kPFS + b].

__device__ __forceinline__ double sys_sum(const double* __restrict__ part, int s, int cnt) {
  __shared__ double sh;
  double a = 0.0;
  for (int b = threadIdx.x; b < cnt; b += kB3) a += part[(size_t)s * kPFS + b];
  a = block_sum3(a);
  if (threadIdx.x == 0) sh = a;
  __syncthreads();
  const double r = sh;
  __syncthreads();
  return r;
}

__device__ __forceinline__ double face_at(const double* v, int nf, int i, int j) {
  return (i >= 0 && i < nf && j >= 0 && j < nf) ? v[(size_t)j * nf + i] : 0.0;
}

// r_s = src (mass = 0) or M_G src (mass = 1), y_s = 0, partials of |r_s|^2
__global__ __launch_bounds__(kB3) void kf_start(const double* __restrict__ src,
                                               double* __restrict__ r, double* __restrict__ y,
                                               int nf, double h, int mass,
                                               double* __restrict__ part) {
  const int s = blockIdx.y;
  const int64_t N = (int64_t)nf * nf;
  const double m0 = h * h / 12.0;
  double acc = 0.0;
  for (int64_t q = blockIdx.x * (int64_t)kB3 + threadIdx.x; q < N; q += (int64_t)gridDim.x * kB3) {
    double v = src[q];
    if (mass) {
      const int i = (int)(q % nf), j = (int)(q / nf);
      v = m0 * (6.0 * src[q] + face_at(src, nf, i + 1, j) + face_at(src, nf, i - 1, j) +
                face_at(src, nf, i, j + 1) + face_at(src, nf, i, j - 1) +
                face_at(src, nf, i + 1, j + 1) + face_at(src, nf, i - 1, j - 1));
    }
    r[(size_t)s * N + q] = v;
    y[(size_t)s * N + q] = 0.0;
    acc += v * v;
  }
  acc = block_sum3(acc);
  if (threadIdx.x == 0) part[(size_t)s * kPFS + blockIdx.x] = acc;
}

// rho_k = r . z (cnt partials), beta = rho_k / rho_{k-1} (0 at k = 0), p_k = z + beta p_{k-1}
// (formed at the neighbours too), q = (alpha A_G + beta_s M_G) p_k, partials of p_k . q
__global__ __launch_bounds__(kB3) void kf_apply1(const double* __restrict__ z,
                                                const double* __restrict__ pold,
                                                double* __restrict__ pnew,
                                                double* __restrict__ qv, int nf, double h,
                                                const Shift3* __restrict__ tab,
                                                FaceCG* __restrict__ cg,
                                                const double* __restrict__ pin, int cnt,
                                                double* __restrict__ part,
                                                int* __restrict__ done) {
  const int s = blockIdx.y;
  if (done[s]) return;
  const double rz = sys_sum(pin, s, cnt);
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  if (!(rz > 0.0) || !isfinite(rz)) {
    if (lead) {
      cg->bad[s] = 1;
      done[s] = 1;
    }
    return;
  }
  const int it = cg->its[s];
  const double be = it ? rz / cg->rho[(it - 1) & 1][s] : 0.0;
  if (lead) cg->rho[it & 1][s] = rz;
  const double al = tab->alpha[s], bm = tab->beta[s];
  const int64_t N = (int64_t)nf * nf;
  const double* zs = z + (size_t)s * N;
  const double* ps = pold + (size_t)s * N;
  const double m0 = h * h / 12.0;
  auto P = [&](int i, int j) {
    return it ? face_at(zs, nf, i, j) + be * face_at(ps, nf, i, j) : face_at(zs, nf, i, j);
  };
  double acc = 0.0;
  for (int64_t q = blockIdx.x * (int64_t)kB3 + threadIdx.x; q < N; q += (int64_t)gridDim.x * kB3) {
    const int i = (int)(q % nf), j = (int)(q / nf);
    const double c = P(i, j);
    const double e = P(i + 1, j), w = P(i - 1, j), no = P(i, j + 1), so = P(i, j - 1);
    const double ne = P(i + 1, j + 1), sw = P(i - 1, j - 1);
    const double a = 4.0 * c - e - w - no - so;
    const double m = m0 * (6.0 * c + e + w + no + so + ne + sw);
    const double v = al * a + bm * m;
    pnew[(size_t)s * N + q] = c;
    qv[(size_t)s * N + q] = v;
    acc += c * v;
  }
  acc = block_sum3(acc);
  if (threadIdx.x == 0) part[(size_t)s * kPFS + blockIdx.x] = acc;
}

// alpha_k = rho_k / (p_k . q) (kPartF partials), y += alpha_k p_k, r' = r - alpha_k q, partials of
// |r'|^2
__global__ __launch_bounds__(kB3) void kf_axpy1(double* __restrict__ y, const double* __restrict__ r,
                                               double* __restrict__ rnew,
                                               const double* __restrict__ p,
                                               const double* __restrict__ qv, int nf,
                                               FaceCG* __restrict__ cg,
                                               const double* __restrict__ pin,
                                               double* __restrict__ part,
                                               int* __restrict__ done) {
  const int s = blockIdx.y;
  if (done[s]) return;
  const double pq = sys_sum(pin, s, kPartF);
  if (!(pq > 0.0) || !isfinite(pq)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      cg->bad[s] = 1;
      done[s] = 1;
    }
    return;
  }
  const double al = cg->rho[cg->its[s] & 1][s] / pq;
  const int64_t N = (int64_t)nf * nf;
  const size_t off = (size_t)s * N;
  double acc = 0.0;
  for (int64_t t = blockIdx.x * (int64_t)kB3 + threadIdx.x; t < N; t += (int64_t)gridDim.x * kB3) {
    y[off + t] += al * p[off + t];
    const double rv = r[off + t] - al * qv[off + t];
    rnew[off + t] = rv;
    acc += rv * rv;
  }
  acc = block_sum3(acc);
  if (threadIdx.x == 0) part[(size_t)s * kPFS + blockIdx.x] = acc;
}

// The update of kf_axpy1 fused into the sine transform along x that starts the preconditioner
// (cyclic-reduction path): W = r' S with r' = r - alpha_k q formed while the row panels of r are
// loaded.  The blocks of the first column tile load every column of their 16-row band, so they
// store r', update y += alpha_k p_k and leave the band's |r'|^2 partial (ceil(nf / 16) per
// system); the convergence test follows in kf_cr.
__global__ __launch_bounds__(256) void kf_dst2u(const double* __restrict__ S,
                                               const double* __restrict__ r,
                                               const double* __restrict__ qv,
                                               const double* __restrict__ p,
                                               double* __restrict__ rnew, double* __restrict__ y,
                                               double* __restrict__ W, int nf,
                                               FaceCG* __restrict__ cg,
                                               const double* __restrict__ pin,
                                               double* __restrict__ part,
                                               int* __restrict__ done) {
  const int s = blockIdx.z;
  if (done[s]) return;
  const double pq = sys_sum(pin, s, kPartF);
  if (!(pq > 0.0) || !isfinite(pq)) {
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
      cg->bad[s] = 1;
      done[s] = 1;
    }
    return;
  }
  const double al = cg->rho[cg->its[s] & 1][s] / pq;
  const size_t off = (size_t)s * nf * nf;
  const bool writer = blockIdx.x == 0;
  __shared__ double ta[16][17], tb[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int col = blockIdx.x * 16 + tx, row = blockIdx.y * 16 + ty;
  double acc = 0.0, rr = 0.0;
  for (int k0 = 0; k0 < nf; k0 += 16) {
    const int ka = k0 + tx, kb = k0 + ty;
    double v = 0.0;
    if (row < nf && ka < nf) {
      const size_t o = off + (size_t)row * nf + ka;
      v = r[o] - al * qv[o];
      if (writer) {
        y[o] += al * p[o];
        rnew[o] = v;
        rr += v * v;
      }
    }
    ta[ty][tx] = v;
    tb[ty][tx] = (kb < nf && col < nf) ? S[(size_t)kb * nf + col] : 0.0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) acc += ta[ty][k] * tb[k][tx];
    __syncthreads();
  }
  if (row < nf && col < nf) W[off + (size_t)row * nf + col] = acc;
  if (writer) {
    rr = block_sum3(rr);
    if (threadIdx.x == 0) part[(size_t)s * kPFS + blockIdx.y] = rr;
  }
}

// C_s = S B_s (LEFT) or B_s S, S the symmetric DST matrix (nf x nf); 16 x 16 output tiles,
// LDS-staged 16-wide panels.  CHECK 1 / 2: first the start / convergence test of system s on
// the kPartF partials of |r|^2 (rr0 = |r_0|^2, its = 0 / its += 1, stop at
// |r|^2 <= tol2 rr0).  EPI 1: C /= alpha lambda(a, b) + beta mu(a, b) (the spectral scaling,
// a the column and b the row index, 1-based); EPI 2: partials of r . C over the tile.
template <bool LEFT, int CHECK, int EPI>
__global__ __launch_bounds__(256) void kf_dst2(const double* __restrict__ S,
                                              const double* __restrict__ B,
                                              double* __restrict__ C, int nf, int n, double h,
                                              const Shift3* __restrict__ tab,
                                              FaceCG* __restrict__ cg,
                                              const double* __restrict__ pin, double tol2,
                                              const double* __restrict__ r,
                                              double* __restrict__ part,
                                              int* __restrict__ done) {
  const int s = blockIdx.z;
  if (done[s]) return;
  if constexpr (CHECK != 0) {
    const double a = sys_sum(pin, s, kPartF);
    const bool lead = blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0;
    const bool bad = !isfinite(a);
    bool halt;
    if constexpr (CHECK == 1) {
      halt = bad || a == 0.0;
      if (lead) {
        cg->rr0[s] = a;
        cg->its[s] = 0;
      }
    } else {
      halt = bad || a <= tol2 * cg->rr0[s];
      if (lead) cg->its[s] += 1;
    }
    if (halt) {
      if (lead) {
        if (bad) cg->bad[s] = 1;
        done[s] = 1;
      }
      return;
    }
  }
  const double* Bs = B + (size_t)s * nf * nf;
  double* Cs = C + (size_t)s * nf * nf;
  __shared__ double ta[16][17], tb[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int col = blockIdx.x * 16 + tx, row = blockIdx.y * 16 + ty;
  // rows index j (the slow direction), columns index i
  double acc = 0.0;
  for (int k0 = 0; k0 < nf; k0 += 16) {
    const int ka = k0 + tx, kb = k0 + ty;
    if (LEFT) {
      ta[ty][tx] = (row < nf && ka < nf) ? S[(size_t)row * nf + ka] : 0.0;
      tb[ty][tx] = (kb < nf && col < nf) ? Bs[(size_t)kb * nf + col] : 0.0;
    } else {
      ta[ty][tx] = (row < nf && ka < nf) ? Bs[(size_t)row * nf + ka] : 0.0;
      tb[ty][tx] = (kb < nf && col < nf) ? S[(size_t)kb * nf + col] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) acc += ta[ty][k] * tb[k][tx];
    __syncthreads();
  }
  const bool in = row < nf && col < nf;
  if constexpr (EPI == 1) {
    const double ca = cos(M_PI * (col + 1) / n), cb = cos(M_PI * (row + 1) / n);
    const double lam = 4.0 - 2.0 * ca - 2.0 * cb;
    const double mu = h * h / 12.0 * (6.0 + 2.0 * ca + 2.0 * cb + 2.0 * ca * cb);
    acc /= tab->alpha[s] * lam + tab->beta[s] * mu;
  }
  if (in) Cs[(size_t)row * nf + col] = acc;
  if constexpr (EPI == 2) {
    double d = in ? r[(size_t)s * nf * nf + (size_t)row * nf + col] * acc : 0.0;
    d = block_sum3(d);
    if (threadIdx.x == 0) part[(size_t)s * kPFS + blockIdx.y * gridDim.x + blockIdx.x] = d;
  }
}

// out = sum_s coef_s y_s (P batch), or out = d0 M x + M sum_s coef_s y_s (H batch, op != 0)
__global__ __launch_bounds__(kB3) void kf_combine(const double* __restrict__ ys, int m, int nf,
                                                 double h, const Shift3* __restrict__ tab,
                                                 int op, const double* __restrict__ x,
                                                 double* __restrict__ tmp,
                                                 double* __restrict__ out) {
  const int64_t N = (int64_t)nf * nf;
  for (int64_t q = blockIdx.x * (int64_t)kB3 + threadIdx.x; q < N; q += (int64_t)gridDim.x * kB3) {
    // summed in system order; the loads are issued eight at a time
    double v = 0.0;
    int s = 0;
    for (; s + 8 <= m; s += 8) {
      double t[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) t[k] = ys[(size_t)(s + k) * N + q];
#pragma unroll
      for (int k = 0; k < 8; ++k) v += tab->coef[s + k] * t[k];
    }
    for (; s < m; ++s) v += tab->coef[s] * ys[(size_t)s * N + q];
    if (op) tmp[q] = v;
    else out[q] = v;
  }
}

// out = d0 M x + M tmp  (second pass of the H combination)
__global__ __launch_bounds__(kB3) void kf_mass2(const double* __restrict__ x,
                                               const double* __restrict__ tmp, int nf, double h,
                                               double d0, double* __restrict__ out) {
  const int64_t N = (int64_t)nf * nf;
  const double m0 = h * h / 12.0;
  for (int64_t q = blockIdx.x * (int64_t)kB3 + threadIdx.x; q < N; q += (int64_t)gridDim.x * kB3) {
    const int i = (int)(q % nf), j = (int)(q / nf);
    auto mass = [&](const double* v) {
      return m0 * (6.0 * v[q] + face_at(v, nf, i + 1, j) + face_at(v, nf, i - 1, j) +
                   face_at(v, nf, i, j + 1) + face_at(v, nf, i, j - 1) +
                   face_at(v, nf, i + 1, j + 1) + face_at(v, nf, i - 1, j - 1));
    };
    out[q] = d0 * mass(x) + mass(tmp);
  }
}

// y = K h (3 p - 1/2 (E + W + N + S) p - u|plane nf) + gamma Hp  (S p with u = L7^{-1} lift p),
// or, with b, the full operator's Gamma rows; partials of p . y.
__global__ __launch_bounds__(kB3) void kf_schur(const double* __restrict__ p,
                                               const double* __restrict__ u, int nf, double h,
                                               double K, double gamma,
                                               const double* __restrict__ Hp,
                                               double* __restrict__ y,
                                               double* __restrict__ part) {
  const int64_t N = (int64_t)nf * nf;
  const size_t P = (size_t)nf + 2;
  double acc = 0.0;
  for (int64_t q = blockIdx.x * (int64_t)kB3 + threadIdx.x; q < N; q += (int64_t)gridDim.x * kB3) {
    const int i = (int)(q % nf), j = (int)(q / nf);
    const double nb = face_at(p, nf, i + 1, j) + face_at(p, nf, i - 1, j) +
                      face_at(p, nf, i, j + 1) + face_at(p, nf, i, j - 1);
    const double ub = u[((size_t)nf * P + (size_t)(j + 1)) * P + (size_t)(i + 1)];
    const double v = K * h * (3.0 * p[q] - 0.5 * nb - ub) + gamma * Hp[q];
    y[q] = v;
    acc += p[q] * v;
  }
  acc = block_sum3(acc);
  if (part && threadIdx.x == 0) part[blockIdx.x] = acc;
}

// Full operator y = K A_Omega x + gamma T^T H T x on all free dofs (interior 7-point times h,
// Gamma row h (3, -1/2 x 4 in-face, -1 below)); optional ||b - y||^2, ||b||^2 partials.
__global__ __launch_bounds__(kB3) void k3_full_operator(int n, double K, double gamma,
                                                       const double* __restrict__ x,
                                                       const double* __restrict__ Hx,
                                                       double* __restrict__ y,
                                                       const double* __restrict__ b,
                                                       double* __restrict__ part) {
  const int m = n - 1;
  const int64_t N = (int64_t)m * m * n;
  const double h = 1.0 / n;
  double e2 = 0.0, b2 = 0.0;
  for (int64_t q = blockIdx.x * (int64_t)kB3 + threadIdx.x; q < N; q += (int64_t)gridDim.x * kB3) {
    const int i = (int)(q % m), j = (int)((q / m) % m), k = (int)(q / ((int64_t)m * m));
    auto X = [&](int ii, int jj, int kk) -> double {
      if (ii < 0 || ii >= m || jj < 0 || jj >= m || kk < 0 || kk >= n) return 0.0;
      return x[((int64_t)kk * m + jj) * m + ii];
    };
    const double c = x[q];
    double v;
    if (k < n - 1) {
      v = K * h * (6.0 * c - X(i - 1, j, k) - X(i + 1, j, k) - X(i, j - 1, k) - X(i, j + 1, k) -
                   X(i, j, k - 1) - X(i, j, k + 1));
    } else {
      v = K * h * (3.0 * c - 0.5 * (X(i - 1, j, k) + X(i + 1, j, k) + X(i, j - 1, k) + X(i, j + 1, k)) -
                   X(i, j, k - 1)) +
          gamma * Hx[(int64_t)j * m + i];
    }
    if (y) y[q] = v;
    if (b) {
      const double d = b[q] - v;
      e2 += d * d;
      b2 += b[q] * b[q];
    }
  }
  if (!part) return;
  e2 = block_sum3(e2);
  b2 = block_sum3(b2);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = e2;
    part[2 * blockIdx.x + 1] = b2;
  }
}

// outer PCG vector steps on the face (compact FP64 vectors).
// kind 0: x += alpha p, r -= alpha y (alpha = rho / pq from st);  kind 1: p = z + beta p
__global__ __launch_bounds__(kB3) void kf_outer_axpy(double* __restrict__ x, double* __restrict__ r,
                                                    double* __restrict__ p,
                                                    const double* __restrict__ y,
                                                    const double* __restrict__ z, int64_t N,
                                                    const double* __restrict__ coef) {
  const double a = *coef;  // alpha or beta of the outer PCG (k3_outer_scalars)
  for (int64_t q = blockIdx.x * (int64_t)kB3 + threadIdx.x; q < N; q += (int64_t)gridDim.x * kB3) {
    if (x) {
      x[q] += a * p[q];
      r[q] -= a * y[q];
    } else {
      p[q] = z[q] + a * p[q];
    }
  }
}

__global__ __launch_bounds__(kB3) void k3_scale_add(double* __restrict__ out,
                                                   const double* __restrict__ u, double c,
                                                   const double* __restrict__ coef,
                                                   int accumulate, int64_t N) {
  if (coef) c = *coef;
  for (int64_t q = blockIdx.x * (int64_t)kB3 + threadIdx.x; q < N; q += (int64_t)gridDim.x * kB3)
    out[q] = (accumulate ? out[q] : 0.0) + c * u[q];
}

// g = b_G + h w|plane nf (right-hand side of the interface problem), x_G = 0
__global__ __launch_bounds__(kB3) void kf_rhs_reduce(const double* __restrict__ bG,
                                                    const double* __restrict__ w, int nf,
                                                    double h, double* __restrict__ g,
                                                    double* __restrict__ xg) {
  const int64_t N = (int64_t)nf * nf;
  const size_t P = (size_t)nf + 2;
  for (int64_t q = blockIdx.x * (int64_t)kB3 + threadIdx.x; q < N; q += (int64_t)gridDim.x * kB3) {
    const int i = (int)(q % nf), j = (int)(q / nf);
    g[q] = bG[q] + h * w[((size_t)nf * P + (size_t)(j + 1)) * P + (size_t)(i + 1)];
    xg[q] = 0.0;
  }
}

// plain block partials of a . b over compact vectors of length N
// sc[slot] = sum of count partials part[q * stride] (one block; thread t adds q = t, t + kB3, ...,
// then a fixed tree), so the outer PCG's dots are summed on the device in a fixed order
__global__ __launch_bounds__(kB3) void k3_sum_partials(const double* __restrict__ part, int count,
                                                       int stride, double* __restrict__ sc,
                                                       int slot) {
  double acc = thread_partials<kB3>(part, count, threadIdx.x, stride);
  acc = block_sum3(acc);
  if (threadIdx.x == 0) sc[slot] = acc;
}

// The outer PCG's step scalars from the summed dots (one thread):
//   mode 0 (start):  rho0 = rho = rz
//   mode 1 (after p.Sp): alpha = rho / pq
//   mode 2 (after the new r.z): beta = rz / rho, rho = rz
__global__ void k3_outer_scalars(double* __restrict__ sc, int mode) {
  if (threadIdx.x != 0) return;
  if (mode == 0) {
    sc[kSc3Rho0] = sc[kSc3Rz];
    sc[kSc3Rho] = sc[kSc3Rz];
  } else if (mode == 1) {
    sc[kSc3Alpha] = sc[kSc3Rho] / sc[kSc3Pq];
  } else {
    sc[kSc3Beta] = sc[kSc3Rz] / sc[kSc3Rho];
    sc[kSc3Rho] = sc[kSc3Rz];
  }
}

__global__ __launch_bounds__(kB3) void kf_vdot(const double* __restrict__ a,
                                              const double* __restrict__ b, int64_t N,
                                              double* __restrict__ part) {
  double acc = 0.0;
  for (int64_t q = blockIdx.x * (int64_t)kB3 + threadIdx.x; q < N; q += (int64_t)gridDim.x * kB3)
    acc += a[q] * b[q];
  acc = block_sum3(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// Middle pass of the preconditioner when nf = 2^K - 1, on W = r S (the sine transform along x,
// by kf_dst2): for each column a, the tridiagonal system along y
// (alpha (4 - 2 c_a) + beta h^2/12 (6 + 2 c_a)) w_j + (-alpha + beta h^2/12 (1 + c_a))
// (w_{j-1} + w_{j+1}) = W_j, c_a = cos(pi a / n), zero beyond the ends, in place.  Its sine
// transform along y is the spectral scaling of kf_dst2 (EPI 1), so the three passes apply the
// same preconditioner as the four.  With 2^K - 1 rows, cyclic reduction keeps one (d, e) pair
// per level: d' = d - 2 e^2 / d, e' = -e^2 / d (diagonal dominance is kept).  A block takes a
// panel of 16 columns of one system, held in LDS.  CHECK as in kf_dst2, on cnt partials.
template <int CHECK>
__global__ __launch_bounds__(256) void kf_cr(double* __restrict__ w, int nf, int K, int n,
                                            double h, const Shift3* __restrict__ tab,
                                            FaceCG* __restrict__ cg,
                                            const double* __restrict__ pin, int cnt, double tol2,
                                            int* __restrict__ done) {
  const int s = blockIdx.y;
  if (done[s]) return;
  if constexpr (CHECK != 0) {
    const double a = sys_sum(pin, s, cnt);
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    const bool bad = !isfinite(a);
    bool halt;
    if constexpr (CHECK == 1) {
      halt = bad || a == 0.0;
      if (lead) {
        cg->rr0[s] = a;
        cg->its[s] = 0;
      }
    } else {
      halt = bad || a <= tol2 * cg->rr0[s];
      if (lead) cg->its[s] += 1;
    }
    if (halt) {
      if (lead) {
        if (bad) cg->bad[s] = 1;
        done[s] = 1;
      }
      return;
    }
  }
  __shared__ double sW[kFaceRows][17];  // row J = j + 1 of the reduction at sW[j]
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int col = blockIdx.x * 16 + tx;
  double* ws = w + (size_t)s * nf * nf;
  if (col < nf)
    for (int j = ty; j < nf; j += 16) sW[j][tx] = ws[(size_t)j * nf + col];
  double dl[8], el[8];
  {
    const double ca = cos(M_PI * (col + 1) / n);
    const double al = tab->alpha[s], be = tab->beta[s], m0 = h * h / 12.0;
    dl[0] = al * (4.0 - 2.0 * ca) + be * m0 * (6.0 + 2.0 * ca);
    el[0] = -al + be * m0 * (1.0 + ca);
#pragma unroll
    for (int l = 0; l + 1 < 8; ++l) {
      const double q = el[l] * el[l] / dl[l];
      dl[l + 1] = dl[l] - 2.0 * q;
      el[l + 1] = -q;
    }
  }
  __syncthreads();
  // forward reduction: level l = 0 .. K - 2 updates the rows J that are multiples of 2^(l+1)
#pragma unroll
  for (int l = 0; l < 7; ++l) {
    if (l + 2 > K) break;
    const int st = 1 << l;
    const double g = el[l] / dl[l];
    if (col < nf)
      for (int J = 2 * st * (ty + 1); J <= nf; J += 2 * st * 16)
        sW[J - 1][tx] -= g * (sW[J - st - 1][tx] + sW[J + st - 1][tx]);
    __syncthreads();
  }
  // the middle row, then back substitution on the odd multiples of 2^l
  if (col < nf && ty == 0) {
    const int J = 1 << (K - 1);
#pragma unroll
    for (int l = 0; l < 8; ++l)
      if (l == K - 1) sW[J - 1][tx] /= dl[l];
  }
  __syncthreads();
#pragma unroll
  for (int l = 6; l >= 0; --l) {
    if (l + 2 > K) continue;
    const int st = 1 << l;
    if (col < nf)
      for (int J = st * (2 * ty + 1); J <= nf; J += 2 * st * 16) {
        const double lo = J - st >= 1 ? sW[J - st - 1][tx] : 0.0;
        const double hi = J + st <= nf ? sW[J + st - 1][tx] : 0.0;
        sW[J - 1][tx] = (sW[J - 1][tx] - el[l] * (lo + hi)) / dl[l];
      }
    __syncthreads();
  }
  if (col < nf)
    for (int j = ty; j < nf; j += 16) ws[(size_t)j * nf + col] = sW[j][tx];
}

// ---- launchers -------------------------------------------------------------------------------

static inline int grid_for(int64_t N, int cap = kPart3) {
  const int64_t g = (N + kB3 - 1) / kB3;
  return (int)(g < cap ? (g < 1 ? 1 : g) : cap);
}

int k3_rows_red(int nf) {
  int r = (nf * nf + 1023) / 1024;
  r = r < 4 ? 4 : r;
  return (r + 3) & ~3;
}

int k3_cvc_fits(const Cvc3& L) {
  if (L.nl < 1 || L.nl > kCvcLevels || L.lev[0] > kCvcMax) return 0;
  int tot = 0;
  for (int l = 0; l < L.nl; ++l) tot += 2 * (L.lev[l] + 2) * (L.lev[l] + 2) * (L.lev[l] + 2);
  return tot <= kCvcLds;
}

static inline dim3 grid3(int nf, int rows) { return dim3((nf + rows - 1) / rows, nf); }
static const dim3 kBlk3(kX3, kY3);

template <typename R>
void k3_launch_zp(hipStream_t s, int mode, const R* f, R* u, int nf, int rows, const R* q, R* rnew,
                  R* x, const R* p, State3* st, const double* pin, int np, double* part,
                  int* stop) {
  if (mode == 0)
    hipLaunchKernelGGL((k3_zp<R, 0>), grid3(nf, rows), kBlk3, 0, s, f, u, nf, rows, q, rnew, x, p,
                       st, pin, np, part, stop);
  else if (mode == 1)
    hipLaunchKernelGGL((k3_zp<R, 1>), grid3(nf, rows), kBlk3, 0, s, f, u, nf, rows, q, rnew, x, p,
                       st, pin, np, part, stop);
  else
    hipLaunchKernelGGL((k3_zp<R, 2>), grid3(nf, rows), kBlk3, 0, s, f, u, nf, rows, q, rnew, x, p,
                       st, pin, np, part, stop);
}
template <typename R>
void k3_launch_hs(hipStream_t s, R* u, const R* f, int nf, int red, int check, State3* st,
                  const double* pin, int np, int* stop) {
  hipLaunchKernelGGL(k3_hs<R>, grid3(nf, 4), kBlk3, 0, s, u, f, nf, 4, red, check, st, pin, np,
                     stop);
}
template <typename R>
void k3_launch_rr(hipStream_t s, const R* u, const R* f, R* fc, int nf, int nc, int check,
                  State3* st, const double* pin, int np, int* stop) {
  hipLaunchKernelGGL(k3_rr<R>, grid3(nc, 4), kBlk3, 0, s, u, f, fc, nf, nc, 4, check, st, pin, np,
                     stop);
}
template <typename R>
void k3_launch_pr(hipStream_t s, const R* u, const R* ec, const R* f, R* uo, int nf, int nc,
                  int* stop) {
  hipLaunchKernelGGL(k3_pr<R>, grid3(nf, 4), kBlk3, 0, s, u, ec, f, uo, nf, nc, 4, stop);
}
template <typename R>
void k3_launch_hsz(hipStream_t s, R* u, const R* f, int nf, int rows, double* part, int* stop) {
  hipLaunchKernelGGL(k3_hsz<R>, grid3(nf, rows), kBlk3, 0, s, u, f, nf, rows, part, stop);
}
template <typename R>
void k3_launch_apply1(hipStream_t s, const R* z, const R* pold, R* pnew, R* q, int nf, int rows,
                      State3* st, const double* pin, int np, double* part, int* stop) {
  hipLaunchKernelGGL(k3_apply1<R>, grid3(nf, rows), kBlk3, 0, s, z, pold, pnew, q, nf, rows, st,
                     pin, np, part, stop);
}
template <typename R>
void k3_launch_cvc(hipStream_t s, const R* fin, R* uout, const Cvc3& L, const double* cinv,
                   int nu, int* stop) {
  hipLaunchKernelGGL(k3_cvc<R>, dim3(1), dim3(kCvcThreads), 0, s, fin, uout, L, cinv, nu, stop);
}
void k3_launch_ir(hipStream_t s, int first, const double* F, const double* xin, const float* e,
                  double* xout, float* r32, int nf, int rows, State3* st, double* part) {
  if (first)
    hipLaunchKernelGGL(k3_ir<true>, grid3(nf, rows), kBlk3, 0, s, F, xin, e, xout, r32, nf, rows,
                       st, part);
  else
    hipLaunchKernelGGL(k3_ir<false>, grid3(nf, rows), kBlk3, 0, s, F, xin, e, xout, r32, nf, rows,
                       st, part);
}
#define K3_INSTANTIATE(R)                                                                        \
  template void k3_launch_zp<R>(hipStream_t, int, const R*, R*, int, int, const R*, R*, R*,     \
                                const R*, State3*, const double*, int, double*, int*);          \
  template void k3_launch_hs<R>(hipStream_t, R*, const R*, int, int, int, State3*,              \
                                const double*, int, int*);                                      \
  template void k3_launch_rr<R>(hipStream_t, const R*, const R*, R*, int, int, int, State3*,    \
                                const double*, int, int*);                                      \
  template void k3_launch_pr<R>(hipStream_t, const R*, const R*, const R*, R*, int, int, int*); \
  template void k3_launch_hsz<R>(hipStream_t, R*, const R*, int, int, double*, int*);           \
  template void k3_launch_apply1<R>(hipStream_t, const R*, const R*, R*, R*, int, int, State3*, \
                                    const double*, int, double*, int*);                         \
  template void k3_launch_cvc<R>(hipStream_t, const R*, R*, const Cvc3&, const double*, int, int*);
K3_INSTANTIATE(float)
K3_INSTANTIATE(double)
#undef K3_INSTANTIATE
void k3_launch_rhs(hipStream_t s, const Rhs3& rhs, double* f, int nf) {
  hipLaunchKernelGGL(k3_rhs, dim3(grid_for((int64_t)nf * nf * nf, 4096)), dim3(kB3), 0, s, rhs, f,
                     nf);
}
void k3_launch_gather(hipStream_t s, const double* u, int nf, double* out, const double* xg) {
  hipLaunchKernelGGL(k3_gather, dim3(grid_for((int64_t)nf * nf * nf + nf * nf, 4096)), dim3(kB3),
                     0, s, u, nf, out, xg);
}
void kf_launch_start(hipStream_t s, const double* src, double* r, double* y, int nf, double h,
                     int m, int mass, double* part) {
  hipLaunchKernelGGL(kf_start, dim3(kPartF, m), dim3(kB3), 0, s, src, r, y, nf, h, mass, part);
}
void kf_launch_apply1(hipStream_t s, const double* z, const double* pold, double* pnew, double* q,
                      int nf, double h, int m, const Shift3* tab, FaceCG* cg, const double* pin,
                      int cnt, double* part, int* done) {
  hipLaunchKernelGGL(kf_apply1, dim3(kPartF, m), dim3(kB3), 0, s, z, pold, pnew, q, nf, h, tab, cg,
                     pin, cnt, part, done);
}

int kf_tiles(int nf) { return ((nf + 15) / 16) * ((nf + 15) / 16); }
int kf_cr_levels(int nf) {
  for (int K = 1; K <= 8; ++K)
    if (nf == (1 << K) - 1) return K;
  return 0;
}
void kf_launch_prec(hipStream_t s, const double* S, const double* r, double* ft, double* z, int nf,
                    int n, double h, int m, const Shift3* tab, FaceCG* cg, const double* pin,
                    double tol2, int check, double* part, int* done) {
  const dim3 g((nf + 15) / 16, (nf + 15) / 16, m);
  const int K = kf_cr_levels(nf);
  if (K >= 2 && nf <= kFaceMax) {
    // x transform, tridiagonal solves along y, inverse x transform
    const dim3 gp((nf + 15) / 16, m);
    if (check == 1)
      hipLaunchKernelGGL((kf_dst2<false, 1, 0>), g, dim3(256), 0, s, S, r, ft, nf, n, h, tab, cg,
                         pin, tol2, nullptr, nullptr, done);
    else
      hipLaunchKernelGGL((kf_dst2<false, 2, 0>), g, dim3(256), 0, s, S, r, ft, nf, n, h, tab, cg,
                         pin, tol2, nullptr, nullptr, done);
    hipLaunchKernelGGL(kf_cr<0>, gp, dim3(256), 0, s, ft, nf, K, n, h, tab, cg, nullptr, 0, tol2,
                       done);
    hipLaunchKernelGGL((kf_dst2<false, 0, 2>), g, dim3(256), 0, s, S, ft, z, nf, n, h, tab, cg,
                       nullptr, tol2, r, part, done);
    return;
  }
  if (check == 1)
    hipLaunchKernelGGL((kf_dst2<true, 1, 0>), g, dim3(256), 0, s, S, r, ft, nf, n, h, tab, cg, pin,
                       tol2, nullptr, nullptr, done);
  else
    hipLaunchKernelGGL((kf_dst2<true, 2, 0>), g, dim3(256), 0, s, S, r, ft, nf, n, h, tab, cg, pin,
                       tol2, nullptr, nullptr, done);
  hipLaunchKernelGGL((kf_dst2<false, 0, 1>), g, dim3(256), 0, s, S, ft, z, nf, n, h, tab, cg,
                     nullptr, tol2, nullptr, nullptr, done);
  hipLaunchKernelGGL((kf_dst2<true, 0, 0>), g, dim3(256), 0, s, S, z, ft, nf, n, h, tab, cg,
                     nullptr, tol2, nullptr, nullptr, done);
  hipLaunchKernelGGL((kf_dst2<false, 0, 2>), g, dim3(256), 0, s, S, ft, z, nf, n, h, tab, cg,
                     nullptr, tol2, r, part, done);
}
void kf_launch_face_update_prec(hipStream_t s, const double* S, const double* r, double* rnew,
                                const double* q, const double* p, double* y, double* ft, double* z,
                                int nf, int n, double h, int m, const Shift3* tab, FaceCG* cg,
                                const double* pq, double tol2, double* part, int* done) {
  const int K = kf_cr_levels(nf);
  if (K >= 2 && nf <= kFaceMax) {
    // update fused into the x transform; test in the cyclic reduction; inverse x transform
    const dim3 g((nf + 15) / 16, (nf + 15) / 16, m), gp((nf + 15) / 16, m);
    hipLaunchKernelGGL(kf_dst2u, g, dim3(256), 0, s, S, r, q, p, rnew, y, ft, nf, cg, pq, part,
                       done);
    hipLaunchKernelGGL(kf_cr<2>, gp, dim3(256), 0, s, ft, nf, K, n, h, tab, cg, part,
                       (nf + 15) / 16, tol2, done);
    hipLaunchKernelGGL((kf_dst2<false, 0, 2>), g, dim3(256), 0, s, S, ft, z, nf, n, h, tab, cg,
                       nullptr, tol2, rnew, part, done);
    return;
  }
  hipLaunchKernelGGL(kf_axpy1, dim3(kPartF, m), dim3(kB3), 0, s, y, r, rnew, p, q, nf, cg, pq,
                     part, done);
  kf_launch_prec(s, S, rnew, ft, z, nf, n, h, m, tab, cg, part, tol2, 2, part, done);
}
void kf_launch_combine(hipStream_t s, const double* ys, int m, int nf, double h, const Shift3* tab,
                       int op, const double* x, double* tmp, double* out, double d0) {
  const int g = grid_for((int64_t)nf * nf, 1024);
  hipLaunchKernelGGL(kf_combine, dim3(g), dim3(kB3), 0, s, ys, m, nf, h, tab, op, x, tmp, out);
  if (op) hipLaunchKernelGGL(kf_mass2, dim3(g), dim3(kB3), 0, s, x, tmp, nf, h, d0, out);
}
void kf_launch_schur(hipStream_t s, const double* p, const double* u, int nf, double h, double K,
                     double gamma, const double* Hp, double* y, double* part) {
  hipLaunchKernelGGL(kf_schur, dim3(kPart3), dim3(kB3), 0, s, p, u, nf, h, K, gamma, Hp, y, part);
}
void k3_launch_full_operator(hipStream_t s, int n, double K, double gamma, const double* x,
                             const double* Hx, double* y, const double* b, double* part) {
  hipLaunchKernelGGL(k3_full_operator, dim3(kPart3), dim3(kB3), 0, s, n, K, gamma, x, Hx, y, b,
                     part);
}
void kf_launch_outer_axpy(hipStream_t s, double* x, double* r, double* p, const double* y,
                          const double* z, int64_t N, const double* coef) {
  hipLaunchKernelGGL(kf_outer_axpy, dim3(grid_for(N, 1024)), dim3(kB3), 0, s, x, r, p, y, z, N,
                     coef);
}
void k3_launch_scale_add(hipStream_t s, double* out, const double* u, double c, int accumulate,
                         int64_t n, const double* coef) {
  hipLaunchKernelGGL(k3_scale_add, dim3(grid_for(n, 2048)), dim3(kB3), 0, s, out, u, c, coef,
                     accumulate, n);
}
void k3_launch_sum_partials(hipStream_t s, const double* part, int count, int stride, double* sc,
                            int slot) {
  hipLaunchKernelGGL(k3_sum_partials, dim3(1), dim3(kB3), 0, s, part, count, stride, sc, slot);
}
void k3_launch_outer_scalars(hipStream_t s, double* sc, int mode) {
  hipLaunchKernelGGL(k3_outer_scalars, dim3(1), dim3(64), 0, s, sc, mode);
}
void kf_launch_rhs_reduce(hipStream_t s, const double* bG, const double* w, int nf, double h,
                          double* g, double* xg) {
  hipLaunchKernelGGL(kf_rhs_reduce, dim3(grid_for((int64_t)nf * nf, 1024)), dim3(kB3), 0, s, bG, w,
                     nf, h, g, xg);
}
void kf_launch_vdot(hipStream_t s, const double* a, const double* b, int64_t N, double* part) {
  hipLaunchKernelGGL(kf_vdot, dim3(kPart3), dim3(kB3), 0, s, a, b, N, part);
}

}  // namespace fdd
