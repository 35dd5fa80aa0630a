// Batched form of the 2D solver: many independent instances (different n, K, mu) advance
// together, and every launch covers all of them.  A level kernel's grid is the concatenated list
// of the tiles of every instance that has that level (a block finds its instance by binary search
// in a prefix table); the coarse-level kernel runs one workgroup per instance; all shifted
// interface systems of all instances (eq. (RA), one per pole) form one launch.  The arithmetic is
// the single-instance device code (mg_device.h, iface_device.h), so a batch of one reproduces
// the single-instance solve.  Instances whose outer PCG has converged return at once.
#include "iface_device.h"
#include "mg_device.h"

namespace fdd {

// Largest i with start[i] <= b, for a non-decreasing prefix table start[0..ninst].
// b is the same for the whole workgroup, and so is the result: the loaded values are made
// wave-uniform so that the instance's descriptor is read with scalar loads.
__device__ __forceinline__ int find_inst(const int* __restrict__ start, int ninst, int b) {
  int lo = 0, hi = ninst;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (__builtin_amdgcn_readfirstlane(start[mid]) <= b) lo = mid;
    else hi = mid;
  }
  return __builtin_amdgcn_readfirstlane(lo);
}

__device__ __forceinline__ int first_tile(const int* __restrict__ start, int i) {
  return __builtin_amdgcn_readfirstlane(start[i]);
}

// XCD-aware order of the concatenated tile list: workgroup b runs on XCD b % 8, so tile
// (b % 8) q + b / 8 (q = grid / 8) gives each XCD one contiguous stretch of the list (whole
// instances, or neighbouring tile rows of one instance), keeping shared halos in one L2.
__device__ __forceinline__ int xcd_linear() {
  const int b = blockIdx.x, nb = gridDim.x;
  const int q = nb >> 3;
  return __builtin_amdgcn_readfirstlane((b < 8 * q) ? (b & 7) * q + (b >> 3) : b);
}

__device__ __forceinline__ bool inst_idle(const DevState* st, int skip_done) {
  return skip_done && st->outer_done;
}

// The outer tail of an instance runs only once its interior solve of this iteration has met its
// tolerance; otherwise the host completes the solve and repeats the tail.
__device__ __forceinline__ bool tail_idle(const DevState* st, int skip_done) {
  return (skip_done && st->outer_done) || !st->solve_done;
}

template <int NU, bool CG, int TT>
__global__ __launch_bounds__(kBlock) void kb_mg_down(const BInst* __restrict__ I, BLists L,
                                                     int level, int k, int cur_r, int cur_p,
                                                     int check, int skip_done) {
  const int b = xcd_linear();
  const int* start = L.tiles[level];
  const int i = find_inst(start, L.ninst, b);
  const BInst& P = I[i];
  DevState* st = P.st;
  if (inst_idle(st, skip_done) || stopped(st)) return;
  const int t = b - first_tile(start, i);
  const int tx = P.tiles_x[level];
  const int tile_x = t % tx, tile_y = t / tx;
  const bool lead = (t == 0);
  const Reductions red = P.red;
  if (check && level == 1 && pcg_converged(st, red, lead)) return;
  if constexpr (CG) {
    d_mg_down<float, NU, true, TT>(P.r[cur_r], P.u[0], P.f[1], P.nf[0], P.pitch[0],
                                   P.pitch[1], P.z, P.p[cur_p], P.p[cur_p ^ 1], P.x,
                                   P.r[cur_r ^ 1], st, red, k, tile_x, tile_y, t, lead, true);
  } else {
    const float* fin = level == 0 ? P.r[cur_r] : P.f[level];
    d_mg_down<float, NU, false, TT>(fin, P.u[level], P.f[level + 1], P.nf[level],
                                    P.pitch[level], P.pitch[level + 1], nullptr, nullptr,
                                    nullptr, nullptr, nullptr, st, red, 0, tile_x, tile_y, t,
                                    lead);
  }
}

// The two dot products of every instance's next PCG update, one block per instance (the
// level-0 down kernel then reads two scalars instead of summing every tile's partials).
__global__ __launch_bounds__(kBlock) void kb_dots(const BInst* __restrict__ I, int k,
                                                  int skip_done) {
  const BInst& P = I[blockIdx.x];
  DevState* st = P.st;
  if (inst_idle(st, skip_done) || stopped(st)) return;
  d_sum_dots(P.red, k, st);
}

// Convergence test of every instance after the last scheduled update of its PCG run (in place of
// the V-cycle that would follow it); a run that has not converged counts the iteration.
__global__ __launch_bounds__(kBlock) void kb_run_check(const BInst* __restrict__ I,
                                                       int skip_done) {
  const BInst& P = I[blockIdx.x];
  DevState* st = P.st;
  if (inst_idle(st, skip_done) || stopped(st)) return;
  if (!pcg_converged(st, P.red, true) && thread0()) {
    st->inner_its += 1;
    st->pcg_k += 1;
    st->run_its_max = max(st->run_its_max, st->pcg_k);
  }
}

template <int NU, bool CG, int TT>
__global__ __launch_bounds__(kBlock) void kb_mg_up(const BInst* __restrict__ I, BLists L,
                                                   int level, int kn, int count, int cur_r,
                                                   int skip_done) {
  const int b = xcd_linear();
  const int* start = L.tiles[level];
  const int i = find_inst(start, L.ninst, b);
  const BInst& P = I[i];
  DevState* st = P.st;
  if (inst_idle(st, skip_done) || stopped(st)) return;
  const int t = b - first_tile(start, i);
  const int tx = P.tiles_x[level];
  const int tile_x = t % tx, tile_y = t / tx;
  const bool lead = (t == 0);
  const Reductions red = P.red;
  if constexpr (CG) {
    d_mg_up<float, NU, true, TT>(P.r[cur_r], P.u[0], P.e[1], P.z, P.nf[0], P.pitch[0],
                                 P.pitch[1], st, red, kn, count, tile_x, tile_y, t, lead);
  } else {
    d_mg_up<float, NU, false, TT>(P.f[level], P.u[level], P.e[level + 1], P.e[level],
                                  P.nf[level], P.pitch[level], P.pitch[level + 1], st, red, 0, 0,
                                  tile_x, tile_y, t, lead);
  }
}

__global__ __launch_bounds__(kCoarseThreads) void kb_coarse(const BInst* __restrict__ I, int check,
                                                            int skip_done) {
  const BInst& P = I[blockIdx.x];
  DevState* st = P.st;
  if (inst_idle(st, skip_done) || stopped(st)) return;
  if (check && P.fc == 1 && pcg_converged(st, P.red, true)) return;
  d_coarse_dst(P.f[P.fc], P.pitch[P.fc], P.e[P.fc], P.nf[P.fc], P.dstS, P.dstL);
}

// Version of the final interface iterate: the converged one, else the last (ver).
__device__ __forceinline__ int final_ver(const DevState* st, int ver) {
  return st->outer_done ? st->o_ver : ver;
}

// Right-hand side of a batched interior solve: b, the lifted p (version ver), or the
// back-substitution b/K + lift(x_G) with x_G the instance's final iterate.
__device__ __forceinline__ RhsDesc b_rhs(const BInst& P, int kind, int ver) {
  if (kind == kRhsB) return RhsDesc{P.b, 1.0, nullptr, 0.0};
  if (kind == kRhsLiftP) return RhsDesc{nullptr, 0.0, P.pG[ver & 1], 1.0};
  return RhsDesc{P.b, 1.0 / P.K, P.xG[final_ver(P.st, ver) & 1], 1.0};
}

__global__ __launch_bounds__(kBlock) void kb_ir_residual(const BInst* __restrict__ I, BLists L,
                                                         int first, int rhs, int ver, int S,
                                                         int cur_r, double tol2, double tau2,
                                                         int skip_done) {
  const int b = xcd_linear();
  const int* start = L.tiles[0];
  const int i = find_inst(start, L.ninst, b);
  const BInst& P = I[i];
  DevState* st = P.st;
  if (inst_idle(st, skip_done)) return;
  const int t = b - first_tile(start, i);
  const int tx = P.tiles_x[0];
  RhsDesc f = b_rhs(P, rhs, ver);
  // the first residual of a lifted-p solve starts from the learned guess, if any, scaled by its
  // Galerkin factor (kb_warm_alpha)
  const bool warm = first && rhs == kRhsLiftP && P.warm;
  d_ir_residual<float>(f, first ? nullptr : P.u64[S & 1], P.x,
                       first ? P.u64[0] : P.u64[(S + 1) & 1], P.r[cur_r], nullptr,
                       P.nf[0], P.pitch[0], first, tol2, tau2, 0, st, P.red, t % tx, t / tx,
                       t, t == 0, warm ? P.warm : nullptr, warm ? &st->warm_alpha : nullptr);
}

// Every instance's p_G of version ver into its row of the network's input (one block each).
__global__ __launch_bounds__(256) void kb_gather_traces(const BInst* __restrict__ I, int ver,
                                                        int skip_done) {
  const BInst& P = I[blockIdx.x];
  if (!P.trace || inst_idle(P.st, skip_done)) return;
  const double* src = P.pG[ver & 1];
  for (int i = threadIdx.x; i < P.ng; i += blockDim.x) P.trace[i] = src[i];
}

// Tile partials of f.g and g.A g for every instance's guess g (over the level-0 tile list).
__global__ __launch_bounds__(kBlock) void kb_warm_dots(const BInst* __restrict__ I, BLists L,
                                                       int ver, int skip_done) {
  const int b = xcd_linear();
  const int* start = L.tiles[0];
  const int i = find_inst(start, L.ninst, b);
  const BInst& P = I[i];
  if (!P.warm || inst_idle(P.st, skip_done)) return;
  const int t = b - first_tile(start, i);
  const int tx = P.tiles_x[0];
  d_warm_dots(b_rhs(P, kRhsLiftP, ver), P.warm, P.nf[0], P.red, t % tx, t / tx, t);
}

__global__ __launch_bounds__(kBlock) void kb_warm_alpha(const BInst* __restrict__ I,
                                                        int skip_done) {
  const BInst& P = I[blockIdx.x];
  if (!P.warm || inst_idle(P.st, skip_done)) return;
  d_warm_alpha(P.st, P.red);
}

__global__ __launch_bounds__(kBlock) void kb_ir_finalize(const BInst* __restrict__ I,
                                                         int skip_done) {
  const BInst& P = I[blockIdx.x];
  if (inst_idle(P.st, skip_done)) return;
  d_ir_finalize(P.st, P.red);
}

// which = 0: preconditioner batch on r (sel 0: r_G[0], sel 1: r_G[(ver + 1) & 1], part of the
// outer tail); which = 1: operator batch on p_G[ver & 1].
__global__ __launch_bounds__(kIfaceThreads) void kb_iface_solve(const BInst* __restrict__ I,
                                                                BLists L, int which, int sel,
                                                                int ver, int skip_done) {
  const int b = blockIdx.x;
  const int* start = which ? L.sysH : L.sysP;
  const int i = find_inst(start, L.ninst, b);
  const BInst& P = I[i];
  if (which == 0 && sel ? tail_idle(P.st, skip_done) : inst_idle(P.st, skip_done)) return;
  const int k = b - first_tile(start, i);
  const ShiftTable* tab = which ? P.tabH : P.tabP;
  const double* in = which ? P.pG[ver & 1] : (sel ? P.rG[(ver + 1) & 1] : P.rG[0]);
  double* out = (which ? P.scrH : P.scrP) + (size_t)k * P.ng;
  d_iface_solve(P.ng, P.h, tab->alpha[k], tab->beta[k], tab->coef[k],
                which ? kIfaceOperator : kIfacePrecond, in, out);
}

__global__ __launch_bounds__(kIfaceThreads) void kb_iface_combine(const BInst* __restrict__ I,
                                                                  int which, int ver, int first,
                                                                  double rtol2, int skip_done) {
  const BInst& P = I[blockIdx.x];
  if (which == 0 && !first ? tail_idle(P.st, skip_done) : inst_idle(P.st, skip_done)) return;
  if (which) {
    d_iface_combine(P.ng, P.h, P.mH, P.tabH->d0, kIfaceOperator, P.pG[ver & 1], P.Hp, P.scrH,
                    P.st, nullptr, nullptr, ver, 0, -1.0);
  } else {
    const double* r = first ? P.rG[0] : P.rG[(ver + 1) & 1];
    double* pn = first ? P.pG[0] : P.pG[(ver + 1) & 1];
    d_iface_combine(P.ng, P.h, P.mP, 0.0, kIfacePrecondOuter, r, P.zG, P.scrP, P.st,
                    P.pG[ver & 1], pn, ver, first, rtol2);
  }
}

__global__ __launch_bounds__(kIfaceThreads) void kb_schur_gather(const BInst* __restrict__ I,
                                                                 int S, int ver, int skip_done) {
  const BInst& P = I[blockIdx.x];
  if (tail_idle(P.st, skip_done)) return;
  const int a = ver & 1, bb = (ver + 1) & 1;
  d_schur_gather(P.ng, P.nf[0], P.pitch[0], P.K, P.gamma, P.pG[a], P.u64[S & 1], P.Hp, P.yG,
                 P.xG[a], P.xG[bb], P.rG[a], P.rG[bb], P.st, 1, ver);
}

// g = b_G + u|row nf, x_G = 0, and the outer state of every instance reset.
__global__ __launch_bounds__(256) void kb_rhs_reduce(const BInst* __restrict__ I, int S) {
  const BInst& P = I[blockIdx.x];
  const size_t row = (size_t)(P.nf[0] - 1) * P.pitch[0];
  const double* u = P.u64[S & 1];
  const double* bG = P.b + (size_t)P.nf[0] * P.nf[0];
  for (int i = threadIdx.x; i < P.ng; i += blockDim.x) {
    P.rG[0][i] = bG[i] + u[row + i];
    P.xG[0][i] = 0.0;
  }
  if (threadIdx.x == 0) {
    P.st->outer_done = 0;
    P.st->o_ver = 0;
    P.st->o_its = 0;
  }
}

// Interior accumulator over the level-0 tile list: init = 1: x_I(0) = u / K; init = 0:
// x_I(ver+1) = x_I(ver) + alpha u (alpha from the Schur product of this iteration), with u the
// interior solve's FP64 result.  Runs with the outer tail (after the Schur product, before the
// convergence test may retire the instance).
__global__ __launch_bounds__(kBlock) void kb_interior_axpy(const BInst* __restrict__ I, BLists L,
                                                           int S, int ver, int init,
                                                           int skip_done) {
  const int b = xcd_linear();
  const int* start = L.tiles[0];
  const int i = find_inst(start, L.ninst, b);
  const BInst& P = I[i];
  if (!init && tail_idle(P.st, skip_done)) return;
  const int t = b - first_tile(start, i);
  const int tx = P.tiles_x[0];
  const int i0 = (t % tx) * kTile, j0 = (t / tx) * kTile;
  const int nf = P.nf[0], pitch = P.pitch[0];
  const double* u = P.u64[S & 1];
  const double c = init ? 1.0 / P.K : P.st->o_alpha;
  const double* a = init ? nullptr : P.xI[ver & 1];
  double* out = init ? P.xI[0] : P.xI[(ver + 1) & 1];
  for (int q = flat_tid(); q < kTile * kTile; q += kBlock) {
    const int ii = i0 + (q % kTile), jj = j0 + q / kTile;
    if (ii >= nf || jj >= nf) continue;
    const unsigned o = (unsigned)(jj * pitch + ii);
    stg(out, o, (a ? ldg(a, o) : 0.0) + c * ldg(u, o));
  }
}

// Interior solution (padded) and the final interface iterate into the caller's vector.
__global__ __launch_bounds__(256) void kb_scatter(const BInst* __restrict__ I, int S, int ver,
                                                  int from_xI) {
  const BInst& P = I[blockIdx.x];
  const int nf = P.nf[0];
  const int64_t NI = (int64_t)nf * nf;
  const double* u = from_xI ? P.xI[final_ver(P.st, ver) & 1] : P.u64[S & 1];
  const double* xG = P.xG[final_ver(P.st, ver) & 1];
  for (int64_t k = threadIdx.x + (int64_t)blockIdx.y * blockDim.x; k < NI + nf;
       k += (int64_t)blockDim.x * gridDim.y) {
    if (k < NI) P.xout[k] = u[(size_t)(k / nf) * P.pitch[0] + (k % nf)];
    else P.xout[k] = xG[k - NI];
  }
}

// Copies every instance's DevState into one array (one read-back per synchronization).
__global__ void kb_gather_states(const BInst* __restrict__ I, int ninst, DevState* out) {
  const int i = blockIdx.x;
  if (i >= ninst) return;
  const unsigned* src = reinterpret_cast<const unsigned*>(I[i].st);
  unsigned* dst = reinterpret_cast<unsigned*>(out + i);
  for (int w = threadIdx.x; w < (int)(sizeof(DevState) / 4); w += blockDim.x) dst[w] = src[w];
}

// ---- launchers ------------------------------------------------------------------------------

static inline dim3 tb() { return dim3(32, kBlock / 32); }

template <int NU>
static void b_tail(const BatchCtx& c, int check) {
  for (int l = 1; l < c.max_tiled; ++l) {
    if (c.tiles_total[l] == 0) continue;
    if (c.tile_edge[l] == kMidTile)
      hipLaunchKernelGGL((kb_mg_down<NU, false, kMidTile>), dim3(c.tiles_total[l]), tb(), 0,
                         c.stream, c.inst, c.lists, l, 0, 0, 0, check, c.skip_done);
    else
      hipLaunchKernelGGL((kb_mg_down<NU, false, kTile>), dim3(c.tiles_total[l]), tb(), 0,
                         c.stream, c.inst, c.lists, l, 0, 0, 0, check, c.skip_done);
  }
  launch_timed(c.hook, kTimeCoarse, kb_coarse, dim3(c.lists.ninst), dim3(kCoarseThreads),
               c.stream, c.inst, check, c.skip_done);
  for (int l = c.max_tiled - 1; l >= 1; --l) {
    if (c.tiles_total[l] == 0) continue;
    if (c.tile_edge[l] == kMidTile)
      hipLaunchKernelGGL((kb_mg_up<NU, false, kMidTile>), dim3(c.tiles_total[l]), tb(), 0,
                         c.stream, c.inst, c.lists, l, 0, 0, 0, c.skip_done);
    else
      hipLaunchKernelGGL((kb_mg_up<NU, false, kTile>), dim3(c.tiles_total[l]), tb(), 0,
                         c.stream, c.inst, c.lists, l, 0, 0, 0, c.skip_done);
  }
}

template <int NU>
static void b_step(const BatchCtx& c, int rhs, int ver, int its, int S, int& cur_r, int& cur_p) {
  // PCG start: z = V r, w = A z, r.z and z.w
  hipLaunchKernelGGL((kb_mg_down<NU, false, kTile>), dim3(c.tiles_total[0]), tb(), 0, c.stream,
                     c.inst, c.lists, 0, 0, cur_r, cur_p, 0, c.skip_done);
  b_tail<NU>(c, 0);
  hipLaunchKernelGGL((kb_mg_up<NU, true, kTile>), dim3(c.tiles_total[0]), tb(), 0, c.stream,
                     c.inst, c.lists, 0, 0, 0, cur_r, c.skip_done);
  for (int k = 0; k < its; ++k) {
    hipLaunchKernelGGL(kb_dots, dim3(c.lists.ninst), tb(), 0, c.stream, c.inst, k, c.skip_done);
    launch_timed(c.hook, kTimeDown0, kb_mg_down<NU, true, kTile>, dim3(c.tiles_total[0]), tb(),
                 c.stream,
                 c.inst, c.lists, 0, k, cur_r, cur_p, 0, c.skip_done);
    if (k == its - 1) {
      // the refinement residual follows: no V-cycle for a z that would not be used
      hipLaunchKernelGGL(kb_run_check, dim3(c.lists.ninst), tb(), 0, c.stream, c.inst,
                         c.skip_done);
      cur_r ^= 1;
      cur_p ^= 1;
      break;
    }
    b_tail<NU>(c, 1);
    launch_timed(c.hook, kTimeUp0, kb_mg_up<NU, true, kTile>, dim3(c.tiles_total[0]), tb(),
                 c.stream,
                 c.inst, c.lists, 0, k + 1, 1, cur_r ^ 1, c.skip_done);
    cur_r ^= 1;
    cur_p ^= 1;
  }
  hipLaunchKernelGGL(kb_ir_residual, dim3(c.tiles_total[0]), tb(), 0, c.stream, c.inst, c.lists,
                     0, rhs, ver, S, cur_r, 0.0, 0.0, c.skip_done);
  hipLaunchKernelGGL(kb_ir_finalize, dim3(c.lists.ninst), dim3(kBlock), 0, c.stream, c.inst,
                     c.skip_done);
}

void launch_b_inner_start(const BatchCtx& c, int rhs, int ver, double tol2, double tau2) {
  hipLaunchKernelGGL(kb_ir_residual, dim3(c.tiles_total[0]), tb(), 0, c.stream, c.inst, c.lists,
                     1, rhs, ver, 0, 0, tol2, tau2, c.skip_done);
  hipLaunchKernelGGL(kb_ir_finalize, dim3(c.lists.ninst), dim3(kBlock), 0, c.stream, c.inst,
                     c.skip_done);
}

void launch_b_inner_step(const BatchCtx& c, int rhs, int ver, int its, int S, int& cur_r,
                         int& cur_p) {
  if (c.nu == 2) b_step<2>(c, rhs, ver, its, S, cur_r, cur_p);
  else b_step<1>(c, rhs, ver, its, S, cur_r, cur_p);
}

void launch_b_gather_traces(const BatchCtx& c, int ver) {
  hipLaunchKernelGGL(kb_gather_traces, dim3(c.lists.ninst), dim3(256), 0, c.stream, c.inst, ver,
                     c.skip_done);
}

void launch_b_warm_alpha(const BatchCtx& c, int ver) {
  hipLaunchKernelGGL(kb_warm_dots, dim3(c.tiles_total[0]), tb(), 0, c.stream, c.inst, c.lists, ver,
                     c.skip_done);
  hipLaunchKernelGGL(kb_warm_alpha, dim3(c.lists.ninst), dim3(kBlock), 0, c.stream, c.inst,
                     c.skip_done);
}

void launch_b_rhs_reduce(const BatchCtx& c, int S) {
  hipLaunchKernelGGL(kb_rhs_reduce, dim3(c.lists.ninst), dim3(256), 0, c.stream, c.inst, S);
}

void launch_b_precond_init(const BatchCtx& c, double rtol) {
  hipLaunchKernelGGL(kb_iface_solve, dim3(c.sysP_total), dim3(kIfaceThreads), 0, c.stream, c.inst,
                     c.lists, 0, 0, 0, 0);
  hipLaunchKernelGGL(kb_iface_combine, dim3(c.lists.ninst), dim3(kIfaceThreads), 0, c.stream,
                     c.inst, 0, 0, 1, rtol * rtol, 0);
}

void launch_b_operator(const BatchCtx& c, int v) {
  hipLaunchKernelGGL(kb_iface_solve, dim3(c.sysH_total), dim3(kIfaceThreads), 0, c.stream, c.inst,
                     c.lists, 1, 0, v, c.skip_done);
  hipLaunchKernelGGL(kb_iface_combine, dim3(c.lists.ninst), dim3(kIfaceThreads), 0, c.stream,
                     c.inst, 1, v, 0, -1.0, c.skip_done);
}

void launch_b_xI_init(const BatchCtx& c, int S) {
  hipLaunchKernelGGL(kb_interior_axpy, dim3(c.tiles_total[0]), tb(), 0, c.stream, c.inst, c.lists,
                     S, 0, 1, 0);
}

void launch_b_outer_tail(const BatchCtx& c, int S, int v, double rtol, bool accumulate) {
  hipLaunchKernelGGL(kb_schur_gather, dim3(c.lists.ninst), dim3(kIfaceThreads), 0, c.stream,
                     c.inst, S, v, c.skip_done);
  if (accumulate)
    hipLaunchKernelGGL(kb_interior_axpy, dim3(c.tiles_total[0]), tb(), 0, c.stream, c.inst,
                       c.lists, S, v, 0, c.skip_done);
  hipLaunchKernelGGL(kb_iface_solve, dim3(c.sysP_total), dim3(kIfaceThreads), 0, c.stream, c.inst,
                     c.lists, 0, 1, v, c.skip_done);
  hipLaunchKernelGGL(kb_iface_combine, dim3(c.lists.ninst), dim3(kIfaceThreads), 0, c.stream,
                     c.inst, 0, v, 0, rtol * rtol, c.skip_done);
}

void launch_b_scatter(const BatchCtx& c, int S, int ver, bool from_xI) {
  hipLaunchKernelGGL(kb_scatter, dim3(c.lists.ninst, 64), dim3(256), 0, c.stream, c.inst, S, ver,
                     from_xI ? 1 : 0);
}

void launch_b_gather_states(const BatchCtx& c, DevState* out) {
  hipLaunchKernelGGL(kb_gather_states, dim3(c.lists.ninst), dim3(64), 0, c.stream, c.inst,
                     c.lists.ninst, out);
}

}  // namespace fdd
