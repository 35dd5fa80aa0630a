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
//     neighbour.  The first level with at most 63 x 63 points is solved in one workgroup: in
//     FP32 exactly, by sine transforms on the matrix cores; in FP64 by a V-cycle in LDS down to
//     a dense inverse on the coarsest grid.
//   - The PCG runs in its single-reduction form (Chronopoulos and Gear 1989): the vector updates
//     are fused into the level-0 down kernel, w = A z into the level-0 up kernel, and r . z and
//     z . A z are reduced together, so an iteration is one V-cycle and nothing else.
//   - Dot products are reduced without atomics or fences: every block stores its partial sum,
//     and each block of the kernel that needs the scalar sums all partials in the same fixed
//     order (kernel boundaries make the partials visible), so every block sees bit-identical
//     scalars and the result is deterministic.
//   - Scalars and flags stay on the device; every kernel returns at once when its solve has
//     converged, so the host can enqueue (or replay as a graph) a fixed schedule.
#include "mg_device.h"

namespace fdd {

// --------------------------------------------------------------------------------------------
// single-instance kernels
// --------------------------------------------------------------------------------------------

template <typename T, int NU, bool CG, int TT = kTile, bool RESIDENT = false>
__global__ __launch_bounds__(kBlock) void k_mg_down(
    const T* __restrict__ fin, T* __restrict__ uout, T* __restrict__ fc, int nf, int pitch,
    int pc, const T* __restrict__ z, const T* __restrict__ pold, T* __restrict__ pnew,
    T* __restrict__ x, T* __restrict__ rout, DevState* st, Reductions red, int k, int check,
    int finalize, int presum) {
  if (finalize) {
    // the kernel that starts a PCG run after a refinement residual also does that step's
    // bookkeeping (instead of a one-block kernel of its own)
    if (ir_finalize_here(st, red, block0())) return;
  } else {
    if (stopped(st)) return;
    if (check && pcg_converged(st, red, block0())) return;
  }
  int tile_x, tile_y;
  const int tile = xcd_tile(&tile_x, &tile_y);
  d_mg_down<T, NU, CG, TT, RESIDENT>(fin, uout, fc, nf, pitch, pc, z, pold, pnew, x, rout, st,
                                     red, k, tile_x, tile_y, tile, block0(), presum != 0);
}

__global__ __launch_bounds__(kBlock) void k_sum_dots(DevState* st, Reductions red, int k) {
  if (stopped(st)) return;
  d_sum_dots(red, k, st);
}

template <typename T, int NU, bool CG, int TT = kTile>
__global__ __launch_bounds__(kBlock) void k_mg_up(
    const T* __restrict__ fin, const T* __restrict__ upre, const T* __restrict__ ec,
    T* __restrict__ eout, int nf, int pitch, int pc, DevState* st, Reductions red, int kn,
    int count_iteration) {
  if (stopped(st)) return;
  int tile_x, tile_y;
  const int tile = xcd_tile(&tile_x, &tile_y);
  d_mg_up<T, NU, CG, TT>(fin, upre, ec, eout, nf, pitch, pc, st, red, kn, count_iteration,
                         tile_x, tile_y, tile, block0());
}

template <typename T, int NU>
__global__ __launch_bounds__(kPairThreads) void k_pair_down(
    const T* __restrict__ fin0, T* __restrict__ uout0, T* __restrict__ fout1,
    T* __restrict__ uout1, T* __restrict__ fout2, int nf0, int p0, int p1, int p2, DevState* st,
    Reductions red, int check) {
  if (stopped(st)) return;
  if (check && pcg_converged(st, red, block0())) return;
  int tile_x, tile_y;
  (void)xcd_tile(&tile_x, &tile_y);
  d_pair_down<T, NU>(fin0, uout0, fout1, uout1, fout2, nf0, p0, p1, p2, tile_x, tile_y);
}

template <typename T, int NU>
__global__ __launch_bounds__(kPairThreads) void k_pair_up(
    const T* __restrict__ f0, const T* __restrict__ u0pre, const T* __restrict__ f1,
    const T* __restrict__ u1pre, const T* __restrict__ e2, T* __restrict__ eout0, int nf0, int p0,
    int p1, int p2, DevState* st) {
  if (stopped(st)) return;
  int tile_x, tile_y;
  (void)xcd_tile(&tile_x, &tile_y);
  d_pair_up<T, NU>(f0, u0pre, f1, u1pre, e2, eout0, nf0, p0, p1, p2, tile_x, tile_y);
}

template <int NU>
__global__ __launch_bounds__(kPairThreads) void k_triple_up(
    const float* __restrict__ f0, const float* __restrict__ u0pre, const float* __restrict__ f1,
    const float* __restrict__ u1pre, const float* __restrict__ f2, const float* __restrict__ u2pre,
    const float* __restrict__ f3, const float* __restrict__ S, const float* __restrict__ lam,
    float* __restrict__ eout0, int nf0, int p0, int p1, int p2, int p3, DevState* st) {
  if (stopped(st)) return;
  int tile_x, tile_y;
  (void)xcd_tile(&tile_x, &tile_y);
  d_triple_up<NU>(f0, u0pre, f1, u1pre, f2, u2pre, f3, S, lam, eout0, nf0, p0, p1, p2, p3, tile_x,
                  tile_y);
}

template <int NU>
__global__ __launch_bounds__(kPairThreads) void k_quad_up(
    const float* __restrict__ f0, const float* __restrict__ u0pre, const float* __restrict__ f1,
    const float* __restrict__ u1pre, const float* __restrict__ f2, const float* __restrict__ u2pre,
    const float* __restrict__ f3, const float* __restrict__ u3pre, const float* __restrict__ f4,
    const float* __restrict__ S, const float* __restrict__ lam, float* __restrict__ z, int nf0,
    int p0, int p1, int p2, int p3, int p4, DevState* st, Reductions red, int kn,
    int count_iteration) {
  if (stopped(st)) return;
  int tile_x, tile_y;
  (void)xcd_tile(&tile_x, &tile_y);
  d_quad_up<NU>(f0, u0pre, f1, u1pre, f2, u2pre, f3, u3pre, f4, S, lam, z, nf0, p0, p1, p2, p3, p4,
                st, red, kn, count_iteration, tile_x, tile_y, block0());
}

template <typename T, int NU>
__global__ __launch_bounds__(kCoarseThreads) void k_coarse_vcycle(
    const T* __restrict__ fin, int pin, T* __restrict__ eout, LaunchLevels lv,
    const T* __restrict__ cinv, DevState* st, Reductions red, int check) {
  if (stopped(st)) return;
  if (check && pcg_converged(st, red, true)) return;
  d_coarse_vcycle<T, NU>(fin, pin, eout, lv, cinv);
}

__global__ __launch_bounds__(kCoarseThreads) void k_coarse_dst(
    const float* __restrict__ fin, int pin, float* __restrict__ eout, int m,
    const float* __restrict__ S, const float* __restrict__ lam, DevState* st, Reductions red,
    int check) {
  if (stopped(st)) return;
  if (check && pcg_converged(st, red, true)) return;
  d_coarse_dst(fin, pin, eout, m, S, lam);
}

template <typename E>
__global__ __launch_bounds__(kBlock) void k_ir_residual(
    RhsDesc f, const double* __restrict__ uin, const E* __restrict__ e, double* __restrict__ uout,
    float* __restrict__ r32, double* __restrict__ r64, int nf, int pitch, int first, double tol2,
    double tau2, int pcg_is_final, DevState* st, Reductions red, const float* __restrict__ warm,
    const double* __restrict__ wscale, int run_check) {
  int tile_x, tile_y;
  const int tile = xcd_tile(&tile_x, &tile_y);
  d_ir_residual<E>(f, uin, e, uout, r32, r64, nf, pitch, first, tol2, tau2, pcg_is_final, st, red,
                   tile_x, tile_y, tile, block0(), warm, wscale, run_check != 0);
}

__global__ __launch_bounds__(kBlock) void k_warm_dots(RhsDesc f, const float* __restrict__ g,
                                                      int nf, Reductions red) {
  d_warm_dots(f, g, nf, red, blockIdx.x, blockIdx.y, blockIdx.y * gridDim.x + blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void k_warm_alpha(DevState* st, Reductions red) {
  d_warm_alpha(st, red);
}

__global__ __launch_bounds__(kBlock) void k_ir_finalize(DevState* st, Reductions red) {
  d_ir_finalize(st, red);
}

// --------------------------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------------------------

static inline dim3 tiles(int nf) {
  const int t = (nf + kTile - 1) / kTile;
  return dim3(t, t);
}
static inline dim3 tblock() { return dim3(32, kBlock / 32); }
static inline dim3 mtiles(int nf) {
  const int t = (nf + kMidTile - 1) / kMidTile;
  return dim3(t, t);
}
static inline dim3 ptiles(int nf) {
  const int t = (nf + kPairTile - 1) / kPairTile;
  return dim3(t, t);
}

// FP32 V-cycles whose tiled levels below the finest are exactly 1, 2, 3 (the coarse solve on level
// 4; n = 1024 and 768): the whole up side runs as one kernel (k_quad_up) in the CG iterations
template <typename T>
static bool quad_up(const LaunchCtx& c) {
  return sizeof(T) == 4 && c.first_coarse == 4 && c.nlev >= 5;
}

template <typename T, int NU>
static void vcycle_tail_nu(const LaunchCtx& c, const MGBuffers<T>& mg, int check,
                           bool skip_up = false) {
  // levels 1 .. first_coarse-1 go down, the coarse kernel, then back up to level 1; in FP32 the
  // tiled levels run in pairs (1, 2), (3, 4), ... in one kernel each, an odd last one alone (the
  // FP64 windows of a pair exceed the LDS); the first of these kernels also runs the PCG
  // convergence test when `check` is set
  const int fc = c.first_coarse;
  const dim3 pblock(32, kPairThreads / 32);
  constexpr bool kPairs = sizeof(T) == 4;
  auto pair = [&](int l) { return kPairs && l + 1 < fc; };  // l odd: does level l start a pair?
  for (int l = 1; l < fc; l += pair(l) ? 2 : 1) {
    const Level& L = c.lev[l];
    const int chk = l == 1 ? check : 0;
    if (pair(l)) {
      if constexpr (kPairs)
        hipLaunchKernelGGL((k_pair_down<float, NU>), ptiles(c.lev[l + 1].nf), pblock, 0, c.stream,
                           (const float*)mg.f[l], mg.u[l], mg.f[l + 1], mg.u[l + 1], mg.f[l + 2],
                           L.nf, L.pitch, c.lev[l + 1].pitch, c.lev[l + 2].pitch, c.st, c.red, chk);
    } else {
      // (in FP32 a level that runs alone is the last tiled one, at most 127^2 points: 64 tiles,
      // all in flight at once)
      hipLaunchKernelGGL((k_mg_down<T, NU, false, kMidTile, sizeof(T) == 4>), mtiles(L.nf),
                         tblock(), 0, c.stream, mg.f[l], mg.u[l], mg.f[l + 1], L.nf, L.pitch,
                         c.lev[l + 1].pitch,
                         (const T*)nullptr, (const T*)nullptr, (T*)nullptr, (T*)nullptr,
                         (T*)nullptr, c.st, c.red, 0, chk, 0, 0);
    }
  }
  // (FP32 with an odd number of at least three tiled levels: the coarse solve runs inside the
  // three-level up kernel)
  const bool triple = kPairs && fc - 1 >= 3 && (fc - 1) % 2 == 1;
  if constexpr (sizeof(T) == 4) {
    if (!triple)
      launch_timed(c.hook, kTimeCoarse, k_coarse_dst, dim3(1), dim3(kCoarseThreads), c.stream,
                   (const float*)mg.f[fc], c.lev[fc].pitch, (float*)mg.e[fc], c.lev[fc].nf,
                   c.dst_S, c.dst_lam, c.st, c.red, fc == 1 ? check : 0);
  } else {
    LaunchLevels lv;
    lv.first = fc;
    lv.nlev = c.nlev;
    for (int l = 0; l < c.nlev; ++l) lv.nf[l] = c.lev[l].nf;
    launch_timed(c.hook, kTimeCoarse, k_coarse_vcycle<T, NU>, dim3(1), dim3(kCoarseThreads),
                 c.stream, (const T*)mg.f[fc], c.lev[fc].pitch, mg.e[fc], lv,
                 (const T*)c.coarse_inv64, c.st, c.red, fc == 1 ? check : 0);
  }
  // going up: an odd last tiled level alone, then the pairs from the bottom (FP64: every level
  // alone)
  const int ntiled = fc - 1;
  int l = fc - 1;
  for (; !kPairs && l >= 1; --l) {
    const Level& L = c.lev[l];
    hipLaunchKernelGGL((k_mg_up<T, NU, false, kMidTile>), mtiles(L.nf), tblock(), 0, c.stream,
                       mg.f[l], mg.u[l], mg.e[l + 1], mg.e[l], L.nf, L.pitch, c.lev[l + 1].pitch,
                       c.st, c.red, 0, 0);
  }
  if (skip_up) return;  // the caller's k_quad_up does the up side
  if (kPairs && ntiled % 2 == 1) {
    if constexpr (kPairs) {
      if (ntiled >= 3) {
        // the coarse solve, the level that ran alone and the pair above it, in one kernel
        const int a = l - 2;
        hipLaunchKernelGGL((k_triple_up<NU>), ptiles(c.lev[a + 1].nf), pblock, 0, c.stream,
                           (const float*)mg.f[a], (const float*)mg.u[a],
                           (const float*)mg.f[a + 1], (const float*)mg.u[a + 1],
                           (const float*)mg.f[a + 2], (const float*)mg.u[a + 2],
                           (const float*)mg.f[a + 3], c.dst_S, c.dst_lam, mg.e[a], c.lev[a].nf,
                           c.lev[a].pitch, c.lev[a + 1].pitch, c.lev[a + 2].pitch,
                           c.lev[a + 3].pitch, c.st);
        l -= 3;
      } else {
        const Level& L = c.lev[l];
        hipLaunchKernelGGL((k_mg_up<T, NU, false, kMidTile>), mtiles(L.nf), tblock(), 0,
                           c.stream, mg.f[l], mg.u[l], mg.e[l + 1], mg.e[l], L.nf, L.pitch,
                           c.lev[l + 1].pitch, c.st, c.red, 0, 0);
        --l;
      }
    }
  }
  if constexpr (kPairs) {
    for (; l >= 2; l -= 2) {
      const int a = l - 1;  // the pair (a, a + 1)
      hipLaunchKernelGGL((k_pair_up<float, NU>), ptiles(c.lev[a + 1].nf), pblock, 0, c.stream,
                         (const float*)mg.f[a], (const float*)mg.u[a], (const float*)mg.f[a + 1],
                         (const float*)mg.u[a + 1], (const float*)mg.e[a + 2], mg.e[a],
                         c.lev[a].nf, c.lev[a].pitch, c.lev[a + 1].pitch, c.lev[a + 2].pitch,
                         c.st);
    }
  }
}

template <int NU>
static void launch_quad_up(const LaunchCtx& c, const MGBuffers<float>& mg, const float* r, float* z,
                           int kn, int count_iteration) {
  const dim3 pblock(32, kPairThreads / 32);
  launch_timed(c.hook, kTimeUp0, k_quad_up<NU>, ptiles(c.lev[2].nf), pblock, c.stream, r,
               (const float*)mg.u[0], (const float*)mg.f[1], (const float*)mg.u[1],
               (const float*)mg.f[2], (const float*)mg.u[2], (const float*)mg.f[3],
               (const float*)mg.u[3], (const float*)mg.f[4], c.dst_S, c.dst_lam, z, c.lev[0].nf,
               c.lev[0].pitch, c.lev[1].pitch, c.lev[2].pitch, c.lev[3].pitch, c.lev[4].pitch,
               c.st, c.red, kn, count_iteration);
}

template <typename T, int NU>
static void pcg_init_nu(const LaunchCtx& c, const MGBuffers<T>& mg, const T* r, T* z) {
  const Level& L = c.lev[0];
  // (FP32 grids of at most kResidentTiles tiles: the RESIDENT form, as in the iterations)
  auto down0 = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, tiles(L.nf), tblock(), 0, c.stream, r, mg.u[0], mg.f[1], L.nf,
                       L.pitch, c.lev[1].pitch, (const T*)nullptr, (const T*)nullptr, (T*)nullptr,
                       (T*)nullptr, (T*)nullptr, c.st, c.red, 0, 0, 1, 0);
  };
  if constexpr (sizeof(T) == 4) {
    if (c.red.nb0 <= kResidentTiles) down0(k_mg_down<T, NU, false, kTile, true>);
    else down0(k_mg_down<T, NU, false, kTile, false>);
  } else {
    down0(k_mg_down<T, NU, false, kTile, false>);
  }
  const bool quad = quad_up<T>(c);
  vcycle_tail_nu<T, NU>(c, mg, 0, quad);
  if (quad) {
    if constexpr (sizeof(T) == 4) launch_quad_up<NU>(c, mg, r, z, 0, 0);
    return;
  }
  hipLaunchKernelGGL((k_mg_up<T, NU, true>), tiles(L.nf), tblock(), 0, c.stream, r, mg.u[0],
                     mg.e[1], z, L.nf, L.pitch, c.lev[1].pitch, c.st, c.red, 0, 0);
}

template <typename T>
void launch_pcg_init(const LaunchCtx& c, const MGBuffers<T>& mg, const T* r, T* z) {
  if (c.nu == 2) pcg_init_nu<T, 2>(c, mg, r, z);
  else pcg_init_nu<T, 1>(c, mg, r, z);
}

template <typename T, int NU>
static void vcycle_nu(const LaunchCtx& c, const MGBuffers<T>& mg, const T* f, T* z) {
  const Level& L = c.lev[0];
  auto down0 = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, tiles(L.nf), tblock(), 0, c.stream, f, mg.u[0], mg.f[1], L.nf,
                       L.pitch, c.lev[1].pitch, (const T*)nullptr, (const T*)nullptr, (T*)nullptr,
                       (T*)nullptr, (T*)nullptr, c.st, c.red, 0, 0, 0, 0);
  };
  if constexpr (sizeof(T) == 4) {
    if (c.red.nb0 <= kResidentTiles) down0(k_mg_down<T, NU, false, kTile, true>);
    else down0(k_mg_down<T, NU, false, kTile, false>);
  } else {
    down0(k_mg_down<T, NU, false, kTile, false>);
  }
  vcycle_tail_nu<T, NU>(c, mg, 0);
  hipLaunchKernelGGL((k_mg_up<T, NU, false>), tiles(L.nf), tblock(), 0, c.stream, f, mg.u[0],
                     mg.e[1], z, L.nf, L.pitch, c.lev[1].pitch, c.st, c.red, 0, 0);
}

template <typename T>
void launch_vcycle(const LaunchCtx& c, const MGBuffers<T>& mg, const T* f, T* z) {
  if (c.nu == 2) vcycle_nu<T, 2>(c, mg, f, z);
  else vcycle_nu<T, 1>(c, mg, f, z);
}

// The reductions as the level-0 down kernel of a PCG iteration reads them: the quad up kernel
// stores one r.z and one z.A z partial per block (64 x 64 level-0 cells), the finest up kernel
// one per 32 x 32 tile.
template <typename T>
static Reductions dot_red(const LaunchCtx& c) {
  Reductions red = c.red;
  if (quad_up<T>(c)) {
    const dim3 g = ptiles(c.lev[2].nf);
    red.nbd = (int)(g.x * g.y);
  }
  return red;
}

template <typename T, int NU>
static void pcg_iter_nu(const LaunchCtx& c, const MGBuffers<T>& mg, int k, T* x, T* r_old,
                        T* r_new, T* z, T* p_old, T* p_new, bool update_only) {
  const Level& L = c.lev[0];
  // beyond kPresumTiles tiles the dot products are summed once, by one block, instead of by
  // every block of the down kernel (same order, same values)
  const int presum = c.red.nb0 > kPresumTiles ? 1 : 0;
  const Reductions red = dot_red<T>(c);
  if (presum) hipLaunchKernelGGL(k_sum_dots, dim3(1), dim3(kBlock), 0, c.stream, c.st, red, k);
  // FP32 grids of at most kResidentTiles tiles run the down kernel's RESIDENT form (every tile
  // in flight at once, four blocks per compute unit)
  auto down0 = [&](auto kernel) {
    launch_timed(c.hook, kTimeDown0, kernel, tiles(L.nf), tblock(), c.stream, (const T*)r_old,
                 mg.u[0], mg.f[1], L.nf, L.pitch, c.lev[1].pitch, (const T*)z, (const T*)p_old,
                 p_new, x, r_new, c.st, red, k, 0, 0, presum);
  };
  if constexpr (sizeof(T) == 4) {
    if (c.red.nb0 <= kResidentTiles) down0(k_mg_down<T, NU, true, kTile, true>);
    else down0(k_mg_down<T, NU, true, kTile, false>);
  } else {
    down0(k_mg_down<T, NU, true, kTile, false>);
  }
  if (update_only) return;  // the refinement residual that follows takes the run's test
  const bool quad = quad_up<T>(c);
  vcycle_tail_nu<T, NU>(c, mg, 1, quad);
  if (quad) {
    if constexpr (sizeof(T) == 4) launch_quad_up<NU>(c, mg, r_new, z, k + 1, 1);
    return;
  }
  launch_timed(c.hook, kTimeUp0, k_mg_up<T, NU, true>, tiles(L.nf), tblock(), c.stream,
               (const T*)r_new, (const T*)mg.u[0], (const T*)mg.e[1], z, L.nf, L.pitch,
               c.lev[1].pitch, c.st, c.red, k + 1, 1);
}

template <typename T>
void launch_pcg_iteration(const LaunchCtx& c, const MGBuffers<T>& mg, int k, T* x, T* r_old,
                          T* r_new, T* z, T* p_old, T* p_new, bool update_only) {
  if (c.nu == 2) pcg_iter_nu<T, 2>(c, mg, k, x, r_old, r_new, z, p_old, p_new, update_only);
  else pcg_iter_nu<T, 1>(c, mg, k, x, r_old, r_new, z, p_old, p_new, update_only);
}

void launch_ir_residual(const LaunchCtx& c, const RhsDesc& f, const double* uin, const float* e32,
                        const double* e64, double* uout, float* r32, double* r64, int first,
                        double tol2, double tau2, int pcg_is_final, const float* warm,
                        const double* wscale, bool finalize, bool run_check) {
  const Level& L = c.lev[0];
  if (e64 || !e32)
    hipLaunchKernelGGL((k_ir_residual<double>), tiles(L.nf), tblock(), 0, c.stream, f, uin, e64,
                       uout, r32, r64, L.nf, L.pitch, first, tol2, tau2, pcg_is_final, c.st,
                       c.red, warm, wscale, run_check ? 1 : 0);
  else
    hipLaunchKernelGGL((k_ir_residual<float>), tiles(L.nf), tblock(), 0, c.stream, f, uin, e32,
                       uout, r32, r64, L.nf, L.pitch, first, tol2, tau2, pcg_is_final, c.st,
                       c.red, warm, wscale, run_check ? 1 : 0);
  if (finalize) hipLaunchKernelGGL(k_ir_finalize, dim3(1), dim3(kBlock), 0, c.stream, c.st, c.red);
}

void launch_warm_alpha(const LaunchCtx& c, const RhsDesc& f, const float* g) {
  const Level& L = c.lev[0];
  hipLaunchKernelGGL(k_warm_dots, tiles(L.nf), tblock(), 0, c.stream, f, g, L.nf, c.red);
  hipLaunchKernelGGL(k_warm_alpha, dim3(1), dim3(kBlock), 0, c.stream, c.st, c.red);
}

template void launch_pcg_init<float>(const LaunchCtx&, const MGBuffers<float>&, const float*,
                                     float*);
template void launch_pcg_init<double>(const LaunchCtx&, const MGBuffers<double>&, const double*,
                                      double*);
template void launch_vcycle<float>(const LaunchCtx&, const MGBuffers<float>&, const float*,
                                   float*);
template void launch_vcycle<double>(const LaunchCtx&, const MGBuffers<double>&, const double*,
                                    double*);
template void launch_pcg_iteration<float>(const LaunchCtx&, const MGBuffers<float>&, int, float*,
                                          float*, float*, float*, float*, float*, bool);
template void launch_pcg_iteration<double>(const LaunchCtx&, const MGBuffers<double>&, int,
                                           double*, double*, double*, double*, double*, double*,
                                           bool);

}  // namespace fdd
