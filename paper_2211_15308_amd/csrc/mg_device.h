// Device-side building blocks of the interior multigrid-PCG solve (2D P1 grid, 5-point
// stencil 4, -1, -1, -1, -1), shared by the single-instance kernels (kernels_mg.hip) and the
// batched kernels (kernels_batch.hip).  See kernels_mg.hip for the method.
#pragma once
#include <type_traits>

#include "fdd_internal.h"

namespace fdd {

// --------------------------------------------------------------------------------------------
// helpers
// --------------------------------------------------------------------------------------------

__device__ __forceinline__ bool is_red(int i, int j) { return ((i + j) & 1) == 0; }

// Element o of a vector in global memory, addressed by a 32-bit byte offset (every vector here
// is below 2^31 bytes).  The pointer is cast to the global address space, so the access is a
// global (not flat) one with a wave-uniform base and one lane register, also where the pointer
// was read from memory (the batched kernels' instance descriptors) rather than passed as a
// kernel argument.
template <typename T>
using GlobalT = __attribute__((address_space(1))) T;
template <typename T>
__device__ __forceinline__ T ldg(const T* p, unsigned o) {
  return *(const GlobalT<T>*)((const GlobalT<char>*)p + o * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void stg(T* p, unsigned o, T v) {
  *(GlobalT<T>*)((GlobalT<char>*)p + o * (unsigned)sizeof(T)) = v;
}

__device__ __forceinline__ int flat_tid() { return threadIdx.y * blockDim.x + threadIdx.x; }
__device__ __forceinline__ int nthreads() { return blockDim.x * blockDim.y; }

// Sum over the block, broadcast to every thread (fixed order: deterministic).
__device__ __forceinline__ double block_sum_all(double v) {
  __shared__ double sh[kCoarseThreads / 64 + 1];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int t = flat_tid();
  const int lane = t & 63, wid = t >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  if (t == 0) {
    double s = 0.0;
    const int nw = (nthreads() + 63) >> 6;
    for (int w = 0; w < nw; ++w) s += sh[w];
    sh[kCoarseThreads / 64] = s;
  }
  __syncthreads();
  return sh[kCoarseThreads / 64];
}

// Fixed-order sum of nb partials, identical in every block of equal size.
__device__ __forceinline__ double sum_partials(const double* __restrict__ p, int nb) {
  // a thread's partials k = tid, tid + B, ... are added in that order, eight loads in flight at
  // a time (a loop adding each value as it arrives waits once per partial)
  constexpr int U = 8;
  const int nt = nthreads();
  double v = 0.0;
  for (int k0 = flat_tid(); k0 < nb; k0 += U * nt) {
    double a[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + u * nt;
      a[u] = k < nb ? ldg(p, (unsigned)k) : 0.0;
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (k0 + u * nt < nb) v += a[u];
  }
  return block_sum_all(v);
}

__device__ __forceinline__ bool block0() { return blockIdx.x == 0 && blockIdx.y == 0; }

// XCD-aware tile order.  Workgroups are dispatched round-robin over the 8 XCDs by linear id, so
// the linear id b runs on XCD b % 8.  Tile t = (b % 8) q + b / 8 (q = nb / 8; the remainder keeps
// t = b) gives each XCD a contiguous strip of tile rows, so halos shared by neighbouring tiles are
// fetched into one L2 instead of several.  Returns the tile id; (tx, ty) are its coordinates.
__device__ __forceinline__ int xcd_tile(int* tx, int* ty) {
  const int nbx = gridDim.x, nb = gridDim.x * gridDim.y;
  const int b = blockIdx.y * nbx + blockIdx.x;
  const int q = nb >> 3;
  const int t = (b < 8 * q) ? (b & 7) * q + (b >> 3) : b;
  *tx = t % nbx;
  *ty = t / nbx;
  return t;
}
__device__ __forceinline__ bool thread0() { return threadIdx.x == 0 && threadIdx.y == 0; }

__device__ __forceinline__ bool stopped(const DevState* st) {
  return (st->inner_done | st->solve_done) != 0;
}

// Convergence test of the running PCG from the partials of ||r||^2 (stored by the level-0
// down kernel).  Called by every block of the first kernel after it; returns true if the run
// is over (converged or broken down).
__device__ __forceinline__ bool pcg_converged(DevState* st, const Reductions& red, bool lead) {
  const double rr = sum_partials(red.rr, red.nb0);
  const bool bad = !isfinite(rr);
  const bool conv = bad || rr <= st->tau2 * st->rr0;
  if (lead && thread0()) {
    st->rr = rr;
    if (bad) st->breakdown |= 4;
    if (conv) {
      st->inner_done = 1;
      if (st->pcg_is_final) st->solve_done = 1;
    }
  }
  return conv;
}

// NS red-black Gauss-Seidel half-sweeps (alternating colours, the first red if red_first) over
// the window cells 1..W-2 that lie inside the domain.  Each thread owns a pair of adjacent
// columns over a segment of SEG rows and keeps their f and u in registers.  In every row of the
// segment exactly one cell of the pair has the sweep's colour; its update needs one LDS read (the
// horizontal neighbour outside the pair), the rest comes from registers, except above and below
// the segment.  Reads are unconditional (rows clamped into the window), so a half-sweep waits for
// LDS once; the new values go to LDS for the neighbouring threads and a barrier ends it.  Cells of
// one colour only read the other colour, so reads and writes of a half-sweep do not conflict.
// The update is u = (f + u_w + u_e + u_s + u_n) / 4 in that order of summation.
template <typename T, int W, int NS, int NT = kBlock, bool EDGE = true>
__device__ __forceinline__ void tile_sweeps(T (*su)[W + 1], const T (*sf)[W + 1], int ib, int jb,
                                            int nf, bool red_first) {
  constexpr int R = W - 2;  // updated rows and columns: 1 .. R (R even)
  constexpr int PAIRS = R / 2;
  constexpr int SEG = (R + NT / PAIRS - 1) / (NT / PAIRS);
  constexpr int NSEG = (R + SEG - 1) / SEG;
  static_assert(R % 2 == 0 && PAIRS * NSEG <= NT, "column pairs x segments fit the block");
  const int t = flat_tid();
  const int pr = t % PAIRS, sg = t / PAIRS;
  const bool act = sg < NSEG;
  const int la = 1 + 2 * pr;  // left column of the pair; the right one is la + 1
  const int lj0 = 1 + sg * SEG;
  const int ia = ib + la;
  auto rowc = [](int lj) { return lj < W - 1 ? lj : W - 1; };
  T fa[SEG], fb[SEG], ua[SEG], ub[SEG];
  bool ma[SEG], mb[SEG];
#pragma unroll
  for (int k = 0; k < SEG; ++k) {
    const int lj = lj0 + k, j = jb + lj;
    const bool rowok = act && lj <= R && (!EDGE || (j >= 1 && j <= nf));
    ma[k] = rowok && (!EDGE || (ia >= 1 && ia <= nf));
    mb[k] = rowok && (!EDGE || (ia + 1 >= 1 && ia + 1 <= nf));
    const int lr = rowc(lj);
    fa[k] = sf[lr][la];
    fb[k] = sf[lr][la + 1];
    ua[k] = su[lr][la];
    ub[k] = su[lr][la + 1];
  }
  const int par0 = (ia + jb + lj0) & 1;  // colour parity of cell (la, lj0); 0: red
  bool red = red_first;
#pragma unroll
  for (int h = 0; h < NS; ++h) {
    const int want = red ? 0 : 1;
    T nv[SEG];
#pragma unroll
    for (int k = 0; k < SEG; ++k) {
      const bool left = ((par0 + k) & 1) == want;  // the updated cell of row k is column la
      const int lj = lj0 + k;
      const int col = left ? la : la + 1;
      const T hn = su[rowc(lj)][left ? la - 1 : la + 2];
      const T hin = left ? ub[k] : ua[k];
      const T fv = left ? fa[k] : fb[k];
      const T up = k > 0 ? (left ? ua[k - 1] : ub[k - 1]) : su[lj - 1][col];
      const T dn = k + 1 < SEG ? (left ? ua[k + 1] : ub[k + 1]) : su[rowc(lj + 1)][col];
      const T uw = left ? hn : hin;
      const T ue = left ? hin : hn;
      nv[k] = T(0.25) * (fv + uw + ue + up + dn);
    }
#pragma unroll
    for (int k = 0; k < SEG; ++k) {
      const bool left = ((par0 + k) & 1) == want;
      if (left ? ma[k] : mb[k]) {
        su[lj0 + k][left ? la : la + 1] = nv[k];
        if (left) ua[k] = nv[k];
        else ub[k] = nv[k];
      }
    }
    __syncthreads();
    red = !red;
  }
}

// Sums of two values over the block, broadcast to every thread (fixed order: deterministic).
__device__ __forceinline__ void block_sum2(double& a, double& b) {
  __shared__ double sh[2][kBlock / 64 + 1];
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_down(a, o, 64);
    b += __shfl_down(b, o, 64);
  }
  const int t = flat_tid();
  const int lane = t & 63, wid = t >> 6;
  __syncthreads();
  if (lane == 0) {
    sh[0][wid] = a;
    sh[1][wid] = b;
  }
  __syncthreads();
  if (t == 0) {
    double sa = 0.0, sb = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) {
      sa += sh[0][w];
      sb += sh[1][w];
    }
    sh[0][kBlock / 64] = sa;
    sh[1][kBlock / 64] = sb;
  }
  __syncthreads();
  a = sh[0][kBlock / 64];
  b = sh[1][kBlock / 64];
}

// r . z and z . A z of inner PCG iteration k from the level-0 partials, summed by one block of
// kBlock threads in the order every block of the level-0 down kernel would use, into st->dots.
// On large grids (and batches) this pass replaces the per-block sums of that kernel, whose L2
// reads grow with the square of the tile count.
__device__ __forceinline__ void d_sum_dots(const Reductions& red, int k, DevState* st) {
  const double* rzp = (k & 1) ? red.rz[1] : red.rz[0];
  const double* zwp = (k & 1) ? red.zw[1] : red.zw[0];
  double gam = 0.0, del = 0.0;
  for (int q = flat_tid(); q < red.nbd; q += kBlock) {
    gam += ldg(rzp, (unsigned)q);
    del += ldg(zwp, (unsigned)q);
  }
  block_sum2(gam, del);
  if (thread0()) {
    st->dots[0] = gam;
    st->dots[1] = del;
  }
}

// Inside the grid (1..nf in both directions); always true for the bodies of interior tiles.
template <bool EDGE>
__device__ __forceinline__ bool in_grid(int i, int j, int nf) {
  return !EDGE || (i >= 1 && i <= nf && j >= 1 && j <= nf);
}

// True if every cell a tiled level kernel with halo H touches for this tile lies inside the grid:
// the window, one ring beyond it (the PCG update's p) and the coarse patch of the prolongation.
// Such tiles (all but the outermost ring of tiles) run the kernel body without its per-cell
// domain tests (EDGE = false); the arithmetic is the same.
template <int H, int TT>
__device__ __forceinline__ bool tile_inner(int tile_x, int tile_y, int nf) {
  constexpr int W = TT + 2 * H;
  constexpr int CW = W / 2 + 2;
  const int ib = tile_x * TT + 1 - H, jb = tile_y * TT + 1 - H;
  const int nc = (nf - 1) >> 1;
  return ib >= 2 && jb >= 2 && ib + W <= nf && jb + W <= nf && (ib >> 1) + CW - 1 <= nc &&
         (jb >> 1) + CW - 1 <= nc;
}

// --------------------------------------------------------------------------------------------
// fused level kernels
// --------------------------------------------------------------------------------------------
// The tiled kernels run 256 threads on a TT x TT tile plus a halo (TT = kTile = 32 on the
// finest level, 16 on an intermediate level that runs alone).  Window cells are enumerated
// row-major over the flat thread index (cell t + 256 q), own cells likewise over the tile, so
// loads are row-contiguous and no lane idles on a short row.
// All global loads of a window are issued into registers before the first use, so a block waits
// for one memory latency.

// Register slots of a W x W window in the 32 x 8 layout (cell (ty + 8 a, tx + 32 b)).
template <int W>
struct Slots {
  static constexpr int RY = (W + 7) / 8;
  static constexpr int RX = (W + 31) / 32;
};

template <int W>
struct Flat {
  static constexpr int N = (W * W + kBlock - 1) / kBlock;  // window slots per thread
};
constexpr int kOwnSlots = kTile * kTile / kBlock;

// Going down one level: u = S^nu(0; f) (red first), r = f - A u, f_c = P^T r.
// CG = true (level 0, inner PCG iteration k, single-reduction form):
//   gamma_k = r_k . z_k and delta_k = z_k . A z_k come from the partials of the previous V-cycle
//   (summed here in one pass); beta_k = gamma_k / gamma_{k-1}, alpha_k = gamma_k / (delta_k -
//   beta_k gamma_k / alpha_{k-1}) (beta_0 = 0, alpha_0 = gamma_0 / delta_0), with gamma_{k-1}
//   and alpha_{k-1} recorded by the previous iteration.  p_k = z_k + beta_k p_{k-1} is formed
//   one cell beyond the window, so that s_k = A p_k is a stencil in LDS (no stored recurrence
//   for A p); on the window f = r_{k+1} = r_k - alpha_k s_k; on own points x += alpha_k p_k and
//   r_{k+1}, p_k are stored; ||r_{k+1}||^2 goes to red.rr.
template <typename T, int NU, bool CG, int TT, bool EDGE, bool RESIDENT>
__device__ __forceinline__ void d_mg_down_body(T* sf_, T* su_, T* s3_,
    const T* __restrict__ fin, T* __restrict__ uout, T* __restrict__ fc, int nf, int pitch,
    int pc, const T* __restrict__ z, const T* __restrict__ pold, T* __restrict__ pnew,
    T* __restrict__ x, T* __restrict__ rout, DevState* st, const Reductions& red, int k,
    int tile_x, int tile_y, int tile, bool lead, bool presum = false) {
  constexpr int H = 2 * NU + 1;
  constexpr int W = TT + 2 * H;
  constexpr int PW = CG ? W + 2 : 1;  // window of p: one cell beyond the f window
  constexpr int NW = Flat<W>::N;
  constexpr int NPW = CG ? Flat<PW>::N : 1;
  auto sf = reinterpret_cast<T(*)[W + 1]>(sf_);
  auto su = reinterpret_cast<T(*)[W + 1]>(su_);
  auto sp = reinterpret_cast<T(*)[PW + 1]>(s3_);
  const int i0 = tile_x * TT, j0 = tile_y * TT;
  const int ib = i0 + 1 - H, jb = j0 + 1 - H;  // global index of window cell (0, 0)
  const int t = flat_tid();
  // RESIDENT (every tile of the grid runs at once): with the thread range known, the compiler
  // computes every window offset up front, in about twice the registers, which shortens the
  // critical path of a block but would cost occupancy when tiles queue for compute units
  if constexpr (RESIDENT) __builtin_assume(t >= 0 && t < kBlock);
  // element offsets as a block-uniform base plus a small per-cell part (row index times pitch:
  // a 24-bit product, as every vector here has fewer than 2^29 elements)
  const unsigned rb = (unsigned)((jb - 1) * pitch + (ib - 1));  // f window cell (0, 0)
  const unsigned rbp = rb - (unsigned)pitch - 1u;                 // p window cell (0, 0)
  const unsigned ro = (unsigned)(j0 * pitch + i0);               // own cell (0, 0)
  T fr[NW];
  T zr[NPW], pr[NPW], xr[NPW];
  // the partials of r.z and z.A z (CG) are loaded first: their sum is needed before any window
  // value, and loads complete in issue order (presum: d_sum_dots has summed them, in the same
  // order, into st->dots)
  constexpr int NP = CG ? 4 : 1;
  double rzr[NP], zwr[NP];
  // (parity selects, not indexing: a runtime index into the struct would put it in scratch)
  const double* rzp = (k & 1) ? red.rz[1] : red.rz[0];
  const double* zwp = (k & 1) ? red.zw[1] : red.zw[0];
#pragma unroll
  for (int a = 0; a < NP; ++a) {
    const int q = t + kBlock * a;
    const bool ok = CG && !presum && q < red.nbd;
    rzr[a] = ok ? ldg(rzp, (unsigned)q) : 0.0;
    zwr[a] = ok ? ldg(zwp, (unsigned)q) : 0.0;
  }
#pragma unroll
  for (int q = 0; q < NW; ++q) {
    const int c = t + kBlock * q;
    const int lj = c / W, li = c % W;
    const int i = ib + li, j = jb + lj;
    const bool in = c < W * W && in_grid<EDGE>(i, j, nf);
    fr[q] = in ? ldg(fin, rb + (__umul24(lj, pitch) + li)) : T(0);
  }
  if constexpr (CG) {
#pragma unroll
    for (int q = 0; q < NPW; ++q) {
      const int c = t + kBlock * q;
      const int lj = c / PW, li = c % PW;
      const int i = ib - 1 + li, j = jb - 1 + lj;
      const bool in = c < PW * PW && in_grid<EDGE>(i, j, nf);
      const unsigned o = rbp + (__umul24(lj, pitch) + li);
      // own cells of the tile: p window cells H + 1 .. H + TT
      const bool own = in && li > H && li <= H + TT && lj > H && lj <= H + TT;
      zr[q] = in ? ldg(z, o) : T(0);
      pr[q] = (in && k > 0) ? ldg(pold, o) : T(0);
      xr[q] = (own && k > 0) ? ldg((const T*)x, o) : T(0);
    }
  }
  T alpha = T(0), beta = T(0);
  if constexpr (CG) {
    double gam = 0.0, del = 0.0;
    if (presum) {
      gam = st->dots[0];
      del = st->dots[1];
    } else {
#pragma unroll
      for (int a = 0; a < NP; ++a) {
        gam += rzr[a];
        del += zwr[a];
      }
      for (int q = t + kBlock * NP; q < red.nbd; q += kBlock) {
        gam += ldg(rzp, (unsigned)q);
        del += ldg(zwp, (unsigned)q);
      }
      block_sum2(gam, del);
    }
    double b = 0.0, den = del;
    if (k > 0) {
      b = gam / st->cg_gam[(k - 1) & 1];
      den = del - b * gam / st->cg_alpha[(k - 1) & 1];
    }
    if (!(gam > 0.0) || !(den > 0.0) || !isfinite(den) || !isfinite(gam)) {
      // gamma = 0: the residual is exactly zero and the run is over; otherwise a breakdown
      if (lead && thread0()) {
        if (gam != 0.0) st->breakdown |= (isfinite(den) && isfinite(gam)) ? 1 : 4;
        st->inner_done = 1;
      }
      return;
    }
    const double al = gam / den;
    if (lead && thread0()) {
      st->cg_alpha[k & 1] = al;
      st->cg_gam[k & 1] = gam;
    }
    alpha = (T)al;
    beta = (T)b;
    // p_k on its window (zero outside the domain, where z and p_{k-1} are zero); on own cells
    // p_k and x + alpha_k p_k are stored
#pragma unroll
    for (int q = 0; q < NPW; ++q) {
      const int c = t + kBlock * q;
      if (c >= PW * PW) continue;
      const int lj = c / PW, li = c % PW;
      const T pv = zr[q] + beta * pr[q];
      sp[lj][li] = pv;
      const int i = ib - 1 + li, j = jb - 1 + lj;
      if (li > H && li <= H + TT && lj > H && lj <= H + TT && (!EDGE || (i <= nf && j <= nf))) {
        const unsigned o = rbp + (__umul24(lj, pitch) + li);
        stg(pnew, o, pv);
        stg(x, o, xr[q] + alpha * pv);
      }
    }
    __syncthreads();
  }
  double rr = 0.0;
#pragma unroll
  for (int q = 0; q < NW; ++q) {
    const int c = t + kBlock * q;
    if (c >= W * W) continue;
    const int lj = c / W, li = c % W;
    const int i = ib + li, j = jb + lj;
    T f = fr[q];
    if constexpr (CG) {
      if (in_grid<EDGE>(i, j, nf)) {
        const int pj = lj + 1, pi = li + 1;
        const T sv = T(4) * sp[pj][pi] - sp[pj][pi - 1] - sp[pj][pi + 1] - sp[pj - 1][pi] -
                     sp[pj + 1][pi];
        f = f - alpha * sv;
        if (li >= H && li < H + TT && lj >= H && lj < H + TT) {
          stg(rout, rb + (__umul24(lj, pitch) + li), f);
          rr += (double)f * (double)f;
        }
      }
    }
    sf[lj][li] = f;
    // first red half-sweep from a zero iterate: u = f / 4 on red points, 0 on black points
    su[lj][li] = is_red(i, j) ? T(0.25) * f : T(0);
  }
  __syncthreads();
  tile_sweeps<T, W, 2 * NU - 1, kBlock, EDGE>(su, sf, ib, jb, nf, false);  // black, red, ...
  // residual, in place of f, on the cells the restriction reads (window rows and columns
  // H .. H + TT); each reads its own f and the neighbours' u
  constexpr int RW = TT + 1;
  for (int c = t; c < RW * RW; c += kBlock) {
    const int lj = H + c / RW, li = H + c % RW;
    sf[lj][li] = sf[lj][li] - (T(4) * su[lj][li] - su[lj][li - 1] - su[lj][li + 1] -
                               su[lj - 1][li] - su[lj + 1][li]);
  }
  __syncthreads();
  // restriction to the coarse points whose fine index 2I lies in this tile (one per thread)
  {
    const int nc = (nf - 1) >> 1;
    constexpr int TC = TT / 2;
    static_assert(TC * TC <= kBlock, "at most one coarse point per thread");
    const int J = (j0 >> 1) + 1 + t / TC, I = (i0 >> 1) + 1 + t % TC;
    if (t < TC * TC && (!EDGE || (J <= nc && I <= nc))) {
      const int li = 2 * I - ib, lj = 2 * J - jb;
      const T v = sf[lj][li] + T(0.5) * (sf[lj][li - 1] + sf[lj][li + 1] + sf[lj - 1][li] +
                                         sf[lj + 1][li] + sf[lj - 1][li - 1] +
                                         sf[lj + 1][li + 1]);
      stg(fc, (unsigned)((j0 >> 1) * pc + (i0 >> 1)) + (__umul24(t / TC, pc) + t % TC), v);
    }
  }
  // store the pre-smoothed iterate on own points
#pragma unroll
  for (int q = 0; q < (TT * TT / kBlock); ++q) {
    const int c = t + kBlock * q;
    const int bi = c % TT, bj = c / TT;
    const int i = i0 + 1 + bi, j = j0 + 1 + bj;
    if (EDGE && (j > nf || i > nf)) continue;
    stg(uout, ro + (__umul24(bj, pitch) + bi), su[bj + H][bi + H]);
  }
  if (CG) {
    const double tot = block_sum_all(rr);
    if (thread0()) red.rr[tile] = tot;
  }
}

// The body above for one tile; interior tiles take it without the per-cell domain tests (both
// variants share the LDS windows).
template <typename T, int NU, bool CG, int TT = kTile, bool RESIDENT = false>
__device__ __forceinline__ void d_mg_down(
    const T* __restrict__ fin, T* __restrict__ uout, T* __restrict__ fc, int nf, int pitch,
    int pc, const T* __restrict__ z, const T* __restrict__ pold, T* __restrict__ pnew,
    T* __restrict__ x, T* __restrict__ rout, DevState* st, const Reductions& red, int k,
    int tile_x, int tile_y, int tile, bool lead, bool presum = false) {
  constexpr int H = 2 * NU + 1;
  constexpr int W = TT + 2 * H;
  constexpr int PW = CG ? W + 2 : 1;
  __shared__ T sf[W][W + 1];
  __shared__ T su[W][W + 1];
  __shared__ T sp[PW][PW + 1];
  if (tile_inner<H, TT>(tile_x, tile_y, nf))
    d_mg_down_body<T, NU, CG, TT, false, RESIDENT>(&sf[0][0], &su[0][0], &sp[0][0], fin, uout,
                                                   fc, nf, pitch, pc, z, pold, pnew, x, rout, st,
                                                   red, k, tile_x, tile_y, tile, lead, presum);
  else
    d_mg_down_body<T, NU, CG, TT, true, RESIDENT>(&sf[0][0], &su[0][0], &sp[0][0], fin, uout, fc,
                                                  nf, pitch, pc, z, pold, pnew, x, rout, st, red,
                                                  k, tile_x, tile_y, tile, lead, presum);
}

// Going up one level: u = u_pre + P e_c, then nu (black, red) pairs; result to eout.
// CG = true (level 0): the result z is kept valid one cell beyond the tile, so that A z is
// formed on own points too; z is stored and the block's parts of r . z and z . A z go to
// red.rz[kn & 1] and red.zw[kn & 1] (f is r).
template <typename T, int NU, bool CG, int TT, bool EDGE>
__device__ __forceinline__ void d_mg_up_body(T* sf_, T* su_, T* s3_,
    const T* __restrict__ fin, const T* __restrict__ upre, const T* __restrict__ ec,
    T* __restrict__ eout, int nf, int pitch, int pc, DevState* st, const Reductions& red, int kn,
    int count_iteration, int tile_x, int tile_y, int tile, bool lead) {
  constexpr int H = 2 * NU + (CG ? 1 : 0);
  constexpr int W = TT + 2 * H;
  constexpr int NW = Flat<W>::N;
  constexpr int CW = W / 2 + 2;  // coarse patch edge
  constexpr int NC = Flat<CW>::N;
  auto sf = reinterpret_cast<T(*)[W + 1]>(sf_);
  auto su = reinterpret_cast<T(*)[W + 1]>(su_);
  auto sc = reinterpret_cast<T(*)[CW + 1]>(s3_);
  const int i0 = tile_x * TT, j0 = tile_y * TT;
  const int ib = i0 + 1 - H, jb = j0 + 1 - H;
  const int Ib = ib >> 1, Jb = jb >> 1;  // floor (arithmetic shift)
  const int nc = (nf - 1) >> 1;
  const int t = flat_tid();
  __builtin_assume(t >= 0 && t < kBlock);
  // element offsets as a block-uniform base plus a small per-cell part (row index times pitch:
  // a 24-bit product, as every vector here has fewer than 2^29 elements)
  const unsigned rb = (unsigned)((jb - 1) * pitch + (ib - 1));  // window cell (0, 0)
  const unsigned rc = (unsigned)((Jb - 1) * pc + (Ib - 1));     // coarse patch cell (0, 0)
  const unsigned ro = (unsigned)(j0 * pitch + i0);              // own cell (0, 0)
  T fr[NW], ur[NW], cr[NC];
#pragma unroll
  for (int q = 0; q < NW; ++q) {
    const int c = t + kBlock * q;
    const int lj = c / W, li = c % W;
    const int i = ib + li, j = jb + lj;
    const bool in = c < W * W && in_grid<EDGE>(i, j, nf);
    const unsigned o = rb + (__umul24(lj, pitch) + li);
    fr[q] = in ? ldg(fin, o) : T(0);
    ur[q] = in ? ldg(upre, o) : T(0);
  }
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int c = t + kBlock * q;
    const int lj = c / CW, li = c % CW;
    const int I = Ib + li, J = Jb + lj;
    const bool in = c < CW * CW && (!EDGE || (I >= 1 && I <= nc && J >= 1 && J <= nc));
    cr[q] = in ? ldg(ec, rc + (__umul24(lj, pc) + li)) : T(0);
  }
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int c = t + kBlock * q;
    if (c < CW * CW) sc[c / CW][c % CW] = cr[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NW; ++q) {
    const int c = t + kBlock * q;
    if (c >= W * W) continue;
    const int lj = c / W, li = c % W;
    const int i = ib + li, j = jb + lj;
    T u = T(0);
    if (in_grid<EDGE>(i, j, nf)) {
      // P1 interpolation of the coarse correction (nested diagonal-split meshes): the mean of
      // the coarse values at (i >> 1, j >> 1) and at that point shifted by the parities of
      // (i, j); at coincident points both are the same value, and 0.5 (a + a) = a exactly.
      // Branch-free, so the reads of all window slots are issued together.
      const int ci = (li + (ib & 1)) >> 1, cj = (lj + (jb & 1)) >> 1;  // (i >> 1) - Ib, ...
      const T e = T(0.5) * (sc[cj][ci] + sc[cj + (j & 1)][ci + (i & 1)]);
      u = ur[q] + e;
    }
    sf[lj][li] = fr[q];
    su[lj][li] = u;
  }
  __syncthreads();
  tile_sweeps<T, W, 2 * NU, kBlock, EDGE>(su, sf, ib, jb, nf, false);  // black, red, ...
  double rz = 0.0, zw = 0.0;
#pragma unroll
  for (int q = 0; q < (TT * TT / kBlock); ++q) {
    const int c = t + kBlock * q;
    const int bi = c % TT, bj = c / TT;
    const int i = i0 + 1 + bi, j = j0 + 1 + bj;
    if (EDGE && (j > nf || i > nf)) continue;
    const int lj = bj + H, li = bi + H;
    const T zv = su[lj][li];
    const unsigned o = ro + (__umul24(bj, pitch) + bi);
    stg(eout, o, zv);
    if (CG) {
      const T wv = T(4) * zv - su[lj][li - 1] - su[lj][li + 1] - su[lj - 1][li] - su[lj + 1][li];
      rz += (double)sf[lj][li] * (double)zv;
      zw += (double)zv * (double)wv;
    }
  }
  if (CG) {
    block_sum2(rz, zw);
    if (thread0()) {
      stg((kn & 1) ? red.rz[1] : red.rz[0], (unsigned)tile, rz);
      stg((kn & 1) ? red.zw[1] : red.zw[0], (unsigned)tile, zw);
      if (count_iteration && lead) {
        st->inner_its += 1;
        st->pcg_k += 1;
        st->run_its_max = max(st->run_its_max, st->pcg_k);
      }
    }
  }
}

// The body above for one tile; interior tiles take it without the per-cell domain tests.
template <typename T, int NU, bool CG, int TT = kTile>
__device__ __forceinline__ void d_mg_up(
    const T* __restrict__ fin, const T* __restrict__ upre, const T* __restrict__ ec,
    T* __restrict__ eout, int nf, int pitch, int pc, DevState* st, const Reductions& red, int kn,
    int count_iteration, int tile_x, int tile_y, int tile, bool lead) {
  constexpr int H = 2 * NU + (CG ? 1 : 0);
  constexpr int W = TT + 2 * H;
  constexpr int CW = W / 2 + 2;
  __shared__ T sf[W][W + 1];
  __shared__ T su[W][W + 1];
  __shared__ T sc[CW][CW + 1];
  if (tile_inner<H, TT>(tile_x, tile_y, nf))
    d_mg_up_body<T, NU, CG, TT, false>(&sf[0][0], &su[0][0], &sc[0][0], fin, upre, ec, eout, nf,
                                       pitch, pc, st, red, kn, count_iteration, tile_x, tile_y,
                                       tile, lead);
  else
    d_mg_up_body<T, NU, CG, TT, true>(&sf[0][0], &su[0][0], &sc[0][0], fin, upre, ec, eout, nf,
                                      pitch, pc, st, red, kn, count_iteration, tile_x, tile_y,
                                      tile, lead);
}


// --------------------------------------------------------------------------------------------
// two intermediate levels in one kernel
// --------------------------------------------------------------------------------------------
// A block of kPairThreads threads owns a kPairTile x kPairTile tile of level l+1 and the 2 kPairTile x 2 kPairTile
// level-l cells above it.  Going down it smooths level l on a window wide enough that the
// restricted residual gives f_{l+1} on the whole level-(l+1) window, then does level l+1 as the
// tiled kernel does; going up it corrects and smooths level l+1 on a window whose valid part is
// the coarse patch that level l interpolates from, then does level l.  The arithmetic of every
// cell is that of the single-level kernels (the redundantly computed halos are discarded), so the
// results are bit-identical to them; one launch and one inter-kernel gap fewer per level pair.
constexpr int kPairThreads = 1024;
constexpr int kPairTile = 16;  // level-(l+1) tile edge of a pair block

template <int NU>
struct PairDown {
  static constexpr int H1 = 2 * NU + 1;               // level-(l+1) halo, as the tiled kernel
  static constexpr int W1 = kPairTile + 2 * H1;           // level-(l+1) window
  // level l: r_l on 2 W1 + 1 cells, u_l valid one further, 2 NU - 1 half-sweeps after the red
  // start each lose one cell at the edge; one more column and row make the sweep extent even
  static constexpr int S0 = 2 * NU - 1;
  static constexpr int W0 = 2 * W1 + 3 + 2 * S0 + 1;
  static constexpr int N0 = (W0 * W0 + kPairThreads - 1) / kPairThreads;
};

// Levels l (nf0 points per side, pitch p0) and l+1 going down: u_l = S^nu(0; f_l) stored on the
// block's level-l cells, f_{l+1} = P^T (f_l - A u_l) and u_{l+1} = S^nu(0; f_{l+1}) stored on its
// level-(l+1) tile, f_{l+2} = P^T (f_{l+1} - A u_{l+1}) on the coarse points of the tile.
template <typename T, int NU>
__device__ __forceinline__ void d_pair_down(const T* __restrict__ fin0, T* __restrict__ uout0,
                                            T* __restrict__ fout1, T* __restrict__ uout1,
                                            T* __restrict__ fout2, int nf0, int p0, int p1,
                                            int p2, int tile_x, int tile_y) {
  using G = PairDown<NU>;
  constexpr int H1 = G::H1, W1 = G::W1, W0 = G::W0, S0 = G::S0;
  __shared__ T sf0[W0][W0 + 1];
  __shared__ T su0[W0][W0 + 1];
  __shared__ T sf1[W1][W1 + 1];
  __shared__ T su1[W1][W1 + 1];
  const int t = flat_tid();
  // one block per compute unit, every block in flight: the thread range is known to the compiler
  __builtin_assume(t >= 0 && t < kPairThreads);
  const int nf1 = (nf0 - 1) >> 1;
  const int I0 = tile_x * kPairTile, J0 = tile_y * kPairTile;
  const int Ib = I0 + 1 - H1, Jb = J0 + 1 - H1;          // level-(l+1) window origin
  const int ib0 = 2 * Ib - 2 - S0, jb0 = 2 * Jb - 2 - S0;  // level-l window origin
  T fr[G::N0];
#pragma unroll
  for (int q = 0; q < G::N0; ++q) {
    const int c = t + kPairThreads * q;
    const int lj = c / W0, li = c % W0;
    const int i = ib0 + li, j = jb0 + lj;
    const bool in = c < W0 * W0 && i >= 1 && i <= nf0 && j >= 1 && j <= nf0;
    fr[q] = in ? ldg(fin0, (__umul24(j - 1, p0) + (i - 1))) : T(0);
  }
#pragma unroll
  for (int q = 0; q < G::N0; ++q) {
    const int c = t + kPairThreads * q;
    if (c >= W0 * W0) continue;
    const int lj = c / W0, li = c % W0;
    sf0[lj][li] = fr[q];
    su0[lj][li] = is_red(ib0 + li, jb0 + lj) ? T(0.25) * fr[q] : T(0);
  }
  __syncthreads();
  tile_sweeps<T, W0, S0, kPairThreads>(su0, sf0, ib0, jb0, nf0, false);  // black, red, black, ...
  // level-l residual (in place of f) on the cells the restriction reads: window cells S0 + 1 ..
  // S0 + 1 + 2 W1
  constexpr int RW0 = 2 * W1 + 1;
  for (int c = t; c < RW0 * RW0; c += kPairThreads) {
    const int lj = S0 + 1 + c / RW0, li = S0 + 1 + c % RW0;
    sf0[lj][li] = sf0[lj][li] - (T(4) * su0[lj][li] - su0[lj][li - 1] - su0[lj][li + 1] -
                                 su0[lj - 1][li] - su0[lj + 1][li]);
  }
  // the block's level-l cells: 2 I0 + 1 .. 2 I0 + 2 kPairTile
  for (int c = t; c < 4 * kPairTile * kPairTile; c += kPairThreads) {
    const int bi = c % (2 * kPairTile), bj = c / (2 * kPairTile);
    const int i = 2 * I0 + 1 + bi, j = 2 * J0 + 1 + bj;
    if (i <= nf0 && j <= nf0)
      stg(uout0, (__umul24(j - 1, p0) + (i - 1)), su0[j - jb0][i - ib0]);
  }
  __syncthreads();
  // f_{l+1} on the level-(l+1) window (zero outside the level), stored on the tile; red start
  for (int c = t; c < W1 * W1; c += kPairThreads) {
    const int LJ = c / W1, LI = c % W1;
    const int I = Ib + LI, J = Jb + LJ;
    T v = T(0);
    if (I >= 1 && I <= nf1 && J >= 1 && J <= nf1) {
      const int li = 2 * I - ib0, lj = 2 * J - jb0;
      v = sf0[lj][li] + T(0.5) * (sf0[lj][li - 1] + sf0[lj][li + 1] + sf0[lj - 1][li] +
                                  sf0[lj + 1][li] + sf0[lj - 1][li - 1] + sf0[lj + 1][li + 1]);
      if (LI >= H1 && LI < H1 + kPairTile && LJ >= H1 && LJ < H1 + kPairTile)
        stg(fout1, (__umul24(J - 1, p1) + (I - 1)), v);
    }
    sf1[LJ][LI] = v;
    su1[LJ][LI] = is_red(I, J) ? T(0.25) * v : T(0);
  }
  __syncthreads();
  tile_sweeps<T, W1, 2 * NU - 1, kPairThreads>(su1, sf1, Ib, Jb, nf1, false);
  constexpr int RW1 = kPairTile + 1;
  for (int c = t; c < RW1 * RW1; c += kPairThreads) {
    const int lj = H1 + c / RW1, li = H1 + c % RW1;
    sf1[lj][li] = sf1[lj][li] - (T(4) * su1[lj][li] - su1[lj][li - 1] - su1[lj][li + 1] -
                                 su1[lj - 1][li] - su1[lj + 1][li]);
  }
  __syncthreads();
  {
    const int nc = (nf1 - 1) >> 1;
    constexpr int TC = kPairTile / 2;
    if (t < TC * TC) {
      const int J = (J0 >> 1) + 1 + t / TC, I = (I0 >> 1) + 1 + t % TC;
      if (J <= nc && I <= nc) {
        const int li = 2 * I - Ib, lj = 2 * J - Jb;
        const T v = sf1[lj][li] + T(0.5) * (sf1[lj][li - 1] + sf1[lj][li + 1] + sf1[lj - 1][li] +
                                            sf1[lj + 1][li] + sf1[lj - 1][li - 1] +
                                            sf1[lj + 1][li + 1]);
        stg(fout2, (__umul24(J - 1, p2) + (I - 1)), v);
      }
    }
  }
  for (int c = t; c < kPairTile * kPairTile; c += kPairThreads) {
    const int bi = c % kPairTile, bj = c / kPairTile;
    const int I = I0 + 1 + bi, J = J0 + 1 + bj;
    if (I <= nf1 && J <= nf1) stg(uout1, (__umul24(J - 1, p1) + (I - 1)), su1[bj + H1][bi + H1]);
  }
}

template <int NU>
struct PairUp {
  static constexpr int H = 2 * NU;                  // halo of an up window (no w = A z here)
  static constexpr int W0 = 2 * kPairTile + 2 * H;      // level-l window
  static constexpr int CW = W0 / 2 + 2;             // its coarse patch (valid part of level l+1)
  static constexpr int W1 = CW + 2 * H;             // level-(l+1) window
  static constexpr int CW2 = W1 / 2 + 2;            // coarse patch of level l+2
  static constexpr int N0 = (W0 * W0 + kPairThreads - 1) / kPairThreads;
  static constexpr int N1 = (W1 * W1 + kPairThreads - 1) / kPairThreads;
  static constexpr int N2 = (CW2 * CW2 + kPairThreads - 1) / kPairThreads;
};

// Levels l+1 and l going up: u_{l+1} = u_{l+1,pre} + P e_{l+2}, 2 nu half-sweeps, on a window
// whose valid part covers the coarse patch of level l; then u_l = u_{l,pre} + P e_{l+1} and 2 nu
// half-sweeps; e_l stored on the block's level-l cells.
template <typename T, int NU>
__device__ __forceinline__ void d_pair_up(const T* __restrict__ f0, const T* __restrict__ u0pre,
                                          const T* __restrict__ f1, const T* __restrict__ u1pre,
                                          const T* __restrict__ e2, T* __restrict__ eout0, int nf0,
                                          int p0, int p1, int p2, int tile_x, int tile_y) {
  using G = PairUp<NU>;
  constexpr int H = G::H, W0 = G::W0, W1 = G::W1, CW2 = G::CW2;
  __shared__ T sf0[W0][W0 + 1];
  __shared__ T su0[W0][W0 + 1];
  __shared__ T sf1[W1][W1 + 1];
  __shared__ T su1[W1][W1 + 1];
  __shared__ T sc2[CW2][CW2 + 1];
  const int t = flat_tid();
  // one block per compute unit, every block in flight: the thread range is known to the compiler
  __builtin_assume(t >= 0 && t < kPairThreads);
  const int nf1 = (nf0 - 1) >> 1, nf2 = (nf1 - 1) >> 1;
  const int I0 = tile_x * kPairTile, J0 = tile_y * kPairTile;
  const int ib0 = 2 * I0 + 1 - H, jb0 = 2 * J0 + 1 - H;  // level-l window origin
  const int Ic = ib0 >> 1, Jc = jb0 >> 1;                // its coarse patch origin (floor)
  const int ib1 = Ic - H, jb1 = Jc - H;                  // level-(l+1) window origin
  const int Ic2 = ib1 >> 1, Jc2 = jb1 >> 1;              // coarse patch of level l+2
  T f1r[G::N1], u1r[G::N1], f0r[G::N0], u0r[G::N0], c2r[G::N2];
#pragma unroll
  for (int q = 0; q < G::N2; ++q) {
    const int c = t + kPairThreads * q;
    const int I = Ic2 + c % CW2, J = Jc2 + c / CW2;
    const bool in = c < CW2 * CW2 && I >= 1 && I <= nf2 && J >= 1 && J <= nf2;
    c2r[q] = in ? ldg(e2, (__umul24(J - 1, p2) + (I - 1))) : T(0);
  }
#pragma unroll
  for (int q = 0; q < G::N1; ++q) {
    const int c = t + kPairThreads * q;
    const int i = ib1 + c % W1, j = jb1 + c / W1;
    const bool in = c < W1 * W1 && i >= 1 && i <= nf1 && j >= 1 && j <= nf1;
    const unsigned o = (__umul24(j - 1, p1) + (i - 1));
    f1r[q] = in ? ldg(f1, o) : T(0);
    u1r[q] = in ? ldg(u1pre, o) : T(0);
  }
#pragma unroll
  for (int q = 0; q < G::N0; ++q) {
    const int c = t + kPairThreads * q;
    const int i = ib0 + c % W0, j = jb0 + c / W0;
    const bool in = c < W0 * W0 && i >= 1 && i <= nf0 && j >= 1 && j <= nf0;
    const unsigned o = (__umul24(j - 1, p0) + (i - 1));
    f0r[q] = in ? ldg(f0, o) : T(0);
    u0r[q] = in ? ldg(u0pre, o) : T(0);
  }
#pragma unroll
  for (int q = 0; q < G::N2; ++q) {
    const int c = t + kPairThreads * q;
    if (c < CW2 * CW2) sc2[c / CW2][c % CW2] = c2r[q];
  }
  __syncthreads();
  // level l+1: prolongation of e_{l+2} (the mean of the values at (i >> 1, j >> 1) and at that
  // point shifted by the parities of (i, j)) plus the pre-smoothed iterate
#pragma unroll
  for (int q = 0; q < G::N1; ++q) {
    const int c = t + kPairThreads * q;
    if (c >= W1 * W1) continue;
    const int lj = c / W1, li = c % W1;
    const int i = ib1 + li, j = jb1 + lj;
    T u = T(0);
    if (i >= 1 && i <= nf1 && j >= 1 && j <= nf1) {
      const int ci = (i >> 1) - Ic2, cj = (j >> 1) - Jc2;
      const T e = T(0.5) * (sc2[cj][ci] + sc2[cj + (j & 1)][ci + (i & 1)]);
      u = u1r[q] + e;
    }
    sf1[lj][li] = f1r[q];
    su1[lj][li] = u;
  }
  __syncthreads();
  tile_sweeps<T, W1, 2 * NU, kPairThreads>(su1, sf1, ib1, jb1, nf1, false);  // black, red, ...
  // level l: the corrected level-(l+1) values on the patch are su1[H + c][H + d]
#pragma unroll
  for (int q = 0; q < G::N0; ++q) {
    const int c = t + kPairThreads * q;
    if (c >= W0 * W0) continue;
    const int lj = c / W0, li = c % W0;
    const int i = ib0 + li, j = jb0 + lj;
    T u = T(0);
    if (i >= 1 && i <= nf0 && j >= 1 && j <= nf0) {
      const int ci = H + (i >> 1) - Ic, cj = H + (j >> 1) - Jc;
      const T e = T(0.5) * (su1[cj][ci] + su1[cj + (j & 1)][ci + (i & 1)]);
      u = u0r[q] + e;
    }
    sf0[lj][li] = f0r[q];
    su0[lj][li] = u;
  }
  __syncthreads();
  tile_sweeps<T, W0, 2 * NU, kPairThreads>(su0, sf0, ib0, jb0, nf0, false);
  for (int c = t; c < 4 * kPairTile * kPairTile; c += kPairThreads) {
    const int bi = c % (2 * kPairTile), bj = c / (2 * kPairTile);
    const int i = 2 * I0 + 1 + bi, j = 2 * J0 + 1 + bj;
    if (i <= nf0 && j <= nf0)
      stg(eout0, (__umul24(j - 1, p0) + (i - 1)), su0[bj + H][bi + H]);
  }
}

// --------------------------------------------------------------------------------------------
// coarse levels in one workgroup
// --------------------------------------------------------------------------------------------
// Each level lives in LDS with a one-cell zero border ((nf + 2)^2 cells, row pitch nf + 2), so
// stencils need no bounds tests.  The 1024 threads form a 32 x 32 grid; thread (tx, ty) owns the
// points (tx + 1 + 32 a, ty + 1 + 32 b) of a level, at most 2 x 2 of them (nf <= 63).

constexpr int kCinvLds = 64;  // coarsest inverses up to 64 x 64 are staged in LDS

template <typename T>
struct CoarseLds;  // padded sizes of the in-LDS hierarchy
template <>
struct CoarseLds<double> {
  static constexpr int kMaxNf = 31;
  static constexpr int kElems = 33 * 33 + 17 * 17 + 9 * 9 + 5 * 5 + 3 * 3 + 128;
};

// one red or black half-sweep of a padded level (all reads of a thread before its writes)
template <typename T>
__device__ __forceinline__ void lds_halfsweep(T* u, const T* f, int nf, bool red) {
  const int pw = nf + 2;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  T acc[4];
  int off[4];
  bool ok[4];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int q = 2 * b + a;
      const int i = tx + 1 + 32 * a, j = ty + 1 + 32 * b;
      const int o = j * pw + i;
      ok[q] = i <= nf && j <= nf && is_red(i, j) == red;
      off[q] = o;
      acc[q] = ok[q] ? (f[o] + u[o - 1] + u[o + 1] + u[o - pw] + u[o + pw]) : T(0);
    }
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (ok[q]) u[off[q]] = T(0.25) * acc[q];
  __syncthreads();
}

// Levels first..nlev-1 entirely in LDS: V-cycle from the right-hand side fin (level `first`,
// global memory) to the result eout (global).  The coarsest level is solved exactly with the
// dense inverse cinv (nfc^2 x nfc^2, row-major), staged in LDS when small.
template <typename T, int NU>
__device__ __forceinline__ void d_coarse_vcycle(const T* __restrict__ fin, int pin,
                                                T* __restrict__ eout, const LaunchLevels& lv,
                                                const T* __restrict__ cinv) {
  __shared__ T buf[2 * CoarseLds<T>::kElems];
  __shared__ T scinv[kCinvLds * kCinvLds];
  const int first = lv.first, last = lv.nlev - 1;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  // Level sizes and offsets into buf go to LDS (read with constant indices here), so that later
  // accesses by level number neither index a private array nor lose the LDS address space.
  __shared__ int s_nf[kMaxLevels];
  __shared__ int s_off[kMaxLevels];
  int tot = 0, nf0 = 0, nfl = 0;
#pragma unroll
  for (int l = 0; l < kMaxLevels; ++l) {
    const int nfv = lv.nf[l];
    if (threadIdx.x == 0) {
      s_nf[l] = nfv;
      s_off[l] = tot;
    }
    if (l == first) nf0 = nfv;
    if (l == last) nfl = nfv;
    if (l >= first && l <= last) tot += 2 * (nfv + 2) * (nfv + 2);
  }
  auto UL = [&](int l) { return buf + s_off[l]; };
  auto FL = [&](int l) { return buf + s_off[l] + (s_nf[l] + 2) * (s_nf[l] + 2); };
  // issue the loads of the first level's right-hand side and of a small inverse first
  T v[2][2];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int i = tx + 1 + 32 * a, j = ty + 1 + 32 * b;
      v[b][a] = (i <= nf0 && j <= nf0) ? ldg(fin, (unsigned)((j - 1) * pin + (i - 1))) : T(0);
    }
  const int npc = nfl * nfl;
  if (npc <= kCinvLds) {
    constexpr int RC = kCinvLds * kCinvLds / kCoarseThreads;
    T cv[RC];
#pragma unroll
    for (int t = 0; t < RC; ++t) {
      const int k = threadIdx.x + t * kCoarseThreads;
      cv[t] = k < npc * npc ? ldg(cinv, (unsigned)k) : T(0);
    }
#pragma unroll
    for (int t = 0; t < RC; ++t) scinv[threadIdx.x + t * kCoarseThreads] = cv[t];
  }
  for (int k = threadIdx.x; k < tot; k += blockDim.x) buf[k] = T(0);
  __syncthreads();
  {
    const int pw = nf0 + 2;
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int i = tx + 1 + 32 * a, j = ty + 1 + 32 * b;
        if (i <= nf0 && j <= nf0) FL(first)[j * pw + i] = v[b][a];
      }
  }
  __syncthreads();
  // down: pre-smooth from zero (red first), restrict the residual
  for (int l = first; l < last; ++l) {
    const int nf = s_nf[l], nc = s_nf[l + 1];
    const int pw = nf + 2, pcw = nc + 2;
    T* u = UL(l);
    const T* f = FL(l);
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int i = tx + 1 + 32 * a, j = ty + 1 + 32 * b;
        if (i <= nf && j <= nf && is_red(i, j)) u[j * pw + i] = T(0.25) * f[j * pw + i];
      }
    __syncthreads();
    for (int s = 1; s < 2 * NU; ++s) lds_halfsweep(u, f, nf, !(s & 1));
    // coarse points: one per thread (nc <= 31)
    {
      const int I = tx + 1, J = ty + 1;
      if (I <= nc && J <= nc) {
        const int di[7] = {0, -1, 1, 0, 0, -1, 1};
        const int dj[7] = {0, 0, 0, -1, 1, -1, 1};
        T acc = T(0);
#pragma unroll
        for (int t = 0; t < 7; ++t) {
          const int o = (2 * J + dj[t]) * pw + (2 * I + di[t]);
          const T r = f[o] - (T(4) * u[o] - u[o - 1] - u[o + 1] - u[o - pw] - u[o + pw]);
          acc += (t == 0 ? T(1) : T(0.5)) * r;
        }
        FL(l + 1)[J * pcw + I] = acc;
      }
    }
    __syncthreads();
  }
  // coarsest: exact solve with the dense inverse; the right-hand side is first packed densely
  // (into the zero border-free tail of the buffer) so the product runs without index arithmetic
  {
    const int nf = nfl, pw = nf + 2;
    const int np = nf * nf;
    T* u = UL(last);
    const T* f = FL(last);
    T* fpk = buf + tot;  // room after the last level: np <= 256 cells
    for (int k = threadIdx.x; k < np; k += blockDim.x) fpk[k] = f[(k / nf + 1) * pw + (k % nf + 1)];
    __syncthreads();
    for (int k = threadIdx.x; k < np; k += blockDim.x) {
      T acc = T(0);
      if (np <= kCinvLds) {
#pragma unroll 7
        for (int m = 0; m < np; ++m) acc += scinv[k * np + m] * fpk[m];
      } else {
#pragma unroll 8
        for (int m = 0; m < np; ++m) acc += ldg(cinv, (unsigned)(k * np + m)) * fpk[m];
      }
      u[(k / nf + 1) * pw + (k % nf + 1)] = acc;
    }
    __syncthreads();
  }
  // up: prolongate and correct, post-smooth (black first)
  for (int l = last - 1; l >= first; --l) {
    const int nf = s_nf[l], pw = nf + 2, pcw = s_nf[l + 1] + 2;
    T* u = UL(l);
    const T* ec = UL(l + 1);
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int i = tx + 1 + 32 * a, j = ty + 1 + 32 * b;
        if (i > nf || j > nf) continue;
        const int o = (j >> 1) * pcw + (i >> 1);
        const T e = T(0.5) * (ec[o] + ec[o + (j & 1) * pcw + (i & 1)]);
        u[j * pw + i] += e;
      }
    __syncthreads();
    for (int s = 0; s < 2 * NU; ++s) lds_halfsweep(u, FL(l), nf, (s & 1));
  }
  {
    const int pw = nf0 + 2;
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int i = tx + 1 + 32 * a, j = ty + 1 + 32 * b;
        if (i <= nf0 && j <= nf0) stg(eout, (unsigned)((j - 1) * pin + (i - 1)), UL(first)[j * pw + i]);
      }
  }
}

// --------------------------------------------------------------------------------------------
// FP32 coarse-grid solve by sine transforms
// --------------------------------------------------------------------------------------------
// The 5-point operator on an m x m grid with zero Dirichlet values is diagonalised by the
// orthonormal sine transform S (S_ab = sqrt(2 / (m + 1)) sin(pi (a + 1)(b + 1) / (m + 1))):
// A = S diag(c_p + c_q) S with c_k = 2 - 2 cos(pi (k + 1) / (m + 1)).  The first level handled by
// one workgroup is solved exactly as U = S ((S F S) ./ (c_p + c_q)) S: four 64 x 64 products in
// LDS on the matrix cores (v_mfma_f32_16x16x4_f32), each of the 16 waves owning a 16 x 16 tile.
// Rows and columns beyond m are zero in S, so the padding stays zero.
constexpr int kDstP = kDstN + 1;  // LDS row pitch (odd: a fragment's 16 rows hit 16 banks)
typedef float dst_f4 __attribute__((ext_vector_type(4)));

// Tile (ti, tj) of A B (A, B: kDstN x kDstN in LDS).  Fragment layout of the 16x16x4 FP32
// instruction: lane l supplies A(row l % 16, k l / 16) and B(k l / 16, col l % 16); result
// register q holds C(row 4 (l / 16) + q, col l % 16).
__device__ __forceinline__ dst_f4 dst_tile(const float* A, const float* B, int ti, int tj,
                                           int lane) {
  dst_f4 acc = {0.f, 0.f, 0.f, 0.f};
  const int r = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int k0 = 0; k0 < kDstN; k0 += 4) {
    const float a = A[(16 * ti + r) * kDstP + k0 + kq];
    const float b = B[(k0 + kq) * kDstP + 16 * tj + r];
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
  }
  return acc;
}

// Operands of the sine-transform solve, loaded into registers by 1024 threads (S, the right-hand
// side f of the m x m level with row pitch pin, zero-padded to kDstN x kDstN, and the symbols).
struct DstIn {
  static constexpr int Q = kDstN * kDstN / 1024;
  float sv[Q], fv[Q], lv;
};
__device__ __forceinline__ void dst_load(DstIn& in, const float* __restrict__ fin, int pin, int m,
                                         const float* __restrict__ Sg,
                                         const float* __restrict__ lamg, int t) {
#pragma unroll
  for (int q = 0; q < DstIn::Q; ++q) {
    const int idx = t + 1024 * q;
    const int row = idx / kDstN, col = idx % kDstN;
    in.sv[q] = ldg(Sg, (unsigned)idx);
    in.fv[q] = (row < m && col < m) ? ldg(fin, (unsigned)(row * pin + col)) : 0.f;
  }
  in.lv = t < kDstN ? ldg(lamg, (unsigned)t) : 0.f;
}

// e = A^{-1} f on the m x m level (m <= kDstN - 1) from the loaded operands, in the LDS arrays
// sS, sX, sY (kDstN x kDstP each) and sl (kDstN); needs 1024 threads (16 waves, each owning a
// 16 x 16 tile of every product).  e(p, q) goes to out[(p + off) * opitch + q + off], a global
// array (GLOBAL) or an LDS one.
template <bool GLOBAL>
__device__ __forceinline__ void dst_solve(const DstIn& in, float* sS, float* sX, float* sY,
                                          float* sl, int m, int t, float* out, int opitch,
                                          int off) {
  static_assert(kDstN == 64, "4 x 4 tiles of 16 x 16");
#pragma unroll
  for (int q = 0; q < DstIn::Q; ++q) {
    const int idx = t + 1024 * q;
    const int row = idx / kDstN, col = idx % kDstN;
    sS[row * kDstP + col] = in.sv[q];
    sX[row * kDstP + col] = in.fv[q];
  }
  if (t < kDstN) sl[t] = in.lv;
  __syncthreads();
  const int w = t >> 6, lane = t & 63;
  const int ti = w >> 2, tj = w & 3;
  const int col = 16 * tj + (lane & 15), row0 = 16 * ti + 4 * (lane >> 4);
  // Y = S F
  dst_f4 acc = dst_tile(sS, sX, ti, tj, lane);
#pragma unroll
  for (int q = 0; q < 4; ++q) sY[(row0 + q) * kDstP + col] = acc[q];
  __syncthreads();
  // X = (Y S) ./ (c_p + c_q)
  acc = dst_tile(sY, sS, ti, tj, lane);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int p = row0 + q;
    sX[p * kDstP + col] = (p < m && col < m) ? acc[q] / (sl[p] + sl[col]) : 0.f;
  }
  __syncthreads();
  // Y = S X
  acc = dst_tile(sS, sX, ti, tj, lane);
#pragma unroll
  for (int q = 0; q < 4; ++q) sY[(row0 + q) * kDstP + col] = acc[q];
  __syncthreads();
  // e = Y S
  acc = dst_tile(sY, sS, ti, tj, lane);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int p = row0 + q;
    if (p < m && col < m) {
      const unsigned o = (unsigned)((p + off) * opitch + col + off);
      if constexpr (GLOBAL) stg(out, o, acc[q]);
      else out[o] = acc[q];
    }
  }
}

// e = A^{-1} f on the m x m level (m <= kDstN - 1); f and e in global memory with row pitch pin.
// Needs kCoarseThreads = 1024 threads (16 waves).
__device__ __forceinline__ void d_coarse_dst(const float* __restrict__ fin, int pin,
                                             float* __restrict__ eout, int m,
                                             const float* __restrict__ Sg,
                                             const float* __restrict__ lamg) {
  static_assert(kCoarseThreads == 1024, "16 waves");
  __shared__ float sS[kDstN * kDstP];
  __shared__ float sX[kDstN * kDstP];
  __shared__ float sY[kDstN * kDstP];
  __shared__ float sl[kDstN];
  const int t = threadIdx.x;
  DstIn in;
  dst_load(in, fin, pin, m, Sg, lamg, t);
  dst_solve<true>(in, sS, sX, sY, sl, m, t, eout, pin, 0);
}

// The coarse solve and three levels going up, in FP32: every block first solves the coarse level
// l+3 (m x m points) exactly by sine transforms, as d_coarse_dst does, into LDS; then level l+2
// as the intermediate-level up kernel does (u_{l+2} = u_{l+2,pre} + P e_{l+3}, 2 nu half-sweeps),
// on a window whose valid part covers the coarse patch that level l+1 interpolates from; then
// levels l+1 and l as d_pair_up.  It replaces the coarse kernel, that up kernel and the pair
// kernel above it (two launches fewer per V-cycle where the last tiled level runs alone); each
// block repeats the coarse solve (a few microseconds of matrix-core work, in parallel on every
// compute unit) instead of waiting for it.  Every value sees the same operations as in the
// separate kernels, so the results are bit-identical.
template <int NU>
struct TripleUp {
  using G = PairUp<NU>;
  static constexpr int H = G::H;
  static constexpr int W2r = G::CW2 + 2 * H;            // level-(l+2) window around the patch
  static constexpr int W2 = W2r + (W2r & 1);             // (even: the sweeps take column pairs)
  static constexpr int N2 = (W2 * W2 + kPairThreads - 1) / kPairThreads;
};

template <int NU>
__device__ __forceinline__ void d_triple_up(
    const float* __restrict__ f0, const float* __restrict__ u0pre, const float* __restrict__ f1,
    const float* __restrict__ u1pre, const float* __restrict__ f2, const float* __restrict__ u2pre,
    const float* __restrict__ f3, const float* __restrict__ Sg, const float* __restrict__ lamg,
    float* __restrict__ eout0, int nf0, int p0, int p1, int p2, int p3, int tile_x, int tile_y) {
  using T = float;
  using G = PairUp<NU>;
  using G3 = TripleUp<NU>;
  constexpr int H = G::H, W0 = G::W0, W1 = G::W1, W2 = G3::W2;
  static_assert(kPairThreads == 1024, "16 waves");
  __shared__ T sf0[W0][W0 + 1];
  __shared__ T su0[W0][W0 + 1];
  __shared__ T sf1[W1][W1 + 1];
  __shared__ T su1[W1][W1 + 1];
  __shared__ T sf2[W2][W2 + 1];
  __shared__ T su2[W2][W2 + 1];
  __shared__ float sS[kDstN * kDstP];
  __shared__ float sX[kDstN * kDstP];
  __shared__ float sY[kDstN * kDstP];
  __shared__ float sl[kDstN];
  __shared__ float se[kDstN + 1][kDstN + 2];  // e_{l+3} by coarse index, zero ring
  const int t = flat_tid();
  __builtin_assume(t >= 0 && t < kPairThreads);
  const int nf1 = (nf0 - 1) >> 1, nf2 = (nf1 - 1) >> 1, nf3 = (nf2 - 1) >> 1;
  const int I0 = tile_x * kPairTile, J0 = tile_y * kPairTile;
  const int ib0 = 2 * I0 + 1 - H, jb0 = 2 * J0 + 1 - H;  // level-l window origin
  const int Ic = ib0 >> 1, Jc = jb0 >> 1;                // its coarse patch origin (floor)
  const int ib1 = Ic - H, jb1 = Jc - H;                  // level-(l+1) window origin
  const int Ic2 = ib1 >> 1, Jc2 = jb1 >> 1;              // coarse patch of level l+2
  const int ib2 = Ic2 - H, jb2 = Jc2 - H;                // level-(l+2) window origin
  const int m = nf3;                                     // coarse level: m x m points
  DstIn din;
  dst_load(din, f3, p3, m, Sg, lamg, t);
  T f2r[G3::N2], u2r[G3::N2], f1r[G::N1], u1r[G::N1], f0r[G::N0], u0r[G::N0];
#pragma unroll
  for (int q = 0; q < G3::N2; ++q) {
    const int c = t + kPairThreads * q;
    const int i = ib2 + c % W2, j = jb2 + c / W2;
    const bool in = c < W2 * W2 && i >= 1 && i <= nf2 && j >= 1 && j <= nf2;
    const unsigned o = (__umul24(j - 1, p2) + (i - 1));
    f2r[q] = in ? ldg(f2, o) : T(0);
    u2r[q] = in ? ldg(u2pre, o) : T(0);
  }
#pragma unroll
  for (int q = 0; q < G::N1; ++q) {
    const int c = t + kPairThreads * q;
    const int i = ib1 + c % W1, j = jb1 + c / W1;
    const bool in = c < W1 * W1 && i >= 1 && i <= nf1 && j >= 1 && j <= nf1;
    const unsigned o = (__umul24(j - 1, p1) + (i - 1));
    f1r[q] = in ? ldg(f1, o) : T(0);
    u1r[q] = in ? ldg(u1pre, o) : T(0);
  }
#pragma unroll
  for (int q = 0; q < G::N0; ++q) {
    const int c = t + kPairThreads * q;
    const int i = ib0 + c % W0, j = jb0 + c / W0;
    const bool in = c < W0 * W0 && i >= 1 && i <= nf0 && j >= 1 && j <= nf0;
    const unsigned o = (__umul24(j - 1, p0) + (i - 1));
    f0r[q] = in ? ldg(f0, o) : T(0);
    u0r[q] = in ? ldg(u0pre, o) : T(0);
  }
  // the coarse solve, as in d_coarse_dst, into se (zero ring)
  for (int c = t; c < (kDstN + 1) * (kDstN + 2); c += kPairThreads) (&se[0][0])[c] = 0.f;
  dst_solve<false>(din, sS, sX, sY, sl, m, t, &se[0][0], kDstN + 2, 1);
  __syncthreads();
  // level l+2: prolongation of e_{l+3} plus the pre-smoothed iterate, 2 nu half-sweeps
#pragma unroll
  for (int q = 0; q < G3::N2; ++q) {
    const int c = t + kPairThreads * q;
    if (c >= W2 * W2) continue;
    const int lj = c / W2, li = c % W2;
    const int i = ib2 + li, j = jb2 + lj;
    T u = T(0);
    if (i >= 1 && i <= nf2 && j >= 1 && j <= nf2) {
      const int ci = i >> 1, cj = j >> 1;
      const T e = T(0.5) * (se[cj][ci] + se[cj + (j & 1)][ci + (i & 1)]);
      u = u2r[q] + e;
    }
    sf2[lj][li] = f2r[q];
    su2[lj][li] = u;
  }
  __syncthreads();
  tile_sweeps<T, W2, 2 * NU, kPairThreads>(su2, sf2, ib2, jb2, nf2, false);  // black, red, ...
  // level l+1: the corrected level-(l+2) values on its patch are su2[H + c][H + d]
#pragma unroll
  for (int q = 0; q < G::N1; ++q) {
    const int c = t + kPairThreads * q;
    if (c >= W1 * W1) continue;
    const int lj = c / W1, li = c % W1;
    const int i = ib1 + li, j = jb1 + lj;
    T u = T(0);
    if (i >= 1 && i <= nf1 && j >= 1 && j <= nf1) {
      const int ci = H + (i >> 1) - Ic2, cj = H + (j >> 1) - Jc2;
      const T e = T(0.5) * (su2[cj][ci] + su2[cj + (j & 1)][ci + (i & 1)]);
      u = u1r[q] + e;
    }
    sf1[lj][li] = f1r[q];
    su1[lj][li] = u;
  }
  __syncthreads();
  tile_sweeps<T, W1, 2 * NU, kPairThreads>(su1, sf1, ib1, jb1, nf1, false);
  // level l
#pragma unroll
  for (int q = 0; q < G::N0; ++q) {
    const int c = t + kPairThreads * q;
    if (c >= W0 * W0) continue;
    const int lj = c / W0, li = c % W0;
    const int i = ib0 + li, j = jb0 + lj;
    T u = T(0);
    if (i >= 1 && i <= nf0 && j >= 1 && j <= nf0) {
      const int ci = H + (i >> 1) - Ic, cj = H + (j >> 1) - Jc;
      const T e = T(0.5) * (su1[cj][ci] + su1[cj + (j & 1)][ci + (i & 1)]);
      u = u0r[q] + e;
    }
    sf0[lj][li] = f0r[q];
    su0[lj][li] = u;
  }
  __syncthreads();
  tile_sweeps<T, W0, 2 * NU, kPairThreads>(su0, sf0, ib0, jb0, nf0, false);
  for (int c = t; c < 4 * kPairTile * kPairTile; c += kPairThreads) {
    const int bi = c % (2 * kPairTile), bj = c / (2 * kPairTile);
    const int i = 2 * I0 + 1 + bi, j = 2 * J0 + 1 + bj;
    if (i <= nf0 && j <= nf0)
      stg(eout0, (__umul24(j - 1, p0) + (i - 1)), su0[bj + H][bi + H]);
  }
}

// The whole up side of an FP32 V-cycle whose tiled levels are 1 (the finest's first coarse
// level), 2 and 3, with the coarse level 4 solved by sine transforms, in one launch: every
// 1024-thread block solves level 4 (as d_triple_up), then corrects and smooths levels 3, 2 and 1
// on windows whose valid parts cover the coarse patch each finer window interpolates from, and
// finally does the finest level as the CG up kernel does (u_0 = u_0,pre + P e_1, 2 nu half-sweeps,
// z stored, the dots r.z and z.A z) on a 64 x 64 tile.  It replaces d_triple_up and the finest
// up kernel (one launch and one inter-kernel gap fewer per V-cycle).  Every value sees the same
// operations as in the separate kernels; the dots are summed per block (one r.z and one z.A z
// partial per 64 x 64 tile, a quarter of the finest up kernel's count), so the same products are
// summed in another order.
template <int NU>
struct QuadUp {
  static constexpr int H0 = 2 * NU + 1;            // finest halo (z valid one beyond the tile)
  static constexpr int T0 = 4 * kPairTile;         // finest tile edge (64)
  static constexpr int W0 = T0 + 2 * H0;           // finest window
  static constexpr int CW0 = W0 / 2 + 2;           // its coarse patch (valid part of level 1)
  static constexpr int H = 2 * NU;                 // halo of the coarser up windows
  static constexpr int W1 = CW0 + 2 * H + ((CW0 + 2 * H) & 1);   // even: sweeps take pairs
  static constexpr int CW1 = W1 / 2 + 2;
  static constexpr int W2 = CW1 + 2 * H + ((CW1 + 2 * H) & 1);
  static constexpr int CW2 = W2 / 2 + 2;
  static constexpr int W3 = CW2 + 2 * H + ((CW2 + 2 * H) & 1);
  static constexpr int N0 = (W0 * W0 + kPairThreads - 1) / kPairThreads;
  static constexpr int N1 = (W1 * W1 + kPairThreads - 1) / kPairThreads;
  static constexpr int N2 = (W2 * W2 + kPairThreads - 1) / kPairThreads;
  static constexpr int N3 = (W3 * W3 + kPairThreads - 1) / kPairThreads;
  static_assert(2 * W0 * (W0 + 1) <= 3 * kDstN * kDstP, "the finest windows fit the DST arrays");
};

// A window of an up kernel with kPairThreads threads: f and u_pre into registers (zero outside
// the grid), all loads issued before any is used.
template <int N, int W>
__device__ __forceinline__ void up_window_load(float (&fr)[N], float (&ur)[N], int t, int ib,
                                               int jb, int nf, int pitch,
                                               const float* __restrict__ fin,
                                               const float* __restrict__ upre) {
#pragma unroll
  for (int q = 0; q < N; ++q) {
    const int c = t + kPairThreads * q;
    const int i = ib + c % W, j = jb + c / W;
    const bool in = c < W * W && i >= 1 && i <= nf && j >= 1 && j <= nf;
    const unsigned o = (__umul24(j - 1, pitch) + (i - 1));
    fr[q] = in ? ldg(fin, o) : 0.f;
    ur[q] = in ? ldg(upre, o) : 0.f;
  }
}

// u = u_pre + P e on a window (e from the coarser level's values coarse(J - cjb, I - cib), valid
// there), f and u into LDS.
template <int N, int W, typename C>
__device__ __forceinline__ void up_window_init(float (*sf)[W + 1], float (*su)[W + 1],
                                               const float (&fr)[N], const float (&ur)[N], int t,
                                               int ib, int jb, int nf, const C& coarse, int cib,
                                               int cjb) {
#pragma unroll
  for (int q = 0; q < N; ++q) {
    const int c = t + kPairThreads * q;
    if (c >= W * W) continue;
    const int lj = c / W, li = c % W;
    const int i = ib + li, j = jb + lj;
    float u = 0.f;
    if (i >= 1 && i <= nf && j >= 1 && j <= nf) {
      const int ci = (i >> 1) - cib, cj = (j >> 1) - cjb;
      const float e = 0.5f * (coarse(cj, ci) + coarse(cj + (j & 1), ci + (i & 1)));
      u = ur[q] + e;
    }
    sf[lj][li] = fr[q];
    su[lj][li] = u;
  }
  __syncthreads();
}

template <int NU>
__device__ __forceinline__ void d_quad_up(
    const float* __restrict__ f0, const float* __restrict__ u0pre, const float* __restrict__ f1,
    const float* __restrict__ u1pre, const float* __restrict__ f2, const float* __restrict__ u2pre,
    const float* __restrict__ f3, const float* __restrict__ u3pre, const float* __restrict__ f4,
    const float* __restrict__ Sg, const float* __restrict__ lamg, float* __restrict__ z,
    int nf0, int p0, int p1, int p2, int p3, int p4, DevState* st, const Reductions& red, int kn,
    int count_iteration, int tile_x, int tile_y, bool lead) {
  using T = float;
  using G = QuadUp<NU>;
  constexpr int H0 = G::H0, H = G::H, W0 = G::W0, W1 = G::W1, W2 = G::W2, W3 = G::W3;
  constexpr int TT = G::T0;
  static_assert(kPairThreads == 1024, "16 waves");
  // the sine-transform arrays; after the coarse solve they hold the finest level's windows
  __shared__ float sdst[3 * kDstN * kDstP];
  __shared__ float sl[kDstN];
  __shared__ float se[kDstN + 1][kDstN + 2];  // e_4 by coarse index, zero ring
  __shared__ T sf1[W1][W1 + 1];
  __shared__ T su1[W1][W1 + 1];
  __shared__ T sf2[W2][W2 + 1];
  __shared__ T su2[W2][W2 + 1];
  __shared__ T sf3[W3][W3 + 1];
  __shared__ T su3[W3][W3 + 1];
  __shared__ double sdot[kPairThreads / 64][8];
  float* sS = sdst;
  float* sX = sdst + kDstN * kDstP;
  float* sY = sdst + 2 * kDstN * kDstP;
  auto sf0 = reinterpret_cast<T(*)[W0 + 1]>(sdst);
  auto su0 = reinterpret_cast<T(*)[W0 + 1]>(sdst + W0 * (W0 + 1));
  const int t = flat_tid();
  __builtin_assume(t >= 0 && t < kPairThreads);
  const int nf1 = (nf0 - 1) >> 1, nf2 = (nf1 - 1) >> 1, nf3 = (nf2 - 1) >> 1, m = (nf3 - 1) >> 1;
  const int i0 = tile_x * TT, j0 = tile_y * TT;
  const int ib0 = i0 + 1 - H0, jb0 = j0 + 1 - H0;           // finest window origin
  const int ib1 = (ib0 >> 1) - H, jb1 = (jb0 >> 1) - H;     // level-1 window (floor shifts)
  const int ib2 = (ib1 >> 1) - H, jb2 = (jb1 >> 1) - H;
  const int ib3 = (ib2 >> 1) - H, jb3 = (jb2 >> 1) - H;
  DstIn din;
  dst_load(din, f4, p4, m, Sg, lamg, t);
  T f3r[G::N3], u3r[G::N3], f2r[G::N2], u2r[G::N2], f1r[G::N1], u1r[G::N1], f0r[G::N0], u0r[G::N0];
  up_window_load<G::N3, W3>(f3r, u3r, t, ib3, jb3, nf3, p3, f3, u3pre);
  up_window_load<G::N2, W2>(f2r, u2r, t, ib2, jb2, nf2, p2, f2, u2pre);
  up_window_load<G::N1, W1>(f1r, u1r, t, ib1, jb1, nf1, p1, f1, u1pre);
  up_window_load<G::N0, W0>(f0r, u0r, t, ib0, jb0, nf0, p0, f0, u0pre);
  // the coarse solve into se (zero ring)
  for (int c = t; c < (kDstN + 1) * (kDstN + 2); c += kPairThreads) (&se[0][0])[c] = 0.f;
  dst_solve<false>(din, sS, sX, sY, sl, m, t, &se[0][0], kDstN + 2, 1);
  __syncthreads();
  // each level: u = u_pre + P e from the coarser level's (valid) values, then 2 nu half-sweeps
  up_window_init<G::N3, W3>(sf3, su3, f3r, u3r, t, ib3, jb3, nf3,
                            [&](int a, int b) { return se[a][b]; }, 0, 0);
  tile_sweeps<T, W3, 2 * NU, kPairThreads>(su3, sf3, ib3, jb3, nf3, false);  // black, red, ...
  up_window_init<G::N2, W2>(sf2, su2, f2r, u2r, t, ib2, jb2, nf2,
                            [&](int a, int b) { return su3[a][b]; }, ib3, jb3);
  tile_sweeps<T, W2, 2 * NU, kPairThreads>(su2, sf2, ib2, jb2, nf2, false);
  up_window_init<G::N1, W1>(sf1, su1, f1r, u1r, t, ib1, jb1, nf1,
                            [&](int a, int b) { return su2[a][b]; }, ib2, jb2);
  tile_sweeps<T, W1, 2 * NU, kPairThreads>(su1, sf1, ib1, jb1, nf1, false);
  up_window_init<G::N0, W0>(sf0, su0, f0r, u0r, t, ib0, jb0, nf0,
                            [&](int a, int b) { return su1[a][b]; }, ib1, jb1);
  tile_sweeps<T, W0, 2 * NU, kPairThreads>(su0, sf0, ib0, jb0, nf0, false);
  // z on the own cells; r.z and z.A z per 32 x 32 sub-tile first (sub-tile column by lane half,
  // row by slot half: thread t covers cells (t % 64, t / 64 + 16 q))
  double dz[2][2] = {{0.0, 0.0}, {0.0, 0.0}};   // [sub-tile row][r.z, z.A z]
#pragma unroll
  for (int q = 0; q < TT * TT / kPairThreads; ++q) {
    const int c = t + kPairThreads * q;
    const int bi = c % TT, bj = c / TT;
    const int i = i0 + 1 + bi, j = j0 + 1 + bj;
    if (j > nf0 || i > nf0) continue;
    const int lj = bj + H0, li = bi + H0;
    const T zv = su0[lj][li];
    stg(z, (__umul24(j - 1, p0) + (i - 1)), zv);
    const T wv = T(4) * zv - su0[lj][li - 1] - su0[lj][li + 1] - su0[lj - 1][li] - su0[lj + 1][li];
    const int sy = q >= (TT * TT / kPairThreads) / 2 ? 1 : 0;
    dz[sy][0] += (double)sf0[lj][li] * (double)zv;
    dz[sy][1] += (double)zv * (double)wv;
  }
  // each half-wave (32 lanes) holds one sub-tile column: reduce within halves, fixed order
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
      for (int o = 16; o > 0; o >>= 1) dz[a][b] += __shfl_down(dz[a][b], o, 32);
  const int lane = t & 63, w = t >> 6;
  if ((lane & 31) == 0) {
    const int sx = lane >> 5;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) sdot[w][(a * 2 + sx) * 2 + b] = dz[a][b];
  }
  __syncthreads();
  // one partial of each per block, stored at the block's tile index (the down kernels read
  // gridDim.x * gridDim.y of them, red.nbd): lane 2 sub + b sums sub-tile sub's value b over
  // the waves, then lanes 0 and 1 add the four sub-tiles in order
  if (t < 8) {
    double v = 0.0;
    for (int q = 0; q < kPairThreads / 64; ++q) v += sdot[q][t];
    const double v2 = __shfl_down(v, 2, 8), v4 = __shfl_down(v, 4, 8), v6 = __shfl_down(v, 6, 8);
    if (t < 2) {
      double* dst = t == 0 ? ((kn & 1) ? red.rz[1] : red.rz[0]) : ((kn & 1) ? red.zw[1] : red.zw[0]);
      stg(dst, (unsigned)(tile_y * gridDim.x + tile_x), ((v + v2) + v4) + v6);
    }
  }
  if (count_iteration && lead && thread0()) {
    st->inner_its += 1;
    st->pcg_k += 1;
    st->run_its_max = max(st->run_its_max, st->pcg_k);
  }
}

// --------------------------------------------------------------------------------------------
// FP64 residual of the interior solve (iterative refinement)
// --------------------------------------------------------------------------------------------

__device__ __forceinline__ double rhs_at(const RhsDesc& f, int nf, int i, int j) {
  double v = 0.0;
  if (f.b) v = f.sb * ldg(f.b, (unsigned)((j - 1) * nf + (i - 1)));
  if (f.g && j == nf) v += f.sg * ldg(f.g, (unsigned)(i - 1));
  return v;
}

// first: u_out = 0, r = f.  Otherwise u_out = u_in + e and r = f - A u_out, or, once the solve
// has converged, the copy u_out = u_in (so buffer parity follows the schedule).  r is written as
// FP32 or FP64; the block's ||r||^2 goes to red.ir (and red.ff on the first call).
template <typename E>
__device__ __forceinline__ void d_ir_residual(
    const RhsDesc& f, const double* __restrict__ uin, const E* __restrict__ e,
    double* __restrict__ uout, float* __restrict__ r32, double* __restrict__ r64, int nf,
    int pitch, int first, double tol2, double tau2, int pcg_is_final, DevState* st,
    const Reductions& red, int tile_x, int tile_y, int tile, bool lead,
    const float* __restrict__ warm = nullptr, const double* __restrict__ wscale = nullptr,
    bool run_check = false) {
  constexpr int W = kTile + 2;
  __shared__ double su[W][W + 1];
  const int i0 = tile_x * kTile, j0 = tile_y * kTile;
  if (!first && st->solve_done) {
    for (int b = threadIdx.y; b < kTile; b += blockDim.y) {
      const int j = j0 + 1 + b;
      if (j > nf) continue;
      for (int a = threadIdx.x; a < kTile; a += blockDim.x) {
        const int i = i0 + 1 + a;
        if (i > nf) continue;
        const unsigned o = (unsigned)((j - 1) * pitch + (i - 1));
        stg(uout, o, ldg(uin, o));
      }
    }
    return;
  }
  // run_check: the PCG run that ends here stopped after an update without a V-cycle; the lead
  // block takes its convergence test (a run that has not converged counts the iteration, so
  // that its recorded length tells the schedule that it needed more)
  if (run_check && lead && !stopped(st)) {
    if (!pcg_converged(st, red, true) && thread0()) {
      st->inner_its += 1;
      st->pcg_k += 1;
      st->run_its_max = max(st->run_its_max, st->pcg_k);
    }
  }
  constexpr int RY = Slots<W>::RY, RX = Slots<W>::RX;
  // first call: u = 0, or u = s g for a learned guess g (compact FP32 image) with scale s
  const double ws = (first && warm) ? *wscale : 0.0;
  // window loads at clamped offsets (cells outside the grid read element 0 and are zeroed), all
  // issued before any is used: one memory latency for the window, not one per slot
  double ur[RY][RX];
  if (!first) {
    double ua[RY][RX];
    E ea[RY][RX];
#pragma unroll
    for (int a = 0; a < RY; ++a)
#pragma unroll
      for (int b = 0; b < RX; ++b) {
        const int lj = threadIdx.y + 8 * a, li = threadIdx.x + 32 * b;
        const int i = i0 + li, j = j0 + lj;
        const bool cell = lj < W && li < W && i >= 1 && i <= nf && j >= 1 && j <= nf;
        const unsigned o = cell ? (unsigned)((j - 1) * pitch + (i - 1)) : 0u;
        ua[a][b] = ldg(uin, o);
        ea[a][b] = ldg(e, o);
      }
#pragma unroll
    for (int a = 0; a < RY; ++a)
#pragma unroll
      for (int b = 0; b < RX; ++b) {
        const int lj = threadIdx.y + 8 * a, li = threadIdx.x + 32 * b;
        const int i = i0 + li, j = j0 + lj;
        const bool cell = lj < W && li < W && i >= 1 && i <= nf && j >= 1 && j <= nf;
        ur[a][b] = cell ? ua[a][b] + (double)ea[a][b] : 0.0;
      }
  } else {
    float wa[RY][RX];
#pragma unroll
    for (int a = 0; a < RY; ++a)
#pragma unroll
      for (int b = 0; b < RX; ++b) {
        const int lj = threadIdx.y + 8 * a, li = threadIdx.x + 32 * b;
        const int i = i0 + li, j = j0 + lj;
        const bool cell = lj < W && li < W && i >= 1 && i <= nf && j >= 1 && j <= nf;
        wa[a][b] = warm ? ldg(warm, cell ? (unsigned)((j - 1) * nf + (i - 1)) : 0u) : 0.f;
        ur[a][b] = (warm && cell) ? ws * (double)wa[a][b] : 0.0;
      }
  }
#pragma unroll
  for (int a = 0; a < RY; ++a)
#pragma unroll
    for (int b = 0; b < RX; ++b) {
      const int lj = threadIdx.y + 8 * a, li = threadIdx.x + 32 * b;
      if (lj < W && li < W) su[lj][li] = ur[a][b];
    }
  __syncthreads();
  // own cells: column threadIdx.x, rows threadIdx.y + 8 q (32 x 8 threads); the right-hand side
  // of all of them is loaded first (clamped offsets, as above)
  constexpr int NQ = kTile / 8;
  double fb[NQ];
  const double gv = f.g ? ldg(f.g, (unsigned)min(i0 + (int)threadIdx.x, nf - 1)) : 0.0;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int i = i0 + 1 + (int)threadIdx.x, j = j0 + 1 + (int)threadIdx.y + 8 * q;
    const bool own = i <= nf && j <= nf;
    fb[q] = f.b ? ldg(f.b, own ? (unsigned)((j - 1) * nf + (i - 1)) : 0u) : 0.0;
  }
  double rr = 0.0, fsq = 0.0;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int b = (int)threadIdx.y + 8 * q, a = (int)threadIdx.x;
    const int j = j0 + 1 + b, i = i0 + 1 + a;
    if (j > nf || i > nf) continue;
    {
      const int li = a + 1, lj = b + 1;
      const double u = su[lj][li];
      // f = sb b + (on the row next to Gamma) sg g, in that order
      double fv = 0.0;
      if (f.b) fv = f.sb * fb[q];
      if (f.g && j == nf) fv += f.sg * gv;
      const double r = fv - (4.0 * u - su[lj][li - 1] - su[lj][li + 1] - su[lj - 1][li] -
                             su[lj + 1][li]);
      const unsigned o = (unsigned)((j - 1) * pitch + (i - 1));
      stg(uout, o, u);
      if (r32) stg(r32, o, (float)r);
      if (r64) stg(r64, o, r);
      rr += r * r;
      fsq += fv * fv;
    }
  }
  const double tot = block_sum_all(rr);
  const double ftot = first ? block_sum_all(fsq) : 0.0;
  if (thread0()) {
    red.ir[tile] = tot;
    if (first) red.ff[tile] = ftot;
    if (lead) {
      if (first) {
        st->tol2 = tol2;
        st->tau2 = tau2;
        st->pcg_is_final = pcg_is_final;
        st->breakdown = 0;
        st->inner_its = 0;
        st->refine_steps = 0;
        st->run_its_max = 0;
        for (int q = 0; q < 8; ++q) st->run_len[q] = 0;
        st->solve_done = 0;
      } else {
        if (st->refine_steps < 8) st->run_len[st->refine_steps] = st->pcg_k;
        st->refine_steps += 1;
      }
    }
  }
}

// A learned initial guess g for A u = f enters scaled by the Galerkin factor
// alpha = f.g / g.A g, the minimizer of the energy error ||u - alpha g||_A over alpha; the guess is
// used when alpha > 0 (then alpha g has a smaller energy error than the zero guess) and dropped
// (alpha = 0) otherwise.  d_warm_dots stores the tile partials of f.g and g.A g (g is the FP32
// image with pitch nf; A the 5-point operator with zero Dirichlet values); d_warm_alpha sums
// them and sets st->warm_alpha, which the first residual then applies.
__device__ __forceinline__ void d_warm_dots(const RhsDesc& f, const float* __restrict__ g, int nf,
                                            const Reductions& red, int tile_x, int tile_y,
                                            int tile) {
  const int i0 = tile_x * kTile, j0 = tile_y * kTile;
  auto gv = [&](int i, int j) -> double {
    return (i >= 1 && i <= nf && j >= 1 && j <= nf)
               ? (double)ldg(g, (unsigned)((j - 1) * nf + (i - 1)))
               : 0.0;
  };
  double fg = 0.0, gag = 0.0;
  for (int b = threadIdx.y; b < kTile; b += blockDim.y) {
    const int j = j0 + 1 + b;
    if (j > nf) continue;
    for (int a = threadIdx.x; a < kTile; a += blockDim.x) {
      const int i = i0 + 1 + a;
      if (i > nf) continue;
      const double c = gv(i, j);
      const double ag = 4.0 * c - gv(i - 1, j) - gv(i + 1, j) - gv(i, j - 1) - gv(i, j + 1);
      fg += rhs_at(f, nf, i, j) * c;
      gag += c * ag;
    }
  }
  const double tfg = block_sum_all(fg);
  const double tgag = block_sum_all(gag);
  if (thread0()) {
    red.ir[tile] = tfg;
    red.ff[tile] = tgag;
  }
}

__device__ __forceinline__ void d_warm_alpha(DevState* st, const Reductions& red) {
  const double fg = sum_partials(red.ir, red.nb0);
  const double gag = sum_partials(red.ff, red.nb0);
  if (thread0()) {
    const double al = fg / gag;
    const bool ok = gag > 0.0 && isfinite(al) && al > 0.0;
    st->warm_alpha = ok ? al : 0.0;
    st->warm_used = ok ? 1 : 0;
  }
}

// Reads the refinement residual back from the partials and sets the solve's state for the next
// PCG run (or ends the solve).  Run by every block of the kernel that starts the next PCG run (or
// by a one-block kernel): all blocks sum the same partials in the same order, so they agree on
// whether the solve is over, and only the lead block records the state.  Returns true when the
// solve is over.
__device__ __forceinline__ bool ir_finalize_here(DevState* st, const Reductions& red, bool lead) {
  if (st->solve_done) return true;
  const double r2 = sum_partials(red.ir, red.nb0);
  const double ff = sum_partials(red.ff, red.nb0);
  const bool bad = !isfinite(r2);
  const bool done = bad || r2 <= st->tol2 * ff;
  if (lead && thread0()) {
    st->ff = ff;
    st->res2 = r2;
    st->rr0 = r2;
    st->inner_done = 0;
    st->pcg_k = 0;
    if (bad) st->breakdown |= 4;
    if (done) st->solve_done = 1;
  }
  return done;
}

__device__ __forceinline__ void d_ir_finalize(DevState* st, const Reductions& red) {
  (void)ir_finalize_here(st, red, true);
}


}  // namespace fdd
