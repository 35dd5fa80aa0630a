// The paper's own model problem in 2D (Sec. 3, eq. (model_problem)): K(-Delta + I) x +
// gamma (-Delta_Gamma + I)^t x = b on the unit square with Gamma the whole boundary, P1 on the
// diagonal-split mesh, every node a dof.  FP64 kernels for gfx950.
//
// Layouts: interior nodes (i, j), 1 <= i, j <= n-1, on the padded level-0 grid of the interior
// multigrid (row j-1 at (j-1) pitch, column i-1); the 4n boundary nodes as one loop vector,
// counter-clockwise from the corner (0, 0): bottom (i, 0) -> i, right (n, j) -> n + j, top (i, n)
// -> 2n + (n - i), left (0, j) -> 3n + (n - j).  Caller vectors: the (n-1)^2 interior nodes
// (i fastest), then the loop.
//
// The operator K (A_Omega + M_Omega) is applied node by node as the sum over the (up to six)
// triangles around the node of their element matrices (stiffness + mass), which gives the
// natural boundary rows at edges and corners without special cases.  A cell (a, b) holds the
// lower triangle (a,b), (a+1,b), (a+1,b+1) and the upper triangle (a,b), (a+1,b+1), (a,b+1); in
// both the right angle sits at the middle vertex, so the P1 stiffness is 1 at the right angle,
// 1/2 at the other two vertices, -1/2 between the right angle and each other vertex and 0 between
// those two; the mass is (h^2 / 24)(1 + delta).
//
// The boundary loop is a closed P1 curve: A_G = (1/h) circ(-1, 2, -1), M_G = (h/6) circ(1, 4, 1),
// L = A_G + M_G.  A shifted system (alpha A_G + beta M_G) y = r is cyclic tridiagonal; it is
// solved by the Sherman-Morrison reduction to a tridiagonal system with two right-hand sides,
// each by parallel cyclic reduction in LDS (one workgroup per system, all m + 1 systems of a
// rational table in one launch, eq. (RA)).
#include "iface_device.h"

namespace fdd {

namespace {

constexpr int kModelThreads = 256;
constexpr int kLoopMax = 4096;  // 4 n, n <= 1024

inline int mblocks(int64_t tot) {
  return (int)std::min<int64_t>((tot + kModelThreads - 1) / kModelThreads, 2048);
}

// loop index of boundary node (i, j) (one of i, j is 0 or n)
__device__ __forceinline__ int loop_index(int n, int i, int j) {
  if (j == 0 && i < n) return i;
  if (i == n && j < n) return n + j;
  if (j == n && i > 0) return 2 * n + (n - i);
  return 3 * n + (n - j);
}

// value of the FE vector at node (i, j): interior part xI (padded, may be null: zero), boundary
// part xG (loop, may be null: zero)
__device__ __forceinline__ double node_val(int n, int pitch, const double* xI, const double* xG,
                                           int i, int j) {
  if (i > 0 && i < n && j > 0 && j < n) return xI ? xI[(size_t)(j - 1) * pitch + (i - 1)] : 0.0;
  return xG ? xG[loop_index(n, i, j)] : 0.0;
}

// (A_Omega + M_Omega) x at node (i, j), summed over the triangles around it.
__device__ __forceinline__ double omega_row(int n, int pitch, double h2, const double* xI,
                                            const double* xG, int i, int j) {
  // element matrix of a right triangle with vertex order (acute, right angle, acute)
  const double ms = h2 / 24.0;
  auto tri = [&](int v, int ia, int ja, int ib, int jb, int ic, int jc) -> double {
    // v: local index (0, 1, 2) of the node in (a, b, c); b is the right angle
    const double xa = node_val(n, pitch, xI, xG, ia, ja);
    const double xb = node_val(n, pitch, xI, xG, ib, jb);
    const double xc = node_val(n, pitch, xI, xG, ic, jc);
    double s;
    if (v == 1) s = xb - 0.5 * xa - 0.5 * xc;          // right angle: 1, -1/2, -1/2
    else if (v == 0) s = 0.5 * xa - 0.5 * xb;          // acute: 1/2, -1/2, 0
    else s = 0.5 * xc - 0.5 * xb;
    const double xv = v == 0 ? xa : (v == 1 ? xb : xc);
    return s + ms * (xa + xb + xc + xv);               // mass (h^2/24)(1 + delta)
  };
  double y = 0.0;
  // lower triangles (a,b),(a+1,b),(a+1,b+1): right angle at (a+1,b); upper (a,b),(a,b+1),(a+1,b+1)
  // written in (acute, right, acute) order: ((a,b), (a,b+1), (a+1,b+1))
  // cells around (i, j): (i, j), (i-1, j), (i-1, j-1), (i, j-1)
  if (i < n && j < n) {            // cell (i, j): node is (a, b) of both triangles
    y += tri(0, i, j, i + 1, j, i + 1, j + 1);
    y += tri(0, i, j, i, j + 1, i + 1, j + 1);
  }
  if (i > 0 && j < n) {            // cell (i-1, j): node is (a+1, b) = right angle of the lower
    y += tri(1, i - 1, j, i, j, i, j + 1);
  }
  if (i > 0 && j > 0) {            // cell (i-1, j-1): node is (a+1, b+1) of both
    y += tri(2, i - 1, j - 1, i, j - 1, i, j);
    y += tri(2, i - 1, j - 1, i - 1, j, i, j);
  }
  if (i < n && j > 0) {            // cell (i, j-1): node is (a, b+1) = right angle of the upper
    y += tri(1, i, j - 1, i, j, i + 1, j);
  }
  return y;
}

// block sum of one value per thread into partials[blockIdx.x]
__device__ __forceinline__ void mblock_partial(double v, double* partials) {
  __shared__ double sw[kModelThreads / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0;
    for (int w = 0; w < kModelThreads / 64; ++w) a += sw[w];
    partials[blockIdx.x] = a;
  }
}

}  // namespace

// ---- operator kernels -----------------------------------------------------------------------

// Interior rows of scale (A_Omega + M_Omega)(xI, xG) (+ add_scale addc) into yI (padded).
__global__ __launch_bounds__(kModelThreads) void km_interior_rows(int n, int pitch, double h2,
                                                                  double scale,
                                                                  const double* __restrict__ xI,
                                                                  const double* __restrict__ xG,
                                                                  double* __restrict__ yI,
                                                                  const double* __restrict__ addc,
                                                                  double add_scale) {
  const int nf = n - 1;
  const int64_t tot = (int64_t)nf * nf;
  for (int64_t k = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; k < tot;
       k += (int64_t)blockDim.x * gridDim.x) {
    const int i = (int)(k % nf) + 1, j = (int)(k / nf) + 1;
    double v = scale * omega_row(n, pitch, h2, xI, xG, i, j);
    if (addc) v += add_scale * addc[k];
    yI[(size_t)(j - 1) * pitch + (i - 1)] = v;
  }
}

// Loop rows: yG = add + scale (A_Omega + M_Omega)(xI, xG) + gamma Hp (add, Hp may be null).
__global__ __launch_bounds__(kModelThreads) void km_loop_rows(int n, int pitch, double h2,
                                                              double scale, double gamma,
                                                              const double* __restrict__ xI,
                                                              const double* __restrict__ xG,
                                                              const double* __restrict__ Hp,
                                                              const double* __restrict__ add,
                                                              double* __restrict__ yG) {
  const int m = 4 * n;
  for (int k = threadIdx.x + blockIdx.x * blockDim.x; k < m; k += blockDim.x * gridDim.x) {
    int i, j;
    if (k < n) { i = k; j = 0; }
    else if (k < 2 * n) { i = n; j = k - n; }
    else if (k < 3 * n) { i = n - (k - 2 * n); j = n; }
    else { i = 0; j = n - (k - 3 * n); }
    double v = scale * omega_row(n, pitch, h2, xI, xG, i, j);
    if (Hp) v += gamma * Hp[k];
    if (add) v += add[k];
    yG[k] = v;
  }
}

// y = K (A_Omega + M_Omega) x + gamma T^T H x on all dofs, caller layout (x compact: interior
// (n-1)^2 then the loop); optionally the partials of ||b - y||^2 and ||b||^2.
__global__ __launch_bounds__(kModelThreads) void km_full_apply(int n, double h2, double K,
                                                               double gamma,
                                                               const double* __restrict__ x,
                                                               const double* __restrict__ Hx,
                                                               double* __restrict__ y,
                                                               const double* __restrict__ b,
                                                               double* __restrict__ partials) {
  const int nf = n - 1;
  const int64_t NI = (int64_t)nf * nf;
  const int64_t N = NI + 4 * n;
  const double* xG = x + NI;
  double e2 = 0.0, b2 = 0.0;
  for (int64_t k = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; k < N;
       k += (int64_t)blockDim.x * gridDim.x) {
    double v;
    if (k < NI) {
      const int i = (int)(k % nf) + 1, j = (int)(k / nf) + 1;
      v = K * omega_row(n, nf, h2, x, xG, i, j);  // compact interior: pitch n - 1
    } else {
      const int q = (int)(k - NI);
      int i, j;
      if (q < n) { i = q; j = 0; }
      else if (q < 2 * n) { i = n; j = q - n; }
      else if (q < 3 * n) { i = n - (q - 2 * n); j = n; }
      else { i = 0; j = n - (q - 3 * n); }
      v = K * omega_row(n, nf, h2, x, xG, i, j) + gamma * Hx[q];
    }
    if (y) y[k] = v;
    if (b) {
      const double d = b[k] - v;
      e2 += d * d;
      b2 += b[k] * b[k];
    }
  }
  if (!b) return;
  __shared__ double sw[2][kModelThreads / 64];
  for (int o = 32; o > 0; o >>= 1) {
    e2 += __shfl_down(e2, o, 64);
    b2 += __shfl_down(b2, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    sw[0][threadIdx.x >> 6] = e2;
    sw[1][threadIdx.x >> 6] = b2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, c = 0.0;
    for (int w = 0; w < kModelThreads / 64; ++w) {
      a += sw[0][w];
      c += sw[1][w];
    }
    partials[2 * blockIdx.x] = a;
    partials[2 * blockIdx.x + 1] = c;
  }
}

__global__ __launch_bounds__(kModelThreads) void km_sum2(const double* __restrict__ partials,
                                                         int nb, double* res) {
  const double a = block_sum_partials(partials, nb, 2);
  const double c = block_sum_partials(partials + 1, nb, 2);
  if (threadIdx.x == 0) {
    res[0] = a;
    res[1] = c;
  }
}

// ---- loop (interface) kernels ------------------------------------------------------------------

__device__ __forceinline__ double loop_mass(const double* v, int m, double h, int i) {
  return (h / 6.0) * (4.0 * v[i] + v[(i + m - 1) % m] + v[(i + 1) % m]);
}
__device__ __forceinline__ double loop_stiff(const double* v, int m, double h, int i) {
  return (2.0 * v[i] - v[(i + m - 1) % m] - v[(i + 1) % m]) / h;
}

// Block k solves (alpha_k A_G + beta_k M_G) y = rhs on the loop (rhs = in, or M_G in in operator
// mode) and stores coef_k y in scratch[k].
__global__ __launch_bounds__(kIfaceThreads) void km_loop_solve(int m, double h, ShiftTable tab,
                                                               int mode,
                                                               const double* __restrict__ in,
                                                               double* __restrict__ scratch) {
  __shared__ double sa[kLoopMax], sd[kLoopMax], su[kLoopMax];
  const int k = blockIdx.x;
  const double al = tab.alpha[k], be = tab.beta[k], ck = tab.coef[k];
  const double off = -al / h + be * h / 6.0;
  const double dia = 2.0 * al / h + 4.0 * be * h / 6.0;
  // Sherman-Morrison: C = T' + u v^T with u = (g, 0, ..., 0, off), v = (1, 0, ..., 0, off / g),
  // g = -dia, so T' is tridiagonal with diagonal (dia - g, dia, ..., dia, dia - off^2 / g);
  // C x = r  =>  x = y - (v.y / (1 + v.z)) z,  T' y = r,  T' z = u.
  const double g = -dia;
  // rows normalized by their diagonal: x_i + a_i x_{i-1} + a_i x_{i+1} = d_i (off-diagonals equal);
  // a thread's right-hand-side loads (nodes tid + 1024 t and their loop neighbours) are all
  // issued before the first is used
  constexpr int R = kLoopMax / kIfaceThreads;
  double vc[R], vl[R], vr[R];
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int i = threadIdx.x + t * kIfaceThreads;
    const int ic = i < m ? i : 0;
    vc[t] = in[ic];
    vl[t] = in[(ic + m - 1) % m];
    vr[t] = in[(ic + 1) % m];
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int i = threadIdx.x + t * kIfaceThreads;
    if (i >= m) continue;
    const double di = (i == 0) ? dia - g : (i == m - 1 ? dia - off * off / g : dia);
    // (the operator-mode right-hand side is M_G in, as loop_mass forms it)
    const double rhs = (mode == kIfaceOperator) ? (h / 6.0) * (4.0 * vc[t] + vl[t] + vr[t]) : vc[t];
    const double u = (i == 0) ? g : (i == m - 1 ? off : 0.0);
    sa[i] = off / di;
    sd[i] = rhs / di;
    su[i] = u / di;
  }
  __syncthreads();
  // parallel cyclic reduction with two right-hand sides (rows beyond the ends are zero)
  // lower and upper coefficients of a row evolve separately once rows are combined
  __shared__ double sc[kLoopMax];
  for (int i = threadIdx.x; i < m; i += blockDim.x) sc[i] = sa[i];
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    if (i == 0) sa[i] = 0.0;        // no x_{-1}
    if (i == m - 1) sc[i] = 0.0;    // no x_m
  }
  __syncthreads();
  for (int s = 1; s < m; s <<= 1) {
    double na[R], nc[R], nd[R], nu[R];
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int i = threadIdx.x + t * kIfaceThreads;
      if (i >= m) continue;
      const double ai = sa[i], ci = sc[i], di = sd[i], ui = su[i];
      const bool lo = i - s >= 0, hi = i + s < m;
      const double am = lo ? sa[i - s] : 0.0, cm = lo ? sc[i - s] : 0.0;
      const double dm = lo ? sd[i - s] : 0.0, um = lo ? su[i - s] : 0.0;
      const double ap = hi ? sa[i + s] : 0.0, cp = hi ? sc[i + s] : 0.0;
      const double dp = hi ? sd[i + s] : 0.0, up = hi ? su[i + s] : 0.0;
      const double den = 1.0 / (1.0 - ai * cm - ci * ap);
      na[t] = -ai * am * den;
      nc[t] = -ci * cp * den;
      nd[t] = (di - ai * dm - ci * dp) * den;
      nu[t] = (ui - ai * um - ci * up) * den;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int i = threadIdx.x + t * kIfaceThreads;
      if (i >= m) continue;
      sa[i] = na[t];
      sc[i] = nc[t];
      sd[i] = nd[t];
      su[i] = nu[t];
    }
    __syncthreads();
  }
  // y = sd, z = su; x = y - (v.y / (1 + v.z)) z with v = (1, 0, ..., 0, off / g)
  const double vy = sd[0] + (off / g) * sd[m - 1];
  const double vz = su[0] + (off / g) * su[m - 1];
  const double f = vy / (1.0 + vz);
  for (int i = threadIdx.x; i < m; i += blockDim.x) scratch[(size_t)k * m + i] = ck * (sd[i] - f * su[i]);
}

// Weighted sum of the systems (in system order) and the epilogue:
//   precond mode:  out = sum
//   operator mode: out = dL L in + d0 M in + M sum   (the RA realization of L^t)
constexpr int kCombineThreads = 256;
__global__ __launch_bounds__(kCombineThreads) void km_loop_combine(int m, double h, int nsys,
                                                                   double d0, double dL, int mode,
                                                                   const double* __restrict__ in,
                                                                   const double* __restrict__ scratch,
                                                                   double* __restrict__ out) {
  // the block's nodes i0 .. i0 + 255 and one more on each side of the loop (cyclic): the
  // operator epilogue applies M_G to the sum; each sum adds the systems in order, eight loads in
  // flight at a time
  __shared__ double s[kCombineThreads + 2];
  const int i0 = blockIdx.x * kCombineThreads;
  for (int c = threadIdx.x; c < kCombineThreads + 2; c += kCombineThreads) {
    const int i = ((i0 - 1 + c) % m + m) % m;
    constexpr int U = 8;
    double v = 0.0;
    for (int k0 = 0; k0 < nsys; k0 += U) {
      double a[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = k0 + u < nsys ? k0 + u : k0;
        a[u] = scratch[(size_t)k * m + i];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (k0 + u < nsys) v += a[u];
    }
    s[c] = v;
  }
  __syncthreads();
  const int i = i0 + threadIdx.x;
  if (i >= m) return;
  if (mode == kIfaceOperator) {
    const double Lin = loop_stiff(in, m, h, i) + loop_mass(in, m, h, i);
    const int c = threadIdx.x + 1;  // node i in s (its neighbours at c - 1 and c + 1)
    const double Ms = (h / 6.0) * (4.0 * s[c] + s[c - 1] + s[c + 1]);
    out[i] = dL * Lin + d0 * loop_mass(in, m, h, i) + Ms;
  } else {
    out[i] = s[threadIdx.x + 1];
  }
}

// ---- interior PCG (A_II = A_Omega + M_Omega on the interior nodes, Dirichlet-zero boundary) ---

// rz = r . Z zs from the partials of km_ii_rz (every block sums them in the same order), beta =
// rz / rho (first: 0); p = Z zs + beta p' (formed where read; first: p = Z zs), q = B_II p,
// partials of p.q into pq_partials.  rho is read here by every block, so block 0 parks rz in
// cg_gam[0] and km_ii_update moves it to rho.
template <typename VT>
__global__ __launch_bounds__(kModelThreads) void km_ii_apply(int n, int pitch, double h2,
                                                             const VT* __restrict__ Z, double zs,
                                                             const double* __restrict__ po,
                                                             double* __restrict__ pn,
                                                             double* __restrict__ q, DevState* st,
                                                             int first,
                                                             const double* __restrict__ rz_partials,
                                                             int nb_rz,
                                                             double* __restrict__ pq_partials) {
  if (st->inner_done) return;
  const double rz = block_sum_partials(rz_partials, nb_rz, 1);
  if (!(rz > 0.0) || !isfinite(rz)) {  // r = 0 ends the solve; otherwise M is not SPD
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      if (rz != 0.0) st->breakdown |= isfinite(rz) ? 1 : 4;
      st->inner_done = 1;
    }
    return;
  }
  const double beta = first ? 0.0 : rz / st->rho;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->cg_gam[0] = rz;
    st->cg_gam[1] = beta;
  }
  const int nf = n - 1;
  const double c4 = 4.0 + h2 / 2.0, c1 = -1.0 + h2 / 12.0, cd = h2 / 12.0;
  // the seven points c, w, e, s, n, ne, sw: offsets (di, dj) from the node
  constexpr int kDi[7] = {0, -1, 1, 0, 0, 1, -1}, kDj[7] = {0, 0, 0, -1, 1, 1, -1};
  double acc = 0.0;
  const int64_t tot = (int64_t)nf * nf;
  for (int64_t k = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; k < tot;
       k += (int64_t)blockDim.x * gridDim.x) {
    const int i = (int)(k % nf), j = (int)(k / nf);
    const size_t o = (size_t)j * pitch + i;
    // p at the seven points (zero outside the interior), every load issued before the first use:
    // a point outside reads the node's own entries and is zeroed
    bool in[7];
    size_t oo[7];
    VT zr[7];
    double pr[7];
#pragma unroll
    for (int a = 0; a < 7; ++a) {
      const int ii = i + kDi[a], jj = j + kDj[a];
      in[a] = ii >= 0 && ii < nf && jj >= 0 && jj < nf;
      oo[a] = in[a] ? (size_t)jj * pitch + ii : o;
    }
#pragma unroll
    for (int a = 0; a < 7; ++a) {
      zr[a] = Z[oo[a]];
      pr[a] = first ? 0.0 : po[oo[a]];
    }
    __builtin_amdgcn_sched_barrier(0);
    double P[7];
#pragma unroll
    for (int a = 0; a < 7; ++a) {
      const double z = (double)zr[a] * zs;
      P[a] = in[a] ? (first ? z : z + beta * pr[a]) : 0.0;
    }
    const double c = P[0];
    const double v = c4 * c + c1 * (P[1] + P[2] + P[3] + P[4]) + cd * (P[5] + P[6]);
    pn[o] = c;
    q[o] = v;
    acc += c * v;
  }
  mblock_partial(acc, pq_partials);
}

// p.q from the partials of km_ii_apply (every block, same order), alpha = rz / p.q;
// x += alpha p, r -= alpha q, vr = r (V-cycle input), partials of ||r||^2.  Block 0 records
// p.q, alpha and rho = rz.
template <typename VT>
__global__ __launch_bounds__(kModelThreads) void km_ii_update(int nf, int pitch,
                                                              double* __restrict__ x,
                                                              double* __restrict__ r,
                                                              const double* __restrict__ p,
                                                              const double* __restrict__ q,
                                                              VT* __restrict__ vr, DevState* st,
                                                              const double* __restrict__ pq_partials,
                                                              int nb_pq,
                                                              double* __restrict__ partials) {
  if (st->inner_done) return;
  const double pq = block_sum_partials(pq_partials, nb_pq, 1);
  const double rz = st->cg_gam[0];
  const bool ok = pq > 0.0 && isfinite(pq);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->pq = pq;
    st->cg_alpha[0] = ok ? rz / pq : 0.0;
    st->rho = rz;
    if (!ok) {
      st->breakdown |= isfinite(pq) ? 1 : 4;
      st->inner_done = 1;
    }
  }
  if (!ok) return;
  const double al = rz / pq;
  double acc = 0.0;
  const int64_t tot = (int64_t)nf * nf;
  for (int64_t k = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; k < tot;
       k += (int64_t)blockDim.x * gridDim.x) {
    const size_t o = (size_t)(k / nf) * pitch + (size_t)(k % nf);
    x[o] += al * p[o];
    const double rv = r[o] - al * q[o];
    r[o] = rv;
    vr[o] = (VT)rv;
    acc += rv * rv;
  }
  mblock_partial(acc, partials);
}

// start of an interior solve: x = 0, r = f (padded), vr = r, partials of ||f||^2
template <typename VT>
__global__ __launch_bounds__(kModelThreads) void km_ii_start(int nf, int pitch,
                                                             const double* __restrict__ f,
                                                             double* __restrict__ x,
                                                             double* __restrict__ r,
                                                             VT* __restrict__ vr, DevState* st,
                                                             double* __restrict__ partials,
                                                             double tol2) {
  double acc = 0.0;
  const int64_t tot = (int64_t)nf * nf;
  for (int64_t k = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; k < tot;
       k += (int64_t)blockDim.x * gridDim.x) {
    const size_t o = (size_t)(k / nf) * pitch + (size_t)(k % nf);
    const double v = f[o];
    x[o] = 0.0;
    r[o] = v;
    vr[o] = (VT)v;
    acc += v * v;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->inner_done = 0;
    st->solve_done = 0;
    st->breakdown &= ~1;
    st->inner_its = 0;
    st->tol2 = tol2;
  }
  mblock_partial(acc, partials);
}

// ||r||^2 from partials: the stop test ||r|| <= tol ||f|| (start: ||f||^2 is recorded; a zero
// right-hand side ends the solve at once)
__global__ __launch_bounds__(kModelThreads) void km_ii_check(DevState* st,
                                                            const double* __restrict__ partials,
                                                            int nb, int start) {
  if (st->inner_done) return;
  const double rr = block_sum_partials(partials, nb, 1);
  if (threadIdx.x != 0) return;
  if (start) st->ff = rr;
  st->rr = rr;
  if (!start) st->inner_its += 1;
  if (!isfinite(rr)) {
    st->breakdown |= 4;
    st->inner_done = 1;
  } else if (rr <= st->tol2 * st->ff) {
    st->inner_done = 1;  // the V-cycles and updates enqueued after this return at once
  }
}

// partials of rz = r . Z zs (summed by the next km_ii_apply)
template <typename VT>
__global__ __launch_bounds__(kModelThreads) void km_ii_rz(int nf, int pitch,
                                                          const double* __restrict__ r,
                                                          const VT* __restrict__ Z, double zs,
                                                          const DevState* st,
                                                          double* __restrict__ partials) {
  if (st->inner_done) return;
  double acc = 0.0;
  const int64_t tot = (int64_t)nf * nf;
  for (int64_t k = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; k < tot;
       k += (int64_t)blockDim.x * gridDim.x) {
    const size_t o = (size_t)(k / nf) * pitch + (size_t)(k % nf);
    acc += r[o] * ((double)Z[o] * zs);
  }
  mblock_partial(acc, partials);
}

// ---- outer PCG on the loop (one block each) ---------------------------------------------------

__device__ __forceinline__ double mblock_sum(double v) {
  __shared__ double sw[kIfaceThreads / 64];
  __shared__ double tot;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) a += sw[w];
    tot = a;
  }
  __syncthreads();
  return tot;
}

// alpha = rho / p.y, x += alpha p, r -= alpha y
__global__ __launch_bounds__(kIfaceThreads) void km_outer_update(int m, const double* __restrict__ p,
                                                                 const double* __restrict__ y,
                                                                 double* __restrict__ x,
                                                                 double* __restrict__ r,
                                                                 DevState* st) {
  if (st->outer_done) return;
  double acc = 0.0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) acc += p[i] * y[i];
  const double pq = mblock_sum(acc);
  const bool ok = pq > 0.0 && isfinite(pq);
  const double al = ok ? st->o_rho[0] / pq : 0.0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    x[i] += al * p[i];
    r[i] -= al * y[i];
  }
  if (threadIdx.x == 0) {
    st->o_pq = pq;
    st->o_alpha = al;
    if (!ok) {
      st->breakdown |= isfinite(pq) ? 2 : 4;
      st->outer_done = 1;
    }
  }
}

// rho' = r.z, beta = rho' / rho, p' = z + beta p, stop when rho' <= rtol2 rho_0 (first: rho_0)
__global__ __launch_bounds__(kIfaceThreads) void km_outer_direction(
    int m, const double* __restrict__ r, const double* __restrict__ z,
    const double* __restrict__ po, double* __restrict__ pn, DevState* st, int first,
    double rtol2) {
  if (!first && st->outer_done) return;  // (the first call starts a new outer PCG)
  double acc = 0.0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) acc += r[i] * z[i];
  const double rz = mblock_sum(acc);
  const double beta = first ? 0.0 : rz / st->o_rho[0];
  for (int i = threadIdx.x; i < m; i += blockDim.x) pn[i] = first ? z[i] : z[i] + beta * po[i];
  if (threadIdx.x == 0) {
    if (first) {
      st->o_rho0 = rz;
      st->breakdown = 0;
      st->outer_done = 0;
    }
    st->o_rho[0] = rz;
    st->o_beta = beta;
    if (!isfinite(rz)) st->breakdown |= 4;
    else if (rz < 0.0) st->breakdown |= 2;
    // (rz_0 = 0: a zero right-hand side, the solve is over at once)
    if (!(rz > rtol2 * (first ? rz : st->o_rho0)) || st->breakdown) st->outer_done = 1;
  }
}

// ---- launchers --------------------------------------------------------------------------------

void launch_model_outer_update(hipStream_t s, int m, const double* p, const double* y, double* x,
                               double* r, DevState* st) {
  hipLaunchKernelGGL(km_outer_update, dim3(1), dim3(kIfaceThreads), 0, s, m, p, y, x, r, st);
}

void launch_model_outer_direction(hipStream_t s, int m, const double* r, const double* z,
                                  const double* p_old, double* p_new, DevState* st, int first,
                                  double rtol2) {
  hipLaunchKernelGGL(km_outer_direction, dim3(1), dim3(kIfaceThreads), 0, s, m, r, z, p_old, p_new,
                     st, first, rtol2);
}

void launch_model_interior_rows(hipStream_t s, int n, int pitch, double scale, const double* xI,
                                const double* xG, double* yI, const double* addc,
                                double add_scale) {
  const double h = 1.0 / n;
  hipLaunchKernelGGL(km_interior_rows, dim3(mblocks((int64_t)(n - 1) * (n - 1))),
                     dim3(kModelThreads), 0, s, n, pitch, h * h, scale, xI, xG, yI, addc,
                     add_scale);
}

void launch_model_loop_rows(hipStream_t s, int n, int pitch, double scale, double gamma,
                            const double* xI, const double* xG, const double* Hp,
                            const double* add, double* yG) {
  const double h = 1.0 / n;
  hipLaunchKernelGGL(km_loop_rows, dim3(mblocks(4 * n)), dim3(kModelThreads), 0, s, n, pitch,
                     h * h, scale, gamma, xI, xG, Hp, add, yG);
}

void launch_model_full_apply(hipStream_t s, int n, double K, double gamma, const double* x,
                             const double* Hx, double* y, const double* b, double* partials,
                             double* res) {
  const double h = 1.0 / n;
  const int nb = mblocks((int64_t)(n - 1) * (n - 1) + 4 * n);
  hipLaunchKernelGGL(km_full_apply, dim3(nb), dim3(kModelThreads), 0, s, n, h * h, K, gamma, x,
                     Hx, y, b, partials);
  if (b) hipLaunchKernelGGL(km_sum2, dim3(1), dim3(kModelThreads), 0, s, (const double*)partials,
                            nb, res);
}

void launch_model_loop_batch(hipStream_t s, int n, const ShiftTable& tab, int mode,
                             const double* in, double* out, double* scratch) {
  const int m = 4 * n;
  const double h = 1.0 / n;
  hipLaunchKernelGGL(km_loop_solve, dim3(tab.m), dim3(kIfaceThreads), 0, s, m, h, tab, mode, in,
                     scratch);
  hipLaunchKernelGGL(km_loop_combine, dim3((m + kCombineThreads - 1) / kCombineThreads),
                     dim3(kCombineThreads), 0, s, m, h, tab.m, tab.d0, tab.dL, mode, in,
                     (const double*)scratch, out);
}

template <typename VT>
void launch_model_ii_start(hipStream_t s, int nf, int pitch, const double* f, double* x,
                           double* r, VT* vr, DevState* st, double* partials, double tol2) {
  const int nb = mblocks((int64_t)nf * nf);
  hipLaunchKernelGGL(km_ii_start<VT>, dim3(nb), dim3(kModelThreads), 0, s, nf, pitch, f, x, r, vr,
                     st, partials, tol2);
  hipLaunchKernelGGL(km_ii_check, dim3(1), dim3(kModelThreads), 0, s, st,
                     (const double*)partials, nb, 1);
}

template <typename VT>
void launch_model_ii_rz(hipStream_t s, int nf, int pitch, const double* r, const VT* Z, double zs,
                        DevState* st, double* partials) {
  const int nb = mblocks((int64_t)nf * nf);
  hipLaunchKernelGGL(km_ii_rz<VT>, dim3(nb), dim3(kModelThreads), 0, s, nf, pitch, r, Z, zs,
                     (const DevState*)st, partials);
}

// The r.z and ||r||^2 partials sit in partials[0, 2048), the p.q partials in [4096, 6144): the
// kernel that sums one set writes the other, so no block overwrites a partial another block of
// the same launch is still reading.
template <typename VT>
void launch_model_ii_step(hipStream_t s, int n, int pitch, const VT* Z, double zs, double* p_old,
                          double* p_new, double* q, double* x, double* r, VT* vr, DevState* st,
                          double* partials, int first) {
  const int nf = n - 1;
  const int nb = mblocks((int64_t)nf * nf);
  const double h = 1.0 / n;
  double* pq_partials = partials + 4096;
  hipLaunchKernelGGL(km_ii_apply<VT>, dim3(nb), dim3(kModelThreads), 0, s, n, pitch, h * h, Z, zs,
                     (const double*)p_old, p_new, q, st, first, (const double*)partials, nb,
                     pq_partials);
  hipLaunchKernelGGL(km_ii_update<VT>, dim3(nb), dim3(kModelThreads), 0, s, nf, pitch, x, r,
                     (const double*)p_new, (const double*)q, vr, st, (const double*)pq_partials,
                     nb, partials);
  hipLaunchKernelGGL(km_ii_check, dim3(1), dim3(kModelThreads), 0, s, st,
                     (const double*)partials, nb, 0);
}

#define FDD_MODEL_INST(VT)                                                                        \
  template void launch_model_ii_start<VT>(hipStream_t, int, int, const double*, double*, double*, \
                                          VT*, DevState*, double*, double);                       \
  template void launch_model_ii_rz<VT>(hipStream_t, int, int, const double*, const VT*, double,   \
                                       DevState*, double*);                                       \
  template void launch_model_ii_step<VT>(hipStream_t, int, int, const VT*, double, double*,       \
                                         double*, double*, double*, double*, VT*, DevState*,      \
                                         double*, int);
FDD_MODEL_INST(float)
FDD_MODEL_INST(double)
#undef FDD_MODEL_INST

}  // namespace fdd
