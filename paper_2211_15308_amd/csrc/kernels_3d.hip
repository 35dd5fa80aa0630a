// The 3D solver's kernels (unit cube, Kuhn tetrahedra, Gamma the face z = 1), FP64, for gfx950.
//
// Interior block: on the uniform Kuhn mesh the P1 stiffness of an interior node is h times the
// 7-point stencil (6, -1 x 6), so A_II = h L7 and every interior solve is a solve with L7.  It
// runs by multigrid-preconditioned CG: red-black Gauss-Seidel (red then black before the coarse
// correction, black then red after), P1 interpolation between nested Kuhn meshes (a fine node at
// 2I + d, d in {0,1}^3, takes the mean of the coarse nodes I and I + d: every such d is an edge
// direction of the Kuhn mesh), restriction = its transpose times 1/2 (the Galerkin coarse
// operator P^T L7 P is 2 L7), and a dense inverse on the coarsest grid.  Grids are stored with a
// one-cell zero border, (nf + 2)^3 cells, x fastest, so stencils need no bounds tests.
//
// Interface: A_G is the 2D 5-point stencil on the (n-1)^2 face nodes and M_G the consistent P1
// mass of the face triangles, (h^2 / 12) (6, 1 on the x, y and (1,1) diagonal neighbours).  The
// shifted systems (alpha A_G + beta M_G) y = r of the rational approximation (eq. (RA)) are
// solved all at once (one grid dimension per system) by CG preconditioned with the operator in
// which M_G is replaced by its part diagonal in the sine basis; that preconditioner is applied
// as S D S with S the orthonormal DST-I matrix, i.e. two batched dense FP64 GEMMs.
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

// Half-sweep of colour `red` ((i + j + k) even) of L7 u = f.  from_zero: the first red
// half-sweep from u = 0 (u = f / 6 on red points, 0 on black ones).
__global__ __launch_bounds__(kB3) void k3_rb(double* __restrict__ u, const double* __restrict__ f,
                                            int nf, int red, int from_zero,
                                            const int* __restrict__ stop) {
  if (stop && *stop) return;
  const size_t P = (size_t)nf + 2, PP = P * P;
  const int64_t N = (int64_t)nf * nf * nf;
  for (int64_t q = blockIdx.x * (int64_t)kB3 + threadIdx.x; q < N; q += (int64_t)gridDim.x * kB3) {
    int i, j, k;
    const size_t o = pidx(q, nf, &i, &j, &k);
    const bool is_red = ((i + j + k) & 1) == 0;
    if (from_zero) {
      u[o] = is_red ? f[o] * (1.0 / 6.0) : 0.0;
    } else if (is_red == (red != 0)) {
      u[o] = (f[o] + u[o - 1] + u[o + 1] + u[o - P] + u[o + P] + u[o - PP] + u[o + PP]) *
             (1.0 / 6.0);
    }
  }
}

// t = f - L7 u
__global__ __launch_bounds__(kB3) void k3_resid(const double* __restrict__ u,
                                               const double* __restrict__ f,
                                               double* __restrict__ t, int nf,
                                               const int* __restrict__ stop) {
  if (stop && *stop) return;
  const size_t P = (size_t)nf + 2, PP = P * P;
  const int64_t N = (int64_t)nf * nf * nf;
  for (int64_t q = blockIdx.x * (int64_t)kB3 + threadIdx.x; q < N; q += (int64_t)gridDim.x * kB3) {
    int i, j, k;
    const size_t o = pidx(q, nf, &i, &j, &k);
    t[o] = f[o] - (6.0 * u[o] - u[o - 1] - u[o + 1] - u[o - P] - u[o + P] - u[o - PP] - u[o + PP]);
  }
}

// f_c(I) = 1/2 [t(2I) + 1/2 sum over the 14 Kuhn-edge neighbours 2I +- d of t]
__global__ __launch_bounds__(kB3) void k3_restrict(const double* __restrict__ t,
                                                  double* __restrict__ fc, int nf, int nc,
                                                  const int* __restrict__ stop) {
  if (stop && *stop) return;
  const size_t P = (size_t)nf + 2, PP = P * P;
  const int64_t N = (int64_t)nc * nc * nc;
  for (int64_t q = blockIdx.x * (int64_t)kB3 + threadIdx.x; q < N; q += (int64_t)gridDim.x * kB3) {
    int I, J, K;
    const size_t oc = pidx(q, nc, &I, &J, &K);
    const size_t o = ((size_t)(2 * K) * P + (size_t)(2 * J)) * P + (size_t)(2 * I);
    // Kuhn edge directions: e1, e2, e3, e1+e2, e1+e3, e2+e3, e1+e2+e3
    const size_t d1 = 1, d2 = P, d3 = PP;
    const double s = t[o + d1] + t[o - d1] + t[o + d2] + t[o - d2] + t[o + d3] + t[o - d3] +
                     t[o + d1 + d2] + t[o - d1 - d2] + t[o + d1 + d3] + t[o - d1 - d3] +
                     t[o + d2 + d3] + t[o - d2 - d3] + t[o + d1 + d2 + d3] + t[o - d1 - d2 - d3];
    fc[oc] = 0.5 * (t[o] + 0.5 * s);
  }
}

// u += P e_c
__global__ __launch_bounds__(kB3) void k3_prolong(const double* __restrict__ ec,
                                                 double* __restrict__ u, int nf, int nc,
                                                 const int* __restrict__ stop) {
  if (stop && *stop) return;
  const size_t Pc = (size_t)nc + 2;
  const int64_t N = (int64_t)nf * nf * nf;
  for (int64_t q = blockIdx.x * (int64_t)kB3 + threadIdx.x; q < N; q += (int64_t)gridDim.x * kB3) {
    int i, j, k;
    const size_t o = pidx(q, nf, &i, &j, &k);
    const int I = i >> 1, J = j >> 1, K = k >> 1;
    const size_t oc = ((size_t)K * Pc + (size_t)J) * Pc + (size_t)I;
    const size_t od = ((size_t)(k & 1) * Pc + (size_t)(j & 1)) * Pc + (size_t)(i & 1);
    u[o] += od ? 0.5 * (ec[oc] + ec[oc + od]) : ec[oc];
  }
}

// coarsest grid: u = C^{-1} f with the dense inverse (nc^3 <= 64 unknowns), one block
__global__ __launch_bounds__(kB3) void k3_coarse(const double* __restrict__ f,
                                                double* __restrict__ u, int nc,
                                                const double* __restrict__ cinv,
                                                const int* __restrict__ stop) {
  if (stop && *stop) return;
  __shared__ double fp[64];
  const int np = nc * nc * nc;
  const size_t P = (size_t)nc + 2;
  auto pad = [&](int q) {
    const int i = q % nc + 1, j = (q / nc) % nc + 1, k = q / (nc * nc) + 1;
    return ((size_t)k * P + (size_t)j) * P + (size_t)i;
  };
  for (int q = threadIdx.x; q < np; q += kB3) fp[q] = f[pad(q)];
  __syncthreads();
  for (int q = threadIdx.x; q < np; q += kB3) {
    double a = 0.0;
    for (int m = 0; m < np; ++m) a += cinv[(size_t)q * np + m] * fp[m];
    u[pad(q)] = a;
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

// dot-product partials: part[block] = sum of a . b over the block's points
__global__ __launch_bounds__(kB3) void k3_dot(const double* __restrict__ a,
                                             const double* __restrict__ b, int nf,
                                             double* __restrict__ part,
                                             const int* __restrict__ stop) {
  if (stop && *stop) return;
  const int64_t N = (int64_t)nf * nf * nf;
  double s = 0.0;
  for (int64_t q = blockIdx.x * (int64_t)kB3 + threadIdx.x; q < N; q += (int64_t)gridDim.x * kB3) {
    int i, j, k;
    const size_t o = pidx(q, nf, &i, &j, &k);
    s += a[o] * b[o];
  }
  s = block_sum3(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// q = L7 p with partials of p . q
__global__ __launch_bounds__(kB3) void k3_apply(const double* __restrict__ p,
                                               double* __restrict__ qv, int nf,
                                               double* __restrict__ part,
                                               const int* __restrict__ stop) {
  if (stop && *stop) return;
  const size_t P = (size_t)nf + 2, PP = P * P;
  const int64_t N = (int64_t)nf * nf * nf;
  double s = 0.0;
  for (int64_t q = blockIdx.x * (int64_t)kB3 + threadIdx.x; q < N; q += (int64_t)gridDim.x * kB3) {
    int i, j, k;
    const size_t o = pidx(q, nf, &i, &j, &k);
    const double v = 6.0 * p[o] - p[o - 1] - p[o + 1] - p[o - P] - p[o + P] - p[o - PP] - p[o + PP];
    qv[o] = v;
    s += p[o] * v;
  }
  s = block_sum3(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// x += alpha p, r -= alpha q, partials of r . r
__global__ __launch_bounds__(kB3) void k3_update(double* __restrict__ x, double* __restrict__ r,
                                                const double* __restrict__ p,
                                                const double* __restrict__ qv, int nf,
                                                const State3* __restrict__ st,
                                                double* __restrict__ part,
                                                const int* __restrict__ stop) {
  if (stop && *stop) return;
  const double al = st->alpha;
  const int64_t N = (int64_t)nf * nf * nf;
  double s = 0.0;
  for (int64_t q = blockIdx.x * (int64_t)kB3 + threadIdx.x; q < N; q += (int64_t)gridDim.x * kB3) {
    int i, j, k;
    const size_t o = pidx(q, nf, &i, &j, &k);
    x[o] += al * p[o];
    const double rv = r[o] - al * qv[o];
    r[o] = rv;
    s += rv * rv;
  }
  s = block_sum3(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// p = z + beta p (beta = 0: p = z)
__global__ __launch_bounds__(kB3) void k3_pupdate(double* __restrict__ p,
                                                 const double* __restrict__ z, int nf,
                                                 const State3* __restrict__ st, int first,
                                                 const int* __restrict__ stop) {
  if (stop && *stop) return;
  const double be = first ? 0.0 : st->beta;
  const int64_t N = (int64_t)nf * nf * nf;
  for (int64_t q = blockIdx.x * (int64_t)kB3 + threadIdx.x; q < N; q += (int64_t)gridDim.x * kB3) {
    int i, j, k;
    const size_t o = pidx(q, nf, &i, &j, &k);
    p[o] = z[o] + be * p[o];
  }
}

// Scalar steps of the PCG, one thread block.  kind 0: start (ff = |f|^2 = rr0, rho = r.z);
// 1: alpha = rho / p.q; 2: convergence test on |r|^2; 3: beta = rho_new / rho (rho_new = r.z).
__global__ __launch_bounds__(kB3) void k3_scalars(State3* __restrict__ st, const double* part0,
                                                 const double* part1, int nb, int kind,
                                                 int* __restrict__ stop) {
  if (kind != 0 && *stop) return;
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < nb; k += kB3) {
    a += part0[k];
    if (part1) b += part1[k];
  }
  a = block_sum3(a);
  b = block_sum3(b);
  if (threadIdx.x != 0) return;
  if (kind == 0) {
    st->ff = a;
    st->rr = a;
    st->rho = b;
    st->its = 0;
    st->breakdown = 0;
    *stop = (a == 0.0) ? 1 : 0;
    if (!isfinite(a) || !isfinite(b)) {
      st->breakdown = 4;
      *stop = 1;
    }
  } else if (kind == 1) {
    const bool ok = a > 0.0 && isfinite(a);
    st->alpha = ok ? st->rho / a : 0.0;
    if (!ok) {
      st->breakdown = isfinite(a) ? 1 : 4;
      *stop = 1;
    }
  } else if (kind == 2) {
    st->rr = a;
    st->its += 1;
    if (!isfinite(a)) {
      st->breakdown = 4;
      *stop = 1;
    } else if (a <= st->tol2 * st->ff) {
      *stop = 1;
    }
  } else {
    st->beta = a / st->rho;
    st->rho = a;
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

__device__ __forceinline__ double face_at(const double* v, int nf, int i, int j) {
  return (i >= 0 && i < nf && j >= 0 && j < nf) ? v[(size_t)j * nf + i] : 0.0;
}

// y = (alpha A_G + beta M_G) x for every system (alpha, beta from the shift table; mode_mass
// != 0: the input of every system is M_G x0 of one shared vector x0 is applied instead).
__global__ __launch_bounds__(kB3) void kf_apply(const double* __restrict__ x, int x_shared,
                                               double* __restrict__ y, int nf, double h,
                                               const Shift3* __restrict__ tab,
                                               double* __restrict__ part,
                                               const int* __restrict__ done) {
  const int s = blockIdx.y;
  if (done && done[s]) return;
  const double al = tab->alpha[s], be = tab->beta[s];
  const double* xs = x + (x_shared ? 0 : (size_t)s * nf * nf);
  double* ys = y + (size_t)s * nf * nf;
  const double m0 = h * h / 12.0;
  const int64_t N = (int64_t)nf * nf;
  double acc = 0.0;
  for (int64_t q = blockIdx.x * (int64_t)kB3 + threadIdx.x; q < N; q += (int64_t)gridDim.x * kB3) {
    const int i = (int)(q % nf), j = (int)(q / nf);
    const double c = xs[q];
    const double e = face_at(xs, nf, i + 1, j), w = face_at(xs, nf, i - 1, j);
    const double no = face_at(xs, nf, i, j + 1), so = face_at(xs, nf, i, j - 1);
    const double ne = face_at(xs, nf, i + 1, j + 1), sw = face_at(xs, nf, i - 1, j - 1);
    const double a = 4.0 * c - e - w - no - so;
    const double m = m0 * (6.0 * c + e + w + no + so + ne + sw);
    const double v = al * a + be * m;
    ys[q] = v;
    acc += c * v;
  }
  acc = block_sum3(acc);
  if (part && threadIdx.x == 0) part[(size_t)s * gridDim.x + blockIdx.x] = acc;
}

// C_s = S B_s (left) or B_s S (right) for every system s, S the symmetric DST matrix (nf x nf).
// 16 x 16 output tiles, LDS-staged 16-wide panels.
__global__ __launch_bounds__(256) void kf_dst(const double* __restrict__ S,
                                             const double* __restrict__ B,
                                             double* __restrict__ C, int nf, int left,
                                             const int* __restrict__ done) {
  const int s = blockIdx.z;
  if (done && done[s]) return;
  const double* Bs = B + (size_t)s * nf * nf;
  double* Cs = C + (size_t)s * nf * nf;
  __shared__ double ta[16][17], tb[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int col = blockIdx.x * 16 + tx, row = blockIdx.y * 16 + ty;
  // rows index j (the slow direction), columns index i
  double acc = 0.0;
  for (int k0 = 0; k0 < nf; k0 += 16) {
    // left: C[row][col] = sum_k S[row][k] B[k][col];  right: C[row][col] = sum_k B[row][k] S[k][col]
    const int ka = k0 + tx, kb = k0 + ty;
    if (left) {
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
  if (row < nf && col < nf) Cs[(size_t)row * nf + col] = acc;
}

// spectral scaling of the preconditioner: z_hat(a, b) /= (alpha lambda(a, b) + beta mu(a, b))
__global__ __launch_bounds__(kB3) void kf_diag(double* __restrict__ z, int nf, int n, double h,
                                              const Shift3* __restrict__ tab,
                                              const int* __restrict__ done) {
  const int s = blockIdx.y;
  if (done && done[s]) return;
  const double al = tab->alpha[s], be = tab->beta[s];
  double* zs = z + (size_t)s * nf * nf;
  const int64_t N = (int64_t)nf * nf;
  for (int64_t q = blockIdx.x * (int64_t)kB3 + threadIdx.x; q < N; q += (int64_t)gridDim.x * kB3) {
    const int a = (int)(q % nf) + 1, b = (int)(q / nf) + 1;
    const double ca = cos(M_PI * a / n), cb = cos(M_PI * b / n);
    const double lam = 4.0 - 2.0 * ca - 2.0 * cb;
    const double mu = h * h / 12.0 * (6.0 + 2.0 * ca + 2.0 * cb + 2.0 * ca * cb);
    zs[q] /= (al * lam + be * mu);
  }
}

// per-system dot partials: part[s][block] = sum a_s . b_s
__global__ __launch_bounds__(kB3) void kf_dot(const double* __restrict__ a,
                                             const double* __restrict__ b, int nf,
                                             double* __restrict__ part,
                                             const int* __restrict__ done) {
  const int s = blockIdx.y;
  if (done && done[s]) return;
  const double* as = a + (size_t)s * nf * nf;
  const double* bs = b + (size_t)s * nf * nf;
  const int64_t N = (int64_t)nf * nf;
  double acc = 0.0;
  for (int64_t q = blockIdx.x * (int64_t)kB3 + threadIdx.x; q < N; q += (int64_t)gridDim.x * kB3)
    acc += as[q] * bs[q];
  acc = block_sum3(acc);
  if (threadIdx.x == 0) part[(size_t)s * gridDim.x + blockIdx.x] = acc;
}

// y_s += alpha_s p_s, r_s -= alpha_s q_s (kind 0); p_s = z_s + beta_s p_s (kind 1, first: p = z)
__global__ __launch_bounds__(kB3) void kf_axpy(double* __restrict__ y, double* __restrict__ r,
                                              double* __restrict__ p,
                                              const double* __restrict__ q,
                                              const double* __restrict__ z, int nf,
                                              const double* __restrict__ coef, int kind,
                                              int first, const int* __restrict__ done) {
  const int s = blockIdx.y;
  if (done && done[s]) return;
  const size_t off = (size_t)s * nf * nf;
  const int64_t N = (int64_t)nf * nf;
  const double c = (kind == 1 && first) ? 0.0 : coef[s];
  for (int64_t t = blockIdx.x * (int64_t)kB3 + threadIdx.x; t < N; t += (int64_t)gridDim.x * kB3) {
    if (kind == 0) {
      y[off + t] += c * p[off + t];
      r[off + t] -= c * q[off + t];
    } else {
      p[off + t] = z[off + t] + c * p[off + t];
    }
  }
}

// Per-system CG scalars, one block per system.  kind 0: start (rr0 = r.r, rho = r.z);
// 1: alpha = rho / p.q; 2: convergence test on r.r; 3: beta = rho_new / rho (rho_new = r.z).
__global__ __launch_bounds__(kB3) void kf_scalars(FaceCG* __restrict__ cg, const double* part0,
                                                 const double* part1, int nb, int kind,
                                                 int* __restrict__ done, double tol2) {
  const int s = blockIdx.x;
  if (kind != 0 && done[s]) return;
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < nb; k += kB3) {
    a += part0[(size_t)s * nb + k];
    if (part1) b += part1[(size_t)s * nb + k];
  }
  a = block_sum3(a);
  b = block_sum3(b);
  if (threadIdx.x != 0) return;
  if (kind == 0) {
    cg->rr0[s] = a;
    cg->rho[s] = b;
    cg->its[s] = 0;
    done[s] = (a == 0.0) ? 1 : 0;
    if (!isfinite(a) || !isfinite(b)) {
      cg->bad[s] = 1;
      done[s] = 1;
    }
  } else if (kind == 1) {
    const bool ok = a > 0.0 && isfinite(a);
    cg->alpha[s] = ok ? cg->rho[s] / a : 0.0;
    if (!ok) {
      cg->bad[s] = 1;
      done[s] = 1;
    }
  } else if (kind == 2) {
    cg->its[s] += 1;
    if (!isfinite(a)) {
      cg->bad[s] = 1;
      done[s] = 1;
    } else if (a <= tol2 * cg->rr0[s]) {
      done[s] = 1;
    }
  } else {
    cg->beta[s] = a / cg->rho[s];
    cg->rho[s] = a;
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
    double v = 0.0;
    for (int s = 0; s < m; ++s) v += tab->coef[s] * ys[(size_t)s * N + q];
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
                                                    double a) {
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
                                                   int accumulate, int64_t N) {
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
__global__ __launch_bounds__(kB3) void kf_vdot(const double* __restrict__ a,
                                              const double* __restrict__ b, int64_t N,
                                              double* __restrict__ part) {
  double acc = 0.0;
  for (int64_t q = blockIdx.x * (int64_t)kB3 + threadIdx.x; q < N; q += (int64_t)gridDim.x * kB3)
    acc += a[q] * b[q];
  acc = block_sum3(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// dst_s = src (mass = 0), M src (mass = 1) or 0 (src = null), for every system s
__global__ __launch_bounds__(kB3) void kf_bcast(const double* __restrict__ src,
                                               double* __restrict__ dst, int nf, double h,
                                               int mass) {
  const int s = blockIdx.y;
  const int64_t N = (int64_t)nf * nf;
  const double m0 = h * h / 12.0;
  for (int64_t q = blockIdx.x * (int64_t)kB3 + threadIdx.x; q < N; q += (int64_t)gridDim.x * kB3) {
    double v = 0.0;
    if (src) {
      if (mass) {
        const int i = (int)(q % nf), j = (int)(q / nf);
        v = m0 * (6.0 * src[q] + face_at(src, nf, i + 1, j) + face_at(src, nf, i - 1, j) +
                  face_at(src, nf, i, j + 1) + face_at(src, nf, i, j - 1) +
                  face_at(src, nf, i + 1, j + 1) + face_at(src, nf, i - 1, j - 1));
      } else {
        v = src[q];
      }
    }
    dst[(size_t)s * N + q] = v;
  }
}

// ---- launchers -------------------------------------------------------------------------------

static inline int grid_for(int64_t N, int cap = kPart3) {
  const int64_t g = (N + kB3 - 1) / kB3;
  return (int)(g < cap ? (g < 1 ? 1 : g) : cap);
}

void k3_launch_rb(hipStream_t s, double* u, const double* f, int nf, int red, int from_zero,
                  const int* stop) {
  hipLaunchKernelGGL(k3_rb, dim3(grid_for((int64_t)nf * nf * nf, 4096)), dim3(kB3), 0, s, u, f, nf,
                     red, from_zero, stop);
}
void k3_launch_resid(hipStream_t s, const double* u, const double* f, double* t, int nf,
                     const int* stop) {
  hipLaunchKernelGGL(k3_resid, dim3(grid_for((int64_t)nf * nf * nf, 4096)), dim3(kB3), 0, s, u, f,
                     t, nf, stop);
}
void k3_launch_restrict(hipStream_t s, const double* t, double* fc, int nf, int nc,
                        const int* stop) {
  hipLaunchKernelGGL(k3_restrict, dim3(grid_for((int64_t)nc * nc * nc, 4096)), dim3(kB3), 0, s, t,
                     fc, nf, nc, stop);
}
void k3_launch_prolong(hipStream_t s, const double* ec, double* u, int nf, int nc,
                       const int* stop) {
  hipLaunchKernelGGL(k3_prolong, dim3(grid_for((int64_t)nf * nf * nf, 4096)), dim3(kB3), 0, s, ec,
                     u, nf, nc, stop);
}
void k3_launch_coarse(hipStream_t s, const double* f, double* u, int nc, const double* cinv,
                      const int* stop) {
  hipLaunchKernelGGL(k3_coarse, dim3(1), dim3(kB3), 0, s, f, u, nc, cinv, stop);
}
void k3_launch_rhs(hipStream_t s, const Rhs3& rhs, double* f, int nf) {
  hipLaunchKernelGGL(k3_rhs, dim3(grid_for((int64_t)nf * nf * nf, 4096)), dim3(kB3), 0, s, rhs, f,
                     nf);
}
void k3_launch_dot(hipStream_t s, const double* a, const double* b, int nf, double* part,
                   const int* stop) {
  hipLaunchKernelGGL(k3_dot, dim3(kPart3), dim3(kB3), 0, s, a, b, nf, part, stop);
}
void k3_launch_apply(hipStream_t s, const double* p, double* q, int nf, double* part,
                     const int* stop) {
  hipLaunchKernelGGL(k3_apply, dim3(kPart3), dim3(kB3), 0, s, p, q, nf, part, stop);
}
void k3_launch_update(hipStream_t s, double* x, double* r, const double* p, const double* q,
                      int nf, const State3* st, double* part, const int* stop) {
  hipLaunchKernelGGL(k3_update, dim3(kPart3), dim3(kB3), 0, s, x, r, p, q, nf, st, part, stop);
}
void k3_launch_pupdate(hipStream_t s, double* p, const double* z, int nf, const State3* st,
                       int first, const int* stop) {
  hipLaunchKernelGGL(k3_pupdate, dim3(grid_for((int64_t)nf * nf * nf, 4096)), dim3(kB3), 0, s, p,
                     z, nf, st, first, stop);
}
void k3_launch_scalars(hipStream_t s, State3* st, const double* part0, const double* part1,
                       int kind, int* stop) {
  hipLaunchKernelGGL(k3_scalars, dim3(1), dim3(kB3), 0, s, st, part0, part1, kPart3, kind, stop);
}
void k3_launch_gather(hipStream_t s, const double* u, int nf, double* out, const double* xg) {
  hipLaunchKernelGGL(k3_gather, dim3(grid_for((int64_t)nf * nf * nf + nf * nf, 4096)), dim3(kB3),
                     0, s, u, nf, out, xg);
}
void kf_launch_apply(hipStream_t s, const double* x, int x_shared, double* y, int nf, double h,
                     int m, const Shift3* tab, double* part, const int* done) {
  hipLaunchKernelGGL(kf_apply, dim3(kPartF, m), dim3(kB3), 0, s, x, x_shared, y, nf, h, tab, part,
                     done);
}
void kf_launch_dst(hipStream_t s, const double* S, const double* B, double* C, int nf, int m,
                   int left, const int* done) {
  const dim3 g((nf + 15) / 16, (nf + 15) / 16, m);
  hipLaunchKernelGGL(kf_dst, g, dim3(256), 0, s, S, B, C, nf, left, done);
}
void kf_launch_diag(hipStream_t s, double* z, int nf, int n, double h, int m, const Shift3* tab,
                    const int* done) {
  hipLaunchKernelGGL(kf_diag, dim3(kPartF, m), dim3(kB3), 0, s, z, nf, n, h, tab, done);
}
void kf_launch_dot(hipStream_t s, const double* a, const double* b, int nf, int m, double* part,
                   const int* done) {
  hipLaunchKernelGGL(kf_dot, dim3(kPartF, m), dim3(kB3), 0, s, a, b, nf, part, done);
}
void kf_launch_axpy(hipStream_t s, double* y, double* r, double* p, const double* q,
                    const double* z, int nf, int m, const double* coef, int kind, int first,
                    const int* done) {
  hipLaunchKernelGGL(kf_axpy, dim3(kPartF, m), dim3(kB3), 0, s, y, r, p, q, z, nf, coef, kind,
                     first, done);
}
void kf_launch_scalars(hipStream_t s, FaceCG* cg, const double* part0, const double* part1, int m,
                       int kind, int* done, double tol2) {
  hipLaunchKernelGGL(kf_scalars, dim3(m), dim3(kB3), 0, s, cg, part0, part1, kPartF, kind, done,
                     tol2);
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
                          const double* z, int64_t N, double a) {
  hipLaunchKernelGGL(kf_outer_axpy, dim3(grid_for(N, 1024)), dim3(kB3), 0, s, x, r, p, y, z, N, a);
}
void k3_launch_scale_add(hipStream_t s, double* out, const double* u, double c, int accumulate,
                         int64_t n) {
  hipLaunchKernelGGL(k3_scale_add, dim3(grid_for(n, 2048)), dim3(kB3), 0, s, out, u, c,
                     accumulate, n);
}
void kf_launch_rhs_reduce(hipStream_t s, const double* bG, const double* w, int nf, double h,
                          double* g, double* xg) {
  hipLaunchKernelGGL(kf_rhs_reduce, dim3(grid_for((int64_t)nf * nf, 1024)), dim3(kB3), 0, s, bG, w,
                     nf, h, g, xg);
}
void kf_launch_bcast(hipStream_t s, const double* src, double* dst, int nf, double h, int m,
                     int mass) {
  hipLaunchKernelGGL(kf_bcast, dim3(kPartF, m), dim3(kB3), 0, s, src, dst, nf, h, mass);
}
void kf_launch_vdot(hipStream_t s, const double* a, const double* b, int64_t N, double* part) {
  hipLaunchKernelGGL(kf_vdot, dim3(kPart3), dim3(kB3), 0, s, a, b, N, part);
}

}  // namespace fdd
