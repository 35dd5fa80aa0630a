// Rational approximation tables for the paper's eq. (RA), built on the host in FP64.
//
// The solution operator c0 M^{-1} + sum_k c_k (L + p_k M)^{-1} equals U f_RA(Lambda) U^T with
// f_RA(lam) = c0 + sum_k c_k / (lam + p_k)  (Sec. 2, footnote with eq. (RA)), so a table is a
// scalar rational approximation of f on the interval [lam_lo, lam_hi] that holds the discrete
// spectrum of (L_h, M_h).  Construction:
//   1. AAA (adaptive Antoulas-Anderson; Nakatsukasa, Sete, Trefethen 2018) with relative
//      weights on log-spaced samples of lam / lam_hi: greedy support points, barycentric weights
//      from the smallest right singular vector of the row-weighted Loewner matrix.
//   2. Poles: zeros of the barycentric denominator sum_j w_j / (z - z_j).  They are the
//      eigenvalues of the oblique projection (I - 1 w^T / w^T 1) diag(z) restricted to the
//      complement of w (an (m-1) x (m-1) matrix), computed by shifted Hessenberg QR.
//   3. Only real poles on the negative axis are kept (shifts p_k = -pole * lam_hi >= 0, so each
//      L + p_k M stays SPD); the residues c0, c_k are refit by least squares with weights 1/|f|.
//   4. The kept poles are relocated by a few vector-fitting iterations, then refit.
//   5. For the preconditioner symbol, the table is first derived exactly from the table of
//      lam^{-1/2} (see derive_precond); direct AAA on the symbol is the alternative.
//   6. Accepted when the max relative error over the samples and the check points (the exact
//      eigenvalues in 2D) is within 10 x tol; otherwise resampled more densely.
// The linear algebra (Householder QR, one-sided Jacobi SVD, complex shifted Hessenberg QR) is
// written here because the product links no LAPACK.
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "fdd_internal.h"

namespace fdd {

using cplx = std::complex<double>;

// ---- Householder QR: A (rows x cols, column-major) -> R (cols x cols, column-major) ----------
// Also applies Q^T to the extra right-hand side b (length rows) when given.
static void householder_r(int rows, int cols, std::vector<double>& A, std::vector<double>& R,
                          std::vector<double>* b) {
  std::vector<double> v(rows);
  for (int j = 0; j < cols; ++j) {
    double nrm = 0.0;
    for (int i = j; i < rows; ++i) nrm += A[(size_t)j * rows + i] * A[(size_t)j * rows + i];
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) continue;
    const double a0 = A[(size_t)j * rows + j];
    const double alpha = a0 >= 0 ? -nrm : nrm;
    double vn = 0.0;
    for (int i = j; i < rows; ++i) {
      v[i] = A[(size_t)j * rows + i];
      if (i == j) v[i] -= alpha;
      vn += v[i] * v[i];
    }
    if (vn == 0.0) continue;
    for (int c = j; c < cols; ++c) {
      double s = 0.0;
      for (int i = j; i < rows; ++i) s += v[i] * A[(size_t)c * rows + i];
      s = 2.0 * s / vn;
      for (int i = j; i < rows; ++i) A[(size_t)c * rows + i] -= s * v[i];
    }
    if (b) {
      double s = 0.0;
      for (int i = j; i < rows; ++i) s += v[i] * (*b)[i];
      s = 2.0 * s / vn;
      for (int i = j; i < rows; ++i) (*b)[i] -= s * v[i];
    }
  }
  R.assign((size_t)cols * cols, 0.0);
  for (int c = 0; c < cols; ++c)
    for (int i = 0; i <= c && i < rows; ++i) R[(size_t)c * cols + i] = A[(size_t)c * rows + i];
}

// ---- one-sided Jacobi: columns of B (k x k, column-major) made orthogonal by rotations that
// are accumulated in V; afterwards B = U diag(sigma), so the input equals B V^T. -------------
static void jacobi_orthogonalize(int k, std::vector<double>& B, std::vector<double>& V) {
  V.assign((size_t)k * k, 0.0);
  for (int i = 0; i < k; ++i) V[(size_t)i * k + i] = 1.0;
  const double eps = 1e-15;
  for (int sweep = 0; sweep < 80; ++sweep) {
    bool any = false;
    for (int p = 0; p < k - 1; ++p) {
      for (int q = p + 1; q < k; ++q) {
        double a = 0.0, b = 0.0, g = 0.0;
        double* cp = &B[(size_t)p * k];
        double* cq = &B[(size_t)q * k];
        for (int i = 0; i < k; ++i) {
          a += cp[i] * cp[i];
          b += cq[i] * cq[i];
          g += cp[i] * cq[i];
        }
        if (g == 0.0 || std::fabs(g) <= eps * std::sqrt(a * b)) continue;
        any = true;
        const double zeta = (b - a) / (2.0 * g);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
        for (int i = 0; i < k; ++i) {
          const double x = cp[i], y = cq[i];
          cp[i] = c * x - s * y;
          cq[i] = s * x + c * y;
        }
        double* vp = &V[(size_t)p * k];
        double* vq = &V[(size_t)q * k];
        for (int i = 0; i < k; ++i) {
          const double x = vp[i], y = vq[i];
          vp[i] = c * x - s * y;
          vq[i] = s * x + c * y;
        }
      }
    }
    if (!any) break;
  }
}

int svd_min_right(int rows, int cols, const double* A, double* v, double* smin, double* smax) {
  if (rows < 1 || cols < 1) return -1;
  std::vector<double> M(A, A + (size_t)rows * cols), R, V;
  if (rows >= cols) {
    householder_r(rows, cols, M, R, nullptr);
  } else {
    // pad with zero rows: the right singular vectors are unchanged
    R.assign((size_t)cols * cols, 0.0);
    for (int c = 0; c < cols; ++c)
      for (int i = 0; i < rows; ++i) R[(size_t)c * cols + i] = M[(size_t)c * rows + i];
  }
  jacobi_orthogonalize(cols, R, V);
  int jmin = 0;
  double lo = INFINITY, hi = 0.0;
  for (int j = 0; j < cols; ++j) {
    double s = 0.0;
    for (int i = 0; i < cols; ++i) s += R[(size_t)j * cols + i] * R[(size_t)j * cols + i];
    s = std::sqrt(s);
    if (s < lo) {
      lo = s;
      jmin = j;
    }
    hi = std::max(hi, s);
  }
  for (int i = 0; i < cols; ++i) v[i] = V[(size_t)jmin * cols + i];
  if (smin) *smin = lo;
  if (smax) *smax = hi;
  return 0;
}

// ---- eigenvalues of a real square matrix: Householder reduction to Hessenberg form, then
// single-shift QR in complex arithmetic with Wilkinson shifts and deflation. ----------------
int eig_real_general(int n, const double* A, double* wr, double* wi) {
  if (n <= 0) return 0;
  std::vector<cplx> H((size_t)n * n);
  {
    std::vector<double> a(A, A + (size_t)n * n), v(n);
    for (int k = 0; k < n - 2; ++k) {
      double nrm = 0.0;
      for (int i = k + 1; i < n; ++i) nrm += a[(size_t)i * n + k] * a[(size_t)i * n + k];
      nrm = std::sqrt(nrm);
      if (nrm == 0.0) continue;
      const double x0 = a[(size_t)(k + 1) * n + k];
      const double alpha = x0 >= 0 ? -nrm : nrm;
      double vn = 0.0;
      for (int i = k + 1; i < n; ++i) {
        v[i] = a[(size_t)i * n + k] - (i == k + 1 ? alpha : 0.0);
        vn += v[i] * v[i];
      }
      if (vn == 0.0) continue;
      // left: rows k+1..n-1
      for (int c = 0; c < n; ++c) {
        double s = 0.0;
        for (int i = k + 1; i < n; ++i) s += v[i] * a[(size_t)i * n + c];
        s = 2.0 * s / vn;
        for (int i = k + 1; i < n; ++i) a[(size_t)i * n + c] -= s * v[i];
      }
      // right: columns k+1..n-1
      for (int r = 0; r < n; ++r) {
        double s = 0.0;
        for (int i = k + 1; i < n; ++i) s += a[(size_t)r * n + i] * v[i];
        s = 2.0 * s / vn;
        for (int i = k + 1; i < n; ++i) a[(size_t)r * n + i] -= s * v[i];
      }
    }
    for (int r = 0; r < n; ++r)
      for (int c = 0; c < n; ++c) H[(size_t)r * n + c] = (c + 1 >= r) ? a[(size_t)r * n + c] : 0.0;
  }
  auto h = [&](int r, int c) -> cplx& { return H[(size_t)r * n + c]; };
  const double eps = 2.220446049250313e-16;
  int hi = n - 1;
  int iter = 0, total = 0;
  std::vector<cplx> gc(n), gs(n);
  while (hi >= 0) {
    if (hi == 0) {
      wr[0] = h(0, 0).real();
      wi[0] = h(0, 0).imag();
      break;
    }
    int lo = hi;
    while (lo > 0) {
      const double sub = std::abs(h(lo, lo - 1));
      if (sub <= eps * (std::abs(h(lo, lo)) + std::abs(h(lo - 1, lo - 1)))) {
        h(lo, lo - 1) = 0.0;
        break;
      }
      --lo;
    }
    if (lo == hi) {
      wr[hi] = h(hi, hi).real();
      wi[hi] = h(hi, hi).imag();
      --hi;
      iter = 0;
      continue;
    }
    if (++total > 100 * n) return -1;
    // Wilkinson shift from the trailing 2 x 2 block of the active window
    const cplx a = h(hi - 1, hi - 1), b = h(hi - 1, hi), c = h(hi, hi - 1), d = h(hi, hi);
    const cplx tr2 = 0.5 * (a + d);
    const cplx disc = std::sqrt(0.25 * (a - d) * (a - d) + b * c);
    cplx mu = (std::abs(tr2 + disc - d) < std::abs(tr2 - disc - d)) ? tr2 + disc : tr2 - disc;
    if (iter > 0 && iter % 12 == 0) mu = d + cplx(std::abs(c), 0.5 * std::abs(c));  // exceptional
    ++iter;
    // explicit shifted QR step on rows/columns lo..hi: H - mu I = Q R, H <- R Q + mu I
    for (int k = lo; k <= hi; ++k) h(k, k) -= mu;
    for (int k = lo; k < hi; ++k) {
      const cplx x = h(k, k), y = h(k + 1, k);
      const double rr = std::sqrt(std::norm(x) + std::norm(y));
      cplx cs = 1.0, sn = 0.0;
      if (rr > 0.0) {
        cs = x / rr;
        sn = y / rr;
      }
      gc[k] = cs;
      gs[k] = sn;
      // rows k, k+1 <- [conj(cs) conj(sn); -sn cs] * rows
      for (int col = k; col <= hi; ++col) {
        const cplx u = h(k, col), w = h(k + 1, col);
        h(k, col) = std::conj(cs) * u + std::conj(sn) * w;
        h(k + 1, col) = -sn * u + cs * w;
      }
    }
    for (int k = lo; k < hi; ++k) {
      const cplx cs = gc[k], sn = gs[k];
      const int rmax = std::min(k + 2, hi);
      for (int r = lo; r <= rmax; ++r) {
        const cplx u = h(r, k), w = h(r, k + 1);
        h(r, k) = u * cs + w * sn;
        h(r, k + 1) = -u * std::conj(sn) + w * std::conj(cs);
      }
    }
    for (int k = lo; k <= hi; ++k) h(k, k) += mu;
  }
  return 0;
}

// ---- the approximated functions ---------------------------------------------------------------
// which = 0: f(lam) = 1 / (K lam^{1/2} + gamma lam^t) (the preconditioner of eq. (schur_precond)
// with s = 1/2); which = 1: lam^t (the operator's fractional power).  The Riesz map of the facet
// problems has t = -1/2.
static inline double fval(int which, double K, double gamma, double t, double lam) {
  if (t == -0.5) {
    if (which == 1) return 1.0 / std::sqrt(lam);
    const double s = std::sqrt(lam);
    return 1.0 / (K * s + gamma / s);
  }
  if (which == 1) return std::pow(lam, t);
  return 1.0 / (K * std::sqrt(lam) + gamma * std::pow(lam, t));
}

static inline double ra_value(const RaResult& r, double lam) {
  double v = r.c0;
  for (int k = 0; k < r.m; ++k) v += r.c[k] / (lam + r.p[k]);
  return v;
}

double ra_eval_rel_err(int which, double K, double gamma, const RaResult& r, const double* pts,
                       int npts, double t) {
  double e = 0.0;
  for (int i = 0; i < npts; ++i) {
    const double f = fval(which, K, gamma, t, pts[i]);
    e = std::max(e, std::fabs(f - ra_value(r, pts[i])) / std::fabs(f));
  }
  return e;
}

// ---- AAA ------------------------------------------------------------------------------------
struct Bary {
  std::vector<double> z, f, w;
};

static Bary aaa(const std::vector<double>& Z, const std::vector<double>& F, double tol, int mmax,
                double* best_err) {
  const int M = (int)Z.size();
  std::vector<char> sup(M, 0);
  std::vector<double> R(M), wgt(M);
  double mean = 0.0;
  for (int i = 0; i < M; ++i) {
    mean += F[i];
    wgt[i] = 1.0 / std::fabs(F[i]);
  }
  mean /= M;
  for (int i = 0; i < M; ++i) R[i] = mean;
  Bary B, best;
  double beste = INFINITY;
  int since_best = 0;
  std::vector<double> L, v;
  for (int it = 0; it < mmax && it < M - 1; ++it) {
    int jmax = -1;
    double emax = -1.0;
    for (int i = 0; i < M; ++i) {
      if (sup[i]) continue;
      const double e = std::fabs(F[i] - R[i]) * wgt[i];
      if (e > emax) {
        emax = e;
        jmax = i;
      }
    }
    sup[jmax] = 1;
    B.z.push_back(Z[jmax]);
    B.f.push_back(F[jmax]);
    const int m = (int)B.z.size();
    const int rows = M - m;
    L.assign((size_t)rows * m, 0.0);
    int r = 0;
    for (int i = 0; i < M; ++i) {
      if (sup[i]) continue;
      for (int c = 0; c < m; ++c)
        L[(size_t)c * rows + r] = (F[i] - B.f[c]) / (Z[i] - B.z[c]) * wgt[i];
      ++r;
    }
    v.assign(m, 0.0);
    svd_min_right(rows, m, L.data(), v.data(), nullptr, nullptr);
    B.w = v;
    double err = 0.0;
    for (int i = 0; i < M; ++i) {
      if (sup[i]) {
        R[i] = F[i];
        continue;
      }
      double nn = 0.0, dd = 0.0;
      for (int c = 0; c < m; ++c) {
        const double q = B.w[c] / (Z[i] - B.z[c]);
        nn += q * B.f[c];
        dd += q;
      }
      R[i] = nn / dd;
      err = std::max(err, std::fabs(F[i] - R[i]) * wgt[i]);
    }
    if (err < 0.5 * beste) since_best = 0;
    else ++since_best;
    if (err < beste) {
      beste = err;
      best = B;
    }
    // stop at the tolerance, or once the rounding floor is reached (no halving in 4 steps)
    if (err <= tol || since_best >= 4) break;
  }
  if (best_err) *best_err = beste;
  return best;
}

// zeros of sum_j w_j / (z - z_j)
static int bary_poles(const Bary& B, std::vector<cplx>& out) {
  const int m = (int)B.z.size();
  out.clear();
  if (m < 2) return 0;
  double wn = 0.0, ws = 0.0;
  for (int j = 0; j < m; ++j) {
    wn += B.w[j] * B.w[j];
    ws += B.w[j];
  }
  wn = std::sqrt(wn);
  if (std::fabs(ws) <= 1e-14 * wn * std::sqrt((double)m)) return -1;
  // Householder reflector H with H w = (.) e_0; Q = columns 1..m-1 of H span w-perp
  std::vector<double> hv(B.w);
  hv[0] += (B.w[0] >= 0 ? wn : -wn);
  double hn = 0.0;
  for (double x : hv) hn += x * x;
  const int k = m - 1;
  std::vector<double> Q((size_t)m * k);  // row-major m x k
  for (int i = 0; i < m; ++i)
    for (int c = 0; c < k; ++c)
      Q[(size_t)i * k + c] = (i == c + 1 ? 1.0 : 0.0) - 2.0 * hv[i] * hv[c + 1] / hn;
  // B = Q^T Z Q - (Q^T 1)(w^T Z Q) / (w^T 1)
  std::vector<double> Qt1(k, 0.0), wZQ(k, 0.0), Bm((size_t)k * k, 0.0);
  for (int c = 0; c < k; ++c)
    for (int i = 0; i < m; ++i) {
      Qt1[c] += Q[(size_t)i * k + c];
      wZQ[c] += B.w[i] * B.z[i] * Q[(size_t)i * k + c];
    }
  for (int a = 0; a < k; ++a)
    for (int b = 0; b < k; ++b) {
      double s = 0.0;
      for (int i = 0; i < m; ++i) s += Q[(size_t)i * k + a] * B.z[i] * Q[(size_t)i * k + b];
      Bm[(size_t)a * k + b] = s - Qt1[a] * wZQ[b] / ws;
    }
  std::vector<double> wr(k), wi(k);
  if (eig_real_general(k, Bm.data(), wr.data(), wi.data()) != 0) return -2;
  for (int i = 0; i < k; ++i) out.emplace_back(wr[i], wi[i]);
  return 0;
}

// Least squares min ||A x - b||_2 (A: rows x k, column-major) by column scaling, Householder QR
// and a one-sided Jacobi SVD of R with singular values below 1e-15 sigma_max dropped.
static bool lsq_solve(int rows, int k, std::vector<double>& A, std::vector<double>& b,
                      std::vector<double>& x) {
  if (rows < k) return false;
  std::vector<double> scale(k, 1.0);
  for (int j = 0; j < k; ++j) {
    double s = 0.0;
    for (int i = 0; i < rows; ++i) s += A[(size_t)j * rows + i] * A[(size_t)j * rows + i];
    scale[j] = s > 0 ? 1.0 / std::sqrt(s) : 1.0;
    for (int i = 0; i < rows; ++i) A[(size_t)j * rows + i] *= scale[j];
  }
  std::vector<double> R, V;
  householder_r(rows, k, A, R, &b);
  jacobi_orthogonalize(k, R, V);
  // R V = U diag(sigma): x = V diag(1/sigma^2) (R V)^T (Q^T b)_top
  std::vector<double> sig(k);
  double smax = 0.0;
  for (int j = 0; j < k; ++j) {
    double s = 0.0;
    for (int i = 0; i < k; ++i) s += R[(size_t)j * k + i] * R[(size_t)j * k + i];
    sig[j] = std::sqrt(s);
    smax = std::max(smax, sig[j]);
  }
  x.assign(k, 0.0);
  for (int j = 0; j < k; ++j) {
    if (sig[j] <= 1e-15 * smax) continue;
    double t = 0.0;
    for (int i = 0; i < k; ++i) t += R[(size_t)j * k + i] * b[i];
    t /= sig[j] * sig[j];
    for (int i = 0; i < k; ++i) x[i] += t * V[(size_t)j * k + i];
  }
  for (int j = 0; j < k; ++j) x[j] *= scale[j];
  return true;
}

// weighted least squares for c0, c_k with fixed poles (scaled variable z)
static bool refit(const std::vector<double>& Z, const std::vector<double>& F,
                  const std::vector<double>& poles, double* c0, std::vector<double>& c) {
  const int M = (int)Z.size(), k = (int)poles.size() + 1;
  std::vector<double> A((size_t)M * k), b(M), x;
  for (int i = 0; i < M; ++i) {
    const double w = 1.0 / std::fabs(F[i]);
    A[i] = w;
    for (int j = 1; j < k; ++j) A[(size_t)j * M + i] = w / (Z[i] - poles[j - 1]);
    b[i] = F[i] * w;
  }
  if (!lsq_solve(M, k, A, b, x)) return false;
  *c0 = x[0];
  c.assign(x.begin() + 1, x.end());
  return true;
}

// Pole relocation by vector fitting (Gustavsen and Semlyen 1999): with the current poles a_k,
// fit sigma(z) = 1 + sum d_k / (z - a_k) and (sigma f)(z) = c0 + sum c_k / (z - a_k) jointly by
// linear least squares (relative weights); the zeros of sigma, the eigenvalues of
// diag(a) - 1 d^T, become the new poles.  Relocated poles off the negative real axis are
// dropped.  The pole set with the smallest refit error over the iterations is returned.
static double refit_error(const std::vector<double>& Z, const std::vector<double>& F,
                          const std::vector<double>& poles) {
  double c0;
  std::vector<double> c;
  if (!refit(Z, F, poles, &c0, c)) return INFINITY;
  double e = 0.0;
  for (size_t i = 0; i < Z.size(); ++i) {
    double v = c0;
    for (size_t k = 0; k < poles.size(); ++k) v += c[k] / (Z[i] - poles[k]);
    e = std::max(e, std::fabs(v - F[i]) / std::fabs(F[i]));
  }
  return e;
}

static void vf_refine(const std::vector<double>& Z, const std::vector<double>& F,
                      std::vector<double>& poles, int iters) {
  const int M = (int)Z.size();
  std::vector<double> best = poles;
  double beste = refit_error(Z, F, poles);
  for (int it = 0; it < iters; ++it) {
    const int k = (int)poles.size();
    if (k == 0) break;
    const int nu = 2 * k + 1;
    std::vector<double> A((size_t)M * nu), b(M), x;
    for (int i = 0; i < M; ++i) {
      const double w = 1.0 / std::fabs(F[i]);
      A[i] = w;
      for (int j = 0; j < k; ++j) {
        const double q = 1.0 / (Z[i] - poles[j]);
        A[(size_t)(1 + j) * M + i] = w * q;
        A[(size_t)(1 + k + j) * M + i] = -w * F[i] * q;
      }
      b[i] = F[i] * w;
    }
    if (!lsq_solve(M, nu, A, b, x)) break;
    std::vector<double> T((size_t)k * k), wr(k), wi(k);
    for (int r = 0; r < k; ++r)
      for (int c = 0; c < k; ++c) T[(size_t)r * k + c] = (r == c ? poles[r] : 0.0) - x[1 + k + c];
    if (eig_real_general(k, T.data(), wr.data(), wi.data()) != 0) break;
    std::vector<double> np;
    for (int j = 0; j < k; ++j)
      if (std::fabs(wi[j]) <= 1e-8 * std::hypot(wr[j], wi[j]) && wr[j] < 0.0) np.push_back(wr[j]);
    if (np.empty()) break;
    poles.swap(np);
    const double e = refit_error(Z, F, poles);
    if (e < beste) {
      beste = e;
      best = poles;
    }
  }
  poles = best;
}

static RaResult build_direct(int which, double K, double gamma, double lam_lo, double lam_hi,
                             const double* check_pts, int ncheck, double tol, int max_poles,
                             double t) {
  RaResult best;
  std::memset(&best, 0, sizeof(best));
  best.status = -4;  // FDD_E_RA until something acceptable is found
  best.max_rel_err = INFINITY;
  if (!(lam_lo > 0) || !(lam_hi > lam_lo) || !(tol > 0)) return best;
  max_poles = std::min(std::max(max_poles, 1), kMaxPoles);
  const int sample_counts[3] = {1200, 3000, 6000};
  std::vector<double> extra;
  for (int attempt = 0; attempt < 3; ++attempt) {
    const int ns = sample_counts[attempt];
    std::vector<double> lam(ns);
    for (int i = 0; i < ns; ++i)
      lam[i] = std::exp(std::log(lam_lo) + (std::log(lam_hi) - std::log(lam_lo)) * i / (ns - 1));
    for (double e : extra) lam.push_back(e);
    std::vector<double> Z(lam.size()), F(lam.size());
    for (size_t i = 0; i < lam.size(); ++i) {
      Z[i] = lam[i] / lam_hi;
      F[i] = fval(which, K, gamma, t, lam[i]);
    }
    const double aaa_tol = tol * (attempt == 0 ? 0.5 : 0.1);
    double aaa_err = 0.0;
    Bary B = aaa(Z, F, aaa_tol, max_poles + 1, &aaa_err);
    std::vector<cplx> pl;
    if (bary_poles(B, pl) != 0) continue;
    std::vector<double> keep;
    int dropped = 0;
    for (const cplx& z : pl) {
      const bool real = std::fabs(z.imag()) <= 1e-8 * std::abs(z);
      if (real && z.real() < 0.0) keep.push_back(z.real());
      else ++dropped;
    }
    if ((int)keep.size() > max_poles) keep.resize(max_poles);
    vf_refine(Z, F, keep, 6);
    double c0;
    std::vector<double> c;
    if (!refit(Z, F, keep, &c0, c)) continue;
    RaResult r;
    std::memset(&r, 0, sizeof(r));
    r.c0 = c0;
    r.m = (int)keep.size();
    for (int k = 0; k < r.m; ++k) {
      r.p[k] = -keep[k] * lam_hi;
      r.c[k] = c[k] * lam_hi;
    }
    r.aaa_support = (int)B.z.size();
    r.dropped = dropped;
    double err = ra_eval_rel_err(which, K, gamma, r, lam.data(), (int)lam.size(), t);
    if (check_pts && ncheck > 0)
      err = std::max(err, ra_eval_rel_err(which, K, gamma, r, check_pts, ncheck, t));
    // positivity of the approximate inverse on the spectrum
    bool positive = true;
    for (double x : lam) positive = positive && (ra_value(r, x) > 0.0);
    for (int i = 0; i < ncheck && check_pts; ++i)
      positive = positive && (ra_value(r, check_pts[i]) > 0.0);
    r.max_rel_err = err;
    r.status = (positive && err <= 10.0 * tol) ? 0 : -4;
    if (r.status == 0 && (best.status != 0 || err < best.max_rel_err)) best = r;
    else if (best.status != 0 && err < best.max_rel_err) best = r;
    if (best.status == 0 && err <= tol) break;
    // densify near the worst check points for the next attempt
    if (check_pts && ncheck > 0) {
      extra.clear();
      for (int i = 0; i < ncheck; ++i) {
        const double f = fval(which, K, gamma, t, check_pts[i]);
        if (std::fabs(f - ra_value(r, check_pts[i])) / std::fabs(f) > tol) extra.push_back(check_pts[i]);
        if (extra.size() > 400) break;
      }
    }
  }
  return best;
}


// f(lam) = 1 / (K lam^{1/2} + gamma lam^{-1/2}) = lam g(lam) / (K (lam + a)) with g = lam^{-1/2}
// and a = gamma / K.  Given g_RA = d0 + sum d_k / (lam + q_k), the product lam g_RA / (K (lam + a))
// is rational with the real shifts {a, q_k}, and its relative error equals that of g_RA at every
// lam because the factor lam / (K (lam + a)) is exact and positive.  Partial fractions:
//   lam / (lam + a)              = 1 - a / (lam + a)
//   lam / ((lam + a)(lam + q))   = (a / (a - q)) / (lam + a) - (q / (a - q)) / (lam + q).
static RaResult derive_precond(const RaResult& g, double K, double gamma) {
  RaResult r;
  std::memset(&r, 0, sizeof(r));
  r.status = -4;
  const double a = gamma / K;
  if (g.m + 1 > kMaxPoles) return r;
  double ca = -g.c0 * a;
  for (int k = 0; k < g.m; ++k) {
    const double dq = a - g.p[k];
    if (std::fabs(dq) <= 1e-12 * std::max(a, g.p[k])) return r;  // coincident shifts
    ca += g.c[k] * a / dq;
    r.p[k] = g.p[k];
    r.c[k] = -g.c[k] * g.p[k] / dq / K;
  }
  r.c0 = g.c0 / K;
  r.p[g.m] = a;
  r.c[g.m] = ca / K;
  r.m = g.m + 1;
  r.status = 0;
  r.aaa_support = g.aaa_support;
  r.dropped = g.dropped;
  return r;
}

RaResult build_rational(int which, double K, double gamma, double lam_lo, double lam_hi,
                        const double* check_pts, int ncheck, double tol, int max_poles, double t) {
  if (which == 1)
    return build_direct(1, K, gamma, lam_lo, lam_hi, check_pts, ncheck, tol, max_poles, t);
  // preconditioner: the product form first, direct AAA as the alternative.  The preconditioner
  // only steers the iteration, so a table within 1e-9 is accepted even when 10 tol is below
  // the rounding floor of the partial-fraction form (large a = gamma / K nearly cancels c0).
  const double accept = std::max(10.0 * tol, 1e-9);
  RaResult best;
  std::memset(&best, 0, sizeof(best));
  best.status = -4;
  best.max_rel_err = INFINITY;
  // (the product form needs t = -1/2 and gamma > 0: f = lam g / (K (lam + gamma / K)))
  const RaResult g = (t == -0.5 && gamma > 0)
                         ? build_direct(1, K, gamma, lam_lo, lam_hi, check_pts, ncheck, tol,
                                        std::max(1, max_poles - 1), t)
                         : RaResult{};
  if (t == -0.5 && gamma > 0 && g.status == 0) {
    RaResult r = derive_precond(g, K, gamma);
    if (r.status == 0) {
      std::vector<double> pts;
      const int ns = 4000;
      for (int i = 0; i < ns; ++i)
        pts.push_back(std::exp(std::log(lam_lo) + (std::log(lam_hi) - std::log(lam_lo)) * i / (ns - 1)));
      for (int i = 0; i < ncheck && check_pts; ++i) pts.push_back(check_pts[i]);
      r.max_rel_err = ra_eval_rel_err(0, K, gamma, r, pts.data(), (int)pts.size(), t);
      bool positive = true;
      for (double x : pts) positive = positive && (ra_value(r, x) > 0.0);
      r.status = (positive && r.max_rel_err <= accept) ? 0 : -4;
      best = r;
      if (r.status == 0 && r.max_rel_err <= tol) return r;
    }
  }
  RaResult d = build_direct(0, K, gamma, lam_lo, lam_hi, check_pts, ncheck, tol, max_poles, t);
  if (d.status != 0 && d.max_rel_err <= accept && d.m > 0) d.status = 0;
  if (d.status == 0 && (best.status != 0 || d.max_rel_err < best.max_rel_err)) return d;
  if (best.status != 0 && d.max_rel_err < best.max_rel_err) return d;
  return best;
}

}  // namespace fdd
