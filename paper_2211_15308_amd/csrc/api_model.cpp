// The paper's own model problem in 2D (Sec. 3, eq. (model_problem)): find x in V = H^1(Omega),
// Omega = (0, 1)^2, with K (-Delta + I) x + gamma (-Delta_Gamma + I)^t x = b, Gamma = the whole
// boundary.  The same method as the facet problems, on another mesh and interface layer:
//   * interior Dirichlet block A_II = A_Omega + M_Omega (7-point: stiffness plus P1 mass),
//     inverted by PCG preconditioned with V-cycles of the interior multigrid (the 5-point
//     Laplacian's V-cycle: the mass term changes the spectrum by under 1/(2 pi^2), so the
//     V-cycle stays a uniform preconditioner), FP64 recurrences, FP32 or FP64 V-cycles;
//   * the interface is the closed boundary loop (4n nodes), L = -Delta_Gamma + I on it, the
//     preconditioner S_Gamma = K L^{1/2} + gamma L^t and the operator's L^t by rational tables
//     (eq. (RA)) whose shifted systems are cyclic tridiagonal (kernels_model.hip);
//   * Schur-complement PCG on the loop (x_0 = 0, stop rule of Sec. 3), then the interior part by
//     one more interior solve.
// Every step runs in kernels; the host enqueues and reads the stop flags back.
#include <chrono>
#include <cmath>
#include <cstring>

#include "api_internal.h"

using namespace fdd;

namespace {

// Buffers of the model problem inside the 2D workspace plan (interior padded FP64 vectors and
// loop vectors of 4n entries).
struct MBufs {
  double *x, *r, *p[2], *q;          // interior PCG (padded FP64)
  double *f, *xI;                    // interior right-hand side and a kept interior solution
  double *xG, *rG, *pG[2], *zG, *yG, *Hp;  // outer PCG on the loop
};

MBufs mbufs(fdd_problem_s* P) {
  MBufs b{};
  b.x = P->s64.x;
  b.r = P->s64.r[0];
  b.p[0] = P->s64.p[0];
  b.p[1] = P->s64.p[1];
  b.q = P->s64.z;
  b.f = P->xI[1];
  b.xI = P->xI[0];
  b.xG = P->xG[0];
  b.rG = P->rG[0];
  b.pG[0] = P->pG[0];
  b.pG[1] = P->pG[1];
  b.zG = P->zG;
  b.yG = P->yG;
  b.Hp = P->Hp;
  return b;
}

template <typename VT>
struct VSet {
  VT *vr, *Z;
  const MGBuffers<VT>* mg;
};
VSet<double> vset64(fdd_problem_s* P) { return VSet<double>{P->u64[0], P->u64[1], &P->s64.mg}; }
VSet<float> vset32(fdd_problem_s* P) { return VSet<float>{P->s32.r[0], P->s32.r[1], &P->s32.mg}; }

// A_II u = f (f in b.f, u into b.x), to ||f - A_II u|| <= rtol ||f||.  Iterations are enqueued
// ahead of the read-back (as many as this problem's last interior solve took; kernels after the
// stop return at once).  Returns the iteration count through *its.
template <typename VT>
int model_inner_t(fdd_problem_s* P, hipStream_t s, const fdd_opts& o, const VSet<VT>& v,
                  const MBufs& b, int* its) {
  const int n = P->n, nf = n - 1, pitch = P->lev[0].pitch;
  const LaunchCtx c = make_ctx(P, s, o.mg_nu, sizeof(VT) == 8);
  launch_model_ii_start<VT>(s, nf, pitch, b.f, b.x, b.r, v.vr, P->st, P->partials,
                            o.inner_rtol * o.inner_rtol);
  launch_vcycle<VT>(c, *v.mg, v.vr, v.Z);
  launch_model_ii_rz<VT>(s, nf, pitch, b.r, v.Z, 1.0, P->st, P->partials);
  int k = 0, want = std::max(P->model_its_hint, 2), rc;
  for (;;) {
    for (; k < want && k < o.inner_maxit; ++k) {
      launch_model_ii_step<VT>(s, n, pitch, v.Z, 1.0, b.p[k & 1], b.p[(k + 1) & 1], b.q, b.x, b.r,
                               v.vr, P->st, P->partials, k == 0 ? 1 : 0);
      launch_vcycle<VT>(c, *v.mg, v.vr, v.Z);
      launch_model_ii_rz<VT>(s, nf, pitch, b.r, v.Z, 1.0, P->st, P->partials);
    }
    HIPCHK(hipGetLastError());
    if ((rc = read_state(P, s))) return rc;
    const DevState& h = *P->host_st;
    if (h.breakdown & 5)
      return fail(h.breakdown & 4 ? FDD_E_NONFINITE : FDD_E_BREAKDOWN,
                  "model interior solve: breakdown (flags %d)", h.breakdown);
    if (h.inner_done) break;
    if (k >= o.inner_maxit)
      return fail(FDD_NOT_CONVERGED, "model interior solve: %d iterations, residual %.3e of %.3e", k,
                  std::sqrt(h.rr), std::sqrt(h.ff));
    want = k + 2;
  }
  *its = P->host_st->inner_its;
  P->model_its_hint = std::max(*its, 1);
  return FDD_OK;
}

int model_inner(fdd_problem_s* P, hipStream_t s, const fdd_opts& o, const MBufs& b, int* its) {
  return o.precision == FDD_FP64 ? model_inner_t<double>(P, s, o, vset64(P), b, its)
                                 : model_inner_t<float>(P, s, o, vset32(P), b, its);
}

// y_G = S p = K (A+M)_{GG} p + K (A+M)_{GI} E p + gamma L^t_RA p, with E p from one interior
// solve of A_II u = -(A+M)_{IG} p.
int model_schur_product(fdd_problem_s* P, hipStream_t s, const fdd_opts& o, const MBufs& b,
                        const ShiftTable& tH, const double* p, double* y, int* its) {
  const int n = P->n, pitch = P->lev[0].pitch;
  launch_model_interior_rows(s, n, pitch, -1.0, nullptr, p, b.f);
  int rc = model_inner(P, s, o, b, its);
  if (rc) return rc;
  launch_model_loop_batch(s, n, tH, kIfaceOperator, p, b.Hp, P->scratchH);
  launch_model_loop_rows(s, n, pitch, P->K, P->gamma, b.x, p, b.Hp, nullptr, y);
  HIPCHK(hipGetLastError());
  return FDD_OK;
}

}  // namespace

namespace fdd {

int model_interior_solve(fdd_problem_s* P, const double* f, double* u, const fdd_opts& o,
                         hipStream_t s, int* its) {
  const MBufs b = mbufs(P);
  const int nf = P->n - 1, pitch = P->lev[0].pitch;
  launch_copy_rows(s, f, nf, b.f, pitch, nf, nf);
  int k = 0;
  int rc = model_inner(P, s, o, b, &k);
  if (its) *its = k;
  if (rc < 0) return rc;
  launch_copy_rows(s, b.x, pitch, u, nf, nf, nf);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return rc;
}

int model_precond_apply(fdd_problem_s* P, const fdd_ratpc_s* T, const double* r, double* z,
                        hipStream_t s) {
  launch_model_loop_batch(s, P->n, make_table(T), kIfacePrecond, r, z, P->scratchP);
  HIPCHK(hipGetLastError());
  return FDD_OK;
}

int model_apply_operator(fdd_problem_s* P, const fdd_ratpc_s* H, const double* x, double* y,
                         hipStream_t s) {
  launch_model_loop_batch(s, P->n, make_table(H), kIfaceOperator, x + P->NI, P->Hp, P->scratchH);
  launch_model_full_apply(s, P->n, P->K, P->gamma, x, P->Hp, y, nullptr, P->partials, nullptr);
  HIPCHK(hipGetLastError());
  return FDD_OK;
}

int model_schur_apply(fdd_problem_s* P, const fdd_ratpc_s* H, const double* x, double* y,
                      const fdd_opts& o, hipStream_t s) {
  const MBufs b = mbufs(P);
  int its = 0;
  int rc = model_schur_product(P, s, o, b, make_table(H), x, y, &its);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(s));
  return FDD_OK;
}

int model_solve(fdd_problem_s* P, const fdd_ratpc_s* PT, const fdd_ratpc_s* HT, const double* bv,
                double* x, const fdd_opts& o, hipStream_t s, fdd_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  fdd_stats st;
  std::memset(&st, 0, sizeof(st));
  st.true_rel_res = -1.0;
  const MBufs b = mbufs(P);
  const int n = P->n, nf = n - 1, pitch = P->lev[0].pitch, m = 4 * n;
  const ShiftTable tP = make_table(PT), tH = make_table(HT);
  const double rtol2 = o.outer_rtol * o.outer_rtol;
  const double* bG = bv + P->NI;
  auto finish = [&](int code) {
    st.status = code;
    st.t_solve_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = st;
    return code;
  };
  auto inner = [&](int* k) {
    int rc = model_inner(P, s, o, b, k);
    st.inner_solves += 1;
    st.inner_its_total += *k;
    st.inner_its_max = std::max(st.inner_its_max, *k);
    return rc;
  };
  // g = b_G - (A+M)_{GI} A_II^{-1} b_I; x_G = 0
  launch_copy_rows(s, bv, nf, b.f, pitch, nf, nf);
  int k = 0, rc = inner(&k);
  if (rc) return finish(rc);
  launch_model_loop_rows(s, n, pitch, -1.0, 0.0, b.x, nullptr, nullptr, bG, b.rG);
  HIPCHK(hipMemsetAsync(b.xG, 0, sizeof(double) * m, s));
  // z = S_Gamma^{-1} r, p = z, rho_0 (the outer state starts here)
  launch_model_loop_batch(s, n, tP, kIfacePrecond, b.rG, b.zG, P->scratchP);
  launch_model_outer_direction(s, m, b.rG, b.zG, b.pG[1], b.pG[0], P->st, 1, rtol2);
  HIPCHK(hipGetLastError());
  int its = 0;
  for (;;) {
    if ((rc = read_state(P, s))) return finish(rc);
    if (P->host_st->outer_done || its >= o.outer_maxit) break;
    const int a = its & 1;
    if ((rc = model_schur_product(P, s, o, b, tH, b.pG[a], b.yG, &k))) return finish(rc);
    st.inner_solves += 1;
    st.inner_its_total += k;
    st.inner_its_max = std::max(st.inner_its_max, k);
    launch_model_outer_update(s, m, b.pG[a], b.yG, b.xG, b.rG, P->st);
    launch_model_loop_batch(s, n, tP, kIfacePrecond, b.rG, b.zG, P->scratchP);
    launch_model_outer_direction(s, m, b.rG, b.zG, b.pG[a], b.pG[a ^ 1], P->st, 0, rtol2);
    HIPCHK(hipGetLastError());
    ++its;
  }
  const DevState h = *P->host_st;
  st.outer_its = its;
  if (h.breakdown & 6)
    return finish(fail(h.breakdown & 4 ? FDD_E_NONFINITE : FDD_E_BREAKDOWN,
                       "model outer PCG breakdown at iteration %d (flags %d)", its, h.breakdown));
  st.rel_precond_res = h.o_rho0 > 0 ? std::sqrt(std::max(h.o_rho[0], 0.0) / h.o_rho0) : 0.0;
  // x_I = A_II^{-1} (b_I / K - (A+M)_{IG} x_G)
  launch_model_interior_rows(s, n, pitch, -1.0, nullptr, b.xG, b.f, bv, 1.0 / P->K);
  if ((rc = inner(&k))) return finish(rc);
  launch_copy_rows(s, b.x, pitch, x, nf, nf, nf);
  HIPCHK(hipMemcpyAsync(x + P->NI, b.xG, sizeof(double) * m, hipMemcpyDeviceToDevice, s));
  if (o.check_true_residual) {
    launch_model_loop_batch(s, n, tH, kIfaceOperator, x + P->NI, P->Hp, P->scratchH);
    launch_model_full_apply(s, n, P->K, P->gamma, x, P->Hp, nullptr, bv, P->partials,
                            P->st->t_res);
  }
  HIPCHK(hipGetLastError());
  if ((rc = read_state(P, s))) return finish(rc);
  if (o.check_true_residual && P->host_st->t_res[1] > 0)
    st.true_rel_res = std::sqrt(P->host_st->t_res[0] / P->host_st->t_res[1]);
  return finish(h.outer_done ? FDD_OK : FDD_NOT_CONVERGED);
}

}  // namespace fdd

extern "C" {

int fdd_setup_model(int n, double K, double gamma, double t, int hip_device, fdd_problem* out) {
  if (!out) return fail(FDD_E_ARG, "null argument");
  *out = nullptr;
  // the loop interface kernels hold one loop vector (4n entries) per workgroup in LDS
  if (n < 4 || (n & 1) || n > 1024)
    return fail(FDD_E_ARG, "model problem: n must be even, 4 <= n <= 1024 (got %d)", n);
  if (!(K > 0) || !std::isfinite(K) || !(gamma >= 0) || !std::isfinite(gamma))
    return fail(FDD_E_ARG, "model problem: K > 0 and gamma >= 0 must be finite");
  if (!(t > -1.0 && t < 1.0)) return fail(FDD_E_ARG, "model problem: t must lie in (-1, 1)");
  fdd_desc d{2, n, K, 1.0};
  fdd_problem P = nullptr;
  int rc = fdd_setup_mesh(&d, hip_device, &P);
  if (rc) return rc;
  P->kind = kProblemModel;
  P->tpow = t;
  P->gamma = gamma;
  P->mu = gamma > 0 ? 1.0 / gamma : INFINITY;
  P->NG = 4 * (int64_t)n;
  P->N = P->NI + P->NG;
  // spectrum of (A_G + M_G, M_G) on the loop (circulant): 1 + (2 - 2 cos th) / h / ((h/6)(4 + 2 cos th))
  const double h = 1.0 / n;
  P->eig.resize(4 * (size_t)n);
  for (int q = 0; q < 4 * n; ++q) {
    const double th = 2.0 * M_PI * q / (4.0 * n);
    P->eig[q] = 1.0 + (2.0 - 2.0 * std::cos(th)) / h / ((h / 6.0) * (4.0 + 2.0 * std::cos(th)));
  }
  P->lam_lo = 1.0;
  P->lam_hi = 1.0 + 12.0 / (h * h);
  *out = P;
  return FDD_OK;
}

}  // extern "C"
