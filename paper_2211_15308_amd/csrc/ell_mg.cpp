// PCG preconditioned by a multigrid V-cycle on a typed-ELL hierarchy (ell_mg.h).
#include "ell_mg.h"

#include <algorithm>
#include <cmath>

#include "api_internal.h"

namespace fdd {

int ell_read_state(const EllHier& H, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(H.hst, H.st, sizeof(HdState), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return FDD_OK;
}

void ell_vcycle(const EllHier& H, hipStream_t s, int nu, int l, const double* b, double* x,
                const HdState* stop) {
  const HdLevel& L = H.lev[l];
  if (l == H.nlev - 1) {
    if (H.cinv) {
      launch_hd_coarse(s, H.cinv, L.n0, b, x, stop);
    } else {
      launch_hd_patch_solve(s, L, b, stop);
      launch_hd_patch_sum(s, L, H.theta, x, 0, stop);
    }
    return;
  }
  const HdLevel& C = H.lev[l + 1];
  launch_hd_patch_solve(s, L, b, stop);
  launch_hd_patch_sum(s, L, H.theta, x, 0, stop);
  for (int k = 1; k < nu; ++k) {
    launch_hd_residual(s, view(L.A), b, x, L.r, stop);
    launch_hd_patch_solve(s, L, L.r, stop);
    launch_hd_patch_sum(s, L, H.theta, x, 1, stop);
  }
  launch_hd_residual(s, view(L.A), b, x, L.r, stop);
  launch_hd_spmv(s, view(L.R), L.r, C.b, 1.0, 0.0, stop);
  ell_vcycle(H, s, nu, l + 1, C.b, C.x, stop);
  launch_hd_spmv(s, view(L.P), C.x, x, 1.0, 1.0, stop);
  for (int k = 0; k < nu; ++k) {
    launch_hd_residual(s, view(L.A), b, x, L.r, stop);
    launch_hd_patch_solve(s, L, L.r, stop);
    launch_hd_patch_sum(s, L, H.theta, x, 1, stop);
  }
}

int ell_pcg(const EllHier& H, hipStream_t s, int nu, double rtol, int maxit, const double* f,
            double* u, int* hint, int* its, const char* what) {
  const int n0 = H.n0;
  const HdLevel& L0 = H.lev[0];
  launch_hd_pcg_start(s, n0, f, u, H.r, H.partials, H.st, rtol * rtol);
  double* p[2] = {H.p, H.p + n0};
  int k = 0, want = std::max(*hint, 2);
  for (;;) {
    for (; k < want && k < maxit; ++k) {
      ell_vcycle(H, s, nu, 0, H.r, H.z, H.st);
      launch_hd_pcg_rz(s, n0, H.r, H.z, H.partials, H.st, k == 0);
      launch_hd_pcg_pq(s, view(L0.A), H.z, p[(k + 1) & 1], p[k & 1], H.q, H.partials, H.st,
                       k == 0);
      launch_hd_pcg_update(s, n0, p[k & 1], H.q, u, H.r, H.partials, H.st);
    }
    HIPCHK(hipGetLastError());
    int rc = ell_read_state(H, s);
    if (rc) return rc;
    const HdState& h = *H.hst;
    if (h.breakdown & 5)
      return fail(h.breakdown & 4 ? FDD_E_NONFINITE : FDD_E_BREAKDOWN, "%s: breakdown (flags %d)",
                  what, h.breakdown);
    if (h.done) break;
    if (k >= maxit)
      return fail(FDD_NOT_CONVERGED, "%s: %d iterations, residual %.3e of %.3e", what, k,
                  std::sqrt(h.rr), std::sqrt(h.ff));
    want = k + 2;
  }
  *its = H.hst->its;
  *hint = std::max(*its, 1);
  return FDD_OK;
}

}  // namespace fdd
