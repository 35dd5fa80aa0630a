// Full-system PCG with the lazy block preconditioner (paper, Sec. 2 eq. (dd_preconditioner) and
// the remark on evaluating the operator in Sec. 3): PCG on A x = b itself, A = K A_Omega +
// gamma T^T H_RA T with H by its rational table, preconditioned by B of eq. (dd_preconditioner)
// whose leading block (A^00)^{-1} is one multigrid V-cycle V / K and whose interface block is the
// rational preconditioner table.  B stays symmetric (V is a symmetric V-cycle and the two
// off-diagonal factors are each other's transposes), so PCG applies.  No interior solve runs to
// a tolerance: every iteration costs two V-cycles, two batches of shifted interface solves and
// two stencil passes, and the iteration count stays bounded in h (Fig. 4-left).
#include <chrono>
#include <cmath>
#include <cstring>

#include "api_internal.h"

using namespace fdd;

namespace {

FullCtx make_full_ctx(const fdd_problem_s* P, hipStream_t s) {
  FullCtx c{};
  c.stream = s;
  c.nf = P->lev[0].nf;
  c.pitch = P->lev[0].pitch;
  c.K = P->K;
  c.gamma = P->gamma;
  c.h = P->h;
  c.xI = P->xI[0];
  c.rI = P->xI[1];
  c.pI[0] = P->s64.p[0];
  c.pI[1] = P->s64.p[1];
  c.qI = P->s64.x;
  c.xG = P->xG[0];
  c.rG = P->rG[0];
  c.pG[0] = P->pG[0];
  c.pG[1] = P->pG[1];
  c.qG = P->xG[1];
  c.zG = P->zG;
  c.tG = P->yG;
  c.Hp = P->Hp;
  c.scratchP = P->scratchP;
  c.scratchH = P->scratchH;
  c.partials = P->partials;
  c.st = P->st;
  return c;
}

// The V-cycle buffers of one precision: inputs vr (r_I) and vf (r_I + K lift(z_G)), outputs
// W = V vr and Z = V vf, and the hierarchy.  FP64 uses the FP64 set (plus the refinement
// accumulators), FP32 the FP32 set; neither overlaps the FP64 vectors of make_full_ctx.
template <typename VT>
struct VBufs {
  VT *vr, *vf, *W, *Z;
  const MGBuffers<VT>* mg;
};

VBufs<double> vbufs64(fdd_problem_s* P) {
  return VBufs<double>{P->s64.r[0], P->s64.r[1], P->u64[0], P->u64[1], &P->s64.mg};
}
VBufs<float> vbufs32(fdd_problem_s* P) {
  return VBufs<float>{P->s32.r[0], P->s32.r[1], P->s32.p[0], P->s32.p[1], &P->s32.mg};
}

// z = B r for the r already in place (r_I, r_G and the V-cycle inputs): both V-cycles and the
// interface block; Z holds V (r_I + K lift(z_G)), so z_I = Z / K.
template <typename VT>
void enqueue_precond(const LaunchCtx& c, const FullCtx& fc, const ShiftTable& tabP, const VBufs<VT>& v) {
  launch_vcycle<VT>(c, *v.mg, v.vr, v.W);
  launch_full_precond_tail<VT>(fc, tabP, v.W, v.vf);
  launch_vcycle<VT>(c, *v.mg, v.vf, v.Z);
}

int check_full_args(fdd_problem_s* P, fdd_ratpc PT, const double* in, const double* out,
                    const fdd_opts& o) {
  if (P->dim != 2 || P->kind != kProblemFacet)
    return fail(FDD_E_ARG, "the full-system PCG is built for the 2D facet problem");
  if (!in || !out) return fail(FDD_E_ARG, "null vector");
  if (!opts_ok(&o)) return fail(FDD_E_ARG, "invalid options");
  if (o.warmstart) return fail(FDD_E_ARG, "the full-system PCG takes no warm start");
  return check_table(P, PT, FDD_RA_PRECOND);
}

template <typename VT>
int solve_full_t(fdd_problem_s* P, const fdd_ratpc_s* PT, const fdd_ratpc_s* HT, const double* b,
                 double* x, const fdd_opts& o, hipStream_t s, fdd_stats& st,
                 const VBufs<VT>& v) {
  const LaunchCtx c = make_ctx(P, s, o.mg_nu, sizeof(VT) == 8);
  const FullCtx fc = make_full_ctx(P, s);
  const ShiftTable tP = make_table(PT), tH = make_table(HT);
  const double rtol2 = o.outer_rtol * o.outer_rtol;
  // r = b, x = 0, z = B r, p = z
  launch_full_init<VT>(fc, b, v.vr, v.vf);
  enqueue_precond<VT>(c, fc, tP, v);
  launch_full_rz<VT>(fc, v.Z, 0, 1, rtol2, 0);
  HIPCHK(hipGetLastError());
  // iterations are enqueued ahead of the read-back: as many as this problem's last solve took
  // (kernels of iterations beyond the stop return at once), then one at a time
  int its = 0, want = std::max(P->full_its_hint, 1), rc = FDD_OK;
  for (;;) {
    for (; its < want && its < o.outer_maxit; ++its) {
      const int a = its & 1;
      launch_full_step<VT>(fc, tH, v.Z, a, a, its == 0 ? 1 : 0, v.vr, v.vf, its);
      enqueue_precond<VT>(c, fc, tP, v);
      launch_full_rz<VT>(fc, v.Z, a ^ 1, 0, rtol2, its + 1);
    }
    HIPCHK(hipGetLastError());
    if ((rc = read_state(P, s))) return rc;
    if (P->host_st->outer_done || its >= o.outer_maxit) break;
    want = its + 1;
  }
  launch_full_clear_stop(fc);
  if (P->host_st->outer_done) its = P->host_st->o_its;
  P->full_its_hint = its;
  const DevState& h = *P->host_st;
  st.outer_its = its;
  st.inner_solves = 2 * (its + 1);  // V-cycles
  if (h.breakdown)
    return fail(h.breakdown & 4 ? FDD_E_NONFINITE : FDD_E_BREAKDOWN,
                "full-system PCG breakdown at iteration %d (flags %d)", its, h.breakdown);
  const double rz = h.o_rho[its & 1];
  st.rel_precond_res = h.o_rho0 > 0 ? std::sqrt(std::max(rz, 0.0) / h.o_rho0) : 0.0;
  launch_full_scatter<double>(fc, fc.xI, 1.0, fc.xG, x);
  if (o.check_true_residual) {
    launch_iface_batch(s, (int)P->NG, P->h, tH, kIfaceOperator, x + P->NI, P->Hp, P->scratchH,
                       P->st, nullptr, nullptr, 0, 0);
    launch_full_operator(s, P->n, P->K, P->gamma, x, P->Hp, nullptr, b, P->partials,
                         P->st->t_res);
  }
  HIPCHK(hipGetLastError());
  if ((rc = read_state(P, s))) return rc;
  if (o.check_true_residual && P->host_st->t_res[1] > 0)
    st.true_rel_res = std::sqrt(P->host_st->t_res[0] / P->host_st->t_res[1]);
  return P->host_st->outer_done ? FDD_OK : FDD_NOT_CONVERGED;
}

}  // namespace

extern "C" {

int fdd_dd_precond_apply(fdd_problem P, fdd_ratpc PT, const double* r, double* z,
                         const fdd_opts* opts, void* stream) {
  int rc = check_problem(P);
  if (rc) return rc;
  fdd_opts o;
  if (opts) o = *opts;
  else fdd_opts_default(&o);
  if ((rc = check_full_args(P, PT, r, z, o))) return rc;
  HIPCHK(hipSetDevice(P->device));
  hipStream_t s = (hipStream_t)stream;
  const FullCtx fc = make_full_ctx(P, s);
  const ShiftTable tP = make_table(PT);
  if (o.precision == FDD_FP64) {
    const auto v = vbufs64(P);
    launch_full_init<double>(fc, r, v.vr, v.vf);
    enqueue_precond<double>(make_ctx(P, s, o.mg_nu, true), fc, tP, v);
    launch_full_scatter<double>(fc, v.Z, 1.0 / P->K, fc.zG, z);
  } else {
    const auto v = vbufs32(P);
    launch_full_init<float>(fc, r, v.vr, v.vf);
    enqueue_precond<float>(make_ctx(P, s, o.mg_nu, false), fc, tP, v);
    launch_full_scatter<float>(fc, v.Z, 1.0 / P->K, fc.zG, z);
  }
  HIPCHK(hipGetLastError());
  return FDD_OK;
}

int fdd_solve_full(fdd_problem P, fdd_ratpc PT, fdd_ratpc HT, const double* b, double* x,
                   const fdd_opts* opts, void* stream, fdd_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  int rc = check_problem(P);
  if (rc) return rc;
  fdd_opts o;
  if (opts) o = *opts;
  else fdd_opts_default(&o);
  if ((rc = check_full_args(P, PT, b, x, o))) return rc;
  if ((rc = check_table(P, HT, FDD_RA_OPERATOR))) return rc;
  HIPCHK(hipSetDevice(P->device));
  hipStream_t s = (hipStream_t)stream;
  fdd_stats st;
  std::memset(&st, 0, sizeof(st));
  st.true_rel_res = -1.0;
  if (o.precision == FDD_FP64) rc = solve_full_t<double>(P, PT, HT, b, x, o, s, st, vbufs64(P));
  else rc = solve_full_t<float>(P, PT, HT, b, x, o, s, st, vbufs32(P));
  st.status = rc;
  st.t_solve_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (stats) *stats = st;
  return rc;
}

}  // extern "C"
