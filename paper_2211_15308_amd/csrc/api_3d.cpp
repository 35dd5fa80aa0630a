// Host orchestration of the 3D solver (dim = 3 problems of the C ABI): the unit cube with Kuhn
// tetrahedra, Gamma the face z = 1.  The method is the 2D one (paper, Sec. 2): outer PCG on the
// interface Schur complement, interior solves by multigrid-preconditioned CG, the rational
// preconditioner and operator of eq. (RA).  In 3D every interior block is h L7 (L7 the 7-point
// stencil), the Gamma row of the stiffness is h (3, -1/2 x 4 in the face, -1 below), and the
// shifted interface systems are 2D face problems solved by batched CG (kernels_3d.hip).  The
// interface work is FP64; interior solves run FP32 multigrid-PCG inside FP64 iterative refinement
// (or FP64 multigrid-PCG).  Krylov iterations are replayed from captured graphs; the host enqueues
// as many as the previous solve of the same kind took, then reads the device flags and adds
// one iteration at a time.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "api_internal.h"
#include "k3_internal.h"

using namespace fdd;

// Captured runs of a Krylov iteration k: one iteration for each parity of k, and 4 and 8
// iterations from an even k (the buffers alternate with the parity of k).
struct Chunks {
  hipGraphExec_t one[2] = {nullptr, nullptr};
  hipGraphExec_t four = nullptr, eight = nullptr;
  void clear() {
    for (hipGraphExec_t* g : {&one[0], &one[1], &four, &eight}) {
      if (*g) (void)hipGraphExecDestroy(*g);
      *g = nullptr;
    }
  }
};

// buffers of one face batch (device, except the pinned read-back mirrors)
struct FaceBufs {
  double *y = nullptr, *z = nullptr, *q = nullptr, *t = nullptr, *tmp = nullptr;
  double* r[2] = {};  // r_k in r[k & 1]
  double* p[2] = {};  // p_k in p[k & 1]
  double *part0 = nullptr, *part1 = nullptr;
  FaceCG* cg = nullptr;
  int* done = nullptr;
  int* hdone = nullptr;
  int* hits = nullptr;
  int enq = 0;  // iterations enqueued
};

// multigrid-PCG of the interior in precision R: level iterates and right-hand sides, the PCG
// vectors (r_k in Rv[k & 1], p_k in PB[k & 1]) and its captured work (the first V-cycle of a run;
// chunks of iterations); pred = iterations of the last run (enqueued before the first check)
template <typename R>
struct Mg3 {
  R* u[kMaxLevels] = {};   // pre-smoothed iterates (level 0: scratch)
  R* uo[kMaxLevels] = {};  // iterates after the coarse correction, levels < lc (level 0: z)
  R* f[kMaxLevels] = {};   // right-hand sides of the levels >= 1
  R* x = nullptr;
  R* Rv[2] = {};
  R* PB[2] = {};
  R* q = nullptr;
  hipGraphExec_t g_init = nullptr;
  Chunks g_it;
  int g_nu = 0;
  int pred = 8;
};

struct Problem3D {
  int n = 0, nf = 0, nlev = 0, nc = 0;
  int lnf[kMaxLevels] = {};
  int lc = 1;     // levels lc .. nlev - 1 run in the one-workgroup coarse kernel
  Cvc3 cvc{};     // their sizes
  int rows0 = 4;  // rows per block of the level-0 reduction kernels
  int np0 = 0;    // their partials
  Mg3<double> m64;  // FP64 multigrid-PCG
  Mg3<float> m32;   // FP32 multigrid-PCG inside FP64 refinement
  double* F64 = nullptr;        // FP64 right-hand side of a refined solve (padded)
  double* X64[2] = {};          // its FP64 iterates (x' = x + e written to the other buffer)
  int xcur = 0;
  double* x = nullptr;          // the last interior solution (FP64, padded)
  double* xI = nullptr;  // interior part of the solution, accumulated during the outer PCG
  double *part0 = nullptr, *part1 = nullptr;
  State3* st = nullptr;
  int* stop = nullptr;
  double* cinv = nullptr;
  std::vector<double> cinv_h;
  double* S = nullptr;  // DST-I matrix of the face, nf x nf
  std::vector<double> S_h;
  Shift3* tabs = nullptr;  // [0] preconditioner batch, [1] operator batch
  FaceBufs fb[2];  // [0] preconditioner batch, [1] operator batch
  double *xG = nullptr, *rG = nullptr, *pG = nullptr, *zG = nullptr, *yG = nullptr, *Hp = nullptr;
  double* gpart = nullptr;
  double* sc = nullptr;  // the outer PCG's scalars (kSc3*), summed and derived on the device
  // pinned host mirrors
  State3* hst = nullptr;
  int* hstop = nullptr;
  double* hpart = nullptr;
  Shift3* htab = nullptr;  // [2]

  bool mixed = false;  // the running interior solve refines an FP32 multigrid-PCG
  int maxit = 0, nu = 1;
  int steps = 0;       // refinement steps enqueued after the first
  int runs_pred = 2;   // FP32 runs of the last refined solve
  int run_pred[kRuns3] = {8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8};  // its iterations per run
  // one face-CG iteration k per (batch, parity of k); iterations of the last batch of each kind
  Chunks g_face[2];
  int g_face_m[2] = {0, 0};
  int pred_face[2] = {12, 12};
  bool use_graph = true;
  // second stream (the H batch runs on it beside the interior solve of a Schur product)
  hipStream_t s2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int enq = 0;  // interior iterations enqueued
};

namespace {

constexpr double kFaceTolP = 1e-10;  // shifted solves of the preconditioner (steer the iteration)
constexpr double kFaceTolH = 1e-13;  // shifted solves of the operator H (enter the solution)

size_t vol(int nf) { return (size_t)(nf + 2) * (nf + 2) * (nf + 2); }

size_t plan3(fdd_problem_s* P, char* base) {
  Problem3D* Q = P->p3;
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    off = align_up(off, 256);
    char* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  };
  const size_t v0 = vol(Q->nf);
  auto mg = [&](auto& M, size_t w) {
    for (int l = 1; l < Q->nlev; ++l) {
      M.u[l] = (decltype(M.x))take(w * vol(Q->lnf[l]));
      M.f[l] = (decltype(M.x))take(w * vol(Q->lnf[l]));
      if (l < Q->lc) M.uo[l] = (decltype(M.x))take(w * vol(Q->lnf[l]));
    }
    M.u[0] = (decltype(M.x))take(w * v0);
    M.uo[0] = (decltype(M.x))take(w * v0);
    M.x = (decltype(M.x))take(w * v0);
    for (int b = 0; b < 2; ++b) {
      M.Rv[b] = (decltype(M.x))take(w * v0);
      M.PB[b] = (decltype(M.x))take(w * v0);
    }
    M.q = (decltype(M.x))take(w * v0);
  };
  mg(Q->m64, 8);
  mg(Q->m32, 4);
  Q->F64 = (double*)take(8 * v0);
  Q->X64[0] = (double*)take(8 * v0);
  Q->X64[1] = (double*)take(8 * v0);
  Q->x = Q->m64.x;
  Q->xI = (double*)take(8 * v0);
  Q->part0 = (double*)take(8 * kPart0);
  Q->part1 = (double*)take(8 * kPart0);
  Q->st = (State3*)take(sizeof(State3));
  Q->stop = (int*)take(sizeof(int));
  const size_t nc3 = (size_t)Q->nc * Q->nc * Q->nc;
  Q->cinv = (double*)take(8 * nc3 * nc3);
  Q->S = (double*)take(8 * (size_t)Q->nf * Q->nf);
  Q->tabs = (Shift3*)take(2 * sizeof(Shift3));
  const size_t ng = (size_t)Q->nf * Q->nf;
  for (FaceBufs& B : Q->fb) {
    B.cg = (FaceCG*)take(sizeof(FaceCG));
    B.done = (int*)take(sizeof(int) * kMaxSys3);
    B.part0 = (double*)take(8 * (size_t)kMaxSys3 * kPFS);
    B.part1 = (double*)take(8 * (size_t)kMaxSys3 * kPFS);
    for (double** v : {&B.y, &B.r[0], &B.r[1], &B.p[0], &B.p[1], &B.q, &B.z, &B.t})
      *v = (double*)take(8 * ng * kMaxSys3);
    B.tmp = (double*)take(8 * ng);
  }
  for (double** v : {&Q->xG, &Q->rG, &Q->pG, &Q->zG, &Q->yG, &Q->Hp})
    *v = (double*)take(8 * ng);
  Q->gpart = (double*)take(8 * 2 * kPart3);
  Q->sc = (double*)take(8 * kSc3Count);
  return align_up(off, 256);
}

// exact inverse of L7 on an nc^3 grid (Gauss-Jordan with pivoting)
std::vector<double> dense_inverse_7pt(int nc) {
  const int np = nc * nc * nc;
  std::vector<double> A((size_t)np * np, 0.0), X((size_t)np * np, 0.0);
  auto id = [&](int i, int j, int k) { return (k * nc + j) * nc + i; };
  for (int k = 0; k < nc; ++k)
    for (int j = 0; j < nc; ++j)
      for (int i = 0; i < nc; ++i) {
        const int r = id(i, j, k);
        A[(size_t)r * np + r] = 6.0;
        if (i > 0) A[(size_t)r * np + id(i - 1, j, k)] = -1.0;
        if (i < nc - 1) A[(size_t)r * np + id(i + 1, j, k)] = -1.0;
        if (j > 0) A[(size_t)r * np + id(i, j - 1, k)] = -1.0;
        if (j < nc - 1) A[(size_t)r * np + id(i, j + 1, k)] = -1.0;
        if (k > 0) A[(size_t)r * np + id(i, j, k - 1)] = -1.0;
        if (k < nc - 1) A[(size_t)r * np + id(i, j, k + 1)] = -1.0;
        X[(size_t)r * np + r] = 1.0;
      }
  for (int c = 0; c < np; ++c) {
    int piv = c;
    for (int r = c + 1; r < np; ++r)
      if (std::fabs(A[(size_t)r * np + c]) > std::fabs(A[(size_t)piv * np + c])) piv = r;
    if (piv != c)
      for (int k = 0; k < np; ++k) {
        std::swap(A[(size_t)c * np + k], A[(size_t)piv * np + k]);
        std::swap(X[(size_t)c * np + k], X[(size_t)piv * np + k]);
      }
    const double d = 1.0 / A[(size_t)c * np + c];
    for (int k = 0; k < np; ++k) {
      A[(size_t)c * np + k] *= d;
      X[(size_t)c * np + k] *= d;
    }
    for (int r = 0; r < np; ++r) {
      if (r == c) continue;
      const double fac = A[(size_t)r * np + c];
      if (fac == 0.0) continue;
      for (int k = 0; k < np; ++k) {
        A[(size_t)r * np + k] -= fac * A[(size_t)c * np + k];
        X[(size_t)r * np + k] -= fac * X[(size_t)c * np + k];
      }
    }
  }
  return X;
}

// V-cycle z = V r on the interior (nu red-black pairs per level: red, black, ... going down,
// black, red, ... going up).  mode 1: the start of a run (r_0 in Rv[0]; its |r_0|^2 partials
// come from the first pass, or, for a refined run, from the refinement step); mode 2: inside
// PCG iteration k (r_{k+1} = r_k - alpha_k q formed by the first pass, which leaves it in
// Rv[(k + 1) & 1]).  The pass after the first holds the convergence test.  The last pass leaves
// z in uo[0] and the partials of r . z in part0.
template <typename R>
void vcycle3(Problem3D* Q, Mg3<R>& M, hipStream_t s, int nu, int mode, int k, bool refined) {
  const int nf = Q->nf, np0 = Q->np0;
  int* stop = Q->stop;
  R* f0 = mode == 1 ? M.Rv[0] : M.Rv[(k + 1) & 1];
  if (mode == 1)
    k3_launch_zp<R>(s, refined ? 0 : 1, f0, M.u[0], nf, Q->rows0, nullptr, nullptr, nullptr,
                    nullptr, Q->st, nullptr, 0, Q->part0, stop);
  else
    k3_launch_zp<R>(s, 2, M.Rv[k & 1], M.u[0], nf, Q->rows0, M.q, f0, M.x, M.PB[k & 1], Q->st,
                    Q->part1, np0, Q->part0, stop);
  int check = mode;
  for (int sw = 2; sw < 2 * nu; ++sw) {
    k3_launch_hs<R>(s, M.u[0], f0, nf, !(sw & 1), check, Q->st, Q->part0, np0, stop);
    check = 0;
  }
  k3_launch_rr<R>(s, M.u[0], f0, M.f[1], nf, Q->lnf[1], check, Q->st, Q->part0, np0, stop);
  for (int l = 1; l < Q->lc; ++l) {
    const int n = Q->lnf[l];
    k3_launch_zp<R>(s, 0, M.f[l], M.u[l], n, 4, nullptr, nullptr, nullptr, nullptr, Q->st,
                    nullptr, 0, nullptr, stop);
    for (int sw = 2; sw < 2 * nu; ++sw)
      k3_launch_hs<R>(s, M.u[l], M.f[l], n, !(sw & 1), 0, Q->st, nullptr, 0, stop);
    k3_launch_rr<R>(s, M.u[l], M.f[l], M.f[l + 1], n, Q->lnf[l + 1], 0, Q->st, nullptr, 0, stop);
  }
  k3_launch_cvc<R>(s, M.f[Q->lc], M.u[Q->lc], Q->cvc, Q->cinv, nu, stop);
  auto fin = [&](int l) { return l < Q->lc ? M.uo[l] : M.u[l]; };
  for (int l = Q->lc - 1; l >= 1; --l) {
    const int n = Q->lnf[l];
    k3_launch_pr<R>(s, M.u[l], fin(l + 1), M.f[l], M.uo[l], n, Q->lnf[l + 1], stop);
    for (int sw = 1; sw < 2 * nu; ++sw)
      k3_launch_hs<R>(s, M.uo[l], M.f[l], n, sw & 1, 0, Q->st, nullptr, 0, stop);
  }
  k3_launch_pr<R>(s, M.u[0], fin(1), f0, M.uo[0], nf, Q->lnf[1], stop);
  for (int sw = 1; sw + 1 < 2 * nu; ++sw)
    k3_launch_hs<R>(s, M.uo[0], f0, nf, sw & 1, 0, Q->st, nullptr, 0, stop);
  k3_launch_hsz<R>(s, M.uo[0], f0, nf, Q->rows0, Q->part0, stop);
}

// PCG iteration k: p_k, q = L7 p_k, then the V-cycle that starts with the residual update
template <typename R>
void iteration3(Problem3D* Q, Mg3<R>& M, hipStream_t s, int nu, int k) {
  k3_launch_apply1<R>(s, M.uo[0], M.PB[(k + 1) & 1], M.PB[k & 1], M.q, Q->nf, Q->rows0, Q->st,
                      Q->part0, Q->np0, Q->part1, Q->stop);
  vcycle3<R>(Q, M, s, nu, 2, k, false);
}

int sync_state(Problem3D* Q, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(Q->hst, Q->st, sizeof(State3), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(Q->hstop, Q->stop, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return FDD_OK;
}

// Captures the launches of fn on s into an executable graph.
template <typename Fn>
int capture(hipStream_t s, Fn fn, hipGraphExec_t* out) {
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  fn();
  hipError_t e = hipStreamEndCapture(s, &g);
  if (e != hipSuccess) return fail(FDD_E_HIP, "graph capture: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(FDD_E_HIP, "graph instantiate: %s", hipGetErrorString(e));
  return FDD_OK;
}

// Captures the chunks of iteration it(k).
template <typename It>
int capture_chunks(hipStream_t s, It it, Chunks* c) {
  c->clear();
  int rc = FDD_OK;
  for (int par = 0; par < 2 && !rc; ++par) rc = capture(s, [&]() { it(par); }, &c->one[par]);
  if (!rc) rc = capture(s, [&]() { for (int k = 0; k < 4; ++k) it(k); }, &c->four);
  if (!rc) rc = capture(s, [&]() { for (int k = 0; k < 8; ++k) it(k); }, &c->eight);
  return rc;
}

// Enqueues iterations k0 .. k1 - 1 (captured chunks, or it(k) launched one by one).
template <typename It>
int enqueue_iterations(hipStream_t s, bool graphs, const Chunks& c, It it, int k0, int k1) {
  int k = k0;
  while (k < k1) {
    if (!graphs) {
      it(k);
      ++k;
    } else if (!(k & 1) && k1 - k >= 8) {
      HIPCHK(hipGraphLaunch(c.eight, s));
      k += 8;
    } else if (!(k & 1) && k1 - k >= 4) {
      HIPCHK(hipGraphLaunch(c.four, s));
      k += 4;
    } else {
      HIPCHK(hipGraphLaunch(c.one[k & 1], s));
      ++k;
    }
  }
  return FDD_OK;
}

// L7 x = f (f from rhs), to ||f - L7 x|| <= tol ||f||; x is left in Q->x (padded FP64).  Mixed
// precision: runs of FP32 multigrid-PCG, each to a residual reduction of step_rtol, inside FP64
// iterative refinement (k3_ir: x += e, r = f - L7 x in FP64, the next run's right-hand side; the
// run that starts on a small enough r ends the solve at once); FP64: one run.  The runs and
// iterations of the last solve are enqueued before the state is first read back (a run cut
// short by the next refinement step leaves a valid, smaller correction; an iteration enqueued
// after its run stopped returns at once in every pass), then one iteration, or one more
// refinement step, at a time.
template <typename R>
int run_start(Problem3D* Q, Mg3<R>& M, hipStream_t s, bool refined, int iters) {
  const int nu = Q->nu;
  auto it = [&](int k) { iteration3<R>(Q, M, s, nu, k); };
  if (Q->use_graph && M.g_nu != nu) {
    if (M.g_init) (void)hipGraphExecDestroy(M.g_init);
    M.g_init = nullptr;
    int rc = capture(s, [&]() { vcycle3<R>(Q, M, s, nu, 1, 0, refined); }, &M.g_init);
    if (!rc) rc = capture_chunks(s, it, &M.g_it);
    if (rc) return rc;
    M.g_nu = nu;
  }
  HIPCHK(hipMemsetAsync(M.x, 0, sizeof(R) * vol(Q->nf), s));
  HIPCHK(hipMemsetAsync(Q->stop, 0, sizeof(int), s));
  if (Q->use_graph) HIPCHK(hipGraphLaunch(M.g_init, s));
  else vcycle3<R>(Q, M, s, nu, 1, 0, refined);
  Q->enq = iters;
  int rc = enqueue_iterations(s, Q->use_graph, M.g_it, it, 0, iters);
  if (rc) return rc;
  HIPCHK(hipGetLastError());
  return FDD_OK;
}

// refinement step after the first: x += e, r = F - L7 x, then a new FP32 run with `iters`
// iterations enqueued
int refine_step(Problem3D* Q, hipStream_t s, int iters) {
  k3_launch_ir(s, 0, Q->F64, Q->X64[Q->xcur], Q->m32.x, Q->X64[Q->xcur ^ 1], Q->m32.Rv[0], Q->nf,
               Q->rows0, Q->st, Q->part0);
  Q->xcur ^= 1;
  ++Q->steps;
  return run_start<float>(Q, Q->m32, s, true, iters);
}

int interior_start(fdd_problem_s* P, hipStream_t s, const Rhs3& rhs, double tol, int maxit,
                   int nu, bool mixed, double step_rtol) {
  Problem3D* Q = P->p3;
  const int nf = Q->nf;
  Q->mixed = mixed;
  Q->maxit = maxit;
  Q->nu = nu;
  State3& h = *Q->hst;
  h = State3{};
  h.tol2 = mixed ? step_rtol * step_rtol : tol * tol;
  h.tol2s = tol * tol;
  HIPCHK(hipMemcpyAsync(Q->st, Q->hst, sizeof(State3), hipMemcpyHostToDevice, s));
  if (!mixed) {
    k3_launch_rhs(s, rhs, Q->m64.Rv[0], nf);
    return run_start<double>(Q, Q->m64, s, false, std::min(std::max(Q->m64.pred - 1, 1), maxit));
  }
  k3_launch_rhs(s, rhs, Q->F64, nf);
  HIPCHK(hipMemsetAsync(Q->X64[0], 0, 8 * vol(nf), s));
  Q->xcur = 0;
  Q->steps = 0;
  k3_launch_ir(s, 1, Q->F64, nullptr, nullptr, nullptr, Q->m32.Rv[0], nf, Q->rows0, Q->st,
               Q->part0);
  // each run gets one iteration more than it took in the last solve, so that a run is rarely
  // cut short by the next step (which stays correct, but makes the iterates depend on history)
  auto budget = [&](int r) { return std::min(Q->run_pred[std::min(r, kRuns3 - 1)] + 1, maxit); };
  int rc = run_start<float>(Q, Q->m32, s, true, budget(0));
  // the further runs the last solve took, then the step expected to end the solve
  for (int r = 1; r < Q->runs_pred && !rc; ++r) rc = refine_step(Q, s, budget(r));
  if (!rc) rc = refine_step(Q, s, 0);
  return rc;
}

int interior_finish(fdd_problem_s* P, hipStream_t s, int* its) {
  Problem3D* Q = P->p3;
  constexpr int kMaxRefine = 12;
  int done = 0;
  while (true) {
    int rc = sync_state(Q, s);
    if (rc) return rc;
    const State3& h = *Q->hst;
    if (h.breakdown) break;
    if (*Q->hstop && (!Q->mixed || h.done)) {
      done = 1;
      break;
    }
    if (h.its_total >= Q->maxit) break;
    if (*Q->hstop) {
      // the last run stopped short of the solve's tolerance: one more refinement step
      if (Q->steps >= kMaxRefine) break;
      rc = refine_step(Q, s, std::min(Q->run_pred[std::min(Q->steps + 1, kRuns3 - 1)] + 1,
                                      Q->maxit - h.its_total));
      if (rc) return rc;
      continue;
    }
    auto it = [&](int k) {
      if (Q->mixed) iteration3<float>(Q, Q->m32, s, Q->nu, k);
      else iteration3<double>(Q, Q->m64, s, Q->nu, k);
    };
    rc = enqueue_iterations(s, Q->use_graph, Q->mixed ? Q->m32.g_it : Q->m64.g_it, it, Q->enq,
                            Q->enq + 1);
    if (rc) return rc;
    ++Q->enq;
    HIPCHK(hipGetLastError());
  }
  const State3& h = *Q->hst;
  if (Q->mixed) {
    // runs that iterated: every refinement step but the one that ended the solve
    if (done && h.its_total > 0) {
      Q->runs_pred = std::max(std::min(h.run, kRuns3), 1);
      for (int r = 0; r < Q->runs_pred; ++r) Q->run_pred[r] = std::max(h.run_its[r], 1);
    }
  } else if (done && h.its > 0) {
    Q->m64.pred = h.its;
  }
  Q->x = Q->mixed ? Q->X64[Q->xcur] : Q->m64.x;
  if (its) *its = h.its_total;
  if (h.breakdown)
    return fail(h.breakdown & 4 ? FDD_E_NONFINITE : FDD_E_BREAKDOWN,
                "3D interior solve: breakdown (flags %d)", h.breakdown);
  if (!done)
    return fail(FDD_NOT_CONVERGED, "3D interior solve: %d iterations, residual %.3e of %.3e",
                h.its_total, std::sqrt(h.rr), std::sqrt(h.F2));
  return FDD_OK;
}

int interior3(fdd_problem_s* P, hipStream_t s, const Rhs3& rhs, const fdd_opts& o, int* its) {
  int rc = interior_start(P, s, rhs, o.inner_rtol, o.inner_maxit, o.mg_nu,
                          o.precision == FDD_MIXED, o.step_rtol);
  return rc ? rc : interior_finish(P, s, its);
}

Shift3 table3(const fdd_ratpc_s* t) {
  Shift3 T{};
  const RaResult& r = t->r;
  if (t->which == FDD_RA_PRECOND) {
    T.m = r.m + 1;
    T.alpha[0] = 0.0;
    T.beta[0] = 1.0;
    T.coef[0] = r.c0;
    for (int k = 0; k < r.m; ++k) {
      T.alpha[k + 1] = 1.0;
      T.beta[k + 1] = r.p[k];
      T.coef[k + 1] = r.c[k];
    }
  } else {
    T.m = std::max(r.m, 1);
    T.alpha[0] = 1.0;
    T.beta[0] = 1.0;
    T.coef[0] = 0.0;
    for (int k = 0; k < r.m; ++k) {
      T.alpha[k] = 1.0;
      T.beta[k] = r.p[k];
      T.coef[k] = r.c[k];
    }
    T.d0 = r.c0;
  }
  return T;
}

// face-CG iteration k of a batch (both vector passes, then the preconditioner with the test)
void face_iteration(Problem3D* Q, FaceBufs& B, hipStream_t s, const Shift3* tab, int m,
                    double tol2, int k) {
  const int nf = Q->nf;
  const double h = 1.0 / Q->n;
  kf_launch_apply1(s, B.z, B.p[(k + 1) & 1], B.p[k & 1], B.q, nf, h, m, tab, B.cg, B.part0,
                   kf_tiles(nf), B.part1, B.done);
  kf_launch_face_update_prec(s, Q->S, B.r[k & 1], B.r[(k + 1) & 1], B.q, B.p[k & 1], B.y, B.t,
                             B.z, nf, Q->n, h, m, tab, B.cg, B.part1, tol2, B.part0, B.done);
}

// out = preconditioner (which 0) or H_RA (which 1) applied to `in` (face vectors).  The
// iterations of the last batch of the same kind are enqueued first (face_start), then the flags
// are read back and one iteration at a time is added until every system has converged
// (face_finish).
struct FaceRun {
  int which, m;
  double tol2;
  Shift3* tab;
};

int face_start(fdd_problem_s* P, hipStream_t s, const fdd_ratpc_s* T, const double* in,
               FaceRun* run) {
  Problem3D* Q = P->p3;
  const int nf = Q->nf;
  const double h = 1.0 / Q->n;
  const int which = T->which == FDD_RA_OPERATOR ? 1 : 0;
  const Shift3 tabh = table3(T);
  const int m = tabh.m;
  if (m > kMaxSys3) return fail(FDD_E_RA, "%d shifted systems exceed the batch limit %d", m, kMaxSys3);
  Q->htab[which] = tabh;
  Shift3* tab = Q->tabs + which;
  HIPCHK(hipMemcpyAsync(tab, Q->htab + which, sizeof(Shift3), hipMemcpyHostToDevice, s));
  const double tol = which ? kFaceTolH : kFaceTolP;
  const double tol2 = tol * tol;
  *run = FaceRun{which, m, tol2, tab};
  FaceBufs& B = Q->fb[which];
  auto it = [&](int k) { face_iteration(Q, B, s, tab, m, tol2, k); };
  if (Q->use_graph && Q->g_face_m[which] != m) {
    int rc = capture_chunks(s, it, &Q->g_face[which]);
    if (rc) return rc;
    Q->g_face_m[which] = m;
  }
  HIPCHK(hipMemsetAsync(B.done, 0, sizeof(int) * kMaxSys3, s));
  HIPCHK(hipMemsetAsync(B.cg, 0, sizeof(FaceCG), s));
  kf_launch_start(s, in, B.r[0], B.y, nf, h, m, which, B.part0);
  kf_launch_prec(s, Q->S, B.r[0], B.t, B.z, nf, Q->n, h, m, tab, B.cg, B.part0, tol2, 1, B.part0,
                 B.done);
  B.enq = std::max(Q->pred_face[which] - 1, 1);
  int rc = enqueue_iterations(s, Q->use_graph, Q->g_face[which], it, 0, B.enq);
  if (rc) return rc;
  HIPCHK(hipGetLastError());
  return FDD_OK;
}

int face_finish(fdd_problem_s* P, hipStream_t s, const FaceRun& run, const double* in,
                double* out) {
  Problem3D* Q = P->p3;
  const int nf = Q->nf, m = run.m, which = run.which;
  const double h = 1.0 / Q->n;
  FaceBufs& B = Q->fb[which];
  auto it = [&](int k) { face_iteration(Q, B, s, run.tab, m, run.tol2, k); };
  constexpr int kMaxFace = 400;
  bool all = false;
  while (true) {
    HIPCHK(hipMemcpyAsync(B.hdone, B.done, sizeof(int) * m, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(B.hits, B.cg->its, sizeof(int) * m, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    all = true;
    for (int k = 0; k < m; ++k) all = all && B.hdone[k];
    if (all || B.enq >= kMaxFace) break;
    int rc = enqueue_iterations(s, Q->use_graph, Q->g_face[which], it, B.enq, B.enq + 1);
    if (rc) return rc;
    ++B.enq;
    HIPCHK(hipGetLastError());
  }
  if (!all) return fail(FDD_NOT_CONVERGED, "3D face solves did not converge");
  int most = 1;
  for (int k = 0; k < m; ++k) most = std::max(most, B.hits[k]);
  Q->pred_face[which] = most;
  kf_launch_combine(s, B.y, m, nf, h, run.tab, which, in, B.tmp, out, Q->htab[which].d0);
  HIPCHK(hipGetLastError());
  return FDD_OK;
}

int face_batch(fdd_problem_s* P, hipStream_t s, const fdd_ratpc_s* T, const double* in,
               double* out) {
  FaceRun run{};
  int rc = face_start(P, s, T, in, &run);
  return rc ? rc : face_finish(P, s, run, in, out);
}

// a.b into the device scalar `slot` (partials summed on the device), also returned to the host
// (for the stop and breakdown tests)
double face_dot(Problem3D* Q, hipStream_t s, const double* a, const double* b, int slot, int* rc) {
  const int64_t N = (int64_t)Q->nf * Q->nf;
  kf_launch_vdot(s, a, b, N, Q->gpart);
  k3_launch_sum_partials(s, Q->gpart, kPart3, 1, Q->sc, slot);
  if (hipMemcpyAsync(Q->hpart, Q->sc, 8 * kSc3Count, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    *rc = fail(FDD_E_HIP, "device read-back failed");
    return 0.0;
  }
  return Q->hpart[slot];
}

// y = S p (Schur complement with H_RA); u = L7^{-1} lift(p) is left in Q->x
int schur3(fdd_problem_s* P, hipStream_t s, const fdd_ratpc_s* HT, const double* p, double* y,
           const fdd_opts& o, int* its, double* pq) {
  Problem3D* Q = P->p3;
  // the interior solve on s and the H batch on the second stream run at the same time
  if (!Q->s2) {
    HIPCHK(hipStreamCreateWithFlags(&Q->s2, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&Q->ev_fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&Q->ev_join, hipEventDisableTiming));
  }
  HIPCHK(hipEventRecord(Q->ev_fork, s));
  HIPCHK(hipStreamWaitEvent(Q->s2, Q->ev_fork, 0));
  const Rhs3 lift{nullptr, 0.0, p, 1.0};
  int rc = interior_start(P, s, lift, o.inner_rtol, o.inner_maxit, o.mg_nu,
                          o.precision == FDD_MIXED, o.step_rtol);
  FaceRun run{};
  if (!rc) rc = face_start(P, Q->s2, HT, p, &run);
  if (!rc) rc = interior_finish(P, s, its);
  if (!rc) rc = face_finish(P, Q->s2, run, p, Q->Hp);
  // join in every case, so that no work of the second stream outlives the call unordered
  (void)hipEventRecord(Q->ev_join, Q->s2);
  (void)hipStreamWaitEvent(s, Q->ev_join, 0);
  if (rc) return rc;
  kf_launch_schur(s, p, Q->x, Q->nf, 1.0 / Q->n, P->K, P->gamma, Q->Hp, y, Q->gpart);
  HIPCHK(hipGetLastError());
  if (pq) {
    // p.Sp summed on the device into the outer PCG's scalars; the host reads it for the test
    k3_launch_sum_partials(s, Q->gpart, kPart3, 1, Q->sc, kSc3Pq);
    HIPCHK(hipMemcpyAsync(Q->hpart, Q->sc, 8 * kSc3Count, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *pq = Q->hpart[kSc3Pq];
  }
  return FDD_OK;
}

// The 3D work runs on the problem's own stream (graphs cannot be captured on the legacy default
// stream), ordered after the caller's stream on entry and before it on exit.
struct LibStream {
  fdd_problem_s* P;
  hipStream_t user, s;
  int rc = FDD_OK;
  LibStream(fdd_problem_s* P_, hipStream_t us) : P(P_), user(us), s(us) {
    if (!P->gstream) {
      if (hipStreamCreateWithFlags(&P->gstream, hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&P->ev_in, hipEventDisableTiming) != hipSuccess ||
          hipEventCreateWithFlags(&P->ev_out, hipEventDisableTiming) != hipSuccess) {
        rc = fail(FDD_E_HIP, "stream creation failed");
        return;
      }
    }
    if (hipEventRecord(P->ev_in, us) != hipSuccess || hipStreamWaitEvent(P->gstream, P->ev_in, 0) != hipSuccess) {
      rc = fail(FDD_E_HIP, "stream ordering failed");
      return;
    }
    s = P->gstream;
  }
  ~LibStream() {
    if (s != user) {
      (void)hipEventRecord(P->ev_out, s);
      (void)hipStreamWaitEvent(user, P->ev_out, 0);
    }
  }
};

}  // namespace

namespace fdd {

int setup3(const fdd_desc* d, int hip_device, fdd_problem_s* P) {
  const int n = d->n;
  if (n < 4 || (n & 1) || n > 256)
    return fail(FDD_E_ARG, "3D: n must be even, 4 <= n <= 256 (got %d)", n);
  Problem3D* Q = new (std::nothrow) Problem3D();
  if (!Q) return fail(FDD_E_NOMEM, "out of host memory");
  Q->n = n;
  Q->nf = n - 1;
  int nf = n - 1, l = 0;
  while (true) {
    Q->lnf[l] = nf;
    // coarsest: 3^3 (dense inverse), or 1 below a finest level of 3^3
    if (!(nf & 1) || nf <= 1 || (nf <= 3 && l > 0)) break;
    nf = (nf - 1) / 2;
    if (++l >= kMaxLevels) {
      delete Q;
      return fail(FDD_E_ARG, "too many multigrid levels");
    }
  }
  Q->nlev = l + 1;
  Q->nc = Q->lnf[l];
  if (Q->nc > 4) {
    const int nc = Q->nc;
    delete Q;
    return fail(FDD_E_ARG, "3D: n = %d leaves a %d^3 coarsest grid (max 4^3)", n, nc);
  }
  // the coarse levels that fit one workgroup's LDS (level 0 always runs on the full grid)
  Q->lc = 1;
  while (Q->lc < Q->nlev && Q->lnf[Q->lc] > kCvcMax) ++Q->lc;
  Q->cvc.nl = Q->nlev - Q->lc;
  for (int k = 0; k < Q->cvc.nl && k < kCvcLevels; ++k) Q->cvc.lev[k] = Q->lnf[Q->lc + k];
  if (Q->lc >= Q->nlev || !k3_cvc_fits(Q->cvc)) {
    delete Q;
    return fail(FDD_E_ARG, "3D: n = %d: the coarse levels do not fit one workgroup", n);
  }
  Q->rows0 = k3_rows_red(Q->nf);
  Q->np0 = ((Q->nf + Q->rows0 - 1) / Q->rows0) * Q->nf;
  Q->cinv_h = dense_inverse_7pt(Q->nc);
  const int m = Q->nf;
  Q->S_h.resize((size_t)m * m);
  for (int a = 0; a < m; ++a)
    for (int b = 0; b < m; ++b)
      Q->S_h[(size_t)a * m + b] = std::sqrt(2.0 / n) * std::sin(M_PI * (a + 1) * (b + 1) / n);
  P->p3 = Q;
  P->dim = 3;
  P->n = n;
  P->device = hip_device;
  P->K = d->K;
  P->mu = d->mu;
  P->gamma = 1.0 / d->mu;
  P->h = 1.0 / n;
  P->N = (int64_t)m * m * n;
  P->NI = (int64_t)m * m * m;
  P->NG = (int64_t)m * m;
  // rigorous enclosure of the face spectrum: conforming P1 eigenvalues lie above the continuous
  // ones (2 pi^2 on the unit square), and the element bound gives at most 36 / h^2
  P->lam_lo = 2.0 * M_PI * M_PI;
  P->lam_hi = 36.0 * n * (double)n;
  return FDD_OK;
}

size_t workspace3(fdd_problem_s* P) {
  Problem3D tmp = *P->p3;
  fdd_problem_s pt = *P;
  pt.p3 = &tmp;
  return plan3(&pt, nullptr);
}

int bind3(fdd_problem_s* P, void* dev, size_t bytes, hipStream_t s) {
  Problem3D* Q = P->p3;
  const size_t need = workspace3(P);
  if (bytes < need) return fail(FDD_E_WORKSPACE, "workspace %zu bytes < %zu needed", bytes, need);
  HIPCHK(hipSetDevice(P->device));
  // captured graphs hold pointers into the old workspace: capture again on the next solve
  for (hipGraphExec_t* g : {&Q->m64.g_init, &Q->m32.g_init}) {
    if (*g) (void)hipGraphExecDestroy(*g);
    *g = nullptr;
  }
  Q->m64.g_it.clear();
  Q->m32.g_it.clear();
  Q->m64.g_nu = Q->m32.g_nu = 0;
  for (Chunks& c : Q->g_face) c.clear();
  Q->g_face_m[0] = Q->g_face_m[1] = 0;
  P->ws = (char*)dev;
  P->ws_bytes = bytes;
  plan3(P, P->ws);
  if (!Q->hst) {
    HIPCHK(hipHostMalloc((void**)&Q->hst, sizeof(State3), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&Q->hstop, sizeof(int), hipHostMallocDefault));
    for (FaceBufs& B : Q->fb) {
      HIPCHK(hipHostMalloc((void**)&B.hdone, sizeof(int) * kMaxSys3, hipHostMallocDefault));
      HIPCHK(hipHostMalloc((void**)&B.hits, sizeof(int) * kMaxSys3, hipHostMallocDefault));
    }
    HIPCHK(hipHostMalloc((void**)&Q->hpart, 8 * 2 * kPart3, hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&Q->htab, 2 * sizeof(Shift3), hipHostMallocDefault));
  }
  HIPCHK(hipMemsetAsync(P->ws, 0, need, s));
  HIPCHK(hipMemcpyAsync(Q->cinv, Q->cinv_h.data(), 8 * Q->cinv_h.size(), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(Q->S, Q->S_h.data(), 8 * Q->S_h.size(), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return FDD_OK;
}

void destroy3(fdd_problem_s* P) {
  Problem3D* Q = P->p3;
  if (!Q) return;
  for (void* h : {(void*)Q->hst, (void*)Q->hstop, (void*)Q->fb[0].hdone, (void*)Q->fb[0].hits,
                  (void*)Q->fb[1].hdone, (void*)Q->fb[1].hits, (void*)Q->hpart, (void*)Q->htab,
})
    if (h) (void)hipHostFree(h);
  for (hipGraphExec_t g : {Q->m64.g_init, Q->m32.g_init})
    if (g) (void)hipGraphExecDestroy(g);
  Q->m64.g_it.clear();
  Q->m32.g_it.clear();
  for (Chunks& c : Q->g_face) c.clear();
  if (Q->ev_fork) (void)hipEventDestroy(Q->ev_fork);
  if (Q->ev_join) (void)hipEventDestroy(Q->ev_join);
  if (Q->s2) (void)hipStreamDestroy(Q->s2);
  delete Q;
  P->p3 = nullptr;
}

int interior_solve3(fdd_problem_s* P, const double* f, double* u, const fdd_opts& o, hipStream_t us,
                    int* its) {
  Problem3D* Q = P->p3;
  LibStream ls(P, us);
  if (ls.rc) return ls.rc;
  const hipStream_t s = ls.s;
  Q->use_graph = o.use_graph != 0;
  // A_II u = f with A_II = h L7
  int rc = interior3(P, s, Rhs3{f, 1.0 / P->h, nullptr, 0.0}, o,
                     its);
  if (rc < 0) return rc;
  k3_launch_gather(s, Q->x, Q->nf, u, nullptr);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return rc;
}

int precond_apply3(fdd_problem_s* P, const fdd_ratpc_s* T, const double* r, double* z,
                   hipStream_t us) {
  LibStream ls(P, us);
  if (ls.rc) return ls.rc;
  return face_batch(P, ls.s, T, r, z);
}

int schur_apply3(fdd_problem_s* P, const fdd_ratpc_s* H, const double* x, double* y,
                 const fdd_opts& o, hipStream_t us) {
  LibStream ls(P, us);
  if (ls.rc) return ls.rc;
  const hipStream_t s = ls.s;
  P->p3->use_graph = o.use_graph != 0;
  int rc = schur3(P, s, H, x, y, o, nullptr, nullptr);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(s));
  return FDD_OK;
}

int apply_operator3(fdd_problem_s* P, const fdd_ratpc_s* H, const double* x, double* y,
                    hipStream_t us) {
  Problem3D* Q = P->p3;
  LibStream ls(P, us);
  if (ls.rc) return ls.rc;
  const hipStream_t s = ls.s;
  int rc = face_batch(P, s, H, x + P->NI, Q->Hp);
  if (rc) return rc;
  k3_launch_full_operator(s, P->n, P->K, P->gamma, x, Q->Hp, y, nullptr, nullptr);
  HIPCHK(hipGetLastError());
  return FDD_OK;
}

int solve3(fdd_problem_s* P, const fdd_ratpc_s* PT, const fdd_ratpc_s* HT, const double* b,
           double* x, const fdd_opts& o, hipStream_t us, fdd_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  Problem3D* Q = P->p3;
  LibStream ls(P, us);
  if (ls.rc) return ls.rc;
  const hipStream_t s = ls.s;
  Q->use_graph = o.use_graph != 0;
  fdd_stats st{};
  st.true_rel_res = -1.0;
  const int nf = Q->nf;
  const int64_t NG = P->NG;
  const double h = P->h;
  auto finish = [&](int code) {
    st.status = code;
    st.t_solve_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = st;
    return code;
  };
  auto inner = [&](const Rhs3& rhs) {
    int its = 0;
    int rc = interior3(P, s, rhs, o, &its);
    st.inner_solves += 1;
    st.inner_its_total += its;
    st.inner_its_max = std::max(st.inner_its_max, its);
    return rc;
  };
  // 1. g = b_G - A_GI A_II^{-1} b_I = b_G + h w|plane nf,  w = L7^{-1} (b_I / h)
  int rc = inner(Rhs3{b, 1.0 / h, nullptr, 0.0});
  if (rc) return finish(rc);
  kf_launch_rhs_reduce(s, b + P->NI, Q->x, nf, h, Q->rG, Q->xG);
  // x_I(0) = A_II^{-1} b_I / K (unless the back-substitution is solved at the end)
  if (!o.back_solve) k3_launch_scale_add(s, Q->xI, Q->x, 1.0 / P->K, 0, (int64_t)vol(nf));
  // 2. outer PCG from x_G = 0
  if ((rc = face_batch(P, s, PT, Q->rG, Q->zG))) return finish(rc);
  const double rho0 = face_dot(Q, s, Q->rG, Q->zG, kSc3Rz, &rc);
  if (rc) return finish(rc);
  k3_launch_outer_scalars(s, Q->sc, 0);
  if (!(rho0 >= 0.0)) return finish(fail(FDD_E_BREAKDOWN, "preconditioner not positive"));
  HIPCHK(hipMemcpyAsync(Q->pG, Q->zG, 8 * NG, hipMemcpyDeviceToDevice, s));
  double rho = rho0;
  bool conv = !(rho0 > 0.0);
  while (!conv && st.outer_its < o.outer_maxit) {
    double pq = 0.0;
    int its = 0;
    rc = schur3(P, s, HT, Q->pG, Q->yG, o, &its, &pq);
    st.inner_solves += 1;
    st.inner_its_total += its;
    st.inner_its_max = std::max(st.inner_its_max, its);
    if (rc) return finish(rc);
    if (!(pq > 0.0) || !std::isfinite(pq))
      return finish(fail(std::isfinite(pq) ? FDD_E_BREAKDOWN : FDD_E_NONFINITE,
                         "3D outer PCG breakdown (p.Sp = %g)", pq));
    // alpha = rho / p.Sp on the device, then x += alpha p, r -= alpha S p
    k3_launch_outer_scalars(s, Q->sc, 1);
    kf_launch_outer_axpy(s, Q->xG, Q->rG, Q->pG, Q->yG, nullptr, NG, Q->sc + kSc3Alpha);
    // x_I += alpha E p (Q->x holds E p = L7^{-1} lift(p) from the Schur product)
    if (!o.back_solve)
      k3_launch_scale_add(s, Q->xI, Q->x, 0.0, 1, (int64_t)vol(nf), Q->sc + kSc3Alpha);
    if ((rc = face_batch(P, s, PT, Q->rG, Q->zG))) return finish(rc);
    const double rho_new = face_dot(Q, s, Q->rG, Q->zG, kSc3Rz, &rc);
    if (rc) return finish(rc);
    ++st.outer_its;
    if (!(rho_new >= 0.0)) return finish(fail(FDD_E_BREAKDOWN, "3D outer r.z < 0"));
    conv = std::sqrt(rho_new) <= o.outer_rtol * std::sqrt(rho0);
    rho = rho_new;
    // beta = rho_new / rho and p = z + beta p on the device
    k3_launch_outer_scalars(s, Q->sc, 2);
    if (!conv) kf_launch_outer_axpy(s, nullptr, nullptr, Q->pG, nullptr, Q->zG, NG, Q->sc + kSc3Beta);
  }
  st.rel_precond_res = rho0 > 0 ? std::sqrt(std::max(rho, 0.0) / rho0) : 0.0;
  // 3. x_I = A_II^{-1} (b_I / K - A_IG x_G) = L7^{-1} (b_I / (K h) + lift(x_G)): accumulated
  //    during the outer PCG, or one more interior solve
  if (o.back_solve) {
    if ((rc = inner(Rhs3{b, 1.0 / (P->K * h), Q->xG, 1.0}))) return finish(rc);
    k3_launch_gather(s, Q->x, nf, x, Q->xG);
  } else {
    k3_launch_gather(s, Q->xI, nf, x, Q->xG);
  }
  if (o.check_true_residual) {
    if ((rc = face_batch(P, s, HT, x + P->NI, Q->Hp))) return finish(rc);
    k3_launch_full_operator(s, P->n, P->K, P->gamma, x, Q->Hp, nullptr, b, Q->gpart);
    k3_launch_sum_partials(s, Q->gpart, kPart3, 2, Q->sc, kSc3E2);
    k3_launch_sum_partials(s, Q->gpart + 1, kPart3, 2, Q->sc, kSc3B2);
    HIPCHK(hipMemcpyAsync(Q->hpart, Q->sc, 8 * kSc3Count, hipMemcpyDeviceToHost, s));
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  if (o.check_true_residual && Q->hpart[kSc3B2] > 0)
    st.true_rel_res = std::sqrt(Q->hpart[kSc3E2] / Q->hpart[kSc3B2]);
  return finish(conv ? FDD_OK : FDD_NOT_CONVERGED);
}

}  // namespace fdd
