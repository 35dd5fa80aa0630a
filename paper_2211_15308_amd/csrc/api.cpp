// C ABI of the solver (declared in include/fdd.h): problem set-up, workspace planning, and the
// host orchestration of the Schur-complement PCG (paper, Sec. 2) on top of the HIP kernels.
#include "fdd.h"

#include <chrono>
#include <cstdarg>
#include <type_traits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "fdd_internal.h"

using namespace fdd;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(call)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess) return fail(FDD_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
inline int round_up(int x, int a) { return (x + a - 1) / a * a; }

// Per-precision multigrid-PCG buffers of level 0 plus the hierarchy.
template <typename T>
struct PcgSet {
  T* x = nullptr;
  T* r[2] = {nullptr, nullptr};
  T* p[2] = {nullptr, nullptr};
  T* z = nullptr;
  T* q = nullptr;
  MGBuffers<T> mg{};
};

}  // namespace

struct fdd_problem_s {
  int dim = 2, n = 0, device = 0;
  double K = 1, mu = 1, gamma = 1, h = 1;
  int64_t N = 0, NI = 0, NG = 0;
  double lam_lo = 0, lam_hi = 0;
  int nlev = 0;
  int first_coarse32 = 1, first_coarse64 = 1;
  Level lev[kMaxLevels];
  std::vector<double> cinv;  // dense inverse on the coarsest level
  std::vector<double> eig;   // exact interface eigenvalues (2D), check points of the RA builder
  // workspace views
  char* ws = nullptr;
  size_t ws_bytes = 0;
  DevState* st = nullptr;
  double* partials = nullptr;
  float* cinv32 = nullptr;
  double* cinv64 = nullptr;
  PcgSet<float> s32;
  PcgSet<double> s64;
  double* u64[2] = {nullptr, nullptr};  // refinement accumulators
  double* xG[2] = {nullptr, nullptr};
  double* rG[2] = {nullptr, nullptr};
  double* pG[2] = {nullptr, nullptr};
  double* zG = nullptr;
  double* yG = nullptr;
  double* Hp = nullptr;
  double* scratchP = nullptr;
  double* scratchH = nullptr;
  DevState* host_st = nullptr;  // pinned copy
  // adaptive inner schedule
  int sched_steps = 3, sched_its = 6, sched_its64 = 12;
};

struct fdd_ratpc_s {
  int which = 0;
  const fdd_problem_s* prob = nullptr;
  int n = 0;
  double K = 0, mu = 0;
  RaResult r{};
};

namespace {

// Assign (or just size) every workspace view.  When base is null only the size is computed.
size_t plan_workspace(fdd_problem_s* P, char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    off = align_up(off, 256);
    char* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  };
  const Level& L0 = P->lev[0];
  const size_t v0 = (size_t)L0.nf * L0.pitch;
  P->st = (DevState*)take(sizeof(DevState));
  const int t0 = (L0.nf + kTile - 1) / kTile;
  P->partials = (double*)take(sizeof(double) * (size_t)std::max(t0 * t0, 4096) * 2);
  const int nfc = P->lev[P->nlev - 1].nf;
  P->cinv32 = (float*)take(sizeof(float) * (size_t)nfc * nfc * nfc * nfc);
  P->cinv64 = (double*)take(sizeof(double) * (size_t)nfc * nfc * nfc * nfc);
  auto pcg = [&](auto& S, size_t esz) {
    using T = std::remove_pointer_t<decltype(S.x)>;
    S.x = (T*)take(esz * v0);
    for (int k = 0; k < 2; ++k) S.r[k] = (T*)take(esz * v0);
    for (int k = 0; k < 2; ++k) S.p[k] = (T*)take(esz * v0);
    S.z = (T*)take(esz * v0);
    S.q = (T*)take(esz * v0);
    S.mg.u[0] = (T*)take(esz * v0);
    S.mg.e[0] = S.z;
    S.mg.f[0] = nullptr;
    for (int l = 1; l < P->nlev; ++l) {
      const size_t vl = (size_t)P->lev[l].nf * P->lev[l].pitch;
      S.mg.f[l] = (T*)take(esz * vl);
      S.mg.u[l] = (T*)take(esz * vl);
      S.mg.e[l] = (T*)take(esz * vl);
    }
  };
  pcg(P->s32, sizeof(float));
  pcg(P->s64, sizeof(double));
  for (int k = 0; k < 2; ++k) P->u64[k] = (double*)take(sizeof(double) * v0);
  const size_t g = sizeof(double) * (size_t)std::max<int64_t>(P->NG, 1);
  for (int k = 0; k < 2; ++k) P->xG[k] = (double*)take(g);
  for (int k = 0; k < 2; ++k) P->rG[k] = (double*)take(g);
  for (int k = 0; k < 2; ++k) P->pG[k] = (double*)take(g);
  P->zG = (double*)take(g);
  P->yG = (double*)take(g);
  P->Hp = (double*)take(g);
  P->scratchP = (double*)take(g * (kMaxPoles + 1));
  P->scratchH = (double*)take(g * (kMaxPoles + 1));
  return align_up(off, 256);
}

// exact inverse of the 5-point operator on an nf x nf grid (Gauss-Jordan with pivoting)
std::vector<double> dense_inverse_5pt(int nf) {
  const int np = nf * nf;
  std::vector<double> A((size_t)np * np, 0.0), X((size_t)np * np, 0.0);
  for (int j = 0; j < nf; ++j)
    for (int i = 0; i < nf; ++i) {
      const int r = j * nf + i;
      A[(size_t)r * np + r] = 4.0;
      if (i > 0) A[(size_t)r * np + r - 1] = -1.0;
      if (i < nf - 1) A[(size_t)r * np + r + 1] = -1.0;
      if (j > 0) A[(size_t)r * np + r - nf] = -1.0;
      if (j < nf - 1) A[(size_t)r * np + r + nf] = -1.0;
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
      const double f = A[(size_t)r * np + c];
      if (f == 0.0) continue;
      for (int k = 0; k < np; ++k) {
        A[(size_t)r * np + k] -= f * A[(size_t)c * np + k];
        X[(size_t)r * np + k] -= f * X[(size_t)c * np + k];
      }
    }
  }
  return X;
}

LaunchCtx make_ctx(const fdd_problem_s* P, hipStream_t s, int nu, bool fp64) {
  LaunchCtx c{};
  c.stream = s;
  c.nlev = P->nlev;
  c.first_coarse = fp64 ? P->first_coarse64 : P->first_coarse32;
  for (int l = 0; l < P->nlev; ++l) c.lev[l] = P->lev[l];
  c.nu = nu;
  c.coarse_inv = P->cinv32;
  c.coarse_inv64 = P->cinv64;
  c.st = P->st;
  c.partials = P->partials;
  return c;
}

ShiftTable make_table(const fdd_ratpc_s* t) {
  ShiftTable T{};
  const RaResult& r = t->r;
  if (t->which == FDD_RA_PRECOND) {
    T.m = r.m + 1;
    T.alpha[0] = 0.0;  // c0 M^{-1}
    T.beta[0] = 1.0;
    T.coef[0] = r.c0;
    for (int k = 0; k < r.m; ++k) {
      T.alpha[k + 1] = 1.0;
      T.beta[k + 1] = r.p[k];
      T.coef[k + 1] = r.c[k];
    }
    T.d0 = 0.0;
  } else {
    T.m = std::max(r.m, 1);
    T.alpha[0] = 0.0;
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

struct InnerState {
  int cur_r = 0, cur_p = 0;  // ping-pong parities of the level-0 PCG
};

bool opts_ok(const fdd_opts* o) {
  return o && o->outer_rtol > 0 && o->inner_rtol > 0 && o->outer_maxit > 0 &&
         o->inner_maxit > 0 && (o->precision == FDD_MIXED || o->precision == FDD_FP64) &&
         (o->mg_nu == 1 || o->mg_nu == 2) && o->inner_chunk > 0 && o->warmstart == nullptr &&
         o->use_graph == 0;
}

constexpr double kTau32 = 1e-5;  // FP32 PCG relative reduction per refinement step

// Enqueue `steps` refinement steps (mixed) or `its` PCG iterations (FP64) of an interior solve.
void enqueue_inner_mixed(fdd_problem_s* P, const LaunchCtx& c, const RhsDesc& f, InnerState& s,
                         int steps, int its) {
  auto& S = P->s32;
  for (int st = 0; st < steps; ++st) {
    launch_pcg_init<float>(c, S.mg, S.r[s.cur_r], S.z);
    for (int k = 0; k < its; ++k) {
      launch_pcg_iteration<float>(c, S.mg, S.x, S.r[s.cur_r], S.r[s.cur_r ^ 1], S.z,
                                  S.p[s.cur_p], S.p[s.cur_p ^ 1], S.q);
      s.cur_r ^= 1;
      s.cur_p ^= 1;
    }
    launch_ir_residual(c, f, P->u64[0], P->u64[1], S.x, nullptr, P->u64[0], P->u64[1],
                       S.r[s.cur_r], nullptr, 0, 0, 0, 0);
  }
}

int read_state(fdd_problem_s* P, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(P->host_st, P->st, sizeof(DevState), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return FDD_OK;
}

// A complete interior solve A_II u = f: enqueue the predicted schedule, synchronize, top up
// until converged.  On return the solution is in the buffers given by inner_result().
int interior_solve(fdd_problem_s* P, hipStream_t s, const RhsDesc& f, const fdd_opts& o,
                   int* its_out, int* steps_out) {
  const bool fp64 = (o.precision == FDD_FP64);
  LaunchCtx c = make_ctx(P, s, o.mg_nu, fp64);
  InnerState is;
  const double tol2 = o.inner_rtol * o.inner_rtol;
  if (!fp64) {
    launch_ir_residual(c, f, P->u64[0], P->u64[1], nullptr, nullptr, P->u64[0], P->u64[1],
                       P->s32.r[is.cur_r], nullptr, 1, tol2, kTau32 * kTau32, 0);
    int steps = P->sched_steps, its = std::max(P->sched_its, 1);
    int total_its_sched = 0;
    for (int round = 0;; ++round) {
      enqueue_inner_mixed(P, c, f, is, steps, its);
      total_its_sched += steps * its;
      int rc = read_state(P, s);
      if (rc) return rc;
      const DevState& h = *P->host_st;
      if (h.breakdown) return fail(h.breakdown & 4 ? FDD_E_NONFINITE : FDD_E_BREAKDOWN,
                                   "interior solve: breakdown flags %d", h.breakdown);
      if (h.solve_done) {
        if (its_out) *its_out = h.inner_its;
        if (steps_out) *steps_out = h.refine_steps;
        // adapt the schedule to what this solve needed
        if (round == 0 && h.refine_steps > 0) {
          P->sched_steps = h.refine_steps;
          P->sched_its = std::max(1, (h.inner_its + h.refine_steps - 1) / h.refine_steps);
        }
        return FDD_OK;
      }
      if (h.inner_its >= o.inner_maxit || total_its_sched > 4 * o.inner_maxit) {
        if (its_out) *its_out = h.inner_its;
        return fail(FDD_NOT_CONVERGED, "interior solve: %d iterations, residual %.3e of %.3e",
                    h.inner_its, std::sqrt(h.res2), std::sqrt(h.ff));
      }
      // not yet: one more step at a time, with a longer PCG run
      P->sched_steps = std::max(P->sched_steps, h.refine_steps + 1);
      steps = 1;
      its = std::max(its, 2 * P->sched_its);
    }
  } else {
    auto& S = P->s64;
    launch_ir_residual(c, f, P->u64[0], P->u64[1], nullptr, nullptr, P->u64[0], P->u64[1],
                       nullptr, S.r[is.cur_r], 1, tol2, tol2, 1);
    launch_pcg_init<double>(c, S.mg, S.r[is.cur_r], S.z);
    int its = std::max(P->sched_its64, 1);
    for (int round = 0;; ++round) {
      for (int k = 0; k < its; ++k) {
        launch_pcg_iteration<double>(c, S.mg, S.x, S.r[is.cur_r], S.r[is.cur_r ^ 1], S.z,
                                     S.p[is.cur_p], S.p[is.cur_p ^ 1], S.q);
        is.cur_r ^= 1;
        is.cur_p ^= 1;
      }
      int rc = read_state(P, s);
      if (rc) return rc;
      const DevState& h = *P->host_st;
      if (h.breakdown) return fail(h.breakdown & 4 ? FDD_E_NONFINITE : FDD_E_BREAKDOWN,
                                   "interior solve: breakdown flags %d", h.breakdown);
      if (h.solve_done) {
        if (its_out) *its_out = h.inner_its;
        if (steps_out) *steps_out = 0;
        if (round == 0) P->sched_its64 = std::max(1, h.inner_its);
        return FDD_OK;
      }
      if (h.inner_its >= o.inner_maxit) {
        if (its_out) *its_out = h.inner_its;
        return fail(FDD_NOT_CONVERGED, "interior solve (fp64): %d iterations", h.inner_its);
      }
      its = std::max(2, P->sched_its64 / 2);
      P->sched_its64 += its;
    }
  }
}

// where the last interior solution lives
void inner_result(const fdd_problem_s* P, const fdd_opts& o, const double** u0, const double** u1,
                  const int** sel) {
  if (o.precision == FDD_FP64) {
    *u0 = *u1 = P->s64.x;
    *sel = nullptr;
  } else {
    *u0 = P->u64[0];
    *u1 = P->u64[1];
    *sel = &P->st->refine_steps;
  }
}

int check_problem(fdd_problem_s* P) {
  if (!P) return fail(FDD_E_ARG, "null problem");
  if (!P->ws) return fail(FDD_E_WORKSPACE, "no workspace bound");
  return FDD_OK;
}

int check_table(const fdd_problem_s* P, const fdd_ratpc_s* t, int which) {
  if (!t) return fail(FDD_E_ARG, "null rational table");
  if (t->which != which) return fail(FDD_E_STATE, "rational table of the wrong kind");
  if (t->n != P->n || (which == FDD_RA_PRECOND && (t->K != P->K || t->mu != P->mu)))
    return fail(FDD_E_STATE, "rational table built for another problem");
  return FDD_OK;
}

}  // namespace

extern "C" {

void fdd_opts_default(fdd_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->outer_rtol = 1e-8;
  o->outer_maxit = 200;
  o->inner_rtol = 1e-10;
  o->inner_maxit = 400;
  o->precision = FDD_MIXED;
  o->mg_nu = 1;
  o->inner_chunk = 6;
  o->check_true_residual = 0;
  o->warmstart = nullptr;
  o->use_graph = 0;
}

const char* fdd_last_error(void) { return g_err.c_str(); }
const char* fdd_version(void) { return "fdd 0.1 (gfx950)"; }

int fdd_setup_mesh(const fdd_desc* d, int hip_device, fdd_problem* out) {
  if (!d || !out) return fail(FDD_E_ARG, "null argument");
  *out = nullptr;
  if (d->dim != 2) return fail(FDD_E_ARG, "dim must be 2 (got %d)", d->dim);
  // the interface kernels hold one Gamma vector per workgroup in LDS: n - 1 <= 2047
  if (d->n < 4 || (d->n & 1) || d->n > 2048)
    return fail(FDD_E_ARG, "n must be even, 4 <= n <= 2048 (got %d)", d->n);
  if (!(d->K > 0) || !std::isfinite(d->K) || !(d->mu > 0) || !std::isfinite(d->mu))
    return fail(FDD_E_ARG, "K and mu must be positive and finite");
  fdd_problem_s* P = new (std::nothrow) fdd_problem_s();
  if (!P) return fail(FDD_E_NOMEM, "out of host memory");
  P->dim = 2;
  P->n = d->n;
  P->device = hip_device;
  P->K = d->K;
  P->mu = d->mu;
  P->gamma = 1.0 / d->mu;
  P->h = 1.0 / d->n;
  const int n = d->n;
  P->N = (int64_t)n * (n - 1);
  P->NI = (int64_t)(n - 1) * (n - 1);
  P->NG = n - 1;
  // multigrid hierarchy: halve while the point count is odd; the coarsest level is the first
  // below the finest with <= 7 points per side or an even count
  int nf = n - 1, l = 0;
  while (true) {
    if (l >= kMaxLevels) {
      delete P;
      return fail(FDD_E_ARG, "too many multigrid levels");
    }
    P->lev[l].nf = nf;
    P->lev[l].pitch = round_up(nf, 64);
    if (l >= 1 && (nf <= 7 || !(nf & 1))) break;
    nf = (nf - 1) / 2;
    ++l;
  }
  P->nlev = l + 1;
  const int nfc = P->lev[P->nlev - 1].nf;
  if (nfc > kMaxCoarsestNf) {
    delete P;
    return fail(FDD_E_ARG, "n = %d leaves a %d x %d coarsest grid (max %d)", n, nfc, nfc,
                kMaxCoarsestNf);
  }
  P->first_coarse32 = P->nlev - 1;
  P->first_coarse64 = P->nlev - 1;
  for (int k = P->nlev - 1; k >= 1; --k) {
    if (P->lev[k].nf <= 63) P->first_coarse32 = k;
    if (P->lev[k].nf <= 31) P->first_coarse64 = k;
  }
  P->cinv = dense_inverse_5pt(nfc);
  // exact interface spectrum (1D P1, Dirichlet ends): lambda_q = 6 (1 - cos t) / (h^2 (2 + cos t))
  P->eig.resize(n - 1);
  for (int q = 1; q < n; ++q) {
    const double t = q * M_PI / n;
    P->eig[q - 1] = 6.0 * (1.0 - std::cos(t)) / (P->h * P->h * (2.0 + std::cos(t)));
  }
  P->lam_lo = P->eig.front();
  P->lam_hi = P->eig.back();
  *out = P;
  return FDD_OK;
}

int fdd_problem_info(fdd_problem P, int64_t* N, int64_t* NI, int64_t* NG, double* lo, double* hi) {
  if (!P) return fail(FDD_E_ARG, "null problem");
  if (N) *N = P->N;
  if (NI) *NI = P->NI;
  if (NG) *NG = P->NG;
  if (lo) *lo = P->lam_lo;
  if (hi) *hi = P->lam_hi;
  return FDD_OK;
}

int fdd_workspace_bytes(fdd_problem P, const fdd_opts* o, size_t* bytes) {
  (void)o;
  if (!P || !bytes) return fail(FDD_E_ARG, "null argument");
  fdd_problem_s tmp = *P;
  *bytes = plan_workspace(&tmp, nullptr);
  return FDD_OK;
}

int fdd_bind_workspace(fdd_problem P, void* dev, size_t bytes, void* stream) {
  if (!P || !dev) return fail(FDD_E_ARG, "null argument");
  if (((uintptr_t)dev) & 255) return fail(FDD_E_WORKSPACE, "workspace must be 256-byte aligned");
  fdd_problem_s tmp = *P;
  const size_t need = plan_workspace(&tmp, nullptr);
  if (bytes < need) return fail(FDD_E_WORKSPACE, "workspace %zu bytes < %zu needed", bytes, need);
  HIPCHK(hipSetDevice(P->device));
  hipStream_t s = (hipStream_t)stream;
  P->ws = (char*)dev;
  P->ws_bytes = bytes;
  plan_workspace(P, P->ws);
  if (!P->host_st) HIPCHK(hipHostMalloc((void**)&P->host_st, sizeof(DevState), hipHostMallocDefault));
  HIPCHK(hipMemsetAsync(P->ws, 0, need, s));
  const size_t np = P->cinv.size();
  std::vector<float> c32(np);
  for (size_t k = 0; k < np; ++k) c32[k] = (float)P->cinv[k];
  HIPCHK(hipMemcpyAsync(P->cinv64, P->cinv.data(), np * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(P->cinv32, c32.data(), np * sizeof(float), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return FDD_OK;
}

int fdd_build_rational_pc(fdd_problem P, int which, double tol, int max_poles, fdd_ratpc* out) {
  if (!P || !out) return fail(FDD_E_ARG, "null argument");
  *out = nullptr;
  if (which != FDD_RA_PRECOND && which != FDD_RA_OPERATOR) return fail(FDD_E_ARG, "bad kind");
  if (!(tol > 0) || tol >= 1) return fail(FDD_E_ARG, "tol must be in (0, 1)");
  if (max_poles < 1 || max_poles > kMaxPoles)
    return fail(FDD_E_ARG, "max_poles must be in [1, %d]", kMaxPoles);
  RaResult r = build_rational(which, P->K, P->gamma, P->lam_lo, P->lam_hi, P->eig.data(),
                              (int)P->eig.size(), tol, max_poles);
  if (r.status != 0)
    return fail(FDD_E_RA, "no admissible rational approximation: best error %.3e > %.3e",
                r.max_rel_err, 10 * tol);
  fdd_ratpc_s* t = new (std::nothrow) fdd_ratpc_s();
  if (!t) return fail(FDD_E_NOMEM, "out of host memory");
  t->which = which;
  t->prob = P;
  t->n = P->n;
  t->K = P->K;
  t->mu = P->mu;
  t->r = r;
  *out = t;
  return FDD_OK;
}

int fdd_ratpc_from_table(fdd_problem P, int which, int m, double c0, const double* c,
                         const double* p, fdd_ratpc* out) {
  if (!P || !out || (m > 0 && (!c || !p))) return fail(FDD_E_ARG, "null argument");
  *out = nullptr;
  if (which != FDD_RA_PRECOND && which != FDD_RA_OPERATOR) return fail(FDD_E_ARG, "bad kind");
  if (m < 0 || m > kMaxPoles) return fail(FDD_E_ARG, "m must be in [0, %d]", kMaxPoles);
  if (!std::isfinite(c0)) return fail(FDD_E_RA, "non-finite c0");
  for (int k = 0; k < m; ++k) {
    if (!std::isfinite(c[k]) || !std::isfinite(p[k])) return fail(FDD_E_RA, "non-finite entry");
    if (p[k] < 0) return fail(FDD_E_RA, "shift p[%d] = %g < 0 makes L + p M indefinite", k, p[k]);
  }
  fdd_ratpc_s* t = new (std::nothrow) fdd_ratpc_s();
  if (!t) return fail(FDD_E_NOMEM, "out of host memory");
  t->which = which;
  t->prob = P;
  t->n = P->n;
  t->K = P->K;
  t->mu = P->mu;
  t->r.status = 0;
  t->r.c0 = c0;
  t->r.m = m;
  for (int k = 0; k < m; ++k) {
    t->r.c[k] = c[k];
    t->r.p[k] = p[k];
  }
  t->r.max_rel_err = ra_eval_rel_err(which, P->K, P->gamma, t->r, P->eig.data(), (int)P->eig.size());
  *out = t;
  return FDD_OK;
}

int fdd_ratpc_query(fdd_ratpc t, int* m, double* c0, double* c, double* p, double* err) {
  if (!t) return fail(FDD_E_ARG, "null table");
  if (m) *m = t->r.m;
  if (c0) *c0 = t->r.c0;
  for (int k = 0; k < t->r.m; ++k) {
    if (c) c[k] = t->r.c[k];
    if (p) p[k] = t->r.p[k];
  }
  if (err) *err = t->r.max_rel_err;
  return FDD_OK;
}

int fdd_interior_solve(fdd_problem P, const double* f, double* u, const fdd_opts* opts,
                       void* stream, int* its) {
  int rc = check_problem(P);
  if (rc) return rc;
  if (!f || !u) return fail(FDD_E_ARG, "null vector");
  fdd_opts o;
  if (opts) o = *opts;
  else fdd_opts_default(&o);
  if (!opts_ok(&o)) return fail(FDD_E_ARG, "invalid options");
  HIPCHK(hipSetDevice(P->device));
  hipStream_t s = (hipStream_t)stream;
  RhsDesc rd{f, 1.0, nullptr, 0.0};
  rc = interior_solve(P, s, rd, o, its, nullptr);
  if (rc < 0) return rc;
  const double *u0, *u1;
  const int* sel;
  inner_result(P, o, &u0, &u1, &sel);
  launch_scatter(s, (int)P->NG, P->lev[0].pitch, u0, u1, sel, nullptr, u);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return rc;
}

int fdd_precond_apply(fdd_problem P, fdd_ratpc T, const double* r, double* z, void* stream) {
  int rc = check_problem(P);
  if (rc) return rc;
  if ((rc = check_table(P, T, FDD_RA_PRECOND))) return rc;
  if (!r || !z) return fail(FDD_E_ARG, "null vector");
  HIPCHK(hipSetDevice(P->device));
  ShiftTable tab = make_table(T);
  launch_iface_batch((hipStream_t)stream, (int)P->NG, P->h, tab, kIfacePrecond, r, z, P->scratchP,
                     P->st, nullptr, nullptr, 0, 0);
  HIPCHK(hipGetLastError());
  return FDD_OK;
}

int fdd_schur_apply(fdd_problem P, fdd_ratpc H, const double* x, double* y, const fdd_opts* opts,
                    void* stream) {
  int rc = check_problem(P);
  if (rc) return rc;
  if ((rc = check_table(P, H, FDD_RA_OPERATOR))) return rc;
  if (!x || !y) return fail(FDD_E_ARG, "null vector");
  fdd_opts o;
  if (opts) o = *opts;
  else fdd_opts_default(&o);
  if (!opts_ok(&o)) return fail(FDD_E_ARG, "invalid options");
  HIPCHK(hipSetDevice(P->device));
  hipStream_t s = (hipStream_t)stream;
  RhsDesc rd{nullptr, 0.0, x, 1.0};
  rc = interior_solve(P, s, rd, o, nullptr, nullptr);
  if (rc) return rc;
  ShiftTable tab = make_table(H);
  launch_iface_batch(s, (int)P->NG, P->h, tab, kIfaceOperator, x, P->Hp, P->scratchH, P->st,
                     nullptr, nullptr, 0, 0);
  const double *u0, *u1;
  const int* sel;
  inner_result(P, o, &u0, &u1, &sel);
  launch_schur_gather(s, (int)P->NG, P->lev[0].nf, P->lev[0].pitch, P->K, P->gamma, x, u0, u1,
                      sel, P->Hp, y, nullptr, nullptr, nullptr, nullptr, P->st, 0, 0);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return FDD_OK;
}

int fdd_apply_operator(fdd_problem P, fdd_ratpc H, const double* x, double* y, void* stream) {
  int rc = check_problem(P);
  if (rc) return rc;
  if ((rc = check_table(P, H, FDD_RA_OPERATOR))) return rc;
  if (!x || !y) return fail(FDD_E_ARG, "null vector");
  HIPCHK(hipSetDevice(P->device));
  hipStream_t s = (hipStream_t)stream;
  ShiftTable tab = make_table(H);
  launch_iface_batch(s, (int)P->NG, P->h, tab, kIfaceOperator, x + P->NI, P->Hp, P->scratchH,
                     P->st, nullptr, nullptr, 0, 0);
  launch_full_operator(s, P->n, P->K, P->gamma, x, P->Hp, y, nullptr, P->partials,
                       &P->st->counters[9], P->st->t_res);
  HIPCHK(hipGetLastError());
  return FDD_OK;
}

int fdd_solve(fdd_problem P, fdd_ratpc PT, fdd_ratpc HT, const double* b, double* x,
              const fdd_opts* opts, void* stream, fdd_stats* stats) {
  const auto t_start = std::chrono::steady_clock::now();
  fdd_stats st{};
  st.true_rel_res = -1.0;
  int rc = check_problem(P);
  if (rc) return rc;
  if ((rc = check_table(P, PT, FDD_RA_PRECOND))) return rc;
  if ((rc = check_table(P, HT, FDD_RA_OPERATOR))) return rc;
  if (!b || !x) return fail(FDD_E_ARG, "null vector");
  fdd_opts o;
  if (opts) o = *opts;
  else fdd_opts_default(&o);
  if (!opts_ok(&o)) return fail(FDD_E_ARG, "invalid options");
  HIPCHK(hipSetDevice(P->device));
  hipStream_t s = (hipStream_t)stream;
  const int ng = (int)P->NG, nf = P->lev[0].nf, pitch = P->lev[0].pitch;
  const ShiftTable tabP = make_table(PT), tabH = make_table(HT);
  const double *u0, *u1;
  const int* sel;
  inner_result(P, o, &u0, &u1, &sel);
  auto inner = [&](const RhsDesc& f) -> int {
    int its = 0, steps = 0;
    int r = interior_solve(P, s, f, o, &its, &steps);
    st.inner_solves += 1;
    st.inner_its_total += its;
    st.inner_its_max = std::max(st.inner_its_max, its);
    st.refine_steps += steps;
    return r;
  };
  auto finish = [&](int code) -> int {
    st.status = code;
    st.t_solve_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    if (stats) *stats = st;
    return code;
  };
  // 1. g = b_G - A_GI A_II^{-1} b_I
  rc = inner(RhsDesc{b, 1.0, nullptr, 0.0});
  if (rc) return finish(rc);
  launch_rhs_reduce(s, ng, pitch, b + P->NI, u0, u1, sel, P->rG[0], P->xG[0]);
  // 2. outer PCG from x_G = 0: z = P r, rho0 = r.z, p = z
  launch_iface_batch(s, ng, P->h, tabP, kIfacePrecondOuter, P->rG[0], P->zG, P->scratchP, P->st,
                     nullptr, P->pG[0], 0, 1);
  HIPCHK(hipGetLastError());
  if ((rc = read_state(P, s))) return finish(rc);
  const double rho0 = P->host_st->o_rho0;
  if (P->host_st->breakdown) return finish(fail(FDD_E_BREAKDOWN, "preconditioner not positive"));
  int v = 0;
  double rho = rho0;
  bool converged = !(rho0 > 0.0);
  while (!converged && st.outer_its < o.outer_maxit) {
    const int a = v & 1, bnx = (v + 1) & 1;
    // interior solve for the lifted p, then H p, then the Schur product and the x/r updates
    rc = inner(RhsDesc{nullptr, 0.0, P->pG[a], 1.0});
    if (rc) return finish(rc);
    launch_iface_batch(s, ng, P->h, tabH, kIfaceOperator, P->pG[a], P->Hp, P->scratchH, P->st,
                       nullptr, nullptr, 0, 0);
    launch_schur_gather(s, ng, nf, pitch, P->K, P->gamma, P->pG[a], u0, u1, sel, P->Hp, P->yG,
                        P->xG[a], P->xG[bnx], P->rG[a], P->rG[bnx], P->st, 1, v);
    launch_iface_batch(s, ng, P->h, tabP, kIfacePrecondOuter, P->rG[bnx], P->zG, P->scratchP,
                       P->st, P->pG[a], P->pG[bnx], v, 0);
    HIPCHK(hipGetLastError());
    if ((rc = read_state(P, s))) return finish(rc);
    const DevState& h = *P->host_st;
    if (h.breakdown)
      return finish(fail(h.breakdown & 4 ? FDD_E_NONFINITE : FDD_E_BREAKDOWN,
                         "outer PCG breakdown (flags %d, p.Sp = %g)", h.breakdown, h.o_pq));
    ++v;
    ++st.outer_its;
    rho = h.o_rho[v & 1];
    if (!(rho >= 0.0)) return finish(fail(FDD_E_BREAKDOWN, "outer r.z < 0"));
    converged = std::sqrt(rho) <= o.outer_rtol * std::sqrt(rho0);
  }
  st.rel_precond_res = rho0 > 0 ? std::sqrt(std::max(rho, 0.0) / rho0) : 0.0;
  // 3. back-substitution x_I = A_II^{-1} (b_I / K - A_IG x_G)
  rc = inner(RhsDesc{b, 1.0 / P->K, P->xG[v & 1], 1.0});
  if (rc) return finish(rc);
  launch_scatter(s, nf, pitch, u0, u1, sel, P->xG[v & 1], x);
  if (o.check_true_residual) {
    launch_iface_batch(s, ng, P->h, tabH, kIfaceOperator, x + P->NI, P->Hp, P->scratchH, P->st,
                       nullptr, nullptr, 0, 0);
    launch_full_operator(s, P->n, P->K, P->gamma, x, P->Hp, nullptr, b, P->partials,
                         &P->st->counters[9], P->st->t_res);
  }
  HIPCHK(hipGetLastError());
  if ((rc = read_state(P, s))) return finish(rc);
  if (o.check_true_residual && P->host_st->t_res[1] > 0)
    st.true_rel_res = std::sqrt(P->host_st->t_res[0] / P->host_st->t_res[1]);
  return finish(converged ? FDD_OK : FDD_NOT_CONVERGED);
}

void fdd_destroy_problem(fdd_problem P) {
  if (!P) return;
  if (P->host_st) (void)hipHostFree(P->host_st);
  delete P;
}

void fdd_destroy_ratpc(fdd_ratpc t) { delete t; }

}  // extern "C"
