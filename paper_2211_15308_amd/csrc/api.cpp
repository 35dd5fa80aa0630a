// C ABI of the solver (declared in include/fdd.h): problem set-up, workspace planning, and the
// host orchestration of the Schur-complement PCG (paper, Sec. 2) on top of the HIP kernels.
#include "fdd.h"

#include <chrono>
#include <cstdarg>
#include <type_traits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <tuple>
#include <string>
#include <vector>

#include "api_internal.h"

using namespace fdd;

namespace fdd {

namespace {
thread_local std::string g_err;
}

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

}  // namespace fdd

namespace fdd {

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
  const size_t nb0 = (size_t)t0 * t0;
  P->partials = (double*)take(sizeof(double) * 4096 * 2);
  P->red.nb0 = (int)nb0;
  P->red.nbd = (int)nb0;
  P->red.pq = (double*)take(sizeof(double) * nb0);
  P->red.rr = (double*)take(sizeof(double) * nb0);
  P->red.rz[0] = (double*)take(sizeof(double) * nb0);
  P->red.rz[1] = (double*)take(sizeof(double) * nb0);
  P->red.zw[0] = (double*)take(sizeof(double) * nb0);
  P->red.zw[1] = (double*)take(sizeof(double) * nb0);
  P->red.ir = (double*)take(sizeof(double) * nb0);
  P->red.ff = (double*)take(sizeof(double) * nb0);
  const int nfc = P->lev[P->nlev - 1].nf;
  P->dstS = (float*)take(sizeof(float) * kDstN * kDstN);
  P->dstL = (float*)take(sizeof(float) * kDstN);
  P->cinv64 = (double*)take(sizeof(double) * (size_t)nfc * nfc * nfc * nfc);
  auto pcg = [&](auto& S, size_t esz) {
    using T = std::remove_pointer_t<decltype(S.x)>;
    S.x = (T*)take(esz * v0);
    for (int k = 0; k < 2; ++k) S.r[k] = (T*)take(esz * v0);
    for (int k = 0; k < 2; ++k) S.p[k] = (T*)take(esz * v0);
    S.z = (T*)take(esz * v0);
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
  for (int k = 0; k < 2; ++k) P->xI[k] = (double*)take(sizeof(double) * v0);
  const size_t g = sizeof(double) * (size_t)std::max<int64_t>(P->NG, 1);
  for (int k = 0; k < 2; ++k) P->xG[k] = (double*)take(g);
  for (int k = 0; k < 2; ++k) P->rG[k] = (double*)take(g);
  for (int k = 0; k < 2; ++k) P->pG[k] = (double*)take(g);
  P->zG = (double*)take(g);
  P->yG = (double*)take(g);
  P->Hp = (double*)take(g);
  P->lk_lmu = (double*)take(2 * sizeof(double));
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
  c.hook = P->hook.kind != kTimeNone ? const_cast<EventHook*>(&P->hook) : nullptr;
  c.stream = s;
  c.nlev = P->nlev;
  c.first_coarse = fp64 ? P->first_coarse64 : P->first_coarse32;
  for (int l = 0; l < P->nlev; ++l) c.lev[l] = P->lev[l];
  c.nu = nu;
  c.dst_S = P->dstS;
  c.dst_lam = P->dstL;
  c.coarse_inv64 = P->cinv64;
  c.st = P->st;
  c.red = P->red;
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
      T.beta[k + 1] = t->shift0 + r.p[k];  // L + p_k M = A_G + (shift0 + p_k) M_G
      T.coef[k + 1] = r.c[k];
    }
    T.d0 = 0.0;
  } else {
    T.m = std::max(r.m, 1);
    T.alpha[0] = 0.0;
    T.beta[0] = 1.0;
    T.coef[0] = 0.0;
    double csum = 0.0;
    for (int k = 0; k < r.m; ++k) {
      T.alpha[k] = 1.0;
      T.beta[k] = t->shift0 + r.p[k];
      T.coef[k] = r.c[k];
      csum += r.c[k];
    }
    T.d0 = r.c0;
    if (t->lam_factor) {
      // the table approximates lam^(t-1); lam^t = c0 lam + sum_k c_k - sum_k c_k p_k / (lam + p_k)
      T.dL = r.c0;
      T.d0 = csum;
      for (int k = 0; k < r.m; ++k) T.coef[k] = -r.c[k] * r.p[k];
    }
  }
  return T;
}

bool opts_ok(const fdd_opts* o) {
  return o && o->outer_rtol > 0 && o->inner_rtol > 0 && o->outer_maxit > 0 &&
         o->inner_maxit > 0 && (o->precision == FDD_MIXED || o->precision == FDD_FP64) &&
         (o->mg_nu == 1 || o->mg_nu == 2) && o->step_rtol >= 1e-7 && o->step_rtol <= 1e-2 &&
         (o->warmstart == nullptr || o->precision == FDD_MIXED) &&
         (o->use_graph == 0 || o->use_graph == 1);
}

double step_tau(const fdd_opts& o) { return o.step_rtol; }

// Kinds of interior right-hand sides with separate launch schedules: the iteration counts of
// solves for a full right-hand side (b, the back-substitution) and for a lifted interface vector
// (one row of data) differ, and a shared schedule would pad the cheaper kind to the other.
enum SchedKind { kSchedGeneral = 0, kSchedLift = 1, kSchedLiftWarm = 2 };

void schedule_record(Schedule* sc, int steps_needed, const int* run_len, int run_its_max) {
  // the converging iteration of a run is the one after its last counted one
  sc->its = std::max(sc->its, run_its_max + 1);
  for (int q = 0; q < std::min(steps_needed, 8); ++q)
    sc->step_its[q] = std::max(sc->step_its[q], run_len[q] + 1);
  const int need = std::max(steps_needed, 1);
  if (!sc->calibrated) {
    sc->steps = need;
    sc->over = sc->under = 0;
    return;
  }
  if (need > sc->steps) {
    sc->under = 0;
    sc->over += 2;
    if (sc->over >= 4) {  // two such solves in close succession
      sc->steps += 1;
      sc->over = 0;
    }
  } else {
    sc->over = std::max(sc->over - 1, 0);
    sc->under = need < sc->steps ? sc->under + 1 : 0;
    if (sc->under >= 16) {
      sc->steps -= 1;
      sc->under = 0;
    }
  }
}

// Selects the problem's schedule for these options and right-hand-side kind.
void use_schedule(fdd_problem_s* P, const fdd_opts& o, int kind) {
  P->sc = &P->scheds[std::make_tuple(o.mg_nu, o.precision == FDD_FP64 ? 0.0 : o.step_rtol, kind)];
}

// Host-side record of an interior solve in flight: which buffers hold what.  Buffer parities
// follow the enqueued schedule (kernels of a converged solve copy instead of skipping), so the
// host always knows where the result is.
struct InnerTrack {
  bool fp64 = false;
  RhsDesc f{};
  int cur_r = 0, cur_p = 0;
  int S = 0;  // refinement steps enqueued after the first residual (mixed precision)
  int k = 0;  // PCG iterations enqueued in the running PCG (FP64)
};

const double* inner_u(const fdd_problem_s* P, const InnerTrack& t) {
  return t.fp64 ? P->s64.x : P->u64[t.S & 1];
}

// First residual (u = 0, or the learned guess `warm` scaled by its Galerkin factor) of an
// interior solve, and in FP64 the start of its PCG.
void enqueue_inner_start(fdd_problem_s* P, const LaunchCtx& c, InnerTrack& t, const fdd_opts& o,
                         const float* warm = nullptr) {
  const double tol2 = o.inner_rtol * o.inner_rtol;
  t.cur_r = t.cur_p = 0;
  t.S = t.k = 0;
  if (!t.fp64) {
    if (warm) launch_warm_alpha(c, t.f, warm);
    // (its bookkeeping is done by the first kernel of the PCG run that always follows)
    launch_ir_residual(c, t.f, nullptr, nullptr, nullptr, P->u64[0], P->s32.r[t.cur_r], nullptr, 1,
                       tol2, step_tau(o) * step_tau(o), 0, warm, warm ? &P->st->warm_alpha : nullptr,
                       false);
  } else {
    launch_ir_residual(c, t.f, nullptr, nullptr, nullptr, P->u64[0], nullptr, P->s64.r[t.cur_r], 1,
                       tol2, tol2, 1, nullptr, nullptr, false);
    launch_pcg_init<double>(c, P->s64.mg, P->s64.r[t.cur_r], P->s64.z);
  }
}

// `steps` refinement steps of `its` FP32 PCG iterations (mixed; its < 0: the per-step
// schedule), or `its` more FP64 iterations.
void enqueue_inner_more(fdd_problem_s* P, const LaunchCtx& c, InnerTrack& t, int steps, int its) {
  if (!t.fp64) {
    auto& S = P->s32;
    for (int st = 0; st < steps; ++st) {
      launch_pcg_init<float>(c, S.mg, S.r[t.cur_r], S.z);
      const int n_its = its >= 0 ? its : (t.S < 8 ? P->sc->step_its[t.S] : P->sc->its);
      for (int k = 0; k < n_its; ++k) {
        // the refinement residual follows the last iteration: it needs no new z
        launch_pcg_iteration<float>(c, S.mg, k, S.x, S.r[t.cur_r], S.r[t.cur_r ^ 1], S.z,
                                    S.p[t.cur_p], S.p[t.cur_p ^ 1], k == n_its - 1);
        t.cur_r ^= 1;
        t.cur_p ^= 1;
      }
      // the next step's first kernel does this residual's bookkeeping; the last one of the
      // sequence gets a kernel of its own (the host or the outer tail reads its outcome)
      launch_ir_residual(c, t.f, P->u64[t.S & 1], S.x, nullptr, P->u64[(t.S + 1) & 1],
                         S.r[t.cur_r], nullptr, 0, 0, 0, 0, nullptr, nullptr, st == steps - 1,
                         n_its > 0);
      t.S += 1;
    }
  } else {
    auto& S = P->s64;
    for (int k = 0; k < its; ++k) {
      launch_pcg_iteration<double>(c, S.mg, t.k, S.x, S.r[t.cur_r], S.r[t.cur_r ^ 1], S.z,
                                   S.p[t.cur_p], S.p[t.cur_p ^ 1]);
      t.k += 1;
      t.cur_r ^= 1;
      t.cur_p ^= 1;
    }
  }
}

int read_state(fdd_problem_s* P, hipStream_t s) {
  if (P->host_seq && P->hook.kind == kTimeNone) {
    // the state is published by a kernel behind the queued work; the host waits for its
    // sequence word (no stream synchronization), checking the stream for errors now and then
    // and falling back to a synchronization after a second
    const unsigned seq = ++P->pub_seq;
    launch_publish_state(s, P->st, P->host_st, P->host_seq, seq);
    HIPCHK(hipGetLastError());
    const auto t0 = std::chrono::steady_clock::now();
    for (unsigned long spin = 0;; ++spin) {
      if (__atomic_load_n(P->host_seq, __ATOMIC_ACQUIRE) == seq) return FDD_OK;
      if ((spin & 4095) == 4095) {
        const hipError_t q = hipStreamQuery(s);
        if (q != hipSuccess && q != hipErrorNotReady)
          return fail(FDD_E_HIP, "device state read-back: %s", hipGetErrorString(q));
        if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(1)) break;
      }
    }
    HIPCHK(hipStreamSynchronize(s));
    if (__atomic_load_n(P->host_seq, __ATOMIC_ACQUIRE) == seq) return FDD_OK;
    return fail(FDD_E_HIP, "device state read-back: the published state did not arrive");
  }
  HIPCHK(hipMemcpyAsync(P->host_st, P->st, sizeof(DevState), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  // harvest the kernel timer: every recorded pair has completed
  for (int i = 0; i < P->hook.used; ++i) {
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, P->hook.ev[2 * i], P->hook.ev[2 * i + 1]));
    P->timed_ms += ms;
    P->timed_launches += 1;
    if (ms >= P->timer_split_ms) {
      P->timed_long_ms += ms;
      P->timed_long += 1;
    }
  }
  P->hook.used = 0;
  return FDD_OK;
}

struct InnerResult {
  int its = 0, steps = 0;
};

// After a synchronization: finish the interior solve tracked by t, topping up eagerly until it
// has converged.  `enqueued_its` counts what the schedule allowed so far.
int inner_finish(fdd_problem_s* P, hipStream_t s, InnerTrack& t, const fdd_opts& o,
                 InnerResult* res) {
  LaunchCtx c = make_ctx(P, s, o.mg_nu, t.fp64);
  for (int round = 0;; ++round) {
    const DevState& h = *P->host_st;
    if (h.breakdown)
      return fail(h.breakdown & 4 ? FDD_E_NONFINITE : FDD_E_BREAKDOWN,
                  "interior solve: breakdown flags %d", h.breakdown);
    if (h.solve_done) {
      res->its = h.inner_its;
      res->steps = h.refine_steps;
      if (!t.fp64) {
        schedule_record(P->sc, h.refine_steps, h.run_len, h.run_its_max);
        if (std::getenv("FDD_TRACE_SCHEDULE")) {
          // diagnostic: the runs of this interior solve against the schedule it ran on
          std::fprintf(stderr, "[fdd schedule] n=%d steps=%d runs=", P->n, h.refine_steps);
          for (int q = 0; q < std::min(h.refine_steps, 8); ++q) std::fprintf(stderr, "%d ", h.run_len[q]);
          std::fprintf(stderr, "schedule=%d:", P->sc->steps);
          for (int q = 0; q < std::min(P->sc->steps, 8); ++q) std::fprintf(stderr, "%d ", P->sc->step_its[q]);
          std::fprintf(stderr, "top-up rounds=%d\n", round);
        }
      } else {
        P->sc->its64 = std::max(P->sc->its64, std::max(h.inner_its, 1));
      }
      return FDD_OK;
    }
    if (h.inner_its >= o.inner_maxit || round > o.inner_maxit) {
      res->its = h.inner_its;
      return fail(FDD_NOT_CONVERGED, "interior solve: %d iterations, residual %.3e of %.3e",
                  h.inner_its, std::sqrt(h.res2), std::sqrt(h.ff));
    }
    // top-up: one more refinement step (long runs while the schedule is being measured)
    if (!t.fp64) enqueue_inner_more(P, c, t, 1, P->sc->calibrated ? P->sc->its : 30);
    else enqueue_inner_more(P, c, t, 0, std::max(P->sc->its64 / 2, 2));
    int rc = read_state(P, s);
    if (rc) return rc;
  }
}

// A complete interior solve A_II u = f, eager launches.
int interior_solve(fdd_problem_s* P, hipStream_t s, const RhsDesc& f, const fdd_opts& o,
                   InnerTrack& t, InnerResult* res) {
  const bool fp64 = (o.precision == FDD_FP64);
  LaunchCtx c = make_ctx(P, s, o.mg_nu, fp64);
  t = InnerTrack{};
  t.fp64 = fp64;
  t.f = f;
  enqueue_inner_start(P, c, t, o);
  if (!P->sc->calibrated) {
    // the first solve of a problem measures the schedule: long PCG runs, one step at a time
    if (!fp64) enqueue_inner_more(P, c, t, 1, 30);
    else enqueue_inner_more(P, c, t, 0, 60);
  } else if (!fp64) {
    enqueue_inner_more(P, c, t, P->sc->steps, -1);
  } else {
    enqueue_inner_more(P, c, t, 0, P->sc->its64);
  }
  int rc = read_state(P, s);
  if (rc) return rc;
  rc = inner_finish(P, s, t, o, res);
  if (rc == FDD_OK) P->sc->calibrated = true;
  return rc;
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
  if (t->tpow != P->tpow || (t->shift0 != 0.0) != (P->kind == kProblemModel))
    return fail(FDD_E_STATE, "rational table built for another problem");
  return FDD_OK;
}

}  // namespace fdd

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
  o->step_rtol = 1e-5;
  o->check_true_residual = 0;
  o->warmstart = nullptr;
  o->use_graph = 1;
}

const char* fdd_last_error(void) { return g_err.c_str(); }
const char* fdd_version(void) { return "fdd 0.1 (gfx950)"; }

int fdd_setup_mesh(const fdd_desc* d, int hip_device, fdd_problem* out) {
  if (!d || !out) return fail(FDD_E_ARG, "null argument");
  *out = nullptr;
  if (d->dim != 2 && d->dim != 3) return fail(FDD_E_ARG, "dim must be 2 or 3 (got %d)", d->dim);
  if (d->dim == 3) {
    if (!(d->K > 0) || !std::isfinite(d->K) || !(d->mu > 0) || !std::isfinite(d->mu))
      return fail(FDD_E_ARG, "K and mu must be positive and finite");
    fdd_problem_s* P = new (std::nothrow) fdd_problem_s();
    if (!P) return fail(FDD_E_NOMEM, "out of host memory");
    const int rc = setup3(d, hip_device, P);
    if (rc) {
      delete P;
      return rc;
    }
    *out = P;
    return FDD_OK;
  }
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
  if (P->dim == 3) {
    *bytes = workspace3(P);
    return FDD_OK;
  }
  if (P->kind == kProblemHdiv) {
    *bytes = hdiv_workspace_bytes(P);
    return FDD_OK;
  }
  if (P->kind == kProblemDarcyStokes) {
    *bytes = ds_workspace_bytes(P);
    return *bytes ? FDD_OK : fail(FDD_E_ARG, "Darcy-Stokes workspace size unavailable");
  }
  fdd_problem_s tmp = *P;
  *bytes = plan_workspace(&tmp, nullptr);
  return FDD_OK;
}

int fdd_bind_workspace(fdd_problem P, void* dev, size_t bytes, void* stream) {
  if (!P || !dev) return fail(FDD_E_ARG, "null argument");
  if (((uintptr_t)dev) & 255) return fail(FDD_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (P->dim == 3) return bind3(P, dev, bytes, (hipStream_t)stream);
  if (P->kind == kProblemHdiv) return hdiv_bind(P, dev, bytes, (hipStream_t)stream);
  if (P->kind == kProblemDarcyStokes) return ds_bind(P, dev, bytes, (hipStream_t)stream);
  fdd_problem_s tmp = *P;
  const size_t need = plan_workspace(&tmp, nullptr);
  if (bytes < need) return fail(FDD_E_WORKSPACE, "workspace %zu bytes < %zu needed", bytes, need);
  HIPCHK(hipSetDevice(P->device));
  hipStream_t s = (hipStream_t)stream;
  // captured graphs hold pointers into the old workspace
  for (auto& kv : P->graphs)
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
  P->graphs.clear();
  P->ws = (char*)dev;
  P->ws_bytes = bytes;
  plan_workspace(P, P->ws);
  if (!P->host_st) HIPCHK(hipHostMalloc((void**)&P->host_st, sizeof(DevState), hipHostMallocDefault));
  if (!P->host_seq) {
    HIPCHK(hipHostMalloc((void**)&P->host_seq, sizeof(unsigned), hipHostMallocDefault));
    *P->host_seq = 0;
    P->pub_seq = 0;
  }
  HIPCHK(hipMemsetAsync(P->ws, 0, need, s));
  const size_t np = P->cinv.size();
  HIPCHK(hipMemcpyAsync(P->cinv64, P->cinv.data(), np * sizeof(double), hipMemcpyHostToDevice, s));
  // FP32 coarse solve on the first level with <= 63 points per side: orthonormal sine transform
  // S_ab = sqrt(2 / (m + 1)) sin(pi (a + 1)(b + 1) / (m + 1)) and symbols 2 - 2 cos(pi (k + 1) / (m + 1))
  const int m = P->lev[P->first_coarse32].nf;
  std::vector<float> S((size_t)kDstN * kDstN, 0.0f), L(kDstN, 0.0f);
  for (int a = 0; a < m; ++a) {
    for (int b = 0; b < m; ++b)
      S[(size_t)a * kDstN + b] =
          (float)(std::sqrt(2.0 / (m + 1)) * std::sin(M_PI * (a + 1) * (b + 1) / (m + 1)));
    L[a] = (float)(2.0 - 2.0 * std::cos(M_PI * (a + 1) / (m + 1)));
  }
  HIPCHK(hipMemcpyAsync(P->dstS, S.data(), S.size() * sizeof(float), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(P->dstL, L.data(), L.size() * sizeof(float), hipMemcpyHostToDevice, s));
  const double lkm[2] = {std::log10(P->K), std::log10(P->mu)};
  HIPCHK(hipMemcpyAsync(P->lk_lmu, lkm, sizeof(lkm), hipMemcpyHostToDevice, s));
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
  if (P->kind == kProblemHdiv && which == FDD_RA_OPERATOR)
    return fail(FDD_E_ARG, "the H(div) problem's operator has no fractional term (no operator table)");
  // the model problem with t >= 0: the operator table approximates lam^(t-1) (L^t = L (table)(L))
  const bool lam_factor = P->kind == kProblemModel && which == FDD_RA_OPERATOR && P->tpow >= 0;
  const double texp = lam_factor ? P->tpow - 1.0 : P->tpow;
  RaResult r = build_rational(which, P->K, P->gamma, P->lam_lo, P->lam_hi, P->eig.data(),
                              (int)P->eig.size(), tol, max_poles, texp);
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
  t->tpow = P->tpow;
  t->shift0 = P->kind == kProblemModel ? 1.0 : 0.0;
  t->lam_factor = lam_factor ? 1 : 0;
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
  if (P->kind == kProblemHdiv && which == FDD_RA_OPERATOR)
    return fail(FDD_E_ARG, "the H(div) problem's operator has no fractional term (no operator table)");
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
  const bool lam_factor = P->kind == kProblemModel && which == FDD_RA_OPERATOR && P->tpow >= 0;
  t->tpow = P->tpow;
  t->shift0 = P->kind == kProblemModel ? 1.0 : 0.0;
  t->lam_factor = lam_factor ? 1 : 0;
  t->r.status = 0;
  t->r.c0 = c0;
  t->r.m = m;
  for (int k = 0; k < m; ++k) {
    t->r.c[k] = c[k];
    t->r.p[k] = p[k];
  }
  t->r.max_rel_err = ra_eval_rel_err(which, P->K, P->gamma, t->r, P->eig.data(), (int)P->eig.size(),
                                     lam_factor ? P->tpow - 1.0 : P->tpow);
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
  if (P->kind == kProblemDarcyStokes)
    return fail(FDD_E_ARG, "the Darcy-Stokes problem is solved by fdd_ds_solve");
  if (!f || !u) return fail(FDD_E_ARG, "null vector");
  fdd_opts o;
  if (opts) o = *opts;
  else fdd_opts_default(&o);
  if (!opts_ok(&o)) return fail(FDD_E_ARG, "invalid options");
  use_schedule(P, o, kSchedGeneral);
  HIPCHK(hipSetDevice(P->device));
  hipStream_t s = (hipStream_t)stream;
  if (P->dim == 3) return interior_solve3(P, f, u, o, s, its);
  if (P->kind == kProblemModel) return model_interior_solve(P, f, u, o, s, its);
  if (P->kind == kProblemHdiv) return hdiv_interior_solve(P, f, u, o, s, its);
  InnerTrack t;
  InnerResult res;
  rc = interior_solve(P, s, RhsDesc{f, 1.0, nullptr, 0.0}, o, t, &res);
  if (its) *its = res.its;
  if (rc < 0) return rc;
  launch_scatter(s, (int)P->NG, P->lev[0].pitch, inner_u(P, t), nullptr, nullptr, nullptr, u);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return rc;
}

int fdd_precond_apply(fdd_problem P, fdd_ratpc T, const double* r, double* z, void* stream) {
  int rc = check_problem(P);
  if (rc) return rc;
  if (P->kind == kProblemDarcyStokes)
    return fail(FDD_E_ARG, "the Darcy-Stokes problem is solved by fdd_ds_solve");
  if ((rc = check_table(P, T, FDD_RA_PRECOND))) return rc;
  if (!r || !z) return fail(FDD_E_ARG, "null vector");
  HIPCHK(hipSetDevice(P->device));
  if (P->dim == 3) return precond_apply3(P, T, r, z, (hipStream_t)stream);
  if (P->kind == kProblemModel) return model_precond_apply(P, T, r, z, (hipStream_t)stream);
  if (P->kind == kProblemHdiv) return hdiv_precond_apply(P, T, r, z, (hipStream_t)stream);
  ShiftTable tab = make_table(T);
  launch_iface_batch((hipStream_t)stream, (int)P->NG, P->h, tab, kIfacePrecond, r, z, P->scratchP,
                     P->st, nullptr, nullptr, 0, 0);
  HIPCHK(hipGetLastError());
  return FDD_OK;
}

int fdd_precond_apply_static(fdd_problem P, fdd_ratpc T, const double* r, double* z, void* stream) {
  if (!P) return fail(FDD_E_ARG, "null problem");
  int rc = check_table(P, T, FDD_RA_PRECOND);
  if (rc) return rc;
  if (!r || !z) return fail(FDD_E_ARG, "null vector");
  if (P->dim != 2 || P->kind != kProblemFacet)
    return fail(FDD_E_ARG, "the static-scratch preconditioner apply is for the 2D facet problem only");
  ShiftTable tab = make_table(T);
  if (tab.m > kStaticPrecondSystems || P->NG > kStaticPrecondN)
    return fail(FDD_E_ARG, "%d systems of %lld unknowns exceed the static scratch (%d x %d)", tab.m,
                (long long)P->NG, kStaticPrecondSystems, kStaticPrecondN);
  HIPCHK(hipSetDevice(P->device));
  double* scratch = nullptr;
  if (static_precond_scratch(P->device, &scratch))
    return fail(FDD_E_HIP, "device %d: no address for the static scratch", P->device);
  launch_iface_batch((hipStream_t)stream, (int)P->NG, P->h, tab, kIfacePrecond, r, z, scratch,
                     nullptr, nullptr, nullptr, 0, 0);
  HIPCHK(hipGetLastError());
  return FDD_OK;
}

int fdd_schur_apply(fdd_problem P, fdd_ratpc H, const double* x, double* y, const fdd_opts* opts,
                    void* stream) {
  int rc = check_problem(P);
  if (rc) return rc;
  if (P->kind == kProblemDarcyStokes)
    return fail(FDD_E_ARG, "the Darcy-Stokes problem is solved by fdd_ds_solve");
  if (P->kind == kProblemHdiv && H)
    return fail(FDD_E_ARG, "the H(div) problem takes no operator table (pass NULL)");
  if (P->kind != kProblemHdiv && (rc = check_table(P, H, FDD_RA_OPERATOR))) return rc;
  if (!x || !y) return fail(FDD_E_ARG, "null vector");
  fdd_opts o;
  if (opts) o = *opts;
  else fdd_opts_default(&o);
  if (!opts_ok(&o)) return fail(FDD_E_ARG, "invalid options");
  use_schedule(P, o, kSchedLift);
  HIPCHK(hipSetDevice(P->device));
  hipStream_t s = (hipStream_t)stream;
  if (P->dim == 3) return schur_apply3(P, H, x, y, o, s);
  if (P->kind == kProblemModel) return model_schur_apply(P, H, x, y, o, s);
  if (P->kind == kProblemHdiv) return hdiv_schur_apply(P, x, y, o, s);
  InnerTrack t;
  InnerResult res;
  rc = interior_solve(P, s, RhsDesc{nullptr, 0.0, x, 1.0}, o, t, &res);
  if (rc) return rc;
  ShiftTable tab = make_table(H);
  launch_iface_batch(s, (int)P->NG, P->h, tab, kIfaceOperator, x, P->Hp, P->scratchH, P->st,
                     nullptr, nullptr, 0, 0);
  launch_schur_gather(s, (int)P->NG, P->lev[0].nf, P->lev[0].pitch, P->K, P->gamma, x,
                      inner_u(P, t), nullptr, nullptr, P->Hp, y, nullptr, nullptr, nullptr,
                      nullptr, P->st, 0, 0);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return FDD_OK;
}

int fdd_apply_operator(fdd_problem P, fdd_ratpc H, const double* x, double* y, void* stream) {
  int rc = check_problem(P);
  if (rc) return rc;
  const bool no_table = P->kind == kProblemHdiv || P->kind == kProblemDarcyStokes;
  if (no_table && H)
    return fail(FDD_E_ARG, "this problem's operator has no fractional term (pass NULL)");
  if (!no_table && (rc = check_table(P, H, FDD_RA_OPERATOR))) return rc;
  if (!x || !y) return fail(FDD_E_ARG, "null vector");
  HIPCHK(hipSetDevice(P->device));
  hipStream_t s = (hipStream_t)stream;
  if (P->dim == 3) return apply_operator3(P, H, x, y, s);
  if (P->kind == kProblemModel) return model_apply_operator(P, H, x, y, s);
  if (P->kind == kProblemHdiv) return hdiv_apply_operator(P, x, y, s);
  if (P->kind == kProblemDarcyStokes) return ds_apply_operator(P, x, y, s);
  ShiftTable tab = make_table(H);
  launch_iface_batch(s, (int)P->NG, P->h, tab, kIfaceOperator, x + P->NI, P->Hp, P->scratchH,
                     P->st, nullptr, nullptr, 0, 0);
  launch_full_operator(s, P->n, P->K, P->gamma, x, P->Hp, y, nullptr, P->partials,
                       P->st->t_res);
  HIPCHK(hipGetLastError());
  return FDD_OK;
}

namespace {

// FNV-1a digest of a shift table as the kernels receive it (by value).
uint64_t table_digest(const ShiftTable& T) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void* p, size_t nb) {
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < nb; ++i) h = (h ^ b[i]) * 1099511628211ull;
  };
  mix(&T.m, sizeof(T.m));
  mix(T.alpha, sizeof(double) * T.m);
  mix(T.beta, sizeof(double) * T.m);
  mix(T.coef, sizeof(double) * T.m);
  mix(&T.d0, sizeof(T.d0));
  return h;
}

// One outer PCG step after the interior solve for the lifted p (version v -> v+1):
// the Schur product y = S p, alpha, x and r updates, then z = P r, rho, beta and p.
void enqueue_outer_tail(fdd_problem_s* P, hipStream_t s, const ShiftTable& tabP, const double* u,
                        int v, bool accumulate) {
  const int a = v & 1, b = (v + 1) & 1;
  launch_schur_gather(s, (int)P->NG, P->lev[0].nf, P->lev[0].pitch, P->K, P->gamma, P->pG[a], u,
                      nullptr, nullptr, P->Hp, P->yG, P->xG[a], P->xG[b], P->rG[a], P->rG[b],
                      P->st, 1, v);
  // x_I(v+1) = x_I(v) + alpha E p (u = E p; versioned, so a repeated tail gives the same result)
  if (accumulate)
    launch_interior_axpy(s, P->lev[0].nf, P->lev[0].pitch, P->xI[a], u, &P->st->o_alpha, 0.0,
                         P->xI[b]);
  launch_iface_batch(s, (int)P->NG, P->h, tabP, kIfacePrecondOuter, P->rG[b], P->zG, P->scratchP,
                     P->st, P->pG[a], P->pG[b], v, 0);
}

// Everything of outer iteration v up to the synchronization: interior solve for the lifted p
// (on the current schedule), H p, and the outer tail.
void enqueue_outer_iteration(fdd_problem_s* P, hipStream_t s, const ShiftTable& tabP,
                             const ShiftTable& tabH, const fdd_opts& o, int v, InnerTrack& t) {
  const int a = v & 1;
  LaunchCtx c = make_ctx(P, s, o.mg_nu, t.fp64);
  t.f = RhsDesc{nullptr, 0.0, P->pG[a], 1.0};
  const float* warm = nullptr;
  const double* wscale = nullptr;
  if (o.warmstart)  // checked by the caller; the network's guess for E p (any scale)
    (void)cnn_warm_guess((fdd_cnn_s*)o.warmstart, s, P->pG[a], P->n, P->lk_lmu, &warm, &wscale);
  enqueue_inner_start(P, c, t, o, warm);
  if (!P->sc->calibrated) {
    // the first solve on this schedule measures it: long PCG runs, one step at a time
    if (!t.fp64) enqueue_inner_more(P, c, t, 1, 30);
    else enqueue_inner_more(P, c, t, 0, 60);
  } else if (!t.fp64) {
    enqueue_inner_more(P, c, t, P->sc->steps, -1);
  } else {
    enqueue_inner_more(P, c, t, 0, P->sc->its64);
  }
  launch_iface_batch(s, (int)P->NG, P->h, tabH, kIfaceOperator, P->pG[a], P->Hp, P->scratchH,
                     P->st, nullptr, nullptr, 0, 0);
  enqueue_outer_tail(P, s, tabP, inner_u(P, t), v, !o.back_solve);
}

// Replays (capturing first if needed) the graph of outer iteration v for the current schedule.
int launch_outer_graph(fdd_problem_s* P, hipStream_t s, const ShiftTable& tabP,
                       const ShiftTable& tabH, const fdd_opts& o, int v, InnerTrack& t) {
  // everything the captured launch sequence depends on: the schedule, the options passed to the
  // kernels by value (tolerances as bit patterns), and both rational tables by content (their
  // shifts, weights and system counts are kernel arguments, so a table of another tol or
  // max_poles, or one given by fdd_ratpc_from_table, needs a graph of its own)
  std::vector<int> key = {v & 1, (int)t.fp64, o.mg_nu, P->sc->steps, P->sc->its, P->sc->its64,
                          o.back_solve ? 1 : 0};
  key.insert(key.end(), P->sc->step_its, P->sc->step_its + 8);
  push_bits(key, o.step_rtol);
  push_bits(key, o.inner_rtol);
  push_bits(key, table_digest(tabP));
  push_bits(key, table_digest(tabH));
  push_bits(key, (uint64_t)(uintptr_t)o.warmstart);
  if (o.warmstart) push_bits(key, cnn_binding_id((const fdd_cnn_s*)o.warmstart));
  auto it = P->graphs.find(key);
  if (it == P->graphs.end()) {
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    enqueue_outer_iteration(P, s, tabP, tabH, o, v, t);
    hipError_t e = hipStreamEndCapture(s, &g);
    if (e != hipSuccess) return fail(FDD_E_HIP, "graph capture: %s", hipGetErrorString(e));
    GraphEntry ge;
    e = hipGraphInstantiate(&ge.exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(FDD_E_HIP, "graph instantiate: %s", hipGetErrorString(e));
    ge.cur_r = t.cur_r;
    ge.cur_p = t.cur_p;
    ge.S = t.S;
    ge.k = t.k;
    it = P->graphs.emplace(key, ge).first;
  }
  t.cur_r = it->second.cur_r;
  t.cur_p = it->second.cur_p;
  t.S = it->second.S;
  t.k = it->second.k;
  t.f = RhsDesc{nullptr, 0.0, P->pG[v & 1], 1.0};
  HIPCHK(hipGraphLaunch(it->second.exec, s));
  return FDD_OK;
}

}  // namespace

int fdd_solve(fdd_problem P, fdd_ratpc PT, fdd_ratpc HT, const double* b, double* x,
              const fdd_opts* opts, void* stream, fdd_stats* stats) {
  const auto t_start = std::chrono::steady_clock::now();
  fdd_stats st{};
  st.true_rel_res = -1.0;
  int rc = check_problem(P);
  if (rc) return rc;
  if (P->kind == kProblemDarcyStokes)
    return fail(FDD_E_ARG, "the Darcy-Stokes problem is solved by fdd_ds_solve");
  if ((rc = check_table(P, PT, FDD_RA_PRECOND))) return rc;
  if (P->kind == kProblemHdiv && HT)
    return fail(FDD_E_ARG, "the H(div) problem takes no operator table (pass NULL)");
  if (P->kind != kProblemHdiv && (rc = check_table(P, HT, FDD_RA_OPERATOR))) return rc;
  if (!b || !x) return fail(FDD_E_ARG, "null vector");
  fdd_opts o;
  if (opts) o = *opts;
  else fdd_opts_default(&o);
  if (!opts_ok(&o)) return fail(FDD_E_ARG, "invalid options");
  if (P->dim == 3) {
    if (o.warmstart) return fail(FDD_E_ARG, "3D solves take no warm start");
    HIPCHK(hipSetDevice(P->device));
    return solve3(P, PT, HT, b, x, o, (hipStream_t)stream, stats);
  }
  if (P->kind == kProblemModel) {
    if (o.warmstart) return fail(FDD_E_ARG, "the model problem takes no warm start");
    HIPCHK(hipSetDevice(P->device));
    return model_solve(P, PT, HT, b, x, o, (hipStream_t)stream, stats);
  }
  if (P->kind == kProblemHdiv) {
    if (o.warmstart) return fail(FDD_E_ARG, "the H(div) problem takes no warm start");
    HIPCHK(hipSetDevice(P->device));
    return hdiv_solve(P, PT, b, x, o, (hipStream_t)stream, stats);
  }
  if (o.warmstart && (rc = cnn_check_for((const fdd_cnn_s*)o.warmstart, P->n))) return rc;
  use_schedule(P, o, kSchedGeneral);
  HIPCHK(hipSetDevice(P->device));
  hipStream_t us = (hipStream_t)stream;
  hipStream_t s = us;
  if (P->hook.kind != kTimeNone) o.use_graph = 0;  // timed launches carry their own events
  if (o.use_graph) {
    // graphs are captured and replayed on the library's own stream (default priority), ordered
    // after the caller's stream at entry and before it at exit
    if (!P->gstream) {
      HIPCHK(hipStreamCreateWithFlags(&P->gstream, hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&P->ev_in, hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&P->ev_out, hipEventDisableTiming));
    }
    HIPCHK(hipEventRecord(P->ev_in, us));
    HIPCHK(hipStreamWaitEvent(P->gstream, P->ev_in, 0));
    s = P->gstream;
  }
  const bool fp64 = (o.precision == FDD_FP64);
  const int ng = (int)P->NG, nf = P->lev[0].nf, pitch = P->lev[0].pitch;
  const ShiftTable tabP = make_table(PT), tabH = make_table(HT);
  auto account = [&](const InnerResult& r) {
    st.inner_solves += 1;
    st.inner_its_total += r.its;
    st.inner_its_max = std::max(st.inner_its_max, r.its);
    st.refine_steps += r.steps;
  };
  auto finish = [&](int code) -> int {
    if (o.use_graph) {
      (void)hipEventRecord(P->ev_out, s);
      (void)hipStreamWaitEvent(us, P->ev_out, 0);
    }
    st.status = code;
    st.t_solve_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    if (stats) *stats = st;
    return code;
  };
  // 1. g = b_G - A_GI A_II^{-1} b_I
  InnerTrack t;
  InnerResult res;
  rc = interior_solve(P, s, RhsDesc{b, 1.0, nullptr, 0.0}, o, t, &res);
  account(res);
  if (rc) return finish(rc);
  launch_rhs_reduce(s, ng, pitch, b + P->NI, inner_u(P, t), nullptr, nullptr, P->rG[0], P->xG[0]);
  if (!o.back_solve)  // x_I(0) = A_II^{-1} b_I / K
    launch_interior_axpy(s, nf, pitch, nullptr, inner_u(P, t), nullptr, 1.0 / P->K, P->xI[0]);
  // 2. outer PCG from x_G = 0: z = P r, rho0 = r.z, p = z
  launch_iface_batch(s, ng, P->h, tabP, kIfacePrecondOuter, P->rG[0], P->zG, P->scratchP, P->st,
                     nullptr, P->pG[0], 0, 1);
  HIPCHK(hipGetLastError());
  if ((rc = read_state(P, s))) return finish(rc);
  use_schedule(P, o, o.warmstart ? kSchedLiftWarm : kSchedLift);
  const double rho0 = P->host_st->o_rho0;
  if (P->host_st->breakdown) return finish(fail(FDD_E_BREAKDOWN, "preconditioner not positive"));
  int v = 0;
  double rho = rho0;
  bool converged = !(rho0 > 0.0);
  while (!converged && st.outer_its < o.outer_maxit) {
    t = InnerTrack{};
    t.fp64 = fp64;
    if (o.use_graph && P->sc->calibrated) {
      if ((rc = launch_outer_graph(P, s, tabP, tabH, o, v, t))) return finish(rc);
    } else {
      enqueue_outer_iteration(P, s, tabP, tabH, o, v, t);
    }
    HIPCHK(hipGetLastError());
    if ((rc = read_state(P, s))) return finish(rc);
    if (!P->host_st->solve_done && !P->host_st->breakdown) {
      // the schedule was short for this right-hand side: finish the interior solve eagerly and
      // redo the outer tail (it reads only version-v vectors, so it can be repeated)
      rc = inner_finish(P, s, t, o, &res);
      account(res);
      if (rc) return finish(rc);
      P->sc->calibrated = true;
      enqueue_outer_tail(P, s, tabP, inner_u(P, t), v, !o.back_solve);
      HIPCHK(hipGetLastError());
      if ((rc = read_state(P, s))) return finish(rc);
    } else {
      rc = inner_finish(P, s, t, o, &res);
      account(res);
      if (rc) return finish(rc);
      P->sc->calibrated = true;
    }
    if (o.warmstart) {
      st.warm_starts += 1;
      st.warm_accepted += P->host_st->warm_used;
    }
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
  // 3. back-substitution x_I = A_II^{-1} (b_I / K - A_IG x_G): accumulated during the outer
  //    PCG, or one more interior solve
  if (o.back_solve) {
    use_schedule(P, o, kSchedGeneral);
    rc = interior_solve(P, s, RhsDesc{b, 1.0 / P->K, P->xG[v & 1], 1.0}, o, t, &res);
    account(res);
    if (rc) return finish(rc);
    launch_scatter(s, nf, pitch, inner_u(P, t), nullptr, nullptr, P->xG[v & 1], x);
  } else {
    launch_scatter(s, nf, pitch, P->xI[v & 1], nullptr, nullptr, P->xG[v & 1], x);
  }
  if (o.check_true_residual) {
    launch_iface_batch(s, ng, P->h, tabH, kIfaceOperator, x + P->NI, P->Hp, P->scratchH, P->st,
                       nullptr, nullptr, 0, 0);
    launch_full_operator(s, P->n, P->K, P->gamma, x, P->Hp, nullptr, b, P->partials,
                         P->st->t_res);
  }
  HIPCHK(hipGetLastError());
  if ((rc = read_state(P, s))) return finish(rc);
  if (o.check_true_residual && P->host_st->t_res[1] > 0)
    st.true_rel_res = std::sqrt(P->host_st->t_res[0] / P->host_st->t_res[1]);
  return finish(converged ? FDD_OK : FDD_NOT_CONVERGED);
}

int fdd_set_kernel_timer(fdd_problem P, int kind, double split_us) {
  if (!P) return fail(FDD_E_ARG, "null problem");
  if (!(split_us >= 0)) return fail(FDD_E_ARG, "split_us must be >= 0");
  P->timer_split_ms = split_us * 1e-3;
  if (kind < FDD_KT_NONE || kind > FDD_KT_COARSE) return fail(FDD_E_ARG, "bad timer kind");
  HIPCHK(hipSetDevice(P->device));
  if (kind != FDD_KT_NONE && !P->hook.ev) {
    const int cap = 4096;
    P->hook.ev = new (std::nothrow) hipEvent_t[2 * cap];
    if (!P->hook.ev) return fail(FDD_E_NOMEM, "out of host memory");
    for (int i = 0; i < 2 * cap; ++i) HIPCHK(hipEventCreate(&P->hook.ev[i]));
    P->hook.cap = cap;
  }
  P->hook.kind = kind;
  P->hook.used = 0;
  P->hook.skipped = 0;
  P->timed_launches = P->timed_long = 0;
  P->timed_ms = P->timed_long_ms = 0.0;
  return FDD_OK;
}

int fdd_get_kernel_timer(fdd_problem P, int64_t* launches, double* total_ms, int64_t* long_launches,
                         double* long_ms, int64_t* untimed) {
  if (!P) return fail(FDD_E_ARG, "null problem");
  if (launches) *launches = P->timed_launches;
  if (total_ms) *total_ms = P->timed_ms;
  if (long_launches) *long_launches = P->timed_long;
  if (long_ms) *long_ms = P->timed_long_ms;
  if (untimed) *untimed = P->hook.skipped;
  return FDD_OK;
}

void fdd_destroy_problem(fdd_problem P) {
  if (!P) return;
  destroy3(P);
  hdiv_destroy(P);
  ds_destroy(P);
  if (P->hook.ev) {
    for (int i = 0; i < 2 * P->hook.cap; ++i) (void)hipEventDestroy(P->hook.ev[i]);
    delete[] P->hook.ev;
  }
  for (auto& kv : P->graphs)
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
  if (P->gstream) (void)hipStreamDestroy(P->gstream);
  if (P->ev_in) (void)hipEventDestroy(P->ev_in);
  if (P->ev_out) (void)hipEventDestroy(P->ev_out);
  if (P->host_st) (void)hipHostFree(P->host_st);
  if (P->host_seq) (void)hipHostFree(P->host_seq);
  delete P;
}

void fdd_destroy_ratpc(fdd_ratpc t) { delete t; }

}  // extern "C"
