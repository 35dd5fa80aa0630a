// Host-side state of the C ABI, shared by the single-problem (api.cpp) and batched
// (api_batch.cpp) orchestration.
#pragma once
#include "fdd.h"

#include <cstdint>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "fdd_internal.h"

namespace fdd {

// Records the message of a failed call (returned by fdd_last_error) and returns code.
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

#define HIPCHK(call)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess) return fail(FDD_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Appends the bit pattern of a value to a graph-cache key (exact: distinct tolerances never
// share a captured graph).
inline void push_bits(std::vector<int>& key, uint64_t v) {
  key.push_back((int)(uint32_t)(v & 0xffffffffu));
  key.push_back((int)(uint32_t)(v >> 32));
}
inline void push_bits(std::vector<int>& key, double v) {
  uint64_t u;
  std::memcpy(&u, &v, sizeof(u));
  push_bits(key, u);
}
inline int round_up(int x, int a) { return (x + a - 1) / a * a; }

// Launch schedule of the interior solves: refinement steps x FP32 PCG iterations per step
// (mixed), or FP64 PCG iterations.  It only grows; the first solve runs every PCG to its own
// criterion and measures it.
struct Schedule {
  int steps = 1, its = 2, its64 = 4;
  int step_its[8] = {2, 2, 2, 2, 2, 2, 2, 2};
  bool calibrated = false;
  int over = 0;   // recent solves that needed more refinement steps than scheduled (weighted)
  int under = 0;  // consecutive solves that needed fewer
};

// Records what one interior solve (or the slowest instance of a batched one) needed in mixed
// precision: its refinement steps and the PCG iterations of the runs of its first steps.
// Per-step iteration counts only grow (plus the converging iteration).  The step count follows
// the common case: a step more is added once solves keep needing it (a rare longer solve is
// topped up instead of padding every replay), and one is dropped after a long streak of shorter
// solves.
void schedule_record(Schedule* sc, int steps_needed, const int* run_len, int run_its_max);

// Per-precision multigrid-PCG buffers of level 0 plus the hierarchy.
template <typename T>
struct PcgSet {
  T* x = nullptr;
  T* r[2] = {nullptr, nullptr};
  T* p[2] = {nullptr, nullptr};
  T* z = nullptr;
  MGBuffers<T> mg{};
};

// An instantiated graph of one outer iteration and the host-side buffer state after it.
struct GraphEntry {
  hipGraphExec_t exec = nullptr;
  int cur_r = 0, cur_p = 0, S = 0, k = 0;
};

}  // namespace fdd

using fdd::DevState;
using fdd::EventHook;
using fdd::GraphEntry;
using fdd::Level;
using fdd::PcgSet;
using fdd::RaResult;
using fdd::Reductions;
using fdd::kMaxLevels;

struct Problem3D;  // the 3D solver's state (api_3d.cpp)
namespace fdd {
struct ProblemHdiv;  // the H(div) problem's state (hdiv_setup.cpp, api_hdiv.cpp)
struct ProblemDS;    // the Darcy-Stokes problem's state (ds_setup.cpp, api_ds.cpp)
}

struct fdd_problem_s {
  int dim = 2, n = 0, device = 0;
  int kind = 0;                 // fdd::kProblemFacet, kProblemModel (Gamma = the boundary),
                                // kProblemHdiv or kProblemDarcyStokes
  double tpow = -0.5;           // exponent t of the perturbation (the facet problems: -1/2)
  int model_its_hint = 0;       // iterations of the model problem's last interior solve
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
  double* partials = nullptr;   // true-residual reduction
  Reductions red{};
  float* dstS = nullptr;    // FP32 coarse solve: sine-transform matrix and symbols
  float* dstL = nullptr;
  double* cinv64 = nullptr;
  PcgSet<float> s32;
  PcgSet<double> s64;
  double* u64[2] = {nullptr, nullptr};  // refinement accumulators
  double* xI[2] = {nullptr, nullptr};   // interior part of the solution, by outer version
  double* xG[2] = {nullptr, nullptr};
  double* rG[2] = {nullptr, nullptr};
  double* pG[2] = {nullptr, nullptr};
  double* zG = nullptr;
  double* yG = nullptr;
  double* Hp = nullptr;
  double* lk_lmu = nullptr;     // {log10 K, log10 mu} for the warm-start network
  Problem3D* p3 = nullptr;      // dim = 3: everything of the 3D path
  fdd::ProblemHdiv* ph = nullptr;  // the H(div) problem: everything of its path
  fdd::ProblemDS* pds = nullptr;   // the Darcy-Stokes problem: everything of its path
  double* scratchP = nullptr;
  double* scratchH = nullptr;
  DevState* host_st = nullptr;  // pinned copy
  unsigned* host_seq = nullptr;  // pinned word: sequence number of the last published state
  unsigned pub_seq = 0;
  // inner schedule (refinement steps x PCG iterations, or FP64 PCG iterations); only grows
  // one schedule per (smoother sweeps, per-step reduction); `sc` is the current one
  // launch schedules by (mg_nu, step_rtol (0 in FP64), right-hand-side kind)
  std::map<std::tuple<int, double, int>, fdd::Schedule> scheds;
  fdd::Schedule* sc = nullptr;
  int full_its_hint = 0;        // iterations of the last full-system PCG (enqueued ahead)
  // captured outer iterations, keyed by everything their launches bake in (parity, schedule,
  // precision, smoother, tolerances, table contents, warm-start binding)
  std::map<std::vector<int>, GraphEntry> graphs;
  hipStream_t gstream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // kernel timer (HIP events around every launch of one kernel kind)
  EventHook hook;
  long long timed_launches = 0, timed_long = 0;
  double timed_ms = 0.0, timed_long_ms = 0.0;
  double timer_split_ms = 0.008;
};

struct fdd_ratpc_s {
  int which = 0;
  const fdd_problem_s* prob = nullptr;
  int n = 0;
  double K = 0, mu = 0;
  double tpow = -0.5;           // the problem's exponent t
  double shift0 = 0.0;          // L = A_G + shift0 M_G (the model problem's L = -Delta_Gamma + I)
  int lam_factor = 0;           // operator table of lam^(t-1): L^t = L (table)(L) (t >= 0)
  RaResult r{};
};


namespace fdd {

enum ProblemKind { kProblemFacet = 0, kProblemModel = 1, kProblemHdiv = 2, kProblemDarcyStokes = 3 };

ShiftTable make_table(const fdd_ratpc_s* t);
// the paper's model problem in 2D (api_model.cpp)
// the H(div) problem (api_hdiv.cpp)
size_t ds_workspace_bytes(fdd_problem_s* P);
int ds_bind(fdd_problem_s* P, void* dev, size_t bytes, hipStream_t s);
void ds_destroy(fdd_problem_s* P);
int ds_apply_operator(fdd_problem_s* P, const double* x, double* y, hipStream_t s);
size_t hdiv_workspace_bytes(fdd_problem_s* P);
int hdiv_bind(fdd_problem_s* P, void* dev, size_t bytes, hipStream_t s);
void hdiv_destroy(fdd_problem_s* P);
int hdiv_interior_solve(fdd_problem_s* P, const double* f, double* u, const fdd_opts& o,
                        hipStream_t s, int* its);
int hdiv_precond_apply(fdd_problem_s* P, const fdd_ratpc_s* T, const double* r, double* z,
                       hipStream_t s);
int hdiv_schur_apply(fdd_problem_s* P, const double* x, double* y, const fdd_opts& o,
                     hipStream_t s);
int hdiv_apply_operator(fdd_problem_s* P, const double* x, double* y, hipStream_t s);
int hdiv_solve(fdd_problem_s* P, const fdd_ratpc_s* PT, const double* b, double* x,
               const fdd_opts& o, hipStream_t s, fdd_stats* stats);
int model_interior_solve(fdd_problem_s* P, const double* f, double* u, const fdd_opts& o,
                         hipStream_t s, int* its);
int model_precond_apply(fdd_problem_s* P, const fdd_ratpc_s* T, const double* r, double* z,
                        hipStream_t s);
int model_apply_operator(fdd_problem_s* P, const fdd_ratpc_s* H, const double* x, double* y,
                         hipStream_t s);
int model_schur_apply(fdd_problem_s* P, const fdd_ratpc_s* H, const double* x, double* y,
                      const fdd_opts& o, hipStream_t s);
int model_solve(fdd_problem_s* P, const fdd_ratpc_s* PT, const fdd_ratpc_s* HT, const double* b,
                double* x, const fdd_opts& o, hipStream_t s, fdd_stats* stats);
bool opts_ok(const fdd_opts* o);
double step_tau(const fdd_opts& o);
// the 3D path (api_3d.cpp)
int setup3(const fdd_desc* d, int hip_device, fdd_problem_s* P);
size_t workspace3(fdd_problem_s* P);
int bind3(fdd_problem_s* P, void* dev, size_t bytes, hipStream_t s);
void destroy3(fdd_problem_s* P);
int interior_solve3(fdd_problem_s* P, const double* f, double* u, const fdd_opts& o, hipStream_t s,
                    int* its);
int precond_apply3(fdd_problem_s* P, const fdd_ratpc_s* T, const double* r, double* z,
                   hipStream_t s);
int schur_apply3(fdd_problem_s* P, const fdd_ratpc_s* H, const double* x, double* y,
                 const fdd_opts& o, hipStream_t s);
int apply_operator3(fdd_problem_s* P, const fdd_ratpc_s* H, const double* x, double* y,
                    hipStream_t s);
int solve3(fdd_problem_s* P, const fdd_ratpc_s* PT, const fdd_ratpc_s* HT, const double* b,
           double* x, const fdd_opts& o, hipStream_t s, fdd_stats* stats);
// warm-start network (api_cnn.cpp)
int cnn_check_for(const fdd_cnn_s* C, int n);
// identifies the network's current workspace binding (its buffers are kernel arguments)
uint64_t cnn_binding_id(const fdd_cnn_s* C);
int cnn_warm_guess(fdd_cnn_s* C, hipStream_t s, const double* trace, int n, const double* lk_lmu,
                   const float** guess, const double** scale);
// batched form: B traces of one size n in one forward pass (the batched solver's warm start)
int cnn_warm_guess_batch(fdd_cnn_s* C, hipStream_t s, const double* traces, int ld, int B, int n,
                         const double* lk, const double* lmu, float* out);
float* cnn_output(fdd_cnn_s* C, int64_t* capacity);
int cnn_batch_max(const fdd_cnn_s* C);
int check_problem(fdd_problem_s* P);
int check_table(const fdd_problem_s* P, const fdd_ratpc_s* t, int which);
LaunchCtx make_ctx(const fdd_problem_s* P, hipStream_t s, int nu, bool fp64);
// copies the device state to the pinned host copy (synchronizes the stream)
int read_state(fdd_problem_s* P, hipStream_t s);

}  // namespace fdd
