// Batched solves: many independent 2D problems (different n, K, mu, rational tables) advance
// through the Schur-complement PCG together.  Every launch covers the whole batch (one grid over
// the concatenated tiles of all instances, one grid over all shifted interface systems), all
// instances share one enqueue schedule, and an outer iteration is one hipGraph replay for the
// batch.  Per-instance state lives on the device: an instance whose outer PCG has converged is
// skipped by every kernel of the outer loop, so the launch sequence stays fixed.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "api_internal.h"

using namespace fdd;

namespace {

struct BGraph {
  hipGraphExec_t exec = nullptr;
  int cur_r = 0, cur_p = 0, S = 0;
};

struct BTrack {
  int cur_r = 0, cur_p = 0, S = 0;
};

}  // namespace

struct fdd_batch_s {
  int count = 0, device = 0;
  std::vector<fdd_problem_s*> probs;
  std::vector<const fdd_ratpc_s*> tabP, tabH;
  // launch geometry
  int max_tiled = 1;
  int tiles_total[kMaxLevels] = {};
  int tile_edge[kMaxLevels] = {};  // kTile, or kMidTile on intermediate levels with few tiles
  int mid_tile = 0;                // intermediate-level tile edge: 0 (by tile count), 16 or 32
  bool tiles_dirty = false;        // tile lists changed since the workspace was written
  int sysP_total = 0, sysH_total = 0;
  std::vector<int> tiles_prefix[kMaxLevels];
  std::vector<int> sysP_prefix, sysH_prefix;
  // workspace views
  char* ws = nullptr;
  size_t ws_bytes = 0;
  BInst* d_inst = nullptr;
  int* d_tiles[kMaxLevels] = {};
  int* d_sysP = nullptr;
  int* d_sysH = nullptr;
  ShiftTable* d_tab = nullptr;  // P tables, then H tables
  DevState* d_states = nullptr;
  // learned warm start: the network's input traces (one row of tmax per instance, in the order
  // of `slot`), log10 K and log10 mu per row; instances grouped by n (one forward pass a group)
  int tmax = 1;
  double* d_traces = nullptr;
  double* d_lk = nullptr;
  double* d_lmu = nullptr;
  std::vector<int> slot;              // row of instance i
  struct Group { int n, off, count; int64_t img; };  // img: offset of its first output image
  std::vector<Group> groups;
  const fdd_cnn_s* warm_for = nullptr; // the network the rows/groups were last prepared for
  const fdd_cnn_s* warm = nullptr;     // the network of the running solve (null: no warm start)
  // pinned host mirrors
  BInst* h_inst = nullptr;      // staging of the descriptors
  DevState* h_states = nullptr;
  std::vector<BInst> uploaded;  // descriptors as last uploaded
  // shared enqueue schedule per (smoother sweeps, per-step reduction); only grows
  // launch schedules by (mg_nu, step_rtol, right-hand-side kind: 0 full, 1 lifted interface
  // vector); the two kinds need different iteration counts
  std::map<std::tuple<int, double, int>, Schedule> scheds;
  Schedule* sc = nullptr;
  std::map<std::vector<int>, BGraph> graphs;
  hipStream_t gstream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // kernel timer (HIP events attached to every launch of one kernel kind)
  EventHook hook;
  long long timed_launches = 0, timed_long = 0;
  double timed_ms = 0.0, timed_long_ms = 0.0;
  double timer_split_ms = 0.008;
};

namespace {

size_t plan_batch(fdd_batch_s* B, char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    off = align_up(off, 256);
    char* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  };
  const size_t c = (size_t)B->count;
  B->d_inst = (BInst*)take(sizeof(BInst) * c);
  for (int l = 0; l < kMaxLevels; ++l) B->d_tiles[l] = (int*)take(sizeof(int) * (c + 1));
  B->d_sysP = (int*)take(sizeof(int) * (c + 1));
  B->d_sysH = (int*)take(sizeof(int) * (c + 1));
  B->d_tab = (ShiftTable*)take(sizeof(ShiftTable) * 2 * c);
  B->d_states = (DevState*)take(sizeof(DevState) * c);
  B->d_traces = (double*)take(sizeof(double) * c * (size_t)B->tmax);
  B->d_lk = (double*)take(sizeof(double) * c);
  B->d_lmu = (double*)take(sizeof(double) * c);
  return align_up(off, 256);
}

// Tile edge of every tiled level and the concatenated tile lists.  Level 0 always runs 32 x 32
// tiles.  An intermediate level takes B->mid_tile (16 or 32) when set; otherwise (0) 16 x 16 tiles
// where the batch has fewer than four 32 x 32 tiles per compute unit on that level (latency-bound:
// smaller tiles spread it further), else 32 x 32 (less halo re-read).
void plan_tiles(fdd_batch_s* B) {
  const int count = B->count;
  for (int l = 0; l < kMaxLevels; ++l) {
    int t32 = 0;
    for (int i = 0; i < count; ++i)
      if (l < B->probs[i]->first_coarse32) {
        const int tx = (B->probs[i]->lev[l].nf + kTile - 1) / kTile;
        t32 += tx * tx;
      }
    if (l == 0) B->tile_edge[l] = kTile;
    else if (B->mid_tile) B->tile_edge[l] = B->mid_tile;
    else B->tile_edge[l] = t32 < 4 * 256 ? kMidTile : kTile;
    auto& pre = B->tiles_prefix[l];
    pre.assign(count + 1, 0);
    for (int i = 0; i < count; ++i) {
      const fdd_problem_s* Q = B->probs[i];
      int t = 0;
      if (l < Q->first_coarse32) {
        const int tt = B->tile_edge[l];
        const int tx = (Q->lev[l].nf + tt - 1) / tt;
        t = tx * tx;
      }
      pre[i + 1] = pre[i] + t;
    }
    B->tiles_total[l] = pre[count];
  }
}

// Copies the tile lists to the batch workspace (on stream s).
int upload_tiles(fdd_batch_s* B, hipStream_t s) {
  for (int l = 0; l < kMaxLevels; ++l)
    HIPCHK(hipMemcpyAsync(B->d_tiles[l], B->tiles_prefix[l].data(), sizeof(int) * (B->count + 1),
                          hipMemcpyHostToDevice, s));
  return FDD_OK;
}

// Descriptor of instance i from its problem's bound workspace and the caller's vectors.
BInst make_inst(const fdd_batch_s* B, int i, const double* b, double* x) {
  const fdd_problem_s* P = B->probs[i];
  BInst I;
  std::memset(&I, 0, sizeof(I));
  I.nlev = P->nlev;
  I.fc = P->first_coarse32;
  for (int l = 0; l < P->nlev; ++l) {
    I.nf[l] = P->lev[l].nf;
    I.pitch[l] = P->lev[l].pitch;
    const int tt = B->tile_edge[l];  // tile edge of the level (as the tile lists)
    I.tiles_x[l] = l < I.fc ? (P->lev[l].nf + tt - 1) / tt : 0;
    I.f[l] = P->s32.mg.f[l];
    I.u[l] = P->s32.mg.u[l];
    I.e[l] = P->s32.mg.e[l];
  }
  I.x = P->s32.x;
  for (int k = 0; k < 2; ++k) {
    I.r[k] = P->s32.r[k];
    I.p[k] = P->s32.p[k];
    I.u64[k] = P->u64[k];
    I.xI[k] = P->xI[k];
    I.xG[k] = P->xG[k];
    I.rG[k] = P->rG[k];
    I.pG[k] = P->pG[k];
  }
  I.z = P->s32.z;
  I.dstS = P->dstS;
  I.dstL = P->dstL;
  I.st = P->st;
  I.red = P->red;
  I.ng = (int)P->NG;
  I.mP = make_table(B->tabP[i]).m;
  I.mH = make_table(B->tabH[i]).m;
  I.h = P->h;
  I.K = P->K;
  I.gamma = P->gamma;
  I.b = b;
  I.xout = x;
  I.zG = P->zG;
  I.yG = P->yG;
  I.Hp = P->Hp;
  I.scrP = P->scratchP;
  I.scrH = P->scratchH;
  I.tabP = B->d_tab + i;
  I.tabH = B->d_tab + B->count + i;
  I.warm = nullptr;
  I.trace = nullptr;
  if (B->warm) {
    const int sl = B->slot[i];
    for (const auto& g : B->groups)
      if (sl >= g.off && sl < g.off + g.count)
        I.warm = cnn_output(const_cast<fdd_cnn_s*>(B->warm), nullptr) + g.img +
                 (int64_t)(sl - g.off) * (g.n - 1) * (g.n - 1);
    I.trace = B->d_traces + (size_t)sl * B->tmax;
  }
  return I;
}

BatchCtx make_bctx(const fdd_batch_s* B, hipStream_t s, int nu, int skip_done) {
  BatchCtx c{};
  c.hook = B->hook.kind != kTimeNone ? const_cast<EventHook*>(&B->hook) : nullptr;
  c.stream = s;
  c.inst = B->d_inst;
  for (int l = 0; l < kMaxLevels; ++l) c.lists.tiles[l] = B->d_tiles[l];
  c.lists.sysP = B->d_sysP;
  c.lists.sysH = B->d_sysH;
  c.lists.ninst = B->count;
  c.nu = nu;
  c.max_tiled = B->max_tiled;
  for (int l = 0; l < kMaxLevels; ++l) {
    c.tiles_total[l] = B->tiles_total[l];
    c.tile_edge[l] = B->tile_edge[l];
  }
  c.sysP_total = B->sysP_total;
  c.sysH_total = B->sysH_total;
  c.skip_done = skip_done;
  return c;
}

int read_states(fdd_batch_s* B, hipStream_t s) {
  BatchCtx c = make_bctx(B, s, 1, 0);
  launch_b_gather_states(c, B->d_states);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(B->h_states, B->d_states, sizeof(DevState) * B->count,
                        hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int i = 0; i < B->hook.used; ++i) {
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, B->hook.ev[2 * i], B->hook.ev[2 * i + 1]));
    B->timed_ms += ms;
    B->timed_launches += 1;
    if (ms >= B->timer_split_ms) {
      B->timed_long_ms += ms;
      B->timed_long += 1;
    }
  }
  B->hook.used = 0;
  return FDD_OK;
}

void enqueue_start(const BatchCtx& c, BTrack& t, int rhs, int ver, const fdd_opts& o) {
  t = BTrack{};
  launch_b_inner_start(c, rhs, ver, o.inner_rtol * o.inner_rtol, step_tau(o) * step_tau(o));
}

// `steps` refinement steps; its < 0 takes the per-step schedule.
void enqueue_steps(const fdd_batch_s* B, const BatchCtx& c, BTrack& t, int rhs, int ver,
                   int steps, int its) {
  for (int q = 0; q < steps; ++q) {
    const int n_its = its >= 0 ? its : (t.S < 8 ? B->sc->step_its[t.S] : B->sc->its);
    launch_b_inner_step(c, rhs, ver, n_its, t.S, t.cur_r, t.cur_p);
    t.S += 1;
  }
}

// After a synchronization: completes the interior solve of every instance marked in `live`
// (eager top-up steps for the whole batch), then records iteration counts and grows the
// shared schedule.
int finish_inner(fdd_batch_s* B, hipStream_t s, const BatchCtx& c, BTrack& t, int rhs, int ver,
                 const std::vector<char>& live, const fdd_opts& o, std::vector<fdd_stats>& st) {
  for (int round = 0;; ++round) {
    bool all = true;
    for (int i = 0; i < B->count; ++i) {
      if (!live[i]) continue;
      const DevState& h = B->h_states[i];
      if (h.breakdown)
        return fail(h.breakdown & 4 ? FDD_E_NONFINITE : FDD_E_BREAKDOWN,
                    "batch instance %d: interior solve breakdown (flags %d)", i, h.breakdown);
      if (!h.solve_done) {
        all = false;
        if (h.inner_its >= o.inner_maxit || round > o.inner_maxit)
          return fail(FDD_NOT_CONVERGED, "batch instance %d: interior solve did not converge in %d "
                      "iterations", i, h.inner_its);
      }
    }
    if (all) break;
    // top-up: one more refinement step (long runs while the schedule is being measured)
    enqueue_steps(B, c, t, rhs, ver, 1, B->sc->calibrated ? B->sc->its : 30);
    HIPCHK(hipGetLastError());
    int rc = read_states(B, s);
    if (rc) return rc;
  }
  // the batch needs what its slowest instance needs
  int steps = 0, its_max = 0;
  int run_len[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int i = 0; i < B->count; ++i) {
    if (!live[i]) continue;
    const DevState& h = B->h_states[i];
    st[i].inner_solves += 1;
    if (rhs == kRhsLiftP && B->warm) {
      st[i].warm_starts += 1;
      st[i].warm_accepted += h.warm_used;
    }
    st[i].inner_its_total += h.inner_its;
    st[i].inner_its_max = std::max(st[i].inner_its_max, h.inner_its);
    st[i].refine_steps += h.refine_steps;
    steps = std::max(steps, h.refine_steps);
    its_max = std::max(its_max, h.run_its_max);
    for (int q = 0; q < std::min(h.refine_steps, 8); ++q) run_len[q] = std::max(run_len[q], h.run_len[q]);
  }
  schedule_record(B->sc, steps, run_len, its_max);
  return FDD_OK;
}

// One batched interior solve from the enqueue of its first residual to completion (eager).
int batch_inner(fdd_batch_s* B, hipStream_t s, const BatchCtx& c, BTrack& t, int rhs, int ver,
                const std::vector<char>& live, const fdd_opts& o, std::vector<fdd_stats>& st) {
  enqueue_start(c, t, rhs, ver, o);
  if (!B->sc->calibrated) enqueue_steps(B, c, t, rhs, ver, 1, 30);  // measures the schedule
  else enqueue_steps(B, c, t, rhs, ver, B->sc->steps, -1);
  HIPCHK(hipGetLastError());
  int rc = read_states(B, s);
  if (rc) return rc;
  rc = finish_inner(B, s, c, t, rhs, ver, live, o, st);
  if (rc == FDD_OK) B->sc->calibrated = true;
  return rc;
}

// The network's guesses for every instance's p_G of version v (one forward pass per group of
// instances of equal n, all images in the network's output buffer) and their Galerkin factors.
void enqueue_warm(const fdd_batch_s* B, const BatchCtx& c, int v) {
  launch_b_gather_traces(c, v);
  fdd_cnn_s* C = const_cast<fdd_cnn_s*>(B->warm);
  float* out = cnn_output(C, nullptr);
  for (const auto& g : B->groups)
    (void)cnn_warm_guess_batch(C, c.stream, B->d_traces + (size_t)g.off * B->tmax, B->tmax, g.count,
                               g.n, B->d_lk + g.off, B->d_lmu + g.off, out + g.img);
  launch_b_warm_alpha(c, v);
}

// Everything of outer iteration v up to the synchronization, for the instances still running.
void enqueue_outer(const fdd_batch_s* B, const BatchCtx& c, BTrack& t, int v, const fdd_opts& o) {
  if (B->warm) enqueue_warm(B, c, v);
  enqueue_start(c, t, kRhsLiftP, v, o);
  if (!B->sc->calibrated) enqueue_steps(B, c, t, kRhsLiftP, v, 1, 30);  // measures the schedule
  else enqueue_steps(B, c, t, kRhsLiftP, v, B->sc->steps, -1);
  launch_b_operator(c, v);
  launch_b_outer_tail(c, t.S, v, o.outer_rtol, !o.back_solve);
}

int replay_outer(fdd_batch_s* B, hipStream_t s, const BatchCtx& c, BTrack& t, int v,
                 const fdd_opts& o) {
  // everything the captured launches bake in: the schedule and the options passed by value
  // (the inner and per-step tolerances of the residual kernels, the outer tolerance of the
  // device-side stop test), tolerances as bit patterns
  std::vector<int> key = {v & 1, o.mg_nu, B->sc->steps, B->sc->its, o.back_solve ? 1 : 0};
  key.insert(key.end(), B->sc->step_its, B->sc->step_its + 8);
  push_bits(key, o.step_rtol);
  push_bits(key, o.inner_rtol);
  push_bits(key, o.outer_rtol);
  // the network's buffers and parameters are kernel arguments of a warm-started iteration
  push_bits(key, (uint64_t)(uintptr_t)B->warm);
  if (B->warm) push_bits(key, cnn_binding_id(B->warm));
  auto it = B->graphs.find(key);
  if (it == B->graphs.end()) {
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    enqueue_outer(B, c, t, v, o);
    hipError_t e = hipStreamEndCapture(s, &g);
    if (e != hipSuccess) return fail(FDD_E_HIP, "graph capture: %s", hipGetErrorString(e));
    BGraph ge;
    e = hipGraphInstantiate(&ge.exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(FDD_E_HIP, "graph instantiate: %s", hipGetErrorString(e));
    ge.cur_r = t.cur_r;
    ge.cur_p = t.cur_p;
    ge.S = t.S;
    it = B->graphs.emplace(key, ge).first;
  }
  t.cur_r = it->second.cur_r;
  t.cur_p = it->second.cur_p;
  t.S = it->second.S;
  HIPCHK(hipGraphLaunch(it->second.exec, s));
  return FDD_OK;
}

}  // namespace

extern "C" {

int fdd_batch_create(int count, const fdd_problem* probs, const fdd_ratpc* P, const fdd_ratpc* H,
                     fdd_batch* out) {
  if (!out) return fail(FDD_E_ARG, "null argument");
  *out = nullptr;
  if (count < 1 || !probs || !P || !H) return fail(FDD_E_ARG, "empty batch or null array");
  for (int i = 0; i < count; ++i) {
    int rc = check_problem(probs[i]);
    if (rc) return fail(rc, "batch instance %d: %s", i, fdd_last_error());
    if ((rc = check_table(probs[i], P[i], FDD_RA_PRECOND)) ||
        (rc = check_table(probs[i], H[i], FDD_RA_OPERATOR)))
      return fail(rc, "batch instance %d: %s", i, fdd_last_error());
    if (probs[i]->device != probs[0]->device)
      return fail(FDD_E_ARG, "batch instances on different devices");
    if (probs[i]->dim != 2 || probs[i]->kind != kProblemFacet)
      return fail(FDD_E_ARG, "batch instance %d: batched solves are for the 2D facet problem", i);
  }
  std::vector<fdd_problem_s*> sorted(probs, probs + count);
  std::sort(sorted.begin(), sorted.end());
  if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
    return fail(FDD_E_ARG, "a problem appears twice in the batch (instances need their own workspace)");
  fdd_batch_s* B = new (std::nothrow) fdd_batch_s();
  if (!B) return fail(FDD_E_NOMEM, "out of host memory");
  B->count = count;
  B->device = probs[0]->device;
  B->probs.assign(probs, probs + count);
  B->tabP.assign(P, P + count);
  B->tabH.assign(H, H + count);
  B->max_tiled = 1;
  for (int i = 0; i < count; ++i) B->max_tiled = std::max(B->max_tiled, probs[i]->first_coarse32);
  plan_tiles(B);
  B->sysP_prefix.assign(count + 1, 0);
  B->sysH_prefix.assign(count + 1, 0);
  for (int i = 0; i < count; ++i) {
    B->sysP_prefix[i + 1] = B->sysP_prefix[i] + make_table(P[i]).m;
    B->sysH_prefix[i + 1] = B->sysH_prefix[i] + make_table(H[i]).m;
  }
  B->sysP_total = B->sysP_prefix[count];
  B->sysH_total = B->sysH_prefix[count];
  B->tmax = 1;
  for (int i = 0; i < count; ++i) B->tmax = std::max(B->tmax, (int)probs[i]->NG);
  *out = B;
  return FDD_OK;
}

int fdd_batch_workspace_bytes(fdd_batch B, size_t* bytes) {
  if (!B || !bytes) return fail(FDD_E_ARG, "null argument");
  fdd_batch_s tmp;
  tmp.count = B->count;
  tmp.tmax = B->tmax;
  *bytes = plan_batch(&tmp, nullptr);
  return FDD_OK;
}

int fdd_batch_bind_workspace(fdd_batch B, void* dev, size_t bytes, void* stream) {
  if (!B || !dev) return fail(FDD_E_ARG, "null argument");
  if (((uintptr_t)dev) & 255) return fail(FDD_E_WORKSPACE, "workspace must be 256-byte aligned");
  fdd_batch_s tmp;
  tmp.count = B->count;
  tmp.tmax = B->tmax;
  const size_t need = plan_batch(&tmp, nullptr);
  if (bytes < need) return fail(FDD_E_WORKSPACE, "workspace %zu bytes < %zu needed", bytes, need);
  HIPCHK(hipSetDevice(B->device));
  hipStream_t s = (hipStream_t)stream;
  B->ws = (char*)dev;
  B->ws_bytes = bytes;
  plan_batch(B, B->ws);
  if (!B->h_inst)
    HIPCHK(hipHostMalloc((void**)&B->h_inst, sizeof(BInst) * B->count, hipHostMallocDefault));
  if (!B->h_states)
    HIPCHK(hipHostMalloc((void**)&B->h_states, sizeof(DevState) * B->count, hipHostMallocDefault));
  B->uploaded.clear();
  B->warm_for = nullptr;
  std::vector<ShiftTable> tabs(2 * (size_t)B->count);
  for (int i = 0; i < B->count; ++i) {
    tabs[i] = make_table(B->tabP[i]);
    tabs[B->count + i] = make_table(B->tabH[i]);
  }
  HIPCHK(hipMemsetAsync(B->ws, 0, need, s));
  int rc = upload_tiles(B, s);
  if (rc) return rc;
  B->tiles_dirty = false;
  HIPCHK(hipMemcpyAsync(B->d_sysP, B->sysP_prefix.data(), sizeof(int) * (B->count + 1),
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(B->d_sysH, B->sysH_prefix.data(), sizeof(int) * (B->count + 1),
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(B->d_tab, tabs.data(), sizeof(ShiftTable) * tabs.size(),
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return FDD_OK;
}

int fdd_batch_set_mid_tile(fdd_batch B, int edge) {
  if (!B) return fail(FDD_E_ARG, "null batch");
  if (edge != 0 && edge != kMidTile && edge != kTile)
    return fail(FDD_E_ARG, "intermediate-level tile edge must be 0, %d or %d (got %d)", kMidTile,
                kTile, edge);
  if (edge == B->mid_tile) return FDD_OK;
  B->mid_tile = edge;
  plan_tiles(B);
  // captured graphs bake in the grid sizes
  for (auto& kv : B->graphs)
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
  B->graphs.clear();
  B->tiles_dirty = true;
  return FDD_OK;
}

int fdd_batch_tile_edges(fdd_batch B, int* levels, int* edges) {
  if (!B || !levels) return fail(FDD_E_ARG, "null argument");
  *levels = B->max_tiled;
  if (edges)
    for (int l = 0; l < B->max_tiled; ++l) edges[l] = B->tile_edge[l];
  return FDD_OK;
}

int fdd_solve_batched(fdd_batch B, const double* const* b, double* const* x, const fdd_opts* opts,
                      void* stream, fdd_stats* stats) {
  const auto t_start = std::chrono::steady_clock::now();
  if (!B || !b || !x) return fail(FDD_E_ARG, "null argument");
  if (!B->ws) return fail(FDD_E_WORKSPACE, "no batch workspace bound");
  for (int i = 0; i < B->count; ++i) {
    if (!b[i] || !x[i]) return fail(FDD_E_ARG, "batch instance %d: null vector", i);
    if (!B->probs[i]->ws) return fail(FDD_E_WORKSPACE, "batch instance %d: no workspace bound", i);
  }
  fdd_opts o;
  if (opts) o = *opts;
  else fdd_opts_default(&o);
  if (!opts_ok(&o)) return fail(FDD_E_ARG, "invalid options");
  if (o.precision != FDD_MIXED)
    return fail(FDD_E_ARG, "batched solves run FP32 multigrid-PCG inside FP64 refinement only");
  B->warm = nullptr;
  if (o.warmstart) {
    // the network must take every instance's n and the whole batch in its output buffer
    const fdd_cnn_s* C = (const fdd_cnn_s*)o.warmstart;
    for (int i = 0; i < B->count; ++i) {
      int rc0 = cnn_check_for(C, B->probs[i]->n);
      if (rc0) return fail(rc0, "batch instance %d: %s", i, fdd_last_error());
    }
    if (cnn_batch_max(C) < B->count)
      return fail(FDD_E_ARG, "the network takes %d images per pass, the batch has %d instances",
                  cnn_batch_max(C), B->count);
    if (B->warm_for != C) {
      // rows ordered by n: one forward pass per group of equal n
      std::vector<int> order(B->count);
      for (int i = 0; i < B->count; ++i) order[i] = i;
      std::stable_sort(order.begin(), order.end(),
                       [&](int a, int b2) { return B->probs[a]->n < B->probs[b2]->n; });
      B->slot.assign(B->count, 0);
      B->groups.clear();
      std::vector<double> lk(B->count), lmu(B->count);
      int64_t img = 0;
      for (int r = 0; r < B->count; ++r) {
        const fdd_problem_s* Q = B->probs[order[r]];
        B->slot[order[r]] = r;
        lk[r] = std::log10(Q->K);
        lmu[r] = std::log10(Q->mu);
        if (B->groups.empty() || B->groups.back().n != Q->n) {
          if (!B->groups.empty()) {
            const auto& g = B->groups.back();
            img += (int64_t)g.count * (g.n - 1) * (g.n - 1);
          }
          B->groups.push_back({Q->n, r, 0, img});
        }
        B->groups.back().count += 1;
      }
      const auto& last = B->groups.back();
      int64_t cap = 0;
      (void)cnn_output(const_cast<fdd_cnn_s*>(C), &cap);
      if (img + (int64_t)last.count * (last.n - 1) * (last.n - 1) > cap)
        return fail(FDD_E_ARG, "the batch's guesses exceed the network's output buffer");
      HIPCHK(hipSetDevice(B->device));
      HIPCHK(hipMemcpy(B->d_lk, lk.data(), sizeof(double) * B->count, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(B->d_lmu, lmu.data(), sizeof(double) * B->count, hipMemcpyHostToDevice));
      B->warm_for = C;
    }
    B->warm = C;
  }
  B->sc = &B->scheds[std::make_tuple(o.mg_nu, o.step_rtol, 0)];
  HIPCHK(hipSetDevice(B->device));
  hipStream_t us = (hipStream_t)stream;
  hipStream_t s = us;
  if (B->hook.kind != kTimeNone) o.use_graph = 0;  // timed launches carry their own events
  if (o.use_graph) {
    if (!B->gstream) {
      HIPCHK(hipStreamCreateWithFlags(&B->gstream, hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&B->ev_in, hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&B->ev_out, hipEventDisableTiming));
    }
    HIPCHK(hipEventRecord(B->ev_in, us));
    HIPCHK(hipStreamWaitEvent(B->gstream, B->ev_in, 0));
    s = B->gstream;
  }
  const int n = B->count;
  std::vector<fdd_stats> st(n);
  for (auto& q : st) {
    std::memset(&q, 0, sizeof(q));
    q.true_rel_res = -1.0;
  }
  auto finish = [&](int code) -> int {
    if (o.use_graph) {
      (void)hipEventRecord(B->ev_out, s);
      (void)hipStreamWaitEvent(us, B->ev_out, 0);
    }
    const double ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    for (int i = 0; i < n; ++i) {
      if (code < 0) st[i].status = code;
      st[i].t_solve_ms = ms;
    }
    if (stats) std::memcpy(stats, st.data(), sizeof(fdd_stats) * n);
    return code;
  };
  if (B->tiles_dirty) {
    int rc0 = upload_tiles(B, s);
    if (rc0) return finish(rc0);
    B->tiles_dirty = false;
  }
  // descriptors (uploaded when a vector, a problem's workspace or the tile plan changed)
  std::vector<BInst> cur(n);
  for (int i = 0; i < n; ++i) cur[i] = make_inst(B, i, b[i], x[i]);
  if (B->uploaded.size() != (size_t)n ||
      std::memcmp(B->uploaded.data(), cur.data(), sizeof(BInst) * n) != 0) {
    std::memcpy(B->h_inst, cur.data(), sizeof(BInst) * n);
    HIPCHK(hipMemcpyAsync(B->d_inst, B->h_inst, sizeof(BInst) * n, hipMemcpyHostToDevice, s));
    B->uploaded = cur;
  }
  const std::vector<char> all(n, 1);
  BatchCtx c0 = make_bctx(B, s, o.mg_nu, 0), c1 = make_bctx(B, s, o.mg_nu, 1);
  BTrack t;
  // 1. g = b_G - A_GI A_II^{-1} b_I for every instance
  int rc = batch_inner(B, s, c0, t, kRhsB, 0, all, o, st);
  if (rc) return finish(rc);
  launch_b_rhs_reduce(c0, t.S);
  if (!o.back_solve) launch_b_xI_init(c0, t.S);
  // 2. outer PCG from x_G = 0 (device-side convergence test per instance)
  launch_b_precond_init(c0, o.outer_rtol);
  HIPCHK(hipGetLastError());
  if ((rc = read_states(B, s))) return finish(rc);
  // lifted-p solves have their own schedule, warm-started ones another
  B->sc = &B->scheds[std::make_tuple(o.mg_nu, o.step_rtol, B->warm ? 2 : 1)];
  std::vector<char> live(n);
  int nlive = 0;
  for (int i = 0; i < n; ++i) {
    if (B->h_states[i].breakdown)
      return finish(fail(FDD_E_BREAKDOWN, "batch instance %d: preconditioner not positive", i));
    live[i] = !B->h_states[i].outer_done;
    nlive += live[i];
  }
  int v = 0;
  while (nlive > 0 && v < o.outer_maxit) {
    if (o.use_graph && B->sc->calibrated) {
      if ((rc = replay_outer(B, s, c1, t, v, o))) return finish(rc);
    } else {
      enqueue_outer(B, c1, t, v, o);
    }
    HIPCHK(hipGetLastError());
    if ((rc = read_states(B, s))) return finish(rc);
    bool short_solve = false;
    for (int i = 0; i < n; ++i)
      if (live[i] && !B->h_states[i].solve_done && !B->h_states[i].breakdown) short_solve = true;
    if ((rc = finish_inner(B, s, c1, t, kRhsLiftP, v, live, o, st))) return finish(rc);
    B->sc->calibrated = true;
    if (short_solve) {
      // the schedule was short for some instance: its tail was skipped; now that every interior
      // solve is complete, repeat the tail (it depends on version-v data only)
      launch_b_outer_tail(c1, t.S, v, o.outer_rtol, !o.back_solve);
      HIPCHK(hipGetLastError());
      if ((rc = read_states(B, s))) return finish(rc);
    }
    ++v;
    for (int i = 0; i < n; ++i) {
      if (!live[i]) continue;
      const DevState& h = B->h_states[i];
      if (h.breakdown)
        return finish(fail(h.breakdown & 4 ? FDD_E_NONFINITE : FDD_E_BREAKDOWN,
                           "batch instance %d: outer PCG breakdown (flags %d, p.Sp = %g)", i,
                           h.breakdown, h.o_pq));
      st[i].outer_its = v;
      if (h.outer_done) {
        live[i] = 0;
        --nlive;
      }
    }
  }
  // 3. back-substitution x_I = A_II^{-1} (b_I / K - A_IG x_G) for every instance: accumulated
  //    during the outer PCG, or one more batched interior solve
  B->sc = &B->scheds[std::make_tuple(o.mg_nu, o.step_rtol, 0)];
  if (o.back_solve && (rc = batch_inner(B, s, c0, t, kRhsBack, v, all, o, st))) return finish(rc);
  launch_b_scatter(c0, t.S, v, !o.back_solve);
  HIPCHK(hipGetLastError());
  if ((rc = read_states(B, s))) return finish(rc);
  int code = FDD_OK;
  for (int i = 0; i < n; ++i) {
    const DevState& h = B->h_states[i];
    const int fv = h.outer_done ? h.o_ver : v;
    const double rho = h.o_rho[fv & 1];
    st[i].rel_precond_res = h.o_rho0 > 0 ? std::sqrt(std::max(rho, 0.0) / h.o_rho0) : 0.0;
    st[i].status = h.outer_done ? FDD_OK : FDD_NOT_CONVERGED;
    if (!h.outer_done) code = FDD_NOT_CONVERGED;
  }
  return finish(code);
}

int fdd_batch_set_kernel_timer(fdd_batch B, int kind, double split_us) {
  if (!B) return fail(FDD_E_ARG, "null batch");
  if (!(split_us >= 0)) return fail(FDD_E_ARG, "split_us must be >= 0");
  if (kind < FDD_KT_NONE || kind > FDD_KT_COARSE) return fail(FDD_E_ARG, "bad timer kind");
  HIPCHK(hipSetDevice(B->device));
  if (kind != FDD_KT_NONE && !B->hook.ev) {
    const int cap = 4096;
    B->hook.ev = new (std::nothrow) hipEvent_t[2 * cap];
    if (!B->hook.ev) return fail(FDD_E_NOMEM, "out of host memory");
    for (int i = 0; i < 2 * cap; ++i) HIPCHK(hipEventCreate(&B->hook.ev[i]));
    B->hook.cap = cap;
  }
  B->timer_split_ms = split_us * 1e-3;
  B->hook.kind = kind;
  B->hook.used = 0;
  B->hook.skipped = 0;
  B->timed_launches = B->timed_long = 0;
  B->timed_ms = B->timed_long_ms = 0.0;
  return FDD_OK;
}

int fdd_batch_get_kernel_timer(fdd_batch B, int64_t* launches, double* total_ms,
                               int64_t* long_launches, double* long_ms, int64_t* untimed) {
  if (!B) return fail(FDD_E_ARG, "null batch");
  if (launches) *launches = B->timed_launches;
  if (total_ms) *total_ms = B->timed_ms;
  if (long_launches) *long_launches = B->timed_long;
  if (long_ms) *long_ms = B->timed_long_ms;
  if (untimed) *untimed = B->hook.skipped;
  return FDD_OK;
}

void fdd_batch_destroy(fdd_batch B) {
  if (!B) return;
  if (B->hook.ev) {
    for (int i = 0; i < 2 * B->hook.cap; ++i) (void)hipEventDestroy(B->hook.ev[i]);
    delete[] B->hook.ev;
  }
  for (auto& kv : B->graphs)
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
  if (B->gstream) (void)hipStreamDestroy(B->gstream);
  if (B->ev_in) (void)hipEventDestroy(B->ev_in);
  if (B->ev_out) (void)hipEventDestroy(B->ev_out);
  if (B->h_inst) (void)hipHostFree(B->h_inst);
  if (B->h_states) (void)hipHostFree(B->h_states);
  delete B;
}

}  // extern "C"
