// Types and launchers of the 3D solver's kernels (kernels_3d.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace fdd {

constexpr int kPart3 = 1024;  // blocks (and partials) of the face-vector and full-operator reductions
constexpr int kPartF = 64;    // blocks per system of the face kernels
constexpr int kMaxSys3 = 80;  // shifted systems in one face batch

// interior right-hand side: sb b (compact interior order) + sg g on the plane next to Gamma
struct Rhs3 {
  const double* b;
  double sb;
  const double* g;
  double sg;
};

// device scalars of the interior solve: the PCG run (rho[k & 1] = r_k . z_k; ff = |r_0|^2 of the
// run, its = iterations of the run) and, around it, the FP64 refinement (F2 = |F|^2 of the right-
// hand side, run = refinement step; done: the solve has converged; its_total = iterations of all
// runs).  A run stops at |r|^2 <= max(tol2 ff, tol2s F2); the solve at |F - L7 x|^2 <= tol2s F2.
constexpr int kRuns3 = 12;  // refinement steps of one interior solve at most
struct State3 {
  double ff, rr, rho[2], tol2, tol2s, F2;
  int its, breakdown, run, done, its_total;
  int run_its[kRuns3];  // iterations of each run (recorded when the next step starts)
};

// levels of the one-workgroup coarse V-cycle (padded grids of edge lev + 2 in LDS)
constexpr int kCvcLevels = 4;
constexpr int kCvcMax = 15;  // finest level it takes
struct Cvc3 {
  int nl;
  int lev[kCvcLevels];
};
int k3_cvc_fits(const Cvc3& L);  // the levels fit the kernel's LDS

// block partials of the level-0 reduction kernels (at most ceil(nf / rows) nf < 1024 + nf)
constexpr int kPart0 = 2048;
int k3_rows_red(int nf);  // rows per block of the level-0 reduction kernels

// shift table of a face batch: system s is (alpha_s A_G + beta_s M_G) y = rhs, weight coef_s
struct Shift3 {
  double alpha[kMaxSys3], beta[kMaxSys3], coef[kMaxSys3];
  double d0;
  int m;
};

// device scalars of a face batch (per system; rho[k & 1] = r_k . z_k)
struct FaceCG {
  double rr0[kMaxSys3], rho[2][kMaxSys3];
  int its[kMaxSys3], bad[kMaxSys3];
};
constexpr int kPFS = 256;      // partials per system of the face kernels (>= 64 and ceil(nf / 16)^2)
constexpr int kFaceMax = 255;  // largest face edge nf (n <= 256)
constexpr int kFaceRows = 256;  // kFaceMax rounded up to whole row groups of 16

// multigrid and PCG kernels of the interior solve (see kernels_3d.hip for what each computes), in
// the working precision R (float: inside FP64 refinement; double); rows: grid rows per block;
// pin/np: partials read; part: partials written
template <typename R>
void k3_launch_zp(hipStream_t s, int mode, const R* f, R* u, int nf, int rows, const R* q, R* rnew,
                  R* x, const R* p, State3* st, const double* pin, int np, double* part, int* stop);
template <typename R>
void k3_launch_hs(hipStream_t s, R* u, const R* f, int nf, int red, int check, State3* st,
                  const double* pin, int np, int* stop);
template <typename R>
void k3_launch_rr(hipStream_t s, const R* u, const R* f, R* fc, int nf, int nc, int check,
                  State3* st, const double* pin, int np, int* stop);
template <typename R>
void k3_launch_pr(hipStream_t s, const R* u, const R* ec, const R* f, R* uo, int nf, int nc,
                  int* stop);
template <typename R>
void k3_launch_hsz(hipStream_t s, R* u, const R* f, int nf, int rows, double* part, int* stop);
template <typename R>
void k3_launch_apply1(hipStream_t s, const R* z, const R* pold, R* pnew, R* q, int nf, int rows,
                      State3* st, const double* pin, int np, double* part, int* stop);
template <typename R>
void k3_launch_cvc(hipStream_t s, const R* fin, R* uout, const Cvc3& L, const double* cinv,
                   int nu, int* stop);
// FP64 refinement step (first: r = F; else x' = x + e, r = F - L7 x'), r also as FP32
void k3_launch_ir(hipStream_t s, int first, const double* F, const double* xin, const float* e,
                  double* xout, float* r32, int nf, int rows, State3* st, double* part);
void k3_launch_rhs(hipStream_t s, const Rhs3& rhs, double* f, int nf);
void k3_launch_gather(hipStream_t s, const double* u, int nf, double* out, const double* xg);
// batched face CG (kernels_3d.hip): start (r = src or M src, y = 0), the two vector passes of
// an iteration, and the preconditioner z = S D^{-1} S r (four DST passes; check 1: start test,
// 2: convergence test, on the |r|^2 partials pin; part: r . z partials, kf_tiles(nf) per system)
void kf_launch_start(hipStream_t s, const double* src, double* r, double* y, int nf, double h,
                     int m, int mass, double* part);
void kf_launch_apply1(hipStream_t s, const double* z, const double* pold, double* pnew, double* q,
                      int nf, double h, int m, const Shift3* tab, FaceCG* cg, const double* pin,
                      int cnt, double* part, int* done);
// the rest of a face-CG iteration after kf_launch_apply1: y += alpha p, r' = r - alpha q (pq: the
// p . q partials), the convergence test, z = preconditioner(r'), r' . z partials to part
void kf_launch_face_update_prec(hipStream_t s, const double* S, const double* r, double* rnew,
                                const double* q, const double* p, double* y, double* ft, double* z,
                                int nf, int n, double h, int m, const Shift3* tab, FaceCG* cg,
                                const double* pq, double tol2, double* part, int* done);
void kf_launch_prec(hipStream_t s, const double* S, const double* r, double* ft, double* z, int nf,
                    int n, double h, int m, const Shift3* tab, FaceCG* cg, const double* pin,
                    double tol2, int check, double* part, int* done);
int kf_tiles(int nf);
void kf_launch_combine(hipStream_t s, const double* ys, int m, int nf, double h, const Shift3* tab,
                       int op, const double* x, double* tmp, double* out, double d0);
void kf_launch_schur(hipStream_t s, const double* p, const double* u, int nf, double h, double K,
                     double gamma, const double* Hp, double* y, double* part);
void k3_launch_full_operator(hipStream_t s, int n, double K, double gamma, const double* x,
                             const double* Hx, double* y, const double* b, double* part);
// outer PCG vector steps with the device scalar *coef: x += a p, r -= a y (x given), or
// p = z + a p
void kf_launch_outer_axpy(hipStream_t s, double* x, double* r, double* p, const double* y,
                          const double* z, int64_t N, const double* coef);
// out = (accumulate ? out : 0) + c u over n elements (c = *coef when coef is given)
void k3_launch_scale_add(hipStream_t s, double* out, const double* u, double c, int accumulate,
                         int64_t n, const double* coef = nullptr);
// slots of the outer PCG's device scalars
enum { kSc3Rho0 = 0, kSc3Rho, kSc3Rz, kSc3Pq, kSc3Alpha, kSc3Beta, kSc3E2, kSc3B2, kSc3Count };
void k3_launch_sum_partials(hipStream_t s, const double* part, int count, int stride, double* sc,
                            int slot);
void k3_launch_outer_scalars(hipStream_t s, double* sc, int mode);
void kf_launch_rhs_reduce(hipStream_t s, const double* bG, const double* w, int nf, double h,
                          double* g, double* xg);
void kf_launch_vdot(hipStream_t s, const double* a, const double* b, int64_t N, double* part);

}  // namespace fdd
