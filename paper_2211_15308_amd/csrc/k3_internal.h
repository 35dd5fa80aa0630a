// Types and launchers of the 3D solver's kernels (kernels_3d.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace fdd {

constexpr int kPart3 = 1024;  // blocks (and partials) of the interior dot-product kernels
constexpr int kPartF = 64;    // blocks per system of the face kernels
constexpr int kMaxSys3 = 80;  // shifted systems in one face batch

// interior right-hand side: sb b (compact interior order) + sg g on the plane next to Gamma
struct Rhs3 {
  const double* b;
  double sb;
  const double* g;
  double sg;
};

// device scalars of the interior PCG
struct State3 {
  double ff, rr, rho, alpha, beta, tol2;
  int its, breakdown;
};

// shift table of a face batch: system s is (alpha_s A_G + beta_s M_G) y = rhs, weight coef_s
struct Shift3 {
  double alpha[kMaxSys3], beta[kMaxSys3], coef[kMaxSys3];
  double d0;
  int m;
};

// device scalars of a face batch (per system)
struct FaceCG {
  double rr0[kMaxSys3], rho[kMaxSys3], alpha[kMaxSys3], beta[kMaxSys3];
  int its[kMaxSys3], bad[kMaxSys3];
};

void k3_launch_rb(hipStream_t s, double* u, const double* f, int nf, int red, int from_zero,
                  const int* stop);
void k3_launch_resid(hipStream_t s, const double* u, const double* f, double* t, int nf,
                     const int* stop);
void k3_launch_restrict(hipStream_t s, const double* t, double* fc, int nf, int nc,
                        const int* stop);
void k3_launch_prolong(hipStream_t s, const double* ec, double* u, int nf, int nc,
                       const int* stop);
void k3_launch_coarse(hipStream_t s, const double* f, double* u, int nc, const double* cinv,
                      const int* stop);
void k3_launch_rhs(hipStream_t s, const Rhs3& rhs, double* f, int nf);
void k3_launch_dot(hipStream_t s, const double* a, const double* b, int nf, double* part,
                   const int* stop);
void k3_launch_apply(hipStream_t s, const double* p, double* q, int nf, double* part,
                     const int* stop);
void k3_launch_update(hipStream_t s, double* x, double* r, const double* p, const double* q,
                      int nf, const State3* st, double* part, const int* stop);
void k3_launch_pupdate(hipStream_t s, double* p, const double* z, int nf, const State3* st,
                       int first, const int* stop);
void k3_launch_scalars(hipStream_t s, State3* st, const double* part0, const double* part1,
                       int kind, int* stop);
void k3_launch_gather(hipStream_t s, const double* u, int nf, double* out, const double* xg);
void kf_launch_apply(hipStream_t s, const double* x, int x_shared, double* y, int nf, double h,
                     int m, const Shift3* tab, double* part, const int* done);
void kf_launch_dst(hipStream_t s, const double* S, const double* B, double* C, int nf, int m,
                   int left, const int* done);
void kf_launch_diag(hipStream_t s, double* z, int nf, int n, double h, int m, const Shift3* tab,
                    const int* done);
void kf_launch_dot(hipStream_t s, const double* a, const double* b, int nf, int m, double* part,
                   const int* done);
void kf_launch_axpy(hipStream_t s, double* y, double* r, double* p, const double* q,
                    const double* z, int nf, int m, const double* coef, int kind, int first,
                    const int* done);
void kf_launch_scalars(hipStream_t s, FaceCG* cg, const double* part0, const double* part1, int m,
                       int kind, int* done, double tol2);
void kf_launch_combine(hipStream_t s, const double* ys, int m, int nf, double h, const Shift3* tab,
                       int op, const double* x, double* tmp, double* out, double d0);
void kf_launch_schur(hipStream_t s, const double* p, const double* u, int nf, double h, double K,
                     double gamma, const double* Hp, double* y, double* part);
void k3_launch_full_operator(hipStream_t s, int n, double K, double gamma, const double* x,
                             const double* Hx, double* y, const double* b, double* part);
void kf_launch_outer_axpy(hipStream_t s, double* x, double* r, double* p, const double* y,
                          const double* z, int64_t N, double a);
// out = (accumulate ? out : 0) + c u over n elements
void k3_launch_scale_add(hipStream_t s, double* out, const double* u, double c, int accumulate,
                         int64_t n);
void kf_launch_rhs_reduce(hipStream_t s, const double* bG, const double* w, int nf, double h,
                          double* g, double* xg);
void kf_launch_vdot(hipStream_t s, const double* a, const double* b, int64_t N, double* part);
void kf_launch_bcast(hipStream_t s, const double* src, double* dst, int nf, double h, int m,
                     int mass);

}  // namespace fdd
