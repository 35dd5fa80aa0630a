// PCG preconditioned by a multigrid V-cycle on a typed-ELL hierarchy (host orchestration of the
// kernels of kernels_hdiv.hip).  Used by the H(div) problem's interior block A^00 and by the
// Stokes blocks of the Darcy-Stokes preconditioner.
#pragma once

#include "hdiv_internal.h"

namespace fdd {

// A hierarchy with its PCG vectors and device state (all device pointers in one workspace).
//   lev[0..nlev)  levels, finest first (lev[l].P / R: transfers to level l + 1)
//   cinv          dense row-major inverse of the coarsest matrix; null: the coarsest level is
//                 smoothed once from zero instead (with nlev = 1: one damped patch-Jacobi step,
//                 i.e. the patch smoother itself is the preconditioner)
//   theta         damping of the additive Schwarz smoother
//   n0            unknowns of the finest level
//   r, z, q       n0 each; p: 2 n0 (two directions, alternating); partials: 2 kHdPartials
//   st, hst       device state and its pinned host copy
struct EllHier {
  const HdLevel* lev = nullptr;
  int nlev = 0;
  const double* cinv = nullptr;
  double theta = 0.5;
  int n0 = 0;
  double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
  double* partials = nullptr;
  HdState* st = nullptr;
  HdState* hst = nullptr;
};

// x = V b on level l (V(nu, nu) from x_0 = 0); kernels return at once once stop->done is set.
void ell_vcycle(const EllHier& H, hipStream_t s, int nu, int l, const double* b, double* x,
                const HdState* stop);

// PCG for A u = f (A = lev[0].A, u_0 = 0) to ||f - A u|| <= rtol ||f||, at most maxit iterations.
// As many iterations as *hint are enqueued ahead of the first read-back of the device state
// (kernels past the stop return at once); *hint is updated to the count taken.  `what` names the
// solve in error messages.  Returns FDD_OK, FDD_NOT_CONVERGED or an error; *its the count.
int ell_pcg(const EllHier& H, hipStream_t s, int nu, double rtol, int maxit, const double* f,
            double* u, int* hint, int* its, const char* what);

// Reads the device state into the pinned copy (stream-ordered, then synchronizes).
int ell_read_state(const EllHier& H, hipStream_t s);

}  // namespace fdd
