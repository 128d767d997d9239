// Internal interface of the adjoint kernels (rsst_adjoint.hip).  Not part of
// the ABI.
#pragma once

#include <hip/hip_runtime.h>

namespace rsstk {

struct AdjointPlan {
  int ndim;
  int n[3];
  int refl_lo[3], refl_hi[3];
  double inv_dx[3];
  double g[3];
  double gamma, xi;
  int form;
  long long ncell;
  double* work;  // adjoint_workspace_doubles(ndim, ncell) doubles
};

// Doubles of adjoint workspace for a grid of ncell cells, n[0..ndim-1] per
// axis.
size_t adjoint_workspace_doubles(int ndim, const int n[3], long long ncell);

// The workspace from this offset on must be zero before the first adjoint
// step (the run accumulator of a 2D grid; every run leaves it at zero).
size_t adjoint_zeroed_offset(int ndim, const int n[3], long long ncell);

// lam <- (dU'/dU)^T lam for the step U -> U' of fixed dt, whose stage value
// U1 = U + dt R(U) is given; dJdxi += (dU'/dxi)^T lam (device scalar).
// defer (2D grids): the dJ/dxi share goes into the per-tile run accumulator
// instead, folded into dJdxi by launch_adjoint_xi_fold.
hipError_t launch_adjoint_step(const AdjointPlan& p, const double* U, const double* U1, double* lam, double dt,
                               double* dJdxi, bool defer, hipStream_t s);
hipError_t launch_adjoint_xi_fold(const AdjointPlan& p, double* dJdxi, hipStream_t s);

}  // namespace rsstk
