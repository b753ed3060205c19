// Solver entry points used by the C ABI layer.
#pragma once

#include <vector>

#include "common.h"

namespace stokes {

struct SolveStats {
  int inner_u = 0, inner_p = 0, outer = 0, sweeps = 0;
  double seconds_orth = 0;
  std::vector<double> rel_res;  // per right-hand side, final true residual
  std::vector<double> inv_bn;   // per right-hand side, 1 / ||b|| (0 for b = 0)
  std::vector<double> hist;     // per outer iteration: estimated relative residual (max over right-hand sides)
};

// Solve K x = b with b = (F, g) in the internal FP64 layout, x = (xu, xp) as
// initial guess and result.  method 0 = coupled FGMRES, 1 = Schur FCG.
// Returns STOKES_OK or STOKES_NOT_CONVERGED.
// x_zero: (xu, xp) hold zero on entry, so the first residual is b itself.
int solve_internal(stokes_ctx* c, const stokes_solve_opts& o, int method, int nrb, const double* F, const double* g,
                   double* xu, double* xp, SolveStats& st, bool x_zero);

// One pressure-correction step from p_old (internal layout, may be null):
// u and p in xu / xp.  rel_res = the largest final relative residual of its
// three linear solves.
int projection_internal(stokes_ctx* c, const stokes_solve_opts& o, int nrb, const double* F, const double* g,
                        const double* pold, double* xu, double* xp, SolveStats& st);

// z = the degree-`degree` Chebyshev-Jacobi polynomial of A_II applied to r
// (internal velocity layout, W = dim nrb values per row): the FIXED-mode
// velocity preconditioner of the coupled solves, in T (FP32: the
// half-precision A_II D^{-1} copy and the bfloat16 direction).
template <class T>
void vel_cheb_apply(stokes_ctx* c, int nrb, int degree, const T* r, T* z);

}  // namespace stokes
