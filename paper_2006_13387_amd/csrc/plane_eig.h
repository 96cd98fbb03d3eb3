// Per-neighbourhood state of the subspace iterations on row- or
// plane-blocked pencils (the 3D heat pencils and the 2D elasticity
// pencils), kept in device memory between the iteration's kernels.
#pragma once
#include "common.h"

namespace msp {

struct Eig3State {
  int done, conv;
  double theta[MAXM], theta_old[MAXM];
  double GA[MAXM * MAXM], GM[MAXM * MAXM];
  double V[MAXM * MAXM];      // Ritz coefficients, columns in ascending order
};

}  // namespace msp
