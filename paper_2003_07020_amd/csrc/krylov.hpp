// Device-side pieces of the FGMRES outer iteration (FP64), beyond the declarations shared by
// every source in rfde_internal.hpp.
#pragma once
#include "rfde_internal.hpp"

namespace rfde {

// CGS2 of w against the nvec (<= 64) basis vectors V (stride N): w -= V (h1 + h2) with
// h1 = V^T w and h2 = V^T (w - V h1), in three sweeps over V; out[0..nvec) = h1,
// out[CGS2_H2 + i] = h2_i, out[CGS2_NRM] = |w| after both corrections (out: 256 doubles).
constexpr int CGS2_H2 = 64, CGS2_NRM = 128;
int launch_cgs2(const Plan& p, const double* V, int nvec, double* w, double* out);

}  // namespace rfde
