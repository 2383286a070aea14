// Device-side pieces of the FGMRES outer iteration (FP64), beyond the declarations shared by
// every source in rfde_internal.hpp.
//
// Arnoldi basis without the third sweep.  The stored basis vectors u_0..u_j are the CGS
// vectors after the first projection (u_0 = r); the orthonormal basis is V = U R^{-1} with R
// upper triangular: column k of R holds the second-projection coefficients of u_k and, on the
// diagonal, the norm of u_k after that projection.  CGS2 of a new vector w then needs two
// sweeps over U instead of three over V plus a normalisation:
//   sweep A:  a = U^T w;                  h1 = R^{-T} a (= V^T w),  c1 = R^{-1} h1
//   sweep B:  w1 = w - U c1 (= w - V h1), b = U^T w1, s = |w1|^2;  h2 = R^{-T} b (= V^T w1)
//   new column of R: (h2, n) with n = sqrt(s - |h2|^2) = |w1 - V h2|; u_{j+1} = w1.
// h1 + h2 and n are CGS2's Hessenberg column: w = V (h1 + h2) + n v_{j+1}.  The device keeps
// Q = R^{-1} (its new column is (-Q h2 / n, 1 / n)), so the small coefficient maps between the
// sweeps are products that one wave computes with a lane per entry.
#pragma once
#include "rfde_internal.hpp"

namespace rfde {

// Layout of the Arnoldi results written per step to a host-visible buffer `hout` (pinned host
// memory mapped into the device address space, read by the host after a stream
// synchronisation): [0, 64) h1, [CGS2_H2, +64) h2, CGS2_NRM n (the Hessenberg subdiagonal).
// Layout of the plan's device scalar area `redout` (CGS2_OUT_SIZE doubles):
//   [0, 64)          norms and the solution coefficients at a restart (set by the host)
//   [CGS2_C, +64)    c1, the first projection's coefficients in the U basis
//   [CGS2_VS, +65)   1 / |u_k|, the scale that turns u_k into a unit preconditioner input
constexpr int CGS2_H2 = 64, CGS2_NRM = 128, CGS2_C = 192, CGS2_VS = 256;
constexpr int CGS2_OUT_SIZE = 512;
// R^{-1} (column-major, leading dimension CGS2_R_LD) sits in the plan's partials buffer `red`
// after the CGS2_R_OFF reduction partials.
constexpr int CGS2_R_LD = 65;
constexpr size_t CGS2_R_OFF = (size_t)70 * 1024;
constexpr size_t CGS2_RED_SIZE = CGS2_R_OFF + (size_t)CGS2_R_LD * CGS2_R_LD;

// Start of a restart cycle: u_0 = r with |r| = beta: R^{-1}(0,0) = out[CGS2_VS] = 1 / beta.
int launch_cgs2_start(const Plan& p, double beta, double* out);
// Step with nvec = j + 1 stored vectors U (stride N, <= 64): orthogonalises w (in place, it
// becomes u_{j+1}), writes h1, h2 and n to hout, appends column nvec of R^{-1} and
// out[CGS2_VS + nvec].
int launch_cgs2(const Plan& p, const double* U, int nvec, double* w, double* out, double* hout);
// Step (a) of P^-1 with its input scaled by the device scalar *vs (vs == nullptr: by 1).
int launch_time_fwd_scaled(const Plan& p, const double* v, void* z1, const double* vs);

}  // namespace rfde
