// Precision schedule of a run (host only, no HIP): which directional steps
// run their contractions in the requested reduced precision, the a-priori
// bound on the resulting ln Z/N error against the FP64 result, and the
// cheapest precision that meets a tolerance.
//
// Error model.  The contractions of step k in reduced precision perturb the
// coarse tensor T_k by rounding of relative size ~u_p (FP32 2^-24, split
// BF16 ~2^-17).  T_k stands for 2^k sites, so the perturbation moves
// ln Z / N by ~2^-k times a model-dependent factor; ln Z / N is a sum of the
// steps' log-norms weighted 2^-k (Sec. 2), and a perturbation made at step k
// enters only through that weight and what follows it.  Measured on the
// Ising and XY workloads (Ising at T = 2.0, T_c, 2.5 with D_cut 32, 64, 80;
// XY with n_max = 4 at beta 0.6 .. 1.6 with D_cut 24, 48, 80; the steps from
// k0 on reduced, all others FP64), the relative change of ln Z/N divided by
// sum_{reduced k} 2^-k reaches at most 7.8e-6 (FP32) and 3.5e-5 (split BF16),
// largest in the disordered XY phase; kErrPerStep holds about 2.5 times
// these.  A run whose steps k >= k0 are reduced therefore has a relative error
// below  kErrPerStep[p] * sum_{k >= k0, reduced} 2^-k  <=  kErrPerStep[p] 2^{1-k0}.
// Steps before the steady state (a leg still smaller than D_cut) are always
// FP64; `tol` > 0 moves k0 later until the bound meets it.
#pragma once

#include <algorithm>
#include <climits>
#include <cmath>

#include "../../include/hotrg.h"

namespace hotrg {

// relative ln Z/N error a reduced step k may add, times 2^k (by precision)
constexpr double kErrPerStep[3] = {0.0, 2.0e-5, 1.0e-4};

// Relative residual at which the block eigensolver of a step in precision p
// stops.  The environment of a reduced step carries rounding of relative size
// ~u_p (FP32 2^-24, split BF16 ~2^-17), which already moves its eigenvectors
// by ~u_p / gap; a residual below 2^-10 u_p adds a thousandth of that, so
// the sweeps past it buy nothing the step's result can show.  FP64 steps
// iterate to 5e-14.
constexpr double kEnvRounding[3] = {0.0, 5.9604644775390625e-08, 7.62939453125e-06};
inline double eig_tolerance(int p) {
  return std::max(5e-14, std::ldexp(kEnvRounding[p], -10));
}

// Whole-step contraction rates on one MI355X (TFLOP/s of algorithmic flops,
// measured at D_cut = 64) used to compare precisions at admission.
constexpr double kStepRate[3] = {65.0, 120.0, 270.0};

// First step (1-based) that may run in precision p for tolerance tol.
inline int first_reduced_step(int p, double tol) {
  if (p == HOTRG_FP64) return INT_MAX;
  if (!(tol > 0.0)) return 1;
  const double k0 = 1.0 + std::log2(kErrPerStep[p] / tol);
  return std::max(1, (int)std::ceil(k0 - 1e-9));
}

// Whether step k (1-based) with dims (dx, dy) runs reduced.
inline bool step_is_reduced(int p, int k, int dx, int dy, int d_cut, int k0) {
  return p != HOTRG_FP64 && dx >= d_cut && dy >= d_cut && k >= k0;
}

struct PrecPlan {
  int prec;           // precision of the reduced steps (HOTRG_FP64: none)
  int first_reduced;  // first step that may be reduced
  double err_bound;   // a-priori relative ln Z/N error bound vs FP64
  double seconds;     // estimated contraction time
};

inline PrecPlan plan_precision(int p, double tol, int dx, int dy, int d_cut, int n_steps) {
  PrecPlan pl{p, first_reduced_step(p, tol), 0.0, 0.0};
  for (int k = 1; k <= n_steps; ++k) {
    const int dn = (int)std::min<long long>(d_cut, (long long)dx * dx);
    const double x = dx, y = dy, n = dn;
    const double flops = 2.0 * (2 * x * x * x * y * y * y + x * x * x * x * y * y +
                                x * x * x * y * y * n + n * x * x * x * y * y * y +
                                n * n * x * x * y * y);
    const bool red = step_is_reduced(p, k, dx, dy, d_cut, pl.first_reduced);
    if (red) pl.err_bound += kErrPerStep[p] * std::ldexp(1.0, -k);
    pl.seconds += flops / (kStepRate[red ? p : HOTRG_FP64] * 1e12);
    const int ndx = dy;
    dy = dn;
    dx = ndx;
  }
  return pl;
}

// HOTRG_PREC_AUTO: the precision with the least estimated time whose bound
// meets tol (FP64 always does).
inline PrecPlan plan_auto(double tol, int dx, int dy, int d_cut, int n_steps) {
  PrecPlan best = plan_precision(HOTRG_FP64, tol, dx, dy, d_cut, n_steps);
  for (int p : {HOTRG_FP32, HOTRG_BF16X3}) {
    const PrecPlan pl = plan_precision(p, tol, dx, dy, d_cut, n_steps);
    if (pl.err_bound <= tol && pl.seconds < best.seconds) best = pl;
  }
  return best;
}

}  // namespace hotrg
