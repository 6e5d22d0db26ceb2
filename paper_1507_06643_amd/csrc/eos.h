// Internal equation of state eps(theta) and its inversion (eq.
// DPDE_internalEOS: eps = int_0^T C_v).  Linear EOS: eps = cv theta.  Einstein
// EOS: eps = n w/(exp(w/theta) - 1) + c0 theta, whose heat capacity
// n (w/theta)^2 e^{w/theta}/(e^{w/theta}-1)^2 + c0 increases with theta, so
// eps(theta) is increasing and convex and Newton started right of the root
// converges monotonically.
#pragma once

#include "common.h"

namespace dpde {

enum : int { THETA_NEWTON = 0, THETA_MLP = 1, THETA_MLP_NEWTON = 2 };

// Einstein part through t = exp(-w/theta): n w t/(1-t) with 1-t = -expm1(-x).
__device__ __forceinline__ double eos_energy_dev(const Phys& P, double th) {
  if (P.eos == 0) return P.cv * th;
  const double x = P.eos_omega / th;
  const double t = exp(-x);
  const double omt = -expm1(-x);
  return P.eos_n * P.eos_omega * t / omt + P.eos_c0 * th;
}

// Newton iteration on f(theta) = eps(theta) - eps from theta0; stops once the
// correction is within 4 ulp of theta or after 60 iterations.
__device__ __forceinline__ double theta_newton_dev(const Phys& P, double eps, double th, int& it) {
  it = 0;
  for (; it < 60;) {
    const double x = P.eos_omega / th;
    const double t = exp(-x);
    const double omt = -expm1(-x);
    const double f = P.eos_n * P.eos_omega * t / omt + P.eos_c0 * th - eps;
    const double c = P.eos_n * x * x * t / (omt * omt) + P.eos_c0;
    const double dth = f / c;
    double next = th - dth;
    if (!(next > 0.0)) next = 0.5 * th;
    th = next;
    ++it;
    if (fabs(dth) <= 4.0 * 2.220446049250313e-16 * th) break;
  }
  return th;
}

// High-temperature asymptote: x/(e^x - 1) >= 1 - x/2 gives
// eps(theta) >= (n + c0) theta - n w / 2, so this start is right of the root.
__device__ __forceinline__ double theta_start_dev(const Phys& P, double eps) {
  return (eps + 0.5 * P.eos_n * P.eos_omega) / (P.eos_n + P.eos_c0);
}

}  // namespace dpde
