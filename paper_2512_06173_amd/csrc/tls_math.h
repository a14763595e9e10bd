// Exact two-level propagator shared by the emitter kernels.
#pragma once

#include "mlk_internal.h"

namespace mlk {

// Exact two-level step for one emitter; returns the new state and mu_dot.
__device__ __forceinline__ void tls_advance(double w0, const double d[3], const double et[3],
                                            double dt, double st[3], double md[3]) {
  const double gg = et[0] * d[0] + et[1] * d[1] + et[2] * d[2];
  const double hx = -gg, hz = -0.5 * w0;
  const double om = sqrt(hx * hx + hz * hz);
  const double p = st[0];
  const double rx = 2.0 * st[1], ry = -2.0 * st[2];
  double rx2 = rx, ry2 = ry, p2 = p;
  if (om > 0.0) {
    const double th = 2.0 * om * dt;
    const double kx = hx / om, kz = hz / om;
    const double c = cos(th), s = sin(th);
    const double sh = sin(0.5 * th);
    const double omc = 2.0 * sh * sh;  // 1 - cos(th) without cancellation
    const double rz = 1.0 - 2.0 * p;
    const double kr = kx * rx + kz * rz;
    rx2 = rx * c - kz * ry * s + kx * kr * omc;
    ry2 = ry * c + (kz * rx - kx * rz) * s;
    // rho11' = (1 - rz')/2 written so that no O(1) terms cancel
    p2 = 0.5 * (omc * (kx * kx - kx * kz * rx + 2.0 * kz * kz * p) + 2.0 * p * c - kx * ry * s);
  }
  st[0] = p2;
  st[1] = 0.5 * rx2;
  st[2] = -0.5 * ry2;
  const double f = w0 * ry2;  // -2 w0 Im(rho01)
  md[0] = f * d[0];
  md[1] = f * d[1];
  md[2] = f * d[2];
}

}  // namespace mlk
