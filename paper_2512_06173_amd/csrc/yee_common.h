// Device helpers shared by the Yee sweep kernels.
#pragma once

#include "mlk_internal.h"

namespace mlk {

// Value one cell up along an axis (stride s) from linear index id at axis
// coordinate q: wraps on a periodic axis, otherwise the virtual wall plane
// q = n, where the tangential E of the metallic wall is zero.  The load is
// unconditional (beyond a wall it reads the cell itself and discards it), so a
// thread's neighbour loads are all in flight together.
template <typename T>
__device__ __forceinline__ T fwd(const T* a, size_t id, int q, int n, int periodic, size_t s) {
  const bool in = q + 1 < n;
  const size_t nid = in ? id + s : (periodic ? id - (size_t)(n - 1) * s : id);
  const T v = a[nid];
  return (in || periodic) ? v : T(0);
}

// Value one cell down: wraps on a periodic axis; below index 0 of a wall axis
// the value is never used (those E components are held at zero).
template <typename T>
__device__ __forceinline__ T bwd(const T* a, size_t id, int q, int n, int periodic, size_t s) {
  const bool in = q > 0;
  const size_t nid = in ? id - s : (periodic ? id + (size_t)(n - 1) * s : id);
  const T v = a[nid];
  return (in || periodic) ? v : T(0);
}

// Convolutional PML stretching of a derivative d taken along axis a, at the
// positions of `field` (0: E, integer positions along a; 1: H, half-integer)
// for component c:  psi <- b psi + c d ;  d <- d / kappa + psi  (inside the
// layers only).  psi is read from `in` and, if `out` is set, the new value is
// stored there (the fused sweep reads one buffer and writes the other; halo
// recomputations store nothing).
template <typename T>
__device__ __forceinline__ T stretch(const Geom& g, const T* tab, const T* in, T* out, int field,
                                     int c, int a, int i, int j, int k, T d) {
  if (!has_cpml(g, a)) return d;
  const int q = a == 0 ? i : (a == 1 ? j : k);
  if (!in_layer(g, a, q)) return d;
  const size_t po = psi_offset(g, field, c, a) + psi_index(g, a, i, j, k);
  const int n = g.n[a];
  const T* t = tab + tab_offset(g, a) + (size_t)field * n + q;
  const T p = t[0] * in[po] + t[2 * n] * d;
  if (out) out[po] = p;
  return t[4 * n] * d + p;
}

// True when E component c at (i,j,k) lies on a metallic wall plane (index 0
// of a non-periodic axis other than c), where the tangential field is zero.
__device__ __forceinline__ bool tangential_wall(const Geom& g, int c, int i, int j, int k) {
  return (c != 0 && g.wall[0] && i == 0) || (c != 1 && g.wall[1] && j == 0) ||
         (c != 2 && g.wall[2] && k == 0);
}

// Gaussian-pulse time profile of a soft source at time t.
__device__ __forceinline__ double pulse_value(const Source& s, double t) {
  const double u = t - s.t0;
  return s.amp * cos(s.omega * u) * exp(-u * u / (2.0 * s.tau * s.tau));
}

}  // namespace mlk
