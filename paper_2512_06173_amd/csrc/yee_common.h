// Device helpers shared by the Yee sweep kernels.
#pragma once

#include "mlk_internal.h"

namespace mlk {

// Value one cell up along an axis (stride s) from linear index id at axis
// coordinate q: wraps on a periodic axis, otherwise the virtual wall plane
// q = n, where the tangential E of the metallic wall is zero.
template <typename T>
__device__ __forceinline__ T fwd(const T* a, size_t id, int q, int n, int periodic, size_t s) {
  if (q + 1 < n) return a[id + s];
  return periodic ? a[id - (size_t)(n - 1) * s] : T(0);
}

// Value one cell down: wraps on a periodic axis; below index 0 of a wall
// axis the value is never used (those E components are held at zero).
template <typename T>
__device__ __forceinline__ T bwd(const T* a, size_t id, int q, int n, int periodic, size_t s) {
  if (q > 0) return a[id - s];
  return periodic ? a[id + (size_t)(n - 1) * s] : T(0);
}

// Convolutional PML stretching of a derivative d taken along axis a:
// psi <- b psi + c d ; d <- d / kappa + psi  (inside the layers only).
template <typename T>
__device__ __forceinline__ T stretch(const FieldPtrs<T>& f, const Geom& g, T* psi, int a, int half,
                                     int i, int j, int k, T d) {
  if (psi == nullptr) return d;
  const int q = a == 0 ? i : (a == 1 ? j : k);
  if (!in_layer(g, a, q)) return d;
  const size_t pid = psi_index(g, a, i, j, k);
  const T p = f.cb[a][half][q] * psi[pid] + f.cc[a][half][q] * d;
  psi[pid] = p;
  return f.ck[a][half][q] * d + p;
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

// Source current density at cell (i,j,k) for the step read from *step,
// evaluated at t = (n + 1/2) dt; added to J[comp].
template <typename T>
__device__ __forceinline__ void source_current(const SourceSet& src, const Geom& g,
                                               const int64_t* step, int i, int j, int k, T J[3]) {
#pragma unroll
  for (int q = 0; q < kMaxSources; ++q) {
    if (q >= src.count) break;
    const Source& s = src.s[q];
    bool hit;
    double scale;
    if (s.kind == 0) {
      const int pos = s.axis == 0 ? i : (s.axis == 1 ? j : k);
      hit = pos == s.index;
      scale = g.inv_dx;
    } else {
      hit = i == s.ijk[0] && j == s.ijk[1] && k == s.ijk[2];
      scale = g.inv_dx * g.inv_dx * g.inv_dx;
    }
    if (hit) {
      const double t = ((double)(*step) + 0.5) * g.dt;
      const T v = (T)(pulse_value(s, t) * scale);
      if (s.comp == 0) J[0] += v;
      else if (s.comp == 1) J[1] += v;
      else J[2] += v;
    }
  }
}

}  // namespace mlk
