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
#pragma clang fp contract(off)  // see the cell updates
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

// Column (x, y) of the grid seen through the closure rules: periodic axes
// wrap, beyond a metallic wall the value is zero (valid = false).
struct Col {
  size_t off;  // x + nx*y of the (wrapped) column
  bool valid;
};

__device__ __forceinline__ int wrap_mod(int q, int n) {
  const int r = q % n;
  return r < 0 ? r + n : r;
}

__device__ __forceinline__ Col column(const Geom& g, int x, int y) {
  bool ok = true;
  if (x < 0 || x >= g.n[0]) {
    ok = ok && g.periodic[0];
    x = wrap_mod(x, g.n[0]);
  }
  if (y < 0 || y >= g.n[1]) {
    ok = ok && g.periodic[1];
    y = wrap_mod(y, g.n[1]);
  }
  Col c;
  c.valid = ok;
  c.off = ok ? (size_t)x + (size_t)g.n[0] * (size_t)y : 0;
  return c;
}

// Offset of plane z with the closure rule along z (valid = false: zero plane).
__device__ __forceinline__ Col plane(const Geom& g, int z) {
  Col c;
  c.valid = true;
  if (z < 0 || z >= g.n[2]) {
    c.valid = g.periodic[2] != 0;
    z = wrap_mod(z, g.n[2]);
  }
  c.off = c.valid ? (size_t)z * (size_t)g.n[0] * (size_t)g.n[1] : 0;
  return c;
}

// Loads of one staged slot are issued without any branch or select on the
// loaded value (an invalid slot reads index 0, a safe address, and is zeroed
// when it is written to LDS), so prefetched loads stay in flight until used.
template <typename T>
__device__ __forceinline__ bool load3(const FieldPtrs<T>& f, Col col, Col pl, T v[3]) {
  const bool ok = col.valid && pl.valid;
  const size_t id = ok ? col.off + pl.off : 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) v[c] = f.E[c][id];
  return ok;
}

// Cell (i, j, k) of entry t of the compact CPML-shell enumeration (see ShellMap).
__device__ __forceinline__ void shell_cell(const Geom& g, const ShellMap& m, unsigned t, int& i,
                                           int& j, int& k) {
  const unsigned nx = (unsigned)g.n[0];
  if ((long long)t < m.nslab) {
    const unsigned plane = nx * (unsigned)g.n[1];
    const unsigned p = div_by(t, plane, m.inv_plane);
    const unsigned r = t - p * plane;
    k = (int)p < m.nzlo ? (int)p : m.in.hi[2] + ((int)p - m.nzlo);
    j = (int)div_by(r, nx, m.inv_nx);
    i = (int)(r - (unsigned)j * nx);
    return;
  }
  const unsigned u = t - (unsigned)m.nslab;
  const unsigned p = div_by(u, (unsigned)m.per_plane, m.inv_per_plane);
  unsigned r = u - p * (unsigned)m.per_plane;
  k = m.in.lo[2] + (int)p;
  if ((int)r < m.full_cells) {
    const int row = (int)div_by(r, nx, m.inv_nx);
    i = (int)(r - (unsigned)row * nx);
    j = row < m.ylo_rows ? row : m.in.hi[1] + (row - m.ylo_rows);
    return;
  }
  r -= (unsigned)m.full_cells;
  const int row = (int)div_by(r, (unsigned)m.strip, m.inv_strip);
  const int c = (int)r - row * m.strip;
  j = m.in.lo[1] + row;
  i = c < m.in.lo[0] ? c : m.in.hi[0] + (c - m.in.lo[0]);
}

}  // namespace mlk
