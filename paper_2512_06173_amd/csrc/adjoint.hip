// Discrete adjoint (reverse mode) of the coupled step, for gradients of the
// time-integrated flux through the flux plane, or of a weighted sum of final
// populations, with respect to eps_r in a box of cells and to each two-level
// emitter's dipole vector.
//
// The forward step n (as the library executes it) is
//   E~ = G E^n;  g = E~ . d;  (rho, mu_dot) = TLS(rho, g);      (gather, emitter step)
//   H^{n+1/2} = H^{n-1/2} - dt curl_s E^n;                       (H update, CPML psi_H)
//   E^{n+1}  = E^n + dt eps^-1 (curl_s H^{n+1/2} - J_src - S mu_dot), walls 0
//   F^{n+1/2} = dx^2 sum_plane (Ebar_u Hhat_v - Ebar_v Hhat_u)   (flux detector)
// with S = G^T / dx^3.  Its reverse, with adjoint fields Eb, Hb, psib and
// emitter adjoints sb (the state), is, for n = T-1 ... 0:
//   flux:   Eb(plane) += dt dF/dE^{n+1};  Hb(planes) += dt dF/dH^{n+1/2}
//   eps:    d/d eps of E^{n+1} is -(E^{n+1} - E^n)/eps, so g_eps -= Eb . (E^{n+1}-E^n) eps^-1
//   mu_dot: mub = -(dt / dx^3) gamma G(eps^-1 Eb)
//   E update transposed (k_adj_E), then the H update transposed (k_adj_H)
//   TLS:    the step is a rotation R(g) of the Bloch vector, so the state adjoint
//           turns back by R^T, and gb = rb' . dR/dg r (dual numbers in g)
//   gather: Eb += G^T (gb d)  (a scatter)
//   flux:   Eb(plane) += dt dF/dE^n
// Each linear update y = A x is transposed in gather form: a thread owns one
// cell and collects, from its own and its neighbours' stencils, every
// coefficient through which its value entered the forward update.  The CPML
// recursion psi' = b psi + c d, s = kappa^-1 d + psi' transposes to
//   db = (kappa^-1 + c) w + c psib,   psib <- b (w + psib)
// where w is the adjoint of the stretched derivative; neighbours read the old
// psib, so it is double-buffered.
#include "mlk_internal.h"
#include "launch.h"
#include "yee_common.h"

namespace mlk {

namespace {

template <typename T>
struct AdjPtrs {
  T* E[3];           // adjoint of E
  T* H[3];           // adjoint of H
  const T* epsinv;   // null in vacuum (eps_r = 1) for the transposed sweep
  const T* tab;      // CPML tables (b, c, 1/kappa) of the forward sweep
  const T* psi_in;   // adjoint of psi (both fields), read
  T* psi_out;        // adjoint of psi, written
};

// Adjoint of the plain derivative from w, the adjoint of the stretched one, at
// (i,j,k) for `field` (0: E, 1: H), component c, derivative axis a; `lay` says
// whether the position lies in a CPML layer of axis a (q: its coordinate there).
template <typename T>
__device__ __forceinline__ T dbar(const Geom& g, const AdjPtrs<T>& p, bool lay, int field, int c,
                                  int a, int q, int i, int j, int k, T w) {
  if (!lay) return w;
  const size_t po = psi_offset(g, field, c, a) + psi_index(g, a, i, j, k);
  const int n = g.n[a];
  const T* t = p.tab + tab_offset(g, a) + (size_t)field * n + q;
  return (t[4 * n] + t[2 * n]) * w + t[2 * n] * p.psi_in[po];
}

template <typename T>
__device__ __forceinline__ void psib_update(const Geom& g, const AdjPtrs<T>& p, bool lay,
                                            int field, int c, int a, int q, int i, int j, int k,
                                            T w) {
  if (!lay) return;
  const size_t po = psi_offset(g, field, c, a) + psi_index(g, a, i, j, k);
  const int n = g.n[a];
  const T* t = p.tab + tab_offset(g, a) + (size_t)field * n + q;
  p.psi_out[po] = t[0] * (w + p.psi_in[po]);
}

// A cell's neighbour one step along each axis (dir = +1 or -1): linear index,
// coordinate along the axis, existence (false beyond a non-periodic face) and
// CPML-layer membership.
struct Nbrs {
  size_t id[3];
  int q[3];
  bool ok[3], lay[3];
};

__device__ __forceinline__ Nbrs neighbours(const Geom& g, int i, int j, int k, size_t id, int dir) {
  const size_t st[3] = {1, (size_t)g.n[0], (size_t)g.n[0] * g.n[1]};
  const int q0[3] = {i, j, k};
  Nbrs nb;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    int q = q0[a] + dir;
    size_t nid = dir > 0 ? id + st[a] : id - st[a];
    bool ok = true;
    if (q < 0 || q >= g.n[a]) {
      ok = g.periodic[a] != 0;
      q = q < 0 ? q + g.n[a] : q - g.n[a];
      nid = dir > 0 ? id - (size_t)(g.n[a] - 1) * st[a] : id + (size_t)(g.n[a] - 1) * st[a];
    }
    nb.id[a] = ok ? nid : id;
    nb.q[a] = q;
    nb.ok[a] = ok;
    nb.lay[a] = ok && has_cpml(g, a) && in_layer(g, a, q);
  }
  return nb;
}

// curl terms of component c: derivative axis and component of the other field,
// with the sign of the term
constexpr int kAx[3][2] = {{1, 2}, {2, 0}, {0, 1}};
constexpr int kOt[3][2] = {{2, 1}, {0, 2}, {1, 0}};

}  // namespace

// Cell updates of the transposed step.  Every field load of a thread is issued
// up front, unconditionally (a missing neighbour reads the cell itself and its
// term is zeroed afterwards), so the loads are in flight together; only the
// CPML terms load inside branches.  In place (OOP = false), p holds Eb and Hb;
// out of place, Eb and Hb are read from p and written to o.

// Transposed E update.  Eb holds the adjoint of E^{n+1}; Hb gains the curl
// part.  In place, Eb leaves holding that of E^n (identity part, zero on the
// walls, stored only where a wall zeroes it); out of place the H pass applies
// the mask.
template <typename T, bool OOP>
__device__ __forceinline__ void adj_e_cell(const AdjPtrs<T>& p, const AdjPtrs<T>& o,
                                           const Geom& g, int i, int j, int k) {
  const size_t id = (size_t)i + (size_t)g.n[0] * ((size_t)j + (size_t)g.n[1] * (size_t)k);
  const T dt = (T)g.dt, idx = (T)g.inv_dx;
  const int qo[3] = {i, j, k};
  const Nbrs nb = neighbours(g, i, j, k, id, +1);
  T eo[3], hv[3], en[3][3], epn[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) eo[c] = p.E[c][id];
  const T ei = p.epsinv ? p.epsinv[id] : T(1);  // null: eps_r = 1 everywhere
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    epn[a] = p.epsinv ? p.epsinv[nb.id[a]] : T(1);
#pragma unroll
    for (int c = 0; c < 3; ++c) en[a][c] = c != a ? p.E[c][nb.id[a]] : T(0);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) hv[c] = p.H[c][id];
  // wall planes through this cell (a wall zeroes the tangential E on it)
  const bool w0 = g.wall[0] && i == 0, w1 = g.wall[1] && j == 0, w2 = g.wall[2] && k == 0;
  const bool wl[3] = {w0, w1, w2};
  T u[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const bool m = (c != 0 && w0) || (c != 1 && w1) || (c != 2 && w2);
    u[c] = m ? T(0) : eo[c];
  }
  T hb[3] = {T(0), T(0), T(0)};
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int a = kAx[c][s], h = kOt[c][s];
      const T sg = s == 0 ? T(1) : T(-1);
      const bool lay = has_cpml(g, a) && in_layer(g, a, qo[a]);
      // own stencil: d = (H_h(cell) - H_h(cell - e_a)) / dx
      const T w = sg * dt * ei * u[c];
      psib_update(g, p, lay, 0, c, a, qo[a], i, j, k, w);
      hb[h] += dbar(g, p, lay, 0, c, a, qo[a], i, j, k, w) * idx;
      // the stencil of the E cell above along a reads H_h(cell) with a minus sign;
      // that cell shares this cell's planes across the other two axes, so the
      // walls through it are those of the other axes (no term beyond a face)
      bool m = false;
#pragma unroll
      for (int b = 0; b < 3; ++b) m = m || (b != a && b != c && wl[b]);
      const T wn = (m || !nb.ok[a]) ? T(0) : sg * dt * epn[a] * en[a][c];
      const int ii = a == 0 ? nb.q[0] : i, jj = a == 1 ? nb.q[1] : j, kk = a == 2 ? nb.q[2] : k;
      hb[h] -= dbar(g, p, nb.lay[a], 0, c, a, nb.q[a], ii, jj, kk, wn) * idx;
    }
  if (!OOP && (w0 || w1 || w2)) {
#pragma unroll
    for (int c = 0; c < 3; ++c) p.E[c][id] = u[c];
  }
  const AdjPtrs<T>& d = OOP ? o : p;
#pragma unroll
  for (int c = 0; c < 3; ++c) __builtin_nontemporal_store(hv[c] + hb[c], &d.H[c][id]);
}

// Transposed H update.  Hb holds the adjoint of H^{n+1/2} (unchanged: identity
// part); Eb gains the curl part.  Out of place, Hb is read from o (the E pass
// wrote it there) and Eb from p, masked on the walls.
template <typename T, bool OOP>
__device__ __forceinline__ void adj_h_cell(const AdjPtrs<T>& p, const AdjPtrs<T>& o,
                                           const Geom& g, int i, int j, int k) {
  const size_t id = (size_t)i + (size_t)g.n[0] * ((size_t)j + (size_t)g.n[1] * (size_t)k);
  const T dt = (T)g.dt, idx = (T)g.inv_dx;
  const int qo[3] = {i, j, k};
  const Nbrs nb = neighbours(g, i, j, k, id, -1);
  const AdjPtrs<T>& hs = OOP ? o : p;
  T hv[3], hn[3][3], ev[3];
#pragma unroll
  for (int h = 0; h < 3; ++h) hv[h] = hs.H[h][id];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int h = 0; h < 3; ++h) hn[a][h] = h != a ? hs.H[h][nb.id[a]] : T(0);
#pragma unroll
  for (int c = 0; c < 3; ++c) ev[c] = p.E[c][id];
  if (OOP) {
    const bool w0 = g.wall[0] && i == 0, w1 = g.wall[1] && j == 0, w2 = g.wall[2] && k == 0;
#pragma unroll
    for (int c = 0; c < 3; ++c)
      if ((c != 0 && w0) || (c != 1 && w1) || (c != 2 && w2)) ev[c] = T(0);
  }
  T eb[3] = {T(0), T(0), T(0)};
#pragma unroll
  for (int h = 0; h < 3; ++h)
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int a = kAx[h][s], e = kOt[h][s];
      const T sg = s == 0 ? T(1) : T(-1);
      const bool lay = has_cpml(g, a) && in_layer(g, a, qo[a]);
      // own stencil: d = (E_e(cell + e_a) - E_e(cell)) / dx, H -= dt sg s(d)
      const T w = -sg * dt * hv[h];
      psib_update(g, p, lay, 1, h, a, qo[a], i, j, k, w);
      eb[e] -= dbar(g, p, lay, 1, h, a, qo[a], i, j, k, w) * idx;
      // the stencil of the H cell below along a reads E_e(cell) with a plus sign
      const T wn = nb.ok[a] ? -sg * dt * hn[a][h] : T(0);
      const int ii = a == 0 ? nb.q[0] : i, jj = a == 1 ? nb.q[1] : j, kk = a == 2 ? nb.q[2] : k;
      eb[e] += dbar(g, p, nb.lay[a], 1, h, a, nb.q[a], ii, jj, kk, wn) * idx;
    }
  const AdjPtrs<T>& d = OOP ? o : p;
#pragma unroll
  for (int c = 0; c < 3; ++c) __builtin_nontemporal_store(ev[c] + eb[c], &d.E[c][id]);
}

// Whole-grid transposed sweep in place: one thread per cell, 64 x 4 cells per
// workgroup over (x, y), one z plane per grid row.
template <typename T>
__global__ __launch_bounds__(256) void k_adj_E(AdjPtrs<T> p, Geom g) {
  const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y, k = blockIdx.z;
  if (i >= g.n[0] || j >= g.n[1]) return;
  adj_e_cell<T, false>(p, p, g, i, j, k);
}

template <typename T>
__global__ __launch_bounds__(256) void k_adj_H(AdjPtrs<T> p, Geom g) {
  const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y, k = blockIdx.z;
  if (i >= g.n[0] || j >= g.n[1]) return;
  adj_h_cell<T, false>(p, p, g, i, j, k);
}

// The cells outside the fused transposed sweep's box (compact enumeration),
// out of place: the E pass (E_PASS) writes o.H, then the H pass writes o.E.
template <typename T, bool E_PASS>
__global__ __launch_bounds__(256) void k_adj_shell(AdjPtrs<T> p, AdjPtrs<T> o, Geom g,
                                                   ShellMap m) {
  const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
  if ((long long)t >= m.total) return;
  int i, j, k;
  shell_cell(g, m, t, i, j, k);
  if (E_PASS) adj_e_cell<T, true>(p, o, g, i, j, k);
  else adj_h_cell<T, true>(p, o, g, i, j, k);
}

// Flux detector: part 0 adds dt dF/dE^{n+1} and dt dF/dH^{n+1/2}, part 1 adds
// dt dF/dE^n.  The tape of step n holds, per plane cell (np of them), eight
// FP64 planes: E_u^n, E_v^n, E_u^{n+1}, E_v^{n+1}, H_u and H_v at index-1, H_u
// and H_v at index.
template <typename T>
__global__ __launch_bounds__(256) void k_adj_flux(AdjPtrs<T> p, Geom g, int axis, int index,
                                                  const double* tape, int part) {
  const int u = (axis + 1) % 3, v = (axis + 2) % 3;
  const int nu = g.n[u], nv = g.n[v], np = nu * nv;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= np) return;
  const int iu = t % nu, iv = t / nu;
  int q[3], r[3];
  q[axis] = index;
  q[u] = iu;
  q[v] = iv;
  r[axis] = index - 1;
  r[u] = iu;
  r[v] = iv;
  const size_t id = cell_index(g, q[0], q[1], q[2]), jd = cell_index(g, r[0], r[1], r[2]);
  const double c = 0.5 * g.dt * g.dx * g.dx;
  const double Hu = 0.5 * (tape[4 * (size_t)np + t] + tape[6 * (size_t)np + t]);
  const double Hv = 0.5 * (tape[5 * (size_t)np + t] + tape[7 * (size_t)np + t]);
  p.E[u][id] += (T)(c * Hv);
  p.E[v][id] -= (T)(c * Hu);
  if (part == 0) {
    const double Eu = 0.5 * (tape[t] + tape[2 * (size_t)np + t]);
    const double Ev = 0.5 * (tape[(size_t)np + t] + tape[3 * (size_t)np + t]);
    p.H[v][id] += (T)(c * Eu);
    p.H[v][jd] += (T)(c * Eu);
    p.H[u][id] -= (T)(c * Ev);
    p.H[u][jd] -= (T)(c * Ev);
  }
}

// eps gradient over a box: g -= sum_c Eb_c (E^{n+1}_c - E^n_c) eps^-1; the tape
// holds the box values of E (3 components, box order x fastest).
template <typename T>
__global__ __launch_bounds__(256) void k_adj_eps(AdjPtrs<T> p, Geom g, Box box, const T* e_n,
                                                 const T* e_n1, double* geps) {
  const int bx = box.hi[0] - box.lo[0], by = box.hi[1] - box.lo[1], bz = box.hi[2] - box.lo[2];
  const size_t nb = (size_t)bx * by * bz;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nb) return;
  const int i = box.lo[0] + (int)(t % bx), j = box.lo[1] + (int)((t / bx) % by),
            k = box.lo[2] + (int)(t / ((size_t)bx * by));
  const size_t id = cell_index(g, i, j, k);
  double acc = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c)
    acc += (double)p.E[c][id] * ((double)e_n1[c * nb + t] - (double)e_n[c * nb + t]);
  geps[t] -= acc * (double)p.epsinv[id];
}

namespace {

// first-order dual numbers in the local field g
struct Dual {
  double v, d;
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ Dual operator*(double s, Dual a) { return {s * a.v, s * a.d}; }
__device__ __forceinline__ Dual operator/(Dual a, Dual b) {
  return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)};
}
__device__ __forceinline__ Dual dsqrt(Dual a) {
  const double r = sqrt(a.v);
  return {r, a.d / (2.0 * r)};
}
__device__ __forceinline__ void dsincos(Dual a, Dual& s, Dual& c) {
  double sv, cv;
  sincos(a.v, &sv, &cv);
  s = {sv, cv * a.d};
  c = {cv, -sv * a.d};
}

}  // namespace

// Reverse of the two-level step of every emitter.  Bloch vector r = (2 Re rho01,
// -2 Im rho01, 1 - 2 rho11); the step rotates it about k = h/|h|, h = (-g, 0,
// -w0/2), by th = 2|h| dt:  r' = c r + s k x r + (1 - c) k (k . r); mu_dot =
// w0 r'_y d.  mub: raw gather of eps^-1 Eb (times gamma), scaled here by
// -dt/dx^3.  Writes the adjoint amplitude gb d for the scatter into etb.
__global__ __launch_bounds__(256) void k_adj_tls(TlsPtrs tls, double dt, double mub_scale,
                                                 const double* tape_s, const double* tape_et,
                                                 const double* mub, double* sb, double* gd,
                                                 double* etb) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= tls.count) return;
  const int e = tls.gid[m];
  const double w0 = tls.omega0[m];
  const double d[3] = {tls.dip[3 * m], tls.dip[3 * m + 1], tls.dip[3 * m + 2]};
  const double et[3] = {tape_et[3 * e], tape_et[3 * e + 1], tape_et[3 * e + 2]};
  const double p0 = tape_s[3 * m], x0 = tape_s[3 * m + 1], y0 = tape_s[3 * m + 2];
  const double r[3] = {2.0 * x0, -2.0 * y0, 1.0 - 2.0 * p0};
  const Dual G = {et[0] * d[0] + et[1] * d[1] + et[2] * d[2], 1.0};
  const Dual hz = {-0.5 * w0, 0.0};
  const Dual hx = {-G.v, -1.0};
  const Dual om = dsqrt(hx * hx + hz * hz);
  Dual s, c;
  dsincos(2.0 * dt * om, s, c);
  const Dual kx = hx / om, kz = hz / om;
  const Dual one = {1.0, 0.0};
  const Dual omc = one - c;
  const Dual rx = {r[0], 0.0}, ry = {r[1], 0.0}, rz = {r[2], 0.0};
  const Dual kr = kx * rx + kz * rz;
  const Dual r1x = c * rx - s * (kz * ry) + omc * (kx * kr);
  const Dual r1y = c * ry + s * (kz * rx - kx * rz);
  const Dual r1z = c * rz + s * (kx * ry) + omc * (kz * kr);
  // mu_dot = a d with a = w0 r'_y
  double mb[3], abar = 0.0;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    mb[q] = mub_scale * mub[3 * e + q];
    gd[3 * m + q] += w0 * r1y.v * mb[q];
    abar += mb[q] * d[q];
  }
  // state adjoint -> Bloch adjoint: s = (p, x, y), r = (2x, -2y, 1 - 2p)
  const double rbx = 0.5 * sb[3 * m + 1];
  const double rby = -0.5 * sb[3 * m + 2] + w0 * abar;
  const double rbz = -0.5 * sb[3 * m];
  const double gb = rbx * r1x.d + rby * r1y.d + rbz * r1z.d;
  // back through the rotation: R^T = rotation by -th
  const double kxv = kx.v, kzv = kz.v, cv = c.v, sv = s.v, omcv = omc.v;
  const double krb = kxv * rbx + kzv * rbz;
  const double qx = cv * rbx + sv * (kzv * rby) + omcv * kxv * krb;
  const double qy = cv * rby - sv * (kzv * rbx - kxv * rbz);
  const double qz = cv * rbz - sv * (kxv * rby) + omcv * kzv * krb;
  sb[3 * m] = -2.0 * qz;
  sb[3 * m + 1] = 2.0 * qx;
  sb[3 * m + 2] = -2.0 * qy;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    gd[3 * m + q] += gb * et[q];
    etb[3 * e + q] = gb * d[q];
  }
}

// Tape packing after a forward step: the box values of E (3 components).
template <typename T>
__global__ __launch_bounds__(256) void k_pack_box(FieldPtrs<T> f, Geom g, Box box, T* out) {
  const int bx = box.hi[0] - box.lo[0], by = box.hi[1] - box.lo[1], bz = box.hi[2] - box.lo[2];
  const size_t nb = (size_t)bx * by * bz;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nb) return;
  const int i = box.lo[0] + (int)(t % bx), j = box.lo[1] + (int)((t / bx) % by),
            k = box.lo[2] + (int)(t / ((size_t)bx * by));
  const size_t id = cell_index(g, i, j, k);
#pragma unroll
  for (int c = 0; c < 3; ++c) out[c * nb + t] = f.E[c][id];
}

// Tape packing after a forward step: the eight flux planes (see k_adj_flux).
template <typename T>
__global__ __launch_bounds__(256) void k_pack_flux(FieldPtrs<T> f, Geom g, FluxPlane fp,
                                                   double* out) {
  const int a = fp.axis, u = (a + 1) % 3, v = (a + 2) % 3;
  const int nu = g.n[u], nv = g.n[v], np = nu * nv;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= np) return;
  const int iu = t % nu, iv = t / nu;
  int q[3], r[3];
  q[a] = fp.index;
  q[u] = iu;
  q[v] = iv;
  r[a] = fp.index - 1;
  r[u] = iu;
  r[v] = iv;
  const size_t id = cell_index(g, q[0], q[1], q[2]), jd = cell_index(g, r[0], r[1], r[2]);
  out[t] = fp.Eu0[t];
  out[(size_t)np + t] = fp.Ev0[t];
  out[2 * (size_t)np + t] = (double)f.E[u][id];
  out[3 * (size_t)np + t] = (double)f.E[v][id];
  out[4 * (size_t)np + t] = (double)f.H[u][jd];
  out[5 * (size_t)np + t] = (double)f.H[v][jd];
  out[6 * (size_t)np + t] = (double)f.H[u][id];
  out[7 * (size_t)np + t] = (double)f.H[v][id];
}

// ----------------------------------------------------------------- launchers
template <typename T>
static hipError_t launch_adj_sweep(const AdjSweep<T>& a, const Geom& g, hipStream_t st) {
  AdjPtrs<T> p{};
  for (int c = 0; c < 3; ++c) {
    p.E[c] = a.E[c];
    p.H[c] = a.H[c];
  }
  p.epsinv = a.vacuum ? nullptr : a.epsinv;  // null: eps_r = 1 everywhere
  p.tab = a.tab;
  p.psi_in = a.psi[0];
  p.psi_out = a.psi[1];
  if (a.Eo[0]) {
    // fused transposed sweep on its box, then the shell cells, out of place
    const Box box = adj_interior_box(g, sizeof(T) == 4);
    hipError_t e;
    if constexpr (sizeof(T) == 4) e = adj_fused_f32(a, g, box, st);
    else e = adj_fused_f64(a, g, box, st);
    if (e != hipSuccess) return e;
    const ShellMap m = shell_map(g, box);
    if (m.total == 0) return hipSuccess;
    if (m.total >= 0x7fffff00LL) return hipErrorInvalidValue;  // 32-bit cell index
    AdjPtrs<T> o = p;
    for (int c = 0; c < 3; ++c) {
      o.E[c] = a.Eo[c];
      o.H[c] = a.Ho[c];
    }
    const unsigned blocks = (unsigned)((m.total + 255) / 256);
    hipLaunchKernelGGL((k_adj_shell<T, true>), dim3(blocks), dim3(256), 0, st, p, o, g, m);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_adj_shell<T, false>), dim3(blocks), dim3(256), 0, st, p, o, g, m);
    return hipGetLastError();
  }
  if (g.n[2] > 65535) return hipErrorInvalidValue;  // one grid row per z plane
  const dim3 grid((g.n[0] + 63) / 64, (g.n[1] + 3) / 4, g.n[2]), block(64, 4, 1);
  hipLaunchKernelGGL(k_adj_E<T>, grid, block, 0, st, p, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_adj_H<T>, grid, block, 0, st, p, g);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_adj_flux(const AdjSweep<T>& a, const Geom& g, int axis, int index,
                                  const double* tape, int part, hipStream_t st) {
  AdjPtrs<T> p{};
  for (int c = 0; c < 3; ++c) {
    p.E[c] = a.E[c];
    p.H[c] = a.H[c];
  }
  const int np = g.n[(axis + 1) % 3] * g.n[(axis + 2) % 3];
  hipLaunchKernelGGL(k_adj_flux<T>, dim3((np + 255) / 256), dim3(256), 0, st, p, g, axis, index,
                     tape, part);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_adj_eps(const AdjSweep<T>& a, const Geom& g, const Box& box,
                                 const T* e_n, const T* e_n1, double* geps, hipStream_t st) {
  AdjPtrs<T> p{};
  for (int c = 0; c < 3; ++c) p.E[c] = a.E[c];
  p.epsinv = a.epsinv;
  const size_t nb = (size_t)(box.hi[0] - box.lo[0]) * (box.hi[1] - box.lo[1]) * (box.hi[2] - box.lo[2]);
  hipLaunchKernelGGL(k_adj_eps<T>, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, p, g,
                     box, e_n, e_n1, geps);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_pack(const FieldPtrs<T>& f, const Geom& g, const Box& box, T* box_out,
                              const FluxPlane* fp, double* flux_out, hipStream_t st) {
  if (box_out) {
    const size_t nb = (size_t)(box.hi[0] - box.lo[0]) * (box.hi[1] - box.lo[1]) * (box.hi[2] - box.lo[2]);
    hipLaunchKernelGGL(k_pack_box<T>, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, f, g,
                       box, box_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (fp && flux_out) {
    const int np = g.n[(fp->axis + 1) % 3] * g.n[(fp->axis + 2) % 3];
    hipLaunchKernelGGL(k_pack_flux<T>, dim3((np + 255) / 256), dim3(256), 0, st, f, g, *fp,
                       flux_out);
    return hipGetLastError();
  }
  return hipSuccess;
}

hipError_t adj_sweep_f64(const AdjSweep<double>& a, const Geom& g, hipStream_t st) {
  return launch_adj_sweep<double>(a, g, st);
}
hipError_t adj_sweep_f32(const AdjSweep<float>& a, const Geom& g, hipStream_t st) {
  return launch_adj_sweep<float>(a, g, st);
}
hipError_t adj_flux_f64(const AdjSweep<double>& a, const Geom& g, int axis, int index,
                        const double* tape, int part, hipStream_t st) {
  return launch_adj_flux<double>(a, g, axis, index, tape, part, st);
}
hipError_t adj_flux_f32(const AdjSweep<float>& a, const Geom& g, int axis, int index,
                        const double* tape, int part, hipStream_t st) {
  return launch_adj_flux<float>(a, g, axis, index, tape, part, st);
}
hipError_t adj_eps_f64(const AdjSweep<double>& a, const Geom& g, const Box& box, const double* e_n,
                       const double* e_n1, double* geps, hipStream_t st) {
  return launch_adj_eps<double>(a, g, box, e_n, e_n1, geps, st);
}
hipError_t adj_eps_f32(const AdjSweep<float>& a, const Geom& g, const Box& box, const float* e_n,
                       const float* e_n1, double* geps, hipStream_t st) {
  return launch_adj_eps<float>(a, g, box, e_n, e_n1, geps, st);
}
hipError_t adj_tls(const TlsPtrs& tls, double dt, double mub_scale, const double* tape_s,
                   const double* tape_et, const double* mub, double* sb, double* gd, double* etb,
                   hipStream_t st) {
  if (tls.count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_tls, dim3((tls.count + 255) / 256), dim3(256), 0, st, tls, dt,
                     mub_scale, tape_s, tape_et, mub, sb, gd, etb);
  return hipGetLastError();
}
hipError_t pack_tape_f64(const FieldPtrs<double>& f, const Geom& g, const Box& box,
                         double* box_out, const FluxPlane* fp, double* flux_out, hipStream_t st) {
  return launch_pack<double>(f, g, box, box_out, fp, flux_out, st);
}
hipError_t pack_tape_f32(const FieldPtrs<float>& f, const Geom& g, const Box& box, float* box_out,
                         const FluxPlane* fp, double* flux_out, hipStream_t st) {
  return launch_pack<float>(f, g, box, box_out, fp, flux_out, st);
}

}  // namespace mlk
