// Fused transposed sweep: the reverse of one Yee step (see adjoint.hip) in one
// pass over a box of cells clear of every CPML layer.
//
// With u = Eb masked on the metallic walls (the adjoint of E^{n+1}), the
// transposed E update followed by the transposed H update is, away from the
// layers,
//   W    = dt eps^-1 u                       (per cell and component)
//   Hb' = Hb + curl_f W / dx                 (forward differences, as H^{n+1/2})
//   Eb' = u - dt curl_b Hb' / dx             (backward differences, as E^{n+1})
// the same leapfrog shape as the forward step, so this kernel marches z-chunks
// of 64 x TY tiles like the forward fused sweep: W of plane k+1 is staged in
// LDS with a one-cell ring, Hb' of plane k is computed on the tile plus the
// low-x / low-y halo that the backward curl needs (recomputed, not read), and
// Eb' of plane k follows in the same pass.  Eb and Hb are read from one pair of
// buffers and written to the other.
//
// The stretching of a CPML layer acts, in the reverse step, at the cell whose
// forward update used the derivative: the transposed E update needs the psi
// adjoint at the +1 neighbours as well.  Along y (and z with FP64 fields) the
// box therefore keeps a one-cell margin above the low layers (the recomputed
// halo) and one below the high layers (the staged +1 neighbours); the cells
// outside it are updated by the shell passes in adjoint.hip.  With FP32 fields
// the box spans every z plane: a cell's z-terms come from its own column, so
// they are formed in registers a plane ahead (see ZL below).  Along x the box
// normally spans every
// column and the x layers are handled here: each cell turns its own x-derivative
// terms into their stretched adjoints, D = dbar(+-W) for the transposed E update
// and G = dbar(-+dt Hb') for the transposed H update (psi adjoint prefetched a
// plane ahead), and its neighbours read them from LDS.  The host takes that box
// only when no tile's low-x halo column or high-x ring column lies in an x
// layer, so those stay plain.
#include "mlk_internal.h"
#include "yee_common.h"

namespace mlk {

template <typename T>
struct AdjFused {
  const T* E[3];  // adjoint of E^{n+1}
  const T* H[3];  // adjoint of H^{n+1/2}
  T* Eo[3];       // adjoint of E^n
  T* Ho[3];       // adjoint of H^{n+1/2} after the transposed E update
  const T* epsinv;
  const T* tab;      // CPML tables of the forward sweep
  const T* psi_in;   // psi adjoint (E and H), read
  T* psi_out;        // psi adjoint, written
};

namespace {

// Loads of one staged slot (Eb and 1/eps), unconditional from a safe address.
template <typename T>
__device__ __forceinline__ bool load4(const AdjFused<T>& p, Col col, Col pl, T v[3], T& ei) {
  const bool ok = col.valid && pl.valid;
  const size_t id = ok ? col.off + pl.off : 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) v[c] = p.E[c][id];
  ei = p.epsinv ? p.epsinv[id] : T(1);  // null: eps_r = 1 everywhere
  return ok;
}

// Wall mask of cell (x, y, z): component c is zero on the wall planes (index 0
// of a metallic axis other than c) through the cell.
__device__ __forceinline__ bool wall_masked(const Geom& g, int c, int x, int y, int z) {
  return (c != 0 && g.wall[0] && x == 0) || (c != 1 && g.wall[1] && y == 0) ||
         (c != 2 && g.wall[2] && z == 0);
}

}  // namespace

template <typename T, int TY, bool ZL>
__global__ __launch_bounds__(64 * TY) void k_adj_fused(AdjFused<T> p, Geom g, Box box, int kz,
                                                       int ntx, int nty, int nblocks) {
  constexpr int EW = 66, EH = TY + 2;   // W plane in LDS: x in [-1, 64], y in [-1, TY]
  constexpr int HW = 65, HH = TY + 1;   // Hb' plane in LDS: x in [-1, 63], y in [-1, TY-1]
  constexpr int NHALO = 2 * EW + 2 * TY;
  static_assert(64 * TY >= NHALO, "one thread per ring slot of the staged plane");
  __shared__ T wL[2][3][EH * EW];
  __shared__ T hL[3][HH * HW];
  __shared__ T dL[2][HH * EW];  // D of the y and z x-terms, plane k, rows -1..TY-1
  __shared__ T gL[2][HH * HW];  // G of the y and z x-terms, rows -1..TY-1
  __shared__ T xc[2][3][64];    // x CPML b, c, 1/kappa + c of the tile's columns

  const int bid = xcd_block(blockIdx.x, nblocks);
  const int tile_x = bid % ntx, tile_y = (bid / ntx) % nty, chunk = bid / (ntx * nty);
  // x tiles start on a 128-byte boundary at or below the box; cells below
  // box.lo[0] are computed too and overwritten by the shell passes
  const int x0 = (box.lo[0] & ~31) + tile_x * 64, y0 = box.lo[1] + tile_y * TY;
  const int k0 = box.lo[2] + chunk * kz, k1 = min(k0 + kz, box.hi[2]);

  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6, tid = threadIdx.x;
  const int i = x0 + tx, j = y0 + ty;
  const bool own = i < box.hi[0] && j < box.hi[1];
  const T dt = (T)g.dt, idx = (T)g.inv_dx;
  const size_t plane_sz = (size_t)g.n[0] * g.n[1];

  const Col ocol = column(g, i, j);
  const int oslot = (ty + 1) * EW + tx + 1;
  int rslot = 0, rx = 0, ry = 0;
  Col rcol{0, false};
  if (tid < NHALO) {
    int xs, ys;
    if (tid < EW) {
      xs = tid - 1;
      ys = -1;
    } else if (tid < 2 * EW) {
      xs = tid - EW - 1;
      ys = TY;
    } else {
      const int c2 = tid - 2 * EW;
      ys = c2 >> 1;
      xs = (c2 & 1) ? 64 : -1;
    }
    rslot = (ys + 1) * EW + xs + 1;
    rx = x0 + xs;
    ry = y0 + ys;
    rcol = column(g, rx, ry);
  }
  const bool hx_on = tx == 0 && j < box.hi[1] && (x0 > 0 || g.periodic[0]);
  const int ih = x0 > 0 ? x0 - 1 : g.n[0] - 1;
  const bool hy_on = ty == 0 && i < box.hi[0] && (y0 > 0 || g.periodic[1]);
  const int jh = y0 > 0 ? y0 - 1 : g.n[1] - 1;
  const size_t own_off = own ? (size_t)i + (size_t)g.n[0] * j : 0;
  const size_t hx_off = hx_on ? (size_t)ih + (size_t)g.n[0] * j : 0;
  const size_t hy_off = hy_on ? (size_t)i + (size_t)g.n[0] * jh : 0;

  // x layers: own cells and low-y halo cells in them; psi adjoint (x compressed to
  // the layers; slots E y, E z, H y, H z) through 32-bit indices (checked on the host)
  const bool lay_i = has_cpml(g, 0) && i < g.n[0] && in_layer(g, 0, i);
  const bool xl = lay_i && i >= box.lo[0] && own;
  const bool xhl = lay_i && hy_on;
  const unsigned nl = (unsigned)(g.nlo[0] + g.nhi[0]);
  const unsigned nlny = nl * (unsigned)g.n[1];
  const size_t P = (size_t)nlny * (unsigned)g.n[2];
  const unsigned li = lay_i ? (unsigned)layer_index(g, 0, i) : 0u;
  const unsigned pb = li + nl * (unsigned)j, pby = li + nl * (unsigned)jh;
  if (ty == 0 && lay_i) {
    const T* t = p.tab + tab_offset(g, 0);
    const int n = g.n[0];
#pragma unroll
    for (int f = 0; f < 2; ++f) {
      const T c = t[2 * n + f * n + i];
      xc[f][0][tx] = t[f * n + i];
      xc[f][1][tx] = c;
      xc[f][2][tx] = t[4 * n + f * n + i] + c;
    }
  }
  lds_barrier();  // the prologue uses the coefficients
  // adjoint of a stretched derivative from w: (1/kappa + c) w + c psi_in
  auto dbar = [&](int f, T w, T ps) -> T { return xc[f][2][tx] * w + xc[f][1][tx] * ps; };

  // z layers (ZL: the chunks at the two z faces, FP32 fields): whole planes.  The
  // z-terms of a cell are its own column's, so they stay in registers: D(k+1)
  // of the transposed E update is formed one plane early (it enters Hb'(k)),
  // G(k) of the transposed H update is carried to plane k+1.  Coefficients are
  // uniform loads; the psi adjoint (z compressed to the layers; slots E x, E y,
  // H x, H y) is read a plane ahead through 32-bit indices from one base
  // (checked on the host).  Without ZL the same terms take their plain form.
  const bool zcp = ZL && has_cpml(g, 2);
  const int nzc = g.n[2];
  const T* ztab = p.tab + (zcp ? tab_offset(g, 2) : 0);
  const size_t zbase = zcp ? psi_offset(g, 0, 0, 2) : 0;
  const T* zin = p.psi_in + zbase;
  T* zout = p.psi_out + zbase;
  const unsigned Pz = zcp ? (unsigned)psi_size(g, 2) : 0u;
  const unsigned nxy = (unsigned)g.n[0] * (unsigned)g.n[1];
  const unsigned oxy = (unsigned)own_off, hxy = (unsigned)hx_off, yxy = (unsigned)hy_off;
  auto zlay = [&](int kk) -> bool { return zcp && kk >= 0 && kk < nzc && in_layer(g, 2, kk); };
  auto zix = [&](unsigned xy, int kk) -> unsigned {
    return xy + nxy * (unsigned)layer_index(g, 2, kk);
  };
  // coefficients of plane kk: b, c and 1/kappa + c, of E (f = 0) or H (f = 1)
  struct ZC {
    T b, c, kc;
  };
  auto zcoef = [&](int f, int kk) -> ZC {
    const T c = ztab[(2 + f) * nzc + kk];
    return ZC{ztab[f * nzc + kk], c, ztab[(4 + f) * nzc + kk] + c};
  };

  auto W_at = [&](int q, int c, int xs, int ys) -> T { return wL[q][c][(ys + 1) * EW + xs + 1]; };
  // D of the x-term of the E component y (c = 0: -W_y) or z (c = 1: +W_z) at slot
  // (xs, ys) of plane q; the ring columns lie outside the x layers (host check)
  auto D_at = [&](int q, int c, int xs, int ys) -> T {
    if (xs == 64 || xs == -1) return c == 0 ? -W_at(q, 1, xs, ys) : W_at(q, 2, xs, ys);
    return dL[c][(ys + 1) * EW + xs + 1];
  };
  // W = dt eps^-1 u of a staged slot (zero outside the closure); the own slot's
  // u is returned in u
  auto put = [&](int q, int z, const T o[3], T oe, bool ov, T u[3], T w[3], const T r[3], T re,
                 bool rv) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      u[c] = (ov && !wall_masked(g, c, i, j, z)) ? o[c] : T(0);
      w[c] = dt * oe * u[c];
      wL[q][c][oslot] = w[c];
    }
    if (tid < NHALO) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
        wL[q][c][rslot] = (rv && !wall_masked(g, c, rx, ry, z)) ? dt * re * r[c] : T(0);
    }
  };

  T wk[3], wk1[3], uk[3], uk1[3], hpx = T(0), hpy = T(0);
  // z-terms carried between planes: D of plane k (own, low-x halo, low-y halo) and
  // G of plane k-1 (own); without a z layer D = -W_x / +W_y and G = dt Hb'_x /
  // -dt Hb'_y
  T dzx = T(0), dzy = T(0), dzxh = T(0), dzyh = T(0), gzx = T(0), gzy = T(0);
  T nEo[3], nEr[3] = {T(0), T(0), T(0)}, nEoe = T(0), nEre = T(0);
  bool nEov = false, nErv = false;

  // prologue: Hb' of plane k0-1 on the own column (x and y components)
  {
    const int km = k0 - 1;
    const int pm = (km + 2) & 1, p0 = k0 & 1;
    T em[3], emr[3], ek[3], ekr[3], eme, emre, eke, ekre, um[3], wm[3];
    const Col plm = plane(g, km), pl0 = plane(g, k0);
    const bool emv = load4(p, ocol, plm, em, eme), ekv = load4(p, ocol, pl0, ek, eke);
    const bool emrv = load4(p, rcol, plm, emr, emre), ekrv = load4(p, rcol, pl0, ekr, ekre);
    const int kmw = km < 0 ? km + g.n[2] : km;
    put(pm, kmw, em, eme, emv, um, wm, emr, emre, emrv);
    put(p0, k0, ek, eke, ekv, uk, wk, ekr, ekre, ekrv);
    // D of plane km (z component) for the own cell, read-only psi
    dL[1][oslot] = (xl && plm.valid)
                       ? dbar(0, wm[2], p.psi_in[P + pb + nlny * (unsigned)kmw]) : wm[2];
    lds_barrier();
    if constexpr (!ZL) {
      if (own && plm.valid) {
        const size_t id = own_off + plm.off;
        const T dWz_dy = W_at(pm, 2, tx, ty + 1) - wm[2];
        const T dWy_dz = wk[1] - wm[1];
        const T dWx_dz = wk[0] - wm[0];
        hpx = p.H[0][id] + idx * (dWz_dy - dWy_dz);
        hpy = p.H[1][id] + idx * (dWx_dz + (dL[1][oslot] - D_at(pm, 1, tx + 1, ty)));
      }
    } else {
    // z-terms D of planes km (read-only psi) and k0 (psi adjoint updated: this
    // chunk owns plane k0); the halo cells' D of plane k0 (read-only)
    T dmx = -wm[0], dmy = wm[1];
    dzx = -wk[0];
    dzy = wk[1];
    dzxh = -W_at(p0, 0, -1, ty);
    dzyh = W_at(p0, 1, tx, -1);
    if (zlay(km) && own) {
      const ZC z = zcoef(0, km);
      const unsigned q = zix(oxy, km);
      dmx = z.kc * dmx + z.c * zin[q];
      dmy = z.kc * dmy + z.c * zin[Pz + q];
    }
    if (zlay(k0)) {
      const ZC z = zcoef(0, k0);
      if (own) {
        const unsigned q = zix(oxy, k0);
        const T px = zin[q], py = zin[Pz + q];
        zout[q] = z.b * (dzx + px);
        zout[Pz + q] = z.b * (dzy + py);
        dzx = z.kc * dzx + z.c * px;
        dzy = z.kc * dzy + z.c * py;
      }
      if (tx == 0 && hx_on) dzxh = z.kc * dzxh + z.c * zin[zix(hxy, k0)];
      if (ty == 0 && hy_on) dzyh = z.kc * dzyh + z.c * zin[Pz + zix(yxy, k0)];
    }
    if (own && plm.valid) {
      const size_t id = own_off + plm.off;
      const T dWz_dy = W_at(pm, 2, tx, ty + 1) - wm[2];
      hpx = p.H[0][id] + idx * (dWz_dy + (dmy - dzy));
      hpy = p.H[1][id] + idx * ((dmx - dzx) + (dL[1][oslot] - D_at(pm, 1, tx + 1, ty)));
    }
    // G of plane km (read-only psi)
    gzx = dt * hpx;
    gzy = -dt * hpy;
    if (zlay(km) && own) {
      const ZC z = zcoef(1, km);
      const unsigned q = zix(oxy, km);
      gzx = z.kc * gzx + z.c * zin[2 * Pz + q];
      gzy = z.kc * gzy + z.c * zin[3 * Pz + q];
    }
    }
    const Col pl1 = plane(g, k0 + 1);
    nEov = load4(p, ocol, pl1, nEo, nEoe);
    nErv = load4(p, rcol, pl1, nEr, nEre);
    lds_barrier();
  }

  // prefetched Hb of plane k (own) and of the low-x / low-y halo cells
  T nH[3] = {T(0), T(0), T(0)}, nHx[2] = {T(0), T(0)}, nHy[2] = {T(0), T(0)};
  auto prefetch_h = [&](int k) {
    const size_t po = (size_t)min(k, g.n[2] - 1) * plane_sz;
    nH[0] = p.H[0][own_off + po];
    nH[1] = p.H[1][own_off + po];
    nH[2] = p.H[2][own_off + po];
    nHx[0] = p.H[1][hx_off + po];
    nHx[1] = p.H[2][hx_off + po];
    nHy[0] = p.H[0][hy_off + po];
    nHy[1] = p.H[2][hy_off + po];
  };
  prefetch_h(k0);
  // psi adjoint of plane k for the x-layer cells, read one iteration ahead:
  // own E y, E z, H y, H z, and E y of the low-y halo cell
  T nP[4] = {T(0), T(0), T(0), T(0)}, nPy = T(0);
  auto prefetch_psi = [&](int k) {
    if (k >= k1) return;
    if (xl) {
      const unsigned pk = pb + nlny * (unsigned)k;
#pragma unroll
      for (int q = 0; q < 4; ++q) nP[q] = p.psi_in[(size_t)q * P + pk];
    }
    if (xhl) nPy = p.psi_in[pby + nlny * (unsigned)k];
  };
  prefetch_psi(k0);
  T nZe[2] = {T(0), T(0)}, nZh[2] = {T(0), T(0)}, nZxh = T(0), nZyh = T(0);
  auto prefetch_z = [&](int k) {
    if (!ZL || k >= k1) return;
    if (zlay(k + 1)) {
      const unsigned q = zix(oxy, k + 1);
      if (own) {
        nZe[0] = zin[q];
        nZe[1] = zin[Pz + q];
      }
      if (tx == 0 && hx_on) nZxh = zin[zix(hxy, k + 1)];
      if (ty == 0 && hy_on) nZyh = zin[Pz + zix(yxy, k + 1)];
    }
    if (zlay(k) && own) {
      const unsigned q = zix(oxy, k);
      nZh[0] = zin[2 * Pz + q];
      nZh[1] = zin[3 * Pz + q];
    }
  };
  prefetch_z(k0);

  for (int k = k0; k < k1; ++k) {
    const int p0 = k & 1, p1 = (k + 1) & 1;
    const int kn = k + 1 < g.n[2] ? k + 1 : k + 1 - g.n[2];
    put(p1, kn, nEo, nEoe, nEov, uk1, wk1, nEr, nEre, nErv);
    // D of plane k: own cell (psi adjoint updated: psi <- b (w + psi)) and low-y halo
    {
      const T wy = -wk[1], wz = wk[2];
      T dy = wy, dz = wz;
      if (xl) {
        const unsigned pk = pb + nlny * (unsigned)k;
        dy = dbar(0, wy, nP[0]);
        dz = dbar(0, wz, nP[1]);
        p.psi_out[pk] = xc[0][0][tx] * (wy + nP[0]);
        p.psi_out[P + pk] = xc[0][0][tx] * (wz + nP[1]);
      }
      dL[0][oslot] = dy;
      dL[1][oslot] = dz;
      if (ty == 0) {
        const T why = -W_at(p0, 1, tx, -1);
        dL[0][tx + 1] = xhl ? dbar(0, why, nPy) : why;
      }
    }
    T hx = nH[0], hy = nH[1], hz = nH[2];
    const T hxh_y = nHx[0], hxh_z = nHx[1], hyh_x = nHy[0], hyh_z = nHy[1];
    if (k + 1 < k1) {  // the chunk's last plane needs neither W(k+2) nor Hb(k+1)
      const Col pl2 = plane(g, k + 2);
      nEov = load4(p, ocol, pl2, nEo, nEoe);
      nErv = load4(p, rcol, pl2, nEr, nEre);
      prefetch_h(k + 1);
    }
    lds_barrier();

    // z-terms D of plane k+1 (psi adjoint updated when the plane is this chunk's)
    T dzx1 = T(0), dzy1 = T(0), dzxh1 = T(0), dzyh1 = T(0);
    if constexpr (ZL) {
      dzx1 = -wk1[0];
      dzy1 = wk1[1];
      dzxh1 = -W_at(p1, 0, -1, ty);
      dzyh1 = W_at(p1, 1, tx, -1);
    }
    if (zlay(k + 1)) {
      const ZC z = zcoef(0, k + 1);
      if (own && k + 1 < k1) {
        const unsigned q = zix(oxy, k + 1);
        zout[q] = z.b * (dzx1 + nZe[0]);
        zout[Pz + q] = z.b * (dzy1 + nZe[1]);
      }
      dzx1 = z.kc * dzx1 + z.c * nZe[0];
      dzy1 = z.kc * dzy1 + z.c * nZe[1];
      dzxh1 = z.kc * dzxh1 + z.c * nZxh;
      dzyh1 = z.kc * dzyh1 + z.c * nZyh;
    }

    const size_t id = own_off + (size_t)k * plane_sz;
    // Hb' of plane k on the own cell: Hb + curl_f W / dx
    if (own) {
      const T dWz_dy = W_at(p0, 2, tx, ty + 1) - wk[2];
      const T dWx_dy = W_at(p0, 0, tx, ty + 1) - wk[0];
      // z-terms: D(k) - D(k+1), D = -W_x (y component), +W_y (x component)
      // x-terms: D(cell) - D(cell + x), D = +W_z (y component), -W_y (z component)
      if constexpr (ZL) {
        hx += idx * (dWz_dy + (dzy - dzy1));
        hy += idx * ((dzx - dzx1) + (dL[1][oslot] - D_at(p0, 1, tx + 1, ty)));
      } else {
        const T dWy_dz = wk1[1] - wk[1];
        const T dWx_dz = wk1[0] - wk[0];
        hx += idx * (dWz_dy - dWy_dz);
        hy += idx * (dWx_dz + (dL[1][oslot] - D_at(p0, 1, tx + 1, ty)));
      }
      hz += idx * ((dL[0][oslot] - D_at(p0, 0, tx + 1, ty)) - dWx_dy);
      // streaming stores, as in the forward sweep
      __builtin_nontemporal_store(hx, &p.Ho[0][id]);
      __builtin_nontemporal_store(hy, &p.Ho[1][id]);
      __builtin_nontemporal_store(hz, &p.Ho[2][id]);
    }
    // G of the own cell: x-terms of the transposed H update (psi adjoint updated)
    {
      const T wy = dt * hy, wz = -dt * hz;
      T gy = wy, gz = wz;
      if (xl) {
        const unsigned pk = pb + nlny * (unsigned)k;
        gy = dbar(1, wy, nP[2]);
        gz = dbar(1, wz, nP[3]);
        p.psi_out[2 * P + pk] = xc[1][0][tx] * (wy + nP[2]);
        p.psi_out[3 * P + pk] = xc[1][0][tx] * (wz + nP[3]);
      }
      gL[0][(ty + 1) * HW + tx + 1] = gy;
      gL[1][(ty + 1) * HW + tx + 1] = gz;
    }
    // G of the own cell: z-terms (psi adjoint updated)
    T gzx1 = T(0), gzy1 = T(0);
    if constexpr (ZL) {
      gzx1 = dt * hx;
      gzy1 = -dt * hy;
    }
    if (zlay(k) && own) {
      const ZC z = zcoef(1, k);
      const unsigned q = zix(oxy, k);
      zout[2 * Pz + q] = z.b * (gzx1 + nZh[0]);
      zout[3 * Pz + q] = z.b * (gzy1 + nZh[1]);
      gzx1 = z.kc * gzx1 + z.c * nZh[0];
      gzy1 = z.kc * gzy1 + z.c * nZh[1];
    }
    hL[0][(ty + 1) * HW + tx + 1] = hx;
    hL[1][(ty + 1) * HW + tx + 1] = hy;
    hL[2][(ty + 1) * HW + tx + 1] = hz;
    // halo Hb' at x0-1 (y and z components) for the own row, by lane 0 of each wave
    if (tx == 0) {
      T hyh = T(0), hzh = T(0);
      if (hx_on) {
        const T dWx_dy = W_at(p0, 0, -1, ty + 1) - W_at(p0, 0, -1, ty);
        const T dzh = ZL ? dzxh - dzxh1 : W_at(p1, 0, -1, ty) - W_at(p0, 0, -1, ty);
        hyh = hxh_y + idx * (dzh + (D_at(p0, 1, -1, ty) - D_at(p0, 1, 0, ty)));
        hzh = hxh_z + idx * ((D_at(p0, 0, -1, ty) - D_at(p0, 0, 0, ty)) - dWx_dy);
      }
      hL[1][(ty + 1) * HW] = hyh;
      hL[2][(ty + 1) * HW] = hzh;
      gL[0][(ty + 1) * HW] = dt * hyh;   // the halo column lies outside the x layers
      gL[1][(ty + 1) * HW] = -dt * hzh;
    }
    // halo Hb' at y0-1 (x and z components) for the own column, by the first wave
    if (ty == 0) {
      T hxh = T(0), hzh = T(0);
      if (hy_on) {
        const T dWz_dy = W_at(p0, 2, tx, 0) - W_at(p0, 2, tx, -1);
        const T dWx_dy = W_at(p0, 0, tx, 0) - W_at(p0, 0, tx, -1);
        if constexpr (ZL) {
          hxh = hyh_x + idx * (dWz_dy + (dzyh - dzyh1));
        } else {
          const T dWy_dz = W_at(p1, 1, tx, -1) - W_at(p0, 1, tx, -1);
          hxh = hyh_x + idx * (dWz_dy - dWy_dz);
        }
        hzh = hyh_z + idx * ((D_at(p0, 0, tx, -1) - D_at(p0, 0, tx + 1, -1)) - dWx_dy);
      }
      hL[0][tx + 1] = hxh;
      hL[2][tx + 1] = hzh;
    }
    lds_barrier();

    // Eb' of plane k on the own cell: u - dt curl_b Hb' / dx
    if (own) {
      const T dHz_dy = hz - hL[2][ty * HW + tx + 1];
      const T dHx_dy = hx - hL[0][ty * HW + tx + 1];
      const T cf = -dt * idx;
      // z-terms: G(k-1) - G(k), G = -dt Hb'_y (x component), dt Hb'_x (y)
      // x-terms: G(cell - x) - G(cell), G = dt Hb'_y (z component), -dt Hb'_z (y)
      const int sw = (ty + 1) * HW + tx;
      T e0, e1;
      if constexpr (ZL) {
        e0 = uk[0] + (cf * dHz_dy + idx * (gzy - gzy1));
        e1 = uk[1] + (idx * (gzx - gzx1) + idx * (gL[1][sw] - gL[1][sw + 1]));
      } else {
        const T dHy_dz = hy - hpy;
        const T dHx_dz = hx - hpx;
        e0 = uk[0] + cf * (dHz_dy - dHy_dz);
        e1 = uk[1] + (cf * dHx_dz + idx * (gL[1][sw] - gL[1][sw + 1]));
      }
      const T e2 = uk[2] + (idx * (gL[0][sw] - gL[0][sw + 1]) - cf * dHx_dy);
      __builtin_nontemporal_store(e0, &p.Eo[0][id]);
      __builtin_nontemporal_store(e1, &p.Eo[1][id]);
      __builtin_nontemporal_store(e2, &p.Eo[2][id]);
    }
    hpx = hx;
    hpy = hy;
    dzx = dzx1;
    dzy = dzy1;
    dzxh = dzxh1;
    dzyh = dzyh1;
    gzx = gzx1;
    gzy = gzy1;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      wk[c] = wk1[c];
      uk[c] = uk1[c];
    }
    prefetch_psi(k + 1);
    prefetch_z(k + 1);
  }
}

// Box of the fused transposed sweep: per axis, one cell of margin above the low
// CPML layers and one below the high layers (none on an axis without layers on
// that side).
// Along x every column when the low-x halo column (x = 64t - 1, t >= 1) and the
// high-x ring column (x = 64t, t < number of tiles) of every tile lie outside the
// x layers and the x psi arrays index in 32 bits.
// Along z (zl: FP32 fields) every plane when the z psi arrays index in 32 bits.
Box adj_interior_box(const Geom& g, bool zl) {
  Box b{};
  for (int a = 0; a < 3; ++a) {
    b.lo[a] = g.nlo[a] > 0 ? g.nlo[a] + 1 : 0;
    b.hi[a] = g.nhi[a] > 0 ? g.n[a] - g.nhi[a] - 1 : g.n[a];
    if (b.hi[a] < b.lo[a]) b.hi[a] = b.lo[a];
  }
  if (zl && has_cpml(g, 2) && 4.0 * (double)psi_size(g, 2) < 4294967296.0) {
    b.lo[2] = 0;
    b.hi[2] = g.n[2];
  }
  const int n = g.n[0], ntx = (n + 63) / 64;
  if (has_cpml(g, 0) && g.nlo[0] <= 63 && 64 * (ntx - 1) < n - g.nhi[0] &&
      (double)(g.nlo[0] + g.nhi[0]) * g.n[1] * g.n[2] < 4294967296.0) {
    b.lo[0] = 0;
    b.hi[0] = n;
  }
  return b;
}

template <typename T, bool ZL>
static hipError_t launch_adj_box(const AdjFused<T>& p, const Geom& g, const Box& box, int kz,
                                 hipStream_t st) {
  constexpr int TY = 4;
  const int ex = box.hi[0] - box.lo[0], ey = box.hi[1] - box.lo[1], ez = box.hi[2] - box.lo[2];
  if (ex <= 0 || ey <= 0 || ez <= 0) return hipSuccess;
  const int ntx = (box.hi[0] - (box.lo[0] & ~31) + 63) / 64, nty = (ey + TY - 1) / TY;
  const int nblocks = ntx * nty * ((ez + kz - 1) / kz);
  hipLaunchKernelGGL((k_adj_fused<T, TY, ZL>), dim3(nblocks), dim3(64 * TY), 0, st, p, g, box, kz,
                     ntx, nty, nblocks);
  return hipGetLastError();
}

// The box of adj_interior_box.  When it spans every z plane of a grid with z
// layers, the chunks whose planes (and the planes just outside them) keep clear
// of the layers run without the z-layer terms, and the two slabs at the z faces
// with them.
template <typename T>
static hipError_t launch_adj_fused(const AdjSweep<T>& a, const Geom& g, const Box& box,
                                   hipStream_t st) {
  const int kz = a.kz > 0 ? a.kz : 16;
  AdjFused<T> p{};
  for (int c = 0; c < 3; ++c) {
    p.E[c] = a.E[c];
    p.H[c] = a.H[c];
    p.Eo[c] = a.Eo[c];
    p.Ho[c] = a.Ho[c];
  }
  p.epsinv = a.vacuum ? nullptr : a.epsinv;
  p.tab = a.tab;
  p.psi_in = a.psi[0];
  p.psi_out = a.psi[1];
  if (!(sizeof(T) == 4 && has_cpml(g, 2) && box.lo[2] == 0 && box.hi[2] == g.n[2]))
    return launch_adj_box<T, false>(p, g, box, kz, st);
  const int zlo = g.nlo[2] > 0 ? g.nlo[2] + 1 : 0;
  const int zhi = g.nhi[2] > 0 ? g.n[2] - g.nhi[2] - 1 : g.n[2];
  if (zlo >= zhi) return launch_adj_box<T, true>(p, g, box, kz, st);
  Box mid = box, lo = box, hi = box;
  mid.lo[2] = zlo;
  mid.hi[2] = zhi;
  lo.hi[2] = zlo;
  hi.lo[2] = zhi;
  // a face slab is a few planes deep: short chunks give it enough workgroups
  // (measured at 256^3, CPML 10: 16-plane chunks 41 us per slab, 4-plane ones
  // less than half of that)
  const int kzs = kz < 4 ? kz : 4;
  hipError_t e = launch_adj_box<T, false>(p, g, mid, kz, st);
  if (e == hipSuccess) e = launch_adj_box<T, true>(p, g, lo, kzs, st);
  if (e == hipSuccess) e = launch_adj_box<T, true>(p, g, hi, kzs, st);
  return e;
}

hipError_t adj_fused_f32(const AdjSweep<float>& a, const Geom& g, const Box& box,
                         hipStream_t st) {
  return launch_adj_fused<float>(a, g, box, st);
}
hipError_t adj_fused_f64(const AdjSweep<double>& a, const Geom& g, const Box& box,
                         hipStream_t st) {
  return launch_adj_fused<double>(a, g, box, st);
}

}  // namespace mlk
