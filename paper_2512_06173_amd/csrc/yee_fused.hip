// Fused Yee sweep: H^{n+1/2} and E^{n+1} in one pass over the interior of the grid.
//
//   H^{n+1/2} = H^{n-1/2} - dt curl E^n
//   E^{n+1}   = E^n + (dt/eps_r) curl H^{n+1/2}
// (eq. Maxwell with D = eps_r E and B = H) with metallic or periodic closure.
// This kernel covers a box of cells whose y and z positions keep their own
// update and recomputed halo outside the y and z CPML layers (those layers
// plus a one-cell margin are updated by the plain passes, whole rows of the
// grid).  Along x the box normally spans every column and cells in the x
// layers stretch their x derivatives here: they are a few lanes at the two
// ends of each row, which the plain passes would otherwise handle as short,
// badly coalesced strips.  The host chooses that box only when no tile's
// low-x halo column lies in an x layer, so halo recomputations never need
// psi.  Source and molecular currents are added by their own passes.
//
// A workgroup owns a tile of 64 x TY columns and marches over a chunk of z
// planes.  For plane k it stages E^n(k+1) (with a one-cell halo ring) in LDS,
// computes H^{n+1/2}(k) on the tile plus the low-x / low-y halo that the curl
// of H needs (the halo H is recomputed here rather than read from a
// neighbour), keeps it in LDS, then updates E(k).  H(k-1) and E(k+1) of the
// thread's own column stay in registers, so E and H cross HBM once per step:
// 48 bytes per cell read or written plus 4 for 1/eps_r in FP32.
//
// The sweep reads the old fields and writes new ones (two buffers swapped
// every step), so halo reads of one tile never see values another tile has
// already advanced.  Block indices are remapped so that the tiles one XCD
// runs are spatial neighbours and share its L2.
#include "mlk_internal.h"
#include "yee_common.h"

namespace mlk {

template <typename T, int TY>
__device__ __forceinline__ void fused_body(const FieldPtrs<T>& a, const FieldPtrs<T>& b,
                                           const Geom& g, const Box& box, int kz, int ntx,
                                           int nty, int nblocks, int bid_in) {
  constexpr int EW = 66, EH = TY + 2;   // E plane in LDS: x in [-1, 64], y in [-1, TY]
  constexpr int HW = 65, HH = TY + 1;   // H plane in LDS: x in [-1, 63], y in [-1, TY-1]
  constexpr int NHALO = 2 * EW + 2 * TY;  // ring of the E plane
  static_assert(64 * TY >= NHALO, "one thread per ring slot of the staged E plane");
  __shared__ T eL[2][3][EH * EW];
  __shared__ T hL[3][HH * HW];
  __shared__ T xc[2][3][64];  // x CPML b, c, 1/kappa of the tile's columns (E, H positions)

  // XCD-aware tile order: consecutive blocks go to different XCDs; map the
  // blocks one XCD receives onto a contiguous range of tiles.
  int bid = bid_in;
  const int q8 = nblocks / 8;
  if (bid < 8 * q8) bid = (bid % 8) * q8 + bid / 8;
  const int tile_x = bid % ntx, tile_y = (bid / ntx) % nty, chunk = bid / (ntx * nty);
  // x tiles start on a 128-byte boundary at or below the box; the extra cells
  // below box.lo[0] are updated too (they belong to the CPML shell, whose own
  // pass overwrites them)
  const int x0 = (box.lo[0] & ~31) + tile_x * 64, y0 = box.lo[1] + tile_y * TY;
  const int k0 = box.lo[2] + chunk * kz, k1 = min(k0 + kz, box.hi[2]);

  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6, tid = threadIdx.x;
  const int i = x0 + tx, j = y0 + ty;
  const bool own = i < box.hi[0] && j < box.hi[1];
  const T dt = (T)g.dt, idx = (T)g.inv_dx;
  const size_t plane_sz = (size_t)g.n[0] * g.n[1];

  // the columns this thread stages: its own slot and (for tid < NHALO) one ring slot
  const Col ocol = column(g, i, j);
  const int oslot = (ty + 1) * EW + tx + 1;
  int rslot = 0;
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
    rcol = column(g, x0 + xs, y0 + ys);
  }
  // halo H columns: x0-1 (lane 0 of every wave), y0-1 (first wave)
  const bool hx_on = tx == 0 && j < box.hi[1] && (x0 > 0 || g.periodic[0]);
  const int ih = x0 > 0 ? x0 - 1 : g.n[0] - 1;
  const bool hy_on = ty == 0 && i < box.hi[0] && (y0 > 0 || g.periodic[1]);
  const int jh = y0 > 0 ? y0 - 1 : g.n[1] - 1;
  const size_t own_off = own ? (size_t)i + (size_t)g.n[0] * j : 0;
  // x CPML: own cells in the x layers stretch their x derivatives, psi <- b psi
  // + c d, d <- d / kappa + psi.  The coefficients of the tile's columns sit in
  // LDS; psi (one array per field component, x compressed to the layers) is
  // read at plane k through a 32-bit index (32-bit range checked on the host).
  const bool xl = has_cpml(g, 0) && i >= box.lo[0] && i < box.hi[0] && j < box.hi[1] &&
                  in_layer(g, 0, i);
  const unsigned nl = (unsigned)(g.nlo[0] + g.nhi[0]);
  const unsigned nlny = nl * (unsigned)g.n[1];
  const size_t P = (size_t)nlny * (unsigned)g.n[2];  // psi values per component array
  const unsigned li = xl ? (unsigned)layer_index(g, 0, i) : 0u;
  const unsigned pb = li + nl * (unsigned)j, pby = li + nl * (unsigned)jh;
  // psi arrays of axis x: E of y, E of z, H of y, H of z
  auto psi_at = [&](const FieldPtrs<T>& f, int slot, unsigned id) -> T& {
    return f.psi[(size_t)slot * P + id];
  };
  if (ty == 0 && xl) {
    const T* t = a.tab + tab_offset(g, 0);
    const int n = g.n[0];
#pragma unroll
    for (int fld = 0; fld < 2; ++fld) {
      xc[fld][0][tx] = t[fld * n + i];
      xc[fld][1][tx] = t[2 * n + fld * n + i];
      xc[fld][2][tx] = t[4 * n + fld * n + i];
    }
  }
  const size_t hx_off = hx_on ? (size_t)ih + (size_t)g.n[0] * j : 0;
  const size_t hy_off = hy_on ? (size_t)i + (size_t)g.n[0] * jh : 0;

  auto E_at = [&](int p, int c, int xs, int ys) -> T { return eL[p][c][(ys + 1) * EW + xs + 1]; };
  // write a staged plane to LDS, zeroing slots outside the closure; the own
  // values (zeroed likewise) are returned in o
  auto put = [&](int p, T o[3], bool ov, const T r[3], bool rv) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      o[c] = ov ? o[c] : T(0);
      eL[p][c][oslot] = o[c];
    }
    if (tid < NHALO) {
#pragma unroll
      for (int c = 0; c < 3; ++c) eL[p][c][rslot] = rv ? r[c] : T(0);
    }
  };

  T ek[3], ek1[3], hpx = T(0), hpy = T(0);
  T nEo[3], nEr[3] = {T(0), T(0), T(0)};
  bool nEov = false, nErv = false;

  // prologue: H^{n+1/2}(k0-1) of the own column (Hx, Hy), needed by E(k0)
  {
    const int km = k0 - 1;
    const int pm = (km + 2) & 1, p0 = k0 & 1;
    T em[3], emr[3], ekr[3];
    const Col plm = plane(g, km), pl0 = plane(g, k0);
    const bool emv = load3(a, ocol, plm, em), ekv = load3(a, ocol, pl0, ek);
    const bool emrv = load3(a, rcol, plm, emr), ekrv = load3(a, rcol, pl0, ekr);
    put(pm, em, emv, emr, emrv);
    put(p0, ek, ekv, ekr, ekrv);
    lds_barrier();
    if (own && plm.valid) {
      const size_t id = own_off + plm.off;
      T dEz_dy = (E_at(pm, 2, tx, ty + 1) - em[2]) * idx;
      T dEy_dz = (ek[1] - em[1]) * idx;
      T dEx_dz = (ek[0] - em[0]) * idx;
      T dEz_dx = (E_at(pm, 2, tx + 1, ty) - em[2]) * idx;
      if (xl) {
        const unsigned kmw = (unsigned)(km < 0 ? km + g.n[2] : km);
        const T q = xc[1][0][tx] * psi_at(a, 2, pb + nlny * kmw) + xc[1][1][tx] * dEz_dx;
        dEz_dx = xc[1][2][tx] * dEz_dx + q;
      }
      hpx = a.H[0][id] - dt * (dEz_dy - dEy_dz);
      hpy = a.H[1][id] - dt * (dEx_dz - dEz_dx);
    }
    // first prefetch: E(k0+1)
    const Col pl1 = plane(g, k0 + 1);
    nEov = load3(a, ocol, pl1, nEo);
    nErv = load3(a, rcol, pl1, nEr);
    lds_barrier();
  }

  // prefetched H^{n-1/2}(k), 1/eps(k) and the halo H of plane k
  T nH[3] = {T(0), T(0), T(0)}, nEps = T(0), nHx[2] = {T(0), T(0)}, nHy[2] = {T(0), T(0)};
  // unconditional loads from safe addresses (offsets are 0 for unused slots)
  auto prefetch_h = [&](int k) {
    const size_t po = (size_t)min(k, g.n[2] - 1) * plane_sz;
    nH[0] = a.H[0][own_off + po];
    nH[1] = a.H[1][own_off + po];
    nH[2] = a.H[2][own_off + po];
    nEps = a.epsinv[own_off + po];
    nHx[0] = a.H[1][hx_off + po];
    nHx[1] = a.H[2][hx_off + po];
    nHy[0] = a.H[0][hy_off + po];
    nHy[1] = a.H[2][hy_off + po];
  };
  prefetch_h(k0);
  // psi of plane k for the x-layer cells, read one iteration ahead after the
  // plane's field prefetch: own E y/z and H y/z, and H z of the low-y halo cell
  T nP[4] = {T(0), T(0), T(0), T(0)}, nPy = T(0);
  auto prefetch_psi = [&](int k) {
    if (xl && k < k1) {
      const unsigned pk = pb + nlny * (unsigned)k;
#pragma unroll
      for (int q = 0; q < 4; ++q) nP[q] = psi_at(a, q, pk);
      if (hy_on) nPy = psi_at(a, 3, pby + nlny * (unsigned)k);
    }
  };
  prefetch_psi(k0);

  for (int k = k0; k < k1; ++k) {
    const int p0 = k & 1, p1 = (k + 1) & 1;
    put(p1, nEo, nEov, nEr, nErv);
#pragma unroll
    for (int c = 0; c < 3; ++c) ek1[c] = nEo[c];
    T hx = nH[0], hy = nH[1], hz = nH[2];
    const T ce = dt * nEps;
    const T hxh_y = nHx[0], hxh_z = nHx[1], hyh_x = nHy[0], hyh_z = nHy[1];
    // prefetch the next plane while this one is computed (the last plane of the
    // chunk needs neither E(k+2) nor H(k+1))
    if (k + 1 < k1) {
      const Col pl2 = plane(g, k + 2);
      nEov = load3(a, ocol, pl2, nEo);
      nErv = load3(a, rcol, pl2, nEr);
      prefetch_h(k + 1);
    }
    lds_barrier();

    const size_t id = own_off + (size_t)k * plane_sz;
    // H^{n+1/2}(k) on the own cell
    if (own) {
      T dEz_dy = (E_at(p0, 2, tx, ty + 1) - ek[2]) * idx;
      T dEy_dz = (ek1[1] - ek[1]) * idx;
      T dEx_dz = (ek1[0] - ek[0]) * idx;
      T dEz_dx = (E_at(p0, 2, tx + 1, ty) - ek[2]) * idx;
      T dEy_dx = (E_at(p0, 1, tx + 1, ty) - ek[1]) * idx;
      T dEx_dy = (E_at(p0, 0, tx, ty + 1) - ek[0]) * idx;
      if (xl) {
        const unsigned pk = pb + nlny * (unsigned)k;
        const T bh = xc[1][0][tx], ch = xc[1][1][tx], kh = xc[1][2][tx];
        const T qy = bh * nP[2] + ch * dEz_dx;
        const T qz = bh * nP[3] + ch * dEy_dx;
        psi_at(b, 2, pk) = qy;
        psi_at(b, 3, pk) = qz;
        dEz_dx = kh * dEz_dx + qy;
        dEy_dx = kh * dEy_dx + qz;
      }
      hx -= dt * (dEz_dy - dEy_dz);
      hy -= dt * (dEx_dz - dEz_dx);
      hz -= dt * (dEy_dx - dEx_dy);
      b.H[0][id] = hx;
      b.H[1][id] = hy;
      b.H[2][id] = hz;
    }
    hL[0][(ty + 1) * HW + tx + 1] = hx;
    hL[1][(ty + 1) * HW + tx + 1] = hy;
    hL[2][(ty + 1) * HW + tx + 1] = hz;
    // halo H at x0-1 (Hy, Hz) for the own row, by lane 0 of each wave
    if (tx == 0) {
      T hyh = T(0), hzh = T(0);
      if (hx_on) {
        T dEx_dz = (E_at(p1, 0, -1, ty) - E_at(p0, 0, -1, ty)) * idx;
        T dEz_dx = (E_at(p0, 2, 0, ty) - E_at(p0, 2, -1, ty)) * idx;
        T dEy_dx = (E_at(p0, 1, 0, ty) - E_at(p0, 1, -1, ty)) * idx;
        T dEx_dy = (E_at(p0, 0, -1, ty + 1) - E_at(p0, 0, -1, ty)) * idx;
        hyh = hxh_y - dt * (dEx_dz - dEz_dx);
        hzh = hxh_z - dt * (dEy_dx - dEx_dy);
      }
      hL[1][(ty + 1) * HW] = hyh;
      hL[2][(ty + 1) * HW] = hzh;
    }
    // halo H at y0-1 (Hx, Hz) for the own column, by the first wave
    if (ty == 0) {
      T hxh = T(0), hzh = T(0);
      if (hy_on) {
        T dEz_dy = (E_at(p0, 2, tx, 0) - E_at(p0, 2, tx, -1)) * idx;
        T dEy_dz = (E_at(p1, 1, tx, -1) - E_at(p0, 1, tx, -1)) * idx;
        T dEy_dx = (E_at(p0, 1, tx + 1, -1) - E_at(p0, 1, tx, -1)) * idx;
        T dEx_dy = (E_at(p0, 0, tx, 0) - E_at(p0, 0, tx, -1)) * idx;
        if (xl) dEy_dx = xc[1][2][tx] * dEy_dx + (xc[1][0][tx] * nPy + xc[1][1][tx] * dEy_dx);
        hxh = hyh_x - dt * (dEz_dy - dEy_dz);
        hzh = hyh_z - dt * (dEy_dx - dEx_dy);
      }
      hL[0][tx + 1] = hxh;
      hL[2][tx + 1] = hzh;
    }
    lds_barrier();

    // E^{n+1}(k) on the own cell
    if (own) {
      T dHz_dy = (hz - hL[2][ty * HW + tx + 1]) * idx;
      T dHy_dz = (hy - hpy) * idx;
      T dHx_dz = (hx - hpx) * idx;
      T dHz_dx = (hz - hL[2][(ty + 1) * HW + tx]) * idx;
      T dHy_dx = (hy - hL[1][(ty + 1) * HW + tx]) * idx;
      T dHx_dy = (hx - hL[0][ty * HW + tx + 1]) * idx;
      if (xl) {
        const unsigned pk = pb + nlny * (unsigned)k;
        const T be = xc[0][0][tx], ce0 = xc[0][1][tx], ke = xc[0][2][tx];
        const T qy = be * nP[0] + ce0 * dHz_dx;
        const T qz = be * nP[1] + ce0 * dHy_dx;
        psi_at(b, 0, pk) = qy;
        psi_at(b, 1, pk) = qz;
        dHz_dx = ke * dHz_dx + qy;
        dHy_dx = ke * dHy_dx + qz;
      }
      const T cx = dHz_dy - dHy_dz;
      const T cy = dHx_dz - dHz_dx;
      const T cz = dHy_dx - dHx_dy;
      b.E[0][id] = tangential_wall(g, 0, i, j, k) ? T(0) : ek[0] + ce * cx;
      b.E[1][id] = tangential_wall(g, 1, i, j, k) ? T(0) : ek[1] + ce * cy;
      b.E[2][id] = tangential_wall(g, 2, i, j, k) ? T(0) : ek[2] + ce * cz;
    }
    hpx = hx;
    hpy = hy;
#pragma unroll
    for (int c = 0; c < 3; ++c) ek[c] = ek1[c];
    prefetch_psi(k + 1);
  }
}

template <typename T, int TY>
__global__ __launch_bounds__(64 * TY) void k_fused(FieldPtrs<T> a, FieldPtrs<T> b, Geom g,
                                                   Box box, int kz, int ntx, int nty,
                                                   int nblocks) {
  fused_body<T, TY>(a, b, g, box, kz, ntx, nty, nblocks, blockIdx.x);
}

// One launch over the jobs of a batch of domains (see BatchJobs).
template <typename T, int TY>
__global__ __launch_bounds__(64 * TY) void k_fused_batch(const FusedJob<T>* jobs,
                                                         const int* start, int njobs) {
  const int j = find_job(start, njobs, blockIdx.x);
  const FusedJob<T>& J = jobs[j];
  const int bid = blockIdx.x - start[j];
  if (J.ty != TY || bid >= J.nblocks) return;
  fused_body<T, TY>(J.a, J.b, J.g, J.box, J.kz, J.ntx, J.nty, J.nblocks, bid);
}

template <typename T, int TY>
static hipError_t launch_fused(const FieldPtrs<T>& a, const FieldPtrs<T>& b, const Geom& g,
                               const Box& box, int kz, hipStream_t st) {
  const int ex = box.hi[0] - box.lo[0], ey = box.hi[1] - box.lo[1], ez = box.hi[2] - box.lo[2];
  if (ex <= 0 || ey <= 0 || ez <= 0) return hipSuccess;
  const int ntx = (box.hi[0] - (box.lo[0] & ~31) + 63) / 64, nty = (ey + TY - 1) / TY;
  const int nch = (ez + kz - 1) / kz;
  const int nblocks = ntx * nty * nch;
  hipLaunchKernelGGL((k_fused<T, TY>), dim3(nblocks), dim3(64 * TY), 0, st, a, b, g, box, kz, ntx,
                     nty, nblocks);
  return hipGetLastError();
}

// Tile grid of the fused kernel over a box: x tiles of 64 from the 128-byte
// boundary at or below box.lo, y tiles of TY, z chunks of kz planes.
template <typename T>
void fused_job_shape(FusedJob<T>& J) {
  const Box& box = J.box;
  const int ex = box.hi[0] - box.lo[0], ey = box.hi[1] - box.lo[1], ez = box.hi[2] - box.lo[2];
  if (ex <= 0 || ey <= 0 || ez <= 0) {
    J.ntx = J.nty = J.nblocks = 0;
    return;
  }
  J.ntx = (box.hi[0] - (box.lo[0] & ~31) + 63) / 64;
  J.nty = (ey + J.ty - 1) / J.ty;
  J.nblocks = J.ntx * J.nty * ((ez + J.kz - 1) / J.kz);
}
template void fused_job_shape<float>(FusedJob<float>&);
template void fused_job_shape<double>(FusedJob<double>&);

template <typename T>
static hipError_t launch_fused_any(const FieldPtrs<T>& a, const FieldPtrs<T>& b, const Geom& g,
                                   const Box& box, int kz, int ty, hipStream_t st) {
  if (ty == 16) return launch_fused<T, 16>(a, b, g, box, kz, st);
  if (ty == 8) return launch_fused<T, 8>(a, b, g, box, kz, st);
  return launch_fused<T, 4>(a, b, g, box, kz, st);
}

template <typename T>
static hipError_t launch_fused_batch(const FusedJob<T>* jobs, const int* start, int njobs,
                                     int nblocks, int ty, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  if (ty == 16)
    hipLaunchKernelGGL((k_fused_batch<T, 16>), dim3(nblocks), dim3(1024), 0, st, jobs, start, njobs);
  else if (ty == 8)
    hipLaunchKernelGGL((k_fused_batch<T, 8>), dim3(nblocks), dim3(512), 0, st, jobs, start, njobs);
  else
    hipLaunchKernelGGL((k_fused_batch<T, 4>), dim3(nblocks), dim3(256), 0, st, jobs, start, njobs);
  return hipGetLastError();
}

hipError_t sweep_fused_f64(const FieldPtrs<double>& a, const FieldPtrs<double>& b, const Geom& g,
                           const Box& box, int kz, int ty, hipStream_t st) {
  return launch_fused_any<double>(a, b, g, box, kz, ty, st);
}
hipError_t sweep_fused_f32(const FieldPtrs<float>& a, const FieldPtrs<float>& b, const Geom& g,
                           const Box& box, int kz, int ty, hipStream_t st) {
  return launch_fused_any<float>(a, b, g, box, kz, ty, st);
}
hipError_t sweep_fused_batch_f64(const FusedJob<double>* jobs, const int* start, int njobs,
                                 int nblocks, int ty, hipStream_t st) {
  return launch_fused_batch<double>(jobs, start, njobs, nblocks, ty, st);
}
hipError_t sweep_fused_batch_f32(const FusedJob<float>* jobs, const int* start, int njobs,
                                 int nblocks, int ty, hipStream_t st) {
  return launch_fused_batch<float>(jobs, start, njobs, nblocks, ty, st);
}

}  // namespace mlk
