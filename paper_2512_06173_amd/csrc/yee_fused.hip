// Fused Yee sweep: H^{n+1/2} and E^{n+1} in one pass over the interior of the grid.
//
//   H^{n+1/2} = H^{n-1/2} - dt curl E^n
//   E^{n+1}   = E^n + (dt/eps_r) curl H^{n+1/2}
// (eq. Maxwell with D = eps_r E and B = H) with metallic or periodic closure.
// This kernel normally covers the whole grid, CPML layers included: a cell in
// the layers of an axis stretches its derivatives along that axis here.
//  * x layers are a few lanes at the two ends of each row, in half the tiles:
//    their coefficients sit in LDS and their psi is prefetched a plane ahead.
//    The host takes a full x extent only when no tile's low-x halo column lies
//    in an x layer (else x is limited to the cells clear of the layers plus a
//    margin, and the plain passes update the rest).
//  * y layers are whole rows (a wavefront each in 64-wide tiles, half of one in
//    32-wide tiles) and z layers whole planes:
//    the coefficients of the tile's rows sit in LDS, those of a plane are
//    uniform loads, and psi (own cell and the halo cells of the curl) is
//    prefetched a plane ahead in branches uniform across a wavefront or the
//    workgroup.  The recomputed halo H (low-y row, low-x column, the plane
//    below the chunk) reads psi without storing it.
// A psi value used in the iteration that loads it would make the wavefront
// wait for every load issued before it, the next plane's prefetch included
// (vector memory counters retire in order).
// Source and molecular currents are added by their own passes.
//
// A workgroup owns a tile of TX x TY columns (TX = 64 or 32) and marches over a chunk of z
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

// Element access by a 32-bit index: each field array, and the psi buffer, holds less
// than 4 GiB (checked on the host), so an element's byte offset fits 32 bits and a
// load takes the array's base from scalar registers plus one 32-bit offset register,
// which the arrays read at the same cell share.
template <typename T>
__device__ __forceinline__ T ld32(const T* base, unsigned i) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + i * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void st32(T* base, unsigned i, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + i * (unsigned)sizeof(T)) = v;
}
template <typename T>
__device__ __forceinline__ void st32nt(T* base, unsigned i, T v) {
  __builtin_nontemporal_store(v, reinterpret_cast<T*>(reinterpret_cast<char*>(base) +
                                                      i * (unsigned)sizeof(T)));
}
// column / plane offsets as 32-bit element indices (valid = false: a zero cell)
struct Col32 {
  unsigned off;
  bool valid;
};
__device__ __forceinline__ Col32 column32(const Geom& g, int x, int y) {
  const Col c = column(g, x, y);
  return Col32{(unsigned)c.off, c.valid};
}
__device__ __forceinline__ Col32 plane32(const Geom& g, int z) {
  const Col c = plane(g, z);
  return Col32{(unsigned)c.off, c.valid};
}
template <typename T>
__device__ __forceinline__ bool load3_32(const FieldPtrs<T>& f, Col32 col, Col32 pl, T v[3]) {
  const bool ok = col.valid && pl.valid;
  const unsigned id = ok ? col.off + pl.off : 0u;
#pragma unroll
  for (int c = 0; c < 3; ++c) v[c] = ld32(f.E[c], id);
  return ok;
}

// CPM: the CPML code compiled in: 0 none, 1 the x layers, 2 every axis (FP32; the
// FP64 kernel carries the x layers only).  Fewer layers, fewer registers: about 71
// VGPRs without any in FP32, against 118 with all of them.  TX, the tile width, is
// 64 (a row per wavefront) or 32 (two rows per wavefront: narrower tiles, more of
// them, for domains too small to give 64-wide tiles enough workgroups).

// Cost of a z-layer plane (its psi traffic and stretching) relative to an interior
// plane in the full FP32 kernel, as measured at 256^3: of first and last chunks
// shortened by 0, 4, 8 or 12 planes, 4 was fastest (a cost of 1.8); costs of 1.5 to
// 2.1 were slower.
constexpr float kZLayerCost = 1.8f;

// First plane of chunk c of nch over the box's planes [lo, hi) (c = nch gives hi), the
// chunks cut at equal shares of the summed plane cost where z-layer planes cost
// kZLayerCost times an interior one (without z layers in the box: equal depths to
// within a plane).  At the tile shapes tuned for large grids a launch runs its
// workgroups in one or two rounds, so it lasts about as long as its heaviest ones:
// equal-length chunks left those holding the layer planes, or a ragged last chunk,
// out of step with the rest.  Every workgroup evaluates the same expression for a
// boundary, so neighbouring chunks agree on it; each chunk keeps at least one plane.
__device__ __forceinline__ int chunk_start(const Geom& g, int lo, int hi, int c, int nch) {
  if (c <= 0) return lo;
  const int ez = hi - lo;
  if (c >= nch) return hi;
  // layer planes at the bottom [0, A) and the top [B, ez) of the box, counted from lo
  const int A = min(max(g.nlo[2] - lo, 0), ez);
  const int B = max(min(g.n[2] - g.nhi[2] - lo, ez), A);
  const float r = kZLayerCost;
  const float total = (float)ez + (r - 1.f) * (float)(A + ez - B);
  const float y = total * (float)c / (float)nch;
  float z;
  if (y <= r * (float)A) z = y / r;
  else if (y <= r * (float)A + (float)(B - A)) z = y - (r - 1.f) * (float)A;
  else z = (float)B + (y - r * (float)A - (float)(B - A)) / r;
  return lo + min(max((int)(z + 0.5f), c), ez - (nch - c));
}

template <typename T, int TX, int TY, int CPM = 2>
__device__ __forceinline__ void fused_body(const FieldPtrs<T>& a, const FieldPtrs<T>& b,
                                           const Geom& g, const Box& box, int kz, int ntx,
                                           int nty, int nblocks, int bid_in) {
  // A cell's H is computed by the tile that owns it and recomputed as halo by its
  // neighbours (CPML stretching included); both must round alike, so no product
  // is contracted into a fused multiply-add here, whatever the code around it.
#pragma clang fp contract(off)
  static_assert(TX == 64 || TX == 32, "tiles are 64 or 32 cells wide");
  constexpr int EW = TX + 2, EH = TY + 2;  // E plane in LDS: x in [-1, TX], y in [-1, TY]
  constexpr int HW = TX + 1, HH = TY + 1;  // H plane in LDS: x in [-1, TX-1], y in [-1, TY-1]
  constexpr int NHALO = 2 * EW + 2 * TY;  // ring of the E plane
  static_assert(TX * TY >= NHALO, "one thread per ring slot of the staged E plane");
  __shared__ T eL[2][3][EH * EW];
  __shared__ T hL[3][HH * HW];
  __shared__ T xc[2][3][TX];  // x CPML b, c, 1/kappa of the tile's columns (E, H positions)
  __shared__ T yc[2][3][TY + 1];  // y CPML b, c, 1/kappa of rows y0-1 .. y0+TY-1

  int tile_x, tile_y, chunk, k0, k1;
  if (CPM == 2 && sizeof(T) == 4 && (has_cpml(g, 1) || has_cpml(g, 2))) {
    // Heaviest first: the workgroups whose rows or planes lie in the y or z layers
    // carry the psi traffic and arithmetic and take longest.  Rows of tiles (a y tile
    // of one z chunk) are taken from the two y edges inwards, and within each the z
    // chunks likewise, so the lighter ones fill in behind the heavy ones instead of
    // the launch waiting on a few heavy workgroups at its end.  Consecutive rows go
    // to consecutive XCDs (workgroups are dealt to the 8 XCDs in turn), which spreads
    // the heavy ones evenly, and the x tiles of one row run one after another on the
    // same XCD: the cache lines that neighbouring x tiles share (the E ring's x = -1
    // and x = TX columns, the halo H column) are then read once into that XCD's L2.
    auto fold = [](int q, int n) { return (q & 1) ? n - 1 - (q >> 1) : (q >> 1); };
    // Rows are dealt to the XCDs eight at a time; when their count is not a multiple
    // of eight, the rows past the last multiple take their x tiles one after another.
    const int nch = nblocks / (ntx * nty);
    const int r8 = nty * nch / 8 * 8;
    int r;
    if (bid_in < r8 * ntx) {
      const int xcd = bid_in % 8, m = bid_in / 8;
      tile_x = m % ntx;
      r = (m / ntx) * 8 + xcd;
    } else {
      tile_x = bid_in % ntx;
      r = bid_in / ntx;
    }
    chunk = fold(r % nch, nch);
    tile_y = fold(r / nch, nty);
    k0 = chunk_start(g, box.lo[2], box.hi[2], chunk, nch);
    k1 = chunk_start(g, box.lo[2], box.hi[2], chunk + 1, nch);
  } else {
    // XCD-aware tile order: consecutive blocks go to different XCDs; map the
    // blocks one XCD receives onto a contiguous range of tiles.
    int bid = bid_in;
    const int q8 = nblocks / 8;
    if (bid < 8 * q8) bid = (bid % 8) * q8 + bid / 8;
    tile_x = bid % ntx;
    tile_y = (bid / ntx) % nty;
    chunk = bid / (ntx * nty);
    const int nch = nblocks / (ntx * nty);
    k0 = chunk_start(g, box.lo[2], box.hi[2], chunk, nch);
    k1 = chunk_start(g, box.lo[2], box.hi[2], chunk + 1, nch);
  }
  // x tiles start on a 128-byte boundary at or below the box; the extra cells
  // below box.lo[0] are updated too (they belong to the CPML shell, whose own
  // pass overwrites them)
  const int x0 = (box.lo[0] & ~31) + tile_x * TX, y0 = box.lo[1] + tile_y * TY;

  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX, tid = threadIdx.x;
  const int i = x0 + tx, j = y0 + ty;
  const bool own = i < box.hi[0] && j < box.hi[1];
  const T dt = (T)g.dt, idx = (T)g.inv_dx;
  const unsigned plane_sz = (unsigned)g.n[0] * (unsigned)g.n[1];

  // the columns this thread stages: its own slot and (for tid < NHALO) one ring slot
  const Col32 ocol = column32(g, i, j);
  const int oslot = (ty + 1) * EW + tx + 1;
  int rslot = 0;
  Col32 rcol{0u, false};
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
      xs = (c2 & 1) ? TX : -1;
    }
    rslot = (ys + 1) * EW + xs + 1;
    rcol = column32(g, x0 + xs, y0 + ys);
  }
  // halo H columns: x0-1 (first lane of every row), y0-1 (first row)
  const bool hx_on = tx == 0 && j < box.hi[1] && (x0 > 0 || g.periodic[0]);
  const int ih = x0 > 0 ? x0 - 1 : g.n[0] - 1;
  const bool hy_on = ty == 0 && i < box.hi[0] && (y0 > 0 || g.periodic[1]);
  const int jh = y0 > 0 ? y0 - 1 : g.n[1] - 1;
  const unsigned own_off = own ? (unsigned)i + (unsigned)g.n[0] * (unsigned)j : 0u;
  // x CPML: own cells in the x layers stretch their x derivatives, psi <- b psi
  // + c d, d <- d / kappa + psi.  The coefficients of the tile's columns sit in
  // LDS; psi (one array per field component, x compressed to the layers) is
  // read at plane k through a 32-bit index (32-bit range checked on the host).
  const bool xl = CPM >= 1 && has_cpml(g, 0) && i >= box.lo[0] && i < box.hi[0] &&
                  j < box.hi[1] && in_layer(g, 0, i);
  const unsigned nl = (unsigned)(g.nlo[0] + g.nhi[0]);
  const unsigned nlny = nl * (unsigned)g.n[1];
  const unsigned P = nlny * (unsigned)g.n[2];  // psi values per component array
  const unsigned li = xl ? (unsigned)layer_index(g, 0, i) : 0u;
  const unsigned pb = li + nl * (unsigned)j, pby = li + nl * (unsigned)jh;
  // y layers (own row and low-y halo row, uniform across a wavefront) and z
  // layers (per plane, uniform across the workgroup).  The psi arrays of an
  // axis are addressed from one base pointer with 32-bit indices (slot x array
  // size + cell; range checked on the host), and the coefficients of a row or
  // plane are uniform loads.
  // (FP32 only: the FP64 kernel's box keeps clear of the y and z layers)
  constexpr bool YZ = CPM == 2 && sizeof(T) == 4;
  const bool yl = YZ && has_cpml(g, 1) && j < g.n[1] && in_layer(g, 1, j);
  const bool yhl = YZ && has_cpml(g, 1) && in_layer(g, 1, jh);
  auto zlay = [&](int k) { return YZ && has_cpml(g, 2) && in_layer(g, 2, k); };
  const unsigned unx = (unsigned)g.n[0], uny = (unsigned)g.n[1];
  const unsigned nly = (unsigned)(g.nlo[1] + g.nhi[1]);
  const unsigned Py = has_cpml(g, 1) ? unx * nly * (unsigned)g.n[2] : 0u;
  const unsigned Pz = has_cpml(g, 2) ? unx * uny * (unsigned)(g.nlo[2] + g.nhi[2]) : 0u;
  const unsigned oy = has_cpml(g, 1) ? (unsigned)psi_offset(g, 0, 0, 1) : 0u;
  const unsigned oz = has_cpml(g, 2) ? (unsigned)psi_offset(g, 0, 0, 2) : 0u;
  const T* ty_tab = a.tab + (has_cpml(g, 1) ? tab_offset(g, 1) : 0);
  const T* tz_tab = a.tab + (has_cpml(g, 2) ? tab_offset(g, 2) : 0);
  const unsigned lyo = yl ? (unsigned)layer_index(g, 1, j) : 0u;
  const unsigned lyh = yhl ? (unsigned)layer_index(g, 1, jh) : 0u;
  // psi <- b psi + c d, d <- d / kappa + psi for the y derivative at row q (layer
  // index lq) and column x of plane k; slot: 0 E x, 1 E z, 2 H x, 3 H z
  auto sty = [&](int slot, int q, unsigned lq, int x, int k, T d, bool store) -> T {
    const int field = slot >> 1;
    const T* t = ty_tab + field * g.n[1] + q;
    const unsigned id = (unsigned)slot * Py + (unsigned)x + unx * (lq + nly * (unsigned)k);
    const T p = t[0] * ld32(a.psi, oy + id) + t[2 * g.n[1]] * d;
    if (store) st32(b.psi, oy + id, p);
    return t[4 * g.n[1]] * d + p;
  };
  // the same for a z derivative at cell (x, y) of plane k; slot: 0 E x, 1 E y,
  // 2 H x, 3 H y
  auto stz = [&](int slot, int x, int y, int k, T d, bool store) -> T {
    const int field = slot >> 1;
    const T* t = tz_tab + field * g.n[2] + k;
    const unsigned lz = (unsigned)layer_index(g, 2, k);
    const unsigned id = (unsigned)slot * Pz + (unsigned)x + unx * ((unsigned)y + uny * lz);
    const T p = t[0] * ld32(a.psi, oz + id) + t[2 * g.n[2]] * d;
    if (store) st32(b.psi, oz + id, p);
    return t[4 * g.n[2]] * d + p;
  };
  // psi arrays of axis x: E of y, E of z, H of y, H of z
  auto psi_ld = [&](int slot, unsigned id) -> T { return ld32(a.psi, (unsigned)slot * P + id); };
  auto psi_st = [&](int slot, unsigned id, T v) { st32(b.psi, (unsigned)slot * P + id, v); };
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
  if (YZ && has_cpml(g, 1)) {
    for (int t = tid; t < 2 * 3 * (TY + 1); t += TX * TY) {
      const int fld = t / (3 * (TY + 1)), w = (t / (TY + 1)) % 3, r = t % (TY + 1);
      const int q = y0 - 1 + r;
      yc[fld][w][r] = (q >= 0 && q < g.n[1] && in_layer(g, 1, q))
                          ? ty_tab[w * 2 * g.n[1] + fld * g.n[1] + q] : T(0);
    }
  }
  const unsigned hx_off = hx_on ? (unsigned)ih + (unsigned)g.n[0] * (unsigned)j : 0u;
  const unsigned hy_off = hy_on ? (unsigned)i + (unsigned)g.n[0] * (unsigned)jh : 0u;

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
    const Col32 plm = plane32(g, km), pl0 = plane32(g, k0);
    const bool emv = load3_32(a, ocol, plm, em), ekv = load3_32(a, ocol, pl0, ek);
    const bool emrv = load3_32(a, rcol, plm, emr), ekrv = load3_32(a, rcol, pl0, ekr);
    put(pm, em, emv, emr, emrv);
    put(p0, ek, ekv, ekr, ekrv);
    lds_barrier();
    if (own && plm.valid) {
      const unsigned id = own_off + plm.off;
      T dEz_dy = (E_at(pm, 2, tx, ty + 1) - em[2]) * idx;
      T dEy_dz = (ek[1] - em[1]) * idx;
      T dEx_dz = (ek[0] - em[0]) * idx;
      T dEz_dx = (E_at(pm, 2, tx + 1, ty) - em[2]) * idx;
      const int kmw = km < 0 ? km + g.n[2] : km;
      if (xl) {
        const T q = xc[1][0][tx] * psi_ld(2, pb + nlny * (unsigned)kmw) + xc[1][1][tx] * dEz_dx;
        dEz_dx = xc[1][2][tx] * dEz_dx + q;
      }
      if (yl) dEz_dy = sty(2, j, lyo, i, kmw, dEz_dy, false);
      if (zlay(kmw)) {
        dEy_dz = stz(2, i, j, kmw, dEy_dz, false);
        dEx_dz = stz(3, i, j, kmw, dEx_dz, false);
      }
      hpx = ld32(a.H[0], id) - dt * (dEz_dy - dEy_dz);
      hpy = ld32(a.H[1], id) - dt * (dEx_dz - dEz_dx);
    }
    // first prefetch: E(k0+1)
    const Col32 pl1 = plane32(g, k0 + 1);
    nEov = load3_32(a, ocol, pl1, nEo);
    nErv = load3_32(a, rcol, pl1, nEr);
    lds_barrier();
  }

  // prefetched H^{n-1/2}(k), 1/eps(k) and the halo H of plane k
  T nH[3] = {T(0), T(0), T(0)}, nEps = T(0), nHx[2] = {T(0), T(0)}, nHy[2] = {T(0), T(0)};
  // unconditional loads from safe addresses (offsets are 0 for unused slots)
  auto prefetch_h = [&](int k) {
    const unsigned po = (unsigned)min(k, g.n[2] - 1) * plane_sz;
    nH[0] = ld32(a.H[0], own_off + po);
    nH[1] = ld32(a.H[1], own_off + po);
    nH[2] = ld32(a.H[2], own_off + po);
    nEps = a.epsinv ? ld32(a.epsinv, own_off + po) : T(1);  // null: eps_r = 1 everywhere
    nHx[0] = ld32(a.H[1], hx_off + po);
    nHx[1] = ld32(a.H[2], hx_off + po);
    nHy[0] = ld32(a.H[0], hy_off + po);
    nHy[1] = ld32(a.H[2], hy_off + po);
  };
  prefetch_h(k0);
  // psi of plane k for the x-layer cells, read one iteration ahead after the
  // plane's field prefetch: own E y/z and H y/z, and H z of the low-y halo cell
  T nP[4] = {T(0), T(0), T(0), T(0)}, nPy = T(0);
  // y and z layers, by psi slot: own y (E x, E z, H x, H z), own z (E x, E y,
  // H x, H y); low-x halo cell: z H y, y H z; low-y halo cell: y H x, y H z, z H x
  T nYo[4] = {T(0), T(0), T(0), T(0)}, nZo[4] = {T(0), T(0), T(0), T(0)};
  T nXh[2] = {T(0), T(0)}, nYh[3] = {T(0), T(0), T(0)};
  auto iy = [&](int slot, int x, unsigned lq, int k) -> unsigned {
    return (unsigned)slot * Py + (unsigned)x + unx * (lq + nly * (unsigned)k);
  };
  auto iz = [&](int slot, int x, int y, int k) -> unsigned {
    return (unsigned)slot * Pz + (unsigned)x +
           unx * ((unsigned)y + uny * (unsigned)layer_index(g, 2, k));
  };
  auto prefetch_psi = [&](int k) {
    if (k >= k1) return;
    if (xl) {
      const unsigned pk = pb + nlny * (unsigned)k;
#pragma unroll
      for (int q = 0; q < 4; ++q) nP[q] = psi_ld(q, pk);
      if (hy_on) nPy = psi_ld(3, pby + nlny * (unsigned)k);
    }
    if (own && yl) {
#pragma unroll
      for (int q = 0; q < 4; ++q) nYo[q] = ld32(a.psi, oy + iy(q, i, lyo, k));
    }
    if (hx_on && yl) nXh[1] = ld32(a.psi, oy + iy(3, ih, lyo, k));
    if (hy_on && yhl) {
      nYh[0] = ld32(a.psi, oy + iy(2, i, lyh, k));
      nYh[1] = ld32(a.psi, oy + iy(3, i, lyh, k));
    }
    if (zlay(k)) {
      if (own) {
#pragma unroll
        for (int q = 0; q < 4; ++q) nZo[q] = ld32(a.psi, oz + iz(q, i, j, k));
      }
      if (hx_on) nXh[0] = ld32(a.psi, oz + iz(3, ih, j, k));
      if (hy_on) nYh[2] = ld32(a.psi, oz + iz(2, i, jh, k));
    }
  };
  // stretched derivative from a prefetched psi (the new psi in pn): y at LDS row
  // r, z at plane k
  auto fy = [&](int field, int r, T ps, T d, T& pn) -> T {
    pn = yc[field][0][r] * ps + yc[field][1][r] * d;
    return yc[field][2][r] * d + pn;
  };
  auto fz = [&](int field, int k, T ps, T d, T& pn) -> T {
    const T* t = tz_tab + field * g.n[2] + k;
    pn = t[0] * ps + t[2 * g.n[2]] * d;
    return t[4 * g.n[2]] * d + pn;
  };
  prefetch_psi(k0);

  for (int k = k0; k < k1; ++k) {
    const int p0 = k & 1, p1 = (k + 1) & 1;
    const bool zl = zlay(k);  // plane k in a z layer (uniform across the workgroup)
    put(p1, nEo, nEov, nEr, nErv);
#pragma unroll
    for (int c = 0; c < 3; ++c) ek1[c] = nEo[c];
    T hx = nH[0], hy = nH[1], hz = nH[2];
    const T ce = dt * nEps;
    const T hxh_y = nHx[0], hxh_z = nHx[1], hyh_x = nHy[0], hyh_z = nHy[1];
    // prefetch the next plane while this one is computed (the last plane of the
    // chunk needs neither E(k+2) nor H(k+1))
    if (k + 1 < k1) {
      const Col32 pl2 = plane32(g, k + 2);
      nEov = load3_32(a, ocol, pl2, nEo);
      nErv = load3_32(a, rcol, pl2, nEr);
      prefetch_h(k + 1);
    }
    lds_barrier();

    const unsigned id = own_off + (unsigned)k * plane_sz;
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
        psi_st(2, pk, qy);
        psi_st(3, pk, qz);
        dEz_dx = kh * dEz_dx + qy;
        dEy_dx = kh * dEy_dx + qz;
      }
      T pn;
      if (yl) {
        dEz_dy = fy(1, ty + 1, nYo[2], dEz_dy, pn);
        st32(b.psi, oy + iy(2, i, lyo, k), pn);
        dEx_dy = fy(1, ty + 1, nYo[3], dEx_dy, pn);
        st32(b.psi, oy + iy(3, i, lyo, k), pn);
      }
      if (zl) {
        dEy_dz = fz(1, k, nZo[2], dEy_dz, pn);
        st32(b.psi, oz + iz(2, i, j, k), pn);
        dEx_dz = fz(1, k, nZo[3], dEx_dz, pn);
        st32(b.psi, oz + iz(3, i, j, k), pn);
      }
      hx -= dt * (dEz_dy - dEy_dz);
      hy -= dt * (dEx_dz - dEz_dx);
      hz -= dt * (dEy_dx - dEx_dy);
      // streaming stores: the new fields are read again only in the next step,
      // long after this sweep has passed through the caches
      st32nt(b.H[0], id, hx);
      st32nt(b.H[1], id, hy);
      st32nt(b.H[2], id, hz);
    }
    hL[0][(ty + 1) * HW + tx + 1] = hx;
    hL[1][(ty + 1) * HW + tx + 1] = hy;
    hL[2][(ty + 1) * HW + tx + 1] = hz;
    // halo H at x0-1 (Hy, Hz) for the own row, by its first lane
    if (tx == 0) {
      T hyh = T(0), hzh = T(0);
      if (hx_on) {
        T dEx_dz = (E_at(p1, 0, -1, ty) - E_at(p0, 0, -1, ty)) * idx;
        T dEz_dx = (E_at(p0, 2, 0, ty) - E_at(p0, 2, -1, ty)) * idx;
        T dEy_dx = (E_at(p0, 1, 0, ty) - E_at(p0, 1, -1, ty)) * idx;
        T dEx_dy = (E_at(p0, 0, -1, ty + 1) - E_at(p0, 0, -1, ty)) * idx;
        T pn;
        if (zl) dEx_dz = fz(1, k, nXh[0], dEx_dz, pn);
        if (yl) dEx_dy = fy(1, ty + 1, nXh[1], dEx_dy, pn);
        hyh = hxh_y - dt * (dEx_dz - dEz_dx);
        hzh = hxh_z - dt * (dEy_dx - dEx_dy);
      }
      hL[1][(ty + 1) * HW] = hyh;
      hL[2][(ty + 1) * HW] = hzh;
    }
    // halo H at y0-1 (Hx, Hz) for the own column, by the first row
    if (ty == 0) {
      T hxh = T(0), hzh = T(0);
      if (hy_on) {
        T dEz_dy = (E_at(p0, 2, tx, 0) - E_at(p0, 2, tx, -1)) * idx;
        T dEy_dz = (E_at(p1, 1, tx, -1) - E_at(p0, 1, tx, -1)) * idx;
        T dEy_dx = (E_at(p0, 1, tx + 1, -1) - E_at(p0, 1, tx, -1)) * idx;
        T dEx_dy = (E_at(p0, 0, tx, 0) - E_at(p0, 0, tx, -1)) * idx;
        if (xl) dEy_dx = xc[1][2][tx] * dEy_dx + (xc[1][0][tx] * nPy + xc[1][1][tx] * dEy_dx);
        T pn;
        if (yhl) {
          dEz_dy = fy(1, 0, nYh[0], dEz_dy, pn);
          dEx_dy = fy(1, 0, nYh[1], dEx_dy, pn);
        }
        if (zl) dEy_dz = fz(1, k, nYh[2], dEy_dz, pn);
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
        psi_st(0, pk, qy);
        psi_st(1, pk, qz);
        dHz_dx = ke * dHz_dx + qy;
        dHy_dx = ke * dHy_dx + qz;
      }
      T pn;
      if (yl) {
        dHz_dy = fy(0, ty + 1, nYo[0], dHz_dy, pn);
        st32(b.psi, oy + iy(0, i, lyo, k), pn);
        dHx_dy = fy(0, ty + 1, nYo[1], dHx_dy, pn);
        st32(b.psi, oy + iy(1, i, lyo, k), pn);
      }
      if (zl) {
        dHy_dz = fz(0, k, nZo[0], dHy_dz, pn);
        st32(b.psi, oz + iz(0, i, j, k), pn);
        dHx_dz = fz(0, k, nZo[1], dHx_dz, pn);
        st32(b.psi, oz + iz(1, i, j, k), pn);
      }
      const T cx = dHz_dy - dHy_dz;
      const T cy = dHx_dz - dHz_dx;
      const T cz = dHy_dx - dHx_dy;
      const T e0 = tangential_wall(g, 0, i, j, k) ? T(0) : ek[0] + ce * cx;
      const T e1 = tangential_wall(g, 1, i, j, k) ? T(0) : ek[1] + ce * cy;
      const T e2 = tangential_wall(g, 2, i, j, k) ? T(0) : ek[2] + ce * cz;
      st32nt(b.E[0], id, e0);
      st32nt(b.E[1], id, e1);
      st32nt(b.E[2], id, e2);
    }
    hpx = hx;
    hpy = hy;
#pragma unroll
    for (int c = 0; c < 3; ++c) ek[c] = ek1[c];
    prefetch_psi(k + 1);
  }
}

template <typename T, int TX, int TY>
__global__ __launch_bounds__(TX * TY, 4) void k_fused(FieldPtrs<T> a, FieldPtrs<T> b, Geom g,
                                                   Box box, int kz, int ntx, int nty,
                                                   int nblocks) {
  fused_body<T, TX, TY>(a, b, g, box, kz, ntx, nty, nblocks, blockIdx.x);
}

// Boxes where no y or z layer needs stretching (x layers at most): the same body
// without the y/z layer code, built for more waves per SIMD.
template <typename T, int TX, int TY, int CPM, int W>
__global__ __launch_bounds__(TX * TY, W) void k_fused_lean(FieldPtrs<T> a, FieldPtrs<T> b, Geom g,
                                                        Box box, int kz, int ntx, int nty,
                                                        int nblocks) {
  fused_body<T, TX, TY, CPM>(a, b, g, box, kz, ntx, nty, nblocks, blockIdx.x);
}

// The frame of y and z layers around such a box, up to four boxes in one launch
// (full kernel, 64 x 4 tiles): block b belongs to the job whose start range holds it.
template <typename T>
__global__ __launch_bounds__(256, 4) void k_fused_frame(FrameJobs<T> fj) {
  int j = 0;
  while (j + 1 < fj.njobs && (int)blockIdx.x >= fj.start[j + 1]) ++j;
  const FusedJob<T>& J = fj.job[j];
  fused_body<T, 64, 4>(J.a, J.b, J.g, J.box, J.kz, J.ntx, J.nty, J.nblocks,
                   (int)blockIdx.x - fj.start[j]);
}

// One launch over the jobs of a batch of domains (see BatchJobs); CPM and W as for
// the single-domain kernels (the lean form when no job's box reaches a y or z layer).
template <typename T, int TX, int TY, int CPM, int W>
__global__ __launch_bounds__(TX * TY, W) void k_fused_batch(const FusedJob<T>* jobs,
                                                         const int* start, int njobs) {
  const int j = find_job(start, njobs, blockIdx.x);
  const FusedJob<T> J = load_job(jobs, j);
  const int bid = blockIdx.x - start[j];
  if (J.tx != TX || J.ty != TY || bid >= J.nblocks) return;
  fused_body<T, TX, TY, CPM>(J.a, J.b, J.g, J.box, J.kz, J.ntx, J.nty, J.nblocks, bid);
}

// Waves per SIMD the lean kernels are built for: FP32 without layer code needs about
// 71 VGPRs (six waves), with the x layers 87 (five); FP64 and 1024-thread blocks four.
template <typename T, int TX, int TY, int CPM>
struct LeanWaves {
  static constexpr int value = (sizeof(T) == 4 && TX * TY < 1024) ? (CPM == 0 ? 6 : 5) : 4;
};

// cpm: 0 no layer code (no CPML face), 1 x layers only (the box keeps clear of the y
// and z layers), 2 the full kernel
template <typename T, int TX, int TY>
static hipError_t launch_fused(const FieldPtrs<T>& a, const FieldPtrs<T>& b, const Geom& g,
                               const Box& box, int kz, int cpm, hipStream_t st) {
  const int ex = box.hi[0] - box.lo[0], ey = box.hi[1] - box.lo[1], ez = box.hi[2] - box.lo[2];
  if (ex <= 0 || ey <= 0 || ez <= 0) return hipSuccess;
  const int ntx = (box.hi[0] - (box.lo[0] & ~31) + TX - 1) / TX, nty = (ey + TY - 1) / TY;
  const int nch = (ez + kz - 1) / kz;
  const int nblocks = ntx * nty * nch;
  constexpr int W0 = LeanWaves<T, TX, TY, 0>::value, W1 = LeanWaves<T, TX, TY, 1>::value;
  if (cpm == 0)
    hipLaunchKernelGGL((k_fused_lean<T, TX, TY, 0, W0>), dim3(nblocks), dim3(TX * TY), 0, st, a,
                       b, g, box, kz, ntx, nty, nblocks);
  else if (cpm == 1)
    hipLaunchKernelGGL((k_fused_lean<T, TX, TY, 1, W1>), dim3(nblocks), dim3(TX * TY), 0, st, a,
                       b, g, box, kz, ntx, nty, nblocks);
  else
    hipLaunchKernelGGL((k_fused<T, TX, TY>), dim3(nblocks), dim3(TX * TY), 0, st, a, b, g, box,
                       kz, ntx, nty, nblocks);
  return hipGetLastError();
}

// Tile grid of the fused kernel over a box: x tiles of J.tx from the 128-byte
// boundary at or below box.lo, y tiles of J.ty, z chunks of J.kz planes.
template <typename T>
void fused_job_shape(FusedJob<T>& J) {
  const Box& box = J.box;
  const int ex = box.hi[0] - box.lo[0], ey = box.hi[1] - box.lo[1], ez = box.hi[2] - box.lo[2];
  if (ex <= 0 || ey <= 0 || ez <= 0) {
    J.ntx = J.nty = J.nblocks = 0;
    return;
  }
  J.ntx = (box.hi[0] - (box.lo[0] & ~31) + J.tx - 1) / J.tx;
  J.nty = (ey + J.ty - 1) / J.ty;
  J.nblocks = J.ntx * J.nty * ((ez + J.kz - 1) / J.kz);
}
template void fused_job_shape<float>(FusedJob<float>&);
template void fused_job_shape<double>(FusedJob<double>&);

// The leanest kernel that covers the box: none of the layer code when no CPML
// layer reaches it (a halo cell included), the x layers alone when the y and z
// layers stay clear, else everything.
int fused_cpm(const Geom& g, const Box& box) {
  auto clear = [&](int a) {
    if (!has_cpml(g, a)) return true;
    const int lo = g.nlo[a] > 0 ? g.nlo[a] + 1 : 0, hi = g.n[a] - g.nhi[a];
    return box.lo[a] >= lo && box.hi[a] <= hi;
  };
  if (!clear(1) || !clear(2)) return 2;
  return has_cpml(g, 0) ? 1 : 0;
}

template <typename T, int TX>
static hipError_t launch_fused_tx(const FieldPtrs<T>& a, const FieldPtrs<T>& b, const Geom& g,
                                  const Box& box, int kz, int ty, int cpm, hipStream_t st) {
  if (ty == 16) return launch_fused<T, TX, 16>(a, b, g, box, kz, cpm, st);
  if (ty == 8) return launch_fused<T, TX, 8>(a, b, g, box, kz, cpm, st);
  return launch_fused<T, TX, 4>(a, b, g, box, kz, cpm, st);
}

template <typename T>
static hipError_t launch_fused_any(const FieldPtrs<T>& a, const FieldPtrs<T>& b, const Geom& g,
                                   const Box& box, int kz, int tx, int ty, hipStream_t st) {
  const int cpm = fused_cpm(g, box);
  if (tx == 32) return launch_fused_tx<T, 32>(a, b, g, box, kz, ty, cpm, st);
  return launch_fused_tx<T, 64>(a, b, g, box, kz, ty, cpm, st);
}

// The y/z layer frame around an interior box: up to four boxes (the z slabs over
// the whole x-y plane, the y slabs over the box's z range), one launch of the full
// kernel with 64 x 4 tiles.  The slabs are thin, so their chunks are short to give the
// launch enough workgroups: kz planes in the y slabs, four in the z slabs.
template <typename T>
static hipError_t launch_frame(const FieldPtrs<T>& a, const FieldPtrs<T>& b, const Geom& g,
                               const Box& inner, int kz, hipStream_t st) {
  FrameJobs<T> fj{};
  Box boxes[4];
  int nb = 0;
  auto add = [&](int x0, int y0, int z0, int x1, int y1, int z1) {
    if (x1 <= x0 || y1 <= y0 || z1 <= z0) return;
    Box& bx = boxes[nb++];
    bx.lo[0] = x0; bx.lo[1] = y0; bx.lo[2] = z0;
    bx.hi[0] = x1; bx.hi[1] = y1; bx.hi[2] = z1;
  };
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  add(0, 0, 0, nx, ny, inner.lo[2]);
  add(0, 0, inner.hi[2], nx, ny, nz);
  add(0, 0, inner.lo[2], nx, inner.lo[1], inner.hi[2]);
  add(0, inner.hi[1], inner.lo[2], nx, ny, inner.hi[2]);
  int total = 0;
  for (int q = 0; q < nb; ++q) {
    FusedJob<T>& J = fj.job[fj.njobs];
    J.a = a;
    J.b = b;
    J.g = g;
    J.box = boxes[q];
    J.tx = 64;
    J.ty = 4;
    const int ez = boxes[q].hi[2] - boxes[q].lo[2];
    J.kz = std::max(1, std::min(q < 2 ? 4 : kz, ez));
    fused_job_shape(J);
    if (J.nblocks <= 0) continue;
    fj.start[fj.njobs] = total;
    total += J.nblocks;
    ++fj.njobs;
  }
  fj.start[fj.njobs] = total;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fused_frame<T>, dim3(total), dim3(256), 0, st, fj);
  return hipGetLastError();
}

template <typename T, int TX, int TY>
static void launch_fused_batch_t(const FusedJob<T>* jobs, const int* start, int njobs,
                                 int nblocks, bool lean, hipStream_t st) {
  if (lean)
    hipLaunchKernelGGL((k_fused_batch<T, TX, TY, 1, LeanWaves<T, TX, TY, 1>::value>),
                       dim3(nblocks), dim3(TX * TY), 0, st, jobs, start, njobs);
  else
    hipLaunchKernelGGL((k_fused_batch<T, TX, TY, 2, 4>), dim3(nblocks), dim3(TX * TY), 0, st,
                       jobs, start, njobs);
}

template <typename T, int TX>
static void launch_fused_batch_tx(const FusedJob<T>* jobs, const int* start, int njobs,
                                  int nblocks, int ty, bool lean, hipStream_t st) {
  if (ty == 16) launch_fused_batch_t<T, TX, 16>(jobs, start, njobs, nblocks, lean, st);
  else if (ty == 8) launch_fused_batch_t<T, TX, 8>(jobs, start, njobs, nblocks, lean, st);
  else launch_fused_batch_t<T, TX, 4>(jobs, start, njobs, nblocks, lean, st);
}

template <typename T>
static hipError_t launch_fused_batch(const FusedJob<T>* jobs, const int* start, int njobs,
                                     int nblocks, int tx, int ty, bool lean, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  if (tx == 32) launch_fused_batch_tx<T, 32>(jobs, start, njobs, nblocks, ty, lean, st);
  else launch_fused_batch_tx<T, 64>(jobs, start, njobs, nblocks, ty, lean, st);
  return hipGetLastError();
}

hipError_t sweep_fused_f64(const FieldPtrs<double>& a, const FieldPtrs<double>& b, const Geom& g,
                           const Box& box, int kz, int tx, int ty, hipStream_t st) {
  return launch_fused_any<double>(a, b, g, box, kz, tx, ty, st);
}
hipError_t sweep_fused_f32(const FieldPtrs<float>& a, const FieldPtrs<float>& b, const Geom& g,
                           const Box& box, int kz, int tx, int ty, hipStream_t st) {
  return launch_fused_any<float>(a, b, g, box, kz, tx, ty, st);
}
hipError_t sweep_frame_f64(const FieldPtrs<double>& a, const FieldPtrs<double>& b, const Geom& g,
                           const Box& inner, int kz, hipStream_t st) {
  return launch_frame<double>(a, b, g, inner, kz, st);
}
hipError_t sweep_frame_f32(const FieldPtrs<float>& a, const FieldPtrs<float>& b, const Geom& g,
                           const Box& inner, int kz, hipStream_t st) {
  return launch_frame<float>(a, b, g, inner, kz, st);
}
hipError_t sweep_fused_batch_f64(const FusedJob<double>* jobs, const int* start, int njobs,
                                 int nblocks, int tx, int ty, bool lean, hipStream_t st) {
  return launch_fused_batch<double>(jobs, start, njobs, nblocks, tx, ty, lean, st);
}
hipError_t sweep_fused_batch_f32(const FusedJob<float>* jobs, const int* start, int njobs,
                                 int nblocks, int tx, int ty, bool lean, hipStream_t st) {
  return launch_fused_batch<float>(jobs, start, njobs, nblocks, tx, ty, lean, st);
}

}  // namespace mlk
