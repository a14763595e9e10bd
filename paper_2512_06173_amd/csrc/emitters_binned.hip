// Tile-binned emitter phase.
//
// gather (eq. E_regu_Emi): the emitters are grouped by the bin of their
// centre cell.  The workgroup of a bin stages E over the bin plus a halo of
// kHalo cells in LDS, which holds every window of its emitters.  Eight lanes
// (FP32 fields) or sixteen (FP64) serve one emitter, lane (i, h) taking the x
// offset i of its window and the h-th share of its rows: a lane sums its rows
// along y in the field precision, weights them along z into FP64, and the
// lanes of the emitter add up their sums (FP64).  The weights come from the
// emitter's record into registers.  Bins are handed out XCD by XCD so that
// neighbouring bins, whose halos overlap, share one L2.  Extra workgroups of
// the same launch save the flux plane's E^n.
//
// step (eq. von-Neumann-tls, eq. dipole_derivative): one thread per two-level
// emitter advances its state with the exact propagator and writes mu_dot.
//
// scatter (eqs. J_mol, Polarization_mol):  E_c(p) -= (dt/eps_r(p)) gamma mu_dot^c
// w^c_{m,p} / dx^3.  A workgroup owns a bin of cells and takes every (emitter,
// bin) pair whose window touches the bin, eight lanes per pair; the pair
// carries its window's runs inside the bin, set up on the host.  Contributions
// are summed in LDS (as fixed-point integers, see scatter_body) and each cell
// is written once by its owner (no global atomics).  The pairs' records are
// copied into LDS with 16-byte loads, so the inner loops touch LDS only.
//
// Window weights are the separable factors wx wy wz set up by k_windows, kept
// per emitter as a union-window record (WinRec); a component uses the
// half-integer variant on its own axis.
#include "mlk_internal.h"
#include "tls_math.h"

namespace mlk {

template <typename T>
struct BinCfg;
template <>
struct BinCfg<float> {
  // gather: 16 x 8 x 8 bins, 24 x 16 x 16 tile (74 KB); scatter: 16^3 bins (48 KB)
  static constexpr int GX = 16, GY = 8, GZ = 8;
  static constexpr int SX = 16, SY = 16, SZ = 16;
};
template <>
struct BinCfg<double> {
  // gather: 8 x 8 x 8 bins, 16 x 16 x 16 tile (98 KB); scatter: 16 x 16 x 8 bins (48 KB)
  static constexpr int GX = 8, GY = 8, GZ = 8;
  static constexpr int SX = 16, SY = 16, SZ = 8;
};

// A gather bin of at most this many emitters is light: it stages only the cells
// that its windows cover (7^3 per window against the 24 x 16 x 16 tile).
int gather_light_max() { return 4; }

void bin_shape(bool fp32, int G[3], int S[3]) {
  if (fp32) {
    G[0] = BinCfg<float>::GX; G[1] = BinCfg<float>::GY; G[2] = BinCfg<float>::GZ;
    S[0] = BinCfg<float>::SX; S[1] = BinCfg<float>::SY; S[2] = BinCfg<float>::SZ;
  } else {
    G[0] = BinCfg<double>::GX; G[1] = BinCfg<double>::GY; G[2] = BinCfg<double>::GZ;
    S[0] = BinCfg<double>::SX; S[1] = BinCfg<double>::SY; S[2] = BinCfg<double>::SZ;
  }
}

namespace {

constexpr int kLanesPerEmitter = 8;  // = kMaxWin: one lane per window x offset
constexpr int kLightThreads = 256;   // threads per block of the light-emitter gather
constexpr int kThreads = 512;
constexpr int kGroups = kThreads / kLanesPerEmitter;  // emitters in flight per workgroup
// Gather launch shape.  The tile fill is latency-bound, so a bin runs sixteen
// wavefronts: in FP32 two workgroups share a CU (LDS and registers: at most 64
// VGPRs, eight wavefronts per SIMD), in FP64 one (98 KB of tile).  An emitter
// takes `lanes` lanes: lane (i, h) on window x offset i and rows h*rows ..
// h*rows+rows-1.  FP64 splits the rows over sixteen lanes, which halves the
// chain of each lane's sums and its registers (122, within the 128 that 1024
// threads allow); measured, FP32 is faster with eight.
template <typename T>
struct GatherCfg {
  static constexpr int threads = 1024;
  static constexpr int waves_per_simd = sizeof(T) == 4 ? 8 : 1;
  static constexpr int lanes = sizeof(T) == 4 ? 8 : 16;
  static constexpr int rows = kMaxWin * kLanesPerEmitter / lanes;
};

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// sum over the L consecutive lanes of one gather emitter
template <int L>
__device__ __forceinline__ double gather_lane_sum(double v) {
#pragma unroll
  for (int off = L / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, L);
  return v;
}

// One plane's term of an emitter's z sum, a + wz s, rounded alike by every gather
// path: in FP64 as one fused multiply-add, in FP32 with the product rounded in FP32
// and the sum in FP64.
__device__ __forceinline__ double zterm(double a, double wz, double s) {
  return __builtin_fma(wz, s, a);
}
__device__ __forceinline__ double zterm(double a, float wz, float s) {
  return a + (double)(wz * s);
}

// The part of an emitter's window record that one gather lane needs, in
// registers: the union window, the lane's own x weights, the y weights of its
// rows and every z weight (the lanes of an emitter read the same record).
template <typename T>
struct LaneWin {
  int org[3], n[3];
  T wx0, wx1;
  T wy[2][GatherCfg<T>::rows], wz[2][kMaxWin];
};

template <typename T>
__device__ __forceinline__ void load_lane_win(const WinRec<T>& r, int i, int j0, LaneWin<T>& w) {
  const int4 o = *reinterpret_cast<const int4*>(&r.org[0]);  // org[0..2], n[0]
  const int2 nn = *reinterpret_cast<const int2*>(&r.n[1]);
  w.org[0] = o.x;
  w.org[1] = o.y;
  w.org[2] = o.z;
  w.n[0] = o.w;
  w.n[1] = nn.x;
  w.n[2] = nn.y;
  w.wx0 = r.wr[0][0][i];
  w.wx1 = r.wr[0][1][i];
#pragma unroll
  for (int v = 0; v < 2; ++v) {
#pragma unroll
    for (int d = 0; d < GatherCfg<T>::rows; ++d) w.wy[v][d] = r.wr[1][v][j0 + d];
#pragma unroll
    for (int d = 0; d < kMaxWin; ++d) w.wz[v][d] = r.wr[2][v][d];
  }
}

}  // namespace

// gather; see the file comment.  Writes E~ = gamma * sum w E (FP64) per emitter.
// WEPS: gather eps_r^-1 E instead of E (the adjoint step needs it).
template <typename T, bool WEPS = false>
__device__ __forceinline__ void gather_body(const FieldPtrs<T>& f, const Geom& g,
                                            const BinPtrs& bins, const WindowPtrs<T>& win,
                                            double* Et, int bid) {
  constexpr int BX = BinCfg<T>::GX, BY = BinCfg<T>::GY, BZ = BinCfg<T>::GZ;
  constexpr int NT = GatherCfg<T>::threads, LG = GatherCfg<T>::lanes, NG = NT / LG;
  constexpr int RG = GatherCfg<T>::rows;
  constexpr int TX = BX + 2 * kHalo, TY = BY + 2 * kHalo, TZ = BZ + 2 * kHalo;
  __shared__ T sE[3][TX * TY * TZ];
  const int tid = threadIdx.x;
  const bool light = bid >= bins.gdense;  // uniform across the block
  const int bin = light ? bid : xcd_block(bid, bins.gdense);
  // tile origin in the unwrapped frame of the emitters' window indices
  const int x0 = bins.gbin_org[3 * bin] - kHalo;
  const int y0 = bins.gbin_org[3 * bin + 1] - kHalo;
  const int z0 = bins.gbin_org[3 * bin + 2] - kHalo;
  // the bin's emitter range and each group's first emitter id, loaded with the
  // tile so that the sums start right after the barrier
  const int grp = tid / LG, i = tid % kLanesPerEmitter;
  const int q0 = bins.gbin_start[bin], q1 = bins.gbin_start[bin + 1];
  int e_next = q0 + grp < q1 ? bins.gbin_em[q0 + grp] : 0;

  // E (times 1/eps_r with WEPS) of tile cell (li, lj, lk), from a safe index:
  // zero beyond a non-periodic face
  auto tile_cell = [&](int li, int lj, int lk, T& e0, T& e1, T& e2) {
    int q[3] = {x0 + li, y0 + lj, z0 + lk};
    bool ok = true;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      if (g.periodic[ax]) {
        const int m = q[ax] % g.n[ax];
        q[ax] = m < 0 ? m + g.n[ax] : m;
      } else {
        ok = ok && q[ax] >= 0 && q[ax] < g.n[ax];
      }
    }
    const size_t id = ok ? cell_index(g, q[0], q[1], q[2]) : 0;
    e0 = f.E[0][id];
    e1 = f.E[1][id];
    e2 = f.E[2][id];
    if (WEPS && f.epsinv) {  // null: eps_r = 1 everywhere
      const T ei = f.epsinv[id];
      e0 *= ei;
      e1 *= ei;
      e2 *= ei;
    }
    e0 = ok ? e0 : T(0);
    e1 = ok ? e1 : T(0);
    e2 = ok ? e2 : T(0);
  };
  if (light) {
    // A light bin stages only the box that its few windows cover (the union of
    // [org, org + n) per axis): the same values at the cells its sums read.
    int lo[3] = {TX, TY, TZ}, hi[3] = {0, 0, 0};
    for (int q = q0; q < q1; ++q) {
      const WinRec<T>& r = win.rec[bins.gbin_em[q]];
      const int4 o = *reinterpret_cast<const int4*>(&r.org[0]);  // org[0..2], n[0]
      const int2 nn = *reinterpret_cast<const int2*>(&r.n[1]);
      lo[0] = min(lo[0], o.x - x0);
      lo[1] = min(lo[1], o.y - y0);
      lo[2] = min(lo[2], o.z - z0);
      hi[0] = max(hi[0], o.x - x0 + o.w);
      hi[1] = max(hi[1], o.y - y0 + nn.x);
      hi[2] = max(hi[2], o.z - z0 + nn.y);
    }
    const int nx = hi[0] - lo[0], ny = hi[1] - lo[1], nxy = nx * (hi[1] - lo[1]);
    const int cells = nxy * (hi[2] - lo[2]);
    for (int t = tid; t < cells; t += NT) {
      const int li = lo[0] + t % nx, lj = lo[1] + (t / nx) % ny, lk = lo[2] + t / nxy;
      T e0, e1, e2;
      tile_cell(li, lj, lk, e0, e1, e2);
      const int s = li + TX * (lj + TY * lk);
      sE[0][s] = e0;
      sE[1][s] = e1;
      sE[2][s] = e2;
    }
  } else {
    // stage the tile: every load of a thread is issued before the first LDS
    // store, so they are in flight together
    constexpr int NTILE = TX * TY * TZ;
    static_assert(NTILE % NT == 0, "the tile is a whole number of workgroup passes");
    constexpr int RF = NTILE / NT;
    T v[RF][3];
#pragma unroll
    for (int r = 0; r < RF; ++r) {
      const int t = tid + r * NT;
      tile_cell(t % TX, (t / TX) % TY, t / (TX * TY), v[r][0], v[r][1], v[r][2]);
    }
#pragma unroll
    for (int r = 0; r < RF; ++r) {
      const int t = tid + r * NT;
      sE[0][t] = v[r][0];
      sE[1][t] = v[r][1];
      sE[2][t] = v[r][2];
    }
  }

  __syncthreads();

  const int j0 = (tid / kLanesPerEmitter) % (LG / kLanesPerEmitter) * RG;
  for (int q = q0 + grp; q < q1; q += NG) {  // uniform across the lanes of an emitter
    const int e = e_next;
    if (q + NG < q1) e_next = bins.gbin_em[q + NG];
    LaneWin<T> w;
    load_lane_win(win.rec[e], i, j0, w);
    double ax = 0.0, ay = 0.0, az = 0.0;
    if (i < w.n[0]) {
      const int ny = w.n[1] - j0, nz = w.n[2];
      int s = (w.org[0] + i - x0) + TX * (w.org[1] + j0 - y0) + TX * TY * (w.org[2] - z0);
      // The sums read every row of a plane before adding them up (no branch per
      // row), one component at a time, so that the reads of a plane are in flight
      // together.  Rows past the window (j >= ny) read the window's first row, a
      // staged cell, with the record's zero weight: their terms are zeros and leave
      // the sums as they are.  (FP64: emitter phase 131 -> 118 us at 256^3 with
      // 100,000 emitters; FP32 unchanged, its row-by-row form ran as fast.)
      int roff[RG];
#pragma unroll
      for (int j = 0; j < RG; ++j) roff[j] = j < ny ? TX * j : -TX * j0;
      // Ex and Ez take the integer y weights, Ey the half-integer ones; Ez the
      // half-integer z weights
      auto comp = [&](const T* sEc, const T* wy, const T* wz) -> double {
        double a = 0.0;
        int sk = s;
#pragma unroll
        for (int k = 0; k < kMaxWin; ++k, sk += TX * TY) {
          if (k < nz) {
            T v[RG];
#pragma unroll
            for (int j = 0; j < RG; ++j) v[j] = sEc[sk + roff[j]];
            T sc = T(0);
#pragma unroll
            for (int j = 0; j < RG; ++j) sc += wy[j] * v[j];
            a = zterm(a, wz[k], sc);
          }
        }
        return a;
      };
      ax = comp(sE[0], w.wy[0], w.wz[0]);
      ay = comp(sE[1], w.wy[1], w.wz[0]);
      az = comp(sE[2], w.wy[0], w.wz[1]);
      // Ex sits at half-integer x (variant 1); Ey, Ez at integer x
      ax *= (double)w.wx1;
      ay *= (double)w.wx0;
      az *= (double)w.wx0;
    }
    ax = gather_lane_sum<LG>(ax);
    ay = gather_lane_sum<LG>(ay);
    az = gather_lane_sum<LG>(az);
    if (i == 0) {
      const double gm = win.gamma[e];
      Et[3 * e] = gm * ax;
      Et[3 * e + 1] = gm * ay;
      Et[3 * e + 2] = gm * az;
    }
  }
}

// The emitters of the light bins, without a tile: a wavefront per emitter, lane
// (i, k) on window x offset i and plane k, reading its window cells from global
// memory (every row of its plane, for each of the row groups h that the tiled
// gather gives separate lanes).  A lane forms the tiled gather's row sums
// sum_j wy E for its plane; the plane-0 lanes then take the z sums in plane order,
// scale by the x weight, join the row groups and sum over x as the tiled gather's
// lanes do, so E~ is the same bit for bit.  All planes' loads are
// in flight together (a lane per plane), where a lane walking the planes one after
// another would wait on each.  em: the emitter ids, count of them.
template <typename T>
__device__ __forceinline__ void light_body(const FieldPtrs<T>& f, const Geom& g, const int* em,
                                           int count, const WindowPtrs<T>& win, double* Et,
                                           int bid) {
  constexpr int RG = GatherCfg<T>::rows, H = GatherCfg<T>::lanes / kLanesPerEmitter;
  constexpr int NG = kLightThreads / 64;
  static_assert(kLanesPerEmitter * kMaxWin == 64, "one lane per (x offset, plane)");
  const int tid = threadIdx.x, lane = tid & 63;
  const int i = lane % kLanesPerEmitter, k = lane / kLanesPerEmitter;
  const int q = bid * NG + tid / 64;
  if (q >= count) return;  // uniform across the wavefront
  const int e = em[q];
  const WinRec<T>& r = win.rec[e];
  const int4 o = *reinterpret_cast<const int4*>(&r.org[0]);  // org[0..2], n[0]
  const int2 nn = *reinterpret_cast<const int2*>(&r.n[1]);
  const int nz = nn.y;
  T t[H][3];  // the lane's row sums of its plane, per row group and component
#pragma unroll
  for (int h = 0; h < H; ++h) t[h][0] = t[h][1] = t[h][2] = T(0);
  if (i < o.w && k < nz) {
    // window cells in the grid: wrapped on a periodic axis; beyond a wall the tile
    // holds zero, and so does this path
    int cx = o.x + i, cz = o.z + k;
    bool ok0 = true;
    if (g.periodic[0]) {
      cx %= g.n[0];
      cx = cx < 0 ? cx + g.n[0] : cx;
    } else {
      ok0 = cx >= 0 && cx < g.n[0];
    }
    if (g.periodic[2]) {
      cz %= g.n[2];
      cz = cz < 0 ? cz + g.n[2] : cz;
    } else {
      ok0 = ok0 && cz >= 0 && cz < g.n[2];
    }
    T v[H][RG][3];
    unsigned okm[H];
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const int ny = nn.x - h * RG;
      okm[h] = 0u;
#pragma unroll
      for (int j = 0; j < RG; ++j) {
        int cy = o.y + h * RG + j;
        bool ok = ok0 && j < ny;
        if (g.periodic[1]) {
          cy %= g.n[1];
          cy = cy < 0 ? cy + g.n[1] : cy;
        } else {
          ok = ok && cy >= 0 && cy < g.n[1];
        }
        okm[h] |= ok ? (1u << j) : 0u;
        const size_t id = ok ? cell_index(g, cx, cy, cz) : 0;
        v[h][j][0] = f.E[0][id];
        v[h][j][1] = f.E[1][id];
        v[h][j][2] = f.E[2][id];
      }
    }
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const int ny = nn.x - h * RG;
      T sx = T(0), sy = T(0), sz = T(0);
#pragma unroll
      for (int j = 0; j < RG; ++j) {
        if (j < ny) {
          const bool ok = (okm[h] >> j) & 1u;
          const T wy0 = r.wr[1][0][h * RG + j], wy1 = r.wr[1][1][h * RG + j];
          sx += wy0 * (ok ? v[h][j][0] : T(0));
          sy += wy1 * (ok ? v[h][j][1] : T(0));
          sz += wy0 * (ok ? v[h][j][2] : T(0));
        }
      }
      t[h][0] = sx;
      t[h][1] = sy;
      t[h][2] = sz;
    }
  }
  // the z sums in plane order (every lane takes part in the shuffles; the plane-0
  // lanes keep the sums); Ez takes the half-integer z weights
  double a[H][3];
#pragma unroll
  for (int h = 0; h < H; ++h) a[h][0] = a[h][1] = a[h][2] = 0.0;
#pragma unroll
  for (int kk = 0; kk < kMaxWin; ++kk) {
    if (kk < nz) {  // uniform across the wavefront
      const T wz0 = r.wr[2][0][kk], wz1 = r.wr[2][1][kk];
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const int src = i + kLanesPerEmitter * kk;
        a[h][0] = zterm(a[h][0], wz0, __shfl(t[h][0], src, 64));
        a[h][1] = zterm(a[h][1], wz0, __shfl(t[h][1], src, 64));
        a[h][2] = zterm(a[h][2], wz1, __shfl(t[h][2], src, 64));
      }
    }
  }
  if (i < o.w) {
    // Ex sits at half-integer x (variant 1); Ey, Ez at integer x
    const double wx0 = (double)r.wr[0][0][i], wx1 = (double)r.wr[0][1][i];
#pragma unroll
    for (int h = 0; h < H; ++h) {
      a[h][0] *= wx1;
      a[h][1] *= wx0;
      a[h][2] *= wx0;
    }
  }
  // the row groups of one x offset, then the x offsets: the tiled gather's lane sum
  double ax = a[0][0], ay = a[0][1], az = a[0][2];
  if (H == 2) {
    ax += a[H - 1][0];
    ay += a[H - 1][1];
    az += a[H - 1][2];
  }
  ax = gather_lane_sum<kLanesPerEmitter>(ax);
  ay = gather_lane_sum<kLanesPerEmitter>(ay);
  az = gather_lane_sum<kLanesPerEmitter>(az);
  if (lane == 0) {
    const double gm = win.gamma[e];
    Et[3 * e] = gm * ax;
    Et[3 * e + 1] = gm * ay;
    Et[3 * e + 2] = gm * az;
  }
}

template <typename T>
__global__ __launch_bounds__(kLightThreads) void k_gather_light(FieldPtrs<T> f, Geom g,
                                                                const int* em, int count,
                                                                WindowPtrs<T> win, double* Et) {
  light_body(f, g, em, count, win, Et, blockIdx.x);
}

template <typename T>
__global__ __launch_bounds__(kLightThreads) void k_gather_light_batch(const LightJob<T>* jobs,
                                                                      const int* start,
                                                                      int njobs) {
  const int j = find_job(start, njobs, blockIdx.x);
  const LightJob<T> J = load_job(jobs, j);
  const int bid = blockIdx.x - start[j];
  if (bid >= J.nblocks) return;
  light_body(J.f, J.g, J.em, J.count, J.win, J.Et, bid);
}

// The staged bins (the light ones have a kernel of their own); the blocks past them,
// if any, save the flux plane's E^n (one launch fewer per step; both read E^n only).
template <typename T>
__global__ __launch_bounds__(GatherCfg<T>::threads, GatherCfg<T>::waves_per_simd) void k_gather_bins(
    FieldPtrs<T> f, Geom g, BinPtrs bins, WindowPtrs<T> win, double* Et, FluxPlane fp) {
  if ((int)blockIdx.x >= bins.gdense) {  // uniform across the block
    flux_save_body(f, g, fp, ((int)blockIdx.x - bins.gdense) * GatherCfg<T>::threads +
                                 (int)threadIdx.x);
    return;
  }
  gather_body(f, g, bins, win, Et, blockIdx.x);
}

template <typename T>
__global__ __launch_bounds__(GatherCfg<T>::threads, GatherCfg<T>::waves_per_simd) void k_gather_batch(const GatherJob<T>* jobs,
                                                           const int* start, int njobs,
                                                           const int2* order) {
  int j, bid;
  if (order) {  // (job, bin) of the block, heaviest first across the jobs
    const int2 o = order[blockIdx.x];
    j = o.x;
    bid = o.y;
  } else {
    j = find_job(start, njobs, blockIdx.x);
    bid = blockIdx.x - start[j];
    if (bid >= jobs[j].nblocks) return;
  }
  const GatherJob<T> J = load_job(jobs, j);
  gather_body(J.f, J.g, J.bins, J.win, J.Et, bid);
}

// Exact two-level step of every two-level emitter under its E~ (one thread each).
__device__ __forceinline__ void tls_body(const TlsPtrs& tls, double dt, const double* Et,
                                         double* mudot, const int64_t* pop_off, const Series& ser,
                                         const int64_t* step, int m) {
  if (m >= tls.count) return;
  const int e = tls.gid[m];
  const double et[3] = {Et[3 * e], Et[3 * e + 1], Et[3 * e + 2]};
  const double d[3] = {tls.dip[3 * m], tls.dip[3 * m + 1], tls.dip[3 * m + 2]};
  double st[3] = {tls.rho[3 * m], tls.rho[3 * m + 1], tls.rho[3 * m + 2]};
  double md[3];
  tls_advance(tls.omega0[m], d, et, dt, st, md);
  if (!isfinite(st[0] + st[1] + st[2] + md[0] + md[1] + md[2])) flag_nonfinite(ser, *step);
  tls.rho[3 * m] = st[0];
  tls.rho[3 * m + 1] = st[1];
  tls.rho[3 * m + 2] = st[2];
  mudot[3 * e] = md[0];
  mudot[3 * e + 1] = md[1];
  mudot[3 * e + 2] = md[2];
  if (ser.pop_every > 0) {
    const int64_t n = *step;
    if (n % ser.pop_every == 0) ser.pop[(n / ser.pop_every) * ser.npop + pop_off[e]] = st[0];
  }
}

__global__ __launch_bounds__(256) void k_tls_step(TlsPtrs tls, double dt, const double* Et,
                                                  double* mudot, const int64_t* pop_off,
                                                  Series ser, const int64_t* step) {
  tls_body(tls, dt, Et, mudot, pop_off, ser, step, blockIdx.x * blockDim.x + threadIdx.x);
}

// Cavity mode with two-level emitters only: each thread forms the mode's common
// field E~ = -(eps q_l + d_l / V) e_l for its emitter, steps it, and the block
// sums <mu> + (dt/2) mu_dot of the new state, x and y (the emitter's share of
// the mode's total dipole at the next integer time), in a fixed tree order into
// c.partial[block].  <mu> = 2 Re rho01 d.
__global__ __launch_bounds__(kTlsThreads) void k_cavity_tls(TlsPtrs tls, double dt, CavityDev c,
                                                            double* Et, double* mudot,
                                                            const int64_t* pop_off, Series ser,
                                                            const int64_t* step) {
  __shared__ double rx[kTlsThreads], ry[kTlsThreads];
  const int t = threadIdx.x, m = blockIdx.x * kTlsThreads + t;
  double sx = 0.0, sy = 0.0;
  if (m < tls.count) {
    const int e = tls.gid[m];
    Et[3 * e + 0] = -(c.eps * c.st[0] + c.st[4] / c.V);
    Et[3 * e + 1] = -(c.eps * c.st[1] + c.st[5] / c.V);
    Et[3 * e + 2] = 0.0;
    tls_body(tls, dt, Et, mudot, pop_off, ser, step, m);
    const double mu = 2.0 * tls.rho[3 * m + 1];
    sx = mu * tls.dip[3 * m + 0] + 0.5 * dt * mudot[3 * e + 0];
    sy = mu * tls.dip[3 * m + 1] + 0.5 * dt * mudot[3 * e + 1];
  }
  rx[t] = sx;
  ry[t] = sy;
  __syncthreads();
  for (int w = kTlsThreads / 2; w > 0; w >>= 1) {
    if (t < w) {
      rx[t] += rx[t + w];
      ry[t] += ry[t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    c.partial[2 * blockIdx.x + 0] = rx[0];
    c.partial[2 * blockIdx.x + 1] = ry[0];
  }
}

__global__ __launch_bounds__(256) void k_tls_batch(const TlsJob* jobs, const int* start,
                                                   int njobs) {
  const int j = find_job(start, njobs, blockIdx.x);
  const TlsJob J = load_job(jobs, j);
  const int lb = blockIdx.x - start[j];
  if (lb >= J.nblocks) return;
  tls_body(J.tls, J.dt, J.Et, J.mudot, J.pop_off, J.ser, J.step, lb * blockDim.x + threadIdx.x);
}

// Fixed-point accumulator of the scatter: 32-bit for FP32 fields, 64-bit for FP64.
template <typename T>
struct Acc;
template <>
struct Acc<float> {
  using U = unsigned int;
  using S = int;
  static constexpr int BITS = 30;
  // onto the grid by truncation (one conversion); the grid step is 2^-30 of the
  // bin's bound, far below the FP32 rounding of a cell's sum
  __device__ static S round(float v) { return (S)v; }
};
template <>
struct Acc<double> {
  using U = unsigned long long;
  using S = long long;
  static constexpr int BITS = 62;
  __device__ static S round(double v) { return __double2ll_rn(v); }
};

// scatter; see the file comment.  Contributions are rounded to a fixed-point
// grid chosen per bin and summed as integers in LDS: integer addition is exact
// and order-independent, so the result is deterministic.  In FP32 the Ex and Ey
// sums of a cell share one 64-bit integer, Ey 2^32 + Ex: its sum is exact, and
// since each component's sum stays below 2^30 in magnitude, Ex is the low 32 bits
// read as a signed value and Ey the rest (two LDS atomics per cell, not three).  The grid is
// 2^-BITS of a bound on any cell's sum (|amp| times the largest window weight,
// summed over the bin's emitters): 2^-62 for FP64 fields, far below FP64
// rounding; 2^-30 for FP32 fields, at the level of FP32 rounding of a cell's
// sum.  A contribution is formed in the field precision.
// E_c(p) -= [eps_r^-1(p) if EPS] amp0 gamma a^c w^c_p over the windows, with
// a = mudot (the forward current: amp0 = dt / dx^3, EPS) or any other per-emitter
// amplitude (the adjoint step: amp0 = -1, no EPS).
//
// A pair (emitter, bin) comes with its window's runs inside the bin, one per
// axis, set up on the host (see PairDesc): window offsets d0 .. d0+c-1 on the
// bin-local cells l0 .. l0+c-1.  A window that wraps inside one bin (a periodic
// axis no longer than the bin) is split into several pairs.
//
// Blocks from bins.nscatter on (when fp is given) form the flux partials of the plane
// instead, in the accumulators' LDS.
template <typename T, bool EPS = true>
__device__ __forceinline__ void scatter_body(const FieldPtrs<T>& f, const Geom& g,
                                             const BinPtrs& bins, const WindowPtrs<T>& win,
                                             const double* mudot, double amp0, int bid,
                                             const FluxPlane* fp = nullptr) {
  using A = Acc<T>;
  constexpr int BX = BinCfg<T>::SX, BY = BinCfg<T>::SY, BZ = BinCfg<T>::SZ;
  constexpr int CELLS = BX * BY * BZ;
  constexpr int NW = kThreads / 64;
  constexpr int R4 = sizeof(WinRec<T>) / sizeof(int4);       // 16-byte pieces of a record
  constexpr int NP = (kGroups * R4 + kThreads - 1) / kThreads;  // pieces per thread and chunk
  static_assert(BX <= 16 && BY <= 16 && BZ <= 16, "bin-local run starts take four bits");
  // emitter ids of a bin's pairs kept in LDS (beyond: read from HBM); sized so
  // that two workgroups still fit one CU's LDS
  constexpr int kIdCap = sizeof(T) == 4 ? 4096 : 1024;
  __shared__ alignas(16) typename A::U sJ[3][CELLS];
  // FP32: Ex and Ey share one 64-bit accumulator per cell (sJ[0] and sJ[1] reused),
  // two LDS atomics per cell instead of three
  constexpr bool kPackXY = sizeof(T) == 4;
  unsigned long long* const sJxy = reinterpret_cast<unsigned long long*>(&sJ[0][0]);
  __shared__ WinRec<T> sW[kGroups];
  __shared__ T sAmp[kGroups][3];
  __shared__ unsigned sRun[kGroups];
  __shared__ int sId[kIdCap];
  __shared__ double sRed[NW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (fp && bid >= bins.nscatter) {  // uniform across the block
    flux_partial_sum(f, g, *fp, bid - bins.nscatter, fp->nblocks,
                     reinterpret_cast<double*>(&sJ[0][0]));
    return;
  }
  const int b = bins.sbin_id[bid];
  const int bx = b % bins.nbx, by = (b / bins.nbx) % bins.nby, bz = b / (bins.nbx * bins.nby);
  const int x0 = bx * BX, y0 = by * BY, z0 = bz * BZ;
  const int ex = min(BX, g.n[0] - x0), ey = min(BY, g.n[1] - y0), ez = min(BZ, g.n[2] - z0);
  const int q0 = bins.sbin_start[bid], q1 = bins.sbin_start[bid + 1];
  {
    // cleared 16 bytes at a time (the three accumulator arrays are contiguous)
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    u4* z = reinterpret_cast<u4*>(&sJ[0][0]);
    constexpr int NZ = 3 * CELLS * (int)sizeof(typename A::U) / 16;
    for (int t = tid; t < NZ; t += kThreads) z[t] = u4{0u, 0u, 0u, 0u};
  }
  double bound = 0.0;
  for (int q = q0 + tid; q < q1; q += kThreads) {
    const int4 pd = bins.sbin_pair[q];
    if (q - q0 < kIdCap) sId[q - q0] = pd.x;
    bound += (double)__int_as_float(pd.z) *
             (fabs(mudot[3 * pd.x]) + fabs(mudot[3 * pd.x + 1]) + fabs(mudot[3 * pd.x + 2]));
  }
  bound = wave_sum64(bound);
  if (lane == 0) sRed[wave] = bound;
  __syncthreads();
  bound = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) bound += sRed[w];
  bound *= fabs(amp0);
  if (!(bound > 0.0)) return;  // nothing to add in this bin (uniform across the block)
  // scale = 2^(BITS - e) with bound < 2^e: every partial sum stays below 2^BITS
  const int ebits = ilogb(bound) + 1;
  const double scale = ldexp(1.0, A::BITS - ebits);
  const double inv_scale = ldexp(1.0, ebits - A::BITS);

  // The pairs are taken in chunks of kGroups.  With FP32 fields the next
  // chunk's window records, runs and amplitudes (gamma, mu_dot) are loaded into
  // registers while the current chunk is summed, and moved to LDS behind an
  // LDS-only barrier, so their HBM latency overlaps the atomics instead of
  // stalling every chunk.  FP64 records are twice as large: holding them across
  // the sums would cost the second workgroup per CU, so FP64 loads each chunk
  // right before storing it.
  constexpr bool kPipe = sizeof(T) == 4;
  typedef int piece_t __attribute__((ext_vector_type(4)));  // kept in registers
  piece_t piece[NP];
  double pg = 0.0, pm0 = 0.0, pm1 = 0.0, pm2 = 0.0;
  unsigned prun = 0;
  // Eight lanes per pair, lane i on the i-th window x offset of the pair's x run;
  // the group walks the cy x cz rows and planes of its y and z runs, so a
  // wavefront runs its eight groups' loops side by side for as many steps as its
  // longest group; the host orders the pairs of a bin by (cz, cy) so that
  // neighbouring groups have equal counts.
  const int grp = tid / kLanesPerEmitter, i = tid % kLanesPerEmitter;
  // loads of the chunk at c: pieces (clamped to the chunk's last record) and, for
  // tid < the chunk size, the runs and amplitude inputs of pair tid
#define MLK_STAGE_LOAD(c)                                                             \
  {                                                                                  \
    const int cl = min(kGroups, q1 - (c)) - 1;                                       \
    _Pragma("unroll") for (int p = 0; p < NP; ++p) {                                 \
      const int idx = tid + p * kThreads, sl = min(idx / R4, cl);                    \
      const int q = (c) + sl;                                                        \
      const int em = q - q0 < kIdCap ? sId[q - q0] : bins.sbin_pair[q].x;            \
      piece[p] = reinterpret_cast<const piece_t*>(win.rec + em)[idx % R4];           \
    }                                                                                \
    const int q = (c) + min(tid, cl);                                                \
    const int4 pd = bins.sbin_pair[q];                                               \
    prun = (unsigned)pd.y;                                                           \
    pg = win.gamma[pd.x];                                                            \
    pm0 = mudot[3 * pd.x];                                                           \
    pm1 = mudot[3 * pd.x + 1];                                                       \
    pm2 = mudot[3 * pd.x + 2];                                                       \
  }
  if (kPipe) MLK_STAGE_LOAD(q0)
  for (int c0 = q0; c0 < q1; c0 += kGroups) {
    const int cn = min(kGroups, q1 - c0);
    if (c0 > q0) lds_barrier();  // the previous chunk's records are no longer read
    if (!kPipe) MLK_STAGE_LOAD(c0)
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const int idx = tid + p * kThreads;
      if (idx < cn * R4) reinterpret_cast<piece_t*>(sW + idx / R4)[idx % R4] = piece[p];
    }
    if (tid < cn) {
      const double ge = amp0 * pg * scale;
      sAmp[tid][0] = (T)(ge * pm0);
      sAmp[tid][1] = (T)(ge * pm1);
      sAmp[tid][2] = (T)(ge * pm2);
      sRun[tid] = prun;
    }
    lds_barrier();
    if (kPipe && c0 + kGroups < q1) MLK_STAGE_LOAD(c0 + kGroups)
    if (grp >= cn) continue;
    const unsigned run = sRun[grp];
    const int nx = ((run >> 7) & 7) + 1;
    if (i >= nx) continue;
    const WinRec<T>& w = sW[grp];
    const int li = (run & 15) + i, dxi = ((run >> 4) & 7) + i;
    const int ly0 = (run >> 10) & 15, dy0 = (run >> 14) & 7, cj = ((run >> 17) & 7) + 1;
    const int lz0 = (run >> 20) & 15, dz0 = (run >> 24) & 7, ck = ((run >> 27) & 7) + 1;
    T wy0[kMaxWin], wy1[kMaxWin], wz0[kMaxWin], wz1[kMaxWin];
#pragma unroll
    for (int r = 0; r < kMaxWin; ++r) {
      // offsets past the run are clamped into the record and never used
      const int dy = min(dy0 + r, kMaxWin - 1), dz = min(dz0 + r, kMaxWin - 1);
      wy0[r] = w.wr[1][0][dy];
      wy1[r] = w.wr[1][1][dy];
      wz0[r] = w.wr[2][0][dz];
      wz1[r] = w.wr[2][1][dz];
    }
    const T cx = sAmp[grp][0] * w.wr[0][1][dxi];
    const T cy = sAmp[grp][1] * w.wr[0][0][dxi];
    const T cz = sAmp[grp][2] * w.wr[0][0][dxi];
    const int base = BX * (ly0 + BY * lz0) + li;
#pragma unroll
    for (int k = 0; k < kMaxWin; ++k) {
      if (k >= ck) break;
      const T cxk = cx * wz0[k], cyk = cy * wz0[k], czk = cz * wz1[k];
      const int pk = base + BX * BY * k;
#pragma unroll
      for (int j = 0; j < kMaxWin; ++j) {
        if (j >= cj) break;
        const int s = pk + BX * j;
        if constexpr (kPackXY) {
          // Ex and Ey in one 64-bit integer, Ey 2^32 + Ex (both sums stay below 2^30)
          const long long pxy = (long long)A::round(cyk * wy1[j]) * 4294967296LL +
                                (long long)A::round(cxk * wy0[j]);
          atomicAdd(sJxy + s, (unsigned long long)pxy);
        } else {
          atomicAdd(&sJ[0][s], (typename A::U)A::round(cxk * wy0[j]));
          atomicAdd(&sJ[1][s], (typename A::U)A::round(cyk * wy1[j]));
        }
        atomicAdd(&sJ[2][s], (typename A::U)A::round(czk * wy0[j]));
      }
    }
  }
#undef MLK_STAGE_LOAD
  __syncthreads();
  // owner write: E -= [eps^-1] J on the cells of this bin; the loads of a thread's
  // cells are issued together (unconditional, from a safe index: cell 0 for a
  // cell that no window reaches, so only touched cells cost HBM reads), then the
  // stores
  static_assert(CELLS % kThreads == 0, "the bin is a whole number of workgroup passes");
  constexpr int RW = CELLS / kThreads;
  typename A::S jv[RW][3];
  size_t idw[RW];
  T ev[RW][3], eiv[RW];
#pragma unroll
  for (int r = 0; r < RW; ++r) {
    const int t = tid + r * kThreads;
    const int li = t % BX, lj = (t / BX) % BY, lk = t / (BX * BY);
    const bool in = li < ex && lj < ey && lk < ez;
#pragma unroll
    for (int c = 0; c < 3; ++c) jv[r][c] = in ? (typename A::S)sJ[c][t] : 0;
    if constexpr (kPackXY) {
      // the packed sum is Ey 2^32 + Ex exactly; |Ex| < 2^31, so Ex is its low 32 bits
      // read as a signed value, and Ey what remains
      const long long pxy = in ? (long long)sJxy[t] : 0LL;
      const int lx = (int)(unsigned)(unsigned long long)pxy;
      jv[r][0] = lx;
      jv[r][1] = (typename A::S)((pxy - (long long)lx) / 4294967296LL);
    }
    const bool hit = in && (jv[r][0] | jv[r][1] | jv[r][2]) != 0;
    idw[r] = hit ? cell_index(g, x0 + li, y0 + lj, z0 + lk) : 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) ev[r][c] = f.E[c][idw[r]];
    eiv[r] = (EPS && f.epsinv) ? f.epsinv[idw[r]] : T(1);  // null: eps_r = 1 everywhere
  }
#pragma unroll
  for (int r = 0; r < RW; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      if (jv[r][c] != 0) f.E[c][idw[r]] = ev[r][c] - eiv[r] * (T)((double)jv[r][c] * inv_scale);
}

template <typename T>
__global__ __launch_bounds__(kThreads, 4) void k_scatter_bins(FieldPtrs<T> f, Geom g, BinPtrs bins,
                                                           WindowPtrs<T> win,
                                                           const double* mudot) {
  scatter_body(f, g, bins, win, mudot, g.dt * g.inv_dx * g.inv_dx * g.inv_dx, blockIdx.x);
}

// The scatter with the flux partials of the plane in fp.nblocks more workgroups.
template <typename T>
__global__ __launch_bounds__(kThreads, 4) void k_scatter_flux(FieldPtrs<T> f, Geom g, BinPtrs bins,
                                                           WindowPtrs<T> win,
                                                           const double* mudot, FluxPlane fp) {
  scatter_body(f, g, bins, win, mudot, g.dt * g.inv_dx * g.inv_dx * g.inv_dx, blockIdx.x, &fp);
}

template <typename T>
__global__ __launch_bounds__(kThreads, 4) void k_scatter_batch(const ScatterJob<T>* jobs,
                                                            const int* start, int njobs,
                                                            const int2* order) {
  int j, bid;
  if (order) {  // (job, bin) of the block, heaviest first across the jobs
    const int2 o = order[blockIdx.x];
    j = o.x;
    bid = o.y;
  } else {
    j = find_job(start, njobs, blockIdx.x);
    bid = blockIdx.x - start[j];
    if (bid >= jobs[j].nblocks) return;
  }
  const ScatterJob<T> J = load_job(jobs, j);
  scatter_body(J.f, J.g, J.bins, J.win, J.mudot, J.g.dt * J.g.inv_dx * J.g.inv_dx * J.g.inv_dx,
               bid);
}

template <typename T>
static hipError_t launch_gather_step(const FieldPtrs<T>& f, const Geom& g, const BinPtrs& b,
                                     const WindowPtrs<T>& win, const TlsPtrs& tls,
                                     double* Et, double* mudot, const int64_t* pop_off,
                                     const Series& ser, const int64_t* step,
                                     const FluxPlane* fp, hipStream_t st) {
  if (b.ngather <= 0) return fp ? hipErrorInvalidValue : hipSuccess;
  int nflux = 0;
  FluxPlane fpv{};
  if (fp) {
    const int a = fp->axis, u = (a + 1) % 3, v = (a + 2) % 3;
    nflux = (g.n[u] * g.n[v] + GatherCfg<T>::threads - 1) / GatherCfg<T>::threads;
    fpv = *fp;
  }
  if (b.gdense + nflux > 0)
    hipLaunchKernelGGL(k_gather_bins<T>, dim3(b.gdense + nflux), dim3(GatherCfg<T>::threads), 0,
                       st, f, g, b, win, Et, fpv);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && b.nlight > 0) {
    constexpr int NG = kLightThreads / 64;  // a wavefront per emitter
    hipLaunchKernelGGL(k_gather_light<T>, dim3((b.nlight + NG - 1) / NG), dim3(kLightThreads),
                       0, st, f, g, b.gbin_em + b.glight0, b.nlight, win, Et);
    e = hipGetLastError();
  }
  if (e != hipSuccess || tls.count == 0) return e;
  hipLaunchKernelGGL(k_tls_step, dim3((tls.count + 255) / 256), dim3(256), 0, st, tls, g.dt, Et,
                     mudot, pop_off, ser, step);
  return hipGetLastError();
}

// Two-level step of every two-level emitter under a given E~ (emitter-id order).
hipError_t cavity_tls_step(const TlsPtrs& tls, double dt, const CavityDev& c, double* Et,
                           double* mudot, const int64_t* pop_off, const Series& ser,
                           const int64_t* step, hipStream_t st) {
  if (tls.count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cavity_tls, dim3(cavity_tls_blocks(tls.count)), dim3(kTlsThreads), 0, st,
                     tls, dt, c, Et, mudot, pop_off, ser, step);
  return hipGetLastError();
}

hipError_t tls_step(const TlsPtrs& tls, double dt, const double* Et, double* mudot,
                    const int64_t* pop_off, const Series& ser, const int64_t* step,
                    hipStream_t st) {
  if (tls.count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tls_step, dim3((tls.count + 255) / 256), dim3(256), 0, st, tls, dt, Et,
                     mudot, pop_off, ser, step);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_scatter(const FieldPtrs<T>& f, const Geom& g, const BinPtrs& b,
                                 const WindowPtrs<T>& win, const double* mudot,
                                 const FluxPlane* fp, hipStream_t st) {
  if (b.nscatter <= 0) return hipSuccess;
  if (fp && fp->on && fp->nblocks > 0)
    hipLaunchKernelGGL(k_scatter_flux<T>, dim3(b.nscatter + fp->nblocks), dim3(kThreads), 0, st,
                       f, g, b, win, mudot, *fp);
  else
    hipLaunchKernelGGL(k_scatter_bins<T>, dim3(b.nscatter), dim3(kThreads), 0, st, f, g, b, win,
                       mudot);
  return hipGetLastError();
}

hipError_t bin_gather_step_f64(const FieldPtrs<double>& f, const Geom& g, const BinPtrs& b,
                               const WindowPtrs<double>& win, const TlsPtrs& tls, double* Et,
                               double* mudot, const int64_t* pop_off, const Series& ser,
                               const int64_t* step, const FluxPlane* fp, hipStream_t st) {
  return launch_gather_step<double>(f, g, b, win, tls, Et, mudot, pop_off, ser, step, fp, st);
}
hipError_t bin_gather_step_f32(const FieldPtrs<float>& f, const Geom& g, const BinPtrs& b,
                               const WindowPtrs<float>& win, const TlsPtrs& tls, double* Et,
                               double* mudot, const int64_t* pop_off, const Series& ser,
                               const int64_t* step, const FluxPlane* fp, hipStream_t st) {
  return launch_gather_step<float>(f, g, b, win, tls, Et, mudot, pop_off, ser, step, fp, st);
}
hipError_t bin_scatter_f64(const FieldPtrs<double>& f, const Geom& g, const BinPtrs& b,
                           const WindowPtrs<double>& win, const double* mudot,
                           const FluxPlane* fp, hipStream_t st) {
  return launch_scatter<double>(f, g, b, win, mudot, fp, st);
}
hipError_t bin_scatter_f32(const FieldPtrs<float>& f, const Geom& g, const BinPtrs& b,
                           const WindowPtrs<float>& win, const double* mudot,
                           const FluxPlane* fp, hipStream_t st) {
  return launch_scatter<float>(f, g, b, win, mudot, fp, st);
}

template <typename T>
static hipError_t launch_gather_batch(const GatherJob<T>* jobs, const int* start, int njobs,
                                      const int2* order, int nblocks, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_batch<T>, dim3(nblocks), dim3(GatherCfg<T>::threads), 0, st, jobs,
                     start, njobs, order);
  return hipGetLastError();
}
template <typename T>
static hipError_t launch_scatter_batch(const ScatterJob<T>* jobs, const int* start, int njobs,
                                       const int2* order, int nblocks, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_batch<T>, dim3(nblocks), dim3(kThreads), 0, st, jobs, start, njobs,
                     order);
  return hipGetLastError();
}

hipError_t gather_batch_f64(const GatherJob<double>* jobs, const int* start, int njobs,
                            const int2* order, int nblocks, hipStream_t st) {
  return launch_gather_batch<double>(jobs, start, njobs, order, nblocks, st);
}
hipError_t gather_batch_f32(const GatherJob<float>* jobs, const int* start, int njobs,
                            const int2* order, int nblocks, hipStream_t st) {
  return launch_gather_batch<float>(jobs, start, njobs, order, nblocks, st);
}
template <typename T>
static hipError_t launch_light_batch(const LightJob<T>* jobs, const int* start, int njobs,
                                     int nblocks, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_light_batch<T>, dim3(nblocks), dim3(kLightThreads), 0, st, jobs,
                     start, njobs);
  return hipGetLastError();
}
hipError_t light_batch_f64(const LightJob<double>* jobs, const int* start, int njobs,
                           int nblocks, hipStream_t st) {
  return launch_light_batch<double>(jobs, start, njobs, nblocks, st);
}
hipError_t light_batch_f32(const LightJob<float>* jobs, const int* start, int njobs, int nblocks,
                           hipStream_t st) {
  return launch_light_batch<float>(jobs, start, njobs, nblocks, st);
}
int light_per_block(bool) {
  return kLightThreads / 64;  // a wavefront per emitter
}
hipError_t scatter_batch_f64(const ScatterJob<double>* jobs, const int* start, int njobs,
                             const int2* order, int nblocks, hipStream_t st) {
  return launch_scatter_batch<double>(jobs, start, njobs, order, nblocks, st);
}
hipError_t scatter_batch_f32(const ScatterJob<float>* jobs, const int* start, int njobs,
                             const int2* order, int nblocks, hipStream_t st) {
  return launch_scatter_batch<float>(jobs, start, njobs, order, nblocks, st);
}
hipError_t tls_batch(const TlsJob* jobs, const int* start, int njobs, int nblocks,
                     hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tls_batch, dim3(nblocks), dim3(256), 0, st, jobs, start, njobs);
  return hipGetLastError();
}

// ---- adjoint-step variants
template <typename T>
__global__ __launch_bounds__(GatherCfg<T>::threads, GatherCfg<T>::waves_per_simd) void k_gather_epsw(FieldPtrs<T> f, Geom g, BinPtrs bins,
                                                          WindowPtrs<T> win, double* out) {
  gather_body<T, true>(f, g, bins, win, out, blockIdx.x);
}
template <typename T>
__global__ __launch_bounds__(kThreads, 4) void k_scatter_plain(FieldPtrs<T> f, Geom g, BinPtrs bins,
                                                            WindowPtrs<T> win, const double* amp,
                                                            double amp0) {
  scatter_body<T, false>(f, g, bins, win, amp, amp0, blockIdx.x);
}
template <typename T>
static hipError_t launch_gather_epsw(const FieldPtrs<T>& f, const Geom& g, const BinPtrs& b,
                                     const WindowPtrs<T>& win, double* out, hipStream_t st) {
  if (b.ngather <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_epsw<T>, dim3(b.ngather), dim3(GatherCfg<T>::threads), 0, st, f, g, b, win, out);
  return hipGetLastError();
}
template <typename T>
static hipError_t launch_scatter_plain(const FieldPtrs<T>& f, const Geom& g, const BinPtrs& b,
                                       const WindowPtrs<T>& win, const double* amp, double amp0,
                                       hipStream_t st) {
  if (b.nscatter <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_plain<T>, dim3(b.nscatter), dim3(kThreads), 0, st, f, g, b, win,
                     amp, amp0);
  return hipGetLastError();
}
hipError_t gather_epsw_f64(const FieldPtrs<double>& f, const Geom& g, const BinPtrs& b,
                           const WindowPtrs<double>& win, double* out, hipStream_t st) {
  return launch_gather_epsw<double>(f, g, b, win, out, st);
}
hipError_t gather_epsw_f32(const FieldPtrs<float>& f, const Geom& g, const BinPtrs& b,
                           const WindowPtrs<float>& win, double* out, hipStream_t st) {
  return launch_gather_epsw<float>(f, g, b, win, out, st);
}
hipError_t scatter_plain_f64(const FieldPtrs<double>& f, const Geom& g, const BinPtrs& b,
                             const WindowPtrs<double>& win, const double* amp, double amp0,
                             hipStream_t st) {
  return launch_scatter_plain<double>(f, g, b, win, amp, amp0, st);
}
hipError_t scatter_plain_f32(const FieldPtrs<float>& f, const Geom& g, const BinPtrs& b,
                             const WindowPtrs<float>& win, const double* amp, double amp0,
                             hipStream_t st) {
  return launch_scatter_plain<float>(f, g, b, win, amp, amp0, st);
}

}  // namespace mlk
