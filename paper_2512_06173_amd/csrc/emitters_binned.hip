// Tile-binned emitter phase.
//
// gather + step (eq. E_regu_Emi, then eq. von-Neumann-tls and eq.
// dipole_derivative): the emitters are grouped by the bin of their centre
// cell.  The workgroup of a bin stages E over the bin plus a halo of kHalo
// cells in LDS, which holds every window of its emitters; one wavefront then
// takes one emitter at a time, 64 lanes over the (x, y) points of its window
// and a loop over z, all three components per pass, sums in FP64, and lane 0
// advances the two-level state and writes E~ and mu_dot.
//
// scatter (eqs. J_mol, Polarization_mol):  E_c(p) -= (dt/eps_r(p)) gamma mu_dot^c
// w^c_{m,p} / dx^3.  A workgroup owns a bin of cells and takes every emitter
// whose window touches the bin; contributions are summed in LDS (as 64-bit
// fixed-point integers, see k_scatter_bins) and each cell is written once by
// its owner (no global atomics).
//
// Window weights are the separable factors wx wy wz set up by k_windows, kept
// per emitter as a union-window record (WinRec); a component uses the
// half-integer variant on its own axis.  Records of a chunk of emitters are
// copied into LDS with 16-byte loads, so the inner loops touch LDS only.
#include "mlk_internal.h"
#include "tls_math.h"

namespace mlk {

template <typename T>
struct BinCfg;
template <>
struct BinCfg<float> {
  // gather: 16 x 8 x 8 bins, 24 x 16 x 16 tile (74 KB); scatter: 32 x 8 x 8 bins
  static constexpr int GX = 16, GY = 8, GZ = 8, GCHUNK = 16;
  static constexpr int SX = 32, SY = 8, SZ = 8, SCHUNK = 32;
};
template <>
struct BinCfg<double> {
  // gather: 8 x 8 x 8 bins, 16 x 16 x 16 tile (98 KB); scatter: 32 x 8 x 8 bins
  static constexpr int GX = 8, GY = 8, GZ = 8, GCHUNK = 16;
  static constexpr int SX = 32, SY = 8, SZ = 8, SCHUNK = 16;
};

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

__device__ __forceinline__ int wrap_once(int q, int n) {
  q += q < 0 ? n : 0;
  q -= q >= n ? n : 0;
  return q;
}

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Copy the window records of emitters ids[0..cn) into LDS (16-byte pieces).
template <typename T, int NT>
__device__ __forceinline__ void stage_records(const WinRec<T>* rec, const int* ids, int cn,
                                              WinRec<T>* dst, int tid) {
  constexpr int R4 = sizeof(WinRec<T>) / sizeof(int4);
  for (int i = tid; i < cn * R4; i += NT) {
    const int slot = i / R4, part = i % R4;
    const int4* src = reinterpret_cast<const int4*>(rec + ids[slot]);
    reinterpret_cast<int4*>(dst + slot)[part] = src[part];
  }
}

}  // namespace

// gather + two-level step; see the file comment.
template <typename T>
__global__ __launch_bounds__(512) void k_gather_step(FieldPtrs<T> f, Geom g, BinPtrs bins,
                                                     WindowPtrs<T> win, TlsPtrs tls,
                                                     const int* tls_slot, double* Et,
                                                     double* mudot, const int64_t* pop_off,
                                                     Series ser, const int64_t* step) {
  constexpr int BX = BinCfg<T>::GX, BY = BinCfg<T>::GY, BZ = BinCfg<T>::GZ;
  constexpr int CH = BinCfg<T>::GCHUNK;
  constexpr int TX = BX + 2 * kHalo, TY = BY + 2 * kHalo, TZ = BZ + 2 * kHalo;
  constexpr int NW = 8, NT = 512;
  __shared__ T sE[3][TX * TY * TZ];
  __shared__ WinRec<T> sW[CH];
  __shared__ double sEt[CH][3];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // tile origin in the unwrapped frame of the emitters' window indices
  const int x0 = bins.gbin_org[3 * blockIdx.x] - kHalo;
  const int y0 = bins.gbin_org[3 * blockIdx.x + 1] - kHalo;
  const int z0 = bins.gbin_org[3 * blockIdx.x + 2] - kHalo;

  for (int t = tid; t < TX * TY * TZ; t += NT) {
    const int li = t % TX, lj = (t / TX) % TY, lk = t / (TX * TY);
    int q[3] = {x0 + li, y0 + lj, z0 + lk};
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (g.periodic[a]) {
        const int r = q[a] % g.n[a];
        q[a] = r < 0 ? r + g.n[a] : r;
      } else {
        ok = ok && q[a] >= 0 && q[a] < g.n[a];
      }
    }
    T v0 = T(0), v1 = T(0), v2 = T(0);
    if (ok) {
      const size_t id = cell_index(g, q[0], q[1], q[2]);
      v0 = f.E[0][id];
      v1 = f.E[1][id];
      v2 = f.E[2][id];
    }
    sE[0][t] = v0;
    sE[1][t] = v1;
    sE[2][t] = v2;
  }

  const int ix = lane & 7, iy = lane >> 3;
  const int q0 = bins.gbin_start[blockIdx.x], q1 = bins.gbin_start[blockIdx.x + 1];
  for (int c0 = q0; c0 < q1; c0 += CH) {
    const int cn = min(CH, q1 - c0);
    stage_records<T, NT>(win.rec, bins.gbin_em + c0, cn, sW, tid);
    __syncthreads();
    for (int k = wave; k < cn; k += NW) {
      const WinRec<T>& w = sW[k];
      double ax = 0.0, ay = 0.0, az = 0.0;
      if (ix < w.n[0] && iy < w.n[1]) {
        const T wx0 = w.wr[0][0][ix], wx1 = w.wr[0][1][ix];
        const T wy0 = w.wr[1][0][iy], wy1 = w.wr[1][1][iy];
        const T cx = wx1 * wy0, cy = wx0 * wy1, cz = wx0 * wy0;
        // unwrapped window coordinates lie inside the tile by construction
        int s = (w.org[0] + ix - x0) + TX * (w.org[1] + iy - y0) + TX * TY * (w.org[2] - z0);
        const int nz = w.n[2];
        for (int d = 0; d < nz; ++d, s += TX * TY) {
          const T wz0 = w.wr[2][0][d], wz1 = w.wr[2][1][d];
          ax += (double)(cx * wz0) * (double)sE[0][s];
          ay += (double)(cy * wz0) * (double)sE[1][s];
          az += (double)(cz * wz1) * (double)sE[2][s];
        }
      }
      ax = wave_sum64(ax);
      ay = wave_sum64(ay);
      az = wave_sum64(az);
      if (lane == 0) {
        sEt[k][0] = ax;
        sEt[k][1] = ay;
        sEt[k][2] = az;
      }
    }
    __syncthreads();
    // one thread per emitter: E~, the exact two-level step, mu_dot, population
    if (tid < cn) {
      const int e = bins.gbin_em[c0 + tid];
      const double gm = win.gamma[e];
      const double et[3] = {gm * sEt[tid][0], gm * sEt[tid][1], gm * sEt[tid][2]};
      Et[3 * e] = et[0];
      Et[3 * e + 1] = et[1];
      Et[3 * e + 2] = et[2];
      const int m = tls_slot[e];
      if (m >= 0) {
        const double d[3] = {tls.dip[3 * m], tls.dip[3 * m + 1], tls.dip[3 * m + 2]};
        double st[3] = {tls.rho[3 * m], tls.rho[3 * m + 1], tls.rho[3 * m + 2]};
        double md[3];
        tls_advance(tls.omega0[m], d, et, g.dt, st, md);
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
    }
    __syncthreads();
  }
}

// Fixed-point accumulator of the scatter: 32-bit for FP32 fields, 64-bit for FP64.
template <typename T>
struct Acc;
template <>
struct Acc<float> {
  using U = unsigned int;
  using S = int;
  static constexpr int BITS = 30;
  __device__ static S round(double v) { return __float2int_rn((float)v); }
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
// and order-independent, so the result is deterministic.  The grid is
// 2^-BITS of a bound on any cell's sum (|amp| times the largest window weight,
// summed over the bin's emitters): 2^-62 for FP64 fields, far below FP64
// rounding; 2^-30 for FP32 fields, at the level of FP32 rounding of a cell's
// sum.
template <typename T>
__global__ __launch_bounds__(512) void k_scatter_bins(FieldPtrs<T> f, Geom g, BinPtrs bins,
                                                      WindowPtrs<T> win, const double* mudot) {
  using A = Acc<T>;
  constexpr int BX = BinCfg<T>::SX, BY = BinCfg<T>::SY, BZ = BinCfg<T>::SZ;
  constexpr int CH = BinCfg<T>::SCHUNK;
  constexpr int PX = BX + 8, PLANE = PX * BY, CELLS = PLANE * BZ;
  constexpr int NW = 8, NT = 512;
  __shared__ typename A::U sJ[3][CELLS];
  __shared__ WinRec<T> sW[CH];
  __shared__ double sAmp[CH][3];
  __shared__ double sRed[NW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int b = bins.sbin_id[blockIdx.x];
  const int bx = b % bins.nbx, by = (b / bins.nbx) % bins.nby, bz = b / (bins.nbx * bins.nby);
  const int x0 = bx * BX, y0 = by * BY, z0 = bz * BZ;
  const int ex = min(BX, g.n[0] - x0), ey = min(BY, g.n[1] - y0), ez = min(BZ, g.n[2] - z0);
  const int q0 = bins.sbin_start[blockIdx.x], q1 = bins.sbin_start[blockIdx.x + 1];
  const double amp0 = g.dt * g.inv_dx * g.inv_dx * g.inv_dx;
  for (int t = tid; t < CELLS; t += NT) {
    sJ[0][t] = 0;
    sJ[1][t] = 0;
    sJ[2][t] = 0;
  }
  double bound = 0.0;
  for (int q = q0 + tid; q < q1; q += NT) {
    const int e = bins.sbin_em[q];
    const double ge = fabs(amp0 * win.gamma[e]) * (double)win.rec[e].wmax;
    bound += ge * (fabs(mudot[3 * e]) + fabs(mudot[3 * e + 1]) + fabs(mudot[3 * e + 2]));
  }
  bound = wave_sum64(bound);
  if (lane == 0) sRed[wave] = bound;
  __syncthreads();
  bound = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) bound += sRed[w];
  if (!(bound > 0.0)) return;  // nothing to add in this bin (uniform across the block)
  // scale = 2^(BITS - e) with bound < 2^e: every partial sum stays below 2^BITS
  const int ebits = ilogb(bound) + 1;
  const double scale = ldexp(1.0, A::BITS - ebits);
  const double inv_scale = ldexp(1.0, ebits - A::BITS);

  const int ix = lane & 7, iy = lane >> 3;
  for (int c0 = q0; c0 < q1; c0 += CH) {
    const int cn = min(CH, q1 - c0);
    stage_records<T, NT>(win.rec, bins.sbin_em + c0, cn, sW, tid);
    if (tid < cn) {
      const int e = bins.sbin_em[c0 + tid];
      const double ge = amp0 * win.gamma[e] * scale;
      sAmp[tid][0] = ge * mudot[3 * e];
      sAmp[tid][1] = ge * mudot[3 * e + 1];
      sAmp[tid][2] = ge * mudot[3 * e + 2];
    }
    __syncthreads();
    for (int k = wave; k < cn; k += NW) {
      const WinRec<T>& w = sW[k];
      // z points of the window inside this bin: window offsets d in [d0, d1).  A
      // periodic axis held by a single bin may see a window from both ends; then
      // every offset is wrapped on its own.
      const int nz = w.n[2];
      const bool whole = g.periodic[2] && ez == g.n[2];
      int zs = w.org[2] - z0;
      if (g.periodic[2] && !whole) {
        if (zs + nz <= 0) zs += g.n[2];
        else if (zs >= ez) zs -= g.n[2];
      }
      const int d0 = whole ? 0 : max(0, -zs), d1 = whole ? nz : min(nz, ez - zs);
      if (d0 >= d1) continue;  // uniform across the wave
      if (ix >= w.n[0] || iy >= w.n[1]) continue;
      const int li = wrap_once(w.org[0] + ix, g.n[0]) - x0;
      const int lj = wrap_once(w.org[1] + iy, g.n[1]) - y0;
      if (li < 0 || li >= ex || lj < 0 || lj >= ey) continue;
      const double wx0 = (double)w.wr[0][0][ix], wx1 = (double)w.wr[0][1][ix];
      const double wy0 = (double)w.wr[1][0][iy], wy1 = (double)w.wr[1][1][iy];
      const double cx = sAmp[k][0] * wx1 * wy0, cy = sAmp[k][1] * wx0 * wy1,
                   cz = sAmp[k][2] * wx0 * wy0;
      const int base = li + PX * lj;
      for (int d = d0; d < d1; ++d) {
        const int lk = whole ? wrap_once(w.org[2] + d, g.n[2]) : zs + d;
        const int s = base + PLANE * lk;
        const typename A::S vx = A::round(cx * (double)w.wr[2][0][d]);
        const typename A::S vy = A::round(cy * (double)w.wr[2][0][d]);
        const typename A::S vz = A::round(cz * (double)w.wr[2][1][d]);
        if (vx != 0) atomicAdd(&sJ[0][s], (typename A::U)vx);
        if (vy != 0) atomicAdd(&sJ[1][s], (typename A::U)vy);
        if (vz != 0) atomicAdd(&sJ[2][s], (typename A::U)vz);
      }
    }
    __syncthreads();
  }
  // owner write: E -= (dt/eps) J on the touched cells of this bin
  for (int t = tid; t < BX * BY * BZ; t += NT) {
    const int li = t % BX, lj = (t / BX) % BY, lk = t / (BX * BY);
    if (li >= ex || lj >= ey || lk >= ez) continue;
    const int s = li + PX * lj + PLANE * lk;
    const typename A::S j0 = (typename A::S)sJ[0][s], j1 = (typename A::S)sJ[1][s],
                        j2 = (typename A::S)sJ[2][s];
    if (j0 == 0 && j1 == 0 && j2 == 0) continue;
    const size_t id = cell_index(g, x0 + li, y0 + lj, z0 + lk);
    const T ei = f.epsinv[id];
    if (j0 != 0) f.E[0][id] -= ei * (T)((double)j0 * inv_scale);
    if (j1 != 0) f.E[1][id] -= ei * (T)((double)j1 * inv_scale);
    if (j2 != 0) f.E[2][id] -= ei * (T)((double)j2 * inv_scale);
  }
}

template <typename T>
static hipError_t launch_gather_step(const FieldPtrs<T>& f, const Geom& g, const BinPtrs& b,
                                     const WindowPtrs<T>& win, const TlsPtrs& tls,
                                     const int* tls_slot, double* Et, double* mudot,
                                     const int64_t* pop_off, const Series& ser,
                                     const int64_t* step, hipStream_t st) {
  if (b.ngather <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_step<T>, dim3(b.ngather), dim3(512), 0, st, f, g, b, win, tls,
                     tls_slot, Et, mudot, pop_off, ser, step);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_scatter(const FieldPtrs<T>& f, const Geom& g, const BinPtrs& b,
                                 const WindowPtrs<T>& win, const double* mudot, hipStream_t st) {
  if (b.nscatter <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_bins<T>, dim3(b.nscatter), dim3(512), 0, st, f, g, b, win, mudot);
  return hipGetLastError();
}

hipError_t bin_gather_step_f64(const FieldPtrs<double>& f, const Geom& g, const BinPtrs& b,
                               const WindowPtrs<double>& win, const TlsPtrs& tls,
                               const int* tls_slot, double* Et, double* mudot,
                               const int64_t* pop_off, const Series& ser, const int64_t* step,
                               hipStream_t st) {
  return launch_gather_step<double>(f, g, b, win, tls, tls_slot, Et, mudot, pop_off, ser, step,
                                    st);
}
hipError_t bin_gather_step_f32(const FieldPtrs<float>& f, const Geom& g, const BinPtrs& b,
                               const WindowPtrs<float>& win, const TlsPtrs& tls,
                               const int* tls_slot, double* Et, double* mudot,
                               const int64_t* pop_off, const Series& ser, const int64_t* step,
                               hipStream_t st) {
  return launch_gather_step<float>(f, g, b, win, tls, tls_slot, Et, mudot, pop_off, ser, step,
                                   st);
}
hipError_t bin_scatter_f64(const FieldPtrs<double>& f, const Geom& g, const BinPtrs& b,
                           const WindowPtrs<double>& win, const double* mudot, hipStream_t st) {
  return launch_scatter<double>(f, g, b, win, mudot, st);
}
hipError_t bin_scatter_f32(const FieldPtrs<float>& f, const Geom& g, const BinPtrs& b,
                           const WindowPtrs<float>& win, const double* mudot, hipStream_t st) {
  return launch_scatter<float>(f, g, b, win, mudot, st);
}

}  // namespace mlk
