// Emitter set-up and the atomic scatter variant.
//
// Windows (eq. Polarization_mol, eq. E_regu_Emi): for component c the weights are
// the Gaussian exp(-|p - r|^2 / 2 sigma^2) sampled at the Yee points of c inside a
// box of half-width R sigma and normalised to unit sum (the discrete unit-integral
// kernel).  The box and the Gaussian are separable, so each emitter stores three
// normalised 1-D weight vectors per component and a window weight is their
// product; k_records repacks them as the union-window records of the binned
// kernels.
//
// Atomic scatter (eqs. J_mol, Polarization_mol): E_c(p) -= (dt/eps_r) gamma mu_dot^c
// w / dx^3 with one wavefront per emitter and floating-point atomics: the sum
// order is not fixed, so results agree with the owner-computes scatter only to
// rounding.
#include <climits>

#include "mlk_internal.h"

namespace mlk {

__device__ __forceinline__ int wrap_index(int q, int n) {
  int r = q % n;
  return r < 0 ? r + n : r;
}


// One thread per (emitter, axis, position variant): window start, length and
// the normalised 1-D Gaussian weights along that axis.  The window holds the
// points q + v/2 with (q + v/2 - r)^2 <= (R sigma)^2; on an invariant axis
// (one periodic cell) it is that cell with weight 1.
template <typename T>
__global__ void k_windows(int count, const double* pos, const double* sigma, double R, Geom g,
                          int* lo, int* len, T* w) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count * 6) return;
  const int m = t / 6, a = (t / 2) % 3, v = t % 2;
  const int slot = win_slot(m, a, v);
  T* wv = w + (size_t)slot * kMaxWin;
  for (int q = 0; q < kMaxWin; ++q) wv[q] = T(0);
  if (g.n[a] == 1 && g.periodic[a]) {
    lo[slot] = 0;
    len[slot] = 1;
    wv[0] = T(1);
    return;
  }
  const double r = pos[3 * m + a];
  const double s = sigma[m];
  const double rs = R * s;
  const double sh = 0.5 * v;
  const int q0 = (int)floor(r - sh - rs) - 1;
  int firstq = INT_MAX, lastq = INT_MIN;
  for (int q = q0; q <= q0 + kMaxWin + 3; ++q) {
    const double o = (double)q + sh - r;
    if (o * o <= rs * rs) {
      if (firstq == INT_MAX) firstq = q;
      lastq = q;
    }
  }
  int L = lastq - firstq + 1;
  if (L > kMaxWin) L = kMaxWin;  // rejected on the host before launch
  double sum = 0.0;
  for (int q = 0; q < L; ++q) {
    const double o = (double)(firstq + q) + sh - r;
    sum += exp(-o * o / (2.0 * s * s));
  }
  for (int q = 0; q < L; ++q) {
    const double o = (double)(firstq + q) + sh - r;
    wv[q] = (T)(exp(-o * o / (2.0 * s * s)) / sum);
  }
  lo[slot] = firstq;
  len[slot] = L;
}

// One thread per (emitter, axis, variant): the union-window record of the
// binned kernels (see WinRec).
template <typename T>
__global__ void k_records(int count, const int* lo, const int* len, const T* w, WinRec<T>* rec) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count * 6) return;
  const int m = t / 6, a = (t / 2) % 3, v = t % 2;
  const int lo0 = lo[win_slot(m, a, 0)], n0 = len[win_slot(m, a, 0)];
  const int lo1 = lo[win_slot(m, a, 1)], n1 = len[win_slot(m, a, 1)];
  const int org = min(lo0, lo1);
  const int end = max(lo0 + n0, lo1 + n1);
  const int l = v ? lo1 : lo0, n = v ? n1 : n0;
  const T* wv = w + (size_t)win_slot(m, a, v) * kMaxWin;
  WinRec<T>& r = rec[m];
  for (int d = 0; d < kMaxWin; ++d) {
    const int k = org + d - l;
    r.wr[a][v][d] = (k >= 0 && k < n) ? wv[k] : T(0);
  }
  if (v == 0) {
    r.org[a] = org;
    r.n[a] = min(end - org, kMaxWin);
  }
  if (t % 6 == 0) {
    // largest product of 1-D factors over the three component windows
    double best = 0.0;
    for (int c = 0; c < 3; ++c) {
      double p = 1.0;
      for (int b = 0; b < 3; ++b) {
        const int sl = win_slot(m, b, b == c);
        double mx = 0.0;
        for (int d = 0; d < len[sl]; ++d) mx = fmax(mx, (double)w[(size_t)sl * kMaxWin + d]);
        p *= mx;
      }
      best = fmax(best, p);
    }
    r.wmax = (float)(best * (1.0 + 1e-6));
    r.pad = 0;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_scatter_atomic(FieldPtrs<T> f, Geom g, WindowPtrs<T> win,
                                                        int count, const double* mudot) {
  const int lane = threadIdx.x & 63;
  const int e = (int)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) >> 6);
  if (e >= count) return;
  const double vol = g.inv_dx * g.inv_dx * g.inv_dx;
  for (int c = 0; c < 3; ++c) {
    const double amp = g.dt * win.gamma[e] * mudot[3 * e + c] * vol;
    if (amp == 0.0) continue;
    const int sx = win_slot(e, 0, c == 0), sy = win_slot(e, 1, c == 1), sz = win_slot(e, 2, c == 2);
    const int lx = win.lo[sx], ly = win.lo[sy], lz = win.lo[sz];
    const int Lx = win.len[sx], Ly = win.len[sy], Lz = win.len[sz];
    const T* wx = win.w + (size_t)sx * kMaxWin;
    const T* wy = win.w + (size_t)sy * kMaxWin;
    const T* wz = win.w + (size_t)sz * kMaxWin;
    T* Ec = f.E[c];
    for (int q = lane; q < Ly * Lz; q += 64) {
      const int dy = q % Ly, dz = q / Ly;
      const int jj = wrap_index(ly + dy, g.n[1]);
      const int kk = wrap_index(lz + dz, g.n[2]);
      const size_t row = (size_t)g.n[0] * ((size_t)jj + (size_t)g.n[1] * (size_t)kk);
      const double a = amp * (double)wy[dy] * (double)wz[dz];
      for (int dx = 0; dx < Lx; ++dx) {
        const size_t id = row + wrap_index(lx + dx, g.n[0]);
        const T inc = (T)(a * (double)wx[dx] * (double)f.epsinv[id]);
        unsafeAtomicAdd(&Ec[id], -inc);
      }
    }
  }
}

template <typename T>
static hipError_t launch_windows(int count, const double* pos, const double* sigma, double R,
                                 const Geom& g, int* lo, int* len, T* w, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int threads = 256;
  const int blocks = (count * 6 + threads - 1) / threads;
  hipLaunchKernelGGL(k_windows<T>, dim3(blocks), dim3(threads), 0, st, count, pos, sigma, R, g,
                     lo, len, w);
  return hipGetLastError();
}

hipError_t windows_f64(int count, const double* pos, const double* sigma, double R, const Geom& g,
                       int* lo, int* len, double* w, hipStream_t st) {
  return launch_windows<double>(count, pos, sigma, R, g, lo, len, w, st);
}

template <typename T>
static hipError_t launch_records(int count, const int* lo, const int* len, const T* w,
                                 WinRec<T>* rec, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_records<T>, dim3((count * 6 + 255) / 256), dim3(256), 0, st, count, lo, len,
                     w, rec);
  return hipGetLastError();
}
hipError_t records_f64(int count, const int* lo, const int* len, const double* w,
                       WinRec<double>* rec, hipStream_t st) {
  return launch_records<double>(count, lo, len, w, rec, st);
}
hipError_t records_f32(int count, const int* lo, const int* len, const float* w,
                       WinRec<float>* rec, hipStream_t st) {
  return launch_records<float>(count, lo, len, w, rec, st);
}
hipError_t windows_f32(int count, const double* pos, const double* sigma, double R, const Geom& g,
                       int* lo, int* len, float* w, hipStream_t st) {
  return launch_windows<float>(count, pos, sigma, R, g, lo, len, w, st);
}

template <typename T>
static hipError_t launch_scatter_atomic(const FieldPtrs<T>& f, const Geom& g,
                                        const WindowPtrs<T>& win, int count, const double* mudot,
                                        hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int waves_per_block = 4;
  const int blocks = (count + waves_per_block - 1) / waves_per_block;
  hipLaunchKernelGGL(k_scatter_atomic<T>, dim3(blocks), dim3(64 * waves_per_block), 0, st, f, g,
                     win, count, mudot);
  return hipGetLastError();
}

hipError_t scatter_atomic_f64(const FieldPtrs<double>& f, const Geom& g,
                              const WindowPtrs<double>& win, int count, const double* mudot,
                              hipStream_t st) {
  return launch_scatter_atomic<double>(f, g, win, count, mudot, st);
}
hipError_t scatter_atomic_f32(const FieldPtrs<float>& f, const Geom& g,
                              const WindowPtrs<float>& win, int count, const double* mudot,
                              hipStream_t st) {
  return launch_scatter_atomic<float>(f, g, win, count, mudot, st);
}

// Classical-path field of a travelling pulse (eq. E_analytical, +z at c = 1): the
// emitter at height z sees gamma amp f(t - (z - z0)) pol over the step centred at
// t, with the Gaussian pulse of App. B, f(u) = cos(omega (u - t0)) exp(-(u - t0)^2 /
// (2 tau^2)).  One thread per emitter (id order).
__global__ void k_wave_field(int M, const double* pos, const double* gamma, WaveDesc w, double t,
                             double* Et) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M) return;
  const double u = t - (pos[3 * (size_t)e + 2] - w.z0) - w.t0;
  const double f = gamma[e] * w.amp * cos(w.omega * u) * exp(-u * u / (2.0 * w.tau * w.tau));
  Et[3 * (size_t)e] = f * w.pol[0];
  Et[3 * (size_t)e + 1] = f * w.pol[1];
  Et[3 * (size_t)e + 2] = f * w.pol[2];
}

hipError_t wave_field(int M, const double* pos, const double* gamma, const WaveDesc& w, double t,
                      double* Et, hipStream_t st) {
  if (M <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_wave_field, dim3((M + 255) / 256), dim3(256), 0, st, M, pos, gamma, w, t,
                     Et);
  return hipGetLastError();
}

}  // namespace mlk
