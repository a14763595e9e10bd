// Dispersive media: Lorentz and Drude poles over cell boxes (the dielectric
// functions of eq. Dromega, chi(w) = sigma w0^2 / (kappa w0^2 - w^2 - i w gamma),
// kappa = 1 Lorentz, 0 Drude).  Each pole carries a polarisation P with
// P'' + gamma P' + kappa w0^2 P = sigma w0^2 E, advanced by central
// differences; D = eps_inf E + sum P advances by dt (curl H - J), so
//   E^{n+1} = E^n + (dt (curl H - J) - sum_k (P_k^{n+1} - P_k^n)) / eps_inf.
// The sweep, the scatter and the sources already add dt (curl H - J) / eps_inf;
// the two passes here supply the rest.  Each pole keeps P^n and the increment
// Q = P^n - P^{n-1} in place (two arrays, no host-side rotation):
//   pre  (E = E^n):   Q <- P^{n+1} - P^n,  P^{n+1} = (a P^n - b (P^n - Q) + c E^n) / (1 + g)
//   post (E = E^{n+1} without the poles):  E -= Q / eps_inf,  P += Q.
// One thread per box cell for all three components (one 1/eps_inf read and one
// index computation per cell), x fastest: coalesced along rows.
#include "launch.h"

namespace mlk {

namespace {

constexpr int kPoleThreads = 256;

__device__ __forceinline__ size_t pole_cell(const PoleDev& p, const Geom& g, size_t b) {
  const int i = (int)(b % p.n[0]);
  const size_t r = b / p.n[0];
  const int j = (int)(r % p.n[1]);
  const int k = (int)(r / p.n[1]);
  return (size_t)(p.lo[0] + i) + (size_t)g.n[0] * ((size_t)(p.lo[1] + j) +
                                                   (size_t)g.n[1] * (size_t)(p.lo[2] + k));
}

template <typename T>
__global__ __launch_bounds__(kPoleThreads) void k_pole_pre(PoleDev p, FieldPtrs<T> f, Geom g,
                                                           size_t nb) {
  const size_t b = (size_t)blockIdx.x * kPoleThreads + threadIdx.x;
  if (b >= nb) return;
  const size_t id = pole_cell(p, g, b);
  const T* P = (const T*)p.P;
  T* Q = (T*)p.Q;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const size_t t = (size_t)c * nb + b;
    const double e = (double)f.E[c][id];
    const double pn = (double)P[t], pm = pn - (double)Q[t];
    const double pnew = (p.a * pn - p.b * pm + p.c * e) / p.g1;
    Q[t] = (T)(pnew - pn);
  }
}

template <typename T>
__global__ __launch_bounds__(kPoleThreads) void k_pole_post(PoleDev p, FieldPtrs<T> f, Geom g,
                                                            const T* __restrict__ epsinv,
                                                            size_t nb) {
  const size_t b = (size_t)blockIdx.x * kPoleThreads + threadIdx.x;
  if (b >= nb) return;
  const size_t id = pole_cell(p, g, b);
  const T ei = epsinv[id];
  T* P = (T*)p.P;
  const T* Q = (const T*)p.Q;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const size_t t = (size_t)c * nb + b;
    const T q = Q[t];
    f.E[c][id] -= ei * q;
    P[t] += q;
  }
}

size_t pole_cells(const PoleDev& p) { return (size_t)p.n[0] * p.n[1] * p.n[2]; }

template <typename T>
hipError_t pole_pre(const PoleDev& p, const FieldPtrs<T>& f, const Geom& g, hipStream_t st) {
  const size_t nb = pole_cells(p);
  if (nb == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((nb + kPoleThreads - 1) / kPoleThreads);
  hipLaunchKernelGGL(k_pole_pre<T>, dim3(blocks), dim3(kPoleThreads), 0, st, p, f, g, nb);
  return hipGetLastError();
}

template <typename T>
hipError_t pole_post(const PoleDev& p, const FieldPtrs<T>& f, const Geom& g, const T* epsinv,
                     hipStream_t st) {
  const size_t nb = pole_cells(p);
  if (nb == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((nb + kPoleThreads - 1) / kPoleThreads);
  hipLaunchKernelGGL(k_pole_post<T>, dim3(blocks), dim3(kPoleThreads), 0, st, p, f, g, epsinv,
                     nb);
  return hipGetLastError();
}

}  // namespace

hipError_t pole_pre_f64(const PoleDev& p, const FieldPtrs<double>& f, const Geom& g, hipStream_t st) {
  return pole_pre<double>(p, f, g, st);
}
hipError_t pole_pre_f32(const PoleDev& p, const FieldPtrs<float>& f, const Geom& g, hipStream_t st) {
  return pole_pre<float>(p, f, g, st);
}
hipError_t pole_post_f64(const PoleDev& p, const FieldPtrs<double>& f, const Geom& g,
                         const double* epsinv, hipStream_t st) {
  return pole_post<double>(p, f, g, epsinv, st);
}
hipError_t pole_post_f32(const PoleDev& p, const FieldPtrs<float>& f, const Geom& g,
                         const float* epsinv, hipStream_t st) {
  return pole_post<float>(p, f, g, epsinv, st);
}

}  // namespace mlk
