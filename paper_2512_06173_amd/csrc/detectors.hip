// Detectors: probes, Poynting flux through a plane, and the step counter.
//
// Flux through plane `index` of axis a, with (a, u, v) cyclic:
//   F^{n+1/2} = dx^2 sum_{plane} (E_u H_v - E_v H_u),
// E averaged over t_n and t_{n+1} at the plane, H at t_{n+1/2} averaged over the
// half cells on either side (indices index-1 and index along a).  The plane
// values of E^n are saved before the sweep overwrites them.  The sum is done
// in FP64 in a fixed order (block partials, then one block), so it is
// deterministic.
#include "mlk_internal.h"

namespace mlk {

// Partial flux of block b of nb (256 threads, grid-stride over the plane).
template <typename T>
__device__ __forceinline__ void flux_partial_body(const FieldPtrs<T>& f, const Geom& g,
                                                  const FluxPlane& fp, int b, int nb) {
  __shared__ double red[256];
  flux_partial_sum(f, g, fp, b, nb, red);
}

// Single block: probe samples, the flux total, then the step counter moves on.
template <typename T>
__device__ __forceinline__ void finish_body(const FieldPtrs<T>& f, const Geom& g,
                                            const FluxPlane& fp, const Series& ser,
                                            int64_t* step) {
  __shared__ double red[256];
  const int64_t n = *step;
  const int t = threadIdx.x;
  if (t < ser.nprobe) {
    const int comp = ser.probe_comp[t];
    const T* a = comp < 3 ? f.E[comp] : f.H[comp - 3];
    const double v = (double)a[ser.probe_idx[t]];
    ser.probe[(size_t)t * ser.cap + n] = v;
    if (!isfinite(v)) flag_nonfinite(ser, n);
  }
  if (fp.on) {
    double s = 0.0;
    for (int q = t; q < fp.nblocks; q += blockDim.x) s += fp.partial[q];
    red[t] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (t < w) red[t] += red[t + w];
      __syncthreads();
    }
    if (t == 0) {
      const double F = red[0] * g.dx * g.dx;
      fp.series[n] = F;
      *fp.total += g.dt * F;
      if (!isfinite(F)) flag_nonfinite(ser, n);
    }
  }
  __syncthreads();
  if (t == 0) *step = n + 1;
}

template <typename T>
__global__ void k_flux_save(FieldPtrs<T> f, Geom g, FluxPlane fp) {
  flux_save_body(f, g, fp, blockIdx.x * blockDim.x + threadIdx.x);
}
template <typename T>
__global__ __launch_bounds__(256) void k_flux_partial(FieldPtrs<T> f, Geom g, FluxPlane fp) {
  flux_partial_body(f, g, fp, blockIdx.x, gridDim.x);
}
template <typename T>
__global__ __launch_bounds__(256) void k_finish(FieldPtrs<T> f, Geom g, FluxPlane fp, Series ser,
                                                int64_t* step) {
  finish_body(f, g, fp, ser, step);
}

// Batched forms: kind 0 flux save, 1 flux partials, 2 finish (one block per job).
template <typename T, int KIND>
__global__ __launch_bounds__(256) void k_detect_batch(const FluxJob<T>* jobs, const int* start,
                                                      int njobs) {
  const int j = find_job(start, njobs, blockIdx.x);
  const FluxJob<T>& J = jobs[j];  // (a copy would put its probe arrays in scratch)
  const int lb = blockIdx.x - start[j];
  if (lb >= J.nblocks) return;
  if (KIND == 0) flux_save_body(J.f, J.g, J.fp, lb * blockDim.x + threadIdx.x);
  else if (KIND == 1) flux_partial_body(J.f, J.g, J.fp, lb, J.nblocks);
  else finish_body(J.f, J.g, J.fp, J.ser, J.step);
}

// Discrete field energy (Poynting's theorem on the Yee grid; invariant without
// currents, sources or absorbing layers):
//   W^n = dx^3 [ 1/2 sum eps_r |E^n|^2 + 1/2 sum H^{n+1/2} . H^{n-1/2} ].
// The fused sweep leaves E^n and H^{n-1/2} in the spare buffers (`old`) and
// H^{n+1/2} in the current ones, so W^n is formed right after the sweep; FP64
// partial sums per block, then one block adds them in a fixed order.
template <typename T>
__global__ __launch_bounds__(256) void k_energy_partial(FieldPtrs<T> old, FieldPtrs<T> cur,
                                                        size_t ncell, EnergyRec er,
                                                        const int64_t* step) {
  __shared__ double red[256];
  if (*step % er.every != 0) return;  // uniform across the grid
  double s = 0.0;
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < ncell;
       q += (size_t)gridDim.x * blockDim.x) {
    const double ex = old.E[0][q], ey = old.E[1][q], ez = old.E[2][q];
    const double eps = old.epsinv ? 1.0 / (double)old.epsinv[q] : 1.0;
    const double hh = (double)cur.H[0][q] * (double)old.H[0][q] +
                      (double)cur.H[1][q] * (double)old.H[1][q] +
                      (double)cur.H[2][q] * (double)old.H[2][q];
    s += 0.5 * eps * (ex * ex + ey * ey + ez * ez) + 0.5 * hh;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) er.partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_energy_finish(EnergyRec er, const int64_t* step) {
  __shared__ double red[256];
  const int64_t n = *step;
  if (n % er.every != 0) return;
  const int t = threadIdx.x;
  double s = 0.0;
  for (int q = t; q < er.nblocks; q += blockDim.x) s += er.partial[q];
  red[t] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (t == 0) er.series[n / er.every] = red[0] * er.dv;
}

template <typename T>
static hipError_t launch_energy(const FieldPtrs<T>& old, const FieldPtrs<T>& cur, size_t ncell,
                                const EnergyRec& er, const int64_t* step, hipStream_t st) {
  hipLaunchKernelGGL(k_energy_partial<T>, dim3(er.nblocks), dim3(256), 0, st, old, cur, ncell, er,
                     step);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_energy_finish, dim3(1), dim3(256), 0, st, er, step);
  return hipGetLastError();
}

hipError_t energy_f64(const FieldPtrs<double>& old, const FieldPtrs<double>& cur, size_t ncell,
                      const EnergyRec& er, const int64_t* step, hipStream_t st) {
  return launch_energy<double>(old, cur, ncell, er, step, st);
}
hipError_t energy_f32(const FieldPtrs<float>& old, const FieldPtrs<float>& cur, size_t ncell,
                      const EnergyRec& er, const int64_t* step, hipStream_t st) {
  return launch_energy<float>(old, cur, ncell, er, step, st);
}

template <typename T>
static hipError_t launch_flux_save(const FieldPtrs<T>& f, const Geom& g, const FluxPlane& fp,
                                   hipStream_t st) {
  const int a = fp.axis, u = (a + 1) % 3, v = (a + 2) % 3;
  const int np = g.n[u] * g.n[v];
  hipLaunchKernelGGL(k_flux_save<T>, dim3((np + 255) / 256), dim3(256), 0, st, f, g, fp);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_finish(const FieldPtrs<T>& f, const Geom& g, const FluxPlane& fp,
                                const Series& ser, int64_t* step, bool partials_done,
                                hipStream_t st) {
  if (fp.on && !partials_done) {
    hipLaunchKernelGGL(k_flux_partial<T>, dim3(fp.nblocks), dim3(256), 0, st, f, g, fp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_finish<T>, dim3(1), dim3(256), 0, st, f, g, fp, ser, step);
  return hipGetLastError();
}

hipError_t flux_save_f64(const FieldPtrs<double>& f, const Geom& g, const FluxPlane& fp,
                         hipStream_t st) {
  return launch_flux_save<double>(f, g, fp, st);
}
hipError_t flux_save_f32(const FieldPtrs<float>& f, const Geom& g, const FluxPlane& fp,
                         hipStream_t st) {
  return launch_flux_save<float>(f, g, fp, st);
}
hipError_t finish_f64(const FieldPtrs<double>& f, const Geom& g, const FluxPlane& fp,
                      const Series& ser, int64_t* step, bool partials_done, hipStream_t st) {
  return launch_finish<double>(f, g, fp, ser, step, partials_done, st);
}
hipError_t finish_f32(const FieldPtrs<float>& f, const Geom& g, const FluxPlane& fp,
                      const Series& ser, int64_t* step, bool partials_done, hipStream_t st) {
  return launch_finish<float>(f, g, fp, ser, step, partials_done, st);
}

template <typename T>
static hipError_t launch_detect_batch(const FluxJob<T>* jobs, const int* start, int njobs,
                                      int nblocks, int kind, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  if (kind == 0)
    hipLaunchKernelGGL((k_detect_batch<T, 0>), dim3(nblocks), dim3(256), 0, st, jobs, start, njobs);
  else if (kind == 1)
    hipLaunchKernelGGL((k_detect_batch<T, 1>), dim3(nblocks), dim3(256), 0, st, jobs, start, njobs);
  else
    hipLaunchKernelGGL((k_detect_batch<T, 2>), dim3(nblocks), dim3(256), 0, st, jobs, start, njobs);
  return hipGetLastError();
}
hipError_t detect_batch_f64(const FluxJob<double>* jobs, const int* start, int njobs, int nblocks,
                            int kind, hipStream_t st) {
  return launch_detect_batch<double>(jobs, start, njobs, nblocks, kind, st);
}
hipError_t detect_batch_f32(const FluxJob<float>* jobs, const int* start, int njobs, int nblocks,
                            int kind, hipStream_t st) {
  return launch_detect_batch<float>(jobs, start, njobs, nblocks, kind, st);
}

}  // namespace mlk
