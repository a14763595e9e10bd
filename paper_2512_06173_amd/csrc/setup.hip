// Set-up kernels: CPML coefficient tables, 1/eps_r, and precision conversion.
#include "mlk_internal.h"

namespace mlk {

// Convolutional PML coefficients along axis a at integer (half = 0) and
// half-integer (half = 1) positions x = i + half/2.  Inside a layer of d cells,
// at relative depth u in [0, 1] measured at x:
//   sigma = sigma_max u^m, kappa = 1 + (kappa_max - 1) u^m, alpha = alpha_max (1 - u),
//   b = exp(-(sigma/kappa + alpha) dt), c = sigma (b - 1) / (sigma kappa + kappa^2 alpha).
// Outside the layers b = 1, c = 0, 1/kappa = 1, which leaves a zero psi at zero.
template <typename T>
__global__ void k_cpml_tables(Geom g, int a, double m, double sigma_max, double kmax,
                              double amax, T* b, T* c, T* kinv) {
  const int N = g.n[a];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * N) return;
  const int half = t / N, i = t % N;
  const double x = (double)i + 0.5 * half;
  double depth = -1.0, d = 1.0;
  if (g.nlo[a] > 0 && x < (double)g.nlo[a]) {
    d = (double)g.nlo[a];
    depth = d - x;
  } else if (g.nhi[a] > 0 && x > (double)(N - g.nhi[a])) {
    d = (double)g.nhi[a];
    depth = x - ((double)N - d);
  }
  double bb = 1.0, cc = 0.0, ki = 1.0;
  if (depth >= 0.0) {
    const double u = depth / d;
    const double um = pow(u, m);
    const double sig = sigma_max * um;
    const double kap = 1.0 + (kmax - 1.0) * um;
    const double alp = amax * (1.0 - u);
    bb = exp(-(sig / kap + alp) * g.dt);
    cc = sig > 0.0 ? sig * (bb - 1.0) / (sig * kap + kap * kap * alp) : 0.0;
    ki = 1.0 / kap;
  }
  b[t] = (T)bb;
  c[t] = (T)cc;
  kinv[t] = (T)ki;
}

template <typename T>
__global__ void k_inverse(const double* src, T* dst, size_t n) {
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n;
       q += (size_t)gridDim.x * blockDim.x)
    dst[q] = (T)(1.0 / src[q]);
}

template <typename T>
__global__ void k_convert_in(const double* src, T* dst, size_t n) {
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n;
       q += (size_t)gridDim.x * blockDim.x)
    dst[q] = (T)src[q];
}

template <typename T>
__global__ void k_convert_out(const T* src, double* dst, size_t n) {
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n;
       q += (size_t)gridDim.x * blockDim.x)
    dst[q] = (double)src[q];
}

static dim3 grid_for(size_t n) {
  size_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  if (b == 0) b = 1;
  return dim3((unsigned)b);
}

hipError_t cpml_tables(bool fp32, const Geom& g, int a, double m, double sigma_max, double kmax,
                       double amax, void* b, void* c, void* kinv, hipStream_t st) {
  const int n = 2 * g.n[a];
  if (fp32)
    hipLaunchKernelGGL(k_cpml_tables<float>, dim3((n + 255) / 256), dim3(256), 0, st, g, a, m,
                       sigma_max, kmax, amax, (float*)b, (float*)c, (float*)kinv);
  else
    hipLaunchKernelGGL(k_cpml_tables<double>, dim3((n + 255) / 256), dim3(256), 0, st, g, a, m,
                       sigma_max, kmax, amax, (double*)b, (double*)c, (double*)kinv);
  return hipGetLastError();
}

hipError_t inverse_to(bool fp32, const double* src, void* dst, size_t n, hipStream_t st) {
  if (fp32)
    hipLaunchKernelGGL(k_inverse<float>, grid_for(n), dim3(256), 0, st, src, (float*)dst, n);
  else
    hipLaunchKernelGGL(k_inverse<double>, grid_for(n), dim3(256), 0, st, src, (double*)dst, n);
  return hipGetLastError();
}

hipError_t convert_in(bool fp32, const double* src, void* dst, size_t n, hipStream_t st) {
  if (fp32)
    hipLaunchKernelGGL(k_convert_in<float>, grid_for(n), dim3(256), 0, st, src, (float*)dst, n);
  else
    hipLaunchKernelGGL(k_convert_in<double>, grid_for(n), dim3(256), 0, st, src, (double*)dst, n);
  return hipGetLastError();
}

hipError_t convert_out(bool fp32, const void* src, double* dst, size_t n, hipStream_t st) {
  if (fp32)
    hipLaunchKernelGGL(k_convert_out<float>, grid_for(n), dim3(256), 0, st, (const float*)src, dst,
                       n);
  else
    hipLaunchKernelGGL(k_convert_out<double>, grid_for(n), dim3(256), 0, st, (const double*)src,
                       dst, n);
  return hipGetLastError();
}

// 1/eps_r over a box from its eps_r values (box order, x fastest).
template <typename T>
__global__ void k_eps_box(const double* eps, Geom g, Box box, T* epsinv) {
  const int bx = box.hi[0] - box.lo[0], by = box.hi[1] - box.lo[1], bz = box.hi[2] - box.lo[2];
  const size_t nb = (size_t)bx * by * bz;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nb) return;
  const int i = box.lo[0] + (int)(t % bx), j = box.lo[1] + (int)((t / bx) % by),
            k = box.lo[2] + (int)(t / ((size_t)bx * by));
  epsinv[cell_index(g, i, j, k)] = (T)(1.0 / eps[t]);
}
template <typename T>
static hipError_t launch_eps_box(const double* eps, const Geom& g, const Box& box, T* epsinv,
                                 hipStream_t st) {
  const size_t nb = (size_t)(box.hi[0] - box.lo[0]) * (box.hi[1] - box.lo[1]) * (box.hi[2] - box.lo[2]);
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_eps_box<T>, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, eps, g,
                     box, epsinv);
  return hipGetLastError();
}
hipError_t eps_box_f64(const double* eps, const Geom& g, const Box& box, double* epsinv,
                       hipStream_t st) {
  return launch_eps_box<double>(eps, g, box, epsinv, st);
}
hipError_t eps_box_f32(const double* eps, const Geom& g, const Box& box, float* epsinv,
                       hipStream_t st) {
  return launch_eps_box<float>(eps, g, box, epsinv, st);
}

}  // namespace mlk
