// Single-mode cavity in place of the grid (Sec. II.A.2: the normal-mode field
// Hamiltonian with the dipole self-energy, its equations of motion and the
// coupling eps = w / sqrt(V) in the single-mode limit, eps0 = 1).
//
// One photonic mode of frequency w with an x and a y polarisation, mode
// function e_l / sqrt(V).  Every emitter feels the same regularised field
//   E~ = -sum_l (eps q_l + d_l / V) e_l,     d_l = sum_m <mu_l^(m)>,
// and the mode obeys q_l'' = -w^2 q_l - eps d_l.  The discretisation follows
// the grid scheme: q at integer steps, p = q' half a step before, emitters at
// half steps, and the total dipole advanced with the same dipole rate that the
// grid would receive as current, d^{n+1} = d^n + dt sum_m mu_dot^{n+1/2}.
//
// Per step, general case: one launch writes E~ for every emitter, the emitter
// kernels advance the states and leave mu_dot, a grid of blocks sums
// mu_dot_x,y in FP64 into per-block partials, and one block adds the partials
// in a fixed order, advances (p, q, d) and moves the step counter on.  With
// two-level emitters only, one launch forms E~, steps the emitters and leaves
// the per-block partials itself (the step is launch-bound, so two launches
// instead of four).  The mode state is six doubles in device memory: q_x, q_y,
// p_x, p_y, d_x, d_y.
#include "launch.h"

namespace mlk {

namespace {

constexpr int kCavThreads = 256;

__global__ __launch_bounds__(kCavThreads) void k_cavity_field(const double* __restrict__ st,
                                                              double eps, double V,
                                                              double* __restrict__ Et, int M) {
  const int m = blockIdx.x * kCavThreads + threadIdx.x;
  if (m >= M) return;
  const double ex = -(eps * st[0] + st[4] / V);
  const double ey = -(eps * st[1] + st[5] / V);
  Et[3 * (size_t)m + 0] = ex;
  Et[3 * (size_t)m + 1] = ey;
  Et[3 * (size_t)m + 2] = 0.0;
}

// Sum of two doubles over the block, in a fixed tree order; the result is
// valid in thread 0.
__device__ __forceinline__ void block_sum2(double& x, double& y) {
  __shared__ double rx[kCavThreads], ry[kCavThreads];
  const int t = threadIdx.x;
  rx[t] = x;
  ry[t] = y;
  __syncthreads();
  for (int w = kCavThreads / 2; w > 0; w >>= 1) {
    if (t < w) {
      rx[t] += rx[t + w];
      ry[t] += ry[t + w];
    }
    __syncthreads();
  }
  x = rx[0];
  y = ry[0];
}

__global__ __launch_bounds__(kCavThreads) void k_cavity_partial(const double* __restrict__ mudot,
                                                                int M,
                                                                double* __restrict__ partial) {
  double sx = 0.0, sy = 0.0;
  for (int m = blockIdx.x * kCavThreads + threadIdx.x; m < M; m += gridDim.x * kCavThreads) {
    sx += mudot[3 * (size_t)m + 0];
    sy += mudot[3 * (size_t)m + 1];
  }
  block_sum2(sx, sy);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x + 0] = sx;
    partial[2 * blockIdx.x + 1] = sy;
  }
}

__global__ __launch_bounds__(kCavThreads) void k_cavity_update(double* __restrict__ st,
                                                               const double* __restrict__ partial,
                                                               int nb, double dt, double w,
                                                               double eps,
                                                               int64_t* __restrict__ step) {
  const int t = threadIdx.x;
  double sx = 0.0, sy = 0.0;
  for (int q = t; q < nb; q += kCavThreads) {
    sx += partial[2 * q + 0];
    sy += partial[2 * q + 1];
  }
  block_sum2(sx, sy);
  if (t == 0) {
    const double sum[2] = {sx, sy};
    const double w2 = w * w;
    for (int l = 0; l < 2; ++l) {
      const double q = st[l], d = st[4 + l];
      const double p = st[2 + l] - dt * (w2 * q + eps * d);
      st[2 + l] = p;
      st[l] = q + dt * p;
      st[4 + l] = d + dt * sum[l];
    }
    *step = *step + 1;
  }
}

}  // namespace

int cavity_blocks(int M) {
  const int nb = (M + 4 * kCavThreads - 1) / (4 * kCavThreads);
  return nb < 1 ? 1 : (nb > kCavThreads ? kCavThreads : nb);
}

hipError_t cavity_field(const CavityDev& c, double* Et, int M, hipStream_t st) {
  if (M <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cavity_field, dim3((M + kCavThreads - 1) / kCavThreads), dim3(kCavThreads),
                     0, st, c.st, c.eps, c.V, Et, M);
  return hipGetLastError();
}

hipError_t cavity_advance(const CavityDev& c, int npartial, double dt, int64_t* step,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_cavity_update, dim3(1), dim3(kCavThreads), 0, st, c.st, c.partial,
                     npartial, dt, c.w, c.eps, step);
  return hipGetLastError();
}

hipError_t cavity_update(const CavityDev& c, const double* mudot, int M, double dt, int64_t* step,
                         hipStream_t st) {
  const int nb = cavity_blocks(M);
  if (M > 0) {
    hipLaunchKernelGGL(k_cavity_partial, dim3(nb), dim3(kCavThreads), 0, st, mudot, M, c.partial);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return cavity_advance(c, M > 0 ? nb : 0, dt, step, st);
}

}  // namespace mlk
