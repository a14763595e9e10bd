// Single-mode cavity in place of the grid (Sec. II.A.2: the normal-mode field
// Hamiltonian with the dipole self-energy, its equations of motion and the
// coupling eps = w / sqrt(V) in the single-mode limit, eps0 = 1).
//
// One photonic mode of frequency w with an x and a y polarisation, mode
// function e_l / sqrt(V).  Every emitter feels the same regularised field
//   E~ = -sum_l (eps q_l + d_l / V) e_l,     d_l = sum_m <mu_l^(m)>,
// and the mode obeys q_l'' = -w^2 q_l - eps d_l.  The discretisation follows
// the grid scheme: q at integer steps, p = q' half a step before, emitters at
// half steps.  The total dipole at t_n is the sum of the expectation values of
// the latest states (t_{n-1/2}) carried half a step forward by their own rate,
//   d^n = sum_m [ <mu_m>(rho^{n-1/2}) + (dt/2) mu_dot_m(rho^{n-1/2}) ],
// (eq. dklambda_def at the integer time, second order); mu_dot depends on the
// state alone, so the sum is a function of the states.
//
// Per step, general case: one launch writes E~ for every emitter, the emitter
// kernels advance the states, a grid of blocks forms <mu> + (dt/2) mu_dot of
// the new states in FP64 and leaves per-block partial sums, and one block adds
// the partials in a fixed order, advances (p, q) with the old d, stores the new
// d and moves the step counter on.  With two-level emitters only, one launch
// forms E~, steps the emitters and leaves the per-block partials itself (the
// step is launch-bound, so two launches instead of four).  The mode state is
// six doubles in device memory: q_x, q_y, p_x, p_y, d_x, d_y.
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

// <mu_x,y> + (dt/2) mu_dot_x,y of every emitter from its state, summed per
// block (two-level slots first, then multilevel slots, each block a fixed
// range).  Two-level: <mu> = 2 Re rho01 d, mu_dot = -2 w0 Im rho01 d.
// Multilevel (mu = d M, rho = R + i I in the zero-padded frame):
// <mu> = d sum_ab R_ab M_ab, mu_dot = d (-2 sum_{a<b} M_ab [I_ab (E_b - E_a) + gphi R_ab]).
__global__ __launch_bounds__(kCavThreads) void k_cavity_partial(TlsPtrs tls, MlDev ml, double dt,
                                                                double* __restrict__ partial) {
  constexpr int F = kMaxLevels;
  const int total = tls.count + ml.count;
  double sx = 0.0, sy = 0.0;
  for (int q = blockIdx.x * kCavThreads + threadIdx.x; q < total; q += gridDim.x * kCavThreads) {
    double mu, rate, dx, dy;
    if (q < tls.count) {
      const double w0 = tls.omega0[q];
      mu = 2.0 * tls.rho[3 * (size_t)q + 1];
      rate = -2.0 * w0 * tls.rho[3 * (size_t)q + 2];
      dx = tls.dip[3 * (size_t)q + 0];
      dy = tls.dip[3 * (size_t)q + 1];
    } else {
      const size_t m = (size_t)(q - tls.count), n = (size_t)ml.count;
      const double g = ml.gphi[m];
      mu = 0.0;
      rate = 0.0;
      for (int a = 0; a < F; ++a) {
        const double ea = ml.en[a * n + m];
        mu += ml.rho[(size_t)(2 * (a * F + a)) * n + m] * ml.M[(size_t)(a * F + a) * n + m];
        for (int b = a + 1; b < F; ++b) {
          const double Mab = ml.M[(size_t)(a * F + b) * n + m];
          const double R = ml.rho[(size_t)(2 * (a * F + b)) * n + m];
          const double I = ml.rho[(size_t)(2 * (a * F + b) + 1) * n + m];
          mu += 2.0 * R * Mab;
          rate += -2.0 * Mab * (I * (ml.en[b * n + m] - ea) + g * R);
        }
      }
      dx = ml.dip[m];
      dy = ml.dip[n + m];
    }
    const double v = mu + 0.5 * dt * rate;
    sx += v * dx;
    sy += v * dy;
  }
  block_sum2(sx, sy);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x + 0] = sx;
    partial[2 * blockIdx.x + 1] = sy;
  }
}

// Sum of the partials in a fixed order; with advance, the leapfrog of (p, q) with
// the old d, then the new d and the step counter; without, only the new d.
__global__ __launch_bounds__(kCavThreads) void k_cavity_update(double* __restrict__ st,
                                                               const double* __restrict__ partial,
                                                               int nb, double dt, double w,
                                                               double eps, int advance,
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
      if (advance) {
        const double q = st[l], d = st[4 + l];
        const double p = st[2 + l] - dt * (w2 * q + eps * d);
        st[2 + l] = p;
        st[l] = q + dt * p;
      }
      st[4 + l] = sum[l];
    }
    if (advance) *step = *step + 1;
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
                     npartial, dt, c.w, c.eps, 1, step);
  return hipGetLastError();
}

static hipError_t cavity_partials(const CavityDev& c, const TlsPtrs& tls, const MlDev& ml,
                                  double dt, int* nb, hipStream_t st) {
  const int M = tls.count + ml.count;
  *nb = M > 0 ? cavity_blocks(M) : 0;
  if (M <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cavity_partial, dim3(*nb), dim3(kCavThreads), 0, st, tls, ml, dt,
                     c.partial);
  return hipGetLastError();
}

hipError_t cavity_update(const CavityDev& c, const TlsPtrs& tls, const MlDev& ml, double dt,
                         int64_t* step, hipStream_t st) {
  int nb = 0;
  const hipError_t e = cavity_partials(c, tls, ml, dt, &nb, st);
  if (e != hipSuccess) return e;
  return cavity_advance(c, nb, dt, step, st);
}

hipError_t cavity_set_dipole(const CavityDev& c, const TlsPtrs& tls, const MlDev& ml, double dt,
                             hipStream_t st) {
  int nb = 0;
  const hipError_t e = cavity_partials(c, tls, ml, dt, &nb, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cavity_update, dim3(1), dim3(kCavThreads), 0, st, c.st, c.partial, nb,
                     dt, c.w, c.eps, 0, nullptr);
  return hipGetLastError();
}

}  // namespace mlk
