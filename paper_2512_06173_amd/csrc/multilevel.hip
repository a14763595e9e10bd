// Multilevel emitters: the open model of Sec. II.B.1 with pure dephasing.
//
// d rho/dt = -i [H_eff, rho] + sum_k (L_k rho L_k^+ - {L_k^+ L_k, rho}/2),
// H_eff = H0 - E~ . mu, H0 = diag(E_0..E_{n-1}), mu^c = d^c M (M real
// symmetric), L_k = sqrt(gphi) |k><k|   (eq. von-Neumann-tls with the
// Lindblad term).
//
// One step over dt (Strang splitting, second order):
//   dephase(dt/2): rho_ab *= exp(-gphi dt/2) for a != b   (exact for this dissipator)
//   unitary:       rho <- U rho U^+, U = exp(-i H_eff dt) = C - i S,
//                  C = Q cos(L dt) Q^T, S = Q sin(L dt) Q^T from H_eff = Q L Q^T
//   dephase(dt/2)
// then mu_dot^c = Tr(rho_dot mu^c) (eq. dipole_derivative) at the new state.  For
// this model the trace has a closed form (with rho = R + i I):
//   Tr(rho_dot M) = -2 sum_{a<b} M_ab [ I_ab (E_b - E_a) + gphi R_ab ]
// (the field term drops out because [M, M] = 0; the dissipator only damps
// the coherences).  For n = 2 it reduces to the two-level -2 w0 Im rho01.
//
// One thread per emitter, the level count n a template parameter so that every
// matrix lives in registers; emitters are grouped by n and each group is one
// launch.  State is stored structure-of-arrays (entry-major) so that
// neighbouring threads read neighbouring words.
#include "mlk_internal.h"

namespace mlk {

namespace {

// packed index of the upper triangle (a <= b) of an N x N symmetric matrix
template <int N>
__device__ constexpr int up(int a, int b) {
  return a <= b ? a * N - a * (a - 1) / 2 + (b - a) : b * N - b * (b - 1) / 2 + (a - b);
}

template <int N>
__device__ __forceinline__ void jacobi(double (&A)[N][N], double (&Q)[N][N]) {
#pragma unroll
  for (int a = 0; a < N; ++a)
#pragma unroll
    for (int b = 0; b < N; ++b) Q[a][b] = a == b ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 32; ++sweep) {
    double off = 0.0, diag = 0.0;
#pragma unroll
    for (int a = 0; a < N; ++a) {
      diag += A[a][a] * A[a][a];
#pragma unroll
      for (int b = a + 1; b < N; ++b) off += A[a][b] * A[a][b];
    }
    if (!(off > 1e-34 * (diag + 2.0 * off))) break;
#pragma unroll
    for (int p = 0; p < N - 1; ++p)
#pragma unroll
      for (int q = p + 1; q < N; ++q) {
        const double apq = A[p][q];
        if (apq == 0.0) continue;
        // rotation in the (p, q) plane that zeroes A[p][q]
        const double th = (A[q][q] - A[p][p]) / (2.0 * apq);
        const double t = copysign(1.0, th) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        A[p][p] -= t * apq;
        A[q][q] += t * apq;
        A[p][q] = A[q][p] = 0.0;
#pragma unroll
        for (int r = 0; r < N; ++r) {
          if (r == p || r == q) continue;
          const double arp = A[r][p], arq = A[r][q];
          A[r][p] = A[p][r] = c * arp - s * arq;
          A[r][q] = A[q][r] = s * arp + c * arq;
        }
#pragma unroll
        for (int r = 0; r < N; ++r) {
          const double qrp = Q[r][p], qrq = Q[r][q];
          Q[r][p] = c * qrp - s * qrq;
          Q[r][q] = s * qrp + c * qrq;
        }
      }
  }
}

}  // namespace

template <int N>
__device__ __forceinline__ void ml_body(const MlDev& ml, int first, int count, double dt,
                                        const double* Et, double* mudot, const int64_t* pop_off,
                                        const Series& ser, const int64_t* step, int t) {
  constexpr int NS = N * (N + 1) / 2;
  const int m = first + t;
  if (t >= count) return;
  const size_t st = (size_t)ml.count;
  const int e = ml.gid[m];
  const double gphi = ml.gphi[m];
  const double g = Et[3 * e] * ml.dip[m] + Et[3 * e + 1] * ml.dip[st + m] +
                   Et[3 * e + 2] * ml.dip[2 * st + m];

  // U = exp(-i H_eff dt) = C - i S (C, S symmetric, packed upper triangles)
  double C[NS], S[NS];
  {
    double A[N][N], Q[N][N];
#pragma unroll
    for (int a = 0; a < N; ++a)
#pragma unroll
      for (int b = a; b < N; ++b) {
        const double v = (a == b ? ml.en[a * st + m] : 0.0) - g * ml.M[(a * kMaxLevels + b) * st + m];
        A[a][b] = A[b][a] = v;
      }
    jacobi<N>(A, Q);
    double cl[N], sl[N];
#pragma unroll
    for (int q = 0; q < N; ++q) sincos(A[q][q] * dt, &sl[q], &cl[q]);
#pragma unroll
    for (int a = 0; a < N; ++a)
#pragma unroll
      for (int b = a; b < N; ++b) {
        double c = 0.0, s = 0.0;
#pragma unroll
        for (int q = 0; q < N; ++q) {
          const double qq = Q[a][q] * Q[b][q];
          c += qq * cl[q];
          s += qq * sl[q];
        }
        C[up<N>(a, b)] = c;
        S[up<N>(a, b)] = s;
      }
  }

  // rho = R + i I after the first half dephasing (R symmetric, I antisymmetric;
  // upper triangles, the diagonal of I unused)
  const double f = exp(-0.5 * gphi * dt);
  double R[NS], I[NS];
#pragma unroll
  for (int a = 0; a < N; ++a)
#pragma unroll
    for (int b = a; b < N; ++b) {
      const size_t q = (size_t)(a * kMaxLevels + b);
      const double k = a == b ? 1.0 : f;
      R[up<N>(a, b)] = k * ml.rho[(2 * q) * st + m];
      I[up<N>(a, b)] = a == b ? 0.0 : k * ml.rho[(2 * q + 1) * st + m];
    }
  auto Rf = [&](int a, int b) { return R[up<N>(a, b)]; };
  auto If = [&](int a, int b) { return a < b ? I[up<N>(a, b)] : (a > b ? -I[up<N>(b, a)] : 0.0); };

  // rho' = U rho U^+ row by row: T = U rho (row a), rho'_ab = (T U^+)_ab for b >= a;
  // the second half dephasing, the store, the population and the trace follow
  double tr = 0.0, diag = 0.0;
  const int64_t n = *step;
  const bool rec = ser.pop_every > 0 && n % ser.pop_every == 0;
#pragma unroll
  for (int a = 0; a < N; ++a) {
    double Tr_[N], Ti_[N];
#pragma unroll
    for (int b = 0; b < N; ++b) {
      // (C - iS)(R + iI) = (C R + S I) + i (C I - S R)
      double re = 0.0, im = 0.0;
#pragma unroll
      for (int c = 0; c < N; ++c) {
        const double cac = C[up<N>(a, c)], sac = S[up<N>(a, c)];
        re += cac * Rf(c, b) + sac * If(c, b);
        im += cac * If(c, b) - sac * Rf(c, b);
      }
      Tr_[b] = re;
      Ti_[b] = im;
    }
#pragma unroll
    for (int b = a; b < N; ++b) {
      // T (C + iS) with C, S symmetric: column b of C is row b
      double re = 0.0, im = 0.0;
#pragma unroll
      for (int c = 0; c < N; ++c) {
        const double ccb = C[up<N>(c, b)], scb = S[up<N>(c, b)];
        re += Tr_[c] * ccb - Ti_[c] * scb;
        im += Tr_[c] * scb + Ti_[c] * ccb;
      }
      const size_t q = (size_t)(a * kMaxLevels + b);
      if (a == b) {
        diag += re;
        ml.rho[(2 * q) * st + m] = re;
        ml.rho[(2 * q + 1) * st + m] = 0.0;
        if (rec && a > 0)
          ser.pop[(n / ser.pop_every) * ser.npop + pop_off[e] + (a - 1)] = re;
      } else {
        re *= f;
        im *= f;
        const size_t qt = (size_t)(b * kMaxLevels + a);
        ml.rho[(2 * q) * st + m] = re;
        ml.rho[(2 * q + 1) * st + m] = im;
        ml.rho[(2 * qt) * st + m] = re;
        ml.rho[(2 * qt + 1) * st + m] = -im;
        const double Mab = ml.M[(a * kMaxLevels + b) * st + m];
        tr += Mab * (im * (ml.en[b * st + m] - ml.en[a * st + m]) + gphi * re);
      }
    }
  }
  tr *= -2.0;
  if (!isfinite(tr + diag)) flag_nonfinite(ser, n);
  mudot[3 * e] = tr * ml.dip[m];
  mudot[3 * e + 1] = tr * ml.dip[st + m];
  mudot[3 * e + 2] = tr * ml.dip[2 * st + m];
}

template <int N>
__global__ __launch_bounds__(64) void k_ml_step(MlDev ml, int first, int count, double dt,
                                                const double* Et, double* mudot,
                                                const int64_t* pop_off, Series ser,
                                                const int64_t* step) {
  ml_body<N>(ml, first, count, dt, Et, mudot, pop_off, ser, step,
             blockIdx.x * blockDim.x + threadIdx.x);
}

template <int N>
__global__ __launch_bounds__(64) void k_ml_batch(const MlJob* jobs, const int* start, int njobs) {
  const int j = find_job(start, njobs, blockIdx.x);
  const MlJob J = load_job(jobs, j);
  const int lb = blockIdx.x - start[j];
  if (lb >= J.nblocks) return;
  ml_body<N>(J.ml, J.first, J.count, J.dt, J.Et, J.mudot, J.pop_off, J.ser, J.step,
             lb * blockDim.x + threadIdx.x);
}

// Batched multilevel step; every job of the table has `nl` levels.
hipError_t ml_batch(const MlJob* jobs, const int* start, int njobs, int nblocks, int nl,
                    hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  const dim3 grid(nblocks), block(64);
  switch (nl) {
    case 2: hipLaunchKernelGGL(k_ml_batch<2>, grid, block, 0, st, jobs, start, njobs); break;
    case 3: hipLaunchKernelGGL(k_ml_batch<3>, grid, block, 0, st, jobs, start, njobs); break;
    case 4: hipLaunchKernelGGL(k_ml_batch<4>, grid, block, 0, st, jobs, start, njobs); break;
    case 5: hipLaunchKernelGGL(k_ml_batch<5>, grid, block, 0, st, jobs, start, njobs); break;
    case 6: hipLaunchKernelGGL(k_ml_batch<6>, grid, block, 0, st, jobs, start, njobs); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t ml_step(const MlDev& ml, const int* range, double dt, const double* Et, double* mudot,
                   const int64_t* pop_off, const Series& ser, const int64_t* step,
                   hipStream_t st) {
  for (int nl = 2; nl <= kMaxLevels; ++nl) {
    const int first = range[nl], count = range[nl + 1] - range[nl];
    if (count <= 0) continue;
    const dim3 grid((count + 63) / 64), block(64);
    switch (nl) {
      case 2: hipLaunchKernelGGL(k_ml_step<2>, grid, block, 0, st, ml, first, count, dt, Et, mudot, pop_off, ser, step); break;
      case 3: hipLaunchKernelGGL(k_ml_step<3>, grid, block, 0, st, ml, first, count, dt, Et, mudot, pop_off, ser, step); break;
      case 4: hipLaunchKernelGGL(k_ml_step<4>, grid, block, 0, st, ml, first, count, dt, Et, mudot, pop_off, ser, step); break;
      case 5: hipLaunchKernelGGL(k_ml_step<5>, grid, block, 0, st, ml, first, count, dt, Et, mudot, pop_off, ser, step); break;
      case 6: hipLaunchKernelGGL(k_ml_step<6>, grid, block, 0, st, ml, first, count, dt, Et, mudot, pop_off, ser, step); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace mlk
