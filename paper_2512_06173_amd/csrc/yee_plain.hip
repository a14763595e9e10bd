// Plain (unfused) Yee sweeps: one pass for H, one for E, one thread per cell.
// This is the reference GPU sweep (and the "plain" variant of the benchmark);
// the fused single-pass sweep lives in yee_fused.hip.
//
// H^{n+1/2} = H^{n-1/2} - dt curl E^n,  E^{n+1} = E^n + (dt/eps_r)(curl H^{n+1/2} - J_src)
// (eq. Maxwell with D = eps_r E, B = H), convolutional PML stretching of each
// spatial derivative inside the absorbing layers, metallic (tangential E = 0)
// or periodic closure.  The molecular current is added by the scatter pass.
#include "mlk_internal.h"
#include "yee_common.h"

namespace mlk {

template <typename T>
__global__ __launch_bounds__(256) void k_update_h(FieldPtrs<T> f, Geom g) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= g.n[0] || j >= g.n[1]) return;
  const size_t sx = 1, sy = (size_t)g.n[0], sz = (size_t)g.n[0] * g.n[1];
  const size_t id = cell_index(g, i, j, k);
  const T idx = (T)g.inv_dx;
  const T ex = f.E[0][id], ey = f.E[1][id], ez = f.E[2][id];
  T dEz_dy = (fwd(f.E[2], id, j, g.n[1], g.periodic[1], sy) - ez) * idx;
  T dEy_dz = (fwd(f.E[1], id, k, g.n[2], g.periodic[2], sz) - ey) * idx;
  T dEx_dz = (fwd(f.E[0], id, k, g.n[2], g.periodic[2], sz) - ex) * idx;
  T dEz_dx = (fwd(f.E[2], id, i, g.n[0], g.periodic[0], sx) - ez) * idx;
  T dEy_dx = (fwd(f.E[1], id, i, g.n[0], g.periodic[0], sx) - ey) * idx;
  T dEx_dy = (fwd(f.E[0], id, j, g.n[1], g.periodic[1], sy) - ex) * idx;
  dEz_dy = stretch(f, g, f.psiH[0][1], 1, 1, i, j, k, dEz_dy);
  dEy_dz = stretch(f, g, f.psiH[0][2], 2, 1, i, j, k, dEy_dz);
  dEx_dz = stretch(f, g, f.psiH[1][2], 2, 1, i, j, k, dEx_dz);
  dEz_dx = stretch(f, g, f.psiH[1][0], 0, 1, i, j, k, dEz_dx);
  dEy_dx = stretch(f, g, f.psiH[2][0], 0, 1, i, j, k, dEy_dx);
  dEx_dy = stretch(f, g, f.psiH[2][1], 1, 1, i, j, k, dEx_dy);
  const T dt = (T)g.dt;
  f.H[0][id] -= dt * (dEz_dy - dEy_dz);
  f.H[1][id] -= dt * (dEx_dz - dEz_dx);
  f.H[2][id] -= dt * (dEy_dx - dEx_dy);
}

template <typename T>
__global__ __launch_bounds__(256) void k_update_e(FieldPtrs<T> f, Geom g, SourceSet src,
                                                  const int64_t* step) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= g.n[0] || j >= g.n[1]) return;
  const size_t sx = 1, sy = (size_t)g.n[0], sz = (size_t)g.n[0] * g.n[1];
  const size_t id = cell_index(g, i, j, k);
  const T idx = (T)g.inv_dx;
  const T hx = f.H[0][id], hy = f.H[1][id], hz = f.H[2][id];
  T dHz_dy = (hz - bwd(f.H[2], id, j, g.n[1], g.periodic[1], sy)) * idx;
  T dHy_dz = (hy - bwd(f.H[1], id, k, g.n[2], g.periodic[2], sz)) * idx;
  T dHx_dz = (hx - bwd(f.H[0], id, k, g.n[2], g.periodic[2], sz)) * idx;
  T dHz_dx = (hz - bwd(f.H[2], id, i, g.n[0], g.periodic[0], sx)) * idx;
  T dHy_dx = (hy - bwd(f.H[1], id, i, g.n[0], g.periodic[0], sx)) * idx;
  T dHx_dy = (hx - bwd(f.H[0], id, j, g.n[1], g.periodic[1], sy)) * idx;
  dHz_dy = stretch(f, g, f.psiE[0][1], 1, 0, i, j, k, dHz_dy);
  dHy_dz = stretch(f, g, f.psiE[0][2], 2, 0, i, j, k, dHy_dz);
  dHx_dz = stretch(f, g, f.psiE[1][2], 2, 0, i, j, k, dHx_dz);
  dHz_dx = stretch(f, g, f.psiE[1][0], 0, 0, i, j, k, dHz_dx);
  dHy_dx = stretch(f, g, f.psiE[2][0], 0, 0, i, j, k, dHy_dx);
  dHx_dy = stretch(f, g, f.psiE[2][1], 1, 0, i, j, k, dHx_dy);
  T J[3] = {T(0), T(0), T(0)};
  source_current(src, g, step, i, j, k, J);
  const T ce = (T)g.dt * f.epsinv[id];
  const T cx = dHz_dy - dHy_dz - J[0];
  const T cy = dHx_dz - dHz_dx - J[1];
  const T cz = dHy_dx - dHx_dy - J[2];
  f.E[0][id] = tangential_wall(g, 0, i, j, k) ? T(0) : f.E[0][id] + ce * cx;
  f.E[1][id] = tangential_wall(g, 1, i, j, k) ? T(0) : f.E[1][id] + ce * cy;
  f.E[2][id] = tangential_wall(g, 2, i, j, k) ? T(0) : f.E[2][id] + ce * cz;
}

template <typename T>
static hipError_t launch_plain(const FieldPtrs<T>& f, const Geom& g, const SourceSet& src,
                               const int64_t* step, hipStream_t st) {
  dim3 block(64, 4, 1);
  dim3 grid((g.n[0] + 63) / 64, (g.n[1] + 3) / 4, g.n[2]);
  hipLaunchKernelGGL(k_update_h<T>, grid, block, 0, st, f, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_update_e<T>, grid, block, 0, st, f, g, src, step);
  return hipGetLastError();
}

hipError_t sweep_plain_f64(const FieldPtrs<double>& f, const Geom& g, const SourceSet& src,
                           const int64_t* step, hipStream_t st) {
  return launch_plain<double>(f, g, src, step, st);
}

hipError_t sweep_plain_f32(const FieldPtrs<float>& f, const Geom& g, const SourceSet& src,
                           const int64_t* step, hipStream_t st) {
  return launch_plain<float>(f, g, src, step, st);
}

}  // namespace mlk
