// Plain (unfused) Yee sweeps: one pass for H, one for E, one thread per cell,
// over a box of cells.
//
// H^{n+1/2} = H^{n-1/2} - dt curl E^n,   E^{n+1} = E^n + (dt/eps_r) curl H^{n+1/2}
// (eq. Maxwell with D = eps_r E, B = H), convolutional PML stretching of each
// spatial derivative inside the absorbing layers, metallic (tangential E = 0)
// or periodic closure.  Source and molecular currents are added by their own
// passes.
//
// The passes read one field buffer (`in`) and write another (`out`); with
// in == out they update in place, which is how the plain sweep runs on the whole
// grid.  The fused sweep uses them, out of place, on the CPML shell: the cells
// outside its interior box, enumerated compactly by one launch per pass.
#include "mlk_internal.h"
#include "yee_common.h"

namespace mlk {

// H^{n+1/2} at cell (i,j,k) from E^n of `in`.
template <typename T>
__device__ __forceinline__ void update_h_cell(const FieldPtrs<T>& in, const FieldPtrs<T>& out,
                                              const Geom& g, int i, int j, int k) {
  // products are not contracted into fused multiply-adds, as in the fused sweep,
  // so that every way of splitting the grid between the two rounds alike
#pragma clang fp contract(off)
  const size_t sx = 1, sy = (size_t)g.n[0], sz = (size_t)g.n[0] * g.n[1];
  const size_t id = cell_index(g, i, j, k);
  const T idx = (T)g.inv_dx;
  const T ex = in.E[0][id], ey = in.E[1][id], ez = in.E[2][id];
  T dEz_dy = (fwd(in.E[2], id, j, g.n[1], g.periodic[1], sy) - ez) * idx;
  T dEy_dz = (fwd(in.E[1], id, k, g.n[2], g.periodic[2], sz) - ey) * idx;
  T dEx_dz = (fwd(in.E[0], id, k, g.n[2], g.periodic[2], sz) - ex) * idx;
  T dEz_dx = (fwd(in.E[2], id, i, g.n[0], g.periodic[0], sx) - ez) * idx;
  T dEy_dx = (fwd(in.E[1], id, i, g.n[0], g.periodic[0], sx) - ey) * idx;
  T dEx_dy = (fwd(in.E[0], id, j, g.n[1], g.periodic[1], sy) - ex) * idx;
  dEz_dy = stretch(g, in.tab, in.psi, out.psi, 1, 0, 1, i, j, k, dEz_dy);
  dEy_dz = stretch(g, in.tab, in.psi, out.psi, 1, 0, 2, i, j, k, dEy_dz);
  dEx_dz = stretch(g, in.tab, in.psi, out.psi, 1, 1, 2, i, j, k, dEx_dz);
  dEz_dx = stretch(g, in.tab, in.psi, out.psi, 1, 1, 0, i, j, k, dEz_dx);
  dEy_dx = stretch(g, in.tab, in.psi, out.psi, 1, 2, 0, i, j, k, dEy_dx);
  dEx_dy = stretch(g, in.tab, in.psi, out.psi, 1, 2, 1, i, j, k, dEx_dy);
  const T dt = (T)g.dt;
  const T h0 = in.H[0][id] - dt * (dEz_dy - dEy_dz);
  const T h1 = in.H[1][id] - dt * (dEx_dz - dEz_dx);
  const T h2 = in.H[2][id] - dt * (dEy_dx - dEx_dy);
  // streaming stores (as in the fused sweep)
  __builtin_nontemporal_store(h0, &out.H[0][id]);
  __builtin_nontemporal_store(h1, &out.H[1][id]);
  __builtin_nontemporal_store(h2, &out.H[2][id]);
}

// E^{n+1} at cell (i,j,k); H^{n+1/2} is read from `out` (already advanced
// everywhere), E^n from `in`.
template <typename T>
__device__ __forceinline__ void update_e_cell(const FieldPtrs<T>& in, const FieldPtrs<T>& out,
                                              const Geom& g, int i, int j, int k) {
  // products are not contracted into fused multiply-adds, as in the fused sweep,
  // so that every way of splitting the grid between the two rounds alike
#pragma clang fp contract(off)
  const size_t sx = 1, sy = (size_t)g.n[0], sz = (size_t)g.n[0] * g.n[1];
  const size_t id = cell_index(g, i, j, k);
  const T idx = (T)g.inv_dx;
  const T hx = out.H[0][id], hy = out.H[1][id], hz = out.H[2][id];
  T dHz_dy = (hz - bwd(out.H[2], id, j, g.n[1], g.periodic[1], sy)) * idx;
  T dHy_dz = (hy - bwd(out.H[1], id, k, g.n[2], g.periodic[2], sz)) * idx;
  T dHx_dz = (hx - bwd(out.H[0], id, k, g.n[2], g.periodic[2], sz)) * idx;
  T dHz_dx = (hz - bwd(out.H[2], id, i, g.n[0], g.periodic[0], sx)) * idx;
  T dHy_dx = (hy - bwd(out.H[1], id, i, g.n[0], g.periodic[0], sx)) * idx;
  T dHx_dy = (hx - bwd(out.H[0], id, j, g.n[1], g.periodic[1], sy)) * idx;
  dHz_dy = stretch(g, in.tab, in.psi, out.psi, 0, 0, 1, i, j, k, dHz_dy);
  dHy_dz = stretch(g, in.tab, in.psi, out.psi, 0, 0, 2, i, j, k, dHy_dz);
  dHx_dz = stretch(g, in.tab, in.psi, out.psi, 0, 1, 2, i, j, k, dHx_dz);
  dHz_dx = stretch(g, in.tab, in.psi, out.psi, 0, 1, 0, i, j, k, dHz_dx);
  dHy_dx = stretch(g, in.tab, in.psi, out.psi, 0, 2, 0, i, j, k, dHy_dx);
  dHx_dy = stretch(g, in.tab, in.psi, out.psi, 0, 2, 1, i, j, k, dHx_dy);
  const T ce = (T)g.dt * in.epsinv[id];
  const T e0 = in.E[0][id], e1 = in.E[1][id], e2 = in.E[2][id];
  const T cx = dHz_dy - dHy_dz;
  const T cy = dHx_dz - dHz_dx;
  const T cz = dHy_dx - dHx_dy;
  const T n0 = tangential_wall(g, 0, i, j, k) ? T(0) : e0 + ce * cx;
  const T n1 = tangential_wall(g, 1, i, j, k) ? T(0) : e1 + ce * cy;
  const T n2 = tangential_wall(g, 2, i, j, k) ? T(0) : e2 + ce * cz;
  __builtin_nontemporal_store(n0, &out.E[0][id]);
  __builtin_nontemporal_store(n1, &out.E[1][id]);
  __builtin_nontemporal_store(n2, &out.E[2][id]);
}

template <typename T, bool H>
__global__ __launch_bounds__(256) void k_update_box(FieldPtrs<T> in, FieldPtrs<T> out, Geom g,
                                                    Box box) {
  const int i = box.lo[0] + blockIdx.x * blockDim.x + threadIdx.x;
  const int j = box.lo[1] + blockIdx.y * blockDim.y + threadIdx.y;
  const int k = box.lo[2] + blockIdx.z;
  if (i >= box.hi[0] || j >= box.hi[1]) return;
  if (H) update_h_cell(in, out, g, i, j, k);
  else update_e_cell(in, out, g, i, j, k);
}

template <typename T, bool H>
__global__ __launch_bounds__(256) void k_update_shell(FieldPtrs<T> in, FieldPtrs<T> out, Geom g,
                                                      ShellMap m) {
  const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
  if ((long long)t >= m.total) return;
  int i, j, k;
  shell_cell(g, m, t, i, j, k);
  if (H) update_h_cell(in, out, g, i, j, k);
  else update_e_cell(in, out, g, i, j, k);
}

template <typename T, bool H>
__global__ __launch_bounds__(256) void k_update_shell_batch(const ShellJob<T>* jobs,
                                                            const int* start, int njobs) {
  const int jb = find_job(start, njobs, blockIdx.x);
  const ShellJob<T> J = load_job(jobs, jb);
  const unsigned t = (blockIdx.x - start[jb]) * blockDim.x + threadIdx.x;
  if ((long long)t >= J.m.total) return;
  int i, j, k;
  shell_cell(J.g, J.m, t, i, j, k);
  if (H) update_h_cell(J.in, J.out, J.g, i, j, k);
  else update_e_cell(J.in, J.out, J.g, i, j, k);
}

// Soft source currents J at t = (n + 1/2) dt:  E -= (dt/eps_r) J.  One thread per
// cell of each source's support (a plane, or one cell); metallic-wall cells of
// the driven component keep E = 0.
template <typename T>
__device__ __forceinline__ void source_body(const FieldPtrs<T>& f, const Geom& g, const Source& s,
                                            const int64_t* step, int t) {
  int i, j, k;
  double scale;
  if (s.kind == 0) {
    const int u = (s.axis + 1) % 3, v = (s.axis + 2) % 3;
    if (t >= g.n[u] * g.n[v]) return;
    int p[3];
    p[s.axis] = s.index;
    p[u] = t % g.n[u];
    p[v] = t / g.n[u];
    i = p[0];
    j = p[1];
    k = p[2];
    scale = g.inv_dx;
  } else {
    if (t > 0) return;
    i = s.ijk[0];
    j = s.ijk[1];
    k = s.ijk[2];
    scale = g.inv_dx * g.inv_dx * g.inv_dx;
  }
  if (tangential_wall(g, s.comp, i, j, k)) return;
  const double tm = ((double)(*step) + 0.5) * g.dt;
  const size_t id = cell_index(g, i, j, k);
  const double J = pulse_value(s, tm) * scale;
  f.E[s.comp][id] -= (T)((double)g.dt * (double)f.epsinv[id] * J);
}

template <typename T>
__global__ void k_sources(FieldPtrs<T> f, Geom g, SourceSet src, const int64_t* step) {
  const int q = blockIdx.y;
  if (q >= src.count) return;
  source_body(f, g, src.s[q], step, blockIdx.x * blockDim.x + threadIdx.x);
}

template <typename T>
__global__ __launch_bounds__(256) void k_sources_batch(const SourceJob<T>* jobs, const int* start,
                                                       int njobs) {
  const int jb = find_job(start, njobs, blockIdx.x);
  const SourceJob<T>& J = jobs[jb];  // (a copy would put its source array in scratch)
  const int lb = blockIdx.x - start[jb];
  if (lb >= J.nblocks) return;
  const int q = lb / J.bx;
  source_body(J.f, J.g, J.src.s[q], J.step, (lb - q * J.bx) * blockDim.x + threadIdx.x);
}

// Blocks of 256 threads per source of a set (the largest support).
inline int source_blocks(const Geom& g, const SourceSet& src) {
  int maxp = 1;
  for (int q = 0; q < src.count; ++q)
    if (src.s[q].kind == 0) {
      const int u = (src.s[q].axis + 1) % 3, v = (src.s[q].axis + 2) % 3;
      maxp = max(maxp, g.n[u] * g.n[v]);
    }
  return (maxp + 255) / 256;
}

template <typename T>
static hipError_t launch_plain(const FieldPtrs<T>& in, const FieldPtrs<T>& out, const Geom& g,
                               const Box* boxes, int nbox, bool h_pass, bool e_pass,
                               hipStream_t st) {
  dim3 block(64, 4, 1);
  for (int pass = 0; pass < 2; ++pass) {
    if ((pass == 0 && !h_pass) || (pass == 1 && !e_pass)) continue;
    for (int q = 0; q < nbox; ++q) {
      const Box& b = boxes[q];
      const int ex = b.hi[0] - b.lo[0], ey = b.hi[1] - b.lo[1], ez = b.hi[2] - b.lo[2];
      if (ex <= 0 || ey <= 0 || ez <= 0) continue;
      dim3 grid((ex + 63) / 64, (ey + 3) / 4, ez);
      if (pass == 0) hipLaunchKernelGGL((k_update_box<T, true>), grid, block, 0, st, in, out, g, b);
      else hipLaunchKernelGGL((k_update_box<T, false>), grid, block, 0, st, in, out, g, b);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

ShellMap shell_map(const Geom& g, const Box& inner) {
  ShellMap m{};
  m.in = inner;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const int wy = inner.hi[1] - inner.lo[1], wz = inner.hi[2] - inner.lo[2];
  m.nzlo = inner.lo[2];
  m.nslab = (long long)(nz - wz) * nx * ny;
  m.ylo_rows = inner.lo[1];
  m.full_cells = (ny - wy) * nx;
  m.strip = inner.lo[0] + (nx - inner.hi[0]);
  m.per_plane = m.full_cells + wy * m.strip;
  m.total = m.nslab + (long long)wz * m.per_plane;
  m.inv_plane = 1.0 / ((double)nx * ny);
  m.inv_per_plane = m.per_plane > 0 ? 1.0 / m.per_plane : 0.0;
  m.inv_nx = 1.0 / nx;
  m.inv_strip = m.strip > 0 ? 1.0 / m.strip : 0.0;
  return m;
}

int source_blocks_of(const Geom& g, const SourceSet& src) { return source_blocks(g, src); }

template <typename T>
static hipError_t launch_shell(const FieldPtrs<T>& in, const FieldPtrs<T>& out, const Geom& g,
                               const Box& inner, bool h_pass, hipStream_t st) {
  const ShellMap m = shell_map(g, inner);
  if (m.total == 0) return hipSuccess;
  if (m.total >= 0x7fffff00LL) return hipErrorInvalidValue;  // 32-bit cell index
  const long long blocks = (m.total + 255) / 256;
  if (h_pass)
    hipLaunchKernelGGL((k_update_shell<T, true>), dim3((unsigned)blocks), dim3(256), 0, st, in,
                       out, g, m);
  else
    hipLaunchKernelGGL((k_update_shell<T, false>), dim3((unsigned)blocks), dim3(256), 0, st, in,
                       out, g, m);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_sources(const FieldPtrs<T>& f, const Geom& g, const SourceSet& src,
                                 const int64_t* step, hipStream_t st) {
  if (src.count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sources<T>, dim3(source_blocks(g, src), src.count), dim3(256), 0, st, f, g,
                     src, step);
  return hipGetLastError();
}

hipError_t sweep_plain_f64(const FieldPtrs<double>& in, const FieldPtrs<double>& out,
                           const Geom& g, const Box* boxes, int nbox, bool h_pass, bool e_pass,
                           hipStream_t st) {
  return launch_plain<double>(in, out, g, boxes, nbox, h_pass, e_pass, st);
}
hipError_t sweep_plain_f32(const FieldPtrs<float>& in, const FieldPtrs<float>& out, const Geom& g,
                           const Box* boxes, int nbox, bool h_pass, bool e_pass, hipStream_t st) {
  return launch_plain<float>(in, out, g, boxes, nbox, h_pass, e_pass, st);
}
hipError_t sweep_shell_f64(const FieldPtrs<double>& in, const FieldPtrs<double>& out,
                           const Geom& g, const Box& inner, bool h_pass, hipStream_t st) {
  return launch_shell<double>(in, out, g, inner, h_pass, st);
}
hipError_t sweep_shell_f32(const FieldPtrs<float>& in, const FieldPtrs<float>& out, const Geom& g,
                           const Box& inner, bool h_pass, hipStream_t st) {
  return launch_shell<float>(in, out, g, inner, h_pass, st);
}
template <typename T>
static hipError_t launch_shell_batch(const ShellJob<T>* jobs, const int* start, int njobs,
                                     int nblocks, bool h_pass, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  if (h_pass)
    hipLaunchKernelGGL((k_update_shell_batch<T, true>), dim3(nblocks), dim3(256), 0, st, jobs,
                       start, njobs);
  else
    hipLaunchKernelGGL((k_update_shell_batch<T, false>), dim3(nblocks), dim3(256), 0, st, jobs,
                       start, njobs);
  return hipGetLastError();
}
template <typename T>
static hipError_t launch_sources_batch(const SourceJob<T>* jobs, const int* start, int njobs,
                                       int nblocks, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sources_batch<T>, dim3(nblocks), dim3(256), 0, st, jobs, start, njobs);
  return hipGetLastError();
}
hipError_t shell_batch_f64(const ShellJob<double>* jobs, const int* start, int njobs, int nblocks,
                           bool h_pass, hipStream_t st) {
  return launch_shell_batch<double>(jobs, start, njobs, nblocks, h_pass, st);
}
hipError_t shell_batch_f32(const ShellJob<float>* jobs, const int* start, int njobs, int nblocks,
                           bool h_pass, hipStream_t st) {
  return launch_shell_batch<float>(jobs, start, njobs, nblocks, h_pass, st);
}
hipError_t sources_batch_f64(const SourceJob<double>* jobs, const int* start, int njobs,
                             int nblocks, hipStream_t st) {
  return launch_sources_batch<double>(jobs, start, njobs, nblocks, st);
}
hipError_t sources_batch_f32(const SourceJob<float>* jobs, const int* start, int njobs,
                             int nblocks, hipStream_t st) {
  return launch_sources_batch<float>(jobs, start, njobs, nblocks, st);
}
hipError_t sources_f64(const FieldPtrs<double>& f, const Geom& g, const SourceSet& src,
                       const int64_t* step, hipStream_t st) {
  return launch_sources<double>(f, g, src, step, st);
}
hipError_t sources_f32(const FieldPtrs<float>& f, const Geom& g, const SourceSet& src,
                       const int64_t* step, hipStream_t st) {
  return launch_sources<float>(f, g, src, step, st);
}

}  // namespace mlk
