// Internal definitions shared by the HIP sources of libmlk (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mlk {

constexpr int kMaxWin = 12;     // kernel window points per axis (R*sigma <= 5.5 cells)
constexpr int kMaxSources = 8;  // soft sources per simulation
constexpr int kMaxLevels = 6;   // multilevel emitters: 2..6 levels

// Geometry and boundary description passed by value to every grid kernel.
struct Geom {
  int n[3];          // cells per axis
  int nlo[3];        // CPML thickness on the low face (0 if none)
  int nhi[3];        // CPML thickness on the high face
  int periodic[3];   // 1 if the axis wraps
  int wall[3];       // 1 if the low face is metallic (PEC or CPML-backed)
  double dt;
  double inv_dx;
  double dx;
};

__host__ __device__ inline size_t cell_index(const Geom& g, int i, int j, int k) {
  return (size_t)i + (size_t)g.n[0] * ((size_t)j + (size_t)g.n[1] * (size_t)k);
}

// CPML layer membership of index q along axis a (both the integer and the
// half-integer positions of the layers are stored in the same planes).
__host__ __device__ inline bool in_layer(const Geom& g, int a, int q) {
  return q < g.nlo[a] || q >= g.n[a] - g.nhi[a];
}

// Compressed layer index along axis a.
__host__ __device__ inline int layer_index(const Geom& g, int a, int q) {
  return q < g.nlo[a] ? q : q - (g.n[a] - g.nhi[a]) + g.nlo[a];
}

// Index into the psi array of derivative axis a (that axis compressed to its layers).
__host__ __device__ inline size_t psi_index(const Geom& g, int a, int i, int j, int k) {
  int q[3] = {i, j, k};
  int d[3] = {g.n[0], g.n[1], g.n[2]};
  q[a] = layer_index(g, a, q[a]);
  d[a] = g.nlo[a] + g.nhi[a];
  return (size_t)q[0] + (size_t)d[0] * ((size_t)q[1] + (size_t)d[1] * (size_t)q[2]);
}

__host__ __device__ inline size_t psi_size(const Geom& g, int a) {
  size_t s = 1;
  for (int b = 0; b < 3; ++b) s *= (size_t)(b == a ? g.nlo[a] + g.nhi[a] : g.n[b]);
  return s;
}

// Field storage of one precision.
template <typename T>
struct FieldPtrs {
  T* E[3];
  T* H[3];
  const T* epsinv;
  T* psiE[3][3];  // [E component][derivative axis], null when that axis has no CPML
  T* psiH[3][3];
  const T* cb[3][2];  // CPML tables per axis: [0] integer positions, [1] half-integer
  const T* cc[3][2];
  const T* ck[3][2];
};

struct Source {
  int kind;  // 0 plane, 1 point
  int axis, index, comp;
  int ijk[3];
  double amp, omega, tau, t0;
};

struct SourceSet {
  int count;
  Source s[kMaxSources];
};

// Emitter tables (structure of arrays).  Window data per emitter m,
// component c, axis a at [(m*3 + c)*3 + a].
template <typename T>
struct WindowPtrs {
  const int* lo;     // first (unwrapped) index of the window
  const int* len;    // number of points
  const T* w;        // normalised 1-D weights, kMaxWin per (m, c, a)
  const double* gamma;
};

struct TlsPtrs {
  int count;
  const int* gid;          // [M] emitter id of each two-level emitter
  const double* omega0;    // [M]
  const double* dip;       // [3M]
  double* rho;             // [3M] rho11, Re rho01, Im rho01
};

struct MlPtrs {
  int count;
  const int* gid;          // [M] emitter id of each multilevel emitter
  const int* nlev;         // [M]
  const int64_t* eoff;     // energies offset
  const int64_t* moff;     // matrix offset (entries)
  const double* energies;
  const double* mop;
  const double* dip;       // [3M]
  const double* gphi;      // [M]
  double* rho;             // complex n*n interleaved, at 2*moff
};

struct Series {
  double* probe;       // [nprobe][cap]
  int nprobe;
  int probe_comp[16];
  int64_t probe_idx[16];
  int64_t cap;
  double* pop;         // [records][npop]
  int pop_every;
  int64_t npop;
  int64_t pop_cap;     // records
};

struct FluxPlane {
  int on;
  int axis, index;
  double* Eu0;      // saved E_u^n on the plane (FP64)
  double* Ev0;
  double* partial;  // per-block partial sums
  int nblocks;
  double* series;   // [cap]
  double* total;    // running dt * sum F
};

}  // namespace mlk
