// Internal definitions shared by the HIP sources of libmlk (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mlk {

constexpr int kMaxWin = 8;      // kernel window points per axis (R*sigma <= 3.5 cells)
constexpr int kHalo = 4;        // reach of a window beyond its centre cell (R*sigma + 1/2)
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

// XCD-aware order: hardware hands consecutive workgroups to the 8 XCDs in turn;
// map them so that each XCD gets a contiguous range of work items (tiles, bins,
// rows), whose neighbours then meet in the same L2.
__device__ __forceinline__ int xcd_block(int bid, int nblocks) {
  const int q8 = nblocks / 8;
  return bid < 8 * q8 ? (bid % 8) * q8 + bid / 8 : bid;
}

// Workgroup barrier that orders LDS only: global loads in flight (prefetches)
// stay in flight across it, unlike __syncthreads(), whose fence also waits for
// every outstanding global memory operation.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

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

// Field storage of one precision.  All CPML psi arrays of a field buffer live
// in one allocation (see psi_offset) and all CPML coefficient tables in another
// (see tab_offset), so a kernel needs two pointers for them.
template <typename T>
struct FieldPtrs {
  T* E[3];
  T* H[3];
  const T* epsinv;
  T* psi;
  const T* tab;
};

__host__ __device__ inline bool has_cpml(const Geom& g, int a) { return g.nlo[a] + g.nhi[a] > 0; }

// psi arrays: for each axis a with a CPML, in axis order, four arrays of
// psi_size(g, a) values: E of the lower-numbered other component, E of the
// higher, then H of the lower and of the higher.  field: 0 = E, 1 = H.
__host__ __device__ inline size_t psi_offset(const Geom& g, int field, int c, int a) {
  size_t off = 0;
  for (int b = 0; b < a; ++b)
    if (has_cpml(g, b)) off += 4 * psi_size(g, b);
  const int lower = a == 0 ? 1 : 0;
  return off + (size_t)(2 * field + (c == lower ? 0 : 1)) * psi_size(g, a);
}

__host__ __device__ inline size_t psi_total(const Geom& g) {
  size_t t = 0;
  for (int a = 0; a < 3; ++a)
    if (has_cpml(g, a)) t += 4 * psi_size(g, a);
  return t;
}

// CPML tables: for each axis with a CPML, in axis order, b, c and 1/kappa, each
// at the n integer positions then the n half-integer positions.
__host__ __device__ inline size_t tab_offset(const Geom& g, int a) {
  size_t off = 0;
  for (int b = 0; b < a; ++b)
    if (has_cpml(g, b)) off += 6 * (size_t)g.n[b];
  return off;
}

__host__ __device__ inline size_t tab_total(const Geom& g) {
  size_t t = 0;
  for (int a = 0; a < 3; ++a)
    if (has_cpml(g, a)) t += 6 * (size_t)g.n[a];
  return t;
}

// Half-open box of cells [lo, hi) per axis.
struct Box {
  int lo[3];
  int hi[3];
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

// Kernel windows of the emitters.  For emitter m, axis a and position variant v
// (v = 0: integer positions, v = 1: half-integer positions; component c uses
// v = 1 on its own axis and v = 0 on the others), slot q = m*6 + 2a + v holds
// the first (unwrapped) index lo[q], the length len[q] <= kMaxWin and the
// normalised 1-D weights w[q*kMaxWin ...].
// The same window in the form the binned kernels stage in LDS.  Per axis the
// union of the two position variants starts at org[a] and spans n[a] <= kMaxWin
// points (the integer points of [r - R sigma - 1/2, r + R sigma]); wr[a][v][d] is
// the weight of variant v at point org[a] + d, zero outside that variant's
// window, so loops over the union need no bounds checks.
template <typename T>
struct alignas(16) WinRec {
  int org[3];
  int n[3];
  float wmax;  // largest 3-D weight of any component's window
  int pad;
  T wr[3][2][kMaxWin];
};

template <typename T>
struct WindowPtrs {
  const int* lo;
  const int* len;
  const T* w;
  const double* gamma;
  const WinRec<T>* rec;  // [M]
};

__host__ __device__ inline int win_slot(int m, int a, int v) { return m * 6 + 2 * a + v; }


struct TlsPtrs {
  int count;
  const int* gid;          // [M] emitter id of each two-level emitter
  const double* omega0;    // [M]
  const double* dip;       // [3M]
  double* rho;             // [3M] rho11, Re rho01, Im rho01
};

// Multilevel emitters on the device, structure-of-arrays over the slots
// (slot = entry index; slots are grouped by level count).  Matrices sit in a
// kMaxLevels x kMaxLevels frame: entry (a, b) of slot m is at
// (a * kMaxLevels + b) * count + m (complex: re at 2q, im at 2q + 1).
struct MlDev {
  int count;
  const int* gid;       // [count] emitter id
  const double* en;     // [kMaxLevels][count] H0 eigenvalues
  const double* M;      // [kMaxLevels^2][count] real symmetric
  const double* dip;    // [3][count]
  const double* gphi;   // [count]
  double* rho;          // [2 kMaxLevels^2][count]
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
  // non-finite watchdog: 0 while every checked value is finite, else 1 + the first
  // step at which an emitter state, dipole rate, probe sample or flux value was not
  unsigned long long* numeric;
};

// Record step n as the first non-finite one (the earliest record wins the race only
// within a launch; launches run in step order, so the first launch to set it wins).
__device__ __forceinline__ void flag_nonfinite(const Series& ser, int64_t n) {
  if (ser.numeric) atomicCAS(ser.numeric, 0ull, (unsigned long long)n + 1ull);
}

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

// Travelling pulse of the classical-path mode: amp f(t - (z - z0)) pol.
struct WaveDesc {
  double pol[3];
  double amp, omega, tau, t0, z0;
};

// Discrete field energy W^n, recorded every `every` steps (0: off).
struct EnergyRec {
  int every;
  double* partial;  // per-block partial sums (FP64)
  int nblocks;
  double* series;   // [records]
  double dv;        // cell volume dx^3
};

// One Lorentz or Drude pole over a cell box: P^{n+1} (1 + g) = a P^n - b P^{n-1} + c E^n.
struct PoleDev {
  int lo[3], n[3];    // box origin and extent (cells)
  double a, b, c, g1; // 2 - kappa w0^2 dt^2, 1 - g, sigma w0^2 dt^2, 1 + g (g = gamma dt / 2)
  void* P;            // P^n, 3 x box cells of the field type, component-major, x fastest
  void* Q;            // P^n - P^{n-1}; after the pre-sweep pass P^{n+1} - P^n
};

// Single-mode cavity that replaces the grid: mode state and coupling.
struct CavityDev {
  double* st;       // q_x, q_y, p_x, p_y, d_x, d_y (FP64)
  double* partial;  // per-block partial sums of mu_dot_x, mu_dot_y
  double w, V, eps; // mode frequency, effective volume, eps = w / sqrt(V)
};
// Two-level-only cavity step: one block of kTlsThreads slots per partial sum.
constexpr int kTlsThreads = 256;
inline int cavity_tls_blocks(int ntls) { return (ntls + kTlsThreads - 1) / kTlsThreads; }

// Cell (index along axis a; iu, iv along the two others in cyclic order) of a plane.
__device__ __forceinline__ size_t plane_cell(const Geom& g, int a, int index, int iu, int iv) {
  const int u = (a + 1) % 3, v = (a + 2) % 3;
  int q[3];
  q[a] = index;
  q[u] = iu;
  q[v] = iv;
  return cell_index(g, q[0], q[1], q[2]);
}

// Saves E_u^n, E_v^n of plane cell t (the flux needs E^n after the sweep).
template <typename T>
__device__ __forceinline__ void flux_save_body(const FieldPtrs<T>& f, const Geom& g,
                                               const FluxPlane& fp, int t) {
  const int a = fp.axis, u = (a + 1) % 3, v = (a + 2) % 3;
  const int nu = g.n[u], nv = g.n[v];
  if (t >= nu * nv) return;
  const int iu = t % nu, iv = t / nu;
  const size_t id = plane_cell(g, a, fp.index, iu, iv);
  fp.Eu0[t] = (double)f.E[u][id];
  fp.Ev0[t] = (double)f.E[v][id];
}

// Partial flux of block b of nb: 256 threads a block, grid-stride over the plane,
// summed in FP64 in red (256 doubles of LDS) in a fixed order, so the partials do not
// depend on the launch that forms them.  Threads from 256 on (a larger block) only
// take part in the barriers.
template <typename T>
__device__ __forceinline__ void flux_partial_sum(const FieldPtrs<T>& f, const Geom& g,
                                                 const FluxPlane& fp, int b, int nb,
                                                 double* red) {
  const int a = fp.axis, u = (a + 1) % 3, v = (a + 2) % 3;
  const int nu = g.n[u], nv = g.n[v];
  const int tid = threadIdx.x;
  if (tid < 256) {
    double s = 0.0;
    for (int t = b * 256 + tid; t < nu * nv; t += nb * 256) {
      const int iu = t % nu, iv = t / nu;
      const size_t id = plane_cell(g, a, fp.index, iu, iv);
      const size_t jd = plane_cell(g, a, fp.index - 1, iu, iv);
      const double Eu = 0.5 * (fp.Eu0[t] + (double)f.E[u][id]);
      const double Ev = 0.5 * (fp.Ev0[t] + (double)f.E[v][id]);
      const double Hv = 0.5 * ((double)f.H[v][id] + (double)f.H[v][jd]);
      const double Hu = 0.5 * ((double)f.H[u][id] + (double)f.H[u][jd]);
      s += Eu * Hv - Ev * Hu;
    }
    red[tid] = s;
  }
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) fp.partial[b] = red[0];
}


// Binned emitter phase.
// Gather bins: every emitter belongs to the bin of its centre cell; the
// workgroup of a bin stages the bin plus a halo of kHalo cells.
// Scatter bins: every (bin, emitter) pair whose window touches the bin.
// Gather bins of at most a few emitters ("light" bins) come after the others and
// stage only the part of their tile that their windows cover.
struct BinPtrs {
  int nbx, nby, nbz;        // scatter bins per axis
  int ngather;              // gather bins holding at least one centre
  int gdense;               // bins [0, gdense) stage the whole tile, the rest are light
  int glight0, nlight;      // gbin_em[glight0 .. glight0 + nlight): the light bins' emitters
  const int* gbin_org;      // [3*ngather] bin origin in unwrapped cells (centre-cell frame)
  const int* gbin_start;    // [ngather+1] CSR into gbin_em
  const int* gbin_em;       // emitter ids
  int nscatter;             // scatter bins touched by at least one window
  const int* sbin_id;       // [nscatter]
  const int* sbin_start;    // [nscatter+1] CSR into sbin_pair
  const int4* sbin_pair;    // one PairDesc per (emitter, bin) pair
};

// A batch kernel's job, read from its table through the constant address space.
// The tables are written before the launch and only read by kernels, and pointers
// read from constant memory are known to point to global memory, so the kernel
// reaches the fields through global instructions.  Read from an ordinary pointer,
// the job's pointers would be generic: the compiler would emit flat instructions,
// which also count against the LDS and scalar wait counter.  (The host pass only
// parses kernels; it reads the table directly.)
template <typename J>
__device__ __forceinline__ J load_job(const J* jobs, int j) {
#if defined(__HIP_DEVICE_COMPILE__)
  return ((__attribute__((address_space(4))) const J*)jobs)[j];
#else
  return jobs[j];
#endif
}

// A scatter pair: emitter e and, per axis a, the run of its union window inside
// the bin: window offsets d0 .. d0+c-1 on the bin-local cells l0 .. l0+c-1, packed
// as l0 | d0 << 4 | (c-1) << 7 at bit 10a of runs.  gw = |gamma| times the
// record's wmax, rounded up to FP32 (the per-bin bound of the fixed-point grid).
struct PairDesc {
  int e;
  unsigned runs;
  float gw;
  int pad;
};
static_assert(sizeof(PairDesc) == 16, "a pair is loaded as one int4");
inline unsigned pack_run(int l0, int d0, int c) {
  return (unsigned)l0 | (unsigned)d0 << 4 | (unsigned)(c - 1) << 7;
}

// ---------------------------------------------------------------- batches
// A batched launch covers the jobs of several domains: job j owns blocks
// [start[j], start[j+1]) of the grid; starts are multiples of 8 so that the
// XCD-aware block order of a job is preserved.
__device__ inline int find_job(const int* start, int njobs, int b) {
  int lo = 0, hi = njobs;  // start[lo] <= b < start[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (start[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <typename T>
struct FusedJob {
  FieldPtrs<T> a, b;
  Geom g;
  Box box;
  int kz, tx, ty, ntx, nty, nblocks;  // planes per chunk, tile width and rows, tile grid
};

// Up to four boxes of one sim swept by one launch of the full fused kernel (the
// layer frame around an interior box), passed by value.
template <typename T>
struct FrameJobs {
  FusedJob<T> job[4];
  int start[5];
  int njobs;
};

// The cells of the grid outside an interior box, enumerated in memory order:
// the whole planes below and above the box in z, then, plane by plane inside
// it, the whole rows below and above it in y followed by the two x strips of
// each remaining row.
struct ShellMap {
  Box in;
  int nzlo;              // whole planes below the box
  long long nslab;       // cells in the whole planes (both sides)
  int ylo_rows;          // whole rows below the box, per middle plane
  int full_cells;        // cells in the whole rows of one middle plane
  int strip;             // cells in the two x strips of one row
  int per_plane;         // shell cells of one middle plane
  long long total;       // below 2^31 (checked at launch)
  // reciprocals for the index arithmetic (exact after one correction step)
  double inv_plane, inv_per_plane, inv_nx, inv_strip;
};

// n / d for n < 2^31 from a rounded reciprocal of d: the quotient estimate is off
// by at most one, which the remainder test corrects.
__device__ __forceinline__ unsigned div_by(unsigned n, unsigned d, double inv) {
  unsigned q = (unsigned)((double)n * inv);
  const int r = (int)(n - q * d);
  q = q + (r >= (int)d ? 1u : 0u) - (r < 0 ? 1u : 0u);
  return q;
}

template <typename T>
struct ShellJob {
  FieldPtrs<T> in, out;
  Geom g;
  ShellMap m;
  int nblocks;
};

template <typename T>
struct SourceJob {
  FieldPtrs<T> f;
  Geom g;
  SourceSet src;
  const int64_t* step;
  int bx;       // blocks per source
  int nblocks;  // bx * src.count
};

// The light bins' emitters of one domain, gathered without a tile.
template <typename T>
struct LightJob {
  FieldPtrs<T> f;
  Geom g;
  const int* em;
  int count;
  WindowPtrs<T> win;
  double* Et;
  int nblocks;
};

template <typename T>
struct GatherJob {
  FieldPtrs<T> f;
  Geom g;
  BinPtrs bins;
  WindowPtrs<T> win;
  double* Et;
  int nblocks;  // bins.gdense (the light bins go to LightJob)
};

struct TlsJob {
  TlsPtrs tls;
  double dt;
  const double* Et;
  double* mudot;
  const int64_t* pop_off;
  Series ser;
  const int64_t* step;
  int nblocks;
};

struct MlJob {
  MlDev ml;
  int first, count;  // slots of one level count
  double dt;
  const double* Et;
  double* mudot;
  const int64_t* pop_off;
  Series ser;
  const int64_t* step;
  int nblocks;
};

template <typename T>
struct ScatterJob {
  FieldPtrs<T> f;
  Geom g;
  BinPtrs bins;
  WindowPtrs<T> win;
  const double* mudot;
  int nblocks;  // bins.nscatter
};

template <typename T>
struct FluxJob {
  FieldPtrs<T> f;
  Geom g;
  FluxPlane fp;
  Series ser;
  int64_t* step;
  int nblocks;
};

// Adjoint fields of one sweep: adjoints of E and H, the forward's 1/eps and
// CPML tables, and the adjoint of psi double-buffered (read psi[0], write psi[1]).
template <typename T>
struct AdjSweep {
  T* E[3];
  T* H[3];
  const T* epsinv;
  const T* tab;
  T* psi[2];
  // out of place (fused transposed sweep plus shell passes): the updated
  // adjoint fields go here; null: whole-grid update in place
  T* Eo[3];
  T* Ho[3];
  int kz;  // z planes per workgroup of the fused transposed sweep
  int vacuum;  // eps_r = 1 everywhere: the fused transposed sweep reads no 1/eps_r
};

}  // namespace mlk
