// libmlk runtime: the C ABI declared in include/mlk.h.
//
// Owns the device state of one simulation, validates inputs, and enqueues
// the per-step kernel sequence on the simulation's stream:
//   [flux: save E^n on the plane] -> emitter gather + step + dipole rate
//   -> Yee sweep (H then E, with soft sources) -> current scatter
//   -> [flux partial sums] -> finish (probes, flux total, step counter).
// Every numerical step runs in the HIP kernels; this file only moves data
// and checks arguments.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <climits>
#include <cstdint>
#include <algorithm>
#include <string>
#include <array>
#include <vector>
#include <mutex>

#include "launch.h"
#include "mlk.h"

using namespace mlk;

namespace {

thread_local std::string g_err;

mlk_status fail(mlk_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(e_ == hipErrorOutOfMemory ? MLK_ENOMEM : MLK_EDEVICE, "%s: %s", #expr, \
                  hipGetErrorString(e_));                                              \
  } while (0)

#define STCHK(expr)                   \
  do {                                \
    mlk_status s_ = (expr);           \
    if (s_ != MLK_OK) return s_;      \
  } while (0)

template <typename P>
hipError_t dalloc(P** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) return hipSuccess;
  return hipMalloc((void**)p, bytes);
}

template <typename P>
void dfree(P*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

// Device buffer owned by a scope.
template <typename T>
struct DevBuf {
  T* p = nullptr;
  ~DevBuf() { dfree(p); }
  hipError_t alloc(size_t n) {
    dfree(p);
    if (n == 0) return hipSuccess;
    return dalloc(&p, n * sizeof(T));
  }
};

}  // namespace

struct mlk_sim {
  mlk_grid_desc desc{};
  // phase timing: event pool, pending (phase, start event, end event) marks
  int timing = 0;  // bit p set: phase p is timed
  std::vector<hipEvent_t> events;
  size_t next_event = 0;
  std::vector<std::array<int, 3>> marks;
  double phase_ms[MLK_PHASE_COUNT] = {};
  int64_t phase_n[MLK_PHASE_COUNT] = {};
  Geom g{};
  bool fp32 = false;
  size_t esz = 8;
  size_t ncell = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;

  void* E[3] = {};  // current fields
  void* H[3] = {};
  void* E2[3] = {};  // second buffers of the fused sweep (swapped every step)
  void* H2[3] = {};
  void* psi2 = nullptr;
  // the two field sets of the fused sweep have swapped an odd number of times: the
  // current fields are in set 1 (set 0 is the one E[] held at creation)
  bool swapped = false;
  // device buffers the caller owns (mlk_bind_device_buffers): never freed here
  std::vector<const void*> borrowed;
  bool states_bound = false;
  int kz = 0;       // z planes per workgroup of the fused sweep
  int ty = 4;       // y rows per workgroup of the fused sweep (4, 8 or 16)
  int tx = 64;      // x cells per workgroup of the fused sweep (64 or 32)
  int layer_mode = 0;  // y/z CPML layers: 0 shell passes, 1 in the fused kernel, 2 frame launch
  bool vacuum = true;   // eps_r = 1 in every cell: the fused sweep reads no 1/eps_r
  hipStream_t batch_stream = nullptr;  // stream of the batch this sim belongs to
  bool in_batch = false;
  double adj_forward_ms = 0.0, adj_reverse_ms = 0.0;  // phases of the last adjoint call
  void* epsinv = nullptr;
  void* psi = nullptr;  // every CPML psi array of the current buffer (psi_offset layout)
  void* tab = nullptr;  // CPML coefficient tables (tab_offset layout)

  // emitters, host mirror (by emitter id)
  int nem = 0;
  std::vector<double> pos, sigma, gamma;
  std::vector<int64_t> pop_off;
  int64_t npop = 0;
  std::vector<int> tls_gid;
  std::vector<int> tls_slot;  // by emitter id: index among two-level emitters, or -1
  std::vector<double> tls_w0, tls_dip, tls_rho0;
  // multilevel emitters, host mirror in add order (matrices in a kMaxLevels frame)
  std::vector<int> ml_gid, ml_nlev;
  std::vector<double> ml_en, ml_M, ml_dip, ml_gphi, ml_rho0;  // 6, 36, 3, 1, 72 per emitter
  std::vector<int> ml_slot;   // by emitter id: device slot among multilevel emitters, or -1
  int ml_range[kMaxLevels + 2] = {};  // device slots with n levels: ml_range[n]..ml_range[n+1]
  int* d_ml_gid = nullptr;
  double* d_ml_en = nullptr;
  double* d_ml_M = nullptr;
  double* d_ml_dip = nullptr;
  double* d_ml_gphi = nullptr;
  double* d_ml_rho = nullptr;
  // device emitter tables
  int* d_wlo = nullptr;
  int* d_wlen = nullptr;
  void* d_w = nullptr;
  void* d_rec = nullptr;  // WinRec<T>[M]
  double* d_pos = nullptr;
  double* d_sigma = nullptr;
  double* d_gamma = nullptr;
  double* d_Et = nullptr;
  double* d_mudot = nullptr;
  int64_t* d_popoff = nullptr;
  int* d_tls_gid = nullptr;
  double* d_tls_w0 = nullptr;
  double* d_tls_dip = nullptr;
  double* d_tls_rho = nullptr;
  // binned emitter phase
  int nbx = 0, nby = 0, nbz = 0;
  int ngather = 0, nscatter = 0, gdense = 0, glight0 = 0, nlight = 0;
  // estimated work of each gather / scatter launch block (host; orders a batch's blocks)
  std::vector<float> gwork, swork;
  // per axis, the planes that some emitter's union window reaches (the cells the
  // scatter may change)
  std::vector<unsigned char> wplane[3];
  int* d_gbin_org = nullptr;
  int* d_gbin_start = nullptr;
  int* d_gbin_em = nullptr;
  int* d_sbin_id = nullptr;
  int* d_sbin_start = nullptr;
  PairDesc* d_sbin_pair = nullptr;
  int* d_tls_slot = nullptr;

  SourceSet src{};

  int nprobe = 0;
  int probe_comp[16] = {};
  int64_t probe_idx[16] = {};
  double* d_probe = nullptr;
  int64_t series_cap = 0;

  FluxPlane fp{};
  double* d_flux_series = nullptr;

  int pop_every = 0;
  double* d_pop = nullptr;
  int64_t pop_cap = 0;

  EnergyRec er{};          // discrete field energy detector (off: er.every == 0)
  int64_t energy_cap = 0;  // records

  int64_t* d_step = nullptr;
  int64_t host_step = 0;
  // non-finite watchdog (see Series::numeric)
  unsigned long long* d_numeric = nullptr;

  // single-mode cavity in place of the grid (off unless mlk_set_cavity was called)
  bool cav_on = false;
  CavityDev cav{};

  // dispersive poles (Lorentz / Drude over cell boxes), in add order
  int npole = 0;
  PoleDev pole[8] = {};
};

namespace {

// Wait for every piece of work on the sim: its own stream and, while it is a
// member of a batch, the batch's stream.
mlk_status sync_sim(mlk_sim* s) {
  HIPCHK(hipStreamSynchronize(s->stream));
  if (s->batch_stream) HIPCHK(hipStreamSynchronize(s->batch_stream));
  return MLK_OK;
}


template <typename T>
FieldPtrs<T> field_ptrs(const mlk_sim* s);

template <typename T>
FieldPtrs<T> spare_ptrs(const mlk_sim* s) {
  FieldPtrs<T> f = field_ptrs<T>(s);
  for (int c = 0; c < 3; ++c) {
    f.E[c] = (T*)s->E2[c];
    f.H[c] = (T*)s->H2[c];
  }
  f.psi = (T*)s->psi2;
  return f;
}

void swap_buffers(mlk_sim* s) {
  for (int c = 0; c < 3; ++c) {
    std::swap(s->E[c], s->E2[c]);
    std::swap(s->H[c], s->H2[c]);
  }
  std::swap(s->psi, s->psi2);
  s->swapped = !s->swapped;
}

template <typename T>
FieldPtrs<T> field_ptrs(const mlk_sim* s) {
  FieldPtrs<T> f{};
  for (int c = 0; c < 3; ++c) {
    f.E[c] = (T*)s->E[c];
    f.H[c] = (T*)s->H[c];
  }
  f.epsinv = (const T*)s->epsinv;
  f.psi = (T*)s->psi;
  f.tab = (const T*)s->tab;
  return f;
}

template <typename T>
WindowPtrs<T> window_ptrs(const mlk_sim* s) {
  WindowPtrs<T> w{};
  w.lo = s->d_wlo;
  w.len = s->d_wlen;
  w.w = (const T*)s->d_w;
  w.gamma = s->d_gamma;
  w.rec = (const WinRec<T>*)s->d_rec;
  return w;
}

TlsPtrs tls_ptrs(const mlk_sim* s) {
  TlsPtrs tls{};
  tls.count = (int)s->tls_gid.size();
  tls.gid = s->d_tls_gid;
  tls.omega0 = s->d_tls_w0;
  tls.dip = s->d_tls_dip;
  tls.rho = s->d_tls_rho;
  return tls;
}

Series series_of(const mlk_sim* s) {
  Series ser{};
  ser.probe = s->d_probe;
  ser.nprobe = s->nprobe;
  for (int p = 0; p < s->nprobe; ++p) {
    ser.probe_comp[p] = s->probe_comp[p];
    ser.probe_idx[p] = s->probe_idx[p];
  }
  ser.cap = s->series_cap;
  ser.pop = s->d_pop;
  ser.pop_every = s->pop_every;
  ser.npop = s->npop;
  ser.pop_cap = s->pop_cap;
  ser.numeric = s->d_numeric;
  return ser;
}

// The watchdog's record after the sim's work is done (0: every checked value finite).
mlk_status read_numeric(mlk_sim* s, unsigned long long* v) {
  STCHK(sync_sim(s));
  HIPCHK(hipMemcpy(v, s->d_numeric, sizeof(*v), hipMemcpyDeviceToHost));
  return MLK_OK;
}

mlk_status check_numeric(mlk_sim* s) {
  unsigned long long v = 0;
  STCHK(read_numeric(s, &v));
  if (v)
    return fail(MLK_ENUMERIC,
                "non-finite state: an emitter state, dipole rate, probe sample or flux value "
                "was not finite at step %llu",
                v - 1);
  return MLK_OK;
}

bool in_range_face(const mlk_sim* s, int a, double x, double reach) {
  const Geom& g = s->g;
  if (g.periodic[a]) return true;
  const double lo = (double)g.nlo[a];
  const double hi = (double)(g.n[a] - g.nhi[a]);
  return x - reach >= lo && x + reach <= hi;
}

// Checks shared by every emitter kind: width, window size and distance to walls.
mlk_status check_emitter_geometry(const mlk_sim* s, const double* p, double sig) {
  if (!(sig > 0.0) || !std::isfinite(sig)) return fail(MLK_EINVAL, "sigma must be > 0");
  const double rs = s->desc.window_r * sig;
  if (rs < 0.5) return fail(MLK_EINVAL, "kernel window R*sigma = %.3f is below half a cell", rs);
  if (2.0 * rs + 1.0 > (double)kMaxWin)
    return fail(MLK_EUNSUPPORTED, "kernel window %.2f cells exceeds %d points per axis",
                2.0 * rs + 1.0, kMaxWin);
  for (int a = 0; a < 3; ++a) {
    if (!std::isfinite(p[a])) return fail(MLK_EINVAL, "emitter position not finite");
    if (s->g.periodic[a]) {
      if (s->g.n[a] > 1 && (double)s->g.n[a] < 2.0 * rs + 2.0)
        return fail(MLK_EINVAL, "periodic axis %d too short for the kernel window", a);
      if (p[a] < 0.0 || p[a] > (double)s->g.n[a])
        return fail(MLK_EINVAL, "emitter outside the domain on axis %d", a);
    } else if (!in_range_face(s, a, p[a], rs + 1.0)) {
      return fail(MLK_EINVAL,
                  "emitter at %.3f on axis %d: kernel window reaches a wall or the CPML", p[a],
                  a);
    }
  }
  return MLK_OK;
}

template <typename T>
mlk_status upload(T** dptr, const std::vector<T>& v) {
  dfree(*dptr);
  if (v.empty()) return MLK_OK;
  HIPCHK(dalloc(dptr, v.size() * sizeof(T)));
  HIPCHK(hipMemcpy(*dptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return MLK_OK;
}

BinPtrs bin_ptrs(const mlk_sim* s) {
  BinPtrs b{};
  b.nbx = s->nbx;
  b.nby = s->nby;
  b.nbz = s->nbz;
  b.ngather = s->ngather;
  b.gdense = s->gdense;
  b.glight0 = s->glight0;
  b.nlight = s->nlight;
  b.gbin_org = s->d_gbin_org;
  b.gbin_start = s->d_gbin_start;
  b.gbin_em = s->d_gbin_em;
  b.nscatter = s->nscatter;
  b.sbin_id = s->d_sbin_id;
  b.sbin_start = s->d_sbin_start;
  b.sbin_pair = reinterpret_cast<const int4*>(s->d_sbin_pair);
  return b;
}

// Union windows of the emitters as the binned kernels see them: origin and
// length per axis and the largest 3-D weight, read back from the records.
template <typename T>
mlk_status read_unions(const mlk_sim* s, std::vector<int>& org, std::vector<int>& n,
                       std::vector<double>& wmax) {
  std::vector<WinRec<T>> rec(s->nem);
  if (s->nem > 0)
    HIPCHK(hipMemcpy(rec.data(), s->d_rec, rec.size() * sizeof(WinRec<T>),
                     hipMemcpyDeviceToHost));
  for (int e = 0; e < s->nem; ++e) {
    for (int a = 0; a < 3; ++a) {
      org[3 * e + a] = rec[e].org[a];
      n[3 * e + a] = rec[e].n[a];
    }
    wmax[e] = rec[e].wmax;
  }
  return MLK_OK;
}

// Emitter bins (index bookkeeping only).  Gather bins group emitters by the
// bin of their centre cell; scatter bins list, for every bin, the emitters
// whose windows (as computed on the device) touch it.
mlk_status build_bins(mlk_sim* s) {
  const Geom& g = s->g;
  int G[3], B[3];
  bin_shape(s->fp32, G, B);
  int nb[3];
  for (int a = 0; a < 3; ++a) nb[a] = (g.n[a] + B[a] - 1) / B[a];
  s->nbx = nb[0];
  s->nby = nb[1];
  s->nbz = nb[2];
  const int M = s->nem;

  // gather: key = bin of the (unwrapped) centre cell
  struct Key {
    int b[3];
    int e;
  };
  std::vector<Key> keys(M);
  for (int e = 0; e < M; ++e) {
    keys[e].e = e;
    for (int a = 0; a < 3; ++a) {
      const int c = (int)std::floor(s->pos[3 * e + a]);
      keys[e].b[a] = (c >= 0 ? c : c - G[a] + 1) / G[a];
    }
  }
  std::stable_sort(keys.begin(), keys.end(), [](const Key& x, const Key& y) {
    if (x.b[2] != y.b[2]) return x.b[2] < y.b[2];
    if (x.b[1] != y.b[1]) return x.b[1] < y.b[1];
    return x.b[0] < y.b[0];
  });
  std::vector<int> gorg, gstart, gem;
  for (int q = 0; q < M; ++q) {
    if (q == 0 || keys[q].b[0] != keys[q - 1].b[0] || keys[q].b[1] != keys[q - 1].b[1] ||
        keys[q].b[2] != keys[q - 1].b[2]) {
      gstart.push_back(q);
      for (int a = 0; a < 3; ++a) gorg.push_back(keys[q].b[a] * G[a]);
    }
    gem.push_back(keys[q].e);
  }
  gstart.push_back(M);
  {
    // light bins (at most gather_light_max() emitters) after the others, keeping the
    // order within each kind: the heavier bins are dispatched first
    const int light_max = gather_light_max();
    const int nbin = (int)gstart.size() - 1;
    std::vector<int> org2, start2, em2;
    for (int pass = 0; pass < 2; ++pass) {
      for (int b = 0; b < nbin; ++b) {
        const bool light = gstart[b + 1] - gstart[b] <= light_max;
        if (light != (pass == 1)) continue;
        start2.push_back((int)em2.size());
        for (int a = 0; a < 3; ++a) org2.push_back(gorg[3 * b + a]);
        for (int q = gstart[b]; q < gstart[b + 1]; ++q) em2.push_back(gem[q]);
      }
      if (pass == 0) s->gdense = (int)start2.size();
    }
    start2.push_back((int)em2.size());
    gorg.swap(org2);
    gstart.swap(start2);
    gem.swap(em2);
    s->ngather = nbin;
    // the light bins' emitters, one run of gem (the forward gather serves them
    // without a tile)
    s->glight0 = gstart[s->gdense];
    s->nlight = M - s->glight0;
    // work of launch block q of the staged bins (taken through the kernel's XCD
    // order): its emitter count
    const int nd = s->gdense, q8 = nd / 8;
    s->gwork.assign(nd, 0.f);
    for (int q = 0; q < nd; ++q) {
      const int bin = q < 8 * q8 ? (q % 8) * q8 + q / 8 : q;
      s->gwork[q] = (float)(gstart[bin + 1] - gstart[bin]);
    }
  }

  // scatter: the union window of each emitter (org, n per axis, as in its
  // record) split, per axis, into runs inside one bin: consecutive window
  // offsets on consecutive cells.  A pair is one run per axis; a window wraps
  // inside a bin only on a periodic axis no longer than the bin, where it gives
  // two runs.
  std::vector<int> worg((size_t)M * 3), wn((size_t)M * 3);
  std::vector<double> wmax(M);
  if (s->fp32)
    STCHK(read_unions<float>(s, worg, wn, wmax));
  else
    STCHK(read_unions<double>(s, worg, wn, wmax));
  for (int a = 0; a < 3; ++a) {
    const int n = g.n[a];
    s->wplane[a].assign(n, 0);
    for (int e = 0; e < M; ++e)
      for (int d = 0; d < wn[3 * e + a]; ++d) {
        int q = worg[3 * e + a] + d;
        if (g.periodic[a]) q = ((q % n) + n) % n;
        if (q >= 0 && q < n) s->wplane[a][q] = 1;
      }
  }
  // FP32 gather: the eight emitters of a wavefront read their window rows from the
  // staged tile at the same row and plane offsets, so lane i of emitter m reads word
  // s_m + i + (a common offset), and emitters whose windows start in the same LDS
  // banks conflict.  The bank of s_m is (x offset + tile width x y offset) mod 64 (the
  // tile's plane stride is a multiple of 64 words).  Within a staged bin, the
  // emitters are sorted by that bank and dealt to the wavefronts with a stride, so
  // those of one wavefront (and of each half) start in banks spread around the 64.
  // Only the assignment of emitters to lanes changes, not any result.
  if (s->fp32) {
    const int TXg = G[0] + 2 * kHalo;
    std::vector<std::pair<int, int>> v;
    for (int b = 0; b < s->gdense; ++b) {
      const int q0 = gstart[b], q1 = gstart[b + 1], n = q1 - q0;
      const int x0 = gorg[3 * b] - kHalo, y0 = gorg[3 * b + 1] - kHalo;
      v.clear();
      for (int q = q0; q < q1; ++q) {
        const int e = gem[q];
        v.push_back({((worg[3 * e] - x0) + TXg * (worg[3 * e + 1] - y0)) & 63, e});
      }
      std::stable_sort(v.begin(), v.end(), [](const std::pair<int, int>& x,
                                              const std::pair<int, int>& y) {
        return x.first < y.first;
      });
      const int nw = (n + 7) / 8;
      int q = q0;
      for (int w = 0; w < nw; ++w)
        for (int k = 0; k < 8; ++k)
          if (w + k * nw < n) gem[q++] = v[w + k * nw].second;
    }
  }
  struct Run {
    int bin, l0, d0, c;
  };
  auto runs_of = [&](int e, int a, std::vector<Run>& out) {
    out.clear();
    for (int d = 0; d < wn[3 * e + a]; ++d) {
      int w = (worg[3 * e + a] + d) % g.n[a];
      if (w < 0) w += g.n[a];
      const int bq = w / B[a], l = w - bq * B[a];
      if (!out.empty()) {
        Run& r = out.back();
        if (r.bin == bq && r.d0 + r.c == d && r.l0 + r.c == l) {
          ++r.c;
          continue;
        }
      }
      out.push_back({bq, l, d, 1});
    }
  };
  const size_t nball = (size_t)nb[0] * nb[1] * nb[2];
  std::vector<std::vector<std::pair<int, PairDesc>>> per_em(M);  // (bin, pair)
  std::vector<Run> rx, ry, rz;
  for (int e = 0; e < M; ++e) {
    runs_of(e, 0, rx);
    runs_of(e, 1, ry);
    runs_of(e, 2, rz);
    float gw = (float)(std::fabs(s->gamma[e]) * wmax[e]);
    if ((double)gw < std::fabs(s->gamma[e]) * wmax[e]) gw = std::nextafter(gw, INFINITY);
    for (const Run& z : rz)
      for (const Run& y : ry)
        for (const Run& x : rx) {
          PairDesc pd;
          pd.e = e;
          pd.runs = pack_run(x.l0, x.d0, x.c) | pack_run(y.l0, y.d0, y.c) << 10 |
                    pack_run(z.l0, z.d0, z.c) << 20;
          pd.gw = gw;
          pd.pad = 0;
          per_em[e].push_back({x.bin + nb[0] * (y.bin + nb[1] * z.bin), pd});
        }
  }
  std::vector<int> count(nball, 0);
  size_t npairs = 0;
  for (int e = 0; e < M; ++e)
    for (const auto& bp : per_em[e]) {
      ++count[bp.first];
      ++npairs;
    }
  if (npairs > (size_t)INT32_MAX) return fail(MLK_EUNSUPPORTED, "too many emitter-bin pairs");
  std::vector<int> sid, sstart(1, 0), slot_of(nball, -1);
  for (size_t b = 0; b < nball; ++b)
    if (count[b]) {
      slot_of[b] = (int)sid.size();
      sid.push_back((int)b);
      sstart.push_back(sstart.back() + count[b]);
    }
  std::vector<int> fill(sstart.begin(), sstart.end() - 1);
  std::vector<PairDesc> spair(npairs);
  // emitters in gather order, so neighbouring pairs touch neighbouring windows
  for (int q = 0; q < M; ++q)
    for (const auto& bp : per_em[gem[q]]) spair[fill[slot_of[bp.first]]++] = bp.second;
  // within a bin, pairs by decreasing numbers of planes (z), then rows (y): the
  // workgroup runs eight pairs per wavefront side by side, each looping over its
  // own planes and rows, so equal counts keep its lanes busy (stable: ties stay
  // in gather order)
  for (size_t sl = 0; sl < sid.size(); ++sl) {
    auto rows = [](const PairDesc& p) {
      return 16 * (int)((p.runs >> 27) & 7) + (int)((p.runs >> 17) & 7);
    };
    std::stable_sort(spair.begin() + sstart[sl], spair.begin() + sstart[sl + 1],
                     [&](const PairDesc& x, const PairDesc& y) { return rows(x) > rows(y); });
  }
  // bins heaviest first: a workgroup per bin, two per CU, and the bins along the
  // emitter region's faces hold few pairs; started first, the heavy bins run side by
  // side and the light ones fill in behind them instead of sharing rounds with them.
  // Work of a bin: its pairs' row loops (eight pairs per wavefront) plus the clear
  // and the owner write, which cost every bin the same.
  {
    const size_t nsl = sid.size();
    std::vector<double> work(nsl, 0.0);
    for (size_t sl = 0; sl < nsl; ++sl) {
      double w = 256.0;  // clear, bound and owner write, in row-loop units
      for (int q = sstart[sl]; q < sstart[sl + 1]; ++q) {
        const unsigned ru = spair[q].runs;
        w += (double)((((ru >> 17) & 7) + 1) * (((ru >> 27) & 7) + 1)) / 8.0 + 1.0;
      }
      work[sl] = w;
    }
    std::vector<int> order(nsl);
    for (size_t q = 0; q < nsl; ++q) order[q] = (int)q;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return work[x] > work[y]; });
    std::vector<int> sid2, sstart2(1, 0);
    std::vector<PairDesc> spair2;
    spair2.reserve(spair.size());
    s->swork.clear();
    for (int sl : order) {
      s->swork.push_back((float)work[sl]);
      sid2.push_back(sid[sl]);
      spair2.insert(spair2.end(), spair.begin() + sstart[sl], spair.begin() + sstart[sl + 1]);
      sstart2.push_back((int)spair2.size());
    }
    sid.swap(sid2);
    sstart.swap(sstart2);
    spair.swap(spair2);
  }
  s->nscatter = (int)sid.size();
  STCHK(upload(&s->d_gbin_org, gorg));
  STCHK(upload(&s->d_gbin_start, gstart));
  STCHK(upload(&s->d_gbin_em, gem));
  STCHK(upload(&s->d_sbin_id, sid));
  STCHK(upload(&s->d_sbin_start, sstart));
  STCHK(upload(&s->d_sbin_pair, spair));
  STCHK(upload(&s->d_tls_slot, s->tls_slot));
  return MLK_OK;
}

// Device layout of the multilevel emitters: slots sorted by level count (stable
// in id order), every array entry-major over the slots.
mlk_status upload_multilevel(mlk_sim* s) {
  const int nml = (int)s->ml_gid.size();
  s->ml_slot.assign(s->nem, -1);
  for (int& r : s->ml_range) r = 0;
  if (nml == 0) return MLK_OK;
  std::vector<int> order(nml);
  for (int q = 0; q < nml; ++q) order[q] = q;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return s->ml_nlev[x] < s->ml_nlev[y]; });
  constexpr int L = kMaxLevels;
  std::vector<int> gid(nml);
  std::vector<double> en((size_t)L * nml, 0.0), M((size_t)L * L * nml, 0.0),
      dip((size_t)3 * nml), gphi(nml), rho((size_t)2 * L * L * nml, 0.0);
  for (int m = 0; m < nml; ++m) {
    const int q = order[m];
    gid[m] = s->ml_gid[q];
    s->ml_slot[gid[m]] = m;
    for (int a = 0; a < L; ++a) en[(size_t)a * nml + m] = s->ml_en[(size_t)L * q + a];
    for (int a = 0; a < L * L; ++a) M[(size_t)a * nml + m] = s->ml_M[(size_t)L * L * q + a];
    for (int a = 0; a < 2 * L * L; ++a)
      rho[(size_t)a * nml + m] = s->ml_rho0[(size_t)2 * L * L * q + a];
    for (int c = 0; c < 3; ++c) dip[(size_t)c * nml + m] = s->ml_dip[3 * q + c];
    gphi[m] = s->ml_gphi[q];
  }
  for (int n = 0; n <= L + 1; ++n) {
    int c = 0;
    for (int m = 0; m < nml; ++m) c += s->ml_nlev[order[m]] < n;
    s->ml_range[n] = c;
  }
  STCHK(upload(&s->d_ml_gid, gid));
  STCHK(upload(&s->d_ml_en, en));
  STCHK(upload(&s->d_ml_M, M));
  STCHK(upload(&s->d_ml_dip, dip));
  STCHK(upload(&s->d_ml_gphi, gphi));
  STCHK(upload(&s->d_ml_rho, rho));
  return MLK_OK;
}

MlDev ml_dev(mlk_sim* s) {
  MlDev d{};
  d.count = (int)s->ml_gid.size();
  d.gid = s->d_ml_gid;
  d.en = s->d_ml_en;
  d.M = s->d_ml_M;
  d.dip = s->d_ml_dip;
  d.gphi = s->d_ml_gphi;
  d.rho = s->d_ml_rho;
  return d;
}

// Rebuild every device emitter table from the host mirror (set-up only).
mlk_status rebuild_emitters(mlk_sim* s) {
  STCHK(sync_sim(s));
  const int M = s->nem;
  if (M == 0) return MLK_OK;
  STCHK(upload(&s->d_pos, s->pos));
  STCHK(upload(&s->d_sigma, s->sigma));
  STCHK(upload(&s->d_gamma, s->gamma));
  STCHK(upload(&s->d_popoff, s->pop_off));
  STCHK(upload(&s->d_tls_gid, s->tls_gid));
  STCHK(upload(&s->d_tls_w0, s->tls_w0));
  STCHK(upload(&s->d_tls_dip, s->tls_dip));
  STCHK(upload(&s->d_tls_rho, s->tls_rho0));
  STCHK(upload_multilevel(s));
  dfree(s->d_wlo);
  dfree(s->d_wlen);
  dfree(s->d_w);
  dfree(s->d_Et);
  dfree(s->d_mudot);
  HIPCHK(dalloc(&s->d_wlo, (size_t)M * 6 * sizeof(int)));
  HIPCHK(dalloc(&s->d_wlen, (size_t)M * 6 * sizeof(int)));
  HIPCHK(dalloc(&s->d_w, (size_t)M * 6 * kMaxWin * s->esz));
  HIPCHK(dalloc(&s->d_Et, (size_t)M * 3 * sizeof(double)));
  HIPCHK(dalloc(&s->d_mudot, (size_t)M * 3 * sizeof(double)));
  HIPCHK(hipMemset(s->d_Et, 0, (size_t)M * 3 * sizeof(double)));
  HIPCHK(hipMemset(s->d_mudot, 0, (size_t)M * 3 * sizeof(double)));
  if (s->fp32)
    HIPCHK(windows_f32(M, s->d_pos, s->d_sigma, s->desc.window_r, s->g, s->d_wlo, s->d_wlen,
                       (float*)s->d_w, s->stream));
  else
    HIPCHK(windows_f64(M, s->d_pos, s->d_sigma, s->desc.window_r, s->g, s->d_wlo, s->d_wlen,
                       (double*)s->d_w, s->stream));
  dfree(s->d_rec);
  if (s->fp32) {
    HIPCHK(dalloc(&s->d_rec, (size_t)M * sizeof(WinRec<float>)));
    HIPCHK(records_f32(M, s->d_wlo, s->d_wlen, (const float*)s->d_w, (WinRec<float>*)s->d_rec,
                       s->stream));
  } else {
    HIPCHK(dalloc(&s->d_rec, (size_t)M * sizeof(WinRec<double>)));
    HIPCHK(records_f64(M, s->d_wlo, s->d_wlen, (const double*)s->d_w, (WinRec<double>*)s->d_rec,
                       s->stream));
  }
  STCHK(sync_sim(s));
  return build_bins(s);
}

// Grow the on-device series buffers so that nsteps more steps fit.
mlk_status reserve_series(mlk_sim* s, int64_t nsteps) {
  const int64_t need = s->host_step + nsteps;
  if ((s->nprobe > 0 || s->fp.on) && need > s->series_cap) {
    STCHK(sync_sim(s));
    int64_t cap = s->series_cap ? 2 * s->series_cap : 1024;
    while (cap < need) cap *= 2;
    if (s->nprobe > 0) {
      double* np = nullptr;
      HIPCHK(dalloc(&np, (size_t)s->nprobe * cap * sizeof(double)));
      if (s->d_probe && s->host_step > 0)
        HIPCHK(hipMemcpy2D(np, cap * sizeof(double), s->d_probe, s->series_cap * sizeof(double),
                           s->host_step * sizeof(double), s->nprobe, hipMemcpyDeviceToDevice));
      dfree(s->d_probe);
      s->d_probe = np;
    }
    if (s->fp.on) {
      double* nf = nullptr;
      HIPCHK(dalloc(&nf, (size_t)cap * sizeof(double)));
      if (s->d_flux_series && s->host_step > 0)
        HIPCHK(hipMemcpy(nf, s->d_flux_series, s->host_step * sizeof(double),
                         hipMemcpyDeviceToDevice));
      dfree(s->d_flux_series);
      s->d_flux_series = nf;
      s->fp.series = nf;
    }
    s->series_cap = cap;
  }
  if (s->er.every > 0) {
    const int64_t rec = (need + s->er.every - 1) / s->er.every;
    if (rec > s->energy_cap) {
      STCHK(sync_sim(s));
      int64_t cap = s->energy_cap ? 2 * s->energy_cap : 64;
      while (cap < rec) cap *= 2;
      double* ne = nullptr;
      HIPCHK(dalloc(&ne, (size_t)cap * sizeof(double)));
      const int64_t have = s->host_step > 0 ? (s->host_step - 1) / s->er.every + 1 : 0;
      if (s->er.series && have > 0)
        HIPCHK(hipMemcpy(ne, s->er.series, (size_t)have * sizeof(double),
                         hipMemcpyDeviceToDevice));
      dfree(s->er.series);
      s->er.series = ne;
      s->energy_cap = cap;
    }
  }
  if (s->pop_every > 0 && s->npop > 0) {
    const int64_t rec = (need + s->pop_every - 1) / s->pop_every;
    if (rec > s->pop_cap) {
      STCHK(sync_sim(s));
      int64_t cap = s->pop_cap ? 2 * s->pop_cap : 64;
      while (cap < rec) cap *= 2;
      double* np = nullptr;
      HIPCHK(dalloc(&np, (size_t)cap * s->npop * sizeof(double)));
      const int64_t have = s->host_step > 0 ? (s->host_step - 1) / s->pop_every + 1 : 0;
      if (s->d_pop && have > 0)
        HIPCHK(hipMemcpy(np, s->d_pop, (size_t)have * s->npop * sizeof(double),
                         hipMemcpyDeviceToDevice));
      dfree(s->d_pop);
      s->d_pop = np;
      s->pop_cap = cap;
    }
  }
  return MLK_OK;
}

// Phase timing: record an event before a phase; `mark_end` records the
// closing event and keeps the pair until mlk_get_phase_time reads it.
hipError_t next_event(mlk_sim* s, hipEvent_t* ev) {
  if (s->next_event == s->events.size()) {
    hipEvent_t e;
    hipError_t err = hipEventCreate(&e);
    if (err != hipSuccess) return err;
    s->events.push_back(e);
  }
  *ev = s->events[s->next_event++];
  return hipSuccess;
}

int mark_begin(mlk_sim* s, int phase) {
  if (!(s->timing & (1 << phase))) return -1;
  hipEvent_t e;
  if (next_event(s, &e) != hipSuccess) return -1;
  if (hipEventRecord(e, s->stream) != hipSuccess) return -1;
  return (int)s->next_event - 1;
}

void mark_end(mlk_sim* s, int phase, int begin) {
  if (begin < 0) return;
  hipEvent_t e;
  if (next_event(s, &e) != hipSuccess) return;
  if (hipEventRecord(e, s->stream) != hipSuccess) return;
  s->marks.push_back({phase, begin, (int)s->next_event - 1});
}

// Fold the pending marks into the per-phase totals (the stream must be idle).
hipError_t collect_marks(mlk_sim* s) {
  for (const auto& m : s->marks) {
    float ms = 0.f;
    hipError_t e = hipEventElapsedTime(&ms, s->events[m[1]], s->events[m[2]]);
    if (e != hipSuccess) return e;
    s->phase_ms[m[0]] += ms;
    s->phase_n[m[0]] += 1;
  }
  s->marks.clear();
  s->next_event = 0;
  return hipSuccess;
}

// Box of the fused sweep.  With FP32 fields (layers): the whole grid, the
// kernel stretching the derivatives of cells in the CPML layers itself; with
// FP64 fields the y and z extent stops one cell of margin above the low layers
// and at the high layers (the FP64 kernel carries the x layers only, keeping
// its registers within occupancy), the plain passes updating the rest.  In both
// the x extent is every column provided the low-x halo column of each tx-wide
// tile (x = tx t - 1, t >= 1) lies outside the x layers and the x psi arrays
// index in 32 bits; otherwise x is limited like y and z.  The y and z psi
// arrays must index in 32 bits too for a full y and z extent.  The cells
// outside the box form the CPML shell.
// z planes per chunk of the frame launch's y slabs
constexpr int kFrameKz = 8;

Box interior_box(const Geom& g, bool layers, int tx) {
  Box inner{};
  const int n = g.n[0], ntx = (n + tx - 1) / tx;
  const double plane = (double)g.n[0] * g.n[1] * g.n[2];
  const bool x_full = !has_cpml(g, 0) ||
                      (g.nlo[0] <= tx - 1 && tx * (ntx - 1) <= n - g.nhi[0] &&
                       (double)(g.nlo[0] + g.nhi[0]) * g.n[1] * g.n[2] < 4294967296.0);
  const bool yz_full = layers && 4.0 * plane * (g.nlo[1] + g.nhi[1]) / g.n[1] < 4294967296.0 &&
                       4.0 * plane * (g.nlo[2] + g.nhi[2]) / g.n[2] < 4294967296.0;
  for (int a = 0; a < 3; ++a) {
    const bool full = a == 0 ? x_full : yz_full;
    inner.lo[a] = full ? 0 : (g.nlo[a] > 0 ? g.nlo[a] + 1 : 0);
    inner.hi[a] = full ? g.n[a] : std::max(inner.lo[a], g.n[a] - g.nhi[a]);
  }
  return inner;
}

Box sweep_box(const mlk_sim* s) {
  return interior_box(s->g, s->fp32 && s->layer_mode == 1, s->tx);
}

// The frame launch can take the y/z layers when the fused box of the other modes
// spans every x column (the x layers then stay in the box's own kernel) and some
// y or z face has layers.  FP32 only (the FP64 kernel carries the x layers alone).
bool split_ok(const mlk_sim* s) {
  if (!s->fp32 || (!has_cpml(s->g, 1) && !has_cpml(s->g, 2))) return false;
  const Box b = interior_box(s->g, false, s->tx);
  return b.lo[0] == 0 && b.hi[0] == s->g.n[0];
}

// The fused launch over the sim's box and the passes for the cells outside it:
// the frame launch (layer mode 2) or the two plain shell passes.
template <typename T>
hipError_t sweep_passes(const mlk_sim* s, const FieldPtrs<T>& a, const FieldPtrs<T>& ar,
                        const FieldPtrs<T>& b, const Box& inner, int kz, int tx, int ty) {
  hipError_t e = hipSuccess;
  if constexpr (sizeof(T) == 4) {
    e = sweep_fused_f32(ar, b, s->g, inner, kz, tx, ty, s->stream);
    if (e == hipSuccess && s->layer_mode == 2 && split_ok(s))
      return sweep_frame_f32(ar, b, s->g, inner, kFrameKz, s->stream);
    if (e == hipSuccess) e = sweep_shell_f32(a, b, s->g, inner, true, s->stream);
    if (e == hipSuccess) e = sweep_shell_f32(a, b, s->g, inner, false, s->stream);
  } else {
    e = sweep_fused_f64(ar, b, s->g, inner, kz, tx, ty, s->stream);
    if (e == hipSuccess) e = sweep_shell_f64(a, b, s->g, inner, true, s->stream);
    if (e == hipSuccess) e = sweep_shell_f64(a, b, s->g, inner, false, s->stream);
  }
  return e;
}

// The fields as the fused sweep reads them: no 1/eps_r array in vacuum.
template <typename T>
FieldPtrs<T> sweep_reads(const mlk_sim* s) {
  FieldPtrs<T> f = field_ptrs<T>(s);
  if (s->vacuum) f.epsinv = nullptr;
  return f;
}

template <typename T>
mlk_status sweep(mlk_sim* s) {
  constexpr bool f32 = sizeof(T) == 4;
  const FieldPtrs<T> f = field_ptrs<T>(s);
  if (s->desc.sweep == MLK_SWEEP_FUSED) {
    const FieldPtrs<T> nf = spare_ptrs<T>(s), fr = sweep_reads<T>(s);
    const Box inner = sweep_box(s);
    if (f32 && s->layer_mode == 2 && split_ok(s)) {
      // the lean interior, then the layer frame in one launch of the full kernel
      int t0 = mark_begin(s, MLK_PHASE_SWEEP);
      if constexpr (f32) HIPCHK(sweep_fused_f32(fr, nf, s->g, inner, s->kz, s->tx, s->ty, s->stream));
      mark_end(s, MLK_PHASE_SWEEP, t0);
      t0 = mark_begin(s, MLK_PHASE_SHELL);
      if constexpr (f32) HIPCHK(sweep_frame_f32(fr, nf, s->g, inner, kFrameKz, s->stream));
      mark_end(s, MLK_PHASE_SHELL, t0);
    } else {
      int t0 = mark_begin(s, MLK_PHASE_SWEEP);
      if constexpr (f32) HIPCHK(sweep_fused_f32(fr, nf, s->g, inner, s->kz, s->tx, s->ty, s->stream));
      else HIPCHK(sweep_fused_f64(fr, nf, s->g, inner, s->kz, s->tx, s->ty, s->stream));
      mark_end(s, MLK_PHASE_SWEEP, t0);
      t0 = mark_begin(s, MLK_PHASE_SHELL);
      if constexpr (f32) {
        HIPCHK(sweep_shell_f32(f, nf, s->g, inner, true, s->stream));
        HIPCHK(sweep_shell_f32(f, nf, s->g, inner, false, s->stream));
      } else {
        HIPCHK(sweep_shell_f64(f, nf, s->g, inner, true, s->stream));
        HIPCHK(sweep_shell_f64(f, nf, s->g, inner, false, s->stream));
      }
      mark_end(s, MLK_PHASE_SHELL, t0);
    }
    swap_buffers(s);
  } else {
    Box all{};
    for (int a = 0; a < 3; ++a) {
      all.lo[a] = 0;
      all.hi[a] = s->g.n[a];
    }
    const int t0 = mark_begin(s, MLK_PHASE_SWEEP);
    if constexpr (f32) HIPCHK(sweep_plain_f32(f, f, s->g, &all, 1, true, true, s->stream));
    else HIPCHK(sweep_plain_f64(f, f, s->g, &all, 1, true, true, s->stream));
    mark_end(s, MLK_PHASE_SWEEP, t0);
  }
  if (s->src.count > 0) {
    const FieldPtrs<T> cur = field_ptrs<T>(s);
    const int t0 = mark_begin(s, MLK_PHASE_SOURCES);
    if constexpr (f32) HIPCHK(sources_f32(cur, s->g, s->src, s->d_step, s->stream));
    else HIPCHK(sources_f64(cur, s->g, s->src, s->d_step, s->stream));
    mark_end(s, MLK_PHASE_SOURCES, t0);
  }
  return MLK_OK;
}

template <typename T>
mlk_status enqueue_steps(mlk_sim* s, int64_t nsteps) {
  const WindowPtrs<T> win = window_ptrs<T>(s);
  const Series ser = series_of(s);
  const TlsPtrs tls = tls_ptrs(s);
  constexpr bool f32 = sizeof(T) == 4;
  const bool binned = s->desc.scatter == MLK_SCATTER_OWNER && s->nem > 0;
  const BinPtrs bins = bin_ptrs(s);
  const MlDev ml = ml_dev(s);
  // the gather launch saves the flux plane too when it runs
  const bool fold_save = s->fp.on && s->nem > 0 && s->ngather > 0;
  const FluxPlane* fsave = fold_save ? &s->fp : nullptr;
  // and the scatter launch forms the flux partials when no window reaches the plane
  // (the owner write changes no cell the flux reads) and no pole pass runs between them
  const bool fold_flux = binned && s->fp.on && s->npole == 0 && s->nscatter > 0 &&
                         (int)s->wplane[s->fp.axis].size() == s->g.n[s->fp.axis] &&
                         !s->wplane[s->fp.axis][s->fp.index];
  const FluxPlane* fpart = fold_flux ? &s->fp : nullptr;
  for (int64_t q = 0; q < nsteps; ++q) {
    FieldPtrs<T> f = field_ptrs<T>(s);
    if (s->fp.on && !fold_save) {
      const int t0 = mark_begin(s, MLK_PHASE_DETECTORS);
      if constexpr (f32) HIPCHK(flux_save_f32(f, s->g, s->fp, s->stream));
      else HIPCHK(flux_save_f64(f, s->g, s->fp, s->stream));
      mark_end(s, MLK_PHASE_DETECTORS, t0);
    }
    int t0 = mark_begin(s, MLK_PHASE_EMITTERS);
    if (s->nem > 0) {
      // gather of every emitter, then the two-level and the multilevel steps
      if constexpr (f32)
        HIPCHK(bin_gather_step_f32(f, s->g, bins, win, tls, s->d_Et, s->d_mudot, s->d_popoff,
                                   ser, s->d_step, fsave, s->stream));
      else
        HIPCHK(bin_gather_step_f64(f, s->g, bins, win, tls, s->d_Et, s->d_mudot, s->d_popoff,
                                   ser, s->d_step, fsave, s->stream));
      if (ml.count > 0)
        HIPCHK(ml_step(ml, s->ml_range, s->g.dt, s->d_Et, s->d_mudot, s->d_popoff, ser,
                       s->d_step, s->stream));
    }
    mark_end(s, MLK_PHASE_EMITTERS, t0);
    t0 = s->npole ? mark_begin(s, MLK_PHASE_POLES) : -1;
    for (int k = 0; k < s->npole; ++k) {
      if constexpr (f32) HIPCHK(pole_pre_f32(s->pole[k], f, s->g, s->stream));
      else HIPCHK(pole_pre_f64(s->pole[k], f, s->g, s->stream));
    }
    mark_end(s, MLK_PHASE_POLES, t0);
    STCHK(sweep<T>(s));
    f = field_ptrs<T>(s);
    if (s->er.every > 0) {
      // W^n: E^n and H^{n-1/2} are in the spare buffers now, H^{n+1/2} in the current
      t0 = mark_begin(s, MLK_PHASE_DETECTORS);
      if constexpr (f32) HIPCHK(energy_f32(spare_ptrs<T>(s), f, s->ncell, s->er, s->d_step, s->stream));
      else HIPCHK(energy_f64(spare_ptrs<T>(s), f, s->ncell, s->er, s->d_step, s->stream));
      mark_end(s, MLK_PHASE_DETECTORS, t0);
    }
    t0 = mark_begin(s, MLK_PHASE_SCATTER);
    if (binned) {
      // in vacuum the owner write reads no 1/eps_r
      FieldPtrs<T> fs = f;
      if (s->vacuum) fs.epsinv = nullptr;
      if constexpr (f32)
        HIPCHK(bin_scatter_f32(fs, s->g, bins, win, s->d_mudot, fpart, s->stream));
      else
        HIPCHK(bin_scatter_f64(fs, s->g, bins, win, s->d_mudot, fpart, s->stream));
    } else if (s->nem > 0) {
      if constexpr (f32)
        HIPCHK(scatter_atomic_f32(f, s->g, win, s->nem, s->d_mudot, s->stream));
      else
        HIPCHK(scatter_atomic_f64(f, s->g, win, s->nem, s->d_mudot, s->stream));
    }
    mark_end(s, MLK_PHASE_SCATTER, t0);
    t0 = s->npole ? mark_begin(s, MLK_PHASE_POLES) : -1;
    for (int k = 0; k < s->npole; ++k) {
      if constexpr (f32) HIPCHK(pole_post_f32(s->pole[k], f, s->g, (const float*)s->epsinv, s->stream));
      else HIPCHK(pole_post_f64(s->pole[k], f, s->g, (const double*)s->epsinv, s->stream));
    }
    mark_end(s, MLK_PHASE_POLES, t0);
    t0 = mark_begin(s, MLK_PHASE_DETECTORS);
    if constexpr (f32) HIPCHK(finish_f32(f, s->g, s->fp, ser, s->d_step, fold_flux, s->stream));
    else HIPCHK(finish_f64(f, s->g, s->fp, ser, s->d_step, fold_flux, s->stream));
    mark_end(s, MLK_PHASE_DETECTORS, t0);
  }
  return MLK_OK;
}

// Cavity steps: E~ from the mode, the emitter steps, then the mode update
// (which also moves the step counter on).  The grid is left alone.
mlk_status enqueue_cavity_steps(mlk_sim* s, int64_t nsteps) {
  const Series ser = series_of(s);
  const TlsPtrs tls = tls_ptrs(s);
  const MlDev ml = ml_dev(s);
  const int ntls = (int)s->tls_gid.size();
  for (int64_t q = 0; q < nsteps; ++q) {
    const int t0 = mark_begin(s, MLK_PHASE_EMITTERS);
    if (ml.count == 0 && ntls > 0) {
      // two-level emitters only: field, step and partial sums in one launch
      HIPCHK(cavity_tls_step(tls, s->g.dt, s->cav, s->d_Et, s->d_mudot, s->d_popoff, ser,
                             s->d_step, s->stream));
      HIPCHK(cavity_advance(s->cav, cavity_tls_blocks(ntls), s->g.dt, s->d_step, s->stream));
      mark_end(s, MLK_PHASE_EMITTERS, t0);
      continue;
    }
    if (s->nem > 0) {
      HIPCHK(cavity_field(s->cav, s->d_Et, s->nem, s->stream));
      HIPCHK(tls_step(tls, s->g.dt, s->d_Et, s->d_mudot, s->d_popoff, ser, s->d_step, s->stream));
      if (ml.count > 0)
        HIPCHK(ml_step(ml, s->ml_range, s->g.dt, s->d_Et, s->d_mudot, s->d_popoff, ser,
                       s->d_step, s->stream));
    }
    HIPCHK(cavity_update(s->cav, tls, ml, s->g.dt, s->d_step, s->stream));
    mark_end(s, MLK_PHASE_EMITTERS, t0);
  }
  return MLK_OK;
}

void release(mlk_sim* s) {
  for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
  s->events.clear();
  // caller-owned buffers are dropped, not freed
  auto drop = [&](void*& p) {
    if (p && std::find(s->borrowed.begin(), s->borrowed.end(), p) != s->borrowed.end())
      p = nullptr;
  };
  for (int c = 0; c < 3; ++c) {
    drop(s->E[c]);
    drop(s->H[c]);
    drop(s->E2[c]);
    drop(s->H2[c]);
  }
  drop(s->psi);
  drop(s->psi2);
  {
    void* t = s->d_tls_rho;
    drop(t);
    if (!t) s->d_tls_rho = nullptr;
    void* m = s->d_ml_rho;
    drop(m);
    if (!m) s->d_ml_rho = nullptr;
  }
  for (int c = 0; c < 3; ++c) {
    dfree(s->E[c]);
    dfree(s->H[c]);
    dfree(s->E2[c]);
    dfree(s->H2[c]);
  }
  dfree(s->psi);
  dfree(s->psi2);
  dfree(s->tab);
  dfree(s->epsinv);
  dfree(s->d_wlo);
  dfree(s->d_wlen);
  dfree(s->d_w);
  dfree(s->d_rec);
  dfree(s->d_pos);
  dfree(s->d_sigma);
  dfree(s->d_gamma);
  dfree(s->d_Et);
  dfree(s->d_mudot);
  dfree(s->d_popoff);
  dfree(s->d_tls_gid);
  dfree(s->d_tls_w0);
  dfree(s->d_tls_dip);
  dfree(s->d_tls_rho);
  dfree(s->d_ml_gid);
  dfree(s->d_ml_en);
  dfree(s->d_ml_M);
  dfree(s->d_ml_dip);
  dfree(s->d_ml_gphi);
  dfree(s->d_ml_rho);
  dfree(s->d_gbin_org);
  dfree(s->d_gbin_start);
  dfree(s->d_gbin_em);
  dfree(s->d_sbin_id);
  dfree(s->d_sbin_start);
  dfree(s->d_sbin_pair);
  dfree(s->d_tls_slot);
  dfree(s->d_probe);
  dfree(s->d_flux_series);
  dfree(s->fp.Eu0);
  dfree(s->fp.Ev0);
  dfree(s->fp.partial);
  dfree(s->fp.total);
  dfree(s->d_pop);
  dfree(s->d_step);
  dfree(s->d_numeric);
  dfree(s->er.partial);
  dfree(s->er.series);
  dfree(s->cav.st);
  dfree(s->cav.partial);
  for (int k = 0; k < s->npole; ++k) {
    dfree(s->pole[k].P);
    dfree(s->pole[k].Q);
  }
  if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
  s->stream = nullptr;
}

// Device buffers that make up the evolving state, in checkpoint order.
struct Piece {
  void* p;
  size_t bytes;
};

std::vector<Piece> state_pieces(mlk_sim* s) {
  std::vector<Piece> v;
  for (int c = 0; c < 3; ++c) v.push_back({s->E[c], s->ncell * s->esz});
  for (int c = 0; c < 3; ++c) v.push_back({s->H[c], s->ncell * s->esz});
  if (s->psi) v.push_back({s->psi, psi_total(s->g) * s->esz});
  if (!s->tls_gid.empty()) v.push_back({s->d_tls_rho, s->tls_gid.size() * 3 * sizeof(double)});
  if (!s->ml_gid.empty())
    v.push_back({s->d_ml_rho, s->ml_gid.size() * 2 * kMaxLevels * kMaxLevels * sizeof(double)});
  if (s->nem > 0) {
    v.push_back({s->d_Et, (size_t)s->nem * 3 * sizeof(double)});
    v.push_back({s->d_mudot, (size_t)s->nem * 3 * sizeof(double)});
  }
  v.push_back({s->d_step, sizeof(int64_t)});
  if (s->fp.on) v.push_back({s->fp.total, sizeof(double)});
  if (s->cav_on) v.push_back({s->cav.st, 6 * sizeof(double)});
  for (int k = 0; k < s->npole; ++k) {
    const size_t nb = 3 * (size_t)s->pole[k].n[0] * s->pole[k].n[1] * s->pole[k].n[2];
    v.push_back({s->pole[k].P, nb * s->esz});
    v.push_back({s->pole[k].Q, nb * s->esz});
  }
  return v;
}

// Restore the evolving state from a checkpoint (the watchdog is left alone).
mlk_status load_state(mlk_sim* s, const void* src, int32_t mem_kind) {
  STCHK(sync_sim(s));
  const char* o = (const char*)src;
  const hipMemcpyKind kind =
      mem_kind == MLK_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  for (const Piece& p : state_pieces(s)) {
    HIPCHK(hipMemcpy(p.p, o, p.bytes, kind));
    o += p.bytes;
  }
  int64_t step = 0;
  HIPCHK(hipMemcpy(&step, s->d_step, sizeof(int64_t), hipMemcpyDeviceToHost));
  if (step > s->host_step) STCHK(reserve_series(s, step - s->host_step));
  s->host_step = step;
  return MLK_OK;
}

}  // namespace

extern "C" {

void mlk_grid_desc_init(mlk_grid_desc* g) {
  if (!g) return;
  std::memset(g, 0, sizeof(*g));
  g->nx = g->ny = g->nz = 32;
  g->dx = 1.0;
  g->courant = 0.5;
  g->precision = MLK_FP64;
  for (int f = 0; f < 6; ++f) {
    g->bc[f] = MLK_BC_PEC;
    g->cpml_cells[f] = 0;
  }
  g->cpml_m = 3.0;
  g->cpml_sigma_scale = 0.8;
  g->cpml_kappa_max = 1.0;
  g->cpml_alpha_max = 0.0;
  g->window_r = 3.0;
  g->stream = nullptr;
  g->device = 0;
  g->sweep = MLK_SWEEP_FUSED;
  g->scatter = MLK_SCATTER_OWNER;
}

const char* mlk_last_error(void) { return g_err.c_str(); }

const char* mlk_version(void) { return "mlk 0.1 gfx950"; }

mlk_status mlk_create(const mlk_grid_desc* gd, mlk_sim** out) {
  if (!gd || !out) return fail(MLK_EINVAL, "null argument");
  *out = nullptr;
  const int n[3] = {gd->nx, gd->ny, gd->nz};
  for (int a = 0; a < 3; ++a)
    if (n[a] < 1) return fail(MLK_EINVAL, "grid size must be >= 1 on every axis");
  if (!(gd->dx > 0.0) || !std::isfinite(gd->dx)) return fail(MLK_EINVAL, "dx must be > 0");
  if (!(gd->courant > 0.0) || gd->courant > 1.0 / std::sqrt(3.0))
    return fail(MLK_EINVAL, "courant %.6f outside (0, 1/sqrt(3)]", gd->courant);
  if (gd->precision != MLK_FP64 && gd->precision != MLK_FP32_FIELDS)
    return fail(MLK_EINVAL, "unknown precision %d", gd->precision);
  if (!(gd->window_r > 0.0)) return fail(MLK_EINVAL, "window_r must be > 0");
  if (gd->sweep != MLK_SWEEP_PLAIN && gd->sweep != MLK_SWEEP_FUSED)
    return fail(MLK_EINVAL, "unknown sweep %d", gd->sweep);
  if (gd->scatter != MLK_SCATTER_ATOMIC && gd->scatter != MLK_SCATTER_OWNER)
    return fail(MLK_EINVAL, "unknown scatter %d", gd->scatter);
  for (int a = 0; a < 3; ++a) {
    const int lo = gd->bc[2 * a], hi = gd->bc[2 * a + 1];
    for (int b : {lo, hi})
      if (b < MLK_BC_PEC || b > MLK_BC_CPML) return fail(MLK_EINVAL, "unknown boundary %d", b);
    if ((lo == MLK_BC_PERIODIC) != (hi == MLK_BC_PERIODIC))
      return fail(MLK_EINVAL, "periodic boundaries must pair on axis %d", a);
    for (int f = 0; f < 2; ++f)
      if (gd->bc[2 * a + f] == MLK_BC_CPML &&
          (gd->cpml_cells[2 * a + f] < 1 || gd->cpml_cells[2 * a + f] > n[a] / 2))
        return fail(MLK_EINVAL, "CPML thickness on face %d must be 1..%d", 2 * a + f, n[a] / 2);
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
    return fail(MLK_EDEVICE, "no HIP device available");
  if (gd->device < 0 || gd->device >= ndev) return fail(MLK_EINVAL, "bad device %d", gd->device);
  HIPCHK(hipSetDevice(gd->device));

  mlk_sim* s = new mlk_sim();
  s->desc = *gd;
  s->fp32 = gd->precision == MLK_FP32_FIELDS;
  s->esz = s->fp32 ? 4 : 8;
  Geom& g = s->g;
  for (int a = 0; a < 3; ++a) {
    g.n[a] = n[a];
    g.periodic[a] = gd->bc[2 * a] == MLK_BC_PERIODIC;
    g.wall[a] = !g.periodic[a];
    g.nlo[a] = gd->bc[2 * a] == MLK_BC_CPML ? gd->cpml_cells[2 * a] : 0;
    g.nhi[a] = gd->bc[2 * a + 1] == MLK_BC_CPML ? gd->cpml_cells[2 * a + 1] : 0;
  }
  g.dx = gd->dx;
  g.inv_dx = 1.0 / gd->dx;
  g.dt = gd->courant * gd->dx;
  s->ncell = (size_t)n[0] * n[1] * n[2];

  auto bail = [&](mlk_status st) {
    release(s);
    delete s;
    return st;
  };
  if (gd->stream) {
    s->stream = (hipStream_t)gd->stream;
  } else {
    if (hipStreamCreate(&s->stream) != hipSuccess)
      return bail(fail(MLK_EDEVICE, "hipStreamCreate failed"));
    s->own_stream = true;
  }
  auto alloc_zero = [&](void** p, size_t bytes) -> bool {
    if (dalloc(p, bytes) != hipSuccess) return false;
    return hipMemsetAsync(*p, 0, bytes, s->stream) == hipSuccess;
  };
  const bool fused = gd->sweep == MLK_SWEEP_FUSED;
  // the fused kernels address a field array and the psi buffer by 32-bit byte offsets
  if (fused && (s->ncell * s->esz >= ((size_t)1 << 32) || psi_total(g) * s->esz >= ((size_t)1 << 32)))
    return bail(fail(MLK_EUNSUPPORTED, "the fused sweep needs field arrays and psi buffer "
                                       "under 4 GiB (%zu and %zu bytes): use the plain sweep",
                     s->ncell * s->esz, psi_total(g) * s->esz));
  for (int c = 0; c < 3; ++c) {
    if (!alloc_zero(&s->E[c], s->ncell * s->esz) || !alloc_zero(&s->H[c], s->ncell * s->esz))
      return bail(fail(MLK_ENOMEM, "field allocation of %zu bytes failed", s->ncell * s->esz));
    if (fused && (!alloc_zero(&s->E2[c], s->ncell * s->esz) ||
                  !alloc_zero(&s->H2[c], s->ncell * s->esz)))
      return bail(fail(MLK_ENOMEM, "field allocation of %zu bytes failed", s->ncell * s->esz));
  }
  {
    // z planes per workgroup of the fused sweep: enough workgroups to fill the chip
    const int ntile = ((n[0] + 63) / 64) * ((n[1] + 3) / 4);
    int kz = (int)(((long long)n[2] * ntile + 2047) / 2048);
    s->kz = std::max(8, std::min(kz, n[2]));
  }
  // FP32: the fused sweep takes the y and z layers when they are a small part of
  // the grid (on small, layer-heavy grids the plain shell passes are faster);
  // mlk_autotune measures both
  {
    const bool thin = (double)(s->g.nlo[1] + s->g.nhi[1]) / n[1] +
                          (double)(s->g.nlo[2] + s->g.nhi[2]) / n[2] <= 0.25;
    s->layer_mode = s->fp32 && thin ? 1 : 0;
  }
  if (dalloc(&s->epsinv, s->ncell * s->esz) != hipSuccess)
    return bail(fail(MLK_ENOMEM, "eps allocation failed"));
  {
    // eps_r = 1 everywhere
    double* d1 = nullptr;
    if (dalloc(&d1, s->ncell * sizeof(double)) != hipSuccess)
      return bail(fail(MLK_ENOMEM, "eps staging allocation failed"));
    std::vector<double> h(s->ncell, 1.0);
    hipError_t e = hipMemcpy(d1, h.data(), s->ncell * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = inverse_to(s->fp32, d1, s->epsinv, s->ncell, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    dfree(d1);
    if (e != hipSuccess) return bail(fail(MLK_EDEVICE, "eps init: %s", hipGetErrorString(e)));
  }
  const double sigma_max = gd->cpml_sigma_scale * (gd->cpml_m + 1.0) / gd->dx;
  if (psi_total(g) > 0) {
    if (!alloc_zero(&s->psi, psi_total(g) * s->esz) ||
        (fused && !alloc_zero(&s->psi2, psi_total(g) * s->esz)))
      return bail(fail(MLK_ENOMEM, "psi allocation failed"));
    if (dalloc(&s->tab, tab_total(g) * s->esz) != hipSuccess)
      return bail(fail(MLK_ENOMEM, "CPML table allocation failed"));
    for (int a = 0; a < 3; ++a) {
      if (!has_cpml(g, a)) continue;
      char* t = (char*)s->tab + tab_offset(g, a) * s->esz;
      const size_t blk = (size_t)2 * n[a] * s->esz;
      if (cpml_tables(s->fp32, g, a, gd->cpml_m, sigma_max, gd->cpml_kappa_max,
                      gd->cpml_alpha_max, t, t + blk, t + 2 * blk, s->stream) != hipSuccess)
        return bail(fail(MLK_EDEVICE, "CPML table kernel failed"));
    }
  }
  if (dalloc(&s->d_step, sizeof(int64_t)) != hipSuccess ||
      dalloc(&s->d_numeric, sizeof(unsigned long long)) != hipSuccess)
    return bail(fail(MLK_ENOMEM, "step counter allocation failed"));
  if (hipMemsetAsync(s->d_step, 0, sizeof(int64_t), s->stream) != hipSuccess ||
      hipMemsetAsync(s->d_numeric, 0, sizeof(unsigned long long), s->stream) != hipSuccess ||
      hipStreamSynchronize(s->stream) != hipSuccess)
    return bail(fail(MLK_EDEVICE, "initialisation failed"));
  *out = s;
  return MLK_OK;
}

mlk_status mlk_destroy(mlk_sim* s) {
  if (!s) return MLK_OK;
  if (s->in_batch) return fail(MLK_ESTATE, "destroy the batch this sim belongs to first");
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  release(s);
  delete s;
  return MLK_OK;
}

mlk_status mlk_set_eps(mlk_sim* s, const double* eps, int32_t mem_kind) {
  if (!s || !eps) return fail(MLK_EINVAL, "null argument");
  std::vector<double> h;
  const double* src = eps;
  if (mem_kind == MLK_MEM_DEVICE) {
    h.resize(s->ncell);
    HIPCHK(hipMemcpy(h.data(), eps, s->ncell * sizeof(double), hipMemcpyDeviceToHost));
    src = h.data();
  } else if (mem_kind != MLK_MEM_HOST) {
    return fail(MLK_EINVAL, "bad mem_kind");
  }
  bool vac = true;
  for (size_t q = 0; q < s->ncell; ++q) {
    if (!(src[q] >= 1.0) || !std::isfinite(src[q]))
      return fail(MLK_EINVAL, "eps_r[%zu] = %g must be finite and >= 1", q, src[q]);
    vac = vac && src[q] == 1.0;
  }
  double* d = nullptr;
  HIPCHK(dalloc(&d, s->ncell * sizeof(double)));
  hipError_t e = hipMemcpy(d, src, s->ncell * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e == hipSuccess) e = inverse_to(s->fp32, d, s->epsinv, s->ncell, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  dfree(d);
  if (e != hipSuccess) return fail(MLK_EDEVICE, "set_eps: %s", hipGetErrorString(e));
  s->vacuum = vac;
  return MLK_OK;
}

mlk_status mlk_set_field(mlk_sim* s, int32_t comp, const double* src, int32_t mem_kind) {
  if (!s || !src) return fail(MLK_EINVAL, "null argument");
  if (comp < 0 || comp > 5) return fail(MLK_EINVAL, "component %d outside 0..5", comp);
  double* d = nullptr;
  HIPCHK(dalloc(&d, s->ncell * sizeof(double)));
  hipError_t e = hipStreamSynchronize(s->stream);
  if (e == hipSuccess)
    e = hipMemcpy(d, src, s->ncell * sizeof(double),
                  mem_kind == MLK_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice);
  void* dst = comp < 3 ? s->E[comp] : s->H[comp - 3];
  if (e == hipSuccess) e = convert_in(s->fp32, d, dst, s->ncell, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  dfree(d);
  if (e != hipSuccess) return fail(MLK_EDEVICE, "set_field: %s", hipGetErrorString(e));
  return MLK_OK;
}

mlk_status mlk_add_tls(mlk_sim* s, int32_t n, const double* pos, const double* sigma,
                       const double* gamma, const double* omega0, const double* dipole,
                       const double* rho0, int32_t* first_id) {
  if (!s || !pos || !sigma || !gamma || !omega0 || !dipole || !rho0)
    return fail(MLK_EINVAL, "null argument");
  if (n < 0) return fail(MLK_EINVAL, "negative count");
  if (s->host_step > 0) return fail(MLK_ESTATE, "emitters must be added before stepping");
  if (s->cav_on) return fail(MLK_ESTATE, "emitters must be added before the cavity is set");
  if (s->states_bound)
    return fail(MLK_ESTATE, "emitters must be added before their states are bound");
  for (int q = 0; q < n; ++q) {
    STCHK(check_emitter_geometry(s, pos + 3 * q, sigma[q]));
    const double p = rho0[3 * q], re = rho0[3 * q + 1], im = rho0[3 * q + 2];
    if (!(p >= 0.0 && p <= 1.0) || !std::isfinite(re) || !std::isfinite(im) ||
        re * re + im * im > p * (1.0 - p) * (1.0 + 1e-12) + 1e-300)
      return fail(MLK_EINVAL, "emitter %d: initial state is not a density matrix", q);
    if (!std::isfinite(omega0[q]) || !std::isfinite(gamma[q]))
      return fail(MLK_EINVAL, "emitter %d: parameters not finite", q);
  }
  if (first_id) *first_id = s->nem;
  for (int q = 0; q < n; ++q) {
    const int e = s->nem++;
    for (int a = 0; a < 3; ++a) s->pos.push_back(pos[3 * q + a]);
    s->sigma.push_back(sigma[q]);
    s->gamma.push_back(gamma[q]);
    s->pop_off.push_back(s->npop);
    s->npop += 1;
    s->tls_slot.push_back((int)s->tls_gid.size());
    s->tls_gid.push_back(e);
    s->tls_w0.push_back(omega0[q]);
    for (int a = 0; a < 3; ++a) s->tls_dip.push_back(dipole[3 * q + a]);
    for (int a = 0; a < 3; ++a) s->tls_rho0.push_back(rho0[3 * q + a]);
  }
  return rebuild_emitters(s);
}

mlk_status mlk_add_multilevel(mlk_sim* s, int32_t n, const int32_t* nlev, const int64_t* eoff,
                              const int64_t* moff, const double* energies, const double* mop,
                              const double* dipole, const double* gphi, const double* rho0,
                              const double* pos, const double* sigma, const double* gamma,
                              int32_t* first_id) {
  if (!s || !nlev || !eoff || !moff || !energies || !mop || !dipole || !gphi || !rho0 || !pos ||
      !sigma || !gamma)
    return fail(MLK_EINVAL, "null argument");
  if (n < 0) return fail(MLK_EINVAL, "negative count");
  if (s->host_step > 0) return fail(MLK_ESTATE, "emitters must be added before stepping");
  if (s->cav_on) return fail(MLK_ESTATE, "emitters must be added before the cavity is set");
  if (s->states_bound)
    return fail(MLK_ESTATE, "emitters must be added before their states are bound");
  for (int q = 0; q < n; ++q) {
    const int L = nlev[q];
    if (L < 2 || L > kMaxLevels)
      return fail(MLK_EUNSUPPORTED, "emitter %d: %d levels (2..%d supported)", q, L, kMaxLevels);
    if (eoff[q] < 0 || moff[q] < 0) return fail(MLK_EINVAL, "emitter %d: negative offset", q);
    STCHK(check_emitter_geometry(s, pos + 3 * q, sigma[q]));
    if (!(gphi[q] >= 0.0) || !std::isfinite(gphi[q]) || !std::isfinite(gamma[q]))
      return fail(MLK_EINVAL, "emitter %d: parameters not finite or negative dephasing", q);
    const double* E = energies + eoff[q];
    const double* M = mop + moff[q];
    const double* r = rho0 + 2 * moff[q];
    double trace = 0.0;
    for (int a = 0; a < L; ++a) {
      if (!std::isfinite(E[a])) return fail(MLK_EINVAL, "emitter %d: energy not finite", q);
      trace += r[2 * (a * L + a)];
      if (!(r[2 * (a * L + a)] >= -1e-12) || std::fabs(r[2 * (a * L + a) + 1]) > 1e-12)
        return fail(MLK_EINVAL, "emitter %d: initial state is not a density matrix", q);
      for (int b = 0; b < L; ++b) {
        if (!std::isfinite(M[a * L + b]) || M[a * L + b] != M[b * L + a])
          return fail(MLK_EINVAL, "emitter %d: dipole matrix not real symmetric", q);
        const double dre = r[2 * (a * L + b)] - r[2 * (b * L + a)];
        const double dim = r[2 * (a * L + b) + 1] + r[2 * (b * L + a) + 1];
        if (!(std::fabs(dre) <= 1e-12 && std::fabs(dim) <= 1e-12))
          return fail(MLK_EINVAL, "emitter %d: initial state is not Hermitian", q);
      }
    }
    if (!(std::fabs(trace - 1.0) <= 1e-10))
      return fail(MLK_EINVAL, "emitter %d: initial state has trace %g", q, trace);
  }
  if (first_id) *first_id = s->nem;
  constexpr int F = kMaxLevels;
  for (int q = 0; q < n; ++q) {
    const int e = s->nem++;
    const int L = nlev[q];
    for (int a = 0; a < 3; ++a) s->pos.push_back(pos[3 * q + a]);
    s->sigma.push_back(sigma[q]);
    s->gamma.push_back(gamma[q]);
    s->pop_off.push_back(s->npop);
    s->npop += L - 1;
    s->tls_slot.push_back(-1);
    s->ml_gid.push_back(e);
    s->ml_nlev.push_back(L);
    for (int a = 0; a < F; ++a) s->ml_en.push_back(a < L ? energies[eoff[q] + a] : 0.0);
    for (int a = 0; a < F; ++a)
      for (int b = 0; b < F; ++b)
        s->ml_M.push_back(a < L && b < L ? mop[moff[q] + a * L + b] : 0.0);
    for (int a = 0; a < F; ++a)
      for (int b = 0; b < F; ++b)
        for (int c = 0; c < 2; ++c)
          s->ml_rho0.push_back(a < L && b < L ? rho0[2 * (moff[q] + a * L + b) + c] : 0.0);
    for (int c = 0; c < 3; ++c) s->ml_dip.push_back(dipole[3 * q + c]);
    s->ml_gphi.push_back(gphi[q]);
  }
  return rebuild_emitters(s);
}

static mlk_status add_source(mlk_sim* s, const Source& src) {
  if (s->cav_on) return fail(MLK_EUNSUPPORTED, "the cavity replaces the grid: no sources");
  if (s->src.count >= kMaxSources) return fail(MLK_EINVAL, "at most %d sources", kMaxSources);
  if (!(src.tau > 0.0) || !std::isfinite(src.amp) || !std::isfinite(src.omega) ||
      !std::isfinite(src.t0))
    return fail(MLK_EINVAL, "bad source parameters");
  s->src.s[s->src.count++] = src;
  return MLK_OK;
}

mlk_status mlk_add_plane_source(mlk_sim* s, int32_t axis, int32_t index, int32_t comp,
                                double amp, double omega, double tau, double t0) {
  if (!s) return fail(MLK_EINVAL, "null argument");
  if (axis < 0 || axis > 2 || comp < 0 || comp > 2 || index < 0 || index >= s->g.n[axis])
    return fail(MLK_EINVAL, "bad plane source axis/index/component");
  Source src{};
  src.kind = 0;
  src.axis = axis;
  src.index = index;
  src.comp = comp;
  src.amp = amp;
  src.omega = omega;
  src.tau = tau;
  src.t0 = t0;
  return add_source(s, src);
}

mlk_status mlk_add_point_source(mlk_sim* s, int32_t comp, const int32_t ijk[3], double amp,
                                double omega, double tau, double t0) {
  if (!s || !ijk) return fail(MLK_EINVAL, "null argument");
  if (comp < 0 || comp > 2) return fail(MLK_EINVAL, "bad component");
  for (int a = 0; a < 3; ++a)
    if (ijk[a] < 0 || ijk[a] >= s->g.n[a]) return fail(MLK_EINVAL, "point source outside grid");
  Source src{};
  src.kind = 1;
  src.comp = comp;
  for (int a = 0; a < 3; ++a) src.ijk[a] = ijk[a];
  src.amp = amp;
  src.omega = omega;
  src.tau = tau;
  src.t0 = t0;
  return add_source(s, src);
}

mlk_status mlk_add_probe(mlk_sim* s, int32_t comp, const int32_t ijk[3], int32_t* id) {
  if (!s || !ijk) return fail(MLK_EINVAL, "null argument");
  if (s->host_step > 0) return fail(MLK_ESTATE, "probes must be added before stepping");
  if (s->cav_on) return fail(MLK_EUNSUPPORTED, "the cavity replaces the grid: no probes");
  if (s->nprobe >= 16) return fail(MLK_EINVAL, "at most 16 probes");
  if (comp < 0 || comp > 5) return fail(MLK_EINVAL, "bad component");
  for (int a = 0; a < 3; ++a)
    if (ijk[a] < 0 || ijk[a] >= s->g.n[a]) return fail(MLK_EINVAL, "probe outside grid");
  const int p = s->nprobe++;
  s->probe_comp[p] = comp;
  s->probe_idx[p] = (int64_t)cell_index(s->g, ijk[0], ijk[1], ijk[2]);
  if (id) *id = p;
  dfree(s->d_probe);
  s->series_cap = 0;
  return MLK_OK;
}

mlk_status mlk_add_flux_plane(mlk_sim* s, int32_t axis, int32_t index) {
  if (!s) return fail(MLK_EINVAL, "null argument");
  if (s->host_step > 0) return fail(MLK_ESTATE, "detectors must be added before stepping");
  if (s->fp.on) return fail(MLK_EINVAL, "one flux plane per simulation");
  if (s->cav_on) return fail(MLK_EUNSUPPORTED, "the cavity replaces the grid: no flux plane");
  if (axis < 0 || axis > 2 || index < 1 || index >= s->g.n[axis])
    return fail(MLK_EINVAL, "flux plane index must be 1..n-1");
  const int u = (axis + 1) % 3, v = (axis + 2) % 3;
  const size_t np = (size_t)s->g.n[u] * s->g.n[v];
  s->fp.axis = axis;
  s->fp.index = index;
  s->fp.nblocks = (int)std::min<size_t>((np + 255) / 256, 1024);
  HIPCHK(dalloc(&s->fp.Eu0, np * sizeof(double)));
  HIPCHK(dalloc(&s->fp.Ev0, np * sizeof(double)));
  HIPCHK(dalloc(&s->fp.partial, (size_t)s->fp.nblocks * sizeof(double)));
  HIPCHK(dalloc(&s->fp.total, sizeof(double)));
  HIPCHK(hipMemset(s->fp.total, 0, sizeof(double)));
  s->fp.on = 1;
  dfree(s->d_probe);
  s->series_cap = 0;
  return MLK_OK;
}

mlk_status mlk_buffer_bytes(mlk_sim* s, size_t bytes[4]) {
  if (!s || !bytes) return fail(MLK_EINVAL, "null argument");
  bytes[0] = s->ncell * s->esz;
  bytes[1] = psi_total(s->g) * s->esz;
  bytes[2] = s->tls_gid.size() * 3 * sizeof(double);
  bytes[3] = s->ml_gid.size() * 2 * kMaxLevels * kMaxLevels * sizeof(double);
  return MLK_OK;
}

mlk_status mlk_get_field_set(mlk_sim* s, int32_t* set) {
  if (!s || !set) return fail(MLK_EINVAL, "null argument");
  *set = s->swapped ? 1 : 0;
  return MLK_OK;
}

mlk_status mlk_bind_device_buffers(mlk_sim* s, const mlk_buffers* b) {
  if (!s || !b) return fail(MLK_EINVAL, "null argument");
  if (s->in_batch) return fail(MLK_ESTATE, "the sim belongs to a batch");
  const bool fused = s->desc.sweep == MLK_SWEEP_FUSED;
  const size_t fbytes = s->ncell * s->esz, pbytes = psi_total(s->g) * s->esz;
  const size_t tbytes = s->tls_gid.size() * 3 * sizeof(double);
  const size_t mbytes = s->ml_gid.size() * 2 * kMaxLevels * kMaxLevels * sizeof(double);
  auto aligned = [](const void* p) { return ((uintptr_t)p & 15u) == 0; };
  for (int q = 0; q < 2; ++q) {
    for (int c = 0; c < 6; ++c)
      if (b->field[q][c] && (!aligned(b->field[q][c]) || (q == 1 && !fused)))
        return fail(MLK_EINVAL, "field set %d component %d: %s", q, c,
                    q == 1 && !fused ? "the plain sweep has one field set" : "not 16-byte aligned");
    if (b->psi[q] && (!aligned(b->psi[q]) || pbytes == 0 || (q == 1 && !fused)))
      return fail(MLK_EINVAL, "psi set %d: no such buffer, or not 16-byte aligned", q);
  }
  if ((b->tls_state && (tbytes == 0 || !aligned(b->tls_state))) ||
      (b->ml_state && (mbytes == 0 || !aligned(b->ml_state))))
    return fail(MLK_EINVAL, "emitter state buffer without emitters, or not 16-byte aligned");
  HIPCHK(hipSetDevice(s->desc.device));
  STCHK(sync_sim(s));
  // move the contents into the caller's buffer, free the library's, use the caller's
  auto adopt = [&](void*& slot, void* dst, size_t bytes) -> mlk_status {
    if (!dst || dst == slot) return MLK_OK;
    if (slot && bytes) HIPCHK(hipMemcpy(dst, slot, bytes, hipMemcpyDeviceToDevice));
    if (std::find(s->borrowed.begin(), s->borrowed.end(), slot) == s->borrowed.end()) dfree(slot);
    slot = dst;
    s->borrowed.push_back(dst);
    return MLK_OK;
  };
  const int cur = s->swapped ? 1 : 0;
  for (int q = 0; q < 2; ++q) {
    const bool here = q == cur;  // set q is the one the sim reads now
    for (int c = 0; c < 3; ++c) {
      STCHK(adopt(here ? s->E[c] : s->E2[c], b->field[q][c], fbytes));
      STCHK(adopt(here ? s->H[c] : s->H2[c], b->field[q][3 + c], fbytes));
    }
    STCHK(adopt(here ? s->psi : s->psi2, b->psi[q], pbytes));
  }
  if (b->tls_state) {
    void* p = s->d_tls_rho;
    STCHK(adopt(p, b->tls_state, tbytes));
    s->d_tls_rho = (double*)p;
  }
  if (b->ml_state) {
    void* p = s->d_ml_rho;
    STCHK(adopt(p, b->ml_state, mbytes));
    s->d_ml_rho = (double*)p;
  }
  if (b->tls_state || b->ml_state) s->states_bound = true;
  return MLK_OK;
}

mlk_status mlk_record_energy(mlk_sim* s, int32_t every) {
  if (!s) return fail(MLK_EINVAL, "null argument");
  if (s->host_step > 0) return fail(MLK_ESTATE, "detectors must be set before stepping");
  if (s->in_batch) return fail(MLK_ESTATE, "the sim belongs to a batch");
  if (every < 0) return fail(MLK_EINVAL, "every must be >= 0");
  if (every > 0 && s->desc.sweep != MLK_SWEEP_FUSED)
    return fail(MLK_EUNSUPPORTED, "the energy detector reads both field buffers of the fused sweep");
  if (s->cav_on) return fail(MLK_EUNSUPPORTED, "the cavity replaces the grid: no field energy");
  HIPCHK(hipSetDevice(s->desc.device));
  dfree(s->er.series);
  dfree(s->er.partial);
  s->energy_cap = 0;
  s->er.every = every;
  if (every == 0) return MLK_OK;
  s->er.nblocks = (int)std::max<size_t>(1, std::min<size_t>((s->ncell + 255) / 256, 1024));
  s->er.dv = s->g.dx * s->g.dx * s->g.dx;
  HIPCHK(dalloc(&s->er.partial, (size_t)s->er.nblocks * sizeof(double)));
  return MLK_OK;
}

mlk_status mlk_record_populations(mlk_sim* s, int32_t every) {
  if (!s) return fail(MLK_EINVAL, "null argument");
  if (s->host_step > 0) return fail(MLK_ESTATE, "detectors must be set before stepping");
  if (every < 0) return fail(MLK_EINVAL, "every must be >= 0");
  s->pop_every = every;
  dfree(s->d_pop);
  s->pop_cap = 0;
  return MLK_OK;
}

mlk_status mlk_step(mlk_sim* s, int64_t nsteps) {
  if (!s) return fail(MLK_EINVAL, "null argument");
  if (nsteps < 0) return fail(MLK_EINVAL, "negative step count");
  if (nsteps == 0) return MLK_OK;
  HIPCHK(hipSetDevice(s->desc.device));
  if (s->batch_stream) HIPCHK(hipStreamSynchronize(s->batch_stream));
  STCHK(reserve_series(s, nsteps));
  mlk_status st = s->cav_on ? enqueue_cavity_steps(s, nsteps)
                  : s->fp32 ? enqueue_steps<float>(s, nsteps)
                            : enqueue_steps<double>(s, nsteps);
  if (st == MLK_OK) s->host_step += nsteps;
  return st;
}

}  // extern "C"

namespace {

// Classical-path steps shared by the two entry points.  With host buffers the field
// and the recorded states pass through device staging of `cap` doubles at stage,
// K steps at a time (K >= 1, checked by the caller); with device buffers stage is
// not used.
mlk_status prescribed_steps(mlk_sim* s, int64_t nsteps, const double* Et, bool host,
                            double* tls_out, double* stage, int64_t K) {
  const size_t per = 3 * (size_t)s->nem, nt = s->tls_gid.size();
  const TlsPtrs tls = tls_ptrs(s);
  const MlDev ml = ml_dev(s);
  Series ser = series_of(s);
  ser.pop_every = 0;  // no series: the step counter does not move
  double* dE = host ? stage : nullptr;
  double* dO = host ? stage + (size_t)K * per : nullptr;
  if (!host) K = nsteps;
  for (int64_t c0 = 0; c0 < nsteps; c0 += K) {
    const int64_t kc = std::min(K, nsteps - c0);
    const double* e = host ? dE : Et + (size_t)c0 * per;
    double* o = tls_out && nt ? (host ? dO : tls_out + (size_t)c0 * 3 * nt) : nullptr;
    if (host)
      HIPCHK(hipMemcpyAsync(dE, Et + (size_t)c0 * per, (size_t)kc * per * sizeof(double),
                            hipMemcpyHostToDevice, s->stream));
    for (int64_t q = 0; q < kc; ++q) {
      const double* eq = e + (size_t)q * per;
      HIPCHK(tls_step(tls, s->g.dt, eq, s->d_mudot, s->d_popoff, ser, s->d_step, s->stream));
      if (ml.count > 0)
        HIPCHK(ml_step(ml, s->ml_range, s->g.dt, eq, s->d_mudot, s->d_popoff, ser, s->d_step,
                       s->stream));
      if (o)
        HIPCHK(hipMemcpyAsync(o + (size_t)q * 3 * nt, s->d_tls_rho, 3 * nt * sizeof(double),
                              hipMemcpyDeviceToDevice, s->stream));
    }
    // E~ of the last step, as mlk_get_emitter_io reports it
    if (c0 + kc == nsteps)
      HIPCHK(hipMemcpyAsync(s->d_Et, e + (size_t)(kc - 1) * per, per * sizeof(double),
                            hipMemcpyDeviceToDevice, s->stream));
    if (host && o)
      HIPCHK(hipMemcpyAsync(tls_out + (size_t)c0 * 3 * nt, dO, (size_t)kc * 3 * nt * sizeof(double),
                            hipMemcpyDeviceToHost, s->stream));
    if (host) HIPCHK(hipStreamSynchronize(s->stream));  // staging is reused
  }
  return MLK_OK;
}

// Argument checks shared by the two entry points; *go is false when there is
// nothing to do.
mlk_status prescribed_args(mlk_sim* s, int64_t nsteps, const double* Et, int32_t mem_kind,
                           bool* go) {
  *go = false;
  if (!s) return fail(MLK_EINVAL, "null argument");
  if (nsteps < 0) return fail(MLK_EINVAL, "negative step count");
  if (mem_kind != MLK_MEM_HOST && mem_kind != MLK_MEM_DEVICE) return fail(MLK_EINVAL, "bad mem_kind");
  if (s->cav_on) return fail(MLK_ESTATE, "the cavity sets the field");
  if (nsteps == 0 || s->nem == 0) return MLK_OK;
  if (!Et) return fail(MLK_EINVAL, "null field");
  HIPCHK(hipSetDevice(s->desc.device));
  if (s->batch_stream) HIPCHK(hipStreamSynchronize(s->batch_stream));
  *go = true;
  return MLK_OK;
}

}  // namespace

extern "C" {

mlk_status mlk_step_prescribed_wave(mlk_sim* s, int64_t nsteps, const double pol[3], double amp,
                                    double omega, double tau, double t0, double z0,
                                    double t_start, double* tls_out) {
  if (!pol) return fail(MLK_EINVAL, "null polarisation");
  for (double v : {pol[0], pol[1], pol[2], amp, omega, t0, z0, t_start})
    if (!std::isfinite(v)) return fail(MLK_EINVAL, "non-finite pulse parameter");
  if (!(tau > 0.0) || !std::isfinite(tau)) return fail(MLK_EINVAL, "tau must be > 0");
  bool go = false;
  STCHK(prescribed_args(s, nsteps, pol, MLK_MEM_HOST, &go));
  if (!go) return MLK_OK;
  const size_t nt = s->tls_gid.size();
  const TlsPtrs tls = tls_ptrs(s);
  const MlDev ml = ml_dev(s);
  Series ser = series_of(s);
  ser.pop_every = 0;  // no series: the step counter does not move
  WaveDesc w{};
  for (int c = 0; c < 3; ++c) w.pol[c] = pol[c];
  w.amp = amp;
  w.omega = omega;
  w.tau = tau;
  w.t0 = t0;
  w.z0 = z0;
  // recorded states go through device staging of at most about 64 MB at a time
  const int64_t K = tls_out && nt ? std::max<int64_t>(1, std::min<int64_t>(
                                        nsteps, (int64_t)((64u << 20) / (24 * nt))))
                                  : nsteps;
  DevBuf<double> stage;
  if (tls_out && nt) HIPCHK(stage.alloc((size_t)K * 3 * nt));
  for (int64_t c0 = 0; c0 < nsteps; c0 += K) {
    const int64_t kc = std::min(K, nsteps - c0);
    for (int64_t q = 0; q < kc; ++q) {
      const double t = t_start + (double)(c0 + q) * s->g.dt;
      HIPCHK(wave_field(s->nem, s->d_pos, s->d_gamma, w, t, s->d_Et, s->stream));
      HIPCHK(tls_step(tls, s->g.dt, s->d_Et, s->d_mudot, s->d_popoff, ser, s->d_step, s->stream));
      if (ml.count > 0)
        HIPCHK(ml_step(ml, s->ml_range, s->g.dt, s->d_Et, s->d_mudot, s->d_popoff, ser,
                       s->d_step, s->stream));
      if (stage.p)
        HIPCHK(hipMemcpyAsync(stage.p + (size_t)q * 3 * nt, s->d_tls_rho, 3 * nt * sizeof(double),
                              hipMemcpyDeviceToDevice, s->stream));
    }
    if (stage.p) {
      HIPCHK(hipMemcpyAsync(tls_out + (size_t)c0 * 3 * nt, stage.p,
                            (size_t)kc * 3 * nt * sizeof(double), hipMemcpyDeviceToHost,
                            s->stream));
      HIPCHK(hipStreamSynchronize(s->stream));
    }
  }
  return MLK_OK;
}

mlk_status mlk_step_prescribed(mlk_sim* s, int64_t nsteps, const double* Et, int32_t mem_kind,
                               double* tls_out) {
  bool go = false;
  STCHK(prescribed_args(s, nsteps, Et, mem_kind, &go));
  if (!go) return MLK_OK;
  const bool host = mem_kind == MLK_MEM_HOST;
  const size_t per = 3 * (size_t)s->nem, nt = s->tls_gid.size();
  // host data goes through device staging in chunks of at most about 64 MB
  const int64_t K = host ? std::max<int64_t>(1, std::min<int64_t>(nsteps, (int64_t)((64u << 20) /
                                                                                   (8 * per))))
                         : nsteps;
  DevBuf<double> stage;
  if (host) HIPCHK(stage.alloc((size_t)K * (per + (tls_out ? 3 * nt : 0))));
  return prescribed_steps(s, nsteps, Et, host, tls_out, stage.p, K);
}

}  // extern "C"

namespace {

// Staging of mlk_step_prescribed_noalloc: a fixed device array, one copy on each
// GPU the library runs on, held until the process ends.  In host code its name
// only stands for the symbol: the device address comes from hipGetSymbolAddress,
// taken once per device with that device current, and only that address is
// handed to copies and kernels.
constexpr size_t kScratchDoubles = (size_t)(16u << 20) / sizeof(double);  // 16 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kScratchDevices] = {};

// Device address of the staging array on device dev (current on entry).
mlk_status scratch_address(int dev, double** out) {
  if (dev < 0 || dev >= kScratchDevices)
    return fail(MLK_EUNSUPPORTED, "device %d: the fixed staging covers devices 0..%d", dev,
                kScratchDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return MLK_OK;
}

}  // namespace

extern "C" {

mlk_status mlk_step_prescribed_noalloc(mlk_sim* s, int64_t nsteps, const double* Et,
                                       int32_t mem_kind, double* tls_out) {
  bool go = false;
  STCHK(prescribed_args(s, nsteps, Et, mem_kind, &go));
  if (!go) return MLK_OK;
  if (mem_kind == MLK_MEM_DEVICE)  // device buffers need no staging
    return prescribed_steps(s, nsteps, Et, false, tls_out, nullptr, nsteps);
  const size_t per = 3 * (size_t)s->nem, nt = s->tls_gid.size();
  const size_t need = per + (tls_out ? 3 * nt : 0);  // staging doubles per step
  if (need > kScratchDoubles)
    return fail(MLK_EINVAL,
                "one step of %d emitters needs %zu doubles of staging, more than the %zu of "
                "the fixed staging array",
                s->nem, need, kScratchDoubles);
  const int64_t K = std::min<int64_t>(nsteps, (int64_t)(kScratchDoubles / need));
  double* ptr = nullptr;
  STCHK(scratch_address(s->desc.device, &ptr));
  return prescribed_steps(s, nsteps, Et, true, tls_out, ptr, K);
}

mlk_status mlk_set_cavity(mlk_sim* s, double omega, double volume, const double q0[2],
                          const double p0[2]) {
  if (!s || !q0 || !p0) return fail(MLK_EINVAL, "null argument");
  if (!(omega > 0.0) || !(volume > 0.0) || !std::isfinite(omega) || !std::isfinite(volume))
    return fail(MLK_EINVAL, "cavity frequency and volume must be positive");
  for (int l = 0; l < 2; ++l)
    if (!std::isfinite(q0[l]) || !std::isfinite(p0[l])) return fail(MLK_EINVAL, "bad mode state");
  if (s->host_step > 0) return fail(MLK_ESTATE, "the cavity must be set before stepping");
  if (s->in_batch) return fail(MLK_ESTATE, "the sim belongs to a batch");
  if (s->src.count > 0 || s->nprobe > 0 || s->fp.on || s->npole > 0)
    return fail(MLK_EUNSUPPORTED,
                "the cavity replaces the grid: no sources, probes, flux plane or poles");
  HIPCHK(hipSetDevice(s->desc.device));
  STCHK(sync_sim(s));
  const size_t nt = s->tls_gid.size();
  double st[6] = {q0[0], q0[1], p0[0], p0[1], 0.0, 0.0};
  if (!s->cav.st) HIPCHK(dalloc(&s->cav.st, 6 * sizeof(double)));
  // partial sums: at most 256 blocks in the general path, one per 256 two-level
  // emitters in the two-level path
  const size_t npart = std::max<size_t>(256, (nt + 255) / 256);
  dfree(s->cav.partial);
  HIPCHK(dalloc(&s->cav.partial, 2 * npart * sizeof(double)));
  HIPCHK(hipMemcpy(s->cav.st, st, sizeof(st), hipMemcpyHostToDevice));
  s->cav.w = omega;
  s->cav.V = volume;
  s->cav.eps = omega / std::sqrt(volume);
  // d^0 from the initial states: sum of <mu> + (dt/2) mu_dot
  HIPCHK(cavity_set_dipole(s->cav, tls_ptrs(s), ml_dev(s), s->g.dt, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  s->cav_on = true;
  return MLK_OK;
}

mlk_status mlk_add_susceptibility(mlk_sim* s, const int32_t box[6], double omega0, double gamma,
                                  double sigma, int32_t drude) {
  if (!s || !box) return fail(MLK_EINVAL, "null argument");
  if (s->host_step > 0) return fail(MLK_ESTATE, "poles must be added before stepping");
  if (s->in_batch) return fail(MLK_ESTATE, "the sim belongs to a batch");
  if (s->cav_on) return fail(MLK_EUNSUPPORTED, "the cavity replaces the grid: no poles");
  if (s->npole >= 8) return fail(MLK_EINVAL, "at most 8 poles");
  if (!(omega0 > 0.0) || !(gamma >= 0.0) || !std::isfinite(omega0) || !std::isfinite(gamma) ||
      !std::isfinite(sigma))
    return fail(MLK_EINVAL, "pole needs omega0 > 0, gamma >= 0, finite sigma");
  PoleDev p{};
  for (int a = 0; a < 3; ++a) {
    const int lo = box[a], hi = box[3 + a];
    int lmin = 0, hmax = s->g.n[a];
    if (!s->g.periodic[a]) {
      lmin = std::max(s->g.nlo[a], 1);  // clear of the CPML and of the index-0 wall plane
      hmax = s->g.n[a] - s->g.nhi[a];
    }
    if (lo < lmin || hi > hmax || lo >= hi)
      return fail(MLK_EINVAL, "pole box axis %d: [%d, %d) outside [%d, %d)", a, lo, hi, lmin, hmax);
    p.lo[a] = lo;
    p.n[a] = hi - lo;
  }
  const double dt = s->g.dt, g = 0.5 * gamma * dt, w2 = omega0 * omega0;
  p.a = 2.0 - (drude ? 0.0 : w2 * dt * dt);
  p.b = 1.0 - g;
  p.c = sigma * w2 * dt * dt;
  p.g1 = 1.0 + g;
  const size_t bytes = 3 * (size_t)p.n[0] * p.n[1] * p.n[2] * s->esz;
  HIPCHK(hipSetDevice(s->desc.device));
  STCHK(sync_sim(s));
  HIPCHK(dalloc(&p.P, bytes));
  if (dalloc(&p.Q, bytes) != hipSuccess) {
    dfree(p.P);
    return fail(MLK_ENOMEM, "pole state");
  }
  HIPCHK(hipMemset(p.P, 0, bytes));
  HIPCHK(hipMemset(p.Q, 0, bytes));
  s->pole[s->npole++] = p;
  return MLK_OK;
}

mlk_status mlk_get_cavity(mlk_sim* s, double out[6]) {
  if (!s || !out) return fail(MLK_EINVAL, "null argument");
  if (!s->cav_on) return fail(MLK_ESTATE, "no cavity");
  STCHK(sync_sim(s));
  HIPCHK(hipMemcpy(out, s->cav.st, 6 * sizeof(double), hipMemcpyDeviceToHost));
  return MLK_OK;
}

mlk_status mlk_set_timing(mlk_sim* s, int32_t on) {
  if (!s) return fail(MLK_EINVAL, "null argument");
  STCHK(sync_sim(s));
  s->marks.clear();
  s->next_event = 0;
  for (int p = 0; p < MLK_PHASE_COUNT; ++p) {
    s->phase_ms[p] = 0.0;
    s->phase_n[p] = 0;
  }
  s->timing = on & ((1 << MLK_PHASE_COUNT) - 1);
  return MLK_OK;
}

mlk_status mlk_get_phase_time(mlk_sim* s, int32_t phase, double* total_ms, int64_t* launches) {
  if (!s || !total_ms || !launches) return fail(MLK_EINVAL, "null argument");
  if (phase < 0 || phase >= MLK_PHASE_COUNT) return fail(MLK_EINVAL, "phase %d unknown", phase);
  STCHK(sync_sim(s));
  HIPCHK(collect_marks(s));
  *total_ms = s->phase_ms[phase];
  *launches = s->phase_n[phase];
  return MLK_OK;
}

mlk_status mlk_get_interior_box(mlk_sim* s, int32_t box[6]) {
  if (!s || !box) return fail(MLK_EINVAL, "null argument");
  const Box b = sweep_box(s);
  for (int a = 0; a < 3; ++a) {
    box[a] = b.lo[a];
    box[3 + a] = b.hi[a];
  }
  return MLK_OK;
}

mlk_status mlk_sync(mlk_sim* s) {
  if (!s) return fail(MLK_EINVAL, "null argument");
  return check_numeric(s);
}

mlk_status mlk_step_count(mlk_sim* s, int64_t* n) {
  if (!s || !n) return fail(MLK_EINVAL, "null argument");
  *n = s->host_step;
  return MLK_OK;
}

mlk_status mlk_get_field(mlk_sim* s, int32_t comp, double* dst, int32_t mem_kind) {
  if (!s || !dst) return fail(MLK_EINVAL, "null argument");
  if (comp < 0 || comp > 5) return fail(MLK_EINVAL, "component %d outside 0..5", comp);
  const void* src = comp < 3 ? s->E[comp] : s->H[comp - 3];
  STCHK(sync_sim(s));
  if (mem_kind == MLK_MEM_DEVICE) {
    HIPCHK(convert_out(s->fp32, src, dst, s->ncell, s->stream));
    STCHK(sync_sim(s));
    return MLK_OK;
  }
  double* d = nullptr;
  HIPCHK(dalloc(&d, s->ncell * sizeof(double)));
  hipError_t e = convert_out(s->fp32, src, d, s->ncell, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e == hipSuccess) e = hipMemcpy(dst, d, s->ncell * sizeof(double), hipMemcpyDeviceToHost);
  dfree(d);
  if (e != hipSuccess) return fail(MLK_EDEVICE, "get_field: %s", hipGetErrorString(e));
  return MLK_OK;
}

mlk_status mlk_get_tls_state(mlk_sim* s, int32_t first, int32_t count, double* dst) {
  if (!s || !dst) return fail(MLK_EINVAL, "null argument");
  STCHK(sync_sim(s));
  const int nt = (int)s->tls_gid.size();
  std::vector<double> all((size_t)nt * 3);
  if (nt) HIPCHK(hipMemcpy(all.data(), s->d_tls_rho, all.size() * sizeof(double),
                           hipMemcpyDeviceToHost));
  // map emitter ids to two-level slots
  if (first < 0 || count < 0 || first + count > s->nem)
    return fail(MLK_EINVAL, "emitter range outside 0..%d", s->nem);
  for (int q = 0; q < count; ++q) {
    const int id = first + q;
    const int slot = s->tls_slot[id];
    if (slot < 0) return fail(MLK_EINVAL, "emitter %d is not a two-level emitter", id);
    for (int a = 0; a < 3; ++a) dst[3 * q + a] = all[3 * slot + a];
  }
  return MLK_OK;
}

mlk_status mlk_get_rho(mlk_sim* s, int32_t id, double* dst, int32_t cap, int32_t* nlev) {
  if (!s || !dst) return fail(MLK_EINVAL, "null argument");
  if (id < 0 || id >= s->nem) return fail(MLK_EINVAL, "bad emitter id");
  const int slot = s->ml_slot.empty() ? -1 : s->ml_slot[id];
  if (slot >= 0) {
    int n = 2;
    for (int k = 2; k <= kMaxLevels; ++k)
      if (slot >= s->ml_range[k] && slot < s->ml_range[k + 1]) n = k;
    if (cap < 2 * n * n) return fail(MLK_EINVAL, "dst too small");
    STCHK(sync_sim(s));
    const size_t cnt = s->ml_gid.size();
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b)
        for (int c = 0; c < 2; ++c) {
          const size_t q = (size_t)(2 * (a * kMaxLevels + b) + c) * cnt + slot;
          HIPCHK(hipMemcpy(dst + 2 * (a * n + b) + c, s->d_ml_rho + q, sizeof(double),
                           hipMemcpyDeviceToHost));
        }
    if (nlev) *nlev = n;
    return MLK_OK;
  }
  double st[3];
  STCHK(mlk_get_tls_state(s, id, 1, st));
  if (cap < 8) return fail(MLK_EINVAL, "dst too small");
  dst[0] = 1.0 - st[0];
  dst[1] = 0.0;
  dst[2] = st[1];
  dst[3] = st[2];
  dst[4] = st[1];
  dst[5] = -st[2];
  dst[6] = st[0];
  dst[7] = 0.0;
  if (nlev) *nlev = 2;
  return MLK_OK;
}

mlk_status mlk_get_emitter_io(mlk_sim* s, double* Et, double* mudot) {
  if (!s) return fail(MLK_EINVAL, "null argument");
  STCHK(sync_sim(s));
  const size_t b = (size_t)s->nem * 3 * sizeof(double);
  if (Et && b) HIPCHK(hipMemcpy(Et, s->d_Et, b, hipMemcpyDeviceToHost));
  if (mudot && b) HIPCHK(hipMemcpy(mudot, s->d_mudot, b, hipMemcpyDeviceToHost));
  return MLK_OK;
}

mlk_status mlk_get_series(mlk_sim* s, int32_t kind, int32_t id, double* dst, int64_t cap,
                          int64_t* len) {
  if (!s) return fail(MLK_EINVAL, "null argument");
  STCHK(sync_sim(s));
  int64_t n = 0;
  const double* src = nullptr;
  if (kind == MLK_SERIES_PROBE) {
    if (id < 0 || id >= s->nprobe) return fail(MLK_EINVAL, "bad probe id");
    n = s->host_step;
    src = s->d_probe ? s->d_probe + (size_t)id * s->series_cap : nullptr;
  } else if (kind == MLK_SERIES_FLUX) {
    if (!s->fp.on) return fail(MLK_EINVAL, "no flux plane");
    n = s->host_step;
    src = s->d_flux_series;
  } else if (kind == MLK_SERIES_POPULATION) {
    const int64_t rec =
        (s->pop_every > 0 && s->host_step > 0) ? (s->host_step - 1) / s->pop_every + 1 : 0;
    n = rec * s->npop;
    src = s->d_pop;
  } else if (kind == MLK_SERIES_ENERGY) {
    if (s->er.every <= 0) return fail(MLK_EINVAL, "no energy record");
    n = s->host_step > 0 ? (s->host_step - 1) / s->er.every + 1 : 0;
    src = s->er.series;
  } else {
    return fail(MLK_EINVAL, "bad series kind");
  }
  if (len) *len = n;
  if (dst && n > 0 && src) {
    const int64_t m = n < cap ? n : cap;
    HIPCHK(hipMemcpy(dst, src, (size_t)m * sizeof(double), hipMemcpyDeviceToHost));
  }
  return MLK_OK;
}

mlk_status mlk_get_flux_total(mlk_sim* s, double* total) {
  if (!s || !total) return fail(MLK_EINVAL, "null argument");
  if (!s->fp.on) return fail(MLK_EINVAL, "no flux plane");
  STCHK(sync_sim(s));
  HIPCHK(hipMemcpy(total, s->fp.total, sizeof(double), hipMemcpyDeviceToHost));
  return MLK_OK;
}

mlk_status mlk_checkpoint_size(mlk_sim* s, size_t* bytes) {
  if (!s || !bytes) return fail(MLK_EINVAL, "null argument");
  size_t b = 0;
  for (const Piece& p : state_pieces(s)) b += p.bytes;
  *bytes = b;
  return MLK_OK;
}

mlk_status mlk_checkpoint_save(mlk_sim* s, void* dst, int32_t mem_kind) {
  if (!s || !dst) return fail(MLK_EINVAL, "null argument");
  STCHK(sync_sim(s));
  char* o = (char*)dst;
  const hipMemcpyKind kind =
      mem_kind == MLK_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  for (const Piece& p : state_pieces(s)) {
    HIPCHK(hipMemcpy(o, p.p, p.bytes, kind));
    o += p.bytes;
  }
  return MLK_OK;
}

mlk_status mlk_checkpoint_load(mlk_sim* s, const void* src, int32_t mem_kind) {
  if (!s || !src) return fail(MLK_EINVAL, "null argument");
  STCHK(load_state(s, src, mem_kind));
  // a new state: the watchdog starts afresh
  const unsigned long long zero = 0;
  HIPCHK(hipMemcpy(s->d_numeric, &zero, sizeof(zero), hipMemcpyHostToDevice));
  return MLK_OK;
}

}  // extern "C"

// ====================================================================== adjoint
//
// Checkpointed reverse pass: the forward run saves the whole state every K
// steps in device memory; then, segment by segment from the last, the state is
// restored, the K steps are run again while a tape records what the reverse
// steps need (E on the design box, the flux planes, every emitter's state
// before the step and its E~), and the adjoint steps undo them in reverse.
// Memory: one state per segment plus one segment of tape.  The sim is left as
// it was before the call.

namespace {

template <typename T>
mlk_status adjoint_run(mlk_sim* s, int kind, const double* weights, int64_t T_steps, int K,
                       const Box& box, double* grad_eps, double* grad_dip, double* value) {
  constexpr bool f32 = sizeof(T) == 4;
  hipStream_t st = s->stream;
  const int M = s->nem, nt = (int)s->tls_gid.size();
  const size_t nc = s->ncell;
  const size_t nb = (size_t)(box.hi[0] - box.lo[0]) * (box.hi[1] - box.lo[1]) * (box.hi[2] - box.lo[2]);
  const int np = s->fp.on ? s->g.n[(s->fp.axis + 1) % 3] * s->g.n[(s->fp.axis + 2) % 3] : 0;
  const int nseg = (int)((T_steps + K - 1) / K);
  size_t ck = 0;
  STCHK(mlk_checkpoint_size(s, &ck));
  STCHK(reserve_series(s, T_steps));
  const int64_t step0 = s->host_step;

  DevBuf<char> ckpt;
  HIPCHK(ckpt.alloc(ck * (size_t)nseg));
  hipEvent_t ev[3];
  for (auto& e : ev) HIPCHK(hipEventCreate(&e));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() {
      for (int q = 0; q < 3; ++q) (void)hipEventDestroy(e[q]);
    }
  } ev_guard{ev};
  HIPCHK(hipEventRecord(ev[0], st));
  double ftot0 = 0.0;
  if (s->fp.on) HIPCHK(hipMemcpy(&ftot0, s->fp.total, sizeof(double), hipMemcpyDeviceToHost));
  // forward pass with the checkpoints
  for (int seg = 0; seg < nseg; ++seg) {
    STCHK(mlk_checkpoint_save(s, ckpt.p + ck * (size_t)seg, MLK_MEM_DEVICE));
    const int64_t ns = std::min<int64_t>(K, T_steps - (int64_t)seg * K);
    STCHK(enqueue_steps<T>(s, ns));
    s->host_step += ns;
  }
  HIPCHK(hipEventRecord(ev[1], st));
  STCHK(sync_sim(s));
  double J = 0.0;
  if (kind == MLK_OBJ_FLUX) {
    double f1 = 0.0;
    HIPCHK(hipMemcpy(&f1, s->fp.total, sizeof(double), hipMemcpyDeviceToHost));
    J = f1 - ftot0;
  } else {
    std::vector<double> rho((size_t)nt * 3);
    if (nt) HIPCHK(hipMemcpy(rho.data(), s->d_tls_rho, rho.size() * sizeof(double),
                             hipMemcpyDeviceToHost));
    for (int m = 0; m < nt; ++m) J += weights[s->tls_gid[m]] * rho[3 * m];
  }
  *value = J;

  // adjoint state; a fused-sweep sim takes the transposed sweep out of place
  // (fused box plus shell), with two sets of adjoint fields used in turn
  const bool oop = s->desc.sweep == MLK_SWEEP_FUSED;
  DevBuf<T> Eb[2][3], Hb[2][3], psib[2];
  for (int q = 0; q < (oop ? 2 : 1); ++q)
    for (int c = 0; c < 3; ++c) {
      HIPCHK(Eb[q][c].alloc(nc));
      HIPCHK(Hb[q][c].alloc(nc));
      HIPCHK(hipMemsetAsync(Eb[q][c].p, 0, nc * sizeof(T), st));
      HIPCHK(hipMemsetAsync(Hb[q][c].p, 0, nc * sizeof(T), st));
    }
  const size_t npsi = psi_total(s->g);
  for (int q = 0; q < 2; ++q) {
    HIPCHK(psib[q].alloc(npsi));
    if (npsi) HIPCHK(hipMemsetAsync(psib[q].p, 0, npsi * sizeof(T), st));
  }
  DevBuf<double> sb, gd, mub, etb, geps;
  HIPCHK(sb.alloc((size_t)3 * nt));
  HIPCHK(gd.alloc((size_t)3 * nt));
  HIPCHK(mub.alloc((size_t)3 * M));
  HIPCHK(etb.alloc((size_t)3 * M));
  HIPCHK(geps.alloc(nb));
  if (nt) HIPCHK(hipMemsetAsync(gd.p, 0, (size_t)3 * nt * sizeof(double), st));
  if (M) HIPCHK(hipMemsetAsync(etb.p, 0, (size_t)3 * M * sizeof(double), st));
  if (nb) HIPCHK(hipMemsetAsync(geps.p, 0, nb * sizeof(double), st));
  if (nt) {
    std::vector<double> s0((size_t)3 * nt, 0.0);
    if (kind == MLK_OBJ_POPULATION)
      for (int m = 0; m < nt; ++m) s0[3 * m] = weights[s->tls_gid[m]];
    HIPCHK(hipMemcpy(sb.p, s0.data(), s0.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  // tape of one segment
  DevBuf<T> tbox;
  DevBuf<double> ts, tg, tf;
  HIPCHK(tbox.alloc(nb * 3 * (size_t)(K + 1)));
  HIPCHK(ts.alloc((size_t)3 * nt * K));
  HIPCHK(tg.alloc((size_t)3 * M * K));
  HIPCHK(tf.alloc((size_t)8 * np * K));

  const WindowPtrs<T> win = window_ptrs<T>(s);
  const BinPtrs bins = bin_ptrs(s);
  const TlsPtrs tls = tls_ptrs(s);
  AdjSweep<T> adj{};
  FieldPtrs<T> fb{};  // the adjoint of E as a field, for the gather and the scatter
  int cur = 0;        // the set holding the current adjoint fields
  auto bind = [&]() {
    for (int c = 0; c < 3; ++c) {
      adj.E[c] = Eb[cur][c].p;
      adj.H[c] = Hb[cur][c].p;
      adj.Eo[c] = oop ? Eb[cur ^ 1][c].p : nullptr;
      adj.Ho[c] = oop ? Hb[cur ^ 1][c].p : nullptr;
      fb.E[c] = Eb[cur][c].p;
    }
  };
  bind();
  adj.epsinv = (const T*)s->epsinv;
  adj.tab = (const T*)s->tab;
  adj.psi[0] = psib[0].p;
  adj.psi[1] = psib[1].p;
  adj.kz = 16;
  adj.vacuum = s->vacuum;
  // in vacuum the adjoint gather reads no 1/eps_r (the scatter never does)
  fb.epsinv = s->vacuum ? nullptr : (T*)s->epsinv;
  const double mub_scale = -s->g.dt * s->g.inv_dx * s->g.inv_dx * s->g.inv_dx;
  const FluxPlane* fpp = s->fp.on ? &s->fp : nullptr;

  for (int seg = nseg - 1; seg >= 0; --seg) {
    STCHK(load_state(s, ckpt.p + ck * (size_t)seg, MLK_MEM_DEVICE));
    const int64_t ns = std::min<int64_t>(K, T_steps - (int64_t)seg * K);
    // recompute the segment, recording the tape
    if (nb) {
      if constexpr (f32) HIPCHK(pack_tape_f32(field_ptrs<T>(s), s->g, box, tbox.p, nullptr, nullptr, st));
      else HIPCHK(pack_tape_f64(field_ptrs<T>(s), s->g, box, tbox.p, nullptr, nullptr, st));
    }
    for (int64_t q = 0; q < ns; ++q) {
      if (nt) HIPCHK(hipMemcpyAsync(ts.p + (size_t)3 * nt * q, s->d_tls_rho,
                                    (size_t)3 * nt * sizeof(double), hipMemcpyDeviceToDevice, st));
      STCHK(enqueue_steps<T>(s, 1));
      s->host_step += 1;
      if (M) HIPCHK(hipMemcpyAsync(tg.p + (size_t)3 * M * q, s->d_Et, (size_t)3 * M * sizeof(double),
                                   hipMemcpyDeviceToDevice, st));
      T* bo = nb ? tbox.p + nb * 3 * (size_t)(q + 1) : nullptr;
      double* fo = kind == MLK_OBJ_FLUX ? tf.p + (size_t)8 * np * q : nullptr;
      if constexpr (f32) HIPCHK(pack_tape_f32(field_ptrs<T>(s), s->g, box, bo, fpp, fo, st));
      else HIPCHK(pack_tape_f64(field_ptrs<T>(s), s->g, box, bo, fpp, fo, st));
    }
    // reverse steps
    for (int64_t q = ns - 1; q >= 0; --q) {
      const double* tfq = tf.p + (size_t)8 * np * q;
      if (kind == MLK_OBJ_FLUX) {
        if constexpr (f32) HIPCHK(adj_flux_f32(adj, s->g, s->fp.axis, s->fp.index, tfq, 0, st));
        else HIPCHK(adj_flux_f64(adj, s->g, s->fp.axis, s->fp.index, tfq, 0, st));
      }
      if (nb) {
        const T* e0 = tbox.p + nb * 3 * (size_t)q;
        const T* e1 = tbox.p + nb * 3 * (size_t)(q + 1);
        if constexpr (f32) HIPCHK(adj_eps_f32(adj, s->g, box, e0, e1, geps.p, st));
        else HIPCHK(adj_eps_f64(adj, s->g, box, e0, e1, geps.p, st));
      }
      if (M) {
        if constexpr (f32) HIPCHK(gather_epsw_f32(fb, s->g, bins, win, mub.p, st));
        else HIPCHK(gather_epsw_f64(fb, s->g, bins, win, mub.p, st));
      }
      if constexpr (f32) HIPCHK(adj_sweep_f32(adj, s->g, st));
      else HIPCHK(adj_sweep_f64(adj, s->g, st));
      std::swap(adj.psi[0], adj.psi[1]);
      if (oop) {
        cur ^= 1;
        bind();
      }
      if (nt) {
        HIPCHK(adj_tls(tls, s->g.dt, mub_scale, ts.p + (size_t)3 * nt * q,
                       tg.p + (size_t)3 * M * q, mub.p, sb.p, gd.p, etb.p, st));
        if constexpr (f32) HIPCHK(scatter_plain_f32(fb, s->g, bins, win, etb.p, -1.0, st));
        else HIPCHK(scatter_plain_f64(fb, s->g, bins, win, etb.p, -1.0, st));
      }
      if (kind == MLK_OBJ_FLUX) {
        if constexpr (f32) HIPCHK(adj_flux_f32(adj, s->g, s->fp.axis, s->fp.index, tfq, 1, st));
        else HIPCHK(adj_flux_f64(adj, s->g, s->fp.axis, s->fp.index, tfq, 1, st));
      }
    }
  }
  HIPCHK(hipEventRecord(ev[2], st));
  HIPCHK(hipEventSynchronize(ev[2]));
  float f_ms = 0.f, r_ms = 0.f;
  HIPCHK(hipEventElapsedTime(&f_ms, ev[0], ev[1]));
  HIPCHK(hipEventElapsedTime(&r_ms, ev[1], ev[2]));
  s->adj_forward_ms = f_ms;
  s->adj_reverse_ms = r_ms;
  // back to the state before the call
  STCHK(load_state(s, ckpt.p, MLK_MEM_DEVICE));
  s->host_step = step0;
  STCHK(sync_sim(s));
  if (nb && grad_eps) HIPCHK(hipMemcpy(grad_eps, geps.p, nb * sizeof(double), hipMemcpyDeviceToHost));
  if (grad_dip) {
    std::vector<double> g((size_t)3 * nt);
    if (nt) HIPCHK(hipMemcpy(g.data(), gd.p, g.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int e = 0; e < 3 * M; ++e) grad_dip[e] = 0.0;
    for (int m = 0; m < nt; ++m)
      for (int c = 0; c < 3; ++c) grad_dip[3 * s->tls_gid[m] + c] = g[3 * m + c];
  }
  return MLK_OK;
}

}  // namespace

extern "C" {

mlk_status mlk_adjoint(mlk_sim* s, const mlk_objective* obj, int64_t nsteps, int32_t ckpt_every,
                       const int32_t box[6], double* grad_eps, double* grad_dipole,
                       double* value) {
  if (!s || !obj || !box || !value) return fail(MLK_EINVAL, "null argument");
  if (s->in_batch) return fail(MLK_ESTATE, "the sim belongs to a batch");
  if (s->cav_on) return fail(MLK_EUNSUPPORTED, "the adjoint covers the grid, not the cavity");
  if (s->npole > 0) return fail(MLK_EUNSUPPORTED, "the adjoint covers non-dispersive media only");
  if (nsteps <= 0 || ckpt_every <= 0) return fail(MLK_EINVAL, "steps and checkpoint interval must be positive");
  if (!s->ml_gid.empty()) return fail(MLK_EUNSUPPORTED, "the adjoint covers two-level emitters only");
  if (obj->kind == MLK_OBJ_FLUX) {
    if (!s->fp.on) return fail(MLK_EINVAL, "the flux objective needs a flux plane");
  } else if (obj->kind == MLK_OBJ_POPULATION) {
    if (!obj->weights) return fail(MLK_EINVAL, "the population objective needs weights");
  } else {
    return fail(MLK_EINVAL, "unknown objective %d", obj->kind);
  }
  Box b{};
  for (int a = 0; a < 3; ++a) {
    b.lo[a] = box[a];
    b.hi[a] = box[3 + a];
    if (b.lo[a] < 0 || b.hi[a] > s->g.n[a] || b.lo[a] > b.hi[a])
      return fail(MLK_EINVAL, "design box outside the grid");
  }
  HIPCHK(hipSetDevice(s->desc.device));
  STCHK(sync_sim(s));
  const int K = (int)std::min<int64_t>(ckpt_every, nsteps);
  unsigned long long before = 0, after = 0;
  STCHK(read_numeric(s, &before));
  STCHK(s->fp32 ? adjoint_run<float>(s, obj->kind, obj->weights, nsteps, K, b, grad_eps,
                                     grad_dipole, value)
                : adjoint_run<double>(s, obj->kind, obj->weights, nsteps, K, b, grad_eps,
                                      grad_dipole, value));
  // the runs inside the call leave the watchdog as they found it, and report
  STCHK(read_numeric(s, &after));
  if (after != before) {
    HIPCHK(hipMemcpy(s->d_numeric, &before, sizeof(before), hipMemcpyHostToDevice));
    return fail(MLK_ENUMERIC, "non-finite state in the adjoint's forward runs at step %llu",
                after - 1);
  }
  if (!std::isfinite(*value)) return fail(MLK_ENUMERIC, "non-finite objective");
  return MLK_OK;
}

mlk_status mlk_get_adjoint_times(mlk_sim* s, double* forward_ms, double* reverse_ms) {
  if (!s || !forward_ms || !reverse_ms) return fail(MLK_EINVAL, "null argument");
  *forward_ms = s->adj_forward_ms;
  *reverse_ms = s->adj_reverse_ms;
  return MLK_OK;
}

mlk_status mlk_set_eps_box(mlk_sim* s, const int32_t box[6], const double* eps, int32_t mem_kind) {
  if (!s || !box || !eps) return fail(MLK_EINVAL, "null argument");
  Box b{};
  size_t nb = 1;
  for (int a = 0; a < 3; ++a) {
    b.lo[a] = box[a];
    b.hi[a] = box[3 + a];
    if (b.lo[a] < 0 || b.hi[a] > s->g.n[a] || b.lo[a] > b.hi[a])
      return fail(MLK_EINVAL, "box outside the grid");
    nb *= (size_t)(b.hi[a] - b.lo[a]);
  }
  if (nb == 0) return MLK_OK;
  std::vector<double> h(nb);
  if (mem_kind == MLK_MEM_DEVICE) {
    STCHK(sync_sim(s));
    HIPCHK(hipMemcpy(h.data(), eps, nb * sizeof(double), hipMemcpyDeviceToHost));
  } else {
    std::memcpy(h.data(), eps, nb * sizeof(double));
  }
  bool vac = true;
  for (double v : h) {
    if (!(v >= 1.0) || !std::isfinite(v)) return fail(MLK_EINVAL, "eps_r must be finite and >= 1");
    vac = vac && v == 1.0;
  }
  STCHK(sync_sim(s));
  double* d = nullptr;
  HIPCHK(dalloc(&d, nb * sizeof(double)));
  hipError_t e = hipMemcpy(d, h.data(), nb * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = s->fp32 ? eps_box_f32(d, s->g, b, (float*)s->epsinv, s->stream)
                : eps_box_f64(d, s->g, b, (double*)s->epsinv, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  dfree(d);
  HIPCHK(e);
  s->vacuum = s->vacuum && vac;
  return MLK_OK;
}

mlk_status mlk_set_tls_dipoles(mlk_sim* s, int32_t first, int32_t count, const double* dipole) {
  if (!s || !dipole) return fail(MLK_EINVAL, "null argument");
  if (first < 0 || count < 0 || first + count > s->nem)
    return fail(MLK_EINVAL, "emitter range outside 0..%d", s->nem);
  for (int q = 0; q < count; ++q)
    if (s->tls_slot[first + q] < 0)
      return fail(MLK_EINVAL, "emitter %d is not a two-level emitter", first + q);
  STCHK(sync_sim(s));
  for (int q = 0; q < count; ++q) {
    const int m = s->tls_slot[first + q];
    for (int c = 0; c < 3; ++c) s->tls_dip[3 * m + c] = dipole[3 * q + c];
  }
  HIPCHK(hipMemcpy(s->d_tls_dip, s->tls_dip.data(), s->tls_dip.size() * sizeof(double),
                   hipMemcpyHostToDevice));
  if (s->cav_on) {
    // the mode's total dipole is a sum over the states with these dipoles
    HIPCHK(cavity_set_dipole(s->cav, tls_ptrs(s), ml_dev(s), s->g.dt, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
  }
  return MLK_OK;
}

}  // extern "C"

// ====================================================================== batches
//
// A batch steps many independent sims together: every phase of the step is one
// launch over the jobs of all members (see find_job), so a step costs about a
// dozen launches whatever the number of domains.  The job tables hold device
// pointers; the fused sweep's two field buffers alternate, so each table exists
// for both buffer parities.  A captured hipGraph replays a fixed number of
// steps (even in the fused mode, so that every replay starts on the same
// parity).

namespace {

constexpr int kTileSlots = 6;  // fused tile shapes a batch launches, see tile_slot

template <typename J>
struct DevTable {
  J* jobs = nullptr;
  int* start = nullptr;
  int njobs = 0;
  int nblocks = 0;
  int2* order = nullptr;  // optional: (job, block) of each launch block
  int norder = 0;
};

template <typename J>
void free_table(DevTable<J>& t) {
  dfree(t.jobs);
  dfree(t.start);
  dfree(t.order);
  t = DevTable<J>{};
}

// One launch order for a table's blocks across its jobs, heaviest first by the
// given estimated work of each job's blocks (the jobs as uploaded): the kernel
// reads its (job, block) from it instead of searching the job starts, so that
// the heavy blocks of every job start first and the light ones fill in behind.
template <typename J>
mlk_status make_order(DevTable<J>& t, const std::vector<const std::vector<float>*>& work) {
  if ((int)work.size() != t.njobs) return fail(MLK_EINVAL, "block work does not match the jobs");
  std::vector<std::pair<float, int2>> all;
  for (int j = 0; j < t.njobs; ++j)
    for (int q = 0; q < (int)work[j]->size(); ++q) all.push_back({(*work[j])[q], make_int2(j, q)});
  std::stable_sort(all.begin(), all.end(),
                   [](const std::pair<float, int2>& x, const std::pair<float, int2>& y) {
                     return x.first > y.first;
                   });
  std::vector<int2> ord(all.size());
  for (size_t k = 0; k < all.size(); ++k) ord[k] = all[k].second;
  if (ord.empty()) return MLK_OK;
  STCHK(upload(&t.order, ord));
  t.norder = (int)ord.size();
  return MLK_OK;
}

// Upload the non-empty jobs; job starts are padded to multiples of 8 blocks.
template <typename J>
mlk_status make_table(DevTable<J>& t, const std::vector<J>& all) {
  free_table(t);
  std::vector<J> jobs;
  for (const J& j : all)
    if (j.nblocks > 0) jobs.push_back(j);
  if (jobs.empty()) return MLK_OK;
  std::vector<int> st(jobs.size() + 1);
  long long acc = 0;
  for (size_t q = 0; q < jobs.size(); ++q) {
    st[q] = (int)acc;
    acc += ((long long)jobs[q].nblocks + 7) / 8 * 8;
    if (acc > 0x7fffffffLL) return fail(MLK_EUNSUPPORTED, "batch grid too large");
  }
  st[jobs.size()] = (int)acc;
  STCHK(upload(&t.jobs, jobs));
  STCHK(upload(&t.start, st));
  t.njobs = (int)jobs.size();
  t.nblocks = (int)acc;
  return MLK_OK;
}

template <typename T>
struct BatchTables {
  DevTable<FluxJob<T>> fsave, fpart, finish;
  DevTable<GatherJob<T>> gather;
  DevTable<LightJob<T>> light;  // the light bins' emitters
  DevTable<FusedJob<T>> fused[kTileSlots];  // by tile shape, see tile_slot
  bool fused_lean[kTileSlots] = {};  // no job's box reaches a y or z layer
  DevTable<ShellJob<T>> shell;
  DevTable<SourceJob<T>> sources;
  DevTable<ScatterJob<T>> scatter;
  void release() {
    free_table(fsave);
    free_table(fpart);
    free_table(finish);
    free_table(gather);
    free_table(light);
    for (auto& f : fused) free_table(f);
    free_table(shell);
    free_table(sources);
    free_table(scatter);
  }
};

// Fused tile shapes (TX, TY): 64 x {4, 8, 16}, then 32 x {4, 8, 16}.
int tile_slot(int tx, int ty) { return (tx == 32 ? 3 : 0) + (ty == 16 ? 2 : (ty == 8 ? 1 : 0)); }
int slot_tx(int k) { return k < 3 ? 64 : 32; }
int slot_ty(int k) { return 4 << (k % 3); }

}  // namespace

struct mlk_batch {
  std::vector<mlk_sim*> sims;
  bool fp32 = false;
  bool fused = false;
  hipStream_t stream = nullptr;
  int parity = 0;  // number of buffer swaps since the tables were built, mod 2
  BatchTables<float> t32[2];
  BatchTables<double> t64[2];
  DevTable<TlsJob> tls;
  DevTable<MlJob> ml[kMaxLevels + 1];
  std::vector<const void*> series_snapshot;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t replay_steps = 0;
  int capture_parity = 0;  // buffer parity the captured steps start from
};

namespace {

std::vector<const void*> series_pointers(const mlk_batch* b) {
  std::vector<const void*> v;
  for (const mlk_sim* s : b->sims) {
    v.push_back(s->d_probe);
    v.push_back(s->d_flux_series);
    v.push_back(s->d_pop);
  }
  return v;
}

// Job tables for the current state of the members; parity q means q swaps of
// the fused buffers after now.
template <typename T>
mlk_status build_tables(mlk_batch* b, BatchTables<T> (&tab)[2]) {
  for (int q = 0; q < 2; ++q) {
    std::vector<FluxJob<T>> fs, fpj, fin;
    std::vector<GatherJob<T>> ga;
    std::vector<FusedJob<T>> fu[kTileSlots];
    std::vector<ShellJob<T>> sh;
    std::vector<SourceJob<T>> so;
    std::vector<ScatterJob<T>> sc;
    std::vector<const std::vector<float>*> gw, sw;  // block work of the non-empty jobs
    std::vector<LightJob<T>> li;
    for (mlk_sim* s : b->sims) {
      if (q == 1 && b->fused) swap_buffers(s);
      const FieldPtrs<T> cur = field_ptrs<T>(s);
      const FieldPtrs<T> nxt = b->fused ? spare_ptrs<T>(s) : cur;
      const Series ser = series_of(s);
      if (s->fp.on) {
        const int a = s->fp.axis;
        const int np = s->g.n[(a + 1) % 3] * s->g.n[(a + 2) % 3];
        fs.push_back({cur, s->g, s->fp, ser, s->d_step, (np + 255) / 256});
        fpj.push_back({nxt, s->g, s->fp, ser, s->d_step, s->fp.nblocks});
      }
      fin.push_back({nxt, s->g, s->fp, ser, s->d_step, 1});
      if (s->nem > 0) {
        ga.push_back({cur, s->g, bin_ptrs(s), window_ptrs<T>(s), s->d_Et, s->gdense});
        sc.push_back({nxt, s->g, bin_ptrs(s), window_ptrs<T>(s), s->d_mudot, s->nscatter});
        if (s->gdense > 0) gw.push_back(&s->gwork);
        if (s->nlight > 0) {
          const int per = light_per_block(s->fp32);
          li.push_back({cur, s->g, s->d_gbin_em + s->glight0, s->nlight, window_ptrs<T>(s),
                        s->d_Et, (s->nlight + per - 1) / per});
        }
        if (s->nscatter > 0) sw.push_back(&s->swork);
      }
      Box inner{};
      if (b->fused) {
        inner = sweep_box(s);
        FusedJob<T> J{};
        J.a = cur;
        if (s->vacuum) J.a.epsinv = nullptr;
        J.b = nxt;
        J.g = s->g;
        J.box = inner;
        J.kz = s->kz;
        J.tx = s->tx;
        J.ty = s->ty;
        fused_job_shape(J);
        fu[tile_slot(s->tx, s->ty)].push_back(J);
      }
      ShellJob<T> S{};
      S.in = cur;
      S.out = nxt;
      S.g = s->g;
      S.m = shell_map(s->g, inner);
      if (S.m.total >= 0x7fffff00LL) return fail(MLK_EUNSUPPORTED, "domain too large for a batch");
      S.nblocks = (int)((S.m.total + 255) / 256);
      sh.push_back(S);
      if (s->src.count > 0) {
        SourceJob<T> J{};
        J.f = nxt;
        J.g = s->g;
        J.src = s->src;
        J.step = s->d_step;
        J.bx = source_blocks_of(s->g, s->src);
        J.nblocks = J.bx * s->src.count;
        so.push_back(J);
      }
      if (q == 1 && b->fused) swap_buffers(s);
    }
    BatchTables<T>& t = tab[q];
    STCHK(make_table(t.fsave, fs));
    STCHK(make_table(t.fpart, fpj));
    STCHK(make_table(t.finish, fin));
    STCHK(make_table(t.gather, ga));
    STCHK(make_order(t.gather, gw));
    STCHK(make_table(t.light, li));
    for (int k = 0; k < kTileSlots; ++k) {
      // the smallest members first (by workgroups; measured a little faster than the
      // members' own order, and than the largest first)
      std::stable_sort(fu[k].begin(), fu[k].end(), [](const FusedJob<T>& x, const FusedJob<T>& y) {
        return x.nblocks < y.nblocks;
      });
      STCHK(make_table(t.fused[k], fu[k]));
      bool lean = true;
      for (const FusedJob<T>& J : fu[k]) lean = lean && fused_cpm(J.g, J.box) <= 1;
      t.fused_lean[k] = lean;
    }
    STCHK(make_table(t.shell, sh));
    STCHK(make_table(t.sources, so));
    STCHK(make_table(t.scatter, sc));
    STCHK(make_order(t.scatter, sw));
  }
  std::vector<TlsJob> tj;
  std::vector<MlJob> mj[kMaxLevels + 1];
  for (mlk_sim* s : b->sims) {
    const Series ser = series_of(s);
    const TlsPtrs tls = tls_ptrs(s);
    if (tls.count > 0)
      tj.push_back({tls, s->g.dt, s->d_Et, s->d_mudot, s->d_popoff, ser, s->d_step,
                    (tls.count + 255) / 256});
    const MlDev ml = ml_dev(s);
    for (int n = 2; n <= kMaxLevels; ++n) {
      const int first = s->ml_range[n], count = s->ml_range[n + 1] - s->ml_range[n];
      if (count > 0)
        mj[n].push_back({ml, first, count, s->g.dt, s->d_Et, s->d_mudot, s->d_popoff, ser,
                         s->d_step, (count + 63) / 64});
    }
  }
  STCHK(make_table(b->tls, tj));
  for (int n = 2; n <= kMaxLevels; ++n) STCHK(make_table(b->ml[n], mj[n]));
  b->parity = 0;
  b->series_snapshot = series_pointers(b);
  return MLK_OK;
}

mlk_status rebuild_tables(mlk_batch* b) {
  for (auto& t : b->t32) t.release();
  for (auto& t : b->t64) t.release();
  free_table(b->tls);
  for (auto& t : b->ml) free_table(t);
  return b->fp32 ? build_tables<float>(b, b->t32) : build_tables<double>(b, b->t64);
}

// Enqueue one batched step on tables of parity q.
template <typename T>
mlk_status enqueue_batch_step(mlk_batch* b, const BatchTables<T>& t) {
  constexpr bool f32 = sizeof(T) == 4;
  hipStream_t st = b->stream;
  auto detect = [&](const DevTable<FluxJob<T>>& d, int kind) -> hipError_t {
    if constexpr (f32) return detect_batch_f32(d.jobs, d.start, d.njobs, d.nblocks, kind, st);
    else return detect_batch_f64(d.jobs, d.start, d.njobs, d.nblocks, kind, st);
  };
  HIPCHK(detect(t.fsave, 0));
  if constexpr (f32) HIPCHK(gather_batch_f32(t.gather.jobs, t.gather.start, t.gather.njobs,
                                             t.gather.order, t.gather.norder, st));
  else HIPCHK(gather_batch_f64(t.gather.jobs, t.gather.start, t.gather.njobs, t.gather.order,
                               t.gather.norder, st));
  if constexpr (f32) HIPCHK(light_batch_f32(t.light.jobs, t.light.start, t.light.njobs,
                                            t.light.nblocks, st));
  else HIPCHK(light_batch_f64(t.light.jobs, t.light.start, t.light.njobs, t.light.nblocks, st));
  HIPCHK(tls_batch(b->tls.jobs, b->tls.start, b->tls.njobs, b->tls.nblocks, st));
  for (int n = 2; n <= kMaxLevels; ++n)
    HIPCHK(ml_batch(b->ml[n].jobs, b->ml[n].start, b->ml[n].njobs, b->ml[n].nblocks, n, st));
  for (int k = 0; k < kTileSlots; ++k) {
    const DevTable<FusedJob<T>>& f = t.fused[k];
    if constexpr (f32)
      HIPCHK(sweep_fused_batch_f32(f.jobs, f.start, f.njobs, f.nblocks, slot_tx(k), slot_ty(k),
                                   t.fused_lean[k], st));
    else
      HIPCHK(sweep_fused_batch_f64(f.jobs, f.start, f.njobs, f.nblocks, slot_tx(k), slot_ty(k),
                                   t.fused_lean[k], st));
  }
  for (int h = 1; h >= 0; --h) {
    if constexpr (f32) HIPCHK(shell_batch_f32(t.shell.jobs, t.shell.start, t.shell.njobs,
                                              t.shell.nblocks, h == 1, st));
    else HIPCHK(shell_batch_f64(t.shell.jobs, t.shell.start, t.shell.njobs, t.shell.nblocks,
                                h == 1, st));
  }
  if constexpr (f32) HIPCHK(sources_batch_f32(t.sources.jobs, t.sources.start, t.sources.njobs,
                                              t.sources.nblocks, st));
  else HIPCHK(sources_batch_f64(t.sources.jobs, t.sources.start, t.sources.njobs,
                                t.sources.nblocks, st));
  if constexpr (f32) HIPCHK(scatter_batch_f32(t.scatter.jobs, t.scatter.start, t.scatter.njobs,
                                              t.scatter.order, t.scatter.norder, st));
  else HIPCHK(scatter_batch_f64(t.scatter.jobs, t.scatter.start, t.scatter.njobs,
                                t.scatter.order, t.scatter.norder, st));
  HIPCHK(detect(t.fpart, 1));
  HIPCHK(detect(t.finish, 2));
  return MLK_OK;
}

// Make room in every member's series for n more steps; rebuild the tables (and
// drop a captured graph) when a series had to move.
mlk_status batch_reserve(mlk_batch* b, int64_t n) {
  for (mlk_sim* s : b->sims) STCHK(reserve_series(s, n));
  if (series_pointers(b) != b->series_snapshot) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->replay_steps = 0;
    STCHK(rebuild_tables(b));
  }
  return MLK_OK;
}

// Enqueue n steps starting from the batch's current parity (no host bookkeeping).
mlk_status enqueue_batch(mlk_batch* b, int64_t n, int parity0) {
  for (int64_t k = 0; k < n; ++k) {
    const int q = b->fused ? (int)((parity0 + k) & 1) : 0;
    if (b->fp32) STCHK(enqueue_batch_step<float>(b, b->t32[q]));
    else STCHK(enqueue_batch_step<double>(b, b->t64[q]));
  }
  return MLK_OK;
}

void batch_advance(mlk_batch* b, int64_t n) {
  for (mlk_sim* s : b->sims) {
    s->host_step += n;
    if (b->fused && (n & 1)) swap_buffers(s);
  }
  if (b->fused) b->parity = (int)((b->parity + n) & 1);
}

}  // namespace

extern "C" {

mlk_status mlk_batch_create(mlk_sim* const* sims, int32_t n, mlk_batch** out) {
  if (!sims || !out || n <= 0) return fail(MLK_EINVAL, "null argument or empty batch");
  *out = nullptr;
  auto* b = new mlk_batch();
  for (int q = 0; q < n; ++q) {
    mlk_sim* s = sims[q];
    if (!s) {
      delete b;
      return fail(MLK_EINVAL, "member %d is null", q);
    }
    for (mlk_sim* o : b->sims)
      if (o == s) {
        delete b;
        return fail(MLK_EINVAL, "member %d appears twice", q);
      }
    if (s->er.every > 0) {
      return fail(MLK_EUNSUPPORTED, "member %d records the field energy", q);
    }
    if (s->cav_on || s->npole > 0) {
      delete b;
      return fail(MLK_EUNSUPPORTED, "member %d steps a cavity or dispersive media", q);
    }
    const mlk_sim* s0 = sims[0];
    if (s->fp32 != s0->fp32 || s->desc.sweep != s0->desc.sweep || s->host_step != s0->host_step ||
        s->desc.device != s0->desc.device) {
      delete b;
      return fail(MLK_EINVAL, "members must share precision, sweep, device and step count");
    }
    if (s->nem > 0 && s->desc.scatter != MLK_SCATTER_OWNER) {
      delete b;
      return fail(MLK_EUNSUPPORTED, "batched members use the owner-computes scatter");
    }
    if (s->batch_stream) {
      delete b;
      return fail(MLK_ESTATE, "member %d already belongs to a batch", q);
    }
    b->sims.push_back(s);
  }
  b->fp32 = sims[0]->fp32;
  b->fused = sims[0]->desc.sweep == MLK_SWEEP_FUSED;
  b->stream = sims[0]->stream;
  for (mlk_sim* s : b->sims) {
    mlk_status st = sync_sim(s);
    if (st != MLK_OK) {
      delete b;
      return st;
    }
  }
  for (mlk_sim* s : b->sims) {
    if (s != sims[0]) s->batch_stream = b->stream;
    s->in_batch = true;
  }
  mlk_status st = rebuild_tables(b);
  if (st != MLK_OK) {
    for (mlk_sim* s : b->sims) {
      s->batch_stream = nullptr;
      s->in_batch = false;
    }
    for (auto& t : b->t32) t.release();
    for (auto& t : b->t64) t.release();
    delete b;
    return st;
  }
  *out = b;
  return MLK_OK;
}

mlk_status mlk_batch_step(mlk_batch* b, int64_t nsteps) {
  if (!b) return fail(MLK_EINVAL, "null argument");
  if (nsteps < 0) return fail(MLK_EINVAL, "negative step count");
  if (nsteps == 0) return MLK_OK;
  HIPCHK(hipSetDevice(b->sims[0]->desc.device));
  for (mlk_sim* s : b->sims)
    if (s->stream != b->stream) HIPCHK(hipStreamSynchronize(s->stream));
  STCHK(batch_reserve(b, nsteps));
  STCHK(enqueue_batch(b, nsteps, b->parity));
  batch_advance(b, nsteps);
  return MLK_OK;
}

mlk_status mlk_batch_capture(mlk_batch* b, int64_t steps_per_replay) {
  if (!b) return fail(MLK_EINVAL, "null argument");
  if (steps_per_replay <= 0) return fail(MLK_EINVAL, "steps per replay must be positive");
  if (b->fused && (steps_per_replay & 1))
    return fail(MLK_EINVAL, "the fused sweep alternates two buffers: capture an even step count");
  HIPCHK(hipSetDevice(b->sims[0]->desc.device));
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->replay_steps = 0;
  HIPCHK(hipStreamSynchronize(b->stream));
  HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  mlk_status st = enqueue_batch(b, steps_per_replay, b->parity);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->stream, &g);
  if (st != MLK_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(MLK_EDEVICE, "graph capture: %s", hipGetErrorString(e));
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(MLK_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
  }
  b->graph = g;
  b->exec = x;
  b->replay_steps = steps_per_replay;
  b->capture_parity = b->parity;
  return MLK_OK;
}

mlk_status mlk_batch_replay(mlk_batch* b, int64_t nreplays) {
  if (!b) return fail(MLK_EINVAL, "null argument");
  if (!b->exec && b->replay_steps <= 0) return fail(MLK_ESTATE, "nothing captured");
  if (nreplays < 0) return fail(MLK_EINVAL, "negative replay count");
  HIPCHK(hipSetDevice(b->sims[0]->desc.device));
  for (mlk_sim* s : b->sims)
    if (s->stream != b->stream) HIPCHK(hipStreamSynchronize(s->stream));
  const int64_t spr = b->replay_steps;
  STCHK(batch_reserve(b, nreplays * spr));
  if (!b->exec || b->capture_parity != b->parity) {
    // a series had to grow (the captured pointers are stale), the tables were
    // rebuilt (tuning), or odd eager steps since the capture left the fused
    // buffers the other way round: capture again
    STCHK(mlk_batch_capture(b, spr));
  }
  for (int64_t r = 0; r < nreplays; ++r) {
    HIPCHK(hipGraphLaunch(b->exec, b->stream));
    batch_advance(b, spr);
  }
  return MLK_OK;
}

mlk_status mlk_batch_sync(mlk_batch* b) {
  if (!b) return fail(MLK_EINVAL, "null argument");
  HIPCHK(hipStreamSynchronize(b->stream));
  for (mlk_sim* s : b->sims) {
    const mlk_status st = check_numeric(s);
    if (st != MLK_OK) return st;
  }
  return MLK_OK;
}

mlk_status mlk_batch_destroy(mlk_batch* b) {
  if (!b) return MLK_OK;
  (void)hipStreamSynchronize(b->stream);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (auto& t : b->t32) t.release();
  for (auto& t : b->t64) t.release();
  free_table(b->tls);
  for (auto& t : b->ml) free_table(t);
  for (mlk_sim* s : b->sims) {
    s->batch_stream = nullptr;
    s->in_batch = false;
  }
  delete b;
  return MLK_OK;
}

}  // extern "C"

// ==================================================================== autotuner
//
// The fused sweep has two tile parameters: the rows per workgroup (TY = 4, 8 or
// 16; 64 x TY threads) and the z planes each workgroup marches (kz).  They trade
// LDS halo re-reads (larger TY) and prologue cost (larger kz) against the
// number of workgroups in flight.  mlk_autotune times every pair on the sim's
// own grid as it runs inside a step: the fused launch followed by the two CPML
// shell passes (all read the current fields and write the spare buffers, which
// the next step overwrites, so the state is untouched).  Back-to-back launches
// of the fused kernel alone rank the pairs differently from the step.  The
// pairs are timed in three interleaved rounds and each keeps its best round,
// so a slow spell of the device does not decide the choice.  Results are cached
// in a small JSON file keyed by precision, grid and interior box, one entry per
// line.

namespace {

std::string tune_key(const mlk_sim* s) {
  const Geom& g = s->g;
  char k[200];
  std::snprintf(k, sizeof k, "%s %d %d %d cpml %d %d %d %d %d %d periodic %d %d %d",
                s->fp32 ? "fp32" : "fp64", g.n[0], g.n[1], g.n[2], g.nlo[0], g.nhi[0], g.nlo[1],
                g.nhi[1], g.nlo[2], g.nhi[2], g.periodic[0], g.periodic[1], g.periodic[2]);
  return k;
}

struct TuneEntry {
  std::string key;
  int ty, kz, layers;
  double us;
  int tx;
};

bool valid_entry(const TuneEntry& e) {
  return (e.tx == 64 || e.tx == 32) && (e.ty == 4 || e.ty == 8 || e.ty == 16) && e.kz > 0;
}

std::vector<TuneEntry> read_cache(const char* path) {
  std::vector<TuneEntry> v;
  FILE* f = path ? std::fopen(path, "r") : nullptr;
  if (!f) return v;
  char line[512];
  while (std::fgets(line, sizeof line, f)) {
    char key[200];
    TuneEntry e{};
    e.tx = 64;  // entries written before the tile width was tuned
    if (std::sscanf(line,
                    " \"%199[^\"]\": {\"ty\": %d, \"kz\": %d, \"layers\": %d, \"us\": %lf, \"tx\": %d",
                    key, &e.ty, &e.kz, &e.layers, &e.us, &e.tx) >= 5) {
      e.key = key;
      v.push_back(e);
    }
  }
  std::fclose(f);
  return v;
}

bool write_cache(const char* path, const std::vector<TuneEntry>& v) {
  FILE* f = std::fopen(path, "w");
  if (!f) return false;
  std::fprintf(f, "{\n");
  for (size_t q = 0; q < v.size(); ++q)
    std::fprintf(f, "\"%s\": {\"ty\": %d, \"kz\": %d, \"layers\": %d, \"us\": %.3f, \"tx\": %d}%s\n",
                 v[q].key.c_str(), v[q].ty, v[q].kz, v[q].layers, v[q].us, v[q].tx,
                 q + 1 < v.size() ? "," : "");
  std::fprintf(f, "}\n");
  return std::fclose(f) == 0;
}

template <typename T>
mlk_status time_fused(mlk_sim* s, int tx, int ty, int kz, double* us) {
  const FieldPtrs<T> a = field_ptrs<T>(s), b = spare_ptrs<T>(s), ar = sweep_reads<T>(s);
  const Box inner = sweep_box(s);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  hipError_t err = hipSuccess;
  constexpr int kReps = 4;
  for (int r = -1; r < kReps && err == hipSuccess; ++r) {
    if (r == 0) err = hipEventRecord(e0, s->stream);
    if (err == hipSuccess) err = sweep_passes<T>(s, a, ar, b, inner, kz, tx, ty);
  }
  if (err == hipSuccess) err = hipEventRecord(e1, s->stream);
  if (err == hipSuccess) err = hipEventSynchronize(e1);
  float ms = 0.f;
  if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIPCHK(err);
  *us = 1e3 * ms / kReps;
  return MLK_OK;
}

}  // namespace

extern "C" {

mlk_status mlk_set_tuning(mlk_sim* s, int32_t ty, int32_t kz) {
  if (!s) return fail(MLK_EINVAL, "null argument");
  if (ty != 4 && ty != 8 && ty != 16)
    return fail(MLK_EINVAL, "rows per workgroup must be 4, 8 or 16");
  if (kz < 1) return fail(MLK_EINVAL, "planes per workgroup must be positive");
  if (s->in_batch) return fail(MLK_ESTATE, "tune members before forming the batch");
  s->ty = ty;
  s->kz = kz;
  return MLK_OK;
}

mlk_status mlk_get_tuning(mlk_sim* s, int32_t* ty, int32_t* kz) {
  if (!s || !ty || !kz) return fail(MLK_EINVAL, "null argument");
  *ty = s->ty;
  *kz = s->kz;
  return MLK_OK;
}

mlk_status mlk_set_tile_width(mlk_sim* s, int32_t tx) {
  if (!s) return fail(MLK_EINVAL, "null argument");
  if (tx != 64 && tx != 32) return fail(MLK_EINVAL, "tile width %d: 64 or 32", tx);
  if (s->in_batch) return fail(MLK_ESTATE, "tune members before forming the batch");
  STCHK(sync_sim(s));
  const int old = s->tx;
  s->tx = tx;
  // the frame launch needs a fused box over every x column, which depends on the width
  if (s->layer_mode == 2 && !split_ok(s)) {
    s->tx = old;
    return fail(MLK_EUNSUPPORTED, "the frame launch needs a fused box spanning every x "
                                  "column, which %d-wide tiles do not give here", tx);
  }
  return MLK_OK;
}

mlk_status mlk_get_tile_width(mlk_sim* s, int32_t* tx) {
  if (!s || !tx) return fail(MLK_EINVAL, "null argument");
  *tx = s->tx;
  return MLK_OK;
}

mlk_status mlk_set_sweep_layers(mlk_sim* s, int32_t on) {
  if (!s) return fail(MLK_EINVAL, "null argument");
  if (s->in_batch) return fail(MLK_ESTATE, "tune members before forming the batch");
  if (on < 0 || on > 2) return fail(MLK_EINVAL, "layer mode %d: 0, 1 or 2", on);
  if (on && !s->fp32)
    return fail(MLK_EUNSUPPORTED, "the FP64 fused sweep leaves the y and z layers to the shell");
  if (on == 2 && !split_ok(s))
    return fail(MLK_EUNSUPPORTED, "the frame launch needs y or z layers and a fused box "
                                  "spanning every x column");
  STCHK(sync_sim(s));
  s->layer_mode = on;
  return MLK_OK;
}

mlk_status mlk_get_sweep_layers(mlk_sim* s, int32_t* on) {
  if (!s || !on) return fail(MLK_EINVAL, "null argument");
  *on = s->layer_mode;
  return MLK_OK;
}

mlk_status mlk_autotune(mlk_sim* s, const char* cache_path) {
  if (!s) return fail(MLK_EINVAL, "null argument");
  if (s->in_batch) return fail(MLK_ESTATE, "tune members before forming the batch");
  if (s->desc.sweep != MLK_SWEEP_FUSED) return MLK_OK;  // nothing to tune
  const std::string key = tune_key(s);
  std::vector<TuneEntry> cache = read_cache(cache_path);
  for (const TuneEntry& e : cache)
    if (e.key == key && valid_entry(e)) {
      s->tx = e.tx;
      s->ty = e.ty;
      s->kz = e.kz;
      s->layer_mode = !s->fp32 ? 0 : (e.layers == 2 && !split_ok(s) ? 1 : e.layers);
      return MLK_OK;
    }
  HIPCHK(hipSetDevice(s->desc.device));
  STCHK(sync_sim(s));
  // candidates: layer mode (FP32: with or without the y and z layers in the
  // fused kernel, or in the frame launch) x tile width x rows per workgroup x
  // planes per workgroup
  struct Cand {
    int layers, tx, ty, kz;
    double us;
  };
  std::vector<Cand> cands;
  for (int lay = 0; lay <= (s->fp32 ? 2 : 0); ++lay)
    for (int tx : {64, 32}) {
      s->layer_mode = lay;
      s->tx = tx;
      if (lay == 2 && !split_ok(s)) continue;
      const Box inner = sweep_box(s);
      const int ez = inner.hi[2] - inner.lo[2];
      if (ez <= 0) continue;
      for (int ty : {4, 8, 16})
        for (int kz : {4, 8, 16, 32, 64, 128})
          if (kz <= std::max(4, ez)) cands.push_back({lay, tx, ty, kz, 1e300});
    }
  for (int round = 0; round < 3; ++round)
    for (Cand& c : cands) {
      double us = 0.0;
      s->layer_mode = c.layers;
      s->tx = c.tx;
      STCHK(s->fp32 ? time_fused<float>(s, c.tx, c.ty, c.kz, &us)
                    : time_fused<double>(s, c.tx, c.ty, c.kz, &us));
      c.us = std::min(c.us, us);
    }
  double best = 1e300;
  int blay = 0, btx = 64, bty = s->ty, bkz = s->kz;
  for (const Cand& c : cands)
    if (c.us < best) {
      best = c.us;
      blay = c.layers;
      btx = c.tx;
      bty = c.ty;
      bkz = c.kz;
    }
  s->layer_mode = blay;
  s->tx = btx;
  s->ty = bty;
  s->kz = bkz;
  if (cache_path) {
    cache.push_back({key, bty, bkz, blay, best, btx});
    if (!write_cache(cache_path, cache))
      return fail(MLK_EINVAL, "cannot write the tuning cache %s", cache_path);
  }
  return MLK_OK;
}

}  // extern "C"

namespace {

// Device time of the sweep phase of one batched step (every fused launch plus
// the two shell passes) on the tables of the current parity, best of kReps; the
// members' state is untouched (both write the spare buffers).
template <typename T>
mlk_status time_batch_sweep(mlk_batch* b, const BatchTables<T>& t, double* us) {
  constexpr bool f32 = sizeof(T) == 4;
  hipStream_t st = b->stream;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  hipError_t err = hipSuccess;
  auto once = [&]() {
    for (int k = 0; k < kTileSlots && err == hipSuccess; ++k) {
      const DevTable<FusedJob<T>>& f = t.fused[k];
      if constexpr (f32)
        err = sweep_fused_batch_f32(f.jobs, f.start, f.njobs, f.nblocks, slot_tx(k), slot_ty(k),
                                    t.fused_lean[k], st);
      else
        err = sweep_fused_batch_f64(f.jobs, f.start, f.njobs, f.nblocks, slot_tx(k), slot_ty(k),
                                    t.fused_lean[k], st);
    }
    for (int h = 1; h >= 0 && err == hipSuccess; --h) {
      if constexpr (f32)
        err = shell_batch_f32(t.shell.jobs, t.shell.start, t.shell.njobs, t.shell.nblocks, h == 1, st);
      else
        err = shell_batch_f64(t.shell.jobs, t.shell.start, t.shell.njobs, t.shell.nblocks, h == 1, st);
    }
  };
  constexpr int kReps = 3;
  once();  // warm-up
  double best = 1e300;
  for (int r = 0; r < kReps && err == hipSuccess; ++r) {
    err = hipEventRecord(e0, st);
    once();
    if (err == hipSuccess) err = hipEventRecord(e1, st);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    best = std::min(best, 1e3 * (double)ms);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIPCHK(err);
  *us = best;
  return MLK_OK;
}

// Cache key of a batch: precision, member count and an FNV-1a hash of the
// members' grid keys in order.
std::string batch_key(const mlk_batch* b) {
  uint64_t h = 1469598103934665603ull;
  for (const mlk_sim* s : b->sims)
    for (char c : tune_key(s) + ";") {
      h ^= (unsigned char)c;
      h *= 1099511628211ull;
    }
  char k[96];
  std::snprintf(k, sizeof k, "batch %s %zu %016llx", b->fp32 ? "fp32" : "fp64", b->sims.size(),
                (unsigned long long)h);
  return k;
}

void set_members(mlk_batch* b, int layers, int tx, int ty, int kz) {
  for (mlk_sim* s : b->sims) {
    s->layer_mode = b->fp32 && layers != 0 ? 1 : 0;
    s->tx = tx;
    s->ty = ty;
    s->kz = kz;
  }
}

}  // namespace

extern "C" {

mlk_status mlk_batch_autotune(mlk_batch* b, const char* cache_path) {
  if (!b) return fail(MLK_EINVAL, "null argument");
  if (!b->fused) return MLK_OK;  // nothing to tune
  HIPCHK(hipSetDevice(b->sims[0]->desc.device));
  // the captured graph refers to the tables about to be rebuilt; the next replay
  // captures the same step count again
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  HIPCHK(hipStreamSynchronize(b->stream));
  const std::string key = batch_key(b);
  std::vector<TuneEntry> cache = read_cache(cache_path);
  for (const TuneEntry& e : cache)
    if (e.key == key && valid_entry(e)) {
      set_members(b, e.layers, e.tx, e.ty, e.kz);
      return rebuild_tables(b);
    }
  struct Cand {
    int layers, tx, ty, kz;
    double us;
  };
  std::vector<Cand> cands;
  for (int lay = 0; lay <= (b->fp32 ? 1 : 0); ++lay)
    for (int tx : {64, 32})
      for (int ty : {4, 8, 16})
        for (int kz : {4, 8, 16, 32}) cands.push_back({lay, tx, ty, kz, 1e300});
  for (int round = 0; round < 3; ++round)
    for (Cand& c : cands) {
      set_members(b, c.layers, c.tx, c.ty, c.kz);
      STCHK(rebuild_tables(b));
      double us = 0.0;
      STCHK(b->fp32 ? time_batch_sweep<float>(b, b->t32[0], &us)
                    : time_batch_sweep<double>(b, b->t64[0], &us));
      c.us = std::min(c.us, us);
    }
  const Cand* best = &cands[0];
  for (const Cand& c : cands)
    if (c.us < best->us) best = &c;
  set_members(b, best->layers, best->tx, best->ty, best->kz);
  STCHK(rebuild_tables(b));
  if (cache_path) {
    cache.push_back({key, best->ty, best->kz, best->layers, best->us, best->tx});
    if (!write_cache(cache_path, cache))
      return fail(MLK_EINVAL, "cannot write the tuning cache %s", cache_path);
  }
  return MLK_OK;
}

}  // extern "C"
