// Host-side launchers of the libmlk kernels (one per kernel family and precision).
#pragma once

#include "mlk_internal.h"

namespace mlk {

hipError_t cpml_tables(bool fp32, const Geom& g, int a, double m, double sigma_max, double kmax,
                       double amax, void* b, void* c, void* kinv, hipStream_t st);
hipError_t inverse_to(bool fp32, const double* src, void* dst, size_t n, hipStream_t st);
hipError_t convert_in(bool fp32, const double* src, void* dst, size_t n, hipStream_t st);
hipError_t convert_out(bool fp32, const void* src, double* dst, size_t n, hipStream_t st);

hipError_t sweep_plain_f64(const FieldPtrs<double>& in, const FieldPtrs<double>& out,
                           const Geom& g, const Box* boxes, int nbox, bool h_pass, bool e_pass,
                           hipStream_t st);
hipError_t sweep_plain_f32(const FieldPtrs<float>& in, const FieldPtrs<float>& out, const Geom& g,
                           const Box* boxes, int nbox, bool h_pass, bool e_pass, hipStream_t st);
hipError_t sweep_shell_f64(const FieldPtrs<double>& in, const FieldPtrs<double>& out,
                           const Geom& g, const Box& inner, bool h_pass, hipStream_t st);
hipError_t sweep_shell_f32(const FieldPtrs<float>& in, const FieldPtrs<float>& out, const Geom& g,
                           const Box& inner, bool h_pass, hipStream_t st);
// Two-level step of every two-level emitter under E~ (M x 3, emitter-id order).
// E~ of every emitter (id order) under the travelling pulse at time t.
hipError_t wave_field(int M, const double* pos, const double* gamma, const WaveDesc& w, double t,
                      double* Et, hipStream_t st);
hipError_t tls_step(const TlsPtrs& tls, double dt, const double* Et, double* mudot,
                    const int64_t* pop_off, const Series& ser, const int64_t* step,
                    hipStream_t st);
// Multilevel step of every slot; range[n]..range[n+1] are the slots with n levels.
hipError_t ml_step(const MlDev& ml, const int* range, double dt, const double* Et, double* mudot,
                   const int64_t* pop_off, const Series& ser, const int64_t* step,
                   hipStream_t st);
hipError_t sources_f64(const FieldPtrs<double>& f, const Geom& g, const SourceSet& src,
                       const int64_t* step, hipStream_t st);
hipError_t sources_f32(const FieldPtrs<float>& f, const Geom& g, const SourceSet& src,
                       const int64_t* step, hipStream_t st);
// The frame of y and z CPML layers around an interior box (which the fused sweep
// covers with its lean kernel), by the full fused kernel in one launch.
hipError_t sweep_frame_f64(const FieldPtrs<double>& a, const FieldPtrs<double>& b, const Geom& g,
                           const Box& inner, int kz, hipStream_t st);
hipError_t sweep_frame_f32(const FieldPtrs<float>& a, const FieldPtrs<float>& b, const Geom& g,
                           const Box& inner, int kz, hipStream_t st);
hipError_t sweep_fused_f64(const FieldPtrs<double>& a, const FieldPtrs<double>& b, const Geom& g,
                           const Box& box, int kz, int tx, int ty, hipStream_t st);
hipError_t sweep_fused_f32(const FieldPtrs<float>& a, const FieldPtrs<float>& b, const Geom& g,
                           const Box& box, int kz, int tx, int ty, hipStream_t st);

hipError_t windows_f64(int count, const double* pos, const double* sigma, double R, const Geom& g,
                       int* lo, int* len, double* w, hipStream_t st);
hipError_t windows_f32(int count, const double* pos, const double* sigma, double R, const Geom& g,
                       int* lo, int* len, float* w, hipStream_t st);
hipError_t records_f64(int count, const int* lo, const int* len, const double* w,
                       WinRec<double>* rec, hipStream_t st);
hipError_t records_f32(int count, const int* lo, const int* len, const float* w,
                       WinRec<float>* rec, hipStream_t st);
hipError_t scatter_atomic_f64(const FieldPtrs<double>& f, const Geom& g,
                              const WindowPtrs<double>& win, int count, const double* mudot,
                              hipStream_t st);
hipError_t scatter_atomic_f32(const FieldPtrs<float>& f, const Geom& g,
                              const WindowPtrs<float>& win, int count, const double* mudot,
                              hipStream_t st);

hipError_t flux_save_f64(const FieldPtrs<double>& f, const Geom& g, const FluxPlane& fp,
                         hipStream_t st);
hipError_t flux_save_f32(const FieldPtrs<float>& f, const Geom& g, const FluxPlane& fp,
                         hipStream_t st);
// W^n from the spare (E^n, H^{n-1/2}) and current (H^{n+1/2}) buffers of the fused
// sweep, into er.series on steps with n % er.every == 0.
hipError_t energy_f64(const FieldPtrs<double>& old, const FieldPtrs<double>& cur, size_t ncell,
                      const EnergyRec& er, const int64_t* step, hipStream_t st);
hipError_t energy_f32(const FieldPtrs<float>& old, const FieldPtrs<float>& cur, size_t ncell,
                      const EnergyRec& er, const int64_t* step, hipStream_t st);
// partials_done: the flux partials of this step are formed already (by the scatter
// launch), so only the finishing block runs
hipError_t finish_f64(const FieldPtrs<double>& f, const Geom& g, const FluxPlane& fp,
                      const Series& ser, int64_t* step, bool partials_done, hipStream_t st);
hipError_t finish_f32(const FieldPtrs<float>& f, const Geom& g, const FluxPlane& fp,
                      const Series& ser, int64_t* step, bool partials_done, hipStream_t st);

// fp: when given, the same launch saves the flux plane's E^n (needs ngather > 0)
hipError_t bin_gather_step_f64(const FieldPtrs<double>& f, const Geom& g, const BinPtrs& b,
                               const WindowPtrs<double>& win, const TlsPtrs& tls, double* Et,
                               double* mudot, const int64_t* pop_off, const Series& ser,
                               const int64_t* step, const FluxPlane* fp, hipStream_t st);
hipError_t bin_gather_step_f32(const FieldPtrs<float>& f, const Geom& g, const BinPtrs& b,
                               const WindowPtrs<float>& win, const TlsPtrs& tls, double* Et,
                               double* mudot, const int64_t* pop_off, const Series& ser,
                               const int64_t* step, const FluxPlane* fp, hipStream_t st);
// fp: when given, fp->nblocks more workgroups of the same launch form the flux
// partials of the plane (no window may reach the plane's E cells)
hipError_t bin_scatter_f64(const FieldPtrs<double>& f, const Geom& g, const BinPtrs& b,
                           const WindowPtrs<double>& win, const double* mudot,
                           const FluxPlane* fp, hipStream_t st);
hipError_t bin_scatter_f32(const FieldPtrs<float>& f, const Geom& g, const BinPtrs& b,
                           const WindowPtrs<float>& win, const double* mudot,
                           const FluxPlane* fp, hipStream_t st);
// bin edge lengths (cells) of the gather (G) and scatter (S) bins for a field precision
void bin_shape(bool fp32, int G[3], int S[3]);
// Gather bins of at most this many emitters are light (stage only their windows).
int gather_light_max();

// ---- batched launches (one launch per phase over the jobs of many domains)
template <typename T>
void fused_job_shape(FusedJob<T>& J);
ShellMap shell_map(const Geom& g, const Box& inner);
int source_blocks_of(const Geom& g, const SourceSet& src);
hipError_t sweep_fused_batch_f64(const FusedJob<double>* jobs, const int* start, int njobs,
                                 int nblocks, int tx, int ty, bool lean, hipStream_t st);
hipError_t sweep_fused_batch_f32(const FusedJob<float>* jobs, const int* start, int njobs,
                                 int nblocks, int tx, int ty, bool lean, hipStream_t st);
// CPML code a fused launch over the box needs: 0 none, 1 x layers only (the box keeps
// clear of the y and z layers), 2 every layer.
int fused_cpm(const Geom& g, const Box& box);
hipError_t shell_batch_f64(const ShellJob<double>* jobs, const int* start, int njobs, int nblocks,
                           bool h_pass, hipStream_t st);
hipError_t shell_batch_f32(const ShellJob<float>* jobs, const int* start, int njobs, int nblocks,
                           bool h_pass, hipStream_t st);
hipError_t sources_batch_f64(const SourceJob<double>* jobs, const int* start, int njobs,
                             int nblocks, hipStream_t st);
hipError_t sources_batch_f32(const SourceJob<float>* jobs, const int* start, int njobs,
                             int nblocks, hipStream_t st);
hipError_t gather_batch_f64(const GatherJob<double>* jobs, const int* start, int njobs,
                            const int2* order, int nblocks, hipStream_t st);
hipError_t gather_batch_f32(const GatherJob<float>* jobs, const int* start, int njobs,
                            const int2* order, int nblocks, hipStream_t st);
hipError_t tls_batch(const TlsJob* jobs, const int* start, int njobs, int nblocks,
                     hipStream_t st);
hipError_t ml_batch(const MlJob* jobs, const int* start, int njobs, int nblocks, int nl,
                    hipStream_t st);
// The light bins' emitters of a batch (no tile); light_per_block: emitters per block.
hipError_t light_batch_f64(const LightJob<double>* jobs, const int* start, int njobs,
                           int nblocks, hipStream_t st);
hipError_t light_batch_f32(const LightJob<float>* jobs, const int* start, int njobs, int nblocks,
                           hipStream_t st);
int light_per_block(bool fp32);
hipError_t scatter_batch_f64(const ScatterJob<double>* jobs, const int* start, int njobs,
                             const int2* order, int nblocks, hipStream_t st);
hipError_t scatter_batch_f32(const ScatterJob<float>* jobs, const int* start, int njobs,
                             const int2* order, int nblocks, hipStream_t st);
hipError_t detect_batch_f64(const FluxJob<double>* jobs, const int* start, int njobs, int nblocks,
                            int kind, hipStream_t st);
hipError_t detect_batch_f32(const FluxJob<float>* jobs, const int* start, int njobs, int nblocks,
                            int kind, hipStream_t st);

// ---- adjoint
hipError_t gather_epsw_f64(const FieldPtrs<double>& f, const Geom& g, const BinPtrs& b,
                           const WindowPtrs<double>& win, double* out, hipStream_t st);
hipError_t gather_epsw_f32(const FieldPtrs<float>& f, const Geom& g, const BinPtrs& b,
                           const WindowPtrs<float>& win, double* out, hipStream_t st);
hipError_t scatter_plain_f64(const FieldPtrs<double>& f, const Geom& g, const BinPtrs& b,
                             const WindowPtrs<double>& win, const double* amp, double amp0,
                             hipStream_t st);
hipError_t scatter_plain_f32(const FieldPtrs<float>& f, const Geom& g, const BinPtrs& b,
                             const WindowPtrs<float>& win, const double* amp, double amp0,
                             hipStream_t st);
Box adj_interior_box(const Geom& g, bool zl);
hipError_t adj_fused_f64(const AdjSweep<double>& a, const Geom& g, const Box& box,
                         hipStream_t st);
hipError_t adj_fused_f32(const AdjSweep<float>& a, const Geom& g, const Box& box,
                         hipStream_t st);
hipError_t adj_sweep_f64(const AdjSweep<double>& a, const Geom& g, hipStream_t st);
hipError_t adj_sweep_f32(const AdjSweep<float>& a, const Geom& g, hipStream_t st);
hipError_t adj_flux_f64(const AdjSweep<double>& a, const Geom& g, int axis, int index,
                        const double* tape, int part, hipStream_t st);
hipError_t adj_flux_f32(const AdjSweep<float>& a, const Geom& g, int axis, int index,
                        const double* tape, int part, hipStream_t st);
hipError_t adj_eps_f64(const AdjSweep<double>& a, const Geom& g, const Box& box, const double* e_n,
                       const double* e_n1, double* geps, hipStream_t st);
hipError_t adj_eps_f32(const AdjSweep<float>& a, const Geom& g, const Box& box, const float* e_n,
                       const float* e_n1, double* geps, hipStream_t st);
hipError_t adj_tls(const TlsPtrs& tls, double dt, double mub_scale, const double* tape_s,
                   const double* tape_et, const double* mub, double* sb, double* gd, double* etb,
                   hipStream_t st);
hipError_t pack_tape_f64(const FieldPtrs<double>& f, const Geom& g, const Box& box,
                         double* box_out, const FluxPlane* fp, double* flux_out, hipStream_t st);
hipError_t pack_tape_f32(const FieldPtrs<float>& f, const Geom& g, const Box& box, float* box_out,
                         const FluxPlane* fp, double* flux_out, hipStream_t st);
// Dispersive poles: before the sweep, Q <- P^{n+1} - P^n from P, Q and E^n; after
// the sweep, the scatter and the sources, E -= (1/eps_inf) Q and P += Q.
hipError_t pole_pre_f64(const PoleDev& p, const FieldPtrs<double>& f, const Geom& g, hipStream_t st);
hipError_t pole_pre_f32(const PoleDev& p, const FieldPtrs<float>& f, const Geom& g, hipStream_t st);
hipError_t pole_post_f64(const PoleDev& p, const FieldPtrs<double>& f, const Geom& g,
                         const double* epsinv, hipStream_t st);
hipError_t pole_post_f32(const PoleDev& p, const FieldPtrs<float>& f, const Geom& g,
                         const float* epsinv, hipStream_t st);
// Single-mode cavity: E~ of every emitter from the mode state, then the
// sum of mu_dot over the emitters, the (p, q, d) update and the step counter.
int cavity_blocks(int M);
hipError_t cavity_field(const CavityDev& c, double* Et, int M, hipStream_t st);
// Partial sums of <mu> + (dt/2) mu_dot over the states, then the (p, q) leapfrog
// with the old d, the new d and the step counter.
hipError_t cavity_update(const CavityDev& c, const TlsPtrs& tls, const MlDev& ml, double dt,
                         int64_t* step, hipStream_t st);
// The same sums, stored as d without advancing the mode (set-up, new dipoles).
hipError_t cavity_set_dipole(const CavityDev& c, const TlsPtrs& tls, const MlDev& ml, double dt,
                             hipStream_t st);
// The (p, q, d) update from npartial per-block partial sums already in c.partial.
hipError_t cavity_advance(const CavityDev& c, int npartial, double dt, int64_t* step,
                          hipStream_t st);
// Two-level emitters only: E~ from the mode, the two-level step, and the partial sums
// of <mu> + (dt/2) mu_dot (x, y) of each block of kTlsThreads slots of the new states
// into c.partial.
hipError_t cavity_tls_step(const TlsPtrs& tls, double dt, const CavityDev& c, double* Et,
                           double* mudot, const int64_t* pop_off, const Series& ser,
                           const int64_t* step, hipStream_t st);
hipError_t eps_box_f64(const double* eps, const Geom& g, const Box& box, double* epsinv,
                       hipStream_t st);
hipError_t eps_box_f32(const double* eps, const Geom& g, const Box& box, float* epsinv,
                       hipStream_t st);

}  // namespace mlk
