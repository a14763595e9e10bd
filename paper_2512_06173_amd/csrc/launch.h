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
// Multilevel step of every slot; range[n]..range[n+1] are the slots with n levels.
hipError_t ml_step(const MlDev& ml, const int* range, double dt, const double* Et, double* mudot,
                   const int64_t* pop_off, const Series& ser, const int64_t* step,
                   hipStream_t st);
hipError_t sources_f64(const FieldPtrs<double>& f, const Geom& g, const SourceSet& src,
                       const int64_t* step, hipStream_t st);
hipError_t sources_f32(const FieldPtrs<float>& f, const Geom& g, const SourceSet& src,
                       const int64_t* step, hipStream_t st);
hipError_t sweep_fused_f64(const FieldPtrs<double>& a, const FieldPtrs<double>& b, const Geom& g,
                           const Box& box, int kz, hipStream_t st);
hipError_t sweep_fused_f32(const FieldPtrs<float>& a, const FieldPtrs<float>& b, const Geom& g,
                           const Box& box, int kz, hipStream_t st);

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
hipError_t finish_f64(const FieldPtrs<double>& f, const Geom& g, const FluxPlane& fp,
                      const Series& ser, int64_t* step, hipStream_t st);
hipError_t finish_f32(const FieldPtrs<float>& f, const Geom& g, const FluxPlane& fp,
                      const Series& ser, int64_t* step, hipStream_t st);

hipError_t bin_gather_step_f64(const FieldPtrs<double>& f, const Geom& g, const BinPtrs& b,
                               const WindowPtrs<double>& win, const TlsPtrs& tls, double* Et,
                               double* mudot, const int64_t* pop_off, const Series& ser,
                               const int64_t* step, hipStream_t st);
hipError_t bin_gather_step_f32(const FieldPtrs<float>& f, const Geom& g, const BinPtrs& b,
                               const WindowPtrs<float>& win, const TlsPtrs& tls, double* Et,
                               double* mudot, const int64_t* pop_off, const Series& ser,
                               const int64_t* step, hipStream_t st);
hipError_t bin_scatter_f64(const FieldPtrs<double>& f, const Geom& g, const BinPtrs& b,
                           const WindowPtrs<double>& win, const double* mudot, hipStream_t st);
hipError_t bin_scatter_f32(const FieldPtrs<float>& f, const Geom& g, const BinPtrs& b,
                           const WindowPtrs<float>& win, const double* mudot, hipStream_t st);
// bin edge lengths (cells) of the gather (G) and scatter (S) bins for a field precision
void bin_shape(bool fp32, int G[3], int S[3]);

}  // namespace mlk
