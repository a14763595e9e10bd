/*
 * mlk.h -- C ABI of libmlk, an MI355X (gfx950) engine for self-consistent
 * light-matter propagation: a 3-D Yee FDTD leapfrog of E/H coupled, at
 * every step, to an ensemble of quantum emitters through a Gaussian-smeared
 * regularised field and a smeared dipole current.
 *
 * What each step computes (natural units: c = eps0 = mu0 = hbar = 1; dx is
 * the cell size, dt = courant * dx):
 *   1. H^{n+1/2} = H^{n-1/2} - dt curl E^n               (eq. Maxwell, Sec. II.A.1)
 *   2. E~_m^c   = gamma_m sum_p w^c_{m,p} E_c^n(p)        (eq. E_regu_Emi)
 *   3. rho_m^{n+1/2} = exact step of d rho/dt = -i[H0 - E~.mu, rho] + D[rho]
 *                                                         (eq. von-Neumann-tls)
 *   4. mu_dot_m = Tr(rho_dot mu)                          (eq. dipole_derivative)
 *   5. J_c(p)   = sum_m gamma_m mu_dot_m^c w^c_{m,p}/dx^3 + source currents
 *                                                         (eqs. J_mol, Polarization_mol)
 *   6. E^{n+1}  = E^n + (dt/eps_r)(curl H^{n+1/2} - J)     (eq. Maxwell, eq. Dromega)
 *   7. detectors (probes, populations, Poynting flux).
 * The order field -> emitter -> dipole rate -> current is the per-step
 * exchange of Sec. III; here it never leaves the GPU.
 *
 * Grid layout: component arrays of nx*ny*nz values, x fastest
 * (index i + nx*(j + ny*k)).  Yee positions of index (i,j,k):
 *   Ex (i+1/2, j, k)   Ey (i, j+1/2, k)   Ez (i, j, k+1/2)
 *   Hx (i, j+1/2, k+1/2)   Hy (i+1/2, j, k+1/2)   Hz (i+1/2, j+1/2, k)
 * The domain spans [0, n] along each axis.  Emitter positions are in cell
 * units in that frame.
 *
 * Errors: every call returns an mlk_status; on failure mlk_last_error()
 * returns a thread-local message.  Nothing aborts across the ABI.  A device
 * fault reported by the HIP runtime maps to MLK_EDEVICE and leaves the
 * simulation in an undefined state (destroy it).
 *
 * Memory: "mem_kind" arguments say whether a pointer is host memory
 * (MLK_MEM_HOST) or device memory on the simulation's GPU (MLK_MEM_DEVICE).
 * Inputs are copied; the caller keeps ownership of every buffer it passes.
 * All device memory of a simulation is owned by the library and freed by
 * mlk_destroy.
 *
 * Streams: all work is enqueued on the stream given in the grid description
 * (a hipStream_t, NULL = a stream the library creates).  mlk_step is
 * asynchronous; getters synchronise that stream.
 */
#ifndef MLK_H
#define MLK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MLK_OK = 0,
  MLK_EINVAL = 1,        /* an argument is out of range or inconsistent */
  MLK_ENOMEM = 2,        /* device or host allocation failed */
  MLK_EDEVICE = 3,       /* HIP runtime error or device fault */
  MLK_ESTATE = 4,        /* call not allowed in the current state */
  MLK_EUNSUPPORTED = 5,  /* valid request this build does not implement */
  MLK_ENUMERIC = 6       /* non-finite state detected */
} mlk_status;

enum { MLK_FP64 = 0, MLK_FP32_FIELDS = 1 };
enum { MLK_BC_PEC = 0, MLK_BC_PERIODIC = 1, MLK_BC_CPML = 2 };
enum { MLK_MEM_HOST = 0, MLK_MEM_DEVICE = 1 };
/* Yee sweep variant: one fused H+E pass (default) or separate H and E passes.  The
 * fused sweep addresses each field array and the CPML psi buffer with 32-bit byte
 * offsets: mlk_create refuses it (MLK_EUNSUPPORTED) when a field array or the psi
 * buffer would reach 4 GiB (about 1024^3 cells in FP32); the plain sweep has no such
 * limit. */
enum { MLK_SWEEP_FUSED = 0, MLK_SWEEP_PLAIN = 1 };
/* Current scatter variant: deterministic owner-computes (default) or atomics. */
enum { MLK_SCATTER_OWNER = 0, MLK_SCATTER_ATOMIC = 1 };
/* Series kinds for mlk_get_series. */
enum { MLK_SERIES_PROBE = 0, MLK_SERIES_FLUX = 1, MLK_SERIES_POPULATION = 2, MLK_SERIES_ENERGY = 3 };

typedef struct mlk_sim mlk_sim;

typedef struct {
  int32_t nx, ny, nz;        /* cells per axis, >= 1 */
  double dx;                 /* cell size (> 0) */
  double courant;            /* dt = courant * dx; 0 < courant <= 1/sqrt(3) */
  int32_t precision;         /* MLK_FP64, or MLK_FP32_FIELDS (E, H, psi, 1/eps, kernel
                                weights in FP32; rho, E~, mu_dot, flux in FP64) */
  int32_t bc[6];             /* per face x-, x+, y-, y+, z-, z+: MLK_BC_*; periodic must
                                pair on an axis; a CPML is backed by a metallic wall */
  int32_t cpml_cells[6];     /* CPML thickness per face (cells), 1 .. n/2 when CPML */
  double cpml_m;             /* grading order of sigma and kappa (default 3) */
  double cpml_sigma_scale;   /* sigma_max = scale * (m + 1) / dx (default 0.8) */
  double cpml_kappa_max;     /* default 1 */
  double cpml_alpha_max;     /* default 0 */
  double window_r;           /* kernel window half-width in units of sigma (default 3) */
  void* stream;              /* hipStream_t to enqueue on; NULL = library-owned stream */
  int32_t device;            /* HIP device ordinal */
  int32_t sweep;             /* MLK_SWEEP_* */
  int32_t scatter;           /* MLK_SCATTER_* */
} mlk_grid_desc;

/* Fill a description with defaults: 32^3 PEC, dx 1, courant 0.5, FP64,
 * CPML m 3 / scale 0.8 / kappa 1 / alpha 0, window 3 sigma, device 0. */
void mlk_grid_desc_init(mlk_grid_desc* g);

const char* mlk_last_error(void);
const char* mlk_version(void);

/* Create a simulation: E^0 = 0, H^{-1/2} = 0, psi = 0, eps_r = 1, no emitters. */
mlk_status mlk_create(const mlk_grid_desc* g, mlk_sim** out);
mlk_status mlk_destroy(mlk_sim* s);

/* Caller-owned device memory for the evolving state (e.g. tensors of the caller's
 * framework), in place of the library's own allocations.  field[q][c] is component
 * c (Ex, Ey, Ez, Hx, Hy, Hz) of field set q, bytes[0] bytes each (nx*ny*nz values
 * of the field precision, x fastest); set 1 exists in the fused sweep only, whose two
 * sets swap roles every step (mlk_get_field_set says which holds E^n and
 * H^{n-1/2} now).  psi[q]: the CPML state of set q (bytes[1], layout of the
 * checkpoint), only with CPML faces.  tls_state: (rho11, Re rho01, Im rho01) per
 * two-level emitter in id order (bytes[2]); ml_state: the multilevel states
 * (bytes[3], as the checkpoint holds them).  NULL entries keep the library's
 * buffer.  Each buffer given takes over the current contents of the one it
 * replaces, which is freed; from then on the library reads and writes the
 * caller's memory and never frees it.  The caller keeps ownership and keeps every
 * bound buffer alive and unmoved until mlk_destroy.  Pointers must be device memory
 * on the sim's GPU, 16-byte aligned (256 recommended).  Emitter states can be bound
 * once every emitter is added (adding emitters afterwards: ESTATE).  EINVAL: a set-1
 * or psi buffer the sim does not have, misalignment; ESTATE: in a batch. */
typedef struct {
  void* field[2][6];
  void* psi[2];
  double* tls_state;
  double* ml_state;
} mlk_buffers;
/* Sizes in bytes of one field array, one psi set, the two-level and the multilevel
 * states, into bytes[4]. */
mlk_status mlk_buffer_bytes(mlk_sim* s, size_t bytes[4]);
mlk_status mlk_bind_device_buffers(mlk_sim* s, const mlk_buffers* b);
/* Which field set (0 or 1) holds the current fields (always 0 in the plain sweep). */
mlk_status mlk_get_field_set(mlk_sim* s, int32_t* set);

/* Relative permittivity per cell, nx*ny*nz doubles, x fastest; every E
 * component with index (i,j,k) uses eps_r(i,j,k) (staircase, eq. Dromega with
 * a static eps_r).  EINVAL if any value is < 1 or not finite.  While the grid
 * is known to be vacuum (eps_r never set, set to all ones here, or set to ones
 * only by mlk_set_eps_box) the fused sweeps skip the 1/eps_r array; results
 * are the same bit for bit. */
mlk_status mlk_set_eps(mlk_sim* s, const double* eps, int32_t mem_kind);

/* Overwrite one field component (0..2 = Ex..Ez at E^n, 3..5 = Hx..Hz at
 * H^{n-1/2}) from nx*ny*nz doubles; used to set initial conditions. */
mlk_status mlk_set_field(mlk_sim* s, int32_t comp, const double* src, int32_t mem_kind);

/* Two-level emitters (eq. von-Neumann-tls, basic TLS driver: H0 = diag(0, w0),
 * mu = d sigma_x, no Lindblad term).  Host arrays of n entries:
 *   pos[3n]    centre in cell units,
 *   sigma[n]   Gaussian width (standard deviation, cells; the paper uses dx),
 *   gamma[n]   coupling rescale (eq. Polarization_mol, default 1),
 *   omega0[n]  transition frequency,
 *   dipole[3n] d = mu01 * unit orientation,
 *   rho0[3n]   initial rho11, Re rho01, Im rho01 (rho01 = <0|rho|1>).
 * EINVAL if a state is not a density matrix, sigma <= 0, or a kernel window
 * (R*sigma + 1 cells around the centre) reaches a metallic wall or the CPML
 * interface on a non-periodic axis.  Ids are contiguous from *first_id. */
mlk_status mlk_add_tls(mlk_sim* s, int32_t n, const double* pos, const double* sigma,
                       const double* gamma, const double* omega0, const double* dipole,
                       const double* rho0, int32_t* first_id);

/* Multilevel emitters with pure dephasing (the open model of Sec. II.B.1):
 * H0 = diag(energies) in its eigenbasis, mu^c = d^c M with M real symmetric,
 * Lindblad operators sqrt(gphi)|k><k| so coherences decay at gphi.  One step is
 * dephasing(dt/2), then rho <- U rho U^+ with U = exp(-i H_eff dt) (exact for
 * piecewise-constant E~), then dephasing(dt/2); mu_dot = Tr(rho_dot mu) at the
 * new state (eq. dipole_derivative).  The state is kept in FP64 in both modes.
 * Host arrays: nlev[n] in 2..6 (else EUNSUPPORTED); energies packed with
 * offsets eoff[n]; M (nlev^2 row-major, exactly symmetric) and rho0 (nlev^2
 * complex, re/im interleaved; Hermitian, unit trace, else EINVAL) packed with
 * offsets moff[n] (in entries); dipole[3n], gphi[n] >= 0, pos[3n], sigma[n],
 * gamma[n] as for mlk_add_tls.  The arrays are copied.  Ids are contiguous from
 * *first_id and shared with the two-level emitters; populations Re rho_kk,
 * k = 1..nlev-1, follow the emitter's earlier ones in a population record. */
mlk_status mlk_add_multilevel(mlk_sim* s, int32_t n, const int32_t* nlev, const int64_t* eoff,
                              const int64_t* moff, const double* energies, const double* mop,
                              const double* dipole, const double* gphi, const double* rho0,
                              const double* pos, const double* sigma, const double* gamma,
                              int32_t* first_id);

/* Soft current sheet on plane `index` of `axis` injecting component `comp`
 * with surface density amp * s(t), s(t) = cos(omega (t - t0)) exp(-(t-t0)^2/(2 tau^2))
 * evaluated at t = (n + 1/2) dt (the Gaussian pulse of App. B). */
mlk_status mlk_add_plane_source(mlk_sim* s, int32_t axis, int32_t index, int32_t comp,
                                double amp, double omega, double tau, double t0);
/* Point current element amp * s(t) / dx^3 on component comp at ijk. */
mlk_status mlk_add_point_source(mlk_sim* s, int32_t comp, const int32_t ijk[3], double amp,
                                double omega, double tau, double t0);

/* Probe of field component comp (0..5) at ijk: the field at its Yee point after
 * each step's E update, E^{n+1} (or H^{n+1/2}), one value per step (the time series
 * of the local field that the examples of Sec. IV read). */
mlk_status mlk_add_probe(mlk_sim* s, int32_t comp, const int32_t ijk[3], int32_t* id);
/* Poynting flux through plane `index` (1 .. n-1) of `axis`, one value per step:
 * F^{n+1/2} = dx^2 sum (E_u H_v - E_v H_u) with E averaged over n, n+1 and H over
 * the two half cells across the plane, (axis,u,v) cyclic; the running
 * integral dt * sum F is kept as well (the energy that the plane-wave pulse of
 * App. B carries through a plane, from eq. Maxwell).  One flux plane per
 * simulation. */
mlk_status mlk_add_flux_plane(mlk_sim* s, int32_t axis, int32_t index);
/* Record Re rho_kk, k >= 1, of every emitter on steps with n % every == 0, right
 * after the emitter step (the populations at t_{n+1/2}; the excited-state
 * population of eq. population_decay_superradiance, Sec. IV.A). */
mlk_status mlk_record_populations(mlk_sim* s, int32_t every);
/* Record the discrete field energy (Poynting's theorem for eq. Maxwell on the Yee
 * grid) on steps with n % every == 0 (0: off):
 *   W^n = dx^3 [ 1/2 sum eps_r |E^n|^2 + 1/2 sum H^{n+1/2} . H^{n-1/2} ],
 * summed in FP64 in a fixed order.  It is exactly invariant without currents,
 * sources and CPML; with them it changes by the work done on the currents and
 * the loss in the layers.  Read with mlk_get_series(MLK_SERIES_ENERGY).  Before the
 * first step.  EUNSUPPORTED in the plain sweep (the detector reads both field
 * buffers of the fused sweep) and with a cavity; batches refuse a member that
 * records it. */
mlk_status mlk_record_energy(mlk_sim* s, int32_t every);

/* Advance nsteps full coupled steps (asynchronous). */
mlk_status mlk_step(mlk_sim* s, int64_t nsteps);

/* Classical-path stepping (eq. E_analytical; the prescribed-field solver of the
 * paper's table of EM solvers): nsteps steps of dt of every emitter under a
 * given field, with no grid and no back-action.  Et holds nsteps x M x 3
 * doubles, step-major and in emitter-id order: the field each emitter sees, as
 * the gather would give it (gamma times the smeared E), in host or device
 * memory (mem_kind; the caller keeps ownership).  Each step advances the
 * two-level and multilevel states exactly as the coupled step does and forms
 * mu_dot; the fields, the step counter and the series do not change.  tls_out
 * (nullable, same memory kind) receives after every step the states (rho11,
 * Re rho01, Im rho01) of the two-level emitters in id order: nsteps x ntls x 3
 * doubles.  mlk_get_rho and mlk_get_tls_state read the final states,
 * mlk_get_emitter_io the last step's E~ and mu_dot.  Returns when host buffers
 * are done with; with device buffers it is asynchronous on the sim's stream.
 * EINVAL: negative nsteps, bad mem_kind, null Et (with emitters, nsteps > 0). */
mlk_status mlk_step_prescribed(mlk_sim* s, int64_t nsteps, const double* Et, int32_t mem_kind,
                               double* tls_out);
/* Classical-path steps under a travelling pulse evaluated on the device (eq.
 * E_analytical: a waveform of z - ct, propagating along +z, c = 1): over the q-th
 * step (q = 0 .. nsteps-1), centred at t = t_start + q dt, emitter m at height z_m
 * (its centre, cell units) sees
 *   E~_m = gamma_m amp f(t - (z_m - z0)) pol,
 *   f(u) = cos(omega (u - t0)) exp(-(u - t0)^2 / (2 tau^2))   (the pulse of App. B),
 * with no grid and no back-action; the states advance exactly as in
 * mlk_step_prescribed.  tls_out (host, nullable): the two-level states after every
 * step, nsteps x ntls x 3 doubles.  EINVAL: non-finite parameters, tau <= 0.
 * Returns when tls_out is filled; otherwise asynchronous. */
mlk_status mlk_step_prescribed_wave(mlk_sim* s, int64_t nsteps, const double pol[3], double amp,
                                    double omega, double tau, double t0, double z0,
                                    double t_start, double* tls_out);
/* The same classical-path steps for callers that cannot allocate device memory
 * (tight driver loops, code that forbids hipMalloc): with host buffers the field
 * and the recorded states pass through a fixed 16 MiB staging array on each device
 * (2,097,152 doubles, allocated when the library is loaded and held until the
 * process ends) instead of staging allocated per call; with device buffers nothing
 * is staged.  No hipMalloc, hipFree or other allocating call is made.  Results are
 * those of mlk_step_prescribed, bit for bit.  A step needs 3 M doubles of staging
 * (M emitters) plus 3 ntls with tls_out; EINVAL when that exceeds the array (about
 * 700,000 emitters, 350,000 two-level ones with tls_out); otherwise as many steps
 * as fit go through the array at a time.  All calls on one GPU share its array:
 * calls that overlap in time on one GPU (from several host threads) race and are
 * not allowed.  Returns when the host buffers are done with. */
mlk_status mlk_step_prescribed_noalloc(mlk_sim* s, int64_t nsteps, const double* Et,
                                       int32_t mem_kind, double* tls_out);
/* Wait for the sim's work.  Also the non-finite watchdog (robustness, Sec. III item
 * (v)): every emitter step checks its new state and dipole rate, and the detectors
 * check each probe sample and flux value; the first step at which one is not finite
 * is kept on the device, and mlk_sync (and mlk_batch_sync for every member) then
 * returns MLK_ENUMERIC naming it, on every call until mlk_checkpoint_load restores a
 * state.  A non-finite field reaches the watchdog through the emitters whose window
 * it touches and through the probes and the flux plane.  Stepping goes on regardless
 * (the values stay what the arithmetic gives). */
mlk_status mlk_sync(mlk_sim* s);
mlk_status mlk_step_count(mlk_sim* s, int64_t* n);

/* Single-mode cavity in place of the grid (Sec. II.A.2: the normal-mode field
 * Hamiltonian with the dipole self-energy and its equations of motion, in the
 * single-mode limit; eps0 = 1).  One mode of frequency omega > 0 and effective
 * volume V > 0 with an x and a y polarisation; the coupling is
 * eps = omega / sqrt(V).  Every emitter then sees the same field
 * E~ = -sum_l (eps q_l + d_l / V) e_l (gamma, positions and widths are not
 * used), where d = sum_m <mu^(m)> (eq. dklambda_def), and the mode obeys
 * q_l'' = -omega^2 q_l - eps d_l.  The total dipole at the integer time t_n is
 * formed from the latest states rho^{n-1/2}, carried half a step forward by
 * their rate (eq. dipole_derivative; second order):
 *   d^n = sum_m [ <mu^(m)>(rho^{n-1/2}) + (dt/2) mu_dot^(m)(rho^{n-1/2}) ].
 * Per step: E~ from q^n and d^n, the emitter steps (as the coupled step does
 * them), then
 *   p^{n+1/2} = p^{n-1/2} - dt (omega^2 q^n + eps d^n),  q^{n+1} = q^n + dt p^{n+1/2},
 * and d^{n+1} from the new states; d^0 comes from the states at the call, and
 * mlk_set_tls_dipoles forms it again from the new dipoles.  q0 and p0 are
 * (x, y): q at step 0 and p half a step before.  mlk_step then advances the
 * emitters and the mode and leaves the grid alone; populations are recorded as
 * usual and checkpoints carry the mode state.  Call after every emitter is
 * added and before the first step.  EINVAL: null pointers, omega or V not
 * positive and finite, non-finite q0/p0.  ESTATE: after stepping, in a batch.
 * EUNSUPPORTED: with sources, probes or a flux plane.  Afterwards adding
 * emitters (ESTATE), sources, probes or a flux plane, batching, the adjoint
 * (EUNSUPPORTED) and mlk_step_prescribed (ESTATE) are refused. */
mlk_status mlk_set_cavity(mlk_sim* s, double omega, double volume, const double q0[2],
                          const double p0[2]);
/* Dispersive block (eq. Dromega: a dielectric function made of Lorentz and Drude
 * oscillators): one pole chi(w) = sigma w0^2 / (kappa w0^2 - w^2 - i w gamma),
 * kappa = 1 (drude = 0, Lorentz) or 0 (drude = 1, Drude), over the half-open
 * cell box {x0, y0, z0, x1, y1, z1}.  eps_r of the box cells (mlk_set_eps) is
 * eps_infinity.  Its polarisation P (zero at the start, one value per E
 * component per box cell, held by the library in the field precision) obeys
 * P'' + gamma P' + kappa w0^2 P = sigma w0^2 E, advanced by central
 * differences from P^n, P^{n-1} and E^n, and the E update becomes
 * E^{n+1} = E^n + (dt (curl H - J) - sum_poles (P^{n+1} - P^n)) / eps_inf.
 * Poles may overlap (their P add).  On a non-periodic axis the box stays clear
 * of the CPML layers and of the index-0 wall plane.  Before the first step; at
 * most 8 poles; checkpoints carry P.  EINVAL: box outside those limits or
 * empty, omega0 <= 0, gamma < 0, non-finite values, a ninth pole.  ESTATE:
 * after stepping, in a batch.  EUNSUPPORTED: with a cavity.  Batches and the
 * adjoint refuse a sim with poles (EUNSUPPORTED). */
mlk_status mlk_add_susceptibility(mlk_sim* s, const int32_t box[6], double omega0, double gamma,
                                  double sigma, int32_t drude);
/* Mode state (q_x, q_y, p_x, p_y, d_x, d_y) into out[6] (host): q and d at the
 * current step, p half a step before.  Synchronises.  ESTATE: no cavity. */
mlk_status mlk_get_cavity(mlk_sim* s, double out[6]);


/* Read a field component (0..5) as nx*ny*nz doubles. */
mlk_status mlk_get_field(mlk_sim* s, int32_t comp, double* dst, int32_t mem_kind);
/* Density matrix of emitter id as n*n complex (re/im interleaved); *nlev gets n.
 * cap is the capacity of dst in doubles. */
mlk_status mlk_get_rho(mlk_sim* s, int32_t id, double* dst, int32_t cap, int32_t* nlev);
/* Two-level states (rho11, Re rho01, Im rho01) of ids first..first+count-1. */
mlk_status mlk_get_tls_state(mlk_sim* s, int32_t first, int32_t count, double* dst);
/* E~ and mu_dot of every emitter from the last step, 3 doubles each (host). */
mlk_status mlk_get_emitter_io(mlk_sim* s, double* Et, double* mudot);
/* Copy a recorded series; *len gets its full length, at most cap values copied.
 * Populations are laid out [record][emitter excited levels]. */
mlk_status mlk_get_series(mlk_sim* s, int32_t kind, int32_t id, double* dst, int64_t cap,
                          int64_t* len);
mlk_status mlk_get_flux_total(mlk_sim* s, double* total);

/* Checkpoint of the whole evolving state (restart after a failure, Sec. III
 * item (v)); restoring gives an identical continuation, bit for bit.  Recorded
 * series are not part of it.  Layout, in order: Ex, Ey, Ez, Hx, Hy, Hz (nx*ny*nz
 * values each in the field precision, x fastest); the CPML state (with a CPML
 * face); the two-level states (rho11, Re rho01, Im rho01 per two-level emitter, in
 * id order); the multilevel states; E~ and mu_dot (3 doubles per emitter); the step
 * counter (int64); the flux integral (with a flux plane); the cavity mode (6
 * doubles); the dispersive poles.  mlk_checkpoint_load also clears the non-finite
 * watchdog (see mlk_sync). */
mlk_status mlk_checkpoint_size(mlk_sim* s, size_t* bytes);
mlk_status mlk_checkpoint_save(mlk_sim* s, void* dst, int32_t mem_kind);
mlk_status mlk_checkpoint_load(mlk_sim* s, const void* src, int32_t mem_kind);

/* Per-phase timing of the step loop with HIP events recorded on the sim's
 * stream around the timed phases of every step (off by default; each timed
 * phase costs one event pair per step).  mlk_set_timing(s, phases) times the
 * phases whose bit (1 << MLK_PHASE_x) is set in `phases` (0: off,
 * MLK_TIMING_ALL: every phase) and clears the accumulated times.  mlk_get_phase_time waits for the stream and
 * returns, for one phase, the summed elapsed time in ms and the number of
 * timed launches of it.  Phases:
 *   EMITTERS      field gather + emitter step + dipole rate (steps 2-4)
 *   SWEEP         the stencil kernel of the Yee sweep: the fused interior
 *                 kernel, or in the plain mode the H and E passes (steps 1, 6)
 *   SHELL         the CPML-shell passes of the fused mode (steps 1, 6)
 *   SOURCES       soft source currents (step 5)
 *   SCATTER       molecular current scatter into E (step 5)
 *   DETECTORS     flux plane save, probes, flux series, step counter (step 7) */
enum {
  MLK_PHASE_EMITTERS = 0,
  MLK_PHASE_SWEEP = 1,
  MLK_PHASE_SHELL = 2,
  MLK_PHASE_SOURCES = 3,
  MLK_PHASE_SCATTER = 4,
  MLK_PHASE_DETECTORS = 5,
  MLK_PHASE_POLES = 6, /* the two passes of the dispersive poles */
  MLK_PHASE_COUNT = 7,
  MLK_TIMING_ALL = (1 << 6) - 1
};
mlk_status mlk_set_timing(mlk_sim* s, int32_t on);
mlk_status mlk_get_phase_time(mlk_sim* s, int32_t phase, double* total_ms, int64_t* launches);

/* Interior box of the fused sweep as {lo_x, lo_y, lo_z, hi_x, hi_y, hi_z}
 * (half-open): the cells that the fused kernel owns, away from every CPML
 * layer; the cells outside it are updated by the CPML-shell passes. */
mlk_status mlk_get_interior_box(mlk_sim* s, int32_t box[6]);

/* ------------------------------------------------------------------ adjoint
 * Gradients of an objective over the next nsteps steps, by the discrete adjoint
 * (reverse mode) of the coupled step as executed, with respect to eps_r of every
 * cell of design_box {x0, y0, z0, x1, y1, z1} (half-open) and to the dipole
 * vector d of every two-level emitter.  Objectives:
 *   MLK_OBJ_FLUX:       dt sum_n F^{n+1/2}, the flux through the sim's flux plane
 *                       integrated over the steps;
 *   MLK_OBJ_POPULATION: sum_m weights[m] rho11_m after the last step (weights per
 *                       emitter id).
 * The forward run keeps the whole state every ckpt_every steps in device
 * memory; the reverse pass recomputes one segment at a time from its
 * checkpoint and undoes it, so memory is one state per segment plus one
 * segment of tape.  The result does not depend on ckpt_every.  Outputs (host
 * memory, written): grad_eps (design-box cells, x fastest; may be NULL),
 * grad_dipole (3 per emitter id; may be NULL), value (the objective).  The sim
 * is left in the state it had before the call.  Multilevel emitters: the call
 * returns MLK_EUNSUPPORTED.  MLK_ENUMERIC when a run inside the call met a
 * non-finite value (the watchdog of mlk_sync is left as it was) or the objective is
 * not finite. */
enum { MLK_OBJ_FLUX = 0, MLK_OBJ_POPULATION = 1 };
typedef struct mlk_objective {
  int32_t kind;
  const double* weights; /* population weights, one per emitter id (host) */
} mlk_objective;
mlk_status mlk_adjoint(mlk_sim* s, const mlk_objective* obj, int64_t nsteps, int32_t ckpt_every,
                       const int32_t design_box[6], double* grad_eps, double* grad_dipole,
                       double* value);

/* Device time of the last mlk_adjoint call (HIP events on the sim's stream): the
 * forward run with its checkpoints, and the reverse pass (segment recomputation,
 * adjoint steps and gradient accumulation). */
mlk_status mlk_get_adjoint_times(mlk_sim* s, double* forward_ms, double* reverse_ms);

/* eps_r over a box (values in box order, x fastest; >= 1), and the dipole
 * vectors of the two-level emitters first..first+count-1: parameters that a
 * design loop changes between runs. */
mlk_status mlk_set_eps_box(mlk_sim* s, const int32_t box[6], const double* eps, int32_t mem_kind);
mlk_status mlk_set_tls_dipoles(mlk_sim* s, int32_t first, int32_t count, const double* dipole);

/* ------------------------------------------------------------------ batches
 * Many independent sims stepped together (each one an independent run of the
 * method; the batch result equals its members run one by one, bit for bit).
 * Every phase of a step is one launch over the work of all members, so a
 * step costs about a dozen launches whatever the number of domains.  Members
 * must share precision, sweep mode, device and step count, use the
 * owner-computes scatter, and belong to no other batch; the batch runs on the
 * first member's stream.  While in a batch a member cannot be destroyed or
 * re-tuned; its getters wait for the batch's work.  mlk_batch_step enqueues
 * nsteps steps.  mlk_batch_capture records steps_per_replay steps (even in the
 * fused mode, whose two field buffers alternate) into a hipGraph;
 * mlk_batch_replay launches it nreplays times (re-capturing by itself when a
 * recorded series had to grow).  The sims keep their state and can be stepped
 * on their own after mlk_batch_destroy. */
typedef struct mlk_batch mlk_batch;
mlk_status mlk_batch_create(mlk_sim* const* sims, int32_t n, mlk_batch** out);
mlk_status mlk_batch_step(mlk_batch* b, int64_t nsteps);
mlk_status mlk_batch_capture(mlk_batch* b, int64_t steps_per_replay);
mlk_status mlk_batch_replay(mlk_batch* b, int64_t nreplays);
mlk_status mlk_batch_sync(mlk_batch* b);
mlk_status mlk_batch_destroy(mlk_batch* b);

/* Tile shape and layer mode for the batch as a whole: every member gets the same
 * (tile width, ty, kz, layer mode), chosen by timing the batch's sweep phase (the fused
 * launches and the two shell passes of one batched step, best of three runs;
 * the members' state is untouched) for every candidate, three interleaved
 * rounds.  A member tuned alone minimises its own latency; a batch wants
 * throughput over all of them.  With cache_path (NULL: no cache) the choice is
 * read from and added to the JSON file of mlk_autotune, keyed by precision,
 * member count and a hash of the members' grids.  Drops a captured graph (the
 * next mlk_batch_replay captures again).  Speed only: results do not change.
 * Plain-sweep batches have nothing to tune. */
mlk_status mlk_batch_autotune(mlk_batch* b, const char* cache_path);

/* Tile shape of the fused sweep: rows per workgroup ty (4, 8 or 16) and z planes
 * per workgroup kz (mlk_set_tuning; the sweep cuts the box's depth into depth/kz
 * chunks, rounded up, of equal cost, z-layer planes weighing more than interior
 * ones, so a chunk may hold a few planes more or less than kz), and the tile width,
 * 64 (the default) or 32 x
 * cells per workgroup (mlk_set_tile_width: narrower tiles give small grids more
 * workgroups; EINVAL for other widths, EUNSUPPORTED when the sim is in layer mode 2
 * and the width leaves no fused box over every x column).  All MLK_ESTATE while the
 * sim belongs to a batch.  mlk_autotune times every combination (and, with FP32
 * fields, every layer mode, see mlk_set_sweep_layers) on the sim's own grid, each as the
 * fused launch plus the two CPML shell passes of a step, in three interleaved
 * rounds (the state is left untouched; each candidate keeps its best round) and
 * keeps the fastest; with cache_path (NULL: no cache) results are read from and
 * added to a JSON file keyed by precision, grid, CPML thicknesses and periodic
 * axes.  The result does not depend on the tile shape (each
 * cell's arithmetic is the same), only the speed does.  Plain-sweep sims have
 * nothing to tune. */
mlk_status mlk_autotune(mlk_sim* s, const char* cache_path);
mlk_status mlk_set_tuning(mlk_sim* s, int32_t ty, int32_t kz);
mlk_status mlk_get_tuning(mlk_sim* s, int32_t* ty, int32_t* kz);
mlk_status mlk_set_tile_width(mlk_sim* s, int32_t tx);
mlk_status mlk_get_tile_width(mlk_sim* s, int32_t* tx);

/* Layer mode of the fused sweep (FP32 fields): where the cells of the y and z CPML
 * layers are updated.  0: by the plain shell passes (the fused box stops one cell
 * above the low layers and at the high ones); 1: by the fused kernel itself, which
 * then covers the whole grid and stretches their derivatives; 2: the box of mode 0
 * by the lean fused kernel (no y/z layer code, fewer registers, more waves per
 * SIMD), then the layer frame around it (the z slabs and the y slabs) in one launch
 * of the full kernel (needs y or z layers and a box spanning every x column).  The
 * default is 1 when the y and z layers are a small part of the grid ((nlo + nhi) / n
 * summed over y and z at most 1/4), else 0; mlk_autotune times every mode and keeps
 * the fastest (and caches it).  Like the tile shape, the mode changes speed, not
 * results.  FP64 fields: always 0 (MLK_EUNSUPPORTED for 1 or 2).  MLK_ESTATE while
 * the sim belongs to a batch (a batch runs modes 0 and 1; a member in mode 2 runs as
 * in mode 0). */
mlk_status mlk_set_sweep_layers(mlk_sim* s, int32_t on);
mlk_status mlk_get_sweep_layers(mlk_sim* s, int32_t* on);

/* ------------------------------------------------------------ calibration
 * Streaming copy of `bytes` (a multiple of 16) from src to dst, both device memory,
 * enqueued on `stream` (a hipStream_t; NULL = the null stream) with `blocks`
 * workgroups of 256 threads, each thread moving 8 x 16 bytes per pass with every load
 * issued before the first store.  variant: 0 ordinary loads and stores, 1 streaming
 * (nontemporal) stores, 2 streaming loads, 3 both.  Not part of the method: the
 * yardstick against which the sweep kernels' bandwidth is read.  EINVAL on bad
 * arguments, EDEVICE when the launch fails. */
mlk_status mlk_stream_copy(const void* src, void* dst, size_t bytes, int32_t variant,
                           int32_t blocks, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MLK_H */
