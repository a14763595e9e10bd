/*
 * mlk_oracle.c -- plain double-precision CPU oracle for the coupled
 * Yee-FDTD / quantum-emitter time step.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle and is
 * loaded by the test-suite, by the package smoke check and by the CPU
 * baseline leg of the benchmark.  The HIP library never links, includes or
 * calls it, and it shares no code, header or table with that library.
 *
 * Every quantity is FP64.  Each routine is the direct definition of one
 * step of the method, in the order the method takes them:
 *   - Maxwell's curl equations with the molecular current (Sec. II.A.1,
 *     eq. Maxwell), constitutive relation D = eps_r E with a static
 *     per-cell eps_r and mu = mu0 (eq. Dromega and the text after it),
 *     discretised on Yee's staggered grid; optional Lorentz and Drude
 *     poles (the dielectric functions of eq. Dromega) as polarisation
 *     oscillators advanced by central differences;
 *   - a single-mode cavity in place of the grid (Sec. II.A.2);
 *   - textbook convolutional PML backed by a perfect conductor, periodic
 *     and metallic walls (the boundary conditions of Sec. III);
 *   - Gaussian kernel normalised to unit integral, the regularised field
 *     E~ = int E . gamma kappa (eqs. Polarization_mol, E_regu_Emi);
 *   - von Neumann step of each emitter under H0 - E~ . mu (eq.
 *     von-Neumann-tls), with an optional pure-dephasing Lindblad term
 *     (Sec. II.B.1, the QuTiP-style open model);
 *   - the dipole derivative Tr(rho_dot mu) (eq. dipole_derivative) and,
 *     for the two-level system, its closed form -2 w0 mu01 Im(rho01);
 *   - the molecular current J = sum_m gamma mu_dot kappa (eqs. J_mol,
 *     Polarization_mol) that drives the next E update;
 *   - soft sources and detectors (probe, populations, Poynting flux,
 *     discrete energy).
 * The per-step order (field -> emitter -> mu_dot -> current) is the
 * exchange described in Sec. III (the socket hub's data flow).
 *
 * Units are natural: c = eps0 = mu0 = hbar = 1, lengths in cells of size dx.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_PEC 0
#define ORA_PERIODIC 1
#define ORA_CPML 2

#define ORA_OK 0
#define ORA_EINVAL 1
#define ORA_ENOMEM 2

typedef double complex cplx;

typedef struct {
  int n;          /* number of levels */
  int tls;        /* 1: exact SU(2) propagator of the basic TLS driver */
  double pos[3], sigma, gamma;
  double d[3];    /* dipole operator mu^c = d^c M */
  double en[6];   /* H0 eigenvalues (H0 is diagonal in this basis) */
  double M[36];   /* real symmetric, n x n row-major */
  double gphi;    /* pure-dephasing rate of the Lindblad term */
  cplx rho[36];
  int lo[3][3], len[3][3]; /* [component][axis] window start (unwrapped) and length */
  double* w[3];            /* normalised weights per component, x fastest */
  double Et[3], mudot[3];
} ora_emitter;

typedef struct {
  int kind;  /* 0 plane, 1 point */
  int axis, index, comp, ijk[3];
  double amp, omega, tau, t0;
} ora_source;

typedef struct {
  double* v;
  int64_t len, cap;
} ora_series;

/* One Lorentz or Drude pole of a dispersive block (Sec. II.A.1, eq. Dromega):
 * chi(w) = sigma w0^2 / (kappa w0^2 - w^2 - i w gamma), kappa = 1 (Lorentz) or
 * 0 (Drude), over the half-open cell box [lo, hi).  Its polarisation obeys
 * P'' + gamma P' + kappa w0^2 P = sigma w0^2 E for every E component stored
 * in the box; P at integer steps, current and previous. */
typedef struct {
  int lo[3], hi[3];
  double w0, gamma, sigma;
  int drude;
  double *P[3], *Pm[3];
} ora_pole;

typedef struct ora_sim {
  int N[3];
  double dx, dt, courant;
  int bc[6], npml[6];
  double pml_m, pml_sscale, pml_kmax, pml_amax, R;
  size_t ncell;
  double *E[3], *H[3], *Hprev[3], *J[3], *eps;
  double *psiE[3][3], *psiH[3][3]; /* [field component][derivative axis] */
  /* 1-D CPML tables: [axis][0 = integer positions, 1 = half-integer] */
  double *tb[3][2], *tc[3][2], *tk[3][2];
  unsigned char* tin[3][2];
  int64_t step;
  ora_emitter* em;
  int nem, cap_em;
  ora_source* src;
  int nsrc;
  int nprobe;
  int probe_comp[64], probe_ijk[64][3];
  ora_series probe_series[64];
  int flux_on, flux_axis, flux_index;
  ora_series flux_series;
  double flux_total;
  double* flux_Eu; /* E^n on the flux plane, saved before the E update */
  double* flux_Ev;
  int pop_every;
  ora_series pop_series;
  int energy_on;
  ora_series energy_series;
  /* single-mode cavity (no grid): frequency, effective volume, coupling, and the
   * mode coordinates q (integer steps), p = dq/dt (half steps) and the total
   * dipole d (integer steps), for the x and y polarisations */
  int cav_on;
  double cav_w, cav_V, cav_eps, cav_q[2], cav_p[2], cav_d[2];
  /* dispersive blocks; eps holds eps_infinity in their cells */
  ora_pole pole[8];
  int npole;
} ora_sim;

static void series_push(ora_series* s, double v) {
  if (s->len == s->cap) {
    int64_t nc = s->cap ? 2 * s->cap : 1024;
    double* p = (double*)realloc(s->v, (size_t)nc * sizeof(double));
    if (!p) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
    s->v = p;
    s->cap = nc;
  }
  s->v[s->len++] = v;
}

static inline size_t IDX(const ora_sim* s, int i, int j, int k) {
  return (size_t)i + (size_t)s->N[0] * ((size_t)j + (size_t)s->N[1] * (size_t)k);
}

/* Value of a field array at integer index (i,j,k) with the wall rules:
 * periodic axes wrap; beyond a metallic (or PML-backing) wall the value is
 * the tangential E on the wall, i.e. zero. */
static inline double fetch(const ora_sim* s, const double* a, int i, int j, int k) {
  int q[3] = {i, j, k};
  for (int ax = 0; ax < 3; ++ax) {
    if (q[ax] < 0 || q[ax] >= s->N[ax]) {
      if (s->bc[2 * ax] == ORA_PERIODIC) {
        q[ax] = ((q[ax] % s->N[ax]) + s->N[ax]) % s->N[ax];
      } else {
        return 0.0;
      }
    }
  }
  return a[IDX(s, q[0], q[1], q[2])];
}

/* CPML grading at coordinate x along an axis (textbook convolutional PML,
 * polynomial grading of order m for sigma and kappa, linear alpha). */
static void pml_profile(const ora_sim* s, int ax, double x, double* b, double* c, double* kinv,
                        unsigned char* inside) {
  double Nn = (double)s->N[ax];
  double depth = -1.0, d = 0.0;
  if (s->bc[2 * ax] == ORA_CPML && x < (double)s->npml[2 * ax]) {
    d = (double)s->npml[2 * ax];
    depth = d - x;
  } else if (s->bc[2 * ax + 1] == ORA_CPML && x > Nn - (double)s->npml[2 * ax + 1]) {
    d = (double)s->npml[2 * ax + 1];
    depth = x - (Nn - d);
  }
  if (depth < 0.0) {
    *b = 1.0; *c = 0.0; *kinv = 1.0; *inside = 0;
    return;
  }
  double u = depth / d;
  double smax = s->pml_sscale * (s->pml_m + 1.0) / s->dx;
  double sig = smax * pow(u, s->pml_m);
  double kap = 1.0 + (s->pml_kmax - 1.0) * pow(u, s->pml_m);
  double alp = s->pml_amax * (1.0 - u);
  *b = exp(-(sig / kap + alp) * s->dt);
  *c = (sig > 0.0) ? sig * (*b - 1.0) / (sig * kap + kap * kap * alp) : 0.0;
  *kinv = 1.0 / kap;
  *inside = 1;
}

/* Spatial derivative with the CPML stretching: (1/kappa) dF + psi, where
 * psi <- b psi + c dF.  Outside the layers it is dF itself. */
static inline double stretched(const ora_sim* s, int ax, int half, int pos, double dF, double* psi,
                               size_t id) {
  if (!s->tin[ax][half][pos]) return dF;
  psi[id] = s->tb[ax][half][pos] * psi[id] + s->tc[ax][half][pos] * dF;
  return s->tk[ax][half][pos] * dF + psi[id];
}

ora_sim* ora_create(const int* N, double dx, double courant, const int* bc, const int* npml,
                    double pml_m, double pml_sscale, double pml_kmax, double pml_amax, double R,
                    int* status) {
  *status = ORA_EINVAL;
  if (courant <= 0.0 || courant > 1.0 / sqrt(3.0) || dx <= 0.0 || R <= 0.0) return NULL;
  for (int ax = 0; ax < 3; ++ax) {
    if (N[ax] < 1) return NULL;
    if ((bc[2 * ax] == ORA_PERIODIC) != (bc[2 * ax + 1] == ORA_PERIODIC)) return NULL;
    for (int f = 0; f < 2; ++f) {
      if (bc[2 * ax + f] < 0 || bc[2 * ax + f] > 2) return NULL;
      if (bc[2 * ax + f] == ORA_CPML && (npml[2 * ax + f] < 1 || npml[2 * ax + f] > N[ax] / 2))
        return NULL;
    }
  }
  ora_sim* s = (ora_sim*)calloc(1, sizeof(ora_sim));
  if (!s) { *status = ORA_ENOMEM; return NULL; }
  memcpy(s->N, N, 3 * sizeof(int));
  s->dx = dx;
  s->courant = courant;
  s->dt = courant * dx; /* c = 1 */
  memcpy(s->bc, bc, 6 * sizeof(int));
  for (int f = 0; f < 6; ++f) s->npml[f] = (bc[f] == ORA_CPML) ? npml[f] : 0;
  s->pml_m = pml_m;
  s->pml_sscale = pml_sscale;
  s->pml_kmax = pml_kmax;
  s->pml_amax = pml_amax;
  s->R = R;
  s->ncell = (size_t)N[0] * N[1] * N[2];
  for (int c = 0; c < 3; ++c) {
    s->E[c] = (double*)calloc(s->ncell, sizeof(double));
    s->H[c] = (double*)calloc(s->ncell, sizeof(double));
    s->J[c] = (double*)calloc(s->ncell, sizeof(double));
  }
  s->eps = (double*)malloc(s->ncell * sizeof(double));
  for (size_t q = 0; q < s->ncell; ++q) s->eps[q] = 1.0;
  for (int ax = 0; ax < 3; ++ax) {
    int has = (bc[2 * ax] == ORA_CPML) || (bc[2 * ax + 1] == ORA_CPML);
    for (int c = 0; c < 3; ++c) {
      if (has && c != ax) {
        s->psiE[c][ax] = (double*)calloc(s->ncell, sizeof(double));
        s->psiH[c][ax] = (double*)calloc(s->ncell, sizeof(double));
      }
    }
    for (int h = 0; h < 2; ++h) {
      s->tb[ax][h] = (double*)malloc(N[ax] * sizeof(double));
      s->tc[ax][h] = (double*)malloc(N[ax] * sizeof(double));
      s->tk[ax][h] = (double*)malloc(N[ax] * sizeof(double));
      s->tin[ax][h] = (unsigned char*)malloc(N[ax]);
      for (int i = 0; i < N[ax]; ++i)
        pml_profile(s, ax, (double)i + 0.5 * h, &s->tb[ax][h][i], &s->tc[ax][h][i],
                    &s->tk[ax][h][i], &s->tin[ax][h][i]);
    }
  }
  *status = ORA_OK;
  return s;
}

void ora_destroy(ora_sim* s) {
  if (!s) return;
  for (int c = 0; c < 3; ++c) {
    free(s->E[c]); free(s->H[c]); free(s->Hprev[c]); free(s->J[c]);
    for (int ax = 0; ax < 3; ++ax) { free(s->psiE[c][ax]); free(s->psiH[c][ax]); }
    for (int h = 0; h < 2; ++h) {
      free(s->tb[c][h]); free(s->tc[c][h]); free(s->tk[c][h]); free(s->tin[c][h]);
    }
  }
  free(s->eps);
  for (int k = 0; k < s->npole; ++k)
    for (int c = 0; c < 3; ++c) { free(s->pole[k].P[c]); free(s->pole[k].Pm[c]); }
  for (int m = 0; m < s->nem; ++m)
    for (int c = 0; c < 3; ++c) free(s->em[m].w[c]);
  free(s->em);
  free(s->src);
  for (int p = 0; p < s->nprobe; ++p) free(s->probe_series[p].v);
  free(s->flux_series.v); free(s->flux_Eu); free(s->flux_Ev);
  free(s->pop_series.v);
  free(s->energy_series.v);
  free(s);
}

double ora_dt(const ora_sim* s) { return s->dt; }
int64_t ora_step_count(const ora_sim* s) { return s->step; }

int ora_set_eps(ora_sim* s, const double* eps) {
  for (size_t q = 0; q < s->ncell; ++q)
    if (!(eps[q] >= 1.0)) return ORA_EINVAL;
  memcpy(s->eps, eps, s->ncell * sizeof(double));
  return ORA_OK;
}

/* comp 0..2 = Ex,Ey,Ez (E^n); 3..5 = Hx,Hy,Hz (H^{n-1/2}) */
int ora_set_field(ora_sim* s, int comp, const double* v) {
  if (comp < 0 || comp > 5) return ORA_EINVAL;
  double* dst = comp < 3 ? s->E[comp] : s->H[comp - 3];
  memcpy(dst, v, s->ncell * sizeof(double));
  return ORA_OK;
}

int ora_get_field(const ora_sim* s, int comp, double* v) {
  if (comp < 0 || comp > 5) return ORA_EINVAL;
  const double* src = comp < 3 ? s->E[comp] : s->H[comp - 3];
  memcpy(v, src, s->ncell * sizeof(double));
  return ORA_OK;
}

/* ---------------------------------------------------------------- kernel */

/* Window of component c of an emitter: every Yee point of that component
 * whose offset from the centre is within R*sigma on each axis; weights
 * are the Gaussian exp(-|p-r|^2 / 2 sigma^2) normalised to unit sum, the
 * discrete form of a unit-integral kernel (eq. Polarization_mol). */
static int build_window(ora_sim* s, ora_emitter* e) {
  double rs = s->R * e->sigma;
  for (int ax = 0; ax < 3; ++ax) {
    if (s->bc[2 * ax] == ORA_PERIODIC) {
      /* a periodic axis of one cell is an invariant direction (2-D run) */
      if (s->N[ax] > 1 && (double)s->N[ax] < 2.0 * rs + 2.0) return ORA_EINVAL;
    } else {
      double lo = (double)s->npml[2 * ax], hi = (double)(s->N[ax] - s->npml[2 * ax + 1]);
      if (e->pos[ax] - (rs + 1.0) < lo || e->pos[ax] + (rs + 1.0) > hi) return ORA_EINVAL;
    }
  }
  for (int c = 0; c < 3; ++c) {
    for (int ax = 0; ax < 3; ++ax) {
      double sh = (ax == c) ? 0.5 : 0.0;
      if (s->N[ax] == 1 && s->bc[2 * ax] == ORA_PERIODIC) {
        /* invariant direction: the kernel is uniform along it, so the window
         * is the single cell layer and its factor cancels in the normalisation */
        e->lo[c][ax] = 0;
        e->len[c][ax] = 1;
        continue;
      }
      int first = 1, lo = 0, hi = -1;
      int a0 = (int)floor(e->pos[ax] - rs) - 2, a1 = (int)ceil(e->pos[ax] + rs) + 2;
      for (int i = a0; i <= a1; ++i) {
        double off = (double)i + sh - e->pos[ax];
        if (off * off <= rs * rs) {
          if (first) { lo = i; first = 0; }
          hi = i;
        }
      }
      e->lo[c][ax] = lo;
      e->len[c][ax] = hi - lo + 1;
      if (e->len[c][ax] < 1) return ORA_EINVAL;
    }
    int L0 = e->len[c][0], L1 = e->len[c][1], L2 = e->len[c][2];
    e->w[c] = (double*)malloc((size_t)L0 * L1 * L2 * sizeof(double));
    if (!e->w[c]) return ORA_ENOMEM;
    double sum = 0.0;
    for (int kk = 0; kk < L2; ++kk)
      for (int jj = 0; jj < L1; ++jj)
        for (int ii = 0; ii < L0; ++ii) {
          double p[3] = {e->lo[c][0] + ii + (c == 0 ? 0.5 : 0.0),
                         e->lo[c][1] + jj + (c == 1 ? 0.5 : 0.0),
                         e->lo[c][2] + kk + (c == 2 ? 0.5 : 0.0)};
          double r2 = 0.0;
          for (int ax = 0; ax < 3; ++ax) r2 += (p[ax] - e->pos[ax]) * (p[ax] - e->pos[ax]);
          double g = exp(-r2 / (2.0 * e->sigma * e->sigma));
          e->w[c][ii + L0 * (jj + L1 * kk)] = g;
          sum += g;
        }
    for (int q = 0; q < L0 * L1 * L2; ++q) e->w[c][q] /= sum;
  }
  return ORA_OK;
}

static inline size_t window_cell(const ora_sim* s, const ora_emitter* e, int c, int ii, int jj,
                                 int kk) {
  int q[3] = {e->lo[c][0] + ii, e->lo[c][1] + jj, e->lo[c][2] + kk};
  for (int ax = 0; ax < 3; ++ax) q[ax] = ((q[ax] % s->N[ax]) + s->N[ax]) % s->N[ax];
  return IDX(s, q[0], q[1], q[2]);
}

static int grow_emitters(ora_sim* s, int n) {
  if (s->nem + n <= s->cap_em) return ORA_OK;
  int nc = s->cap_em ? s->cap_em : 16;
  while (nc < s->nem + n) nc *= 2;
  ora_emitter* p = (ora_emitter*)realloc(s->em, (size_t)nc * sizeof(ora_emitter));
  if (!p) return ORA_ENOMEM;
  s->em = p;
  s->cap_em = nc;
  return ORA_OK;
}

/* Two-level emitters: H0 = diag(0, w0), mu = d sigma_x (eq. von-Neumann-tls).
 * rho0 per emitter: (rho11, Re rho01, Im rho01). */
int ora_add_tls(ora_sim* s, int n, const double* pos, const double* sigma, const double* gamma,
                const double* omega0, const double* dipole, const double* rho0) {
  if (grow_emitters(s, n)) return ORA_ENOMEM;
  for (int q = 0; q < n; ++q) {
    double p11 = rho0[3 * q], r = rho0[3 * q + 1], im = rho0[3 * q + 2];
    if (!(p11 >= 0.0 && p11 <= 1.0) || r * r + im * im > p11 * (1.0 - p11) * (1.0 + 1e-12) + 1e-300)
      return ORA_EINVAL;
    if (!(sigma[q] > 0.0)) return ORA_EINVAL;
  }
  int base = s->nem;
  for (int q = 0; q < n; ++q) {
    ora_emitter* e = &s->em[base + q];
    memset(e, 0, sizeof(*e));
    e->n = 2;
    e->tls = 1;
    memcpy(e->pos, pos + 3 * q, 3 * sizeof(double));
    e->sigma = sigma[q];
    e->gamma = gamma[q];
    memcpy(e->d, dipole + 3 * q, 3 * sizeof(double));
    e->en[0] = 0.0;
    e->en[1] = omega0[q];
    e->M[1] = 1.0;
    e->M[2] = 1.0;
    e->gphi = 0.0;
    double p11 = rho0[3 * q];
    cplx r01 = rho0[3 * q + 1] + I * rho0[3 * q + 2];
    e->rho[0] = 1.0 - p11;
    e->rho[1] = r01;
    e->rho[2] = conj(r01);
    e->rho[3] = p11;
    int st = build_window(s, e);
    if (st) {
      for (int c = 0; c < 3; ++c) free(e->w[c]);
      for (int r2 = 0; r2 < q; ++r2)
        for (int c = 0; c < 3; ++c) free(s->em[base + r2].w[c]);
      return st;
    }
  }
  s->nem += n;
  return ORA_OK;
}

/* Multilevel emitters with pure dephasing (QuTiP-style open model).
 * nlev[q] in 2..6; energies packed at eoff, M (n*n real symmetric) and
 * rho0 (n*n complex, interleaved re/im) packed at moff. */
int ora_add_multilevel(ora_sim* s, int n, const int* nlev, const int64_t* eoff,
                       const int64_t* moff, const double* energies, const double* mop,
                       const double* dipole, const double* gphi, const double* rho0,
                       const double* pos, const double* sigma, const double* gamma) {
  if (grow_emitters(s, n)) return ORA_ENOMEM;
  for (int q = 0; q < n; ++q) {
    int L = nlev[q];
    if (L < 2 || L > 6 || !(sigma[q] > 0.0) || !(gphi[q] >= 0.0)) return ORA_EINVAL;
    const double* Mq = mop + moff[q];
    for (int a = 0; a < L; ++a)
      for (int b = 0; b < L; ++b)
        if (Mq[a * L + b] != Mq[b * L + a]) return ORA_EINVAL;
  }
  int base = s->nem;
  for (int q = 0; q < n; ++q) {
    ora_emitter* e = &s->em[base + q];
    memset(e, 0, sizeof(*e));
    int L = nlev[q];
    e->n = L;
    e->tls = 0;
    memcpy(e->pos, pos + 3 * q, 3 * sizeof(double));
    e->sigma = sigma[q];
    e->gamma = gamma[q];
    memcpy(e->d, dipole + 3 * q, 3 * sizeof(double));
    for (int a = 0; a < L; ++a) e->en[a] = energies[eoff[q] + a];
    for (int a = 0; a < L * L; ++a) {
      e->M[a] = mop[moff[q] + a];
      e->rho[a] = rho0[2 * (moff[q] + a)] + I * rho0[2 * (moff[q] + a) + 1];
    }
    e->gphi = gphi[q];
    int st = build_window(s, e);
    if (st) {
      for (int c = 0; c < 3; ++c) free(e->w[c]);
      for (int r2 = 0; r2 < q; ++r2)
        for (int c = 0; c < 3; ++c) free(s->em[base + r2].w[c]);
      return st;
    }
  }
  s->nem += n;
  return ORA_OK;
}

int ora_num_emitters(const ora_sim* s) { return s->nem; }

int ora_get_rho(const ora_sim* s, int m, double* out) {
  if (m < 0 || m >= s->nem) return ORA_EINVAL;
  const ora_emitter* e = &s->em[m];
  for (int a = 0; a < e->n * e->n; ++a) {
    out[2 * a] = creal(e->rho[a]);
    out[2 * a + 1] = cimag(e->rho[a]);
  }
  return e->n;
}

int ora_set_rho(ora_sim* s, int m, const double* in) {
  if (m < 0 || m >= s->nem) return ORA_EINVAL;
  ora_emitter* e = &s->em[m];
  for (int a = 0; a < e->n * e->n; ++a) e->rho[a] = in[2 * a] + I * in[2 * a + 1];
  return ORA_OK;
}

/* Window weights of emitter m, component c, and their grid indices. */
int ora_get_window(const ora_sim* s, int m, int c, int64_t* idx, double* w, int cap) {
  const ora_emitter* e = &s->em[m];
  int L0 = e->len[c][0], L1 = e->len[c][1], L2 = e->len[c][2];
  if (L0 * L1 * L2 > cap) return -1;
  int q = 0;
  for (int kk = 0; kk < L2; ++kk)
    for (int jj = 0; jj < L1; ++jj)
      for (int ii = 0; ii < L0; ++ii, ++q) {
        idx[q] = (int64_t)window_cell(s, e, c, ii, jj, kk);
        w[q] = e->w[c][q];
      }
  return q;
}

void ora_get_emitter_io(const ora_sim* s, double* Et, double* mudot) {
  for (int m = 0; m < s->nem; ++m)
    for (int c = 0; c < 3; ++c) {
      if (Et) Et[3 * m + c] = s->em[m].Et[c];
      if (mudot) mudot[3 * m + c] = s->em[m].mudot[c];
    }
}

/* ---------------------------------------------------------- sources etc. */

int ora_add_plane_source(ora_sim* s, int axis, int index, int comp, double amp, double omega,
                         double tau, double t0) {
  if (axis < 0 || axis > 2 || comp < 0 || comp > 2 || index < 0 || index >= s->N[axis] ||
      !(tau > 0.0))
    return ORA_EINVAL;
  ora_source* p = (ora_source*)realloc(s->src, (s->nsrc + 1) * sizeof(ora_source));
  if (!p) return ORA_ENOMEM;
  s->src = p;
  ora_source* q = &s->src[s->nsrc++];
  memset(q, 0, sizeof(*q));
  q->kind = 0; q->axis = axis; q->index = index; q->comp = comp;
  q->amp = amp; q->omega = omega; q->tau = tau; q->t0 = t0;
  return ORA_OK;
}

int ora_add_point_source(ora_sim* s, int comp, const int* ijk, double amp, double omega,
                         double tau, double t0) {
  if (comp < 0 || comp > 2 || !(tau > 0.0)) return ORA_EINVAL;
  for (int ax = 0; ax < 3; ++ax)
    if (ijk[ax] < 0 || ijk[ax] >= s->N[ax]) return ORA_EINVAL;
  ora_source* p = (ora_source*)realloc(s->src, (s->nsrc + 1) * sizeof(ora_source));
  if (!p) return ORA_ENOMEM;
  s->src = p;
  ora_source* q = &s->src[s->nsrc++];
  memset(q, 0, sizeof(*q));
  q->kind = 1; q->comp = comp;
  memcpy(q->ijk, ijk, 3 * sizeof(int));
  q->amp = amp; q->omega = omega; q->tau = tau; q->t0 = t0;
  return ORA_OK;
}

/* Gaussian-pulse time profile of the plane-wave excitation (App. B,
 * plasmonic heating: a Gaussian pulse with a centre frequency and a width). */
static double pulse(const ora_source* q, double t) {
  double u = t - q->t0;
  return cos(q->omega * u) * exp(-u * u / (2.0 * q->tau * q->tau));
}

int ora_add_probe(ora_sim* s, int comp, const int* ijk) {
  if (s->nprobe >= 64 || comp < 0 || comp > 5) return -1;
  for (int ax = 0; ax < 3; ++ax)
    if (ijk[ax] < 0 || ijk[ax] >= s->N[ax]) return -1;
  int id = s->nprobe++;
  s->probe_comp[id] = comp;
  memcpy(s->probe_ijk[id], ijk, 3 * sizeof(int));
  memset(&s->probe_series[id], 0, sizeof(ora_series));
  return id;
}

int ora_add_flux_plane(ora_sim* s, int axis, int index) {
  if (axis < 0 || axis > 2 || index < 1 || index >= s->N[axis] || s->flux_on) return ORA_EINVAL;
  s->flux_on = 1;
  s->flux_axis = axis;
  s->flux_index = index;
  int u = (axis + 1) % 3, v = (axis + 2) % 3;
  size_t np = (size_t)s->N[u] * s->N[v];
  s->flux_Eu = (double*)calloc(np, sizeof(double));
  s->flux_Ev = (double*)calloc(np, sizeof(double));
  return ORA_OK;
}

void ora_record_populations(ora_sim* s, int every) { s->pop_every = every; }
int ora_record_energy(ora_sim* s, int on) {
  if (on && !s->Hprev[0])
    for (int c = 0; c < 3; ++c) {
      s->Hprev[c] = (double*)calloc(s->ncell, sizeof(double));
      if (!s->Hprev[c]) return ORA_ENOMEM;
    }
  s->energy_on = on;
  return ORA_OK;
}

int64_t ora_get_series(const ora_sim* s, int which, int id, double* out, int64_t cap) {
  const ora_series* q = NULL;
  if (which == 0) { if (id < 0 || id >= s->nprobe) return -1; q = &s->probe_series[id]; }
  else if (which == 1) q = &s->flux_series;
  else if (which == 2) q = &s->pop_series;
  else if (which == 3) q = &s->energy_series;
  else return -1;
  if (out) {
    int64_t n = q->len < cap ? q->len : cap;
    memcpy(out, q->v, (size_t)n * sizeof(double));
  }
  return q->len;
}

double ora_flux_total(const ora_sim* s) { return s->flux_total; }

/* ------------------------------------------------------------ the fields */

/* H^{n+1/2} = H^{n-1/2} - dt curl E^n  (eq. Maxwell, second line, B = H). */
static void update_H(ora_sim* s) {
  const int nx = s->N[0], ny = s->N[1], nz = s->N[2];
  const double dt = s->dt, idx = 1.0 / s->dx;
  double *Ex = s->E[0], *Ey = s->E[1], *Ez = s->E[2];
  double *Hx = s->H[0], *Hy = s->H[1], *Hz = s->H[2];
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        size_t id = IDX(s, i, j, k);
        double dEz_dy = (fetch(s, Ez, i, j + 1, k) - Ez[id]) * idx;
        double dEy_dz = (fetch(s, Ey, i, j, k + 1) - Ey[id]) * idx;
        double dEx_dz = (fetch(s, Ex, i, j, k + 1) - Ex[id]) * idx;
        double dEz_dx = (fetch(s, Ez, i + 1, j, k) - Ez[id]) * idx;
        double dEy_dx = (fetch(s, Ey, i + 1, j, k) - Ey[id]) * idx;
        double dEx_dy = (fetch(s, Ex, i, j + 1, k) - Ex[id]) * idx;
        /* H components sit at half-integer positions along their derivative axes */
        double cx = stretched(s, 1, 1, j, dEz_dy, s->psiH[0][1], id) -
                    stretched(s, 2, 1, k, dEy_dz, s->psiH[0][2], id);
        double cy = stretched(s, 2, 1, k, dEx_dz, s->psiH[1][2], id) -
                    stretched(s, 0, 1, i, dEz_dx, s->psiH[1][0], id);
        double cz = stretched(s, 0, 1, i, dEy_dx, s->psiH[2][0], id) -
                    stretched(s, 1, 1, j, dEx_dy, s->psiH[2][1], id);
        Hx[id] -= dt * cx;
        Hy[id] -= dt * cy;
        Hz[id] -= dt * cz;
      }
}

/* E^{n+1} = E^n + (dt/eps_r) (curl H^{n+1/2} - J^{n+1/2})  (eq. Maxwell,
 * first line, D = eps_r E), then the tangential E on metallic walls is 0. */
/* Polarisation of every pole from P^n, P^{n-1} and E^n by central differences
 * of its oscillator equation (the standard auxiliary-equation form):
 *   (P^{n+1} - 2 P^n + P^{n-1}) / dt^2 + gamma (P^{n+1} - P^{n-1}) / (2 dt)
 *     + kappa w0^2 P^n = sigma w0^2 E^n.
 * Writes P^{n+1} into out[k][c]. */
static void poles_advance(const ora_sim* s, double* out[8][3]) {
  const double dt = s->dt;
  for (int k = 0; k < s->npole; ++k) {
    const ora_pole* p = &s->pole[k];
    const double g = 0.5 * p->gamma * dt, w2 = p->w0 * p->w0;
    const double kappa = p->drude ? 0.0 : 1.0;
    const int bx = p->hi[0] - p->lo[0], by = p->hi[1] - p->lo[1], bz = p->hi[2] - p->lo[2];
    for (int c = 0; c < 3; ++c)
      for (int kk = 0; kk < bz; ++kk)
        for (int j = 0; j < by; ++j)
          for (int i = 0; i < bx; ++i) {
            size_t b = (size_t)i + (size_t)bx * (j + (size_t)by * kk);
            double e = s->E[c][IDX(s, p->lo[0] + i, p->lo[1] + j, p->lo[2] + kk)];
            out[k][c][b] = ((2.0 - kappa * w2 * dt * dt) * p->P[c][b] -
                            (1.0 - g) * p->Pm[c][b] + p->sigma * w2 * dt * dt * e) / (1.0 + g);
          }
  }
}

static void update_E(ora_sim* s) {
  /* D = eps_inf E + sum_k P_k advances by dt (curl H - J): the poles move first,
   * from E^n, and E^{n+1} = E^n + (dt (curl H - J) - sum_k (P_k^{n+1} - P_k^n)) / eps_inf */
  double* Pn[8][3] = {{0}};
  for (int k = 0; k < s->npole; ++k) {
    const ora_pole* p = &s->pole[k];
    size_t nb = (size_t)(p->hi[0] - p->lo[0]) * (p->hi[1] - p->lo[1]) * (p->hi[2] - p->lo[2]);
    for (int c = 0; c < 3; ++c) Pn[k][c] = (double*)malloc(nb * sizeof(double));
  }
  poles_advance(s, Pn);
  const int nx = s->N[0], ny = s->N[1], nz = s->N[2];
  const double dt = s->dt, idx = 1.0 / s->dx;
  double *Ex = s->E[0], *Ey = s->E[1], *Ez = s->E[2];
  double *Hx = s->H[0], *Hy = s->H[1], *Hz = s->H[2];
  double *Jx = s->J[0], *Jy = s->J[1], *Jz = s->J[2];
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        size_t id = IDX(s, i, j, k);
        double dHz_dy = (Hz[id] - fetch(s, Hz, i, j - 1, k)) * idx;
        double dHy_dz = (Hy[id] - fetch(s, Hy, i, j, k - 1)) * idx;
        double dHx_dz = (Hx[id] - fetch(s, Hx, i, j, k - 1)) * idx;
        double dHz_dx = (Hz[id] - fetch(s, Hz, i - 1, j, k)) * idx;
        double dHy_dx = (Hy[id] - fetch(s, Hy, i - 1, j, k)) * idx;
        double dHx_dy = (Hx[id] - fetch(s, Hx, i, j - 1, k)) * idx;
        /* E components sit at integer positions along their derivative axes */
        double cx = stretched(s, 1, 0, j, dHz_dy, s->psiE[0][1], id) -
                    stretched(s, 2, 0, k, dHy_dz, s->psiE[0][2], id);
        double cy = stretched(s, 2, 0, k, dHx_dz, s->psiE[1][2], id) -
                    stretched(s, 0, 0, i, dHz_dx, s->psiE[1][0], id);
        double cz = stretched(s, 0, 0, i, dHy_dx, s->psiE[2][0], id) -
                    stretched(s, 1, 0, j, dHx_dy, s->psiE[2][1], id);
        double ce = dt / s->eps[id];
        Ex[id] += ce * (cx - Jx[id]);
        Ey[id] += ce * (cy - Jy[id]);
        Ez[id] += ce * (cz - Jz[id]);
      }
  for (int k = 0; k < s->npole; ++k) {
    ora_pole* p = &s->pole[k];
    const int bx = p->hi[0] - p->lo[0], by = p->hi[1] - p->lo[1], bz = p->hi[2] - p->lo[2];
    for (int c = 0; c < 3; ++c) {
      for (int kk = 0; kk < bz; ++kk)
        for (int j = 0; j < by; ++j)
          for (int i = 0; i < bx; ++i) {
            size_t b = (size_t)i + (size_t)bx * (j + (size_t)by * kk);
            size_t id = IDX(s, p->lo[0] + i, p->lo[1] + j, p->lo[2] + kk);
            s->E[c][id] -= (Pn[k][c][b] - p->P[c][b]) / s->eps[id];
          }
      free(p->Pm[c]);
      p->Pm[c] = p->P[c];
      p->P[c] = Pn[k][c];
    }
  }
  /* metallic walls (also behind each PML): E tangential to the wall plane
   * at index 0 of that axis is held at zero */
  for (int ax = 0; ax < 3; ++ax) {
    if (s->bc[2 * ax] == ORA_PERIODIC) continue;
    int u = (ax + 1) % 3, v = (ax + 2) % 3;
    for (int c = 0; c < 3; ++c) {
      if (c == ax) continue;
      for (int jv = 0; jv < s->N[v]; ++jv)
        for (int iu = 0; iu < s->N[u]; ++iu) {
          int q[3];
          q[ax] = 0; q[u] = iu; q[v] = jv;
          s->E[c][IDX(s, q[0], q[1], q[2])] = 0.0;
        }
    }
  }
}

/* ------------------------------------------------------------ emitters */

/* E~_m^c = gamma_m sum_p w^c_{m,p} E_c(p)  (eq. E_regu_Emi, discrete). */
static void gather_one(const ora_sim* s, ora_emitter* e) {
  for (int c = 0; c < 3; ++c) {
    int L0 = e->len[c][0], L1 = e->len[c][1], L2 = e->len[c][2];
    double acc = 0.0;
    for (int kk = 0; kk < L2; ++kk)
      for (int jj = 0; jj < L1; ++jj)
        for (int ii = 0; ii < L0; ++ii)
          acc += e->w[c][ii + L0 * (jj + L1 * kk)] * s->E[c][window_cell(s, e, c, ii, jj, kk)];
    e->Et[c] = e->gamma * acc;
  }
}

static void matmul(int n, const cplx* A, const cplx* B, cplx* C) {
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      cplx acc = 0.0;
      for (int q = 0; q < n; ++q) acc += A[a * n + q] * B[q * n + b];
      C[a * n + b] = acc;
    }
}

static void adjoint(int n, const cplx* A, cplx* B) {
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) B[a * n + b] = conj(A[b * n + a]);
}

/* rho <- U rho U^dagger */
static void conjugate_by(int n, const cplx* U, cplx* rho) {
  cplx T[36], Ud[36], R[36];
  matmul(n, U, rho, T);
  adjoint(n, U, Ud);
  matmul(n, T, Ud, R);
  memcpy(rho, R, (size_t)n * n * sizeof(cplx));
}

/* Cyclic Jacobi eigen-decomposition of a real symmetric n x n matrix:
 * A = Q diag(lam) Q^T (columns of Q are eigenvectors). */
void ora_jacobi_eig(int n, const double* Ain, double* lam, double* Q) {
  double A[36];
  memcpy(A, Ain, (size_t)n * n * sizeof(double));
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) Q[a * n + b] = (a == b) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        tot += A[a * n + b] * A[a * n + b];
        if (a != b) off += A[a * n + b] * A[a * n + b];
      }
    if (off <= 1e-34 * tot || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A[p * n + q];
        if (apq == 0.0) continue;
        double app = A[p * n + p], aqq = A[q * n + q];
        /* rotation angle that annihilates A[p][q] */
        double theta = (aqq - app) / (2.0 * apq);
        double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
        for (int r = 0; r < n; ++r) {
          double arp = A[r * n + p], arq = A[r * n + q];
          A[r * n + p] = c * arp - sn * arq;
          A[r * n + q] = sn * arp + c * arq;
        }
        for (int r = 0; r < n; ++r) {
          double apr = A[p * n + r], aqr = A[q * n + r];
          A[p * n + r] = c * apr - sn * aqr;
          A[q * n + r] = sn * apr + c * aqr;
        }
        for (int r = 0; r < n; ++r) {
          double qrp = Q[r * n + p], qrq = Q[r * n + q];
          Q[r * n + p] = c * qrp - sn * qrq;
          Q[r * n + q] = sn * qrp + c * qrq;
        }
      }
  }
  for (int a = 0; a < n; ++a) lam[a] = A[a * n + a];
}

/* Effective Hamiltonian H0 - E~ . mu with mu^c = d^c M (eq. von-Neumann-tls). */
static void effective_h(const ora_emitter* e, double* Heff) {
  double g = e->Et[0] * e->d[0] + e->Et[1] * e->d[1] + e->Et[2] * e->d[2];
  int n = e->n;
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) Heff[a * n + b] = (a == b ? e->en[a] : 0.0) - g * e->M[a * n + b];
}

/* Two-level exact propagator over dt for constant E~:
 * H = (w0/2) I + h.sigma with h = (-g, 0, -w0/2), V = cos(|h|dt) - i sin(|h|dt) h.sigma/|h|. */
static void step_tls(const ora_sim* s, ora_emitter* e) {
  double g = e->Et[0] * e->d[0] + e->Et[1] * e->d[1] + e->Et[2] * e->d[2];
  double w0 = e->en[1] - e->en[0];
  double hx = -g, hz = -0.5 * w0;
  double Om = sqrt(hx * hx + hz * hz);
  double ph = Om * s->dt;
  double cs = cos(ph), sn = (Om > 0.0) ? sin(ph) / Om : s->dt;
  cplx V[4];
  V[0] = cs - I * sn * hz;
  V[1] = -I * sn * hx;
  V[2] = -I * sn * hx;
  V[3] = cs + I * sn * hz;
  conjugate_by(2, V, e->rho);
}

/* Exact pure-dephasing map over tau: coherences decay as exp(-gphi tau). */
static void dephase(ora_emitter* e, double tau) {
  double f = exp(-e->gphi * tau);
  for (int a = 0; a < e->n; ++a)
    for (int b = 0; b < e->n; ++b)
      if (a != b) e->rho[a * e->n + b] *= f;
}

/* Strang splitting: dephasing(dt/2), unitary exp(-i Heff dt), dephasing(dt/2). */
static void step_lindblad(const ora_sim* s, ora_emitter* e) {
  int n = e->n;
  double Heff[36] = {0}, lam[6], Q[36];
  dephase(e, 0.5 * s->dt);
  effective_h(e, Heff);
  ora_jacobi_eig(n, Heff, lam, Q);
  cplx U[36];
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      cplx acc = 0.0;
      for (int q = 0; q < n; ++q) acc += Q[a * n + q] * cexp(-I * lam[q] * s->dt) * Q[b * n + q];
      U[a * n + b] = acc;
    }
  conjugate_by(n, U, e->rho);
  dephase(e, 0.5 * s->dt);
}

/* Full right-hand side: -i[Heff, rho] + sum_k (L rho L^+ - {L^+ L, rho}/2),
 * L_k = sqrt(gphi) |k><k| (standard GKSL dissipator). */
static void rhs(const ora_emitter* e, cplx* out) {
  int n = e->n;
  double Heff[36];
  effective_h(e, Heff);
  cplx Hc[36], A[36], B[36];
  for (int a = 0; a < n * n; ++a) Hc[a] = Heff[a];
  matmul(n, Hc, e->rho, A);
  matmul(n, e->rho, Hc, B);
  for (int a = 0; a < n * n; ++a) out[a] = -I * (A[a] - B[a]);
  for (int k = 0; k < n; ++k) {
    cplx P[36];
    memset(P, 0, sizeof(P));
    P[k * n + k] = 1.0;
    cplx PrP[36], Pr[36], rP[36], T[36];
    matmul(n, P, e->rho, Pr);
    matmul(n, Pr, P, PrP);
    matmul(n, e->rho, P, rP);
    (void)T;
    for (int a = 0; a < n * n; ++a) out[a] += e->gphi * (PrP[a] - 0.5 * (Pr[a] + rP[a]));
  }
}

/* d<mu>/dt = Tr(rho_dot mu) (eq. dipole_derivative); for the TLS its closed
 * form -2 w0 Im(rho01) d. */
static void dipole_rate(ora_emitter* e) {
  if (e->tls) {
    double w0 = e->en[1] - e->en[0];
    double f = -2.0 * w0 * cimag(e->rho[1]);
    for (int c = 0; c < 3; ++c) e->mudot[c] = f * e->d[c];
    return;
  }
  int n = e->n;
  cplx rd[36];
  rhs(e, rd);
  cplx tr = 0.0;
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) tr += rd[a * n + b] * e->M[b * n + a];
  for (int c = 0; c < 3; ++c) e->mudot[c] = creal(tr) * e->d[c];
}

/* Brute-force Tr(rho_dot mu^c) for any emitter (test helper). */
void ora_dipole_rate_trace(const ora_sim* s, int m, const double* Et, double* out) {
  ora_emitter e = s->em[m];
  memcpy(e.Et, Et, 3 * sizeof(double));
  int n = e.n;
  cplx rd[36];
  rhs(&e, rd);
  cplx tr = 0.0;
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) tr += rd[a * n + b] * e.M[b * n + a];
  for (int c = 0; c < 3; ++c) out[c] = creal(tr) * e.d[c];
}

static void emitter_advance(const ora_sim* s, ora_emitter* e) {
  if (e->tls) step_tls(s, e);
  else step_lindblad(s, e);
  dipole_rate(e);
}

/* Expectation value of the dipole operator, <mu^c> = d^c Tr(rho M). */
static void dipole_expect(const ora_emitter* e, double out[3]) {
  int n = e->n;
  double tr = 0.0;
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) tr += creal(e->rho[a * n + b]) * e->M[b * n + a];
  for (int c = 0; c < 3; ++c) out[c] = tr * e->d[c];
}

/* Single-mode cavity (Sec. II.A.2: eqs. H_F_normalmode, eom_cavmd,
 * varepsilon_cavmd, dklambda_def, E_normalmode in the single-mode limit): one
 * photonic mode of frequency w, polarised along x and along y, with mode function
 * e_l / sqrt(V); with eps0 = 1 the coupling is eps = w / sqrt(V).  Every emitter
 * feels the same field E~ = -sum_l (eps q_l + d_l / V) e_l and the mode obeys
 * q_l'' = -w^2 q_l - eps d_l, where d_l = sum_m <mu_l^(m)> is the total dipole
 * (eq. dklambda_def with f = e_l / sqrt(V)).  Discretised as the grid scheme is:
 * q at integer steps, p = q' at half steps (leapfrog), emitters at half steps.
 * The total dipole at the integer time t_n is formed from the expectation values
 * of the latest states, rho^{n-1/2}, carried half a step forward by their own
 * rate (eq. dipole_derivative):
 *   d^n = sum_m [ <mu^(m)>(rho_m^{n-1/2}) + (dt/2) mu_dot_m(rho_m^{n-1/2}) ],
 * second-order accurate like the rest of the scheme (a bare <mu> at t_{n-1/2}
 * would lag by half a step).  mu_dot is a function of the state alone (the field
 * term of Tr(rho_dot mu) vanishes because mu commutes with itself), so d^0 comes
 * from the initial states.  Step n -> n+1:
 *   E~^n from q^n and d^n; rho^{n-1/2} -> rho^{n+1/2}, mu_dot^{n+1/2};
 *   p^{n+1/2} = p^{n-1/2} - dt (w^2 q^n + eps d^n);  q^{n+1} = q^n + dt p^{n+1/2};
 *   d^{n+1} from the new states (emitters summed in index order).
 * The grid is left alone.  Call after the emitters are added and before the
 * first step. */
static void cavity_dipole(ora_sim* s, double out[2]) {
  out[0] = out[1] = 0.0;
  for (int m = 0; m < s->nem; ++m) {
    double mu[3];
    dipole_expect(&s->em[m], mu);
    out[0] += mu[0] + 0.5 * s->dt * s->em[m].mudot[0];
    out[1] += mu[1] + 0.5 * s->dt * s->em[m].mudot[1];
  }
}

int ora_set_cavity(ora_sim* s, double w, double V, const double q0[2], const double p0[2]) {
  if (!(w > 0.0) || !(V > 0.0) || s->step != 0 || s->npole > 0) return -1;
  s->cav_on = 1;
  s->cav_w = w;
  s->cav_V = V;
  s->cav_eps = w / sqrt(V);
  /* the rates of the initial states (no field has acted yet) */
  for (int m = 0; m < s->nem; ++m) dipole_rate(&s->em[m]);
  cavity_dipole(s, s->cav_d);
  for (int l = 0; l < 2; ++l) {
    s->cav_q[l] = q0[l];
    s->cav_p[l] = p0[l];
  }
  return 0;
}

/* q_x, q_y, p_x, p_y, d_x, d_y at the current step (p at the half step before). */
void ora_get_cavity(const ora_sim* s, double out[6]) {
  for (int l = 0; l < 2; ++l) {
    out[l] = s->cav_q[l];
    out[2 + l] = s->cav_p[l];
    out[4 + l] = s->cav_d[l];
  }
}

/* A Lorentz (drude = 0) or Drude (drude = 1) pole over the half-open box
 * (x0, y0, z0, x1, y1, z1), P = 0 initially.  The box keeps clear of the CPML
 * layers and of the index-0 wall plane of every non-periodic axis.  eps of the
 * box cells is taken as eps_infinity.  Before the first step; at most 8. */
int ora_add_susceptibility(ora_sim* s, const int box[6], double w0, double gamma, double sigma,
                           int drude) {
  if (s->step != 0 || s->npole >= 8 || s->cav_on) return -1;
  if (!(w0 > 0.0) || !(gamma >= 0.0) || !isfinite(sigma) || !isfinite(gamma)) return -1;
  ora_pole* p = &s->pole[s->npole];
  for (int a = 0; a < 3; ++a) {
    int lo = box[a], hi = box[3 + a];
    int lmin = 0, hmax = s->N[a];
    if (s->bc[2 * a] != ORA_PERIODIC) {
      lmin = s->npml[2 * a] > 1 ? s->npml[2 * a] : 1;
      hmax = s->N[a] - s->npml[2 * a + 1];
    }
    if (lo < lmin || hi > hmax || lo >= hi) return -1;
    p->lo[a] = lo;
    p->hi[a] = hi;
  }
  p->w0 = w0;
  p->gamma = gamma;
  p->sigma = sigma;
  p->drude = drude ? 1 : 0;
  size_t nb = (size_t)(p->hi[0] - p->lo[0]) * (p->hi[1] - p->lo[1]) * (p->hi[2] - p->lo[2]);
  for (int c = 0; c < 3; ++c) {
    p->P[c] = (double*)calloc(nb, sizeof(double));
    p->Pm[c] = (double*)calloc(nb, sizeof(double));
  }
  s->npole++;
  return 0;
}

static void cavity_step(ora_sim* s) {
  const double dt = s->dt, w2 = s->cav_w * s->cav_w, eps = s->cav_eps;
  double Et[3] = {-(eps * s->cav_q[0] + s->cav_d[0] / s->cav_V),
                  -(eps * s->cav_q[1] + s->cav_d[1] / s->cav_V), 0.0};
#pragma omp parallel for schedule(static)
  for (int m = 0; m < s->nem; ++m) {
    memcpy(s->em[m].Et, Et, 3 * sizeof(double));
    emitter_advance(s, &s->em[m]);
  }
  double dnew[2];
  cavity_dipole(s, dnew);
  for (int l = 0; l < 2; ++l) {
    s->cav_p[l] -= dt * (w2 * s->cav_q[l] + eps * s->cav_d[l]);
    s->cav_q[l] += dt * s->cav_p[l];
    s->cav_d[l] = dnew[l];
  }
  if (s->pop_every > 0 && s->step % s->pop_every == 0)
    for (int m = 0; m < s->nem; ++m)
      for (int k = 1; k < s->em[m].n; ++k)
        series_push(&s->pop_series, creal(s->em[m].rho[k * s->em[m].n + k]));
  s->step++;
}

/* Advance every emitter by one step under a prescribed field E~ (M x 3),
 * without any grid: the classical-path mode of eq. E_analytical. */
void ora_emitters_step_prescribed(ora_sim* s, const double* Et) {
#pragma omp parallel for schedule(static)
  for (int m = 0; m < s->nem; ++m) {
    memcpy(s->em[m].Et, Et + 3 * m, 3 * sizeof(double));
    emitter_advance(s, &s->em[m]);
  }
}

/* Classical-path step under a travelling pulse (eq. E_analytical, propagation along
 * +z at c = 1): emitter m at height z_m sees, over the step centred at time t,
 * E~_m = gamma_m amp f(t - (z_m - z0)) pol with the Gaussian pulse of App. B,
 * f(u) = cos(omega (u - t0)) exp(-(u - t0)^2 / (2 tau^2)). */
void ora_emitters_step_wave(ora_sim* s, const double* pol, double amp, double omega, double tau,
                            double t0, double z0, double t) {
#pragma omp parallel for schedule(static)
  for (int m = 0; m < s->nem; ++m) {
    ora_emitter* e = &s->em[m];
    double u = t - (e->pos[2] - z0) - t0;
    double f = amp * cos(omega * u) * exp(-u * u / (2.0 * tau * tau));
    for (int c = 0; c < 3; ++c) e->Et[c] = e->gamma * f * pol[c];
    emitter_advance(s, e);
  }
}

/* Gather of the current E into E~ (M x 3). */
void ora_gather(ora_sim* s, double* Et) {
#pragma omp parallel for schedule(static)
  for (int m = 0; m < s->nem; ++m) gather_one(s, &s->em[m]);
  if (Et)
    for (int m = 0; m < s->nem; ++m)
      for (int c = 0; c < 3; ++c) Et[3 * m + c] = s->em[m].Et[c];
}

/* J_c(p) = sum_m gamma_m mu_dot_m^c w^c_{m,p} / dx^3 (eqs. J_mol and
 * Polarization_mol with the kernel's unit integral); emitters in index order. */
static void scatter_into(const ora_sim* s, const double* mudot, double* const J[3]) {
  double iv = 1.0 / (s->dx * s->dx * s->dx);
  for (int m = 0; m < s->nem; ++m) {
    const ora_emitter* e = &s->em[m];
    for (int c = 0; c < 3; ++c) {
      double amp = e->gamma * mudot[3 * m + c] * iv;
      int L0 = e->len[c][0], L1 = e->len[c][1], L2 = e->len[c][2];
      for (int kk = 0; kk < L2; ++kk)
        for (int jj = 0; jj < L1; ++jj)
          for (int ii = 0; ii < L0; ++ii)
            J[c][window_cell(s, e, c, ii, jj, kk)] += amp * e->w[c][ii + L0 * (jj + L1 * kk)];
    }
  }
}

/* Scatter of a given mu_dot (M x 3) into fresh current arrays (test helper). */
void ora_scatter(const ora_sim* s, const double* mudot, double* Jx, double* Jy, double* Jz) {
  memset(Jx, 0, s->ncell * sizeof(double));
  memset(Jy, 0, s->ncell * sizeof(double));
  memset(Jz, 0, s->ncell * sizeof(double));
  double* J[3] = {Jx, Jy, Jz};
  scatter_into(s, mudot, J);
}

/* Soft source currents at t = (n + 1/2) dt. */
static void add_sources(ora_sim* s, double t) {
  for (int q = 0; q < s->nsrc; ++q) {
    const ora_source* src = &s->src[q];
    double sv = src->amp * pulse(src, t);
    if (src->kind == 1) {
      s->J[src->comp][IDX(s, src->ijk[0], src->ijk[1], src->ijk[2])] +=
          sv / (s->dx * s->dx * s->dx);
      continue;
    }
    /* current sheet of surface density amp*s(t) on plane `index` of `axis` */
    for (int k = 0; k < s->N[2]; ++k)
      for (int j = 0; j < s->N[1]; ++j)
        for (int i = 0; i < s->N[0]; ++i) {
          int q3[3] = {i, j, k};
          if (q3[src->axis] != src->index) continue;
          s->J[src->comp][IDX(s, i, j, k)] += sv / s->dx;
        }
  }
}

static void flux_save_plane(ora_sim* s) {
  int a = s->flux_axis, u = (a + 1) % 3, v = (a + 2) % 3;
  for (int jv = 0; jv < s->N[v]; ++jv)
    for (int iu = 0; iu < s->N[u]; ++iu) {
      int q[3];
      q[a] = s->flux_index; q[u] = iu; q[v] = jv;
      size_t id = IDX(s, q[0], q[1], q[2]);
      s->flux_Eu[iu + (size_t)s->N[u] * jv] = s->E[u][id];
      s->flux_Ev[iu + (size_t)s->N[u] * jv] = s->E[v][id];
    }
}

/* F^{n+1/2} = sum over the plane of (E_u H_v - E_v H_u) dx^2 with E averaged
 * over n and n+1 and H averaged over the two half-cells across the plane. */
static double flux_eval(const ora_sim* s) {
  int a = s->flux_axis, u = (a + 1) % 3, v = (a + 2) % 3;
  double F = 0.0;
  for (int jv = 0; jv < s->N[v]; ++jv)
    for (int iu = 0; iu < s->N[u]; ++iu) {
      int q[3], r[3];
      q[a] = s->flux_index; q[u] = iu; q[v] = jv;
      r[a] = s->flux_index - 1; r[u] = iu; r[v] = jv;
      size_t id = IDX(s, q[0], q[1], q[2]), jd = IDX(s, r[0], r[1], r[2]);
      size_t pp = iu + (size_t)s->N[u] * jv;
      double Eu = 0.5 * (s->flux_Eu[pp] + s->E[u][id]);
      double Ev = 0.5 * (s->flux_Ev[pp] + s->E[v][id]);
      double Hv = 0.5 * (s->H[v][id] + s->H[v][jd]);
      double Hu = 0.5 * (s->H[u][id] + s->H[u][jd]);
      F += Eu * Hv - Ev * Hu;
    }
  return F * s->dx * s->dx;
}

/* W^n = 1/2 sum eps |E^n|^2 + 1/2 sum H^{n+1/2} . H^{n-1/2}  (times dx^3). */
static double energy(const ora_sim* s) {
  double w = 0.0;
  for (size_t q = 0; q < s->ncell; ++q) {
    double e2 = s->E[0][q] * s->E[0][q] + s->E[1][q] * s->E[1][q] + s->E[2][q] * s->E[2][q];
    double hh = s->H[0][q] * s->Hprev[0][q] + s->H[1][q] * s->Hprev[1][q] +
                s->H[2][q] * s->Hprev[2][q];
    w += 0.5 * s->eps[q] * e2 + 0.5 * hh;
  }
  return w * s->dx * s->dx * s->dx;
}

/* One full coupled step n -> n+1. */
static void step_once(ora_sim* s) {
  double t_half = ((double)s->step + 0.5) * s->dt;
  if (s->energy_on)
    for (int c = 0; c < 3; ++c) memcpy(s->Hprev[c], s->H[c], s->ncell * sizeof(double));
  /* 1. H^{n+1/2} from E^n */
  update_H(s);
  if (s->energy_on) series_push(&s->energy_series, energy(s));
  /* 2-4. field -> emitters -> dipole rates (E~^n, rho^{n+1/2}, mu_dot^{n+1/2}) */
#pragma omp parallel for schedule(static)
  for (int m = 0; m < s->nem; ++m) {
    gather_one(s, &s->em[m]);
    emitter_advance(s, &s->em[m]);
  }
  /* 5. molecular plus source current J^{n+1/2} */
  for (int c = 0; c < 3; ++c) memset(s->J[c], 0, s->ncell * sizeof(double));
  if (s->nem) {
    double* md = (double*)malloc((size_t)s->nem * 3 * sizeof(double));
    for (int m = 0; m < s->nem; ++m)
      for (int c = 0; c < 3; ++c) md[3 * m + c] = s->em[m].mudot[c];
    scatter_into(s, md, s->J);
    free(md);
  }
  add_sources(s, t_half);
  if (s->flux_on) flux_save_plane(s);
  /* 6. E^{n+1} */
  update_E(s);
  /* 7. detectors */
  for (int p = 0; p < s->nprobe; ++p) {
    int c = s->probe_comp[p];
    const double* a = c < 3 ? s->E[c] : s->H[c - 3];
    series_push(&s->probe_series[p],
                a[IDX(s, s->probe_ijk[p][0], s->probe_ijk[p][1], s->probe_ijk[p][2])]);
  }
  if (s->flux_on) {
    double F = flux_eval(s);
    series_push(&s->flux_series, F);
    s->flux_total += s->dt * F;
  }
  if (s->pop_every > 0 && s->step % s->pop_every == 0)
    for (int m = 0; m < s->nem; ++m)
      for (int k = 1; k < s->em[m].n; ++k)
        series_push(&s->pop_series, creal(s->em[m].rho[k * s->em[m].n + k]));
  s->step++;
}

void ora_step(ora_sim* s, int64_t nsteps) {
  for (int64_t q = 0; q < nsteps; ++q) {
    if (s->cav_on) cavity_step(s);
    else step_once(s);
  }
}

int ora_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void ora_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ================================================================ adjoint
 *
 * Reverse-mode discrete adjoint of the coupled step as the oracle executes it
 * (two-level emitters only), for the objectives
 *   kind 0: J = dt sum_n F^{n+1/2}        (time-integrated flux through the flux plane)
 *   kind 1: J = sum_m w_m rho11_m          (populations after the last step)
 * and its gradients with respect to eps_r of every cell of a box and to each
 * emitter's dipole vector d_m.  The forward pass stores every E^n, H^{n+1/2},
 * emitter state rho^{n-1/2} and E~^n (the oracle is for small grids), then the
 * steps are undone in reverse.  Each linear update y = A x is transposed
 * operation by operation: every contribution A_ij x_j of the forward pass is
 * scattered back as xbar_j += A_ij ybar_i.  The state of the sim is restored
 * afterwards. */

/* index of the cell one step along axis a from (i,j,k) (delta = +1 or -1), with
 * periodic wrap, or -1 when it lies beyond a non-periodic face */
static long long nb_cell(const ora_sim* s, int i, int j, int k, int a, int delta) {
  int q[3] = {i, j, k};
  q[a] += delta;
  if (q[a] < 0 || q[a] >= s->N[a]) {
    if (s->bc[2 * a] != ORA_PERIODIC) return -1;
    q[a] = (q[a] + s->N[a]) % s->N[a];
  }
  return (long long)IDX(s, q[0], q[1], q[2]);
}

/* curl terms of component c: axis, sign and the other field's component */
static const int CURL_AX[3][2] = {{1, 2}, {2, 0}, {0, 1}};
static const int CURL_SG[3][2] = {{1, -1}, {1, -1}, {1, -1}};
static const int CURL_OT[3][2] = {{2, 1}, {0, 2}, {1, 0}};

/* adjoint of the stretched derivative: w is the adjoint of the stretched value,
 * *pb the adjoint of psi after the update (replaced by the adjoint before it);
 * returns the adjoint of the plain derivative */
static inline double stretched_bar(const ora_sim* s, int ax, int half, int pos, double w,
                                   double* pb) {
  if (!s->tin[ax][half][pos]) return w;
  double b = s->tb[ax][half][pos], c = s->tc[ax][half][pos], kinv = s->tk[ax][half][pos];
  double dbar = (kinv + c) * w + c * (*pb);
  *pb = b * (w + *pb);
  return dbar;
}

static int is_wall_E(const ora_sim* s, int c, int i, int j, int k) {
  int q[3] = {i, j, k};
  for (int ax = 0; ax < 3; ++ax)
    if (ax != c && s->bc[2 * ax] != ORA_PERIODIC && q[ax] == 0) return 1;
  return 0;
}

/* Transposed E update: Eb is the adjoint of E^{n+1} (replaced by that of E^n,
 * through the identity part), Hb gains the curl part, psiEb is updated.
 * Returns nothing; the adjoint of the current J is -(dt/eps) Eb_masked, which
 * the caller forms from ub (the wall-masked Eb, filled here). */
static void adjoint_update_E(const ora_sim* s, double* Eb[3], double* Hb[3], double* psiEb[3][3],
                             double* ub[3]) {
  const double dt = s->dt, idx = 1.0 / s->dx;
  for (int k = 0; k < s->N[2]; ++k)
    for (int j = 0; j < s->N[1]; ++j)
      for (int i = 0; i < s->N[0]; ++i) {
        size_t id = IDX(s, i, j, k);
        int pos[3] = {i, j, k};
        for (int c = 0; c < 3; ++c) {
          double u = is_wall_E(s, c, i, j, k) ? 0.0 : Eb[c][id];
          ub[c][id] = u;
          Eb[c][id] = u; /* E^{n+1} = E^n + ... off the walls */
          for (int t = 0; t < 2; ++t) {
            int a = CURL_AX[c][t], h = CURL_OT[c][t];
            double w = CURL_SG[c][t] * dt / s->eps[id] * u;
            double dummy = 0.0;
            double* pb = psiEb[c][a] ? &psiEb[c][a][id] : &dummy;
            double dbar = stretched_bar(s, a, 0, pos[a], w, pb) * idx;
            /* d = (H_h(cell) - H_h(cell - e_a)) / dx */
            Hb[h][id] += dbar;
            long long m = nb_cell(s, i, j, k, a, -1);
            if (m >= 0) Hb[h][m] -= dbar;
          }
        }
      }
}

/* Transposed H update: Hb is the adjoint of H^{n+1/2} (the identity part keeps
 * it as that of H^{n-1/2}), Eb gains the curl part, psiHb is updated. */
static void adjoint_update_H(const ora_sim* s, double* Eb[3], double* Hb[3], double* psiHb[3][3]) {
  const double dt = s->dt, idx = 1.0 / s->dx;
  for (int k = 0; k < s->N[2]; ++k)
    for (int j = 0; j < s->N[1]; ++j)
      for (int i = 0; i < s->N[0]; ++i) {
        size_t id = IDX(s, i, j, k);
        int pos[3] = {i, j, k};
        for (int h = 0; h < 3; ++h) {
          for (int t = 0; t < 2; ++t) {
            int a = CURL_AX[h][t], e = CURL_OT[h][t];
            double w = -CURL_SG[h][t] * dt * Hb[h][id];
            double dummy = 0.0;
            double* pb = psiHb[h][a] ? &psiHb[h][a][id] : &dummy;
            double dbar = stretched_bar(s, a, 1, pos[a], w, pb) * idx;
            /* d = (E_e(cell + e_a) - E_e(cell)) / dx */
            long long m = nb_cell(s, i, j, k, a, +1);
            if (m >= 0) Eb[e][m] += dbar;
            Eb[e][id] -= dbar;
          }
        }
      }
}

/* Two-level state s = (rho11, Re rho01, Im rho01) after one exact step under
 * field g, by V rho V^+ as in step_tls. */
static void tls_map(double w0, double dt, double g, const double in[3], double out[3]) {
  double hx = -g, hz = -0.5 * w0;
  double Om = sqrt(hx * hx + hz * hz);
  double cs = cos(Om * dt), sn = (Om > 0.0) ? sin(Om * dt) / Om : dt;
  cplx V[4] = {cs - I * sn * hz, -I * sn * hx, -I * sn * hx, cs + I * sn * hz};
  cplx r[4] = {1.0 - in[0], in[1] + I * in[2], in[1] - I * in[2], in[0]};
  conjugate_by(2, V, r);
  out[0] = creal(r[3]);
  out[1] = creal(r[1]);
  out[2] = cimag(r[1]);
}

/* d(out)/dg of tls_map, from dV/dg: d(V r V^+) = dV r V^+ + V r dV^+. */
static void tls_map_dg(double w0, double dt, double g, const double in[3], double dout[3]) {
  double hx = -g, hz = -0.5 * w0;
  double Om = sqrt(hx * hx + hz * hz);
  double cs = cos(Om * dt), sn_raw = sin(Om * dt);
  double sn = (Om > 0.0) ? sn_raw / Om : dt;
  /* dOm/dg = g / Om; d(sin(Om dt)/Om)/dOm = dt cos/Om - sin/Om^2 */
  double dOm = (Om > 0.0) ? g / Om : 0.0;
  double dcs = -dt * sn_raw * dOm;
  double dsn = (Om > 0.0) ? (dt * cs / Om - sn_raw / (Om * Om)) * dOm : 0.0;
  /* V = cs I - i sn (hx sigma_x + hz sigma_z), dhx/dg = -1 */
  cplx V[4] = {cs - I * sn * hz, -I * sn * hx, -I * sn * hx, cs + I * sn * hz};
  cplx dV[4] = {dcs - I * dsn * hz, -I * (dsn * hx - sn), -I * (dsn * hx - sn), dcs + I * dsn * hz};
  cplx r[4] = {1.0 - in[0], in[1] + I * in[2], in[1] - I * in[2], in[0]};
  cplx Vd[4], dVd[4], T1[4], A[4], B[4];
  adjoint(2, V, Vd);
  adjoint(2, dV, dVd);
  matmul(2, dV, r, T1);
  matmul(2, T1, Vd, A);
  matmul(2, V, r, T1);
  matmul(2, T1, dVd, B);
  dout[0] = creal(A[3] + B[3]);
  dout[1] = creal(A[1] + B[1]);
  dout[2] = cimag(A[1] + B[1]);
}

int ora_adjoint(ora_sim* s, int kind, const double* weights, int64_t T, const int* box,
                double* grad_eps, double* grad_dip, double* value) {
  if (T <= 0 || s->npole > 0) return ORA_EINVAL;
  if (kind == 0 && !s->flux_on) return ORA_EINVAL;
  if (kind == 1 && !weights) return ORA_EINVAL;
  for (int m = 0; m < s->nem; ++m)
    if (!s->em[m].tls) return ORA_EINVAL;
  for (int a = 0; a < 3; ++a)
    if (box[a] < 0 || box[3 + a] > s->N[a] || box[a] >= box[3 + a]) return ORA_EINVAL;
  const size_t nc = s->ncell, M = (size_t)s->nem;
  /* snapshot of the evolving state, restored at the end */
  double *E0[3], *H0[3], *pE0[3][3] = {{0}}, *pH0[3][3] = {{0}};
  for (int c = 0; c < 3; ++c) {
    E0[c] = (double*)malloc(nc * sizeof(double));
    H0[c] = (double*)malloc(nc * sizeof(double));
    memcpy(E0[c], s->E[c], nc * sizeof(double));
    memcpy(H0[c], s->H[c], nc * sizeof(double));
    for (int a = 0; a < 3; ++a) {
      if (s->psiE[c][a]) {
        pE0[c][a] = (double*)malloc(nc * sizeof(double));
        memcpy(pE0[c][a], s->psiE[c][a], nc * sizeof(double));
      }
      if (s->psiH[c][a]) {
        pH0[c][a] = (double*)malloc(nc * sizeof(double));
        memcpy(pH0[c][a], s->psiH[c][a], nc * sizeof(double));
      }
    }
  }
  ora_emitter* em0 = (ora_emitter*)malloc((M ? M : 1) * sizeof(ora_emitter));
  if (M) memcpy(em0, s->em, M * sizeof(ora_emitter));
  int64_t step0 = s->step;
  double ftot0 = s->flux_total;
  int64_t len_probe[64], len_flux = s->flux_series.len, len_pop = s->pop_series.len,
          len_en = s->energy_series.len;
  for (int p = 0; p < s->nprobe; ++p) len_probe[p] = s->probe_series[p].len;

  /* forward pass with the tape */
  double* tE = (double*)malloc((size_t)(T + 1) * 3 * nc * sizeof(double));
  double* tH = (double*)malloc((size_t)T * 3 * nc * sizeof(double));
  double* tS = (double*)malloc((size_t)T * (M ? M : 1) * 3 * sizeof(double));
  double* tG = (double*)malloc((size_t)T * (M ? M : 1) * 3 * sizeof(double));
  if (!tE || !tH || !tS || !tG) { free(tE); free(tH); free(tS); free(tG); return ORA_ENOMEM; }
  for (int c = 0; c < 3; ++c) memcpy(tE + (size_t)c * nc, s->E[c], nc * sizeof(double));
  for (int64_t n = 0; n < T; ++n) {
    for (size_t m = 0; m < M; ++m) {
      double* st = tS + ((size_t)n * M + m) * 3;
      st[0] = creal(s->em[m].rho[3]);
      st[1] = creal(s->em[m].rho[1]);
      st[2] = cimag(s->em[m].rho[1]);
    }
    step_once(s);
    for (int c = 0; c < 3; ++c) {
      memcpy(tE + ((size_t)(n + 1) * 3 + c) * nc, s->E[c], nc * sizeof(double));
      memcpy(tH + ((size_t)n * 3 + c) * nc, s->H[c], nc * sizeof(double));
    }
    for (size_t m = 0; m < M; ++m)
      for (int c = 0; c < 3; ++c) tG[((size_t)n * M + m) * 3 + c] = s->em[m].Et[c];
  }
  double J = 0.0;
  if (kind == 0) J = s->flux_total - ftot0;
  else
    for (size_t m = 0; m < M; ++m) J += weights[m] * creal(s->em[m].rho[3]);
  *value = J;

  /* reverse pass */
  double *Eb[3], *Hb[3], *ub[3], *psiEb[3][3] = {{0}}, *psiHb[3][3] = {{0}};
  for (int c = 0; c < 3; ++c) {
    Eb[c] = (double*)calloc(nc, sizeof(double));
    Hb[c] = (double*)calloc(nc, sizeof(double));
    ub[c] = (double*)calloc(nc, sizeof(double));
    for (int a = 0; a < 3; ++a) {
      if (s->psiE[c][a]) psiEb[c][a] = (double*)calloc(nc, sizeof(double));
      if (s->psiH[c][a]) psiHb[c][a] = (double*)calloc(nc, sizeof(double));
    }
  }
  double* geps = (double*)calloc(nc, sizeof(double));
  double* sb = (double*)calloc((M ? M : 1) * 3, sizeof(double));
  double* gd = (double*)calloc((M ? M : 1) * 3, sizeof(double));
  if (kind == 1)
    for (size_t m = 0; m < M; ++m) sb[3 * m] = weights[m];
  const int fa = s->flux_axis, fu = (fa + 1) % 3, fv = (fa + 2) % 3;
  const double fc = 0.5 * s->dt * s->dx * s->dx;
  const double iv = 1.0 / (s->dx * s->dx * s->dx);
  for (int64_t n = T - 1; n >= 0; --n) {
    const double* En = tE + (size_t)n * 3 * nc;
    const double* En1 = tE + (size_t)(n + 1) * 3 * nc;
    const double* Hh = tH + (size_t)n * 3 * nc;
    /* flux F^{n+1/2}: its E^{n+1} and H^{n+1/2} parts */
    if (kind == 0) {
      for (int jv = 0; jv < s->N[fv]; ++jv)
        for (int iu = 0; iu < s->N[fu]; ++iu) {
          int q[3], r[3];
          q[fa] = s->flux_index; q[fu] = iu; q[fv] = jv;
          r[fa] = s->flux_index - 1; r[fu] = iu; r[fv] = jv;
          size_t id = IDX(s, q[0], q[1], q[2]), jd = IDX(s, r[0], r[1], r[2]);
          double Hv = 0.5 * (Hh[(size_t)fv * nc + id] + Hh[(size_t)fv * nc + jd]);
          double Hu = 0.5 * (Hh[(size_t)fu * nc + id] + Hh[(size_t)fu * nc + jd]);
          double Eu = 0.5 * (En[(size_t)fu * nc + id] + En1[(size_t)fu * nc + id]);
          double Ev = 0.5 * (En[(size_t)fv * nc + id] + En1[(size_t)fv * nc + id]);
          Eb[fu][id] += fc * Hv;
          Eb[fv][id] -= fc * Hu;
          Hb[fv][id] += fc * Eu;
          Hb[fv][jd] += fc * Eu;
          Hb[fu][id] -= fc * Ev;
          Hb[fu][jd] -= fc * Ev;
        }
    }
    /* eps: E^{n+1} - E^n = (dt/eps)(curl H - J), so dE^{n+1}/d eps = -(E^{n+1} - E^n)/eps */
    for (size_t q = 0; q < nc; ++q)
      for (int c = 0; c < 3; ++c)
        geps[q] -= Eb[c][q] * (En1[(size_t)c * nc + q] - En[(size_t)c * nc + q]) / s->eps[q];
    /* E update (fills ub, the wall-masked adjoint of E^{n+1}) */
    adjoint_update_E(s, Eb, Hb, psiEb, ub);
    /* J^{n+1/2} enters as -(dt/eps) J: the adjoint of mu_dot_m^c is
       sum_p (gamma w_p / dx^3) * (-(dt/eps_p) ub_c(p)) */
    double* mdb = (double*)calloc((M ? M : 1) * 3, sizeof(double));
    for (size_t m = 0; m < M; ++m) {
      const ora_emitter* e = &s->em[m];
      for (int c = 0; c < 3; ++c) {
        int L0 = e->len[c][0], L1 = e->len[c][1], L2 = e->len[c][2];
        double acc = 0.0;
        for (int kk = 0; kk < L2; ++kk)
          for (int jj = 0; jj < L1; ++jj)
            for (int ii = 0; ii < L0; ++ii) {
              size_t p = window_cell(s, e, c, ii, jj, kk);
              acc += e->w[c][ii + L0 * (jj + L1 * kk)] * (-s->dt / s->eps[p]) * ub[c][p];
            }
        mdb[3 * m + c] = e->gamma * iv * acc;
      }
    }
    /* H update */
    adjoint_update_H(s, Eb, Hb, psiHb);
    /* emitters: mu_dot = -2 w0 Im(rho01') d, rho' = step(rho, g), g = E~ . d */
    for (size_t m = 0; m < M; ++m) {
      ora_emitter* e = &s->em[m];
      const double* st = tS + ((size_t)n * M + m) * 3;
      const double* Et = tG + ((size_t)n * M + m) * 3;
      double w0 = e->en[1] - e->en[0];
      double g = Et[0] * e->d[0] + Et[1] * e->d[1] + Et[2] * e->d[2];
      double sp[3];
      tls_map(w0, s->dt, g, st, sp);
      double a = -2.0 * w0 * sp[2];
      double abar = 0.0;
      for (int c = 0; c < 3; ++c) {
        gd[3 * m + c] += a * mdb[3 * m + c];
        abar += mdb[3 * m + c] * e->d[c];
      }
      double spb[3] = {sb[3 * m], sb[3 * m + 1], sb[3 * m + 2] - 2.0 * w0 * abar};
      /* the step is affine in the state: columns from basis states */
      double z[3] = {0, 0, 0}, f0[3], col[3][3];
      tls_map(w0, s->dt, g, z, f0);
      for (int q = 0; q < 3; ++q) {
        double eq[3] = {0, 0, 0};
        eq[q] = 1.0;
        double fq[3];
        tls_map(w0, s->dt, g, eq, fq);
        for (int r = 0; r < 3; ++r) col[q][r] = fq[r] - f0[r];
      }
      double dsp[3];
      tls_map_dg(w0, s->dt, g, st, dsp);
      double gbar = spb[0] * dsp[0] + spb[1] * dsp[1] + spb[2] * dsp[2];
      for (int q = 0; q < 3; ++q)
        sb[3 * m + q] = col[q][0] * spb[0] + col[q][1] * spb[1] + col[q][2] * spb[2];
      for (int c = 0; c < 3; ++c) gd[3 * m + c] += gbar * Et[c];
      /* E~ = gamma sum w E^n: scatter gbar d back into Eb */
      for (int c = 0; c < 3; ++c) {
        double amp = e->gamma * gbar * e->d[c];
        int L0 = e->len[c][0], L1 = e->len[c][1], L2 = e->len[c][2];
        for (int kk = 0; kk < L2; ++kk)
          for (int jj = 0; jj < L1; ++jj)
            for (int ii = 0; ii < L0; ++ii)
              Eb[c][window_cell(s, e, c, ii, jj, kk)] += amp * e->w[c][ii + L0 * (jj + L1 * kk)];
      }
    }
    free(mdb);
    /* flux: its E^n part */
    if (kind == 0) {
      for (int jv = 0; jv < s->N[fv]; ++jv)
        for (int iu = 0; iu < s->N[fu]; ++iu) {
          int q[3], r[3];
          q[fa] = s->flux_index; q[fu] = iu; q[fv] = jv;
          r[fa] = s->flux_index - 1; r[fu] = iu; r[fv] = jv;
          size_t id = IDX(s, q[0], q[1], q[2]), jd = IDX(s, r[0], r[1], r[2]);
          double Hv = 0.5 * (Hh[(size_t)fv * nc + id] + Hh[(size_t)fv * nc + jd]);
          double Hu = 0.5 * (Hh[(size_t)fu * nc + id] + Hh[(size_t)fu * nc + jd]);
          Eb[fu][id] += fc * Hv;
          Eb[fv][id] -= fc * Hu;
        }
    }
  }
  /* outputs */
  size_t b = 0;
  for (int k = box[2]; k < box[5]; ++k)
    for (int j = box[1]; j < box[4]; ++j)
      for (int i = box[0]; i < box[3]; ++i) grad_eps[b++] = geps[IDX(s, i, j, k)];
  for (size_t m = 0; m < 3 * M; ++m) grad_dip[m] = gd[m];

  /* restore */
  for (int c = 0; c < 3; ++c) {
    memcpy(s->E[c], E0[c], nc * sizeof(double));
    memcpy(s->H[c], H0[c], nc * sizeof(double));
    free(E0[c]); free(H0[c]); free(Eb[c]); free(Hb[c]); free(ub[c]);
    for (int a = 0; a < 3; ++a) {
      if (pE0[c][a]) { memcpy(s->psiE[c][a], pE0[c][a], nc * sizeof(double)); free(pE0[c][a]); }
      if (pH0[c][a]) { memcpy(s->psiH[c][a], pH0[c][a], nc * sizeof(double)); free(pH0[c][a]); }
      free(psiEb[c][a]); free(psiHb[c][a]);
    }
  }
  for (size_t m = 0; m < M; ++m) {
    /* keep the window arrays (same pointers), restore state */
    memcpy(s->em[m].rho, em0[m].rho, sizeof(em0[m].rho));
    memcpy(s->em[m].Et, em0[m].Et, sizeof(em0[m].Et));
    memcpy(s->em[m].mudot, em0[m].mudot, sizeof(em0[m].mudot));
  }
  free(em0);
  s->step = step0;
  s->flux_total = ftot0;
  s->flux_series.len = len_flux;
  s->pop_series.len = len_pop;
  s->energy_series.len = len_en;
  for (int p = 0; p < s->nprobe; ++p) s->probe_series[p].len = len_probe[p];
  free(tE); free(tH); free(tS); free(tG); free(geps); free(sb); free(gd);
  return ORA_OK;
}

/* ---- the linear Yee/CPML step alone, on a packed state, and its transpose
 * (for the dot-product test).  Packed state: E (3 nc), H (3 nc), then every
 * allocated psiE[c][a], then every allocated psiH[c][a], in (c, a) order. */
int64_t ora_state_len(const ora_sim* s) {
  int64_t n = 6 * (int64_t)s->ncell;
  for (int c = 0; c < 3; ++c)
    for (int a = 0; a < 3; ++a) n += (s->psiE[c][a] ? (int64_t)s->ncell : 0) +
                                     (s->psiH[c][a] ? (int64_t)s->ncell : 0);
  return n;
}

static void pack_state(const ora_sim* s, double* const E[3], double* const H[3],
                       double* const pE[3][3], double* const pH[3][3], double* out, int in) {
  size_t nc = s->ncell, o = 0;
  double* arrs[24];
  int na = 0;
  for (int c = 0; c < 3; ++c) arrs[na++] = E[c];
  for (int c = 0; c < 3; ++c) arrs[na++] = H[c];
  for (int c = 0; c < 3; ++c)
    for (int a = 0; a < 3; ++a)
      if (s->psiE[c][a]) arrs[na++] = pE[c][a];
  for (int c = 0; c < 3; ++c)
    for (int a = 0; a < 3; ++a)
      if (s->psiH[c][a]) arrs[na++] = pH[c][a];
  for (int q = 0; q < na; ++q, o += nc) {
    if (in) memcpy(arrs[q], out + o, nc * sizeof(double));
    else memcpy(out + o, arrs[q], nc * sizeof(double));
  }
}

/* x <- L x: one source-free, emitter-free step (H update, E update) */
void ora_linear_step(ora_sim* s, double* x) {
  pack_state(s, s->E, s->H, s->psiE, s->psiH, x, 1);
  update_H(s);
  for (int c = 0; c < 3; ++c) memset(s->J[c], 0, s->ncell * sizeof(double));
  update_E(s);
  pack_state(s, s->E, s->H, s->psiE, s->psiH, x, 0);
}

/* y <- L^T y */
void ora_linear_step_adjoint(ora_sim* s, double* y) {
  size_t nc = s->ncell;
  double *Eb[3], *Hb[3], *ub[3], *pE[3][3] = {{0}}, *pH[3][3] = {{0}};
  for (int c = 0; c < 3; ++c) {
    Eb[c] = (double*)malloc(nc * sizeof(double));
    Hb[c] = (double*)malloc(nc * sizeof(double));
    ub[c] = (double*)malloc(nc * sizeof(double));
    for (int a = 0; a < 3; ++a) {
      if (s->psiE[c][a]) pE[c][a] = (double*)malloc(nc * sizeof(double));
      if (s->psiH[c][a]) pH[c][a] = (double*)malloc(nc * sizeof(double));
    }
  }
  pack_state(s, Eb, Hb, pE, pH, y, 1);
  adjoint_update_E(s, Eb, Hb, pE, ub);
  adjoint_update_H(s, Eb, Hb, pH);
  pack_state(s, Eb, Hb, pE, pH, y, 0);
  for (int c = 0; c < 3; ++c) {
    free(Eb[c]); free(Hb[c]); free(ub[c]);
    for (int a = 0; a < 3; ++a) { free(pE[c][a]); free(pH[c][a]); }
  }
}

int ora_set_tls_dipole(ora_sim* s, int m, const double* d) {
  if (m < 0 || m >= s->nem) return ORA_EINVAL;
  memcpy(s->em[m].d, d, 3 * sizeof(double));
  if (s->cav_on) {
    /* the mode's total dipole follows the new dipole vector */
    dipole_rate(&s->em[m]);
    cavity_dipole(s, s->cav_d);
  }
  return ORA_OK;
}
