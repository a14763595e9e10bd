"""ctypes front-end of the plain FP64 CPU oracle (``mlk_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Only the tests, the package smoke check and the
benchmark's CPU-baseline leg may import this module; the HIP product path
never does.  It shares no code with that path: the arithmetic lives in
``mlk_oracle.c``; this file only marshals arguments.

Array convention: grid arrays are numpy arrays of shape (nz, ny, nx)
(x fastest), float64.  Boundary kinds: "pec", "periodic", "cpml", listed per
face as (x-, x+, y-, y+, z-, z+).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mlk_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

BC = {"pec": 0, "periodic": 1, "cpml": 2}

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_lp = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def build(verbose: bool = False) -> str:
    """Compile liboracle.so with gcc (portable -O3, OpenMP)."""
    # built beside the library and renamed over it, so a process that has the old
    # library loaded keeps its copy intact
    tmp = f"{_LIB}.{os.getpid()}.tmp"
    cmd = ["gcc", "-O3", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    L = C.CDLL(_LIB)
    L.ora_create.restype = C.c_void_p
    L.ora_create.argtypes = [_ip, C.c_double, C.c_double, _ip, _ip, C.c_double, C.c_double,
                             C.c_double, C.c_double, C.c_double, C.POINTER(C.c_int)]
    L.ora_destroy.argtypes = [C.c_void_p]
    L.ora_dt.restype = C.c_double
    L.ora_dt.argtypes = [C.c_void_p]
    L.ora_step_count.restype = C.c_int64
    L.ora_step_count.argtypes = [C.c_void_p]
    L.ora_set_eps.argtypes = [C.c_void_p, _dp]
    L.ora_set_field.argtypes = [C.c_void_p, C.c_int, _dp]
    L.ora_get_field.argtypes = [C.c_void_p, C.c_int, _dp]
    L.ora_add_tls.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp, _dp, _dp, _dp]
    L.ora_add_multilevel.argtypes = [C.c_void_p, C.c_int, _ip, _lp, _lp, _dp, _dp, _dp, _dp,
                                     _dp, _dp, _dp, _dp]
    L.ora_num_emitters.argtypes = [C.c_void_p]
    L.ora_get_rho.argtypes = [C.c_void_p, C.c_int, _dp]
    L.ora_set_rho.argtypes = [C.c_void_p, C.c_int, _dp]
    L.ora_get_window.argtypes = [C.c_void_p, C.c_int, C.c_int, _lp, _dp, C.c_int]
    L.ora_get_emitter_io.argtypes = [C.c_void_p, _dp, _dp]
    L.ora_add_plane_source.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_double,
                                       C.c_double, C.c_double, C.c_double]
    L.ora_add_point_source.argtypes = [C.c_void_p, C.c_int, _ip, C.c_double, C.c_double,
                                       C.c_double, C.c_double]
    L.ora_add_probe.argtypes = [C.c_void_p, C.c_int, _ip]
    L.ora_add_flux_plane.argtypes = [C.c_void_p, C.c_int, C.c_int]
    L.ora_record_populations.argtypes = [C.c_void_p, C.c_int]
    L.ora_record_energy.argtypes = [C.c_void_p, C.c_int]
    L.ora_get_series.restype = C.c_int64
    L.ora_get_series.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_int64]
    L.ora_flux_total.restype = C.c_double
    L.ora_flux_total.argtypes = [C.c_void_p]
    L.ora_step.argtypes = [C.c_void_p, C.c_int64]
    L.ora_jacobi_eig.argtypes = [C.c_int, _dp, _dp, _dp]
    L.ora_emitters_step_prescribed.argtypes = [C.c_void_p, _dp]
    L.ora_emitters_step_wave.argtypes = [C.c_void_p, _dp, C.c_double, C.c_double, C.c_double,
                                         C.c_double, C.c_double, C.c_double]
    L.ora_set_cavity.argtypes = [C.c_void_p, C.c_double, C.c_double, _dp, _dp]
    L.ora_set_cavity.restype = C.c_int
    L.ora_get_cavity.argtypes = [C.c_void_p, _dp]
    L.ora_add_susceptibility.argtypes = [C.c_void_p, C.POINTER(C.c_int), C.c_double, C.c_double,
                                         C.c_double, C.c_int]
    L.ora_add_susceptibility.restype = C.c_int
    L.ora_gather.argtypes = [C.c_void_p, _dp]
    L.ora_scatter.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
    L.ora_dipole_rate_trace.argtypes = [C.c_void_p, C.c_int, _dp, _dp]
    L.ora_adjoint.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_int64, _ip, _dp, _dp,
                              C.POINTER(C.c_double)]
    L.ora_state_len.restype = C.c_int64
    L.ora_state_len.argtypes = [C.c_void_p]
    L.ora_linear_step.argtypes = [C.c_void_p, _dp]
    L.ora_linear_step_adjoint.argtypes = [C.c_void_p, _dp]
    L.ora_set_tls_dipole.argtypes = [C.c_void_p, C.c_int, _dp]
    L.ora_threads.restype = C.c_int
    L.ora_set_threads.argtypes = [C.c_int]
    _lib = L
    return L


def threads() -> int:
    return lib().ora_threads()


def set_threads(n: int) -> None:
    lib().ora_set_threads(int(n))


def jacobi_eig(A: np.ndarray):
    """Eigen-decomposition of a real symmetric matrix by the oracle's Jacobi routine."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    lam = np.zeros(n)
    Q = np.zeros((n, n))
    lib().ora_jacobi_eig(n, A, lam, Q)
    return lam, Q


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


class Oracle:
    """One FP64 CPU simulation; same problem statement as the GPU library."""

    def __init__(self, shape, dx=1.0, courant=0.5, bc=("pec",) * 6, cpml=(0,) * 6,
                 pml_m=3.0, pml_sigma_scale=0.8, pml_kappa_max=1.0, pml_alpha_max=0.0,
                 window_r=3.0):
        L = lib()
        nx, ny, nz = (int(v) for v in shape)
        self.shape = (nx, ny, nz)
        st = C.c_int(0)
        bcs = np.array([BC[b] if isinstance(b, str) else int(b) for b in bc], dtype=np.int32)
        self._h = L.ora_create(np.array([nx, ny, nz], dtype=np.int32), dx, courant, bcs,
                               np.array(cpml, dtype=np.int32), pml_m, pml_sigma_scale,
                               pml_kappa_max, pml_alpha_max, window_r, C.byref(st))
        if not self._h:
            raise ValueError(f"oracle: invalid grid description (status {st.value})")
        self.nlev = []
        self.dt = L.ora_dt(self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().ora_destroy(h)
            self._h = None

    @property
    def ncell(self):
        nx, ny, nz = self.shape
        return nx * ny * nz

    @property
    def step_count(self):
        return lib().ora_step_count(self._h)

    def _check(self, st, what):
        if st != 0:
            raise ValueError(f"oracle: {what} failed (status {st})")

    def set_eps(self, eps):
        self._check(lib().ora_set_eps(self._h, _f64(eps).ravel()), "set_eps")

    def set_field(self, comp, arr):
        self._check(lib().ora_set_field(self._h, comp, _f64(arr).ravel()), "set_field")

    def get_field(self, comp):
        nx, ny, nz = self.shape
        out = np.zeros(self.ncell)
        self._check(lib().ora_get_field(self._h, comp, out), "get_field")
        return out.reshape(nz, ny, nx)

    def fields(self):
        return [self.get_field(c) for c in range(6)]

    def add_tls(self, pos, sigma, gamma, omega0, dipole, rho0):
        pos = _f64(pos, (-1, 3))
        n = pos.shape[0]
        bc = lambda v: _f64(np.broadcast_to(np.asarray(v, dtype=np.float64), (n,)))
        st = lib().ora_add_tls(self._h, n, pos.ravel(), bc(sigma), bc(gamma), bc(omega0),
                               _f64(dipole, (n, 3)).ravel(), _f64(rho0, (n, 3)).ravel())
        self._check(st, "add_tls")
        self.nlev += [2] * n

    def add_multilevel(self, nlev, energies, mop, dipole, gphi, rho0, pos, sigma, gamma):
        """nlev: (n,) ints; energies: list of (L,) arrays; mop: list of (L,L) real symmetric;
        rho0: list of (L,L) complex; dipole/pos: (n,3); gphi/sigma/gamma: (n,)."""
        n = len(nlev)
        nl = np.asarray(nlev, dtype=np.int32)
        eoff = np.zeros(n, dtype=np.int64)
        moff = np.zeros(n, dtype=np.int64)
        eo = mo = 0
        for q in range(n):
            eoff[q], moff[q] = eo, mo
            eo += nl[q]
            mo += nl[q] * nl[q]
        en = _f64(np.concatenate([np.asarray(e, dtype=np.float64).ravel() for e in energies]))
        mm = _f64(np.concatenate([np.asarray(m, dtype=np.float64).ravel() for m in mop]))
        rr = np.concatenate([np.asarray(r, dtype=np.complex128).ravel() for r in rho0])
        ri = _f64(np.stack([rr.real, rr.imag], axis=1).ravel())
        bc = lambda v: _f64(np.broadcast_to(np.asarray(v, dtype=np.float64), (n,)))
        st = lib().ora_add_multilevel(self._h, n, nl, eoff, moff, en, mm,
                                      _f64(dipole, (n, 3)).ravel(), bc(gphi), ri,
                                      _f64(pos, (n, 3)).ravel(), bc(sigma), bc(gamma))
        self._check(st, "add_multilevel")
        self.nlev += [int(v) for v in nl]

    @property
    def num_emitters(self):
        return lib().ora_num_emitters(self._h)

    def rho(self, m):
        L = self.nlev[m]
        out = np.zeros(2 * L * L)
        lib().ora_get_rho(self._h, m, out)
        return (out[0::2] + 1j * out[1::2]).reshape(L, L)

    def set_rho(self, m, rho):
        rho = np.asarray(rho, dtype=np.complex128).ravel()
        lib().ora_set_rho(self._h, m, _f64(np.stack([rho.real, rho.imag], axis=1).ravel()))

    def tls_state(self):
        """(M,3) array of (rho11, Re rho01, Im rho01)."""
        out = np.zeros((len(self.nlev), 3))
        for m in range(len(self.nlev)):
            r = self.rho(m)
            out[m] = (r[1, 1].real, r[0, 1].real, r[0, 1].imag)
        return out

    def window(self, m, c):
        idx = np.zeros(4096, dtype=np.int64)
        w = np.zeros(4096)
        n = lib().ora_get_window(self._h, m, c, idx, w, 4096)
        return idx[:n].copy(), w[:n].copy()

    def emitter_io(self):
        M = len(self.nlev)
        Et = np.zeros(3 * max(M, 1))
        md = np.zeros(3 * max(M, 1))
        lib().ora_get_emitter_io(self._h, Et, md)
        return Et[:3 * M].reshape(M, 3), md[:3 * M].reshape(M, 3)

    def add_plane_source(self, axis, index, comp, amp, omega, tau, t0):
        self._check(lib().ora_add_plane_source(self._h, axis, index, comp, amp, omega, tau, t0),
                    "add_plane_source")

    def add_point_source(self, comp, ijk, amp, omega, tau, t0):
        self._check(lib().ora_add_point_source(self._h, comp, np.asarray(ijk, dtype=np.int32),
                                               amp, omega, tau, t0), "add_point_source")

    def add_probe(self, comp, ijk):
        pid = lib().ora_add_probe(self._h, comp, np.asarray(ijk, dtype=np.int32))
        if pid < 0:
            raise ValueError("oracle: bad probe")
        return pid

    def add_flux_plane(self, axis, index):
        self._check(lib().ora_add_flux_plane(self._h, axis, index), "add_flux_plane")

    def record_populations(self, every=1):
        lib().ora_record_populations(self._h, int(every))

    def record_energy(self, on=True):
        self._check(lib().ora_record_energy(self._h, int(bool(on))), "record_energy")

    def _series(self, which, sid=0):
        n = lib().ora_get_series(self._h, which, sid, None, 0)
        if n < 0:
            raise ValueError("oracle: bad series id")
        out = np.zeros(max(n, 1))
        lib().ora_get_series(self._h, which, sid, out.ctypes.data_as(C.c_void_p), n)
        return out[:n].copy()

    def probe(self, pid):
        return self._series(0, pid)

    def flux_series(self):
        return self._series(1)

    def flux_total(self):
        return lib().ora_flux_total(self._h)

    # ------------------------------------------------------------ adjoint
    def adjoint(self, objective, nsteps, box, weights=None):
        """Discrete adjoint over the next nsteps steps (two-level emitters only).
        objective: "flux" (dt sum F over the steps) or "population" (sum_m w_m rho11_m at
        the end).  box: ((x0, y0, z0), (x1, y1, z1)) half-open.  Returns (value,
        grad_eps (z, y, x) over the box, grad_dipole (M, 3)); the state is unchanged."""
        (x0, y0, z0), (x1, y1, z1) = box
        b = np.array([x0, y0, z0, x1, y1, z1], dtype=np.int32)
        ge = np.zeros((z1 - z0) * (y1 - y0) * (x1 - x0))
        M = len(self.nlev)
        gd = np.zeros(max(1, 3 * M))
        val = C.c_double()
        kind = {"flux": 0, "population": 1}[objective]
        w = None
        if kind == 1:
            w = np.ascontiguousarray(np.broadcast_to(weights, (M,)), dtype=np.float64)
        st = lib().ora_adjoint(self._h, kind, w.ctypes.data if w is not None else None,
                               int(nsteps), b, ge, gd, C.byref(val))
        if st != 0:
            raise ValueError(f"oracle adjoint refused the request (status {st})")
        return val.value, ge.reshape(z1 - z0, y1 - y0, x1 - x0), gd[:3 * M].reshape(M, 3)

    def state_len(self):
        return lib().ora_state_len(self._h)

    def linear_step(self, x):
        """One source- and emitter-free Yee/CPML step of a packed state (E, H, psi)."""
        x = np.array(x, dtype=np.float64)
        lib().ora_linear_step(self._h, x)
        return x

    def linear_step_adjoint(self, y):
        """The transpose of linear_step."""
        y = np.array(y, dtype=np.float64)
        lib().ora_linear_step_adjoint(self._h, y)
        return y

    def set_tls_dipole(self, m, d):
        d = np.ascontiguousarray(d, dtype=np.float64)
        if lib().ora_set_tls_dipole(self._h, int(m), d) != 0:
            raise ValueError("bad emitter index")

    def populations(self):
        """(nrec, sum_m (nlev_m - 1)) array of Re rho_kk, k >= 1, per recorded step."""
        v = self._series(2)
        per = sum(L - 1 for L in self.nlev)
        return v.reshape(-1, per) if per else v.reshape(0, 0)

    def energy_series(self):
        return self._series(3)

    def step(self, n=1):
        lib().ora_step(self._h, int(n))

    def gather(self):
        M = len(self.nlev)
        out = np.zeros(3 * max(M, 1))
        lib().ora_gather(self._h, out)
        return out[:3 * M].reshape(M, 3)

    def scatter(self, mudot):
        M = len(self.nlev)
        nx, ny, nz = self.shape
        J = [np.zeros(self.ncell) for _ in range(3)]
        lib().ora_scatter(self._h, _f64(mudot, (M, 3)).ravel(), J[0], J[1], J[2])
        return [j.reshape(nz, ny, nx) for j in J]

    def set_cavity(self, omega, volume, q0=(0.0, 0.0), p0=(0.0, 0.0)):
        """Single-mode cavity instead of the grid (x and y polarisations); call after
        adding the emitters, before stepping."""
        st = lib().ora_set_cavity(self._h, float(omega), float(volume),
                                  _f64(q0, (2,)), _f64(p0, (2,)))
        if st != 0:
            raise ValueError("oracle: bad cavity")

    def add_susceptibility(self, box, omega0, gamma, sigma, drude=False):
        """Lorentz (or Drude) pole chi = sigma w0^2 / (kappa w0^2 - w^2 - i w gamma) over
        the half-open cell box (x0, y0, z0, x1, y1, z1); eps of its cells is eps_inf."""
        b = (C.c_int * 6)(*[int(v) for v in box])
        st = lib().ora_add_susceptibility(self._h, b, float(omega0), float(gamma), float(sigma),
                                          1 if drude else 0)
        if st != 0:
            raise ValueError("oracle: bad susceptibility")

    def cavity(self):
        """(q_x, q_y, p_x, p_y, d_x, d_y): q and d at the current step, p half a step
        before."""
        out = np.zeros(6)
        lib().ora_get_cavity(self._h, out)
        return out

    def emitters_step_prescribed(self, Et):
        M = len(self.nlev)
        lib().ora_emitters_step_prescribed(self._h, _f64(Et, (M, 3)).ravel())


    def emitters_step_wave(self, pol, amp, omega, tau, t0, z0, t):
        """One classical-path step of every emitter under the travelling pulse
        amp f(t - (z_m - z0)) pol (eq. E_analytical), the step centred at time t."""
        lib().ora_emitters_step_wave(self._h, _f64(pol, (3,)), amp, omega, tau, t0, z0, t)
    def dipole_rate_trace(self, m, Et):
        out = np.zeros(3)
        lib().ora_dipole_rate_trace(self._h, m, _f64(Et, (3,)), out)
        return out
