"""ctypes binding of libmlk (include/mlk.h): argument marshalling only.

Every numerical step runs in the HIP kernels of ``libmlk.so``.  PyTorch is
used only to hand over the current HIP stream when the caller wants the
library to run on it.  If the library is missing this module raises; there
is no fallback path.

Grid arrays are numpy arrays of shape (nz, ny, nx) (x fastest), float64.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmlk.so")

MLK_OK, MLK_EINVAL, MLK_ENOMEM, MLK_EDEVICE, MLK_ESTATE, MLK_EUNSUPPORTED, MLK_ENUMERIC = range(7)
FP64, FP32_FIELDS = 0, 1
BC = {"pec": 0, "periodic": 1, "cpml": 2}
MEM_HOST, MEM_DEVICE = 0, 1
SWEEP = {"fused": 0, "plain": 1}
SCATTER = {"owner": 0, "atomic": 1}
SERIES_PROBE, SERIES_FLUX, SERIES_POPULATION, SERIES_ENERGY = 0, 1, 2, 3

_STATUS = {1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ESTATE", 5: "EUNSUPPORTED", 6: "ENUMERIC"}


class MlkError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"mlk {_STATUS.get(status, status)}: {msg}")
        self.status = status


class GridDesc(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("dx", C.c_double), ("courant", C.c_double),
        ("precision", C.c_int32),
        ("bc", C.c_int32 * 6), ("cpml_cells", C.c_int32 * 6),
        ("cpml_m", C.c_double), ("cpml_sigma_scale", C.c_double),
        ("cpml_kappa_max", C.c_double), ("cpml_alpha_max", C.c_double),
        ("window_r", C.c_double),
        ("stream", C.c_void_p),
        ("device", C.c_int32),
        ("sweep", C.c_int32),
        ("scatter", C.c_int32),
    ]


_lib = None

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_lp = C.POINTER(C.c_int64)


class Buffers(C.Structure):
    """mlk_buffers: caller-owned device memory for the evolving state."""
    _fields_ = [("field", (C.c_void_p * 6) * 2), ("psi", C.c_void_p * 2),
                ("tls_state", C.c_void_p), ("ml_state", C.c_void_p)]


class Objective(C.Structure):
    _fields_ = [("kind", C.c_int32), ("weights", C.c_void_p)]


def lib():
    """Load libmlk.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2512_06173_amd/build.py")
    # torch ships its own HIP runtime under the same soname as the system one that
    # libmlk links.  Loading torch first makes the library bind to that runtime, so the
    # process holds one HIP runtime and torch's streams and device memory are valid
    # handles for the library (loaded the other way round, two runtimes would share
    # the GPU and torch would find no device).
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    st = C.c_int
    sim = C.c_void_p
    sigs = {
        "mlk_grid_desc_init": (None, [C.POINTER(GridDesc)]),
        "mlk_last_error": (C.c_char_p, []),
        "mlk_version": (C.c_char_p, []),
        "mlk_create": (st, [C.POINTER(GridDesc), C.POINTER(C.c_void_p)]),
        "mlk_destroy": (st, [sim]),
        "mlk_set_eps": (st, [sim, _dp, C.c_int32]),
        "mlk_set_field": (st, [sim, C.c_int32, _dp, C.c_int32]),
        "mlk_add_tls": (st, [sim, C.c_int32, _dp, _dp, _dp, _dp, _dp, _dp, _ip]),
        "mlk_add_multilevel": (st, [sim, C.c_int32, _ip, _lp, _lp, _dp, _dp, _dp, _dp, _dp, _dp,
                                    _dp, _dp, _ip]),
        "mlk_add_plane_source": (st, [sim, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_double,
                                      C.c_double, C.c_double]),
        "mlk_add_point_source": (st, [sim, C.c_int32, _ip, C.c_double, C.c_double, C.c_double,
                                      C.c_double]),
        "mlk_add_probe": (st, [sim, C.c_int32, _ip, _ip]),
        "mlk_add_flux_plane": (st, [sim, C.c_int32, C.c_int32]),
        "mlk_record_populations": (st, [sim, C.c_int32]),
        "mlk_record_energy": (st, [sim, C.c_int32]),
        "mlk_step": (st, [sim, C.c_int64]),
        "mlk_sync": (st, [sim]),
        "mlk_step_count": (st, [sim, _lp]),
        "mlk_get_field": (st, [sim, C.c_int32, _dp, C.c_int32]),
        "mlk_get_rho": (st, [sim, C.c_int32, _dp, C.c_int32, _ip]),
        "mlk_get_tls_state": (st, [sim, C.c_int32, C.c_int32, _dp]),
        "mlk_get_emitter_io": (st, [sim, _dp, _dp]),
        "mlk_get_series": (st, [sim, C.c_int32, C.c_int32, _dp, C.c_int64, _lp]),
        "mlk_get_flux_total": (st, [sim, _dp]),
        "mlk_checkpoint_size": (st, [sim, C.POINTER(C.c_size_t)]),
        "mlk_checkpoint_save": (st, [sim, C.c_void_p, C.c_int32]),
        "mlk_checkpoint_load": (st, [sim, C.c_void_p, C.c_int32]),
        "mlk_set_timing": (st, [sim, C.c_int32]),
        "mlk_get_phase_time": (st, [sim, C.c_int32, _dp, _lp]),
        "mlk_get_interior_box": (st, [sim, _ip]),
        "mlk_batch_create": (st, [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_void_p)]),
        "mlk_batch_step": (st, [C.c_void_p, C.c_int64]),
        "mlk_batch_capture": (st, [C.c_void_p, C.c_int64]),
        "mlk_batch_replay": (st, [C.c_void_p, C.c_int64]),
        "mlk_batch_sync": (st, [C.c_void_p]),
        "mlk_batch_destroy": (st, [C.c_void_p]),
        "mlk_batch_autotune": (st, [C.c_void_p, C.c_char_p]),
        "mlk_step_prescribed": (st, [sim, C.c_int64, C.c_void_p, C.c_int32, C.c_void_p]),
        "mlk_step_prescribed_noalloc": (st, [sim, C.c_int64, C.c_void_p, C.c_int32,
                                             C.c_void_p]),
        "mlk_step_prescribed_wave": (st, [sim, C.c_int64, _dp, C.c_double, C.c_double,
                                          C.c_double, C.c_double, C.c_double, C.c_double,
                                          C.c_void_p]),
        "mlk_set_cavity": (st, [sim, C.c_double, C.c_double, _dp, _dp]),
        "mlk_get_cavity": (st, [sim, _dp]),
        "mlk_add_susceptibility": (st, [sim, _ip, C.c_double, C.c_double, C.c_double, C.c_int32]),
        "mlk_adjoint": (st, [sim, C.POINTER(Objective), C.c_int64, C.c_int32, _ip, C.c_void_p,
                             C.c_void_p, C.POINTER(C.c_double)]),
        "mlk_set_eps_box": (st, [sim, _ip, _dp, C.c_int32]),
        "mlk_get_adjoint_times": (st, [sim, _dp, _dp]),
        "mlk_set_tls_dipoles": (st, [sim, C.c_int32, C.c_int32, _dp]),
        "mlk_autotune": (st, [sim, C.c_char_p]),
        "mlk_set_tuning": (st, [sim, C.c_int32, C.c_int32]),
        "mlk_get_tuning": (st, [sim, _ip, _ip]),
        "mlk_set_tile_width": (st, [sim, C.c_int32]),
        "mlk_get_tile_width": (st, [sim, _ip]),
        "mlk_set_sweep_layers": (st, [sim, C.c_int32]),
        "mlk_get_sweep_layers": (st, [sim, _ip]),
        "mlk_stream_copy": (st, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int32, C.c_int32,
                                 C.c_void_p]),
        "mlk_buffer_bytes": (st, [sim, C.POINTER(C.c_size_t)]),
        "mlk_bind_device_buffers": (st, [sim, C.POINTER(Buffers)]),
        "mlk_get_field_set": (st, [sim, _ip]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def exported_symbols():
    """Names the binding expects the library to export."""
    return ["mlk_grid_desc_init", "mlk_last_error", "mlk_version", "mlk_create", "mlk_destroy",
            "mlk_set_eps", "mlk_set_field", "mlk_add_tls", "mlk_add_multilevel",
            "mlk_add_plane_source", "mlk_add_point_source", "mlk_add_probe", "mlk_add_flux_plane",
            "mlk_record_populations", "mlk_record_energy", "mlk_step", "mlk_step_prescribed",
            "mlk_step_prescribed_noalloc", "mlk_step_prescribed_wave",
            "mlk_set_cavity", "mlk_get_cavity", "mlk_add_susceptibility", "mlk_sync", "mlk_step_count", "mlk_get_field",
            "mlk_get_rho", "mlk_get_tls_state", "mlk_get_emitter_io", "mlk_get_series",
            "mlk_get_flux_total", "mlk_checkpoint_size", "mlk_checkpoint_save",
            "mlk_checkpoint_load", "mlk_set_timing", "mlk_get_phase_time",
            "mlk_get_interior_box", "mlk_batch_create", "mlk_batch_step", "mlk_batch_capture",
            "mlk_batch_replay", "mlk_batch_sync", "mlk_batch_destroy", "mlk_batch_autotune",
            "mlk_autotune",
            "mlk_set_tuning", "mlk_get_tuning", "mlk_set_tile_width", "mlk_get_tile_width",
            "mlk_set_sweep_layers", "mlk_get_sweep_layers", "mlk_adjoint", "mlk_set_eps_box",
            "mlk_set_tls_dipoles", "mlk_get_adjoint_times", "mlk_stream_copy",
            "mlk_buffer_bytes", "mlk_bind_device_buffers", "mlk_get_field_set"]


def _check(st):
    if st != MLK_OK:
        raise MlkError(st, lib().mlk_last_error().decode(errors="replace"))


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_ip)


def _i64(a):
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(_lp)


def current_stream_handle():
    """HIP stream of torch's current stream on the current device (ROCm build)."""
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def stream_copy(src, dst, variant=1, blocks=4096):
    """Calibration copy of the bytes of torch tensor src into dst (same size, device
    memory) on torch's current stream (mlk_stream_copy)."""
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes
    _check(lib().mlk_stream_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nbytes,
                                 int(variant), int(blocks), current_stream_handle()))


class Simulation:
    """One coupled Yee-FDTD / emitter simulation on one GPU."""

    def __init__(self, shape, dx=1.0, courant=0.5, precision="fp64", bc=("pec",) * 6,
                 cpml=(0,) * 6, pml_m=3.0, pml_sigma_scale=0.8, pml_kappa_max=1.0,
                 pml_alpha_max=0.0, window_r=3.0, sweep="fused", scatter="owner", stream=None,
                 device=0):
        L = lib()
        d = GridDesc()
        L.mlk_grid_desc_init(C.byref(d))
        d.nx, d.ny, d.nz = (int(v) for v in shape)
        d.dx, d.courant = float(dx), float(courant)
        d.precision = FP64 if precision == "fp64" else FP32_FIELDS
        for f in range(6):
            d.bc[f] = BC[bc[f]] if isinstance(bc[f], str) else int(bc[f])
            d.cpml_cells[f] = int(cpml[f])
        d.cpml_m, d.cpml_sigma_scale = float(pml_m), float(pml_sigma_scale)
        d.cpml_kappa_max, d.cpml_alpha_max = float(pml_kappa_max), float(pml_alpha_max)
        d.window_r = float(window_r)
        d.stream = stream.value if isinstance(stream, C.c_void_p) else stream
        d.device = int(device)
        d.sweep = SWEEP[sweep] if isinstance(sweep, str) else int(sweep)
        d.scatter = SCATTER[scatter] if isinstance(scatter, str) else int(scatter)
        h = C.c_void_p()
        _check(L.mlk_create(C.byref(d), C.byref(h)))
        self._h = h
        self.shape = (d.nx, d.ny, d.nz)
        self.precision = precision
        self.fused = d.sweep == SWEEP["fused"]
        self._bound = None
        self.dt = courant * dx
        self.nlev = []
        self.n_tls = 0  # two-level emitters (mlk_add_tls), in id order
        self.nprobe = 0

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _check(lib().mlk_destroy(h))  # refused while the sim belongs to a batch
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def ncell(self):
        nx, ny, nz = self.shape
        return nx * ny * nz

    # ------------------------------------------------------------ set-up
    # ------------------------------------------------------------ caller memory
    def buffer_bytes(self):
        """Bytes of one field array, one psi set, the two-level and multilevel states."""
        v = (C.c_size_t * 4)()
        _check(lib().mlk_buffer_bytes(self._h, v))
        return tuple(int(x) for x in v)

    def bind_torch(self, fields=True, psi=True, states=True):
        """Back the evolving state with torch tensors on the sim's device (allocated
        here, kept referenced by the sim): field sets, CPML state and emitter states
        (mlk_bind_device_buffers).  Bind the emitter states after the last emitter is
        added.  Returns the dict of tensors."""
        import torch
        fb, pb, tb, mb = self.buffer_bytes()
        dt = torch.float32 if self.precision == "fp32" else torch.float64
        esz = 4 if self.precision == "fp32" else 8
        b = Buffers()
        out = {"field": [[None] * 6 for _ in range(2)], "psi": [None, None], "tls": None,
               "ml": None}
        sets = 2 if self.fused else 1
        for q in range(sets):
            if fields:
                for c in range(6):
                    t = torch.empty(fb // esz, dtype=dt, device="cuda")
                    out["field"][q][c] = t
                    b.field[q][c] = t.data_ptr()
            if psi and pb:
                t = torch.empty(pb // esz, dtype=dt, device="cuda")
                out["psi"][q] = t
                b.psi[q] = t.data_ptr()
        if states and tb:
            out["tls"] = torch.empty(tb // 8, dtype=torch.float64, device="cuda")
            b.tls_state = out["tls"].data_ptr()
        if states and mb:
            out["ml"] = torch.empty(mb // 8, dtype=torch.float64, device="cuda")
            b.ml_state = out["ml"].data_ptr()
        torch.cuda.synchronize()
        _check(lib().mlk_bind_device_buffers(self._h, C.byref(b)))
        self._bound = out
        return out

    def field_set(self):
        v = np.zeros(1, dtype=np.int32)
        _check(lib().mlk_get_field_set(self._h, v.ctypes.data_as(_ip)))
        return int(v[0])

    def field_tensor(self, comp):
        """The bound torch tensor holding the current values of component comp (0..5),
        shaped (nz, ny, nx)."""
        nx, ny, nz = self.shape
        return self._bound["field"][self.field_set()][comp].view(nz, ny, nx)

    def set_eps(self, eps):
        a, p = _d(np.asarray(eps, dtype=np.float64).ravel())
        _check(lib().mlk_set_eps(self._h, p, MEM_HOST))

    def set_field(self, comp, arr):
        a, p = _d(np.asarray(arr, dtype=np.float64).ravel())
        _check(lib().mlk_set_field(self._h, comp, p, MEM_HOST))

    def add_tls(self, pos, sigma, gamma, omega0, dipole, rho0):
        pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
        n = pos.shape[0]
        b = lambda v: _d(np.broadcast_to(np.asarray(v, dtype=np.float64), (n,)).copy())
        keep = [_d(pos), b(sigma), b(gamma), b(omega0),
                _d(np.asarray(dipole, dtype=np.float64).reshape(n, 3)),
                _d(np.asarray(rho0, dtype=np.float64).reshape(n, 3))]
        first = C.c_int32()
        _check(lib().mlk_add_tls(self._h, n, *[k[1] for k in keep], C.byref(first)))
        self.nlev += [2] * n
        self.n_tls += n
        return first.value

    def add_multilevel(self, nlev, energies, mop, dipole, gphi, rho0, pos, sigma, gamma):
        n = len(nlev)
        nl = np.asarray(nlev, dtype=np.int32)
        eoff = np.zeros(n, dtype=np.int64)
        moff = np.zeros(n, dtype=np.int64)
        eo = mo = 0
        for q in range(n):
            eoff[q], moff[q] = eo, mo
            eo += nl[q]
            mo += nl[q] * nl[q]
        en = np.concatenate([np.asarray(e, dtype=np.float64).ravel() for e in energies])
        mm = np.concatenate([np.asarray(m, dtype=np.float64).ravel() for m in mop])
        rr = np.concatenate([np.asarray(r, dtype=np.complex128).ravel() for r in rho0])
        ri = np.stack([rr.real, rr.imag], axis=1).ravel()
        b = lambda v: _d(np.broadcast_to(np.asarray(v, dtype=np.float64), (n,)).copy())
        keep = [_i32(nl), _i64(eoff), _i64(moff), _d(en), _d(mm),
                _d(np.asarray(dipole, dtype=np.float64).reshape(n, 3)), b(gphi), _d(ri),
                _d(np.asarray(pos, dtype=np.float64).reshape(n, 3)), b(sigma), b(gamma)]
        first = C.c_int32()
        _check(lib().mlk_add_multilevel(self._h, n, *[k[1] for k in keep], C.byref(first)))
        self.nlev += [int(v) for v in nl]
        return first.value

    def add_plane_source(self, axis, index, comp, amp, omega, tau, t0):
        _check(lib().mlk_add_plane_source(self._h, axis, index, comp, amp, omega, tau, t0))

    def add_point_source(self, comp, ijk, amp, omega, tau, t0):
        a, p = _i32(ijk)
        _check(lib().mlk_add_point_source(self._h, comp, p, amp, omega, tau, t0))

    def add_probe(self, comp, ijk):
        a, p = _i32(ijk)
        pid = C.c_int32()
        _check(lib().mlk_add_probe(self._h, comp, p, C.byref(pid)))
        self.nprobe += 1
        return pid.value

    def add_flux_plane(self, axis, index):
        _check(lib().mlk_add_flux_plane(self._h, axis, index))

    def record_populations(self, every=1):
        _check(lib().mlk_record_populations(self._h, int(every)))

    def record_energy(self, every=1):
        _check(lib().mlk_record_energy(self._h, int(every)))

    # ------------------------------------------------------------ stepping
    def step(self, n=1):
        _check(lib().mlk_step(self._h, int(n)))

    def sync(self):
        _check(lib().mlk_sync(self._h))

    def step_prescribed(self, Et, record=False):
        """Classical-path steps: every emitter advanced under the given field (no grid,
        no back-action).  Et: (nsteps, M, 3) or (M, 3), gamma times the smeared field per
        emitter.  With record, returns the two-level states after every step,
        (nsteps, ntls, 3) as (rho11, Re rho01, Im rho01)."""
        return self._prescribed(lib().mlk_step_prescribed, Et, record)

    def step_prescribed_noalloc(self, Et, record=False):
        """As step_prescribed, through the library's fixed staging array: the call
        allocates no device memory."""
        return self._prescribed(lib().mlk_step_prescribed_noalloc, Et, record)

    def step_wave(self, nsteps, pol, amp, omega, tau, t0, z0=0.0, t_start=0.0, record=False):
        """Classical-path steps under the travelling pulse amp f(t - (z - z0)) pol of eq.
        E_analytical, evaluated on the device; returns the recorded two-level states
        (nsteps, ntls, 3) with record."""
        p = np.ascontiguousarray(np.asarray(pol, dtype=np.float64).reshape(3))
        out = np.zeros((int(nsteps), self.n_tls, 3)) if record else None
        _check(lib().mlk_step_prescribed_wave(
            self._h, int(nsteps), p.ctypes.data_as(_dp), float(amp), float(omega), float(tau),
            float(t0), float(z0), float(t_start),
            out.ctypes.data_as(C.c_void_p) if record and self.n_tls else None))
        return out

    def _prescribed(self, fn, Et, record):
        M = len(self.nlev)
        E = np.ascontiguousarray(np.asarray(Et, dtype=np.float64).reshape(-1, M, 3))
        out = np.zeros((E.shape[0], self.n_tls, 3)) if record else None
        _check(fn(self._h, E.shape[0], E.ctypes.data_as(C.c_void_p), MEM_HOST,
                  out.ctypes.data_as(C.c_void_p) if record and self.n_tls else None))
        return out

    def add_susceptibility(self, box, omega0, gamma, sigma, drude=False):
        """Lorentz (or Drude) pole chi = sigma w0^2 / (kappa w0^2 - w^2 - i w gamma) over the
        half-open cell box (x0, y0, z0, x1, y1, z1); eps of its cells is eps_inf."""
        b = np.ascontiguousarray(np.asarray(box, dtype=np.int32).reshape(6))
        _check(lib().mlk_add_susceptibility(self._h, b.ctypes.data_as(_ip), float(omega0),
                                            float(gamma), float(sigma), 1 if drude else 0))

    def set_cavity(self, omega, volume, q0=(0.0, 0.0), p0=(0.0, 0.0)):
        """Single-mode cavity in place of the grid (x and y polarisations); call after
        adding the emitters, before stepping."""
        q = np.ascontiguousarray(np.asarray(q0, dtype=np.float64).reshape(2))
        p = np.ascontiguousarray(np.asarray(p0, dtype=np.float64).reshape(2))
        _check(lib().mlk_set_cavity(self._h, float(omega), float(volume),
                                    q.ctypes.data_as(_dp), p.ctypes.data_as(_dp)))

    def cavity(self):
        """(q_x, q_y, p_x, p_y, d_x, d_y): q and d at the current step, p half a step
        before."""
        out = np.zeros(6)
        _check(lib().mlk_get_cavity(self._h, out.ctypes.data_as(_dp)))
        return out

    @property
    def step_count(self):
        v = C.c_int64()
        _check(lib().mlk_step_count(self._h, C.byref(v)))
        return v.value

    # ------------------------------------------------------------ read-back
    def get_field(self, comp):
        nx, ny, nz = self.shape
        out = np.empty(self.ncell)
        _check(lib().mlk_get_field(self._h, comp, out.ctypes.data_as(_dp), MEM_HOST))
        return out.reshape(nz, ny, nx)

    def fields(self):
        return [self.get_field(c) for c in range(6)]

    def rho(self, m):
        L = self.nlev[m]
        out = np.zeros(2 * L * L)
        nl = C.c_int32()
        _check(lib().mlk_get_rho(self._h, m, out.ctypes.data_as(_dp), out.size, C.byref(nl)))
        return (out[0::2] + 1j * out[1::2]).reshape(L, L)

    def tls_state(self, first=0, count=None):
        if count is None:
            count = len(self.nlev) - first
        out = np.zeros((count, 3))
        _check(lib().mlk_get_tls_state(self._h, first, count, out.ctypes.data_as(_dp)))
        return out

    def emitter_io(self):
        M = len(self.nlev)
        Et = np.zeros((max(M, 1), 3))
        md = np.zeros((max(M, 1), 3))
        _check(lib().mlk_get_emitter_io(self._h, Et.ctypes.data_as(_dp), md.ctypes.data_as(_dp)))
        return Et[:M], md[:M]

    def _series(self, kind, sid=0):
        n = C.c_int64()
        _check(lib().mlk_get_series(self._h, kind, sid, None, 0, C.byref(n)))
        out = np.zeros(max(n.value, 1))
        _check(lib().mlk_get_series(self._h, kind, sid, out.ctypes.data_as(_dp), n.value,
                                    C.byref(n)))
        return out[:n.value]

    def probe(self, pid):
        return self._series(SERIES_PROBE, pid)

    def flux_series(self):
        return self._series(SERIES_FLUX)

    def flux_total(self):
        v = C.c_double()
        _check(lib().mlk_get_flux_total(self._h, C.byref(v)))
        return v.value

    def energy_series(self):
        """W^n on the recorded steps (mlk_record_energy)."""
        return self._series(SERIES_ENERGY)

    def populations(self):
        v = self._series(SERIES_POPULATION)
        per = sum(L - 1 for L in self.nlev)
        return v.reshape(-1, per) if per else v.reshape(0, 0)

    # ------------------------------------------------------------ checkpoints
    def checkpoint_size(self):
        v = C.c_size_t()
        _check(lib().mlk_checkpoint_size(self._h, C.byref(v)))
        return v.value

    def checkpoint_save(self):
        buf = np.zeros(self.checkpoint_size(), dtype=np.uint8)
        _check(lib().mlk_checkpoint_save(self._h, buf.ctypes.data_as(C.c_void_p), MEM_HOST))
        return buf

    def checkpoint_save_device(self):
        """The checkpoint in a torch uint8 tensor on the GPU (no host copy)."""
        import torch
        t = torch.empty(self.checkpoint_size(), dtype=torch.uint8, device="cuda")
        _check(lib().mlk_checkpoint_save(self._h, C.c_void_p(t.data_ptr()), MEM_DEVICE))
        return t

    def checkpoint_load_device(self, t):
        _check(lib().mlk_checkpoint_load(self._h, C.c_void_p(t.data_ptr()), MEM_DEVICE))

    def objective_value(self, objective, nsteps, weights=None):
        """The adjoint's objective over the next nsteps steps, by one plain run from a
        device checkpoint of the current state, which is then restored: "flux" (dt sum F
        over the steps) or "population" (sum_m weights[m] rho11_m after the last
        step, two-level emitters)."""
        blob = self.checkpoint_save_device()
        f0 = self.flux_total() if objective == "flux" else 0.0
        self.step(nsteps)
        if objective == "flux":
            val = self.flux_total() - f0
        else:
            w = np.broadcast_to(np.asarray(weights, dtype=np.float64), (len(self.nlev),))
            st = self.tls_state(0, self.n_tls)
            val = 0.0
            for m in range(self.n_tls):
                val += float(w[m]) * float(st[m, 0])
        self.checkpoint_load_device(blob)
        return val

    def checkpoint_load(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        _check(lib().mlk_checkpoint_load(self._h, buf.ctypes.data_as(C.c_void_p), MEM_HOST))


    # ------------------------------------------------------------ timing
    def set_timing(self, phases=True):
        """Per-phase HIP-event timing of the step loop (clears totals): True times every
        phase, False none, or an iterable of names from PHASES."""
        if phases is True:
            mask = (1 << len(PHASES)) - 1
        elif phases is False or phases is None:
            mask = 0
        else:
            mask = 0
            for name in phases:
                mask |= 1 << PHASES[name]
        _check(lib().mlk_set_timing(self._h, mask))

    def phase_time(self, phase):
        """(summed ms, timed launches) of a phase name from PHASES."""
        ms = C.c_double()
        n = C.c_int64()
        _check(lib().mlk_get_phase_time(self._h, PHASES[phase], C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def interior_box(self):
        """Interior box of the fused sweep, ((lo_x, lo_y, lo_z), (hi_x, hi_y, hi_z))."""
        b, pb = _i32(np.zeros(6))
        _check(lib().mlk_get_interior_box(self._h, pb))
        return tuple(int(v) for v in b[:3]), tuple(int(v) for v in b[3:])


    # ------------------------------------------------------------ adjoint
    def adjoint(self, objective, nsteps, box, weights=None, checkpoint_every=200):
        """Value and gradients of an objective over the next nsteps steps by the
        checkpointed discrete adjoint.  objective: "flux" (dt sum F over the steps) or
        "population" (sum_m weights[m] rho11_m at the end).  box: ((x0, y0, z0), (x1, y1,
        z1)) half-open design box.  Returns (value, grad_eps (z, y, x) over the box,
        grad_dipole (M, 3)); the state of the sim is unchanged."""
        (x0, y0, z0), (x1, y1, z1) = box
        b, pb = _i32(np.array([x0, y0, z0, x1, y1, z1]))
        M = len(self.nlev)
        ge = np.zeros(max(1, (z1 - z0) * (y1 - y0) * (x1 - x0)))
        gd = np.zeros(max(1, 3 * M))
        kind = {"flux": 0, "population": 1}[objective]
        w = None
        if kind == 1:
            w = np.ascontiguousarray(np.broadcast_to(np.asarray(weights, dtype=np.float64), (M,)))
        obj = Objective(kind, w.ctypes.data if w is not None else None)
        val = C.c_double()
        _check(lib().mlk_adjoint(self._h, C.byref(obj), int(nsteps), int(checkpoint_every), pb,
                                 ge.ctypes.data, gd.ctypes.data, C.byref(val)))
        return (val.value, ge[:(z1 - z0) * (y1 - y0) * (x1 - x0)].reshape(z1 - z0, y1 - y0, x1 - x0),
                gd[:3 * M].reshape(M, 3))

    def adjoint_times(self):
        """(forward-with-checkpoints ms, reverse ms) of the last adjoint call."""
        f, r = C.c_double(), C.c_double()
        _check(lib().mlk_get_adjoint_times(self._h, C.byref(f), C.byref(r)))
        return f.value, r.value

    def set_eps_box(self, box, eps):
        """eps_r over a half-open box ((x0, y0, z0), (x1, y1, z1)); eps shaped (z, y, x)."""
        (x0, y0, z0), (x1, y1, z1) = box
        b, pb = _i32(np.array([x0, y0, z0, x1, y1, z1]))
        e, pe = _d(np.asarray(eps, dtype=np.float64).reshape(-1))
        _check(lib().mlk_set_eps_box(self._h, pb, pe, MEM_HOST))

    def set_tls_dipoles(self, first, dipoles):
        d, pd = _d(np.asarray(dipoles, dtype=np.float64).reshape(-1, 3))
        _check(lib().mlk_set_tls_dipoles(self._h, int(first), d.shape[0], pd))

    # ------------------------------------------------------------ tuning
    def autotune(self, cache_path=None):
        """Pick the fused sweep's tile shape by timing (optionally cached in JSON);
        returns (ty, kz, tile width)."""
        _check(lib().mlk_autotune(self._h, cache_path.encode() if cache_path else None))
        return self.tuning() + (self.tile_width(),)

    def tuning(self):
        ty, kz = C.c_int32(), C.c_int32()
        _check(lib().mlk_get_tuning(self._h, C.byref(ty), C.byref(kz)))
        return ty.value, kz.value

    def set_tuning(self, ty, kz):
        _check(lib().mlk_set_tuning(self._h, int(ty), int(kz)))

    def tile_width(self):
        """x cells per workgroup of the fused sweep: 64 or 32."""
        tx = C.c_int32()
        _check(lib().mlk_get_tile_width(self._h, C.byref(tx)))
        return tx.value

    def set_tile_width(self, tx):
        _check(lib().mlk_set_tile_width(self._h, int(tx)))

    def sweep_layers(self):
        """Where the fused sweep updates the y and z CPML layers (FP32): 0 the plain shell
        passes, 1 the fused kernel itself, 2 one launch of the full kernel over the layer
        frame around a box that the lean kernel sweeps."""
        on = C.c_int32()
        _check(lib().mlk_get_sweep_layers(self._h, C.byref(on)))
        return on.value

    def set_sweep_layers(self, mode):
        _check(lib().mlk_set_sweep_layers(self._h, int(mode)))


class Batch:
    """Independent simulations stepped together: one launch per phase for all of them,
    optionally replayed from a captured hipGraph."""

    def __init__(self, sims):
        self.sims = list(sims)
        arr = (C.c_void_p * len(self.sims))(*[s._h for s in self.sims])
        h = C.c_void_p()
        _check(lib().mlk_batch_create(arr, len(self.sims), C.byref(h)))
        self._h = h

    def step(self, n=1):
        _check(lib().mlk_batch_step(self._h, int(n)))

    def capture(self, steps_per_replay):
        _check(lib().mlk_batch_capture(self._h, int(steps_per_replay)))

    def replay(self, n=1):
        _check(lib().mlk_batch_replay(self._h, int(n)))

    def sync(self):
        _check(lib().mlk_batch_sync(self._h))

    def autotune(self, cache_path=None):
        """One tile shape and layer mode for every member, chosen by timing the batch's
        sweep phase (optionally cached in JSON); returns (ty, kz, layers, tile width)."""
        _check(lib().mlk_batch_autotune(self._h, cache_path.encode() if cache_path else None))
        ty, kz = self.sims[0].tuning()
        return ty, kz, self.sims[0].sweep_layers(), self.sims[0].tile_width()

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().mlk_batch_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def coupled_objective(sim, eps_box, dipoles, objective, nsteps, box, weights=None,
                      checkpoint_every=200):
    """Differentiable objective of a run: eps_box (z, y, x) sets eps_r in the design box
    and dipoles (M, 3) the two-level emitters' dipoles, then nsteps coupled steps run
    from the sim's current state (which is left unchanged).  forward runs the steps
    once from a device checkpoint and reads the objective (flux through the sim's flux
    plane integrated over the steps, or sum_m weights[m] rho11_m at the end); backward
    calls the checkpointed adjoint (mlk_adjoint) for the gradients.  A forward-only
    evaluation therefore costs one plain run."""
    import torch

    class _Fn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, e, d):
            en = e.detach().cpu().double().numpy()
            dn = d.detach().cpu().double().numpy()
            sim.set_eps_box(box, en)
            sim.set_tls_dipoles(0, dn)
            val = sim.objective_value(objective, nsteps, weights)
            ctx.params = (en, dn)
            return torch.tensor(val, dtype=e.dtype, device=e.device)

        @staticmethod
        def backward(ctx, gout):
            en, dn = ctx.params
            sim.set_eps_box(box, en)
            sim.set_tls_dipoles(0, dn)
            _, ge, gd = sim.adjoint(objective, nsteps, box, weights, checkpoint_every)
            return (gout * torch.from_numpy(ge).to(gout.device, gout.dtype),
                    gout * torch.from_numpy(gd).to(gout.device, gout.dtype))

    return _Fn.apply(eps_box, dipoles)


PHASES = {"emitters": 0, "sweep": 1, "shell": 2, "sources": 3, "scatter": 4, "detectors": 5,
          "poles": 6}


def from_workload(w, pop_every=None, **kw):
    """Build a Simulation from a seeded Workload (paper_2512_06173_amd.workloads)."""
    kw.setdefault("precision", w.precision)
    sim = Simulation(w.shape, dx=w.dx, courant=w.courant, bc=w.bc, cpml=w.cpml, **kw)
    if w.eps is not None:
        sim.set_eps(w.eps)
    if w.tls is not None and len(w.tls):
        t = w.tls
        sim.add_tls(t.pos, t.sigma, t.gamma, t.omega0, t.dipole, t.rho0)
    if w.multilevel is not None and len(w.multilevel):
        m = w.multilevel
        sim.add_multilevel(m.nlev, m.energies, m.mop, m.dipole, m.gphi, m.rho0, m.pos, m.sigma,
                           m.gamma)
    for s in w.plane_sources:
        sim.add_plane_source(s.axis, s.index, s.comp, s.amp, s.omega, s.tau, s.t0)
    for s in w.point_sources:
        sim.add_point_source(s.comp, s.ijk, s.amp, s.omega, s.tau, s.t0)
    for comp, ijk in w.probes:
        sim.add_probe(comp, ijk)
    if w.flux is not None:
        sim.add_flux_plane(*w.flux)
    pe = w.pop_every if pop_every is None else pop_every
    if pe:
        sim.record_populations(pe)
    return sim
