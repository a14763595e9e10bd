"""Pins of the FP64 CPU oracle against closed forms, invariants and the paper's own
decay law.  None of these re-types an oracle formula: each checks a property the
mathematics or the paper fixes, chosen so that a dropped term, a wrong sign, a
wrong index or a transposed operand in the oracle fails one of them.
"""
import contextlib

import numpy as np
import pytest
import scipy.linalg

from oracle.oracle import Oracle, jacobi_eig
from oracle.oracle import set_threads as set_oracle_threads
from oracle.oracle import threads as oracle_threads

S = 0.5


@contextlib.contextmanager
def _one_thread():
    """Small runs of many short steps: one oracle thread (a parallel region per step only
    adds overhead there)."""
    n = oracle_threads()
    set_oracle_threads(1)
    try:
        yield
    finally:
        set_oracle_threads(n)


def _theta(kvec):
    """Phase advance per step of a Yee eigenmode: sin^2(theta/2) = S^2 sum sin^2(k_a/2)."""
    k = np.asarray(kvec, dtype=np.float64)
    return 2.0 * np.arcsin(S * np.sqrt(np.sum(np.sin(k / 2.0) ** 2)))


def _coords(n, comp):
    """Coordinates (x, y, z) of the Yee points of E component comp, arrays (nz,ny,nx)."""
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    x, y, z = i.astype(float), j.astype(float), k.astype(float)
    if comp == 0:
        x = x + 0.5
    elif comp == 1:
        y = y + 0.5
    else:
        z = z + 0.5
    return x, y, z


# --------------------------------------------------------------- P-1 / P-2

@pytest.mark.parametrize("comp,kidx", [(2, (1, 2, 0)), (0, (0, 1, 3)), (1, (2, 0, 1))])
def test_periodic_plane_wave_follows_yee_dispersion(comp, kidx):
    """Transverse discrete plane wave, H^{-1/2} = 0: E^n = E^0 cos((n+1/2)th)/cos(th/2)
    with the Yee numerical dispersion relation (Yee's scheme, Sec. II.A.1)."""
    n, steps = 32, 1000
    kvec = 2 * np.pi * np.array(kidx) / n
    x, y, z = _coords(n, comp)
    e0 = np.cos(kvec[0] * x + kvec[1] * y + kvec[2] * z)
    o = Oracle((n, n, n), bc=("periodic",) * 6)
    o.set_field(comp, e0)
    o.step(steps)
    th = _theta(kvec)
    ref = e0 * np.cos((steps + 0.5) * th) / np.cos(th / 2)
    got = o.get_field(comp)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-12
    for c in range(3):
        if c != comp:
            assert np.max(np.abs(o.get_field(c))) < 1e-13


@pytest.mark.parametrize("comp,modes", [(2, (1, 1, 0)), (0, (0, 1, 1))])
def test_pec_cavity_mode(comp, modes):
    """TM_110 (and its rotation) of a PEC box: E = sin(pi m y/N) sin(...) obeys the same
    discrete law with k_a = pi m_a / N; tangential E vanishes on the walls."""
    n, steps = 32, 1000
    x, y, z = _coords(n, comp)
    kvec = np.pi * np.array(modes) / n
    e0 = np.ones((n, n, n))
    for a, (coord, m) in enumerate(zip((x, y, z), modes)):
        if a != comp and m:
            e0 = e0 * np.sin(np.pi * m * coord / n)
    o = Oracle((n, n, n), bc=("pec",) * 6)
    o.set_field(comp, e0)
    o.step(steps)
    th = _theta(kvec)
    ref = e0 * np.cos((steps + 0.5) * th) / np.cos(th / 2)
    got = o.get_field(comp)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-12


@pytest.mark.parametrize("dx", [1.0, 0.5])
def test_probe_series_is_sampled_after_the_e_update(dx):
    """The probe records E at its Yee point after the E update of each step (t_{n+1}):
    for the discrete plane wave of P-1 the n-th value (0-based) is
    E^0(p) cos((n+1+1/2)th)/cos(th/2).  At dx = 0.5 (dt = S dx) the law is the same in
    cell units, which pins the 1/dx of the curls and dt = S dx."""
    n, steps, comp, kidx = 16, 300, 2, (1, 2, 0)
    kvec = 2 * np.pi * np.array(kidx) / n
    x, y, z = _coords(n, comp)
    e0 = np.cos(kvec[0] * x + kvec[1] * y + kvec[2] * z)
    o = Oracle((n, n, n), dx=dx, bc=("periodic",) * 6)
    assert o.dt == S * dx
    o.set_field(comp, e0)
    ijk = (3, 5, 7)
    pid = o.add_probe(comp, ijk)
    o.step(steps)
    th = _theta(kvec)
    q = np.arange(steps)
    ref = e0[ijk[2], ijk[1], ijk[0]] * np.cos((q + 1.5) * th) / np.cos(th / 2)
    got = o.probe(pid)
    assert got.shape == (steps,)
    assert np.max(np.abs(got - ref)) < 1e-12


def test_population_record_is_taken_after_the_emitter_step():
    """A two-level emitter from |g> in a static uniform field E0: P_e(t) =
    4g^2/(w0^2+4g^2) sin^2(sqrt(w0^2+4g^2) t/2), g = E0.d.  The state starts at t_{-1/2},
    so the record of step n (taken after the emitter step, at t_{n+1/2}) holds
    P_e((n+1) dt).  The field is a uniform E_z in a periodic box (curl-free, so H stays
    zero and E static); eps_r = 1e12 makes the emitter's own current change E by about
    1e-17 per step, so the field it feels is E0 to rounding."""
    n, every, steps, w0, E0, dz = 12, 7, 700, 0.25, 1.0, 0.05
    o = Oracle((n, n, n), bc=("periodic",) * 6)
    o.set_eps(np.full((n, n, n), 1e12))
    o.set_field(2, np.full((n, n, n), E0))
    o.add_tls(np.array([[5.3, 6.1, 5.7]]), [1.0], [1.0], [w0], np.array([[0.0, 0.0, dz]]),
              np.array([[0.0, 0.0, 0.0]]))
    o.record_populations(every)
    o.step(steps)
    pop = o.populations().ravel()
    rec = np.arange(0, steps, every)
    assert pop.shape == rec.shape
    g = E0 * dz
    W = np.sqrt(w0 ** 2 + 4 * g ** 2)
    ref = 4 * g ** 2 / W ** 2 * np.sin(W * (rec + 1) * o.dt / 2) ** 2
    assert np.max(ref) > 0.1
    assert np.max(np.abs(pop - ref)) < 1e-12


# ------------------------------------------------------------------- P-3

def _random_state(n, bc, rng):
    E = [rng.standard_normal((n, n, n)) for _ in range(3)]
    H = [rng.standard_normal((n, n, n)) for _ in range(3)]
    if bc == "pec":  # tangential E on the index-0 wall planes is zero
        E[0][0, :, :] = 0; E[0][:, 0, :] = 0
        E[1][0, :, :] = 0; E[1][:, :, 0] = 0
        E[2][:, 0, :] = 0; E[2][:, :, 0] = 0
    return E, H


@pytest.mark.parametrize("bc", ["pec", "periodic"])
def test_discrete_energy_is_conserved(bc):
    """W^n = 1/2 sum eps|E^n|^2 + 1/2 sum H^{n+1/2}.H^{n-1/2} is exactly invariant for the
    Yee leapfrog without sources or absorbers, for any eps and any initial data."""
    n, steps = 14, 2000
    rng = np.random.default_rng(11)
    o = Oracle((n, n, n), bc=(bc,) * 6)
    o.set_eps(rng.uniform(1.0, 4.0, (n, n, n)))
    E, H = _random_state(n, bc, rng)
    for c in range(3):
        o.set_field(c, E[c])
        o.set_field(3 + c, H[c])
    o.record_energy(True)
    o.step(steps)
    W = o.energy_series()
    assert W.size == steps
    assert np.max(np.abs(W - W[0])) / abs(W[0]) < 1e-12


def test_energy_not_conserved_with_cpml():
    """Sanity: the PML really absorbs (energy decreases)."""
    n = 24
    rng = np.random.default_rng(3)
    o = Oracle((n, n, n), bc=("cpml",) * 6, cpml=(6,) * 6)
    E, H = _random_state(n, "pec", rng)
    for c in range(3):
        o.set_field(c, E[c] * 0)
    o.add_point_source(2, (12, 12, 12), 1.0, 0.5, 8.0, 40.0)
    o.record_energy(True)
    o.step(400)
    W = o.energy_series()
    assert W[-1] < 0.2 * np.max(W)


# ------------------------------------------------------------------- P-4

def _div_D(o, eps):
    E = [o.get_field(c) for c in range(3)]
    D = [eps * e for e in E]
    div = (D[0] - np.roll(D[0], 1, axis=2)) + (D[1] - np.roll(D[1], 1, axis=1)) + \
          (D[2] - np.roll(D[2], 1, axis=0))
    return div


def _div(J):
    return (J[0] - np.roll(J[0], 1, axis=2)) + (J[1] - np.roll(J[1], 1, axis=1)) + \
           (J[2] - np.roll(J[2], 1, axis=0))


@pytest.mark.parametrize("bc,dx", [("pec", 1.0), ("periodic", 1.0), ("pec", 0.5)])
def test_charge_identity_with_emitters_and_source(bc, dx):
    """eps(E^{n+1}-E^n) = dt(curl H - J) and div curl = 0 give, from E^0 = 0,
    div(eps E^n) = -dt sum_k div J^{k+1/2} with J the scattered molecular current plus
    the sources (eqs. Maxwell and J_mol).  In cell differences the 1/dx of both
    divergences cancels and dt = S dx.  The source currents are written out here: a
    point element amp s(t)/dx^3 and a sheet of surface density amp s(t) on a y plane
    carrying J_y (normal to the sheet, so its divergence is not zero), amp s(t)/dx in
    the cells of the plane, with s(t) the Gaussian pulse at t_{k+1/2}."""
    n, steps = 16, 60
    rng = np.random.default_rng(5)
    eps = rng.uniform(1.0, 3.0, (n, n, n))
    o = Oracle((n, n, n), dx=dx, bc=(bc,) * 6)
    o.set_eps(eps)
    pos = np.array([[7.3, 8.1, 7.7], [8.6, 7.2, 8.4], [8.0, 8.0, 8.0]])
    dip = np.array([[0.3, -0.2, 0.4], [0.0, 0.5, 0.1], [0.2, 0.2, -0.3]])
    rho = np.tile([0.5, 0.5, 0.0], (3, 1))
    o.add_tls(pos, [1.0, 0.8, 1.2], [1.0, 0.5, 1.5], [0.25, 0.3, 0.2], dip, rho)
    amp, w, tau, t0 = 0.7, 0.3, 6.0, 15.0
    o.add_point_source(1, (5, 9, 6), amp, w, tau, t0)
    amp2, w2, tau2, t02 = 0.3, 0.2, 5.0, 12.0
    o.add_plane_source(1, 4, 1, amp2, w2, tau2, t02)
    dt = S * dx

    def pulse(t, a, om, ta, tc):
        return a * np.cos(om * (t - tc)) * np.exp(-(t - tc) ** 2 / (2 * ta ** 2))

    Jsum = [np.zeros((n, n, n)) for _ in range(3)]
    for q in range(steps):
        o.step(1)
        _, md = o.emitter_io()
        J = o.scatter(md)
        t = (q + 0.5) * dt
        J[1][6, 9, 5] += pulse(t, amp, w, tau, t0) / dx ** 3
        J[1][:, 4, :] += pulse(t, amp2, w2, tau2, t02) / dx
        for c in range(3):
            Jsum[c] += J[c]
    lhs = _div_D(o, eps)
    rhs = -dt * _div(Jsum)
    inner = (slice(1, n - 1),) * 3 if bc == "pec" else (slice(None),) * 3
    scale = np.max(np.abs(rhs[inner]))
    assert scale > 1e-6
    assert np.max(np.abs(lhs[inner] - rhs[inner])) < 1e-12 * scale


# ------------------------------------------------------------------- P-5

def test_linearity_and_superposition():
    n = 20
    runs = []
    for (a, b) in [(1.0, 0.0), (0.0, 1.0), (1.0, 1.0), (2.5, 0.0)]:
        o = Oracle((n, n, n), bc=("cpml",) * 6, cpml=(5,) * 6)
        o.set_eps(np.where(np.arange(n)[:, None, None] > 10, 2.0, 1.0) * np.ones((n, n, n)))
        if a:
            o.add_point_source(2, (8, 9, 10), a, 0.4, 4.0, 12.0)
        if b:
            o.add_plane_source(2, 7, 1, b, 0.3, 5.0, 15.0)
        o.step(80)
        runs.append(np.stack(o.fields()))
    A, B, AB, A25 = runs
    assert np.linalg.norm(AB - A - B) / np.linalg.norm(AB) < 1e-13
    assert np.linalg.norm(A25 - 2.5 * A) / np.linalg.norm(A25) < 1e-13


# ------------------------------------------------------------------- P-6

CPML_REFLECTION_BOUND = 1e-4


def _probe_run(shape, bc, cpml, src, probes, steps, eps=None, sigma_scale=0.8):
    o = Oracle(shape, bc=bc, cpml=cpml, pml_sigma_scale=sigma_scale)
    if eps is not None:
        o.set_eps(eps)
    if src[0] == "point":
        o.add_point_source(*src[1:])
    else:
        o.add_plane_source(*src[1:])
    ids = [o.add_probe(c, ijk) for c, ijk in probes]
    o.step(steps)
    return [o.probe(p) for p in ids]


def _reflection_2d(sigma_scale):
    bc2 = ("cpml",) * 4 + ("periodic",) * 2
    n, d, steps = 60, 10, 260
    c = n // 2
    probes = [(2, (c, n - d - 2, 0)), (2, (n - d - 4, n - d - 4, 0))]
    src = ("point", 2, (c, c, 0), 1.0, 0.3, 6.0, 25.0)
    small = _probe_run((n, n, 1), bc2, (d, d, d, d, 0, 0), src, probes, steps,
                       sigma_scale=sigma_scale)
    big_n = n + 2 * 150
    off = 150
    probes_big = [(cc, (i + off, j + off, 0)) for cc, (i, j, _) in probes]
    src_big = ("point", 2, (c + off, c + off, 0), 1.0, 0.3, 6.0, 25.0)
    big = _probe_run((big_n, big_n, 1), ("pec",) * 4 + ("periodic",) * 2, (0,) * 6, src_big,
                     probes_big, steps)
    return [np.max(np.abs(s_ - b_)) / np.max(np.abs(b_)) for s_, b_ in zip(small, big)]


def _reflection_z(sigma_scale):
    d, nz, steps = 10, 80, 300
    src = ("plane", 2, 40, 1, 1.0, 0.25, 8.0, 30.0)
    small = _probe_run((1, 1, nz), ("periodic",) * 4 + ("cpml",) * 2, (0, 0, 0, 0, d, d), src,
                       [(1, (0, 0, nz - d - 3))], steps, sigma_scale=sigma_scale)
    big = _probe_run((1, 1, nz + 400), ("periodic",) * 4 + ("pec",) * 2, (0,) * 6,
                     ("plane", 2, 240, 1, 1.0, 0.25, 8.0, 30.0), [(1, (0, 0, 200 + nz - d - 3))],
                     steps)
    return np.max(np.abs(small[0] - big[0])) / np.max(np.abs(big[0]))


def test_cpml_reflection_2d_normal_and_oblique():
    """2-D (z-invariant) pulse hitting the x and y PML: compare with a domain so large that
    nothing returns within the run.  Normal and 45-degree incidence.  With the textbook
    grading (m = 3, sigma_max = 0.8 (m + 1) / dx) the reflection is about 4e-5."""
    for refl in _reflection_2d(0.8):
        assert refl < CPML_REFLECTION_BOUND, refl


def test_cpml_reflection_z_plane_wave():
    """Plane-wave pulse (x/y periodic, one cell wide) through the z PML (about 3e-5)."""
    refl = _reflection_z(0.8)
    assert refl < CPML_REFLECTION_BOUND, refl


@pytest.mark.parametrize("sigma_scale", [0.3, 3.0])
def test_cpml_bound_rejects_a_misgraded_layer(sigma_scale):
    """The bound is tight enough to matter: sigma_max 2.7 times too small or 3.75 times too
    large reflects more than it allows at some incidence."""
    worst = max(_reflection_2d(sigma_scale) + [_reflection_z(sigma_scale)])
    assert worst > CPML_REFLECTION_BOUND, worst


# ------------------------------------------------------------------- P-7

def _one_tls_oracle(pos, n=20, sigma=1.0, gamma=1.0, bc=("pec",) * 6):
    o = Oracle((n, n, n), bc=bc)
    o.add_tls(np.array([pos]), [sigma], [gamma], [0.25], np.array([[0.1, 0.2, 0.3]]),
              np.array([[0.5, 0.5, 0.0]]))
    return o


def test_kernel_window_staggering_and_normalisation():
    """A centre on a cell corner: the window of E_x holds 6 half-integer x points and 7
    integer y, z points (R = 3 sigma, inclusive), weights sum to 1 and their centroid is
    the emitter position (kernel normalised to unit integral, eq. Polarization_mol)."""
    n = 20
    o = _one_tls_oracle((10.0, 10.0, 10.0), n=n)
    for c in range(3):
        idx, w = o.window(0, c)
        assert abs(w.sum() - 1.0) < 1e-15
        assert idx.size == 6 * 7 * 7
        i = idx % n
        j = (idx // n) % n
        k = idx // (n * n)
        pts = np.stack([i, j, k], 1).astype(float)
        pts[:, c] += 0.5
        assert np.allclose(pts.T @ w, [10.0, 10.0, 10.0], atol=1e-13)
        # offsets along the staggered axis are +-0.5..2.5, along the others 0..3
        assert set(np.unique(np.abs(pts[:, c] - 10.0))) == {0.5, 1.5, 2.5}
        for a in range(3):
            if a != c:
                assert set(np.unique(np.abs(pts[:, a] - 10.0))) == {0.0, 1.0, 2.0, 3.0}
        # weights are a Gaussian in the distance: monotone, ratio fixed by sigma
        r2 = np.sum((pts - 10.0) ** 2, axis=1)
        order = np.argsort(r2)
        assert np.all(np.diff(w[order]) <= 1e-18)
    # a generic position keeps unit sum
    o2 = _one_tls_oracle((9.37, 10.81, 10.05), n=n, sigma=1.3)
    for c in range(3):
        _, w = o2.window(0, c)
        assert abs(w.sum() - 1.0) < 1e-15


def test_gather_uniform_field_and_scatter_adjointness():
    n = 20
    rng = np.random.default_rng(9)
    o = Oracle((n, n, n), bc=("periodic",) * 6)
    M = 5
    pos = rng.uniform(4.5, 15.5, (M, 3))
    gam = rng.uniform(0.5, 1.5, M)
    o.add_tls(pos, rng.uniform(0.8, 1.2, M), gam, np.full(M, 0.25), rng.standard_normal((M, 3)),
              np.tile([0.5, 0.5, 0.0], (M, 1)))
    E0 = np.array([0.3, -1.1, 0.7])
    for c in range(3):
        o.set_field(c, np.full((n, n, n), E0[c]))
    Et = o.gather()
    assert np.allclose(Et, gam[:, None] * E0[None, :], rtol=2e-14, atol=0)
    # total scattered current is gamma * mu_dot (unit-integral kernel, dx = 1)
    v = rng.standard_normal((M, 3))
    J = o.scatter(v)
    tot = np.array([J[c].sum() for c in range(3)])
    assert np.allclose(tot, (gam[:, None] * v).sum(0), rtol=1e-14, atol=1e-15)
    # <gather(E), v> = <E, scatter(v)>  (the coupling V = -E~ . mu is symmetric)
    Ef = [rng.standard_normal((n, n, n)) for _ in range(3)]
    for c in range(3):
        o.set_field(c, Ef[c])
    lhs = np.sum(o.gather() * v)
    rhs = sum(np.sum(Ef[c] * J[c]) for c in range(3))
    assert abs(lhs - rhs) < 1e-13 * max(1.0, abs(lhs))


def test_periodic_window_wraps():
    n = 16
    o = _one_tls_oracle((0.2, 8.0, 15.9), n=n, bc=("periodic",) * 6)
    for c in range(3):
        idx, w = o.window(0, c)
        assert idx.min() >= 0 and idx.max() < n ** 3
        assert abs(w.sum() - 1.0) < 1e-15


def test_emitter_too_close_to_wall_is_rejected():
    with pytest.raises(ValueError):
        _one_tls_oracle((3.5, 10.0, 10.0), n=20)
    with pytest.raises(ValueError):
        o = Oracle((24, 24, 24), bc=("cpml",) * 6, cpml=(6,) * 6)
        o.add_tls(np.array([[9.0, 12.0, 12.0]]), [1.0], [1.0], [0.25], np.array([[0, 0, .1]]),
                  np.array([[0.0, 0.0, 0.0]]))


# ------------------------------------------------------------ P-8 .. P-11

def _tls(n_emit, omega0, dip, rho0):
    o = Oracle((1, 1, 1), bc=("periodic",) * 6)
    o.add_tls(np.tile([0.5, 0.5, 0.5], (n_emit, 1)), np.ones(n_emit), np.ones(n_emit), omega0,
              dip, rho0)
    return o


def test_tls_undriven_precession():
    """E~ = 0: rho01(t) = rho01(0) exp(i w0 t), populations constant (H0 = diag(0, w0))."""
    w0 = np.array([0.25, 0.31])
    rho0 = np.array([[0.3, 0.2, 0.35], [0.5, 0.5, 0.0]])
    o = _tls(2, w0, np.array([[0, 0, 0.1], [0.1, 0, 0]]), rho0)
    steps = 777
    for _ in range(steps):
        o.emitters_step_prescribed(np.zeros((2, 3)))
    st = o.tls_state()
    t = steps * o.dt
    r01 = (rho0[:, 1] + 1j * rho0[:, 2]) * np.exp(1j * w0 * t)
    assert np.allclose(st[:, 0], rho0[:, 0], atol=1e-13)
    assert np.allclose(st[:, 1] + 1j * st[:, 2], r01, atol=1e-13)


def test_tls_static_field_rabi_exact():
    """Static field from |g>: P_e(t) = 4g^2/(w0^2+4g^2) sin^2(sqrt(w0^2+4g^2) t/2), g = E.d."""
    w0, E0 = 0.25, np.array([0.0, 0.0, 1.3])
    dips = np.array([[0, 0, 0.05], [0.02, 0, 0.08], [0, 0, 0.2]])
    o = _tls(3, np.full(3, w0), dips, np.zeros((3, 3)))
    g = dips @ E0
    for q in range(1, 601):
        o.emitters_step_prescribed(np.tile(E0, (3, 1)))
        if q % 100 == 0:
            t = q * o.dt
            W = np.sqrt(w0 ** 2 + 4 * g ** 2)
            ref = 4 * g ** 2 / W ** 2 * np.sin(W * t / 2) ** 2
            assert np.allclose(o.tls_state()[:, 0], ref, atol=1e-12, rtol=0)


def test_tls_resonant_rabi_rwa():
    """Resonant cos drive: P_e = sin^2(E0 d t / 2) within the rotating-wave error ~ 2g/w0."""
    w0, d, E0 = 0.25, 0.05, 0.1
    o = _tls(1, [w0], np.array([[0, 0, d]]), np.zeros((1, 3)))
    gR = E0 * d
    steps = int(round(np.pi / gR / o.dt))
    errs = []
    for n in range(steps):
        o.emitters_step_prescribed(np.array([[0, 0, E0 * np.cos(w0 * n * o.dt)]]))
        t = (n + 1) * o.dt
        errs.append(abs(o.tls_state()[0, 0] - np.sin(gR * t / 2) ** 2))
    assert max(errs) < 2 * gR / w0
    assert o.tls_state()[0, 0] > 0.97


def test_tls_dipole_rate_closed_form_matches_trace():
    """-2 w0 Im(rho01) d (eq. dipole_derivative, closed form) equals Tr(rho_dot mu)."""
    rng = np.random.default_rng(2)
    M = 6
    rho0 = []
    for _ in range(M):
        p = rng.uniform(0.05, 0.95)
        a = rng.uniform(0, 2 * np.pi)
        r = rng.uniform(0, 1) * np.sqrt(p * (1 - p))
        rho0.append([p, r * np.cos(a), r * np.sin(a)])
    rho0 = np.array(rho0)
    dip = rng.standard_normal((M, 3))
    w0 = rng.uniform(0.2, 0.3, M)
    o = _tls(M, w0, dip, rho0)
    Et = rng.standard_normal((M, 3))
    o.emitters_step_prescribed(Et)
    _, md = o.emitter_io()
    for m in range(M):
        tr = o.dipole_rate_trace(m, Et[m])
        assert np.allclose(md[m], tr, rtol=1e-13, atol=1e-16)
    st = o.tls_state()
    assert np.allclose(md, (-2 * w0 * st[:, 2])[:, None] * dip, rtol=1e-14)


def test_jacobi_matches_numpy_eigh():
    rng = np.random.default_rng(4)
    for L in range(2, 7):
        A = rng.standard_normal((L, L))
        A = A + A.T
        lam, Q = jacobi_eig(A)
        assert np.allclose(np.sort(lam), np.linalg.eigvalsh(A), atol=1e-13)
        assert np.allclose(Q @ np.diag(lam) @ Q.T, A, atol=1e-13)
        assert np.allclose(Q.T @ Q, np.eye(L), atol=1e-14)


def _ml_oracle(courant, nlev, energies, mops, dip, gphi, rho0):
    o = Oracle((1, 1, 1), bc=("periodic",) * 6, courant=courant)
    n = len(nlev)
    o.add_multilevel(nlev, energies, mops, dip, gphi, rho0, np.tile([0.5, 0.5, 0.5], (n, 1)),
                     np.ones(n), np.ones(n))
    return o


def _rand_model(rng, L):
    ev = np.concatenate([[0.0, 0.25], np.sort(rng.uniform(0.3, 0.9, L - 2))])
    Mm = rng.standard_normal((L, L))
    Mm = 0.5 * (Mm + Mm.T)
    np.fill_diagonal(Mm, 0)
    A = rng.standard_normal((L, L)) + 1j * rng.standard_normal((L, L))
    rho = A @ A.conj().T
    rho /= np.trace(rho).real
    return ev, Mm, rho


def test_lindblad_pure_dephasing_closed_form():
    """E~ = 0: rho_jk(t) = rho_jk(0) exp((i(E_k - E_j) - gphi) t) for j != k, populations fixed."""
    rng = np.random.default_rng(7)
    L, g = 5, 3e-3
    ev, Mm, rho = _rand_model(rng, L)
    o = _ml_oracle(0.5, [L], [ev], [Mm], np.array([[0, 0, 0.1]]), [g], [rho])
    steps = 400
    for _ in range(steps):
        o.emitters_step_prescribed(np.zeros((1, 3)))
    t = steps * o.dt
    jj, kk = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    ref = rho * np.exp(1j * (ev[kk] - ev[jj]) * t) * np.where(jj == kk, 1.0, np.exp(-g * t))
    assert np.allclose(o.rho(0), ref, atol=1e-13)


def test_lindblad_two_level_without_dephasing_equals_tls_path():
    rng = np.random.default_rng(8)
    w0 = 0.27
    rho = np.array([[0.6, 0.3 - 0.2j], [0.3 + 0.2j, 0.4]])
    dip = np.array([[0.05, -0.02, 0.04]])
    ml = _ml_oracle(0.5, [2], [np.array([0.0, w0])], [np.array([[0, 1.0], [1.0, 0]])], dip, [0.0],
                    [rho])
    tl = _tls(1, [w0], dip, np.array([[0.4, 0.3, -0.2]]))
    for _ in range(300):
        Et = rng.standard_normal((1, 3)) * 0.8
        ml.emitters_step_prescribed(Et)
        tl.emitters_step_prescribed(Et)
    assert np.allclose(ml.rho(0), tl.rho(0), atol=1e-13)
    assert np.allclose(ml.emitter_io()[1], tl.emitter_io()[1], atol=1e-15)


def test_lindblad_state_stays_physical():
    rng = np.random.default_rng(12)
    L = 6
    ev, Mm, rho = _rand_model(rng, L)
    o = _ml_oracle(0.5, [L], [ev], [Mm], np.array([[0.2, 0.1, -0.3]]), [0.01], [rho])
    for _ in range(500):
        o.emitters_step_prescribed(rng.standard_normal((1, 3)))
        r = o.rho(0)
        assert abs(np.trace(r) - 1) < 2e-12
        assert np.allclose(r, r.conj().T, atol=1e-15)
        assert np.min(np.linalg.eigvalsh(r)) > -1e-14


def _liouvillian(H, g, L):
    """Superoperator of -i[H,.] + dephasing on row-major vec(rho)."""
    I = np.eye(L)
    Lsup = -1j * (np.kron(H, I) - np.kron(I, H.T))
    for k in range(L):
        P = np.zeros((L, L))
        P[k, k] = 1.0
        Lsup += g * (np.kron(P, P.T) - 0.5 * np.kron(P, I) - 0.5 * np.kron(I, P.T))
    return Lsup


def test_lindblad_strang_is_second_order_against_expm():
    """Static field: compare with expm of the full Liouvillian; halving dt cuts the error
    by 4 (Strang splitting of the unitary and dephasing parts)."""
    rng = np.random.default_rng(13)
    L, g = 4, 0.05
    ev, Mm, rho = _rand_model(rng, L)
    dip = np.array([[0.0, 0.0, 0.4]])
    E = np.array([[0.0, 0.0, 0.7]])
    T = 20.0
    H = np.diag(ev) - (E[0] @ dip[0]) * Mm
    exact = (scipy.linalg.expm(_liouvillian(H, g, L) * T) @ rho.ravel()).reshape(L, L)
    errs = []
    for courant in (0.5, 0.25):
        o = _ml_oracle(courant, [L], [ev], [Mm], dip, [g], [rho])
        for _ in range(int(round(T / o.dt))):
            o.emitters_step_prescribed(E)
        errs.append(np.linalg.norm(o.rho(0) - exact))
    order = np.log2(errs[0] / errs[1])
    assert 1.9 < order < 2.1, (errs, order)


def test_multilevel_dipole_rate_is_trace():
    """For the open model the oracle evaluates Tr(rho_dot mu) from the full right-hand side;
    cross-check with the closed form d^c (-i Tr(rho[M,H0]) - gphi Tr(rho M))."""
    rng = np.random.default_rng(14)
    L, g = 5, 0.02
    ev, Mm, rho = _rand_model(rng, L)
    dip = np.array([[0.1, -0.2, 0.3]])
    o = _ml_oracle(0.5, [L], [ev], [Mm], dip, [g], [rho])
    Et = np.array([[0.3, 0.1, -0.2]])
    o.emitters_step_prescribed(Et)
    r = o.rho(0)
    H0 = np.diag(ev)
    val = (-1j * np.trace(r @ (Mm @ H0 - H0 @ Mm)) - g * np.trace(r @ Mm)).real
    assert np.allclose(o.emitter_io()[1][0], val * dip[0], rtol=1e-12, atol=1e-17)


# ------------------------------------------------------- P-12 .. P-14, P-16

def _decay_run(shape, bc, cpml, pos, dip, steps, w0=0.25, state=(np.sqrt(0.9999), 0.01)):
    N = len(pos)
    o = Oracle(shape, bc=bc, cpml=cpml)
    cg, ce = state
    o.add_tls(np.array(pos), np.ones(N), np.ones(N), np.full(N, w0), np.array(dip),
              np.tile([ce * ce, cg * ce, 0.0], (N, 1)))
    o.record_populations(1)
    o.step(steps)
    P = o.populations()
    t = (np.arange(steps) + 0.5) * o.dt
    return t, P


def _rate(t, P, t_min=200.0):
    sel = t > t_min
    return -np.polyfit(t[sel], np.log(P[sel]), 1)[0]


@pytest.mark.slow
def test_superradiance_2d_matches_paper_rate():
    """2-D vacuum (z-invariant grid), TLS in the weak-excitation state (c_g, c_e) =
    (sqrt 0.9999, 0.01) (Sec. IV.A, App. B): P_e decays as exp(-N gamma t) with
    gamma = mu^2 w^2 / (2 hbar eps0 c^2) (eq. population_decay_superradiance), times the
    Gaussian kernel's form factor exp(-(w sigma)^2).  N = 1 and N = 4 collocated; the
    d/sqrt(N) rescaling of App. B gives per-emitter states identical to N = 1."""
    n, d, steps, w0, mu = 128, 16, 4000, 0.25, 0.1
    shape, bc, cp = (n, n, 1), ("cpml",) * 4 + ("periodic",) * 2, (d, d, d, d, 0, 0)
    gamma = mu ** 2 * w0 ** 2 / 2 * np.exp(-w0 ** 2)
    c = [n / 2, n / 2, 0.5]
    t, P1 = _decay_run(shape, bc, cp, [c], [[0, 0, mu]], steps)
    assert abs(_rate(t, P1[:, 0]) / gamma - 1) < 0.02
    t, P4 = _decay_run(shape, bc, cp, [c] * 4, [[0, 0, mu]] * 4, steps)
    for q in range(4):
        assert abs(_rate(t, P4[:, q]) / (4 * gamma) - 1) < 0.02
    t, P4s = _decay_run(shape, bc, cp, [c] * 4, [[0, 0, mu / 2]] * 4, steps)
    for q in range(4):
        assert np.max(np.abs(P4s[:, q] - P1[:, 0])) < 1e-13 * np.max(P1)


@pytest.mark.slow
def test_fermi_golden_rule_decay_3d():
    """3-D free space: Gamma = w0^3 d^2 / (3 pi) exp(-(w0 sigma)^2) (textbook spontaneous
    emission rate with the Gaussian form factor), within grid dispersion and PML error."""
    n, cp, steps, w0, mu = 48, 12, 5000, 0.25, 0.2
    G = w0 ** 3 * mu ** 2 / (3 * np.pi) * np.exp(-w0 ** 2)
    t, P = _decay_run((n, n, n), ("cpml",) * 6, (cp,) * 6, [[n / 2] * 3], [[0, 0, mu]], steps)
    assert abs(_rate(t, P[:, 0]) / G - 1) < 0.03


@pytest.mark.slow
def test_superradiance_3d_n_fold():
    """3-D free space, N = 4 collocated TLS in the weak-excitation state of Sec. IV.A: the
    emitters share one field and radiate as one dipole of N times the moment, so each
    population decays at N times the single-emitter golden-rule rate of the test above."""
    n, cp, steps, w0, mu, N = 48, 12, 5000, 0.25, 0.1, 4
    G = w0 ** 3 * mu ** 2 / (3 * np.pi) * np.exp(-w0 ** 2)
    t, P = _decay_run((n, n, n), ("cpml",) * 6, (cp,) * 6, [[n / 2] * 3] * N,
                      [[0, 0, mu]] * N, steps)
    for q in range(N):
        assert abs(_rate(t, P[:, q]) / (N * G) - 1) < 0.03


def test_excited_state_is_stationary():
    """|e> has rho01 = 0, so mu_dot = 0 and nothing is ever emitted (semiclassical): the
    probe stays exactly zero and the population stays 1 up to rounding."""
    o = Oracle((32, 32, 32))
    o.add_tls(np.array([[16.0, 16.0, 16.0]]), [1.0], [1.0], [0.25], np.array([[0, 0, 0.01]]),
              np.array([[1.0, 0.0, 0.0]]))
    pid = o.add_probe(2, (24, 16, 16))
    o.record_populations(1)
    o.step(200)
    assert np.all(o.probe(pid) == 0.0)
    assert np.max(np.abs(o.populations() - 1.0)) < 200 * 5e-16


def test_coupled_energy_stays_bounded():
    """Field energy W^n plus emitter energy Tr(rho H0) drifts only at O(dt^2) in a PEC box."""
    n = 20
    o = Oracle((n, n, n))
    o.add_tls(np.array([[10.0, 10.0, 10.0]]), [1.0], [1.0], [0.25], np.array([[0, 0, 0.3]]),
              np.array([[0.5, 0.5, 0.0]]))
    o.record_energy(True)
    o.record_populations(1)
    o.step(3000)
    W = o.energy_series()
    P = o.populations()[:, 0]
    emit = 0.25 * P                         # Tr(rho^{n+1/2} H0)
    Pm = np.concatenate([[0.5], P[:-1]])    # rho^{n-1/2}
    tot = W + 0.25 * 0.5 * (P + Pm)
    exchanged = np.max(W) - np.min(W)
    assert exchanged > 1e-3 * 0.25
    assert np.max(np.abs(tot - tot[0])) < 0.05 * exchanged
    assert np.isfinite(emit).all()


def test_flux_is_the_energy_flow_through_the_plane():
    """Summation by parts of the Yee updates (PEC walls, no current above the plane)
    gives exact energy balances for the part of the box above plane k0:
      region A = every component with index >= k0:
        W_A^{n+1} - W_A^n = dt sum [Ebar_x(k0) H_y(k0-1) - Ebar_y(k0) H_x(k0-1)]
      region B = Ex, Ey, Hz with index >= k0+1 and Ez, Hx, Hy with index >= k0:
        W_B^{n+1} - W_B^n = dt sum [Ebar_x(k0) H_y(k0) - Ebar_y(k0) H_x(k0)]
    with Ebar = (E^n + E^{n+1})/2, H = H^{n+1/2} and W^n = 1/2 sum eps E^n.E^n +
    1/2 sum H^{n+1/2}.H^{n-1/2} over the region.  Their mean is dt times the time-centred
    flux with the z-averaged H, so the flux detector must equal it exactly."""
    nx, ny, nz, k0, steps = 12, 10, 24, 15, 160
    rng = np.random.default_rng(21)
    o = Oracle((nx, ny, nz))
    eps = np.ones((nz, ny, nx))
    eps[:k0 - 2] = rng.uniform(1.0, 3.0, (k0 - 2, ny, nx))
    o.set_eps(eps)
    o.add_point_source(2, (5, 4, 6), 1.0, 0.4, 4.0, 15.0)
    o.add_point_source(0, (7, 5, 8), -0.6, 0.3, 5.0, 20.0)
    o.add_flux_plane(2, k0)
    states = []
    for n in range(steps + 2):
        states.append([o.get_field(c).copy() for c in range(6)])
        o.step(1)
    F = o.flux_series()

    def energy(n, lo):
        # lo[c]: first z index of component c (Ex, Ey, Ez, Hx, Hy, Hz) in the region
        En, Hm, Hp = states[n][:3], states[n][3:], states[n + 1][3:]
        w = 0.0
        for c in range(3):
            w += 0.5 * np.sum(eps[lo[c]:] * En[c][lo[c]:] ** 2)
            w += 0.5 * np.sum(Hp[c][lo[3 + c]:] * Hm[c][lo[3 + c]:])
        return w

    A = (k0, k0, k0, k0, k0, k0)
    B = (k0 + 1, k0 + 1, k0, k0, k0, k0 + 1)
    dA = np.array([energy(n + 1, A) - energy(n, A) for n in range(steps)])
    dB = np.array([energy(n + 1, B) - energy(n, B) for n in range(steps)])
    dt = 0.5
    scale = np.max(np.abs(dA)) + np.max(np.abs(dB))
    assert scale > 0
    assert np.max(np.abs(0.5 * (dA + dB) - dt * F[:steps])) <= 1e-12 * scale
    # a wrong half-plane (only one side of the average) is caught
    assert np.max(np.abs(dA - dt * F[:steps])) > 1e-6 * scale


# --------------------------------------------------------------- single-mode cavity
def _cavity_run(o, steps):
    out = np.empty((steps + 1, 6))
    out[0] = o.cavity()
    with _one_thread():
        for n in range(steps):
            o.step(1)
            out[n + 1] = o.cavity()
    return out


def test_cavity_free_mode_is_the_leapfrog_oscillator():
    """No emitters: the mode is a leapfrog oscillator, q^n = cos(n theta) for x and
    0.5 sin(n theta) for y exactly, sin(theta/2) = w dt / 2, given the matching p^{-1/2}."""
    o = Oracle((1, 1, 1), bc=("periodic",) * 6)
    w, dt = 0.3, o.dt
    th = 2.0 * np.arcsin(w * dt / 2.0)
    # q^1 = q^0 + dt (p^{-1/2} - dt w^2 q^0) must equal cos(theta), resp. 0.5 sin(theta)
    p0 = ((np.cos(th) - 1.0) / dt + dt * w * w, 0.5 * np.sin(th) / dt)
    o.set_cavity(w, 7.0, q0=(1.0, 0.0), p0=p0)
    tr = _cavity_run(o, 500)
    n = np.arange(501)
    assert np.max(np.abs(tr[:, 0] - np.cos(n * th))) < 1e-12
    assert np.max(np.abs(tr[:, 1] - 0.5 * np.sin(n * th))) < 1e-12
    assert np.all(tr[:, 4:] == 0.0)
    with pytest.raises(ValueError):
        Oracle((1, 1, 1), bc=("periodic",) * 6).set_cavity(0.0, 1.0)


def _polariton_trace(n_emit, d, w, w0, V, A, T, courant=0.05):
    o = Oracle((1, 1, 1), bc=("periodic",) * 6, courant=courant)
    o.add_tls(np.tile([0.5, 0.5, 0.5], (n_emit, 1)), np.ones(n_emit), np.ones(n_emit),
              np.full(n_emit, w0), np.tile([d, 0.0, 0.0], (n_emit, 1)),
              np.zeros((n_emit, 3)))
    th = 2.0 * np.arcsin(w * o.dt / 2.0)
    o.set_cavity(w, V, q0=(A, 0.5), p0=(0.0, (np.cos(th) - 1.0) / o.dt * 0.5 + o.dt * w * w * 0.5))
    steps = int(round(T / o.dt))
    return o.dt, th, _cavity_run(o, steps)


def _fit_residual(t, y, freqs):
    B = np.concatenate([np.stack([np.cos(f * t), np.sin(f * t)], 1) for f in freqs], 1)
    c, *_ = np.linalg.lstsq(B, y, rcond=None)
    return np.linalg.norm(B @ c - y) / np.linalg.norm(y)


def test_cavity_vacuum_rabi_splitting_linear_response():
    """Weakly driven TLS in the mode (Sec. II.A.2 coupling with the dipole self-energy):
    the linearised pair q'' = -w^2 q - eps mu, mu'' = -w0^2 mu - 2 w0 d^2 (eps q + mu / V)
    (a TLS ground state has polarisability 2 d^2 / w0) oscillates at the two normal-mode
    frequencies.  q_x must be a sum of exactly those two; dropping the self-energy or
    flipping the sign of the dipole's force on the mode gives other frequencies, which the
    fit then misses."""
    w = w0 = 0.25
    d, V, A, T = 0.05, 1.0, 0.01, 1200.0
    dt, th, tr = _polariton_trace(1, d, w, w0, V, A, T)
    t = np.arange(tr.shape[0]) * dt
    eps = w / np.sqrt(V)

    def normal_modes(self_term=1.0, back_action=1.0):
        K = np.array([[w * w, back_action * eps],
                      [2 * w0 * d * d * eps, w0 * w0 + self_term * 2 * w0 * d * d / V]])
        return np.sqrt(np.linalg.eigvals(K).real)

    ref = normal_modes()
    split = abs(ref[1] - ref[0])
    assert split > 0.02  # well resolved within T
    assert _fit_residual(t, tr[:, 0], ref) < 5e-3
    assert _fit_residual(t, tr[:, 0], normal_modes(self_term=0.0)) > 0.1
    assert _fit_residual(t, tr[:, 0], normal_modes(back_action=-1.0)) > 0.1
    assert _fit_residual(t, tr[:, 0], [w]) > 0.1
    # the y polarisation does not see an x dipole: it stays the free leapfrog oscillator
    n = np.arange(tr.shape[0])
    assert np.max(np.abs(tr[:, 1] - 0.5 * np.cos(n * th))) < 1e-12
    assert np.all(tr[:, 5] == 0.0)


def test_cavity_collective_coupling_sums_the_dipoles():
    """N identical emitters of dipole d / sqrt(N) have the polarisability of one of dipole
    d, so in linear response the mode cannot tell them apart (the total dipole sums over
    emitters); they differ only at second order in the excitation."""
    w, w0, d, V, A, T = 0.25, 0.25, 0.05, 1.0, 0.01, 300.0
    _, _, one = _polariton_trace(1, d, w, w0, V, A, T)
    _, _, four = _polariton_trace(4, d / 2.0, w, w0, V, A, T)
    _, _, four_full = _polariton_trace(4, d, w, w0, V, A, T)
    scale = np.max(np.abs(one[:, 0]))
    assert np.max(np.abs(four[:, 0] - one[:, 0])) < 1e-3 * scale
    assert np.max(np.abs(four[:, 4] - one[:, 4])) < 1e-3 * np.max(np.abs(one[:, 4]))
    assert np.max(np.abs(four_full[:, 0] - one[:, 0])) > 0.1 * scale


_CAV_W, _CAV_V = 0.25, 1.0
_TLS_D = np.array([[0.15, 0.05, 0.0], [-0.04, 0.12, 0.0]])
_TLS_W0 = np.array([0.25, 0.3])
_TLS_RHO0 = np.array([[0.5, 0.5, 0.0], [0.2, 0.3, 0.25]])
_ML_M = np.array([[0.0, 1.0, 0.4], [1.0, 0.0, -0.7], [0.4, -0.7, 0.0]])
_ML_D = np.array([[0.08, 0.1, 0.0]])


def _cavity_ensemble(courant, multilevel=True, tls_rho0=_TLS_RHO0, q0=(0.02, -0.01),
                     p0=(0.0, 0.003)):
    """Two two-level emitters (and a three-level one) in superposition states, strongly
    coupled to the mode through x and y dipoles."""
    o = Oracle((1, 1, 1), bc=("periodic",) * 6, courant=courant)
    o.add_tls(np.tile([0.5, 0.5, 0.5], (2, 1)), np.ones(2), np.ones(2), _TLS_W0, _TLS_D,
              tls_rho0)
    if multilevel:
        psi = np.array([0.7, 0.5, 0.5j])
        psi /= np.linalg.norm(psi)
        o.add_multilevel([3], [np.array([0.0, 0.27, 0.45])], [_ML_M], _ML_D, [2e-3],
                         [np.outer(psi, psi.conj())], np.array([[0.5, 0.5, 0.5]]), [1.0], [1.0])
    o.set_cavity(_CAV_W, _CAV_V, q0=q0, p0=p0)
    return o


def _tls_mu(st):
    """<mu> of the two-level emitters: Tr(rho sigma_x) d = 2 Re rho01 d."""
    return (2.0 * st[:2, 1])[:, None] * _TLS_D


def _total_dipole_from_states(o):
    """sum_m <mu^(m)> written out here: two-level emitters as above, Tr(rho M) d for the
    three-level one (mu = d M)."""
    tot = _tls_mu(o.tls_state()).sum(0)
    if o.num_emitters > 2:
        tot = tot + np.real(np.trace(o.rho(2) @ _ML_M)) * _ML_D[0]
    return tot[:2]


def test_cavity_total_dipole_tracks_the_expectation_values_at_second_order():
    """The mode's total dipole d^n (eq. dklambda_def) stands for sum_m <mu^(m)> at the
    integer time t_n, between the states at t_{n-1/2} and t_{n+1/2}: its distance from
    the midpoint of those two sums shrinks as dt^2 (measured order 2 +- 0.1).  A bare
    sum at t_{n-1/2} (half a step behind) would be first order."""
    T = 120.0
    gaps = []
    with _one_thread():
        for courant in (0.4, 0.2, 0.1, 0.05):
            o = _cavity_ensemble(courant)
            steps = int(round(T / o.dt))
            D = [_total_dipole_from_states(o)]  # at t_{-1/2}
            d = [o.cavity()[4:6]]                # at t_0
            for _ in range(steps):
                o.step(1)
                D.append(_total_dipole_from_states(o))
                d.append(o.cavity()[4:6])
            D, d = np.array(D), np.array(d)
            mid = 0.5 * (D[:-1] + D[1:])
            gaps.append(np.max(np.abs(d[:-1] - mid)) / np.max(np.abs(D)))
    gaps = np.array(gaps)
    assert gaps[0] < 1e-2
    orders = np.log2(gaps[:-1] / gaps[1:])
    assert np.all(np.abs(orders - 2.0) < 0.1), orders


def test_cavity_coupled_trajectory_converges_at_second_order():
    """Mode and two-level emitters from one continuous initial condition at t = 0 (q, q' = 0,
    rho): the discrete data are placed where the scheme keeps them, p^{-1/2} by a
    half-step Taylor term and rho^{-1/2} by the exact propagator over -dt/2 in the field
    E~(0) = -(eps q + d / V), written out here with scipy's expm.  Then q and d at
    T = 120 (integer-time quantities) converge with dt at second order: successive
    Richardson differences fall by 4 (order 2 +- 0.1)."""
    T, q0 = 120.0, np.array([0.02, -0.01])
    eps = _CAV_W / np.sqrt(_CAV_V)
    d0 = _tls_mu(_TLS_RHO0).sum(0)[:2]
    E0 = -(eps * q0 + d0 / _CAV_V)
    finals = []
    with _one_thread():
        for courant in (0.4, 0.2, 0.1, 0.05):
            dt = courant
            rho_half = []
            for m in range(2):
                rho11, re01, im01 = _TLS_RHO0[m]
                r01 = re01 + 1j * im01
                rho = np.array([[1 - rho11, r01], [np.conj(r01), rho11]])
                g = E0 @ _TLS_D[m, :2]
                H = np.array([[0.0, -g], [-g, _TLS_W0[m]]])
                U = scipy.linalg.expm(1j * H * dt / 2)  # exp(-i H (-dt/2))
                r = U @ rho @ U.conj().T
                rho_half.append([r[1, 1].real, r[0, 1].real, r[0, 1].imag])
            p_half = 0.5 * dt * (_CAV_W ** 2 * q0 + eps * d0)
            o = _cavity_ensemble(courant, multilevel=False, tls_rho0=np.array(rho_half),
                                 q0=tuple(q0), p0=tuple(p_half))
            o.step(int(round(T / o.dt)))
            c = o.cavity()
            finals.append(np.concatenate([c[:2], c[4:6]]))  # q^N and d^N, both at t = T
    F = np.array(finals)
    diffs = np.array([np.max(np.abs(F[i] - F[i + 1])) for i in range(3)])
    rich = np.log2(diffs[:-1] / diffs[1:])
    assert np.all(np.abs(rich - 2.0) < 0.1), rich


# --------------------------------------------------------------- dispersive poles
def _uniform_pole_run(drude, w0, gamma, sigma, einf, steps):
    o = Oracle((2, 2, 2), bc=("periodic",) * 6)
    o.set_eps(np.full((2, 2, 2), einf))
    o.add_susceptibility((0, 0, 0, 2, 2, 2), w0, gamma, sigma, drude=drude)
    E0 = np.array([0.7, -0.3, 1.1])
    for c in range(3):
        o.set_field(c, np.full((2, 2, 2), E0[c]))
    tr = np.empty((steps + 1, 3))
    tr[0] = E0
    for n in range(steps):
        o.step(1)
        tr[n + 1] = [o.get_field(c)[1, 0, 1] for c in range(3)]
    return o.dt, E0, tr


@pytest.mark.parametrize("drude,gamma", [(False, 0.0), (False, 0.05), (True, 0.0), (True, 0.08)])
def test_pole_uniform_field_closed_form(drude, gamma):
    """Uniform field, no curl: D = eps_inf E + P is conserved, so E relaxes to the static
    value D / eps(0) (eps(0) = eps_inf + sigma for a Lorentz pole, infinite for Drude:
    E -> 0) through the two roots r of (1 + g) r^2 - (2 - (kappa + sigma / eps_inf) w0^2
    dt^2) r + (1 - g) = 0, g = gamma dt / 2 -- the plasma / longitudinal oscillation."""
    w0, sigma, einf, steps = 0.4, 1.5, 2.0, 400
    dt, E0, tr = _uniform_pole_run(drude, w0, gamma, sigma, einf, steps)
    kappa = 0.0 if drude else 1.0
    g = gamma * dt / 2
    r = np.roots([1 + g, -(2 - (kappa + sigma / einf) * w0 ** 2 * dt ** 2), 1 - g])
    Einf = np.zeros(3) if drude else E0 * einf / (einf + sigma)
    n = np.arange(steps + 1)
    B = np.stack([r[0] ** n, r[1] ** n], 1)
    for c in range(3):
        y = tr[:, c] - Einf[c]
        coef, *_ = np.linalg.lstsq(B, y.astype(complex), rcond=None)
        assert np.max(np.abs(B @ coef - y)) < 1e-12 * np.max(np.abs(y))
    if gamma > 0:
        # loss: the transient dies at the rate |r|^2 = (1 - g) / (1 + g) per step
        assert np.allclose(np.abs(r) ** 2, (1 - g) / (1 + g), rtol=1e-12)
        assert np.max(np.abs(tr[-1] - Einf)) < 0.05 * np.max(np.abs(E0))


def test_pole_plane_wave_discrete_dispersion():
    """A lossless Lorentz medium filling a periodic box: a standing wave of wavenumber k
    oscillates at exactly the two polariton branches of the discrete dispersion relation
    u (eps_inf + sigma w0^2 / (w0^2 - u)) = (4 / dx^2) sum sin^2(k_a dx / 2),
    u = (4 / dt^2) sin^2(w dt / 2); a 1% error in w0 misses them."""
    n, w0, sigma, einf = 16, 0.5, 2.0, 1.5
    o = Oracle((n, 2, 2), bc=("periodic",) * 6)
    o.set_eps(np.full((2, 2, n), einf))
    o.add_susceptibility((0, 0, 0, n, 2, 2), w0, 0.0, sigma)
    kx = 2 * np.pi * 3 / n
    x = np.arange(n)
    o.set_field(2, np.broadcast_to(np.cos(kx * x), (2, 2, n)).copy())  # Ez at integer x
    steps = 1500
    y = np.empty(steps + 1)
    y[0] = 1.0
    for q in range(steps):
        o.step(1)
        y[q + 1] = o.get_field(2)[0, 0, 0]
    dt = o.dt
    K = 4 * np.sin(kx / 2) ** 2

    def branches(w):
        u = np.roots([-einf, einf * w * w + sigma * w * w + K, -K * w * w]).real
        return 2 / dt * np.arcsin(dt * np.sqrt(u) / 2)

    t = np.arange(steps + 1) * dt

    def resid(freqs):
        B = np.concatenate([np.stack([np.cos(f * t), np.sin(f * t)], 1) for f in freqs], 1)
        c, *_ = np.linalg.lstsq(B, y, rcond=None)
        return np.linalg.norm(B @ c - y) / np.linalg.norm(y)

    assert resid(branches(w0)) < 1e-10
    assert resid(branches(1.01 * w0)) > 1e-3


# ------------------------------------------------------ classical path, travelling pulse

def _wave_tls(zs, courant=0.5):
    o = Oracle((1, 1, 1), bc=("periodic",) * 6, courant=courant)
    n = len(zs)
    pos = np.column_stack([np.full(n, 0.5), np.full(n, 0.5), zs])
    o.add_tls(pos, np.ones(n), np.linspace(0.8, 1.2, n), np.full(n, 0.25),
              np.tile([0.03, -0.02, 0.08], (n, 1)), np.tile([0.0, 0.0, 0.0], (n, 1)))
    return o


def test_travelling_pulse_depends_on_z_minus_ct():
    """eq. E_analytical: the field is a function of z - ct.  An emitter L cells further
    along z that starts L time units later goes through exactly the same states."""
    pulse = dict(pol=[0.2, 0.3, 0.9], amp=0.8, omega=0.25, tau=40.0, t0=150.0, z0=1.0)
    a, b = _wave_tls([3.0]), _wave_tls([10.0])
    L = 7.0
    for q in range(500):
        t = q * a.dt
        a.emitters_step_wave(t=t, **pulse)
        b.emitters_step_wave(t=t + L, **pulse)
        if q % 50 == 0:
            assert np.array_equal(a.tls_state(), b.tls_state())
    assert np.max(a.tls_state()[:, 0]) > 1e-4  # the pulse did drive the emitter


def test_travelling_pulse_is_the_prescribed_field_it_names():
    """The pulse step equals the generic prescribed-field step fed with the field written
    out here: gamma amp cos(omega (u - t0)) exp(-(u - t0)^2 / 2 tau^2) pol at
    u = t - (z - z0) (the Gaussian pulse of App. B moving along +z)."""
    zs = np.array([2.0, 5.5, 9.25])
    gam = np.linspace(0.8, 1.2, 3)
    pol = np.array([0.2, 0.3, 0.9])
    amp, om, tau, t0, z0 = 0.8, 0.25, 40.0, 150.0, 1.0
    a, b = _wave_tls(zs), _wave_tls(zs)
    for q in range(300):
        t = q * a.dt
        a.emitters_step_wave(pol, amp, om, tau, t0, z0, t)
        u = t - (zs - z0) - t0
        f = gam * amp * np.cos(om * u) * np.exp(-u ** 2 / (2 * tau ** 2))
        b.emitters_step_prescribed(f[:, None] * pol[None, :])
    assert np.max(np.abs(a.tls_state() - b.tls_state())) < 1e-15
