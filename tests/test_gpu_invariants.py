"""Invariants of the method checked on the GPU fields themselves: the discrete field
energy W^n (Poynting's theorem on the Yee grid, eq. Maxwell) recorded by the library
against the oracle's and conserved without currents; and the discrete charge identity
div(eps E^n) = -dt sum_k div J^{k+1/2} (eqs. Maxwell and J_mol) on the library's E, with
J formed outside the library: the analytic source currents plus the oracle's scatter
(pinned by its own tests) of the dipole rates the library reports each step."""
import numpy as np
import pytest

from oracle.feed import build_oracle
from paper_2512_06173_amd import workloads as W

pytestmark = pytest.mark.gpu


def mlk():
    from paper_2512_06173_amd import mlk as m
    return m


def say(msg):
    print(msg, flush=True)


def random_state(n, bc, rng):
    E = [rng.standard_normal((n, n, n)) for _ in range(3)]
    H = [rng.standard_normal((n, n, n)) for _ in range(3)]
    if bc == "pec":  # tangential E on the index-0 wall planes is zero
        E[0][0, :, :] = 0; E[0][:, 0, :] = 0
        E[1][0, :, :] = 0; E[1][:, :, 0] = 0
        E[2][:, 0, :] = 0; E[2][:, :, 0] = 0
    return E, H


@pytest.mark.parametrize("bc", ["pec", "periodic"])
def test_energy_is_conserved_over_ten_thousand_steps_fp64(bc):
    """No currents, sources or layers: W^n is invariant for any eps and initial data; the
    FP64 drift over 10^4 steps stays at rounding."""
    n, steps = 32, 10000
    rng = np.random.default_rng(21)
    s = mlk().Simulation((n, n, n), bc=(bc,) * 6, precision="fp64")
    s.set_eps(rng.uniform(1.0, 4.0, (n, n, n)))
    E, H = random_state(n, bc, rng)
    for c in range(3):
        s.set_field(c, E[c])
        s.set_field(3 + c, H[c])
    s.record_energy(1)
    s.step(steps)
    Wn = s.energy_series()
    assert Wn.size == steps
    drift = np.max(np.abs(Wn - Wn[0])) / abs(Wn[0])
    say(f"[energy] {bc} 32^3, {steps} steps: drift {drift:.2e}")
    assert drift <= 1e-12


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_energy_series_matches_the_oracle(precision, tol):
    """With emitters, a point source, a dielectric and CPML the energy changes; the
    library's W^n (every step, and every third step) follows the oracle's."""
    w = W.radiating_cube(n=36, n_emit=60, steps=0, cpml=6, precision=precision)
    rng = np.random.default_rng(4)
    w.eps = rng.uniform(1.0, 2.5, (36, 36, 36))
    w.point_sources = [W.PointSource(1, (18, 17, 16), 1.0, 0.3, 5.0, 15.0)]
    steps = 90
    ora = build_oracle(w)
    ora.record_energy(True)
    ora.step(steps)
    ref = ora.energy_series()
    for every in (1, 3):
        s = mlk().from_workload(w)
        s.record_energy(every)
        s.step(steps)
        got = s.energy_series()
        r = ref[::every]
        assert got.shape == r.shape
        err = np.max(np.abs(got - r)) / np.max(np.abs(r))
        say(f"[energy] {precision} every {every}: max rel {err:.2e}")
        assert err <= tol


def test_energy_detector_needs_the_fused_sweep():
    s = mlk().Simulation((16, 16, 16), sweep="plain")
    with pytest.raises(mlk().MlkError) as e:
        s.record_energy(1)
    assert e.value.status == 5  # MLK_EUNSUPPORTED


def _div(F):
    return (F[0] - np.roll(F[0], 1, axis=2)) + (F[1] - np.roll(F[1], 1, axis=1)) + \
           (F[2] - np.roll(F[2], 1, axis=0))


@pytest.mark.parametrize("bc,dx", [("pec", 1.0), ("periodic", 1.0), ("pec", 0.5)])
def test_charge_identity_on_the_gpu_fields(bc, dx):
    n, steps, S = 20, 50, 0.5
    rng = np.random.default_rng(9)
    eps = rng.uniform(1.0, 3.0, (n, n, n))
    tls = W.TLSSet(pos=np.array([[9.3, 10.1, 9.7], [10.6, 9.2, 10.4], [10.0, 10.0, 10.0]]),
                   sigma=np.array([1.0, 0.8, 1.1]), gamma=np.array([1.0, 0.5, 1.5]),
                   omega0=np.array([0.25, 0.3, 0.2]),
                   dipole=np.array([[0.3, -0.2, 0.4], [0.0, 0.5, 0.1], [0.2, 0.2, -0.3]]),
                   rho0=np.tile([0.5, 0.5, 0.0], (3, 1)))
    pt = W.PointSource(1, (6, 11, 8), 0.7, 0.3, 6.0, 15.0)
    sheet = W.PlaneSource(axis=1, index=5, comp=1, amp=0.3, omega=0.2, tau=5.0, t0=12.0)
    w = W.Workload(name="charge", shape=(n, n, n), bc=(bc,) * 6, dx=dx, eps=eps, tls=tls,
                   point_sources=[pt], plane_sources=[sheet], steps=steps, precision="fp64")
    sim = mlk().from_workload(w)
    ora = build_oracle(w)  # its scatter only

    def pulse(t, a, om, ta, tc):
        return a * np.cos(om * (t - tc)) * np.exp(-(t - tc) ** 2 / (2 * ta ** 2))

    dt = S * dx
    Jsum = [np.zeros((n, n, n)) for _ in range(3)]
    for q in range(steps):
        sim.step(1)
        _, md = sim.emitter_io()
        J = ora.scatter(md)
        t = (q + 0.5) * dt
        J[1][8, 11, 6] += pulse(t, pt.amp, pt.omega, pt.tau, pt.t0) / dx ** 3
        J[1][:, 5, :] += pulse(t, sheet.amp, sheet.omega, sheet.tau, sheet.t0) / dx
        for c in range(3):
            Jsum[c] += J[c]
    E = sim.fields()[:3]
    lhs = _div([eps * e for e in E])
    rhs = -dt * _div(Jsum)
    inner = (slice(1, n - 1),) * 3 if bc == "pec" else (slice(None),) * 3
    scale = np.max(np.abs(rhs[inner]))
    err = np.max(np.abs(lhs[inner] - rhs[inner])) / scale
    say(f"[charge] {bc} dx {dx}: {err:.2e} of {scale:.2e}")
    assert scale > 1e-6
    assert err <= 1e-12
