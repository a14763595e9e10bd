"""Classical-path (prescribed-field) stepping (eq. E_analytical, the prescribed-field
solver of the paper's table of EM solvers): every emitter advanced under a given field,
with no grid and no back-action, against the oracle's prescribed-field step and the
closed-form static-field Rabi oscillation."""
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


def mixed(precision, seed=5):
    """Two-level emitters (ids first) and 2-6 level Lindblad emitters in a small Bragg
    stack; the grid is not used by the prescribed steps."""
    w = W.bragg(nx=16, ny=16, nz=112, n_emit=10, steps=0, pairs_per_mirror=3,
                precision=precision, seed=seed)
    ml = w.multilevel
    ml.dipole = ml.dipole * 20.0
    ml.gphi = np.full(len(ml), 2e-3)
    rng = np.random.default_rng(seed)
    zc = ml.pos[:, 2].mean()
    Mt = 7
    pos = np.column_stack([rng.uniform(0, 16, Mt), rng.uniform(0, 16, Mt),
                           rng.uniform(zc - 5, zc + 5, Mt)])
    w.tls = W.TLSSet(pos=pos, sigma=np.ones(Mt), gamma=np.ones(Mt),
                     omega0=rng.uniform(0.24, 0.26, Mt), dipole=0.3 * rng.standard_normal((Mt, 3)),
                     rho0=np.tile([0.2, 0.4, 0.0], (Mt, 1)))
    return w, Mt


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_prescribed_steps_match_the_oracle(precision):
    """40 steps under a random field sequence: every state after every step (two-level,
    recorded) and at the end (multilevel), and the last mu_dot, against the oracle's
    prescribed-field step.  The emitter arithmetic is FP64 in both precisions."""
    w, Mt = mixed(precision)
    sim = mlk().from_workload(w)
    ora = build_oracle(w)
    M = len(sim.nlev)
    rng = np.random.default_rng(17)
    Et = 0.05 * rng.standard_normal((40, M, 3))
    rec = sim.step_prescribed(Et, record=True)
    assert rec.shape == (40, Mt, 3)
    ref = np.zeros_like(rec)
    for q in range(40):
        ora.emitters_step_prescribed(Et[q])
        ref[q] = ora.tls_state()[:Mt]
    e_tls = np.max(np.abs(rec - ref))
    e_ml = max(np.max(np.abs(sim.rho(m) - ora.rho(m))) for m in range(Mt, M))
    et_g, md_g = sim.emitter_io()
    et_o, md_o = ora.emitter_io()
    e_md = np.max(np.abs(md_g - md_o)) / np.max(np.abs(md_o))
    say(f"[prescribed] {precision}: tls {e_tls:.2e}, multilevel {e_ml:.2e}, mu_dot {e_md:.2e}")
    assert np.array_equal(et_g, Et[-1])
    assert e_tls <= 1e-13 and e_ml <= 1e-13 and e_md <= 1e-12
    assert sim.step_count == 0  # no grid step was taken
    assert all(np.count_nonzero(f) == 0 for f in sim.fields())


def test_prescribed_static_field_rabi_closed_form():
    """From the ground state under a static field E0: P_e(t) = (4g^2/(w0^2 + 4g^2))
    sin^2(sqrt(w0^2 + 4g^2) t / 2), g = E0 . d, exact for the two-level propagator."""
    w0, E0 = 0.25, 0.3
    d = np.array([[0.0, 0.0, 0.5], [0.3, 0.2, 0.0], [0.0, 0.2, 0.1]])
    w = W.Workload(name="rabi", shape=(16, 16, 16), steps=0, precision="fp64",
                   tls=W.TLSSet(pos=np.full((3, 3), 8.0), sigma=np.ones(3), gamma=np.ones(3),
                                omega0=np.full(3, w0), dipole=d,
                                rho0=np.tile([0.0, 0.0, 0.0], (3, 1))))
    sim = mlk().from_workload(w)
    nsteps = 2000
    field = np.array([0.0, E0 / 3, E0])
    rec = sim.step_prescribed(np.tile(field, (nsteps, 3, 1)), record=True)
    t = (np.arange(nsteps) + 1) * sim.dt
    for m in range(3):
        g = field @ d[m]
        W2 = w0 ** 2 + 4 * g ** 2
        pe = 4 * g ** 2 / W2 * np.sin(np.sqrt(W2) * t / 2) ** 2
        err = np.max(np.abs(rec[:, m, 0] - pe))
        say(f"  emitter {m}: g = {g:.3f}, max |P_e - closed form| = {err:.2e}")
        assert err <= 1e-12


def test_prescribed_from_device_memory_and_errors():
    """A device-resident field sequence gives the same states as a host one; bad calls
    are rejected."""
    import ctypes as C
    import torch
    w, Mt = mixed("fp64", seed=6)
    a = mlk().from_workload(w)
    b = mlk().from_workload(w)
    M = len(a.nlev)
    Et = 0.04 * np.random.default_rng(3).standard_normal((25, M, 3))
    a.step_prescribed(Et)
    dev = torch.tensor(Et, dtype=torch.float64, device="cuda").contiguous()
    out = torch.zeros((25, Mt, 3), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()  # the library works on a stream of its own
    L = mlk().lib()
    mlk()._check(L.mlk_step_prescribed(b._h, 25, C.c_void_p(dev.data_ptr()), mlk().MEM_DEVICE,
                                       C.c_void_p(out.data_ptr())))
    b.sync()
    assert np.array_equal(a.tls_state(0, Mt), b.tls_state(0, Mt))
    assert np.array_equal(out[-1].cpu().numpy(), b.tls_state(0, Mt))
    for m in range(Mt, M):
        assert np.array_equal(a.rho(m), b.rho(m))
    with pytest.raises(mlk().MlkError):
        mlk()._check(L.mlk_step_prescribed(a._h, -1, None, mlk().MEM_HOST, None))
    with pytest.raises(mlk().MlkError):
        mlk()._check(L.mlk_step_prescribed(a._h, 3, None, mlk().MEM_HOST, None))
    with pytest.raises(mlk().MlkError):
        mlk()._check(L.mlk_step_prescribed(a._h, 1, C.c_void_p(dev.data_ptr()), 7, None))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_travelling_pulse_on_the_device_matches_the_oracle(precision):
    """eq. E_analytical evaluated on the device for two-level and multilevel emitters at
    different heights: every recorded two-level state and the final multilevel states
    against the oracle's pulse step (the emitter states are FP64 in both modes)."""
    from oracle.oracle import Oracle
    from paper_2512_06173_amd import workloads as W
    rng = np.random.default_rng(17)
    n_tls, n_ml = 40, 12
    pos_t = np.column_stack([rng.uniform(0, 16, n_tls), rng.uniform(0, 16, n_tls),
                             rng.uniform(0, 16, n_tls)])
    tls = W.tls_ensemble(rng, n_tls, 0.0, 16.0, "superposition")
    tls.pos = pos_t
    ml = W.random_multilevel(rng, n_ml, rng.uniform(0.0, 16.0, (n_ml, 3)), dmag=0.05)
    sim = mlk().Simulation((16, 16, 16), bc=("periodic",) * 6, precision=precision)
    ora = Oracle((16, 16, 16), bc=("periodic",) * 6)
    for o in (sim, ora):
        o.add_tls(tls.pos, tls.sigma, tls.gamma, tls.omega0, tls.dipole, tls.rho0)
        o.add_multilevel(ml.nlev, ml.energies, ml.mop, ml.dipole, ml.gphi, ml.rho0, ml.pos,
                         ml.sigma, ml.gamma)
    pulse = dict(pol=[0.3, -0.2, 0.9], amp=2.0, omega=0.25, tau=20.0, t0=60.0, z0=2.0)
    steps = 300
    rec = sim.step_wave(steps, t_start=1.5, record=True, **pulse)
    worst = 0.0
    for q in range(steps):
        ora.emitters_step_wave(t=1.5 + q * ora.dt, **pulse)
        worst = max(worst, np.max(np.abs(rec[q] - ora.tls_state()[:n_tls])))
    wml = max(np.max(np.abs(sim.rho(m) - ora.rho(m))) for m in range(n_tls, n_tls + n_ml))
    print(f"[wave] {precision}: two-level {worst:.2e}, multilevel {wml:.2e}", flush=True)
    assert np.max(rec[:, :, 0]) > 1e-6
    assert worst <= 1e-12 and wml <= 1e-12
