"""Dispersive media (Lorentz and Drude poles over cell boxes, the dielectric functions of
eq. Dromega): the coupled step with poles against the oracle, element by element, in both
sweeps and both field precisions; the uniform-field relaxation to D / eps(0); checkpoints
carry the polarisation; refused combinations."""
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


def rel_l2(a, b):
    a = np.concatenate([np.ravel(x) for x in a])
    b = np.concatenate([np.ravel(x) for x in b])
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# Lorentz with loss, a Drude metal overlapping it, and a lossless Lorentz slab
POLES = [((7, 6, 9, 17, 16, 21), 0.45, 0.02, 1.2, False),
         ((10, 8, 12, 15, 14, 18), 0.6, 0.1, 2.5, True),
         ((6, 6, 20, 18, 16, 23), 0.3, 0.0, 0.8, False)]


def dispersive_block(precision, seed=4):
    """24 x 22 x 30 cells, CPML 5 on every face, eps_inf in the pole boxes, a pulsed point
    source and a plane source, two emitters beside the block, a probe and a flux plane."""
    nx, ny, nz = 24, 22, 30
    rng = np.random.default_rng(seed)
    eps = np.ones((nz, ny, nx))
    for (x0, y0, z0, x1, y1, z1), *_ in POLES:
        eps[z0:z1, y0:y1, x0:x1] = 1.5
    tls = W.TLSSet(pos=np.array([[11.3, 11.0, 9.3], [12.6, 10.4, 20.6]]), sigma=np.ones(2),
                   gamma=np.ones(2), omega0=np.array([0.45, 0.5]),
                   dipole=np.array([[0.0, 0.2, 1.0], [0.3, 0.0, 0.8]]),
                   rho0=np.array([[0.9, 0.3, 0.0], [0.0, 0.0, 0.0]]))
    return W.Workload(name="dispersive", shape=(nx, ny, nz), bc=("cpml",) * 6, cpml=(5,) * 6,
                      eps=eps, tls=tls,
                      plane_sources=[W.PlaneSource(2, 7, 0, 0.3, 0.5, 6.0, 18.0)],
                      point_sources=[W.PointSource(1, (12, 11, 10), 1.0, 0.45, 5.0, 15.0)],
                      probes=[(0, (12, 11, 14)), (2, (9, 10, 19))], flux=(2, 22), pop_every=1,
                      steps=240, precision=precision)


def add_poles(o):
    for box, w0, g, s, drude in POLES:
        o.add_susceptibility(box, w0, g, s, drude=drude)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("sweep", ["fused", "plain"])
def test_dispersive_step_matches_the_oracle(precision, sweep):
    """240 coupled steps with three overlapping poles: the six fields (relative L2), the
    probes, the flux series and the populations against the oracle.  FP64 within 1e-12,
    FP32 fields within 1e-4."""
    w = dispersive_block(precision)
    say(f"[dispersive] {precision} {sweep}: {w.shape}, {len(POLES)} poles, {w.steps} steps")
    sim = mlk().from_workload(w, sweep=sweep)
    ora = build_oracle(w)
    add_poles(sim)
    add_poles(ora)
    sim.step(w.steps)
    ora.step(w.steps)
    ef = rel_l2(sim.fields(), ora.fields())
    ep = max(rel_l2([sim.probe(p)], [ora.probe(p)]) for p in range(2))
    efl = rel_l2([sim.flux_series()], [ora.flux_series()])
    epop = np.max(np.abs(sim.populations() - ora.populations()))
    say(f"  fields {ef:.2e}, probes {ep:.2e}, flux {efl:.2e}, populations {epop:.2e}")
    tol = 1e-12 if precision == "fp64" else 1e-4
    assert ef <= tol and ep <= tol and efl <= tol
    assert epop <= (1e-12 if precision == "fp64" else 1e-6)
    # the poles matter: without them the fields differ at the percent level
    plain = build_oracle(w)
    plain.step(w.steps)
    assert rel_l2(plain.fields(), ora.fields()) > 1e-2


@pytest.mark.parametrize("drude", [False, True])
def test_uniform_field_relaxes_to_the_static_permittivity(drude):
    """A periodic box filled with a lossy pole: D = eps_inf E + P is conserved, so a
    uniform E relaxes to D / (eps_inf + sigma) (Lorentz) or to 0 (Drude)."""
    einf, sigma, w0, gamma = 2.0, 1.5, 0.4, 0.2
    sim = mlk().Simulation((4, 4, 4), bc=("periodic",) * 6)
    sim.set_eps(np.full((4, 4, 4), einf))
    sim.add_susceptibility((0, 0, 0, 4, 4, 4), w0, gamma, sigma, drude=drude)
    E0 = (0.5, -1.0, 0.25)
    for c in range(3):
        sim.set_field(c, np.full((4, 4, 4), E0[c]))
    sim.step(1500)
    target = np.zeros(3) if drude else np.array(E0) * einf / (einf + sigma)
    got = np.array([sim.get_field(c)[2, 1, 3] for c in range(3)])
    say(f"[dispersive] uniform {'drude' if drude else 'lorentz'}: E = {got}, target {target}")
    assert np.max(np.abs(got - target)) < 1e-8


def test_dispersive_checkpoint_round_trip():
    """A checkpoint taken mid-run carries P and its increment: reloading it and stepping
    again reproduces the fields bit for bit."""
    w = dispersive_block("fp64", seed=5)
    w.pop_every = 0
    sim = mlk().from_workload(w)
    add_poles(sim)
    sim.step(50)
    ck = sim.checkpoint_save()
    sim.step(40)
    f1 = sim.fields()
    sim.checkpoint_load(ck)
    sim.step(40)
    assert all(np.array_equal(a, b) for a, b in zip(sim.fields(), f1))


def test_dispersive_refusals():
    """Boxes that reach the CPML, the wall plane or outside the grid, bad parameters, a
    ninth pole, late poles, batches, the adjoint and a cavity are refused."""
    m = mlk()

    def status(fn, *a, **k):
        with pytest.raises(m.MlkError) as ex:
            fn(*a, **k)
        return ex.value.status

    w = dispersive_block("fp64", seed=6)
    w.pop_every = 0
    sim = m.from_workload(w)
    assert status(sim.add_susceptibility, (4, 6, 9, 10, 16, 21), 0.4, 0.0, 1.0) == m.MLK_EINVAL
    assert status(sim.add_susceptibility, (7, 6, 9, 20, 16, 21), 0.4, 0.0, 1.0) == m.MLK_EINVAL
    assert status(sim.add_susceptibility, (7, 6, 9, 7, 16, 21), 0.4, 0.0, 1.0) == m.MLK_EINVAL
    assert status(sim.add_susceptibility, (7, 6, 9, 10, 16, 21), 0.0, 0.0, 1.0) == m.MLK_EINVAL
    assert status(sim.add_susceptibility, (7, 6, 9, 10, 16, 21), 0.4, -0.1, 1.0) == m.MLK_EINVAL
    pec = m.Simulation((8, 8, 8))
    assert status(pec.add_susceptibility, (0, 1, 1, 4, 4, 4), 0.4, 0.0, 1.0) == m.MLK_EINVAL
    pec.add_susceptibility((1, 1, 1, 8, 8, 8), 0.4, 0.0, 1.0)
    for _ in range(7):
        pec.add_susceptibility((1, 1, 1, 4, 4, 4), 0.4, 0.0, 1.0)
    assert status(pec.add_susceptibility, (1, 1, 1, 4, 4, 4), 0.4, 0.0, 1.0) == m.MLK_EINVAL
    assert status(pec.set_cavity, 0.2, 1.0) == m.MLK_EUNSUPPORTED
    add_poles(sim)
    assert status(m.Batch, [sim]) == m.MLK_EUNSUPPORTED
    assert status(sim.adjoint, "population", 10, ((8, 8, 8), (12, 12, 12)),
                  weights=np.ones(2)) == m.MLK_EUNSUPPORTED
    sim.step(2)
    assert status(sim.add_susceptibility, (7, 6, 9, 10, 16, 21), 0.4, 0.0, 1.0) == m.MLK_ESTATE


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_single_cell_poles_at_the_box_limits(precision):
    """Degenerate boxes: one cell next to the CPML on the low side and one touching the
    CPML on the high side of every axis, a Drude and a Lorentz pole, against the oracle."""
    w = dispersive_block(precision, seed=7)
    nx, ny, nz = w.shape
    poles = [((5, 5, 5, 6, 6, 6), 0.5, 0.05, 2.0, True),
             ((nx - 6, ny - 6, nz - 6, nx - 5, ny - 5, nz - 5), 0.4, 0.0, 1.0, False),
             ((5, 10, 12, nx - 5, 11, 13), 0.35, 0.02, 1.5, False)]
    sim = mlk().from_workload(w)
    ora = build_oracle(w)
    for o in (sim, ora):
        for box, w0, g, s, drude in poles:
            o.add_susceptibility(box, w0, g, s, drude=drude)
    sim.step(120)
    ora.step(120)
    e = rel_l2(sim.fields(), ora.fields())
    say(f"[dispersive] single-cell boxes {precision}: fields {e:.2e}")
    assert e <= (1e-12 if precision == "fp64" else 1e-4)
