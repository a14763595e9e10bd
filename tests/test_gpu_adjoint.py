"""The checkpointed GPU adjoint against the FP64 oracle adjoint (itself pinned to
central differences), its independence of the checkpoint interval, the state left as it
was, and the torch.autograd wrapper."""
import numpy as np
import pytest

from oracle.feed import build_oracle
from paper_2512_06173_amd import workloads as W

pytestmark = pytest.mark.gpu

BOX = ((8, 8, 8), (14, 14, 14))


def mlk():
    from paper_2512_06173_amd import mlk as m
    return m


def say(msg):
    print(msg, flush=True)


def problem(precision="fp64", seed=7):
    """22^3, CPML 4, a point-source pulse, 6 strongly coupled TLS in the centre, flux
    plane at z = 15; 60 steps (the problem of the oracle's adjoint pins)."""
    rng = np.random.default_rng(seed)
    n, M = 22, 6
    pos = rng.uniform(9.5, 12.5, size=(M, 3))
    tls = W.TLSSet(pos=pos, sigma=np.full(M, 0.8), gamma=np.ones(M),
                   omega0=rng.uniform(0.45, 0.55, M), dipole=0.6 * rng.standard_normal((M, 3)),
                   rho0=np.tile([0.5, 0.5, 0.0], (M, 1)))
    eps = rng.uniform(1.0, 2.0, (n, n, n))
    return W.Workload(name="adj", shape=(n, n, n), bc=("cpml",) * 6, cpml=(4,) * 6, eps=eps,
                      tls=tls, point_sources=[W.PointSource(1, (11, 10, 9), 1.0, 0.5, 2.0, 6.0)],
                      flux=(2, 15), steps=60, precision=precision)


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


@pytest.mark.parametrize("sweep", ["fused", "plain"])
@pytest.mark.parametrize("objective", ["flux", "population"])
def test_adjoint_matches_oracle_fp64(objective, sweep):
    w = problem()
    weights = np.linspace(1.0, 2.0, len(w.tls))
    ov, oge, ogd = build_oracle(w).adjoint(objective, w.steps, BOX, weights=weights)
    sim = mlk().from_workload(w, sweep=sweep)
    gv, gge, ggd = sim.adjoint(objective, w.steps, BOX, weights=weights, checkpoint_every=25)
    say(f"[adjoint] {objective} {sweep}: value {abs(gv - ov) / abs(ov):.2e}, "
        f"eps {rel(gge, oge):.2e}, dipole {rel(ggd, ogd):.2e}")
    assert abs(gv - ov) <= 1e-14 * abs(ov)
    assert rel(gge, oge) <= 1e-13
    assert rel(ggd, ogd) <= 1e-13


@pytest.mark.parametrize("bc, cpml", [
    (("periodic", "periodic", "pec", "pec", "cpml", "cpml"), (0, 0, 0, 0, 5, 6)),
    (("periodic",) * 6, (0,) * 6),
    (("cpml", "pec", "pec", "cpml", "cpml", "cpml"), (7, 0, 0, 6, 5, 4)),
])
@pytest.mark.parametrize("sweep", ["fused", "plain"])
def test_adjoint_closures_tiles_and_chunks_fp64(bc, cpml, sweep):
    """70 x 26 x 40 (two x tiles, one ragged; several z chunks) with periodic, metallic
    and uneven CPML faces: the fused transposed sweep (box plus shell passes) and the
    whole-grid one against the oracle adjoint, flux objective."""
    rng = np.random.default_rng(11)
    shape = (70, 26, 40)
    M = 5
    pos = np.column_stack([rng.uniform(30, 40, M), rng.uniform(11, 15, M),
                           rng.uniform(17, 23, M)])
    tls = W.TLSSet(pos=pos, sigma=np.full(M, 0.8), gamma=np.ones(M),
                   omega0=rng.uniform(0.45, 0.55, M), dipole=0.6 * rng.standard_normal((M, 3)),
                   rho0=np.tile([0.5, 0.5, 0.0], (M, 1)))
    eps = rng.uniform(1.0, 2.0, (shape[2], shape[1], shape[0]))
    w = W.Workload(name="adj_closures", shape=shape, bc=bc, cpml=cpml, eps=eps, tls=tls,
                   point_sources=[W.PointSource(1, (33, 12, 19), 1.0, 0.5, 2.0, 6.0)],
                   flux=(2, 29), steps=40, precision="fp64")
    box = ((30, 10, 17), (37, 16, 24))
    ov, oge, ogd = build_oracle(w).adjoint("flux", w.steps, box)
    sim = mlk().from_workload(w, sweep=sweep)
    gv, gge, ggd = sim.adjoint("flux", w.steps, box, checkpoint_every=15)
    say(f"[adjoint closures] {bc} {sweep}: value {abs(gv - ov) / abs(ov):.2e}, "
        f"eps {rel(gge, oge):.2e}, dipole {rel(ggd, ogd):.2e}")
    assert abs(gv - ov) <= 1e-14 * abs(ov)
    assert rel(gge, oge) <= 1e-13
    assert rel(ggd, ogd) <= 1e-13


@pytest.mark.parametrize("bc, cpml", [
    (("periodic", "periodic", "pec", "pec", "cpml", "cpml"), (0, 0, 0, 0, 5, 6)),
    (("cpml", "pec", "pec", "cpml", "cpml", "cpml"), (7, 0, 0, 6, 5, 4)),
])
def test_fused_transposed_sweep_fp32_matches_plain(bc, cpml):
    """FP32 fields: the fused transposed sweep carries the z layers itself (every z
    plane in its box); against the whole-grid transposed sweep in FP32 and against the
    FP64 oracle, on the closures problem of 70 x 26 x 40 cells."""
    rng = np.random.default_rng(12)
    shape = (70, 26, 40)
    M = 5
    pos = np.column_stack([rng.uniform(30, 40, M), rng.uniform(11, 15, M),
                           rng.uniform(17, 23, M)])
    tls = W.TLSSet(pos=pos, sigma=np.full(M, 0.8), gamma=np.ones(M),
                   omega0=rng.uniform(0.45, 0.55, M), dipole=0.6 * rng.standard_normal((M, 3)),
                   rho0=np.tile([0.5, 0.5, 0.0], (M, 1)))
    eps = rng.uniform(1.0, 2.0, (shape[2], shape[1], shape[0]))
    w = W.Workload(name="adj_fp32_z", shape=shape, bc=bc, cpml=cpml, eps=eps, tls=tls,
                   point_sources=[W.PointSource(1, (33, 12, 3), 1.0, 0.5, 2.0, 6.0)],
                   flux=(2, 37), steps=40, precision="fp32")
    box = ((30, 10, 2), (37, 16, 9))
    res = {}
    for sweep in ("fused", "plain"):
        sim = mlk().from_workload(w, sweep=sweep)
        res[sweep] = sim.adjoint("flux", w.steps, box, checkpoint_every=15)
    ov, oge, ogd = build_oracle(w).adjoint("flux", w.steps, box)
    (fv, fge, fgd), (pv, pge, pgd) = res["fused"], res["plain"]
    say(f"[adjoint fp32 z] {bc}: fused/plain value {abs(fv - pv) / abs(pv):.2e}, "
        f"eps {rel(fge, pge):.2e}, dipole {rel(fgd, pgd):.2e}; fused/oracle eps "
        f"{rel(fge, oge):.2e}")
    assert abs(fv - pv) <= 1e-5 * abs(pv)
    assert rel(fge, pge) <= 2e-5
    assert rel(fgd, pgd) <= 2e-5
    assert rel(fge, oge) <= 1e-5
    assert rel(fgd, ogd) <= 1e-5


@pytest.mark.parametrize("objective", ["flux", "population"])
def test_adjoint_fp32_fields(objective):
    w = problem("fp32")
    weights = np.linspace(1.0, 2.0, len(w.tls))
    ov, oge, ogd = build_oracle(w).adjoint(objective, w.steps, BOX, weights=weights)
    sim = mlk().from_workload(w)
    gv, gge, ggd = sim.adjoint(objective, w.steps, BOX, weights=weights, checkpoint_every=25)
    say(f"[adjoint fp32] {objective}: value {abs(gv - ov) / abs(ov):.2e}, "
        f"eps {rel(gge, oge):.2e}, dipole {rel(ggd, ogd):.2e}")
    assert abs(gv - ov) <= 1e-6 * abs(ov)
    assert rel(gge, oge) <= 1e-5
    assert rel(ggd, ogd) <= 1e-5


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_adjoint_in_vacuum_matches_the_eps_array_path(precision):
    """In vacuum the forward and transposed sweeps and the adjoint gather read no
    1/eps_r array; with the array present (all ones) every result is the same bit
    for bit, and the FP64 one matches the oracle."""
    w = problem(precision)
    w = W.Workload(name="adj_vacuum", shape=w.shape, bc=w.bc, cpml=w.cpml, eps=None,
                   tls=w.tls, point_sources=w.point_sources, flux=w.flux, steps=w.steps,
                   precision=precision)
    out = []
    for eps_array in (False, True):
        sim = mlk().from_workload(w)
        if eps_array:
            sim.set_eps_box(((3, 3, 3), (6, 6, 6)), np.full((3, 3, 3), 2.0))
            sim.set_eps_box(((3, 3, 3), (6, 6, 6)), np.ones((3, 3, 3)))
        out.append(sim.adjoint("flux", w.steps, BOX, checkpoint_every=25))
    v, ge, gd = out[0]
    assert v == out[1][0]
    assert np.array_equal(ge, out[1][1]) and np.array_equal(gd, out[1][2])
    if precision == "fp64":
        ov, oge, ogd = build_oracle(w).adjoint("flux", w.steps, BOX)
        say(f"[adjoint vacuum] value {abs(v - ov) / abs(ov):.2e}, eps {rel(ge, oge):.2e}, "
            f"dipole {rel(gd, ogd):.2e}")
        assert abs(v - ov) <= 1e-14 * abs(ov)
        assert rel(ge, oge) <= 1e-13
        assert rel(gd, ogd) <= 1e-13


def test_checkpoint_interval_does_not_change_the_result():
    w = problem()
    out = []
    for k in (7, 25, 60, 200):
        sim = mlk().from_workload(w)
        out.append(sim.adjoint("flux", w.steps, BOX, checkpoint_every=k))
    for v, ge, gd in out[1:]:
        assert v == out[0][0]
        assert np.array_equal(ge, out[0][1]) and np.array_equal(gd, out[0][2])


def test_adjoint_leaves_the_state_unchanged():
    w = problem()
    a = mlk().from_workload(w)
    b = mlk().from_workload(w)
    a.step(9)
    b.step(9)
    before = a.fields()
    a.adjoint("flux", 30, BOX, checkpoint_every=8)
    assert all(np.array_equal(x, y) for x, y in zip(before, a.fields()))
    a.step(5)
    b.step(5)
    assert all(np.array_equal(x, y) for x, y in zip(a.fields(), b.fields()))
    assert np.array_equal(a.flux_series(), b.flux_series())


def test_torch_autograd_wrapper():
    import torch
    w = problem()
    sim = mlk().from_workload(w)
    (x0, y0, z0), (x1, y1, z1) = BOX
    e = torch.tensor(w.eps[z0:z1, y0:y1, x0:x1], dtype=torch.float64, requires_grad=True)
    d = torch.tensor(w.tls.dipole, dtype=torch.float64, requires_grad=True)
    J = mlk().coupled_objective(sim, e, d, "flux", w.steps, BOX, checkpoint_every=20)
    # the forward pass is one plain run: no adjoint has run yet
    assert sim.adjoint_times() == (0.0, 0.0)
    J.backward()
    assert sim.adjoint_times()[1] > 0.0
    v, ge, gd = mlk().from_workload(w).adjoint("flux", w.steps, BOX, checkpoint_every=20)
    assert float(J) == v
    assert np.array_equal(e.grad.numpy(), ge) and np.array_equal(d.grad.numpy(), gd)


def test_adjoint_refuses_multilevel_emitters():
    w = W.bragg(nx=16, ny=16, nz=112, n_emit=4, steps=10, pairs_per_mirror=3, precision="fp64")
    w.flux = (2, 90)
    sim = mlk().from_workload(w)
    with pytest.raises(mlk().MlkError):
        sim.adjoint("flux", 10, ((2, 2, 40), (6, 6, 44)))


def test_torch_autograd_population_objective():
    """The population objective through the autograd wrapper: forward is one plain run,
    backward the adjoint; both agree with a direct adjoint call, and a second forward
    from the restored state gives the same value."""
    import torch
    w = problem()
    weights = np.linspace(1.0, 2.0, len(w.tls))
    sim = mlk().from_workload(w)
    (x0, y0, z0), (x1, y1, z1) = BOX
    e = torch.tensor(w.eps[z0:z1, y0:y1, x0:x1], dtype=torch.float64, requires_grad=True)
    d = torch.tensor(w.tls.dipole, dtype=torch.float64, requires_grad=True)
    J = mlk().coupled_objective(sim, e, d, "population", w.steps, BOX, weights=weights,
                                checkpoint_every=20)
    J2 = mlk().coupled_objective(sim, e, d, "population", w.steps, BOX, weights=weights)
    assert float(J) == float(J2)
    J.backward()
    v, ge, gd = mlk().from_workload(w).adjoint("population", w.steps, BOX, weights=weights,
                                                checkpoint_every=20)
    assert abs(float(J) - v) <= 1e-15 * abs(v)
    assert np.array_equal(e.grad.numpy(), ge) and np.array_equal(d.grad.numpy(), gd)
