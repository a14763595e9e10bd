"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle on the
same seeded inputs.  FP64 mode: relative L2 <= 1e-12 over the six field arrays
together and over each probe series; populations to 1e-12 absolute.  FP32-field mode:
relative L2 <= 1e-4 on fields, 1e-6 absolute on populations."""
import sys

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2512_06173_amd import workloads as W
from oracle.feed import build_oracle

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_FIELD_TOL = 1e-4
FP32_POP_TOL = 1e-6


def mlk():
    from paper_2512_06173_amd import mlk as m
    return m


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.concatenate([np.ravel(x) for x in a])
    b = np.concatenate([np.ravel(x) for x in b])
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a - b)


def run_both(w, steps=None, **kw):
    steps = w.steps if steps is None else steps
    say(f"[parity] {w.name} precision={w.precision} steps={steps} {kw}")
    sim = mlk().from_workload(w, **kw)
    ora = build_oracle(w)
    sim.step(steps)
    ora.step(steps)
    return sim, ora


def check(sim, ora, w, field_tol=None, pop_tol=None):
    fp64 = w.precision == "fp64"
    field_tol = field_tol or (FP64_TOL if fp64 else FP32_FIELD_TOL)
    pop_tol = pop_tol or (FP64_TOL if fp64 else FP32_POP_TOL)
    e = rel_l2(sim.fields(), ora.fields())
    say(f"  fields rel L2 = {e:.3e}")
    assert e <= field_tol
    for p in range(len(w.probes)):
        ep = rel_l2([sim.probe(p)], [ora.probe(p)])
        say(f"  probe {p} rel L2 = {ep:.3e}")
        assert ep <= field_tol
    if w.pop_every and w.n_emitters:
        pg, po = sim.populations(), ora.populations()
        assert pg.shape == po.shape
        d = np.max(np.abs(pg - po))
        say(f"  populations max abs = {d:.3e}")
        assert d <= pop_tol
    if w.flux is not None:
        fg, fo = sim.flux_series(), ora.flux_series()
        ef = rel_l2([fg], [fo])
        say(f"  flux rel L2 = {ef:.3e}")
        assert ef <= field_tol
        assert abs(sim.flux_total() - ora.flux_total()) <= field_tol * max(
            1e-300, np.sum(np.abs(fo)) * w.dx * w.courant)


@pytest.mark.parametrize("comp,kidx", [(2, (1, 2, 0)), (0, (0, 1, 3))])
def test_periodic_plane_wave_fp64(comp, kidx):
    n = 32
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    kv = 2 * np.pi * np.array(kidx) / n
    xyz = [i + (comp == 0) * 0.5, j + (comp == 1) * 0.5, k + (comp == 2) * 0.5]
    e0 = np.cos(kv[0] * xyz[0] + kv[1] * xyz[1] + kv[2] * xyz[2])
    w = W.Workload(name="plane_wave", shape=(n, n, n), bc=("periodic",) * 6, steps=500)
    sim = mlk().Simulation(w.shape, bc=w.bc)
    ora = Oracle(w.shape, bc=w.bc)
    sim.set_field(comp, e0)
    ora.set_field(comp, e0)
    sim.step(500)
    ora.step(500)
    check(sim, ora, w)


def test_pec_cavity_mode_fp64():
    n = 32
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    e0 = np.sin(np.pi * i / n) * np.sin(np.pi * j / n)
    w = W.Workload(name="pec_mode", shape=(n, n, n), steps=500)
    sim = mlk().Simulation(w.shape)
    ora = Oracle(w.shape)
    sim.set_field(2, e0)
    ora.set_field(2, e0)
    sim.step(500)
    ora.step(500)
    check(sim, ora, w)


def _sources_workload(shape, bc, cpml, precision, steps, seed=1):
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    eps = rng.choice([1.0, 2.25, 4.0], size=(nz, ny, nx))
    src = [W.PointSource(2, (nx // 2, ny // 2, nz // 2), 1.0, 0.3, 5.0, 20.0),
           W.PointSource(0, (nx // 3, ny // 2 + 1, nz // 2 - 2), -0.7, 0.4, 4.0, 18.0)]
    planes = [W.PlaneSource(2, max(1, cpml[4] + 2), 1, 0.5, 0.25, 8.0, 30.0)]
    probes = [(2, (nx // 2 + 3, ny // 2, nz // 2)), (4, (nx // 2, ny // 2 - 2, nz // 2 + 1))]
    return W.Workload(name=f"sources_{nx}x{ny}x{nz}", shape=shape, bc=bc, cpml=cpml, eps=eps,
                      point_sources=src, plane_sources=planes, probes=probes, steps=steps,
                      precision=precision)


@pytest.mark.parametrize("sweep", ["fused", "plain"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_cpml_dielectric_sources(precision, sweep):
    w = _sources_workload((40, 36, 44), ("cpml",) * 6, (8, 6, 7, 5, 8, 9), precision, 220)
    sim, ora = run_both(w, sweep=sweep)
    check(sim, ora, w)


def test_fused_sweep_many_tiles_and_chunks_fp64():
    """Several x tiles (one ragged), many y tiles and z chunks, CPML on all faces,
    dielectric, point and plane sources: fused sweep against the oracle."""
    w = _sources_workload((150, 37, 70), ("cpml",) * 6, (9, 7, 5, 6, 10, 8), "fp64", 120)
    sim, ora = run_both(w, sweep="fused")
    check(sim, ora, w)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("nx, tx, full", [(72, 64, True), (70, 64, False), (72, 32, True),
                                          (36, 64, True), (36, 32, False)])
def test_fused_box_layers_and_fallback(nx, tx, full, precision):
    """With FP32 fields and the layer mode on, the fused sweep covers the whole grid and
    stretches the derivatives of the CPML cells itself; the FP64 kernel carries the x
    layers only (its y and z extent stops at the layers, with a margin).  The x layers go
    to the plain passes when the low-x halo column of a tile falls into one (nx = 70
    with 8 layers: the second 64-wide tile's halo column x = 63 is a layer cell; nx = 36:
    one 64-wide tile, but the second 32-wide tile's halo column x = 31 is).  Every box
    against the oracle."""
    w = _sources_workload((nx, 30, 36), ("cpml",) * 6, (8, 8, 6, 7, 8, 6), precision, 150)
    say(f"[parity] {w.name} precision={precision} tile width {tx} layers in the fused sweep")
    sim = mlk().from_workload(w, sweep="fused")
    sim.set_tile_width(tx)
    if precision == "fp32":
        sim.set_sweep_layers(True)
    lo, hi = sim.interior_box()
    assert (lo[0], hi[0]) == ((0, nx) if full else (9, nx - 8))
    yz = (0, 30, 0, 36) if precision == "fp32" else (7, 23, 9, 30)
    assert (lo[1], hi[1], lo[2], hi[2]) == yz
    ora = build_oracle(w)
    sim.step(w.steps)
    ora.step(w.steps)
    check(sim, ora, w)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_sweep_decompositions_agree_bitwise(precision):
    """The plain sweep, the fused sweep with the CPML shell, and (FP32) the fused sweep
    carrying every layer, or its lean kernel on the interior with the layer frame in one
    launch of the full kernel, in 64- or 32-wide tiles, give the same fields bit for bit:
    each cell's arithmetic is the same expression, rounded alike, whichever kernel (and
    tile) evaluates it.  In vacuum the
    fused sweep reads no 1/eps_r array; with the array (all ones) it agrees bit for
    bit."""
    w = W.radiating_cube(n=72, n_emit=60, steps=0, cpml=8, precision=precision)
    runs = []
    for sweep, layers, eps_array, tx in (("plain", None, True, 64), ("fused", 0, False, 64),
                                         ("fused", 1, False, 64), ("fused", 2, False, 64),
                                         ("fused", 2, True, 64), ("fused", 0, True, 64),
                                         ("fused", 0, False, 32), ("fused", 1, False, 32),
                                         ("fused", 2, False, 32)):
        if layers and precision == "fp64":
            continue
        sim = mlk().from_workload(w, sweep=sweep)
        if sweep == "fused":
            sim.set_tile_width(tx)
        if layers is not None:
            sim.set_sweep_layers(layers)
        if eps_array:
            # a box set to 2 and back to 1: the grid is vacuum again, but no longer
            # known to be, so the fused sweep reads the 1/eps_r array
            box = ((20, 20, 20), (30, 30, 30))
            sim.set_eps_box(box, np.full((10, 10, 10), 2.0))
            sim.set_eps_box(box, np.ones((10, 10, 10)))
        say(f"[decomposition] {precision} {sweep} layers={layers} eps_array={eps_array} "
            f"tx={tx} box={sim.interior_box()}")
        sim.step(40)
        runs.append(sim.fields())
    for other in runs[1:]:
        for x, y in zip(runs[0], other):
            assert np.array_equal(x, y)
    if precision == "fp64":
        with pytest.raises(mlk().MlkError):
            mlk().from_workload(w, sweep="fused").set_sweep_layers(True)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_chunk_cuts_do_not_change_results(precision):
    """The fused sweep cuts the z extent of its box into chunks of equal cost (z-layer
    planes weigh more), so chunk lengths differ from kz and from each other.  With
    uneven z layers (3 planes at the bottom, 9 at the top), dielectric and sources, every
    kz from one plane per chunk to the whole depth gives the plain sweep's fields bit
    for bit (FP32: every layer in the fused kernel; FP64: the interior box)."""
    w = _sources_workload((40, 24, 37), ("cpml",) * 6, (6, 5, 4, 7, 3, 9), precision, 0)
    ref = mlk().from_workload(w, sweep="plain")
    ref.step(30)
    want = ref.fields()
    for kz in (1, 3, 5, 8, 13, 37):
        sim = mlk().from_workload(w, sweep="fused")
        if precision == "fp32":
            sim.set_sweep_layers(1)
        sim.set_tuning(8, kz)
        say(f"[chunks] {precision} kz={kz} box={sim.interior_box()}")
        sim.step(30)
        assert all(np.array_equal(x, y) for x, y in zip(want, sim.fields())), kz
        sim.close()
    ref.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("bc, lo", [("periodic", 40.2), ("pec", 8.2)])
def test_light_and_tiled_gather_agree_bitwise(precision, bc, lo):
    """An emitter alone in its gather bin is gathered without a tile (a light bin); with
    nine more emitters of zero dipole in the same bin, the bin stages its tile.  The
    extra emitters add nothing to the field, so both runs give the same fields, state
    and gathered field bit for bit.  On the periodic grid the bin sits at the corner
    where the windows wrap."""
    rng = np.random.default_rng(17)
    n = 48
    pos = rng.uniform(lo, lo + 7.6, size=(10, 3))  # one bin in both precisions' binnings
    dip = np.zeros((10, 3))
    dip[0] = (0.3, -0.2, 0.25)
    fields = [1e-2 * rng.standard_normal((n, n, n)) for _ in range(6)]
    runs = []
    for m in (1, 10):
        sim = mlk().Simulation((n, n, n), precision=precision, bc=(bc,) * 6)
        for c in range(6):
            sim.set_field(c, fields[c])
        sim.add_tls(pos[:m], np.ones(m), np.ones(m), 0.25, dip[:m],
                    np.tile([0.5, 0.5, 0.0], (m, 1)))
        say(f"[gather] {precision} {bc} {m} emitter(s) in the bin")
        sim.step(25)
        runs.append((sim.fields(), sim.tls_state(0, 1), sim.emitter_io()[0][0]))
    (fa, ta, ea), (fb, tb, eb) = runs
    assert all(np.array_equal(x, y) for x, y in zip(fa, fb))
    assert np.array_equal(ta, tb) and np.array_equal(ea, eb)
    assert np.any(ea != 0.0)


def test_fused_sweep_refuses_arrays_of_4_gib():
    """The fused kernels address a field array by 32-bit byte offsets: a grid whose
    FP32 arrays would reach 4 GiB (1024^3 cells) is refused before anything is
    allocated, with a message that names the plain sweep."""
    with pytest.raises(mlk().MlkError) as err:
        mlk().Simulation((1024, 1024, 1024), precision="fp32", sweep="fused")
    assert "plain sweep" in str(err.value)


def test_ragged_mixed_boundaries_fp64():
    """x periodic with a ragged tail (nx not a multiple of 64), y metallic, z CPML; emitters
    whose windows wrap across the periodic axis."""
    rng = np.random.default_rng(3)
    nx, ny, nz = 70, 29, 37
    w = _sources_workload((nx, ny, nz), ("periodic", "periodic", "pec", "pec", "cpml", "cpml"),
                          (0, 0, 0, 0, 6, 6), "fp64", 160)
    M = 12
    pos = np.column_stack([rng.uniform(0, nx, M), rng.uniform(5, ny - 5, M),
                           rng.uniform(11, nz - 11, M)])
    pos[0, 0] = 0.3
    pos[1, 0] = nx - 0.2
    w.tls = W.TLSSet(pos=pos, sigma=rng.uniform(0.8, 1.2, M), gamma=rng.uniform(0.5, 1.5, M),
                     omega0=rng.uniform(0.24, 0.26, M), dipole=0.3 * rng.standard_normal((M, 3)),
                     rho0=np.tile([0.5, 0.5, 0.0], (M, 1)))
    w.pop_every = 1
    for scatter, sweep in (("owner", "fused"), ("atomic", "plain"), ("owner", "plain")):
        sim, ora = run_both(w, scatter=scatter, sweep=sweep)
        check(sim, ora, w)


def test_single_emitter_excited_is_exactly_dark():
    w = W.single_emitter("excited")
    sim, ora = run_both(w)
    assert np.all(sim.probe(0) == 0.0)
    for f in sim.fields():
        assert np.all(f == 0.0)
    assert np.max(np.abs(sim.populations() - 1.0)) < 1000 * 5e-16


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_single_emitter_superposition(precision):
    w = W.single_emitter("superposition", precision=precision)
    sim, ora = run_both(w)
    check(sim, ora, w)


@pytest.mark.parametrize("scatter", ["owner", "atomic"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_slab_scaled(precision, scatter):
    w = W.slab(n=48, n_emit=80, steps=600, cpml=8, thick=12, precision=precision)
    w.pop_every = 5
    sim, ora = run_both(w, scatter=scatter)
    check(sim, ora, w)


@pytest.mark.parametrize("scatter", ["owner", "atomic"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_radiating_cube_scaled_flux(precision, scatter):
    w = W.radiating_cube(n=40, n_emit=150, steps=300, cpml=8, precision=precision)
    w.pop_every = 10
    sim, ora = run_both(w, scatter=scatter)
    check(sim, ora, w)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_checkpoint_gives_identical_continuation(precision):
    """Restoring a checkpoint continues the run bit for bit: every kernel of the step is
    deterministic (the owner-computes scatter sums fixed-point integers, whose addition
    does not depend on order), so the restored run repeats the original exactly."""
    w = W.radiating_cube(n=32, n_emit=40, steps=0, cpml=6, precision=precision)
    w.pop_every = 0
    a = mlk().from_workload(w)
    a.step(50)
    blob = a.checkpoint_save()
    a.step(70)
    ref = a.fields()
    ref_state = a.tls_state()
    b = mlk().from_workload(w)
    b.checkpoint_load(blob)
    assert b.step_count == 50
    b.step(70)
    assert all(np.array_equal(x, y) for x, y in zip(b.fields(), ref))
    assert np.array_equal(b.tls_state(), ref_state)


def test_invalid_inputs_are_rejected():
    m = mlk()
    with pytest.raises(m.MlkError) as ei:
        m.Simulation((16, 16, 16), courant=0.7)
    assert ei.value.status == m.MLK_EINVAL
    sim = m.Simulation((20, 20, 20))
    with pytest.raises(m.MlkError) as ei:
        sim.add_tls([[3.0, 10, 10]], 1.0, 1.0, 0.25, [[0, 0, .1]], [[0, 0, 0]])
    assert ei.value.status == m.MLK_EINVAL
    with pytest.raises(m.MlkError):
        sim.add_tls([[10.0, 10, 10]], 1.0, 1.0, 0.25, [[0, 0, .1]], [[0.5, 0.6, 0]])
    with pytest.raises(m.MlkError):
        sim.set_eps(np.full((20, 20, 20), 0.5))
    sim.step(1)
    with pytest.raises(m.MlkError) as ei:
        sim.add_probe(0, (1, 1, 1))
    assert ei.value.status == m.MLK_ESTATE


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_periodic_thin_axis_windows_wrap_inside_one_bin(precision):
    """z periodic and only 8 cells deep: a single bin holds the whole axis and windows
    of emitters near z = 0 wrap into the same bin from both ends."""
    rng = np.random.default_rng(21)
    nx, ny, nz = 40, 24, 8
    M = 20
    pos = np.column_stack([rng.uniform(0, nx, M), rng.uniform(0, ny, M), rng.uniform(0, nz, M)])
    pos[:4, 2] = [0.1, 7.9, 0.6, 7.4]
    w = W.Workload(name="thin_periodic", shape=(nx, ny, nz), bc=("periodic",) * 6, steps=150,
                   precision=precision, pop_every=3,
                   tls=W.TLSSet(pos=pos, sigma=rng.uniform(0.6, 1.0, M),
                                gamma=np.ones(M), omega0=rng.uniform(0.24, 0.26, M),
                                dipole=0.3 * rng.standard_normal((M, 3)),
                                rho0=np.tile([0.5, 0.5, 0.0], (M, 1))),
                   probes=[(2, (5, 5, 0)), (0, (20, 12, 7))])
    for scatter in ("owner", "atomic"):
        sim, ora = run_both(w, scatter=scatter)
        check(sim, ora, w)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_periodic_axis_just_longer_than_a_bin(precision):
    """y periodic with 18 cells (scatter bins of 16), z periodic with 12 (FP64 bins of 8):
    the window of an emitter near the end of such an axis wraps round and meets the first
    bin at both of its ends, so the window rows inside that bin are not one contiguous run
    of window offsets."""
    rng = np.random.default_rng(29)
    nx, ny, nz = 40, 18, 12
    M = 24
    pos = np.column_stack([rng.uniform(0, nx, M), rng.uniform(0, ny, M), rng.uniform(0, nz, M)])
    pos[:8, 1] = [16.3, 17.2, 15.6, 17.8, 0.4, 16.9, 1.5, 15.9]
    pos[:8, 2] = [9.6, 10.4, 11.2, 9.1, 10.8, 0.3, 9.9, 11.7]
    w = W.Workload(name="just_longer_periodic", shape=(nx, ny, nz), bc=("periodic",) * 6,
                   steps=150, precision=precision, pop_every=3,
                   tls=W.TLSSet(pos=pos, sigma=rng.uniform(0.8, 1.1, M),
                                gamma=np.ones(M), omega0=rng.uniform(0.24, 0.26, M),
                                dipole=0.3 * rng.standard_normal((M, 3)),
                                rho0=np.tile([0.5, 0.5, 0.0], (M, 1))),
                   probes=[(2, (5, 17, 0)), (1, (20, 0, 11))])
    for scatter in ("owner", "atomic"):
        sim, ora = run_both(w, scatter=scatter)
        check(sim, ora, w)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_two_dimensional_superradiance_run(precision):
    """z-invariant grid (one periodic cell): the 2-D set-up of the paper's superradiance
    example, N = 4 collocated emitters in the weak-excitation state."""
    n, d = 96, 12
    w = W.Workload(name="2d_superradiance", shape=(n, n, 1),
                   bc=("cpml",) * 4 + ("periodic",) * 2, cpml=(d, d, d, d, 0, 0), steps=800,
                   precision=precision, pop_every=1,
                   tls=W.TLSSet(pos=np.tile([n / 2, n / 2, 0.5], (4, 1)), sigma=np.ones(4),
                                gamma=np.ones(4), omega0=np.full(4, 0.25),
                                dipole=np.tile([0.0, 0.0, 0.1], (4, 1)),
                                rho0=np.tile([1e-4, np.sqrt(0.9999) * 0.01, 0.0], (4, 1))),
                   probes=[(2, (n // 2 + 10, n // 2, 0))])
    sim, ora = run_both(w)
    check(sim, ora, w)


@pytest.mark.parametrize("sweep", ["fused", "plain"])
def test_shell_and_interior_regions_fp64(sweep):
    """Asymmetric CPML thicknesses (one face metallic) so that the fused sweep's interior
    box and its shell slabs have uneven sizes; emitters and sources straddle the seams."""
    rng = np.random.default_rng(33)
    nx, ny, nz = 77, 45, 52
    w = _sources_workload((nx, ny, nz), ("cpml", "pec", "pec", "cpml", "cpml", "cpml"),
                          (7, 0, 0, 9, 6, 11), "fp64", 140)
    M = 25
    pos = np.column_stack([rng.uniform(12, nx - 5, M), rng.uniform(5, ny - 14, M),
                           rng.uniform(11, nz - 16, M)])
    w.tls = W.TLSSet(pos=pos, sigma=np.ones(M), gamma=np.ones(M),
                     omega0=rng.uniform(0.24, 0.26, M), dipole=0.3 * rng.standard_normal((M, 3)),
                     rho0=np.tile([0.5, 0.5, 0.0], (M, 1)))
    w.pop_every = 2
    sim, ora = run_both(w, sweep=sweep)
    check(sim, ora, w)


def _small_bragg(precision, n_emit=48, steps=300, dmag=0.2, gphi=1e-3, seed=3):
    w = W.bragg(nx=16, ny=16, nz=112, n_emit=n_emit, steps=steps, pairs_per_mirror=3,
                precision=precision, seed=seed)
    ml = w.multilevel
    ml.dipole = ml.dipole * (dmag / 0.01)
    ml.gphi = np.full(len(ml), gphi)
    w.pop_every = 3
    return w


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_bragg_multilevel(precision):
    """Multilevel (2-6 level) Lindblad emitters in a small Bragg resonator, periodic
    x/y, CPML z, a probe in the defect."""
    w = _small_bragg(precision)
    sim, ora = run_both(w)
    check(sim, ora, w)
    if precision == "fp64":
        for m in (0, 7, len(w.multilevel) - 1):
            d = np.max(np.abs(sim.rho(m) - ora.rho(m)))
            say(f"  rho[{m}] max abs = {d:.3e}")
            assert d <= 1e-12


def test_multilevel_strong_dephasing_fp64():
    w = _small_bragg("fp64", n_emit=20, steps=200, dmag=0.3, gphi=0.05, seed=11)
    sim, ora = run_both(w)
    check(sim, ora, w)


def test_two_level_multilevel_matches_tls_path_fp64():
    """A two-level emitter entered as a multilevel one (M = sigma_x, E = (0, w0), no
    dephasing) takes the same step as the two-level kernel."""
    rng = np.random.default_rng(5)
    n, M = 24, 6
    pos = rng.uniform(8, 16, size=(M, 3))
    w0 = rng.uniform(0.24, 0.26, M)
    dip = 0.3 * rng.standard_normal((M, 3))
    c = np.sqrt(0.5)
    runs = []
    for kind in ("tls", "ml"):
        sim = mlk().Simulation((n, n, n), precision="fp64")
        if kind == "tls":
            sim.add_tls(pos, np.ones(M), np.ones(M), w0, dip, np.tile([0.5, 0.5, 0.0], (M, 1)))
        else:
            rho = np.array([[0.5, 0.5], [0.5, 0.5]], dtype=complex)
            sim.add_multilevel([2] * M, [np.array([0.0, w]) for w in w0],
                               [np.array([[0.0, 1.0], [1.0, 0.0]])] * M, dip, np.zeros(M),
                               [rho] * M, pos, np.ones(M), np.ones(M))
        sim.record_populations(1)
        sim.step(200)
        runs.append((sim.fields(), sim.populations()))
    e = rel_l2(runs[0][0], runs[1][0])
    d = np.max(np.abs(runs[0][1] - runs[1][1]))
    say(f"  tls vs multilevel: fields rel L2 {e:.3e}, populations {d:.3e}")
    assert e <= 1e-12 and d <= 1e-12


def test_mixed_tls_and_multilevel_fp64():
    w = _small_bragg("fp64", n_emit=16, steps=200, seed=4)
    rng = np.random.default_rng(9)
    zc = w.multilevel.pos[:, 2].mean()
    Mt = 10
    pos = np.column_stack([rng.uniform(0, 16, Mt), rng.uniform(0, 16, Mt),
                           rng.uniform(zc - 5, zc + 5, Mt)])
    w.tls = W.TLSSet(pos=pos, sigma=np.ones(Mt), gamma=np.ones(Mt),
                     omega0=rng.uniform(0.24, 0.26, Mt), dipole=0.2 * rng.standard_normal((Mt, 3)),
                     rho0=np.tile([0.5, 0.5, 0.0], (Mt, 1)))
    sim, ora = run_both(w)
    check(sim, ora, w)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_superradiance_2d_rate_on_the_gpu(precision):
    """The paper's 2-D validation on the GPU path: z-invariant vacuum grid, TLS in the
    weak-excitation state; P_e decays as exp(-N gamma t) with gamma = mu^2 w^2 / 2 times
    the Gaussian kernel's form factor exp(-(w sigma)^2), for N = 1 and N = 4 collocated
    emitters (the rate law pinned on the oracle)."""
    n, d, steps, w0, mu = 128, 16, 4000, 0.25, 0.1
    gamma = mu ** 2 * w0 ** 2 / 2 * np.exp(-w0 ** 2)
    for N in (1, 4):
        w = W.Workload(name="2d_rate", shape=(n, n, 1),
                       bc=("cpml",) * 4 + ("periodic",) * 2, cpml=(d, d, d, d, 0, 0),
                       steps=steps, precision=precision, pop_every=1,
                       tls=W.TLSSet(pos=np.tile([n / 2, n / 2, 0.5], (N, 1)), sigma=np.ones(N),
                                    gamma=np.ones(N), omega0=np.full(N, w0),
                                    dipole=np.tile([0.0, 0.0, mu], (N, 1)),
                                    rho0=np.tile([1e-4, np.sqrt(0.9999) * 0.01, 0.0], (N, 1))))
        sim = mlk().from_workload(w)
        sim.step(steps)
        P = sim.populations()
        t = (np.arange(P.shape[0]) + 0.5) * sim.dt
        sel = t > 200.0
        for q in range(N):
            rate = -np.polyfit(t[sel], np.log(P[sel, q]), 1)[0]
            say(f"  {precision} N={N} emitter {q}: rate / (N gamma) = {rate / (N * gamma):.4f}")
            assert abs(rate / (N * gamma) - 1) < 0.02
