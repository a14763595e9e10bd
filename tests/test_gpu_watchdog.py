"""The non-finite watchdog (robustness, Sec. III item (v)): a NaN put into an emitter's
density matrix through a checkpoint is reported by mlk_sync as MLK_ENUMERIC, naming the
step; a clean checkpoint clears it; batches report it for their members; a clean run
never raises it."""
import numpy as np
import pytest

from paper_2512_06173_amd import workloads as W

pytestmark = pytest.mark.gpu

MLK_ENUMERIC = 6


def mlk():
    from paper_2512_06173_amd import mlk as m
    return m


def poisoned(blob, shape, esz, which=1):
    """A copy of a checkpoint with entry `which` of the first two-level state set to NaN:
    the states follow the six field arrays (no CPML face in these grids)."""
    bad = np.array(blob, copy=True)
    off = 6 * int(np.prod(shape)) * esz + 8 * which
    bad[off:off + 8] = np.frombuffer(np.float64(np.nan).tobytes(), dtype=np.uint8)
    return bad


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_nan_in_rho_is_reported_and_cleared(precision):
    w = W.single_emitter("superposition", steps=0, precision=precision)
    s = mlk().from_workload(w)
    s.step(5)
    s.sync()
    blob = s.checkpoint_save()
    s.checkpoint_load(poisoned(blob, w.shape, 8 if precision == "fp64" else 4))
    s.step(3)
    with pytest.raises(mlk().MlkError) as e:
        s.sync()
    assert e.value.status == MLK_ENUMERIC
    assert "step 5" in str(e.value)
    with pytest.raises(mlk().MlkError):
        s.sync()  # stays reported
    s.checkpoint_load(blob)
    s.step(3)
    s.sync()
    assert np.all(np.isfinite(s.tls_state()))


def test_batch_sync_reports_a_member():
    ws = [W.single_emitter("superposition", n=n, steps=0, precision="fp32") for n in (32, 40)]
    sims = [mlk().from_workload(w) for w in ws]
    blob = sims[1].checkpoint_save()
    sims[1].checkpoint_load(poisoned(blob, ws[1].shape, 4, which=0))
    with mlk().Batch(sims) as b:
        b.step(2)
        with pytest.raises(mlk().MlkError) as e:
            b.sync()
        assert e.value.status == MLK_ENUMERIC


def test_clean_runs_do_not_trip_the_watchdog():
    w = W.radiating_cube(n=40, n_emit=150, steps=0, cpml=8, precision="fp32")
    w.pop_every = 1
    s = mlk().from_workload(w)
    s.step(60)
    s.sync()
