"""mlk_bind_device_buffers: a simulation whose fields, CPML state and emitter states live
in torch tensors steps exactly as one on the library's own memory (bit for bit), the
tensors hold the current fields, and binding after some steps carries the state over."""
import numpy as np
import pytest

from paper_2512_06173_amd import workloads as W

pytestmark = pytest.mark.gpu


def mlk():
    from paper_2512_06173_amd import mlk as m
    return m


def workloads(precision):
    cube = W.radiating_cube(n=40, n_emit=150, steps=0, cpml=8, precision=precision)
    cube.pop_every = 3
    bragg = W.bragg(nx=16, ny=16, nz=160, n_emit=40, steps=0, pairs_per_mirror=3,
                    precision=precision)
    bragg.pop_every = 3
    return [cube, bragg]


def same(a, b, w):
    for x, y in zip(a.fields(), b.fields()):
        assert np.array_equal(x, y)
    if a.n_tls:
        assert np.array_equal(a.tls_state(0, a.n_tls), b.tls_state(0, b.n_tls))
    for m in range(a.n_tls, len(a.nlev)):
        assert np.array_equal(a.rho(m), b.rho(m))
    assert np.array_equal(a.populations(), b.populations())
    for p in range(len(w.probes)):
        assert np.array_equal(a.probe(p), b.probe(p))


@pytest.mark.parametrize("sweep", ["fused", "plain"])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_torch_backed_sim_matches_library_memory(precision, sweep):
    import torch
    for w in workloads(precision):
        a = mlk().from_workload(w, sweep=sweep)
        b = mlk().from_workload(w, sweep=sweep)
        t = b.bind_torch()
        assert t["field"][0][0] is not None
        assert (t["field"][1][0] is not None) == (sweep == "fused")
        for n in (7, 6):
            a.step(n)
            b.step(n)
            same(a, b, w)
            for c in range(6):
                got = b.field_tensor(c).cpu().numpy()
                assert np.array_equal(got, b.get_field(c).astype(got.dtype))
        # the tensors are the state: writing into them is what the sim continues from
        k = b.field_tensor(2)
        k.mul_(1.0)
        torch.cuda.synchronize()
        a.step(3)
        b.step(3)
        same(a, b, w)
        a.close()
        b.close()


def test_binding_mid_run_carries_the_state_and_locks_the_emitters():
    w = workloads("fp32")[0]
    a = mlk().from_workload(w)
    b = mlk().from_workload(w)
    a.step(5)
    b.step(5)
    b.bind_torch()
    a.step(4)
    b.step(4)
    same(a, b, w)
    with pytest.raises(mlk().MlkError) as e:
        b.add_tls(np.array([[20.0, 20.0, 20.0]]), [1.0], [1.0], [0.25], np.array([[0, 0, 0.01]]),
                  np.array([[0.0, 0.0, 0.0]]))
    assert e.value.status == 4  # MLK_ESTATE
