"""mlk_step_prescribed_noalloc (the classical-path steps staged through the library's
fixed device array, no allocation) against mlk_step_prescribed on the same inputs:
recorded two-level states, final states of every emitter and the last E~ / mu_dot,
bit for bit.  Two calls in a row, the second smaller; the first spans several passes
through the array with a ragged last one.  Sizes beyond the array are refused."""
import numpy as np
import pytest

from paper_2512_06173_amd import workloads as W

pytestmark = pytest.mark.gpu


def mlk():
    from paper_2512_06173_amd import mlk as m
    return m


def pair(n_tls, n_ml, seed):
    """Two identical sims (periodic 16^3 box) with two-level and multilevel emitters."""
    rng = np.random.default_rng(seed)
    tls = W.tls_ensemble(rng, n_tls, 0.0, 16.0, "superposition")
    ml = W.random_multilevel(rng, n_ml, rng.uniform(0.0, 16.0, (n_ml, 3))) if n_ml else None
    sims = []
    for _ in range(2):
        s = mlk().Simulation((16, 16, 16), bc=("periodic",) * 6)
        s.add_tls(tls.pos, tls.sigma, tls.gamma, tls.omega0, tls.dipole, tls.rho0)
        if ml is not None:
            s.add_multilevel(ml.nlev, ml.energies, ml.mop, ml.dipole, ml.gphi, ml.rho0, ml.pos,
                             ml.sigma, ml.gamma)
        sims.append(s)
    return sims


def check_same(a, b, M):
    assert np.array_equal(a.tls_state(0, a.n_tls), b.tls_state(0, b.n_tls))
    for m in range(a.n_tls, M):
        assert np.array_equal(a.rho(m), b.rho(m))
    ea, ma = a.emitter_io()
    eb, mb = b.emitter_io()
    assert np.array_equal(ea, eb) and np.array_equal(ma, mb)


def test_noalloc_matches_the_allocating_entry_point_twice():
    rng = np.random.default_rng(11)
    # first call: 60,500 emitters, 23 steps; a step stages 361,500 doubles, so the
    # 2,097,152-double array takes 5 steps at a time (5 + 5 + 5 + 5 + 3)
    for n_tls, n_ml, steps in [(60000, 500, 23), (1000, 50, 7)]:
        print(f"[noalloc] {n_tls} two-level + {n_ml} multilevel emitters, {steps} steps",
              flush=True)
        ref, new = pair(n_tls, n_ml, n_tls)
        M = n_tls + n_ml
        Et = 0.2 * rng.standard_normal((steps, M, 3))
        out_ref = ref.step_prescribed(Et, record=True)
        out_new = new.step_prescribed_noalloc(Et, record=True)
        assert out_new.shape == (steps, n_tls, 3)
        assert np.array_equal(out_ref, out_new)
        assert np.any(out_new[-1] != out_new[0])
        check_same(ref, new, M)
        # and without recording
        Et2 = 0.1 * rng.standard_normal((3, M, 3))
        ref.step_prescribed(Et2)
        new.step_prescribed_noalloc(Et2)
        check_same(ref, new, M)
        ref.close()
        new.close()


def test_noalloc_refuses_sizes_beyond_its_array():
    n = 349526  # 6 n doubles per recorded step > 2,097,152
    s = mlk().Simulation((16, 16, 16), bc=("periodic",) * 6)
    rng = np.random.default_rng(3)
    t = W.tls_ensemble(rng, n, 0.0, 16.0, "superposition")
    s.add_tls(t.pos, t.sigma, t.gamma, t.omega0, t.dipole, t.rho0)
    Et = np.zeros((1, n, 3))
    with pytest.raises(mlk().MlkError) as e:
        s.step_prescribed_noalloc(Et, record=True)
    assert e.value.status == 1  # MLK_EINVAL
    s.step_prescribed_noalloc(Et)  # 3 n doubles per step fit
    s.close()
