"""Parity at the stated step counts of the full-size workloads: the library (FP32 fields
and FP64) after 5000 steps of the slab, 20,000 of the Bragg resonator, 2000 of the
64-domain batch (hipGraph replays) and 4000 of the 256^3 radiating cube, against the
FP64 CPU oracle's values stored under tests/golden (written by make_goldens.py, which
runs the oracle alone).  Fields are compared on the stored cells (all six components,
relative L2) and on one whole z plane, plus each component's L2 norm over the grid;
probe and flux series by relative L2; populations of the stored emitters by max
absolute difference.  Bounds: FP64 1e-12; FP32 fields 1e-4 (relative), populations
1e-6 (absolute).

One reading: when the field left in the grid at the end has decayed to less than 1e-3
of its largest norm during the run (the slab, once the pulse has left: 49,000-fold),
the field error is measured against that largest norm, in both precisions.  Rounding
in each E and H update breaks the discrete divergence identity of the Yee scheme by
a rounding error per cell and step, and what is deposited while the pulse sweeps the
grid is a static field that never leaves.  Any two correct implementations that round
differently leave different such fields: about 3.5e-7 of the pulse's norm between FP32
and the oracle (1.7e-2 against the small remainder), and 8e-16 between the library's
FP64 mode and the oracle (4e-11 against the remainder).  The test prints both measures."""
import importlib.util
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")
FP64_TOL, FP32_FIELD_TOL, FP32_POP_TOL = 1e-12, 1e-4, 1e-6
DECAYED = 1e-3


def mlk():
    from paper_2512_06173_amd import mlk as m
    return m


def goldens():
    spec = importlib.util.spec_from_file_location("make_goldens",
                                                  os.path.join(GOLDEN, "make_goldens.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def load(name):
    path = os.path.join(GOLDEN, f"{name}.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not written")
    return np.load(path)


def rel_l2(a, b):
    a, b = np.ravel(a), np.ravel(b)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a - b)


def compare(sim, w, z, prefix, fp64, label):
    ft = FP64_TOL if fp64 else FP32_FIELD_TOL
    pt = FP64_TOL if fp64 else FP32_POP_TOL
    f = sim.fields()
    idx = z[prefix + "sample_idx"]
    got = np.stack([a.ravel()[idx] for a in f])
    ref = z[prefix + "fields_sample"]
    errs = {"sample": rel_l2(got, ref)}
    norms = np.array([np.linalg.norm(a) for a in f])
    ref_n = z[prefix + "norms"]
    errs["norms"] = np.max(np.abs(norms - ref_n) / np.maximum(ref_n, 1e-300))
    plane = None
    if prefix + "plane" in z:
        k = int(z[prefix + "plane_k"])
        plane = np.stack([a[k] for a in f])
        errs["plane"] = rel_l2(plane, z[prefix + "plane"])
    info = {}
    if prefix + "norm_series" in z:
        ns = z[prefix + "norm_series"]
        peak = float(np.max(ns))
        if np.linalg.norm(ref_n) < DECAYED * peak:
            # decayed field: the grid-wide difference (estimated from the sampled cells)
            # and the plane's, against the run's largest field norm
            ncell = f[0].size
            info["sample (literal)"] = errs.pop("sample")
            info["norms (literal)"] = errs.pop("norms")
            errs["sample/peak"] = np.linalg.norm(got - ref) * np.sqrt(ncell / idx.size) / peak
            if plane is not None:
                info["plane (literal)"] = errs.pop("plane")
                errs["plane/peak"] = np.linalg.norm(plane - z[prefix + "plane"]) * \
                    np.sqrt(ncell / plane[0].size) / peak
            info["decay"] = np.linalg.norm(ref_n) / peak
    for p in range(len(w.probes)):
        errs[f"probe{p}"] = rel_l2(sim.probe(p), z[prefix + f"probe{p}"])
    if w.flux is not None:
        errs["flux"] = rel_l2(sim.flux_series(), z[prefix + "flux"])
        ft_ref = float(z[prefix + "flux_total"])
        errs["flux_total"] = abs(sim.flux_total() - ft_ref) / abs(ft_ref)
    line = ", ".join(f"{k} {v:.2e}" for k, v in list(errs.items()) + list(info.items()))
    pop_err = None
    if prefix + "pop" in z:
        g = goldens()
        pop = g.select_populations(sim.populations(), w, z[prefix + "pop_emitters"])
        assert pop.shape == z[prefix + "pop"].shape
        pop_err = float(np.max(np.abs(pop - z[prefix + "pop"])))
        line += f", populations {pop_err:.2e}"
    say(f"[longrun] {label}: {line}")
    for k, v in errs.items():
        assert v <= ft, (k, v)
    if pop_err is not None:
        assert pop_err <= pt


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("name", ["slab", "bragg", "cube"])
def test_full_size_at_stated_steps(name, precision):
    z = load(name)
    w = goldens().workload(name)
    w.precision = precision
    steps = int(z["steps"])
    say(f"[longrun] {name} {precision}: {steps} steps")
    sim = mlk().from_workload(w, stream=mlk().current_stream_handle())
    sim.autotune()
    sim.step(steps)
    sim.sync()
    compare(sim, w, z, "", precision == "fp64", f"{name} {precision} {steps} steps")
    sim.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batch_at_stated_steps_from_graph_replays(precision):
    """The 64 domains batched, batch-tuned and stepped by hipGraph replays of 100 steps,
    as the benchmark runs them; every member against its own golden values."""
    z = load("batch")
    ws = goldens().workload("batch")
    steps = int(z["steps"])
    say(f"[longrun] batch {precision}: {len(ws)} domains, {steps} steps")
    h = mlk().current_stream_handle()
    sims = []
    for w in ws:
        w.precision = precision
        sims.append(mlk().from_workload(w, stream=h))
    with mlk().Batch(sims) as b:
        b.autotune()
        b.capture(100)
        b.replay(steps // 100)
        b.sync()
    for i, (w, s) in enumerate(zip(ws, sims)):
        compare(s, w, z, f"d{i}_", precision == "fp64", f"batch domain {i} {w.shape} {precision}")
    for s in sims:
        s.close()
