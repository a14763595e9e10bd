"""Write the long-run expected values of the full-size workloads with the FP64 CPU
oracle (and nothing else): the slab (128^3, 5000 steps), the Bragg resonator
(64x64x1024, 20,000 steps), the 64-domain batch (2000 steps) and the radiating cube
(256^3, 100,000 emitters, 4000 steps).  The GPU tests compare the library with these
files at the same step counts.

Usage:  python tests/golden/make_goldens.py [slab|bragg|batch|cube ...] [--threads N]

Each file ``<name>.npz`` holds, in FP64:
  * ``steps``, ``pop_every``, ``threads`` and ``seconds`` (the oracle's wall time);
  * ``norm_steps`` and ``norm_series``: the whole-grid L2 norm of the six components
    along the run (the field's own scale, against which a late, decayed field is read);
  * ``sample_idx`` (cell indices, x fastest) and ``fields_sample`` (6 x S: Ex..Hz at
    those cells, E^n and H^{n-1/2} after the last step);
  * ``norms`` (6: the L2 norm of each whole component array);
  * ``plane_k`` and ``plane`` (6 x ny x nx: every component on one z plane);
  * ``probe<i>`` (each probe's series), ``flux`` and ``flux_total`` where the workload
    has a flux plane;
  * ``pop_emitters`` (emitter ids) and ``pop`` (records x their excited-level
    populations, in record order, each emitter's levels 1..n-1).
The batch file holds the same per domain with a ``d<i>_`` prefix (no plane).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from oracle.feed import build_oracle  # noqa: E402
from paper_2512_06173_amd import workloads as W  # noqa: E402

# What each golden run uses: the workload, the population record interval, the field
# samples, the emitters whose populations are kept and the z plane stored whole.
SPECS = {
    "slab": dict(make=lambda: W.slab(), pop_every=100, n_sample=32768, n_pop=1000,
                 plane_k=64, norm_every=50),
    "bragg": dict(make=lambda: W.bragg(), pop_every=1000, n_sample=32768, n_pop=1000,
                  plane_k=None),
    "cube": dict(make=lambda: W.radiating_cube(), pop_every=400, n_sample=32768, n_pop=2000,
                 plane_k=128),
    "batch": dict(make=lambda: W.batch(), pop_every=100, n_sample=2048, n_pop=256,
                  plane_k=None),
}
SAMPLE_SEED = 20251206


def workload(name):
    """The workload of a golden run (FP32 fields, as the benchmark runs it; the oracle is
    FP64 whatever the workload says) with its record interval set."""
    spec = SPECS[name]
    ws = spec["make"]()
    for w in ws if isinstance(ws, list) else [ws]:
        w.pop_every = spec["pop_every"]
    return ws


def bragg_plane(w):
    """The z plane through the middle of the Bragg defect (where the probe sits)."""
    return w.probes[0][1][2]


def sample_cells(ncell, n, seed):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(ncell, size=min(n, ncell), replace=False)).astype(np.int64)


def pop_emitters(w, n, seed):
    ne = w.n_emitters
    rng = np.random.default_rng(seed + 1)
    return np.sort(rng.choice(ne, size=min(n, ne), replace=False)).astype(np.int64)


def level_counts(w):
    """Number of levels of each emitter in id order (two-level emitters first, as both
    the oracle and the library number them)."""
    nt = len(w.tls) if w.tls is not None else 0
    nl = [2] * nt
    if w.multilevel is not None:
        nl += [int(v) for v in w.multilevel.nlev]
    return np.array(nl, dtype=np.int64)


def select_populations(pop, w, ids):
    """Rows of the population record (records x all excited levels) restricted to the
    excited levels of the emitters in ids."""
    nl = level_counts(w)
    off = np.concatenate([[0], np.cumsum(nl - 1)])
    cols = np.concatenate([np.arange(off[m], off[m + 1]) for m in ids])
    return pop.reshape(-1, off[-1])[:, cols]


def record(o, w, spec, prefix, out, seed):
    nx, ny, nz = w.shape
    f = o.fields()
    idx = sample_cells(w.ncell, spec["n_sample"], seed)
    out[prefix + "sample_idx"] = idx
    out[prefix + "fields_sample"] = np.stack([a.ravel()[idx] for a in f])
    out[prefix + "norms"] = np.array([np.linalg.norm(a) for a in f])
    if spec.get("plane_k") is not None:
        k = spec["plane_k"]
        out[prefix + "plane_k"] = np.int64(k)
        out[prefix + "plane"] = np.stack([a[k] for a in f])
    for p in range(len(w.probes)):
        out[prefix + f"probe{p}"] = o.probe(p)
    if w.flux is not None:
        out[prefix + "flux"] = o.flux_series()
        out[prefix + "flux_total"] = np.float64(o.flux_total())
    if w.pop_every and w.n_emitters:
        ids = pop_emitters(w, spec["n_pop"], seed)
        out[prefix + "pop_emitters"] = ids
        out[prefix + "pop"] = select_populations(o.populations(), w, ids)


def field_norm(o):
    return float(np.sqrt(sum(np.sum(a * a) for a in o.fields())))


def run_stepped(o, steps, label, out=None, prefix="", every=None):
    """Step in chunks, keeping the whole-grid L2 norm of the six components after each
    chunk (norm_steps, norm_series) when out is given."""
    t0 = time.time()
    chunk = every or max(1, steps // 20)
    done = 0
    nsteps, norms = [], []
    while done < steps:
        n = min(chunk, steps - done)
        o.step(n)
        done += n
        if out is not None:
            nsteps.append(done)
            norms.append(field_norm(o))
        print(f"[golden] {label}: {done}/{steps} steps, {time.time() - t0:.0f} s", flush=True)
    if out is not None:
        out[prefix + "norm_steps"] = np.array(nsteps, dtype=np.int64)
        out[prefix + "norm_series"] = np.array(norms)
    return time.time() - t0


def make(name, threads):
    spec = dict(SPECS[name])
    if name == "bragg":
        spec["plane_k"] = bragg_plane(workload(name))
    out = {"pop_every": np.int64(spec["pop_every"]), "threads": np.int64(threads)}
    if name == "batch":
        ws = workload(name)
        out["steps"] = np.int64(ws[0].steps)
        secs = 0.0
        for i, w in enumerate(ws):
            o = build_oracle(w)
            secs += run_stepped(o, w.steps, f"batch domain {i} {w.shape}", out, f"d{i}_",
                                spec.get("norm_every"))
            record(o, w, spec, f"d{i}_", out, SAMPLE_SEED + i)
            del o
        out["seconds"] = np.float64(secs)
    else:
        w = workload(name)
        o = build_oracle(w)
        out["steps"] = np.int64(w.steps)
        out["seconds"] = np.float64(run_stepped(o, w.steps, name, out, "",
                                                spec.get("norm_every")))
        record(o, w, spec, "", out, SAMPLE_SEED)
    path = os.path.join(HERE, f"{name}.npz")
    np.savez_compressed(path, **out)
    print(f"[golden] wrote {path} ({os.path.getsize(path) / 1e6:.1f} MB)", flush=True)


def main(argv):
    threads = O.threads()
    names = []
    it = iter(argv)
    for a in it:
        if a == "--threads":
            threads = int(next(it))
        else:
            names.append(a)
    O.set_threads(threads)
    for name in names or list(SPECS):
        make(name, threads)


if __name__ == "__main__":
    main(sys.argv[1:])
