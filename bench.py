"""Throughput of the coupled Yee / quantum-emitter step on one MI355X.

One step is one pass of the whole coupled leapfrog (H update, field gather,
emitter step, dipole rate, current scatter, E update, sources, detectors)
over the radiating-cube workload: a 256^3 grid with 10-cell CPML on every
face, 100,000 two-level emitters in the central 128^3 box starting in the
superposition state, and a Poynting-flux plane at z = 200.  Fields are FP32,
emitter states FP64; everything stays on the device.

Prints ONE JSON line: Gcell-updates/s of the fused FP32 step (the value),
emitter-steps/s, the fused/plain FP32/FP64 comparison on the same GPU, the
roofline of the dominant kernel (the fused interior sweep) measured with HIP
events on the library's stream, and the CPU oracle timed on the host cores
on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--no-cpu] [--no-compare] [--no-batch]
                    [--no-adjoint] [--adjoint-steps N]
    python bench.py --copy-calib     # plain copy kernel of known size (counter scaling)
"""
import argparse
import copy
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# the CPU baseline's threads stay on neighbouring cores (read when OpenMP starts)
os.environ.setdefault("OMP_PROC_BIND", "close")

HBM_PEAK_GBS = 8000.0
FUSED_SRC = os.path.join(ROOT, "paper_2512_06173_amd", "csrc", "yee_fused.hip")
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_fused_f32_radiating_cube_256_traffic.md")
# Algorithmic bytes, per unit (see the roofline section of the design notes):
#   cell-step: read + write of the 6 field components and one read of 1/eps_r
#   (credited also in vacuum, where the fused sweep skips that read)
#   CPML layer membership: read + write of the 4 psi values of that axis
#   two-level emitter step: state, parameters, E~ and mu_dot
CELL_WORDS = 13
PSI_WORDS = 8
TLS_STEP_BYTES = 100


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=1000)
    p.add_argument("--warmup", type=int, default=50)
    p.add_argument("--n", type=int, default=256, help="grid edge (cells)")
    p.add_argument("--emitters", type=int, default=100000)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--no-compare", action="store_true", help="skip the plain/FP64 legs")
    p.add_argument("--cpu-steps", type=int, default=30)
    p.add_argument("--no-batch", action="store_true", help="skip the 64-domain batch leg")
    p.add_argument("--no-adjoint", action="store_true", help="skip the adjoint leg")
    p.add_argument("--adjoint-steps", type=int, default=4000)
    p.add_argument("--copy-calib", action="store_true")
    p.add_argument("--dispersive-only", action="store_true",
                   help="only the leg with a Lorentz pole block (profiling runs; needs --tile)")
    p.add_argument("--cavity-only", action="store_true",
                   help="only the leg with the emitters in one cavity mode (profiling runs)")
    p.add_argument("--batch-only", action="store_true",
                   help="only the 64-domain batch leg (profiling runs)")
    p.add_argument("--tile", type=lambda v: tuple(int(x) for x in v.split(",")), default=None,
                   help="fused tile TY,KZ[,TX[,LAYER_MODE]] instead of autotuning (profiling runs)")
    return p.parse_args()


def box_memberships(lo, hi, shape, cpml):
    """Sum over axes of the cells of the box [lo, hi) lying in that axis's CPML layers."""
    tot = 0
    for a in range(3):
        n, nlo, nhi = shape[a], cpml[2 * a], cpml[2 * a + 1]
        in_layers = sum(1 for q in range(lo[a], hi[a]) if q < nlo or q >= n - nhi)
        other = 1
        for b in range(3):
            if b != a:
                other *= hi[b] - lo[b]
        tot += in_layers * other
    return tot


def layer_memberships(shape, cpml):
    """Sum over axes of the cells lying in that axis's CPML layers."""
    nx, ny, nz = shape
    n = (nx, ny, nz)
    tot = 0
    for a in range(3):
        lo, hi = cpml[2 * a], cpml[2 * a + 1]
        tot += (lo + hi) * (nx * ny * nz // n[a])
    return tot


def copy_calibration():
    """Achievable streaming bandwidth: torch's copy and the library's hand-written
    streaming copy (four cache-policy variants, several grid sizes) of 256 MiB and
    1 GiB, each timed with events over 20 launches (median).  Bytes moved = 2 x size."""
    import torch
    from paper_2512_06173_amd import mlk
    out = {"unit": "GB/s", "runs": []}
    for nbytes in (256 << 20, 1 << 30):
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)

        def timed(fn, reps=20):
            ts = []
            for _ in range(3):
                fn()
            for _ in range(reps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                fn()
                e1.record()
                e1.synchronize()
                ts.append(e0.elapsed_time(e1) * 1e-3)
            ts.sort()
            return 2 * nbytes / ts[len(ts) // 2] / 1e9

        out["runs"].append({"bytes": nbytes, "kernel": "torch copy_",
                            "GBs": round(timed(lambda: b.copy_(a)), 1)})
        for variant in range(4):
            for blocks in (1024, 2048, 4096, 8192, 16384):
                gbs = timed(lambda: mlk.stream_copy(a, b, variant, blocks))
                out["runs"].append({"bytes": nbytes, "kernel": "mlk_stream_copy",
                                    "variant": variant, "blocks": blocks, "GBs": round(gbs, 1)})
        assert torch.equal(a, b)
        del a, b
    best = max(out["runs"], key=lambda r: r["GBs"])
    out["best"] = best
    print(json.dumps(out), flush=True)


def traffic_from_profile(launch_cells, tile):
    """HBM bytes per launch of the fused kernel from the committed counter summary,
    or None when it is absent, was taken on a different kernel source or box, or
    holds no line for this tile (tx, ty, kz, layer mode)."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    txt = open(TRAFFIC_SUMMARY).read()
    want = hashlib.sha256(open(FUSED_SRC, "rb").read()).hexdigest()
    m = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", txt)
    c = re.search(r"cells_per_launch:\s*(\d+)", txt)
    if not (m and c) or m.group(1) != want or int(c.group(1)) != launch_cells:
        return None
    for k in re.finditer(r"tile_traffic:\s*(\d+)\s+(\d+)\s+(\d+)\s+(\d+)\s+([0-9.eE+]+)", txt):
        if tuple(int(v) for v in k.groups()[:4]) == tuple(tile):
            return float(k.group(5))
    return None


def run_gpu(w, precision, sweep, steps, warmup, timing, tile=None, poles=()):
    import torch
    from paper_2512_06173_amd import mlk
    sim = mlk.from_workload(w, precision=precision, sweep=sweep, scatter="owner",
                            stream=mlk.current_stream_handle())
    for box, w0, gamma, sigma, drude in poles:
        sim.add_susceptibility(box, w0, gamma, sigma, drude=drude)
    if tile:
        sim.set_tuning(*tile[:2])
        if len(tile) > 2:
            sim.set_tile_width(tile[2])
        if len(tile) > 3:
            sim.set_sweep_layers(tile[3])
    else:
        sim.autotune()  # tile shape of the fused sweep (untimed; plain sweeps have none)
    sim.step(warmup)
    sim.sync()
    sim.set_timing(timing or False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    phases = {}
    if timing:
        for name in mlk.PHASES:
            ms, n = sim.phase_time(name)
            if n:
                phases[name] = (ms, n)
    box = sim.interior_box()
    tuning = sim.tuning() + (sim.tile_width(), sim.sweep_layers())
    sim.close()
    return dt, phases, box, tuning


def batch_leg(steps, spr=20):
    """64 independent domains (edges 32..96, CPML 8, 1..256 TLS each, FP32 fields),
    batched (one launch per phase, replayed from a captured hipGraph), with both sweeps:
    the fused sweep (one tile shape and layer mode for all members, chosen by the batch
    tuner) and the plain one; the faster is the leg's headline.  Against it: the same
    domains stepped one after another on one stream, and (context) each domain on a
    stream of its own, so that their launches overlap."""
    import torch
    from paper_2512_06173_amd import mlk, workloads as W
    ws = W.batch(n_domains=64, steps=0)
    cells = sum(w.shape[0] * w.shape[1] * w.shape[2] for w in ws)
    nem = sum(w.n_emitters for w in ws)
    # one stream for every domain (torch's default stream has a null handle, which
    # would give each sim a stream of its own)
    one = torch.cuda.Stream()
    h = mlk.C.c_void_p(one.cuda_stream)
    reps = max(1, steps // spr)
    nsteps = reps * spr

    def timed(run):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    rate = lambda t: {"gcell_updates_per_s": round(cells * nsteps / t / 1e9, 3),
                      "ms_per_step": round(t * 1e3 / nsteps, 4)}
    legs, tuned = {}, None
    for sweep in ("fused", "plain"):
        sims = [mlk.from_workload(w, stream=h, sweep=sweep) for w in ws]
        b = mlk.Batch(sims)
        if sweep == "fused":
            tuned = b.autotune()
        b.step(2)
        b.capture(spr)
        b.replay(1)
        b.sync()
        legs[sweep] = timed(lambda: (b.replay(reps), b.sync()))
        b.close()
        for s in sims:
            s.close()
    best = min(legs, key=legs.get)

    def one_by_one(sims):
        for s in sims:
            s.step(nsteps)
        for s in sims:
            s.sync()

    sims = [mlk.from_workload(w, stream=h, sweep=best) for w in ws]
    if best == "fused":
        for s in sims:
            s.set_tuning(tuned[0], tuned[1])
            s.set_sweep_layers(tuned[2])
            s.set_tile_width(tuned[3])
    for s in sims:
        s.step(2)
    tu = timed(lambda: one_by_one(sims))
    for s in sims:
        s.close()
    sims = [mlk.from_workload(w, sweep=best) for w in ws]  # library-owned stream each
    for s in sims:
        s.step(2)
    tc = timed(lambda: one_by_one(sims))
    for s in sims:
        s.close()
    return {"workload": f"{len(ws)} cubic domains, edges 32..96 (8 x U{{4..12}}), CPML 8, "
                        f"eps per 8^3 block, {nem} TLS in all; FP32 fields",
            "cells": cells, "emitters": nem, "steps": nsteps, "sweep": best,
            "batch_tuning": {"tx": tuned[3], "ty": tuned[0], "kz": tuned[1],
                             "layers": int(tuned[2])},
            "batched_graph": rate(legs[best]),
            "batched_graph_by_sweep": {k: rate(v) for k, v in legs.items()},
            "one_by_one": rate(tu), "speedup": round(tu / legs[best], 2),
            "own_streams": rate(tc), "speedup_vs_own_streams": round(tc / legs[best], 2)}


# Algorithmic bytes per pole cell and step (FP32): the pre-sweep pass reads E, P, Q and
# writes Q (4 words per component), the post pass reads E, Q, P and writes E, P (5 per
# component), and 1/eps_inf is read once per cell.
POLE_BYTES_PER_CELL = 3 * 9 * 4 + 4


def dispersive_leg(w, steps, tuning, ms_plain):
    """The same workload with a Lorentz pole over the central eighth of the domain."""
    n = w.shape[0]
    lo, hi = n // 4, 3 * n // 4
    poles = [((lo, lo, lo, hi, hi, hi), 0.3, 0.01, 1.5, False)]
    d, ph, _, _ = run_gpu(w, "fp32", "fused", steps, 5, ["poles"], tuning, poles)
    ms, nl = ph["poles"]
    cells = (hi - lo) ** 3
    t_pair = ms / (nl / 2) * 1e-3  # pre + post per step
    achieved = cells * POLE_BYTES_PER_CELL / t_pair / 1e9
    return {"pole_cells": cells, "ms_per_step": round(d * 1e3 / steps, 4),
            "extra_ms_per_step": round(d * 1e3 / steps - ms_plain, 4),
            "pole_passes_us_per_step": round(t_pair * 1e6, 2),
            "bytes_per_pole_cell": POLE_BYTES_PER_CELL,
            "pole_passes_GBs": round(achieved, 1),
            "frac_of_hbm_peak": round(achieved / HBM_PEAK_GBS, 4), "steps": steps}


def cavity_leg(w, steps):
    """The workload's emitters in one cavity mode instead of the grid (FP64 states)."""
    import torch
    from paper_2512_06173_amd import mlk
    w = copy.copy(w)
    w.flux, w.probes, w.pop_every = None, [], 0
    sim = mlk.from_workload(w, stream=mlk.current_stream_handle())
    sim.set_cavity(0.25, 2.0e4, (0.05, 0.0), (0.0, 0.0))
    sim.step(10)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    dt = time.perf_counter() - t0
    nem = len(w.tls.pos)
    sim.close()
    return {"emitters": nem, "steps": steps, "ms_per_step": round(dt * 1e3 / steps, 4),
            "emitter_steps_per_s": round(nem * steps / dt, 1)}


def adjoint_leg(w, steps, ms_forward, ckpt=200):
    """Gradients of the time-integrated flux through the z = 200 plane over `steps`
    steps with respect to eps_r in the design box [96,160)^3 and every emitter's dipole,
    checkpoint every `ckpt` steps.  Ratio = reverse pass (segment recomputation +
    adjoint steps + gradient accumulation) / plain forward steps of the same count."""
    from paper_2512_06173_amd import mlk
    sim = mlk.from_workload(w, stream=mlk.current_stream_handle())
    db = w.design_box  # (x0, x1, y0, y1, z0, z1)
    box = ((db[0], db[2], db[4]), (db[1], db[3], db[5]))
    t0 = time.perf_counter()
    sim.adjoint("flux", steps, box, checkpoint_every=ckpt)
    wall = time.perf_counter() - t0
    f_ms, r_ms = sim.adjoint_times()
    sim.close()
    plain = ms_forward * steps
    return {"workload": f"flux through z={w.flux[1]} over {steps} steps; d/d eps_r on the "
                        f"design box {box[0]}..{box[1]} and d/d dipole of {len(w.tls.pos)} "
                        f"emitters; checkpoint every {ckpt} steps",
            "forward_with_checkpoints_ms": round(f_ms, 2), "reverse_ms": round(r_ms, 2),
            "plain_forward_ms": round(plain, 2), "wall_s": round(wall, 2),
            "adjoint_forward_ratio": round(r_ms / plain, 3),
            "total_forward_ratio": round((f_ms + r_ms) / plain, 3)}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, steps, slab_steps=6):
    """The FP64 oracle on the host cores: a bounded sample of the benchmark workload with
    every thread, and the 128^3 slab workload (1000 emitters and the plane-wave source)
    with one thread."""
    from oracle import oracle
    from oracle.feed import build_oracle
    from paper_2512_06173_amd import workloads as W
    oracle.build()
    threads = oracle.threads()
    ora = build_oracle(w)
    ora.step(1)  # first touch of the arrays
    t0 = time.perf_counter()
    ora.step(steps)
    dt = time.perf_counter() - t0
    del ora
    cells = w.shape[0] * w.shape[1] * w.shape[2]
    sl = W.slab()
    oracle.set_threads(1)
    o1 = build_oracle(sl)
    o1.step(1)
    t1 = time.perf_counter()
    o1.step(slab_steps)
    d1 = time.perf_counter() - t1
    oracle.set_threads(threads)
    return {"value": cells * steps / dt / 1e9, "unit": "Gcell-updates/s",
            "cores": threads, "kind": "oracle",
            "sample": f"{steps} steps of the same {w.shape[0]}x{w.shape[1]}x{w.shape[2]} "
                      f"workload with all {len(w.tls.pos)} emitters (FP64, after 1 untimed "
                      f"step); {dt:.1f} s",
            "emitter_steps_per_s": len(w.tls.pos) * steps / dt,
            "cpu_model": cpu_model(), "omp_proc_bind": os.environ.get("OMP_PROC_BIND"),
            "one_thread_slab_128": {
                "gcell_updates_per_s": sl.ncell * slab_steps / d1 / 1e9,
                "sample": f"{slab_steps} steps of the 128^3 slab workload (1000 emitters, "
                          f"plane-wave source), one thread; {d1:.1f} s"}}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print("bench.py measures one GPU: multi-GPU sharding of the grid is described in the "
              "design notes but not built; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.copy_calib:
        copy_calibration()
        return
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    from paper_2512_06173_amd import workloads as W
    from paper_2512_06173_amd import mlk
    mlk.lib()

    w = W.radiating_cube(n=args.n, n_emit=args.emitters)
    if args.batch_only:
        print(json.dumps({"batch": batch_leg(max(100, args.steps))}), flush=True)
        return
    if args.cavity_only:
        print(json.dumps({"cavity": cavity_leg(w, args.steps)}), flush=True)
        return
    if args.dispersive_only:
        print(json.dumps({"dispersive": dispersive_leg(w, args.steps, args.tile, 0.0)}), flush=True)
        return
    nx, ny, nz = w.shape
    cells = nx * ny * nz
    nem = len(w.tls.pos)
    esz = 4
    memb = layer_memberships(w.shape, w.cpml)
    step_bytes = cells * CELL_WORDS * esz + memb * PSI_WORDS * esz + nem * TLS_STEP_BYTES

    # timed region: events around the fused sweep launch only
    dt, phases, box, tuning = run_gpu(w, "fp32", "fused", args.steps, args.warmup, ["sweep"],
                                      args.tile)
    # per-phase breakdown from a separate, shorter run with every phase timed
    _, breakdown, _, _ = run_gpu(w, "fp32", "fused", max(1, args.steps // 5), 5, True,
                                 tuning)
    ms_step = dt * 1e3 / args.steps
    gcells = cells * args.steps / dt / 1e9
    emit_rate = nem * args.steps / dt

    # dominant kernel: the fused interior sweep (one launch per step)
    sweep_ms, sweep_n = phases["sweep"]
    lo, hi = box
    launch_cells = (hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2])
    # a cell of the launch also reads and writes 8 psi words per CPML layer it lies in
    launch_memb = box_memberships(lo, hi, w.shape, w.cpml)
    launch_bytes = launch_cells * CELL_WORDS * esz + launch_memb * PSI_WORDS * esz
    t_launch = sweep_ms / sweep_n * 1e-3
    achieved = launch_bytes / t_launch / 1e9
    traffic = traffic_from_profile(launch_cells, (tuning[2], tuning[0], tuning[1], tuning[3]))
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "kernel": f"k_fused<float, {tuning[2]}, {tuning[0]}>",
                "tile": {"tx": tuning[2], "ty": tuning[0], "kz": tuning[1],
                         "layer_mode": tuning[3]},
                "cells_per_launch": launch_cells, "bytes_per_launch": launch_bytes,
                "avg_launch_us": round(t_launch * 1e6, 2)}
    emitter_ms = sum(breakdown[p][0] / breakdown[p][1] for p in ("emitters", "scatter")
                     if p in breakdown)
    out = {
        "metric": "Gcell-updates/s + emitter-steps/s (fused vs plain FP64); adjoint/forward "
                  "time ratio",
        "value": round(gcells, 3), "unit": "Gcell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"radiating cube {nx}^3, CPML 10 on 6 faces, {nem} two-level "
                               f"emitters in the central box, flux plane z={w.flux[1]}; "
                               f"FP32 fields, FP64 emitter states",
                   "cells": cells, "emitters": nem, "sweep": "fused", "scatter": "owner"},
        "emitter_steps_per_s": round(emit_rate, 1),
        "emitter_phase_steps_per_s": round(nem / (emitter_ms * 1e-3), 1) if emitter_ms else None,
        "step_roofline": {"bytes_per_step": step_bytes,
                          "achieved_GBs": round(step_bytes / (ms_step * 1e-3) / 1e9, 1),
                          "frac": round(step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "phases_us_per_step": {k: round(v[0] * 1e3 / v[1], 2) for k, v in breakdown.items()},
        "roofline": roofline,
        "adjoint_forward_ratio": None,
    }
    if not args.no_compare:
        cmp = {}
        ksteps = max(100, args.steps // 5)
        for prec, sweep in (("fp32", "plain"), ("fp64", "fused"), ("fp64", "plain")):
            d, _, _, _ = run_gpu(w, prec, sweep, ksteps, max(1, args.warmup // 2), False)
            cmp[f"{sweep}_{prec}"] = {"gcell_updates_per_s": round(cells * ksteps / d / 1e9, 3),
                                      "emitter_steps_per_s": round(nem * ksteps / d, 1),
                                      "ms_per_step": round(d * 1e3 / ksteps, 4),
                                      "steps": ksteps}
        cmp["fused_fp32"] = {"gcell_updates_per_s": round(gcells, 3),
                             "emitter_steps_per_s": round(emit_rate, 1),
                             "ms_per_step": round(ms_step, 4), "steps": args.steps}
        out["comparison"] = cmp
    if not args.no_adjoint:
        adj = adjoint_leg(w, args.adjoint_steps, ms_step)
        out["adjoint"] = adj
        out["adjoint_forward_ratio"] = adj["adjoint_forward_ratio"]
    if not args.no_batch:
        out["batch"] = batch_leg(max(100, args.steps // 5))
    if not args.no_compare:
        out["dispersive"] = dispersive_leg(w, max(20, args.steps // 5), tuning, ms_step)
        out["cavity"] = cavity_leg(w, max(20, args.steps // 5))
    out["cpu_baseline"] = None if args.no_cpu else cpu_baseline(w, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
