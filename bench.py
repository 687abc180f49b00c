"""Throughput of the adaptive PBF step on one MI355X.

Workload: the 1,048,576-particle tank (128 x 64 x 128 lattice, spacing
0.05, h = 0.1, velocities N(0, 0.1^2), box 6.4^3) with distance-to-camera
levels N_i in {5..10}.  One step = the whole hot path: levels, forces and
prediction, counting sort of cell keys with reorder, neighbour lists, level
buckets, the gated lambda / correction iterations, velocity and position
update.  Inputs are resident in HBM before the timed region; every step is
one hipGraph replay on the context's stream.

Prints ONE JSON line: particle-iterations/s (sum over steps of sum_i N_i,
counted on the device, divided by the timed wall time), ms/step, the same
for plain PBF with N = 10 and N = 5 on the same scene, the roofline of the
dominant kernel from HIP events around each of its launches, and the FP64
oracle's rate on the host cores over a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

METRIC = "particle-iterations/s and ms/step at 1M particles, APBF vs PBF(N=10)"

# FP32 operations per (active particle, neighbour) pair as written in the
# kernels (an FMA counts 2, max/select 0): lambda pass 26 (difference 3,
# |d|^2 5, poly6 term 4, rsqrt and r 2, spiky factor 3, gradient sum 6,
# squared norm 3); update pass 21 (difference 3, |d|^2 5, rsqrt and r 2,
# spiky factor and lambda sum 5, correction sum 6).
FLOP_PER_PAIR = {"lambda": 26.0, "update": 21.0}
# compulsory HBM bytes per active particle: lambda reads x* (16) and
# writes lambda (4); update reads x* and lambda (16 + 4) and writes x* (16)
BYTES_PER_ACTIVE = {"lambda": 20.0, "update": 36.0}
# bytes the kernel design moves per active particle-iteration besides the
# 16-byte neighbour-code groups (counted exactly, per group): metadata and
# slot 8, the result (lambda 4, position 16), and the particle's share of
# its tile's LDS stage, 6^3 cells staged for 4^3 own cells at 16 bytes an
# entry (3.375 x 16 = 54)
DESIGN_BYTES = {"lambda": {"per_active": 8.0 + 4.0 + 54.0},
                "update": {"per_active": 8.0 + 16.0 + 54.0}}
NBR_CAP = 256  # neighbour capacity of every tank run (APBF, DTVS, PBF): like for like
# A PBF run that compresses the tank beyond NBR_CAP neighbours is repeated at
# this capacity, and its entry says so (then it is not like for like).
NBR_CAP_RETRY = 2 * NBR_CAP
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3  # published vector FP32 peak (counts dual-issue)


TRAFFIC_FILE = ROOT / "profiles" / "tank_1m_traffic.json"


def kernel_sources_digest() -> str:
    """SHA-1 over the forward-step kernel sources: the key under which
    hardware-counter traffic figures are stored."""
    import hashlib
    h = hashlib.sha1()
    csrc = ROOT / "paper_1608_04721_amd" / "csrc"
    for name in ("pbf_internal.h", "pbf_kernels.hip"):
        h.update(name.encode())
        h.update((csrc / name).read_bytes())
    return h.hexdigest()


def _timed_run(sim, steps, warmup, stream, torch):
    sim.set_graph(True)
    sim.step(warmup)
    sim.sync()
    pit0 = sim.stats()["total_particle_iterations"] if warmup else 0
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    for k in range(steps):
        evs[k].record(stream)
        sim.step(1)
    evs[steps].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(steps)])
    total_ms = float(evs[0].elapsed_time(evs[steps]))
    sim.sync()
    st = sim.stats()
    pit = st["total_particle_iterations"] - pit0
    mean_rho, max_rho = sim.density()  # after the timed region
    return {"ms_per_step": total_ms / steps, "ms_median": float(np.median(per)),
            "wall_s": wall, "particle_iterations": int(pit),
            "value": pit / (total_ms * 1e-3), "mean_levels": pit / (steps * sim.n),
            "max_neighbours": st["max_neighbours"],
            "density": {"mean_rho_over_rho0": round(mean_rho, 6), "max_rho_over_rho0": round(max_rho, 6)}}


def _profile(sc, steps, Sim, stream, cap):
    """Per-kernel HIP-event timings over `steps` direct-launch steps, plus
    the exact pair counts of every lambda/update launch and the bytes the
    kernel design moves for them (see DESIGN_BYTES)."""
    sim = Sim(sc, stream=stream, max_neighbours=cap)
    sim.step(2)  # same warm start as the timed run's graphs
    sim.sync()
    sim.profile_enable(True)
    pairs = {"lambda": 0, "update": 0}
    active = {"lambda": 0, "update": 0}
    groups = 0
    launches = 0
    for _ in range(steps):
        sim.step(1)
        lv = sim.debug_levels().astype(np.int64)
        cnt = sim.debug_neighbour_counts().astype(np.int64)
        K = int(sc.n_max)
        for k in range(K):
            act = lv > k
            pairs["lambda"] += int(cnt[act].sum())
            pairs["update"] += int(cnt[act].sum())
            active["lambda"] += int(act.sum())
            active["update"] += int(act.sum())
            groups += int(((cnt[act] + 7) // 8).sum())
        launches += K
    prof = sim.profile_read()
    sim.close()
    design = {k: DESIGN_BYTES[k]["per_active"] * active[k] + 16.0 * groups
              for k in ("lambda", "update")}
    return prof, pairs, active, launches, design


def _counters(kernel, avg_s):
    """HBM traffic and VALU issue share of `kernel` from the committed
    counter runs (None when the kernel sources have changed since)."""
    try:
        rec = json.loads(TRAFFIC_FILE.read_text())
    except (OSError, ValueError):
        return None, None, None
    if rec.get("sources_sha1") != kernel_sources_digest():
        return None, None, None
    t = rec.get("bytes_per_dispatch", {}).get(kernel)
    v = rec.get("valu_issue", {}).get(kernel)
    return t, (round(t / rec["dispatch_s"][kernel] / 1e9 / PEAK_HBM_GBS, 4)
               if t and rec.get("dispatch_s", {}).get(kernel) else None), v


def _roofline(prof, pairs, active, design):
    tot = {k: v[0] for k, v in prof.items()}
    dom = max(("lambda", "update"), key=lambda k: tot[k])
    ms, n_launch = prof[dom]
    avg_s = ms * 1e-3 / n_launch
    flops = FLOP_PER_PAIR[dom] * pairs[dom] / n_launch
    bytes_ = BYTES_PER_ACTIVE[dom] * active[dom] / n_launch
    dbytes = design[dom] / n_launch
    tflops = flops / avg_s / 1e12
    gbs = bytes_ / avg_s / 1e9
    f_alu, f_hbm = tflops / PEAK_FP32_TFLOPS, gbs / PEAK_HBM_GBS
    traffic, hbm_frac, valu = _counters(dom, avg_s)
    if f_alu >= f_hbm:
        roof = {"bound": "alu", "achieved": round(tflops, 3), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": round(f_alu, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(f_hbm, 4)}
    roof.update({"traffic": traffic, "kernel": dom, "avg_launch_us": round(avg_s * 1e6, 2),
                 "algorithmic_bytes_per_launch": int(bytes_),
                 "algorithmic_flop_per_launch": int(flops),
                 "design_bytes_per_launch": int(dbytes),
                 "hbm_model_gbs": round(gbs, 1), "design_model_gbs": round(dbytes / avg_s / 1e9, 1),
                 "alu_tflops": round(tflops, 3),
                 "counter_hbm_frac": hbm_frac, "valu_issue_share": valu})
    kernels = {k: {"total_ms": round(v[0], 4), "launches": v[1],
                   "avg_us": round(1e3 * v[0] / v[1], 2) if v[1] else None}
               for k, v in prof.items() if v[1]}
    return roof, kernels


def _cpu_model() -> str:
    try:
        for line in Path("/proc/cpuinfo").read_text().splitlines():
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _oracle_rate(sc, steps, threads):
    import oracle
    oracle.set_threads(threads)
    x, v = sc.x0.astype(np.float64), sc.v0.astype(np.float64)
    pit = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        lv = oracle.levels(sc, x)
        pit += int(lv.sum())
        x, v, _ = oracle.apbf_step(sc, x, v)
    dt = time.perf_counter() - t0
    return pit / dt, dt, oracle.get_threads()


def _cpu_baseline(sc, steps, steps_1t=1):
    """The FP64 oracle on the host: every core (up to 16) over the first
    `steps` steps, and one thread over the first `steps_1t` steps, of the
    same workload from the same initial state."""
    import oracle
    oracle.build(force=False)
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, 16))
    rate, dt, used = _oracle_rate(sc, steps, cores)
    out = {"value": round(rate, 1), "unit": "particle-iterations/s",
           "cores": used, "kind": "oracle",
           "sample": f"first {steps} steps of the same {sc.n:,}-particle APBF workload "
                     f"from the same initial state ({dt:.1f} s)",
           "ms_per_step": round(1e3 * dt / steps, 1), "cpu_model": _cpu_model()}
    if steps_1t:
        rate1, dt1, _ = _oracle_rate(sc, steps_1t, 1)
        out["one_thread"] = {"value": round(rate1, 1), "ms_per_step": round(1e3 * dt1 / steps_1t, 1),
                             "sample": f"first {steps_1t} step(s), 1 thread ({dt1:.1f} s)"}
    return out


def _full_run(sc, steps, Sim, stream, torch, cap, **kw):
    """`steps` graph-replayed steps from the scene's initial state, timed as
    a whole with HIP events on the context stream; a device fault is
    reported with the first step that raised it (found again untimed, one
    synchronised step at a time)."""
    from paper_1608_04721_amd import PbfError
    with Sim(sc, stream=stream, max_neighbours=cap, **kw) as sim:
        sim.set_graph(True)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sim.step(steps)
        e1.record(stream)
        try:
            sim.sync()
        except PbfError as err:
            msg = str(err)
        else:
            ms = e0.elapsed_time(e1)
            st = sim.stats()
            pit = st["total_particle_iterations"]
            return {"steps": steps, "ms_per_step": round(ms / steps, 4),
                    "value": round(pit / (ms * 1e-3), 1),
                    "mean_levels": round(pit / (steps * sim.n), 4),
                    "max_neighbours_last_step": st["max_neighbours"]}
    with Sim(sc, stream=stream, max_neighbours=cap, **kw) as sim:
        sim.set_graph(True)
        for k in range(1, steps + 1):
            sim.step(1)
            try:
                sim.sync()
            except PbfError:
                return {"steps": steps, "error": msg, "first_fault_step": k}
    return {"steps": steps, "error": msg}


def run_batch(args, torch, stream):
    """64 independent dam-break scenes (log-uniform sizes 4,096..131,072,
    per-scene level ranges within 3..10, distance-to-camera levels): one
    batched context, every pass one launch over all scenes, a step one graph
    replay, block sizes from the autotuner; against 64 serial contexts (one
    graph replay each per step) on the same stream."""
    import scenes
    from paper_1608_04721_amd import Sim, autotune

    scs = scenes.dam_break_batch()
    n_tot = sum(s.n for s in scs)
    print(f"[bench] batch: {len(scs)} scenes, {n_tot} particles", file=sys.stderr, flush=True)
    with Sim(scs, stream=stream) as sim:
        sizes = autotune.tune(sim, steps=2, verbose=True)
    with Sim(scs, stream=stream) as sim:
        autotune.apply(sim, sizes)
        batched = _timed_run(sim, args.steps, args.warmup, stream, torch)
    print("[bench] serial contexts", file=sys.stderr, flush=True)
    sims = [Sim(sc, stream=stream) for sc in scs]
    try:
        for sm in sims:
            autotune.apply(sm, sizes)
            sm.set_graph(True)
            sm.step(args.warmup)
        for sm in sims:
            sm.sync()
        pit0 = sum(sm.stats()["total_particle_iterations"] for sm in sims)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            for sm in sims:
                sm.step(1)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        pit = sum(sm.stats()["total_particle_iterations"] for sm in sims) - pit0
    finally:
        for sm in sims:
            sm.close()
    serial = {"ms_per_step": ms / args.steps, "value": pit / (ms * 1e-3)}
    return {
        "metric": "batched particle-iterations/s and ms/step, 64 dam-break scenes, batched vs serial",
        "value": round(batched["value"], 1), "unit": "particle-iterations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(batched["ms_per_step"], 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "dam_break_batch: 64 scenes, 4,096..131,072 particles each "
                               "(log-uniform, seed 4), levels within 3..10 by distance to "
                               "camera, dt=1/120", "particles": n_tot, "scenes": len(scs),
                   "launch": "hipGraph per step, one launch per pass for all scenes",
                   "block_sizes": sizes},
        "serial": {"ms_per_step": round(serial["ms_per_step"], 4),
                   "value": round(serial["value"], 1)},
        "speedup_vs_serial": round(serial["ms_per_step"] / batched["ms_per_step"], 4),
        "mean_levels": round(batched["mean_levels"], 4),
        "density": batched["density"],
    }


def run_rollout(args, torch, stream):
    """The differentiable-rollout workload: 32,768 particles (32^3 lattice),
    N = 6, dt = 1/120, 20 steps, loss = mean squared distance of the final
    positions to a seeded target cloud, gradient with respect to the initial
    (x, v) by the library's reverse mode with checkpoints every 5 steps.
    Reports the wall time of the reverse pass against that of the forward
    rollout (with checkpoints) and of 20 plain graph-launched steps."""
    import scenes
    from paper_1608_04721_amd import Sim

    sc = scenes.rollout_32k()
    T, every = int(sc.steps), 5
    reps = max(1, args.steps // 20)
    n = sc.n
    tgt = sc.target.astype(np.float32)
    zero = np.zeros((n, 3), np.float32)
    with Sim(sc, stream=stream) as sim:
        x0, v0, _ = sim.get_state()
        sim.set_graph(True)
        # warm-up: one of each
        sim.step(T)
        sim.sync()
        sim.set_state(x0, v0)
        sim.rollout_forward(T, every)
        sim.sync()
        g = ((2.0 / n) * (sim.positions() - tgt)).astype(np.float32)
        sim.rollout_backward(g, zero)
        t_plain, t_fwd, t_bwd = [], [], []
        for _ in range(reps):
            sim.set_state(x0, v0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.step(T)
            sim.sync()
            t_plain.append(time.perf_counter() - t0)
            sim.set_state(x0, v0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.rollout_forward(T, every)
            sim.sync()
            t_fwd.append(time.perf_counter() - t0)
            g = ((2.0 / n) * (sim.positions() - tgt)).astype(np.float32)
            t0 = time.perf_counter()
            gx, gv = sim.rollout_backward(g, zero)
            t_bwd.append(time.perf_counter() - t0)
        loss = float(np.mean(np.sum((sim.positions().astype(np.float64) - tgt) ** 2, axis=1)))
    plain, fwd, bwd = (1e3 * float(np.median(a)) for a in (t_plain, t_fwd, t_bwd))
    return {
        "metric": "adjoint/forward wall-time ratio, 32,768-particle 20-step differentiable rollout",
        "value": round(bwd / fwd, 4), "unit": "x", "n_gpus": 1, "steps": reps * T,
        "warmup": T, "ms_per_step": round((fwd + bwd) / T, 4), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "rollout_32k: 32,768 particles (32^3 lattice), N=6, dt=1/120, "
                               "20 steps, loss = mean squared distance to a seeded target cloud, "
                               "checkpoints every 5 steps", "particles": n, "steps": T,
                   "ckpt_every": every, "repeats": reps},
        "ms_forward_plain_graph": round(plain, 3),
        "ms_rollout_forward": round(fwd, 3),
        "ms_rollout_backward": round(bwd, 3),
        "backward_vs_plain_forward": round(bwd / plain, 4),
        "loss": loss, "grad_v_norm": float(np.linalg.norm(gv)),
    }


def run_multidam(args, torch, stream):
    """The multi-dam-break scene of Section 7.3: four blocks of 35 x 46 x 35
    particles (225,400 in all) in the corners of a 6.4 x 3.2 x 6.4 box around
    a solid cone (base radius 1.5, height 2.0) standing at its centre;
    distance-to-camera levels N_i in {4..8}, one pre-stabilisation iteration
    for N_i < 6, dt = 1/120.  The first 60 steps (untimed) bring the fluid
    onto the cone; the timed steps follow.  Against plain PBF with N = 8 and
    N = 4 and against APBF without the cone, from the same state."""
    import dataclasses

    import scenes
    from paper_1608_04721_amd import PBF_LOD_UNIFORM, PbfError, Sim

    sc = scenes.multi_dam_break()
    warm = max(args.warmup, 60)
    runs = {}
    # plain PBF: every N_i = N, so the pre-stabilised set N_i < S is empty
    variants = [("apbf", sc),
                ("pbf8", dataclasses.replace(sc.with_lod(PBF_LOD_UNIFORM, n_min=8, n_max=8), stab_s=1)),
                ("pbf4", dataclasses.replace(sc.with_lod(PBF_LOD_UNIFORM, n_min=4, n_max=4), stab_s=1)),
                ("apbf_no_cone", dataclasses.replace(sc, obstacles=(), stab_iters=0, stab_s=1))]
    for name, s in variants:
        print(f"[bench] multidam {name}", file=sys.stderr, flush=True)
        with Sim(s, stream=stream, max_neighbours=128) as sim:
            try:
                runs[name] = _timed_run(sim, args.steps, warm, stream, torch)
                runs[name]["contacts_last_step"] = int(np.count_nonzero(sim.debug_contacts()))
            except PbfError as e:
                runs[name] = {"error": str(e)}
    # per-kernel times over a few direct-launch steps from the warmed state
    with Sim(sc, stream=stream, max_neighbours=128) as sim:
        sim.set_graph(True)
        sim.step(warm)
        sim.sync()
        sim.set_graph(False)
        sim.profile_enable(True)
        sim.step(args.profile_steps)
        prof = sim.profile_read()
    kernels = {k: {"total_ms": round(v[0], 4), "launches": v[1],
                   "avg_us": round(1e3 * v[0] / v[1], 2) if v[1] else None}
               for k, v in prof.items() if v[1]}
    a = runs["apbf"]

    def short(r):
        if "error" in r:
            return r
        return {"ms_per_step": round(r["ms_per_step"], 4), "value": round(r["value"], 1),
                "mean_levels": round(r["mean_levels"], 4), "density": r["density"],
                "contacts_last_step": r["contacts_last_step"]}

    line = {
        "metric": "particle-iterations/s and ms/step, multi dam break with a central cone, "
                  "APBF vs PBF(N=8)",
        "value": round(a["value"], 1), "unit": "particle-iterations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": warm, "ms_per_step": round(a["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "multi_dam_break: 4 blocks of 35x46x35 particles (225,400), box "
                               "6.4x3.2x6.4, solid cone r=1.5 h=2.0 at the centre, "
                               "distance-to-camera levels 4..8, pre-stabilisation 1 iteration "
                               "for N_i < 6, dt=1/120, timed after 60 steps",
                   "particles": sc.n, "levels": [sc.n_min, sc.n_max],
                   "launch": "hipGraph per step"},
        "ms_median": round(a["ms_median"], 4), "mean_levels": round(a["mean_levels"], 4),
        "density": a["density"], "contacts_last_step": a["contacts_last_step"],
        "pbf": {"8": short(runs["pbf8"]), "4": short(runs["pbf4"])},
        "apbf_no_cone": short(runs["apbf_no_cone"]),
        "kernels": kernels,
    }
    if "error" not in runs["pbf8"]:
        line["speedup_vs_pbf8"] = round(runs["pbf8"]["ms_per_step"] / a["ms_per_step"], 4)
    return line


def run_traffic(args, torch, stream):
    """A short run for hardware-counter passes (rocprofv3 --pmc FETCH_SIZE,
    then WRITE_SIZE): first a plain device copy of 256 MiB, three times,
    whose counter readings calibrate the counters against a known byte
    count; then the tank workload, 2 warm-up steps and 3 steps, with direct
    launches so every kernel is a dispatch of its own."""
    import scenes
    from paper_1608_04721_amd import Sim

    nbytes = 256 << 20
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    with torch.cuda.stream(stream):
        for _ in range(3):
            dst.copy_(src)
    torch.cuda.synchronize()
    sc = scenes.tank_1m()
    with Sim(sc, stream=stream) as sim:
        sim.set_graph(False)
        sim.step(2)
        sim.sync()
        sim.step(3)
        sim.sync()
        st = sim.stats()
    return {"workload": "traffic", "copy_bytes": nbytes, "steps": 3,
            "particle_iterations_last_step": st["particle_iterations"],
            "neighbour_pairs_last_step": st["neighbour_pairs"]}


VALU_PEAK_WAVE_INSTR = 256 * 4 * 2.4e9 / 4  # wave64 VALU instructions/s: 4 cycles each per SIMD
COPY_BYTES = 256 << 20


def summarize_counters(root: Path) -> dict:
    """Per-kernel figures from the rocprofv3 passes over `--workload
    traffic` under `root` (sub-folders fetch, write, sq1, sq2 with their
    *_counter_collection.csv): HBM bytes per dispatch calibrated by the
    256 MiB copy of the same run, the VALU issue share, the LDS bank
    conflict ratio and the wait share."""
    import collections
    import csv
    import re

    def short(name):
        m = re.search(r"(k_\w+)", name)
        return m.group(1).replace("k_", "", 1) if m else name.split("(")[0]

    per = collections.defaultdict(lambda: collections.defaultdict(float))
    disp = collections.defaultdict(dict)  # kernel -> dispatch -> seconds
    copies = collections.defaultdict(list)
    for sub in ("fetch", "write", "sq1", "sq2"):
        files = sorted((root / sub).rglob("*counter_collection.csv"))
        if not files:
            continue
        for r in csv.DictReader(open(files[0])):
            k, c, v = short(r["Kernel_Name"]), r["Counter_Name"], float(r["Counter_Value"])
            did = (sub, r["Dispatch_Id"])
            t = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
            if c in ("FETCH_SIZE", "WRITE_SIZE") and "copyBuffer" in r["Kernel_Name"]:
                copies[c].append(v)
            per[k][c] += v
            disp[k].setdefault(did, t)
    out = {"fetch_factor": None, "write_factor": None, "bytes_per_dispatch": {}, "dispatch_s": {},
           "valu_issue": {}, "lds_conflict_ratio": {}, "wait_share": {},
           "sources_sha1": kernel_sources_digest()}
    kib = COPY_BYTES / 1024
    big_w = [v for v in copies["WRITE_SIZE"] if abs(v - kib) < 0.01 * kib]
    big_f = sorted(copies["FETCH_SIZE"])[-len(big_w):] if big_w else []
    if big_w and big_f:
        out["write_factor"] = sum(big_w) / len(big_w) / kib
        out["fetch_factor"] = sum(big_f) / len(big_f) / kib
    for k, cs in per.items():
        if not k or "copyBuffer" in k:
            continue
        n = {sub: sum(1 for (s_, _) in disp[k] if s_ == sub) for sub in ("fetch", "write", "sq1", "sq2")}
        dur = {sub: sum(t for (s_, _), t in disp[k].items() if s_ == sub) for sub in n}
        if n["fetch"] and n["write"] and out["fetch_factor"]:
            out["bytes_per_dispatch"][k] = int(1024 * (cs["FETCH_SIZE"] / n["fetch"] / out["fetch_factor"] +
                                                       cs["WRITE_SIZE"] / n["write"] / out["write_factor"]))
            out["dispatch_s"][k] = (dur["fetch"] + dur["write"]) / (n["fetch"] + n["write"])
        if n["sq1"] and cs.get("SQ_INSTS_VALU"):
            out["valu_issue"][k] = round(cs["SQ_INSTS_VALU"] / dur["sq1"] / VALU_PEAK_WAVE_INSTR, 4)
            if cs.get("SQ_WAVE_CYCLES") and n["sq2"]:
                out["wait_share"][k] = round((cs["SQ_WAIT_INST_ANY"] / n["sq2"]) /
                                             (cs["SQ_WAVE_CYCLES"] / n["sq1"]), 4)
        if cs.get("SQ_ACTIVE_INST_LDS"):
            out["lds_conflict_ratio"][k] = round(cs["SQ_LDS_BANK_CONFLICT"] / cs["SQ_ACTIVE_INST_LDS"], 3)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--workload", choices=("tank", "batch", "rollout", "multidam", "traffic"),
                    default="tank",
                    help="tank: the 1M-particle headline line (default); batch: 64 scenes; "
                         "rollout: reverse-mode cost on the 32k-particle rollout; multidam: "
                         "four dam breaks around a solid cone with pre-stabilisation; traffic: "
                         "short run for hardware-counter passes")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--profile-steps", type=int, default=5)
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps-1t", type=int, default=1,
                    help="steps of the one-thread oracle rate (0 skips it)")
    ap.add_argument("--batch-steps", type=int, default=20)
    ap.add_argument("--no-pbf", action="store_true", help="skip the PBF(10)/PBF(5) runs")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 100-step runs, the 262k dam break, the batch and the rollout")
    ap.add_argument("--summarize-counters", metavar="DIR",
                    help="write profiles/tank_1m_traffic.json from the rocprofv3 counter "
                         "passes under DIR (fetch, write, sq1, sq2) and exit; no GPU needed")
    args = ap.parse_args(argv)
    if args.summarize_counters:
        rec = summarize_counters(Path(args.summarize_counters))
        TRAFFIC_FILE.write_text(json.dumps(rec, indent=1, sort_keys=True) + "\n")
        print(json.dumps(rec, indent=1, sort_keys=True))
        return 0
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the solver has no multi-GPU path)",
              file=sys.stderr)
        return 2

    import torch

    import scenes
    from paper_1608_04721_amd import PBF_LOD_UNIFORM, PbfError, Sim

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()  # default priority
    if args.workload == "batch":
        print(json.dumps(run_batch(args, torch, stream)), flush=True)
        return 0
    if args.workload == "rollout":
        print(json.dumps(run_rollout(args, torch, stream)), flush=True)
        return 0
    if args.workload == "traffic":
        print(json.dumps(run_traffic(args, torch, stream)), flush=True)
        return 0
    if args.workload == "multidam":
        print(json.dumps(run_multidam(args, torch, stream)), flush=True)
        return 0
    sc = scenes.tank_1m()
    steps, warm = args.steps, args.warmup
    cap = NBR_CAP

    print(f"[bench] APBF {sc.name}: n={sc.n}, levels {sc.n_min}..{sc.n_max}", file=sys.stderr,
          flush=True)
    with Sim(sc, stream=stream, max_neighbours=cap) as sim:
        apbf = _timed_run(sim, steps, warm, stream, torch)
    # the same tank with distance-to-the-visible-surface levels (the paper's
    # second adaption model), seen from the same camera
    # (0..4 m behind the visible surface -> levels 10..5: mean level 7.2 at
    # t = 0, close to the distance-to-camera run's 7.4)
    scv = scenes.with_dtvs(sc, camera=sc.camera, target=(3.2, 1.6, 3.2), d_far=4.0)
    print("[bench] APBF with visible-surface levels", file=sys.stderr, flush=True)
    with Sim(scv, stream=stream, max_neighbours=cap) as sim:
        try:
            dtvs = _timed_run(sim, steps, warm, stream, torch)
        except PbfError as e:
            dtvs = {"error": str(e)}
    out_pbf = {}
    if not args.no_pbf:
        for N in (10, 5):
            scp = sc.with_lod(PBF_LOD_UNIFORM, n_min=N, n_max=N)
            print(f"[bench] PBF N={N}", file=sys.stderr, flush=True)
            # plain PBF with few iterations may compress this deep tank far
            # beyond rest density; a fault is reported instead of ending the run
            with Sim(scp, stream=stream, max_neighbours=cap) as sim:
                try:
                    out_pbf[N] = _timed_run(sim, steps, warm, stream, torch)
                except PbfError as e:
                    out_pbf[N] = {"error": str(e)}
            if "error" in out_pbf[N] and "capacity" in out_pbf[N]["error"]:
                print(f"[bench] PBF N={N} again at capacity {NBR_CAP_RETRY}", file=sys.stderr, flush=True)
                with Sim(scp, stream=stream, max_neighbours=NBR_CAP_RETRY) as sim:
                    try:
                        r = _timed_run(sim, steps, warm, stream, torch)
                        r["neighbour_capacity"] = NBR_CAP_RETRY
                        r["at_capacity_%d" % cap] = out_pbf[N]["error"]
                        out_pbf[N] = r
                    except PbfError as e:
                        out_pbf[N]["error_at_capacity_%d" % NBR_CAP_RETRY] = str(e)
    print("[bench] profiling kernels", file=sys.stderr, flush=True)
    prof, pairs, active, _, design = _profile(sc, args.profile_steps, Sim, stream, cap)
    roof, kernels = _roofline(prof, pairs, active, design)
    extra = {}
    if not args.no_extra:
        # the stated 100-step runs from t = 0, like for like (same capacity)
        full = {}
        for name, s_ in (("apbf", sc), ("pbf10", sc.with_lod(PBF_LOD_UNIFORM, n_min=10, n_max=10)),
                         ("pbf5", sc.with_lod(PBF_LOD_UNIFORM, n_min=5, n_max=5))):
            print(f"[bench] {name}: {sc.steps} steps from t = 0", file=sys.stderr, flush=True)
            full[name] = _full_run(s_, int(sc.steps), Sim, stream, torch, cap)
            if name != "apbf" and "error" in full[name] and "capacity" in full[name]["error"]:
                r = _full_run(s_, int(sc.steps), Sim, stream, torch, NBR_CAP_RETRY)
                r["neighbour_capacity"] = NBR_CAP_RETRY
                r["at_capacity_%d" % cap] = {k: v for k, v in full[name].items() if k != "steps"}
                full[name] = r
        for ref in ("pbf10", "pbf5"):
            if "error" not in full["apbf"] and "error" not in full[ref]:
                full["speedup_vs_" + ref] = round(full[ref]["ms_per_step"] / full["apbf"]["ms_per_step"], 4)
        extra["tank_1m_100_steps"] = full
        # the 262,144-particle dam break, plain PBF with N = 10, 100 steps
        sd = scenes.dam_break_262k()
        print(f"[bench] {sd.name}: {sd.steps} steps", file=sys.stderr, flush=True)
        r = _full_run(sd, int(sd.steps), Sim, stream, torch, cap)
        r["workload"] = ("dam_break_262k: 262,144 particles (64^3 lattice) in the corner of a "
                         "12.8x6.4x6.4 tank, plain PBF N=10, dt=1/120, 100 steps from t = 0")
        extra["dam_break_262k"] = r
        # 64 batched scenes against 64 serial contexts
        nb = argparse.Namespace(steps=args.batch_steps, warmup=3)
        b = run_batch(nb, torch, stream)
        extra["batch_64"] = {"particles": b["config"]["particles"], "steps": b["steps"],
                             "ms_per_step": b["ms_per_step"], "value": b["value"],
                             "serial_ms_per_step": b["serial"]["ms_per_step"],
                             "speedup_vs_serial": b["speedup_vs_serial"],
                             "block_sizes": b["config"]["block_sizes"]}
        # reverse mode against the forward rollout, 32k particles, 20 steps
        ro = run_rollout(argparse.Namespace(steps=20), torch, stream)
        extra["rollout_32k"] = {"adjoint_vs_forward": ro["value"],
                                "ms_rollout_forward": ro["ms_rollout_forward"],
                                "ms_rollout_backward": ro["ms_rollout_backward"],
                                "ms_forward_plain_graph": ro["ms_forward_plain_graph"],
                                "backward_vs_plain_forward": ro["backward_vs_plain_forward"]}
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] oracle CPU baseline", file=sys.stderr, flush=True)
        cpu = _cpu_baseline(sc, args.cpu_steps, args.cpu_steps_1t)

    line = {
        "metric": METRIC,
        "value": round(apbf["value"], 1),
        "unit": "particle-iterations/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": round(apbf["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "tank_1m: 1,048,576 particles (128x64x128 lattice, s=0.05, "
                               "h=0.1, v~N(0,0.1^2)), box 6.4^3, distance-to-camera levels "
                               "5..10, dt=1/120",
                   "particles": sc.n, "levels": [sc.n_min, sc.n_max], "lod": "dtc",
                   "launch": "hipGraph per step", "neighbour_capacity": cap},
        "ms_median": round(apbf["ms_median"], 4),
        "mean_levels": round(apbf["mean_levels"], 4),
        "roofline": roof,
        "cpu_baseline": cpu,
        "kernels": kernels,
    }
    line["max_neighbours"] = apbf["max_neighbours"]
    # the paper's quality measure: average density over all particles after
    # warm-up + timed steps (APBF and PBF(10) from the same initial state)
    line["density"] = {"apbf": apbf["density"]}
    line["dtvs"] = ({"error": dtvs["error"]} if "error" in dtvs else
                    {"ms_per_step": round(dtvs["ms_per_step"], 4), "value": round(dtvs["value"], 1),
                     "mean_levels": round(dtvs["mean_levels"], 4), "density": dtvs["density"]})
    line["dtvs"]["levels"] = "distance to the visible surface, 0..4 m -> 10..5, same camera"
    if out_pbf:
        line["pbf"] = {str(N): ({k: v for k, v in r.items() if "error" in k} if "error" in r else
                                {"ms_per_step": round(r["ms_per_step"], 4),
                                 "ms_median": round(r["ms_median"], 4),
                                 "value": round(r["value"], 1),
                                 "max_neighbours": r["max_neighbours"],
                                 "density": r["density"],
                                 **{k: v for k, v in r.items()
                                    if k == "neighbour_capacity" or k.startswith("at_capacity")}})
                       for N, r in out_pbf.items()}
        for N in (10, 5):
            if "error" not in out_pbf[N]:
                line[f"speedup_vs_pbf{N}"] = round(out_pbf[N]["ms_per_step"] / apbf["ms_per_step"], 4)
        if "error" not in out_pbf[10] and "error" not in dtvs:
            line["dtvs"]["speedup_vs_pbf10"] = round(out_pbf[10]["ms_per_step"] / dtvs["ms_per_step"], 4)
    line.update(extra)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
