"""Block-size autotuner for libpbf contexts.

For every kernel class whose launch shape may change, try the candidate
threads-per-block values one kernel at a time (coordinate descent, the
other kernels at their current best), timing each candidate with the
library's per-launch HIP events over a few steps on the caller's own
workload.  The winners are applied to the context and cached on disk, keyed
by the workload's shape, so later contexts of the same shape skip the search.

The search changes only launch shapes, never results: every kernel is a
gather with a fixed summation order, so any block size gives bit-identical
output.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
from pathlib import Path
from typing import Dict, Optional

from . import _lib, kernel_names

# candidate threads per block for each tunable kernel class
CANDIDATES: Dict[str, tuple] = {
    "lod_predict": (128, 256, 512, 1024),
    "sort_scatter": (128, 256, 512, 1024),
    "sort_finish": (128, 256, 512, 1024),
    "tile_prepare": (64, 128, 256, 512),
    "neighbours": (128, 256, 384, 512),
    "lambda": (128, 256, 384, 512),
    "update": (128, 256, 384, 512),
    "commit": (128, 256, 512, 1024),
    "contacts": (128, 256, 512, 1024),
    "lod_range": (128, 256, 512, 1024),
}


def cache_path() -> Path:
    env = os.environ.get("PBF_TUNE_CACHE")
    if env:
        return Path(env)
    return Path.home() / ".cache" / "paper_1608_04721_amd" / "block_sizes.json"


def signature(sim) -> str:
    """Workload key: particle and scene counts, level ranges, grid sizes and
    the library file (a rebuilt library is tuned again)."""
    lib = _lib.LIB_PATH
    st = lib.stat()
    parts = [str(sim.n), str(sim.n_scenes), f"{st.st_size}:{int(st.st_mtime)}"]
    for s in sim.scenes:
        parts.append(f"{s.n}/{s.n_min}/{s.n_max}/{tuple(int(d) for d in s.dims)}/{s.lod_mode}")
    return hashlib.sha1("|".join(parts).encode()).hexdigest()


def _load() -> dict:
    p = cache_path()
    if p.exists():
        try:
            return json.loads(p.read_text())
        except (OSError, ValueError):
            return {}
    return {}


def _store(table: dict) -> None:
    p = cache_path()
    try:
        p.parent.mkdir(parents=True, exist_ok=True)
        tmp = p.with_suffix(".tmp")
        tmp.write_text(json.dumps(table, indent=1, sort_keys=True))
        os.replace(tmp, p)
    except OSError:
        pass  # a read-only home only costs a new search next time


def _time_kernels(sim, steps: int) -> Dict[str, float]:
    """Average milliseconds per step of each kernel class over `steps` steps."""
    sim.set_graph(False)
    sim.profile_enable(True)
    sim.step(steps)
    prof = sim.profile_read()
    sim.profile_enable(False)
    return {k: v[0] / steps for k, v in prof.items()}


def tune(sim, steps: int = 3, use_cache: bool = True, verbose: bool = False) -> Dict[str, int]:
    """Pick block sizes for `sim` (advancing it by a few steps per candidate)
    and apply them; returns {kernel name: threads}."""
    key = signature(sim)
    table = _load() if use_cache else {}
    names = kernel_names()
    if key in table:
        best = {k: int(v) for k, v in table[key].items()}
        for k, t in best.items():
            if k in names:
                sim.set_block_size(k, t)
        return best
    best = {}
    # first-touch and cold-cache costs stay out of the timings; kernels that
    # this workload never launches are not tuned
    launched = {k for k, ms in _time_kernels(sim, 1).items() if ms > 0.0}
    for kname, cands in CANDIDATES.items():
        if kname not in launched:
            continue
        timings = {}
        for t in cands:
            sim.set_block_size(kname, t)
            timings[t] = _time_kernels(sim, steps)[kname]
        pick = min(timings, key=timings.get)
        sim.set_block_size(kname, pick)
        best[kname] = pick
        if verbose:
            print(f"[tune] {kname}: " + ", ".join(f"{t}:{ms * 1e3:.1f}us" for t, ms in timings.items())
                  + f" -> {pick}", file=sys.stderr, flush=True)
    if use_cache:
        table = _load()
        table[key] = best
        _store(table)
    return best


def apply(sim, sizes: Optional[Dict[str, int]]) -> None:
    for k, t in (sizes or {}).items():
        sim.set_block_size(k, t)
