"""Autotuner for the pass kernels' tile and launch parameters.

The best tile for a workload depends on the memory system's response to the
pass's access pattern and on the kernel's register and LDS footprint, which are
measured, not modelled. ``tune`` therefore times every candidate setting of a
plan on the caller's own buffers. A candidate is:

* tile bits;
* carrier bits;
* the lane order of the IO stages;
* register bits per thread;
* resident workgroups per CU;
* the team size and threshold of the batched launch.

Timing uses HIP events around a few graph replays. ``tune`` keeps the fastest
setting, leaves it applied to the plan, and returns it with the table of
timings.

If ``PK_TUNE_CACHE`` names a JSON file, choices are remembered there. The key
is the device name and a hash of the library's sources, the precision, the
operation and the problem's structure (sizes, gate kinds, qubits, CPHASEK
exponents and QFT registers). A later ``tune`` of the same workload
then applies the cached choice without timing.
"""

import hashlib
import itertools
import json
import os

import numpy as np

from . import paperkern as pk

FIELDS = ("tile_bits", "carrier_bits", "lane_order", "reg_bits", "wgs_per_cu", "team_size", "min_team_tiles")


def candidates(prec, op):
    """Candidate settings for one precision (pk.PK_FP64 / pk.PK_FP32) and operation
    ("eval" or "batched").  Single-instance evaluations also try 3 register bits
    (more threads a tile: 4 resident waves per SIMD at 2^13 FP64 tiles) and 3
    carriers (fewer passes where the circuit needs many tile bits, as the QFT does);
    the batched launch has 4 and 5 register bits only."""
    kmax = 13 if prec == pk.PK_FP64 else 14
    tiles = [kmax, kmax - 1, kmax - 2]
    if op == "batched":
        tiles.append(kmax - 3)
    teams = ((16, 64), (16, 8)) if op == "batched" else ((16, 64),)
    carriers = (4, 5) if op == "batched" else (3, 4, 5)
    regs = (4, 5) if op == "batched" else (3, 4, 5)
    out = []
    for k, c, rb, (ts, mt) in itertools.product(tiles, carriers, regs, teams):
        if k - rb < 6 or k - rb > 10:
            continue
        out.append({"tile_bits": k, "carrier_bits": c, "lane_order": 1, "reg_bits": rb, "wgs_per_cu": 0,
                    "team_size": ts, "min_team_tiles": mt})
    return out


def apply(plan, cfg):
    # 4 register bits while the tile changes keep the workgroup within 1024 threads
    # whatever the previous and the next setting are
    plan.set_launch(cfg["wgs_per_cu"], 4)
    plan.set_tiling(cfg["tile_bits"], cfg["carrier_bits"], 1, cfg["lane_order"], cfg.get("page_cap", -1))
    plan.set_launch(cfg["wgs_per_cu"], cfg["reg_bits"])
    plan.set_batch(cfg.get("team_size", 16), cfg.get("min_team_tiles", 64))


WALKS = (0, 2, 4, 16, 64, -1)


def has_overlap(plan):
    """Whether Pass::overlap can change a forward pass of this plan: the
    single-instance kernels with 4 register bits have the overlapped tile loop."""
    if plan.n_inst != 1:
        return False
    return any(p["rbits"] == 4 for p in plan.describe()["instances"][0]["forward"])


def tune_walk(plan, psi_in, psi_out, reps=3, walks=WALKS, overlap=True):
    """Per-pass choice of the tile walk of a single-instance plan (0 strided over
    the grid, c runs of c consecutive tiles, -1 one block a workgroup) and, where
    the kernel has it, of the overlapped tile loop (pk_set_pass_overlap): every
    pass timed (pk.time_passes, HIP events) under each combination; each pass
    keeps its fastest.  Returns (walk per pass, {setting: per-pass ms}), the
    settings named by the walk, with "+o" for the overlapped loop."""
    n = plan.passes()
    modes = (0, 1) if overlap and has_overlap(plan) else (0,)
    times = {}
    for ov in modes:
        plan.set_pass_overlap([ov] * n)
        for w in walks:
            plan.set_pass_walk([w] * n)
            pk.time_passes(plan, psi_in, psi_out)
            times[(w, ov)] = np.median(np.array([pk.time_passes(plan, psi_in, psi_out) for _ in range(reps)]), axis=0)
    best = [min(times, key=lambda c: times[c][p]) for p in range(n)]
    plan.set_pass_overlap([c[1] for c in best] if len(modes) > 1 else [])
    plan.set_pass_walk([c[0] for c in best])
    named = {("%d+o" % w if ov else str(w)): [float(v) for v in t] for (w, ov), t in times.items()}
    return [c[0] for c in best], named


def tune_backward_walk(plan, psi_out, dL, angles=None, reps=2, walks=WALKS):
    """One tile walk for every backward pass of a single-instance plan, the fastest
    whole pk_backward among ``walks`` (HIP events); the forward passes keep theirs.
    Returns (walk, {walk: ms})."""
    import torch
    d = plan.describe()["instances"][0]
    fwd = [p["walk"] for p in d["forward"]]
    nb = len(d["backward"])
    times = {}
    for w in walks:
        plan.set_pass_walk(fwd + [w] * nb)
        pk.backward(plan, psi_out, dL, angles=angles)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            pk.backward(plan, psi_out, dL, angles=angles)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        times[w] = float(np.median(ts))
    best = min(walks, key=lambda w: times[w])
    plan.set_pass_walk(fwd + [best] * nb)
    return best, times


def _sources_hash():
    """Hash of the library's kernel and planner sources: a choice timed on one
    version of the kernels is not reused by another."""
    h = hashlib.sha256()
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".cpp", ".h")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:12]


def _gate_structure(g):
    """What of a gate tuple the schedule depends on: its kind and every integer
    field (qubits, the CPHASEK exponent, a QFT register's first qubit and size);
    not angles or operator entries."""
    kind = g[0]
    if kind in ("ONEOP", "D2"):
        ints = (g[1],)
    elif kind in ("TWOOP", "D4"):
        ints = (g[1], g[2])
    else:
        ints = tuple(v for v in g[1:] if isinstance(v, (int, np.integer)) and not isinstance(v, bool))
    return "%s%s" % (kind, ints)


def signature(plan, op):
    """Hash of what the schedule depends on: the library sources, precision,
    operation, and per instance the size, each gate's kind and integer fields and
    the number of marks (not angles, operators or mark values)."""
    h = hashlib.sha256()
    h.update(("%s|%s|%s|" % (_sources_hash(), plan.prec, op)).encode())
    for p in plan.problems:
        h.update(("n%d:" % p["nq"]).encode())
        for g in p["gates"]:
            h.update((_gate_structure(g) + ",").encode())
        h.update(("m%d;" % len(p.get("marked", []))).encode())
    return h.hexdigest()[:20]


def _device_name(torch):
    try:
        return torch.cuda.get_device_name(0)
    except Exception:  # pragma: no cover - name lookup is informational
        return "unknown"


def _load_cache(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _time(torch, run, reps, warmup):
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        run()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(plan, run, op="eval", reps=3, warmup=1, cands=None, use_cache=True):
    """Times ``run()`` (one evaluation with ``plan``) under every candidate setting;
    applies and returns (best setting, [(setting, ms), ...]) sorted by time."""
    import torch

    key = "%s|%s" % (_device_name(torch), signature(plan, op))
    path = os.environ.get("PK_TUNE_CACHE")
    if use_cache and path:
        hit = _load_cache(path).get(key)
        if hit:
            apply(plan, hit["best"])
            return hit["best"], [(c, ms) for c, ms in hit["table"]]
    table = []
    for cfg in (cands if cands is not None else candidates(plan.prec, op)):
        try:
            apply(plan, cfg)
        except pk.PaperkernError:
            continue
        table.append((dict(cfg), _time(torch, run, reps, warmup)))
    if not table:
        raise pk.PaperkernError(pk.PK_EINVAL, "no candidate setting was accepted")
    table.sort(key=lambda t: t[1])
    best = table[0][0]
    apply(plan, best)
    if path:
        cache = _load_cache(path)
        cache[key] = {"best": best, "table": table}
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, path)
    return best, table
