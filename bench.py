#!/usr/bin/env python
"""Throughput of the noisy Grover iteration on one MI355X.

Default workload: one noisy Grover iteration (Oracle, HALL, Inv, HALL plus one D2
noise rotation) on an n_q = 30 state in FP64 (2^30 amplitudes, 16 GiB), seed 1,
inputs resident in HBM.  One step = one evaluation of that iteration (every
pass over the state plus the FP64 readout of L and the norm).  Prints one JSON
line: evaluations/s, the roofline of the dominant kernel (the fused pass), the
FP32 variant's speedup and error, the 4096-instance batched form (FP64 and FP32,
at the setting recorded in paper_0902_0699_amd/tuning.json) against a loop of
single launches, the n_q = 30 gradient (adjoint kernel timed, 64 inputs against
central differences), and the oracle leg: the CPU oracle's rate on a bounded
sample, and the error of the FP64 and FP32 outputs against the oracle over all
2^30 amplitudes (outside the timed regions).

    python bench.py [--steps K] [--warmup W] [--extra] [--retune OUT.json]

--extra adds a two-qubit (TwoOpA) brickwork circuit at n_q = 30, Shor's data
path at n_q = 30 (load, QFT of register one, marginal; M = 899), the ensemble
density matrix of 4096 noisy Grover universes at n_q = 12 with its spectrum, and
the full Grover search (n_t iterations) at n_q = 20 and 24.  --retune runs the
autotuner on the batched workload instead of the recorded setting and writes
the new record to OUT.json.
"""

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "hot-path evaluations/sec on 1 MI355X + % roofline; mixed vs FP64 speedup at tol"
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_pass_kernel.json")
CSRC = os.path.join(ROOT, "paper_0902_0699_amd", "csrc")
FP32_TOL = 1e-5
CPU_SAMPLE_NQ = 26
TUNING_FILE = os.path.join(ROOT, "paper_0902_0699_amd", "tuning.json")


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_sha():
    """Hash of the kernel and plan sources: counters taken before a change are stale."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel_name):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None when
    the kernel source changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha") != kernel_sha() or t.get("kernel") not in kernel_name:
        return None
    return t.get("bytes_per_launch")


def single_run(torch, pk, W, autotune, prec, seed, nq, steps, warmup):
    """Times `steps` evaluations of one instance; returns a dict of figures."""
    t0 = time.perf_counter()
    inst = W.single_instance(seed, nq)
    log("generated n_q=%d seed %d input in %.1fs" % (nq, seed, time.perf_counter() - t0))
    plan = pk.Plan({"nq": nq, "gates": inst["gates"], "marked": inst["marked"]}, prec=prec)
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    x = torch.from_numpy(inst["psi"]).to(dt).to("cuda")
    del inst["psi"]
    y = torch.empty_like(x)
    L = torch.empty(1, dtype=torch.float64, device="cuda")
    norm = torch.empty(1, dtype=torch.float64, device="cuda")
    # per pass, the faster of the two tile walks, measured on these buffers
    walk, walk_ms = autotune.tune_walk(plan, x, y)
    log("%s: tile walk per pass %s (0 strided, c runs of c tiles, -1 blocks, +o overlapped loop; per-pass ms %s)"
        % (prec, walk, {w: [round(v, 2) for v in t] for w, t in walk_ms.items()}))
    for _ in range(warmup):
        pk.evaluate_into(plan, x, y, L, norm)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        pk.evaluate_into(plan, x, y, L, norm)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = ev0.elapsed_time(ev1) / steps
    log("%s: %.3f ms/evaluation over %d steps (wall %.3fs)" % (prec, ms, steps, wall))
    # per-launch durations of the pass kernel, HIP events around each launch
    reps = []
    for _ in range(3):
        reps.append(pk.time_passes(plan, x, y))
    per_pass = [float(np.mean([r[p] for r in reps])) for p in range(len(reps[0]))]
    return {"plan": plan, "x": x, "y": y, "L": float(L.item()), "norm": float(norm.item()),
            "ms": ms, "wall": wall, "per_pass_ms": per_pass, "passes": plan.passes(), "inst": inst,
            "walk": walk, "overlap": [p["overlap"] for p in plan.describe()["instances"][0]["forward"]]}


COPY_SLICE_BYTES = 1 << 30


def copy_probe(torch, x, y):
    """Bandwidth of a plain streaming kernel on the same buffers: torch's elementwise
    negation over 1 GiB slices, each one kernel launch that reads 1 GiB and writes
    1 GiB (a same-type copy_ would go to the DMA engine instead).  The slices give
    the counter calibration a dispatch of known size."""
    step = COPY_SLICE_BYTES // x.element_size()
    slices = [(x[i:i + step], y[i:i + step]) for i in range(0, x.numel(), step)]

    def sweep():
        for a, b in slices:
            torch.neg(a, out=b)

    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    sweep()
    e0.record()
    for _ in range(3):
        sweep()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 3
    return 2.0 * x.numel() * x.element_size() / (ms * 1e-3) / 1e9, ms


def host_description():
    """CPU model and thread counts of the host the oracle runs on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "usable_cpus": usable}


def cpu_baseline(W, O, nq_target, amp_sweeps_target):
    """The oracle, as it stands, on one bounded sample: one evaluation of the same
    noisy iteration at n_q = CPU_SAMPLE_NQ (26), scaled to n_q = nq_target by the
    amplitude sweeps.  NumPy's elementwise loops run on one thread, so one core."""
    inst = W.single_instance(1, CPU_SAMPLE_NQ)
    t0 = time.perf_counter()
    O.evaluate(CPU_SAMPLE_NQ, inst["gates"], inst["marked"], inst["psi"])
    t = time.perf_counter() - t0
    sweeps_sample = 2 * CPU_SAMPLE_NQ + 2
    scale = (2.0 ** nq_target / 2.0 ** CPU_SAMPLE_NQ) * (amp_sweeps_target / sweeps_sample)
    log("cpu oracle: %.2fs at n_q=%d, x%.1f to n_q=%d" % (t, CPU_SAMPLE_NQ, scale, nq_target))
    out = {"value": 1.0 / (t * scale), "unit": "evaluations/s", "cores": 1, "kind": "oracle",
           "sample": "one FP64 NumPy oracle evaluation of the same noisy iteration at n_q=%d (seed 1), "
                     "%.2f s, scaled by N*(2 n_q + 2) amplitude-sweeps to n_q=%d" % (CPU_SAMPLE_NQ, t, nq_target),
           "sample_seconds": t}
    out.update(host_description())
    return out


ACC_CHUNK = 1 << 24


def whole_state_error(torch, O, nq, gates, marked, psi_in, y, workers):
    """Normwise error of the device output y against the oracle's closed route for
    one Grover iteration (half sums of psi_in once, then every label in chunks,
    expected values computed in threads) and the oracle's L."""
    from concurrent.futures import ThreadPoolExecutor
    amp, L_ref = O.grover_sampler(nq, gates, marked, psi_in)
    n = 1 << nq
    starts = list(range(0, n, ACC_CHUNK))
    want_of = lambda a: amp(np.arange(a, min(a + ACC_CHUNK, n), dtype=np.int64))
    d2 = r2 = 0.0
    with ThreadPoolExecutor(max_workers=workers) as ex:
        futs = {i: ex.submit(want_of, a) for i, a in enumerate(starts[:workers])}
        for i, a in enumerate(starts):
            got = y[a:a + ACC_CHUNK].cpu().numpy().astype(np.complex128)
            want = futs.pop(i).result()
            if i + workers < len(starts):
                futs[i + workers] = ex.submit(want_of, starts[i + workers])
            d2 += float(np.sum(np.abs(got - want) ** 2))
            r2 += float(np.sum(np.abs(want) ** 2))
    return math.sqrt(d2 / r2), L_ref


def oracle_leg(torch, W, nq, kept, line):
    """The oracle on the host: its rate on a bounded sample (cpu_baseline), then the
    error of each kept device output against it over every amplitude."""
    import oracle as O
    line["cpu_baseline"] = cpu_baseline(W, O, nq, 2 * nq + 2)
    workers = max(1, min(16, line["cpu_baseline"]["usable_cpus"] or 1))
    acc = {}
    for prec, seed, y, L_gpu in kept:
        t0 = time.perf_counter()
        inst = W.single_instance(seed, nq)
        err, L_ref = whole_state_error(torch, O, nq, inst["gates"], inst["marked"], inst["psi"], y, workers)
        del inst
        acc[prec] = {"rel_err_psi": err, "abs_err_L": abs(L_gpu - L_ref), "L_oracle": L_ref,
                     "amplitudes_compared": 1 << nq,
                     "tol": 1e-12 if prec == "fp64" else FP32_TOL}
        acc[prec]["within_tol"] = err <= acc[prec]["tol"] and acc[prec]["abs_err_L"] <= acc[prec]["tol"]
        log("oracle accuracy %s: normwise %.3e over 2^%d amplitudes, |dL| %.3e (%.1fs)"
            % (prec, err, nq, acc[prec]["abs_err_L"], time.perf_counter() - t0))
    line["accuracy_vs_oracle"] = {
        "reference": "oracle closed route for one Grover iteration (HALL.Inv.HALL = 2|s><s| - I), every "
                     "amplitude, from the original FP64 input (FP32 error includes the input rounding)",
        **acc}
    if "mixed" in line and "fp32" in acc:
        line["mixed"]["rel_err_psi"] = acc["fp32"]["rel_err_psi"]
        line["mixed"]["abs_err_L"] = acc["fp32"]["abs_err_L"]
        line["mixed"]["within_tol"] = acc["fp32"]["within_tol"]
        line["mixed"]["reference"] = "FP64 oracle, every amplitude, original FP64 input"


def load_tuning():
    try:
        with open(TUNING_FILE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def batched_run(torch, pk, W, autotune, steps, warmup, prec, insts, record=None, loop=True):
    """The 4096-instance batch (Sec. 6.2) in one persistent graph-replayed launch, at
    the recorded setting (or retuned when ``record`` is None), against a loop of
    single-instance evaluations of the same instances."""
    probs = [{"nq": i["nq"], "gates": i["gates"], "marked": i["marked"]} for i in insts]
    plan = pk.Plan(probs, prec=prec)
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    packed = torch.from_numpy(np.concatenate([i["psi"] for i in insts])).to(dt).to("cuda")
    out = torch.empty_like(packed)
    if record is not None:
        best, n_cands, tuned = record["setting"], None, False
        autotune.apply(plan, best)
    else:
        t0 = time.perf_counter()
        best, table = autotune.tune(plan, lambda: pk.evaluate_batched(plan, packed, out=out), op="batched",
                                    use_cache=False)
        n_cands, tuned = len(table), True
        log("batched %s: tuned over %d settings in %.1fs: %s (%.3f ms)"
            % (prec, len(table), time.perf_counter() - t0, best, table[0][1]))
    for _ in range(warmup):
        pk.evaluate_batched(plan, packed, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        pk.evaluate_batched(plan, packed, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms_batched = e0.elapsed_time(e1) / steps
    # plain form: one single-instance evaluation per instance, back to back
    offs = plan.offsets()
    ms_loop = None
    if loop:
        singles = [pk.Plan(p, prec=prec) for p in probs]
        views = [(packed[offs[k]:offs[k + 1]], out[offs[k]:offs[k + 1]]) for k in range(len(probs))]
        for sp, (a, b) in zip(singles, views):
            pk.evaluate(sp, a, out=b)
        torch.cuda.synchronize()
        e0.record()
        for sp, (a, b) in zip(singles, views):
            pk.evaluate(sp, a, out=b)
        e1.record()
        torch.cuda.synchronize()
        ms_loop = e0.elapsed_time(e1)
    total = offs[-1]
    esz = 16 if prec == "fp64" else 8
    log("batched %s: %.3f ms per batch, loop of singles %s ms" % (prec, ms_batched, ms_loop))
    res = {"instances": len(insts), "amplitudes": total, "dtype": "f64" if prec == "fp64" else "f32",
           "ms_per_batch": ms_batched, "instances_per_s": len(insts) / (ms_batched * 1e-3),
           "ms_loop_of_singles": ms_loop, "speedup_vs_loop": ms_loop / ms_batched if ms_loop else None,
           "compulsory_GBs": 2.0 * total * esz / (ms_batched * 1e-3) / 1e9,
           "compulsory_frac": 2.0 * total * esz / (ms_batched * 1e-3) / 1e9 / PEAK_HBM_GBS,
           "setting": {k: best[k] for k in autotune.FIELDS if k in best},
           "setting_from": "autotuned now over %d settings" % n_cands if tuned else "tuning record",
           "passes_max": max(plan.passes(i) for i in range(len(insts)))}
    if record is not None:
        res["record_sources"] = record.get("sources")
    del packed, out
    return res, best


def gradient_run(torch, pk, W, autotune, nq):
    inst = W.single_instance(W.SEEDS["gradient"], nq)
    plan = pk.Plan({"nq": nq, "gates": inst["gates"], "marked": inst["marked"]})
    x = torch.from_numpy(inst["psi"]).to("cuda")
    ang = torch.tensor(list(inst["noise"][2:5]), dtype=torch.float64, device="cuda")
    out, L, _ = pk.evaluate(plan, x, angles=ang, want_norm=False)
    dL = torch.ones(1, dtype=torch.float64, device="cuda")
    walk, walk_ms = autotune.tune_backward_walk(plan, out, dL, angles=ang)
    log("gradient: backward tile walk %d (ms per walk %s)" % (walk, {w: round(t, 1) for w, t in walk_ms.items()}))
    gpsi, gang = pk.backward(plan, out, dL, angles=ang)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        pk.backward(plan, out, dL, angles=ang)
    e1.record()
    torch.cuda.synchronize()
    ms_bwd = e0.elapsed_time(e1) / 3
    comps = W.fd_subset(W.SEEDS["gradient"], inst)
    h = 1e-6
    L_of = lambda xx, aa: pk.evaluate(plan, xx, angles=aa, want_norm=False)[1].item()
    fd, ad = [], []
    for q, (kind, where) in enumerate(comps):
        if q % 16 == 0:
            log("gradient: central differences, input %d of %d" % (q, len(comps)))
        if kind == "angle":
            ap, am = ang.clone(), ang.clone()
            ap[where] += h
            am[where] -= h
            fd.append((L_of(x, ap) - L_of(x, am)) / (2 * h))
            ad.append(gang[where].item())
        else:
            idx, part = where
            step = h if part == 0 else 1j * h
            orig = x[idx].clone()
            x[idx] = orig + step
            lp = L_of(x, ang)
            x[idx] = orig - step
            lm = L_of(x, ang)
            x[idx] = orig
            fd.append((lp - lm) / (2 * h))
            g = gpsi[idx].item()
            ad.append(g.real if part == 0 else g.imag)
    fd, ad = np.array(fd), np.array(ad)
    err = float(np.max(np.abs(fd - ad)) / np.max(np.abs(ad)))
    return {"nq": nq, "ms_backward": ms_bwd, "fd_inputs": len(comps), "fd_h": h,
            "normwise_rel_err": err, "tol": 1e-6, "within_tol": err <= 1e-6,
            "backward_passes": len(plan.describe()["instances"][0]["backward"]), "backward_tile_walk": walk}


def brickwork_gates(nq, seed):
    """Two layers of random unitary two-qubit gates on neighbouring qubits:
    (1,2), (3,4), ..., then (2,3), (4,5), ... (seeded, QR of complex normals)."""
    rng = np.random.default_rng(seed)
    pairs = [(q, q + 1) for q in range(1, nq, 2)] + [(q, q + 1) for q in range(2, nq, 2)]
    gates = []
    for a, b in pairs:
        m, _ = np.linalg.qr(rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4)))
        gates.append(("TWOOP", a, b, m))
    return gates


def two_qubit_run(torch, pk, autotune, nq, steps):
    """TwoOpA sweeps (Eq. resmat2) at full size: a brickwork circuit, fused and one
    sweep per gate; the unitary circuit must keep the norm."""
    gates = brickwork_gates(nq, 5)
    N = 1 << nq
    x = torch.randn(N, dtype=torch.complex128, device="cuda")
    x /= torch.linalg.vector_norm(x)
    y = torch.empty_like(x)
    L = torch.empty(1, dtype=torch.float64, device="cuda")
    norm = torch.empty(1, dtype=torch.float64, device="cuda")
    out = {"workload": "brickwork of %d random unitary TwoOpA gates on neighbouring qubits, n_q=%d, FP64"
                       % (len(gates), nq), "gates": len(gates)}
    for label, fuse in (("fused", 1), ("unfused", 0)):
        plan = pk.Plan({"nq": nq, "gates": gates, "marked": [0]})
        if not fuse:
            plan.set_tiling(13, 4, 0)
        else:
            walk, _ = autotune.tune_walk(plan, x, y)
            out["fused_tile_walk"] = walk
            out["fused_overlap"] = [p["overlap"] for p in plan.describe()["instances"][0]["forward"]]
        pk.evaluate_into(plan, x, y, L, norm)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = steps if fuse else 2
        e0.record()
        for _ in range(reps):
            pk.evaluate_into(plan, x, y, L, norm)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        per_pass = [float(t) for t in pk.time_passes(plan, x, y)]
        out[label] = {"passes": plan.passes(), "ms": ms, "gates_per_s": len(gates) / (ms * 1e-3),
                      "mean_pass_GBs": 32.0 * N / (np.mean(per_pass) * 1e-3) / 1e9,
                      "min_pass_GBs": 32.0 * N / (max(per_pass) * 1e-3) / 1e9,
                      "norm_minus_1": float(norm.item()) - 1.0}
        log("two-qubit %s: %d passes, %.2f ms" % (label, plan.passes(), ms))
    out["fused_speedup"] = out["unfused"]["ms"] / out["fused"]["ms"]
    return out


def shor_run(torch, pk, W, autotune, steps, prec, qft_tiling=None):
    """Shor's data path at n_q = 30 (Sec. 5.2): the loaded state of Eq. Shor2, the QFT
    of register one (App. A) in place, and the distribution of register one; each
    part timed with HIP events on the current stream.  The QFT plan's tiling is
    tuned first on the same buffer, or fixed to ``qft_tiling`` = (tile bits, carrier
    bits, register bits), which keeps a profiled run's dispatches the same each
    time: the first evaluation's passes come first."""
    cands = None
    if qft_tiling:
        t, c, r = qft_tiling
        cands = [{"tile_bits": t, "carrier_bits": c, "lane_order": 1, "reg_bits": r, "wgs_per_cu": 0}]
    M = W.SHOR_M
    x = W.shor_xguess(W.SEEDS["shor"])
    n1, n2 = pk.shor_register_sizes(M)
    nq = n1 + n2
    N = 1 << nq
    esz = 16 if prec == "fp64" else 8
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    psi = torch.empty(N, dtype=dt, device="cuda")
    p = torch.empty(1 << n1, dtype=torch.float64, device="cuda")
    L = torch.empty(1, dtype=torch.float64, device="cuda")
    plan = pk.Plan({"nq": nq, "gates": [("QFT", 1, n1)], "marked": []}, prec=prec)
    pk.shor_state(n1, n2, x, M, prec=prec, out=psi)
    best, _ = autotune.tune(plan, lambda: pk.evaluate_into(plan, psi, psi, L), op="eval", use_cache=False,
                            cands=cands)
    walk, _ = autotune.tune_walk(plan, psi, psi)

    def run(ev=None):
        if ev:
            ev[0].record()
        pk.shor_state(n1, n2, x, M, prec=prec, out=psi)
        if ev:
            ev[1].record()
        pk.evaluate_into(plan, psi, psi, L)
        if ev:
            ev[2].record()
        pk.marginal(psi, nq, n2, out=p)
        if ev:
            ev[3].record()

    run()
    torch.cuda.synchronize()
    parts = np.zeros(3)
    for _ in range(steps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        run(ev)
        torch.cuda.synchronize()
        parts += [ev[i].elapsed_time(ev[i + 1]) for i in range(3)]
    parts /= steps
    per_pass = [float(t) for t in pk.time_passes(plan, psi, psi)]
    run()
    sum_p = float(p.sum().item())
    ms = float(parts.sum())
    out = {"workload": "Shor data path, M=%d xguess=%d: n1=%d, n2=%d (n_q=%d), %s" % (M, x, n1, n2, nq, prec.upper()),
           "ms": ms, "runs_per_s": 1e3 / ms, "qft_passes": plan.passes(),
           "qft_tiling": {k: best[k] for k in ("tile_bits", "carrier_bits", "reg_bits")}, "qft_tile_walk": walk,
           "load_ms": parts[0], "qft_ms": parts[1], "marginal_ms": parts[2],
           "load_GBs": esz * N / (parts[0] * 1e-3) / 1e9,
           "qft_mean_pass_GBs": 2.0 * esz * N / (np.mean(per_pass) * 1e-3) / 1e9,
           "qft_min_pass_GBs": 2.0 * esz * N / (max(per_pass) * 1e-3) / 1e9,
           "marginal_GBs": esz * N / (parts[2] * 1e-3) / 1e9, "sum_p_minus_1": sum_p - 1.0}
    log("shor %s: load %.2f ms, QFT %.2f ms (%d passes), marginal %.2f ms"
        % (prec, parts[0], parts[1], plan.passes(), parts[2]))
    # A labelled variant, not the paper's circuit: the QFT without its final pair
    # swaps and the marginal read with register one's bits reversed (same p(n)).
    p_ref = p.clone()
    plan2 = pk.Plan({"nq": nq, "gates": [("QFT_NOSWAP", 1, n1)], "marked": []}, prec=prec)
    pk.shor_state(n1, n2, x, M, prec=prec, out=psi)
    best2, _ = autotune.tune(plan2, lambda: pk.evaluate_into(plan2, psi, psi, L), op="eval", use_cache=False,
                             cands=cands)
    walk2, _ = autotune.tune_walk(plan2, psi, psi)

    def run2(ev):
        ev[0].record()
        pk.shor_state(n1, n2, x, M, prec=prec, out=psi)
        ev[1].record()
        pk.evaluate_into(plan2, psi, psi, L)
        ev[2].record()
        pk.marginal(psi, nq, n2, out=p, bitrev=True)
        ev[3].record()

    parts2 = np.zeros(3)
    for _ in range(steps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        run2(ev)
        torch.cuda.synchronize()
        parts2 += [ev[i].elapsed_time(ev[i + 1]) for i in range(3)]
    parts2 /= steps
    out["noswap_variant"] = {
        "method": "QFT without the final pair swaps, marginal with register one bit-reversed (not the paper's circuit)",
        "ms": float(parts2.sum()), "qft_ms": parts2[1], "qft_passes": plan2.passes(), "marginal_ms": parts2[2],
        "qft_tiling": {k: best2[k] for k in ("tile_bits", "carrier_bits", "reg_bits")}, "qft_tile_walk": walk2,
        "max_abs_dp_vs_paper_form": float((p - p_ref).abs().max().item())}
    log("shor %s, no-swap variant: QFT %.2f ms (%d passes), whole path %.2f ms"
        % (prec, parts2[1], plan2.passes(), parts2.sum()))
    del psi
    return out


def density_run(torch, pk, W, steps):
    """The ensemble density matrix (Sec. 6.1) of 4096 noisy Grover universes at
    n_q = 12, equal weights: the FP64 matrix-core kernel timed with HIP events on
    the current stream, then the spectrum (rocSOLVER) once."""
    nq, A = W.DENSITY_NQ, W.DENSITY_UNIVERSES
    N = 1 << nq
    gates, x = W.density_universes(W.SEEDS["density"], nq, A)
    plan = pk.Plan([{"nq": nq, "gates": g, "marked": [x]} for g in gates])
    s = torch.full((A * N,), 2.0 ** (-nq / 2), dtype=torch.complex128, device="cuda")
    C, _, _ = pk.evaluate_batched(plan, s)
    P = torch.full((A,), 1.0 / A, dtype=torch.float64, device="cuda")
    rho = torch.empty((N, N), dtype=torch.complex128, device="cuda")
    pk.density_matrix(C, P, out=rho)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        pk.density_matrix(C, P, out=rho)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    trace = float(torch.diagonal(rho).real.sum().item())
    t0 = time.time()
    lam, S, pur = pk.density_spectrum(rho)
    spec_s = time.time() - t0
    useful = 8.0 * A * N * (N + 1) / 2  # real flops of the lower triangle with the diagonal
    out = {"workload": "density matrix of %d noisy Grover universes, n_q=%d, FP64, equal weights" % (A, nq),
           "ms": ms, "achieved_TFLOPs": useful / (ms * 1e-3) / 1e12, "peak_TFLOPs": 78.6,
           "frac": useful / (ms * 1e-3) / 1e12 / 78.6, "trace_minus_1": trace - 1.0,
           "spectrum_s": spec_s, "entropy_bits": float(S), "purity": float(pur)}
    log("density: %.2f ms (%.1f TFLOP/s), spectrum %.2f s, S = %.4f bits, Tr rho^2 = %.4f"
        % (ms, out["achieved_TFLOPs"], spec_s, float(S), float(pur)))
    return out


def search_run(torch, pk, W, autotune, reps):
    """The full Grover search of Sec. 5.1: n_t = floor((pi/4) sqrt(N)) noise-free
    iterations from the uniform state in one replayed graph (pk_evaluate_repeat,
    which schedules 8 iterations at a time as one gate list), at n_q = 20 and 24,
    FP64; L is the success probability after n_t iterations.
    The tile is tuned on one iteration first (a 2^20 state gives only 128 tiles of
    the default size, half the CUs)."""
    out = {}
    for nq in (20, 24):
        nt = pk.grover_iterations(nq)
        x = int(np.random.default_rng(W.SEEDS["small_fp64"]).integers(0, 1 << nq))
        plan = pk.Plan({"nq": nq, "gates": W.grover_gates(), "marked": [x]})
        s = torch.full((1 << nq,), 2.0 ** (-nq / 2), dtype=torch.complex128, device="cuda")
        y = torch.empty_like(s)
        L = torch.empty(1, dtype=torch.float64, device="cuda")
        best, _ = autotune.tune(plan, lambda: pk.evaluate_into(plan, s, y, L), op="eval", reps=5, warmup=2,
                                use_cache=False)
        ws = plan.workspace(pk.PK_OP_EVAL, s.device)
        st = pk._stream(s.device)

        def run():
            rc = pk.lib().pk_evaluate_repeat(plan.handle, nt, pk._ptr(s), pk._ptr(y), pk._ptr(L), None, None,
                                             pk._ptr(ws), st)
            pk._check(rc, plan.handle)

        run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            run()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        theta = math.asin(2.0 ** (-nq / 2))
        passes = pk.repeat_launches(plan, nt)  # 8 iterations fused into one schedule
        out["nq%d" % nq] = {"iterations": nt, "passes": passes, "passes_one_at_a_time": plan.passes() * nt,
                            "ms": ms, "iterations_per_s": nt / (ms * 1e-3),
                            "tile_bits": best["tile_bits"], "carrier_bits": best["carrier_bits"],
                            "mean_pass_GBs": 32.0 * (1 << nq) * passes / (ms * 1e-3) / 1e9,
                            "L": float(L.item()), "L_closed_form": math.sin((2 * nt + 1) * theta) ** 2}
        log("search n_q=%d: %d iterations, %d passes, %.2f ms, L = %.12f" % (nq, nt, passes, ms, L.item()))
        # the labelled variant through 2|s><s| - I: one pass per iteration, not the paper's form
        pk.search_diffusion(nq, [x], nt, s, out=y)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            _, Ld = pk.search_diffusion(nq, [x], nt, s, out=y)
        e1.record()
        torch.cuda.synchronize()
        msd = e0.elapsed_time(e1) / reps
        out["nq%d" % nq]["diffusion_variant"] = {
            "method": "(2|s><s| - I) . Oracle, one pass per iteration (not the paper's HALL form)",
            "ms": msd, "iterations_per_s": nt / (msd * 1e-3),
            "pass_GBs": 2.0 * (1 << nq) * 16 * nt / (msd * 1e-3) / 1e9, "L": float(Ld.item())}
        log("search n_q=%d, diffusion variant: %.2f ms, L = %.12f" % (nq, msd, Ld.item()))
        del s, y
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--nq", type=int, default=30)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--extra", action="store_true",
                    help="also time the two-qubit brickwork, Shor's data path, the density matrix and the search")
    ap.add_argument("--legs", default="batched,gradient,two_qubit,shor,density,search",
                    help="comma-separated legs to run (batched and gradient always, the others with --extra)")
    ap.add_argument("--qft-tiling", metavar="T,C,R",
                    help="fixed QFT tiling for the shor leg (tile, carrier, register bits) instead of tuning")
    ap.add_argument("--shor-precs", default="fp64,fp32", help="precisions of the shor leg")
    ap.add_argument("--no-loop", action="store_true",
                    help="skip the batched leg's loop of single launches (for counter runs: thousands of dispatches)")
    ap.add_argument("--retune", metavar="OUT.json",
                    help="autotune the batched workload instead of using the recorded setting; write the record")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this library runs on one GPU; a run on %d GPUs is not provided "
              "(instances and amplitude blocks would shard across GPUs, but that path is not built)"
              % max(args.gpus, world), file=sys.stderr)
        sys.exit(2)
    qft_tiling = tuple(int(v) for v in args.qft_tiling.split(",")) if args.qft_tiling else None
    if qft_tiling is not None and len(qft_tiling) != 3:
        ap.error("--qft-tiling takes three integers")

    import torch
    from paper_0902_0699_amd import autotune
    from paper_0902_0699_amd import paperkern as pk
    from paper_0902_0699_amd import workload as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    nq = args.nq
    N = 1 << nq
    r64 = single_run(torch, pk, W, autotune, "fp64", W.SEEDS["large_fp64"], nq, args.steps, args.warmup)
    value = 1000.0 / r64["ms"]
    passes = r64["passes"]
    # dominant kernel: the fused pass (every pass moves the whole state once: 32 B per amplitude)
    bytes_per_launch = 32.0 * N
    pass_ms = float(np.mean(r64["per_pass_ms"]))
    achieved = bytes_per_launch / (pass_ms * 1e-3) / 1e9
    kname = "pk::pass_kernel<double, 1, 13, 4>"  # demangled name as the profiler prints it
    traffic = stored_traffic(kname)
    copy_gbs, copy_ms = copy_probe(torch, r64["x"], r64["y"])
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "evaluations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "one noisy Grover iteration (Oracle, HALL, Inv, HALL, one D2 rotation) on "
                               "a Haar-random n_q=%d state, FP64, seed 1" % nq,
                   "nq": nq, "amplitudes": N, "passes": passes, "marked": 1},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "kernel": kname, "algorithmic_bytes_per_launch": bytes_per_launch,
                     "avg_launch_ms": pass_ms, "per_pass_ms": r64["per_pass_ms"],
                     "tile_walk": r64["walk"], "overlap": r64["overlap"]},
        "compulsory_floor_frac": (32.0 * N / (r64["ms"] * 1e-3) / 1e9) / PEAK_HBM_GBS,
        "copy_probe": {"GBs": copy_gbs, "ms": copy_ms, "frac_of_peak": copy_gbs / PEAK_HBM_GBS,
                       "pass_frac_of_copy": achieved / copy_gbs},
        "L": r64["L"], "norm": r64["norm"],
    }
    torch.cuda.empty_cache()
    # the copy probe overwrote y: one more evaluation restores the output kept for the oracle leg
    pk.evaluate_into(r64["plan"], r64["x"], r64["y"], torch.empty(1, dtype=torch.float64, device="cuda"))
    kept = [("fp64", W.SEEDS["large_fp64"], r64["y"], r64["L"])]
    del r64["x"]
    if not args.no_mixed:
        r32 = single_run(torch, pk, W, autotune, "fp32", W.SEEDS["large_fp32"], nq, args.steps, args.warmup)
        line["mixed"] = {"dtype": "f32", "value": 1000.0 / r32["ms"], "ms_per_step": r32["ms"],
                         "speedup_vs_fp64": line["ms_per_step"] / r32["ms"], "passes": r32["passes"],
                         "rel_err_psi": None, "abs_err_L": None, "L": r32["L"], "tol": FP32_TOL,
                         "within_tol": None, "reference": "set by the oracle leg",
                         "avg_launch_ms": float(np.mean(r32["per_pass_ms"])),
                         "achieved_GBs": 16.0 * N / (float(np.mean(r32["per_pass_ms"])) * 1e-3) / 1e9,
                         "tile_walk": r32["walk"], "overlap": r32["overlap"]}
        kept.append(("fp32", W.SEEDS["large_fp32"], r32["y"], r32["L"]))
        del r32["x"]
        torch.cuda.empty_cache()
    legs = set(args.legs.split(","))
    k = max(3, args.steps // 4)
    if "batched" in legs:
        t0 = time.perf_counter()
        insts = W.batch_instances(W.SEEDS["batched"])
        log("generated %d batched instances in %.1fs" % (len(insts), time.perf_counter() - t0))
        records = load_tuning()
        line["batched"] = {"workload": "%d noisy Grover instances, n_q = 10..19 log-uniform, seed %d, one "
                                       "persistent graph-replayed launch" % (len(insts), W.SEEDS["batched"])}
        new_records = {}
        for p in ("fp64", "fp32"):
            rec = None if args.retune else records.get("batched_" + p)
            line["batched"][p], best = batched_run(torch, pk, W, autotune, k, 1, p, insts, rec, not args.no_loop)
            new_records["batched_" + p] = {"setting": best, "sources": autotune._sources_hash(),
                                           "device": torch.cuda.get_device_name(0),
                                           "ms_per_batch": line["batched"][p]["ms_per_batch"]}
            torch.cuda.empty_cache()
        if args.retune:
            with open(args.retune, "w") as f:
                json.dump(new_records, f, indent=1)
        del insts
    if "gradient" in legs:
        line["gradient"] = gradient_run(torch, pk, W, autotune, nq)
        log("gradient: backward %.2f ms (%d passes), FD normwise rel err %.3e"
            % (line["gradient"]["ms_backward"], line["gradient"]["backward_passes"],
               line["gradient"]["normwise_rel_err"]))
        torch.cuda.empty_cache()
    if args.extra:
        runs = [("two_qubit", lambda: two_qubit_run(torch, pk, autotune, nq, k)),
                ("shor", lambda: {p: shor_run(torch, pk, W, autotune, k, p, qft_tiling)
                                  for p in args.shor_precs.split(",")}),
                ("density", lambda: density_run(torch, pk, W, k)),
                ("search", lambda: search_run(torch, pk, W, autotune, 3))]
        for name, run in runs:
            if name in legs:
                line[name] = run()
                torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        oracle_leg(torch, W, nq, kept, line)
    del kept
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
