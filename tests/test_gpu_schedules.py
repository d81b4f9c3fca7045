"""GPU parity of every element at the pass schedules the full-size runs use.

At the default tiling a forward evaluation takes 3 passes up to n_q = 22 and 5
from n_q = 23 (the n_q = 30 headline runs 5); the backward takes 5 passes from
n_q = 21 and 7 from n_q = 29.  These tests compare the whole output of those
schedules with the FP64 oracle:

  * forward at n_q = 23 and 24 (5 passes), FP64 and FP32, every noise placement,
    against the gate-by-gate oracle (Sec. 5.1, G = HALL.Inv.HALL.Oracle, built from
    the Eq. resmat1 sweeps of Sec. 3);
  * backward at n_q = 21 and 22 (5 passes) and at forced small tiles that give 5
    and 7 backward passes, against the oracle's store-all adjoint;
  * n_q = 30 (FP64 and FP32 forward, FP64 backward): every one of the 2^30
    amplitudes, in chunks, against oracle.grover_sampler -- the closed route
    through HALL.Inv.HALL = 2|s><s| - I, pinned against the gate-by-gate oracle
    on the CPU -- whose half sums are computed once.  The gradient uses
    grad psi_in = 2 dL C~_x U^dagger|x> for the one marked label x.

Every test prints its case and the measured normwise error before asserting.
"""

import math
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle as O
from paper_0902_0699_amd import workload as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5
TOL_GRAD = 1e-10


def _pk():
    from paper_0902_0699_amd import paperkern as pk
    return pk


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _relerr(got, want):
    return float(np.linalg.norm(got - want) / np.linalg.norm(want))


def _case(nq, eloc, seed):
    """One noisy iteration at n_q with the noise at stage boundary ``eloc``; the
    input is rounded to complex64 so that the FP64 and FP32 paths share it."""
    inst = W.single_instance(seed, nq)
    qhit, _, alpha, beta, gamma = inst["noise"]
    gates = W.grover_gates((qhit, eloc, alpha, beta, gamma))
    psi = inst["psi"].astype(np.complex64).astype(np.complex128)
    return gates, inst["marked"], psi


_ORACLE_CACHE = {}


def _oracle_forward(nq, eloc, seed):
    key = (nq, eloc, seed)
    if key not in _ORACLE_CACHE:
        _ORACLE_CACHE.clear()  # one n_q = 24 result at a time (256 MiB each)
        gates, marked, psi = _case(nq, eloc, seed)
        _ORACLE_CACHE[key] = (gates, marked, psi) + O.evaluate(nq, gates, marked, psi)
    return _ORACLE_CACHE[key]


FORWARD_CASES = [(23, e) for e in range(5)] + [(24, 1), (24, 3)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nq,eloc", FORWARD_CASES)
def test_forward_five_pass_schedule_every_element(nq, eloc, prec):
    pk = _pk()
    seed = 100 + nq
    _say("forward schedule: n_q=%d eloc=%d %s" % (nq, eloc, prec))
    gates, marked, psi, want, Lw, nw = _oracle_forward(nq, eloc, seed)
    plan = pk.Plan({"nq": nq, "gates": gates, "marked": marked}, prec=prec)
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    x = torch.from_numpy(psi).to(dt).to("cuda")
    out, L, norm = pk.evaluate(plan, x)
    got = out.cpu().numpy().astype(np.complex128)
    L, norm = float(L.item()), float(norm.item())
    err = _relerr(got, want)
    tol = TOL64 if prec == "fp64" else TOL32
    _say("  passes %d  normwise err %.3e  |dL| %.3e  |dnorm| %.3e" % (plan.passes(), err, abs(L - Lw), abs(norm - nw)))
    assert plan.passes() == 5
    assert err <= tol
    assert abs(L - Lw) <= tol * max(1.0, Lw)
    assert abs(norm - nw) <= tol * nw


def _backward_case(nq, eloc, tile, seed):
    pk = _pk()
    gates, marked, psi = _case(nq, eloc, seed)
    plan = pk.Plan({"nq": nq, "gates": gates, "marked": marked})
    if tile is not None:
        plan.set_tiling(tile, 4, 1)
    nb = len(plan.describe()["instances"][0]["backward"])
    _say("backward schedule: n_q=%d eloc=%d tile %s -> %d backward passes" % (nq, eloc, tile, nb))
    x = torch.from_numpy(psi).to("cuda")
    out, _, _ = pk.evaluate(plan, x, want_norm=False)
    dL = torch.tensor([0.75], dtype=torch.float64, device="cuda")
    gpsi, gang = pk.backward(plan, out, dL)
    gpsi = gpsi.cpu().numpy()
    gang = gang.cpu().numpy()
    wpsi, wang = O.adjoint_grad(nq, gates, marked, psi, 0.75)
    err = _relerr(gpsi, wpsi)
    aerr = float(np.max(np.abs(gang - wang.reshape(-1))) / max(1e-300, float(np.max(np.abs(wang)))))
    _say("  grad psi normwise err %.3e  angle grads rel err %.3e" % (err, aerr))
    return nb, err, aerr


@pytest.mark.parametrize("nq,eloc", [(21, e) for e in range(5)] + [(22, 2)])
def test_backward_five_pass_schedule_every_element(nq, eloc):
    nb, err, aerr = _backward_case(nq, eloc, None, 200 + nq)
    assert nb == 5
    assert err <= TOL_GRAD and aerr <= TOL_GRAD


@pytest.mark.parametrize("tile,passes", [(7, 7), (8, 5)])
@pytest.mark.parametrize("eloc", range(5))
def test_backward_small_tiles_five_and_seven_passes(tile, passes, eloc):
    """Tiles of 2^7 and 2^8 amplitudes at n_q = 16 give the 7- and 5-pass backward
    schedules.  With the rotation before the Oracle (eloc 0) it is the last gate
    walked back, after the Oracle's flip, which needs every Hadamard undone first:
    at these tiles it then takes a pass of its own."""
    nb, err, aerr = _backward_case(16, eloc, tile, 300 + eloc)
    assert nb == passes + (1 if eloc == 0 else 0)
    assert err <= TOL_GRAD and aerr <= TOL_GRAD


# --------------------------------------------------------------------------- n_q = 30, every element

NQ = W.NQ_LARGE
CHUNK = 1 << 24
WORKERS = 8


def _chunked_error(nq, amp, dev_vec, scale=1.0):
    """(sum |got - want|^2, sum |want|^2) over every label, chunk by chunk; want =
    scale * amp(labels).  Expected values are computed in threads (NumPy releases
    the GIL in its array loops) while the device chunks are copied out in order."""
    n = 1 << nq
    starts = list(range(0, n, CHUNK))

    def want_of(a):
        return scale * amp(np.arange(a, min(a + CHUNK, n), dtype=np.int64))

    d2 = r2 = 0.0
    with ThreadPoolExecutor(max_workers=WORKERS) as ex:
        futs = {}
        for i, a in enumerate(starts[:WORKERS]):
            futs[i] = ex.submit(want_of, a)
        for i, a in enumerate(starts):
            got = dev_vec[a:a + CHUNK].cpu().numpy().astype(np.complex128)
            want = futs.pop(i).result()
            if i + WORKERS < len(starts):
                futs[i + WORKERS] = ex.submit(want_of, starts[i + WORKERS])
            d2 += float(np.sum(np.abs(got - want) ** 2))
            r2 += float(np.sum(np.abs(want) ** 2))
            if i % 16 == 15:
                _say("    chunk %d/%d" % (i + 1, len(starts)))
    return d2, r2


@pytest.mark.parametrize("nq,prec", [(16, "fp64"), (26, "fp64"), (30, "fp64"), (30, "fp32")])
def test_tile_walks_are_bit_identical(nq, prec):
    """The tile walk (pk_set_pass_walk: strided, runs of c tiles, one block a
    workgroup) changes only which workgroup computes which tile: the state and L
    equal those of the strided walk bit for bit, at the sizes the bench tunes the
    walk on.  The norm partial of a tile is summed by whichever of the tile loop's
    two register buffers holds it, code the compiler may round differently (FP32
    sums a thread's terms in FP32), so the norm agrees to 1e-12 relative."""
    pk = _pk()
    seed = W.SEEDS["large_fp64"] if prec == "fp64" else W.SEEDS["large_fp32"]
    inst = W.single_instance(seed, nq)
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    plan = pk.Plan({"nq": nq, "gates": inst["gates"], "marked": inst["marked"]}, prec=prec)
    x = torch.from_numpy(inst["psi"]).to(dt).to("cuda")
    del inst["psi"]
    n = plan.passes()
    a, La, na = pk.evaluate(plan, x)
    for walks in ([-1] * n, [2] * n, [64] * n, [(0, 2, 4, 16, -1)[p % 5] for p in range(n)], [3] * n):
        _say("tile walk %s, n_q=%d %s" % (walks, nq, prec))
        plan.set_pass_walk(walks)
        assert [p["walk"] for p in plan.describe()["instances"][0]["forward"]] == walks
        b, Lb, nb = pk.evaluate(plan, x)
        torch.cuda.synchronize()
        same = bool(torch.equal(a, b))
        del b
        assert same and La.item() == Lb.item() and abs(na.item() - nb.item()) <= 1e-12 * abs(na.item())
    del a, x
    torch.cuda.empty_cache()


@pytest.mark.parametrize("nq", [14, 24])
def test_backward_tile_walks_are_bit_identical(nq):
    """Tile walks of the backward passes (pk_set_pass_walk with backward entries)
    leave the gradient bit for bit as with the strided walk."""
    pk = _pk()
    gates, marked, psi = _case(nq, 2, 40 + nq)
    plan = pk.Plan({"nq": nq, "gates": gates, "marked": marked})
    out, _, _ = pk.evaluate(plan, torch.from_numpy(psi).to("cuda"))
    dL = torch.tensor([0.5], dtype=torch.float64, device="cuda")
    g0, a0 = pk.backward(plan, out, dL)
    nf, nb = plan.passes(), len(plan.describe()["instances"][0]["backward"])
    for w in (2, 64, -1, 3):
        _say("backward tile walk %d, n_q=%d" % (w, nq))
        plan.set_pass_walk([0] * nf + [w] * nb)
        g1, a1 = pk.backward(plan, out, dL)
        torch.cuda.synchronize()
        assert bool(torch.equal(g0, g1)) and bool(torch.equal(a0, a1))


@pytest.mark.parametrize("kind,nq,prec", [("grover", 16, "fp64"), ("grover", 30, "fp64"), ("phases", 20, "fp64"),
                                          ("qft", 22, "fp64"), ("grover", 22, "fp32"), ("phases", 18, "fp32")])
def test_overlapped_tile_loop_is_bit_identical(kind, nq, prec):
    """The overlapped tile loop (pk_set_pass_overlap) only changes when the next
    tile's loads are waited for: state and L equal those of the default loop bit
    for bit, with every tile walk the bench may pick for it, at the headline size
    (whose last pass streams), on passes with product tables, and in FP32 with 4
    register bits.  The norm partial is summed by code the compiler may round
    differently in the two loops: FP64 partials agree to 1e-12 relative; FP32 sums
    FP32 terms |C|^2 whose rounding may differ (a fused multiply-add or not), each
    by at most 2^-24 of a nonnegative term, so the norm agrees to 2^-23 relative."""
    pk = _pk()
    rng = np.random.default_rng(700 + nq)
    if kind == "grover":
        seed = W.SEEDS["large_fp64"]
        inst = W.single_instance(seed, nq)
        gates, marked, psi = inst["gates"], inst["marked"], inst["psi"]
        del inst
    else:
        gates = W.phase_circuit(rng, nq, 40) if kind == "phases" else [("QFT", 1, nq)]
        marked = [int(rng.integers(0, 1 << nq))]
        v = rng.standard_normal(1 << nq) + 1j * rng.standard_normal(1 << nq)
        psi = v / np.linalg.norm(v)
    plan = pk.Plan({"nq": nq, "gates": gates, "marked": marked}, prec=prec)
    if prec == "fp32":
        plan.set_launch(0, 4)  # the FP32 kernels with the overlapped loop
    x = torch.from_numpy(psi).to(torch.complex128 if prec == "fp64" else torch.complex64).to("cuda")
    del psi
    n = plan.passes()
    a, La, na = pk.evaluate(plan, x)
    for walks in ([0] * n, [2] * n, [64] * n, [-1] * n):
        _say("overlapped loop, walks %s: %s n_q=%d %s" % (walks, kind, nq, prec))
        plan.set_pass_walk(walks)
        plan.set_pass_overlap([1] * n)
        assert all(p["overlap"] == 1 for p in plan.describe()["instances"][0]["forward"])
        b, Lb, nb = pk.evaluate(plan, x)
        torch.cuda.synchronize()
        same = bool(torch.equal(a, b))
        del b
        ntol = 1e-12 if prec == "fp64" else 2.0 ** -23
        assert same and La.item() == Lb.item() and abs(na.item() - nb.item()) <= ntol * abs(na.item())
        plan.set_pass_overlap([])
    del a, x
    torch.cuda.empty_cache()


@pytest.mark.parametrize("kind,nq,prec", [("grover", 18, "fp64"), ("grover", 20, "fp32"), ("phases", 16, "fp64"),
                                           ("phases", 16, "fp32"), ("qft", 14, "fp64"), ("qft", 20, "fp32")])
def test_lane_maps_are_bit_identical(kind, nq, prec):
    """The LDS lane maps (pk_set_lane_maps) change only which thread holds which
    amplitudes between exchanges: forward state, L and norm, and the backward's
    gradient of psi_in, equal those of the ascending thread map bit for bit.  The
    D2 angle gradients are tile sums taken thread by thread in the layout of the
    stage that holds the D2, so another thread map adds the same terms in another
    order: they agree to 1e-13 relative."""
    pk = _pk()
    rng = np.random.default_rng(500 + nq)
    if kind == "grover":
        gates, marked, psi = _case(nq, 2, 60 + nq)
    else:
        gates = W.phase_circuit(rng, nq, 40) if kind == "phases" else [("QFT", 1, nq)]
        marked = [int(rng.integers(0, 1 << nq))]
        v = rng.standard_normal(1 << nq) + 1j * rng.standard_normal(1 << nq)
        psi = v / np.linalg.norm(v)
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    plan = pk.Plan({"nq": nq, "gates": gates, "marked": marked}, prec=prec)
    inst = plan.describe()["instances"][0]
    assert any(s["nlanes"] for p in inst["forward"] + inst["backward"] for s in p["subs"])
    x = torch.from_numpy(psi).to(dt).to("cuda")
    runs = []
    for on in (1, 0):
        _say("lane maps %d: %s n_q=%d %s" % (on, kind, nq, prec))
        plan.set_lane_maps(on)
        y, L, norm = pk.evaluate(plan, x)
        grads = None
        if prec == "fp64":
            dL = torch.tensor([0.5], dtype=torch.float64, device="cuda")
            grads = pk.backward(plan, y, dL)
        torch.cuda.synchronize()
        runs.append((y, L.item(), norm.item(), grads))
    (a, La, na, ga), (b, Lb, nb, gb) = runs
    assert bool(torch.equal(a, b)) and La == Lb and na == nb
    if ga is not None:
        assert bool(torch.equal(ga[0], gb[0]))
        assert ga[1].shape == gb[1].shape
        if ga[1].numel():
            scale = float(torch.max(torch.abs(ga[1])))
            assert float(torch.max(torch.abs(ga[1] - gb[1]))) <= 1e-13 * max(scale, 1e-300)


@pytest.mark.slow
@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_full_size_forward_every_element(prec):
    pk = _pk()
    seed = W.SEEDS["large_fp64"] if prec == "fp64" else W.SEEDS["large_fp32"]
    _say("full size, every element: n_q=%d %s seed %d" % (NQ, prec, seed))
    inst = W.single_instance(seed, NQ)
    psi = inst["psi"]
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    if prec == "fp32":
        psi = psi.astype(np.complex64).astype(np.complex128)  # the input the FP32 path sees
        inst["psi"] = None
    plan = pk.Plan({"nq": NQ, "gates": inst["gates"], "marked": inst["marked"]}, prec=prec)
    x = torch.from_numpy(psi).to(dt).to("cuda")
    y, L, norm = pk.evaluate(plan, x)
    del x
    L, norm = float(L.item()), float(norm.item())
    amp, L_ref = O.grover_sampler(NQ, inst["gates"], inst["marked"], psi)
    d2, r2 = _chunked_error(NQ, amp, y)
    err = math.sqrt(d2 / r2)
    norm_in = float(np.vdot(psi, psi).real)
    tol = TOL64 if prec == "fp64" else TOL32
    _say("  passes %d  normwise err over all 2^%d amplitudes %.3e  |dL| %.3e  |dnorm| %.3e"
         % (plan.passes(), NQ, err, abs(L - L_ref), abs(norm - norm_in)))
    del y
    torch.cuda.empty_cache()
    assert plan.passes() == 5
    assert err <= tol
    assert abs(L - L_ref) <= tol * max(1.0, L_ref) * norm_in
    assert abs(norm - norm_in) <= tol * norm_in


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_full_size_backward_every_element():
    """grad psi_in of the 7-pass backward at n_q = 30 against 2 dL C~_x U^dagger|x>,
    every element (seed of the gradient workload)."""
    pk = _pk()
    seed = W.SEEDS["gradient"]
    _say("full size backward, every element: n_q=%d fp64 seed %d" % (NQ, seed))
    inst = W.single_instance(seed, NQ)
    psi = inst["psi"]
    gates, marked = inst["gates"], inst["marked"]
    plan = pk.Plan({"nq": NQ, "gates": gates, "marked": marked})
    nb = len(plan.describe()["instances"][0]["backward"])
    x = torch.from_numpy(psi).to("cuda")
    out, _, _ = pk.evaluate(plan, x, want_norm=False)
    del x
    dl = 0.75
    dL = torch.tensor([dl], dtype=torch.float64, device="cuda")
    gpsi, _ = pk.backward(plan, out, dL)
    del out
    amp, _ = O.grover_sampler(NQ, gates, marked, psi)
    cx = complex(amp(np.array(marked, dtype=np.int64))[0])
    del amp, psi, inst["psi"]
    back, _ = O.grover_sampler(NQ, O.adjoint_gates(gates), marked, ("basis", marked[0], dl * cx))
    d2, r2 = _chunked_error(NQ, back, gpsi, scale=2.0)
    err = math.sqrt(d2 / r2)
    _say("  backward passes %d  normwise err of grad psi_in over all 2^%d amplitudes %.3e" % (nb, NQ, err))
    del gpsi
    torch.cuda.empty_cache()
    assert nb == 7
    assert err <= TOL_GRAD
