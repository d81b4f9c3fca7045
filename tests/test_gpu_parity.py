"""GPU parity: the HIP path through the C-ABI against the FP64 oracle.

Tolerances (floating point, normwise over the whole state):
  FP64: ||psi_gpu - psi_ref|| / ||psi_ref|| <= 1e-12 and |L_gpu - L_ref| <= 1e-12
  FP32: the same metrics <= 1e-5
Integer / sign work (pair labels, Oracle and Inv alone) is compared bit for bit.
"""

import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_0902_0699_amd import workload as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


def _pk():
    from paper_0902_0699_amd import paperkern as pk
    return pk


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(psi, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(psi)).to(dtype).to("cuda")


def _relerr(got, want):
    return float(np.linalg.norm(got - want) / np.linalg.norm(want))


def _run(problem, psi, prec="fp64", tiling=None, inplace=False, launch=None):
    pk = _pk()
    plan = pk.Plan(problem, prec=prec)
    if tiling:
        plan.set_tiling(*tiling)
    if launch:
        plan.set_launch(*launch)
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    x = _dev(psi, dt)
    out = x if inplace else None
    psi_out, L, norm = pk.evaluate(plan, x, out=out)
    torch.cuda.synchronize()
    return plan, psi_out.cpu().numpy().astype(np.complex128), float(L.item()), float(norm.item())


def _state(rng, nq):
    v = rng.standard_normal(1 << nq) + 1j * rng.standard_normal(1 << nq)
    return v / np.linalg.norm(v)


# --------------------------------------------------------------------------- index map


@pytest.mark.parametrize("nq", [1, 3, 10, 20])
def test_pair_indices_bit_exact(nq):
    pk = _pk()
    _say("pair_indices nq=%d" % nq)
    for i_s in range(1, nq + 1):
        n0, n1 = pk.pair_indices(nq, i_s, 0, 1 << (nq - 1))
        w0, w1 = O.pair_indices(nq, i_s)
        np.testing.assert_array_equal(n0.cpu().numpy(), w0)
        np.testing.assert_array_equal(n1.cpu().numpy(), w1)


def test_pair_indices_at_thirty_qubits_sampled():
    pk = _pk()
    nq = 30
    for i_s in (1, 2, 17, 29, 30):
        for first in (0, (1 << 29) - 4096, 123456789):
            n0, n1 = pk.pair_indices(nq, i_s, first, 4096)
            b = nq - i_s
            r = np.arange(first, first + 4096, dtype=np.int64)
            want0 = ((r >> b) << (b + 1)) | (r & ((1 << b) - 1))
            np.testing.assert_array_equal(n0.cpu().numpy(), want0)
            np.testing.assert_array_equal(n1.cpu().numpy(), want0 + (1 << b))
            assert np.all(((want0 >> b) & 1) == 0)


# --------------------------------------------------------------------------- forward parity


def test_small_config_fp64():
    """The single-instance parity workload: n_q = 20, seed 0, noisy iteration."""
    inst = W.single_instance(W.SEEDS["small_fp64"], W.NQ_SMALL)
    prob = {"nq": inst["nq"], "gates": inst["gates"], "marked": inst["marked"]}
    _say("small config fp64 noise=%s" % (inst["noise"],))
    plan, got, L, norm = _run(prob, inst["psi"])
    want, Lw, nw = O.evaluate(inst["nq"], inst["gates"], inst["marked"], inst["psi"])
    assert _relerr(got, want) <= TOL64
    assert abs(L - Lw) <= TOL64
    assert abs(norm - nw) <= TOL64
    assert plan.passes() == 3


@pytest.mark.parametrize("nq", [1, 2, 3, 4, 5, 9, 10, 12, 13, 14, 17])
@pytest.mark.parametrize("eloc", [0, 2, 3])
def test_ragged_sizes_fp64(nq, eloc):
    rng = np.random.default_rng(nq * 7 + eloc)
    qhit = int(rng.integers(1, nq + 1))
    marked = sorted({int(v) for v in rng.integers(0, 1 << nq, 3)})
    prob = {"nq": nq, "gates": W.grover_gates((qhit, eloc, 0.7, 2.2, 0.3)), "marked": marked}
    psi = _state(rng, nq)
    _say("ragged nq=%d eloc=%d" % (nq, eloc))
    _, got, L, norm = _run(prob, psi)
    want, Lw, nw = O.evaluate(nq, prob["gates"], marked, psi)
    assert _relerr(got, want) <= TOL64
    assert abs(L - Lw) <= TOL64 and abs(norm - nw) <= TOL64


@pytest.mark.parametrize("tiling,launch", [((4, 0, 1), None), ((6, 2, 1), None), ((10, 4, 1), None),
                                           ((11, 4, 1), (2, 4)), ((12, 4, 1), None), ((13, 6, 1), None),
                                           ((10, 4, 0), None), ((13, 4, 0), None), ((13, 4, 1), (0, 5)),
                                           ((12, 4, 1), (0, 5)), ((7, 2, 1), (0, 5)), ((11, 3, 1), (1, 5)),
                                           ((13, 4, 1), (0, 3)), ((12, 3, 1), (0, 3)), ((9, 2, 1), (0, 3))])
def test_tilings_fp64(tiling, launch):
    nq = 15
    rng = np.random.default_rng(sum(tiling))
    prob = {"nq": nq, "gates": W.grover_gates((4, 1, 0.3, 1.1, 0.0)) + [("ONEOP", 15, O.PAULI_Y), ("H", 3)],
            "marked": [17, 30000]}
    psi = _state(rng, nq)
    _say("tiling %s launch %s" % (tiling, launch))
    _, got, L, _ = _run(prob, psi, tiling=tiling, launch=launch)
    want, Lw, _ = O.evaluate(nq, prob["gates"], prob["marked"], psi)
    assert _relerr(got, want) <= TOL64 and abs(L - Lw) <= TOL64


@pytest.mark.parametrize("lane_order", [0, 1])
def test_lane_orders_fp64(lane_order):
    """n_q = 20 tiles mix state bits 8..17 with bits >= 18, so the two lane orders
    lay the tiles out differently in registers and LDS; both match the oracle."""
    inst = W.single_instance(W.SEEDS["small_fp64"], W.NQ_SMALL)
    prob = {"nq": inst["nq"], "gates": inst["gates"], "marked": inst["marked"]}
    _say("lane_order %d at n_q=%d" % (lane_order, inst["nq"]))
    _, got, L, _ = _run(prob, inst["psi"], tiling=(13, 4, 1, lane_order))
    want, Lw, _ = O.evaluate(inst["nq"], prob["gates"], prob["marked"], inst["psi"])
    assert _relerr(got, want) <= TOL64 and abs(L - Lw) <= TOL64


def test_sign_operations_bit_exact():
    """Oracle and Inv alone only change signs: exact equality, any size and tiling."""
    rng = np.random.default_rng(5)
    for nq, tiling in [(3, None), (14, None), (16, (6, 2, 1))]:
        psi = _state(rng, nq)
        marked = [1, (1 << nq) - 1]
        prob = {"nq": nq, "gates": [("ORACLE",), ("INV",), ("ORACLE",), ("INV",), ("INV",)], "marked": marked}
        _, got, _, _ = _run(prob, psi, tiling=tiling)
        want, _, _ = O.evaluate(nq, prob["gates"], marked, psi)
        assert np.array_equal(got, want)


def test_empty_gate_list_and_no_marks():
    rng = np.random.default_rng(6)
    psi = _state(rng, 11)
    _, got, L, norm = _run({"nq": 11, "gates": [], "marked": []}, psi)
    assert np.array_equal(got, psi) and L == 0.0
    assert abs(norm - 1.0) < 1e-14


def test_in_place_evaluation():
    rng = np.random.default_rng(7)
    nq = 16
    psi = _state(rng, nq)
    prob = {"nq": nq, "gates": W.grover_gates((2, 4, 1.0, 1.0, 0.0)), "marked": [99]}
    _, got, L, _ = _run(prob, psi, inplace=True)
    want, Lw, _ = O.evaluate(nq, prob["gates"], [99], psi)
    assert _relerr(got, want) <= TOL64 and abs(L - Lw) <= TOL64


def test_random_gate_lists_fp64():
    rng = np.random.default_rng(8)
    for trial in range(6):
        nq = int(rng.integers(3, 16))
        gates = []
        for _ in range(25):
            q = int(rng.integers(1, nq + 1))
            r = int(rng.integers(0, 6))
            gates.append([("H", q), ("ONEOP", q, rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))),
                          ("D2", q, *rng.uniform(0, 3, 3)), ("ORACLE",), ("INV",), ("HALL",)][r])
        marked = [int(rng.integers(0, 1 << nq))]
        psi = _state(rng, nq)
        _say("random list trial %d nq=%d" % (trial, nq))
        _, got, L, _ = _run({"nq": nq, "gates": gates, "marked": marked}, psi)
        want, Lw, _ = O.evaluate(nq, gates, marked, psi)
        assert _relerr(got, want) <= TOL64
        assert abs(L - Lw) <= TOL64 * max(1.0, abs(Lw))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("seed,nq,tiling", [(4, 16, (5, 0, 1)), (5, 16, (5, 0, 1)), (6, 16, None), (7, 3, None),
                                           (8, 7, None)])
def test_phase_product_tables_against_oracle(prec, seed, nq, tiling):
    """Circuits dense in controlled phases: every path of the phase step (tile-part
    tables read from the lanes, the thread-part table, the per-phase loop, the
    last in the backward passes), forward and, in FP64, backward.  At n_q = 3 and
    7 most threads of the workgroup hold no amplitude."""
    pk = _pk()
    rng = np.random.default_rng(seed)
    gates = W.phase_circuit(rng, nq, 120 if nq > 8 else 30)
    prob = {"nq": nq, "gates": gates, "marked": [int(rng.integers(0, 1 << nq))]}
    psi = _state(rng, nq)
    _say("phase tables seed %d n_q=%d %s %s" % (seed, nq, prec, tiling))
    plan, got, L, _ = _run(prob, psi, prec=prec, tiling=tiling)
    want, Lw, _ = O.evaluate(nq, gates, prob["marked"], psi)
    tol = TOL64 if prec == "fp64" else TOL32
    assert _relerr(got, want) <= tol and abs(L - Lw) <= tol
    if prec == "fp64":
        out, _, _ = pk.evaluate(plan, _dev(psi))
        dL = torch.tensor([0.75], dtype=torch.float64, device="cuda")
        gpsi, _ = pk.backward(plan, out, dL)
        torch.cuda.synchronize()
        wpsi, _ = O.adjoint_grad(nq, gates, prob["marked"], psi, 0.75)
        assert _relerr(gpsi.cpu().numpy(), wpsi) <= 1e-10


def test_phase_tables_at_the_per_pass_limit_against_oracle():
    """Passes that list the 64 tile-part tables a pass may hold (one per lane of a
    wave), with the phases past the limit in the per-phase loop: forward and
    backward against the oracle."""
    pk = _pk()
    rng = np.random.default_rng(2)
    nq = 14
    gates = W.phase_circuit(rng, nq, 500)
    prob = {"nq": nq, "gates": gates, "marked": [int(rng.integers(0, 1 << nq))]}
    psi = _state(rng, nq)
    _say("phase tables at the per-pass limit, n_q=%d" % nq)
    plan, got, L, _ = _run(prob, psi, tiling=(8, 2, 1))
    assert max(len(p["urefs"]) for p in plan.describe()["instances"][0]["forward"]) == 64
    want, Lw, _ = O.evaluate(nq, gates, prob["marked"], psi)
    assert _relerr(got, want) <= TOL64 and abs(L - Lw) <= TOL64
    out, _, _ = pk.evaluate(plan, _dev(psi))
    gpsi, _ = pk.backward(plan, out, torch.tensor([0.75], dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    wpsi, _ = O.adjoint_grad(nq, gates, prob["marked"], psi, 0.75)
    assert _relerr(gpsi.cpu().numpy(), wpsi) <= 1e-10


def test_graph_replay_is_stable():
    """Repeated calls on the same buffers replay one captured graph; every replay
    matches the first, with eager torch work in between."""
    pk = _pk()
    inst = W.single_instance(11, 18)
    plan = pk.Plan({"nq": 18, "gates": inst["gates"], "marked": inst["marked"]})
    x = _dev(inst["psi"])
    y = torch.empty_like(x)
    L = torch.empty(1, dtype=torch.float64, device="cuda")
    n = torch.empty(1, dtype=torch.float64, device="cuda")
    pk.evaluate_into(plan, x, y, L, n)
    first = y.clone()
    L0 = L.clone()
    for _ in range(4):
        y.zero_()
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        pk.evaluate_into(plan, x, y, L, n)
        torch.cuda.synchronize()
        assert torch.equal(y, first) and torch.equal(L, L0)
        del junk


def test_angles_override_matches_rebuilt_plan():
    pk = _pk()
    rng = np.random.default_rng(9)
    nq = 14
    psi = _state(rng, nq)
    gates = W.grover_gates((3, 2, 0.4, 0.5, 0.0))
    plan = pk.Plan({"nq": nq, "gates": gates, "marked": [7]})
    ang = torch.tensor([1.3, 2.1, -0.2], dtype=torch.float64, device="cuda")
    out, L, _ = pk.evaluate(plan, _dev(psi), angles=ang)
    gates2 = W.grover_gates((3, 2, 1.3, 2.1, -0.2))
    want, Lw, _ = O.evaluate(nq, gates2, [7], psi)
    assert _relerr(out.cpu().numpy(), want) <= TOL64 and abs(L.item() - Lw) <= TOL64


# --------------------------------------------------------------------------- FP32


@pytest.mark.parametrize("nq,reg_bits", [(3, 4), (12, 4), (20, 4), (12, 5), (20, 5)])
def test_fp32_against_fp64_oracle(nq, reg_bits):
    inst = W.single_instance(W.SEEDS["large_fp32"], nq)
    prob = {"nq": nq, "gates": inst["gates"], "marked": inst["marked"]}
    _say("fp32 nq=%d reg_bits=%d" % (nq, reg_bits))
    _, got, L, norm = _run(prob, inst["psi"], prec="fp32", launch=(0, reg_bits))
    want, Lw, nw = O.evaluate(nq, inst["gates"], inst["marked"], inst["psi"])
    err = _relerr(got, want)
    _say("fp32 nq=%d normwise error %.3e |dL| %.3e" % (nq, err, abs(L - Lw)))
    assert err <= TOL32
    assert abs(L - Lw) <= TOL32 * max(Lw, 1.0 / (1 << nq))
    assert abs(norm - nw) <= TOL32


# --------------------------------------------------------------------------- batched


@pytest.mark.parametrize("prec,reg_bits", [("fp64", 4), ("fp32", 4), ("fp64", 5), ("fp32", 5)])
def test_batched_against_oracle(prec, reg_bits):
    pk = _pk()
    insts = W.batch_instances(W.SEEDS["batched"], count=48, nq_min=3, span=13)
    probs = [{"nq": i["nq"], "gates": i["gates"], "marked": i["marked"]} for i in insts]
    plan = pk.Plan(probs, prec=prec)
    plan.set_launch(0, reg_bits)
    offs = plan.offsets()
    packed = np.concatenate([i["psi"] for i in insts])
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    out, L, norm = pk.evaluate_batched(plan, _dev(packed, dt))
    torch.cuda.synchronize()
    out = out.cpu().numpy().astype(np.complex128)
    L = L.cpu().numpy()
    norm = norm.cpu().numpy()
    tol = TOL64 if prec == "fp64" else TOL32
    for k, inst in enumerate(insts):
        want, Lw, nw = O.evaluate(inst["nq"], inst["gates"], inst["marked"], inst["psi"])
        got = out[offs[k]:offs[k + 1]]
        assert _relerr(got, want) <= tol, k
        assert abs(L[k] - Lw) <= tol * max(1.0, Lw), k
        assert abs(norm[k] - nw) <= tol, k


@pytest.mark.parametrize("nq,prec,tile", [(16, "fp64", None), (20, "fp64", None), (24, "fp64", None),
                                          (20, "fp32", None), (18, "fp64", 10), (22, "fp32", 12)])
def test_brickwork_two_pairs_per_stage_against_oracle(nq, prec, tile):
    """Random unitary TwoOpA gates on neighbouring qubits (Eq. resmat2) in two
    brickwork layers: stages hold two disjoint qubit pairs (register bits 0, 1 and
    2, 3).  Every element against the gate-by-gate oracle."""
    import bench
    rng = np.random.default_rng(800 + nq)
    gates = bench.brickwork_gates(nq, 11 + nq)
    marked = [int(rng.integers(0, 1 << nq))]
    prob = {"nq": nq, "gates": gates, "marked": marked}
    psi = _state(rng, nq)
    _say("brickwork n_q=%d %s tile %s" % (nq, prec, tile))
    plan, got, L, norm = _run(prob, psi, prec=prec, tiling=(tile, 4, 1) if tile else None)
    desc = plan.describe()["instances"][0]["forward"]
    assert any(u["mat4b"] >= 0 for p in desc for u in p["subs"])
    want, Lw, nw = O.evaluate(nq, gates, marked, psi)
    tol = TOL64 if prec == "fp64" else TOL32
    err = _relerr(got, want)
    _say("  passes %d  normwise err %.3e" % (plan.passes(), err))
    assert err <= tol and abs(L - Lw) <= tol and abs(norm - nw) <= tol


# --------------------------------------------------------------------------- gradients


@pytest.mark.parametrize("nq,eloc", [(3, 0), (8, 1), (12, 2), (14, 3), (16, 4)])
def test_backward_against_oracle_adjoint(nq, eloc):
    pk = _pk()
    rng = np.random.default_rng(40 + nq)
    gates = W.grover_gates((int(rng.integers(1, nq + 1)), eloc, 2.0, 1.2, 0.4))
    marked = [int(rng.integers(0, 1 << nq))]
    psi = _state(rng, nq)
    plan = pk.Plan({"nq": nq, "gates": gates, "marked": marked})
    out, L, _ = pk.evaluate(plan, _dev(psi))
    dL = torch.tensor([0.75], dtype=torch.float64, device="cuda")
    gpsi, gang = pk.backward(plan, out, dL)
    torch.cuda.synchronize()
    wpsi, wang = O.adjoint_grad(nq, gates, marked, psi, 0.75)
    assert _relerr(gpsi.cpu().numpy(), wpsi) <= 1e-10
    np.testing.assert_allclose(gang.cpu().numpy(), wang.reshape(-1), rtol=1e-10, atol=1e-13)


@pytest.mark.parametrize("team_size,tile_bits,prec", [(4, 8, "fp64"), (64, 6, "fp64"), (16, 8, "fp32"),
                                                      (0, 8, "fp64")])
def test_batched_teams_against_oracle(team_size, tile_bits, prec):
    """Large instances run by teams of workgroups (a device-scope barrier between
    passes), the rest by single workgroups; small tiles make instances of
    2^10..2^14 amplitudes large enough for teams.  team_size 0: teams off."""
    pk = _pk()
    insts = W.batch_instances(W.SEEDS["batched"], count=40, nq_min=10, span=5)
    probs = [{"nq": i["nq"], "gates": i["gates"], "marked": i["marked"]} for i in insts]
    plan = pk.Plan(probs, prec=prec)
    plan.set_tiling(tile_bits, 4, 1)
    plan.set_batch(team_size, 2)
    n_teams, n_team_inst = plan.batch_teams()
    _say("batched teams: size %d tile %d %s -> %d teams, %d team instances"
         % (team_size, tile_bits, prec, n_teams, n_team_inst))
    if team_size:
        assert n_teams > 0 and n_team_inst > 0
    else:
        assert n_teams == 0 and n_team_inst == 0
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    packed = _dev(np.concatenate([i["psi"] for i in insts]), dt)
    tol = TOL64 if prec == "fp64" else TOL32
    for rep in range(2):  # graph replay: counters and barriers start from zero each launch
        res, L, norm = pk.evaluate_batched(plan, packed)
        torch.cuda.synchronize()
        res = res.cpu().numpy().astype(np.complex128)
        offs = plan.offsets()
        for k, (p, inst) in enumerate(zip(probs, insts)):
            want, Lw, nw = O.evaluate(p["nq"], p["gates"], p["marked"], inst["psi"])
            assert _relerr(res[offs[k]:offs[k + 1]], want) <= tol
            assert abs(float(L[k]) - Lw) <= tol and abs(float(norm[k]) - nw) <= tol


def test_batched_large_instances_run_by_teams():
    """Default settings: instances of 2^23 amplitudes go to teams (one workgroup per
    instance would leave most CUs idle), small ones to the queue.  Outputs are
    checked at sampled labels against the oracle's closed form."""
    pk = _pk()
    rng = np.random.default_rng(31)
    insts = [W.draw_instance(rng, nq) for nq in (23, 11, 23, 9)]
    probs = [{"nq": i["nq"], "gates": i["gates"], "marked": i["marked"]} for i in insts]
    plan = pk.Plan(probs)
    n_teams, n_team_inst = plan.batch_teams()
    _say("large batch: %d teams, %d team instances" % (n_teams, n_team_inst))
    assert n_teams > 0 and n_team_inst == 2
    packed = _dev(np.concatenate([i["psi"] for i in insts]))
    res, L, norm = pk.evaluate_batched(plan, packed)
    torch.cuda.synchronize()
    offs = plan.offsets()
    for k, inst in enumerate(insts):
        nq = inst["nq"]
        idx = np.unique(np.concatenate([rng.integers(0, 1 << nq, 4096), inst["marked"]]))
        want, Lw = O.grover_sampled(nq, inst["gates"], inst["marked"], inst["psi"], idx)
        got = res[offs[k]:offs[k + 1]][torch.from_numpy(idx).to("cuda")].cpu().numpy()
        err = math.sqrt(np.mean(np.abs(got - want) ** 2) * (1 << nq))
        assert err <= TOL64 and abs(float(L[k]) - Lw) <= TOL64 and abs(float(norm[k]) - 1.0) <= TOL64
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = {}
    for ts in (16, 0):
        plan.set_batch(ts, 64)
        out = torch.empty_like(packed)
        pk.evaluate_batched(plan, packed, out=out)
        e0.record()
        pk.evaluate_batched(plan, packed, out=out)
        e1.record()
        torch.cuda.synchronize()
        times[ts] = e0.elapsed_time(e1)
    _say("  teams %.3f ms, single workgroups %.3f ms" % (times[16], times[0]))


def test_autotuned_batched_plan_matches_oracle():
    """The tuner times every candidate on the caller's buffers and leaves the fastest
    applied; the tuned plan still matches the oracle instance by instance."""
    pk = _pk()
    from paper_0902_0699_amd import autotune as AT
    insts = W.batch_instances(W.SEEDS["batched"], count=48, nq_min=6, span=10)
    probs = [{"nq": i["nq"], "gates": i["gates"], "marked": i["marked"]} for i in insts]
    plan = pk.Plan(probs)
    packed = _dev(np.concatenate([i["psi"] for i in insts]))
    out = torch.empty_like(packed)
    _say("autotune batched 48 instances")
    best, table = AT.tune(plan, lambda: pk.evaluate_batched(plan, packed, out=out), op="batched",
                          reps=2, use_cache=False)
    assert best == table[0][0] and all(table[i][1] <= table[i + 1][1] for i in range(len(table) - 1))
    res, L, _ = pk.evaluate_batched(plan, packed)
    torch.cuda.synchronize()
    res = res.cpu().numpy()
    offs = plan.offsets()
    for k, (p, inst) in enumerate(zip(probs, insts)):
        want, Lw, _ = O.evaluate(p["nq"], p["gates"], p["marked"], inst["psi"])
        assert _relerr(res[offs[k]:offs[k + 1]], want) <= TOL64
        assert abs(float(L[k]) - Lw) <= TOL64


def test_backward_rejects_non_unitary_oneop():
    pk = _pk()
    plan = pk.Plan({"nq": 5, "gates": [("ONEOP", 2, [[2.0, 0], [0, 1.0]])], "marked": [1]})
    x = _dev(_state(np.random.default_rng(1), 5))
    out, _, _ = pk.evaluate(plan, x)
    with pytest.raises(pk.PaperkernError) as e:
        pk.backward(plan, out, torch.ones(1, dtype=torch.float64, device="cuda"))
    assert e.value.code == pk.PK_EUNSUPPORTED


def test_autograd_function_gradcheck():
    pk = _pk()
    nq = 5
    rng = np.random.default_rng(12)
    gates = W.grover_gates((2, 2, 0.9, 1.4, 0.1))
    plan = pk.Plan({"nq": nq, "gates": gates, "marked": [6, 19]})
    psi = _dev(_state(rng, nq)).requires_grad_(True)
    ang = torch.tensor([0.9, 1.4, 0.1], dtype=torch.float64, device="cuda", requires_grad=True)

    def f(p, a):
        return pk.grover_eval(plan, p, a)[0]

    assert torch.autograd.gradcheck(f, (psi, ang), eps=1e-6, atol=1e-8, rtol=1e-6)


# --------------------------------------------------------------------------- two-qubit gates


def _gates2(rng, nq, count, unitary=True):
    """Random lists mixing one-qubit gates, diagonal ops and the two-qubit kinds
    (TWOOP, CNOT, CPHASE, CPHASEK, SWAP, D4 of Sec. 4 and Sec. 6.3)."""
    gates = []
    for _ in range(count):
        r = int(rng.integers(0, 11))
        q1, q2 = (int(v) for v in rng.choice(np.arange(1, nq + 1), 2, replace=False))
        if r == 0:
            gates.append(("H", q1))
        elif r == 1:
            gates.append(("D2", q1, *rng.uniform(0, 3, 3)))
        elif r == 2:
            gates.append(("ORACLE",))
        elif r == 3:
            gates.append(("INV",))
        elif r == 4:
            m = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
            if unitary:
                m, _ = np.linalg.qr(m)
            gates.append(("TWOOP", q1, q2, m))
        elif r == 5:
            gates.append(("CNOT", q1, q2))
        elif r == 6:
            gates.append(("CPHASE", q1, q2))
        elif r == 7:
            gates.append(("CPHASEK", q1, q2, int(rng.integers(1, 6))))
        elif r == 8:
            gates.append(("SWAP", q1, q2))
        elif r == 9:
            gates.append(("D4", q1, q2, *rng.uniform(-2, 2, 3)))
        else:
            gates.append(("HALL",))
    return gates


@pytest.mark.parametrize("nq,tiling,launch,prec", [(2, None, None, "fp64"), (5, None, None, "fp64"),
                                                   (10, (6, 2, 1), None, "fp64"), (14, None, None, "fp64"),
                                                   (14, (13, 4, 1), (0, 5), "fp64"), (12, (5, 0, 0), None, "fp64"),
                                                   (15, (10, 4, 1), (2, 4), "fp64"), (14, None, None, "fp32"),
                                                   (9, (6, 2, 1), (0, 4), "fp32"), (14, (13, 4, 1), (0, 3), "fp64"),
                                                   (13, (12, 3, 1), (0, 3), "fp32")])
def test_two_qubit_gates_against_oracle(nq, tiling, launch, prec):
    rng = np.random.default_rng(500 + nq + (tiling[0] if tiling else 0))
    gates = _gates2(rng, nq, 24, unitary=(nq % 2 == 0)) + [("CNOT", 1, nq), ("D4", nq, 1, 0.3, 1.9, -0.6)]
    prob = {"nq": nq, "gates": gates, "marked": sorted({int(v) for v in rng.integers(0, 1 << nq, 2)})}
    psi = _state(rng, nq)
    _say("two-qubit n_q=%d tiling %s launch %s %s" % (nq, tiling, launch, prec))
    _, got, L, norm = _run(prob, psi, prec=prec, tiling=tiling, launch=launch)
    want, Lw, nw = O.evaluate(nq, gates, prob["marked"], psi)
    tol = TOL64 if prec == "fp64" else TOL32
    scale = max(1.0, float(np.linalg.norm(want)))
    assert _relerr(got, want) <= tol
    assert abs(L - Lw) <= tol * scale * scale and abs(norm - nw) <= tol * scale * scale


def test_named_two_qubit_gates_bit_exact():
    """CNOT, CPHASE and SWAP permute or negate amplitudes: the products with 0 and 1
    entries are exact, so the GPU matches the oracle bit for bit."""
    rng = np.random.default_rng(77)
    nq = 12
    gates = [("CNOT", 3, 9), ("SWAP", 12, 1), ("CPHASE", 5, 2), ("CNOT", 11, 4), ("SWAP", 6, 7), ("ORACLE",)]
    psi = _state(rng, nq)
    _, got, _, _ = _run({"nq": nq, "gates": gates, "marked": [100]}, psi)
    want, _, _ = O.evaluate(nq, gates, [100], psi)
    np.testing.assert_array_equal(got, want)


def test_two_qubit_batched_against_oracle():
    pk = _pk()
    rng = np.random.default_rng(78)
    probs, psis = [], []
    for nq in (3, 9, 14, 6, 11, 2):
        probs.append({"nq": nq, "gates": _gates2(rng, nq, 12) + [("SWAP", 1, nq)], "marked": [0, (1 << nq) - 1]})
        psis.append(_state(rng, nq))
    plan = pk.Plan(probs)
    res, L, _ = pk.evaluate_batched(plan, _dev(np.concatenate(psis)))
    torch.cuda.synchronize()
    res = res.cpu().numpy()
    offs = plan.offsets()
    for k, (p, psi) in enumerate(zip(probs, psis)):
        want, Lw, _ = O.evaluate(p["nq"], p["gates"], p["marked"], psi)
        assert _relerr(res[offs[k]:offs[k + 1]], want) <= TOL64 and abs(float(L[k]) - Lw) <= TOL64


@pytest.mark.parametrize("nq", [4, 9, 14])
def test_two_qubit_backward_against_oracle_adjoint(nq):
    pk = _pk()
    rng = np.random.default_rng(600 + nq)
    gates = (W.grover_gates((2, 1, 0.5, 1.2, 0.3)) + [("D4", nq, 1, 0.4, -1.3, 0.8)] + _gates2(rng, nq, 16)
             + [("D4", 2, 3, 1.1, 0.7, -0.2), ("CPHASEK", 1, nq, 3)])
    marked = [int(rng.integers(0, 1 << nq)), 3]
    psi = _state(rng, nq)
    plan = pk.Plan({"nq": nq, "gates": gates, "marked": marked})
    x = _dev(psi)
    out, _, _ = pk.evaluate(plan, x, want_norm=False)
    dL = torch.tensor([0.6], dtype=torch.float64, device="cuda")
    _say("two-qubit backward n_q=%d" % nq)
    gpsi, gang = pk.backward(plan, out, dL)
    torch.cuda.synchronize()
    wpsi, wang = O.adjoint_grad(nq, gates, marked, psi, 0.6)
    assert _relerr(gpsi.cpu().numpy(), wpsi) <= 1e-10
    np.testing.assert_allclose(gang.cpu().numpy().reshape(-1, 3), wang, rtol=1e-9, atol=1e-12)


def test_gradcheck_with_d4_angles():
    pk = _pk()
    nq = 5
    rng = np.random.default_rng(13)
    gates = [("HALL",), ("D4", 2, 5, 0.3, 1.1, -0.4), ("CNOT", 1, 3), ("D2", 4, 0.2, 0.9, 0.0), ("ORACLE",),
             ("HALL",), ("INV",), ("HALL",)]
    plan = pk.Plan({"nq": nq, "gates": gates, "marked": [6, 19]})
    psi = _dev(_state(rng, nq)).requires_grad_(True)
    ang = torch.tensor([0.3, 1.1, -0.4, 0.2, 0.9, 0.0], dtype=torch.float64, device="cuda", requires_grad=True)

    def f(p, a):
        return pk.grover_eval(plan, p, a)[0]

    assert torch.autograd.gradcheck(f, (psi, ang), eps=1e-6, atol=1e-8, rtol=1e-6)
