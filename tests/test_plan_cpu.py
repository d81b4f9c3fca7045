"""Host logic of the library on the CPU: exported symbols, argument checks, and the
pass schedules the plan compiler emits (executed by tests/schedule_emulator.py
and compared with the oracle).  No GPU call is made here."""

import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_0902_0699_amd import paperkern as pk
from paper_0902_0699_amd import workload as W
from schedule_emulator import run_backward, run_forward

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "paperkern.h")


def _state(rng, nq):
    v = rng.standard_normal(1 << nq) + 1j * rng.standard_normal(1 << nq)
    return v / np.linalg.norm(v)


def test_library_exports_every_declared_symbol():
    with open(HEADER) as f:
        text = f.read()
    declared = set(re.findall(r"^\s*(?:int|void|const char\*)\s+(pk_\w+)\s*\(", text, re.M))
    assert len(declared) >= 15
    lib = pk.lib()
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert set(pk.SIGNATURES) == declared


def test_error_codes_and_strings():
    lib = pk.lib()
    assert lib.pk_strerror(pk.PK_EINVAL) == b"invalid argument"
    assert lib.pk_strerror(pk.PK_EUNSUPPORTED) == b"unsupported request"
    assert lib.pk_strerror(12345) == b"unknown error code"


@pytest.mark.parametrize("bad,msg", [
    ({"nq": 0, "gates": [], "marked": []}, "nq"),
    ({"nq": 31, "gates": [], "marked": []}, "nq"),
    ({"nq": 4, "gates": [("H", 5)], "marked": []}, "qubit"),
    ({"nq": 4, "gates": [("D2", 0, 0.1, 0.2, 0.0)], "marked": []}, "qubit"),
    ({"nq": 4, "gates": [("ONEOP", 2, [[np.nan, 0], [0, 1]])], "marked": []}, "non-finite"),
    ({"nq": 4, "gates": [("D2", 1, np.inf, 0.2, 0.0)], "marked": []}, "non-finite"),
    ({"nq": 4, "gates": [], "marked": [16]}, "out of range"),
    ({"nq": 4, "gates": [], "marked": [3, 3]}, "duplicate"),
])
def test_create_rejects_bad_problems(bad, msg):
    with pytest.raises(pk.PaperkernError) as e:
        pk.Plan(bad)
    assert e.value.code == pk.PK_EINVAL
    assert msg in str(e.value)


def test_fp32_allows_31_qubits_and_tiling_limits():
    plan = pk.Plan({"nq": 31, "gates": [("HALL",)], "marked": [5]}, prec="fp32")
    assert plan.passes() >= 3
    with pytest.raises(pk.PaperkernError):
        plan.set_tiling(15)
    plan64 = pk.Plan({"nq": 8, "gates": [("HALL",)], "marked": []})
    with pytest.raises(pk.PaperkernError):
        plan64.set_tiling(14)
    with pytest.raises(pk.PaperkernError):
        plan64.set_launch(0, 6)
    with pytest.raises(pk.PaperkernError):
        plan64.set_launch(9, 4)
    with pytest.raises(pk.PaperkernError):
        plan64.set_tiling(10, carrier_bits=7)
    with pytest.raises(pk.PaperkernError):
        plan64.set_tiling(10, fuse=2)
    with pytest.raises(pk.PaperkernError):
        plan64.set_tiling(10, lane_order=2)
    with pytest.raises(pk.PaperkernError):
        plan64.set_batch(65, 4)
    with pytest.raises(pk.PaperkernError):
        plan64.set_batch(16, 0)
    plan64.set_batch(0, 1)


def test_offsets_and_angles_bookkeeping():
    probs = [{"nq": n, "gates": W.grover_gates((1, 2, 0.5, 0.25, 0.0)) if n != 3 else W.grover_gates(),
              "marked": [1]} for n in (3, 5, 4)]
    plan = pk.Plan(probs)
    assert plan.offsets() == [0, 8, 40, 56]
    assert plan.n_angles() == 2
    assert plan.workspace_bytes(pk.PK_OP_EVAL) > 0
    assert plan.workspace_bytes(pk.PK_OP_BACKWARD) >= plan.workspace_bytes(pk.PK_OP_EVAL)


def test_pass_counts_at_thirty_qubits():
    """One noisy Grover iteration at n_q = 30 with 2^13-amplitude tiles, 4 carriers:
    13 + 9 + 8 qubits per group, so 5 passes (2 groups x 2 HALLs + the Inv pass)."""
    inst = W.draw_instance(np.random.default_rng(1), 30, with_state=False)
    plan = pk.Plan({"nq": 30, "gates": inst["gates"], "marked": inst["marked"]})
    assert plan.passes() == 5
    plan32 = pk.Plan({"nq": 30, "gates": inst["gates"], "marked": inst["marked"]}, prec="fp32")
    assert plan32.passes() == 5
    plan.set_launch(0, 5)
    assert plan.passes() == 5
    stages = [len(p["stages"]) for p in plan.describe()["instances"][0]["forward"]]
    assert sum(stages) <= 13  # five register bits: fewer LDS exchanges than with four
    plan.set_tiling(13, 4, fuse=0)
    assert plan.passes() == 61  # one sweep per one-qubit gate (2 HALL x 30 + D2)


@pytest.mark.parametrize("lane_order", [0, 1])
def test_lane_order_relabels_tile_bits_only(lane_order):
    """With lane_order 1 a tile that mixes state bits 8..17 with bits >= 18 lists the
    latter first after the carriers; either order computes the oracle's state."""
    nq = 20
    inst = W.single_instance(0, nq)
    prob = {"nq": nq, "gates": inst["gates"], "marked": inst["marked"]}
    plan = pk.Plan(prob)
    plan.set_tiling(13, 4, 1, lane_order)
    desc = plan.describe()
    tbs = [p["tile_bits"] for p in desc["instances"][0]["forward"]]
    mixed = [tb for tb in tbs if any(8 <= b < 18 for b in tb) and any(b >= 18 for b in tb)]
    assert mixed
    for tb in mixed:
        assert tb[:4] == [0, 1, 2, 3]
        rest = tb[4:]
        if lane_order == 0:
            assert rest == sorted(rest)
        else:
            good = [b for b in rest if b < 8 or b >= 18]
            assert rest[:len(good)] == sorted(good) and rest != sorted(rest)
    got, L = run_forward([prob], desc, 0, inst["psi"])
    want, Lw, _ = O.evaluate(nq, prob["gates"], prob["marked"], inst["psi"])
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)
    assert abs(L - Lw) < 1e-13


def test_autotune_candidates_are_accepted_and_signature_is_structural():
    from paper_0902_0699_amd import autotune as AT
    insts = W.batch_instances(3, count=12)
    probs = [{"nq": i["nq"], "gates": i["gates"], "marked": i["marked"]} for i in insts]
    for prec in ("fp64", "fp32"):
        plan = pk.Plan(probs, prec=prec)
        cands = AT.candidates(plan.prec, "batched")
        assert len(cands) >= 8 and all(set(c) == set(AT.FIELDS) for c in cands)
        for c in cands:
            AT.apply(plan, c)  # host-side recompile; raises if a candidate were invalid
        assert plan.passes() >= 1
        assert all(c["reg_bits"] in (4, 5) for c in cands)
        single = pk.Plan(probs[:1], prec=prec)
        ev = AT.candidates(single.prec, "eval")
        assert {c["reg_bits"] for c in ev} == {3, 4, 5} and {c["carrier_bits"] for c in ev} == {3, 4, 5}
        for c in ev:
            AT.apply(single, c)
            assert c["tile_bits"] - c["reg_bits"] <= 10
    # same structure, other angles and marks: same key; other qubit: other key
    a = [{"nq": 12, "gates": W.grover_gates((3, 2, 0.1, 0.2, 0.0)), "marked": [5]}]
    b = [{"nq": 12, "gates": W.grover_gates((3, 2, 1.1, 2.2, 0.0)), "marked": [77]}]
    c = [{"nq": 12, "gates": W.grover_gates((4, 2, 0.1, 0.2, 0.0)), "marked": [5]}]
    sig = lambda pr: AT.signature(pk.Plan(pr), "eval")
    assert sig(a) == sig(b) != sig(c)
    # every structural field counts: QFT register start and size, the qubits of
    # two-qubit gates, the CPHASEK exponent, D4 qubits
    one = lambda *g: [{"nq": 24, "gates": list(g), "marked": []}]
    keys = [sig(one(("QFT", 1, 20))), sig(one(("QFT", 1, 10))), sig(one(("QFT", 2, 10))),
            sig(one(("QFT_NOSWAP", 1, 20))), sig(one(("CNOT", 1, 2))), sig(one(("CNOT", 2, 1))),
            sig(one(("CNOT", 3, 4))), sig(one(("CPHASEK", 1, 2, 3))), sig(one(("CPHASEK", 1, 2, 4))),
            sig(one(("SWAP", 1, 2))), sig(one(("SWAP", 5, 9))), sig(one(("D4", 1, 2, 0.1, 0.2, 0.3))),
            sig(one(("D4", 2, 3, 0.1, 0.2, 0.3))), sig(one(("TWOOP", 1, 2, np.eye(4)))),
            sig(one(("TWOOP", 1, 3, np.eye(4))))]
    assert len(set(keys)) == len(keys)
    assert sig(one(("D4", 1, 2, 0.1, 0.2, 0.3))) == sig(one(("D4", 1, 2, 1.1, 1.2, 1.3)))
    assert sig(one(("TWOOP", 1, 2, np.eye(4)))) == sig(one(("TWOOP", 1, 2, 2 * np.eye(4))))


def test_three_register_bits_limits():
    """reg_bits 3: at most 1024 threads a workgroup (tile_bits - reg_bits <= 10), and
    the batched launch, which has 4 and 5 register bits only, refuses the plan
    before it touches the device."""
    import ctypes
    prob = {"nq": 16, "gates": W.grover_gates((3, 2, 0.4, 0.2, 0.1)), "marked": [5]}
    p32 = pk.Plan(prob, prec="fp32")
    p32.set_tiling(14, 4, 1)
    with pytest.raises(pk.PaperkernError, match="1024 threads"):
        p32.set_launch(0, 3)
    p32.set_tiling(13, 4, 1)
    p32.set_launch(0, 3)
    with pytest.raises(pk.PaperkernError, match="1024 threads"):
        p32.set_tiling(14, 4, 1)
    assert pk.lib().pk_evaluate_batched(p32.handle, None, None, None, None, None, None, None) == pk.PK_EUNSUPPORTED
    d = p32.describe()
    assert {p["rbits"] for p in d["instances"][0]["forward"]} == {3}
    assert all(p["rbits"] == 4 for p in d["instances"][0]["backward"])


def test_binding_step_one_register_sizes_and_search_length():
    """The binding's host helpers that set up GPU cases: Shor's Step 1 register sizes
    against the footnote values and the oracle, and n_t = floor((pi/4) sqrt(N)) (the
    floor reading of Sec. 5.1) against an exact integer test: n_t is the largest k
    with 16 k^2 <= pi^2 N, pi^2 taken to 40 digits."""
    from decimal import Decimal, getcontext
    with open(os.path.join(ROOT, "tests", "golden", "shor_examples.txt")) as f:
        rows = [ln.split(":") for ln in f if ln.startswith("sizes:")]
    assert rows
    for _, m, sizes in rows:
        assert pk.shor_register_sizes(int(m)) == tuple(int(v) for v in sizes.split())
    for M in range(2, 5000):
        assert pk.shor_register_sizes(M) == O.shor_register_sizes(M)
    getcontext().prec = 60
    pi2 = Decimal("9.869604401089358618834490999876151135313699407240790626413349")
    for nq in range(1, 41):
        n_t = pk.grover_iterations(nq)
        N = Decimal(1 << nq)
        assert 16 * Decimal(n_t) ** 2 <= pi2 * N < 16 * Decimal(n_t + 1) ** 2
        if nq >= 3:  # the rotation closed form: success probability after n_t steps
            th = math.asin(2.0 ** (-nq / 2))
            assert math.sin((2 * n_t + 1) * th) ** 2 > 0.9


def test_page_cap_spreads_large_stride_bits_over_passes():
    """FP64 default (page_cap 4): no n_q = 30 tile holds more than 5 state bits >= 17
    (2 MiB byte stride), still 5 passes; without the cap the pass holding Inv has 8."""
    inst = W.draw_instance(np.random.default_rng(1), 30, with_state=False)
    prob = {"nq": 30, "gates": inst["gates"], "marked": inst["marked"]}
    plan = pk.Plan(prob)
    tiles = [p["tile_bits"] for p in plan.describe()["instances"][0]["forward"]]
    assert len(tiles) == 5 and max(sum(b >= 17 for b in tb) for tb in tiles) <= 5
    plan.set_tiling(13, 4, 1, 1, 0)
    tiles0 = [p["tile_bits"] for p in plan.describe()["instances"][0]["forward"]]
    assert len(tiles0) == 5 and max(sum(b >= 17 for b in tb) for tb in tiles0) == 8
    with pytest.raises(pk.PaperkernError):
        plan.set_tiling(13, 4, 1, 1, 17)


def test_pair_indices_rejects_bad_ranges():
    lib = pk.lib()
    assert lib.pk_pair_indices(0, 1, 0, 1, None, None, None) == pk.PK_EINVAL
    assert lib.pk_pair_indices(5, 6, 0, 1, None, None, None) == pk.PK_EINVAL
    assert lib.pk_pair_indices(5, 2, 10, 7, None, None, None) == pk.PK_EINVAL


# --------------------------------------------------------------------------- schedules


def _check_forward(problem, psi, tiling=None, prec="fp64", reg_bits=4):
    plan = pk.Plan(problem, prec=prec)
    if tiling:
        plan.set_tiling(*tiling)
    if reg_bits != 4:
        plan.set_launch(0, reg_bits)
    desc = plan.describe()
    got, L = run_forward([problem], desc, 0, psi)
    want, Lw, _ = O.evaluate(problem["nq"], problem["gates"], problem["marked"], psi)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)
    assert abs(L - Lw) < 1e-13
    return plan, desc


@pytest.mark.parametrize("nq", [1, 2, 3, 4, 5, 8, 13, 14, 16])
@pytest.mark.parametrize("eloc", [0, 2, 4])
@pytest.mark.parametrize("reg_bits", [3, 4, 5])
def test_grover_schedule_matches_oracle(nq, eloc, reg_bits):
    rng = np.random.default_rng(nq * 10 + eloc)
    qhit = int(rng.integers(1, nq + 1))
    prob = {"nq": nq, "gates": W.grover_gates((qhit, eloc, 1.1, 0.6, 0.2)),
            "marked": [int(rng.integers(0, 1 << nq))]}
    _check_forward(prob, _state(rng, nq), reg_bits=reg_bits)


@pytest.mark.parametrize("tiling", [(4, 0, 1), (5, 2, 1), (6, 3, 1), (7, 4, 1), (6, 2, 0), (10, 6, 1)])
@pytest.mark.parametrize("eloc", [1, 3])
def test_grover_schedule_small_tiles(tiling, eloc):
    nq = 12
    rng = np.random.default_rng(eloc)
    prob = {"nq": nq, "gates": W.grover_gates((7, eloc, 2.1, 1.3, 0.0)), "marked": [5, 4000]}
    plan, _ = _check_forward(prob, _state(rng, nq), tiling)
    assert plan.passes() >= 2


def _random_gates(rng, nq, count):
    gates = []
    for _ in range(count):
        r = rng.integers(0, 7)
        q = int(rng.integers(1, nq + 1))
        if r == 0:
            gates.append(("H", q))
        elif r == 1:
            m = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
            gates.append(("ONEOP", q, m))
        elif r == 2:
            gates.append(("D2", q, *rng.uniform(0, 3, 3)))
        elif r == 3:
            gates.append(("ORACLE",))
        elif r == 4:
            gates.append(("INV",))
        elif r == 5:
            gates.append(("HALL",))
        else:
            gates.append(("ONEOP", q, O.PAULI_Y))
    return gates


@pytest.mark.parametrize("seed", range(12))
def test_random_gate_lists(seed):
    rng = np.random.default_rng(1000 + seed)
    nq = int(rng.integers(1, 11))
    gates = _random_gates(rng, nq, int(rng.integers(0, 40)))
    marked = sorted({int(v) for v in rng.integers(0, 1 << nq, int(rng.integers(0, 4)))})
    prob = {"nq": nq, "gates": gates, "marked": marked}
    tiling = [None, (4, 1, 1), (6, 2, 1), (5, 0, 0)][seed % 4]
    if tiling and tiling[0] > nq:
        tiling = None
    _check_forward(prob, _state(rng, nq), tiling)


@pytest.mark.parametrize("nq,eloc,tiling", [(3, 0, None), (6, 1, None), (9, 2, (5, 2, 1)), (12, 3, (6, 2, 1)),
                                            (14, 4, None), (11, 2, (4, 0, 0))])
def test_backward_schedule_matches_oracle_adjoint(nq, eloc, tiling):
    rng = np.random.default_rng(77 + nq)
    gates = W.grover_gates((int(rng.integers(1, nq + 1)), eloc, 1.7, 0.8, 0.3)) + [("D2", 1, 0.2, 1.9, -0.4)]
    prob = {"nq": nq, "gates": gates, "marked": [int(rng.integers(0, 1 << nq)), 0]}
    psi = _state(rng, nq)
    plan = pk.Plan(prob)
    if tiling:
        plan.set_tiling(*tiling)
    desc = plan.describe()
    psi_out, _, _ = O.evaluate(nq, gates, prob["marked"], psi)
    gpsi, gang = run_backward([prob], desc, 0, psi_out, 0.5)
    wpsi, wang = O.adjoint_grad(nq, gates, prob["marked"], psi, 0.5)
    np.testing.assert_allclose(gpsi, wpsi, rtol=0, atol=1e-12)
    np.testing.assert_allclose(gang, wang, rtol=0, atol=1e-12)


def _random_gates2(rng, nq, count, unitary=True):
    """Random lists mixing one-qubit gates, diagonal ops and the two-qubit kinds."""
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


@pytest.mark.parametrize("seed", range(10))
def test_two_qubit_gate_schedules_match_oracle(seed):
    rng = np.random.default_rng(3000 + seed)
    nq = int(rng.integers(2, 11))
    gates = _random_gates2(rng, nq, int(rng.integers(1, 30)), unitary=(seed % 2 == 0))
    marked = sorted({int(v) for v in rng.integers(0, 1 << nq, int(rng.integers(0, 3)))})
    prob = {"nq": nq, "gates": gates, "marked": marked}
    tiling = [None, (4, 1, 1), (6, 2, 1), (5, 0, 0), (7, 3, 1)][seed % 5]
    if tiling and tiling[0] > nq:
        tiling = None
    plan, desc = _check_forward(prob, _state(rng, nq), tiling, reg_bits=5 if seed % 3 == 2 else 4)
    for p in desc["instances"][0]["forward"]:
        for st in p["stages"]:
            pairs = {(st["rb"][op["a"]], st["rb"][op["a"] + 1]) for op in st["ops"] if op["kind"] == "MAT4"}
            assert len(pairs) <= 2 and len({b for pr in pairs for b in pr}) == 2 * len(pairs)


@pytest.mark.parametrize("nq,tiling,reg_bits", [(8, (6, 2, 1), 4), (12, (7, 3, 1), 4), (14, (8, 4, 1), 5),
                                                (16, None, 4), (11, (6, 2, 1), 5)])
def test_brickwork_stages_hold_two_disjoint_pairs(nq, tiling, reg_bits):
    """A brickwork of random unitary TwoOpA gates on neighbouring qubits (Eq. resmat2):
    stages take two disjoint qubit pairs, on register bits 0, 1 and 2, 3; the packed
    schedule, executed on the CPU, equals the gate-by-gate oracle, forward and back."""
    import bench
    rng = np.random.default_rng(500 + nq)
    gates = bench.brickwork_gates(nq, 7 + nq)
    prob = {"nq": nq, "gates": gates, "marked": [int(rng.integers(0, 1 << nq))]}
    psi = _state(rng, nq)
    plan, desc = _check_forward(prob, psi, tiling, reg_bits=reg_bits)
    two = [st for p in desc["instances"][0]["forward"] for st in p["stages"]
           if len({op["a"] for op in st["ops"] if op["kind"] == "MAT4"}) == 2]
    assert two, "no stage holds two pairs"
    subs = [u for p in desc["instances"][0]["forward"] for u in p["subs"]]
    assert any(u["mat4b"] >= 0 for u in subs)
    psi_out, _, _ = O.evaluate(nq, gates, prob["marked"], psi)
    gpsi, _ = run_backward([prob], desc, 0, psi_out, 0.5)
    wpsi, _ = O.adjoint_grad(nq, gates, prob["marked"], psi, 0.5)
    np.testing.assert_allclose(gpsi, wpsi, rtol=0, atol=1e-12)


def test_brickwork_at_thirty_qubits_takes_four_passes():
    """The 29-gate brickwork at n_q = 30 in 2^13 tiles: 4 passes.  The large-stride
    tile-bit preference (page_cap) would cost three more here, so the compiler drops
    it for this list; the noisy Grover iteration keeps it (5 passes either way)."""
    import bench
    plan = pk.Plan({"nq": 30, "gates": bench.brickwork_gates(30, 5), "marked": [0]})
    assert plan.passes() == 4
    stages = [len(p["stages"]) for p in plan.describe()["instances"][0]["forward"]]
    assert sum(stages) <= 18
    inst = W.draw_instance(np.random.default_rng(1), 30, with_state=False)
    g = pk.Plan({"nq": 30, "gates": inst["gates"], "marked": inst["marked"]})
    assert g.passes() == 5
    # bits at byte strides of 2 MiB or more (17 and up in FP64) stay spread: at most 5 a pass
    big = [sum(b >= 17 for b in p["tile_bits"]) for p in g.describe()["instances"][0]["forward"]]
    assert max(big) <= 5


@pytest.mark.parametrize("nq,tiling", [(6, None), (9, (5, 2, 1)), (12, (6, 2, 1)), (11, (4, 0, 0))])
def test_two_qubit_backward_schedule_matches_oracle_adjoint(nq, tiling):
    rng = np.random.default_rng(90 + nq)
    gates = (W.grover_gates((3, 2, 0.4, 1.3, 0.2)) + [("D4", nq, 1, 0.7, -1.1, 0.5), ("CNOT", 2, nq)]
             + _random_gates2(rng, nq, 10) + [("D4", 2, 3, -0.3, 2.2, 1.0)])
    prob = {"nq": nq, "gates": gates, "marked": [int(rng.integers(0, 1 << nq)), 1]}
    psi = _state(rng, nq)
    plan = pk.Plan(prob)
    if tiling:
        plan.set_tiling(*tiling)
    desc = plan.describe()
    psi_out, _, _ = O.evaluate(nq, gates, prob["marked"], psi)
    gpsi, gang = run_backward([prob], desc, 0, psi_out, 0.5)
    wpsi, wang = O.adjoint_grad(nq, gates, prob["marked"], psi, 0.5)
    np.testing.assert_allclose(gpsi, wpsi, rtol=0, atol=1e-12)
    np.testing.assert_allclose(gang, wang, rtol=0, atol=1e-12)


@pytest.mark.parametrize("bad,msg", [
    ({"nq": 4, "gates": [("CNOT", 2, 2)], "marked": []}, "second qubit"),
    ({"nq": 4, "gates": [("SWAP", 1, 5)], "marked": []}, "second qubit"),
    ({"nq": 4, "gates": [("CPHASEK", 1, 2, 0)], "marked": []}, "CPHASEK"),
    ({"nq": 4, "gates": [("D4", 1, 2, np.nan, 0.0, 0.0)], "marked": []}, "non-finite"),
    ({"nq": 4, "gates": [("TWOOP", 1, 2, np.full((4, 4), np.inf))], "marked": []}, "non-finite"),
])
def test_create_rejects_bad_two_qubit_gates(bad, msg):
    with pytest.raises(pk.PaperkernError) as e:
        pk.Plan(bad)
    assert msg in str(e.value)


def test_batched_plan_schedules_each_instance():
    insts = W.batch_instances(3, count=6, nq_min=3, span=6)
    probs = [{"nq": i["nq"], "gates": i["gates"], "marked": i["marked"]} for i in insts]
    plan = pk.Plan(probs)
    desc = plan.describe()
    for k, (p, inst) in enumerate(zip(probs, insts)):
        got, L = run_forward(probs, desc, k, inst["psi"])
        want, Lw, _ = O.evaluate(p["nq"], p["gates"], p["marked"], inst["psi"])
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)
        assert abs(L - Lw) < 1e-13


def test_scale_is_exact_power_of_two_for_even_hadamard_count():
    desc = pk.Plan({"nq": 20, "gates": W.grover_gates(), "marked": [3]}).describe()
    scales = [p["scale"] for p in desc["instances"][0]["forward"]]
    for s in scales:
        m, e = math.frexp(abs(s))
        assert m == 0.5


# --------------------------------------------------------------------------- QFT, controlled phases, SWAP relabelling


@pytest.mark.parametrize("nq,first,n,tiling,reg_bits", [
    (6, 1, 6, None, 4), (9, 1, 6, None, 5), (10, 3, 5, (5, 2, 1), 4), (12, 1, 8, (6, 2, 1), 4),
    (13, 2, 9, (7, 3, 1), 5), (11, 1, 11, (6, 1, 1), 4), (12, 4, 7, (5, 0, 1), 4), (9, 1, 9, (6, 2, 0), 4),
    (14, 1, 10, None, 4), (14, 1, 12, (9, 3, 1), 3), (12, 2, 8, None, 3),
])
def test_qft_schedule_matches_dft(nq, first, n, tiling, reg_bits):
    rng = np.random.default_rng(nq * 31 + first * 7 + n)
    gates = [("H", nq), ("QFT", first, n), ("ORACLE",), ("D2", first, 0.3, 1.1, -0.2)]
    prob = {"nq": nq, "gates": gates, "marked": [int(rng.integers(0, 1 << nq))]}
    _check_forward(prob, _state(rng, nq), tiling, reg_bits=reg_bits)


@pytest.mark.parametrize("nq,n1,tiling", [(8, 5, None), (12, 8, (6, 2, 1)), (11, 7, (5, 1, 1))])
def test_qft_ladder_gate_list_matches_dft(nq, n1, tiling):
    rng = np.random.default_rng(nq + n1)
    ladder = O.qft_gates(n1)  # the explicit H / CPHASEK / SWAP list of App. A
    prob = {"nq": nq, "gates": ladder, "marked": []}
    psi = _state(rng, nq)
    plan = pk.Plan(prob)
    if tiling:
        plan.set_tiling(*tiling)
    got, _ = run_forward([prob], plan.describe(), 0, psi)
    np.testing.assert_allclose(got, O.qft_register(psi, nq, 1, n1), rtol=0, atol=1e-12)


@pytest.mark.parametrize("nq,tiling", [(8, None), (11, (5, 2, 1)), (12, (6, 2, 1)), (10, (4, 0, 0))])
def test_backward_through_phases_and_relabelled_swaps(nq, tiling):
    rng = np.random.default_rng(500 + nq)
    gates = (W.grover_gates((2, 1, 0.9, 0.4, 0.1)) + [("QFT", 2, nq - 2), ("CPHASEK", 1, nq, 3),
             ("SWAP", 3, nq - 1), ("D4", 1, 4, 0.3, -0.8, 1.2), ("CPHASE", nq, 2)])
    prob = {"nq": nq, "gates": gates, "marked": [int(rng.integers(0, 1 << nq)), 3]}
    psi = _state(rng, nq)
    plan = pk.Plan(prob)
    if tiling:
        plan.set_tiling(*tiling)
    desc = plan.describe()
    psi_out, _, _ = O.evaluate(nq, gates, prob["marked"], psi)
    gpsi, gang = run_backward([prob], desc, 0, psi_out, 0.5)
    wpsi, wang = O.adjoint_grad(nq, gates, prob["marked"], psi, 0.5)
    np.testing.assert_allclose(gpsi, wpsi, rtol=0, atol=1e-12)
    np.testing.assert_allclose(gang, wang, rtol=0, atol=1e-12)


def _table_use(desc):
    """Slots (forward and backward passes) using the first / second tile-part
    table, the thread-part table, and the phases left to the kernel's loop."""
    c = {"ut0": 0, "ut1": 0, "tt": 0, "loop": 0}
    for inst in desc["instances"]:
        for p in inst["forward"] + inst["backward"]:
            for u in p["subs"]:
                for k in range(4):
                    if u["phase_cnt"][k]:
                        c["ut0"] += u["phase_ut0"][k] >= 0
                        c["ut1"] += u["phase_ut1"][k] >= 0
                        c["tt"] += u["phase_tt"][k] >= 0
                        c["loop"] += u["phase_cnt"][k] - u["phase_ucnt"][k]
    return c


@pytest.mark.parametrize("seed", [4, 5])
def test_phase_product_tables_match_oracle(seed):
    """Circuits dense in controlled phases at 16 qubits in 2^5 tiles (11 tile-index
    bits): their slots use the second tile-part table, the thread-part table and
    (in the backward passes, where a phase can miss every register bit) the
    kernel's loop; the emulated schedules still equal the oracle both ways."""
    rng = np.random.default_rng(seed)
    nq = 16
    gates = W.phase_circuit(rng, nq, 120)
    prob = {"nq": nq, "gates": gates, "marked": [int(rng.integers(0, 1 << nq))]}
    psi = _state(rng, nq)
    plan, desc = _check_forward(prob, psi, (5, 0, 1))
    use = _table_use(desc)
    assert use["ut0"] > 0 and use["tt"] > 0
    if seed == 4:
        assert use["ut1"] > 0
    else:
        assert use["loop"] > 0
    psi_out, _, _ = O.evaluate(nq, gates, prob["marked"], psi)
    gpsi, _ = run_backward([prob], desc, 0, psi_out, 0.5)
    wpsi, _ = O.adjoint_grad(nq, gates, prob["marked"], psi, 0.5)
    np.testing.assert_allclose(gpsi, wpsi, rtol=0, atol=1e-12)


def test_phase_tables_at_the_per_pass_limit():
    """500 controlled phases at 14 qubits in 2^8 tiles: passes reach the 64 tile-part
    tables a pass may list (one per lane); the slots past the limit keep their
    phases in the kernel's loop, and the emulated schedules still equal the oracle."""
    rng = np.random.default_rng(2)
    nq = 14
    gates = W.phase_circuit(rng, nq, 500)
    prob = {"nq": nq, "gates": gates, "marked": [int(rng.integers(0, 1 << nq))]}
    psi = _state(rng, nq)
    plan, desc = _check_forward(prob, psi, (8, 2, 1))
    passes = desc["instances"][0]["forward"] + desc["instances"][0]["backward"]
    assert max(len(p["urefs"]) for p in passes) == 64
    assert _table_use(desc)["loop"] > 0
    psi_out, _, _ = O.evaluate(nq, gates, prob["marked"], psi)
    gpsi, _ = run_backward([prob], desc, 0, psi_out, 0.5)
    wpsi, _ = O.adjoint_grad(nq, gates, prob["marked"], psi, 0.5)
    np.testing.assert_allclose(gpsi, wpsi, rtol=0, atol=1e-12)


def test_only_the_last_pass_of_a_large_fp64_state_streams():
    """PASS_STREAM (64) marks the last forward pass of an FP64 instance of at least
    1 GiB (n_q >= 26) that stores in the layout it read: never another pass, a
    backward pass, FP32, a smaller state or a relabelling last pass."""
    gates = W.grover_gates((3, 2, 0.4, 0.2, 0.1))
    for nq, prec, want in ((30, "fp64", True), (26, "fp64", True), (25, "fp64", False), (30, "fp32", False)):
        d = pk.Plan({"nq": nq, "gates": gates, "marked": [5]}, prec=prec).describe()["instances"][0]
        flags = [p["flags"] for p in d["forward"]]
        assert [bool(f & 64) for f in flags] == [want and i == len(flags) - 1 for i in range(len(flags))]
        assert bool(flags[-1] & 2)
        assert not any(p["flags"] & 64 for p in d["backward"])
    # a last pass that writes the tile back relabelled (the QFT's SWAPs) does not stream
    d = pk.Plan({"nq": 30, "gates": [("QFT", 1, 20)], "marked": []}).describe()["instances"][0]
    assert d["forward"][-1]["tile_bits"] != d["forward"][-1]["store_bits"]
    assert not any(p["flags"] & 64 for p in d["forward"])


def test_qft_of_register_one_at_thirty_qubits_takes_four_passes():
    for prec in ("fp64", "fp32"):
        desc = pk.Plan({"nq": 30, "gates": [("QFT", 1, 20)], "marked": []}, prec=prec).describe()
        fw = desc["instances"][0]["forward"]
        assert len(fw) == 4
        # every pair swap is a relabelling: no 4x4 matrix, and 20 state bits change place
        assert not any(op["kind"] == "MAT4" for p in fw for st in p["stages"] for op in st["ops"])
        assert sum(sum(a != b for a, b in zip(p["tile_bits"], p["store_bits"])) for p in fw) == 20
        assert sum(op["kind"] == "PHASE" for p in fw for st in p["stages"] for op in st["ops"]) == 190


def test_swap_on_a_carrier_bit_stays_a_matrix():
    # carriers are written in contiguous runs, so a SWAP touching one is applied as a 4x4
    desc = pk.Plan({"nq": 8, "gates": [("SWAP", 8, 2)], "marked": []}).describe()
    p = desc["instances"][0]["forward"][0]
    assert p["tile_bits"] == p["store_bits"]
    assert any(op["kind"] == "MAT4" for st in p["stages"] for op in st["ops"])
    desc = pk.Plan({"nq": 8, "gates": [("SWAP", 1, 2)], "marked": []}).describe()
    p = desc["instances"][0]["forward"][0]
    assert p["tile_bits"] != p["store_bits"]


def test_batched_plan_with_qft_instances():
    rng = np.random.default_rng(8)
    probs = [{"nq": nq, "gates": [("QFT", 1, nq - 2), ("CPHASEK", 1, nq, 2)], "marked": [1]} for nq in (5, 9, 12, 7)]
    plan = pk.Plan(probs)
    desc = plan.describe()
    for k, p in enumerate(probs):
        psi = _state(rng, p["nq"])
        got, L = run_forward(probs, desc, k, psi)
        want, Lw, _ = O.evaluate(p["nq"], p["gates"], p["marked"], psi)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)


@pytest.mark.parametrize("bad,msg", [
    ({"nq": 4, "gates": [("QFT", 3, 3)], "marked": []}, "QFT"),
    ({"nq": 4, "gates": [("QFT", 1, 0)], "marked": []}, "QFT"),
    ({"nq": 4, "gates": [("QFT", 0, 2)], "marked": []}, "QFT"),
])
def test_create_rejects_bad_qft(bad, msg):
    with pytest.raises(pk.PaperkernError) as e:
        pk.Plan(bad)
    assert msg in str(e.value)


def test_relabelling_passes_have_an_exchange():
    """A pass that writes its tile with another map than it read it with must have
    at least two stages: the LDS exchange's barrier makes every thread's loads
    complete before any thread stores in place."""
    for nq, n1, prec in ((24, 14, "fp64"), (30, 20, "fp64"), (30, 20, "fp32"), (12, 8, "fp64"), (16, 12, "fp32")):
        desc = pk.Plan({"nq": nq, "gates": [("QFT", 1, n1)], "marked": [1]}, prec=prec).describe()
        for p in desc["instances"][0]["forward"] + desc["instances"][0]["backward"]:
            if p["tile_bits"] != p["store_bits"]:
                assert len(p["stages"]) >= 2
                assert any(u["exchange"] for u in p["subs"][1:])


# --------------------------------------------------------------------------- argument checks of the plan-less entry points


def _einval(rc, text):
    assert rc == pk.PK_EINVAL
    assert text in pk.lib().pk_last_error(None).decode()


def test_shor_marginal_density_search_entry_points_reject_bad_arguments():
    """Every check runs before any device call, so these need no GPU."""
    lib = pk.lib()
    buf = ctypes.c_void_p(4096)  # an aligned non-NULL address; never dereferenced on these paths
    _einval(lib.pk_shor_state(0, 4, 7, 15, pk.PK_FP64, buf, None), "register sizes")
    _einval(lib.pk_shor_state(20, 11, 7, 15, pk.PK_FP64, buf, None), "register sizes")
    _einval(lib.pk_shor_state(8, 4, 7, 17, pk.PK_FP64, buf, None), "M must")
    _einval(lib.pk_shor_state(8, 4, 15, 15, pk.PK_FP64, buf, None), "xguess")
    _einval(lib.pk_shor_state(8, 4, 7, 15, 7, buf, None), "prec")
    _einval(lib.pk_shor_state(8, 4, 7, 15, pk.PK_FP64, ctypes.c_void_p(4097), None), "aligned")
    _einval(lib.pk_marginal(12, 13, pk.PK_FP64, buf, buf, None), "n_low")
    _einval(lib.pk_marginal(31, 3, pk.PK_FP64, buf, buf, None), "nq")
    _einval(lib.pk_marginal(12, 3, pk.PK_FP64, None, buf, None), "NULL")
    _einval(lib.pk_marginal_bitrev(12, 13, pk.PK_FP64, buf, buf, None), "n_low")
    _einval(lib.pk_marginal_bitrev(12, 3, 7, buf, buf, None), "prec")
    _einval(lib.pk_marginal_bitrev(12, 3, pk.PK_FP64, buf, None, None), "NULL")
    _einval(lib.pk_density_matrix(17, 4, buf, buf, buf, None), "nq")
    _einval(lib.pk_density_matrix(8, 0, buf, buf, buf, None), "universe")
    _einval(lib.pk_density_spectrum(16, buf, buf, buf, None), "nq")
    one = (ctypes.c_int64 * 2)(3, 3)
    _einval(lib.pk_search_diffusion(6, pk.PK_FP64, one, 2, 5, buf, buf, buf, buf, None), "duplicate")
    _einval(lib.pk_search_diffusion(6, pk.PK_FP64, one, 1, 0, buf, buf, buf, buf, None), "iterations")
    big = (ctypes.c_int64 * 1)(64)
    _einval(lib.pk_search_diffusion(6, pk.PK_FP64, big, 1, 5, buf, buf, buf, buf, None), "out of range")
    _einval(lib.pk_search_diffusion(6, pk.PK_FP64, one, 65, 5, buf, buf, buf, buf, None), "0..64")


def test_pass_walk_settings():
    """pk_set_pass_walk sets each forward pass's tile walk (0 strided, c runs of c
    tiles, -1 blocks) and nothing else; a tiling change resets it; wrong lengths,
    values and batched plans are refused."""
    prob = {"nq": 20, "gates": W.grover_gates((3, 2, 0.4, 0.2, 0.1)), "marked": [5]}
    plan = pk.Plan(prob)
    n = plan.passes()
    walks = [-1, 0, 2, 64, 4][:n]
    plan.set_pass_walk(walks)
    d = plan.describe()["instances"][0]
    assert [p["walk"] for p in d["forward"]] == walks
    assert all(p["walk"] == 0 for p in d["backward"])
    for bad in ([0] * (n + 1), [1] + [0] * (n - 1), [-2] + [0] * (n - 1), [1 << 17] + [0] * (n - 1)):
        with pytest.raises(pk.PaperkernError):
            plan.set_pass_walk(bad)
    assert [p["walk"] for p in plan.describe()["instances"][0]["forward"]] == walks
    plan.set_tiling(12, 4, 1)
    assert all(p["walk"] == 0 for p in plan.describe()["instances"][0]["forward"])
    plan.set_pass_walk(walks[:1] * plan.passes())
    plan.set_pass_walk([])
    assert all(p["walk"] == 0 for p in plan.describe()["instances"][0]["forward"])
    nb = len(plan.describe()["instances"][0]["backward"])
    plan.set_pass_walk([0] * plan.passes() + [64] * nb)
    d = plan.describe()["instances"][0]
    assert all(p["walk"] == 0 for p in d["forward"]) and all(p["walk"] == 64 for p in d["backward"])
    with pytest.raises(pk.PaperkernError):
        plan.set_pass_walk([0] * (plan.passes() + nb + 1))
    batch = pk.Plan([prob, prob])
    with pytest.raises(pk.PaperkernError):
        batch.set_pass_walk([0])


def test_repeat_launch_counts():
    """pk_evaluate_repeat fuses 8 applications into one schedule when the plan has
    no angle parameters: at n_q = 20 a Grover iteration takes 3 passes, 8 take 17,
    so n_t = 804 iterations take 100 x 17 + 4 x 3 launches; a noisy plan (D2
    angles) and fewer than 8 applications are not fused."""
    g20 = pk.Plan({"nq": 20, "gates": W.grover_gates(), "marked": [5]})
    assert g20.passes() == 3
    assert pk.repeat_launches(g20, 804) == 100 * 17 + 4 * 3
    assert pk.repeat_launches(g20, 7) == 21
    assert pk.repeat_launches(g20, 8) == 17
    noisy = pk.Plan({"nq": 20, "gates": W.grover_gates((3, 2, 0.1, 0.2, 0.3)), "marked": [5]})
    assert pk.repeat_launches(noisy, 804) == 804 * noisy.passes()
    with pytest.raises(pk.PaperkernError):
        pk.repeat_launches(g20, 0)
    batch = pk.Plan([{"nq": 10, "gates": W.grover_gates(), "marked": [1]}] * 2)
    with pytest.raises(pk.PaperkernError):
        pk.repeat_launches(batch, 10)


def test_evaluate_repeat_rejects_bad_reps_before_the_device():
    plan = pk.Plan({"nq": 6, "gates": W.grover_gates(), "marked": [1]})
    buf = ctypes.c_void_p(4096)
    rc = pk.lib().pk_evaluate_repeat(plan.handle, 0, buf, buf, buf, None, None, buf, None)
    assert rc == pk.PK_EINVAL and "reps" in pk.lib().pk_last_error(plan.handle).decode()
    batch = pk.Plan([{"nq": 4, "gates": [], "marked": []}] * 2)
    rc = pk.lib().pk_evaluate_repeat(batch.handle, 3, buf, buf, buf, None, None, buf, None)
    assert rc == pk.PK_EINVAL and "single-instance" in pk.lib().pk_last_error(batch.handle).decode()


def test_qft_noswap_lowers_to_the_ladder_without_swaps():
    """QFT_NOSWAP (a labelled variant) is the App. A ladder minus its pair swaps:
    at n_q = 30 with a 20-qubit register it needs 3 passes where the full QFT needs
    4, and it keeps the full QFT's validation."""
    full = pk.Plan({"nq": 30, "gates": [("QFT", 1, 20)], "marked": []})
    nosw = pk.Plan({"nq": 30, "gates": [("QFT_NOSWAP", 1, 20)], "marked": []})
    assert full.passes() == 4 and nosw.passes() == 3
    gates = lambda d: sum(len(p["stages"]) for p in d["instances"][0]["forward"])
    assert gates(nosw.describe()) <= gates(full.describe())
    for bad in ([("QFT_NOSWAP", 0, 3)], [("QFT_NOSWAP", 5, 7)], [("QFT_NOSWAP", 1, 0)]):
        with pytest.raises(pk.PaperkernError):
            pk.Plan({"nq": 10, "gates": bad, "marked": []})


@pytest.mark.parametrize("nq,n1,tiling", [(8, 5, None), (12, 8, (6, 2, 1)), (11, 7, (5, 1, 1)), (10, 10, (4, 0, 0))])
def test_qft_noswap_schedule_matches_the_permuted_dft(nq, n1, tiling):
    """The CPU emulation of a QFT_NOSWAP schedule equals the oracle's DFT of the
    register with the register's qubit order reversed."""
    rng = np.random.default_rng(7 * nq + n1)
    prob = {"nq": nq, "gates": [("QFT_NOSWAP", 1, n1)], "marked": []}
    psi = _state(rng, nq)
    plan = pk.Plan(prob)
    if tiling:
        plan.set_tiling(*tiling)
    got, _ = run_forward([prob], plan.describe(), 0, psi)
    want = O.qft_register(psi, nq, 1, n1)
    idx = np.arange(1 << nq)
    low = nq - n1
    reg = idx >> low
    rev = np.zeros_like(reg)
    for b in range(n1):
        rev |= ((reg >> b) & 1) << (n1 - 1 - b)
    np.testing.assert_allclose(got, want[(rev << low) | (idx & ((1 << low) - 1))], rtol=0, atol=1e-12)


def _thread_label(sub, tid):
    """The label base a thread holds in one sub-stage's layout (the kernel's
    make_layout, restated): ascending over the free local bits, or the lane map."""
    if sub["nlanes"] == 0:
        t = tid
        for p in sorted(b for b in sub["rb"] if b >= 0):
            t = ((t >> p) << (p + 1)) | (t & ((1 << p) - 1))
        return t
    w = sub["nlanes"]
    t = 0
    for i, p in enumerate(sub["lanes"]):
        t |= ((tid >> i) & 1) << p
    x = tid >> w
    rest = [b for b in range(32) if sub["lanes_rest"] >> b & 1]
    for p in rest:
        t |= (x & 1) << p
        x >>= 1
    return t


def _bank_group_conflicts(sub, k, w):
    """Lane groups (2^w consecutive threads: 256 bytes of amplitudes) of one layout
    whose LDS slots, under the XOR swizzle of 2^w-slot groups, repeat a bank."""
    nrb = sum(1 for b in sub["rb"] if b >= 0)
    m = (1 << w) - 1
    bad = 0
    for g in range(0, 1 << (k - nrb), 1 << w):
        slots = set()
        for tid in range(g, g + (1 << w)):
            j = _thread_label(sub, tid)
            slots.add((j ^ (j >> w) ^ (j >> 2 * w) ^ (j >> 3 * w)) & m)
        bad += len(slots) < (1 << w)
    return bad


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_lane_maps_spread_lds_banks(prec):
    """Stage layouts that move through LDS only get a thread map whose lane groups
    hit distinct banks; the first and last layout of each pass (the HBM load and
    store) keep the ascending map; every map is a bijection onto the labels with
    zero register bits; pk_set_lane_maps(0) turns the maps off."""
    w = 4 if prec == "fp64" else 5
    rng = np.random.default_rng(11)
    probs = [
        {"nq": 30, "gates": W.grover_gates((16, 3, 0.9, 3.0, 0.0)), "marked": [5]},
        {"nq": 30, "gates": [("QFT", 1, 20)], "marked": []},
        {"nq": 24, "gates": W.phase_circuit(rng, 24, 40), "marked": [3]},
    ]
    seen = 0
    for prob in probs:
        plan = pk.Plan(prob, prec=prec)
        before = None
        for on in (0, 1):
            plan.set_lane_maps(on)
            inst = plan.describe()["instances"][0]
            conflicts = 0
            for p in inst["forward"] + inst["backward"]:
                k = p["k"]
                groups = []
                for s in p["subs"]:
                    if s["exchange"] or not groups:
                        groups.append([])
                    groups[-1].append(s)
                for gi, grp in enumerate(groups):
                    assert all(s["nlanes"] == grp[0]["nlanes"] and s["lanes"] == grp[0]["lanes"] for s in grp)
                    sub = grp[0]
                    if on == 0 or gi == 0 or gi == len(groups) - 1:
                        assert sub["nlanes"] == 0
                    nrb = sum(1 for b in sub["rb"] if b >= 0)
                    if k - nrb > 12:
                        continue
                    labels = sorted(_thread_label(sub, t) for t in range(1 << (k - nrb)))
                    regmask = sum(1 << b for b in sub["rb"] if b >= 0)
                    assert labels == [j for j in range(1 << k) if not j & regmask]
                    if sub["nlanes"]:
                        seen += 1
                        assert [q % w for q in sub["lanes"]] == list(range(w))
                    if 0 < gi < len(groups) - 1 and k - nrb >= w:
                        conflicts += _bank_group_conflicts(sub, k, w)
            if on == 0:
                before = conflicts
            else:
                assert conflicts <= before
                if prec == "fp64":
                    assert conflicts == 0
    assert seen > 0


def test_pass_overlap_settings():
    """pk_set_pass_overlap sets each forward pass's tile-loop pipelining (0 or 1)
    and nothing else; walks survive it, a tiling change resets it; wrong lengths,
    values and batched plans are refused."""
    prob = {"nq": 24, "gates": W.grover_gates((3, 2, 0.4, 0.2, 0.1)), "marked": [5]}
    plan = pk.Plan(prob)
    n = plan.passes()
    plan.set_pass_walk([2] * n)
    before = plan.describe()["instances"][0]
    on = [p % 2 for p in range(n)]
    plan.set_pass_overlap(on)
    d = plan.describe()["instances"][0]
    assert [p["overlap"] for p in d["forward"]] == on
    assert [p["walk"] for p in d["forward"]] == [2] * n
    strip = lambda inst: [{k: v for k, v in p.items() if k != "overlap"} for p in inst["forward"] + inst["backward"]]
    assert strip(d) == strip(before)
    for bad in ([0] * (n + 1), [2] + [0] * (n - 1), [-1] + [0] * (n - 1)):
        with pytest.raises(pk.PaperkernError):
            plan.set_pass_overlap(bad)
    assert [p["overlap"] for p in plan.describe()["instances"][0]["forward"]] == on
    plan.set_pass_overlap([])
    assert all(p["overlap"] == 0 for p in plan.describe()["instances"][0]["forward"])
    plan.set_pass_overlap([1] * n)
    plan.set_tiling(12, 4, 1)
    assert all(p["overlap"] == 0 for p in plan.describe()["instances"][0]["forward"])
    batch = pk.Plan([prob, prob])
    with pytest.raises(pk.PaperkernError):
        batch.set_pass_overlap([0])
