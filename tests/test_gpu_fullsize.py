"""GPU parity at the full workload sizes (n_q = 30), in the launch configuration that
bench.py times (default tiling and launch).

The gate-by-gate oracle cannot hold a 2^30-amplitude state in reasonable time, so
the expected values come from oracle.grover_sampled: exact amplitudes of one Grover
iteration at sampled labels through the diffusion identity (pinned against the
gate-by-gate oracle on the CPU).  Compared per config:

  * amplitudes at 2^16 seeded random labels plus the marked label, its partner on
    the noisy qubit, 0 and N - 1: the root-mean-square error scaled by sqrt(N)
    estimates the normwise error ||psi_gpu - psi_ref|| / ||psi_ref||;
  * L against the closed form; the norm against ||psi_in||^2 (unitary circuit);
  * the gradient (c4) against central differences on the 64-input subset.

Each test prints its config before touching the GPU and needs ~50 GiB of host
memory at most (the FP64 input state plus the generator's blocks).
"""

import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_0902_0699_amd import workload as W

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]

NQ = W.NQ_LARGE
TOL64 = 1e-12
TOL32 = 1e-5
SAMPLES = 1 << 16


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _labels(inst, seed):
    nq = inst["nq"]
    rng = np.random.default_rng(seed + 2000)
    x = inst["marked"][0]
    extra = [x, 0, (1 << nq) - 1]
    if inst["noise"] is not None:
        extra.append(x ^ (1 << (nq - inst["noise"][0])))
    return np.unique(np.concatenate([rng.integers(0, 1 << nq, SAMPLES), np.array(extra, dtype=np.int64)]))


def _check_sampled(prec, seed):
    from paper_0902_0699_amd import paperkern as pk

    _say("full size: n_q=%d %s seed %d" % (NQ, prec, seed))
    inst = W.single_instance(seed, NQ)
    psi = inst["psi"]
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    if prec == "fp32":
        psi = psi.astype(np.complex64).astype(np.complex128)  # the input the FP32 path sees
    idx = _labels(inst, seed)
    want, L_ref = O.grover_sampled(NQ, inst["gates"], inst["marked"], psi, idx)
    norm_in = float(np.vdot(psi, psi).real)

    plan = pk.Plan({"nq": NQ, "gates": inst["gates"], "marked": inst["marked"]}, prec=prec)
    x = torch.from_numpy(psi).to(dt).to("cuda")
    del psi, inst["psi"]
    y, L, norm = pk.evaluate(plan, x)
    got = y[torch.from_numpy(idx).to("cuda")].cpu().numpy().astype(np.complex128)
    L, norm = float(L.item()), float(norm.item())
    del x, y
    torch.cuda.empty_cache()

    err = math.sqrt(np.mean(np.abs(got - want) ** 2) * (1 << NQ) / norm_in)
    tol = TOL64 if prec == "fp64" else TOL32
    _say("  passes %d  est. normwise err %.3e  |dL| %.3e (L %.6e)  |dnorm| %.3e"
         % (plan.passes(), err, abs(L - L_ref), L_ref, abs(norm - norm_in)))
    assert err <= tol
    assert abs(L - L_ref) <= tol * max(1.0, L_ref) * norm_in
    assert abs(norm - norm_in) <= tol * norm_in


@pytest.mark.timeout(900)
def test_c1_fp64_full_size_sampled():
    _check_sampled("fp64", W.SEEDS["large_fp64"])


@pytest.mark.timeout(900)
def test_c2_fp32_full_size_sampled():
    _check_sampled("fp32", W.SEEDS["large_fp32"])


@pytest.mark.timeout(900)
def test_c4_gradient_full_size_against_finite_differences():
    from paper_0902_0699_amd import paperkern as pk

    seed = W.SEEDS["gradient"]
    _say("full size gradient: n_q=%d fp64 seed %d" % (NQ, seed))
    inst = W.single_instance(seed, NQ)
    comps = W.fd_subset(seed, inst)
    plan = pk.Plan({"nq": NQ, "gates": inst["gates"], "marked": inst["marked"]})
    x = torch.from_numpy(inst["psi"]).to("cuda")
    del inst["psi"]
    ang = torch.tensor(list(inst["noise"][2:5]), dtype=torch.float64, device="cuda")
    out, _, _ = pk.evaluate(plan, x, angles=ang, want_norm=False)
    dL = torch.ones(1, dtype=torch.float64, device="cuda")
    gpsi, gang = pk.backward(plan, out, dL, angles=ang)
    del out
    h = 1e-6

    def L_of(aa):
        return pk.evaluate(plan, x, angles=aa, want_norm=False)[1].item()

    fd, ad = [], []
    for kind, where in comps:
        if kind == "angle":
            ap, am = ang.clone(), ang.clone()
            ap[where] += h
            am[where] -= h
            fd.append((L_of(ap) - L_of(am)) / (2 * h))
            ad.append(gang[where].item())
        else:
            i, part = where
            step = h if part == 0 else 1j * h
            orig = x[i].clone()
            x[i] = orig + step
            lp = L_of(ang)
            x[i] = orig - step
            lm = L_of(ang)
            x[i] = orig
            fd.append((lp - lm) / (2 * h))
            g = gpsi[i].item()
            ad.append(g.real if part == 0 else g.imag)
    fd, ad = np.array(fd), np.array(ad)
    err = float(np.max(np.abs(fd - ad)) / np.max(np.abs(ad)))
    _say("  64 inputs: normwise FD vs adjoint %.3e; angle grads %s" % (err, gang.cpu().numpy()))
    assert err <= 1e-6


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec,tile", [("fp64", None), ("fp64", 12), ("fp32", None), ("fp32", 12)])
def test_shor_path_full_size(prec, tile):
    """Shor's data path at n_q = 30 (M = 899: n1 = 20, n2 = 10) at the default tile
    and at the 2^12 tile the autotuner picks in bench.py: load (Eq. Shor2), QFT of
    register one (App. A), marginal.  Every p(n) against Eq. probshor; amplitudes at
    sampled labels (half of them on the support of the state) against the direct
    sum of Eq. QFT1."""
    from paper_0902_0699_amd import paperkern as pk

    M = W.SHOR_M
    x = W.shor_xguess(W.SEEDS["shor"])
    n1, n2 = pk.shor_register_sizes(M)
    nq = n1 + n2
    _say("full size Shor path: M=%d x=%d n1=%d n2=%d %s tile %s" % (M, x, n1, n2, prec, tile))
    psi = pk.shor_state(n1, n2, x, M, prec=prec)
    plan = pk.Plan({"nq": nq, "gates": [("QFT", 1, n1)], "marked": []}, prec=prec)
    if tile is not None:
        plan.set_tiling(tile, 4, 1)
    pk.evaluate(plan, psi, out=psi, want_norm=False)
    p = pk.marginal(psi, nq, n2).cpu().numpy()
    rng = np.random.default_rng(2024)
    fvals = np.array([pow(x, j, M) for j in range(200)])
    n = rng.integers(0, 1 << n1, 4096)
    on = (n[:2048] << n2) + fvals[rng.integers(0, 200, 2048)]
    labels = np.unique(np.concatenate([on, rng.integers(0, 1 << nq, 2048)]))
    got = psi[torch.from_numpy(labels).to("cuda")].cpu().numpy().astype(np.complex128)
    del psi
    torch.cuda.empty_cache()
    want_p = O.probshor_marginal(n1, x, M)
    want_a = O.shor_qft_amplitudes(n1, n2, x, M, labels)
    tol = TOL64 if prec == "fp64" else TOL32
    ep = float(np.max(np.abs(p - want_p)) / np.max(want_p))
    ea = float(np.max(np.abs(got - want_a)) / np.max(np.abs(want_a)))
    _say("  passes %d  max |dp|/max p %.3e  max |dC|/max |C| %.3e  sum p - 1 = %.3e"
         % (plan.passes(), ep, ea, p.sum() - 1.0))
    assert ep <= tol and ea <= tol and abs(p.sum() - 1.0) <= tol


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_shor_noswap_variant_full_size(prec):
    """The labelled no-swap variant at n_q = 30 at the 2^12 tile: QFT_NOSWAP on
    register one and the bit-reversed marginal.  Every p(n) against Eq. probshor;
    sampled amplitudes against the direct sum of Eq. QFT1 at the bit-reversed
    register value."""
    from paper_0902_0699_amd import paperkern as pk

    M = W.SHOR_M
    x = W.shor_xguess(W.SEEDS["shor"])
    n1, n2 = pk.shor_register_sizes(M)
    nq = n1 + n2
    _say("full size Shor path, no-swap variant: M=%d x=%d n1=%d n2=%d %s" % (M, x, n1, n2, prec))
    psi = pk.shor_state(n1, n2, x, M, prec=prec)
    plan = pk.Plan({"nq": nq, "gates": [("QFT_NOSWAP", 1, n1)], "marked": []}, prec=prec)
    plan.set_tiling(12, 4, 1)
    pk.evaluate(plan, psi, out=psi, want_norm=False)
    p = pk.marginal(psi, nq, n2, bitrev=True).cpu().numpy()
    rng = np.random.default_rng(2025)
    labels = np.unique(rng.integers(0, 1 << nq, 4096))
    got = psi[torch.from_numpy(labels).to("cuda")].cpu().numpy().astype(np.complex128)
    del psi
    torch.cuda.empty_cache()
    r = labels >> n2
    rr = np.zeros_like(r)
    for b in range(n1):
        rr |= ((r >> b) & 1) << (n1 - 1 - b)
    want_a = O.shor_qft_amplitudes(n1, n2, x, M, (rr << n2) | (labels & ((1 << n2) - 1)))
    want_p = O.probshor_marginal(n1, x, M)
    tol = TOL64 if prec == "fp64" else TOL32
    ep = float(np.max(np.abs(p - want_p)) / np.max(want_p))
    ea = float(np.max(np.abs(got - want_a)) / np.max(np.abs(want_a)))
    _say("  passes %d  max |dp|/max p %.3e  max |dC|/max |C| %.3e" % (plan.passes(), ep, ea))
    assert plan.passes() == 3 and ep <= tol and ea <= tol


@pytest.mark.timeout(900)
def test_density_matrix_full_size():
    """The ensemble density matrix (Sec. 6.1) in the configuration bench.py times:
    4096 noisy Grover universes at n_q = 12 from the library's batched launch,
    equal weights.  Every element of rho against the oracle's sum over the same
    states, Tr rho = 1, Tr rho^2 against the Gram route, and the spectrum, entropy
    and purity against LAPACK."""
    from paper_0902_0699_amd import paperkern as pk

    nq, A = W.DENSITY_NQ, W.DENSITY_UNIVERSES
    N = 1 << nq
    _say("full size density matrix: %d universes, n_q=%d" % (A, nq))
    gates, x = W.density_universes(W.SEEDS["density"], nq, A)
    plan = pk.Plan([{"nq": nq, "gates": g, "marked": [x]} for g in gates])
    s = torch.full((A * N,), 2.0 ** (-nq / 2), dtype=torch.complex128, device="cuda")
    C, _, _ = pk.evaluate_batched(plan, s)
    P = np.full(A, 1.0 / A)
    rho = pk.density_matrix(C, torch.from_numpy(P).to("cuda"))
    got = rho.cpu().numpy()
    lam, S, pur = pk.density_spectrum(rho)
    lam = lam.cpu().numpy()
    Ch = C.cpu().numpy().reshape(A, N)
    del C, s, rho
    torch.cuda.empty_cache()
    want = O.density_matrix(Ch, P)
    err = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
    wl = O.spectrum(want)
    _say("  max |drho| / max |rho| %.3e  Tr rho - 1 %.3e  max |dlambda| %.3e  S %.6f bits (LAPACK %.6f)"
         % (err, np.trace(got).real - 1.0, np.max(np.abs(lam - wl)), float(S), O.entropy_bits(wl)))
    assert err <= 1e-12
    np.testing.assert_array_equal(got, got.conj().T)
    assert abs(np.trace(got).real - 1.0) <= 1e-12
    assert abs(O.purity(got) - O.purity_gram(Ch, P)) <= 1e-12
    assert np.max(np.abs(lam - wl)) <= 1e-12
    assert abs(float(S) - O.entropy_bits(wl)) <= 1e-9 and abs(float(pur) - O.purity(want)) <= 1e-12


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec,tiling", [("fp64", None), ("fp64", (12, 5)), ("fp32", None), ("fp32", (12, 4))])
def test_c3_batched_full_size(prec, tiling):
    """c3 as bench.py times it: 4096 instances with n_q in [10, 20), seed 3, one
    persistent launch, at the default tile and at the tile the autotuner picked in
    bench.py.  L of every instance against the closed form (oracle.grover_sampled at
    the marked label); the whole state of 24 instances (the noise-free one, the
    largest, the smallest and a seeded sample) against the gate-by-gate oracle."""
    from paper_0902_0699_amd import paperkern as pk

    insts = W.batch_instances(W.SEEDS["batched"])
    _say("full size c3: %d instances %s tiling %s" % (len(insts), prec, tiling))
    plan = pk.Plan([{"nq": b["nq"], "gates": b["gates"], "marked": b["marked"]} for b in insts], prec=prec)
    if tiling:
        plan.set_tiling(tiling[0], tiling[1], 1, 1, -1)
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    psi_all = np.concatenate([b["psi"] for b in insts])
    if prec == "fp32":
        psi_all = psi_all.astype(np.complex64).astype(np.complex128)
    out, L, norm = pk.evaluate_batched(plan, torch.from_numpy(psi_all).to(dt).to("cuda"))
    L = L.cpu().numpy()
    norm = norm.cpu().numpy()
    offs = plan.offsets()
    tol = TOL64 if prec == "fp64" else TOL32
    worst_L = 0.0
    for k, b in enumerate(insts):
        psi = psi_all[offs[k]:offs[k + 1]]
        _, Lw = O.grover_sampled(b["nq"], b["gates"], b["marked"], psi, [b["marked"][0]])
        worst_L = max(worst_L, abs(L[k] - Lw))
        assert abs(norm[k] - 1.0) <= tol
    rng = np.random.default_rng(33)
    sizes = np.array([b["nq"] for b in insts])
    pick = sorted({0, int(np.argmax(sizes)), int(np.argmin(sizes))} | {int(v) for v in rng.integers(0, len(insts), 21)})
    worst = 0.0
    for k in pick:
        b = insts[k]
        psi = psi_all[offs[k]:offs[k + 1]]
        want, _, _ = O.evaluate(b["nq"], b["gates"], b["marked"], psi)
        got = out[offs[k]:offs[k + 1]].cpu().numpy().astype(np.complex128)
        worst = max(worst, float(np.linalg.norm(got - want) / np.linalg.norm(want)))
    _say("  max |dL| over %d instances %.3e; max normwise err over %d instances %.3e"
         % (len(insts), worst_L, len(pick), worst))
    assert worst_L <= tol and worst <= tol


@pytest.mark.timeout(900)
def test_fp32_at_thirty_one_qubits_sampled():
    """The largest FP32 state (n_q = 31, 16 GiB; byte offsets beyond 32 bits) against
    oracle.grover_sampled, as c2."""
    from paper_0902_0699_amd import paperkern as pk

    nq = 31
    _say("full size: n_q=%d fp32 seed %d" % (nq, W.SEEDS["large_fp32"]))
    inst = W.single_instance(W.SEEDS["large_fp32"], nq)
    psi = inst["psi"].astype(np.complex64)
    del inst["psi"]
    x = torch.from_numpy(psi).to("cuda")
    psi = psi.astype(np.complex128)
    idx = _labels(dict(inst, nq=nq), W.SEEDS["large_fp32"])
    want, L_ref = O.grover_sampled(nq, inst["gates"], inst["marked"], psi, idx)
    norm_in = float(np.vdot(psi, psi).real)
    del psi
    plan = pk.Plan({"nq": nq, "gates": inst["gates"], "marked": inst["marked"]}, prec="fp32")
    y, L, norm = pk.evaluate(plan, x)
    got = y[torch.from_numpy(idx).to("cuda")].cpu().numpy().astype(np.complex128)
    L, norm = float(L.item()), float(norm.item())
    del x, y
    torch.cuda.empty_cache()
    err = math.sqrt(np.mean(np.abs(got - want) ** 2) * (1 << nq) / norm_in)
    _say("  passes %d  est. normwise err %.3e  |dL| %.3e  |dnorm| %.3e" % (plan.passes(), err, abs(L - L_ref),
                                                                          abs(norm - norm_in)))
    assert err <= TOL32 and abs(L - L_ref) <= TOL32 * max(1.0, L_ref) * norm_in
    assert abs(norm - norm_in) <= TOL32 * norm_in
