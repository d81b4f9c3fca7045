"""pk_evaluate_static (the entry point that allocates nothing) against pk_evaluate.

Two calls in a row through the C-ABI, the second on a smaller instance, each
compared with pk_evaluate on the same plan and input: the same kernels on the
same schedule, so psi_out, L and the norm must agree bit for bit.  Also the
documented refusals: a plan whose tables are not on the device yet, and a plan
whose workspace exceeds the static buffer.
"""

import sys

import numpy as np
import pytest

from paper_0902_0699_amd import workload as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _pair(pk, nq, seed, prec):
    inst = W.single_instance(seed, nq)
    plan = pk.Plan({"nq": nq, "gates": inst["gates"], "marked": inst["marked"]}, prec=prec)
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    x = torch.from_numpy(inst["psi"]).to(dt).to("cuda")
    return plan, x


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_static_entry_point_matches_evaluate_on_two_calls(prec):
    from paper_0902_0699_amd import paperkern as pk

    for nq, seed in ((22, 11), (13, 12)):  # the second call is the smaller one
        _say("static evaluate: n_q=%d %s" % (nq, prec))
        plan, x = _pair(pk, nq, seed, prec)
        ref, L_ref, n_ref = pk.evaluate(plan, x)  # also uploads the plan's tables
        y = torch.full_like(x, float("nan"))
        L = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        norm = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        pk.evaluate_static(plan, x, y, L, norm)
        torch.cuda.synchronize()
        _say("  max |dpsi| %.3e  dL %.3e  dnorm %.3e"
             % ((y - ref).abs().max().item(), L.item() - L_ref.item(), norm.item() - n_ref.item()))
        assert torch.equal(y, ref)
        assert L.item() == L_ref.item() and norm.item() == n_ref.item()


def test_static_entry_point_in_place_and_refusals():
    from paper_0902_0699_amd import paperkern as pk

    _say("static evaluate: refusals, in place")
    plan, x = _pair(pk, 16, 13, "fp64")
    L = torch.empty(1, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    with pytest.raises(pk.PaperkernError) as e:  # tables not uploaded yet
        pk.evaluate_static(plan, x, y, L)
    assert e.value.code == pk.PK_EINVAL and "not on this device" in str(e.value)
    ref, L_ref, _ = pk.evaluate(plan, x)
    z = x.clone()
    pk.evaluate_static(plan, z, z, L)  # in place, no norm
    torch.cuda.synchronize()
    assert torch.equal(z, ref) and L.item() == L_ref.item()
    # 2^4-amplitude tiles at n_q = 24: 2^20 norm partials, beyond the 8 MiB buffer
    big, xb = _pair(pk, 24, 14, "fp64")
    big.set_tiling(4, 2, 1)
    assert big.workspace_bytes() > 8 << 20
    with pytest.raises(pk.PaperkernError) as e:
        pk.evaluate_static(big, xb, torch.empty_like(xb), L)
    assert e.value.code == pk.PK_EINVAL and "static buffer" in str(e.value)
