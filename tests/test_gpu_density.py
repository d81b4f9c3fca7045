"""GPU parity of the ensemble density matrix (Sec. 6.1) through the C-ABI.

  * pk_density_matrix against the oracle's sum, element by element, at ragged
    sizes (fewer amplitudes than one 64 x 64 block, universe counts that are not
    multiples of the 16-universe stage): max |drho| <= 1e-12 max |rho| (FP64 sums
    of depth A on the matrix cores, in another order than the oracle's);
  * exact Hermitian symmetry and real diagonal (by construction);
  * universes from the library's own batched Grover evaluation (noisy
    multiverses, Sec. 6.2 / 6.3): Tr rho = 1 and Tr rho^2 against the Gram route;
  * pk_density_spectrum: eigenvalues against LAPACK (1e-12), entropy and purity,
    the pure state (S = 0), orthonormal universes (eigenvalues = weights) and the
    basis ensemble (S = n_q bits).
Each test prints its case before touching the GPU.
"""

import sys

import numpy as np
import pytest

import oracle as O
from paper_0902_0699_amd import workload as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _pk():
    from paper_0902_0699_amd import paperkern as pk
    return pk


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _states(rng, A, nq):
    C = rng.standard_normal((A, 1 << nq)) + 1j * rng.standard_normal((A, 1 << nq))
    return C / np.linalg.norm(C, axis=1, keepdims=True)


def _rho(C, P):
    pk = _pk()
    rho = pk.density_matrix(torch.from_numpy(np.ascontiguousarray(C)).to("cuda"),
                            torch.from_numpy(np.ascontiguousarray(P)).to("cuda"))
    torch.cuda.synchronize()
    return rho.cpu().numpy()


@pytest.mark.parametrize("nq,A", [(1, 1), (3, 3), (5, 16), (6, 17), (7, 50), (9, 33), (10, 16), (8, 1)])
def test_density_matrix_against_oracle(nq, A):
    rng = np.random.default_rng(nq * 100 + A)
    C = _states(rng, A, nq)
    P = rng.uniform(0.0, 1.0, A)
    P /= P.sum()
    _say("density n_q=%d A=%d" % (nq, A))
    got = _rho(C, P)
    want = O.density_matrix(C, P)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    np.testing.assert_array_equal(got, got.conj().T)
    assert np.all(np.diag(got).imag == 0.0)
    assert abs(np.trace(got).real - 1.0) < 1e-12


def test_density_of_grover_multiverses():
    """Universes from the library's batched evaluation: one noisy Grover iteration
    each from HALL|0>, universe 0 noise-free, equal weights."""
    pk = _pk()
    nq, A = 9, 40
    rng = np.random.default_rng(17)
    s = np.full(1 << nq, 2.0 ** (-nq / 2), dtype=np.complex128)
    probs = []
    for a in range(A):
        noise = None if a == 0 else (int(rng.integers(1, nq + 1)), int(rng.integers(0, 5)),
                                     float(rng.uniform(0, 2 * np.pi)), float(rng.uniform(0, np.pi)), 0.0)
        probs.append({"nq": nq, "gates": W.grover_gates(noise), "marked": [77]})
    plan = pk.Plan(probs)
    _say("density of %d Grover universes, n_q=%d" % (A, nq))
    out, _, _ = pk.evaluate_batched(plan, torch.from_numpy(np.tile(s, A)).to("cuda"))
    P = torch.full((A,), 1.0 / A, dtype=torch.float64, device="cuda")
    rho = pk.density_matrix(out, P)
    torch.cuda.synchronize()
    C = out.cpu().numpy().reshape(A, -1)
    got = rho.cpu().numpy()
    want = O.density_matrix(C, np.full(A, 1.0 / A))
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    assert abs(np.trace(got).real - 1.0) < 1e-12
    pur = O.purity(got)
    assert abs(pur - O.purity_gram(C, np.full(A, 1.0 / A))) < 1e-12 and pur < 1.0


@pytest.mark.parametrize("nq,A", [(4, 3), (7, 20), (9, 64)])
def test_spectrum_entropy_purity(nq, A):
    pk = _pk()
    rng = np.random.default_rng(nq + A)
    C = _states(rng, A, nq)
    P = rng.uniform(0.0, 1.0, A)
    P /= P.sum()
    _say("spectrum n_q=%d A=%d" % (nq, A))
    rho = pk.density_matrix(torch.from_numpy(C).to("cuda"), torch.from_numpy(P).to("cuda"))
    want_rho = O.density_matrix(C, P)
    lam, S, pur = pk.density_spectrum(rho)
    torch.cuda.synchronize()
    lam = lam.cpu().numpy()
    want = O.spectrum(want_rho)
    np.testing.assert_allclose(lam, want, rtol=0, atol=1e-12)
    assert abs(float(S) - O.entropy_bits(want)) < 1e-10
    assert abs(float(pur) - O.purity(want_rho)) < 1e-12


def test_spectrum_special_cases():
    pk = _pk()
    nq = 6
    N = 1 << nq
    rng = np.random.default_rng(3)
    _say("spectrum special cases n_q=%d" % nq)
    # pure state: eigenvalues 1 and N - 1 zeros, S = 0, Tr rho^2 = 1
    psi = _states(rng, 1, nq)
    lam, S, pur = pk.density_spectrum(pk.density_matrix(torch.from_numpy(psi).to("cuda"),
                                                        torch.ones(1, dtype=torch.float64, device="cuda")))
    lam = lam.cpu().numpy()
    assert abs(lam[-1] - 1.0) < 1e-12 and np.all(np.abs(lam[:-1]) < 1e-12)
    assert abs(float(S)) < 1e-9 and abs(float(pur) - 1.0) < 1e-12
    # orthonormal universes: the weights are the nonzero eigenvalues
    Q, _ = np.linalg.qr(rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)))
    P = rng.uniform(0.1, 1.0, 5)
    P /= P.sum()
    lam, S, _ = pk.density_spectrum(pk.density_matrix(torch.from_numpy(np.ascontiguousarray(Q[:, :5].T)).to("cuda"),
                                                      torch.from_numpy(P).to("cuda")))
    lam = lam.cpu().numpy()
    np.testing.assert_allclose(lam[-5:], np.sort(P), atol=1e-12)
    assert abs(float(S) - float(-np.sum(P * np.log2(P)))) < 1e-10
    # the basis ensemble with equal weights is maximally mixed: S = n_q bits
    lam, S, pur = pk.density_spectrum(pk.density_matrix(torch.eye(N, dtype=torch.complex128, device="cuda"),
                                                        torch.full((N,), 1.0 / N, dtype=torch.float64, device="cuda")))
    assert abs(float(S) - nq) < 1e-10 and abs(float(pur) - 1.0 / N) < 1e-14


def test_density_rejects_bad_arguments():
    pk = _pk()
    with pytest.raises(pk.PaperkernError):
        pk.lib()  # the library is loaded
        rc = pk.lib().pk_density_matrix(0, 1, None, None, None, None)
        pk._check(rc, None)
    with pytest.raises(pk.PaperkernError):
        rc = pk.lib().pk_density_spectrum(16, None, None, None, None)
        pk._check(rc, None)
