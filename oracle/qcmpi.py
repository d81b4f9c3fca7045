"""Plain, slow, obviously-correct FP64 reference for one noisy Grover iteration.

TEST INFRASTRUCTURE ONLY (see the package docstring): never imported by the
product path.

Conventions (all from the paper, Sec. 2.2 "Multi-qubit states"):
  * an n_q-qubit state is the array C_n, n = 0 .. 2^n_q - 1, in standard order;
  * n = sum_i q_i 2^(n_q - i) (Eq. staten): qubit 1 is the most significant
    bit, qubit n_q the least significant;
  * a one-qubit operator on qubit i_s couples the partner pair
    n_1 = n_0 + 2^(n_q - i_s) (Eqs. pair0, pair1 and the "stride" of Sec. 3).

Gate lists are sequences of tuples, applied left to right (first tuple first):
  ("H", i_s)                      Hadamard on qubit i_s (Eq. NOTH)
  ("ONEOP", i_s, op)              any 2x2 complex operator, op[a][b] = <a|op|b>
  ("HALL",)                       Hadamard on every qubit (Eq. HALL, Sec. 4.3)
  ("ORACLE",)                     sign flip of every marked item (Eq. oracle1)
  ("INV",)                        2|0..0><0..0| - I (Eq. inversion)
  ("D2", i_s, alpha, beta, gamma) Wigner D^(1/2) noise rotation (Sec. 6.3)
  ("TWOOP", is1, is2, V)          any 4x4 operator on qubits is1, is2 (Eq. resmat2);
                                  V[ab][cd] = <a b|V|c d>, a the value of qubit is1
  ("CNOT", is1, is2)              control is1, target is2 (Sec. 4.2)
  ("CPHASE", is1, is2)            diag(1, 1, 1, -1) (Sec. 4.2)
  ("CPHASEK", is1, is2, k)        diag(1, 1, 1, e^{2 pi i / 2^k}) (Eq. cphasek)
  ("SWAP", is1, is2)              exchanges the two qubits (the QFT of App. A)
  ("D4", is1, is2, alpha, beta, gamma)  Wigner D^(3/2) two-qubit noise (Sec. 6.3)
  ("QFT", first, n)               quantum Fourier transform of the register of qubits
                                  first .. first+n-1 (App. A), applied by its definition
                                  <n|QFT|n'> = N^(-1/2) e^{2 pi i n n'/N}, N = 2^n

The Shor section (Sec. 5.2, Steps 1-6; App. A) adds the register sizes, the
loaded state of Eq. Shor2, the QFT ladder of App. A as a gate list, the
register-1 marginal p(n) = sum_k |C_{n,k}|^2 and its closed form (Eq. probshor).

The density-matrix section (Sec. 6.1) adds the ensemble density matrix of
weighted universes, its purity Tr rho^2 and its entropy.
"""

import math

import numpy as np

__all__ = [
    "stride", "pair_indices", "pair_indices_loop", "quartet_indices",
    "section_seat", "same_section",
    "PAULI_X", "PAULI_Y", "PAULI_Z", "IDENTITY", "NOT", "HADAMARD",
    "apply_oneop", "apply_oneop_loop", "hall", "hall2_sign", "hall2",
    "oracle_flip", "inversion",
    "rz", "ry", "d2_matrix", "d2_derivatives",
    "grover_gates", "apply_gate", "apply_gate_adjoint", "evaluate",
    "readout", "adjoint_grad", "fd_grad_angles", "fd_grad_psi",
    "kron_operator", "dense_circuit",
    "grover_closed_form", "diffusion_closed_form", "grover_sampled", "grover_sampler",
    "adjoint_gates",
    "CNOT", "CPHASE", "SWAP", "cphasek", "apply_twoop", "apply_twoop_loop",
    "wigner_small_d", "wigner_small_d_prime", "wigner_d", "d4_matrix", "d4_derivatives",
    "kron_twoop", "TWO_QUBIT", "PARAMETRIC",
    "ceil_log2", "shor_register_sizes", "shor_f", "shor_state", "qft_register", "qft_gates",
    "marginal", "multiplicative_order", "probshor_marginal", "shor_qft_amplitudes",
    "density_matrix", "density_matrix_loop", "purity", "purity_gram", "entropy_bits", "spectrum",
]

# ---------------------------------------------------------------------------
# Index map (Sec. 2.2, Eqs. staten / pair0 / pair1; Sec. 3; Sec. 4 Eq. twoopB)
# ---------------------------------------------------------------------------


def stride(nq, i_s):
    """Stride of qubit i_s: the step 2^(n_q - i_s) from n_0 to its partner (Sec. 3)."""
    if not 1 <= i_s <= nq:
        raise ValueError("qubit label must lie in 1..nq")
    return 1 << (nq - i_s)


def pair_indices(nq, i_s):
    """All 2^n_q / 2 partner pairs (n_0, n_1) for qubit i_s, n_0 ascending.

    Eq. pair0 gives n_0 = n - q_{i_s} 2^(n_q-i_s); the pairs are enumerated by
    the labels n whose qubit i_s is 0, and n_1 = n_0 + stride (Sec. 3).
    """
    n = np.arange(1 << nq, dtype=np.int64)
    q = (n >> (nq - i_s)) & 1
    n0 = n[q == 0]
    return n0, n0 + stride(nq, i_s)


def pair_indices_loop(nq, i_s):
    """Pure-Python version of :func:`pair_indices` through binary labels.

    Builds each label's bit array B(1..n_q) (the dectobin routine of Sec. 2.2),
    keeps labels with B(i_s) = 0, and forms the partner by setting B(i_s) = 1
    and converting back (bintodec).  For small n_q only.
    """
    pairs0, pairs1 = [], []
    for n in range(1 << nq):
        bits = [(n >> (nq - i)) & 1 for i in range(1, nq + 1)]
        if bits[i_s - 1] == 0:
            partner = list(bits)
            partner[i_s - 1] = 1
            pairs0.append(sum(b << (nq - i) for i, b in enumerate(bits, start=1)))
            pairs1.append(sum(b << (nq - i) for i, b in enumerate(partner, start=1)))
    return np.array(pairs0, dtype=np.int64), np.array(pairs1, dtype=np.int64)


def quartet_indices(nq, is1, is2):
    """Amplitude quartets (n_00, n_01, n_10, n_11) of Sec. 4, Eq. twoopB.

    n_01 = n_00 + 2^(n_q - is2), n_10 = n_00 + 2^(n_q - is1); 2^n_q / 4 quartets.
    """
    if is1 == is2:
        raise ValueError("two-qubit operator needs two distinct qubits")
    n = np.arange(1 << nq, dtype=np.int64)
    free = (((n >> (nq - is1)) & 1) == 0) & (((n >> (nq - is2)) & 1) == 0)
    n00 = n[free]
    s1, s2 = stride(nq, is1), stride(nq, is2)
    return n00, n00 + s2, n00 + s1, n00 + s1 + s2


def section_seat(n, nq, p):
    """Processor (section) and seat of label n with N_P = 2^p ranks (Sec. 3.2)."""
    nx = (1 << nq) >> p  # NPART = 2^(n_q - p)
    return n // nx, n % nx


def same_section(nq, i_s, p):
    """Locality rule of Sec. 3.1: the pair of qubit i_s is on one rank iff i_s > p."""
    return i_s > p


# ---------------------------------------------------------------------------
# One-qubit operators (Eq. Pauli, Eq. NOTH; Eq. resmat1 of Sec. 3)
# ---------------------------------------------------------------------------

IDENTITY = np.eye(2, dtype=np.complex128)
PAULI_X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
PAULI_Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
PAULI_Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
NOT = PAULI_X
HADAMARD = (PAULI_X + PAULI_Z) / math.sqrt(2.0)


def apply_oneop(psi, nq, i_s, op):
    """Return Omega_s psi for a 2x2 operator on qubit i_s (Eq. resmat1).

    For every pair, (C~_n0, C~_n1) = op (C_n0, C_n1) with op[a][b] = <a|op|b>.
    The state is viewed as (2^(i_s-1), 2, 2^(n_q-i_s)); axis 1 is q_{i_s}, so
    v[:, 0, :] are the C_n0 and v[:, 1, :] their partners one stride away.
    """
    psi = np.asarray(psi, dtype=np.complex128)
    op = np.asarray(op, dtype=np.complex128)
    v = psi.reshape(1 << (i_s - 1), 2, 1 << (nq - i_s))
    c0, c1 = v[:, 0, :], v[:, 1, :]
    out = np.empty_like(v)
    out[:, 0, :] = op[0, 0] * c0 + op[0, 1] * c1
    out[:, 1, :] = op[1, 0] * c0 + op[1, 1] * c1
    return out.reshape(-1)


def apply_oneop_loop(psi, nq, i_s, op):
    """Eq. resmat1 pair by pair over :func:`pair_indices_loop` (small n_q only)."""
    out = np.array(psi, dtype=np.complex128)
    n0s, n1s = pair_indices_loop(nq, i_s)
    for n0, n1 in zip(n0s, n1s):
        a, b = psi[n0], psi[n1]
        out[n0] = op[0][0] * a + op[0][1] * b
        out[n1] = op[1][0] * a + op[1][1] * b
    return out


def hall(psi, nq):
    """HALL: the Hadamard on qubits 1..n_q in turn (Eq. HALL, Sec. 4.3)."""
    for i_s in range(1, nq + 1):
        psi = apply_oneop(psi, nq, i_s, HADAMARD)
    return psi


def hall2_sign(nq, n, n_prime):
    """The sign s_{n,n'} of Sec. 4.3 (function SH).

    (-1)^delta where delta counts the qubits i with B(i) = B'(i) = 1.
    """
    delta = sum(((n >> (nq - i)) & 1) & ((n_prime >> (nq - i)) & 1) for i in range(1, nq + 1))
    return -1 if delta % 2 else 1


def hall2(psi, nq):
    """HALL2: C~_n = 2^(-n_q/2) sum_n' s_{n,n'} C_n' (Sec. 4.3), O(4^n_q), brute force."""
    size = 1 << nq
    s = np.empty((size, size), dtype=np.float64)
    for n in range(size):
        for m in range(size):
            s[n, m] = hall2_sign(nq, n, m)
    return (s @ np.asarray(psi, dtype=np.complex128)) / (2.0 ** (nq / 2.0))


def oracle_flip(psi, marked):
    """Oracle of Eq. oracle1, extended to several marked items: C_x -> -C_x."""
    out = np.array(psi, dtype=np.complex128)
    for x in marked:
        out[x] = -out[x]
    return out


def inversion(psi):
    """Inv = 2|0..0><0..0| - I (Eq. inversion): every C_n with n != 0 changes sign."""
    out = -np.asarray(psi, dtype=np.complex128)
    out[0] = psi[0]
    return out


# ---------------------------------------------------------------------------
# Two-qubit operators (Sec. 4: Eqs. twoopA, twoopB, resmat2; Sec. 4.2)
# ---------------------------------------------------------------------------
#
# Basis order of a 4x4 operator: |q_is1 q_is2> = |00>, |01>, |10>, |11>, index
# 2 q_is1 + q_is2, whatever the significance of is1 and is2 in the label n
# (Eq. twoopB lists n_00, n_01, n_10, n_11 that way).

TWO_QUBIT = ("TWOOP", "CNOT", "CPHASE", "CPHASEK", "SWAP", "D4")
PARAMETRIC = ("D2", "D4")

CNOT = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=np.complex128)
CPHASE = np.diag([1, 1, 1, -1]).astype(np.complex128)
SWAP = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=np.complex128)


def cphasek(k):
    """CPHASEK of Eq. cphasek: the phase e^{2 pi i / 2^k} on |11> only."""
    return np.diag([1, 1, 1, np.exp(2j * math.pi / (1 << k))]).astype(np.complex128)


def apply_twoop(psi, nq, is1, is2, op):
    """Return V psi for a 4x4 operator on qubits is1, is2 (Eq. resmat2).

    Every amplitude quartet (n_00, n_01, n_10, n_11) of Eq. twoopB (from
    :func:`quartet_indices`) is replaced by V times it.
    """
    psi = np.asarray(psi, dtype=np.complex128)
    op = np.asarray(op, dtype=np.complex128)
    quart = quartet_indices(nq, is1, is2)
    q = np.stack([psi[n] for n in quart])
    r = op @ q
    out = psi.copy()
    for n, row in zip(quart, r):
        out[n] = row
    return out


def apply_twoop_loop(psi, nq, is1, is2, op):
    """Eq. resmat2 quartet by quartet in pure Python (small n_q only)."""
    out = np.array(psi, dtype=np.complex128)
    s1, s2 = stride(nq, is1), stride(nq, is2)
    for n in range(1 << nq):
        if (n // s1) % 2 or (n // s2) % 2:
            continue
        labels = [n, n + s2, n + s1, n + s1 + s2]
        vals = [psi[m] for m in labels]
        for a, m in enumerate(labels):
            out[m] = sum(op[a][c] * vals[c] for c in range(4))
    return out


# ---------------------------------------------------------------------------
# Noise rotation D^(1/2)(alpha, beta, gamma) (Sec. 6.3, subroutine D2)
# ---------------------------------------------------------------------------
#
# Reading adopted where the paper is silent: D = R_z(alpha) R_y(beta) R_z(gamma),
# R_z(phi) = diag(e^{-i phi/2}, e^{+i phi/2}), R_y(beta) the real rotation by
# beta/2; rows/columns are m = +1/2 (spin up = |0>, Sec. 2.1) then m = -1/2.


def rz(phi):
    return np.array([[np.exp(-0.5j * phi), 0.0], [0.0, np.exp(0.5j * phi)]], dtype=np.complex128)


def ry(beta):
    c, s = math.cos(0.5 * beta), math.sin(0.5 * beta)
    return np.array([[c, -s], [s, c]], dtype=np.complex128)


def _drz(phi):
    return np.array([[-0.5j * np.exp(-0.5j * phi), 0.0], [0.0, 0.5j * np.exp(0.5j * phi)]],
                    dtype=np.complex128)


def _dry(beta):
    c, s = math.cos(0.5 * beta), math.sin(0.5 * beta)
    return 0.5 * np.array([[-s, -c], [c, -s]], dtype=np.complex128)


def d2_matrix(alpha, beta, gamma):
    """Wigner rotation D^(1/2)(alpha, beta, gamma) as the product of three rotations."""
    return rz(alpha) @ ry(beta) @ rz(gamma)


def d2_derivatives(alpha, beta, gamma):
    """(dD/dalpha, dD/dbeta, dD/dgamma) by the product rule on the three factors."""
    return (_drz(alpha) @ ry(beta) @ rz(gamma),
            rz(alpha) @ _dry(beta) @ rz(gamma),
            rz(alpha) @ ry(beta) @ _drz(gamma))


# ---------------------------------------------------------------------------
# Two-qubit noise D^(3/2)(alpha, beta, gamma) (Sec. 6.3, subroutine D4)
# ---------------------------------------------------------------------------
#
# Reading adopted where the paper is silent: the 4x4 Wigner function of j = 3/2,
# D_{m'm} = e^{-i m' alpha} d_{m'm}(beta) e^{-i m gamma} (the same Euler
# convention as D2: for j = 1/2 it gives R_z(alpha) R_y(beta) R_z(gamma)), with
# rows and columns m = 3/2, 1/2, -1/2, -3/2 taken as the two-qubit basis
# |00>, |01>, |10>, |11>: m = 3/2 - (2 q_is1 + q_is2).


def wigner_small_d(twoj, beta):
    """d^j_{m'm}(beta), j = twoj / 2, from Wigner's formula; rows/cols m = j, j-1, .., -j.

    d = sum_s (-1)^(m'-m+s) sqrt((j+m')!(j-m')!(j+m)!(j-m)!)
        / ((j+m-s)! s! (m'-m+s)! (j-m'-s)!) cos(beta/2)^(2j+m-m'-2s) sin(beta/2)^(m'-m+2s).
    """
    return _wigner_small_d(twoj, beta, derivative=False)


def wigner_small_d_prime(twoj, beta):
    """d/dbeta of :func:`wigner_small_d`, term by term."""
    return _wigner_small_d(twoj, beta, derivative=True)


def _wigner_small_d(twoj, beta, derivative):
    f = math.factorial
    c, s = math.cos(0.5 * beta), math.sin(0.5 * beta)
    n = twoj + 1
    out = np.zeros((n, n))
    # work with integers J = 2j, M = 2m so that factorial arguments stay integral
    for r in range(n):
        mp = twoj - 2 * r  # 2 m'
        for col in range(n):
            m = twoj - 2 * col  # 2 m
            jpm, jmm = (twoj + mp) // 2, (twoj - mp) // 2  # j + m', j - m'
            jpn, jmn = (twoj + m) // 2, (twoj - m) // 2  # j + m, j - m
            dm = (mp - m) // 2  # m' - m
            pref = math.sqrt(f(jpm) * f(jmm) * f(jpn) * f(jmn))
            total = 0.0
            for k in range(0, max(jpn, jmm) + 1):
                if jpn - k < 0 or dm + k < 0 or jmm - k < 0:
                    continue
                coef = (-1) ** (dm + k) * pref / (f(jpn - k) * f(k) * f(dm + k) * f(jmm - k))
                pc = twoj - dm - 2 * k  # exponent of cos
                ps = dm + 2 * k  # exponent of sin
                if not derivative:
                    total += coef * c ** pc * s ** ps
                else:
                    term = 0.0
                    if pc:
                        term += -0.5 * pc * c ** (pc - 1) * s ** (ps + 1)
                    if ps:
                        term += 0.5 * ps * c ** (pc + 1) * s ** (ps - 1)
                    total += coef * term
            out[r, col] = total
    return out


def wigner_d(twoj, alpha, beta, gamma):
    """D^j_{m'm}(alpha, beta, gamma) = e^{-i m' alpha} d^j_{m'm}(beta) e^{-i m gamma}."""
    m = np.array([0.5 * (twoj - 2 * r) for r in range(twoj + 1)])
    left = np.exp(-1j * m * alpha)
    right = np.exp(-1j * m * gamma)
    return left[:, None] * wigner_small_d(twoj, beta) * right[None, :]


def d4_matrix(alpha, beta, gamma):
    """D^(3/2)(alpha, beta, gamma) in the basis |q_is1 q_is2> (m = 3/2 - index)."""
    return wigner_d(3, alpha, beta, gamma)


def d4_derivatives(alpha, beta, gamma):
    """(dD/dalpha, dD/dbeta, dD/dgamma) of :func:`d4_matrix`."""
    m = np.array([1.5, 0.5, -0.5, -1.5])
    D = d4_matrix(alpha, beta, gamma)
    left = np.exp(-1j * m * alpha)
    right = np.exp(-1j * m * gamma)
    dbeta = left[:, None] * wigner_small_d_prime(3, beta) * right[None, :]
    return (-1j * m[:, None] * D, dbeta, D * (-1j * m[None, :]))


# ---------------------------------------------------------------------------
# Circuits: the Grover operator of Sec. 5.1 with the noise of Sec. 6.3
# ---------------------------------------------------------------------------


def grover_gates(noise=None):
    """One Grover iteration G = HALL . Inv . HALL . Oracle (Sec. 5.1).

    Operator products act right to left, so the Oracle comes first in the list.
    ``noise`` = (qhit, eloc, alpha, beta, gamma) inserts one D2 at stage
    boundary eloc in 0..4 (before the Oracle, after the Oracle, after the first
    HALL, after Inv, after the second HALL), as in Sec. 6.3.
    """
    steps = [("ORACLE",), ("HALL",), ("INV",), ("HALL",)]
    if noise is None:
        return steps
    qhit, eloc, alpha, beta, gamma = noise
    if not 0 <= eloc <= 4:
        raise ValueError("eloc must be a stage boundary 0..4")
    return steps[:eloc] + [("D2", int(qhit), float(alpha), float(beta), float(gamma))] + steps[eloc:]


def _gate_matrix(gate):
    kind = gate[0]
    if kind == "H":
        return HADAMARD
    if kind == "ONEOP":
        return np.asarray(gate[2], dtype=np.complex128)
    if kind == "D2":
        return d2_matrix(*gate[2:5])
    if kind == "TWOOP":
        return np.asarray(gate[3], dtype=np.complex128)
    if kind == "CNOT":
        return CNOT
    if kind == "CPHASE":
        return CPHASE
    if kind == "CPHASEK":
        return cphasek(gate[3])
    if kind == "SWAP":
        return SWAP
    if kind == "D4":
        return d4_matrix(*gate[3:6])
    raise ValueError(kind)


def _angles(gate):
    return gate[2:5] if gate[0] == "D2" else gate[3:6]


def _derivatives(gate):
    return d2_derivatives(*_angles(gate)) if gate[0] == "D2" else d4_derivatives(*_angles(gate))


def _apply_matrix(psi, nq, gate, m):
    if gate[0] in TWO_QUBIT:
        return apply_twoop(psi, nq, gate[1], gate[2], m)
    return apply_oneop(psi, nq, gate[1], m)


def apply_gate(psi, nq, gate, marked):
    """Apply one gate tuple (see the module docstring) to psi."""
    kind = gate[0]
    if kind in ("H", "ONEOP", "D2") or kind in TWO_QUBIT:
        return _apply_matrix(psi, nq, gate, _gate_matrix(gate))
    if kind == "HALL":
        return hall(psi, nq)
    if kind == "ORACLE":
        return oracle_flip(psi, marked)
    if kind == "INV":
        return inversion(psi)
    if kind == "QFT":
        return qft_register(psi, nq, gate[1], gate[2])
    raise ValueError("unknown gate kind %r" % (kind,))


def apply_gate_adjoint(psi, nq, gate, marked):
    """Apply the Hermitian adjoint of one gate (HALL, Oracle and Inv are self-adjoint)."""
    kind = gate[0]
    if kind in ("H", "ONEOP", "D2") or kind in TWO_QUBIT:
        return _apply_matrix(psi, nq, gate, _gate_matrix(gate).conj().T)
    if kind == "QFT":
        return qft_register(psi, nq, gate[1], gate[2], inverse=True)
    return apply_gate(psi, nq, gate, marked)


def readout(psi, marked):
    """(L, norm): L = sum_{n in M} |C_n|^2, the success probability read out in Sec. 5.1,
    and sum_n |C_n|^2; both correctly rounded with math.fsum."""
    p = np.abs(np.asarray(psi)) ** 2
    return math.fsum(float(p[x]) for x in marked), math.fsum(p.tolist())


def evaluate(nq, gates, marked, psi_in):
    """Apply ``gates`` in list order to psi_in (used as given, not renormalised).

    Returns (psi_out, L, norm) with L and norm from :func:`readout`.
    """
    psi = np.array(psi_in, dtype=np.complex128)
    if psi.shape != (1 << nq,):
        raise ValueError("psi_in must have 2^nq amplitudes")
    for g in gates:
        psi = apply_gate(psi, nq, g, marked)
    L, norm = readout(psi, marked)
    return psi, L, norm


# ---------------------------------------------------------------------------
# Gradients (not in the paper): store-all adjoint and central differences
# ---------------------------------------------------------------------------


def adjoint_grad(nq, gates, marked, psi_in, dL=1.0):
    """Gradient of dL * L by a store-all reverse sweep.

    Keeps every intermediate state psi_k, seeds lambda_K = dL * P_M psi_K,
    and for each gate from last to first adds 2 Re <lambda_k| dU_k/dtheta |psi_{k-1}>
    to the angle gradient before setting lambda_{k-1} = U_k^dagger lambda_k.
    Returns (grad_psi, grad_angles): grad_psi = 2 lambda_0 in the real-pair
    convention (real part = dL/dRe psi_in, imaginary part = dL/dIm psi_in) and
    grad_angles a (n_param, 3) array, one row per D2 or D4 gate in gate-list order.
    """
    states = [np.array(psi_in, dtype=np.complex128)]
    for g in gates:
        states.append(apply_gate(states[-1], nq, g, marked))
    lam = np.zeros_like(states[-1])
    for x in marked:
        lam[x] = dL * states[-1][x]
    positions = [k for k, g in enumerate(gates) if g[0] in PARAMETRIC]
    grads = np.zeros((len(positions), 3))
    for k in range(len(gates) - 1, -1, -1):
        g = gates[k]
        if g[0] in PARAMETRIC:
            row = positions.index(k)
            for t, dmat in enumerate(_derivatives(g)):
                dpsi = _apply_matrix(states[k], nq, g, dmat)
                grads[row, t] = 2.0 * float(np.vdot(lam, dpsi).real)
        lam = apply_gate_adjoint(lam, nq, g, marked)
    return 2.0 * lam, grads


def _with_angle(gates, row, t, value):
    positions = [k for k, g in enumerate(gates) if g[0] in PARAMETRIC]
    k = positions[row]
    g = list(gates[k])
    g[(2 if g[0] == "D2" else 3) + t] = value
    out = list(gates)
    out[k] = tuple(g)
    return out


def fd_grad_angles(nq, gates, marked, psi_in, h=1e-6):
    """Central differences of L with respect to every D2 and D4 angle."""
    positions = [k for k, g in enumerate(gates) if g[0] in PARAMETRIC]
    out = np.zeros((len(positions), 3))
    for row, k in enumerate(positions):
        for t in range(3):
            base = _angles(gates[k])[t]
            lp = evaluate(nq, _with_angle(gates, row, t, base + h), marked, psi_in)[1]
            lm = evaluate(nq, _with_angle(gates, row, t, base - h), marked, psi_in)[1]
            out[row, t] = (lp - lm) / (2.0 * h)
    return out


def fd_grad_psi(nq, gates, marked, psi_in, index, part, h=1e-6):
    """Central difference of L with respect to Re (part=0) or Im (part=1) of psi_in[index]."""
    step = h if part == 0 else 1j * h
    pp = np.array(psi_in, dtype=np.complex128)
    pm = np.array(psi_in, dtype=np.complex128)
    pp[index] += step
    pm[index] -= step
    return (evaluate(nq, gates, marked, pp)[1] - evaluate(nq, gates, marked, pm)[1]) / (2.0 * h)


# ---------------------------------------------------------------------------
# Brute force and closed forms (independent routes used as pins)
# ---------------------------------------------------------------------------


def kron_operator(nq, i_s, op):
    """Full 2^n_q x 2^n_q matrix I x .. x op x .. x I with qubit 1 leftmost.

    Uses the tensor-product rule of the footnote in Sec. 2.1; independent of the
    stride formula.  Small n_q only.
    """
    m = np.ones((1, 1), dtype=np.complex128)
    for i in range(1, nq + 1):
        m = np.kron(m, np.asarray(op, dtype=np.complex128) if i == i_s else IDENTITY)
    return m


def kron_twoop(nq, is1, is2, op):
    """Full matrix of a 4x4 operator on qubits is1, is2 as a sum of Kronecker products:
    sum_{ab,cd} V_{ab;cd} (.. x |a><c| at is1 x .. x |b><d| at is2 x ..), identity on
    every other qubit, qubit 1 leftmost.  Independent of the quartet formula."""
    op = np.asarray(op, dtype=np.complex128)
    size = 1 << nq
    out = np.zeros((size, size), dtype=np.complex128)
    for a, b, c, d in np.ndindex(2, 2, 2, 2):
        v = op[2 * a + b, 2 * c + d]
        if v == 0:
            continue
        m = np.ones((1, 1), dtype=np.complex128)
        for i in range(1, nq + 1):
            if i == is1:
                f = np.zeros((2, 2)); f[a, c] = 1.0
            elif i == is2:
                f = np.zeros((2, 2)); f[b, d] = 1.0
            else:
                f = IDENTITY
            m = np.kron(m, f)
        out += v * m
    return out


def dense_circuit(nq, gates, marked):
    """Dense matrix of a gate list, built from Kronecker products (small n_q only)."""
    size = 1 << nq
    u = np.eye(size, dtype=np.complex128)
    for g in gates:
        kind = g[0]
        if kind in ("H", "ONEOP", "D2"):
            m = kron_operator(nq, g[1], _gate_matrix(g))
        elif kind in TWO_QUBIT:
            m = kron_twoop(nq, g[1], g[2], _gate_matrix(g))
        elif kind == "HALL":
            m = np.ones((1, 1), dtype=np.complex128)
            for _ in range(nq):
                m = np.kron(m, HADAMARD)
        elif kind == "ORACLE":
            m = np.eye(size, dtype=np.complex128)
            for x in marked:
                m[x, x] = -1.0
        elif kind == "INV":
            e0 = np.zeros((size, 1))
            e0[0, 0] = 1.0
            m = 2.0 * (e0 @ e0.T) - np.eye(size)
        else:
            raise ValueError(kind)
        u = m @ u
    return u


def grover_closed_form(nq, k, x):
    """Amplitudes after k noise-free Grover iterations from HALL|0..0>.

    Textbook rotation picture behind the paper's n_t (Sec. 5.1):
    C_x = sin((2k+1) theta), C_{n != x} = cos((2k+1) theta) / sqrt(N - 1),
    sin theta = N^(-1/2).
    """
    size = 1 << nq
    theta = math.asin(1.0 / math.sqrt(size))
    out = np.full(size, math.cos((2 * k + 1) * theta) / math.sqrt(size - 1), dtype=np.complex128)
    out[x] = math.sin((2 * k + 1) * theta)
    return out


def diffusion_closed_form(psi):
    """HALL . Inv . HALL psi = 2 <s|psi> |s> - psi, i.e. C~_n = 2 mean(C) - C_n.

    Follows from Inv = 2|0><0| - I (Eq. inversion) and HALL|0..0> = |s>, the
    uniform state (Eq. Shor1); valid at any n_q.
    """
    psi = np.asarray(psi, dtype=np.complex128)
    return 2.0 * psi.mean() - psi


def adjoint_gates(gates):
    """The gate list of U^dagger for the list of U: the gates in reverse order, each
    replaced by its Hermitian adjoint.  HALL, ORACLE and INV are self-adjoint (real
    symmetric); a D2 or ONEOP becomes ("ONEOP", i_s, its conjugate transpose)."""
    out = []
    for g in reversed(list(gates)):
        if g[0] in ("D2", "ONEOP"):
            out.append(("ONEOP", g[1], _gate_matrix(g).conj().T))
        elif g[0] in ("HALL", "ORACLE", "INV"):
            out.append(g)
        else:
            raise ValueError("adjoint_gates takes HALL, ORACLE, INV, D2 and ONEOP gates")
    return out


def grover_sampler(nq, gates, marked, psi_in):
    """Exact amplitudes of one Grover iteration, or of its adjoint, at any labels
    and any n_q, without sweeping the state gate by gate.

    ``gates``: the iteration ORACLE, HALL, INV, HALL (Sec. 5.1) or the adjoint
    order HALL, INV, HALL, ORACLE, with at most one one-qubit rotation (D2 or
    ONEOP) anywhere between them (Sec. 6.3).  ``psi_in``: 2^nq amplitudes, or a
    basis vector given as ("basis", label, coefficient).

    Three identities remove every sweep:

      * HALL . Inv . HALL = 2|s><s| - I, from Inv = 2|0><0| - I (Eq. inversion),
        HALL|0..0> = |s> (Eq. Shor1) and HALL^2 = I;
      * HALL . D_q . HALL = (H D H)_q, since H^2 = I on every other qubit;
      * <0|HALL v> = N^(-1/2) sum_n v_n and <2^b|HALL v> = N^(-1/2) sum_n (-1)^(n_b) v_n.

    Every intermediate vector v is then known through a function giving v_n at
    any labels and its two half sums V_c = sum over n with bit b = c of v_n (b
    the state bit of the rotated qubit).  The half sums of psi_in are the only
    pass over the whole state, made once here.  Returns (amp, L): amp(indices)
    gives the output amplitudes at an int64 label array, L the readout
    sum_{x in M} |C_x|^2.
    """
    size = 1 << nq
    kinds = [g[0] for g in gates]
    rot = [k for k, g in enumerate(gates) if g[0] in ("D2", "ONEOP")]
    steps = [k for k in kinds if k not in ("D2", "ONEOP")]
    if steps not in (["ORACLE", "HALL", "INV", "HALL"], ["HALL", "INV", "HALL", "ORACLE"]) or len(rot) > 1:
        raise ValueError("grover_sampler takes one Grover iteration (or its adjoint) with at most one rotation")
    if rot:
        b = nq - gates[rot[0]][1]
        D = _gate_matrix(gates[rot[0]])
    else:
        b, D = 0, IDENTITY
    Ms = np.array(sorted(set(int(x) for x in marked)), dtype=np.int64)
    bit = 1 << b

    if isinstance(psi_in, tuple) and psi_in[0] == "basis":
        label, coeff = int(psi_in[1]), complex(psi_in[2])

        def f(n):
            n = np.asarray(n, dtype=np.int64)
            return np.where(n == label, coeff, 0.0 + 0.0j)
        V = (coeff, 0j) if not (label >> b) & 1 else (0j, coeff)
    else:
        psi = np.asarray(psi_in, dtype=np.complex128)
        if psi.shape != (size,):
            raise ValueError("psi_in must have 2^nq amplitudes")
        f = lambda n: psi[n]
        w = psi.reshape(size >> (b + 1), 2, bit)
        V = (w[:, 0, :].sum(), w[:, 1, :].sum())

    def oracle(f, V):
        def g(n):
            out = np.array(f(n), dtype=np.complex128)
            out[np.isin(n, Ms)] *= -1.0
            return out
        fx = f(Ms)
        up = ((Ms >> b) & 1).astype(bool)
        return g, (V[0] - 2.0 * fx[~up].sum(), V[1] - 2.0 * fx[up].sum())

    def one_qubit(f, V, M):  # Eq. resmat1 on bit b
        def g(n):
            up = ((n >> b) & 1).astype(bool)
            n0 = n & ~np.int64(bit)
            a0, a1 = f(n0), f(n0 | bit)
            return np.where(up, M[1, 0] * a0 + M[1, 1] * a1, M[0, 0] * a0 + M[0, 1] * a1)
        return g, (M[0, 0] * V[0] + M[0, 1] * V[1], M[1, 0] * V[0] + M[1, 1] * V[1])

    def diffusion(f, V, where):
        # HALL . Inv . HALL                                        (where None)
        # HALL . Inv . D . HALL = 2 |s> <0|D HALL - (H D H)_q       (where 0: D after the first HALL)
        # HALL . D . Inv . HALL = 2 HALL D|0> <0|HALL - (H D H)_q   (where 1: D after Inv)
        tot, alt = V[0] + V[1], V[0] - V[1]
        if where is None:
            return (lambda n: 2.0 * tot / size - f(n)), (tot - V[0], tot - V[1])
        g_dt, W_dt = one_qubit(f, V, HADAMARD @ D @ HADAMARD)
        if where == 0:
            c = D[0, 0] * tot + D[0, 1] * alt
            return (lambda n: 2.0 * c / size - g_dt(n)), (c - W_dt[0], c - W_dt[1])
        c0, c1 = tot * (D[0, 0] + D[1, 0]), tot * (D[0, 0] - D[1, 0])

        def g(n):
            up = ((n >> b) & 1).astype(bool)
            return 2.0 * np.where(up, c1, c0) / size - g_dt(n)
        return g, (c0 - W_dt[0], c1 - W_dt[1])

    k = 0
    while k < len(gates):
        kind = kinds[k]
        if kind == "ORACLE":
            f, V = oracle(f, V)
            k += 1
        elif kind in ("D2", "ONEOP"):
            f, V = one_qubit(f, V, D)
            k += 1
        else:  # HALL, then Inv and HALL, with the rotation possibly on either side of Inv
            block = kinds[k:k + 4]
            if block[:3] == ["HALL", "INV", "HALL"]:
                f, V = diffusion(f, V, None)
                k += 3
            elif block[1] in ("D2", "ONEOP"):
                f, V = diffusion(f, V, 0)
                k += 4
            else:
                f, V = diffusion(f, V, 1)
                k += 4
    L = math.fsum(float(abs(v) ** 2) for v in f(Ms)) if len(Ms) else 0.0
    return f, L


def grover_sampled(nq, gates, marked, psi_in, indices):
    """Amplitudes of one Grover iteration at the labels ``indices`` and L, through
    :func:`grover_sampler` (any n_q, one pass over psi_in).  Returns (values, L)."""
    amp, L = grover_sampler(nq, gates, marked, psi_in)
    return amp(np.asarray(indices, dtype=np.int64)), L


# ---------------------------------------------------------------------------
# Shor's data path (Sec. 5.2, Steps 1-6) and the QFT (App. A)
# ---------------------------------------------------------------------------


def ceil_log2(x):
    """Smallest integer e with 2^e >= x, for an integer x >= 1 (exact)."""
    x = int(x)
    if x < 1:
        raise ValueError("ceil_log2 needs x >= 1")
    return (x - 1).bit_length()


def shor_register_sizes(M):
    """(n_1, n_2) of Step 1: n_1 = Ceiling(log2 Q) with Q = 2^Ceiling(log2 M^2), so
    that register one holds M^2; n_2 = Ceiling(log2 M), so that register two
    holds every value below M."""
    M = int(M)
    if M < 2:
        raise ValueError("M must be at least 2")
    Q = 1 << ceil_log2(M * M)
    return ceil_log2(Q), ceil_log2(M)


def shor_f(xguess, M, n1):
    """f(j) = xguess^j mod M for j = 0 .. 2^n_1 - 1 (Step 3, Eq. fperiod), by
    repeated multiplication in Python integers."""
    out = np.empty(1 << n1, dtype=np.int64)
    v = 1 % M
    for j in range(1 << n1):
        out[j] = v
        v = (v * xguess) % M
    return out


def shor_state(n1, n2, xguess, M):
    """The loaded two-register state of Eq. Shor2:
    |Psi> = 2^(-n_1/2) sum_n |n>_{n_1} |f(n)>_{n_2}, register one on qubits
    1 .. n_1 (the high bits), so the amplitude of |n>|f(n)> sits at label
    n 2^(n_2) + f(n).  The amplitude is the correctly rounded double of
    2^(-n_1/2): sqrt(2) (correctly rounded) times an exact power of two."""
    if M > (1 << n2):
        raise ValueError("register two cannot hold M")
    amp = 2.0 ** (-(n1 // 2)) if n1 % 2 == 0 else math.sqrt(2.0) * 2.0 ** (-((n1 + 1) // 2))
    psi = np.zeros(1 << (n1 + n2), dtype=np.complex128)
    f = shor_f(xguess, M, n1)
    psi[(np.arange(1 << n1, dtype=np.int64) << n2) + f] = amp
    return psi


def qft_register(psi, nq, first, n, inverse=False):
    """QFT of the register of qubits first .. first+n-1 (App. A):
    <n|QFT|n'> = N^(-1/2) e^{2 pi i n n'/N}, N = 2^n, i.e. sqrt(N) times the
    inverse DFT along that register's axis (numpy.fft.ifft; the adjoint is
    N^(-1/2) times the forward DFT)."""
    if not (1 <= first and n >= 1 and first + n - 1 <= nq):
        raise ValueError("register out of range")
    psi = np.asarray(psi, dtype=np.complex128)
    hi = 1 << (first - 1)
    lo = 1 << (nq - first - n + 1)
    v = psi.reshape(hi, 1 << n, lo)
    N = float(1 << n)
    if inverse:
        out = np.fft.fft(v, axis=1) / math.sqrt(N)
    else:
        out = np.fft.ifft(v, axis=1) * math.sqrt(N)
    return out.reshape(-1)


def qft_gates(n1, first=1):
    """The QFT of the register of qubits first .. first+n_1-1 as a list of the paper's
    gates (Hadamards, CPHASEK, SWAP; App. A), derived from its definition Eq. QFT1.

    Write the input value n' = sum_r b_r 2^(n_1-r) over the register's qubits
    r = 1..n_1 (qubit 1 most significant) and the output value n = sum_s c_s
    2^(n_1-s).  The phase 2 pi n n' / 2^(n_1) = 2 pi sum_(r,s) b_r c_s 2^(n_1-r-s)
    is a multiple of 2 pi whenever r + s <= n_1, so only the bit pairs with
    r + s > n_1 contribute, each a factor e^(2 pi i b_r c_s / 2^(r+s-n_1)).

    A Hadamard on qubit r maps the input bit b_r to the output bit c_s with
    s = n_1 + 1 - r and supplies that pair's sign (-1)^(b_r c_s), the term
    r + s = n_1 + 1; the output therefore comes out in reversed qubit order.  The
    term of b_r with an output bit c_s that an earlier qubit q = n_1 + 1 - s < r
    already holds is the controlled phase of exponent r + s - n_1 = r + 1 - q
    between qubits r and q.  So, qubit by qubit: the phases of qubit r with the
    output bits of every earlier qubit, then the Hadamard on r; finally the swaps
    of qubits q and n_1 + 1 - q restore standard order.
    """
    def wire(r):
        return first - 1 + r

    g = []
    for r in range(1, n1 + 1):
        for s in range(n1 + 2 - r, n1 + 1):
            g.append(("CPHASEK", wire(r), wire(n1 + 1 - s), r + s - n1))
        g.append(("H", wire(r)))
    for q in range(1, n1 // 2 + 1):
        g.append(("SWAP", wire(q), wire(n1 + 1 - q)))
    return g


def marginal(psi, nq, n_low):
    """p(n) = sum_k |C_{n,k}|^2 over the n_low low qubits (register two), for every
    value n of the high nq - n_low qubits: the distribution of a measurement of
    register one (Step 6).  FP64 sums."""
    psi = np.asarray(psi, dtype=np.complex128)
    v = psi.reshape(-1, 1 << n_low)
    return (v.real ** 2 + v.imag ** 2).sum(axis=1)


def multiplicative_order(xguess, M):
    """The period r of f (Eq. fperiod): the smallest r > 0 with xguess^r = 1 mod M
    (brute force; needs gcd(xguess, M) = 1)."""
    if math.gcd(int(xguess), int(M)) != 1:
        raise ValueError("xguess must be coprime to M")
    v, r = xguess % M, 1
    while v != 1 % M:
        v = (v * xguess) % M
        r += 1
    return r


def probshor_marginal(n1, xguess, M):
    """Closed form of the register-one distribution after the QFT (Eqs. QFT1,
    QFT2, probshor).  With N = 2^n_1 and the period r, the r register-two values
    k = f(n_k), n_k = 0 .. r-1, each appear D_k = ceil((N - n_k)/r) times, and

        |C_{n,k}|^2 = N^-2 [sin(D_k pi n r/N) / sin(pi n r/N)]^2,

    which is D_k^2 / N^2 where n r/N is an integer (the 0/0 limit, the sum of D_k
    ones).  Returns p(n) = sum_k |C_{n,k}|^2, n = 0 .. N-1.  Only sin^2 enters, so
    each sine is taken of an exactly reduced argument in [0, pi/2]: with
    a = n r mod N, sin^2(pi a/N) = sin^2(pi min(a, N - a)/N) (and likewise for
    D n r mod N); near pi the rounded argument would cost relative accuracy."""
    N = 1 << n1
    r = multiplicative_order(xguess, M)
    n = np.arange(N, dtype=np.int64)
    a = (n * r) % N
    s1 = np.sin(np.pi * np.minimum(a, N - a) / N)
    p = np.zeros(N)
    # D_k takes at most two values; group the k by it
    counts = {}
    for nk in range(r):
        d = (N - nk + r - 1) // r
        counts[d] = counts.get(d, 0) + 1
    for d, cnt in counts.items():
        b = (d * a) % N
        s2 = np.sin(np.pi * np.minimum(b, N - b) / N)
        with np.errstate(divide="ignore", invalid="ignore"):
            ratio2 = np.where(a == 0, float(d) * d, (s2 / np.where(a == 0, 1.0, s1)) ** 2)
        p += cnt * ratio2 / (float(N) * N)
    return p


def shor_qft_amplitudes(n1, n2, xguess, M, labels):
    """Amplitudes of QFT(register one) applied to the state of Eq. Shor2, at chosen
    labels n 2^n2 + k, for any n1 (Eq. QFT1 before the sum over j is done):

        C_{n,k} = N^-1 sum_{j < N, f(j) = k} e^{2 pi i n j / N},   N = 2^n1,

    with j running over n_k + d r (n_k < r the first j with f(j) = k, r the period);
    zero when k is not a value of f.  Each phase is taken of the exactly reduced
    n j mod N."""
    N = 1 << n1
    r = multiplicative_order(xguess, M)
    first = {}
    v = 1 % M
    for j in range(r):
        first.setdefault(v, j)
        v = (v * xguess) % M
    labels = np.asarray(labels, dtype=np.int64)
    out = np.zeros(len(labels), dtype=np.complex128)
    for i, lab in enumerate(labels):
        n, k = int(lab) >> n2, int(lab) & ((1 << n2) - 1)
        if k not in first:
            continue
        j = np.arange(first[k], N, r, dtype=np.int64)
        ph = (n * j) % N
        out[i] = np.exp(2j * np.pi * ph / N).sum() / N
    return out


# ---------------------------------------------------------------------------
# Ensemble density matrix (Sec. 6.1)
# ---------------------------------------------------------------------------


def density_matrix(states, weights):
    """<n|rho|n'> = sum_alpha P_alpha C_alpha(n) C_alpha^*(n') (Sec. 6.1), for the
    universes' states as rows of ``states`` (A x N) and their weights P_alpha.
    One library matmul: rho = (C^T diag(P)) conj(C)."""
    C = np.asarray(states, dtype=np.complex128)
    P = np.asarray(weights, dtype=np.float64)
    return (C.T * P) @ C.conj()


def density_matrix_loop(states, weights):
    """The same sum written out element by element (small sizes only)."""
    C = np.asarray(states, dtype=np.complex128)
    A, N = C.shape
    rho = np.zeros((N, N), dtype=np.complex128)
    for n in range(N):
        for m in range(N):
            rho[n, m] = sum(weights[a] * C[a, n] * np.conj(C[a, m]) for a in range(A))
    return rho


def purity(rho):
    """Tr rho^2 = sum_{n,n'} |rho_{n n'}|^2 for Hermitian rho (1 for a pure state,
    below 1 for a mixed one: the footnote to Sec. 6.1 and the noise discussion of
    Sec. 6.3)."""
    r = np.asarray(rho)
    return float(np.sum(np.abs(r) ** 2))


def purity_gram(states, weights):
    """Tr rho^2 from the universes alone: sum_{a,b} P_a P_b |<a|b>|^2, with no N x N
    matrix."""
    C = np.asarray(states, dtype=np.complex128)
    P = np.asarray(weights, dtype=np.float64)
    G = C.conj() @ C.T
    return float(np.sum(np.outer(P, P) * np.abs(G) ** 2))


def spectrum(rho):
    """Eigenvalues of the Hermitian rho, ascending (LAPACK through numpy)."""
    return np.linalg.eigvalsh(np.asarray(rho, dtype=np.complex128))


def entropy_bits(eigenvalues):
    """S = -sum_i lambda_i log2 lambda_i over the positive eigenvalues (Sec. 6.1 leaves
    the base open; base 2 gives S = n_q for the maximally mixed state).  Eigenvalues
    at or below zero, which rounding leaves in place of exact zeros, add nothing."""
    lam = np.asarray(eigenvalues, dtype=np.float64)
    lam = lam[lam > 0]
    return float(-np.sum(lam * np.log2(lam)))
