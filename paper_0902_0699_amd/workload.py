"""Seeded synthetic inputs shaped like the paper's Grover workload.

This module is shared by the tests, the benchmark and the CPU reference.  It
draws random numbers and assembles gate lists; it holds none of the method's
arithmetic (no gate is applied here).

Draw order for one instance, from ``numpy.random.default_rng(seed)`` (PCG64):
  x     = integers(0, N)          marked item (the Oracle's target, Sec. 5.1)
  qhit  = integers(1, nq + 1)     qubit struck by the noise rotation (Sec. 6.3)
  eloc  = integers(0, 5)          stage boundary of the noise rotation
  alpha = uniform(0, 2 pi), beta = uniform(0, pi), gamma = 0 (Sec. 6.3 footnote)
  key   = integers(0, 2^63), then psi from per-block streams keyed by (key, block)
          (see haar_state): complex normals, normalised -- a Haar-random pure
          state, the paper's domain being normalised states.
The batched workload first draws every n_q, then the instances in index order;
instance 0 is the noise-free universe (its noise draws are made and ignored so
that the stream does not depend on that rule).

Gate lists use the tuple vocabulary of the paper's routines:
  ("H", i_s), ("ONEOP", i_s, op2x2), ("HALL",), ("ORACLE",), ("INV",),
  ("D2", i_s, alpha, beta, gamma); tuples apply left to right.
"""

import math
import os

import numpy as np

BLOCK = 1 << 20  # amplitudes per independent random stream

# Workload sizes: the single-instance parity case, the paper's largest case
# ("up to 30 qubits", Sec. 1), and the multiverse batch.
NQ_SMALL = 20
NQ_LARGE = 30
BATCH_INSTANCES = 4096
BATCH_NQ_MIN = 10
BATCH_NQ_SPAN = 10

SEEDS = {"small_fp64": 0, "large_fp64": 1, "large_fp32": 2, "batched": 3, "gradient": 4, "shor": 6, "density": 7}

# The ensemble density matrix (Sec. 6.1): universes of the paper's largest
# tabulated size (Sec. 7.1) in the batch's count.
DENSITY_NQ = 12
DENSITY_UNIVERSES = 4096

# Shor's data path at n_q = 30: M = 899 = 29 * 31 gives registers of n1 = 20 and
# n2 = 10 qubits (Step 1), the largest FP64 state of one GPU's share.
SHOR_M = 899


def _block_normals(key, block, size):
    """2*size normals of block ``block``: its own PCG64 stream keyed by (key, block)."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([key, block])))
    return g.standard_normal(2 * size)


def haar_state(rng, nq, threads=None):
    """Haar-random pure state: complex normals, then normalised.

    A 63-bit key is drawn from ``rng``; amplitude block b (BLOCK amplitudes)
    takes 2*BLOCK normals from its own PCG64 stream seeded by (key, b): real
    parts first, then imaginary parts.  Blocks are independent, so they are
    drawn in parallel threads; the result does not depend on the thread count.
    """
    size = 1 << nq
    key = int(rng.integers(0, 1 << 63))
    psi = np.empty(size, dtype=np.complex128)
    pairs = psi.view(np.float64).reshape(size, 2)
    bsize = min(size, BLOCK)
    nblocks = size // bsize

    def fill(b):
        z = _block_normals(key, b, bsize)
        seg = pairs[b * bsize:(b + 1) * bsize]
        seg[:, 0] = z[:bsize]
        seg[:, 1] = z[bsize:]
        return float(np.einsum("ij,ij->", seg, seg))

    if nblocks == 1:
        sums = [fill(0)]
    else:
        from concurrent.futures import ThreadPoolExecutor
        workers = threads or min(16, os.cpu_count() or 1)
        with ThreadPoolExecutor(max_workers=workers) as ex:
            sums = list(ex.map(fill, range(nblocks)))
    psi /= math.sqrt(math.fsum(sums))
    return psi


def grover_gates(noise=None):
    """Gate list of one Grover iteration, Oracle first (G = HALL.Inv.HALL.Oracle),
    with an optional D2 inserted at stage boundary eloc."""
    steps = [("ORACLE",), ("HALL",), ("INV",), ("HALL",)]
    if noise is None:
        return steps
    qhit, eloc, alpha, beta, gamma = noise
    return steps[:eloc] + [("D2", int(qhit), float(alpha), float(beta), float(gamma))] + steps[eloc:]


def phase_circuit(rng, nq, count):
    """Hadamards on every qubit, then ``count`` controlled phases (CPHASE, or
    CPHASEK with k in 1..5) on random distinct qubit pairs, each followed by a
    Hadamard on a random qubit with probability 0.1: a circuit whose stages carry
    many controlled phases over tile-index, thread and register bits at once."""
    gates = [("H", q) for q in range(1, nq + 1)]
    for _ in range(count):
        a, b = rng.choice(np.arange(1, nq + 1), 2, replace=False)
        if rng.random() < 0.5:
            gates.append(("CPHASE", int(a), int(b)))
        else:
            gates.append(("CPHASEK", int(a), int(b), int(rng.integers(1, 6))))
        if rng.random() < 0.1:
            gates.append(("H", int(rng.integers(1, nq + 1))))
    return gates


def draw_instance(rng, nq, noisy=True, with_state=True):
    """One noisy Grover instance: dict(nq, marked, noise, gates, psi)."""
    size = 1 << nq
    x = int(rng.integers(0, size))
    qhit = int(rng.integers(1, nq + 1))
    eloc = int(rng.integers(0, 5))
    alpha = float(rng.uniform(0.0, 2.0 * math.pi))
    beta = float(rng.uniform(0.0, math.pi))
    noise = (qhit, eloc, alpha, beta, 0.0) if noisy else None
    inst = {"nq": nq, "marked": [x], "noise": noise, "gates": grover_gates(noise)}
    inst["psi"] = haar_state(rng, nq) if with_state else None
    return inst


def single_instance(seed, nq):
    """The single-instance workloads: one noisy iteration at n_q qubits from ``seed``."""
    return draw_instance(np.random.default_rng(seed), nq)


def batch_sizes(rng, count=BATCH_INSTANCES, nq_min=BATCH_NQ_MIN, span=BATCH_NQ_SPAN):
    """n_q,i = nq_min + floor(span * u), u ~ U[0,1): sizes log-uniform over 2^span."""
    u = rng.random(count)
    return [nq_min + int(math.floor(span * v)) for v in u]


def batch_instances(seed, count=BATCH_INSTANCES, nq_min=BATCH_NQ_MIN, span=BATCH_NQ_SPAN):
    """The multiverse batch: instance 0 noise-free, the others each with one D2."""
    rng = np.random.default_rng(seed)
    sizes = batch_sizes(rng, count, nq_min, span)
    return [draw_instance(rng, nq, noisy=(i != 0)) for i, nq in enumerate(sizes)]


def fd_subset(seed, inst, count=64):
    """Inputs checked by central differences: the three angles, Re/Im of psi[x],
    then count-5 further (index, part) components drawn from a stream seeded by
    ``seed`` + 1000."""
    rng = np.random.default_rng(seed + 1000)
    size = 1 << inst["nq"]
    x = inst["marked"][0]
    comps = [("angle", 0), ("angle", 1), ("angle", 2), ("psi", (x, 0)), ("psi", (x, 1))]
    idx = rng.integers(0, size, count - 5)
    part = rng.integers(0, 2, count - 5)
    comps += [("psi", (int(i), int(p))) for i, p in zip(idx, part)]
    return comps


def shor_xguess(seed, M=SHOR_M):
    """Step 3's random choice: integers drawn uniformly from 2 .. M-1 until one is
    coprime to M (the GCD test), from ``default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    while True:
        x = int(rng.integers(2, M))
        if math.gcd(x, M) == 1:
            return x


def density_universes(seed, nq=DENSITY_NQ, count=DENSITY_UNIVERSES):
    """Noisy multiverses of one Grover search (Sec. 6.2, 6.3): one marked item x
    shared by all universes, each universe one noisy iteration from the uniform
    state (the same noise draws as ``draw_instance``), universe 0 noise-free.
    Returns (gate lists, x); the caller starts every universe from HALL|0..0>."""
    rng = np.random.default_rng(seed)
    x = int(rng.integers(0, 1 << nq))
    gates = []
    for a in range(count):
        qhit = int(rng.integers(1, nq + 1))
        eloc = int(rng.integers(0, 5))
        alpha = float(rng.uniform(0.0, 2.0 * math.pi))
        beta = float(rng.uniform(0.0, math.pi))
        gates.append(grover_gates(None if a == 0 else (qhit, eloc, alpha, beta, 0.0)))
    return gates, x
