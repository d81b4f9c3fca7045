"""Executes a compiled pass schedule (the JSON of pk_plan_describe) on the CPU.

Test helper for the host plan compiler: it applies every op of every stage in
schedule order to the whole state, addressing each op the way the kernel
does (local tile bit -> state bit through the pass's tile bits; Flip entries
as (tile, local label)), with unnormalised Hadamard butterflies and the pass
scales the compiler chose.  Agreement with the oracle shows that the
compiler's reordering, scale bookkeeping, matrix indices and flip encoding
are right; the kernels are checked separately on the GPU.
"""

import numpy as np

import oracle as O


def _matrix_table(problems, desc):
    statics = []
    statics4 = []
    d2 = []
    d4 = []
    for p in problems:
        for g in p["gates"]:
            if g[0] == "ONEOP":
                statics.append(np.asarray(g[2], dtype=np.complex128))
            if g[0] == "D2":
                d2.append(tuple(float(v) for v in g[2:5]))
            if g[0] == "TWOOP":
                statics4.append(np.asarray(g[3], dtype=np.complex128))
            if g[0] in ("CNOT", "SWAP"):
                statics4.append(getattr(O, g[0]))
            if g[0] == "QFT":  # lowered with one SWAP per pair of the reversal
                statics4.extend([O.SWAP] * (g[2] // 2))
            if g[0] == "D4":
                d4.append(tuple(float(v) for v in g[3:6]))
    assert len(statics) == desc["n_static"] and len(d2) == desc["n_d2"]
    assert len(statics4) == desc["n_static4"] and len(d4) == desc["n_d4"]

    def mat4(m):
        ns = desc["n_static4"]
        if m < 2 * ns:
            M = statics4[m // 2]
            return M if m % 2 == 0 else M.conj().T
        d, r = divmod(m - 2 * ns, 5)
        D = O.d4_matrix(*d4[d])
        if r == 0:
            return D
        if r == 1:
            return D.conj().T
        return O.d4_derivatives(*d4[d])[r - 2]

    def mat(m):
        ns = desc["n_static"]
        if m < 2 * ns:
            M = statics[m // 2]
            return M if m % 2 == 0 else M.conj().T
        d, r = divmod(m - 2 * ns, 5)
        D = O.d2_matrix(*d2[d])
        if r == 0:
            return D
        if r == 1:
            return D.conj().T
        return O.d2_derivatives(*d2[d])[r - 2]

    mat.four = mat4
    return mat


def _apply_bit(vec, nq, bit, M):
    v = vec.reshape(1 << (nq - 1 - bit), 2, 1 << bit)
    a, b = v[:, 0, :].copy(), v[:, 1, :].copy()
    v[:, 0, :] = M[0, 0] * a + M[0, 1] * b
    v[:, 1, :] = M[1, 0] * a + M[1, 1] * b


def _apply_pair(vec, nq, bit1, bit2, M):
    """4x4 M on the state bits (bit1, bit2) in the basis |q_bit1 q_bit2>."""
    out = O.apply_twoop(vec, nq, nq - bit1, nq - bit2, M)
    vec[:] = out


def _param_row(desc, kind, slot):
    """Row of the angle-gradient array (the angle triple index) of a D2 / D4 slot."""
    return [i for i, p in enumerate(desc["params"]) if p == [kind, slot]][0]


def _global_index(nq, tbits, tile, j):
    free = [b for b in range(nq) if b not in tbits]
    g = 0
    for l, b in enumerate(tbits):
        g |= ((j >> l) & 1) << b
    for f, b in enumerate(free):
        g |= ((tile >> f) & 1) << b
    return g


def check_stage_shapes(nq, p):
    """Register bits are distinct local bits; gate ops name a register bit."""
    k = p["k"]
    for st in p["stages"]:
        rb = [r for r in st["rb"] if r >= 0]
        assert len(rb) == min(p["rbits"], k) and len(set(rb)) == len(rb) and all(0 <= r < k for r in rb)
        for op in st["ops"]:
            if op["kind"] in ("H", "MAT", "D2BWD"):
                assert 0 <= op["a"] < len(rb)
            if op["kind"] == "MAT4":  # a pair on register bits 0, 1 or (second pair) 2, 3
                assert op["a"] in (0, 2) and len(rb) >= op["a"] + 2
            if op["kind"] == "D4BWD":
                assert op["a"] == 0 and len(rb) >= 2
    assert len(set(p["tile_bits"])) == len(p["tile_bits"]) == k
    assert all(0 <= b < nq for b in p["tile_bits"])


def _store(vec, nq, tb, sb):
    """The pass's write-back: local bit l, read from state bit tb[l], goes to sb[l]."""
    if list(tb) == list(sb):
        return vec
    idx = np.arange(1 << nq, dtype=np.int64)
    dst = idx.copy()
    for a, b in zip(tb, sb):
        dst &= ~np.int64(1 << a)
    for a, b in zip(tb, sb):
        dst |= ((idx >> a) & 1) << b
    out = np.empty_like(vec)
    out[dst] = vec
    return out


def _phase_mask(nq, b1, b2):
    idx = np.arange(1 << nq, dtype=np.int64)
    return (((idx >> b1) & 1) == 1) & (((idx >> b2) & 1) == 1)


def _local_label(nq, tb, g):
    j = np.zeros_like(g)
    for l, b in enumerate(tb):
        j |= ((g >> b) & 1) << l
    return j


def _tile_index(nq, tb, g):
    free = [b for b in range(nq) if b not in tb]
    t = np.zeros_like(g)
    for f, b in enumerate(free):
        t |= ((g >> b) & 1) << f
    return t


def _extract(x, mask):
    """Bits of x at mask's set positions, packed from the least significant."""
    out = np.zeros_like(x)
    k = 0
    for b in range(64):
        if mask >> b & 1:
            out |= ((x >> b) & 1) << k
            k += 1
    return out


def _run_phases(desc, nq, tb, p, u, vecs):
    """The sub-stage's controlled phases as the kernel applies them: per slot, the
    leading phase_ucnt phases through the product tables (two of the pass's tile-part
    tables, indexed by tile-index bits, and one indexed by the thread's label bits),
    the rest one factor each with their
    conditions on the tile index (fmask) and the thread's label bits (tmask); the
    product applies where the slot's register bits are set, the local label
    decoded through the read map."""
    g = np.arange(1 << nq, dtype=np.int64)
    j = _local_label(nq, tb, g)
    tile = _tile_index(nq, tb, g)
    rb = u["rb"]
    twid = desc["twid"]
    assert twid is not None, "product tables are described for small plans only"
    tw = np.array(twid[0::2]) + 1j * np.array(twid[1::2])
    assert tw[0] == 1  # what lanes without a table load
    # stored grouped by slot, with the counts the kernel loops over
    slots = [desc["phases"][q][0] for q in range(u["phase_first"], u["phase_first"] + u["phase_count"])]
    assert slots == sorted(slots) and [slots.count(k) for k in range(4)] == u["phase_cnt"]
    q = u["phase_first"]
    for slot in range(4):
        cnt = u["phase_cnt"][slot]
        if cnt == 0:
            continue
        pm = u["phase_pm"][slot]
        assert pm >= 0
        rmask = 0
        for a in range(5):
            if pm >> a & 1:
                assert rb[a] >= 0
                rmask |= 1 << rb[a]
        fac = np.ones(1 << nq, dtype=complex)
        assert len(p["urefs"]) <= 64
        for r in (u["phase_ut0"][slot], u["phase_ut1"][slot]):
            if r >= 0:
                first, mask = p["urefs"][r]
                assert bin(mask).count("1") <= 10
                fac *= tw[first + _extract(tile, mask)]
        if u["phase_tt"][slot] >= 0:
            mask = u["phase_ttm"][slot]
            assert bin(mask).count("1") <= 10 and not mask & rmask
            fac *= tw[u["phase_tt"][slot] + _extract(j, mask)]
        for r in range(q + u["phase_ucnt"][slot], q + cnt):
            _, tmask, fmask, cm1, s = desc["phases"][r]
            assert not tmask & rmask
            hit = ((tile & fmask) == fmask) & ((j & tmask) == tmask)
            fac[hit] *= complex(1.0 + cm1, s)  # stored as c - 1
        q += cnt
        sel = (j & rmask) == rmask
        for v in vecs:
            v[sel] *= fac[sel]


_STEP_BITS = [("exchange", lambda v: v == 1), ("seed", lambda v: v >= 0), ("flip_pre", lambda v: v >= 0),
              ("phase_count", lambda v: v > 0), ("mat_pre_a", lambda v: v >= 0), ("hmask1", lambda v: v != 0),
              ("flip_mid", lambda v: v >= 0), ("hmask2", lambda v: v != 0), ("mat_post_a", lambda v: v >= 0),
              ("mat4", lambda v: v >= 0), ("d2b_a", lambda v: v >= 0), ("d4b_mat", lambda v: v >= 0),
              ("scale", lambda v: v != 0), ("read", lambda v: v >= 0), ("mat4b", lambda v: v >= 0)]


def _steps_of(u):
    """The step mask the kernel branches on, recomputed from the sub-stage's fields."""
    return sum(1 << i for i, (name, present) in enumerate(_STEP_BITS) if present(u[name]))


def _flip_index(desc, nq, tb, f):
    tile, j, slot = desc["flips"][f]
    return _global_index(nq, tb, tile, j), slot


def _run_subs(problems, desc, inst, direction, psi, lam=None, dL=1.0):
    """Executes the packed sub-stages (the form the kernel runs) of one direction."""
    mat = _matrix_table(problems, desc)
    info = desc["instances"][inst]
    nq = info["nq"]
    H = np.array([[1, 1], [1, -1]], dtype=np.complex128)
    vecs = [psi] if lam is None else [psi, lam]
    reads, grads = {}, {}
    for p in info[direction]:
        check_stage_shapes(nq, p)
        tb = p["tile_bits"]
        assert p["subs"] and p["subs"][0]["exchange"] == 1
        for u in p["subs"]:
            rb = u["rb"]
            assert u["steps"] == _steps_of(u)
            if u["seed"] >= 0:
                g, _ = _flip_index(desc, nq, tb, u["seed"])
                vecs[1][g] = dL * vecs[0][g]
            if u["flip_pre"] >= 0:
                g, _ = _flip_index(desc, nq, tb, u["flip_pre"])
                for v in vecs:
                    v[g] *= -1
            if u["phase_count"] > 0:
                _run_phases(desc, nq, tb, p, u, vecs)
            if u["mat_pre_a"] >= 0:
                for v in vecs:
                    _apply_bit(v, nq, tb[rb[u["mat_pre_a"]]], mat(u["mat_pre"]))
            for a in range(5):
                if u["hmask1"] >> a & 1:
                    for v in vecs:
                        _apply_bit(v, nq, tb[rb[a]], H)
            if u["flip_mid"] >= 0:
                g, _ = _flip_index(desc, nq, tb, u["flip_mid"])
                for v in vecs:
                    v[g] *= -1
            for a in range(5):
                if u["hmask2"] >> a & 1:
                    for v in vecs:
                        _apply_bit(v, nq, tb[rb[a]], H)
            if u["mat_post_a"] >= 0:
                for v in vecs:
                    _apply_bit(v, nq, tb[rb[u["mat_post_a"]]], mat(u["mat_post"]))
            if u["mat4"] >= 0:
                for v in vecs:
                    _apply_pair(v, nq, tb[rb[0]], tb[rb[1]], mat.four(u["mat4"]))
            if u["mat4b"] >= 0:
                for v in vecs:
                    _apply_pair(v, nq, tb[rb[2]], tb[rb[3]], mat.four(u["mat4b"]))
            if u["d2b_a"] >= 0:
                bit = tb[rb[u["d2b_a"]]]
                m0 = u["d2b_mat"]
                _apply_bit(vecs[0], nq, bit, mat(m0 + 1))
                d = _param_row(desc, 0, (m0 - 2 * desc["n_static"]) // 5)
                for t in range(3):
                    dpsi = vecs[0].copy()
                    _apply_bit(dpsi, nq, bit, mat(m0 + 2 + t))
                    grads[(d, t)] = 2.0 * u["d2b_gscale"] * float(np.vdot(vecs[1], dpsi).real)
                _apply_bit(vecs[1], nq, bit, mat(m0 + 1))
            if u["d4b_mat"] >= 0:
                b1, b2 = tb[rb[0]], tb[rb[1]]
                m0 = u["d4b_mat"]
                _apply_pair(vecs[0], nq, b1, b2, mat.four(m0 + 1))
                d = _param_row(desc, 1, (m0 - 2 * desc["n_static4"]) // 5)
                for t in range(3):
                    dpsi = vecs[0].copy()
                    _apply_pair(dpsi, nq, b1, b2, mat.four(m0 + 2 + t))
                    grads[(d, t)] = 2.0 * u["d4b_gscale"] * float(np.vdot(vecs[1], dpsi).real)
                _apply_pair(vecs[1], nq, b1, b2, mat.four(m0 + 1))
            if u["scale"]:
                for v in vecs:
                    v *= p["scale"]
            if u["read"] >= 0:
                g, slot = _flip_index(desc, nq, tb, u["read"])
                reads[slot] = abs(vecs[0][g]) ** 2
        vecs = [_store(v, nq, tb, p["store_bits"]) for v in vecs]
    return vecs, reads, grads


def run_forward(problems, desc, inst, psi_in):
    """Returns (psi_out, L) of instance ``inst`` by executing its packed forward schedule,
    after checking that the op-level form gives the same state."""
    psi_ops, L_ops = run_forward_ops(problems, desc, inst, psi_in)
    vecs, reads, _ = _run_subs(problems, desc, inst, "forward", np.array(psi_in, dtype=np.complex128))
    L = sum(reads[s] for s in sorted(reads))
    np.testing.assert_allclose(vecs[0], psi_ops, rtol=0, atol=1e-13)
    assert abs(L - L_ops) <= 1e-14 * max(1.0, abs(L_ops)), (L, L_ops)
    return vecs[0], L


def run_forward_ops(problems, desc, inst, psi_in):
    """Returns (psi_out, L) of instance ``inst`` by executing its forward schedule."""
    mat = _matrix_table(problems, desc)
    info = desc["instances"][inst]
    nq = info["nq"]
    psi = np.array(psi_in, dtype=np.complex128)
    reads = {}
    H = np.array([[1, 1], [1, -1]], dtype=np.complex128)
    for p in info["forward"]:
        check_stage_shapes(nq, p)
        tb = p["tile_bits"]
        for st in p["stages"]:
            for op in st["ops"]:
                kind = op["kind"]
                if kind in ("H", "MAT"):
                    bit = tb[st["rb"][op["a"]]]
                    _apply_bit(psi, nq, bit, H if kind == "H" else mat(op["arg"]))
                elif kind == "MAT4":
                    a = op["a"]
                    _apply_pair(psi, nq, tb[st["rb"][a]], tb[st["rb"][a + 1]], mat.four(op["arg"]))
                elif kind == "PHASE":
                    psi[_phase_mask(nq, op["b1"], op["b2"])] *= complex(op["c"], op["s"])
                elif kind == "FLIP":
                    psi[_global_index(nq, tb, op["tile"], op["j"])] *= -1
                elif kind == "SCALE":
                    psi *= p["scale"]
                elif kind == "READ":
                    g = _global_index(nq, tb, op["tile"], op["j"])
                    reads[op["slot"]] = abs(psi[g]) ** 2
                else:
                    raise AssertionError("unexpected forward op %s" % kind)
        psi = _store(psi, nq, tb, p["store_bits"])
    return psi, sum(reads[s] for s in sorted(reads))


def run_backward(problems, desc, inst, psi_out, dL):
    """Returns (grad_psi_in, grad_angles) from the packed backward schedule, after
    checking it against the op-level form."""
    g_ops, a_ops = run_backward_ops(problems, desc, inst, psi_out, dL)
    psi = np.array(psi_out, dtype=np.complex128)
    vecs, _, grads = _run_subs(problems, desc, inst, "backward", psi, np.zeros_like(psi), dL)
    n_d2 = len({d for d, _ in grads})
    ga = np.zeros((n_d2, 3))
    d0 = min([d for d, _ in grads], default=0)
    for (d, t), v in grads.items():
        ga[d - d0, t] = v
    np.testing.assert_allclose(vecs[1], g_ops, rtol=0, atol=1e-13)
    np.testing.assert_allclose(ga, a_ops, rtol=0, atol=1e-13)
    return vecs[1], ga


def run_backward_ops(problems, desc, inst, psi_out, dL):
    """Returns (grad_psi_in, grad_angles) by executing the backward schedule."""
    mat = _matrix_table(problems, desc)
    info = desc["instances"][inst]
    nq = info["nq"]
    psi = np.array(psi_out, dtype=np.complex128)
    lam = np.zeros_like(psi)
    grads = {}
    H = np.array([[1, 1], [1, -1]], dtype=np.complex128)
    for p in info["backward"]:
        check_stage_shapes(nq, p)
        tb = p["tile_bits"]
        for st in p["stages"]:
            for op in st["ops"]:
                kind = op["kind"]
                if kind in ("H", "MAT"):
                    bit = tb[st["rb"][op["a"]]]
                    M = H if kind == "H" else mat(op["arg"])
                    _apply_bit(psi, nq, bit, M)
                    _apply_bit(lam, nq, bit, M)
                elif kind == "MAT4":
                    b1, b2 = tb[st["rb"][op["a"]]], tb[st["rb"][op["a"] + 1]]
                    _apply_pair(psi, nq, b1, b2, mat.four(op["arg"]))
                    _apply_pair(lam, nq, b1, b2, mat.four(op["arg"]))
                elif kind == "D4BWD":
                    b1, b2 = tb[st["rb"][0]], tb[st["rb"][1]]
                    _apply_pair(psi, nq, b1, b2, mat.four(op["arg"] + 1))
                    d = _param_row(desc, 1, (op["arg"] - 2 * desc["n_static4"]) // 5)
                    for t in range(3):
                        dpsi = psi.copy()
                        _apply_pair(dpsi, nq, b1, b2, mat.four(op["arg"] + 2 + t))
                        grads[(d, t)] = 2.0 * op["gscale"] * float(np.vdot(lam, dpsi).real)
                    _apply_pair(lam, nq, b1, b2, mat.four(op["arg"] + 1))
                elif kind == "PHASE":
                    m = _phase_mask(nq, op["b1"], op["b2"])
                    psi[m] *= complex(op["c"], op["s"])
                    lam[m] *= complex(op["c"], op["s"])
                elif kind == "FLIP":
                    g = _global_index(nq, tb, op["tile"], op["j"])
                    psi[g] *= -1
                    lam[g] *= -1
                elif kind == "SCALE":
                    psi *= p["scale"]
                    lam *= p["scale"]
                elif kind == "SEED":
                    g = _global_index(nq, tb, op["tile"], op["j"])
                    lam[g] = dL * psi[g]
                elif kind == "D2BWD":
                    bit = tb[st["rb"][op["a"]]]
                    _apply_bit(psi, nq, bit, mat(op["arg"] + 1))
                    for t in range(3):
                        dpsi = psi.copy()
                        _apply_bit(dpsi, nq, bit, mat(op["arg"] + 2 + t))
                        d = _param_row(desc, 0, (op["arg"] - 2 * desc["n_static"]) // 5)
                        grads[(d, t)] = 2.0 * op["gscale"] * float(np.vdot(lam, dpsi).real)
                    _apply_bit(lam, nq, bit, mat(op["arg"] + 1))
                else:
                    raise AssertionError("unexpected backward op %s" % kind)
        psi = _store(psi, nq, tb, p["store_bits"])
        lam = _store(lam, nq, tb, p["store_bits"])
    n_d2 = len({d for d, _ in grads})
    ga = np.zeros((n_d2, 3))
    d0 = min([d for d, _ in grads], default=0)
    for (d, t), v in grads.items():
        ga[d - d0, t] = v
    return lam, ga
