"""Python binding of libpaperkern: argument marshalling only.

Every step of the computation runs in the HIP library; this module converts
gate lists to ``pk_gate`` structs, passes torch device pointers and the current
HIP stream across the C-ABI, and maps error codes to exceptions.  It raises
when the library is missing: there is no fallback.

Gate tuples (applied left to right):
    ("H", i_s), ("ONEOP", i_s, op2x2), ("HALL",), ("ORACLE",), ("INV",),
    ("D2", i_s, alpha, beta, gamma)
"""

import ctypes
import json
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpaperkern.so")

PK_OK, PK_EINVAL, PK_ENOMEM, PK_EDEVICE, PK_EUNSUPPORTED = 0, -1, -2, -3, -4
PK_FP64, PK_FP32 = 0, 1
PK_OP_EVAL, PK_OP_BACKWARD = 0, 1
GATE_KINDS = {"ONEOP": 0, "H": 1, "HALL": 2, "ORACLE": 3, "INV": 4, "D2": 5,
              "TWOOP": 6, "CNOT": 7, "CPHASE": 8, "CPHASEK": 9, "SWAP": 10, "D4": 11, "QFT": 12, "QFT_NOSWAP": 13}
TWO_QUBIT = ("TWOOP", "CNOT", "CPHASE", "CPHASEK", "SWAP", "D4")

# Entry points declared in include/paperkern.h with their ctypes signatures.
_c_int32, _c_int64, _c_double, _vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p


class PkGate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("is1", ctypes.c_int32), ("is2", ctypes.c_int32),
                ("k", ctypes.c_int32), ("op", ctypes.c_double * 32), ("angle", ctypes.c_double * 3)]


class PkProblem(ctypes.Structure):
    _fields_ = [("nq", ctypes.c_int32), ("n_gates", ctypes.c_int32), ("gates", ctypes.POINTER(PkGate)),
                ("n_marked", ctypes.c_int64), ("marked", ctypes.POINTER(ctypes.c_int64))]


SIGNATURES = {
    "pk_create": (ctypes.c_int, [ctypes.POINTER(PkProblem), _c_int32, _c_int32, ctypes.POINTER(_vp)]),
    "pk_set_tiling": (ctypes.c_int, [_vp, _c_int32, _c_int32, _c_int32, _c_int32, _c_int32]),
    "pk_set_batch": (ctypes.c_int, [_vp, _c_int32, _c_int32]),
    "pk_batch_teams": (ctypes.c_int, [_vp, ctypes.POINTER(_c_int32), ctypes.POINTER(_c_int32)]),
    "pk_set_launch": (ctypes.c_int, [_vp, _c_int32, _c_int32]),
    "pk_plan_passes": (ctypes.c_int, [_vp, _c_int32, ctypes.POINTER(_c_int32)]),
    "pk_plan_describe": (ctypes.c_int, [_vp, ctypes.c_char_p, _c_int64, ctypes.POINTER(_c_int64)]),
    "pk_plan_offsets": (ctypes.c_int, [_vp, ctypes.POINTER(_c_int64)]),
    "pk_plan_n_angles": (ctypes.c_int, [_vp, ctypes.POINTER(_c_int64)]),
    "pk_workspace_bytes": (ctypes.c_int, [_vp, _c_int32, ctypes.POINTER(_c_int64)]),
    "pk_evaluate": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "pk_evaluate_batched": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "pk_evaluate_repeat": (ctypes.c_int, [_vp, _c_int64, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "pk_repeat_launches": (ctypes.c_int, [_vp, _c_int64, ctypes.POINTER(_c_int64)]),
    "pk_set_pass_walk": (ctypes.c_int, [_vp, _c_int32, ctypes.POINTER(_c_int32)]),
    "pk_set_lane_maps": (ctypes.c_int, [_vp, _c_int32]),
    "pk_set_pass_overlap": (ctypes.c_int, [_vp, _c_int32, ctypes.POINTER(_c_int32)]),
    "pk_evaluate_static": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "pk_backward": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "pk_pair_indices": (ctypes.c_int, [_c_int32, _c_int32, _c_int64, _c_int64, _vp, _vp, _vp]),
    "pk_shor_state": (ctypes.c_int, [_c_int32, _c_int32, _c_int64, _c_int64, _c_int32, _vp, _vp]),
    "pk_marginal": (ctypes.c_int, [_c_int32, _c_int32, _c_int32, _vp, _vp, _vp]),
    "pk_marginal_bitrev": (ctypes.c_int, [_c_int32, _c_int32, _c_int32, _vp, _vp, _vp]),
    "pk_density_matrix": (ctypes.c_int, [_c_int32, _c_int32, _vp, _vp, _vp, _vp]),
    "pk_search_diffusion": (ctypes.c_int, [_c_int32, _c_int32, _vp, _c_int32, _c_int64, _vp, _vp, _vp, _vp, _vp]),
    "pk_search_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(_c_int64)]),
    "pk_density_spectrum": (ctypes.c_int, [_c_int32, _vp, _vp, _vp, _vp]),
    "pk_time_passes": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(_c_double),
                                      _c_int32, ctypes.POINTER(_c_int32)]),
    "pk_destroy": (None, [_vp]),
    "pk_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "pk_last_error": (ctypes.c_char_p, [_vp]),
}

_lib = None


class PaperkernError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_lib.pk_strerror(code).decode() if _lib else "error", code, msg))
        self.code = code


def lib():
    """Load libpaperkern.so (built in-tree by ``paper_0902_0699_amd.build``); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libpaperkern.so is not built (%s); run paper_0902_0699_amd/build.py" % LIB_PATH)
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def _check(rc, plan_handle=None):
    if rc != PK_OK:
        msg = lib().pk_last_error(plan_handle).decode()
        raise PaperkernError(rc, msg)


def make_gate(g, nq=None):
    """Convert one gate tuple to a PkGate."""
    pg = PkGate()
    kind = g[0]
    if kind not in GATE_KINDS:
        raise ValueError("unknown gate kind %r" % (kind,))
    pg.kind = GATE_KINDS[kind]
    if kind in ("H", "ONEOP", "D2") or kind in TWO_QUBIT:
        pg.is1 = int(g[1])
    if kind in TWO_QUBIT:
        pg.is2 = int(g[2])
    if kind == "ONEOP":
        op = np.asarray(g[2], dtype=np.complex128).reshape(2, 2)
        for a in range(2):
            for b in range(2):
                pg.op[2 * (2 * a + b)] = op[a, b].real
                pg.op[2 * (2 * a + b) + 1] = op[a, b].imag
    if kind == "TWOOP":
        op = np.asarray(g[3], dtype=np.complex128).reshape(4, 4)
        for a in range(4):
            for b in range(4):
                pg.op[2 * (4 * a + b)] = op[a, b].real
                pg.op[2 * (4 * a + b) + 1] = op[a, b].imag
    if kind == "CPHASEK":
        pg.k = int(g[3])
    if kind in ("QFT", "QFT_NOSWAP"):  # (kind, first qubit, register size)
        pg.is1 = int(g[1])
        pg.k = int(g[2])
    if kind in ("D2", "D4"):
        first = 2 if kind == "D2" else 3
        for t in range(3):
            pg.angle[t] = float(g[first + t])
    return pg


class Plan:
    """A compiled gate schedule for one or more instances (C-ABI ``pk_plan``)."""

    def __init__(self, problems, prec="fp64"):
        if isinstance(problems, dict):
            problems = [problems]
        self.prec = {"fp64": PK_FP64, "fp32": PK_FP32}[prec]
        self.problems = problems
        keep = []
        arr = (PkProblem * len(problems))()
        for i, p in enumerate(problems):
            gates = (PkGate * max(1, len(p["gates"])))(*[make_gate(g) for g in p["gates"]])
            marked = (ctypes.c_int64 * max(1, len(p["marked"])))(*[int(x) for x in p["marked"]])
            keep += [gates, marked]
            arr[i].nq = int(p["nq"])
            arr[i].n_gates = len(p["gates"])
            arr[i].gates = ctypes.cast(gates, ctypes.POINTER(PkGate))
            arr[i].n_marked = len(p["marked"])
            arr[i].marked = ctypes.cast(marked, ctypes.POINTER(ctypes.c_int64))
        h = ctypes.c_void_p()
        _check(lib().pk_create(arr, len(problems), self.prec, ctypes.byref(h)))
        self.handle = h
        self._ws = {}

    def close(self):
        if getattr(self, "handle", None):
            lib().pk_destroy(self.handle)
            self.handle = None
            self._ws = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- host queries -----------------------------------------------------------------
    @property
    def n_inst(self):
        return len(self.problems)

    def set_tiling(self, tile_bits, carrier_bits=4, fuse=1, lane_order=1, page_cap=-1):
        _check(lib().pk_set_tiling(self.handle, tile_bits, carrier_bits, fuse, lane_order, page_cap), self.handle)
        self._ws = {}

    def set_batch(self, team_size=16, min_team_tiles=64):
        _check(lib().pk_set_batch(self.handle, team_size, min_team_tiles), self.handle)
        self._ws = {}

    def batch_teams(self):
        """(teams, instances run by teams) of the batched launch on the current device."""
        t, n = _c_int32(), _c_int32()
        _check(lib().pk_batch_teams(self.handle, ctypes.byref(t), ctypes.byref(n)), self.handle)
        return t.value, n.value

    def set_launch(self, wgs_per_cu=0, reg_bits=0):
        _check(lib().pk_set_launch(self.handle, wgs_per_cu, reg_bits), self.handle)
        self._ws = {}

    def set_pass_walk(self, walk):
        """Per forward pass: 0 strided over the grid, c > 1 runs of c consecutive
        tiles, -1 one contiguous block per workgroup; an empty list resets."""
        walk = [int(c) for c in walk]
        arr = (_c_int32 * max(1, len(walk)))(*walk)
        _check(lib().pk_set_pass_walk(self.handle, len(walk), arr), self.handle)
        self._ws = {}

    def set_pass_overlap(self, on):
        """Per forward pass: 1 keeps the next tile's loads in flight through the LDS
        exchanges (FP64 kernels with 4 register bits, full tiles); an empty list resets."""
        on = [int(c) for c in on]
        arr = (_c_int32 * max(1, len(on)))(*on)
        _check(lib().pk_set_pass_overlap(self.handle, len(on), arr), self.handle)
        self._ws = {}

    def set_lane_maps(self, on):
        """1: bank-spreading thread maps for the LDS-only stage layouts (default); 0: off."""
        _check(lib().pk_set_lane_maps(self.handle, int(on)), self.handle)
        self._ws = {}

    def passes(self, inst=0):
        n = ctypes.c_int32()
        _check(lib().pk_plan_passes(self.handle, inst, ctypes.byref(n)), self.handle)
        return n.value

    def describe(self):
        need = ctypes.c_int64()
        _check(lib().pk_plan_describe(self.handle, None, 0, ctypes.byref(need)), self.handle)
        buf = ctypes.create_string_buffer(need.value)
        _check(lib().pk_plan_describe(self.handle, buf, need.value, ctypes.byref(need)), self.handle)
        return json.loads(buf.value.decode())

    def offsets(self):
        out = (ctypes.c_int64 * (self.n_inst + 1))()
        _check(lib().pk_plan_offsets(self.handle, out), self.handle)
        return list(out)

    def n_angles(self):
        n = ctypes.c_int64()
        _check(lib().pk_plan_n_angles(self.handle, ctypes.byref(n)), self.handle)
        return n.value

    def workspace_bytes(self, op=PK_OP_EVAL):
        n = ctypes.c_int64()
        _check(lib().pk_workspace_bytes(self.handle, op, ctypes.byref(n)), self.handle)
        return n.value

    # ---- device calls ---------------------------------------------------------------------
    def workspace(self, op, device):
        import torch
        key = (op, str(device))
        if key not in self._ws:
            nbytes = self.workspace_bytes(op)
            self._ws[key] = torch.empty(nbytes, dtype=torch.uint8, device=device)
        return self._ws[key]

    @property
    def complex_dtype(self):
        import torch
        return torch.complex128 if self.prec == PK_FP64 else torch.complex64


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_state(plan, t, nelem, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if t.dtype != plan.complex_dtype or not t.is_contiguous() or t.numel() != nelem:
        raise ValueError("%s must be a contiguous %s tensor of %d elements" % (name, plan.complex_dtype, nelem))


def _check_f64(t, n, name, device):
    import torch
    if t is None:
        return
    if (not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_contiguous()
            or t.numel() < n or t.device != device):
        raise ValueError("%s must be a contiguous float64 tensor of >= %d elements on %s" % (name, n, device))


def evaluate_into(plan, psi_in, psi_out, L_out, norm_out=None, angles=None):
    """pk_evaluate on preallocated device tensors (L_out, norm_out: float64 [1])."""
    nelem = plan.offsets()[-1]
    _check_f64(L_out, 1, "L_out", psi_in.device)
    _check_f64(norm_out, 1, "norm_out", psi_in.device)
    _check_f64(angles, 3 * plan.n_angles(), "angles", psi_in.device)
    _check_state(plan, psi_in, nelem, "psi_in")
    _check_state(plan, psi_out, nelem, "psi_out")
    ws = plan.workspace(PK_OP_EVAL, psi_in.device)
    rc = lib().pk_evaluate(plan.handle, _ptr(psi_in), _ptr(psi_out), _ptr(L_out), _ptr(norm_out), _ptr(angles),
                           _ptr(ws), _stream(psi_in.device))
    _check(rc, plan.handle)


def evaluate_static(plan, psi_in, psi_out, L_out, norm_out=None, angles=None):
    """pk_evaluate_static: pk_evaluate with the library's static workspace, on
    preallocated device tensors; allocates nothing (the plan's tables must already
    be on the device, e.g. after one ``evaluate``)."""
    nelem = plan.offsets()[-1]
    _check_f64(L_out, 1, "L_out", psi_in.device)
    _check_f64(norm_out, 1, "norm_out", psi_in.device)
    _check_f64(angles, 3 * plan.n_angles(), "angles", psi_in.device)
    _check_state(plan, psi_in, nelem, "psi_in")
    _check_state(plan, psi_out, nelem, "psi_out")
    rc = lib().pk_evaluate_static(plan.handle, _ptr(psi_in), _ptr(psi_out), _ptr(L_out), _ptr(norm_out),
                                  _ptr(angles), _stream(psi_in.device))
    _check(rc, plan.handle)


def evaluate(plan, psi_in, angles=None, want_norm=True, out=None):
    """Apply a single-instance plan: returns (psi_out, L, norm) as device tensors."""
    import torch
    dev = psi_in.device
    psi_out = torch.empty_like(psi_in) if out is None else out
    L = torch.empty(1, dtype=torch.float64, device=dev)
    norm = torch.empty(1, dtype=torch.float64, device=dev) if want_norm else None
    evaluate_into(plan, psi_in, psi_out, L, norm, angles)
    return psi_out, L, norm


def evaluate_repeat(plan, psi_in, reps, angles=None, want_norm=True, out=None):
    """U^reps psi_in for a single-instance plan (pk_evaluate_repeat): (psi_out, L, norm)."""
    import torch
    dev = psi_in.device
    psi_out = torch.empty_like(psi_in) if out is None else out
    nelem = plan.offsets()[-1]
    _check_state(plan, psi_in, nelem, "psi_in")
    _check_state(plan, psi_out, nelem, "psi_out")
    _check_f64(angles, 3 * plan.n_angles(), "angles", dev)
    L = torch.empty(1, dtype=torch.float64, device=dev)
    norm = torch.empty(1, dtype=torch.float64, device=dev) if want_norm else None
    ws = plan.workspace(PK_OP_EVAL, dev)
    rc = lib().pk_evaluate_repeat(plan.handle, int(reps), _ptr(psi_in), _ptr(psi_out), _ptr(L), _ptr(norm),
                                  _ptr(angles), _ptr(ws), _stream(dev))
    _check(rc, plan.handle)
    return psi_out, L, norm


def repeat_launches(plan, reps):
    """Pass launches of evaluate_repeat(plan, ..., reps) (pk_repeat_launches)."""
    n = ctypes.c_int64()
    _check(lib().pk_repeat_launches(plan.handle, int(reps), ctypes.byref(n)), plan.handle)
    return n.value


def search_diffusion(nq, marked, iterations, psi_in, out=None, workspace=None):
    """The noise-free search through 2|s><s| - I (pk_search_diffusion, a labelled
    variant of the HALL-based iteration): returns (psi_out, L)."""
    import torch
    dev = psi_in.device
    if psi_in.dtype not in (torch.complex128, torch.complex64) or psi_in.numel() != (1 << nq):
        raise ValueError("psi_in must hold 2^nq complex amplitudes")
    prec = PK_FP64 if psi_in.dtype == torch.complex128 else PK_FP32
    psi_out = torch.empty_like(psi_in) if out is None else out
    L = torch.empty(1, dtype=torch.float64, device=dev)
    if workspace is None:
        nb = ctypes.c_int64()
        _check(lib().pk_search_workspace_bytes(ctypes.byref(nb)), None)
        workspace = torch.empty(nb.value, dtype=torch.uint8, device=dev)
    labels = (ctypes.c_int64 * max(1, len(marked)))(*[int(v) for v in marked])
    rc = lib().pk_search_diffusion(nq, prec, labels, len(marked), int(iterations), _ptr(psi_in), _ptr(psi_out),
                                   _ptr(L), _ptr(workspace), _stream(dev))
    _check(rc, None)
    return psi_out, L


def grover_iterations(nq):
    """n_t = floor((pi/4) sqrt(2^nq)), the iteration count of Sec. 5.1 (reading: floor)."""
    return int(math.floor(math.pi / 4.0 * math.sqrt(float(1 << nq))))


def evaluate_batched(plan, psi_in, angles=None, want_norm=True, out=None):
    """All instances in one persistent launch; states packed at plan.offsets()."""
    import torch
    nelem = plan.offsets()[-1]
    _check_state(plan, psi_in, nelem, "psi_in")
    dev = psi_in.device
    psi_out = torch.empty_like(psi_in) if out is None else out
    _check_state(plan, psi_out, nelem, "psi_out")
    L = torch.empty(plan.n_inst, dtype=torch.float64, device=dev)
    norm = torch.empty(plan.n_inst, dtype=torch.float64, device=dev) if want_norm else None
    _check_f64(angles, 3 * plan.n_angles(), "angles", dev)
    ws = plan.workspace(PK_OP_EVAL, dev)
    rc = lib().pk_evaluate_batched(plan.handle, _ptr(psi_in), _ptr(psi_out), _ptr(L), _ptr(norm), _ptr(angles),
                                   _ptr(ws), _stream(dev))
    _check(rc, plan.handle)
    return psi_out, L, norm


def backward(plan, psi_out, dL, angles=None):
    """pk_backward: returns (grad_psi_in, grad_angles) for the scalar sum dL * L."""
    import torch
    nelem = plan.offsets()[-1]
    _check_state(plan, psi_out, nelem, "psi_out")
    dev = psi_out.device
    _check_f64(dL, plan.n_inst, "dL", dev)
    _check_f64(angles, 3 * plan.n_angles(), "angles", dev)
    grad_psi = torch.empty_like(psi_out)
    n_d2 = plan.n_angles()
    grad_ang = torch.zeros(max(1, 3 * n_d2), dtype=torch.float64, device=dev)
    ws = plan.workspace(PK_OP_BACKWARD, dev)
    rc = lib().pk_backward(plan.handle, _ptr(psi_out), _ptr(dL), _ptr(grad_psi), _ptr(grad_ang) if n_d2 else None,
                           _ptr(angles), _ptr(ws), _stream(dev))
    _check(rc, plan.handle)
    return grad_psi, grad_ang[:3 * n_d2]


def time_passes(plan, psi_in, psi_out, angles=None):
    """Per-pass kernel durations (ms) of one evaluation, from HIP events on the current stream."""
    import torch
    dev = psi_in.device
    nelem = plan.offsets()[-1]
    _check_state(plan, psi_in, nelem, "psi_in")
    _check_state(plan, psi_out, nelem, "psi_out")
    _check_f64(angles, 3 * plan.n_angles(), "angles", dev)
    L = torch.empty(1, dtype=torch.float64, device=dev)
    ws = plan.workspace(PK_OP_EVAL, dev)
    ms = (ctypes.c_double * 64)()
    n = ctypes.c_int32()
    rc = lib().pk_time_passes(plan.handle, _ptr(psi_in), _ptr(psi_out), _ptr(L), _ptr(angles), _ptr(ws),
                              _stream(dev), ms, 64, ctypes.byref(n))
    _check(rc, plan.handle)
    return [ms[i] for i in range(n.value)]


def pair_indices(nq, i_s, first, count, device="cuda"):
    """Device kernel output of the partner pairs (n0, n1) of qubit i_s."""
    import torch
    n0 = torch.empty(max(1, count), dtype=torch.int64, device=device)
    n1 = torch.empty(max(1, count), dtype=torch.int64, device=device)
    rc = lib().pk_pair_indices(nq, i_s, first, count, _ptr(n0), _ptr(n1), _stream(n0.device))
    _check(rc, None)
    return n0[:count], n1[:count]


def shor_register_sizes(M):
    """(n1, n2) of Shor's Step 1: n1 = Ceiling(log2 Q), Q = 2^Ceiling(log2 M^2); n2 = Ceiling(log2 M)."""
    M = int(M)
    if M < 2:
        raise ValueError("M must be at least 2")
    n1 = ((M * M) - 1).bit_length()  # Ceiling(log2 Q) = Ceiling(log2 M^2)
    return n1, (M - 1).bit_length()


def shor_state(n1, n2, xguess, M, prec="fp64", out=None, device="cuda"):
    """The loaded two-register state of Eq. Shor2 on the device (pk_shor_state)."""
    import torch
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    if out is None:
        # sizes the library rejects get a one-element buffer: the C-ABI reports the error
        ok = n1 >= 1 and n2 >= 1 and n1 + n2 <= (30 if prec == "fp64" else 31)
        out = torch.empty((1 << (n1 + n2)) if ok else 1, dtype=dt, device=device)
    elif out.dtype != dt or out.numel() != (1 << (n1 + n2)) or not out.is_contiguous():
        raise ValueError("out must be a contiguous %s tensor of 2^(n1+n2) amplitudes" % dt)
    rc = lib().pk_shor_state(n1, n2, int(xguess), int(M), PK_FP64 if prec == "fp64" else PK_FP32, _ptr(out),
                             _stream(out.device))
    _check(rc, None)
    return out


def marginal(psi, nq, n_low, out=None, bitrev=False):
    """p[n] = sum over the n_low low qubits of |psi|^2 (pk_marginal), FP64 on the device;
    with ``bitrev`` the high register is read in reversed qubit order (pk_marginal_bitrev)."""
    import torch
    if psi.dtype not in (torch.complex128, torch.complex64) or psi.numel() != (1 << nq) or not psi.is_contiguous():
        raise ValueError("psi must be a contiguous complex tensor of 2^nq amplitudes")
    if out is None:
        out = torch.empty(1 << (nq - n_low) if 0 <= n_low <= nq else 1, dtype=torch.float64, device=psi.device)
    prec = PK_FP64 if psi.dtype == torch.complex128 else PK_FP32
    fn = lib().pk_marginal_bitrev if bitrev else lib().pk_marginal
    rc = fn(nq, n_low, prec, _ptr(psi), _ptr(out), _stream(psi.device))
    _check(rc, None)
    return out


def density_matrix(states, weights, out=None):
    """rho = sum_a P_a C_a C_a^H (pk_density_matrix): ``states`` a contiguous complex128
    device tensor of shape (A, 2^nq) or the packed 1-D batch, ``weights`` float64 (A,)."""
    import torch
    A = int(weights.numel())
    if states.dtype != torch.complex128 or not states.is_contiguous() or states.numel() % max(A, 1):
        raise ValueError("states must be contiguous complex128 holding A states of equal size")
    N = states.numel() // max(A, 1)
    nq = N.bit_length() - 1
    if N != 1 << nq:
        raise ValueError("each state must hold 2^nq amplitudes")
    _check_f64(weights, A, "weights", states.device)
    if out is None:
        out = torch.empty((N, N), dtype=torch.complex128, device=states.device)
    elif out.dtype != torch.complex128 or out.numel() != N * N or not out.is_contiguous():
        raise ValueError("out must be a contiguous complex128 tensor of N * N entries")
    rc = lib().pk_density_matrix(nq, A, _ptr(states), _ptr(weights), _ptr(out), _stream(states.device))
    _check(rc, None)
    return out


def density_spectrum(rho):
    """Eigenvalues (ascending), entropy in bits and Tr rho^2 of a Hermitian rho
    (pk_density_spectrum).  rho is overwritten."""
    import torch
    N = rho.shape[0]
    nq = N.bit_length() - 1
    if rho.dtype != torch.complex128 or rho.numel() != N * N or N != 1 << nq or not rho.is_contiguous():
        raise ValueError("rho must be a contiguous complex128 N x N tensor, N = 2^nq")
    lam = torch.empty(N, dtype=torch.float64, device=rho.device)
    sums = torch.empty(2, dtype=torch.float64, device=rho.device)
    rc = lib().pk_density_spectrum(nq, _ptr(rho), _ptr(lam), _ptr(sums), _stream(rho.device))
    _check(rc, None)
    return lam, sums[0], sums[1]


def _autograd_function():
    import torch

    class GroverEval(torch.autograd.Function):
        """L = sum_{x in M} |(U psi_in)_x|^2 with gradients by the library's adjoint kernel.

        The real-pair gradient dL/dRe + i dL/dIm that pk_backward returns is what
        torch expects for a real output of a complex input, so it is passed through.
        """

        @staticmethod
        def forward(ctx, psi_in, angles, plan):
            psi_out, L, _ = evaluate(plan, psi_in.detach().contiguous(),
                                     angles=angles.detach().contiguous() if angles is not None else None,
                                     want_norm=False)
            ctx.plan = plan
            ctx.save_for_backward(psi_out, angles if angles is not None else torch.empty(0))
            ctx.has_angles = angles is not None
            return L[0], psi_out

        @staticmethod
        def backward(ctx, dL, dpsi_out):
            if dpsi_out is not None and bool(torch.any(dpsi_out != 0)):
                raise NotImplementedError("gradients flow from L only; psi_out is returned for inspection")
            psi_out, angles = ctx.saved_tensors
            dl = dL.detach().reshape(1).to(torch.float64).contiguous()
            gpsi, gang = backward(ctx.plan, psi_out, dl, angles=angles if ctx.has_angles else None)
            return gpsi, (gang if ctx.has_angles else None), None

    return GroverEval


_GROVER_EVAL = None


def grover_eval(plan, psi_in, angles=None):
    """Differentiable evaluation: returns (L, psi_out); L.backward() runs pk_backward."""
    global _GROVER_EVAL
    if _GROVER_EVAL is None:
        _GROVER_EVAL = _autograd_function()
    return _GROVER_EVAL.apply(psi_in, angles, plan)
