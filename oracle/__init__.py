"""CPU oracle for the state-vector hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never loads it, and
it shares no code with the HIP path: the complex128 arithmetic lives in
``sv_oracle.c`` (plain loops written from the definitions), the brute-force
pin in :mod:`oracle.brute` (full 2^n x 2^n Kronecker products), the qubit
reordering oracle is a ``numpy.transpose`` of the state tensor, and the
schedules are written from the paper's algorithms in :mod:`oracle.schedule`.

Parity status: every function here is pinned by a ``-m "not gpu"`` test
(brute force, closed forms, invariants, worked examples) except where
:mod:`oracle.schedule` says "parity unpinned".
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "sv_oracle.c")

# Gate kind codes of sv_oracle.c (the oracle's own numbering).
KIND_CODE = {"H": 0, "X": 1, "Y": 2, "Z": 3, "S": 4, "T": 5, "RX": 6, "RY": 7, "RZ": 8,
             "CNOT": 9, "CZ": 10, "CPHASE": 11, "GIVENS": 12, "SWAP": 13, "U1": 14, "U2": 15}
PARAM_KINDS = ("RX", "RY", "RZ", "CPHASE", "GIVENS")


def build(force: bool = True) -> str:
    """Compile sv_oracle.c into liboracle.so (gcc, OpenMP)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        up = ctypes.POINTER(ctypes.c_uint64)
        L.orc_apply_gate.argtypes = [dp, ctypes.c_int, ctypes.c_int, ip, ctypes.c_double, dp, ctypes.c_int]
        L.orc_apply_gate.restype = ctypes.c_int
        L.orc_apply_circuit.argtypes = [dp, ctypes.c_int, ctypes.c_int, ip, ip, dp, dp]
        L.orc_apply_circuit.restype = ctypes.c_int
        L.orc_apply_generator.argtypes = [dp, ctypes.c_int, ctypes.c_int, ip]
        L.orc_apply_generator.restype = ctypes.c_int
        L.orc_pauli_apply.argtypes = [dp, dp, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64]
        L.orc_pauli_apply.restype = None
        L.orc_expectation.argtypes = [dp, ctypes.c_int, ctypes.c_int, up, up, dp, ctypes.c_int,
                                      ip, dp, dp]
        L.orc_expectation.restype = ctypes.c_double
        L.orc_hpsi.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, up, up, dp]
        L.orc_hpsi.restype = None
        L.orc_adjoint_grad.argtypes = [dp, ctypes.c_int, ctypes.c_int, ip, ip, dp, dp, ip, dp,
                                       ctypes.c_int, ctypes.c_int, up, up, dp, dp, dp]
        L.orc_adjoint_grad.restype = ctypes.c_int
        L.orc_threads.argtypes = []
        L.orc_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _up(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _gate_arrays(gates, theta):
    """Gate tuples -> C arrays (kinds, qs[m*2], angles, params, scales, umats).

    A gate is (kind, qubits, param[, extra[, scale]]): with param >= 0 its
    angle is scale * theta[param] + extra (extra defaults to 0, scale to 1);
    with param = -1 the angle is extra (U1/U2: extra is the matrix)."""
    m = len(gates)
    kinds = np.zeros(m, dtype=np.int32)
    qs = np.zeros(2 * m, dtype=np.int32)
    ang = np.zeros(m, dtype=np.float64)
    par = np.full(m, -1, dtype=np.int32)
    scl = np.ones(m, dtype=np.float64)
    um = None
    for i, gt in enumerate(gates):
        kind, qub, p = gt[0], gt[1], gt[2]
        kinds[i] = KIND_CODE[kind]
        qs[2 * i] = qub[0]
        qs[2 * i + 1] = qub[1] if len(qub) > 1 else 0
        if kind in ("U1", "U2"):
            if um is None:
                um = np.zeros(32 * max(1, m), dtype=np.float64)
            mat = np.asarray(gt[3], dtype=np.complex128).reshape(-1)
            um[32 * i:32 * i + 2 * mat.size] = mat.view(np.float64)
        elif p is not None and p >= 0:
            off = float(gt[3]) if len(gt) > 3 else 0.0
            scl[i] = float(gt[4]) if len(gt) > 4 else 1.0
            ang[i] = scl[i] * theta[p] + off
            par[i] = p
        elif len(gt) > 3:
            ang[i] = gt[3]
    return kinds, qs, ang, par, scl, um


def basis_state(n: int, index: int) -> np.ndarray:
    v = np.zeros(1 << n, dtype=np.complex128)
    v[index] = 1.0
    return v


def apply_gate(psi: np.ndarray, kind: str, qubits, angle: float = 0.0, umat=None,
               dagger: bool = False) -> np.ndarray:
    psi = np.ascontiguousarray(psi, dtype=np.complex128).copy()
    n = int(psi.shape[0]).bit_length() - 1
    q = np.array(list(qubits) + [0] * (2 - len(qubits)), dtype=np.int32)
    um = np.zeros(32) if umat is None else np.ascontiguousarray(
        np.asarray(umat, dtype=np.complex128).reshape(-1).view(np.float64))
    rc = lib().orc_apply_gate(_dp(psi.view(np.float64)), n, KIND_CODE[kind], _ip(q),
                              float(angle), _dp(um), int(dagger))
    if rc:
        raise ValueError(kind)
    return psi


def apply_circuit(psi: np.ndarray, gates, theta) -> np.ndarray:
    """U_{m-1}...U_0 psi in the given gate order (eq. update_sv_gate)."""
    psi = np.ascontiguousarray(psi, dtype=np.complex128).copy()
    n = int(psi.shape[0]).bit_length() - 1
    kinds, qs, ang, _, _, um = _gate_arrays(gates, theta)
    rc = lib().orc_apply_circuit(_dp(psi.view(np.float64)), n, len(gates), _ip(kinds), _ip(qs),
                                 _dp(ang), _dp(um) if um is not None else None)
    if rc:
        raise ValueError("bad gate")
    return psi


def apply_circuit_inplace(psi: np.ndarray, gates, theta) -> None:
    """Like :func:`apply_circuit` but updates ``psi`` (complex128, contiguous)
    in place; used to time the oracle without a full-state copy."""
    n = int(psi.shape[0]).bit_length() - 1
    kinds, qs, ang, _, _, um = _gate_arrays(gates, theta)
    rc = lib().orc_apply_circuit(_dp(psi.view(np.float64)), n, len(gates), _ip(kinds), _ip(qs),
                                 _dp(ang), _dp(um) if um is not None else None)
    if rc:
        raise ValueError("bad gate")


def threads() -> int:
    """OpenMP threads the oracle runs with."""
    return int(lib().orc_threads())


def run_circuit(circ) -> np.ndarray:
    """psi = U(theta)|psi0> for a :class:`workloads.Circuit`."""
    return apply_circuit(basis_state(circ.n, circ.psi0_index), circ.gates, circ.theta)


def apply_generator(psi, kind, qubits):
    psi = np.ascontiguousarray(psi, dtype=np.complex128).copy()
    n = int(psi.shape[0]).bit_length() - 1
    q = np.array(list(qubits) + [0] * (2 - len(qubits)), dtype=np.int32)
    if lib().orc_apply_generator(_dp(psi.view(np.float64)), n, KIND_CODE[kind], _ip(q)):
        raise ValueError(kind)
    return psi


def pauli_apply(psi, x: int, z: int) -> np.ndarray:
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    n = int(psi.shape[0]).bit_length() - 1
    out = np.empty_like(psi)
    lib().orc_pauli_apply(_dp(out.view(np.float64)), _dp(psi.view(np.float64)), n,
                          int(x), int(z))
    return out


def expectation(psi, ham, g: int = 0, pos=None, with_chunks: bool = False,
                with_imag: bool = False):
    """E = sum_t a_t <psi|P_t|psi> (eq. evc); optional per-chunk sums (eq. local_evc)."""
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    n = int(psi.shape[0]).bit_length() - 1
    x = np.ascontiguousarray(ham.x, dtype=np.uint64)
    z = np.ascontiguousarray(ham.z, dtype=np.uint64)
    a = np.ascontiguousarray(ham.coef, dtype=np.float64)
    chunks = np.zeros(1 << g, dtype=np.float64) if with_chunks else None
    p = None if pos is None else np.ascontiguousarray(pos, dtype=np.int32)
    im = np.zeros(1, dtype=np.float64)
    e = lib().orc_expectation(_dp(psi.view(np.float64)), n, len(a), _up(x), _up(z), _dp(a), g,
                              _ip(p) if p is not None else None,
                              _dp(chunks) if chunks is not None else None, _dp(im))
    out = [e]
    if with_chunks:
        out.append(chunks)
    if with_imag:
        out.append(float(im[0]))
    return out[0] if len(out) == 1 else tuple(out)


def hpsi(psi, ham) -> np.ndarray:
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    n = int(psi.shape[0]).bit_length() - 1
    out = np.empty_like(psi)
    lib().orc_hpsi(_dp(out.view(np.float64)), _dp(psi.view(np.float64)), n, len(ham.coef),
                   _up(np.ascontiguousarray(ham.x, dtype=np.uint64)),
                   _up(np.ascontiguousarray(ham.z, dtype=np.uint64)),
                   _dp(np.ascontiguousarray(ham.coef, dtype=np.float64)))
    return out


def energy(circ, ham, theta=None) -> float:
    th = circ.theta if theta is None else theta
    psi = apply_circuit(basis_state(circ.n, circ.psi0_index), circ.gates, th)
    return expectation(psi, ham)


def adjoint_grad(circ, ham, theta=None):
    """(E, dE/dtheta) by the adjoint recursion (sv_oracle.c: orc_adjoint_grad)."""
    th = np.ascontiguousarray(circ.theta if theta is None else theta, dtype=np.float64)
    psi = basis_state(circ.n, circ.psi0_index)
    kinds, qs, ang, par, scl, um = _gate_arrays(circ.gates, th)
    grad = np.zeros(len(th), dtype=np.float64)
    e = np.zeros(1, dtype=np.float64)
    rc = lib().orc_adjoint_grad(_dp(psi.view(np.float64)), circ.n, len(circ.gates), _ip(kinds),
                                _ip(qs), _dp(ang), _dp(um) if um is not None else None, _ip(par),
                                _dp(scl), len(th), len(ham.coef),
                                _up(np.ascontiguousarray(ham.x, dtype=np.uint64)),
                                _up(np.ascontiguousarray(ham.z, dtype=np.uint64)),
                                _dp(np.ascontiguousarray(ham.coef, dtype=np.float64)), _dp(grad),
                                _dp(e))
    if rc:
        raise ValueError(f"oracle adjoint failed ({rc})")
    return float(e[0]), grad


def fd_grad(circ, ham, params=None, h: float = 1e-4):
    """Central finite differences [E(t+h e_p) - E(t-h e_p)] / 2h."""
    th = np.array(circ.theta, dtype=np.float64)
    idx = range(len(th)) if params is None else params
    out = []
    for p in idx:
        tp = th.copy(); tp[p] += h
        tm = th.copy(); tm[p] -= h
        out.append((energy(circ, ham, tp) - energy(circ, ham, tm)) / (2 * h))
    return np.array(out)


# Shift rules.  One-frequency gates (RX, RY, RZ, CPHASE: generator spectrum
# with a single gap 1): f' = [f(t + pi/2) - f(t - pi/2)] / 2.  GIVENS has
# generator eigenvalues {+1/2, -1/2, 0, 0}, i.e. gaps {1/2, 1}; the
# equidistant two-frequency rule (Wierichs et al., Quantum 6, 677 (2022))
# with shifts (2k-1)pi/2 gives the coefficients below.
SHIFT_RULES = {
    "RX": ((math.pi / 2, 0.5),),
    "RY": ((math.pi / 2, 0.5),),
    "RZ": ((math.pi / 2, 0.5),),
    "CPHASE": ((math.pi / 2, 0.5),),
    "GIVENS": ((math.pi / 2, (math.sqrt(2) + 1) / (4 * math.sqrt(2))),
               (3 * math.pi / 2, -(math.sqrt(2) - 1) / (4 * math.sqrt(2)))),
}


# The two-term rule applied to every gate whatever its spectrum: exact for
# one-frequency gates only (the nominal two evaluations per parameter).
TWO_TERM_RULE = ((math.pi / 2, 0.5),)


def _gate_angle(gt, th):
    p = gt[2]
    off = float(gt[3]) if len(gt) > 3 else 0.0
    scl = float(gt[4]) if len(gt) > 4 else 1.0
    return scl * th[p] + off, scl


def param_shift_grad(circ, ham, params=None, rule="exact"):
    """Parameter-shift gradient.  A parameter shared by several gates is
    differentiated gate by gate (product rule), each gate's derivative times
    its angle scale (chain rule).  rule="exact" uses SHIFT_RULES;
    rule="two-term" uses TWO_TERM_RULE for every gate."""
    th = np.array(circ.theta, dtype=np.float64)
    idx = range(len(th)) if params is None else params
    out = []
    for p in idx:
        acc = 0.0
        for gi, gt in enumerate(circ.gates):
            if gt[2] != p:
                continue
            ang, scl = _gate_angle(gt, th)
            rules = SHIFT_RULES[gt[0]] if rule == "exact" else TWO_TERM_RULE
            for shift, w in rules:
                vals = []
                for sgn in (+1, -1):
                    gates = list(circ.gates)
                    # shift only this gate: give it a private fixed angle
                    gates[gi] = (gt[0], gt[1], -1, ang + sgn * shift)
                    psi = apply_circuit(basis_state(circ.n, circ.psi0_index), gates, th)
                    vals.append(expectation(psi, ham))
                acc += scl * w * (vals[0] - vals[1])
        out.append(acc)
    return np.array(out)


def qr_permute(buf: np.ndarray, pos_old, pos_new) -> np.ndarray:
    """Relayout a physical buffer: logical qubit q moves from physical bit
    pos_old[q] to pos_new[q].  Written as a transpose of the state reshaped to
    a [2]*n tensor (axis a <-> physical bit n-1-a), independent of any index
    arithmetic."""
    n = len(pos_old)
    t = np.asarray(buf).reshape([2] * n)
    perm = [0] * n
    for q in range(n):
        perm[n - 1 - pos_new[q]] = n - 1 - pos_old[q]
    return np.ascontiguousarray(t.transpose(perm)).reshape(-1)


def to_logical(buf: np.ndarray, pos) -> np.ndarray:
    return qr_permute(buf, pos, list(range(len(pos))))
