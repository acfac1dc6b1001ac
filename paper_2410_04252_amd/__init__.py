"""Python binding of libsvq.so: argument marshalling only.

Every step of the hot path runs in the HIP library; this module converts
Python/numpy/torch arguments into the C ABI of ``include/svq.h`` and back.
Importing fails loudly when the library has not been built.  Functions keep
the C names (``sv_create``, ``sv_apply_circuit``, ...); :class:`State` is a
small convenience wrapper around one handle.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_double, c_int, c_int32, c_size_t, c_uint64, c_void_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsvq.so")

C64, C128 = 0, 1
EAGER, LAZY = 0, 1
KIND = {"H": 0, "X": 1, "Y": 2, "Z": 3, "S": 4, "T": 5, "RX": 6, "RY": 7, "RZ": 8,
        "CNOT": 9, "CZ": 10, "CPHASE": 11, "GIVENS": 12, "SWAP": 13, "U1": 14, "U2": 15}
STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ESHAPE", -5: "EUNSUP",
          -6: "EPOISONED"}


class svq_gate(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("q", c_int32 * 2), ("param", c_int32),
                ("scale", c_double), ("offset", c_double), ("mat", c_double * 32)]


class svq_pauli(ctypes.Structure):
    _fields_ = [("x", c_uint64), ("z", c_uint64), ("coef", c_double)]


class svq_stats(ctypes.Structure):
    _fields_ = [("n_qr", c_int32), ("n_gate_passes", c_int32), ("n_evc_passes", c_int32),
                ("n_groups", c_int32), ("n_phases", c_int32), ("tile_k", c_int32),
                ("bytes", c_double), ("ms_plan", c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class SvqError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


EXPORTS = ("sv_create", "sv_destroy", "sv_set_basis", "sv_set_amplitudes", "sv_get_amplitudes",
           "sv_get_layout", "sv_plan_dump", "sv_device_ptr", "sv_apply_circuit",
           "sv_apply_circuit_static", "sv_qr_permute",
           "sv_expectation", "sv_expectation_qsu", "sv_apply_hamiltonian", "sv_grad", "sv_param_shift_grad", "sv_plan_circuit",
           "sv_plan_circuit_json", "sv_plan_paulis", "sv_plan_ops", "sv_qr_cost", "sv_tune_circuit", "sv_tune_paulis",
           "sv_batch_tune", "sv_tune_save", "sv_tune_load", "sv_profile", "sv_profile_read", "sv_batch_create", "sv_batch_run",
           "sv_batch_destroy", "sv_batch_info", "sv_device_copy", "sv_pass_ceiling", "sv_last_error")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp = c_void_p
    L.sv_create.argtypes = [c_int, c_int, c_int, vp, c_size_t, vp, POINTER(vp)]
    L.sv_destroy.argtypes = [vp]
    L.sv_set_basis.argtypes = [vp, c_uint64]
    L.sv_set_amplitudes.argtypes = [vp, vp]
    L.sv_get_amplitudes.argtypes = [vp, vp]
    L.sv_get_layout.argtypes = [vp, POINTER(c_int32)]
    L.sv_device_ptr.argtypes = [vp, POINTER(vp)]
    L.sv_plan_dump.argtypes = [vp, ctypes.c_char_p, c_size_t, POINTER(c_size_t)]
    L.sv_apply_circuit.argtypes = [vp, POINTER(svq_gate), c_int, POINTER(c_double), c_int, c_int,
                                   c_int, POINTER(svq_stats)]
    L.sv_apply_circuit_static.argtypes = L.sv_apply_circuit.argtypes
    L.sv_qr_permute.argtypes = [vp, POINTER(c_int32)]
    L.sv_expectation.argtypes = [vp, POINTER(svq_pauli), c_int, c_int, POINTER(c_double),
                                 POINTER(c_double), POINTER(c_double), POINTER(svq_stats)]
    L.sv_expectation_qsu.argtypes = [vp, POINTER(svq_pauli), c_int, POINTER(c_double),
                                     POINTER(c_double), POINTER(svq_stats)]
    L.sv_apply_hamiltonian.argtypes = [vp, POINTER(svq_pauli), c_int, vp]
    L.sv_grad.argtypes = [vp, POINTER(svq_gate), c_int, POINTER(c_double), c_int,
                          POINTER(svq_pauli), c_int, c_int, POINTER(c_double), POINTER(c_double),
                          POINTER(c_double), POINTER(c_double), POINTER(svq_stats)]
    L.sv_param_shift_grad.argtypes = [vp, POINTER(svq_gate), c_int, POINTER(c_double), c_int,
                                      POINTER(svq_pauli), c_int, c_int, c_int, POINTER(c_double),
                                      POINTER(c_double), POINTER(c_double), POINTER(c_int),
                                      POINTER(svq_stats)]
    L.sv_plan_circuit.argtypes = [c_int, c_int, POINTER(svq_gate), c_int, c_int, c_int,
                                  POINTER(c_int32), POINTER(c_int32), POINTER(c_int32),
                                  POINTER(c_uint64), POINTER(c_int32), POINTER(c_int32)]
    L.sv_plan_circuit_json.argtypes = [c_int, c_int, POINTER(svq_gate), c_int, c_int, c_int,
                                       ctypes.c_char_p, c_size_t, POINTER(c_size_t)]
    L.sv_plan_paulis.argtypes = [c_int, c_int, POINTER(svq_pauli), c_int, c_int, c_int,
                                 POINTER(c_int32), POINTER(c_int32), POINTER(c_int32),
                                 POINTER(c_uint64), POINTER(c_int32), POINTER(c_int32)]
    L.sv_batch_create.argtypes = [c_int, POINTER(c_int32), POINTER(POINTER(svq_gate)),
                                  POINTER(c_int32), POINTER(c_int32), POINTER(POINTER(svq_pauli)),
                                  POINTER(c_int32), POINTER(c_uint64), c_int, vp, POINTER(vp)]
    L.sv_batch_run.argtypes = [vp, POINTER(POINTER(c_double)), POINTER(c_double),
                               POINTER(c_double), POINTER(c_double)]
    L.sv_batch_destroy.argtypes = [vp]
    ip = POINTER(c_int)
    L.sv_tune_circuit.argtypes = [vp, POINTER(svq_gate), c_int, POINTER(c_double), c_int, c_int,
                                  ip, ip, POINTER(c_double)]
    L.sv_tune_paulis.argtypes = [vp, POINTER(svq_pauli), c_int, ip, ip, POINTER(c_double)]
    L.sv_batch_tune.argtypes = [c_int, POINTER(c_int32), POINTER(POINTER(svq_gate)),
                                POINTER(c_int32), POINTER(c_int32), POINTER(POINTER(svq_pauli)),
                                POINTER(c_int32), POINTER(c_uint64), POINTER(POINTER(c_double)),
                                vp, ip, ip, POINTER(c_double)]
    L.sv_tune_save.argtypes = [ctypes.c_char_p]
    L.sv_tune_load.argtypes = [ctypes.c_char_p]
    L.sv_plan_ops.argtypes = [c_int, c_int, POINTER(c_uint64), c_int, c_int, c_int, c_int,
                              POINTER(c_int32), POINTER(c_uint64), POINTER(c_uint64),
                              POINTER(c_int32), POINTER(c_int32)]
    L.sv_qr_cost.argtypes = [c_int, c_int, c_int, POINTER(c_uint64), c_int, c_int, c_int, c_double,
                             c_double, POINTER(c_int32), POINTER(c_int32), POINTER(c_double)]
    L.sv_batch_info.argtypes = [vp, POINTER(c_double), POINTER(c_int32), POINTER(c_int32)]
    L.sv_pass_ceiling.argtypes = [vp, POINTER(c_int32), c_int, c_int, c_int, POINTER(c_double)]
    L.sv_profile.argtypes = [vp, c_int]
    L.sv_profile_read.argtypes = [vp, c_int, POINTER(c_int), POINTER(c_double)]
    L.sv_device_copy.argtypes = [vp, vp, c_size_t, vp]
    L.sv_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name != "sv_last_error":
            getattr(L, name).restype = c_int
    return L


lib = _load()


def _check(rc):
    if rc != 0:
        raise SvqError(rc, lib.sv_last_error().decode())


# ---------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------

def gates_array(gates):
    """[(kind, qubits, param[, extra[, scale]])] -> ctypes svq_gate array.

    With param >= 0 the angle is scale * theta[param] + extra (extra defaults
    to 0, scale to 1); with param = -1 it is extra.  For U1/U2, extra is the
    matrix."""
    arr = (svq_gate * max(1, len(gates)))()
    for i, gt in enumerate(gates):
        kind, qs, p = gt[0], gt[1], gt[2]
        g = arr[i]
        g.kind = KIND[kind]
        g.q[0] = int(qs[0])
        g.q[1] = int(qs[1]) if len(qs) > 1 else 0
        g.param = int(p) if p is not None and p >= 0 else -1
        g.scale = float(gt[4]) if len(gt) > 4 else 1.0
        if len(gt) > 3:
            extra = gt[3]
            if kind in ("U1", "U2"):
                m = np.ascontiguousarray(np.asarray(extra, dtype=np.complex128).reshape(-1)).view(np.float64)
                for j, v in enumerate(m):
                    g.mat[j] = float(v)
            else:
                g.offset = float(extra)
    return arr


def paulis_array(ham):
    n = len(ham.coef)
    arr = (svq_pauli * max(1, n))()
    for i in range(n):
        arr[i].x = int(ham.x[i])
        arr[i].z = int(ham.z[i])
        arr[i].coef = float(ham.coef[i])
    return arr


def _dptr(a):
    return a.ctypes.data_as(POINTER(c_double))


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return c_void_p(stream)
    return c_void_p(int(stream.cuda_stream))


# ---------------------------------------------------------------------------
# C-named wrappers
# ---------------------------------------------------------------------------

def sv_create(n, g, dtype=C64, dev_buf=None, buf_bytes=0, stream=None):
    h = c_void_p()
    _check(lib.sv_create(n, g, dtype, dev_buf, buf_bytes, _stream_ptr(stream), byref(h)))
    return h


def sv_destroy(h):
    _check(lib.sv_destroy(h))


def sv_set_basis(h, index):
    _check(lib.sv_set_basis(h, int(index)))


def sv_set_amplitudes(h, host):
    _check(lib.sv_set_amplitudes(h, host.ctypes.data_as(c_void_p)))


def sv_get_amplitudes(h, host):
    _check(lib.sv_get_amplitudes(h, host.ctypes.data_as(c_void_p)))


def sv_get_layout(h, n):
    out = (c_int32 * n)()
    _check(lib.sv_get_layout(h, out))
    return list(out)


def sv_plan_dump(h):
    """The handle's last executed plan, parsed from the library's JSON."""
    import json
    need = c_size_t(0)
    _check(lib.sv_plan_dump(h, None, 0, byref(need)))
    buf = ctypes.create_string_buffer(need.value)
    _check(lib.sv_plan_dump(h, buf, need.value, None))
    return json.loads(buf.value.decode())


def sv_device_copy(src_ptr, dst_ptr, nbytes, stream=None):
    _check(lib.sv_device_copy(c_void_p(src_ptr), c_void_p(dst_ptr), nbytes, _stream_ptr(stream)))


def sv_device_ptr(h):
    p = c_void_p()
    _check(lib.sv_device_ptr(h, byref(p)))
    return p.value


def sv_apply_circuit(h, gates_c, m, theta, n_theta, sched, tile_k=0):
    st = svq_stats()
    th = np.ascontiguousarray(theta, dtype=np.float64) if n_theta else np.zeros(1)
    _check(lib.sv_apply_circuit(h, gates_c, m, _dptr(th), n_theta, sched, tile_k, byref(st)))
    return st


def sv_apply_circuit_static(h, gates_c, m, theta, n_theta, sched, tile_k=0):
    """sv_apply_circuit without device allocation (tables in the library's
    static scratch)."""
    st = svq_stats()
    th = np.ascontiguousarray(theta, dtype=np.float64) if n_theta else np.zeros(1)
    _check(lib.sv_apply_circuit_static(h, gates_c, m, _dptr(th), n_theta, sched, tile_k,
                                       byref(st)))
    return st


def sv_qr_permute(h, new_pos):
    arr = (c_int32 * len(new_pos))(*[int(v) for v in new_pos])
    _check(lib.sv_qr_permute(h, arr))


def sv_expectation(h, terms_c, n_terms, sched, energy_dev=None, chunk_dev=None, want_host=True):
    st = svq_stats()
    e = c_double(0.0)
    _check(lib.sv_expectation(h, terms_c, n_terms, sched, byref(e) if want_host else None,
                              ctypes.cast(energy_dev, POINTER(c_double)) if energy_dev else None,
                              ctypes.cast(chunk_dev, POINTER(c_double)) if chunk_dev else None,
                              byref(st)))
    return e.value, st


def sv_expectation_qsu(h, terms_c, n_terms, energy_dev=None, want_host=True):
    st = svq_stats()
    e = c_double(0.0)
    _check(lib.sv_expectation_qsu(h, terms_c, n_terms, byref(e) if want_host else None,
                                  ctypes.cast(energy_dev, POINTER(c_double)) if energy_dev else None,
                                  byref(st)))
    return e.value, st


def sv_apply_hamiltonian(h, terms_c, n_terms, out):
    _check(lib.sv_apply_hamiltonian(h, terms_c, n_terms, out))


def sv_grad(h, gates_c, m, theta, n_theta, terms_c, n_terms, sched, grad_dev=None,
            energy_dev=None, want_host=True):
    st = svq_stats()
    th = np.ascontiguousarray(theta, dtype=np.float64) if n_theta else np.zeros(1)
    e = c_double(0.0)
    g = np.zeros(max(1, n_theta), dtype=np.float64)
    _check(lib.sv_grad(h, gates_c, m, _dptr(th), n_theta, terms_c, n_terms, sched,
                       byref(e) if want_host else None,
                       ctypes.cast(energy_dev, POINTER(c_double)) if energy_dev else None,
                       _dptr(g) if want_host else None,
                       ctypes.cast(grad_dev, POINTER(c_double)) if grad_dev else None,
                       byref(st)))
    return e.value, g[:n_theta], st


SHIFT_EXACT, SHIFT_TWO_TERM = 0, 1


def sv_param_shift_grad(h, gates_c, m, theta, n_theta, terms_c, n_terms, sched, rule=SHIFT_EXACT,
                        grad_dev=None, want_energy=True):
    """(E or None, gradient, number of evaluations, stats) by the parameter-shift rules."""
    st = svq_stats()
    th = np.ascontiguousarray(theta, dtype=np.float64) if n_theta else np.zeros(1)
    e = c_double(0.0)
    g = np.zeros(max(1, n_theta), dtype=np.float64)
    ne = c_int(0)
    _check(lib.sv_param_shift_grad(h, gates_c, m, _dptr(th), n_theta, terms_c, n_terms, sched, rule,
                                   byref(e) if want_energy else None, _dptr(g),
                                   ctypes.cast(grad_dev, POINTER(c_double)) if grad_dev else None,
                                   byref(ne), byref(st)))
    return (e.value if want_energy else None), g[:n_theta], ne.value, st


def sv_plan_circuit(n, g, gates, sched, tile_k=0):
    gc = gates_array(gates)
    m = len(gates)
    order = (c_int32 * max(1, m))()
    qt = (c_int32 * max(1, m))()
    ps = (c_int32 * max(1, m))()
    loc = (c_uint64 * max(1, m))()
    nqr, npass = c_int32(), c_int32()
    _check(lib.sv_plan_circuit(n, g, gc, m, sched, tile_k, order, qt, ps, loc, byref(nqr),
                               byref(npass)))
    return dict(order=list(order)[:m], qr_tile=list(qt)[:m], pass_=list(ps)[:m],
                local=list(loc)[:m], n_qr=nqr.value, n_pass=npass.value)


def sv_plan_circuit_json(n, g, gates, sched, tile_k=0):
    """Host-only plan of a gate list, parsed from the library's JSON."""
    import json
    gc = gates_array(gates)
    need = c_size_t(0)
    _check(lib.sv_plan_circuit_json(n, g, gc, len(gates), sched, tile_k, None, 0, byref(need)))
    buf = ctypes.create_string_buffer(need.value)
    _check(lib.sv_plan_circuit_json(n, g, gc, len(gates), sched, tile_k, buf, need.value, None))
    return json.loads(buf.value.decode())


def sv_tune_circuit(h, gates_c, m, theta, n_theta, sched):
    k, c, ms = c_int(), c_int(), c_double()
    th = np.ascontiguousarray(theta, dtype=np.float64) if n_theta else np.zeros(1)
    _check(lib.sv_tune_circuit(h, gates_c, m, _dptr(th), n_theta, sched, byref(k), byref(c),
                               byref(ms)))
    return k.value, c.value, ms.value


def sv_tune_paulis(h, terms_c, n_terms):
    k, c, ms = c_int(), c_int(), c_double()
    _check(lib.sv_tune_paulis(h, terms_c, n_terms, byref(k), byref(c), byref(ms)))
    return k.value, c.value, ms.value


def sv_tune_save(path):
    _check(lib.sv_tune_save(os.fsencode(path)))


def sv_tune_load(path):
    _check(lib.sv_tune_load(os.fsencode(path)))


PLAN_ADHOC, PLAN_FLAT, PLAN_HIERARCHICAL, PLAN_ADHOC_INDEX = 0, 1, 2, 3


def sv_plan_ops(n, n_local, targets, method, n_intra=0, fill_highest=False):
    """Level-1 plan over operators given as qubit tuples (host only)."""
    m = len(targets)
    tm = (c_uint64 * max(1, m))(*[sum(1 << q for q in t) for t in targets])
    order = (c_int32 * max(1, m))()
    loc = (c_uint64 * max(1, m))()
    intra = (c_uint64 * max(1, m))()
    nqr, ninter = c_int32(), c_int32()
    _check(lib.sv_plan_ops(n, n_local, tm, m, method, n_intra, int(fill_highest), order, loc,
                           intra, byref(nqr), byref(ninter)))
    return dict(order=list(order)[:m], local=list(loc)[:m], intra=list(intra)[:m],
                n_qr=nqr.value, n_inter=ninter.value)


def sv_qr_cost(n, n_local, n_intra, targets, method, w_intra=1.0, w_inter=10.0, fill_highest=False):
    """eq. comm_cost of a level-1 plan (host only): (N_intra, N_inter, cost)."""
    m = len(targets)
    tm = (c_uint64 * max(1, m))(*[sum(1 << q for q in t) for t in targets])
    ni, ne, cost = c_int32(), c_int32(), c_double()
    _check(lib.sv_qr_cost(n, n_local, n_intra, tm, m, method, int(fill_highest), w_intra, w_inter,
                          byref(ni), byref(ne), byref(cost)))
    return ni.value, ne.value, cost.value


def sv_pass_ceiling(h, tile_bits, nphase, reps=5):
    """Average ms of one gate pass without gates over the given tile bits."""
    tb = (c_int32 * len(tile_bits))(*tile_bits)
    ms = c_double()
    _check(lib.sv_pass_ceiling(h, tb, len(tile_bits), nphase, reps, byref(ms)))
    return ms.value


def sv_plan_paulis(n, g, ham, sched, tile_k=0):
    tc = paulis_array(ham)
    nt = len(ham.coef)
    order = (c_int32 * max(1, nt))()
    qt = (c_int32 * max(1, nt))()
    ps = (c_int32 * max(1, nt))()
    loc = (c_uint64 * max(1, nt))()
    nqr, npass = c_int32(), c_int32()
    _check(lib.sv_plan_paulis(n, g, tc, nt, sched, tile_k, order, qt, ps, loc, byref(nqr),
                              byref(npass)))
    ng = len(set(int(x) for x in ham.x))
    return dict(order=list(order)[:ng], qr_tile=list(qt)[:ng], pass_=list(ps)[:ng],
                local=list(loc)[:ng], n_qr=nqr.value, n_pass=npass.value)


PROF_GATE, PROF_QR, PROF_EVC, PROF_HPSI, PROF_ADJ, PROF_PAULI_GATE = 0, 1, 2, 3, 4, 5


def sv_profile(h, enable):
    _check(lib.sv_profile(h, int(enable)))


def sv_profile_read(h, kind):
    c = c_int(0)
    t = c_double(0.0)
    _check(lib.sv_profile_read(h, kind, byref(c), byref(t)))
    return c.value, t.value


# ---------------------------------------------------------------------------
# convenience wrapper
# ---------------------------------------------------------------------------

class State:
    """One state vector on the current HIP device.

    ``buf``: optional torch tensor (complex64/complex128, >= 2^n elements)
    that the state borrows; ``stream``: torch stream (default: current)."""

    def __init__(self, n, g=0, dtype="c64", buf=None, stream=None):
        self.n, self.g = n, g
        self.dtype = C64 if dtype in ("c64", C64) else C128
        self._buf = buf
        ptr = None
        nbytes = 0
        if buf is not None:
            ptr = c_void_p(buf.data_ptr())
            nbytes = buf.numel() * buf.element_size()
        if stream is None:
            try:
                import torch
                if torch.cuda.is_available():
                    stream = torch.cuda.current_stream()
            except ImportError:
                stream = None
        self._stream = stream
        self.h = sv_create(n, g, self.dtype, ptr, nbytes, stream)

    def close(self):
        if self.h is not None:
            sv_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def np_dtype(self):
        return np.complex64 if self.dtype == C64 else np.complex128

    def set_basis(self, idx):
        sv_set_basis(self.h, idx)

    def set_amplitudes(self, v):
        sv_set_amplitudes(self.h, np.ascontiguousarray(v, dtype=self.np_dtype))

    def get_amplitudes(self):
        out = np.empty(1 << self.n, dtype=self.np_dtype)
        sv_get_amplitudes(self.h, out)
        return out

    def layout(self):
        return sv_get_layout(self.h, self.n)

    def plan_dump(self):
        return sv_plan_dump(self.h)

    def apply(self, circuit, theta=None, sched=LAZY, tile_k=0):
        gc = gates_array(circuit.gates)
        th = circuit.theta if theta is None else theta
        return sv_apply_circuit(self.h, gc, len(circuit.gates), th, len(th), sched, tile_k)

    def apply_gates(self, gates, theta=(), sched=LAZY, tile_k=0):
        gc = gates_array(gates)
        return sv_apply_circuit(self.h, gc, len(gates), np.asarray(theta, dtype=np.float64),
                                len(theta), sched, tile_k)

    def qr_permute(self, new_pos):
        sv_qr_permute(self.h, new_pos)

    def expectation(self, ham, sched=LAZY):
        return sv_expectation(self.h, paulis_array(ham), len(ham.coef), sched)

    def expectation_qsu(self, ham):
        """The QSU-based comparison method (Pauli strings applied as gates)."""
        return sv_expectation_qsu(self.h, paulis_array(ham), len(ham.coef))

    def tune(self, circuit, theta=None, sched=LAZY):
        """Time tile widths k and low-bit counts c on this circuit; the
        fastest becomes the default for every state of this (n, g, dtype).
        Overwrites the amplitudes."""
        th = circuit.theta if theta is None else theta
        return sv_tune_circuit(self.h, gates_array(circuit.gates), len(circuit.gates), th,
                               len(th), sched)

    def tune_paulis(self, ham):
        """Same for the Pauli (EVC) passes; the state is read, not changed."""
        return sv_tune_paulis(self.h, paulis_array(ham), len(ham.coef))

    def grad(self, circuit, ham, theta=None, sched=LAZY):
        th = circuit.theta if theta is None else theta
        return sv_grad(self.h, gates_array(circuit.gates), len(circuit.gates), th, len(th),
                       paulis_array(ham), len(ham.coef), sched)

    def param_shift_grad(self, circuit, ham, theta=None, sched=LAZY, rule=SHIFT_EXACT):
        th = circuit.theta if theta is None else theta
        return sv_param_shift_grad(self.h, gates_array(circuit.gates), len(circuit.gates), th,
                                   len(th), paulis_array(ham), len(ham.coef), sched, rule)


class Batch:
    """Many VQE instances evaluated by one persistent, graph-captured launch
    (sv_batch_create / sv_batch_run).  ``instances``: list of (circuit,
    hamiltonian) pairs (workloads.Circuit / workloads.Hamiltonian)."""

    def __init__(self, instances, low_bits=0, stream=None):
        self.n = len(instances)
        self._gates = [gates_array(c.gates) for c, _ in instances]
        self._terms = [paulis_array(h) for _, h in instances]
        self.n_theta = [c.n_params for c, _ in instances]
        nq = (c_int32 * self.n)(*[c.n for c, _ in instances])
        ms = (c_int32 * self.n)(*[len(c.gates) for c, _ in instances])
        nth = (c_int32 * self.n)(*self.n_theta)
        nts = (c_int32 * self.n)(*[len(h.coef) for _, h in instances])
        psi0 = (c_uint64 * self.n)(*[c.psi0_index for c, _ in instances])
        gp = (POINTER(svq_gate) * self.n)(*[ctypes.cast(g, POINTER(svq_gate)) for g in self._gates])
        tp = (POINTER(svq_pauli) * self.n)(*[ctypes.cast(t, POINTER(svq_pauli)) for t in self._terms])
        if stream is None:
            try:
                import torch
                if torch.cuda.is_available():
                    stream = torch.cuda.current_stream()
            except ImportError:
                stream = None
        self.h = c_void_p()
        self._args = (nq, gp, ms, nth, tp, nts, psi0)
        self._stream = stream
        _check(lib.sv_batch_create(self.n, nq, gp, ms, nth, tp, nts, psi0, low_bits,
                                   _stream_ptr(stream), byref(self.h)))
        self.theta0 = [np.ascontiguousarray(c.theta, dtype=np.float64) for c, _ in instances]

    def tune(self, thetas=None):
        """Measured choice of items per stage and low bits for these
        instances (used by later batches created with low_bits = 0)."""
        th = self.theta0 if thetas is None else [np.ascontiguousarray(t, dtype=np.float64)
                                                 for t in thetas]
        ptrs = (POINTER(c_double) * self.n)(*[_dptr(t) if t.size else None for t in th])
        ch, lb, ms = c_int(), c_int(), c_double()
        nq, gp, mm, nth, tp, nts, psi0 = self._args
        _check(lib.sv_batch_tune(self.n, nq, gp, mm, nth, tp, nts, psi0, ptrs,
                                 _stream_ptr(self._stream), byref(ch), byref(lb), byref(ms)))
        return ch.value, lb.value, ms.value

    def run(self, thetas=None):
        th = self.theta0 if thetas is None else [np.ascontiguousarray(t, dtype=np.float64)
                                                 for t in thetas]
        ptrs = (POINTER(c_double) * self.n)(*[_dptr(t) if t.size else None for t in th])
        e = np.zeros(self.n)
        g = np.zeros(max(1, sum(self.n_theta)))
        lat = np.zeros(self.n)
        _check(lib.sv_batch_run(self.h, ptrs, _dptr(e), _dptr(g), _dptr(lat)))
        grads, o = [], 0
        for k in self.n_theta:
            grads.append(g[o:o + k].copy())
            o += k
        return e, grads, lat

    def info(self):
        """(algorithmic HBM bytes of one run, stages, work items)."""
        by, ns, ni = c_double(), c_int32(), c_int32()
        _check(lib.sv_batch_info(self.h, byref(by), byref(ns), byref(ni)))
        return by.value, ns.value, ni.value

    def close(self):
        if self.h is not None and self.h.value:
            _check(lib.sv_batch_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# Measured tile widths / low-bit counts per size class, written by the tuner
# (sv_tune_save) on an MI355X; SVQ_TUNE_FILE names another table, "" none.
TUNE_FILE = os.environ.get("SVQ_TUNE_FILE", os.path.join(_HERE, "tuned_mi355x.txt"))
if TUNE_FILE and os.path.exists(TUNE_FILE):
    sv_tune_load(TUNE_FILE)
