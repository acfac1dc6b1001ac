"""Error paths of the C ABI: every call returns a status and never throws;
invalid arguments leave the handle unchanged; a failed allocation is ENOMEM
and leaves the handle usable."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from tolerances import AMP, amp_ok, grad_ok

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_2410_04252_amd as P
    torch.cuda.set_device(0)
    return P


def _status(P, fn, *args):
    try:
        fn(*args)
    except P.SvqError as e:
        return P.STATUS[e.status]
    return "OK"


def test_enomem_through_allocation_cap(P, monkeypatch):
    import torch
    n, g = 20, 3
    circ, ham = W.fabric(n, 4, 901), W.jw_terms(n, 50, 902)
    monkeypatch.setenv("SVQ_MAX_ALLOC_BYTES", str(1 << 20))
    # the library's own state buffer (8 MiB) exceeds the cap
    with pytest.raises(P.SvqError) as ei:
        P.State(n, g, "c64")
    assert P.STATUS[ei.value.status] == "ENOMEM"
    # a borrowed buffer needs no allocation; the adjoint's lambda does
    buf = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
    st = P.State(n, g, "c64", buf=buf)
    st.set_basis(circ.psi0_index)
    assert _status(P, st.grad, circ, ham) == "ENOMEM"
    # nothing ran: the state is still psi0 in the identity layout
    assert st.layout() == list(range(n))
    want = np.zeros(1 << n, dtype=np.complex64)
    want[circ.psi0_index] = 1
    np.testing.assert_array_equal(st.get_amplitudes(), want)
    # and the handle is not poisoned: lift the cap and it works
    monkeypatch.delenv("SVQ_MAX_ALLOC_BYTES")
    e, grad, _ = st.grad(circ, ham)
    e_ref, g_ref = oracle.adjoint_grad(circ, ham)
    ok, grel = grad_ok(grad, g_ref, ham, "c64")
    assert ok, grel
    st.close()


def test_eshape(P):
    import torch
    buf = torch.empty(1 << 11, dtype=torch.complex64, device="cuda")
    with pytest.raises(P.SvqError) as ei:
        P.State(12, 2, "c64", buf=buf)
    assert P.STATUS[ei.value.status] == "ESHAPE"
    a, b = P.State(12, 2, "c64"), P.State(13, 2, "c64")
    ham = W.jw_terms(12, 10, 903)
    assert _status(P, P.sv_apply_hamiltonian, a.h, P.paulis_array(ham), len(ham.coef), b.h) == "ESHAPE"
    c = P.State(12, 2, "c128")
    assert _status(P, P.sv_apply_hamiltonian, a.h, P.paulis_array(ham), len(ham.coef), c.h) == "ESHAPE"
    # plan text larger than the caller's buffer
    a.apply(W.fabric(12, 2, 904))
    import ctypes
    small = ctypes.create_string_buffer(8)
    rc = P.lib.sv_plan_dump(a.h, small, 8, None)
    assert P.STATUS[rc] == "ESHAPE"
    for s in (a, b, c):
        s.close()


def test_eunsup_batch_instance_needing_a_wide_term(P):
    """A batch instance keeps all qubits local (no reorder): a 14-qubit
    string with X on every qubit fits no 2^10 tile (instances of at most 13
    qubits are held in LDS and take any string)."""
    circ = W.fabric(14, 2, 905)
    ham = W.Hamiltonian(14, np.array([(1 << 14) - 1], dtype=np.uint64),
                        np.array([0], dtype=np.uint64), np.array([0.5]))
    with pytest.raises(P.SvqError) as ei:
        P.Batch([(circ, ham)])
    assert P.STATUS[ei.value.status] == "EUNSUP"


@pytest.mark.parametrize("where", ["theta", "offset", "scale", "matrix"])
def test_nan_angle_is_einval_and_leaves_state(P, where):
    n, g = 12, 2
    v = W.random_state(n, 906, np.complex64)
    st = P.State(n, g, "c64")
    st.set_amplitudes(v)
    st.qr_permute([int(x) for x in np.random.default_rng(907).permutation(n)])
    pos = st.layout()
    theta = np.array([0.3, -0.2])
    gates = [("RY", (0,), 0), ("GIVENS", (1, 5), 1)]
    if where == "theta":
        theta[1] = math.nan
    elif where == "offset":
        gates.append(("RZ", (3,), -1, math.nan))
    elif where == "scale":
        gates.append(("RZ", (3,), 0, 0.1, math.inf))
    else:
        m = np.eye(2, dtype=np.complex128)
        m[0, 1] = complex(math.nan, 0)
        gates.append(("U1", (2,), -1, m))
    assert _status(P, st.apply_gates, gates, theta) == "EINVAL"
    circ = W.Circuit(n, gates, theta, 0)
    assert _status(P, st.grad, circ, W.jw_terms(n, 10, 908)) == "EINVAL"
    assert st.layout() == pos
    np.testing.assert_array_equal(st.get_amplitudes(), v)
    st.close()


def test_einval_gate_and_term_validation(P):
    n, g = 10, 1
    st = P.State(n, g, "c64")
    bad = [
        [("CNOT", (3, 3), -1)],            # repeated qubit
        [("RY", (10,), 0)],                # qubit out of range
        [("RY", (1,), 5)],                 # parameter index out of range
        [("H", (1,), 0)],                  # non-parametric kind with a parameter
    ]
    for gates in bad:
        assert _status(P, st.apply_gates, gates, [0.1]) == "EINVAL", gates
    ham = W.Hamiltonian(n, np.array([1 << 12], dtype=np.uint64), np.array([0], dtype=np.uint64),
                        np.array([1.0]))
    assert _status(P, st.expectation, ham) == "EINVAL"
    ham = W.Hamiltonian(n, np.array([1], dtype=np.uint64), np.array([0], dtype=np.uint64),
                        np.array([math.nan]))
    assert _status(P, st.expectation, ham) == "EINVAL"
    assert _status(P, st.qr_permute, [0] * n) == "EINVAL"
    assert _status(P, P.sv_apply_circuit, st.h, P.gates_array([("H", (0,), -1)]), 1,
                   np.zeros(1), 0, P.LAZY, 14) == "EINVAL"
    st.close()


def test_scaled_shared_parameter_gradient(P):
    """One parameter drives two gates through angle = scale * theta + offset
    with different scales (and a third gate through its own parameter): the
    adjoint applies the chain rule, checked against the oracle's adjoint and
    its exact parameter-shift rule."""
    n, g = 12, 2
    base = W.fabric(n, 3, 909)
    gates = []
    for i, (kind, qs, p) in enumerate(base.gates):
        if p >= 0:
            gates.append((kind, qs, p % 5, 0.1 * (i % 3) - 0.2, (-1.5, 0.5, 2.0)[i % 3]))
        else:
            gates.append((kind, qs, p))
    theta = np.random.default_rng(910).uniform(-math.pi, math.pi, size=5)
    circ = W.Circuit(n, gates, theta, base.psi0_index)
    ham = W.jw_terms(n, 60, 911)
    e_ref, g_ref = oracle.adjoint_grad(circ, ham)
    g_ps = oracle.param_shift_grad(circ, ham)
    assert np.max(np.abs(g_ref - g_ps)) < 1e-10
    for dtype in ("c64", "c128"):
        st = P.State(n, g, dtype)
        st.set_basis(base.psi0_index)
        st.apply(circ)
        ok, mx, rl2 = amp_ok(st.get_amplitudes(), oracle.run_circuit(circ), dtype)
        assert ok, (dtype, mx, rl2)
        st.set_basis(base.psi0_index)
        e, grad, _ = st.grad(circ, ham)
        ok, grel = grad_ok(grad, g_ref, ham, dtype)
        assert ok, (dtype, grel)
        st.close()


def test_plan_dump_describes_the_executed_plan(P):
    cfg = W.config("hea12")
    circ, ham = cfg["circuit"], cfg["ham"]
    st = P.State(12, 2, "c128")
    assert st.plan_dump() == {}
    st.set_basis(0)
    stats = st.apply(circ, sched=P.EAGER, tile_k=8)
    d = st.plan_dump()
    assert d["kind"] == "circuit" and d["schedule"] == "eager" and d["tile_k"] == 8
    assert d["n_qr"] == stats.n_qr == sum(1 for s in d["steps"] if s["type"] == "qr")
    assert sum(s["gates"] for s in d["steps"] if s["type"] == "gate_pass") == len(circ.gates)
    assert sorted(d["order"]) == list(range(len(circ.gates)))
    assert d["pos_after"] == st.layout()
    e, est = st.expectation(ham)
    d = st.plan_dump()
    assert d["kind"] == "paulis" and d["n_qr"] == est.n_qr
    assert d["n_passes"] == est.n_evc_passes
    st.close()
