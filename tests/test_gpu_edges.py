"""GPU edge cases through the C ABI: empty inputs, the smallest states and
tiles, ragged term counts, single gates on global qubits, identity terms."""
import numpy as np
import pytest

import oracle
import workloads as W
from tolerances import AMP, energy_ok

pytestmark = pytest.mark.gpu


def _cdt(dtype):
    """numpy dtype of a handle: inputs are drawn in it, so the oracle and the
    GPU start from the same amplitudes."""
    return np.complex64 if dtype == "c64" else np.complex128


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_2410_04252_amd as P
    torch.cuda.set_device(0)
    return P


def _print(*a):
    print(*a, flush=True)


def _ham(n, strings):
    """strings: [(x, z, coef)] with integer masks."""
    x = np.array([s[0] for s in strings], dtype=np.uint64)
    z = np.array([s[1] for s in strings], dtype=np.uint64)
    c = np.array([s[2] for s in strings], dtype=np.float64)
    return W.Hamiltonian(n, x, z, c)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("sched", [0, 1])
def test_empty_circuit_and_empty_hamiltonian(P, dtype, sched):
    """No gates: the state is untouched (bit for bit) and no pass runs.
    No terms: the energy is exactly 0."""
    n, g = 12, 2
    _print(f"empty inputs {dtype} sched={sched}")
    v = W.random_state(n, 901, _cdt(dtype))
    st = P.State(n, g, dtype)
    st.set_amplitudes(v)
    stats = st.apply_gates([], theta=[], sched=sched)
    assert stats.n_gate_passes == 0 and stats.n_qr == 0
    assert np.array_equal(st.get_amplitudes(), v.astype(st.np_dtype))
    e, stats = st.expectation(_ham(n, []), sched=sched)
    assert e == 0.0
    assert stats.n_evc_passes == 0
    st.close()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n,g", [(8, 0), (9, 1), (10, 2)])
def test_smallest_states(P, dtype, n, g):
    """n - g = 8..9 local qubits: the narrowest tiles (k = 8, 9), a single
    tile per chunk, for gate passes and Pauli passes (one or two cube bits)."""
    _print(f"smallest n={n} g={g} {dtype}")
    circ = W.random_circuit(n, 60, 910 + n)
    v = W.random_state(n, 911 + n, _cdt(dtype))
    ref = oracle.apply_circuit(v, circ.gates, circ.theta)
    ham = W.random_pauli(n, 37, 912 + n)
    for sched in (P.LAZY, P.EAGER):
        st = P.State(n, g, dtype)
        st.set_amplitudes(v)
        st.apply(circ, sched=sched)
        got = st.get_amplitudes()
        assert np.max(np.abs(got - ref)) < AMP[dtype]
        e, _ = st.expectation(ham, sched=sched)
        ok, rel = energy_ok(e, oracle.expectation(ref, ham), ref, ham, dtype)
        assert ok, rel
        st.close()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("nterms", [1, 2, 3, 5, 6, 7])
def test_ragged_term_counts_in_one_group(P, dtype, nterms):
    """One flip-mask group with 1..7 terms: the Pauli pass reads terms four
    at a time, so every remainder of the tail loop is exercised; Y counts
    0..3 reach both the real and the imaginary pair products."""
    n, g = 14, 2
    _print(f"ragged terms {nterms} {dtype}")
    x = (1 << 3) | (1 << 9) | (1 << 12)
    rng = np.random.default_rng(920 + nterms)
    strings = []
    zs = set()
    while len(strings) < nterms:
        z = int(rng.integers(0, 1 << n))
        if z in zs:
            continue
        zs.add(z)
        strings.append((x, z, float(rng.normal(0.0, 0.3))))
    ham = _ham(n, strings)
    v = W.random_state(n, 921, _cdt(dtype))
    e_ref = oracle.expectation(v, ham)
    for sched in (P.LAZY, P.EAGER):
        st = P.State(n, g, dtype)
        st.set_amplitudes(v)
        e, stats = st.expectation(ham, sched=sched)
        ok, rel = energy_ok(e, e_ref, v, ham, dtype)
        assert ok, rel
        assert stats.n_groups == 1
        st.close()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_identity_and_global_only_terms(P, dtype):
    """The identity string gives its coefficient times the norm; strings
    whose X/Y support lies only on global qubits need a reorder first."""
    n, g = 13, 3
    _print(f"identity/global terms {dtype}")
    top = [n - 1, n - 2, n - 3]
    strings = [(0, 0, 0.75),
               (1 << top[0], 0, 0.2),
               ((1 << top[0]) | (1 << top[1]), 1 << top[1], -0.4),
               (1 << top[2], (1 << top[2]) | 1, 0.3),
               (0, (1 << top[0]) | (1 << top[1]) | (1 << top[2]), 0.5)]
    ham = _ham(n, strings)
    v = W.random_state(n, 930, _cdt(dtype))
    e_ref = oracle.expectation(v, ham)
    for sched in (P.LAZY, P.EAGER):
        st = P.State(n, g, dtype)
        st.set_amplitudes(v)
        e, _ = st.expectation(ham, sched=sched)
        ok, rel = energy_ok(e, e_ref, v, ham, dtype)
        assert ok, rel
        st.close()
    st = P.State(n, g, dtype)
    st.set_amplitudes(v)
    e, _ = st.expectation(_ham(n, [(0, 0, 0.75)]))
    assert abs(e - 0.75) < (1e-6 if dtype == "c64" else 1e-12)
    st.close()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("kind", list(W.GATE_KINDS))
def test_single_gate_on_global_qubits(P, dtype, kind):
    """One gate of each kind whose qubits include the highest (global)
    qubit: the lazy and eager schedules both reorder before the pass."""
    n, g = 12, 2
    _print(f"single gate {kind} {dtype}")
    a = W.GATE_ARITY[kind]
    qs = (n - 1,) if a == 1 else (n - 1, 3)
    if kind in W.PARAM_KINDS:
        circ = W.Circuit(n, [(kind, qs, 0)], np.array([0.917]), 0)
    else:
        circ = W.Circuit(n, [(kind, qs, -1)], np.zeros(0), 0)
    v = W.random_state(n, 940, _cdt(dtype))
    ref = oracle.apply_circuit(v, circ.gates, circ.theta)
    for sched in (P.LAZY, P.EAGER):
        st = P.State(n, g, dtype)
        st.set_amplitudes(v)
        stats = st.apply(circ, sched=sched)
        assert stats.n_gate_passes <= 1
        assert np.max(np.abs(st.get_amplitudes() - ref)) < AMP[dtype]
        st.close()
