"""GPU parity: the HIP path through the C ABI against the CPU oracle."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from tolerances import AMP, amp_ok, energy_ok, grad_ok

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


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n,g", [(12, 2), (14, 3), (17, 4)])
def test_qr_permute_bitexact(P, n, g, dtype):
    import torch
    _print(f"qr_permute n={n} g={g} {dtype}")
    rng = np.random.default_rng(n * 7 + g)
    v = W.random_state(n, 5 + n, np.complex64 if dtype == "c64" else np.complex128)
    buf = torch.empty(1 << n, dtype=torch.complex64 if dtype == "c64" else torch.complex128,
                      device="cuda")
    st = P.State(n, g, dtype, buf=buf)
    st.set_amplitudes(v)
    pos = list(range(n))
    for trial in range(4):
        if trial % 2 == 0:   # a QR: disjoint local/global transpositions
            s = int(rng.integers(1, g + 1))
            loc = rng.choice(n - g, size=s, replace=False)
            glo = rng.choice(np.arange(n - g, n), size=s, replace=False)
            phys_new = list(range(n))
            for a, b in zip(loc, glo):
                phys_new[a], phys_new[b] = phys_new[b], phys_new[a]
            new = [phys_new[p] for p in pos]
        else:                # an arbitrary relayout (two passes)
            new = list(rng.permutation(n))
        before = buf.cpu().numpy().copy()
        st.qr_permute(new)
        torch.cuda.synchronize()
        after = buf.cpu().numpy()
        want = oracle.qr_permute(before, pos, new)
        assert np.array_equal(after, want), f"trial {trial}"
        assert st.layout() == [int(x) for x in new]
        pos = [int(x) for x in new]
    np.testing.assert_array_equal(st.get_amplitudes(), v)
    st.close()


CIRCS = {
    "hea12": lambda: (W.hea(12, 4, 4253), 2),
    "fabric16": lambda: (W.fabric(16, 8, 11), 3),
    "random14": lambda: (W.random_circuit(14, 120, 12), 3),
}
# local qubits n - g of each circuit: a tile is at most that wide
_LOCAL = {"hea12": 10, "fabric16": 13, "random14": 11}


@pytest.mark.parametrize("sched", [0, 1])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("name,k", [(nm, k) for k in (8, 10, 12) for nm in CIRCS
                                    if k <= _LOCAL[nm]])
def test_circuit_parity(P, name, dtype, sched, k):
    circ, g = CIRCS[name]()
    n = circ.n
    assert k <= n - g
    _print(f"circuit {name} {dtype} sched={sched} k={k}")
    ref = oracle.run_circuit(circ)
    st = P.State(n, g, dtype)
    st.set_basis(circ.psi0_index)
    stats = st.apply(circ, sched=sched, tile_k=k)
    got = st.get_amplitudes()
    ok, mx, rl2 = amp_ok(got, ref, dtype)
    assert ok, (mx, rl2)
    assert stats.n_gate_passes >= 1
    st.close()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_circuit_random_state_input(P, dtype):
    n, g = 15, 3
    circ = W.fabric(n, 6, 21)
    v = W.random_state(n, 22, _cdt(dtype))
    ref = oracle.apply_circuit(v, circ.gates, circ.theta)
    st = P.State(n, g, dtype)
    st.set_amplitudes(v)
    st.apply(circ)
    got = st.get_amplitudes()
    ok, mx, rl2 = amp_ok(got, ref, dtype)
    assert ok, (mx, rl2)
    st.close()


HAMS = {
    "rand12": lambda: (12, 2, W.random_pauli(12, 64, 4253 + 1000)),
    "jw16": lambda: (16, 3, W.jw_terms(16, 300, 31)),
    "jw18": lambda: (18, 4, W.jw_terms(18, 500, 32)),
}


@pytest.mark.parametrize("sched", [0, 1])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("name", list(HAMS))
def test_expectation_parity(P, name, dtype, sched):
    n, g, ham = HAMS[name]()
    _print(f"expectation {name} {dtype} sched={sched}")
    v = W.random_state(n, 40 + n, _cdt(dtype))
    e_ref = oracle.expectation(v, ham)
    st = P.State(n, g, dtype)
    st.set_amplitudes(v)
    e, stats = st.expectation(ham, sched=sched)
    ok, rel = energy_ok(e, e_ref, v, ham, dtype)
    assert ok, rel
    # the logical state is unchanged by the reorders
    got = st.get_amplitudes()
    assert np.max(np.abs(got - v.astype(got.dtype))) == 0
    st.close()


def test_grad_parity_small(P):
    n, g = 12, 2
    circ = W.fabric(n, 4, 51)
    ham = W.jw_terms(n, 80, 52)
    e_ref, g_ref = oracle.adjoint_grad(circ, ham)
    psi_ref = oracle.run_circuit(circ)
    for dtype in ("c64", "c128"):
        _print(f"grad {dtype}")
        st = P.State(n, g, dtype)
        st.set_basis(circ.psi0_index)
        e, grad, _ = st.grad(circ, ham)
        ok, erel = energy_ok(e, e_ref, psi_ref, ham, dtype)
        assert ok, erel
        ok, grel = grad_ok(grad, g_ref, ham, dtype)
        assert ok, (dtype, grel)
        st.close()


def test_qr_many_pairs_small_n(P):
    """Relayouts that pair most bits (tile of the QR kernel filled with whole
    pairs) on the smallest states."""
    import torch
    for n, g in ((8, 0), (9, 1), (10, 2), (11, 3)):
        rng = np.random.default_rng(100 + n)
        v = W.random_state(n, 7 + n, np.complex64)
        buf = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
        st = P.State(n, g, "c64", buf=buf)
        st.set_amplitudes(v)
        pos = list(range(n))
        for _ in range(3):
            new = [int(x) for x in rng.permutation(n)]
            before = buf.cpu().numpy().copy()
            st.qr_permute(new)
            torch.cuda.synchronize()
            assert np.array_equal(buf.cpu().numpy(), oracle.qr_permute(before, pos, new))
            pos = new
        st.close()


ANGLES = [-3 * math.pi, -math.pi, -math.pi / 2 - 1e-3, -1e-7, 0.0, 1e-7, math.pi / 2 + 1e-3,
          math.pi, 2 * math.pi, 2.5 * math.pi, 7.0]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_unit_modulus_ops_at_boundary_angles(P, dtype):
    """Rotations and phases near the points where the in-place kernels switch
    between R(a) and -R(a - pi) (|a| = pi/2), at zero, at multiples of pi and
    beyond one period, for every unit-modulus kind, on a dense random state."""
    n, g = 13, 2
    gates, theta = [], []
    kinds1 = ["RY", "RZ"]
    kinds2 = ["GIVENS", "CPHASE"]
    for i, a in enumerate(ANGLES):
        q = i % n
        for kd in kinds1:
            gates.append((kd, (q,), len(theta)))
            theta.append(a)
        for kd in kinds2:
            gates.append((kd, (q, (q + 5) % n), len(theta)))
            theta.append(a)
        gates.append(("CZ", ((q + 1) % n, (q + 7) % n), -1))
        for kd in ("Z", "S", "T"):
            gates.append((kd, ((q + 3) % n,), -1))
    circ = W.Circuit(n, gates, np.array(theta), 0)
    v = W.random_state(n, 77, _cdt(dtype))
    ref = oracle.apply_circuit(v, circ.gates, circ.theta)
    _print(f"boundary angles {dtype}")
    for sched in (P.LAZY, P.EAGER):
        st = P.State(n, g, dtype)
        st.set_amplitudes(v)
        st.apply(circ, sched=sched)
        assert np.max(np.abs(st.get_amplitudes() - ref)) < AMP[dtype]
        st.close()
    # the adjoint sweep applies the inverses of the same ops
    ham = W.jw_terms(n, 60, 78)
    circ0 = W.Circuit(n, gates, np.array(theta), 5)
    e_ref, g_ref = oracle.adjoint_grad(circ0, ham)
    st = P.State(n, g, dtype)
    st.set_basis(5)
    e, grad, _ = st.grad(circ0, ham)
    st.close()
    ok, erel = energy_ok(e, e_ref, None, ham, dtype)
    assert ok, erel
    ok, grel = grad_ok(grad, g_ref, ham, dtype)
    assert ok, grel


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("swaps", [((7, 12), (8, 13)), ((6, 11),), ((1, 12), (9, 13)),
                                   ((0, 13), (10, 12), (6, 11))],
                         ids=["rows-2", "rows-1", "tiles-inner-outer", "tiles-mixed"])
def test_qr_paths_with_outer_pairs(P, dtype, swaps):
    """Reorders that take the rows path (every exchanged bit at 6 or above)
    and the tile path with pairs outside the tile, where only the rows or
    tiles that can be the smaller side of their pair are launched."""
    import torch
    n, g = 14, 3
    v = W.random_state(n, 90 + len(swaps), np.complex64 if dtype == "c64" else np.complex128)
    buf = torch.empty(1 << n, dtype=torch.complex64 if dtype == "c64" else torch.complex128,
                      device="cuda")
    st = P.State(n, g, dtype, buf=buf)
    st.set_amplitudes(v)
    pos = list(range(n))
    phys = list(range(n))
    for a, b in swaps:
        phys[a], phys[b] = phys[b], phys[a]
    new = [phys[p] for p in pos]
    _print(f"qr paths {swaps} {dtype}")
    before = buf.cpu().numpy().copy()
    st.qr_permute(new)
    torch.cuda.synchronize()
    assert np.array_equal(buf.cpu().numpy(), oracle.qr_permute(before, pos, new))
    np.testing.assert_array_equal(st.get_amplitudes(), v)
    st.close()


def _haar(rng, d):
    z = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def _dense_circuit(n, seed):
    """Dense U1/U2 blocks (Haar-random unitaries, row-major, q[0] the least
    significant bit of the local index) between RY/GIVENS layers."""
    rng = np.random.default_rng(seed)
    gates, theta = [], []
    for layer in range(3):
        for q in range(0, n - 1, 2):
            gates.append(("U2", (q + layer % 2, (q + 3) % n), -1, _haar(rng, 4)))
        for q in range(n):
            gates.append(("U1", (q,), -1, _haar(rng, 2)))
            gates.append(("RY", (q,), len(theta)))
            theta.append(float(rng.uniform(-math.pi, math.pi)))
        for q in range(0, n - 2, 3):
            gates.append(("GIVENS", (q, q + 2), len(theta)))
            theta.append(float(rng.uniform(-math.pi, math.pi)))
    return gates, np.array(theta)


def _oracle_run(n, gates, theta, psi):
    for gt in gates:
        kind, qs, p = gt[0], gt[1], gt[2]
        if kind in ("U1", "U2"):
            psi = oracle.apply_gate(psi, kind, qs, umat=gt[3])
        else:
            psi = oracle.apply_gate(psi, kind, qs, angle=theta[p] if p >= 0 else 0.0)
    return psi


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_dense_matrix_gates_forward_and_gradient(P, dtype):
    """U1/U2 user matrices through the C ABI: forward parity under both
    schedules, and the adjoint gradient (which applies their conjugate
    transposes) against the oracle's exact parameter-shift gradient."""
    n, g = 11, 2
    gates, theta = _dense_circuit(n, 404)
    psi0 = oracle.basis_state(n, 3)
    ref = _oracle_run(n, gates, theta, psi0)
    _print(f"dense gates {dtype}")
    for sched in (P.LAZY, P.EAGER):
        st = P.State(n, g, dtype)
        st.set_basis(3)
        st.apply_gates(gates, theta=theta, sched=sched)
        assert np.max(np.abs(st.get_amplitudes() - ref)) < AMP[dtype]
        st.close()
    ham = W.jw_terms(n, 40, 405)
    kind_of = {gt[2]: gt[0] for gt in gates if gt[2] >= 0}
    g_ref = np.zeros(len(theta))
    for p in range(len(theta)):
        for shift, w in oracle.SHIFT_RULES[kind_of[p]]:
            for sgn in (+1, -1):
                th = theta.copy()
                th[p] += sgn * shift
                g_ref[p] += sgn * w * oracle.expectation(_oracle_run(n, gates, th, psi0), ham)
    circ = W.Circuit(n, gates, theta, 3)
    st = P.State(n, g, dtype)
    st.set_basis(3)
    e, grad, _ = st.grad(circ, ham)
    st.close()
    ok, rel = energy_ok(e, oracle.expectation(ref, ham), ref, ham, dtype)
    assert ok, rel
    ok, grel = grad_ok(grad, g_ref, ham, dtype)
    assert ok, grel


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("k", [8, 9, 10, 11, 12, 13, 14])
def test_expectation_every_tile_width(P, dtype, k, monkeypatch):
    """E through the Pauli pass with its tile forced to 2^k amplitudes (2^13
    at most for complex128), against the oracle: k = 8 and 9 give 2- and
    4-pair cubes, k >= 10 8-pair cubes; groups with one to many strings
    exercise the first-four-terms load and the four-at-a-time loop."""
    n, g = 15, 1
    ham = W.jw_terms(n, 300, 508 + k)
    v = W.random_state(n, 509 + k, np.complex64 if dtype == "c64" else np.complex128)
    monkeypatch.setenv("SVQ_EVC_K", str(k))
    st = P.State(n, g, dtype)
    st.set_amplitudes(v)
    st.qr_permute([int(x) for x in np.random.default_rng(510 + k).permutation(n)])
    _print(f"expectation tile k={k} {dtype}")
    e, stats = st.expectation(ham)
    assert stats.tile_k == (min(k, 13) if dtype == "c128" else k)
    ok, rel = energy_ok(e, oracle.expectation(v.astype(np.complex128), ham), None, ham, dtype)
    assert ok, rel
    st.close()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("k", [8, 9, 10, 11, 12, 13])
def test_apply_hamiltonian_every_tile_width(P, dtype, k, monkeypatch):
    """lambda = H psi with the H|psi> tile forced to 2^k amplitudes, against
    the oracle: k = 8 gives each thread a 4-entry spectrum, k = 9 an 8-entry
    one, k >= 10 a 16-entry one, so every batch width of the pass's output
    reads and every spectrum size of the XOR-shifted term signs runs."""
    n, g = 14, 1
    ham = W.jw_terms(n, 150, 505 + k)
    v = W.random_state(n, 506 + k, np.complex64 if dtype == "c64" else np.complex128)
    ref = oracle.hpsi(v.astype(np.complex128), ham)
    monkeypatch.setenv("SVQ_EVC_K", str(k))
    st = P.State(n, g, dtype)
    out = P.State(n, g, dtype)
    st.set_amplitudes(v)
    st.qr_permute([int(x) for x in np.random.default_rng(507 + k).permutation(n)])
    out.qr_permute(st.layout())
    _print(f"apply_hamiltonian tile k={k} {dtype}")
    P.sv_apply_hamiltonian(st.h, P.paulis_array(ham), len(ham.coef), out.h)
    got = out.get_amplitudes()
    assert np.max(np.abs(got - ref)) <= AMP[dtype] * max(1.0, float(np.abs(ham.coef).sum()))
    st.close()
    out.close()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("case", ["jw15", "random9-wide"])
def test_apply_hamiltonian_parity(P, dtype, case):
    """lambda = H psi through sv_apply_hamiltonian (the adjoint seed) on a
    dense random state in a permuted layout; the random 9-qubit strings
    include X/Y supports wider than the local qubits (direct kernel)."""
    if case == "jw15":
        n, g, ham = 15, 3, W.jw_terms(15, 200, 501)
    else:
        n, g, ham = 9, 1, W.random_pauli(9, 60, 502)
    v = W.random_state(n, 503, np.complex64 if dtype == "c64" else np.complex128)
    ref = oracle.hpsi(v.astype(np.complex128), ham)
    st = P.State(n, g, dtype)
    out = P.State(n, g, dtype)
    st.set_amplitudes(v)
    st.qr_permute([int(x) for x in np.random.default_rng(504).permutation(n)])
    out.qr_permute(st.layout())
    _print(f"apply_hamiltonian {case} {dtype}")
    P.sv_apply_hamiltonian(st.h, P.paulis_array(ham), len(ham.coef), out.h)
    got = out.get_amplitudes()
    # each output sums up to n_terms products a_t * psi: the amplitude
    # tolerance scales with the Hamiltonian's 1-norm
    assert np.max(np.abs(got - ref)) <= AMP[dtype] * max(1.0, float(np.abs(ham.coef).sum()))
    assert np.max(np.abs(st.get_amplitudes() - v)) == 0
    st.close()
    out.close()
