"""Pins of the CPU oracle against what the paper and the mathematics fix:
brute-force Kronecker products, closed forms, invariants and special cases.
None of these re-uses the oracle's own formulas."""
import math

import numpy as np
import pytest

import oracle
from oracle import brute
import workloads as W

ALL_KINDS = ["H", "X", "Y", "Z", "S", "T", "RX", "RY", "RZ",
             "CNOT", "CZ", "CPHASE", "GIVENS", "SWAP"]


def _full_from_oracle(n, kind, qubits, angle):
    cols = [oracle.apply_gate(oracle.basis_state(n, j), kind, qubits, angle) for j in range(1 << n)]
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("kind", ALL_KINDS)
def test_gate_matrix_vs_generator_expm(kind):
    """Each oracle gate equals the brute-force operator (expm of the generator
    for parametric gates, projector sums for fixed ones) on every basis state."""
    rng = np.random.default_rng(11)
    n = 3
    for _ in range(3):
        ang = float(rng.uniform(-math.pi, math.pi))
        ar = 2 if kind in ("CNOT", "CZ", "CPHASE", "GIVENS", "SWAP") else 1
        qs = tuple(int(v) for v in rng.choice(n, size=ar, replace=False))
        got = _full_from_oracle(n, kind, qs, ang)
        want = brute.embed(n, brute.gate(kind, ang), qs)
        np.testing.assert_allclose(got, want, atol=1e-13)


def test_gate_special_values():
    """Textbook special cases: RY(pi)|0> = |1>, RX(pi) = -iX, Givens(pi)
    maps |a=1,b=0> to |a=0,b=1>, CPHASE(pi) = CZ."""
    v = oracle.apply_gate(oracle.basis_state(1, 0), "RY", (0,), math.pi)
    np.testing.assert_allclose(v, [0, 1], atol=1e-15)
    v = oracle.apply_gate(oracle.basis_state(1, 0), "RX", (0,), math.pi)
    np.testing.assert_allclose(v, [0, -1j], atol=1e-15)
    v = oracle.apply_gate(oracle.basis_state(2, 1), "GIVENS", (0, 1), math.pi)
    np.testing.assert_allclose(v, [0, 0, 1, 0], atol=1e-15)
    a = _full_from_oracle(2, "CPHASE", (0, 1), math.pi)
    b = _full_from_oracle(2, "CZ", (0, 1), 0.0)
    np.testing.assert_allclose(a, b, atol=1e-15)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_random_circuit_vs_kron(seed):
    n = 7
    c = W.random_circuit(n, 40, seed)
    psi0 = W.random_state(n, seed + 100)
    got = oracle.apply_circuit(psi0, c.gates, c.theta)
    want = brute.circuit_unitary(n, c.gates, c.theta) @ psi0
    np.testing.assert_allclose(got, want, atol=1e-12)


def test_hea12_vs_kron_small():
    c = W.hea(8, 2, 5)
    psi = oracle.run_circuit(c)
    want = brute.circuit_unitary(8, c.gates, c.theta)[:, 0]
    np.testing.assert_allclose(psi, want, atol=1e-12)


def test_fabric_vs_kron():
    c = W.fabric(8, 4, 6)
    psi = oracle.run_circuit(c)
    e0 = np.zeros(256, dtype=complex); e0[c.psi0_index] = 1
    want = brute.circuit_unitary(8, c.gates, c.theta) @ e0
    np.testing.assert_allclose(psi, want, atol=1e-12)


def test_pauli_and_expectation_vs_kron():
    n = 6
    h = W.random_pauli(n, 20, 3)
    psi = W.random_state(n, 9)
    Hm = brute.hamiltonian_matrix(n, h)
    e, im = oracle.expectation(psi, h, with_imag=True)
    want = np.vdot(psi, Hm @ psi)
    assert abs(e - want.real) < 1e-12
    assert abs(im) < 1e-12 and abs(want.imag) < 1e-12
    for t in range(len(h)):
        np.testing.assert_allclose(oracle.pauli_apply(psi, int(h.x[t]), int(h.z[t])),
                                   brute.pauli_matrix(n, int(h.x[t]), int(h.z[t])) @ psi,
                                   atol=1e-13)
    np.testing.assert_allclose(oracle.hpsi(psi, h), Hm @ psi, atol=1e-12)


def test_jw_expectation_vs_kron():
    n = 8
    h = W.jw_terms(n, 60, 4)
    psi = W.random_state(n, 10)
    want = np.vdot(psi, brute.hamiltonian_matrix(n, h) @ psi).real
    assert abs(oracle.expectation(psi, h) - want) < 1e-12


def _ghz(n):
    gates = [("H", (0,), -1)] + [("CNOT", (q, q + 1), -1) for q in range(n - 1)]
    return oracle.apply_circuit(oracle.basis_state(n, 0), gates, np.zeros(0))


@pytest.mark.parametrize("n", [3, 12, 20])
def test_ghz_closed_form(n):
    psi = _ghz(n)
    r = 1 / math.sqrt(2)
    assert abs(psi[0] - r) < 1e-14 and abs(psi[-1] - r) < 1e-14
    assert abs(np.vdot(psi, psi).real - 1) < 1e-13
    full = (1 << n) - 1
    terms = W.Hamiltonian(n, np.array([0, full, 0, 0], dtype=np.uint64),
                          np.array([(1 << 0) | (1 << (n - 1)), 0, 1, 1 << (n // 2)], dtype=np.uint64),
                          np.array([1.0, 0.0, 0.0, 0.0]))
    for t, want in enumerate([1.0, 1.0, 0.0, 0.0]):
        one = W.Hamiltonian(n, terms.x[t:t + 1], terms.z[t:t + 1], np.array([1.0]))
        assert abs(oracle.expectation(psi, one) - want) < 1e-12


@pytest.mark.parametrize("n,x", [(5, 0), (5, 19), (8, 201)])
def test_qft_closed_form(n, x):
    """QFT|x> = 2^{-n/2} sum_y exp(2 pi i x y / 2^n)|y> built from H, controlled
    phases CPHASE(pi/2^k) and a final qubit reversal by SWAPs."""
    gates = []
    for j in reversed(range(n)):
        gates.append(("H", (j,), -1))
        for k in reversed(range(j)):
            gates.append(("CPHASE", (k, j), -1, math.pi / 2 ** (j - k)))
    for j in range(n // 2):
        gates.append(("SWAP", (j, n - 1 - j), -1))
    psi = oracle.apply_circuit(oracle.basis_state(n, x), gates, np.zeros(0))
    y = np.arange(1 << n)
    want = np.exp(2j * math.pi * x * y / (1 << n)) / math.sqrt(1 << n)
    np.testing.assert_allclose(psi, want, atol=1e-12)


@pytest.mark.parametrize("n", [6, 16])
def test_product_state_closed_form(n):
    """prod_q RZ(f_q) RY(t_q)|0>: <P> = prod over sites of e(X) = sin t cos f,
    e(Y) = sin t sin f, e(Z) = cos t."""
    c, t, f = W.product_state_circuit(n, 21)
    psi = oracle.run_circuit(c)
    h = W.random_pauli(n, 12, 22)
    for k in range(len(h)):
        x, z = int(h.x[k]), int(h.z[k])
        want = 1.0
        for q in range(n):
            xb, zb = (x >> q) & 1, (z >> q) & 1
            if xb and zb:
                want *= math.sin(t[q]) * math.sin(f[q])
            elif xb:
                want *= math.sin(t[q]) * math.cos(f[q])
            elif zb:
                want *= math.cos(t[q])
        one = W.Hamiltonian(n, h.x[k:k + 1], h.z[k:k + 1], np.array([1.0]))
        assert abs(oracle.expectation(psi, one) - want) < 1e-12


def test_unitarity_and_inverse():
    n = 9
    c = W.random_circuit(n, 60, 44)
    psi0 = W.random_state(n, 45)
    psi = oracle.apply_circuit(psi0, c.gates, c.theta)
    assert abs(np.vdot(psi, psi).real - 1) < 1e-12
    back = psi
    for kind, qs, p in reversed(c.gates):
        back = oracle.apply_gate(back, kind, qs, c.theta[p] if p >= 0 else 0.0, dagger=True)
    np.testing.assert_allclose(back, psi0, atol=1e-12)


def test_basis_state_pauli_special_case():
    """<b|P|b> = 0 if x != 0 else (-1)^{popcount(b & z)}."""
    n = 7
    h = W.random_pauli(n, 30, 5)
    for b in (0, 5, 77, 127):
        psi = oracle.basis_state(n, b)
        for k in range(len(h)):
            x, z = int(h.x[k]), int(h.z[k])
            one = W.Hamiltonian(n, h.x[k:k + 1], h.z[k:k + 1], np.array([1.0]))
            want = 0.0 if x else (-1.0) ** bin(b & z).count("1")
            assert abs(oracle.expectation(psi, one) - want) < 1e-14


def test_chunk_partials_aggregate_and_sign():
    """eq. aggregation: sum_j E_j = E.  eq. par_exp: for P = P_G (x) P_L with
    P_G in {I,Z} on the g global qubits, E = sum_j s_j <psi_j|P_L|psi_j>."""
    n, g = 8, 2
    psi = W.random_state(n, 3)
    h = W.jw_terms(n, 40, 8)
    e, parts = oracle.expectation(psi, h, g=g, with_chunks=True)
    assert abs(parts.sum() - e) < 1e-12
    nl = n - g
    zg = (1 << (n - 1)) | (1 << nl)          # Z on both global qubits
    xl, zl = 0b000101, 0b000110               # a local part with X, Y, Z
    full = W.Hamiltonian(n, np.array([xl], dtype=np.uint64), np.array([zl | zg], dtype=np.uint64),
                         np.array([1.0]))
    local = W.Hamiltonian(nl, np.array([xl], dtype=np.uint64), np.array([zl], dtype=np.uint64),
                          np.array([1.0]))
    acc = 0.0
    for j in range(1 << g):
        sub = psi[j << nl:(j + 1) << nl]
        s = (-1) ** bin(j & 0b11).count("1")
        acc += s * oracle.expectation(sub, local)
    assert abs(acc - oracle.expectation(psi, full)) < 1e-12


def test_chunk_partials_follow_layout():
    """Chunk sums under a permuted layout equal the chunk sums of the permuted
    buffer evaluated in identity layout."""
    n, g = 7, 2
    psi = W.random_state(n, 31)
    h = W.jw_terms(n, 25, 9)
    pos = [3, 0, 6, 1, 4, 2, 5]
    _, parts = oracle.expectation(psi, h, g=g, pos=pos, with_chunks=True)
    buf = oracle.qr_permute(oracle.to_logical(psi, list(range(n))), list(range(n)), pos)
    # evaluate each chunk directly from the physical buffer
    inv = [0] * n
    for q in range(n):
        inv[pos[q]] = q
    acc = np.zeros(1 << g)
    for t in range(len(h)):
        ph = oracle.pauli_apply(psi, int(h.x[t]), int(h.z[t]))
        ph_buf = oracle.qr_permute(ph, list(range(n)), pos)
        prod = np.conj(buf) * ph_buf
        acc += h.coef[t] * prod.reshape(1 << g, -1).sum(axis=1).real
    np.testing.assert_allclose(parts, acc, atol=1e-12)


def test_qr_transpose_vs_index_loop():
    """The transpose-based QR oracle against an explicit per-index loop."""
    n = 6
    rng = np.random.default_rng(3)
    buf = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    pos_old = list(rng.permutation(n))
    pos_new = list(rng.permutation(n))
    got = oracle.qr_permute(buf, pos_old, pos_new)
    want = np.zeros_like(buf)
    for i in range(1 << n):         # i is a logical index
        po = sum(((i >> q) & 1) << pos_old[q] for q in range(n))
        pn = sum(((i >> q) & 1) << pos_new[q] for q in range(n))
        want[pn] = buf[po]
    np.testing.assert_array_equal(got, want)


def test_qr_involution_and_moved_fraction():
    """A QR that exchanges s local/global bit pairs is an involution and moves
    exactly the fraction 1 - 2^{-s} of the elements."""
    n = 10
    rng = np.random.default_rng(4)
    buf = rng.normal(size=1 << n) + 0j
    for pairs in ([(1, 9)], [(0, 8), (3, 9)], [(2, 7), (4, 8), (5, 9)]):
        pos = list(range(n))
        new = list(range(n))
        for a, b in pairs:
            new[a], new[b] = b, a
        once = oracle.qr_permute(buf, pos, new)
        twice = oracle.qr_permute(once, pos, new)
        np.testing.assert_array_equal(twice, buf)
        moved = np.count_nonzero(once != buf) / buf.size
        assert abs(moved - (1 - 2.0 ** -len(pairs))) < 1e-12


def test_grad_closed_form_ry():
    """RY(t)|0> with H = Z: E = cos t, dE/dt = -sin t."""
    for t0 in (0.3, 1.7, -2.4):
        c = W.Circuit(1, [("RY", (0,), 0)], np.array([t0]), 0)
        h = W.Hamiltonian(1, np.array([0], dtype=np.uint64), np.array([1], dtype=np.uint64),
                          np.array([1.0]))
        e, g = oracle.adjoint_grad(c, h)
        assert abs(e - math.cos(t0)) < 1e-14
        assert abs(g[0] + math.sin(t0)) < 1e-13
        assert abs(oracle.param_shift_grad(c, h)[0] + math.sin(t0)) < 1e-13
        assert abs(oracle.fd_grad(c, h)[0] + math.sin(t0)) < 1e-8


@pytest.mark.parametrize("make", ["fabric", "hea", "random"])
def test_adjoint_vs_fd_vs_shift(make):
    if make == "fabric":
        c = W.fabric(8, 4, 7)
        h = W.jw_terms(8, 40, 70)
    elif make == "hea":
        c = W.hea(6, 2, 8)
        h = W.random_pauli(6, 20, 80)
    else:
        c = W.random_circuit(6, 30, 9)
        h = W.random_pauli(6, 20, 90)
    e, ga = oracle.adjoint_grad(c, h)
    assert abs(e - oracle.energy(c, h)) < 1e-12
    gs = oracle.param_shift_grad(c, h)
    gf = oracle.fd_grad(c, h)
    np.testing.assert_allclose(ga, gs, atol=1e-11)
    np.testing.assert_allclose(ga, gf, atol=1e-7)


def test_givens_two_frequency_shift_rule():
    """The 4-term rule is exact for GIVENS (a 2-term rule is not)."""
    c = W.Circuit(2, [("RY", (0,), 0), ("RY", (1,), 1), ("GIVENS", (0, 1), 2)],
                  np.array([0.7, 1.9, 0.4]), 0)
    h = W.Hamiltonian(2, np.array([1, 3], dtype=np.uint64), np.array([2, 1], dtype=np.uint64),
                      np.array([0.8, -0.3]))
    gf = oracle.fd_grad(c, h)[2]
    gs = oracle.param_shift_grad(c, h)[2]
    assert abs(gf - gs) < 1e-8
    two_term = 0.5 * (oracle.energy(c, h, np.array([0.7, 1.9, 0.4 + math.pi / 2]))
                      - oracle.energy(c, h, np.array([0.7, 1.9, 0.4 - math.pi / 2])))
    assert abs(two_term - gf) > 1e-3


def _haar(rng, d):
    z = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def test_adjoint_with_dense_gates_vs_fd_and_kron():
    """Circuits with fixed U1/U2 matrices between parametric gates: the
    adjoint recursion (which applies the matrices' conjugate transposes) equals
    central finite differences, and the final state equals the Kronecker
    product of the gate matrices."""
    rng = np.random.default_rng(606)
    n = 5
    gates, p = [], 0
    for layer in range(2):
        gates.append(("U2", (layer, 3), -1, _haar(rng, 4)))
        for q in range(n):
            gates.append(("U1", (q,), -1, _haar(rng, 2)))
            gates.append(("RY", (q,), p)); p += 1
        gates.append(("GIVENS", (1, 4), p)); p += 1
        gates.append(("CPHASE", (0, 2), p)); p += 1
    c = W.Circuit(n, gates, rng.uniform(-math.pi, math.pi, size=p), 3)
    h = W.random_pauli(n, 12, 607)
    e, ga = oracle.adjoint_grad(c, h)
    assert abs(e - oracle.energy(c, h)) < 1e-12
    np.testing.assert_allclose(ga, oracle.fd_grad(c, h), atol=1e-7)
    np.testing.assert_allclose(ga, oracle.param_shift_grad(c, h), atol=1e-11)
    U = brute.circuit_unitary(n, c.gates, c.theta)
    np.testing.assert_allclose(oracle.run_circuit(c), U[:, 3], atol=1e-12)


def test_scaled_shared_parameter_chain_rule():
    """A parameter read by two gates through angle = scale * theta + offset:
    the oracle's adjoint (chain rule per gate) equals central finite
    differences of the energy in theta and the closed form of the two-gate
    product RY(a1 t + b1) RY(a2 t + b2)|0> with H = Z: E = cos(sum of angles)."""
    for a1, b1, a2, b2, t in ((0.5, 0.3, -2.0, 0.1, 0.7), (3.0, -1.0, 1.5, 0.0, -0.4)):
        c = W.Circuit(1, [("RY", (0,), 0, b1, a1), ("RY", (0,), 0, b2, a2)], np.array([t]), 0)
        h = W.Hamiltonian(1, np.array([0], dtype=np.uint64), np.array([1], dtype=np.uint64),
                          np.array([1.0]))
        e, g = oracle.adjoint_grad(c, h)
        ang = a1 * t + b1 + a2 * t + b2
        assert abs(e - math.cos(ang)) < 1e-14
        assert abs(g[0] + (a1 + a2) * math.sin(ang)) < 1e-13
        assert abs(oracle.fd_grad(c, h)[0] - g[0]) < 1e-7
        assert abs(oracle.param_shift_grad(c, h)[0] - g[0]) < 1e-13
    # on a fabric circuit with every angle scaled and shifted, parameters shared
    rng = np.random.default_rng(608)
    base = W.fabric(8, 4, 609)
    gates = [(k, q, p % 5, float(rng.uniform(-1, 1)), float(rng.choice([-2.0, 0.5, 1.5])))
             for k, q, p in base.gates]
    c = W.Circuit(8, gates, rng.uniform(-math.pi, math.pi, size=5), base.psi0_index)
    h = W.jw_terms(8, 40, 610)
    _, ga = oracle.adjoint_grad(c, h)
    np.testing.assert_allclose(ga, oracle.fd_grad(c, h), atol=1e-7)
    np.testing.assert_allclose(ga, oracle.param_shift_grad(c, h), atol=1e-11)


def test_two_term_rule_exact_for_one_frequency_gates_only():
    """The nominal two-evaluation rule equals the exact gradient for RY/RZ/
    CPHASE parameters and differs for GIVENS ones."""
    c = W.fabric(6, 2, 611)
    h = W.jw_terms(6, 30, 612)
    g_exact = oracle.param_shift_grad(c, h)
    g_two = oracle.param_shift_grad(c, h, rule="two-term")
    gf = oracle.fd_grad(c, h)
    np.testing.assert_allclose(g_exact, gf, atol=1e-7)
    for kind, _, p in c.gates:
        if kind == "CPHASE":
            assert abs(g_two[p] - gf[p]) < 1e-7
    giv = [p for kind, _, p in c.gates if kind == "GIVENS"]
    assert max(abs(g_two[p] - gf[p]) for p in giv) > 1e-4
