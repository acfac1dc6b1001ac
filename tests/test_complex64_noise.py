"""The size of complex64 rounding error, measured without the GPU: circuits
evaluated in plain complex64 numpy arithmetic (every gate a complex64 tensor
contraction with its matrix; H|psi>, energies and gradient sums in float64).
These fix the floor of the parity bounds in tolerances.py: each case misses
the bound without the floor (or with a floor ten times smaller) and meets it
with the floor.  No HIP code is involved."""
import numpy as np

import oracle
import workloads as W
from oracle import brute
from tolerances import ENERGY_REL, GRAD_REL, energy_ok, grad_ok


def _apply(psi, n, qubits, M):
    """complex64 psi <- M on `qubits` (local index bit j = qubit qubits[j])."""
    d = len(qubits)
    t = psi.reshape([2] * n)
    Mt = M.astype(np.complex64).reshape([2] * (2 * d))
    # tensor axes of M: local bit d-1 first; state axis of qubit q is n-1-q
    Mt = Mt.transpose(list(range(d))[::-1] + list(range(d, 2 * d))[::-1])
    out = np.tensordot(Mt, t, axes=(list(range(d, 2 * d)), [n - 1 - q for q in qubits]))
    out = np.moveaxis(out, list(range(d)), [n - 1 - q for q in qubits])
    return np.ascontiguousarray(out, dtype=np.complex64).reshape(-1)


def _angle(gt, theta):
    return theta[gt[2]] if gt[2] >= 0 else 0.0


def _state32(circ):
    psi = np.zeros(1 << circ.n, np.complex64)
    psi[circ.psi0_index] = 1
    for gt in circ.gates:
        psi = _apply(psi, circ.n, gt[1], brute.gate(gt[0], _angle(gt, circ.theta)))
    return psi


def _adjoint32(circ, ham):
    """The adjoint recursion with complex64 states."""
    psi = _state32(circ)
    lam = oracle.hpsi(psi.astype(np.complex128), ham).astype(np.complex64)
    grad = np.zeros(circ.n_params)
    for gt in reversed(circ.gates):
        M = brute.gate(gt[0], _angle(gt, circ.theta))
        if gt[2] >= 0:
            kpsi = _apply(psi, circ.n, gt[1], brute.generator(gt[0]))
            grad[gt[2]] += 2 * np.vdot(lam.astype(np.complex128), kpsi.astype(np.complex128)).imag
        psi = _apply(psi, circ.n, gt[1], M.conj().T)
        lam = _apply(lam, circ.n, gt[1], M.conj().T)
    return grad


def test_complex64_energy_needs_the_floor():
    """A 12-qubit fabric circuit (8 layers, 200 JW-like strings): the
    complex64 energy misses 1e-6 relative to max(|E|, 1e-3 sum |a_t|) and
    meets it relative to max(|E|, 1e-2 sum |a_t|)."""
    circ, ham = W.fabric(12, 8, 9027), W.jw_terms(12, 200, 9527)
    e_ref = oracle.expectation(oracle.run_circuit(circ), ham)
    e32 = oracle.expectation(_state32(circ).astype(np.complex128), ham)
    tenth = max(abs(e_ref), 1e-3 * np.abs(ham.coef).sum())
    assert abs(e32 - e_ref) > ENERGY_REL["c64"] * tenth
    ok, rel = energy_ok(e32, e_ref, None, ham, "c64")
    assert ok, rel


def test_complex64_gradient_needs_the_floor():
    """A 13-qubit random circuit (120 gates, 30 random Pauli strings with
    N(0,1) coefficients): its gradient is small next to the Hamiltonian's
    1-norm, and the complex64 adjoint misses 1e-6 relative to ||g|| but meets
    the floored bound."""
    circ, ham = W.random_circuit(13, 120, 65), W.random_pauli(13, 30, 66)
    _, g_ref = oracle.adjoint_grad(circ, ham)
    g32 = _adjoint32(circ, ham)
    assert np.linalg.norm(g32 - g_ref) > GRAD_REL["c64"] * np.linalg.norm(g_ref)
    ok, rel = grad_ok(g32, g_ref, ham, "c64")
    assert ok, rel


def test_model_is_the_oracle_in_complex128():
    """The same contraction code in complex128 reproduces the oracle, so the
    differences above are complex64 rounding alone."""
    circ, ham = W.random_circuit(9, 60, 67), W.random_pauli(9, 20, 68)
    psi = np.zeros(1 << 9, np.complex128)
    psi[circ.psi0_index] = 1
    for gt in circ.gates:
        t = psi.reshape([2] * 9)
        M = brute.gate(gt[0], _angle(gt, circ.theta))
        d = len(gt[1])
        Mt = M.reshape([2] * (2 * d)).transpose(list(range(d))[::-1] + list(range(d, 2 * d))[::-1])
        out = np.tensordot(Mt, t, axes=(list(range(d, 2 * d)), [8 - q for q in gt[1]]))
        psi = np.ascontiguousarray(np.moveaxis(out, list(range(d)), [8 - q for q in gt[1]])).reshape(-1)
    assert np.max(np.abs(psi - oracle.run_circuit(circ))) < 1e-13
