"""Batched VQE (one graph of level-synchronous launches, or one persistent
launch) against the oracle and against one-at-a-time evaluation."""
import os

import numpy as np
import pytest

import oracle
import workloads as W
from tolerances import grad_ok, energy_ok

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_2410_04252_amd as P
    torch.cuda.set_device(0)
    return P


def _instances(count, lo, hi, seed):
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed + i)
        n = int(rng.integers(lo, hi + 1))
        out.append((W.fabric(n, 6, seed + i), W.jw_terms(n, 60, seed + 500 + i)))
    return out


def test_batch_matches_oracle(P):
    inst = _instances(10, 10, 13, 900)
    print("batch vs oracle", flush=True)
    b = P.Batch(inst)
    e, grads, lat = b.run()
    for i, (c, h) in enumerate(inst):
        e_ref, g_ref = oracle.adjoint_grad(c, h)
        ok, rel = energy_ok(e[i], e_ref, None, h, "c64")
        assert ok, (i, rel)
        ok, grel = grad_ok(grads[i], g_ref, h, "c64")
        assert ok, (i, grel)
    assert np.all(lat > 0)
    # replay with other angles (the graph is reused, the op tables re-uploaded)
    rng = np.random.default_rng(1)
    thetas = [rng.uniform(-np.pi, np.pi, size=c.n_params) for c, _ in inst]
    e2, grads2, _ = b.run(thetas)
    for i, (c, h) in enumerate(inst):
        c2 = W.Circuit(c.n, c.gates, thetas[i], c.psi0_index)
        e_ref, g_ref = oracle.adjoint_grad(c2, h)
        ok, rel = energy_ok(e2[i], e_ref, None, h, "c64")
        assert ok, (i, rel)
        ok, grel = grad_ok(grads2[i], g_ref, h, "c64")
        assert ok, (i, grel)
    b.close()


def test_batch_equals_one_at_a_time(P):
    inst = _instances(24, 10, 18, 1900)
    print("batch vs single", flush=True)
    b = P.Batch(inst)
    e, grads, lat = b.run()
    for i, (c, h) in enumerate(inst):
        st = P.State(c.n, 0, "c64")
        st.set_basis(c.psi0_index)
        e1, g1, _ = st.grad(c, h)
        st.close()
        ok, rel = energy_ok(e[i], e1, None, h, "c64")
        assert ok, (i, rel)
        ok, grel = grad_ok(grads[i], g1, h, "c64")
        assert ok, (i, grel)
    b.close()


def test_lds_instances_with_wide_strings_match_oracle(P):
    """Instances of at most 13 qubits run in one workgroup's LDS and take any
    Pauli string, including one with X/Y on every qubit (which fits no tile
    of the tiled path), dense gates and scaled shared parameters.  200
    Jordan-Wigner-like strings per instance, the regime the complex64
    tolerance floor is set for."""
    inst = []
    for i, n in enumerate((10, 11, 12, 13)):
        base = W.fabric(n, 4, 6100 + i)
        gates = []
        for j, (kind, qs, p) in enumerate(base.gates):
            gates.append((kind, qs, p, 0.1 * (j % 3), (0.5, 1.0, -2.0)[j % 3]) if p >= 0 else (kind, qs, p))
        rng = np.random.default_rng(6200 + i)
        u = np.linalg.qr(rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2)))[0]
        gates.append(("U1", (n - 1,), -1, u))
        circ = W.Circuit(n, gates, base.theta, base.psi0_index)
        h = W.jw_terms(n, 200, 6300 + i)
        full = (1 << n) - 1
        ham = W.Hamiltonian(n, np.concatenate([h.x, np.array([full, full ^ 5], dtype=np.uint64)]),
                            np.concatenate([h.z, np.array([0b1010, full], dtype=np.uint64)]),
                            np.concatenate([h.coef, np.array([0.3, -0.2])]))
        inst.append((circ, ham))
    print("LDS instances with wide strings", flush=True)
    b = P.Batch(inst)
    e, grads, lat = b.run()
    b.close()
    for i, (c, h) in enumerate(inst):
        e_ref, g_ref = oracle.adjoint_grad(c, h)
        ok, rel = energy_ok(e[i], e_ref, None, h, "c64")
        assert ok, (i, rel)
        ok, grel = grad_ok(grads[i], g_ref, h, "c64")
        assert ok, (i, grel)
    assert np.all(lat > 0)


def test_persistent_batch_matches_level_synchronous(P, monkeypatch):
    """The persistent form (one launch, a device queue, bounded waits) gives
    the level-synchronous form's energies and gradients."""
    inst = _instances(12, 10, 15, 2500)
    print("persistent vs level-synchronous", flush=True)
    b = P.Batch(inst)
    e, grads, _ = b.run()
    b.close()
    monkeypatch.setenv("SVQ_BATCH_PERSISTENT", "1")
    b = P.Batch(inst)
    e2, grads2, lat2 = b.run()
    b.close()
    for i, (c, h) in enumerate(inst):
        ok, rel = energy_ok(e2[i], e[i], None, h, "c64")
        assert ok, (i, rel)
        ok, grel = grad_ok(grads2[i], grads[i], h, "c64")
        assert ok, (i, grel)
    assert np.all(lat2 > 0)


def test_batch_bounded_wait_expires_cleanly(P):
    """A spin limit of zero (set from the host) makes every unmet dependency
    wait give up at once: the kernel drains, the call reports EHIP and the
    batch is poisoned, or, if no wait was ever unmet, the results are right."""
    inst = _instances(16, 12, 16, 2900)
    os.environ["SVQ_BATCH_SPIN_LIMIT"] = "0"
    os.environ["SVQ_BATCH_PERSISTENT"] = "1"
    try:
        b = P.Batch(inst)
    finally:
        del os.environ["SVQ_BATCH_SPIN_LIMIT"]
        del os.environ["SVQ_BATCH_PERSISTENT"]
    try:
        e, grads, _ = b.run()
    except P.SvqError as err:
        assert err.status == -3
        with pytest.raises(P.SvqError) as e2:
            b.run()
        assert e2.value.status == -6
    else:
        c, h = inst[0]
        e_ref, _ = oracle.adjoint_grad(c, h)
        assert energy_ok(e[0], e_ref, None, h, "c64")[0]
    b.close()
