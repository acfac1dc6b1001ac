"""The measured tuner: whatever tile width and low-bit count it picks, the
results under the tuned defaults still match the oracle."""
import numpy as np
import pytest

import oracle
import workloads as W
from tolerances import AMP, amp_ok, energy_ok, grad_ok

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_2410_04252_amd as P
    torch.cuda.set_device(0)
    return P


def test_tuned_circuit_and_pauli_passes_match_oracle(P):
    circ = W.fabric(20, 16, 2020)
    ham = W.jw_terms(20, 300, 2021)
    print("tune fabric20", flush=True)
    st = P.State(20, 3, "c64")
    k, c, ms = st.tune(circ)
    assert 10 <= k <= 13 and 3 <= c <= 6 and ms > 0
    st.set_basis(circ.psi0_index)
    stats = st.apply(circ)
    assert stats.tile_k == k
    got = st.get_amplitudes()
    ref = oracle.run_circuit(circ)
    assert np.abs(got - ref).max() <= AMP["c64"]
    k2, c2, ms2 = st.tune_paulis(ham)
    assert 11 <= k2 <= 14 and 3 <= c2 <= 6 and ms2 > 0
    e, _ = st.expectation(ham)
    ok, rel = energy_ok(e, oracle.expectation(ref, ham), ref, ham, "c64")
    assert ok, rel
    st.close()


def test_tuned_batch_matches_oracle(P):
    inst = []
    for i in range(8):
        n = 10 + i % 4
        inst.append((W.fabric(n, 6, 3100 + i), W.jw_terms(n, 60, 3200 + i)))
    print("tune batch", flush=True)
    b = P.Batch(inst)
    ch, lb, ms = b.tune()
    b.close()
    assert ch in (256, 1024) and lb in (3, 4) and ms > 0
    b = P.Batch(inst)                  # built with the tuned values
    e, grads, _ = b.run()
    for i, (c, h) in enumerate(inst):
        e_ref, g_ref = oracle.adjoint_grad(c, h)
        ok, rel = energy_ok(e[i], e_ref, None, h, "c64")
        assert ok, (i, rel)
        ok, grel = grad_ok(grads[i], g_ref, h, "c64")
        assert ok, (i, grel)
    b.close()


@pytest.mark.parametrize("c", [3, 4, 5, 6])
@pytest.mark.parametrize("k", [10, 11, 12, 13])
def test_every_tuner_candidate_matches_oracle(P, k, c, monkeypatch):
    """Every candidate the tuner may pick gives the oracle's results: the 16
    gate-pass pairs (k in 10..13, c in 3..6) and, with the Pauli-pass width
    k_e = 11 + (k + c - 13) mod 4, the 16 Pauli-pass pairs (k_e in 11..14,
    c in 3..6; complex128 Pauli tiles stop at 13)."""
    circ = W.fabric(17, 10, 4040 + k)
    ham = W.jw_terms(17, 250, 4050 + c)
    ref = oracle.run_circuit(circ)
    ke = 11 + (k + c - 13) % 4
    monkeypatch.setenv("SVQ_TILE_K", str(k))
    monkeypatch.setenv("SVQ_LOW_BITS", str(c))
    monkeypatch.setenv("SVQ_EVC_K", str(ke))
    monkeypatch.setenv("SVQ_EVC_LOW_BITS", str(c))
    print(f"tuner candidate gate k={k} c={c}, Pauli k={ke} c={c}", flush=True)
    for dtype in ("c64", "c128"):
        st = P.State(17, 3, dtype)
        st.set_basis(circ.psi0_index)
        stats = st.apply(circ)
        assert stats.tile_k == k
        ok, mx, rl2 = amp_ok(st.get_amplitudes(), ref, dtype)
        assert ok, (dtype, mx, rl2)
        e, stats = st.expectation(ham)
        assert stats.tile_k == (min(ke, 13) if dtype == "c128" else ke)
        ok, rel = energy_ok(e, oracle.expectation(ref, ham), ref, ham, dtype)
        assert ok, (dtype, rel)
        st.close()
