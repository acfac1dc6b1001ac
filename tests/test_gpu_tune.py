"""The measured tuner: whatever tile width and low-bit count it picks, the
results under the tuned defaults still match the oracle."""
import numpy as np
import pytest

import oracle
import workloads as W
from tolerances import AMP, GRAD_REL, energy_ok

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
    assert ch in (16, 32, 64, 128) and lb in (3, 4, 5) and ms > 0
    b = P.Batch(inst)                  # built with the tuned values
    e, grads, _ = b.run()
    for i, (c, h) in enumerate(inst):
        e_ref, g_ref = oracle.adjoint_grad(c, h)
        ok, rel = energy_ok(e[i], e_ref, None, h, "c64")
        assert ok, (i, rel)
        assert np.linalg.norm(grads[i] - g_ref) <= GRAD_REL["c64"] * np.linalg.norm(g_ref), i
    b.close()


@pytest.mark.parametrize("k,c", [(10, 3), (11, 5), (12, 6), (13, 3), (13, 6)])
def test_every_tuner_candidate_matches_oracle(P, k, c, monkeypatch):
    """The candidates the tuner may pick (k in 10..13, c in 3..6 for gate
    passes; k in 11..14 for Pauli passes) all give the oracle's results."""
    circ = W.fabric(17, 10, 4040 + k)
    ham = W.jw_terms(17, 250, 4050 + c)
    ref = oracle.run_circuit(circ)
    monkeypatch.setenv("SVQ_TILE_K", str(k))
    monkeypatch.setenv("SVQ_LOW_BITS", str(c))
    monkeypatch.setenv("SVQ_EVC_K", str(k + 1))
    monkeypatch.setenv("SVQ_EVC_LOW_BITS", str(c))
    print(f"tuner candidate k={k} c={c}", flush=True)
    for dtype in ("c64", "c128"):
        st = P.State(17, 3, dtype)
        st.set_basis(circ.psi0_index)
        stats = st.apply(circ)
        assert stats.tile_k == k
        assert np.abs(st.get_amplitudes() - ref).max() <= AMP[dtype]
        e, _ = st.expectation(ham)
        ok, rel = energy_ok(e, oracle.expectation(ref, ham), ref, ham, dtype)
        assert ok, (dtype, rel)
        st.close()
