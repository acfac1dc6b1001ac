"""QSU-based EVC (the comparison method: Pauli strings applied as gates in
index order with ad hoc reordering, then one inner product) against the
oracle and against the Pauli-basis EVC."""
import numpy as np
import pytest

import oracle
import workloads as W
from tolerances import energy_ok

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_2410_04252_amd as P
    torch.cuda.set_device(0)
    return P


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n,g,nt,seed", [(12, 2, 150, 61), (16, 4, 400, 62), (17, 5, 300, 63)])
def test_qsu_evc_matches_oracle(P, dtype, n, g, nt, seed):
    print(f"qsu evc n={n} g={g} terms={nt} {dtype}", flush=True)
    ham = W.jw_terms(n, nt, seed)
    v = W.random_state(n, seed + 1, np.complex64 if dtype == "c64" else np.complex128)
    ref = oracle.expectation(v.astype(np.complex128), ham)
    st = P.State(n, g, dtype)
    st.set_amplitudes(v)
    e, stats = st.expectation_qsu(ham)
    ok, rel = energy_ok(e, ref, None, ham, dtype)
    assert ok, rel
    sup = [tuple(q for q in range(n) if (int(x) >> q) & 1) for x in ham.x]
    assert stats.n_qr == P.sv_plan_ops(n, n - g, sup, P.PLAN_ADHOC_INDEX)["n_qr"]
    # the reorders left the state intact (layout tracked by the handle)
    got = st.get_amplitudes()
    assert np.abs(got - v).max() == 0.0
    e2, _ = st.expectation(ham)
    ok, rel = energy_ok(e2, e, None, ham, dtype)
    assert ok, rel
    st.close()


def test_qsu_evc_empty_and_diagonal(P):
    n, g = 12, 2
    st = P.State(n, g, "c64")
    v = W.random_state(n, 5, np.complex64)
    st.set_amplitudes(v)
    empty = W.Hamiltonian(n, np.zeros(0, np.uint64), np.zeros(0, np.uint64), np.zeros(0))
    e, stats = st.expectation_qsu(empty)
    assert e == 0.0 and stats.n_qr == 0
    diag = W.Hamiltonian(n, np.zeros(3, np.uint64), np.array([0, 5, 1 << 11], np.uint64),
                         np.array([0.5, -0.25, 1.0]))
    e, stats = st.expectation_qsu(diag)
    ref = oracle.expectation(v.astype(np.complex128), diag)
    assert stats.n_qr == 0
    ok, rel = energy_ok(e, ref, None, diag, "c64")
    assert ok, rel
    st.close()


def test_qsu_evc_fabric30_product_state_subset(P):
    """30 qubits (the benchmark's size), a 64-term sample of the 2000-term JW
    Hamiltonian, on a product state whose <P> factorises per site."""
    import math
    cfg = W.config("fabric30")
    ham, g = cfg["ham"], cfg["g"]
    n = ham.n
    rng = np.random.default_rng(30)
    pick = np.sort(rng.choice(len(ham.coef), size=64, replace=False))
    sub = W.Hamiltonian(n, ham.x[pick], ham.z[pick], ham.coef[pick])
    circ, t, f = W.product_state_circuit(n, 3131)
    want = 0.0
    for k in range(len(sub.coef)):
        x, z = int(sub.x[k]), int(sub.z[k])
        val = 1.0
        for q in range(n):
            xb, zb = (x >> q) & 1, (z >> q) & 1
            if xb and zb:
                val *= math.sin(t[q]) * math.sin(f[q])
            elif xb:
                val *= math.sin(t[q]) * math.cos(f[q])
            elif zb:
                val *= math.cos(t[q])
        want += sub.coef[k] * val
    print("qsu evc fabric30 subset", flush=True)
    st = P.State(n, g, "c64")
    st.set_basis(0)
    st.apply(circ)
    e, stats = st.expectation_qsu(sub)
    ok, rel = energy_ok(e, want, None, sub, "c64")
    assert ok, (e, want, rel)
    st.close()
