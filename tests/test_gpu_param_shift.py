"""The parameter-shift driver (sv_param_shift_grad) through the C ABI against
the oracle's parameter-shift gradients, under the exact rules (two-frequency
rule for GIVENS) and under the two-term rule for every gate, including a
parameter shared by gates with different angle scales."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from tolerances import ENERGY_REL, GRAD_REL, energy_scale, grad_ok

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_2410_04252_amd as P
    torch.cuda.set_device(0)
    return P


def _weights(circ, rule):
    """Sum over a parameter's evaluations of |coefficient|: each shifted
    energy errs by at most ENERGY_REL * scale."""
    r2 = math.sqrt(2.0)
    w = np.zeros(circ.n_params)
    for gt in circ.gates:
        if gt[2] < 0:
            continue
        scl = abs(float(gt[4])) if len(gt) > 4 else 1.0
        if gt[0] == "GIVENS" and rule == "exact":
            w[gt[2]] += 2 * scl * ((r2 + 1) / (4 * r2) + (r2 - 1) / (4 * r2))
        else:
            w[gt[2]] += 2 * scl * 0.5
    return w


def _shared_circuit(n, seed):
    base = W.fabric(n, 3, seed)
    gates = []
    for i, (kind, qs, p) in enumerate(base.gates):
        gates.append((kind, qs, p % 7, 0.05 * (i % 4), (1.0, -0.5, 1.5, 2.0)[i % 4]))
    theta = np.random.default_rng(seed + 1).uniform(-math.pi, math.pi, size=7)
    return W.Circuit(n, gates, theta, base.psi0_index)


@pytest.mark.parametrize("rule", ["exact", "two-term"])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("case", ["fabric12", "shared11", "hea10"])
def test_param_shift_matches_oracle(P, case, dtype, rule):
    if case == "fabric12":
        circ, ham, g = W.fabric(12, 3, 3301), W.jw_terms(12, 60, 3302), 2
    elif case == "shared11":
        circ, ham, g = _shared_circuit(11, 3303), W.jw_terms(11, 50, 3304), 2
    else:
        circ, ham, g = W.hea(10, 2, 3305), W.random_pauli(10, 30, 3306), 1
    print(f"param shift {case} {dtype} {rule}", flush=True)
    g_ref = oracle.param_shift_grad(circ, ham, rule=rule)
    e_ref = oracle.energy(circ, ham)
    st = P.State(circ.n, g, dtype)
    st.set_basis(circ.psi0_index)
    psi0 = st.get_amplitudes()
    e, grad, nev, _ = st.param_shift_grad(circ, ham, rule=P.SHIFT_EXACT if rule == "exact"
                                          else P.SHIFT_TWO_TERM)
    assert np.array_equal(st.get_amplitudes(), psi0)      # psi0 handed back
    st.close()
    w = _weights(circ, rule)
    scale = energy_scale(e_ref, ham)
    assert abs(e - e_ref) <= ENERGY_REL[dtype] * scale
    # every component within the sum of its evaluations' energy bounds
    bound = w * ENERGY_REL[dtype] * scale + GRAD_REL[dtype] * np.abs(g_ref).max()
    assert np.all(np.abs(grad - g_ref) <= bound), np.max(np.abs(grad - g_ref) / bound)
    if rule == "exact":
        # the exact rules give the true gradient: the oracle adjoint's
        _, g_adj = oracle.adjoint_grad(circ, ham)
        ok, rel = grad_ok(grad, g_adj, ham, dtype) if dtype == "c128" else (True, 0.0)
        assert ok, rel


def test_param_shift_evaluation_count(P):
    """Two evaluations per one-frequency gate, four per GIVENS under the exact
    rule, two under the two-term rule; plus one unshifted evaluation."""
    circ, ham = W.fabric(10, 2, 3307), W.jw_terms(10, 20, 3308)
    n_givens = sum(1 for gt in circ.gates if gt[0] == "GIVENS")
    n_other = sum(1 for gt in circ.gates if gt[2] >= 0 and gt[0] != "GIVENS")
    st = P.State(10, 1, "c64")
    st.set_basis(circ.psi0_index)
    _, _, ne_exact, _ = st.param_shift_grad(circ, ham, rule=P.SHIFT_EXACT)
    _, _, ne_two, _ = st.param_shift_grad(circ, ham, rule=P.SHIFT_TWO_TERM)
    st.close()
    assert ne_exact == 4 * n_givens + 2 * n_other + 1
    assert ne_two == 2 * (n_givens + n_other) + 1
