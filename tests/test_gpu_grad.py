"""GPU gradient parity: adjoint sweep through the C ABI and through
torch.autograd against the oracle's adjoint, finite differences and
parameter-shift."""
import numpy as np
import pytest

import oracle
import workloads as W
from tolerances import AMP, energy_ok, grad_ok

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    torch.cuda.set_device(0)
    return torch


def _print(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("make", ["fabric", "hea", "random"])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("sched", [0, 1])
def test_adjoint_grad_vs_oracle(torch_mod, make, dtype, sched):
    import paper_2410_04252_amd as P
    _print(f"grad {make} {dtype} sched={sched}")
    if make == "fabric":
        circ, ham, g = W.fabric(14, 6, 61), W.jw_terms(14, 120, 62), 3
    elif make == "hea":
        circ, ham, g = W.hea(12, 3, 63), W.random_pauli(12, 40, 64), 2
    else:
        circ, ham, g = W.random_circuit(13, 120, 65), W.random_pauli(13, 30, 66), 3
    e_ref, g_ref = oracle.adjoint_grad(circ, ham)
    st = P.State(circ.n, g, dtype)
    st.set_basis(circ.psi0_index)
    e, grad, stats = st.grad(circ, ham, sched=sched)
    ok, grel = grad_ok(grad, g_ref, ham, dtype)
    assert ok, grel
    ok, rel = energy_ok(e, e_ref, oracle.run_circuit(circ), ham, dtype)
    assert ok, rel
    # the reverse sweep hands back psi0
    psi0 = st.get_amplitudes()
    want = np.zeros(1 << circ.n); want[circ.psi0_index] = 1.0
    assert np.max(np.abs(psi0 - want)) < AMP[dtype]
    st.close()


def test_grad_vs_fd_and_shift_oracle(torch_mod):
    import paper_2410_04252_amd as P
    circ, ham = W.fabric(10, 6, 71), W.jw_terms(10, 80, 72)
    st = P.State(10, 2, "c128")
    st.set_basis(circ.psi0_index)
    _, grad, _ = st.grad(circ, ham)
    gf = oracle.fd_grad(circ, ham)
    gs = oracle.param_shift_grad(circ, ham)
    assert np.max(np.abs(grad - gs)) < 1e-11
    assert np.max(np.abs(grad - gf)) < 1e-7
    st.close()


def test_autograd_function(torch_mod):
    torch = torch_mod
    from paper_2410_04252_amd.autograd import Problem, vqe_energy
    circ, ham = W.fabric(12, 6, 81), W.jw_terms(12, 100, 82)
    e_ref, g_ref = oracle.adjoint_grad(circ, ham)
    prob = Problem(circ, ham, g=2, dtype="c64")
    theta = torch.tensor(circ.theta, dtype=torch.float64, requires_grad=True)
    e = vqe_energy(theta, prob)
    (2.0 * e).backward()
    ok, rel = energy_ok(e.item(), e_ref, oracle.run_circuit(circ), ham, "c64")
    assert ok, rel
    got = theta.grad.numpy()
    ok, grel = grad_ok(got / 2, g_ref, ham, "c64")
    assert ok, grel
    prob.close()


def test_autograd_gradcheck_c128(torch_mod):
    torch = torch_mod
    from paper_2410_04252_amd.autograd import Problem, VQEEnergy
    circ, ham = W.fabric(9, 4, 91), W.jw_terms(9, 40, 92)
    prob = Problem(circ, ham, g=1, dtype="c128")
    theta = torch.tensor(circ.theta, dtype=torch.float64, requires_grad=True)
    assert torch.autograd.gradcheck(lambda t: VQEEnergy.apply(t, prob), (theta,), eps=1e-6,
                                    atol=1e-7, rtol=1e-5)
    prob.close()
