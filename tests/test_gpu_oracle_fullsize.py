"""Oracle parity at the benchmark sizes, in the launch configuration that
bench.py times (lazy schedule, tuned tile widths and low bits):

* amplitudes of the 28-qubit (complex64 and complex128) and 30-qubit
  (complex64) fabric circuits, element by element, plus the energy of a
  sample of their Jordan-Wigner-like strings;
* all 400 components of the 24-qubit adjoint gradient, and the GPU
  parameter-shift gradient on a sample of parameters;
* 28-qubit reorders, bit for bit, on the rows path and the tile path;
* the per-chunk partial sums E_j (eq. local_evc) in a permuted layout;
* batch instances of 19 to 22 qubits.

The oracle runs on the host cores (complex128); each test prints its case
before the GPU work starts."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from tolerances import ENERGY_REL, GRAD_REL, amp_ok, energy_ok, energy_scale, grad_ok

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_2410_04252_amd as P
    torch.cuda.set_device(0)
    return P


def _print(*a):
    print(*a, flush=True)


def _oracle_state(circ, label):
    """psi = U(theta)|psi0> on the host, printing progress every 40 gates."""
    psi = oracle.basis_state(circ.n, circ.psi0_index)
    for i in range(0, len(circ.gates), 40):
        oracle.apply_circuit_inplace(psi, circ.gates[i:i + 40], circ.theta)
        _print(f"  oracle {label}: {min(i + 40, len(circ.gates))}/{len(circ.gates)} gates")
    return psi


def _sample_terms(ham, count, seed):
    rng = np.random.default_rng(seed)
    pick = np.sort(rng.choice(len(ham.coef), size=count, replace=False))
    return W.Hamiltonian(ham.n, ham.x[pick], ham.z[pick], ham.coef[pick])


_cache = {}


def _fabric28_ref():
    if "fabric28" not in _cache:
        cfg = W.config("fabric28")
        _cache["fabric28"] = _oracle_state(cfg["circuit"], "fabric28")
    return _cache["fabric28"]


@pytest.mark.timeout(400)
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_fabric28_amplitudes_match_oracle(P, dtype):
    cfg = W.config("fabric28")
    circ, ham, g = cfg["circuit"], cfg["ham"], cfg["g"]
    _print(f"fabric28 {dtype}: oracle state")
    ref = _fabric28_ref()
    _print(f"fabric28 {dtype}: GPU lazy schedule, tuned tile")
    st = P.State(circ.n, g, dtype)
    st.set_basis(circ.psi0_index)
    stats = st.apply(circ, sched=P.LAZY)
    assert stats.n_qr == 1
    sub = _sample_terms(ham, 48, 2801)
    e, _ = st.expectation(sub, sched=P.LAZY)
    got = st.get_amplitudes()
    st.close()
    ok, mx, rl2 = amp_ok(got, ref, dtype)
    _print(f"  max|dpsi| = {mx:.3e}, relative L2 = {rl2:.3e}")
    assert ok, (mx, rl2)
    del got
    e_ref = oracle.expectation(ref, sub)
    ok, rel = energy_ok(e, e_ref, None, sub, dtype)
    _print(f"  energy of 48 strings: {e:.12f} vs {e_ref:.12f} (rel {rel:.2e})")
    assert ok, rel


@pytest.mark.timeout(900)
def test_fabric30_amplitudes_match_oracle(P):
    _cache.clear()
    cfg = W.config("fabric30")
    circ, ham, g = cfg["circuit"], cfg["ham"], cfg["g"]
    _print("fabric30 c64: oracle state (about two minutes on 16 cores)")
    ref = _oracle_state(circ, "fabric30")
    _print("fabric30 c64: GPU lazy schedule, tuned tile")
    st = P.State(circ.n, g, "c64")
    st.set_basis(circ.psi0_index)
    stats = st.apply(circ, sched=P.LAZY)
    assert stats.n_qr == 2
    sub = _sample_terms(ham, 24, 3001)
    e, _ = st.expectation(sub, sched=P.LAZY)
    got = st.get_amplitudes()
    st.close()
    ok, mx, rl2 = amp_ok(got, ref, "c64")
    _print(f"  max|dpsi| = {mx:.3e}, relative L2 = {rl2:.3e}")
    assert ok, (mx, rl2)
    del got
    e_ref = oracle.expectation(ref, sub)
    ok, rel = energy_ok(e, e_ref, None, sub, "c64")
    _print(f"  energy of 24 strings: {e:.12f} vs {e_ref:.12f} (rel {rel:.2e})")
    assert ok, rel


@pytest.mark.timeout(600)
def test_grad24_all_parameters_match_oracle_adjoint(P):
    """cfg: 24 qubits, 400 parameters, 1000 strings, complex64 state with
    FP64 gradient sums, g = 5; every component against the complex128 oracle
    adjoint.  The GPU parameter-shift gradient (exact rules) on a sample of
    parameters must agree within the bound its energy errors allow."""
    cfg = W.config("grad24")
    circ, ham, g = cfg["circuit"], cfg["ham"], cfg["g"]
    assert circ.n_params == 400
    _print("grad24: oracle adjoint gradient")
    e_ref, g_ref = oracle.adjoint_grad(circ, ham)
    _print("grad24: GPU adjoint")
    st = P.State(circ.n, g, "c64")
    st.set_basis(circ.psi0_index)
    e, grad, _ = st.grad(circ, ham)
    ok, grel = grad_ok(grad, g_ref, ham, "c64")
    rel = np.linalg.norm(grad - g_ref) / np.linalg.norm(g_ref)
    _print(f"  gradient error {grel:.3e} of the bound's scale, {rel:.3e} relative to ||g||, "
           f"max component error {np.abs(grad - g_ref).max():.3e}")
    assert ok, grel
    ok, erel = energy_ok(e, e_ref, None, ham, "c64")
    assert ok, erel
    # GPU parameter shift on a sample: each energy is within
    # ENERGY_REL * scale, and the rule's weights sum (in absolute value) to 1
    kind_of = {p: kind for kind, _, p in circ.gates}
    scale = energy_scale(e_ref, ham)
    rng = np.random.default_rng(24)
    for p in rng.choice(circ.n_params, size=6, replace=False):
        acc = 0.0
        wsum = 0.0
        for shift, w in oracle.SHIFT_RULES[kind_of[p]]:
            for sgn in (+1, -1):
                th = circ.theta.copy()
                th[p] += sgn * shift
                st.set_basis(circ.psi0_index)
                st.apply(circ, theta=th)
                ep, _ = st.expectation(ham)
                acc += sgn * w * ep
                wsum += abs(w)
        assert abs(acc - g_ref[p]) <= wsum * ENERGY_REL["c64"] * scale + GRAD_REL["c64"] * np.abs(g_ref).max(), \
            (p, acc, g_ref[p])
    st.close()


@pytest.mark.timeout(300)
@pytest.mark.parametrize("swaps", [((7, 25), (10, 27)), ((1, 24), (9, 26), (3, 12))],
                         ids=["rows", "tiles"])
def test_qr28_bit_exact(P, swaps):
    """A 28-qubit reorder against numpy.transpose of the state tensor: the
    rows path (every exchanged bit at 6 or above) and the tile path (an
    exchanged bit below 6, pairs inside and outside the tile)."""
    import torch
    n, g = 28, 5
    _print(f"qr28 {swaps}")
    v = W.random_state(n, 2828, np.complex64)
    buf = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
    st = P.State(n, g, "c64", buf=buf)
    st.set_amplitudes(v)
    pos = list(range(n))
    phys = list(range(n))
    for a, b in swaps:
        phys[a], phys[b] = phys[b], phys[a]
    new = [phys[p] for p in pos]
    st.qr_permute(new)
    torch.cuda.synchronize()
    got = buf.cpu().numpy()
    want = oracle.qr_permute(v, pos, new)
    assert np.array_equal(got, want)
    del got, want
    # and back: the logical state is unchanged, bit for bit
    np.testing.assert_array_equal(st.get_amplitudes(), v)
    st.close()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_chunk_partials_in_permuted_layout(P, dtype):
    """eq. local_evc / eq. aggregation: the per-chunk sums E_j that
    sv_expectation writes to chunk_dev equal the oracle's sums over the
    indices whose top g physical bits are j, in a permuted layout.  Z sites on
    global qubits give each chunk its sign (eq. par_exp); the X/Y sites are
    local, so the lazy plan needs no reorder and every E_j is one layout's."""
    import torch
    n, g = 16, 3
    rng = np.random.default_rng(1616)
    perm = [int(x) for x in rng.permutation(n)]
    local = [q for q in range(n) if perm[q] < n - g]
    glob = [q for q in range(n) if perm[q] >= n - g]
    xs, zs, cs = [], [], []
    for t in range(90):
        k = int(rng.integers(1, 5))
        xq = rng.choice(local, size=k, replace=False)
        x = sum(1 << int(q) for q in xq)
        z = int(rng.integers(0, 1 << n)) & ~x
        z |= sum(1 << int(q) for q in xq if rng.random() < 0.5)   # some Y
        if t % 3 == 0:
            z |= 1 << int(rng.choice(glob))
        if t % 10 == 0:
            x = 0                                              # diagonal strings
        xs.append(x); zs.append(z); cs.append(float(rng.normal()))
    ham = W.Hamiltonian(n, np.array(xs, dtype=np.uint64), np.array(zs, dtype=np.uint64),
                        np.array(cs))
    v = W.random_state(n, 1617, np.complex64 if dtype == "c64" else np.complex128)
    _print(f"chunk partials {dtype}")
    st = P.State(n, g, dtype)
    st.set_amplitudes(v)
    st.qr_permute(perm)
    chunks = torch.zeros(1 << g, dtype=torch.float64, device="cuda")
    e, stats = P.sv_expectation(st.h, P.paulis_array(ham), len(ham.coef), P.LAZY,
                                chunk_dev=chunks.data_ptr())
    torch.cuda.synchronize()
    assert stats.n_qr == 0 and st.layout() == perm
    e_ref, ch_ref = oracle.expectation(v.astype(np.complex128), ham, g=g, pos=perm,
                                       with_chunks=True)
    got = chunks.cpu().numpy()
    scale = energy_scale(e_ref, ham)
    assert np.max(np.abs(got - ch_ref)) <= ENERGY_REL[dtype] * scale, (got, ch_ref)
    assert abs(float(got.sum()) - e) <= 1e-12 * scale
    ok, rel = energy_ok(e, e_ref, None, ham, dtype)
    assert ok, rel
    st.close()


@pytest.mark.timeout(400)
def test_batch_instances_19_to_22_qubits(P):
    """The largest batch size class: instances of 19-22 qubits (6 fabric
    layers, 200 strings) in one persistent launch, each against the oracle's
    energy and adjoint gradient."""
    inst = []
    for i, n in enumerate((19, 20, 21, 22, 22, 10)):
        inst.append((W.fabric(n, 6, 7700 + i), W.jw_terms(n, 200, 7800 + i)))
    _print("batch 19-22 qubits")
    b = P.Batch(inst)
    e, grads, lat = b.run()
    b.close()
    for i, (c, h) in enumerate(inst):
        e_ref, g_ref = oracle.adjoint_grad(c, h)
        ok, rel = energy_ok(e[i], e_ref, None, h, "c64")
        assert ok, (i, c.n, rel)
        gok, grel = grad_ok(grads[i], g_ref, h, "c64")
        _print(f"  instance {i} ({c.n} qubits): energy rel {rel:.2e}, gradient rel {grel:.2e}")
        assert gok, (i, c.n, grel)
    assert np.all(lat > 0)
