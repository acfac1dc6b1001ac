"""sv_apply_circuit_static: the entry point for callers that cannot allocate
device memory.  Its results must equal sv_apply_circuit's (the same plan and
kernels, tables in the library's static scratch instead of handle buffers),
on two calls in a row, the second with a smaller input; tables larger than the
scratch are refused before anything runs."""
import numpy as np
import pytest

import oracle
import workloads as W
from tolerances import amp_ok

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_2410_04252_amd as P
    torch.cuda.set_device(0)
    return P


def _run(P, n, g, dtype, circ, static, v):
    """Apply circ to v on a handle that borrows its buffer; returns the
    logical amplitudes, the layout and the stats."""
    import torch
    tdt = torch.complex64 if dtype == "c64" else torch.complex128
    buf = torch.empty(1 << n, dtype=tdt, device="cuda")
    st = P.State(n, g, dtype, buf=buf)
    st.set_amplitudes(v)
    fn = P.sv_apply_circuit_static if static else P.sv_apply_circuit
    stats = fn(st.h, P.gates_array(circ.gates), len(circ.gates), circ.theta, len(circ.theta), P.LAZY)
    torch.cuda.synchronize()
    pos = st.layout()
    out = st.get_amplitudes()
    st.close()
    return out, pos, stats


def test_static_equals_allocating_entry_point_twice(P):
    cases = [(17, 3, "c64", W.fabric(17, 10, 7101), 7102),      # first call
             (12, 2, "c128", W.hea(12, 4, 7103), 7104)]         # second, smaller
    for n, g, dtype, circ, seed in cases:
        print(f"static entry point n={n} {dtype}", flush=True)
        v = W.random_state(n, seed, np.complex64 if dtype == "c64" else np.complex128)
        got, pos_s, st_s = _run(P, n, g, dtype, circ, True, v)
        want, pos_a, st_a = _run(P, n, g, dtype, circ, False, v)
        assert pos_s == pos_a
        assert (st_s.n_qr, st_s.n_gate_passes, st_s.tile_k) == (st_a.n_qr, st_a.n_gate_passes, st_a.tile_k)
        assert np.array_equal(got, want)
        ok, mx, rl2 = amp_ok(got, oracle.apply_circuit(v, circ.gates, circ.theta), dtype)
        assert ok, (mx, rl2)


def test_static_refuses_tables_beyond_the_scratch(P):
    """13,000 gates need about 5.0 MB of op descriptors, more than the 4 MiB
    scratch: ESHAPE, and the state is left as it was."""
    n, g = 10, 1
    circ = W.random_circuit(n, 13000, 7105)
    v = W.random_state(n, 7106, np.complex64)
    st = P.State(n, g, "c64")
    st.set_amplitudes(v)
    with pytest.raises(P.SvqError) as ei:
        P.sv_apply_circuit_static(st.h, P.gates_array(circ.gates), len(circ.gates), circ.theta,
                                  len(circ.theta), P.LAZY)
    assert P.STATUS[ei.value.status] == "ESHAPE"
    assert st.layout() == list(range(n))
    assert np.array_equal(st.get_amplitudes(), v)
    st.close()
