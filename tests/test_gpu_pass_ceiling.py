"""sv_pass_ceiling runs the gate-pass kernel with no gates: it must rewrite
every amplitude in place unchanged (bit for bit), for every phase count and
tile shape the measurement uses, and reject shapes outside its range."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_2410_04252_amd as P
    torch.cuda.set_device(0)
    return P


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("k,nphase", [(10, 1), (11, 2), (12, 5), (12, 8), (13, 3)])
def test_empty_pass_leaves_state_unchanged(P, dtype, k, nphase):
    n, g = 18, 3
    rng = np.random.default_rng(100 * k + nphase)
    c = 4
    high = sorted(int(x) for x in rng.choice(np.arange(c, n - g), size=k - c, replace=False))
    tile_bits = list(range(c)) + high
    print(f"empty pass {dtype} k={k} phases={nphase} tile bits {tile_bits}", flush=True)
    v = W.random_state(n, 4000 + k, np.complex64 if dtype == "c64" else np.complex128)
    st = P.State(n, g, dtype)
    st.set_amplitudes(v)
    ms = P.sv_pass_ceiling(st.h, tile_bits, nphase, reps=2)
    assert ms > 0
    np.testing.assert_array_equal(st.get_amplitudes(), v)
    st.close()


def test_empty_pass_rejects_bad_shapes(P):
    st = P.State(14, 2, "c64")
    for tb, nph in (([0, 1, 2, 3, 4, 5, 6, 7, 8], 2),          # k = 9
                    ([0, 1, 2, 3, 4, 5, 6, 7, 8, 12], 2),      # position 12 is global
                    ([0, 1, 2, 3, 4, 5, 6, 7, 9, 8], 2),       # not ascending
                    ([0, 1, 2, 3, 4, 5, 6, 7, 8, 9], 0)):      # no phase
        with pytest.raises(P.SvqError) as ei:
            P.sv_pass_ceiling(st.h, tb, nph)
        assert P.STATUS[ei.value.status] == "EINVAL"
    st.close()


@pytest.mark.parametrize("n16", [1, 2047, 2048, 3 * 2048 + 17, 1 << 20])
def test_device_copy_exact(P, n16):
    """The reference copy moves exactly bytes = 16 * n16 (ragged tails too)
    and leaves the bytes after it alone."""
    import torch
    src = torch.randint(0, 1 << 30, (n16 * 4 + 4,), dtype=torch.int32, device="cuda")
    dst = torch.zeros_like(src)
    P.sv_device_copy(src.data_ptr(), dst.data_ptr(), 16 * n16, torch.cuda.current_stream())
    torch.cuda.synchronize()
    assert torch.equal(dst[:n16 * 4], src[:n16 * 4])
    assert int(dst[n16 * 4:].abs().sum()) == 0
