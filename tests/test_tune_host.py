"""Host side of the measured tuner: the tuned table's text file round trip
and its error paths (no GPU is touched)."""
import os

import pytest


@pytest.fixture(scope="module")
def P():
    import paper_2410_04252_amd as P
    return P


def test_tune_table_round_trip(P, tmp_path):
    src = tmp_path / "in.txt"
    src.write_text("0 30 5 0 12 4 3.500000\n1 30 5 0 14 4 9.250000\n2 0 0 0 16 4 1.000000\n"
                   "3 0 0 0 18 0 1.000000\n"     # batch size classes: no low bits
                   "0 31 5 0 12 0 1.0\n"         # gate pass without low bits: skipped
                   "7 1 1 1 1 1 1.0\n")          # unknown kind: skipped
    P.sv_tune_load(str(src))
    out = tmp_path / "out.txt"
    P.sv_tune_save(str(out))
    rows = {tuple(int(v) for v in ln.split()[:6]) for ln in out.read_text().splitlines()}
    assert {(0, 30, 5, 0, 12, 4), (1, 30, 5, 0, 14, 4), (2, 0, 0, 0, 16, 4), (3, 0, 0, 0, 18, 0)} <= rows
    assert not any(r[0] == 7 for r in rows)
    assert not any(r[:2] == (0, 31) for r in rows)
    # the shipped table again (this process's later users read it)
    P.sv_tune_load(P.TUNE_FILE)


def test_tune_file_errors(P, tmp_path):
    with pytest.raises(P.SvqError) as e:
        P.sv_tune_load(str(tmp_path / "missing.txt"))
    assert e.value.status == -1
    with pytest.raises(P.SvqError):
        P.sv_tune_save(os.path.join(str(tmp_path), "no_dir", "x.txt"))
