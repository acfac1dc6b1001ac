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
                   "7 1 1 1 1 1 1.0\n")          # unknown kind: skipped
    P.sv_tune_load(str(src))
    out = tmp_path / "out.txt"
    P.sv_tune_save(str(out))
    rows = {tuple(int(v) for v in ln.split()[:6]) for ln in out.read_text().splitlines()}
    assert {(0, 30, 5, 0, 12, 4), (1, 30, 5, 0, 14, 4), (2, 0, 0, 0, 16, 4)} <= rows
    assert not any(r[0] == 7 for r in rows)


def test_tune_file_errors(P, tmp_path):
    with pytest.raises(P.SvqError) as e:
        P.sv_tune_load(str(tmp_path / "missing.txt"))
    assert e.value.status == -1
    with pytest.raises(P.SvqError):
        P.sv_tune_save(os.path.join(str(tmp_path), "no_dir", "x.txt"))
