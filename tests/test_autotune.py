"""Host logic of the launch-shape autotuner (paper_2006_10509_amd/autotune.py):
parsing and rewriting csrc/sizes.hpp and the candidate generators.  The
tuning itself needs hipcc and a GPU and is not run here."""
import os

from paper_2006_10509_amd import autotune as at
from paper_2006_10509_amd import build as hb

SIZES = open(os.path.join(hb.CSRC, "sizes.hpp")).read()


def test_every_compiled_length_has_both_configurations():
    rows, cols = at.read_configs(SIZES)
    assert set(rows) == set(cols) == set(hb.lengths())
    for n, (teams, t, ft, rad) in rows.items():
        assert teams * t <= 1024 and teams >= 1 and t >= 1 and ft >= 0
        assert _prod(rad) == n
    for n, (c, t, rad) in cols.items():
        assert c * t <= 1024 and _prod(rad) == n


def _prod(r):
    p = 1
    for v in r:
        p *= v
    return p


def test_rewrite_round_trips_and_restricts_lengths():
    rows, cols = at.read_configs(SIZES)
    new_row = (4, 128, 0, (5, 3, 8, 16))
    new_col = (4, 64, (8, 3, 3, 3, 5))
    text = at.with_configs(SIZES, {1920: new_row}, {1080: new_col}, [1080, 1920])
    r2, c2 = at.read_configs(text)
    assert r2[1920] == new_row and c2[1080] == new_col
    assert {n: v for n, v in r2.items() if n != 1920} == {n: v for n, v in rows.items() if n != 1920}
    tmp_lengths = [int(x) for x in text[text.index("#define HG_FOR_EACH_LENGTH"):].split("\n")[0]
                   .replace("#define HG_FOR_EACH_LENGTH(X)", "").replace("X(", "").replace(")", "").split()]
    assert tmp_lengths == [1080, 1920]
    assert at.with_configs(SIZES, {}, {}) == SIZES


def test_candidates_respect_the_kernel_constraints():
    rows, cols = at.read_configs(SIZES)
    for n in (512, 1024, 1080, 1920, 2048):
        rads = at.radix_orders(n, rows[n][3], 12)
        assert rads[0] == rows[n][3]
        for r in rads:
            assert _prod(r) == n and len(r) >= 2 and all(v in at.RADICES for v in r)
        for teams, t, ft, _ in at.row_shapes(n, rows[n], 12):
            assert (teams * t) % 64 == 0 and teams * t <= 1024
            assert ft == 0 or (t > 64 and t % ft == 0)
        for c, t, _ in at.col_shapes(n, cols[n], 12):
            assert (c * t) % 64 == 0 and c * t <= 1024
