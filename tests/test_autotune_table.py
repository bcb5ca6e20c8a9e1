"""The tuned-tile table round trip (host only): the autotuner's writer and
reader agree, new entries replace old ones of the same key, and the table the
library compiles in parses."""
import os

from paper_2210_12212_amd import autotune


def test_table_round_trip(tmp_path):
    p = os.path.join(tmp_path, "t.inc")
    rows = [(131072, 2048, 0, 0, 3, 3, 16), (131072, 2048, 0, 0, 1, 1, 0), (2048, 256, 1, 0, 2, 2, 4)]
    autotune.write_table(rows, p)
    assert sorted(autotune.read_table(p)) == sorted(rows)
    merged = autotune.merge(rows, [(131072, 2048, 0, 0, 3, 4, 8)])
    assert (131072, 2048, 0, 0, 3, 4, 8) in merged and (131072, 2048, 0, 0, 3, 3, 16) not in merged
    autotune.write_table([], p)
    assert autotune.read_table(p) == []
    txt = open(p).read()
    assert "kNumTunedTiles = 0" in txt


def test_committed_table_parses():
    rows = autotune.read_table()
    for r in rows:
        n, d, dt, prec, nb, q, sp = r
        assert n > 0 and d > 0 and dt in (0, 1) and prec in (0, 1) and nb >= 1
        assert 1 <= q <= 7 and 0 <= sp <= 256


def test_width_ranges():
    assert autotune.parse_range("1-4,8") == [1, 2, 3, 4, 8]
