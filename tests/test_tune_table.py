"""Host logic of the tile-width autotuner (CPU only): the merge of per-size choices
into table rows, and the validity of the committed table."""
import os
import re

from paper_1204_0069_amd import tune

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "..", "paper_1204_0069_amd", "csrc", "ccg_tune_table.h")


class FakeCtx:
    """Timings: width 1 wins below n = 1024, width 4 above 4096 where it fits, else 2."""

    def __init__(self):
        self.calls = []

    def tune_ad(self, prec, P, n, cw, reps):
        self.calls.append((prec, P, n, cw))
        if n < 1024:
            return {1: 1.0, 2: 2.0, 4: 3.0}[cw]
        if n > 4096:
            return {1: 3.0, 2: 2.0, 4: 1.0}[cw]
        return {1: 2.0, 2: 1.0, 4: 3.0}[cw]


def _rows_for(rows, c, P):
    return [(n_max, w) for cc, PP, n_max, w in rows if cc == c and PP == P]


def test_merge_and_limits():
    ctx = FakeCtx()
    rows = tune.tune(ctx, reps=1, log=lambda s: None)
    # FP32, P = 8: 1 up to 512, 2 for 1024..4096, 4 beyond
    assert _rows_for(rows, "PREC_F32", 8) == [(768, 1), (6144, 2), (1 << 30, 4)]
    # FP64, P = 8 may not use 4 columns per wave: 2 from 1024 on
    assert _rows_for(rows, "PREC_F64", 8) == [(768, 1), (1 << 30, 2)]
    # P = 16 never times width 4; no size below P is timed
    assert not any(P == 16 and w == 4 for _, P, _, w in ctx.calls)
    assert all(P <= n for _, P, n, _ in ctx.calls)


def test_written_table_round_trips(tmp_path):
    rows = [("PREC_F64", 8, 1536, 1), ("PREC_F64", 8, 1 << 30, 2)]
    out = tmp_path / "t.h"
    tune.write_table(rows, "test device", str(out))
    text = out.read_text()
    got = re.findall(r"\{(PREC_\w+), (\d+), (\d+), (\d)\}", text)
    assert [(c, int(P), int(n), int(w)) for c, P, n, w in got] == rows


def test_committed_table_is_valid():
    text = open(TABLE).read()
    rows = [(c, int(P), int(n), int(w)) for c, P, n, w in
            re.findall(r"\{(PREC_\w+), (\d+), (\d+), (\d)\}", text)]
    assert rows, "empty tuning table"
    last = {}
    for c, P, n_max, w in rows:
        assert c in ("PREC_F64", "PREC_F32", "PREC_BF16X2")
        assert P in (1, 2, 4, 8, 16) and w in (1, 2, 4)
        assert n_max > last.get((c, P), 0), "rows of one class must grow in n"
        last[(c, P)] = n_max
