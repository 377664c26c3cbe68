"""Host logic of the tile-shape autotuner (CPU only): the candidate shapes, the merge
of per-size choices into table rows, and the validity of the committed table."""
import os
import re

from paper_1204_0069_amd import tune

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "..", "paper_1204_0069_amd", "csrc", "ccg_tune_table.h")
ROW = r"\{(PREC_\w+), (\d+), (\d+), (\d), (\d+)\}"


class FakeCtx:
    """Timings: width 1 wins below n = 1024, width 4 above 4096 where it fits, else 2;
    16 waves per workgroup win from n = 8192 on, 4 below.  The batched kernel times
    the same, except that 16 waves at width 4 are slow there (as a spilling shape)."""

    def __init__(self):
        self.calls = []

    def tune_ad(self, prec, P, n, cw, reps, nw=4, batched=False):
        self.calls.append((prec, P, n, cw, nw))
        if batched and cw == 4 and nw == 16:
            return 100.0
        if n < 1024:
            t = {1: 1.0, 2: 2.0, 4: 3.0}[cw]
        elif n > 4096:
            t = {1: 3.0, 2: 2.0, 4: 1.0}[cw]
        else:
            t = {1: 2.0, 2: 1.0, 4: 3.0}[cw]
        return t * ({4: 1.0, 8: 1.1, 16: 1.2}[nw] if n < 8192 else {4: 1.0, 8: 0.9, 16: 0.8}[nw])


def _rows_for(rows, c, P):
    return [(n_max, w, nw) for cc, PP, n_max, w, nw in rows if cc == c and PP == P]


def test_candidate_shapes_follow_the_register_rules():
    assert (4, 16) in tune.shapes("fp32", 8)
    # FP64, P = 8: 4 columns per wave only as the matrix-core tile
    assert [sh for sh in tune.shapes("fp64", 8) if sh[0] == 4] == [(4, 4), (4, 8)]
    # P = 16: the vector tile at most 2 columns and 4 waves, then the matrix cores
    # (FP64 operands for FP64, FP32 operands for FP32 and BF16x2)
    for prec in ("fp64", "fp32", "bf16x2"):
        assert tune.shapes(prec, 16) == [(1, 4), (2, 4)] + list(tune.MFMA_SHAPES[16])
    assert tune.DEFAULT in tune.shapes("bf16x2", 1)
    # P = 32: FP64 on the matrix cores only
    assert tune.shapes("fp64", 32) == list(tune.MFMA_SHAPES[32]) and tune.shapes("fp32", 32) == []
    # wider vector workgroups only where the engine was measured not to lose with them
    for prec in ("fp64", "fp32", "bf16x2"):
        for P in (1, 2, 4, 8, 16):
            mfma = tune.MFMA_SHAPES.get(P, ()) if prec == "fp64" or P == 16 else ()
            vec = [sh for sh in tune.shapes(prec, P) if sh not in mfma]
            assert any(nw > 4 for _, nw in vec) == (P in tune.WIDE_P)


def test_merge_and_limits():
    ctx = FakeCtx()
    rows = tune.tune(ctx, reps=1, log=lambda s: None)
    # FP32, P = 8: width 1 up to 512, 2 for 1024..4096, then from 8192 on width 4 with
    # 8 waves: 16 waves are faster in the single-system kernel but slow batched
    assert _rows_for(rows, "PREC_F32", 8) == [(768, 1, 4), (6144, 2, 4), (1 << 30, 4, 8)]
    # P = 4 keeps 4 waves per workgroup
    assert all(nw == 4 for _, _, nw in _rows_for(rows, "PREC_F32", 4))
    # FP64, P = 8: 4 columns per wave only as the matrix-core tile, which wins from
    # 8192 on at 8 waves
    assert _rows_for(rows, "PREC_F64", 8) == [(768, 1, 4), (6144, 2, 4), (1 << 30, 4, 8)]
    # at P = 16 the shapes timed are the vector tile's (at most 2 columns, 4 waves)
    # and the matrix cores'; no size below P is timed
    assert all((w <= 2 and nw == 4) or (w, nw) in tune.MFMA_SHAPES[16]
               for prec, P, _, w, nw in ctx.calls if P == 16)
    assert all(P <= n for _, P, n, _, _ in ctx.calls)


def test_written_table_round_trips(tmp_path):
    rows = [("PREC_F64", 8, 1536, 1, 4), ("PREC_F64", 8, 1 << 30, 2, 16)]
    out = tmp_path / "t.h"
    tune.write_table(rows, "test device", str(out))
    got = re.findall(ROW, out.read_text())
    assert [(c, int(P), int(n), int(w), int(nw)) for c, P, n, w, nw in got] == rows


def test_logs_read_the_score(tmp_path):
    log = tmp_path / "new.txt"
    log.write_text("fp64    P= 8 n=  8192 c2w4:    98.54us(98.50/98.54)  c2w8:    93.86us(93.70/93.86)"
                   "  -> 2,8\n")
    assert tune.rows_from_log(str(log)) == [("PREC_F64", 8, 1 << 30, 2, 8)]


def test_old_logs_read_as_four_waves(tmp_path):
    log = tmp_path / "old.txt"
    log.write_text("fp64    P= 8 n=  8192 cw1:   142.41us  cw2:    96.12us  -> 2\n")
    assert tune.rows_from_log(str(log)) == [("PREC_F64", 8, 1 << 30, 2, 4)]


def test_committed_table_is_valid():
    text = open(TABLE).read()
    rows = [(c, int(P), int(n), int(w), int(nw)) for c, P, n, w, nw in re.findall(ROW, text)]
    assert rows, "empty tuning table"
    last = {}
    for c, P, n_max, w, nw in rows:
        assert c in ("PREC_F64", "PREC_F32", "PREC_BF16X2")
        assert P in (1, 2, 4, 8, 16, 32) and w in (1, 2, 4) and nw in (4, 8, 16)
        assert P < 32 or (c == "PREC_F64" and w * nw >= 16), "P = 32: FP64 matrix-core shapes only"
        assert n_max > last.get((c, P), 0), "rows of one class must grow in n"
        last[(c, P)] = n_max
