"""Host logic of the GEMM autotuner (no GPU): launch-log decoding and shape
classes."""
import numpy as np

from paper_2607_00928_amd import tune_gemm as tg


def test_clog2():
    assert [tg.clog2(x) for x in (1, 2, 3, 4, 5, 16, 17, 1 << 20)] == [0, 1, 2, 2, 3, 4, 5, 20]


def test_decode_variant_codes():
    # regular launches: opA * 2 + opB + 10 * splits
    assert tg.decode(10) == (0, 0, False)
    assert tg.decode(11) == (0, 1, False)
    assert tg.decode(12 + 10 * 7) == (1, 0, False)
    assert tg.decode(13) == (1, 1, False)
    # skinny launches: opA * 2 + 10 * splits + 1000 (op(B) = N)
    assert tg.decode(1000 + 2 + 160) == (1, 0, True)
    assert tg.decode(1010) == (0, 0, True)
    # small-output tiles (always A^H B): 2000 + 10 mb + nb, and 3000
    for v in (2011, 2012, 2021, 2022, 3000):
        assert tg.decode(v) == (1, 0, False)


def test_small_tile_candidates():
    assert tg.small_tiles(1, 0, 32, 128) == [1]
    assert tg.small_tiles(1, 0, 16, 20) == [1, 2]
    assert tg.small_tiles(1, 0, 33, 64) == []
    assert tg.small_tiles(0, 0, 16, 64) == []
    assert tg.small_tiles(1, 0, 16, 8) == []
    assert tg.small_tiles(1, 0, 16, 129) == []
    assert tg.TILE_CODES == {1: -5, 2: -6}


def test_classes_bucket_and_rank():
    # cls ms flops nd m n k var
    rows = np.array([
        [1, 5.0, 1e9, 12, 5753, 5753, 5753, 10],
        [1, 7.0, 1e9, 12, 5000, 6000, 5500, 10],    # same class as above
        [2, 1.0, 1e9, 32, 16, 16, 1015804, 642],    # FP64, A^H B, 64 splits
        [0, 9.0, 1e9, 1, 1, 1, 1, 0],               # apply: ignored
        [3, 9.0, 0.0, 64, 512, 0, 0, 1],            # QR panel: ignored
    ])
    cl = tg.classes(rows, top=10)
    assert len(cl) == 2
    (k0, c0), (k1, c1) = cl
    assert k0 == (1, 0, 0, 13, 13, 13, 4) and c0["ms"] == 12.0 and c0["count"] == 2
    assert (c0["m"], c0["n"], c0["k"], c0["nd"]) == (5753, 6000, 5753, 12)
    assert k1 == (0, 1, 0, 4, 4, 20, 5)


def test_classes_accept_step_column():
    # launch logs carry the algorithm step as a ninth column
    rows = np.array([[1, 5.0, 1e9, 12, 5753, 5753, 5753, 10, 9],
                     [1, 2.0, 1e9, 12, 5000, 6000, 5500, 10, 3]])
    cl = tg.classes(rows, top=10)
    assert len(cl) == 1 and cl[0][1]["ms"] == 7.0 and cl[0][1]["count"] == 2


def test_classes_skinny_products():
    # skinny products log as classes 4 (FP32) and 5 (FP64)
    rows = np.array([[4, 3.0, 1e9, 1024, 1042, 1, 256, 1010, 16],
                     [5, 1.0, 1e9, 4, 300, 2, 5000, 1032, 16]])
    cl = dict(tg.classes(rows, top=10))
    assert (1, 0, 0, 11, 0, 8, 10) in cl and (0, 1, 0, 9, 1, 13, 2) in cl


def test_merge_entries():
    a, b, c, d, e = [(1, 0, 0, i, 0, 0, 0) for i in range(5)]
    old = {a: (1, 0), b: (4, 0), c: (0, 2), d: (8, 0)}
    measured = {b: ((4, 0), 1.02),      # same winner, small gain: kept
                c: ((2, 0), 1.03),      # another winner below the threshold: dropped
                d: ((16, 0), 1.30),     # a clear new winner: replaced
                e: ((0, 1), 1.10)}      # new class: added
    out = tg.merge_entries(old, measured)
    assert out == {a: (1, 0), b: (4, 0), d: (16, 0), e: (0, 1)}
    # the heuristic now wins: the old entry goes
    assert tg.merge_entries({a: (1, 0)}, {a: ((1, 0), 0.97)}) == {}


def test_read_table(tmp_path):
    p = tmp_path / "t.inc"
    p.write_text("// header\n// {prec, ...},\n{1, 0, 0, 12, 11, 8, 5, 1},\n"
                 "{1, 1, 0, 5, 5, 10, 5, 0, 2},\n")
    assert tg.read_table(str(p)) == {(1, 0, 0, 12, 11, 8, 5): (1, 0),
                                     (1, 1, 0, 5, 5, 10, 5): (0, 2)}
    assert tg.read_table(str(tmp_path / "missing.inc")) == {}
