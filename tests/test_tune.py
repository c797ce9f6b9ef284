"""Host logic of the schedule autotuner: which (operation, N) classes a set
of codes has, the valid splits, and the versioned table (no GPU)."""
import pytest

from paper_1404_3458_amd import rs, tune


def test_candidates():
    assert tune.candidates(9) == [(4, 5), (5, 4)]
    assert tune.candidates(12) == [(4, 8), (5, 7), (6, 6), (7, 5), (8, 4), (4, 4, 4)]
    assert (8, 8) in tune.candidates(16) and (4, 4, 4, 4) in tune.candidates(16)
    for N in range(9, 17):
        c = tune.candidates(N)
        assert tune.default_split(N) in c                  # the default is always a candidate
        assert all(sum(p) == N and all(4 <= v <= 8 for v in p) and 2 <= len(p) <= 4 for p in c)
        assert len(set(c)) == len(c)


def test_classes():
    got = tune.classes([(16, 8), (64, 48), (256, 224), (1024, 512), (4096, 2048), (1024, 512)])
    assert got == {("dec", 9): [(256, 224)], ("enc", 9): [(1024, 512)], ("dec", 10): [(1024, 512)],
                   ("enc", 11): [(4096, 2048)], ("dec", 12): [(4096, 2048)]}
    assert tune.mother(256, 224) == (512, 256) and tune.mother(300, 200) == (512, 256)


class FakeCodec:
    def __init__(self):
        self.calls = []

    def set_schedule(self, op, N, T1):
        self.calls.append((op, N, T1))

    def set_schedule_tile(self, op, N, cols):
        self.calls.append(("tile", op, N, cols))


def test_table_roundtrip(tmp_path):
    tab = {"version": tune.VERSION, "entries": [{"op": "dec", "N": 12, "parts": [4, 4, 4], "tile": 0},
                                                 {"op": "enc", "N": 11, "parts": [5, 6], "tile": 128}]}
    p = str(tmp_path / "t.json")
    tune.save(tab, p)
    c = FakeCodec()
    assert tune.load(p, c) == tab
    assert c.calls == [(rs.RS_OP_DECODE, 12, (4, 4, 4)), ("tile", rs.RS_OP_DECODE, 12, 0),
                       (rs.RS_OP_ENCODE, 11, (5, 6)), ("tile", rs.RS_OP_ENCODE, 11, 128)]
    assert tune.summary(tab) == {"dec:12": "4/4/4", "enc:11": "5/6 t128"}
    with pytest.raises(ValueError):
        tune.apply(FakeCodec(), {"version": tune.VERSION + 1, "entries": []})
    # a table of the previous version (no tiles) keeps the default tile
    c = FakeCodec()
    tune.apply(c, {"version": 2, "entries": [{"op": "dec", "N": 9, "parts": [5, 4]}]})
    assert c.calls == [(rs.RS_OP_DECODE, 9, (5, 4)), ("tile", rs.RS_OP_DECODE, 9, 0)]
