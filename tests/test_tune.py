"""Host logic of the schedule autotuner: which (operation, N) classes a set
of codes has, the valid splits, and the versioned table (no GPU)."""
import pytest

from paper_1404_3458_amd import rs, tune


def test_candidates():
    assert tune.candidates(9) == [4, 5]
    assert tune.candidates(12) == [4, 5, 6, 7, 8]
    assert tune.candidates(16) == [8]
    for N in range(9, 17):
        assert (N + 1) // 2 in tune.candidates(N)          # the default is always valid


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


def test_table_roundtrip(tmp_path):
    tab = {"version": tune.VERSION, "entries": [{"op": "dec", "N": 12, "T1": 7}, {"op": "enc", "N": 11, "T1": 5}]}
    p = str(tmp_path / "t.json")
    tune.save(tab, p)
    c = FakeCodec()
    assert tune.load(p, c) == tab
    assert c.calls == [(rs.RS_OP_DECODE, 12, 7), (rs.RS_OP_ENCODE, 11, 5)]
    assert tune.summary(tab) == {"dec:12": 7, "enc:11": 5}
    with pytest.raises(ValueError):
        tune.apply(FakeCodec(), {"version": tune.VERSION + 1, "entries": []})
