"""The autotuner's cache logic without a GPU."""
import os

from paper_1609_00999_amd import tune


class FakeLib:
    def __init__(self):
        self.calls = []

    def mont_elem_tune_set(self, op, block, vpt, nt):
        self.calls.append(("elem", op, block, vpt, nt))
        return 0

    def ntt_tune_set(self, threads, radix, gm):
        self.calls.append(("ntt", threads, radix, gm))
        return 0

    def ntt_tune_set_length(self, n, threads, radix, gm):
        self.calls.append(("ntt_len", n, threads, radix, gm))
        return 0


def test_best_entry_and_choose(tmp_path):
    res = [((256, 1, 1), 3.0), ((512, 2, 0), 1.0), ((256, 4, 1), 2.0)]
    e = tune.best_entry(res)
    assert e["config"] == [512, 2, 0] and e["seconds"] == 1.0 and len(e["measured"]) == 3
    cache = {}
    tune.merge(cache, "gfx950", "elem_mul", "24", {"config": [256, 1, 1]})
    tune.merge(cache, "gfx950", "elem_mul", "28", {"config": [512, 4, 0]})
    assert tune.choose(cache, "gfx950", "elem_mul") == [512, 4, 0]     # the largest bucket
    assert tune.choose(cache, "gfx942", "elem_mul") is None
    path = os.path.join(str(tmp_path), "c.json")
    tune.save(cache, path)
    assert tune.load(path) == cache
    assert tune.load(os.path.join(str(tmp_path), "missing.json")) == {}


def test_best_entry_tie_prefers_the_cheaper_config():
    # the transform tuner's rule: within 1 % of the fastest, the smaller grid multiplier
    res = [((512, 4, 1), 9.413), ((512, 4, 2), 9.394), ((512, 3, 1), 10.03), ((256, 4, 1), 9.40)]
    e = tune.best_entry(res, tie=0.01, cost=lambda c: c[2])
    assert e["config"] == [256, 4, 1] and e["seconds"] == 9.40     # cheapest, then fastest
    e = tune.best_entry(res[:3], tie=0.01, cost=lambda c: c[2])
    assert e["config"] == [512, 4, 1]
    e = tune.best_entry(res[:3], tie=0.001, cost=lambda c: c[2])
    assert e["config"] == [512, 4, 2]                              # outside the tie band
    assert tune.best_entry(res)["config"] == [512, 4, 2]           # no tie rule: fastest


def test_apply_uses_the_c_abi():
    cache = {"gfx950": {"elem_mul": {"28": {"config": [512, 2, 1]}}, "ntt": {"batch2048": {"config": [1024, 3, 2]}}}}
    lib = FakeLib()
    applied = tune.apply(cache, "gfx950", lib)
    assert applied == {"elem_mul": [512, 2, 1], "ntt": [1024, 3, 2]}
    assert ("elem", 2, 512, 2, 1) in lib.calls and ("ntt", 1024, 3, 2) in lib.calls
    assert tune.apply(cache, "gfx90a", FakeLib()) == {}


def test_shape_sets_match_the_abi():
    import ctypes
    from paper_1609_00999_amd import mont
    L = mont.lib()
    for b, v, nt in tune.ELEM_SHAPES:
        assert L.mont_elem_tune_set(2, b, v, nt) == 0
    for t, r in tune.NTT_SHAPES:
        for g in tune.GRID_MULTS:
            assert L.ntt_tune_set(t, r, g) == 0
    assert L.ntt_tune_set(128, 3, 1) == -1 and L.ntt_tune_set(512, 5, 1) == -1 and L.ntt_tune_set(512, 4, 3) == -1
    t, r, g = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    assert L.ntt_tune_get(ctypes.byref(t), ctypes.byref(r), ctypes.byref(g)) == 0
    L.ntt_tune_set(512, 4, 1)
    L.mont_elem_tune_set(2, 256, 1, 1)


def test_cache_problems_are_reported(tmp_path):
    """A corrupt cache, a cache that is not an object and an entry the library
    rejects each raise a RuntimeWarning (the built-in shapes stay in force)."""
    import warnings
    import pytest
    bad = os.path.join(str(tmp_path), "bad.json")
    with open(bad, "w") as f:
        f.write("{not json")
    with pytest.warns(RuntimeWarning, match="not loaded"):
        assert tune.load(bad) == {}
    lst = os.path.join(str(tmp_path), "list.json")
    with open(lst, "w") as f:
        f.write("[1, 2]")
    with pytest.warns(RuntimeWarning, match="not a JSON object"):
        assert tune.load(lst) == {}

    class Rejecting(FakeLib):
        def ntt_tune_set(self, threads, radix, gm):
            return -1

    cache = {"gfx950": {"elem_mul": {"28": {"config": [512, 2, 1]}}, "ntt": {"b": {"config": [300, 3, 1]}}}}
    with pytest.warns(RuntimeWarning, match="ntt"):
        applied = tune.apply(cache, "gfx950", Rejecting())
    assert applied == {"elem_mul": [512, 2, 1]}
    broken = {"gfx950": {"elem_to": {"28": {"config": ["x"]}}}}
    with pytest.warns(RuntimeWarning, match="elem_to"):
        assert tune.apply(broken, "gfx950", FakeLib()) == {}
    with warnings.catch_warnings():
        warnings.simplefilter("error")
        assert tune.load(os.path.join(str(tmp_path), "missing.json")) == {}   # no cache yet: silent


def test_apply_sets_per_length_shapes():
    """Per-length buckets set every length of their range through the C ABI."""
    cache = {"gfx950": {"ntt_len": {"14-16": {"config": [256, 4, 1]}, "22-23": {"config": [1024, 3, 2]}}}}
    lib = FakeLib()
    applied = tune.apply(cache, "gfx950", lib)
    assert applied == {"ntt_len_14-16": [256, 4, 1], "ntt_len_22-23": [1024, 3, 2]}
    assert [c for c in lib.calls if c[0] == "ntt_len"] == [("ntt_len", n, 256, 4, 1) for n in (14, 15, 16)] + \
        [("ntt_len", n, 1024, 3, 2) for n in (22, 23)]
    import pytest
    with pytest.warns(RuntimeWarning, match="ntt_len"):
        assert tune.apply({"gfx950": {"ntt_len": {"x": {"config": [1]}}}}, "gfx950", FakeLib()) == {}
    assert [b for b in tune.LEN_BUCKETS] == sorted(tune.LEN_BUCKETS)
    covered = [n for lo, hi in tune.LEN_BUCKETS for n in range(lo, hi + 1)]
    assert covered == list(range(24))


def test_per_length_shapes_through_the_abi():
    """ntt_tune_set_length / get_length (host only): an entry overrides the
    default for its length only; threads 0 removes it; bad shapes are refused."""
    import ctypes
    from paper_1609_00999_amd import mont
    L = mont.lib()
    t, r, g = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    L.ntt_tune_set(512, 4, 1)
    assert L.ntt_tune_set_length(16, 256, 3, 2) == 0
    assert L.ntt_tune_get_length(16, ctypes.byref(t), ctypes.byref(r), ctypes.byref(g)) == 0
    assert (t.value, r.value, g.value) == (256, 3, 2)
    assert L.ntt_tune_get_length(17, ctypes.byref(t), ctypes.byref(r), ctypes.byref(g)) == 0
    assert (t.value, r.value, g.value) == (512, 4, 1)
    assert L.ntt_tune_set_length(16, 0, 0, 0) == 0
    assert L.ntt_tune_get_length(16, ctypes.byref(t), ctypes.byref(r), ctypes.byref(g)) == 0
    assert (t.value, r.value, g.value) == (512, 4, 1)
    assert L.ntt_tune_set_length(24, 512, 4, 1) == -1 and L.ntt_tune_set_length(5, 300, 4, 1) == -1
