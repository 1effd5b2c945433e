"""Host logic of the batch strip autotuner (no device needed)."""
import pytest

from paper_1905_13038_amd import tune


def test_window_classes_cover_every_window():
    assert tune.window_class(1) == tune.WINDOW_CLASSES[0]
    for lo, hi in zip((0,) + tune.WINDOW_CLASSES[:-1], tune.WINDOW_CLASSES):
        assert tune.window_class(lo + 1) == hi
        assert tune.window_class(hi) == hi
    assert tune.window_class(10 ** 6) == tune.WINDOW_CLASSES[-1]


@pytest.mark.parametrize("h,expect", [(1, 32), (11, 32), (16, 32), (17, 34), (51, 102), (64, 128),
                                      (65, 128), (257, 128)])
def test_default_strip_is_twice_the_window_within_bounds(h, expect):
    # the rule the library applies when no strip is given (bz_batched_plan)
    assert tune.default_strip(h) == expect


def test_strips_for_table_and_defaults():
    params = [{"h": 11}, {"h": 31}, {"h": 75}, {"h": 201}]
    assert tune.strips_for(params) == [tune.default_strip(p["h"]) for p in params]
    table = {15: 24, "63": 48}
    got = tune.strips_for(params, table)
    assert got == [24, tune.default_strip(31), tune.default_strip(75), tune.default_strip(201)]
    table2 = {c: 40 for c in tune.WINDOW_CLASSES}
    assert tune.strips_for(params, table2) == [40, 40, 40, 40]


DEV = "AMD Instinct MI355X"


@pytest.mark.parametrize("text", ["", "{", "not json", "[1, 2, 3]", '{"%s": 7}' % DEV,
                                  '{"%s": {"batch": "x"}}' % DEV, '{"%s": {"batch": {"15": "a"}}}' % DEV,
                                  '{"%s": {"batch": {"15": 0}}}' % DEV,
                                  '{"%s": {"plain": [[15, 1024, 8]]}}' % DEV,
                                  '{"%s": {"plain": [[15, 1024, 8, 100]]}}' % DEV,
                                  '{"%s": {"plain": "rows"}}' % DEV])
@pytest.mark.parametrize("kind", ["batch", "plain"])
def test_corrupt_or_foreign_cache_reads_as_missing(tmp_path, text, kind):
    # a cache the tuner cannot use is ignored (the calls keep the built-in
    # plans and the tuner measures again), never an error
    p = tmp_path / "tilings.json"
    p.write_text(text)
    assert tune.load_table(str(p), DEV, kind) is None
    assert tune.load_table(str(tmp_path / "missing.json"), DEV, kind) is None


def test_cache_round_trip_keeps_other_entries(tmp_path):
    p = str(tmp_path / "sub" / "tilings.json")
    tune.save_table(p, DEV, "batch", {15: 24, 63: 48})
    tune.save_table(p, DEV, "plain", [[15, 1024, 8, 256], [257, 8192, 0, 0]])
    tune.save_table(p, "other device", "batch", {31: 32})
    assert tune.load_table(p, DEV, "batch") == {15: 24, 63: 48}
    assert tune.load_table(p, DEV, "plain") == [[15, 1024, 8, 256], [257, 8192, 0, 0]]
    assert tune.load_table(p, "other device", "batch") == {31: 32}
    assert tune.load_table(p, "other device", "plain") is None
    # a corrupt file is replaced by the next save
    with open(p, "w") as f:
        f.write("{garbage")
    tune.save_table(p, DEV, "batch", {15: 16})
    assert tune.load_table(p, DEV, "batch") == {15: 16}


class _FakePlan:
    """Stands in for a BatchPlan: records the strips it is re-planned with."""

    def __init__(self):
        self.strips = None
        self.history = []

    def replan(self, strips):
        self.strips = list(strips)
        self.history.append(list(strips))

    def run(self):
        pass


def test_autotune_plan_takes_each_class_best_strip(monkeypatch):
    # a launch time that is lowest, per window class, at one candidate strip:
    # the greedy search keeps that strip for every class present and leaves
    # the plan re-planned with the result
    params = [{"h": 11}, {"h": 13}, {"h": 51}, {"h": 201}]
    best = {15: 24, 63: 96, 257: 128}
    plan = _FakePlan()

    def fake_time(fn, reps):
        fn()
        cost = 1000.0
        for p, s in zip(params, plan.strips):
            cost += abs(s - best[tune.window_class(p["h"])])
        return cost

    monkeypatch.setattr(tune, "_time", fake_time)
    table = tune.autotune_plan(plan, params)
    # class 257's best is its built-in strip (2 h capped at 128), so it stays out
    assert table == {15: 24, 63: 96}
    assert plan.strips == tune.strips_for(params, table) == [24, 24, 96, 128]


def test_autotune_plan_keeps_builtin_strips_without_gain(monkeypatch):
    # gains under min_gain are not taken: the table stays empty and the plan
    # keeps the built-in strips
    params = [{"h": 31}, {"h": 75}]
    plan = _FakePlan()
    calls = []

    def flat_time(fn, reps):
        fn()
        calls.append(list(plan.strips))
        return 1000.0 - (0.001 if plan.strips[0] == 48 else 0.0)

    monkeypatch.setattr(tune, "_time", flat_time)
    table = tune.autotune_plan(plan, params, min_gain=0.005)
    assert table == {}
    assert plan.strips == [tune.default_strip(31), tune.default_strip(75)]
    # one baseline, then one trial per candidate and class
    assert len(calls) == 1 + len(tune.CANDIDATES) * 2
