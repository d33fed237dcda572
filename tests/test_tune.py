"""Host logic of the schedule tuner (no GPU): the variants it times are the
compiled-in combinations, it keeps the fastest per kernel from the median
of its rounds, holds the other kernels at their current choice, skips a
kernel with no launch, and caches the pick per device, precision and
particle-count bucket."""
import json

from paper_2107_01276_amd import DEFAULT_SCHEDULE, SCHEDULE_CHOICES, SCHEDULE_FIELDS
from paper_2107_01276_amd import tune


class FakeCtx:
    """Launch times from a table: pass A fastest at (8, 4), pass B at
    (1, 4, 1) except for one outlier round; the list is never rebuilt."""

    def __init__(self):
        self.sched = dict(DEFAULT_SCHEDULE)
        self.kern = None
        self.calls = 0
        self.seen = []

    @property
    def schedule(self):
        return dict(self.sched)

    def set_schedule(self, **kw):
        for k, v in kw.items():
            assert v in SCHEDULE_CHOICES[k], (k, v)
        self.sched.update(kw)
        return dict(self.sched)

    def profile(self, on=True, kernels=(), every=1):
        self.kern = kernels[0] if on else None

    def profile_reset(self):
        pass

    def profile_read(self, kern):
        s = self.sched
        self.calls += 1
        self.seen.append((kern, dict(s)))
        if kern == "pass_a":
            t = 1.0 + abs(s["a_lanes"] - 8) * 0.1 + abs(s["a_waves"] - 4) * 0.05
            return 10 * t, 10
        if kern == "pass_b":
            t = 1.0 + abs(s["b_lanes"] - 1) * 0.1 + abs(s["b_unroll"] - 4) * 0.1 + s["b_waves"] * 0.01
            if self.calls % 37 == 0:
                t = 0.1  # one outlier window: the median ignores it
            return 10 * t, 10
        return 0.0, 0


def test_variants_are_the_compiled_product():
    v = tune._variants(("b_lanes", "b_unroll", "b_waves"))
    assert len(v) == 3 * 2 * 2 and len({tuple(sorted(d.items())) for d in v}) == 12
    assert set(SCHEDULE_FIELDS) == set(SCHEDULE_CHOICES)


def test_tune_picks_fastest_and_caches(tmp_path):
    path = str(tmp_path / "sched.json")
    ctx = FakeCtx()
    res = tune.tune_schedule(ctx, lambda k: None, n=200_000, precision="fp32", rounds=3,
                             cache_path=path)
    assert res["source"] == "tuned"
    assert res["schedule"]["a_lanes"] == 8 and res["schedule"]["a_waves"] == 4
    assert (res["schedule"]["b_lanes"], res["schedule"]["b_unroll"], res["schedule"]["b_waves"]) == (1, 4, 1)
    assert res["schedule"]["list_lanes"] == DEFAULT_SCHEDULE["list_lanes"]  # no launch: unchanged
    # while pass B was timed, pass A was held at its pick
    assert all(s["a_lanes"] == 8 and s["a_waves"] == 4 for k, s in ctx.seen if k == "pass_b")
    data = json.load(open(path))
    assert res["key"] in data and res["key"].endswith("|fp32|2^17")
    ctx2 = FakeCtx()
    res2 = tune.tune_schedule(ctx2, lambda k: None, n=150_000, precision="fp32", cache_path=path)
    assert res2["source"] == "cache" and ctx2.calls == 0 and ctx2.sched == res["schedule"]
    res3 = tune.tune_schedule(FakeCtx(), lambda k: None, n=1000, precision="fp32", cache_path=path)
    assert res3["source"] == "tuned"  # another bucket
