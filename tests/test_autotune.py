"""The launch tuner (autotune.tune_run, Schedule, TuneCache) on a stand-in engine whose step
times are scripted: per size class it must pick the fastest launch shape, then the fastest
child-arena size with that shape, give every step its class's choice, skip the classes a
cache already knows, and keep the best so far for a class the run leaves early; then the
refill threshold with that shape.  No GPU."""
import math
from types import SimpleNamespace

import numpy as np

from paper_1412_6426_amd import autotune as AT

MIN_LIVE = 1 << 10


class FakeEngine:
    """Live count growing by `growth` per step; a step's time is live particles times a
    per-particle cost that depends on the shape and the size class."""

    def __init__(self, cost, n0=100, growth=1.25, cap=None):
        self.cost, self.live, self.growth, self.cap = cost, n0, growth, cap
        self.arena = 0
        self.stream = 0
        self.last_ms = 0.0
        self.done = 0
        self.shapes = []

    def counts(self):
        return np.array([[self.live, 0, 0]], dtype=np.int64)

    def set_arena(self, divisor):
        self.arena = divisor

    def step(self, field, params):
        shape = (params.tile, params.grid_blocks, self.arena, params.refill_min)
        self.shapes.append(shape)
        self.done = self.live
        self.last_ms = self.live * self.cost(shape, self.live)
        grown = int(math.ceil(self.live * self.growth))
        self.live = grown if self.cap is None else min(grown, self.cap)

    def stats(self):
        return {"advanced": [self.done, 0, 0], "dropped": 0}


class FakeTimer:
    def __init__(self, engine):
        self.e = engine

    def start(self, stream):
        pass

    def stop_ms(self, stream):
        return self.e.last_ms


CANDS = AT.default_candidates(256)


def cls_of(live):
    return -1 if live < MIN_LIVE else int(math.log(live / MIN_LIVE, 4.0))


def scripted_cost(shape, live):
    """Small classes like 64-particle chunks, large ones 512; arena divisor 8 is best at
    every size; the default grid beats the smaller and larger ones; small classes refill
    every idle lane, large ones in batches of 40."""
    tile, grid, arena, refill = shape
    want_tile = 64 if cls_of(live) < 2 else 512
    c = 1.0 + 0.1 * abs(math.log2(max(tile, 1) / want_tile))
    c += 0.05 if grid else 0.0
    c += {0: 0.02, 2: 0.03, 8: 0.0, 32: 0.04}[arena]
    want_refill = 1 if cls_of(live) < 2 else 40
    c += 0.0 if refill == want_refill else 0.01
    return c


def _tune(e, steps, **kw):
    params = SimpleNamespace(tile=0, grid_blocks=0, refill_min=0)
    return AT.tune_run(e, None, params, steps, CANDS, min_live=MIN_LIVE, timer=FakeTimer(e),
                       sync=lambda: None, **kw)


def test_each_class_gets_its_fastest_launch_shape_then_arena():
    # 1.04 a step: a class (a factor 4) lasts 35 steps, more than its 28 trial steps
    e = FakeEngine(scripted_cost, growth=1.04)
    sched = _tune(e, 240)
    lives = [100]
    for _ in range(239):
        lives.append(int(math.ceil(lives[-1] * 1.04)))
    classes = sorted({cls_of(v) for v in lives if cls_of(v) >= 0})
    assert len(classes) >= 3
    for c in classes[:-1]:  # the last class may be cut short by the end of the run
        want_tile = 64 if c < 2 else 512
        assert sched.choices[c] == (want_tile, 0, 8, 1 if c < 2 else 40), c
    # every step follows its class's choice (trial steps included), the default below
    # min_live, and the trials tried both phases
    for n, live in enumerate(lives):
        c = cls_of(live)
        assert sched.shape_at(n) == (sched.choices.get(c, AT.DEFAULT_SHAPE) if c >= 0
                                     else AT.DEFAULT_SHAPE)
    tried = {(t["tile"], t["grid"], t["arena_div"], t["refill"]) for t in sched.trials}
    assert set(CANDS) <= tried and {(64, 0, 2, 0), (64, 0, 32, 0)} <= tried
    assert {(64, 0, 8, 1), (64, 0, 8, 16), (64, 0, 8, 40)} <= tried
    assert sched.distinct()[0] == AT.DEFAULT_SHAPE
    # the engine really ran the trial shapes, and each class's choice afterwards
    assert e.shapes[0] == AT.DEFAULT_SHAPE
    assert (512, 0, 8, 40) in e.shapes


def test_known_classes_skip_their_trials(tmp_path):
    e = FakeEngine(scripted_cost, growth=1.08)
    first = _tune(e, 160)
    path = str(tmp_path / "tune.json")
    cache = AT.TuneCache(path)
    key = AT.TuneCache.key("gfx950", "f64", "rotating-E cascade")
    cache.put(key, first.choices)
    again = AT.TuneCache(path)
    assert again.get(key) == first.choices
    assert again.get(AT.TuneCache.key("gfx950", "mixed", "rotating-E cascade")) == {}
    e2 = FakeEngine(scripted_cost, growth=1.08)
    second = _tune(e2, 160, known=again.get(key))
    known_classes = set(first.choices)
    assert not [t for t in second.trials if t["cls"] in known_classes]
    assert second.shapes == first.shapes and second.steps == first.steps


def test_a_class_left_early_keeps_its_best_so_far():
    # growth so fast that each class lasts only a few steps: fewer than its trials
    e = FakeEngine(scripted_cost, growth=2.5)
    sched = _tune(e, 12)
    for c, shape in sched.choices.items():
        timed = [t for t in sched.trials if t["cls"] == c]
        assert timed, c
        best = min(timed, key=lambda t: t["ms"] / t["particle_steps"])
        assert shape == (best["tile"], best["grid"], best["arena_div"], best["refill"])


def test_schedule_lookup():
    a, b, c = (0, 0, 0, 0), (64, 0, 8, 40), (512, 0, 2, 1)
    s = AT.Schedule(steps=[0, 5, 9], shapes=[a, b, c])
    assert [s.shape_at(n) for n in (0, 4, 5, 8, 9, 100)] == [a, a, b, b, c, c]
    assert s.distinct() == [a, b, c]
    assert AT.Schedule().distinct() == [AT.DEFAULT_SHAPE]


def test_cache_entries_without_a_refill_threshold_read_as_the_default(tmp_path):
    import json
    path = tmp_path / "old.json"
    path.write_text(json.dumps({"k": {"0": [64, 0, 8], "2": [512, 0, 2]}}))
    assert AT.TuneCache(str(path)).get("k") == {0: (64, 0, 8, 0), 2: (512, 0, 2, 0)}


class ChildEngine(FakeEngine):
    """One child per live particle a step, and arenas of 10^6 / divisor records."""

    RECORDS = 10 ** 6

    def arena_records_for(self, divisor):
        return self.RECORDS if divisor <= 0 else self.RECORDS // divisor

    def stats(self):
        return {"advanced": [self.done, 0, 0], "dropped": 0, "emitted": self.done,
                "pairs": 0}


def test_arenas_without_room_for_the_class_are_not_tried():
    """Divisor 32 is the fastest in the scripted costs below, but an arena that the
    children of a class's last steps would overflow sends them to direct reservations: a
    class whose busiest trial step has n children tries only arenas of at least
    2 x 4 x n records."""
    def cost(shape, live):
        tile, grid, arena, refill = shape
        return 1.0 + {0: 0.02, 2: 0.03, 8: 0.01, 32: 0.0}[arena] + (0.05 if tile != 128 else 0)

    e = ChildEngine(cost, growth=1.04)
    sched = _tune(e, 300)
    seen_small = seen_large = False
    for c, shape in sched.choices.items():
        div = shape[2]
        tried = {t["arena_div"] for t in sched.trials if t["cls"] == c}
        # the busiest step (one child per particle) before the class's arena trials began
        first_arena = min((t["step"] for t in sched.trials
                           if t["cls"] == c and t["arena_div"] > 0), default=None)
        peak = max((t["particle_steps"] for t in sched.trials
                    if t["cls"] == c and (first_arena is None or t["step"] < first_arena)),
                   default=0)
        need = AT.ARENA_ROOM * 4.0 * peak
        for d in tried - {0}:
            assert e.arena_records_for(d) >= need, (c, d, need)
        assert div == 0 or e.arena_records_for(div) >= need
        if 32 in tried:
            seen_small = True
        if need > e.arena_records_for(32):
            seen_large = True
            assert 32 not in tried
    assert seen_small and seen_large


def test_a_class_whose_arena_a_later_step_outgrows_falls_back_to_the_whole_arena():
    """Thinning can bring the live count back into a class with many more children per
    particle than when the class was tuned: its arena choice must then give way to the
    engine's whole arena (divisor 0) in the schedule."""
    def cost(shape, live):
        tile, grid, arena, refill = shape
        return 1.0 + {0: 0.02, 2: 0.03, 8: 0.01, 32: 0.0}[arena]

    class Mix(ChildEngine):
        RECORDS = 10 ** 7

        def __init__(self, *a, **kw):
            super().__init__(*a, **kw)
            self.n = 0

        def step(self, field, params):
            super().step(field, params)
            self.n += 1
            if self.n == 150:  # a thinning: back to a small class, now rich in children
                self.live = 2000
                self.growth = 1.0
                self.per = 200

        def stats(self):
            st = super().stats()
            st["emitted"] = self.done * getattr(self, "per", 1)
            return st

    e = Mix(cost, growth=1.04)
    sched = _tune(e, 200)
    c = cls_of(2000)
    assert c in sched.choices
    assert any(t["cls"] == c and t["arena_div"] == 32 for t in sched.trials)
    # 2000 particles x 200 children outgrow 10^7 / 32 records (x 2 room): the whole arena
    assert sched.choices[c][2] == 0
    assert sched.shape_at(199)[2] == 0
