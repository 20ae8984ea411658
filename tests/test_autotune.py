"""Host logic of the autotuner (no GPU): a stand-in context returns
synthetic per-class launch times for each scheduling candidate; the tuner
must keep each class's fastest candidate, keep the preferred one within the
noise margin, apply its choice, and round-trip the table through JSON."""
import numpy as np
import pytest

from paper_1708_00033_amd import autotune, hfx


class FakeContext:
    """Per-class time of a candidate = times[candidate][class]."""

    def __init__(self, times, fp32_times=None):
        self.times = times
        self.fp32_times = fp32_times
        self.current = None
        self.fp32 = np.ones(21, dtype=int)
        self.applied = {}
        self.timing = False
        self.acc = np.zeros(21)
        self.builds = 0

    def set_class_tuning(self, cls, tq, st=-1, pe=0, dg=-1):
        if cls == -1:
            self.current = (tq, st, pe, dg)
        else:
            self.applied[cls] = (tq, st, pe, dg)

    def set_class_precision(self, cls, on):
        if cls == -1:
            self.fp32[:] = on
        else:
            self.fp32[cls] = on

    def build_fock_dev(self, d, f, s):
        if not self.timing:
            return
        self.builds += 1
        if self.fp32_times is not None:
            self.acc += np.where(self.fp32 == 1, self.fp32_times[1], self.fp32_times[0])
        else:
            self.acc += np.asarray(self.times[self.current])

    def kernel_timing(self, on):
        self.timing = bool(on)
        if on:
            self.acc[:] = 0.0
            self.builds = 0

    def kernel_times(self):
        return self.acc.copy(), np.full(21, self.builds, dtype=np.int64)


def test_fastest_candidate_and_preferred_margin():
    cands = [(2048, 0, 0, -1), (32768, 0, 0, -1), (8192, 1, 2, -1)]
    t = {c: np.full(21, 10.0) for c in cands}
    t[(2048, 0, 0, -1)][0] = 5.0            # class 0: clearly faster elsewhere
    t[(8192, 1, 2, -1)][1] = 9.9            # class 1: within 3 % of the preferred -> preferred kept
    t[(8192, 1, 2, -1)][2] = 9.0            # class 2: 10 % faster -> taken
    ctx = FakeContext(t)
    table = autotune.autotune(ctx, 0, 0, 0, candidates=cands, reps=2, sync=lambda: None,
                              prefer=(32768, 0, 0, -1), margin=0.03)
    names = hfx.CLASS_NAMES
    assert autotune.summary(table)[names[0]] == (2048, 0, 0, -1)
    assert autotune.summary(table)[names[1]] == (32768, 0, 0, -1)
    assert autotune.summary(table)[names[2]] == (8192, 1, 2, -1)
    assert all(autotune.summary(table)[names[k]] == (32768, 0, 0, -1) for k in range(3, 21))
    assert table[names[0]]["ms"] == pytest.approx(5.0)
    # the choice is applied class by class
    assert ctx.applied[0] == (2048, 0, 0, -1) and ctx.applied[2] == (8192, 1, 2, -1)
    assert len(ctx.applied) == 21


def test_short_candidates_are_padded():
    cands = [(512, 0), (4096, 1, 1)]
    t = {(512, 0, 0, -1): np.full(21, 2.0), (4096, 1, 1, -1): np.full(21, 1.0)}
    ctx = FakeContext(t)
    table = autotune.autotune(ctx, 0, 0, 0, candidates=cands, reps=1, sync=lambda: None)
    assert set(autotune.summary(table).values()) == {(4096, 1, 1, -1)}


def test_precision_tuner_keeps_fp32_only_where_faster(tmp_path):
    fp64 = np.full(21, 10.0)
    fp32 = np.full(21, 10.0)
    fp32[4] = 8.0      # faster by 20 %: FP32 kept
    fp32[5] = 9.9      # within the 2 % margin: FP64
    fp32[6] = 12.0     # slower: FP64
    ctx = FakeContext(None, fp32_times=(fp64, fp32))
    table = autotune.autotune_precision(ctx, 0, 0, 0, reps=2, sync=lambda: None, margin=0.02)
    on = [table[n]["fp32"] for n in hfx.CLASS_NAMES]
    assert on[4] == 1 and on[5] == 0 and on[6] == 0 and sum(on) == 1
    assert list(ctx.fp32) == on


def test_table_round_trip(tmp_path):
    cands = [(8192, 0, 0, -1), (32768, 0, 1, 1)]
    t = {c: np.arange(21, dtype=float) + i for i, c in enumerate(cands)}
    ctx = FakeContext(t)
    table = autotune.autotune(ctx, 0, 0, 0, candidates=cands, reps=1, sync=lambda: None)
    p = tmp_path / "tuning.json"
    autotune.save(table, str(p))
    back = autotune.load(str(p))
    assert autotune.summary(back) == autotune.summary(table)
    ctx2 = FakeContext(t)
    autotune.apply(ctx2, back)
    assert ctx2.applied == ctx.applied
