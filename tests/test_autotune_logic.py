"""The autotuner's host logic on the CPU: it measures every candidate, keeps the
fastest, and caches the choice per workload key in its JSON file."""
import json

from paper_2102_00319_amd import runtime


def test_autotuner_picks_fastest_and_caches(tmp_path):
    path = tmp_path / "tune.json"
    t = runtime.Autotuner(str(path))
    cands = [{"graph": g, "chunk": c} for g in (False, True) for c in (0, 16)]
    cost = {(False, 0): 3.0, (False, 16): 2.0, (True, 0): 1.5, (True, 16): 1.7}
    seen = []

    def measure(c):
        seen.append(c)
        return cost[(c["graph"], c["chunk"])]
    best, times = t.tune("k1", cands, measure)
    assert best == {"graph": True, "chunk": 0}
    assert len(seen) == len(cands) and len(times) == len(cands)
    assert runtime.Autotuner(str(path)).lookup("k1") == best
    data = json.loads(path.read_text())
    assert set(data) == {"k1"} and data["k1"]["best"] == best
    assert runtime.Autotuner(str(path)).lookup("missing") is None


def test_kernel_knobs_tuned_on_the_workload(tmp_path):
    """tune_knobs measures every combination of the named knobs (defaults first),
    applies the fastest to every context, and takes a cached choice without measuring."""
    class Ctx:
        def __init__(self):
            self.knobs = {}

        def set_tuning(self, k, v):
            self.knobs[k] = v

    assert runtime.knob_candidates(["ks_fuse_row_inner", "row_wg"]) == [
        {"ks_fuse_row_inner": 1, "row_wg": 128}, {"ks_fuse_row_inner": 1, "row_wg": 256},
        {"ks_fuse_row_inner": 0, "row_wg": 128}, {"ks_fuse_row_inner": 0, "row_wg": 256}]
    ctxs = [Ctx(), Ctx()]
    runs = []

    def run():
        runs.append(dict(ctxs[0].knobs))

    import torch
    sync = torch.cuda.synchronize
    torch.cuda.synchronize = lambda *a, **k: None   # no device here
    clock = iter(range(10 ** 6))
    real = runtime.time.perf_counter
    try:
        # the fourth candidate runs fastest: its run() calls take 1 tick, the others 5
        def fake_clock():
            return next(clock) * (1 if runs and runs[-1] == {"ks_fuse_row_inner": 0, "row_wg": 256} else 5)
        runtime.time.perf_counter = fake_clock
        t = runtime.Autotuner(str(tmp_path / "t.json"))
        best, times = runtime.tune_knobs(t, "w", ctxs, run, ["ks_fuse_row_inner", "row_wg"], reps=1)
    finally:
        runtime.time.perf_counter = real
        torch.cuda.synchronize = sync
    assert best == {"ks_fuse_row_inner": 0, "row_wg": 256} and len(times) == 4
    assert all(c.knobs == best for c in ctxs)
    n = len(runs)
    best2, times2 = runtime.tune_knobs(runtime.Autotuner(str(tmp_path / "t.json")), "w", ctxs, run,
                                       ["ks_fuse_row_inner", "row_wg"])
    assert best2 == best and times2 is None and len(runs) == n


def test_cached_choice_is_per_knob_set(tmp_path):
    """A choice cached for one set of knobs is not taken for another set: the workload
    key carries the knob names, so adding a knob measures again."""
    class Ctx:
        def __init__(self):
            self.knobs = {}

        def set_tuning(self, k, v):
            self.knobs[k] = v

    import torch
    sync = torch.cuda.synchronize
    torch.cuda.synchronize = lambda *a, **k: None   # no device here
    try:
        ctx = Ctx()
        calls = []
        t = runtime.Autotuner(str(tmp_path / "t.json"))
        best1, times1 = runtime.tune_knobs(t, "w", [ctx], lambda: calls.append(1), ["ks_fuse_row_inner"], reps=1)
        n1 = len(calls)
        best2, times2 = runtime.tune_knobs(runtime.Autotuner(str(tmp_path / "t.json")), "w", [ctx],
                                           lambda: calls.append(1), ["ks_fuse_row_inner", "ks_nt"], reps=1)
    finally:
        torch.cuda.synchronize = sync
    assert times1 is not None and times2 is not None and len(calls) > n1
    assert set(best1) == {"ks_fuse_row_inner"} and set(best2) == {"ks_fuse_row_inner", "ks_nt"}
    assert set(json.loads((tmp_path / "t.json").read_text())) == {"w|knobs=ks_fuse_row_inner",
                                                                  "w|knobs=ks_fuse_row_inner,ks_nt"}
