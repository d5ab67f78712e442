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
