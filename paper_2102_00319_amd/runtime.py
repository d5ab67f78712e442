"""Batched execution of uneven work (mixed ring degrees and levels) and the
autotuner that picks its schedule.

A work list is split per parameter set (one context, and one HIP stream, per
ring degree); fhe_batch_run turns each context's list into a few ragged launch
sequences.  The schedule has four knobs, chosen by measurement:
  * graph:      eager launches, or one HIP graph captured over all contexts and
                replayed (no host launch cost on the critical path);
  * concurrent: contexts on their own streams (their launch sequences overlap on
                the GPU) or all on one stream;
  * chunk:      most items per ragged launch sequence (0 = all of a stage);
  * order:      the order in which the contexts' lists are issued.
The library's kernel knobs (fhe_ctx_set_tuning: the fused row pass and key inner
product, the tensor-MAC tile width and two-group tiles, the rescale's row-pass
workgroup) are tuned the same way, on the workload itself (tune_knobs).
"""
import json
import os
import time

import torch

from .fhe import OP_MUL_RELIN_RESCALE, OP_ROTATE, BatchOp, Ciphertext, capture_graph


class Autotuner:
    """Measures candidate configurations and keeps the fastest per workload key
    (a JSON cache, FHE_TUNE_CACHE or a file beside this module)."""

    def __init__(self, path=None):
        self.path = path or os.environ.get("FHE_TUNE_CACHE",
                                           os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                        ".tune_cache.json"))
        try:
            with open(self.path) as f:
                self.cache = json.load(f)
        except (OSError, ValueError):
            self.cache = {}

    def lookup(self, key):
        e = self.cache.get(key)
        return None if e is None else e["best"]

    def tune(self, key, candidates, measure):
        """measure(candidate) -> seconds; returns (best candidate, {name: seconds})."""
        times = {}
        for cand in candidates:
            times[json.dumps(cand, sort_keys=True)] = measure(cand)
        best_name = min(times, key=times.get)
        best = json.loads(best_name)
        self.cache[key] = {"best": best, "seconds": times}
        try:
            with open(self.path, "w") as f:
                json.dump(self.cache, f, indent=1)
        except OSError:
            pass
        return best, times


class UnevenBatch:
    """Jobs over several contexts; job = (context name, a, b): Rescale(Relin(a (x) b))
    then rotations of the product by each of `steps`.  Outputs are allocated once."""

    def __init__(self, ctxs, keys, jobs, steps):
        self.ctxs = ctxs              # name -> Context (each with its own stream)
        self.names = list(ctxs)
        self.ops = {n: [] for n in ctxs}
        self.products, self.rotations = [], []
        for name, a, b in jobs:
            g = ctxs[name]
            rlk, gks = keys[name]
            m = BatchOp(OP_MUL_RELIN_RESCALE, a, rlk, b=b, out=g.new_ct(a.limbs - 1, 2))
            self.ops[name].append(m)
            rot = []
            for r in steps:
                op = BatchOp(OP_ROTATE, m.out, gks[r], step=r, out=g.new_ct(a.limbs - 1, 2))
                self.ops[name].append(op)
                rot.append(op.out)
            self.products.append(m.out)
            self.rotations.append(rot)
        self.streams = {n: ctxs[n].stream for n in ctxs}
        self._graph = None
        self._graph_cfg = None

    def _apply(self, cfg):
        order = cfg.get("order", self.names)
        first = self.streams[order[0]]
        for n in self.names:
            s = self.streams[n] if cfg.get("concurrent", True) else first
            if self.ctxs[n].stream is not s:
                self.ctxs[n].use_stream(s)
            self.ctxs[n].set_tuning("chunk_items", cfg.get("chunk", 0))
        return order

    def run_eager(self, cfg):
        for n in self._apply(cfg):
            self.ctxs[n].batch_run(self.ops[n])

    def _issue(self, order):
        for n in order:
            self.ctxs[n].batch_run(self.ops[n])

    def run(self, cfg):
        """One pass over the whole batch with configuration cfg (asynchronous)."""
        if not cfg.get("graph"):
            self._graph_cfg = None
            return self.run_eager(cfg)
        if self._graph is None or self._graph_cfg != cfg:
            order = self._apply(cfg)
            self._issue(order)                    # eager run: sizes every scratch buffer
            torch.cuda.synchronize()
            if self._graph is not None:
                self._graph.close()
            self._graph = capture_graph([self.ctxs[n] for n in order], lambda: self._issue(order))
            self._graph_cfg = cfg
        self._graph.launch()

    def close(self):
        if self._graph is not None:
            self._graph.close()
            self._graph = None

    def time(self, cfg, reps=3):
        self.run(cfg)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            self.run(cfg)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        ts.sort()
        return ts[len(ts) // 2]

    def candidates(self):
        out = []
        for graph in (False, True):
            for conc in (True, False):
                for chunk in (0, 64, 16):
                    out.append({"graph": graph, "concurrent": conc, "chunk": chunk,
                                "order": sorted(self.names, key=lambda n: -self.ctxs[n].N)})
        return out

    def signature(self):
        parts = []
        for n in sorted(self.ops):
            lv = sorted(op.a.limbs for op in self.ops[n] if op.kind == OP_MUL_RELIN_RESCALE)
            parts.append("%s:%s" % (n, ",".join(map(str, lv))))
        return "uneven|" + "|".join(parts) + "|" + torch.cuda.get_device_name(0)


# kernel knobs of the library (fhe_ctx_set_tuning) and the values tried
KNOB_VALUES = {"ks_fuse_row_inner": (1, 0), "ks_nt": (1, 0), "row_wg": (128, 256)}


def knob_candidates(names):
    """Every combination of the listed knobs' values, the library defaults first."""
    out = [{}]
    for n in names:
        out = [dict(c, **{n: v}) for c in out for v in KNOB_VALUES[n]]
    return out


def apply_knobs(ctxs, knobs):
    for c in ctxs:
        for k, v in knobs.items():
            c.set_tuning(k, v)


def tune_knobs(tuner, key, ctxs, run, names, reps=3):
    """Measure run() (a whole workload step, asynchronous) under every combination of
    the named kernel knobs, applied to every context in ctxs; keep the fastest (cached
    under key by the tuner) and leave it applied.  Returns (best, {candidate: seconds})."""
    def measure(knobs):
        apply_knobs(ctxs, knobs)
        run()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            run()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        ts.sort()
        return ts[len(ts) // 2]
    key = "%s|knobs=%s" % (key, ",".join(names))
    best = tuner.lookup(key)
    times = None
    if best is None or set(best) != set(names):
        best, times = tuner.tune(key, knob_candidates(names), measure)
    apply_knobs(ctxs, best)
    return best, times


class GraphedForward:
    """A layer sequence captured once into a HIP graph and replayed.

    fn(X) enqueues the whole sequence on `ctx` (its own stream, not the default one)
    and returns its output ciphertexts.  The constructor runs fn once eagerly (sizing
    the context's scratch and workspace and filling torch's cache with blocks of the
    right sizes), then captures a second run.  Every buffer allocated during the
    capture is kept for the graph's lifetime, so replays write the same intermediates
    and outputs.  The graph reads its own copies of X, made at construction; run(X2)
    copies new inputs (same levels and scales) into them first.  One replay is one
    launch for the whole sequence: the host work between layer kernels (tables,
    chunking) is done once, at capture."""

    def __init__(self, ctx, fn, X, table_bytes=256 << 20):
        if ctx.stream == torch.cuda.default_stream(ctx.device):
            raise ValueError("GraphedForward: the context needs a stream of its own (use_stream)")
        self.ctx = ctx
        self.X = []                           # the graph's own input buffers
        with torch.cuda.stream(ctx.stream):
            for x in X:
                t = ctx.empty(*x.data.shape)
                t.copy_(x.data)
                self.X.append(Ciphertext(t, x.scale))
        warm = []
        ctx.keep_allocations(warm)
        try:
            fn(self.X)
        finally:
            ctx.keep_allocations(None)
        torch.cuda.synchronize(ctx.device)
        del warm                              # back to torch's cache, sized for the capture
        self._kept, out = [], []
        ctx.keep_allocations(self._kept)
        try:
            self.graph = capture_graph([ctx], lambda: out.append(fn(self.X)), table_bytes)
        finally:
            ctx.keep_allocations(None)
        self.out = out[0]

    def run(self, X=None):
        """Replay (asynchronous on the context's stream); returns the output ciphertexts."""
        if X is not None:
            X = list(X)
            if len(X) != len(self.X):
                raise ValueError("GraphedForward.run: %d inputs, captured with %d" % (len(X), len(self.X)))
            with torch.cuda.stream(self.ctx.stream):
                for dst, src in zip(self.X, X):
                    if src.data.shape != dst.data.shape or src.scale != dst.scale:
                        raise ValueError("GraphedForward.run: inputs must match the captured levels and scales")
                    dst.data.copy_(src.data)
        self.graph.launch()
        return self.out

    def close(self):
        self.graph.close()
        self._kept = []
