"""Host logic of the serving loop on the CPU: admission in arrival order under an
HBM budget, least-recently-used eviction of idle clients only, slot merging of
one client's queued requests with distinct slot ranges, and completion
bookkeeping.  Lanes and clients are stand-ins; no device work is done."""
import types

import numpy as np
import pytest

from paper_2102_00319_amd import serving


class FakeClient:
    def __init__(self, cid, kind, nbytes):
        self.cid, self.kind, self.nbytes, self.set_name = cid, kind, nbytes, "s"
        self.resident, self.inflight, self.last_used, self.loads, self.hold = True, 0, 0.0, 0, False
        self.net = types.SimpleNamespace(H=4, W=4, Cout=1, Ho=2, Wo=2, c1=1, c2=1, k=3)
        self.mirror, self.mirror_bytes = None, 0

    def host_bytes(self):
        return self.mirror_bytes if self.mirror is not None else (0 if self.resident else self.nbytes)

    def evict(self):
        assert self.inflight == 0, "evicted a client with work in flight"
        self.resident = False

    def restore(self):
        self.resident = True
        self.loads += 1


class FakeLane:
    def __init__(self):
        self.ctx = {"s": types.SimpleNamespace(L=2, N=4)}
        self.group, self.thread, self.finished, self.error, self.ws = None, None, False, None, 0


class FakeServer(serving.Server):
    """Every batch finishes on the next poll; records what ran together."""

    def __init__(self, **kw):
        super().__init__(["s"], lane_factory=FakeLane, device="cpu", scratch_bytes=0, **kw)
        self.batches = []

    def _launch(self, lane, group, ws, now_fn):
        # the admitted batch's client state and working set fit the budget
        assert self.resident_bytes() + ws <= self.budget
        assert group[0].client.resident
        self.batches.append([r.rid for r in group])
        for r in group:
            r.scores = np.full((r.n, 1), float(r.rid))
            r.t_done = now_fn()
        lane.group, lane.ws, lane.finished, lane.error = group, ws, True, None
        lane.thread = types.SimpleNamespace(join=lambda: None)


def _ws(srv, req):
    return srv.working_set(req, srv.lanes[0])


def test_merging_takes_distinct_slot_ranges_of_one_client():
    srv = FakeServer(lanes=1, hbm_budget=1e12, merge=True, max_merge=3)
    a, b = FakeClient(0, "slot", 100), FakeClient(1, "slot", 100)
    for c in (a, b):
        srv.add_client(c)
    reqs = [serving.Request(i, c, [None], 1, 64 * t, 0.0, t)
            for i, (c, t) in enumerate([(a, 0), (a, 0), (a, 1), (b, 0), (a, 2), (a, 3)])]
    srv.run(reqs, time_limit=10)
    # first batch: request 0 plus the next requests of the same client with new tags (1 dup skipped), at most 3
    assert srv.batches[0] == [0, 2, 4]
    assert all(r.scores is not None for r in reqs)
    assert {r.rid: r.merged for r in reqs}[0] == 3


def test_budget_admission_and_lru_eviction():
    srv = FakeServer(lanes=2, hbm_budget=0, merge=False)
    cs = [FakeClient(i, "packed", 1000) for i in range(3)]
    for c in cs:
        srv.add_client(c)
    probe = serving.Request(99, cs[0], [None], 1, 0, 0.0, 0)
    ws = _ws(srv, probe)
    # room for two client states and one working set
    srv.budget = 2 * 1000 + ws
    reqs = [serving.Request(i, cs[i % 3], [None], 1, 0, 0.001 * i, 0) for i in range(9)]
    srv.run(reqs, time_limit=10)
    assert all(r.t_done is not None for r in reqs)
    # three clients over two resident slots: evictions and cold loads must have happened
    assert srv.stats["evictions"] > 0 and srv.stats["cold_loads"] > 0
    assert sum(c.resident for c in cs) <= 2
    # admission is in arrival order: completion order follows request ids
    order = [rid for b in srv.batches for rid in b]
    assert order == sorted(order)


def test_request_that_cannot_fit_waits_for_running_work():
    srv = FakeServer(lanes=2, hbm_budget=0, merge=False)
    c0, c1 = FakeClient(0, "packed", 1000), FakeClient(1, "packed", 1000)
    srv.add_client(c0)
    srv.add_client(c1)
    ws = _ws(srv, serving.Request(0, c0, [None], 1, 0, 0.0, 0))
    srv.budget = 1000 + ws          # only one client and one working set at a time
    reqs = [serving.Request(0, c0, [None], 1, 0, 0.0, 0), serving.Request(1, c1, [None], 1, 0, 0.0, 0)]
    srv.run(reqs, time_limit=10)
    assert [b for b in srv.batches] == [[0], [1]]
    assert c1.loads == 0 or c0.resident is False


def test_registration_over_budget_moves_older_clients_to_host():
    srv = FakeServer(lanes=1, hbm_budget=250, merge=False)
    cs = [FakeClient(i, "packed", 100) for i in range(4)]
    for c in cs:
        srv.add_client(c)
        assert c.resident                          # the new client stays
        assert srv.resident_bytes() <= srv.budget
    assert [c.resident for c in cs] == [False, False, True, True]
    assert srv.stats["evictions"] == 2


def test_warm_clients_first_then_overdue_cold_ones():
    srv = FakeServer(lanes=1, hbm_budget=1e12, merge=False, cold_wait=1.0)
    a, b = FakeClient(0, "packed", 100), FakeClient(1, "packed", 100)
    srv.add_client(a)
    srv.add_client(b)
    b.evict()
    q = [serving.Request(0, b, [None], 1, 0, 0.0, 0), serving.Request(1, a, [None], 1, 0, 0.1, 0)]
    assert srv._order(q, 0.2) == [1]          # b's request waits behind the resident client's
    assert srv._order(q, 1.5) == [0, 1]       # overdue: it goes first
    assert srv._order(q[:1], 0.2) == [0]      # nothing warm queued: no reason to wait
    srv.cold_wait = None
    assert srv._order(q, 0.2) == [0, 1]       # arrival order


def test_eviction_spares_clients_with_queued_requests():
    srv = FakeServer(lanes=1, hbm_budget=1e12, merge=False)
    a, b, c = (FakeClient(i, "packed", 100) for i in range(3))
    for x in (a, b, c):
        srv.add_client(x)
    a.last_used, b.last_used, c.last_used = 1.0, 2.0, 3.0
    srv.budget = 200
    queued = [serving.Request(0, a, [None], 1, 0, 0.0, 0)]
    assert srv._make_room(0, c, queued)
    assert a.resident and not b.resident     # b is evicted although a was used less recently


def test_eviction_prefers_the_smallest_sufficient_client():
    srv = FakeServer(lanes=1, hbm_budget=1e12, merge=False)
    big, s1, s2 = FakeClient(0, "slot", 400), FakeClient(1, "packed", 100), FakeClient(2, "packed", 100)
    for x in (big, s1, s2):
        srv.add_client(x)
    big.last_used, s1.last_used, s2.last_used = 1.0, 3.0, 2.0
    srv.budget = 550
    new = FakeClient(3, "packed", 50)
    srv.add_client(new)                      # 650 resident: 100 must go
    assert big.resident and not s2.resident and s1.resident   # not the least recently used big one
    assert srv.resident_bytes() == 550
    srv.budget = 300                         # 250 short: no small client suffices alone
    assert srv._make_room(0, new)
    assert not big.resident and s1.resident


def test_host_budget_keeps_a_client_resident():
    srv = FakeServer(lanes=1, hbm_budget=1e12, merge=False, host_budget=150)
    a, b = FakeClient(0, "packed", 100), FakeClient(1, "packed", 100)
    srv.add_client(a)
    srv.add_client(b)
    srv.budget = 150
    assert srv._make_room(0, b) and not a.resident     # 100 on the host
    srv.budget = 50
    assert not srv._make_room(0, None)                 # b's copy would exceed the host budget
    assert b.resident
    b.mirror, b.mirror_bytes = [], 0                   # a mirror needs no new host memory
    assert srv._make_room(0, None) and not b.resident


def test_mirror_size_packs_objects_into_pinned_blocks():
    blk = serving.PIN_BLOCK
    assert serving.Client.mirror_size([]) == 0
    assert serving.Client.mirror_size([100, 200]) == blk
    assert serving.Client.mirror_size([blk // 2, blk // 2 + 1]) == 2 * blk
    assert serving.Client.mirror_size([blk + 8, 16]) == 2 * blk + 8


def test_make_mirrors_smallest_first_within_host_budget():
    class MirClient(FakeClient):
        objs = ()

        def mirror_size(self, sizes):
            return self.nbytes

        def make_mirror(self, pinned=True):
            self.mirror, self.mirror_bytes = [], self.nbytes

    srv = FakeServer(lanes=1, hbm_budget=1e12, merge=False, host_budget=250)
    big, s1, s2 = MirClient(0, "slot", 200), MirClient(1, "packed", 100), MirClient(2, "packed", 100)
    for x in (big, s1, s2):
        srv.add_client(x)
    assert srv.make_mirrors() == [s1, s2]
    assert big.mirror is None and srv.host_bytes() == 200


def test_mirrored_client_evicted_before_an_equal_one_without():
    srv = FakeServer(lanes=1, hbm_budget=1e12, merge=False)
    a, b, keep = FakeClient(0, "packed", 100), FakeClient(1, "packed", 100), FakeClient(2, "packed", 100)
    for x in (a, b, keep):
        srv.add_client(x)
    a.last_used, b.last_used = 1.0, 2.0
    b.mirror, b.mirror_bytes = [], 100
    srv.budget = 200
    assert srv._make_room(0, keep) and a.resident and not b.resident


def test_refused_pinned_allocation_turns_to_pageable_mirrors():
    class MirClient(FakeClient):
        objs = ()

        def mirror_size(self, sizes):
            return self.nbytes

        def make_mirror(self, pinned=True):
            if self.cid == 1 and pinned:
                raise RuntimeError("HIP error: out of memory\nmore")
            self.mirror, self.mirror_bytes, self.mirror_pinned = [], self.nbytes, pinned

    srv = FakeServer(lanes=1, hbm_budget=1e12, merge=False, host_budget=1000)
    cs = [MirClient(i, "packed", 100 + i) for i in range(3)]
    for x in cs:
        srv.add_client(x)
    assert srv.make_mirrors() == cs
    assert srv.mirror_error == "HIP error: out of memory"
    assert [c.mirror_pinned for c in cs] == [True, False, False]     # pageable after the refusal


def test_cold_load_runs_beside_warm_work():
    import threading
    gate = threading.Event()

    class SlowClient(FakeClient):
        def restore(self):
            assert gate.wait(10)
            super().restore()

    srv = FakeServer(lanes=1, hbm_budget=1e12, merge=False, cold_wait=0.5)
    assert srv.async_loads
    warm, cold = FakeClient(0, "packed", 100), SlowClient(1, "packed", 100)
    srv.add_client(warm)
    srv.add_client(cold)
    cold.evict()
    q = [serving.Request(0, cold, [None], 1, 0, 0.0, 0), serving.Request(1, warm, [None], 1, 0, 0.1, 0),
         serving.Request(2, cold, [None], 1, 0, 0.2, 0)]
    srv._now = lambda: 1.0
    assert srv._admit(srv.lanes[0], q, 1.0)            # overdue cold request: its load starts ...
    assert srv.loading is not None and srv.loading[0] is cold and cold.resident and cold.inflight == 1
    assert srv.batches == [[1]]                        # ... and the warm request runs meanwhile
    assert q[0].cold and q[-1].cold                    # both of the client's queued requests wait on it
    srv._poll()
    assert not srv._admit(srv.lanes[0], q, 1.0)        # nothing admissible while it loads
    srv.budget = 100
    assert srv._make_room(0, None) and cold.resident and not warm.resident   # a loading client stays
    srv.budget = 1e12
    gate.set()
    srv.loading[1].join()
    assert not srv._admit(srv.lanes[0], q, 1.0)        # finished, but not yet seen by the scheduler
    srv._poll_load()
    assert srv.loading is None and srv.stats["cold_loads"] == 1
    assert cold.inflight == 1 and cold.hold          # held for its queued requests
    srv.budget = 100
    assert not srv._make_room(100, None) and cold.resident
    srv.budget = 1e12
    assert srv._admit(srv.lanes[0], q, 1.0) and srv.batches[-1] == [0]
    assert cold.inflight == 1 and not cold.hold      # now only the running batch holds it
    srv._poll()
    assert cold.inflight == 0


def test_async_loads_serve_every_request():
    srv = FakeServer(lanes=2, hbm_budget=0, merge=False, cold_wait=0.002)
    cs = [FakeClient(i, "packed", 1000) for i in range(3)]
    for c in cs:
        srv.add_client(c)
    srv.budget = 2 * 1000 + 2 * _ws(srv, serving.Request(99, cs[0], [None], 1, 0, 0.0, 0))
    reqs = [serving.Request(i, cs[i % 3], [None], 1, 0, 0.001 * i, 0) for i in range(12)]
    srv.run(reqs, time_limit=10)
    assert all(r.t_done is not None for r in reqs)
    assert srv.stats["cold_loads"] > 0 and srv.loading is None
    assert srv.resident_bytes() <= srv.budget
    assert all(c.inflight == 0 and not c.hold for c in cs)     # every client evictable again


def test_library_memory_of_lanes_counts_against_the_budget():
    """A lane gives its library buffers back when its batch ends; the most a batch of a
    network kind held becomes that kind's reservation in later working sets."""
    srv = FakeServer(hbm_budget=10 ** 9)
    held, released = {"bytes": 0}, []
    for lane in srv.lanes:
        lane.library_bytes = lambda: held["bytes"]
        lane.release_buffers = lambda: released.append(1)
    c = FakeClient(0, "slot", 300)
    srv.add_client(c)
    req = serving.Request(0, c, None, 1, 0, 0.0, 0)
    before = _ws(srv, req)
    held["bytes"] = 5000
    srv.run([req])
    assert released and srv.library_peak["slot"] == 5000
    assert _ws(srv, req) == before + 5000      # the reservation of the FakeServer is 0
    assert srv.resident_bytes() == 300          # nothing held once the lanes are idle
