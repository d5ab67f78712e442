"""Serving loop for encrypted inference requests (continuous batching on one GPU).

The paper's setting (Sec. 2.1): a user sends encrypted images, the model is
encrypted under the user's key by its owner, the cloud evaluates.  A serving
process holds, per client, the evaluation keys and the encrypted weights
("client state"), and per request the encrypted images.  This module:
  * admits requests in arrival order as soon as a lane (an execution slot with
    its own contexts and HIP stream) is free and the HBM budget covers the
    client's state plus the request's working set; client state not resident is
    loaded (cold start), evicting idle clients to host memory when the budget
    requires (those with no queued request first, then the smallest one that
    frees enough, then the least recently used); client state is immutable while
    served, so a client may keep a pinned host mirror, and its evictions then
    free device memory without a copy back;
  * merges queued requests of one slot-packed client whose slot ranges are
    disjoint into one batch (ciphertext addition: each request's images sit in
    its own slots), up to max_merge requests;
  * runs the forward passes of different lanes concurrently on the device
    (requests that arrive while others run are admitted as lanes and memory free
    up), and measures latency from arrival to the decrypted scores.
"""
import collections
import threading
import time

import numpy as np
import torch

from .fhe import Context, CtArray

PIN_BLOCK = 1 << 30   # pinned host mirrors are packed into blocks of this size


class Client:
    """One user (secret key, public key, evaluation keys) with a model encrypted under
    its key; kind 'slot' (SlotCNN) or 'packed' (PackedCNN)."""

    def __init__(self, cid, net, ctx, set_name, weights_plain, seeds):
        self.cid, self.net, self.set_name = cid, net, set_name
        self.kind = "packed" if hasattr(net, "frame") else "slot"
        self.sk = ctx.keygen_secret(seeds["secret"])
        self.pk = ctx.keygen_pk(self.sk, seeds["pk"])
        self.rlk, self.gks = net.keygen(ctx, self.sk, seeds["evk"])
        self.weights = net.encrypt_weights(ctx, self.pk, *weights_plain, seeds["weights"])
        self.objs = [self.rlk] + list(self.gks.values()) + [w for grp in self.weights for w in grp]
        self.nbytes = sum(o.data.numel() * 8 for o in self.objs)
        self.resident, self.inflight, self.last_used, self.loads = True, 0, 0.0, 0
        self.hold = False        # loaded for queued requests: kept until one is admitted
        self.device = ctx.device
        self.mirror, self.mirror_bytes, self.mirror_pinned = None, 0, False

    def host_bytes(self):
        """Host memory the client holds: its pinned mirror, else the evicted copy."""
        return self.mirror_bytes if self.mirror is not None else (0 if self.resident else self.nbytes)

    @staticmethod
    def mirror_size(nbytes_list):
        """Pinned bytes make_mirror takes for objects of these sizes."""
        total, used = 0, PIN_BLOCK
        for nb in nbytes_list:
            if nb > PIN_BLOCK:
                total += nb
                continue
            if used + nb > PIN_BLOCK:
                total, used = total + PIN_BLOCK, 0
            used += (nb + 255) & ~255
        return total

    def make_mirror(self, pinned=True):
        """Copy the client state once into host memory: pinned, packed into 1 GiB blocks
        (the pinned allocator rounds each allocation up to a power of two), or pageable.
        A resident client keeps its device copy; an evicted one swaps its host copy for
        the mirror."""
        if not pinned:
            self.mirror = [o.data.to("cpu") for o in self.objs]
            self.mirror_bytes, self.mirror_pinned = self.nbytes, False
            return
        views, size, cur, used = [], 0, None, PIN_BLOCK
        for o in self.objs:
            nb = o.data.numel() * o.data.element_size()
            if nb > PIN_BLOCK:
                blk, off = torch.empty(nb, dtype=torch.uint8, pin_memory=True), 0
                size += nb
            else:
                if used + nb > PIN_BLOCK:
                    cur, used = torch.empty(PIN_BLOCK, dtype=torch.uint8, pin_memory=True), 0
                    size += PIN_BLOCK
                blk, off = cur, used
                used += (nb + 255) & ~255
            h = blk[off:off + nb].view(o.data.dtype).view(o.data.shape)
            h.copy_(o.data)
            views.append(h)
            if not self.resident:
                o.data = h
        self.mirror, self.mirror_bytes, self.mirror_pinned = views, size, True

    def evict(self):
        if self.mirror is not None:
            for o, h in zip(self.objs, self.mirror):
                o.data = h
        else:
            for o in self.objs:
                o.data = o.data.to("cpu")
        self.resident = False

    def restore(self):
        pinned = self.mirror is not None and self.mirror_pinned
        for o in self.objs:
            o.data = o.data.to(self.device, non_blocking=pinned)
        if pinned:
            torch.cuda.current_stream(self.device).synchronize()
        for grp in self.weights:   # packed descriptor arrays hold device addresses
            if isinstance(grp, CtArray):
                grp.refresh()
        self.resident = True
        self.loads += 1


class Request:
    def __init__(self, rid, client, payload, n_images, slot_offset, t_arrival, tag):
        self.rid, self.client, self.payload = rid, client, payload
        self.n, self.off, self.t_arrival, self.tag = n_images, slot_offset, t_arrival, tag
        self.t_admit = self.t_done = None
        self.scores = None
        self.cold = False
        self.merged = 1


class Lane:
    """An execution slot: its own contexts (one per parameter set) on its own HIP
    stream, driven by its own host thread, so that a lane waiting for the device
    never holds up the others."""

    def __init__(self, set_names, device):
        self.stream = torch.cuda.Stream(device=device)
        self.ctx = {n: Context.from_set(n, stream=self.stream) for n in set_names}
        for ctx in self.ctx.values():   # the library's buffers come from torch's cache and budget
            ctx.use_torch_allocator()
        self.group, self.thread, self.finished, self.error, self.ws = None, None, False, None, 0

    def library_bytes(self):
        """Device memory the lane's contexts hold for their scratch and workspaces."""
        return sum(ctx.library_bytes() for ctx in self.ctx.values())

    def release_buffers(self):
        for ctx in self.ctx.values():
            ctx.release_buffers()


class Server:
    def __init__(self, set_names, lanes=4, hbm_budget=250e9, merge=True, max_merge=64, scratch_bytes=4 << 30,
                 device="cuda", lane_factory=None, cold_wait=None, host_budget=160e9, async_loads=None):
        self.device = torch.device(device)
        self.scratch = int(scratch_bytes)   # device scratch a lane may hold while it runs
        make = lane_factory or (lambda: Lane(set_names, self.device))
        self.lanes = [make() for _ in range(lanes)]
        self.budget, self.merge, self.max_merge = float(hbm_budget), merge, max_merge
        # None: admission in arrival order.  A number of seconds: requests of resident
        # clients go first, and a request whose client state sits in host memory is
        # admitted (with its cold load) once it has waited that long or when no request
        # of a resident client is queued, so that an over-budget client mix does not
        # move client state back and forth on every request.
        self.cold_wait = cold_wait
        # with the warm-first policy a cold load runs on a loader thread and its own
        # stream (one at a time: they share the PCIe link) while lanes keep serving
        # resident clients; in arrival order it runs before its request, in line
        self.async_loads = (cold_wait is not None) if async_loads is None else bool(async_loads)
        self.copy_stream = torch.cuda.Stream(device=self.device) if self.device.type == "cuda" else None
        self.loading = None      # (client, thread, box) of the load in progress
        # host memory for client state moved off the device (pinned mirrors and
        # evicted copies); a client whose eviction would exceed it stays resident
        self.host_budget = float(host_budget)
        self.mirror_error = None
        self.clients = []
        self.stats = collections.Counter()
        # the most library memory (scratch and workspace) a batch of each network kind
        # has held, measured when its lane finished
        self.library_peak = {}

    # ------------------------------------------------------------ memory
    def add_client(self, client):
        """Register a client; idle clients move to host memory while the resident state
        exceeds the budget (the new one stays)."""
        self.clients.append(client)
        self._make_room(0, client)

    def make_mirrors(self, progress=None):
        """Give registered clients host mirrors, smallest state first, while the host
        budget holds them: pinned while pinned allocations succeed (the system may lock
        less memory than the budget), pageable after that; returns the clients mirrored."""
        done, pinned = [], True
        for c in sorted(self.clients, key=lambda c: c.nbytes):
            if c.mirror is not None:
                continue
            sizes = [o.data.numel() * o.data.element_size() for o in c.objs]
            size = c.mirror_size(sizes) if pinned else c.nbytes
            if self.host_bytes() - c.host_bytes() + size > self.host_budget:
                continue
            try:
                c.make_mirror(pinned)
            except RuntimeError as e:      # pinned allocation refused: pageable from here on
                self.mirror_error = str(e).splitlines()[0]
                torch._C._host_emptyCache()
                pinned = False
                if self.host_bytes() - c.host_bytes() + c.nbytes > self.host_budget:
                    continue
                c.make_mirror(False)
            done.append(c)
            if progress:
                progress(c)
        return done

    def resident_bytes(self):
        """Client state on the device plus the working sets of the running batches (a
        lane gives its library buffers back when its batch ends)."""
        return sum(c.nbytes for c in self.clients if c.resident) + sum(l.ws for l in self.lanes)

    def host_bytes(self):
        return sum(c.host_bytes() for c in self.clients)

    def working_set(self, req, lane):
        """Device bytes of one batch of `req`'s network beyond the client state: inputs
        and layer outputs (an estimate), plus the library buffers the batch's contexts
        grow to: the most measured for that kind of network so far, at least the
        configured scratch reservation."""
        ctx = lane.ctx[req.client.set_name]
        ct = 2 * ctx.L * ctx.N * 8
        lib = max(self.scratch, self.library_peak.get(req.client.kind, 0))
        if req.client.kind == "slot":
            net = req.client.net
            n_conv = net.Cout * net.Ho * net.Wo
            return int(net.H * net.W * ct * 2 + 3 * n_conv * ct + lib)
        net = req.client.net
        return int(len(req.payload) * ct * (4 + 2 * net.c2 + net.c1 * net.k * net.k) + lib)

    @staticmethod
    def _library_bytes(lane):
        f = getattr(lane, "library_bytes", None)
        return f() if f else 0

    def _make_room(self, need, keep, queue=()):
        """Evict idle clients other than `keep` until `need` more bytes fit, keeping the
        host memory they move to within the host budget."""
        waiting = {id(r.client) for r in queue}
        while self.resident_bytes() + need > self.budget:
            short = self.resident_bytes() + need - self.budget
            idle = [c for c in self.clients if c.resident and c.inflight == 0 and c is not keep
                    and (c.mirror is not None or self.host_bytes() + c.nbytes <= self.host_budget)]
            if not idle:
                return False
            # a client with a queued request is evicted last; of the others, the smallest
            # one that frees enough on its own (its cold load costs least), one with a
            # pinned mirror before one without, else the least recently used
            victim = min(idle, key=lambda c: (id(c) in waiting, c.nbytes < short,
                                              c.nbytes if c.nbytes >= short else 0, c.mirror is None,
                                              c.last_used))
            t0 = time.perf_counter()
            victim.evict()      # its device blocks stay in torch's cache for the next load
            self.stats["evict_s"] += time.perf_counter() - t0
            self.stats["evictions"] += 1
        return True

    # -------------------------------------------------------- scheduling
    def _order(self, queue, now):
        """Queue positions in the order admission tries them."""
        if self.cold_wait is None:
            return list(range(len(queue)))
        loading = self.loading[0] if self.loading is not None else None
        warm = [i for i, r in enumerate(queue) if r.client.resident and r.client is not loading]
        cold = [i for i, r in enumerate(queue) if not r.client.resident
                and (not warm or now - r.t_arrival >= self.cold_wait)]
        overdue = [i for i in cold if now - queue[i].t_arrival >= self.cold_wait]
        return overdue + warm + [i for i in cold if i not in overdue]

    def _start_load(self, c, queue):
        """Move c's state to the device on the loader thread; its queued requests wait
        until the scheduler thread has seen the load finish (_poll_load)."""
        c.resident = True         # counts against the budget from now on
        c.inflight += 1           # not evictable while it loads
        for r in queue:
            if r.client is c:
                r.cold = True
        box = {}

        def work():
            t0 = time.perf_counter()
            try:
                if self.copy_stream is not None:
                    with torch.cuda.stream(self.copy_stream):
                        c.restore()
                else:
                    c.restore()
            except Exception as e:   # reported by the scheduler thread
                box["error"] = e
            box["seconds"] = time.perf_counter() - t0
        th = threading.Thread(target=work, daemon=True)
        self.loading = (c, th, box)
        th.start()

    def _poll_load(self):
        if self.loading is None or self.loading[1].is_alive():
            return
        c, th, box = self.loading
        th.join()
        self.loading = None
        if "error" in box:
            raise box["error"]
        c.hold = True             # stays unevictable until one of its requests is admitted
        self.stats["cold_load_s"] += box["seconds"]
        self.stats["cold_loads"] += 1

    def _admit(self, lane, queue, now):
        for i in self._order(queue, now):
            req = queue[i]
            c = req.client
            if self.loading is not None and self.loading[0] is c:   # its state is still loading
                continue
            if not c.resident and self.async_loads:
                if self.loading is None and (self.resident_bytes() + c.nbytes <= self.budget
                                             or self._make_room(c.nbytes, c, queue)):
                    self._start_load(c, queue)
                continue
            ws = self.working_set(req, lane)
            need = ws + (0 if c.resident else c.nbytes)
            if self.resident_bytes() + need > self.budget and not self._make_room(need, c, queue):
                continue
            cold = not c.resident
            if cold:
                t0 = time.perf_counter()
                c.restore()
                self.stats["cold_load_s"] += time.perf_counter() - t0
                self.stats["cold_loads"] += 1
            group = [req]
            if self.merge and c.kind == "slot":
                used = {req.tag}
                for r2 in queue[i + 1:]:
                    if len(group) >= self.max_merge:
                        break
                    if r2.client is c and r2.tag not in used:
                        group.append(r2)
                        used.add(r2.tag)
            for r in group:
                queue.remove(r)
                r.t_admit = now
                r.cold = r.cold or cold
                r.merged = len(group)
            c.inflight += 1
            if c.hold:
                c.hold = False
                c.inflight -= 1
            c.last_used = now
            self._launch(lane, group, ws, self._now)
            return True
        return False

    def _launch(self, lane, group, ws, now_fn):
        c = group[0].client
        ctx = lane.ctx[c.set_name]

        def work():
            try:
                batch()
            except Exception as e:   # reported by the scheduler thread
                lane.error = e
            lane.finished = True

        def batch():
            with torch.cuda.stream(lane.stream):
                if len(group) == 1:
                    xs = group[0].payload
                else:   # slot merging: the requests' images occupy disjoint slots
                    xs = []
                    for k in range(len(group[0].payload)):
                        acc = ctx.add(group[0].payload[k], group[1].payload[k])
                        for r in group[2:]:
                            acc = ctx.add(acc, r.payload[k], out=acc)
                        xs.append(acc)
                if c.kind == "packed":
                    out = [c.net.forward(ctx, c.rlk, c.gks, [x], c.weights) for x in xs]
                else:
                    out = c.net.forward(ctx, c.rlk, c.gks, xs, c.weights)
                for r in group:   # the user decrypts (decode waits for the stream)
                    if c.kind == "packed":
                        parts, left = [], r.n
                        for z in out:
                            m = min(left, c.net.images_per_ct(ctx))
                            parts.append(c.net.decrypt_scores(ctx, c.sk, z, m))
                            left -= m
                        r.scores = np.concatenate(parts)
                    else:
                        r.scores = c.net.decrypt_scores(ctx, c.sk, out, r.n, r.off)
                    r.t_done = now_fn()

        lane.group, lane.ws, lane.finished, lane.error = group, ws, False, None
        lane.thread = threading.Thread(target=work, daemon=True)
        lane.thread.start()

    def _poll(self):
        done = 0
        for lane in self.lanes:
            if lane.group is None or not lane.finished:
                continue
            lane.thread.join()
            if lane.error is not None:
                raise lane.error
            held = self._library_bytes(lane)
            if held:
                kind = lane.group[0].client.kind
                self.library_peak[kind] = max(self.library_peak.get(kind, 0), held)
                if held > self.stats["library_peak_bytes"]:
                    self.stats["library_peak_bytes"] = held
                lane.release_buffers()
            lane.group[0].client.inflight -= 1
            done += len(lane.group)
            lane.group, lane.thread, lane.ws = None, None, 0
        return done

    def run(self, requests, time_limit=None, progress=None):
        """Serve `requests` (t_arrival in seconds from the start, sorted); returns them.
        progress(finished, total) is called whenever requests complete."""
        t0 = time.perf_counter()

        def now():
            return time.perf_counter() - t0
        self._now = now
        pending = collections.deque(sorted(requests, key=lambda r: r.t_arrival))
        queue, finished, total = [], 0, len(requests)
        while finished < total:
            t = now()
            if time_limit is not None and t > time_limit:
                raise TimeoutError("serving run exceeded its time limit")
            while pending and pending[0].t_arrival <= t:
                queue.append(pending.popleft())
            self._poll_load()
            done = self._poll()
            if done:
                finished += done
                if progress is not None:
                    progress(finished, total)
            busy = False
            for lane in self.lanes:
                if lane.group is None and queue and self._admit(lane, queue, now()):
                    busy = True
            if not busy:
                time.sleep(0.0002)
        if self.loading is not None:      # a load no queued request waits for any more
            self.loading[1].join()
            self._poll_load()
        for c in self.clients:            # nothing is queued any more: release the holds
            if c.hold:
                c.hold = False
                c.inflight -= 1
        return requests


def summarize(requests):
    lat = np.array([r.t_done - r.t_arrival for r in requests])
    wait = np.array([r.t_admit - r.t_arrival for r in requests])
    imgs = sum(r.n for r in requests)
    span = max(r.t_done for r in requests) - min(r.t_arrival for r in requests)
    return {"requests": len(requests), "images": imgs, "images_per_s": round(imgs / span, 2),
            "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
            "mean_admission_wait_ms": round(float(wait.mean()) * 1e3, 2),
            "cold_requests": sum(1 for r in requests if r.cold),
            "mean_merge": round(float(np.mean([r.merged for r in requests])), 2)}
