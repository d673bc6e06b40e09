"""Continuous-batching render server over the HIP library.

Hair assets and their nested LoD hierarchies stay resident in HBM.  Requests (asset,
resolution, view) arrive as they come (Poisson arrivals in the benchmark), wait in a FIFO, and
are admitted when a slot is free and the request's memory footprint fits the scratch budget
next to the memory the other slots really hold.  Each slot owns a HIP stream, a library workspace, a
level buffer and an output buffer, and runs the LoD choice and the frame on its stream; slots
overlap on the device.  LoD (lod="mixed", the default): per group of the coarsest level and per
segment index, the coarsest level whose thick hairs are at most eps_w = 2 px wide (Sec. 5.1
step 5, Sec. 6), rendered as one mixed-level frame (or as that level's own frame when one
level is chosen everywhere); lod="level": one level for the whole asset.  With shadow =
(resolution, layers, layer_depth) every frame gets deep opacity map shadows (mixed frames
over their own rows).
A request's latency is its completion time minus its arrival time.

Memory: the budget is charged with what the workspaces really hold on the device.  A request
is admitted to a free slot when the slot's reservation, max(its workspace's bytes, the
request's estimated footprint), fits beside the busy slots' reservations and the idle slots'
held bytes; the slot's workspace is then limited to that reservation, so no frame can grow
past the budget.  A frame that needs more than its estimate fails in the library with
HAIR_ENOMEM (nothing allocated) and goes back to the head of the queue with twice the
estimate (at most the budget), to wait for memory.  When the head request fits nowhere, idle
slots give their workspace memory back (hair_ws_trim).

    python -m paper_2405_10565_amd.serve [--rates 30 60 120] [--requests 3000] [--warmup 200]
"""
from __future__ import annotations

import argparse
import json
import math
import threading
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import binding as B

RESOLUTIONS = ((1280, 720), (1920, 1080), (3840, 2160))


@dataclass
class Request:
    rid: int
    asset: str
    width: int
    height: int
    azimuth: float
    occupancy: float
    arrival: float = 0.0
    start: float = 0.0
    done: float = 0.0
    level: int = -1
    level_hist: list = None     # mixed LoD: (group, segment) entries per level
    fragments: int = 0
    footprint: int = 0
    status: int = 0
    slot: int = -1
    output: object = None
    levels_used: object = None  # with keep_outputs, mixed LoD: the (group, segment) level map
    retries: int = 0            # re-queued after outgrowing its estimate


@dataclass
class ServedAsset:
    aid: int
    asset: object              # the host-side description (for framing the camera)
    lights: list
    segments_per_level: list   # segments of level 0..n
    groups: int = 0            # groups of the nested hierarchy (0: none)
    assigns: list = None       # cluster assignments of levels 1..n (finer -> coarser)


class Slot:
    def __init__(self, server: "Server", idx: int, max_pixels: int):
        import torch
        self.idx = idx
        self.stream = torch.cuda.Stream(device=server.hctx.device)
        self.ws = server.hctx.workspace()
        self.out = torch.empty(max_pixels * 4, dtype=torch.float32, device=f"cuda:{server.hctx.device}")
        gs = max([a.groups * a.asset.segs for a in server.assets.values()] + [1])
        self.levels = torch.zeros(gs, dtype=torch.int32, device=f"cuda:{server.hctx.device}")
        self.busy = False
        self.held = 0          # bytes the workspace holds (read after each frame)
        self.reserve = 0       # while busy: the workspace's limit for the running request


class Server:
    """FIFO admission by footprint; n_slots requests in flight at most."""

    def __init__(self, hctx: B.Context, assets: dict, n_slots: int = 4, scratch_budget: int = 32 << 30,
                 eps_w: float = 2.0, keep_outputs: bool = False, lod: str = "mixed", shadow=None):
        self.hctx = hctx
        self.assets = assets
        self.lod = lod
        self.shadow = shadow          # (resolution, layers, layer_depth): deep opacity map shadows
        self.scratch_budget = int(scratch_budget)
        self.eps_w = eps_w
        self.keep_outputs = keep_outputs
        max_pixels = max(w * h for w, h in RESOLUTIONS)
        self.slots = [Slot(self, i, max_pixels) for i in range(n_slots)]
        self.free_slots = deque(self.slots)
        self.queue: deque[Request] = deque()
        self.in_flight_bytes = 0          # charged bytes: busy reservations + idle workspaces
        self.peak_bytes = 0
        self.cv = threading.Condition()
        self.done: list[Request] = []
        self.rejected: list[Request] = []
        self.t0 = time.perf_counter()
        self.running = True
        self.peak_in_flight = 0
        self.workers = [threading.Thread(target=self._worker, daemon=True) for _ in range(n_slots)]
        for w in self.workers:
            w.start()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def prewarm(self):
        """Render the largest request class (largest asset, largest resolution, nearest view)
        once on every slot, so that each slot's workspace keeps buffer capacities for the
        request mix and served frames are not rendered a second time to grow them."""
        import torch
        import hairsynth as hs
        name = max(self.assets, key=lambda n: self.assets[n].segments_per_level[0])
        a = self.assets[name]
        w, h = max(RESOLUTIONS, key=lambda r: r[0] * r[1])
        cam = hs.camera_occupancy(a.asset, w, h, 0.6, 0.0)
        with self.cv:
            for slot in self.slots:
                out = slot.out[: w * h * 4].view(h, w, 4)
                slot.ws.set_limit(max(1, self.scratch_budget - self._charged(slot)))
                _, _, rc = self.hctx.render(a.aid, 0, cam, a.lights, out=out, ws=slot.ws, stream=slot.stream,
                                            raise_on_error=False)
                if rc != B.HAIR_OK:        # the budget holds fewer warm slots: keep the rest cold
                    slot.ws.trim()
                slot.held = slot.ws.memory()[0]
            self.in_flight_bytes = self._charged(None)
        torch.cuda.synchronize()

    def footprint(self, req: Request) -> int:
        """Scratch bytes a request may need: workspace upper estimate at the finest level plus
        its output image."""
        a = self.assets[req.asset]
        return int(B.ws_estimate(a.segments_per_level[0], req.width, req.height, 0)) + 16 * req.width * req.height

    def submit(self, req: Request):
        req.footprint = self.footprint(req)
        req.arrival = self.now()
        with self.cv:
            if req.footprint > self.scratch_budget:
                req.status = B.HAIR_ENOMEM
                self.rejected.append(req)
                return
            self.queue.append(req)
            self.cv.notify_all()

    def _charged(self, skip) -> int:
        """Bytes charged to the budget by every slot but `skip`: a busy slot its reservation,
        an idle one what its workspace holds."""
        return sum(s.reserve if s.busy else s.held for s in self.slots if s is not skip)

    def _take(self):
        """(request, slot): the first queued request (FIFO order) that fits on a free slot
        beside the memory the other slots hold; idle slots give their memory back when the
        head request fits nowhere."""
        for attempt in range(2):
            for i, r in enumerate(self.queue):
                for slot in sorted(self.free_slots, key=lambda s: -s.held):
                    if self._charged(slot) + max(slot.held, r.footprint) <= self.scratch_budget:
                        del self.queue[i]
                        self.free_slots.remove(slot)
                        return r, slot
            idle = [s for s in self.free_slots if s.held]
            busy = sum(s.reserve for s in self.slots if s.busy)
            if attempt or not self.queue or not idle or busy + self.queue[0].footprint > self.scratch_budget:
                break
            for s in idle:     # the head request fits once the idle workspaces are emptied
                s.ws.trim()
                s.held = s.ws.memory()[0]
        return None

    def _worker(self):
        while True:
            with self.cv:
                while self.running and (not self.free_slots or not self.queue or (got := self._take()) is None):
                    self.cv.wait()
                if not self.running:
                    return
                req, slot = got
                slot.busy = True
                slot.reserve = max(slot.held, req.footprint)
                slot.ws.set_limit(slot.reserve)
                self.in_flight_bytes = self._charged(None)
                self.peak_bytes = max(self.peak_bytes, self.in_flight_bytes)
                self.peak_in_flight = max(self.peak_in_flight, sum(s.busy for s in self.slots))
            self._run(slot, req)
            with self.cv:
                slot.held = slot.ws.memory()[0]
                slot.busy = False
                slot.reserve = 0
                self.free_slots.append(slot)
                if req.status == B.HAIR_ENOMEM and req.footprint < self.scratch_budget:
                    # outgrew its estimate: wait at the head of the queue with a larger one
                    req.retries += 1
                    req.footprint = min(self.scratch_budget, 2 * max(req.footprint, slot.held))
                    req.status = 0
                    self.queue.appendleft(req)
                else:
                    self.done.append(req)
                self.in_flight_bytes = self._charged(None)
                self.cv.notify_all()

    def _run(self, slot: Slot, req: Request):
        import hairsynth as hs
        a = self.assets[req.asset]
        cam = hs.camera_occupancy(a.asset, req.width, req.height, req.occupancy, req.azimuth)
        req.start = self.now()
        req.slot = slot.idx
        try:
            out = slot.out[: req.width * req.height * 4].view(req.height, req.width, 4)
            if self.lod == "mixed" and a.groups:
                lev = slot.levels[: a.groups * a.asset.segs].view(a.groups, a.asset.segs)
                self.hctx.lod_init(a.aid, cam, self.eps_w, lev, ws=slot.ws, stream=slot.stream)
                lev_host = lev.cpu().numpy()
                if self.keep_outputs:
                    req.levels_used = lev_host.copy()
                hist = np.bincount(lev_host.reshape(-1), minlength=len(a.segments_per_level))
                req.level_hist = hist.tolist()
                req.level = int(np.argmax(hist))
                if hist[req.level] == hist.sum():   # one level everywhere: that level's own frame
                    _, st, rc = self._level_frame(a, req.level, cam, out, slot)
                elif self.shadow is not None:
                    _, st, rc = self.hctx.render_mixed_shadowed(a.aid, cam, a.lights, lev, self.shadow, 0.0, out=out,
                                                                ws=slot.ws, stream=slot.stream, raise_on_error=False)
                else:
                    _, st, rc = self.hctx.render_mixed(a.aid, cam, a.lights, lev, 0.0, out=out, ws=slot.ws,
                                                       stream=slot.stream, raise_on_error=False)
            else:
                req.level = self.hctx.select_level(a.aid, cam, self.eps_w, ws=slot.ws, stream=slot.stream)
                _, st, rc = self._level_frame(a, req.level, cam, out, slot)
            req.status = rc
            req.fragments = int(st["fragments"])
            if self.keep_outputs:
                import torch
                with torch.cuda.stream(slot.stream):   # ordered after the frame on the slot's stream
                    req.output = out.clone()
                slot.stream.synchronize()
        except B.HairError as e:
            req.status = e.code
        req.done = self.now()

    def _level_frame(self, a, level, cam, out, slot):
        if self.shadow is not None:
            return self.hctx.render_shadowed(a.aid, level, cam, a.lights, self.shadow, out=out, ws=slot.ws,
                                             stream=slot.stream, raise_on_error=False)
        return self.hctx.render(a.aid, level, cam, a.lights, out=out, ws=slot.ws, stream=slot.stream,
                                raise_on_error=False)

    def drain(self, timeout: float = 600.0):
        end = time.perf_counter() + timeout
        with self.cv:
            while (self.queue or len(self.free_slots) < len(self.slots)) and time.perf_counter() < end:
                self.cv.wait(timeout=0.05)

    def close(self):
        self.drain()
        with self.cv:
            self.running = False
            self.cv.notify_all()
        for w in self.workers:
            w.join(timeout=10)
        for s in self.slots:
            s.ws.close()


def make_requests(names, n: int, seed: int, resolutions=RESOLUTIONS, occupancy=(0.02, 0.6)):
    """Seeded request mix: asset uniform, resolution uniform, azimuth uniform, screen
    occupancy log-uniform (the paper's far ... near views, Sec. 6)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lo, hi = math.log(occupancy[0]), math.log(occupancy[1])
    reqs = []
    for i in range(n):
        w, h = resolutions[int(rng.integers(len(resolutions)))]
        reqs.append(Request(i, names[int(rng.integers(len(names)))], w, h, float(rng.uniform(0, 2 * math.pi)),
                            float(math.exp(rng.uniform(lo, hi)))))
    return reqs


def run_poisson(server: Server, reqs, rate: float, seed: int, warmup: int = 0):
    """Submit requests with exponential inter-arrival times; returns the measured ones."""
    rng = np.random.Generator(np.random.PCG64(seed + 7))
    t_next = time.perf_counter()
    for r in reqs:
        t_next += float(rng.exponential(1.0 / rate))
        delay = t_next - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        server.submit(r)
    server.drain()
    return [r for r in reqs if r.rid >= warmup]


def summarize(reqs, rate: float):
    ok = [r for r in reqs if r.status == B.HAIR_OK and r.done > 0]
    lat = np.array([(r.done - r.arrival) * 1e3 for r in ok])
    if not len(ok):
        return {"rate": rate, "completed": 0}
    span = max(r.done for r in ok) - min(r.arrival for r in ok)
    frags = sum(r.fragments for r in ok)
    hists = [r.level_hist for r in ok if r.level_hist is not None]
    if hists:   # mixed LoD: share of (group, segment) entries per level over all requests
        n = max(len(h) for h in hists)
        tot = np.zeros(n)
        for h in hists:
            tot[: len(h)] += h
        levels = [round(float(v), 4) for v in tot / tot.sum()]
    else:
        levels = np.bincount([r.level for r in ok]).tolist()
    return {"rate_req_s": rate, "completed": len(ok), "failed": len(reqs) - len(ok),
            "latency_ms_p50": round(float(np.percentile(lat, 50)), 3),
            "latency_ms_p99": round(float(np.percentile(lat, 99)), 3),
            "latency_ms_mean": round(float(lat.mean()), 3),
            "throughput_req_s": round(len(ok) / span, 2) if span > 0 else None,
            "mfragments_s": round(frags / span / 1e6, 2) if span > 0 else None,
            "levels": levels}


def build_assets(hctx: B.Context, specs=((10_000, 16), (100_000, 32), (300_000, 48)), seed: int = 1005,
                 level_divisors=(16, 256, 4096)) -> dict:
    """Upload the serving assets and build their nested thick-hair levels (resident in HBM)."""
    import hairsynth as hs
    out = {}
    for i, (n, segs) in enumerate(specs):
        asset = hs.make_asset(n, segs, 90.0, seed=seed + i, sigma_spread=True)
        aid = hctx.upload_asset(asset)
        ks = [max(1, n // d) for d in level_divisors]
        assigns = hs.kmeans_hierarchy(asset, ks, seed=seed + i, iters=10, init="random")
        hctx.build_lod(aid, assigns)
        _, counts, S = hctx.lod_info(aid)
        out[f"{n / 1000:g}k x {segs}"] = ServedAsset(aid, asset, hs.default_lights(asset, with_point=True),
                                                      [c * S for c in counts], hctx.lod_groups(aid), assigns)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--rates", type=float, nargs="+", default=[30.0, 60.0, 120.0])
    ap.add_argument("--requests", type=int, default=3000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--budget-gib", type=float, default=32.0)
    ap.add_argument("--lod", choices=["mixed", "level"], default="mixed")
    args = ap.parse_args()
    import torch
    assert torch.cuda.is_available()
    hctx = B.Context(0)
    assets = build_assets(hctx)
    for rate in args.rates:
        srv = Server(hctx, assets, n_slots=args.slots, scratch_budget=int(args.budget_gib * (1 << 30)), lod=args.lod)
        srv.prewarm()
        reqs = make_requests(sorted(assets), args.requests + args.warmup, seed=int(rate))
        res = summarize(run_poisson(srv, reqs, rate, seed=int(rate), warmup=args.warmup), rate)
        res["peak_in_flight"] = srv.peak_in_flight
        srv.close()
        print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
