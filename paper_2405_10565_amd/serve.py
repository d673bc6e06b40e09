"""Continuous-batching render server over the HIP library.

Hair assets and their nested LoD hierarchies stay resident in HBM.  Requests (asset,
resolution, view) arrive as they come (Poisson arrivals in the benchmark), wait in a FIFO, and
are admitted when a slot is free and the request's memory footprint fits the scratch budget
next to the requests already on the GPU.  Each slot owns a HIP stream, a library workspace, a
level buffer and an output buffer, and runs the LoD choice and the frame on its stream; slots
overlap on the device.  LoD (lod="mixed", the default): per group of the coarsest level and per
segment index, the coarsest level whose thick hairs are at most eps_w = 2 px wide (Sec. 5.1
step 5, Sec. 6), rendered as one mixed-level frame (or as that level's own frame when one
level is chosen everywhere); lod="level": one level for the whole asset.
A request's latency is its completion time minus its arrival time.

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


@dataclass
class ServedAsset:
    aid: int
    asset: object              # the host-side description (for framing the camera)
    lights: list
    segments_per_level: list   # segments of level 0..n
    groups: int = 0            # groups of the nested hierarchy (0: none)


class Slot:
    def __init__(self, server: "Server", idx: int, max_pixels: int):
        import torch
        self.idx = idx
        self.stream = torch.cuda.Stream(device=server.hctx.device)
        self.ws = server.hctx.workspace()
        self.out = torch.empty(max_pixels * 4, dtype=torch.float32, device=f"cuda:{server.hctx.device}")
        gs = max([a.groups * a.asset.segs for a in server.assets.values()] + [1])
        self.levels = torch.zeros(gs, dtype=torch.int32, device=f"cuda:{server.hctx.device}")


class Server:
    """FIFO admission by footprint; n_slots requests in flight at most."""

    def __init__(self, hctx: B.Context, assets: dict, n_slots: int = 4, scratch_budget: int = 32 << 30,
                 eps_w: float = 2.0, keep_outputs: bool = False, lod: str = "mixed"):
        self.hctx = hctx
        self.assets = assets
        self.lod = lod
        self.scratch_budget = int(scratch_budget)
        self.eps_w = eps_w
        self.keep_outputs = keep_outputs
        max_pixels = max(w * h for w, h in RESOLUTIONS)
        self.slots = [Slot(self, i, max_pixels) for i in range(n_slots)]
        self.free_slots = deque(self.slots)
        self.queue: deque[Request] = deque()
        self.in_flight_bytes = 0
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
        for slot in self.slots:
            out = slot.out[: w * h * 4].view(h, w, 4)
            self.hctx.render(a.aid, 0, cam, a.lights, out=out, ws=slot.ws, stream=slot.stream)
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

    def _take(self):
        """First queued request (FIFO order) whose footprint fits next to the in-flight ones."""
        for i, r in enumerate(self.queue):
            if self.in_flight_bytes + r.footprint <= self.scratch_budget:
                del self.queue[i]
                return r
        return None

    def _worker(self):
        while True:
            with self.cv:
                while self.running and (not self.free_slots or not self.queue or (req := self._take()) is None):
                    self.cv.wait()
                if not self.running:
                    return
                slot = self.free_slots.popleft()
                self.in_flight_bytes += req.footprint
                self.peak_in_flight = max(self.peak_in_flight, len(self.slots) - len(self.free_slots))
            self._run(slot, req)
            with self.cv:
                self.in_flight_bytes -= req.footprint
                self.free_slots.append(slot)
                self.done.append(req)
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
                hist = np.bincount(lev.flatten().cpu().numpy(), minlength=len(a.segments_per_level))
                req.level_hist = hist.tolist()
                req.level = int(np.argmax(hist))
                if hist[req.level] == hist.sum():   # one level everywhere: that level's own frame
                    _, st, rc = self.hctx.render(a.aid, req.level, cam, a.lights, out=out, ws=slot.ws,
                                                 stream=slot.stream, raise_on_error=False)
                else:
                    _, st, rc = self.hctx.render_mixed(a.aid, cam, a.lights, lev, 0.0, out=out, ws=slot.ws,
                                                       stream=slot.stream, raise_on_error=False)
            else:
                req.level = self.hctx.select_level(a.aid, cam, self.eps_w, ws=slot.ws, stream=slot.stream)
                _, st, rc = self.hctx.render(a.aid, req.level, cam, a.lights, out=out, ws=slot.ws,
                                             stream=slot.stream, raise_on_error=False)
            req.status = rc
            req.fragments = int(st["fragments"])
            if self.keep_outputs:
                req.output = out.clone()
                slot.stream.synchronize()
        except B.HairError as e:
            req.status = e.code
        req.done = self.now()

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
        hctx.build_lod(aid, hs.kmeans_hierarchy(asset, ks, seed=seed + i, iters=10, init="random"))
        _, counts, S = hctx.lod_info(aid)
        out[f"{n // 1000}k x {segs}"] = ServedAsset(aid, asset, hs.default_lights(asset, with_point=True),
                                                     [c * S for c in counts], hctx.lod_groups(aid))
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
