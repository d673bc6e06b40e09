"""Benchmark: strand-hair frames through the HIP library on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload: 100,000 strands x 32 segments (3.2 M segments, seeded synthetic generator), one
directional and one point light, 1920 x 1080, strand level.  A step is one request through
the hot path: projection, tile binning, coverage, per-pixel sort, shading and compositing;
inputs are resident in HBM before the timed region.  The asset has only its strand level, so
the per-request level choice in the step returns level 0 without device work (level choice on
assets with thick-hair levels is timed in the serving leg, where it is part of each served
request's latency).  Steps are
pipelined over two workspaces: step k enqueues its frame without waiting (hair_render_async)
and then finishes and checks frame k - 1 (hair_ws_finish), so the GPU does not idle on the
host between frames; every frame is complete and checked inside the timed region.

Prints one JSON line: Mfragments/s over the timed steps (fragments counted by the library,
equal to the CPU oracle's count), frame ms (mean, p50, p99), the roofline of the dominant
kernel (k_batch, measured with HIP events on its launch stream), the CPU oracle timed on
a bounded sample of the same frame, and the served latency (p50 / p99, arrival to
completion) of the continuous-batching render server under Poisson arrivals of 30, 60 and
120 requests/s over three resident assets (10k x 16, 100k x 32 and 300k x 48 strands with
their thick-hair levels; resolution uniform over 720p / 1080p / 2160p).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "hair-100k-strands-32seg-1920x1080-2lights"
METRIC = "Mfragments/s + frame ms (100k strands, 1080p); served p50/p99 latency"

# Algorithmic operations per fragment of the shading kernel k_batch, counted by running the
# oracle's per-fragment definition under an operation counter (tests/golden/count_ops.py ->
# tests/golden/ops_per_fragment.json): alpha and h, world point, frame, each light, blend, and
# ceil(log2 k) compares of the per-pixel sort; operations on values every fragment shares are
# not counted.  Unit: an FP32 lane-operation.  An add, multiply, compare, select or divide is
# one (the definition does not fuse, so a multiply-add counts two); exp, log, sqrt, sin, cos,
# asin, atan2 are one transcendental each, weighted 4 (quarter-rate issue).  Peak: MI355X's
# published FP32 vector rate, 157.3 TFLOP/s = 256 CUs x 128 FP32 lanes x 2.4 GHz x 2 (FMA), i.e.
# 78.6 T lane-operations per second.  (Measured on the device with --rate-probe: unpacked
# v_fma_f32 issues at ~56 T/s, v_exp/v_rcp/v_sqrt at ~18 T/s.)  A kernel that fuses
# multiply-adds issues fewer lane-operations than counted, so the fraction credits fusion.
OPS_FILE = os.path.join(ROOT, "tests", "golden", "ops_per_fragment.json")
TRANS_WEIGHT = 4                                # transcendental unit issues at 1/4 rate
PEAK_LANE_OPS = 256 * 128 * 2.4e9               # 256 CUs x 128 FP32 lanes x 2.4 GHz = 157.3 TFLOP/s / 2
PEAK_HBM = 8.0e12

KERNEL_SOURCES = ["paper_2405_10565_amd/csrc/hair_kernels.hip", "paper_2405_10565_amd/csrc/hair_shading.h",
                  "paper_2405_10565_amd/csrc/hair_internal.h", "paper_2405_10565_amd/csrc/hair_fastmath_coef.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_batch_hair_100k_1080p_traffic.txt")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic():
    """HBM bytes per k_batch launch from the committed counter summary, if it was measured on
    the current kernel sources (else None)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_hash") != kernel_hash():
        return None
    try:
        return float(vals["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def ops_per_fragment(kind: str, lights):
    """(ops, transcendentals) per fragment of k_batch for `kind` ("strand_100k_1080p",
    "thick_1080p" or "strand_shadowed_100k_1080p") and the lights' kinds, from the oracle's
    counted definition (a shadowed frame adds its deep opacity map lookup)."""
    with open(OPS_FILE) as f:
        c = json.load(f)[kind]
    per = {0: next(v for k, v in c.items() if k.endswith("kind0")), 1: next(v for k, v in c.items() if k.endswith("kind1"))}
    look = c.get("lookup", (0.0, 0.0))
    ops = c["base"][0] + c["blend"][0] + c["sort_compares"] + look[0] + sum(per[l.kind][0] for l in lights)
    trans = c["base"][1] + c["blend"][1] + look[1] + sum(per[l.kind][1] for l in lights)
    return ops, trans


def alg_ops(fragments: int, lights, kind: str = "strand_100k_1080p"):
    ops, trans = ops_per_fragment(kind, lights)
    return fragments * ops, fragments * trans


def roofline(fragments: int, lights, t_kernel_s: float, kind: str, kernel: str, traffic=None):
    opf, trf = ops_per_fragment(kind, lights)
    w = fragments * (opf + TRANS_WEIGHT * trf)
    achieved = w / t_kernel_s
    return {"bound": "alu", "achieved": round(achieved / 1e12, 3), "peak": round(PEAK_LANE_OPS / 1e12, 2),
            "unit": "Tops/s", "frac": round(achieved / PEAK_LANE_OPS, 4), "traffic": traffic, "kernel": kernel,
            "ops_per_launch": int(w), "ops_per_fragment": round(opf, 2), "trans_per_fragment": round(trf, 2),
            "trans_weight": TRANS_WEIGHT}


def cpu_baseline(asset, cam, lights, rows: int = 48):
    """The oracle, single-threaded, on a centre band of the frame."""
    import torch
    torch.set_num_threads(1)
    from oracle import render as R
    mat = tuple(float(v) for v in asset.material.as_array())
    y0 = cam.height // 2 - rows // 2
    t0 = time.perf_counter()
    _, ras = R.render(R.strand_level(asset), cam, lights, mat, rect=(0, y0, cam.width, rows))
    dt = time.perf_counter() - t0
    return {"value": round(len(ras.seg) / dt / 1e6, 5), "unit": "Mfragments/s", "cores": 1, "kind": "oracle",
            "sample": f"rows {y0}-{y0 + rows - 1} of the 1920x1080 frame ({len(ras.seg)} fragments, "
                      f"{dt:.1f} s wall, torch/numpy float64 on 1 thread)"}


def _oracle_band(y0: int, rows: int, t_start: float):
    """Worker of cpu_baseline_multicore: the oracle on rows [y0, y0 + rows) of the headline
    frame, single-threaded, starting at wall time t_start (after imports and set-up)."""
    import torch
    torch.set_num_threads(1)
    import hairsynth as hs
    from oracle import render as R
    asset, cam, lights = hs.config(2)
    geom = R.strand_level(asset)
    mat = tuple(float(v) for v in asset.material.as_array())
    while time.time() < t_start:
        time.sleep(0.01)
    t0 = time.time()
    _, ras = R.render(geom, cam, lights, mat, rect=(0, y0, cam.width, rows))
    print(json.dumps({"y0": y0, "fragments": int(len(ras.seg)), "t0": t0, "t1": time.time()}), flush=True)


def cpu_baseline_multicore(rows: int = 48, max_workers: int = 16):
    """The oracle on host cores in parallel: one single-threaded process per band of `rows`
    rows around the frame's centre (as many bands as workers), all starting together; the
    rate is their fragments over the wall time from the common start to the last finish."""
    import subprocess
    n = max(1, min(max_workers, len(os.sched_getaffinity(0))))
    H = 1080
    y_first = H // 2 - (n * rows) // 2
    t_start = time.time() + 30.0 + 2.0 * n        # room for every worker's imports and set-up
    procs = [subprocess.Popen([sys.executable, "-c",
                               f"import sys; sys.path.insert(0, {ROOT!r}); import bench; "
                               f"bench._oracle_band({y_first + i * rows}, {rows}, {t_start})"],
                              stdout=subprocess.PIPE, text=True, cwd=ROOT) for i in range(n)]
    outs = []
    for p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            raise RuntimeError(f"oracle worker failed with status {p.returncode}")
        outs.append(json.loads(out.strip().splitlines()[-1]))
    frags = sum(o["fragments"] for o in outs)
    wall = max(o["t1"] for o in outs) - min(o["t0"] for o in outs)
    return {"value": round(frags / wall / 1e6, 5), "unit": "Mfragments/s", "cores": n, "kind": "oracle",
            "sample": f"rows {y_first}-{y_first + n * rows - 1} of the 1920x1080 frame in {n} bands of {rows} rows, one "
                      f"single-threaded oracle process per band ({frags} fragments, {wall:.1f} s wall from the "
                      f"common start to the last finish)"}


def rttd_frame(ctx, asset, cam, lights, ws, frames: int = 20):
    """The same strand frame with the R / TT / D material (outside the timed region)."""
    import dataclasses
    import numpy as np
    import hairsynth as hs
    aid = ctx.upload_asset(dataclasses.replace(asset, material=hs.Material.rttd()))
    ms = []
    for i in range(frames + 2):
        _, st, _ = ctx.render(aid, 0, cam, lights, ws=ws)
        if i >= 2:
            ms.append(st["ms_total"])
    ctx.release(aid)
    return {"gpu_mean": round(float(np.mean(ms)), 4), "gpu_p50": round(float(np.percentile(ms, 50)), 4),
            "fragments": int(st["fragments"]), "material": "R/TT/D (beta_R 0.1, beta_TT 0.2, gamma_TT 0.3)"}


def thick_frame(ctx, ws, clusters: int = 1000, frames: int = 20):
    """A thick-hair frame of the level sweep (150k strands x 64 segments, seeded k-means to 1k
    thick hairs, 1920 x 1080, directional + point light) with the roofline of its shading
    kernel k_batch<1, 0, false> (outside the timed region)."""
    import numpy as np
    import hairsynth as hs
    t0 = time.perf_counter()
    asset, cam, lights = hs.config(3)
    aid = ctx.upload_asset(asset)
    ctx.build_lod(aid, [hs.kmeans_assign(asset, clusters, seed=1003)])
    ms, tile = [], []
    for i in range(frames + 2):
        _, st, _ = ctx.render(aid, 1, cam, lights, ws=ws)
        if i >= 2:
            ms.append(st["ms_total"])
            tile.append(st["ms_tile"])
    ctx.release(aid)
    t = float(np.mean(tile)) * 1e-3
    print(f"bench: thick-hair frame measured ({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    return {"workload": f"hair-150k-strands-64seg-{clusters}-thick-hairs-1920x1080-2lights",
            "gpu_mean": round(float(np.mean(ms)), 4), "gpu_p50": round(float(np.percentile(ms, 50)), 4),
            "fragments": int(st["fragments"]), "k_batch_ms": round(t * 1e3, 4),
            "roofline": roofline(int(st["fragments"]), lights, t, "thick_1080p", "k_batch<1, 0, false>")}


def shadowed_frame(ctx, aid, cam, lights, ws, shadow=(1024, 4, 0.02), frames: int = 20):
    """The same strand frame with deep opacity map shadows for the directional light
    (outside the timed region; ms includes the shadow pass), with the roofline of its camera
    shading kernel k_batch<0, 0, true>."""
    import numpy as np
    ms, tile = [], []
    for i in range(frames + 2):
        _, st, _ = ctx.render_shadowed(aid, 0, cam, lights, shadow, ws=ws)
        if i >= 2:
            ms.append(st["ms_total"])
            tile.append(st["ms_tile"])
    t = float(np.mean(tile)) * 1e-3
    return {"gpu_mean": round(float(np.mean(ms)), 4), "gpu_p50": round(float(np.percentile(ms, 50)), 4),
            "resolution": shadow[0], "layers": shadow[1], "layer_depth": shadow[2], "k_batch_ms": round(t * 1e3, 4),
            "roofline": roofline(int(st["fragments"]), lights, t, "strand_shadowed_100k_1080p", "k_batch<0, 0, true>")}


def serve_leg(ctx, n_requests: int, warmup: int, rates=(30.0, 60.0, 120.0)):
    """Served latency: Poisson arrivals at each rate over the three resident serving assets
    (a progress line per rate goes to stderr)."""
    from paper_2405_10565_amd import serve as S
    t0 = time.perf_counter()
    assets = S.build_assets(ctx)
    print(f"bench: serving assets built in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    out = {"rates_req_s": list(rates), "requests_per_rate": n_requests, "warmup_per_rate": warmup,
           "slots": 4, "scratch_budget_gib": 32, "lod": "mixed per group and segment, eps_w 2 px",
           "p50_ms": [], "p99_ms": [], "throughput_req_s": [],
           "mfragments_s": [], "failed": [], "retried": [], "peak_gib": [], "levels": []}
    for rate in rates:
        srv = S.Server(ctx, assets, n_slots=4, scratch_budget=32 << 30)
        srv.prewarm()
        reqs = S.make_requests(sorted(assets), n_requests + warmup, seed=int(rate))
        r = S.summarize(S.run_poisson(srv, reqs, rate, seed=int(rate), warmup=warmup), rate)
        srv.close()
        out["p50_ms"].append(r.get("latency_ms_p50"))
        out["p99_ms"].append(r.get("latency_ms_p99"))
        out["throughput_req_s"].append(r.get("throughput_req_s"))
        out["mfragments_s"].append(r.get("mfragments_s"))
        out["failed"].append(r.get("failed"))
        out["retried"].append(sum(1 for q in reqs if q.retries))
        out["peak_gib"].append(round(srv.peak_bytes / (1 << 30), 3))
        out["levels"].append(r.get("levels"))
        print(f"bench: {rate:g} req/s served: p50 {r.get('latency_ms_p50')} ms, p99 {r.get('latency_ms_p99')} ms "
              f"({time.perf_counter() - t0:.0f} s)", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the served-latency leg")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the R/TT/D and shadowed frames reported beside the main frame")
    ap.add_argument("--serve-requests", type=int, default=3000, help="measured requests per arrival rate")
    ap.add_argument("--serve-warmup", type=int, default=200, help="unmeasured requests before them, per rate")
    ap.add_argument("--rate-probe", action="store_true",
                    help="only measure the device's issue rates of fma, exp, rcp, sqrt and integer multiplies")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy 5 times (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": src.numel() * 4, "launches": 5}))
        return
    if args.rate_probe:
        from paper_2405_10565_amd import binding as B
        ctx = B.Context(0)
        names = ["v_fma_f32", "v_exp_f32", "v_rcp_f32", "v_sqrt_f32", "v_mul_lo_u32", "v_mul_u32_u24"]
        rates = {n: round(ctx.issue_rate(k, 8192) / 1e12, 3) for k, n in enumerate(names)}
        ctx.close()
        print(json.dumps({"issue_rate_tops": rates, "peak_lane_ops_tops": round(PEAK_LANE_OPS / 1e12, 2)}))
        return
    if args.gpus != 1:
        print(f"bench.py: the renderer runs on one GPU; --gpus {args.gpus} is not supported "
              "(the renderer's multi-GPU split is a design note only)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import hairsynth as hs
    from paper_2405_10565_amd import binding as B

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    asset, cam, lights = hs.config(2)
    ctx = B.Context(0)
    aid = ctx.upload_asset(asset)
    # two workspaces and outputs: step k enqueues its frame (hair_render_async) and then
    # finishes and checks frame k - 1, so the stream never waits for the host between frames
    wss = [ctx.workspace(), ctx.workspace()]
    ws = wss[0]
    outs = [torch.empty((cam.height, cam.width, 4), dtype=torch.float32, device="cuda:0") for _ in wss]
    stream = torch.cuda.current_stream()

    def run(n):
        frames = []
        for k in range(n):
            w = wss[k % 2]
            level = ctx.select_level(aid, cam, 2.0, ws=w, stream=stream)
            ctx.render_async(aid, level, cam, lights, outs[k % 2], w, stream=stream)
            if k >= 1:
                frames.append(wss[(k - 1) % 2].finish()[0])
        if n:
            frames.append(wss[(n - 1) % 2].finish()[0])
        return frames

    run(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    frames = run(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    frags = sum(f["fragments"] for f in frames)
    ms_frame = np.array([f["ms_total"] for f in frames])
    ms_tile = np.array([f["ms_tile"] for f in frames])
    f1 = frames[0]["fragments"]
    t_tile = float(ms_tile.mean()) * 1e-3
    traffic = read_traffic()
    res = {
        "metric": METRIC,
        "value": round(frags / wall / 1e6, 3),
        "unit": "Mfragments/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded generator; paper grooms not available)",
        "config": {"workload": WORKLOAD, "strands": asset.n_strands, "segments": asset.n_segments,
                   "width": cam.width, "height": cam.height, "lights": len(lights), "level": 0,
                   "fragments_per_frame": f1, "pairs_per_frame": frames[0]["pairs"]},
        "frame_ms": {"gpu_mean": round(float(ms_frame.mean()), 4), "gpu_p50": round(float(np.percentile(ms_frame, 50)), 4),
                     "gpu_p99": round(float(np.percentile(ms_frame, 99)), 4),
                     "front": round(float(np.mean([f["ms_project"] for f in frames])), 4),
                     "tile": round(float(ms_tile.mean()), 4)},
        "roofline": roofline(f1, lights, t_tile, "strand_100k_1080p", "k_batch<0, 0, false>", traffic),
        "cpu_baseline": None,
    }
    if not args.no_extras:
        res["frame_ms_rttd"] = rttd_frame(ctx, asset, cam, lights, ws)
        res["frame_ms_shadowed"] = shadowed_frame(ctx, aid, cam, lights, ws)
        res["frame_ms_thick"] = thick_frame(ctx, ws)
    for w in wss:
        w.close()
    if not args.no_serve:
        res["serving"] = serve_leg(ctx, args.serve_requests, args.serve_warmup)
    ctx.close()
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(asset, cam, lights)
        print("bench: single-core oracle timed", file=sys.stderr, flush=True)
        res["cpu_baseline_multicore"] = cpu_baseline_multicore()
        print("bench: multi-core oracle timed", file=sys.stderr, flush=True)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
