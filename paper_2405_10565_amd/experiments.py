"""LoD experiments on the GPU library (JSON lines on stdout).

    python -m paper_2405_10565_amd.experiments lod-sweep [--scale S]
    python -m paper_2405_10565_amd.experiments fit [--iters N] [--scale S] [--locks]
    python -m paper_2405_10565_amd.experiments shadow [--iters N]
    python -m paper_2405_10565_amd.experiments curved [--scale S]
    python -m paper_2405_10565_amd.experiments views [--scale S]

lod-sweep: 150k strands x 64 segments at 1920 x 1080, clustered by k-means on root position
and first tangent into 10k, 1k and 100 thick hairs (Sec. 5.1); every level is rendered and
timed, and its RGB error against the strand render is reported (RMSE, PSNR with the strand
render's peak as signal).

fit: 50k strands x 32 segments reduced to 500 thick hairs, 8 views on a ring at 512 x 512,
one directional light; the thick hairs' semi-axes, radius and absorption are fitted by Adam
(log parameters, lr 1e-2) so the coarse render matches the strand render; the adjoint is
checked against central differences (h = 1e-3 in log space) on 20 random parameters.

curved: the LoD sweep's groom reduced to 1k thick hairs at 1080p, rendered with polyline
centre lines and with curved ones tessellated to at most 4, 2 and 1 px per step (Sec. 5.2,
Sec. 6); steps, fragments, frame ms and the RGB difference to the polyline frame.

views: 100k x 32 strands in locks of 16 following a smooth flow (then the random-walk groom of
the other workloads) with nested levels of 6250 / 1562 / 390 thick hairs (k-means on the
strands' paths), at the near, middle and far views of Sec. 6 (the bounding sphere covering
50%, 10% and 0.3% of a 1920 x 1080 image): the strand frame, the level chosen per request at
eps_w = 2 px and the per-group mixed-level frame; fragments, GPU ms and the RGB error against
the strand frame.

shadow: the 100k-strand 1080p frame with deep opacity map shadows (1024 x 1024 texels, 4
layers of 2 cm, Sec. 5.2) rendered N times after two warm-up frames; GPU ms per frame.
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import binding as B


def _rgb_error(img, ref):
    import torch
    d = (img[..., :3] - ref[..., :3]).double()
    mse = float((d * d).mean())
    peak = float(ref[..., :3].max())
    psnr = 10.0 * math.log10(peak * peak / mse) if mse > 0 else float("inf")
    return math.sqrt(mse), psnr


def lod_sweep(hctx: B.Context, scale: float = 1.0, repeats: int = 20):
    import torch
    import hairsynth as hs
    c = hs.CONFIGS[3]
    asset, cam, lights = hs.config(3, scale)
    t0 = time.perf_counter()
    assigns = [hs.kmeans_assign(asset, max(1, int(round(k * scale))), seed=1003) for k in c["levels"]]
    t_kmeans = time.perf_counter() - t0
    aid = hctx.upload_asset(asset)
    hctx.build_lod(aid, assigns)
    ws = hctx.workspace()
    n_levels, counts, S = hctx.lod_info(aid)
    out = {"experiment": "lod-sweep", "strands": asset.n_strands, "segments": asset.n_segments,
           "width": cam.width, "height": cam.height, "kmeans_s": round(t_kmeans, 2), "levels": []}
    ref = None
    for level in range(n_levels + 1):
        img, st, _ = hctx.render(aid, level, cam, lights, ws=ws)
        torch.cuda.synchronize()
        ms, tile = [], []
        for _ in range(repeats):
            _, s2, _ = hctx.render(aid, level, cam, lights, out=img, ws=ws)
            ms.append(s2["ms_total"])
            tile.append(s2["ms_tile"])
        img = img.clone()
        if level == 0:
            ref = img
        rmse, psnr = _rgb_error(img, ref)
        out["levels"].append({"level": level, "clusters": None if level == 0 else int(counts[level]),
                              "segments": int(st["segments"]), "fragments": int(st["fragments"]),
                              "frame_ms_p50": round(float(np.percentile(ms, 50)), 4),
                              "shading_ms_p50": round(float(np.percentile(tile, 50)), 4),
                              "rmse": round(rmse, 6), "psnr_db": round(psnr, 2)})
    ws.close()
    hctx.release(aid)
    return out


def fit_report(hctx: B.Context, iters: int = 200, scale: float = 1.0, n_fd: int = 20, seed: int = 4004,
               locks: bool = False):
    """locks: the groom in 500 locks following a smooth flow (one lock per thick hair, k-means
    on the strands' paths) instead of the random-walk groom."""
    import torch
    import hairsynth as hs
    from . import fit as F
    from .autograd import render_lod
    c = hs.CONFIGS[4]
    asset, _, lights = hs.config(4, scale)
    k = max(1, int(round(c["levels"][0] * scale)))
    if locks:
        asset = hs.make_asset(asset.n_strands, asset.segs, c["cap"], seed=1004, clumps=k, flow=0.99)
    cams = hs.ring_cameras(asset, c["views"], *c["res"])
    aid = hctx.upload_asset(asset)
    hctx.build_lod(aid, [hs.kmeans_assign(asset, k, seed=1004, features="path" if locks else "root")])
    ws = hctx.workspace()
    dev = torch.device(f"cuda:{hctx.device}")
    targets = F.strand_targets(hctx, aid, cams, lights, ws)
    lod0 = hctx.get_lod(aid, 1)
    base = [torch.tensor(lod0.axes, device=dev).log(), torch.tensor(lod0.r, device=dev).log(),
            torch.tensor(lod0.sigma_a, device=dev).clamp_min(1e-6).log()]

    n_seg = int(lod0.axes.shape[0] * lod0.axes.shape[1])

    def loss_and_radii(p):
        """Loss of log parameters p, and every view's integer coverage radii."""
        hctx.set_cluster_params(aid, 1, p[0].exp().contiguous(), p[1].exp().contiguous(), p[2].exp().contiguous())
        total, radii = 0.0, []
        for cam, tgt in zip(cams, targets):
            img, _, _ = hctx.render(aid, 1, cam, lights, ws=ws)
            total += float(((img[..., :3] - tgt[..., :3]).double() ** 2).mean())
            radii.append(hctx.debug_segments(ws, n_seg)[0][:, 4].copy())
        return total / len(cams), radii

    # adjoint (autograd through the library's backward) against central differences of the
    # loss in log parameters (h = 1e-3, Richardson with h/2); parameters whose step moves an
    # integer coverage radius in any view sit on a discontinuity and are skipped
    params = [b.clone().requires_grad_(True) for b in base]
    F.lod_loss(hctx, aid, 1, cams, lights, targets, params[0].exp(), params[1].exp(), params[2].exp(),
               ws).backward()
    grads = [p.grad.detach().clone() for p in params]
    rng = np.random.Generator(np.random.PCG64(seed))
    h = 1e-3
    results, tried = [], 0
    with torch.no_grad():
        _, radii0 = loss_and_radii(base)
        while len(results) < n_fd and tried < 20 * n_fd:
            tried += 1
            which = int(rng.choice([0, 0, 0, 1, 2]))
            idx = tuple(int(rng.integers(n)) for n in base[which].shape)
            vals, same = {}, True
            for step in (h, 0.5 * h):
                for sgn in (1, -1):
                    p = [b.clone() for b in base]
                    p[which][idx] += sgn * step
                    vals[(step, sgn)], radii = loss_and_radii(p)
                    same &= all(np.array_equal(a, b) for a, b in zip(radii, radii0))
            if not same:
                continue
            f1 = (vals[(h, 1)] - vals[(h, -1)]) / (2 * h)
            f2 = (vals[(0.5 * h, 1)] - vals[(0.5 * h, -1)]) / h
            results.append((which, idx, (4 * f2 - f1) / 3, float(grads[which][idx])))
    scale_g = max(abs(r[3]) for r in results) if results else 0.0
    passed = sum(abs(fd - an) <= 2e-2 * abs(an) + 5e-3 * scale_g for _, _, fd, an in results)
    res = F.fit_level(hctx, aid, 1, cams, lights, iters=iters, lr=1e-2, ws=ws, targets=targets)
    out = {"experiment": "fit", "groom": "500 locks, smooth flow" if locks else "random walk",
           "strands": asset.n_strands, "segments": asset.n_segments,
           "clusters": int(lod0.r.shape[0]), "views": len(cams), "resolution": list(c["res"]),
           "iters": iters, "loss_before": res.loss_history[0], "loss_after": res.loss_history[-1],
           "loss_ratio": res.loss_history[-1] / res.loss_history[0],
           "seconds": round(res.seconds, 2), "ms_per_iter": round(1e3 * res.seconds / max(1, iters), 2),
           "fd_checked": len(results), "fd_passed": int(passed), "fd_tried": tried,
           "fd_worst_rel": max((abs(fd - an) / max(abs(an), 1e-30) for _, _, fd, an in results), default=None)}
    ws.close()
    hctx.release(aid)
    return out


def curved_frames(hctx: B.Context, scale: float = 1.0, repeats: int = 20, clusters: int = 1000):
    import torch
    import hairsynth as hs
    asset, cam, lights = hs.config(3, scale)
    aid = hctx.upload_asset(asset)
    hctx.build_lod(aid, [hs.kmeans_assign(asset, max(1, int(round(clusters * scale))), seed=1003)])
    ws = hctx.workspace()

    def timed(fn):
        img, st, _ = fn()
        torch.cuda.synchronize()
        ms = []
        for _ in range(repeats):
            _, s2, _ = fn()
            ms.append(s2["ms_total"])
        return img.clone(), st, float(np.percentile(ms, 50))

    out = {"experiment": "curved", "strands": asset.n_strands, "clusters": clusters, "width": cam.width,
           "height": cam.height, "frames": []}
    poly, st, ms = timed(lambda: hctx.render(aid, 1, cam, lights, ws=ws))
    out["frames"].append({"centre_lines": "polyline", "steps": int(st["segments"]), "fragments": int(st["fragments"]),
                          "frame_ms_p50": round(ms, 4), "rmse_vs_polyline": 0.0})
    for max_px in (4, 2, 1):
        img, st, ms = timed(lambda: hctx.render_curved(aid, 1, cam, lights, max_px, 16, ws=ws))
        rmse, _ = _rgb_error(img, poly)
        out["frames"].append({"centre_lines": f"curved, <= {max_px} px per step", "steps": int(st["segments"]),
                              "fragments": int(st["fragments"]), "frame_ms_p50": round(ms, 4),
                              "rmse_vs_polyline": round(rmse, 6)})
    ws.close()
    hctx.release(aid)
    return out


def shadow_frames(hctx: B.Context, iters: int = 20, shadow=(1024, 4, 0.02)):
    import torch
    import hairsynth as hs
    asset, cam, lights = hs.config(2)
    aid = hctx.upload_asset(asset)
    ws = hctx.workspace()
    ms = []
    for i in range(iters + 2):
        _, st, _ = hctx.render_shadowed(aid, 0, cam, lights, shadow, ws=ws)
        if i >= 2:
            ms.append(st["ms_total"])
    torch.cuda.synchronize()
    plain = []
    for i in range(iters + 2):
        _, st0, _ = hctx.render(aid, 0, cam, lights, ws=ws)
        if i >= 2:
            plain.append(st0["ms_total"])
    out = {"experiment": "shadow", "strands": asset.n_strands, "width": cam.width, "height": cam.height,
           "resolution": shadow[0], "layers": shadow[1], "layer_depth": shadow[2], "frames": iters,
           "fragments": int(st["fragments"]), "frame_ms_p50": round(float(np.percentile(ms, 50)), 4),
           "frame_ms_mean": round(float(np.mean(ms)), 4),
           "plain_frame_ms_p50": round(float(np.percentile(plain, 50)), 4)}
    hctx.release(aid)
    # a mixed-level frame (per-group LoD of the serving asset of the same size: 100k strands
    # x 32 segments with 6250 / 390 / 24 thick hairs, initial levels at eps_w = 8 px so that
    # a share of the (group, segment) cells goes coarse), plain and shadowed
    from . import serve as S
    assets = S.build_assets(hctx, specs=((100_000, 32),), seed=1002)
    a = next(iter(assets.values()))
    lev = torch.empty((a.groups, a.asset.segs), dtype=torch.int32, device=f"cuda:{hctx.device}")
    hctx.lod_init(a.aid, cam, 8.0, lev, ws=ws)
    hist = np.bincount(lev.cpu().numpy().reshape(-1), minlength=len(a.segments_per_level))
    mixed_plain, mixed_sh = [], []
    for i in range(iters + 2):
        _, s1, _ = hctx.render_mixed(a.aid, cam, a.lights, lev, ws=ws)
        _, s2, _ = hctx.render_mixed_shadowed(a.aid, cam, a.lights, lev, shadow, ws=ws)
        if i >= 2:
            mixed_plain.append(s1["ms_total"])
            mixed_sh.append(s2["ms_total"])
    torch.cuda.synchronize()
    out["mixed"] = {"asset": "100k x 32 strands, 6250 / 390 / 24 thick hairs", "eps_w": 8.0,
                    "cells_per_level": [round(float(v), 4) for v in hist / hist.sum()],
                    "segments": int(s1["segments"]), "fragments": int(s1["fragments"]),
                    "plain_ms_p50": round(float(np.percentile(mixed_plain, 50)), 4),
                    "shadowed_ms_p50": round(float(np.percentile(mixed_sh, 50)), 4)}
    hctx.release(a.aid)
    ws.close()
    return out


def view_distances(hctx: B.Context, occupancies=(0.5, 0.1, 0.003), repeats: int = 20, eps_w: float = 2.0,
                   spec=(100_000, 32), clumped: bool = True, width: int = 1920, height: int = 1080):
    """The LoD at the near, middle and far views of Sec. 6 (the groom's bounding sphere covering
    50%, 10% and 0.3% of the image): the strand frame against the level chosen per request
    (hair_select_level at eps_w) and the per-group mixed-level frame (hair_lod_init at eps_w),
    each timed and compared with the strand frame of the same view.  The groom: spec strands
    in locks of 16 that follow a smooth flow (clumped), or the random-walk groom of the other
    workloads; levels of one thick hair per 16 / 64 / 256 strands (the cross-section growing
    about fourfold per level, Sec. 5.1), nested k-means on the strands' paths (4 points each,
    the metric of Sec. 5.1 step 1), the 390 coarsest clusters being the LoD groups."""
    import torch
    import hairsynth as hs
    from . import serve as S
    n, segs = spec
    asset = hs.make_asset(n, segs, 90.0, seed=1002, sigma_spread=True, clumps=max(1, n // 16) if clumped else 0,
                          flow=0.99 if clumped else 0.0)
    aid = hctx.upload_asset(asset)
    t0 = time.perf_counter()
    assigns = hs.kmeans_hierarchy(asset, [max(1, n // d) for d in (16, 64, 256)], seed=1002, iters=20,
                                  features="path")
    t_kmeans = time.perf_counter() - t0
    hctx.build_lod(aid, assigns)
    _, counts, S_ = hctx.lod_info(aid)
    a = S.ServedAsset(aid, asset, hs.default_lights(asset, with_point=True), [c * S_ for c in counts],
                      hctx.lod_groups(aid), assigns)
    ws = hctx.workspace()
    out = {"experiment": "views", "groom": "locks of 16 strands, smooth flow" if clumped else "random walk",
           "strands": a.asset.n_strands, "segments": a.asset.n_segments, "kmeans_s": round(t_kmeans, 2),
           "thick_hairs_per_level": [int(c) for c in counts[1:]], "width": width,
           "height": height, "eps_w": eps_w, "views": []}

    def timed(fn):
        img, st, _ = fn(None)
        ms = []
        for _ in range(repeats):
            _, s2, _ = fn(img)
            ms.append(s2["ms_total"])
        torch.cuda.synchronize()
        return img.clone(), st, round(float(np.percentile(ms, 50)), 4)

    for occ in occupancies:
        cam = hs.camera_occupancy(a.asset, width, height, occ)
        ref, st0, ms0 = timed(lambda o: hctx.render(a.aid, 0, cam, a.lights, out=o, ws=ws))
        level = hctx.select_level(a.aid, cam, eps_w, ws=ws)
        img1, st1, ms1 = timed(lambda o: hctx.render(a.aid, level, cam, a.lights, out=o, ws=ws))
        lev = torch.empty((a.groups, a.asset.segs), dtype=torch.int32, device=f"cuda:{hctx.device}")
        hctx.lod_init(a.aid, cam, eps_w, lev, ws=ws)
        hist = np.bincount(lev.cpu().numpy().reshape(-1), minlength=len(a.segments_per_level))
        img2, st2, ms2 = timed(lambda o: hctx.render_mixed(a.aid, cam, a.lights, lev, out=o, ws=ws))
        v = {"occupancy": occ,
             "strands": {"segments": int(st0["segments"]), "fragments": int(st0["fragments"]), "frame_ms_p50": ms0},
             "selected_level": {"level": int(level), "segments": int(st1["segments"]),
                                "fragments": int(st1["fragments"]), "frame_ms_p50": ms1},
             "mixed": {"cells_per_level": [round(float(x), 4) for x in hist / hist.sum()],
                       "segments": int(st2["segments"]), "fragments": int(st2["fragments"]), "frame_ms_p50": ms2}}
        for key, img in (("selected_level", img1), ("mixed", img2)):
            rmse, psnr = _rgb_error(img, ref)
            v[key]["rmse"] = round(rmse, 6)
            v[key]["psnr_db"] = round(psnr, 2)
        out["views"].append(v)
        print(json.dumps({"occupancy": occ, "done": True}), flush=True)
    ws.close()
    hctx.release(a.aid)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["lod-sweep", "fit", "shadow", "curved", "views"])
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--iters", type=int, default=200)
    ap.add_argument("--locks", action="store_true", help="fit: a groom of locks instead of the random walk")
    args = ap.parse_args()
    import torch
    assert torch.cuda.is_available()
    hctx = B.Context(0)
    if args.what == "lod-sweep":
        print(json.dumps(lod_sweep(hctx, args.scale)), flush=True)
    elif args.what == "curved":
        print(json.dumps(curved_frames(hctx, args.scale)), flush=True)
    elif args.what == "views":
        spec = (max(1, int(round(100_000 * args.scale))), 32)
        for clumped in (True, False):
            print(json.dumps(view_distances(hctx, spec=spec, clumped=clumped)), flush=True)
    elif args.what == "shadow":
        print(json.dumps(shadow_frames(hctx, args.iters if args.iters != 200 else 20)), flush=True)
    else:
        print(json.dumps(fit_report(hctx, args.iters, args.scale, locks=args.locks)), flush=True)
    hctx.close()


if __name__ == "__main__":
    main()
