"""Serving loop: every request renders the same alone and inside a concurrent mix (mixed
per-group LoD and one level per request), served outputs match the oracle, admission charges
the memory the workspaces really hold, and a request that outgrows its estimate waits instead
of failing."""
import numpy as np
import pytest
import torch

import hairsynth as hs
from oracle import lod as OL
from oracle import mixed as M
from oracle import render as R

pytestmark = pytest.mark.gpu

SMALL_RES = ((320, 180), (640, 360), (480, 480))
RTOL, ATOL = 1e-4, 1e-7
UHD = 7            # index of the request served at 3840x2160


@pytest.fixture(scope="module")
def served(hip):
    from paper_2405_10565_amd import serve as S
    ctx = hip.Context(0)
    assets = S.build_assets(ctx, specs=((1500, 8), (4000, 12), (800, 16)), level_divisors=(8, 64))
    # every level's data from the oracle's construction (the memberships stay those of
    # hair_build_lod), so that served frames and the oracle render the same level data
    lods = {}
    for name, a in assets.items():
        lods[name] = [OL.build_level(a.asset, asg) for asg in a.assigns]
        for l, lod in enumerate(lods[name], 1):
            ctx.set_lod(a.aid, l, lod)
        assert ctx.lod_groups(a.aid) == a.groups
    yield ctx, assets, lods
    ctx.close()


def _mix(S, names, seed):
    reqs = S.make_requests(names, 36, seed=seed, resolutions=SMALL_RES)
    reqs[UHD].width, reqs[UHD].height = 3840, 2160
    return reqs


def _camera(a, r):
    return hs.camera_occupancy(a.asset, r.width, r.height, r.occupancy, r.azimuth)


def _oracle_geom(a, lods, r):
    """The geometry a served request rendered: its mixed level map, or its single level."""
    if r.levels_used is not None and len(np.unique(r.levels_used)) > 1:
        geoms = M.level_geoms(a.asset, lods)
        return M.mixed_geometry(geoms, M.groups(a.assigns), r.levels_used), "mixed"
    if r.level == 0:
        return R.strand_level(a.asset), "level 0"
    return R.cluster_level(lods[r.level - 1]), f"level {r.level}"


def _check_against_oracle(a, lods, r, rect=None):
    geom, what = _oracle_geom(a, lods, r)
    cam = _camera(a, r)
    mat = tuple(float(v) for v in a.asset.material.as_array())
    ref, ras = R.render(geom, cam, a.lights, mat, rect=rect)
    got = r.output.cpu().numpy().astype(np.float64)
    if rect is None:
        assert r.fragments == len(ras.seg), (r.rid, what)
    else:
        x0, y0, w, h = rect
        got, ref = got[y0:y0 + h, x0:x0 + w], ref[y0:y0 + h, x0:x0 + w]
    err = np.abs(got - ref) - (RTOL * np.abs(ref) + ATOL)
    print(f"served request {r.rid} ({r.asset}, {r.width}x{r.height}, {what}, rect {rect}): "
          f"{int((err > 0).sum())} violations", flush=True)
    assert int((err > 0).sum()) == 0, (r.rid, what)
    return what


@pytest.mark.parametrize("lod", ["mixed", "level"])
def test_mix_equals_alone(hip, served, lod):
    print(f"case: serving mix vs alone, lod={lod}", flush=True)
    from paper_2405_10565_amd import serve as S
    ctx, assets, lods = served
    names = sorted(assets)
    eps = 6.0                       # wide enough that many (group, segment) cells go coarse
    mix = _mix(S, names, 5)
    srv = S.Server(ctx, assets, n_slots=4, keep_outputs=True, lod=lod, eps_w=eps)
    S.run_poisson(srv, mix, rate=2000.0, seed=5)
    peak = srv.peak_in_flight
    srv.close()
    assert all(r.status == 0 for r in mix)
    assert peak >= 2                             # requests really overlapped
    alone = _mix(S, names, 5)
    srv1 = S.Server(ctx, assets, n_slots=1, keep_outputs=True, lod=lod, eps_w=eps)
    for r in alone:
        srv1.submit(r)
        srv1.drain()
    srv1.close()
    for a, b in zip(mix, alone):
        assert (a.asset, a.width, a.level) == (b.asset, b.width, b.level)
        assert torch.equal(a.output.view(torch.int32), b.output.view(torch.int32)), a.rid
    res = S.summarize(mix, 2000.0)
    print(res, flush=True)
    assert res["completed"] == 36 and res["latency_ms_p99"] >= res["latency_ms_p50"] > 0
    if lod != "mixed":
        return
    # served outputs of the concurrent mix against the oracle: a mixed-level request and a
    # single-level one in full, and a rectangle at the densest pixel of the 2160p request
    kinds = []
    mixed = [r for r in mix if r.levels_used is not None and len(np.unique(r.levels_used)) > 1
             and r.width * r.height <= 640 * 360]
    single = [r for r in mix if r.levels_used is not None and len(np.unique(r.levels_used)) == 1
              and r.width * r.height <= 640 * 360]
    assert mixed and single
    kinds.append(_check_against_oracle(assets[mixed[0].asset], lods[mixed[0].asset], mixed[0]))
    kinds.append(_check_against_oracle(assets[single[0].asset], lods[single[0].asset], single[0]))
    uhd = mix[UHD]
    alpha = uhd.output[..., 3].cpu().numpy()
    y, x = np.unravel_index(np.argmax(alpha), alpha.shape)
    x0, y0 = int(min(max(x - 12, 0), uhd.width - 24)), int(min(max(y - 12, 0), uhd.height - 24))
    kinds.append(_check_against_oracle(assets[uhd.asset], lods[uhd.asset], uhd, rect=(x0, y0, 24, 24)))
    assert "mixed" in kinds


def test_shadowed_serving_equals_alone_and_oracle(hip, served):
    """Served frames with deep opacity map shadows (mixed frames over their own rows): the same
    alone and in the mix, and a mixed-level one against the oracle."""
    print("case: shadowed serving", flush=True)
    from paper_2405_10565_amd import serve as S
    ctx, assets, lods = served
    names = sorted(assets)
    sh = (128, 4, 0.02)
    mix = S.make_requests(names, 16, seed=8, resolutions=SMALL_RES[:2])
    srv = S.Server(ctx, assets, n_slots=4, keep_outputs=True, eps_w=6.0, shadow=sh)
    S.run_poisson(srv, mix, rate=2000.0, seed=8)
    srv.close()
    alone = S.make_requests(names, 16, seed=8, resolutions=SMALL_RES[:2])
    srv1 = S.Server(ctx, assets, n_slots=1, keep_outputs=True, eps_w=6.0, shadow=sh)
    for r in alone:
        srv1.submit(r)
        srv1.drain()
    srv1.close()
    assert all(r.status == 0 for r in mix + alone)
    for a, b in zip(mix, alone):
        assert torch.equal(a.output.view(torch.int32), b.output.view(torch.int32)), a.rid
    mixed = [r for r in mix if r.levels_used is not None and len(np.unique(r.levels_used)) > 1]
    assert mixed
    r = mixed[0]
    a = assets[r.asset]
    geom, _ = _oracle_geom(a, lods[r.asset], r)
    ref, ras = R.render(geom, _camera(a, r), a.lights, tuple(float(v) for v in a.asset.material.as_array()), shadow=sh)
    got = r.output.cpu().numpy().astype(np.float64)
    err = np.abs(got - ref) - (RTOL * np.abs(ref) + ATOL)
    print(f"shadowed served request {r.rid}: {int((err > 0).sum())} violations", flush=True)
    assert int((err > 0).sum()) == 0 and r.fragments == len(ras.seg)


def test_admission_by_footprint(hip, served):
    print("case: admission", flush=True)
    from paper_2405_10565_amd import serve as S
    ctx, assets, _ = served
    names = sorted(assets)
    reqs = S.make_requests(names[:1], 12, seed=9, resolutions=((640, 360),))
    fp = S.Server.footprint(type("X", (), {"assets": assets})(), reqs[0])
    # equal footprints and room for exactly one of them, even with four slots
    srv = S.Server(ctx, assets, n_slots=4, scratch_budget=fp + fp // 2)
    S.run_poisson(srv, reqs, rate=5000.0, seed=9)
    assert srv.peak_in_flight == 1
    assert all(r.status == 0 for r in reqs)
    assert srv.peak_bytes <= fp + fp // 2
    held = sum(s.ws.memory()[0] for s in srv.slots)
    assert 0 < held <= fp + fp // 2                 # the memory really held stays in the budget
    srv.close()
    # a request larger than the whole budget is rejected, not queued forever
    srv2 = S.Server(ctx, assets, n_slots=2, scratch_budget=1024)
    r = S.make_requests(names, 1, seed=1, resolutions=((640, 360),))[0]
    srv2.submit(r)
    srv2.close()
    assert r in srv2.rejected and r.status == -2


def test_request_outgrowing_its_estimate_waits(hip, served):
    """Estimates far below what the frames really allocate: each frame fails in the library
    (its workspace is limited to its reservation), goes back to the queue with a larger
    estimate and completes; the workspaces never hold more than the budget."""
    print("case: admission with underestimated footprints", flush=True)
    from paper_2405_10565_amd import serve as S
    ctx, assets, _ = served
    names = sorted(assets)

    class Tight(S.Server):
        def footprint(self, req):
            return 1 << 20

    ref = S.make_requests(names, 10, seed=13, resolutions=((640, 360), (480, 480)))
    need = max(S.Server.footprint(type("X", (), {"assets": assets})(), r) for r in ref)
    budget = need + need // 4
    srv = Tight(ctx, assets, n_slots=3, scratch_budget=budget, keep_outputs=True)
    reqs = S.make_requests(names, 10, seed=13, resolutions=((640, 360), (480, 480)))
    S.run_poisson(srv, reqs, rate=5000.0, seed=13)
    peak_bytes = srv.peak_bytes
    held = [s.ws.memory()[0] for s in srv.slots]
    srv.close()
    assert all(r.status == 0 for r in reqs), [r.status for r in reqs]
    assert len(srv.done) == len(reqs)
    assert sum(r.retries for r in reqs) > 0          # estimates were outgrown and retried
    assert peak_bytes <= budget and sum(held) <= budget
    # and the outputs equal the same requests served with the regular estimate
    srv1 = S.Server(ctx, assets, n_slots=1, keep_outputs=True)
    again = S.make_requests(names, 10, seed=13, resolutions=((640, 360), (480, 480)))
    for r in again:
        srv1.submit(r)
        srv1.drain()
    srv1.close()
    for a, b in zip(reqs, again):
        assert torch.equal(a.output.view(torch.int32), b.output.view(torch.int32)), a.rid
