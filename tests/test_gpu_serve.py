"""Serving loop: every request renders the same alone and inside a concurrent mix; admission
respects the scratch budget."""
import numpy as np
import pytest
import torch

import hairsynth as hs

pytestmark = pytest.mark.gpu

SMALL_RES = ((320, 180), (640, 360), (480, 480))


@pytest.fixture(scope="module")
def served(hip):
    from paper_2405_10565_amd import serve as S
    ctx = hip.Context(0)
    assets = S.build_assets(ctx, specs=((1500, 8), (4000, 12), (800, 16)), level_divisors=(8, 64))
    yield ctx, assets
    ctx.close()


def test_mix_equals_alone(hip, served):
    print("case: serving mix vs alone", flush=True)
    from paper_2405_10565_amd import serve as S
    ctx, assets = served
    names = sorted(assets)
    mix = S.make_requests(names, 36, seed=5, resolutions=SMALL_RES)
    srv = S.Server(ctx, assets, n_slots=4, keep_outputs=True)
    S.run_poisson(srv, mix, rate=2000.0, seed=5)
    peak = srv.peak_in_flight
    srv.close()
    assert all(r.status == 0 for r in mix)
    assert peak >= 2                             # requests really overlapped
    alone = S.make_requests(names, 36, seed=5, resolutions=SMALL_RES)
    srv1 = S.Server(ctx, assets, n_slots=1, keep_outputs=True)
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


def test_admission_by_footprint(hip, served):
    print("case: admission", flush=True)
    from paper_2405_10565_amd import serve as S
    ctx, assets = served
    names = sorted(assets)
    reqs = S.make_requests(names[:1], 12, seed=9, resolutions=((640, 360),))
    fp = S.Server.footprint(type("X", (), {"assets": assets})(), reqs[0])
    # equal footprints and room for exactly one of them, even with four slots
    srv = S.Server(ctx, assets, n_slots=4, scratch_budget=fp + fp // 2)
    S.run_poisson(srv, reqs, rate=5000.0, seed=9)
    assert srv.peak_in_flight == 1
    assert all(r.status == 0 for r in reqs)
    srv.close()
    # a request larger than the whole budget is rejected, not queued forever
    srv2 = S.Server(ctx, assets, n_slots=2, scratch_budget=1024)
    r = S.make_requests(names, 1, seed=1, resolutions=((640, 360),))[0]
    srv2.submit(r)
    srv2.close()
    assert r in srv2.rejected and r.status == -2
