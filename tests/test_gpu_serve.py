"""Render server (continuous batching of mixed-size views of one resident
scene): results in the mix equal the same request alone, capacity re-runs,
resumed solves, budget admission, cancellation and scheduled arrivals."""
import numpy as np
import pytest
import torch

import paper_2405_05446_amd as G
import workloads as wl
from oracle.render import render as orender
from tests.gpu_util import say, np_

pytestmark = pytest.mark.gpu

SIZES = [(64, 48), (128, 96), (200, 160), (320, 180)]
MG = dict(tol=1e-6, max_cycles=30)


@pytest.fixture(scope="module")
def scene():
    sc = wl.make_scene(20000, seed=0, z=(2.0, 20.0), ls=(-5.0, 0.7))
    return sc, G.DeviceScene.from_host(sc)


def rings():
    return {(W, H): torch.from_numpy(wl.reference_image(H, W, seed=1).astype(np.float32)).cuda()
            for W, H in SIZES}


def requests(n, seed=7):
    rng = np.random.default_rng(seed)
    return [(SIZES[int(rng.integers(len(SIZES)))], i) for i in range(n)]


def test_mixed_equals_alone_and_plain_renderer(scene):
    sc, ds = scene
    reqs = requests(24)
    ring = rings()
    # alone: one request at a time through a one-stream server
    alone = {}
    with G.Server(ds, budget=1 << 30, streams=1, mg=G.mg_params(**MG)) as srv:
        for (W, H), i in reqs:
            rid, u = srv.submit(wl.make_camera(W, H, pose_index=i), ring[(W, H)], tag=i)
            c = srv.drain(1)[0]
            assert c["status"] == 0 and c["converged"] == 1 and c["tag"] == i
            alone[i] = u.clone()
    # mixed: everything at once over four streams
    with G.Server(ds, budget=1 << 30, streams=4, mg=G.mg_params(**MG)) as srv:
        for (W, H), i in reqs:
            srv.submit(wl.make_camera(W, H, pose_index=i), ring[(W, H)], tag=i)
        done = srv.drain(len(reqs))
        st = srv.state()
    say(f"[serve] mixed: {len(done)} done, state {st}")
    assert sorted(c["tag"] for c in done) == list(range(len(reqs)))
    for c in done:
        assert c["status"] == 0 and c["converged"] == 1
        assert torch.equal(c["u"], alone[c["tag"]]), c
        assert c["admit_ns"] >= c["arrival_ns"] and c["done_ns"] >= c["admit_ns"]
    assert st["running"] == 0 and st["waiting"] == 0 and st["peak_bytes"] <= st["budget_bytes"]
    # the plain per-request path gives the same bits
    for (W, H), i in reqs[:6]:
        r = G.Renderer(ds, W, H, G.mg_params(**MG))
        u = r.render(wl.make_camera(W, H, pose_index=i), ring[(W, H)])
        torch.cuda.synchronize()
        assert torch.equal(u, alone[i])


SERVE_SIZES = [(256, 256), (512, 512), (800, 800), (1920, 1080)]


def test_serving_workload_mixed_equals_alone_renderer_and_oracle():
    """The serving workload's resident 500k-splat scene with two requests of
    each size (256^2, 512^2, 800^2, 1920x1080): all of them at once over four
    streams give the same bits as each alone on a one-stream server and as
    the plain Renderer; at 256^2, 800^2 and 1080p the composite matches the
    oracle on 300 sampled pixels and the solve matches the exact DST-I solve
    of the GPU's gradients."""
    from oracle import poisson as P
    from oracle.project import project as oproject
    from tests.gpu_util import gpu_stages, composite_parity
    cfg = wl.CONFIGS["serve"]
    say(f"[serve] serving workload, K={cfg['K']}")
    sc = wl.make_scene(cfg["K"], seed=0, z=cfg["z"], ls=cfg["ls"])
    ds = G.DeviceScene.from_host(sc)
    reqs = [(sz, 40 + 2 * k + r) for k, sz in enumerate(SERVE_SIZES) for r in range(2)]
    ring = {sz: torch.from_numpy(wl.reference_image(sz[1], sz[0], seed=1).astype(np.float32))
            .cuda() for sz in SERVE_SIZES}
    mg = G.mg_params(**MG)
    alone = {}
    with G.Server(ds, budget=4 << 30, streams=1, mg=mg) as srv:
        for (W, H), i in reqs:
            srv.submit(wl.make_camera(W, H, pose_index=i), ring[(W, H)], tag=i)
            c = srv.drain(1)[0]
            assert c["status"] == 0 and c["converged"] == 1
            alone[i] = c["u"].clone()
    for batched in (False, True):
        with G.Server(ds, budget=4 << 30, streams=3 if batched else 4, mg=mg,
                      batched=batched) as srv:
            for (W, H), i in reqs[::-1]:
                srv.submit(wl.make_camera(W, H, pose_index=i), ring[(W, H)], tag=i)
            done = srv.drain(len(reqs))
        assert sorted(c["tag"] for c in done) == sorted(i for _, i in reqs)
        for c in done:
            assert c["status"] == 0 and c["converged"] == 1
            assert torch.equal(c["u"], alone[c["tag"]]), (batched, c["tag"])
    for (W, H), i in reqs[::2]:
        r = G.Renderer(ds, W, H, mg)
        u = r.render(wl.make_camera(W, H, pose_index=i), ring[(W, H)])
        torch.cuda.synchronize()
        assert torch.equal(u, alone[i]), (W, H)
    for (W, H), i in [reqs[0], reqs[4], reqs[6]]:
        cam = wl.make_camera(W, H, pose_index=i)
        g = gpu_stages(sc, cam)
        o = oproject(sc, cam)
        rows, cols = wl.sample_pixels(H, W, 300, seed=30 + i)
        e1, ties = composite_parity(g, o, sc, H, W, rows, cols)
        exact = P.solve_dst(P.divergence(g["grad"].astype(np.float32)),
                            np_(ring[(W, H)]).astype(np.float64))
        e2 = np.abs(np_(alone[i]) - exact).max()
        say(f"  {W}x{H}: composite max-abs {e1:.3e} ({ties} tie pixels), solve max-abs {e2:.3e}")
        assert e2 <= 1e-4


def test_batched_rounds_equal_alone_and_plain_renderer(scene):
    """Batched solves (one device table, persistent-kernel rounds, completion
    ring): 24 mixed requests at once give the bits of the same requests
    solved alone on a one-stream per-request server and of the plain
    Renderer; one request alone in the batch gives them too."""
    sc, ds = scene
    reqs = requests(24, seed=9)
    ring = rings()
    mg = G.mg_params(**MG)
    alone = {}
    with G.Server(ds, budget=1 << 30, streams=1, mg=mg) as srv:
        for (W, H), i in reqs:
            srv.submit(wl.make_camera(W, H, pose_index=i), ring[(W, H)], tag=i)
            c = srv.drain(1)[0]
            assert c["status"] == 0 and c["converged"] == 1
            alone[i] = c["u"].clone()
    with G.Server(ds, budget=1 << 30, streams=3, mg=mg, batched=True) as srv:
        for (W, H), i in reqs:
            srv.submit(wl.make_camera(W, H, pose_index=i), ring[(W, H)], tag=i)
        done = srv.drain(len(reqs))
        # a finished solve's slot is released once the rounds that may still
        # read it have completed
        import time
        t0 = time.perf_counter()
        while srv.state()["running"] > 0 and time.perf_counter() - t0 < 5.0:
            time.sleep(0.001)
        st = srv.state()
    say(f"[serve batched] {len(done)} done, state {st}")
    assert sorted(c["tag"] for c in done) == list(range(len(reqs)))
    for c in done:
        assert c["status"] == 0 and c["converged"] == 1, c
        assert torch.equal(c["u"], alone[c["tag"]]), c["tag"]
    assert st["running"] == 0 and st["waiting"] == 0
    # one at a time through the batched path
    with G.Server(ds, budget=1 << 30, streams=1, mg=mg, batched=True) as srv:
        for (W, H), i in reqs[:5]:
            srv.submit(wl.make_camera(W, H, pose_index=i), ring[(W, H)], tag=i)
            c = srv.drain(1)[0]
            assert c["status"] == 0 and torch.equal(c["u"], alone[i]), i
    for (W, H), i in reqs[:4]:
        r = G.Renderer(ds, W, H, mg)
        u = r.render(wl.make_camera(W, H, pose_index=i), ring[(W, H)])
        torch.cuda.synchronize()
        assert torch.equal(u, alone[i])


def test_batched_capacity_rerun_limit_and_cancel(scene):
    """Batched solves: a pair-capacity overflow re-runs the front half with a
    larger capacity and still gives the alone bits; a cycle limit below the
    need completes unconverged with exactly that many cycles; a cancelled
    request completes as cancelled and the others are unaffected."""
    sc, ds = scene
    mg = G.mg_params(**MG)
    # large splats: far more pairs than the initial capacity of 65536
    big = G.DeviceScene.from_host(wl.make_scene(5000, seed=5, z=(2.0, 6.0), ls=(-2.0, 0.3)))
    W, H = 320, 180
    cam = wl.make_camera(W, H, pose_index=2)
    want = G.Renderer(big, W, H, mg).render(cam).clone()
    torch.cuda.synchronize()
    with G.Server(big, budget=1 << 30, streams=2, mg=mg, batched=True) as srv:
        srv.submit(cam, None, tag=1)
        c = srv.drain(1)[0]
    say(f"[serve batched] big splats: {c['num_pairs']} pairs, attempts {c['attempts']}")
    assert c["status"] == 0 and c["converged"] == 1 and c["attempts"] >= 2
    assert c["num_pairs"] > 65536 and torch.equal(c["u"], want)
    W, H = 200, 160
    ring = torch.from_numpy(wl.reference_image(H, W, seed=1).astype(np.float32)).cuda()
    cam = wl.make_camera(W, H, pose_index=2)
    with G.Server(ds, budget=1 << 30, streams=2, mg=G.mg_params(tol=1e-6, max_cycles=3),
                  batched=True) as srv:
        srv.submit(cam, ring, tag=2)
        c = srv.drain(1)[0]
        assert c["status"] == 0 and c["converged"] == 0 and c["cycles"] == 3
    with G.Server(ds, budget=1 << 30, streams=1, mg=mg, batched=True) as srv:
        ids = [srv.submit(wl.make_camera(W, H, pose_index=k), ring, tag=k)[0] for k in range(4)]
        srv.cancel(ids[3])
        done = {c["tag"]: c for c in srv.drain(4)}
        assert done[3]["status"] == 8
        for k in range(3):
            assert done[k]["status"] == 0 and done[k]["converged"] == 1


def test_small_view_against_the_oracle(scene):
    sc, ds = scene
    W, H = 64, 48
    ring = torch.from_numpy(wl.reference_image(H, W, seed=1).astype(np.float32)).cuda()
    cam = wl.make_camera(W, H, pose_index=3)
    with G.Server(ds, budget=256 << 20, streams=2, mg=G.mg_params(**MG)) as srv:
        srv.submit(cam, ring)
        c = srv.drain(1)[0]
    o = orender(sc, cam, np_(ring).astype(np.float64))
    err = np.abs(np_(c["u"]) - o["u"]).max()
    say(f"[serve] 64x48 vs oracle max-abs {err:.3e}")
    assert c["status"] == 0 and err <= 1e-4


def test_capacity_rerun_and_cycle_limit():
    # large splats: far more pairs than the initial capacity of 65536
    sc = wl.make_scene(5000, seed=5, z=(2.0, 6.0), ls=(-2.0, 0.3))
    ds = G.DeviceScene.from_host(sc)
    W, H = 320, 180
    cam = wl.make_camera(W, H, pose_index=2)
    with G.Server(ds, budget=1 << 30, streams=2, mg=G.mg_params(**MG)) as srv:
        srv.submit(cam, None)
        c = srv.drain(1)[0]
    say(f"[serve] big splats: {c['num_pairs']} pairs, attempts {c['attempts']}")
    assert c["status"] == 0 and c["num_pairs"] > 65536 and c["attempts"] >= 2
    r = G.Renderer(ds, W, H, G.mg_params(**MG))
    assert torch.equal(r.render(cam), c["u"])
    # one V-cycle allowed: reported as not converged, 1 cycle
    with G.Server(ds, budget=1 << 30, streams=1, mg=G.mg_params(tol=1e-12, max_cycles=1)) as srv:
        srv.submit(cam, None)
        c1 = srv.drain(1)[0]
    assert c1["status"] == 0 and c1["converged"] == 0 and c1["cycles"] == 1


def test_budget_cancel_and_scheduled_arrival(scene):
    sc, ds = scene
    with G.Server(ds, budget=64 << 20, streams=2, mg=G.mg_params(**MG)) as srv:
        with pytest.raises(G.GdgsError) as e:
            srv.submit(wl.make_camera(1920, 1080), None)      # cannot fit 64 MiB
        assert e.value.status == 4
        # a request scheduled 30 s ahead is cancelled while it waits
        far = G.now_ns() + 30_000_000_000
        rid, _ = srv.submit(wl.make_camera(64, 48), None, tag=5, arrival_ns=far)
        srv.cancel(rid)
        c = srv.drain(1)[0]
        assert c["id"] == rid and c["status"] == 8
        with pytest.raises(G.GdgsError):
            srv.cancel(rid)
        # a request scheduled 50 ms ahead does not start before then
        t = G.now_ns() + 50_000_000
        srv.submit(wl.make_camera(64, 48, pose_index=1), None, tag=6, arrival_ns=t)
        c = srv.drain(1)[0]
        assert c["status"] == 0 and c["arrival_ns"] == t and c["admit_ns"] >= t
        assert srv.state()["completed"] == 2


def test_warm_started_requests_along_a_camera_path(scene):
    # each view of a moving camera starts from the previous view's image
    sc, ds = scene
    W, H = 320, 180
    cams = [wl.trajectory_camera(W, H, i) for i in range(6)]
    mg = G.mg_params(**MG)
    cold, warm, cyc_cold, cyc_warm = [], [], [], []
    with G.Server(ds, budget=1 << 30, streams=2, mg=mg) as srv:
        for cam in cams:
            srv.submit(cam, None)
            c = srv.drain(1)[0]
            assert c["status"] == 0 and c["converged"] == 1
            cold.append(c["u"].clone())
            cyc_cold.append(c["cycles"])
        prev = None
        for cam in cams:
            srv.submit(cam, None, u_init=prev)
            c = srv.drain(1)[0]
            assert c["status"] == 0 and c["converged"] == 1
            warm.append(c["u"].clone())
            cyc_warm.append(c["cycles"])
            prev = c["u"]
    say(f"[serve] camera path cycles cold {cyc_cold}, warm {cyc_warm}")
    assert sum(cyc_warm[1:]) < sum(cyc_cold[1:])
    for a, b in zip(cold, warm):
        assert (a - b).abs().max().item() <= 1e-4
    # the plain path's warm start gives the same bits
    r = G.Renderer(ds, W, H, mg, warm_start=True)
    for cam, b in zip(cams, warm):
        u = r.render(cam)
        torch.cuda.synchronize()
        assert torch.equal(u, b)


def test_neumann_server_equals_plain_path(scene):
    # the paper's boundary condition in serving: mixed sizes, results equal to
    # the plain per-request path's; a request with boundary data is refused
    sc, ds = scene
    mg = G.mg_params(tol=1e-6, max_cycles=30, flags=G.NEUMANN)
    reqs = requests(12, seed=3)
    with G.Server(ds, budget=1 << 30, streams=4, mg=mg) as srv:
        for (W, H), i in reqs:
            srv.submit(wl.make_camera(W, H, pose_index=i), None, tag=i)
        done = srv.drain(len(reqs))
        W, H = SIZES[0]
        with pytest.raises(G.GdgsError):
            srv.submit(wl.make_camera(W, H), torch.zeros((3, H, W), device="cuda"))
    assert all(c["status"] == 0 and c["converged"] == 1 for c in done)
    by_tag = {c["tag"]: c["u"] for c in done}
    for (W, H), i in reqs[:6]:
        r = G.Renderer(ds, W, H, mg)
        u = r.render(wl.make_camera(W, H, pose_index=i))
        torch.cuda.synchronize()
        assert torch.equal(u, by_tag[i])
        assert abs(float(u.double().mean())) <= 1e-6
