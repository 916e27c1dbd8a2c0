"""End-to-end render (project -> bin -> composite -> Poisson) against the oracle."""
import numpy as np
import pytest
import torch

import paper_2405_05446_amd as G
import workloads as wl
from oracle import composite as oc, poisson as P
from oracle.project import project as oproject
from oracle.render import render as orender
from tests.gpu_util import say, np_, gpu_stages, composite_parity

pytestmark = pytest.mark.gpu
TOL = 1e-4


def test_tiny_workload_end_to_end():
    cfg = wl.CONFIGS["tiny"]
    say("[render] tiny workload end to end")
    sc = wl.make_scene(cfg["K"], seed=0, z=cfg["z"], ls=cfg["ls"])
    cam = wl.make_camera(cfg["W"], cfg["H"])
    ds = G.DeviceScene.from_host(sc)
    # the oracle solves to relative residual 1e-8 in FP64 (dense LU); the FP32
    # solve stops on a 1e-6 relative correction
    u, st = G.gdgs_render(ds, cam, None, G.mg_params(levels=cfg["levels"], tol=1e-6,
                                                     max_cycles=40), sync_stats=True)
    torch.cuda.synchronize()
    o = orender(sc, cam, None)
    err = np.abs(np_(u) - o["u"]).max()
    s = G.read_stats(st)
    say(f"  max-abs {err:.3e}, stats {s}")
    assert err <= TOL
    assert P.relative_residual(o["u"], o["rho"]).max() <= 1e-8


def test_ragged_posed_render_with_reference_ring():
    H, W = 72, 100
    sc = wl.make_scene(3000, seed=3, ls=(-3, 0.6))
    cam = wl.make_camera(W, H, pose_index=4)
    ring = wl.reference_image(H, W, seed=1).astype(np.float32)
    ds = G.DeviceScene.from_host(sc)
    u, st = G.gdgs_render(ds, cam, torch.from_numpy(ring).cuda(), G.mg_params(tol=1e-7),
                          sync_stats=True)
    torch.cuda.synchronize()
    o = orender(sc, cam, ring.astype(np.float64))
    assert np.abs(np_(u) - o["u"]).max() <= TOL


@pytest.mark.parametrize("name", ["mid", "full"])
def test_workload_stagewise(name):
    cfg = wl.CONFIGS[name]
    say(f"[render] {name} workload stage-wise")
    sc = wl.make_scene(cfg["K"], seed=0, z=cfg["z"], ls=cfg["ls"])
    cam = wl.make_camera(cfg["W"], cfg["H"], pose_index=0 if name == "full" else None)
    H, W = cfg["H"], cfg["W"]
    ring = wl.reference_image(H, W, seed=1).astype(np.float32)
    ds = G.DeviceScene.from_host(sc)
    mg = G.mg_params(levels=cfg["levels"], tol=cfg["tol"])
    u, st = G.gdgs_render(ds, cam, torch.from_numpy(ring).cuda(), mg, sync_stats=True)
    torch.cuda.synchronize()
    s = G.read_stats(st)
    say(f"  stats {s}")
    g = gpu_stages(sc, cam)
    # composite on sampled pixels vs brute force over all splats
    o = oproject(sc, cam)
    rows, cols = wl.sample_pixels(H, W, 2000 if name == "full" else 1000, seed=12)
    e1, ties = composite_parity(g, o, sc, H, W, rows, cols)
    # Poisson of the GPU's gradients vs the exact DST-I solve
    exact = P.solve_dst(P.divergence(g["grad"].astype(np.float32)), ring.astype(np.float64))
    e2 = np.abs(np_(u) - exact).max()
    say(f"  composite max-abs {e1:.3e} ({ties} depth-tie pixels), poisson max-abs {e2:.3e}")
    assert e2 <= TOL and s["converged"] and not s["overflow"]


def test_render_capacity_overflow_status():
    sc = wl.make_scene(2000, seed=0)
    cam = wl.make_camera(64, 64)
    ds = G.DeviceScene.from_host(sc)
    with pytest.raises(G.GdgsError) as e:
        G.gdgs_render(ds, cam, None, capacity=10, sync_stats=True)
    assert e.value.status == 2


def test_renderer_retries_on_overflow():
    sc = wl.make_scene(2000, seed=0)
    cam = wl.make_camera(64, 64)
    r = G.Renderer(G.DeviceScene.from_host(sc), 64, 64, G.mg_params(tol=1e-6, max_cycles=40),
                   capacity=16)
    u = r.render(cam)
    o = orender(sc, cam, None)
    assert np.abs(np_(u) - o["u"]).max() <= TOL
    assert r.capacity >= r.last["num_pairs"] and r.last["converged"]


def test_renderer_budget_and_warm_continuation_match_full_solve():
    H, W = 90, 160
    sc = wl.make_scene(4000, seed=8, ls=(-3, 0.6))
    ring = torch.from_numpy(wl.reference_image(H, W, seed=1).astype(np.float32)).cuda()
    r = G.Renderer(G.DeviceScene.from_host(sc), W, H, G.mg_params(tol=1e-6, max_cycles=30))
    us = []
    for i in range(4):
        cam = wl.make_camera(W, H, pose_index=i)
        if i == 2:
            r.budget = 1          # force the warm continuation path
        u = r.render(cam, ring).clone()
        assert r.last["converged"], r.last
        o = orender(sc, cam, np_(ring).astype(np.float64))
        assert np.abs(np_(u) - o["u"]).max() <= TOL
        us.append(r.last["total_cycles"])
    say(f"[render] cycles per frame {us}")


def test_graph_replays_match_eager_launches():
    """Every replay of the captured launch sequence equals an eager run, with
    eager work and synchronisation between the replays."""
    H, W = 72, 100
    sc = wl.make_scene(3000, seed=9, ls=(-3, 0.6))
    cam = wl.make_camera(W, H, pose_index=5)
    ds = G.DeviceScene.from_host(sc)
    ring = torch.from_numpy(wl.reference_image(H, W, seed=1).astype(np.float32)).cuda()
    lib = G.load()
    mg = G.mg_params(tol=1e-6)
    cap = 1 << 16
    ws = G.workspace(G.render_workspace_size(ds.K, W, H, cap, mg))
    u = torch.empty((3, H, W), device="cuda")
    stats = G.new_stats()
    lib.gdgs_set_graphs(0)
    G.gdgs_render(ds, cam, ring, mg, cap, u, stats, ws, sync_stats=True)
    eager = np_(u).copy()
    lib.gdgs_set_graphs(1)
    try:
        for rep in range(4):
            u.fill_(float("nan"))
            G.gdgs_render(ds, cam, ring, mg, cap, u, stats, ws, sync_stats=True)
            torch.cuda.synchronize()
            assert np.array_equal(np_(u), eager), rep
            # eager work between replays
            lib.gdgs_set_graphs(0)
            G.gdgs_render(ds, wl.make_camera(W, H, pose_index=rep), ring, mg, cap, u, stats, ws,
                          sync_stats=True)
            lib.gdgs_set_graphs(1)
    finally:
        lib.gdgs_set_graphs(1)


def test_render_sequence_equals_render_frame_by_frame():
    """Pipelined sequence (host enqueues view i + 1 before settling view i,
    two buffer sets) == render() per view, bit for bit; a capacity overflow
    in the middle of the sequence is re-rendered."""
    H, W = 64, 96
    sc = wl.make_scene(5000, seed=13, ls=(-3, 0.6))
    ds = G.DeviceScene.from_host(sc)
    ring = torch.from_numpy(wl.reference_image(H, W, seed=1).astype(np.float32)).cuda()
    cams = [wl.make_camera(W, H, pose_index=i) for i in range(7)]
    ref = G.Renderer(ds, W, H, G.mg_params(tol=1e-6, max_cycles=30))
    want = [ref.render(c, ring).clone() for c in cams]
    seq = G.Renderer(ds, W, H, G.mg_params(tol=1e-6, max_cycles=30), capacity=64)
    got = {}
    seq.render_sequence(cams, ring, on_frame=lambda i, u, st: got.__setitem__(i, (u.clone(), st)))
    torch.cuda.synchronize()
    assert sorted(got) == list(range(len(cams)))
    for i, (u, st) in got.items():
        assert st["converged"] and torch.equal(u, want[i]), i
    assert seq.capacity > 64


def test_render_sequence_with_two_frames_in_flight_equals_render():
    """The two buffer sets on streams of their own (two frames on the device
    at once) == render() per view, bit for bit, including a capacity overflow
    in the middle; the consumer's copies on the caller's stream are ordered
    before the buffers are reused."""
    H, W = 64, 96
    sc = wl.make_scene(5000, seed=13, ls=(-3, 0.6))
    ds = G.DeviceScene.from_host(sc)
    ring = torch.from_numpy(wl.reference_image(H, W, seed=1).astype(np.float32)).cuda()
    cams = [wl.make_camera(W, H, pose_index=i) for i in range(9)]
    ref = G.Renderer(ds, W, H, G.mg_params(tol=1e-6, max_cycles=30))
    want = [ref.render(c, ring).clone() for c in cams]
    seq = G.Renderer(ds, W, H, G.mg_params(tol=1e-6, max_cycles=30), capacity=64)
    got = {}
    for rnd in range(2):
        got.clear()
        seq.render_sequence(cams, ring, overlap=True,
                            on_frame=lambda i, u, st: got.__setitem__(i, (u.clone(), st)))
        torch.cuda.synchronize()
        assert sorted(got) == list(range(len(cams)))
        for i, (u, st) in got.items():
            assert st["converged"] and torch.equal(u, want[i]), (rnd, i)
    assert seq.capacity > 64


def test_two_frames_in_flight_with_resumed_solves_equal_render():
    """Two frames in flight on their own streams while every solve is resumed
    (a one-cycle budget, continued two cycles at a time on the frame's
    stream): the statistics are read only after that stream's work, and the
    results equal render() bit for bit."""
    H, W = 64, 96
    sc = wl.make_scene(5000, seed=14, ls=(-3, 0.6))
    ds = G.DeviceScene.from_host(sc)
    ring = torch.from_numpy(wl.reference_image(H, W, seed=1).astype(np.float32)).cuda()
    cams = [wl.make_camera(W, H, pose_index=i) for i in range(6)]
    mg = G.mg_params(tol=1e-6, max_cycles=30)
    ref = G.Renderer(ds, W, H, mg)
    want = [ref.render(c, ring).clone() for c in cams]
    seq = G.Renderer(ds, W, H, mg, adaptive=False)
    seq.budget = 1
    got = {}
    seq.render_sequence(cams, ring, overlap=True,
                        on_frame=lambda i, u, st: got.__setitem__(i, (u.clone(), st)))
    torch.cuda.synchronize()
    assert sorted(got) == list(range(len(cams)))
    for i, (u, st) in got.items():
        assert st["converged"] and st["total_cycles"] > 1, (i, st)
        assert torch.equal(u, want[i]), i


def test_warm_start_along_a_trajectory_meets_the_tolerance_in_fewer_cycles():
    """Consecutive views of a moving camera (Sec. 2.2: one view per pose):
    starting each solve from the previous image gives the same images within
    the image tolerance, in fewer V-cycles."""
    W, H, K = 320, 180, 20000
    sc = wl.make_scene(K, seed=0, z=(2.0, 20.0), ls=(-5.0, 0.7))
    ds = G.DeviceScene.from_host(sc)
    ring = torch.from_numpy(wl.reference_image(H, W, seed=1).astype(np.float32)).cuda()
    mg = G.mg_params(tol=1e-6, max_cycles=30)
    cams = [wl.trajectory_camera(W, H, i) for i in range(8)]
    out = {}
    for warm in (False, True):
        r = G.Renderer(ds, W, H, mg, warm_start=warm)
        us, cyc = [], []
        r.render_sequence(cams, ring, on_frame=lambda i, u, st: (us.append(u.clone()),
                                                                 cyc.append(st["total_cycles"])))
        torch.cuda.synchronize()
        out[warm] = (us, cyc)
    say(f"[render] trajectory cycles cold {out[False][1]} warm {out[True][1]}")
    for a, b in zip(out[False][0], out[True][0]):
        assert (a - b).abs().max().item() <= 1e-4
    assert sum(out[True][1][1:]) < sum(out[False][1][1:])


def test_largest_workload_4k_4m_splats():
    # four times the pixels and the splats of the 1080p workload: pair counts,
    # tile indices and the multigrid plan at scale (composite on sampled pixels
    # vs brute force over all splats, the solve vs the exact DST-I solve)
    W, H, K = 3840, 2160, 4_000_000
    say(f"[render] largest workload {W}x{H}, {K} splats")
    sc = wl.make_scene(K, seed=5, z=(2.0, 20.0), ls=(-5.0, 0.7))
    cam = wl.make_camera(W, H, pose_index=3)
    ring = wl.reference_image(H, W, seed=1).astype(np.float32)
    ds = G.DeviceScene.from_host(sc)
    cap = 24 * K
    u, st = G.gdgs_render(ds, cam, torch.from_numpy(ring).cuda(), G.mg_params(tol=1e-6),
                          capacity=cap, sync_stats=True)
    torch.cuda.synchronize()
    s = G.read_stats(st)
    g = gpu_stages(sc, cam, capacity=cap)
    say(f"  pairs {g['num_pairs']}, cycles {s['cycles']}")
    assert g["num_pairs"] <= cap and s["converged"] and not s["overflow"]
    o = oproject(sc, cam)
    rows, cols = wl.sample_pixels(H, W, 120, seed=13)
    ref = oc.render_grad(o, sc.opacity, sc.value, H, W, rows, cols)
    e1 = np.abs(g["grad"][:, rows, cols] - ref).max()
    exact = P.solve_dst(P.divergence(g["grad"].astype(np.float32)), ring.astype(np.float64))
    e2 = np.abs(np_(u) - exact).max()
    say(f"  composite max-abs {e1:.3e}, poisson max-abs {e2:.3e}")
    assert e1 <= TOL and e2 <= TOL


@pytest.mark.parametrize("form", ["neumann", "laplacian_threshold"])
def test_two_frames_in_flight_other_forms_equal_render(form):
    """Two frames in flight (front halves on the caller's stream, solves on
    the renderer's solve stream) for the Neumann problem and for thresholded
    Laplacian splats: every frame equals render() bit for bit."""
    H, W = 90, 140
    base = wl.make_scene(6000, seed=21, ls=(-3, 0.6))
    if form == "neumann":
        sc = base
        mk = lambda: G.Renderer(G.DeviceScene.from_host(sc), W, H,
                                G.mg_params(tol=1e-6, max_cycles=40), neumann=True)
        ring = None
    else:
        sc = wl.laplacian_scene(base, seed=21)
        mk = lambda: G.Renderer(G.DeviceScene.from_host(sc), W, H,
                                G.mg_params(tol=1e-6, max_cycles=40), threshold=2e-3)
        ring = torch.from_numpy(wl.reference_image(H, W, seed=1).astype(np.float32)).cuda()
    cams = [wl.make_camera(W, H, pose_index=i) for i in range(5)]
    ref = mk()
    want = []
    for c in cams:
        want.append(ref.render(c, ring).clone())
    seq = mk()
    got = {}
    seq.render_sequence(cams, ring, overlap=True,
                        on_frame=lambda i, u, st: got.__setitem__(i, (u.clone(), st)))
    torch.cuda.synchronize()
    say(f"[render] two in flight, {form}: cycles "
        f"{[got[i][1]['total_cycles'] for i in sorted(got)]}")
    assert sorted(got) == list(range(len(cams)))
    for i, (u, st) in got.items():
        assert st["converged"] and torch.equal(u, want[i]), i
