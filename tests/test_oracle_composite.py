"""Pins of the oracle's compositing (Eq. 11 / Eq. 20) by closed forms,
order-independent identities and invariants."""
import math

import numpy as np

import workloads as wl
from oracle import composite as oc
from oracle.constants import E_CUT
from oracle.project import project_2d


def splats2d(mx, my, conic, depth, opacity, value):
    f = lambda a: np.asarray(a, dtype=np.float64)
    return dict(mean2d=f([mx, my]), conic=f(conic), depth=f(depth),
                opacity=f(opacity), value=f(value))


def test_single_splat_closed_form_no_half_in_exponent():
    # isotropic conic 1/s^2: at distance d from the centre G = exp(-d^2/s^2)
    s = 1.7
    sp = splats2d([10.5], [8.5], [[1 / s ** 2], [0.0], [1 / s ** 2]], [3.0], [0.8],
                  np.arange(1, 7, dtype=float).reshape(6, 1))
    proj = project_2d(sp["mean2d"], sp["conic"], sp["depth"], 24, 20)
    for (i, j) in [(8, 10), (8, 12), (6, 11), (9, 7)]:
        d2 = (j + 0.5 - 10.5) ** 2 + (i + 0.5 - 8.5) ** 2
        out = oc.composite_pixel(i, j, proj, sp["opacity"], sp["value"])
        assert np.allclose(out, np.arange(1, 7) * 0.8 * math.exp(-d2 / s ** 2), rtol=1e-14)


def test_two_splats_front_one_first():
    # splat 1 is deeper than splat 0 ... so the front one is splat 0
    sp = splats2d([5.5, 5.5], [5.5, 5.5], [[0.1, 0.2], [0, 0], [0.1, 0.2]], [1.0, 2.0],
                  [0.6, 0.3], np.array([[1.0, 10.0]] * 6))
    proj = project_2d(sp["mean2d"], sp["conic"], sp["depth"], 12, 12)
    a0, a1 = 0.6, 0.3
    out = oc.composite_pixel(5, 5, proj, sp["opacity"], sp["value"])
    assert np.allclose(out, 1.0 * a0 + 10.0 * a1 * (1 - a0), rtol=1e-14)
    # swap depths: now splat 1 is in front
    sp["depth"] = np.array([2.0, 1.0])
    proj = project_2d(sp["mean2d"], sp["conic"], sp["depth"], 12, 12)
    out = oc.composite_pixel(5, 5, proj, sp["opacity"], sp["value"])
    assert np.allclose(out, 10.0 * a1 + 1.0 * a0 * (1 - a1), rtol=1e-14)


def test_equal_depth_ties_go_to_lower_index():
    sp = splats2d([5.5, 5.5], [5.5, 5.5], [[0.1, 0.2], [0, 0], [0.1, 0.2]], [2.0, 2.0],
                  [0.6, 0.3], np.array([[1.0, 10.0]] * 6))
    proj = project_2d(sp["mean2d"], sp["conic"], sp["depth"], 12, 12)
    out = oc.composite_pixel(5, 5, proj, sp["opacity"], sp["value"])
    assert np.allclose(out, 1.0 * 0.6 + 10.0 * 0.3 * 0.4, rtol=1e-14)


def test_depths_equal_in_fp32_are_ties():
    d = 3.0
    d_next = float(np.nextafter(np.float32(d), np.float32(10)))
    sp = splats2d([5.5, 5.5], [5.5, 5.5], [[0.1, 0.2], [0, 0], [0.1, 0.2]],
                  [d + 0.25 * (d_next - d), d], [0.6, 0.3], np.array([[1.0, 10.0]] * 6))
    proj = project_2d(sp["mean2d"], sp["conic"], sp["depth"], 12, 12)
    out = oc.composite_pixel(5, 5, proj, sp["opacity"], sp["value"])
    # FP32 keys tie -> index order (splat 0 first) although FP64 says splat 1 is nearer
    assert np.allclose(out, 1.0 * 0.6 + 10.0 * 0.3 * 0.4, rtol=1e-14)


def _random_scene(K, seed, W=40, H=30):
    rs = wl.raster_scene(K, W, H, seed=seed, ls=(-1.8, 0.4), fx=W)
    return rs, project_2d(rs["mean2d"], rs["conic"], rs["depth"], W, H)


def test_all_ones_channel_is_one_minus_product_any_order():
    rs, proj = _random_scene(150, 1)
    value = np.ones((6, 150))
    rng = np.random.default_rng(0)
    for _ in range(20):
        i, j = rng.integers(0, 30), rng.integers(0, 40)
        out = oc.composite_pixel(i, j, proj, rs["opacity"], value)
        idx, G, _, _ = oc.pixel_terms(i, j, proj, rs["opacity"])
        a = rs["opacity"].astype(np.float64)[idx] * G
        rng.shuffle(a)
        assert np.allclose(out, 1.0 - np.prod(1.0 - a), rtol=1e-13, atol=1e-15)


def test_weights_plus_final_transmittance_is_one_and_linear_in_values():
    rs, proj = _random_scene(150, 2)
    rng = np.random.default_rng(1)
    v1 = rng.normal(size=(6, 150))
    v2 = rng.normal(size=(6, 150))
    for _ in range(20):
        i, j = rng.integers(0, 30), rng.integers(0, 40)
        ones = oc.composite_pixel(i, j, proj, rs["opacity"], np.ones((1, 150)))[0]
        T = oc.transmittance(i, j, proj, rs["opacity"])
        assert abs(ones + T - 1.0) < 1e-14
        o1 = oc.composite_pixel(i, j, proj, rs["opacity"], v1)
        o2 = oc.composite_pixel(i, j, proj, rs["opacity"], v2)
        o12 = oc.composite_pixel(i, j, proj, rs["opacity"], 2.0 * v1 - 3.0 * v2)
        assert np.allclose(o12, 2 * o1 - 3 * o2, rtol=1e-12, atol=1e-14)


def test_transmittance_non_increasing_over_depth_prefixes():
    rs, proj = _random_scene(200, 3)
    order = np.argsort(rs["depth"], kind="stable")
    rng = np.random.default_rng(2)
    for _ in range(10):
        i, j = rng.integers(0, 30), rng.integers(0, 40)
        prev = 1.0
        for cut in range(0, 201, 20):
            keep = np.zeros(200, bool)
            keep[order[:cut]] = True
            sub = dict(proj)
            sub["valid"] = proj["valid"] & keep
            T = oc.transmittance(i, j, sub, rs["opacity"])
            assert T <= prev + 1e-15
            prev = T


def test_support_cutoff_is_exact_zero_beyond_ecut():
    s = 1.0
    # pixel (0, 0) centre at (0.5, 0.5); place the mean so E is just above/below E_CUT
    for E_target, expect_zero in [(E_CUT * (1 + 1e-9), True), (E_CUT * (1 - 1e-9), False)]:
        d = math.sqrt(E_target) * s
        sp = splats2d([0.5 + d], [0.5], [[1 / s ** 2], [0], [1 / s ** 2]], [2.0], [0.9],
                      np.ones((6, 1)))
        proj = project_2d(sp["mean2d"], sp["conic"], sp["depth"], 20, 4)
        out = oc.composite_pixel(0, 0, proj, sp["opacity"], sp["value"])
        if expect_zero:
            assert (out == 0).all()
        else:
            assert np.allclose(out, 0.9 * math.exp(-E_target), rtol=1e-12)


def test_box_prefilter_changes_nothing():
    sc = wl.make_scene(400, seed=5, ls=(-2.5, 0.5))
    cam = wl.make_camera(48, 40)
    from oracle.project import project
    proj = project(sc, cam)
    rng = np.random.default_rng(4)
    for _ in range(15):
        i, j = rng.integers(0, 40), rng.integers(0, 48)
        a = oc.composite_pixel(i, j, proj, sc.opacity, sc.value, use_box=True)
        b = oc.composite_pixel(i, j, proj, sc.opacity, sc.value, use_box=False)
        assert np.array_equal(a, b)
