"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds random draws and their memory layout only.  It performs no
step of the rendering or reconstruction method (no projection, compositing,
divergence or Poisson arithmetic), so both the FP64 oracle and the HIP path can
consume the very same FP32 arrays without sharing any of the method's code.

Distributions follow the workload recipes of the benchmark configurations:
means uniform in x, y in [-1, 1] and z in a depth range, per-axis log-scales
normal, random unit quaternions, opacity = sigmoid(N(0, 1)), six gradient
values per splat drawn from Laplace(0, 0.05) so the gradient field is sparse.
The paper's own scenes (Banana, Train, Truck) are not available; these
synthetic scenes stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "CONFIGS", "Scene", "Camera", "make_scene", "make_camera", "pose",
    "reference_image", "raster_scene", "sample_pixels",
]


@dataclass
class Scene:
    """Structure-of-arrays splat scene, every array FP32 and C-contiguous.

    mean[3][K] world position, log_scale[3][K] per-axis log standard scale,
    quat[4][K] rotation quaternion (w, x, y, z), opacity[K] in (0, 1),
    value[6][K] gradient amplitudes, channel index 2*c + d with c in RGB and
    d = 0 for the derivative along image columns, 1 along image rows (or
    value[3][K], one Laplacian per colour channel, in the Laplacian-splat form).
    """
    mean: np.ndarray
    log_scale: np.ndarray
    quat: np.ndarray
    opacity: np.ndarray
    value: np.ndarray

    @property
    def K(self) -> int:
        return int(self.opacity.shape[0])


@dataclass
class Camera:
    """Pinhole camera in OpenCV axes (x right, y down, +z forward).

    R (3x3) and t (3) map world to camera coordinates, x_c = R x + t.
    fx, fy are focal lengths in pixels; (cx, cy) the principal point.
    """
    W: int
    H: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray = field(default_factory=lambda: np.eye(3))
    t: np.ndarray = field(default_factory=lambda: np.zeros(3))


# Workload recipes.  Keys: image size, splat count, depth range, log-scale
# distribution, multigrid levels and stopping tolerance, boundary ring source.
CONFIGS = {
    "tiny": dict(W=64, H=64, K=2000, z=(2.0, 6.0), ls=(-4.0, 0.5), levels=4,
                 tol=1e-8, ring="zero"),
    "mid": dict(W=800, H=800, K=200_000, z=(2.0, 6.0), ls=(-4.0, 0.5), levels=7,
                tol=1e-6, ring="reference"),
    "full": dict(W=1920, H=1080, K=1_000_000, z=(2.0, 20.0), ls=(-5.0, 0.7),
                 levels=8, tol=1e-6, ring="reference"),
    "diff": dict(W=512, H=512, K=100_000, z=(2.0, 6.0), ls=(-4.0, 0.5), levels=7,
                 tol=1e-6, ring="zero"),
    "serve": dict(W=1920, H=1080, K=500_000, z=(2.0, 20.0), ls=(-5.0, 0.7),
                  levels=8, tol=1e-6, ring="reference"),
    # the sparse regime of the paper's trained scenes: a few thousand splats
    # per scene (5,100 is the largest count reported) carrying Laplacian
    # values, at 1080p, with the full workload's distributions
    "sparse": dict(W=1920, H=1080, K=5_100, z=(2.0, 20.0), ls=(-5.0, 0.7),
                   levels=8, tol=1e-6, ring="reference"),
}

# Serving mix: request sizes drawn uniformly from these (W, H).
SERVE_SIZES = [(256, 256), (512, 512), (800, 800), (1920, 1080)]


def serving_requests(n: int = 256, seed: int = 7):
    """n requests: (W, H) uniform over SERVE_SIZES and pose index i (pose(i)
    is the camera pose of request i; focal length W)."""
    rng = np.random.default_rng(seed)
    return [(SERVE_SIZES[int(k)], i) for i, k in enumerate(rng.integers(0, len(SERVE_SIZES), n))]


def poisson_arrivals(n: int, qps: float, seed: int = 7) -> np.ndarray:
    """Arrival offsets in seconds of a Poisson process of rate qps (first at 0)."""
    rng = np.random.default_rng(seed + 1)
    gaps = rng.exponential(1.0 / qps, n)
    gaps[0] = 0.0
    return np.cumsum(gaps)


def make_scene(K: int, seed: int = 0, z=(2.0, 6.0), ls=(-4.0, 0.5),
               xy=(-1.0, 1.0)) -> Scene:
    """Draw a K-splat scene.  Draw order: means x, y, z; log-scales (K x 3);
    quaternions (K x 4, normalised in FP64); opacity logits; values (K x 6)."""
    rng = np.random.default_rng(seed)
    mx = rng.uniform(xy[0], xy[1], K)
    my = rng.uniform(xy[0], xy[1], K)
    mz = rng.uniform(z[0], z[1], K)
    log_scale = rng.normal(ls[0], ls[1], (K, 3))
    q = rng.normal(0.0, 1.0, (K, 4))
    nrm = np.sqrt((q * q).sum(axis=1, keepdims=True))
    q = q / np.where(nrm > 0, nrm, 1.0)
    logits = rng.normal(0.0, 1.0, K)
    opacity = 1.0 / (1.0 + np.exp(-logits))
    value = rng.laplace(0.0, 0.05, (K, 6))
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Scene(mean=f32(np.stack([mx, my, mz])), log_scale=f32(log_scale.T),
                 quat=f32(q.T), opacity=f32(opacity), value=f32(value.T))


def laplacian_scene(scene: Scene, seed: int = 0) -> Scene:
    """The same splats carrying three Laplacian values each (the Laplacian-splat
    form): Laplace(0, 0.05) draws, K x 3, from their own generator (seed + 2000)."""
    rng = np.random.default_rng(seed + 2000)
    K = scene.opacity.shape[0]
    lap = rng.laplace(0.0, 0.05, (K, 3))
    return Scene(mean=scene.mean, log_scale=scene.log_scale, quat=scene.quat,
                 opacity=scene.opacity, value=np.ascontiguousarray(lap.T, dtype=np.float32))


def _axis_angle(axis: np.ndarray, angle: float) -> np.ndarray:
    """Rotation matrix of a unit axis and an angle (Rodrigues' formula)."""
    x, y, z = axis
    K = np.array([[0.0, -z, y], [z, 0.0, -x], [-y, x, 0.0]])
    return np.eye(3) + math.sin(angle) * K + (1.0 - math.cos(angle)) * (K @ K)


def pose(i: int):
    """Camera pose number i (seed 1000 + i): rotation about an axis uniform on
    the sphere by an angle uniform in [0, 5] degrees, camera centre uniform in
    [-0.1, 0.1]^3.  Returns (R, t) with x_c = R x + t."""
    rng = np.random.default_rng(1000 + i)
    axis = rng.normal(0.0, 1.0, 3)
    axis /= np.linalg.norm(axis)
    angle = math.radians(rng.uniform(0.0, 5.0))
    centre = rng.uniform(-0.1, 0.1, 3)
    R = _axis_angle(axis, angle)
    return R, -R @ centre


def make_camera(W: int, H: int, fx: float | None = None, pose_index: int | None = None) -> Camera:
    """Camera with fx = fy = W unless given, principal point at the image
    centre, identity pose unless a pose index is given."""
    f = float(W if fx is None else fx)
    cam = Camera(W=W, H=H, fx=f, fy=f, cx=W / 2.0, cy=H / 2.0)
    if pose_index is not None:
        cam.R, cam.t = pose(pose_index)
    return cam


def trajectory_camera(W: int, H: int, i: int, seed: int = 11,
                      deg_per_frame: float = 0.02, step: float = 5e-4) -> Camera:
    """Frame i of a smooth camera path: rotation about a fixed axis (uniform on
    the sphere, seed) by i * deg_per_frame degrees, centre moved i * step
    along a fixed unit direction (seed + 1); fx = fy = W."""
    rng = np.random.default_rng(seed)
    axis = rng.normal(0.0, 1.0, 3)
    axis /= np.linalg.norm(axis)
    d = np.random.default_rng(seed + 1).normal(0.0, 1.0, 3)
    d /= np.linalg.norm(d)
    R = _axis_angle(axis, math.radians(deg_per_frame * i))
    cam = make_camera(W, H)
    cam.R, cam.t = R, -R @ (d * step * i)
    return cam


def reference_image(H: int, W: int, seed: int = 1) -> np.ndarray:
    """Smooth seeded reference image [3][H][W] (FP64): 0.5 plus four products
    of sines with random amplitudes in [-0.1, 0.1], integer frequencies 1..3
    and random phases.  Its one-pixel ring is the Dirichlet data of the solve."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-0.1, 0.1, (3, 4))
    k = rng.integers(1, 4, 4)
    l = rng.integers(1, 4, 4)
    phi = rng.uniform(0.0, 2 * math.pi, 4)
    psi = rng.uniform(0.0, 2 * math.pi, 4)
    j = np.arange(W)[None, :]
    i = np.arange(H)[:, None]
    img = np.full((3, H, W), 0.5)
    for m in range(4):
        basis = np.sin(math.pi * k[m] * j / W + phi[m]) * np.sin(math.pi * l[m] * i / H + psi[m])
        img += a[:, m, None, None] * basis[None]
    return img


def raster_scene(K: int, W: int, H: int, seed: int = 0, ls=(-4.0, 0.5), z=(2.0, 6.0),
                 fx: float | None = None):
    """Rasteriser-level inputs for the differentiation workload, drawn directly
    in image space: mean2d[2][K] uniform over the image, conic[3][K] = (a, b, c)
    of R(theta) diag(1/s1^2, 1/s2^2) R(theta)^T with s = fx * exp(N(ls)) / z,
    opacity[K], value[6][K], depth[K] uniform in z.  All FP32."""
    rng = np.random.default_rng(seed)
    f = float(W if fx is None else fx)
    mx = rng.uniform(0.0, W, K)
    my = rng.uniform(0.0, H, K)
    depth = rng.uniform(z[0], z[1], K)
    s = f * np.exp(rng.normal(ls[0], ls[1], (2, K))) / depth[None]
    th = rng.uniform(0.0, math.pi, K)
    c, sn = np.cos(th), np.sin(th)
    i1, i2 = 1.0 / s[0] ** 2, 1.0 / s[1] ** 2
    ca = c * c * i1 + sn * sn * i2
    cb = c * sn * (i1 - i2)
    cc = sn * sn * i1 + c * c * i2
    logits = rng.normal(0.0, 1.0, K)
    opacity = 1.0 / (1.0 + np.exp(-logits))
    value = rng.laplace(0.0, 0.05, (6, K))
    f32 = lambda a_: np.ascontiguousarray(a_, dtype=np.float32)
    return dict(mean2d=f32(np.stack([mx, my])), conic=f32(np.stack([ca, cb, cc])),
                opacity=f32(opacity), value=f32(value), depth=f32(depth))


def sample_pixels(H: int, W: int, n: int, seed: int = 5):
    """n distinct seeded pixel coordinates (rows, cols), always including the
    four corners so image borders and ragged tile tails are sampled."""
    rng = np.random.default_rng(seed)
    flat = rng.choice(H * W, size=min(n, H * W), replace=False)
    corners = np.array([0, W - 1, (H - 1) * W, H * W - 1])
    flat = np.unique(np.concatenate([flat, corners]))
    return flat // W, flat % W

