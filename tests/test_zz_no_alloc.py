"""gdgs_poisson_solve_static (scratch in the library's fixed device array, no
allocation) against gdgs_poisson_solve with a caller workspace, through the C
ABI: two calls in a row, the second on a smaller image, plus the exact solve
of the oracle and the size limit."""
import numpy as np
import pytest
import torch

import paper_2405_05446_amd as G
import workloads as wl
from oracle import poisson as P
from tests.gpu_util import say, np_

pytestmark = pytest.mark.gpu
TOL = 1e-4


def _gradients(H, W, seed):
    """Forward differences of the seeded reference image plus Laplace noise
    (a non-integrable field, as composited gradients are)."""
    f = wl.reference_image(H, W, seed=seed)
    g = np.zeros((6, H, W))
    g[0::2, :, :-1] = f[:, :, 1:] - f[:, :, :-1]
    g[1::2, :-1, :] = f[:, 1:, :] - f[:, :-1, :]
    g += np.random.default_rng(seed).laplace(0.0, 0.01, g.shape)
    return g.astype(np.float32)


def _both(H, W, seed, mg):
    grad = torch.from_numpy(_gradients(H, W, seed)).cuda()
    ring = torch.from_numpy(wl.reference_image(H, W, seed=1).astype(np.float32)).cuda()
    u_ws, st_ws = G.gdgs_poisson_solve(grad, ring, W, H, mg)
    st = G.new_stats()
    u_s, _ = G.api.gdgs_poisson_solve_static(grad, ring, W, H, mg, stats=st)
    torch.cuda.synchronize()
    return grad, ring, u_ws, G.read_stats(st_ws), u_s, G.read_stats(st)


def test_static_scratch_solve_equals_workspace_solve_twice():
    mg = G.mg_params(tol=1e-6)
    for (W, H, seed) in [(1920, 1080, 3), (300, 200, 4)]:
        say(f"[static scratch] {W}x{H}")
        grad, ring, u_ws, s_ws, u_s, s_s = _both(H, W, seed, mg)
        err = (u_s - u_ws).abs().max().item()
        say(f"  max-abs vs workspace solve {err:.3e} (bitwise {torch.equal(u_s, u_ws)}), "
            f"cycles {s_s['cycles']} vs {s_ws['cycles']}")
        assert s_s["converged"] and s_ws["converged"]
        assert err <= TOL
        exact = P.solve_dst(P.divergence(np_(grad).astype(np.float64)),
                            np_(ring).astype(np.float64))
        e2 = np.abs(np_(u_s) - exact).max()
        say(f"  max-abs vs exact solve {e2:.3e}")
        assert e2 <= TOL


def test_static_scratch_rejects_sizes_beyond_the_array():
    W, H = 2048, 2048
    grad = torch.zeros((6, H, W), device="cuda")
    with pytest.raises(G.GdgsError) as e:
        G.api.gdgs_poisson_solve_static(grad, None, W, H, G.mg_params())
    assert e.value.status == 3 and "static array" in str(e.value)
