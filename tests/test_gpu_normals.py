"""Normal estimation (30 nearest points, FP64 PCA) through the C ABI
against the oracle: the neighbour sets are the same (exact FP32 keys) and
the covariance sums run in the same order; the eigen-solvers differ (GPU
cyclic Jacobi, oracle one-sided Jacobi SVD), so the FP32 normals agree to a
few units in the last place. A point-to-plane registration with estimated
normals reaches the accuracy of one with the analytic normals."""
import numpy as np
import pytest

import oracle
from paper_2007_07627_amd import binding as B
from paper_2007_07627_amd import metrics, synth

from gpu_common import announce, ctx  # noqa: F401

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [30, 3000, 20000])
def test_normals_equal_oracle(ctx, n):
    Q = synth.bumpy_sphere(synth.rng_for(2, 60), n)[0].astype(np.float32)
    announce(f"normals N={n}")
    g = B.icp_estimate_normals(ctx, Q)
    o = oracle.estimate_normals(Q)
    diff = np.abs(g.astype(np.float64) - o.astype(np.float64)).max(axis=1)
    print(f"bitwise equal {np.mean(diff == 0):.4f}, max diff {diff.max():.3g}", flush=True)
    assert diff.max() < 2e-6


def test_normals_of_a_tilted_plane(ctx):
    g2 = np.stack(np.meshgrid(np.arange(30), np.arange(30), indexing="ij"), -1).reshape(-1, 2) * 0.05
    n0 = np.array([0.3, -0.2, 1.0])
    n0 /= np.linalg.norm(n0)
    a = np.cross(n0, [1.0, 0, 0]); a /= np.linalg.norm(a)
    b = np.cross(n0, a)
    Q = (np.array([0.2, -0.1, 2.0]) + g2[:, :1] * a + g2[:, 1:] * b).astype(np.float32)
    announce("normals tilted plane")
    g = B.icp_estimate_normals(ctx, Q).astype(np.float64)
    assert np.abs(g + n0).max() < 1e-5


def test_point_to_plane_registration_with_estimated_normals(ctx):
    d = synth.height_field_pair(synth.rng_for(3, 61), m=5000, n=20000)
    announce("p2pl registration with estimated normals")
    Qn = B.icp_estimate_normals(ctx, d["Q"])
    prm = B.icp_params_default(B.ICP_P2PL_WELSCH, anderson_m=6, nu_min=d["nu_min"])
    est = B.icp_register(ctx, d["P"], d["Q"], Qn, prm)
    ana = B.icp_register(ctx, d["P"], d["Q"], d["Qn"], prm)
    r_est = metrics.rmse(d["T_gt"], est["T"], d["P"])
    r_ana = metrics.rmse(d["T_gt"], ana["T"], d["P"])
    print(f"rmse estimated {r_est:.3g} analytic {r_ana:.3g}", flush=True)
    assert r_est < 2.0 * r_ana + 1e-3


def test_normals_invalid_arguments(ctx):
    rc, _ = B.icp_estimate_normals(ctx, np.zeros((29, 3), np.float32), raw=True)
    assert rc == B.ICP_ERR_INVALID_ARG
    Q = np.random.default_rng(0).standard_normal((50, 3)).astype(np.float32)
    Q[7, 0] = np.inf
    rc, _ = B.icp_estimate_normals(ctx, Q, raw=True)
    assert rc == B.ICP_ERR_NONFINITE
