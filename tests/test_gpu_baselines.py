"""The comparison methods of Sec. 6 with their App. E settings through the C
ABI against the oracle: classical ICP (point-to-point, L2, no mixing) and
ICP-l (point-to-plane, L2, Gauss-Newton with unit weights), both stopping at
1000 iterations or ||dT||_F^2 < 1e-5. Without mixing the trajectory is
reproducible, so the GPU takes the oracle's steps: same iteration and pass
counts, transforms to 1e-9 along the trace."""
import numpy as np
import pytest

import oracle
from paper_2007_07627_amd import binding as B
from paper_2007_07627_amd import metrics, synth

from gpu_common import announce, ctx  # noqa: F401

pytestmark = pytest.mark.gpu


def _run_both(ctx, d, mode, nn=B.ICP_NN_AUTO, **kw):
    Qn = d["Qn"] if mode == B.ICP_P2PL_L2 else None
    prm = B.icp_params_classical(mode, nn=nn, **kw)
    g = B.icp_register_trace(ctx, d["P"], d["Q"], Qn, prm, cap=4000)
    o = oracle.register(d["P"], d["Q"], Qn, params=oracle.classical_params(mode), trace_cap=4000, **kw)
    print(f"mode {mode}: iters {g['iterations']}/{o['iterations']} passes {g['nn_passes']}/{o['nn_passes']} "
          f"E {g['energy']:.12g}/{o['energy']:.12g} flags {g['status_flags']}/{o['flags']}", flush=True)
    return g, o


def _check_trajectory(g, o, diag):
    assert g["iterations"] == o["iterations"] and g["nn_passes"] == o["nn_passes"]
    assert g["status_flags"] == o["flags"]
    gt, ot = g["trace"], o["trace"]
    assert gt[:, :20].shape == ot.shape
    assert np.abs(gt[:, 4:20] - ot[:, 4:20]).max() < 1e-9
    assert np.all(np.abs(gt[:, 0] - ot[:, 0]) <= 1e-9 * np.maximum(1.0, np.abs(ot[:, 0])))
    assert metrics.rotation_error_rad(g["T"], o["T"]) <= 1e-9
    assert metrics.translation_error(g["T"], o["T"]) <= 1e-9 * diag
    assert abs(g["energy"] - o["energy"]) <= 1e-9 * max(1.0, abs(o["energy"]))
    assert g["nu_final"] == 0.0 and g["stages"] == 1


@pytest.mark.parametrize("seed", [0, 1])
@pytest.mark.parametrize("nn", [B.ICP_NN_BRUTE, B.ICP_NN_CLUSTER])
def test_classical_icp_matches_oracle(ctx, seed, nn):
    d = synth.partial_sphere_pair(synth.rng_for(2, 300 + seed), m=4000, n=5000)
    announce(f"classical ICP seed={seed} nn={nn}")
    g, o = _run_both(ctx, d, B.ICP_P2P_L2, nn=nn)
    _check_trajectory(g, o, d["diag"])


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("nn", [B.ICP_NN_BRUTE, B.ICP_NN_CLUSTER])
def test_icp_l_matches_oracle(ctx, seed, nn):
    d = synth.height_field_pair(synth.rng_for(3, 300 + seed), m=3000, n=8000)
    announce(f"ICP-l seed={seed} nn={nn}")
    g, o = _run_both(ctx, d, B.ICP_P2PL_L2, nn=nn)
    _check_trajectory(g, o, d["diag"])
    assert g["status_flags"] & B.ICP_FLAG_CONVERGED


def test_icp_l_iteration_cap_and_tight_threshold(ctx):
    """A cap that ends the run (MAX_ITER, cap + 2 passes) and a threshold so
    tight that the run goes to a full fixed point on noise-free data."""
    d = synth.height_field_pair(synth.rng_for(3, 310), m=2000, n=6000)
    announce("ICP-l cap 8")
    g, o = _run_both(ctx, d, B.ICP_P2PL_L2, eps=1e-300, iter_first=8, iter_cap=8)
    _check_trajectory(g, o, d["diag"])
    assert g["iterations"] == 8 and g["nn_passes"] == 10 and g["status_flags"] & B.ICP_FLAG_MAX_ITER
    h = synth.height_field_pair(synth.rng_for(3, 311), m=3000, n=3000, outliers=0.0, noise=0.0,
                                max_angle=3.0, trans_frac=0.01)
    R, t = synth.random_motion(synth.rng_for(3, 312), 3.0, 0.02)
    P = (h["Q"].astype(np.float64) @ R.T + t).astype(np.float32)
    Tgt = np.eye(4)
    Tgt[:3, :3] = R.T
    Tgt[:3, 3] = -R.T @ t
    announce("ICP-l noise-free exact recovery")
    g = B.icp_register(ctx, P, h["Q"], h["Qn"], B.icp_params_classical(B.ICP_P2PL_L2, eps=1e-10))
    assert metrics.rotation_error_rad(g["T"], Tgt) < 1e-6 and metrics.translation_error(g["T"], Tgt) < 1e-6


def test_icp_l_map_along_oracle_trajectory(ctx):
    """icp_eval in the ICP-l mode at the oracle's transforms: energy sum B^2
    to 1e-10 relative and the Gauss-Newton update to 1e-9."""
    d = synth.height_field_pair(synth.rng_for(3, 320), m=3000, n=8000)
    o = oracle.register(d["P"], d["Q"], d["Qn"], params=oracle.classical_params(oracle.P2PL_L2), trace_cap=2000)
    rows = o["trace"]
    announce(f"ICP-l eval-map rows={len(rows)}")
    for i in np.unique(np.linspace(0, len(rows) - 1, 10).astype(int)):
        T = rows[i, 4:20].reshape(4, 4)
        Eg, Tg, fg = B.icp_eval(ctx, d["P"], d["Q"], d["Qn"], B.ICP_P2PL_L2, T)
        Eo, To, fo = oracle.eval_map(d["P"], d["Q"], d["Qn"], oracle.P2PL_L2, T)
        assert fg == fo
        assert abs(Eg - Eo) <= 1e-10 * max(1.0, abs(Eo)), (i, Eg, Eo)
        assert metrics.rotation_error_rad(Tg, To) <= 1e-9 and metrics.translation_error(Tg, To) <= 1e-9, i


def test_baselines_in_a_batch_equal_alone(ctx):
    reqs = []
    for s in range(3):
        h = synth.height_field_pair(synth.rng_for(3, 330 + s), m=2000 + 500 * s, n=5000)
        reqs.append((h["P"], h["Q"], h["Qn"], B.icp_params_classical(B.ICP_P2PL_L2)))
        p = synth.partial_sphere_pair(synth.rng_for(2, 330 + s), m=3000, n=3000 + 700 * s)
        reqs.append((p["P"], p["Q"], None, B.icp_params_classical(B.ICP_P2P_L2)))
    announce("baselines batch of 6")
    tickets = B.icp_batch_submit(ctx, reqs)
    B.icp_batch_wait_all(ctx)
    for t, (P, Q, Qn, prm) in zip(tickets, reqs):
        rc, g = B.icp_poll(ctx, t)
        assert rc == B.ICP_OK
        a = B.icp_register(ctx, P, Q, Qn, prm)
        assert np.array_equal(g["T"], a["T"]) and g["nn_passes"] == a["nn_passes"]


def test_icp_l_needs_normals(ctx):
    P = np.random.default_rng(0).standard_normal((50, 3)).astype(np.float32)
    rc, _ = B.icp_register(ctx, P, P, None, B.icp_params_classical(B.ICP_P2PL_L2), raw=True)
    assert rc == B.ICP_ERR_NO_NORMALS
    rc = B.icp_eval(ctx, P, P, None, B.ICP_P2PL_L2, np.eye(4), raw=True)
    assert rc == B.ICP_ERR_NO_NORMALS
