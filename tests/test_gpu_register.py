"""Registration parity through the C ABI against the oracle: final transforms
within 1e-5 rad and 1e-5 x bbox diagonal, energies within 1e-6 relative;
plain vs. graph engines and repeated runs bit-identical."""
import numpy as np
import pytest

import oracle
from paper_2007_07627_amd import binding as B
from paper_2007_07627_amd import metrics, synth

from gpu_common import announce, ctx  # noqa: F401

pytestmark = pytest.mark.gpu

ROT_TOL = 1e-5
TR_TOL = 1e-5


def _compare(g, o, diag, tag):
    rot = metrics.rotation_error_rad(g["T"], o["T"])
    tr = metrics.translation_error(g["T"], o["T"])
    print(f"{tag}: rot {rot:.2e} tr {tr:.2e} passes gpu {g['nn_passes']} oracle {o['nn_passes']} "
          f"iters {g['iterations']}/{o['iterations']} E {g['energy']:.9g}/{o['energy']:.9g}", flush=True)
    assert rot <= ROT_TOL and tr <= TR_TOL * diag, (tag, rot, tr)
    assert abs(g["energy"] - o["energy"]) <= 1e-6 * max(1.0, abs(o["energy"])), (tag, g["energy"], o["energy"])


def _fast(seed, n=4096):
    return synth.fast_icp_pair(synth.rng_for(1, seed), n=n)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_fast_icp_config1(ctx, seed):
    d = _fast(seed)
    announce(f"register fast-icp seed={seed}")
    prm = B.icp_params_default(B.ICP_P2P_L2, eps=1e-6, iter_first=50, iter_cap=50, nn=B.ICP_NN_BRUTE)
    g = B.icp_register(ctx, d["P"], d["Q"], None, prm)
    o = oracle.register(d["P"], d["Q"], mode=0, anderson_m=5, eps=1e-6, iter_first=50, iter_cap=50)
    _compare(g, o, d["diag"], f"fast{seed}")
    assert metrics.rmse(d["T_gt"], g["T"], d["P"]) < 5e-3 * d["diag"]


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("nn", [B.ICP_NN_BRUTE, B.ICP_NN_CLUSTER])
def test_robust_p2p_plain_mm(ctx, seed, nn):
    """Algorithm 1 without mixing (m = 0): the trajectory is reproducible, so
    the GPU must land on the oracle's transform."""
    d = synth.partial_sphere_pair(synth.rng_for(2, 100 + seed), m=4000, n=5000)
    announce(f"register robust-p2p m=0 seed={seed} nn={nn}")
    prm = B.icp_params_default(B.ICP_P2P_WELSCH, anderson_m=0, nu_min=d["nu_min"], nn=nn)
    g = B.icp_register(ctx, d["P"], d["Q"], None, prm)
    o = oracle.register(d["P"], d["Q"], mode=1, anderson_m=0, nu_min=d["nu_min"])
    _compare(g, o, d["diag"], f"p2p-mm{seed}")
    assert g["nn_passes"] == o["nn_passes"] and g["iterations"] == o["iterations"]


@pytest.mark.parametrize("mode", [B.ICP_P2P_L2, B.ICP_P2P_WELSCH, B.ICP_P2PL_WELSCH])
def test_map_evaluation_along_oracle_trajectory(ctx, mode):
    """icp_eval (one un-accelerated map application) at transforms taken from
    the oracle's own trajectory: energies to 1e-10 relative, updates to 1e-9."""
    if mode == B.ICP_P2PL_WELSCH:
        d = synth.height_field_pair(synth.rng_for(3, 200), m=3000, n=8000)
        o = oracle.register(d["P"], d["Q"], d["Qn"], mode=2, anderson_m=6, nu_min=d["nu_min"], trace_cap=2000)
    else:
        d = synth.partial_sphere_pair(synth.rng_for(2, 200), m=4000, n=5000)
        o = oracle.register(d["P"], d["Q"], mode=mode, anderson_m=5, nu_min=d["nu_min"], trace_cap=2000,
                            eps=1e-6, iter_first=60, iter_cap=60)
    rows = o["trace"]
    pick = np.unique(np.linspace(0, len(rows) - 1, 12).astype(int))
    announce(f"eval-map mode={mode} rows={len(rows)}")
    for i in pick:
        T = rows[i, 4:20].reshape(4, 4)
        nu = rows[i, 1]
        Eg, Tg, fg = B.icp_eval(ctx, d["P"], d["Q"], d["Qn"], mode, T, nu)
        Eo, To, fo = oracle.eval_map(d["P"], d["Q"], d["Qn"], mode, T, nu)
        assert fg == fo
        assert abs(Eg - Eo) <= 1e-10 * max(1.0, abs(Eo)), (i, Eg, Eo)
        assert abs(Eo - rows[i, 0]) <= 1e-12 * max(1.0, abs(Eo))
        assert metrics.rotation_error_rad(Tg, To) <= 1e-9 and metrics.translation_error(Tg, To) <= 1e-9, i


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_robust_p2pl_small(ctx, seed):
    d = synth.height_field_pair(synth.rng_for(3, 100 + seed), m=3000, n=8000)
    announce(f"register robust-p2pl seed={seed}")
    prm = B.icp_params_default(B.ICP_P2PL_WELSCH, anderson_m=6, nu_min=d["nu_min"])
    g = B.icp_register(ctx, d["P"], d["Q"], d["Qn"], prm)
    o = oracle.register(d["P"], d["Q"], d["Qn"], mode=2, anderson_m=6, nu_min=d["nu_min"])
    _compare(g, o, d["diag"], f"p2pl{seed}")


def test_plain_and_graph_engines_bit_identical(ctx):
    d = synth.partial_sphere_pair(synth.rng_for(2, 7), m=3000, n=3000)
    announce("register engines plain vs graph")
    res = []
    for eng in (B.ICP_ENGINE_GRAPH, B.ICP_ENGINE_PLAIN, B.ICP_ENGINE_GRAPH):
        prm = B.icp_params_default(B.ICP_P2P_WELSCH, nu_min=d["nu_min"], engine=eng)
        res.append(B.icp_register(ctx, d["P"], d["Q"], None, prm))
    for r in res[1:]:
        assert np.array_equal(r["T"], res[0]["T"])
        assert r["nn_passes"] == res[0]["nn_passes"] and r["energy"] == res[0]["energy"]


def test_register_invalid_arguments(ctx):
    P = np.zeros((10, 3), np.float32)
    # nu_min unset selects the automatic rule, which needs 7 targets
    prm = B.icp_params_default(B.ICP_P2P_WELSCH)
    rc, _ = B.icp_register(ctx, P, P[:6], None, prm, raw=True)
    assert rc == B.ICP_ERR_INVALID_ARG
    prm = B.icp_params_default(B.ICP_P2P_WELSCH, nu_min=float("nan"))
    rc, _ = B.icp_register(ctx, P, P, None, prm, raw=True)
    assert rc == B.ICP_ERR_INVALID_ARG
    prm = B.icp_params_default(B.ICP_P2PL_WELSCH, nu_min=1e-3)
    rc, _ = B.icp_register(ctx, P, P, None, prm, raw=True)
    assert rc == B.ICP_ERR_NO_NORMALS
    prm = B.icp_params_default(B.ICP_P2P_L2, anderson_m=7)
    rc, _ = B.icp_register(ctx, P, P, None, prm, raw=True)
    assert rc == B.ICP_ERR_INVALID_ARG
    Pn = P.copy()
    Pn[3, 2] = np.inf
    rc, _ = B.icp_register(ctx, Pn, P, None, B.icp_params_default(B.ICP_P2P_L2), raw=True)
    assert rc == B.ICP_ERR_NONFINITE


def test_repeat_runs_bit_identical(ctx):
    d = synth.height_field_pair(synth.rng_for(3, 9), m=3000, n=6000)
    prm = B.icp_params_default(B.ICP_P2PL_WELSCH, anderson_m=6, nu_min=d["nu_min"])
    a = B.icp_register(ctx, d["P"], d["Q"], d["Qn"], prm)
    b = B.icp_register(ctx, d["P"], d["Q"], d["Qn"], prm)
    assert np.array_equal(a["T"], b["T"]) and a["energy"] == b["energy"]


def test_eval_invalid(ctx):
    P = np.zeros((10, 3), np.float32)
    assert B.icp_eval(ctx, P, P, None, B.ICP_P2P_WELSCH, np.eye(4), 0.0, raw=True) == B.ICP_ERR_INVALID_ARG
    assert B.icp_eval(ctx, P, P, None, B.ICP_P2PL_WELSCH, np.eye(4), 1.0, raw=True) == B.ICP_ERR_NO_NORMALS
