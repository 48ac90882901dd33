"""Automatic nu_min (Sec. 4.3 point-to-point, Sec. 5 point-to-plane, App. C)
through the C ABI against the oracle: the GPU's six-nearest-neighbour search
uses the same exact FP32 distances and tie rule and the same medians, so the
values agree bit for bit; a registration with nu_min <= 0 equals the one
given that value explicitly."""
import math

import numpy as np
import pytest

import oracle
from paper_2007_07627_amd import binding as B
from paper_2007_07627_amd import synth

from gpu_common import announce, ctx  # noqa: F401

pytestmark = pytest.mark.gpu


def _lattice(n=40, h=2.0 ** -6):
    g = np.stack(np.meshgrid(np.arange(n) * h, np.arange(n) * h, indexing="ij"), -1).reshape(-1, 2)
    return np.c_[g, np.zeros(len(g))].astype(np.float32), h


@pytest.mark.parametrize("n", [7, 300, 3000, 30000])
def test_point_to_point_equals_oracle(ctx, n):
    Q = synth.bumpy_sphere(synth.rng_for(2, 50), n)[0].astype(np.float32)
    announce(f"nu_min auto p2p N={n}")
    g = B.icp_nu_min_auto(ctx, Q, None, B.ICP_P2P_WELSCH)
    o = oracle.nu_min_auto(Q, None, oracle.P2P_WELSCH)
    assert g == o, (g, o)


@pytest.mark.parametrize("n", [500, 20000])
def test_point_to_plane_equals_oracle(ctx, n):
    d = synth.height_field_pair(synth.rng_for(3, 51), m=1000, n=n)
    announce(f"nu_min auto p2pl N={n}")
    g = B.icp_nu_min_auto(ctx, d["Q"], d["Qn"], B.ICP_P2PL_WELSCH)
    o = oracle.nu_min_auto(d["Q"], d["Qn"], oracle.P2PL_WELSCH)
    assert g == o, (g, o)


def test_lattices_ties_and_duplicates(ctx):
    """Square lattice (ties among the diagonals), the same with every point
    twice (duplicates at distance 0), and the lifted lattice for the
    point-to-plane rule: the closed forms of the oracle pins, on the GPU."""
    Q, h = _lattice()
    announce("nu_min auto lattices")
    assert B.icp_nu_min_auto(ctx, Q, None, B.ICP_P2P_WELSCH) == h / (3.0 * math.sqrt(3.0))
    assert B.icp_nu_min_auto(ctx, np.concatenate([Q, Q]), None, B.ICP_P2P_WELSCH) == h / (3.0 * math.sqrt(3.0))
    a = 2.0 ** -14
    Ql = Q.copy()
    Ql[(np.arange(len(Q)) % 40) % 2 == 1, 2] = a
    Qn = np.tile(np.float32([0, 0, 1]), (len(Q), 1))
    assert B.icp_nu_min_auto(ctx, Ql, Qn, B.ICP_P2PL_WELSCH) == a / 6.0


def test_far_outliers_and_clusters_far_apart(ctx):
    """Two dense blobs far apart plus isolated far points: the search must
    reach clusters well away along the curve for the isolated points."""
    rng = np.random.default_rng(52)
    A = rng.standard_normal((2000, 3)) * 0.01
    Bb = rng.standard_normal((2000, 3)) * 0.01 + 50.0
    far = rng.uniform(-100, 100, (40, 3))
    Q = np.concatenate([A, far, Bb]).astype(np.float32)
    announce("nu_min auto blobs + far points")
    assert B.icp_nu_min_auto(ctx, Q, None, B.ICP_P2P_WELSCH) == oracle.nu_min_auto(Q, None, oracle.P2P_WELSCH)


def test_registration_with_automatic_nu_min_equals_explicit(ctx):
    d = synth.partial_sphere_pair(synth.rng_for(2, 53), m=5000, n=5000)
    nu = B.icp_nu_min_auto(ctx, d["Q"], None, B.ICP_P2P_WELSCH)
    announce(f"registration nu_min auto vs explicit {nu}")
    a = B.icp_register(ctx, d["P"], d["Q"], None, B.icp_params_default(B.ICP_P2P_WELSCH, nu_min=0.0))
    b = B.icp_register(ctx, d["P"], d["Q"], None, B.icp_params_default(B.ICP_P2P_WELSCH, nu_min=nu))
    assert np.array_equal(a["T"], b["T"]) and a["nn_passes"] == b["nn_passes"]
    assert a["nu_final"] == nu
    h = synth.height_field_pair(synth.rng_for(3, 53), m=3000, n=6000)
    nu = B.icp_nu_min_auto(ctx, h["Q"], h["Qn"], B.ICP_P2PL_WELSCH)
    a = B.icp_register(ctx, h["P"], h["Q"], h["Qn"],
                       B.icp_params_default(B.ICP_P2PL_WELSCH, anderson_m=6, nu_min=-1.0))
    b = B.icp_register(ctx, h["P"], h["Q"], h["Qn"],
                       B.icp_params_default(B.ICP_P2PL_WELSCH, anderson_m=6, nu_min=nu))
    assert np.array_equal(a["T"], b["T"]) and a["nn_passes"] == b["nn_passes"]


def test_invalid_arguments(ctx):
    Q = np.zeros((6, 3), np.float32)
    rc, _ = B.icp_nu_min_auto(ctx, Q, None, B.ICP_P2P_WELSCH, raw=True)
    assert rc == B.ICP_ERR_INVALID_ARG
    Q = np.random.default_rng(0).standard_normal((50, 3)).astype(np.float32)
    rc, _ = B.icp_nu_min_auto(ctx, Q, None, B.ICP_P2PL_WELSCH, raw=True)
    assert rc == B.ICP_ERR_NO_NORMALS
    rc, _ = B.icp_nu_min_auto(ctx, Q, None, B.ICP_P2P_L2, raw=True)
    assert rc == B.ICP_ERR_INVALID_ARG
    Qb = Q.copy()
    Qb[3, 1] = np.nan
    rc, _ = B.icp_nu_min_auto(ctx, Qb, None, B.ICP_P2P_WELSCH, raw=True)
    assert rc == B.ICP_ERR_NONFINITE
    # a registration asking for the automatic rule with too few targets
    with pytest.raises(B.ICPError):
        B.icp_register(ctx, Q, Q[:6], None, B.icp_params_default(B.ICP_P2P_WELSCH, nu_min=0.0))
