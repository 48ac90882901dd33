"""Numerical-outcome flags against the oracle (they are flags, not errors):
ZERO_WEIGHT when every Welsch weight underflows (nu far below the residuals),
DEGENERATE when the alignment or the 6x6 Gauss-Newton system is rank
deficient (collinear sources; planar sources against a plane), AA_SINGULAR
when the Anderson least-squares columns are linearly dependent (an iteration
confined to one axis)."""
import numpy as np
import pytest

import oracle
from paper_2007_07627_amd import binding as B
from paper_2007_07627_amd import synth

from gpu_common import announce, ctx  # noqa: F401

pytestmark = pytest.mark.gpu

H = 1.0 / 16.0


def _grid(nx, ny):
    """Dyadic planar grid symmetric about the origin (every coordinate, sum and
    product below is exact in FP32 / FP64)."""
    kx = (np.arange(nx) - (nx - 1) / 2) * H
    ky = (np.arange(ny) - (ny - 1) / 2) * H
    X, Y = np.meshgrid(kx, ky, indexing="ij")
    return np.c_[X.ravel(), Y.ravel(), np.zeros(X.size)].astype(np.float32)


@pytest.mark.parametrize("mode", [B.ICP_P2P_WELSCH, B.ICP_P2PL_WELSCH])
def test_zero_weight(ctx, mode):
    if mode == B.ICP_P2PL_WELSCH:
        d = synth.height_field_pair(synth.rng_for(3, 300), m=2000, n=4000)
    else:
        d = synth.partial_sphere_pair(synth.rng_for(2, 300), m=2000, n=3000)
    nu = 1e-9 * d["diag"]
    Qn = d["Qn"] if mode == B.ICP_P2PL_WELSCH else None
    announce(f"flags zero weight mode={mode}")
    g = B.icp_register(ctx, d["P"], d["Q"], Qn, B.icp_params_default(mode, nu_max=nu, nu_min=nu))
    o = oracle.register(d["P"], d["Q"], Qn, mode=int(mode), nu_max=nu, nu_min=nu,
                        anderson_m=6 if mode == B.ICP_P2PL_WELSCH else 5)
    assert g["status_flags"] & B.ICP_FLAG_ZERO_WEIGHT and o["flags"] & oracle.FLAG_ZERO_WEIGHT
    assert g["status_flags"] == o["flags"]
    assert np.abs(g["T"] - o["T"]).max() <= 1e-15
    assert g["energy"] == o["energy"] == float(len(d["P"]))  # psi = 1 at every source
    assert g["iterations"] == o["iterations"] == 0


def test_degenerate_plane_against_plane(ctx):
    """Sources and targets in the plane z = 0, normals +z: rotations about z and
    translations in x, y leave every B_i unchanged, so the Gauss-Newton system
    is singular at the first evaluation and the registration stops at T0."""
    Q = _grid(40, 40)
    Qn = np.tile(np.float32([0, 0, 1]), (len(Q), 1))
    P = _grid(20, 20) + np.float32([3 * H, -5 * H, 0])
    announce("flags degenerate p2pl plane")
    prm = B.icp_params_default(B.ICP_P2PL_WELSCH, nu_max=1.0, nu_min=1e-3)
    g = B.icp_register(ctx, P, Q, Qn, prm)
    o = oracle.register(P, Q, Qn, mode=oracle.P2PL_WELSCH, anderson_m=6, nu_max=1.0, nu_min=1e-3)
    assert g["status_flags"] & B.ICP_FLAG_DEGENERATE and o["flags"] & oracle.FLAG_DEGENERATE
    assert g["status_flags"] == o["flags"]
    assert np.array_equal(g["T"], np.eye(4)) and np.array_equal(o["T"], np.eye(4))
    # with the 3 x median rule every initial residual is 0, so nu_max = 0 and
    # no weight is defined: both report ZERO_WEIGHT and return T0
    prm = B.icp_params_default(B.ICP_P2PL_WELSCH, nu_min=1e-3)
    g = B.icp_register(ctx, P, Q, Qn, prm)
    o = oracle.register(P, Q, Qn, mode=oracle.P2PL_WELSCH, anderson_m=6, nu_min=1e-3)
    assert o["flags"] & oracle.FLAG_ZERO_WEIGHT and g["status_flags"] == o["flags"]
    assert np.array_equal(g["T"], np.eye(4)) and np.array_equal(o["T"], np.eye(4))


def test_degenerate_collinear_alignment(ctx):
    """Every source matched to one column of targets: the weighted cross
    covariance has rank one and the rotation about that line is not
    determined. Both raise the flag (the rotation each picks is not compared:
    several are optimal)."""
    Q = _grid(32, 32)
    P = _grid(8, 32)
    P[:, 0] += np.float32(40.125 * H)
    announce("flags degenerate p2p collinear")
    prm = B.icp_params_default(B.ICP_P2P_L2, eps=1e-9, iter_first=3, iter_cap=3, nn=B.ICP_NN_BRUTE)
    g = B.icp_register(ctx, P, Q, None, prm)
    o = oracle.register(P, Q, mode=oracle.P2P_L2, anderson_m=5, eps=1e-9, iter_first=3, iter_cap=3)
    assert g["status_flags"] & B.ICP_FLAG_DEGENERATE and o["flags"] & oracle.FLAG_DEGENERATE


def test_aa_singular_one_axis_iteration(ctx):
    """A symmetric dyadic grid shifted along x: the cross covariance stays
    diagonal, every update is a pure x translation, so all Anderson columns
    are parallel and the least-squares system is singular from its second
    column on (theta = 0 is used). Exact arithmetic throughout: both land on
    the same transform after the same iterations."""
    Q = _grid(32, 32)
    P = _grid(32, 32)
    P[:, 0] += np.float32(20.375 * H)
    announce("flags aa singular")
    prm = B.icp_params_default(B.ICP_P2P_L2, eps=1e-9, iter_first=100, iter_cap=100, nn=B.ICP_NN_BRUTE)
    g = B.icp_register(ctx, P, Q, None, prm)
    o = oracle.register(P, Q, mode=oracle.P2P_L2, anderson_m=5, eps=1e-9, iter_first=100, iter_cap=100)
    assert o["flags"] & oracle.FLAG_AA_SINGULAR and o["flags"] & oracle.FLAG_CONVERGED
    assert g["status_flags"] == o["flags"]
    assert g["iterations"] == o["iterations"] and g["nn_passes"] == o["nn_passes"]
    assert np.abs(g["T"] - o["T"]).max() <= 1e-12
    assert np.array_equal(o["T"][:3, :3], np.eye(3)) and o["T"][1, 3] == 0.0 == o["T"][2, 3]
