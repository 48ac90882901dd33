"""The allocation-free closest-point query (icp_nn_query_dev_noalloc) against
the device query it is a variant of (icp_nn_query_dev), bit for bit (indices
and FP32 squared distances): two calls in a row on one stream, the second with
a smaller input, for both search methods; the size limit of its fixed working
array is reported as ICP_ERR_OOM before any launch."""
import numpy as np
import pytest
import torch

from paper_2007_07627_amd import binding as B
from paper_2007_07627_amd import synth

from gpu_common import announce, ctx  # noqa: F401

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def _tensors(P, Q):
    return torch.from_numpy(np.ascontiguousarray(P)).to(DEV), torch.from_numpy(np.ascontiguousarray(Q)).to(DEV)


def _outputs(m):
    return (torch.full((m,), -7, dtype=torch.int32, device=DEV),
            torch.full((m,), float("nan"), dtype=torch.float32, device=DEV))


def _motion(seed):
    R, t = synth.random_motion(np.random.default_rng(seed), 20.0, 0.1)
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = t
    return T


@pytest.mark.parametrize("method", [B.ICP_NN_BRUTE, B.ICP_NN_CLUSTER, B.ICP_NN_AUTO])
def test_noalloc_equals_device_query_two_calls(ctx, method):
    stream = torch.cuda.current_stream()
    big = synth.partial_sphere_pair(synth.rng_for(2, 500), m=60_013, n=70_001)
    small = synth.height_field_pair(synth.rng_for(3, 501), m=3_001, n=5_003)
    cases = [(big["P"], big["Q"], _motion(1)), (small["P"], small["Q"], _motion(2))]
    got = []
    for k, (P, Q, T) in enumerate(cases):
        announce(f"noalloc call {k} M={len(P)} N={len(Q)} method={method}")
        Pt, Qt = _tensors(P, Q)
        i0, d0 = _outputs(len(P))
        i1, d1 = _outputs(len(P))
        B.icp_nn_query_dev(ctx, Pt, Qt, T, method, i0, d0, stream)
        B.icp_nn_query_dev_noalloc(Pt, Qt, T, method, i1, d1, stream)
        torch.cuda.synchronize()
        got.append((i0.cpu().numpy(), d0.cpu().numpy(), i1.cpu().numpy(), d1.cpu().numpy()))
    for k, (i0, d0, i1, d1) in enumerate(got):
        assert (i0 >= 0).all(), k
        assert np.array_equal(i0, i1), k
        assert np.array_equal(d0.view(np.uint32), d1.view(np.uint32)), k


def test_noalloc_back_to_back_on_one_stream(ctx):
    """Two queries enqueued before any synchronisation: the second reuses the
    array after the first on the same stream; both equal the device query."""
    stream = torch.cuda.current_stream()
    a = synth.partial_sphere_pair(synth.rng_for(2, 502), m=40_000, n=30_000)
    b = synth.partial_sphere_pair(synth.rng_for(2, 503), m=1_000, n=2_000)
    Pa, Qa = _tensors(a["P"], a["Q"])
    Pb, Qb = _tensors(b["P"], b["Q"])
    ia, da = _outputs(len(a["P"]))
    ib, db = _outputs(len(b["P"]))
    announce("noalloc back to back")
    B.icp_nn_query_dev_noalloc(Pa, Qa, _motion(3), B.ICP_NN_CLUSTER, ia, da, stream)
    B.icp_nn_query_dev_noalloc(Pb, Qb, _motion(4), B.ICP_NN_CLUSTER, ib, db, stream)
    torch.cuda.synchronize()
    for P, Q, T, i, d in ((Pa, Qa, _motion(3), ia, da), (Pb, Qb, _motion(4), ib, db)):
        i0, d0 = _outputs(P.shape[0])
        B.icp_nn_query_dev(ctx, P, Q, T, B.ICP_NN_CLUSTER, i0, d0, stream)
        torch.cuda.synchronize()
        assert torch.equal(i0, i) and torch.equal(d0.view(torch.int32), d.view(torch.int32))


def test_noalloc_size_limit_and_arguments(ctx):
    stream = torch.cuda.current_stream()
    n = 262_144
    d = synth.resampled_sphere_pair(synth.rng_for(2, 504), m=n, n=n)
    Pt, Qt = _tensors(d["P"], d["Q"])
    i1, d1 = _outputs(n)
    announce("noalloc at 262144 x 262144")
    B.icp_nn_query_dev_noalloc(Pt, Qt, np.eye(4), B.ICP_NN_CLUSTER, i1, d1, stream)
    i0, d0 = _outputs(n)
    B.icp_nn_query_dev(ctx, Pt, Qt, np.eye(4), B.ICP_NN_CLUSTER, i0, d0, stream)
    torch.cuda.synchronize()
    assert torch.equal(i0, i1) and torch.equal(d0.view(torch.int32), d1.view(torch.int32))
    big = torch.zeros((500_000, 3), dtype=torch.float32, device=DEV)
    ib, db = _outputs(500_000)
    rc = B.icp_nn_query_dev_noalloc(big, big, np.eye(4), B.ICP_NN_AUTO, ib, db, stream, raw=True)
    assert rc == B.ICP_ERR_OOM
    torch.cuda.synchronize()
    assert (ib == -7).all()  # nothing was launched
    T = np.eye(4)
    T[0, 0] = 1.5
    assert B.icp_nn_query_dev_noalloc(Pt, Qt, T, B.ICP_NN_AUTO, i1, d1, stream, raw=True) == B.ICP_ERR_INVALID_ARG
    assert B.icp_nn_query_dev_noalloc(Pt, Qt, np.eye(4), 7, i1, d1, stream, raw=True) == B.ICP_ERR_INVALID_ARG
