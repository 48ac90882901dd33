"""The autotuner's work partition never changes a result: registrations under
extreme tuned values are bit-identical to the defaults (one-slot cluster and
exhaustive searches, the batch engine's exhaustive items); the table lookup
follows its bucket rules; a search stores a winner for its bucket."""
import numpy as np
import pytest

from paper_2007_07627_amd import binding as B
from paper_2007_07627_amd import synth

from gpu_common import announce

pytestmark = pytest.mark.gpu

EXTREMES = [dict(slice_min=1, list_margin=0.0, brute_clusters=1, brute_items=64, grid_per_cu=1),
            dict(slice_min=64, list_margin=1.0, brute_clusters=4096, brute_items=1 << 20, grid_per_cu=64),
            dict(slice_min=3, list_margin=0.3, brute_clusters=3, brute_items=1000, grid_per_cu=5)]


def _bucket(n):
    return int(n).bit_length() - 1


@pytest.fixture
def fresh():
    h = B.icp_create(0, 4 << 30)
    yield h
    B.icp_destroy(h)


@pytest.fixture
def empty(monkeypatch, tmp_path):
    """A context whose tuning table starts empty (no cache file to load)."""
    monkeypatch.setenv("ICP_TUNING_CACHE", str(tmp_path / "absent.json"))
    h = B.icp_create(0, 4 << 30)
    yield h
    B.icp_destroy(h)


def _set_all(ctx, M, N, mode, method, t):
    for fam in (B.ICP_P2P_WELSCH, B.ICP_P2PL_WELSCH):
        for batch in (0, 1):
            B.icp_tuning_set(ctx, B.make_entry(_bucket(M), _bucket(N), fam, method, batch=batch, **t))


@pytest.mark.parametrize("case", ["cluster-p2p", "cluster-p2pl", "brute-l2"])
def test_tuned_values_do_not_change_results(fresh, case):
    if case == "cluster-p2p":
        d = synth.partial_sphere_pair(synth.rng_for(2, 600), m=20_000, n=30_000)
        prm = B.icp_params_default(B.ICP_P2P_WELSCH, nu_min=d["nu_min"], nn=B.ICP_NN_CLUSTER)
        Qn, method = None, B.ICP_NN_CLUSTER
    elif case == "cluster-p2pl":
        d = synth.height_field_pair(synth.rng_for(3, 600), m=15_000, n=40_000)
        prm = B.icp_params_default(B.ICP_P2PL_WELSCH, anderson_m=6, nu_min=d["nu_min"], nn=B.ICP_NN_CLUSTER)
        Qn, method = d["Qn"], B.ICP_NN_CLUSTER
    else:
        d = synth.fast_icp_pair(synth.rng_for(1, 600))
        prm = B.icp_params_default(B.ICP_P2P_L2, eps=1e-6, iter_first=50, iter_cap=50, nn=B.ICP_NN_BRUTE)
        Qn, method = None, B.ICP_NN_BRUTE
    announce(f"tuning invariance {case}")
    ref = B.icp_register(fresh, d["P"], d["Q"], Qn, prm)
    for t in EXTREMES:
        _set_all(fresh, len(d["P"]), len(d["Q"]), prm.mode, method, t)
        got, found = B.icp_tuning_lookup(fresh, len(d["P"]), len(d["Q"]), prm.mode, method)
        assert found == 2 and got["slice_min"] == t["slice_min"] and got["grid_per_cu"] == t["grid_per_cu"]
        g = B.icp_register(fresh, d["P"], d["Q"], Qn, prm)
        assert np.array_equal(g["T"], ref["T"]), t
        assert g["nn_passes"] == ref["nn_passes"] and g["energy"] == ref["energy"]
        idx0, d20 = B.icp_nn_query(fresh, d["P"], d["Q"], d["T_gt"], method)
        B.icp_tuning_set(fresh, B.make_entry(_bucket(len(d["P"])), _bucket(len(d["Q"])), B.ICP_P2P_WELSCH,
                                             method))
        idx1, d21 = B.icp_nn_query(fresh, d["P"], d["Q"], d["T_gt"], method)
        assert np.array_equal(idx0, idx1) and np.array_equal(d20.view(np.uint32), d21.view(np.uint32))


def test_batch_exhaustive_items_do_not_change_results(fresh):
    reqs = []
    for i, (m, n) in enumerate([(3000, 2500), (1200, 4000), (4096, 4096)]):
        d = synth.fast_icp_pair(synth.rng_for(41, 60 + i), n=max(m, n))
        P, Q = np.ascontiguousarray(d["P"][:m]), np.ascontiguousarray(d["Q"][:n])
        reqs.append((P, Q, None, B.icp_params_default(B.ICP_P2P_WELSCH, nu_min=1e-3, nn=B.ICP_NN_BRUTE)))
    announce("tuning invariance batch exhaustive items")
    alone = [B.icp_register(fresh, *r) for r in reqs]
    for cpi in (1, 5, 4096):
        for P, Q, _, prm in reqs:
            _set_all(fresh, len(P), len(Q), prm.mode, B.ICP_NN_BRUTE, dict(brute_clusters=cpi))
        tk = B.icp_batch_submit(fresh, reqs)
        B.icp_batch_wait_all(fresh)
        for t, a in zip(tk, alone):
            rc, g = B.icp_poll(fresh, t)
            assert rc == B.ICP_OK and np.array_equal(g["T"], a["T"]), cpi


def test_lookup_rules_and_validation(empty):
    fresh = empty
    assert B.icp_tuning_entries(fresh) == []
    d0 = B.icp_tuning_default()
    t, f = B.icp_tuning_lookup(fresh, 100_000, 100_000, B.ICP_P2P_WELSCH, B.ICP_NN_CLUSTER)
    assert f in (0, 1, 2)
    B.icp_tuning_set(fresh, B.make_entry(10, 10, B.ICP_P2P_WELSCH, B.ICP_NN_CLUSTER, slice_min=9))
    t, f = B.icp_tuning_lookup(fresh, 1 << 10, (1 << 11) - 1, B.ICP_P2P_L2, B.ICP_NN_CLUSTER)
    assert f == 2 and t["slice_min"] == 9          # same bucket, same point-to-point family
    t, f = B.icp_tuning_lookup(fresh, 1 << 11, 1 << 11, B.ICP_P2P_WELSCH, B.ICP_NN_CLUSTER)
    assert f == 1 and t["slice_min"] == 9          # two octaves away
    t, f = B.icp_tuning_lookup(fresh, 1 << 12, 1 << 11, B.ICP_P2P_WELSCH, B.ICP_NN_CLUSTER)
    assert f == 0 and t == d0                      # three octaves: defaults
    t, f = B.icp_tuning_lookup(fresh, 1 << 10, 1 << 10, B.ICP_P2PL_WELSCH, B.ICP_NN_CLUSTER)
    assert f == 0                                  # other family
    t, f = B.icp_tuning_lookup(fresh, 1 << 10, 1 << 10, B.ICP_P2P_WELSCH, B.ICP_NN_CLUSTER, batch=1)
    assert f == 0 and t == d0                      # the batch engine's kind is separate
    bad = B.make_entry(10, 10, B.ICP_P2P_WELSCH, B.ICP_NN_CLUSTER, grid_per_cu=0)
    assert B.icp_tuning_set(fresh, bad, raw=True) == B.ICP_ERR_INVALID_ARG
    assert B.icp_device_arch(0).startswith("gfx")


@pytest.mark.parametrize("M,N,mode,method,batch", [(20_000, 20_000, B.ICP_P2P_WELSCH, B.ICP_NN_CLUSTER, 0),
                                                   (20_000, 20_000, B.ICP_P2P_WELSCH, B.ICP_NN_CLUSTER, 1),
                                                   (2048, 3000, B.ICP_P2PL_WELSCH, B.ICP_NN_BRUTE, 0),
                                                   (2048, 3000, B.ICP_P2PL_WELSCH, B.ICP_NN_BRUTE, 1)])
def test_autotune_stores_a_winner(empty, M, N, mode, method, batch):
    fresh = empty
    announce(f"autotune M={M} N={N} mode={mode} method={method} batch={batch}")
    e = B.icp_autotune(fresh, M, N, mode, method, batch)
    assert e.m_bucket == _bucket(M) and e.n_bucket == _bucket(N) and e.method == method and e.ms > 0
    assert e.batch == batch
    t, f = B.icp_tuning_lookup(fresh, M, N, mode, method, batch)
    assert f == 2 and t == B.tuning_dict(e.tuning)
    t, f = B.icp_tuning_lookup(fresh, M, N, mode, method, 1 - batch)
    assert f == 0
    print(B.entry_dict(e), flush=True)
