"""Batched serving (meg_server_* of the C ABI): many instances advanced by one
persistent launch, each on its own team of workgroups.

- Parity: each instance's free-running trajectory against the FP64 oracle on
  the matrix its bf16 planes represent, to the mixed-precision tolerance.
- Isolation: an instance's result is bitwise the same alone and in a mix of
  other instances arriving at other times.
- Admission: with an arena too small for everything, requests wait in the
  queue and are admitted as memory frees up; all complete, and never more
  is resident than fits.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import meg_oracle as O
from tests.helpers import TOL_X, gapped_spiked, isolated_linear, rel_x_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def meg():
    from paper_2012_10469_amd import meg as m

    m.load_library()
    return m


def print_case(**kw):
    print("CASE " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def device_f32(M):
    import torch

    return torch.from_numpy(np.ascontiguousarray(M, dtype=np.float32)).cuda()


def drain(srv, rounds=10000):
    for _ in range(rounds):
        if srv.run(1) == 0:
            return
    raise AssertionError("server did not drain")


def test_serving_matches_oracle(meg):
    import torch

    cases = [(256, 2, 3), (320, 1, 2), (520, 3, 5), (200, 1, 1)]  # (n, rank of the signal, r)
    T = 12
    with meg.MegServer(launch_steps=5) as srv:
        ids, refs, keep = [], [], []
        for i, (n, rank, r) in enumerate(cases):
            print_case(test="serving_oracle", n=n, rank=rank, r=r)
            M, V0, lam0 = gapped_spiked(n, rank, seed=40 + i)
            M32 = M.astype(np.float32)
            hi, lo = W.bf16_planes(M32)
            run = O.run_lowrank_meg(O.DenoiseObjective(W.planes_value(hi, lo, n)), V0, lam0, r, 1.0, T)
            dM = device_f32(M32)
            keep.append(dM)
            torch.cuda.synchronize()
            ids.append(srv.submit(dM, V0, lam0, r, max_iters=T, max_inner=30, seed=i))
            refs.append((n, r, run))
        drain(srv)
        for rid, (n, r, run) in zip(ids, refs):
            st = srv.query(rid)
            assert st["state"] == 2 and st["status"] == 0 and st["iterations"] == T, st
            V, d, a = srv.result(rid, n, r)
            err = rel_x_err((V, d, a, T + 1), run["states"][T])
            print(f"  n={n} r={r} team={st['team']} err={err:.2e} L={st['last']['cert_L']:.3f}/{run['L'][-1]:.3f}",
                  flush=True)
            assert err <= TOL_X[2]
            # trace and positivity of the returned iterate
            assert abs(n * a + float(np.sum(d)) - 1.0) <= 1e-6
            assert a > 0 and float(np.min(a + d)) > 0


def _instance(i, n, r):
    M, _, _ = gapped_spiked(n, 1, seed=100 + i)
    w, V = np.linalg.eigh(M)
    return M.astype(np.float32), V[:, -1:].copy(), np.ones(1)


def test_serving_same_alone_and_in_mix(meg):
    """One instance run alone, then again while others of other sizes arrive
    before, with and after it: its iterate, certificate and iteration count
    are bitwise identical."""
    import torch

    n, r, iters = 384, 4, 14
    MA, VA, lA = _instance(0, n, r)
    with meg.MegServer(launch_steps=3) as srv:
        print_case(test="serving_alone", n=n, r=r)
        dA = device_f32(MA)
        torch.cuda.synchronize()
        a_id = srv.submit(dA, VA, lA, r, max_iters=iters, seed=7)
        drain(srv)
        alone = srv.result(a_id, n, r)
        alone_st = srv.query(a_id)

        print_case(test="serving_mix", n=n, r=r)
        others = [(1, 256, 2), (2, 640, 6), (3, 1000, 3), (4, 300, 8), (5, 512, 1)]
        keep = []
        ids = []
        for i, (j, m, rr) in enumerate(others[:2]):
            M, V, l = _instance(j, m, rr)
            keep.append(device_f32(M))
            torch.cuda.synchronize()
            ids.append(srv.submit(keep[-1], V, l, rr, max_iters=9 + j, seed=j))
        srv.run(1)
        b_id = srv.submit(dA, VA, lA, r, max_iters=iters, seed=7)
        srv.run(2)
        for i, (j, m, rr) in enumerate(others[2:]):
            M, V, l = _instance(j, m, rr)
            keep.append(device_f32(M))
            torch.cuda.synchronize()
            ids.append(srv.submit(keep[-1], V, l, rr, max_iters=5 + 3 * j, seed=j))
            srv.run(1)
        drain(srv)
        mixed = srv.result(b_id, n, r)
        mixed_st = srv.query(b_id)
        for rid in ids:
            assert srv.query(rid)["state"] == 2
    assert mixed_st["iterations"] == alone_st["iterations"] == iters
    assert mixed_st["team"] == alone_st["team"]
    assert np.array_equal(alone[0], mixed[0]) and np.array_equal(alone[1], mixed[1]) and alone[2] == mixed[2]
    assert mixed_st["last"]["cert_L"] == alone_st["last"]["cert_L"]


def test_serving_admits_as_memory_frees(meg):
    """An arena with room for two n = 1024 instances: five requests queue up,
    at most two are resident at once, all complete, each with the result it
    has alone."""
    import torch

    n, r = 1024, 3
    with meg.MegServer(launch_steps=4) as probe_srv:
        team = probe_srv.team(n)[1]
    # per-instance block: planes 4 n^2 + blocks and buffers (< 1 MB)
    budget = 2 * (4 * n * n + (1 << 20)) + (1 << 19)
    with meg.MegServer(budget_bytes=budget, launch_steps=4) as srv:
        print_case(test="serving_admission", n=n, team=team, budget=budget)
        keep, ids, specs = [], [], []
        for i in range(5):
            M, V, l = _instance(10 + i, n, r)
            keep.append(device_f32(M))
            specs.append((M, V, l))
        torch.cuda.synchronize()
        for i in range(5):
            ids.append(srv.submit(keep[i], specs[i][1], specs[i][2], r, max_iters=6 + i, seed=i))
        max_res = 0
        while True:
            pend = srv.run(1)
            s = srv.stats()
            max_res = max(max_res, s["resident"])
            assert s["arena_used"] <= s["arena_bytes"]
            if pend == 0:
                break
        assert max_res <= 2
        assert srv.stats()["completed"] == 5
        res = [srv.result(rid, n, r) for rid in ids]
        st = [srv.query(rid) for rid in ids]
        assert all(q["state"] == 2 for q in st)
        assert st[4]["admit_ms"] >= st[0]["done_ms"] or st[4]["admit_ms"] >= st[1]["done_ms"]
    # the last one alone
    with meg.MegServer(launch_steps=4) as srv:
        M, V, l = specs[4]
        dM = device_f32(M)
        torch.cuda.synchronize()
        rid = srv.submit(dM, V, l, r, max_iters=10, seed=4)
        drain(srv)
        alone = srv.result(rid, n, r)
        if srv.query(rid)["team"] == st[4]["team"]:
            assert np.array_equal(alone[0], res[4][0]) and np.array_equal(alone[1], res[4][1])


def test_serving_stop_rule_and_rejects(meg):
    import torch

    n, r = 256, 1
    M, V, l = _instance(20, n, r)
    # the stop rule: a linear instance whose (r+1)-th eigenvalue is isolated,
    # so the certificate resolves (it is claimed only on a resolved pair)
    C, VC, lC = isolated_linear(n, r, seed=20)
    with meg.MegServer(launch_steps=8) as srv:
        dM = device_f32(M)
        dC = device_f32(C)
        torch.cuda.synchronize()
        tol = 1e-3
        rid = srv.submit(dC, VC, lC, r, kind=meg.MEG_GRAD_LINEAR_DENSE, max_iters=300, tol=tol)
        drain(srv)
        st = srv.query(rid)
        print_case(test="serving_stop", iterations=st["iterations"], bound=st["last"]["cert_bound"])
        # 2 eps_t <= 1e-3 from t = 29 on
        assert st["state"] == 2 and 29 <= st["iterations"] < 60
        assert st["last"]["cert_resolved"] == 1 and st["last"]["cert_bound"] <= tol
        assert st["last"]["cert_L"] + st["last"]["resid_r1"] <= tol
        # a spiked instance (noise bulk below lambda_{r+1}): the pair stays
        # unresolved, no certificate is claimed, the request runs to its cap
        rid2 = srv.submit(dM, V, l, r, max_iters=40, tol=tol)
        drain(srv)
        st2 = srv.query(rid2)
        assert st2["state"] == 2 and st2["iterations"] == 40 and st2["last"]["cert_holds"] == 0
        with pytest.raises(meg.MegError) as e:
            srv.submit(dM, V, l, 12)  # k = 32: not served
        assert e.value.status == meg.MEG_ERR_UNSUPPORTED
        with pytest.raises(meg.MegError) as e:
            srv.submit(dM, V, l, r, kind=meg.MEG_GRAD_MASKED_CSR)
        assert e.value.status == meg.MEG_ERR_UNSUPPORTED
        with pytest.raises(meg.MegError) as e:
            srv.submit(dM, V, np.array([0.5]), r)  # weights do not sum to 1
        assert e.value.status == meg.MEG_ERR_INVALID_ARG


def test_serving_graph_replay_matches_direct_launches(meg):
    """Graph mode (one captured round replayed with new tables each time,
    host work between replays) gives bitwise the results of direct
    cooperative launches, for every instance of a mix."""
    import torch

    specs = [(256, 2, 11), (384, 4, 9), (520, 6, 13), (1000, 3, 7), (300, 8, 10)]
    inst = [(_instance(30 + i, n, r), n, r, it) for i, (n, r, it) in enumerate(specs)]
    keep = [device_f32(M) for (M, _, _), _, _, _ in inst]
    torch.cuda.synchronize()
    out = {}
    for graph in (False, True):
        print_case(test="serving_graph", graph=graph)
        with meg.MegServer(launch_steps=2, graph=graph, fixed_team=2) as srv:
            ids = [srv.submit(keep[i], V, l, r, max_iters=it, seed=i)
                   for i, ((M, V, l), n, r, it) in enumerate(inst)]
            rounds = 0
            while srv.run(1) > 0:
                rounds += 1
            assert rounds >= 3  # several replays
            if graph:
                print(f"  graph node: {srv.stats()['graph_node']} (1 cooperative, 2 ordinary)", flush=True)
                assert srv.stats()["graph_node"] in (1, 2)
            out[graph] = [(srv.result(rid, n, r), srv.query(rid)) for rid, (_, n, r, _) in zip(ids, inst)]
    for (ra, sa), (rb, sb) in zip(out[False], out[True]):
        assert sa["iterations"] == sb["iterations"] and sa["team"] == sb["team"] == 2
        assert np.array_equal(ra[0], rb[0]) and np.array_equal(ra[1], rb[1]) and ra[2] == rb[2]
        assert sa["last"]["cert_L"] == sb["last"]["cert_L"]
