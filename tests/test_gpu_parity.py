"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Iterates are compared as matrices X = alpha I + V diag(d) V^T (relative
Frobenius error), never as eigenvectors, which are defined only up to sign and
rotation.  Tolerances: 1e-5 (FP32 state), 1e-9 (FP64 state); objective 1e-6
relative plus the first-order effect of rounding X to the working precision.
Steps whose oracle eigen-gap mu_r - mu_{r+1} is too small for the top-r
subspace to be determined to that accuracy are compared on what is unique
there (the certificate and the objective) and logged.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import meg_oracle as O
from tests.helpers import (TOL_CERT, TOL_X, check_certificate, dev, f_tol, gapped_spiked, isolated_linear, make_csr,
                           make_dense, np_dtype, rel_x_err)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def meg():
    from paper_2012_10469_amd import meg as m

    m.load_library()
    return m


def print_case(**kw):
    print("CASE " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def linear_instance(n, r, seed, gap=4.0):
    rng = np.random.default_rng([77, seed, n])
    Q, R = np.linalg.qr(rng.standard_normal((n, n)))
    Q = Q * np.sign(np.diag(R))
    c = np.concatenate([np.sort(rng.random(r)), [gap], gap + 0.5 + np.sort(rng.random(n - r - 1))])
    C = (Q * c) @ Q.T
    C = 0.5 * (C + C.T)
    lam0 = rng.random(r) + 0.3
    lam0 /= lam0.sum()
    return C, Q[:, :r].copy(), lam0


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec,n,r", [(0, 64, 3), (1, 300, 5), (1, 257, 1), (0, 200, 12)])
def test_linear_dense_trajectory(meg, prec, n, r):
    print_case(test="linear_dense", prec=prec, n=n, r=r)
    C, V0, lam0 = linear_instance(n, r, seed=n)
    Cq = C.astype(np_dtype(prec)).astype(np.float64)
    eta, T = 0.8, 8
    run = O.run_lowrank_meg(O.LinearObjective(Cq), V0, lam0, r, eta, T)
    # the (r+1)-th eigenvalue is separated here: it is always iterated to
    # cert_tol, so the certificate is resolved every step and must match
    cert_tol = 1e-9 if prec == 0 else 1e-5
    with make_dense(Cq, meg.MEG_GRAD_LINEAR_DENSE, V0, lam0, r, prec, eta=eta, max_inner=60,
                    cert_tol=cert_tol) as g:
        for t in range(1, T + 1):
            info = g.step()
            assert info["t"] == t
            st = g.get_iterate()
            assert st[3] == t + 1
            err = rel_x_err(st, run["states"][t])
            assert err <= TOL_X[prec], (t, err)
            assert info["cert_resolved"] == 1
            check_certificate(info, run["L"][t - 1], run["eps"][t - 1], prec)
            assert info["eps_t"] == pytest.approx(O.eps_schedule(t), rel=1e-14)
            X = run["states"][t - 1].dense()
            tol = f_tol(run["f"][t - 1], np.linalg.norm(Cq), np.linalg.norm(X), prec)
            assert abs(info["f"] - run["f"][t - 1]) <= tol


@pytest.mark.parametrize("prec,n,rank", [(0, 200, 1), (1, 200, 1), (1, 333, 3), (0, 96, 3)])
def test_denoise_gapped_free_running(meg, prec, n, rank):
    print_case(test="denoise_gapped", prec=prec, n=n, rank=rank)
    M, V0, lam0 = gapped_spiked(n, rank, seed=n + rank)
    Mq = M.astype(np_dtype(prec)).astype(np.float64)
    T = 30
    obj = O.DenoiseObjective(Mq)
    run = O.run_lowrank_meg(obj, V0, lam0, rank, 1.0, T)
    worst = 0.0
    resolved = 0
    # lambda_{r+1} of M_t sits at the top of the noise bulk, where its Ritz
    # pair does not resolve; the certificate is claimed on the deflated
    # Lanczos bound of mu_{r+1}, armed before every step
    with make_dense(Mq, meg.MEG_GRAD_DENOISE_DENSE, V0, lam0, rank, prec, eta=1.0, max_inner=20) as g:
        for t in range(1, T + 1):
            bnd = g.certificate_bound(max_steps=n, tol=1e-10)
            assert bnd["t"] == t
            mu_ref = run["mu"][t - 1][rank]
            assert bnd["mu_up"] >= mu_ref - 1e-9 * (1.0 + abs(mu_ref)), (t, bnd, mu_ref)
            info = g.step()
            assert info["mu_r1_up"] == bnd["mu_up"] or info["cert_resolved"]
            st = g.get_iterate()
            err = rel_x_err(st, run["states"][t])
            worst = max(worst, err)
            assert err <= TOL_X[prec], (t, err)
            X = run["states"][t - 1].dense()
            tol = f_tol(run["f"][t - 1], np.linalg.norm(X - Mq), np.linalg.norm(X), prec)
            assert abs(info["f"] - run["f"][t - 1]) <= tol, (t, info["f"], run["f"][t - 1])
            # strictly complementary instance: the certificate holds on both
            # sides (the default resolves the (r+1)-th pair whenever its lower
            # bound of L could hold, and claims only on L + residual <= 2 eps)
            L_ref, e_ref = run["L"][t - 1], run["eps"][t - 1]
            check_certificate(info, L_ref, e_ref, prec)
            resolved += info["cert_resolved"]
            # the bound is sharp here: the certificate is claimed where the
            # oracle's holds with a margin
            if L_ref <= 2 * e_ref - 1e-3:
                assert info["cert_holds"] == 1, (t, info["cert_L_up"], L_ref, e_ref)
            print(f"  t={t} sweeps={info['inner_iters']} resolved={info['cert_resolved']} holds={info['cert_holds']} "
                  f"L={info['cert_L']:.5f}/{L_ref:.5f} up={info['cert_L_up']:.5f} lz={bnd['steps']}", flush=True)
    print(f"worst rel X error {worst:.3e}, resolved {resolved}/{T}")


@pytest.mark.parametrize("n,ld,rank,r", [(304, 312, 1, 1), (520, 520, 3, 3), (264, 264, 2, 16)])
def test_denoise_bf16x3_planes(meg, n, ld, rank, r):
    """Matrix-core form: M given as bf16 planes hi + lo (row length ld), the
    apply on three bf16 MFMA products with FP32 accumulation.  The oracle runs
    on the matrix the planes represent.  Teacher-forced steps: f(X_t) and
    X_{t+1} against the oracle's step from the same X_t; then a free-running
    trajectory.  Tolerance: the mixed-precision bound 1e-3."""
    import torch

    print_case(test="bf16x3", n=n, ld=ld, rank=rank, r=r)
    M, V0, lam0 = gapped_spiked(n, rank, seed=n + 7 * rank)
    hi, lo = W.bf16_planes(M.astype(np.float32), ld)
    Meff = W.planes_value(hi, lo, n)
    obj = O.DenoiseObjective(Meff)
    T = 12  # the start has q = rank columns; the solver fills the rest of r
    run = O.run_lowrank_meg(obj, V0, lam0, r, 1.0, T)
    dh = torch.from_numpy(hi.view(np.int16)).cuda()
    dl = torch.from_numpy(lo.view(np.int16)).cuda()
    kw = dict(prec=meg.MEG_PREC_F32_BF16X3, eta=1.0, dense=dh, dense_lo=dl, max_inner=30)
    with meg.LowRankMEG(n, r, meg.MEG_GRAD_DENOISE_DENSE, V0, lam0, **kw) as g:
        for t in range(1, T + 1):
            st = run["states"][t - 1]
            g.set_iterate(st.V, st.d, st.alpha, t)
            info = g.step()
            X = st.dense()
            tol = f_tol(run["f"][t - 1], np.linalg.norm(X - Meff), np.linalg.norm(X), 2)
            assert abs(info["f"] - run["f"][t - 1]) <= tol, (t, info["f"], run["f"][t - 1])
            err = rel_x_err(g.get_iterate(), run["states"][t])
            assert err <= TOL_X[2], (t, err)
            check_certificate(info, run["L"][t - 1], run["eps"][t - 1], 2)
    worst = 0.0
    with meg.LowRankMEG(n, r, meg.MEG_GRAD_DENOISE_DENSE, V0, lam0, **kw) as g:
        for t in range(1, T + 1):
            g.step(info=False)
            worst = max(worst, rel_x_err(g.get_iterate(), run["states"][t]))
    print(f"free-running worst rel X error {worst:.2e}")
    assert worst <= TOL_X[2]


@pytest.mark.parametrize("prec,n,r", [(1, 500, 10), (0, 300, 6), (1, 96, 3)])
def test_masked_csr_teacher_forced(meg, prec, n, r):
    print_case(test="masked_csr_tf", prec=prec, n=n, r=r)
    p = W.matrix_completion(n, seed=3, rank=min(5, r), p=0.1, r=r, dtype=np_dtype(prec))
    obj = O.MaskedObjective(n, p.row_ptr, p.col, p.val.astype(np.float64))
    T = 8
    run = O.run_lowrank_meg(obj, p.V0, p.lam0, r, 1.0, T)
    checked = 0
    with make_csr(p, meg.MEG_GRAD_MASKED_CSR, r, prec, eta=1.0, max_inner=40) as g:
        for t in range(1, T + 1):
            st = run["states"][t - 1]
            g.set_iterate(st.V, st.d, st.alpha, t)
            info = g.step()
            X = st.dense()
            G = obj.grad(X)
            tol = f_tol(run["f"][t - 1], np.linalg.norm(G), np.linalg.norm(X), prec)
            assert abs(info["f"] - run["f"][t - 1]) <= tol, (t, info["f"], run["f"][t - 1])
            mu = run["mu"][t - 1]
            rel_gap = run["gap"][t - 1] / max(1.0, abs(mu[0] - mu[-1]))
            err = rel_x_err(g.get_iterate(), run["states"][t])
            print(f"t={t} gap={run['gap'][t-1]:.3e} relgap={rel_gap:.2e} inner={info['inner_iters']} "
                  f"conv={info['converged']} err={err:.2e} L={info['cert_L']:.4f}/{run['L'][t-1]:.4f}")
            check_certificate(info, run["L"][t - 1], run["eps"][t - 1], prec)
            if rel_gap < 1e-3:
                continue
            checked += 1
            assert err <= TOL_X[prec], (t, err)
    assert checked >= T // 2


def test_linear_csr_permuted_diagonal(meg):
    n, r = 1000, 4
    print_case(test="linear_csr_diag", n=n, r=r)
    p, c = W.linear_csr_diag(n, r, seed=5, dtype=np.float32)
    C = np.diag(c)
    T = 10
    run = O.run_lowrank_meg(O.LinearObjective(C), p.V0, p.lam0, r, 0.9, T)
    with make_csr(p, meg.MEG_GRAD_LINEAR_CSR, r, 1, eta=0.9, max_inner=30) as g:
        for t in range(1, T + 1):
            info = g.step()
            err = rel_x_err(g.get_iterate(), run["states"][t])
            assert err <= TOL_X[1], (t, err)
            # lambda_{r+1} sits in a cluster of n - r values on [4, 5] (times
            # eta): unresolved, cert_L is a lower bound and nothing is claimed
            check_certificate(info, run["L"][t - 1], run["eps"][t - 1], 1)


def test_resume_and_batched_launch_bitwise(meg):
    """Six single-step launches equal one six-step launch bit for bit, and a
    saved state resumes bit for bit (reductions have a fixed order)."""
    n, r = 256, 4
    print_case(test="resume_batched", n=n, r=r)
    p = W.matrix_completion(n, seed=11, rank=3, p=0.2, r=r)

    def fresh():
        return make_csr(p, meg.MEG_GRAD_MASKED_CSR, r, 1, eta=1.0)

    with fresh() as a, fresh() as b:
        for _ in range(6):
            a.step(info=False)
        b.solve(6)
        Va, da, aa, ta = a.get_iterate()
        Vb, db, ab, tb = b.get_iterate()
        assert ta == tb == 7
        assert np.array_equal(Va, Vb) and np.array_equal(da, db) and aa == ab
        # work counters: same work either way, one launch vs six
        ca, cb = a.counters(), b.counters(reset=True)
        assert (ca["launches"], cb["launches"]) == (6, 1)
        assert ca["iterations"] == cb["iterations"] == 6
        assert ca["applies"] == cb["applies"] and 6 <= ca["applies"] <= 6 * 64
        assert ca["jacobi_sweeps"] == cb["jacobi_sweeps"] > 0
        assert ca["extrapolated"] == cb["extrapolated"] and ca["unconverged"] == cb["unconverged"]
        assert ca["kernel_ms"] > 0 and cb["kernel_ms"] > 0
        assert b.counters() == {"launches": 0, "iterations": 0, "applies": 0, "workgroups": cb["workgroups"],
                                "jacobi_sweeps": 0, "kernel_ms": 0.0, "extrapolated": 0, "unconverged": 0}
        blob = a.get_state()
        for _ in range(3):
            a.step(info=False)
        Va2, da2, aa2, ta2 = a.get_iterate()
    with fresh() as c:
        c.set_state(blob)
        for _ in range(3):
            c.step(info=False)
        Vc, dc, ac, tc = c.get_iterate()
    assert tc == ta2 == 10
    assert np.array_equal(Va2, Vc) and np.array_equal(da2, dc) and aa2 == ac


@pytest.mark.parametrize("prec,n,r,p_obs", [(1, 700, 6, 0.1), (0, 300, 4, 0.3)])
def test_csr_lds_cache_is_bitwise_neutral(meg, prec, n, r, p_obs):
    """The per-workgroup LDS copy of the CSR data changes where the data is
    read from, not the arithmetic: iterates and certificates are bitwise equal
    with and without it, over several launches of several iterations."""
    print_case(test="lds_cache", prec=prec, n=n, r=r)
    p = W.matrix_completion(n, seed=21, rank=3, p=p_obs, r=r, dtype=np_dtype(prec))
    with make_csr(p, meg.MEG_GRAD_MASKED_CSR, r, prec, eta=1.0) as a, \
            make_csr(p, meg.MEG_GRAD_MASKED_CSR, r, prec, eta=1.0, flags=meg.MEG_FLAG_NO_LDS_CACHE) as b:
        for _ in range(3):
            la, lb = a.solve(5), b.solve(5)
            assert la["cert_L"] == lb["cert_L"] and la["inner_iters"] == lb["inner_iters"]
        fa, fb = a.objective(), b.objective()
        Va, da, aa, ta = a.get_iterate()
        Vb, db, ab, tb = b.get_iterate()
    assert ta == tb == 16
    assert np.array_equal(Va, Vb) and np.array_equal(da, db) and aa == ab and fa == fb


def test_solve_stops_on_certificate(meg):
    """meg_solve stops at the first step whose resolved certificate bound is
    <= tol, on an instance whose (r+1)-th eigenvalue is isolated (so its
    Ritz pair resolves within a few sweeps)."""
    n, r = 200, 2
    print_case(test="solve", n=n)
    C, V0, lam0 = isolated_linear(n, r, seed=9)
    run = O.run_lowrank_meg(O.LinearObjective(C.astype(np.float32).astype(np.float64)), V0, lam0, r, 1.0, 30)
    with make_dense(C.astype(np.float32), meg.MEG_GRAD_LINEAR_DENSE, V0, lam0, r, 1) as g:
        last = g.solve(200, tol=2e-3)
        # bound = max(2 eps_t, L_t) <= 2e-3 needs eps_t <= 1e-3, i.e. t >= 18;
        # the oracle's certificate holds by then
        assert all(L <= 2e-3 for L in run["L"][17:])
        assert last["cert_resolved"] == 1
        assert last["cert_bound"] <= 2e-3
        # the stop acts on the upper bound of the exact L
        assert last["cert_L"] + last["resid_r1"] <= 2e-3
        assert last["t"] == 18
        t_after = g.get_iterate()[3]
        assert t_after == last["t"] + 1
        info = g.step()  # continues normally after a stopped solve
        assert info["t"] == t_after


def test_invalid_state_blob(meg):
    n = 64
    M, V0, lam0 = gapped_spiked(n, 1, seed=1)
    with make_dense(M.astype(np.float32), meg.MEG_GRAD_DENOISE_DENSE, V0, lam0, 1, 1) as g:
        blob = g.get_state()
        with pytest.raises(meg.MegError):
            g.set_state(blob[:-8])
        bad = bytearray(blob)
        bad[0] ^= 0xFF
        with pytest.raises(meg.MegError):
            g.set_state(bytes(bad))
        g.set_state(blob)
        g.step()
