"""The two readings of the step and exact MEG on the GPU.

- Dual-averaging reading (MEG_FLAG_DUAL_AVERAGE, the accumulate-forever form):
  against its oracle (run_lowrank_meg_dual_average), equal to the paper's
  form (Algorithm 2) for linear f with a start on eigenvectors of C, and
  measurably different from it for denoising from a start off M's
  eigenvectors.
- Exact MEG (Algorithm 1, meg_exact_*): its dense iterates against the
  oracle's run_exact_meg, and the Bregman distance B(W_t, X_t) between the
  exact and the low-rank iterates (the experiments' comparison of the two
  methods) against the oracle's trajectories.
"""
import math

import numpy as np
import pytest

from oracle import meg_oracle as O
from tests.helpers import TOL_X, dev, f_tol, make_dense, np_dtype, rel_x_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def meg():
    from paper_2012_10469_amd import meg as m

    m.load_library()
    return m


def print_case(**kw):
    print("CASE " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def linear_on_eigvecs(n, r, seed):
    rng = np.random.default_rng([90, seed, n])
    Q, R = np.linalg.qr(rng.standard_normal((n, n)))
    Q = Q * np.sign(np.diag(R))
    c = np.concatenate([np.sort(rng.random(r)), 4.0 + np.sort(rng.random(n - r))])
    C = (Q * c) @ Q.T
    lam0 = rng.random(r) + 0.3
    return 0.5 * (C + C.T), Q[:, :r].copy(), lam0 / lam0.sum()


def denoise_off_eigvecs(n, seed):
    """M = U diag(2, 1.6) U^T + noise, start on a perturbation of U (off M's
    eigenvectors, where the two readings part)."""
    rng = np.random.default_rng([91, seed, n])
    U, _ = np.linalg.qr(rng.standard_normal((n, 2)))
    G = rng.standard_normal((n, n))
    M = (U * np.array([2.0, 1.6])) @ U.T + 0.01 * (G + G.T) / math.sqrt(2 * n)
    V0, _ = np.linalg.qr(U + 0.3 * rng.standard_normal((n, 2)))
    return 0.5 * (M + M.T), V0, np.array([0.5, 0.5])


@pytest.mark.parametrize("prec,n,r", [(0, 120, 3), (1, 300, 4)])
def test_dual_average_equals_algorithm2_for_linear_aligned(meg, prec, n, r):
    print_case(test="da_linear", prec=prec, n=n, r=r)
    C, V0, lam0 = linear_on_eigvecs(n, r, seed=n)
    Cq = C.astype(np_dtype(prec)).astype(np.float64)
    T = 8
    run = O.run_lowrank_meg(O.LinearObjective(Cq), V0, lam0, r, 0.8, T)
    kw = dict(eta=0.8, max_inner=40)
    with make_dense(Cq, meg.MEG_GRAD_LINEAR_DENSE, V0, lam0, r, prec, flags=meg.MEG_FLAG_DUAL_AVERAGE, **kw) as a, \
            make_dense(Cq, meg.MEG_GRAD_LINEAR_DENSE, V0, lam0, r, prec, **kw) as b:
        for t in range(1, T + 1):
            ia = a.step()
            b.step()
            ea = rel_x_err(a.get_iterate(), run["states"][t])
            eb = rel_x_err(b.get_iterate(), run["states"][t])
            print(f"  t={t} dual-average {ea:.2e} paper form {eb:.2e} sweeps {ia['inner_iters']}", flush=True)
            assert ea <= TOL_X[prec] and eb <= TOL_X[prec]
            X = run["states"][t - 1].dense()
            assert ia["t"] == t
            assert abs(ia["f"] - run["f"][t - 1]) <= f_tol(run["f"][t - 1], np.linalg.norm(Cq), np.linalg.norm(X), prec)


@pytest.mark.parametrize("prec,n", [(0, 100), (1, 240)])
def test_dual_average_denoising_follows_its_oracle_not_algorithm2(meg, prec, n):
    print_case(test="da_denoise", prec=prec, n=n)
    M, V0, lam0 = denoise_off_eigvecs(n, seed=n)
    Mq = M.astype(np_dtype(prec)).astype(np.float64)
    obj = O.DenoiseObjective(Mq)
    T = 8
    da = O.run_lowrank_meg_dual_average(obj, V0, lam0, 2, 1.0, T)
    pf = O.run_lowrank_meg(obj, V0, lam0, 2, 1.0, T)
    apart = 0.0
    with make_dense(Mq, meg.MEG_GRAD_DENOISE_DENSE, V0, lam0, 2, prec, eta=1.0, max_inner=64,
                    flags=meg.MEG_FLAG_DUAL_AVERAGE) as g:
        for t in range(1, T + 1):
            info = g.step()
            st = g.get_iterate()
            err = rel_x_err(st, da["states"][t])
            other = rel_x_err(st, pf["states"][t])
            apart = max(apart, other)
            print(f"  t={t} vs its oracle {err:.2e}, vs Algorithm 2 {other:.2e}, sweeps {info['inner_iters']}",
                  flush=True)
            assert err <= TOL_X[prec]
            X = da["states"][t - 1].dense()
            assert abs(info["f"] - da["f"][t - 1]) <= f_tol(da["f"][t - 1], np.linalg.norm(X - Mq), np.linalg.norm(X),
                                                            prec)
    assert apart > 1e-2  # the readings differ far beyond the tolerance


def test_dual_average_rejects_unsupported_uses(meg):
    n, r = 64, 2
    C, V0, lam0 = linear_on_eigvecs(n, r, seed=3)
    with make_dense(C, meg.MEG_GRAD_LINEAR_DENSE, V0, lam0, r, 0, flags=meg.MEG_FLAG_DUAL_AVERAGE) as g:
        g.step(info=False)
        with pytest.raises(meg.MegError) as e:
            g.certificate_bound()
        assert e.value.status == meg.MEG_ERR_UNSUPPORTED


@pytest.mark.parametrize("kind,n", [("denoise", 160), ("linear", 96)])
def test_exact_meg_matches_the_oracle(meg, kind, n):
    print_case(test="exact_meg", kind=kind, n=n)
    if kind == "denoise":
        M, V0, lam0 = denoise_off_eigvecs(n, seed=7)
        obj, k = O.DenoiseObjective(M), meg.MEG_GRAD_DENOISE_DENSE
    else:
        M, V0, lam0 = linear_on_eigvecs(n, 3, seed=7)
        obj, k = O.LinearObjective(M), meg.MEG_GRAD_LINEAR_DENSE
    # linear: eta 0.3 keeps the spectrum of W_t within e^-20 of its top over
    # 12 steps (the oracle takes matrix logarithms of W_t)
    T, eta = 12, (1.0 if kind == "denoise" else 0.3)
    W1 = O.initial_iterate(V0, lam0, O.eps_schedule(0)).dense()
    ref = O.run_exact_meg(obj, W1, eta, T)
    with meg.ExactMEG(n, k, V0, lam0, dev(M), eta=eta) as h:
        W, t = h.get()
        assert t == 1 and np.abs(W - W1).max() <= 1e-15
        for t in range(1, T + 1):
            info = h.step()
            W, tt = h.get()
            err = np.linalg.norm(W - ref[t]) / np.linalg.norm(ref[t])
            print(f"  t={t} rel err {err:.2e} tr {np.trace(W):.15f}", flush=True)
            assert tt == t + 1 and info["t"] == t
            assert err <= 1e-10
            assert abs(info["f"] - obj.value(ref[t - 1])) <= 1e-10 * (1.0 + abs(obj.value(ref[t - 1])))
            assert np.trace(W) == pytest.approx(1.0, abs=1e-13)


def test_exact_and_lowrank_bregman_distance(meg):
    """B(W_t, X_t) between the exact and the low-rank iterates, both on the
    GPU from the same W_1 = X_1, against the oracle's two trajectories."""
    n, r = 200, 2
    print_case(test="exact_vs_lowrank", n=n, r=r)
    M, V0, lam0 = denoise_off_eigvecs(n, seed=11)
    obj = O.DenoiseObjective(M)
    T = 10
    W1 = O.initial_iterate(V0, lam0, O.eps_schedule(0)).dense()
    ex = O.run_exact_meg(obj, W1, 1.0, T)
    lr = O.run_lowrank_meg(obj, V0, lam0, r, 1.0, T)
    with meg.ExactMEG(n, meg.MEG_GRAD_DENOISE_DENSE, V0, lam0, dev(M)) as h, \
            make_dense(M, meg.MEG_GRAD_DENOISE_DENSE, V0, lam0, r, 0, eta=1.0, max_inner=40) as g:
        for t in range(1, T + 2):
            V, d, a, tt = g.get_iterate()
            B = h.bregman(V, d, a)
            Bref = O.bregman(ex[t - 1], lr["states"][t - 1].dense())
            print(f"  t={t} B(W_t, X_t) {B:.10e} / oracle {Bref:.10e}", flush=True)
            assert tt == t
            assert abs(B - Bref) <= 1e-9 + 1e-6 * abs(Bref)
            if t <= T:
                h.step()
                g.step(info=False)
