"""Edge cases of the step against the FP64 oracle: the block as large as the
space (n = k = 16, so Rayleigh-Ritz is exact), an empty sampling pattern
(G = 0: the step only renormalises the top r eigenvalues of log X_t), and a
pattern with empty rows (ragged CSR)."""
import numpy as np
import pytest

import workloads as W
from oracle import meg_oracle as O
from tests.helpers import TOL_X, f_tol, gapped_spiked, make_csr, make_dense, rel_x_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def meg():
    from paper_2012_10469_amd import meg as m

    m.load_library()
    return m


def print_case(**kw):
    print("CASE " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


@pytest.mark.parametrize("n,rank", [(16, 3), (17, 1)])
def test_block_as_large_as_the_space(meg, n, rank):
    """k = roundup16(r + 1 + 4) = 16 >= n - 1: the subspace is (nearly) all
    of R^n, the free-running trajectory matches the oracle's."""
    print_case(test="whole_space", n=n, rank=rank)
    M, V0, lam0 = gapped_spiked(n, rank, seed=900 + n)
    T = 6
    run = O.run_lowrank_meg(O.DenoiseObjective(M), V0, lam0, rank, 1.0, T)
    with make_dense(M, meg.MEG_GRAD_DENOISE_DENSE, V0, lam0, rank, 0, eta=1.0, max_inner=40) as g:
        assert g.k == 16
        for t in range(1, T + 1):
            info = g.step()
            err = rel_x_err(g.get_iterate(), run["states"][t])
            print(f"  t={t} err={err:.2e} sweeps={info['inner_iters']} gap={run['gap'][t - 1]:.3e}", flush=True)
            assert err <= TOL_X[0], (t, err)


def _csr_problem(n, rp, col, val, V0, lam0):
    return W.CSRProblem("masked", n, np.asarray(rp, np.int32), np.asarray(col, np.int32),
                        np.asarray(val, np.float32), V0, lam0)


def test_empty_pattern(meg):
    """nnz = 0: the gradient vanishes and X_{t+1} keeps V_t with the weights
    (1 - eps_t) softmax(log(alpha + d)) (Definition 1 with M_t = log X_t)."""
    n, r = 64, 2
    print_case(test="empty_pattern", n=n, r=r)
    rng = np.random.default_rng([91, n])
    V0 = np.linalg.qr(rng.standard_normal((n, r)))[0]
    lam0 = np.array([0.7, 0.3])
    p = _csr_problem(n, np.zeros(n + 1), np.zeros(0), np.zeros(0), V0, lam0)
    obj = O.MaskedObjective(n, p.row_ptr, p.col, p.val.astype(np.float64))
    T = 4
    run = O.run_lowrank_meg(obj, V0, lam0, r, 1.0, T)
    with make_csr(p, meg.MEG_GRAD_MASKED_CSR, r, 1, eta=1.0, max_inner=20) as g:
        for t in range(1, T + 1):
            info = g.step()
            err = rel_x_err(g.get_iterate(), run["states"][t])
            print(f"  t={t} err={err:.2e} f={info['f']:.3e} sweeps={info['inner_iters']}", flush=True)
            assert info["f"] == 0.0
            assert err <= TOL_X[1], (t, err)


@pytest.mark.parametrize("cache", [True, False])
def test_pattern_with_empty_rows(meg, cache):
    """Rows (and, by symmetry, columns) 0..19 carry no samples; teacher-forced
    steps against the oracle, with the sparse data in LDS or read from memory."""
    n, r = 200, 3
    print_case(test="empty_rows", n=n, r=r, cache=cache)
    p = W.matrix_completion(n, seed=13, rank=3, p=0.2, r=r, dtype=np.float32)
    rows = np.repeat(np.arange(n), np.diff(p.row_ptr))
    keep = (rows >= 20) & (p.col >= 20)
    rows, col, val = rows[keep], p.col[keep], p.val[keep]
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, rows + 1, 1)
    q = _csr_problem(n, np.cumsum(rp), col, val, p.V0, p.lam0)
    assert np.all(np.diff(q.row_ptr)[:20] == 0)
    obj = O.MaskedObjective(n, q.row_ptr, q.col, q.val.astype(np.float64))
    T = 5
    run = O.run_lowrank_meg(obj, q.V0, q.lam0, r, 1.0, T)
    flags = 0 if cache else meg.MEG_FLAG_NO_LDS_CACHE
    checked = 0
    with make_csr(q, meg.MEG_GRAD_MASKED_CSR, r, 1, eta=1.0, max_inner=40, flags=flags) as g:
        for t in range(1, T + 1):
            st = run["states"][t - 1]
            g.set_iterate(st.V, st.d, st.alpha, t)
            info = g.step()
            mu = run["mu"][t - 1]
            rel_gap = run["gap"][t - 1] / max(1.0, abs(mu[0] - mu[-1]))
            err = rel_x_err(g.get_iterate(), run["states"][t])
            f_ref = obj.value(st.dense())
            print(f"  t={t} err={err:.2e} relgap={rel_gap:.2e} f={info['f']:.6e}/{f_ref:.6e}", flush=True)
            X = st.dense()
            assert abs(info["f"] - f_ref) <= f_tol(f_ref, np.linalg.norm(obj.grad(X)), np.linalg.norm(X), 1)
            if rel_gap < 1e-3:
                continue
            checked += 1
            assert err <= TOL_X[1], (t, err)
    assert checked >= 3
