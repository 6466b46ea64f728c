"""External gradient (meg_step_external of the C ABI): the caller supplies
G_t at the current iterate every step, dense or CSR, and the step takes its
shift from Gershgorin bounds of that G_t.

Teacher-forced against the FP64 oracle: from the GPU's own X_t the test forms
G_t on the host (denoising: X_t - M, dense; matrix completion:
P_Omega_t(X_t - M) / p on a sampling pattern drawn afresh every step, sent as
CSR or as a dense matrix on alternate steps), rounds it to the state's
precision and uploads it; the oracle takes the step (Algorithm 2) from the
same X_t with the same rounded G_t.  Compared per step: X_{t+1} (relative
Frobenius error), the certificate, and the shift, which must bound
eta lambda_max(G_t) from above and follow the Gershgorin rule.
"""
import math

import numpy as np
import pytest

from oracle import meg_oracle as O
from tests.helpers import TOL_X, check_certificate, dev, gapped_spiked, np_dtype, rel_x_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def meg():
    from paper_2012_10469_amd import meg as m

    m.load_library()
    return m


def print_case(**kw):
    print("CASE " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def gersh_sigma(G, eta, it, r):
    """The shift the step must use: eta times the largest Gershgorin bound of
    G, minus the most negative log-eigenvalue offset of X_t, plus the
    documented relative allowance."""
    off = np.sum(np.abs(G), axis=1) - np.abs(np.diag(G))
    gmax = float(np.max(np.diag(G) + off))
    c_it = np.log(it.alpha + it.d[:r]) - math.log(it.alpha)
    cmin = min(0.0, float(np.min(c_it)))
    cmax = max(0.0, float(np.max(c_it)))
    base = eta * gmax - cmin
    return base + 1e-3 * (abs(base) + cmax), cmin


def check_shift(info, G, eta, it, r):
    sig_ref, cmin = gersh_sigma(G, eta, it, r)
    lmax = float(np.linalg.eigvalsh(G)[-1])
    assert info["sigma"] >= eta * lmax - cmin - 1e-9 * abs(eta * lmax), (info["sigma"], eta * lmax - cmin)
    assert info["sigma"] == pytest.approx(sig_ref, rel=1e-6), (info["sigma"], sig_ref)


def csr_of(G):
    """CSR (int32 indices) of the nonzeros of G, rows in order, columns sorted."""
    rows, cols = np.nonzero(G)
    rp = np.zeros(G.shape[0] + 1, dtype=np.int64)
    np.add.at(rp, rows + 1, 1)
    return np.cumsum(rp).astype(np.int32), cols.astype(np.int32), G[rows, cols]


@pytest.mark.parametrize("prec,n,rank", [(0, 96, 2), (1, 300, 3), (1, 257, 1)])
def test_external_dense_denoising(meg, prec, n, rank):
    print_case(test="external_dense", prec=prec, n=n, rank=rank)
    M, V0, lam0 = gapped_spiked(n, rank, seed=500 + n)
    eta, T = 1.0, 6
    g = meg.LowRankMEG(n, rank, meg.MEG_GRAD_EXTERNAL, V0, lam0, prec=prec, eta=eta, max_inner=60,
                       cert_tol=1e-9 if prec == 0 else 1e-5)
    try:
        for t in range(1, T + 1):
            V, d, a, tt = g.get_iterate()
            assert tt == t
            it = O.FactoredIterate(V, d, a, t)
            Gq = (it.dense() - M).astype(np_dtype(prec)).astype(np.float64)
            ref, ri = O.lowrank_step(it, Gq, eta, O.eps_schedule(t), rank)
            info = g.step_external(dense=dev(Gq.astype(np_dtype(prec))))
            err = rel_x_err(g.get_iterate(), ref)
            print(f"  t={t} err={err:.2e} gap={ri['gap']:.3f} sweeps={info['inner_iters']} "
                  f"sigma={info['sigma']:.4f} L={info['cert_L']:.4e}/{ri['L']:.4e}", flush=True)
            assert info["t"] == t and math.isnan(info["f"])
            check_shift(info, Gq, eta, it, rank)
            check_certificate(info, ri["L"], O.eps_schedule(t), prec)
            assert err <= TOL_X[prec]
    finally:
        g.close()


@pytest.mark.parametrize("prec,n,rank,p", [(1, 257, 2, 0.3), (0, 128, 1, 0.5)])
def test_external_masked_changing_pattern(meg, prec, n, rank, p):
    """Matrix completion with a new sampling pattern every step (the
    stochastic use of an external gradient): odd steps send G_t as CSR, even
    steps as a dense matrix, so the operator family changes between steps."""
    import torch

    print_case(test="external_masked", prec=prec, n=n, rank=rank, p=p)
    M, V0, lam0 = gapped_spiked(n, rank, seed=600 + n)
    eta, T = 0.5, 6
    rng = np.random.default_rng([61, n])
    g = meg.LowRankMEG(n, rank, meg.MEG_GRAD_EXTERNAL, V0, lam0, prec=prec, eta=eta, max_inner=60,
                       cert_tol=1e-9 if prec == 0 else 1e-5)
    try:
        for t in range(1, T + 1):
            V, d, a, tt = g.get_iterate()
            it = O.FactoredIterate(V, d, a, t)
            up = np.triu(rng.random((n, n)) < p)
            mask = up | up.T
            Gq = np.where(mask, (it.dense() - M) / p, 0.0).astype(np_dtype(prec)).astype(np.float64)
            ref, ri = O.lowrank_step(it, Gq, eta, O.eps_schedule(t), rank)
            if t % 2:
                rp, col, val = csr_of(Gq)
                keep = (dev(rp), dev(col), dev(val.astype(np_dtype(prec))))
                torch.cuda.synchronize()
                info = g.step_external(row_ptr=keep[0], col=keep[1], val=keep[2])
            else:
                dG = dev(Gq.astype(np_dtype(prec)))
                torch.cuda.synchronize()
                info = g.step_external(dense=dG)
            err = rel_x_err(g.get_iterate(), ref)
            print(f"  t={t} {'csr' if t % 2 else 'dense'} nnz={int(np.count_nonzero(Gq))} err={err:.2e} "
                  f"gap={ri['gap']:.3f} sweeps={info['inner_iters']} sigma={info['sigma']:.4f}", flush=True)
            check_shift(info, Gq, eta, it, rank)
            check_certificate(info, ri["L"], O.eps_schedule(t), prec)
            assert err <= TOL_X[prec]
    finally:
        g.close()


def test_external_rejects(meg):
    """meg_step / meg_solve are refused on an external context; a CSR gradient
    with a column out of range is refused before any kernel reads through it,
    and the context still steps afterwards."""
    import torch

    n, rank = 64, 1
    M, V0, lam0 = gapped_spiked(n, rank, seed=7)
    print_case(test="external_rejects", n=n)
    g = meg.LowRankMEG(n, rank, meg.MEG_GRAD_EXTERNAL, V0, lam0, eta=1.0, max_inner=30)
    try:
        with pytest.raises(meg.MegError) as e:
            g.step()
        assert e.value.status == meg.MEG_ERR_INVALID_ARG
        with pytest.raises(meg.MegError) as e:
            g.solve(3)
        assert e.value.status == meg.MEG_ERR_INVALID_ARG
        with pytest.raises(meg.MegError) as e:
            g.profile_step()
        assert e.value.status == meg.MEG_ERR_INVALID_ARG
        with pytest.raises(meg.MegError) as e:
            g.objective()
        assert e.value.status == meg.MEG_ERR_UNSUPPORTED
        with pytest.raises(meg.MegError) as e:  # a dense G_t with ld < n
            g.step_external(dense=dev(np.zeros((n, n - 1), dtype=np.float32)))
        assert e.value.status == meg.MEG_ERR_INVALID_ARG
        G = np.eye(n, dtype=np.float32)
        rp, col, val = csr_of(G)
        col[5] = n  # one past the last column
        bad = (dev(rp), dev(col), dev(val))
        torch.cuda.synchronize()
        with pytest.raises(meg.MegError) as e:
            g.step_external(row_ptr=bad[0], col=bad[1], val=bad[2])
        assert e.value.status == meg.MEG_ERR_INVALID_ARG
        V, d, a, t = g.get_iterate()
        assert t == 1
        it = O.FactoredIterate(V, d, a, 1)
        Gq = (it.dense() - M).astype(np.float32)
        info = g.step_external(dense=dev(Gq))
        ref, _ = O.lowrank_step(it, Gq.astype(np.float64), 1.0, O.eps_schedule(1), rank)
        assert info["t"] == 1 and rel_x_err(g.get_iterate(), ref) <= TOL_X[1]
    finally:
        g.close()
