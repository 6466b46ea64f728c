"""The full-trace certificate (meg_trace_exp, meg_certificate_full) against the
FP64 oracle.

Every case sets an iterate the oracle built (initial iterate and oracle steps,
uploaded with meg_set_iterate), so the oracle's M_t = log X_t - eta grad f(X_t)
is formed from its own state.  With the n canonical basis vectors as probes
and weight 1 the deflated estimate is exactly tr exp(M_t) (any deflation
basis), which makes a deterministic parity case: log b against log of the sum
of exp of the oracle's eigenvalues, within 1e-9 (FP64 state) or 1e-5 (FP32
state: the basis and the gradient values are rounded to FP32).  Gaussian
probes are checked statistically, with fixed seeds: the estimate lies within
5 of its own standard errors of the exact value.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import meg_oracle as O
from tests.helpers import gapped_spiked, make_csr, make_dense, np_dtype

pytestmark = pytest.mark.gpu

TOL = {0: 1e-9, 1: 1e-5, 2: 1e-5}


@pytest.fixture(scope="module")
def meg():
    from paper_2012_10469_amd import meg as m

    m.load_library()
    return m


def print_case(**kw):
    print("CASE " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def oracle_iterate(obj, V0, lam0, r, eta, steps):
    """X_1 from the start, then `steps` oracle iterations."""
    it = O.initial_iterate(V0, lam0, O.eps_schedule(0))
    for _ in range(steps):
        it, _ = O.lowrank_step(it, obj.grad(it.dense()), eta, O.eps_schedule(it.t), r, full=False)
    return it


def oracle_mt(it, obj, eta):
    return it.log_dense() - eta * O.sym(obj.grad(it.dense()))


def canonical(g, n, max_steps=128):
    import torch

    probes = torch.eye(n, dtype=torch.float64, device="cuda")
    return g.trace_exp(probes, weight=1.0, max_steps=max_steps, tol=1e-12)


def check_canonical(g, it, obj, eta, prec, label):
    g.set_iterate(it.V, it.d, it.alpha, it.t)
    Mt = oracle_mt(it, obj, eta)
    exact = O.logsumexp(np.linalg.eigvalsh(Mt))
    info, tr = canonical(g, it.n)
    print(f"  {label} t={it.t}: log_b={info['log_b']:.12f} exact={exact:.12f} defl={info['log_b_defl']:.6f} "
          f"tail={info['log_b_tail']:.6f} kd={info['kd']} steps={info['steps']} batches={info['batches']} "
          f"conv={info['converged']}", flush=True)
    assert info["t"] == it.t
    assert info["converged"] == 1
    assert abs(info["log_b"] - exact) <= TOL[prec]
    # the deflated part alone is a lower bound (exp(M_t) is positive definite)
    assert info["log_b_defl"] <= exact + TOL[prec]
    return info, tr


def test_trace_linear_dense_f64(meg):
    prec, n, r = 0, 100, 3
    print_case(test="trace_linear_dense", prec=prec, n=n)
    rng = np.random.default_rng([91, n])
    C = rng.standard_normal((n, n))
    C = 0.5 * (C + C.T)
    V0 = np.linalg.qr(rng.standard_normal((n, r)))[0]
    lam0 = np.full(r, 1.0 / r)
    obj = O.LinearObjective(C)
    it = oracle_iterate(obj, V0, lam0, r, 0.5, 2)
    with make_dense(C, meg.MEG_GRAD_LINEAR_DENSE, V0, lam0, r, prec, eta=0.5, max_inner=40) as g:
        info, _ = check_canonical(g, it, obj, 0.5, prec, "linear dense")
        assert info["batches"] == 2 and info["kd"] == 16


@pytest.mark.parametrize("prec,n", [(0, 96), (1, 150)])
def test_trace_denoise_dense(meg, prec, n):
    print_case(test="trace_denoise_dense", prec=prec, n=n)
    M, V0, lam0 = gapped_spiked(n, 2, seed=910 + n)
    Mq = M.astype(np_dtype(prec)).astype(np.float64)
    obj = O.DenoiseObjective(Mq)
    it = oracle_iterate(obj, V0, lam0, 2, 1.0, 3)
    with make_dense(Mq, meg.MEG_GRAD_DENOISE_DENSE, V0, lam0, 2, prec, eta=1.0, max_inner=40) as g:
        check_canonical(g, it, obj, 1.0, prec, "denoise dense")


def test_trace_masked_csr_f32(meg):
    prec, n, r = 1, 200, 3
    print_case(test="trace_masked_csr", prec=prec, n=n)
    p = W.matrix_completion(n, seed=9, rank=2, p=0.3, r=r, dtype=np.float32)
    obj = O.MaskedObjective(n, p.row_ptr, p.col, p.val.astype(np.float64))
    it = oracle_iterate(obj, p.V0, p.lam0, r, 1.0, 2)
    with make_csr(p, meg.MEG_GRAD_MASKED_CSR, r, prec, eta=1.0, max_inner=40) as g:
        check_canonical(g, it, obj, 1.0, prec, "masked csr")
        # the next step recomputes its own gradient values: it matches the
        # oracle's step from the same iterate
        info = g.step()
        ref, _ = O.lowrank_step(it, obj.grad(it.dense()), 1.0, O.eps_schedule(it.t), r, full=False)
        V, d, a, t = g.get_iterate()
        err = O.factored_diff_frob(V, d, a, ref.V, ref.d, ref.alpha) / O.factored_frob(ref.V, ref.d, ref.alpha)
        assert t == ref.t and err <= 1e-5 and info["converged"] == 1


def test_trace_linear_csr_f64(meg):
    prec, n, r = 0, 130, 2
    print_case(test="trace_linear_csr", prec=prec, n=n)
    p = W.matrix_completion(n, seed=12, rank=3, p=0.2, r=r, dtype=np.float64)
    obj = O.MaskedObjective(n, p.row_ptr, p.col, p.val, kind="linear")
    it = oracle_iterate(obj, p.V0, p.lam0, r, 0.7, 2)
    with make_csr(p, meg.MEG_GRAD_LINEAR_CSR, r, prec, eta=0.7, max_inner=40) as g:
        check_canonical(g, it, obj, 0.7, prec, "linear csr")


def test_trace_bf16_planes(meg):
    import torch

    n, rank = 192, 2
    print_case(test="trace_planes", n=n)
    M, V0, lam0 = gapped_spiked(n, rank, seed=93)
    hi, lo = W.bf16_planes(M.astype(np.float32))
    Mp = W.planes_value(hi, lo, n)
    obj = O.DenoiseObjective(Mp)
    it = oracle_iterate(obj, V0, lam0, rank, 1.0, 2)
    g = meg.LowRankMEG(n, rank, meg.MEG_GRAD_DENOISE_DENSE, V0, lam0, prec=meg.MEG_PREC_F32_BF16X3, eta=1.0,
                       dense=torch.from_numpy(hi.view(np.int16)).cuda(),
                       dense_lo=torch.from_numpy(lo.view(np.int16)).cuda(), max_inner=40)
    try:
        check_canonical(g, it, obj, 1.0, 2, "bf16 planes")
    finally:
        g.close()


@pytest.mark.parametrize("n", [16, 17])
def test_trace_block_spans_the_space(meg, n):
    """k = 16 >= n - 1: the deflated part holds (nearly) all of the trace; at
    n = 16 every projected probe vanishes and the tail is empty."""
    prec, r = 0, 2
    print_case(test="trace_small", n=n)
    rng = np.random.default_rng([92, n])
    C = rng.standard_normal((n, n))
    C = 0.5 * (C + C.T)
    V0 = np.linalg.qr(rng.standard_normal((n, r)))[0]
    lam0 = np.full(r, 0.5)
    obj = O.LinearObjective(C)
    it = oracle_iterate(obj, V0, lam0, r, 1.0, 1)
    with make_dense(C, meg.MEG_GRAD_LINEAR_DENSE, V0, lam0, r, prec, eta=1.0, max_inner=40) as g:
        info, _ = check_canonical(g, it, obj, 1.0, prec, "small")
        assert info["kd"] == min(16, n)
        if n == 16:
            assert info["log_b_tail"] == -math.inf


def test_certificate_full_matches_the_oracle(meg):
    """The all-eigenvalue certificate of the step from X_t: GPU (exact b_n from
    canonical probes, mu_{r+1} and eps_t of the step) against the oracle's
    lowrank_step; it is never above the cheap b^{r+1} certificate."""
    prec, n, r = 0, 96, 2
    print_case(test="certificate_full", n=n)
    # three spikes and r = 2: mu_{r+1} is isolated, so the step resolves it
    M, V3, _ = gapped_spiked(n, 3, seed=94)
    V0, lam0 = V3[:, :r].copy(), np.full(r, 1.0 / r)
    obj = O.DenoiseObjective(M)
    it = oracle_iterate(obj, V0, lam0, r, 1.0, 2)
    with make_dense(M, meg.MEG_GRAD_DENOISE_DENSE, V0, lam0, r, prec, eta=1.0, max_inner=60,
                    inner_tol=1e-13, cert_tol=1e-12) as g:
        info, tr = check_canonical(g, it, obj, 1.0, prec, "before step")
        with pytest.raises(meg.MegError) as e:  # no step from X_t yet
            g.certificate_full(tr)
        assert e.value.status == meg.MEG_ERR_INVALID_ARG
        step = g.step()
        L, holds = g.certificate_full(tr)
        _, ref = O.lowrank_step(it, obj.grad(it.dense()), 1.0, O.eps_schedule(it.t), r, full=True)
        print(f"  L_full={L:.10f} oracle={ref['L_full']:.10f} cheap={step['cert_L']:.10f} "
              f"eps={step['eps_t']:.3e} holds={holds} resid_r1={step['resid_r1']:.2e} "
              f"mu_r1={step['mu_r1']:.12f}/{ref['mu'][r]:.12f}", flush=True)
        assert step["t"] == it.t and step["eps_t"] == pytest.approx(ref["eps"], rel=1e-15)
        assert abs(L - ref["L_full"]) <= 1e-7
        assert L <= step["cert_L"] + 1e-12
        assert holds == (1 if L <= 2 * step["eps_t"] else 0)


def test_trace_gaussian_probes_masked(meg):
    """Gaussian probes (weight 1/p) on a matrix-completion iterate at n = 1024,
    r = 10: within 5 standard errors of the exact trace, and the deflation
    leaves a small relative error."""
    import torch

    prec, n, r, p = 1, 1024, 10, 32
    print_case(test="trace_gaussian", n=n, p=p)
    prob = W.matrix_completion(n, seed=15, rank=5, p=0.1, r=r, dtype=np.float32)
    obj = O.MaskedObjective(n, prob.row_ptr, prob.col, prob.val.astype(np.float64))
    it = oracle_iterate(obj, prob.V0, prob.lam0, r, 1.0, 2)
    Mt = oracle_mt(it, obj, 1.0)
    exact = O.logsumexp(np.linalg.eigvalsh(Mt))
    U = np.random.default_rng([95, n]).standard_normal((n, p))
    with make_csr(prob, meg.MEG_GRAD_MASKED_CSR, r, prec, eta=1.0, max_inner=40) as g:
        g.set_iterate(it.V, it.d, it.alpha, it.t)
        info, _ = g.trace_exp(torch.from_numpy(U).cuda(), max_steps=96, tol=1e-10)
        rel = math.expm1(info["log_b"] - exact)
        print(f"  log_b={info['log_b']:.10f} exact={exact:.10f} rel={rel:.3e} "
              f"stderr={info['tail_rel_stderr']:.3e} steps={info['steps']} conv={info['converged']}", flush=True)
        assert info["converged"] == 1 and info["batches"] == 1
        assert abs(rel) <= 5.0 * info["tail_rel_stderr"] + 1e-5
        assert info["tail_rel_stderr"] < 0.05
        # p = 0: the deflated part alone, a lower bound
        info0, _ = g.trace_exp(None, max_steps=96, tol=1e-10)
        assert info0["log_b"] == info0["log_b_defl"] and info0["log_b"] <= exact + 1e-5
        assert info0["log_b_tail"] == -math.inf and math.isnan(info0["tail_rel_stderr"])


def test_trace_rejects(meg):
    import ctypes

    import torch

    n, r = 64, 2
    M, V0, lam0 = gapped_spiked(n, 1, seed=4)
    print_case(test="trace_rejects", n=n)
    g = meg.LowRankMEG(n, r, meg.MEG_GRAD_EXTERNAL, V0, lam0, eta=1.0)
    try:
        with pytest.raises(meg.MegError) as e:
            g.trace_exp(None)
        assert e.value.status == meg.MEG_ERR_UNSUPPORTED
    finally:
        g.close()
    with make_dense(M, meg.MEG_GRAD_DENOISE_DENSE, V0, lam0, r, 1) as g2:
        probes = torch.zeros((n, 2), dtype=torch.float64, device="cuda")
        for kw in ({"weight": 0.0}, {"max_steps": 0}, {"tol": -1.0}):
            with pytest.raises(meg.MegError) as e:
                g2.trace_exp(probes, **kw)
            assert e.value.status == meg.MEG_ERR_INVALID_ARG
        lib = meg.load_library()
        out = meg.MegTraceInfo()
        assert lib.meg_trace_exp(g2._ctx, None, 2, 0.5, 16, 0.0, ctypes.byref(out)) == meg.MEG_ERR_INVALID_ARG
        assert lib.meg_trace_exp(g2._ctx, None, -1, 0.5, 16, 0.0, ctypes.byref(out)) == meg.MEG_ERR_INVALID_ARG
        with pytest.raises(ValueError):
            g2.trace_exp(probes.float())
