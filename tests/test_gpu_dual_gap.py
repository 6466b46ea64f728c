"""The dual gap of Section 7 (meg_dual_gap) against the FP64 oracle.

At the GPU's own iterate X_t (read back with meg_get_iterate) the oracle forms
G = grad f(X_t) densely and returns <X_t, G> - lambda_min(G) (eigvalsh); the
GPU accumulates <X_t, G> in FP64 and takes lambda_min from a Lanczos run on
G.  Tolerances are relative to |<X, G>| + ||G||_2: 1e-9 for an FP64 state,
1e-5 for FP32 (the GPU evaluates X from its basis rounded to FP32 and
multiplies G by FP32 vectors).
"""
import numpy as np
import pytest

import workloads as W
from oracle import meg_oracle as O
from tests.helpers import dev, gapped_spiked, make_csr, make_dense, np_dtype

pytestmark = pytest.mark.gpu

TOL = {0: 1e-9, 1: 1e-5, 2: 1e-5}


@pytest.fixture(scope="module")
def meg():
    from paper_2012_10469_amd import meg as m

    m.load_library()
    return m


def print_case(**kw):
    print("CASE " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def compare(g, G_of_X, prec, label):
    V, d, a, t = g.get_iterate()
    it = O.FactoredIterate(V, d, a, t)
    X = it.dense()
    G = G_of_X(X)
    ev = np.linalg.eigvalsh(O.sym(G))
    ref_xg = float(np.sum(X * G))
    ref = O.dual_gap(X, G)
    out = g.dual_gap(max_steps=256, tol=1e-12 if prec == 0 else 1e-8)
    scale = abs(ref_xg) + float(np.abs(ev).max())
    print(f"  {label} t={t}: gap={out['gap']:.10e} ref={ref:.10e} xg={out['x_dot_g']:.6e}/{ref_xg:.6e} "
          f"lmin={out['lambda_min']:.8e}/{ev[0]:.8e} steps={out['steps']} conv={out['converged']}", flush=True)
    assert out["t"] == t
    assert abs(out["x_dot_g"] - ref_xg) <= TOL[prec] * scale
    assert abs(out["lambda_min"] - ev[0]) <= TOL[prec] * scale
    assert abs(out["gap"] - ref) <= 2 * TOL[prec] * scale
    assert out["converged"] == 1
    return out, ref


@pytest.mark.parametrize("prec,n,rank", [(0, 96, 2), (1, 300, 3)])
def test_dual_gap_denoise(meg, prec, n, rank):
    print_case(test="dual_gap_denoise", prec=prec, n=n, rank=rank)
    M, V0, lam0 = gapped_spiked(n, rank, seed=700 + n)
    Mq = M.astype(np_dtype(prec)).astype(np.float64)
    with make_dense(Mq, meg.MEG_GRAD_DENOISE_DENSE, V0, lam0, rank, prec, eta=1.0, max_inner=40) as g:
        gaps = []
        for steps in (0, 3, 12):
            for _ in range(steps):
                g.step(info=False)
            out, ref = compare(g, lambda X: X - Mq, prec, f"after {steps} more steps")
            gaps.append(ref)
        assert gaps[-1] < gaps[0]  # the iterates approach the optimum


def test_dual_gap_masked(meg):
    prec, n = 1, 257
    print_case(test="dual_gap_masked", prec=prec, n=n)
    p = W.matrix_completion(n, seed=5, rank=2, p=0.3, r=3, dtype=np.float32)
    Mvals = p.val.astype(np.float64)
    rows = np.repeat(np.arange(n), np.diff(p.row_ptr))
    with make_csr(p, meg.MEG_GRAD_MASKED_CSR, 3, prec, eta=1.0, max_inner=40) as g:
        for _ in range(4):
            g.step(info=False)

        def grad(X):
            G = np.zeros((n, n))
            G[rows, p.col] = X[rows, p.col] - Mvals
            return G

        compare(g, grad, prec, "masked")
        # the step after the gap recomputes its own gradient values: the
        # trajectory continues undisturbed
        info = g.step()
        assert info["converged"] in (0, 1) and np.isfinite(info["cert_L"])


def test_dual_gap_linear(meg):
    prec, n, r = 0, 120, 3
    print_case(test="dual_gap_linear", prec=prec, n=n)
    rng = np.random.default_rng([90, n])
    C = rng.standard_normal((n, n))
    C = 0.5 * (C + C.T)
    V0 = np.linalg.qr(rng.standard_normal((n, r)))[0]
    lam0 = np.full(r, 1.0 / r)
    with make_dense(C, meg.MEG_GRAD_LINEAR_DENSE, V0, lam0, r, prec, eta=0.5, max_inner=40) as g:
        for _ in range(5):
            g.step(info=False)
        out, ref = compare(g, lambda X: C, prec, "linear")
        # for a linear objective the gap is exactly the suboptimality f(X_t) - lambda_min(C)
        assert out["gap"] == pytest.approx(g.objective() - np.linalg.eigvalsh(C)[0], abs=1e-9)


def test_dual_gap_bf16_planes(meg):
    n, rank = 256, 2
    print_case(test="dual_gap_planes", n=n)
    M, V0, lam0 = gapped_spiked(n, rank, seed=77)
    hi, lo = W.bf16_planes(M.astype(np.float32))
    Mp = W.planes_value(hi, lo, n)
    import torch

    g = meg.LowRankMEG(n, rank, meg.MEG_GRAD_DENOISE_DENSE, V0, lam0, prec=meg.MEG_PREC_F32_BF16X3, eta=1.0,
                       dense=torch.from_numpy(hi.view(np.int16)).cuda(),
                       dense_lo=torch.from_numpy(lo.view(np.int16)).cuda(), max_inner=40)
    try:
        for _ in range(4):
            g.step(info=False)
        compare(g, lambda X: X - Mp, 2, "planes")
    finally:
        g.close()


def test_dual_gap_rejects(meg):
    import torch

    n, r = 64, 2
    M, V0, lam0 = gapped_spiked(n, 1, seed=3)
    print_case(test="dual_gap_rejects", n=n)
    g = meg.LowRankMEG(n, r, meg.MEG_GRAD_EXTERNAL, V0, lam0, eta=1.0)
    try:
        with pytest.raises(meg.MegError) as e:
            g.dual_gap()
        assert e.value.status == meg.MEG_ERR_UNSUPPORTED
    finally:
        g.close()
    with make_dense(M, meg.MEG_GRAD_DENOISE_DENSE, V0, lam0, r, 1) as g2:
        with pytest.raises(meg.MegError) as e:
            g2.dual_gap(max_steps=0)
        assert e.value.status == meg.MEG_ERR_INVALID_ARG


def test_solve_to_gap_stops_at_the_first_small_gap(meg):
    """meg_solve_to_gap with a check after every iteration stops at the first
    iterate whose dual gap is <= tol: the same iterate that stepping one
    iteration at a time and evaluating the gap reaches (the launches give
    bitwise the same trajectory), and its gap is <= tol by the oracle."""
    prec, n, rank, tol = 0, 96, 2, 2e-3
    print_case(test="solve_to_gap", n=n, tol=tol)
    M, V0, lam0 = gapped_spiked(n, rank, seed=800)
    with make_dense(M, meg.MEG_GRAD_DENOISE_DENSE, V0, lam0, rank, prec, eta=1.0, max_inner=40) as a, \
            make_dense(M, meg.MEG_GRAD_DENOISE_DENSE, V0, lam0, rank, prec, eta=1.0, max_inner=40) as b:
        info, gap = a.solve_to_gap(200, tol, check_every=1)
        steps = 0
        while b.dual_gap(256, 1e-8)["gap"] > tol:
            b.step(info=False)
            steps += 1
            assert steps < 200
        ta, tb = a.get_iterate()[3], b.get_iterate()[3]
        print(f"  stopped at t={ta} (stepwise t={tb}), gap={gap['gap']:.4e}", flush=True)
        assert ta == tb == steps + 1 and gap["t"] == ta and gap["gap"] <= tol
        out, ref = compare(a, lambda X: X - M, prec, "at stop")
        assert ref <= tol * (1 + 1e-9)
        # coarser checks stop at or after that point
        with make_dense(M, meg.MEG_GRAD_DENOISE_DENSE, V0, lam0, rank, prec, eta=1.0, max_inner=40) as c:
            _, gc = c.solve_to_gap(200, tol, check_every=5)
            assert gc["gap"] <= tol and gc["t"] >= ta and (gc["t"] - 1) % 5 == 0
