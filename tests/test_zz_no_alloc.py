"""meg_dual_gap_static, the allocation-free variant of meg_dual_gap (its
Lanczos workspace is the library's fixed device array): its result equals
meg_dual_gap's on the same iterate, on two calls in a row, the second with a
smaller input; sizes beyond the array are rejected before any work."""
import numpy as np
import pytest

import workloads as W
from oracle import meg_oracle as O
from tests.helpers import make_csr, make_dense

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def meg():
    from paper_2012_10469_amd import meg as m

    m.load_library()
    return m


def _compare(g, prec, steps):
    # Lanczos tolerance and the bar: FP64 products resolve lambda_min to
    # ~1e-12 of the scale from any start; FP32 products (rounded inputs) to
    # ~1e-7 (the same bars as the dual gap's parity tests)
    lz_tol, tol = (1e-12, 1e-11) if prec == 0 else (1e-8, 1e-6)
    a = g.dual_gap(max_steps=steps, tol=lz_tol)      # context workspace (warm start)
    b = g.dual_gap_static(max_steps=steps, tol=lz_tol)  # fixed array, fresh start
    scale = abs(a["x_dot_g"]) + abs(a["lambda_min"])
    print(f"  gap {a['gap']:.15e} / static {b['gap']:.15e} (steps {a['steps']} / {b['steps']})", flush=True)
    if prec == 0:
        assert b["converged"] == 1 and a["converged"] == 1
    assert b["t"] == a["t"]
    assert b["x_dot_g"] == a["x_dot_g"]  # the same pass over the data
    assert abs(b["gap"] - a["gap"]) <= tol * scale
    return b


def test_static_dual_gap_matches_dual_gap(meg):
    # first call: masked objective, n = 1024, FP64
    p = W.matrix_completion(1024, seed=5, rank=3, p=0.1, r=4, dtype=np.float64)
    print("CASE test=no_alloc_dual_gap n=1024 prec=0", flush=True)
    with make_csr(p, meg.MEG_GRAD_MASKED_CSR, 4, 0, eta=1.0) as g:
        for _ in range(3):
            g.step(info=False)
        b = _compare(g, 0, 200)
        V, d, a, t = g.get_iterate()
        X = O.FactoredIterate(V, d, a, t).dense()
        obj = O.MaskedObjective(p.n, p.row_ptr, p.col, p.val.astype(np.float64))
        ref = O.dual_gap(X, obj.grad(X))
        assert abs(b["gap"] - ref) <= 1e-9 * (1.0 + abs(ref))
    # second call, smaller input: denoising, n = 300, FP32
    print("CASE test=no_alloc_dual_gap n=300 prec=1", flush=True)
    prob = W.spiked_denoise(300, 3)
    with make_dense(prob.M.astype(np.float32), meg.MEG_GRAD_DENOISE_DENSE, prob.V0, prob.lam0, 2, 1) as g:
        for _ in range(2):
            g.step(info=False)
        _compare(g, 1, 120)


def test_static_dual_gap_rejects_sizes_beyond_its_array(meg):
    n, r = 4096, 2
    print("CASE test=no_alloc_limit n=4096", flush=True)
    pr, c = W.linear_csr_diag(n, r, seed=3, dtype=np.float32)
    with make_csr(pr, meg.MEG_GRAD_LINEAR_CSR, r, 1, eta=0.9) as g:
        # (1100 + 1) x 4096 doubles of basis exceed the 4 Mi-double array
        with pytest.raises(meg.MegError) as e:
            g.dual_gap_static(max_steps=1100, tol=1e-10)
        assert e.value.status == meg.MEG_ERR_INVALID_ARG
        ok = g.dual_gap_static(max_steps=200, tol=1e-10)
        assert ok["steps"] >= 1
