"""The benchmark configurations as stated, against the oracle.

- Plain method, FP64, n = 200: M = u u^T + 0.01 (G + G^T)/sqrt(2n), r = 5,
  eta = 1, 100 iterations from the top eigenvector of M.  Every step from the
  oracle's own iterate (teacher-forced) to the FP64 bar, except where the
  oracle's eigen-gap mu_r - mu_{r+1} leaves the top-r subspace undetermined to
  that accuracy (reading 9 of the design: X_{t+1} is not unique there); the
  free-running trajectory's drift is reported beside it.
- Precision form, n = 16384 (BF16x3 apply, FP32 state): X_2 against the
  oracle's step from the same X_1 (its top 17 eigenpairs of M_1 by a Lanczos
  eigensolver on the host), to the mixed-precision bar 1e-3; the FP64 errors
  of X, f and the certificate are printed.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import meg_oracle as O
from tests.helpers import TOL_X, check_certificate, make_dense, rel_x_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def meg():
    from paper_2012_10469_amd import meg as m

    m.load_library()
    return m


def print_case(**kw):
    print("CASE " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def test_plain_configuration_fp64_n200(meg):
    n, r, T = 200, 5, 100
    print_case(test="config1", n=n, r=r, T=T)
    prob = W.spiked_denoise(n, seed=1, start="top1")
    obj = O.DenoiseObjective(prob.M)
    run = O.run_lowrank_meg(obj, prob.V0, prob.lam0, r, 1.0, T)
    checked, worst_tf, worst_fr, skipped = 0, 0.0, 0.0, []
    with make_dense(prob.M, meg.MEG_GRAD_DENOISE_DENSE, prob.V0, prob.lam0, r, 0, eta=1.0, max_inner=64) as g, \
            make_dense(prob.M, meg.MEG_GRAD_DENOISE_DENSE, prob.V0, prob.lam0, r, 0, eta=1.0, max_inner=64) as h:
        for t in range(1, T + 1):
            # free-running
            h.step(info=False)
            worst_fr = max(worst_fr, rel_x_err(h.get_iterate(), run["states"][t]))
            # teacher-forced from the oracle's X_t
            st = run["states"][t - 1]
            g.set_iterate(st.V, st.d, st.alpha, t)
            info = g.step()
            err = rel_x_err(g.get_iterate(), run["states"][t])
            mu = run["mu"][t - 1]
            rel_gap = run["gap"][t - 1] / max(1.0, abs(mu[0] - mu[-1]))
            check_certificate(info, run["L"][t - 1], run["eps"][t - 1], 0)
            assert abs(info["f"] - run["f"][t - 1]) <= 1e-12 * abs(run["f"][t - 1])
            if rel_gap < 1e-3:
                skipped.append((t, rel_gap, err))
                continue
            checked += 1
            worst_tf = max(worst_tf, err)
            assert err <= TOL_X[0], (t, err, rel_gap)
    print(f"  teacher-forced worst {worst_tf:.2e} over {checked} steps; {len(skipped)} steps with relative gap "
          f"< 1e-3 (e.g. {skipped[:3]}); free-running worst {worst_fr:.2e}", flush=True)
    assert checked >= T // 2


def test_precision_configuration_against_the_oracle(meg):
    import torch

    n, r, rank = 16384, 16, 8
    print_case(test="config4_oracle", n=n, r=r)
    prob = W.lowrank_noise_denoise(n, rank=rank, seed=1, noise=1e-3, r=r, dtype=np.float32, start="top1")
    hi, lo = W.bf16_planes(prob.M)
    del prob.M
    Mp = W.planes_value(hi, lo, n)  # the matrix the planes represent, FP64
    Q = np.random.default_rng([92, n]).standard_normal((n, r))
    for _ in range(8):
        Q, _ = np.linalg.qr(Mp @ Q)
    V0, lam0 = Q, np.full(r, 1.0 / r)
    dhi = torch.from_numpy(hi.view(np.int16)).cuda()
    dlo = torch.from_numpy(lo.view(np.int16)).cuda()
    del hi, lo
    torch.cuda.synchronize()
    g = meg.LowRankMEG(n, r, meg.MEG_GRAD_DENOISE_DENSE, V0, lam0, prec=meg.MEG_PREC_F32_BF16X3,
                       eta=1.0, dense=dhi, dense_lo=dlo, max_inner=40)
    try:
        V1, d1, a1, t1 = g.get_iterate()
        info = g.step()
        it1 = O.FactoredIterate(V1, d1, a1, t1)
        X1v = lambda x: a1 * x + V1 @ (d1[:, None] * (V1.T @ x))  # noqa: E731
        ref, ri = O.lowrank_step_operator(it1, lambda x: X1v(x) - Mp @ x, 1.0, O.eps_schedule(t1), r)
        err = rel_x_err(g.get_iterate(), ref)
        # f(X_1) = 1/2 ||X_1 - M||_F^2 without forming X_1
        f_ref = 0.5 * (float(np.sum(Mp * Mp)) - 2.0 * (a1 * float(np.trace(Mp)) +
                                                      float(np.sum(d1 * np.einsum("ij,ij->j", V1, Mp @ V1))))
                       + n * a1 * a1 + 2.0 * a1 * float(np.sum(d1)) + float(np.sum(d1 * d1)))
        print(f"  X_2 FP64 error {err:.2e}, f {info['f']:.10e} / {f_ref:.10e} (rel {abs(info['f'] - f_ref) / f_ref:.1e}),"
              f" L {info['cert_L']:.6f} / {ri['L']:.6f}, sweeps {info['inner_iters']}, gap {ri['gap']:.3e}",
              flush=True)
        assert err <= TOL_X[2]
        assert abs(info["f"] - f_ref) <= 1e-6 * abs(f_ref)
        check_certificate(info, ri["L"], O.eps_schedule(t1), 2)
    finally:
        g.close()
        del dhi, dlo
        torch.cuda.empty_cache()
