"""Shared helpers of the GPU parity tests: device upload, running the HIP path
through the C ABI, and comparing factored iterates with the oracle's."""
from __future__ import annotations

import math

import numpy as np

from oracle import meg_oracle as O

# tolerances (relative Frobenius error of X; relative objective error)
TOL_X = {0: 1e-9, 1: 1e-5, 2: 1e-3}
TOL_F = 1e-6
UNIT = {0: 2.0 ** -53, 1: 2.0 ** -24, 2: 2.0 ** -24}
# |cert_L - L_oracle| once the (r+1)-th Ritz pair is resolved
TOL_CERT = {0: 1e-8, 1: 1e-4, 2: 1e-4}


def check_certificate(info, L_ref, eps_ref, prec):
    """The step's certificate against the oracle's L_t (exact eigenvalues).

    cert_L comes from the Ritz values: the (r+1)-th one is a lower bound of
    mu_{r+1} (interlacing) and L does not decrease with it, so cert_L is a
    lower bound of the oracle's L.  Resolved (r+1)-th pair: cert_L within
    TOL_CERT of the oracle's.  cert_L_up is an upper bound of it.  In every
    case a claimed certificate holds for the oracle too: cert_holds is never 1
    where the exact L_t > 2 eps_t."""
    tol = TOL_CERT[prec]
    L = info["cert_L"]
    assert L <= L_ref + tol, ("lower bound", L, L_ref)
    if info["cert_resolved"]:
        assert abs(L - L_ref) <= tol, ("resolved", L, L_ref)
    # the upper bound behind any claim (resolved pair or an armed deflated
    # Lanczos bound; +inf without either)
    assert L_ref <= info["cert_L_up"] + tol, ("upper bound", info["cert_L_up"], L_ref)
    if info["cert_holds"]:
        assert info["cert_L_up"] <= 2.0 * eps_ref
        assert L_ref <= 2.0 * eps_ref, ("claim the oracle does not make", L, L_ref, eps_ref)


def torch_dtype(prec):
    import torch

    return torch.float64 if prec == 0 else torch.float32


def np_dtype(prec):
    return np.float64 if prec == 0 else np.float32


def dev(a, dtype=None):
    import torch

    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda().contiguous()


def make_dense(M_, kind, V0, lam0, r, prec, **kw):
    from paper_2012_10469_amd import meg

    D = dev(np.asarray(M_, dtype=np_dtype(prec)))
    return meg.LowRankMEG(D.shape[0], r, kind, V0, lam0, prec=prec, dense=D, **kw)


def make_csr(p, kind, r, prec, V0=None, lam0=None, **kw):
    from paper_2012_10469_amd import meg
    import torch

    rp = dev(p.row_ptr.astype(np.int32))
    col = dev(p.col.astype(np.int32))
    val = dev(p.val.astype(np_dtype(prec)))
    V0 = p.V0 if V0 is None else V0
    lam0 = p.lam0 if lam0 is None else lam0
    return meg.LowRankMEG(p.n, r, kind, V0, lam0, prec=prec, row_ptr=rp, col=col, val=val, **kw)


def rel_x_err(gpu_state, it: O.FactoredIterate) -> float:
    V, d, a, _ = gpu_state
    num = O.factored_diff_frob(V, d, a, it.V, it.d, it.alpha)
    return num / O.factored_frob(it.V, it.d, it.alpha)


def f_tol(f_ref: float, gradnorm_f: float, xnorm_f: float, prec: int) -> float:
    """|f_gpu - f_ref| allowance: TOL_F relative, plus the first-order effect of
    rounding the iterate to the working precision (|<grad f, dX>| with
    ||dX||_F <= 4 u ||X||_F)."""
    return TOL_F * abs(f_ref) + 4.0 * UNIT[prec] * gradnorm_f * xnorm_f


def oracle_state_at(run, t):
    """Oracle iterate X_t (t >= 1)."""
    return run["states"][t - 1]


def gapped_spiked(n, rank, seed, noise=0.01):
    """M = U diag(2, 1.8, ...) U^T + noise (G + G^T)/sqrt(2n) (rank <= 5,
    strictly complementary at r = rank), with its top-`rank` eigenvectors as
    the start."""
    rng = np.random.default_rng([78, seed, n])
    U, _ = np.linalg.qr(rng.standard_normal((n, rank)))
    s = 2.0 - 0.2 * np.arange(rank)
    G = rng.standard_normal((n, n))
    M = (U * s) @ U.T + noise * (G + G.T) / math.sqrt(2 * n)
    M = 0.5 * (M + M.T)
    w, V = np.linalg.eigh(M)
    V0 = V[:, ::-1][:, :rank].copy()
    lam0 = np.full(rank, 1.0 / rank)
    return M, V0, lam0


def isolated_linear(n, r, seed):
    """Linear objective f = <C, X>, C = U diag(c) U^T: c_1..c_r on [0, 0.5],
    c_{r+1} = 2, the rest on [3, 4], so the (r+1)-th eigenvalue of M_t is
    isolated (eta apart from the others) and its Ritz pair resolves; start on
    U[:, :r] with equal weights."""
    rng = np.random.default_rng([79, seed, n])
    U, R = np.linalg.qr(rng.standard_normal((n, n)))
    U = U * np.sign(np.diag(R))
    c = np.concatenate([np.sort(0.5 * rng.random(r)), [2.0], 3.0 + np.sort(rng.random(n - r - 1))])
    C = (U * c) @ U.T
    return 0.5 * (C + C.T), U[:, :r].copy(), np.full(r, 1.0 / r)
