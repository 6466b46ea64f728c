"""FP64 CPU oracle for the low-rank Matrix Exponentiated Gradient (MEG) method.

TEST INFRASTRUCTURE.  Only the test-suite, the package smoke check and the
benchmark's CPU-baseline leg may import or run this module; the product path
(the HIP library and its Python binding) never does, and this module imports
nothing from the product.  It is deliberately plain and slow: dense n x n
matrices in float64, LAPACK symmetric eigendecompositions via NumPy/SciPy, no
blocking or fusion beyond the definitions it restates.

Source: D. Garber, A. Kaplan, "On the Efficient Implementation of the Matrix
Exponentiated Gradient Algorithm for Low-Rank Matrix Optimization"
(arXiv 2012.10469).  Each function cites the passage it follows.

Notation used here (the paper reuses Y, M and W for several objects):
  X_t  = alpha I + V diag(d) V^T      the factored iterate (Section 3)
  M_t  = log X_t - eta grad f(X_t)    the log-domain matrix of Section 3
  mu   = eigenvalues of M_t, descending; the paper's Y_t = exp(M_t) has
         eigenvalues exp(mu)
Parity status: every function below is pinned by a test under ``tests/``
(test_oracle_*.py); none is "parity unpinned".
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional, Sequence

import numpy as np
import scipy.linalg as sla

__all__ = [
    "eps_schedule",
    "sym",
    "eig_desc",
    "mat_log",
    "mat_exp",
    "logsumexp",
    "softmax",
    "bregman",
    "LinearObjective",
    "DenoiseObjective",
    "MaskedObjective",
    "QuadMeasObjective",
    "BilinearObjective",
    "exact_meg_step",
    "run_exact_meg",
    "FactoredIterate",
    "initial_iterate",
    "lowrank_step",
    "lowrank_step_factored",
    "lowrank_step_operator",
    "run_lowrank_meg",
    "run_lowrank_meg_dual_average",
    "certificate",
    "project_spectrahedron",
    "factored_diff_frob",
    "factored_frob",
    "dual_gap",
    "trace_exp_deflated",
    "certificate_from_log_b",
]


# ---------------------------------------------------------------------------
# schedules and small helpers
# ---------------------------------------------------------------------------
def eps_schedule(t: int, scale: float = 0.8, c: float = 10.0, power: float = 2.0) -> float:
    """epsilon_t = scale / (t + c + 1)^power, t >= 0.

    Section 7 sets epsilon_t = (4/5)/(t + c + 1)^2 with c = 10; the theory
    sections use other powers, so the exponent is a parameter."""
    return float(scale) / float(t + c + 1.0) ** float(power)


def sym(G: np.ndarray) -> np.ndarray:
    """(G + G^T)/2: Section 1 (footnote) replaces a non-symmetric gradient by
    its symmetric part, which leaves <Y, grad f> unchanged on symmetric Y."""
    return 0.5 * (G + G.T)


def eig_desc(A: np.ndarray, top: Optional[int] = None):
    """Eigenpairs of a symmetric matrix, eigenvalues in non-increasing order
    (the paper's lambda_i(X) is the i-th largest eigenvalue, Section 2.1).
    ``top`` = k returns only the k largest pairs (LAPACK subset driver)."""
    A = sym(np.asarray(A, dtype=np.float64))
    n = A.shape[0]
    if top is None or top >= n:
        w, U = np.linalg.eigh(A)
    else:
        w, U = sla.eigh(A, subset_by_index=[n - top, n - 1])
    return w[::-1].copy(), U[:, ::-1].copy()


def logsumexp(x: np.ndarray) -> float:
    x = np.asarray(x, dtype=np.float64)
    m = float(np.max(x))
    return m + math.log(float(np.sum(np.exp(x - m))))


def softmax(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    e = np.exp(x - np.max(x))
    return e / e.sum()


def mat_log(X: np.ndarray) -> np.ndarray:
    """log X = U diag(log w) U^T for X positive definite (Section 2.1)."""
    w, U = np.linalg.eigh(sym(X))
    if np.min(w) <= 0:
        raise ValueError("mat_log needs a positive definite matrix")
    return (U * np.log(w)) @ U.T


def mat_exp(A: np.ndarray) -> np.ndarray:
    """exp A = U diag(exp w) U^T for symmetric A (Section 2.1)."""
    w, U = np.linalg.eigh(sym(A))
    return (U * np.exp(w)) @ U.T


def bregman(X: np.ndarray, Y: np.ndarray) -> float:
    """Bregman distance of the von Neumann entropy on the spectrahedron
    (Section 2.2): B(X, Y) = tr(X log X - X log Y), with 0 log 0 := 0.
    Y must be positive definite; X may be singular."""
    wx, Ux = np.linalg.eigh(sym(X))
    wx = np.clip(wx, 0.0, None)
    xlogx = float(np.sum(np.where(wx > 0, wx * np.log(np.where(wx > 0, wx, 1.0)), 0.0)))
    return xlogx - float(np.sum(sym(X) * mat_log(Y)))


# ---------------------------------------------------------------------------
# objectives (dense FP64 gradients)
# ---------------------------------------------------------------------------
class LinearObjective:
    """f(X) = <C, X>, grad f = C (symmetric)."""

    def __init__(self, C: np.ndarray):
        self.C = sym(np.asarray(C, dtype=np.float64))
        self.n = self.C.shape[0]

    def grad(self, X: np.ndarray) -> np.ndarray:
        return self.C

    def value(self, X: np.ndarray) -> float:
        return float(np.sum(self.C * X))


class DenoiseObjective:
    """f(X) = 1/2 ||X - M||_F^2, grad f = X - M; beta = 1 w.r.t. (||.||_*, ||.||_2)."""

    def __init__(self, M: np.ndarray):
        self.M = sym(np.asarray(M, dtype=np.float64))
        self.n = self.M.shape[0]

    def grad(self, X: np.ndarray) -> np.ndarray:
        return X - self.M

    def value(self, X: np.ndarray) -> float:
        R = X - self.M
        return 0.5 * float(np.sum(R * R))


class MaskedObjective:
    """f(X) = 1/2 sum over the stored entries (i, j) of Omega of (X_ij - M_ij)^2,
    Omega symmetric (both (i,j) and (j,i) are stored); grad f = P_Omega(X - M).

    For kind == "linear" the stored values are C_ij and f = <C, X>."""

    def __init__(self, n: int, row_ptr, col, val, kind: str = "masked"):
        self.n = int(n)
        rp = np.asarray(row_ptr, dtype=np.int64)
        self.rows = np.repeat(np.arange(self.n), np.diff(rp))
        self.cols = np.asarray(col, dtype=np.int64)
        self.vals = np.asarray(val, dtype=np.float64)
        self.kind = kind

    def _dense(self, v: np.ndarray) -> np.ndarray:
        D = np.zeros((self.n, self.n))
        D[self.rows, self.cols] = v
        return D

    def grad(self, X: np.ndarray) -> np.ndarray:
        if self.kind == "linear":
            return self._dense(self.vals)
        return self._dense(X[self.rows, self.cols] - self.vals)

    def value(self, X: np.ndarray) -> float:
        if self.kind == "linear":
            return float(np.sum(X[self.rows, self.cols] * self.vals))
        r = X[self.rows, self.cols] - self.vals
        return 0.5 * float(np.sum(r * r))


class QuadMeasObjective:
    """f(X) = 1/(2m) sum_i (a_i^T X a_i - b_i)^2 over a pool A = [a_1..a_m].

    grad f = (1/m) sum_i (a_i^T X a_i - b_i) a_i a_i^T.  The stochastic
    estimate of Section 6 averages L sampled terms; the sample indices are an
    input (``batch``), never drawn here."""

    def __init__(self, A: np.ndarray, b: np.ndarray):
        self.A = np.asarray(A, dtype=np.float64)
        self.b = np.asarray(b, dtype=np.float64)
        self.n, self.m = self.A.shape

    def residuals(self, X: np.ndarray, idx: Optional[np.ndarray] = None) -> np.ndarray:
        A = self.A if idx is None else self.A[:, idx]
        b = self.b if idx is None else self.b[idx]
        return np.einsum("ij,ij->j", A, X @ A) - b

    def grad(self, X: np.ndarray, batch: Optional[np.ndarray] = None) -> np.ndarray:
        A = self.A if batch is None else self.A[:, batch]
        w = self.residuals(X, batch)
        return (A * w) @ A.T / A.shape[1]

    def value(self, X: np.ndarray) -> float:
        w = self.residuals(X)
        return 0.5 * float(np.dot(w, w)) / self.m

    def residuals_factored(self, it: "FactoredIterate", idx: Optional[np.ndarray] = None) -> np.ndarray:
        """a_i^T X a_i - b_i for X = alpha I + V diag(d) V^T without forming X:
        a_i^T X a_i = alpha ||a_i||^2 + sum_l d_l (v_l^T a_i)^2."""
        A = self.A if idx is None else self.A[:, idx]
        b = self.b if idx is None else self.b[idx]
        P = it.V.T @ A  # q x L
        x = it.alpha * np.sum(A * A, axis=0) + np.sum(it.d[:, None] * P * P, axis=0)
        return x - b

    def grad_factor(self, it: "FactoredIterate", batch: np.ndarray):
        """The minibatch gradient in factored form F diag(c) F^T: F = A_B
        (n x L), c_i = (a_i^T X a_i - b_i)/L."""
        F = self.A[:, batch]
        return F, self.residuals_factored(it, batch) / F.shape[1]

    def value_factored(self, it: "FactoredIterate") -> float:
        w = self.residuals_factored(it)
        return 0.5 * float(np.dot(w, w)) / self.m


# ---------------------------------------------------------------------------
# exact MEG (Algorithm 1)
# ---------------------------------------------------------------------------
def exact_meg_step(Z: np.ndarray, G: np.ndarray, eta: float) -> np.ndarray:
    """Z_+ = exp(log Z - eta G) / tr exp(log Z - eta G)  (Section 2.2, the
    von Neumann mirror step; one iteration of Algorithm 1).  The trace
    normalisation is applied to the eigenvalues (a softmax), which is the
    same matrix without overflow."""
    A = mat_log(Z) - eta * sym(G)
    w, U = np.linalg.eigh(sym(A))
    return (U * softmax(w)) @ U.T


def run_exact_meg(obj, Z1: np.ndarray, eta: float, T: int, grads: Optional[Sequence] = None):
    """Algorithm 1 for T iterations from Z_1; returns [Z_1, ..., Z_{T+1}].
    ``grads`` (optional) supplies the gradient used at each iteration (for
    stochastic runs), otherwise obj.grad(Z_t)."""
    Zs = [np.asarray(Z1, dtype=np.float64)]
    for t in range(T):
        G = grads[t] if grads is not None else obj.grad(Zs[-1])
        Zs.append(exact_meg_step(Zs[-1], G, eta))
    return Zs


# ---------------------------------------------------------------------------
# low-rank MEG (Definition 1, Algorithm 2)
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class FactoredIterate:
    """X = alpha I + V diag(d) V^T with V (n x q, orthonormal columns, q <= r).

    Section 3 stores the low-rank iterate this way: with
    X = (1 - eps) V Lambda V^T + eps/(n - r) (I - V V^T) one has
    alpha = eps/(n - r) and d = (1 - eps) lambda - alpha; the first iterate of
    Algorithm 2 uses the level eps_0/n instead."""

    V: np.ndarray
    d: np.ndarray
    alpha: float
    t: int = 1

    @property
    def n(self) -> int:
        return self.V.shape[0]

    def eigenvalues_on_V(self) -> np.ndarray:
        return self.alpha + self.d

    def dense(self) -> np.ndarray:
        return self.alpha * np.eye(self.n) + (self.V * self.d) @ self.V.T

    def log_dense(self) -> np.ndarray:
        """log X = V diag(log(alpha + d)) V^T + log(alpha) (I - V V^T): the
        closed form of the logarithm of the factored iterate (Section 3)."""
        lv = np.log(self.alpha + self.d)
        la = math.log(self.alpha)
        return (self.V * lv) @ self.V.T + la * (np.eye(self.n) - self.V @ self.V.T)

    def copy(self) -> "FactoredIterate":
        return FactoredIterate(self.V.copy(), self.d.copy(), float(self.alpha), int(self.t))


def initial_iterate(V0: np.ndarray, lam0: np.ndarray, eps0: float, n: Optional[int] = None) -> FactoredIterate:
    """Initialisation of Algorithm 2: X_1 = (1 - eps_0) X_0 + (eps_0/n) I with
    X_0 = V0 diag(lam0) V0^T.  Note the complement level is eps_0/n here, not
    eps_0/(n - r) as in later iterates."""
    V0 = np.asarray(V0, dtype=np.float64)
    n = V0.shape[0] if n is None else n
    lam0 = np.asarray(lam0, dtype=np.float64)
    return FactoredIterate(V0.copy(), (1.0 - eps0) * lam0, eps0 / n, 1)


def certificate(mu_desc: np.ndarray, r: int, eps: float, n: int, k: Optional[int] = None) -> float:
    """log((n - r) lambda_{r+1}(Y) / (eps b_k)) with lambda_i(Y) = exp(mu_i) and
    b_k = sum_{i<=k} lambda_i(Y).

    k = n (all eigenvalues) is the condition of the approximation-error lemma
    of Section 3.1.1; k = r + 1 is the cheap certificate of the same section
    and of Section 7, sufficient because b_{r+1} <= b_n.  The step is
    certified when the value is <= 2 eps."""
    mu = np.asarray(mu_desc, dtype=np.float64)
    k = mu.size if k is None else k
    return math.log(n - r) + float(mu[r]) - math.log(eps) - logsumexp(mu[:k])


def lowrank_step(it: FactoredIterate, G: np.ndarray, eta: float, eps: float, r: int,
                 full: bool = True):
    """One iteration of Algorithm 2 (Definition 1) from X_t = ``it`` with
    gradient G at X_t, approximation parameter eps = eps_t and rank r.

    M_t = log X_t - eta G (Section 3, with log X_t from the factored form);
    Y_t = exp(M_t) is never formed.  Its top-r eigenpairs (mu_i, v_i) give
    a_t = sum_{i<=r} exp(mu_i) and
        X_{t+1} = (1 - eps) V diag(exp(mu_{1..r}))/a_t V^T + eps/(n-r) (I - V V^T).
    ``full`` = True computes every eigenpair (also returns the exact MEG step
    Z_+ = exp(M_t)/b and the all-eigenvalue certificate); False computes only
    the top r + 1 pairs.

    Returns (new FactoredIterate, info dict)."""
    n = it.n
    if not (1 <= r <= n - 1):
        raise ValueError("rank parameter r must lie in {1, ..., n-1}")
    Mt = it.log_dense() - eta * sym(G)
    mu, U = eig_desc(Mt, None if full else r + 1)
    lam_tilde = softmax(mu[:r])  # exp(mu_i)/a_t
    alpha_new = eps / (n - r)
    d_new = (1.0 - eps) * lam_tilde - alpha_new
    new = FactoredIterate(U[:, :r].copy(), d_new, alpha_new, it.t + 1)
    info = {
        "mu": mu,
        "U": U,
        "gap": float(mu[r - 1] - mu[r]),
        "L": certificate(mu, r, eps, n, r + 1),
        "L_full": certificate(mu, r, eps, n, n) if full else None,
        "eps": eps,
        "lam_tilde": lam_tilde,
    }
    if full:
        info["Zplus"] = (U * softmax(mu)) @ U.T
    return new, info


def lowrank_step_operator(it: FactoredIterate, grad_mv: Callable[[np.ndarray], np.ndarray], eta: float,
                          eps: float, r: int, tol: float = 1e-13):
    """lowrank_step with the gradient given only as its action x -> G x (for
    sizes where a dense eigendecomposition of M_t is out of reach): the top
    r + 1 eigenpairs of M_t = log X_t - eta G (log X_t from the factored form,
    Section 3) by a Lanczos eigensolver (ARPACK, residual tolerance ``tol``),
    then the same exponentiation, normalisation and certificate (Definition 1,
    Section 3.1.1).  Returns (new FactoredIterate, info with mu (top r + 1),
    gap, L)."""
    from scipy.sparse.linalg import LinearOperator, eigsh

    n = it.n
    la = math.log(it.alpha)
    c = np.log(it.alpha + it.d) - la
    V = it.V

    def mv(x):
        x = np.asarray(x, dtype=np.float64).reshape(n, -1)
        y = la * x + V @ (c[:, None] * (V.T @ x)) - eta * grad_mv(x)
        return y if y.shape[1] > 1 else y.reshape(-1)

    op = LinearOperator((n, n), matvec=mv, matmat=mv, dtype=np.float64)
    v0 = np.random.default_rng([93, n]).standard_normal(n)
    w, U = eigsh(op, k=r + 1, which="LA", tol=tol, v0=v0, maxiter=100 * n, ncv=min(n, max(4 * (r + 1), 40)))
    order = np.argsort(w)[::-1]
    mu, U = w[order], U[:, order]
    alpha_new = eps / (n - r)
    new = FactoredIterate(U[:, :r].copy(), (1.0 - eps) * softmax(mu[:r]) - alpha_new, alpha_new, it.t + 1)
    return new, {"mu": mu, "gap": float(mu[r - 1] - mu[r]), "L": certificate(mu, r, eps, n, r + 1), "eps": eps}


def lowrank_step_factored(it: FactoredIterate, F: np.ndarray, c: np.ndarray, eta: float, eps: float, r: int):
    """lowrank_step for a gradient given as G = F diag(c) F^T (F n x p), without
    any n x n matrix.  M_t - log(alpha) I = V diag(log(alpha + d) - log alpha) V^T
    - eta F diag(c) F^T vanishes on the orthogonal complement of S = span[V, F],
    so S is an invariant subspace: with U an orthonormal basis of S (dimension
    s), the eigenvalues of M_t are those of U^T M_t U and log(alpha) with
    multiplicity n - s, and the eigenvectors of the first kind are U times
    those of the s x s matrix.  Same outputs as lowrank_step with full=True,
    except that ``U``/``Zplus`` are omitted and ``L_full`` counts the n - s
    eigenvalues log(alpha) analytically."""
    n = it.n
    if not (1 <= r <= n - 1):
        raise ValueError("rank parameter r must lie in {1, ..., n-1}")
    F = np.asarray(F, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    la = math.log(it.alpha)
    basis = np.concatenate([it.V, F], axis=1)
    Uq, sv, _ = np.linalg.svd(basis, full_matrices=False)
    U = Uq[:, sv > sv[0] * 1e-12]
    s = U.shape[1]
    cv = np.log(it.alpha + it.d) - la
    PV = U.T @ it.V
    PF = U.T @ F
    H = (PV * cv) @ PV.T - eta * (PF * c) @ PF.T + la * np.eye(s)
    mu_s, S = eig_desc(H)
    # merge with the n - s eigenvalues log(alpha) of the complement
    if s < n:
        mu = np.concatenate([mu_s, np.full(n - s, la)])
        order = np.argsort(-mu, kind="stable")
        mu = mu[order]
    else:
        order = np.arange(n)
        mu = mu_s
    if np.any(order[:r] >= s):
        raise ValueError("a top-r eigenvalue of M_t lies on the complement of span[V, F]")
    Vn = U @ S[:, order[:r]]
    lam_tilde = softmax(mu[:r])
    alpha_new = eps / (n - r)
    d_new = (1.0 - eps) * lam_tilde - alpha_new
    new = FactoredIterate(Vn, d_new, alpha_new, it.t + 1)
    info = {
        "mu": mu,
        "gap": float(mu[r - 1] - mu[r]),
        "L": certificate(mu, r, eps, n, r + 1),
        "L_full": certificate(mu, r, eps, n, n),
        "eps": eps,
        "lam_tilde": lam_tilde,
        "subspace_dim": s,
    }
    return new, info


def run_lowrank_meg(obj, V0, lam0, r: int, eta: float, T: int, eps_params=(0.8, 10.0, 2.0),
                    full: bool = True, grad_fn: Optional[Callable] = None, keep_states: bool = True):
    """Algorithm 2 for T iterations (t = 1..T), producing X_2 .. X_{T+1}.

    Returns a dict with per-iteration lists: ``states`` (X_1..X_{T+1} as
    FactoredIterate), ``f`` (f(X_t) at the point where the gradient is
    taken), ``L``, ``L_full``, ``gap``, ``eps`` and ``mu``.  ``grad_fn(t, X)``
    overrides the gradient (stochastic runs pass minibatch estimates)."""
    V0 = np.asarray(V0, dtype=np.float64)
    n = V0.shape[0]
    it = initial_iterate(V0, lam0, eps_schedule(0, *eps_params), n)
    out = {k: [] for k in ("states", "f", "L", "L_full", "gap", "eps", "mu")}
    out["states"].append(it.copy())
    for t in range(1, T + 1):
        X = it.dense()
        G = grad_fn(t, X) if grad_fn is not None else obj.grad(X)
        out["f"].append(obj.value(X) if obj is not None else float("nan"))
        e = eps_schedule(t, *eps_params)
        it, info = lowrank_step(it, G, eta, e, r, full=full)
        out["L"].append(info["L"])
        out["L_full"].append(info["L_full"])
        out["gap"].append(info["gap"])
        out["eps"].append(e)
        out["mu"].append(info["mu"])
        if keep_states:
            out["states"].append(it.copy())
    if not keep_states:
        out["states"].append(it.copy())
    return out


def run_lowrank_meg_dual_average(obj, V0, lam0, r: int, eta: float, T: int, eps_params=(0.8, 10.0, 2.0)):
    """The dual-averaging reading of the low-rank step (the accumulate-forever
    form of the benchmark spec, reading C1 of the design): the log-domain
    matrix is accumulated, Y_1 = log X_1 and Y_{t+1} = Y_t - eta grad f(X_t),
    never rebuilt from the factored iterate, and X_{t+1} is formed from the
    top-r eigenpairs of Y_{t+1} exactly as Definition 1 forms it from those of
    M_t (softmax of the top r eigenvalues, mixed with eps_t/(n - r) on the
    complement).  With f linear and V0 spanning eigenvectors of its C this
    coincides with Algorithm 2 (softmax composes and ignores shifts); it
    differs otherwise.  Returns the same dict as run_lowrank_meg (mu: the
    eigenvalues of Y_{t+1})."""
    V0 = np.asarray(V0, dtype=np.float64)
    n = V0.shape[0]
    it = initial_iterate(V0, lam0, eps_schedule(0, *eps_params), n)
    Y = it.log_dense()
    out = {k: [] for k in ("states", "f", "L", "gap", "eps", "mu")}
    out["states"].append(it.copy())
    for t in range(1, T + 1):
        X = it.dense()
        out["f"].append(obj.value(X))
        Y = Y - eta * sym(obj.grad(X))
        e = eps_schedule(t, *eps_params)
        mu, U = eig_desc(Y, r + 1)
        alpha_new = e / (n - r)
        it = FactoredIterate(U[:, :r].copy(), (1.0 - e) * softmax(mu[:r]) - alpha_new, alpha_new, t + 1)
        out["L"].append(certificate(mu, r, e, n, r + 1))
        out["gap"].append(float(mu[r - 1] - mu[r]))
        out["eps"].append(e)
        out["mu"].append(mu)
        out["states"].append(it.copy())
    return out


class BilinearObjective:
    """f(X) = 1/2 sum_i (tr(A_i^T X B_i) - y_i)^2, the recovery problem of
    Section 7 (full, deterministic gradients): rank-1 measurements a_i^T X b_i
    (A, B: m x n, rows a_i, b_i), or measurement matrices A_i, B_i with p
    columns (A, B: m x p x n, A[i, q] the q-th column of A_i).

    grad f = sum_i r_i A_i B_i^T with r_i = tr(A_i^T X B_i) - y_i; the method
    uses its symmetric part (Section 1), 1/2 sum_i r_i (A_i B_i^T + B_i A_i^T)."""

    def __init__(self, A: np.ndarray, B: np.ndarray, y: np.ndarray):
        A = np.asarray(A, dtype=np.float64)
        B = np.asarray(B, dtype=np.float64)
        self.p = 1 if A.ndim == 2 else A.shape[1]
        self.A = A.reshape(-1, A.shape[-1])  # (m p) x n, rows grouped by measurement
        self.B = B.reshape(-1, B.shape[-1])
        self.y = np.asarray(y, dtype=np.float64)

    def residuals(self, X: np.ndarray) -> np.ndarray:
        t = np.sum((self.A @ X) * self.B, axis=1)
        return t.reshape(-1, self.p).sum(axis=1) - self.y

    def grad(self, X: np.ndarray) -> np.ndarray:
        r = np.repeat(self.residuals(X), self.p)
        H = self.A.T @ (r[:, None] * self.B)
        return 0.5 * (H + H.T)

    def value(self, X: np.ndarray) -> float:
        r = self.residuals(X)
        return 0.5 * float(np.dot(r, r))


# ---------------------------------------------------------------------------
# Euclidean projection (Section 2.3) and the dual gap (Section 7)
# ---------------------------------------------------------------------------
def project_spectrahedron(A: np.ndarray, tau: float = 1.0) -> np.ndarray:
    """Euclidean projection onto {X >= 0, tr X = tau}: U diag(max(0, w - l)) U^T
    with the scalar l solving sum_i max(0, w_i - l) = tau (Section 2.3),
    found by bisection."""
    w, U = np.linalg.eigh(sym(np.asarray(A, dtype=np.float64)))
    lo, hi = float(w.min()) - tau, float(w.max())
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if np.sum(np.maximum(w - mid, 0.0)) > tau:
            lo = mid
        else:
            hi = mid
    lam = np.maximum(w - 0.5 * (lo + hi), 0.0)
    lam *= tau / lam.sum()
    return (U * lam) @ U.T


def dual_gap(X: np.ndarray, G: np.ndarray, tau: float = 1.0) -> float:
    """max_{Z in tau-spectrahedron} <X - Z, G> = <X, G> - tau lambda_min(G) (Section 7)."""
    return float(np.sum(X * G)) - tau * float(np.linalg.eigvalsh(sym(G))[0])


# ---------------------------------------------------------------------------
# the full-trace certificate: b_n = tr exp(M_t) (Section 3.1.1)
# ---------------------------------------------------------------------------
def trace_exp_deflated(Mt: np.ndarray, Q: Optional[np.ndarray], probes: np.ndarray, weight: float) -> dict:
    """Deflated randomised estimate of b_n = tr exp(M_t), the sum of all
    eigenvalues of Y_t = exp(M_t) in the certificate of Section 3.1.1.

    Section 3.1.1 notes (footnote) that b_n could instead be estimated from
    E_u[u^T Y u] = tr Y over Gaussian u (Hutchinson's estimator), with the
    products exp(M)u from Lanczos.  The estimate here splits the trace by an
    orthonormal basis Q of a k-dimensional subspace: with P = I - Q Q^T,
        tr A = tr(Q^T A Q) + tr(P A P)      (any orthonormal Q),
    computes the first term and estimates the second by
        weight * sum_j (P u_j)^T A (P u_j)
    (the deflation used by Hutch++: Meyer, Musco, Musco, Woodruff, 2021).
    It is exact for the n canonical basis vectors as probes with weight 1,
    and unbiased for E[u u^T] = I with weight = 1/p.

    Q: n x k, any full-column-rank basis (only its span matters), None or
    k = 0 for no deflation; probes: n x p.  Returns b, b_defl = tr(Q^T A Q),
    b_tail, the p terms (P u_j)^T A (P u_j), and the standard error of
    b_tail, weight * sqrt(p) * (sample standard deviation of the terms)
    (NaN for p < 2)."""
    A = mat_exp(Mt)
    n = A.shape[0]
    U = np.asarray(probes, dtype=np.float64).reshape(n, -1)
    if Q is None or np.asarray(Q).size == 0:
        Qo = np.zeros((n, 0))
    else:
        Qo, _ = np.linalg.qr(np.asarray(Q, dtype=np.float64).reshape(n, -1))
    b_defl = float(np.trace(Qo.T @ A @ Qo))
    PU = U - Qo @ (Qo.T @ U)
    terms = np.einsum("ij,ij->j", PU, A @ PU)
    p = terms.size
    b_tail = float(weight) * float(np.sum(terms))
    se = float(weight) * math.sqrt(p) * float(np.std(terms, ddof=1)) if p >= 2 else float("nan")
    return {"b": b_defl + b_tail, "b_defl": b_defl, "b_tail": b_tail, "terms": terms, "stderr": se}


def certificate_from_log_b(mu_r1: float, log_b: float, r: int, eps: float, n: int) -> float:
    """log((n - r) lambda_{r+1}(Y) / (eps b)) with lambda_{r+1}(Y) = exp(mu_{r+1})
    and a given log b (Section 3.1.1): the certificate for an estimate of b_n."""
    return math.log(n - r) + float(mu_r1) - math.log(eps) - float(log_b)


# ---------------------------------------------------------------------------
# comparisons of factored iterates (FP64, no n x n matrix)
# ---------------------------------------------------------------------------
def factored_frob(V: np.ndarray, d: np.ndarray, alpha: float) -> float:
    """||alpha I + V diag(d) V^T||_F without forming the matrix."""
    return factored_diff_frob(V, d, alpha, np.zeros((np.asarray(V).shape[0], 0)), np.zeros(0), 0.0)


def factored_diff_frob(Va, da, aa, Vb, db, ab) -> float:
    """||X_a - X_b||_F for X = alpha I + V diag(d) V^T without forming X.

    Compares iterates, not eigenvectors: V is defined only up to sign and
    rotation inside equal eigenvalues, X is not.  With U = [V_a V_b] = Q R
    (thin QR) and D = diag(d_a, -d_b), X_a - X_b = dA I + Q (R D R^T) Q^T, so
    the norm splits into the 2r x 2r block dA I + R D R^T (formed entry by
    entry) and dA on the n - 2r dimensional complement.  No difference of
    squared norms is taken, so nearly equal iterates are resolved to rounding
    level rather than to its square root."""
    Va = np.asarray(Va, dtype=np.float64)
    Vb = np.asarray(Vb, dtype=np.float64)
    n = Va.shape[0]
    U = np.concatenate([Va, Vb], axis=1)
    D = np.concatenate([np.asarray(da, dtype=np.float64), -np.asarray(db, dtype=np.float64)])
    dA = float(aa) - float(ab)
    if U.shape[1] == 0:
        return math.sqrt(n) * abs(dA)
    Q, R = np.linalg.qr(U)
    K = (R * D) @ R.T + dA * np.eye(R.shape[0])
    rest = max(n - R.shape[0], 0)
    return math.sqrt(float(np.sum(K * K)) + rest * dA * dA)
