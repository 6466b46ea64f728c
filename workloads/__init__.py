"""Seeded synthetic inputs for the low-rank MEG workloads.

This module only *generates data*: objective matrices, observation masks,
measurement pools, starting points and arrival streams.  It holds none of the
MEG method's arithmetic (no gradient step, no matrix logarithm/exponential, no
eigen-solver of the iteration, no certificate), so that the FP64 oracle under
``oracle/`` and the HIP path can both be fed from it without sharing code.

Every generator draws from ``numpy.random.default_rng([tag, seed, ...])`` so a
workload is fully determined by its arguments.  Data that the GPU consumes in
FP32 is rounded to FP32 *here*, once; the oracle receives exactly the same
rounded values (as float64), so both sides solve the same problem.

Shapes follow the experiments and problem statement of Garber & Kaplan,
"On the Efficient Implementation of the Matrix Exponentiated Gradient
Algorithm for Low-Rank Matrix Optimization" (arXiv 2012.10469):

* spiked denoising      f(X) = 1/2 ||X - M||_F^2,  M = s*u u^T + noise
* matrix completion     f(X) = 1/2 sum_Omega (X_ij - M_ij)^2, M = W W^T / tr
* low-rank + noise      f(X) = 1/2 ||X - M||_F^2,  M = W W^T/||W||_F^2 + noise
* linear                f(X) = <C, X>          (closed-form test instances)
* quadratic measurements (stochastic)  f(X) = 1/(2m) sum_i (a_i^T X a_i - b_i)^2

The warm start of Section 7 (the initialisation equation of the experiments)
is input preparation and is computed here in FP64 with its own simplex
projection; see ``exp_init_from_operator``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional

import numpy as np

__all__ = [
    "rng",
    "DenseProblem",
    "CSRProblem",
    "spiked_denoise",
    "lowrank_noise_denoise",
    "matrix_completion",
    "linear_aligned",
    "linear_csr_diag",
    "top1_start",
    "exp_init_from_operator",
    "exp_init_dense",
    "exp_init_csr",
    "gaussian_columns",
    "serving_stream",
    "quadmeas_problem",
]


def rng(*key: int) -> np.random.Generator:
    """Seeded PCG64 generator keyed by a tuple of non-negative integers."""
    return np.random.default_rng([int(k) for k in key])


# ---------------------------------------------------------------------------
# containers
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class DenseProblem:
    """Dense symmetric data matrix (n x n, row-major) for the linear or the
    denoising objective.  ``M`` already carries the working precision's
    rounding (float32 for the FP32/mixed paths)."""

    kind: str  # "denoise" or "linear"
    M: np.ndarray
    V0: np.ndarray  # n x q starting basis, float64
    lam0: np.ndarray  # q weights, float64, >= 0, sum 1

    @property
    def n(self) -> int:
        return self.M.shape[0]


@dataclasses.dataclass
class CSRProblem:
    """Symmetric sparse data on a symmetric pattern Omega, CSR, sorted columns.

    ``kind`` is "masked" (f = 1/2 sum_Omega (X_ij - M_ij)^2) or "linear"
    (f = <C, X> with C supported on Omega)."""

    kind: str
    n: int
    row_ptr: np.ndarray  # int32[n+1]
    col: np.ndarray  # int32[nnz]
    val: np.ndarray  # float32 or float64 [nnz]
    V0: np.ndarray
    lam0: np.ndarray
    factor: Optional[np.ndarray] = None  # generating factor W (diagnostics only)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def rows(self) -> np.ndarray:
        """Row index of every stored entry (int64)."""
        return np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))


# ---------------------------------------------------------------------------
# helpers
# ---------------------------------------------------------------------------
def _sym_noise(g: np.random.Generator, n: int) -> np.ndarray:
    """(G + G^T)/sqrt(2n) with G i.i.d. N(0,1): spectrum on [-2, 2] (semicircle)."""
    G = g.standard_normal((n, n))
    return (G + G.T) / math.sqrt(2.0 * n)


def _round(A: np.ndarray, dtype) -> np.ndarray:
    return np.ascontiguousarray(A.astype(dtype))


def gaussian_columns(n: int, k: int, *key: int) -> np.ndarray:
    """n x k standard Gaussian block (float64), e.g. to seed solver columns."""
    return rng(*key).standard_normal((n, k))


def _simplex_projection(z: np.ndarray, tau: float) -> np.ndarray:
    """Euclidean projection of z onto {x >= 0, sum x = tau} (sort-and-threshold).

    Used only to build the paper's warm start; independent of the oracle's
    spectrahedron projection."""
    z = np.asarray(z, dtype=np.float64)
    s = np.sort(z)[::-1]
    cs = np.cumsum(s) - tau
    idx = np.arange(1, z.size + 1)
    ok = s - cs / idx > 0
    rho = int(np.nonzero(ok)[0][-1])
    theta = cs[rho] / (rho + 1.0)
    return np.maximum(z - theta, 0.0)


def top1_start(M: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """X0 = v1 v1^T with v1 the top eigenvector of the data matrix (q = 1)."""
    A = np.asarray(M, dtype=np.float64)
    n = A.shape[0]
    if n <= 2500:
        w, U = np.linalg.eigh(A)
        v = U[:, -1]
    else:  # pragma: no cover - large inputs
        from scipy.sparse.linalg import eigsh

        w, U = eigsh(A, k=1, which="LA")
        v = U[:, 0]
    return v.reshape(n, 1).copy(), np.ones(1)


def exp_init_from_operator(
    matvec: Callable[[np.ndarray], np.ndarray], n: int, r: int, tau: float = 1.0, seed: int = 0
) -> tuple[np.ndarray, np.ndarray]:
    """Warm start of the experiments (Section 7, initialisation equation).

    X0 = V_r diag(P_simplex(lambda_r)) V_r^T with (V_r, lambda_r) the top-r
    eigenpairs of -grad f(tau U U^T); the caller passes ``matvec`` = the
    action of -grad f(tau U U^T).  Reading (the printed formula negates the
    eigenvalues once more, which would favour the smallest of the top-r
    eigenvalues): the top-r eigenvalues of -grad f are projected onto the
    tau-simplex.  Zero weights are kept (rank-deficient X0 is allowed by the
    factored form).  Returns (V0 n x r, lam0 r) in float64, sum(lam0) = 1.
    """
    from scipy.sparse.linalg import LinearOperator, eigsh

    op = LinearOperator((n, n), matvec=matvec, dtype=np.float64)
    v0 = rng(9000, seed).standard_normal(n)
    w, U = eigsh(op, k=r, which="LA", v0=v0, tol=1e-12, maxiter=20000)
    order = np.argsort(w)[::-1]
    w, U = w[order], U[:, order]
    lam = _simplex_projection(w, tau) / tau
    return np.ascontiguousarray(U), lam


def _unit_frob_gaussian(n: int, r: int, *key: int) -> np.ndarray:
    U = rng(*key).standard_normal((n, r))
    return U / np.linalg.norm(U)


def exp_init_dense(M: np.ndarray, r: int, seed: int, tau: float = 1.0):
    """Warm start for f = 1/2||X - M||^2: -grad f(tau UU^T) = M - tau U U^T."""
    n = M.shape[0]
    U = _unit_frob_gaussian(n, r, 9100, seed)
    A = np.asarray(M, dtype=np.float64)

    def mv(x):
        x = np.asarray(x, dtype=np.float64).reshape(-1)
        return A @ x - tau * (U @ (U.T @ x))

    return exp_init_from_operator(mv, n, r, tau, seed)


def exp_init_csr(p: "CSRProblem", r: int, seed: int, tau: float = 1.0):
    """Warm start for f = 1/2 sum_Omega (X_ij - M_ij)^2:
    -grad f(tau UU^T) = P_Omega(M - tau U U^T) (sparse, symmetric)."""
    import scipy.sparse as sp

    n = p.n
    U = _unit_frob_gaussian(n, r, 9200, seed)
    rows = p.rows()
    cols = p.col.astype(np.int64)
    uu = np.einsum("ij,ij->i", U[rows], U[cols])
    vals = p.val.astype(np.float64) - tau * uu
    A = sp.csr_matrix((vals, cols, p.row_ptr.astype(np.int64)), shape=(n, n))
    return exp_init_from_operator(lambda x: A @ np.asarray(x).reshape(-1), n, r, tau, seed)


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------
def spiked_denoise(n: int, seed: int, spike: float = 1.0, noise: float = 0.01,
                   dtype=np.float64, start: str = "top1", r: int = 1) -> DenseProblem:
    """M = spike * u u^T + noise * (G + G^T)/sqrt(2n), u unit Gaussian.

    spike = 1: the plain n = 200 FP64 workload (rank-1 signal plus noise,
    top-1 eigenvector warm start).  spike = 2: the gapped variant for which the
    optimum is rank one with a strict-complementarity gap close to 1.
    """
    g = rng(1, seed, n)
    u = g.standard_normal(n)
    u /= np.linalg.norm(u)
    M = spike * np.outer(u, u) + noise * _sym_noise(g, n)
    M = 0.5 * (M + M.T)
    M = _round(M, dtype)
    if start == "top1":
        V0, lam0 = top1_start(M)
    else:
        V0, lam0 = exp_init_dense(M, r, seed)
    return DenseProblem("denoise", M, V0, lam0)


def lowrank_noise_denoise(n: int, rank: int, seed: int, noise: float = 1e-3, r: int = 16,
                          dtype=np.float32, start: str = "exp") -> DenseProblem:
    """M = W W^T / ||W||_F^2 + noise * (G + G^T)/sqrt(2n), W n x rank Gaussian
    (the n = 16384 precision-form workload at full size)."""
    g = rng(4, seed, n)
    W = g.standard_normal((n, rank))
    M = (W @ W.T) / np.sum(W * W)
    if noise:
        M += noise * _sym_noise(g, n)
    M = 0.5 * (M + M.T)
    M = _round(M, dtype)
    if start == "exp":
        V0, lam0 = exp_init_dense(M, r, seed)
    else:
        V0, lam0 = top1_start(M)
    return DenseProblem("denoise", M, V0, lam0)


def bf16_planes(M: np.ndarray, ld: Optional[int] = None) -> tuple[np.ndarray, np.ndarray]:
    """Split a float32 matrix into bf16 planes hi + lo (bit patterns as uint16,
    rows padded with zeros to ``ld`` columns): hi = bf16(M), lo = bf16(M - hi),
    both rounded to nearest even.  This is the input format of the
    matrix-core (F32_BF16X3) form; ``planes_value(hi, lo)`` is the matrix it
    represents."""
    M = np.ascontiguousarray(M, dtype=np.float32)
    n, m = M.shape
    ld = m if ld is None else ld

    def rne(x):
        u = x.view(np.uint32).astype(np.uint64)
        u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
        return u.astype(np.uint16)

    hi = rne(M)
    lo = rne((M - (hi.astype(np.uint32) << 16).view(np.float32)).astype(np.float32))
    H = np.zeros((n, ld), np.uint16)
    L = np.zeros((n, ld), np.uint16)
    H[:, :m] = hi
    L[:, :m] = lo
    return H, L


def planes_value(hi: np.ndarray, lo: np.ndarray, cols: Optional[int] = None) -> np.ndarray:
    """The float64 matrix hi + lo of two bf16 planes (exact)."""
    f = lambda p: (p.astype(np.uint32) << 16).view(np.float32).astype(np.float64)  # noqa: E731
    V = f(hi) + f(lo)
    return V if cols is None else V[:, :cols]


def _symmetric_bernoulli_pattern(n: int, p: float, g: np.random.Generator):
    """Upper triangle (diagonal included) Bernoulli(p), mirrored; CSR arrays."""
    rows_l, cols_l = [], []
    # draw row by row to keep memory at O(n) per row
    for i in range(n):
        m = g.random(n - i) < p
        js = np.nonzero(m)[0] + i
        rows_l.append(np.full(js.size, i, dtype=np.int64))
        cols_l.append(js.astype(np.int64))
    ru = np.concatenate(rows_l)
    cu = np.concatenate(cols_l)
    off = ru != cu
    rr = np.concatenate([ru, cu[off]])
    cc = np.concatenate([cu, ru[off]])
    order = np.lexsort((cc, rr))
    rr, cc = rr[order], cc[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, rr + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return row_ptr.astype(np.int32), cc.astype(np.int32), rr


def matrix_completion(n: int, seed: int, rank: int = 5, p: float = 0.1, r: int = 10,
                      dtype=np.float32, start: str = "exp") -> CSRProblem:
    """Matrix-completion-style objective: M = W W^T / tr(W W^T) (W n x rank
    Gaussian), symmetric Bernoulli(p) mask with the diagonal, CSR, M_Omega in
    ``dtype``.  Warm start: the experiments' initialisation (tau = 1)."""
    g = rng(2, seed, n)
    W = g.standard_normal((n, rank))
    W /= math.sqrt(np.sum(W * W))  # tr(W W^T) = 1 after scaling
    row_ptr, col, rows = _symmetric_bernoulli_pattern(n, p, g)
    vals = np.einsum("ij,ij->i", W[rows], W[col.astype(np.int64)])
    vals = _round(vals, dtype)
    prob = CSRProblem("masked", n, row_ptr, col, vals, np.zeros((n, 0)), np.zeros(0), factor=W)
    if start == "exp":
        prob.V0, prob.lam0 = exp_init_csr(prob, r, seed)
    return prob


def linear_aligned(n: int, r: int, seed: int, c_top: Optional[np.ndarray] = None,
                   c_gap: float = 4.0, c_rest_scale: float = 1.0, dtype=np.float64,
                   lam0: Optional[np.ndarray] = None) -> tuple[DenseProblem, np.ndarray, np.ndarray]:
    """Linear objective f = <C, X>, C = U diag(c) U^T with U Haar-orthogonal.

    The r smallest eigenvalues c_1..c_r are spread on [0, 1]; the others lie in
    [c_gap, c_gap + c_rest_scale].  The start V0 = U[:, :r] spans the bottom-r
    eigenvectors (the aligned start of the closed-form test).  Returns
    (problem, U, c)."""
    g = rng(6, seed, n)
    A = g.standard_normal((n, n))
    U, R = np.linalg.qr(A)
    U = U * np.sign(np.diag(R))
    if c_top is None:
        c_top = np.sort(g.random(r))
    rest = c_gap + c_rest_scale * g.random(n - r)
    c = np.concatenate([np.asarray(c_top, dtype=np.float64), rest])
    C = (U * c) @ U.T
    C = 0.5 * (C + C.T)
    C = _round(C, dtype)
    if lam0 is None:
        lam0 = np.full(r, 1.0 / r)
    return DenseProblem("linear", C, np.ascontiguousarray(U[:, :r]), np.asarray(lam0, float)), U, c


def linear_csr_diag(n: int, r: int, seed: int, c_gap: float = 4.0, dtype=np.float64,
                    permute: bool = True) -> tuple[CSRProblem, np.ndarray]:
    """Linear objective with a (permuted) diagonal C stored as CSR: C = P diag(c) P^T.

    The bottom-r eigenvectors are coordinate vectors e_{perm[i]}, so the
    aligned start is V0 = [e_perm[0], ..., e_perm[r-1]].  Returns (problem, c)
    where c is indexed by coordinate."""
    g = rng(7, seed, n)
    c_sorted = np.concatenate([np.sort(g.random(r)), c_gap + g.random(n - r)])
    perm = g.permutation(n) if permute else np.arange(n)
    c = np.empty(n)
    c[perm] = c_sorted
    row_ptr = np.arange(n + 1, dtype=np.int32)
    col = np.arange(n, dtype=np.int32)
    val = _round(c, dtype)
    V0 = np.zeros((n, r))
    V0[perm[:r], np.arange(r)] = 1.0
    prob = CSRProblem("linear", n, row_ptr, col, val, V0, np.full(r, 1.0 / r))
    return prob, val.astype(np.float64)


def serving_stream(count: int, seed: int, sizes=(256, 512, 1024, 2048), r_max: int = 8,
                   rate_hz: float = 200.0):
    """Request stream of independent spiked-denoising instances.

    n uniform over ``sizes``, r uniform over {1..r_max}, Poisson arrivals at
    ``rate_hz`` (exponential inter-arrival times).  Returns a list of dicts
    with keys id, n, r, seed, t_arrive (seconds)."""
    g = rng(5, seed)
    ns = g.choice(np.asarray(sizes), size=count)
    rs = g.integers(1, r_max + 1, size=count)
    gaps = g.exponential(1.0 / rate_hz, size=count)
    t = np.cumsum(gaps) - gaps[0]
    return [dict(id=i, n=int(ns[i]), r=int(rs[i]), seed=int(1000 + i), t_arrive=float(t[i]))
            for i in range(count)]


def quadmeas_problem(n: int, m: int, seed: int, rank: int = 3, dtype=np.float32):
    """Quadratic measurements b_i = a_i^T X* a_i, X* = F F^T/||F||_F^2
    (F n x rank Gaussian), pool A (n x m, column i = a_i) Gaussian.

    Host-side generator for small pools (tests).  Returns (A, b, Xstar_factor)."""
    g = rng(3, seed, n)
    F = g.standard_normal((n, rank))
    F /= np.linalg.norm(F)
    A = _round(g.standard_normal((n, m)), dtype)
    Af = A.astype(np.float64)
    proj = F.T @ Af  # rank x m
    b = _round(np.sum(proj * proj, axis=0), dtype)
    return A, b, F


def quadmeas_rows(n: int, m: int, seed: int, rank: int = 3, dtype=np.float32, lda: Optional[int] = None):
    """The pool of ``quadmeas_problem`` in the library's layout: an m x lda
    array whose row i is a_i (columns n..lda-1 zero), with b and the factor
    F of X* = F F^T (||F||_F = 1)."""
    A, b, F = quadmeas_problem(n, m, seed, rank, dtype)
    lda = n if lda is None else lda
    rows = np.zeros((m, lda), dtype=A.dtype)
    rows[:, :n] = A.T
    return rows, b, F


def quadmeas_batches(m: int, L: int, steps: int, seed: int) -> np.ndarray:
    """Minibatch indices: `steps` rows of L draws, uniform with replacement
    over the pool (int32)."""
    return rng(3, 1, seed).integers(0, m, size=(steps, L)).astype(np.int32)


def exp_init_quadmeas(rows: np.ndarray, b: np.ndarray, n: int, r: int, seed: int, tau: float = 1.0):
    """Warm start (Section 7, initialisation equation) for quadratic
    measurements, with the gradient taken over the given sample of
    measurements (rows: s x >=n, row i = a_i):
    -grad f(tau U U^T) = (1/s) sum_i (b_i - tau a_i^T U U^T a_i) a_i a_i^T."""
    Ar = np.asarray(rows[:, :n], dtype=np.float64)
    U = _unit_frob_gaussian(n, r, 9300, seed)
    proj = Ar @ U
    w = (np.asarray(b, dtype=np.float64) - tau * np.sum(proj * proj, axis=1)) / Ar.shape[0]

    def mv(x):
        x = np.asarray(x, dtype=np.float64).reshape(-1)
        return Ar.T @ (w * (Ar @ x))

    return exp_init_from_operator(mv, n, r, tau, seed)


@dataclasses.dataclass
class BilinearProblem:
    """The recovery problem of the experiments (Section 7): ground truth
    M = (sqrt(n) W)(sqrt(n) W)^T, W n x rank Gaussian with ||W||_F = 1 (so
    tr M = n); m = 20 n rank pairs (a_i, b_i) of uniform unit vectors;
    y = y0 + kappa ||y0|| v with y0_i = a_i^T M b_i and v a uniform unit vector;
    trace bound tau (0.5 tr M for rank 1 and 5, 0.65 tr M for rank 20);
    smoothness beta = 0.4 sqrt(rank n), step size 1/beta.

    The unit-trace method runs on X' = X / tau: f(tau X') has the gradient
    tau * grad g(X') with g the same objective on y' = y / tau, so the
    library and the oracle take y' and the step size tau / beta."""
    n: int
    rank: int
    A: np.ndarray       # m x n, rows a_i (p = 1), or m x p x n, A[i, q] = column q of A_i
    B: np.ndarray       # likewise for b_i / B_i
    y: np.ndarray       # m, the noisy measurements
    M: np.ndarray       # n x n ground truth
    tau: float
    beta: float
    U: np.ndarray       # n x rank, the start's Gaussian block (||U||_F = 1)

    @property
    def m(self) -> int:
        return self.A.shape[0]

    @property
    def p(self) -> int:
        return 1 if self.A.ndim == 2 else self.A.shape[1]

    def _flat(self, Z: np.ndarray) -> np.ndarray:
        return Z.reshape(-1, self.n)

    @property
    def y_unit(self) -> np.ndarray:
        return self.y / self.tau

    @property
    def eta_unit(self) -> float:
        return self.tau / self.beta


def bilinear_recovery(n: int, rank: int, seed: int, kappa: float = 0.5, r: Optional[int] = None,
                      m_rank: Optional[int] = None, p: int = 1, beta_coeff: float = 0.4) -> BilinearProblem:
    """``r``: the rank parameter when it exceeds rank(M) (the start's block U
    has r columns; Table 3); ``m_rank``: the rank in m = 20 n m_rank
    (default rank(M)); ``p`` > 1: measurement matrices A_i, B_i (n x p) with
    orthonormal columns, y0_i = tr(A_i^T M B_i) (Table 4, which also takes
    beta = 12 sqrt(r n): ``beta_coeff`` = 12)."""
    r = rank if r is None else r
    g = rng(11, seed, n, rank)
    W_ = g.standard_normal((n, rank))
    W_ /= np.linalg.norm(W_)
    M = n * (W_ @ W_.T)
    m = 20 * n * (rank if m_rank is None else m_rank)
    if p == 1:
        A = g.standard_normal((m, n))
        A /= np.linalg.norm(A, axis=1, keepdims=True)
        B = g.standard_normal((m, n))
        B /= np.linalg.norm(B, axis=1, keepdims=True)
        y0 = np.sum((A @ M) * B, axis=1)
    else:
        A = np.swapaxes(np.linalg.qr(g.standard_normal((m, n, p)))[0], 1, 2).copy()  # m x p x n
        B = np.swapaxes(np.linalg.qr(g.standard_normal((m, n, p)))[0], 1, 2).copy()
        y0 = np.sum((A.reshape(-1, n) @ M) * B.reshape(-1, n), axis=1).reshape(m, p).sum(axis=1)
    v = g.standard_normal(m)
    v /= np.linalg.norm(v)
    y = y0 + kappa * np.linalg.norm(y0) * v
    tau = (0.65 if rank >= 20 else 0.5) * float(np.trace(M))
    U = g.standard_normal((n, r))
    U /= np.linalg.norm(U)
    return BilinearProblem(n, rank, A, B, y, M, tau, beta_coeff * math.sqrt(r * n), U)


def exp_init_bilinear(p: BilinearProblem, r: int):
    """Warm start (Section 7, initialisation equation) of the recovery
    problem, as printed: (V_r, Lambda_r) the top-r eigenpairs of
    -grad f(tau U U^T) (symmetric part), weights the projection of -Lambda_r
    onto the tau-simplex, divided by tau.  The sign as printed favours the
    smallest of the r eigenvalues; Table 1's initialisation errors (rank 5
    and 20) match it and not the other sign."""
    X = p.tau * (p.U @ p.U.T)
    A2, B2 = p._flat(p.A), p._flat(p.B)
    res = np.sum((A2 @ X) * B2, axis=1).reshape(p.m, p.p).sum(axis=1) - p.y
    H = A2.T @ (np.repeat(res, p.p)[:, None] * B2)
    Gm = -0.5 * (H + H.T)
    w, Q = np.linalg.eigh(Gm)
    w, Q = w[::-1][:r], Q[:, ::-1][:, :r]
    lam = _simplex_projection(-w, p.tau) / p.tau
    return np.ascontiguousarray(Q), lam


def bilinear_rows(p: BilinearProblem, dtype=np.float32, lda: Optional[int] = None) -> np.ndarray:
    """The library's layout of the measurement vectors: 2mp rows of length
    lda >= n (columns n..lda-1 zero); row i p + q is column q of A_i (a_i for
    p = 1), row m p + i p + q column q of B_i."""
    lda = p.n if lda is None else lda
    mp = p.m * p.p
    rows = np.zeros((2 * mp, lda), dtype=dtype)
    rows[:mp, : p.n] = p._flat(p.A)
    rows[mp:, : p.n] = p._flat(p.B)
    return rows


def quadmeas_pool_device(n: int, m: int, seed: int, rank: int = 3, chunk: int = 1 << 16):
    """Full-size pool generated on the GPU (torch's counter-based generator,
    seeded): A (m x n float32, row i = a_i, standard Gaussian), b_i =
    a_i^T X* a_i with X* = F F^T, F n x rank Gaussian with ||F||_F = 1 (drawn
    on the host), b accumulated in float64 and rounded to float32.
    Returns (A, b, F) with A and b on the device."""
    import torch

    g = torch.Generator(device="cuda")
    g.manual_seed(int(rng(3, 2, seed).integers(0, 2**62)))
    F = rng(3, 3, seed).standard_normal((n, rank))
    F /= np.linalg.norm(F)
    A = torch.empty((m, n), dtype=torch.float32, device="cuda")
    b = torch.empty((m,), dtype=torch.float32, device="cuda")
    Fd = torch.as_tensor(F, dtype=torch.float64, device="cuda")
    for i0 in range(0, m, chunk):
        i1 = min(m, i0 + chunk)
        A[i0:i1].normal_(generator=g)
        P = A[i0:i1].to(torch.float64) @ Fd
        b[i0:i1] = (P * P).sum(dim=1).to(torch.float32)
    return A, b, F


def spiked_denoise_device(n: int, seed: int, spike: float = 1.0, noise: float = 0.01, power_iters: int = 30):
    """The plain-configuration denoising instance drawn on the GPU (torch's
    seeded generator): M = spike u u^T + noise (G + G^T)/sqrt(2n) in FP32,
    u a unit Gaussian vector.  Also returns the warm start of that
    configuration, the top eigenvector of M, by power iteration from u (the
    spike's gap makes a few dozen products enough).
    Returns (M on the device, v0 host float64 n x 1)."""
    import torch

    gen = torch.Generator(device="cuda")
    gen.manual_seed(int(rng(5, 1, seed).integers(0, 2**62)))
    u = torch.randn(n, generator=gen, device="cuda", dtype=torch.float64)
    u /= torch.linalg.norm(u)
    G = torch.randn((n, n), generator=gen, device="cuda", dtype=torch.float32)
    M = (G + G.T) * (noise / math.sqrt(2.0 * n))
    M += (spike * torch.outer(u, u)).to(torch.float32)
    v = u.clone()
    Md = M.to(torch.float64)
    for _ in range(power_iters):
        v = Md @ v
        v /= torch.linalg.norm(v)
    return M.contiguous(), v.cpu().numpy().reshape(n, 1)
