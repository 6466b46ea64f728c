"""Benchmark: low-rank MEG iterations/s on one MI355X.

Default workload: the matrix-completion objective at n = 4096, rank-5 ground
truth, symmetric Bernoulli(0.1) mask (~1.68M stored entries, CSR), rank
parameter r = 10, FP32 state, warm start of the paper's experiments.  One
"step" is one full iteration t -> t+1 of the low-rank MEG method (gradient on
the mask, warm-started block subspace iteration with Rayleigh-Ritz,
exponentiation/normalisation, certificate).

Prints ONE JSON line: metric/value/unit, ms_per_step, a roofline object for
the step kernel (the only kernel in the timed region; its average launch time
comes from the library's HIP event pair around every launch on the context's
stream, its algorithmic bytes from the iterations and operator applies the
launches performed) and the FP64 CPU oracle timed on a bounded sample of the
same workload.

The same line carries a "serving" object: the batched server on a stream of
plain-configuration instances (Poisson arrivals, then saturation), against
the single-instance FP32 path on a sample (`--no-serving` skips it).

A "recovery" object times the paper's own workload (Section 7's recovery
problem from bilinear measurements, full gradients, FP32 state) at Table 1's
largest rank-5 size, n = 600 (m = 60000 measurement pairs), against the FP64
oracle on a sample of iterations (`--no-recovery` skips it).

Three more objects cover the other configurations: "config1" (the plain
method, FP64, n = 200, r = 5, 100 iterations: iterations/s and the FP64
error against the oracle), "config3" (stochastic gradients, n = 8192, a pool
of 10^6 measurements on the device, L = 256, r = 8: iterations/s with the
count of steps whose inner solve did not converge) and "precision" (n = 16384
dense denoising, r = 16: the BF16x3 matrix-core apply against the plain FP32
apply, each with its FP64 error against the FP64 path on the same matrix);
`--no-configs` skips them.

`--write-workload PATH` only writes the workload for the native driver
paper_2012_10469_amd/meg_bench (used under rocprofv3) and exits;
`--write-dense-workload PATH` writes the precision-form workload of the same
driver (n = 16384, r = 16, M = W W^T/||W||_F^2 + 1e-3 symmetric noise split
into bf16 planes, top-eigenvector start) and exits; `--write-bilinear-workload
PATH` writes the recovery workload (n = 600, rank 5) of the same driver.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published

# HBM traffic of the timed launch of the step kernel on the default workload
# in the default launch configuration (20 iterations in one launch after 5
# warmup iterations), from rocprofv3 FETCH_SIZE / WRITE_SIZE runs scaled by a
# plain copy's readings (profiles/k_step_matrix_completion_n4096_r10_traffic.md);
# valid only for the kernel sources and the launch it was measured on.
TRAFFIC = {"bytes_per_launch": 151.1e6, "iterations_per_launch": 20, "warmup": 5, "applies_per_iteration": 2.0,
           "fetch_bytes": 90.6e6, "write_bytes": 60.5e6, "fetch_factor": 2.0, "write_factor": 1.0,
           "source_hash": "3a81338834665f7d"}
KERNEL_SOURCES = ["meg_device.hpp", "meg_small.hpp", "meg_kernels.hpp", "meg_api.hip"]


def kernel_source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2012_10469_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def matrix_completion_workload(n: int, r: int, seed: int):
    import numpy as np

    import workloads as W

    t0 = time.time()
    p = W.matrix_completion(n, seed=seed, rank=5, p=0.1, r=r, dtype=np.float32)
    log(f"[bench] workload n={n} nnz={p.nnz} r={r} generated in {time.time() - t0:.1f}s")
    return p


def apply_bytes(n: int, nnz: int, k: int, es: int, first: bool) -> int:
    """Algorithmic HBM bytes of one sweep of the CSR operator apply: every
    stored entry's column index and value once (the first sweep of a step
    reads M_Omega and writes the gradient values; later sweeps read them
    back), the row pointers, the input block Zin and the basis block B (the
    same block in the first sweep) read once, and the output block written
    once."""
    if first:
        return nnz * (4 + 2 * es) + 4 * (n + 1) + 2 * n * k * es
    return nnz * (4 + es) + 4 * (n + 1) + 3 * n * k * es


def step_bytes(n: int, nnz: int, k: int, es: int, sweeps: float) -> float:
    """Algorithmic HBM bytes of one iteration with `sweeps` operator applies
    (the first one forms the gradient; the step has no other pass over the
    data or the n x k blocks)."""
    return apply_bytes(n, nnz, k, es, True) + (sweeps - 1.0) * apply_bytes(n, nnz, k, es, False)


def write_workload(p, r: int, path: str) -> None:
    """Binary workload of the native driver (layout in csrc/meg_bench.cpp)."""
    import numpy as np

    V0 = np.asarray(p.V0, dtype=np.float64)
    lam0 = np.asarray(p.lam0, dtype=np.float64)
    if V0.ndim == 1:
        V0 = V0[:, None]
    with open(path, "wb") as f:
        f.write(b"MEGW0001")
        f.write(np.array([p.n, p.nnz], dtype="<i8").tobytes())
        f.write(np.array([r, V0.shape[1]], dtype="<i4").tobytes())
        f.write(np.ascontiguousarray(p.row_ptr, dtype="<i4").tobytes())
        f.write(np.ascontiguousarray(p.col, dtype="<i4").tobytes())
        f.write(np.ascontiguousarray(p.val, dtype="<f4").tobytes())
        f.write(np.asfortranarray(V0, dtype="<f8").tobytes(order="F"))
        f.write(np.ascontiguousarray(lam0, dtype="<f8").tobytes())


def write_dense_workload(path: str, n: int = 16384, r: int = 16, seed: int = 1) -> None:
    """Precision-form workload of the native driver: "MEGD0001", int64 n,
    int64 ld, int32 r, int32 q, uint16 hi[n*ld], uint16 lo[n*ld],
    double V0[n*q] (column-major), double lambda0[q]."""
    import numpy as np

    import workloads as W

    t0 = time.time()
    prob = W.lowrank_noise_denoise(n, rank=8, seed=seed, noise=1e-3, r=r, dtype=np.float32, start="top1")
    hi, lo = W.bf16_planes(prob.M)
    V0 = np.asarray(prob.V0, dtype=np.float64)
    if V0.ndim == 1:
        V0 = V0[:, None]
    with open(path, "wb") as f:
        f.write(b"MEGD0001")
        f.write(np.array([n, hi.shape[1]], dtype="<i8").tobytes())
        f.write(np.array([r, V0.shape[1]], dtype="<i4").tobytes())
        f.write(np.ascontiguousarray(hi, dtype="<u2").tobytes())
        f.write(np.ascontiguousarray(lo, dtype="<u2").tobytes())
        f.write(np.asfortranarray(V0, dtype="<f8").tobytes(order="F"))
        f.write(np.ascontiguousarray(prob.lam0, dtype="<f8").tobytes())
    log(f"[bench] dense workload n={n} written in {time.time() - t0:.1f}s")


def write_bilinear_workload(path: str, n: int = 600, rank: int = 5, seed: int = 0) -> None:
    """Recovery workload of the native driver: "MEGB0001", int64 n, int64 m,
    int32 r, int32 q, double eta, float A[2m*n] (rows a_1..a_m, b_1..b_m),
    float y[m] (y / tau), double V0[n*q] (column-major), double lambda0[q]."""
    import numpy as np

    import workloads as W

    p = W.bilinear_recovery(n, rank, seed)
    V0, lam0 = W.exp_init_bilinear(p, rank)
    with open(path, "wb") as f:
        f.write(b"MEGB0001")
        f.write(np.array([n, p.m], dtype="<i8").tobytes())
        f.write(np.array([rank, rank], dtype="<i4").tobytes())
        f.write(np.array([p.eta_unit], dtype="<f8").tobytes())
        f.write(np.ascontiguousarray(W.bilinear_rows(p, np.float32), dtype="<f4").tobytes())
        f.write(np.ascontiguousarray(p.y_unit, dtype="<f4").tobytes())
        f.write(np.asfortranarray(V0, dtype="<f8").tobytes(order="F"))
        f.write(np.ascontiguousarray(lam0, dtype="<f8").tobytes())
    log(f"[bench] bilinear workload n={n} m={p.m} written")


def recovery_bench(meg, torch, steps: int = 50, cpu_samples: int = 2, n: int = 600, rank: int = 5, seed: int = 0):
    """Section 7's recovery problem (bilinear measurements, full gradient) at
    n = 600, rank 5 (m = 60000): GPU iterations/s over `steps` iterations after
    5 warmup, the objective before and after, and the FP64 oracle's time per
    iteration on `cpu_samples` iterations from the same start."""
    import numpy as np

    import workloads as W

    p = W.bilinear_recovery(n, rank, seed)
    V0, lam0 = W.exp_init_bilinear(p, rank)
    A = torch.from_numpy(W.bilinear_rows(p, np.float32)).cuda()
    y = torch.from_numpy(p.y_unit.astype(np.float32)).cuda()
    g = meg.LowRankMEG(n, rank, meg.MEG_GRAD_BILINEAR, V0, lam0, prec=meg.MEG_PREC_F32, eta=p.eta_unit, A=A, b=y,
                       max_inner=40)
    try:
        f0 = g.objective()
        g.solve(5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        last = g.solve(steps)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        f1 = g.objective()
        cnt = g.counters(reset=False)
    finally:
        g.close()
    m = p.m
    # the gradient's n(n+1)/2 distinct entries take 4m flops each, the residuals 4 n rank flops per
    # measurement; both passes read the 2m measurement rows at least once
    flops = 2.0 * n * (n + 1) * m + 4.0 * m * n * rank
    nbytes = 2 * (2 * m * n * 4)
    from oracle import meg_oracle as O

    obj = O.BilinearObjective(p.A, p.B, p.y_unit)
    it = O.initial_iterate(V0, lam0, O.eps_schedule(0))
    c0 = time.perf_counter()
    for _ in range(cpu_samples):
        it, _ = O.lowrank_step(it, obj.grad(it.dense()), p.eta_unit, O.eps_schedule(it.t), rank, full=False)
    cpu_s = (time.perf_counter() - c0) / cpu_samples
    try:
        from threadpoolctl import threadpool_info

        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    out = {"workload": "recovery_bilinear", "n": n, "rank": rank, "m": m, "dtype": "f32", "steps": steps,
           "iter_per_s": steps / secs, "ms_per_iter": secs * 1e3 / steps,
           "applies_per_iter": cnt["applies"] / max(cnt["iterations"], 1),
           "objective_start": f0 * p.tau ** 2, "objective_end": f1 * p.tau ** 2, "t": last["t"],
           "cert_L": last["cert_L"], "gradient_flops_per_iter": flops, "measurement_bytes_per_iter": nbytes,
           "cpu_baseline": {"value": 1.0 / cpu_s, "unit": "iter/s", "cores": int(threads),
                            "kind": "oracle", "sample": f"{cpu_samples} iterations from the same start"}}
    log(f"[recovery] n={n} rank {rank} m={m}: {out['iter_per_s']:.1f} iter/s ({out['ms_per_iter']:.3f} ms), "
        f"f {out['objective_start']:.4e} -> {out['objective_end']:.4e}; oracle {1.0 / cpu_s:.2f} iter/s")
    return out


def _threads() -> int:
    try:
        from threadpoolctl import threadpool_info

        return int(max([i.get("num_threads", 1) for i in threadpool_info()] or [1]))
    except Exception:  # pragma: no cover
        return os.cpu_count() or 1


def config1_bench(meg, torch, T: int = 100):
    """The plain configuration: FP64, n = 200, M = u u^T + 0.01 (G + G^T)/sqrt(2n),
    r = 5, eta = 1, T = 100 iterations from the top eigenvector of M.  GPU
    iterations/s of the whole run (one 100-iteration meg_solve after a warmup
    context), its FP64 error against the oracle (every step from the oracle's
    iterate; the free-running final iterate), and the oracle's own time."""
    import numpy as np

    import workloads as W
    from oracle import meg_oracle as O

    n, r = 200, 5
    prob = W.spiked_denoise(n, seed=1, start="top1")
    M = torch.from_numpy(np.ascontiguousarray(prob.M)).cuda()
    kw = dict(prec=meg.MEG_PREC_F64, eta=1.0, dense=M, max_inner=64)
    with meg.LowRankMEG(n, r, meg.MEG_GRAD_DENOISE_DENSE, prob.V0, prob.lam0, **kw) as w:
        w.solve(5)
    with meg.LowRankMEG(n, r, meg.MEG_GRAD_DENOISE_DENSE, prob.V0, prob.lam0, **kw) as g:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.solve(T)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        cnt = g.counters()
        final = g.get_iterate()
        c0 = time.perf_counter()
        run = O.run_lowrank_meg(O.DenoiseObjective(prob.M), prob.V0, prob.lam0, r, 1.0, T)
        cpu_s = time.perf_counter() - c0
        tf = []
        for t in range(1, T + 1):
            st = run["states"][t - 1]
            g.set_iterate(st.V, st.d, st.alpha, t)
            g.step(info=False)
            V, d, a, _ = g.get_iterate()
            ref = run["states"][t]
            rel_gap = run["gap"][t - 1] / max(1.0, abs(run["mu"][t - 1][0] - run["mu"][t - 1][-1]))
            e = O.factored_diff_frob(V, d, a, ref.V, ref.d, ref.alpha) / O.factored_frob(ref.V, ref.d, ref.alpha)
            tf.append((e, rel_gap))
    ref = run["states"][T]
    fr = O.factored_diff_frob(*final[:3], ref.V, ref.d, ref.alpha) / O.factored_frob(ref.V, ref.d, ref.alpha)
    out = {"workload": "spiked_denoise_fp64", "n": n, "r": r, "iterations": T, "dtype": "f64",
           "iter_per_s": T / secs, "ms_per_iter": secs * 1e3 / T,
           "applies_per_iter": cnt["applies"] / cnt["iterations"], "unconverged": cnt["unconverged"],
           "error_vs_oracle": {"teacher_forced_max": max(e for e, gp in tf if gp >= 1e-3),
                               "steps_with_relative_gap_below_1e-3": sum(1 for _, gp in tf if gp < 1e-3),
                               "free_running_final": fr},
           "cpu_baseline": {"value": T / cpu_s, "unit": "iter/s", "cores": _threads(), "kind": "oracle",
                            "sample": f"the whole {T}-iteration run"}}
    log(f"[config1] n={n} r={r} FP64: {out['iter_per_s']:.0f} iter/s over {T} iterations "
        f"({out['applies_per_iter']:.2f} applies/iter); teacher-forced error {out['error_vs_oracle']['teacher_forced_max']:.1e}, "
        f"free-running {fr:.1e}; oracle {T / cpu_s:.1f} iter/s")
    return out


def config3_bench(meg, torch, steps: int = 200):
    """Stochastic gradients: n = 8192, pool of m = 10^6 Gaussian measurements
    (drawn on the device), minibatch L = 256, r = 8, eta = 1/(3 + n/L), from
    the experiments' warm start.  GPU iterations/s over `steps` iterations
    after 10 warmup, with the number of steps whose inner solve did not
    converge (max_inner 12); the oracle's time on one iteration."""
    import numpy as np

    import workloads as W
    from oracle import meg_oracle as O

    n, m, L, r, bsteps, seed = 8192, 1_000_000, 256, 8, 64, 3
    t0 = time.time()
    A, b, F = W.quadmeas_pool_device(n, m, seed)
    bi = W.quadmeas_batches(m, L, bsteps, seed)
    sample = A[:1024].cpu().numpy()
    V0, lam0 = W.exp_init_quadmeas(sample, b[:1024].cpu().numpy(), n, r, seed)
    eta = 1.0 / (3.0 + n / L)
    idx = torch.as_tensor(bi.astype(np.int32)).cuda()
    log(f"[config3] pool of {m} measurements (n={n}) and warm start in {time.time() - t0:.1f}s")
    try:
        g = meg.LowRankMEG(n, r, meg.MEG_GRAD_QUADMEAS, V0, lam0, prec=meg.MEG_PREC_F32, eta=eta, A=A, b=b,
                           batch_idx=idx, max_inner=12)
        g.solve(10)
        torch.cuda.synchronize()
        g.counters(reset=True)
        t0 = time.perf_counter()
        g.solve(steps)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        cnt = g.counters()
        V, d, a, t = g.get_iterate()
        g.close()
        # the oracle on one iteration (factored minibatch gradient, invariant-subspace eigensolve)
        it = O.FactoredIterate(V, d, a, t)
        rows = A[torch.as_tensor(bi[(t - 1) % bsteps].astype(np.int64)).cuda()].cpu().numpy().astype(np.float64)
        local = O.QuadMeasObjective(rows.T, b[torch.as_tensor(bi[(t - 1) % bsteps].astype(np.int64)).cuda()]
                                    .cpu().numpy().astype(np.float64))
        c0 = time.perf_counter()
        Fm, c = local.grad_factor(it, np.arange(L))
        O.lowrank_step_factored(it, Fm, c, eta, O.eps_schedule(t), r)
        cpu_s = time.perf_counter() - c0
    finally:
        del A, b
        torch.cuda.empty_cache()
    out = {"workload": "quadmeas_stochastic", "n": n, "m": m, "L": L, "r": r, "dtype": "f32", "steps": steps,
           "iter_per_s": steps / secs, "ms_per_iter": secs * 1e3 / steps,
           "applies_per_iter": cnt["applies"] / cnt["iterations"], "unconverged_steps": cnt["unconverged"],
           "converged": cnt["unconverged"] == 0,
           "cpu_baseline": {"value": 1.0 / cpu_s, "unit": "iter/s", "cores": _threads(), "kind": "oracle",
                            "sample": "1 iteration (factored gradient, exact invariant-subspace eigensolve)"}}
    log(f"[config3] {out['iter_per_s']:.0f} iter/s over {steps} iterations, {out['applies_per_iter']:.2f} "
        f"applies/iter, {cnt['unconverged']} unconverged steps; oracle {1.0 / cpu_s:.2f} iter/s")
    return out


def precision_bench(meg, torch, T: int = 20):
    """The precision form: n = 16384 dense denoising (M = rank-8 + 1e-3 noise),
    r = 16 (k = 32), T iterations from the top eigenvector of M, three ways:
    BF16x3 apply (the bf16 planes of M, FP32 state), the plain FP32 dense
    apply, and the FP64 path on the same matrix (the planes' value).  Reports
    iterations/s of the first two and their FP64 errors against the third
    (relative Frobenius of X_{T+1}, relative f, absolute cert_L)."""
    import numpy as np

    import workloads as W
    from oracle import meg_oracle as O

    n, r = 16384, 16
    t0 = time.time()
    prob = W.lowrank_noise_denoise(n, rank=8, seed=1, noise=1e-3, r=r, dtype=np.float32, start="top1")
    hi, lo = W.bf16_planes(prob.M)
    del prob.M
    Mp = W.planes_value(hi, lo, n)
    log(f"[precision] n={n} workload in {time.time() - t0:.1f}s")
    dhi = torch.from_numpy(hi.view(np.int16)).cuda()
    dlo = torch.from_numpy(lo.view(np.int16)).cuda()
    del hi, lo
    res = {}
    for name, kw in (("bf16x3", dict(prec=meg.MEG_PREC_F32_BF16X3, dense=dhi, dense_lo=dlo)),
                     ("f32", dict(prec=meg.MEG_PREC_F32, dense=torch.from_numpy(Mp.astype(np.float32)).cuda())),
                     ("f64", dict(prec=meg.MEG_PREC_F64, dense=torch.from_numpy(Mp).cuda()))):
        torch.cuda.synchronize()
        g = meg.LowRankMEG(n, r, meg.MEG_GRAD_DENOISE_DENSE, prob.V0, prob.lam0, eta=1.0, max_inner=40, **kw)
        try:
            g.solve(2)  # first iterations, kernels loaded
            torch.cuda.synchronize()
            g.counters(reset=True)
            t1 = time.perf_counter()
            g.solve(T - 2)
            torch.cuda.synchronize()
            secs = time.perf_counter() - t1
            cnt = g.counters()
            last = g.certificate()
            f = g.objective()
            res[name] = {"iter_per_s": (T - 2) / secs, "applies_per_iter": cnt["applies"] / cnt["iterations"],
                         "unconverged": cnt["unconverged"], "state": g.get_iterate(), "f": f,
                         "cert_L": last["cert_L"]}
        finally:
            g.close()
            del kw["dense"]
            torch.cuda.empty_cache()
    del dhi, dlo, Mp
    ref = res["f64"]
    Vr, dr, ar, _ = ref["state"]
    out = {"workload": "lowrank_noise_denoise_dense", "n": n, "r": r, "k": 32, "iterations": T,
           "reference": "the FP64 path on the same matrix (parity-tested against the oracle)"}
    for name in ("bf16x3", "f32"):
        V, d, a, _ = res[name]["state"]
        ex = O.factored_diff_frob(V, d, a, Vr, dr, ar) / O.factored_frob(Vr, dr, ar)
        out[name] = {"iter_per_s": res[name]["iter_per_s"], "applies_per_iter": res[name]["applies_per_iter"],
                     "unconverged": res[name]["unconverged"],
                     "fp64_error": {"X": ex, "f": abs(res[name]["f"] - ref["f"]) / abs(ref["f"]),
                                    "cert_L": abs(res[name]["cert_L"] - ref["cert_L"])}}
    out["f64"] = {"iter_per_s": ref["iter_per_s"], "applies_per_iter": ref["applies_per_iter"]}
    out["speedup_bf16x3_vs_f32"] = out["bf16x3"]["iter_per_s"] / out["f32"]["iter_per_s"]
    log(f"[precision] BF16x3 {out['bf16x3']['iter_per_s']:.0f} iter/s (X err {out['bf16x3']['fp64_error']['X']:.1e}), "
        f"FP32 {out['f32']['iter_per_s']:.0f} iter/s (X err {out['f32']['fp64_error']['X']:.1e}), "
        f"FP64 {ref['iter_per_s']:.0f} iter/s")
    return out


def cpu_baseline(p, r: int, samples: int):
    """The FP64 oracle as it stands, on the same problem: `samples` iterations
    (dense gradient, top-(r+1) LAPACK eigendecomposition)."""
    import numpy as np

    from oracle import meg_oracle as O

    try:
        from threadpoolctl import threadpool_info

        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    obj = O.MaskedObjective(p.n, p.row_ptr, p.col, p.val.astype(np.float64))
    it = O.initial_iterate(p.V0, p.lam0, O.eps_schedule(0), p.n)
    t0 = time.time()
    done = 0
    for t in range(1, samples + 1):
        X = it.dense()
        G = obj.grad(X)
        it, _ = O.lowrank_step(it, G, 1.0, O.eps_schedule(t), r, full=False)
        done += 1
    dt = time.time() - t0
    return {"value": done / dt, "unit": "iter/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{done} iterations of the FP64 oracle (dense n x n gradient, LAPACK top-(r+1) eigh) "
                      f"at n={p.n}, r={r} from the same warm start; {dt:.1f} s"}


def serving_bench(meg, torch, args) -> dict:
    """Batched serving of the plain configuration's instances (spiked
    denoising, top-1 warm start): n uniform over {256, 512, 1024, 2048}, r
    uniform over 1..8, each run to max(2 eps_t, L_t) <= 1e-4 or 300
    iterations; FP32 state, BF16x3 apply.  Inputs are drawn on the device
    before any timing.  (1) Poisson arrivals at the offered rate: solves/s
    and p50/p99 latency from arrival to the host seeing the result.  (2)
    Saturation, everything arriving at once: solves/s and aggregate
    algorithmic HBM traffic of the planes.  Each scheduling round replays
    one captured hipGraph (graph mode of the server).  (3) The plain FP32 single-instance
    path (meg_init/meg_solve per instance, dense FP32 apply) on a sample, at
    the same stop rule."""
    import numpy as np

    import workloads as W

    reqs = W.serving_stream(args.serve_count, args.seed, rate_hz=args.serve_rate)
    t0 = time.time()
    mats, starts = [], []
    for q in reqs:
        M, v = W.spiked_denoise_device(q["n"], q["seed"])
        mats.append(M)
        starts.append(v)
    torch.cuda.synchronize()
    log(f"[serve] {len(reqs)} instances drawn on the device in {time.time() - t0:.1f}s")
    tol, cap = 1e-4, 300
    lam = np.ones(1)
    srv = meg.MegServer(budget_bytes=8 << 30, launch_steps=args.serve_launch_steps, graph=True)
    teams = {int(n): srv.team(int(n)) for n in sorted({q["n"] for q in reqs})}
    log(f"[serve] team sizes (latency, throughput): {teams}")

    def submit(i):
        q = reqs[i]
        return srv.submit(mats[i], starts[i], lam, q["r"], tol=tol, max_iters=cap, seed=q["seed"])

    # (1) offered load
    lat, iters, sweeps = [], [], []
    outstanding = {}
    i = 0
    t0 = time.perf_counter()
    while i < len(reqs) or outstanding:
        now = time.perf_counter() - t0
        while i < len(reqs) and reqs[i]["t_arrive"] <= now:
            outstanding[submit(i)] = reqs[i]["t_arrive"]
            i += 1
        if not outstanding:
            time.sleep(max(0.0, reqs[i]["t_arrive"] - (time.perf_counter() - t0)))
            continue
        srv.run(1)
        done_t = time.perf_counter() - t0
        for rid in list(outstanding):
            st = srv.query(rid)
            if st["state"] >= 2:
                assert st["state"] == 2, st
                lat.append(done_t - outstanding.pop(rid))
                iters.append(st["iterations"])
                sweeps.append(st["applies"] / max(1, st["iterations"]))
                srv.release(rid)
    wall1 = time.perf_counter() - t0
    lat_ms = np.sort(np.asarray(lat)) * 1e3
    offered = {"rate_hz": args.serve_rate, "requests": len(reqs), "wall_s": wall1,
               "solves_per_s": len(reqs) / wall1, "p50_ms": float(np.percentile(lat_ms, 50)),
               "p99_ms": float(np.percentile(lat_ms, 99)), "max_ms": float(lat_ms[-1]),
               "mean_iterations": float(np.mean(iters)), "sweeps_per_iteration": float(np.mean(sweeps))}
    log(f"[serve] offered {args.serve_rate:.0f}/s: {offered['solves_per_s']:.1f} solves/s, "
        f"p50 {offered['p50_ms']:.1f} ms, p99 {offered['p99_ms']:.1f} ms, mean iterations {offered['mean_iterations']:.1f}, "
        f"{offered['sweeps_per_iteration']:.2f} sweeps per iteration")

    # (2) saturation
    st0 = srv.stats()
    t0 = time.perf_counter()
    ids = [submit(j) for j in range(len(reqs))]
    while srv.run(1) > 0:
        pass
    wall2 = time.perf_counter() - t0
    st1 = srv.stats()
    nbytes = 0.0
    for j, rid in enumerate(ids):
        st = srv.query(rid)
        assert st["state"] == 2, st
        n = reqs[j]["n"]
        nbytes += st["applies"] * (4.0 * n * ((n + 7) // 8 * 8) + 2.0 * n * 16 * 4)
        srv.release(rid)
    gbs = nbytes / wall2 / 1e9
    kms = st1["kernel_ms"] - st0["kernel_ms"]
    saturated = {"wall_s": wall2, "solves_per_s": len(reqs) / wall2, "algorithmic_gbs": gbs,
                 "graph_node": {0: "none", 1: "cooperative", 2: "ordinary"}[st1["graph_node"]],
                 "frac_hbm": gbs / HBM_PEAK_GBS, "kernel_busy_frac": kms * 1e-3 / wall2,
                 "launches": st1["launches"] - st0["launches"], "arena_peak_bytes": st1["arena_peak"]}
    log(f"[serve] saturated: {saturated['solves_per_s']:.1f} solves/s, {gbs:.0f} GB/s of planes "
        f"({100 * gbs / HBM_PEAK_GBS:.1f} % of HBM), kernel busy {100 * saturated['kernel_busy_frac']:.0f} %")
    srv.close()

    # (3) plain FP32 single-instance path on a sample
    sample = min(args.serve_plain_sample, len(reqs))
    t0 = time.perf_counter()
    for j in range(sample):
        q = reqs[j]
        with meg.LowRankMEG(q["n"], q["r"], meg.MEG_GRAD_DENOISE_DENSE, starts[j], lam, prec=meg.MEG_PREC_F32,
                            eta=1.0, dense=mats[j], max_inner=12) as g:
            g.solve(cap, tol)
    torch.cuda.synchronize()
    wall3 = time.perf_counter() - t0
    plain = {"sample": sample, "solves_per_s": sample / wall3,
             "note": "one instance at a time through meg_init/meg_solve, dense FP32 apply, same stop rule"}
    log(f"[serve] plain FP32 one-at-a-time: {plain['solves_per_s']:.1f} solves/s on {sample} instances")
    return {"workload": "spiked denoising instances (plain configuration), n ~ U{256,512,1024,2048}, r ~ U{1..8}",
            "stop": "max(2 eps_t, L_t) <= 1e-4 or 300 iterations", "dtype": "f32 state, bf16x3 apply",
            "launch_steps": args.serve_launch_steps, "teams": {str(k): v for k, v in teams.items()},
            "offered": offered, "saturated": saturated, "plain_f32": plain,
            "speedup_vs_plain": saturated["solves_per_s"] / plain["solves_per_s"]}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=512)
    ap.add_argument("--warmup", type=int, default=64)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--r", type=int, default=10)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--profile-steps", type=int, default=10)
    ap.add_argument("--cpu-samples", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--launch-steps", type=int, default=64,
                    help="iterations per launch of the persistent step kernel (1: one meg_step per iteration)")
    ap.add_argument("--no-serving", action="store_true", help="skip the batched-serving measurement")
    ap.add_argument("--no-recovery", action="store_true", help="skip the recovery-problem measurement")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the plain (n=200 FP64), stochastic (n=8192) and precision-form (n=16384) objects")
    ap.add_argument("--serve-count", type=int, default=2048)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-launch-steps", type=int, default=8)
    ap.add_argument("--serve-plain-sample", type=int, default=32)
    ap.add_argument("--write-workload", default=None, metavar="PATH",
                    help="write the workload file of the native driver and exit (no GPU use)")
    ap.add_argument("--write-dense-workload", default=None, metavar="PATH",
                    help="write the precision-form workload file of the native driver and exit (no GPU use)")
    ap.add_argument("--write-bilinear-workload", default=None, metavar="PATH",
                    help="write the recovery-problem workload file of the native driver and exit (no GPU use)")
    args = ap.parse_args()

    if args.write_bilinear_workload:
        write_bilinear_workload(args.write_bilinear_workload)
        return 0

    if args.write_dense_workload:
        write_dense_workload(args.write_dense_workload, seed=args.seed)
        return 0

    if args.write_workload:
        p = matrix_completion_workload(args.n, args.r, args.seed)
        write_workload(p, args.r, args.write_workload)
        log(f"[bench] workload written to {args.write_workload}")
        return 0

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        return 2

    import numpy as np
    import torch

    from paper_2012_10469_amd import meg

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    p = matrix_completion_workload(args.n, args.r, args.seed)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()  # noqa: E731
    rp, col, val = dev(p.row_ptr.astype(np.int32)), dev(p.col.astype(np.int32)), dev(p.val)
    stream = torch.cuda.Stream()  # default priority; graph replay needs a non-null stream
    torch.cuda.synchronize()
    g = meg.LowRankMEG(p.n, args.r, meg.MEG_GRAD_MASKED_CSR, p.V0, p.lam0, prec=meg.MEG_PREC_F32, eta=1.0,
                       row_ptr=rp, col=col, val=val, max_inner=12, stream=stream.cuda_stream)
    k = g.k

    def run(steps: int) -> None:
        if args.launch_steps <= 1:
            for _ in range(steps):
                g.step(info=False)
        else:
            left = steps
            while left > 0:
                m = min(args.launch_steps, left)
                g.solve(m)
                left -= m

    log(f"[bench] context ready k={k}; warmup {args.warmup}")
    run(args.warmup)
    torch.cuda.synchronize()
    g.counters(reset=True)
    log(f"[bench] timing {args.steps} steps ({args.launch_steps} per launch)")
    t0 = time.perf_counter()
    run(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    secs = t1 - t0
    cnt = g.counters()
    cert = g.certificate()
    log(f"[bench] {args.steps} steps in {secs:.3f}s; last step inner sweeps {cert['inner_iters']} "
        f"cert_L {cert['cert_L']:.4f} eps {cert['eps_t']:.3e}; {cnt['extrapolated']} of {cnt['iterations']} "
        f"steps ended extrapolated")
    assert cnt["iterations"] == args.steps, cnt
    launches = cnt["launches"]
    avg_launch_ms = cnt["kernel_ms"] / launches
    iters_per_launch = cnt["iterations"] / launches
    sweeps = cnt["applies"] / cnt["iterations"]
    nbytes = step_bytes(p.n, p.nnz, k, 4, sweeps) * iters_per_launch
    achieved = nbytes / (avg_launch_ms * 1e-3) / 1e9
    log(f"[bench] step kernel: {launches} launches, {avg_launch_ms * 1e3:.1f} us each ({iters_per_launch:.1f} "
        f"iterations, {sweeps:.2f} applies per iteration) -> {achieved:.0f} GB/s algorithmic")

    # one-step launches with HIP events around the step kernel, on its stream,
    # plus the kernel's own phase stamps
    kms, prep, fin, act, app, small, wgs = [], [], [], [], [], [], []
    for _ in range(args.profile_steps):
        pr = g.profile_step()
        wgs.append(pr)
        kms.append(pr["kernel_ms"])
        prep.append(pr["prep_ms"])
        fin.append(pr["finalize_ms"])
        act.append(pr["sweeps_active"])
        app += pr["apply_ms"]
        small += pr["small_ms"]
    phases = None
    if kms:
        apply_gbs = (apply_bytes(p.n, p.nnz, k, 4, True) + apply_bytes(p.n, p.nnz, k, 4, False)) / 2 \
            / (float(np.mean(app)) * 1e-3) / 1e9
        phases = {"one_iteration_launch_us": float(np.mean(kms)) * 1e3, "grad_us": float(np.mean(prep)) * 1e3,
                  "apply_us": float(np.mean(app)) * 1e3, "apply_gbs": apply_gbs,
                  "reduce_rr_us": float(np.mean(small)) * 1e3, "finalize_us": float(np.mean(fin)) * 1e3,
                  "sweeps": float(np.mean(act))}
        for sw in range(2):
            rows = [w for w in wgs if len(w["wg_apply_ms"]) > sw]
            if rows:
                mn, av, mx = (float(np.mean([w["wg_apply_ms"][sw][q] for w in rows])) * 1e3 for q in range(3))
                sk = float(np.mean([w["wg_skew_ms"][sw] for w in rows])) * 1e3
                rd = float(np.mean([w["reduce_ms"][sw] for w in rows])) * 1e3
                phases[f"sweep{sw + 1}_wg_us"] = {"min": mn, "mean": av, "max": mx, "start_skew": sk, "reduce": rd}
                log(f"[bench]   sweep {sw + 1}: workgroup apply {mn:.1f}/{av:.1f}/{mx:.1f} us (min/mean/max), "
                    f"start skew {sk:.1f} us, tree reduction {rd:.1f} us")
        rr = np.mean([w["rr_ms"] for w in wgs], axis=0) * 1e3
        js = float(np.mean([w["jacobi_sweeps"] for w in wgs]))
        phases["rayleigh_ritz_us"] = {"pre": rr[0], "jacobi": rr[1], "test": rr[2], "tail": rr[3], "jacobi_sweeps": js}
        log(f"[bench]   first Rayleigh-Ritz: pre {rr[0]:.1f} us, Jacobi {rr[1]:.1f} us ({js:.1f} sweeps), "
            f"sort+residuals {rr[2]:.1f} us, tail {rr[3]:.1f} us")
        log(f"[bench] one-iteration launch {phases['one_iteration_launch_us']:.1f} us (grid {pr['workgroups']} WGs): "
            f"grad {phases['grad_us']:.1f} us, apply {phases['apply_us']:.1f} us x {phases['sweeps']:.2f} "
            f"({apply_gbs:.0f} GB/s), reduce+RR {phases['reduce_rr_us']:.1f} us, finalize {phases['finalize_us']:.1f} us")

    # dual gap of the final iterate (Section 7's near-optimality measure), not timed with the steps
    t0 = time.perf_counter()
    dg = g.dual_gap(max_steps=256, tol=1e-8)
    dg["ms"] = (time.perf_counter() - t0) * 1e3
    log(f"[bench] dual gap at t={dg['t']}: {dg['gap']:.4e} (<X,G> {dg['x_dot_g']:.4e}, lambda_min {dg['lambda_min']:.4e}, "
        f"{dg['steps']} Lanczos steps, {dg['ms']:.1f} ms)")

    # the all-eigenvalue certificate of the next step (Section 3.1.1): b_n = tr exp(M_t) from the
    # solver block plus 48 Gaussian probes (one 64-vector Lanczos batch), then that step's L_full
    # next to its cheap b^{r+1} certificate; not timed with the steps
    U = torch.from_numpy(np.random.default_rng([17, p.n]).standard_normal((p.n, 48))).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tri, tr = g.trace_exp(U, max_steps=64, tol=1e-8)
    tri["ms"] = (time.perf_counter() - t0) * 1e3
    st = g.step()
    L_full, holds = g.certificate_full(tr)
    tri.update({"probes": 48, "cert_L_full": L_full, "cert_holds_full": holds, "cert_L": st["cert_L"],
                "eps_t": st["eps_t"]})
    log(f"[bench] trace of exp(M_t) at t={tri['t']}: log b_n {tri['log_b']:.6f} (block {tri['log_b_defl']:.6f}, "
        f"probes {tri['log_b_tail']:.4f}, rel. std. error {tri['tail_rel_stderr']:.2e}), {tri['steps']} Lanczos "
        f"steps, {tri['ms']:.1f} ms; certificate L_full {L_full:.4f} vs L {st['cert_L']:.4f} (2 eps {2 * st['eps_t']:.2e})")

    base = None
    if not args.no_cpu_baseline:
        log(f"[bench] CPU oracle baseline: {args.cpu_samples} iterations")
        base = cpu_baseline(p, args.r, args.cpu_samples)
    g.close()
    serving = None if args.no_serving else serving_bench(meg, torch, args)
    recovery = None if args.no_recovery else recovery_bench(meg, torch)
    config1 = None if args.no_configs else config1_bench(meg, torch)
    config3 = None if args.no_configs else config3_bench(meg, torch)
    precision = None if args.no_configs else precision_bench(meg, torch)
    # measured HBM bytes per launch (counter runs), only for the kernel they were taken on
    traffic, traffic_note = None, "kernel sources changed since the counter runs"
    if kernel_source_hash() == TRAFFIC["source_hash"]:
        traffic_note = "counters were taken on another launch configuration"
        if (launches == 1 and cnt["iterations"] == TRAFFIC["iterations_per_launch"]
                and args.warmup == TRAFFIC["warmup"]):
            traffic = TRAFFIC["bytes_per_launch"]
            traffic_note = (f"HBM bytes of this launch configuration ({TRAFFIC['iterations_per_launch']} iterations "
                            f"in one launch after {TRAFFIC['warmup']}; FETCH_SIZE x {TRAFFIC['fetch_factor']} + "
                            f"WRITE_SIZE x {TRAFFIC['write_factor']}, {TRAFFIC['applies_per_iteration']} applies "
                            f"per iteration when measured)")

    out = {
        "metric": "low-rank MEG iterations/s (matrix completion, n=4096, r=10, FP32)",
        "value": args.steps / secs,
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": secs * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "matrix_completion_csr", "n": p.n, "r": args.r, "k": k, "nnz": p.nnz,
                   "mask_p": 0.1, "truth_rank": 5, "eta": 1.0, "eps": "0.8/(t+11)^2",
                   "sweeps_per_step": sweeps, "extrapolated_per_step": cnt["extrapolated"] / cnt["iterations"],
                   "steps_per_launch": args.launch_steps},
        "roofline": {"bound": "hbm", "kernel": "k_step", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_note": traffic_note,
                     "bytes_per_launch": nbytes, "avg_launch_us": avg_launch_ms * 1e3,
                     "iterations_per_launch": iters_per_launch, "applies_per_iteration": sweeps,
                     "jacobi_sweeps_per_iteration": cnt["jacobi_sweeps"] / cnt["iterations"],
                     "launches": launches, "phases": phases},
        "dual_gap": dg,
        "trace_exp": tri,
        "cpu_baseline": base,
        "serving": serving,
        "recovery": recovery,
        "config1": config1,
        "config3": config3,
        "precision": precision,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
