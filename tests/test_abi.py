"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/meg.h, the ctypes structures match the C layout (checked
against a gcc-compiled probe), and argument validation rejects bad inputs
before any device call."""
import ctypes
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "meg.h")


@pytest.fixture(scope="module")
def M():
    from paper_2012_10469_amd import meg

    if not os.path.exists(meg.LIB_PATH):
        from paper_2012_10469_amd import build

        build.build()
    meg.load_library()
    return meg


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:meg_status|int32_t|void|const char\*)\s+(meg_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_every_declared_symbol_is_exported(M):
    names = declared_functions()
    assert len(names) >= 12
    lib = ctypes.CDLL(M.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(M.EXPORTED) == names


def test_struct_layout_matches_header(M):
    probe = r"""
#include <stdio.h>
#include <stddef.h>
#include "meg.h"
#define P(T) printf(#T " %zu\n", sizeof(T));
#define O(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
int main(void) {
  P(meg_params) P(meg_objective) P(meg_start) P(meg_step_info) P(meg_kernel_times) P(meg_counters) P(meg_dual_gap_info)
  P(meg_trace_info) O(meg_trace_info, tail_rel_stderr) O(meg_trace_info, t) O(meg_trace_info, kd)
  O(meg_trace_info, converged) O(meg_trace_info, batches)
  O(meg_kernel_times, apply_ms) O(meg_kernel_times, finalize_ms) O(meg_kernel_times, workgroups)
  O(meg_kernel_times, wg_apply_ms) O(meg_kernel_times, wg_skew_ms) O(meg_kernel_times, reduce_ms)
  O(meg_kernel_times, rr_ms) O(meg_kernel_times, rr_tail_ms) O(meg_kernel_times, jacobi_sweeps)
  O(meg_counters, applies) O(meg_counters, workgroups) O(meg_counters, jacobi_sweeps) O(meg_counters, kernel_ms)
  O(meg_counters, extrapolated) O(meg_counters, unconverged)
  O(meg_dual_gap_info, lambda_min) O(meg_dual_gap_info, t) O(meg_dual_gap_info, steps) O(meg_dual_gap_info, converged)
  O(meg_params, eta) O(meg_params, seed) O(meg_params, flags) O(meg_params, inner_tol)
  O(meg_objective, dense) O(meg_objective, ld) O(meg_objective, nnz) O(meg_objective, batch_idx)
  O(meg_objective, batch_steps) O(meg_start, V0) O(meg_start, lambda0)
  O(meg_step_info, cert_holds) O(meg_step_info, ritz_gap) O(meg_step_info, converged) O(meg_step_info, resid_r1)
  O(meg_step_info, cert_resolved) O(meg_step_info, cert_L_up) O(meg_step_info, mu_r1_up)
  P(meg_cert_bound_info) O(meg_cert_bound_info, resid) O(meg_cert_bound_info, t) O(meg_cert_bound_info, converged)
  P(meg_server_params) P(meg_request) P(meg_request_status) P(meg_server_stats)
  O(meg_server_params, max_resident) O(meg_server_params, flags) O(meg_server_params, fixed_team)
  O(meg_request, n) O(meg_request, M) O(meg_request, q) O(meg_request, V0) O(meg_request, eta)
  O(meg_request, tol) O(meg_request, max_inner) O(meg_request, seed)
  O(meg_request_status, iterations) O(meg_request_status, done_ms) O(meg_request_status, team)
  O(meg_request_status, last) O(meg_request_status, applies)
  O(meg_server_stats, kernel_ms) O(meg_server_stats, capacity_wg) O(meg_server_stats, graph_node)
  O(meg_server_stats, arena_peak)
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "p.c")
        exe = os.path.join(d, "p")
        open(c, "w").write(probe)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    want = {}
    for line in out.strip().splitlines():
        k, v = line.split()
        want[k] = int(v)
    S = {"meg_params": M.MegParams, "meg_objective": M.MegObjective, "meg_start": M.MegStart,
         "meg_step_info": M.MegStepInfo, "meg_kernel_times": M.MegKernelTimes, "meg_counters": M.MegCounters, "meg_dual_gap_info": M.MegDualGapInfo,
         "meg_trace_info": M.MegTraceInfo, "meg_cert_bound_info": M.MegCertBoundInfo,
         "meg_server_params": M.MegServerParams, "meg_request": M.MegRequest,
         "meg_request_status": M.MegRequestStatus, "meg_server_stats": M.MegServerStats}
    for k, v in want.items():
        if "." in k:
            s, f = k.split(".")
            assert getattr(S[s], f).offset == v, k
        else:
            assert ctypes.sizeof(S[k]) == v, k


def test_block_size_and_status_strings(M):
    assert M.meg_block_size(10, 4) == 16
    assert M.meg_block_size(5, 4) == 16
    assert M.meg_block_size(16, 4) == 32
    assert M.meg_block_size(27, 4) == 32
    assert M.meg_block_size(28, 4) == 0
    assert M.meg_block_size(0, 4) == 0
    assert M.meg_block_size(3, -1) == 0
    for s in range(8):
        assert isinstance(M.meg_status_str(s), str) and M.meg_status_str(s)


def _start(n, q=1):
    V = np.zeros((n, q))
    V[np.arange(q), np.arange(q)] = 1.0
    return V, np.full(q, 1.0 / q)


def _dense_obj(M, kind=0):
    # fake (never dereferenced) device address: validation fails first
    return M.MegObjective(kind=kind, dense=0x1000, ld=64)


@pytest.mark.parametrize("field,value", [
    ("n", 1), ("r", 0), ("r", 64), ("oversample", -1), ("r", 28), ("prec", 7), ("eta", 0.0),
    ("eta", float("nan")), ("eps_scale", 0.0), ("eps_scale", 100.0), ("min_inner", 0), ("max_inner", 0),
    ("max_inner", 65), ("inner_tol", -1.0),
])
def test_init_rejects_bad_params(M, field, value):
    n = 64
    p = M.make_params(n, 4)
    setattr(p, field, value)
    V, lam = _start(n)
    st, ctx = M.meg_init(p, _dense_obj(M), V, lam)
    assert st == M.MEG_ERR_INVALID_ARG
    assert not ctx.value


def test_init_rejects_bad_start_and_objective(M):
    n = 64
    p = M.make_params(n, 4)
    V, lam = _start(n, 2)
    assert M.meg_init(p, _dense_obj(M), V, np.array([0.7, 0.7]))[0] == M.MEG_ERR_INVALID_ARG  # sum != 1
    assert M.meg_init(p, _dense_obj(M), V, np.array([1.2, -0.2]))[0] == M.MEG_ERR_INVALID_ARG  # negative
    Vbad = V.copy(); Vbad[0, 1] = 0.5
    assert M.meg_init(p, _dense_obj(M), Vbad, lam)[0] == M.MEG_ERR_INVALID_ARG  # not orthonormal
    V5, lam5 = _start(n, 5)
    assert M.meg_init(p, _dense_obj(M), V5, lam5)[0] == M.MEG_ERR_INVALID_ARG  # q > r
    assert M.meg_init(p, M.MegObjective(kind=0, dense=None, ld=64), V, lam)[0] == M.MEG_ERR_INVALID_ARG
    assert M.meg_init(p, M.MegObjective(kind=0, dense=0x1000, ld=10), V, lam)[0] == M.MEG_ERR_INVALID_ARG
    assert M.meg_init(p, M.MegObjective(kind=9, dense=0x1000, ld=64), V, lam)[0] == M.MEG_ERR_INVALID_ARG
    assert M.meg_init(p, M.MegObjective(kind=3, row_ptr=None), V, lam)[0] == M.MEG_ERR_INVALID_ARG
    assert M.meg_init(p, M.MegObjective(kind=3, row_ptr=0x1000, nnz=5, col=None, val=0x1000), V, lam)[0] \
        == M.MEG_ERR_INVALID_ARG
    # k = 16 > n
    p2 = M.make_params(12, 4)
    assert M.meg_init(p2, M.MegObjective(kind=0, dense=0x1000, ld=12), _start(12)[0], _start(12)[1])[0] \
        == M.MEG_ERR_INVALID_ARG


def test_init_rejects_bad_bf16_planes(M):
    """The matrix-core form takes two 16-byte-aligned bf16 planes with a row
    length that is a multiple of 8; CSR data has no such form."""
    n = 64
    p = M.make_params(n, 4, prec=M.MEG_PREC_F32_BF16X3)
    V, lam = _start(n)
    dense = lambda **kw: M.MegObjective(kind=M.MEG_GRAD_DENOISE_DENSE, **kw)  # noqa: E731
    assert M.meg_init(p, dense(dense=0x1000, dense_lo=None, ld=64), V, lam)[0] == M.MEG_ERR_INVALID_ARG
    assert M.meg_init(p, dense(dense=0x1000, dense_lo=0x2000, ld=68), V, lam)[0] == M.MEG_ERR_INVALID_ARG
    assert M.meg_init(p, dense(dense=0x1008, dense_lo=0x2000, ld=64), V, lam)[0] == M.MEG_ERR_INVALID_ARG
    assert M.meg_init(p, dense(dense=0x1000, dense_lo=0x2004, ld=64), V, lam)[0] == M.MEG_ERR_INVALID_ARG
    csr = M.MegObjective(kind=M.MEG_GRAD_MASKED_CSR, row_ptr=0x1000, col=0x2000, val=0x3000, nnz=10)
    assert M.meg_init(p, csr, V, lam)[0] == M.MEG_ERR_UNSUPPORTED


def test_init_rejects_bad_quadmeas(M):
    """Quadratic measurements: pool rows of at least n elements on 16-byte
    boundaries, 1 <= L <= 1024, at least one minibatch; no bf16-plane form."""
    n = 64
    p = M.make_params(n, 4)
    V, lam = _start(n)

    def q(**kw):
        base = dict(kind=M.MEG_GRAD_QUADMEAS, A=0x1000, lda=64, b=0x2000, m=100, batch=32, batch_idx=0x3000,
                    batch_steps=4)
        base.update(kw)
        return M.MegObjective(**base)

    for bad in (dict(A=None), dict(b=None), dict(batch_idx=None), dict(m=0), dict(lda=60), dict(lda=66),
                dict(A=0x1004), dict(batch=0), dict(batch=1025), dict(batch_steps=0)):
        assert M.meg_init(p, q(**bad), V, lam)[0] == M.MEG_ERR_INVALID_ARG, bad
    p3 = M.make_params(n, 4, prec=M.MEG_PREC_F32_BF16X3)
    assert M.meg_init(p3, q(), V, lam)[0] == M.MEG_ERR_UNSUPPORTED
    assert M.meg_init(p3, M.MegObjective(kind=M.MEG_GRAD_EXTERNAL), V, lam)[0] == M.MEG_ERR_UNSUPPORTED
    p64 = M.make_params(n, 4, prec=M.MEG_PREC_F64)
    assert M.meg_init(p64, q(lda=65), V, lam)[0] == M.MEG_ERR_INVALID_ARG  # 65 doubles: rows not 16-byte aligned


def test_init_validates_bilinear(M):
    """Bilinear measurements: A (2m rows), y and m >= 1, lda >= n; not in the
    bf16-plane form.  Validation runs before any device call."""
    n = 64
    p = M.make_params(n, 4)
    V, lam = _start(n)

    def q(**kw):
        base = dict(kind=M.MEG_GRAD_BILINEAR, A=0x1000, lda=64, b=0x2000, m=100)
        base.update(kw)
        return M.MegObjective(**base)

    for bad in (dict(A=None), dict(b=None), dict(m=0), dict(lda=60)):
        assert M.meg_init(p, q(**bad), V, lam)[0] == M.MEG_ERR_INVALID_ARG, bad
    p3 = M.make_params(n, 4, prec=M.MEG_PREC_F32_BF16X3)
    assert M.meg_init(p3, q(), V, lam)[0] == M.MEG_ERR_UNSUPPORTED


def test_server_null_handle_and_bad_params(M):
    """Server entry points reject a null handle and invalid parameters before
    touching the device."""
    lib = M.load_library()
    st = M.MegRequestStatus()
    assert lib.meg_server_query(None, 1, ctypes.byref(st)) == M.MEG_ERR_INVALID_ARG
    assert lib.meg_server_run(None, 1, None) == M.MEG_ERR_INVALID_ARG
    assert lib.meg_server_release(None, 1) == M.MEG_ERR_INVALID_ARG
    stats = M.MegServerStats()
    assert lib.meg_server_get_stats(None, ctypes.byref(stats)) == M.MEG_ERR_INVALID_ARG
    h = ctypes.c_void_p()
    for kw in (dict(launch_steps=0, max_resident=8), dict(launch_steps=8, max_resident=0),
               dict(launch_steps=8, max_resident=257), dict(launch_steps=2000, max_resident=8),
               dict(launch_steps=8, max_resident=8, budget_bytes=-1), dict(launch_steps=8, max_resident=8, flags=2),
               dict(launch_steps=8, max_resident=8, fixed_team=-1)):
        p = M.MegServerParams(**kw)
        assert lib.meg_server_create(ctypes.byref(h), ctypes.byref(p), None) == M.MEG_ERR_INVALID_ARG, kw
        assert not h.value
    lib.meg_server_destroy(None)  # no-op


def test_null_context_calls(M):
    lib = M.load_library()
    info = M.MegStepInfo()
    assert lib.meg_step(None, ctypes.byref(info)) == M.MEG_ERR_INVALID_ARG
    assert lib.meg_solve(None, 1, 0.0, None) == M.MEG_ERR_INVALID_ARG
    assert lib.meg_certificate(None, ctypes.byref(info)) == M.MEG_ERR_INVALID_ARG
    cnt = M.MegCounters()
    assert lib.meg_get_counters(None, ctypes.byref(cnt), 0) == M.MEG_ERR_INVALID_ARG
    g = M.MegObjective(kind=M.MEG_GRAD_LINEAR_DENSE, dense=0x1000, ld=64)
    assert lib.meg_step_external(None, ctypes.byref(g), None) == M.MEG_ERR_INVALID_ARG
    dg = M.MegDualGapInfo()
    assert lib.meg_dual_gap(None, 64, 1e-10, ctypes.byref(dg)) == M.MEG_ERR_INVALID_ARG
    assert lib.meg_solve_to_gap(None, 10, 1e-3, 4, None, ctypes.byref(dg)) == M.MEG_ERR_INVALID_ARG
    tr = M.MegTraceInfo()
    assert lib.meg_trace_exp(None, None, 0, 1.0, 32, 1e-10, ctypes.byref(tr)) == M.MEG_ERR_INVALID_ARG
    L, h = ctypes.c_double(), ctypes.c_int32()
    assert lib.meg_certificate_full(None, ctypes.byref(tr), ctypes.byref(L), ctypes.byref(h)) == M.MEG_ERR_INVALID_ARG
    lib.meg_destroy(None)  # no-op
