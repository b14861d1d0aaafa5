"""FP16 stored rows on the 2D Galerkin levels (coarse_bits = 16 with the
complex64 cycle; section 3 keeps coarse data in half precision).  Each level's
rows are divided by one power of two, rounded to FP16 and summed in FP32, so a
residual row differs from the exact one by at most the FP16 unit roundoff
2^-11 times sum |a_ij| |x_j| (plus FP32 rounding); the cycle moves by about
that much relative to the oracle's; solves reach their tolerance in about the
same iterations.  The 256^2 level with more than 8 sources is served by the
LDS-staged kernel, which reads the FP32 compact stencil: its half-sweeps are
the same to the bit with FP16 or FP32 rows."""
import numpy as np
import pytest

from _helpers import (say, workload, small_hetero, oracle_problem, oracle_hierarchy, rand_cvec, to_dev,
                      from_dev, rhs_matrix)

pytestmark = pytest.mark.gpu

U16 = 2.0 ** -11
U32 = 2.0 ** -24


def _solver(w, **over):
    from paper_1806_11277_amd import ehh
    return ehh.solver_for_workload(w, **over)


def test_fp16_rows_2d_level_residual_within_the_rounding_bound():
    import torch
    w = small_hetero((96, 64), "h16", levels=4, damping=(0.75, 0.5, 0.5), precond_bits=32)
    H = oracle_hierarchy(w)
    S16, S32 = _solver(w, coarse_bits=16), _solver(w, coarse_bits=32)
    for l in (1, 2):   # the levels with stored rows (the coarsest is solved exactly)
        A = H.A[l]
        N = A.shape[0]
        x = rand_cvec(N, 3, 70 + l)
        xd = to_dev(x, torch.float32)
        x32 = from_dev(xd)     # the FP32 input both sides use
        out = {}
        for cb, S in ((16, S16), (32, S32)):
            y = torch.zeros_like(xd)
            S.level_apply(0, l, xd, y)
            torch.cuda.synchronize()
            out[cb] = from_dev(y)
        absA = abs(A)
        for r in range(3):
            ref = A @ x32[r]
            mag = absA @ np.abs(x32[r])
            d16 = np.abs(out[16][r] - ref)
            d32 = np.abs(out[32][r] - ref)
            say(f"[fp16 rows 2d level {l} source {r}] max err / (|A||x|): fp16 {np.max(d16 / mag):.2e}, "
                f"fp32 {np.max(d32 / mag):.2e}")
            # (coefficients far below a level's largest fall into FP16's subnormal
            # range, where the rounding is absolute: the last term)
            assert np.all(d32 <= 64 * U32 * mag + 1e-12 * mag.max())
            assert np.all(d16 <= (U16 + 64 * U32) * mag + 1e-9 * mag.max())
            assert np.max(d16 / mag) > 8 * U32      # the FP16 rows are the ones used
    S16.close()
    S32.close()


def test_fp16_rows_2d_cycle_and_solve():
    import torch
    w = workload("c3s_hetero128_batch8_fp32")
    say("[fp16 rows 2d: cycle and solve, c3s]")
    pb = oracle_problem(w)
    H = oracle_hierarchy(w, pb)
    A = pb.matrix()
    B = rhs_matrix(w)
    v = rand_cvec(pb.size, 2, 62)
    out, iters = {}, {}
    for cb in (32, 16):
        S = _solver(w, coarse_bits=cb)
        z = torch.zeros_like(to_dev(v))
        S.precondition(to_dev(v), z)
        torch.cuda.synchronize()
        out[cb] = from_dev(z)
        x = torch.zeros_like(to_dev(B))
        st, stats = S.solve(to_dev(B), x, tol=1e-8, maxit=600)
        torch.cuda.synchronize()
        assert st == 0, stats
        got = from_dev(x)
        for r in range(B.shape[0]):
            assert np.linalg.norm(B[r] - A @ got[r]) / np.linalg.norm(B[r]) <= 1.01e-8
        iters[cb] = max(s_["iters"] for s_ in stats)
        S.close()
    for r in range(2):
        ref = H.cycle(v[r])
        e16 = np.linalg.norm(out[16][r] - ref) / np.linalg.norm(ref)
        e32 = np.linalg.norm(out[32][r] - ref) / np.linalg.norm(ref)
        say(f"  source {r}: cycle error vs oracle fp32 rows {e32:.2e}, fp16 rows {e16:.2e}")
        assert e32 <= 2e-5
        assert 0 < e16 <= 2 * U16
    say(f"  iterations fp32 rows {iters[32]}, fp16 rows {iters[16]}")
    assert iters[16] <= int(1.1 * iters[32]) + 1


def test_fp16_rows_2d_lds_level_reads_the_fp32_stencil():
    import torch
    w = workload("c3_hetero512_batch32_fp32")
    S16, S32 = _solver(w, coarse_bits=16), _solver(w, coarse_bits=32)
    info = S16.level_info(0, 1)
    assert info["n"][:2] == [256, 256]
    N = info["N"]
    for nrhs, same in ((12, True), (4, False)):
        b = to_dev(rand_cvec(N, nrhs, 90), torch.float32)
        e = to_dev(rand_cvec(N, nrhs, 91), torch.float32)
        out = {}
        for cb, S in ((16, S16), (32, S32)):
            o = torch.zeros_like(b)
            S.level_relax(0, 1, 0, b, e, o)
            torch.cuda.synchronize()
            out[cb] = o.cpu()
        d = float((out[16] - out[32]).abs().max())
        say(f"[fp16 rows 2d, 256^2 level, {nrhs} sources] max |fp16 rows - fp32 rows| {d:.2e}")
        assert (d == 0.0) == same
        if not same:
            assert d <= 1e-2 * float(out[32].abs().max())
    S16.close()
    S32.close()
