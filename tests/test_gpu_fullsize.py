"""Parity at the benchmark sizes, in the configuration bench.py times.

c2 and c3 (512^2): one whole preconditioner cycle is compared with the oracle's
cycle (every one of c3's 32 sources, norm-wise and per component), and solves at
tol 1e-10 are compared with the oracle's direct solution (every source).
c4 (128^3, 8 padded 72^3 subdomains): the cycle of one subdomain on all 16
sources is compared with the oracle's cycle of that subdomain; a direct
factorisation of the whole 128^3 operator is out of reach on the host, so the
full solve is checked through its residual recomputed by the oracle's sparse
operator.  (The c4 solver configuration is compared whole with the oracle's DD
preconditioner at 32^3 and with its direct solution at 16^3.)"""
import numpy as np
import pytest

from _helpers import (say, workload, oracle_problem, oracle_hierarchy, rand_cvec, to_dev, from_dev, rhs_matrix,
                      component_errors)

pytestmark = pytest.mark.gpu


def _solver(w, **over):
    import torch
    from paper_1806_11277_amd import ehh
    torch.cuda.synchronize()
    return ehh.solver_for_workload(w, **over)


@pytest.fixture(scope="module")
def c2_oracle():
    w = workload("c2_hetero512_fp64")
    say("[c2 full size: oracle problem and hierarchy]")
    pb = oracle_problem(w)
    H = oracle_hierarchy(w, pb)
    return w, pb, H


def test_c2_cycle_matches_oracle(c2_oracle):
    import torch
    w, pb, H = c2_oracle
    say("[c2 full-size W-cycle, FP64]")
    S = _solver(w)
    r = rand_cvec(pb.size, 1, 70)
    e = torch.zeros_like(to_dev(r))
    S.vcycle(to_dev(r), e)
    torch.cuda.synchronize()
    got = from_dev(e)[0]
    ref = H.cycle(r[0])
    assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)
    ec = component_errors(w.n, got, ref)
    say(f"  per-component error {['%.1e' % v for v in ec]}")
    assert max(ec) <= 1e-9
    S.close()


def test_c3_cycle_matches_oracle(c2_oracle):
    """The complex64 cycle of c3 (same medium and hierarchy as c2) on 32
    right-hand sides, every one compared with the FP64 oracle cycle, norm-wise
    and per component."""
    import torch
    w2, pb, H = c2_oracle
    w = workload("c3_hetero512_batch32_fp32")
    say("[c3 full-size W-cycle, complex64, 32 right-hand sides]")
    S = _solver(w)
    r = rand_cvec(pb.size, 32, 71)
    e = torch.zeros((32, 2 * pb.size), dtype=torch.float32, device="cuda")
    S.vcycle(to_dev(r, torch.float32), e)
    torch.cuda.synchronize()
    got = from_dev(e)
    worst = [0.0, 0.0]
    for q in range(32):
        ref = H.cycle(r[q])
        e2 = np.linalg.norm(got[q] - ref) / np.linalg.norm(ref)
        ec = max(component_errors(w.n, got[q], ref))
        worst = [max(worst[0], e2), max(worst[1], ec)]
        assert e2 <= 2e-5 and ec <= 2e-4, (q, e2, ec)
    say(f"  worst norm-wise {worst[0]:.2e}, worst per component {worst[1]:.2e}")
    S.close()


@pytest.fixture(scope="module")
def c2_direct(c2_oracle):
    """The oracle's direct solver of the 512^2 operator (c2 and c3 share it)."""
    from oracle import direct
    w, pb, H = c2_oracle
    say("[512^2 operator: oracle direct factorisation]")
    return direct.factorize(pb)


@pytest.mark.timeout(900)
def test_c2_solve_matches_direct_solution(c2_oracle, c2_direct):
    """c2 (FP64 cycle, one source) solved to 1e-10: within 1e-6 of the oracle's
    direct solution."""
    import torch
    w, pb, H = c2_oracle
    say("[c2 full-size solve at 1e-10 vs direct]")
    B = rhs_matrix(w)
    S = _solver(w)
    x = torch.zeros_like(to_dev(B))
    st, stats = S.solve(to_dev(B), x, tol=1e-10, maxit=1500)
    torch.cuda.synchronize()
    S.close()
    assert st == 0, stats
    xd = c2_direct.solve(B[0])
    err = np.linalg.norm(from_dev(x)[0] - xd) / np.linalg.norm(xd)
    say(f"  iters {stats[0]['iters']} residual {stats[0]['rel_res_true']:.2e} error vs direct {err:.2e}")
    assert stats[0]["rel_res_true"] <= 1e-10 and err <= 1e-6


@pytest.mark.timeout(900)
def test_c3_solve_matches_direct_solution(c2_oracle, c2_direct):
    """c3 (complex64 cycle in FP64 FGMRES, 32 sources) solved to 1e-10: every
    source within 1e-6 of the oracle's direct solution."""
    import torch
    w = workload("c3_hetero512_batch32_fp32")
    say("[c3 full-size solve at 1e-10 vs direct, 32 sources]")
    B = rhs_matrix(w)
    S = _solver(w)
    x = torch.zeros_like(to_dev(B))
    st, stats = S.solve(to_dev(B), x, tol=1e-10, maxit=1500)
    torch.cuda.synchronize()
    S.close()
    assert st == 0, [s_["rel_res_true"] for s_ in stats]
    got = from_dev(x)
    worst = 0.0
    for r in range(32):
        xd = c2_direct.solve(B[r])
        err = np.linalg.norm(got[r] - xd) / np.linalg.norm(xd)
        worst = max(worst, err)
        assert stats[r]["rel_res_true"] <= 1e-10 and err <= 1e-6, (r, err)
    say(f"  iterations {min(s_['iters'] for s_ in stats)}-{max(s_['iters'] for s_ in stats)}, "
        f"worst error vs direct {worst:.2e}")


@pytest.mark.timeout(900)
def test_c4_subdomain_cycle_matches_oracle():
    """c4 at full size: the V(2,1) cycle of one padded 72^3 subdomain (4 levels, 36^3
    and 18^3 Galerkin levels, 9^3 coarsest) on all 16 sources at once, the launch
    shapes the bench runs, compared source by source with the oracle's cycle of
    the same subdomain operator."""
    import torch
    from oracle import dd as ddm, multigrid as mg
    w = workload("c4_layered128_dd8_batch16_fp32")
    say("[c4 full size: oracle hierarchy of subdomain 0]")
    pb = oracle_problem(w)
    subs = ddm.make_subdomains(w.n, w.dd_parts[:3], w.dd_overlap, w.dd_pad)
    sub = subs[0]
    assert sub.nloc == (72, 72, 72)
    H = mg.Hierarchy(ddm.local_operator(pb, sub, w.abl_max), sub.nloc, w.levels, list(w.damping),
                     economic=(w.vanka == 0), cycle=w.cycle, nu1=w.nu1, nu2=w.nu2)
    say("[c4 subdomain 0 cycle, 16 sources]")
    S = _solver(w)
    assert S.subdomain_info(0)["n"] == [72, 72, 72]
    N = H.A[0].shape[0]
    assert S.level_info(0, 0)["N"] == N
    r = rand_cvec(N, 16, 72)
    e = torch.zeros((16, 2 * N), dtype=torch.float32, device="cuda")
    S.vcycle(to_dev(r, torch.float32), e, sub=0)
    torch.cuda.synchronize()
    S.close()
    got = from_dev(e)
    worst = [0.0, 0.0]
    for q in range(16):
        ref = H.cycle(r[q])
        e2 = np.linalg.norm(got[q] - ref) / np.linalg.norm(ref)
        ec = max(component_errors(sub.nloc, got[q], ref))
        worst = [max(worst[0], e2), max(worst[1], ec)]
        assert e2 <= 2e-5 and ec <= 2e-4, (q, e2, ec)
    say(f"  worst norm-wise {worst[0]:.2e}, worst per component {worst[1]:.2e}")


def test_c2_solve_true_residual(c2_oracle):
    import torch
    w, pb, H = c2_oracle
    say("[c2 full-size solve, residual recomputed by the oracle]")
    A = pb.matrix()
    B = rhs_matrix(w)
    S = _solver(w)
    x = torch.zeros_like(to_dev(B))
    st, stats = S.solve(to_dev(B), x, tol=1e-6, maxit=400)
    torch.cuda.synchronize()
    assert st == 0
    got = from_dev(x)[0]
    res = np.linalg.norm(B[0] - A @ got) / np.linalg.norm(B[0])
    say(f"  iters {stats[0]['iters']} library residual {stats[0]['rel_res_true']:.3e} oracle residual {res:.3e}")
    assert res <= 1e-6
    assert abs(res - stats[0]["rel_res_true"]) <= 1e-9
    S.close()


def test_c4_solve_true_residual():
    """128^3, 2 x 2 x 2 padded subdomains, complex64 DD-MG preconditioner with the
    multicolour schedule; two of the 16 sources, residual recomputed by the
    oracle's sparse operator."""
    import dataclasses
    import torch
    w = workload("c4_layered128_dd8_batch16_fp32")
    srcs = w.sources()[:2]
    w = dataclasses.replace(w, sources_fn=lambda w_, s=srcs: s)
    w._media_cache = None
    say("[c4 full-size solve (2 sources)]")
    S = _solver(w)
    B = rhs_matrix(w)
    x = torch.zeros_like(to_dev(B))
    st, stats = S.solve(to_dev(B), x, tol=1e-6, maxit=500)
    torch.cuda.synchronize()
    assert st == 0, stats
    got = from_dev(x)
    S.close()
    say("  oracle assembly of the 128^3 operator")
    A = oracle_problem(w).matrix()
    for r in range(2):
        res = np.linalg.norm(B[r] - A @ got[r]) / np.linalg.norm(B[r])
        say(f"  source {r}: iters {stats[r]['iters']} library {stats[r]['rel_res_true']:.3e} oracle {res:.3e}")
        assert res <= 1e-6
        assert abs(res - stats[r]["rel_res_true"]) <= 1e-9


def test_c5_gradient_matches_oracle_and_differences():
    """256^2, 16 sources, 128 receivers, complex64 cycle in FP64 FGMRES at
    tol 1e-10: the autograd media gradient against the oracle's adjoint-state
    gradient (sparse direct solves), and central differences (step 1e-4 of the
    cell value) through the library's solves on 20 random cells among those
    with at least 5 % of the largest sensitivity of their medium."""
    import test_gpu_gradient as T
    from paper_1806_11277_amd.autograd import spec_for_workload
    say("[c5 full size: oracle data, forward and adjoint fields]")
    w, m, mu_bar, rho_bar, B, rec, d_obs, pb = T._fwi_case("c5_fwi256_batch16")
    L_ref, ref = T._oracle_gradient(pb, B, rec, d_obs)
    spec = spec_for_workload(w, mu_bar=mu_bar, rho_bar=rho_bar)
    say("  library gradient")
    L, grads, _ = T._gpu_loss_and_grad(w, spec, m, B, rec, d_obs)
    say(f"  misfit gpu {L:.8e} oracle {L_ref:.8e}")
    assert abs(L - L_ref) <= 1e-8 * L_ref
    for name, got, want in zip(("lam", "mu", "rho"), grads, ref):
        err = np.max(np.abs(got - want)) / np.max(np.abs(want))
        say(f"  {name}: max error / max entry {err:.3e}")
        assert err <= 1e-6
    rng = np.random.default_rng(84)
    names = ["lam", "mu", "rho"]
    worst = 0.0
    for j in range(20):
        which = j % 3
        gflat = np.abs(grads[which]).reshape(-1)
        c = int(rng.choice(np.flatnonzero(gflat >= 0.05 * gflat.max())))
        base = m[names[which]]
        step = 1e-4 * abs(base.reshape(-1)[c])
        vals = []
        for sgn in (1.0, -1.0):
            pert = dict(m)
            arr = base.copy().reshape(-1)
            arr[c] += sgn * step
            pert[names[which]] = arr.reshape(base.shape)
            vals.append(T._gpu_loss(spec, pert, B, rec, d_obs))
        fd = (vals[0] - vals[1]) / (2 * step)
        an = grads[which].reshape(-1)[c]
        worst = max(worst, abs(fd - an) / abs(an))
        say(f"  {names[which]} cell {c}: fd {fd:.6e} adjoint {an:.6e}")
        assert abs(fd - an) <= 1e-4 * abs(an)
    say(f"  worst relative difference {worst:.3e}")


@pytest.mark.parametrize("with_e", [False, True])
@pytest.mark.parametrize("colour", [0, 1])
def test_c2_level1_relax_many_sources(c2_oracle, colour, with_e):
    """The 256^2 Galerkin level relaxed for 12 right-hand sides at once, the
    launch that stages each source's tile in LDS (more than eight sources),
    compared source by source with the oracle's half-sweep."""
    import torch
    w, pb, H = c2_oracle
    say(f"[c2 level 1 half-sweep, 12 sources, colour={colour} e_in={with_e}]")
    S = _solver(w)
    N = H.A[1].shape[0]
    assert S.level_info(0, 1)["N"] == N
    b = rand_cvec(N, 12, 80 + colour)
    e = rand_cvec(N, 12, 90 + colour) if with_e else np.zeros((12, N), complex)
    out = torch.zeros_like(to_dev(b))
    S.level_relax(0, 1, colour, to_dev(b), to_dev(e) if with_e else None, out)
    torch.cuda.synchronize()
    got = from_dev(out)
    for q in range(12):
        ref = H.relax(1, b[q], e[q], colour)
        assert np.linalg.norm(got[q] - ref) <= 1e-11 * np.linalg.norm(ref), q
    S.close()


@pytest.fixture(scope="module")
def ragged_oracle():
    from _helpers import small_hetero
    w = small_hetero((528, 520), "ragged528x520", levels=4)
    say("[528 x 520: oracle problem and hierarchy]")
    pb = oracle_problem(w)
    H = oracle_hierarchy(w, pb)
    return w, pb, H


@pytest.mark.parametrize("colour", [0, 1])
def test_ragged_level1_relax_many_sources(ragged_oracle, colour):
    """The LDS-staged half-sweep on a 264 x 260 Galerkin level, whose sides are
    not multiples of the 16 x 8 cell tile (partial tiles at the right and top
    walls), for 12 sources, against the oracle's half-sweep."""
    import torch
    w, pb, H = ragged_oracle
    say(f"[264 x 260 level half-sweep, 12 sources, colour={colour}]")
    S = _solver(w)
    N = H.A[1].shape[0]
    assert S.level_info(0, 1)["N"] == N
    b = rand_cvec(N, 12, 100 + colour)
    e = rand_cvec(N, 12, 110 + colour)
    out = torch.zeros_like(to_dev(b))
    S.level_relax(0, 1, colour, to_dev(b), to_dev(e), out)
    torch.cuda.synchronize()
    got = from_dev(out)
    for q in range(12):
        ref = H.relax(1, b[q], e[q], colour)
        assert np.linalg.norm(got[q] - ref) <= 1e-11 * np.linalg.norm(ref), q
    S.close()


def test_c2_level1_relax_component_damping(c2_oracle):
    """The LDS-staged half-sweep (256^2 Galerkin level, 12 sources) with the
    component damping (w_u, w_p) = (0.6, 0.4), against the oracle."""
    import torch
    from oracle import multigrid as mg
    w, pb, H = c2_oracle
    say("[c2 level 1 half-sweep, 12 sources, component damping]")
    H2 = mg.Hierarchy(H.A[0], pb.n, 2, [0.85], damping_p=[0.65])
    H2.A[1] = H.A[1]
    H2.blocks = [H2.blocks[0], mg.vanka_blocks(H.A[1], H.n[1])]
    H2.damping, H2.damping_p = [0.85, 0.6], [0.65, 0.4]
    S = _solver(w, damping=(0.85, 0.6, 0.5, 0.5), damping_p=(0.65, 0.4, 0.5, 0.5))
    N = H.A[1].shape[0]
    b = rand_cvec(N, 12, 170)
    e = rand_cvec(N, 12, 171)
    for colour in (0, 1):
        out = torch.zeros_like(to_dev(b))
        S.level_relax(0, 1, colour, to_dev(b), to_dev(e), out)
        torch.cuda.synchronize()
        got = from_dev(out)
        for q in range(12):
            ref = H2.relax(1, b[q], e[q], colour)
            assert np.linalg.norm(got[q] - ref) <= 1e-11 * np.linalg.norm(ref), (colour, q)
    S.close()
