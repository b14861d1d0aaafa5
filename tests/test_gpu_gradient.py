"""Parity of the adjoint solve, the media-gradient contraction kernel and the
torch.autograd binding with the oracle, and of the gradient with central finite
differences through the library's own solves."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from _helpers import say, workload, small_hetero, oracle_problem, rand_cvec, to_dev, from_dev, rhs_matrix
from oracle import discretisation as D
from oracle import gradient as G

pytestmark = pytest.mark.gpu


def _solver(w, **over):
    import torch
    from paper_1806_11277_amd import ehh
    torch.cuda.synchronize()
    return ehh.solver_for_workload(w, **over)


def _media_t(m):
    import torch
    t = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda").contiguous()
    return t(m["lam"]), t(m["mu"]), t(m["rho"])


@pytest.mark.parametrize("n,levels", [((48, 40), 2), ((12, 10, 14), 2), ((64, 64), 3)])
def test_media_gradient_kernel_matches_oracle(n, levels):
    """Same random adjoint and forward fields on both sides; every cell of the
    three gradients within 1e-12 of the largest entry; accumulate adds."""
    import torch
    w = small_hetero(n, "gradk", levels=levels, damping=(0.75, 0.5))
    say(f"[media gradient kernel {n}]")
    pb = oracle_problem(w)
    S = _solver(w)
    sc = S.scaling()
    y = rand_cvec(pb.size, 3, 80)
    x = rand_cvec(pb.size, 3, 81)
    shape = tuple(reversed(n))
    outs = [torch.full(shape, np.nan, dtype=torch.float64, device="cuda") for _ in range(3)]
    S.media_gradient(to_dev(y), to_dev(x), *outs)
    torch.cuda.synchronize()
    ref = G.media_gradient(pb.n, pb.omega, pb.lam, pb.mu, pb.rho, pb.gamma_hat, y, x,
                           pb.nd["mu_bar"], pb.nd["rho_bar"])
    assert abs(sc["mu_bar"] - pb.nd["mu_bar"]) <= 1e-12 * pb.nd["mu_bar"]
    for got, want in zip(outs, ref):
        g = got.cpu().numpy()
        assert np.max(np.abs(g - want)) <= 1e-12 * np.max(np.abs(want))
    S.media_gradient(to_dev(y), to_dev(x), *outs, accumulate=True)
    torch.cuda.synchronize()
    for got, want in zip(outs, ref):
        assert np.max(np.abs(got.cpu().numpy() - 2 * want)) <= 2e-12 * np.max(np.abs(want))
    S.close()


@pytest.mark.parametrize("bits", [64, 32])
def test_adjoint_solve_matches_oracle(bits):
    import torch
    w = workload("c1_homog64", precond_bits=bits)
    say(f"[adjoint solve bits={bits}]")
    pb = oracle_problem(w)
    A = pb.matrix()
    g = rand_cvec(pb.size, 2, 82)
    want = G.adjoint_solve(A, g)
    S = _solver(w)
    y = torch.zeros((2, 2 * pb.size), dtype=torch.float64, device="cuda")
    st, stats = S.solve_adjoint(to_dev(g), y, tol=1e-10, maxit=600)
    torch.cuda.synchronize()
    assert st == 0, stats
    got = from_dev(y)
    for r in range(2):
        assert stats[r]["rel_res_true"] <= 1e-10
        assert np.linalg.norm(got[r] - want[r]) <= 1e-6 * np.linalg.norm(want[r])
        # the residual of the adjoint system itself, recomputed by the oracle
        assert np.linalg.norm(A.conj().T @ got[r] - g[r]) <= 1.01e-10 * np.linalg.norm(g[r])
    S.close()


def _fwi_case(name, **over):
    """Background and true media, fixed units (the background means), the
    right-hand sides, receiver offsets and the observed data (true model, sparse
    direct solve by the oracle)."""
    from workloads.configs import receiver_offsets
    w = workload(name, **over)
    m = w.media()
    mt = w.true_media_fn()
    mu_bar, rho_bar = float(np.mean(m["mu"])), float(np.mean(m["rho"]))
    B = rhs_matrix(w)
    rec = receiver_offsets(w)
    pt = D.Problem(w.n, w.h, w.omega, mt["lam"], mt["mu"], mt["rho"], w.abl_cells, w.abl_max, w.atten0,
                   mu_bar=mu_bar, rho_bar=rho_bar)
    lu = spla.splu(pt.matrix().tocsc())
    d_obs = np.stack([lu.solve(b)[rec] for b in B])
    pb = D.Problem(w.n, w.h, w.omega, m["lam"], m["mu"], m["rho"], w.abl_cells, w.abl_max, w.atten0,
                   mu_bar=mu_bar, rho_bar=rho_bar)
    return w, m, mu_bar, rho_bar, B, rec, d_obs, pb


def _oracle_gradient(pb, B, rec, d_obs):
    A = pb.matrix()
    lu = spla.splu(A.tocsc())
    X = np.stack([lu.solve(b) for b in B])
    L, g = G.receiver_misfit(X, rec, d_obs)
    Y = G.adjoint_solve(A, g)
    return L, G.media_gradient(pb.n, pb.omega, pb.lam, pb.mu, pb.rho, pb.gamma_hat, Y, X,
                               pb.nd["mu_bar"], pb.nd["rho_bar"])


def _torch_misfit(x, rec, d_obs):
    import torch
    N = x.shape[1] // 2
    idx = torch.as_tensor(rec, device=x.device)
    dr = torch.as_tensor(d_obs.real, device=x.device)
    di = torch.as_tensor(d_obs.imag, device=x.device)
    return 0.5 * (((x[:, idx] - dr) ** 2).sum() + ((x[:, N + idx] - di) ** 2).sum())


def _gpu_loss_and_grad(w, spec, m, B, rec, d_obs, media_grad=True):
    import torch
    from paper_1806_11277_amd.autograd import elastic_helmholtz_solve
    lam, mu, rho = (t.requires_grad_(media_grad) for t in _media_t(m))
    b = to_dev(B).requires_grad_(True)
    x = elastic_helmholtz_solve(b, lam, mu, rho, spec)
    L = _torch_misfit(x, rec, d_obs)
    L.backward()
    torch.cuda.synchronize()
    return float(L), [t.grad.cpu().numpy() for t in (lam, mu, rho)], b.grad


def _gpu_loss(spec, media, B, rec, d_obs):
    import torch
    from paper_1806_11277_amd.autograd import elastic_helmholtz_solve
    with torch.no_grad():
        x = elastic_helmholtz_solve(to_dev(B), *_media_t(media), spec)
        return float(_torch_misfit(x, rec, d_obs))


def test_autograd_gradient_matches_oracle_and_differences():
    """64 x 64, 4 sources, 32 receivers, FP64 cycle, tol 1e-12: the autograd
    gradient equals the oracle's adjoint-state gradient to 1e-7 of its largest
    entry; dL/db equals the oracle's adjoint field; central differences (step
    1e-4 of the cell value) through the library's solves agree to 1e-4."""
    from paper_1806_11277_amd.autograd import spec_for_workload
    w, m, mu_bar, rho_bar, B, rec, d_obs, pb = _fwi_case("c5s_fwi64_batch4")
    say("[autograd c5s]")
    spec = spec_for_workload(w, mu_bar=mu_bar, rho_bar=rho_bar, tol=1e-12, maxit=800)
    L, grads, gb = _gpu_loss_and_grad(w, spec, m, B, rec, d_obs)
    L_ref, ref = _oracle_gradient(pb, B, rec, d_obs)
    say(f"  misfit gpu {L:.6e} oracle {L_ref:.6e}")
    assert abs(L - L_ref) <= 1e-9 * L_ref
    for got, want in zip(grads, ref):
        assert np.max(np.abs(got - want)) <= 1e-7 * np.max(np.abs(want))
    # dL/db = y (adjoint field of the misfit gradient)
    A = pb.matrix()
    lu = spla.splu(A.tocsc())
    X = np.stack([lu.solve(b) for b in B])
    _, gx = G.receiver_misfit(X, rec, d_obs)
    Y = G.adjoint_solve(A, gx)
    assert np.linalg.norm(from_dev(gb) - Y) <= 1e-8 * np.linalg.norm(Y)
    # central differences on cells with a sizeable sensitivity
    rng = np.random.default_rng(83)
    names = ["lam", "mu", "rho"]
    for j in range(6):
        which = j % 3
        gflat = np.abs(grads[which]).reshape(-1)
        cand = np.flatnonzero(gflat >= 0.05 * gflat.max())
        c = int(rng.choice(cand))
        base = m[names[which]]
        step = 1e-4 * abs(base.reshape(-1)[c])
        vals = []
        for sgn in (1.0, -1.0):
            pert = dict(m)
            arr = base.copy().reshape(-1)
            arr[c] += sgn * step
            pert[names[which]] = arr.reshape(base.shape)
            vals.append(_gpu_loss(spec, pert, B, rec, d_obs))
        fd = (vals[0] - vals[1]) / (2 * step)
        an = grads[which].reshape(-1)[c]
        say(f"  {names[which]} cell {c}: fd {fd:.6e} adjoint {an:.6e}")
        assert abs(fd - an) <= 1e-4 * abs(an)


def test_autograd_requires_fixed_units():
    from paper_1806_11277_amd.autograd import spec_for_workload, elastic_helmholtz_solve
    w = workload("c5s_fwi64_batch4")
    lam, mu, rho = (t.requires_grad_(True) for t in _media_t(w.media()))
    with pytest.raises(ValueError):
        elastic_helmholtz_solve(to_dev(rhs_matrix(w)), lam, mu, rho, spec_for_workload(w))
