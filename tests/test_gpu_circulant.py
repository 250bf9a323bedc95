"""Circulant preconditioner (T. Chan's optimal circulant of the Jacobi-scaled
weight-space system) on the GPU against the FP64 oracle, through the C ABI.

Parity of the eigenvalues with the oracle's dense definition (Rayleigh
quotients at the Fourier vectors): 1e-9 relative in precision 64, 1e-4 in
precision 32 (float FFTs of the autocorrelation and of the wrapped sums).
Parity of preconditioned CG: the residual histories of the GPU and oracle
PCG agree while rounding has not yet separated them, and both reach the
dense solution.  The gain claim (fewer iterations than Jacobi and plain CG
on clustered points) is checked at N = 1e7 in 3D.
"""
import numpy as np
import pytest
import torch

import oracle as O
import synth

pytestmark = pytest.mark.gpu
C = pytest.importorskip("paper_2210_10210_amd.capi")

KERN = {"se": O.SE, "matern": O.MATERN}


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _points(d, n, seed, clustered):
    if clustered:
        return synth.mixture_points(n, d, seed)
    return synth.uniform_points(n, d, seed)


def _data(x, seed):
    d = x.shape[0]
    w = torch.tensor([3.0, 2.0, 4.0][:d], dtype=torch.float64)
    return synth.f_plane_wave(x, w) + synth.noise((x.shape[1],), 0.04, seed)


# name, d, kernel, ell, nu, eps, m, N, sigma2, clustered, seed
EIG_CASES = [
    ("1d_se_m40", 1, "se", 0.05, None, 1e-6, 40, 3000, 0.01, False, 1),
    ("2d_matern32_mix_m16", 2, "matern", 0.1, 1.5, 1e-3, 16, 20000, 0.05, True, 2),
    ("2d_se_uniform_m12", 2, "se", 0.15, None, 1e-4, 12, 5000, 0.2, False, 3),
    ("3d_se_mix_m5", 3, "se", 0.3, None, 1e-3, 5, 4000, 0.04, True, 4),
]


@pytest.mark.parametrize("case", EIG_CASES, ids=[c[0] for c in EIG_CASES])
@pytest.mark.parametrize("precision", [64, 32])
def test_eigenvalues_match_oracle_definition(case, precision):
    name, d, kern, ell, nu, eps, m, N, s2, clustered, seed = case
    print(f"[circulant eigs] {name} precision {precision}", flush=True)
    x = _points(d, N, seed, clustered)
    y = _data(x, seed)
    P = O.Problem(d, KERN[kern], ell, nu, eps, m=m)
    v = O.toeplitz_vector(x.numpy(), P.h, P.m)
    K = O.circulant_period(m)
    ref = O.circulant_precond_eigs(v, P.D, s2, N, m, d, K)
    dt = torch.float64 if precision == 64 else torch.float32
    plan = C.efgp_setup(x.to(dt).cuda(), y.to(dt).cuda(), s2, kernel=kern, lengthscale=ell, nu=nu or 0.0,
                        eps=eps, m=m)
    lam, Kg = C.efgp_circulant_eigs(plan)
    assert Kg == K
    got = lam.double().cpu().numpy()
    assert rel(got, ref) <= (1e-9 if precision == 64 else 1e-4)
    # the eigenvalues are bounded below by (K^d - M + sum sigma^2/J) / K^d
    s0 = np.sum(s2 / (N * P.D ** 2 + s2))
    assert got.min() >= (K ** d - P.M + s0) / K ** d * (1 - 1e-6)


def test_eigenvalues_per_system_and_errors():
    x = synth.uniform_points(3000, 2, 9)
    y = torch.stack([_data(x, 9), _data(x, 10), _data(x, 11)])
    s2 = (0.01, 0.1, 1.0)
    plan = C.efgp_setup(x.cuda(), y.cuda(), s2, kernel="se", lengthscale=0.2, eps=1e-4, m=10)
    P = O.Problem(2, O.SE, 0.2, None, 1e-4, m=10)
    v = O.toeplitz_vector(x.numpy(), P.h, P.m)
    for r in range(3):
        lam, K = C.efgp_circulant_eigs(plan, r)
        assert rel(lam.cpu().numpy(), O.circulant_precond_eigs(v, P.D, s2[r], 3000, 10, 2, K)) <= 1e-9
    assert C.lib.efgp_circulant_eigs(plan.handle, 3, None, None, None) == C.EFGP_EINVAL
    assert C.lib.efgp_circulant_eigs(plan.handle, -1, None, None, None) == C.EFGP_EINVAL
    assert C.lib.efgp_circulant_eigs(None, 0, None, None, None) == C.EFGP_EINVAL
    # a kernel-only plan (prior sampling) has no points and no system
    prior = C.efgp_prior_setup(2, kernel="se", lengthscale=0.2, eps=1e-4, nsamp=1)
    assert C.lib.efgp_circulant_eigs(prior.handle, 0, None, None, None) == C.EFGP_EINVAL


@pytest.mark.parametrize("d,m,clustered", [(1, 60, True), (2, 18, True), (3, 5, False)])
def test_pcg_history_matches_oracle_fp64(d, m, clustered):
    """Same preconditioner on both sides (the oracle's from its dense
    definition): the residual histories coincide until rounding separates
    them, and both reach the dense solution."""
    print(f"[circulant pcg fp64] d={d} m={m}", flush=True)
    N, s2, ell, eps = 20000, 0.02, (0.05, 0.1, 0.3)[d - 1], 1e-4
    x = _points(d, N, 20 + d, clustered)
    y = _data(x, 20 + d)
    P = O.Problem(d, O.MATERN, ell, 2.5, eps, m=m)
    v, b = O.setup(P, x.numpy(), y.numpy())
    lam = O.circulant_precond_eigs(v, P.D, s2, N, m, d)
    apply = lambda z: O.system_apply(v, P.D, s2, z, m, d, fast=True)
    pre = lambda r: O.circulant_precond_apply(lam, P.D, s2, N, m, d, r)
    xo, ho, ito = O.cg(apply, b, 1e-10, 5000, precond=pre)
    exact = O.solve_dense(v, P.D, s2, b, m, d)
    plan = C.efgp_setup(x.cuda(), y.cuda(), s2, kernel="matern", nu=2.5, lengthscale=ell, eps=eps, m=m)
    beta, st, ss = C.efgp_solve(plan, rel_tol=1e-10, max_iter=5000, precond=C.PRECOND_CIRCULANT,
                                record_history=True)
    assert st == C.EFGP_OK and ss["fell_back"] == 0
    hg = np.array(ss["history"])
    n = min(15, len(hg), len(ho) - 1)
    np.testing.assert_allclose(hg[:n], np.array(ho[1:n + 1]), rtol=1e-6)
    # late iterations drift apart by rounding at this conditioning
    assert abs(ss["iterations"] - ito) <= max(3, 0.1 * ito)
    # A >= sigma^2 I: two approximate solutions differ by at most the sum of
    # their residuals / sigma^2 (residuals taken by the oracle's product)
    bg = beta[0].cpu().numpy()
    rg = np.linalg.norm(b - apply(bg))
    re = np.linalg.norm(b - apply(exact))
    assert rg <= 1.1e-10 * np.linalg.norm(b)
    assert np.linalg.norm(bg - exact) <= (rg + re) / s2
    assert np.linalg.norm(bg - xo) <= (rg + np.linalg.norm(b - apply(xo))) / s2


def _cfg3_plan(n, dtype=torch.float32):
    """3D SE, lengthscale 0.2, eps 1e-5, points from a 20-component Gaussian
    mixture (std 0.05) clipped to the cube, y = prod sin(4 pi x_i) + N(0, 0.04)."""
    x = synth.mixture_points(n, 3, 7, dtype=dtype, device="cuda")
    y = (synth.f_sinprod(x) + synth.noise((n,), 0.04, 7, dtype=dtype, device="cuda")).contiguous()
    return C.efgp_setup(x, y, 0.04, kernel="se", lengthscale=0.2, eps=1e-5), x


def test_clustered_3d_fewer_iterations_than_jacobi_and_plain():
    plan, x = _cfg3_plan(10_000_000)
    it = {}
    betas = {}
    for name, pc in (("plain", C.PRECOND_NONE), ("jacobi", C.PRECOND_JACOBI), ("circulant", C.PRECOND_CIRCULANT)):
        beta, st, ss = C.efgp_solve(plan, rel_tol=1e-5, max_iter=50000, precond=pc)
        assert st in (C.EFGP_OK, C.EFGP_FELL_BACK), name
        assert ss["rel_residual"] <= 1.1e-5, name
        it[name] = ss["iterations"]
        betas[name] = beta.clone()
    print(f"[circulant cfg3] iterations {it}", flush=True)
    assert it["circulant"] < it["jacobi"] and it["circulant"] < it["plain"]
    # Same answer class: at the data points the mean is Phi beta and, with
    # A = Phi^H Phi + sigma^2 I (D folded into Phi), |Phi e|^2 <= e^H A e =
    # r^H A^-1 r <= |r|^2 / sigma^2 for the error e of a solution with
    # residual r, so the two means differ by at most (|r_c| + |r_j|) / sigma
    # in l2 over the N points (plus the two evaluations' own NUFFT error).
    bn = float(torch.linalg.vector_norm(C.efgp_get_rhs(plan)))
    mu_c = C.efgp_mean_at_points(plan, betas["circulant"], x).double()
    mu_j = C.efgp_mean_at_points(plan, betas["jacobi"], x).double()
    diff = float(torch.linalg.vector_norm(mu_c - mu_j))
    bound = 2 * 1.1e-5 * bn / 0.2 + 1e-5 * float(torch.linalg.vector_norm(mu_j))
    print(f"[circulant cfg3] |mu_c - mu_j| = {diff:.3e}, bound {bound:.3e}", flush=True)
    assert diff <= bound


def test_graph_and_plain_launch_identical_multi_rhs():
    x = synth.mixture_points(400_000, 2, 12, dtype=torch.float32, device="cuda")
    y = torch.stack([(synth.f_plane_wave(x, torch.tensor([3.0, 1.0 + k])) +
                      synth.noise((x.shape[1],), 0.05, 30 + k, dtype=torch.float32, device="cuda")).float()
                     for k in range(3)]).contiguous()
    plan = C.efgp_setup(x, y, (0.02, 0.05, 0.2), kernel="matern", nu=1.5, lengthscale=0.1, eps=1e-3)
    b1, s1, a1 = C.efgp_solve(plan, rel_tol=1e-5, max_iter=20000, precond=C.PRECOND_CIRCULANT,
                              launch=C.LAUNCH_GRAPH)
    b2, s2, a2 = C.efgp_solve(plan, rel_tol=1e-5, max_iter=20000, precond=C.PRECOND_CIRCULANT,
                              launch=C.LAUNCH_PLAIN)
    assert s1 == C.EFGP_OK and s2 == C.EFGP_OK
    assert a1["iterations"] == a2["iterations"] and torch.equal(b1, b2)
    assert a1["converged"] == 3 and a1["rel_residual"] <= 1.1e-5


def test_stall_fallback_and_warm_start():
    x = synth.mixture_points(300_000, 2, 13, dtype=torch.float32, device="cuda")
    y = (synth.f_cos2d(x) + synth.noise((x.shape[1],), 0.05, 13, dtype=torch.float32, device="cuda")).contiguous()
    plan = C.efgp_setup(x, y, 0.05, kernel="matern", nu=1.5, lengthscale=0.1, eps=1e-3)
    # a stall window of one iteration forces the fallback to plain CG
    beta, st, ss = C.efgp_solve(plan, rel_tol=1e-5, max_iter=50000, precond=C.PRECOND_CIRCULANT,
                                stall_window=1, iters_per_sync=4)
    assert st in (C.EFGP_FELL_BACK, C.EFGP_OK) and ss["rel_residual"] <= 1.1e-5
    # warm start from a coarse solution: the restart recomputes z = P r
    coarse, st, sc = C.efgp_solve(plan, rel_tol=1e-2, precond=C.PRECOND_CIRCULANT)
    fine, st, sf = C.efgp_solve(plan, rel_tol=1e-5, max_iter=50000, precond=C.PRECOND_CIRCULANT,
                                beta_init=coarse, record_history=True)
    cold, st2, sc2 = C.efgp_solve(plan, rel_tol=1e-5, max_iter=50000, precond=C.PRECOND_CIRCULANT)
    assert st == C.EFGP_OK and st2 == C.EFGP_OK
    assert sf["rel_residual"] <= 1.1e-5
    # the warm run continues from the coarse residual (a cold start begins
    # near 1); CG's hard phase is the last digits, so it saves few iterations
    assert sf["history"][0] <= 3e-2 and sf["iterations"] <= 1.2 * sc2["iterations"]


def test_variance_with_circulant_matches_jacobi_fp64():
    x = synth.mixture_points(5000, 2, 14)
    y = _data(x, 14)
    plan = C.efgp_setup(x.cuda(), y.cuda(), 0.05, kernel="matern", nu=1.5, lengthscale=0.1, eps=1e-3)
    t = synth.uniform_points(70, 2, 15).cuda()
    vj, sj, _ = C.efgp_variance(plan, t, rel_tol=1e-10, max_iter=20000, precond=C.PRECOND_JACOBI)
    vc, sc, stc = C.efgp_variance(plan, t, rel_tol=1e-10, max_iter=20000, precond=C.PRECOND_CIRCULANT)
    assert sj == C.EFGP_OK and sc == C.EFGP_OK and stc["converged"] == 70
    # each variance sigma^2 phi^H u is off by at most |phi| |r| <= rho |phi|^2
    # (A >= sigma^2 I), and |phi|^2 = sum_j D_j^2
    phi2 = float((C.efgp_get_weights(plan) ** 2).sum())
    assert float((vc - vj).abs().max()) <= 2.2e-10 * phi2


def test_large_grid_multikernel_path_fp64():
    """A K^d grid too large for one workgroup's LDS (K = 125 in 2D, precision
    64: 250 KB) takes the multi-kernel application; its solution matches the
    oracle's CG solution within the residual bound and it beats Jacobi on
    clustered points."""
    d, m, N, s2 = 2, 60, 200_000, 0.02
    x = synth.mixture_points(N, d, 40)
    y = _data(x, 40)
    P = O.Problem(d, O.MATERN, 0.05, 1.5, 1e-4, m=m)
    v, b = O.setup(P, x.numpy(), y.numpy())
    apply = lambda z: O.system_apply(v, P.D, s2, z, m, d, fast=True)
    xo, _, _ = O.cg(apply, b, 1e-11, 20000, precond=1.0 / (N * P.D ** 2 + s2))
    plan = C.efgp_setup(x.cuda(), y.cuda(), s2, kernel="matern", nu=1.5, lengthscale=0.05, eps=1e-4, m=m)
    assert O.circulant_period(m) ** 2 * 16 > 160 * 1024
    bc, st, sc = C.efgp_solve(plan, rel_tol=1e-10, max_iter=20000, precond=C.PRECOND_CIRCULANT)
    _, stj, sj = C.efgp_solve(plan, rel_tol=1e-10, max_iter=20000, precond=C.PRECOND_JACOBI)
    assert st == C.EFGP_OK and stj == C.EFGP_OK and sc["fell_back"] == 0
    print(f"[circulant large grid] iterations circulant {sc['iterations']} jacobi {sj['iterations']}", flush=True)
    assert sc["iterations"] < sj["iterations"]
    bg = bc[0].cpu().numpy()
    rg = np.linalg.norm(b - apply(bg))
    assert rg <= 1.1e-10 * np.linalg.norm(b)
    assert np.linalg.norm(bg - xo) <= (rg + np.linalg.norm(b - apply(xo))) / s2
