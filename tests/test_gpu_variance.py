"""Posterior variance (Remark r:var: one solve per target) against the
oracle's dense weight-space formula, itself pinned to the function-space
variance of the k~-GP."""
import numpy as np
import pytest
import torch

import oracle as O
import synth

pytestmark = pytest.mark.gpu
C = pytest.importorskip("paper_2210_10210_amd.capi")

KERN = {"se": O.SE, "matern": O.MATERN}
# name, d, kernel, ell, nu, eps, N, sigma2, seed   (M small enough for dense Cholesky)
CASES = [
    ("1d_se", 1, "se", 0.1, None, 1e-8, 2000, 0.01, 51),
    ("2d_matern32", 2, "matern", 0.3, 1.5, 1e-3, 5000, 0.05, 52),
    ("3d_se", 3, "se", 0.4, None, 1e-3, 3000, 0.04, 53),
]


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


@pytest.mark.parametrize("prec", [torch.float32, torch.float64])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_variance_matches_dense_oracle(case, prec):
    name, d, kern, ell, nu, eps, N, s2, seed = case
    print(f"[variance] {name} {prec}", flush=True)
    x = synth.uniform_points(N, d, seed)
    y = torch.cos(6.0 * x.double().sum(0)) + synth.noise((N,), s2, seed)
    kw = dict(kernel=kern, lengthscale=ell, nu=nu or 0.0, eps=eps)
    if prec == torch.float64:
        kw["nufft_tol"] = 1e-12
    plan = C.efgp_setup(x.to(prec).cuda(), y.to(prec).cuda(), s2, **kw)
    P = O.Problem(d, KERN[kern], ell, nu, eps)
    assert plan.m == P.m
    xo = x.to(prec).double().numpy()
    v = O.toeplitz_vector(xo, P.h, P.m)
    # 70 targets: a full batch of 64 systems and a ragged one of 6
    t = synth.uniform_points(70, d, seed + 100).to(prec)
    rho = 1e-5 if prec == torch.float32 else 1e-12
    var, st, ss = C.efgp_variance(plan, t.cuda(), rel_tol=rho, max_iter=50000)
    assert st == C.EFGP_OK and ss["converged"] == 70 and ss["rel_residual"] <= 1.1 * rho
    want = O.posterior_variance(v, P.D, s2, P.m, d, P.h, t.double().numpy())
    got = var.cpu().double().numpy()
    # a solve to relative residual rho perturbs sigma^2 phi^H u by at most
    # rho |phi|^2 = rho k~(0); precision 32 adds float rounding of the grid
    k0 = float((P.D ** 2).sum())
    if prec == torch.float64:
        assert rel(got, want) <= 1e-8, rel(got, want)
    else:
        assert np.all(np.abs(got - want) <= 20 * rho * k0 + 1e-4 * want), np.abs(got - want).max()
    # the Jacobi-preconditioned solves give the same variances
    vj, stj, _ = C.efgp_variance(plan, t.cuda(), rel_tol=rho, max_iter=50000, precond=C.PRECOND_JACOBI)
    assert stj == C.EFGP_OK
    gj = vj.cpu().double().numpy()
    if prec == torch.float64:
        assert rel(gj, want) <= 1e-8
    else:
        assert np.all(np.abs(gj - want) <= 20 * rho * k0 + 1e-4 * want)


def test_variance_errors_and_bounds():
    d, N = 2, 4000
    x = synth.uniform_points(N, d, 61)
    y = torch.ones(N, dtype=torch.float64)
    plan = C.efgp_setup(x.cuda(), y.cuda(), 0.05, kernel="matern", nu=1.5, lengthscale=0.3, eps=1e-3)
    bad = torch.tensor([[0.5, 1.2], [0.5, 0.5]], dtype=torch.float64).cuda()
    with pytest.raises(C.EfgpError) as e:
        C.efgp_variance(plan, bad, rel_tol=1e-8)
    assert e.value.status == C.EFGP_EDOMAIN
    with pytest.raises(C.EfgpError) as e:
        C.efgp_variance(plan, bad[:, :1].contiguous(), r=1)
    assert e.value.status == C.EFGP_EINVAL
    # 0 < s <= k~(0)
    t = synth.uniform_points(40, d, 62).cuda()
    var, st, _ = C.efgp_variance(plan, t, rel_tol=1e-10, max_iter=20000)
    P = O.Problem(d, O.MATERN, 0.3, 1.5, 1e-3)
    k0 = float((P.D ** 2).sum())
    assert st == C.EFGP_OK and float(var.min()) > 0 and float(var.max()) <= k0 * (1 + 1e-9)


def test_refined_fp32_variance_matches_dense_oracle():
    """Precision 32 with refined solves (double residuals, single-precision
    inner PCG): the variances at 70 targets meet a residual of 1e-10 and
    match the oracle's dense weight-space formula to the FP32 setup's
    rounding, far tighter than the plain single-precision solve allows."""
    name, d, kern, ell, nu, eps, N, s2, seed = CASES[1]
    x = synth.uniform_points(N, d, seed)
    y = torch.cos(6.0 * x.double().sum(0)) + synth.noise((N,), s2, seed)
    plan = C.efgp_setup(x.float().cuda(), y.float().cuda(), s2, kernel=kern, lengthscale=ell, nu=nu, eps=eps)
    P = O.Problem(d, KERN[kern], ell, nu, eps)
    v = O.toeplitz_vector(x.float().double().numpy(), P.h, P.m)
    t = synth.uniform_points(70, d, seed + 100).float()
    var, st, ss = C.efgp_variance(plan, t.cuda(), rel_tol=1e-10, max_iter=200000, precond=C.PRECOND_JACOBI,
                                  refine=16)
    assert st in (C.EFGP_OK, C.EFGP_FELL_BACK) and ss["converged"] == 70 and ss["rel_residual"] <= 1.1e-10
    want = O.posterior_variance(v, P.D, s2, P.m, d, P.h, t.double().numpy())
    got = var.cpu().double().numpy()
    print(f"[variance] refined FP32 max rel err {np.max(np.abs(got - want) / want):.2e}")
    assert np.all(np.abs(got - want) <= 1e-4 * want)
