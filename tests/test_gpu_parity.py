"""GPU parity: every stage of the HIP path against the FP64 oracle on the
same seeded inputs (through the C ABI).

Tolerances (relative l2 over the whole vector; posterior means, v and b are
also held to an l-infinity bound, max|err| / max|want| <= 3 tol, so that one
bad entry cannot hide in the l2 norm):
  precision 64: 1e-9 for v, b, A beta, mu and the solve (the target for the
                double path; NUFFT tolerance 1e-12);
  precision 32: 1e-4 on the posterior mean against the FP64 oracle; stage
                values are checked at 1e-4 as well (float spreading at the
                plan's NUFFT tolerance plus float FFTs).
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
import synth

pytestmark = pytest.mark.gpu

C = pytest.importorskip("paper_2210_10210_amd.capi")


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def rel_inf(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


def close(a, b, tol, what=""):
    """Relative l2 error <= tol and relative max error <= 3 tol."""
    e2, ei = rel(a, b), rel_inf(a, b)
    print(f"[close] {what} l2 {e2:.2e} linf {ei:.2e} tol {tol:.0e}", flush=True)
    return e2 <= tol and ei <= 3 * tol


KERN = {"se": O.SE, "matern": O.MATERN}

# name, d, kernel, ell, nu, eps, N, sigma2, seed
CASES = [
    ("1d_se_n2000", 1, "se", 0.1, None, 1e-8, 2000, 0.01, 1),
    ("2d_matern32_n20000", 2, "matern", 0.1, 1.5, 1e-4, 20000, 0.09, 2),
    ("3d_se_n3000", 3, "se", 0.2, None, 1e-5, 3000, 0.04, 3),
    ("2d_se_ragged_n37", 2, "se", 0.25, None, 1e-6, 37, 0.05, 4),
    # nu > 5/2: h and m from the uniform-error rule, eq. (maternhm)
    ("2d_matern72_n5000", 2, "matern", 0.3, 3.5, 1e-3, 5000, 0.05, 5),
]


def _inputs(d, N, seed, f=None):
    x = synth.uniform_points(N, d, seed)
    w = torch.tensor([3.0, 6.0, 4.0][:d], dtype=torch.float64) / math.sqrt(5.0)
    y = synth.f_plane_wave(x, w) + synth.noise((N,), 0.09, seed)
    return x, y


def _oracle_exact(v, P, s2, b):
    """Exact weight-space solution: dense Cholesky when small, else the
    oracle's CG with the paper's fast Toeplitz product to 1e-13."""
    if P.M <= 6000:
        return O.solve_dense(v, P.D, s2, b, P.m, P.dim)
    apply = lambda z: O.system_apply(v, P.D, s2, z, P.m, P.dim, fast=True)
    xk, hist, _ = O.cg(apply, b, 1e-13, 100000)
    return xk


def _oracle_setup(case, x, y):
    name, d, kern, ell, nu, eps, N, s2, seed = case
    P = O.Problem(d, KERN[kern], ell, nu, eps)
    v, b = O.setup(P, x, y)
    return P, v, b


@pytest.fixture(scope="module", params=CASES, ids=[c[0] for c in CASES])
def fp64_case(request):
    case = request.param
    name, d, kern, ell, nu, eps, N, s2, seed = case
    print(f"[parity fp64] {name}", flush=True)
    x, y = _inputs(d, N, seed)
    xn, yn = x.numpy(), y.numpy()
    P, v, b = _oracle_setup(case, xn, yn)
    plan = C.efgp_setup(x.cuda(), y.cuda(), s2, kernel=kern, lengthscale=ell, nu=nu or 0.0, eps=eps)
    return case, x, y, P, v, b, plan


def test_parameters_match_oracle(fp64_case):
    case, x, y, P, v, b, plan = fp64_case
    assert plan.m == P.m
    assert plan.h == pytest.approx(P.h, rel=1e-13)
    D = C.efgp_get_weights(plan).cpu().numpy()
    assert rel(D, P.D) <= 1e-13


def test_setup_v_and_b(fp64_case):
    case, x, y, P, v, b, plan = fp64_case
    vg = C.efgp_get_toeplitz(plan).cpu().numpy()
    bg = C.efgp_get_rhs(plan).cpu().numpy()[0]
    assert close(vg, v, 1e-9, "v")
    assert close(bg, b, 1e-9, "b")
    N = x.shape[1]
    c = (vg.size - 1) // 2
    assert abs(vg[c] - N) <= 1e-9 * N
    np.testing.assert_allclose(vg[::-1], np.conj(vg), atol=1e-9 * N)


def test_apply_matches_dense_toeplitz(fp64_case):
    case, x, y, P, v, b, plan = fp64_case
    s2 = case[7]
    g = torch.Generator().manual_seed(11)
    beta = torch.randn(P.M, dtype=torch.complex128, generator=g)
    out = C.efgp_apply(plan, beta.reshape(1, -1).cuda()).cpu().numpy()[0]
    want = O.system_apply(v, P.D, s2, beta.numpy(), P.m, P.dim)
    assert rel(out, want) <= 1e-9


def test_apply_fp64_largest_embedding():
    """2D at m = 250: L = 1024, the largest embedding the plan limits allow.
    In double precision the column pass that multiplies by FFT(v) needs just
    over 64 KB of LDS for its one line per block; the product (eq. (97) by
    the embedding FFT) still matches the oracle's to 1e-9."""
    d, N, m, s2 = 2, 40, 250, 0.05
    x, y = _inputs(d, N, 31)
    P = O.Problem(d, O.SE, 0.02, None, 1e-6, m=m)
    v, _ = O.setup(P, x.numpy(), y.numpy())
    plan = C.efgp_setup(x.cuda(), y.cuda(), s2, kernel="se", lengthscale=0.02, eps=1e-6, m=m)
    assert plan.m == m and plan.info.L == 1024
    g = torch.Generator().manual_seed(32)
    beta = torch.randn(P.M, dtype=torch.complex128, generator=g)
    out = C.efgp_apply(plan, beta.reshape(1, -1).cuda()).cpu().numpy()[0]
    want = O.system_apply(v, P.D, s2, beta.numpy(), m, d, fast=True)
    assert rel(out, want) <= 1e-9


def test_eval_matches_direct_sum(fp64_case):
    case, x, y, P, v, b, plan = fp64_case
    d = P.dim
    g = torch.Generator().manual_seed(12)
    # a Hermitian-symmetric beta (real data give one) -> real posterior mean
    beta = torch.randn(P.M, dtype=torch.complex128, generator=g).numpy()
    beta = 0.5 * (beta + np.conj(beta[::-1]))
    t = synth.uniform_points(777, d, 99)
    mu = C.efgp_eval(plan, torch.as_tensor(beta).reshape(1, -1).cuda(), t.cuda()).cpu().numpy()[0]
    want, im = O.posterior_mean(beta, P.D, P.h, P.m, t.numpy())
    assert close(mu, want, 1e-9, "eval")
    assert C.efgp_eval_status(plan) == C.EFGP_OK


def test_mean_at_points_matches_direct_sum(fp64_case):
    """Step 7 (eq. (bmu)): the mean at the N observation points is the type-2
    sum at q = N; it equals efgp_eval at targets = x bit for bit."""
    case, x, y, P, v, b, plan = fp64_case
    g = torch.Generator().manual_seed(13)
    beta = torch.randn(P.M, dtype=torch.complex128, generator=g).numpy()
    beta = 0.5 * (beta + np.conj(beta[::-1]))
    bt = torch.as_tensor(beta).reshape(1, -1).cuda()
    mu = C.efgp_mean_at_points(plan, bt, x.cuda())
    want, _ = O.posterior_mean(beta, P.D, P.h, P.m, x.numpy())
    assert close(mu.cpu().numpy()[0], want, 1e-9, "mean at points")
    assert torch.equal(mu, C.efgp_eval(plan, bt, x.cuda()))


@pytest.mark.parametrize("eps", [1e-2, 1e-3, 1e-5])
def test_eval_fp32_2d_widths_and_edges(eps):
    """Single-precision 2D interpolation from the LDS window against the
    oracle's direct type-2 sum (eq. (bmu)), for the widths 4, 5 and 7 (three
    kernel width classes), three coefficient vectors, and targets on the
    domain's edges and corners, where the stencil reaches the window's last
    rows and columns."""
    d, N = 2, 3000
    x, y = _inputs(d, N, 71)
    ys = torch.stack([y, 0.5 * y, -y])
    plan = C.efgp_setup(x.float().cuda(), ys.float().cuda(), [0.09] * 3, kernel="matern", nu=1.5,
                        lengthscale=0.1, eps=eps)
    info = C.efgp_get_info(plan)
    P = O.Problem(d, O.MATERN, 0.1, 1.5, eps)
    assert P.m == plan.m
    g = torch.Generator().manual_seed(72)
    beta = torch.randn(3, P.M, dtype=torch.complex128, generator=g).numpy()
    beta = 0.5 * (beta + np.conj(beta[:, ::-1]))
    edge = np.array([[0.0, 1.0, 0.0, 1.0, 0.5, 0.5, 0.0, 1.0, 1.0 - 1e-7],
                     [0.0, 1.0, 1.0, 0.0, 0.0, 1.0, 0.5, 0.5, 1.0 - 1e-7]])
    t = np.concatenate([synth.uniform_points(700, d, 73).numpy(), edge], axis=1)
    t32 = torch.as_tensor(t).float()
    mu = C.efgp_eval(plan, torch.as_tensor(beta).to(torch.complex64).cuda(), t32.cuda()).cpu().double().numpy()
    tol = max(10 * info["nufft_tol"], 1e-5)
    for r in range(3):
        b32 = torch.as_tensor(beta[r]).to(torch.complex64).to(torch.complex128).numpy()
        want, _ = O.posterior_mean(b32, P.D, P.h, P.m, t32.double().numpy())
        assert close(mu[r], want, tol, f"fp32 eval eps {eps} r {r}"), r
    assert C.efgp_eval_status(plan) == C.EFGP_OK


@pytest.mark.parametrize("prec", [torch.float32, torch.float64])
def test_eval_global_grid_fallback(prec):
    """A type-2 grid whose active window exceeds LDS (2D, m = 120) takes the
    global-memory interpolation; it matches the direct sum like the LDS path."""
    d, N = 2, 3000
    x, y = _inputs(d, N, 21)
    kw = dict(kernel="matern", nu=1.5, lengthscale=0.1, eps=1e-4, m=120)
    if prec == torch.float64:
        kw["nufft_tol"] = 1e-12
    plan = C.efgp_setup(x.to(prec).cuda(), y.to(prec).cuda(), 0.09, **kw)
    assert plan.m == 120
    P = O.Problem(d, O.MATERN, 0.1, 1.5, 1e-4)
    D = O.spectral_weights(P.h, 120, d, O.MATERN, 0.1, 1.5)
    g = torch.Generator().manual_seed(14)
    beta = torch.randn(241 * 241, dtype=torch.complex128, generator=g).numpy()
    beta = 0.5 * (beta + np.conj(beta[::-1]))
    t = synth.uniform_points(500, d, 98)
    cdt = torch.complex64 if prec == torch.float32 else torch.complex128
    mu = C.efgp_eval(plan, torch.as_tensor(beta).to(cdt).reshape(1, -1).cuda(), t.to(prec).cuda())
    want, _ = O.posterior_mean(beta, D, P.h, 120, t.to(prec).double().numpy())
    assert close(mu.cpu().double().numpy()[0], want, 1e-5 if prec == torch.float32 else 1e-9, "global-grid eval")


def test_solve_residual_and_mean(fp64_case):
    case, x, y, P, v, b, plan = fp64_case
    s2 = case[7]
    beta, st, stats = C.efgp_solve(plan, rel_tol=1e-11, max_iter=20000)
    assert st == C.EFGP_OK, stats
    bg = beta.cpu().numpy()[0]
    # the oracle's own residual of the GPU solution (kappa-free check)
    r = O.system_apply(v, P.D, s2, bg, P.m, P.dim) - b
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1.1e-11 + 1e-9
    assert stats["rel_residual"] <= 1.1e-11
    # posterior mean against the oracle's exact (Cholesky) solution
    exact = _oracle_exact(v, P, s2, b)
    t = synth.uniform_points(500, P.dim, 98)
    mu = C.efgp_eval(plan, beta, t.cuda()).cpu().numpy()[0]
    want, _ = O.posterior_mean(exact, P.D, P.h, P.m, t.numpy())
    assert close(mu, want, 1e-9, "solved mean")


@pytest.mark.parametrize("launch", ["graph", "plain", "block"])
def test_systems_stopping_at_different_iterations(launch):
    """Three data vectors with sigma^2 a factor 1000 apart stop at very
    different iterations.  Each keeps full products until it stops (blocks of
    stopped systems return early): the oracle's own residual of every GPU
    solution is at the tolerance, its posterior mean matches the one of the
    oracle's exact dense solve, and each system's iteration count equals that
    of its own one-vector solve."""
    d, N, m = 2, 3000, 15
    x, y0 = _inputs(d, N, 61)
    y = torch.stack([y0, -0.5 * y0 + 0.2, torch.cos(7.0 * x[0]) * y0])
    s2 = [1.0, 0.03, 0.001]
    kw = dict(kernel="matern", nu=1.5, lengthscale=0.1, eps=1e-4, m=m, nufft_tol=1e-12)
    lm = {"graph": C.LAUNCH_GRAPH, "plain": C.LAUNCH_PLAIN, "block": C.LAUNCH_BLOCK}[launch]
    plan = C.efgp_setup(x.cuda(), y.cuda(), s2, **kw)
    beta, st, ss = C.efgp_solve(plan, rel_tol=1e-10, max_iter=20000, launch=lm)
    assert st == C.EFGP_OK and ss["converged"] == 3
    P = O.Problem(d, O.MATERN, 0.1, 1.5, 1e-4, m=m)
    t = synth.uniform_points(300, d, 62).numpy()
    its = []
    for r in range(3):
        v, b = O.setup(P, x.numpy(), y[r].numpy())
        br = beta[r].cpu().numpy()
        res = O.system_apply(v, P.D, s2[r], br, m, d) - b
        assert np.linalg.norm(res) / np.linalg.norm(b) <= 1.1e-10 + 1e-9, r
        exact = O.solve_dense(v, P.D, s2[r], b, m, d)
        mu, _ = O.posterior_mean(br, P.D, P.h, m, t)
        want, _ = O.posterior_mean(exact, P.D, P.h, m, t)
        assert close(mu, want, 1e-7, f"system {r} mean"), r
        one = C.efgp_setup(x.cuda(), y[r:r + 1].contiguous().cuda(), s2[r], **kw)
        _, _, s1 = C.efgp_solve(one, rel_tol=1e-10, max_iter=20000, launch=lm)
        its.append(s1["iterations"])
    assert len(set(its)) == 3, its          # they do stop at different iterations
    # (double-atomic setups differ in the last bits, which can move a count
    # of a few thousand iterations by one or two)
    assert abs(ss["iterations"] - max(its)) <= max(2, 0.02 * max(its)), (ss["iterations"], its)


@pytest.mark.parametrize("prec", [torch.float64, torch.float32])
@pytest.mark.parametrize("m", [11, 15])
def test_hermitian_product_matches_general_path(prec, m):
    """Real data keep the 2D CG vectors Hermitian, and Jacobi PCG then runs
    the product on rows 0..m with paired columns.  The same iteration
    through the general path (the same Jacobi diagonal passed as a caller's
    diagonal, which does not assume symmetry) follows the same trajectory:
    after 16 iterations the iterates and the residual histories agree to
    rounding, for an odd (m = 11: L = 45) and an even (m = 15: L = 64)
    embedding and three systems; the Hermitian iterate is exactly
    Hermitian (x[M-1-j] = conj x[j], the centre real)."""
    d, N = 2, 4000
    x, y0 = _inputs(d, N, 63)
    y = torch.stack([y0, -0.5 * y0 + 0.2, torch.cos(7.0 * x[0]) * y0]).to(prec)
    s2 = [1.0, 0.03, 0.001]
    kw = dict(kernel="matern", nu=1.5, lengthscale=0.1, eps=1e-4, m=m)
    if prec == torch.float64:
        kw["nufft_tol"] = 1e-12
    plan = C.efgp_setup(x.to(prec).cuda(), y.cuda(), s2, **kw)
    # 16 steps: before CG's loss of orthogonality lets two rounding
    # sequences drift apart (at 48 steps a system with sigma^2 = 0.03 differs
    # by 5e-7 in double precision; the residuals the oracle computes for
    # solutions of this path are checked elsewhere)
    nit = 16
    run = dict(rel_tol=1e-30, max_iter=nit, iters_per_sync=16, record_history=True, raise_on_error=False)
    bh, sth, ssh = C.efgp_solve(plan, precond=C.PRECOND_JACOBI, **run)
    hh = np.array(ssh["history"])
    D = C.efgp_get_weights(plan).double()
    diag = torch.stack([1.0 / (N * D ** 2 + v) for v in s2]).to(prec).cuda()
    bg, stg, ssg = C.efgp_solve(plan, precond=C.PRECOND_DIAG, precond_diag=diag, **run)
    hg = np.array(ssg["history"])
    assert ssh["iterations"] == ssg["iterations"] == nit
    # a wrong operator would differ at O(1)
    tol = 1e-8 if prec == torch.float64 else 2e-3
    np.testing.assert_allclose(hh, hg, rtol=tol)
    bh, bg = bh.cpu().numpy(), bg.cpu().numpy()
    for r in range(3):
        e = rel(bh[r], bg[r])
        print(f"[herm] prec {prec} m {m} system {r}: rel {e:.2e}, residual {hh[-1]:.2e}", flush=True)
        assert e <= tol, (r, e)
        assert np.array_equal(bh[r][::-1], np.conj(bh[r]))


def test_cg_trajectory_matches_dense_cg(fp64_case):
    """CG is deterministic given A, b and beta_0 = 0: the first residuals of
    the GPU iteration equal those of the oracle's CG on its own operator."""
    case, x, y, P, v, b, plan = fp64_case
    s2 = case[7]
    _, _, stats = C.efgp_solve(plan, rel_tol=1e-30, max_iter=8, record_history=True, iters_per_sync=1)
    apply = lambda z: O.system_apply(v, P.D, s2, z, P.m, P.dim)
    _, hist, _ = O.cg(apply, b, 0.0, 8)
    got = np.array(stats["history"][:8])
    np.testing.assert_allclose(got, np.array(hist[1:9]), rtol=1e-7)


# ------------------------------------------------------------------ FP32

@pytest.mark.parametrize("case", CASES[:3], ids=[c[0] for c in CASES[:3]])
def test_fp32_posterior_mean(case):
    name, d, kern, ell, nu, eps, N, s2, seed = case
    print(f"[parity fp32] {name}", flush=True)
    x, y = _inputs(d, N, seed)
    x32, y32 = x.float(), y.float()
    xn, yn = x32.double().numpy(), y32.double().numpy()   # exact promotion
    P, v, b = _oracle_setup(case, xn, yn)
    plan = C.efgp_setup(x32.cuda(), y32.cuda(), s2, kernel=kern, lengthscale=ell, nu=nu or 0.0, eps=eps)
    vg = C.efgp_get_toeplitz(plan).cpu().numpy()
    assert close(vg, v, 1e-4, "fp32 v")
    bg = C.efgp_get_rhs(plan).cpu().numpy()[0]
    assert close(bg, b, 1e-4, "fp32 b")
    beta, st, stats = C.efgp_solve(plan, rel_tol=1e-6, max_iter=50000)
    assert st in (C.EFGP_OK, C.EFGP_NOT_CONVERGED)
    t = synth.uniform_points(600, d, 97)
    mu = C.efgp_eval(plan, beta, t.float().cuda()).cpu().double().numpy()[0]
    exact = _oracle_exact(v, P, s2, b)
    want, _ = O.posterior_mean(exact, P.D, P.h, P.m, t.numpy())
    assert close(mu, want, 1e-4, f"fp32 mean {name}"), stats


# ------------------------------------------------------------ edge cases

def test_edge_single_point_and_boundaries():
    x = torch.tensor([[0.0, 1.0, 0.5, 1.0], [1.0, 0.0, 0.25, 1.0]], dtype=torch.float64)
    y = torch.tensor([1.0, -1.0, 0.5, 2.0], dtype=torch.float64)
    P = O.Problem(2, O.SE, 0.3, None, 1e-6)
    v, b = O.setup(P, x.numpy(), y.numpy())
    plan = C.efgp_setup(x.cuda(), y.cuda(), 0.1, kernel="se", lengthscale=0.3, eps=1e-6)
    assert rel(C.efgp_get_toeplitz(plan).cpu().numpy(), v) <= 1e-9
    assert rel(C.efgp_get_rhs(plan).cpu().numpy()[0], b) <= 1e-9
    one = C.efgp_setup(x[:, :1].contiguous().cuda(), y[:1].contiguous().cuda(), 0.1, kernel="se",
                       lengthscale=0.3, eps=1e-6)
    v1 = C.efgp_get_toeplitz(one).cpu().numpy()
    np.testing.assert_allclose(np.abs(v1), 1.0, atol=1e-9)


def test_edge_domain_errors():
    x = torch.tensor([[0.2, 1.5, 0.3]], dtype=torch.float64).cuda()
    y = torch.zeros(3, dtype=torch.float64).cuda()
    with pytest.raises(C.EfgpError) as e:
        C.efgp_setup(x, y, 0.1, kernel="se", lengthscale=0.2, eps=1e-4)
    assert e.value.status == C.EFGP_EDOMAIN
    xn = torch.tensor([[0.2, float("nan"), 0.3]], dtype=torch.float32).cuda()
    with pytest.raises(C.EfgpError) as e:
        C.efgp_setup(xn, y.float(), 0.1, kernel="se", lengthscale=0.2, eps=1e-4)
    assert e.value.status == C.EFGP_EDOMAIN
    good = C.efgp_setup(torch.tensor([[0.2, 0.4]], dtype=torch.float64).cuda(),
                        torch.ones(2, dtype=torch.float64).cuda(), 0.1, kernel="se",
                        lengthscale=0.2, eps=1e-4)
    beta, st, _ = C.efgp_solve(good)
    C.efgp_eval(good, beta, torch.tensor([[0.5, -0.1]], dtype=torch.float64).cuda())
    assert C.efgp_eval_status(good) == C.EFGP_EDOMAIN
    assert C.efgp_eval_status(good) == C.EFGP_OK  # the flag is cleared once read


def test_max_iter_reports_not_converged():
    x, y = _inputs(2, 500, 5)
    plan = C.efgp_setup(x.cuda(), y.cuda(), 0.01, kernel="matern", nu=1.5, lengthscale=0.1, eps=1e-4)
    beta, st, stats = C.efgp_solve(plan, rel_tol=1e-12, max_iter=1, iters_per_sync=1)
    assert st == C.EFGP_NOT_CONVERGED
    assert torch.isfinite(torch.view_as_real(beta)).all()


def test_binding_rejects_wrong_sizes():
    """The library reads and writes as many elements as the plan says; the
    binding refuses a tensor of another size (or targets of another
    dimension) before calling it."""
    x, y = _inputs(2, 500, 5)
    plan = C.efgp_setup(x.cuda(), y.cuda(), 0.01, kernel="matern", nu=1.5, lengthscale=0.1, eps=1e-4)
    beta, _, _ = C.efgp_solve(plan, rel_tol=1e-6, max_iter=500)
    short = beta[:, :-1].contiguous()
    t = synth.uniform_points(10, 2, 6).cuda()
    bad = [lambda: C.efgp_eval(plan, short, t),
           lambda: C.efgp_eval(plan, beta, t[:1].contiguous()),
           lambda: C.efgp_eval(plan, beta, t, mu_out=torch.empty(9, dtype=torch.float64, device="cuda")),
           lambda: C.efgp_apply(plan, short),
           lambda: C.efgp_apply(plan, beta, out=short),
           lambda: C.efgp_solve(plan, beta_out=short),
           lambda: C.efgp_solve(plan, beta_init=short),
           lambda: C.efgp_mean_at_points(plan, short, x.cuda()),
           lambda: C.efgp_variance(plan, t, var_out=torch.empty(11, dtype=torch.float64, device="cuda")),
           lambda: C.efgp_mlp_forward(torch.zeros(C.MLP_NPARAM - 1, device="cuda"),
                                      torch.zeros(4, C.NFEAT, device="cuda")),
           lambda: C.efgp_mlp_forward(torch.zeros(C.MLP_NPARAM, device="cuda"), torch.zeros(4, 3, device="cuda"))]
    for f in bad:
        with pytest.raises(ValueError):
            f()
    pp = C.efgp_prior_setup(2, kernel="se", lengthscale=0.2, eps=1e-4, nsamp=2)
    with pytest.raises(ValueError):
        C.efgp_sample_prior(pp, torch.zeros(1, pp.M, dtype=torch.complex64, device="cuda"), t.float())


def test_nonfinite_data_rejected():
    x = torch.tensor([[0.2, 0.4, 0.6]], dtype=torch.float32).cuda()
    y = torch.tensor([1.0, float("inf"), 0.0], dtype=torch.float32).cuda()
    with pytest.raises(C.EfgpError) as e:
        C.efgp_setup(x, y, 0.1, kernel="se", lengthscale=0.2, eps=1e-4)
    assert e.value.status == C.EFGP_EINVAL


def _sampled_setup_errors(plan, P, xh, yh, count, seed):
    """Largest |v_gpu(j) - v(j)| / N and |b_gpu(j) - b(j)| / (D_j sum|y|) over
    sampled frequencies (the corners of J_2m, J_m and random ones), against
    the oracle's direct sums at those frequencies (eqs. (88), (rhs))."""
    d = P.dim
    rng = np.random.default_rng(seed)

    def pick(K):
        J = [np.zeros(d, dtype=int), np.full(d, K), -np.full(d, K)]
        J += [rng.integers(-K, K + 1, size=d) for _ in range(count)]
        J = np.array(J)
        idx = np.zeros(len(J), dtype=np.int64)
        for l in range(d):
            idx = idx * (2 * K + 1) + (J[:, l] + K)
        return J, idx

    N = xh.shape[1]
    Jv, iv = pick(2 * P.m)
    vg = C.efgp_get_toeplitz(plan).cpu().numpy()
    ev = np.abs(vg[iv] - O.type1_at(xh, None, Jv, P.h, +1)).max() / N
    Jb, ib = pick(P.m)
    bg = C.efgp_get_rhs(plan).cpu().numpy()[0]
    eb = (np.abs(bg[ib] - P.D[ib] * O.type1_at(xh, yh, Jb, P.h, +1)) / (P.D[ib] * np.abs(yh).sum())).max()
    return ev, eb, vg


@pytest.mark.parametrize("prec", [torch.float32, torch.float64])
def test_spreaders_agree(prec):
    """The sorted-tile and whole-region spreaders compute the same grid
    (FP32: both fixed-point; FP64: both double) up to rounding, and each
    matches the oracle's direct sums at sampled frequencies within the
    plan's spreading tolerance (errors relative to N for v and to
    D_j sum|y| for b, the l1 norms of the strengths).  Precision 32 runs the
    whole-region spreader with 1024-point epochs, so every workgroup
    flushes and re-zeroes its accumulator several times."""
    d, N = 2, 300_000
    x = synth.uniform_points(N, d, 21).to(prec)
    y = (synth.f_smooth5(x.double()) + synth.noise((N,), 0.09, 21)).to(prec)
    kw = dict(kernel="matern", nu=1.5, lengthscale=0.1, eps=1e-3)
    if prec == torch.float64:  # keep the double active region within LDS
        kw.update(m=8, nufft_tol=1e-6)
    a = C.efgp_setup(x.cuda(), y.cuda(), 0.09, spread_method=C.SPREAD_TILES, **kw)
    b = C.efgp_setup(x.cuda(), y.cuda(), 0.09, spread_method=C.SPREAD_GRID_LDS,
                     spread_epoch=1024 if prec == torch.float32 else 0, **kw)
    assert a.info.spread_method == C.SPREAD_TILES and b.info.spread_method == C.SPREAD_GRID_LDS
    va, vb = C.efgp_get_toeplitz(a).cpu().numpy(), C.efgp_get_toeplitz(b).cpu().numpy()
    ba, bb = C.efgp_get_rhs(a).cpu().numpy(), C.efgp_get_rhs(b).cpu().numpy()
    tol = 1e-6 if prec == torch.float32 else 1e-12
    assert rel(va, vb) <= tol
    assert rel(ba, bb) <= tol
    assert va.shape == ((4 * a.m + 1) ** 2,)
    P = O.Problem(d, O.MATERN, 0.1, 1.5, 1e-3, m=kw.get("m", 0) or None)
    assert P.m == a.m
    xh, yh = x.double().numpy(), y.double().numpy()
    ntol = a.info.nufft_tol
    for plan in (a, b):
        ev, eb, vg = _sampled_setup_errors(plan, P, xh, yh, 12, 22)
        print(f"[spreaders] {prec} method {plan.info.spread_method}: v err/N {ev:.2e}, b err {eb:.2e}, "
              f"v0 - N {vg[(vg.size - 1) // 2].real - N:.3e}")
        assert ev <= ntol and eb <= ntol, (ev, eb, ntol)
        # v_0 = N up to the kernel's periodic-sum deviation averaged over the
        # points (~ tol / sqrt(N)) and, in precision 32, rounding
        v0_tol = 10 * ntol / math.sqrt(N) + (2e-7 if prec == torch.float32 else 1e-12)
        assert abs(vg[(vg.size - 1) // 2] - N) <= v0_tol * N


@pytest.mark.parametrize("method", ["tiles", "grid", "regions"])
def test_fixed_point_overflow_repeats_with_the_safe_scale(method):
    """Precision 32 sets the unit channel's fixed-point scale from the
    expected load of a cell.  2^20 points at one location overload their
    cells: the spreader detects the overflow (a unit-channel word that wraps
    or turns negative against the exact mass of the points) and the setup
    repeats with the worst-case scale.  The result is exact: every point
    has the same phase, so v_j = N exp(2 pi i h <j, x0>) and b_j = D_j
    exp(2 pi i h <j, x0>) sum y."""
    d, N = 2, 1 << 20
    x0 = np.array([0.3, 0.7])
    x = torch.tensor(x0, dtype=torch.float32)[:, None].repeat(1, N).contiguous()
    y = (0.5 + 0.1 * torch.randn(N, generator=torch.Generator().manual_seed(5), dtype=torch.float64)).float()
    sm = {"tiles": C.SPREAD_TILES, "grid": C.SPREAD_GRID_LDS, "regions": C.SPREAD_REGIONS}[method]
    plan = C.efgp_setup(x.cuda(), y.cuda(), 0.09, kernel="matern", nu=1.5, lengthscale=0.1, eps=1e-3,
                        spread_method=sm, tile=40 if method == "regions" else 0)
    assert plan.info.spread_method == sm
    assert plan.info.setup_passes >= 2
    P = O.Problem(d, O.MATERN, 0.1, 1.5, 1e-3)
    xs = x[:, 0].double().numpy()
    J2 = O.freq_grid(2 * P.m, d)
    v = N * np.exp(2j * np.pi * P.h * (J2 @ xs))
    vg = C.efgp_get_toeplitz(plan).cpu().numpy()
    tol = plan.info.nufft_tol
    assert rel(vg, v) <= tol
    J1 = O.freq_grid(P.m, d)
    b = P.D * np.exp(2j * np.pi * P.h * (J1 @ xs)) * float(y.double().sum())
    assert rel(C.efgp_get_rhs(plan).cpu().numpy()[0], b) <= tol


def test_fp32_setup_matches_fp64_setup():
    """Fixed-point resolution of the precision-32 setup at full epochs
    (2^18 points per workgroup and epoch, N = 2^26 + 12345): with the
    load-based scale, v and b of the FP32 whole-region spreader match the
    FP64 setup at the same spreading tolerance to 1e-5 (relative l2), and
    v_0 = N to 1e-6 (the worst-case scale of such epochs, a quantum of
    2^-12, rounded the small stencil weights away and biased v_0 by
    -2.3e-5 N and b by -1.6e-4)."""
    d, N = 2, (1 << 26) + 12345
    x = synth.uniform_points(N, d, 23, dtype=torch.float32, device="cuda")
    y = (synth.f_smooth5(x.double()) + synth.noise((N,), 0.09, 23, device="cuda")).float()
    kw = dict(kernel="matern", nu=1.5, lengthscale=0.1, eps=1e-3)
    p32 = C.efgp_setup(x, y, 0.09, spread_method=C.SPREAD_GRID_LDS, **kw)
    p64 = C.efgp_setup(x.double(), y.double(), 0.09, nufft_tol=p32.info.nufft_tol, **kw)
    assert p32.info.setup_passes == 1 and p32.info.w == p64.info.w
    v32, v64 = C.efgp_get_toeplitz(p32).cpu().numpy(), C.efgp_get_toeplitz(p64).cpu().numpy()
    b32, b64 = C.efgp_get_rhs(p32).cpu().numpy()[0], C.efgp_get_rhs(p64).cpu().numpy()[0]
    c = (v32.size - 1) // 2
    print(f"[fp32 setup] v rel {rel(v32, v64):.2e}, b rel {rel(b32, b64):.2e}, v0-N {v32[c].real - N:.2f}")
    assert abs(v32[c] - N) <= 1e-6 * N
    assert rel(v32, v64) <= 1e-5
    assert rel(b32, b64) <= 1e-5


@pytest.mark.parametrize("d,kw", [
    (1, dict(kernel="matern", nu=1.5, lengthscale=0.05, eps=1e-3)),
    (3, dict(kernel="se", lengthscale=0.5, eps=1e-3)),
])
def test_spreaders_agree_fp32_1d_3d(d, kw):
    """Precision 32 whole-region spreader in 1D and 3D (both channels packed
    into one 64-bit LDS add per cell) against the tile spreader and against
    the oracle's direct sums."""
    N = 200_000 if d == 1 else 40_000
    x = synth.uniform_points(N, d, 31 + d)
    y = torch.cos(2 * math.pi * 3.0 * x.double().sum(0)) + synth.noise((N,), 0.09, 31 + d) - 0.3
    a = C.efgp_setup(x.float().cuda(), y.float().cuda(), 0.09, spread_method=C.SPREAD_TILES, **kw)
    b = C.efgp_setup(x.float().cuda(), y.float().cuda(), 0.09, spread_method=C.SPREAD_GRID_LDS, **kw)
    assert b.info.spread_method == C.SPREAD_GRID_LDS
    va, vb = C.efgp_get_toeplitz(a).cpu().numpy(), C.efgp_get_toeplitz(b).cpu().numpy()
    ba, bb = C.efgp_get_rhs(a).cpu().numpy()[0], C.efgp_get_rhs(b).cpu().numpy()[0]
    assert rel(va, vb) <= 1e-6 and rel(ba, bb) <= 1e-6
    P = O.Problem(d, O.MATERN if kw["kernel"] == "matern" else O.SE, kw["lengthscale"], kw.get("nu"), kw["eps"])
    assert P.m == b.m
    xh = x.float().double().numpy()
    yh = y.float().double().numpy()
    v = O.toeplitz_vector(xh, P.h, P.m)
    rhs = O.rhs(xh, yh, P.h, P.m, P.D)
    assert rel(vb, v) <= 1e-4
    assert rel(bb, rhs) <= 1e-4


@pytest.mark.parametrize("d,nrhs,N", [(2, 64, 30_011), (2, 17, 20_003), (1, 16, 50_001), (1, 64, 9_999),
                                      (2, 16, 37), (1, 33, 5)])
def test_channel_parallel_spreader(d, nrhs, N):
    """Precision 32 with 16 or more data vectors in 1D/2D spreads with one
    lane per data vector (data point-major, sorted by a permutation).  Every
    vector's b equals that vector's own setup (the one-vector spreader) to
    fixed-point rounding; v and a few vectors' b match the oracle's direct
    sums (eqs. (88), (rhs)).  Ragged N, odd and maximal vector counts, and
    vectors of different magnitudes and signs (one scale per vector)."""
    x = synth.uniform_points(N, d, 51 + d)
    g = torch.Generator().manual_seed(52 + nrhs)
    base = torch.cos(2 * math.pi * 3.0 * x.sum(0))
    amp = torch.logspace(-2, 2, nrhs, dtype=torch.float64)[:, None]
    y = amp * (base[None, :] + 0.3 * torch.randn(nrhs, N, generator=g, dtype=torch.float64))
    y[3] -= 5.0 * amp[3]          # one vector of nearly constant sign
    ell = 0.1 if d == 2 else 0.05
    kw = dict(kernel="matern", nu=1.5, lengthscale=ell, eps=1e-3, spread_method=C.SPREAD_TILES)
    xf, yf = x.float().cuda(), y.float().cuda()
    plan = C.efgp_setup(xf, yf, [0.09] * nrhs, **kw)
    assert plan.info.spread_method == C.SPREAD_TILES
    P = O.Problem(d, O.MATERN, ell, 1.5, 1e-3)
    assert P.m == plan.m
    bg = C.efgp_get_rhs(plan).cpu().numpy()
    vg = C.efgp_get_toeplitz(plan).cpu().numpy()
    for r in range(nrhs):
        one = C.efgp_setup(xf, yf[r:r + 1].contiguous(), 0.09, **kw)
        assert rel(bg[r], C.efgp_get_rhs(one).cpu().numpy()[0]) <= 1e-5, r
        assert rel(vg, C.efgp_get_toeplitz(one).cpu().numpy()) <= 1e-6, r
    xh = x.float().double().numpy()
    assert rel(vg, O.toeplitz_vector(xh, P.h, P.m)) <= 1e-4
    for r in (0, 3, nrhs // 2, nrhs - 1):
        rhs = O.rhs(xh, y[r].float().double().numpy(), P.h, P.m, P.D)
        assert rel(bg[r], rhs) <= 1e-4, r


@pytest.mark.parametrize("prec", [torch.float32, torch.float64])
@pytest.mark.parametrize("badval", [1.5, -0.25, float("nan"), float("inf")])
def test_grid_spreader_domain_errors(prec, badval):
    """The whole-region spreader rejects a point outside [0,1]^2 (or a
    non-finite one) anywhere in a large input with EDOMAIN, and the plan
    cache keeps working afterwards."""
    N = 100_000
    x = synth.uniform_points(N, 2, 41).to(prec)
    x[1, 77_777] = badval
    y = torch.ones(N, dtype=prec)
    kw = dict(kernel="matern", nu=1.5, lengthscale=0.1, eps=1e-3, spread_method=C.SPREAD_GRID_LDS)
    if prec == torch.float64:
        kw.update(m=8, nufft_tol=1e-6)
    with pytest.raises(C.EfgpError) as e:
        C.efgp_setup(x.cuda(), y.cuda(), 0.09, **kw)
    assert e.value.status == C.EFGP_EDOMAIN
    x[1, 77_777] = 0.5
    ok = C.efgp_setup(x.cuda(), y.cuda(), 0.09, **kw)
    assert ok.info.spread_method == C.SPREAD_GRID_LDS


@pytest.mark.parametrize("badval", [float("nan"), float("inf"), -float("inf")])
@pytest.mark.parametrize("n,where", [(300_000, 5), (300_000, 299_999),
                                     # 256 blocks of two 2^18-point epochs: a bad
                                     # value in a block's second epoch, and the last point
                                     (67_121_209, 1_052_148), (67_121_209, 67_121_208)])
def test_grid_spreader_rejects_nonfinite_data(badval, n, where):
    """A non-finite datum anywhere in a large precision-32 input on the grid
    spreader (first, middle or last block epoch) is rejected with EINVAL
    before any spreading."""
    g = torch.Generator(device="cuda").manual_seed(43)
    x = torch.rand((2, n), generator=g, device="cuda", dtype=torch.float32)
    y = torch.ones(n, dtype=torch.float32, device="cuda")
    y[where] = badval
    with pytest.raises(C.EfgpError) as e:
        C.efgp_setup(x, y, 0.09, kernel="matern", nu=1.5, lengthscale=0.1, eps=1e-3,
                     spread_method=C.SPREAD_GRID_LDS)
    assert e.value.status == C.EFGP_EINVAL


@pytest.mark.parametrize("d,N,kw,tile", [
    (2, 100_000, dict(kernel="matern", nu=1.5, lengthscale=0.1, eps=1e-4), 16),
    (2, 60_001, dict(kernel="matern", nu=1.5, lengthscale=0.1, eps=1e-3), 0),
    (1, 200_003, dict(kernel="matern", nu=1.5, lengthscale=0.05, eps=1e-3), 48),
    (3, 40_000, dict(kernel="se", lengthscale=0.5, eps=1e-3), 6),
])
def test_region_spreader_matches_oracle(d, N, kw, tile):
    """The region spreader (points partitioned by grid region, each region's
    window accumulated in LDS in packed fixed point, the slots gathered per
    grid cell) against the oracle's direct sums of eqs. (88) and (rhs) and
    against the tiled spreader.  Small region edges give many regions, so
    most stencils straddle a region boundary and every cell near one sums
    two to four windows; a ragged N leaves short last runs."""
    x = synth.uniform_points(N, d, 81 + d)
    y = torch.cos(2 * math.pi * 3.0 * x.double().sum(0)) + synth.noise((N,), 0.09, 81 + d) - 0.3
    xf, yf = x.float(), y.float()
    a = C.efgp_setup(xf.cuda(), yf.cuda(), 0.09, spread_method=C.SPREAD_REGIONS, tile=tile, **kw)
    t = C.efgp_setup(xf.cuda(), yf.cuda(), 0.09, spread_method=C.SPREAD_TILES, **kw)
    assert a.info.spread_method == C.SPREAD_REGIONS and a.info.setup_passes == 1
    if tile:
        assert a.info.tile <= tile
    va, vt = C.efgp_get_toeplitz(a).cpu().numpy(), C.efgp_get_toeplitz(t).cpu().numpy()
    ba, bt = C.efgp_get_rhs(a).cpu().numpy()[0], C.efgp_get_rhs(t).cpu().numpy()[0]
    assert close(va, vt, 1e-6, "regions vs tiles v") and close(ba, bt, 1e-6, "regions vs tiles b")
    P = O.Problem(d, O.MATERN if kw["kernel"] == "matern" else O.SE, kw["lengthscale"], kw.get("nu"), kw["eps"])
    assert P.m == a.m
    xh, yh = xf.double().numpy(), yf.double().numpy()
    ntol = a.info.nufft_tol
    if P.M <= 5000:
        assert close(va, O.toeplitz_vector(xh, P.h, P.m), 1e-4, "regions v")
        assert close(ba, O.rhs(xh, yh, P.h, P.m, P.D), 1e-4, "regions b")
    ev, eb, vg = _sampled_setup_errors(a, P, xh, yh, 12, 83)
    print(f"[regions] d={d} R={a.info.tile}: v err/N {ev:.2e}, b err {eb:.2e} (tol {ntol:.0e})")
    assert ev <= ntol and eb <= ntol, (ev, eb, ntol)


def test_region_spreader_auto_and_deterministic():
    """Where the active region exceeds LDS (2D, eps = 1e-4: about 200^2
    cells) and there are several points per stencil origin, the automatic
    choice is the region spreader.  Its result is the same bit for bit on a
    repeated setup (the order of points within a region differs between
    runs, the fixed-point sums do not), v_0 = N to fixed-point rounding, and
    sampled entries match the oracle's direct sums."""
    d, N = 2, 1_000_003
    x = synth.uniform_points(N, d, 91, dtype=torch.float32, device="cuda")
    y = (synth.f_smooth5(x.double()) + synth.noise((N,), 0.09, 91, device="cuda")).float()
    kw = dict(kernel="matern", nu=1.5, lengthscale=0.1, eps=1e-4)
    a = C.efgp_setup(x, y, 0.09, **kw)
    assert a.info.spread_method == C.SPREAD_REGIONS
    b = C.efgp_setup(x, y, 0.09, **kw)
    va, vb = C.efgp_get_toeplitz(a), C.efgp_get_toeplitz(b)
    assert torch.equal(va, vb)
    assert torch.equal(C.efgp_get_rhs(a), C.efgp_get_rhs(b))
    va = va.cpu().numpy()
    c = (va.size - 1) // 2
    assert abs(va[c] - N) <= 1e-6 * N
    P = O.Problem(d, O.MATERN, 0.1, 1.5, 1e-4)
    ev, eb, _ = _sampled_setup_errors(a, P, x.double().cpu().numpy(), y.double().cpu().numpy(), 8, 92)
    assert ev <= a.info.nufft_tol and eb <= a.info.nufft_tol, (ev, eb)


@pytest.mark.parametrize("N", [1, 2, 37, 4097])
def test_region_spreader_small_inputs(N):
    """A handful of points on the region spreader (most regions empty, one
    short run): v and b equal the oracle's direct sums."""
    d = 2
    x = synth.uniform_points(N, d, 95)
    x[:, 0] = torch.tensor([0.0, 1.0])      # a corner of the domain
    y = torch.cos(7.0 * x[0]) - 0.5 * x[1]
    kw = dict(kernel="matern", nu=1.5, lengthscale=0.1, eps=1e-3)
    a = C.efgp_setup(x.float().cuda(), y.float().cuda(), 0.09, spread_method=C.SPREAD_REGIONS, tile=20, **kw)
    assert a.info.spread_method == C.SPREAD_REGIONS
    P = O.Problem(d, O.MATERN, 0.1, 1.5, 1e-3)
    xh, yh = x.float().double().numpy(), y.float().double().numpy()
    v = O.toeplitz_vector(xh, P.h, P.m)
    tol = 10 * a.info.nufft_tol
    assert np.abs(C.efgp_get_toeplitz(a).cpu().numpy() - v).max() <= tol * N
    rhs = O.rhs(xh, yh, P.h, P.m, P.D)
    assert np.abs(C.efgp_get_rhs(a).cpu().numpy()[0] - rhs).max() <= tol * np.abs(yh).sum() * P.D.max()


@pytest.mark.parametrize("badval", [1.5, -0.25, float("nan")])
def test_region_spreader_domain_errors(badval):
    """A point outside [0,1]^2 on the region spreader is EDOMAIN; the same
    input with the point moved inside then sets up."""
    N = 200_000
    x = synth.uniform_points(N, 2, 97).float()
    x[0, 123_456] = badval
    y = torch.ones(N, dtype=torch.float32)
    kw = dict(kernel="matern", nu=1.5, lengthscale=0.1, eps=1e-4, spread_method=C.SPREAD_REGIONS)
    with pytest.raises(C.EfgpError) as e:
        C.efgp_setup(x.cuda(), y.cuda(), 0.09, **kw)
    assert e.value.status == C.EFGP_EDOMAIN
    x[0, 123_456] = 0.5
    assert C.efgp_setup(x.cuda(), y.cuda(), 0.09, **kw).info.spread_method == C.SPREAD_REGIONS


def test_region_spreader_refusals():
    """The region spreader takes precision 32 with one data vector (else
    EINVAL) and a region edge whose window fits in LDS (else ETOOLARGE)."""
    N = 1000
    x = synth.uniform_points(N, 2, 99)
    y = torch.ones(N, dtype=torch.float64)
    kw = dict(kernel="matern", nu=1.5, lengthscale=0.1, eps=1e-3, spread_method=C.SPREAD_REGIONS)
    with pytest.raises(C.EfgpError) as e:
        C.efgp_setup(x.cuda(), y.cuda(), 0.09, **kw)
    assert e.value.status == C.EFGP_EINVAL
    with pytest.raises(C.EfgpError) as e:
        C.efgp_setup(x.float().cuda(), y.float().repeat(2, 1).cuda(), [0.09, 0.09], **kw)
    assert e.value.status == C.EFGP_EINVAL
    with pytest.raises(C.EfgpError) as e:
        C.efgp_setup(x.float().cuda(), y.float().cuda(), 0.09, tile=1000, **kw)
    assert e.value.status == C.EFGP_ETOOLARGE


def test_fp32_refined_solve_reaches_fp64_accuracy():
    """Precision 32 with iterative refinement (residuals b - A beta formed in
    double, corrections by single-precision Jacobi PCG): the solve reaches a
    double residual of 1e-10, where plain single-precision CG stops near
    1e-6, and its posterior mean matches the FP64 path's at the same
    spreading tolerance and residual to 2e-5 (what remains is the FP32
    spreading's rounding)."""
    d, N = 2, 2_000_000
    x = synth.uniform_points(N, d, 24, dtype=torch.float32, device="cuda")
    y = (synth.f_smooth5(x.double()) + synth.noise((N,), 0.09, 24, device="cuda")).float()
    kw = dict(kernel="matern", nu=1.5, lengthscale=0.1, eps=1e-3)
    p32 = C.efgp_setup(x, y, 0.09, **kw)
    p64 = C.efgp_setup(x.double(), y.double(), 0.09, nufft_tol=p32.info.nufft_tol, **kw)
    b32, s32, ss32 = C.efgp_solve(p32, rel_tol=1e-10, max_iter=200000, precond=C.PRECOND_JACOBI, refine=16)
    b64, s64, ss64 = C.efgp_solve(p64, rel_tol=1e-10, max_iter=200000, precond=C.PRECOND_JACOBI,
                                  stall_window=1000000)
    print(f"[refine] {ss32['refine_steps']} steps, {ss32['iterations']} inner iterations, residual "
          f"{ss32['rel_residual']:.2e}; FP64 {ss64['iterations']} iterations")
    assert s32 in (C.EFGP_OK, C.EFGP_FELL_BACK) and ss32["rel_residual"] <= 1.1e-10
    assert ss32["refine_steps"] >= 2
    assert s64 == C.EFGP_OK
    t = synth.uniform_points(20000, d, 25, dtype=torch.float32, device="cuda")
    m32 = C.efgp_eval(p32, b32, t)[0].double()
    m64 = C.efgp_eval(p64, b64, t.double())[0]
    e2 = float(torch.linalg.norm(m32 - m64) / torch.linalg.norm(m64))
    print(f"[refine] mean rel l2 {e2:.2e}, rel linf {float((m32 - m64).abs().max() / m64.abs().max()):.2e}")
    assert e2 <= 2e-5
    # refinement is opt-in: the same plan without it is plain single-precision CG
    _, _, plain = C.efgp_solve(p32, rel_tol=1e-5, precond=C.PRECOND_JACOBI)
    assert plain["refine_steps"] == 0
