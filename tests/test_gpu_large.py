"""GPU parity at large m: FFT lines too long for two LDS buffers.

The spreading grid (n_f >= 2(4m+1)), the Toeplitz embedding (L >= 4m+1) and
the type-2 grid (n_f2 >= 2(2m+1)) reach several thousand points per line for
the small tolerances of a converged reference solution (2D Matern-3/2,
lengthscale 0.1, eps = 1e-8 gives m = 659).  Those lines are transformed in
one LDS buffer (in-register Stockham stages).  Each stage is checked here
against the oracle through the C ABI:
  - v and b (eqs. (88), (rhs)) against the direct sums, FP64, 1e-9;
  - the product of eq. (97) against the oracle's fast Toeplitz algorithm
    (Sec. 3.2, numpy FFTs at (4m+1)^d), 1e-9 in FP64 and 1e-5 in FP32;
  - the type-2 evaluation (eq. (muws)) against its direct sum, 1e-9;
  - the first CG residuals against the oracle's CG on the same operator.
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


def _inputs(d, N, seed):
    x = synth.uniform_points(N, d, seed)
    w = torch.tensor([3.0, 4.0][:d], dtype=torch.float64)
    y = synth.f_plane_wave(x, w) + synth.noise((N,), 0.09, seed)
    return x, y


def _hermitian(M, seed, dtype=torch.complex128):
    g = torch.Generator().manual_seed(seed)
    beta = torch.randn(M, dtype=torch.complex128, generator=g).numpy()
    return 0.5 * (beta + np.conj(beta[::-1]))


# d, m, N: 2D at m = 659 (eps = 1e-8 for Matern-3/2, lengthscale 0.1: L = 2700,
# n_f = 5400, n_f2 = 2700) and 1D at m = 1000 (L = 4000, n_f = 8100, the
# largest sizes the plan accepts are 4096 and 8192)
LONG = [(2, 659, 40), (1, 1000, 300)]


@pytest.fixture(scope="module", params=LONG, ids=[f"d{c[0]}_m{c[1]}" for c in LONG])
def long_case(request):
    d, m, N = request.param
    print(f"[large] d={d} m={m} N={N}", flush=True)
    x, y = _inputs(d, N, 90 + d)
    P = O.Problem(d, O.MATERN, 0.1, 1.5, 1e-8, m=m)
    v, b = O.setup(P, x.numpy(), y.numpy())
    plan = C.efgp_setup(x.cuda(), y.cuda(), 0.09, kernel="matern", nu=1.5, lengthscale=0.1, eps=1e-8, m=m,
                        nufft_tol=1e-12)
    return d, m, N, x, y, P, v, b, plan


def test_long_sizes_are_long(long_case):
    d, m, N, x, y, P, v, b, plan = long_case
    info = C.efgp_get_info(plan)
    assert info["m"] == m
    assert info["L"] > 1024 and info["nf"] > 4096 and info["nf_eval"] >= 2 * (2 * m + 1)


def test_long_setup_v_and_b(long_case):
    d, m, N, x, y, P, v, b, plan = long_case
    vg = C.efgp_get_toeplitz(plan).cpu().numpy()
    bg = C.efgp_get_rhs(plan).cpu().numpy()[0]
    assert rel(vg, v) <= 1e-9
    assert rel(bg, b) <= 1e-9
    c = (vg.size - 1) // 2
    assert abs(vg[c] - N) <= 1e-9 * N


def test_long_apply_fp64(long_case):
    d, m, N, x, y, P, v, b, plan = long_case
    beta = _hermitian(P.M, 11)
    out = C.efgp_apply(plan, torch.as_tensor(beta).reshape(1, -1).cuda()).cpu().numpy()[0]
    want = O.system_apply(v, P.D, 0.09, beta, m, d, fast=True)
    assert rel(out, want) <= 1e-9


def test_long_eval_fp64(long_case):
    d, m, N, x, y, P, v, b, plan = long_case
    beta = _hermitian(P.M, 12)
    t = synth.uniform_points(60, d, 13)
    mu = C.efgp_eval(plan, torch.as_tensor(beta).reshape(1, -1).cuda(), t.cuda()).cpu().numpy()[0]
    want, _ = O.posterior_mean(beta, P.D, P.h, m, t.numpy())
    assert rel(mu, want) <= 1e-9
    assert rel_inf(mu, want) <= 3e-9


def test_long_cg_trajectory(long_case):
    """The CG iteration (graph-captured, long-line passes, fixed-order line
    sums) reproduces the oracle's CG residuals on the same operator."""
    d, m, N, x, y, P, v, b, plan = long_case
    _, _, stats = C.efgp_solve(plan, rel_tol=1e-30, max_iter=6, record_history=True, iters_per_sync=1)
    apply = lambda z: O.system_apply(v, P.D, 0.09, z, m, d, fast=True)
    _, hist, _ = O.cg(apply, b, 0.0, 6)
    np.testing.assert_allclose(np.array(stats["history"][:6]), np.array(hist[1:7]), rtol=1e-7)


@pytest.mark.parametrize("d,m", [(2, 600), (1, 1000)])
def test_long_apply_fp32(d, m):
    """Precision 32 with L > 2048 (long float lines): the product of eq. (97)
    against the oracle's FP64 fast Toeplitz algorithm on the same rounded
    inputs, 1e-5."""
    x, y = _inputs(d, 50, 70 + d)
    xf, yf = x.float(), y.float()
    P = O.Problem(d, O.MATERN, 0.1, 1.5, 1e-8, m=m)
    v, _ = O.setup(P, xf.double().numpy(), yf.double().numpy())
    plan = C.efgp_setup(xf.cuda(), yf.cuda(), 0.09, kernel="matern", nu=1.5, lengthscale=0.1, eps=1e-8, m=m)
    assert C.efgp_get_info(plan)["L"] > 2048
    beta = _hermitian(P.M, 21).astype(np.complex64)
    out = C.efgp_apply(plan, torch.as_tensor(beta).reshape(1, -1).cuda()).cpu().numpy()[0]
    want = O.system_apply(v, P.D, 0.09, beta.astype(np.complex128), m, d, fast=True)
    assert rel(out, want) <= 1e-5


def test_limits_rejected_before_allocation():
    """Beyond the largest embedding (4m+1 > 4096) the plan is refused with
    ETOOLARGE before any work."""
    x, y = _inputs(1, 10, 5)
    with pytest.raises(C.EfgpError) as e:
        C.efgp_setup(x.cuda(), y.cuda(), 0.09, kernel="matern", nu=1.5, lengthscale=0.1, eps=1e-8, m=1024)
    assert e.value.status == C.EFGP_ETOOLARGE
