"""Plan lifetime and the process-wide caches (device buffers, pinned staging,
streams, events and captured CG graphs reused by later plans of the same
sizes).  A cached resource must never change a result: repeated plans give
bitwise identical answers, two live plans of identical sizes get distinct
buffers, and releasing the caches between plans changes nothing."""
import gc

import pytest
import torch

import synth

pytestmark = pytest.mark.gpu
C = pytest.importorskip("paper_2210_10210_amd.capi")


def _inputs(n, seed):
    x = synth.uniform_points(n, 2, seed).float().cuda()
    y = (torch.cos(6.0 * x[0].double()) * torch.sin(4.0 * x[1].double())).float()
    y = (y + 0.3 * synth.noise((n,), 1.0, seed).float().cuda()).contiguous()
    t = synth.uniform_points(5000, 2, seed + 100).float().cuda()
    return x, y, t


def _pipeline(x, y, t):
    # the grid spreader accumulates in fixed point: bitwise reproducible
    plan = C.efgp_setup(x, y, 0.09, kernel="matern", nu=1.5, lengthscale=0.1, eps=1e-3,
                        spread_method=C.SPREAD_GRID_LDS)
    beta, st, ss = C.efgp_solve(plan, rel_tol=1e-5, max_iter=20000, precond=C.PRECOND_JACOBI)
    assert st == C.EFGP_OK
    mu = C.efgp_eval(plan, beta, t)
    return plan, beta.clone(), mu.clone(), ss["iterations"]


def test_repeated_plans_are_bitwise_identical():
    x, y, t = _inputs(200_000, 3)
    ref = None
    for cycle in range(4):
        plan, beta, mu, it = _pipeline(x, y, t)
        del plan
        gc.collect()
        if ref is None:
            ref = (beta, mu, it)
        else:
            assert it == ref[2], cycle
            assert torch.equal(beta, ref[0]) and torch.equal(mu, ref[1]), cycle


def test_two_live_plans_of_equal_size_are_independent():
    x, y, t = _inputs(150_000, 5)
    x2, y2, t2 = _inputs(150_000, 6)
    pa, ba, ma, ia = _pipeline(x, y, t)
    alone_b = (ba, ma, ia)
    del pa
    gc.collect()
    # both alive at once, interleaved calls
    pa = C.efgp_setup(x, y, 0.09, kernel="matern", nu=1.5, lengthscale=0.1, eps=1e-3,
                      spread_method=C.SPREAD_GRID_LDS)
    pb = C.efgp_setup(x2, y2, 0.09, kernel="matern", nu=1.5, lengthscale=0.1, eps=1e-3,
                      spread_method=C.SPREAD_GRID_LDS)
    bb, sb, _ = C.efgp_solve(pb, rel_tol=1e-5, max_iter=20000, precond=C.PRECOND_JACOBI)
    ba2, sa, ssa = C.efgp_solve(pa, rel_tol=1e-5, max_iter=20000, precond=C.PRECOND_JACOBI)
    assert sa == C.EFGP_OK and sb == C.EFGP_OK
    assert ssa["iterations"] == alone_b[2]
    assert torch.equal(ba2, alone_b[0])
    assert torch.equal(C.efgp_eval(pa, ba2, t), alone_b[1])
    assert not torch.equal(bb, ba2)


def test_release_workspace_between_and_during_plans():
    x, y, t = _inputs(120_000, 8)
    p1, b1, m1, i1 = _pipeline(x, y, t)
    C.efgp_release_workspace()   # p1 is alive: only idle resources go
    b1b, st, ss = C.efgp_solve(p1, rel_tol=1e-5, max_iter=20000, precond=C.PRECOND_JACOBI)
    assert st == C.EFGP_OK and ss["iterations"] == i1 and torch.equal(b1b, b1)
    del p1
    gc.collect()
    C.efgp_release_workspace()
    p2, b2, m2, i2 = _pipeline(x, y, t)
    assert i2 == i1 and torch.equal(b2, b1) and torch.equal(m2, m1)


def test_different_sizes_interleaved():
    """Plans of different sizes alternate; each keeps its own graph and
    buffers from the caches."""
    outs = {}
    for rep in range(2):
        for n, seed in ((60_000, 11), (90_000, 12)):
            x, y, t = _inputs(n, seed)
            for eps in (1e-3, 1e-2):
                plan = C.efgp_setup(x, y, 0.09, kernel="matern", nu=1.5, lengthscale=0.1, eps=eps,
                                    spread_method=C.SPREAD_GRID_LDS)
                beta, st, ss = C.efgp_solve(plan, rel_tol=1e-5, max_iter=20000)
                assert st == C.EFGP_OK
                key = (n, eps)
                if rep == 0:
                    outs[key] = (beta.clone(), ss["iterations"])
                else:
                    assert ss["iterations"] == outs[key][1]
                    assert torch.equal(beta, outs[key][0])
                del plan
                gc.collect()
