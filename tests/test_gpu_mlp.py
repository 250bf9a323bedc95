"""GPU network kernels (bf16 MFMA, float accumulation) against the FP64
oracle of the same architecture on bf16-rounded operands.

Tolerances: forward 1e-4 relative (same rounding points, different
accumulation order); gradients per tensor 2e-2 relative and cosine >= 0.999
(the GPU also rounds the back-propagated signals to bf16 as matrix-core
operands, the oracle does not); Adam 1e-6.
"""
import numpy as np
import pytest
import torch

from oracle import mlp as N

pytestmark = pytest.mark.gpu
C = pytest.importorskip("paper_2210_10210_amd.capi")


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-30))


def _params(seed):
    return N.init_params(seed).astype(np.float32)


@pytest.mark.parametrize("rows", [1, 15, 16, 1000, 70001])
def test_forward_matches_oracle(rows):
    print(f"[mlp forward] rows={rows}", flush=True)
    p = _params(3)
    rng = np.random.default_rng(rows)
    X = rng.normal(size=(rows, N.F)).astype(np.float32)
    out = C.efgp_mlp_forward(torch.from_numpy(p).cuda(), torch.from_numpy(X).cuda()).cpu().numpy()
    want, _ = N.forward(p.astype(np.float64), X.astype(np.float64), bf16=True)
    assert rel(out, want) <= 1e-4


def test_loss_and_gradient_match_oracle():
    p = _params(4)
    rng = np.random.default_rng(5)
    R = 5000
    X = rng.normal(size=(R, N.F)).astype(np.float32)
    t = rng.normal(size=R).astype(np.float32)
    w = rng.uniform(0.2, 2.0, size=R).astype(np.float32)
    loss, grad = C.efgp_mlp_loss_grad(torch.from_numpy(p).cuda(), torch.from_numpy(X).cuda(),
                                      torch.from_numpy(t).cuda(), torch.from_numpy(w).cuda())
    L, g = N.loss_grad(p.astype(np.float64), X.astype(np.float64), t.astype(np.float64),
                       w.astype(np.float64), bf16=True)
    assert float(loss.cpu()[0]) == pytest.approx(L, rel=1e-4)
    gg = grad.cpu().numpy().astype(np.float64)
    o = 0
    for name, shape in N.SIZES:
        n = int(np.prod(shape))
        a, b = gg[o:o + n], g[o:o + n]
        o += n
        assert rel(a, b) <= 2e-2, (name, rel(a, b))
        if n > 1:
            cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))
            assert cos >= 0.999, (name, cos)


def test_adam_step_matches_formula():
    rng = np.random.default_rng(6)
    p, g = rng.normal(size=N.NPARAM), rng.normal(size=N.NPARAM)
    m, v = rng.normal(size=N.NPARAM) * 0.1, rng.uniform(0, 0.1, size=N.NPARAM)
    tp, tg, tm, tv = (torch.from_numpy(a.astype(np.float32)).cuda() for a in (p, g, m, v))
    C.efgp_mlp_adam(tp, tg, tm, tv, step=7, lr=1e-3)
    p2, m2, v2 = N.adam(p.astype(np.float32).astype(np.float64), g.astype(np.float32).astype(np.float64),
                        m.astype(np.float32).astype(np.float64), v.astype(np.float32).astype(np.float64),
                        7, 1e-3)
    assert rel(tp.cpu().numpy(), p2) <= 1e-6
    assert rel(tm.cpu().numpy(), m2) <= 1e-6
    assert rel(tv.cpu().numpy(), v2) <= 1e-6


def test_training_reduces_loss():
    """A few hundred Adam steps on the GPU kernels fit a smooth target."""
    rng = np.random.default_rng(7)
    R = 4096
    X = rng.uniform(-1, 1, size=(R, N.F)).astype(np.float32)
    t = (np.sin(2 * X[:, 0]) + 0.5 * X[:, 1] * X[:, 2]).astype(np.float32)
    p = torch.from_numpy(_params(8) * 0.5).cuda()
    tX, tt = torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda()
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    first = None
    for step in range(1, 301):
        loss, grad = C.efgp_mlp_loss_grad(p, tX, tt)
        if first is None:
            first = float(loss.cpu()[0])
        C.efgp_mlp_adam(p, grad, m, v, step, lr=3e-3)
    last = float(C.efgp_mlp_loss_grad(p, tX, tt)[0].cpu()[0])
    assert last < 0.1 * first, (first, last)
