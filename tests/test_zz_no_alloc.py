"""The allocation-free Toeplitz product (efgp_apply_noalloc): its FFT
intermediates live in the library's static device scratch, and its output
equals efgp_apply's bit for bit, on two calls in a row whose second has a
smaller input (the scratch keeps the first call's contents), in precision
32 and 64, and for a 3D plan.  A plan whose buffers exceed the scratch is
refused with EFGP_ETOOLARGE."""
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu
C = pytest.importorskip("paper_2210_10210_amd.capi")


def _plan(d, n, m, nrhs, dtype, seed, kernel="matern"):
    x = synth.uniform_points(n, d, seed).to(dtype)
    y = torch.stack([synth.f_plane_wave(x.double(), (3.0, 4.0, 2.0)[:d]) + synth.noise((n,), 0.09, seed + r)
                     for r in range(nrhs)]).to(dtype)
    s2 = [0.09 * (r + 1) for r in range(nrhs)]
    return C.efgp_setup(x.cuda(), y.cuda(), s2 if nrhs > 1 else s2[0], kernel=kernel, nu=1.5, lengthscale=0.1,
                        eps=1e-4, m=m)


def _check(plan, seed):
    cdt = torch.complex64 if plan.precision == 32 else torch.complex128
    g = torch.Generator(device="cuda").manual_seed(seed)
    inp = torch.randn(plan.nrhs, plan.M, dtype=cdt, device="cuda", generator=g)
    want = C.efgp_apply(plan, inp)
    got = torch.full_like(inp, float("nan"))
    C.efgp_apply_noalloc(plan, inp, got)
    torch.cuda.synchronize()
    assert torch.equal(got, want)
    return got


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_product_equals_apply_on_two_calls(dtype):
    print(f"[noalloc] 2D {dtype}", flush=True)
    big = _plan(2, 20000, 60, 3, dtype, 41)
    small = _plan(2, 3000, 12, 1, dtype, 42)
    _check(big, 1)
    _check(small, 2)          # smaller input: the scratch still holds the first call's data
    _check(big, 3)


def test_noalloc_product_3d():
    print("[noalloc] 3D", flush=True)
    _check(_plan(3, 5000, 10, 2, torch.float32, 43, kernel="se"), 4)


def test_noalloc_refuses_plans_beyond_the_scratch():
    print("[noalloc] size limit", flush=True)
    plan = _plan(2, 200, 100, 32, torch.float64, 44)   # 2 buffers * 16 B * 201 * 405 * 32 = 83 MB > 64 MiB
    inp = torch.zeros(plan.nrhs, plan.M, dtype=torch.complex128, device="cuda")
    out = torch.zeros_like(inp)
    with pytest.raises(C.EfgpError) as e:
        C.efgp_apply_noalloc(plan, inp, out)
    assert e.value.status == C.EFGP_ETOOLARGE
