"""Spread autotuner: the measured fastest spreader is stored per problem
shape and used by later automatic setups of that shape; the tuned setup gives
the same Toeplitz vector and right-hand side as an explicit setup with the
chosen spreader, bit for bit (both accumulate in fixed point)."""
import os

import pytest
import torch

import synth

pytestmark = pytest.mark.gpu
C = pytest.importorskip("paper_2210_10210_amd.capi")


def _data(n, d, seed):
    x = synth.uniform_points(n, d, seed, dtype=torch.float32, device="cuda")
    y = (synth.f_plane_wave(x, [3.0, 2.0, 1.0][:d]) +
         synth.noise((n,), 0.05, seed, dtype=torch.float32, device="cuda")).contiguous()
    return x, y


@pytest.mark.parametrize("d,n,kw", [(2, 4_000_000, dict(kernel="matern", nu=1.5, lengthscale=0.1, eps=1e-3)),
                                    (3, 2_000_000, dict(kernel="se", lengthscale=0.2, eps=1e-4))])
def test_tuned_spreader_is_used_and_matches_explicit(d, n, kw, tmp_path):
    print(f"[tune] d={d} n={n}", flush=True)
    C.efgp_tune_clear()
    x, y = _data(n, d, 50 + d)
    res = C.efgp_tune_spread(x, y, 0.05, **kw)
    print(f"[tune] chose method {res['spread_method']} tile {res['tile']}: {res['ms_setup']:.2f} ms "
          f"of {res['candidates']} candidates", flush=True)
    assert res["spread_method"] in (C.SPREAD_TILES, C.SPREAD_GRID_LDS, C.SPREAD_REGIONS)
    assert res["candidates"] >= 3 and res["ms_setup"] > 0
    if res["spread_method"] in (C.SPREAD_TILES, C.SPREAD_REGIONS):
        assert res["tile"] > 0
    auto = C.efgp_setup(x, y, 0.05, **kw)
    assert auto.info.spread_method == res["spread_method"]
    if res["spread_method"] in (C.SPREAD_TILES, C.SPREAD_REGIONS):
        assert auto.info.tile == res["tile"]
    expl = C.efgp_setup(x, y, 0.05, spread_method=res["spread_method"], tile=res["tile"], **kw)
    assert torch.equal(C.efgp_get_toeplitz(auto), C.efgp_get_toeplitz(expl))
    assert torch.equal(C.efgp_get_rhs(auto), C.efgp_get_rhs(expl))
    # the table survives a save / clear / load cycle
    path = os.path.join(str(tmp_path), "tune.txt")
    C.efgp_tune_save(path)
    C.efgp_tune_clear()
    assert C.efgp_tune_load(path) == 1
    again = C.efgp_setup(x, y, 0.05, **kw)
    assert again.info.spread_method == res["spread_method"]
    # another size class (floor(log2 N) differs) is not covered by the entry
    half = n // 3
    other = C.efgp_setup(x[:, :half].contiguous(), y[:half].contiguous(), 0.05, **kw)
    assert other.info.spread_method in (C.SPREAD_TILES, C.SPREAD_GRID_LDS, C.SPREAD_REGIONS)
    C.efgp_tune_clear()


def test_tune_reports_problem_errors():
    x, y = _data(100_000, 2, 60)
    x[0, 5] = 1.5   # a point outside the unit square
    with pytest.raises(C.EfgpError) as e:
        C.efgp_tune_spread(x, y, 0.05, kernel="se", lengthscale=0.2, eps=1e-3)
    assert e.value.status == C.EFGP_EDOMAIN
    C.efgp_tune_clear()
