"""The C ABI library loads and exports every symbol the header declares, and
rejects invalid arguments before touching the GPU (runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "efgp.h")
LIB = os.path.join(ROOT, "paper_2210_10210_amd", "libefgp.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(efgp_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libefgp.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n


def test_binding_lists_the_same_symbols():
    from paper_2210_10210_amd import build  # noqa: F401  (module import only)
    src = open(os.path.join(ROOT, "paper_2210_10210_amd", "capi.py")).read()
    listed = re.search(r"SYMBOLS = \[(.*?)\]", src, re.S).group(1)
    listed = sorted(re.findall(r'"(efgp_[a-z_0-9]+)"', listed))
    assert listed == _declared()


def test_strerror_and_argument_errors_without_gpu(lib):
    import paper_2210_10210_amd.capi as C  # loads the library (no HIP call)
    assert C.efgp_strerror(0) == "ok"
    assert "outside" in C.efgp_strerror(C.EFGP_EDOMAIN)
    h = ctypes.c_void_p()
    assert C.lib.efgp_setup(None, ctypes.byref(h)) == C.EFGP_EINVAL
    s2 = (ctypes.c_double * 1)(0.1)
    base = dict(dim=2, kernel=C.KERNEL_MATERN, lengthscale=0.1, nu=1.5, variance=1.0, eps=1e-3,
                precision=32, nufft_tol=0.0, n=10, x=ctypes.c_void_p(16), nrhs=1,
                y=ctypes.c_void_p(32), sigma2=s2, stream=None, m_override=0, spread_method=0,
                tile=0, spread_epoch=0)
    bad = [dict(dim=4), dict(dim=0), dict(kernel=7), dict(lengthscale=0.0), dict(nu=0.25),
           dict(eps=0.0), dict(eps=1.5), dict(precision=16), dict(n=0), dict(nrhs=0),
           dict(x=None), dict(y=None), dict(nrhs=65), dict(variance=-1.0), dict(nufft_tol=2.0),
           dict(spread_method=9), dict(spread_method=4), dict(lengthscale=float("nan")), dict(spread_epoch=1000),
           dict(spread_epoch=512), dict(spread_epoch=1 << 25)]
    for b in bad:
        kw = dict(base)
        kw.update(b)
        pr = C.efgp_problem(**kw)
        h = ctypes.c_void_p(123)
        assert C.lib.efgp_setup(ctypes.byref(pr), ctypes.byref(h)) == C.EFGP_EINVAL, b
        assert h.value is None  # *out = NULL on error
    for v in (0.0, -1.0, float("inf")):
        s2b = (ctypes.c_double * 1)(v)
        kw = dict(base)
        kw["sigma2"] = s2b
        pr = C.efgp_problem(**kw)
        assert C.lib.efgp_setup(ctypes.byref(pr), ctypes.byref(h)) == C.EFGP_EINVAL
    # sizes beyond the limits are refused before any allocation
    kw = dict(base)
    kw.update(m_override=5000)
    pr = C.efgp_problem(**kw)
    assert C.lib.efgp_setup(ctypes.byref(pr), ctypes.byref(h)) == C.EFGP_ETOOLARGE
    assert C.lib.efgp_solve(None, None, None, None) == C.EFGP_EINVAL
    assert C.lib.efgp_eval(None, None, 0, None, None, None) == C.EFGP_EINVAL
    assert C.lib.efgp_get_info(None, None) == C.EFGP_EINVAL
    C.lib.efgp_destroy(None)  # NULL is safe


def test_spread_tuning_table_file_round_trip(lib, tmp_path):
    """The tuning table's save/load/clear are host-only: a saved table loads
    back entry for entry, a malformed or missing file is refused and changes
    nothing, and the tuner rejects an invalid problem before any GPU work."""
    import paper_2210_10210_amd.capi as C
    C.efgp_tune_clear()
    good = tmp_path / "tune.txt"
    good.write_text("efgp-spread-tune 1\n"
                    "0 2 32 1 216 5 29 2 0 9.250000\n"
                    "0 3 32 1 90 7 23 1 8 8.800000\n")
    assert C.efgp_tune_load(str(good)) == 2
    out = tmp_path / "out.txt"
    C.efgp_tune_save(str(out))
    lines = out.read_text().splitlines()
    assert lines[0] == "efgp-spread-tune 1"
    assert sorted(l.split()[:9] for l in lines[1:]) == sorted(l.split()[:9] for l in good.read_text().splitlines()[1:])
    bad = tmp_path / "bad.txt"
    bad.write_text("efgp-spread-tune 1\n0 2 32 1 216 5 29 7 0 1.0\n")   # method 7 does not exist
    with pytest.raises(C.EfgpError):
        C.efgp_tune_load(str(bad))
    (tmp_path / "hdr.txt").write_text("something else\n")
    with pytest.raises(C.EfgpError):
        C.efgp_tune_load(str(tmp_path / "hdr.txt"))
    with pytest.raises(C.EfgpError):
        C.efgp_tune_load(str(tmp_path / "missing.txt"))
    C.efgp_tune_save(str(out))
    assert len(out.read_text().splitlines()) == 3   # unchanged by the refused loads
    C.efgp_tune_clear()
    C.efgp_tune_save(str(out))
    assert out.read_text().splitlines() == ["efgp-spread-tune 1"]
    assert C.lib.efgp_tune_save(None) == C.EFGP_EINVAL
    assert C.lib.efgp_tune_load(None, None) == C.EFGP_EINVAL
    assert C.lib.efgp_tune_spread(None, None) == C.EFGP_EINVAL
    s2 = (ctypes.c_double * 1)(0.1)
    pr = C.efgp_problem(dim=4, kernel=C.KERNEL_MATERN, lengthscale=0.1, nu=1.5, variance=1.0, eps=1e-3,
                        precision=32, nufft_tol=0.0, n=10, x=ctypes.c_void_p(16), nrhs=1, y=ctypes.c_void_p(32),
                        sigma2=s2, stream=None, m_override=0, spread_method=0, tile=0, spread_epoch=0)
    res = C.efgp_tune_result()
    assert C.lib.efgp_tune_spread(ctypes.byref(pr), ctypes.byref(res)) == C.EFGP_EINVAL
