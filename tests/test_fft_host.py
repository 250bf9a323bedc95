"""The LDS FFT's stage arithmetic checked on the host, without a GPU.

`fft_host_check.hip` is built for the host against the device header (the
register DFTs of radices 2-16 and the Stockham butterfly are host-callable)
and the library's stage planner (`fft_shape`, largest radices first or capped
at 5), then runs every plan of every 2,3,5-smooth length up to 1500 and a few
long lines in both directions against direct DFT sums: relative error
<= 1e-13 in double and <= 2e-6 in single precision.  A wrong twiddle, a
transposed index or a radix left out of a plan would fail it.  It also runs
udiv22, the kernels' division by a float reciprocal, against integer
division for every numerator below 2^22 and 124 divisors."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PKG = os.path.join(ROOT, "paper_2210_10210_amd")
LIB = os.path.join(PKG, "libefgp.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_fft_stage_arithmetic_matches_direct_dft(tmp_path):
    assert os.path.exists(LIB), "build the library first (python -c 'import __graft_entry__ as g; g.build()')"
    exe = str(tmp_path / "fft_host_check")
    cmd = [HIPCC, "-std=c++17", "-O2", "--offload-arch=gfx950", "--offload-host-only",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(PKG, "csrc"),
           os.path.join(HERE, "fft_host_check.hip"), "-L" + PKG, "-lefgp", "-Wl,-rpath," + PKG, "-o", exe]
    b = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert b.returncode == 0, b.stdout[-2000:]
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=300)
    print(r.stdout.strip())
    lines = r.stdout.strip().splitlines()
    assert r.returncode == 0 and lines and lines[-1].startswith("ok:"), r.stdout[-2000:]
