"""Seeded synthetic inputs for EFGP workloads.

This module holds input generators only (points, data, noise, targets) and
none of the method's arithmetic.  Both the oracle side (tests, CPU baseline)
and the GPU side (tests, benchmark) draw their inputs from here; each draw is
fully determined by (seed, stream, device, dtype), so the same arrays can be
handed to both sides.

Workload recipes follow the paper's synthetic experiments (Sec. 5:
iid-uniform points on [0,1]^d, y = f(x) + N(0, sigma^2), targets on the grid
{0, 1/n_t, ..., (n_t-1)/n_t}^d), with the sizes and kernels of the workloads
this project measures.
"""
import math
from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np
import torch

# stream ids mixed into the seed
POINTS, NOISE, TARGETS, CENTERS, FIELD = 0, 1, 2, 3, 4


def _gen(seed: int, stream: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed((int(seed) * 1_000_003 + int(stream) * 7919) & 0x7FFF_FFFF_FFFF_FFFF)
    return g


def uniform_points(n: int, d: int, seed: int, dtype=torch.float64, device="cpu") -> torch.Tensor:
    """(d, n) iid uniform points on [0,1)^d (structure of arrays)."""
    g = _gen(seed, POINTS, device)
    return torch.rand((d, n), generator=g, dtype=dtype, device=device)


def mixture_points(n: int, d: int, seed: int, ncomp: int = 20, std: float = 0.05,
                   lo: float = 0.15, hi: float = 0.85, dtype=torch.float64,
                   device="cpu") -> torch.Tensor:
    """(d, n) points from an equal-weight isotropic Gaussian mixture with
    ncomp centers iid uniform on [lo, hi]^d, clamped to [0,1]^d."""
    gc = _gen(seed, CENTERS, "cpu")
    centers = lo + (hi - lo) * torch.rand((d, ncomp), generator=gc, dtype=torch.float64)
    g = _gen(seed, POINTS, device)
    comp = torch.randint(0, ncomp, (n,), generator=g, device=device)
    x = centers.to(device=device, dtype=dtype)[:, comp]
    x = x + std * torch.randn((d, n), generator=g, dtype=dtype, device=device)
    return x.clamp_(0.0, 1.0)


def grid_targets(nt: int, d: int, dtype=torch.float64, device="cpu") -> torch.Tensor:
    """(d, nt^d) tensor-product grid {0, 1/nt, ..., (nt-1)/nt}^d, C order."""
    ax = torch.arange(nt, dtype=torch.float64) / nt
    g = torch.meshgrid(*([ax] * d), indexing="ij")
    return torch.stack([t.reshape(-1) for t in g]).to(device=device, dtype=dtype)


def noise(shape, sigma2: float, seed: int, dtype=torch.float64, device="cpu") -> torch.Tensor:
    g = _gen(seed, NOISE, device)
    return math.sqrt(sigma2) * torch.randn(shape, generator=g, dtype=dtype, device=device)


# -- test functions f(x) ----------------------------------------------------

def f_plane_wave(x: torch.Tensor, omega, phase: float = 1.3) -> torch.Tensor:
    """cos(2 pi <x, omega> + phase) (the paper's eq. (fdef))."""
    w = torch.as_tensor(omega, dtype=x.dtype, device=x.device).reshape(-1, 1)
    return torch.cos(2.0 * math.pi * (w * x).sum(0) + phase)


def f_sin1d(x):
    return torch.sin(6.0 * math.pi * x[0])


def f_cos2d(x):
    return torch.cos(2.0 * math.pi * (3.0 * x[0] + 2.0 * x[1]))


def f_sinprod(x):
    return torch.prod(torch.sin(4.0 * math.pi * x), dim=0)


def f_smooth5(x):
    return f_plane_wave(x, (3.0, 4.0), 1.3)


def rff_gp_samples(x: torch.Tensor, nrhs: int, ell: float, nu: float, seed0: int,
                   nfeat: int = 64) -> torch.Tensor:
    """(nrhs, n) approximate draws from a zero-mean unit-variance Matern-nu GP
    by random Fourier features (Rahimi & Recht): omega = g sqrt(2 nu / u) / ell
    with g ~ N(0, I), u ~ chi^2_{2 nu}, f = sqrt(2/R) sum cos(<omega, x> + b).
    Sample r uses seed seed0 + r; every draw comes from a generator of its own
    (no global random state is read or changed)."""
    d, n = x.shape
    out = torch.empty((nrhs, n), dtype=x.dtype, device=x.device)
    for r in range(nrhs):
        g = _gen(seed0 + r, FIELD, "cpu")
        gauss = torch.randn((nfeat, d), generator=g, dtype=torch.float64)
        rng = np.random.default_rng([int(seed0) + r, FIELD])
        u = torch.from_numpy(rng.chisquare(2.0 * nu, nfeat))
        omega = gauss * torch.sqrt(2.0 * nu / u)[:, None] / ell
        b = 2.0 * math.pi * torch.rand((nfeat,), generator=g, dtype=torch.float64)
        ph = omega.to(x.device, x.dtype) @ x + b.to(x.device, x.dtype)[:, None]
        out[r] = math.sqrt(2.0 / nfeat) * torch.cos(ph).sum(0)
    return out


# -- workloads --------------------------------------------------------------

@dataclass
class Workload:
    name: str
    dim: int
    kernel: str            # "se" or "matern"
    ell: float
    nu: Optional[float]
    eps: float
    n: int
    sigma2: Tuple[float, ...]
    nrhs: int = 1
    points: str = "uniform"
    f: str = ""
    targets: Tuple[str, int] = ("uniform", 1000)
    seed: int = 0
    rel_tol: Optional[float] = None
    notes: str = field(default="")


WORKLOADS = {
    "1d_se_n2000": Workload("1d_se_n2000", 1, "se", 0.1, None, 1e-8, 2000, (0.01,),
                            f="sin1d", targets=("uniform", 1000), seed=1, rel_tol=1e-10),
    "2d_matern32_n1e6": Workload("2d_matern32_n1e6", 2, "matern", 0.1, 1.5, 1e-4, 1_000_000,
                                 (0.09,), f="cos2d", targets=("uniform", 100_000), seed=2),
    "3d_se_mix_n1e7": Workload("3d_se_mix_n1e7", 3, "se", 0.2, None, 1e-5, 10_000_000, (0.04,),
                               points="mixture", f="sinprod", targets=("grid", 60), seed=3),
    "2d_matern32_n1e7_64rhs": Workload("2d_matern32_n1e7_64rhs", 2, "matern", 0.05, 1.5, 1e-4,
                                       10_000_000, tuple(), nrhs=64, f="rff",
                                       targets=("grid", 1000), seed=4),
    "2d_matern32_n1e9": Workload("2d_matern32_n1e9", 2, "matern", 0.1, 1.5, 1e-3, 1_000_000_000,
                                 (0.09,), f="smooth5", targets=("grid", 1000), seed=5),
}


def sigma2_list(w: Workload) -> Tuple[float, ...]:
    """Per-RHS noise variances; the 64-RHS workload draws them log-uniform
    on [0.01, 0.3] from its seed."""
    if w.sigma2:
        return w.sigma2
    g = _gen(w.seed, NOISE + 100, "cpu")
    u = torch.rand((w.nrhs,), generator=g, dtype=torch.float64)
    return tuple(float(math.exp(math.log(0.01) + (math.log(0.3) - math.log(0.01)) * t)) for t in u)


def make_points(w: Workload, n: Optional[int] = None, dtype=torch.float64, device="cpu"):
    n = w.n if n is None else n
    if w.points == "mixture":
        return mixture_points(n, w.dim, w.seed, dtype=dtype, device=device)
    return uniform_points(n, w.dim, w.seed, dtype=dtype, device=device)


def make_data(w: Workload, x: torch.Tensor) -> torch.Tensor:
    """(nrhs, n) data y = f(x) + noise."""
    s2 = sigma2_list(w)
    if w.f == "rff":
        f = rff_gp_samples(x, w.nrhs, w.ell, w.nu, seed0=0)
    else:
        f = {"sin1d": f_sin1d, "cos2d": f_cos2d, "sinprod": f_sinprod,
             "smooth5": f_smooth5}[w.f](x)[None, :]
    y = torch.empty((w.nrhs, x.shape[1]), dtype=x.dtype, device=x.device)
    for r in range(w.nrhs):
        y[r] = f[r] + noise((x.shape[1],), s2[r], w.seed * 1000 + r, dtype=x.dtype,
                            device=x.device)
    return y


def make_targets(w: Workload, q: Optional[int] = None, dtype=torch.float64, device="cpu"):
    kind, size = w.targets
    if kind == "grid":
        return grid_targets(size, w.dim, dtype=dtype, device=device)
    q = size if q is None else q
    g = _gen(w.seed, TARGETS, device)
    return torch.rand((w.dim, q), generator=g, dtype=dtype, device=device)
