"""Training of the learned per-frequency diagonal preconditioner.

Data come from the method itself on the GPU: for each generated regression
problem the library builds the weight-space system, and preconditioned CG
(efgp_solve with a given diagonal) is run to the same residual tolerance for
every member of the family P_j = (N D_j^2 + tau)^(-s) (s = 0 is plain CG,
s = 1 with tau = sigma^2 is Jacobi, since T_jj = v_0 = N).  The iteration
counts of these residual histories pick the best member per problem; its
diagonal, expressed relative to Jacobi, o_j = log(P_j (N D_j^2 + sigma^2)),
is the per-frequency regression target.  The network (efgp_mlp_* kernels:
bf16 matrix cores, float accumulation, Adam) maps the per-frequency features
of efgp_features to o_j.  Preconditioned CG stops on the unpreconditioned
residual, so the network changes iteration counts, never the tolerance met.

Usage (on a GPU):  python -m paper_2210_10210_amd.precond --out DIR
writes DIR/precond_mlp.bin (float32, EFGP_MLP_NPARAM values) and
DIR/precond_mlp.json (problems, search results, losses, held-out gains).
"""
import argparse
import json
import math
import os
import time

import numpy as np
import torch

import synth
from . import capi as C

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "precond_mlp.bin")

S_VALUES = (0.5, 0.75, 0.9, 1.0, 1.1, 1.25)
TAU_FACTORS = (0.25, 1.0, 4.0)


def load_weights(path=WEIGHTS, device="cuda"):
    a = np.fromfile(path, dtype=np.float32)
    if a.size != C.MLP_NPARAM or not np.all(np.isfinite(a)):
        raise ValueError(f"bad preconditioner weights file {path}")
    return torch.from_numpy(a).to(device)


def problem_family(seed, count):
    """Random problems shaped like the paper's workloads: d in {2,3}, SE and
    Matern kernels, lengthscales, noise levels and N spanning the configs."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        d = 2 if rng.uniform() < 0.75 else 3
        if d == 2:
            kern, nu = [("matern", 0.5), ("matern", 1.5), ("matern", 1.5), ("matern", 2.5), ("se", None)][rng.integers(5)]
            ell = float(np.exp(rng.uniform(np.log(0.05), np.log(0.2))))
            eps = float([1e-3, 3e-4, 1e-4][rng.integers(3)])
            if kern == "matern" and nu == 0.5:
                eps, ell = 1e-3, max(ell, 0.1)
        else:
            kern, nu = [("se", None), ("matern", 2.5)][rng.integers(2)]
            ell = float(np.exp(rng.uniform(np.log(0.15), np.log(0.3))))
            eps = float([1e-3, 1e-4, 1e-5][rng.integers(3)])
        n = int(np.exp(rng.uniform(np.log(1e5), np.log(1e9 if d == 2 else 3e7))))
        s2 = float(np.exp(rng.uniform(np.log(0.01), np.log(0.3))))
        pts = "mixture" if rng.uniform() < 0.25 else "uniform"
        out.append(dict(dim=d, kernel=kern, nu=nu, ell=ell, eps=eps, n=n, sigma2=s2, points=pts,
                        seed=int(seed * 1000 + i)))
    return out


def large_n_family(seed, count):
    """Training-only problems in the large-N regime of the 1e9-point 2D
    workloads (uniform points, Matern 3/2 or 5/2, N in [2e8, 1e9]), where the
    general family above has few members."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        nu = [1.5, 2.5][rng.integers(2)]
        out.append(dict(dim=2, kernel="matern", nu=nu, ell=float(np.exp(rng.uniform(np.log(0.05), np.log(0.2)))),
                        eps=float([1e-3, 3e-4][rng.integers(2)]),
                        n=int(np.exp(rng.uniform(np.log(2e8), np.log(1e9)))),
                        sigma2=float(np.exp(rng.uniform(np.log(0.01), np.log(0.3)))), points="uniform",
                        seed=int(seed * 1000 + i)))
    return out


def make_problem(pr, device="cuda"):
    w = synth.Workload("train", pr["dim"], pr["kernel"], pr["ell"], pr["nu"], pr["eps"], pr["n"],
                       (pr["sigma2"],), points=pr["points"], f="", seed=pr["seed"])
    x = synth.make_points(w, dtype=torch.float32, device=device)
    omega = torch.tensor([3.0, 4.0, 2.0][:pr["dim"]])
    y = (synth.f_plane_wave(x, omega) + synth.noise((pr["n"],), pr["sigma2"], pr["seed"], dtype=torch.float32,
                                                     device=device)).reshape(1, -1).contiguous()
    plan = C.efgp_setup(x, y, pr["sigma2"], kernel=pr["kernel"], nu=pr["nu"] or 0.0, lengthscale=pr["ell"],
                        eps=pr["eps"])
    return plan


def solve_iters(plan, rho, diag=None, precond=None, weights=None, max_iter=20000):
    if diag is not None:
        _, st, ss = C.efgp_solve(plan, rel_tol=rho, max_iter=max_iter, precond=C.PRECOND_DIAG,
                                 precond_diag=diag, stall_window=max_iter + 1, raise_on_error=False)
    else:
        _, st, ss = C.efgp_solve(plan, rel_tol=rho, max_iter=max_iter,
                                 precond=C.PRECOND_NONE if precond is None else precond,
                                 mlp_weights=weights, raise_on_error=False)
    ok = st in (C.EFGP_OK, C.EFGP_FELL_BACK)
    return (ss["iterations"] if ok else max_iter * 10), ss


def rho_for(pr):
    """Residual tolerance of the searches: eps/100, but not below what FP32
    CG reaches reliably."""
    return max(pr["eps"] / 100, 1e-5)


def search(plan, pr, rho):
    """Iteration counts of the diagonal family on one problem and the
    per-frequency target relative to Jacobi (None if nothing converged).
    The target is Jacobi (zero) unless some member beats it by more than
    10%; then it is the mean log-diagonal of the members within 5% of the
    best, which smooths near-ties between very different diagonals."""
    D = C.efgp_get_weights(plan)
    nd2 = pr["n"] * D * D
    s2 = pr["sigma2"]
    it_plain, _ = solve_iters(plan, rho)
    jac = (1.0 / (nd2 + s2)).float().reshape(1, -1).contiguous()
    it_jac, _ = solve_iters(plan, rho, diag=jac)
    cap = min(20000, 4 * min(it_plain, it_jac) + 200)
    results = [(0.0, 1.0, it_plain), (1.0, 1.0, it_jac)]
    for s in S_VALUES:
        for tf in TAU_FACTORS:
            if s == 1.0 and tf == 1.0:
                continue
            dg = ((nd2 + tf * s2) ** (-s))
            dg = (dg / dg.max()).float().reshape(1, -1).contiguous()
            it, _ = solve_iters(plan, rho, diag=dg, max_iter=cap)
            results.append((s, tf, it))
    best = min(results, key=lambda r: r[2])
    if best[2] >= 20000:
        return results, best, it_plain, it_jac, None
    logjac = torch.log(nd2 + s2)
    if best[2] >= 0.9 * it_jac:
        tgt = torch.zeros_like(logjac)
    else:
        near = [r for r in results if r[2] <= 1.05 * best[2]]
        tgt = torch.zeros_like(logjac)
        for sv, tf, _ in near:
            tgt += (-sv * torch.log(nd2 + tf * s2) if sv > 0 else 0.0) + logjac
        tgt /= len(near)
    return results, best, it_plain, it_jac, tgt.float()


def build_dataset(problems, log=print):
    feats, targets, wts, meta = [], [], [], []
    for k, pr in enumerate(problems):
        t0 = time.time()
        try:
            plan = make_problem(pr)
        except C.EfgpError as e:  # e.g. a size beyond the library limits
            log(f"[precond] {k}: skipped ({e})")
            continue
        rho = rho_for(pr)
        results, best, it_plain, it_jac, tgt = search(plan, pr, rho)
        if tgt is None:
            log(f"[precond] {k}: dropped (no member converged to {rho:g})")
            del plan
            continue
        f, _ = C.efgp_features(plan, 0)
        feats.append(f)
        # centre the target: PCG is invariant to a global scale of P
        targets.append(tgt - tgt.mean())
        wts.append(torch.full((plan.M,), 1.0 / plan.M, device="cuda"))
        meta.append(dict(problem=pr, m=plan.m, M=plan.M, plain=it_plain, jacobi=it_jac, best_s=best[0],
                         best_tau=best[1], best=best[2]))
        log(f"[precond] {k}: d={pr['dim']} {pr['kernel']}{pr['nu'] or ''} ell={pr['ell']:.3f} eps={pr['eps']:g} "
            f"N={pr['n']:.2e} s2={pr['sigma2']:.3f} m={plan.m}: plain {it_plain} jacobi {it_jac} "
            f"best (s={best[0]}, tau={best[1]}x) {best[2]}  [{time.time() - t0:.1f}s]")
        del plan
    X = torch.cat(feats).contiguous()
    T = torch.cat(targets).contiguous()
    W = torch.cat(wts)
    W = (W * (W.numel() / W.sum())).float().contiguous()
    return X, T, W, meta


def init_params(seed=0):
    """He initialisation of the packed network; the last layer starts at zero
    so the untrained network is exactly Jacobi."""
    g = torch.Generator().manual_seed(seed)
    H, F = C.MLP_HIDDEN, C.NFEAT
    parts = [torch.randn(H, F, generator=g) * math.sqrt(2.0 / F), torch.zeros(H),
             torch.randn(H, H, generator=g) * math.sqrt(2.0 / H), torch.zeros(H),
             torch.randn(H, H, generator=g) * math.sqrt(2.0 / H), torch.zeros(H),
             torch.zeros(H), torch.zeros(1)]
    return torch.cat([p.reshape(-1) for p in parts]).float().cuda().contiguous()


def train(X, T, W, steps=3000, lr=2e-3, seed=0, log=print):
    p = init_params(seed)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    hist = []
    for step in range(1, steps + 1):
        loss, grad = C.efgp_mlp_loss_grad(p, X, T, W)
        C.efgp_mlp_adam(p, grad, m, v, step, lr=lr * (0.1 ** (step / steps)))
        if step == 1 or step % 250 == 0 or step == steps:
            val = float(loss.cpu()[0])
            hist.append((step, val))
            log(f"[precond] step {step} loss {val:.5f}")
    return p, hist


def evaluate(problems, weights, log=print):
    rows = []
    for pr in problems:
        try:
            plan = make_problem(pr)
        except C.EfgpError as e:
            log(f"[precond] held-out skipped ({e})")
            continue
        rho = rho_for(pr)
        it_plain, _ = solve_iters(plan, rho)
        it_jac, _ = solve_iters(plan, rho, precond=C.PRECOND_JACOBI)
        it_learn, ss = solve_iters(plan, rho, precond=C.PRECOND_LEARNED, weights=weights)
        rows.append(dict(problem=pr, m=plan.m, plain=it_plain, jacobi=it_jac, learned=it_learn,
                         fell_back=ss["fell_back"]))
        log(f"[precond] held-out d={pr['dim']} {pr['kernel']}{pr['nu'] or ''} N={pr['n']:.2e} "
            f"s2={pr['sigma2']:.3f} eps={pr['eps']:g}: plain {it_plain} jacobi {it_jac} learned {it_learn}")
        del plan
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=HERE)
    ap.add_argument("--train", type=int, default=120)
    ap.add_argument("--test", type=int, default=10)
    ap.add_argument("--large-n", type=int, default=30, help="extra large-N training problems")
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--seed", type=int, default=11)
    a = ap.parse_args()
    torch.cuda.set_device(0)
    log = lambda *s: print(*s, flush=True)
    tr = problem_family(a.seed, a.train) + large_n_family(a.seed + 7, a.large_n)
    te = problem_family(a.seed + 1, a.test)
    # the large 2D Matern-3/2 workload is always among the held-out problems
    te.append(dict(dim=2, kernel="matern", nu=1.5, ell=0.1, eps=1e-3, n=1_000_000_000, sigma2=0.09,
                   points="uniform", seed=5))
    X, T, W, meta = build_dataset(tr, log)
    p, hist = train(X, T, W, steps=a.steps, log=log)
    rows = evaluate(te, p, log)
    os.makedirs(a.out, exist_ok=True)
    p.cpu().numpy().astype(np.float32).tofile(os.path.join(a.out, "precond_mlp.bin"))
    with open(os.path.join(a.out, "precond_mlp.json"), "w") as f:
        json.dump(dict(train=meta, loss=hist, heldout=rows, s_values=S_VALUES, tau_factors=TAU_FACTORS,
                       rho="eps/100"), f, indent=1)
    log(f"[precond] wrote {a.out}/precond_mlp.bin")


if __name__ == "__main__":
    main()
