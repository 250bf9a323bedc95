"""Training of the learned per-frequency diagonal preconditioner.

Data come from the method itself on the GPU: for each generated regression
problem the library builds the weight-space system, and preconditioned CG
(efgp_solve with a given diagonal) is run to the same residual tolerance for
every member of the family P_j = (N D_j^2 + sigma^2)^(-s), s in
{0, 0.5, 0.75, 0.9, 1, 1.1, 1.25} (s = 0 is plain CG, s = 1 is Jacobi, since
T_jj = v_0 = N).  The searches run in double precision at the tolerance the
single-precision solves use: single-precision iteration counts vary by tens
of percent with rounding, which made near-ties look like gains.  The
iteration counts of these residual histories give each problem its target
exponent s* (1 unless a member needs 10% fewer iterations than Jacobi).  The
network (efgp_mlp_* kernels: bf16 matrix cores, float accumulation, Adam)
maps each frequency's features (efgp_features) to s*; the solver averages
its outputs over the frequencies into one exponent s_bar, so the diagonal is
a member of the family (smooth across frequencies by construction) and
equals Jacobi when |s_bar - 1| is below the gate EFGP_MLP_GATE.  The gate is
set from the training problems.  Preconditioned CG stops on the
unpreconditioned residual, so the network changes iteration counts, never
the tolerance met.

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

S_VALUES = (0.0, 0.5, 0.75, 0.9, 1.0, 1.1, 1.25)


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


def make_problem(pr, device="cuda", precision=32, spread_method=None):
    """The problem's plan.  Inputs are drawn in single precision; a
    precision-64 plan takes them promoted exactly, spread at the same
    tolerance eps/10 as the single-precision plan.  spread_method: an
    explicit spreader (default: the automatic choice)."""
    w = synth.Workload("train", pr["dim"], pr["kernel"], pr["ell"], pr["nu"], pr["eps"], pr["n"],
                       (pr["sigma2"],), points=pr["points"], f="", seed=pr["seed"])
    x = synth.make_points(w, dtype=torch.float32, device=device)
    omega = torch.tensor([3.0, 4.0, 2.0][:pr["dim"]])
    y = (synth.f_plane_wave(x, omega) + synth.noise((pr["n"],), pr["sigma2"], pr["seed"], dtype=torch.float32,
                                                     device=device)).reshape(1, -1).contiguous()
    extra = {}
    if spread_method is not None:
        extra["spread_method"] = spread_method
    if precision == 64:
        x, y = x.double(), y.double()
        extra["nufft_tol"] = pr["eps"] / 10
    plan = C.efgp_setup(x, y, pr["sigma2"], kernel=pr["kernel"], nu=pr["nu"] or 0.0, lengthscale=pr["ell"],
                        eps=pr["eps"], **extra)
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


def rho_for(pr, precision=32):
    """Residual tolerance of the searches and of the held-out comparison:
    eps/100, but not below what FP32 CG reaches reliably (the deployed
    solves are single precision; the best diagonal depends on the
    tolerance, so the double-precision searches use the same one)."""
    return max(pr["eps"] / 100, 1e-5)


def search(plan, pr, rho):
    """Iteration counts of the diagonal family on one problem and its target
    exponent s* (None if nothing converged): Jacobi's s = 1 unless a member
    needs 10% fewer iterations; then the best member's s."""
    D = C.efgp_get_weights(plan)
    a = pr["n"] * D * D + pr["sigma2"]
    rdt = torch.float32 if plan.precision == 32 else torch.float64
    results = []
    it_jac, _ = solve_iters(plan, rho, diag=(1.0 / a).to(rdt).reshape(1, -1).contiguous())
    it_plain, _ = solve_iters(plan, rho)
    cap = min(20000, 4 * min(it_plain, it_jac) + 200)
    for sv in S_VALUES:
        if sv == 1.0:
            results.append((sv, it_jac))
        elif sv == 0.0:
            results.append((sv, it_plain))
        else:
            dg = a ** (-sv)
            dg = (dg / dg.max()).to(rdt).reshape(1, -1).contiguous()
            results.append((sv, solve_iters(plan, rho, diag=dg, max_iter=cap)[0]))
    best = min(results, key=lambda r: r[1])
    if best[1] >= 20000:
        return results, best, it_plain, it_jac, None
    target = 1.0 if best[1] >= 0.9 * it_jac else best[0]
    return results, best, it_plain, it_jac, target


def build_dataset(problems, log=print):
    feats, targets, wts, meta = [], [], [], []
    for k, pr in enumerate(problems):
        t0 = time.time()
        try:
            plan = make_problem(pr, precision=64)
        except C.EfgpError as e:  # e.g. a size beyond the library limits
            log(f"[precond] {k}: skipped ({e})")
            continue
        rho = rho_for(pr, 64)
        results, best, it_plain, it_jac, tgt = search(plan, pr, rho)
        if tgt is None:
            log(f"[precond] {k}: dropped (no member converged to {rho:g})")
            del plan
            continue
        f, _ = C.efgp_features(plan, 0)
        feats.append(f)
        targets.append(torch.full((plan.M,), float(tgt), device="cuda"))
        wts.append(torch.full((plan.M,), 1.0 / plan.M, device="cuda"))
        meta.append(dict(problem=pr, m=plan.m, M=plan.M, plain=it_plain, jacobi=it_jac, best_s=best[0],
                         best=best[1], target_s=tgt, counts={str(sv): it for sv, it in results}))
        log(f"[precond] {k}: d={pr['dim']} {pr['kernel']}{pr['nu'] or ''} {pr['points']} ell={pr['ell']:.3f} "
            f"eps={pr['eps']:g} N={pr['n']:.2e} s2={pr['sigma2']:.3f} m={plan.m}: plain {it_plain} jacobi {it_jac} "
            f"best s={best[0]} {best[1]} -> target {tgt}  [{time.time() - t0:.1f}s]")
        del plan
    X = torch.cat(feats).contiguous()
    T = torch.cat(targets).contiguous()
    W = torch.cat(wts)
    W = (W * (W.numel() / W.sum())).float().contiguous()
    return X, T, W, meta, feats


def init_params(seed=0):
    """He initialisation of the packed network; the last layer starts at
    zero weights and bias 1, so the untrained network is exactly Jacobi."""
    g = torch.Generator().manual_seed(seed)
    H, F = C.MLP_HIDDEN, C.NFEAT
    parts = [torch.randn(H, F, generator=g) * math.sqrt(2.0 / F), torch.zeros(H),
             torch.randn(H, H, generator=g) * math.sqrt(2.0 / H), torch.zeros(H),
             torch.randn(H, H, generator=g) * math.sqrt(2.0 / H), torch.zeros(H),
             torch.zeros(H), torch.ones(1)]
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


def exponent(weights, feats):
    """The network's exponent on one problem, as the library forms it: the
    mean of the per-frequency outputs (each clamped to [-1, 3], non-finite
    ones counted as 1), clamped to the searched range [0, 1.25]."""
    o = C.efgp_mlp_forward(weights, feats).double()
    o = torch.where(torch.isfinite(o), o.clamp(-1.0, 3.0), torch.ones_like(o))
    return min(max(float(o.mean()), 0.0), 1.25)


def choose_gate(weights, feats_list, meta):
    """Gate around s = 1, chosen on the training problems: the width that
    minimises their geometric-mean iteration count relative to Jacobi, where
    a problem outside the gate is charged the searched count of the family
    member nearest to its s_bar (the largest such width on ties)."""
    sb = [exponent(weights, f) for f in feats_list]

    def cost(delta):
        tot = 0.0
        for v, m in zip(sb, meta):
            if abs(v - 1.0) >= delta:
                near = min(S_VALUES, key=lambda s: abs(s - v))
                tot += math.log(max(1, m["counts"][str(near)]) / max(1, m["jacobi"]))
        return tot / max(1, len(sb))

    grid = [0.025 * k for k in range(41)]
    best = min(cost(dl) for dl in grid)
    gate = max(dl for dl in grid if cost(dl) <= best + 1e-12)
    return gate, sb


def evaluate(problems, weights, gate, log=print):
    """Held-out iteration counts: single precision as deployed (the library
    applies its compiled gate) and double precision (stable counts, the
    comparison of the two diagonals themselves)."""
    rows = []
    for pr in problems:
        row = dict(problem=pr)
        for prec in (32, 64):
            try:
                plan = make_problem(pr, precision=prec)
            except C.EfgpError as e:
                log(f"[precond] held-out skipped ({e})")
                break
            rho = rho_for(pr, prec)
            it_plain, _ = solve_iters(plan, rho)
            it_jac, _ = solve_iters(plan, rho, precond=C.PRECOND_JACOBI)
            it_learn, ss = solve_iters(plan, rho, precond=C.PRECOND_LEARNED, weights=weights)
            f, _ = C.efgp_features(plan, 0)
            sb = exponent(weights, f)
            key = "" if prec == 32 else "_fp64"
            row.update({"m": plan.m, "plain" + key: it_plain, "jacobi" + key: it_jac, "learned" + key: it_learn,
                        "fell_back" + key: ss["fell_back"], "rho" + key: rho, "s_bar" + key: sb,
                        "gated_to_jacobi" + key: bool(abs(sb - 1.0) < gate)})
            log(f"[precond] held-out FP{prec} d={pr['dim']} {pr['kernel']}{pr['nu'] or ''} {pr['points']} "
                f"N={pr['n']:.2e} s2={pr['sigma2']:.3f} eps={pr['eps']:g}: plain {it_plain} jacobi {it_jac} "
                f"learned {it_learn} (s_bar {sb:.3f}, gate {gate:.3f})")
            del plan
        else:
            rows.append(row)
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=HERE)
    ap.add_argument("--train", type=int, default=120)
    ap.add_argument("--test", type=int, default=10)
    ap.add_argument("--large-n", type=int, default=30, help="extra large-N training problems")
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--seed", type=int, default=11)
    ap.add_argument("--save-dataset", default="", help="write the searched dataset here and stop")
    ap.add_argument("--load-dataset", default="", help="train on a dataset written by --save-dataset")
    ap.add_argument("--eval-only", default="", help="evaluate these weights on the held-out problems "
                    "(with the library's gate) and update DIR/precond_mlp.json")
    a = ap.parse_args()
    torch.cuda.set_device(0)
    log = lambda *s: print(*s, flush=True)
    tr = problem_family(a.seed, a.train) + large_n_family(a.seed + 7, a.large_n)
    te = problem_family(a.seed + 1, a.test)
    # the large 2D Matern-3/2 workload is always among the held-out problems
    te.append(dict(dim=2, kernel="matern", nu=1.5, ell=0.1, eps=1e-3, n=1_000_000_000, sigma2=0.09,
                   points="uniform", seed=5))
    if a.eval_only:
        p = load_weights(a.eval_only)
        rows = evaluate(te, p, C.MLP_GATE, log)
        path = os.path.join(a.out, "precond_mlp.json")
        d = json.load(open(path)) if os.path.exists(path) else {}
        d["heldout"] = rows
        d["gate_library"] = C.MLP_GATE
        with open(path, "w") as f:
            json.dump(d, f, indent=1)
        log(f"[precond] updated {path}")
        return
    if a.load_dataset:
        d = torch.load(a.load_dataset, weights_only=True)
        X, T, W = d["X"].cuda(), d["T"].cuda(), d["W"].cuda()
        per = [f.cuda() for f in d["per"]]
        meta = json.loads(d["meta"])
    else:
        X, T, W, meta, per = build_dataset(tr, log)
        if a.save_dataset:
            torch.save(dict(X=X.cpu(), T=T.cpu(), W=W.cpu(), per=[f.cpu() for f in per], meta=json.dumps(meta)),
                       a.save_dataset)
            log(f"[precond] wrote {a.save_dataset}")
            return
    p, hist = train(X, T, W, steps=a.steps, log=log)
    gate, sbs = choose_gate(p, per, meta)
    for mrow, v in zip(meta, sbs):
        mrow["s_bar"] = v
    log(f"[precond] gate {gate:.4f} (library: {C.MLP_GATE:.4f})")
    rows = evaluate(te, p, gate, log)
    os.makedirs(a.out, exist_ok=True)
    p.cpu().numpy().astype(np.float32).tofile(os.path.join(a.out, "precond_mlp.bin"))
    with open(os.path.join(a.out, "precond_mlp.json"), "w") as f:
        json.dump(dict(train=meta, loss=hist, heldout=rows, s_values=S_VALUES,
                       rho="max(eps/100, 1e-5); searches in FP64", gate=gate), f, indent=1)
    log(f"[precond] wrote {a.out}/precond_mlp.bin")


if __name__ == "__main__":
    main()
