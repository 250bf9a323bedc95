"""Thin ctypes binding of libefgp.so (declared in include/efgp.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch tensors supply device memory and the current HIP
stream.  Importing this module loads the library and fails loudly if it is
missing — there is no fallback path.
"""
import ctypes
import os
from ctypes import POINTER, c_double, c_float, c_int32, c_int64, c_void_p

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libefgp.so")

EFGP_OK, EFGP_NOT_CONVERGED, EFGP_FELL_BACK = 0, 1, 2
EFGP_EINVAL, EFGP_EDOMAIN, EFGP_ETOOLARGE, EFGP_ENOMEM, EFGP_EHIP, EFGP_EMODEL = -1, -2, -3, -4, -5, -6
KERNEL_SE, KERNEL_MATERN = 0, 1
PRECOND_NONE, PRECOND_JACOBI, PRECOND_LEARNED, PRECOND_DIAG, PRECOND_CIRCULANT = 0, 1, 2, 3, 4
SPREAD_AUTO, SPREAD_TILES, SPREAD_GRID_LDS, SPREAD_REGIONS = 0, 1, 2, 3
LAUNCH_AUTO, LAUNCH_PLAIN, LAUNCH_GRAPH, LAUNCH_BLOCK = 0, 1, 2, 3
NFEAT = 5
MLP_HIDDEN = 64
MLP_GATE = 0.15   # EFGP_MLP_GATE of include/efgp.h
MLP_NPARAM = 64 * 5 + 64 + 64 * 64 + 64 + 64 * 64 + 64 + 64 + 1


class efgp_problem(ctypes.Structure):
    _fields_ = [("dim", c_int32), ("kernel", c_int32), ("lengthscale", c_double), ("nu", c_double),
                ("variance", c_double), ("eps", c_double), ("precision", c_int32),
                ("nufft_tol", c_double), ("n", c_int64), ("x", c_void_p), ("nrhs", c_int32),
                ("y", c_void_p), ("sigma2", POINTER(c_double)), ("stream", c_void_p),
                ("m_override", c_int32), ("spread_method", c_int32), ("tile", c_int32),
                ("spread_epoch", c_int32)]


class efgp_info(ctypes.Structure):
    _fields_ = [("dim", c_int32), ("precision", c_int32), ("nrhs", c_int32), ("kernel", c_int32),
                ("m", c_int32), ("L", c_int32), ("nf", c_int32), ("nf_eval", c_int32), ("w", c_int32),
                ("spread_method", c_int32), ("tile", c_int32), ("setup_passes", c_int32),
                ("M", c_int64), ("n", c_int64), ("h", c_double), ("es_beta", c_double),
                ("nufft_tol", c_double), ("kernel_l2", c_double), ("ms_sort", c_double),
                ("ms_spread", c_double), ("ms_fft", c_double), ("ms_deconv", c_double),
                ("ms_setup_total", c_double)]


class efgp_tune_result(ctypes.Structure):
    _fields_ = [("spread_method", c_int32), ("tile", c_int32), ("ms_setup", c_double), ("candidates", c_int32),
                ("reserved", c_int32)]


class efgp_solve_opts(ctypes.Structure):
    _fields_ = [("rel_tol", c_double), ("max_iter", c_int64), ("precond", c_int32),
                ("iters_per_sync", c_int32), ("beta_init", c_void_p), ("precond_diag", c_void_p),
                ("mlp_weights", c_void_p), ("stall_window", c_int64), ("stream", c_void_p),
                ("record_history", c_int32), ("launch", c_int32), ("refine", c_int32), ("reserved", c_int32)]


class efgp_solve_stats(ctypes.Structure):
    _fields_ = [("iterations", c_int64), ("converged", c_int32), ("fell_back", c_int32),
                ("rel_residual", c_double), ("ms_solve", c_double), ("history", POINTER(c_double)),
                ("history_len", c_int64), ("refine_steps", c_int32), ("reserved", c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"EFGP HIP library not built: {LIB_PATH} is missing "
                          "(run __graft_entry__.build() or paper_2210_10210_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    P = c_void_p
    sig = {
        "efgp_setup": ([POINTER(efgp_problem), POINTER(c_void_p)], c_int32),
        "efgp_solve": ([P, POINTER(efgp_solve_opts), P, POINTER(efgp_solve_stats)], c_int32),
        "efgp_eval": ([P, P, c_int64, P, P, P], c_int32),
        "efgp_mean_at_points": ([P, P, P, P, P], c_int32),
        "efgp_prior_setup": ([POINTER(efgp_problem), POINTER(c_void_p)], c_int32),
        "efgp_sample_prior": ([P, P, c_int64, P, P, P], c_int32),
        "efgp_variance": ([P, c_int32, c_int64, P, P, POINTER(efgp_solve_opts), POINTER(efgp_solve_stats)],
                          c_int32),
        "efgp_eval_status": ([P], c_int32),
        "efgp_get_toeplitz": ([P, P, P], c_int32),
        "efgp_get_rhs": ([P, P, P], c_int32),
        "efgp_get_weights": ([P, P, P], c_int32),
        "efgp_apply": ([P, P, P, P], c_int32),
        "efgp_apply_noalloc": ([P, P, P, P], c_int32),
        "efgp_tune_spread": ([POINTER(efgp_problem), POINTER(efgp_tune_result)], c_int32),
        "efgp_tune_save": ([ctypes.c_char_p], c_int32),
        "efgp_tune_load": ([ctypes.c_char_p, P], c_int32),
        "efgp_tune_clear": ([], None),
        "efgp_features": ([P, c_int32, P, P, P], c_int32),
        "efgp_circulant_eigs": ([P, c_int32, P, P, P], c_int32),
        "efgp_get_info": ([P, POINTER(efgp_info)], c_int32),
        "efgp_destroy": ([P], None),
        "efgp_release_workspace": ([], None),
        "efgp_strerror": ([c_int32], ctypes.c_char_p),
        "efgp_mlp_forward": ([P, c_int64, P, P, P], c_int32),
        "efgp_mlp_loss_grad": ([P, c_int64, P, P, P, P, P, P], c_int32),
        "efgp_mlp_adam": ([P, P, P, P, c_int64, c_float, c_float, c_float, c_float, P], c_int32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


lib = _load()

# exported names, in the order include/efgp.h declares them
SYMBOLS = ["efgp_setup", "efgp_prior_setup", "efgp_solve", "efgp_eval", "efgp_sample_prior",
           "efgp_mean_at_points", "efgp_variance", "efgp_eval_status", "efgp_tune_spread", "efgp_tune_save",
           "efgp_tune_load", "efgp_tune_clear", "efgp_get_toeplitz",
           "efgp_get_rhs", "efgp_get_weights", "efgp_apply", "efgp_apply_noalloc", "efgp_features", "efgp_circulant_eigs", "efgp_get_info",
           "efgp_destroy", "efgp_release_workspace", "efgp_strerror", "efgp_mlp_forward", "efgp_mlp_loss_grad",
           "efgp_mlp_adam"]


class EfgpError(RuntimeError):
    def __init__(self, status, where):
        self.status = int(status)
        super().__init__(f"{where}: {efgp_strerror(status)} (status {status})")


def efgp_strerror(status: int) -> str:
    return lib.efgp_strerror(int(status)).decode()


def _stream(stream):
    if stream is None:
        return c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return c_void_p(stream.cuda_stream)
    return c_void_p(int(stream))


def _dev(t, dtype, name, numel=None):
    """Device pointer of a contiguous tensor of the given dtype; with numel,
    the tensor must hold exactly that many elements (the library reads or
    writes that many and cannot check the size itself)."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must hold {numel} elements, got {t.numel()}")
    return c_void_p(t.data_ptr())


def _targets(t, dim, name="targets"):
    """Number of points of a (dim, q) coordinate tensor."""
    if not isinstance(t, torch.Tensor) or t.dim() != 2 or t.shape[0] != dim:
        raise ValueError(f"{name} must be a ({dim}, q) tensor")
    return int(t.shape[1])


def _cplx_dtype(precision):
    return torch.complex64 if precision == 32 else torch.complex128


class Plan:
    """Owner of an efgp_plan handle (destroyed with the object)."""

    def __init__(self, handle, info):
        self.handle = handle
        self.info = info

    @property
    def M(self):
        return int(self.info.M)

    @property
    def m(self):
        return int(self.info.m)

    @property
    def h(self):
        return float(self.info.h)

    @property
    def dim(self):
        return int(self.info.dim)

    @property
    def nrhs(self):
        return int(self.info.nrhs)

    @property
    def precision(self):
        return int(self.info.precision)

    def __del__(self):
        if getattr(self, "handle", None) and lib is not None:
            lib.efgp_destroy(self.handle)
            self.handle = None


def _problem(x, y, sigma2, kernel, lengthscale, nu, eps, variance, nufft_tol, m, spread_method, tile, stream,
             spread_epoch=0):
    if x.dim() != 2:
        raise ValueError("x must be (d, n)")
    dt = x.dtype
    if dt not in (torch.float32, torch.float64):
        raise TypeError("x must be float32 or float64")
    if y.dim() == 1:
        y = y.reshape(1, -1)
    d, n = x.shape
    nrhs = y.shape[0]
    if y.shape[1] != n:
        raise ValueError("y must have n columns")
    s2 = [float(sigma2)] * nrhs if isinstance(sigma2, (int, float)) else [float(s) for s in sigma2]
    if len(s2) != nrhs:
        raise ValueError("need one sigma2 per data vector")
    arr = (c_double * nrhs)(*s2)
    pr = efgp_problem()
    pr.dim = d
    pr.kernel = {"se": KERNEL_SE, "matern": KERNEL_MATERN}[kernel] if isinstance(kernel, str) else int(kernel)
    pr.lengthscale = float(lengthscale)
    pr.nu = float(nu or 0.0)
    pr.variance = float(variance)
    pr.eps = float(eps)
    pr.precision = 32 if dt == torch.float32 else 64
    pr.nufft_tol = float(nufft_tol)
    pr.n = n
    pr.x = _dev(x, dt, "x")
    pr.nrhs = nrhs
    pr.y = _dev(y, dt, "y")
    pr.sigma2 = arr
    pr.stream = _stream(stream)
    pr.m_override = int(m)
    pr.spread_method = int(spread_method)
    pr.tile = int(tile)
    pr.spread_epoch = int(spread_epoch)
    return pr


def efgp_setup(x, y, sigma2, *, kernel="se", lengthscale, nu=0.0, eps, variance=1.0,
               nufft_tol=0.0, m=0, spread_method=SPREAD_AUTO, tile=0, spread_epoch=0, stream=None) -> Plan:
    """Steps 1-3 of the EFGP algorithm.  x: (d, n) device tensor in [0,1]^d
    (float32 -> precision 32, float64 -> precision 64); y: (nrhs, n) or (n,)
    of the same dtype; sigma2: float or sequence of nrhs floats."""
    pr = _problem(x, y, sigma2, kernel, lengthscale, nu, eps, variance, nufft_tol, m, spread_method, tile, stream,
                  spread_epoch)
    h = c_void_p()
    st = lib.efgp_setup(ctypes.byref(pr), ctypes.byref(h))
    if st != EFGP_OK:
        raise EfgpError(st, "efgp_setup")
    info = efgp_info()
    lib.efgp_get_info(h, ctypes.byref(info))
    return Plan(h, info)


def efgp_tune_spread(x, y, sigma2, *, kernel="se", lengthscale, nu=0.0, eps, variance=1.0, nufft_tol=0.0, m=0,
                     stream=None):
    """Time every candidate spreader on this problem's setup and store the
    fastest for later automatic setups of the same shape.  Returns a dict
    (spread_method, tile, ms_setup, candidates)."""
    pr = _problem(x, y, sigma2, kernel, lengthscale, nu, eps, variance, nufft_tol, m, SPREAD_AUTO, 0, stream)
    res = efgp_tune_result()
    st = lib.efgp_tune_spread(ctypes.byref(pr), ctypes.byref(res))
    if st != EFGP_OK:
        raise EfgpError(st, "efgp_tune_spread")
    return {"spread_method": int(res.spread_method), "tile": int(res.tile), "ms_setup": float(res.ms_setup),
            "candidates": int(res.candidates)}


def efgp_tune_save(path):
    st = lib.efgp_tune_save(os.fsencode(path))
    if st != EFGP_OK:
        raise EfgpError(st, "efgp_tune_save")


def efgp_tune_load(path):
    """Merge a saved tuning table; returns the number of entries read."""
    n = c_int32(0)
    st = lib.efgp_tune_load(os.fsencode(path), ctypes.byref(n))
    if st != EFGP_OK:
        raise EfgpError(st, "efgp_tune_load")
    return int(n.value)


def efgp_tune_clear():
    lib.efgp_tune_clear()


def efgp_prior_setup(dim, *, kernel="se", lengthscale, nu=0.0, eps, variance=1.0, precision=32,
                     nsamp=1, nufft_tol=0.0, m=0, stream=None) -> Plan:
    """Kernel-only plan for GP prior sampling (nsamp coefficient vectors per
    call); no points or data."""
    pr = efgp_problem()
    pr.dim = int(dim)
    pr.kernel = {"se": KERNEL_SE, "matern": KERNEL_MATERN}[kernel] if isinstance(kernel, str) else int(kernel)
    pr.lengthscale = float(lengthscale)
    pr.nu = float(nu or 0.0)
    pr.variance = float(variance)
    pr.eps = float(eps)
    pr.precision = int(precision)
    pr.nufft_tol = float(nufft_tol)
    pr.n = 0
    pr.nrhs = int(nsamp)
    pr.stream = _stream(stream)
    pr.m_override = int(m)
    h = c_void_p()
    st = lib.efgp_prior_setup(ctypes.byref(pr), ctypes.byref(h))
    if st != EFGP_OK:
        raise EfgpError(st, "efgp_prior_setup")
    info = efgp_info()
    lib.efgp_get_info(h, ctypes.byref(info))
    return Plan(h, info)


def efgp_sample_prior(plan: Plan, xi, targets, f_out=None, stream=None):
    """f_r(t) = Re sum_j D_j xi_rj exp(-2 pi i h <j,t>) at targets (d, q);
    xi: (nsamp, M) complex with iid N(0,1) real and imaginary parts."""
    cdt = _cplx_dtype(plan.precision)
    rdt = torch.float32 if plan.precision == 32 else torch.float64
    q = _targets(targets, plan.dim)
    if f_out is None:
        f_out = torch.empty((plan.nrhs, q), dtype=rdt, device="cuda")
    st = lib.efgp_sample_prior(plan.handle, _dev(xi, cdt, "xi", plan.nrhs * plan.M), q,
                               _dev(targets, rdt, "targets"), _dev(f_out, rdt, "f_out", plan.nrhs * q),
                               _stream(stream))
    if st != EFGP_OK:
        raise EfgpError(st, "efgp_sample_prior")
    return f_out


def efgp_release_workspace():
    lib.efgp_release_workspace()


def efgp_get_info(plan: Plan):
    info = efgp_info()
    st = lib.efgp_get_info(plan.handle, ctypes.byref(info))
    if st != EFGP_OK:
        raise EfgpError(st, "efgp_get_info")
    plan.info = info
    return {k: getattr(info, k) for k, _ in info._fields_}


def efgp_solve(plan: Plan, beta_out=None, *, rel_tol=0.0, max_iter=0, precond=PRECOND_NONE,
               iters_per_sync=0, beta_init=None, precond_diag=None, mlp_weights=None,
               stall_window=0, record_history=False, launch=None, refine=0, stream=None,
               raise_on_error=True):
    """Step 4: (P)CG.  Returns (beta, status, stats dict).  beta: (nrhs, M)
    complex tensor in the plan's precision.  refine > 0 (precision 32):
    iterative refinement with double residuals, at most `refine` steps."""
    cdt = _cplx_dtype(plan.precision)
    rdt = torch.float32 if plan.precision == 32 else torch.float64
    if beta_out is None:
        beta_out = torch.empty((plan.nrhs, plan.M), dtype=cdt, device="cuda")
    o = efgp_solve_opts()
    o.rel_tol = float(rel_tol)
    o.max_iter = int(max_iter)
    o.precond = int(precond)
    o.iters_per_sync = int(iters_per_sync)
    nm = plan.nrhs * plan.M
    o.beta_init = _dev(beta_init, cdt, "beta_init", nm) if beta_init is not None else None
    o.precond_diag = _dev(precond_diag, rdt, "precond_diag", nm) if precond_diag is not None else None
    o.mlp_weights = (_dev(mlp_weights, torch.float32, "mlp_weights", MLP_NPARAM)
                     if mlp_weights is not None else None)
    o.stall_window = int(stall_window)
    o.stream = _stream(stream)
    o.record_history = 1 if record_history else 0
    o.launch = LAUNCH_AUTO if launch is None else int(launch)
    o.refine = int(refine)
    stt = efgp_solve_stats()
    st = lib.efgp_solve(plan.handle, ctypes.byref(o), _dev(beta_out, cdt, "beta_out", nm), ctypes.byref(stt))
    if st < 0 and raise_on_error:
        raise EfgpError(st, "efgp_solve")
    hist = [stt.history[i] for i in range(stt.history_len)] if stt.history_len > 0 else []
    stats = {"iterations": int(stt.iterations), "converged": int(stt.converged),
             "fell_back": int(stt.fell_back), "rel_residual": float(stt.rel_residual),
             "ms_solve": float(stt.ms_solve), "history": hist, "refine_steps": int(stt.refine_steps)}
    return beta_out, int(st), stats


def efgp_variance(plan: Plan, targets, var_out=None, *, r=0, rel_tol=0.0, max_iter=0, precond=PRECOND_NONE,
                  iters_per_sync=0, mlp_weights=None, stall_window=0, refine=0, stream=None,
                  raise_on_error=True):
    """Posterior variance at targets (d, q) for data vector r's sigma^2 (one
    solve per target, batched by 64).  Returns (var (q,), status, stats)."""
    rdt = torch.float32 if plan.precision == 32 else torch.float64
    q = _targets(targets, plan.dim)
    if var_out is None:
        var_out = torch.empty(q, dtype=rdt, device="cuda")
    o = efgp_solve_opts()
    o.rel_tol = float(rel_tol)
    o.max_iter = int(max_iter)
    o.precond = int(precond)
    o.iters_per_sync = int(iters_per_sync)
    o.mlp_weights = (_dev(mlp_weights, torch.float32, "mlp_weights", MLP_NPARAM)
                     if mlp_weights is not None else None)
    o.stall_window = int(stall_window)
    o.stream = _stream(stream)
    o.launch = LAUNCH_AUTO
    o.refine = int(refine)
    stt = efgp_solve_stats()
    st = lib.efgp_variance(plan.handle, int(r), q, _dev(targets, rdt, "targets"), _dev(var_out, rdt, "var_out", q),
                           ctypes.byref(o), ctypes.byref(stt))
    if st < 0 and raise_on_error:
        raise EfgpError(st, "efgp_variance")
    stats = {"iterations": int(stt.iterations), "converged": int(stt.converged), "fell_back": int(stt.fell_back),
             "rel_residual": float(stt.rel_residual), "ms_solve": float(stt.ms_solve)}
    return var_out, int(st), stats


def efgp_eval(plan: Plan, beta, targets, mu_out=None, stream=None):
    """Step 6: posterior mean at targets (d, q) -> (nrhs, q) real tensor."""
    cdt = _cplx_dtype(plan.precision)
    rdt = torch.float32 if plan.precision == 32 else torch.float64
    q = _targets(targets, plan.dim)
    if mu_out is None:
        mu_out = torch.empty((plan.nrhs, q), dtype=rdt, device="cuda")
    st = lib.efgp_eval(plan.handle, _dev(beta, cdt, "beta", plan.nrhs * plan.M), q, _dev(targets, rdt, "targets"),
                       _dev(mu_out, rdt, "mu_out", plan.nrhs * q), _stream(stream))
    if st != EFGP_OK:
        raise EfgpError(st, "efgp_eval")
    return mu_out


def efgp_mean_at_points(plan: Plan, beta, x, mu_out=None, stream=None):
    """Step 7: posterior mean at the plan's own N points x (d, N) -> (nrhs, N)."""
    cdt = _cplx_dtype(plan.precision)
    rdt = torch.float32 if plan.precision == 32 else torch.float64
    n = _targets(x, plan.dim, "x")
    if n != plan.info.n:
        raise ValueError("x must be the plan's points")
    if mu_out is None:
        mu_out = torch.empty((plan.nrhs, n), dtype=rdt, device="cuda")
    st = lib.efgp_mean_at_points(plan.handle, _dev(beta, cdt, "beta", plan.nrhs * plan.M), _dev(x, rdt, "x"),
                                 _dev(mu_out, rdt, "mu_out", plan.nrhs * n), _stream(stream))
    if st != EFGP_OK:
        raise EfgpError(st, "efgp_mean_at_points")
    return mu_out


def efgp_eval_status(plan: Plan) -> int:
    return int(lib.efgp_eval_status(plan.handle))


def efgp_get_toeplitz(plan: Plan, stream=None):
    W2 = 4 * plan.m + 1
    out = torch.empty(W2 ** plan.dim, dtype=torch.complex128, device="cuda")
    st = lib.efgp_get_toeplitz(plan.handle, _dev(out, torch.complex128, "v_out"), _stream(stream))
    if st != EFGP_OK:
        raise EfgpError(st, "efgp_get_toeplitz")
    return out


def efgp_get_rhs(plan: Plan, stream=None):
    out = torch.empty((plan.nrhs, plan.M), dtype=torch.complex128, device="cuda")
    st = lib.efgp_get_rhs(plan.handle, _dev(out, torch.complex128, "b_out"), _stream(stream))
    if st != EFGP_OK:
        raise EfgpError(st, "efgp_get_rhs")
    return out


def efgp_get_weights(plan: Plan, stream=None):
    out = torch.empty(plan.M, dtype=torch.float64, device="cuda")
    st = lib.efgp_get_weights(plan.handle, _dev(out, torch.float64, "d_out"), _stream(stream))
    if st != EFGP_OK:
        raise EfgpError(st, "efgp_get_weights")
    return out


def efgp_apply(plan: Plan, inp, out=None, stream=None):
    cdt = _cplx_dtype(plan.precision)
    if out is None:
        out = torch.empty_like(inp)
    nm = plan.nrhs * plan.M
    st = lib.efgp_apply(plan.handle, _dev(inp, cdt, "in", nm), _dev(out, cdt, "out", nm), _stream(stream))
    if st != EFGP_OK:
        raise EfgpError(st, "efgp_apply")
    return out


def efgp_apply_noalloc(plan: Plan, inp, out, stream=None):
    """efgp_apply without any allocation inside the library (FFT
    intermediates in its static device scratch); the caller passes both
    tensors.  Calls that overlap on one GPU race."""
    cdt = _cplx_dtype(plan.precision)
    nm = plan.nrhs * plan.M
    st = lib.efgp_apply_noalloc(plan.handle, _dev(inp, cdt, "in", nm), _dev(out, cdt, "out", nm), _stream(stream))
    if st != EFGP_OK:
        raise EfgpError(st, "efgp_apply_noalloc")
    return out


def efgp_features(plan: Plan, r=0, stream=None):
    feats = torch.empty((plan.M, NFEAT), dtype=torch.float32, device="cuda")
    jac = torch.empty(plan.M, dtype=torch.float32, device="cuda")
    st = lib.efgp_features(plan.handle, int(r), _dev(feats, torch.float32, "feats"),
                           _dev(jac, torch.float32, "jacobi"), _stream(stream))
    if st != EFGP_OK:
        raise EfgpError(st, "efgp_features")
    return feats, jac


def efgp_circulant_eigs(plan: Plan, r=0, stream=None):
    """Eigenvalues (K^d reals, plan precision, C order) of the circulant
    preconditioner of system r, and the period K."""
    K = c_int32(0)
    st = lib.efgp_circulant_eigs(plan.handle, int(r), ctypes.byref(K), None, _stream(stream))
    if st != EFGP_OK:
        raise EfgpError(st, "efgp_circulant_eigs")
    dt = torch.float32 if plan.precision == 32 else torch.float64
    lam = torch.empty(K.value ** plan.dim, dtype=dt, device="cuda")
    st = lib.efgp_circulant_eigs(plan.handle, int(r), None, _dev(lam, dt, "lam"), _stream(stream))
    if st != EFGP_OK:
        raise EfgpError(st, "efgp_circulant_eigs")
    return lam, K.value


def _rows(feats):
    if not isinstance(feats, torch.Tensor) or feats.dim() != 2 or feats.shape[1] != NFEAT:
        raise ValueError(f"feats must be a (rows, {NFEAT}) tensor")
    return int(feats.shape[0])


def efgp_mlp_forward(params, feats, out=None, stream=None):
    rows = _rows(feats)
    if out is None:
        out = torch.empty(rows, dtype=torch.float32, device="cuda")
    st = lib.efgp_mlp_forward(_dev(params, torch.float32, "params", MLP_NPARAM), rows,
                              _dev(feats, torch.float32, "feats"), _dev(out, torch.float32, "out", rows),
                              _stream(stream))
    if st != EFGP_OK:
        raise EfgpError(st, "efgp_mlp_forward")
    return out


def efgp_mlp_loss_grad(params, feats, target, weights=None, grad=None, loss=None, stream=None):
    rows = _rows(feats)
    if grad is None:
        grad = torch.empty(MLP_NPARAM, dtype=torch.float32, device="cuda")
    if loss is None:
        loss = torch.empty(1, dtype=torch.float64, device="cuda")
    w = _dev(weights, torch.float32, "weights", rows) if weights is not None else None
    st = lib.efgp_mlp_loss_grad(_dev(params, torch.float32, "params", MLP_NPARAM), rows,
                                _dev(feats, torch.float32, "feats"),
                                _dev(target, torch.float32, "target", rows), w,
                                _dev(grad, torch.float32, "grad", MLP_NPARAM), _dev(loss, torch.float64, "loss", 1),
                                _stream(stream))
    if st != EFGP_OK:
        raise EfgpError(st, "efgp_mlp_loss_grad")
    return loss, grad


def efgp_mlp_adam(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    P = MLP_NPARAM
    st = lib.efgp_mlp_adam(_dev(params, torch.float32, "params", P), _dev(grad, torch.float32, "grad", P),
                           _dev(m, torch.float32, "m", P), _dev(v, torch.float32, "v", P), int(step),
                           float(lr), float(beta1), float(beta2), float(eps), _stream(stream))
    if st != EFGP_OK:
        raise EfgpError(st, "efgp_mlp_adam")
