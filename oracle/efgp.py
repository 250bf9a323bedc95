"""EFGP oracle in float64 (test infrastructure only; see package docstring).

Sign convention (the paper prints both signs; Sec. 3.2 eqs. (205), (88),
(rhs), (223)): the type-1 sums that build the Toeplitz vector v and the
right-hand side use exp(+2 pi i h <j, x>), so that T_{pl} = v_{j_p - j_l}
(a convolution, matching the extraction window of the fast Toeplitz
algorithm), and the posterior mean is evaluated with exp(-2 pi i h <j, x>).
This is the consistent factorization with design matrix
Phi_{nj} = D_j exp(-2 pi i h <j, x_n>); flipping every sign gives the same
real posterior mean because D is even in j.

Frequency arrays over J_K are C-ordered with offset j^(l)+K per dimension,
last dimension fastest.  Point arrays are (d, n) float64.
"""
import ctypes
import math
import os

import numpy as np
import scipy.linalg
import scipy.special

from . import build as _build

__all__ = [
    "SE", "MATERN", "kernel_value", "kernel_hat", "kernel_l2_norm", "choose_h_m",
    "freq_grid", "spectral_weights", "type1", "type2", "toeplitz_vector", "rhs",
    "toeplitz_apply", "toeplitz_apply_fft", "system_apply", "system_dense",
    "solve_dense", "cg", "posterior_mean", "ktilde_value", "gp_mean_dense",
    "Problem", "setup", "eepm", "rmse", "num_threads", "exact_kfun", "ktilde_kfun", "type1_at",
    "prior_sample", "posterior_variance", "gp_variance_dense",
    "optimal_circulant_eigs", "circulant_matrix", "circulant_period", "scaled_system_extended",
    "circulant_precond_eigs", "circulant_precond_apply",
]

SE = 0
MATERN = 1

# --------------------------------------------------------------------------
# C direct sums
# --------------------------------------------------------------------------
_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        lib.or_type1.argtypes = [ctypes.c_int, ctypes.c_int64, P, P, P, ctypes.c_int,
                                 ctypes.c_double, ctypes.c_int, P]
        lib.or_type2.argtypes = [ctypes.c_int, ctypes.c_int64, P, P, ctypes.c_int,
                                 ctypes.c_double, ctypes.c_int, P]
        lib.or_toeplitz_apply.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P]
        lib.or_system_dense.argtypes = [ctypes.c_int, ctypes.c_int, P, P, ctypes.c_double, P]
        lib.or_type1_select.argtypes = [ctypes.c_int, ctypes.c_int64, P, P, ctypes.c_int, P,
                                        ctypes.c_double, ctypes.c_int, P]
        lib.or_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().or_num_threads())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _points(x):
    x = np.ascontiguousarray(np.atleast_2d(np.asarray(x, dtype=np.float64)))
    return x


# --------------------------------------------------------------------------
# Kernels and spectral densities (Sec. 5 eqs. (Gker), (Cker); Fourier
# convention of Sec. 3.1: khat(xi) = int k(x) exp(-2 pi i <xi, x>) dx)
# --------------------------------------------------------------------------

def kernel_value(r, kernel, ell, nu=None, variance=1.0):
    """k(r) at distance r: squared exponential (Gker) or Matern (Cker)."""
    r = np.asarray(r, dtype=np.float64)
    if kernel == SE:
        return variance * np.exp(-r * r / (2.0 * ell * ell))
    z = np.sqrt(2.0 * nu) * r / ell
    with np.errstate(invalid="ignore", over="ignore"):
        val = 2.0 ** (1.0 - nu) / scipy.special.gamma(nu) * z ** nu * scipy.special.kv(nu, z)
    val = np.where(z == 0.0, 1.0, val)
    val = np.where(np.isfinite(val), val, 0.0)
    return variance * val


def kernel_hat(xi_norm, kernel, ell, nu, dim, variance=1.0):
    """Spectral density khat(|xi|) in dimension d (textbook closed forms in the
    convention of Sec. 3.1; Rasmussen & Williams eqs. 4.15 and 4.20)."""
    s = np.asarray(xi_norm, dtype=np.float64)
    if kernel == SE:
        return variance * (2.0 * math.pi * ell * ell) ** (dim / 2.0) * np.exp(
            -2.0 * math.pi ** 2 * ell * ell * s * s)
    c = (2.0 ** dim * math.pi ** (dim / 2.0) * math.gamma(nu + dim / 2.0) * (2.0 * nu) ** nu
         / (math.gamma(nu) * ell ** (2.0 * nu)))
    return variance * c * (2.0 * nu / ell ** 2 + 4.0 * math.pi ** 2 * s * s) ** (-(nu + dim / 2.0))


def kernel_l2_norm(kernel, ell, nu, dim, nodes=64):
    """||k||_{L2([-1,1]^d)} of the unit-variance kernel (used by eq. (maternheur)):
    tensor Gauss-Legendre with each axis split at 0 (Matern-1/2 has a kink
    there)."""
    g, w = np.polynomial.legendre.leggauss(nodes)
    t = np.concatenate([(g - 1.0) / 2.0, (g + 1.0) / 2.0])
    wt = np.concatenate([w / 2.0, w / 2.0])
    grids = np.meshgrid(*([t] * dim), indexing="ij")
    wgrids = np.meshgrid(*([wt] * dim), indexing="ij")
    r = np.sqrt(sum(gg * gg for gg in grids))
    wprod = np.prod(np.stack(wgrids), axis=0)
    k = kernel_value(r, kernel, ell, nu)
    return math.sqrt(float(np.sum(wprod * k * k)))


def choose_h_m(kernel, dim, eps, ell, nu=None):
    """Step 1 of the EFGP algorithm: frequency spacing h and half-width m.

    SE: the rule stated in Sec. 4.2 (aliasing and truncation each eps/2).
    Matern with 1/2 <= nu <= 5/2: the heuristic eq. (maternheur) with
    eps~ = eps * ||k||_{L2[-1,1]^d}.  Matern with nu > 5/2: eq. (maternhm).
    Logarithms are natural; m is rounded up.
    """
    d = dim
    if kernel == SE:
        h = 1.0 / (1.0 + ell * math.sqrt(2.0 * math.log(4.0 * d * 3.0 ** d / eps)))
        m = math.ceil(math.sqrt(0.5 * math.log(4.0 ** (d + 1) * d / eps)) / (math.pi * ell * h))
        return h, int(m)
    if nu <= 2.5:
        et = eps * kernel_l2_norm(kernel, ell, nu, d)
        h = 1.0 / (1.0 + 0.85 * (ell / math.sqrt(nu)) * math.log(1.0 / et))
        m = math.ceil((1.0 / h) * (math.pi ** (nu + d / 2.0) * ell ** (2.0 * nu) * et / 0.15)
                      ** (-1.0 / (2.0 * nu + d / 2.0)))
        return h, int(m)
    h = 1.0 / (1.0 + ell * math.sqrt(2.0 * d / nu) * math.log(d * 3.0 ** d / eps))
    m = math.ceil((d * 5.0 ** (d - 1) / (math.pi ** (d / 2.0) * eps)) ** (1.0 / (2.0 * nu))
                  * 1.6 * math.sqrt(nu) / (math.pi * h * ell))
    return h, int(m)


def freq_grid(m, dim):
    """Multi-indices of J_m as a (M, d) int array in C order (last fastest)."""
    ax = np.arange(-m, m + 1)
    g = np.meshgrid(*([ax] * dim), indexing="ij")
    return np.stack([gg.reshape(-1) for gg in g], axis=1)


def spectral_weights(h, m, dim, kernel, ell, nu=None, variance=1.0):
    """D_j = sqrt(h^d khat(h j)), j in J_m (eqs. (basis), (117)); full weight
    at the end points (footnote to eq. (110))."""
    J = freq_grid(m, dim)
    xi = h * np.sqrt(np.sum(J.astype(np.float64) ** 2, axis=1))
    return np.sqrt(h ** dim * kernel_hat(xi, kernel, ell, nu, dim, variance))


def ktilde_value(xdiff, h, m, kernel, ell, nu=None, variance=1.0):
    """Approximate kernel of eq. (110): sum_j h^d khat(hj) exp(2 pi i h <j, x>)
    (real part; the sum is real for an even khat).  xdiff: (d, q)."""
    xdiff = _points(xdiff)
    dim = xdiff.shape[0]
    J = freq_grid(m, dim).astype(np.float64)
    w = h ** dim * kernel_hat(h * np.sqrt(np.sum(J ** 2, axis=1)), kernel, ell, nu, dim, variance)
    ph = 2.0 * math.pi * h * (J @ xdiff)  # (M, q)
    return (w[:, None] * np.cos(ph)).sum(axis=0)


# --------------------------------------------------------------------------
# Direct sums (eqs. (88), (rhs), (muws))
# --------------------------------------------------------------------------

def type1(x, c, K, h, sign=+1):
    """sum_n c_n exp(sign 2 pi i h <j, x_n>) for j in J_K, by direct sums.
    c: None (unit strengths), real or complex (n,)."""
    x = _points(x)
    d, n = x.shape
    cre = cim = None
    if c is not None:
        c = np.asarray(c)
        cre = np.ascontiguousarray(np.real(c), dtype=np.float64)
        if np.iscomplexobj(c):
            cim = np.ascontiguousarray(np.imag(c), dtype=np.float64)
    out = np.empty(((2 * K + 1) ** d) * 2, dtype=np.float64)
    rc = _load().or_type1(d, n, _ptr(x), _ptr(cre), _ptr(cim), K, h, sign, _ptr(out))
    if rc != 0:
        raise RuntimeError(f"or_type1 failed ({rc})")
    return out.view(np.complex128).copy()


def type2(t, coef, K, h, sign=-1):
    """sum_{j in J_K} coef_j exp(sign 2 pi i h <j, t_i>) at targets t (d, q)."""
    t = _points(t)
    d, q = t.shape
    coef = np.ascontiguousarray(coef, dtype=np.complex128)
    assert coef.size == (2 * K + 1) ** d
    out = np.empty(2 * q, dtype=np.float64)
    rc = _load().or_type2(d, q, _ptr(t), _ptr(coef.view(np.float64)), K, h, sign, _ptr(out))
    if rc != 0:
        raise RuntimeError(f"or_type2 failed ({rc})")
    return out.view(np.complex128).copy()


def type1_at(x, c, J, h, sign=+1):
    """sum_n c_n exp(sign 2 pi i h <j, x_n>) at the multi-indices J (k, d),
    by direct sums (for sampled checks of large problems).  c: None or real."""
    x = _points(x)
    d, n = x.shape
    J = np.ascontiguousarray(np.asarray(J, dtype=np.int32).reshape(-1, d))
    cre = None if c is None else np.ascontiguousarray(c, dtype=np.float64)
    out = np.empty(2 * J.shape[0], dtype=np.float64)
    rc = _load().or_type1_select(d, n, _ptr(x), _ptr(cre), J.shape[0], _ptr(J), h, sign, _ptr(out))
    if rc != 0:
        raise RuntimeError("or_type1_select failed")
    return out.view(np.complex128).copy()


def toeplitz_vector(x, h, m):
    """v_j = sum_n exp(2 pi i h <j, x_n>), j in J_2m (eq. (88))."""
    return type1(x, None, 2 * m, h, +1)


def rhs(x, y, h, m, D):
    """b = D (F* y) with (F* y)_j = sum_n exp(2 pi i h <j, x_n>) y_n, j in J_m
    (eq. (rhs)); y may be (n,) or (nrhs, n)."""
    y = np.asarray(y, dtype=np.float64)
    if y.ndim == 1:
        return D * type1(x, y, m, h, +1)
    return np.stack([D * type1(x, yy, m, h, +1) for yy in y])


# --------------------------------------------------------------------------
# System matrix (eqs. (97), (223)) and the fast Toeplitz algorithm
# --------------------------------------------------------------------------

def toeplitz_apply(v, beta, m, dim):
    """(F*F) beta with (F*F)_{pl} = v_{j_p - j_l} (eq. (223)), O(M^2)."""
    v = np.ascontiguousarray(v, dtype=np.complex128)
    beta = np.ascontiguousarray(beta, dtype=np.complex128)
    out = np.empty_like(beta)
    rc = _load().or_toeplitz_apply(dim, m, _ptr(v.view(np.float64)), _ptr(beta.view(np.float64)),
                                   _ptr(out.view(np.float64)))
    if rc != 0:
        raise RuntimeError("or_toeplitz_apply failed")
    return out


def toeplitz_apply_fft(v, beta, m, dim):
    """The fast Toeplitz product exactly as the paper's algorithm states it
    (Sec. 3.2): FFT of v at size (4m+1)^d; zero-pad beta to (4m+1)^d; FFT;
    multiply; inverse FFT; keep indices 2m+1..4m+1 (1-based) per dimension."""
    W2 = 4 * m + 1
    vt = np.asarray(v, dtype=np.complex128).reshape((W2,) * dim)
    bt = np.zeros((W2,) * dim, dtype=np.complex128)
    bt[(slice(0, 2 * m + 1),) * dim] = np.asarray(beta).reshape((2 * m + 1,) * dim)
    conv = np.fft.ifftn(np.fft.fftn(vt) * np.fft.fftn(bt))
    return conv[(slice(2 * m, 4 * m + 1),) * dim].reshape(-1)


def system_apply(v, D, sigma2, beta, m, dim, fast=False):
    """(D F*F D + sigma^2 I) beta (eq. (97))."""
    tb = (toeplitz_apply_fft if fast else toeplitz_apply)(v, D * beta, m, dim)
    return D * tb + sigma2 * beta


def system_dense(v, D, sigma2, m, dim):
    """Dense M x M matrix of eq. (97)."""
    M = (2 * m + 1) ** dim
    v = np.ascontiguousarray(v, dtype=np.complex128)
    D = np.ascontiguousarray(D, dtype=np.float64)
    out = np.empty((M, M), dtype=np.complex128)
    rc = _load().or_system_dense(dim, m, _ptr(v.view(np.float64)), _ptr(D), float(sigma2),
                                 _ptr(out.view(np.float64)))
    if rc != 0:
        raise RuntimeError("or_system_dense failed")
    return out


def solve_dense(v, D, sigma2, b, m, dim):
    """Exact solution of eq. (be) by dense Hermitian Cholesky."""
    A = system_dense(v, D, sigma2, m, dim)
    c = scipy.linalg.cho_factor(A, lower=True, overwrite_a=True, check_finite=False)
    return scipy.linalg.cho_solve(c, b, check_finite=False)


def cg(apply, b, rho, maxiter, x0=None, precond=None):
    """Conjugate gradients on a Hermitian positive definite operator (step 4
    of the EFGP algorithm), stopping when ||r||/||b|| <= rho.  Inner products
    conjugate their first argument.  precond, if given, is a positive
    diagonal P (an array) or a Hermitian positive definite operator (a
    callable r -> P r), and the method is the preconditioned variant with
    z = P r; the stopping test uses the unpreconditioned residual.
    Returns (x, list of relative residuals, iterations)."""
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    r = b - apply(x) if x0 is not None else b.copy()
    bn = np.linalg.norm(b)
    pre = (lambda u: u) if precond is None else (precond if callable(precond) else (lambda u: precond * u))
    z = pre(r)
    p = z.copy()
    rz = np.vdot(r, z).real
    hist = [np.linalg.norm(r) / bn]
    it = 0
    while hist[-1] > rho and it < maxiter:
        q = apply(p)
        alpha = rz / np.vdot(p, q).real
        x = x + alpha * p
        r = r - alpha * q
        z = pre(r)
        rz_new = np.vdot(r, z).real
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
        hist.append(np.linalg.norm(r) / bn)
    return x, hist, it


def posterior_mean(beta, D, h, m, targets):
    """mu(x*) = sum_j D_j beta_j exp(-2 pi i h <j, x*>) (eq. (muws), step 6 of
    the EFGP algorithm), returned as (real part, imaginary part)."""
    mu = type2(targets, D * beta, m, h, -1)
    return mu.real.copy(), mu.imag.copy()


def prior_sample(xi, D, h, m, targets):
    """A draw from the GP prior in the equispaced Fourier basis (Sec. 6:
    evaluate the basis expansion with iid random coefficients by the type-2
    sum of step 6): f(t) = Re sum_j D_j xi_j exp(-2 pi i h <j, t>) with the
    real and imaginary parts of xi iid N(0,1), so that
    E f(t) f(t') = sum_j D_j^2 cos(2 pi h <j, t - t'>) = k~(t - t') (eq. (110))."""
    return type2(targets, np.asarray(D) * np.asarray(xi), m, h, -1).real.copy()


def posterior_variance(v, D, sigma2, m, dim, h, targets):
    """Posterior variance in weight space (Remark r:var: one solve per
    target): s(t) = sigma^2 phi(t)^H A^{-1} phi(t), phi_j(t) = D_j
    exp(+2 pi i h <j, t>), A = D T D + sigma^2 I the dense system matrix of
    eq. (223), solved by Cholesky."""
    t = _points(targets)
    J = freq_grid(m, dim).astype(np.float64)
    Phi = np.asarray(D)[:, None] * np.exp(2j * math.pi * h * (J @ t))   # (M, q)
    A = system_dense(v, D, sigma2, m, dim)
    c = np.linalg.cholesky(A)
    z = np.linalg.solve(c, Phi)
    return sigma2 * np.real(np.sum(np.conj(z) * z, axis=0))


# --------------------------------------------------------------------------
# Circulant preconditioner for the weight-space system (the open direction
# named in the conclusions: preconditioning Toeplitz-plus-diagonal systems).
# T. Chan's optimal circulant (SIAM J. Sci. Stat. Comput. 9, 1988): among all
# circulant matrices C, the one nearest to a matrix A in the Frobenius norm is
# F^H diag(lambda) F with lambda_s = f_s^H A f_s, the Rayleigh quotients of A
# at the Fourier vectors f_s(j) = exp(2 pi i <s, j> / K) / K^(d/2).
# --------------------------------------------------------------------------

def _fourier_matrix(K, dim):
    """F with rows f_s^H: F[s, j] = exp(-2 pi i <s, j> / K) / K^(d/2), s and j
    over {0..K-1}^d in C order."""
    k = np.arange(K)
    F1 = np.exp(-2j * math.pi * np.outer(k, k) / K) / math.sqrt(K)
    F = F1
    for _ in range(dim - 1):
        F = np.kron(F, F1)
    return F


def optimal_circulant_eigs(A, K, dim):
    """Eigenvalues of T. Chan's optimal circulant approximation of the
    K^d x K^d matrix A (indices on the periodic grid {0..K-1}^d, C order):
    lambda_s = f_s^H A f_s, written out densely."""
    F = _fourier_matrix(K, dim)
    return np.einsum("sj,jk,sk->s", F, np.asarray(A, dtype=np.complex128), F.conj(), optimize=True)


def circulant_matrix(lam, K, dim):
    """The circulant F^H diag(lam) F (dense), for checks."""
    F = _fourier_matrix(K, dim)
    return F.conj().T @ (np.asarray(lam)[:, None] * F)


def circulant_period(m):
    """Smallest K >= 2m+1 whose only prime factors are 2, 3 and 5 (the period
    of the circulant, so that its FFTs factor into small radices)."""
    K = 2 * m + 1
    while True:
        k = K
        for q in (2, 3, 5):
            while k % q == 0:
                k //= q
        if k == 1:
            return K
        K += 1


def scaled_system_extended(v, D, sigma2, n, m, dim, K):
    """E (+) I on the periodic grid {0..K-1}^d: E = J^(-1/2) A J^(-1/2) is the
    system matrix of eq. (97) scaled by its diagonal J = N D^2 + sigma^2
    (T_jj = v_0 = N), placed on the indices j + m in {0..2m}^d; the remaining
    K^d - M grid indices carry the identity (E has unit diagonal)."""
    W = 2 * m + 1
    A = system_dense(v, D, sigma2, m, dim)
    js = 1.0 / np.sqrt(n * np.asarray(D) ** 2 + sigma2)
    E = js[:, None] * A * js[None, :]
    grid = np.arange(K ** dim).reshape((K,) * dim)
    pos = grid[(slice(0, W),) * dim].reshape(-1)
    Ehat = np.eye(K ** dim, dtype=np.complex128)
    Ehat[np.ix_(pos, pos)] = E
    return Ehat


def circulant_precond_eigs(v, D, sigma2, n, m, dim, K=None):
    """Eigenvalues (real, K^d, C order) of the optimal circulant of E (+) I."""
    K = circulant_period(m) if K is None else K
    return optimal_circulant_eigs(scaled_system_extended(v, D, sigma2, n, m, dim, K), K, dim).real


def circulant_precond_apply(lam, D, sigma2, n, m, dim, r, K=None):
    """z = P r for the preconditioner P = J^(-1/2) R^T C^(-1) R J^(-1/2) of
    the weight-space system, with C = F^H diag(lam) F and R the restriction
    of the K^d grid to the M frequencies (zero padding for R^T).  P is
    Hermitian positive definite when lam > 0."""
    K = circulant_period(m) if K is None else K
    W = 2 * m + 1
    js = 1.0 / np.sqrt(n * np.asarray(D) ** 2 + sigma2)
    u = np.zeros((K,) * dim, dtype=np.complex128)
    u[(slice(0, W),) * dim] = (js * np.asarray(r)).reshape((W,) * dim)
    w = np.fft.ifftn(np.fft.fftn(u) / np.asarray(lam).reshape((K,) * dim))
    return js * w[(slice(0, W),) * dim].reshape(-1)


# --------------------------------------------------------------------------
# Function-space GP (eqs. (mu), (362)) for the exact reference
# --------------------------------------------------------------------------

def _pairwise_dist(a, b):
    a = _points(a)
    b = _points(b)
    d2 = np.zeros((a.shape[1], b.shape[1]))
    for l in range(a.shape[0]):
        d2 += (a[l][:, None] - b[l][None, :]) ** 2
    return np.sqrt(d2)


def gp_mean_dense(x, y, targets, sigma2, kfun):
    """mu(x*) = k_{x*}^T (K + sigma^2 I)^{-1} y by dense Cholesky (eqs. (mu),
    (362)).  kfun maps a (d, q) array of differences... here: a distance
    matrix to kernel values, or (for a non-radial kernel) receives the
    difference array via kfun.diff."""
    x = _points(x)
    targets = _points(targets)
    K = kfun(x, x)
    Ks = kfun(targets, x)
    K = K + sigma2 * np.eye(K.shape[0])
    c = scipy.linalg.cho_factor(K, lower=True)
    alpha = scipy.linalg.cho_solve(c, np.asarray(y, dtype=np.float64))
    return Ks @ alpha, alpha


def gp_variance_dense(x, targets, sigma2, kfun):
    """s(x*) = k(x*, x*) - k_{x*}^T (K + sigma^2 I)^{-1} k_{x*} by dense
    Cholesky (function-space posterior variance, Remark r:var)."""
    x = _points(x)
    targets = _points(targets)
    K = kfun(x, x) + sigma2 * np.eye(x.shape[1])
    Ks = kfun(targets, x)                                   # (q, N)
    kss = np.array([kfun(targets[:, i:i + 1], targets[:, i:i + 1])[0, 0] for i in range(targets.shape[1])])
    c = scipy.linalg.cho_factor(K, lower=True)
    return kss - np.sum(Ks * scipy.linalg.cho_solve(c, Ks.T).T, axis=1)


def exact_kfun(kernel, ell, nu=None, variance=1.0):
    return lambda a, b: kernel_value(_pairwise_dist(a, b), kernel, ell, nu, variance)


def ktilde_kfun(h, m, kernel, ell, nu=None, variance=1.0):
    def f(a, b):
        a = _points(a)
        b = _points(b)
        d = a.shape[0]
        diff = np.stack([(a[l][:, None] - b[l][None, :]).reshape(-1) for l in range(d)])
        return ktilde_value(diff, h, m, kernel, ell, nu, variance).reshape(a.shape[1], b.shape[1])
    return f


# --------------------------------------------------------------------------
# Whole method (the EFGP algorithm, steps 1-6)
# --------------------------------------------------------------------------

class Problem:
    """Setup quantities of the EFGP algorithm for one point set."""

    def __init__(self, dim, kernel, ell, nu, eps, variance=1.0, h=None, m=None):
        self.dim, self.kernel, self.ell, self.nu, self.eps = dim, kernel, ell, nu, eps
        self.variance = variance
        if h is None or m is None:
            h0, m0 = choose_h_m(kernel, dim, eps, ell, nu)
            h = h0 if h is None else h
            m = m0 if m is None else m
        self.h, self.m = float(h), int(m)
        self.M = (2 * self.m + 1) ** dim
        self.D = spectral_weights(self.h, self.m, dim, kernel, ell, nu, variance)


def setup(prob, x, y):
    """Steps 2-3: v on J_2m (eq. (88)) and b = D F* y (eq. (rhs))."""
    v = toeplitz_vector(x, prob.h, prob.m)
    b = rhs(x, y, prob.h, prob.m, prob.D)
    return v, b


# --------------------------------------------------------------------------
# Metrics (Sec. 5)
# --------------------------------------------------------------------------

def eepm(mu_hat, mu_ref):
    return float(np.sqrt(np.mean((np.asarray(mu_hat) - np.asarray(mu_ref)) ** 2)))


def rmse(mu_hat, y_test):
    return float(np.sqrt(np.mean((np.asarray(mu_hat) - np.asarray(y_test)) ** 2)))
