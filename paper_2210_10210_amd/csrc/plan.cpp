// Host-side plan computations: the EFGP parameter rules, the kernels'
// spectral densities, the exponential-of-semicircle (ES) spreading kernel
// and its Fourier transform, and FFT size factorisation.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "efgp_internal.h"

namespace efgp {

static const double kPi = 3.14159265358979323846;

// Gauss-Legendre nodes/weights on [-1,1] by Newton iteration on P_n.
static void gauss_legendre_compute(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; i++) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
        double pp = 0.0;
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; k++) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            pp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / pp;
            z -= dz;
            if (std::fabs(dz) <= 1e-15 * std::fabs(z) + 1e-300) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; k++) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        pp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
}

// cached per order: every setup needs the same few rules
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    static std::mutex mu;
    static std::map<int, std::pair<std::vector<double>, std::vector<double>>> cache;
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(n);
    if (it == cache.end()) {
        std::vector<double> a, b;
        gauss_legendre_compute(n, a, b);
        it = cache.emplace(n, std::make_pair(std::move(a), std::move(b))).first;
    }
    x = it->second.first;
    w = it->second.second;
}

// Unit-variance kernel at distance r: SE (Gker) or Matern (Cker).
static double kernel_value(int kernel, double ell, double nu, double r) {
    if (kernel == EFGP_KERNEL_SE) return std::exp(-r * r / (2.0 * ell * ell));
    double a = std::sqrt(2.0 * nu) * r / ell;
    if (a == 0.0) return 1.0;
    if (nu == 0.5) return std::exp(-a);
    if (nu == 1.5) return (1.0 + a) * std::exp(-a);
    if (nu == 2.5) return (1.0 + a + a * a / 3.0) * std::exp(-a);
    if (a > 700.0) return 0.0;
    return std::pow(2.0, 1.0 - nu) / std::tgamma(nu) * std::pow(a, nu) * std::cyl_bessel_k(nu, a);
}

// ||k||_{L2([-1,1]^d)}: tensor Gauss-Legendre on [0,1]^d times 2^d (the
// integrand is even in every coordinate; integrating each half-axis
// separately keeps the cusp of k at r = 0 at a panel end).  Results are
// cached per (kernel, ell, nu, d): repeated setups skip the quadrature.
static double kernel_l2_norm_quad(int kernel, double ell, double nu, int dim) {
    const int nq = dim == 3 ? 40 : 64;
    std::vector<double> g, gw;
    gauss_legendre(nq, g, gw);
    std::vector<double> t(nq), tw(nq);
    for (int i = 0; i < nq; i++) {
        t[i] = (g[i] + 1.0) / 2.0;
        tw[i] = gw[i] / 2.0;
    }
    double s = 0.0;
    if (dim == 1) {
        for (int i = 0; i < nq; i++) {
            const double k = kernel_value(kernel, ell, nu, t[i]);
            s += tw[i] * k * k;
        }
    } else if (dim == 2) {
        for (int i = 0; i < nq; i++)
            for (int j = 0; j < nq; j++) {
                const double k = kernel_value(kernel, ell, nu, std::sqrt(t[i] * t[i] + t[j] * t[j]));
                s += tw[i] * tw[j] * k * k;
            }
    } else {
        for (int i = 0; i < nq; i++)
            for (int j = 0; j < nq; j++)
                for (int l = 0; l < nq; l++) {
                    const double k = kernel_value(kernel, ell, nu, std::sqrt(t[i] * t[i] + t[j] * t[j] + t[l] * t[l]));
                    s += tw[i] * tw[j] * tw[l] * k * k;
                }
    }
    return std::sqrt(std::ldexp(s, dim));
}

double kernel_l2_norm(int kernel, double ell, double nu, int dim) {
    static std::mutex mu;
    static std::map<std::vector<double>, double> cache;
    const std::vector<double> key = {(double)kernel, ell, nu, (double)dim};
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    const double v = kernel_l2_norm_quad(kernel, ell, nu, dim);
    std::lock_guard<std::mutex> g(mu);
    if (cache.size() > 4096) cache.clear();
    cache[key] = v;
    return v;
}

void choose_h_m(int kernel, int d, double eps, double ell, double nu, double* h, int* m,
                double* kl2) {
    *kl2 = 0.0;
    if (kernel == EFGP_KERNEL_SE) {
        // Sec. 4.2: aliasing and truncation each bounded by eps/2.
        *h = 1.0 / (1.0 + ell * std::sqrt(2.0 * std::log(4.0 * d * std::pow(3.0, d) / eps)));
        *m = (int)std::ceil(std::sqrt(0.5 * std::log(std::pow(4.0, d + 1) * d / eps)) /
                            (kPi * ell * *h));
        return;
    }
    if (nu <= 2.5) {
        // eq. (maternheur): relative L2 precision eps, eps~ = eps ||k||.
        *kl2 = kernel_l2_norm(kernel, ell, nu, d);
        double et = eps * *kl2;
        *h = 1.0 / (1.0 + 0.85 * (ell / std::sqrt(nu)) * std::log(1.0 / et));
        double base = std::pow(kPi, nu + d / 2.0) * std::pow(ell, 2.0 * nu) * et / 0.15;
        *m = (int)std::ceil(std::pow(base, -1.0 / (2.0 * nu + d / 2.0)) / *h);
        return;
    }
    // eq. (maternhm): uniform error eps.
    *h = 1.0 / (1.0 + ell * std::sqrt(2.0 * d / nu) * std::log(d * std::pow(3.0, d) / eps));
    *m = (int)std::ceil(std::pow(d * std::pow(5.0, d - 1) / (std::pow(kPi, d / 2.0) * eps),
                                 1.0 / (2.0 * nu)) *
                        1.6 * std::sqrt(nu) / (kPi * *h * ell));
}

// Spectral density in the convention khat(xi) = int k(x) e^{-2 pi i xi.x} dx,
// as a function of |xi|^2 with the xi-independent factors evaluated once.
struct KernelHat {
    int kernel, d;
    double variance, ell, nu, logc = 0.0;
    explicit KernelHat(const Plan& P) : kernel(P.kernel), d(P.dim), variance(P.variance), ell(P.ell), nu(P.nu) {
        if (kernel != EFGP_KERNEL_SE)
            logc = d * std::log(2.0) + 0.5 * d * std::log(kPi) + std::lgamma(nu + d / 2.0) +
                   nu * std::log(2.0 * nu) - std::lgamma(nu) - 2.0 * nu * std::log(ell);
    }
    double operator()(double xi2) const {
        if (kernel == EFGP_KERNEL_SE)
            return variance * std::pow(2.0 * kPi * ell * ell, d / 2.0) *
                   std::exp(-2.0 * kPi * kPi * ell * ell * xi2);
        const double base = 2.0 * nu / (ell * ell) + 4.0 * kPi * kPi * xi2;
        return variance * std::exp(logc - (nu + d / 2.0) * std::log(base));
    }
};

double kernel_hat(const Plan& P, double xi) { return KernelHat(P)(xi * xi); }

// D_j = sqrt(h^d khat(h |j|)) for j in J_m, C order (eq. (117)); khat
// depends on |j|^2 only, so each distinct |j|^2 is evaluated once.
std::vector<double> spectral_weights(const Plan& P) {
    const KernelHat kh(P);
    const int W = 2 * P.m + 1;
    const double hd = std::pow(P.h, P.dim);
    std::vector<double> byj2((size_t)P.dim * P.m * P.m + 1, -1.0);
    std::vector<double> D((size_t)P.M);
    for (int64_t idx = 0; idx < P.M; idx++) {
        int64_t rem = idx, jn2 = 0;
        for (int l = 0; l < P.dim; l++) {
            const int64_t j = rem % W - P.m;
            rem /= W;
            jn2 += j * j;
        }
        double& v = byj2[(size_t)jn2];
        if (v < 0.0) v = std::sqrt(hd * kh(P.h * P.h * (double)jn2));
        D[idx] = v;
    }
    return D;
}

// ES kernel phi(z) = exp(beta (sqrt(1 - z^2) - 1)) on |z| <= 1 (Barnett,
// Magland, af Klinteberg 2019): width w = ceil(log10(1/tol)) + 1 grid cells
// and beta = 2.30 w for upsampling factor 2.
void es_params(double tol, int* w, double* beta) {
    int ww = (int)std::ceil(std::log10(1.0 / tol)) + 1;
    ww = std::max(2, std::min(16, ww));
    *w = ww;
    *beta = 2.30 * ww;
}

// psihat(k) = int phi(t / (w/2)) e^{i k (2 pi / nfine) t} dt
//           = w int_0^1 phi(z) cos(k (2 pi / nfine) (w/2) z) dz,
// by Gauss-Legendre quadrature; returns 1/psihat for k = -K..K.
std::vector<double> es_deconv_table(int w, double beta, int nfine, int K) {
    const int nq = 200;
    std::vector<double> g, gw;
    gauss_legendre(nq, g, gw);
    std::vector<double> z(nq), f(nq);
    for (int i = 0; i < nq; i++) {
        z[i] = (g[i] + 1.0) / 2.0;
        f[i] = gw[i] / 2.0 * std::exp(beta * (std::sqrt(1.0 - z[i] * z[i]) - 1.0));
    }
    std::vector<double> out(2 * K + 1);
    const double a = 2.0 * kPi / nfine * (w / 2.0);
    for (int k = -K; k <= K; k++) {
        double s = 0.0;
        for (int i = 0; i < nq; i++) s += f[i] * std::cos(k * a * z[i]);
        out[k + K] = 1.0 / (w * s);
    }
    return out;
}

bool is_smooth235(int n) {
    if (n < 1) return false;
    for (int p : {2, 3, 5})
        while (n % p == 0) n /= p;
    return n == 1;
}

int next_smooth235(int n) {
    while (!is_smooth235(n)) n++;
    return n;
}

FftShape fft_shape(int n, int maxr) {
    FftShape s;
    s.n = n;
    int k = n;
    // the largest radix that divides what is left, stage by stage: fewer,
    // larger stages (each a register DFT) mean fewer LDS passes
    static const int kRadices[] = {16, 15, 12, 10, 9, 8, 6, 5, 4, 3, 2};
    while (k > 1) {
        int r = 0;
        for (int c : kRadices)
            if (c <= maxr && k % c == 0) { r = c; break; }
        if (r == 0 || s.nst >= 8) throw StatusError{EFGP_ETOOLARGE, "FFT length is not a product of 2, 3, 5 in 8 stages"};
        s.radix[s.nst++] = r;
        k /= r;
    }
    for (int i = 0; i < s.nst; i++) s.code |= (unsigned)(s.radix[i] & 15) << (4 * i);   // 16 -> 0
    return s;
}

int max_radix(const FftShape& s) {
    int r = 0;
    for (int i = 0; i < s.nst; i++) r = std::max(r, s.radix[i]);
    return r;
}

void* dalloc(Plan& P, size_t bytes) {
    void* ptr = pool_alloc(bytes);
    P.allocs.push_back({ptr, bytes});
    return ptr;
}

void* palloc(Plan& P, size_t bytes) {
    void* ptr = pinned_alloc(bytes);
    P.pinned.push_back({ptr, bytes});
    return ptr;
}

void upload_async(Plan& P, void* dst, const void* src, size_t bytes, hipStream_t s) {
    if (bytes == 0) return;
    void* st = palloc(P, bytes);
    std::memcpy(st, src, bytes);
    EFGP_HIP(hipMemcpyAsync(dst, st, bytes, hipMemcpyHostToDevice, s));
}

namespace {
struct Chunk {
    void* ptr;
    size_t size;
    size_t used;
};
std::mutex g_scratch_mu;
std::map<int, std::vector<Chunk>> g_chunks;  // per device
}  // namespace

Scratch::Scratch() {
    g_scratch_mu.lock();
    dev_ = 0;
    (void)hipGetDevice(&dev_);
}

Scratch::~Scratch() {
    for (Chunk& c : g_chunks[dev_]) c.used = 0;
    g_scratch_mu.unlock();
}

void* Scratch::take(size_t bytes) {
    bytes = (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
    std::vector<Chunk>& cs = g_chunks[dev_];
    for (Chunk& c : cs) {
        if (c.size - c.used >= bytes) {
            void* p = static_cast<char*>(c.ptr) + c.used;
            c.used += bytes;
            return p;
        }
    }
    // new chunk: at least 64 MiB so small requests share one
    const size_t sz = std::max<size_t>(bytes, (size_t)64 << 20);
    void* ptr = nullptr;
    if (hipMalloc(&ptr, sz) != hipSuccess) {
        (void)hipGetLastError();
        // drop idle chunks and retry once
        std::vector<Chunk> keep;
        for (Chunk& c : cs) {
            if (c.used == 0) (void)hipFree(c.ptr);
            else keep.push_back(c);
        }
        cs.swap(keep);
        if (hipMalloc(&ptr, sz) != hipSuccess) {
            (void)hipGetLastError();
            throw StatusError{EFGP_ENOMEM, "device allocation failed (setup scratch)"};
        }
    }
    cs.push_back(Chunk{ptr, sz, bytes});
    return ptr;
}

void release_scratch() {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto& kv : g_chunks) {
        (void)hipSetDevice(kv.first);
        for (Chunk& c : kv.second) (void)hipFree(c.ptr);
        kv.second.clear();
    }
    (void)hipSetDevice(cur);
}

template <typename T>
static std::vector<cpx<T>> twiddle_table(int n) {
    std::vector<cpx<T>> h(n);
    for (int k = 0; k < n; k++) {
        double a = -2.0 * kPi * (double)k / (double)n;
        h[k].x = (T)std::cos(a);
        h[k].y = (T)std::sin(a);
    }
    return h;
}

template <typename T>
void upload_twiddles(Plan& P, int n, void** out, hipStream_t s) {
    const std::vector<cpx<T>> h = twiddle_table<T>(n);
    void* d = dalloc(P, sizeof(cpx<T>) * n);
    upload_async(P, d, h.data(), sizeof(cpx<T>) * n, s);
    *out = d;
}

template <typename T>
void upload_twiddles_to(Plan& P, int n, void* dst, hipStream_t s) {
    const std::vector<cpx<T>> h = twiddle_table<T>(n);
    upload_async(P, dst, h.data(), sizeof(cpx<T>) * n, s);
}
template void upload_twiddles<float>(Plan&, int, void**, hipStream_t);
template void upload_twiddles<double>(Plan&, int, void**, hipStream_t);
template void upload_twiddles_to<float>(Plan&, int, void*, hipStream_t);
template void upload_twiddles_to<double>(Plan&, int, void*, hipStream_t);

}  // namespace efgp
