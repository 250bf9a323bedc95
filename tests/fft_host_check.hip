// Host build of the LDS FFT's stage arithmetic (the register DFTs of every
// radix and the Stockham butterfly, driven stage by stage as the device
// kernels drive them, with the library's own stage plans) against direct
// DFT sums.  Exits non-zero on the first length whose error is too large.
#include <complex>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "fft_device.h"

using namespace efgp;

template <typename T, int SIGN, int R>
static void stage(const std::vector<cpx<T>>& a, std::vector<cpx<T>>& b, int n, int Ns, const std::vector<cpx<T>>& tw) {
    const int nb = n / R, twstep = n / (Ns * R);
    for (int j = 0; j < nb; j++) stockham_bfly<T, SIGN, R>(a.data(), b.data(), nb, Ns, j, j % Ns, twstep, tw.data());
}

template <typename T, int SIGN>
static void fft_host(std::vector<cpx<T>>& a, const FftShape& s, const std::vector<cpx<T>>& tw) {
    std::vector<cpx<T>> b(a.size());
    int Ns = 1;
    for (int st = 0; st < s.nst; st++) {
        const int R = stage_radix(s.code, st);
        switch (R) {
            case 2: stage<T, SIGN, 2>(a, b, s.n, Ns, tw); break;
            case 3: stage<T, SIGN, 3>(a, b, s.n, Ns, tw); break;
            case 4: stage<T, SIGN, 4>(a, b, s.n, Ns, tw); break;
            case 5: stage<T, SIGN, 5>(a, b, s.n, Ns, tw); break;
            case 6: stage<T, SIGN, 6>(a, b, s.n, Ns, tw); break;
            case 8: stage<T, SIGN, 8>(a, b, s.n, Ns, tw); break;
            case 9: stage<T, SIGN, 9>(a, b, s.n, Ns, tw); break;
            case 10: stage<T, SIGN, 10>(a, b, s.n, Ns, tw); break;
            case 12: stage<T, SIGN, 12>(a, b, s.n, Ns, tw); break;
            case 15: stage<T, SIGN, 15>(a, b, s.n, Ns, tw); break;
            case 16: stage<T, SIGN, 16>(a, b, s.n, Ns, tw); break;
            default: std::printf("radix %d not expected\n", R); std::exit(2);
        }
        a.swap(b);
        Ns *= R;
    }
}

// relative error (max over the checked outputs / max |X|) of one transform
template <typename T, int SIGN>
static double check(int n, int maxr) {
    const FftShape s = fft_shape(n, maxr);
    if (max_radix(s) > maxr) { std::printf("n %d: radix above %d\n", n, maxr); std::exit(2); }
    int prod = 1;
    for (int i = 0; i < s.nst; i++) prod *= s.radix[i];
    if (prod != n || s.nst > 4 + (maxr < 16 ? 4 : 0)) { std::printf("n %d: bad plan\n", n); std::exit(2); }
    std::vector<cpx<T>> tw(n), a(n);
    for (int k = 0; k < n; k++) tw[k] = mk<T>((T)std::cos(-2 * M_PI * k / n), (T)std::sin(-2 * M_PI * k / n));
    std::mt19937 g(n * 3 + maxr);
    std::uniform_real_distribution<double> u(-1, 1);
    std::vector<std::complex<double>> x(n);
    for (int i = 0; i < n; i++) {
        a[i] = mk<T>((T)u(g), (T)u(g));
        x[i] = {(double)a[i].x, (double)a[i].y};
    }
    fft_host<T, SIGN>(a, s, tw);
    const int nk = n <= 256 ? n : 16;
    double err = 0, nrm = 0;
    for (int q = 0; q < nk; q++) {
        const int k = n <= 256 ? q : (int)((long long)q * 7919 % n);
        std::complex<double> sum = 0;
        for (int m = 0; m < n; m++) sum += x[m] * std::polar(1.0, SIGN * 2 * M_PI * (double)((long long)m * k % n) / n);
        err = std::max(err, std::abs(sum - std::complex<double>(a[k].x, a[k].y)));
        nrm = std::max(nrm, std::abs(sum));
    }
    return err / nrm;
}

// udiv22 (floor division by a float reciprocal with one correction each
// way) against integer division for every a < 2^22 and a spread of divisors
static bool check_udiv22() {
    std::vector<int> ds;
    for (int d = 1; d <= 64; d++) ds.push_back(d);
    for (int d = 65; d < (1 << 22); d = d * 5 / 4 + 1) ds.push_back(d);
    for (int d : {100, 108, 125, 135, 216, 1440, 2880, 4096, 8192, (1 << 22) - 1}) ds.push_back(d);
    for (int d : ds) {
        const float rd = 1.0f / (float)d;
        for (int a = 0; a < (1 << 22); a++) {
            int r;
            const int q = udiv22(a, d, rd, &r);
            if (q != a / d || r != a % d) {
                std::printf("FAIL udiv22 a %d d %d: %d %d\n", a, d, q, r);
                return false;
            }
        }
    }
    std::printf("udiv22 exact for a < 2^22 and %zu divisors\n", ds.size());
    return true;
}

int main() {
    if (!check_udiv22()) return 1;
    std::vector<int> ns;
    for (int n = 2; n <= 1500; n++)
        if (is_smooth235(n)) ns.push_back(n);
    for (int n : {1728, 2048, 2880, 4096, 6000, 8192}) ns.push_back(n);
    double w64 = 0, w32 = 0;
    for (int n : ns) {
        for (int maxr : {16, 5}) {
            const double e = std::max(check<double, -1>(n, maxr), check<double, 1>(n, maxr));
            w64 = std::max(w64, e);
            if (e > 1e-13) { std::printf("FAIL double n %d maxr %d: %.2e\n", n, maxr, e); return 1; }
        }
        const double f = std::max(check<float, -1>(n, 16), check<float, 1>(n, 16));
        w32 = std::max(w32, f);
        if (f > 2e-6) { std::printf("FAIL float n %d: %.2e\n", n, f); return 1; }
    }
    std::printf("ok: %zu lengths, both directions; worst relative error %.2e (double), %.2e (float)\n", ns.size(),
                w64, w32);
    return 0;
}
