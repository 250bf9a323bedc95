// Device-side mixed-radix Stockham FFT on lines staged in LDS.
//
// A line of length n = prod(radix) is transformed in place-order (natural
// order in, natural order out) by ping-ponging between two LDS buffers.
// Radices 2, 3, 4, 5 are direct butterflies; 6, 8, 9, 10, 12, 15, 16 are
// computed in registers as two nested small DFTs, so a line takes fewer
// LDS passes and far fewer index computations per point.
// Stage s with radix R and span Ns (product of earlier radices) maps
// butterfly j (0 <= j < n/R) from inputs src[j + r n/R] (twiddled by
// w^(r (j mod Ns)) with w = exp(sign 2 pi i / (Ns R))) through an R-point DFT
// to outputs dst[(j - j mod Ns) R + (j mod Ns) + r Ns].
#pragma once

#include <type_traits>

#include "efgp_internal.h"

namespace efgp {

// The register DFTs and the Stockham butterfly are host-callable as well, so
// that a host build can check them against direct sums.
#define EFGP_HD __host__ __device__ __forceinline__

// a*b for |a|, |b| < 2^23: the full-rate 24-bit multiply on the device
EFGP_HD int mul24(int a, int b) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __mul24(a, b);
#else
    return a * b;
#endif
}

template <typename T> EFGP_HD cpx<T> mk(T a, T b) {
    cpx<T> z;
    z.x = a;
    z.y = b;
    return z;
}
#define EFGP_CPX_OPS(CT, RT)                                                                               \
    EFGP_HD CT cadd(CT a, CT b) { return CT{a.x + b.x, a.y + b.y}; }                  \
    EFGP_HD CT csub(CT a, CT b) { return CT{a.x - b.x, a.y - b.y}; }                  \
    EFGP_HD CT cmul(CT a, CT b) { return CT{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; } \
    EFGP_HD CT cscale(CT a, RT s) { return CT{a.x * s, a.y * s}; }
EFGP_CPX_OPS(float2, float)
EFGP_CPX_OPS(double2, double)
#undef EFGP_CPX_OPS
// multiply by sign*i
template <typename T, int SIGN> EFGP_HD cpx<T> mul_si(cpx<T> a) {
    return SIGN > 0 ? mk<T>(-a.y, a.x) : mk<T>(a.y, -a.x);
}

template <typename T, int SIGN>
EFGP_HD void dft2(cpx<T>* v) {
    cpx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <typename T, int SIGN>
EFGP_HD void dft4(cpx<T>* v) {
    cpx<T> s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    cpx<T> s13 = cadd(v[1], v[3]), d13 = mul_si<T, SIGN>(csub(v[1], v[3]));
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, d13);
    v[3] = csub(d02, d13);
}

template <typename T, int SIGN>
EFGP_HD void dft3(cpx<T>* v) {
    const T c = (T)-0.5, s = (T)0.86602540378443864676;  // cos, sin of 2 pi / 3
    cpx<T> t = cadd(v[1], v[2]), u = mul_si<T, SIGN>(csub(v[1], v[2]));
    cpx<T> a = mk<T>(v[0].x + c * t.x, v[0].y + c * t.y);
    v[0] = cadd(v[0], t);
    v[1] = mk<T>(a.x + s * u.x, a.y + s * u.y);
    v[2] = mk<T>(a.x - s * u.x, a.y - s * u.y);
}

template <typename T, int SIGN>
EFGP_HD void dft5(cpx<T>* v) {
    const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;  // cos 2pi/5, 4pi/5
    const T s1 = (T)0.95105651629515357212, s2 = (T)0.58778525229247312917;   // sin 2pi/5, 4pi/5
    cpx<T> t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    cpx<T> u1 = mul_si<T, SIGN>(csub(v[1], v[4])), u2 = mul_si<T, SIGN>(csub(v[2], v[3]));
    cpx<T> a = mk<T>(v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y);
    cpx<T> b = mk<T>(v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y);
    cpx<T> e = mk<T>(s1 * u1.x + s2 * u2.x, s1 * u1.y + s2 * u2.y);
    cpx<T> f = mk<T>(s2 * u1.x - s1 * u2.x, s2 * u1.y - s1 * u2.y);
    v[0] = cadd(v[0], cadd(t1, t2));
    v[1] = cadd(a, e);
    v[4] = csub(a, e);
    v[2] = cadd(b, f);
    v[3] = csub(b, f);
}

// cos and sin of 2 pi e / N, e < N, for the composite radices (values
// rounded to double from extended-precision evaluation)
template <int N> __host__ __device__ constexpr double root_cos(int e);
template <int N> __host__ __device__ constexpr double root_sin(int e);
template <> __host__ __device__ constexpr double root_cos<6>(int e) {
    constexpr double t[6] = {1.0, 0.5, -0.5, -1.0, -0.5, 0.5};
    return t[e];
}
template <> __host__ __device__ constexpr double root_sin<6>(int e) {
    constexpr double t[6] = {0.0, 0.8660254037844386, 0.8660254037844386, 0.0, -0.8660254037844386, -0.8660254037844386};
    return t[e];
}
template <> __host__ __device__ constexpr double root_cos<8>(int e) {
    constexpr double t[8] = {1.0, 0.7071067811865476, 0.0, -0.7071067811865476, -1.0, -0.7071067811865476, 0.0, 0.7071067811865476};
    return t[e];
}
template <> __host__ __device__ constexpr double root_sin<8>(int e) {
    constexpr double t[8] = {0.0, 0.7071067811865476, 1.0, 0.7071067811865476, 0.0, -0.7071067811865476, -1.0, -0.7071067811865476};
    return t[e];
}
template <> __host__ __device__ constexpr double root_cos<9>(int e) {
    constexpr double t[9] = {1.0, 0.766044443118978, 0.17364817766693036, -0.5, -0.9396926207859084, -0.9396926207859084, -0.5, 0.17364817766693036, 0.766044443118978};
    return t[e];
}
template <> __host__ __device__ constexpr double root_sin<9>(int e) {
    constexpr double t[9] = {0.0, 0.6427876096865394, 0.984807753012208, 0.8660254037844386, 0.3420201433256687, -0.3420201433256687, -0.8660254037844386, -0.984807753012208, -0.6427876096865394};
    return t[e];
}
template <> __host__ __device__ constexpr double root_cos<10>(int e) {
    constexpr double t[10] = {1.0, 0.8090169943749475, 0.30901699437494745, -0.30901699437494745, -0.8090169943749475, -1.0, -0.8090169943749475, -0.30901699437494745, 0.30901699437494745, 0.8090169943749475};
    return t[e];
}
template <> __host__ __device__ constexpr double root_sin<10>(int e) {
    constexpr double t[10] = {0.0, 0.5877852522924731, 0.9510565162951535, 0.9510565162951535, 0.5877852522924731, 0.0, -0.5877852522924731, -0.9510565162951535, -0.9510565162951535, -0.5877852522924731};
    return t[e];
}
template <> __host__ __device__ constexpr double root_cos<12>(int e) {
    constexpr double t[12] = {1.0, 0.8660254037844386, 0.5, 0.0, -0.5, -0.8660254037844386, -1.0, -0.8660254037844386, -0.5, 0.0, 0.5, 0.8660254037844386};
    return t[e];
}
template <> __host__ __device__ constexpr double root_sin<12>(int e) {
    constexpr double t[12] = {0.0, 0.5, 0.8660254037844386, 1.0, 0.8660254037844386, 0.5, 0.0, -0.5, -0.8660254037844386, -1.0, -0.8660254037844386, -0.5};
    return t[e];
}
template <> __host__ __device__ constexpr double root_cos<15>(int e) {
    constexpr double t[15] = {1.0, 0.9135454576426009, 0.6691306063588582, 0.30901699437494745, -0.10452846326765347, -0.5, -0.8090169943749475, -0.9781476007338057, -0.9781476007338057, -0.8090169943749475, -0.5, -0.10452846326765347, 0.30901699437494745, 0.6691306063588582, 0.9135454576426009};
    return t[e];
}
template <> __host__ __device__ constexpr double root_sin<15>(int e) {
    constexpr double t[15] = {0.0, 0.4067366430758002, 0.7431448254773942, 0.9510565162951535, 0.9945218953682733, 0.8660254037844386, 0.5877852522924731, 0.20791169081775934, -0.20791169081775934, -0.5877852522924731, -0.8660254037844386, -0.9945218953682733, -0.9510565162951535, -0.7431448254773942, -0.4067366430758002};
    return t[e];
}
template <> __host__ __device__ constexpr double root_cos<16>(int e) {
    constexpr double t[16] = {1.0, 0.9238795325112867, 0.7071067811865476, 0.3826834323650898, 0.0, -0.3826834323650898, -0.7071067811865476, -0.9238795325112867, -1.0, -0.9238795325112867, -0.7071067811865476, -0.3826834323650898, 0.0, 0.3826834323650898, 0.7071067811865476, 0.9238795325112867};
    return t[e];
}
template <> __host__ __device__ constexpr double root_sin<16>(int e) {
    constexpr double t[16] = {0.0, 0.3826834323650898, 0.7071067811865476, 0.9238795325112867, 1.0, 0.9238795325112867, 0.7071067811865476, 0.3826834323650898, 0.0, -0.3826834323650898, -0.7071067811865476, -0.9238795325112867, -1.0, -0.9238795325112867, -0.7071067811865476, -0.3826834323650898};
    return t[e];
}

template <typename T, int SIGN, int R> EFGP_HD void dft_r(cpx<T>* v);

// multiply by w^e, w = exp(SIGN 2 pi i / N), e a compile-time constant
// after unrolling (1, -1 and +-i without multiplications)
template <typename T, int SIGN, int N>
EFGP_HD cpx<T> root_mul(cpx<T> a, int e) {
    if (e == 0) return a;
    if (2 * e == N) return mk<T>(-a.x, -a.y);
    if (4 * e == N) return mul_si<T, SIGN>(a);
    if (4 * e == 3 * N) return mul_si<T, -SIGN>(a);
    return cmul(a, mk<T>((T)root_cos<N>(e), (T)(SIGN * root_sin<N>(e))));
}

// N = N1 N2 point DFT in registers (Cooley-Tukey, natural order in and
// out): for each n2 an N1-point DFT of v[N2 n1 + n2], twiddled by
// w_N^(n2 k1); then for each k1 an N2-point DFT over n2 gives
// X[k1 + N1 k2].
template <typename T, int SIGN, int N1, int N2>
EFGP_HD void dft_ct(cpx<T>* v) {
    constexpr int N = N1 * N2;
    cpx<T> y[N];
#pragma unroll
    for (int n2 = 0; n2 < N2; n2++) {
        cpx<T> t[N1];
#pragma unroll
        for (int n1 = 0; n1 < N1; n1++) t[n1] = v[N2 * n1 + n2];
        dft_r<T, SIGN, N1>(t);
#pragma unroll
        for (int k1 = 0; k1 < N1; k1++) y[n2 * N1 + k1] = root_mul<T, SIGN, N>(t[k1], n2 * k1);
    }
#pragma unroll
    for (int k1 = 0; k1 < N1; k1++) {
        cpx<T> t[N2];
#pragma unroll
        for (int n2 = 0; n2 < N2; n2++) t[n2] = y[n2 * N1 + k1];
        dft_r<T, SIGN, N2>(t);
#pragma unroll
        for (int k2 = 0; k2 < N2; k2++) v[k1 + N1 * k2] = t[k2];
    }
}

// the R-point DFT of the stage radices
template <typename T, int SIGN, int R>
EFGP_HD void dft_r(cpx<T>* v) {
    if constexpr (R == 2) dft2<T, SIGN>(v);
    else if constexpr (R == 3) dft3<T, SIGN>(v);
    else if constexpr (R == 4) dft4<T, SIGN>(v);
    else if constexpr (R == 5) dft5<T, SIGN>(v);
    else if constexpr (R == 6) dft_ct<T, SIGN, 3, 2>(v);
    else if constexpr (R == 8) dft_ct<T, SIGN, 4, 2>(v);
    else if constexpr (R == 9) dft_ct<T, SIGN, 3, 3>(v);
    else if constexpr (R == 10) dft_ct<T, SIGN, 5, 2>(v);
    else if constexpr (R == 12) dft_ct<T, SIGN, 4, 3>(v);
    else if constexpr (R == 15) dft_ct<T, SIGN, 5, 3>(v);
    else {
        static_assert(R == 16, "unsupported radix");
        dft_ct<T, SIGN, 4, 4>(v);
    }
}

// radix of stage s from the packed code (4 bits a stage; 0 stands for 16)
EFGP_HD int stage_radix(unsigned code, int s) {
    const int r = (int)((code >> (4 * s)) & 15u);
    return r == 0 ? 16 : r;
}

// call(integral_constant<R>) for the stage radix R (a uniform switch).
// Radices above MAXR are not compiled in: a kernel whose register budget
// cannot hold their butterflies takes stage plans of radices <= MAXR
// (fft_shape's maxr), which the host builds for it.
template <int MAXR, typename F>
__device__ __forceinline__ void radix_switch(int R, F&& call) {
    using std::integral_constant;
    switch (R) {
        case 2: call(integral_constant<int, 2>{}); break;
        case 3: call(integral_constant<int, 3>{}); break;
        case 4: call(integral_constant<int, 4>{}); break;
        case 5: call(integral_constant<int, 5>{}); break;
        case 6: if constexpr (MAXR >= 6) call(integral_constant<int, 6>{}); break;
        case 8: if constexpr (MAXR >= 8) call(integral_constant<int, 8>{}); break;
        case 9: if constexpr (MAXR >= 9) call(integral_constant<int, 9>{}); break;
        case 10: if constexpr (MAXR >= 10) call(integral_constant<int, 10>{}); break;
        case 12: if constexpr (MAXR >= 12) call(integral_constant<int, 12>{}); break;
        case 15: if constexpr (MAXR >= 15) call(integral_constant<int, 15>{}); break;
        default: if constexpr (MAXR >= 16) call(integral_constant<int, 16>{}); break;
    }
}

// floor(a / d) for 0 <= a < 2^22 and 1 <= d < 2^22, with rd = 1/d in float
// (a per-stage constant): the float quotient is within 2^-22 (relative) of
// a / d < 2^22, so within one of the floor, and one correction step each
// way makes it exact.  *rem = a - d floor(a / d).  Branch-free, with a
// 24-bit product (q d < a + d < 2^23); a runtime integer division costs
// about three times as many VALU instructions.
EFGP_HD int udiv22(int a, int d, float rd, int* rem) {
    int q = (int)((float)a * rd);
    int r = a - mul24(q, d);
    const bool lo = r < 0, hi = r >= d;
    q += (hi ? 1 : 0) - (lo ? 1 : 0);
    r += (lo ? d : 0) - (hi ? d : 0);
    *rem = r;
    return q;
}

// One radix-R butterfly of a Stockham stage: j < nb = n/R, k = j mod Ns,
// twstep = n / (Ns R).
template <typename T, int SIGN, int R>
EFGP_HD void stockham_bfly(const cpx<T>* __restrict__ src, cpx<T>* __restrict__ dst,
                                              int nb, int Ns, int j, int k, int twstep,
                                              const cpx<T>* __restrict__ tw) {
    cpx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; r++) v[r] = src[j + r * nb];
    if (Ns > 1) {
        const int kt = mul24(k, twstep);   // k twstep < n
#pragma unroll
        for (int r = 1; r < R; r++) {
            cpx<T> t = tw[r * kt];
            if (SIGN > 0) t.y = -t.y;
            v[r] = cmul(v[r], t);
        }
    }
    dft_r<T, SIGN, R>(v);
    const int d0 = (j - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; r++) dst[d0 + r * Ns] = v[r];
}

// Transform nl lines (line l at a + l*ld) of length f.s.n held in LDS.  All
// threads of the block must call this.  Returns the buffer holding the
// result (a or b).  Ends with a barrier.  The plan's radices are <= MAXR.
template <typename T, int SIGN, int MAXR = 16>
__device__ cpx<T>* fft_lds(cpx<T>* a, cpx<T>* b, int ld, int nl, const FftDev<T>& f) {
    const int n = f.s.n;
    int Ns = 1;
    for (int s = 0; s < f.s.nst; s++) {
        const int R = stage_radix(f.s.code, s);
        const int nb = n / R;
        const int total = nb * nl;
        const int twstep = n / (Ns * R);
        const float rnb = 1.0f / (float)nb, rns = 1.0f / (float)Ns;
        for (int t = threadIdx.x; t < total; t += blockDim.x) {
            int j = t, k;
            const int line = nl == 1 ? 0 : udiv22(t, nb, rnb, &j);
            (void)udiv22(j, Ns, rns, &k);
            const cpx<T>* src = a + __mul24(line, ld);
            cpx<T>* dst = b + __mul24(line, ld);
            radix_switch<MAXR>(R, [&](auto rc) {
                stockham_bfly<T, SIGN, decltype(rc)::value>(src, dst, nb, Ns, j, k, twstep, f.tw);
            });
        }
        __syncthreads();
        cpx<T>* t = a;
        a = b;
        b = t;
        Ns *= R;
    }
    return a;
}

// ---------------------------------------------- long lines: one LDS buffer
// Lines too long for two LDS buffers (double lines of more than ~1500 points
// in 48 KB) are transformed in one buffer: each stage reads every input of
// the thread's butterflies into registers, computes them, waits for the
// whole block, then writes the outputs to their autosorted places.  A
// thread takes at most kLongB(R) butterflies per stage, so the block must
// satisfy nl * n <= kLongMax with blockDim.x == kLongThreads.
constexpr int kLongThreads = 1024;
constexpr int kLongMax = 8192;   // points per block (all lines together)
template <int R> constexpr int kLongB() { return (kLongMax / R + kLongThreads - 1) / kLongThreads; }

template <typename T, int SIGN, int R>
__device__ __forceinline__ void stage_1buf(cpx<T>* a, int ld, int nl, int n, int Ns, const cpx<T>* __restrict__ tw) {
    constexpr int MB = kLongB<R>();
    const int nb = n / R;
    const int total = nb * nl;
    const int twstep = n / (Ns * R);
    const float rnb = 1.0f / (float)nb, rns = 1.0f / (float)Ns;
    cpx<T> v[MB][R];
    int d0[MB];
#pragma unroll
    for (int q = 0; q < MB; q++) {
        const int t = threadIdx.x + q * kLongThreads;
        d0[q] = -1;
        if (t < total) {
            int j = t, k;
            const int line = nl == 1 ? 0 : udiv22(t, nb, rnb, &j);
            (void)udiv22(j, Ns, rns, &k);
            const cpx<T>* src = a + __mul24(line, ld);
#pragma unroll
            for (int r = 0; r < R; r++) v[q][r] = src[j + r * nb];
            if (Ns > 1) {
                const int kt = __mul24(k, twstep);
#pragma unroll
                for (int r = 1; r < R; r++) {
                    cpx<T> w = tw[r * kt];
                    if (SIGN > 0) w.y = -w.y;
                    v[q][r] = cmul(v[q][r], w);
                }
            }
            dft_r<T, SIGN, R>(v[q]);
            d0[q] = __mul24(line, ld) + (j - k) * R + k;
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MB; q++) {
        if (d0[q] >= 0) {
#pragma unroll
            for (int r = 0; r < R; r++) a[d0[q] + r * Ns] = v[q][r];
        }
    }
    __syncthreads();
}

// Transform nl lines (line l at a + l*ld) of length f.s.n in place in one
// LDS buffer; twiddles are read through f.tw (global memory is fine: the
// table is small and stays in cache).  Requires blockDim.x == kLongThreads
// and nl * n <= kLongMax.  All threads of the block must call this; the
// caller's writes to the lines must be complete (barrier) before the call.
// Ends with a barrier.  The plan's radices are <= MAXR (by default 5: the
// 1024-thread kernels hold every butterfly of a stage across a barrier).
template <typename T, int SIGN, int MAXR = 5>
__device__ void fft_lds_1(cpx<T>* a, int ld, int nl, const FftDev<T>& f) {
    const int n = f.s.n;
    int Ns = 1;
    for (int s = 0; s < f.s.nst; s++) {
        const int R = stage_radix(f.s.code, s);
        radix_switch<MAXR>(R, [&](auto rc) { stage_1buf<T, SIGN, decltype(rc)::value>(a, ld, nl, n, Ns, f.tw); });
        Ns *= R;
    }
}

// ------------------------------------------------------- block reductions
__device__ __forceinline__ double warp_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the block; result valid in thread 0.  red must hold >= 16 doubles.
__device__ __forceinline__ double block_sum(double v, double* red) {
    v = warp_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int i = 0; i < nw; i++) s += red[i];
    }
    __syncthreads();
    return s;
}

}  // namespace efgp
