// Evaluation stage of EFGP (step 6 of the EFGP algorithm): the posterior
// mean mu(t) = Re sum_{j in J_m} D_j beta_j exp(-2 pi i h <j, t>) at q
// targets by a type-2 NUFFT:
//   1. c_j = D_j beta_j / psihat(j) placed at grid index j mod nf2
//      (nf2 >= 2(2m+1), the ES kernel's Fourier transform deconvolved),
//   2. FFT with sign - along every axis,
//   3. interpolation: mu(t) = sum_g Re G_g phi((g - u)/(w/2)), u = t h nf2,
//      over the w^d stencil (periodic wrap).
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "fft_device.h"

namespace efgp {

template <typename T>
__global__ void k_zero_c(cpx<T>* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = cpx<T>{(T)0, (T)0};
}

template <typename T, int DIM>
__global__ void k_eval_pad(const cpx<T>* __restrict__ beta, const T* __restrict__ D, const T* __restrict__ dec,
                           int m, int nf2, int64_t M, int nrhs, int64_t gcells, cpx<T>* __restrict__ g) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= M * nrhs) return;
    const int W = 2 * m + 1;
    const int r = (int)(idx / M);
    const int64_t j = idx - (int64_t)r * M;
    int64_t rem = j, gi = 0;
    T f = D[j];
    int js[3];
    for (int l = DIM - 1; l >= 0; l--) { js[l] = (int)(rem % W) - m; rem /= W; }
    for (int l = 0; l < DIM; l++) {
        int a = js[l] < 0 ? js[l] + nf2 : js[l];
        gi = gi * nf2 + a;
        f *= dec[js[l] + m];
    }
    const cpx<T> b = beta[idx];
    g[(int64_t)r * gcells + gi] = cpx<T>{b.x * f, b.y * f};
}

// ES kernel value at 1 - z^2 = t (float: hardware sqrt and exp2 with beta
// pre-multiplied by log2 e, t < 0 from rounding at z = -1 clamped to the
// edge value e^-beta; double: libm, 0 outside the open support)
template <typename T> __device__ __forceinline__ T ev_phi(T t, T beta);
template <> __device__ __forceinline__ float ev_phi<float>(float t, float b2) {
    return __builtin_amdgcn_exp2f(fmaf(b2, __builtin_amdgcn_sqrtf(fmaxf(t, 0.0f)), -b2));
}
template <> __device__ __forceinline__ double ev_phi<double>(double t, double beta) {
    return t > 0.0 ? exp(beta * (sqrt(t) - 1.0)) : 0.0;
}

template <typename T, int DIM, int WMAX>
__global__ void __launch_bounds__(256) k_interp(const cpx<T>* __restrict__ g, int nf2, int64_t gcells, int nrhs,
                                                const T* __restrict__ t, int64_t q, T scale, T beta, int w,
                                                T* __restrict__ mu, int* __restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= q) return;
    const T inv_hw = (T)2 / (T)w, half_w = (T)0.5 * (T)w;
    T wt[DIM][WMAX];
    int g0[DIM];
    bool ok = true;
#pragma unroll
    for (int l = 0; l < DIM; l++) {
        const T a = t[(int64_t)l * q + i];
        ok = ok && (a >= (T)0 && a <= (T)1);
        const T u = a * scale;
        const T g0f = ceil(u - half_w);
        const T z0 = (g0f - u) * inv_hw;
#pragma unroll
        for (int k = 0; k < WMAX; k++) {
            if (k < w) {
                const T z = z0 + (T)k * inv_hw;
                wt[l][k] = ev_phi<T>((T)1 - z * z, beta);
            }
        }
        int gg = (int)g0f % nf2;
        g0[l] = gg < 0 ? gg + nf2 : gg;
    }
    if (!ok) {
        atomicOr(flag, 1);
        for (int r = 0; r < nrhs; r++) mu[(int64_t)r * q + i] = (T)NAN;
        return;
    }
    for (int r = 0; r < nrhs; r++) {
        const cpx<T>* gr = g + (int64_t)r * gcells;
        T acc = (T)0;
        if (DIM == 1) {
#pragma unroll
            for (int a = 0; a < WMAX; a++) {
                if (a < w) {
                    int c = g0[0] + a; c -= c >= nf2 ? nf2 : 0;
                    acc += wt[0][a] * gr[c].x;
                }
            }
        } else if (DIM == 2) {
#pragma unroll
            for (int a = 0; a < WMAX; a++) {
                if (a < w) {
                    int ca = g0[0] + a; ca -= ca >= nf2 ? nf2 : 0;
                    const cpx<T>* row = gr + (int64_t)ca * nf2;
                    T s = (T)0;
#pragma unroll
                    for (int b = 0; b < WMAX; b++) {
                        if (b < w) {
                            int cb = g0[1] + b; cb -= cb >= nf2 ? nf2 : 0;
                            s += wt[1][b] * row[cb].x;
                        }
                    }
                    acc += wt[0][a] * s;
                }
            }
        } else {
#pragma unroll
            for (int a = 0; a < WMAX; a++) {
                if (a < w) {
                    int ca = g0[0] + a; ca -= ca >= nf2 ? nf2 : 0;
                    T sa = (T)0;
#pragma unroll
                    for (int b = 0; b < WMAX; b++) {
                        if (b < w) {
                            int cb = g0[1] + b; cb -= cb >= nf2 ? nf2 : 0;
                            const cpx<T>* row = gr + ((int64_t)ca * nf2 + cb) * nf2;
                            T s = (T)0;
#pragma unroll
                            for (int e = 0; e < WMAX; e++) {
                                if (e < w) {
                                    int ce = g0[2] + e; ce -= ce >= nf2 ? nf2 : 0;
                                    s += wt[2][e] * row[ce].x;
                                }
                            }
                            sa += wt[1][b] * s;
                        }
                    }
                    acc += wt[0][a] * sa;
                }
            }
        }
        mu[(int64_t)r * q + i] = acc;
    }
}

// LDS variant.  Targets in [0,1] only touch the window of grid cells
// -floor(w/2) .. floor(h nf2) + ceil(w/2) along each axis (a fraction h of
// the period, like the spreader's active region), so persistent blocks stage
// the real part of that window, with the periodic wrap resolved, in LDS once
// and then stream targets: per target only its coordinates are read from HBM
// and its value written, and the w^d gathers hit LDS.  The loads of the next
// target are issued before the current target's gathers.
template <typename T, int DIM, int WMAX>
__global__ void __launch_bounds__(1024) k_interp_lds(const cpx<T>* __restrict__ g, int nf2, int64_t gcells,
                                                     int nrhs, int Aw, const T* __restrict__ t, int64_t q, T scale,
                                                     T beta, int w, T* __restrict__ mu, int* __restrict__ flag) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* win = reinterpret_cast<T*>(smem_raw);  // [nrhs][Aw^DIM]
    int64_t wcells = 1;
#pragma unroll
    for (int l = 0; l < DIM; l++) wcells *= Aw;
    const int fw = w / 2;
    for (int64_t e = threadIdx.x; e < wcells * nrhs; e += blockDim.x) {
        const int r = (int)(e / wcells);
        int64_t rem = e - (int64_t)r * wcells, gi = 0;
        int cl[3] = {0, 0, 0};
        for (int l = DIM - 1; l >= 0; l--) { cl[l] = (int)(rem % Aw); rem /= Aw; }
        for (int l = 0; l < DIM; l++) {
            int c = (cl[l] - fw) % nf2;
            c += c < 0 ? nf2 : 0;
            gi = gi * nf2 + c;
        }
        win[e] = g[(int64_t)r * gcells + gi].x;
    }
    __syncthreads();
    const T inv_hw = (T)2 / (T)w, half_w = (T)0.5 * (T)w;
    const int omax = Aw - w;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    T nt[DIM];
    if (i < q) {
#pragma unroll
        for (int l = 0; l < DIM; l++) nt[l] = t[(int64_t)l * q + i];
    }
    bool bad = false;
    for (; i < q; i += stride) {
        T ct[DIM];
#pragma unroll
        for (int l = 0; l < DIM; l++) ct[l] = nt[l];
        const int64_t inext = i + stride;
        if (inext < q) {
#pragma unroll
            for (int l = 0; l < DIM; l++) nt[l] = t[(int64_t)l * q + inext];
        }
        T wt[DIM][WMAX];
        int o[DIM];
        bool ok = true;
#pragma unroll
        for (int l = 0; l < DIM; l++) {
            const T a = ct[l];
            ok = ok && (a >= (T)0 && a <= (T)1);
            const T u = a * scale;
            const T g0f = ceil(u - half_w);
            const T z0 = (g0f - u) * inv_hw;
#pragma unroll
            for (int k = 0; k < WMAX; k++) {
                if (k < w) {
                    const T z = z0 + (T)k * inv_hw;
                    wt[l][k] = ev_phi<T>((T)1 - z * z, beta);
                }
            }
            o[l] = min(max((int)g0f + fw, 0), omax);  // in-window for targets in [0,1]
        }
        bad = bad || !ok;
        for (int r = 0; r < nrhs; r++) {
            const T* wr = win + (int64_t)r * wcells;
            T acc = (T)0;
            if (DIM == 1) {
#pragma unroll
                for (int a = 0; a < WMAX; a++)
                    if (a < w) acc += wt[0][a] * wr[o[0] + a];
            } else if (DIM == 2) {
#pragma unroll
                for (int a = 0; a < WMAX; a++) {
                    if (a < w) {
                        const T* row = wr + (o[0] + a) * Aw + o[1];
                        T sr = (T)0;
#pragma unroll
                        for (int b = 0; b < WMAX; b++)
                            if (b < w) sr += wt[1][b] * row[b];
                        acc += wt[0][a] * sr;
                    }
                }
            } else {
#pragma unroll
                for (int a = 0; a < WMAX; a++) {
                    if (a < w) {
                        T sa = (T)0;
#pragma unroll
                        for (int b = 0; b < WMAX; b++) {
                            if (b < w) {
                                const T* row = wr + ((o[0] + a) * Aw + o[1] + b) * Aw + o[2];
                                T sb = (T)0;
#pragma unroll
                                for (int e = 0; e < WMAX; e++)
                                    if (e < w) sb += wt[2][e] * row[e];
                                sa += wt[1][b] * sb;
                            }
                        }
                        acc += wt[0][a] * sa;
                    }
                }
            }
            mu[(int64_t)r * q + i] = ok ? acc : (T)NAN;
        }
    }
    if (bad) atomicOr(flag, 1);
}

static int ev_lds_limit() {
    int dev = 0, v = 65536;
    if (hipGetDevice(&dev) == hipSuccess) {
        int a = 0;
        if (hipDeviceGetAttribute(&a, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && a > 0) v = a;
    }
    return v;
}
static int ev_num_cus() {
    int dev = 0, v = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        int a = 0;
        if (hipDeviceGetAttribute(&a, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && a > 0) v = a;
    }
    return v;
}

// window edge per axis for the LDS interpolation: floor(h nf2) + w + 1 cells
// (computed from the kernel's own float scale so it covers every target)
template <typename T>
static int interp_window(const Plan& P) {
    const T sc = (T)(P.h * P.nf2);
    return (int)std::floor((double)sc) + P.w + 1;
}

template <typename T, int DIM, int WMAX>
static bool launch_interp_lds(Plan& P, const cpx<T>* g, int64_t gcells, const T* t, int64_t q, T* mu,
                              hipStream_t s) {
    const int Aw = std::min(interp_window<T>(P), P.nf2 + P.w + 1);
    const size_t one = (size_t)ipow(Aw, DIM) * sizeof(T);     // window bytes per coefficient vector
    const size_t budget = (size_t)ev_lds_limit() - 1024;
    if (one > budget) return false;
    // coefficient vectors per launch (all of them when they fit; each launch
    // reads the targets again)
    const int per = (int)std::min<size_t>((size_t)P.nrhs, budget / one);
    const T beta = std::is_same<T, float>::value ? (T)(P.es_beta * 1.4426950408889634) : (T)P.es_beta;
    auto kfn = k_interp_lds<T, DIM, WMAX>;
    for (int r0 = 0; r0 < P.nrhs; r0 += per) {
        const int nr = std::min(per, P.nrhs - r0);
        const size_t bytes = one * nr;
        // blocks per CU that fit the window, at least one; persistent over targets
        const int per_cu = std::max<int>(1, std::min<int>(4, (int)(((size_t)ev_lds_limit()) / (bytes + 1024))));
        const int64_t want = (q + 1023) / 1024;
        const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)ev_num_cus() * per_cu));
        EFGP_HIP(hipFuncSetAttribute((const void*)kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
        hipLaunchKernelGGL(kfn, dim3(nb), dim3(1024), bytes, s, g + (int64_t)r0 * gcells, P.nf2, gcells, nr, Aw, t,
                           q, (T)(P.h * P.nf2), beta, P.w, mu + (int64_t)r0 * q, P.flag);
        EFGP_HIP(hipGetLastError());
    }
    return true;
}

template <typename T, int DIM, int WMAX>
static void launch_interp(Plan& P, const cpx<T>* g, int64_t gcells, const T* t, int64_t q, T* mu, hipStream_t s) {
    if (launch_interp_lds<T, DIM, WMAX>(P, g, gcells, t, q, mu, s)) return;
    const T beta = std::is_same<T, float>::value ? (T)(P.es_beta * 1.4426950408889634) : (T)P.es_beta;
    hipLaunchKernelGGL((k_interp<T, DIM, WMAX>), dim3(cdiv(q, 256)), dim3(256), 0, s, g, P.nf2, gcells, P.nrhs, t, q,
                       (T)(P.h * P.nf2), beta, P.w, mu, P.flag);
    EFGP_HIP(hipGetLastError());
}

template <typename T, int DIM>
static void eval_typed(Plan& P, const void* beta, int64_t q, const void* targets, void* mu, hipStream_t s) {
    const int64_t gcells = ipow(P.nf2, DIM);
    cpx<T>* g = static_cast<cpx<T>*>(P.g2);
    hipLaunchKernelGGL((k_zero_c<T>), dim3(cdiv(gcells * P.nrhs, 256)), dim3(256), 0, s, g, gcells * P.nrhs);
    hipLaunchKernelGGL((k_eval_pad<T, DIM>), dim3(cdiv(P.M * P.nrhs, 256)), dim3(256), 0, s,
                       static_cast<const cpx<T>*>(beta), static_cast<const T*>(P.Dt), static_cast<const T*>(P.psi2),
                       P.m, P.nf2, P.M, P.nrhs, gcells, g);
    EFGP_HIP(hipGetLastError());
    FftDev<T> f;
    f.s = fft_shape(P.nf2);
    f.tw = static_cast<const cpx<T>*>(P.twE);
    for (int a = 0; a < DIM; a++)
        fft_axis<T>(g, f, ipow(P.nf2, a) * P.nrhs, ipow(P.nf2, DIM - 1 - a), -1, s);
    if (q <= 0) return;
    const T* t = static_cast<const T*>(targets);
    T* out = static_cast<T*>(mu);
    if (P.w <= 4) launch_interp<T, DIM, 4>(P, g, gcells, t, q, out, s);
    else if (P.w <= 6) launch_interp<T, DIM, 6>(P, g, gcells, t, q, out, s);
    else if (P.w <= 8) launch_interp<T, DIM, 8>(P, g, gcells, t, q, out, s);
    else if (P.w <= 12) launch_interp<T, DIM, 12>(P, g, gcells, t, q, out, s);
    else launch_interp<T, DIM, 16>(P, g, gcells, t, q, out, s);
}

void run_eval(Plan& P, const void* beta, int64_t q, const void* t, void* mu, hipStream_t s) {
    if (P.precision == 32) {
        if (P.dim == 1) eval_typed<float, 1>(P, beta, q, t, mu, s);
        else if (P.dim == 2) eval_typed<float, 2>(P, beta, q, t, mu, s);
        else eval_typed<float, 3>(P, beta, q, t, mu, s);
    } else {
        if (P.dim == 1) eval_typed<double, 1>(P, beta, q, t, mu, s);
        else if (P.dim == 2) eval_typed<double, 2>(P, beta, q, t, mu, s);
        else eval_typed<double, 3>(P, beta, q, t, mu, s);
    }
}

}  // namespace efgp
