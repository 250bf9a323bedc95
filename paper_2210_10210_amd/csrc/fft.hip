// Generic batched FFT along one axis of complex arrays laid out as
// [outer][n][inner] (C order).  Each block stages `lpb` lines in LDS, so
// global loads and stores stay coalesced for every axis: along the last axis
// (inner == 1) consecutive threads walk one line; along other axes they walk
// consecutive lines at the same position.
#include "fft_device.h"

namespace efgp {

template <typename T, int SIGN>
__global__ void __launch_bounds__(256) k_fft_axis(cpx<T>* __restrict__ data, FftDev<T> f,
                                                  int64_t nlines, int64_t inner, int lpb) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int n = f.s.n;
    cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* B = A + (size_t)lpb * n;
    const int64_t l0 = (int64_t)blockIdx.x * lpb;
    const int nl = (int)min<int64_t>((int64_t)lpb, nlines - l0);
    const bool contig = (inner == 1);
    for (int e = threadIdx.x; e < nl * n; e += blockDim.x) {
        int line, k;
        if (contig) { line = e / n; k = e - line * n; }
        else { k = e / nl; line = e - k * nl; }
        const int64_t L = l0 + line;
        const int64_t o = L / inner, i = L - o * inner;
        A[line * n + k] = data[(o * n + k) * inner + i];
    }
    __syncthreads();
    cpx<T>* R = fft_lds<T, SIGN>(A, B, n, nl, f);
    for (int e = threadIdx.x; e < nl * n; e += blockDim.x) {
        int line, k;
        if (contig) { line = e / n; k = e - line * n; }
        else { k = e / nl; line = e - k * nl; }
        const int64_t L = l0 + line;
        const int64_t o = L / inner, i = L - o * inner;
        data[(o * n + k) * inner + i] = R[line * n + k];
    }
}

// Long lines (two LDS buffers of the line would not fit): one buffer,
// kLongThreads threads, nl * n <= kLongMax, twiddles read from global memory.
template <typename T, int SIGN>
__global__ void __launch_bounds__(1024) k_fft_axis_long(cpx<T>* __restrict__ data, FftDev<T> f,
                                                        int64_t nlines, int64_t inner, int lpb) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int n = f.s.n;
    cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
    const int64_t l0 = (int64_t)blockIdx.x * lpb;
    const int nl = (int)min<int64_t>((int64_t)lpb, nlines - l0);
    const bool contig = (inner == 1);
    for (int e = threadIdx.x; e < nl * n; e += blockDim.x) {
        int line, k;
        if (contig) { line = e / n; k = e - line * n; }
        else { k = e / nl; line = e - k * nl; }
        const int64_t L = l0 + line;
        const int64_t o = L / inner, i = L - o * inner;
        A[line * n + k] = data[(o * n + k) * inner + i];
    }
    __syncthreads();
    fft_lds_1<T, SIGN>(A, n, nl, f);
    for (int e = threadIdx.x; e < nl * n; e += blockDim.x) {
        int line, k;
        if (contig) { line = e / n; k = e - line * n; }
        else { k = e / nl; line = e - k * nl; }
        const int64_t L = l0 + line;
        const int64_t o = L / inner, i = L - o * inner;
        data[(o * n + k) * inner + i] = A[line * n + k];
    }
}

template <typename T>
void fft_axis(cpx<T>* data, const FftDev<T>& f, int64_t outer, int64_t inner, int sign,
              hipStream_t s) {
    const int n = f.s.n;
    const int64_t nlines = outer * inner;
    if (nlines <= 0) return;
    if (2 * (size_t)n * sizeof(cpx<T>) > 48 * 1024) {
        // long lines: one buffer of up to 64 KB (and at least one line)
        if (n > kLongMax) throw StatusError{EFGP_ETOOLARGE, "FFT line longer than the supported maximum"};
        int lpb = (int)std::max<size_t>(1, std::min<size_t>((size_t)(kLongMax / n), 64 * 1024 / ((size_t)n * sizeof(cpx<T>))));
        if (!(inner == 1) && inner < lpb) lpb = (int)std::max<int64_t>(1, inner);
        const size_t lds = (size_t)lpb * n * sizeof(cpx<T>);
        const unsigned grid = cdiv(nlines, lpb);
        auto kf = sign < 0 ? k_fft_axis_long<T, -1> : k_fft_axis_long<T, 1>;
        if (lds > 64 * 1024)
            EFGP_HIP(hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        FftDev<T> g = f;
        g.s = fft_shape(n, 5);   // the one-buffer kernel's radices
        hipLaunchKernelGGL(kf, dim3(grid), dim3(kLongThreads), lds, s, data, g, nlines, inner, lpb);
        EFGP_HIP(hipGetLastError());
        return;
    }
    int lpb = (int)(48 * 1024 / (2 * (size_t)n * sizeof(cpx<T>)));
    lpb = std::max(1, std::min(lpb, 64));
    if (!(inner == 1) && inner < lpb) lpb = (int)std::max<int64_t>(1, inner);
    const size_t lds = 2 * (size_t)lpb * n * sizeof(cpx<T>);
    const unsigned grid = cdiv(nlines, lpb);
    if (sign < 0)
        hipLaunchKernelGGL((k_fft_axis<T, -1>), dim3(grid), dim3(256), lds, s, data, f, nlines, inner, lpb);
    else
        hipLaunchKernelGGL((k_fft_axis<T, 1>), dim3(grid), dim3(256), lds, s, data, f, nlines, inner, lpb);
    EFGP_HIP(hipGetLastError());
}

template void fft_axis<float>(cpx<float>*, const FftDev<float>&, int64_t, int64_t, int, hipStream_t);
template void fft_axis<double>(cpx<double>*, const FftDev<double>&, int64_t, int64_t, int, hipStream_t);

}  // namespace efgp
