// Circulant preconditioner for the weight-space system (D T D + sigma^2 I)
// beta = b of step 4 (eq. (97)).  The conclusions leave preconditioning of
// these Toeplitz-plus-diagonal systems open; this is T. Chan's optimal
// circulant (1988) applied to the system scaled by its diagonal:
//
//   J = N D_j^2 + sigma^2 (the diagonal: T_jj = v_0 = N),
//   E = J^(-1/2) A J^(-1/2), unit diagonal, extended by the identity to the
//       periodic grid {0..K-1}^d (K = smallest 2,3,5-smooth >= 2m+1, E on the
//       indices j + m in {0..2m}^d),
//   C = F^H diag(lambda) F nearest to that matrix in the Frobenius norm:
//       lambda_s = f_s^H (E (+) I) f_s, f_s(j) = exp(2 pi i <s,j>/K) / K^(d/2),
//   P = J^(-1/2) R^T C^(-1) R J^(-1/2)   (R: restriction to the M frequencies).
//
// With g_j = D_j / sqrt(J_j) and a_u = sum_k g_{k+u} g_k (u in J_2m) the
// quadratic form sums collapse to
//   K^d lambda_s = K^d - M + sum_j sigma^2 / J_j + sum_u a_u v_u exp(-2 pi i <s,u>/K),
// so lambda costs one autocorrelation (FFT at the embedding size L >= 4m+1)
// and one FFT at size K per system, and the last sum is a positive
// semidefinite quadratic form: K^d lambda_s is bounded below by the first two
// terms, which the computed values are clamped to (only rounding can cross
// it).  Applying P costs a forward and an inverse FFT of the K^d grid.
#include <algorithm>
#include <cmath>

#include "fft_device.h"

namespace efgp {

template <typename T> struct CircArgs {
    const cpx<T>* r;    // nrhs*M residuals
    cpx<T>* z;          // nrhs*M, z = P r
    const T* js;        // nrhs*M, 1/sqrt(N D_j^2 + sigma_r^2)
    const T* ilam;      // nrhs*K^d, 1/(K^d lambda_s)
    cpx<T>* cbuf;       // nrhs*K^d
    CgState* st;        // nrhs
    double* slots;      // nrhs*W^(d-1) per-line sums of Re r^H z
    unsigned* counter;  // blocks of the last pass done (reset by the last one)
    int m, W, K, nrhs;
    int64_t M, KD;
};

// batched d-dimensional FFT of nb grids of n^d (C order) on the stream
template <typename T>
static void fft_nd(cpx<T>* data, const FftDev<T>& f, int n, int dim, int64_t nb, int sign, hipStream_t s) {
    for (int l = 0; l < dim; l++) {
        const int64_t outer = nb * ipow(n, l);
        const int64_t inner = ipow(n, dim - 1 - l);
        fft_axis<T>(data, f, outer, inner, sign, s);
    }
}

// ------------------------------------------------------------- eigenvalues
template <typename T>
__global__ void k_circ_js(const double* __restrict__ D, const double* __restrict__ sig2, double nn, int64_t M,
                          int nrhs, T* __restrict__ js) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M * nrhs) return;
    const int r = (int)(i / M);
    const double d = D[i - (int64_t)r * M];
    js[i] = (T)(1.0 / sqrt(nn * d * d + sig2[r]));
}

// g_j = D_j / sqrt(N D_j^2 + sigma^2) placed at {0..2m}^d of an L^d grid
template <typename T, int DIM>
__global__ void k_circ_g(const double* __restrict__ D, double s2, double nn, int W, int L,
                         cpx<T>* __restrict__ grid) {
    int64_t LD = 1;
    for (int l = 0; l < DIM; l++) LD *= L;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= LD) return;
    int64_t rem = i, j = 0, stride = 1;
    bool in = true;
    for (int l = DIM - 1; l >= 0; l--) {
        const int p = (int)(rem % L);
        rem /= L;
        in = in && p < W;
        j += (int64_t)p * stride;
        stride *= W;
    }
    T g = (T)0;
    if (in) {
        const double d = D[j];
        g = (T)(d / sqrt(nn * d * d + s2));
    }
    grid[i] = cpx<T>{g, (T)0};
}

template <typename T>
__global__ void k_circ_abs2(cpx<T>* __restrict__ a, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const cpx<T> z = a[i];
    a[i] = cpx<T>{z.x * z.x + z.y * z.y, (T)0};
}

// c_s = sum over u in J_2m with u = s (mod K) of a_u v_u; a_u is the
// autocorrelation at (u mod L) (unnormalised inverse FFT: times scale)
template <typename T, int DIM>
__global__ void k_circ_wrap(const cpx<T>* __restrict__ acorr, const double2* __restrict__ v, int m, int L, int K,
                            double scale, cpx<T>* __restrict__ out) {
    int64_t KD = 1;
    for (int l = 0; l < DIM; l++) KD *= K;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= KD) return;
    int sl[3] = {0, 0, 0};
    int64_t rem = i;
    for (int l = DIM - 1; l >= 0; l--) { sl[l] = (int)(rem % K); rem /= K; }
    const int W2 = 4 * m + 1;
    double cx = 0.0, cy = 0.0;
    for (int mask = 0; mask < (1 << DIM); mask++) {
        bool ok = true;
        int64_t ia = 0, iv = 0;
        for (int l = 0; l < DIM; l++) {
            const int u = (mask >> l) & 1 ? sl[l] - K : sl[l];
            ok = ok && u >= -2 * m && u <= 2 * m;
            ia = ia * L + (u < 0 ? u + L : u);
            iv = iv * W2 + (u + 2 * m);
        }
        if (!ok) continue;
        const double a = (double)acorr[ia].x * scale;
        const double2 vv = v[iv];
        cx += a * vv.x;
        cy += a * vv.y;
    }
    out[i] = cpx<T>{(T)cx, (T)cy};
}

// K^d lambda_s = max(Re c^_s + base, base); writes 1/(K^d lambda) or lambda
template <typename T>
__global__ void k_circ_lam(const cpx<T>* __restrict__ c, int64_t KD, double base, T* __restrict__ out,
                           int inverse) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= KD) return;
    const double kl = fmax((double)c[i].x + base, base);
    out[i] = inverse ? (T)(1.0 / kl) : (T)(kl / (double)KD);
}

// lambda of system r into out (inverse: 1/(K^d lambda)); cbuf_r is K^d
// complex workspace
template <typename T>
static void eigs_one(Plan& P, int r, const std::vector<double>& Dh, cpx<T>* grid, cpx<T>* cbuf_r, T* out,
                     bool inverse, hipStream_t s) {
    const int d = P.dim, L = P.L, K = P.K;
    const int64_t LD = ipow(L, d), KD = ipow(K, d);
    const double nn = (double)P.n, s2 = P.sigma2[r];
    double s0 = 0.0;
    for (double x : Dh) s0 += s2 / (nn * x * x + s2);
    const double base = (double)(KD - P.M) + s0;
    const FftDev<T> fL{fft_shape(L), static_cast<const cpx<T>*>(P.twL)};
    const FftDev<T> fK{fft_shape(K), static_cast<const cpx<T>*>(P.twK)};
    const double2* v = reinterpret_cast<const double2*>(P.v);
    const unsigned gL = cdiv(LD, 256), gK = cdiv(KD, 256);
    if (d == 1) hipLaunchKernelGGL((k_circ_g<T, 1>), dim3(gL), dim3(256), 0, s, P.D64, s2, nn, P.W, L, grid);
    else if (d == 2) hipLaunchKernelGGL((k_circ_g<T, 2>), dim3(gL), dim3(256), 0, s, P.D64, s2, nn, P.W, L, grid);
    else hipLaunchKernelGGL((k_circ_g<T, 3>), dim3(gL), dim3(256), 0, s, P.D64, s2, nn, P.W, L, grid);
    fft_nd<T>(grid, fL, L, d, 1, -1, s);
    hipLaunchKernelGGL((k_circ_abs2<T>), dim3(gL), dim3(256), 0, s, grid, LD);
    fft_nd<T>(grid, fL, L, d, 1, +1, s);
    const double sc = 1.0 / (double)LD;
    if (d == 1) hipLaunchKernelGGL((k_circ_wrap<T, 1>), dim3(gK), dim3(256), 0, s, grid, v, P.m, L, K, sc, cbuf_r);
    else if (d == 2) hipLaunchKernelGGL((k_circ_wrap<T, 2>), dim3(gK), dim3(256), 0, s, grid, v, P.m, L, K, sc, cbuf_r);
    else hipLaunchKernelGGL((k_circ_wrap<T, 3>), dim3(gK), dim3(256), 0, s, grid, v, P.m, L, K, sc, cbuf_r);
    fft_nd<T>(cbuf_r, fK, K, d, 1, -1, s);
    hipLaunchKernelGGL((k_circ_lam<T>), dim3(gK), dim3(256), 0, s, cbuf_r, KD, base, out, inverse ? 1 : 0);
    EFGP_HIP(hipGetLastError());
}

template <typename T>
static void circ_alloc(Plan& P, hipStream_t s) {
    if (!P.twK) {
        // two line buffers and the twiddles of one period in the default LDS
        if (3 * (size_t)next_smooth235(P.W) * sizeof(cpx<T>) > 64 * 1024)
            throw StatusError{EFGP_ETOOLARGE, "circulant preconditioner period too long"};
        P.K = next_smooth235(P.W);
        upload_twiddles<T>(P, P.K, &P.twK, s);
    }
    const int64_t KD = ipow(P.K, P.dim);
    if (!P.clam) P.clam = dalloc(P, sizeof(T) * KD * P.nrhs);
    if (!P.cbuf) P.cbuf = dalloc(P, 2 * sizeof(T) * KD * P.nrhs);
    if (!P.zbuf) P.zbuf = dalloc(P, 2 * sizeof(T) * P.M * P.nrhs);
    if (!P.cslot) {
        // per-line slots, then the last-pass block counter
        const size_t bytes = sizeof(double) * ipow(P.W, P.dim - 1) * P.nrhs + 64;
        P.cslot = static_cast<double*>(dalloc(P, bytes));
        EFGP_HIP(hipMemsetAsync(P.cslot, 0, bytes, s));
    }
    if (!P.prec) P.prec = dalloc(P, sizeof(T) * P.M * P.nrhs);
}

template <typename T>
void circ_setup(Plan& P, hipStream_t s) {
    circ_alloc<T>(P, s);
    const int64_t KD = ipow(P.K, P.dim), LD = ipow(P.L, P.dim);
    hipLaunchKernelGGL((k_circ_js<T>), dim3(cdiv(P.M * P.nrhs, 256)), dim3(256), 0, s, P.D64, P.sig2, (double)P.n,
                       P.M, P.nrhs, static_cast<T*>(P.prec));
    const std::vector<double> Dh = spectral_weights(P);
    cpx<T>* grid = nullptr;
    EFGP_HIP(hipMallocAsync((void**)&grid, 2 * sizeof(T) * LD, s));
    for (int r = 0; r < P.nrhs; r++)
        eigs_one<T>(P, r, Dh, grid, static_cast<cpx<T>*>(P.cbuf) + r * KD, static_cast<T*>(P.clam) + r * KD, true, s);
    EFGP_HIP(hipFreeAsync(grid, s));
}

template <typename T>
void circ_eigs(Plan& P, int r, void* out, hipStream_t s) {
    circ_alloc<T>(P, s);
    const int64_t LD = ipow(P.L, P.dim);
    const std::vector<double> Dh = spectral_weights(P);
    cpx<T>* grid = nullptr;
    EFGP_HIP(hipMallocAsync((void**)&grid, 2 * sizeof(T) * LD, s));
    eigs_one<T>(P, r, Dh, grid, static_cast<cpx<T>*>(P.cbuf), static_cast<T*>(out), false, s);
    EFGP_HIP(hipFreeAsync(grid, s));
}

// ------------------------------------------------------------- application
// The K^d grids of all systems are transformed line by line ([outer][K]
// [inner] views, lpb lines per workgroup staged in LDS, as the Toeplitz
// product does) in 2d - 1 passes for d >= 2:
//   FIRST  along the last axis: load J^(-1/2) r at {0..2m}^d (zeros elsewhere), forward FFT;
//   FWD    along a middle axis (d = 3): forward FFT;
//   TURN   along axis 0: forward FFT, times 1/(K^d lambda), inverse FFT;
//   INV    along a middle axis: inverse FFT;
//   LAST   along the last axis, only the lines inside {0..2m}^(d-1): inverse
//          FFT, z = J^(-1/2) (first 2m+1 entries), per-line sums of Re r^H z,
//          and in the last block to finish, r^H z into the CG state;
//   ONLY   (d = 1) all of it on one line per system.
enum { CL_FIRST = 0, CL_FWD = 1, CL_TURN = 2, CL_INV = 3, CL_LAST = 4, CL_ONLY = 5 };

template <typename T, int DIM, int OP>
__global__ void __launch_bounds__(256) k_circ_line(CircArgs<T> a, FftDev<T> f, int64_t nlines, int64_t inner,
                                                   int lpb, int fresh) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int lastblk;
    const int K = a.K, W = a.W;
    cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* B = A + (size_t)lpb * K;
    cpx<T>* tws = B + (size_t)lpb * K;
    for (int i = threadIdx.x; i < K; i += blockDim.x) tws[i] = f.tw[i];
    FftDev<T> g = f;
    g.tw = tws;
    const int64_t l0 = (int64_t)blockIdx.x * lpb;
    const int nl = (int)min<int64_t>((int64_t)lpb, nlines - l0);
    const bool contig = (inner == 1);
    // rows of the leading d-1 axes: K^(d-1) per system, W^(d-1) inside the box
    int64_t rowsK = 1, rowsW = 1;
    for (int l = 0; l < DIM - 1; l++) { rowsK *= K; rowsW *= W; }
    constexpr bool FROM_R = (OP == CL_FIRST || OP == CL_ONLY);
    constexpr bool TO_Z = (OP == CL_LAST || OP == CL_ONLY);
    for (int e = threadIdx.x; e < nl * K; e += blockDim.x) {
        int line, k;
        if (contig) { line = e / K; k = e - line * K; }
        else { k = e / nl; line = e - k * nl; }
        const int64_t Lg = l0 + line;
        cpx<T> v = cpx<T>{(T)0, (T)0};
        if (FROM_R) {
            const int64_t r = Lg / rowsK, row = Lg - r * rowsK;
            int64_t rem = row, rowW = 0, sw = 1;
            bool in = k < W;
            for (int l = DIM - 2; l >= 0; l--) {
                const int p = (int)(rem % K);
                rem /= K;
                in = in && p < W;
                rowW += (int64_t)p * sw;
                sw *= W;
            }
            if (in) {
                const int64_t idx = r * a.M + rowW * W + k;
                const T w = a.js[idx];
                const cpx<T> rv = a.r[idx];
                v = cpx<T>{w * rv.x, w * rv.y};
            }
        } else if (OP == CL_LAST) {
            const int64_t r = Lg / rowsW, rowW = Lg - r * rowsW;
            int64_t rem = rowW, rowK = 0, sk = 1;
            for (int l = DIM - 2; l >= 0; l--) {
                const int p = (int)(rem % W);
                rem /= W;
                rowK += (int64_t)p * sk;
                sk *= K;
            }
            v = a.cbuf[r * a.KD + rowK * K + k];
        } else {
            const int64_t o = Lg / inner, i = Lg - o * inner;
            v = a.cbuf[(o * K + k) * inner + i];
        }
        A[line * K + k] = v;
    }
    __syncthreads();
    constexpr int SIGN = (OP == CL_INV || OP == CL_LAST) ? 1 : -1;
    cpx<T>* R = fft_lds<T, SIGN>(A, B, K, nl, g);
    if (OP == CL_TURN || OP == CL_ONLY) {
        for (int e = threadIdx.x; e < nl * K; e += blockDim.x) {
            int line, k;
            if (contig) { line = e / K; k = e - line * K; }
            else { k = e / nl; line = e - k * nl; }
            const int64_t Lg = l0 + line;
            const int64_t o = Lg / inner, i = Lg - o * inner;
            const T w = a.ilam[(o * K + k) * inner + i];
            const cpx<T> c = R[line * K + k];
            R[line * K + k] = cpx<T>{w * c.x, w * c.y};
        }
        __syncthreads();
        R = fft_lds<T, 1>(R, R == A ? B : A, K, nl, g);
    }
    if (TO_Z) {
        // per-element terms of Re r^H z in the buffer the result is not in
        // (nl K >= nl W doubles), then one wavefront per line sums them in a
        // fixed order (strided lane sums and a shuffle tree)
        double* term = reinterpret_cast<double*>(R == A ? B : A);
        for (int e = threadIdx.x; e < nl * W; e += blockDim.x) {
            const int line = e / W, k = e - line * W;
            const int64_t Lg = l0 + line;
            const int64_t idx = Lg * W + k;   // (r * W^(d-1) + rowW) * W + k = r * M + j
            const T w = a.js[idx];
            const cpx<T> c = R[line * K + k];
            const cpx<T> zv = cpx<T>{w * c.x, w * c.y};
            a.z[idx] = zv;
            const cpx<T> rv = a.r[idx];
            term[e] = (double)rv.x * (double)zv.x + (double)rv.y * (double)zv.y;
        }
        __syncthreads();
        {
            const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
            for (int line = wv; line < nl; line += nw) {
                double sum = 0.0;
                for (int k = lane; k < W; k += 64) sum += term[line * W + k];
                sum = warp_sum(sum);
                if (lane == 0) a.slots[l0 + line] = sum;
            }
        }
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) lastblk = (atomicAdd(a.counter, 1u) == gridDim.x - 1) ? 1 : 0;
        __syncthreads();
        if (!lastblk) return;
        __threadfence();
        // the last block: r^H z per system (one wavefront each) into the CG
        // state of every preconditioned active system.  fresh: only those just
        // initialised or restarted (gamma = 0, which they keep, so the next
        // direction is z).  A non-positive or non-finite r^H z means the
        // preconditioner broke down: the system stops with a NaN residual,
        // which the host turns into the plain-CG fallback.
        const int64_t nslot = rowsW;
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
        for (int k = wv; k < a.nrhs; k += nw) {
            double rz = 0.0;
            for (int64_t b = lane; b < nslot; b += 64) rz += ((const volatile double*)a.slots)[(int64_t)k * nslot + b];
            rz = warp_sum(rz);
            if (lane != 0) continue;
            CgState& t = a.st[k];
            if (!t.use_prec || !t.active || (fresh && t.gamma != 0.0)) continue;
            if (!(rz > 0.0) || !(rz < INFINITY)) {
                t.active = 0;
                t.relres = NAN;
            } else {
                if (!fresh) t.gamma = rz / t.rz;
                t.rz = rz;
            }
        }
        if (threadIdx.x == 0) *a.counter = 0u;
    } else {
        for (int e = threadIdx.x; e < nl * K; e += blockDim.x) {
            int line, k;
            if (contig) { line = e / K; k = e - line * K; }
            else { k = e / nl; line = e - k * nl; }
            const int64_t Lg = l0 + line;
            const int64_t o = Lg / inner, i = Lg - o * inner;
            a.cbuf[(o * K + k) * inner + i] = R[line * K + k];
        }
    }
}

template <typename T>
void circ_apply(const Plan& P, bool fresh, hipStream_t s) {
    CircArgs<T> a{};
    a.r = static_cast<const cpx<T>*>(P.r);
    a.z = static_cast<cpx<T>*>(P.zbuf);
    a.js = static_cast<const T*>(P.prec);
    a.ilam = static_cast<const T*>(P.clam);
    a.cbuf = static_cast<cpx<T>*>(P.cbuf);
    a.st = P.st;
    a.slots = P.cslot;
    a.counter = reinterpret_cast<unsigned*>(P.cslot + ipow(P.W, P.dim - 1) * P.nrhs);
    a.m = P.m;
    a.W = P.W;
    a.K = P.K;
    a.nrhs = P.nrhs;
    a.M = P.M;
    a.KD = ipow(P.K, P.dim);
    const FftDev<T> fK{fft_shape(P.K), static_cast<const cpx<T>*>(P.twK)};
    const int d = P.dim;
    const int K = P.K;
    const int64_t nslot = ipow(P.W, d - 1);
    const int64_t rowsK = ipow(K, d - 1);
    auto line = [&](auto kern, int64_t nlines, int64_t inner) {
        // about one element per thread: each thread's loads then go out
        // together instead of one round trip after another
        int lpb = std::max(1, 256 / K);
        if (inner > 1 && inner < lpb) lpb = (int)inner;
        const size_t lds = (2 * (size_t)lpb * K + K) * sizeof(cpx<T>);
        hipLaunchKernelGGL(kern, dim3(cdiv(nlines, lpb)), dim3(256), lds, s, a, fK, nlines, inner, lpb,
                           fresh ? 1 : 0);
    };
    const int64_t nr = P.nrhs;
    if (d == 1) {
        line(k_circ_line<T, 1, CL_ONLY>, nr, 1);
    } else if (d == 2) {
        line(k_circ_line<T, 2, CL_FIRST>, nr * K, 1);
        line(k_circ_line<T, 2, CL_TURN>, nr * K, K);
        line(k_circ_line<T, 2, CL_LAST>, nr * nslot, 1);
    } else {
        line(k_circ_line<T, 3, CL_FIRST>, nr * rowsK, 1);
        line(k_circ_line<T, 3, CL_FWD>, nr * rowsK, K);
        line(k_circ_line<T, 3, CL_TURN>, nr * rowsK, (int64_t)K * K);
        line(k_circ_line<T, 3, CL_INV>, nr * rowsK, K);
        line(k_circ_line<T, 3, CL_LAST>, nr * nslot, 1);
    }
    EFGP_HIP(hipGetLastError());
}

template void circ_setup<float>(Plan&, hipStream_t);
template void circ_setup<double>(Plan&, hipStream_t);
template void circ_apply<float>(const Plan&, bool, hipStream_t);
template void circ_apply<double>(const Plan&, bool, hipStream_t);
template void circ_eigs<float>(Plan&, int, void*, hipStream_t);
template void circ_eigs<double>(Plan&, int, void*, hipStream_t);

}  // namespace efgp
