// Solve stage of EFGP (step 4 of the EFGP algorithm): conjugate gradients on
// (D F*F D + sigma^2 I) beta = b with the fast Toeplitz product (Sec. 3.2).
//
// Toeplitz product.  F*F beta is the restriction to J_m of the linear
// convolution v * beta.  With v (on J_2m) and beta (on J_m) embedded
// periodically at size L >= 4m+1 per dimension (index j -> j mod L) the
// cyclic convolution equals the linear one on J_m, so
//     F*F beta = Extract( IFFT( FFT(v) . FFT(Pad(beta)) ) ).
// Only 2m+1 of the L lines along each axis are nonzero on input and only
// 2m+1 are kept on output, so the passes prune: in d=2 the forward row FFT
// runs on 2m+1 rows, the column pass (FFT, multiply by vhat, inverse FFT)
// on all L columns but keeps 2m+1 rows, and the inverse row FFT on 2m+1
// rows with the extraction, D scaling and sigma^2 term fused in.
//
// CG.  Vectors are in the plan precision; inner products and step scalars
// are double.  The direction update p = z + gamma p (z = P r) is fused into
// the first pass, p^H A p into the last pass, and x/r updates with ||r||^2
// and r^H z into one kernel whose last block finalises the scalars.  One
// iteration is a fixed sequence of kernels with all scalars in device
// memory, so a batch of iterations is captured once in a hipGraph and
// replayed; systems that have converged keep their state.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <mutex>
#include <type_traits>

#include "fft_device.h"

namespace efgp {

enum { MV_APPLY = 0, MV_CG = 1, MV_RESID = 2 };

template <typename T> struct MvArgs {
    const cpx<T>* in;       // APPLY/RESID: input vector; CG: unused (uses p)
    cpx<T>* out;            // APPLY: output
    cpx<T>* x;              // RESID: current iterate
    cpx<T>* r;              // CG/RESID
    cpx<T>* p;              // CG
    cpx<T>* q;              // CG
    const cpx<T>* b;        // RESID
    const T* prec;          // nrhs*M or null (a diagonal preconditioner)
    const cpx<T>* z;        // nrhs*M preconditioned residuals from an operator
                            // preconditioner (circulant), or null
    const T* D;             // M
    const cpx<T>* vhat;     // L^d
    const double* sig2;     // nrhs
    CgState* st;            // nrhs
    cpx<T>* buf1;
    cpx<T>* buf2;
    double* part;           // partial sums: [3][nrhs*rows] per line, then [nrhs][kGmax][3] per block
    FftDev<T> f;
    int m, W, L, nrhs, rows;
    int64_t M;
    int idle_skip;          // CG passes: blocks whose systems have all stopped return
    int herm;               // 2D CG passes on Hermitian vectors (x[M-1-j] = conj x[j]):
                            // only rows i >= 0 of J_m are transformed (rows = m + 1)
};

constexpr int kGmax = 1024;   // max blocks per system in the vector kernel
constexpr int kMidV = 8;      // FFT(v) values per thread held in registers by the column pass
// Largest FFT radix of the 1024-thread kernels on short lines: the fused
// last pass in double, like the one-buffer long-line passes, keeps to
// radices 2..5 (the larger register butterflies would spill)
template <typename T> constexpr int kCg1MaxR = std::is_same<T, float>::value ? 16 : 5;

// partial-sum slots (no same-address atomics: consumers sum the slots)
template <typename T> __device__ __forceinline__ double* slot_pq(const MvArgs<T>& a) { return a.part; }
template <typename T> __device__ __forceinline__ double* slot_rr(const MvArgs<T>& a) { return a.part + (int64_t)a.nrhs * a.rows; }
template <typename T> __device__ __forceinline__ double* slot_rz(const MvArgs<T>& a) { return a.part + 2 * (int64_t)a.nrhs * a.rows; }
template <typename T> __device__ __forceinline__ double* slot_vec(const MvArgs<T>& a) { return a.part + 3 * (int64_t)a.nrhs * a.rows; }

// Copy n >= 1 contiguous values from global memory to LDS with four loads
// in flight per thread before any store (one load-then-store per element
// waits a full memory latency each time).  Slots past the end re-read the
// last value and are not stored.
template <typename V>
__device__ __forceinline__ void stage4(V* __restrict__ dst, const V* __restrict__ src, int n) {
    for (int i0 = threadIdx.x; i0 < n; i0 += 4 * (int)blockDim.x) {
        V v[4];
#pragma unroll
        for (int u = 0; u < 4; u++) v[u] = src[min(i0 + u * (int)blockDim.x, n - 1)];
#pragma unroll
        for (int u = 0; u < 4; u++)
            if (i0 + u * (int)blockDim.x < n) dst[i0 + u * (int)blockDim.x] = v[u];
    }
}

// stage the twiddle table in LDS and return a descriptor pointing at it
template <typename T>
__device__ __forceinline__ FftDev<T> lds_twiddles(const FftDev<T>& f, cpx<T>* tws) {
    stage4(tws, f.tw, f.s.n);
    FftDev<T> g = f;
    g.tw = tws;
    return g;
}

// True (the same in every thread) when idle_skip is set and every line
// l0..l0+nl-1 of the block belongs to a system that has stopped: its
// product would not be used (the vector kernels skip stopped systems, and
// the final residual check recomputes from x), so the block returns before
// any barrier.  A graph of several iterations then costs little past
// convergence.
template <typename T>
__device__ __forceinline__ bool lines_idle(const MvArgs<T>& a, int64_t l0, int nl, int64_t per_sys) {
    if (!a.idle_skip) return false;
    const int64_t r0 = l0 / per_sys, r1 = (l0 + nl - 1) / per_sys;
    for (int64_t r = r0; r <= r1; r++)
        if (a.st[r].active) return false;
    return true;
}

__device__ __forceinline__ int wrapL(int j, int L) { return j < 0 ? j + L : j; }
// inverse of the padding: the index jj in 0..2m whose padded position
// (jj - m) mod L is k, or -1 where the padded line is zero
__device__ __forceinline__ int unpadL(int k, int m, int L) {
    if (k <= m) return k + m;
    if (k >= L - m) return k - L + m;
    return -1;
}

// ---- first pass: pad (D p) along the last axis and FFT it
// LONG: lines too long for two LDS buffers (one buffer, kLongThreads
// threads, twiddles read from global memory; fft_lds_1).
template <typename T, int DIM, int MODE, bool LONG>
__global__ void __launch_bounds__(LONG ? 1024 : 512) k_mv_first(MvArgs<T> a, int lpb) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int L = a.L, W = a.W, m = a.m;
    cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* B = A + (size_t)lpb * L;
    const FftDev<T> f = LONG ? a.f : lds_twiddles(a.f, B + (size_t)lpb * L);
    const int rows = a.rows;
    const int64_t nlines = (int64_t)rows * a.nrhs;
    const int64_t l0 = (int64_t)blockIdx.x * lpb;
    const int nl = (int)min<int64_t>(lpb, nlines - l0);
    if (lines_idle(a, l0, nl, rows)) return;
    // one pass over the padded lines (zeros outside the 2m+1 entries), line
    // by line (the line's system and row are block-uniform): four elements'
    // loads per thread are issued before any store (a store to p would
    // otherwise hold back the next element's loads by a full memory round
    // trip)
    (void)W;
    for (int line = 0; line < nl; line++) {
        const int64_t gl = l0 + line;
        const int r = (int)(gl / rows);
        const int64_t rowi = gl - (int64_t)r * rows;            // Hermitian: row i = rowi >= 0 of J_m
        const int64_t rowj = (a.herm ? rowi + m : rowi) * a.W;
        const int64_t base = (int64_t)r * a.M + rowj;
        const bool mirror = a.herm && rowi > 0;                  // row -i is written as its conjugate
        cpx<T>* Al = A + line * L;
        for (int k0 = threadIdx.x; k0 < L; k0 += 4 * (int)blockDim.x) {
            cpx<T> pv[4], zv[4];
            T dv[4], pr[4];
            int jjs[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int k = k0 + u * (int)blockDim.x;
                const int jj = k < L ? unpadL(k, m, L) : -1;
                jjs[u] = jj;
                if (jj >= 0) {
                    const int64_t idx = base + jj;
                    dv[u] = a.D[rowj + jj];
                    if (MODE == MV_CG) {
                        pv[u] = a.p[idx];
                        zv[u] = (a.z && a.st[r].use_prec) ? a.z[idx] : a.r[idx];
                        pr[u] = a.prec ? a.prec[idx] : (T)1;
                    } else {
                        pv[u] = MODE == MV_RESID ? a.x[idx] : a.in[idx];
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int k = k0 + u * (int)blockDim.x;
                if (k >= L) continue;
                cpx<T> out = cpx<T>{(T)0, (T)0};
                if (jjs[u] >= 0) {
                    cpx<T> val = pv[u];
                    if (MODE == MV_CG) {
                        const CgState& s = a.st[r];
                        if (s.active) {
                            cpx<T> z = zv[u];
                            if (s.use_prec) { z.x *= pr[u]; z.y *= pr[u]; }
                            const T g = (T)s.gamma;
                            val = cpx<T>{z.x + g * val.x, z.y + g * val.y};
                            a.p[base + jjs[u]] = val;
                            if (mirror) a.p[(int64_t)r * a.M + (a.M - 1 - rowj - jjs[u])] = cpx<T>{val.x, -val.y};
                        }
                    }
                    out = cpx<T>{dv[u] * val.x, dv[u] * val.y};
                }
                Al[k] = out;
            }
        }
    }
    __syncthreads();
    cpx<T>* R = A;
    if (LONG) fft_lds_1<T, -1>(A, L, nl, f);
    else R = fft_lds<T, -1>(A, B, L, nl, f);
    cpx<T>* dst = DIM == 1 ? nullptr : a.buf1;
    if (DIM > 1) {
        for (int e = threadIdx.x; e < nl * L; e += blockDim.x) dst[(l0 * L) + e] = R[e];
    }
}

// Block index remapped so that the blocks one XCD runs take a contiguous
// range (the hardware hands consecutive blocks to the 8 XCDs in turn): the
// column passes read a few adjacent columns per block, and neighbouring
// blocks then share cache lines in one L2 instead of fetching them into
// several.  A bijection of 0..gridDim.x-1.
__device__ __forceinline__ unsigned xcd_block() {
    const unsigned nb = gridDim.x, b = blockIdx.x;
    const unsigned q = nb / 8, r = nb % 8, x = b % 8, k = b / 8;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

// ---- middle passes along a non-last axis of [nrhs*outer][n_in][inner]
// INP/OUTP: 1 = pruned (2m+1 entries at j mod L), 0 = full L entries.
// OP: 0 forward FFT, 1 inverse FFT, 2 forward, multiply by vhat, inverse.
template <typename T, int INP, int OUTP, int OP, bool LONG>
__global__ void __launch_bounds__(LONG ? 1024 : 512) k_mv_mid(MvArgs<T> a, const cpx<T>* __restrict__ src,
                                                              cpx<T>* __restrict__ dst, int64_t outer, int64_t inner,
                                                              int lpb) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int L = a.L, W = a.W, m = a.m;
    const int nin = INP ? W : L, nout = OUTP ? W : L;
    cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* B = A + (size_t)lpb * L;
    const FftDev<T> f = LONG ? a.f : lds_twiddles(a.f, B + (size_t)lpb * L);
    const int64_t nlines = (int64_t)a.nrhs * outer * inner;
    const int64_t l0 = (int64_t)xcd_block() * lpb;
    const int nl = (int)min<int64_t>(lpb, nlines - l0);
    if (lines_idle(a, l0, nl, outer * inner)) return;
    // OP 2 (LONG): the block's columns of vhat go to LDS after A, in the same
    // pass as the input.  Otherwise each thread loads the vhat values of the
    // elements it multiplies into registers first (element e = tid + u
    // blockDim, u < kMidV; the host keeps nl L <= kMidV blockDim), so those
    // loads overlap the input's and the block needs no LDS for them.
    cpx<T>* V = B;
    cpx<T> vreg[kMidV];
    const int total = nl * L;
    // line l of the block is (ro, i) of [outer rows][..][inner]: the block's
    // first line l0 = ro0 inner + i0, and its nl <= inner lines wrap past the
    // end of a row at most once (no per-element division)
    const int ro0 = (int)(l0 / inner), i0 = (int)(l0 - (int64_t)ro0 * inner), inn = (int)inner;
    auto line_at = [&](int line, int* ro) {
        int i = i0 + line;
        *ro = ro0;
        if (i >= inn) {
            i -= inn;
            *ro = ro0 + 1;
        }
        return i;
    };
    const float rnl = 1.0f / (float)nl, rL = 1.0f / (float)L;
    if (OP == 2 && !LONG) {
#pragma unroll
        for (int u = 0; u < kMidV; u++) {
            const int e = threadIdx.x + u * (int)blockDim.x;
            if (e < total) {
                int k = e, ro;
                const int line = nl == 1 ? 0 : udiv22(e, L, rL, &k);
                const int i = line_at(line, &ro);
                vreg[u] = a.vhat[(int64_t)k * inner + i];
            }
        }
    }
    // one pass over the padded lines; consecutive threads take consecutive
    // lines, i.e. consecutive columns of the source: coalesced.  Four
    // elements' loads per thread are issued before any LDS store.
    for (int e0 = threadIdx.x; e0 < total; e0 += 4 * (int)blockDim.x) {
        cpx<T> va[4], vv[4];
        int at[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int e = min(e0 + u * (int)blockDim.x, total - 1);   // past the end: not stored
            int line = 0, ro;
            const int k = nl == 1 ? e : udiv22(e, nl, rnl, &line);
            const int i = line_at(line, &ro);
            const int kin = INP ? unpadL(k, m, L) : k;
            at[u] = line * L + k;
            va[u] = cpx<T>{(T)0, (T)0};
            if (kin >= 0) va[u] = src[((int64_t)ro * nin + kin) * inner + i];
            if (OP == 2 && LONG) vv[u] = a.vhat[(int64_t)k * inner + i];
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
            if (e0 + u * (int)blockDim.x < total) {
                A[at[u]] = va[u];
                if (OP == 2 && LONG) V[at[u]] = vv[u];
            }
        }
    }
    __syncthreads();
    cpx<T>* R = A;
    if (LONG) {
        if (OP == 1) {
            fft_lds_1<T, 1>(A, L, nl, f);
        } else {
            fft_lds_1<T, -1>(A, L, nl, f);
            if (OP == 2) {
                for (int e = threadIdx.x; e < nl * L; e += blockDim.x) A[e] = cmul(A[e], V[e]);
                __syncthreads();
                fft_lds_1<T, 1>(A, L, nl, f);
            }
        }
    } else if (OP == 1) {
        R = fft_lds<T, 1>(A, B, L, nl, f);
    } else {
        R = fft_lds<T, -1>(A, B, L, nl, f);
        if (OP == 2) {
#pragma unroll
            for (int u = 0; u < kMidV; u++) {
                const int e = threadIdx.x + u * (int)blockDim.x;
                if (e < total) R[e] = cmul(R[e], vreg[u]);
            }
            __syncthreads();
            cpx<T>* other = (R == A) ? B : A;
            R = fft_lds<T, 1>(R, other, L, nl, f);
        }
    }
    for (int e = threadIdx.x; e < nl * nout; e += blockDim.x) {
        int line = 0, ro;
        const int k = nl == 1 ? e : udiv22(e, nl, rnl, &line);
        const int i = line_at(line, &ro);
        const int pos = OUTP ? wrapL(k - m, L) : k;
        dst[((int64_t)ro * nout + k) * inner + i] = R[line * L + pos];
    }
}

// ---- column pass of the Hermitian 2D product.  The row transforms of a
// Hermitian vector satisfy R_{-i}(k) = conj R_i(k), so buf1 holds rows
// i = 0..m only, and column k (over i mod L) is a Hermitian sequence: its
// transform is real, and so is vhat.  Two columns therefore share one
// complex FFT: Z = c1 + i c2 transforms to X1 + i X2 with X1, X2 the real
// transforms; Y = vhat_1 X1 + i vhat_2 X2 transforms back to y1 + i y2 with
// y1, y2 Hermitian, so y1(i) = (Z(i) + conj Z(-i))/2 and
// y2(i) = (Z(i) - conj Z(-i))/(2i).  Rows i = 0..m of both columns go to
// buf2.  Line = a pair of adjacent columns (2c, 2c+1); an odd L leaves the
// last pair with one column.
// Two adjacent complex values p[0], p[1] (p[1] only if `two`); in single
// precision with `vec` (an even offset from a 16-byte aligned base, both
// present) one 16-byte access instead of two: the column pairs' accesses
// are strided by a whole row, so each one is a separate cache line.
template <typename T>
__device__ __forceinline__ void load_pair(const cpx<T>* p, bool two, bool vec, cpx<T>* a, cpx<T>* b) {
    if constexpr (std::is_same<T, float>::value) {
        if (vec) {
            const float4 q = *reinterpret_cast<const float4*>(p);
            *a = cpx<T>{q.x, q.y};
            *b = cpx<T>{q.z, q.w};
            return;
        }
    }
    *a = p[0];
    *b = two ? p[1] : cpx<T>{(T)0, (T)0};
}
template <typename T>
__device__ __forceinline__ void store_pair(cpx<T>* p, bool two, bool vec, cpx<T> a, cpx<T> b) {
    if constexpr (std::is_same<T, float>::value) {
        if (vec) {
            *reinterpret_cast<float4*>(p) = make_float4(a.x, a.y, b.x, b.y);
            return;
        }
    }
    p[0] = a;
    if (two) p[1] = b;
}

template <typename T>
__global__ void __launch_bounds__(512) k_mv_mid_herm(MvArgs<T> a, int lpb) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int L = a.L, m = a.m, R1 = m + 1;
    const int npair = (L + 1) >> 1;
    cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* B = A + (size_t)lpb * L;
    const FftDev<T> f = lds_twiddles(a.f, B + (size_t)lpb * L);
    const int64_t nlines = (int64_t)a.nrhs * npair;
    const int64_t l0 = (int64_t)xcd_block() * lpb;
    const int nl = (int)min<int64_t>(lpb, nlines - l0);
    if (lines_idle(a, l0, nl, npair)) return;
    // the block's pairs: system r0 from pair c0 on, wrapping at most once
    // (nl <= npair)
    const int r0 = (int)(l0 / npair), c0 = (int)(l0 - (int64_t)r0 * npair);
    auto pair_at = [&](int line, int* r) {
        int c = c0 + line;
        *r = r0;
        if (c >= npair) {
            c -= npair;
            *r = r0 + 1;
        }
        return c;
    };
    const int total = nl * L;
    const float rnl = 1.0f / (float)nl, rL = 1.0f / (float)L;
    const bool even = (L & 1) == 0;   // every pair complete, every pair offset even
    // the real vhat values of the elements this thread multiplies (element
    // e = tid + u blockDim, u < kMidV), loaded before the columns
    T v1[kMidV], v2[kMidV];
#pragma unroll
    for (int u = 0; u < kMidV; u++) {
        const int e = threadIdx.x + u * (int)blockDim.x;
        v1[u] = v2[u] = (T)0;
        if (e < total) {
            int k = e, r;
            const int line = nl == 1 ? 0 : udiv22(e, L, rL, &k);
            const int c = pair_at(line, &r);
            cpx<T> h1, h2;
            load_pair<T>(a.vhat + (int64_t)k * L + 2 * c, 2 * c + 1 < L, even, &h1, &h2);
            v1[u] = h1.x;
            v2[u] = h2.x;
        }
    }
    // the padded columns: element e -> (position k = e / nl, pair e mod nl),
    // so consecutive threads read consecutive pairs (adjacent columns)
    const cpx<T>* src = a.buf1;
    for (int e0 = threadIdx.x; e0 < total; e0 += 4 * (int)blockDim.x) {
        cpx<T> z[4];
        int at[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int e = min(e0 + u * (int)blockDim.x, total - 1);   // past the end: not stored
            int line = 0, r;
            const int k = nl == 1 ? e : udiv22(e, nl, rnl, &line);
            const int c = pair_at(line, &r);
            at[u] = line * L + k;
            z[u] = cpx<T>{(T)0, (T)0};
            const int jj = unpadL(k, m, L);
            if (jj >= 0) {
                const int i = jj - m, ia = i < 0 ? -i : i;
                const int64_t row = ((int64_t)r * R1 + ia) * L + 2 * c;
                cpx<T> w1, w2;
                load_pair<T>(src + row, 2 * c + 1 < L, even, &w1, &w2);
                if (i < 0) {
                    w1.y = -w1.y;
                    w2.y = -w2.y;
                }
                z[u] = cpx<T>{w1.x - w2.y, w1.y + w2.x};
            }
        }
#pragma unroll
        for (int u = 0; u < 4; u++)
            if (e0 + u * (int)blockDim.x < total) A[at[u]] = z[u];
    }
    __syncthreads();
    cpx<T>* R = fft_lds<T, -1>(A, B, L, nl, f);
#pragma unroll
    for (int u = 0; u < kMidV; u++) {
        const int e = threadIdx.x + u * (int)blockDim.x;
        if (e < total) R[e] = cpx<T>{R[e].x * v1[u], R[e].y * v2[u]};
    }
    __syncthreads();
    R = fft_lds<T, 1>(R, R == A ? B : A, L, nl, f);
    cpx<T>* dst = a.buf2;
    for (int e = threadIdx.x; e < nl * R1; e += blockDim.x) {
        int line = 0, r;
        const int i = nl == 1 ? e : udiv22(e, nl, rnl, &line);
        const int c = pair_at(line, &r);
        const cpx<T> zp = R[line * L + i], zm = R[line * L + (i == 0 ? 0 : L - i)];
        const int64_t row = ((int64_t)r * R1 + i) * L + 2 * c;
        store_pair<T>(dst + row, 2 * c + 1 < L, even, cpx<T>{(T)0.5 * (zp.x + zm.x), (T)0.5 * (zp.y - zm.y)},
                      cpx<T>{(T)0.5 * (zp.y + zm.y), (T)-0.5 * (zp.x - zm.x)});
    }
}

// ---- last pass: inverse FFT along the last axis, extract J_m, finish A p
// (for d=1 the whole product happens here, starting from the padded input).
// The per-line sums (p^H A p; for RESID ||r||^2 and r^H P r) are formed in a
// fixed order: every element's term goes to an LDS array, then one
// wavefront per line adds its lanes' strided partial sums and a shuffle tree
// finishes them, so a product is bitwise reproducible from launch to launch.
template <typename T, int DIM, int MODE, bool LONG>
__global__ void __launch_bounds__(LONG ? 1024 : 512) k_mv_last(MvArgs<T> a, int lpb) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int L = a.L, W = a.W, m = a.m;
    cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* B = A + (size_t)lpb * L;
    const FftDev<T> f = LONG ? a.f : lds_twiddles(a.f, B + (size_t)lpb * L);
    const int rows = a.rows;
    const int64_t nlines = (int64_t)rows * a.nrhs;
    const int64_t l0 = (int64_t)blockIdx.x * lpb;
    const int nl = (int)min<int64_t>(lpb, nlines - l0);
    if (lines_idle(a, l0, nl, rows)) return;
    cpx<T>* R = A;
    if (DIM == 1) {
        // pad + forward + multiply + inverse on a single line per system
        for (int e = threadIdx.x; e < nl * L; e += blockDim.x) A[e] = cpx<T>{(T)0, (T)0};
        __syncthreads();
        for (int e = threadIdx.x; e < nl * W; e += blockDim.x) {
            const int line = e / W, jj = e - line * W;
            const int r = (int)(l0 + line);
            const int64_t idx = (int64_t)r * a.M + jj;
            cpx<T> val;
            if (MODE == MV_CG) {
                const CgState& s = a.st[r];
                cpx<T> pn = a.p[idx];
                if (s.active) {
                    cpx<T> z = (a.z && s.use_prec) ? a.z[idx] : a.r[idx];
                    if (s.use_prec && a.prec) { const T pr = a.prec[idx]; z.x *= pr; z.y *= pr; }
                    const T g = (T)s.gamma;
                    pn = cpx<T>{z.x + g * pn.x, z.y + g * pn.y};
                    a.p[idx] = pn;
                }
                val = pn;
            } else {
                val = MODE == MV_RESID ? a.x[idx] : a.in[idx];
            }
            const T d = a.D[jj];
            A[line * L + wrapL(jj - m, L)] = cpx<T>{d * val.x, d * val.y};
        }
        __syncthreads();
        if (LONG) {
            fft_lds_1<T, -1>(A, L, nl, f);
            for (int e = threadIdx.x; e < nl * L; e += blockDim.x) A[e] = cmul(A[e], a.vhat[e % L]);
            __syncthreads();
            fft_lds_1<T, 1>(A, L, nl, f);
        } else {
            R = fft_lds<T, -1>(A, B, L, nl, f);
            for (int e = threadIdx.x; e < nl * L; e += blockDim.x) R[e] = cmul(R[e], a.vhat[e % L]);
            __syncthreads();
            R = fft_lds<T, 1>(R, R == A ? B : A, L, nl, f);
        }
    } else {
        stage4(A, a.buf2 + l0 * L, nl * L);
        __syncthreads();
        if (LONG) fft_lds_1<T, 1>(A, L, nl, f);
        else R = fft_lds<T, 1>(A, B, L, nl, f);
    }
    // per-element terms of the line sums: the buffer the result is not in
    // (it holds nl * L >= nl * W doubles), or (LONG) the area after A
    double* term = LONG ? reinterpret_cast<double*>(A + (size_t)lpb * L)
                        : reinterpret_cast<double*>(R == A ? B : A);
    // line by line, four elements' loads per thread before any store (as in
    // the first pass).  Hermitian passes (rows i = 0..m): row i > 0 also
    // writes row -i as its conjugates and counts twice in the sums; row 0
    // computes k >= 0, writes k < 0 as their conjugates and keeps the centre
    // real, so the vectors stay exactly Hermitian; b is taken symmetrised,
    // (b_j + conj b_{M-1-j}) / 2, as at the start of the solve.
    for (int line = 0; line < nl; line++) {
        const int64_t gl = l0 + line;
        const int r = (int)(gl / rows);
        const int64_t rowi = gl - (int64_t)r * rows;
        const int64_t rowj = (a.herm ? rowi + m : rowi) * W;
        const int64_t base = (int64_t)r * a.M + rowj;
        const int64_t mbase = (int64_t)r * a.M + a.M - 1 - rowj;   // mirror of (row, jj) is mbase - jj
        const bool row0 = a.herm && rowi == 0;
        const T s2 = (T)a.sig2[r];
        const cpx<T>* Rl = R + line * L;
        double* tl = term + line * W;
        for (int j0 = threadIdx.x; j0 < W; j0 += 4 * (int)blockDim.x) {
            cpx<T> xv[4], bv[4], bm[4];
            T dv[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int jj = min(j0 + u * (int)blockDim.x, W - 1);   // past the end: not stored
                const int64_t idx = base + jj;
                dv[u] = a.D[rowj + jj];
                if (MODE == MV_APPLY) xv[u] = a.in[idx];
                else if (MODE == MV_CG) xv[u] = a.p[idx];
                else {
                    xv[u] = a.x[idx];
                    bv[u] = a.b[idx];
                    if (a.herm) bm[u] = a.b[mbase - jj];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int jj = j0 + u * (int)blockDim.x;
                if (jj >= W) continue;
                if (row0 && jj < m) {   // written as the mirror of 2m - jj
                    if (MODE != MV_APPLY) tl[jj] = 0.0;
                    continue;
                }
                const bool mirror = a.herm && !(row0 && jj == m);
                const bool centre = row0 && jj == m;
                const double twice = mirror ? 2.0 : 1.0;
                const int64_t idx = base + jj;
                const cpx<T> o = Rl[wrapL(jj - m, L)];
                const T d = dv[u];
                if (MODE == MV_APPLY) {
                    const cpx<T> in = xv[u];
                    a.out[idx] = cpx<T>{d * o.x + s2 * in.x, d * o.y + s2 * in.y};
                } else if (MODE == MV_CG) {
                    double t = 0.0;
                    if (a.st[r].active) {
                        const cpx<T> pv = xv[u];
                        cpx<T> qv = cpx<T>{d * o.x + s2 * pv.x, d * o.y + s2 * pv.y};
                        if (centre) qv.y = (T)0;
                        a.q[idx] = qv;
                        if (mirror) a.q[mbase - jj] = cpx<T>{qv.x, -qv.y};
                        t = twice * ((double)pv.x * (double)qv.x + (double)pv.y * (double)qv.y);
                    }
                    tl[jj] = t;
                } else {  // RESID: r = b - A x for systems flagged for restart; p = 0
                    double t = 0.0;
                    if (a.st[r].pad) {  // pad doubles as the restart flag
                        const cpx<T> x0 = xv[u];
                        cpx<T> b0 = bv[u];
                        if (a.herm) b0 = cpx<T>{(T)0.5 * (b0.x + bm[u].x), (T)0.5 * (b0.y - bm[u].y)};
                        cpx<T> rv = cpx<T>{b0.x - (d * o.x + s2 * x0.x), b0.y - (d * o.y + s2 * x0.y)};
                        if (centre) rv.y = (T)0;
                        a.r[idx] = rv;
                        a.p[idx] = cpx<T>{(T)0, (T)0};
                        if (mirror) {
                            a.r[mbase - jj] = cpx<T>{rv.x, -rv.y};
                            a.p[mbase - jj] = cpx<T>{(T)0, (T)0};
                        }
                        t = twice * ((double)rv.x * rv.x + (double)rv.y * rv.y);
                    }
                    tl[jj] = t;
                }
            }
        }
    }
    if (MODE == MV_APPLY) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
    // one wavefront per line: strided partial sums, then a shuffle tree
    auto line_sums = [&](double* slot) {
        __syncthreads();
        for (int line = wave; line < nl; line += nwave) {
            double sum = 0.0;
            for (int jj = lane; jj < W; jj += 64) sum += term[line * W + jj];
            sum = warp_sum(sum);
            if (lane == 0) slot[l0 + line] = sum;
        }
    };
    if (MODE == MV_CG) {
        line_sums(slot_pq(a));
    } else {
        line_sums(slot_rr(a));
        __syncthreads();
        // r^H P r: the same terms scaled by the diagonal preconditioner
        for (int line = 0; line < nl; line++) {
            const int64_t gl = l0 + line;
            const int r = (int)(gl / rows);
            const int64_t rowi = gl - (int64_t)r * rows;
            const int64_t base = (int64_t)r * a.M + (a.herm ? rowi + m : rowi) * W;
            const CgState& s = a.st[r];
            for (int jj = threadIdx.x; jj < W; jj += blockDim.x) {
                const double pr = (s.use_prec && a.prec) ? (double)a.prec[base + jj] : 1.0;
                term[line * W + jj] = pr * term[line * W + jj];
            }
        }
        line_sums(slot_rz(a));
    }
}

// ---- CG vector updates (grid: x = chunks, y = system): x += alpha p,
// r -= alpha q, and per-block sums of ||r||^2 and r^H P r (INIT: r = b,
// x = p = 0, and ||b||^2) into the block's slots
template <typename T, bool INIT>
__global__ void __launch_bounds__(256) k_cg_vec(MvArgs<T> a) {
    __shared__ double red[16];
    __shared__ double pq_all;   // not in red: block_sum reuses every slot of red
    const int r = blockIdx.y;
    const CgState& s = a.st[r];
    double rr = 0.0, rz = 0.0, bb = 0.0;
    const bool act = INIT || s.active;
    if (act) {
        double alpha = 0.0;
        if (!INIT) {
            // p^H A p from the per-line slots of the matrix product
            double pq = 0.0;
            for (int i = threadIdx.x; i < a.rows; i += blockDim.x) pq += slot_pq(a)[(int64_t)r * a.rows + i];
            pq = block_sum(pq, red);
            if (threadIdx.x == 0) pq_all = pq;
            __syncthreads();
            alpha = s.rz / pq_all;
        }
        const T al = (T)alpha;
        for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < a.M; j += (int64_t)gridDim.x * blockDim.x) {
            const int64_t idx = (int64_t)r * a.M + j;
            cpx<T> rv;
            if (INIT) {
                rv = a.b[idx];
                if (a.herm) {   // exactly Hermitian from the start: (b_j + conj b_{M-1-j}) / 2
                    const cpx<T> bm = a.b[(int64_t)r * a.M + (a.M - 1 - j)];
                    rv = cpx<T>{(T)0.5 * (rv.x + bm.x), (T)0.5 * (rv.y - bm.y)};
                }
                a.r[idx] = rv;
                a.x[idx] = cpx<T>{(T)0, (T)0};
                a.p[idx] = cpx<T>{(T)0, (T)0};
                bb += (double)rv.x * rv.x + (double)rv.y * rv.y;
            } else {
                const cpx<T> pv = a.p[idx], qv = a.q[idx];
                cpx<T> xv = a.x[idx];
                rv = a.r[idx];
                xv.x += al * pv.x; xv.y += al * pv.y;
                rv.x -= al * qv.x; rv.y -= al * qv.y;
                a.x[idx] = xv;
                a.r[idx] = rv;
            }
            const double n2 = (double)rv.x * rv.x + (double)rv.y * rv.y;
            rr += n2;
            rz += ((s.use_prec && a.prec) ? (double)a.prec[idx] : 1.0) * n2;
        }
    }
    rr = block_sum(rr, red);
    rz = block_sum(rz, red);
    if (INIT) bb = block_sum(bb, red);
    if (threadIdx.x == 0) {
        double* sl = slot_vec(a) + ((int64_t)r * kGmax + blockIdx.x) * 3;
        sl[0] = rr;
        sl[1] = rz;
        sl[2] = bb;
    }
}

// ---- scalar finalisation of system blockIdx.x from the nblk block slots of
// k_cg_vec, in a fixed order (strided per-thread sums, then a block tree).
// A kernel of its own: a last-block pass would serialise nblk same-address
// atomics at the L2.
template <typename T, bool INIT>
__global__ void __launch_bounds__(256) k_cg_fin(MvArgs<T> a, int nblk, double* hist, int64_t hist_cap) {
    __shared__ double red[16];
    const int k = blockIdx.x;
    double rrk = 0.0, rzk = 0.0, bbk = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
        const double* sl = slot_vec(a) + ((int64_t)k * kGmax + b) * 3;
        rrk += sl[0];
        rzk += sl[1];
        bbk += sl[2];
    }
    rrk = block_sum(rrk, red);
    rzk = block_sum(rzk, red);
    bbk = block_sum(bbk, red);
    if (threadIdx.x != 0) return;
    CgState& t = a.st[k];
    if (INIT) {
        t.bb = bbk;
        t.rz = rzk;
        t.gamma = 0.0;
        t.iters = 0;
        t.relres = t.bb > 0.0 ? sqrt(rrk / t.bb) : 0.0;
        t.best = t.relres;
        t.active = (t.bb > 0.0) && (rrk > t.rho2 * t.bb);
    } else if (t.active) {
        // with an operator preconditioner r^H z comes after z = P r
        if (!(a.z && t.use_prec)) {
            t.gamma = rzk / t.rz;
            t.rz = rzk;
        }
        t.iters += 1;
        t.relres = sqrt(rrk / t.bb);
        if (k == 0 && hist && t.iters <= hist_cap) hist[t.iters - 1] = t.relres;
        if (!(t.relres == t.relres) || !(t.gamma == t.gamma)) t.active = 0;  // NaN: stop
        else if (rrk <= t.rho2 * t.bb) t.active = 0;
    }
}

// ---- the same CG update for small systems: one block per system, no
// cross-block reduction (no counter, no last-block pass)
template <typename T>
__global__ void __launch_bounds__(1024) k_cg_vec1(MvArgs<T> a, double* hist, int64_t hist_cap) {
    __shared__ double red[16];
    __shared__ double bc[2];
    __shared__ int act;
    const int r = blockIdx.x;
    if (threadIdx.x == 0) act = a.st[r].active;
    __syncthreads();
    if (!act) return;
    const CgState& s = a.st[r];
    double pq = 0.0;
    for (int i = threadIdx.x; i < a.rows; i += blockDim.x) pq += slot_pq(a)[(int64_t)r * a.rows + i];
    pq = block_sum(pq, red);
    if (threadIdx.x == 0) bc[0] = s.rz / pq;
    __syncthreads();
    const T al = (T)bc[0];
    const bool up = s.use_prec && a.prec;
    double rr = 0.0, rz = 0.0;
    for (int64_t j = threadIdx.x; j < a.M; j += blockDim.x) {
        const int64_t idx = (int64_t)r * a.M + j;
        const cpx<T> pv = a.p[idx], qv = a.q[idx];
        cpx<T> xv = a.x[idx], rv = a.r[idx];
        xv.x += al * pv.x; xv.y += al * pv.y;
        rv.x -= al * qv.x; rv.y -= al * qv.y;
        a.x[idx] = xv;
        a.r[idx] = rv;
        const double n2 = (double)rv.x * rv.x + (double)rv.y * rv.y;
        rr += n2;
        rz += (up ? (double)a.prec[idx] : 1.0) * n2;
    }
    rr = block_sum(rr, red);
    rz = block_sum(rz, red);
    if (threadIdx.x == 0) {
        CgState& t = a.st[r];
        if (!(a.z && t.use_prec)) {
            t.gamma = rz / t.rz;
            t.rz = rz;
        }
        t.iters += 1;
        t.relres = sqrt(rr / t.bb);
        if (r == 0 && hist && t.iters <= hist_cap) hist[t.iters - 1] = t.relres;
        if (!(t.relres == t.relres) || !(t.gamma == t.gamma)) t.active = 0;  // NaN: stop
        else if (rr <= t.rho2 * t.bb) t.active = 0;
    }
}

// ---- the last pass fused with the CG update for small 2D systems: one
// block per system runs the inverse row transforms of all the system's lines
// (rows 0..m in the Hermitian passes, else all W rows), forms q = D o +
// sigma^2 p and p^H q, then alpha, x += alpha p, r -= alpha q, ||r||^2,
// r^H P r and the step scalars, as k_mv_last followed by k_cg_vec1 do,
// without the kernel boundary between them.  Each thread takes the same
// elements in both halves (and, Hermitian, their mirrors), so q stays in
// registers, and all their loads are issued before the transforms.  The
// host keeps the lines within 4096 points (two LDS line buffers and the
// twiddles), hence at most four elements per thread.
template <typename T>
__global__ void __launch_bounds__(1024) k_mv_last_cg1(MvArgs<T> a, double* hist, int64_t hist_cap) {
    constexpr int KE = 4;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[16];
    __shared__ double bc;
    const int L = a.L, W = a.W, m = a.m, rows = a.rows;
    const int r = blockIdx.x;
    if (!a.st[r].active) return;   // block-uniform, before any barrier
    const CgState& s = a.st[r];
    const bool up = s.use_prec && a.prec;
    const int tot = rows * W;
    const float rW = 1.0f / (float)W;
    const int64_t sys = (int64_t)r * a.M;
    // kind: 0 none, 1 one element, 2 an element and its mirror, 3 the centre
    int kind[KE], pos[KE];
    int64_t ix[KE];
    cpx<T> pv[KE], xv[KE], rv[KE];
    T dv[KE], pr[KE];
#pragma unroll
    for (int k = 0; k < KE; k++) {
        const int e = threadIdx.x + k * (int)blockDim.x;
        kind[k] = 0;
        pos[k] = 0;
        ix[k] = sys;
        if (e < tot) {
            int jj;
            const int rowi = udiv22(e, W, rW, &jj);
            const bool row0 = a.herm && rowi == 0;
            if (!(row0 && jj < m)) {   // row 0, k < 0: the mirror of 2m - jj
                kind[k] = !a.herm ? 1 : (row0 && jj == m ? 3 : 2);
                const int64_t rowj = (int64_t)(a.herm ? rowi + m : rowi) * W;
                ix[k] = sys + rowj + jj;
                pos[k] = rowi * L + wrapL(jj - m, L);
                dv[k] = a.D[rowj + jj];
                pv[k] = a.p[ix[k]];
                xv[k] = a.x[ix[k]];
                rv[k] = a.r[ix[k]];
                pr[k] = up ? a.prec[ix[k]] : (T)1;
            }
        }
    }
    cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* B = A + (size_t)rows * L;
    const FftDev<T> f = lds_twiddles(a.f, B + (size_t)rows * L);
    stage4(A, a.buf2 + (int64_t)r * rows * L, rows * L);
    __syncthreads();
    cpx<T>* R = fft_lds<T, 1, kCg1MaxR<T>>(A, B, L, rows, f);
    const T s2 = (T)a.sig2[r];
    cpx<T> qv[KE];
    double pq = 0.0;
#pragma unroll
    for (int k = 0; k < KE; k++) {
        if (kind[k] == 0) continue;
        const cpx<T> o = R[pos[k]];
        cpx<T> q = cpx<T>{dv[k] * o.x + s2 * pv[k].x, dv[k] * o.y + s2 * pv[k].y};
        if (kind[k] == 3) q.y = (T)0;   // the centre stays real
        qv[k] = q;
        pq += (kind[k] == 2 ? 2.0 : 1.0) * ((double)pv[k].x * (double)q.x + (double)pv[k].y * (double)q.y);
    }
    pq = block_sum(pq, red);
    if (threadIdx.x == 0) bc = s.rz / pq;
    __syncthreads();
    const T al = (T)bc;
    double rr = 0.0, rz = 0.0;
#pragma unroll
    for (int k = 0; k < KE; k++) {
        if (kind[k] == 0) continue;
        cpx<T> x1 = xv[k], r1 = rv[k];
        x1.x += al * pv[k].x; x1.y += al * pv[k].y;
        r1.x -= al * qv[k].x; r1.y -= al * qv[k].y;
        a.x[ix[k]] = x1;
        a.r[ix[k]] = r1;
        const double n2 = (double)r1.x * r1.x + (double)r1.y * r1.y;
        double mult = 1.0;
        if (kind[k] == 2) {
            const int64_t mi = sys + (a.M - 1) - (ix[k] - sys);
            a.x[mi] = cpx<T>{x1.x, -x1.y};
            a.r[mi] = cpx<T>{r1.x, -r1.y};
            mult = 2.0;
        }
        rr += mult * n2;
        rz += mult * (double)pr[k] * n2;
    }
    rr = block_sum(rr, red);
    rz = block_sum(rz, red);
    if (threadIdx.x == 0) {
        CgState& t = a.st[r];
        if (!(a.z && t.use_prec)) {
            t.gamma = rz / t.rz;
            t.rz = rz;
        }
        t.iters += 1;
        t.relres = sqrt(rr / t.bb);
        if (r == 0 && hist && t.iters <= hist_cap) hist[t.iters - 1] = t.relres;
        if (!(t.relres == t.relres) || !(t.gamma == t.gamma)) t.active = 0;  // NaN: stop
        else if (rr <= t.rho2 * t.bb) t.active = 0;
    }
}

// ---- whole CG iterations in one block per system, for Hermitian 2D systems
// whose column pass fits the block's LDS.  Each launch runs up to `niter`
// iterations of exactly the recurrences of the three-pass iteration (first
// pass with the direction update, column pairs with FFT(v), last pass fused
// with the vector update), but the lines never leave LDS and the vectors
// never leave registers: a small system's iteration then costs one CU's
// FFT stages and barriers instead of three kernels' launch and memory
// latencies.  Two LDS regions of npair*L values (npair = ceil(L/2) column
// pairs) take every stage in turn; the twiddles follow them.
//
// A thread owns the padded row positions e = tid + k*blockDim (k < KE) of
// rows 0..m: the element of J_m at (row i + m, jj = unpad(e mod L)) with its
// mirror, except in row 0 where jj < m is the mirror of 2m - jj and the
// owner of 2m - jj writes it; it multiplies KV column-pass values by FFT(v).
// Step scalars are double block sums formed in the same order by every
// thread.  Two register budgets: (KE, KV) = (3, 6) and (5, 9).
constexpr int kBlkE = 5;   // padded row positions per thread: (m+1) L <= 5120
constexpr int kBlkV = 9;   // column-pass values per thread: ceil(L/2) L <= 9216

template <typename T>
__device__ __forceinline__ int64_t blk_index(int e, int L, float rL, int m, int W) {
    int kk;
    const int rowi = udiv22(e, L, rL, &kk);
    return (int64_t)(rowi + m) * W + unpadL(kk, m, L);
}

template <typename T, int KE, int KV, int MAXR>
__global__ void __launch_bounds__(1024) k_cg_block(MvArgs<T> a, int niter, double* hist, int64_t hist_cap) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[3][16];
    const int L = a.L, W = a.W, m = a.m, rows = m + 1;
    const int npair = (L + 1) >> 1;
    const int r = blockIdx.x;
    if (!a.st[r].active) return;   // block-uniform, before any barrier
    const int64_t sys = (int64_t)r * a.M;
    cpx<T>* U = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* V = U + (size_t)npair * L;
    const FftDev<T> f = lds_twiddles(a.f, V + (size_t)npair * L);
    const int nw = (blockDim.x + 63) >> 6;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    // sum over the block, the same value in every thread (slots of red are
    // rewritten only after later barriers)
    auto allsum = [&](double v, double* rd) {
        v = warp_sum(v);
        if (lane == 0) rd[wid] = v;
        __syncthreads();
        double t = 0.0;
        for (int i = 0; i < nw; i++) t += rd[i];
        return t;
    };
    // CG state: identical in every thread
    const CgState& s0 = a.st[r];
    double rz = s0.rz, gamma = s0.gamma, relres = s0.relres;
    const double bb = s0.bb, rho2 = s0.rho2;
    const int use_prec = s0.use_prec;
    int iters = s0.iters, active = 1;
    const bool up = use_prec && a.prec;
    const T s2 = (T)a.sig2[r];
    // owned positions; kind 0: zero padding, 1: row 0 mirror (not owned),
    // 2: an element and its mirror, 3: the centre (real)
    const int tot = rows * L;
    const float rL = 1.0f / (float)L;
    int kind[KE], mpos[KE];
    cpx<T> pv[KE], xv[KE], rv[KE];
    T dv[KE], pr[KE];
#pragma unroll
    for (int k = 0; k < KE; k++) {
        const int e = threadIdx.x + k * (int)blockDim.x;
        kind[k] = 1;
        mpos[k] = -1;
        dv[k] = pr[k] = (T)0;
        pv[k] = xv[k] = rv[k] = cpx<T>{(T)0, (T)0};
        if (e >= tot) continue;
        int kk;
        const int rowi = udiv22(e, L, rL, &kk);
        const int jj = unpadL(kk, m, L);
        if (jj < 0) { kind[k] = 0; continue; }
        if (rowi == 0 && jj < m) continue;
        kind[k] = (rowi == 0 && jj == m) ? 3 : 2;
        if (rowi == 0 && jj > m) mpos[k] = wrapL(m - jj, L);   // position of 2m - jj
        const int64_t j = (int64_t)(rowi + m) * W + jj;
        dv[k] = a.D[j];
        pv[k] = a.p[sys + j];
        xv[k] = a.x[sys + j];
        rv[k] = a.r[sys + j];
        pr[k] = a.prec ? a.prec[sys + j] : (T)1;
    }
    // FFT(v) of the column-pass values this thread multiplies (line c = e / L,
    // position e mod L), real parts of columns 2c and 2c + 1
    const int ctot = npair * L;
    T v1[KV], v2[KV];
#pragma unroll
    for (int u = 0; u < KV; u++) {
        const int e = threadIdx.x + u * (int)blockDim.x;
        v1[u] = v2[u] = (T)0;
        if (e < ctot) {
            int kk;
            const int c = udiv22(e, L, rL, &kk);
            v1[u] = a.vhat[(int64_t)kk * L + 2 * c].x;
            if (2 * c + 1 < L) v2[u] = a.vhat[(int64_t)kk * L + 2 * c + 1].x;
        }
    }
    const float rnp = 1.0f / (float)npair;
    for (int it = 0; it < niter && active; it++) {
        // direction p = z + gamma p (z = P r), then D p padded into rows 0..m
        const T g = (T)gamma;
#pragma unroll
        for (int k = 0; k < KE; k++) {
            const int e = threadIdx.x + k * (int)blockDim.x;
            if (e >= tot) continue;
            if (kind[k] == 0) { U[e] = cpx<T>{(T)0, (T)0}; continue; }
            if (kind[k] == 1) continue;
            cpx<T> z = rv[k];
            if (use_prec) { z.x *= pr[k]; z.y *= pr[k]; }
            pv[k] = cpx<T>{z.x + g * pv[k].x, z.y + g * pv[k].y};
            const cpx<T> d = cpx<T>{dv[k] * pv[k].x, dv[k] * pv[k].y};
            U[e] = d;
            if (mpos[k] >= 0) U[mpos[k]] = cpx<T>{d.x, -d.y};
        }
        __syncthreads();
        cpx<T>* R = fft_lds<T, -1, MAXR>(U, V, L, rows, f);
        cpx<T>* C = R == U ? V : U;
        // column pairs: z = w1 + i w2 down padded position k; rows i < 0 are
        // the conjugates of rows -i.  Consecutive threads take consecutive
        // pairs of one position, so the two row reads are contiguous (and the
        // one write strided)
        for (int t = threadIdx.x; t < ctot; t += blockDim.x) {
            int c;
            const int kk = udiv22(t, npair, rnp, &c);
            const int e = c * L + kk;
            const int jj = unpadL(kk, m, L);
            cpx<T> z = cpx<T>{(T)0, (T)0};
            if (jj >= 0) {
                const int i = jj - m, ia = i < 0 ? -i : i;
                cpx<T> w1 = R[ia * L + 2 * c];
                cpx<T> w2 = 2 * c + 1 < L ? R[ia * L + 2 * c + 1] : cpx<T>{(T)0, (T)0};
                if (i < 0) { w1.y = -w1.y; w2.y = -w2.y; }
                z = cpx<T>{w1.x - w2.y, w1.y + w2.x};
            }
            C[e] = z;
        }
        __syncthreads();
        cpx<T>* Q = fft_lds<T, -1, MAXR>(C, R, L, npair, f);
#pragma unroll
        for (int u = 0; u < KV; u++) {
            const int e = threadIdx.x + u * (int)blockDim.x;
            if (e < ctot) Q[e] = cpx<T>{Q[e].x * v1[u], Q[e].y * v2[u]};
        }
        __syncthreads();
        Q = fft_lds<T, 1, MAXR>(Q, Q == U ? V : U, L, npair, f);
        // split the pairs back into rows 0..m
        cpx<T>* S = Q == U ? V : U;
        for (int e = threadIdx.x; e < rows * npair; e += blockDim.x) {
            int c;
            const int i = udiv22(e, npair, rnp, &c);
            const cpx<T> zp = Q[c * L + i], zm = Q[c * L + (i == 0 ? 0 : L - i)];
            S[i * L + 2 * c] = cpx<T>{(T)0.5 * (zp.x + zm.x), (T)0.5 * (zp.y - zm.y)};
            if (2 * c + 1 < L) S[i * L + 2 * c + 1] = cpx<T>{(T)0.5 * (zp.y + zm.y), (T)-0.5 * (zp.x - zm.x)};
        }
        __syncthreads();
        cpx<T>* O = fft_lds<T, 1, MAXR>(S, Q, L, rows, f);
        // q = D o + sigma^2 p and p^H q; q is formed again from O (still in
        // LDS until the next iteration's first barrier) for the update
        auto q_at = [&](int k) {
            const cpx<T> o = O[threadIdx.x + k * (int)blockDim.x];
            cpx<T> q = cpx<T>{dv[k] * o.x + s2 * pv[k].x, dv[k] * o.y + s2 * pv[k].y};
            if (kind[k] == 3) q.y = (T)0;
            return q;
        };
        double pq = 0.0;
#pragma unroll
        for (int k = 0; k < KE; k++) {
            if (kind[k] < 2) continue;
            const cpx<T> q = q_at(k);
            pq += (kind[k] == 2 ? 2.0 : 1.0) * ((double)pv[k].x * (double)q.x + (double)pv[k].y * (double)q.y);
        }
        pq = allsum(pq, red[0]);
        const T al = (T)(rz / pq);
        double rr = 0.0, rzn = 0.0;
#pragma unroll
        for (int k = 0; k < KE; k++) {
            if (kind[k] < 2) continue;
            const cpx<T> q = q_at(k);
            xv[k].x += al * pv[k].x; xv[k].y += al * pv[k].y;
            rv[k].x -= al * q.x; rv[k].y -= al * q.y;
            const double n2 = (double)rv[k].x * rv[k].x + (double)rv[k].y * rv[k].y;
            const double mult = kind[k] == 2 ? 2.0 : 1.0;
            rr += mult * n2;
            rzn += mult * (up ? (double)pr[k] : 1.0) * n2;
        }
        rr = warp_sum(rr);
        rzn = warp_sum(rzn);
        if (lane == 0) {
            red[1][wid] = rr;
            red[2][wid] = rzn;
        }
        __syncthreads();
        rr = rzn = 0.0;
        for (int i = 0; i < nw; i++) {
            rr += red[1][i];
            rzn += red[2][i];
        }
        gamma = rzn / rz;
        rz = rzn;
        iters += 1;
        relres = sqrt(rr / bb);
        if (threadIdx.x == 0 && r == 0 && hist && iters <= hist_cap) hist[iters - 1] = relres;
        if (!(relres == relres) || !(gamma == gamma)) active = 0;   // NaN: stop
        else if (rr <= rho2 * bb) active = 0;
    }
    // vectors and state back to global memory (mirrors as conjugates)
#pragma unroll
    for (int k = 0; k < KE; k++) {
        if (kind[k] < 2) continue;
        const int64_t j = blk_index<T>(threadIdx.x + k * (int)blockDim.x, L, rL, m, W);
        a.p[sys + j] = pv[k];
        a.x[sys + j] = xv[k];
        a.r[sys + j] = rv[k];
        if (kind[k] == 2) {
            const int64_t mi = sys + (a.M - 1) - j;
            a.p[mi] = cpx<T>{pv[k].x, -pv[k].y};
            a.x[mi] = cpx<T>{xv[k].x, -xv[k].y};
            a.r[mi] = cpx<T>{rv[k].x, -rv[k].y};
        }
    }
    if (threadIdx.x == 0) {
        CgState& t = a.st[r];
        t.rz = rz;
        t.gamma = gamma;
        t.iters = iters;
        t.relres = relres;
        t.active = active;
    }
}

// finalise a restart (after MV_RESID), one block per system: new residual,
// fresh direction; the per-line sums are added in a fixed order (strided
// per-thread sums, then a block tree)
template <typename T>
__global__ void __launch_bounds__(256) k_cg_restart_fin(MvArgs<T> a, double accept2) {
    __shared__ double red[16];
    const int k = blockIdx.x;
    if (!a.st[k].pad) return;   // block-uniform
    double rr = 0.0, rz = 0.0;
    for (int i = threadIdx.x; i < a.rows; i += blockDim.x) {
        rr += slot_rr(a)[(int64_t)k * a.rows + i];
        rz += slot_rz(a)[(int64_t)k * a.rows + i];
    }
    rr = block_sum(rr, red);
    rz = block_sum(rz, red);
    if (threadIdx.x == 0) {
        CgState& t = a.st[k];
        t.rz = rz;
        t.gamma = 0.0;
        t.relres = t.bb > 0.0 ? sqrt(rr / t.bb) : 0.0;
        t.best = t.relres;
        // keep iterating while the true residual exceeds the acceptance level
        t.active = (t.bb > 0.0) && (rr > accept2 * t.rho2 * t.bb);
        t.pad = 0;
    }
}

template <typename T>
__global__ void k_copy_cpx(const cpx<T>* __restrict__ in, cpx<T>* __restrict__ out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i];
}

template <typename T>
__global__ void k_zero_cpx(cpx<T>* __restrict__ out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = cpx<T>{(T)0, (T)0};
}

template <typename T>
__global__ void k_jacobi(const T* __restrict__ D, const double* __restrict__ sig2, double nn, int64_t M, int nrhs,
                         T* __restrict__ prec) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M * nrhs) return;
    const int r = (int)(i / M);
    const double d = (double)D[i - (int64_t)r * M];
    prec[i] = (T)(1.0 / (nn * d * d + sig2[r]));
}

// a caller's diagonal preconditioner must be finite and positive (NaN fails
// the comparison)
template <typename T>
__global__ void k_check_diag(const T* __restrict__ d, int64_t n, int* __restrict__ bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !((double)d[i] > 0.0 && (double)d[i] <= 1.7976931348623157e308)) atomicOr(bad, 1);
}

// features of the learned preconditioner (see efgp_features)
template <int DIM>
__global__ void k_features(const double* __restrict__ D, const double2* __restrict__ v, int m, double h, double ell,
                           double nn, double s2, float* __restrict__ feats, float* __restrict__ jac) {
    const int W = 2 * m + 1, W2 = 4 * m + 1;
    int64_t M = 1;
    for (int l = 0; l < DIM; l++) M *= W;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    int64_t rem = j, vi = 0;
    int js[3];
    for (int l = DIM - 1; l >= 0; l--) { js[l] = (int)(rem % W) - m; rem /= W; }
    double jn2 = 0.0;
    for (int l = 0; l < DIM; l++) { vi = vi * W2 + (js[l] + 2 * m); jn2 += (double)js[l] * js[l]; }
    const double d2 = D[j] * D[j];
    // local magnitude of the Toeplitz vector: mean |v_k| over the box
    // |k_l - j_l| <= 2 (clipped to J_2m)
    double vs = 0.0;
    int cnt = 0;
    for (int a = -2; a <= 2; a++)
        for (int b = (DIM > 1 ? -2 : 0); b <= (DIM > 1 ? 2 : 0); b++)
            for (int c = (DIM > 2 ? -2 : 0); c <= (DIM > 2 ? 2 : 0); c++) {
                const int off[3] = {a, b, c};
                int64_t k = 0;
                bool ok = true;
                for (int l = 0; l < DIM; l++) {
                    const int jj = js[l] + off[l];
                    ok = ok && jj >= -2 * m && jj <= 2 * m;
                    k = k * W2 + (jj + 2 * m);
                }
                if (!ok) continue;
                const double2 vk = v[k];
                vs += sqrt(vk.x * vk.x + vk.y * vk.y);
                cnt++;
            }
    (void)vi;
    float* f = feats + j * EFGP_NFEAT;
    f[0] = (float)(h * sqrt(jn2) * ell);
    f[1] = (float)(0.1 * log(nn * d2 / s2 + 1e-300));
    f[2] = (float)(0.2 * log(s2));
    f[3] = (float)(0.5 * log(ell));
    f[4] = (float)(0.1 * log(vs / cnt / nn + 1e-12));
    if (jac) jac[j] = (float)(1.0 / (nn * d2 + s2));
}

template <typename T>
__global__ void k_float_to(const float* __restrict__ in, int64_t n, T* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (T)in[i];
}

// ------------------------------------------------------------------ host
// Long lines: the two-buffer passes would need more than 64 KB of LDS for
// one line (four line buffers in the pass with the FFT(v) columns), i.e.
// L > 1024 in double, L > 2048 in float.  Those passes keep one buffer
// (fft_lds_1, kLongThreads threads) and read the twiddles from global memory.
template <typename T> static bool long_lines(int L) { return 4 * (size_t)L * sizeof(cpx<T>) > 64 * 1024; }

template <typename T>
static MvArgs<T> make_args(Plan& P) {
    MvArgs<T> a{};
    a.r = static_cast<cpx<T>*>(P.r);
    a.p = static_cast<cpx<T>*>(P.p);
    a.q = static_cast<cpx<T>*>(P.q);
    a.x = static_cast<cpx<T>*>(P.x);
    a.b = static_cast<const cpx<T>*>(P.b);
    a.prec = static_cast<const T*>(P.prec);
    a.z = nullptr;
    a.D = static_cast<const T*>(P.Dt);
    a.vhat = static_cast<const cpx<T>*>(P.vhat);
    a.sig2 = P.sig2;
    a.st = P.st;
    a.buf1 = static_cast<cpx<T>*>(P.buf1);
    a.buf2 = static_cast<cpx<T>*>(P.buf2);
    a.part = P.part;
    a.rows = P.dim == 1 ? 1 : (P.dim == 2 ? P.W : P.W * P.W);
    // the one-buffer long-line passes keep to radices 2..5
    a.f.s = fft_shape(P.L, long_lines<T>(P.L) ? 5 : 16);
    a.f.tw = static_cast<const cpx<T>*>(P.twL);
    a.m = P.m;
    a.W = P.W;
    a.L = P.L;
    a.nrhs = P.nrhs;
    a.M = P.M;
    a.idle_skip = 0;
    a.herm = 0;
    return a;
}

// Lines per block: enough blocks to spread a pass over the CUs (the passes
// are latency bound at these sizes), within ~16 KB of LDS per block for the
// two line buffers (measured at L = 320, 64 systems: 16 KB, 3 lines, beats
// 32 KB, 6 lines, by 3%, and 12 KB, 2 lines, by 10%).
template <typename T>
static int lines_per_block(int L, int64_t nlines) {
    int cap = (int)(16 * 1024 / (2 * (size_t)L * sizeof(cpx<T>) + 2 * sizeof(double)));
    cap = std::max(1, std::min(cap, 32));
    const int want = (int)std::max<int64_t>(1, nlines / 512);
    return std::min(cap, want);
}
// About four points per thread: the passes are chains of latency (loads,
// FFT stages with a barrier each), so a long line is shared by up to 512
// threads rather than walked by 256.
static int threads_for(int lpb, int L) {
    int t = (lpb * L / 4 + 63) / 64 * 64;
    return std::max(64, std::min(512, t));
}
// A and B line buffers, twiddles, 2 lpb doubles of line sums (the column
// pass with the vhat product holds its vhat values in registers)
template <typename T>
static size_t lds_bytes(int lpb, int L) {
    return (2 * (size_t)lpb * L + L) * sizeof(cpx<T>) + 2 * (size_t)lpb * sizeof(double);
}

// Lines per block of a column (middle) pass (at most `inner`, the lines
// one row holds).  A block holding more adjacent columns (longer row pieces,
// up to 64 KB of LDS) was measured slower for large batches: fewer blocks
// per CU.
template <typename T>
static int mid_lines(int L, int64_t lines, int64_t inner) {
    int lp = lines_per_block<T>(L, lines);
    if (inner < lp) lp = (int)inner;
    return lp;
}


// Long lines per block of the row passes (first, last): at most kLongMax
// points, 64 KB of line buffer plus the last pass's line-sum terms.
template <typename T>
static int long_rows_per_block(int L, int W, int64_t nlines) {
    const size_t per = (size_t)L * sizeof(cpx<T>) + (size_t)W * sizeof(double);
    int lp = (int)std::min<size_t>((size_t)(kLongMax / L), (64 * 1024) / per);
    lp = std::max(1, lp);
    return (int)std::min<int64_t>(lp, std::max<int64_t>(1, nlines / 256));
}
template <typename T>
static size_t long_row_lds(int lp, int L, int W) {
    return (size_t)lp * L * sizeof(cpx<T>) + (size_t)lp * W * sizeof(double);
}
// Long column passes: adjacent columns per block (coalesced row pieces)
// within kLongMax points and 128 KB of LDS (two buffers with FFT(v)).
template <typename T>
static int long_mid_lines(int L, int64_t inner, bool vhat) {
    const size_t per = (size_t)L * sizeof(cpx<T>) * (vhat ? 2 : 1);
    int lp = (int)std::min<size_t>((size_t)(kLongMax / L), (128 * 1024) / per);
    lp = std::max(1, lp);
    return (int)std::min<int64_t>(lp, inner);
}
template <typename T>
static size_t long_mid_lds(int lp, int L, bool vhat) {
    return (size_t)lp * L * sizeof(cpx<T>) * (vhat ? 2 : 1);
}

static void lds_attr(const void* fn, size_t bytes) {
    if (bytes > 64 * 1024)
        EFGP_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

// Raise the LDS limit of every pass kernel this plan launches beyond 64 KB
// (a host call, made before any launch is captured).  Short lines: only the
// pass with the FFT(v) columns can exceed it (double at L = 1024: one line
// needs 64 KB + 16 B).
template <typename T, int DIM>
static void mv_lds_attrs(const Plan& P) {
    const int L = P.L, W = P.W;
    const int64_t inner2 = DIM == 2 ? L : (int64_t)L * L;
    if (!long_lines<T>(L)) {
        if (DIM < 2) return;
        const int lp = mid_lines<T>(L, (int64_t)P.nrhs * inner2, inner2);
        lds_attr((const void*)k_mv_mid<T, 1, 1, 2, false>, lds_bytes<T>(lp, L));
        if (DIM == 2) {   // the fused last pass, for either line count (rows 0..m, or all W)
            for (int rows : {P.m + 1, W})
                if ((int64_t)rows * L <= 4096)
                    lds_attr((const void*)k_mv_last_cg1<T>, (2 * (size_t)rows * L + L) * sizeof(cpx<T>));
        }
        return;
    }
    const int rows = DIM == 1 ? 1 : (DIM == 2 ? W : W * W);
    const int lpb = long_rows_per_block<T>(L, W, (int64_t)rows * P.nrhs);
    const size_t rb = long_row_lds<T>(lpb, L, W);
    lds_attr((const void*)k_mv_last<T, DIM, MV_APPLY, true>, rb);
    lds_attr((const void*)k_mv_last<T, DIM, MV_CG, true>, rb);
    lds_attr((const void*)k_mv_last<T, DIM, MV_RESID, true>, rb);
    if (DIM < 2) return;
    lds_attr((const void*)k_mv_first<T, DIM, MV_APPLY, true>, rb);
    lds_attr((const void*)k_mv_first<T, DIM, MV_CG, true>, rb);
    lds_attr((const void*)k_mv_first<T, DIM, MV_RESID, true>, rb);
    lds_attr((const void*)k_mv_mid<T, 1, 1, 2, true>, long_mid_lds<T>(long_mid_lines<T>(L, inner2, true), L, true));
    if (DIM == 3) {
        lds_attr((const void*)k_mv_mid<T, 1, 0, 0, true>, long_mid_lds<T>(long_mid_lines<T>(L, L, false), L, false));
        lds_attr((const void*)k_mv_mid<T, 0, 1, 1, true>, long_mid_lds<T>(long_mid_lines<T>(L, L, false), L, false));
    }
}

template <typename T>
static void mv_lds_attrs_dim(const Plan& P) {
    if (P.dim == 1) mv_lds_attrs<T, 1>(P);
    else if (P.dim == 2) mv_lds_attrs<T, 2>(P);
    else mv_lds_attrs<T, 3>(P);
}

template <typename T, int DIM, int MODE, bool LONG>
static void launch_mv_impl(Plan& P, const MvArgs<T>& a_in, hipStream_t s, bool last = true) {
    MvArgs<T> a = a_in;
    a.idle_skip = MODE == MV_CG ? 1 : 0;
    const int L = P.L, W = P.W;
    // Hermitian 2D passes transform rows 0..m only (a.rows = m + 1)
    const bool herm = a.herm != 0;
    if (herm && (DIM != 2 || LONG || MODE == MV_APPLY))
        throw StatusError{EFGP_EINVAL, "internal: Hermitian passes on an unsupported shape"};
    const int rows = herm ? a.rows : (DIM == 1 ? 1 : (DIM == 2 ? W : W * W));
    const int64_t nl = (int64_t)rows * P.nrhs;
    const int lpb = LONG ? long_rows_per_block<T>(L, W, nl) : lines_per_block<T>(L, nl);
    const int rthreads = LONG ? kLongThreads : threads_for(lpb, L);
    const size_t rlds = LONG ? long_row_lds<T>(lpb, L, W) : lds_bytes<T>(lpb, L);
    if (DIM > 1) {
        hipLaunchKernelGGL((k_mv_first<T, DIM, MODE, LONG>), dim3(cdiv(nl, lpb)), dim3(rthreads), rlds, s, a, lpb);
        cpx<T>* b1 = a.buf1;
        cpx<T>* b2 = a.buf2;
        auto mid = [&](auto kern, const cpx<T>* src, cpx<T>* dst, int64_t outer, int64_t inner, bool vh) {
            const int64_t lines = (int64_t)P.nrhs * outer * inner;
            // the column passes index lines in 32 bits
            if (lines >= (int64_t)INT32_MAX - 64) throw StatusError{EFGP_ETOOLARGE, "too many FFT lines"};
            const int lp = LONG ? long_mid_lines<T>(L, inner, vh) : mid_lines<T>(L, lines, inner);
            const int th = LONG ? kLongThreads : threads_for(lp, L);
            // the register-held FFT(v) values of the short-line column pass
            if (!LONG && (int64_t)lp * L > (int64_t)kMidV * th)
                throw StatusError{EFGP_EINVAL, "internal: column pass block too long"};
            hipLaunchKernelGGL(kern, dim3(cdiv(lines, lp)), dim3(th),
                               LONG ? long_mid_lds<T>(lp, L, vh) : lds_bytes<T>(lp, L), s, a, src, dst, outer,
                               inner, lp);
        };
        if (herm) {
            const int64_t pairs = (int64_t)P.nrhs * ((L + 1) / 2);
            const int lp = lines_per_block<T>(L, pairs);
            const int th = threads_for(lp, L);
            if ((int64_t)lp * L > (int64_t)kMidV * th)
                throw StatusError{EFGP_EINVAL, "internal: column pass block too long"};
            hipLaunchKernelGGL((k_mv_mid_herm<T>), dim3(cdiv(pairs, lp)), dim3(th), lds_bytes<T>(lp, L), s, a, lp);
        } else if (DIM == 2) {
            mid(k_mv_mid<T, 1, 1, 2, LONG>, b1, b2, 1, L, true);
        } else {
            mid(k_mv_mid<T, 1, 0, 0, LONG>, b1, b2, W, L, false);              // axis 1 forward
            mid(k_mv_mid<T, 1, 1, 2, LONG>, b2, b1, 1, (int64_t)L * L, true);  // axis 0 fwd * vhat inv
            mid(k_mv_mid<T, 0, 1, 1, LONG>, b1, b2, W, L, false);              // axis 1 inverse
        }
    }
    if (last)
        hipLaunchKernelGGL((k_mv_last<T, DIM, MODE, LONG>), dim3(cdiv(nl, lpb)), dim3(rthreads), rlds, s, a, lpb);
    EFGP_HIP(hipGetLastError());
}

template <typename T, int DIM, int MODE>
static void launch_mv(Plan& P, const MvArgs<T>& a, hipStream_t s) {
    if (long_lines<T>(P.L)) launch_mv_impl<T, DIM, MODE, true>(P, a, s);
    else launch_mv_impl<T, DIM, MODE, false>(P, a, s);
}

template <typename T, int MODE>
static void launch_mv_dim(Plan& P, const MvArgs<T>& a, hipStream_t s) {
    if (P.dim == 1) launch_mv<T, 1, MODE>(P, a, s);
    else if (P.dim == 2) launch_mv<T, 2, MODE>(P, a, s);
    else launch_mv<T, 3, MODE>(P, a, s);
}

void alloc_solver(Plan& P) {
    if (P.precision == 32) mv_lds_attrs_dim<float>(P);
    else mv_lds_attrs_dim<double>(P);
    if (P.r) return;
    const size_t es = P.precision == 32 ? sizeof(float) : sizeof(double);
    const size_t nv = (size_t)P.M * P.nrhs;
    P.x = dalloc(P, 2 * es * nv);
    P.r = dalloc(P, 2 * es * nv);
    P.p = dalloc(P, 2 * es * nv);
    P.q = dalloc(P, 2 * es * nv);
    size_t nb = P.dim == 1 ? 1 : (P.dim == 2 ? (size_t)P.W * P.L : (size_t)P.W * P.L * P.L);
    P.buf1 = dalloc(P, 2 * es * nb * P.nrhs);
    P.buf2 = dalloc(P, 2 * es * nb * P.nrhs);
    // residual history of system 0 (persistent: captured graphs hold the pointer)
    P.hist_cap = 1 << 20;
    P.hist = static_cast<double*>(dalloc(P, sizeof(double) * P.hist_cap));
    {
        const int64_t rows = P.dim == 1 ? 1 : (P.dim == 2 ? P.W : (int64_t)P.W * P.W);
        P.part = static_cast<double*>(dalloc(P, sizeof(double) * P.nrhs * (3 * rows + 3 * kGmax)));
    }
    // the states
    const size_t stb = sizeof(CgState) * P.nrhs;
    P.st = static_cast<CgState*>(dalloc(P, stb));
    EFGP_HIP(hipMemsetAsync(P.st, 0, stb, P.work));
    P.h_st = static_cast<CgState*>(palloc(P, sizeof(CgState) * P.nrhs));
}

template <typename T>
static void apply_typed(Plan& P, const void* in, void* out, hipStream_t s) {
    MvArgs<T> a = make_args<T>(P);
    a.in = static_cast<const cpx<T>*>(in);
    a.out = static_cast<cpx<T>*>(out);
    launch_mv_dim<T, MV_APPLY>(P, a, s);
}

void mv_apply(Plan& P, const void* in, void* out, hipStream_t s) {
    alloc_solver(P);
    if (P.precision == 32) apply_typed<float>(P, in, out, s);
    else apply_typed<double>(P, in, out, s);
}

// ---------------------------------------- allocation-free Toeplitz product
// The FFT intermediates of efgp_apply_noalloc live in this static device
// array: one copy per GPU, held until the process ends.  On the host its
// name stands for a host-side shadow, not device memory, so host code never
// passes it to a kernel or a copy: the device address comes from
// hipGetSymbolAddress, once per device, and only that pointer is used.
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}

void noalloc_init(int dev) {
    if (dev < 0 || dev >= kMaxDevices) throw StatusError{EFGP_EINVAL, "device index out of range"};
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return;
    void* p = nullptr;
    EFGP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw HipError{hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)"};
    g_scratch_ptr[dev] = p;
}

size_t noalloc_bytes(const Plan& P) {
    const size_t es = P.precision == 32 ? sizeof(float) : sizeof(double);
    const size_t nb = P.dim == 1 ? 1 : (P.dim == 2 ? (size_t)P.W * P.L : (size_t)P.W * P.L * P.L);
    // two line buffers, each 256-byte aligned
    const size_t one = (2 * es * nb * P.nrhs + 255) / 256 * 256;
    return 2 * one;
}

void mv_apply_noalloc(Plan& P, const void* in, void* out, hipStream_t s) {
    const size_t need = noalloc_bytes(P);
    if (need > kNoAllocBytes) throw StatusError{EFGP_ETOOLARGE, "product buffers exceed the static scratch"};
    void* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (P.device >= 0 && P.device < kMaxDevices) base = g_scratch_ptr[P.device];
    }
    if (!base) throw StatusError{EFGP_EINVAL, "no static scratch on the plan's device"};
    unsigned char* b = static_cast<unsigned char*>(base);
    if (P.precision == 32) {
        mv_lds_attrs_dim<float>(P);
        MvArgs<float> a = make_args<float>(P);
        a.in = static_cast<const cpx<float>*>(in);
        a.out = static_cast<cpx<float>*>(out);
        a.buf1 = reinterpret_cast<cpx<float>*>(b);
        a.buf2 = reinterpret_cast<cpx<float>*>(b + need / 2);
        launch_mv_dim<float, MV_APPLY>(P, a, s);
    } else {
        mv_lds_attrs_dim<double>(P);
        MvArgs<double> a = make_args<double>(P);
        a.in = static_cast<const cpx<double>*>(in);
        a.out = static_cast<cpx<double>*>(out);
        a.buf1 = reinterpret_cast<cpx<double>*>(b);
        a.buf2 = reinterpret_cast<cpx<double>*>(b + need / 2);
        launch_mv_dim<double, MV_APPLY>(P, a, s);
    }
}

// The CG update: one block of 1024 threads per system (no cross-block
// reduction) for small systems or many systems at once; otherwise about one
// element per thread on up to kGmax blocks of 256 per system, since the
// vectors were just written on other XCDs and the update is bound by load
// latency (one block would keep too few loads in flight).
static bool vec_one_block(const Plan& P) { return P.M <= 4096 || (P.nrhs >= 8 && P.M <= 32768); }
static unsigned vec_blocks(const Plan& P) {
    return std::max(1u, std::min(cdiv(P.M, 256), (unsigned)kGmax));
}

// The last pass and the CG update fused into one block per system: 2D small
// systems whose lines fit the block's LDS (4096 points)
template <typename T>
static bool fused_last(const Plan& P, const MvArgs<T>& a) {
    return P.dim == 2 && !long_lines<T>(P.L) && vec_one_block(P) && (int64_t)a.rows * P.L <= 4096;
}
template <typename T>
static size_t fused_last_lds(const Plan& P, const MvArgs<T>& a) {
    return (2 * (size_t)a.rows * P.L + P.L) * sizeof(cpx<T>);
}

// One block per system runs whole iterations (k_cg_block): Hermitian 2D
// systems whose two column-pair regions and twiddles fit the block's LDS and
// whose positions fit the kernel's per-thread slots
template <typename T>
static size_t cg_block_lds(const Plan& P) {
    const size_t np = (size_t)(P.L + 1) / 2;
    return (2 * np * P.L + P.L) * sizeof(cpx<T>);
}
static int lds_per_block() {
    int dev = 0, v = 65536;
    if (hipGetDevice(&dev) == hipSuccess) {
        int b = 0;
        if (hipDeviceGetAttribute(&b, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && b > 0) v = b;
    }
    return v;
}
static bool cg_block_fits(const Plan& P, int ke, int kv) {
    const int64_t np = (P.L + 1) / 2;
    return (int64_t)(P.m + 1) * P.L <= (int64_t)ke * 1024 && np * P.L <= (int64_t)kv * 1024;
}
template <typename T>
static bool cg_block_ok(const Plan& P, const MvArgs<T>& a) {
    if (!a.herm || P.dim != 2 || a.z) return false;
    return cg_block_fits(P, kBlkE, kBlkV) && cg_block_lds<T>(P) + 1024 <= (size_t)lds_per_block();
}
// the block kernel's largest FFT radix: the small register budget in
// single precision takes the large butterflies, the others keep to 2..5
template <typename T, int KE> constexpr int kBlkMaxR = std::is_same<T, float>::value && KE == 3 ? 12 : 5;
template <typename T>
static void launch_cg_block(Plan& P, const MvArgs<T>& a_in, int niter, hipStream_t s) {
    const size_t lds = cg_block_lds<T>(P);
    const bool small = cg_block_fits(P, 3, 6);
    MvArgs<T> a = a_in;
    a.f.s = fft_shape(P.L, small ? kBlkMaxR<T, 3> : kBlkMaxR<T, kBlkE>);
    const void* fn = small ? (const void*)k_cg_block<T, 3, 6, kBlkMaxR<T, 3>>
                           : (const void*)k_cg_block<T, kBlkE, kBlkV, kBlkMaxR<T, kBlkE>>;
    lds_attr(fn, lds);
    if (small)
        hipLaunchKernelGGL((k_cg_block<T, 3, 6, kBlkMaxR<T, 3>>), dim3(P.nrhs), dim3(1024), lds, s, a, niter, P.hist,
                           P.hist_cap);
    else
        hipLaunchKernelGGL((k_cg_block<T, kBlkE, kBlkV, kBlkMaxR<T, kBlkE>>), dim3(P.nrhs), dim3(1024), lds, s, a,
                           niter, P.hist, P.hist_cap);
    EFGP_HIP(hipGetLastError());
}

template <typename T>
static void launch_iteration(Plan& P, const MvArgs<T>& a, hipStream_t s) {
    if (fused_last<T>(P, a)) {
        launch_mv_impl<T, 2, MV_CG, false>(P, a, s, false);
        MvArgs<T> c = a;
        if (max_radix(c.f.s) > kCg1MaxR<T>) c.f.s = fft_shape(P.L, kCg1MaxR<T>);
        hipLaunchKernelGGL((k_mv_last_cg1<T>), dim3(P.nrhs), dim3(1024), fused_last_lds<T>(P, a), s, c, P.hist,
                           P.hist_cap);
        EFGP_HIP(hipGetLastError());
        if (a.z) circ_apply<T>(P, false, s);
        return;
    }
    launch_mv_dim<T, MV_CG>(P, a, s);
    if (vec_one_block(P)) {
        hipLaunchKernelGGL((k_cg_vec1<T>), dim3(P.nrhs), dim3(1024), 0, s, a, P.hist, P.hist_cap);
    } else {
        hipLaunchKernelGGL((k_cg_vec<T, false>), dim3(vec_blocks(P), P.nrhs), dim3(256), 0, s, a);
        hipLaunchKernelGGL((k_cg_fin<T, false>), dim3(P.nrhs), dim3(256), 0, s, a, (int)vec_blocks(P), P.hist,
                           P.hist_cap);
    }
    EFGP_HIP(hipGetLastError());
    if (a.z) circ_apply<T>(P, false, s);
}

template <typename T>
static void restart(Plan& P, const MvArgs<T>& a, double accept, hipStream_t s) {
    launch_mv_dim<T, MV_RESID>(P, a, s);
    hipLaunchKernelGGL((k_cg_restart_fin<T>), dim3(P.nrhs), dim3(256), 0, s, a, accept * accept);
    EFGP_HIP(hipGetLastError());
    if (a.z) circ_apply<T>(P, true, s);   // z = P r for the restarted systems
}

// Everything a captured iteration bakes into its kernel nodes: the argument
// block (pointers, sizes, the preconditioner pointer), the vector kernel's
// extra arguments, the batch length and the launch geometry's inputs.
template <typename T>
static std::string graph_key(const Plan& P, const MvArgs<T>& a, int ipg) {
    std::string k;
    auto put = [&](const void* v, size_t n) { k.append(static_cast<const char*>(v), n); };
    const void* ptrs[] = {a.in, a.out, a.x, a.r, a.p, a.q, a.b, a.prec, a.z, a.D, a.vhat, a.sig2, a.st,
                          a.buf1, a.buf2, a.part, a.f.tw, P.hist,
                          a.z ? P.prec : nullptr, a.z ? P.clam : nullptr, a.z ? P.cbuf : nullptr,
                          a.z ? P.cslot : nullptr, a.z ? P.twK : nullptr};
    put(ptrs, sizeof(ptrs));
    const int64_t ints[] = {a.m, a.W, a.L, a.nrhs, a.rows, a.herm, a.M, a.f.s.n, (int64_t)a.f.s.code, P.hist_cap,
                            ipg, P.dim, P.precision, a.z ? P.K : 0};
    put(ints, sizeof(ints));
    return k;
}

// stall_stops: a stalled preconditioned system stops where it is instead of
// continuing as plain CG (the inner solves of the refinement, whose outer
// loop carries on from the improved iterate with a fresh double residual:
// single-precision plain CG on a system that single-precision PCG cannot
// resolve makes little progress for many iterations)
template <typename T>
static int solve_typed(Plan& P, const efgp_solve_opts& o, void* beta_out, efgp_solve_stats* stats,
                       bool stall_stops = false) {
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = P.work;
    alloc_solver(P);
    const double rho = o.rel_tol > 0 ? o.rel_tol : P.eps;
    const int64_t max_iter = o.max_iter > 0 ? o.max_iter : 100000;
    if (o.launch < EFGP_LAUNCH_AUTO || o.launch > EFGP_LAUNCH_BLOCK)
        throw StatusError{EFGP_EINVAL, "unknown launch mode"};
    int ipg = o.iters_per_sync > 0 ? o.iters_per_sync : 16;
    const int64_t stall = o.stall_window > 0 ? o.stall_window : 1000;
    const size_t es = sizeof(T);
    const int64_t nv = P.M * P.nrhs;

    // preconditioner
    bool use_prec = false, circ = false;
    if (o.precond != EFGP_PRECOND_NONE) {
        if (!P.prec) P.prec = dalloc(P, es * nv);
        if (o.precond == EFGP_PRECOND_JACOBI) {
            hipLaunchKernelGGL((k_jacobi<T>), dim3(cdiv(nv, 256)), dim3(256), 0, s, static_cast<const T*>(P.Dt),
                               P.sig2, (double)P.n, P.M, P.nrhs, static_cast<T*>(P.prec));
        } else if (o.precond == EFGP_PRECOND_DIAG) {
            if (!o.precond_diag) throw StatusError{EFGP_EINVAL, "precond_diag is NULL"};
            EFGP_HIP(hipMemcpyAsync(P.prec, o.precond_diag, es * nv, hipMemcpyDeviceToDevice, s));
            if (!P.chk) P.chk = static_cast<int*>(dalloc(P, sizeof(int)));
            EFGP_HIP(hipMemsetAsync(P.chk, 0, sizeof(int), s));
            hipLaunchKernelGGL((k_check_diag<T>), dim3(cdiv(nv, 256)), dim3(256), 0, s, static_cast<const T*>(P.prec),
                               nv, P.chk);
            EFGP_HIP(hipGetLastError());
            int bad = 0;
            EFGP_HIP(hipMemcpyAsync(&bad, P.chk, sizeof(int), hipMemcpyDeviceToHost, s));
            EFGP_HIP(hipStreamSynchronize(s));
            if (bad) throw StatusError{EFGP_EINVAL, "precond_diag holds a non-finite or non-positive value"};
        } else if (o.precond == EFGP_PRECOND_LEARNED) {
            if (!o.mlp_weights) throw StatusError{EFGP_EMODEL, "mlp_weights is NULL"};
            mlp_precond(o.mlp_weights, P, P.prec, s);
        } else if (o.precond == EFGP_PRECOND_CIRCULANT) {
            circ_setup<T>(P, s);
            circ = true;
        } else {
            throw StatusError{EFGP_EINVAL, "unknown preconditioner"};
        }
        use_prec = true;
    }
    // initial state
    std::vector<CgState> hs(P.nrhs);
    for (int k = 0; k < P.nrhs; k++) {
        CgState t{};
        t.rho2 = rho * rho;
        t.use_prec = use_prec ? 1 : 0;
        hs[k] = t;
    }
    EFGP_HIP(hipMemcpyAsync(P.st, hs.data(), sizeof(CgState) * P.nrhs, hipMemcpyHostToDevice, s));
    MvArgs<T> a = make_args<T>(P);
    // a diagonal preconditioner scales r in the CG kernels; the circulant
    // one hands them z = P r (P.prec then holds its diagonal scaling)
    a.prec = (use_prec && !circ) ? static_cast<const T*>(P.prec) : nullptr;
    a.z = circ ? static_cast<const cpx<T>*>(P.zbuf) : nullptr;
    // Real data make b = D F*y Hermitian (b_{-j} = conj b_j), and A, with a
    // diagonal that is even in j, keeps every CG vector so: in 2D the
    // product then transforms half the rows and pairs the columns.  Not with
    // a caller's start vector or diagonal (they need not be Hermitian), nor
    // with the circulant (its z is not exactly Hermitian), nor for lines
    // past the two-buffer limit.
    if (P.dim == 2 && !long_lines<T>(P.L) && !o.beta_init && !circ && o.precond != EFGP_PRECOND_DIAG) {
        a.herm = 1;
        a.rows = P.m + 1;
    }
    // whole iterations in one block per system where the system qualifies
    // (AUTO), or on request (BLOCK)
    const bool blk = (o.launch == EFGP_LAUNCH_AUTO || o.launch == EFGP_LAUNCH_BLOCK) && cg_block_ok<T>(P, a);
    if (o.launch == EFGP_LAUNCH_BLOCK && !blk)
        throw StatusError{EFGP_EINVAL, "launch BLOCK needs a Hermitian 2D system whose column pass fits LDS"};
    // a block launch returns as soon as its systems stop, so it may run
    // longer between host checks
    if (blk && o.iters_per_sync <= 0) ipg = 64;
    hipLaunchKernelGGL((k_cg_vec<T, true>), dim3(vec_blocks(P), P.nrhs), dim3(256), 0, s, a);
    hipLaunchKernelGGL((k_cg_fin<T, true>), dim3(P.nrhs), dim3(256), 0, s, a, (int)vec_blocks(P), P.hist,
                       P.hist_cap);
    EFGP_HIP(hipGetLastError());
    if (circ) circ_apply<T>(P, true, s);
    auto read_state = [&]() {
        EFGP_HIP(hipMemcpyAsync(P.h_st, P.st, sizeof(CgState) * P.nrhs, hipMemcpyDeviceToHost, s));
        EFGP_HIP(hipStreamSynchronize(s));
    };
    auto set_restart = [&](const std::vector<int>& which, const std::vector<int>* prec_off) {
        read_state();
        for (int k = 0; k < P.nrhs; k++) {
            if (which[k]) P.h_st[k].pad = 1;
            if (prec_off && (*prec_off)[k]) P.h_st[k].use_prec = 0;
        }
        EFGP_HIP(hipMemcpyAsync(P.st, P.h_st, sizeof(CgState) * P.nrhs, hipMemcpyHostToDevice, s));
        restart<T>(P, a, 1.0, s);
    };
    if (o.beta_init) {
        hipLaunchKernelGGL((k_copy_cpx<T>), dim3(cdiv(nv, 256)), dim3(256), 0, s,
                           static_cast<const cpx<T>*>(o.beta_init), static_cast<cpx<T>*>(P.x), nv);
        set_restart(std::vector<int>(P.nrhs, 1), nullptr);
    }
    // graph of ipg iterations, shared through the process-wide cache by
    // every plan whose captured arguments are identical
    const bool graph = !blk && o.launch != EFGP_LAUNCH_PLAIN;
    if (graph) {
        const std::string id = graph_key<T>(P, a, ipg);
        if (!P.graph || P.graph_id != id) {
            if (P.graph) graph_release(P.device, P.graph_id);
            P.graph = graph_acquire(P.device, id);
            P.graph_id = id;
            if (!P.graph) {
                hipGraph_t g = nullptr;
                EFGP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                for (int k = 0; k < ipg; k++) launch_iteration<T>(P, a, s);
                EFGP_HIP(hipStreamEndCapture(s, &g));
                hipGraphExec_t ex = nullptr;
                const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                EFGP_HIP(e);
                graph_insert(P.device, id, ex);
                P.graph = ex;
            }
        }
    }
    std::vector<int64_t> chk_it(P.nrhs, 0);
    std::vector<double> chk_res(P.nrhs, 1.0);
    int fell_back = 0, checks = 0;
    std::vector<int> fb(P.nrhs, 0), stopped(P.nrhs, 0);
    int64_t done_iters = 0;
    read_state();
    for (int k = 0; k < P.nrhs; k++) chk_res[k] = P.h_st[k].relres;
    while (true) {
        bool any = false;
        for (int k = 0; k < P.nrhs; k++) any = any || P.h_st[k].active;
        if (any && done_iters < max_iter) {
            if (blk) launch_cg_block<T>(P, a, ipg, s);
            else if (graph) EFGP_HIP(hipGraphLaunch(P.graph, s));
            else for (int k = 0; k < ipg; k++) launch_iteration<T>(P, a, s);
            done_iters += ipg;
            read_state();
            // stall of preconditioned CG -> plain CG from the current iterate;
            // breakdown (NaN) -> plain CG from zero, since the step that
            // produced the NaN has already been applied to the iterate
            std::vector<int> who(P.nrhs, 0);
            bool need = false, stop = false;
            for (int k = 0; k < P.nrhs; k++) {
                const CgState& t = P.h_st[k];
                if (!t.use_prec) continue;
                const bool nan = !std::isfinite(t.relres) || !std::isfinite(t.gamma);
                if (t.relres <= chk_res[k] / 2.0) { chk_res[k] = t.relres; chk_it[k] = t.iters; }
                if (stall_stops && !nan && t.active && t.iters - chk_it[k] >= stall) {
                    P.h_st[k].active = 0;
                    stopped[k] = 1;
                    stop = true;
                    continue;
                }
                if (nan || (t.active && t.iters - chk_it[k] >= stall)) { who[k] = 1; need = true; }
                if (nan) {
                    hipLaunchKernelGGL((k_zero_cpx<T>), dim3(cdiv(P.M, 256)), dim3(256), 0, s,
                                       static_cast<cpx<T>*>(P.x) + (int64_t)k * P.M, P.M);
                    EFGP_HIP(hipGetLastError());
                }
            }
            if (stop && !need)
                EFGP_HIP(hipMemcpyAsync(P.st, P.h_st, sizeof(CgState) * P.nrhs, hipMemcpyHostToDevice, s));
            if (need) {
                if (stop)   // set_restart reads the device state back: the stops go first
                    EFGP_HIP(hipMemcpyAsync(P.st, P.h_st, sizeof(CgState) * P.nrhs, hipMemcpyHostToDevice, s));
                for (int k = 0; k < P.nrhs; k++) if (who[k]) { fb[k] = 1; chk_it[k] = P.h_st[k].iters; }
                set_restart(who, &who);
                if (graph) {  // the graph reads use_prec from device state; nothing to rebuild
                }
                read_state();
            }
            continue;
        }
        // converged or out of iterations: recompute the true residual
        std::vector<int> all(P.nrhs, 1);
        read_state();
        std::vector<CgState> before(P.h_st, P.h_st + P.nrhs);
        for (int k = 0; k < P.nrhs; k++) P.h_st[k].pad = 1;
        EFGP_HIP(hipMemcpyAsync(P.st, P.h_st, sizeof(CgState) * P.nrhs, hipMemcpyHostToDevice, s));
        restart<T>(P, a, 1.1, s);
        read_state();
        bool again = false;
        for (int k = 0; k < P.nrhs; k++) {
            P.h_st[k].iters = before[k].iters;
            if (stopped[k]) P.h_st[k].active = 0;   // a stalled system stays where it stopped
            if (P.h_st[k].active) again = true;
        }
        EFGP_HIP(hipMemcpyAsync(P.st, P.h_st, sizeof(CgState) * P.nrhs, hipMemcpyHostToDevice, s));
        if (again && done_iters < max_iter && checks < 8) { checks++; read_state(); continue; }
        break;
    }
    read_state();
    EFGP_HIP(hipMemcpyAsync(beta_out, P.x, 2 * es * nv, hipMemcpyDeviceToDevice, s));
    int conv = 0;
    double worst = 0.0;
    int64_t iters = 0;
    for (int k = 0; k < P.nrhs; k++) {
        const CgState& t = P.h_st[k];
        const bool ok = t.relres <= 1.1 * rho;
        conv += ok ? 1 : 0;
        worst = std::max(worst, t.relres);
        iters = std::max<int64_t>(iters, t.iters);
        fell_back += fb[k];
    }
    if (o.record_history > 0) {
        const int64_t len = std::min<int64_t>(P.h_st[0].iters, P.hist_cap);
        P.h_hist.assign(len, 0.0);
        if (len > 0) EFGP_HIP(hipMemcpyAsync(P.h_hist.data(), P.hist, sizeof(double) * len, hipMemcpyDeviceToHost, s));
    }
    EFGP_HIP(hipStreamSynchronize(s));
    auto t1 = std::chrono::steady_clock::now();
    if (stats) {
        stats->iterations = iters;
        stats->converged = conv;
        stats->fell_back = fell_back;
        stats->rel_residual = worst;
        stats->ms_solve = std::chrono::duration<double, std::milli>(t1 - t0).count();
        stats->history = P.h_hist.empty() ? nullptr : P.h_hist.data();
        stats->history_len = (int64_t)P.h_hist.size();
    }
    if (conv < P.nrhs) return EFGP_NOT_CONVERGED;
    return fell_back ? EFGP_FELL_BACK : EFGP_OK;
}

// ---------------------------------------- mixed-precision refinement
// Precision-32 CG cannot drive the residual of an ill-conditioned system
// much below ~1e-6 (the single-precision product's own error).  With
// opts.refine > 0 the solve is iterative refinement: x (double) starts at
// 0; each outer step forms r = b - A x with the double operator (b and v as
// the setup accumulated them, FFT(v) and the product in double), solves
// A d = r by the single-precision (P)CG, and adds d to x.

// rr[r] = ||a_r||^2 for each system r (one block per system)
static __global__ void __launch_bounds__(1024) k_norms64(const double2* __restrict__ a, int64_t M,
                                                         double* __restrict__ rr) {
    __shared__ double red[16];
    const int r = blockIdx.x;
    double v = 0.0;
    for (int64_t j = threadIdx.x; j < M; j += blockDim.x) {
        const double2 t = a[(int64_t)r * M + j];
        v += t.x * t.x + t.y * t.y;
    }
    v = block_sum(v, red);
    if (threadIdx.x == 0) rr[r] = v;
}
// r = b - ax; the single-precision right-hand side of the inner solve is r
static __global__ void k_resid64(const double2* __restrict__ b, const double2* __restrict__ ax, int64_t n,
                                 double2* __restrict__ r, float2* __restrict__ r32) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double2 t = make_double2(b[i].x - ax[i].x, b[i].y - ax[i].y);
    r[i] = t;
    r32[i] = make_float2((float)t.x, (float)t.y);
}
static __global__ void k_add_correction(const float2* __restrict__ d, int64_t n, double2* __restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = make_double2(x[i].x + (double)d[i].x, x[i].y + (double)d[i].y);
}
static __global__ void k_round_to_float(const double2* __restrict__ x, int64_t n, float2* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = make_float2((float)x[i].x, (float)x[i].y);
}

// ax = A x in double for every system of a precision-32 plan
static void apply64(Plan& P, hipStream_t s) {
    mv_lds_attrs_dim<double>(P);
    MvArgs<double> a = make_args<double>(P);
    a.x = a.r = a.p = a.q = nullptr;
    a.b = nullptr;
    a.prec = nullptr;
    a.st = nullptr;
    a.part = nullptr;
    a.D = P.D64;
    a.vhat = static_cast<const double2*>(P.vhat64);
    a.f.tw = static_cast<const double2*>(P.twL64);
    a.buf1 = static_cast<double2*>(P.buf64a);
    a.buf2 = static_cast<double2*>(P.buf64b);
    a.in = static_cast<const double2*>(P.x64);
    a.out = static_cast<double2*>(P.ax64);
    launch_mv_dim<double, MV_APPLY>(P, a, s);
}

static int solve_refined(Plan& P, const efgp_solve_opts& o, void* beta_out, efgp_solve_stats* stats) {
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = P.work;
    alloc_solver(P);
    const int64_t nv = P.M * P.nrhs;
    if (!P.vhat64) build_vhat64(P, s);
    if (!P.x64) {
        const size_t nb = P.dim == 1 ? 1 : (P.dim == 2 ? (size_t)P.W * P.L : (size_t)P.W * P.L * P.L);
        P.x64 = dalloc(P, 16 * (size_t)nv);
        P.r64 = dalloc(P, 16 * (size_t)nv);
        P.ax64 = dalloc(P, 16 * (size_t)nv);
        P.buf64a = dalloc(P, 16 * nb * P.nrhs);
        P.buf64b = dalloc(P, 16 * nb * P.nrhs);
    }
    double* norms = static_cast<double*>(P.part);   // nrhs slots (the CG reuses them later)
    std::vector<double> bb(P.nrhs), rr(P.nrhs);
    auto read_norms = [&](const void* v, std::vector<double>& out) {
        hipLaunchKernelGGL(k_norms64, dim3(P.nrhs), dim3(1024), 0, s, static_cast<const double2*>(v), P.M, norms);
        EFGP_HIP(hipGetLastError());
        EFGP_HIP(hipMemcpyAsync(out.data(), norms, sizeof(double) * P.nrhs, hipMemcpyDeviceToHost, s));
        EFGP_HIP(hipStreamSynchronize(s));
    };
    const double rho = o.rel_tol > 0 ? o.rel_tol : P.eps;
    const int64_t max_iter = o.max_iter > 0 ? o.max_iter : 100000;
    const unsigned g = cdiv(nv, 256);
    read_norms(P.b64, bb);
    hipLaunchKernelGGL((k_zero_cpx<double>), dim3(g), dim3(256), 0, s, static_cast<double2*>(P.x64), nv);
    hipLaunchKernelGGL((k_zero_cpx<double>), dim3(g), dim3(256), 0, s, static_cast<double2*>(P.ax64), nv);
    if (o.beta_init) {   // x = beta_init, A x in double
        hipLaunchKernelGGL(k_add_correction, dim3(g), dim3(256), 0, s, static_cast<const float2*>(o.beta_init), nv,
                           static_cast<double2*>(P.x64));
        apply64(P, s);
    }
    efgp_solve_opts in = o;
    in.beta_init = nullptr;
    in.record_history = 0;
    int64_t iters = 0;
    int fell_back = 0, steps = 0, st = EFGP_OK;
    double worst = 0.0;
    for (;; steps++) {
        // r = b - A x, its single-precision copy as the inner right-hand side
        hipLaunchKernelGGL(k_resid64, dim3(g), dim3(256), 0, s, reinterpret_cast<const double2*>(P.b64),
                           static_cast<const double2*>(P.ax64), nv, static_cast<double2*>(P.r64),
                           static_cast<float2*>(P.b));
        EFGP_HIP(hipGetLastError());
        read_norms(P.r64, rr);
        worst = 0.0;
        double need = 1.0;   // the inner tolerance that reaches rho for every system
        for (int k = 0; k < P.nrhs; k++) {
            const double res = bb[k] > 0.0 ? std::sqrt(rr[k] / bb[k]) : 0.0;
            worst = std::max(worst, res);
            if (res > 0.0) need = std::min(need, rho / res);
        }
        if (worst <= rho || steps >= o.refine || iters >= max_iter) break;
        // single precision reaches ~1e-6; ask no more of one step.  (Later
        // steps' residuals lie in the directions single precision resolves
        // worst: where u kappa > 1 their preconditioned CG stalls and plain
        // CG finishes them, slowly.)
        in.rel_tol = std::min(0.5, std::max(need, 1e-6));
        in.max_iter = max_iter - iters;
        efgp_solve_stats ist{};
        const int ist_status = solve_typed<float>(P, in, beta_out, &ist, true);
        iters += ist.iterations;
        fell_back += ist.fell_back;
        (void)ist_status;
        hipLaunchKernelGGL(k_add_correction, dim3(g), dim3(256), 0, s, static_cast<const float2*>(beta_out), nv,
                           static_cast<double2*>(P.x64));
        apply64(P, s);
    }
    // the plan's single-precision b again, and beta = x rounded to single
    hipLaunchKernelGGL(k_round_to_float, dim3(g), dim3(256), 0, s, reinterpret_cast<const double2*>(P.b64), nv,
                       static_cast<float2*>(P.b));
    hipLaunchKernelGGL(k_round_to_float, dim3(g), dim3(256), 0, s, static_cast<const double2*>(P.x64), nv,
                       static_cast<float2*>(beta_out));
    EFGP_HIP(hipGetLastError());
    EFGP_HIP(hipStreamSynchronize(s));
    int conv = 0;
    for (int k = 0; k < P.nrhs; k++) conv += (bb[k] <= 0.0 || std::sqrt(rr[k] / bb[k]) <= 1.1 * rho) ? 1 : 0;
    if (stats) {
        stats->iterations = iters;
        stats->converged = conv;
        stats->fell_back = fell_back;
        stats->rel_residual = worst;
        stats->ms_solve = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        stats->history = nullptr;
        stats->history_len = 0;
        stats->refine_steps = steps;
    }
    if (conv < P.nrhs) st = EFGP_NOT_CONVERGED;
    else if (fell_back) st = EFGP_FELL_BACK;
    return st;
}

int run_solve(Plan& P, const efgp_solve_opts& o, void* beta_out, efgp_solve_stats* st) {
    if (st) st->refine_steps = 0;
    if (P.precision == 32 && o.refine > 0) return solve_refined(P, o, beta_out, st);
    if (P.precision == 32) return solve_typed<float>(P, o, beta_out, st);
    return solve_typed<double>(P, o, beta_out, st);
}

void run_features(const Plan& P, int r, float* feats, float* jac, hipStream_t s) {
    const unsigned g = cdiv(P.M, 256);
    const double s2 = P.sigma2[r];
    if (P.dim == 1)
        hipLaunchKernelGGL(k_features<1>, dim3(g), dim3(256), 0, s, P.D64, reinterpret_cast<const double2*>(P.v), P.m,
                           P.h, P.ell, (double)P.n, s2, feats, jac);
    else if (P.dim == 2)
        hipLaunchKernelGGL(k_features<2>, dim3(g), dim3(256), 0, s, P.D64, reinterpret_cast<const double2*>(P.v), P.m,
                           P.h, P.ell, (double)P.n, s2, feats, jac);
    else
        hipLaunchKernelGGL(k_features<3>, dim3(g), dim3(256), 0, s, P.D64, reinterpret_cast<const double2*>(P.v), P.m,
                           P.h, P.ell, (double)P.n, s2, feats, jac);
    EFGP_HIP(hipGetLastError());
}

template <typename T>
void float_to_T(const float* in, int64_t n, void* out, hipStream_t s) {
    hipLaunchKernelGGL((k_float_to<T>), dim3(cdiv(n, 256)), dim3(256), 0, s, in, n, static_cast<T*>(out));
}
template void float_to_T<float>(const float*, int64_t, void*, hipStream_t);
template void float_to_T<double>(const float*, int64_t, void*, hipStream_t);

}  // namespace efgp
