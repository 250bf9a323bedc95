// Setup stage of EFGP (steps 1-3 of the EFGP algorithm, Sec. 3.2):
//   - type-1 spreading of the N points with the exponential-of-semicircle
//     (ES) kernel onto an oversampled periodic grid, 1 + nrhs real channels
//     (unit strengths -> Toeplitz vector v, eq. (88); data y_r -> F* y_r,
//     eq. (rhs)) packed pairwise as complex grids, accumulated globally in
//     double;
//   - FFT of the grid (sign +), Hermitian split of the channel pairs,
//     deconvolution by the ES kernel's Fourier transform, truncation to J_2m
//     (v) and J_m (b = D F* y);
//   - FFT(v) embedded at size L^d >= (4m+1)^d for the Toeplitz product.
//
// Grid geometry.  A point coordinate x in [0,1] maps to the grid position
// u = x h nf (cells), since its phase 2 pi h x sits on a period of nf cells.
// Its stencil is the w cells g0 .. g0+w-1 with g0 = ceil(u - w/2), weight
// phi((g - u)/(w/2)).  With h < 1 all stencils lie in the "active" cells
// -floor(w/2) .. floor(h nf) + ceil(w/2): a fraction h of the period.
//
// Two spreaders:
//   TILES    - counting sort of the points by tile of the shifted stencil
//              origin g0 + floor(w/2); one block per (tile, chunk, channel
//              group) accumulates into a padded tile in LDS and flushes with
//              double atomics.  Works for every size.
//   GRID_LDS - no sort: when the whole active region times the channels fits
//              in LDS, persistent blocks stream contiguous point ranges
//              (one coalesced pass over x and y), accumulate into a private
//              LDS copy of the active region, and write it out; a reduction
//              sums the copies in double.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <type_traits>

#pragma once
#include "fft_device.h"

namespace efgp {

template <typename T> struct Es {
    T beta;      // ES shape (float: pre-multiplied by log2(e) for exp2)
    T inv_hw;    // 1 / (w/2)
    T half_w;    // w/2
    T scale;     // h * nf : coordinate -> grid cells
    int w;
    int fw;      // floor(w/2)
};

// phi at 1 - z^2 = t: float uses the hardware v_sqrt_f32 / v_exp_f32 (2^x,
// with beta pre-multiplied by log2 e; arguments stay far from denormals),
// double the libm forms.  Stencil nodes satisfy -1 <= z < 1, so t < 0 only
// by rounding at z = -1; the float form clamps it to phi(-1) = e^-beta (the
// kernel's value at the edge of its support), the double form returns 0 there.
template <typename T> __device__ __forceinline__ T es_phi(T t, T beta);
template <> __device__ __forceinline__ float es_phi<float>(float t, float b2) {
    return __builtin_amdgcn_exp2f(fmaf(b2, __builtin_amdgcn_sqrtf(fmaxf(t, 0.0f)), -b2));
}
template <> __device__ __forceinline__ double es_phi<double>(double t, double beta) {
    return t > 0.0 ? exp(beta * (sqrt(t) - 1.0)) : 0.0;
}

// Grid position u = x h nf of a coordinate, rounded on its own: the product
// is never fused into a later add, so every kernel that derives a stencil
// origin from a coordinate (sort, partition, spreaders) gets the same one.
__device__ __forceinline__ float grid_pos(float a, float scale) { return __fmul_rn(a, scale); }
__device__ __forceinline__ double grid_pos(double a, double scale) { return __dmul_rn(a, scale); }

// Stencil origin and the w kernel values of one coordinate (registers; the
// loops are fully unrolled to the compile-time bound WMAX).
template <typename T, int WMAX>
__device__ __forceinline__ int es_stencil(T xc, const Es<T>& es, T* wt) {
    const T u = grid_pos(xc, es.scale);
    const T g0f = ceil(u - es.half_w);
    const T z0 = (g0f - u) * es.inv_hw;
#pragma unroll
    for (int k = 0; k < WMAX; k++) {
        if (k < es.w) {
            const T z = z0 + (T)k * es.inv_hw;
            wt[k] = es_phi<T>((T)1 - z * z, es.beta);
        }
    }
    return (int)g0f + es.fw;   // shifted origin, >= 0 for u >= 0
}

template <typename T>
__device__ __forceinline__ T es_weight_at(T xc, const Es<T>& es, int k) {
    const T u = grid_pos(xc, es.scale);
    const T g0f = ceil(u - es.half_w);
    const T z = (g0f - u) * es.inv_hw + (T)k * es.inv_hw;
    return es_phi<T>((T)1 - z * z, es.beta);
}

__device__ __forceinline__ bool in_unit(float a) { return a >= 0.0f && a <= 1.0f; }
__device__ __forceinline__ bool in_unit(double a) { return a >= 0.0 && a <= 1.0; }

template <typename T, int DIM>
__device__ __forceinline__ int tile_of(const T* __restrict__ x, int64_t n, int64_t i, const Es<T>& es,
                                      int T_, int nt, int ntiles, bool* bad) {
    int t = 0;
#pragma unroll
    for (int l = 0; l < DIM; l++) {
        const T a = x[(int64_t)l * n + i];
        if (!in_unit(a)) { *bad = true; return ntiles; }
        const T u = grid_pos(a, es.scale);
        int g = (int)ceil(u - es.half_w) + es.fw;
        int tl = min(max(g, 0) / T_, nt - 1);
        t = t * nt + tl;
    }
    return t;
}

// ------------------------------------------------------------ accumulators
// LDS accumulation type.  Precision 32 accumulates in 32-bit fixed point:
// on gfx950 integer LDS atomics run ~30x faster than float ones, and
// two's-complement sums are exact and order independent.  Channel c uses
// scale S_c chosen on the host so that no block epoch of at most P points
// can overflow: |sum| <= P * max|c| * S_c < 2^31.  Precision 64 accumulates
// in double.
template <typename T> struct Acc;
template <> struct Acc<float> {
    using t = int;
    // round(a b) to the nearest integer (ties to even), exact for |a b| < 2^22:
    // adding 1.5 * 2^23 leaves the rounded integer in the low mantissa bits.
    static __device__ __forceinline__ int mul(float a, float b) {
        return __float_as_int(fmaf(a, b, 12582912.0f)) - 0x4B400000;
    }
};
template <> struct Acc<double> {
    using t = double;
    static __device__ __forceinline__ double mul(double a, double b) { return a * b; }
};
constexpr int kMaxChan = 65;
struct Scales {
    float s[kMaxChan];     // value -> accumulator
    double inv[kMaxChan];  // accumulator -> value
    float lim[kMaxChan];   // |value| bound the scales assume (larger or NaN: flag 8)
};

// Overflow check of a block's fixed-point unit channel.  The unit channel's
// scale S_0 is set from the expected load of a cell, not from the worst case
// (every point of an epoch in one cell), so a cell could exceed 2^31.  Each
// thread sums the exact masses S_0 (sum_a w_a)(sum_b w_b).. of its points and
// the 32-bit words of the unit-channel cells it flushes; the unit channel only
// adds non-negative values, so a word that overflowed either reads negative or
// wrapped past 2^32, which lowers the block's word sum by 2^32 against the
// exact mass sum (rounding moves the two apart by at most half a unit per
// cell contribution, far below 2^31).  Either case raises flag 16 and the
// setup repeats with the worst-case scale.  The data channels need no check:
// their scales satisfy |y| S_c <= S_0, so |data cell| <= unit cell.
struct OvfCheck {
    unsigned long long* csum_s;   // two LDS slots after the accumulator
    double* esum_s;
    double esum = 0.0;
    unsigned long long csum = 0;
    bool neg = false;
    __device__ OvfCheck(unsigned char* smem, size_t acc_bytes) {
        const size_t o = (acc_bytes + 7) & ~(size_t)7;
        csum_s = reinterpret_cast<unsigned long long*>(smem + o);
        esum_s = reinterpret_cast<double*>(smem + o + 8);
        if (threadIdx.x == 0) { *csum_s = 0ull; *esum_s = 0.0; }
    }
    // mass of one point: the product over axes of its stencil weight sums
    template <typename T, int DIM, int WMAX>
    __device__ __forceinline__ void add_point(const T (*wt)[WMAX], int w) {
        T m = (T)1;
#pragma unroll
        for (int l = 0; l < DIM; l++) {
            T sl = (T)0;
#pragma unroll
            for (int k = 0; k < WMAX; k++)
                if (k < w) sl += wt[l][k];
            m *= sl;
        }
        esum += (double)m;
    }
    __device__ __forceinline__ void add_cell(int a) {
        csum += (unsigned)a;
        neg = neg || a < 0;
    }
    // every thread of the block calls this once, after its last flush
    __device__ __forceinline__ void finish(double s0, int* flag) {
        atomicAdd(csum_s, csum);
        atomicAdd(esum_s, esum);
        __syncthreads();
        if (threadIdx.x == 0 && fabs((double)*csum_s - s0 * *esum_s) > 2147483648.0) atomicOr(flag, 16);
        if (neg) atomicOr(flag, 16);
    }
};
constexpr size_t kOvfLds = 24;   // LDS bytes OvfCheck needs past the accumulator (alignment included)

// max |y_r| per data vector (as float bits; non-negative floats order like
// unsigned ints) and a flag for non-finite data.
template <typename T>
__global__ void __launch_bounds__(256) k_absmax(const T* __restrict__ y, int64_t n, unsigned* __restrict__ out,
                                                int* __restrict__ flag) {
    const int r = blockIdx.y;
    const T* yr = y + (int64_t)r * n;
    float mx = 0.0f;
    bool bad = false;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // eight independent loads per step keep enough bytes in flight
    for (; i + 7 * stride < n; i += 8 * stride) {
        T a[8];
#pragma unroll
        for (int k = 0; k < 8; k++) a[k] = yr[i + k * stride];
#pragma unroll
        for (int k = 0; k < 8; k++) {
            if (!(a[k] == a[k]) || a[k] > (T)3.0e38 || a[k] < (T)-3.0e38) bad = true;
            else mx = fmaxf(mx, (float)fabs(a[k]));
        }
    }
    for (; i < n; i += stride) {
        const T a = yr[i];
        if (!(a == a) || a > (T)3.0e38 || a < (T)-3.0e38) bad = true;
        else mx = fmaxf(mx, (float)fabs(a));
    }
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(&out[r], __float_as_uint(mx));
    if (bad) atomicOr(flag, 4);
}

// max |y_r| over gridDim.x contiguous chunks of clen values spread evenly
// over each data vector (NaN skipped, infinities kept so the host sees them)
template <typename T>
__global__ void __launch_bounds__(256) k_absmax_sample(const T* __restrict__ y, int64_t n, int64_t clen,
                                                       unsigned* __restrict__ out) {
    const int r = blockIdx.y;
    const T* yr = y + (int64_t)r * n;
    const int64_t c0 = (int64_t)blockIdx.x * (n / gridDim.x);
    const int64_t c1 = min(n, c0 + clen);
    float mx = 0.0f;
    for (int64_t i = c0 + threadIdx.x; i < c1; i += blockDim.x) {
        const T a = yr[i];
        if (a == a) mx = fmaxf(mx, (float)fabs(a));
    }
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(&out[r], __float_as_uint(mx));
}

// ----------------------------------------------------------------- sorting
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_tile_count(const T* __restrict__ x, int64_t n, Es<T> es,
                                                    int T_, int nt, int ntiles,
                                                    unsigned* __restrict__ counts, int* __restrict__ flag) {
    extern __shared__ unsigned hist[];
    for (int i = threadIdx.x; i <= ntiles; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int t = tile_of<T, DIM>(x, n, i, es, T_, nt, ntiles, &bad);
        atomicAdd(&hist[t], 1u);
    }
    if (bad) atomicOr(flag, 1);
    __syncthreads();
    for (int i = threadIdx.x; i <= ntiles; i += blockDim.x)
        if (hist[i]) atomicAdd(&counts[i], hist[i]);
}

// Scatter points into tile order.  Each block handles a contiguous chunk,
// reserves space per tile with one global atomic, and ranks its points
// within the reservation with LDS atomics.
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_tile_scatter(const T* __restrict__ x, const T* __restrict__ y,
                                                      int64_t n, int nrhs, Es<T> es, int T_, int nt, int ntiles,
                                                      int64_t chunk, unsigned* __restrict__ cursor,
                                                      T* __restrict__ xs, T* __restrict__ ys,
                                                      unsigned* __restrict__ perm) {
    extern __shared__ unsigned sm[];
    unsigned* cnt = sm;                // ntiles+1
    unsigned* base = sm + (ntiles + 1);
    for (int i = threadIdx.x; i <= ntiles; i += blockDim.x) cnt[i] = 0;
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * chunk;
    const int64_t i1 = min(n, i0 + chunk);
    bool bad = false;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        int t = tile_of<T, DIM>(x, n, i, es, T_, nt, ntiles, &bad);
        atomicAdd(&cnt[t], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= ntiles; i += blockDim.x) {
        base[i] = cnt[i] ? atomicAdd(&cursor[i], cnt[i]) : 0u;
        cnt[i] = 0;
    }
    __syncthreads();
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        int t = tile_of<T, DIM>(x, n, i, es, T_, nt, ntiles, &bad);
        if (t >= ntiles) continue;  // outside the domain: dropped (flagged)
        const int64_t pos = (int64_t)base[t] + atomicAdd(&cnt[t], 1u);
        if (pos >= n) continue;  // unreachable when the two passes agree
#pragma unroll
        for (int l = 0; l < DIM; l++) xs[(int64_t)l * n + pos] = x[(int64_t)l * n + i];
        if (perm) perm[pos] = (unsigned)i;   // the data stay in place (point-major)
        else
            for (int r = 0; r < nrhs; r++) ys[(int64_t)r * n + pos] = y[(int64_t)r * n + i];
    }
}

// ---------------------------------------------------- tiled LDS spreader
struct SubProb {
    int tile;
    int c0;       // first channel of the group
    int64_t start;
    int64_t count;
    int e;        // precision 32: this block's scales are the Scales' times 2^e (e <= 0)
    int pad;
};

// Channel c: 0 = unit strengths, 1 + r = y_r.  Channel c accumulates into
// complex grid c/2, component c%2.
template <typename T, int DIM, int WMAX>
__global__ void __launch_bounds__(256) k_spread_tiles(const T* __restrict__ xs, const T* __restrict__ ys,
                                                      int64_t n, int nchan, int cg, Es<T> es, int T_, int nt,
                                                      int nf, const SubProb* __restrict__ sub,
                                                      double* __restrict__ grid, int64_t gcells,
                                                      int* __restrict__ flag, Scales sc) {
    using A = typename Acc<T>::t;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    A* acc = reinterpret_cast<A*>(smem_raw);
    const SubProb sp = sub[blockIdx.x];
    const int P = T_ + es.w - 1;
    int pc = 1;
#pragma unroll
    for (int l = 0; l < DIM; l++) pc *= P;
    const int ncg = min(cg, nchan - sp.c0);
    constexpr bool FIXED = std::is_same<T, float>::value;
    // the block holding the unit channel checks it for overflow (OvfCheck)
    const bool unit = FIXED && sp.c0 == 0;
    OvfCheck ck(smem_raw, (size_t)pc * ncg * sizeof(A));
    for (int i = threadIdx.x; i < pc * ncg; i += blockDim.x) acc[i] = (A)0;
    T csc[8], clim[8];
    const T se = (T)ldexp(1.0, sp.e);          // exact: a power of two
    const double ise = ldexp(1.0, -sp.e);
    for (int c = 0; c < ncg; c++) {
        csc[c] = (T)sc.s[sp.c0 + c] * se;
        clim[c] = (T)sc.lim[sp.c0 + c];
    }
    bool over = false;
    int tl[3] = {0, 0, 0};
    {
        int t = sp.tile;
        for (int l = DIM - 1; l >= 0; l--) { tl[l] = t % nt; t /= nt; }
    }
    __syncthreads();
    bool bad = false;
    for (int64_t k = threadIdx.x; k < sp.count; k += blockDim.x) {
        const int64_t i = sp.start + k;
        T wt[DIM][WMAX];
        int off[DIM];
#pragma unroll
        for (int l = 0; l < DIM; l++) {
            int g = es_stencil<T, WMAX>(xs[(int64_t)l * n + i], es, wt[l]);
            int o = g - tl[l] * T_;
            if (o < 0 || o > T_ - 1) { bad = true; o = min(max(o, 0), T_ - 1); }
            off[l] = o;
        }
        if constexpr (FIXED) {
            if (unit) ck.add_point<T, DIM, WMAX>(wt, es.w);
        }
        T val[8];
        for (int c = 0; c < ncg; c++) {
            const int ch = sp.c0 + c;
            const T yv = ch == 0 ? (T)1 : ys[(int64_t)(ch - 1) * n + i];
            over = over || !(fabs(yv) <= clim[c]);
            val[c] = yv * csc[c];
        }
        if (DIM == 1) {
#pragma unroll
            for (int a = 0; a < WMAX; a++) {
                if (a < es.w) {
                    const int cell = off[0] + a;
                    for (int c = 0; c < ncg; c++) atomicAdd(&acc[c * pc + cell], Acc<T>::mul(wt[0][a], val[c]));
                }
            }
        } else if (DIM == 2) {
#pragma unroll
            for (int a = 0; a < WMAX; a++) {
                if (a < es.w) {
                    const int rowc = (off[0] + a) * P + off[1];
                    T wa[8];
                    for (int c = 0; c < ncg; c++) wa[c] = wt[0][a] * val[c];
#pragma unroll
                    for (int b = 0; b < WMAX; b++) {
                        if (b < es.w) {
                            for (int c = 0; c < ncg; c++) atomicAdd(&acc[c * pc + rowc + b], Acc<T>::mul(wa[c], wt[1][b]));
                        }
                    }
                }
            }
        } else {
            const T x0 = xs[i];
#pragma unroll 1
            for (int a = 0; a < es.w; a++) {
                {
                    const T wa = es_weight_at<T>(x0, es, a);
#pragma unroll
                    for (int b = 0; b < WMAX; b++) {
                        if (b < es.w) {
                            const T wab = wa * wt[1][b];
                            const int rowc = ((off[0] + a) * P + off[1] + b) * P + off[2];
                            T wabc[8];
                            for (int c = 0; c < ncg; c++) wabc[c] = wab * val[c];
#pragma unroll
                            for (int e = 0; e < WMAX; e++) {
                                if (e < es.w) {
                                    for (int c = 0; c < ncg; c++) atomicAdd(&acc[c * pc + rowc + e], Acc<T>::mul(wabc[c], wt[2][e]));
                                }
                            }
                        }
                    }
                }
            }
        }
    }
    if (bad) atomicOr(flag, 2);
    if (over) atomicOr(flag, 8);
    __syncthreads();
    // flush the padded tile to the periodic global grid
    for (int idx = threadIdx.x; idx < pc; idx += blockDim.x) {
        int rem = idx;
        int64_t gi = 0;
        int loc[3] = {0, 0, 0};
        for (int l = DIM - 1; l >= 0; l--) { loc[l] = rem % P; rem /= P; }
        for (int l = 0; l < DIM; l++) {
            int g = tl[l] * T_ + loc[l] - es.fw;
            g %= nf;
            if (g < 0) g += nf;
            gi = gi * nf + g;
        }
        for (int c = 0; c < ncg; c++) {
            const A a = acc[c * pc + idx];
            if constexpr (FIXED) {
                if (unit && c == 0) ck.add_cell(a);
            }
            if (a != (A)0) {
                const int ch = sp.c0 + c;
                atomicAdd(&grid[2 * ((int64_t)(ch >> 1) * gcells + gi) + (ch & 1)], (double)a * (sc.inv[ch] * ise));
            }
        }
    }
    if constexpr (FIXED) {
        if (unit) ck.finish((double)csc[0], flag);   // (unit is the same in every thread of the block)
    }
}

// ------------------------------------- channel-parallel tiled spreader
// Many data vectors (precision 32, d <= 2).  The data go point-major first,
// ypm[i][r] with rows of an even length ld >= nrhs (a zero pad for an odd
// count), through an LDS transpose; the sort then moves only the
// coordinates and a permutation.
template <typename T>
__global__ void __launch_bounds__(256) k_transpose_y(const T* __restrict__ y, int64_t n, int nrhs, int ld,
                                                     T* __restrict__ ypm) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* tile = reinterpret_cast<T*>(smem_raw);   // [nrhs][65]
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    const int cnt = (int)min<int64_t>(64, n - i0);
    for (int e = threadIdx.x; e < nrhs * 64; e += blockDim.x) {
        const int r = e >> 6, j = e & 63;
        if (j < cnt) tile[r * 65 + j] = y[(int64_t)r * n + i0 + j];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < ld * cnt; e += blockDim.x) {
        const int j = e / ld, r = e - j * ld;
        ypm[(i0 + j) * ld + r] = r < nrhs ? tile[r * 65 + j] : (T)0;
    }
}

__device__ __forceinline__ float bcast(float v, int j) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
}

// A wave takes 64 sorted points of its tile at a time.  Lane j computes the
// stencil of point j (and adds the unit channel for it).  Then the wave
// serves two points per step, one per half-wave: the weights of points j
// and j + 32 are broadcast with readlane, and lane p of a half adds data
// vectors 2p and 2p+1 to the w^d cells with one 64-bit LDS add (two signed
// fixed-point words: the sum of the low words stays within int32, so the
// high word is recovered by subtracting the sign-extended low word).  The
// accumulator is [cell][pair], so a half-wave's adds hit consecutive
// words.  Fixed point as in the other precision-32 spreaders; the data
// maxima are exact here (sampled maxima are taken for one data vector only).
// Both words are rounded by the same fma trick (bits of a b + 1.5 2^23 =
// 0x4B400000 + round(a b)); the two biases come off together as one 64-bit
// constant, exact because the low word's raw bits are positive.  EXACT: the
// width is WMAX itself, so the stencil loops carry no width tests.
template <int DIM, int WMAX, bool EXACT>
__global__ void __launch_bounds__(256) k_spread_tiles_ch(const float* __restrict__ xs, const unsigned* __restrict__ perm,
                                                         const float* __restrict__ ypm, int64_t n, int nrhs,
                                                         Es<float> es, int T_, int nt, int nf,
                                                         const SubProb* __restrict__ sub, double* __restrict__ grid,
                                                         int64_t gcells, int* __restrict__ flag, Scales sc) {
    using u64 = unsigned long long;
    constexpr u64 kBias2 = 0x4B4000004B400000ull;
    if (EXACT) {
        es.w = WMAX;
        es.fw = WMAX / 2;
    }
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int* acc0 = reinterpret_cast<int*>(smem_raw);   // unit channel, [cell]
    const SubProb sp = sub[blockIdx.x];
    const int P = T_ + es.w - 1;
    int pc = 1;
#pragma unroll
    for (int l = 0; l < DIM; l++) pc *= P;
    const int npair = (nrhs + 1) >> 1;
    u64* accd = reinterpret_cast<u64*>(acc0 + ((pc + 1) & ~1));   // data pairs, [cell][pair]
    for (int i = threadIdx.x; i < pc; i += blockDim.x) acc0[i] = 0;
    for (int i = threadIdx.x; i < pc * npair; i += blockDim.x) accd[i] = 0ull;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
    const int half = lane >> 5, pr = lane & 31;
    const bool has = pr < npair;
    // the pair's two vectors, one 8-byte load from rows of ld = 2 npair
    // values (the zero pad of an odd count gets scale 0; lanes past the
    // pairs read pair 0 with scale 0)
    const int ld = 2 * npair;
    const int r0 = has ? 2 * pr : 0;
    const float s0 = has ? sc.s[1 + 2 * pr] : 0.0f;
    const float s1 = has && 2 * pr + 1 < nrhs ? sc.s[2 + 2 * pr] : 0.0f;
    const float csc0 = sc.s[0];
    int tl[2] = {0, 0};
    {
        int t = sp.tile;
        for (int l = DIM - 1; l >= 0; l--) { tl[l] = t % nt; t /= nt; }
    }
    __syncthreads();
    bool bad = false;
    for (int64_t b0 = (int64_t)wave * 64; b0 < sp.count; b0 += (int64_t)nwave * 64) {
        const int cnt = (int)min<int64_t>(64, sp.count - b0);
        float wt[DIM][WMAX];
        int off[DIM];
        unsigned row = 0;
#pragma unroll
        for (int l = 0; l < DIM; l++) {
            off[l] = 0;
#pragma unroll
            for (int a = 0; a < WMAX; a++) wt[l][a] = 0.0f;
        }
        if (lane < cnt) {
            const int64_t i = sp.start + b0 + lane;
#pragma unroll
            for (int l = 0; l < DIM; l++) {
                const int g = es_stencil<float, WMAX>(xs[(int64_t)l * n + i], es, wt[l]);
                int o = g - tl[l] * T_;
                if (o < 0 || o > T_ - 1) { bad = true; o = min(max(o, 0), T_ - 1); }
                off[l] = o;
            }
            row = perm[i];
            if constexpr (DIM == 1) {
#pragma unroll
                for (int a = 0; a < WMAX; a++)
                    if (a < es.w) atomicAdd(&acc0[off[0] + a], Acc<float>::mul(wt[0][a], csc0));
            } else {
#pragma unroll
                for (int a = 0; a < WMAX; a++) {
                    if (a < es.w) {
                        const int rowc = (off[0] + a) * P + off[DIM - 1];
                        const float wa = wt[0][a] * csc0;
#pragma unroll
                        for (int b = 0; b < WMAX; b++)
                            if (b < es.w) atomicAdd(&acc0[rowc + b], Acc<float>::mul(wa, wt[DIM - 1][b]));
                    }
                }
            }
        }
        // steps of two points (j and j + 32); 8 steps' data are loaded
        // before any is used, unconditionally so that the loads overlap
        // (slots past the batch read row 0 of a lane that holds no point and
        // are never used; the data are finite)
        const int nstep = min(32, cnt);
        for (int j0 = 0; j0 < nstep; j0 += 8) {
            float2 yv[8];
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const unsigned ra = (unsigned)__builtin_amdgcn_readlane((int)row, j0 + u);
                const unsigned rb = (unsigned)__builtin_amdgcn_readlane((int)row, j0 + u + 32);
                // scaled where used, so that the loads stay in flight
                yv[u] = *reinterpret_cast<const float2*>(ypm + (int64_t)(half ? rb : ra) * ld + r0);
            }
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const int j = j0 + u;
                if (j >= nstep) break;
                const bool act = has && j + 32 * half < cnt;
                int o[DIM];
                float wj[DIM][WMAX];
#pragma unroll
                for (int l = 0; l < DIM; l++) {
                    const int oa = __builtin_amdgcn_readlane(off[l], j);
                    const int ob = __builtin_amdgcn_readlane(off[l], j + 32);
                    o[l] = half ? ob : oa;
#pragma unroll
                    for (int a = 0; a < WMAX; a++) {
                        const float wa = bcast(wt[l][a], j);
                        const float wb = bcast(wt[l][a], j + 32);
                        wj[l][a] = half ? wb : wa;
                    }
                }
                if (!act) continue;
                const float v0 = yv[u].x * s0, v1 = yv[u].y * s1;
                if constexpr (DIM == 1) {
#pragma unroll
                    for (int a = 0; a < WMAX; a++) {
                        if (a < es.w) {
                            const unsigned lo = __float_as_uint(fmaf(wj[0][a], v0, 12582912.0f));
                            const unsigned hi = __float_as_uint(fmaf(wj[0][a], v1, 12582912.0f));
                            atomicAdd(&accd[(o[0] + a) * npair + pr], (((u64)hi << 32) | lo) - kBias2);
                        }
                    }
                } else {
#pragma unroll
                    for (int a = 0; a < WMAX; a++) {
                        if (a < es.w) {
                            const int rowc = (o[0] + a) * P + o[DIM - 1];
                            const float wa0 = wj[0][a] * v0;
                            const float wa1 = wj[0][a] * v1;
#pragma unroll
                            for (int b = 0; b < WMAX; b++) {
                                if (b < es.w) {
                                    const unsigned lo = __float_as_uint(fmaf(wa0, wj[DIM - 1][b], 12582912.0f));
                                    const unsigned hi = __float_as_uint(fmaf(wa1, wj[DIM - 1][b], 12582912.0f));
                                    atomicAdd(&accd[(rowc + b) * npair + pr], (((u64)hi << 32) | lo) - kBias2);
                                }
                            }
                        }
                    }
                }
            }
        }
    }
    if (bad) atomicOr(flag, 2);
    __syncthreads();
    // flush the padded tile to the periodic global grid (channel 0 = unit,
    // 1 + r = data vector r; channel c is component c % 2 of grid c / 2)
    for (int idx = threadIdx.x; idx < pc; idx += blockDim.x) {
        int rem = idx;
        int64_t gi = 0;
        int loc[2] = {0, 0};
        for (int l = DIM - 1; l >= 0; l--) { loc[l] = rem % P; rem /= P; }
        for (int l = 0; l < DIM; l++) {
            int g = tl[l] * T_ + loc[l] - es.fw;
            g %= nf;
            if (g < 0) g += nf;
            gi = gi * nf + g;
        }
        const int a0 = acc0[idx];
        if (a0 != 0) atomicAdd(&grid[2 * gi], (double)a0 * sc.inv[0]);
        for (int q = 0; q < npair; q++) {
            const u64 v = accd[idx * npair + q];
            const int lo = (int)(unsigned)(v & 0xffffffffull);
            const int hi = (int)(unsigned)((v - (u64)(long long)lo) >> 32);
            const int rs[2] = {2 * q, 2 * q + 1};
            const int as[2] = {lo, hi};
#pragma unroll
            for (int k = 0; k < 2; k++) {
                if (rs[k] < nrhs && as[k] != 0) {
                    const int ch = 1 + rs[k];
                    atomicAdd(&grid[2 * ((int64_t)(ch >> 1) * gcells + gi) + (ch & 1)], (double)as[k] * sc.inv[ch]);
                }
            }
        }
    }
}

// ------------------------------------------------- whole-region spreader
// Add one cell's contributions of every channel: wv[c] * wb, quantised.
// PACK (precision 32, two channels): both channels go into one 64-bit LDS
// add, channel 0 (unit strengths, never negative) in the low word and
// channel 1 in the high word.  The low word's epoch sum stays below 2^31, so
// it never carries into the high word, and the high word's sum is exact
// modulo 2^32, hence exact as a signed int: one LDS atomic per cell instead of
// two.  The region is then cell-major ([cell][2]); otherwise channel-major
// ([c][cell]).
template <typename T, int NCH, bool PACK>
__device__ __forceinline__ void add_cell(typename Acc<T>::t* acc, int ac, int cell, const T* wv, T wb) {
    if constexpr (PACK) {
        // Acc<float>::mul with both bias subtractions done by one 64-bit add
        // (the low word's result is non-negative, so nothing borrows)
        const unsigned lo = (unsigned)__float_as_int(fmaf(wv[0], wb, 12582912.0f));
        const unsigned hi = (unsigned)__float_as_int(fmaf(wv[1], wb, 12582912.0f));
        const unsigned long long q = (((unsigned long long)hi << 32) | lo) - 0x4B4000004B400000ull;
        atomicAdd(reinterpret_cast<unsigned long long*>(acc) + cell, q);
    } else {
#pragma unroll
        for (int c = 0; c < NCH; c++) atomicAdd(&acc[c * ac + cell], Acc<T>::mul(wv[c], wb));
    }
}

// EXACT: the kernel width is WMAX itself (a compile-time constant, so the
// stencil loops carry no width tests); otherwise w <= WMAX at run time.
template <typename T, int DIM, int WMAX, int NCH, bool EXACT>
__global__ void __launch_bounds__(1024) k_spread_gridlds(const T* __restrict__ x, const T* __restrict__ y,
                                                         int64_t n, Es<T> es, int A, int64_t chunk, int64_t epoch,
                                                         int nepoch, typename Acc<T>::t* __restrict__ partial,
                                                         int* __restrict__ flag, Scales sc) {
    using Ac = typename Acc<T>::t;
    constexpr bool PACK = std::is_same<T, float>::value && NCH == 2;
    if (EXACT) {
        es.w = WMAX;
        es.fw = WMAX / 2;
    }
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Ac* acc = reinterpret_cast<Ac*>(smem_raw);
    int ac = 1;
#pragma unroll
    for (int l = 0; l < DIM; l++) ac *= A;
    const int omax = A - es.w;
    bool bad = false;
    T csc[NCH], clim[NCH];
#pragma unroll
    for (int c = 0; c < NCH; c++) {
        csc[c] = (T)sc.s[c];
        clim[c] = (T)sc.lim[c];
    }
    bool over = false;
    // overflow check of the fixed-point unit channel (see OvfCheck)
    OvfCheck ck(smem_raw, (size_t)ac * NCH * sizeof(Ac));
    for (int ep = 0; ep < nepoch; ep++) {
    for (int i = threadIdx.x; i < ac * NCH; i += blockDim.x) acc[i] = (Ac)0;
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * chunk + (int64_t)ep * epoch;
    const int64_t i1 = min(min(n, (int64_t)(blockIdx.x + 1) * chunk), i0 + epoch);
    // the next point's coordinates and data are loaded before this point's
    // atomics are issued, so the loads overlap them
    T nx[DIM], ny[NCH > 1 ? NCH - 1 : 1];
    int64_t i = i0 + threadIdx.x;
    if (i < i1) {
#pragma unroll
        for (int l = 0; l < DIM; l++) nx[l] = x[(int64_t)l * n + i];
#pragma unroll
        for (int c = 1; c < NCH; c++) ny[c - 1] = y[(int64_t)(c - 1) * n + i];
    }
    for (; i < i1; i += blockDim.x) {
        T cx[DIM], val[NCH];
#pragma unroll
        for (int l = 0; l < DIM; l++) cx[l] = nx[l];
        val[0] = csc[0];
#pragma unroll
        for (int c = 1; c < NCH; c++) {
            over = over || !(fabs(ny[c - 1]) <= clim[c]);
            val[c] = ny[c - 1] * csc[c];
        }
        const int64_t inext = i + blockDim.x;
        if (inext < i1) {
#pragma unroll
            for (int l = 0; l < DIM; l++) nx[l] = x[(int64_t)l * n + inext];
#pragma unroll
            for (int c = 1; c < NCH; c++) ny[c - 1] = y[(int64_t)(c - 1) * n + inext];
        }
        T wt[DIM][WMAX];
        int off[DIM];
#pragma unroll
        for (int l = 0; l < DIM; l++) {
            // a point outside [0,1] (or NaN) fails the whole setup; it is
            // still spread at a clamped, in-bounds stencil, without a branch
            bad = bad || !in_unit(cx[l]);
            int g = es_stencil<T, WMAX>(cx[l], es, wt[l]);
            off[l] = min(max(g, 0), omax);
        }
        if constexpr (PACK) ck.add_point<T, DIM, WMAX>(wt, es.w);
        if (DIM == 1) {
#pragma unroll
            for (int a = 0; a < WMAX; a++)
                if (a < es.w) add_cell<T, NCH, PACK>(acc, ac, off[0] + a, val, wt[0][a]);
        } else if (DIM == 2) {
#pragma unroll
            for (int a = 0; a < WMAX; a++) {
                if (a < es.w) {
                    const int rowc = (off[0] + a) * A + off[1];
                    T wa[NCH];
#pragma unroll
                    for (int c = 0; c < NCH; c++) wa[c] = wt[0][a] * val[c];
#pragma unroll
                    for (int b = 0; b < WMAX; b++)
                        if (b < es.w) add_cell<T, NCH, PACK>(acc, ac, rowc + b, wa, wt[1][b]);
                }
            }
        } else {
#pragma unroll 1
            for (int a = 0; a < es.w; a++) {
                const T wa = es_weight_at<T>(cx[0], es, a);
#pragma unroll
                for (int b = 0; b < WMAX; b++) {
                    if (b < es.w) {
                        const int rowc = ((off[0] + a) * A + off[1] + b) * A + off[2];
                        T wab[NCH];
#pragma unroll
                        for (int c = 0; c < NCH; c++) wab[c] = wa * wt[1][b] * val[c];
#pragma unroll
                        for (int e = 0; e < WMAX; e++)
                            if (e < es.w) add_cell<T, NCH, PACK>(acc, ac, rowc + e, wab, wt[2][e]);
                    }
                }
            }
        }
    }
    __syncthreads();
    Ac* out = partial + ((int64_t)blockIdx.x * nepoch + ep) * ac * NCH;
    for (int i = threadIdx.x; i < ac * NCH; i += blockDim.x) {
        const Ac a = acc[i];
        out[i] = a;
        if constexpr (PACK) {
            if ((i & 1) == 0) ck.add_cell(a);   // low words: the unit channel
        }
    }
    __syncthreads();
    }
    if (bad) atomicOr(flag, 1);
    if (over) atomicOr(flag, 8);
    if constexpr (PACK) ck.finish((double)csc[0], flag);
}

// Sum the per-block copies of the active region in double and write the
// periodic grid (every grid cell written, so no zero fill is needed).
template <typename T>
using SumT = typename std::conditional<std::is_same<typename Acc<T>::t, int>::value, long long, double>::type;

// Stage 1: sum the block-epoch slots in `nchunk` interleaved chunks.  Thread
// = one accumulator element of the active region, so reads are coalesced and
// every chunk runs in parallel.
template <typename T>
__global__ void __launch_bounds__(256) k_slot_sum(const typename Acc<T>::t* __restrict__ partial, int nslot,
                                                  int64_t elems, int nchunk, SumT<T>* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= elems) return;
    const int k = blockIdx.y;
    SumT<T> s = 0;
    for (int b = k; b < nslot; b += nchunk) s += (SumT<T>)partial[(int64_t)b * elems + e];
    out[(int64_t)k * elems + e] = s;
}

// Stage 2: per grid cell, sum the chunks of every active cell that maps to it.
template <typename T, int DIM>
__global__ void k_reduce_partials(const SumT<T>* __restrict__ partial, int nslot, int A, int nch, bool cell_major,
                                  int fw, int nf, double* __restrict__ grid, int64_t gcells, Scales sc) {
    using Ac = SumT<T>;
    using Sum = SumT<T>;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= gcells) return;
    int gl[3] = {0, 0, 0};
    int64_t rem = g;
    for (int l = DIM - 1; l >= 0; l--) { gl[l] = (int)(rem % nf); rem /= nf; }
    int64_t ac = 1;
    for (int l = 0; l < DIM; l++) ac *= A;
    Sum s[2] = {0, 0};
    // active index a = g + fw + k nf for every k with 0 <= a < A (per dim)
    int a0[3], na[3];
    for (int l = 0; l < 3; l++) { a0[l] = 0; na[l] = 1; }
    for (int l = 0; l < DIM; l++) {
        int a = gl[l] + fw;
        a %= nf;
        a0[l] = a;
        na[l] = a < A ? (A - 1 - a) / nf + 1 : 0;
    }
    for (int i0 = 0; i0 < na[0]; i0++)
        for (int i1 = 0; i1 < (DIM > 1 ? na[1] : 1); i1++)
            for (int i2 = 0; i2 < (DIM > 2 ? na[2] : 1); i2++) {
                int64_t ai = a0[0] + i0 * nf;
                if (DIM > 1) ai = ai * A + a0[1] + i1 * nf;
                if (DIM > 2) ai = ai * A + a0[2] + i2 * nf;
                for (int b = 0; b < nslot; b++) {
                    const Ac* pb = partial + (int64_t)b * ac * nch;
                    for (int c = 0; c < nch; c++) s[c] += (Sum)pb[cell_major ? ai * nch + c : c * ac + ai];
                }
            }
    for (int c = 0; c < nch; c++) grid[2 * ((int64_t)(c >> 1) * gcells + g) + (c & 1)] = (double)s[c] * sc.inv[c];
    if (nch & 1) grid[2 * ((int64_t)(nch >> 1) * gcells + g) + 1] = 0.0;
}

// ----------------------------------------------------- region spreader
// For grids whose active region exceeds LDS (precision 32, one data
// vector).  The stencil origins 0 .. omax of each axis are split into nr
// runs of R; region r = (r_0, .., r_{d-1}) takes the points whose origins
// fall in its runs, and its window of R + w - 1 cells per axis holds all
// their stencils.  A two-pass partition orders the points by region: pass 1
// counts each block's points per region, a scan turns the counts into
// output offsets, and pass 2 ranks every tile of points by region in LDS and
// writes it out in runs (coalesced stores).  Then one block per sub-problem
// (a run of at most S points of one region) accumulates the window in
// packed 64-bit fixed point, as the whole-region spreader does, and writes
// it to its own slot; a gather sums each grid cell's slots in a fixed order.
struct RegionGeom {
    int R;       // stencil origins per region and axis
    int RW;      // window cells per axis, R + w - 1
    int nr;      // regions per axis
    int nreg;    // nr^d
    int omax;    // largest stencil origin, floor(h nf) + 1
    float rR;    // 1 / R, for the region of an origin without an integer division
};

// The shifted stencil origin of es_stencil, clamped to 0 .. omax.
template <typename T>
__device__ __forceinline__ int stencil_origin(T a, const Es<T>& es, int omax) {
    const int g = (int)ceil(grid_pos(a, es.scale) - es.half_w) + es.fw;
    return min(max(g, 0), omax);
}

template <typename T, int DIM>
__device__ __forceinline__ int region_id(const T* cx, const Es<T>& es, const RegionGeom& rg, bool& bad) {
    int r = 0;
#pragma unroll
    for (int l = 0; l < DIM; l++) {
        bad = bad || !in_unit(cx[l]);
        int rem;
        r = r * rg.nr + udiv22(stencil_origin<T>(cx[l], es, rg.omax), rg.R, rg.rR, &rem);
    }
    return r;
}

// Pass 1: counts[r * nblk + b] = points of block b's range in region r.
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_region_count(const T* __restrict__ x, int64_t n, Es<T> es, RegionGeom rg,
                                                      int64_t chunk, unsigned* __restrict__ counts,
                                                      int* __restrict__ flag) {
    extern __shared__ unsigned hist[];
    for (int r = threadIdx.x; r < rg.nreg; r += blockDim.x) hist[r] = 0;
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * chunk;
    const int64_t i1 = min(n, i0 + chunk);
    bool bad = false;
    // four points' loads per thread in flight before their atomics
    for (int64_t ib = i0 + threadIdx.x; ib < i1; ib += 4 * (int64_t)blockDim.x) {
        T cx[4][DIM];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int64_t i = min(ib + u * (int64_t)blockDim.x, i1 - 1);   // past the end: not counted
#pragma unroll
            for (int l = 0; l < DIM; l++) cx[u][l] = x[(int64_t)l * n + i];
        }
#pragma unroll
        for (int u = 0; u < 4; u++)
            if (ib + u * (int64_t)blockDim.x < i1) atomicAdd(&hist[region_id<T, DIM>(cx[u], es, rg, bad)], 1u);
    }
    if (bad) atomicOr(flag, 1);
    __syncthreads();
    for (int r = threadIdx.x; r < rg.nreg; r += blockDim.x) counts[(int64_t)r * gridDim.x + blockIdx.x] = hist[r];
}

// Inclusive prefix sum over a 64-lane wave.
__device__ __forceinline__ unsigned wave_inclusive_scan(unsigned v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// One block per region: counts[r][b] becomes the exclusive prefix over the
// blocks b' < b (the block's offset within the region), totals[r] the
// region's count.
static __global__ void __launch_bounds__(256) k_region_scan(unsigned* __restrict__ counts, int nblk,
                                                     unsigned long long* __restrict__ totals) {
    __shared__ unsigned wsum[4];
    unsigned* c = counts + (int64_t)blockIdx.x * nblk;
    unsigned carry = 0;
    for (int b0 = 0; b0 < nblk; b0 += 256) {
        const int b = b0 + threadIdx.x;
        const unsigned v = b < nblk ? c[b] : 0u;
        const unsigned inc = wave_inclusive_scan(v);
        if ((threadIdx.x & 63) == 63) wsum[threadIdx.x >> 6] = inc;
        __syncthreads();
        unsigned before = carry;
        for (int k = 0; k < (int)(threadIdx.x >> 6); k++) before += wsum[k];
        if (b < nblk) c[b] = before + inc - v;
        carry += wsum[0] + wsum[1] + wsum[2] + wsum[3];
        __syncthreads();
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

// Exclusive prefix sums of in[0 .. cnt) into out (a block of 1024 threads;
// wsum: 16 LDS words).  Ends with a barrier.
__device__ __forceinline__ void block_exclusive_scan_1024(const unsigned* in, unsigned* out, int cnt,
                                                          unsigned* wsum) {
    const int per = (cnt + 1023) >> 10;
    const int b = threadIdx.x * per;
    unsigned s = 0;
    for (int k = 0; k < per; k++)
        if (b + k < cnt) s += in[b + k];
    const unsigned inc = wave_inclusive_scan(s);
    if ((threadIdx.x & 63) == 63) wsum[threadIdx.x >> 6] = inc;
    __syncthreads();
    unsigned run = inc - s;
    for (int k = 0; k < (int)(threadIdx.x >> 6); k++) run += wsum[k];
    for (int k = 0; k < per; k++) {
        if (b + k < cnt) {
            const unsigned t = in[b + k];
            out[b + k] = run;
            run += t;
        }
    }
    __syncthreads();
}

// Pass 2 (1024 threads): block b's range, in tiles of PT * 1024 points.  A
// tile is ranked by region with LDS atomics, staged in region order in LDS,
// and written out in runs: region r's points of this block go to
// rstart[r] + boff[r][b] onwards.  The run ends are checked against pass 1
// (flag 2 if a block's count differs; nothing is written outside [0, n)).
template <typename T, int DIM, int PT>
__global__ void __launch_bounds__(1024) k_region_scatter(const T* __restrict__ x, const T* __restrict__ y, int64_t n,
                                                         Es<T> es, RegionGeom rg, int64_t chunk,
                                                         const unsigned* __restrict__ boff,
                                                         const unsigned long long* __restrict__ rstart,
                                                         const unsigned long long* __restrict__ totals,
                                                         T* __restrict__ xs, T* __restrict__ ys,
                                                         int* __restrict__ flag) {
    constexpr int TS = PT * 1024;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* sx = reinterpret_cast<T*>(smem_raw);                          // [DIM][TS]
    T* sy = sx + DIM * TS;                                             // [TS]
    unsigned short* sreg = reinterpret_cast<unsigned short*>(sy + TS); // [TS]
    unsigned* lcnt = reinterpret_cast<unsigned*>(sreg + TS);           // [nreg]
    unsigned* lofs = lcnt + rg.nreg;                                   // [nreg]
    unsigned* goff = lofs + rg.nreg;                                   // [nreg]
    unsigned* wsum = goff + rg.nreg;                                   // [16]
    const int nreg = rg.nreg;
    const int nblk = gridDim.x;
    for (int r = threadIdx.x; r < nreg; r += 1024) {
        lcnt[r] = 0;
        goff[r] = (unsigned)(rstart[r] + boff[(int64_t)r * nblk + blockIdx.x]);
    }
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * chunk;
    const int64_t i1 = min(n, i0 + chunk);
    bool bad = false;   // out-of-domain points were flagged by pass 1
    // the next tile's loads are issued before this tile is ranked, staged
    // and written, so they overlap that work
    T px[PT][DIM], py[PT];
    auto load_tile = [&](int64_t t0) {
        const int tc = (int)min((int64_t)TS, i1 - t0);
#pragma unroll
        for (int k = 0; k < PT; k++) {
            const int j = k * 1024 + threadIdx.x;
            if (j < tc) {
                const int64_t i = t0 + j;
#pragma unroll
                for (int l = 0; l < DIM; l++) px[k][l] = x[(int64_t)l * n + i];
                py[k] = y[i];
            }
        }
    };
    if (i0 < i1) load_tile(i0);
    for (int64_t t0 = i0; t0 < i1; t0 += TS) {
        const int tcount = (int)min((int64_t)TS, i1 - t0);
        int rid[PT], rk[PT];
        T cx[PT][DIM], cy[PT];
#pragma unroll
        for (int k = 0; k < PT; k++) {
            rid[k] = -1;
            rk[k] = 0;
            cy[k] = py[k];
#pragma unroll
            for (int l = 0; l < DIM; l++) cx[k][l] = px[k][l];
            if (k * 1024 + (int)threadIdx.x < tcount) {
                rid[k] = region_id<T, DIM>(cx[k], es, rg, bad);
                rk[k] = (int)atomicAdd(&lcnt[rid[k]], 1u);
            }
        }
        if (t0 + TS < i1) load_tile(t0 + TS);
        __syncthreads();
        block_exclusive_scan_1024(lcnt, lofs, nreg, wsum);
#pragma unroll
        for (int k = 0; k < PT; k++) {
            if (rid[k] >= 0) {
                const int pos = (int)lofs[rid[k]] + rk[k];
#pragma unroll
                for (int l = 0; l < DIM; l++) sx[l * TS + pos] = cx[k][l];
                sy[pos] = cy[k];
                sreg[pos] = (unsigned short)rid[k];
            }
        }
        __syncthreads();
        for (int j = threadIdx.x; j < tcount; j += 1024) {
            const int r = sreg[j];
            const int64_t g = (int64_t)goff[r] + (j - (int)lofs[r]);
            if (g < n) {
#pragma unroll
                for (int l = 0; l < DIM; l++) xs[(int64_t)l * n + g] = sx[l * TS + j];
                ys[g] = sy[j];
            }
        }
        __syncthreads();
        for (int r = threadIdx.x; r < nreg; r += 1024) {
            goff[r] += lcnt[r];
            lcnt[r] = 0;
        }
        __syncthreads();
    }
    // every run must end where the next block's begins (pass 1's counts)
    for (int r = threadIdx.x; r < nreg; r += 1024) {
        const unsigned long long end = rstart[r] + (blockIdx.x + 1 < (unsigned)nblk
                                                        ? (unsigned long long)boff[(int64_t)r * nblk + blockIdx.x + 1]
                                                        : totals[r]);
        if ((unsigned long long)goff[r] != end) atomicOr(flag, 2);
    }
}

// One block (1024 threads) per sub-problem: the points start .. start+count-1
// of the region-ordered arrays, all in region sp.tile.  The window is
// accumulated like k_spread_gridlds (cell-major packed pairs: unit channel in
// the low word, data in the high word) at this region's scales times 2^e,
// then written to slot blockIdx.x.  A point whose origin lies outside the
// region raises flag 2 (the partition and the spreader disagree).
template <int DIM, int WMAX>
__global__ void __launch_bounds__(1024) k_spread_regions(const float* __restrict__ xs, const float* __restrict__ ys,
                                                         int64_t n, Es<float> es, RegionGeom rg,
                                                         const SubProb* __restrict__ sub,
                                                         unsigned long long* __restrict__ slots,
                                                         int* __restrict__ flag, Scales sc) {
    using u64 = unsigned long long;
    es.w = WMAX;   // one kernel per exact width
    es.fw = WMAX / 2;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int* acc = reinterpret_cast<int*>(smem_raw);
    const SubProb sp = sub[blockIdx.x];
    const int RW = rg.RW;
    int wc = 1;
#pragma unroll
    for (int l = 0; l < DIM; l++) wc *= RW;
    OvfCheck ck(smem_raw, (size_t)wc * 2 * sizeof(int));
    for (int i = threadIdx.x; i < wc; i += blockDim.x) reinterpret_cast<u64*>(acc)[i] = 0ull;
    int ro[3] = {0, 0, 0};
    {
        int t = sp.tile;
        for (int l = DIM - 1; l >= 0; l--) {
            ro[l] = (t % rg.nr) * rg.R;
            t /= rg.nr;
        }
    }
    const float se = ldexpf(1.0f, sp.e);   // exact: a power of two
    const float csc0 = sc.s[0] * se, csc1 = sc.s[1] * se, clim = sc.lim[1];
    bool bad = false, over = false;
    __syncthreads();
    const int64_t i1 = sp.start + sp.count;
    float nx[DIM], ny = 0.0f;
    int64_t i = sp.start + threadIdx.x;
    if (i < i1) {
#pragma unroll
        for (int l = 0; l < DIM; l++) nx[l] = xs[(int64_t)l * n + i];
        ny = ys[i];
    }
    for (; i < i1; i += blockDim.x) {
        float cx[DIM], val[2];
#pragma unroll
        for (int l = 0; l < DIM; l++) cx[l] = nx[l];
        over = over || !(fabsf(ny) <= clim);
        val[0] = csc0;
        val[1] = ny * csc1;
        const int64_t inext = i + blockDim.x;
        if (inext < i1) {
#pragma unroll
            for (int l = 0; l < DIM; l++) nx[l] = xs[(int64_t)l * n + inext];
            ny = ys[inext];
        }
        float wt[DIM][WMAX];
        int off[DIM];
#pragma unroll
        for (int l = 0; l < DIM; l++) {
            const int g = min(max(es_stencil<float, WMAX>(cx[l], es, wt[l]), 0), rg.omax);
            int o = g - ro[l];
            if (o < 0 || o >= rg.R) {
                bad = true;
                o = min(max(o, 0), rg.R - 1);
            }
            off[l] = o;
        }
        ck.add_point<float, DIM, WMAX>(wt, WMAX);
        if (DIM == 1) {
#pragma unroll
            for (int a = 0; a < WMAX; a++) add_cell<float, 2, true>(acc, wc, off[0] + a, val, wt[0][a]);
        } else if (DIM == 2) {
#pragma unroll
            for (int a = 0; a < WMAX; a++) {
                const int rowc = (off[0] + a) * RW + off[1];
                const float wa[2] = {wt[0][a] * val[0], wt[0][a] * val[1]};
#pragma unroll
                for (int b = 0; b < WMAX; b++) add_cell<float, 2, true>(acc, wc, rowc + b, wa, wt[1][b]);
            }
        } else {
#pragma unroll 1
            for (int a = 0; a < WMAX; a++) {
                const float wa = es_weight_at<float>(cx[0], es, a);
#pragma unroll
                for (int b = 0; b < WMAX; b++) {
                    const int rowc = ((off[0] + a) * RW + off[1] + b) * RW + off[2];
                    const float wab[2] = {wa * wt[1][b] * val[0], wa * wt[1][b] * val[1]};
#pragma unroll
                    for (int e = 0; e < WMAX; e++) add_cell<float, 2, true>(acc, wc, rowc + e, wab, wt[2][e]);
                }
            }
        }
    }
    __syncthreads();
    u64* out = slots + (int64_t)blockIdx.x * wc;
    for (int c = threadIdx.x; c < wc; c += blockDim.x) {
        const u64 a = reinterpret_cast<const u64*>(acc)[c];
        out[c] = a;
        ck.add_cell((int)(unsigned)(a & 0xffffffffull));
    }
    if (bad) atomicOr(flag, 2);
    if (over) atomicOr(flag, 8);
    ck.finish((double)csc0, flag);
}

// Per grid cell (every cell written): the sum over the active indices
// a = g + fw + k nf < A of each axis, over the regions whose windows hold a
// (at most two per axis), over each region's slots in order, in double;
// slot values times 2^-e are exact.  sbeg[r] .. sbeg[r+1]-1 are region r's
// sub-problems.
template <int DIM>
__global__ void __launch_bounds__(256) k_region_gather(const unsigned long long* __restrict__ slots,
                                                       const SubProb* __restrict__ sub,
                                                       const int* __restrict__ sbeg, RegionGeom rg, int A, int fw,
                                                       int nf, double* __restrict__ grid, int64_t gcells,
                                                       double inv0, double inv1) {
    using u64 = unsigned long long;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= gcells) return;
    int gl[3] = {0, 0, 0};
    {
        int64_t rem = g;
        for (int l = DIM - 1; l >= 0; l--) { gl[l] = (int)(rem % nf); rem /= nf; }
    }
    int wc = 1;
    for (int l = 0; l < DIM; l++) wc *= rg.RW;
    // per axis: the (active index, region) pairs, at most 2 images x 2 regions
    int ca[3][8], cr[3][8], nc[3] = {1, 1, 1};
    for (int l = 0; l < 3; l++) { ca[l][0] = 0; cr[l][0] = 0; }
    for (int l = 0; l < DIM; l++) {
        nc[l] = 0;
        for (int a = (gl[l] + fw) % nf; a < A; a += nf) {
            const int rlo = a >= rg.RW ? (a - rg.RW) / rg.R + 1 : 0;
            const int rhi = min(rg.nr - 1, a / rg.R);
            for (int r = rlo; r <= rhi && nc[l] < 8; r++) {
                ca[l][nc[l]] = a - r * rg.R;
                cr[l][nc[l]] = r;
                nc[l]++;
            }
        }
    }
    double s0 = 0.0, s1 = 0.0;
    for (int i0 = 0; i0 < nc[0]; i0++)
        for (int i1 = 0; i1 < nc[1]; i1++)
            for (int i2 = 0; i2 < nc[2]; i2++) {
                int reg = cr[0][i0], lc = ca[0][i0];
                if (DIM > 1) { reg = reg * rg.nr + cr[1][i1]; lc = lc * rg.RW + ca[1][i1]; }
                if (DIM > 2) { reg = reg * rg.nr + cr[2][i2]; lc = lc * rg.RW + ca[2][i2]; }
                for (int j = sbeg[reg]; j < sbeg[reg + 1]; j++) {
                    const u64 v = slots[(int64_t)j * wc + lc];
                    const int lo = (int)(unsigned)(v & 0xffffffffull);
                    const int hi = (int)(unsigned)((v - (u64)(long long)lo) >> 32);
                    const double f = ldexp(1.0, -sub[j].e);
                    s0 += (double)lo * f;
                    s1 += (double)hi * f;
                }
            }
    grid[2 * g] = s0 * inv0;
    grid[2 * g + 1] = s1 * inv1;
}

// ---------------------------------------------------------- deconvolution
// Hermitian split of channel c from complex grid c/2 at multi-index j
// (after the grid FFT): returns sum_g chan_c(g) e^{+i k g Delta} at k = j.
__device__ __forceinline__ double2 channel_at(const double2* __restrict__ Z, int64_t gi, int64_t gneg, int part) {
    const double2 a = Z[gi], b = Z[gneg];
    if (part == 0) return make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
    // (a - conj(b)) / (2i)
    return make_double2(0.5 * (a.y + b.y), -0.5 * (a.x - b.x));
}

template <int DIM>
__global__ void k_deconv_v(const double2* __restrict__ Z, int nf, int m, const double* __restrict__ dec,
                           double2* __restrict__ v) {
    const int W2 = 4 * m + 1;
    int64_t tot = 1;
    for (int l = 0; l < DIM; l++) tot *= W2;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= tot) return;
    int64_t rem = idx, gi = 0, gn = 0;
    double f = 1.0;
    int j[3];
    for (int l = DIM - 1; l >= 0; l--) { j[l] = (int)(rem % W2) - 2 * m; rem /= W2; }
    for (int l = 0; l < DIM; l++) {
        int a = j[l] % nf; if (a < 0) a += nf;
        int b = (-j[l]) % nf; if (b < 0) b += nf;
        gi = gi * nf + a;
        gn = gn * nf + b;
        f *= dec[j[l] + 2 * m];
    }
    double2 c = channel_at(Z, gi, gn, 0);
    v[idx] = make_double2(c.x * f, c.y * f);
}

template <typename T, int DIM>
__global__ void k_deconv_b(const double2* __restrict__ Z, int nf, int m, int nrhs, int64_t gcells,
                           const double* __restrict__ dec, const double* __restrict__ D,
                           double2* __restrict__ b64, cpx<T>* __restrict__ bt) {
    const int W = 2 * m + 1;
    int64_t M = 1;
    for (int l = 0; l < DIM; l++) M *= W;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= M * nrhs) return;
    const int r = (int)(idx / M);
    const int64_t jj = idx - (int64_t)r * M;
    int64_t rem = jj, gi = 0, gn = 0;
    double f = D[jj];
    for (int l = DIM - 1; l >= 0; l--) {
        const int j = (int)(rem % W) - m;
        rem /= W;
        f *= dec[j + 2 * m];
    }
    rem = jj;
    int js[3];
    for (int l = DIM - 1; l >= 0; l--) { js[l] = (int)(rem % W) - m; rem /= W; }
    for (int l = 0; l < DIM; l++) {
        int a = js[l] % nf; if (a < 0) a += nf;
        int b = (-js[l]) % nf; if (b < 0) b += nf;
        gi = gi * nf + a;
        gn = gn * nf + b;
    }
    const int ch = r + 1;
    double2 c = channel_at(Z + (int64_t)(ch >> 1) * gcells, gi, gn, ch & 1);
    double2 o = make_double2(c.x * f, c.y * f);
    b64[idx] = o;
    cpx<T> t;
    t.x = (T)o.x;
    t.y = (T)o.y;
    bt[idx] = t;
}

// v (on J_2m) embedded periodically in the L^d array (zero elsewhere).
template <int DIM>
__global__ void k_embed_v(const double2* __restrict__ v, int m, int L, double2* __restrict__ out) {
    int64_t tot = 1;
    for (int l = 0; l < DIM; l++) tot *= L;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= tot) return;
    const int W2 = 4 * m + 1;
    int64_t rem = idx, vi = 0;
    bool inside = true;
    for (int l = DIM - 1; l >= 0; l--) {
        int k = (int)(rem % L);
        rem /= L;
        int j = k <= 2 * m ? k : k - L;  // representative in (-L/2, L/2]
        if (j < -2 * m || j > 2 * m) inside = false;
        (void)j;
    }
    if (!inside) { out[idx] = make_double2(0.0, 0.0); return; }
    rem = idx;
    int js[3];
    for (int l = DIM - 1; l >= 0; l--) {
        int k = (int)(rem % L);
        rem /= L;
        js[l] = k <= 2 * m ? k : k - L;
    }
    for (int l = 0; l < DIM; l++) vi = vi * W2 + (js[l] + 2 * m);
    out[idx] = v[vi];
}

template <typename T>
__global__ void k_scale_to(const double2* __restrict__ in, int64_t n, double s, cpx<T>* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    cpx<T> t;
    t.x = (T)(in[i].x * s);
    t.y = (T)(in[i].y * s);
    out[i] = t;
}

static __global__ void k_scale_inplace(double2* __restrict__ a, int64_t n, double s) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = make_double2(a[i].x * s, a[i].y * s);
}

template <typename T>
__global__ void k_zero_d(T* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (T)0;
}

template <typename T>
__global__ void k_to_T(const double* __restrict__ in, int64_t n, T* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (T)in[i];
}

// ----------------------------------------------------------- orchestration
struct Timer {
    hipEvent_t e[8] = {};
    int k = 0, dev = 0;
    hipStream_t s;
    explicit Timer(hipStream_t st) : dev(current_device()), s(st) {
        for (auto& x : e) x = acquire_event(true);
    }
    void mark() { EFGP_HIP(hipEventRecord(e[k++], s)); }
    double ms(int a, int b) {
        float t = 0;
        EFGP_HIP(hipEventElapsedTime(&t, e[a], e[b]));
        return t;
    }
    ~Timer() {
        for (auto& x : e) release_event(dev, x, true);
    }
};

static int lds_limit_bytes() {
    int dev = 0, v = 65536;
    if (hipGetDevice(&dev) == hipSuccess) {
        int a = 0;
        if (hipDeviceGetAttribute(&a, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && a > 0) v = a;
    }
    return v;
}

static int num_cus() {
    int dev = 0, v = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        int a = 0;
        if (hipDeviceGetAttribute(&a, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && a > 0) v = a;
    }
    return v;
}

template <typename T, int DIM, int WMAX, int NCH, bool EXACT>
static void launch_gridlds(const T* x, const T* y, int64_t n, const Es<T>& es, int A, int nblk, int64_t chunk,
                           int64_t epoch, int nepoch, typename Acc<T>::t* partial, int* flag, size_t lds,
                           const Scales& sc, hipStream_t s) {
    if (EXACT && es.w != WMAX) throw StatusError{EFGP_EINVAL, "internal: spread width mismatch"};
    auto kfn = k_spread_gridlds<T, DIM, WMAX, NCH, EXACT>;
    EFGP_HIP(hipFuncSetAttribute((const void*)kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(kfn, dim3(nblk), dim3(1024), lds, s, x, y, n, es, A, chunk, epoch, nepoch, partial, flag, sc);
    EFGP_HIP(hipGetLastError());
}

template <typename T, int DIM, int WMAX>
static void launch_tiles(const T* xs, const T* ys, int64_t n, int nchan, int cg, const Es<T>& es, int T_, int nt,
                         int nf, const SubProb* sub, int nsub, double* grid, int64_t gcells, int* flag, size_t lds,
                         const Scales& sc, hipStream_t s) {
    auto kfn = k_spread_tiles<T, DIM, WMAX>;
    if (lds > 65536)
        EFGP_HIP(hipFuncSetAttribute((const void*)kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(kfn, dim3(nsub), dim3(256), lds, s, xs, ys, n, nchan, cg, es, T_, nt, nf, sub, grid, gcells,
                       flag, sc);
    EFGP_HIP(hipGetLastError());
}

template <int DIM, int WMAX, bool EXACT>
static void launch_tiles_ch(const float* xs, const unsigned* perm, const float* ypm, int64_t n, int nrhs,
                            const Es<float>& es, int T_, int nt, int nf, const SubProb* sub, int nsub, double* grid,
                            int64_t gcells, int* flag, size_t lds, const Scales& sc, hipStream_t s) {
    auto kfn = k_spread_tiles_ch<DIM, WMAX, EXACT>;
    if (lds > 65536)
        EFGP_HIP(hipFuncSetAttribute((const void*)kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(kfn, dim3(nsub), dim3(256), lds, s, xs, perm, ypm, n, nrhs, es, T_, nt, nf, sub, grid, gcells,
                       flag, sc);
    EFGP_HIP(hipGetLastError());
}

template <int DIM, int WMAX>
static void launch_regions(const float* xs, const float* ys, int64_t n, const Es<float>& es, const RegionGeom& rg,
                           const SubProb* sub, int nsub, unsigned long long* slots, int* flag, size_t lds,
                           const Scales& sc, hipStream_t s) {
    if (es.w != WMAX) throw StatusError{EFGP_EINVAL, "internal: spread width mismatch"};
    auto kfn = k_spread_regions<DIM, WMAX>;
    EFGP_HIP(hipFuncSetAttribute((const void*)kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(kfn, dim3(nsub), dim3(1024), lds, s, xs, ys, n, es, rg, sub, slots, flag, sc);
    EFGP_HIP(hipGetLastError());
}

template <typename T, int DIM, int PT>
static void launch_region_scatter(const T* x, const T* y, int64_t n, const Es<T>& es, const RegionGeom& rg, int nb,
                                  int64_t chunk, const unsigned* boff, const unsigned long long* rstart,
                                  const unsigned long long* totals, T* xs, T* ys, int* flag, size_t lds,
                                  hipStream_t s) {
    auto kfn = k_region_scatter<T, DIM, PT>;
    EFGP_HIP(hipFuncSetAttribute((const void*)kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(kfn, dim3(nb), dim3(1024), lds, s, x, y, n, es, rg, chunk, boff, rstart, totals, xs, ys, flag);
    EFGP_HIP(hipGetLastError());
}

// Region spreader under AUTO: at least this many points per active stencil
// origin (below it the tiled spreader's smaller windows cost less to clear
// and write out)
constexpr double kRegionMinLoad = 4.0;
// most regions the partition ranks in LDS
constexpr int kMaxRegions = 4096;

// Data vectors from which precision 32 in 1D and 2D takes the
// channel-parallel spreader
constexpr int kChanParMin = 16;

// One setup pass.  sampled (precision 32): the data scales come from the
// maximum of a sample of each data vector (contiguous chunks spread over it)
// instead of a pass over all of it.  The power-of-two scale S chosen from it
// keeps the fixed-point sums exact for every |y| <= lim / S (1x to 2x the
// sampled maximum); the spreaders flag any value beyond that bound (or NaN),
// and the pass then returns true and its results are discarded: the caller
// repeats the setup with the exact maximum.  When the whole vector lies
// within the bound, the scale is the one the exact maximum gives whenever
// both maxima fall in the same power-of-two range.
// safe (precision 32): the unit channel's scale assumes every point of an
// epoch in one cell instead of the expected cell load; the pass returns 2
// when a spreader detected an overflow of the load-based scale (the caller
// then repeats the setup with safe set).  Returns 1 for a value beyond the
// sampled bound, 0 when the results stand.
enum { PASS_OK = 0, PASS_REDO_EXACT_MAX = 1, PASS_REDO_SAFE_SCALE = 2 };
template <typename T, int DIM>
static int setup_pass(Plan& P, const efgp_problem& pr, hipStream_t s, bool sampled, bool safe) {
    const T* x = static_cast<const T*>(pr.x);
    const T* y = static_cast<const T*>(pr.y);
    const int64_t n = pr.n;
    const int nf = P.nf, w = P.w;
    const int nchan = 1 + P.nrhs;
    const int ngrid = (nchan + 1) / 2;
    const int64_t gcells = ipow(nf, DIM);

    Es<T> es;
    es.beta = std::is_same<T, float>::value ? (T)(P.es_beta * 1.4426950408889634) : (T)P.es_beta;
    es.inv_hw = (T)(2.0 / w);
    es.half_w = (T)(0.5 * w);
    es.scale = (T)(P.h * nf);
    es.w = w;
    es.fw = w / 2;

    Scratch scratch;  // all temporaries of this setup
    int* flag = static_cast<int*>(scratch.take(sizeof(int) * 4));
    EFGP_HIP(hipMemsetAsync(flag, 0, sizeof(int) * 4, s));
    double* grid = static_cast<double*>(scratch.take(sizeof(double) * 2 * gcells * ngrid));

    Timer tm(s);
    tm.mark();  // 0
    // ---- per-channel accumulator scales (precision 32: fixed point)
    const bool fixed = std::is_same<T, float>::value;
    std::vector<double> ymax(P.nrhs, 1.0);
    if (fixed) {
        unsigned* dmax = static_cast<unsigned*>(scratch.take(sizeof(unsigned) * P.nrhs));
        std::vector<unsigned> hm(P.nrhs);
        // sampled: 256 chunks, 2^24 values in all, only for one data vector
        // (with many, one of them exceeding its bound, and so a second pass,
        // becomes likely) and only when the sample is well short of it
        const int64_t per = (int64_t)1 << 24;
        bool use_sample = sampled && P.nrhs == 1 && n > 4 * per;
        if (use_sample) {
            EFGP_HIP(hipMemsetAsync(dmax, 0, sizeof(unsigned) * P.nrhs, s));
            hipLaunchKernelGGL((k_absmax_sample<T>), dim3(256, P.nrhs), dim3(256), 0, s, y, n, per / 256, dmax);
            EFGP_HIP(hipGetLastError());
            EFGP_HIP(hipMemcpyAsync(hm.data(), dmax, sizeof(unsigned) * P.nrhs, hipMemcpyDeviceToHost, s));
            EFGP_HIP(hipStreamSynchronize(s));
            for (int r = 0; r < P.nrhs; r++) {
                float f;
                std::memcpy(&f, &hm[r], sizeof(float));
                if (!std::isfinite(f)) use_sample = false;   // let the exact pass reject it
                ymax[r] = f > 0.0f ? 1.001 * (double)f : 1.0;
            }
        }
        if (!use_sample) {
            EFGP_HIP(hipMemsetAsync(dmax, 0, sizeof(unsigned) * P.nrhs, s));
            // about 8 blocks per CU over all the vectors together: many more
            // would end in contended atomics on the nrhs maxima
            const unsigned gx = std::max(1u, std::min(cdiv(n, 256), (unsigned)(num_cus() * 8 / P.nrhs)));
            hipLaunchKernelGGL((k_absmax<T>), dim3(gx, P.nrhs), dim3(256), 0, s, y, n, dmax, flag);
            EFGP_HIP(hipGetLastError());
            int hf = 0;
            EFGP_HIP(hipMemcpyAsync(hm.data(), dmax, sizeof(unsigned) * P.nrhs, hipMemcpyDeviceToHost, s));
            EFGP_HIP(hipMemcpyAsync(&hf, flag, sizeof(int), hipMemcpyDeviceToHost, s));
            EFGP_HIP(hipStreamSynchronize(s));
            if (hf & 4) throw StatusError{EFGP_EINVAL, "non-finite data values"};
            for (int r = 0; r < P.nrhs; r++) {
                float f;
                std::memcpy(&f, &hm[r], sizeof(float));
                ymax[r] = f > 0.0f ? 1.001 * (double)f : 1.0;
            }
        }
        sampled = use_sample;
    } else {
        sampled = false;
    }
    // Fixed-point scales for blocks that accumulate at most `pmax` points per
    // epoch, `load` the expected sum of kernel weights one cell receives in
    // an epoch.  The unit channel's scale S_0 is the largest power of two
    // with 8 x load x S_0 <= 2^30 (the spreaders detect an overflow and the
    // setup repeats with the worst-case bound pmax S_0 <= 2^30); 2^21 keeps
    // every product exactly roundable.  A data channel gets the largest power
    // of two S_c <= S_0 / max|y_c|, so |y| S_c <= S_0 and its cells never
    // exceed the unit channel's in magnitude.
    auto make_scales = [&](int64_t pmax, double load) {
        Scales sc;
        for (int c = 0; c < kMaxChan; c++) { sc.s[c] = 1.0f; sc.inv[c] = 1.0; sc.lim[c] = INFINITY; }
        if (fixed) {
            double lim = std::min(1073741824.0 / (double)std::max<int64_t>(1, pmax), 2097152.0);
            if (!safe && load > 0.0) lim = std::max(lim, std::min(1073741824.0 / (8.0 * load), 2097152.0));
            lim = std::exp2(std::floor(std::log2(lim)));
            for (int c = 0; c < nchan && c < kMaxChan; c++) {
                double sv = c == 0 ? lim : lim / ymax[c - 1];
                sv = std::exp2(std::floor(std::log2(sv)));  // power of two: exact decode
                sc.s[c] = (float)sv;
                sc.inv[c] = 1.0 / sv;
                // with sampled maxima every value must stay within what the
                // scale guarantees, |y| sv <= lim (between 1x and 2x the
                // sampled maximum)
                if (c > 0 && sampled) {
                    float fl = (float)(lim / sv);
                    if ((double)fl > lim / sv) fl = std::nextafter(fl, 0.0f);   // never above the bound
                    sc.lim[c] = fl;
                }
            }
        }
        return sc;
    };
    // kernel weight mass of one point: (largest stencil sum over sub-cell
    // offsets)^d, with the stencil rule of es_stencil
    double mass = 1.0;
    {
        double best = 1.0;
        for (int k = 0; k < 16; k++) {
            const double u = 64.0 + (k + 0.5) / 16.0;
            const double g0 = std::ceil(u - 0.5 * w);
            double sum = 0.0;
            for (int j = 0; j < w; j++) {
                const double z = (g0 + j - u) / (0.5 * w);
                if (std::fabs(z) < 1.0) sum += std::exp(P.es_beta * (std::sqrt(1.0 - z * z) - 1.0));
            }
            best = std::max(best, sum);
        }
        for (int l = 0; l < DIM; l++) mass *= best;
    }
    // ---- choose the spreader
    const int lds_max = lds_limit_bytes();
    const int A = (int)std::floor(P.h * nf) + w + 1;
    const size_t lds_grid = (size_t)ipow(A, DIM) * nchan * sizeof(typename Acc<T>::t) + kOvfLds;
    bool use_grid = false;
    if (P.spread_method == EFGP_SPREAD_GRID_LDS || P.spread_method == EFGP_SPREAD_AUTO) {
        bool fits = nchan == 2 && lds_grid + 1024 <= (size_t)lds_max && w <= 16;
        if (P.spread_method == EFGP_SPREAD_GRID_LDS && !fits)
            throw StatusError{EFGP_EINVAL, "active region does not fit in LDS for the grid spreader"};
        // the whole-region spreader pays a zero-fill and write-out of the
        // region per block; it wins when there are many points per cell
        use_grid = fits && (P.spread_method == EFGP_SPREAD_GRID_LDS ||
                            (double)n >= 64.0 * (double)ipow(A, DIM) * num_cus());
    }
    // ---- the region spreader (precision 32, one data vector): the active
    // region exceeds LDS; regions of R origins per axis whose windows fit
    const int ocount_all = (int)std::floor(P.h * nf) + 2;   // stencil origins 0 .. floor(h nf) + 1 per axis
    RegionGeom rg{};
    bool use_regions = false;
    if (!use_grid && (P.spread_method == EFGP_SPREAD_REGIONS || P.spread_method == EFGP_SPREAD_AUTO)) {
        const bool explicit_regions = P.spread_method == EFGP_SPREAD_REGIONS;
        const bool able = fixed && nchan == 2;
        if (explicit_regions && !able)
            throw StatusError{EFGP_EINVAL, "the region spreader takes precision 32 with one data vector"};
        if (able) {
            int RWmax = (int)std::floor(std::pow((double)(lds_max - 1024) / 8.0, 1.0 / DIM) + 1e-9);
            while (RWmax > 1 && (size_t)ipow(RWmax, DIM) * 8 + kOvfLds + 1024 > (size_t)lds_max) RWmax--;
            int Rmax = RWmax - (w - 1);
            if (explicit_regions && P.tile > 0) {
                if (P.tile > Rmax) throw StatusError{EFGP_ETOOLARGE, "region window exceeds LDS"};
                Rmax = P.tile;
            }
            // R >= w keeps every active index in at most two windows per axis
            const int nr = Rmax >= w ? (ocount_all + Rmax - 1) / Rmax : 0;
            if (nr > 0 && ipow(nr, DIM) <= kMaxRegions) {
                const int R = (ocount_all + nr - 1) / nr;
                rg = RegionGeom{R, R + w - 1, nr, (int)ipow(nr, DIM), ocount_all - 1, 1.0f / (float)R};
                // under AUTO only where the whole region does not fit in LDS
                use_regions = explicit_regions || (lds_grid + 1024 > (size_t)lds_max &&
                                                   (double)n >= kRegionMinLoad * (double)ipow(ocount_all, DIM));
            } else if (explicit_regions) {
                throw StatusError{EFGP_ETOOLARGE, "region window below the kernel width or too many regions"};
            }
        }
    }
    if (use_regions) {
        if constexpr (std::is_same<T, float>::value) {
        P.spread_method = EFGP_SPREAD_REGIONS;
        P.tile = rg.R;
        const int nreg = rg.nreg;
        // ---- pass 1: each block's points per region, then offsets
        const int64_t nbt = std::max<int64_t>(1, std::min<int64_t>((int64_t)num_cus() * 8, cdiv(n, 8192)));
        const int64_t chunk = (n + nbt - 1) / nbt;
        const int nb = (int)((n + chunk - 1) / chunk);
        unsigned* counts = static_cast<unsigned*>(scratch.take(sizeof(unsigned) * (size_t)nreg * nb));
        auto* totals = static_cast<unsigned long long*>(scratch.take(sizeof(unsigned long long) * nreg));
        auto* rstart = static_cast<unsigned long long*>(scratch.take(sizeof(unsigned long long) * nreg));
        hipLaunchKernelGGL((k_region_count<T, DIM>), dim3(nb), dim3(256), sizeof(unsigned) * nreg, s, x, n, es, rg,
                           chunk, counts, flag);
        hipLaunchKernelGGL(k_region_scan, dim3(nreg), dim3(256), 0, s, counts, nb, totals);
        EFGP_HIP(hipGetLastError());
        std::vector<unsigned long long> ht(nreg), hs(nreg);
        EFGP_HIP(hipMemcpyAsync(ht.data(), totals, sizeof(unsigned long long) * nreg, hipMemcpyDeviceToHost, s));
        EFGP_HIP(hipStreamSynchronize(s));
        unsigned long long tot = 0;
        for (int r = 0; r < nreg; r++) {
            hs[r] = tot;
            tot += ht[r];
        }
        if (tot != (unsigned long long)n) throw StatusError{EFGP_EHIP, "region histogram does not sum to N"};
        upload_async(P, rstart, hs.data(), sizeof(unsigned long long) * nreg, s);
        // ---- pass 2: the points in region order
        T* xs = static_cast<T*>(scratch.take(sizeof(T) * (size_t)n * DIM));
        T* ys = static_cast<T*>(scratch.take(sizeof(T) * (size_t)n));
        auto lds_scatter = [&](int pt) {
            return (size_t)pt * 1024 * ((DIM + 1) * sizeof(T) + sizeof(unsigned short)) + 3 * sizeof(unsigned) * nreg + 64;
        };
        if (lds_scatter(8) <= (size_t)lds_max)
            launch_region_scatter<T, DIM, 8>(x, y, n, es, rg, nb, chunk, counts, rstart, totals, xs, ys, flag, lds_scatter(8), s);
        else if (lds_scatter(4) <= (size_t)lds_max)
            launch_region_scatter<T, DIM, 4>(x, y, n, es, rg, nb, chunk, counts, rstart, totals, xs, ys, flag, lds_scatter(4), s);
        else
            launch_region_scatter<T, DIM, 1>(x, y, n, es, rg, nb, chunk, counts, rstart, totals, xs, ys, flag, lds_scatter(1), s);
        // ---- sub-problems: each region in equal runs of at most S points
        // (about 8 per CU in all); one scale exponent per region, from its
        // longest run and the expected load of its origins
        const int64_t ep = P.spread_epoch > 0 ? P.spread_epoch : 1 << 20;
        const int64_t S = std::min<int64_t>(ep, std::max<int64_t>(4096, n / ((int64_t)num_cus() * 8) + 1));
        const Scales sc = make_scales(1, 0.0);
        auto reg_exp = [&](int r, int64_t cnt) -> int {
            double org = 1.0;
            int rem = r;
            for (int l = DIM - 1; l >= 0; l--) {
                const int rl = rem % rg.nr;
                rem /= rg.nr;
                org *= (double)std::max(1, std::min(rg.R, ocount_all - rl * rg.R));
            }
            double sv = 1073741824.0 / (double)std::max<int64_t>(1, cnt);
            if (!safe) sv = std::max(sv, 1073741824.0 / (8.0 * (double)cnt * mass / org));
            sv = std::min(sv, 2097152.0);
            return std::min(0, (int)std::floor(std::log2(sv)) - 21);
        };
        std::vector<SubProb> subs;
        std::vector<int> sbeg(nreg + 1, 0);
        for (int r = 0; r < nreg; r++) {
            const int64_t c = (int64_t)ht[r];
            if (c > 0) {
                const int64_t k = (c + S - 1) / S;
                const int64_t Sr = (c + k - 1) / k;
                const int e = reg_exp(r, Sr);
                for (int64_t st = 0; st < c; st += Sr)
                    subs.push_back(SubProb{r, 0, (int64_t)hs[r] + st, std::min(Sr, c - st), e, 0});
            }
            sbeg[r + 1] = (int)subs.size();
        }
        const int nsub = (int)subs.size();
        SubProb* dsub = static_cast<SubProb*>(scratch.take(sizeof(SubProb) * std::max(1, nsub)));
        int* dsbeg = static_cast<int*>(scratch.take(sizeof(int) * (nreg + 1)));
        if (nsub > 0) upload_async(P, dsub, subs.data(), sizeof(SubProb) * nsub, s);
        upload_async(P, dsbeg, sbeg.data(), sizeof(int) * (nreg + 1), s);
        tm.mark();  // 1 (partition)
        const int64_t wc = ipow(rg.RW, DIM);
        auto* slots = static_cast<unsigned long long*>(scratch.take(sizeof(unsigned long long) * wc * std::max(1, nsub)));
        const size_t lds_reg = (size_t)wc * 8 + kOvfLds;
        if (nsub > 0) {
#define EFGP_RG(WM) launch_regions<DIM, WM>(xs, ys, n, es, rg, dsub, nsub, slots, flag, lds_reg, sc, s)
            if (w == 3) EFGP_RG(3);
            else if (w == 4) EFGP_RG(4);
            else if (w == 5) EFGP_RG(5);
            else if (w == 6) EFGP_RG(6);
            else if (w == 7) EFGP_RG(7);
            else if (w == 8) EFGP_RG(8);
            else throw StatusError{EFGP_EINVAL, "internal: precision-32 kernel width above 8"};
#undef EFGP_RG
        }
        hipLaunchKernelGGL((k_region_gather<DIM>), dim3(cdiv(gcells, 256)), dim3(256), 0, s, slots, dsub, dsbeg, rg,
                           ocount_all + w - 1, w / 2, nf, grid, gcells, sc.inv[0], sc.inv[1]);
        EFGP_HIP(hipGetLastError());
        tm.mark();  // 2
        }
    } else if (use_grid) {
        P.spread_method = EFGP_SPREAD_GRID_LDS;
        const int nblk = num_cus();
        // chunks are multiples of the block size so every block's loads stay aligned
        int64_t chunk = (n + nblk - 1) / nblk;
        chunk = (chunk + 1023) / 1024 * 1024;
        const int nb_used = (int)((n + chunk - 1) / chunk);
        // epochs bound the fixed-point sums; double accumulates the whole chunk
        // (default 2^20 points: with the load-based scale the quantum is then
        // ~2^-18 at N = 1e9, and the epoch slots written and summed shrink 4x
        // against 2^18-point epochs)
        const int64_t epoch = fixed ? std::min<int64_t>(chunk, P.spread_epoch > 0 ? P.spread_epoch : 1 << 20) : chunk;
        const int nepoch = (int)((chunk + epoch - 1) / epoch);
        const Scales sc = make_scales(epoch, (double)epoch * mass / (double)ipow(A - w, DIM));
        using Ac = typename Acc<T>::t;
        Ac* partial = static_cast<Ac*>(scratch.take((size_t)nb_used * nepoch * ipow(A, DIM) * nchan * sizeof(Ac)));
        tm.mark();  // 1 (no sort)
#define EFGP_GL(WM, EX)                                                                                   \
    launch_gridlds<T, DIM, WM, 2, EX>(x, y, n, es, A, nb_used, chunk, epoch, nepoch, partial, flag, lds_grid, sc, s)
        // precision 32 (w <= 8 for every tolerance it accepts) gets a kernel
        // per exact width; precision 64 shares width classes
        if (fixed && w == 3) EFGP_GL(3, true);
        else if (fixed && w == 4) EFGP_GL(4, true);
        else if (fixed && w == 5) EFGP_GL(5, true);
        else if (fixed && w == 6) EFGP_GL(6, true);
        else if (fixed && w == 7) EFGP_GL(7, true);
        else if (fixed && w == 8) EFGP_GL(8, true);
        else if (w <= 4) EFGP_GL(4, false);
        else if (w <= 6) EFGP_GL(6, false);
        else if (w <= 8) EFGP_GL(8, false);
        else if (w <= 12) EFGP_GL(12, false);
        else EFGP_GL(16, false);
#undef EFGP_GL
        tm.mark();  // 2 (spread kernel alone)
        {
            const int nslot = nb_used * nepoch;
            const int nchunk = std::min(nslot, 64);
            const int64_t elems = ipow(A, DIM) * nchan;
            SumT<T>* psum = static_cast<SumT<T>*>(scratch.take(sizeof(SumT<T>) * elems * nchunk));
            hipLaunchKernelGGL((k_slot_sum<T>), dim3(cdiv(elems, 256), nchunk), dim3(256), 0, s, partial, nslot,
                               elems, nchunk, psum);
            // precision 32 with two channels packs them cell-major (k_spread_gridlds)
            const bool cell_major = fixed && nchan == 2;
            hipLaunchKernelGGL((k_reduce_partials<T, DIM>), dim3(cdiv(gcells, 256)), dim3(256), 0, s, psum, nchunk,
                               A, nchan, cell_major, w / 2, nf, grid, gcells, sc);
        }
        EFGP_HIP(hipGetLastError());
    } else {
        P.spread_method = EFGP_SPREAD_TILES;
        // ---- tile geometry.  Many data vectors (precision 32, d <= 2) take
        // the channel-parallel spreader, whose tile is sized so that its
        // [cell][channel] accumulator stays near 44 KB (three blocks per CU)
        bool chpar = fixed && DIM <= 2 && P.nrhs >= kChanParMin && w <= 8;
        int T_ = P.tile;
        if (T_ <= 0) T_ = DIM == 1 ? 256 : (DIM == 2 ? 32 : 8);
        if (chpar) {
            const double cells = 44.0 * 1024 / (sizeof(int) * (double)nchan);
            const int Pc = (int)std::floor(std::pow(cells, 1.0 / DIM) + 1e-9);
            T_ = std::max(2, Pc - w + 1);
        }
        const int active = (int)std::floor(P.h * nf) + 3;  // shifted origins 0..floor(h nf)+1, margin 1
        while (ipow((active + T_ - 1) / T_, DIM) > 4096) T_ *= 2;
        // k_spread_tiles_ch: unit channel (int per cell, padded to even) and
        // pairs of data vectors (64-bit per cell and pair)
        const size_t pc_ch = (size_t)ipow(T_ + w - 1, DIM);
        const size_t lds_ch = ((pc_ch + 1) & ~(size_t)1) * sizeof(int) + pc_ch * ((P.nrhs + 1) / 2) * 8;
        if (chpar && lds_ch > (size_t)lds_max) chpar = false;
        const int nt = (active + T_ - 1) / T_;
        const int ntiles = (int)ipow(nt, DIM);
        P.tile = T_;
        const int Pp = T_ + w - 1;
        const size_t tile_cells = (size_t)ipow(Pp, DIM);
        const size_t acc_size = sizeof(typename Acc<T>::t);
        int cg = (int)std::min<size_t>(8, (48 * 1024) / (tile_cells * acc_size));
        if (cg < 1) {
            cg = 1;
            if (tile_cells * acc_size > (size_t)lds_max) throw StatusError{EFGP_ETOOLARGE, "spread tile exceeds LDS"};
        }
        cg = std::min(cg, nchan);
        const size_t lds_tile = tile_cells * cg * acc_size + kOvfLds;

        unsigned* counts = static_cast<unsigned*>(scratch.take(sizeof(unsigned) * (ntiles + 1) * 2));
        unsigned* cursor = counts + (ntiles + 1);
        EFGP_HIP(hipMemsetAsync(counts, 0, sizeof(unsigned) * (ntiles + 1) * 2, s));
        const size_t lds_hist = sizeof(unsigned) * (ntiles + 1);
        const int nblk_count = std::max(1, std::min<int>(num_cus() * 8, (int)cdiv(n, 256)));
        hipLaunchKernelGGL((k_tile_count<T, DIM>), dim3(nblk_count), dim3(256), lds_hist, s, x, n, es, T_, nt, ntiles,
                           counts, flag);
        EFGP_HIP(hipGetLastError());
        std::vector<unsigned> hc(ntiles + 1);
        EFGP_HIP(hipMemcpyAsync(hc.data(), counts, sizeof(unsigned) * (ntiles + 1), hipMemcpyDeviceToHost, s));
        EFGP_HIP(hipStreamSynchronize(s));
        std::vector<unsigned> off(ntiles + 1);
        uint64_t acc = 0;
        for (int t = 0; t <= ntiles; t++) {
            off[t] = (unsigned)acc;
            acc += hc[t];
        }
        if (acc != (uint64_t)n) throw StatusError{EFGP_EHIP, "tile histogram does not sum to N"};
        upload_async(P, cursor, off.data(), sizeof(unsigned) * (ntiles + 1), s);
        T* xs = static_cast<T*>(scratch.take(sizeof(T) * (size_t)n * DIM));
        T* ys = nullptr;
        T* ypm = nullptr;
        unsigned* perm = nullptr;
        if (chpar) {
            // data point-major (one row per point); the sort moves a permutation
            const int ld = (P.nrhs + 1) & ~1;
            ypm = static_cast<T*>(scratch.take(sizeof(T) * (size_t)n * ld));
            perm = static_cast<unsigned*>(scratch.take(sizeof(unsigned) * (size_t)n));
            hipLaunchKernelGGL((k_transpose_y<T>), dim3(cdiv(n, 64)), dim3(256), sizeof(T) * P.nrhs * 65, s, y, n,
                               P.nrhs, ld, ypm);
        } else {
            ys = static_cast<T*>(scratch.take(sizeof(T) * (size_t)n * P.nrhs));
        }
        const int64_t chunk = 4096;
        hipLaunchKernelGGL((k_tile_scatter<T, DIM>), dim3(cdiv(n, chunk)), dim3(256), 2 * lds_hist, s, x, y, n,
                           P.nrhs, es, T_, nt, ntiles, chunk, cursor, xs, ys, perm);
        EFGP_HIP(hipGetLastError());
        // ---- sub-problems: chunks of at most S points per tile and channel group
        // (precision 32 in 3D: at most 2048 points, so that a block's
        // expected cell load allows a fixed-point quantum near 2^-20: the
        // 343-cell stencils of w = 7 hold many small products, which coarser
        // quanta round away, a bias of the whole grid)
        const int tep = P.spread_epoch > 0 ? P.spread_epoch : 1 << 18;
        const int64_t smax = fixed ? (DIM == 3 ? std::min(2048, tep) : tep) : (1 << 20);
        const int64_t S = std::max<int64_t>(std::min<int64_t>(2048, smax),
                                            std::min<int64_t>(smax, n / (int64_t)(num_cus() * 4) + 1));
        int64_t max_count = 1;
        for (int t = 0; t < ntiles; t++) max_count = std::max<int64_t>(max_count, hc[t]);
        // Scales.  The many-vector spreader keeps one worst-case scale for
        // all blocks (no overflow check).  Otherwise each sub-problem gets
        // its own power of two 2^e below the largest scale, from its own
        // count and the expected load of its cells (points spread evenly
        // over the tile's stencil origins; edge tiles hold fewer origins);
        // on an overflow the setup repeats with each block's worst case.
        const int64_t pmax = std::min(S, max_count);
        const Scales sc = make_scales(chpar ? pmax : 1, 0.0);
        const int ocount = (int)std::floor(P.h * nf) + 2;   // stencil origins 0 .. floor(h nf) + 1 per axis
        auto sub_exp = [&](int t, int64_t cnt) -> int {
            if (!fixed || chpar) return 0;
            double org = 1.0;
            int rem = t;
            for (int l = 0; l < DIM; l++) {
                const int tl = rem % nt;
                rem /= nt;
                org *= (double)std::max(1, std::min(T_, ocount - tl * T_));
            }
            double sv = 1073741824.0 / (double)std::max<int64_t>(1, cnt);
            if (!safe) sv = std::max(sv, 1073741824.0 / (8.0 * (double)cnt * mass / org));
            sv = std::min(sv, 2097152.0);
            return std::min(0, (int)std::floor(std::log2(sv)) - 21);
        };
        std::vector<SubProb> subs;
        for (int t = 0; t < ntiles; t++) {
            const int64_t c = hc[t];
            for (int64_t st = 0; st < c; st += S) {
                const int64_t cnt = std::min(S, c - st);
                const int e = sub_exp(t, cnt);
                for (int c0 = 0; c0 < nchan; c0 += chpar ? nchan : cg)
                    subs.push_back(SubProb{t, c0, (int64_t)off[t] + st, cnt, e, 0});
            }
        }
        SubProb* dsub = static_cast<SubProb*>(scratch.take(sizeof(SubProb) * std::max<size_t>(1, subs.size())));
        if (!subs.empty())
            upload_async(P, dsub, subs.data(), sizeof(SubProb) * subs.size(), s);
        hipLaunchKernelGGL(k_zero_d<double>, dim3(cdiv(2 * gcells * ngrid, 256)), dim3(256), 0, s, grid, 2 * gcells * ngrid);
        tm.mark();  // 1
        if (!subs.empty() && chpar) {
            if constexpr (std::is_same<T, float>::value && DIM <= 2) {
                const int nsub = (int)subs.size();
#define EFGP_TC(WM, EX)                                                                                 \
    launch_tiles_ch<DIM, WM, EX>(xs, perm, ypm, n, P.nrhs, es, T_, nt, nf, dsub, nsub, grid, gcells, flag, lds_ch, sc, s)
                // a kernel per exact width 3..8 (w <= 8 in precision 32)
                if (w == 3) EFGP_TC(3, true);
                else if (w == 4) EFGP_TC(4, true);
                else if (w == 5) EFGP_TC(5, true);
                else if (w == 6) EFGP_TC(6, true);
                else if (w == 7) EFGP_TC(7, true);
                else if (w == 8) EFGP_TC(8, true);
                else EFGP_TC(4, false);
#undef EFGP_TC
            }
        } else if (!subs.empty()) {
            const int nsub = (int)subs.size();
            if (w <= 4) launch_tiles<T, DIM, 4>(xs, ys, n, nchan, cg, es, T_, nt, nf, dsub, nsub, grid, gcells, flag, lds_tile, sc, s);
            else if (w <= 6) launch_tiles<T, DIM, 6>(xs, ys, n, nchan, cg, es, T_, nt, nf, dsub, nsub, grid, gcells, flag, lds_tile, sc, s);
            else if (w <= 8) launch_tiles<T, DIM, 8>(xs, ys, n, nchan, cg, es, T_, nt, nf, dsub, nsub, grid, gcells, flag, lds_tile, sc, s);
            else if (w <= 12) launch_tiles<T, DIM, 12>(xs, ys, n, nchan, cg, es, T_, nt, nf, dsub, nsub, grid, gcells, flag, lds_tile, sc, s);
            else launch_tiles<T, DIM, 16>(xs, ys, n, nchan, cg, es, T_, nt, nf, dsub, nsub, grid, gcells, flag, lds_tile, sc, s);
        }
        tm.mark();  // 2
    }

    // ---- FFT of the spread grid (sign +) along every axis, double
    {
        void* tw = scratch.take(sizeof(double2) * nf);
        upload_twiddles_to<double>(P, nf, tw, s);
        FftDev<double> f;
        f.s = fft_shape(nf);
        f.tw = static_cast<const cpx<double>*>(tw);
        double2* Z = reinterpret_cast<double2*>(grid);
        for (int a = 0; a < DIM; a++) {
            const int64_t inner = ipow(nf, DIM - 1 - a);
            const int64_t outer = ipow(nf, a) * ngrid;
            fft_axis<double>(Z, f, outer, inner, +1, s);
        }
    }
    tm.mark();  // 3
    // ---- deconvolve, truncate, split
    {
        std::vector<double> dec = es_deconv_table(w, P.es_beta, nf, 2 * P.m);
        double* ddec = static_cast<double*>(scratch.take(sizeof(double) * dec.size()));
        upload_async(P, ddec, dec.data(), sizeof(double) * dec.size(), s);
        const double2* Z = reinterpret_cast<const double2*>(grid);
        const int64_t nv = ipow(P.W2, DIM);
        hipLaunchKernelGGL((k_deconv_v<DIM>), dim3(cdiv(nv, 256)), dim3(256), 0, s, Z, nf, P.m, ddec,
                           reinterpret_cast<double2*>(P.v));
        hipLaunchKernelGGL((k_deconv_b<T, DIM>), dim3(cdiv(P.M * P.nrhs, 256)), dim3(256), 0, s, Z, nf, P.m, P.nrhs,
                           gcells, ddec, P.D64, reinterpret_cast<double2*>(P.b64), static_cast<cpx<T>*>(P.b));
        EFGP_HIP(hipGetLastError());
        // dec table must outlive the kernels: synchronised below before freeing
    }
    tm.mark();  // 4
    // ---- vhat = FFT(v embedded at L^d) / L^d
    {
        double2* e = static_cast<double2*>(scratch.take(sizeof(double2) * P.LD));
        hipLaunchKernelGGL((k_embed_v<DIM>), dim3(cdiv(P.LD, 256)), dim3(256), 0, s, reinterpret_cast<double2*>(P.v),
                           P.m, P.L, e);
        void* tw = scratch.take(sizeof(double2) * P.L);
        upload_twiddles_to<double>(P, P.L, tw, s);
        FftDev<double> f;
        f.s = fft_shape(P.L);
        f.tw = static_cast<const cpx<double>*>(tw);
        for (int a = 0; a < DIM; a++)
            fft_axis<double>(e, f, ipow(P.L, a), ipow(P.L, DIM - 1 - a), -1, s);
        hipLaunchKernelGGL((k_scale_to<T>), dim3(cdiv(P.LD, 256)), dim3(256), 0, s, e, P.LD, 1.0 / (double)P.LD,
                           static_cast<cpx<T>*>(P.vhat));
        EFGP_HIP(hipGetLastError());
    }
    tm.mark();  // 5
    int hflag[4] = {0, 0, 0, 0};
    EFGP_HIP(hipMemcpyAsync(hflag, flag, sizeof(int) * 4, hipMemcpyDeviceToHost, s));
    EFGP_HIP(hipStreamSynchronize(s));
    P.ms_sort = tm.ms(0, 1);
    P.ms_spread = tm.ms(1, 2);
    P.ms_fft = tm.ms(2, 3);
    P.ms_deconv = tm.ms(3, 5);
    P.ms_total = tm.ms(0, 5);
    if (hflag[0] & 1) throw StatusError{EFGP_EDOMAIN, "a point lies outside [0,1]^d"};
    if (sampled && (hflag[0] & 8)) return PASS_REDO_EXACT_MAX;   // a value above the sampled bound
    if (hflag[0] & 16) return PASS_REDO_SAFE_SCALE;                 // a unit-channel cell overflowed
    if (hflag[0] & 2) throw StatusError{EFGP_EHIP, "spread tile assignment inconsistent"};
    return PASS_OK;
}

// FFT(v) embedded at L^d, scaled by 1/L^d, in double (the iterative
// refinement of precision-32 solves forms its residuals with it); the same
// steps as the setup's own v-hat, kept in P.vhat64.
template <int DIM>
void vhat64_typed(Plan& P, hipStream_t s) {
    if (!P.vhat64) P.vhat64 = dalloc(P, sizeof(double2) * (size_t)P.LD);
    if (!P.twL64) upload_twiddles<double>(P, P.L, &P.twL64, s);
    double2* e = static_cast<double2*>(P.vhat64);
    hipLaunchKernelGGL((k_embed_v<DIM>), dim3(cdiv(P.LD, 256)), dim3(256), 0, s, reinterpret_cast<double2*>(P.v),
                       P.m, P.L, e);
    FftDev<double> f;
    f.s = fft_shape(P.L);
    f.tw = static_cast<const cpx<double>*>(P.twL64);
    for (int a = 0; a < DIM; a++)
        fft_axis<double>(e, f, ipow(P.L, a), ipow(P.L, DIM - 1 - a), -1, s);
    hipLaunchKernelGGL(k_scale_inplace, dim3(cdiv(P.LD, 256)), dim3(256), 0, s, e, P.LD, 1.0 / (double)P.LD);
    EFGP_HIP(hipGetLastError());
}

// Precision 32 may need up to three passes: the first takes sampled data
// maxima and the load-based unit scale; a value beyond the sampled bound
// repeats it with exact maxima, and an overflow of the unit channel repeats
// it with the worst-case scale (which cannot overflow).
template <typename T, int DIM>
void setup_typed(Plan& P, const efgp_problem& pr, hipStream_t s) {
    bool sampled = std::is_same<T, float>::value, safe = false;
    for (P.setup_passes = 1; P.setup_passes <= 3; P.setup_passes++) {
        const int r = setup_pass<T, DIM>(P, pr, s, sampled, safe);
        if (r == PASS_OK) return;
        if (r == PASS_REDO_EXACT_MAX) sampled = false;
        else safe = true;
    }
    throw StatusError{EFGP_EHIP, "setup did not settle in three passes"};
}

}  // namespace efgp
