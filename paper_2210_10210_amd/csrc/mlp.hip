// Preconditioner network: an MLP 5 -> 64 -> 64 -> 64 -> 1 (ReLU) mapping
// per-frequency features to the log of a multiplicative correction of the
// Jacobi diagonal.  Products run on the matrix cores (gfx950
// v_mfma_f32_16x16x32_bf16: bf16 operands, float accumulation); master
// weights, biases, the last layer and the optimiser are float.
//
// Each wave owns 16-row tiles.  MFMA 16x16x32 operand layout (wave64):
//   A (16 x 32, M x K): lane l holds A[l % 16][8 (l / 16) .. 8 (l / 16) + 7]
//   B (32 x 16, K x N): lane l holds B[8 (l / 16) .. + 7][l % 16]
//   C (16 x 16):        lane l holds C[4 (l / 16) + i][l % 16], i = 0..3
// Weights W[out][in] are staged in LDS as bf16, so the forward B operand
// (B[k][n] = W[n][k]) is a contiguous 16-byte read; the backward products
// use transposed copies staged the same way.
#include <cmath>

#include "efgp_internal.h"
#include "fft_device.h"

namespace efgp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kH = EFGP_MLP_HIDDEN;  // 64
constexpr int kF = EFGP_NFEAT;       // 5
constexpr int kK1 = 32;              // first-layer K padded for the MFMA
// offsets into the packed parameter vector
constexpr int oW1 = 0, ob1 = oW1 + kH * kF, oW2 = ob1 + kH, ob2 = oW2 + kH * kH, oW3 = ob2 + kH,
              ob3 = oW3 + kH * kH, oW4 = ob3 + kH, ob4 = oW4 + kH, kNP = ob4 + 1;
static_assert(kNP == EFGP_MLP_NPARAM, "parameter layout");

// Waves of a block run different numbers of tiles, so tile-local LDS
// hand-offs synchronise the wave only: LDS operations of one wave complete in
// issue order, and the fence keeps the compiler from reordering across it.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ f32x4 mfma(const bf16x8& a, const bf16x8& b, const f32x4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// shared weights of one block
struct MlpLds {
    __bf16 w1[kH][kK1];    // W1 padded to K = 32
    __bf16 w2[kH][kH];
    __bf16 w3[kH][kH];
    __bf16 w2t[kH][kH];    // transposes for the backward products
    __bf16 w3t[kH][kH];
    float b1[kH], b2[kH], b3[kH], w4[kH];
    float b4;
};

__device__ void stage_weights(const float* __restrict__ p, MlpLds& s, bool transposes) {
    for (int i = threadIdx.x; i < kH * kK1; i += blockDim.x) {
        const int o = i / kK1, k = i % kK1;
        s.w1[o][k] = (__bf16)(k < kF ? p[oW1 + o * kF + k] : 0.0f);
    }
    for (int i = threadIdx.x; i < kH * kH; i += blockDim.x) {
        const int o = i / kH, k = i % kH;
        const float a = p[oW2 + i], b = p[oW3 + i];
        s.w2[o][k] = (__bf16)a;
        s.w3[o][k] = (__bf16)b;
        if (transposes) {
            s.w2t[k][o] = (__bf16)a;
            s.w3t[k][o] = (__bf16)b;
        }
    }
    for (int i = threadIdx.x; i < kH; i += blockDim.x) {
        s.b1[i] = p[ob1 + i];
        s.b2[i] = p[ob2 + i];
        s.b3[i] = p[ob3 + i];
        s.w4[i] = p[oW4 + i];
    }
    if (threadIdx.x == 0) s.b4 = p[ob4];
}

// A operand from a row-major float tile act[16][ld] at column offset k0
__device__ __forceinline__ bf16x8 a_rows(const float* act, int ld, int k0, int lane) {
    const float* src = act + (lane & 15) * ld + k0 + 8 * (lane >> 4);
    bf16x8 v;
#pragma unroll
    for (int i = 0; i < 8; i++) v[i] = (__bf16)src[i];
    return v;
}
// B operand from a bf16 matrix W[n][k] (B[k][n] = W[n][k]), tile columns n0..n0+15
template <int LD>
__device__ __forceinline__ bf16x8 b_rows(const __bf16 (*W)[LD], int n0, int k0, int lane) {
    const __bf16* src = &W[n0 + (lane & 15)][k0 + 8 * (lane >> 4)];
    bf16x8 v;
#pragma unroll
    for (int i = 0; i < 8; i++) v[i] = src[i];
    return v;
}

// one dense layer on a 16-row tile: out = relu(in * W^T + b), float tiles in LDS
template <int K, int LD>
__device__ __forceinline__ void layer(const float* in, int ldin, const __bf16 (*W)[LD], const float* b,
                                      float* out, int lane) {
#pragma unroll
    for (int t = 0; t < kH / 16; t++) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k0 = 0; k0 < K; k0 += 32) acc = mfma(a_rows(in, ldin, k0, lane), b_rows<LD>(W, 16 * t, k0, lane), acc);
        const int col = 16 * t + (lane & 15);
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int row = 4 * (lane >> 4) + i;
            out[row * kH + col] = fmaxf(acc[i] + b[col], 0.0f);
        }
    }
}

// per-wave activation tiles
struct WaveTiles {
    float x[16][kK1];
    float h1[16][kH];
    float h2[16][kH];
    float h3[16][kH];
    float dz[16][kH];
    float o[16];
};

__device__ __forceinline__ void forward_tile(const MlpLds& s, WaveTiles& w, const float* __restrict__ feats,
                                             int64_t r0, int64_t rows, int lane) {
    for (int i = lane; i < 16 * kK1; i += 64) {
        const int r = i / kK1, k = i % kK1;
        const int64_t row = r0 + r;
        w.x[r][k] = (k < kF && row < rows) ? feats[row * kF + k] : 0.0f;
    }
    wave_sync();
    layer<kK1, kK1>(&w.x[0][0], kK1, s.w1, s.b1, &w.h1[0][0], lane);
    wave_sync();
    layer<kH, kH>(&w.h1[0][0], kH, s.w2, s.b2, &w.h2[0][0], lane);
    wave_sync();
    layer<kH, kH>(&w.h2[0][0], kH, s.w3, s.b3, &w.h3[0][0], lane);
    wave_sync();
    if (lane < 16) {
        float acc = s.b4;
        for (int k = 0; k < kH; k++) acc += w.h3[lane][k] * s.w4[k];
        w.o[lane] = acc;
    }
    wave_sync();
}

__global__ void __launch_bounds__(256) k_mlp_forward(const float* __restrict__ params, int64_t rows,
                                                     const float* __restrict__ feats, float* __restrict__ out) {
    __shared__ MlpLds s;
    __shared__ WaveTiles tiles[4];
    stage_weights(params, s, false);
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    WaveTiles& w = tiles[wv];
    const int64_t ntile = (rows + 15) / 16;
    for (int64_t t = (int64_t)blockIdx.x * 4 + wv; t < ntile; t += (int64_t)gridDim.x * 4) {
        forward_tile(s, w, feats, t * 16, rows, lane);
        if (lane < 16 && t * 16 + lane < rows) out[t * 16 + lane] = w.o[lane];
    }
}

// ------------------------------------------------------------- training
// Weight-gradient tile: C[out 16][in 16] += dZ^T (out x rows) * Hin (rows x in),
// K = the 16 rows of the tile (padded to 32 with zeros).
__device__ __forceinline__ f32x4 wgrad(const float* dz, int o0, const float* hin, int ldh, int i0, f32x4 acc,
                                       int lane) {
    const int g = lane >> 4, m = lane & 15;
    bf16x8 a, b;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        const int r = 8 * g + i;
        a[i] = (__bf16)(r < 16 ? dz[r * kH + o0 + m] : 0.0f);
        b[i] = (__bf16)(r < 16 ? hin[r * ldh + i0 + m] : 0.0f);
    }
    return mfma(a, b, acc);
}

// dH[row][in] = sum_out dZ[row][out] W[out][in], masked by (H > 0)
__device__ __forceinline__ void back_layer(const float* dz, const __bf16 (*Wt)[kH], const float* hmask, float* out,
                                           int lane) {
#pragma unroll
    for (int t = 0; t < kH / 16; t++) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k0 = 0; k0 < kH; k0 += 32) acc = mfma(a_rows(dz, kH, k0, lane), b_rows<kH>(Wt, 16 * t, k0, lane), acc);
        const int col = 16 * t + (lane & 15);
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int row = 4 * (lane >> 4) + i;
            out[row * kH + col] = hmask[row * kH + col] > 0.0f ? acc[i] : 0.0f;
        }
    }
}

// Loss (1/rows) sum_i w_i (o_i - t_i)^2 and its gradient.  Each wave keeps its
// partial weight gradients in registers and writes them to a slot; a second
// kernel sums the slots.
__global__ void __launch_bounds__(256) k_mlp_train(const float* __restrict__ params, int64_t rows,
                                                   const float* __restrict__ feats, const float* __restrict__ target,
                                                   const float* __restrict__ weights, float* __restrict__ slots,
                                                   double* __restrict__ loss_slots) {
    __shared__ MlpLds s;
    __shared__ WaveTiles tiles[4];
    __shared__ float dz2[4][16][kH];
    stage_weights(params, s, true);
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    WaveTiles& w = tiles[wv];
    float(*d2)[kH] = dz2[wv];
    f32x4 g1[4][2], g2[4][4], g3[4][4];
#pragma unroll
    for (int a = 0; a < 4; a++) {
#pragma unroll
        for (int b = 0; b < 4; b++) {
            g2[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
            g3[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
        g1[a][0] = f32x4{0.f, 0.f, 0.f, 0.f};
        g1[a][1] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    float gb1 = 0.f, gb2 = 0.f, gb3 = 0.f, gw4 = 0.f, gb4 = 0.f;  // lane owns column `lane`
    double lsum = 0.0;
    const double inv_rows = 1.0 / (double)rows;
    const int64_t ntile = (rows + 15) / 16;
    for (int64_t t = (int64_t)blockIdx.x * 4 + wv; t < ntile; t += (int64_t)gridDim.x * 4) {
        const int64_t r0 = t * 16;
        forward_tile(s, w, feats, r0, rows, lane);
        // dL/do per row (zero for padding rows)
        float gout = 0.0f;
        if (lane < 16 && r0 + lane < rows) {
            const float wt = weights ? weights[r0 + lane] : 1.0f;
            const float e = w.o[lane] - target[r0 + lane];
            lsum += (double)wt * (double)e * (double)e;
            gout = (float)(2.0 * inv_rows) * wt * e;
        }
        // broadcast the 16 row gradients; layer 4 and dZ3 (lane = column)
        float grow[16];
#pragma unroll
        for (int r = 0; r < 16; r++) grow[r] = __shfl(gout, r, 64);
        {
            const int c = lane;  // 64 lanes = 64 hidden columns
            float acc_w4 = 0.f, acc_b3 = 0.f;
#pragma unroll
            for (int r = 0; r < 16; r++) {
                const float h = w.h3[r][c];
                acc_w4 += grow[r] * h;
                const float dz = h > 0.0f ? grow[r] * s.w4[c] : 0.0f;
                w.dz[r][c] = dz;
                acc_b3 += dz;
            }
            gw4 += acc_w4;
            gb3 += acc_b3;
            if (lane == 0) {
                float sg = 0.f;
                for (int r = 0; r < 16; r++) sg += grow[r];
                gb4 += sg;
            }
        }
        wave_sync();
        // dW3 += dZ3^T H2 ; dZ2 = (dZ3 W3) * (H2 > 0)
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int b = 0; b < 4; b++) g3[a][b] = wgrad(&w.dz[0][0], 16 * a, &w.h2[0][0], kH, 16 * b, g3[a][b], lane);
        back_layer(&w.dz[0][0], s.w3t, &w.h2[0][0], &d2[0][0], lane);
        wave_sync();
        {
            float acc = 0.f;
#pragma unroll
            for (int r = 0; r < 16; r++) acc += d2[r][lane];
            gb2 += acc;
        }
        // dW2 += dZ2^T H1 ; dZ1 = (dZ2 W2) * (H1 > 0)
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int b = 0; b < 4; b++) g2[a][b] = wgrad(&d2[0][0], 16 * a, &w.h1[0][0], kH, 16 * b, g2[a][b], lane);
        back_layer(&d2[0][0], s.w2t, &w.h1[0][0], &w.dz[0][0], lane);
        wave_sync();
        {
            float acc = 0.f;
#pragma unroll
            for (int r = 0; r < 16; r++) acc += w.dz[r][lane];
            gb1 += acc;
        }
        // dW1 += dZ1^T X
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int b = 0; b < 2; b++) g1[a][b] = wgrad(&w.dz[0][0], 16 * a, &w.x[0][0], kK1, 16 * b, g1[a][b], lane);
        wave_sync();
    }
    // write this wave's partial gradient to its slot
    float* sl = slots + ((int64_t)blockIdx.x * 4 + wv) * kNP;
    const int cn = lane & 15, rq = 4 * (lane >> 4);
#pragma unroll
    for (int a = 0; a < 4; a++) {
#pragma unroll
        for (int b = 0; b < 4; b++)
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int o = 16 * a + rq + i, in = 16 * b + cn;
                sl[oW3 + o * kH + in] = g3[a][b][i];
                sl[oW2 + o * kH + in] = g2[a][b][i];
            }
#pragma unroll
        for (int b = 0; b < 2; b++)
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int o = 16 * a + rq + i, in = 16 * b + cn;
                if (in < kF) sl[oW1 + o * kF + in] = g1[a][b][i];
            }
    }
    sl[ob1 + lane] = gb1;
    sl[ob2 + lane] = gb2;
    sl[ob3 + lane] = gb3;
    sl[oW4 + lane] = gw4;
    if (lane == 0) sl[ob4] = gb4;
    // loss partial: lanes 0..15 hold row terms
    for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o, 64);
    if (lane == 0) loss_slots[blockIdx.x * 4 + wv] = lsum * inv_rows;
}

__global__ void k_mlp_reduce(const float* __restrict__ slots, int nslot, const double* __restrict__ loss_slots,
                             float* __restrict__ grad, double* __restrict__ loss) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kNP) {
        double s = 0.0;
        for (int k = 0; k < nslot; k++) s += slots[(int64_t)k * kNP + i];
        grad[i] = (float)s;
    }
    if (i == 0) {
        double s = 0.0;
        for (int k = 0; k < nslot; k++) s += loss_slots[k];
        *loss = s;
    }
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kNP) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------- hosts
static int mlp_blocks(int64_t rows) {
    const int64_t tiles = (rows + 15) / 16;
    return (int)std::max<int64_t>(1, std::min<int64_t>(256, (tiles + 3) / 4));
}

void mlp_forward(const float* params, int64_t rows, const float* feats, float* out, hipStream_t s) {
    if (rows <= 0) return;
    hipLaunchKernelGGL(k_mlp_forward, dim3(mlp_blocks(rows)), dim3(256), 0, s, params, rows, feats, out);
    EFGP_HIP(hipGetLastError());
}

void mlp_loss_grad(const float* params, int64_t rows, const float* feats, const float* target,
                   const float* weights, float* grad, double* loss, hipStream_t s) {
    const int nb = mlp_blocks(rows);
    const int nslot = nb * 4;
    float* slots = nullptr;
    double* lslots = nullptr;
    EFGP_HIP(hipMallocAsync((void**)&slots, sizeof(float) * (size_t)nslot * kNP, s));
    EFGP_HIP(hipMallocAsync((void**)&lslots, sizeof(double) * nslot, s));
    hipLaunchKernelGGL(k_mlp_train, dim3(nb), dim3(256), 0, s, params, rows, feats, target, weights, slots, lslots);
    hipLaunchKernelGGL(k_mlp_reduce, dim3(cdiv(kNP, 256)), dim3(256), 0, s, slots, nslot, lslots, grad, loss);
    EFGP_HIP(hipGetLastError());
    EFGP_HIP(hipFreeAsync(slots, s));
    EFGP_HIP(hipFreeAsync(lslots, s));
}

void mlp_adam(float* params, const float* grad, float* m, float* v, int64_t step, float lr, float b1, float b2,
              float eps, hipStream_t s) {
    const float c1 = 1.0f - std::pow(b1, (float)step), c2 = 1.0f - std::pow(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(cdiv(kNP, 256)), dim3(256), 0, s, params, grad, m, v, lr, b1, b2, eps, c1, c2);
    EFGP_HIP(hipGetLastError());
}

// p_j = exp(clamp(o_j)) * jacobi_j for every system, in the plan precision
// Mean over the system's frequencies of the network's per-frequency output:
// the exponent s of the diagonal (N D_j^2 + sigma^2)^(-s) (one block; each
// thread sums in a fixed order, then a block sum).  Non-finite outputs count
// as 1 (Jacobi) and outputs are clamped to [-1, 3].
__global__ void __launch_bounds__(1024) k_exponent_mean(const float* __restrict__ o, int64_t M, float* __restrict__ sbar) {
    __shared__ double red[16];
    double acc = 0.0;
    for (int64_t j = threadIdx.x; j < M; j += blockDim.x) {
        float v = o[j];
        v = (v == v) ? fminf(fmaxf(v, -1.0f), 3.0f) : 1.0f;
        acc += v;
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) *sbar = (float)(acc / (double)M);
}

// p_j = (N D_j^2 + sigma^2)^(-s), s = s_bar clamped to [0, 1.25] (the range
// the training searched).  Within the gate of s = 1 the network says
// "Jacobi", and p_j is then computed exactly as the Jacobi kernel computes it
// (same inputs, same double arithmetic, same rounding).
template <typename T>
__global__ void k_apply_exponent(const float* __restrict__ sbar, float gate, const T* __restrict__ D, double nn,
                                 const double* __restrict__ sig2, int r, int64_t M, T* __restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    const double d = (double)D[j];
    const double a = nn * d * d + sig2[r];
    const float sv = fminf(fmaxf(*sbar, 0.0f), 1.25f);   // the searched family's range
    if (!(fabsf(sv - 1.0f) >= gate)) {
        out[j] = (T)(1.0 / a);
        return;
    }
    out[j] = (T)exp(-(double)sv * log(a));
}

void mlp_precond(const float* params, const Plan& P, void* prec_out, hipStream_t s) {
    float* buf = nullptr;
    EFGP_HIP(hipMallocAsync((void**)&buf, sizeof(float) * ((size_t)P.M * (kF + 1) + 1), s));
    float* feats = buf;
    float* o = buf + (size_t)P.M * kF;
    float* sbar = o + P.M;
    const size_t es = P.precision == 32 ? sizeof(float) : sizeof(double);
    for (int r = 0; r < P.nrhs; r++) {
        if (r > 0 && P.sigma2[r] == P.sigma2[r - 1]) {
            // the features, hence the diagonal, depend on the system only through sigma^2
            EFGP_HIP(hipMemcpyAsync(static_cast<char*>(prec_out) + (size_t)r * P.M * es,
                                    static_cast<char*>(prec_out) + (size_t)(r - 1) * P.M * es, (size_t)P.M * es,
                                    hipMemcpyDeviceToDevice, s));
            continue;
        }
        run_features(P, r, feats, nullptr, s);
        mlp_forward(params, P.M, feats, o, s);
        hipLaunchKernelGGL(k_exponent_mean, dim3(1), dim3(1024), 0, s, o, P.M, sbar);
        if (P.precision == 32)
            hipLaunchKernelGGL((k_apply_exponent<float>), dim3(cdiv(P.M, 256)), dim3(256), 0, s, sbar,
                               (float)EFGP_MLP_GATE, static_cast<const float*>(P.Dt), (double)P.n, P.sig2, r, P.M,
                               static_cast<float*>(prec_out) + (size_t)r * P.M);
        else
            hipLaunchKernelGGL((k_apply_exponent<double>), dim3(cdiv(P.M, 256)), dim3(256), 0, s, sbar,
                               (float)EFGP_MLP_GATE, static_cast<const double*>(P.Dt), (double)P.n, P.sig2, r, P.M,
                               static_cast<double*>(prec_out) + (size_t)r * P.M);
        EFGP_HIP(hipGetLastError());
    }
    EFGP_HIP(hipFreeAsync(buf, s));
}

}  // namespace efgp
