// Posterior variance at targets (Remark r:var: one linear solve per target),
// in weight space.  With Phi the N x M design matrix (Phi_nj =
// D_j exp(-2 pi i h <j, x_n>), so that the mean is Phi beta, eq. (bmu)) and
// phi(t) = (D_j exp(+2 pi i h <j, t>))_j the column of Phi^H for a target t,
// the posterior variance of the GP with kernel k~ is
//     s(t) = sigma^2 phi(t)^H (Phi^H Phi + sigma^2 I)^{-1} phi(t),
// the weight-space form (Woodbury) of k~(t,t) - k~_t^T (K~ + sigma^2 I)^{-1} k~_t
// (eqs. (mu)-(362) with k~).  Phi^H Phi + sigma^2 I is the system matrix of
// step 4, so each target costs one solve with the plan's fast Toeplitz
// product: targets go in batches of up to 64 systems through the batched CG
// solver, on a view of the plan that shares v-hat, D and the twiddles.
#include <algorithm>
#include <cmath>

#include "fft_device.h"

namespace efgp {

// phi(t) for targets q0 .. q0+nb-1: b[r][j] = D_j exp(+2 pi i h <j, t_r>),
// phases reduced in double.  Flags a target outside [0,1]^d.
template <typename T, int DIM>
__global__ void k_var_rhs(const T* __restrict__ t, int64_t q, int64_t q0, int nb, const double* __restrict__ D,
                          int m, double h, int64_t M, cpx<T>* __restrict__ b, double2* __restrict__ b64,
                          int* __restrict__ flag) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= M * nb) return;
    const int r = (int)(idx / M);
    const int64_t j = idx - (int64_t)r * M;
    const int W = 2 * m + 1;
    int64_t rem = j;
    int js[3] = {0, 0, 0};
    for (int l = DIM - 1; l >= 0; l--) { js[l] = (int)(rem % W) - m; rem /= W; }
    double ph = 0.0;
    bool ok = true;
    for (int l = 0; l < DIM; l++) {
        const double a = (double)t[(int64_t)l * q + q0 + r];
        ok = ok && a >= 0.0 && a <= 1.0;
        ph += h * (double)js[l] * a;
    }
    if (!ok && j == 0) atomicOr(flag, 1);
    ph -= floor(ph);  // exp(2 pi i ph) is 1-periodic in ph
    double sn, cs;
    sincos(6.283185307179586 * ph, &sn, &cs);
    b[idx] = cpx<T>{(T)(D[j] * cs), (T)(D[j] * sn)};
    if (b64) b64[idx] = make_double2(D[j] * cs, D[j] * sn);   // (refined solves)
}

// s_r = sigma^2 Re(phi_r^H u_r), one block per target
template <typename T>
__global__ void __launch_bounds__(256) k_var_dot(const cpx<T>* __restrict__ b, const cpx<T>* __restrict__ u,
                                                 int64_t M, double s2, T* __restrict__ out) {
    __shared__ double red[16];
    const int r = blockIdx.x;
    double acc = 0.0;
    for (int64_t j = threadIdx.x; j < M; j += blockDim.x) {
        const cpx<T> bb = b[(int64_t)r * M + j], uu = u[(int64_t)r * M + j];
        acc += (double)bb.x * (double)uu.x + (double)bb.y * (double)uu.y;
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) out[r] = (T)(s2 * acc);
}

template <typename T>
static int variance_typed(Plan& P, int sys, int64_t q, const void* targets, void* var_out,
                          const efgp_solve_opts& o, efgp_solve_stats* stats) {
    hipStream_t s = P.work;
    const double s2 = P.sigma2[sys];
    const int64_t M = P.M;
    int64_t worst_it = 0;
    double worst_res = 0.0, ms = 0.0;
    int conv = 0, fell = 0, status = EFGP_OK;
    EFGP_HIP(hipMemsetAsync(P.flag, 0, sizeof(int), s));
    // refined solves (precision 32) share the plan's double FFT(v)
    const bool refine = P.precision == 32 && o.refine > 0;
    if (refine && !P.vhat64) build_vhat64(P, s);
    for (int64_t q0 = 0; q0 < q; q0 += 64) {
        const int nb = (int)std::min<int64_t>(64, q - q0);
        // a view of the plan with nb systems of noise sigma_sys^2 and its own
        // right-hand sides and solver workspace
        Plan V = P;
        V.allocs.clear();
        V.pinned.clear();
        V.graph = nullptr;
        V.graph_id.clear();
        V.x = V.r = V.p = V.q = V.prec = nullptr;
        V.clam = V.cbuf = V.zbuf = nullptr;
        V.cslot = nullptr;
        V.buf1 = V.buf2 = nullptr;
        V.part = nullptr;
        V.st = nullptr;
        V.h_st = nullptr;
        V.hist = nullptr;
        V.h_hist.clear();
        V.x64 = V.r64 = V.ax64 = V.buf64a = V.buf64b = nullptr;
        V.b64 = nullptr;
        V.nrhs = nb;
        V.sigma2.assign(nb, s2);
        int rc = EFGP_OK;
        efgp_solve_stats st{};
        try {
            V.sig2 = static_cast<double*>(dalloc(V, sizeof(double) * nb));
            upload_async(V, V.sig2, V.sigma2.data(), sizeof(double) * nb, s);
            cpx<T>* b = static_cast<cpx<T>*>(dalloc(V, sizeof(cpx<T>) * M * nb));
            cpx<T>* u = static_cast<cpx<T>*>(dalloc(V, sizeof(cpx<T>) * M * nb));
            V.b = b;
            double2* b64 = nullptr;
            if (refine) {
                b64 = static_cast<double2*>(dalloc(V, sizeof(double2) * M * nb));
                V.b64 = reinterpret_cast<double*>(b64);
            }
            const int d = P.dim;
            const unsigned g = cdiv(M * nb, 256);
            const T* tt = static_cast<const T*>(targets);
            if (d == 1) hipLaunchKernelGGL((k_var_rhs<T, 1>), dim3(g), dim3(256), 0, s, tt, q, q0, nb, P.D64, P.m, P.h, M, b, b64, P.flag);
            else if (d == 2) hipLaunchKernelGGL((k_var_rhs<T, 2>), dim3(g), dim3(256), 0, s, tt, q, q0, nb, P.D64, P.m, P.h, M, b, b64, P.flag);
            else hipLaunchKernelGGL((k_var_rhs<T, 3>), dim3(g), dim3(256), 0, s, tt, q, q0, nb, P.D64, P.m, P.h, M, b, b64, P.flag);
            EFGP_HIP(hipGetLastError());
            rc = run_solve(V, o, u, &st);
            hipLaunchKernelGGL((k_var_dot<T>), dim3(nb), dim3(256), 0, s, b, u, M, s2,
                               static_cast<T*>(var_out) + q0);
            EFGP_HIP(hipGetLastError());
            EFGP_HIP(hipStreamSynchronize(s));
        } catch (...) {
            (void)hipStreamSynchronize(s);
            if (V.graph) graph_release(V.device, V.graph_id);
            for (auto& a : V.allocs) pool_free(V.device, a.first, a.second);
            for (auto& a : V.pinned) pinned_free(a.first, a.second);
            throw;
        }
        if (V.graph) graph_release(V.device, V.graph_id);
        for (auto& a : V.allocs) pool_free(V.device, a.first, a.second);
        for (auto& a : V.pinned) pinned_free(a.first, a.second);
        worst_it = std::max<int64_t>(worst_it, st.iterations);
        worst_res = std::max(worst_res, st.rel_residual);
        conv += st.converged;
        fell += st.fell_back;
        ms += st.ms_solve;
        if (rc < 0) return rc;
        if (rc == EFGP_NOT_CONVERGED) status = EFGP_NOT_CONVERGED;
        else if (rc == EFGP_FELL_BACK && status == EFGP_OK) status = EFGP_FELL_BACK;
    }
    int hf = 0;
    EFGP_HIP(hipMemcpyAsync(&hf, P.flag, sizeof(int), hipMemcpyDeviceToHost, s));
    EFGP_HIP(hipStreamSynchronize(s));
    if (stats) {
        *stats = efgp_solve_stats{};
        stats->iterations = worst_it;
        stats->converged = conv;
        stats->fell_back = fell;
        stats->rel_residual = worst_res;
        stats->ms_solve = ms;
    }
    if (hf & 1) {
        EFGP_HIP(hipMemsetAsync(P.flag, 0, sizeof(int), s));
        return EFGP_EDOMAIN;
    }
    return status;
}

int run_variance(Plan& P, int sys, int64_t q, const void* targets, void* var_out, const efgp_solve_opts& o,
                 efgp_solve_stats* stats) {
    if (P.precision == 32) return variance_typed<float>(P, sys, q, targets, var_out, o, stats);
    return variance_typed<double>(P, sys, q, targets, var_out, o, stats);
}

}  // namespace efgp
