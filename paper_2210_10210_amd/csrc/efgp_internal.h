// Internal declarations of the EFGP gfx950 library: plan layout, device
// helper types and the launchers each translation unit exports.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "efgp.h"

namespace efgp {

// ------------------------------------------------------------------ errors
struct HipError {
    hipError_t err;
    const char* what;
};
#define EFGP_HIP(call)                                                   \
    do {                                                                 \
        hipError_t e_ = (call);                                          \
        if (e_ != hipSuccess) throw ::efgp::HipError{e_, #call};         \
    } while (0)

struct StatusError {
    int status;
    std::string msg;
};

// ------------------------------------------------------------ complex types
template <typename T> struct cx;
template <> struct cx<float> { using t = float2; };
template <> struct cx<double> { using t = double2; };
template <typename T> using cpx = typename cx<T>::t;

// ------------------------------------------------------------- FFT tables
constexpr int kMaxStages = 24;
constexpr int kMaxFft = 8192;  // largest supported line length (spreading grid)
constexpr int kMaxEmbed = 4096; // largest Toeplitz embedding L per dimension

struct FftShape {
    int n = 0;
    int nst = 0;
    int radix[kMaxStages] = {0};
    unsigned code = 0;        // radix of stage s in bits 4s..4s+3 (device side:
                              // no dynamically indexed array, hence no scratch)
};
// factorisation into stages of radix 16, 15, 12, 10, 9, 8, 6, 5, 4, 3 or 2
// (largest first), none above maxr (kernels that cannot hold the larger
// butterflies in registers take maxr = 5)
FftShape fft_shape(int n, int maxr = 16);
int max_radix(const FftShape& s);
bool is_smooth235(int n);
int next_smooth235(int n);

template <typename T>
struct FftDev {               // passed by value to kernels
    FftShape s;
    const cpx<T>* tw;         // tw[k] = exp(-2 pi i k / n), k < n
};

// ---------------------------------------------------------- CG state
struct CgState {
    double rz;       // current r^H z (z = P r, or r)
    double rz_acc;   // accumulator for the next r^H z
    double pq_acc;   // accumulator for p^H A p
    double rr_acc;   // accumulator for ||r||^2
    double bb;       // ||b||^2
    double rho2;     // rel_tol^2
    double gamma;    // rz_new / rz (direction update factor)
    double relres;   // latest recursive ||r|| / ||b||
    double best;     // best relres seen since the last stall check
    int active;      // still iterating
    int use_prec;    // apply the diagonal preconditioner
    int iters;       // iterations done
    int pad;
};

// ------------------------------------------------------------------ plan
struct Plan {
    // problem
    int dim = 0, kernel = 0, precision = 64, nrhs = 1;
    bool prior = false;         // kernel-only plan (prior sampling): no points
    double ell = 0, nu = 0, variance = 1, eps = 0, tol = 0;
    int64_t n = 0;
    std::vector<double> sigma2;

    // parameters
    double h = 0, kl2 = 0;
    int m = 0, W = 0, W2 = 0, L = 0, nf = 0, nf2 = 0, w = 0;
    int64_t M = 0, LD = 0;     // M = W^d, LD = L^d
    double es_beta = 0;
    int spread_method = 0, tile = 0;
    int spread_epoch = 0;        // fixed-point accumulation epoch (points per workgroup); 0: per spreader
    int setup_passes = 0;       // passes the last setup took (1..3, see setup_typed)

    // device data (double unless noted)
    double* D64 = nullptr;      // M
    void* Dt = nullptr;         // M, precision T
    double* v = nullptr;        // W2^d complex
    double* b64 = nullptr;      // nrhs*M complex
    void* b = nullptr;          // nrhs*M complex, T
    void* vhat = nullptr;       // L^d complex, T, scaled by 1/L^d
    void* psi2 = nullptr;       // W entries: 1/psihat_eval(j) per j in -m..m, T
    double* sig2 = nullptr;     // nrhs
    void* twL = nullptr;        // L twiddles, T
    void* twE = nullptr;        // nf2 twiddles, T
    // double operator for the iterative refinement of precision-32 solves
    // (built on first use): FFT(v)/L^d, L twiddles, x, r, A x and two line buffers
    void* vhat64 = nullptr;
    void* twL64 = nullptr;
    void *x64 = nullptr, *r64 = nullptr, *ax64 = nullptr, *buf64a = nullptr, *buf64b = nullptr;

    // solver workspace (T)
    void *x = nullptr, *r = nullptr, *p = nullptr, *q = nullptr, *prec = nullptr;
    void* buf1 = nullptr;       // FFT intermediates
    void* buf2 = nullptr;
    double* part = nullptr;     // partial-sum slots of the CG reductions
    CgState* st = nullptr;      // nrhs states
    CgState* h_st = nullptr;    // pinned host mirror
    double* hist = nullptr;     // device residual history of system 0
    int64_t hist_cap = 0;
    std::vector<double> h_hist;

    // circulant preconditioner (T): period K per dimension, 1/(K^d lambda_s)
    // per system, the K^d FFT workspace, z = P r, reduction slots
    int K = 0;
    void* twK = nullptr;        // K twiddles, T
    void* clam = nullptr;       // nrhs*K^d reals
    void* cbuf = nullptr;       // nrhs*K^d complex
    void* zbuf = nullptr;       // nrhs*M complex
    double* cslot = nullptr;    // nrhs*64 partial sums

    // eval workspace
    void* g2 = nullptr;         // nrhs * nf2^d complex, T
    int* flag = nullptr;        // device domain flag (eval)
    int* chk = nullptr;         // device flag of the solve's argument checks

    // execution
    hipStream_t work = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraphExec_t graph = nullptr;   // cached graph (owned by the cache)

    // timings of the last setup (ms)
    double ms_sort = 0, ms_spread = 0, ms_fft = 0, ms_deconv = 0, ms_total = 0;

    int device = 0;             // device the plan lives on
    std::vector<std::pair<void*, size_t>> allocs;   // device buffers (pooled)
    std::vector<std::pair<void*, size_t>> pinned;   // pinned host buffers (pooled)
    std::string graph_id;       // key of the cached CG graph held by this plan
};

// host-side parameter computations (plan.cpp)
double kernel_hat(const Plan& P, double xi);
std::vector<double> spectral_weights(const Plan& P);   // D_j over J_m
double kernel_l2_norm(int kernel, double ell, double nu, int dim);
void choose_h_m(int kernel, int dim, double eps, double ell, double nu, double* h, int* m,
                double* kl2);
void es_params(double tol, int* w, double* beta);
// 1/psihat(k) of the ES kernel for grid size nfine at integer k = -K..K.
std::vector<double> es_deconv_table(int w, double beta, int nfine, int K);

// device memory helpers
void* dalloc(Plan& P, size_t bytes);
// pinned host staging owned by the plan (released when the plan is)
void* palloc(Plan& P, size_t bytes);
// asynchronous upload of host bytes through pinned staging owned by the plan
void upload_async(Plan& P, void* dst, const void* src, size_t bytes, hipStream_t s);

// process-wide caches (runtime.cpp)
int current_device();
void* pool_alloc(size_t bytes);
void pool_free(int dev, void* p, size_t bytes);
void* pinned_alloc(size_t bytes);
void pinned_free(void* p, size_t bytes);
hipStream_t acquire_stream();
void release_stream(int dev, hipStream_t s);
hipEvent_t acquire_event(bool timing);
void release_event(int dev, hipEvent_t e, bool timing);
hipGraphExec_t graph_acquire(int dev, const std::string& key);   // takes a reference
void graph_insert(int dev, const std::string& key, hipGraphExec_t exec);  // takes a reference
void graph_release(int dev, const std::string& key);
void release_pools();

// Spread tuning table (runtime.cpp): the measured fastest spreader for a
// problem shape; efgp_setup with spread_method AUTO and tile 0 consults it.
struct TuneKey {
    int dev, dim, precision, nrhs, nf, w, nbucket;   // nbucket = floor(log2 N)
    bool operator<(const TuneKey& o) const;
};
struct TuneChoice {
    int method, tile;
    double ms;
};
int n_bucket(int64_t n);
bool tune_lookup(const TuneKey& k, TuneChoice* c);
void tune_insert(const TuneKey& k, const TuneChoice& c);
void tune_clear();
bool tune_save(const char* path);
int tune_load(const char* path);

// Setup scratch: device chunks kept across setups (allocating and freeing
// multi-GB sort buffers on every setup costs far more than the kernels).
// A setup holds the lock for its whole duration; take() bump-allocates and
// the destructor makes every chunk reusable again.
class Scratch {
  public:
    Scratch();
    ~Scratch();
    void* take(size_t bytes);
  private:
    int dev_;
};
void release_scratch();
template <typename T> void upload_twiddles(Plan& P, int n, void** out, hipStream_t s);
// stream-ordered upload of the twiddle table of size n into device memory dst
template <typename T> void upload_twiddles_to(Plan& P, int n, void* dst, hipStream_t s);

// --------------------------------------------------------------- launchers
// setup (setup.hip)
void run_setup(Plan& P, const efgp_problem& pr, hipStream_t s);
void build_vhat64(Plan& P, hipStream_t s);   // P.vhat64 (and P.twL64) from P.v
// solver (solve.hip)
void mv_apply(Plan& P, const void* in, void* out, hipStream_t s);
// allocation-free product: FFT intermediates in a static device array of
// kNoAllocBytes per GPU, whose address noalloc_init(dev) looks up once per
// device (called by every plan build, with that device current)
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
void noalloc_init(int dev);
size_t noalloc_bytes(const Plan& P);
void mv_apply_noalloc(Plan& P, const void* in, void* out, hipStream_t s);
int run_solve(Plan& P, const efgp_solve_opts& o, void* beta_out, efgp_solve_stats* st);
// posterior variance (variance.hip)
int run_variance(Plan& P, int sys, int64_t q, const void* targets, void* var_out, const efgp_solve_opts& o,
                 efgp_solve_stats* stats);
void alloc_solver(Plan& P);
// eval (eval.hip)
void run_eval(Plan& P, const void* beta, int64_t q, const void* t, void* mu, hipStream_t s);
// features (solve.hip)
void run_features(const Plan& P, int r, float* feats, float* jac, hipStream_t s);
// circulant preconditioner (circulant.hip): circ_setup fills P.prec with
// 1/sqrt(N D_j^2 + sigma_r^2) and P.clam; circ_apply computes z = P r into
// P.zbuf and r^H z into the CG state (fresh: only systems with gamma = 0,
// i.e. just initialised or restarted); circ_eigs writes lambda of system r.
template <typename T> void circ_setup(Plan& P, hipStream_t s);
template <typename T> void circ_apply(const Plan& P, bool fresh, hipStream_t s);
template <typename T> void circ_eigs(Plan& P, int r, void* out, hipStream_t s);
// generic FFT along one axis of [outer][n][inner] complex arrays (fft.hip)
template <typename T>
void fft_axis(cpx<T>* data, const FftDev<T>& f, int64_t outer, int64_t inner, int sign,
              hipStream_t s);
// MLP (mlp.hip)
void mlp_forward(const float* params, int64_t rows, const float* feats, float* out, hipStream_t s);
void mlp_loss_grad(const float* params, int64_t rows, const float* feats, const float* target,
                   const float* weights, float* grad, double* loss, hipStream_t s);
void mlp_adam(float* params, const float* grad, float* m, float* v, int64_t step, float lr,
              float b1, float b2, float eps, hipStream_t s);
void mlp_precond(const float* params, const Plan& P, void* prec_out, hipStream_t s);
template <typename T> void float_to_T(const float* in, int64_t n, void* out, hipStream_t s);

inline int64_t ipow(int64_t b, int e) {
    int64_t r = 1;
    while (e-- > 0) r *= b;
    return r;
}
inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace efgp
