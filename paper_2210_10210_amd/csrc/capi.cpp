// C ABI of the EFGP library (declared in include/efgp.h).  Validates
// arguments before any allocation or launch, builds the plan, and orders
// the plan's private stream after the caller's stream with events so that
// every call is stream-ordered for the caller.  No exception crosses the ABI.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "efgp_internal.h"

using namespace efgp;

struct efgp_plan {
    Plan P;
};

namespace {

int guard_status(const StatusError& e) { return e.status; }

template <typename F>
int guarded(F&& f) {
    try {
        return f();
    } catch (const StatusError& e) {
        return guard_status(e);
    } catch (const HipError&) {
        (void)hipGetLastError();
        return EFGP_EHIP;
    } catch (const std::bad_alloc&) {
        return EFGP_ENOMEM;
    } catch (...) {
        return EFGP_EHIP;
    }
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// make `work` wait for what the caller has queued on `caller`
void join_in(Plan& P, void* caller) {
    EFGP_HIP(hipEventRecord(P.ev_in, static_cast<hipStream_t>(caller)));
    EFGP_HIP(hipStreamWaitEvent(P.work, P.ev_in, 0));
}
// make the caller's stream wait for the work queued on `work`
void join_out(Plan& P, void* caller) {
    EFGP_HIP(hipEventRecord(P.ev_out, P.work));
    EFGP_HIP(hipStreamWaitEvent(static_cast<hipStream_t>(caller), P.ev_out, 0));
}

// Return everything the plan holds to the process-wide caches once its
// stream has drained (buffers, pinned staging, stream, events, graph).
void free_plan(Plan& P) {
    if (P.work) (void)hipStreamSynchronize(P.work);
    if (P.graph) graph_release(P.device, P.graph_id);
    P.graph = nullptr;
    for (auto& a : P.allocs) pool_free(P.device, a.first, a.second);
    P.allocs.clear();
    for (auto& a : P.pinned) pinned_free(a.first, a.second);
    P.pinned.clear();
    P.h_st = nullptr;
    release_event(P.device, P.ev_in, false);
    release_event(P.device, P.ev_out, false);
    release_stream(P.device, P.work);
    P.ev_in = P.ev_out = nullptr;
    P.work = nullptr;
}

template <typename T>
void upload_T(Plan& P, const std::vector<double>& h, void** out) {
    std::vector<T> t(h.size());
    for (size_t i = 0; i < h.size(); i++) t[i] = (T)h[i];
    *out = dalloc(P, sizeof(T) * t.size());
    upload_async(P, *out, t.data(), sizeof(T) * t.size(), P.work);
}

}  // namespace

extern "C" {

const char* efgp_strerror(int s) {
    switch (s) {
        case EFGP_OK: return "ok";
        case EFGP_NOT_CONVERGED: return "not converged within max_iter (last iterate returned)";
        case EFGP_FELL_BACK: return "preconditioned CG stalled; plain CG finished the solve";
        case EFGP_EINVAL: return "invalid argument";
        case EFGP_EDOMAIN: return "a point or target lies outside [0,1]^d";
        case EFGP_ETOOLARGE: return "problem exceeds the library size limits";
        case EFGP_ENOMEM: return "device allocation failed";
        case EFGP_EHIP: return "HIP runtime error";
        case EFGP_EMODEL: return "preconditioner network weights unusable";
        default: return "unknown status";
    }
}

// Build a plan.  prior: kernel-only plan (GP prior sampling): no points or
// data, v = b = 0, nrhs = samples per call.
static int build_plan(const efgp_problem* p, efgp_plan** out, bool prior) {
    if (!out) return EFGP_EINVAL;
    *out = nullptr;
    if (!p) return EFGP_EINVAL;
    // ---- argument validation (no allocation yet)
    if (p->dim < 1 || p->dim > 3) return EFGP_EINVAL;
    if (p->kernel != EFGP_KERNEL_SE && p->kernel != EFGP_KERNEL_MATERN) return EFGP_EINVAL;
    if (!finite_pos(p->lengthscale)) return EFGP_EINVAL;
    if (p->kernel == EFGP_KERNEL_MATERN && !(std::isfinite(p->nu) && p->nu >= 0.5)) return EFGP_EINVAL;
    if (!(std::isfinite(p->eps) && p->eps > 0.0 && p->eps < 1.0)) return EFGP_EINVAL;
    if (p->precision != 32 && p->precision != 64) return EFGP_EINVAL;
    if (p->nrhs < 1 || p->nrhs > 64) return EFGP_EINVAL;
    if (!prior) {
        if (p->n < 1) return EFGP_EINVAL;
        if (!p->x || !p->y || !p->sigma2) return EFGP_EINVAL;
        for (int r = 0; r < p->nrhs; r++)
            if (!finite_pos(p->sigma2[r])) return EFGP_EINVAL;
        if (p->n > (int64_t)2000000000) return EFGP_ETOOLARGE;
    }
    if (!(p->variance == 0.0 || finite_pos(p->variance))) return EFGP_EINVAL;
    if (!(p->nufft_tol == 0.0 || (std::isfinite(p->nufft_tol) && p->nufft_tol > 0.0 && p->nufft_tol < 1.0)))
        return EFGP_EINVAL;
    if (p->spread_method < 0 || p->spread_method > 3 || p->tile < 0 || p->m_override < 0) return EFGP_EINVAL;
    if (p->spread_epoch != 0 && (p->spread_epoch < (1 << 10) || p->spread_epoch > (1 << 24) ||
                                 (p->spread_epoch & (p->spread_epoch - 1)) != 0))
        return EFGP_EINVAL;

    // ---- parameters
    double h = 0, kl2 = 0;
    int m = 0;
    choose_h_m(p->kernel, p->dim, p->eps, p->lengthscale, p->nu, &h, &m, &kl2);
    if (p->m_override > 0) m = p->m_override;
    if (!(h > 0.0 && h < 1.0) || m < 1) return EFGP_EINVAL;
    // default spreading tolerance: eps/10 (Sec. 5.1); precision 64 defaults
    // to the 1e-12 parity mode, an explicit value is honoured; precision 32
    // cannot resolve below 1e-7.
    double tol = p->nufft_tol > 0 ? p->nufft_tol : (p->precision == 64 ? std::min(p->eps / 10.0, 1e-12)
                                                                         : p->eps / 10.0);
    if (p->precision == 64) tol = std::max(tol, 1e-15);
    else tol = std::max(tol, 1e-7);
    int w = 0;
    double es_beta = 0;
    es_params(tol, &w, &es_beta);
    if ((int64_t)4 * m + 1 > kMaxEmbed) return EFGP_ETOOLARGE;
    const int W = 2 * m + 1, W2 = 4 * m + 1;
    const int L = next_smooth235(W2);
    const int nf = next_smooth235(std::max(2 * W2, 2 * w + 2));
    const int nf2 = next_smooth235(std::max(2 * W, 2 * w + 2));
    if (L > kMaxEmbed || nf > kMaxFft || nf2 > kMaxFft) return EFGP_ETOOLARGE;
    const int64_t M = ipow(W, p->dim);
    const int64_t gcells = ipow(nf, p->dim);
    const double bytes = 16.0 * gcells * ((1 + p->nrhs + 1) / 2) + 16.0 * M * p->nrhs * 8;
    if (bytes > 64e9) return EFGP_ETOOLARGE;

    efgp_plan* hp = new (std::nothrow) efgp_plan;
    if (!hp) return EFGP_ENOMEM;
    Plan& P = hp->P;
    int st = guarded([&]() -> int {
        P.dim = p->dim;
        P.kernel = p->kernel;
        P.precision = p->precision;
        P.nrhs = p->nrhs;
        P.ell = p->lengthscale;
        P.nu = p->nu;
        P.variance = p->variance > 0 ? p->variance : 1.0;
        P.eps = p->eps;
        P.tol = tol;
        P.n = prior ? 0 : p->n;
        P.prior = prior;
        if (prior) P.sigma2.assign(p->nrhs, 1.0);
        else P.sigma2.assign(p->sigma2, p->sigma2 + p->nrhs);
        P.h = h;
        P.kl2 = kl2;
        P.m = m;
        P.W = W;
        P.W2 = W2;
        P.L = L;
        P.nf = nf;
        P.nf2 = nf2;
        P.w = w;
        P.es_beta = es_beta;
        P.M = M;
        P.LD = ipow(L, p->dim);
        P.spread_method = p->spread_method;
        P.tile = p->tile;
        if (p->spread_epoch > 0) P.spread_epoch = p->spread_epoch;

        P.device = current_device();
        // the static scratch of efgp_apply_noalloc: its device address, once
        // per device, while this device is current
        noalloc_init(P.device);
        // an automatic choice takes the tuned spreader of this shape, if any
        if (!prior && P.spread_method == EFGP_SPREAD_AUTO && P.tile == 0) {
            TuneChoice c{};
            if (tune_lookup(TuneKey{P.device, P.dim, P.precision, P.nrhs, nf, w, n_bucket(P.n)}, &c)) {
                P.spread_method = c.method;
                P.tile = c.tile;
            }
        }
        P.work = acquire_stream();
        P.ev_in = acquire_event(false);
        P.ev_out = acquire_event(false);
        // the caller's prior work (x, y) orders before everything below
        join_in(P, p->stream);

        // spectral weights D_j = sqrt(h^d khat(h |j|)), j in J_m (eq. (117))
        const std::vector<double> D = spectral_weights(P);
        P.D64 = static_cast<double*>(dalloc(P, sizeof(double) * M));
        upload_async(P, P.D64, D.data(), sizeof(double) * M, P.work);
        std::vector<double> dec2 = es_deconv_table(w, es_beta, nf2, m);
        P.sig2 = static_cast<double*>(dalloc(P, sizeof(double) * P.nrhs));
        upload_async(P, P.sig2, P.sigma2.data(), sizeof(double) * P.nrhs, P.work);
        P.v = static_cast<double*>(dalloc(P, 16 * (size_t)ipow(W2, P.dim)));
        P.b64 = static_cast<double*>(dalloc(P, 16 * (size_t)M * P.nrhs));
        const size_t es = P.precision == 32 ? 4 : 8;
        P.b = dalloc(P, 2 * es * (size_t)M * P.nrhs);
        P.vhat = dalloc(P, 2 * es * (size_t)P.LD);
        P.g2 = dalloc(P, 2 * es * (size_t)ipow(nf2, P.dim) * P.nrhs);
        P.flag = static_cast<int*>(dalloc(P, sizeof(int) * 4));
        EFGP_HIP(hipMemsetAsync(P.flag, 0, sizeof(int) * 4, P.work));
        if (P.precision == 32) {
            upload_T<float>(P, D, &P.Dt);
            upload_T<float>(P, dec2, &P.psi2);
            upload_twiddles<float>(P, L, &P.twL, P.work);
            upload_twiddles<float>(P, nf2, &P.twE, P.work);
        } else {
            upload_T<double>(P, D, &P.Dt);
            upload_T<double>(P, dec2, &P.psi2);
            upload_twiddles<double>(P, L, &P.twL, P.work);
            upload_twiddles<double>(P, nf2, &P.twE, P.work);
        }
        if (prior) {
            // no points: v = 0 and b = 0
            EFGP_HIP(hipMemsetAsync(P.v, 0, 16 * (size_t)ipow(W2, P.dim), P.work));
            EFGP_HIP(hipMemsetAsync(P.b64, 0, 16 * (size_t)M * P.nrhs, P.work));
            EFGP_HIP(hipMemsetAsync(P.b, 0, 2 * es * (size_t)M * P.nrhs, P.work));
            EFGP_HIP(hipStreamSynchronize(P.work));
        } else {
            run_setup(P, *p, P.work);
        }
        return EFGP_OK;
    });
    if (st != EFGP_OK) {
        free_plan(P);
        delete hp;
        return st;
    }
    *out = hp;
    return EFGP_OK;
}

int efgp_setup(const efgp_problem* p, efgp_plan** out) { return build_plan(p, out, false); }

int efgp_tune_spread(const efgp_problem* p, efgp_tune_result* out) {
    if (!p || !out) return EFGP_EINVAL;
    std::memset(out, 0, sizeof(*out));
    const int base = p->dim == 1 ? 256 : (p->dim == 2 ? 32 : 8);
    const int cands[][2] = {{EFGP_SPREAD_GRID_LDS, 0},
                            {EFGP_SPREAD_REGIONS, 0},
                            {EFGP_SPREAD_TILES, base / 2},
                            {EFGP_SPREAD_TILES, base},
                            {EFGP_SPREAD_TILES, 2 * base}};
    double best = 0.0;
    int best_method = 0, best_tile = 0, timed = 0;
    TuneKey key{};
    for (const auto& c : cands) {
        efgp_problem q = *p;
        q.spread_method = c[0];
        q.tile = c[1];
        int st = EFGP_OK;
        double ms = 0.0;
        int used_method = 0, used_tile = 0;
        // the first setup warms the caches (buffers, code objects); the
        // second is timed
        for (int rep = 0; rep < 2 && st == EFGP_OK; rep++) {
            efgp_plan* h = nullptr;
            st = build_plan(&q, &h, false);
            if (st != EFGP_OK) break;
            const Plan& P = h->P;
            ms = P.ms_total;
            used_method = P.spread_method;
            used_tile = P.spread_method == EFGP_SPREAD_GRID_LDS ? 0 : P.tile;
            key = TuneKey{P.device, P.dim, P.precision, P.nrhs, P.nf, P.w, n_bucket(P.n)};
            efgp_destroy(h);
        }
        // a candidate the shape cannot take (region or tile beyond LDS) is
        // skipped; any other failure is the problem's and is returned
        if ((st == EFGP_EINVAL && (c[0] == EFGP_SPREAD_GRID_LDS || c[0] == EFGP_SPREAD_REGIONS)) ||
            (st == EFGP_ETOOLARGE && (c[0] == EFGP_SPREAD_TILES || c[0] == EFGP_SPREAD_REGIONS)))
            continue;
        if (st != EFGP_OK) return st;
        if (timed == 0 || ms < best) {
            best = ms;
            best_method = used_method;
            best_tile = used_tile;
        }
        timed++;
    }
    if (timed == 0) return EFGP_ETOOLARGE;
    tune_insert(key, TuneChoice{best_method, best_tile, best});
    out->spread_method = best_method;
    out->tile = best_tile;
    out->ms_setup = best;
    out->candidates = timed;
    return EFGP_OK;
}

int efgp_tune_save(const char* path) {
    if (!path) return EFGP_EINVAL;
    return tune_save(path) ? EFGP_OK : EFGP_EINVAL;
}

int efgp_tune_load(const char* path, int32_t* entries) {
    if (!path) return EFGP_EINVAL;
    const int n = tune_load(path);
    if (n < 0) return EFGP_EINVAL;
    if (entries) *entries = n;
    return EFGP_OK;
}

void efgp_tune_clear(void) { tune_clear(); }

int efgp_prior_setup(const efgp_problem* p, efgp_plan** out) { return build_plan(p, out, true); }

int efgp_solve(efgp_plan* plan, const efgp_solve_opts* opts, void* beta_out, efgp_solve_stats* stats) {
    if (!plan || !beta_out || plan->P.prior) return EFGP_EINVAL;
    efgp_solve_opts o{};
    if (opts) o = *opts;
    if (o.rel_tol < 0 || !std::isfinite(o.rel_tol) || o.max_iter < 0 || o.iters_per_sync < 0 ||
        o.iters_per_sync > 4096 || o.stall_window < 0 || o.refine < 0 || o.refine > 64)
        return EFGP_EINVAL;
    if (o.precond < EFGP_PRECOND_NONE || o.precond > EFGP_PRECOND_CIRCULANT) return EFGP_EINVAL;
    if (o.precond == EFGP_PRECOND_DIAG && !o.precond_diag) return EFGP_EINVAL;
    if (o.precond == EFGP_PRECOND_LEARNED && !o.mlp_weights) return EFGP_EMODEL;
    Plan& P = plan->P;
    return guarded([&]() -> int {
        join_in(P, o.stream);
        int s = run_solve(P, o, beta_out, stats);
        join_out(P, o.stream);
        return s;
    });
}

int efgp_eval(efgp_plan* plan, const void* beta, int64_t q, const void* targets, void* mu_out, void* stream) {
    if (!plan || !beta || q < 0 || (q > 0 && (!targets || !mu_out))) return EFGP_EINVAL;
    Plan& P = plan->P;
    return guarded([&]() -> int {
        join_in(P, stream);
        run_eval(P, beta, q, targets, mu_out, P.work);
        join_out(P, stream);
        return EFGP_OK;
    });
}

int efgp_variance(efgp_plan* plan, int32_t r, int64_t q, const void* targets, void* var_out,
                  const efgp_solve_opts* opts, efgp_solve_stats* stats) {
    if (!plan || plan->P.prior || q < 0 || (q > 0 && (!targets || !var_out))) return EFGP_EINVAL;
    if (r < 0 || r >= plan->P.nrhs) return EFGP_EINVAL;
    efgp_solve_opts o{};
    if (opts) o = *opts;
    if (o.rel_tol < 0 || !std::isfinite(o.rel_tol) || o.max_iter < 0 || o.iters_per_sync < 0 ||
        o.iters_per_sync > 4096 || o.stall_window < 0 || o.beta_init || o.precond == EFGP_PRECOND_DIAG)
        return EFGP_EINVAL;
    if (o.precond < EFGP_PRECOND_NONE || o.precond > EFGP_PRECOND_CIRCULANT) return EFGP_EINVAL;
    if (o.precond == EFGP_PRECOND_LEARNED && !o.mlp_weights) return EFGP_EMODEL;
    Plan& P = plan->P;
    if (q == 0) return EFGP_OK;
    return guarded([&]() -> int {
        join_in(P, o.stream);
        int s = run_variance(P, r, q, targets, var_out, o, stats);
        join_out(P, o.stream);
        return s;
    });
}

int efgp_sample_prior(efgp_plan* plan, const void* xi, int64_t q, const void* targets, void* f_out, void* stream) {
    return efgp_eval(plan, xi, q, targets, f_out, stream);
}

int efgp_mean_at_points(efgp_plan* plan, const void* beta, const void* x, void* mu_out, void* stream) {
    if (!plan || !beta || !x || !mu_out || plan->P.prior) return EFGP_EINVAL;
    return efgp_eval(plan, beta, plan->P.n, x, mu_out, stream);
}

int efgp_eval_status(efgp_plan* plan) {
    if (!plan) return EFGP_EINVAL;
    Plan& P = plan->P;
    return guarded([&]() -> int {
        int f = 0;
        EFGP_HIP(hipMemcpyAsync(&f, P.flag, sizeof(int), hipMemcpyDeviceToHost, P.work));
        EFGP_HIP(hipStreamSynchronize(P.work));
        if (f) {
            EFGP_HIP(hipMemsetAsync(P.flag, 0, sizeof(int), P.work));
            EFGP_HIP(hipStreamSynchronize(P.work));
            return EFGP_EDOMAIN;
        }
        return EFGP_OK;
    });
}

static int copy_out(efgp_plan* plan, void* dst, const void* src, size_t bytes, void* stream) {
    if (!plan || !dst) return EFGP_EINVAL;
    Plan& P = plan->P;
    return guarded([&]() -> int {
        join_in(P, stream);
        EFGP_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, P.work));
        join_out(P, stream);
        return EFGP_OK;
    });
}

int efgp_get_toeplitz(const efgp_plan* plan, double* v_out, void* stream) {
    if (!plan) return EFGP_EINVAL;
    const Plan& P = plan->P;
    return copy_out(const_cast<efgp_plan*>(plan), v_out, P.v, 16 * (size_t)ipow(P.W2, P.dim), stream);
}

int efgp_get_rhs(const efgp_plan* plan, double* b_out, void* stream) {
    if (!plan) return EFGP_EINVAL;
    const Plan& P = plan->P;
    return copy_out(const_cast<efgp_plan*>(plan), b_out, P.b64, 16 * (size_t)P.M * P.nrhs, stream);
}

int efgp_get_weights(const efgp_plan* plan, double* d_out, void* stream) {
    if (!plan) return EFGP_EINVAL;
    const Plan& P = plan->P;
    return copy_out(const_cast<efgp_plan*>(plan), d_out, P.D64, 8 * (size_t)P.M, stream);
}

int efgp_apply(efgp_plan* plan, const void* in, void* out, void* stream) {
    if (!plan || !in || !out) return EFGP_EINVAL;
    Plan& P = plan->P;
    return guarded([&]() -> int {
        join_in(P, stream);
        mv_apply(P, in, out, P.work);
        join_out(P, stream);
        return EFGP_OK;
    });
}

int efgp_apply_noalloc(efgp_plan* plan, const void* in, void* out, void* stream) {
    if (!plan || !in || !out) return EFGP_EINVAL;
    Plan& P = plan->P;
    if (noalloc_bytes(P) > kNoAllocBytes) return EFGP_ETOOLARGE;
    return guarded([&]() -> int {
        join_in(P, stream);
        mv_apply_noalloc(P, in, out, P.work);
        join_out(P, stream);
        return EFGP_OK;
    });
}

int efgp_features(const efgp_plan* plan, int32_t r, float* feats_out, float* jacobi_out, void* stream) {
    if (!plan || !feats_out) return EFGP_EINVAL;
    Plan& P = const_cast<efgp_plan*>(plan)->P;
    if (r < 0 || r >= P.nrhs || P.prior) return EFGP_EINVAL;  // features need the points' v
    return guarded([&]() -> int {
        join_in(P, stream);
        run_features(P, r, feats_out, jacobi_out, P.work);
        join_out(P, stream);
        return EFGP_OK;
    });
}

int efgp_circulant_eigs(efgp_plan* plan, int32_t r, int32_t* period, void* lam_out, void* stream) {
    if (!plan) return EFGP_EINVAL;
    Plan& P = plan->P;
    if (r < 0 || r >= P.nrhs || P.prior) return EFGP_EINVAL;  // the system needs the points' v
    if (period) *period = next_smooth235(P.W);
    if (!lam_out) return EFGP_OK;
    return guarded([&]() -> int {
        join_in(P, stream);
        if (P.precision == 32) circ_eigs<float>(P, r, lam_out, P.work);
        else circ_eigs<double>(P, r, lam_out, P.work);
        join_out(P, stream);
        return EFGP_OK;
    });
}

int efgp_get_info(const efgp_plan* plan, efgp_info* info) {
    if (!plan || !info) return EFGP_EINVAL;
    const Plan& P = plan->P;
    std::memset(info, 0, sizeof(*info));
    info->dim = P.dim;
    info->precision = P.precision;
    info->nrhs = P.nrhs;
    info->kernel = P.kernel;
    info->m = P.m;
    info->L = P.L;
    info->nf = P.nf;
    info->nf_eval = P.nf2;
    info->w = P.w;
    info->spread_method = P.spread_method;
    info->tile = P.tile;
    info->setup_passes = P.setup_passes;
    info->M = P.M;
    info->n = P.n;
    info->h = P.h;
    info->es_beta = P.es_beta;
    info->nufft_tol = P.tol;
    info->kernel_l2 = P.kl2;
    info->ms_sort = P.ms_sort;
    info->ms_spread = P.ms_spread;
    info->ms_fft = P.ms_fft;
    info->ms_deconv = P.ms_deconv;
    info->ms_setup_total = P.ms_total;
    return EFGP_OK;
}

void efgp_destroy(efgp_plan* plan) {
    if (!plan) return;
    free_plan(plan->P);
    delete plan;
}

void efgp_release_workspace(void) {
    release_scratch();
    release_pools();
}

int efgp_mlp_forward(const float* params, int64_t rows, const float* feats, float* out, void* stream) {
    if (!params || rows < 0 || (rows > 0 && (!feats || !out))) return EFGP_EINVAL;
    return guarded([&]() -> int {
        mlp_forward(params, rows, feats, out, static_cast<hipStream_t>(stream));
        return EFGP_OK;
    });
}

int efgp_mlp_loss_grad(const float* params, int64_t rows, const float* feats, const float* target,
                       const float* weights, float* grad_out, double* loss_out, void* stream) {
    if (!params || rows < 1 || !feats || !target || !grad_out || !loss_out) return EFGP_EINVAL;
    return guarded([&]() -> int {
        mlp_loss_grad(params, rows, feats, target, weights, grad_out, loss_out, static_cast<hipStream_t>(stream));
        return EFGP_OK;
    });
}

int efgp_mlp_adam(float* params, const float* grad, float* m, float* v, int64_t step, float lr, float beta1,
                  float beta2, float eps, void* stream) {
    if (!params || !grad || !m || !v || step < 1 || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) ||
        !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return EFGP_EINVAL;
    return guarded([&]() -> int {
        mlp_adam(params, grad, m, v, step, lr, beta1, beta2, eps, static_cast<hipStream_t>(stream));
        return EFGP_OK;
    });
}

}  // extern "C"
