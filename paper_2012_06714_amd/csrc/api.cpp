// C ABI entry points: host-side argument validation, error capture, and the
// mapping of C++ exceptions to status codes.
#include <algorithm>
#include <cmath>
#include <vector>
#include <cstring>
#include <string>

#include "context.hpp"

namespace {

thread_local std::string g_err = "no error";
// setup options of this thread (adc_set_setup_option), applied by adc_setup
thread_local long long g_slice_budget = 0;
thread_local int g_setup_verbose = 0;
thread_local int g_m11_fly = 0;

int fail(adc_ctx* c, int code, const std::string& msg) {
    if (c)
        c->err = msg;
    else
        g_err = msg;
    return code;
}

template <typename F>
int guarded(adc_ctx* c, F&& f) {
    try {
        return f();
    } catch (const adc::Error& e) {
        return fail(c, e.code, e.what());
    } catch (const std::bad_alloc&) {
        return fail(c, ADC_E_OOM, "host allocation failed");
    } catch (const std::exception& e) {
        return fail(c, ADC_E_HIP, e.what());
    }
}

}  // namespace

extern "C" {

int adc_setup(const double* eps, const double* B, int nocc, int nvir, int naux, int order, int kind,
              adc_ctx** out) {
    if (!out) return fail(nullptr, ADC_E_ARG, "adc_setup: out is NULL");
    *out = nullptr;
    if (!eps || !B) return fail(nullptr, ADC_E_ARG, "adc_setup: eps or B is NULL");
    if (nocc < 1 || nvir < 1 || naux < 1)
        return fail(nullptr, ADC_E_ARG, "adc_setup: nocc, nvir and naux must be >= 1");
    if (order != 2 && order != 3) return fail(nullptr, ADC_E_ARG, "adc_setup: order must be 2 or 3");
    if (kind != ADC_IP && kind != ADC_EA)
        return fail(nullptr, ADC_E_ARG, "adc_setup: kind must be ADC_IP or ADC_EA");
    if ((long long)nocc + nvir > 46340)
        return fail(nullptr, ADC_E_ARG, "adc_setup: nocc + nvir too large");
    adc_ctx* c = new (std::nothrow) adc_ctx;
    if (!c) return fail(nullptr, ADC_E_OOM, "adc_setup: host allocation failed");
    c->O = nocc;
    c->V = nvir;
    c->Q = naux;
    c->N = nocc + nvir;
    c->order = order;
    c->kind = kind;
    if (kind == ADC_EA) {
        c->n1 = nvir;
        c->n2x = nocc;
        c->n2p = nvir;
    } else {
        c->n1 = nocc;
        c->n2x = nvir;
        c->n2p = nocc;
    }
    c->dim = c->n1 + c->n2x * c->n2p * c->n2p;
    c->E.scratch.arena = &c->arena;
    if (g_slice_budget > 0) c->E.slice_budget = g_slice_budget;
    c->setup_verbose = g_setup_verbose;
    c->m11_fly = g_m11_fly != 0;
    c->setup_t0 = std::chrono::steady_clock::now();
    int rc = guarded(nullptr, [&]() {
        ADC_BLAS(rocblas_create_handle(&c->E.blas));
        c->own_blas = true;
        ADC_BLAS(rocblas_set_stream(c->E.blas, c->E.stream));
        adc::setup_all(c, eps, B);
        return ADC_OK;
    });
    if (rc != ADC_OK) {
        adc_destroy(c);
        return rc;
    }
    *out = c;
    return ADC_OK;
}

int adc_setup_u(const double* eps_a, const double* eps_b, const double* B_a, const double* B_b,
                int nocc_a, int nocc_b, int nmo, int naux, int order, int kind, adc_ctx** out) {
    if (!out) return fail(nullptr, ADC_E_ARG, "adc_setup_u: out is NULL");
    *out = nullptr;
    if (!eps_a || !eps_b || !B_a || !B_b)
        return fail(nullptr, ADC_E_ARG, "adc_setup_u: eps_a, eps_b, B_a or B_b is NULL");
    if (nocc_a < 1 || nocc_b < 1 || naux < 1 || nocc_a >= nmo || nocc_b >= nmo)
        return fail(nullptr, ADC_E_ARG,
                    "adc_setup_u: need 1 <= nocc_a, nocc_b < nmo and naux >= 1");
    if (order != 2)
        return fail(nullptr, ADC_E_ARG, "adc_setup_u: the unrestricted path is built for order 2");
    if (kind != ADC_IP && kind != ADC_EA)
        return fail(nullptr, ADC_E_ARG, "adc_setup_u: kind must be ADC_IP or ADC_EA");
    if (nmo > 46340) return fail(nullptr, ADC_E_ARG, "adc_setup_u: nmo too large");
    adc_ctx* c = new (std::nothrow) adc_ctx;
    if (!c) return fail(nullptr, ADC_E_OOM, "adc_setup_u: host allocation failed");
    c->uhf = true;
    auto& u = c->uh;
    u.Oa = nocc_a;
    u.Ob = nocc_b;
    u.Va = nmo - nocc_a;
    u.Vb = nmo - nocc_b;
    c->O = u.Oa;
    c->V = u.Va;
    c->Q = naux;
    c->N = nmo;
    c->order = 2;
    c->kind = kind;
    const long long Oa = u.Oa, Ob = u.Ob, Va = u.Va, Vb = u.Vb;
    long long len[6];
    if (kind == ADC_EA) {
        len[0] = Va;
        len[1] = Vb;
        len[2] = Oa * (Va * (Va - 1) / 2);
        len[3] = Ob * Va * Vb;
        len[4] = Oa * Va * Vb;
        len[5] = Ob * (Vb * (Vb - 1) / 2);
    } else {
        len[0] = Oa;
        len[1] = Ob;
        len[2] = Va * (Oa * (Oa - 1) / 2);
        len[3] = Vb * Oa * Ob;
        len[4] = Va * Oa * Ob;
        len[5] = Vb * (Ob * (Ob - 1) / 2);
    }
    u.off[0] = 0;
    for (int k = 0; k < 6; ++k) u.off[k + 1] = u.off[k] + len[k];
    c->dim = u.off[6];
    c->n1 = (int)(len[0] + len[1]);
    c->E.scratch.arena = &c->arena;
    if (g_slice_budget > 0) c->E.slice_budget = g_slice_budget;
    c->setup_verbose = g_setup_verbose;
    c->setup_t0 = std::chrono::steady_clock::now();
    int rc = guarded(nullptr, [&]() {
        ADC_BLAS(rocblas_create_handle(&c->E.blas));
        c->own_blas = true;
        ADC_BLAS(rocblas_set_stream(c->E.blas, c->E.stream));
        adc::setup_uhf(c, eps_a, eps_b, B_a, B_b);
        return ADC_OK;
    });
    if (rc != ADC_OK) {
        adc_destroy(c);
        return rc;
    }
    *out = c;
    return ADC_OK;
}

int adc_set_setup_option(const char* key, double value) {
    if (!key) return fail(nullptr, ADC_E_ARG, "adc_set_setup_option: NULL key");
    std::string k(key);
    if (k == "slice_budget") {
        if (!(value >= 0) || value > 1e15 || value != std::floor(value))
            return fail(nullptr, ADC_E_ARG, "slice_budget: a count of elements >= 0");
        g_slice_budget = (long long)value;
        return ADC_OK;
    }
    if (k == "verbose") {
        if (value != 0 && value != 1) return fail(nullptr, ADC_E_ARG, "verbose: 0 or 1");
        g_setup_verbose = (int)value;
        return ADC_OK;
    }
    if (k == "m11_onthefly") {
        if (value != 0 && value != 1) return fail(nullptr, ADC_E_ARG, "m11_onthefly: 0 or 1");
        g_m11_fly = (int)value;
        return ADC_OK;
    }
    return fail(nullptr, ADC_E_ARG, "adc_set_setup_option: unknown key '" + k + "'");
}

int adc_set_option(adc_ctx* c, const char* key, double value) {
    if (!c) return fail(nullptr, ADC_E_ARG, "adc_set_option: NULL context");
    if (!key) return fail(c, ADC_E_ARG, "adc_set_option: NULL key");
    std::string k(key);
    if (!std::isfinite(value)) return fail(c, ADC_E_ARG, "adc_set_option: value not finite");
    if (k == "precision") {
        if (value != 0 && value != 1 && value != 2)
            return fail(c, ADC_E_ARG, "precision must be 0, 1 or 2");
        c->precision = (int)value;
    } else if (k == "block") {
        if (value < 0 || value > 4096) return fail(c, ADC_E_ARG, "block out of range");
        c->block = (int)value;
    } else if (k == "max_space") {
        if (value < 0 || value > 65536) return fail(c, ADC_E_ARG, "max_space out of range");
        c->max_space = (int)value;
    } else if (k == "max_iter") {
        if (value < 1) return fail(c, ADC_E_ARG, "max_iter must be >= 1");
        c->max_iter = (int)value;
    } else if (k == "tol_e") {
        if (value <= 0) return fail(c, ADC_E_ARG, "tol_e must be > 0");
        c->tol_e = value;
    } else if (k == "tol_r") {
        if (value <= 0) return fail(c, ADC_E_ARG, "tol_r must be > 0");
        c->tol_r = value;
    } else if (k == "eigensolver") {
        if (value != 0 && value != 1 && value != 2 && value != 3)
            return fail(c, ADC_E_ARG, "eigensolver: 0, 1, 2 or 3");
        c->eigensolver = (int)value;
    } else if (k == "verbose") {
        if (value < 0 || value > 2) return fail(c, ADC_E_ARG, "verbose: 0, 1 or 2");
        c->verbose = (int)value;
    } else if (k == "graph") {
        // 1: replay sigma from a captured HIP graph per (vector count, precision)
        if (value != 0 && value != 1) return fail(c, ADC_E_ARG, "graph: 0 or 1");
        c->use_graph = value == 1;
        if (!c->use_graph) adc::drop_graphs(c);
    } else if (k == "record") {
        // Davidson iterates (Ritz vector, residual, value) kept for training pairs
        if (value < 0 || value > 100000) return fail(c, ADC_E_ARG, "record out of range");
        if (value > 0 && c->uhf)
            return fail(c, ADC_E_STATE, "record: training pairs are for closed-shell contexts");
        c->record_max = (int)value;
    } else if (k == "precond") {
        // 0: diagonal; 1: the installed learned correction (adc_precond_mlp)
        if (value != 0 && value != 1) return fail(c, ADC_E_ARG, "precond: 0 or 1");
        if (value == 1 && c->uhf)
            return fail(c, ADC_E_STATE, "precond: the learned correction is for closed-shell contexts");
        if (value == 1 && !c->mlp_params.p)
            return fail(c, ADC_E_STATE, "precond: no network installed (adc_precond_mlp)");
        c->use_mlp = value == 1;
    } else if (k == "autotune") {
        // 0: heuristic tile choice, 1: time candidates per shape (default),
        // 2: as 1 and log each choice on stderr
        if (value != 0 && value != 1 && value != 2) return fail(c, ADC_E_ARG, "autotune: 0, 1 or 2");
        c->E.autotune = value != 0;
        c->E.tune_log = value == 2;
    } else if (k == "pp_blocks") {
        if (value < 0 || value > 1e6 || value != std::floor(value))
            return fail(c, ADC_E_ARG, "pp_blocks: a count >= 0");
        c->pp_blocks = (int)value;
        adc::drop_graphs(c);
    } else if (k == "pp_group") {
        if (value < 0 || value > 1e6 || value != std::floor(value))
            return fail(c, ADC_E_ARG, "pp_group: a count >= 0");
        c->pp_group = (int)value;
        adc::drop_graphs(c);
    } else if (k == "ea_layout") {
        // EA sigma: -1 arranged operands when they fit in memory, else built in
        // blocks per call; 0 generic contractions; 1 arranged; 2 blocked
        if (value != -1 && value != 0 && value != 1 && value != 2)
            return fail(c, ADC_E_ARG, "ea_layout: -1, 0, 1 or 2");
        c->ea_layout = (int)value;
        adc::drop_graphs(c);
    } else if (k == "ctr_log") {
        // 1: time each contraction of sigma with events and print its plan on stderr
        if (value != 0 && value != 1) return fail(c, ADC_E_ARG, "ctr_log: 0 or 1");
        c->E.ctr_log = value == 1;
    } else if (k == "bvv_host") {
        // 1: B_vv (and its reduced-precision copies) in pinned host memory, staged per product
        if (value != 0 && value != 1) return fail(c, ADC_E_ARG, "bvv_host: 0 or 1");
        if (c->kind != ADC_EA || c->uhf)
            return fail(c, ADC_E_ARG, "bvv_host: closed-shell EA contexts only");
        return guarded(c, [&]() {
            adc::bvv_set_host(c, value == 1);
            return ADC_OK;
        });
    } else if (k == "gemm_config") {
        // force one matrix-core tile configuration on every product (-1: automatic)
        if (value < -1 || value > 8 || value != std::floor(value))
            return fail(c, ADC_E_ARG, "gemm_config: -1 or a configuration id 0..8");
        c->E.force_cfg = (int)value;
        adc::drop_graphs(c);
    } else if (k == "pp_slab_mb") {
        if (value < 1 || value > 1048576) return fail(c, ADC_E_ARG, "pp_slab_mb out of range");
        c->pp_slab_bytes = (long long)(value * 1048576.0);
        c->pp_slab_set = true;
        c->E.scratch.erase(30);
    } else if (k == "workspace_limit") {
        if (value <= 0) return fail(c, ADC_E_ARG, "workspace_limit must be > 0");
        c->arena.limit = (size_t)value;
    } else {
        return fail(c, ADC_E_ARG, "adc_set_option: unknown key '" + k + "'");
    }
    return ADC_OK;
}

int adc_set_stream(adc_ctx* c, void* s) {
    if (!c) return fail(nullptr, ADC_E_ARG, "adc_set_stream: NULL context");
    return guarded(c, [&]() {
        c->E.stream = (hipStream_t)s;
        ADC_BLAS(rocblas_set_stream(c->E.blas, c->E.stream));
        return ADC_OK;
    });
}

long long adc_dim(const adc_ctx* c) { return c ? c->dim : -1; }

int adc_diag(adc_ctx* c, double* d) {
    if (!c) return fail(nullptr, ADC_E_ARG, "adc_diag: NULL context");
    if (!d) return fail(c, ADC_E_ARG, "adc_diag: NULL output");
    return guarded(c, [&]() {
        ADC_HIP(hipMemcpyAsync(d, c->diag.p, c->dim * sizeof(double), hipMemcpyDeviceToDevice,
                               c->E.stream));
        ADC_HIP(hipStreamSynchronize(c->E.stream));
        return ADC_OK;
    });
}

int adc_sigma(adc_ctx* c, const double* X, double* Y, int nvec) {
    if (!c) return fail(nullptr, ADC_E_ARG, "adc_sigma: NULL context");
    if (!X || !Y) return fail(c, ADC_E_ARG, "adc_sigma: NULL vector");
    if (nvec < 1) return fail(c, ADC_E_ARG, "adc_sigma: nvec must be >= 1");
    const char* xb = (const char*)X;
    const char* yb = (const char*)Y;
    size_t bytes = (size_t)nvec * c->dim * sizeof(double);
    if (xb < yb + bytes && yb < xb + bytes) return fail(c, ADC_E_ARG, "adc_sigma: X and Y overlap");
    return guarded(c, [&]() {
        adc::sigma(c, X, Y, nvec, c->precision);
        ADC_HIP(hipStreamSynchronize(c->E.stream));
        return ADC_OK;
    });
}

int adc_davidson(adc_ctx* c, int nroots, double* energies, double* spec_factors, double* vecs,
                 int* n_iter) {
    if (!c) return fail(nullptr, ADC_E_ARG, "adc_davidson: NULL context");
    if (!energies) return fail(c, ADC_E_ARG, "adc_davidson: NULL energies");
    if (nroots < 1 || nroots > c->dim) return fail(c, ADC_E_ARG, "adc_davidson: bad nroots");
    return guarded(c, [&]() { return adc::davidson(c, nroots, energies, spec_factors, vecs, n_iter); });
}

int adc_spec_factors(adc_ctx* c, const double* vecs, int nvec, double* P, double* X) {
    if (!c) return fail(nullptr, ADC_E_ARG, "adc_spec_factors: NULL context");
    if (!vecs || !P) return fail(c, ADC_E_ARG, "adc_spec_factors: NULL pointer");
    if (nvec < 1) return fail(c, ADC_E_ARG, "adc_spec_factors: nvec must be >= 1");
    return guarded(c, [&]() {
        adc::DBuf<double> Xs;
        double* Xd = X;
        if (!Xd) {
            Xs.alloc((size_t)nvec * c->nspec(), &c->arena);
            Xd = Xs.p;
        }
        adc::spec_amplitudes(c, vecs, nvec, Xd);
        std::vector<double> xh((size_t)nvec * c->nspec());
        ADC_HIP(hipMemcpyAsync(xh.data(), Xd, xh.size() * sizeof(double), hipMemcpyDeviceToHost,
                               c->E.stream));
        ADC_HIP(hipStreamSynchronize(c->E.stream));
        for (int k = 0; k < nvec; ++k) {
            double s = 0.0;
            const int ns = c->nspec();
            for (int p = 0; p < ns; ++p) s += xh[(size_t)k * ns + p] * xh[(size_t)k * ns + p];
            P[k] = c->spec_scale() * s;
        }
        return ADC_OK;
    });
}

int adc_set_guess(adc_ctx* c, const double* V0, int nvec) {
    if (!c) return fail(nullptr, ADC_E_ARG, "adc_set_guess: NULL context");
    if (nvec < 0 || (nvec > 0 && !V0)) return fail(c, ADC_E_ARG, "adc_set_guess: bad arguments");
    return guarded(c, [&]() {
        c->guess.alloc((size_t)nvec * c->dim, &c->arena);
        if (nvec)
            ADC_HIP(hipMemcpyAsync(c->guess.p, V0, (size_t)nvec * c->dim * sizeof(double),
                                   hipMemcpyDeviceToDevice, c->E.stream));
        ADC_HIP(hipStreamSynchronize(c->E.stream));
        c->nguess = nvec;
        return ADC_OK;
    });
}

int adc_history(const adc_ctx* c, int max_entries, double* seconds, double* theta, double* rnorm,
                int* mixed) {
    if (!c) return fail(nullptr, ADC_E_ARG, "adc_history: NULL context");
    int n = (int)c->hist_t.size();
    int m = max_entries < n ? max_entries : n;
    int nr = c->hist_nroots;
    for (int k = 0; k < m; ++k) {
        if (seconds) seconds[k] = c->hist_t[k];
        if (mixed) mixed[k] = c->hist_mixed[k];
        for (int r = 0; r < nr; ++r) {
            if (theta) theta[(size_t)k * nr + r] = c->hist_theta[(size_t)k * nr + r];
            if (rnorm) rnorm[(size_t)k * nr + r] = c->hist_r[(size_t)k * nr + r];
        }
    }
    return n;
}

int adc_sigma_flops(const adc_ctx* c, int nvec, double* total, double* pp) {
    if (!c) return fail(nullptr, ADC_E_ARG, "adc_sigma_flops: NULL context");
    if (nvec < 1) return fail(const_cast<adc_ctx*>(c), ADC_E_ARG, "adc_sigma_flops: nvec < 1");
    double t = 0.0, p = 0.0;
    adc::sigma_cost(c, nvec, &t, &p);
    if (total) *total = t;
    if (pp) *pp = p;
    return ADC_OK;
}

int adc_sigma_timed(adc_ctx* c, const double* X, double* Y, int nvec, double* ms_pp,
                    double* ms_total) {
    if (!c) return fail(nullptr, ADC_E_ARG, "adc_sigma_timed: NULL context");
    if (!X || !Y) return fail(c, ADC_E_ARG, "adc_sigma_timed: NULL vector");
    if (nvec < 1) return fail(c, ADC_E_ARG, "adc_sigma_timed: nvec must be >= 1");
    return guarded(c, [&]() {
        hipEvent_t e0, e1;
        ADC_HIP(hipEventCreate(&e0));
        ADC_HIP(hipEventCreate(&e1));
        c->E.pp_ms = 0.0;
        c->E.timing = true;
        ADC_HIP(hipEventRecord(e0, c->E.stream));
        adc::sigma(c, X, Y, nvec, c->precision);
        ADC_HIP(hipEventRecord(e1, c->E.stream));
        ADC_HIP(hipEventSynchronize(e1));
        c->E.timing = false;
        float ms = 0.f;
        ADC_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ms_total) *ms_total = ms;
        if (ms_pp) *ms_pp = c->E.pp_ms;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return ADC_OK;
    });
}

// ---- spectra from the solver's outputs -------------------------------------
int adc_spectral_function(const double* omega, int nomega, const double* energies, const double* P,
                          int nroots, double eta, double* A, void* stream) {
    if (!omega || !energies || !P || !A)
        return fail(nullptr, ADC_E_ARG, "adc_spectral_function: NULL pointer");
    if (nomega < 1 || nroots < 1 || !(eta > 0) || !std::isfinite(eta))
        return fail(nullptr, ADC_E_ARG, "adc_spectral_function: nomega, nroots >= 1, eta > 0");
    return guarded(nullptr, [&]() {
        adc::spectral_function((hipStream_t)stream, omega, nomega, energies, P, nroots, eta, A);
        ADC_HIP(hipStreamSynchronize((hipStream_t)stream));
        return ADC_OK;
    });
}

int adc_propagator_diag(const double* omega, int nomega, const double* energies, const double* X,
                        int nroots, int norb, double eta, double* G, void* stream) {
    if (!omega || !energies || !X || !G)
        return fail(nullptr, ADC_E_ARG, "adc_propagator_diag: NULL pointer");
    if (nomega < 1 || nroots < 1 || norb < 1 || !(eta > 0) || !std::isfinite(eta))
        return fail(nullptr, ADC_E_ARG, "adc_propagator_diag: sizes >= 1, eta > 0");
    return guarded(nullptr, [&]() {
        adc::propagator_diag((hipStream_t)stream, omega, nomega, energies, X, nroots, norb, eta, G);
        ADC_HIP(hipStreamSynchronize((hipStream_t)stream));
        return ADC_OK;
    });
}

// ---- the matrix-core product on its own ------------------------------------
int adc_gemm_configs(int dtype, int* ids) {
    if (!ids) return fail(nullptr, ADC_E_ARG, "adc_gemm_configs: NULL ids");
    switch (dtype) {
        case 0: return adc::gemm_candidates<double>(ids);
        case 1: return adc::gemm_candidates<float>(ids);
        case 2:
        case 3: return adc::gemm_candidates<adc::bf16_t>(ids);
        default: return fail(nullptr, ADC_E_ARG, "adc_gemm_configs: dtype must be 0..3");
    }
}

int adc_gemm(int dtype, int ta, int tb, long long M, long long N, long long K, double alpha,
             const void* A, long long lda, const void* B, long long ldb, double beta, void* C,
             long long ldc, const long long* map, int config, void* stream) {
    if (dtype < 0 || dtype > 3) return fail(nullptr, ADC_E_ARG, "adc_gemm: dtype must be 0..3");
    if (M < 1 || N < 1 || K < 0) return fail(nullptr, ADC_E_ARG, "adc_gemm: M, N >= 1, K >= 0");
    if (!A || !B || !C) return fail(nullptr, ADC_E_ARG, "adc_gemm: NULL operand");
    if (lda < (ta ? M : K) || ldb < (tb ? K : N) || (!map && ldc < N))
        return fail(nullptr, ADC_E_ARG, "adc_gemm: leading dimension too small");
    if (config < -1 || config > 8) return fail(nullptr, ADC_E_ARG, "adc_gemm: config -1..8");
    adc::GemmOut out = adc::GemmOut::rowmajor(ldc);
    if (map) {
        if (map[0] < 0 || map[3] < 0)
            return fail(nullptr, ADC_E_ARG, "adc_gemm: bad output map");
        out.rsplit = map[0];
        out.rs1 = map[1];
        out.rs2 = map[2];
        out.csplit = map[3];
        out.cs1 = map[4];
        out.cs2 = map[5];
    }
    return guarded(nullptr, [&]() {
        adc::Engine E;
        E.stream = (hipStream_t)stream;
        E.autotune = false;
        E.force_cfg = config;
        const bool a = ta != 0, b = tb != 0;
        switch (dtype) {
            case 0:
                adc::gemm_run<double, double, double>(E, a, b, M, N, K, alpha, (const double*)A,
                                                      lda, 0, (const double*)B, ldb, 0, beta,
                                                      (double*)C, out, 1);
                break;
            case 1:
                adc::gemm_run<float, float, float>(E, a, b, M, N, K, (float)alpha,
                                                   (const float*)A, lda, 0, (const float*)B, ldb,
                                                   0, (float)beta, (float*)C, out, 1);
                break;
            case 2:
                adc::gemm_run<float, adc::bf16_t, float>(E, a, b, M, N, K, (float)alpha,
                                                         (const float*)A, lda, 0, (const float*)B,
                                                         ldb, 0, (float)beta, (float*)C, out, 1);
                break;
            default:
                adc::gemm_run<adc::bf16_t, adc::bf16_t, float>(
                    E, a, b, M, N, K, (float)alpha, (const adc::bf16_t*)A, lda, 0,
                    (const adc::bf16_t*)B, ldb, 0, (float)beta, (float*)C, out, 1);
        }
        ADC_HIP(hipStreamSynchronize(E.stream));
        return ADC_OK;
    });
}

// ---- learned preconditioner -----------------------------------------------
long long adc_mlp_nparams(void) { return adc::MLP_NPARAM; }

int adc_precond_mlp(adc_ctx* c, const float* params, long long nparams) {
    if (!c) return fail(nullptr, ADC_E_ARG, "adc_precond_mlp: NULL context");
    if (!params) {
        c->use_mlp = false;
        c->mlp_params.release();
        return ADC_OK;
    }
    if (nparams != adc::MLP_NPARAM)
        return fail(c, ADC_E_ARG, "adc_precond_mlp: nparams must equal adc_mlp_nparams()");
    return guarded(c, [&]() {
        c->mlp_params.alloc((size_t)nparams, &c->arena);
        ADC_HIP(hipMemcpyAsync(c->mlp_params.p, params, nparams * sizeof(float),
                               hipMemcpyDeviceToDevice, c->E.stream));
        ADC_HIP(hipStreamSynchronize(c->E.stream));
        c->use_mlp = true;
        return ADC_OK;
    });
}

int adc_mlp_status(const adc_ctx* c, int* installed, int* fallbacks) {
    if (!c) return fail(nullptr, ADC_E_ARG, "adc_mlp_status: NULL context");
    if (installed) *installed = c->use_mlp ? 1 : 0;
    if (fallbacks) *fallbacks = c->mlp_fallbacks;
    return ADC_OK;
}

int adc_mlp_pairs(adc_ctx* c, const double* x, const double* r, double theta, const double* xstar,
                  const long long* idx, long long nidx, float* F, float* a, float* t) {
    if (!c) return fail(nullptr, ADC_E_ARG, "adc_mlp_pairs: NULL context");
    if (!x || !r || !xstar || !idx || !F || !a || !t || nidx < 1 || !std::isfinite(theta))
        return fail(c, ADC_E_ARG, "adc_mlp_pairs: bad arguments");
    if (c->uhf) return fail(c, ADC_E_STATE, "adc_mlp_pairs: closed-shell contexts only");
    return guarded(c, [&]() {
        adc::mlp_pairs(c, x, r, theta, xstar, idx, nidx, F, a, t);
        ADC_HIP(hipStreamSynchronize(c->E.stream));
        return ADC_OK;
    });
}

int adc_mlp_forward_noalloc(const float* params, const float* F, long long n, int bf16, float* y,
                            void* stream) {
    if (!params || !F || !y) return fail(nullptr, ADC_E_ARG, "adc_mlp_forward_noalloc: NULL pointer");
    if (n < 1 || n > adc::MLP_NOALLOC_ROWS)
        return fail(nullptr, ADC_E_ARG,
                    "adc_mlp_forward_noalloc: n must be 1.." + std::to_string(adc::MLP_NOALLOC_ROWS));
    return guarded(nullptr, [&]() {
        adc::mlp_forward_noalloc(params, F, n, bf16 != 0, y, (hipStream_t)stream);
        ADC_HIP(hipGetLastError());
        return ADC_OK;
    });
}

int adc_mlp_forward(adc_ctx* c, const float* params, const float* F, long long n, int bf16,
                    float* y) {
    if (!c) return fail(nullptr, ADC_E_ARG, "adc_mlp_forward: NULL context");
    if (!params || !F || !y || n < 1) return fail(c, ADC_E_ARG, "adc_mlp_forward: bad arguments");
    return guarded(c, [&]() {
        adc::mlp_forward(c, params, F, n, bf16 != 0, y);
        ADC_HIP(hipStreamSynchronize(c->E.stream));
        return ADC_OK;
    });
}

int adc_mlp_loss_grad(adc_ctx* c, const float* params, const float* F, const float* a,
                      const float* t, long long n, float* grad, double* loss) {
    if (!c) return fail(nullptr, ADC_E_ARG, "adc_mlp_loss_grad: NULL context");
    if (!params || !F || !a || !t || !grad || n < 1)
        return fail(c, ADC_E_ARG, "adc_mlp_loss_grad: bad arguments");
    return guarded(c, [&]() {
        double l = adc::mlp_loss_grad(c, params, F, a, t, n, grad);
        if (loss) *loss = l;
        return ADC_OK;
    });
}

int adc_mlp_adam(adc_ctx* c, float* params, const float* grad, float* m, float* v, int step,
                 double lr) {
    if (!c) return fail(nullptr, ADC_E_ARG, "adc_mlp_adam: NULL context");
    if (!params || !grad || !m || !v || step < 1 || !(lr > 0))
        return fail(c, ADC_E_ARG, "adc_mlp_adam: bad arguments");
    return guarded(c, [&]() {
        adc::mlp_adam(c, params, grad, m, v, adc::MLP_NPARAM, step, lr);
        ADC_HIP(hipStreamSynchronize(c->E.stream));
        return ADC_OK;
    });
}

}  // extern "C"

struct adc_batch {
    std::vector<adc_ctx*> ctx;
};

extern "C" {

int adc_setup_batch(int nsys, const adc_system_desc* sys, adc_batch** out) {
    if (!out) return fail(nullptr, ADC_E_ARG, "adc_setup_batch: out is NULL");
    *out = nullptr;
    if (nsys < 1 || !sys) return fail(nullptr, ADC_E_ARG, "adc_setup_batch: bad arguments");
    adc_batch* b = new (std::nothrow) adc_batch;
    if (!b) return fail(nullptr, ADC_E_OOM, "adc_setup_batch: host allocation failed");
    for (int k = 0; k < nsys; ++k) {
        adc_ctx* c = nullptr;
        const adc_system_desc& d = sys[k];
        int rc = adc_setup(d.eps, d.B, d.nocc, d.nvir, d.naux, d.order, d.kind, &c);
        if (rc != ADC_OK) {
            std::string msg = "adc_setup_batch: system " + std::to_string(k) + ": " + g_err;
            adc_batch_destroy(b);
            return fail(nullptr, rc, msg);
        }
        b->ctx.push_back(c);
    }
    *out = b;
    return ADC_OK;
}

int adc_batch_set_option(adc_batch* b, const char* key, double value) {
    if (!b) return fail(nullptr, ADC_E_ARG, "adc_batch_set_option: NULL batch");
    for (size_t k = 0; k < b->ctx.size(); ++k) {
        int rc = adc_set_option(b->ctx[k], key, value);
        if (rc != ADC_OK)
            return fail(nullptr, rc, "adc_batch_set_option: system " + std::to_string(k) + ": " +
                                         b->ctx[k]->err);
    }
    return ADC_OK;
}

int adc_davidson_batch(adc_batch* b, int nroots, int flags, double* energies,
                       double* spec_factors, int* n_iter, int* status, long long* stats) {
    if (!b) return fail(nullptr, ADC_E_ARG, "adc_davidson_batch: NULL batch");
    return adc_batch_davidson(b->ctx.data(), (int)b->ctx.size(), nroots, flags, energies,
                              spec_factors, n_iter, status, stats);
}

adc_ctx* adc_batch_context(adc_batch* b, int k) {
    if (!b || k < 0 || k >= (int)b->ctx.size()) return nullptr;
    return b->ctx[k];
}

void adc_batch_destroy(adc_batch* b) {
    if (!b) return;
    for (adc_ctx* c : b->ctx) adc_destroy(c);
    delete b;
}

int adc_batch_davidson(adc_ctx* const* ctxs, int nsys, int nroots, int flags,
                       double* energies, double* spec_factors, int* n_iter, int* status,
                       long long* stats) {
    // bits 0-1: graph, concurrent; bits 8-15: host threads of the concurrent mode
    if (!ctxs || nsys < 1 || nroots < 1 || !energies || flags < 0 || (flags & ~0xFF07) != 0)
        return fail(nullptr, ADC_E_ARG, "adc_batch_davidson: bad arguments");
    const int nthreads = ((flags >> 8) & 0xFF) ? ((flags >> 8) & 0xFF) : 8;
    if (nthreads > 64) return fail(nullptr, ADC_E_ARG, "adc_batch_davidson: at most 64 threads");
    for (int k = 0; k < nsys; ++k) {
        if (!ctxs[k]) return fail(nullptr, ADC_E_ARG, "adc_batch_davidson: NULL context");
        if (nroots > ctxs[k]->dim)
            return fail(nullptr, ADC_E_ARG, "adc_batch_davidson: nroots exceeds a dimension");
        for (int j = 0; j < k; ++j)
            if (ctxs[j] == ctxs[k])
                return fail(nullptr, ADC_E_ARG, "adc_batch_davidson: a context appears twice");
    }
    const bool use_graph = (flags & 1) != 0;
    if (flags & 2) {
        return guarded(nullptr, [&]() {
            const long long l0 = [&]() {
                long long n = 0;
                for (int k = 0; k < nsys; ++k) n += ctxs[k]->graph_launches;
                return n;
            }();
            long long c0 = 0;
            for (int k = 0; k < nsys; ++k) c0 += ctxs[k]->graph_captures;
            std::vector<int> its(nsys);
            int rc = adc::batch_concurrent(ctxs, nsys, nroots, use_graph, nthreads, energies,
                                           spec_factors, its.data(), status);
            if (n_iter)
                for (int k = 0; k < nsys; ++k) n_iter[k] = its[k];
            if (stats) {
                long long l1 = 0, c1 = 0;
                for (int k = 0; k < nsys; ++k) {
                    l1 += ctxs[k]->graph_launches;
                    c1 += ctxs[k]->graph_captures;
                }
                stats[0] = *std::max_element(its.begin(), its.end());
                stats[1] = l1 - l0;
                stats[2] = c1 - c0;
            }
            return rc;
        });
    }
    return guarded(nullptr, [&]() {
        adc::BatchStats st;
        int rc = adc::batch_davidson(ctxs, nsys, nroots, use_graph, energies, spec_factors,
                                     n_iter, status, &st);
        if (stats) {
            stats[0] = st.iterations;
            stats[1] = st.graph_launches;
            stats[2] = st.captures;
            if (flags & 4) {
                stats[3] = st.launches;
                stats[4] = st.parents;
            }
        }
        return rc;
    });
}

long long adc_graph_launches(const adc_ctx* c) { return c ? c->graph_launches : -1; }

int adc_record_count(const adc_ctx* c) {
    if (!c) return fail(nullptr, ADC_E_ARG, "adc_record_count: NULL context");
    return c->nrec;
}

int adc_record_get(adc_ctx* c, int i, double* x, double* r, double* theta, int* root) {
    if (!c) return fail(nullptr, ADC_E_ARG, "adc_record_get: NULL context");
    if (i < 0 || i >= c->nrec) return fail(c, ADC_E_ARG, "adc_record_get: index out of range");
    return guarded(c, [&]() {
        if (x)
            ADC_HIP(hipMemcpyAsync(x, c->rec_x.p + (size_t)i * c->dim, c->dim * sizeof(double),
                                   hipMemcpyDeviceToDevice, c->E.stream));
        if (r)
            ADC_HIP(hipMemcpyAsync(r, c->rec_r.p + (size_t)i * c->dim, c->dim * sizeof(double),
                                   hipMemcpyDeviceToDevice, c->E.stream));
        ADC_HIP(hipStreamSynchronize(c->E.stream));
        if (theta) *theta = c->rec_theta[i];
        if (root) *root = c->rec_root[i];
        return ADC_OK;
    });
}

const char* adc_last_error(const adc_ctx* c) { return c ? c->err.c_str() : g_err.c_str(); }

int adc_last_stats(const adc_ctx* c, int* iters, long long* sigvec, int* mixed_iters,
                   double* seconds) {
    if (!c) return fail(nullptr, ADC_E_ARG, "adc_last_stats: NULL context");
    if (iters) *iters = c->st_iters;
    if (sigvec) *sigvec = c->st_sigvec;
    if (mixed_iters) *mixed_iters = c->st_mixed;
    if (seconds) *seconds = c->st_seconds;
    return ADC_OK;
}

int adc_workspace(const adc_ctx* c, long long* used, long long* peak) {
    if (!c) return fail(nullptr, ADC_E_ARG, "adc_workspace: NULL context");
    if (used) *used = (long long)c->arena.used;
    if (peak) *peak = (long long)c->arena.peak;
    return ADC_OK;
}

void adc_destroy(adc_ctx* c) {
    if (!c) return;
    if (c->E.stream) (void)hipStreamSynchronize(c->E.stream);
    else (void)hipDeviceSynchronize();
    adc::drop_graphs(c);
    if (c->gstream) {
        (void)hipStreamSynchronize(c->gstream);
        (void)hipStreamDestroy(c->gstream);
    }
    if (c->gdone) (void)hipEventDestroy(c->gdone);
    c->E.scratch.clear();
    for (hipEvent_t& e : c->E.tev)
        if (e) (void)hipEventDestroy(e);
    if (c->own_blas && c->E.blas) rocblas_destroy_handle(c->E.blas);
    if (c->ttu_host) (void)hipHostFree(c->ttu_host);
    adc::bvv_release_host(c);
    delete c;
}

}  // extern "C"
