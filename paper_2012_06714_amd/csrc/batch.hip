// Several independent systems (contexts) solved together: the Davidson
// solvers advance in lockstep, and each iteration applies sigma to the new
// trial vectors of every active system as replays of that system's captured
// sigma graphs (one per vector count and precision, kept by the context),
// issued back to back over a few streams so that unequal systems run side by
// side.  Per-system graphs are captured a handful of times per solve; a
// single graph over the whole active set would have to be captured again
// whenever any system converges or changes its number of new vectors.
#include "context.hpp"

#include <atomic>
#include <thread>
#include <vector>

namespace adc {

namespace {

constexpr int NSTREAM = 4;    // branch streams (default priority)

struct Streams {
    hipStream_t main = nullptr;
    hipStream_t br[NSTREAM] = {};
    hipEvent_t fork = nullptr, join[NSTREAM] = {}, ready = nullptr, sync = nullptr;
    Streams() {
        ADC_HIP(hipStreamCreate(&main));
        for (auto& b : br) ADC_HIP(hipStreamCreate(&b));
        ADC_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
        for (auto& e : join) ADC_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        ADC_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
        ADC_HIP(hipEventCreateWithFlags(&sync, hipEventDisableTiming));
    }
    ~Streams() {
        if (main) (void)hipStreamSynchronize(main);
        for (auto& b : br)
            if (b) {
                (void)hipStreamSynchronize(b);
                (void)hipStreamDestroy(b);
            }
        if (main) (void)hipStreamDestroy(main);
        for (hipEvent_t e : {fork, ready, sync})
            if (e) (void)hipEventDestroy(e);
        for (auto& e : join)
            if (e) (void)hipEventDestroy(e);
    }
};

struct StreamSwap {
    Engine& e;
    hipStream_t old;
    bool tune;
    StreamSwap(Engine& en, hipStream_t s) : e(en), old(en.stream), tune(en.autotune) {
        e.stream = s;
    }
    ~StreamSwap() {
        e.stream = old;
        e.autotune = tune;
        e.scratch.touched = nullptr;
    }
};

}  // namespace

int batch_davidson(adc_ctx* const* ctx, int nsys, int nroots, bool use_graph, double* energies,
                   double* P, int* n_iter, int* status, BatchStats* st) {
    std::vector<Solver*> sol(nsys, nullptr);
    struct Cleanup {
        std::vector<Solver*>& s;
        ~Cleanup() {
            for (Solver* x : s)
                if (x) solver_delete(x);
        }
    } cleanup{sol};
    for (int k = 0; k < nsys; ++k) sol[k] = solver_new(ctx[k], nroots);
    Streams S;
    std::vector<const double*> X(nsys);
    std::vector<double*> W(nsys);
    std::vector<int> nn(nsys), prec(nsys), active;
    while (true) {
        active.clear();
        for (int k = 0; k < nsys; ++k)
            if (solver_request(sol[k], &X[k], &W[k], &nn[k], &prec[k])) active.push_back(k);
        if (active.empty()) break;
        if (st) st->iterations++;
        if (!use_graph) {
            for (int k : active) sigma(ctx[k], X[k], W[k], nn[k], prec[k]);
        } else {
            // each active system replays its own sigma graph (captured per
            // vector count and precision), the systems dealt round-robin to
            // the branch streams so that unequal ones run side by side; each
            // branch waits for its system's stream and the system's stream
            // waits for the branch
            int b = 0;
            for (int k : active) {
                adc_ctx* c = ctx[k];
                hipStream_t br = S.br[b++ % NSTREAM];
                ADC_HIP(hipEventRecord(S.sync, c->E.stream));
                ADC_HIP(hipStreamWaitEvent(br, S.sync, 0));
                const long long cap0 = c->graph_captures;
                {
                    StreamSwap sw(c->E, br);
                    const bool ug = c->use_graph;
                    c->use_graph = true;
                    try {
                        sigma(c, X[k], W[k], nn[k], prec[k]);
                    } catch (...) {
                        c->use_graph = ug;
                        throw;
                    }
                    c->use_graph = ug;
                }
                ADC_HIP(hipEventRecord(S.sync, br));
                ADC_HIP(hipStreamWaitEvent(c->E.stream, S.sync, 0));
                if (st) {
                    st->graph_launches += (nn[k] + 63) / 64;
                    st->captures += c->graph_captures - cap0;
                }
            }
        }
        for (int k : active) {
            // a solver whose space changed shape frees scratch only at its end
            solver_advance(sol[k]);
        }
    }
    int worst = ADC_OK;
    for (int k = 0; k < nsys; ++k) {
        int it = 0;
        int s = solver_finish(sol[k], energies + (size_t)k * nroots,
                              P ? P + (size_t)k * nroots : nullptr, nullptr, &it);
        if (n_iter) n_iter[k] = it;
        if (status) status[k] = s;
        if (s != ADC_OK && worst == ADC_OK) worst = s;
    }
    return worst;
}

// The same systems solved concurrently instead of in lockstep: up to
// `nthreads` host threads each take the next unsolved system and run the
// single-system solver on it, on a stream of its own when the context is
// bound to the null stream.  The host work of one solve (its small
// eigenproblems, the synchronisations that read residual norms back) then
// overlaps the device work of the others.
int batch_concurrent(adc_ctx* const* ctx, int nsys, int nroots, bool use_graph, int nthreads,
                     double* energies, double* P, int* n_iter, int* status) {
    std::atomic<int> next{0};
    std::vector<int> st(nsys, ADC_OK), its(nsys, 0);
    auto solve = [&](int k) {
        adc_ctx* c = ctx[k];
        const hipStream_t old = c->E.stream;
        hipStream_t mine = nullptr;
        const bool ug = c->use_graph;
        try {
            if (!old) {
                ADC_HIP(hipStreamCreate(&mine));
                c->E.stream = mine;
                ADC_BLAS(rocblas_set_stream(c->E.blas, mine));
            }
            c->use_graph = use_graph;
            st[k] = davidson(c, nroots, energies + (size_t)k * nroots,
                             P ? P + (size_t)k * nroots : nullptr, nullptr, &its[k]);
        } catch (const Error& e) {
            st[k] = e.code;
            c->err = e.what();
        } catch (const std::exception& e) {
            st[k] = ADC_E_HIP;
            c->err = e.what();
        }
        c->use_graph = ug;
        if (mine) {
            (void)hipStreamSynchronize(mine);
            c->E.stream = old;
            (void)rocblas_set_stream(c->E.blas, old);
            (void)hipStreamDestroy(mine);
        }
    };
    const int nt = std::max(1, std::min(nthreads, nsys));
    std::vector<std::thread> pool;
    for (int t = 0; t < nt; ++t)
        pool.emplace_back([&]() {
            for (int k = next++; k < nsys; k = next++) solve(k);
        });
    for (auto& t : pool) t.join();
    int worst = ADC_OK;
    for (int k = 0; k < nsys; ++k) {
        if (n_iter) n_iter[k] = its[k];
        if (status) status[k] = st[k];
        if (st[k] != ADC_OK && worst == ADC_OK) worst = st[k];
    }
    return worst;
}

}  // namespace adc
