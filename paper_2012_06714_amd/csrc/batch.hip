// Several independent systems (contexts) solved together: the Davidson
// solvers advance in lockstep, and each iteration applies sigma to the new
// trial vectors of every active system with one graph launch: a parent graph
// holds, for every system whose sigma graph (captured per vector count and
// precision, kept by the context) is ready, the copy of its trial vectors
// into the graph's input, that graph as a child node, and the copy of the
// result out; the systems' branches are independent, so unequal systems run
// side by side.  The parent is instantiated again only when the set of
// (system, vector count, precision) changes; otherwise only its copy nodes
// are pointed at the iteration's vectors.  A system whose graph is not
// captured yet runs its sigma (and the capture) on its own first.
#include "context.hpp"

#include <array>
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

namespace {

// The parent graph of one iteration's sigma replays (see above)
struct Parent {
    std::vector<std::array<long long, 3>> key;   // (system, nvec, precision)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<hipGraphNode_t> in, out;          // copy nodes per entry
    ~Parent() { reset(); }
    void reset() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        in.clear();
        out.clear();
        key.clear();
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
    Parent par;
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
            // systems with a ready graph: one launch of the parent graph
            std::vector<int> ready, rest;
            std::vector<std::array<long long, 3>> key;
            std::vector<hipGraph_t> child;
            for (int k : active) {
                hipGraph_t g = sigma_graph_ready(ctx[k], nn[k], prec[k]);
                if (g) {
                    ready.push_back(k);
                    key.push_back({k, nn[k], prec[k]});
                    child.push_back(g);
                } else {
                    rest.push_back(k);
                }
            }
            if (!ready.empty()) {
                if (key != par.key) {
                    par.reset();
                    ADC_HIP(hipGraphCreate(&par.graph, 0));
                    for (size_t r = 0; r < ready.size(); ++r) {
                        adc_ctx* c = ctx[ready[r]];
                        const size_t bytes = (size_t)nn[ready[r]] * c->dim * sizeof(double);
                        hipGraphNode_t a = nullptr, g = nullptr, b = nullptr;
                        ADC_HIP(hipGraphAddMemcpyNode1D(&a, par.graph, nullptr, 0, c->Xg.p,
                                                        X[ready[r]], bytes,
                                                        hipMemcpyDeviceToDevice));
                        ADC_HIP(hipGraphAddChildGraphNode(&g, par.graph, &a, 1, child[r]));
                        ADC_HIP(hipGraphAddMemcpyNode1D(&b, par.graph, &g, 1, W[ready[r]],
                                                        c->Yg.p, bytes,
                                                        hipMemcpyDeviceToDevice));
                        par.in.push_back(a);
                        par.out.push_back(b);
                    }
                    ADC_HIP(hipGraphInstantiate(&par.exec, par.graph, nullptr, nullptr, 0));
                    par.key = key;
                    if (st) st->parents++;
                } else {
                    for (size_t r = 0; r < ready.size(); ++r) {
                        adc_ctx* c = ctx[ready[r]];
                        const size_t bytes = (size_t)nn[ready[r]] * c->dim * sizeof(double);
                        ADC_HIP(hipGraphExecMemcpyNodeSetParams1D(
                            par.exec, par.in[r], c->Xg.p, X[ready[r]], bytes,
                            hipMemcpyDeviceToDevice));
                        ADC_HIP(hipGraphExecMemcpyNodeSetParams1D(
                            par.exec, par.out[r], W[ready[r]], c->Yg.p, bytes,
                            hipMemcpyDeviceToDevice));
                    }
                }
                // the launch waits for every ready system's stream, and they for it
                for (int k : ready) {
                    ADC_HIP(hipEventRecord(S.sync, ctx[k]->E.stream));
                    ADC_HIP(hipStreamWaitEvent(S.main, S.sync, 0));
                }
                ADC_HIP(hipGraphLaunch(par.exec, S.main));
                ADC_HIP(hipEventRecord(S.ready, S.main));
                for (int k : ready) {
                    ADC_HIP(hipStreamWaitEvent(ctx[k]->E.stream, S.ready, 0));
                    ctx[k]->graph_launches++;
                }
                if (st) {
                    st->graph_launches += (long long)ready.size();
                    st->launches++;
                }
            }
            // the others capture (and run) their graph one by one, the systems
            // dealt round-robin to the branch streams; each branch waits for its
            // system's stream and the system's stream waits for the branch
            int b = 0;
            for (int k : rest) {
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
