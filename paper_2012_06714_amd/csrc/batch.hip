// Several independent systems (contexts) solved together: the Davidson
// solvers advance in lockstep, and each iteration applies sigma to the new
// trial vectors of every active system in one HIP graph launch.  The graph
// holds one branch per system (spread over a few streams, so unequal systems
// run side by side); it is captured after an eager warm-up of every branch and
// reused for as long as the set of (system, vector count, precision) and the
// scratch buffers of its contexts stay the same.  Trial vectors enter and
// results leave through each context's fixed graph buffers.
#include "context.hpp"

#include <vector>

namespace adc {

namespace {

constexpr int NSTREAM = 4;    // branch streams (default priority)

struct BatchGraph {
    std::vector<long long> key;                                   // (system, nvec, precision)...
    std::vector<std::map<int, std::pair<void*, size_t>>> slots;  // scratch per branch
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~BatchGraph() { drop(); }
    void drop() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
};

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
    BatchGraph G;
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
            std::vector<long long> key;
            for (int k : active) {
                key.push_back(k);
                key.push_back(nn[k]);
                key.push_back(prec[k]);
                adc_ctx* c = ctx[k];
                const size_t need = (size_t)nn[k] * c->dim;
                if (c->Xg.n < need) {
                    G.drop();
                    drop_graphs(c);
                    c->Xg.alloc(need, &c->arena);
                    c->Yg.alloc(need, &c->arena);
                }
            }
            bool valid = G.exec && G.key == key;
            for (size_t b = 0; valid && b < active.size(); ++b)
                valid = ctx[active[b]]->E.scratch.still_valid(G.slots[b]);
            // trial vectors in: the main stream waits for each system's own stream
            for (int k : active) {
                adc_ctx* c = ctx[k];
                ADC_HIP(hipEventRecord(S.sync, c->E.stream));
                ADC_HIP(hipStreamWaitEvent(S.main, S.sync, 0));
                ADC_HIP(hipMemcpyAsync(c->Xg.p, X[k], (size_t)nn[k] * c->dim * sizeof(double),
                                       hipMemcpyDeviceToDevice, S.main));
            }
            if (!valid) {
                G.drop();
                // warm-up: every branch once, eagerly (allocations, tile tuning)
                for (int k : active) {
                    StreamSwap sw(ctx[k]->E, S.main);
                    sigma_eager(ctx[k], ctx[k]->Xg.p, ctx[k]->Yg.p, nn[k], prec[k]);
                }
                ADC_HIP(hipStreamSynchronize(S.main));
                G.slots.assign(active.size(), {});
                ADC_HIP(hipStreamBeginCapture(S.main, hipStreamCaptureModeThreadLocal));
                try {
                    ADC_HIP(hipEventRecord(S.fork, S.main));
                    for (auto& b : S.br) ADC_HIP(hipStreamWaitEvent(b, S.fork, 0));
                    for (size_t b = 0; b < active.size(); ++b) {
                        adc_ctx* c = ctx[active[b]];
                        StreamSwap sw(c->E, S.br[b % NSTREAM]);
                        c->E.autotune = false;
                        c->E.scratch.touched = &G.slots[b];
                        sigma_eager(c, c->Xg.p, c->Yg.p, nn[active[b]], prec[active[b]]);
                    }
                    for (int b = 0; b < NSTREAM; ++b) {
                        ADC_HIP(hipEventRecord(S.join[b], S.br[b]));
                        ADC_HIP(hipStreamWaitEvent(S.main, S.join[b], 0));
                    }
                } catch (...) {
                    hipGraph_t dead = nullptr;
                    (void)hipStreamEndCapture(S.main, &dead);
                    if (dead) (void)hipGraphDestroy(dead);
                    throw;
                }
                ADC_HIP(hipStreamEndCapture(S.main, &G.graph));
                ADC_HIP(hipGraphInstantiate(&G.exec, G.graph, nullptr, nullptr, 0));
                G.key = key;
                if (st) st->captures++;
            }
            ADC_HIP(hipGraphLaunch(G.exec, S.main));
            if (st) st->graph_launches++;
            // results out; each system's stream waits for them
            for (int k : active) {
                adc_ctx* c = ctx[k];
                ADC_HIP(hipMemcpyAsync(W[k], c->Yg.p, (size_t)nn[k] * c->dim * sizeof(double),
                                       hipMemcpyDeviceToDevice, S.main));
            }
            ADC_HIP(hipEventRecord(S.ready, S.main));
            for (int k : active) ADC_HIP(hipStreamWaitEvent(ctx[k]->E.stream, S.ready, 0));
        }
        for (int k : active) {
            // a solver whose space changed shape frees scratch only at its end
            solver_advance(sol[k]);
        }
    }
    G.drop();
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

}  // namespace adc
