// Reduced-precision copies of the resident sigma operands, made on the first
// mixed-precision sigma call: FP32 for every tensor the contractions read
// (their GEMMs round to BF16 while staging tiles and accumulate in FP32) and
// BF16 for B_vv, the operand of the particle-particle rebuild.  The FP64
// originals stay resident for the refinement passes.
#include "context.hpp"

namespace adc {

template <typename TO>
__global__ void k_narrow(const double* __restrict__ in, TO* __restrict__ out, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        out[i] = (TO)in[i];
}

template <typename TO>
static void narrow(adc_ctx* c, const DBuf<double>& src, DBuf<TO>& dst) {
    if (!src.p || src.n == 0) {
        dst.release();
        return;
    }
    dst.alloc(src.n, &c->arena);
    size_t g = (src.n + 255) / 256;
    if (g > (1u << 20)) g = 1u << 20;
    hipLaunchKernelGGL(k_narrow<TO>, dim3((unsigned)g), dim3(256), 0, c->E.stream, src.p, dst.p,
                       src.n);
    ADC_HIP(hipGetLastError());
}

// t~ = 2 t_ij^ab - t_ij^ba made again from t (the blocked EA path releases it)
void ensure_tt(adc_ctx* c) {
    if (c->tt.p || c->order != 3) return;
    const size_t n = (size_t)c->O * c->O * c->V * c->V;
    c->tt.alloc(n, &c->arena);
    permute<double>(c->E, -1.0, "ijab", c->t.p, 0.0, "ijba", c->tt.p);
    axpy<double>(c->E, 2.0, c->t.p, c->tt.p, n);
}

void build_mixed(adc_ctx* c, bool big) {
    if (big && !c->big_mixed && c->order == 3) {
        ensure_tt(c);
        narrow(c, c->ovov, c->fovov);
        narrow(c, c->oovv, c->foovv);
        narrow(c, c->t, c->ft);
        narrow(c, c->tt, c->ftt);
        c->big_mixed = true;
    }
    if (c->mixed_ready) return;
    narrow(c, c->Boo, c->fBoo);
    narrow(c, c->Bov, c->fBov);
    narrow(c, c->Bvo, c->fBvo);
    narrow(c, c->M11, c->fM11);
    if (c->order == 3) {
        narrow(c, c->ooov, c->fooov);
        narrow(c, c->gam, c->fgam);
        if (c->kind == ADC_EA) {
            if (!c->bvv_host) narrow(c, c->Bvv, c->hBvv);
        } else {
            narrow(c, c->oooo, c->foooo);
            narrow(c, c->Om, c->fOm);
            narrow(c, c->Pi, c->fPi);
        }
    }
    // the first-order coupling reads B_vv in both kinds (EA: (ac|Q) products)
    if (c->kind == ADC_EA && !c->bvv_host) narrow(c, c->Bvv, c->fBvv);
    c->mixed_ready = true;
}

}  // namespace adc

namespace adc {

// Free the reduced-precision copies (the solver calls this when it enters its
// FP64 phase, so that the FP64 particle-particle slab can use the memory);
// they are made again by the next reduced-precision sigma.
void release_mixed(adc_ctx* c) {
    drop_graphs(c);
    for (DBuf<float>* b : {&c->fBoo, &c->fBov, &c->fBvo, &c->fBvv, &c->fM11, &c->fovov, &c->foovv,
                           &c->fooov, &c->foooo, &c->ft, &c->ftt, &c->fgam, &c->fOm, &c->fPi,
                           &c->eal.fG, &c->eal.fH, &c->eal.fBH, &c->eal.fttT1, &c->eal.fttT2,
                           &c->eal.ftT1, &c->eal.ftD, &c->eal.foovvT, &c->eal.ftT})
        b->release();
    for (DBuf<bf16_t>* b : {&c->hBvv, &c->eal.httT1, &c->eal.httT2, &c->eal.htT1, &c->eal.htD,
                            &c->eal.hoovvT, &c->eal.htT, &c->eal.hovov})
        b->release();
    c->mixed_ready = false;
    c->big_mixed = false;
    c->eal.ready_mixed = false;
    c->eal.ready_f32 = false;
    c->E.scratch.erase(30);   // the slab is sized again from the free memory
}

}  // namespace adc
