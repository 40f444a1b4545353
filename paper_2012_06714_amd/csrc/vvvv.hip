// The particle-particle term rebuilt from the density-fitted factors (the
// four-virtual integrals are never stored whole, Sec. III.C):
//   out[x][a][b] = sum_cd (ac|bd) in[x][c][d],   (ac|bd) = sum_Q B^Q_ac B^Q_bd.
// It is the 2p1h-2p1h first-order ladder of EA sigma (x = vector, occupied
// index) and the particle-particle ladder of the second-order doubles (x = ij).
//
// (ac|bd) = (bd|ac), so for a block A = [a0, a0+na) only the columns b >= a0
// are rebuilt: one matrix-core GEMM over Q,
//   rows (a, c) of B_vv (a in A)  x  rows (b, d) of B_vv (b >= a0),
// whose epilogue scatters the result into the slab K[a][b][c][d].  The slab
// then serves two contractions, both GEMMs contiguous in the summed pair:
//   out[x][a][b] = sum_(cd) in[x][(c,d)]  K[a][b][(c,d)]          (b >= a0)
//   out[x][b][a] = sum_(cd) inT[x][(c,d)] K[a][b][(c,d)]          (b >= a0 + na)
// where inT[x][c][d] = in[x][d][c]; pairs with b < a0 were produced as mirrors
// by earlier blocks.  The rebuild costs Naux V^3 (V + na) flops instead of
// 2 Naux V^4, the contraction 2 nx V^4 as before.
#include "context.hpp"

#include <algorithm>

namespace adc {

template <typename T, typename TO>
void vvvv_apply(adc_ctx* c, const T* Bvv, const T* in, TO* out, long long nx) {
    Engine& E = c->E;
    const long long V = c->V, Q = c->Q, VV = V * V, V3 = VV * V;
    if (nx <= 0) return;
    long long ta_max = std::max<long long>(1, c->pp_slab_bytes / (long long)(sizeof(T) * V3));
    ta_max = std::min(ta_max, V);
    const long long nblk = (V + ta_max - 1) / ta_max;
    const long long ta = (V + nblk - 1) / nblk;            // balanced a-blocks
    T* K = (T*)E.scratch.get(30, sizeof(T) * ta * V3);
    T* inT = nblk > 1 ? (T*)E.scratch.get(29, sizeof(T) * nx * VV) : nullptr;
    if (inT) pair_transform<T, T>(E, in, nx * VV, 0, inT, nx * VV, 0, 1, nx, (int)V, 0.0, 1.0, 0.0);
    using A = typename AccOf<T>::type;
    for (long long a0 = 0; a0 < V; a0 += ta) {
        const long long na = std::min(ta, V - a0), nb = V - a0;
        GemmOut slab;                                      // (a, c) x (b, d) -> [a][b-a0][c][d]
        slab.rsplit = V;
        slab.rs1 = nb * VV;
        slab.rs2 = V;
        slab.csplit = V;
        slab.cs1 = VV;
        slab.cs2 = 1;
        const T* Ba = Bvv + a0 * V * Q;
        gemm_run<T, T, T>(E, false, true, na * V, nb * V, Q, A(1), Ba, Q, 0, Ba, Q, 0, A(0),
                           K, slab, 1, 1);
        GemmOut direct;                                    // x x (a, b-a0) -> out[x][a][b]
        direct.rs2 = VV;
        direct.csplit = nb;
        direct.cs1 = V;
        direct.cs2 = 1;
        gemm_run<T, T, TO>(E, false, true, nx, na * nb, VV, A(1), in, VV, 0, K, VV, 0, A(0),
                            out + a0 * V + a0, direct, 1, 2);
        E.gemm_flops += 2LL * na * V * nb * V * Q + 2LL * nx * na * nb * VV;
        if (nb > na) {
            // mirrors: one GEMM per a, columns b = a0+na .. V-1 -> out[x][b][a]
            GemmOut mirror;
            mirror.rs2 = VV;
            mirror.cs2 = V;
            mirror.sC = 1;
            gemm_run<T, T, TO>(E, false, true, nx, nb - na, VV, A(1), inT, VV, 0,
                                K + na * VV, VV, nb * VV, A(0), out + (a0 + na) * V + a0, mirror,
                                na, 2);
            E.gemm_flops += 2LL * nx * na * (nb - na) * VV;
        }
    }
}

template void vvvv_apply<double, double>(adc_ctx*, const double*, const double*, double*,
                                         long long);
template void vvvv_apply<bf16_t, float>(adc_ctx*, const bf16_t*, const bf16_t*, float*, long long);

}  // namespace adc
