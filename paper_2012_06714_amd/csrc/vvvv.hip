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
//   out[x][b][a] = sum_(cd) inT[x][(c,d)] K[a][b][(c,d)]          (b >= a0)
// where inT[x][c][d] = in[x][d][c]; pairs with b < a0 were produced as mirrors
// by earlier blocks, and pairs with both a and b in the block are written by
// both products (the same value).  The rebuild of a block costs 2 Naux na V^2 (V - a0)
// flops, Naux V^3 (V + na) over all blocks of size na instead of 2 Naux V^4;
// the contraction 2 nx V^4 as before.
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
    // more blocks rebuild fewer mirrored pairs (Naux V^3 (V + na) flops) but
    // make smaller products: at least pp_blocks of them (default: FP64, whose
    // products run near the matrix-core peak at any size, 12 blocks of at
    // least 8 values of a; BF16, whose short-K rebuild is bound by its
    // stores, as few as the slab allows)
    const long long want = c->pp_blocks > 0 ? c->pp_blocks
                           : sizeof(T) == 8 ? std::min<long long>(12, V / 8)
                                            : 1;
    const long long nblk = std::min(V, std::max((V + ta_max - 1) / ta_max, want));
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
        gemm_acc<T, T>(E, false, true, nx, na * nb, VV, A(1), in, VV, K, VV, A(0),
                       out + a0 * V + a0, direct, 2);
        E.gemm_flops += 2LL * na * V * nb * V * Q + 2LL * nx * na * nb * VV;
        if (nb > na) {
            // mirrors out[x][b][a] = sum_(cd) inT[x][(c,d)] K[a][b][(c,d)] as one product
            // over all columns (a, b >= a0): the pairs with b inside the block repeat
            // direct results of the same value, which costs na/nb of the product but
            // keeps every operand row contiguous
            GemmOut mirror;                                // x x (a, b-a0) -> out[x][b][a]
            mirror.rs2 = VV;
            mirror.csplit = nb;
            mirror.cs1 = 1;
            mirror.cs2 = V;
            gemm_acc<T, T>(E, false, true, nx, na * nb, VV, A(1), inT, VV, K, VV, A(0),
                           out + a0 * V + a0, mirror, 2);
            E.gemm_flops += 2LL * nx * na * nb * VV;
        }
    }
}

template void vvvv_apply<double, double>(adc_ctx*, const double*, const double*, double*,
                                         long long);
template void vvvv_apply<bf16_t, float>(adc_ctx*, const bf16_t*, const bf16_t*, float*, long long);
template void vvvv_apply<float, float>(adc_ctx*, const float*, const float*, float*, long long);

}  // namespace adc
