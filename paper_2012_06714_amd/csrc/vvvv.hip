// The particle-particle term rebuilt from the density-fitted factors (the
// four-virtual integrals are never stored whole, Sec. III.C):
//   out[x][a][b] = sum_cd (ac|bd) in[x][c][d],   (ac|bd) = sum_Q B^Q_ac B^Q_bd.
// It is the 2p1h-2p1h first-order ladder of EA sigma (x = vector, occupied
// index) and the particle-particle ladder of the second-order doubles (x = ij).
//
// For a block of a values the rebuild is one matrix-core GEMM over Q,
//   rows (a, c) of B_vv  x  rows (b, d) of B_vv,
// whose epilogue scatters the result into the slab K[a][b][c][d]; the
// contraction is then a second GEMM, out[x][(a,b)] = in[x][(c,d)] K[(a,b)][(c,d)],
// with both operands contiguous in the summed pair (c, d).  The slab is the
// only V^3-sized buffer; its size bounds the a-block.
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
    GemmOut slab;                                          // (a, c) x (b, d) -> [a][b][c][d]
    slab.rsplit = V;
    slab.rs1 = V3;
    slab.rs2 = V;
    slab.csplit = V;
    slab.cs1 = VV;
    slab.cs2 = 1;
    using A = typename AccOf<T>::type;
    for (long long a0 = 0; a0 < V; a0 += ta) {
        const long long na = std::min(ta, V - a0);
        mfma_gemm<T, T, T>(E.stream, false, true, na * V, VV, Q, A(1), Bvv + a0 * V * Q, Q, 0, Bvv,
                           Q, 0, A(0), K, slab, 1, 1);
        mfma_gemm<T, T, TO>(E.stream, false, true, nx, na * V, VV, A(1), in, VV, 0, K, VV, 0, A(0),
                            out + a0 * V, GemmOut::rowmajor(VV), 1, 2);
        E.gemm_flops += 2LL * na * V * VV * Q + 2LL * nx * na * V * VV;
    }
}

template void vvvv_apply<double, double>(adc_ctx*, const double*, const double*, double*,
                                         long long);
template void vvvv_apply<bf16_t, float>(adc_ctx*, const bf16_t*, const bf16_t*, float*, long long);

}  // namespace adc
