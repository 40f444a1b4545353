// The first-order particle-particle term rebuilt from the DF factors:
//   out[x][a][b] = beta*out + sum_cd (ac|bd) in[x][c][d],   (ac|bd) = sum_Q B^Q_ac B^Q_bd
// used for the 2p1h-2p1h block of EA sigma (x = vector, occupied index) and for
// the particle-particle ladder of the second-order doubles (x = ij).  The
// four-index block is never stored whole (V^4 words); this routine rebuilds
// it for a block of a values at a time.
//
// Reference path (rocBLAS): for each a-block A,
//   K[a][c][d][b] = sum_Q Bvv[a][c][Q] Bvv[d][b][Q]     (Bvv symmetric in its pair)
//   out[x][a][b] += sum_(cd) in[x][(cd)] K[a][(cd)][b]   (one GEMM per a, batched)
#include "context.hpp"

#include <algorithm>

namespace adc {

template <typename T>
void vvvv_reference(adc_ctx* c, const T* Bvv, const T* in, T* out, long long nx, T beta) {
    Engine& E = c->E;
    const long long V = c->V, Q = c->Q, VV = V * V;
    // a-block size: keep the rebuilt slab near 1 GiB
    long long ta = std::max<long long>(1, (1LL << 30) / (long long)(sizeof(T) * VV * V));
    ta = std::min(ta, V);
    T* K = (T*)E.scratch.get(30, sizeof(T) * ta * VV * V);
    for (long long a0 = 0; a0 < V; a0 += ta) {
        long long na = std::min(ta, V - a0);
        // K[(a,c)][(d,b)] = Bvv[(a,c)][Q] . Bvv[(d,b)][Q]^T
        gemm_rm<T>(E, false, true, na * V, VV, Q, T(1), Bvv + a0 * V * Q, Q, 0, Bvv, Q, 0, T(0), K,
                   VV, 0, 1);
        // out[x][a][b] for a in block: batch over a, C stride V, ldc V^2
        gemm_rm<T>(E, false, false, nx, V, VV, T(1), in, VV, 0, K, V, VV * V, beta, out + a0 * V,
                   VV, V, na);
    }
}

template void vvvv_reference<double>(adc_ctx*, const double*, const double*, double*, long long,
                                     double);
template void vvvv_reference<float>(adc_ctx*, const float*, const float*, float*, long long, float);

}  // namespace adc
