// The particle-particle term rebuilt from the density-fitted factors (the
// four-virtual integrals are never stored whole, Sec. III.C):
//   out[x][a][b] = sum_cd (ac|bd) in[x][c][d],   (ac|bd) = sum_Q B^Q_ac B^Q_bd.
// It is the 2p1h-2p1h first-order ladder of EA sigma (x = vector, occupied
// index) and the particle-particle ladder of the second-order doubles (x = ij).
//
// (ac|bd) = (bd|ac), so for a block A = [a0, a0+na) only the columns b >= a0
// are rebuilt: one matrix-core GEMM over Q,
//   rows (a, c) of B_vv (a in A)  x  rows (b, d) of B_vv (b >= a0),
// whose epilogue scatters the result into a slab K[a-s0][b-s0][c][d] shared by
// a group of consecutive blocks starting at s0.  The slab then serves the
// direct and the mirrored pairs in one GEMM per group, contiguous in the
// summed pair, over the stacked inputs [in; inT] (inT[x][c][d] = in[x][d][c]):
//   D[x][a][b] = sum_(cd) in[x][(c,d)]  K[a][b][(c,d)]          (b >= s0)
//   T[x][a][b] = sum_(cd) inT[x][(c,d)] K[a][b][(c,d)] = out[x][b][a]
// and out takes D where b lies at or past the first a of a's block, else the
// mirror T[x][b][a] written by the group of b (the pairs b in [s0, a0) of a
// group's later blocks are multiplied but never rebuilt nor used).  The
// rebuild of a block costs 2 Naux na V^2 (V - a0) flops, Naux V^3 (V + na)
// over all blocks of size na instead of 2 Naux V^4; the contraction
// 2 nx V^4 plus the unused pairs of the groups.
#include "context.hpp"

#include <algorithm>

namespace adc {

// out[x][p][q] from the two halves of the per-block products: D[x][p][q]
// (direct) where q lies at or past the first a of p's block, else the
// mirror T[x][q][p] (written when q's block was processed, as p >= q's first
// a).  32x32 tiles of (p, q); the mirror tile is read transposed through LDS.
template <typename TO>
__global__ void k_pp_assemble(const TO* __restrict__ D, const TO* __restrict__ T,
                              TO* __restrict__ out, int V, int ta, int nt) {
    __shared__ TO tile[32][33];
    const int p0 = (blockIdx.x / nt) * 32, q0 = (blockIdx.x % nt) * 32;
    const long long x = blockIdx.y;
    const long long VV = (long long)V * V;
    const TO* Dx = D + x * VV;
    const TO* Tx = T + x * VV;
    TO* ox = out + x * VV;
    const int tx = threadIdx.x, ty = threadIdx.y;   // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int q = q0 + r, p = p0 + tx;
        tile[r][tx] = (q < V && p < V) ? Tx[(long long)q * V + p] : TO(0);   // T[q][p]
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int p = p0 + r, q = q0 + tx;
        if (p >= V || q >= V) continue;
        const long long o = (long long)p * V + q;
        ox[o] = (q >= (p / ta) * ta) ? Dx[o] : tile[tx][r];
    }
}

// Pair-symmetric inputs, in[(i,j)][c][d] = in[(j,i)][d][c] (x = i np + j):
// then out[(i,j)][p][q] = out[(j,i)][q][p], so the mirrored products are rows
// of the direct ones.  Only the direct results (q at or past the first a of
// p's block) are computed; this kernel fills the rest of out in place from
// them (it reads only direct entries and writes only the others).
template <typename TO>
__global__ void k_pp_mirror(TO* __restrict__ out, int V, int ta, int np, int nt) {
    __shared__ TO tile[32][33];
    const int p0 = (blockIdx.x / nt) * 32, q0 = (blockIdx.x % nt) * 32;
    const int plast = min(p0 + 31, V - 1);
    if ((plast / ta) * ta <= q0) return;           // the whole tile is direct
    const long long x = blockIdx.y;
    const long long i = x / np, j = x - i * np, xs = j * np + i;
    const long long VV = (long long)V * V;
    const TO* src = out + xs * VV;
    TO* dst = out + x * VV;
    const int tx = threadIdx.x, ty = threadIdx.y;   // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int q = q0 + r, p = p0 + tx;
        const bool need = p < V && q < V && q < (p / ta) * ta;
        tile[r][tx] = need ? src[(long long)q * V + p] : TO(0);   // out[xs][q][p]
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int p = p0 + r, q = q0 + tx;
        if (p < V && q < V && q < (p / ta) * ta) dst[(long long)p * V + q] = tile[tx][r];
    }
}

template <typename T, typename TO>
void vvvv_apply(adc_ctx* c, const T* Bvv, const T* in, TO* out, long long nx, int npair) {
    Engine& E = c->E;
    const long long V = c->V, Q = c->Q, VV = V * V, V3 = VV * V;
    if (nx <= 0) return;
    // slab bound: the option, or by default the larger of 16 GiB and a third of
    // the device memory free for it (at most 64 GiB) -- large V needs room for
    // several values of a per group (V^3 elements each)
    long long slab_bytes = c->pp_slab_bytes;
    if (!c->pp_slab_set) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        ADC_HIP(hipStreamIsCapturing(E.stream, &cs));
        if (cs == hipStreamCaptureStatusNone) {
            size_t fr = 0, tot = 0;
            if (hipMemGetInfo(&fr, &tot) == hipSuccess) {
                const long long have = (long long)fr + E.scratch.size_of(30);
                c->pp_slab_auto = std::max<long long>(16LL << 30, std::min<long long>(64LL << 30, have / 3));
            } else {
                (void)hipGetLastError();
            }
        }
        if (c->pp_slab_auto > 0) slab_bytes = c->pp_slab_auto;
    }
    long long ta_max = std::max<long long>(1, slab_bytes / (long long)(sizeof(T) * V3));
    ta_max = std::min(ta_max, V);
    // more blocks rebuild fewer mirrored pairs (Naux V^3 (V + na) flops) but
    // make smaller rebuild products: at least pp_blocks of them (default 24
    // blocks of at least 8 values of a in FP64 and FP32, whose products run
    // near the matrix-core peak at any size; 12 in BF16, whose short-K
    // rebuild is bound by its stores)
    const long long want = c->pp_blocks > 0 ? c->pp_blocks
                                            : std::min<long long>(sizeof(T) == 2 ? 12 : 24, V / 8);
    const long long nblk = std::min(V, std::max((V + ta_max - 1) / ta_max, want));
    const long long ta = (V + nblk - 1) / nblk;            // balanced a-blocks
    // the contraction runs per group of up to pp_group consecutive blocks
    // (default 8) sharing one slab [a - s0][b - s0][c][d] (b >= s0): larger
    // products, at the price of the pairs b in [s0, a0) of the group's later
    // blocks, which are never rebuilt and whose results are never used
    const long long grp = std::max<long long>(
        1, std::min<long long>(c->pp_group > 0 ? c->pp_group : 8, ta_max / ta));
    const long long ts = std::min(V, grp * ta);
    T* K = (T*)E.scratch.get(30, sizeof(T) * ts * V3);
    // several blocks: the inputs stacked as [in; inT] (inT[x][c][d] = in[x][d][c])
    // so that one product per group serves the direct and the mirrored pairs,
    // reading the slab once; its results D (rows 0..nx-1) and T (rows nx..)
    // are assembled into out at the end.  Pair-symmetric inputs need only D,
    // written straight into out and mirrored there.
    ADC_REQUIRE(npair == 0 || (long long)npair * npair == nx, "particle-particle term: pair count");
    const bool sym = npair > 0 && nblk > 1;
    T* AB = nullptr;
    TO* DT = nullptr;
    if (nblk > 1 && !sym) {
        AB = (T*)E.scratch.get(29, sizeof(T) * 2 * nx * VV);
        ADC_HIP(hipMemcpyAsync(AB, in, sizeof(T) * nx * VV, hipMemcpyDeviceToDevice, E.stream));
        pair_transform<T, T>(E, in, nx * VV, 0, AB + nx * VV, nx * VV, 0, 1, nx, (int)V, 0.0, 1.0,
                             0.0);
        DT = (TO*)E.scratch.get(27, sizeof(TO) * 2 * nx * VV);
    }
    using A = typename AccOf<T>::type;
    for (long long s0 = 0; s0 < V; s0 += ts) {
        c->phase("particle-particle term: group starting at virtual", s0, V);
        const long long ns = std::min(ts, V - s0), nbs = V - s0;
        for (long long a0 = s0; a0 < s0 + ns; a0 += ta) {
            const long long na = std::min(ta, s0 + ns - a0), nb = V - a0;
            GemmOut slab;                                  // (a, c) x (b, d) -> [a][b-s0][c][d]
            slab.rsplit = V;
            slab.rs1 = nbs * VV;
            slab.rs2 = V;
            slab.csplit = V;
            slab.cs1 = VV;
            slab.cs2 = 1;
            if (Bvv) {
                const T* Ba = Bvv + a0 * V * Q;
                gemm_run<T, T, T>(E, false, true, na * V, nb * V, Q, A(1), Ba, Q, 0, Ba, Q, 0,
                                  A(0), K + ((a0 - s0) * nbs + (a0 - s0)) * VV, slab, 1, 1);
            } else {
                // B_vv in host memory: rows (a, c) of the block, then the columns
                // (b, d) in staged blocks of b
                const T* Ba = bvv_rows<T>(c, a0 * V, na * V, 72);
                const long long nbc = std::max<long long>(1, bvv_chunk_rows(c, sizeof(T)) / V);
                for (long long b0 = a0; b0 < V; b0 += nbc) {
                    const long long nbb = std::min(nbc, V - b0);
                    const T* Bb = bvv_rows<T>(c, b0 * V, nbb * V, 73);
                    gemm_run<T, T, T>(E, false, true, na * V, nbb * V, Q, A(1), Ba, Q, 0, Bb, Q, 0,
                                      A(0), K + ((a0 - s0) * nbs + (b0 - s0)) * VV, slab, 1, 1);
                }
            }
            E.gemm_flops += 2LL * na * V * nb * V * Q;
        }
        GemmOut pairs;                                     // x x (a, b-s0) -> [x][a][b]
        pairs.rs2 = VV;
        pairs.csplit = nbs;
        pairs.cs1 = V;
        pairs.cs2 = 1;
        if (nblk > 1 && !sym)
            gemm_acc<T, T>(E, false, true, 2 * nx, ns * nbs, VV, A(1), AB, VV, K, VV, A(0),
                           DT + s0 * V + s0, pairs, 2);
        else
            gemm_acc<T, T>(E, false, true, nx, ns * nbs, VV, A(1), in, VV, K, VV, A(0),
                           out + s0 * V + s0, pairs, 2);
        E.gemm_flops += 2LL * (nblk > 1 && !sym ? 2 : 1) * nx * ns * nbs * VV;
    }
    if (sym) {
        const int nt = (int)((V + 31) / 32);
        ADC_REQUIRE(nx <= 65535, "particle-particle term: too many rows");
        hipLaunchKernelGGL(k_pp_mirror<TO>, dim3((unsigned)(nt * nt), (unsigned)nx), dim3(32, 8),
                           0, E.stream, out, (int)V, (int)ta, npair, nt);
        ADC_HIP(hipGetLastError());
    } else if (nblk > 1) {
        const int nt = (int)((V + 31) / 32);
        ADC_REQUIRE(nx <= 65535, "particle-particle term: too many rows");
        hipLaunchKernelGGL(k_pp_assemble<TO>, dim3((unsigned)(nt * nt), (unsigned)nx),
                           dim3(32, 8), 0, E.stream, DT, DT + nx * VV, out, (int)V, (int)ta, nt);
        ADC_HIP(hipGetLastError());
    }
}

template void vvvv_apply<double, double>(adc_ctx*, const double*, const double*, double*,
                                         long long, int);
template void vvvv_apply<bf16_t, float>(adc_ctx*, const bf16_t*, const bf16_t*, float*, long long,
                                        int);
template void vvvv_apply<float, float>(adc_ctx*, const float*, const float*, float*, long long,
                                       int);

}  // namespace adc
