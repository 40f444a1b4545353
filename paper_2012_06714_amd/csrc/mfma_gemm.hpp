// Matrix-core GEMM (mfma_gemm.hip): row-major, strided batches, permuted output.
#pragma once

#include "adc_internal.hpp"

namespace adc {

using bf16_t = __bf16;

// accumulation / scaling type of each input type
template <typename T> struct AccOf { using type = T; };
template <> struct AccOf<bf16_t> { using type = float; };

// Output index map.  Row m = m1*rsplit + m2, column n = n1*csplit + n2:
//   offset = m1*rs1 + m2*rs2 + n1*cs1 + n2*cs2 + batch*sC
// The plain row-major store with leading dimension ldc is
//   rsplit = csplit = 0 (no split), rs2 = ldc, cs2 = 1.
struct GemmOut {
    long long rsplit = 0, rs1 = 0, rs2 = 0;
    long long csplit = 0, cs1 = 0, cs2 = 1;
    long long sC = 0;
    static GemmOut rowmajor(long long ldc, long long sC = 0) {
        GemmOut o;
        o.rs2 = ldc;
        o.sC = sC;
        return o;
    }
};

// Two-level batches: batch index z = z1 * n + z2 (z2 fastest, z < batch * n);
// the operands and the result advance by the outer strides (sA, sB, sC) per z1
// and by these inner strides per z2.  Split-K runs its k-chunks as the inner
// level.
struct GemmInner {
    long long n = 1, sA = 0, sB = 0, sC = 0;
};

struct GemmShape {
    long long M, N, K, lda, ldb, sA, sB, sC;
    long long rsplit, rs1, rs2, csplit, cs1, cs2;
    long long n2, sA2, sB2, sC2, z0;
    bool vecA, vecB;
};

// C = alpha op(A) op(B) + beta C on stream st.
//   ta = false: A is [M][K] (lda >= K);  ta = true: A is [K][M] (lda >= M)
//   tb = true:  B is [N][K] (ldb >= K);  tb = false: B is [K][N] (ldb >= N)
// Operands stored as TI, multiplied as T on the matrix cores (TI = FP32 with
// T = BF16 rounds while staging), accumulated in AccOf<T>, written as TO.
// Instantiated for (TI, T, TO) = (f64, f64, f64), (f32, f32, f32),
// (f32, bf16, f32), (bf16, bf16, f32), (bf16, bf16, bf16).
template <typename TI, typename T, typename TO>
void mfma_gemm(hipStream_t st, bool ta, bool tb, long long M, long long N, long long K,
               typename AccOf<T>::type alpha, const TI* A, long long lda, long long sA, const TI* B,
               long long ldb, long long sB, typename AccOf<T>::type beta, TO* C, GemmOut out,
               long long batch, int kind = 0, int cfg = -1, GemmInner inner = GemmInner());

// Tile configurations compiled for compute type T (ids as in gemm_tile_dims);
// returns the count written to ids[] (at most 8).
template <typename T> int gemm_candidates(int* ids);

// mfma_gemm with the tile configuration chosen by the autotuner (tensor.hip):
// the first call of each shape times every candidate configuration on the
// stream (in place when beta = 0, else on a scratch output) and caches the
// fastest; later calls of the shape use it.
template <typename TI, typename T, typename TO>
void gemm_run(Engine& E, bool ta, bool tb, long long M, long long N, long long K,
              typename AccOf<T>::type alpha, const TI* A, long long lda, long long sA,
              const TI* B, long long ldb, long long sB, typename AccOf<T>::type beta, TO* C,
              GemmOut out, long long batch, int kind = 0, GemmInner inner = GemmInner());
// kind only names the kernel in profiles: 0 plain, 1 four-index rebuild,
// 2 particle-particle contraction (1 and 2 are NT only)

// One product C = alpha op(A) op(B) + beta C through the output index map
// `out`, no batch.  The compute type follows the storage type TI: FP64, BF16,
// or FP32 (multiplied in BF16 while the engine's mixed flag is set).  An
// output in the accumulator type goes through split-K when the grid would be
// small (partial products reduced in a fixed order, then stored through the
// map).  Instantiated for (TI, TO) = (f64, f64), (f32, f32),
// (f32, bf16), (bf16, f32), (bf16, bf16).
template <typename TI, typename TO>
void gemm_map(Engine& E, bool ta, bool tb, long long M, long long N, long long K, double alpha,
              const TI* A, long long lda, const TI* B, long long ldb, double beta, TO* C,
              GemmOut out);

// The same for compute type T with the output in its accumulator type,
// tagged with a profile kind (split-K keeps the tag).  Instantiated for
// (TI, T) = (f64, f64), (bf16, bf16), (f32, f32).
template <typename TI, typename T>
void gemm_acc(Engine& E, bool ta, bool tb, long long M, long long N, long long K,
              typename AccOf<T>::type alpha, const TI* A, long long lda, const TI* B, long long ldb,
              typename AccOf<T>::type beta, typename AccOf<T>::type* C, GemmOut out, int kind);

// Tile configuration override for tuning (-1: automatic choice per shape) and
// the tile of a configuration id; returns -1 for an unknown id.
void gemm_force_config(int cfg);
int gemm_tile_dims(int cfg, int* bm, int* bn);

}  // namespace adc
