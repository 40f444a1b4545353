// BF16 (and FP32 operands rounded to BF16) instantiations of the matrix-core GEMM (kernel in mfma_gemm_impl.hpp).
#include "mfma_gemm_impl.hpp"

namespace adc {

#define ADC_INST(TI, T, TO)                                                                    \
    template void mfma_gemm<TI, T, TO>(hipStream_t, bool, bool, long long, long long, long long, \
                                       AccOf<T>::type, const TI*, long long, long long, const TI*, \
                                       long long, long long, AccOf<T>::type, TO*, GemmOut,       \
                                       long long, int, int, GemmInner);
ADC_INST(float, bf16_t, float)
ADC_INST(bf16_t, bf16_t, float)
ADC_INST(bf16_t, bf16_t, bf16_t)
ADC_INST(float, bf16_t, bf16_t)
#undef ADC_INST

template <>
int gemm_candidates<bf16_t>(int* ids) {
    static const int c[] = {0, 1, 6, 7, 8};
    for (int k = 0; k < 5; ++k) ids[k] = c[k];
    return 5;
}

}  // namespace adc
