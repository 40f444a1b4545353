// Host-side tuning state of the matrix-core GEMM (kernels and instantiations
// in mfma_gemm_impl.hpp and mfma_gemm_{f64,f32,bf16}.hip).
#include "mfma_gemm.hpp"

namespace adc {

int g_force_cfg = -1;

void gemm_force_config(int cfg) { g_force_cfg = cfg; }

// Tile configurations: (BM, BN, waves in M, waves in N).
//   0: 64x64 (4x1)    1: 128x128 (2x2)   2: 128x128 (4x2)   3: 128x64 (2x2)
//   4: 256x128 (2x2)  5: 256x256 (2x2)   6: 256x128 (4x2)   7: 256x256 (4x2)
//   8: 256x256 (4x2) with operands loaded straight into LDS (BF16)
int gemm_tile_dims(int cfg, int* bm, int* bn) {
    static const int dims[9][2] = {{64, 64},   {128, 128}, {128, 128}, {128, 64},  {256, 128},
                                   {256, 256}, {256, 128}, {256, 256}, {256, 256}};
    if (cfg < 0 || cfg > 8) return -1;
    *bm = dims[cfg][0];
    *bn = dims[cfg][1];
    return 0;
}

}  // namespace adc
