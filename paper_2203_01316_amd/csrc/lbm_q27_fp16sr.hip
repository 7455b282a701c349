// Kernels of lbm_impl.hpp for D3Q27 with fp16sr storage (one translation unit
// per lattice and storage, so the build compiles them in parallel).
#include "lbm_impl.hpp"

namespace lbm {
LBM_INSTANTIATE(27, ST_FP16_SR, q27_fp16sr)
}  // namespace lbm
