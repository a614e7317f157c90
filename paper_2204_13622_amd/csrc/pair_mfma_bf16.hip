// Pair stage on the matrix cores: BF16 spectra widened to FP16 operands.
#include "pair_mfma_launch.hpp"

namespace fcc {

hipError_t launch_pair_mfma_bf16(const PairArgs& a) {
  return pair_mfma_detail::launch2<SpecBF16, pair_core::OpF16>(a);
}

}  // namespace fcc
