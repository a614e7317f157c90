// Pair stage on the matrix cores: BF16 spectra, BF16 operands.
#include "pair_mfma_launch.hpp"

namespace fcc {

hipError_t launch_pair_mfma_bf16_native(const PairArgs& a) {
  return pair_mfma_detail::launch2<SpecBF16, pair_core::OpBF16>(a);
}

}  // namespace fcc
