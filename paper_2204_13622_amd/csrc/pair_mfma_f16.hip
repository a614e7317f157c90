// Pair stage on the matrix cores: FP16 spectra, FP16 operands.
#include "pair_mfma_launch.hpp"

namespace fcc {

hipError_t launch_pair_mfma_f16(const PairArgs& a) {
  return pair_mfma_detail::launch2<SpecF16, pair_core::OpF16>(a);
}

}  // namespace fcc
