// Pair stage on the matrix cores: e4m3 spectra, e4m3 operands.
#include "pair_mfma_launch.hpp"

namespace fcc {

hipError_t launch_pair_mfma_e4m3_native(const PairArgs& a) {
  return pair_mfma_detail::launch2<SpecE4M3, pair_core::OpF8>(a);
}

}  // namespace fcc
