// Pair stage on the matrix cores, single array: shape checks and dispatch to
// the (storage, operand) combinations, each built in its own translation unit.
#include "pair_mfma_launch.hpp"

namespace fcc {

using pair_mfma_detail::block_waves;
using pair_mfma_detail::native_operands;

bool pair_mfma_supported(const PairArgs& a) {
  const int kb = a.Dpad / 4;
  const bool kb_ok = a.Dpad % 4 == 0 && (kb == 1 || kb == 2 || kb == 3 || kb == 4 || kb == 6 || kb == 8);
  return a.method == FCC_METHOD_FCC && a.precision != FCC_FP32 && a.M <= 16 && a.N >= 32 &&
         (reinterpret_cast<uintptr_t>(a.spec) % 16) == 0 &&
         a.D <= a.Dpad && kb_ok && a.I <= 48 && block_waves(a) > 0 &&
         (!native_operands(a) || (a.prow_op != nullptr && a.gexp_op != nullptr));
}

hipError_t launch_pair_mfma(const PairArgs& a) {
  if (a.T == 0) return hipSuccess;
  if (!pair_mfma_supported(a)) return hipErrorInvalidValue;
  switch (a.precision) {
    case FCC_FP16: return launch_pair_mfma_f16(a);
    case FCC_BF16: return native_operands(a) ? launch_pair_mfma_bf16_native(a) : launch_pair_mfma_bf16(a);
    case FCC_FP8_E4M3: return native_operands(a) ? launch_pair_mfma_e4m3_native(a) : launch_pair_mfma_e4m3(a);
    default: break;
  }
  return hipErrorInvalidValue;
}

}  // namespace fcc
