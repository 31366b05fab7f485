// Shuffle kernels for 16-byte records.
#include "shuffle_impl.h"

namespace bsd {
SingleFn pick_single_16(bool odd, bool wide, const LaunchConfig& c) { return pick_single_eb<16>(odd, wide, c); }
BatchFn pick_batch_16(const LaunchConfig& c) { return pick_batch_eb<16>(c); }
BatchFn pick_batch_small_16() { return pick_batch_small_eb<16>(); }
SingleFn pick_variant_16(uint32_t variant, bool odd, bool wide) {
  switch (variant) {
    case kVarScatter: return pick_variant_eb<16, kScatter, true, kBijPhilox>(odd, wide);
    case kVarTwoPass: return pick_variant_eb<16, kGather, false, kBijPhilox>(odd, wide);
    case kVarLcg: return pick_variant_eb<16, kGather, true, kBijLcg>(odd, wide);
    default: return nullptr;
  }
}
}  // namespace bsd
