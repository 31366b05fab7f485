// Shuffle kernels for 2-byte records.
#include "shuffle_impl.h"

namespace bsd {
SingleFn pick_single_2(bool odd, bool wide, const LaunchConfig& c) { return pick_single_eb<2>(odd, wide, c); }
BatchFn pick_batch_2(const LaunchConfig& c) { return pick_batch_eb<2>(c); }
BatchFn pick_batch_small_2() { return pick_batch_small_eb<2>(); }
SingleFn pick_variant_2(uint32_t variant, bool odd, bool wide) {
  switch (variant) {
    case kVarScatter: return pick_variant_eb<2, kScatter, true, kBijPhilox>(odd, wide);
    case kVarTwoPass: return pick_variant_eb<2, kGather, false, kBijPhilox>(odd, wide);
    case kVarLcg: return pick_variant_eb<2, kGather, true, kBijLcg>(odd, wide);
    default: return nullptr;
  }
}
}  // namespace bsd
