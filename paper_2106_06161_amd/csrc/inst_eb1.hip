// Shuffle kernels for 1-byte records.
#include "shuffle_impl.h"

namespace bsd {
SingleFn pick_single_1(bool odd, bool wide, const LaunchConfig& c) { return pick_single_eb<1>(odd, wide, c); }
BatchFn pick_batch_1(const LaunchConfig& c) { return pick_batch_eb<1>(c); }
BatchFn pick_batch_small_1() { return pick_batch_small_eb<1>(); }
SingleFn pick_variant_1(uint32_t variant, bool odd, bool wide) {
  switch (variant) {
    case kVarScatter: return pick_variant_eb<1, kScatter, true, kBijPhilox>(odd, wide);
    case kVarTwoPass: return pick_variant_eb<1, kGather, false, kBijPhilox>(odd, wide);
    case kVarLcg: return pick_variant_eb<1, kGather, true, kBijLcg>(odd, wide);
    default: return nullptr;
  }
}
}  // namespace bsd
