// Shuffle kernels for 8-byte records.
#include "shuffle_impl.h"

namespace bsd {
SingleFn pick_single_8(bool odd, bool wide, const LaunchConfig& c) { return pick_single_eb<8>(odd, wide, c); }
BatchFn pick_batch_8(const LaunchConfig& c) { return pick_batch_eb<8>(c); }
BatchFn pick_batch_small_8() { return pick_batch_small_eb<8>(); }
SingleFn pick_variant_8(uint32_t variant, bool odd, bool wide) {
  switch (variant) {
    case kVarIndices: return pick_variant_eb<8, kIndices, true, kBijPhilox>(odd, wide);
    case kVarScatter: return pick_variant_eb<8, kScatter, true, kBijPhilox>(odd, wide);
    case kVarTwoPass: return pick_variant_eb<8, kGather, false, kBijPhilox>(odd, wide);
    case kVarLcg: return pick_variant_eb<8, kGather, true, kBijLcg>(odd, wide);
    default: return nullptr;
  }
}
}  // namespace bsd
