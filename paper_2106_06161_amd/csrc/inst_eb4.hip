// Shuffle kernels for 4-byte records.
#include "shuffle_impl.h"

namespace bsd {
SingleFn pick_single_4(bool odd, bool wide, const LaunchConfig& c) { return pick_single_eb<4>(odd, wide, c); }
BatchFn pick_batch_4(const LaunchConfig& c) { return pick_batch_eb<4>(c); }
BatchFn pick_batch_small_4() { return pick_batch_small_eb<4>(); }
SingleFn pick_variant_4(uint32_t variant, bool odd, bool wide) {
  switch (variant) {
    case kVarIndices: return pick_variant_eb<4, kIndices, true, kBijPhilox>(odd, wide);
    case kVarScatter: return pick_variant_eb<4, kScatter, true, kBijPhilox>(odd, wide);
    case kVarTwoPass: return pick_variant_eb<4, kGather, false, kBijPhilox>(odd, wide);
    case kVarFromTable: return pick_variant_eb<4, kIndices, true, kBijTable>(odd, wide);
    case kVarLcg: return pick_variant_eb<4, kGather, true, kBijLcg>(odd, wide);
    default: return nullptr;
  }
}
}  // namespace bsd
