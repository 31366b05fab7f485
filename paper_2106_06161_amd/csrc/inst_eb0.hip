// Shuffle kernels for 0-byte records (no payload: cipher and scan only).
#include "shuffle_impl.h"

namespace bsd {
SingleFn pick_single_0(bool odd, bool wide, const LaunchConfig& c) { return pick_single_eb<0>(odd, wide, c); }
BatchFn pick_batch_0(const LaunchConfig&) { return nullptr; }
SingleFn pick_variant_0(uint32_t, bool, bool) { return nullptr; }
}  // namespace bsd
