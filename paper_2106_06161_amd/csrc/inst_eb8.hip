// Shuffle kernels for 8-byte records.
#include "shuffle_impl.h"

namespace bsd {
SingleFn pick_single_8(bool odd, bool wide, const LaunchConfig& c) { return pick_single_eb<8>(odd, wide, c); }
BatchFn pick_batch_8(const LaunchConfig& c) { return pick_batch_eb<8>(c); }
}  // namespace bsd
