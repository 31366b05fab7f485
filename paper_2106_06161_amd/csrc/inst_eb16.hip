// Shuffle kernels for 16-byte records.
#include "shuffle_impl.h"

namespace bsd {
SingleFn pick_single_16(bool odd, bool wide, const LaunchConfig& c) { return pick_single_eb<16>(odd, wide, c); }
BatchFn pick_batch_16(const LaunchConfig& c) { return pick_batch_eb<16>(c); }
}  // namespace bsd
