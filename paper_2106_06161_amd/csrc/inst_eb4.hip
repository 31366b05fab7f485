// Shuffle kernels for 4-byte records.
#include "shuffle_impl.h"

namespace bsd {
SingleFn pick_single_4(bool odd, bool wide, const LaunchConfig& c) { return pick_single_eb<4>(odd, wide, c); }
BatchFn pick_batch_4(const LaunchConfig& c) { return pick_batch_eb<4>(c); }
}  // namespace bsd
