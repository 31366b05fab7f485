// Shuffle kernels for 2-byte records.
#include "shuffle_impl.h"

namespace bsd {
SingleFn pick_single_2(bool odd, bool wide, const LaunchConfig& c) { return pick_single_eb<2>(odd, wide, c); }
BatchFn pick_batch_2(const LaunchConfig& c) { return pick_batch_eb<2>(c); }
}  // namespace bsd
