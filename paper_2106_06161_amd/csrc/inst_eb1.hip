// Shuffle kernels for 1-byte records.
#include "shuffle_impl.h"

namespace bsd {
SingleFn pick_single_1(bool odd, bool wide, const LaunchConfig& c) { return pick_single_eb<1>(odd, wide, c); }
BatchFn pick_batch_1(const LaunchConfig& c) { return pick_batch_eb<1>(c); }
}  // namespace bsd
