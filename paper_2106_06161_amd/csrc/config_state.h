// Library-internal access to the launch-shape state kept by the C ABI
// (api.hip), for the native autotuner (autotune.hip).
#pragma once

#include <stdint.h>

#include <vector>

#include "kernels.h"

namespace bsd {

// Whether a shape is forced with bs_set_config, and which.
struct ConfigState {
  bool forced;
  LaunchConfig cfg;
};
ConfigState config_state();
void restore_config_state(const ConfigState& s);

// One entry of the tuned table: call kind (0 single, 1 batched), element
// bytes, size class (domain bits, or bits of the mean segment size), shape.
struct TunedEntry {
  uint32_t kind, elem_bytes, size_bits;
  LaunchConfig cfg;
};
std::vector<TunedEntry> tuned_snapshot();

// Single-shuffle size classes where bs_shuffle prefers the staged form.
struct StagedEntry {
  uint32_t elem_bytes, size_bits;
  bool prefer;
};
void set_staged_preference(uint32_t elem_bytes, uint32_t size_bits, bool prefer);
std::vector<StagedEntry> staged_snapshot();

}  // namespace bsd
