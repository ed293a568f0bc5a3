// Launcher registry: generated tables map (configuration id, layout) to a
// host launcher of the compiled kernel instantiation.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kt {

struct GemmArgs;

typedef hipError_t (*LaunchFn)(const GemmArgs&, hipStream_t);

struct LaunchEntry {
  int32_t id;
  int32_t ta, tb;
  LaunchFn fn;
};

struct ConfigDef {
  int32_t bm, bn, t, bk;
};

struct PartRef {
  LaunchEntry* entries;
  const int* count;
};

extern const ConfigDef f32_config_table[];
extern const int f32_config_count;
extern const PartRef f32_parts[];
extern const int f32_part_count;

}  // namespace kt
