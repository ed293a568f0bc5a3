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

// A split-K variant: configuration `base` run over `slices` slices of K.
struct SplitDef {
  int32_t base, slices;
};

struct PartRef {
  LaunchEntry* entries;
  const int* count;
};

struct DtypeRegistry {
  const ConfigDef* configs;   // the configuration space of the dtype (id = index)
  int n_configs;
  const SplitDef* splits;     // split-K variants (kernel id = n_configs + index)
  int n_splits;
  const PartRef* parts;       // compiled instantiations
  int n_parts;
};

// Indexed by kt_dtype (F32, BF16, FP8E4M3).
extern const DtypeRegistry dtype_registry[3];

}  // namespace kt
