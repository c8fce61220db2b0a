// Test double of the kernel side of the runtime (the launch table of rs_kernels.hip) for the
// host-sanitizer build of rs_runtime.cpp, which has no device code: the same table of offered
// (kind, strategy, width), a fixed occupancy, and launches that fail as when no device code is
// loaded.  Only the host paths that end before a launch run against it.
#include <hip/hip_runtime_api.h>

#include "regionstream.h"
#include "rs_internal.h"

namespace rs {

uint32_t lanes_of(uint32_t ensemble_width) { return ensemble_width ? 64u : 0u; }

bool kernel_supported(uint32_t kind, uint32_t strategy, uint32_t width) {
    const bool w_ok = width == 64 || width == 128 || width == 256 || width == 512 || width == 1024;
    if (kind < RS_MODFILTER || kind > RS_HASH_TREE || !w_ok) return false;
    const bool u32_kind = kind != RS_TEXT_WORDS;
    switch (strategy) {
        case RS_TAG:
        case RS_SIGNAL: return true;
        case RS_SIGNAL_LANES: return u32_kind && width <= 256;
        case RS_ENUM_TAG: return kind == RS_HASH_EXPAND || kind == RS_HASH_TREE || kind == RS_TEXT_WORDS;
        default: return false;
    }
}

int blocks_per_cu(uint32_t kind, uint32_t strategy, uint32_t width, uint32_t, uint32_t) {
    return kernel_supported(kind, strategy, width) ? 4 : 0;
}

uint32_t dyn_lds_bytes(uint32_t, uint32_t, uint32_t, uint32_t, uint32_t) { return 0; }

int launch_pipeline(uint32_t, uint32_t, uint32_t, const LaunchArgs &, uint32_t, void *, void *, void *) {
    return (int)hipErrorNoBinaryForGpu;
}

int launch_probe_copy(const void *, void *, unsigned long long, uint32_t, void *) { return (int)hipErrorNoBinaryForGpu; }

int noalloc_scratch(void **out) {
    *out = nullptr;
    return (int)hipErrorNoBinaryForGpu;
}

int launch_noalloc_init(void *, const NoallocTable &, void *) { return (int)hipErrorNoBinaryForGpu; }

}  // namespace rs
