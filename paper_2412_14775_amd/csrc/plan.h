// plan.h -- host-side internals of librfi shared by api.hip and serve.hip.
#pragma once

#include <cstddef>
#include <cstdint>

#include "../../include/rfi.h"

namespace rfi {

// A number that names a plan for the life of the process.  Unlike the plan's
// address it is never reused after rfi_destroy, so the serving loop keys its
// cached graphs (which hold a plan's kernel arguments) by it.
uint64_t plan_uid(const rfi_plan *plan);

// Bytes of the optional statistics output of one rfi_screen call: [B][C/F][T/M][3] float32.
// Not part of rfi_plan_footprint; the serving loop adds it for requests that write stats.
size_t plan_stats_bytes(const rfi_plan *plan);

}  // namespace rfi
