// Deterministic output order: the solution records a solve wrote, sorted on
// the device by (query, v[0], u[0]) without a host round trip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/spoly.h"

namespace spoly {

// Device workspace bytes for sorting up to `cap` records.
size_t sort_solutions_bytes(int64_t cap);

// Sorts out[0 .. min(*count, cap)) in place on stream s; `work` holds
// sort_solutions_bytes(cap) bytes.
hipError_t sort_solutions(spoly_solution* out, int64_t cap, const unsigned long long* count, void* work,
                          size_t work_bytes, hipStream_t s);

}  // namespace spoly
