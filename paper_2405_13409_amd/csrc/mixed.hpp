// Persistent mixed-batch solve: arguments and launcher.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "onebounce.hpp"
#include "twobounce.hpp"

namespace spoly {

struct MixedArgs {
    OneBounceArgs r;     // one-vertex instances (queries 0 .. r.nq-1)
    TTArgs t;            // two-vertex tuples (queries r.nq .. r.nq + t.nq - 1)
    int64_t n_r_tiles;   // ceil(r.nq / r_tile)
    int64_t n_items;     // n_r_tiles + t.nq
    int32_t r_tile;      // one-vertex instances per work item (multiple of 64)
    int32_t order;       // 0: two-vertex items first, 1: one-vertex first, 2: interleaved
    unsigned long long* queue;
};

hipError_t launch_mixed(const MixedArgs& M, int ev, int prec, int workgroups, hipStream_t stream);

}  // namespace spoly
