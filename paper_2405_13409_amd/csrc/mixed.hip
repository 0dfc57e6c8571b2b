// One persistent launch over a mixed queue of one-vertex instances (tiles
// of r_tile lanes) and two-vertex tuples (one wave each).  Every wave takes the
// next work item from a global counter until the queue is drained, so uneven
// costs (a degree-9/12 resultant per lane vs. a 101-sample determinant scan
// per tuple) balance dynamically; the wave never waits on other waves and
// exits when the counter passes the last item.
#include "spoly_dev.hpp"
#include "mixed.hpp"

namespace spoly {

__device__ __forceinline__ void decode_item(const MixedArgs& M, int64_t item, bool& is_r, int64_t& idx)
{
    const int64_t nr = M.n_r_tiles, nt = M.t.nq;
    if (M.order == 0) {
        is_r = item >= nt;
        idx = is_r ? item - nt : item;
    } else if (M.order == 1) {
        is_r = item < nr;
        idx = is_r ? item : item - nr;
    } else {
        const int64_t m = nr < nt ? nr : nt;
        if (item < 2 * m) {
            is_r = (item & 1) == 0;
            idx = item >> 1;
        } else {
            is_r = nr > nt;
            idx = item - m;
        }
    }
}

template <typename R, int EV>
__global__ void __launch_bounds__(64) k_mixed(MixedArgs M)
{
    __shared__ double lds[kLdsDoubles];
    __shared__ TTGeo sgeo;
    __shared__ unsigned long long smask[kSignWords], cmask[kSignWords];
    const int lane = lane_id();
    for (;;) {
        unsigned long long item = 0;
        if (lane == 0) item = atomicAdd(M.queue, 1ull);
        item = __shfl(item, 0, kWave);
        if (item >= (unsigned long long)M.n_items) break;
        bool is_r;
        int64_t idx;
        decode_item(M, int64_t(item), is_r, idx);
        if (is_r) {
            const int64_t b0 = idx * M.r_tile;
            int64_t b1 = b0 + M.r_tile;
            if (b1 > M.r.nq) b1 = M.r.nq;
            for (int64_t b = b0; b < b1; b += kWave) {
                const int64_t q = b + lane;
                onebounce_lane<R, EV>(M.r, q, q < b1, 0);
            }
        } else {
            tt_tuple(M.t, idx, lds, &sgeo, smask, cmask, M.r.nq);
        }
        __syncthreads();
    }
}

hipError_t launch_mixed(const MixedArgs& M, int ev, int prec, int workgroups, hipStream_t stream)
{
    if (M.n_items <= 0) return hipSuccess;
    const dim3 grid = dim3(static_cast<unsigned>(workgroups));
    const dim3 block = dim3(kWave);
    if (ev == SPOLY_R && prec == SPOLY_FP32_POLISH64) hipLaunchKernelGGL((k_mixed<float, SPOLY_R>), grid, block, 0, stream, M);
    else if (ev == SPOLY_R) hipLaunchKernelGGL((k_mixed<double, SPOLY_R>), grid, block, 0, stream, M);
    else hipLaunchKernelGGL((k_mixed<double, SPOLY_T>), grid, block, 0, stream, M);
    return hipGetLastError();
}

}  // namespace spoly
