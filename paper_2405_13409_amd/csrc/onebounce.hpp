// Kernel-argument block and launcher of the one-vertex solve.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/spoly.h"

namespace spoly {

struct OneBounceArgs {
    const double *px, *py, *pz, *nx, *ny, *nz;
    const int32_t* tri;
    const double *x0x, *x0y, *x0z, *x2x, *x2y, *x2z;
    const int32_t *q_x0, *q_x2, *q_tri;
    int64_t nq;
    double eta0, eta1;
    double iso_eps, tau, u_margin, dedup;
    int32_t polish_iters;
    spoly_solution* out;
    int64_t cap;
    unsigned long long* out_count;
    unsigned long long* counters;
    int32_t* diag_q;
};

hipError_t launch_onebounce(const OneBounceArgs& A, int ev, int prec, hipStream_t stream);

struct CullArgs {
    const float4* tri_cone;   // per triangle: (centroid.xyz, radius), (axis.xyz, half angle)
    int32_t n_tris;
    const double *x0x, *x0y, *x0z, *x2x, *x2y, *x2z;
    int32_t n0, n2;
    float eta0, eta1, margin;
    int32_t *out_x0, *out_x2, *out_tri;
    int64_t cap;
    unsigned long long* out_count;
};

hipError_t launch_tri_cones(const double* px, const double* py, const double* pz, const double* nx,
                            const double* ny, const double* nz, const int32_t* tri, int32_t n_tris,
                            float4* tri_cone, hipStream_t stream);
hipError_t launch_cull_1bounce(const CullArgs& A, hipStream_t stream);

}  // namespace spoly
