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
    int32_t refine_v;             // FP32 reflection: a root whose u narrowly misses the triangle is refined in FP64 (fused) or deferred to the FP64 full list (two-phase)
    spoly_solution* out;
    int64_t cap;
    unsigned long long* out_count;
    unsigned long long* counters;
    int32_t* diag_q;
    // two-phase workspace (device), capacity items_cap >= nq each:
    // candidates with 1..kObEmit roots of r(v), and candidates with more
    int32_t* items_q;
    int32_t* items_n;
    double* items_v;              // [kObEmit * items_cap]
    int32_t* full_q;
    void* rlist;                  // r(v) of the listed candidates, [k][list index], float or double
    int32_t* iso_q;               // listed candidates (query ids)
    int32_t* iso_st;              // listed candidates: 0 interpolated normals, 1 flat
    int64_t items_cap;
    unsigned long long* items_count;   // [0] items, [1] full list, [2] isolation list
};

constexpr int kObEmit = 2;        // roots carried per candidate between the two phases
constexpr int kObCoefMax = 13;    // largest number of coefficients of r(v) (refraction, interpolated normals)

// Fused single-kernel solve (used inside the persistent mixed kernel).
hipError_t launch_onebounce(const OneBounceArgs& A, int ev, int prec, hipStream_t stream);
// Two-phase solve.  Front: a coefficient kernel builds r(v) and lists the
// candidates that may have a root in [0,1] (Bernstein test), an isolation
// kernel finds the roots of the listed ones and compacts the candidates with
// 1..kObEmit roots into A.items_* (more roots: A.full_q).  Back: a persistent
// kernel (back_blocks blocks) solves u, polishes and validates the items with
// full waves, and a last kernel solves the rare candidates of the full list
// from scratch.
// stage_events (optional, 5 events): recorded before the first kernel and after
// each kernel of the phase sequence (reflection: 3 kernels, refraction: 4).
hipError_t launch_onebounce_2phase(const OneBounceArgs& A, int ev, int prec, int back_blocks, hipStream_t stream,
                                   hipEvent_t* stage_events = nullptr);

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
