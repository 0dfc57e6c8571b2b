// Kernel arguments and launchers of the two-vertex path (chains RR, RT, TR, TT).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/spoly.h"

namespace spoly {

struct TTArgs {
    const double *px, *py, *pz, *nx, *ny, *nz;
    const int32_t* tri;
    const double *x0x, *x0y, *x0z, *x3x, *x3y, *x3z;
    const int32_t *q_x0, *q_x3, *q_tris;   // q_tris[2q], q_tris[2q+1] = T1, T2
    int64_t nq;
    int32_t ev1, ev2;         // event at x1 and at x2: SPOLY_R or SPOLY_T
    double eta0, eta1, eta2;
    double sqrt_bp[7];        // piece breakpoints of the square-root approximation
    double sqrt_c[24];        // (c0, c1, d0, d1) per piece
    int32_t pieces, bisect_iters, polish_iters;
    double tau, u_margin, dedup;
    spoly_solution* out;
    int64_t cap;
    unsigned long long* out_count;
    unsigned long long* counters;
    int32_t* diag_q;
};

constexpr int kMaxPieces = 4095;                 // pieces of the two-vertex sign scan
constexpr int kSignWords = (kMaxPieces + 1 + 63) / 64;
constexpr int kMaxBisect = 40;                   // bisection steps per sign change

struct LaneTT {
    double u1[4], v1[4], u2[4], v2[4], res[4], edge[4];
    int n;
    int over;  // valid paths past the four kept (counted, not written)
};

hipError_t launch_tt_solve(const TTArgs& A, hipStream_t stream);

struct CullTTArgs {
    const float4* tri_cone;
    int32_t n_tris;
    const double *x0x, *x0y, *x0z, *x3x, *x3y, *x3z;
    int32_t n0, n3;
    float eta0, eta1, eta2, margin;
    int2* pairs;                      // workspace: (t1, t2) pairs passing the x2 test for one light
    int64_t pair_cap;
    unsigned long long* pair_count;   // workspace counter
    int32_t *out_x0, *out_x3, *out_t1, *out_t2;
    int64_t cap;
    unsigned long long* out_count;
};

hipError_t launch_zero_u64(unsigned long long* p, hipStream_t stream);
hipError_t launch_tt_pairs(const CullTTArgs& A, int j3, hipStream_t stream);
hipError_t launch_tt_cull(const CullTTArgs& A, int j3, int64_t n_pairs, hipStream_t stream);

}  // namespace spoly
