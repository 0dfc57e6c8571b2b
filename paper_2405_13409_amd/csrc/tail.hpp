// Path-phase tail (Sec. 5.3): visibility of every segment of a validated
// chain against the mesh, through a linear BVH built on the device, and the
// chain's contribution from an isotropic point light.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/spoly.h"

namespace spoly {

// Internal node of the hierarchy: the boxes of both children (padded outward
// so that a float slab test never loses a triangle the double test would
// hit) and the children, >= 0 for an internal node, ~pos for the leaf at
// Morton position pos.  64 bytes, read as four float4.
struct BvhNode {
    float lo0[3], hi0[3], lo1[3], hi1[3];
    int32_t child[2];
    int32_t pad[2];
};

// Leaf triangle in Morton order: p0, e1 = p1 - p0, e2 = p2 - p0 and its id.
struct BvhTri {
    double p0[3], e1[3], e2[3];
    int32_t id, pad;
};

struct BvhView {
    const BvhNode* nodes;  // n_tris - 1 internal nodes, root 0
    const BvhTri* tris;    // n_tris leaves
    int32_t n_tris;
};

// Device arrays owned by a built hierarchy.
struct BvhStore {
    BvhNode* nodes;
    BvhTri* tris;
    int32_t n_tris;
};

// Builds the hierarchy of the mesh's triangles on `s` and waits for it.
hipError_t bvh_build(const double* px, const double* py, const double* pz, const int32_t* tri, int32_t n_tris,
                     BvhStore* out, hipStream_t s);
void bvh_free(BvhStore* b);

constexpr int kTailBlock = 128;
constexpr int kBvhStack = 64;  // depth bound of a hierarchy over distinct 64-bit keys

// mask bits besides the blocked segments (bit i: x_i -> x_{i+1})
constexpr int32_t kTailSingular = 1 << 30;  // constraint Jacobian singular: contribution undefined
constexpr int32_t kTailOverflow = 1 << 29;  // traversal stack or visit bound exhausted (not reachable for a
                                            // hierarchy over <= 2^31 leaves)

struct TailArgs {
    BvhView bvh;
    const double *nx, *ny, *nz;   // vertex normals
    const int32_t* tri;
    const double *px, *py, *pz;   // vertex positions
    const double *x0x, *x0y, *x0z;
    const double *xlx, *xly, *xlz;
    const int32_t *q_x0, *q_xl;
    const spoly_solution* sols;
    int64_t n;                         // records in sols (grid size)
    const unsigned long long* count;   // optional: only min(*count, n) records are read
    int k;
    int ev[2];
    double eta[3];
    double intensity, rho, teps;
    double rn[3];
    int use_rn;
    int32_t* mask;
    double* contrib;
    double* image;
};

hipError_t launch_tail(const TailArgs& A, hipStream_t s);

}  // namespace spoly
