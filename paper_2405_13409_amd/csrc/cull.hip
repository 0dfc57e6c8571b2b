// Conservative normal-cone cull of (x0, x2, triangle) triples for one
// specular vertex.  h x n = 0 (Eq. eq_ch) needs the generalised half vector
// h = eta0 w0 + eta2 w2 to be parallel to the interpolated normal; the kernel
// rejects a triple only when the cone of possible h directions and the cone of
// possible normal directions cannot meet.
#include "spoly_dev.hpp"
#include "onebounce.hpp"

namespace spoly {

// Per-triangle cones (FP64 math, rounded outward to float):
//   c = centroid, rad = max |p_i - c| (bounding sphere),
//   an = normalize(sum n_i^), thn = max angle(an, n_i^).
// The interpolated normal sum w_i n_i (w_i >= 0) stays inside that cone
// whenever thn < pi/2.
__global__ void __launch_bounds__(256) k_tri_cones(const double* px, const double* py, const double* pz,
                                                   const double* nx, const double* ny, const double* nz,
                                                   const int32_t* tri, int32_t n_tris, float4* cone)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tris) return;
    V3<double> p[3], n[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        int i = tri[3 * t + k];
        p[k] = {px[i], py[i], pz[i]};
        n[k] = normalized(V3<double>{nx[i], ny[i], nz[i]});
    }
    V3<double> c = (p[0] + p[1] + p[2]) * (1.0 / 3.0);
    double rad = fmax(fmax(len(p[0] - c), len(p[1] - c)), len(p[2] - c));
    V3<double> an = normalized(n[0] + n[1] + n[2]);
    double th = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) th = fmax(th, acos(fmin(1.0, fmax(-1.0, dot(an, n[k])))));
    if (!(len(an) > 0.5)) th = 4.0;  // degenerate cone: keep everything
    cone[2 * t] = make_float4(float(c.x), float(c.y), float(c.z), float(rad * (1.0 + 1e-6) + 1e-7));
    cone[2 * t + 1] = make_float4(float(an.x), float(an.y), float(an.z), float(th + 1e-6));
}

constexpr int kCullPts = 64;  // (x0, x2) pairs per thread; one atomic per wave per 64 pairs

__device__ __forceinline__ bool cone_keep(float4 c0, float4 c1, float px, float py, float pz, float qx, float qy,
                                          float qz, float eta0, float eta1, float margin)
{
    float ax = px - c0.x, ay = py - c0.y, az = pz - c0.z;
    float bx = qx - c0.x, by = qy - c0.y, bz = qz - c0.z;
    float da = sqrtf(ax * ax + ay * ay + az * az), db = sqrtf(bx * bx + by * by + bz * bz);
    const float rad = c0.w;
    if (!(da > rad * 1.0001f) || !(db > rad * 1.0001f) || !(c1.w < 1.5707f)) return true;
    float ia = 1.0f / da, ib = 1.0f / db;
    ax *= ia; ay *= ia; az *= ia;
    bx *= ib; by *= ib; bz *= ib;
    float sa = rad * ia, sb = rad * ib;
    float chord_a = sqrtf(fmaxf(0.0f, 2.0f - 2.0f * sqrtf(fmaxf(0.0f, 1.0f - sa * sa))));
    float chord_b = sqrtf(fmaxf(0.0f, 2.0f - 2.0f * sqrtf(fmaxf(0.0f, 1.0f - sb * sb))));
    float hx = eta0 * ax + eta1 * bx, hy = eta0 * ay + eta1 * by, hz = eta0 * az + eta1 * bz;
    float L = sqrtf(hx * hx + hy * hy + hz * hz);
    float delta = (eta0 * chord_a + eta1 * chord_b) * 1.0001f + 1e-6f;
    if (!(delta < L)) return true;
    float lim = c1.w + asinf(fminf(1.0f, delta / L)) + margin;
    if (lim >= 1.5707f) return true;
    float cphi = fabsf(c1.x * hx + c1.y * hy + c1.z * hz) / L;
    return cphi >= cosf(lim) * (1.0f - 1e-6f);
}

// Grid: (pair block) x (triangle block of 256).  Each thread tests one
// triangle against kCullPts consecutive (x0, x2) pairs, keeping the wave's
// per-pair ballots in LDS; the wave then reserves its whole output range with
// one atomic and writes the kept triples pair by pair (coalesced).
__global__ void __launch_bounds__(256) k_cull_1bounce(CullArgs A)
{
    __shared__ unsigned long long s_bal[4][kCullPts];
    const int ntb = (A.n_tris + 255) / 256;
    const int t = int(blockIdx.x % ntb) * blockDim.x + threadIdx.x;
    const int64_t pblock = int64_t(blockIdx.x / ntb);
    const bool tri_ok = t < A.n_tris;
    const int w = threadIdx.x / kWave;
    const int lane = lane_id();
    float4 c0 = make_float4(0, 0, 0, 0), c1 = make_float4(0, 0, 0, 4.0f);
    if (tri_ok) {
        c0 = A.tri_cone[2 * t];
        c1 = A.tri_cone[2 * t + 1];
    }
    const int64_t n_pairs = int64_t(A.n0) * A.n2;
    const int64_t pair0 = pblock * kCullPts;
    const int npairs = int(min<int64_t>(kCullPts, n_pairs - pair0));
    int mine = 0;
    for (int k = 0; k < npairs; ++k) {
        const int64_t pr = pair0 + k;
        const int j0 = int(pr / A.n2), j2 = int(pr % A.n2);
        bool keep = tri_ok && cone_keep(c0, c1, float(A.x0x[j0]), float(A.x0y[j0]), float(A.x0z[j0]), float(A.x2x[j2]),
                                        float(A.x2y[j2]), float(A.x2z[j2]), A.eta0, A.eta1, A.margin);
        const unsigned long long bal = __ballot(keep);
        if (lane == 0) s_bal[w][k] = bal;
        mine += keep ? 1 : 0;
    }
    const int incl = wave_incl_scan(mine);
    const int total = __shfl(incl, kWave - 1, kWave);
    if (total == 0) return;
    unsigned long long base = 0;
    if (lane == kWave - 1) base = atomicAdd(A.out_count, (unsigned long long)total);
    base = __shfl(base, kWave - 1, kWave);
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    unsigned long long off = base;
    const unsigned long long lt = (1ull << lane) - 1ull;
    for (int k = 0; k < npairs; ++k) {
        const unsigned long long bal = s_bal[w][k];
        if ((bal >> lane) & 1ull) {
            const unsigned long long idx = off + (unsigned long long)__popcll(bal & lt);
            if (idx < (unsigned long long)A.cap) {
                const int64_t pr = pair0 + k;
                A.out_x0[idx] = int(pr / A.n2);
                A.out_x2[idx] = int(pr % A.n2);
                A.out_tri[idx] = t;
            }
        }
        off += (unsigned long long)__popcll(bal);
    }
}

hipError_t launch_tri_cones(const double* px, const double* py, const double* pz, const double* nx,
                            const double* ny, const double* nz, const int32_t* tri, int32_t n_tris,
                            float4* tri_cone, hipStream_t stream)
{
    if (n_tris <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tri_cones, dim3((n_tris + 255) / 256), dim3(256), 0, stream, px, py, pz, nx, ny, nz, tri,
                       n_tris, tri_cone);
    return hipGetLastError();
}

hipError_t launch_cull_1bounce(const CullArgs& A, hipStream_t stream)
{
    const int64_t n_pairs = int64_t(A.n0) * A.n2;
    if (n_pairs <= 0 || A.n_tris <= 0) return hipSuccess;
    const int64_t npb = (n_pairs + kCullPts - 1) / kCullPts;
    const int64_t nblk = npb * ((A.n_tris + 255) / 256);
    if (nblk > 2147483647LL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_cull_1bounce, dim3(unsigned(nblk)), dim3(256), 0, stream, A);
    return hipGetLastError();
}

}  // namespace spoly
