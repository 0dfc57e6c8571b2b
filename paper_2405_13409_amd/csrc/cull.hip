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

constexpr int kCullPts = 256;  // (x0, x2) pairs per thread; one atomic per block of 256 x 256 tests

// One side of the half-vector bound: the unit direction from the triangle's
// bounding sphere (centre c, radius rad) towards point p, scaled by eta, and
// eta times the chord 2 sin(theta/2) of the direction cone's half angle
// theta = asin(rad / |p - c|).  Returns false when p lies inside the sphere
// (the direction is then unbounded).
struct ConeSide {
    float hx, hy, hz, dch;
};

__device__ __forceinline__ bool cone_side(float4 c0, float px, float py, float pz, float eta, ConeSide& s)
{
    const float ax = px - c0.x, ay = py - c0.y, az = pz - c0.z;
    const float d2 = ax * ax + ay * ay + az * az;
    const float rl = c0.w * 1.0001f;
    if (!(d2 > rl * rl)) return false;
    const float ia = __builtin_amdgcn_rsqf(d2);
    const float sa = fminf(c0.w * ia * 1.000001f, 1.0f);   // sin theta
    // 2 sin(theta/2) = sin theta sqrt(2 / (1 + cos theta)), and sqrt(2 / (1 + sqrt(1 - s^2)))
    // <= 1 + (sqrt 2 - 1) s^2 on [0,1] (convex in s^2, equal at both ends): an upper bound of
    // the chord without square roots
    const float chord = sa * fmaf(0.41422f, sa * sa, 1.0f) * 1.000001f;
    const float e = eta * ia;
    s.hx = e * ax;
    s.hy = e * ay;
    s.hz = e * az;
    s.dch = eta * chord;
    return true;
}

// Keep unless h = eta_a w_a + eta_b w_b (w in their direction cones) cannot be
// parallel to any normal of the normal cone (axis an, half angle thn).  h lies
// within asin(delta/L) of H = eta_a a_a + eta_b a_b, |H| = L, delta the sum of
// the scaled chords; the test is angle(+-an, H) > thn + margin + asin(delta/L),
// written with cosines: cth = cos(thn + margin), sth = sin(thn + margin).
__device__ __forceinline__ bool cone_meet(float4 c1, float cth, float sth, const ConeSide& a, const ConeSide& b)
{
    const float hx = a.hx + b.hx, hy = a.hy + b.hy, hz = a.hz + b.hz;
    const float iL = __builtin_amdgcn_rsqf(hx * hx + hy * hy + hz * hz);
    const float delta = (a.dch + b.dch) * 1.0001f + 1e-6f;
    const float sphi = delta * iL * 1.000001f;
    if (!(sphi < 1.0f)) return true;
    const float cphi = __builtin_amdgcn_sqrtf(1.0f - sphi * sphi);
    const float clim = cth * cphi - sth * sphi;            // cos(thn + margin + phi)
    if (!(clim > 1e-4f)) return true;                      // the cones reach 90 degrees
    const float cdot = fabsf(c1.x * hx + c1.y * hy + c1.z * hz) * iL;
    return cdot >= clim * (1.0f - 4e-6f);
}

// Position of the r-th set bit (r counted from 0) of a 64-bit mask.
__device__ __forceinline__ int select_bit(unsigned long long m, int r)
{
    int pos = 0;
    int c = __popc(unsigned(m));
    if (r >= c) { r -= c; m >>= 32; pos += 32; }
    unsigned x = unsigned(m);
    c = __popc(x & 0xffffu);
    if (r >= c) { r -= c; x >>= 16; pos += 16; }
    c = __popc(x & 0xffu);
    if (r >= c) { r -= c; x >>= 8; pos += 8; }
    c = __popc(x & 0xfu);
    if (r >= c) { r -= c; x >>= 4; pos += 4; }
    c = __popc(x & 0x3u);
    if (r >= c) { r -= c; x >>= 2; pos += 2; }
    if (r >= int(x & 1u)) pos += 1;
    return pos;
}

// Grid: (pair block) x (triangle block of 256).  Each thread tests one
// triangle against kCullPts consecutive (x0, x2) pairs, keeping the wave's
// per-pair ballots in LDS.  The block reserves its whole output range with
// one atomic (a single counter shared by every block is the bottleneck when
// each wave reserves on its own).  Each wave then writes its kept triples in
// (pair, lane) order with full-width stores: output slot s of the wave is
// mapped back to its pair by a binary search over the per-pair prefix counts
// and to its lane by selecting the right bit of that pair's ballot.  The x2
// side of the bound is recomputed only when x2 changes (with one light: once).
__global__ void __launch_bounds__(256) k_cull_1bounce(CullArgs A)
{
    __shared__ unsigned long long s_bal[4][kCullPts];
    __shared__ int s_cum[4][kCullPts];
    __shared__ int s_j0[kCullPts], s_j2[kCullPts];
    __shared__ float4 s_p0[kCullPts], s_p2[kCullPts];
    __shared__ unsigned long long s_slots[kMaxBlockWaves + 1];
    const int ntb = (A.n_tris + 255) / 256;
    const int64_t nblk = ((int64_t(A.n0) * A.n2 + kCullPts - 1) / kCullPts) * ntb;
    // grid-stride over (pair block, triangle block): a launch may hold at most 2^32 work-items
    for (int64_t vb = blockIdx.x; vb < nblk; vb += gridDim.x) {
        const int t0 = int(vb % ntb) * blockDim.x;
        const int t = t0 + threadIdx.x;
        const int64_t pblock = vb / ntb;
        const bool tri_ok = t < A.n_tris;
        const int w = threadIdx.x / kWave;
        const int lane = lane_id();
        float4 c0 = make_float4(0, 0, 0, 0), c1 = make_float4(0, 0, 0, 4.0f);
        if (tri_ok) {
            c0 = A.tri_cone[2 * t];
            c1 = A.tri_cone[2 * t + 1];
        }
        // a normal cone of 90 degrees or more (with the margin) meets every h
        const float thm = c1.w + A.margin;
        const bool all = !(thm < 1.5707f);
        const float cth = cosf(fminf(thm, 1.5707f)), sth = sinf(fminf(thm, 1.5707f));
        const int64_t n_pairs = int64_t(A.n0) * A.n2;
        const int64_t pair0 = pblock * kCullPts;
        const int npairs = int(min<int64_t>(kCullPts, n_pairs - pair0));
        // stage the block's pairs (ids and float coordinates) in LDS: every
        // lane reads the same pair, and a global load per pair would stall
        for (int k = threadIdx.x; k < npairs; k += blockDim.x) {
            const int64_t pr = pair0 + k;
            const int jj0 = int(pr / A.n2), jj2 = int(pr % A.n2);
            s_j0[k] = jj0;
            s_j2[k] = jj2;
            s_p0[k] = make_float4(float(A.x0x[jj0]), float(A.x0y[jj0]), float(A.x0z[jj0]), 0.0f);
            s_p2[k] = make_float4(float(A.x2x[jj2]), float(A.x2y[jj2]), float(A.x2z[jj2]), 0.0f);
        }
        __syncthreads();
        int j2_side = -1;
        ConeSide sb{0.0f, 0.0f, 0.0f, 0.0f};
        bool b_ok = false;
        int mine = 0;
        for (int k = 0; k < npairs; ++k) {
            bool keep = false;
            if (tri_ok) {
                const int j2 = s_j2[k];
                if (j2 != j2_side) {
                    const float4 x2 = s_p2[k];
                    b_ok = cone_side(c0, x2.x, x2.y, x2.z, A.eta1, sb);
                    j2_side = j2;
                }
                const float4 x0 = s_p0[k];
                ConeSide sa;
                const bool a_ok = cone_side(c0, x0.x, x0.y, x0.z, A.eta0, sa);
                keep = all || !a_ok || !b_ok || cone_meet(c1, cth, sth, sa, sb);
            }
            const unsigned long long bal = __ballot(keep);
            if (lane == 0) s_bal[w][k] = bal;
            mine += keep ? 1 : 0;
        }
        const int incl = wave_incl_scan(mine);
        const int total = __shfl(incl, kWave - 1, kWave);
        __syncthreads();   // ballots and pair indices visible to every lane
        // exclusive per-pair prefix counts of this wave (4 pairs per lane)
        {
            constexpr int kPer = kCullPts / kWave;
            int cnt[kPer], sum = 0;
    #pragma unroll
            for (int i = 0; i < kPer; ++i) {
                const int k = lane * kPer + i;
                cnt[i] = k < npairs ? __popcll(s_bal[w][k]) : 0;
                sum += cnt[i];
            }
            int run = wave_incl_scan(sum) - sum;
    #pragma unroll
            for (int i = 0; i < kPer; ++i) {
                s_cum[w][lane * kPer + i] = run;
                run += cnt[i];
            }
        }
        const unsigned long long base = block_reserve((unsigned long long)total, A.out_count, s_slots);
        for (int sidx = lane; sidx < total; sidx += kWave) {
            // last pair k with s_cum[k] <= sidx
            int lo = 0, hi = npairs - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_cum[w][mid] <= sidx) lo = mid;
                else hi = mid - 1;
            }
            const int src = select_bit(s_bal[w][lo], sidx - s_cum[w][lo]);
            const unsigned long long idx = base + (unsigned long long)sidx;
            if (idx < (unsigned long long)A.cap) {
                A.out_x0[idx] = s_j0[lo];
                A.out_x2[idx] = s_j2[lo];
                A.out_tri[idx] = t0 + w * kWave + src;
            }
        }
        __syncthreads();   // LDS is reused by the next block of the stride
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
    const int64_t grid = nblk < (int64_t(1) << 22) ? nblk : (int64_t(1) << 22);
    hipLaunchKernelGGL(k_cull_1bounce, dim3(unsigned(grid)), dim3(256), 0, stream, A);
    return hipGetLastError();
}

}  // namespace spoly
