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

constexpr int kCullPts = 256;  // (x0, x2) pairs per tile; each listed triangle is tested against all of them

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

// Bounding sphere of a tile's points: centre = mean of the n staged points,
// radius = max distance to it (rounded outward).  Block-wide; every thread calls.
__device__ __forceinline__ float4 tile_sphere(const float4* s_p, int n, float* s_red)
{
    const int w = threadIdx.x / kWave, nw = (blockDim.x + kWave - 1) / kWave;
    float x = 0.0f, y = 0.0f, z = 0.0f;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        x += s_p[k].x;
        y += s_p[k].y;
        z += s_p[k].z;
    }
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
        x += __shfl_xor(x, d, kWave);
        y += __shfl_xor(y, d, kWave);
        z += __shfl_xor(z, d, kWave);
    }
    if (lane_id() == 0) {
        s_red[3 * w] = x;
        s_red[3 * w + 1] = y;
        s_red[3 * w + 2] = z;
    }
    __syncthreads();
    x = y = z = 0.0f;
    for (int i = 0; i < nw; ++i) {
        x += s_red[3 * i];
        y += s_red[3 * i + 1];
        z += s_red[3 * i + 2];
    }
    const float inv = 1.0f / float(n > 0 ? n : 1);
    x *= inv;
    y *= inv;
    z *= inv;
    float r2 = 0.0f;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        const float dx = s_p[k].x - x, dy = s_p[k].y - y, dz = s_p[k].z - z;
        r2 = fmaxf(r2, dx * dx + dy * dy + dz * dz);
    }
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) r2 = fmaxf(r2, __shfl_xor(r2, d, kWave));
    __syncthreads();   // the sums above have been read
    if (lane_id() == 0) s_red[w] = r2;
    __syncthreads();
    r2 = 0.0f;
    for (int i = 0; i < nw; ++i) r2 = fmaxf(r2, s_red[i]);
    __syncthreads();   // s_red may be reused after this call
    return make_float4(x, y, z, __builtin_amdgcn_sqrtf(r2) * 1.0001f + 1e-6f);
}

// One side of the tile bound: the unit direction from the triangle's centre c
// to the tile's centre p, and eta times an upper bound of the angle of the cone
// of directions from the triangle's sphere (radius rad) to the tile's sphere
// (radius rho), asin((rad + rho) / |p - c|) <= s (1 + (pi/2 - 1) s^2) on [0,1]
// (asin(s)/s is convex in s^2 and equal to it at both ends).  The angle, not
// the chord, is what makes the bound hold for every pair of the tile: for a
// point x of the tile, the pair's own direction differs from the tile's by at
// most (angle - pair's angle), and chord <= angle.
__device__ __forceinline__ bool tile_side(float4 c0, float4 p, float eta, ConeSide& s)
{
    const float ax = p.x - c0.x, ay = p.y - c0.y, az = p.z - c0.z;
    const float d2 = ax * ax + ay * ay + az * az;
    const float rl = (c0.w + p.w) * 1.0001f;
    if (!(d2 > rl * rl)) return false;
    const float ia = __builtin_amdgcn_rsqf(d2);
    const float sa = (c0.w + p.w) * ia * 1.000001f;
    if (!(sa < 1.0f)) return false;
    const float e = eta * ia;
    s.hx = e * ax;
    s.hy = e * ay;
    s.hz = e * az;
    s.dch = eta * sa * fmaf(0.5708f, sa * sa, 1.0f) * 1.001f;
    return true;
}

constexpr int kCullTriRange = 4096;   // triangles per block (at most 32 x 256: one mask bit per chunk)

// Two-level cull.  Grid-stride over (tile, triangle range): a tile is kCullPts
// consecutive (x0, x2) pairs, staged in LDS with the bounding spheres of its x0
// and x2 points.  Each triangle of the range is first tested against the whole
// tile (the cone of directions from the triangle to the tile's spheres contains
// every pair's cone, with an outward-rounded angle bound, so a tile rejection
// implies the rejection of each of its pairs); the triangles that pass are
// compacted into an LDS list in triangle order, and each full list of 256 (and
// the rest at the end of the range) is tested pair by pair exactly as a flat
// cull would: one thread per listed triangle, looping over the tile's pairs
// and keeping a 256-bit mask of the kept ones.  The block reserves its output
// range with one atomic; each wave then writes its kept triples in (lane,
// pair) order, lane by lane, the whole wave storing one lane's mask word at a
// time to consecutive slots.  Triangle-major output keeps
// the candidates of one wave of the solve similar (one triangle, neighbouring
// points).  Points that are close in index should be close in space (pixel
// tiles, a Morton order) for the tile test to reject.
__global__ void __launch_bounds__(256) k_cull_1bounce(CullArgs A)
{
    __shared__ int s_j0[kCullPts], s_j2[kCullPts];
    __shared__ float4 s_p0[kCullPts], s_p2[kCullPts];
    __shared__ int s_list[2 * 256];
    __shared__ int s_wc[kMaxBlockWaves];
    __shared__ float s_red[3 * kMaxBlockWaves];
    __shared__ unsigned long long s_slots[kMaxBlockWaves + 1];
    const int ntr = (A.n_tris + kCullTriRange - 1) / kCullTriRange;
    const int64_t n_pairs = int64_t(A.n0) * A.n2;
    const int64_t nblk = ((n_pairs + kCullPts - 1) / kCullPts) * ntr;
    const int w = threadIdx.x / kWave;
    const int lane = lane_id();
    const int nw = blockDim.x / kWave;
    for (int64_t vb = blockIdx.x; vb < nblk; vb += gridDim.x) {
        const int tr0 = int(vb % ntr) * kCullTriRange;
        const int tr1 = min(A.n_tris, tr0 + kCullTriRange);
        const int64_t pair0 = (vb / ntr) * kCullPts;
        const int npairs = int(min<int64_t>(kCullPts, n_pairs - pair0));
        // stage the tile's pairs (ids and float coordinates) in LDS: every
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
        const float4 sph0 = tile_sphere(s_p0, npairs, s_red);
        const float4 sph2 = tile_sphere(s_p2, npairs, s_red);
        // tile test of the whole range first (bit c: triangle tr0 + 256 c + thread),
        // with no barrier between the loads, then compaction chunk by chunk
        unsigned pmask = 0u;
#pragma unroll 4
        for (int c = 0; c < kCullTriRange / 256; ++c) {
            const int t = tr0 + c * 256 + int(threadIdx.x);
            if (t < tr1) {
                const float4 c0 = A.tri_cone[2 * t], c1 = A.tri_cone[2 * t + 1];
                const float thm = c1.w + A.margin;
                bool pass = !(thm < 1.5707f);
                if (!pass) {
                    ConeSide sa, sb;
                    pass = !tile_side(c0, sph0, A.eta0, sa) || !tile_side(c0, sph2, A.eta1, sb) ||
                           cone_meet(c1, cosf(thm), sinf(thm), sa, sb);
                }
                pmask |= (pass ? 1u : 0u) << c;
            }
        }
        int nlist = 0;
        for (int tc = tr0; tc < tr1; tc += blockDim.x) {
            // passing ids of triangles tc .. tc+255 appended in order
            const int t = tc + threadIdx.x;
            const bool pass = (pmask >> ((tc - tr0) / 256)) & 1u;
            const unsigned long long bal = __ballot(pass);
            if (lane == 0) s_wc[w] = __popcll(bal);
            __syncthreads();
            int off = nlist;
            for (int i = 0; i < w; ++i) off += s_wc[i];
            int added = 0;
            for (int i = 0; i < nw; ++i) added += s_wc[i];
            if (pass) off += __popcll(bal & ((1ull << lane) - 1ull));
            if (pass) s_list[off] = t;
            nlist += added;
            __syncthreads();
            const bool last = tc + int(blockDim.x) >= tr1;
            // pair-by-pair test of the first min(256, nlist) listed triangles,
            // while a full list is ready (or, at the end of the range, any)
            while (nlist >= int(blockDim.x) || (last && nlist > 0)) {
                const int nf = min(nlist, int(blockDim.x));
                const bool wave_on = w * kWave < nf;
                const bool tri_ok = int(threadIdx.x) < nf;
                int mine = 0;
                unsigned long long m[kCullPts / kWave];   // pairs kept for this lane's triangle
#pragma unroll
                for (int kw = 0; kw < kCullPts / kWave; ++kw) m[kw] = 0ull;
                if (wave_on) {
                    float4 c0 = make_float4(0, 0, 0, 0), c1 = make_float4(0, 0, 0, 4.0f);
                    if (tri_ok) {
                        const int tt = s_list[threadIdx.x];
                        c0 = A.tri_cone[2 * tt];
                        c1 = A.tri_cone[2 * tt + 1];
                    }
                    // a normal cone of 90 degrees or more (with the margin) meets every h
                    const float thm = c1.w + A.margin;
                    const bool all = !(thm < 1.5707f);
                    const float cth = cosf(fminf(thm, 1.5707f)), sth = sinf(fminf(thm, 1.5707f));
                    int j2_side = -1;
                    ConeSide sb{0.0f, 0.0f, 0.0f, 0.0f};
                    bool b_ok = false;
#pragma unroll
                    for (int kw = 0; kw < kCullPts / kWave; ++kw) {
                        const int kend = min(npairs - kw * kWave, kWave);
                        unsigned long long mk = 0ull;
                        for (int b = 0; b < kend; ++b) {
                            const int k = kw * kWave + b;
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
                            mk |= (unsigned long long)(keep ? 1u : 0u) << b;
                        }
                        m[kw] = mk;
                        mine += __popcll(mk);
                    }
                }
                const int incl = wave_incl_scan(mine);
                const int total = __shfl(incl, kWave - 1, kWave);
                const int lc = incl - mine;
                const int my_tri = tri_ok ? s_list[threadIdx.x] : 0;
                const unsigned long long base = block_reserve((unsigned long long)total, A.out_count, s_slots);
                if (total > 0) {
                    // the wave writes each lane's kept pairs in turn: bit i of
                    // mask word kw of lane L (pair 64 kw + i) goes to
                    // base + lc(L) + (kept pairs of L before it), thread i
                    // handling bit i, so consecutive threads store to
                    // consecutive slots
                    for (int L = 0; L < kWave; ++L) {
                        if (__builtin_amdgcn_readlane(mine, L) == 0) continue;
                        int pos = __builtin_amdgcn_readlane(lc, L);
                        const int tL = __builtin_amdgcn_readlane(my_tri, L);
#pragma unroll
                        for (int kw = 0; kw < kCullPts / kWave; ++kw) {
                            const unsigned wlo = __builtin_amdgcn_readlane(unsigned(m[kw]), L);
                            const unsigned whi = __builtin_amdgcn_readlane(unsigned(m[kw] >> 32), L);
                            if ((wlo | whi) == 0u) continue;
                            const int before = __builtin_amdgcn_mbcnt_hi(whi, __builtin_amdgcn_mbcnt_lo(wlo, 0u));
                            const unsigned mine_bit = lane < 32 ? (wlo >> lane) : (whi >> (lane - 32));
                            if (mine_bit & 1u) {
                                const int k = kw * kWave + lane;
                                const unsigned long long idx = base + (unsigned long long)(pos + before);
                                if (idx < (unsigned long long)A.cap) {
                                    A.out_x0[idx] = s_j0[k];
                                    A.out_x2[idx] = s_j2[k];
                                    A.out_tri[idx] = tL;
                                }
                            }
                            pos += __popc(wlo) + __popc(whi);
                        }
                    }
                }
                __syncthreads();   // the processed list entries are no longer read
                // move the remaining listed triangles to the front
                const int rest = nlist - nf;
                int carry = -1;
                if (int(threadIdx.x) < rest) carry = s_list[nf + threadIdx.x];
                __syncthreads();
                if (carry >= 0) s_list[threadIdx.x] = carry;
                nlist = rest;
                __syncthreads();
            }
        }
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
    const int64_t nblk = npb * ((A.n_tris + kCullTriRange - 1) / kCullTriRange);
    const int64_t grid = nblk < (int64_t(1) << 22) ? nblk : (int64_t(1) << 22);
    hipLaunchKernelGGL(k_cull_1bounce, dim3(unsigned(grid)), dim3(256), 0, stream, A);
    return hipGetLastError();
}

}  // namespace spoly
