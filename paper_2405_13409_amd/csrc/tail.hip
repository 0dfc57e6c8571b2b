// Path-phase tail (Sec. 5.3).  Once a chain has passed the path-space check,
// every segment x_i -> x_{i+1} (x_{k+1} the light) must be free of other
// triangles, and each surviving chain contributes to its endpoint.
//
// Visibility: a linear BVH (Morton-ordered leaves, hierarchy from the
// longest common prefixes of the sorted keys, boxes fitted bottom-up) built
// on the device; one lane per chain runs an any-hit traversal per segment
// with a float slab test on padded boxes and the double-precision
// Moller-Trumbore test on leaves, skipping the triangles that carry the
// segment's own ends and hits within t_eps of either end.
//
// Contribution: the irradiance at x0, on the plane normal to the arriving
// ray, from an isotropic point light of intensity I at x_{k+1}:
//   E = I * prod(F_i) * dw/dA,
// F_i the unpolarised Fresnel transmittance at a refraction and a constant
// reflectance at a reflection.  dw/dA comes from the implicit function
// theorem on the vertex constraints C_i = ((eta_in w_in + eta_out w_out) x
// N_i(u_i, v_i)) . (e1_i, e2_i) = 0 (Eq. eq_ch on two tangents): moving x0
// by (s, t) in that plane moves the barycentrics by -J^-1 K (J, K the
// constraint derivatives in the unknowns and in (s, t), taken exactly with
// forward-mode dual numbers), hence x_k, hence the light direction; dw/dA is
// |w_L . (dx_k/ds x dx_k/dt)| / |x_k - x_L|^2.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include "tail.hpp"

namespace spoly {

// ------------------------------------------------------------------ hierarchy build

namespace {

__device__ __forceinline__ uint32_t spread10(uint32_t x)
{
    x &= 0x3ffu;
    x = (x | (x << 16)) & 0x030000ffu;
    x = (x | (x << 8)) & 0x0300f00fu;
    x = (x | (x << 4)) & 0x030c30c3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

__device__ __forceinline__ void tri_verts(const double* px, const double* py, const double* pz, const int32_t* tri,
                                          int32_t t, double p[3][3])
{
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int32_t v = tri[3 * t + j];
        p[j][0] = px[v];
        p[j][1] = py[v];
        p[j][2] = pz[v];
    }
}

// box of the triangle centroids: one block, lo/hi in out[0..5]
__global__ __launch_bounds__(1024) void k_centroid_box(const double* px, const double* py, const double* pz,
                                                       const int32_t* tri, int32_t n, float* out)
{
    __shared__ float red[6][1024];
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int32_t t = threadIdx.x; t < n; t += blockDim.x) {
        double p[3][3];
        tri_verts(px, py, pz, tri, t, p);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float c = float((p[0][a] + p[1][a] + p[2][a]) * (1.0 / 3.0));
            lo[a] = fminf(lo[a], c);
            hi[a] = fmaxf(hi[a], c);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        red[a][threadIdx.x] = lo[a];
        red[3 + a][threadIdx.x] = hi[a];
    }
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                red[a][threadIdx.x] = fminf(red[a][threadIdx.x], red[a][threadIdx.x + w]);
                red[3 + a][threadIdx.x] = fmaxf(red[3 + a][threadIdx.x], red[3 + a][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) out[threadIdx.x] = red[threadIdx.x][0];
}

// key = 30-bit Morton code of the centroid (10 bits per axis) above the index
__global__ void k_morton(const double* px, const double* py, const double* pz, const int32_t* tri, int32_t n,
                         const float* box, unsigned long long* keys)
{
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    double p[3][3];
    tri_verts(px, py, pz, tri, t, p);
    uint32_t code = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float c = float((p[0][a] + p[1][a] + p[2][a]) * (1.0 / 3.0));
        const float ext = box[3 + a] - box[a];
        const float r = ext > 0.f ? (c - box[a]) / ext : 0.f;
        const uint32_t q = uint32_t(fminf(fmaxf(r * 1024.f, 0.f), 1023.f));
        code |= spread10(q) << (2 - a);
    }
    keys[t] = (static_cast<unsigned long long>(code) << 32) | static_cast<uint32_t>(t);
}

// leaf triangles in key order
__global__ void k_leaves(const double* px, const double* py, const double* pz, const int32_t* tri, int32_t n,
                         const unsigned long long* keys, BvhTri* out)
{
    const int32_t pos = blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= n) return;
    const int32_t t = int32_t(keys[pos] & 0xffffffffull);
    double p[3][3];
    tri_verts(px, py, pz, tri, t, p);
    BvhTri r;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        r.p0[a] = p[0][a];
        r.e1[a] = p[1][a] - p[0][a];
        r.e2[a] = p[2][a] - p[0][a];
    }
    r.id = t;
    r.pad = 0;
    out[pos] = r;
}

// common-prefix length of keys i and j, -1 outside [0, n)
__device__ __forceinline__ int prefix(const unsigned long long* keys, int32_t n, int32_t i, int32_t j)
{
    if (j < 0 || j >= n) return -1;
    return __clzll(keys[i] ^ keys[j]);
}

// internal node i of the hierarchy over the sorted keys: the range of leaves
// it covers extends from i in the direction of the neighbour with the longer
// common prefix, and splits where the prefix grows
__global__ void k_internal(const unsigned long long* keys, int32_t n, BvhNode* nodes, int32_t* parent_int,
                           int32_t* parent_leaf, int32_t* flags)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    const int d = prefix(keys, n, i, i + 1) - prefix(keys, n, i, i - 1) > 0 ? 1 : -1;
    const int dmin = prefix(keys, n, i, i - d);
    int32_t lmax = 2;
    while (prefix(keys, n, i, i + lmax * d) > dmin) lmax *= 2;
    int32_t l = 0;
    for (int32_t t = lmax / 2; t >= 1; t /= 2)
        if (prefix(keys, n, i, i + (l + t) * d) > dmin) l += t;
    const int32_t j = i + l * d;
    const int dnode = prefix(keys, n, i, j);
    int32_t s = 0;
    for (int32_t div = 2;; div *= 2) {
        const int32_t t = (l + div - 1) / div;
        if (prefix(keys, n, i, i + (s + t) * d) > dnode) s += t;
        if (t <= 1) break;
    }
    const int32_t g = i + s * d + (d < 0 ? -1 : 0);
    const int32_t lo = min(i, j), hi = max(i, j);
    const int32_t left = lo == g ? ~g : g;
    const int32_t right = hi == g + 1 ? ~(g + 1) : g + 1;
    nodes[i].child[0] = left;
    nodes[i].child[1] = right;
    nodes[i].pad[0] = nodes[i].pad[1] = 0;
    if (left < 0) parent_leaf[~left] = i; else parent_int[left] = i;
    if (right < 0) parent_leaf[~right] = i; else parent_int[right] = i;
    if (i == 0) parent_int[0] = -1;
    flags[i] = 0;
}

__device__ __forceinline__ float pad_lo(double x) { return float(x - 1e-6 * (1.0 + fabs(x))); }
__device__ __forceinline__ float pad_hi(double x) { return float(x + 1e-6 * (1.0 + fabs(x))); }

// bottom-up box fit: the second of the two children to arrive at a node
// merges both boxes and carries on to the parent
__global__ void k_fit(const double* px, const double* py, const double* pz, const int32_t* tri, int32_t n,
                      const BvhTri* leaves, BvhNode* nodes, const int32_t* parent_int, const int32_t* parent_leaf,
                      int32_t* flags)
{
    const int32_t pos = blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= n) return;
    double p[3][3];
    tri_verts(px, py, pz, tri, leaves[pos].id, p);
    float lo[3], hi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = pad_lo(fmin(fmin(p[0][a], p[1][a]), p[2][a]));
        hi[a] = pad_hi(fmax(fmax(p[0][a], p[1][a]), p[2][a]));
    }
    int32_t child = ~pos;
    int32_t node = parent_leaf[pos];
    // a hierarchy over distinct 64-bit keys is at most 64 levels deep; the
    // bound only guards the loop
    for (int level = 0; node >= 0 && level < 2 * kBvhStack; ++level) {
        volatile BvhNode* nd = nodes + node;
        const int slot = nd->child[0] == child ? 0 : 1;
        volatile float* blo = slot == 0 ? nd->lo0 : nd->lo1;
        volatile float* bhi = slot == 0 ? nd->hi0 : nd->hi1;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            blo[a] = lo[a];
            bhi[a] = hi[a];
        }
        __threadfence();
        if (atomicAdd(flags + node, 1) == 0) return;
        __threadfence();
        volatile float* olo = slot == 0 ? nd->lo1 : nd->lo0;
        volatile float* ohi = slot == 0 ? nd->hi1 : nd->hi0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], olo[a]);
            hi[a] = fmaxf(hi[a], ohi[a]);
        }
        child = node;
        node = parent_int[node];
    }
}

}  // namespace

hipError_t bvh_build(const double* px, const double* py, const double* pz, const int32_t* tri, int32_t n,
                     BvhStore* out, hipStream_t s)
{
    out->nodes = nullptr;
    out->tris = nullptr;
    out->n_tris = n;
    unsigned long long *kin = nullptr, *kout = nullptr;
    float* box = nullptr;
    int32_t *par = nullptr, *flags = nullptr;
    void* tmp = nullptr;
    size_t tmp_bytes = 0;
    hipError_t e = hipSuccess;
    const int nb = (n + 255) / 256;
#define TRY(x)                          \
    do {                                \
        e = (x);                        \
        if (e != hipSuccess) goto done; \
    } while (0)
    TRY(hipMalloc(&out->tris, sizeof(BvhTri) * size_t(n)));
    TRY(hipMalloc(&out->nodes, sizeof(BvhNode) * size_t(n > 1 ? n - 1 : 1)));
    TRY(hipMalloc(&kin, sizeof(unsigned long long) * size_t(n)));
    TRY(hipMalloc(&kout, sizeof(unsigned long long) * size_t(n)));
    TRY(hipMalloc(&box, 6 * sizeof(float)));
    TRY(hipMalloc(&par, sizeof(int32_t) * (2 * size_t(n))));
    TRY(hipMalloc(&flags, sizeof(int32_t) * size_t(n)));
    k_centroid_box<<<1, 1024, 0, s>>>(px, py, pz, tri, n, box);
    k_morton<<<nb, 256, 0, s>>>(px, py, pz, tri, n, box, kin);
    TRY(hipGetLastError());
    TRY(hipcub::DeviceRadixSort::SortKeys(nullptr, tmp_bytes, kin, kout, n, 0, 64, s));
    TRY(hipMalloc(&tmp, tmp_bytes));
    TRY(hipcub::DeviceRadixSort::SortKeys(tmp, tmp_bytes, kin, kout, n, 0, 64, s));
    k_leaves<<<nb, 256, 0, s>>>(px, py, pz, tri, n, kout, out->tris);
    if (n > 1) {
        k_internal<<<(n - 1 + 255) / 256, 256, 0, s>>>(kout, n, out->nodes, par, par + n, flags);
        k_fit<<<nb, 256, 0, s>>>(px, py, pz, tri, n, out->tris, out->nodes, par, par + n, flags);
    }
    TRY(hipGetLastError());
    TRY(hipStreamSynchronize(s));
done:
#undef TRY
    (void)hipFree(kin);
    (void)hipFree(kout);
    (void)hipFree(box);
    (void)hipFree(par);
    (void)hipFree(flags);
    (void)hipFree(tmp);
    if (e != hipSuccess) bvh_free(out);
    return e;
}

void bvh_free(BvhStore* b)
{
    if (b->nodes) (void)hipFree(b->nodes);
    if (b->tris) (void)hipFree(b->tris);
    b->nodes = nullptr;
    b->tris = nullptr;
}

// ------------------------------------------------------------------ visibility

namespace {

struct D3 {
    double x, y, z;
};
__device__ __forceinline__ D3 d3(double x, double y, double z) { return D3{x, y, z}; }
__device__ __forceinline__ D3 operator-(D3 a, D3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ D3 operator+(D3 a, D3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ D3 operator*(D3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ double dot(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ D3 cross(D3 a, D3 b)
{
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// Moller-Trumbore in double: hit at segment parameter t in [teps, 1-teps]
// with closed barycentrics
__device__ __forceinline__ bool leaf_hit(const BvhTri& T, D3 p, D3 d, double teps)
{
    const D3 e1 = d3(T.e1[0], T.e1[1], T.e1[2]), e2 = d3(T.e2[0], T.e2[1], T.e2[2]);
    const D3 pv = cross(d, e2);
    const double det = dot(e1, pv);
    if (det == 0.0) return false;
    const D3 tv = p - d3(T.p0[0], T.p0[1], T.p0[2]);
    const double u = dot(tv, pv) / det;
    const D3 qv = cross(tv, e1);
    const double v = dot(d, qv) / det;
    const double t = dot(e2, qv) / det;
    return u >= 0.0 && v >= 0.0 && 1.0 - u - v >= 0.0 && t - teps >= 0.0 && 1.0 - teps - t >= 0.0;
}

struct FRay {
    float ox, oy, oz, ix, iy, iz;
};

__device__ __forceinline__ float safe_inv(float d) { return 1.0f / (fabsf(d) > 1e-30f ? d : 1e-30f); }

__device__ __forceinline__ bool slab(const FRay& r, const float* lo, const float* hi)
{
    const float tx0 = (lo[0] - r.ox) * r.ix, tx1 = (hi[0] - r.ox) * r.ix;
    const float ty0 = (lo[1] - r.oy) * r.iy, ty1 = (hi[1] - r.oy) * r.iy;
    const float tz0 = (lo[2] - r.oz) * r.iz, tz1 = (hi[2] - r.oz) * r.iz;
    const float tmin = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), -1e-4f));
    const float tmax = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fminf(fmaxf(tz0, tz1), 1.0001f));
    return tmin <= tmax;
}

// any-hit of the segment p -> q; `stack` is this lane's column of the block's
// LDS stack (stride kTailBlock)
__device__ bool blocked(const BvhView& B, D3 p, D3 q, int32_t skip_a, int32_t skip_b, double teps, int32_t* stack,
                        bool& overflow)
{
    const D3 d = q - p;
    if (B.n_tris == 1) {
        const BvhTri T = B.tris[0];
        return T.id != skip_a && T.id != skip_b && leaf_hit(T, p, d, teps);
    }
    FRay r;
    r.ox = float(p.x);
    r.oy = float(p.y);
    r.oz = float(p.z);
    r.ix = safe_inv(float(d.x));
    r.iy = safe_inv(float(d.y));
    r.iz = safe_inv(float(d.z));
    int sp = 0;
    int32_t node = 0;
    // every internal node is visited at most once per segment
    for (int32_t visits = 0; visits <= B.n_tris; ++visits) {
        const float4* raw = reinterpret_cast<const float4*>(B.nodes + node);
        const float4 a = raw[0], b = raw[1], c = raw[2];
        const int4 ch = *reinterpret_cast<const int4*>(raw + 3);
        const float lo0[3] = {a.x, a.y, a.z}, hi0[3] = {a.w, b.x, b.y};
        const float lo1[3] = {b.z, b.w, c.x}, hi1[3] = {c.y, c.z, c.w};
        bool h0 = slab(r, lo0, hi0), h1 = slab(r, lo1, hi1);
        if (h0 && ch.x < 0) {
            const BvhTri T = B.tris[~ch.x];
            if (T.id != skip_a && T.id != skip_b && leaf_hit(T, p, d, teps)) return true;
            h0 = false;
        }
        if (h1 && ch.y < 0) {
            const BvhTri T = B.tris[~ch.y];
            if (T.id != skip_a && T.id != skip_b && leaf_hit(T, p, d, teps)) return true;
            h1 = false;
        }
        if (h0 && h1) {
            if (sp == kBvhStack) {
                overflow = true;
                return false;
            }
            stack[sp++ * kTailBlock] = ch.y;
            node = ch.x;
        } else if (h0) {
            node = ch.x;
        } else if (h1) {
            node = ch.y;
        } else {
            if (sp == 0) return false;
            node = stack[--sp * kTailBlock];
        }
    }
    overflow = true;
    return false;
}

// ------------------------------------------------------------------ contribution

// forward-mode dual number with N tangent directions
template <int N>
struct Dn {
    double v;
    double d[N];
};
template <int N>
__device__ __forceinline__ Dn<N> dconst(double x)
{
    Dn<N> r;
    r.v = x;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = 0.0;
    return r;
}
template <int N>
__device__ __forceinline__ Dn<N> operator+(const Dn<N>& a, const Dn<N>& b)
{
    Dn<N> r;
    r.v = a.v + b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
    return r;
}
template <int N>
__device__ __forceinline__ Dn<N> operator-(const Dn<N>& a, const Dn<N>& b)
{
    Dn<N> r;
    r.v = a.v - b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
    return r;
}
template <int N>
__device__ __forceinline__ Dn<N> operator*(const Dn<N>& a, const Dn<N>& b)
{
    Dn<N> r;
    r.v = a.v * b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
    return r;
}
template <int N>
__device__ __forceinline__ Dn<N> operator*(const Dn<N>& a, double s)
{
    Dn<N> r;
    r.v = a.v * s;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * s;
    return r;
}
template <int N>
__device__ __forceinline__ Dn<N> rsqrt_d(const Dn<N>& a)  // a^(-1/2)
{
    Dn<N> r;
    r.v = 1.0 / sqrt(a.v);
    const double k = -0.5 * r.v / a.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = k * a.d[i];
    return r;
}

template <int N>
struct DV {
    Dn<N> x, y, z;
};
template <int N>
__device__ __forceinline__ DV<N> operator-(const DV<N>& a, const DV<N>& b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <int N>
__device__ __forceinline__ DV<N> operator+(const DV<N>& a, const DV<N>& b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <int N>
__device__ __forceinline__ DV<N> scale(const DV<N>& a, const Dn<N>& s) { return {a.x * s, a.y * s, a.z * s}; }
template <int N>
__device__ __forceinline__ DV<N> scale(const DV<N>& a, double s) { return {a.x * s, a.y * s, a.z * s}; }
template <int N>
__device__ __forceinline__ Dn<N> ddot(const DV<N>& a, const DV<N>& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <int N>
__device__ __forceinline__ Dn<N> ddot(const DV<N>& a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <int N>
__device__ __forceinline__ DV<N> dcross(const DV<N>& a, const DV<N>& b)
{
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <int N>
__device__ __forceinline__ DV<N> dunit(const DV<N>& a) { return scale(a, rsqrt_d(ddot(a, a))); }

// base + du * e1 + dv * e2 with (du, dv) the tangent directions iu, iu + 1
template <int N>
__device__ __forceinline__ DV<N> affine(D3 base, D3 e1, D3 e2, double u, double v, int iu)
{
    DV<N> r;
    r.x = dconst<N>(base.x + u * e1.x + v * e2.x);
    r.y = dconst<N>(base.y + u * e1.y + v * e2.y);
    r.z = dconst<N>(base.z + u * e1.z + v * e2.z);
    r.x.d[iu] = e1.x;
    r.x.d[iu + 1] = e2.x;
    r.y.d[iu] = e1.y;
    r.y.d[iu + 1] = e2.y;
    r.z.d[iu] = e1.z;
    r.z.d[iu + 1] = e2.z;
    return r;
}

struct TriG {
    D3 p0, e1, e2, n0, dn1, dn2;
};

__device__ __forceinline__ TriG load_trig(const TailArgs& A, int32_t t)
{
    TriG g;
    D3 p[3], n[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int32_t v = A.tri[3 * t + j];
        p[j] = d3(A.px[v], A.py[v], A.pz[v]);
        n[j] = d3(A.nx[v], A.ny[v], A.nz[v]);
    }
    g.p0 = p[0];
    g.e1 = p[1] - p[0];
    g.e2 = p[2] - p[0];
    g.n0 = n[0];
    g.dn1 = n[1] - n[0];
    g.dn2 = n[2] - n[0];
    return g;
}

// unpolarised Fresnel transmittance from index n1 into n2 at incidence cosine ci
__device__ __forceinline__ double fresnel_t(double n1, double n2, double ci)
{
    ci = fabs(ci);
    const double r = n1 / n2;
    const double st2 = r * r * (1.0 - ci * ci);
    if (st2 >= 1.0) return 0.0;
    const double ct = sqrt(1.0 - st2);
    const double a = n1 * ci, b = n2 * ct, c = n2 * ci, e = n1 * ct;
    const double rs = (a - b) / (a + b), rp = (c - e) / (c + e);
    return 1.0 - 0.5 * (rs * rs + rp * rp);
}

// orthonormal pair spanning the plane normal to unit w
__device__ __forceinline__ void plane_basis(D3 w, D3& a, D3& b)
{
    const double sg = copysign(1.0, w.z);
    const double k = -1.0 / (sg + w.z);
    const double m = w.x * w.y * k;
    a = d3(1.0 + sg * w.x * w.x * k, sg * m, -sg * w.x);
    b = d3(m, sg + w.y * w.y * k, -w.y);
}

// dw/dA of a chain of K vertices; false when the constraint Jacobian is singular
template <int K>
__device__ bool solid_angle_per_area(const TailArgs& A, const TriG* T, const double* u, const double* v, D3 x0,
                                     D3 xl, double& out)
{
    constexpr int N = 2 * K + 2;  // (u_i, v_i) of every vertex, then (s, t) on the receiver plane
    DV<N> x[K + 2];
    const D3 w0 = [&] {
        const D3 x1 = T[0].p0 + T[0].e1 * u[0] + T[0].e2 * v[0];
        const D3 d = x1 - x0;
        return d * (1.0 / sqrt(dot(d, d)));
    }();
    D3 fa, fb;
    plane_basis(w0, fa, fb);
    x[0] = affine<N>(x0, fa, fb, 0.0, 0.0, 2 * K);
#pragma unroll
    for (int i = 0; i < K; ++i) x[i + 1] = affine<N>(T[i].p0, T[i].e1, T[i].e2, u[i], v[i], 2 * i);
    x[K + 1].x = dconst<N>(xl.x);
    x[K + 1].y = dconst<N>(xl.y);
    x[K + 1].z = dconst<N>(xl.z);

    double J[2 * K][2 * K + 2];  // [J | K] rows of the constraints
#pragma unroll
    for (int i = 1; i <= K; ++i) {
        const TriG& g = T[i - 1];
        const DV<N> nrm = affine<N>(g.n0, g.dn1, g.dn2, u[i - 1], v[i - 1], 2 * (i - 1));
        const DV<N> wi = dunit(x[i - 1] - x[i]), wo = dunit(x[i + 1] - x[i]);
        const DV<N> h = scale(wi, A.eta[i - 1]) + scale(wo, A.eta[i]);
        const DV<N> c = dcross(h, nrm);
        const Dn<N> c0 = ddot(c, g.e1), c1 = ddot(c, g.e2);
#pragma unroll
        for (int j = 0; j < N; ++j) {
            J[2 * (i - 1)][j] = c0.d[j];
            J[2 * (i - 1) + 1][j] = c1.d[j];
        }
    }
    // Gaussian elimination with partial pivoting on [J | K]; X = -J^-1 K
    constexpr int M = 2 * K;
    double scale_j = 0.0;
#pragma unroll
    for (int r = 0; r < M; ++r)
#pragma unroll
        for (int c = 0; c < M; ++c) scale_j = fmax(scale_j, fabs(J[r][c]));
    if (!(scale_j > 0.0)) return false;
#pragma unroll
    for (int c = 0; c < M; ++c) {
        int piv = c;
#pragma unroll
        for (int r = c + 1; r < M; ++r)
            if (fabs(J[r][c]) > fabs(J[piv][c])) piv = r;
        if (!(fabs(J[piv][c]) > 1e-14 * scale_j)) return false;
        if (piv != c) {
#pragma unroll
            for (int j = 0; j < M + 2; ++j) {
                const double t = J[c][j];
                J[c][j] = J[piv][j];
                J[piv][j] = t;
            }
        }
        const double inv = 1.0 / J[c][c];
#pragma unroll
        for (int r = c + 1; r < M; ++r) {
            const double f = J[r][c] * inv;
#pragma unroll
            for (int j = c; j < M + 2; ++j) J[r][j] -= f * J[c][j];
        }
    }
    double X[M][2];
#pragma unroll
    for (int r = M - 1; r >= 0; --r)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            double s = -J[r][M + q];
#pragma unroll
            for (int c = r + 1; c < M; ++c) s -= J[r][c] * X[c][q];
            X[r][q] = s / J[r][r];
        }
    const TriG& gk = T[K - 1];
    const D3 dxs = gk.e1 * X[M - 2][0] + gk.e2 * X[M - 1][0];
    const D3 dxt = gk.e1 * X[M - 2][1] + gk.e2 * X[M - 1][1];
    const D3 xk = gk.p0 + gk.e1 * u[K - 1] + gk.e2 * v[K - 1];
    const D3 r = xk - xl;
    const double r2 = dot(r, r);
    out = fabs(dot(r, cross(dxs, dxt))) / (r2 * sqrt(r2));
    return true;
}

template <int K>
__global__ __launch_bounds__(kTailBlock) void k_tail(TailArgs A)
{
    __shared__ int32_t stack[kBvhStack * kTailBlock];
    const int64_t p = int64_t(blockIdx.x) * kTailBlock + threadIdx.x;
    int64_t n = A.n;
    if (A.count) n = min(n, int64_t(*A.count));
    if (p >= n) return;
    const spoly_solution s = A.sols[p];
    const int32_t j0 = A.q_x0[s.query], jl = A.q_xl[s.query];
    const D3 x0 = d3(A.x0x[j0], A.x0y[j0], A.x0z[j0]);
    const D3 xl = d3(A.xlx[jl], A.xly[jl], A.xlz[jl]);
    TriG T[K];
    D3 x[K + 2];
    double u[K], v[K];
    x[0] = x0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        T[i] = load_trig(A, s.tri[i]);
        u[i] = s.u[i];
        v[i] = s.v[i];
        x[i + 1] = T[i].p0 + T[i].e1 * u[i] + T[i].e2 * v[i];
    }
    x[K + 1] = xl;

    int32_t mask = 0;
    bool overflow = false;
#pragma unroll
    for (int seg = 0; seg <= K; ++seg) {
        const int32_t sa = seg >= 1 ? s.tri[seg - 1] : -1;
        const int32_t sb = seg < K ? s.tri[seg] : -1;
        if (blocked(A.bvh, x[seg], x[seg + 1], sa, sb, A.teps, stack + threadIdx.x, overflow)) mask |= 1 << seg;
    }
    if (overflow) mask |= kTailOverflow;

    double F = 1.0;
#pragma unroll
    for (int i = 1; i <= K; ++i) {
        if (A.ev[i - 1] == SPOLY_R) {
            F *= A.rho;
            continue;
        }
        const D3 nn = T[i - 1].n0 + T[i - 1].dn1 * u[i - 1] + T[i - 1].dn2 * v[i - 1];
        const D3 wl = x[i + 1] - x[i];
        F *= fresnel_t(A.eta[i], A.eta[i - 1], dot(wl, nn) / sqrt(dot(wl, wl) * dot(nn, nn)));
    }
    double g = 0.0;
    if (!solid_angle_per_area<K>(A, T, u, v, x0, xl, g)) mask |= kTailSingular;
    const double E = A.intensity * F * g;
    if (A.mask) A.mask[p] = mask;
    if (A.contrib) A.contrib[p] = E;
    if (A.image && mask == 0 && E > 0.0) {
        double w = E;
        if (A.use_rn) {
            const D3 d = x[1] - x0;
            w *= fabs(d.x * A.rn[0] + d.y * A.rn[1] + d.z * A.rn[2]) / sqrt(dot(d, d));
        }
        atomicAdd(A.image + j0, w);
    }
}

}  // namespace

hipError_t launch_tail(const TailArgs& A, hipStream_t s)
{
    if (A.n == 0) return hipSuccess;
    const dim3 grid(unsigned((A.n + kTailBlock - 1) / kTailBlock));
    if (A.k == 1)
        k_tail<1><<<grid, kTailBlock, 0, s>>>(A);
    else
        k_tail<2><<<grid, kTailBlock, 0, s>>>(A);
    return hipGetLastError();
}

}  // namespace spoly
