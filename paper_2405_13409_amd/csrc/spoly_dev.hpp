// Device-side building blocks of the gfx950 specular-polynomial kernels:
// 3-vectors, bivariate polynomials of compile-time degree in registers, and
// wave64 scan / compaction primitives.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/spoly.h"

namespace spoly {

constexpr int kWave = 64;

// ------------------------------------------------------------------ vectors
template <typename R>
struct V3 {
    R x, y, z;
};
template <typename R>
__device__ __forceinline__ V3<R> mk(R x, R y, R z) { return V3<R>{x, y, z}; }
template <typename R>
__device__ __forceinline__ V3<R> operator+(V3<R> a, V3<R> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <typename R>
__device__ __forceinline__ V3<R> operator-(V3<R> a, V3<R> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <typename R>
__device__ __forceinline__ V3<R> operator*(V3<R> a, R s) { return {a.x * s, a.y * s, a.z * s}; }
template <typename R>
__device__ __forceinline__ R dot(V3<R> a, V3<R> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <typename R>
__device__ __forceinline__ V3<R> cross(V3<R> a, V3<R> b)
{
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <typename R>
__device__ __forceinline__ R len(V3<R> a) { return sqrt(dot(a, a)); }
template <typename R>
__device__ __forceinline__ V3<R> normalized(V3<R> a)
{
    R l = len(a);
    return l > R(0) ? a * (R(1) / l) : a;
}
template <typename R, typename S>
__device__ __forceinline__ V3<R> cvt(V3<S> a) { return {R(a.x), R(a.y), R(a.z)}; }

// ------------------------------------------------------------------ bivariate polynomials
// p(u,v) = sum_{i+j<=D} c[idx(i,j)] u^i v^j, triangular layout: row i (power of u)
// holds D-i+1 coefficients in increasing powers of v.
__host__ __device__ constexpr int tri_size(int D) { return (D + 1) * (D + 2) / 2; }
__host__ __device__ constexpr int tri_idx(int D, int i, int j) { return i * (D + 1) - i * (i - 1) / 2 + j; }

template <typename R, int D>
struct P2 {
    R c[tri_size(D)];
};

template <typename R, int D>
__device__ __forceinline__ P2<R, D> p2_zero()
{
    P2<R, D> p;
#pragma unroll
    for (int k = 0; k < tri_size(D); ++k) p.c[k] = R(0);
    return p;
}
// k0 + ku u + kv v
template <typename R>
__device__ __forceinline__ P2<R, 1> p2_lin(R k0, R ku, R kv)
{
    P2<R, 1> p;
    p.c[tri_idx(1, 0, 0)] = k0;
    p.c[tri_idx(1, 0, 1)] = kv;
    p.c[tri_idx(1, 1, 0)] = ku;
    return p;
}
template <typename R>
__device__ __forceinline__ P2<R, 0> p2_const(R k)
{
    P2<R, 0> p;
    p.c[0] = k;
    return p;
}

template <typename R, int D1, int D2>
__device__ __forceinline__ P2<R, D1 + D2> operator*(const P2<R, D1>& a, const P2<R, D2>& b)
{
    constexpr int D = D1 + D2;
    P2<R, D> r = p2_zero<R, D>();
#pragma unroll
    for (int i = 0; i <= D1; ++i)
#pragma unroll
        for (int j = 0; i + j <= D1; ++j)
#pragma unroll
            for (int k = 0; k <= D2; ++k)
#pragma unroll
                for (int l = 0; k + l <= D2; ++l)
                    r.c[tri_idx(D, i + k, j + l)] =
                        fma(a.c[tri_idx(D1, i, j)], b.c[tri_idx(D2, k, l)], r.c[tri_idx(D, i + k, j + l)]);
    return r;
}

template <int A, int B>
struct cmax {
    static constexpr int v = A > B ? A : B;
};

// sa*a + sb*b
template <typename R, int D1, int D2>
__device__ __forceinline__ P2<R, cmax<D1, D2>::v> lc(R sa, const P2<R, D1>& a, R sb, const P2<R, D2>& b)
{
    constexpr int D = cmax<D1, D2>::v;
    P2<R, D> r;
#pragma unroll
    for (int i = 0; i <= D; ++i)
#pragma unroll
        for (int j = 0; i + j <= D; ++j) {
            R x = (i + j <= D1) ? sa * a.c[tri_idx(D1, i, j)] : R(0);
            R y = (i + j <= D2) ? sb * b.c[tri_idx(D2, i, j)] : R(0);
            r.c[tri_idx(D, i, j)] = x + y;
        }
    return r;
}
template <typename R, int D1, int D2>
__device__ __forceinline__ P2<R, cmax<D1, D2>::v> operator+(const P2<R, D1>& a, const P2<R, D2>& b)
{
    return lc(R(1), a, R(1), b);
}
template <typename R, int D1, int D2>
__device__ __forceinline__ P2<R, cmax<D1, D2>::v> operator-(const P2<R, D1>& a, const P2<R, D2>& b)
{
    return lc(R(1), a, R(-1), b);
}
template <typename R, int D>
__device__ __forceinline__ P2<R, D> scale(const P2<R, D>& a, R s)
{
    P2<R, D> r;
#pragma unroll
    for (int k = 0; k < tri_size(D); ++k) r.c[k] = a.c[k] * s;
    return r;
}

// vectors of bivariate polynomials
template <typename R, int D>
struct VP {
    P2<R, D> x, y, z;
};
template <typename R>
__device__ __forceinline__ VP<R, 1> vp_affine(V3<R> p0, V3<R> eu, V3<R> ev)
{
    return {p2_lin(p0.x, eu.x, ev.x), p2_lin(p0.y, eu.y, ev.y), p2_lin(p0.z, eu.z, ev.z)};
}
template <typename R>
__device__ __forceinline__ VP<R, 0> vp_const(V3<R> c)
{
    return {p2_const(c.x), p2_const(c.y), p2_const(c.z)};
}
template <typename R, int D1, int D2>
__device__ __forceinline__ VP<R, cmax<D1, D2>::v> operator-(const VP<R, D1>& a, const VP<R, D2>& b)
{
    return {a.x - b.x, a.y - b.y, a.z - b.z};
}
template <typename R, int D1, int D2>
__device__ __forceinline__ P2<R, D1 + D2> vdot(const VP<R, D1>& a, const VP<R, D2>& b)
{
    return a.x * b.x + a.y * b.y + a.z * b.z;
}
template <typename R, int D1, int D2>
__device__ __forceinline__ VP<R, D1 + D2> vcross(const VP<R, D1>& a, const VP<R, D2>& b)
{
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
// component along a coordinate axis (0,1,2)
template <typename R, int D>
__device__ __forceinline__ P2<R, D> vcomp(const VP<R, D>& a, int axis)
{
    P2<R, D> r;
#pragma unroll
    for (int k = 0; k < tri_size(D); ++k) r.c[k] = axis == 0 ? a.x.c[k] : (axis == 1 ? a.y.c[k] : a.z.c[k]);
    return r;
}

// ------------------------------------------------------------------ univariate
template <typename R, int D>
__device__ __forceinline__ R horner(const R (&c)[D + 1], R x)
{
    R s = c[D];
#pragma unroll
    for (int k = D - 1; k >= 0; --k) s = fma(s, x, c[k]);
    return s;
}

// binomial coefficient C(n, k) as a double (exact for the small n used here)
__host__ __device__ constexpr double binom(int n, int k)
{
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * double(n - k + i) / double(i);
    return r;
}

// ------------------------------------------------------------------ wave64 primitives
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// inclusive prefix sum over the 64 lanes of a wave (all lanes must participate)
__device__ __forceinline__ int wave_incl_scan(int x)
{
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        int y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    return x;
}
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x)
{
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, kWave);
    return x;
}

// Output reservation shared by the waves of a block: every wave passes its
// total; one atomic on *counter per block (instead of one per wave) returns
// the block's base, and each wave receives base + the totals of the waves
// before it.  All threads of the block must call it (it synchronises the
// block); `slots` is LDS space for kMaxBlockWaves + 1 values.
constexpr int kMaxBlockWaves = 16;
__device__ __forceinline__ unsigned long long block_reserve(unsigned long long wave_total, unsigned long long* counter,
                                                            unsigned long long* slots)
{
    const int w = threadIdx.x / kWave;
    const int nw = (blockDim.x + kWave - 1) / kWave;
    if (lane_id() == 0) slots[w] = wave_total;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long sum = 0;
        for (int i = 0; i < nw; ++i) sum += slots[i];
        slots[kMaxBlockWaves] = sum ? atomicAdd(counter, sum) : 0ull;
    }
    __syncthreads();
    unsigned long long base = slots[kMaxBlockWaves];
    for (int i = 0; i < w; ++i) base += slots[i];
    __syncthreads();   // slots may be reused after this call
    return base;
}

}  // namespace spoly
