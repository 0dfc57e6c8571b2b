// Deterministic output order.  The solves reserve output slots with atomics,
// so the order of their records depends on scheduling.  Sorting them by
// (query, v[0], u[0]) gives one order for one input: three stable radix
// passes over a permutation, least significant key first (u, then v, then
// the query), each key gathered through the permutation so far; records past
// the device count take the largest key and stay at the end.  Within one
// query the triangles are fixed, so the query orders them too.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include "order.hpp"

namespace spoly {

namespace {

// monotone map of a double onto unsigned 64-bit keys
__device__ __forceinline__ unsigned long long ordered_bits(double x)
{
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(x));
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__device__ __forceinline__ int64_t valid_count(const unsigned long long* count, int64_t cap)
{
    const unsigned long long c = *count;
    return c < static_cast<unsigned long long>(cap) ? static_cast<int64_t>(c) : cap;
}

// key of record perm[i] (identity when perm is null): which = 0 u[0], 1 v[0]
__global__ void k_key_f64(const spoly_solution* out, int64_t cap, const unsigned long long* count,
                          const int32_t* perm, int which, unsigned long long* keys, int32_t* ids)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= cap) return;
    const int32_t id = perm ? perm[i] : int32_t(i);
    const int64_t n = valid_count(count, cap);
    keys[i] = id < n ? ordered_bits(which == 0 ? out[id].u[0] : out[id].v[0]) : ~0ull;
    ids[i] = id;
}

__global__ void k_key_query(const spoly_solution* out, int64_t cap, const unsigned long long* count,
                            const int32_t* perm, uint32_t* keys, int32_t* ids)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= cap) return;
    const int32_t id = perm[i];
    const int64_t n = valid_count(count, cap);
    keys[i] = id < n ? static_cast<uint32_t>(out[id].query) : 0xffffffffu;
    ids[i] = id;
}

__global__ void k_copy_records(const spoly_solution* src, spoly_solution* dst, int64_t cap,
                               const unsigned long long* count)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < valid_count(count, cap)) dst[i] = src[i];
}

__global__ void k_gather_records(const spoly_solution* src, const int32_t* perm, spoly_solution* dst, int64_t cap,
                                 const unsigned long long* count)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < valid_count(count, cap)) dst[i] = src[perm[i]];
}

struct Carve {
    unsigned long long *k0, *k1;  // 64-bit keys (the query pass uses their first half)
    int32_t *p0, *p1;             // permutation, ping-pong
    spoly_solution* copy;
    void* tmp;
    size_t tmp_bytes;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

size_t radix_tmp_bytes(int64_t cap)
{
    size_t a = 0, b = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, a, static_cast<unsigned long long*>(nullptr),
                                             static_cast<unsigned long long*>(nullptr), static_cast<int32_t*>(nullptr),
                                             static_cast<int32_t*>(nullptr), int(cap), 0, 64);
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, b, static_cast<uint32_t*>(nullptr),
                                             static_cast<uint32_t*>(nullptr), static_cast<int32_t*>(nullptr),
                                             static_cast<int32_t*>(nullptr), int(cap), 0, 32);
    return a > b ? a : b;
}

Carve carve(void* work, int64_t cap)
{
    char* p = static_cast<char*>(work);
    Carve c;
    c.k0 = reinterpret_cast<unsigned long long*>(p);
    p += align256(8 * size_t(cap));
    c.k1 = reinterpret_cast<unsigned long long*>(p);
    p += align256(8 * size_t(cap));
    c.p0 = reinterpret_cast<int32_t*>(p);
    p += align256(4 * size_t(cap));
    c.p1 = reinterpret_cast<int32_t*>(p);
    p += align256(4 * size_t(cap));
    c.copy = reinterpret_cast<spoly_solution*>(p);
    p += align256(sizeof(spoly_solution) * size_t(cap));
    c.tmp = p;
    c.tmp_bytes = radix_tmp_bytes(cap);
    return c;
}

}  // namespace

size_t sort_solutions_bytes(int64_t cap)
{
    if (cap <= 0) return 0;
    return 2 * align256(8 * size_t(cap)) + 2 * align256(4 * size_t(cap)) +
           align256(sizeof(spoly_solution) * size_t(cap)) + align256(radix_tmp_bytes(cap));
}

hipError_t sort_solutions(spoly_solution* out, int64_t cap, const unsigned long long* count, void* work,
                          size_t work_bytes, hipStream_t s)
{
    if (cap <= 0) return hipSuccess;
    if (cap > INT32_MAX || work_bytes < sort_solutions_bytes(cap)) return hipErrorInvalidValue;
    Carve c = carve(work, cap);
    const unsigned nb = unsigned((cap + 255) / 256);
    size_t tb = c.tmp_bytes;
    hipError_t e;
    // pass 1: u[0]
    k_key_f64<<<nb, 256, 0, s>>>(out, cap, count, nullptr, 0, c.k0, c.p0);
    e = hipcub::DeviceRadixSort::SortPairs(c.tmp, tb, c.k0, c.k1, c.p0, c.p1, int(cap), 0, 64, s);
    if (e != hipSuccess) return e;
    // pass 2: v[0] of the records in the order so far
    k_key_f64<<<nb, 256, 0, s>>>(out, cap, count, c.p1, 1, c.k0, c.p0);
    e = hipcub::DeviceRadixSort::SortPairs(c.tmp, tb, c.k0, c.k1, c.p0, c.p1, int(cap), 0, 64, s);
    if (e != hipSuccess) return e;
    // pass 3: the query
    uint32_t* q0 = reinterpret_cast<uint32_t*>(c.k0);
    uint32_t* q1 = reinterpret_cast<uint32_t*>(c.k1);
    k_key_query<<<nb, 256, 0, s>>>(out, cap, count, c.p1, q0, c.p0);
    e = hipcub::DeviceRadixSort::SortPairs(c.tmp, tb, q0, q1, c.p0, c.p1, int(cap), 0, 32, s);
    if (e != hipSuccess) return e;
    k_copy_records<<<nb, 256, 0, s>>>(out, c.copy, cap, count);
    k_gather_records<<<nb, 256, 0, s>>>(c.copy, c.p1, out, cap, count);
    return hipGetLastError();
}

}  // namespace spoly
