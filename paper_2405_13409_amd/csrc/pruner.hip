// Learned pruner of two-vertex tuples.  An MLP 42 -> 128 -> 128 -> 128 -> 1
// (ReLU, sigmoid) scores each (x0, T1, T2, x3) tuple from the separators and
// the positions / normals of both triangles; tuples scoring below a
// calibrated threshold are not sent to the solver.  Dense layers run on the
// matrix cores: bf16 operands, fp32 accumulation (v_mfma_f32_16x16x32_bf16;
// the scorer takes its last 16 inputs in one v_mfma_f32_16x16x16_bf16 step).
//   training : k_gather -> 4 x (GEMM, bias/ReLU) -> loss gradient -> backward
//              GEMMs (split-K for weight gradients) -> Adam
//   inference: one fused kernel, weights staged in LDS, two 16-tuple tiles per wave.
#include <hip/hip_bf16.h>

#include "spoly_dev.hpp"
#include "pruner.hpp"

namespace spoly {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float f)
{
    // round to nearest even
    unsigned int u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);  // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

// ------------------------------------------------------------------ features
// 42 features: x0/2, x3/2, the three positions of T1 and of T2 divided by 2,
// the three vertex normals of T1 and of T2 (as given).  Padded to kFeat = 48.
__global__ void __launch_bounds__(256) k_gather(PrunerIO io, unsigned short* X, float* Xf)
{
    const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= io.n) return;
    float f[kFeat];
#pragma unroll
    for (int k = 0; k < kFeat; ++k) f[k] = 0.0f;
    const int j0 = io.q_x0[q], j3 = io.q_x3[q];
    const int t1 = io.q_tris[2 * q], t2 = io.q_tris[2 * q + 1];
    f[0] = float(io.x0x[j0] * 0.5); f[1] = float(io.x0y[j0] * 0.5); f[2] = float(io.x0z[j0] * 0.5);
    f[3] = float(io.x3x[j3] * 0.5); f[4] = float(io.x3y[j3] * 0.5); f[5] = float(io.x3z[j3] * 0.5);
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        const int a = io.tri[3 * t1 + v], b = io.tri[3 * t2 + v];
        f[6 + 3 * v + 0] = float(io.px[a] * 0.5); f[6 + 3 * v + 1] = float(io.py[a] * 0.5); f[6 + 3 * v + 2] = float(io.pz[a] * 0.5);
        f[15 + 3 * v + 0] = float(io.px[b] * 0.5); f[15 + 3 * v + 1] = float(io.py[b] * 0.5); f[15 + 3 * v + 2] = float(io.pz[b] * 0.5);
        f[24 + 3 * v + 0] = float(io.nx[a]); f[24 + 3 * v + 1] = float(io.ny[a]); f[24 + 3 * v + 2] = float(io.nz[a]);
        f[33 + 3 * v + 0] = float(io.nx[b]); f[33 + 3 * v + 1] = float(io.ny[b]); f[33 + 3 * v + 2] = float(io.nz[b]);
    }
#pragma unroll
    for (int k = 0; k < kFeat; ++k) {
        X[q * kFeat + k] = f2bf(f[k]);
        if (Xf) Xf[q * kFeat + k] = f[k];
    }
}

// ------------------------------------------------------------------ generic bf16 GEMM on MFMA
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

// C(m,n) (+)= sum_k A(m,k) B(k,n), A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn],
// fp32 C row-major with leading dimension ldc.  64x64 tile per workgroup
// (2x2 waves of 32x32, each 2x2 instructions of 16x16x32), K in steps of 32;
// blockIdx.z splits K: partial sums go to G.part when it is set (summed in
// order by k_split_sum), else they are added atomically (C zeroed by the
// caller).  Each step stages A as [m][k] and B as [n][k] in LDS, read from
// global memory along whichever index is unit-stride so the loads coalesce;
// a lane's fragment -- row (lane & 15), eight consecutive k -- is then one
// 16-byte LDS read.  Rows are padded to 40 bf16 so that the 16 rows a
// quarter-wave reads start in distinct bank groups.
constexpr int kGemmLd = 32 + 8;

__global__ void __launch_bounds__(256) k_gemm(GemmArgs G)
{
    __shared__ __attribute__((aligned(16))) unsigned short As[64 * kGemmLd], Bs[64 * kGemmLd];
    const int lane = lane_id();
    const int w = threadIdx.x / kWave;
    const int bm = blockIdx.y * 64, bn = blockIdx.x * 64;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    const int kchunk = ((G.K + gridDim.z - 1) / gridDim.z + 31) & ~31;
    const int kbeg = blockIdx.z * kchunk;
    const int kend = min(G.K, kbeg + kchunk);
    const bool a_kfast = G.sak == 1, b_kfast = G.sbk == 1;
    v4f acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    const int r = lane & 15, k8 = (lane >> 4) * 8, kq = (lane >> 4) * 4;
    for (int k0 = kbeg; k0 < kend; k0 += 32) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int e = threadIdx.x + 256 * i;   // 0 .. 64*32-1
            const int am = a_kfast ? e >> 5 : e & 63, ak = a_kfast ? e & 31 : e >> 6;
            const int gm = bm + am, gka = k0 + ak;
            As[am * kGemmLd + ak] =
                (gm < G.M && gka < kend) ? G.A[int64_t(gm) * G.sam + int64_t(gka) * G.sak] : (unsigned short)0;
            const int bnn = b_kfast ? e >> 5 : e & 63, bk = b_kfast ? e & 31 : e >> 6;
            const int gn = bn + bnn, gkb = k0 + bk;
            Bs[bnn * kGemmLd + bk] =
                (gn < G.N && gkb < kend) ? G.B[int64_t(gkb) * G.sbk + int64_t(gn) * G.sbn] : (unsigned short)0;
        }
        __syncthreads();
        bf8v af[2], bfr[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            af[t] = *reinterpret_cast<const bf8v*>(As + (wm + 16 * t + r) * kGemmLd + k8);
            bfr[t] = *reinterpret_cast<const bf8v*>(Bs + (wn + 16 * t + r) * kGemmLd + k8);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    // D fragment: lane holds column (lane & 15), rows 4 (lane >> 4) + i
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = bm + wm + 16 * i + kq + e;
                const int n = bn + wn + 16 * j + r;
                if (m < G.M && n < G.N) {
                    float* c = G.C + int64_t(m) * G.ldc + n;
                    if (G.part) G.part[(int64_t(blockIdx.z) * G.M + m) * G.N + n] = acc[i][j][e];
                    else if (gridDim.z > 1) atomicAdd(c, G.alpha * acc[i][j][e]);
                    else *c = G.alpha * acc[i][j][e] + (G.accumulate ? *c : 0.0f);
                }
            }
}

// C = alpha * (sum of the split partials, in split order) (+ C)
__global__ void k_split_sum(GemmArgs G, int split)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t mn = int64_t(G.M) * G.N;
    if (i >= mn) return;
    float acc = 0.0f;
    for (int z = 0; z < split; ++z) acc += G.part[z * mn + i];
    float* c = G.C + (i / G.N) * G.ldc + (i % G.N);
    *c = G.alpha * acc + (G.accumulate ? *c : 0.0f);
}

hipError_t launch_gemm(const GemmArgs& G, int split_k, hipStream_t stream)
{
    if (G.M <= 0 || G.N <= 0 || G.K <= 0) return hipSuccess;
    const int split = split_k < 1 ? 1 : split_k;
    // the partials buffer holds kGemmSplitMax tiles of at most kHid x kHid
    if (G.part && (split > kGemmSplitMax || int64_t(G.M) * G.N > int64_t(kHid) * kHid)) return hipErrorInvalidValue;
    dim3 grid((G.N + 63) / 64, (G.M + 63) / 64, split);
    hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, stream, G);
    if (G.part) {
        const int64_t mn = int64_t(G.M) * G.N;
        hipLaunchKernelGGL(k_split_sum, dim3(unsigned((mn + 255) / 256)), dim3(256), 0, stream, G, split);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ elementwise pieces of training
// Z (fp32, [n x ncol]) += bias; H = relu(Z) in bf16 (row stride ncol)
__global__ void k_bias_relu(float* Z, const float* bias, unsigned short* H, int64_t n, int ncol, int relu)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n * ncol) return;
    const int c = int(i % ncol);
    float z = Z[i] + bias[c];
    Z[i] = z;
    if (H) H[i] = f2bf(relu ? fmaxf(z, 0.0f) : z);
}

// logits z = Z4[:, 0]; weighted BCE; dZ4 (bf16, [n x 16], col 0) = d loss / d z
__global__ void k_loss(const float* Z4, int ld, const float* b4, const float* labels, int64_t n, float pos_w,
                       float inv_norm, unsigned short* dZ4, float* dz_f32, float* loss)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    float l = 0.0f;
    if (i < n) {
        const float z = Z4[i * ld] + b4[0];
        const float y = labels[i];
        const float p = 1.0f / (1.0f + expf(-z));
        const float w = y > 0.5f ? pos_w : 1.0f;
        // -[w y log p + (1-y) log(1-p)] with log p = -softplus(-z), log(1-p) = -softplus(z)
        const float sp_neg = fmaxf(-z, 0.0f) + log1pf(expf(-fabsf(z)));
        const float sp_pos = fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z)));
        l = (w * y * sp_neg + (1.0f - y) * sp_pos) * inv_norm;
        const float g = (w * y * (p - 1.0f) + (1.0f - y) * p) * inv_norm;
#pragma unroll
        for (int c = 0; c < 16; ++c) dZ4[i * 16 + c] = c == 0 ? f2bf(g) : (unsigned short)0;
        if (dz_f32) dz_f32[i] = g;
    }
    float tot = l;
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) tot += __shfl_xor(tot, d, kWave);
    if (lane_id() == 0 && tot != 0.0f) atomicAdd(loss, tot);
}

// dZ = dH * (Z > 0) -> bf16
__global__ void k_relu_bwd(const float* dH, const float* Z, unsigned short* dZ, int64_t cnt)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= cnt) return;
    dZ[i] = f2bf(Z[i] > 0.0f ? dH[i] : 0.0f);
}

// column sums of a bf16 matrix [n x ncol] (row stride ld) into db (fp32, accumulated)
__global__ void k_colsum(const unsigned short* D, int64_t n, int ncol, int ld, float* db)
{
    const int c = blockIdx.x;
    float s = 0.0f;
    for (int64_t r = threadIdx.x; r < n; r += blockDim.x) s += bf2f(D[r * ld + c]);
    __shared__ float red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) db[c] += red[0];
}

// fp32 master parameters -> bf16 operand copies (weights stored [in x out] row-major)
__global__ void k_to_bf16(const float* p, unsigned short* q, int64_t n)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) q[i] = f2bf(p[i]);
}

__global__ void k_fill(float* p, int64_t n, float v)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ------------------------------------------------------------------ fused inference
// Two 16-tuple tiles per wave, activations kept in registers: every layer
// computes H^T = W^T X^T on the matrix cores (weights as the A operand, the
// tile's activations as B), 32 inputs per instruction.  A 16x16 D fragment
// leaves lane l with tuple l & 15 and output neurons 4 (l >> 4) .. + 3 of its
// 16-neuron tile; the two D fragments of neurons 32c .. 32c + 31 together give
// each lane the eight values the next layer's B fragment of k-chunk c needs,
// if that layer's weight columns are stored in the matching order (kperm), so
// no activation goes through LDS.  The k order inside an instruction does not
// matter to the sum as long as A and B agree on it, which they do: both take
// a lane's eight values in the same slots.  Weights and biases sit in LDS,
// transposed to [out][in] so that a lane's eight k of an A fragment are one
// 16-byte read, which serves both tiles' instructions; the output layer's
// row 0 leaves each tuple's logit in lanes 0..15.
// Weight rows are padded by 8 bf16 (16 bytes): with 128 bf16 per row the 16
// rows a quarter-wave reads at one k offset would sit 256 bytes apart, all in
// the same LDS banks; padded, the reads of a quarter-wave cover all 64 banks
// once.
constexpr int kS1 = kFeat + 8, kS2 = kHid + 8;
constexpr int kW1 = kHid * kS1, kW2 = kHid * kS2, kW4 = 16 * kS2;
constexpr int kPruneWaves = 12, kPruneTiles = 2;
constexpr int kPruneLds = (kW1 + 2 * kW2 + kW4) * 2 + 4 * kHid * 4;

typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef float f8v __attribute__((ext_vector_type(8)));

// four floats as a bf16 fragment (round to nearest even, native conversion)
__device__ __forceinline__ v4s frag4(float a, float b, float c, float d)
{
    const bf2v lo = __builtin_convertvector((f2v){a, b}, bf2v);
    const bf2v hi = __builtin_convertvector((f2v){c, d}, bf2v);
    uint2 u;
    u.x = __builtin_bit_cast(unsigned int, lo);
    u.y = __builtin_bit_cast(unsigned int, hi);
    return __builtin_bit_cast(v4s, u);
}

// Storage slot -> hidden neuron of a weight row whose inputs are the previous
// layer's activations: slot 32c + 8g + p holds neuron 32c + 4g + (p & 3) +
// 16 (p >> 2), the neuron a lane of group g holds in element p of its k-chunk
// c fragment (elements 0..3 from D tile 2c, 4..7 from D tile 2c + 1).
__device__ __forceinline__ int kperm(int slot)
{
    const int c = slot >> 5, g = (slot >> 3) & 3, p = slot & 7;
    return 32 * c + 4 * g + (p & 3) + 16 * (p >> 2);
}

// First-layer input slot -> feature index (-1: zero).  The sum over inputs
// does not care about their order, so each lane's twelve slots are chosen to
// be contiguous in memory: slots 8g .. 8g + 7 are floats (g & 1) * 8 .. + 7 of
// the feature row of T1 (g < 2) or T2 (g >= 2), and slots 32 + 4g .. + 3 are
// x0/2 (g = 0), the row's last two floats (g = 1: T1, g = 3: T2) or x3/2
// (g = 2).  A row holds positions/2 (9 floats) then normals (9); features are
// x0/2, x3/2, T1 positions, T2 positions, T1 normals, T2 normals.
__device__ __forceinline__ int scorer_feature(int slot)
{
    if (slot < 32) {
        const int g = slot >> 3, e = (g & 1) * 8 + (slot & 7);
        return e < 9 ? (g < 2 ? 6 : 15) + e : (g < 2 ? 24 : 33) + e - 9;
    }
    if (slot >= 48) return -1;
    const int g = (slot - 32) >> 2, p = slot & 3;
    if (g == 0 || g == 2) return p < 3 ? (g == 0 ? 0 : 3) + p : -1;
    return p < 2 ? (g == 1 ? 24 : 33) + 7 + p : -1;
}

template <int KC, int NT, int LD, int T>
__device__ __forceinline__ void layer32(const unsigned short* wt /*[NT*16][LD], LD >= KC*32*/,
                                        const bf8v (&x)[T][KC], v4f (&acc)[T][NT])
{
    const int lane = lane_id(), r = lane & 15, k8 = (lane >> 4) * 8;
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[t][nt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < KC; ++c) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const bf8v w = *reinterpret_cast<const bf8v*>(wt + (nt * 16 + r) * LD + c * 32 + k8);
#pragma unroll
            for (int t = 0; t < T; ++t)
                acc[t][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, x[t][c], acc[t][nt], 0, 0, 0);
        }
        // keep the weight reads of one k-chunk in flight at a time (the
        // scheduler would otherwise hoist a whole layer's and spill)
        __builtin_amdgcn_sched_barrier(0);
    }
}

// bias + ReLU of the eight output tiles, as the next layer's four B fragments
__device__ __forceinline__ void relu_frags(const v4f (&acc)[8], const float* bias, bf8v (&x)[4])
{
    const int kq = (lane_id() >> 4) * 4;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const float* b0 = bias + 32 * c + kq;
        const float* b1 = b0 + 16;
        const v4f& a0 = acc[2 * c];
        const v4f& a1 = acc[2 * c + 1];
        const f8v v = {fmaxf(a0[0] + b0[0], 0.f), fmaxf(a0[1] + b0[1], 0.f), fmaxf(a0[2] + b0[2], 0.f),
                       fmaxf(a0[3] + b0[3], 0.f), fmaxf(a1[0] + b1[0], 0.f), fmaxf(a1[1] + b1[1], 0.f),
                       fmaxf(a1[2] + b1[2], 0.f), fmaxf(a1[3] + b1[3], 0.f)};
        x[c] = __builtin_convertvector(v, bf8v);
    }
}

// Per-triangle feature rows: the three positions divided by 2, then the three
// vertex normals, as the scorer's features take them (rounded from double
// exactly as the training gather does), so that a tuple's features come from
// two rows instead of six vertex lookups.
__global__ void k_tri_feat(PrunerIO io, int32_t n_tris, float* tf)
{
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tris) return;
    float* row = tf + size_t(t) * kTriFeat;
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        const int vid = io.tri[3 * t + v];
        row[3 * v + 0] = float(io.px[vid] * 0.5);
        row[3 * v + 1] = float(io.py[vid] * 0.5);
        row[3 * v + 2] = float(io.pz[vid] * 0.5);
        row[9 + 3 * v + 0] = float(io.nx[vid]);
        row[9 + 3 * v + 1] = float(io.ny[vid]);
        row[9 + 3 * v + 2] = float(io.nz[vid]);
    }
    row[18] = 0.0f;
    row[19] = 0.0f;
}

__global__ void __launch_bounds__(kPruneWaves * 64) k_prune_score(PrunerIO io, const float* tf, const float* params,
                                                                float threshold, float* scores, int32_t* keep_idx,
                                                                int64_t cap, unsigned long long* keep_count)
{
    extern __shared__ __attribute__((aligned(16))) unsigned short sm[];
    unsigned short* W1t = sm;              // [128][kS1]
    unsigned short* W2t = W1t + kW1;       // [128][kS2]
    unsigned short* W3t = W2t + kW2;
    unsigned short* W4t = W3t + kW2;       // [16][kS2], row 0 real
    float* bias = reinterpret_cast<float*>(W4t + kW4);   // b1, b2, b3 [128 each], b4
    const PrunerLayout L;
    for (int i = threadIdx.x; i < kW1; i += blockDim.x) {
        const int o = i / kS1, f = scorer_feature(i % kS1);
        W1t[i] = f >= 0 ? f2bf(params[L.w1 + f * kHid + o]) : (unsigned short)0;
    }
    for (int i = threadIdx.x; i < kW2; i += blockDim.x) {
        const int o = i / kS2, k = i % kS2;
        const int h = k < kHid ? kperm(k) : 0;
        W2t[i] = k < kHid ? f2bf(params[L.w2 + h * kHid + o]) : (unsigned short)0;
        W3t[i] = k < kHid ? f2bf(params[L.w3 + h * kHid + o]) : (unsigned short)0;
    }
    for (int i = threadIdx.x; i < kW4; i += blockDim.x) {
        const int o = i / kS2, k = i % kS2;
        W4t[i] = (o == 0 && k < kHid) ? f2bf(params[L.w4 + kperm(k)]) : (unsigned short)0;
    }
    for (int i = threadIdx.x; i < kHid; i += blockDim.x) {
        bias[i] = params[L.b1 + i];
        bias[kHid + i] = params[L.b2 + i];
        bias[2 * kHid + i] = params[L.b3 + i];
    }
    if (threadIdx.x == 0) bias[3 * kHid] = params[L.b4];
    __syncthreads();
    const int w = threadIdx.x / kWave, lane = lane_id();
    const int r = lane & 15, g = lane >> 4;
    constexpr int T = kPruneTiles;
    const int64_t ngroup = (io.n + 16 * T - 1) / (16 * T);
    const int64_t stride = int64_t(gridDim.x) * kPruneWaves;
    // the lane's twelve first-layer inputs of tuple q, in scorer_feature's
    // slots: eight floats of a triangle's feature row (two 16-byte loads),
    // then the endpoint or the row's last two floats
    auto load_feats = [&](int64_t q, float (&f)[12]) {
#pragma unroll
        for (int k = 0; k < 12; ++k) f[k] = 0.0f;
        if (q >= io.n) return;
        const int tri = io.q_tris[2 * q + (g >> 1)];
        const float* row = tf + size_t(tri) * kTriFeat + (g & 1) * 8;
        const float4 a = *reinterpret_cast<const float4*>(row);
        const float4 b = *reinterpret_cast<const float4*>(row + 4);
        f[0] = a.x; f[1] = a.y; f[2] = a.z; f[3] = a.w;
        f[4] = b.x; f[5] = b.y; f[6] = b.z; f[7] = b.w;
        if (g & 1) {
            const float2 c = *reinterpret_cast<const float2*>(row + 8);
            f[8] = c.x;
            f[9] = c.y;
        } else {
            const int j = g == 0 ? io.q_x0[q] : io.q_x3[q];
            const double* px = g == 0 ? io.x0x : io.x3x;
            const double* py = g == 0 ? io.x0y : io.x3y;
            const double* pz = g == 0 ? io.x0z : io.x3z;
            f[8] = float(px[j] * 0.5);
            f[9] = float(py[j] * 0.5);
            f[10] = float(pz[j] * 0.5);
        }
    };
    for (int64_t grp = int64_t(blockIdx.x) * kPruneWaves + w; grp < ngroup; grp += stride) {
        const int64_t q0 = grp * 16 * T + r;
        // first layer: inputs 0..31 in one 32-wide step, 32..47 in a 16-wide one
        bf8v x1a[T][1];
        v4s x1b[T];
#pragma unroll
        for (int t = 0; t < T; ++t) {
            float f[12];
            load_feats(q0 + 16 * t, f);
            x1a[t][0] = __builtin_convertvector(((f8v){f[0], f[1], f[2], f[3], f[4], f[5], f[6], f[7]}), bf8v);
            x1b[t] = frag4(f[8], f[9], f[10], f[11]);
        }
        v4f acc[T][8];
        layer32<1, 8, kS1, T>(W1t, x1a, acc);
#pragma unroll
        for (int nt = 0; nt < 8; ++nt) {
            const v4s wv = *reinterpret_cast<const v4s*>(W1t + (nt * 16 + r) * kS1 + 32 + 4 * g);
#pragma unroll
            for (int t = 0; t < T; ++t)
                acc[t][nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wv, x1b[t], acc[t][nt], 0, 0, 0);
        }
        bf8v x[T][4];
#pragma unroll
        for (int t = 0; t < T; ++t) relu_frags(acc[t], bias, x[t]);
        layer32<4, 8, kS2, T>(W2t, x, acc);
#pragma unroll
        for (int t = 0; t < T; ++t) relu_frags(acc[t], bias + kHid, x[t]);
        layer32<4, 8, kS2, T>(W3t, x, acc);
#pragma unroll
        for (int t = 0; t < T; ++t) relu_frags(acc[t], bias + 2 * kHid, x[t]);
        v4f out[T][1];
        layer32<4, 1, kS2, T>(W4t, x, out);
#pragma unroll
        for (int t = 0; t < T; ++t) {
            // lanes 0..15: row 0 of the output tile, the logit of tuple q
            const int64_t q = q0 + 16 * t;
            const float zr = out[t][0][0] + bias[3 * kHid];
            const bool mine = lane < 16 && q < io.n;
            const float p = 1.0f / (1.0f + expf(-zr));
            if (mine && scores) scores[q] = p;
            const bool keep = mine && p >= threshold;
            const unsigned long long bal = __ballot(keep);
            const int tot = __popcll(bal);
            if (tot > 0) {
                unsigned long long base = 0;
                if (lane == 0) base = atomicAdd(keep_count, (unsigned long long)tot);
                base = __shfl(base, 0, kWave);
                if (keep) {
                    const unsigned long long o = base + __popcll(bal & ((1ull << lane) - 1ull));
                    if (o < (unsigned long long)cap) keep_idx[o] = int32_t(q);
                }
            }
        }
    }
}

// ------------------------------------------------------------------ launchers
static inline unsigned nblk(int64_t n, int b) { return unsigned((n + b - 1) / b); }

hipError_t launch_gather(const PrunerIO& io, unsigned short* X, float* Xf, hipStream_t s)
{
    if (io.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3(nblk(io.n, 256)), dim3(256), 0, s, io, X, Xf);
    return hipGetLastError();
}

hipError_t launch_prune_score(const PrunerIO& io, const float* params, float threshold, float* scores,
                              int32_t* keep_idx, int64_t cap, unsigned long long* keep_count, float* tri_feat,
                              int32_t n_tris, hipStream_t s)
{
    if (io.n <= 0) return hipSuccess;
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void*)k_prune_score, hipFuncAttributeMaxDynamicSharedMemorySize, kPruneLds);
        attr = true;
    }
    k_tri_feat<<<nblk(n_tris, 256), 256, 0, s>>>(io, n_tris, tri_feat);
    // persistent: one block per compute unit (its LDS allows no second), each
    // loading the weights once and striding over pairs of 16-tuple tiles
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    const int64_t groups = (io.n + 16 * kPruneTiles - 1) / (16 * kPruneTiles);
    int64_t blocks = (groups + kPruneWaves - 1) / kPruneWaves;
    if (blocks > cus) blocks = cus;
    hipLaunchKernelGGL(k_prune_score, dim3(unsigned(blocks)), dim3(kPruneWaves * 64), kPruneLds, s, io, tri_feat,
                       params, threshold, scores, keep_idx, cap, keep_count);
    return hipGetLastError();
}

// One forward + backward pass of a batch: loss (accumulated into *loss) and
// gradients (written, fp32, same layout as the parameters).
hipError_t pruner_fwd_bwd(const PrunerIO& io, const float* labels, float pos_w, const float* params, float* grads,
                          float* loss, PrunerWork& W, hipStream_t s)
{
    const int64_t n = io.n;
    const PrunerLayout L;
    hipError_t e;
    if ((e = launch_gather(io, W.X, nullptr, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_to_bf16, dim3(nblk(kNParams, 256)), dim3(256), 0, s, params, W.Pb, int64_t(kNParams));
    // forward: Z1 = X W1 (W1 stored [in][out]: B(k,n) = W[k*128 + n])
    hipError_t first_err = hipSuccess;
    auto gemm = [&](const unsigned short* A, int64_t sam, int64_t sak, const unsigned short* B, int64_t sbk,
                    int64_t sbn, float* C, int ldc, int M, int N, int K, int split) {
        // weight gradients (M, N <= 128, K = batch): deterministic split-K
        // through the partials buffer so that the launch fills the chip
        const bool wgrad = split > 1;
        GemmArgs G{A, sam, sak, B, sbk, sbn, C, ldc, M, N, K, 1.0f, 0, wgrad ? W.part : nullptr};
        const hipError_t r = launch_gemm(G, split, s);
        if (r != hipSuccess && first_err == hipSuccess) first_err = r;
    };
    const int nn = int(n);
    gemm(W.X, kFeat, 1, W.Pb + L.w1, kHid, 1, W.Z1, kHid, nn, kHid, kIn, 1);
    hipLaunchKernelGGL(k_bias_relu, dim3(nblk(n * kHid, 256)), dim3(256), 0, s, W.Z1, params + L.b1, W.H1, n, kHid, 1);
    gemm(W.H1, kHid, 1, W.Pb + L.w2, kHid, 1, W.Z2, kHid, nn, kHid, kHid, 1);
    hipLaunchKernelGGL(k_bias_relu, dim3(nblk(n * kHid, 256)), dim3(256), 0, s, W.Z2, params + L.b2, W.H2, n, kHid, 1);
    gemm(W.H2, kHid, 1, W.Pb + L.w3, kHid, 1, W.Z3, kHid, nn, kHid, kHid, 1);
    hipLaunchKernelGGL(k_bias_relu, dim3(nblk(n * kHid, 256)), dim3(256), 0, s, W.Z3, params + L.b3, W.H3, n, kHid, 1);
    // z4 = H3 W4 + b4 (N = 1); the bias is added inside the loss kernel
    gemm(W.H3, kHid, 1, W.Pb + L.w4, 1, 0, W.Z4, 16, nn, 1, kHid, 1);
    hipLaunchKernelGGL(k_loss, dim3(nblk(n, 256)), dim3(256), 0, s, W.Z4, 16, params + L.b4, labels, n, pos_w,
                       1.0f / float(n), W.dZ4, (float*)nullptr, loss);
    // backward
    hipLaunchKernelGGL(k_fill, dim3(nblk(kNParams, 256)), dim3(256), 0, s, grads, int64_t(kNParams), 0.0f);
    // no atomics: the gradients, hence training, are deterministic
    const int split = int(std::max<int64_t>(1, std::min<int64_t>(kGemmSplitMax, n / 512)));
    // dW4 = H3^T dZ4 : A(m=in, k=row) = H3[row*128 + m], B(k=row, n=0) = dZ4[row*16]
    gemm(W.H3, 1, kHid, W.dZ4, 16, 1, grads + L.w4, 1, kHid, 1, nn, split);
    hipLaunchKernelGGL(k_colsum, dim3(1), dim3(256), 0, s, W.dZ4, n, 1, 16, grads + L.b4);
    // dH3 = dZ4 W4^T : A(row, k) = dZ4[row*16 + k] (k < 1), B(k, n) = W4[n*1 + k]
    gemm(W.dZ4, 16, 1, W.Pb + L.w4, 1, 1, W.dH, kHid, nn, kHid, 1, 1);
    hipLaunchKernelGGL(k_relu_bwd, dim3(nblk(n * kHid, 256)), dim3(256), 0, s, W.dH, W.Z3, W.dZ, n * kHid);
    gemm(W.H2, 1, kHid, W.dZ, kHid, 1, grads + L.w3, kHid, kHid, kHid, nn, split);
    hipLaunchKernelGGL(k_colsum, dim3(kHid), dim3(256), 0, s, W.dZ, n, kHid, kHid, grads + L.b3);
    gemm(W.dZ, kHid, 1, W.Pb + L.w3, 1, kHid, W.dH, kHid, nn, kHid, kHid, 1);
    hipLaunchKernelGGL(k_relu_bwd, dim3(nblk(n * kHid, 256)), dim3(256), 0, s, W.dH, W.Z2, W.dZ, n * kHid);
    gemm(W.H1, 1, kHid, W.dZ, kHid, 1, grads + L.w2, kHid, kHid, kHid, nn, split);
    hipLaunchKernelGGL(k_colsum, dim3(kHid), dim3(256), 0, s, W.dZ, n, kHid, kHid, grads + L.b2);
    gemm(W.dZ, kHid, 1, W.Pb + L.w2, 1, kHid, W.dH, kHid, nn, kHid, kHid, 1);
    hipLaunchKernelGGL(k_relu_bwd, dim3(nblk(n * kHid, 256)), dim3(256), 0, s, W.dH, W.Z1, W.dZ, n * kHid);
    gemm(W.X, 1, kFeat, W.dZ, kHid, 1, grads + L.w1, kHid, kIn, kHid, nn, split);
    hipLaunchKernelGGL(k_colsum, dim3(kHid), dim3(256), 0, s, W.dZ, n, kHid, kHid, grads + L.b1);
    return first_err != hipSuccess ? first_err : hipGetLastError();
}

hipError_t pruner_adam(float* p, const float* g, float* m, float* v, int64_t step, float lr, float b1, float b2,
                       float eps, hipStream_t s)
{
    const float c1 = 1.0f - powf(b1, float(step)), c2 = 1.0f - powf(b2, float(step));
    hipLaunchKernelGGL(k_adam, dim3(nblk(kNParams, 256)), dim3(256), 0, s, p, g, m, v, int64_t(kNParams), lr, b1, b2,
                       eps, c1, c2);
    return hipGetLastError();
}

}  // namespace spoly
