// Learned pruner: parameter layout, work buffers and launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spoly {

constexpr int kIn = 42;      // features per tuple
constexpr int kFeat = 48;    // padded feature row
constexpr int kHid = 128;
constexpr int kNParams = kIn * kHid + kHid + 2 * (kHid * kHid + kHid) + kHid + 1;  // 38657

// fp32 parameter vector: W1 [42 x 128] (row = input), b1, W2 [128 x 128], b2, W3, b3, W4 [128], b4
struct PrunerLayout {
    int w1 = 0;
    int b1 = kIn * kHid;
    int w2 = b1 + kHid;
    int b2 = w2 + kHid * kHid;
    int w3 = b2 + kHid;
    int b3 = w3 + kHid * kHid;
    int w4 = b3 + kHid;
    int b4 = w4 + kHid;
};

struct PrunerIO {   // tuples (x0, T1, T2, x3) and the scene they index
    const double *px, *py, *pz, *nx, *ny, *nz;
    const int32_t* tri;
    const double *x0x, *x0y, *x0z, *x3x, *x3y, *x3z;
    const int32_t *q_x0, *q_x3, *q_tris;
    int64_t n;
};

struct GemmArgs {
    const unsigned short* A;
    int64_t sam, sak;
    const unsigned short* B;
    int64_t sbk, sbn;
    float* C;
    int ldc;
    int M, N, K;
    float alpha;
    int accumulate;
    // split-K without atomics: with part set, split k writes its [M x N]
    // partial tile to part + k*M*N and a second kernel adds them in k order
    float* part;
};
constexpr int kGemmSplitMax = 128;

struct PrunerWork {   // per-batch activations (device), sized for `cap` tuples
    int64_t cap;
    unsigned short *X, *Pb, *H1, *H2, *H3, *dZ4, *dZ;
    float *Z1, *Z2, *Z3, *Z4, *dH;
    float* part;   // kGemmSplitMax x kHid x kHid split-K partials
};

hipError_t launch_gemm(const GemmArgs& G, int split_k, hipStream_t stream);
hipError_t launch_gather(const PrunerIO& io, unsigned short* X, float* Xf, hipStream_t s);
// Scores (and keeps) n tuples; tri_feat: device workspace of kTriFeat floats
// per triangle of the mesh (n_tris), filled by the call.
constexpr int kTriFeat = 20;
hipError_t launch_prune_score(const PrunerIO& io, const float* params, float threshold, float* scores,
                              int32_t* keep_idx, int64_t cap, unsigned long long* keep_count, float* tri_feat,
                              int32_t n_tris, hipStream_t s);
hipError_t pruner_fwd_bwd(const PrunerIO& io, const float* labels, float pos_w, const float* params, float* grads,
                          float* loss, PrunerWork& W, hipStream_t s);
hipError_t pruner_adam(float* p, const float* g, float* m, float* v, int64_t step, float lr, float b1, float b2,
                       float eps, hipStream_t s);

}  // namespace spoly
