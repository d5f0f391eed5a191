// Screening network of the learned form: 4 inputs -> 64 (ReLU) -> 64 (ReLU) -> 1 logit.
//
// Parameter vector (FP32), one layout everywhere:  W1[64][4], b1[64], W2[64][64], b2[64], w3[64], b3.
// Every thread evaluates one sample; the weights are wave-uniform, so they come through the scalar
// cache and feed the FMAs as scalar operands.  Training computes per-sample deltas in registers and
// forms the weight gradients (sums over the workgroup's samples) from LDS tiles; workgroup partials are
// summed in a fixed order by the Adam kernel, so a training run is deterministic.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace blk {

namespace {

constexpr int MH = MLP_HIDDEN;
constexpr int OW1 = 0, OB1 = 4 * MH, OW2 = OB1 + MH, OB2 = OW2 + MH * MH, OW3 = OB2 + MH, OB3 = OW3 + MH;
static_assert(OB3 + 1 == MLP_NPARAMS, "parameter layout");

// logit of one sample; h1 receives the first hidden layer (post-ReLU)
__device__ __forceinline__ float mlp_logit(const float* __restrict__ P, const float f[4], float h1[MH]) {
#pragma unroll
    for (int u = 0; u < MH; ++u) {
        float a = P[OB1 + u];
#pragma unroll
        for (int q = 0; q < 4; ++q) a = fmaf(P[OW1 + 4 * u + q], f[q], a);
        h1[u] = fmaxf(a, 0.f);
    }
    float o = P[OB3];
#pragma unroll 2
    for (int u = 0; u < MH; ++u) {
        float a = P[OB2 + u];
#pragma unroll
        for (int q = 0; q < MH; ++q) a = fmaf(P[OW2 + MH * u + q], h1[q], a);
        o = fmaf(P[OW3 + u], fmaxf(a, 0.f), o);
    }
    return o;
}

__device__ __forceinline__ float sigmoidf(float o) { return 1.f / (1.f + expf(-o)); }

__global__ __launch_bounds__(256) void k_mlp_fwd(const float* __restrict__ feat, int64_t m, const float* __restrict__ P,
                                                 float* __restrict__ prob) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const float f[4] = {feat[4 * i], feat[4 * i + 1], feat[4 * i + 2], feat[4 * i + 3]};
        float h1[MH];
        prob[i] = sigmoidf(mlp_logit(P, f, h1));
    }
}

// ---- training -------------------------------------------------------------------------------------------
constexpr int GS = 128;       // samples (threads) per workgroup
constexpr int LDH = MH + 4;   // padded LDS row of per-sample vectors

struct Batch {
    int64_t base, cnt, a, c;
};

__device__ __forceinline__ Batch batch_of(int64_t step, int64_t m, int64_t batch, int64_t nb, const int64_t* perm) {
    Batch b;
    const int64_t e = step / nb, bi = step - e * nb;
    b.base = bi * batch;
    b.cnt = m - b.base < batch ? m - b.base : batch;
    b.a = perm ? perm[2 * e] : 1;
    b.c = perm ? perm[2 * e + 1] : 0;
    return b;
}

// per-workgroup partial gradient of the mean binary cross-entropy over the step's minibatch
__global__ __launch_bounds__(GS) void k_mlp_grad(const float* __restrict__ feat, const float* __restrict__ label,
                                                 int64_t m, int64_t batch, int64_t nb, const int64_t* __restrict__ perm,
                                                 const int64_t* __restrict__ step_ptr, const float* __restrict__ P,
                                                 float* __restrict__ partial, double* __restrict__ loss_part) {
    __shared__ float H1s[GS * LDH];
    __shared__ float D2s[GS * LDH];
    __shared__ float D1s[GS * LDH];
    __shared__ float Fs[GS * 4];
    __shared__ float Ds[GS];
    __shared__ float Ls[GS];
    const int tid = threadIdx.x;
    const int64_t step = step_ptr ? *step_ptr : 0;
    const Batch bt = batch_of(step, m, batch, nb, perm);
    const int64_t sl = (int64_t)blockIdx.x * GS + tid;
    const bool valid = sl < bt.cnt;
    const int64_t i = valid ? (bt.a * (bt.base + sl) + bt.c) % m : 0;
    float f[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) f[q] = valid ? feat[4 * i + q] : 0.f;
    const float y = valid ? label[i] : 0.f;

    // forward; the second hidden layer goes to this sample's D2s row for now
    float h1[MH];
#pragma unroll
    for (int u = 0; u < MH; ++u) {
        float a = P[OB1 + u];
#pragma unroll
        for (int q = 0; q < 4; ++q) a = fmaf(P[OW1 + 4 * u + q], f[q], a);
        h1[u] = fmaxf(a, 0.f);
        H1s[tid * LDH + u] = h1[u];
    }
    float o = P[OB3];
#pragma unroll 2
    for (int u = 0; u < MH; ++u) {
        float a = P[OB2 + u];
#pragma unroll
        for (int q = 0; q < MH; ++q) a = fmaf(P[OW2 + MH * u + q], h1[q], a);
        const float h2 = fmaxf(a, 0.f);
        D2s[tid * LDH + u] = h2;
        o = fmaf(P[OW3 + u], h2, o);
    }
    const float inv = 1.f / (float)(bt.cnt > 0 ? bt.cnt : 1);
    const float dout = valid ? (sigmoidf(o) - y) * inv : 0.f;
    // softplus(o) - y o, computed without overflow
    const float sp = o > 0.f ? o + log1pf(expf(-o)) : log1pf(expf(o));
    Ds[tid] = dout;
    Ls[tid] = valid ? sp - y * o : 0.f;
#pragma unroll
    for (int q = 0; q < 4; ++q) Fs[tid * 4 + q] = f[q];
    __syncthreads();

    // output layer: g_w3[u] = sum_s dout_s h2[s][u], g_b3 = sum_s dout_s; and the loss
    float gw3 = 0.f, gb3 = 0.f;
    double lsum = 0.0;
    if (tid < MH) {
        for (int s = 0; s < GS; ++s) gw3 = fmaf(Ds[s], D2s[s * LDH + tid], gw3);
    } else if (tid == MH) {
        for (int s = 0; s < GS; ++s) gb3 += Ds[s];
    } else if (tid == MH + 1) {
        for (int s = 0; s < GS; ++s) lsum += (double)Ls[s];
    }
    __syncthreads();

    // deltas of the second hidden layer (own row), then of the first
#pragma unroll
    for (int u = 0; u < MH; ++u) {
        const float h2 = D2s[tid * LDH + u];
        D2s[tid * LDH + u] = h2 > 0.f ? dout * P[OW3 + u] : 0.f;
    }
    float acc[MH];
#pragma unroll
    for (int q = 0; q < MH; ++q) acc[q] = 0.f;
#pragma unroll 2
    for (int u = 0; u < MH; ++u) {
        const float d2 = D2s[tid * LDH + u];
#pragma unroll
        for (int q = 0; q < MH; ++q) acc[q] = fmaf(P[OW2 + MH * u + q], d2, acc[q]);
    }
#pragma unroll
    for (int q = 0; q < MH; ++q) D1s[tid * LDH + q] = h1[q] > 0.f ? acc[q] : 0.f;
    __syncthreads();

    // weight gradients over the workgroup's samples
    float* out = partial + (int64_t)blockIdx.x * MLP_NPARAMS;
    {
        const int u = tid >> 1, q0 = (tid & 1) * 32;
        float g[32];
#pragma unroll
        for (int t = 0; t < 32; ++t) g[t] = 0.f;
        float gb = 0.f, gw1a = 0.f, gw1b = 0.f;
        const int qf = (tid & 1) * 2;
        for (int s = 0; s < GS; ++s) {
            const float d2 = D2s[s * LDH + u];
            const float d1 = D1s[s * LDH + u];
#pragma unroll
            for (int t = 0; t < 32; ++t) g[t] = fmaf(d2, H1s[s * LDH + q0 + t], g[t]);
            gb += (tid & 1) ? d1 : d2;
            gw1a = fmaf(d1, Fs[s * 4 + qf], gw1a);
            gw1b = fmaf(d1, Fs[s * 4 + qf + 1], gw1b);
        }
#pragma unroll
        for (int t = 0; t < 32; ++t) out[OW2 + MH * u + q0 + t] = g[t];
        if (tid & 1) out[OB1 + u] = gb;
        else out[OB2 + u] = gb;
        out[OW1 + 4 * u + qf] = gw1a;
        out[OW1 + 4 * u + qf + 1] = gw1b;
    }
    if (tid < MH) out[OW3 + tid] = gw3;
    if (tid == MH) out[OB3] = gb3;
    if (tid == MH + 1) loss_part[blockIdx.x] = lsum;
}

// sum of the workgroup partials (fixed order), then one Adam step per parameter (apply != 0)
__global__ __launch_bounds__(256) void k_mlp_adam(const float* __restrict__ partial, int nblk,
                                                  const double* __restrict__ loss_part, float* __restrict__ P,
                                                  float* __restrict__ mom, float* __restrict__ vel,
                                                  const int64_t* __restrict__ step_ptr, int64_t m, int64_t batch,
                                                  int64_t nb, double lr, double b1, double b2, double eps, int apply,
                                                  float* __restrict__ grad_out, double* __restrict__ loss_out) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t step = step_ptr ? *step_ptr : 0;
    if (idx < MLP_NPARAMS) {
        double g = 0.0;
        for (int b = 0; b < nblk; ++b) g += (double)partial[(int64_t)b * MLP_NPARAMS + idx];
        if (grad_out) grad_out[idx] = (float)g;
        if (apply) {
            const double t = (double)(step + 1);
            const double mo = b1 * (double)mom[idx] + (1.0 - b1) * g;
            const double ve = b2 * (double)vel[idx] + (1.0 - b2) * g * g;
            const double mh = mo / (1.0 - pow(b1, t));
            const double vh = ve / (1.0 - pow(b2, t));
            mom[idx] = (float)mo;
            vel[idx] = (float)ve;
            P[idx] = (float)((double)P[idx] - lr * mh / (sqrt(vh) + eps));
        }
    }
    if (idx == 0 && loss_out) {
        const Batch bt = batch_of(step, m, batch, nb, nullptr);
        double L = 0.0;
        for (int b = 0; b < nblk; ++b) L += loss_part[b];
        loss_out[step_ptr ? step : 0] = L / (double)(bt.cnt > 0 ? bt.cnt : 1);
    }
}

__global__ void k_step_inc(int64_t* step) { *step += 1; }

// histogram of network scores, positives in [bins, 2 bins)
__global__ void k_mlp_hist(const float* __restrict__ prob, const float* __restrict__ label, int64_t m, int bins,
                           uint32_t* __restrict__ hist) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        int b = (int)(prob[i] * (float)bins);
        b = b < 0 ? 0 : (b >= bins ? bins - 1 : b);
        atomicAdd(&hist[(label[i] > 0.5f ? bins : 0) + b], 1u);
    }
}

// ---- in the path -------------------------------------------------------------------------------------------
// strong-rule candidates outside the previous active set: record them (cand) and, when the rule is applied,
// keep only those the network scores above the threshold
__global__ __launch_bounds__(256) void k_learned(uint8_t* __restrict__ strong, const double* __restrict__ beta,
                                                 const float* __restrict__ zh, int64_t p, int s1, int s2, int s3,
                                                 float ratio, const float* __restrict__ P, float tau_logit, int apply,
                                                 uint8_t* __restrict__ cand) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < p; j += (int64_t)gridDim.x * blockDim.x) {
        const bool c = strong[j] && beta[j] == 0.0;
        if (cand) cand[j] = c ? 1 : 0;
        if (c && apply) {
            const float f[4] = {zh[(int64_t)s1 * p + j], zh[(int64_t)s2 * p + j], zh[(int64_t)s3 * p + j], ratio};
            float h1[MH];
            if (!(mlp_logit(P, f, h1) >= tau_logit)) strong[j] = 0;
        }
    }
}

// slot <- |z_j| / lambda for the scanned columns (the slot was cleared before)
__global__ void k_zhist(const int32_t* __restrict__ cols, const int64_t* __restrict__ len_dev, int64_t len_host,
                        const double* __restrict__ z, double lam, float* __restrict__ slot) {
    const int64_t len = len_dev ? *len_dev : len_host;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < len; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = cols ? (int64_t)cols[t] : t;
        slot[j] = (float)(fabs(z[j]) / lam);
    }
}

__global__ void k_zhist_keep(const uint8_t* __restrict__ keep, int64_t p, const double* __restrict__ z, double lam,
                             float* __restrict__ slot) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < p; j += (int64_t)gridDim.x * blockDim.x)
        slot[j] = keep[j] ? (float)(fabs(z[j]) / lam) : 0.f;
}

// training records: features of the listed candidates and whether they are active now
__global__ void k_rec_feat(const int32_t* __restrict__ list, const int64_t* __restrict__ len_dev,
                           const float* __restrict__ zh, int64_t p, int s1, int s2, int s3, float ratio,
                           const double* __restrict__ beta, int64_t cap, const int64_t* __restrict__ count,
                           float* __restrict__ feat, float* __restrict__ label) {
    const int64_t len = *len_dev, off = *count;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < len && off + t < cap;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = list[t], o = off + t;
        feat[4 * o] = zh[(int64_t)s1 * p + j];
        feat[4 * o + 1] = zh[(int64_t)s2 * p + j];
        feat[4 * o + 2] = zh[(int64_t)s3 * p + j];
        feat[4 * o + 3] = ratio;
        label[o] = beta[j] != 0.0 ? 1.f : 0.f;
    }
}

__global__ void k_rec_commit(const int64_t* __restrict__ len_dev, int64_t cap, int64_t* __restrict__ count) {
    const int64_t n = *count + *len_dev;
    *count = n < cap ? n : cap;
}

int grid_of(int64_t work, int per, int maxb) {
    int64_t g = (work + per - 1) / per;
    return (int)(g < 1 ? 1 : (g > maxb ? maxb : g));
}

}  // namespace

hipError_t launch_mlp_fwd(const float* feat, int64_t m, const float* P, float* prob, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    k_mlp_fwd<<<grid_of(m, 256, 8192), 256, 0, st>>>(feat, m, P, prob);
    return hipGetLastError();
}

int mlp_grad_blocks(int64_t batch) { return (int)((batch + GS - 1) / GS); }

hipError_t launch_mlp_grad(const float* feat, const float* label, int64_t m, int64_t batch, int64_t nb,
                           const int64_t* perm, const int64_t* step, const float* P, float* partial,
                           double* loss_part, hipStream_t st) {
    k_mlp_grad<<<mlp_grad_blocks(batch), GS, 0, st>>>(feat, label, m, batch, nb, perm, step, P, partial, loss_part);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(const float* partial, int nblk, const double* loss_part, float* P, float* mom, float* vel,
                           const int64_t* step, int64_t m, int64_t batch, int64_t nb, double lr, double b1,
                           double b2, double eps, int apply, float* grad_out, double* loss_out, hipStream_t st) {
    k_mlp_adam<<<(MLP_NPARAMS + 255) / 256, 256, 0, st>>>(partial, nblk, loss_part, P, mom, vel, step, m, batch, nb,
                                                          lr, b1, b2, eps, apply, grad_out, loss_out);
    return hipGetLastError();
}

hipError_t launch_step_inc(int64_t* step, hipStream_t st) {
    k_step_inc<<<1, 1, 0, st>>>(step);
    return hipGetLastError();
}

hipError_t launch_mlp_hist(const float* prob, const float* label, int64_t m, int bins, uint32_t* hist,
                           hipStream_t st) {
    if (m <= 0) return hipSuccess;
    k_mlp_hist<<<grid_of(m, 256, 4096), 256, 0, st>>>(prob, label, m, bins, hist);
    return hipGetLastError();
}

hipError_t launch_learned(uint8_t* strong, const double* beta, const float* zh, int64_t p, int s1, int s2, int s3,
                          float ratio, const float* P, float tau_logit, int apply, uint8_t* cand, hipStream_t st) {
    k_learned<<<grid_of(p, 256, 8192), 256, 0, st>>>(strong, beta, zh, p, s1, s2, s3, ratio, P, tau_logit, apply,
                                                     cand);
    return hipGetLastError();
}

hipError_t launch_zhist(const int32_t* cols, const int64_t* len_dev, int64_t len_host, const double* z, double lam,
                        float* slot, int64_t p, hipStream_t st) {
    k_zhist<<<grid_of(p, 256, 4096), 256, 0, st>>>(cols, len_dev, len_host, z, lam, slot);
    return hipGetLastError();
}

hipError_t launch_zhist_keep(const uint8_t* keep, int64_t p, const double* z, double lam, float* slot,
                             hipStream_t st) {
    k_zhist_keep<<<grid_of(p, 256, 4096), 256, 0, st>>>(keep, p, z, lam, slot);
    return hipGetLastError();
}

hipError_t launch_rec_feat(const int32_t* list, const int64_t* len_dev, const float* zh, int64_t p, int s1, int s2,
                           int s3, float ratio, const double* beta, int64_t cap, int64_t* count, float* feat,
                           float* label, hipStream_t st) {
    k_rec_feat<<<grid_of(p, 256, 4096), 256, 0, st>>>(list, len_dev, zh, p, s1, s2, s3, ratio, beta, cap, count, feat,
                                                      label);
    k_rec_commit<<<1, 1, 0, st>>>(len_dev, cap, count);
    return hipGetLastError();
}

}  // namespace blk
