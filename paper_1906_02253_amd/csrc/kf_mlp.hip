// Training and batch inference of the learned path-length guess on gfx950:
// bf16 matrix-core forward and backward passes with FP32 accumulation, FP32
// master weights updated by Adam (Kingma & Ba 2015), and the input features.
//
// One training step over a batch of B rows:
//   mlp_grad_kernel    each wave takes 16 rows: forward (mlp_tile), output
//                      error, backward through both tanh layers, and the
//                      wave's partial gradient of all 4801 parameters (the
//                      weight gradients are contractions over the rows, done
//                      on the matrix cores after an LDS transpose);
//   mlp_reduce_kernel  sums the partials, applies Adam to the master weights
//                      and republishes the bf16 copies the forward pass reads.
#include "kf_mlp_api.hpp"

namespace kfmi {

// ------------------------------------------------------------------ features
template <typename T>
__global__ __launch_bounds__(256) void mlp_features_kernel(int64_t n, int64_t ld, const T* __restrict__ par,
                                                           const int32_t* __restrict__ target,
                                                           const kf_layer* __restrict__ layers,
                                                           int n_layers, kf_params prm,
                                                           float* __restrict__ feats)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int l = target[i];
    float f[kMlpIn] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (l >= 0 && l < n_layers) {
        T p[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) p[k] = par[k * ld + i];
        mlp_features(p, layers[l], prm, f);
    }
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k) feats[k * ld + i] = f[k];
}

// ------------------------------------------------------------------ targets
__global__ __launch_bounds__(256) void mlp_targets_kernel(int64_t n, int64_t ld,
                                                          const float* __restrict__ feats,
                                                          const float* __restrict__ path,
                                                          float* __restrict__ target)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float f[kMlpIn];
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k) f[k] = feats[k * ld + i];
    target[i] = mlp_target(f, path[i]);
}

// ------------------------------------------------------------------ inference
// Every lane of every wave takes part (rows beyond n use zero inputs).
__global__ __launch_bounds__(256) void mlp_forward_kernel(int64_t n, int64_t ld, const float* __restrict__ feats,
                                                          MlpDev m, float* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float f[kMlpIn];
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k) f[k] = i < n ? feats[k * ld + i] : 0.0f;
    const float y = mlp_wave(m, f);
    if (i < n) out[i] = y;
}

// ------------------------------------------------------------------ training
constexpr int kGradWaves = 4;        // waves per workgroup, 16 rows each
struct GradLds {                     // one wave's staging area
    float x[16][kMlpIn];
    float h1[16][kMlpHidden];
    float h2[16][kMlpHidden];
    float da1[16][kMlpHidden];
    float da2[16][kMlpHidden];
    float dy[16];
};

__global__ __launch_bounds__(64 * kGradWaves) void mlp_grad_kernel(
    const float* __restrict__ feats, const float* __restrict__ target, int64_t n_rows, int64_t ld,
    const int32_t* __restrict__ rows, int batch, MlpDev m, float* __restrict__ partial,
    float* __restrict__ loss_part)
{
    __shared__ GradLds lds_all[kGradWaves];
    const int wave = threadIdx.x >> 6;
    GradLds& S = lds_all[wave];
    const int ln = threadIdx.x & 63, r = ln & 15, g = ln >> 4;
    const int wg = blockIdx.x * kGradWaves + wave;      // global wave index
    const int b = wg * 16 + r;                           // batch row of this lane's column
    const int64_t rw = b < batch ? rows[b] : -1;
    const bool valid = rw >= 0 && rw < n_rows;      // rows outside [0, n) are skipped
    const int64_t row = valid ? rw : 0;
    // inputs: lane groups 0 / 1 carry the high parts of features 0..3 / 4..7
    // of row r, groups 2 / 3 the low parts of the same features
    float xv[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (valid)
        for (int j = 0; j < 4; ++j) xv[j] = feats[(int64_t)(4 * (g & 1) + j) * ld + row];
    if (g < 2)
        for (int j = 0; j < 4; ++j) S.x[r][4 * g + j] = xv[j];
    const bf16x4 xb = split_inputs(xv, g);
    f32x4 h1[4], h2[4];
    const float y = mlp_tile(m, xb, h1, h2);
    const float t = valid ? target[row] : 0.0f;
    const float err = valid ? y - t : 0.0f;
    const float dy = 2.0f * err / float(batch);
    // output layer error through tanh of layer 2 (D layout, lane-local)
    f32x4 da2[4];
#pragma unroll
    for (int mo = 0; mo < 4; ++mo)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int u = 16 * mo + 4 * g + j;
            da2[mo][j] = m.bias[128 + u] * dy * (1.0f - h2[mo][j] * h2[mo][j]);
        }
    // back through W2: dH1^T = W2^T dA2^T, then through tanh of layer 1
    f32x4 da1[4];
#pragma unroll
    for (int mi = 0; mi < 4; ++mi) {
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ko = 0; ko < 4; ++ko)
            acc = mfma_bf16(load_bf16x4(m.w2t + (16 * mi + r) * 64 + 16 * ko + 4 * g),
                            pack_bf16x4(da2[ko][0], da2[ko][1], da2[ko][2], da2[ko][3]), acc);
#pragma unroll
        for (int j = 0; j < 4; ++j) da1[mi][j] = acc[j] * (1.0f - h1[mi][j] * h1[mi][j]);
    }
    // stage row-major copies for the contractions over the rows
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int u = 16 * q + 4 * g + j;
            S.h1[r][u] = h1[q][j];
            S.h2[r][u] = h2[q][j];
            S.da1[r][u] = da1[q][j];
            S.da2[r][u] = da2[q][j];
        }
    if (g == 0) S.dy[r] = dy;
    __syncthreads();
    float* P = partial + (size_t)wg * kMlpParams;
    // dW2[out][in] = sum_rows dA2[row][out] H1[row][in]: A = dA2^T, B = H1
    {
        bf16x4 bh[4];
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
            bh[mi] = pack_bf16x4(S.h1[4 * g + 0][16 * mi + r], S.h1[4 * g + 1][16 * mi + r],
                                 S.h1[4 * g + 2][16 * mi + r], S.h1[4 * g + 3][16 * mi + r]);
#pragma unroll
        for (int mo = 0; mo < 4; ++mo) {
            const bf16x4 a = pack_bf16x4(S.da2[4 * g + 0][16 * mo + r], S.da2[4 * g + 1][16 * mo + r],
                                         S.da2[4 * g + 2][16 * mo + r], S.da2[4 * g + 3][16 * mo + r]);
#pragma unroll
            for (int mi = 0; mi < 4; ++mi) {
                f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
                acc = mfma_bf16(a, bh[mi], acc);
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    P[kMlpOffW2 + (16 * mo + 4 * g + j) * 64 + 16 * mi + r] = acc[j];
            }
        }
    }
    // dW1[out][k] = sum_rows dA1[row][out] X[row][k]: A = dA1^T, B = X (k < 8)
    {
        const bf16x4 bx = r < kMlpIn ? pack_bf16x4(S.x[4 * g + 0][r], S.x[4 * g + 1][r],
                                                   S.x[4 * g + 2][r], S.x[4 * g + 3][r])
                                     : pack_bf16x4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
        for (int mo = 0; mo < 4; ++mo) {
            const bf16x4 a = pack_bf16x4(S.da1[4 * g + 0][16 * mo + r], S.da1[4 * g + 1][16 * mo + r],
                                         S.da1[4 * g + 2][16 * mo + r], S.da1[4 * g + 3][16 * mo + r]);
            f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            acc = mfma_bf16(a, bx, acc);
            if (r < kMlpIn)
#pragma unroll
                for (int j = 0; j < 4; ++j) P[(16 * mo + 4 * g + j) * kMlpIn + r] = acc[j];
        }
    }
    // biases and the output weights: sums over the 16 rows, lane = unit
    {
        float s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
        for (int q = 0; q < 16; ++q) {
            s1 += S.da1[q][ln];
            s2 += S.da2[q][ln];
            s3 += S.h2[q][ln] * S.dy[q];
        }
        P[kMlpOffB1 + ln] = s1;
        P[kMlpOffB2 + ln] = s2;
        P[kMlpOffW3 + ln] = s3;
        if (ln == 0) {
            float s = 0.0f;
            for (int q = 0; q < 16; ++q) s += S.dy[q];
            P[kMlpOffB3] = s;
        }
    }
    float e2 = g == 0 ? err * err : 0.0f;
    for (int o = 8; o > 0; o >>= 1) e2 += __shfl_xor(e2, o);
    if (ln == 0) loss_part[wg] = e2;
}

// bf16 copies of the master weights for the forward pass, parameter p
__device__ inline void publish_param(int p, float w, uint16_t* w1, uint16_t* w2, uint16_t* w2t,
                                     float* bias)
{
    const uint16_t bw = to_bf16(w);
    if (p < kMlpOffB1) {
        w1[(p / kMlpIn) * 16 + (p % kMlpIn)] = bw;            // times the inputs' high parts
        w1[(p / kMlpIn) * 16 + kMlpIn + (p % kMlpIn)] = bw;   // times their low parts
    } else if (p < kMlpOffW2) {
        bias[p - kMlpOffB1] = from_bf16(bw);
    } else if (p < kMlpOffB2) {
        const int q = p - kMlpOffW2, o = q / 64, i = q % 64;
        w2[o * 64 + i] = bw;
        w2t[i * 64 + o] = bw;
    } else {
        bias[64 + p - kMlpOffB2] = from_bf16(bw);
    }
}

// mode 0: write the summed gradient to grad_out and the loss to loss_out[0];
// mode 1: Adam step on the master weights and republish the bf16 copies.
// A workgroup takes 64 consecutive parameters; its four waves sum every
// fourth partial (coalesced across the parameters), then combine in LDS.
constexpr int kReduceParams = 64;
__global__ __launch_bounds__(256) void mlp_reduce_kernel(const float* __restrict__ partial, int n_waves,
                                                         const float* __restrict__ loss_part, int batch,
                                                         int mode, MlpBuffers mb, AdamStep ad,
                                                         float* __restrict__ grad_out,
                                                         float* __restrict__ loss_out)
{
    __shared__ float part[4][kReduceParams];
    const int ln = threadIdx.x & 63, grp = threadIdx.x >> 6;
    if (blockIdx.x == 0 && grp == 0 && loss_out) {
        float s = 0.0f;
        for (int w = ln; w < n_waves; w += 64) s += loss_part[w];
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
        if (ln == 0) loss_out[0] = s / float(batch);
    }
    const int p = blockIdx.x * kReduceParams + ln;
    float gs = 0.0f;
    if (p < kMlpParams)
        for (int w = grp; w < n_waves; w += 4) gs += partial[(size_t)w * kMlpParams + p];
    part[grp][ln] = gs;
    __syncthreads();
    if (grp != 0 || p >= kMlpParams) return;
    const float gsum = part[0][ln] + part[1][ln] + part[2][ln] + part[3][ln];
    if (mode == 0) {
        grad_out[p] = gsum;
        return;
    }
    const float m = ad.beta1 * mb.m[p] + (1.0f - ad.beta1) * gsum;
    const float v = ad.beta2 * mb.v[p] + (1.0f - ad.beta2) * gsum * gsum;
    mb.m[p] = m;
    mb.v[p] = v;
    const float w = mb.master[p] - ad.lr * (m * ad.c1) / (sqrtf(v * ad.c2) + ad.eps);
    mb.master[p] = w;
    publish_param(p, w, mb.w1, mb.w2, mb.w2t, mb.bias);
}

__global__ __launch_bounds__(256) void mlp_publish_kernel(MlpBuffers mb)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kMlpParams) publish_param(p, mb.master[p], mb.w1, mb.w2, mb.w2t, mb.bias);
}

// ------------------------------------------------------------------ launchers
namespace {
inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }
}

hipError_t launch_mlp_features(const kf_ctx* ctx, const kf_tracks* t, const int32_t* target,
                               float* feats, int prec, hipStream_t s)
{
    if (t->n == 0) return hipSuccess;
    if (prec == KF_PREC_FP64)
        mlp_features_kernel<double><<<nblk(t->n, 256), 256, 0, s>>>(
            t->n, t->ld, (const double*)t->par, target, ctx->d_layers, ctx->n_layers, ctx->params, feats);
    else
        mlp_features_kernel<float><<<nblk(t->n, 256), 256, 0, s>>>(
            t->n, t->ld, (const float*)t->par, target, ctx->d_layers, ctx->n_layers, ctx->params, feats);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const MlpDev& m, const float* feats, int64_t n, int64_t ld, float* out,
                              hipStream_t s)
{
    if (n == 0) return hipSuccess;
    mlp_forward_kernel<<<nblk(n, 256), 256, 0, s>>>(n, ld, feats, m, out);
    return hipGetLastError();
}

size_t mlp_partial_bytes(int batch)
{
    const size_t waves = (size_t)nblk(batch, 16 * kGradWaves) * kGradWaves;
    return waves * kMlpParams * sizeof(float) + waves * sizeof(float) + 256;
}

hipError_t launch_mlp_step(const MlpBuffers& mb, const float* feats, const float* target, int64_t n,
                           int64_t ld, const int32_t* rows, int batch, void* scratch, int mode,
                           const AdamStep& ad, float* grad_out, float* loss_out, hipStream_t s)
{
    const unsigned nb = nblk(batch, 16 * kGradWaves);
    const int n_waves = (int)nb * kGradWaves;
    float* partial = (float*)scratch;
    float* loss_part = partial + (size_t)n_waves * kMlpParams;
    mlp_grad_kernel<<<nb, 64 * kGradWaves, 0, s>>>(feats, target, n, ld, rows, batch, mb.dev(),
                                                   partial, loss_part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    mlp_reduce_kernel<<<nblk(kMlpParams, kReduceParams), 256, 0, s>>>(partial, n_waves, loss_part,
                                                                       batch, mode, mb, ad, grad_out,
                                                                       loss_out);
    return hipGetLastError();
}

hipError_t launch_mlp_publish(const MlpBuffers& mb, hipStream_t s)
{
    mlp_publish_kernel<<<nblk(kMlpParams, 256), 256, 0, s>>>(mb);
    return hipGetLastError();
}

hipError_t launch_mlp_targets(const float* feats, const float* path, int64_t n, int64_t ld,
                              float* target, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    mlp_targets_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, ld, feats, path, target);
    return hipGetLastError();
}

}  // namespace kfmi
