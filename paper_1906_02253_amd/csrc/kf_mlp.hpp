// The learned initial guess of the propagate-to-radius solve: an
// 8 -> 64 (tanh) -> 64 (tanh) -> 1 network evaluated by a whole wavefront on
// bf16 matrix cores (FP32 accumulate).  Not part of the paper; it supplies a
// start for the iterative solve that the paper's layer-to-layer propagation
// (Sec. 3.1) needs, the exact solve staying the arbiter.  The output is the
// correction to the straight-line path length in units of h s_line^2 (see
// mlp_guess): the straight line is exact for straight tracks, and the
// network's error then scales with the correction, not with the path.
//
// Transposed form: a layer computes H^T = W X^T, the rows of the batch along
// the columns of a 16x16 tile.  With v_mfma_f32_16x16x16_bf16, lane l of a
// wave holds A[l%16][4(l/16)+j], B[4(l/16)+j][l%16] and D[4(l/16)+j][l%16]
// (j = 0..3), so the D tile of one layer is, element for element, the B
// operand of the next: no data moves between the layers.
#pragma once

#include "kf_internal.hpp"
#include "kf_math.hpp"

namespace kfmi {

constexpr int kMlpIn = 8;
constexpr int kMlpHidden = 64;
constexpr int kMlpParams = 4801;       // W1[64][8], b1[64], W2[64][64], b2[64], w3[64], b3
constexpr int kMlpOffB1 = 512, kMlpOffW2 = 576, kMlpOffB2 = 4672, kMlpOffW3 = 4736, kMlpOffB3 = 4800;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bf16, round to nearest even (NaN stays NaN)
__device__ inline uint16_t to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ inline float from_bf16(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ inline float round_bf16(float f) { return from_bf16(to_bf16(f)); }

// tanh from the exponential: 1 - 2 / (e^{2x} + 1), saturated beyond |x| = 15
__device__ inline float mlp_tanh(float x)
{
    x = fminf(fmaxf(x, -15.0f), 15.0f);
    return 1.0f - __fdividef(2.0f, __expf(2.0f * x) + 1.0f);
}

__device__ inline f32x4 mfma_bf16(bf16x4 a, bf16x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// four consecutive bf16 from memory (8-byte aligned)
__device__ inline bf16x4 load_bf16x4(const uint16_t* p)
{
    const uint2 v = *(const uint2*)p;
    bf16x4 r;
    r[0] = (short)(v.x & 0xffffu);
    r[1] = (short)(v.x >> 16);
    r[2] = (short)(v.y & 0xffffu);
    r[3] = (short)(v.y >> 16);
    return r;
}

__device__ inline bf16x4 pack_bf16x4(float a, float b, float c, float d)
{
    bf16x4 r;
    r[0] = (short)to_bf16(a);
    r[1] = (short)to_bf16(b);
    r[2] = (short)to_bf16(c);
    r[3] = (short)to_bf16(d);
    return r;
}

// The part of x below its bf16 rounding, itself rounded to bf16: x_hi + x_lo
// carries about 16 significant bits.
__device__ inline float bf16_rest(float x) { return x - round_bf16(x); }

// B operand of the transposed inputs of one 16-row tile from four lane
// values v[0..3]: lane groups 0 and 1 hold the high bf16 parts of inputs
// 0..3 and 4..7, groups 2 and 3 the low parts of the same inputs (the first
// layer's weights are stored twice along K, so one product sums both).
__device__ inline bf16x4 split_inputs(const float v[4], int g)
{
    if (g < 2) return pack_bf16x4(v[0], v[1], v[2], v[3]);
    return pack_bf16x4(bf16_rest(v[0]), bf16_rest(v[1]), bf16_rest(v[2]), bf16_rest(v[3]));
}

// Forward pass of one tile of 16 rows.  xb: split_inputs of the row l%16 of
// the tile (lane l: inputs 4((l/16)%2)..+3).  The weights are bf16; the
// activations enter every product as a high and a low bf16 part (FP32
// accumulation), so they keep about 16 bits.  Fills h1, h2 with the hidden
// activations in D layout (lane l: units 16m + 4(l/16) + j of row l%16) and
// returns the output of row l%16 in every lane.  Must be called by all 64
// lanes of the wave.
__device__ inline float mlp_tile(const MlpDev& m, bf16x4 xb, f32x4 h1[4], f32x4 h2[4])
{
    const int ln = (int)(threadIdx.x & 63);
    const int r = ln & 15, g = ln >> 4;
    bf16x4 hb[4], hl[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
        acc = mfma_bf16(load_bf16x4(m.w1 + (16 * mt + r) * 16 + 4 * g), xb, acc);
#pragma unroll
        for (int j = 0; j < 4; ++j) h1[mt][j] = mlp_tanh(acc[j] + m.bias[16 * mt + 4 * g + j]);
        hb[mt] = pack_bf16x4(h1[mt][0], h1[mt][1], h1[mt][2], h1[mt][3]);
        hl[mt] = pack_bf16x4(bf16_rest(h1[mt][0]), bf16_rest(h1[mt][1]), bf16_rest(h1[mt][2]),
                             bf16_rest(h1[mt][3]));
    }
    float y = 0.0f;
#pragma unroll
    for (int mo = 0; mo < 4; ++mo) {
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) {
            const bf16x4 a = load_bf16x4(m.w2 + (16 * mo + r) * 64 + 16 * kt + 4 * g);
            acc = mfma_bf16(a, hb[kt], acc);
            acc = mfma_bf16(a, hl[kt], acc);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int u = 16 * mo + 4 * g + j;
            h2[mo][j] = mlp_tanh(acc[j] + m.bias[64 + u]);
            y += m.bias[128 + u] * h2[mo][j];
        }
    }
    // the four lane groups hold the four quarters of the output sum
    y += __shfl_xor(y, 16);
    y += __shfl_xor(y, 32);
    return y + m.bias[192];
}

// Whole-wave inference: lane L passes the inputs of its own row and gets its
// own output.  Must be called by all 64 lanes (uniform control flow).  want:
// the lanes whose output is used (a wave-uniform mask); the 16-row tile of a
// group of 16 lanes none of which wants its output is skipped, and those
// lanes get 0.
__device__ inline float mlp_wave(const MlpDev& m, const float f[kMlpIn], uint64_t want = ~0ull)
{
    const int ln = (int)(threadIdx.x & 63);
    const int r = ln & 15, g = ln >> 4;
    float mine = 0.0f;
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        if (((want >> (16 * ct)) & 0xFFFFull) == 0) continue;
        const int src = 16 * ct + r;
        float v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float a = __shfl(f[j], src), b = __shfl(f[4 + j], src);
            v[j] = (g & 1) ? b : a;
        }
        const bf16x4 xb = split_inputs(v, g);
        f32x4 h1[4], h2[4];
        const float y = mlp_tile(m, xb, h1, h2);
        if (g == ct) mine = y;
    }
    return mine;
}

// Path-length guess [cm] for a barrel target from the inputs f and the
// network output y: s_line + k y with k = h s_line^2, the order of the
// curvature correction to the straight line, so that the network predicts
// an O(1) factor and its error scales with the correction.
__device__ inline float mlp_guess(const float f[kMlpIn], float y)
{
    const float k = f[3] * f[5] * f[5] / f[4];
    return 100.0f * (f[5] + k * y);
}

// Training target for a propagation of transverse path length `path` [cm]
// whose inputs are f: the output that makes mlp_guess return `path`,
// (path - s_line) / (h s_line^2) in the inputs' units; 0 where the
// curvature term vanishes (a straight track, or a zero target scale).
__device__ inline float mlp_target(const float f[kMlpIn], float path)
{
    const float k = f[4] != 0.0f ? f[3] * f[5] * f[5] / f[4] : 0.0f;
    return fabsf(k) > 1e-9f ? (path / 100.0f - f[5]) / k : 0.0f;
}

// Network inputs for propagating state p to layer L: rho/100, sin and cos
// of (phi - atan2(y, x)), h * (target radius, or 100 cm for a disk) with h the
// curvature in the field at the start point, target radius or disk z over
// 100, straight-line path length over 100 (tangent-line intersection / exact
// disk path), cot theta, z/100.
template <typename T>
__device__ inline void mlp_features(const T p[6], const kf_layer& L, const kf_params& prm,
                                    float f[kMlpIn])
{
    T bz = T(prm.bz);
    if (prm.field_z0 > 0.0) {
        T bx, by;
        field_at(T(prm.bz), T(prm.field_z0), p[0], p[1], p[2], &bx, &by, &bz);
    }
    const T kb = T(kKappa) * bz;
    const T rho = Tr<T>::sqrt_(p[0] * p[0] + p[1] * p[1]);
    T sph, cph, sth, cth;
    Tr<T>::sincos_(p[4], &sph, &cph);
    Tr<T>::sincos_(p[5], &sth, &cth);
    const bool disk = L.kind == 1;
    const T tgt = T(L.r_or_z);
    const T h = -kb * p[3];
    f[0] = float(rho / T(100));
    f[1] = rho > T(0) ? float((p[0] * sph - p[1] * cph) / rho) : 0.0f;
    f[2] = rho > T(0) ? float((p[0] * cph + p[1] * sph) / rho) : 1.0f;
    f[3] = float(h * (disk ? T(100) : tgt));
    f[4] = float(tgt / T(100));
    const T sl = disk ? (tgt - p[2]) * sth / cth : line_guess(p[0], p[1], cph, sph, tgt);
    f[5] = float(sl / T(100));
    f[6] = float(cth / sth);
    f[7] = float(p[2] / T(100));
}

}  // namespace kfmi
