// surrogate_kernels.hip -- BF16-MFMA 1D convolution network of the learned
// warm start: (emission flux, cathode temperature, bias, neutral density) ->
// (phi / V, ln(n_e / n0), ln(n_i / n0)) at the X cell centres of a diode.
//
// Net: 6 conv1d layers, kernel 5, zero padding 2, channels
// 16 -> 64 -> 64 -> 64 -> 64 -> 64 -> 3 (stored padded to 16), tanh after
// layers 1-5.  Input channels: the 4 normalised parameters and 12 functions of
// the position.  Weights are BF16 (FP32 master copies for Adam), activations
// enter every layer as BF16, all products accumulate in FP32 on
// v_mfma_f32_16x16x32_bf16.
//
// Layouts: activations channels last act[b][x][c] for the forward and input
// gradient GEMMs (K runs over channels), plus channels-first copies
// actT[b][c][x] for the weight gradient (K runs over positions); forward weights
// Wf[co][t*Cin + ci] (K contiguous), transposed weights for the input gradient
// Wb[ci][t*Cout + co]; both padded with zeros to a multiple of 32 in K.
//
// MFMA 16x16x32 (bf16) lane layout: lane l supplies A[l%16][8(l/16)+i] and
// B[8(l/16)+i][l%16], i = 0..7, and receives D[4(l/16)+i][l%16], i = 0..3.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sur {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int KS = 5;     // kernel size
constexpr int OUT = 39;   // output channels: phi / V, ln n_e / n0, ln n_i / n0, 36 velocity quantiles
constexpr int OUTP = 48;  // padded to whole 16-column matrix-core tiles
constexpr int PAD = 2;

__device__ __forceinline__ bf16x8 zero8()
{
    bf16x8 z;
#pragma unroll
    for (int i = 0; i < 8; ++i) z[i] = (__bf16)0.0f;
    return z;
}

__device__ __forceinline__ bf16x8 load8(const __bf16 *p) { return *reinterpret_cast<const bf16x8 *>(p); }

__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

// ---------------------------------------------------------------------------
// Input features.  params[b] = (Gamma m^-2 s^-1, T_c K, V volts, n_g m^-3) are
// mapped to [-1, 1] over the training ranges (log scale for the flux and the
// density); the position features resolve both sheaths and the interior.
// ---------------------------------------------------------------------------
__global__ void k_features(const float *__restrict__ params, __bf16 *__restrict__ feat, __bf16 *__restrict__ featT,
                           double *__restrict__ loss0, int X, int B)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx == 0 && loss0) *loss0 = 0.0;     // the training step's loss accumulator
    if (idx >= X * B) return;
    const int b = idx / X, x = idx - b * X;
    const float g = params[4 * b + 0], T = params[4 * b + 1], V = params[4 * b + 2], ng = params[4 * b + 3];
    const float u = ((float)x + 0.5f) / (float)X;
    float f[16];
    f[0] = 2.0f * (log10f(g / 1e19f) / log10f(12.0f)) - 1.0f;
    f[1] = (T - 2000.0f) / 200.0f;
    f[2] = (V - 12.5f) / 7.5f;
    f[3] = 2.0f * log10f(ng / 1e21f) - 1.0f;
    f[4] = 2.0f * u - 1.0f;
    f[5] = 1.0f - 2.0f * u;
    float s1, c1, s2, c2, s4, c4;
    sincospif(u, &s1, &c1);
    sincospif(2.0f * u, &s2, &c2);
    sincospif(4.0f * u, &s4, &c4);
    f[6] = s1; f[7] = c1; f[8] = s2; f[9] = c2; f[10] = s4; f[11] = c4;
    f[12] = __expf(-64.0f * u);
    f[13] = __expf(-64.0f * (1.0f - u));
    f[14] = __expf(-16.0f * u);
    f[15] = __expf(-16.0f * (1.0f - u));
    __bf16 *o = feat + (size_t)idx * 16;
#pragma unroll
    for (int c = 0; c < 16; ++c) o[c] = (__bf16)f[c];
    if (featT) {
#pragma unroll
        for (int c = 0; c < 16; ++c) featT[((size_t)b * 16 + c) * X + x] = (__bf16)f[c];
    }
}

// Four consecutive positions of one channel, stored as one 8-byte word.
__device__ __forceinline__ void store4T(__bf16 *p, float v0, float v1, float v2, float v3)
{
    typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
    bf16x4 q;
    q[0] = (__bf16)v0;
    q[1] = (__bf16)v1;
    q[2] = (__bf16)v2;
    q[3] = (__bf16)v3;
    *reinterpret_cast<bf16x4 *>(p) = q;
}

// ---------------------------------------------------------------------------
// Weights of a layer staged in LDS once per block: rows of the padded K
// length plus 8 elements, so that the 16 rows one matrix-core fragment reads
// fall on different banks.
// ---------------------------------------------------------------------------
constexpr int BLOCK_POS = 256;   // positions per block of the forward and input-gradient kernels

template <int ROWS, int KP>
__device__ __forceinline__ void stage_rows(__bf16 *lds, const __bf16 *__restrict__ src)
{
    constexpr int V = KP / 8;    // 16-byte vectors per row
    for (int v = threadIdx.x; v < ROWS * V; v += blockDim.x) {
        const int r = v / V, c = (v - r * V) * 8;
        *reinterpret_cast<bf16x8 *>(lds + r * (KP + 8) + c) = load8(src + (size_t)r * KP + c);
    }
}

// ---------------------------------------------------------------------------
// Forward conv: out[b][x][co] = act(bias[co] + sum_{t, ci} W[co][t][ci] in[b][x+t-2][ci]).
// GEMM M = positions, N = COUT, K = 5*CIN (padded to KP).  A block of 4
// waves covers BLOCK_POS positions of one sample with the layer's weights in
// LDS; a wave computes 16 positions x COUT at a time.
// ---------------------------------------------------------------------------
template <int CIN, int COUT, bool TANH>
__global__ __launch_bounds__(256) void k_conv_fwd(const __bf16 *__restrict__ in, const __bf16 *__restrict__ Wf,
                                                  const float *__restrict__ bias, float *__restrict__ yf,
                                                  __bf16 *__restrict__ yb, __bf16 *__restrict__ ybT, int X, int B)
{
    constexpr int K = KS * CIN;
    constexpr int KP = (K + 31) / 32 * 32;
    constexpr int NT = COUT / 16;
    __shared__ __bf16 wl[COUT * (KP + 8)];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int tiles = (X + BLOCK_POS - 1) / BLOCK_POS;
    const int b = blockIdx.x / tiles;
    if (b >= B) return;
    stage_rows<COUT, KP>(wl, Wf);
    __syncthreads();
    const int m = lane & 15, kb = lane >> 4;
    const __bf16 *inb = in + (size_t)b * X * CIN;
    const int xb = (blockIdx.x - b * tiles) * BLOCK_POS;
    for (int x0 = xb + w * 16; x0 < min(X, xb + BLOCK_POS); x0 += 64) {
    f32x4 acc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[nt] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KP / 32; ++ks) {
        const int kappa = ks * 32 + kb * 8;
        bf16x8 a = zero8();
        if (kappa < K) {
            const int t = kappa / CIN, ci = kappa - t * CIN;
            const int xs = x0 + m + t - PAD;
            if (xs >= 0 && xs < X) a = load8(inb + (size_t)xs * CIN + ci);
        }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const bf16x8 bw = *reinterpret_cast<const bf16x8 *>(wl + (nt * 16 + m) * (KP + 8) + kappa);
            acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw, acc[nt], 0, 0, 0);
        }
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int co = nt * 16 + m;
        float v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int x = x0 + kb * 4 + i;
            v[i] = acc[nt][i] + bias[co];
            if (TANH) v[i] = tanhf(v[i]);
            const size_t o = ((size_t)b * X + x) * COUT + co;
            yf[o] = v[i];
            if (yb) yb[o] = (__bf16)v[i];
        }
        if (ybT) store4T(ybT + ((size_t)b * COUT + co) * X + x0 + kb * 4, v[0], v[1], v[2], v[3]);
    }
    }
}

// ---------------------------------------------------------------------------
// Loss: mean over (b, channel < OUT, x) of (out - target)^2.  Writes
// dZ = 2 (out - target) / count as BF16 in the padded OUTP-channel layout.
// target[b][c][x], out[b][x][OUTP].
// ---------------------------------------------------------------------------
__global__ void k_loss(const float *__restrict__ out, const float *__restrict__ target, __bf16 *__restrict__ dz,
                       __bf16 *__restrict__ dzT, double *__restrict__ loss, int X, int B)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const double inv = 1.0 / ((double)OUT * (double)X * (double)B);
    double acc = 0.0;
    if (idx < X * B) {
        const int b = idx / X, x = idx - b * X;
        for (int c = 0; c < OUTP; ++c) {
            float g = 0.0f;
            if (c < OUT) {
                const float d = out[(size_t)idx * OUTP + c] - target[((size_t)b * OUT + c) * X + x];
                acc += (double)d * d;
                g = (float)(2.0 * inv) * d;
            }
            dz[(size_t)idx * OUTP + c] = (__bf16)g;
            dzT[((size_t)b * OUTP + c) * X + x] = (__bf16)g;
        }
    }
    // wave reduction, one atomic per wave
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0 && acc != 0.0) atomicAdd(loss, acc * inv);
}

// ---------------------------------------------------------------------------
// Input gradient: dY[b][x][ci] = sum_{t, co} W[co][t][ci] dZ[b][x-t+2][co],
// then (tanh) dZprev = dY (1 - y^2) stored as BF16.  GEMM M = positions,
// N = CIN, K = 5*COUT (padded), B from the transposed weights Wb[ci][t*COUT+co].
// ---------------------------------------------------------------------------
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_conv_dgrad(const __bf16 *__restrict__ dz, const __bf16 *__restrict__ Wb,
                                                    const float *__restrict__ yprev, __bf16 *__restrict__ dzprev,
                                                    __bf16 *__restrict__ dzprevT, int X, int B)
{
    constexpr int K = KS * COUT;
    constexpr int KP = (K + 31) / 32 * 32;
    constexpr int NT = CIN / 16;
    __shared__ __bf16 wl[CIN * (KP + 8)];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int tiles = (X + BLOCK_POS - 1) / BLOCK_POS;
    const int b = blockIdx.x / tiles;
    if (b >= B) return;
    stage_rows<CIN, KP>(wl, Wb);
    __syncthreads();
    const int m = lane & 15, kb = lane >> 4;
    const __bf16 *dzb = dz + (size_t)b * X * COUT;
    const int xb = (blockIdx.x - b * tiles) * BLOCK_POS;
    for (int x0 = xb + w * 16; x0 < min(X, xb + BLOCK_POS); x0 += 64) {
    f32x4 acc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[nt] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KP / 32; ++ks) {
        const int kappa = ks * 32 + kb * 8;
        bf16x8 a = zero8();
        if (kappa < K) {
            const int t = kappa / COUT, co = kappa - t * COUT;
            const int xs = x0 + m - t + PAD;
            if (xs >= 0 && xs < X) a = load8(dzb + (size_t)xs * COUT + co);
        }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const bf16x8 bw = *reinterpret_cast<const bf16x8 *>(wl + (nt * 16 + m) * (KP + 8) + kappa);
            acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw, acc[nt], 0, 0, 0);
        }
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int ci = nt * 16 + m;
        float v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int x = x0 + kb * 4 + i;
            const size_t o = ((size_t)b * X + x) * CIN + ci;
            const float y = yprev[o];
            v[i] = acc[nt][i] * (1.0f - y * y);
            dzprev[o] = (__bf16)v[i];
        }
        store4T(dzprevT + ((size_t)b * CIN + ci) * X + x0 + kb * 4, v[0], v[1], v[2], v[3]);
    }
    }
}

// ---------------------------------------------------------------------------
// Weight and bias gradients: dW[co][t*CIN+ci] = sum_{b,x} dZ[b][co][x] in[b][ci][x+t-2],
// db[co] = sum_{b,x} dZ[b][co][x], from the channels-first copies.  GEMM M =
// COUT, N = 5*CIN (16-wide tiles, one tap t per tile), K = positions, 32 per
// MFMA.  Lane (m, kb) reads 8 consecutive positions as one 16-byte load for
// A; for B the same 8 positions shifted by t - 2, taken from a 12-element
// window (16 bytes plus one dword on each side, zero outside the sample).
// ---------------------------------------------------------------------------
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <int T>
__device__ __forceinline__ bf16x8 window8(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3, uint32_t w4,
                                          uint32_t w5)
{
    // elements T .. T+7 of the 12-element window w0..w5 (2 per dword, low first)
    u32x4 r;
    if constexpr (T == 0) r = (u32x4){w0, w1, w2, w3};
    else if constexpr (T == 2) r = (u32x4){w1, w2, w3, w4};
    else if constexpr (T == 4) r = (u32x4){w2, w3, w4, w5};
    else if constexpr (T == 1)
        r = (u32x4){(w0 >> 16) | (w1 << 16), (w1 >> 16) | (w2 << 16), (w2 >> 16) | (w3 << 16), (w3 >> 16) | (w4 << 16)};
    else
        r = (u32x4){(w1 >> 16) | (w2 << 16), (w2 >> 16) | (w3 << 16), (w3 >> 16) | (w4 << 16), (w4 >> 16) | (w5 << 16)};
    return __builtin_bit_cast(bf16x8, r);
}

// ---------------------------------------------------------------------------
// Weight and bias gradients as partial sums over slices of WG_SLICE positions
// of one sample: block p = (sample, slice) writes part[p][co][kappa] and
// pbias[p][co]; k_reduce_adam sums the partials in a fixed order.  Wave w of
// the block takes output-channel tile w % MT and half of the input-channel
// tiles (c = w / MT, w / MT + 2, ...), all five taps of each: for every 32
// positions one 16-byte load of dZ (A) is shared by up to 10 MFMAs, and one
// 16-byte window of the input per input tile (B) by its five taps.
// ---------------------------------------------------------------------------
constexpr int WG_SLICE = 512;

template <int CIN, int COUT>
__global__ __launch_bounds__(512) void k_conv_wgrad_part(const __bf16 *__restrict__ dzT, const __bf16 *__restrict__ inT,
                                                         float *__restrict__ part, float *__restrict__ pbias, int X)
{
    constexpr int K = KS * CIN;
    constexpr int KP = (K + 31) / 32 * 32;
    constexpr int MT = COUT / 16, CT = CIN / 16;
    constexpr int CH = CT >= 2 ? 2 : 1;           // waves per output tile
    constexpr int CPW = CT / CH;                  // input tiles per wave
    static_assert(CIN % 16 == 0 && CT % CH == 0, "whole input-channel tiles");
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (w >= MT * CH) return;
    const int mt = w % MT, ch = w / MT;
    const int slices = (X + WG_SLICE - 1) / WG_SLICE;
    const int p = blockIdx.x, b = p / slices;
    const int xb = (p - b * slices) * WG_SLICE, xe = min(X, xb + WG_SLICE);
    const int m = lane & 15, kb = lane >> 4;
    const int co = mt * 16 + m;
    const __bf16 *arow = dzT + ((size_t)b * COUT + co) * X;
    const __bf16 *brow[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c) brow[c] = inT + ((size_t)b * CIN + (ch + CH * c) * 16 + m) * X;
    f32x4 acc[KS][CPW];
#pragma unroll
    for (int t = 0; t < KS; ++t)
#pragma unroll
        for (int c = 0; c < CPW; ++c) acc[t][c] = (f32x4){0.f, 0.f, 0.f, 0.f};
    float bsum = 0.0f;
    for (int x0 = xb; x0 < xe; x0 += 32) {
        const int xa = x0 + kb * 8;
        const bf16x8 a = load8(arow + xa);
        if (ch == 0) {
#pragma unroll
            for (int i = 0; i < 8; ++i) bsum += (float)a[i];
        }
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
            const uint32_t *bw = reinterpret_cast<const uint32_t *>(brow[c]);
            const u32x4 mid = *reinterpret_cast<const u32x4 *>(brow[c] + xa);
            const uint32_t lo = xa > 0 ? bw[(xa >> 1) - 1] : 0u;
            const uint32_t hi = xa + 8 < X ? bw[(xa >> 1) + 4] : 0u;
            acc[0][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, window8<0>(lo, mid[0], mid[1], mid[2], mid[3], hi),
                                                                acc[0][c], 0, 0, 0);
            acc[1][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, window8<1>(lo, mid[0], mid[1], mid[2], mid[3], hi),
                                                                acc[1][c], 0, 0, 0);
            acc[2][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, window8<2>(lo, mid[0], mid[1], mid[2], mid[3], hi),
                                                                acc[2][c], 0, 0, 0);
            acc[3][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, window8<3>(lo, mid[0], mid[1], mid[2], mid[3], hi),
                                                                acc[3][c], 0, 0, 0);
            acc[4][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, window8<4>(lo, mid[0], mid[1], mid[2], mid[3], hi),
                                                                acc[4][c], 0, 0, 0);
        }
    }
    float *out = part + (size_t)p * COUT * KP;
#pragma unroll
    for (int t = 0; t < KS; ++t)
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
            const int kappa = t * CIN + (ch + CH * c) * 16 + m;
#pragma unroll
            for (int i = 0; i < 4; ++i) out[(size_t)(mt * 16 + kb * 4 + i) * KP + kappa] = acc[t][c][i];
        }
    if (ch == 0) {
        bsum += __shfl_xor(bsum, 16, 64);
        bsum += __shfl_xor(bsum, 32, 64);
        if (kb == 0) pbias[(size_t)p * COUT + co] = bsum;
    }
}

// The gradient of one layer from its partials (summed in partial order),
// then Adam on the FP32 master weights and biases and the BF16 copies of the
// weights: forward layout Wf[co][kappa] and transposed Wb[ci][t*COUTP + co].
// One thread per weight (padded [COUTP][KP]) and per bias.
__global__ void k_reduce_adam(const float *__restrict__ part, const float *__restrict__ pbias, int P,
                              float *__restrict__ wm, float *__restrict__ mw, float *__restrict__ vw,
                              float *__restrict__ dw, float *__restrict__ bias, float *__restrict__ mb,
                              float *__restrict__ vb, float *__restrict__ db, __bf16 *__restrict__ Wf,
                              __bf16 *__restrict__ Wb, int cin, int coutp, int cout_real, int kp, int kpb, float lr,
                              float b1, float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int nw = coutp * kp;
    if (i >= nw + coutp) return;
    float *w, *mo, *ve, *g;
    int co, kappa = 0, stride, at;
    if (i < nw) {
        co = i / kp;
        kappa = i - co * kp;
        w = wm + i; mo = mw + i; ve = vw + i; g = dw + i;
        stride = nw;
        at = i;
    } else {
        co = i - nw;
        w = bias + co; mo = mb + co; ve = vb + co; g = db + co;
        stride = coutp;
        at = co;
    }
    const bool live = co < cout_real && (i >= nw || kappa < KS * cin);
    float gi = 0.0f;
    if (live) {
        const float *src = i < nw ? part : pbias;
        for (int q = 0; q < P; ++q) gi += src[(size_t)q * stride + at];
    }
    *g = gi;
    const float m1 = b1 * *mo + (1.0f - b1) * gi;
    const float v1 = b2 * *ve + (1.0f - b2) * gi * gi;
    *mo = m1;
    *ve = v1;
    const float nwv = *w - lr * (m1 / c1) / (sqrtf(v1 / c2) + eps);
    *w = nwv;
    if (i < nw) {
        const __bf16 v = (__bf16)(live ? nwv : 0.0f);
        Wf[i] = v;
        if (kappa < KS * cin) {
            const int t = kappa / cin, ci = kappa - t * cin;
            Wb[(size_t)ci * kpb + t * coutp + co] = v;
        }
    }
}

// masters [COUTP][KP] (kappa = t*CIN + ci) -> Wf (same layout, bf16) and
// Wb[ci][t*COUTP + co] (padded to KPB)
__global__ void k_requant(const float *__restrict__ wm, __bf16 *__restrict__ Wf, __bf16 *__restrict__ Wb, int cin,
                          int coutp, int cout_real, int kp, int kpb)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= coutp * kp) return;
    const int co = i / kp, kappa = i - co * kp;
    const bool live = co < cout_real && kappa < KS * cin;
    const __bf16 v = (__bf16)(live ? wm[i] : 0.0f);
    Wf[i] = v;
    if (kappa < KS * cin) {
        const int t = kappa / cin, ci = kappa - t * cin;
        Wb[(size_t)ci * kpb + t * coutp + co] = v;
    }
}

// Initial weights: N(0, 1/(5*CIN)) from Philox keyed by (layer, seed).
__global__ void k_init_weights(float *__restrict__ wm, int cin, int coutp, int cout_real, int kp, uint32_t layer,
                               uint32_t seed)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= coutp * kp) return;
    const int co = i / kp, kappa = i - co * kp;
    float v = 0.0f;
    if (co < cout_real && kappa < KS * cin) {
        const uint4 r = philox((uint32_t)i, layer, 7u, 0u, seed, 0x5A11u);
        const float u1 = ((float)(r.x >> 8) + 0.5f) * (1.0f / 16777216.0f);
        const float u2 = ((float)(r.y >> 8) + 0.5f) * (1.0f / 16777216.0f);
        float s, c;
        sincospif(2.0f * u2, &s, &c);
        v = sqrtf(-2.0f * logf(u1)) * c * sqrtf(1.0f / (float)(KS * cin));
    }
    wm[i] = v;
}

// Network output -> densities per cell for the warm-start loader:
// dens[d][0][x] = n0 exp(out[d][x][1]), dens[d][1][x] = n0 exp(out[d][x][2]).
__global__ void k_to_densities(const float *__restrict__ out, const double *__restrict__ n0, double *__restrict__ dens,
                               int X, int B)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= X * B) return;
    const int b = idx / X, x = idx - b * X;
    dens[((size_t)b * 2 + 0) * X + x] = n0[b] * exp((double)out[(size_t)idx * OUTP + 1]);
    dens[((size_t)b * 2 + 1) * X + x] = n0[b] * exp((double)out[(size_t)idx * OUTP + 2]);
}

// Network output -> the state the warm-start loader reads, [b][OUT][x]:
// densities as k_to_densities, phi = V out[0], the electron quantiles
// (channels 3..20) times the 1 eV electron speed sqrt(e / m_e), the ion ones
// (21..38) times the 1 eV ion speed sqrt(e / m_i).  params[b][2] is V.
__global__ void k_to_state(const float *__restrict__ out, const float *__restrict__ params,
                           const double *__restrict__ n0, double *__restrict__ state, int X, int B)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= X * B) return;
    const int b = idx / X, x = idx - b * X;
    const float *o = out + (size_t)idx * OUTP;
    double *st = state + (size_t)b * OUT * X + x;
    const double ve = sqrt(1.602176634e-19 / 9.1093837015e-31);
    const double vi = sqrt(1.602176634e-19 / (6.6464731e-27 - 9.1093837015e-31));
    st[0] = n0[b] * exp((double)o[1]);
    st[(size_t)X] = n0[b] * exp((double)o[2]);
    st[(size_t)2 * X] = (double)params[(size_t)b * 4 + 2] * (double)o[0];
    for (int c = 3; c < OUT; ++c) st[(size_t)c * X] = (double)o[c] * (c < 21 ? ve : vi);
}

// Network output [b][x][OUTP] -> caller layout [b][OUT][x].
__global__ void k_unpack(const float *__restrict__ y, float *__restrict__ out, int X, int B)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= X * B) return;
    const int b = idx / X, x = idx - b * X;
    for (int c = 0; c < OUT; ++c) out[((size_t)b * OUT + c) * X + x] = y[(size_t)idx * OUTP + c];
}

}  // namespace sur

// ---------------------------------------------------------------------------
// Launch wrappers
// ---------------------------------------------------------------------------
using namespace sur;

extern "C" hipError_t surx_features(const float *params, __bf16 *feat, __bf16 *featT, double *loss0, int X, int B,
                                    hipStream_t s)
{
    hipLaunchKernelGGL(k_features, dim3((X * B + 255) / 256), dim3(256), 0, s, params, feat, featT, loss0, X, B);
    return hipGetLastError();
}

// ybT may be null (inference: no weight gradient follows)
extern "C" hipError_t surx_conv_fwd(int layer, const __bf16 *in, const __bf16 *Wf, const float *bias, float *yf,
                                    __bf16 *yb, __bf16 *ybT, int X, int B, hipStream_t s)
{
    dim3 g((X + BLOCK_POS - 1) / BLOCK_POS * B), t(256);
    if (layer == 0) hipLaunchKernelGGL((k_conv_fwd<16, 64, true>), g, t, 0, s, in, Wf, bias, yf, yb, ybT, X, B);
    else if (layer < 5) hipLaunchKernelGGL((k_conv_fwd<64, 64, true>), g, t, 0, s, in, Wf, bias, yf, yb, ybT, X, B);
    else hipLaunchKernelGGL((k_conv_fwd<64, OUTP, false>), g, t, 0, s, in, Wf, bias, yf, yb, ybT, X, B);
    return hipGetLastError();
}

extern "C" hipError_t surx_loss(const float *out, const float *target, __bf16 *dz, __bf16 *dzT, double *loss, int X,
                                int B, hipStream_t s)
{
    hipLaunchKernelGGL(k_loss, dim3((X * B + 255) / 256), dim3(256), 0, s, out, target, dz, dzT, loss, X, B);
    return hipGetLastError();
}

// input gradient of layer `layer` (1..5; layer 0 has none)
extern "C" hipError_t surx_conv_dgrad(int layer, const __bf16 *dz, const __bf16 *Wb, const float *yprev,
                                      __bf16 *dzprev, __bf16 *dzprevT, int X, int B, hipStream_t s)
{
    dim3 g((X + BLOCK_POS - 1) / BLOCK_POS * B), t(256);
    if (layer == 5) hipLaunchKernelGGL((k_conv_dgrad<64, OUTP>), g, t, 0, s, dz, Wb, yprev, dzprev, dzprevT, X, B);
    else hipLaunchKernelGGL((k_conv_dgrad<64, 64>), g, t, 0, s, dz, Wb, yprev, dzprev, dzprevT, X, B);
    return hipGetLastError();
}

// partial weight and bias gradients of layer `layer` (grid: batch x slices)
extern "C" hipError_t surx_conv_wgrad_part(int layer, const __bf16 *dzT, const __bf16 *inT, float *part, float *pbias,
                                           int X, int B, hipStream_t s)
{
    const dim3 g((unsigned)(B * ((X + WG_SLICE - 1) / WG_SLICE))), t(512);
    if (layer == 0)
        hipLaunchKernelGGL((k_conv_wgrad_part<16, 64>), g, t, 0, s, dzT, inT, part, pbias, X);
    else if (layer < 5)
        hipLaunchKernelGGL((k_conv_wgrad_part<64, 64>), g, t, 0, s, dzT, inT, part, pbias, X);
    else
        hipLaunchKernelGGL((k_conv_wgrad_part<64, OUTP>), g, t, 0, s, dzT, inT, part, pbias, X);
    return hipGetLastError();
}

extern "C" int surx_wgrad_parts(int X, int B) { return B * ((X + WG_SLICE - 1) / WG_SLICE); }

extern "C" hipError_t surx_reduce_adam(const float *part, const float *pbias, int P, float *wm, float *mw, float *vw,
                                       float *dw, float *bias, float *mb, float *vb, float *db, __bf16 *Wf, __bf16 *Wb,
                                       int cin, int coutp, int cout_real, int kp, int kpb, float lr, float b1,
                                       float b2, float eps, float c1, float c2, hipStream_t s)
{
    const int n = coutp * kp + coutp;
    hipLaunchKernelGGL(k_reduce_adam, dim3((n + 255) / 256), dim3(256), 0, s, part, pbias, P, wm, mw, vw, dw, bias,
                       mb, vb, db, Wf, Wb, cin, coutp, cout_real, kp, kpb, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

extern "C" hipError_t surx_requant(const float *wm, __bf16 *Wf, __bf16 *Wb, int cin, int coutp, int cout_real, int kp,
                                   int kpb, hipStream_t s)
{
    const int n = coutp * kp;
    hipLaunchKernelGGL(k_requant, dim3((n + 255) / 256), dim3(256), 0, s, wm, Wf, Wb, cin, coutp, cout_real, kp, kpb);
    return hipGetLastError();
}

extern "C" hipError_t surx_init_weights(float *wm, int cin, int coutp, int cout_real, int kp, uint32_t layer,
                                        uint32_t seed, hipStream_t s)
{
    const int n = coutp * kp;
    hipLaunchKernelGGL(k_init_weights, dim3((n + 255) / 256), dim3(256), 0, s, wm, cin, coutp, cout_real, kp, layer,
                       seed);
    return hipGetLastError();
}

extern "C" hipError_t surx_to_densities(const float *out, const double *n0, double *dens, int X, int B, hipStream_t s)
{
    hipLaunchKernelGGL(k_to_densities, dim3((X * B + 255) / 256), dim3(256), 0, s, out, n0, dens, X, B);
    return hipGetLastError();
}

extern "C" hipError_t surx_to_state(const float *out, const float *params, const double *n0, double *state, int X,
                                    int B, hipStream_t s)
{
    hipLaunchKernelGGL(k_to_state, dim3((X * B + 255) / 256), dim3(256), 0, s, out, params, n0, state, X, B);
    return hipGetLastError();
}

extern "C" hipError_t surx_unpack(const float *y, float *out, int X, int B, hipStream_t s)
{
    hipLaunchKernelGGL(k_unpack, dim3((X * B + 255) / 256), dim3(256), 0, s, y, out, X, B);
    return hipGetLastError();
}
