// Learned warm start for the level-2 eigenproblems (an extension of the
// method, not in the paper): a 3-layer 3D CNN maps the standardised
// log-permeability patch of each 8^3 element (with a one-cell halo) to k
// cell vectors that start the element's eigensolve.
//
//   a1 = relu(conv([patch, c_0..c_{k-1}], W1) + b1)   1+k -> 32 channels, 10^3 -> 8^3
//   a2 = relu(conv(a1, W2) + b2)                      32 -> 32 channels, zero padding 1
//   X  = c + conv(a2, W3) + b3                        32 -> k channels, zero padding 1
//
// c_j are the k lowest cosine modes of the homogeneous element (the start
// block of the cold eigensolve), cos(pi p (x+1/2)/8) cos(pi q (y+1/2)/8)
// cos(pi r (z+1/2)/8), evaluated on the patch grid (cells -1..8) as input
// channels and on the element (cells 0..7) as the base the network corrects.
// k is even (2, 4, 6 or 8).
//
// conv is the 3x3x3 cross-correlation y[o][p] = sum_c sum_t W[o][c][t]
// x[c][p + t] with t = (dz, dy, dx) in {0,1,2}^3.  Weights are bfloat16
// values, every product is accumulated in float32; activations are float32.
//
// Parameter vector (flat, this order): W1[32][1+k][27], b1[32],
// W2[32][32][27], b2[32], W3[k][32][27], b3[k].
//
// Training loss of one element (S: weight diagonal tr K~ of the element's
// cells normalised to mean 1; Phi: the first k eigenvectors, scaled so that
// Phi^T S Phi = I): loss = || Phi - X^T C* ||_S^2 with
// C* = (X S X^T)^-1 X S Phi, the S-distance of Phi from span(X).  Its
// gradient is dloss/dX = -2 C* (S R)^T with R = Phi - X^T C* (C* minimises
// the inner problem).  The batch loss is the mean over elements.
#include "common.hpp"

namespace specmg {

constexpr int kCnnC = 32;         // hidden channels
constexpr int kCnnIn = 1000;      // 10^3 input patch
constexpr int kCnnTile = 1000;    // LDS tile per input channel (10^3, zero halo for padded layers)

__device__ __forceinline__ float bf_lo(uint32_t u) { return __builtin_bit_cast(float, u << 16); }
__device__ __forceinline__ float bf_hi(uint32_t u) { return __builtin_bit_cast(float, u & 0xFFFF0000u); }

// float -> bfloat16, round to nearest even (NaN kept quiet)
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __builtin_bit_cast(float, (uint32_t)h << 16); }

// cosine mode j (j < 8, by increasing p^2+q^2+r^2, ties x before y before z)
// at integer cell coordinates (x, y, z) of an 8^3 block (-1..8 on the patch
// grid), cos(pi p (x+1/2)/8) cos(pi q (y+1/2)/8) cos(pi r (z+1/2)/8) with
// p, q, r in {0, 1}: a product of 1-D factors, read from c1[x + 1] =
// cos(pi (x+1/2)/8) (a factor with exponent 0 is 1).
// (p, q, r) of mode j as bit j of three masks: p for j in {1, 4, 5, 7},
// q for {2, 4, 6, 7}, r for {3, 5, 6, 7}
__device__ __forceinline__ void cnn_mode_pqr(int j, int& p, int& q, int& r) {
    p = (0xB2 >> j) & 1;
    q = (0xD4 >> j) & 1;
    r = (0xE8 >> j) & 1;
}

// the 10 factors c1[0..9] for x = -1..8; every thread of the block calls it
__device__ __forceinline__ void cnn_cos_table(double* c1) {
    if (threadIdx.x < 10) c1[threadIdx.x] = cos(3.14159265358979323846 / 8.0 * ((int)threadIdx.x - 1 + 0.5));
    __syncthreads();
}

__device__ __forceinline__ float cnn_mode(const double* c1, int j, int x, int y, int z) {
    int p, q, r;
    cnn_mode_pqr(j, p, q, r);
    const double fx = p ? c1[x + 1] : 1.0, fy = q ? c1[y + 1] : 1.0, fz = r ? c1[z + 1] : 1.0;
    return (float)(fx * fy * fz);
}

// ---------------------------------------------------------------------------
// patches: log kappa on the element and its halo (the nearest boundary cell
// repeated outside the domain), standardised by the patch's own mean and
// standard deviation (population, 1e-6 under the root).  Optionally also the
// element's weight diagonal tr K~ = s_scale * kappa (s_scale = 3 / h^2), cell
// order x fastest.
__global__ __launch_bounds__(256) void k_cnn_patches(FineGeom g, const double* __restrict__ perm, int e0,
                                                     double s_scale, float* __restrict__ out,
                                                     double* __restrict__ s_out) {
    __shared__ double sv[kCnnIn];
    __shared__ double sred[4];
    const int e = e0 + blockIdx.x;
    const int ex = e % g.mx, ey = (e / g.mx) % g.my, ez = e / (g.mx * g.my);
    double s1 = 0.0;
    for (int t = threadIdx.x; t < kCnnIn; t += blockDim.x) {
        const int x = t % 10, y = (t / 10) % 10, z = t / 100;
        int gx = ex * 8 + x - 1, gy = ey * 8 + y - 1, gz = ez * 8 + z - 1;
        gx = gx < 0 ? 0 : (gx >= g.nx ? g.nx - 1 : gx);
        gy = gy < 0 ? 0 : (gy >= g.ny ? g.ny - 1 : gy);
        gz = gz < 0 ? 0 : (gz >= g.nz ? g.nz - 1 : gz);
        const double v = log(perm[(size_t)gx + (size_t)g.nx * ((size_t)gy + (size_t)g.ny * gz)]);
        sv[t] = v;
        s1 += v;
    }
    const double mu = block_sum(s1, sred) / kCnnIn;
    double s2 = 0.0;
    for (int t = threadIdx.x; t < kCnnIn; t += blockDim.x) s2 += (sv[t] - mu) * (sv[t] - mu);
    const double inv = 1.0 / sqrt(block_sum(s2, sred) / kCnnIn + 1e-6);
    for (int t = threadIdx.x; t < kCnnIn; t += blockDim.x)
        out[(size_t)blockIdx.x * kCnnIn + t] = (float)((sv[t] - mu) * inv);
    if (s_out) {
        for (int c = threadIdx.x; c < 512; c += blockDim.x) {
            const int x = ex * 8 + (c & 7), y = ey * 8 + ((c >> 3) & 7), z = ez * 8 + (c >> 6);
            s_out[(size_t)blockIdx.x * 512 + c] =
                s_scale * perm[(size_t)x + (size_t)g.nx * ((size_t)y + (size_t)g.ny * z)];
        }
    }
}

// ---------------------------------------------------------------------------
// Staging of input channel c of element e into a 10^3 LDS tile.
//   IN = 1: 8^3 input [e][CIN][512], zero halo (padded layers)
//   IN = 2: the network input: channel 0 the patch [e][1000], channel
//           c >= 1 the cosine mode c-1 on the patch grid
template <int IN>
__device__ __forceinline__ float stage_value(const float* xe, int c, int r, const double* c1) {
    const int X = r % 10 - 1, Y = (r / 10) % 10 - 1, Z = r / 100 - 1;
    if (IN == 1) {
        const bool in = X >= 0 && X < 8 && Y >= 0 && Y < 8 && Z >= 0 && Z < 8;
        return in ? xe[(size_t)c * 512 + X + 8 * Y + 64 * Z] : 0.0f;
    }
    return c == 0 ? xe[r] : cnn_mode(c1, c - 1, X, Y, Z);
}

template <int CIN>
struct ConvChunk {
    static constexpr int CH = CIN <= 9 ? CIN : 8;   // channels staged at once
    static_assert(CIN % CH == 0, "channel chunks");
};

// 3x3x3 convolution over one element per workgroup, one output position per
// thread, all COUT outputs in registers.  Input channels are staged in LDS
// (at most nine at a time) as 10^3 tiles.  Wp[(c*27 + t)*(COUT/2) + o/2]
// holds the bf16 pair of outputs (o, o+1), even o in the low half; the
// address is the same in every lane, so the pairs come through scalar loads.
// ACT: 0 none, 1 relu, 2 keep only where mask > 0 (relu derivative),
//      3 add cosine mode o (the network output).
template <int CIN, int COUT, int IN, int ACT>
__global__ __launch_bounds__(512) void k_conv(const float* __restrict__ x, const uint32_t* __restrict__ Wp,
                                              const float* __restrict__ bias, const float* __restrict__ mask,
                                              float* __restrict__ y) {
    static_assert(COUT % 2 == 0, "output channels come in pairs");
    constexpr int CH = ConvChunk<CIN>::CH;
    constexpr int INSZ = IN == 1 ? 512 : kCnnIn;
    constexpr int ESZ = IN == 1 ? CIN * INSZ : kCnnIn;
    __shared__ float tile[CH * kCnnTile];
    __shared__ double c1[10];
    cnn_cos_table(c1);
    const int e = blockIdx.x;
    const int p = threadIdx.x;
    const int base = (p >> 6) * 100 + ((p >> 3) & 7) * 10 + (p & 7);
    float acc[COUT];
#pragma unroll
    for (int o = 0; o < COUT; ++o) acc[o] = bias ? bias[o] : 0.0f;
    const float* xe = x + (size_t)e * ESZ;
#pragma unroll 1
    for (int c0 = 0; c0 < CIN; c0 += CH) {
        __syncthreads();
        for (int t = threadIdx.x; t < CH * kCnnTile; t += blockDim.x)
            tile[t] = stage_value<IN>(xe, c0 + t / kCnnTile, t % kCnnTile, c1);
        __syncthreads();
#pragma unroll 1
        for (int cl = 0; cl < CH; ++cl) {
            const uint32_t* wc = Wp + (size_t)(c0 + cl) * 27 * (COUT / 2);
            const float* tc = tile + cl * kCnnTile + base;
#pragma unroll
            for (int t = 0; t < 27; ++t) {
                const float v = tc[(t / 9) * 100 + ((t / 3) % 3) * 10 + (t % 3)];
#pragma unroll
                for (int o = 0; o < COUT / 2; ++o) {
                    const uint32_t u = wc[t * (COUT / 2) + o];
                    acc[2 * o] += bf_lo(u) * v;
                    acc[2 * o + 1] += bf_hi(u) * v;
                }
            }
        }
    }
#pragma unroll
    for (int o = 0; o < COUT; ++o) {
        const size_t i = ((size_t)e * COUT + o) * 512 + p;
        float v = acc[o];
        if (ACT == 1) v = fmaxf(v, 0.0f);
        if (ACT == 2) v = mask[i] > 0.0f ? v : 0.0f;
        if (ACT == 3) v += cnn_mode(c1, o, p & 7, (p >> 3) & 7, p >> 6);
        y[i] = v;
    }
}

// ---------------------------------------------------------------------------
// The same convolution for the layers with 32 input channels (a dense
// contraction of K = 27 taps x 32 channels per output), on the bf16 matrix
// cores: v_mfma_f32_16x16x32_bf16, D[16 positions][16 outputs] +=
// A[16 positions][32 channels] B[32 channels][16 outputs] per tap.  Lane l
// supplies A row l%16, channels 8(l/16)..+7, and B column l%16, the same
// channels; it receives D rows 4(l/16)..+3 of column l%16.
// Each activation is split into a bf16 high part and the bf16 rounding of
// the remainder, and both pass through the MFMA: with the weights exactly
// bf16 the products keep about 16 significant bits of the float32
// activation (relative error near 2^-17), and every sum is float32.
// One element per workgroup of 8 waves; the element's input is staged in
// LDS as [part][padded position (10^3)][channel], zero halo, and wave w
// owns position tiles 4w..4w+3 (positions 16 tile + row, x fastest).
// mf[t][o][c] (bf16, c fastest, o < COUTP) holds the weights.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int kMfPos = 1000;   // padded positions of the staged element

template <int COUT, int COUTP, int ACT>
__global__ __launch_bounds__(512) void k_conv_mfma(const float* __restrict__ x, const uint16_t* __restrict__ mf,
                                                   const float* __restrict__ bias, float* __restrict__ y) {
    static_assert(COUTP % 16 == 0 && COUT <= COUTP, "output tiles of 16");
    constexpr int NT = COUTP / 16;
    __shared__ uint4 tile[2 * kMfPos * 4];   // [part][position][4 x 8 channels]
    __shared__ double c1[10];
    if (ACT == 3) cnn_cos_table(c1);
    const int e = blockIdx.x;
    for (int i = threadIdx.x; i < 2 * kMfPos * 4; i += blockDim.x) tile[i] = make_uint4(0u, 0u, 0u, 0u);
    __syncthreads();
    {
        const int p = threadIdx.x;   // one interior position per thread
        const int P = ((p >> 6) + 1) * 100 + (((p >> 3) & 7) + 1) * 10 + (p & 7) + 1;
        const float* xe = x + (size_t)e * 32 * 512 + p;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            uint32_t hw[4], lw[4];
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const float v0 = xe[(size_t)(8 * g + 2 * h) * 512], v1 = xe[(size_t)(8 * g + 2 * h + 1) * 512];
                const uint16_t h0 = f2bf(v0), h1 = f2bf(v1);
                const uint16_t l0 = f2bf(v0 - bf2f(h0)), l1 = f2bf(v1 - bf2f(h1));
                hw[h] = (uint32_t)h0 | ((uint32_t)h1 << 16);
                lw[h] = (uint32_t)l0 | ((uint32_t)l1 << 16);
            }
            tile[P * 4 + g] = make_uint4(hw[0], hw[1], hw[2], hw[3]);
            tile[(kMfPos + P) * 4 + g] = make_uint4(lw[0], lw[1], lw[2], lw[3]);
        }
    }
    __syncthreads();
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int r = l & 15, g = l >> 4;
    int base[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int p = 16 * (4 * w + j) + r;
        base[j] = (p >> 6) * 100 + ((p >> 3) & 7) * 10 + (p & 7);
    }
    f32x4_t acc[4][NT];
#pragma unroll
    for (int n = 0; n < NT; ++n) {
        const int o = 16 * n + r;
        const float b0 = (bias && o < COUT) ? bias[o] : 0.0f;
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j][n] = f32x4_t{b0, b0, b0, b0};
    }
#pragma unroll 1
    for (int t = 0; t < 27; ++t) {
        const int off = (t / 9) * 100 + ((t / 3) % 3) * 10 + (t % 3);
        bf16x8_t bw[NT];
#pragma unroll
        for (int n = 0; n < NT; ++n)
            bw[n] = __builtin_bit_cast(bf16x8_t,
                                       *(const uint4*)(mf + ((size_t)(t * COUTP + 16 * n + r) * 32 + 8 * g)));
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int P = base[j] + off;
            const bf16x8_t ah = __builtin_bit_cast(bf16x8_t, tile[P * 4 + g]);
            const bf16x8_t al = __builtin_bit_cast(bf16x8_t, tile[(kMfPos + P) * 4 + g]);
#pragma unroll
            for (int n = 0; n < NT; ++n) {
                acc[j][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bw[n], acc[j][n], 0, 0, 0);
                acc[j][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bw[n], acc[j][n], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int n = 0; n < NT; ++n) {
        const int o = 16 * n + r;
        if (o >= COUT) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int p0 = 16 * (4 * w + j) + 4 * g;
            float v[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                v[i] = acc[j][n][i];
                if (ACT == 1) v[i] = fmaxf(v[i], 0.0f);
                if (ACT == 3) {
                    const int p = p0 + i;
                    v[i] += cnn_mode(c1, o, p & 7, (p >> 3) & 7, p >> 6);
                }
            }
            *(float4*)(y + ((size_t)e * COUT + o) * 512 + p0) = make_float4(v[0], v[1], v[2], v[3]);
        }
    }
}

// The first layer (C1 = 1 + k <= 8 input channels: the patch and the mode
// channels, valid 3x3x3 over the 10^3 patch grid) on the same matrix-core
// tile: K = 32 is 4 taps x 8 channels (channels >= C1 and the 28th tap are
// zero), so the 27 taps take 7 K-steps.  Lane l supplies tap 4 step + l/16.
// The patch is staged as [part][position (10^3)][8 channels] bf16.
// mf1[step][o][tap in step][8 channels] (bf16) holds the weights.
constexpr int kMf1Steps = 7;

template <int C1>
__global__ __launch_bounds__(512) void k_conv1_mfma(const float* __restrict__ x, const uint16_t* __restrict__ mf,
                                                    const float* __restrict__ bias, float* __restrict__ y) {
    static_assert(C1 <= 8, "at most 8 input channels");
    __shared__ uint4 tile[2 * kMfPos];   // [part][position]: 8 channels
    __shared__ double c1[10];
    cnn_cos_table(c1);
    const int e = blockIdx.x;
    const float* xe = x + (size_t)e * kCnnIn;
    for (int P = threadIdx.x; P < kMfPos; P += blockDim.x) {
        const int X = P % 10 - 1, Y = (P / 10) % 10 - 1, Z = P / 100 - 1;
        uint32_t hw[4], lw[4];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            float v[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int c = 2 * h + u;
                v[u] = c == 0 ? xe[P] : (c < C1 ? cnn_mode(c1, c - 1, X, Y, Z) : 0.0f);
            }
            const uint16_t h0 = f2bf(v[0]), h1 = f2bf(v[1]);
            const uint16_t l0 = f2bf(v[0] - bf2f(h0)), l1 = f2bf(v[1] - bf2f(h1));
            hw[h] = (uint32_t)h0 | ((uint32_t)h1 << 16);
            lw[h] = (uint32_t)l0 | ((uint32_t)l1 << 16);
        }
        tile[P] = make_uint4(hw[0], hw[1], hw[2], hw[3]);
        tile[kMfPos + P] = make_uint4(lw[0], lw[1], lw[2], lw[3]);
    }
    __syncthreads();
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int r = l & 15, g = l >> 4;
    int base[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int p = 16 * (4 * w + j) + r;
        base[j] = (p >> 6) * 100 + ((p >> 3) & 7) * 10 + (p & 7);
    }
    f32x4_t acc[4][2];
#pragma unroll
    for (int n = 0; n < 2; ++n) {
        const float b0 = bias[16 * n + r];
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j][n] = f32x4_t{b0, b0, b0, b0};
    }
#pragma unroll 1
    for (int st = 0; st < kMf1Steps; ++st) {
        const int t = 4 * st + g;   // this lane's tap (t = 27: zero weights)
        const int off = t < 27 ? (t / 9) * 100 + ((t / 3) % 3) * 10 + (t % 3) : 0;
        bf16x8_t bw[2];
#pragma unroll
        for (int n = 0; n < 2; ++n)
            bw[n] = __builtin_bit_cast(bf16x8_t,
                                       *(const uint4*)(mf + ((size_t)(st * 32 + 16 * n + r) * 4 + g) * 8));
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int P = base[j] + off;
            const bf16x8_t ah = __builtin_bit_cast(bf16x8_t, tile[P]);
            const bf16x8_t al = __builtin_bit_cast(bf16x8_t, tile[kMfPos + P]);
#pragma unroll
            for (int n = 0; n < 2; ++n) {
                acc[j][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bw[n], acc[j][n], 0, 0, 0);
                acc[j][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bw[n], acc[j][n], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int n = 0; n < 2; ++n) {
        const int o = 16 * n + r;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int p0 = 16 * (4 * w + j) + 4 * g;
            *(float4*)(y + ((size_t)e * 32 + o) * 512 + p0) =
                make_float4(fmaxf(acc[j][n][0], 0.0f), fmaxf(acc[j][n][1], 0.0f), fmaxf(acc[j][n][2], 0.0f),
                            fmaxf(acc[j][n][3], 0.0f));
        }
    }
}

// ---------------------------------------------------------------------------
// Weight gradients: part[b][(o*CIN + c)*27 + t] = sum over the elements of
// block column b of sum_p gy[e][o][p] x[e][c][p + t] (padded coordinates),
// and part[b][COUT*CIN*27 + o] = sum_p gy[e][o][p].  Thread = (c, o) pair of
// a channel slice (blockIdx.y), 27 tap accumulators in registers; the
// slice's input and all of gy are staged in LDS per element.  blockDim.x
// covers the slice's (c, o) pairs (at most 320).
template <int CIN, int COUT, int IN>
__global__ __launch_bounds__(320) void k_conv_wgrad(const float* __restrict__ x, const float* __restrict__ gy,
                                                    int count, int per_block, float* __restrict__ part,
                                                    int pstride) {
    constexpr int CH = ConvChunk<CIN>::CH;
    constexpr int INSZ = IN == 1 ? 512 : kCnnIn;
    constexpr int ESZ = IN == 1 ? CIN * INSZ : kCnnIn;
    static_assert(CH * COUT <= 320, "one thread per (c, o) pair");
    constexpr int GLD = 513;   // odd row pitch: lanes with different o hit different banks
    __shared__ float tile[CH * kCnnTile];
    __shared__ float sg[COUT * GLD];
    __shared__ double c1[10];
    cnn_cos_table(c1);
    const int c0 = blockIdx.y * CH;
    const int q = threadIdx.x;
    const bool act = q < CH * COUT;
    const int cl = act ? q / COUT : 0, o = act ? q % COUT : 0;
    float acc[27];
#pragma unroll
    for (int t = 0; t < 27; ++t) acc[t] = 0.0f;
    float accb = 0.0f;
    const int e_beg = blockIdx.x * per_block;
    const int e_end = min(count, e_beg + per_block);
#pragma unroll 1
    for (int e = e_beg; e < e_end; ++e) {
        __syncthreads();
        const float* xe = x + (size_t)e * ESZ;
        for (int t = threadIdx.x; t < CH * kCnnTile; t += blockDim.x)
            tile[t] = stage_value<IN>(xe, c0 + t / kCnnTile, t % kCnnTile, c1);
        const float* ge = gy + (size_t)e * COUT * 512;
        for (int t = threadIdx.x; t < COUT * 512; t += blockDim.x) sg[(t >> 9) * GLD + (t & 511)] = ge[t];
        __syncthreads();
        if (act) {
            const float* tc = tile + cl * kCnnTile;
            const float* gr = sg + o * GLD;
#pragma unroll 1
            for (int zy = 0; zy < 64; ++zy) {
                const int z = zy >> 3, yy = zy & 7;
                float gv[8];
#pragma unroll
                for (int px = 0; px < 8; ++px) {
                    gv[px] = gr[zy * 8 + px];
                    accb += gv[px];
                }
#pragma unroll
                for (int dz = 0; dz < 3; ++dz) {
#pragma unroll
                    for (int dy = 0; dy < 3; ++dy) {
                        float row[10];
                        const float* rp = tc + (z + dz) * 100 + (yy + dy) * 10;
#pragma unroll
                        for (int i = 0; i < 10; ++i) row[i] = rp[i];
#pragma unroll
                        for (int dx = 0; dx < 3; ++dx) {
                            float s = 0.0f;
#pragma unroll
                            for (int px = 0; px < 8; ++px) s += gv[px] * row[px + dx];
                            acc[dz * 9 + dy * 3 + dx] += s;
                        }
                    }
                }
            }
        }
    }
    if (act) {
        float* pb = part + (size_t)blockIdx.x * pstride;
#pragma unroll
        for (int t = 0; t < 27; ++t) pb[((size_t)o * CIN + c0 + cl) * 27 + t] = acc[t];
        if (c0 + cl == 0) pb[(size_t)COUT * CIN * 27 + o] = accb;
    }
}

// grad[i] = sum_b part[b][src(i)] for the layer's k-row weights and biases
// (rows o >= k of a padded layer are dropped); fixed summation order.
__global__ void k_cnn_reduce(const float* __restrict__ part, int nblk, int pstride, int nw, int bias_src, int nb,
                             float* __restrict__ grad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nw + nb) return;
    const int src = i < nw ? i : bias_src + (i - nw);
    float s = 0.0f;
    for (int b = 0; b < nblk; ++b) s += part[(size_t)b * pstride + src];
    grad[i] = s;
}

// ---------------------------------------------------------------------------
// Subspace loss and its gradient w.r.t. X, one element per workgroup, one
// cell per thread; the small k x k systems in float64.
template <int KP>
__global__ __launch_bounds__(512) void k_cnn_loss(const float* __restrict__ X, const double* __restrict__ phi,
                                                  int ldphi, const double* __restrict__ s, int k, double inv_m,
                                                  double* __restrict__ loss_part, float* __restrict__ gX) {
    __shared__ double red[8][2 * KP * KP];
    __shared__ double sG[KP * KP], sB[KP * KP], sC[KP * KP];
    __shared__ double sred[8];
    const int e = blockIdx.x, c = threadIdx.x;
    const int lane = c & 63, w = c >> 6;
    const double sc = s[(size_t)e * 512 + c];
    const double mean_s = block_sum(sc, sred) / 512.0;
    const double sb = sc / mean_s, root = sqrt(mean_s);
    double xv[KP], pv[KP];
#pragma unroll
    for (int o = 0; o < KP; ++o) {
        xv[o] = o < k ? (double)X[((size_t)e * KP + o) * 512 + c] : 0.0;
        pv[o] = o < k ? phi[((size_t)e * ldphi + o) * 512 + c] * root : 0.0;
    }
#pragma unroll
    for (int o = 0; o < KP; ++o) {
#pragma unroll
        for (int q = 0; q < KP; ++q) {
            const double gv = wave_sum(sb * xv[o] * xv[q]);
            const double bv = wave_sum(sb * xv[o] * pv[q]);
            if (lane == 0) {
                red[w][o * KP + q] = gv;
                red[w][KP * KP + o * KP + q] = bv;
            }
        }
    }
    __syncthreads();
    if (c < 2 * KP * KP) {
        double t = 0.0;
        for (int ww = 0; ww < 8; ++ww) t += red[ww][c];
        if (c < KP * KP) sG[c] = t;
        else sB[c - KP * KP] = t;
    }
    __syncthreads();
    if (c == 0) {
        // C = G^-1 B by Cholesky of G (k x k), a tiny ridge keeps it definite
        double Lm[KP * KP];
        double tr = 0.0;
        for (int i = 0; i < k; ++i) tr += sG[i * KP + i];
        const double ridge = 1e-12 * tr / k + 1e-300;
        for (int i = 0; i < KP * KP; ++i) Lm[i] = 0.0;
        for (int j = 0; j < k; ++j) {
            double d = sG[j * KP + j] + ridge;
            for (int l = 0; l < j; ++l) d -= Lm[j * KP + l] * Lm[j * KP + l];
            d = sqrt(fmax(d, 1e-300));
            Lm[j * KP + j] = d;
            for (int i = j + 1; i < k; ++i) {
                double v = sG[i * KP + j];
                for (int l = 0; l < j; ++l) v -= Lm[i * KP + l] * Lm[j * KP + l];
                Lm[i * KP + j] = v / d;
            }
        }
        for (int col = 0; col < KP; ++col) {
            double yv[KP];
            for (int i = 0; i < k; ++i) {
                double v = sB[i * KP + col];
                for (int l = 0; l < i; ++l) v -= Lm[i * KP + l] * yv[l];
                yv[i] = v / Lm[i * KP + i];
            }
            for (int i = k - 1; i >= 0; --i) {
                double v = yv[i];
                for (int l = i + 1; l < k; ++l) v -= Lm[l * KP + i] * sC[l * KP + col];
                sC[i * KP + col] = v / Lm[i * KP + i];
            }
            for (int i = k; i < KP; ++i) sC[i * KP + col] = 0.0;
        }
    }
    __syncthreads();
    double r[KP];
    double l2 = 0.0;
#pragma unroll
    for (int j = 0; j < KP; ++j) {
        double v = pv[j];
#pragma unroll
        for (int o = 0; o < KP; ++o) v -= xv[o] * sC[o * KP + j];
        r[j] = j < k ? v : 0.0;
        l2 += sb * r[j] * r[j];
    }
#pragma unroll
    for (int o = 0; o < KP; ++o) {
        double gsum = 0.0;
#pragma unroll
        for (int j = 0; j < KP; ++j) gsum += sC[o * KP + j] * r[j];
        gX[((size_t)e * KP + o) * 512 + c] = o < k ? (float)(-2.0 * inv_m * sb * gsum) : 0.0f;
    }
    const double loss = block_sum(l2, sred);
    if (c == 0) loss_part[e] = loss * inv_m;
}

// ---------------------------------------------------------------------------
// Parameter packing for the convolution kernels.  Values come from the bf16
// vector or, rounded to bf16, from the float32 master vector.
//   fwd1[c][t][16], fwd2[c][t][16], fwd3[c][t][KP/2]       (pairs of outputs)
//   bwd2[o][t][16], bwd3[o][t][16] with flipped taps       (pairs of inputs)
//   mf2[t][32][32], mf3[t][16][32]: bf16 [tap][output][input] for the
//   matrix-core kernel (outputs of layer 3 beyond k are zero), 16-byte aligned;
//   mf1[step][32][4][8]: layer 1 as K-steps of 4 taps x 8 channels (zero
//   beyond C1 channels and beyond tap 26)
struct CnnPacks {
    uint32_t* fwd1;
    uint32_t* fwd2;
    uint32_t* fwd3;
    uint32_t* bwd2;
    uint32_t* bwd3;
    float* b1;
    float* b2;
    float* b3;
    uint16_t* mf2;
    uint16_t* mf3;
    uint16_t* mf1;
};

__device__ __forceinline__ float cnn_param(const float* t32, const uint16_t* t16, size_t i) {
    return t16 ? bf2f(t16[i]) : bf2f(f2bf(t32[i]));
}

__global__ void k_cnn_pack(const float* __restrict__ t32, const uint16_t* __restrict__ t16, int k, int kp,
                           CnnPacks pk) {
    const int c1 = 1 + k;   // input channels of layer 1
    const size_t oW1 = 0, ob1 = (size_t)32 * c1 * 27, oW2 = ob1 + 32, ob2 = oW2 + 32 * 32 * 27, oW3 = ob2 + 32,
                 ob3 = oW3 + (size_t)k * 32 * 27;
    auto W1 = [&](int o, int c, int t) { return cnn_param(t32, t16, oW1 + ((size_t)o * c1 + c) * 27 + t); };
    auto W2 = [&](int o, int c, int t) { return cnn_param(t32, t16, oW2 + ((size_t)o * 32 + c) * 27 + t); };
    auto W3 = [&](int o, int c, int t) {
        return o < k ? cnn_param(t32, t16, oW3 + ((size_t)o * 32 + c) * 27 + t) : 0.0f;
    };
    auto pack = [](float lo, float hi) {
        return (uint32_t)f2bf(lo) | ((uint32_t)f2bf(hi) << 16);
    };
    const int n1 = c1 * 27 * 16, n2 = 32 * 27 * 16, n3 = 32 * 27 * (kp / 2), nb2 = 32 * 27 * 16,
              nb3 = kp * 27 * 16;
    const int total = n1 + n2 + n3 + nb2 + nb3 + 32 + 32 + kp;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        int j = i;
        if (j < n1) {
            const int c = j / (27 * 16), t = (j / 16) % 27, op = j % 16;
            pk.fwd1[j] = pack(W1(2 * op, c, t), W1(2 * op + 1, c, t));
            continue;
        }
        j -= n1;
        if (j < n2) {
            const int c = j / (27 * 16), t = (j / 16) % 27, op = j % 16;
            pk.fwd2[j] = pack(W2(2 * op, c, t), W2(2 * op + 1, c, t));
            continue;
        }
        j -= n2;
        if (j < n3) {
            const int h = kp / 2;
            const int c = j / (27 * h), t = (j / h) % 27, op = j % h;
            pk.fwd3[j] = pack(W3(2 * op, c, t), W3(2 * op + 1, c, t));
            continue;
        }
        j -= n3;
        if (j < nb2) {
            // transposed layer 2: inputs o (32), outputs c (pairs), taps flipped
            const int o = j / (27 * 16), t = (j / 16) % 27, cp = j % 16;
            pk.bwd2[j] = pack(W2(o, 2 * cp, 26 - t), W2(o, 2 * cp + 1, 26 - t));
            continue;
        }
        j -= nb2;
        if (j < nb3) {
            const int o = j / (27 * 16), t = (j / 16) % 27, cp = j % 16;
            pk.bwd3[j] = pack(W3(o, 2 * cp, 26 - t), W3(o, 2 * cp + 1, 26 - t));
            continue;
        }
        j -= nb3;
        if (j < 32) {
            pk.b1[j] = cnn_param(t32, t16, ob1 + j);
            continue;
        }
        j -= 32;
        if (j < 32) {
            pk.b2[j] = cnn_param(t32, t16, ob2 + j);
            continue;
        }
        j -= 32;
        pk.b3[j] = j < k ? cnn_param(t32, t16, ob3 + j) : 0.0f;
    }
}

__global__ void k_cnn_pack_mf(const float* __restrict__ t32, const uint16_t* __restrict__ t16, int k,
                              CnnPacks pk) {
    const int c1 = 1 + k;
    const size_t oW2 = (size_t)32 * c1 * 27 + 32, oW3 = oW2 + 32 * 32 * 27 + 32;
    const int n2 = 27 * 32 * 32, n3 = 27 * 16 * 32, n1 = kMf1Steps * 32 * 4 * 8;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n2 + n3 + n1; i += gridDim.x * blockDim.x) {
        if (i >= n2 + n3) {
            const int j = i - n2 - n3, st = j / 1024, o = (j / 32) % 32, gg = (j / 8) % 4, c = j % 8;
            const int t = 4 * st + gg;
            pk.mf1[j] = (t < 27 && c < c1) ? f2bf(cnn_param(t32, t16, ((size_t)o * c1 + c) * 27 + t)) : (uint16_t)0;
        } else if (i < n2) {
            const int t = i / 1024, o = (i / 32) % 32, c = i % 32;
            pk.mf2[i] = f2bf(cnn_param(t32, t16, oW2 + ((size_t)o * 32 + c) * 27 + t));
        } else {
            const int j = i - n2, t = j / 512, o = (j / 32) % 16, c = j % 32;
            pk.mf3[j] = o < k ? f2bf(cnn_param(t32, t16, oW3 + ((size_t)o * 32 + c) * 27 + t)) : (uint16_t)0;
        }
    }
}

// Adam on the float32 master parameters; the bf16 copy used by inference
// is refreshed in the same pass.
__global__ void k_cnn_adam(float* __restrict__ theta, const float* __restrict__ grad, float* __restrict__ m1,
                           float* __restrict__ m2, int64_t n, float lr, float b1, float b2, float eps, float c1,
                           float c2, uint16_t* __restrict__ theta16) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float g = grad[i];
        const float a = b1 * m1[i] + (1.0f - b1) * g;
        const float b = b2 * m2[i] + (1.0f - b2) * g * g;
        m1[i] = a;
        m2[i] = b;
        const float v = theta[i] - lr * (a * c1) / (sqrtf(b * c2) + eps);
        theta[i] = v;
        if (theta16) theta16[i] = f2bf(v);
    }
}

// ---------------------------------------------------------------------------
// launchers

int64_t cnn_param_count(int k) {
    return (int64_t)32 * (1 + k) * 27 + 32 + 32 * 32 * 27 + 32 + (int64_t)k * 32 * 27 + k;
}

// 32-bit words of the packs before the matrix-core copies, rounded up to 16 bytes
static size_t cnn_pack_words_vec(int kp) {
    const size_t w = (size_t)(1 + kp) * 27 * 16 + 32 * 27 * 16 + 32 * 27 * (kp / 2) + 32 * 27 * 16 +
                     (size_t)kp * 27 * 16 + 32 + 32 + kp;
    return (w + 3) & ~(size_t)3;
}

size_t cnn_pack_words(int kp) {
    return cnn_pack_words_vec(kp) + (27 * 32 * 32 + 27 * 16 * 32 + kMf1Steps * 32 * 4 * 8) / 2;
}

CnnPacks cnn_pack_view(void* base, int kp) {
    CnnPacks p;
    uint32_t* u = (uint32_t*)base;
    p.fwd1 = u;
    p.fwd2 = p.fwd1 + (1 + kp) * 27 * 16;
    p.fwd3 = p.fwd2 + 32 * 27 * 16;
    p.bwd2 = p.fwd3 + 32 * 27 * (kp / 2);
    p.bwd3 = p.bwd2 + 32 * 27 * 16;
    p.b1 = (float*)(p.bwd3 + (size_t)kp * 27 * 16);
    p.b2 = p.b1 + 32;
    p.b3 = p.b2 + 32;
    p.mf2 = (uint16_t*)(u + cnn_pack_words_vec(kp));
    p.mf3 = p.mf2 + 27 * 32 * 32;
    p.mf1 = p.mf3 + 27 * 16 * 32;
    return p;
}

void launch_cnn_patches(const FineGeom& g, const double* perm, int e0, int count, double s_scale, float* out,
                        double* s_out, hipStream_t s) {
    hipLaunchKernelGGL(k_cnn_patches, dim3(count), dim3(256), 0, s, g, perm, e0, s_scale, out, s_out);
}

void launch_cnn_pack(const float* t32, const uint16_t* t16, int k, int kp, void* packs, hipStream_t s) {
    hipLaunchKernelGGL(k_cnn_pack, dim3(64), dim3(256), 0, s, t32, t16, k, kp, cnn_pack_view(packs, kp));
    hipLaunchKernelGGL(k_cnn_pack_mf, dim3(64), dim3(256), 0, s, t32, t16, k, cnn_pack_view(packs, kp));
}

#define SPECMG_KP_DISPATCH(KPV, ...)                                          \
    switch (KPV) {                                                            \
        case 2: { constexpr int KP = 2, C1 = 3; __VA_ARGS__; } break;         \
        case 4: { constexpr int KP = 4, C1 = 5; __VA_ARGS__; } break;         \
        case 6: { constexpr int KP = 6, C1 = 7; __VA_ARGS__; } break;         \
        default: { constexpr int KP = 8, C1 = 9; __VA_ARGS__; } break;        \
    }

// X = network(patches) for `count` elements; a1, a2 receive the hidden
// activations (kept for the backward pass)
void launch_cnn_forward(const void* packs, int kp, const float* patches, int count, float* a1, float* a2, float* X,
                        hipStream_t s) {
    const CnnPacks p = cnn_pack_view(const_cast<void*>(packs), kp);
    if (kp <= 6) {
        SPECMG_KP_DISPATCH(kp, hipLaunchKernelGGL((k_conv1_mfma<(C1 <= 8 ? C1 : 8)>), dim3(count), dim3(512), 0, s,
                                                  patches, p.mf1, p.b1, a1));
    } else {
        SPECMG_KP_DISPATCH(kp, hipLaunchKernelGGL((k_conv<C1, 32, 2, 1>), dim3(count), dim3(512), 0, s, patches,
                                                  p.fwd1, p.b1, nullptr, a1));
    }
    hipLaunchKernelGGL((k_conv_mfma<32, 32, 1>), dim3(count), dim3(512), 0, s, a1, p.mf2, p.b2, a2);
    SPECMG_KP_DISPATCH(kp, hipLaunchKernelGGL((k_conv_mfma<KP, 16, 3>), dim3(count), dim3(512), 0, s, a2, p.mf3,
                                              p.b3, X));
}

void launch_cnn_loss(const float* X, const double* phi, int ldphi, const double* sdiag, int k, int kp, int count,
                     double inv_m, double* loss_part, float* gX, hipStream_t s) {
    SPECMG_KP_DISPATCH(kp, hipLaunchKernelGGL((k_cnn_loss<KP>), dim3(count), dim3(512), 0, s, X, phi, ldphi,
                                              sdiag, k, inv_m, loss_part, gX));
}

// parameter gradient (flat, float32) from dL/dX; g2, g1: scratch of the
// activation size; part: scratch of nblk * (32*32*27 + 32) floats
void launch_cnn_backward(const void* packs, int k, int kp, const float* patches, const float* a1, const float* a2,
                         const float* gX, int count, float* g2, float* g1, float* part, int nblk, float* grad,
                         hipStream_t s) {
    const CnnPacks p = cnn_pack_view(const_cast<void*>(packs), kp);
    const int per = (count + nblk - 1) / nblk;
    const int nb = (count + per - 1) / per;
    const int64_t oW2 = (int64_t)32 * (1 + k) * 27 + 32, oW3 = oW2 + 32 * 32 * 27 + 32;
    // layer 3: weight gradient, then data gradient through the relu of a2
    {
        const int pstride = kp * 32 * 27 + kp;
        SPECMG_KP_DISPATCH(kp, hipLaunchKernelGGL((k_conv_wgrad<32, KP, 1>), dim3(nb, 4), dim3(64), 0, s, a2, gX,
                                                  count, per, part, pstride));
        const int nw = k * 32 * 27;
        hipLaunchKernelGGL(k_cnn_reduce, dim3((nw + k + 255) / 256), dim3(256), 0, s, part, nb, pstride, nw,
                           kp * 32 * 27, k, grad + oW3);
        SPECMG_KP_DISPATCH(kp, hipLaunchKernelGGL((k_conv<KP, 32, 1, 2>), dim3(count), dim3(512), 0, s, gX, p.bwd3,
                                                  nullptr, a2, g2));
    }
    // layer 2
    {
        const int pstride = 32 * 32 * 27 + 32;
        hipLaunchKernelGGL((k_conv_wgrad<32, 32, 1>), dim3(nb, 4), dim3(256), 0, s, a1, g2, count, per, part,
                           pstride);
        const int nw = 32 * 32 * 27;
        hipLaunchKernelGGL(k_cnn_reduce, dim3((nw + 32 + 255) / 256), dim3(256), 0, s, part, nb, pstride, nw, nw,
                           32, grad + oW2);
        hipLaunchKernelGGL((k_conv<32, 32, 1, 2>), dim3(count), dim3(512), 0, s, g2, p.bwd2, nullptr, a1, g1);
    }
    // layer 1 (the network input needs no gradient)
    {
        const int c1 = 1 + k;
        const int pstride = 32 * c1 * 27 + 32;
        const int threads = (c1 * 32 + 63) / 64 * 64;
        SPECMG_KP_DISPATCH(kp, hipLaunchKernelGGL((k_conv_wgrad<C1, 32, 2>), dim3(nb, 1), dim3(threads), 0, s,
                                                  patches, g1, count, per, part, pstride));
        const int nw = 32 * c1 * 27;
        hipLaunchKernelGGL(k_cnn_reduce, dim3((nw + 32 + 255) / 256), dim3(256), 0, s, part, nb, pstride, nw, nw,
                           32, grad);
    }
}

void launch_cnn_adam(float* theta, const float* grad, float* m1, float* m2, int64_t n, float lr, float b1, float b2,
                     float eps, float c1, float c2, uint16_t* theta16, hipStream_t s) {
    hipLaunchKernelGGL(k_cnn_adam, dim3(64), dim3(256), 0, s, theta, grad, m1, m2, n, lr, b1, b2, eps, c1, c2,
                       theta16);
}

}  // namespace specmg
