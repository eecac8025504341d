// Learned palm-pose proposer on gfx950: a PointNet-style encoder and a
// mixture-density head evaluated with BF16 MFMA (FP32 accumulation), its
// training step (mixture NLL, backward, Adam on FP32 master weights) and a
// Philox sampler of palm poses with a uniform fallback.
//
// The paper names data-driven search as a way to skip unproductive regions
// (Sec. 5.7) and leaves it unimplemented.  This network is the project's own
// configuration: a shared per-point MLP 6 -> 128 -> 256 (ReLU) and a max-pool
// over the points (PointNet, Qi et al. 2017); a head 256 -> 256 -> 256 (ReLU)
// -> 152 = 8 components x (logit, 9 means, 9 log-sigmas) of a diagonal
// Gaussian mixture over y = (first two columns of R, t / 0.1 m), mapped back to
// SO(3) by Gram-Schmidt (the 6-D representation of Zhou et al. 2019).
//
// Work decomposition:
//  * k_encode: 2048 points of one object per workgroup of 8 waves; W2 (BF16,
//    68 KiB) is staged in LDS once, then every wave runs its own 64-point
//    steps without a barrier.  Layer 1 is computed transposed (one 32x32x16
//    MFMA per 32 channels, K = 6 padded to 16, the bias as the accumulator),
//    so a lane holds 4-channel groups of one point; a lane-half swap
//    (v_permlane32_swap) turns them into layer 2's A operand in registers.
//    Layer 2 is 8 x 8 MFMAs per 32 points; the max-pool keeps, per lane and
//    channel, the largest pre-activation and its lowest point (a max tree,
//    then a first-match scan); the pairs are merged across the lane halves,
//    the waves (LDS) and the workgroups (64-bit atomicMax of ordered value
//    bits above the inverted point index); bias and ReLU are applied to the
//    pooled maximum.
//  * the head and every backward product are small GEMMs (rows = objects)
//    run by k_gemm, one wave per 32x32 output tile;
//  * the encoder backward is sparse: the max-pool routes each channel's
//    gradient to one point, so only B x 256 point rows are revisited (FP32).

#include <type_traits>

#include "lg_internal.h"

namespace lg {
namespace prop {

constexpr int kIn = 6, kInPad = 16, kH1 = 128, kH2 = 256, kHH = 256, kM = 8, kY = 9;
constexpr int kOut = kM * (1 + 2 * kY);  // 152
constexpr float kInvSP = 10.0f;          // 1 / 0.1 m: input point scale
constexpr float kST = 0.1f;              // m: translation scale of y
constexpr float kLsMin = -5.0f, kLsMax = 2.0f;
constexpr uint32_t kPurposeSample = 7u;  // third Philox counter word of the sampler
constexpr uint32_t kPurposeInit = 9u;    // ... of the weight initialisation

// flat FP32 parameter layout: per layer W [in][out] row-major, then b [out]
constexpr int64_t kW1 = 0, kB1 = kW1 + kIn * kH1;
constexpr int64_t kW2 = kB1 + kH1, kB2 = kW2 + kH1 * kH2;
constexpr int64_t kWa = kB2 + kH2, kBa = kWa + kH2 * kHH;
constexpr int64_t kWb = kBa + kHH, kBb = kWb + kHH * kHH;
constexpr int64_t kWc = kBb + kHH, kBc = kWc + kHH * kOut;
constexpr int64_t kNParams = kBc + kOut;
// BF16 weight copies, transposed to [out][in_pad] so that an MFMA B operand
// (8 consecutive k of one output column) is one 16-byte load
constexpr int64_t kT1 = 0, kT2 = kT1 + kH1 * kInPad, kTa = kT2 + kH2 * kH1;
constexpr int64_t kTb = kTa + kHH * kH2, kTc = kTb + kHH * kHH, kNT = kTc + kOut * kHH;

struct LayerDesc {
    int in, out, in_pad;
    int64_t w, b, t;
    float init_gain;
};
__host__ __device__ inline LayerDesc layer(int l)
{
    switch (l) {
    case 0: return {kIn, kH1, kInPad, kW1, kB1, kT1, 1.0f};
    case 1: return {kH1, kH2, kH1, kW2, kB2, kT2, 1.0f};
    case 2: return {kH2, kHH, kH2, kWa, kBa, kTa, 1.0f};
    case 3: return {kHH, kHH, kHH, kWb, kBb, kTb, 1.0f};
    default: return {kHH, kOut, kHH, kWc, kBc, kTc, 0.1f};
    }
}

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

// float -> bfloat16 bits, round to nearest even (inputs are finite)
__device__ inline uint16_t bf16_bits(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline uint16_t bf16_bits(uint16_t h) { return h; }
__device__ inline float bf16_val(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline f32x16_t mfma(const u16x8_t &a, const u16x8_t &b, const f32x16_t &c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                   __builtin_bit_cast(bf16x8_t, b), c, 0, 0, 0);
}
// 32x32 accumulator layout: register i of lane l holds row c_row(i, l), column l % 32
__device__ inline int c_row(int i, int lane) { return 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3); }

// ---- parameters --------------------------------------------------------------
__global__ void k_init(float *__restrict__ P, uint32_t s_lo, uint32_t s_hi)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= kNParams) return;
    for (int l = 0; l < 5; ++l) {
        const LayerDesc L = layer(l);
        if (idx >= L.w && idx < L.b) {
            uint32_t w[4];
            philox4x32_10((uint32_t)idx, 0u, kPurposeInit, 0u, s_lo, s_hi, w);
            const float a = L.init_gain * sqrtf(6.0f / (float)L.in);  // He-uniform
            P[idx] = (2.0f * u01f(w[0]) - 1.0f) * a;
            return;
        }
        if (idx >= L.b && idx < L.b + L.out) {
            P[idx] = 0.0f;
            return;
        }
    }
}

__global__ void k_refresh_bf16(const float *__restrict__ P, uint16_t *__restrict__ T)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= kNT) return;
    for (int l = 0; l < 5; ++l) {
        const LayerDesc L = layer(l);
        const int64_t n = (int64_t)L.out * L.in_pad;
        if (idx >= L.t && idx < L.t + n) {
            const int o = (int)((idx - L.t) / L.in_pad), i = (int)((idx - L.t) % L.in_pad);
            T[idx] = i < L.in ? bf16_bits(P[L.w + (int64_t)i * L.out + o]) : (uint16_t)0;
            return;
        }
    }
}

__global__ void k_adam(float *__restrict__ P, const float *__restrict__ G, float *__restrict__ Mo,
                       float *__restrict__ Vo, float lr_t, float b1, float b2, float eps)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kNParams) return;
    const float g = G[i];
    const float m = b1 * Mo[i] + (1.0f - b1) * g;
    const float v = b2 * Vo[i] + (1.0f - b2) * g * g;
    Mo[i] = m;
    Vo[i] = v;
    P[i] -= lr_t * m / (sqrtf(v) + eps);
}

__global__ void k_fill_u64(unsigned long long *__restrict__ p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// ---- encoder -----------------------------------------------------------------
constexpr int kEncWaves = 8;
constexpr int kEncThreads = 64 * kEncWaves;
constexpr int kEncPair = 64;                         // points a wave takes per step: two 32-row blocks
constexpr int kEncChunk = kEncPair * kEncWaves * 4;  // points per workgroup (4 steps per wave)
constexpr int kLd = kH1 + 8;                                   // padded LDS row of W2^T (BF16 elements)
static_assert(kEncThreads >= kH2, "the pooled-key merge takes one thread per channel");
static_assert(kEncWaves * kH2 * 8 <= kH2 * kLd * 2, "the pooled-key merge reuses the W2 buffer");

typedef short s16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

__device__ inline u16x8_t input_row(const float *__restrict__ xp)
{
    u16x8_t a = {0, 0, 0, 0, 0, 0, 0, 0};
    a[0] = bf16_bits(xp[0] * kInvSP);
    a[1] = bf16_bits(xp[1] * kInvSP);
    a[2] = bf16_bits(xp[2] * kInvSP);
    a[3] = bf16_bits(xp[3]);
    a[4] = bf16_bits(xp[4]);
    a[5] = bf16_bits(xp[5]);
    return a;
}

// (bf16(relu(a)), bf16(relu(b))) packed low/high.  Round to nearest even, then
// a signed 16-bit max with 0: a negative BF16 (and -0) has its sign bit set.
__device__ inline uint32_t relu_pk_bf16(float a, float b)
{
    const f32x2_t v = {a, b};
    const s16x2_t h = __builtin_bit_cast(s16x2_t, __builtin_convertvector(v, bf16x2_t));
    const s16x2_t z = {0, 0};
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(h, z));
}

// FP32 -> unsigned with the same order (sign-magnitude flipped); 0 never
// comes out of a finite value, so a zero key means "no point"
__device__ inline uint32_t ord_bits(float v)
{
    const uint32_t u = __float_as_uint(v);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float ord_val(uint32_t o) { return __uint_as_float((o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o); }

// Fold one 32-row block of a layer-2 column block into the lane's running
// (max, point) pair: rows ascend with the register index, so the first
// register equal to the maximum is the lowest point.
__device__ inline void fold_rows(f32x16_t a, int row0, int end, int half, float &best, int &bidx)
{
    if (row0 + 32 > end) {  // wave-uniform: the object's last rows
#pragma unroll
        for (int i = 0; i < 16; ++i)
            if (row0 + 8 * (i >> 2) + 4 * half + (i & 3) >= end) a[i] = -INFINITY;
    }
    float m = a[0];
#pragma unroll
    for (int i = 1; i < 16; ++i) m = fmaxf(m, a[i]);
    int ii = 8 * 3 + 3;
#pragma unroll
    for (int i = 14; i >= 0; --i) ii = a[i] == m ? 8 * (i >> 2) + (i & 3) : ii;
    if (m > best) {
        best = m;
        bidx = row0 + 4 * half + ii;
    }
}

// grid (ceil(Np / kEncChunk), B), kEncThreads threads.  Each wave runs its
// own 64-point steps with no barrier: layer 1 is computed transposed
// (channels x points), so a lane ends up holding 4-channel groups of one
// point; one lane-half swap per dword turns them into the layer-2 A operand
// (8 consecutive channels of one point) without going through LDS.
// Registers, not LDS, set the occupancy: the H1 of two row blocks, two
// accumulators and the running pairs take 174 VGPRs, two waves per SIMD.
__global__ __launch_bounds__(kEncThreads) __attribute__((amdgpu_waves_per_eu(2))) void
k_encode(const float *__restrict__ x, int Np, const uint16_t *__restrict__ T, const float *__restrict__ P,
         unsigned long long *__restrict__ keys)
{
    __shared__ __attribute__((aligned(16))) uint16_t sW2[kH2 * kLd];
    __shared__ __attribute__((aligned(16))) float sB1[kH1];
    const int b = blockIdx.y, tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int r = lane & 31, half = lane >> 5;
    for (int i = tid; i < kH2 * (kH1 / 8); i += kEncThreads) {
        const int n = i / (kH1 / 8), k8 = i % (kH1 / 8);
        *(u16x8_t *)&sW2[n * kLd + 8 * k8] = *(const u16x8_t *)&T[kT2 + (int64_t)n * kH1 + 8 * k8];
    }
    for (int i = tid; i < kH1; i += kEncThreads) sB1[i] = P[kB1 + i];
    __syncthreads();

    float best[kH2 / 32];
    int bidx[kH2 / 32];
#pragma unroll
    for (int c = 0; c < kH2 / 32; ++c) {
        best[c] = -INFINITY;
        bidx[c] = 0;
    }
    const int c0 = blockIdx.x * kEncChunk, c1 = min(Np, c0 + kEncChunk);
    for (int p0 = c0 + wave * kEncPair; p0 < c1; p0 += kEncWaves * kEncPair) {
        u16x8_t h[2][kH1 / 16];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int pt = p0 + 32 * j + r;
            u16x8_t xb = {0, 0, 0, 0, 0, 0, 0, 0};
            if (half == 0 && pt < c1) xb = input_row(x + ((int64_t)b * Np + pt) * kIn);
#pragma unroll
            for (int cb = 0; cb < kH1 / 32; ++cb) {
                // D[channel][point] = b1 + W1^T x: the bias enters as the accumulator
                f32x16_t acc;
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const f32x4_t bb = *(const f32x4_t *)&sB1[32 * cb + 8 * g + 4 * half];
#pragma unroll
                    for (int e = 0; e < 4; ++e) acc[4 * g + e] = bb[e];
                }
                const u16x8_t wa = *(const u16x8_t *)&T[kT1 + (32 * cb + r) * kInPad + 8 * half];
                acc = mfma(wa, xb, acc);
                // group g holds channels 32 cb + 8 g + 4 half + (0..3) of point r
                uint32_t pk[4][2];
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    pk[g][0] = relu_pk_bf16(acc[4 * g], acc[4 * g + 1]);
                    pk[g][1] = relu_pk_bf16(acc[4 * g + 2], acc[4 * g + 3]);
                }
                // K-step kk = 2 cb + gg covers groups 2 gg (half 0 needs both halves' copy)
                // and 2 gg + 1 (half 1 likewise): swap the upper lanes of the first
                // with the lower lanes of the second
#pragma unroll
                for (int gg = 0; gg < 2; ++gg) {
                    uint32_t v1[2] = {pk[2 * gg][0], pk[2 * gg][1]};
                    uint32_t v2[2] = {pk[2 * gg + 1][0], pk[2 * gg + 1][1]};
#pragma unroll
                    for (int d = 0; d < 2; ++d) {
                        const auto sw = __builtin_amdgcn_permlane32_swap(v1[d], v2[d], false, false);
                        v1[d] = sw[0];
                        v2[d] = sw[1];
                    }
                    const u32x4_t q = {v1[0], v1[1], v2[0], v2[1]};
                    h[j][2 * cb + gg] = __builtin_bit_cast(u16x8_t, q);
                }
            }
        }
#pragma unroll
        for (int cb2 = 0; cb2 < kH2 / 32; ++cb2) {
            f32x16_t a0 = {}, a1 = {};
#pragma unroll
            for (int kk = 0; kk < kH1 / 16; ++kk) {
                const u16x8_t bv = *(const u16x8_t *)&sW2[(32 * cb2 + r) * kLd + 16 * kk + 8 * half];
                a0 = mfma(h[0][kk], bv, a0);
                a1 = mfma(h[1][kk], bv, a1);
            }
            fold_rows(a0, p0, c1, half, best[cb2], bidx[cb2]);
            fold_rows(a1, p0 + 32, c1, half, best[cb2], bidx[cb2]);
            __builtin_amdgcn_sched_barrier(0);  // keep the next block's LDS reads after this fold
        }
    }

    // merge: the two lane halves, then the waves (through LDS), then the
    // workgroups (64-bit atomicMax of (ordered value, inverted point))
    __syncthreads();  // every wave is done with W2
    unsigned long long *sKey = reinterpret_cast<unsigned long long *>(sW2);
#pragma unroll
    for (int c = 0; c < kH2 / 32; ++c) {
        const unsigned long long key =
            best[c] == -INFINITY ? 0ull
                                 : ((unsigned long long)ord_bits(best[c]) << 32) | (0xFFFFFFFFu - (uint32_t)bidx[c]);
        const uint32_t lo = __shfl_xor((uint32_t)key, 32, 64), hi = __shfl_xor((uint32_t)(key >> 32), 32, 64);
        const unsigned long long other = ((unsigned long long)hi << 32) | lo;
        if (half == 0) sKey[wave * kH2 + 32 * c + r] = key > other ? key : other;
    }
    __syncthreads();
    if (tid < kH2) {
        unsigned long long k = sKey[tid];
#pragma unroll
        for (int w = 1; w < kEncWaves; ++w) {
            const unsigned long long o = sKey[w * kH2 + tid];
            k = o > k ? o : k;
        }
        if (k) atomicMax(&keys[(int64_t)b * kH2 + tid], k);
    }
}

// feat = relu(max pre-activation + b2); arg = its point, or 0 where the
// channel is cut to zero (every point then ties at 0 and the lowest wins).
// Each key is reset to 0 once read, ready for the next pass.
__global__ void k_pool_finish(unsigned long long *__restrict__ keys, int n, const float *__restrict__ P,
                              float *__restrict__ feat, int32_t *__restrict__ arg)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const unsigned long long k = keys[i];
    keys[i] = 0ull;
    float f = 0.0f;
    int32_t a = 0;
    if (k) {
        const float t = ord_val((uint32_t)(k >> 32)) + P[kB2 + i % kH2];
        if (t > 0.0f) {
            f = t;
            a = (int32_t)(0xFFFFFFFFu - (uint32_t)k);
        }
    }
    feat[i] = f;
    arg[i] = a;
}

// ---- small GEMMs -------------------------------------------------------------
// C[m][n] = epi(sum_k A(m,k) B(k,n)), operands rounded to BF16, FP32 accumulate.
// A(m,k) = A[m*a_ms + k*a_ks] (FP32); B(k,n) = B[k*b_ks + n*b_ns] (FP32 or BF16 bits).
enum { kEpiNone = 0, kEpiBias = 1, kEpiBiasRelu = 2, kEpiMask = 3 };
constexpr int kGemmSteps = 8;  // k-steps of 16 per trip of the main loop

// KC: k is contiguous in both operands (a_ks = b_ks = 1, K % 16 = 0, rows
// 16-byte aligned; B is BF16): 8 consecutive k are two float4 loads of A
// and one 16-byte load of B.  The main loop issues the loads of kGemmSteps
// k-steps before their MFMAs, so that they are in flight together.
template <typename TB, int EPI, bool KC>
__global__ __launch_bounds__(64) void k_gemm(int Mr, int Nc, int K, const float *__restrict__ A, int64_t a_ms,
                                             int64_t a_ks, const TB *__restrict__ Bm, int64_t b_ks, int64_t b_ns,
                                             const float *__restrict__ bias, const float *__restrict__ mask,
                                             int64_t mask_ld, float *__restrict__ C, int64_t ldc)
{
    const int lane = threadIdx.x, r = lane & 31, half = lane >> 5;
    const int m0 = blockIdx.y * 32, n0 = blockIdx.x * 32;
    const int m = m0 + r, n = n0 + r;
    f32x16_t acc = {};
    // rows m >= Mr and columns n >= Nc repeat the last one (KC) or read zeros
    // and are not stored
    const float *ar = A + (int64_t)min(m, Mr - 1) * a_ms + 8 * half;
    const TB *br = Bm + (int64_t)min(n, Nc - 1) * b_ns + 8 * half;
    // operands of one k-step (the 8 consecutive k of this lane's half)
    struct Ops {
        float4 a0, a1;
        u16x8_t av, bv;
    };
    auto load = [&](int k0, Ops &o) {
        if constexpr (KC) {
            o.a0 = *(const float4 *)(ar + k0);
            o.a1 = *(const float4 *)(ar + k0 + 4);
            o.bv = *(const u16x8_t *)(br + k0);
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = k0 + 8 * half + j;
                o.av[j] = (m < Mr && k < K) ? bf16_bits(A[m * a_ms + k * a_ks]) : (uint16_t)0;
                o.bv[j] = (n < Nc && k < K) ? bf16_bits(Bm[k * b_ks + n * b_ns]) : (uint16_t)0;
            }
        }
    };
    auto use = [&](Ops &o) {
        if constexpr (KC) {
            o.av[0] = bf16_bits(o.a0.x);
            o.av[1] = bf16_bits(o.a0.y);
            o.av[2] = bf16_bits(o.a0.z);
            o.av[3] = bf16_bits(o.a0.w);
            o.av[4] = bf16_bits(o.a1.x);
            o.av[5] = bf16_bits(o.a1.y);
            o.av[6] = bf16_bits(o.a1.z);
            o.av[7] = bf16_bits(o.a1.w);
        }
        acc = mfma(o.av, o.bv, acc);
    };
    int k0 = 0;
    for (; k0 + 16 * kGemmSteps <= K; k0 += 16 * kGemmSteps) {  // all loads of a trip go out first
        Ops o[kGemmSteps];
#pragma unroll
        for (int t = 0; t < kGemmSteps; ++t) load(k0 + 16 * t, o[t]);
#pragma unroll
        for (int t = 0; t < kGemmSteps; ++t) use(o[t]);
    }
    for (; k0 < K; k0 += 16) {
        Ops o;
        load(k0, o);
        use(o);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int mm = m0 + c_row(i, lane);
        if (mm >= Mr || n >= Nc) continue;
        float v = acc[i];
        if (EPI == kEpiBias) v += bias[n];
        if (EPI == kEpiBiasRelu) v = fmaxf(v + bias[n], 0.0f);
        if (EPI == kEpiMask) v = mask[mm * mask_ld + n] > 0.0f ? v : 0.0f;
        C[mm * ldc + n] = v;
    }
}

__global__ void k_colsum(const float *__restrict__ X, int rows, int cols, int64_t ld, float *__restrict__ out)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    float s = 0.0f;
    for (int r = 0; r < rows; ++r) s += X[r * ld + c];
    out[c] = s;
}

// ---- mixture NLL -------------------------------------------------------------
__device__ inline void log_softmax8(const float *o, float lp[kM])
{
    float mx = o[0];
#pragma unroll
    for (int m = 1; m < kM; ++m) mx = fmaxf(mx, o[m]);
    float s = 0.0f;
#pragma unroll
    for (int m = 0; m < kM; ++m) s += expf(o[m] - mx);
    const float l = mx + logf(s);
#pragma unroll
    for (int m = 0; m < kM; ++m) lp[m] = o[m] - l;
}

__device__ inline float clamp_ls(float v) { return fminf(fmaxf(v, kLsMin), kLsMax); }

// thread per target: NLL and responsibilities
__global__ void k_nll(const float *__restrict__ out, const float *__restrict__ tg, const int32_t *__restrict__ off,
                      int B, int T, float *__restrict__ nll, float *__restrict__ resp)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    int lo = 0, hi = B;  // the object: the last b with off[b] <= t
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= t) lo = mid;
        else hi = mid;
    }
    const float *o = out + (int64_t)lo * kOut;
    const float *y = tg + (int64_t)t * kY;
    float lp[kM], comp[kM];
    log_softmax8(o, lp);
    const float half_log_2pi = 0.91893853320467274f;
    float mx = -INFINITY;
#pragma unroll
    for (int m = 0; m < kM; ++m) {
        float c = lp[m];
        for (int d = 0; d < kY; ++d) {
            const float ls = clamp_ls(o[kM + kM * kY + m * kY + d]);
            const float z = (y[d] - o[kM + m * kY + d]) * expf(-ls);
            c += -0.5f * z * z - ls - half_log_2pi;
        }
        comp[m] = c;
        mx = fmaxf(mx, c);
    }
    float s = 0.0f;
#pragma unroll
    for (int m = 0; m < kM; ++m) s += expf(comp[m] - mx);
    nll[t] = -(mx + logf(s));
#pragma unroll
    for (int m = 0; m < kM; ++m) resp[(int64_t)t * kM + m] = expf(comp[m] - mx) / s;
}

// thread per (object, output): gradient of the batch-mean NLL, targets in order
__global__ void k_dout(const float *__restrict__ out, const float *__restrict__ tg, const int32_t *__restrict__ off,
                       const float *__restrict__ resp, int B, float inv_T, float *__restrict__ dO)
{
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= B * kOut) return;
    const int b = id / kOut, j = id % kOut;
    const float *o = out + (int64_t)b * kOut;
    const int t0 = off[b], t1 = off[b + 1];
    float g = 0.0f;
    if (j < kM) {
        float lp[kM];
        log_softmax8(o, lp);
        const float pi = expf(lp[j]);
        for (int t = t0; t < t1; ++t) g += pi - resp[(int64_t)t * kM + j];
    } else if (j < kM + kM * kY) {
        const int m = (j - kM) / kY, d = (j - kM) % kY;
        const float ls = clamp_ls(o[kM + kM * kY + m * kY + d]);
        const float inv_s = expf(-ls), mu = o[j];
        for (int t = t0; t < t1; ++t) {
            const float z = (tg[(int64_t)t * kY + d] - mu) * inv_s;
            g -= resp[(int64_t)t * kM + m] * z * inv_s;
        }
    } else {
        const int m = (j - kM - kM * kY) / kY, d = (j - kM - kM * kY) % kY;
        const float raw = o[j];
        if (raw > kLsMin && raw < kLsMax) {
            const float inv_s = expf(-raw), mu = o[kM + m * kY + d];
            for (int t = t0; t < t1; ++t) {
                const float z = (tg[(int64_t)t * kY + d] - mu) * inv_s;
                g += resp[(int64_t)t * kM + m] * (1.0f - z * z);
            }
        }
    }
    dO[id] = g * inv_T;
}

// one workgroup of 256: fixed-order sum of the per-target NLL
__global__ __launch_bounds__(256) void k_loss_sum(const float *__restrict__ nll, int T, float *__restrict__ loss)
{
    __shared__ float s[256];
    float a = 0.0f;
    for (int t = threadIdx.x; t < T; t += 256) a += nll[t];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = s[0] / (float)T;
}

// ---- encoder backward (sparse through the max-pool) ---------------------------
// thread per (object, channel): the channel's gradient and the H1 row of its argmax point
__global__ void k_enc_bwd_sel(const float *__restrict__ x, int Np, const uint16_t *__restrict__ T,
                              const float *__restrict__ P, const float *__restrict__ feat,
                              const int32_t *__restrict__ arg, const float *__restrict__ dfeat, int B,
                              float *__restrict__ h1sel, float *__restrict__ gsel)
{
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= B * kH2) return;
    const int b = id / kH2;
    gsel[id] = feat[id] > 0.0f ? dfeat[id] : 0.0f;
    const u16x8_t xa = input_row(x + ((int64_t)b * Np + arg[id]) * kIn);
    float xin[kIn];
#pragma unroll
    for (int i = 0; i < kIn; ++i) xin[i] = bf16_val(xa[i]);
    for (int k = 0; k < kH1; ++k) {
        float z = 0.0f;
#pragma unroll
        for (int i = 0; i < kIn; ++i) z = fmaf(xin[i], bf16_val(T[kT1 + k * kInPad + i]), z);
        h1sel[(int64_t)id * kH1 + k] = bf16_val(bf16_bits(fmaxf(z + P[kB1 + k], 0.0f)));
    }
}

// thread per (channel c, hidden k): dW2[k][c], and db2[c] on k == 0
__global__ void k_enc_bwd_w2(const float *__restrict__ h1sel, const float *__restrict__ gsel, int B,
                             float *__restrict__ G)
{
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= kH2 * kH1) return;
    const int c = id / kH1, k = id % kH1;
    float s = 0.0f, sb = 0.0f;
    for (int b = 0; b < B; ++b) {
        const float g = gsel[b * kH2 + c];
        s = fmaf(h1sel[((int64_t)b * kH2 + c) * kH1 + k], g, s);
        sb += g;
    }
    G[kW2 + (int64_t)k * kH2 + c] = s;
    if (k == 0) G[kB2 + c] = sb;
}

// workgroup per hidden unit k: dW1[0..5][k] and db1[k] over all (object, channel)
__global__ __launch_bounds__(256) void k_enc_bwd_w1(const float *__restrict__ x, int Np,
                                                    const uint16_t *__restrict__ T,
                                                    const float *__restrict__ h1sel,
                                                    const float *__restrict__ gsel,
                                                    const int32_t *__restrict__ arg, int B,
                                                    float *__restrict__ G)
{
    __shared__ float s[kIn + 1][256];
    const int k = blockIdx.x, tid = threadIdx.x;
    float a[kIn + 1] = {0, 0, 0, 0, 0, 0, 0};
    for (int id = tid; id < B * kH2; id += 256) {
        if (h1sel[(int64_t)id * kH1 + k] <= 0.0f) continue;
        const int b = id / kH2, c = id % kH2;
        const float d = bf16_val(T[kT2 + (int64_t)c * kH1 + k]) * gsel[id];
        if (d == 0.0f) continue;
        const float *xp = x + ((int64_t)b * Np + arg[id]) * kIn;
        a[0] = fmaf(xp[0] * kInvSP, d, a[0]);
        a[1] = fmaf(xp[1] * kInvSP, d, a[1]);
        a[2] = fmaf(xp[2] * kInvSP, d, a[2]);
        a[3] = fmaf(xp[3], d, a[3]);
        a[4] = fmaf(xp[4], d, a[4]);
        a[5] = fmaf(xp[5], d, a[5]);
        a[6] += d;
    }
#pragma unroll
    for (int i = 0; i <= kIn; ++i) s[i][tid] = a[i];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
#pragma unroll
            for (int i = 0; i <= kIn; ++i) s[i][tid] += s[i][tid + w];
        }
        __syncthreads();
    }
    if (tid <= kIn) {
        if (tid < kIn) G[kW1 + (int64_t)tid * kH1 + k] = s[tid][0];
        else G[kB1 + k] = s[kIn][0];
    }
}

// ---- sampler -----------------------------------------------------------------
__device__ inline float u01_open(uint32_t w) { return (float)((w >> 8) + 1u) * (1.0f / 16777216.0f); }

__global__ void k_sample(const float *__restrict__ o, int n, uint32_t s_lo, uint32_t s_hi, float ufrac, float d_lo,
                         float d_hi, float *__restrict__ poses)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t w[12];
    philox4x32_10((uint32_t)i, 0u, kPurposeSample, 0u, s_lo, s_hi, w);
    philox4x32_10((uint32_t)i, 1u, kPurposeSample, 0u, s_lo, s_hi, w + 4);
    philox4x32_10((uint32_t)i, 2u, kPurposeSample, 0u, s_lo, s_hi, w + 8);
    float R[3][3], t[3];
    if (u01f(w[0]) < ufrac) {
        // uniform fallback: Shoemake rotation, direction on the +z hemisphere, distance U[d_lo, d_hi]
        const float u1 = u01f(w[1]);
        const float a = sqrtf(1.0f - u1), bq = sqrtf(u1);
        float s2, c2, s3, c3;
        sincospif(2.0f * u01f(w[2]), &s2, &c2);
        sincospif(2.0f * u01f(w[3]), &s3, &c3);
        const float qx = a * s2, qy = a * c2, qz = bq * s3, qw = bq * c3;
        R[0][0] = 1 - 2 * (qy * qy + qz * qz); R[0][1] = 2 * (qx * qy - qz * qw); R[0][2] = 2 * (qx * qz + qy * qw);
        R[1][0] = 2 * (qx * qy + qz * qw); R[1][1] = 1 - 2 * (qx * qx + qz * qz); R[1][2] = 2 * (qy * qz - qx * qw);
        R[2][0] = 2 * (qx * qz - qy * qw); R[2][1] = 2 * (qy * qz + qx * qw); R[2][2] = 1 - 2 * (qx * qx + qy * qy);
        const float cz = u01f(w[4]);
        float sp, cp;
        sincospif(2.0f * u01f(w[5]), &sp, &cp);
        const float d = d_lo + (d_hi - d_lo) * u01f(w[6]);
        const float sz = sqrtf(fmaxf(0.0f, 1.0f - cz * cz));
        t[0] = d * sz * cp;
        t[1] = d * sz * sp;
        t[2] = d * cz;
    } else {
        float lp[kM];
        log_softmax8(o, lp);
        const float uc = u01f(w[1]);
        float cum = 0.0f;
        int m = kM - 1;
        for (int c = 0; c < kM; ++c) {
            cum += expf(lp[c]);
            if (uc < cum) {
                m = c;
                break;
            }
        }
        float z[10];
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            const float rr = sqrtf(-2.0f * logf(u01_open(w[2 + 2 * j])));
            float sn, cs;
            sincospif(2.0f * u01f(w[3 + 2 * j]), &sn, &cs);
            z[2 * j] = rr * cs;
            z[2 * j + 1] = rr * sn;
        }
        float y[kY];
#pragma unroll
        for (int d = 0; d < kY; ++d)
            y[d] = o[kM + m * kY + d] + expf(clamp_ls(o[kM + kM * kY + m * kY + d])) * z[d];
        // Gram-Schmidt of (y0..2, y3..5): columns b1, b2, b1 x b2
        const float n1 = fmaxf(sqrtf(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]), 1e-8f);
        const float b1[3] = {y[0] / n1, y[1] / n1, y[2] / n1};
        const float dp = b1[0] * y[3] + b1[1] * y[4] + b1[2] * y[5];
        float v[3] = {y[3] - dp * b1[0], y[4] - dp * b1[1], y[5] - dp * b1[2]};
        const float n2 = fmaxf(sqrtf(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]), 1e-8f);
        const float b2[3] = {v[0] / n2, v[1] / n2, v[2] / n2};
        const float b3[3] = {b1[1] * b2[2] - b1[2] * b2[1], b1[2] * b2[0] - b1[0] * b2[2],
                             b1[0] * b2[1] - b1[1] * b2[0]};
        for (int r = 0; r < 3; ++r) {
            R[r][0] = b1[r];
            R[r][1] = b2[r];
            R[r][2] = b3[r];
            t[r] = y[6 + r] * kST;
        }
    }
    float *q = poses + (int64_t)i * 12;
    for (int r = 0; r < 3; ++r) {
        q[4 * r + 0] = R[r][0];
        q[4 * r + 1] = R[r][1];
        q[4 * r + 2] = R[r][2];
        q[4 * r + 3] = t[r];
    }
}

inline unsigned blocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace prop
}  // namespace lg

using namespace lg;
using namespace lg::prop;

struct lg_prop {
    int device = 0;
    int max_batch = 0, max_points = 0, max_targets = 0;
    int64_t step = 0;
    void *slab = nullptr;
    float *P, *G, *Mo, *Vo;       // [kNParams]
    uint16_t *T;                  // [kNT]
    unsigned long long *keys;     // [maxB][256], all 0 between forward passes
    bool keys_dirty = false;      // a forward pass stopped between k_encode and k_pool_finish
    float *feat, *ua, *ub, *out;  // [maxB][256] x3, [maxB][152]
    float *dO, *dub, *dua, *dfeat;
    int32_t *arg;                 // [maxB][256]
    float *nll, *resp;            // [maxT], [maxT][8]
    float *h1sel, *gsel;          // [maxB][256][128], [maxB][256]
    float *loss;                  // [1]
};

namespace {

hipStream_t st(void *s) { return reinterpret_cast<hipStream_t>(s); }

template <typename TB, int EPI>
void gemm(hipStream_t s, int Mr, int Nc, int K, const float *A, int64_t a_ms, int64_t a_ks, const TB *Bm,
          int64_t b_ks, int64_t b_ns, const float *bias, const float *mask, int64_t mask_ld, float *C, int64_t ldc)
{
    const bool kc = std::is_same<TB, uint16_t>::value && a_ks == 1 && b_ks == 1 && K % 16 == 0 && a_ms % 4 == 0 &&
                    b_ns % 8 == 0 && ((uintptr_t)A & 15) == 0 && ((uintptr_t)Bm & 15) == 0;
    if (kc)
        hipLaunchKernelGGL((k_gemm<TB, EPI, true>), dim3(blocks(Nc, 32), blocks(Mr, 32)), dim3(64), 0, s, Mr, Nc, K,
                           A, a_ms, a_ks, Bm, b_ks, b_ns, bias, mask, mask_ld, C, ldc);
    else
        hipLaunchKernelGGL((k_gemm<TB, EPI, false>), dim3(blocks(Nc, 32), blocks(Mr, 32)), dim3(64), 0, s, Mr, Nc,
                           K, A, a_ms, a_ks, Bm, b_ks, b_ns, bias, mask, mask_ld, C, ldc);
}

lg_status check_batch(const lg_prop *p, const float *x, int B, int Np)
{
    if (!p) return fail(LG_EINVAL, "null proposer");
    if (!x) return fail(LG_EINVAL, "null input points");
    if (B < 1 || B > p->max_batch) return fail(LG_EINVAL, "batch outside [1, max_batch]");
    if (Np < 1 || Np > p->max_points) return fail(LG_EINVAL, "point count outside [1, max_points]");
    return LG_OK;
}

lg_status forward(lg_prop *p, const float *x, int B, int Np, hipStream_t s)
{
    // k_pool_finish leaves the keys it read at 0, so the next pass needs no fill
    if (p->keys_dirty)
        hipLaunchKernelGGL(k_fill_u64, dim3(blocks((int64_t)p->max_batch * kH2, 256)), dim3(256), 0, s, p->keys,
                           (int64_t)p->max_batch * kH2);
    p->keys_dirty = true;
    hipLaunchKernelGGL(k_encode, dim3(blocks(Np, kEncChunk), B), dim3(kEncThreads), 0, s, x, Np, p->T, p->P,
                       p->keys);
    hipLaunchKernelGGL(k_pool_finish, dim3(blocks((int64_t)B * kH2, 256)), dim3(256), 0, s, p->keys, B * kH2, p->P,
                       p->feat, p->arg);
    if (hipPeekAtLastError() == hipSuccess) p->keys_dirty = false;
    gemm<uint16_t, kEpiBiasRelu>(s, B, kHH, kH2, p->feat, kH2, 1, p->T + kTa, 1, kH2, p->P + kBa, nullptr, 0, p->ua,
                                 kHH);
    gemm<uint16_t, kEpiBiasRelu>(s, B, kHH, kHH, p->ua, kHH, 1, p->T + kTb, 1, kHH, p->P + kBb, nullptr, 0, p->ub,
                                 kHH);
    gemm<uint16_t, kEpiBias>(s, B, kOut, kHH, p->ub, kHH, 1, p->T + kTc, 1, kHH, p->P + kBc, nullptr, 0, p->out,
                             kOut);
    LG_HIP(hipGetLastError());
    return LG_OK;
}

lg_status backward(lg_prop *p, const float *x, int B, int Np, const float *tg, const int32_t *off, int T,
                   hipStream_t s)
{
    lg_status e = forward(p, x, B, Np, s);
    if (e != LG_OK) return e;
    hipLaunchKernelGGL(k_nll, dim3(blocks(T, 256)), dim3(256), 0, s, p->out, tg, off, B, T, p->nll, p->resp);
    hipLaunchKernelGGL(k_loss_sum, dim3(1), dim3(256), 0, s, p->nll, T, p->loss);
    hipLaunchKernelGGL(k_dout, dim3(blocks((int64_t)B * kOut, 256)), dim3(256), 0, s, p->out, tg, off, p->resp, B,
                       1.0f / (float)T, p->dO);
    float *G = p->G;
    // output layer
    gemm<float, kEpiNone>(s, kHH, kOut, B, p->ub, 1, kHH, p->dO, kOut, 1, nullptr, nullptr, 0, G + kWc, kOut);
    hipLaunchKernelGGL(k_colsum, dim3(blocks(kOut, 256)), dim3(256), 0, s, p->dO, B, kOut, (int64_t)kOut, G + kBc);
    gemm<uint16_t, kEpiMask>(s, B, kHH, kOut, p->dO, kOut, 1, p->T + kTc, kHH, 1, nullptr, p->ub, kHH, p->dub, kHH);
    // second head layer
    gemm<float, kEpiNone>(s, kHH, kHH, B, p->ua, 1, kHH, p->dub, kHH, 1, nullptr, nullptr, 0, G + kWb, kHH);
    hipLaunchKernelGGL(k_colsum, dim3(blocks(kHH, 256)), dim3(256), 0, s, p->dub, B, kHH, (int64_t)kHH, G + kBb);
    gemm<uint16_t, kEpiMask>(s, B, kHH, kHH, p->dub, kHH, 1, p->T + kTb, kHH, 1, nullptr, p->ua, kHH, p->dua, kHH);
    // first head layer
    gemm<float, kEpiNone>(s, kH2, kHH, B, p->feat, 1, kH2, p->dua, kHH, 1, nullptr, nullptr, 0, G + kWa, kHH);
    hipLaunchKernelGGL(k_colsum, dim3(blocks(kHH, 256)), dim3(256), 0, s, p->dua, B, kHH, (int64_t)kHH, G + kBa);
    gemm<uint16_t, kEpiNone>(s, B, kH2, kHH, p->dua, kHH, 1, p->T + kTa, kH2, 1, nullptr, nullptr, 0, p->dfeat,
                             kH2);
    // encoder through the max-pool
    hipLaunchKernelGGL(k_enc_bwd_sel, dim3(blocks((int64_t)B * kH2, 256)), dim3(256), 0, s, x, Np, p->T, p->P,
                       p->feat, p->arg, p->dfeat, B, p->h1sel, p->gsel);
    hipLaunchKernelGGL(k_enc_bwd_w2, dim3(blocks((int64_t)kH2 * kH1, 256)), dim3(256), 0, s, p->h1sel, p->gsel, B,
                       G);
    hipLaunchKernelGGL(k_enc_bwd_w1, dim3(kH1), dim3(256), 0, s, x, Np, p->T, p->h1sel, p->gsel, p->arg, B, G);
    LG_HIP(hipGetLastError());
    return LG_OK;
}

}  // namespace

extern "C" {

int64_t lg_prop_num_params(void) { return kNParams; }

lg_status lg_prop_create(const lg_prop_params *params, void *stream, lg_prop **out)
{
    if (!params || !out) return fail(LG_EINVAL, "null params or output handle");
    *out = nullptr;
    const int B = params->max_batch, N = params->max_points, T = params->max_targets;
    if (B < 1 || B > 4096 || N < 1 || N > (1 << 24) || T < 1 || T > (1 << 26))
        return fail(LG_EINVAL, "max_batch in [1, 4096], max_points in [1, 2^24], max_targets in [1, 2^26]");
    lg_prop *p = new lg_prop();
    p->max_batch = B;
    p->max_points = N;
    p->max_targets = T;
    LG_HIP(hipGetDevice(&p->device));
    // one slab: every piece 256-byte aligned
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    const size_t oP = take(kNParams * 4), oG = take(kNParams * 4), oM = take(kNParams * 4), oV = take(kNParams * 4);
    const size_t oT = take(kNT * 2), oK = take((size_t)B * kH2 * 8);
    const size_t oF = take((size_t)B * kH2 * 4), oUa = take((size_t)B * kHH * 4), oUb = take((size_t)B * kHH * 4);
    const size_t oO = take((size_t)B * kOut * 4), oDO = take((size_t)B * kOut * 4);
    const size_t oDub = take((size_t)B * kHH * 4), oDua = take((size_t)B * kHH * 4), oDf = take((size_t)B * kH2 * 4);
    const size_t oA = take((size_t)B * kH2 * 4), oN = take((size_t)T * 4), oR = take((size_t)T * kM * 4);
    const size_t oH = take((size_t)B * kH2 * kH1 * 4), oGs = take((size_t)B * kH2 * 4), oL = take(4);
    hipError_t e = hipMalloc(&p->slab, off);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "hipMalloc(proposer)");
    }
    char *base = static_cast<char *>(p->slab);
    p->P = (float *)(base + oP);
    p->G = (float *)(base + oG);
    p->Mo = (float *)(base + oM);
    p->Vo = (float *)(base + oV);
    p->T = (uint16_t *)(base + oT);
    p->keys = (unsigned long long *)(base + oK);
    p->feat = (float *)(base + oF);
    p->ua = (float *)(base + oUa);
    p->ub = (float *)(base + oUb);
    p->out = (float *)(base + oO);
    p->dO = (float *)(base + oDO);
    p->dub = (float *)(base + oDub);
    p->dua = (float *)(base + oDua);
    p->dfeat = (float *)(base + oDf);
    p->arg = (int32_t *)(base + oA);
    p->nll = (float *)(base + oN);
    p->resp = (float *)(base + oR);
    p->h1sel = (float *)(base + oH);
    p->gsel = (float *)(base + oGs);
    p->loss = (float *)(base + oL);
    hipStream_t s = st(stream);
    hipLaunchKernelGGL(k_init, dim3(blocks(kNParams, 256)), dim3(256), 0, s, p->P,
                       (uint32_t)params->seed, (uint32_t)(params->seed >> 32));
    hipLaunchKernelGGL(k_refresh_bf16, dim3(blocks(kNT, 256)), dim3(256), 0, s, p->P, p->T);
    hipLaunchKernelGGL(k_fill_u64, dim3(blocks((int64_t)B * kH2, 256)), dim3(256), 0, s, p->keys, (int64_t)B * kH2);
    e = hipMemsetAsync(p->Mo, 0, kNParams * 4, s);
    if (e == hipSuccess) e = hipMemsetAsync(p->Vo, 0, kNParams * 4, s);
    if (e == hipSuccess) e = hipMemsetAsync(p->G, 0, kNParams * 4, s);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipFree(p->slab);
        delete p;
        return hip_fail(e, "proposer initialisation");
    }
    *out = p;
    return LG_OK;
}

lg_status lg_prop_release(lg_prop *p)
{
    if (!p) return LG_OK;
    (void)hipDeviceSynchronize();
    hipError_t e = hipFree(p->slab);
    delete p;
    return e == hipSuccess ? LG_OK : hip_fail(e, "hipFree(proposer)");
}

lg_status lg_prop_get_params(const lg_prop *p, float *host_out)
{
    if (!p || !host_out) return fail(LG_EINVAL, "null proposer or output");
    LG_HIP(hipDeviceSynchronize());
    LG_HIP(hipMemcpy(host_out, p->P, kNParams * 4, hipMemcpyDeviceToHost));
    return LG_OK;
}

lg_status lg_prop_set_params(lg_prop *p, const float *host_in)
{
    if (!p || !host_in) return fail(LG_EINVAL, "null proposer or input");
    LG_HIP(hipDeviceSynchronize());
    LG_HIP(hipMemcpy(p->P, host_in, kNParams * 4, hipMemcpyHostToDevice));
    LG_HIP(hipMemset(p->Mo, 0, kNParams * 4));
    LG_HIP(hipMemset(p->Vo, 0, kNParams * 4));
    hipLaunchKernelGGL(k_refresh_bf16, dim3(blocks(kNT, 256)), dim3(256), 0, 0, p->P, p->T);
    LG_HIP(hipGetLastError());
    LG_HIP(hipDeviceSynchronize());
    p->step = 0;
    return LG_OK;
}

lg_status lg_prop_forward(lg_prop *p, const float *x, int32_t B, int32_t Np, float *out, float *feat, int32_t *arg,
                          void *stream)
{
    lg_status e = check_batch(p, x, B, Np);
    if (e != LG_OK) return e;
    hipStream_t s = st(stream);
    e = forward(p, x, B, Np, s);
    if (e != LG_OK) return e;
    if (out) LG_HIP(hipMemcpyAsync(out, p->out, (size_t)B * kOut * 4, hipMemcpyDeviceToDevice, s));
    if (feat) LG_HIP(hipMemcpyAsync(feat, p->feat, (size_t)B * kH2 * 4, hipMemcpyDeviceToDevice, s));
    if (arg) LG_HIP(hipMemcpyAsync(arg, p->arg, (size_t)B * kH2 * 4, hipMemcpyDeviceToDevice, s));
    return LG_OK;
}

lg_status lg_prop_backward(lg_prop *p, const float *x, int32_t B, int32_t Np, const float *targets,
                           const int32_t *offsets, int32_t T, float *loss, float *grad, void *stream)
{
    lg_status e = check_batch(p, x, B, Np);
    if (e != LG_OK) return e;
    if (!targets || !offsets) return fail(LG_EINVAL, "null targets or offsets");
    if (T < 1 || T > p->max_targets) return fail(LG_EINVAL, "target count outside [1, max_targets]");
    hipStream_t s = st(stream);
    e = backward(p, x, B, Np, targets, offsets, T, s);
    if (e != LG_OK) return e;
    if (loss) LG_HIP(hipMemcpyAsync(loss, p->loss, 4, hipMemcpyDeviceToDevice, s));
    if (grad) LG_HIP(hipMemcpyAsync(grad, p->G, kNParams * 4, hipMemcpyDeviceToDevice, s));
    return LG_OK;
}

lg_status lg_prop_adam(lg_prop *p, float lr, float beta1, float beta2, float eps, void *stream)
{
    if (!p) return fail(LG_EINVAL, "null proposer");
    if (!(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return fail(LG_EINVAL, "lr >= 0, beta1 and beta2 in [0, 1), eps > 0");
    hipStream_t s = st(stream);
    p->step += 1;
    const double bc1 = 1.0 - pow((double)beta1, (double)p->step), bc2 = 1.0 - pow((double)beta2, (double)p->step);
    const float lr_t = (float)(lr * sqrt(bc2) / bc1);
    hipLaunchKernelGGL(k_adam, dim3(blocks(kNParams, 256)), dim3(256), 0, s, p->P, p->G, p->Mo, p->Vo, lr_t, beta1,
                       beta2, eps);
    hipLaunchKernelGGL(k_refresh_bf16, dim3(blocks(kNT, 256)), dim3(256), 0, s, p->P, p->T);
    LG_HIP(hipGetLastError());
    return LG_OK;
}

lg_status lg_prop_train_step(lg_prop *p, const float *x, int32_t B, int32_t Np, const float *targets,
                             const int32_t *offsets, int32_t T, float lr, float *loss, void *stream)
{
    lg_status e = lg_prop_backward(p, x, B, Np, targets, offsets, T, loss, nullptr, stream);
    if (e != LG_OK) return e;
    return lg_prop_adam(p, lr, 0.9f, 0.999f, 1e-8f, stream);
}

lg_status lg_prop_sample_mixture(const float *mix, int32_t n_poses, uint64_t seed, float uniform_frac, float d_lo,
                                 float d_hi, float *poses, void *stream)
{
    if (n_poses < 0) return fail(LG_EINVAL, "negative pose count");
    if (n_poses == 0) return LG_OK;
    if (!mix || !poses) return fail(LG_EINVAL, "null mixture or poses");
    if (!(uniform_frac >= 0.0f && uniform_frac <= 1.0f)) return fail(LG_EINVAL, "uniform_frac outside [0, 1]");
    if (!(d_lo >= 0.0f && d_lo <= d_hi)) return fail(LG_EINVAL, "need 0 <= d_lo <= d_hi");
    hipLaunchKernelGGL(k_sample, dim3(blocks(n_poses, 256)), dim3(256), 0, st(stream), mix, n_poses, (uint32_t)seed,
                       (uint32_t)(seed >> 32), uniform_frac, d_lo, d_hi, poses);
    LG_HIP(hipGetLastError());
    return LG_OK;
}

lg_status lg_prop_sample(lg_prop *p, const float *x, int32_t Np, int32_t n_poses, uint64_t seed, float uniform_frac,
                         float d_lo, float d_hi, float *poses, void *stream)
{
    lg_status e = check_batch(p, x, 1, Np);
    if (e != LG_OK) return e;
    if (n_poses < 0) return fail(LG_EINVAL, "negative pose count");
    if (n_poses == 0) return LG_OK;
    if (!poses) return fail(LG_EINVAL, "null poses");
    if (!(uniform_frac >= 0.0f && uniform_frac <= 1.0f)) return fail(LG_EINVAL, "uniform_frac outside [0, 1]");
    if (!(d_lo >= 0.0f && d_lo <= d_hi)) return fail(LG_EINVAL, "need 0 <= d_lo <= d_hi");
    hipStream_t s = st(stream);
    e = forward(p, x, 1, Np, s);
    if (e != LG_OK) return e;
    return lg_prop_sample_mixture(p->out, n_poses, seed, uniform_frac, d_lo, d_hi, poses, stream);
}

}  // extern "C"
