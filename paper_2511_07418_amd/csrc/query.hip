// Object contact query (Sec. 4.2-4.3, Def. 4.3) with the per-dependency-group
// merge of Sec. 5.3.
//
// One workgroup per pose; each wave sweeps 64 consecutive object points
// (structure-of-arrays, Morton-sorted by the caller so a wave touches a
// compact patch of the field).  Per point: x = R p + t folded into one affine
// map per finger window, query normal -R n, its bin, one 4/8-byte gather of
// the finger's merged table, and a wave ballot that yields the 64 domain bits
// of the finger for the chunk.  Counts are popcounts of the ballots.
#include <algorithm>

#include "lg_internal.h"

namespace lg {

constexpr int kQueryThreads = 256;
constexpr int kQueryWaves = kQueryThreads / 64;

template <int W, int FM>
__global__ void __launch_bounds__(kQueryThreads)
k_query(DevHand H, const uint32_t *__restrict__ merged, const float *__restrict__ pts,
        const float *__restrict__ nrm, int N, const float *__restrict__ poses,
        uint32_t *__restrict__ dom_bits, uint32_t *__restrict__ dom_count)
{
    __shared__ float cb[3 * kMaxBins];
    __shared__ uint32_t lut[6 * kLutRes * kLutRes];
    __shared__ Affine aff[FM];
    __shared__ uint32_t cnt[FM][kQueryWaves];
    const int g = blockIdx.x;
    const float *pose = poses + 12 * (int64_t)g;
    for (int i = threadIdx.x; i < 3 * H.B; i += blockDim.x) cb[i] = H.bin_c[i];
    for (int i = threadIdx.x; i < 6 * kLutRes * kLutRes; i += blockDim.x) lut[i] = H.bin_lut[i];
    if (threadIdx.x < H.F) aff[threadIdx.x] = finger_affine(H, pose, threadIdx.x);
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int F = H.F, G = H.G, B = H.B;
    const int64_t G3W = (int64_t)G * G * G * W;
    const int NW = (N + 31) >> 5, nchunks = (N + 63) >> 6;
    float P[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) P[i] = pose[i];
    uint32_t c[FM];
#pragma unroll
    for (int f = 0; f < FM; ++f) c[f] = 0;
    // Waves take blocks of 32 consecutive chunks (2,048 points, a compact
    // patch of the Morton-ordered object) in turn.  The 64 ballot words of a
    // block stay in registers, lane 2j / 2j+1 holding chunk j's halves, and
    // leave as one coalesced 256-byte store per finger.
    const int nblk = (nchunks + 31) >> 5;
    for (int blk = wave; blk < nblk; blk += kQueryWaves) {
        uint32_t acc[FM];
#pragma unroll
        for (int f = 0; f < FM; ++f) acc[f] = 0;
        const int c_end = min(nchunks, (blk + 1) * 32);
        for (int chunk = blk * 32; chunk < c_end; ++chunk) {
            // re-read the per-finger maps from LDS every chunk instead of pinning
            // 12 x F registers for them: halves the register footprint
            asm volatile("" ::: "memory");
            const int i = chunk * 64 + lane;
            const bool valid = i < N;
            float px = 0.f, py = 0.f, pz = 0.f, nx = 0.f, ny = 0.f, nz = 1.f;
            if (valid) {
                px = pts[i];
                py = pts[N + i];
                pz = pts[2 * N + i];
                nx = nrm[i];
                ny = nrm[N + i];
                nz = nrm[2 * N + i];
            }
            float qx, qy, qz;
            query_dir(P, nx, ny, nz, qx, qy, qz);
            const int b = nearest_bin_lut(lut, cb, B, qx, qy, qz);
            // one 32-bit word per finger: the word of the table that holds bit b;
            // all finger gathers are issued before any is consumed
            uint32_t word[FM];
#pragma unroll
            for (int f = 0; f < FM; ++f) {
                word[f] = 0;
                if (f < F) {
                    const int v = window_voxel(aff[f], G, px, py, pz);
                    const uint32_t *tab = merged + f * G3W;  // uniform base, 32-bit lane offsets
                    if (valid && v >= 0) word[f] = tab[(uint32_t)v * W + (uint32_t)(b >> 5)];
                }
            }
            const int j2 = 2 * (chunk - blk * 32);
#pragma unroll
            for (int f = 0; f < FM; ++f) {
                if (f >= F) break;
                const bool hit = (word[f] >> (b & 31)) & 1u;
                const unsigned long long m = __ballot(hit);
                c[f] += (uint32_t)__popcll(m);
                acc[f] = lane == j2 ? (uint32_t)m : lane == j2 + 1 ? (uint32_t)(m >> 32) : acc[f];
            }
        }
        const int wi = blk * 64 + lane;
        if (wi < NW) {
#pragma unroll
            for (int f = 0; f < FM; ++f)
                if (f < F) dom_bits[((int64_t)g * F + f) * NW + wi] = acc[f];
        }
    }
    if (lane == 0) {
#pragma unroll
        for (int f = 0; f < FM; ++f)
            if (f < F) cnt[f][wave] = c[f];
    }
    __syncthreads();
    if (threadIdx.x < F) {
        uint32_t s = 0;
        for (int w = 0; w < kQueryWaves; ++w) s += cnt[threadIdx.x][w];
        dom_count[(int64_t)g * F + threadIdx.x] = s;
    }
}

// Cone query (Sec. 4.3's theta_hit test): a query (x, -R n) hits finger f if
// a bin b set in the finger's merged word(s) at voxel(x) has c_b . q >= cos_hit.
// Same sweep and block stores as k_query; the set bits of the voxel's entry
// are tested one by one against the cone.
template <int W, int FM>
__global__ void __launch_bounds__(kQueryThreads)
k_query_cone(DevHand H, const uint32_t *__restrict__ merged, const float *__restrict__ pts,
             const float *__restrict__ nrm, int N, const float *__restrict__ poses, float cos_hit,
             uint32_t *__restrict__ dom_bits, uint32_t *__restrict__ dom_count)
{
    __shared__ float cb[3 * kMaxBins];
    __shared__ Affine aff[FM];
    __shared__ uint32_t cnt[FM][kQueryWaves];
    const int g = blockIdx.x;
    const float *pose = poses + 12 * (int64_t)g;
    for (int i = threadIdx.x; i < 3 * H.B; i += blockDim.x) cb[i] = H.bin_c[i];
    if (threadIdx.x < H.F) aff[threadIdx.x] = finger_affine(H, pose, threadIdx.x);
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int F = H.F, G = H.G;
    const int64_t G3W = (int64_t)G * G * G * W;
    const int NW = (N + 31) >> 5, nchunks = (N + 63) >> 6;
    float P[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) P[i] = pose[i];
    uint32_t c[FM];
#pragma unroll
    for (int f = 0; f < FM; ++f) c[f] = 0;
    const int nblk = (nchunks + 31) >> 5;
    for (int blk = wave; blk < nblk; blk += kQueryWaves) {
        uint32_t acc[FM];
#pragma unroll
        for (int f = 0; f < FM; ++f) acc[f] = 0;
        const int c_end = min(nchunks, (blk + 1) * 32);
        for (int chunk = blk * 32; chunk < c_end; ++chunk) {
            asm volatile("" ::: "memory");
            const int i = chunk * 64 + lane;
            const bool valid = i < N;
            float px = 0.f, py = 0.f, pz = 0.f, nx = 0.f, ny = 0.f, nz = 1.f;
            if (valid) {
                px = pts[i];
                py = pts[N + i];
                pz = pts[2 * N + i];
                nx = nrm[i];
                ny = nrm[N + i];
                nz = nrm[2 * N + i];
            }
            float qx, qy, qz;
            query_dir(P, nx, ny, nz, qx, qy, qz);
            unsigned long long ent[FM];
#pragma unroll
            for (int f = 0; f < FM; ++f) {
                ent[f] = 0ull;
                if (f < F) {
                    const int v = window_voxel(aff[f], G, px, py, pz);
                    const uint32_t *tab = merged + f * G3W;
                    if (valid && v >= 0) {
                        if (W == 2) ent[f] = *reinterpret_cast<const unsigned long long *>(tab + (uint32_t)v * 2u);
                        else ent[f] = tab[(uint32_t)v];
                    }
                }
            }
            const int j2 = 2 * (chunk - blk * 32);
#pragma unroll
            for (int f = 0; f < FM; ++f) {
                if (f >= F) break;
                bool hit = false;
                unsigned long long m = ent[f];
                while (m) {
                    const int b = __ffsll((long long)m) - 1;
                    m &= m - 1ull;
                    if (fmaf(cb[3 * b], qx, fmaf(cb[3 * b + 1], qy, cb[3 * b + 2] * qz)) >= cos_hit) {
                        hit = true;
                        break;
                    }
                }
                const unsigned long long bm = __ballot(hit);
                c[f] += (uint32_t)__popcll(bm);
                acc[f] = lane == j2 ? (uint32_t)bm : lane == j2 + 1 ? (uint32_t)(bm >> 32) : acc[f];
            }
        }
        const int wi = blk * 64 + lane;
        if (wi < NW) {
#pragma unroll
            for (int f = 0; f < FM; ++f)
                if (f < F) dom_bits[((int64_t)g * F + f) * NW + wi] = acc[f];
        }
    }
    if (lane == 0) {
#pragma unroll
        for (int f = 0; f < FM; ++f)
            if (f < F) cnt[f][wave] = c[f];
    }
    __syncthreads();
    if (threadIdx.x < F) {
        uint32_t s = 0;
        for (int w = 0; w < kQueryWaves; ++w) s += cnt[threadIdx.x][w];
        dom_count[(int64_t)g * F + threadIdx.x] = s;
    }
}

}  // namespace lg

using namespace lg;

extern "C" lg_status lg_query_domains(const lg_field *field, const float *pts, const float *nrm, int32_t n_points,
                                      const float *poses, int32_t n_poses, uint32_t *dom_bits, uint32_t *dom_count,
                                      void *stream)
{
    if (!field) return fail(LG_EINVAL, "null field");
    if (n_points < 0 || n_poses < 0) return fail(LG_EINVAL, "negative size");
    if (n_poses == 0) return LG_OK;
    if (!poses || !dom_count || (n_points > 0 && (!pts || !nrm || !dom_bits)))
        return fail(LG_EINVAL, "null device buffer");
    hipStream_t s = as_stream(stream);
    const DevHand &H = field->dh;
#define LG_QUERY(W, FM)                                                                                     \
    hipLaunchKernelGGL((k_query<W, FM>), dim3(n_poses), dim3(kQueryThreads), 0, s, H, field->d_merged, pts, nrm, \
                       n_points, poses, dom_bits, dom_count)
    if (H.W == 1) {
        if (H.F <= 3) LG_QUERY(1, 3); else if (H.F <= 4) LG_QUERY(1, 4); else if (H.F <= 5) LG_QUERY(1, 5); else LG_QUERY(1, 8);
    } else {
        if (H.F <= 3) LG_QUERY(2, 3); else if (H.F <= 4) LG_QUERY(2, 4); else if (H.F <= 5) LG_QUERY(2, 5); else LG_QUERY(2, 8);
    }
#undef LG_QUERY
    LG_HIP(hipGetLastError());
    return LG_OK;
}

extern "C" lg_status lg_query_domains_cone(const lg_field *field, const float *pts, const float *nrm, int32_t n_points,
                                           const float *poses, int32_t n_poses, float cos_hit, uint32_t *dom_bits,
                                           uint32_t *dom_count, void *stream)
{
    if (!field) return fail(LG_EINVAL, "null field");
    if (n_points < 0 || n_poses < 0) return fail(LG_EINVAL, "negative size");
    if (!(cos_hit >= -1.0f && cos_hit <= 1.0f)) return fail(LG_EINVAL, "cos_hit outside [-1, 1]");
    if (n_poses == 0) return LG_OK;
    if (!poses || !dom_count || (n_points > 0 && (!pts || !nrm || !dom_bits)))
        return fail(LG_EINVAL, "null device buffer");
    hipStream_t s = as_stream(stream);
    const DevHand &H = field->dh;
#define LG_QCONE(W, FM)                                                                                        \
    hipLaunchKernelGGL((k_query_cone<W, FM>), dim3(n_poses), dim3(kQueryThreads), 0, s, H, field->d_merged, pts, \
                       nrm, n_points, poses, cos_hit, dom_bits, dom_count)
    if (H.W == 1) {
        if (H.F <= 3) LG_QCONE(1, 3); else if (H.F <= 4) LG_QCONE(1, 4); else if (H.F <= 5) LG_QCONE(1, 5); else LG_QCONE(1, 8);
    } else {
        if (H.F <= 3) LG_QCONE(2, 3); else if (H.F <= 4) LG_QCONE(2, 4); else if (H.F <= 5) LG_QCONE(2, 5); else LG_QCONE(2, 8);
    }
#undef LG_QCONE
    LG_HIP(hipGetLastError());
    return LG_OK;
}
