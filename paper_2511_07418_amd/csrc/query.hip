// Object contact query (Sec. 4.2-4.3, Def. 4.3) with the per-dependency-group
// merge of Sec. 5.3.
//
// One workgroup per pose; each wave sweeps 64 consecutive object points
// (structure-of-arrays).  Per point: the query normal -R n and its bin, the
// point's voxel in each finger window, one 4-byte gather per finger from the
// plane of its merged table that holds the bin, and a wave ballot that yields
// the 64 domain bits of the finger for the chunk.  Counts are popcounts of
// the ballots.
//
// Windows in lattice form (a shared rotation, origins a whole number of
// 4-voxel bricks apart) take one affine map per point instead of one per
// finger: the point's lattice cell is packed as x | y << 10 | z << 20, and
// finger f's in-window test is one subtraction of its packed offset and one
// mask (a field that went negative or reached G sets a bit of lat_hi).  The
// bricked table word is linear in the cell, so one per-point byte offset
// serves every finger, each finger's offset folded into its scalar base.
//
// With chunk bounds (a bounding sphere per 64 consecutive points, a one-level
// bounding-volume hierarchy over the object; tight when the points are in
// Morton order), a (chunk, finger) pair whose sphere misses the finger's
// window is skipped: its 64 domain bits are zero without a lookup, and a
// chunk that misses every window is not loaded at all.
#include <math.h>

#include <algorithm>
#include <utility>
#include <vector>

#include "lg_internal.h"

namespace lg {

constexpr int kQueryThreads = 256;
constexpr int kQueryWaves = kQueryThreads / 64;
constexpr float kCullMargin = 1e-3f;  // voxels added to a chunk's radius (float rounding is ~1e-4)

// the LLVM writelane intrinsic: lane `lane` (uniform) of v replaced by the uniform x
extern "C" __device__ int lg_writelane(int x, int lane, int v) __asm("llvm.amdgcn.writelane");
__device__ inline uint32_t write_lane(uint32_t v, uint32_t x, int lane)
{
    return (uint32_t)lg_writelane((int)x, lane, (int)v);
}

// Bounding sphere (centre of the box, largest distance) of each chunk of 64
// consecutive points; one wave per chunk, radius padded for rounding.
__global__ void __launch_bounds__(256)
k_chunk_bounds(const float *__restrict__ pts, int N, float4 *__restrict__ bounds)
{
    const int nchunks = (N + 63) >> 6;
    const int chunk = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (chunk >= nchunks) return;  // uniform per wave
    const int i = min(chunk * 64 + lane, N - 1);  // lanes past N repeat the last point
    const float x = pts[i], y = pts[N + i], z = pts[2 * N + i];
    float lo[3] = {x, y, z}, hi[3] = {x, y, z};
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], __shfl_xor(lo[a], off, 64));
            hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], off, 64));
        }
    const float cx = 0.5f * (lo[0] + hi[0]), cy = 0.5f * (lo[1] + hi[1]), cz = 0.5f * (lo[2] + hi[2]);
    const float dx = x - cx, dy = y - cy, dz = z - cz;
    float r = sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
    for (int off = 32; off > 0; off >>= 1) r = fmaxf(r, __shfl_xor(r, off, 64));
    if (lane == 0) bounds[chunk] = make_float4(cx, cy, cz, fmaf(r, 1e-5f, r + 1e-7f));
}

// skip[f] bit j: chunk blk * 32 + j cannot reach finger f's window (all 0
// without bounds); returns the chunks that reach no window.  Lane l tests
// chunk l % 32 against finger f0 + l / 32, two fingers per ballot: the distance
// from the sphere's centre (voxel coordinates of map aff[LAT ? 0 : f]) to the
// finger's window box [lo, lo + G]^3 against its radius; lo = G for a
// finger's own (biased) map, lat_o[f] in lattice coordinates.
template <int FM, bool LAT>
__device__ inline uint32_t block_skip(const float4 *__restrict__ bounds, const Affine *aff, const DevHand &H,
                                      int blk, int nchunks, int lane, uint32_t (&skip)[FM])
{
    const int F = H.F, G = H.G;
#pragma unroll
    for (int f = 0; f < FM; ++f) skip[f] = 0u;
    if (!bounds) return 0u;
#pragma unroll
    for (int f0 = 0; f0 < FM; f0 += 2) {
        if (f0 >= F) break;
        const int f = min(f0 + (lane >> 5), F - 1);
        const int ch = blk * 32 + (lane & 31);
        bool out = true;
        if (ch < nchunks) {
            const float4 sb = bounds[ch];
            const Affine &a = aff[LAT ? 0 : f];
            const float ux = fmaf(a.m[0], sb.x, fmaf(a.m[1], sb.y, fmaf(a.m[2], sb.z, a.m[3])));
            const float uy = fmaf(a.m[4], sb.x, fmaf(a.m[5], sb.y, fmaf(a.m[6], sb.z, a.m[7])));
            const float uz = fmaf(a.m[8], sb.x, fmaf(a.m[9], sb.y, fmaf(a.m[10], sb.z, a.m[11])));
            const float lx = LAT ? (float)H.lat_o[f][0] : (float)G, ly = LAT ? (float)H.lat_o[f][1] : (float)G,
                        lz = LAT ? (float)H.lat_o[f][2] : (float)G;
            const float dx = fmaxf(fmaxf(lx - ux, ux - (lx + G)), 0.f);
            const float dy = fmaxf(fmaxf(ly - uy, uy - (ly + G)), 0.f);
            const float dz = fmaxf(fmaxf(lz - uz, uz - (lz + G)), 0.f);
            const float rv = fmaf(sb.w, H.inv_h, kCullMargin);
            out = fmaf(dx, dx, fmaf(dy, dy, dz * dz)) > rv * rv;
        }
        const unsigned long long m = __ballot(out);
        skip[f0] = (uint32_t)m;
        if (f0 + 1 < FM) skip[f0 + 1] = (uint32_t)(m >> 32);
    }
    uint32_t all = ~0u;
#pragma unroll
    for (int f = 0; f < FM; ++f)
        if (f < F) all &= skip[f];
    return all;
}

// argmax_b <d, c_b> (ties to the lowest b, as nearest_bin) through the
// cube-map candidate table: the four candidate slots of the direction's cell
// (absent ones repeat the first, so the result is unchanged) are evaluated
// without a branch.  Their centres are float4 rows in LDS, all four read
// before the first dot product.  A cell with more than four candidates scans
// every bin.
__device__ inline int nearest_bin_lut4(const uint32_t *lut, const float4 *c4, int B, float dx, float dy, float dz)
{
    // face and face coordinates by the cube-map instructions (the table is
    // built in their convention): ma = 2 x the major component, so
    // (sc / |major| + 1) R / 2 = sc R / |ma| + R / 2
    const int face = (int)__builtin_amdgcn_cubeid(dx, dy, dz);
    const float sc = __builtin_amdgcn_cubesc(dx, dy, dz), tc = __builtin_amdgcn_cubetc(dx, dy, dz);
    const float sf = (float)kLutRes * __builtin_amdgcn_rcpf(fabsf(__builtin_amdgcn_cubema(dx, dy, dz)));
    const int is = min(max((int)fmaf(sc, sf, 0.5f * kLutRes), 0), kLutRes - 1);
    const int it = min(max((int)fmaf(tc, sf, 0.5f * kLutRes), 0), kLutRes - 1);
    // byte offset of the entry; the row by a 24-bit multiply (full rate; the
    // compiler would otherwise pick the quarter-rate 32-bit multiply)
    uint32_t row;
    asm("v_mul_u32_u24 %0, %1, %2" : "=v"(row) : "n"(4 * kLutRes), "v"((uint32_t)(face * kLutRes + it)));
    const uint32_t boff = row + ((uint32_t)is << 2);
    const uint32_t e = *reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(lut) + boff);
    float best = -3.0e38f;
    int bi = 0;
    if (e == 0xffffffffu) {  // more than four candidates: every bin
        for (int b = 0; b < B; ++b) {
            const float4 c = c4[b];
            const float sc = fmaf(c.x, dx, fmaf(c.y, dy, c.z * dz));
            if (sc > best) {
                best = sc;
                bi = b;
            }
        }
        return bi;
    }
    // byte offsets (bin * 16) of the four slots' float4 centres
    const uint32_t off[4] = {(e << 4) & 0xff0u, (e >> 4) & 0xff0u, (e >> 12) & 0xff0u, (e >> 20) & 0xff0u};
    float4 ck[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) ck[k] = *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(c4) + off[k]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float sc = fmaf(ck[k].x, dx, fmaf(ck[k].y, dy, ck[k].z * dz));
        if (sc > best) {
            best = sc;
            bi = (int)(off[k] >> 4);
        }
    }
    return bi;
}

// LDS of one query block
template <int FM, bool LAT>
struct QueryLds {
    float4 cb4[kMaxBins];
    uint32_t lut[6 * kLutRes * kLutRes];
    Affine aff[LAT ? 1 : FM];
    uint32_t cnt[FM][kQueryWaves];
};

// the domains of pose g (one block)
template <int W, int FM, bool LAT>
__device__ __forceinline__ void query_pose(QueryLds<FM, LAT> &L, const DevHand &H, const uint32_t *__restrict__ merged,
                                           const float *__restrict__ pts, const float *__restrict__ nrm, int N,
                                           const float *__restrict__ poses, const float4 *__restrict__ bounds,
                                           uint32_t *__restrict__ dom_bits, uint32_t *__restrict__ dom_count, int g)
{
    float4 *cb4 = L.cb4;
    uint32_t *lut = L.lut;
    Affine *aff = L.aff;
    auto &cnt = L.cnt;
    const float *pose = poses + 12 * (int64_t)g;
    for (int i = threadIdx.x; i < H.B; i += kQueryThreads)
        cb4[i] = make_float4(H.bin_c[3 * i], H.bin_c[3 * i + 1], H.bin_c[3 * i + 2], 0.0f);
    for (int i = threadIdx.x; i < 6 * kLutRes * kLutRes; i += kQueryThreads) lut[i] = H.bin_lut[i];
    if (LAT) {
        if (threadIdx.x == 0) aff[0] = lattice_affine(H, pose);
    } else if (threadIdx.x < H.F) {
        aff[threadIdx.x] = finger_affine(H, pose, threadIdx.x);
    }
    __syncthreads();
    // the wave index is uniform: in a scalar register, the block and chunk
    // bookkeeping (and the skip tests) stay on the scalar unit
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int F = H.F, G = H.G, B = H.B;
    const uint32_t GB = (uint32_t)(G >> 2), G3 = (uint32_t)G * G * G;
    // Byte offset of finger f's table less (lattice form) the word of its
    // window origin, or (general form) of the +G bias of each coordinate, so
    // that it plus 4 * (word of the point's cell) addresses the finger's word.
    // The sum is taken in 32 bits: it wraps to the right offset for every
    // lane inside the window (the tables are far below 4 GiB).
    const char *mbase = reinterpret_cast<const char *>(merged);
    uint32_t koff[FM];
#pragma unroll
    for (int f = 0; f < FM; ++f)
        koff[f] = 4u * ((uint32_t)f * W * G3 - (LAT ? H.lat_idx[f < F ? f : 0] : brick_word(G, G, G, GB)));
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
        uint32_t skip[FM];
        const uint32_t skip_all = block_skip<FM, LAT>(bounds, aff, H, blk, nchunks, lane, skip);
        for (int chunk = blk * 32; chunk < c_end; ++chunk) {
            const uint32_t cbit = 1u << (chunk - blk * 32);
            if (skip_all & cbit) continue;  // no window in reach: its ballot words stay 0
            // re-read the maps from LDS every chunk instead of pinning their
            // registers for the whole sweep
            asm volatile("" ::: "memory");
            const int i = chunk * 64 + lane;
            const bool valid = i < N;
            // lanes past N read the last point (in bounds, no branch); they
            // are outside every window through `valid`
            const uint32_t il = (uint32_t)min(i, N - 1);
            const char *pb = reinterpret_cast<const char *>(pts), *nb = reinterpret_cast<const char *>(nrm);
            const uint32_t o0 = il << 2, o1 = o0 + ((uint32_t)N << 2), o2 = o1 + ((uint32_t)N << 2);
            const float px = *reinterpret_cast<const float *>(pb + o0);
            const float py = *reinterpret_cast<const float *>(pb + o1);
            const float pz = *reinterpret_cast<const float *>(pb + o2);
            const float nx = *reinterpret_cast<const float *>(nb + o0);
            const float ny = *reinterpret_cast<const float *>(nb + o1);
            const float nz = *reinterpret_cast<const float *>(nb + o2);
            float qx, qy, qz;
            query_dir(P, nx, ny, nz, qx, qy, qz);
            const int b = nearest_bin_lut4(lut, cb4, B, qx, qy, qz);
            const uint32_t plane = W == 2 ? __umul24((uint32_t)(b >> 5), G3) : 0u;
            uint32_t word[FM];  // 0 outside the window
            uint32_t voff = 0, ip = 0;
            if (LAT) {
                int Ix, Iy, Iz;
                lattice_cell(aff[0], px, py, pz, Ix, Iy, Iz);
                Ix = min(max(Ix, 0), 1023);
                Iy = min(max(Iy, 0), 1023);
                Iz = min(max(Iz, 0), 1023);
                ip = (uint32_t)Ix | (uint32_t)Iy << 10 | (uint32_t)Iz << 20;
                voff = (brick_word_u24((uint32_t)Ix, (uint32_t)Iy, (uint32_t)Iz, GB) + plane) << 2;
                asm volatile("" : "+v"(voff));  // one add per finger below, not a re-associated pair
            }
            // all finger gathers are issued before any is consumed
#pragma unroll
            for (int f = 0; f < FM; ++f) {
                word[f] = 0u;
                if (f < F && !(skip[f] & cbit)) {
                    uint32_t off;
                    bool in;
                    if (LAT) {
                        in = ((int)valid & (int)(((ip - H.lat_pk[f]) & H.lat_hi) == 0u)) != 0;
                        off = voff;
                    } else {
                        // biased window coordinates (see window_voxel): inside iff all in [G, 2G)
                        const Affine &a = aff[f];
                        const float ux = fmaf(a.m[0], px, fmaf(a.m[1], py, fmaf(a.m[2], pz, a.m[3])));
                        const float uy = fmaf(a.m[4], px, fmaf(a.m[5], py, fmaf(a.m[6], pz, a.m[7])));
                        const float uz = fmaf(a.m[8], px, fmaf(a.m[9], py, fmaf(a.m[10], pz, a.m[11])));
                        const int Ix = (int)ux, Iy = (int)uy, Iz = (int)uz;
                        in = ((int)valid & (int)(min(Ix, min(Iy, Iz)) >= G) & (int)(max(Ix, max(Iy, Iz)) < 2 * G)) != 0;
                        off = (brick_word_u24((uint32_t)Ix, (uint32_t)Iy, (uint32_t)Iz, GB) + plane) << 2;
                    }
                    if (in) word[f] = *reinterpret_cast<const uint32_t *>(mbase + (off + koff[f]));
                }
            }
            const int j2 = 2 * (chunk - blk * 32);
#pragma unroll
            for (int f = 0; f < FM; ++f) {
                if (f >= F) break;
                if (skip[f] & cbit) continue;  // the ballot would be 0
                const bool hit = ((word[f] >> (b & 31)) & 1u) != 0u;
                const unsigned long long m = __ballot(hit);
                // the chunk's two ballot halves into lanes j2, j2 + 1 (j2 is uniform)
                acc[f] = write_lane(acc[f], (uint32_t)m, j2);
                acc[f] = write_lane(acc[f], (uint32_t)(m >> 32), j2 + 1);
            }
        }
        const int wi = blk * 64 + lane;
        if (wi < NW) {
#pragma unroll
            for (int f = 0; f < FM; ++f)
                if (f < F) dom_bits[((int64_t)g * F + f) * NW + wi] = acc[f];
        }
        // counts per lane from the block's words (bits past N are 0)
#pragma unroll
        for (int f = 0; f < FM; ++f) c[f] += (uint32_t)__popc(acc[f]);
    }
#pragma unroll
    for (int f = 0; f < FM; ++f)
        for (int off = 32; off > 0; off >>= 1) c[f] += __shfl_xor(c[f], off, 64);
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

template <int W, int FM, bool LAT>
__global__ void __launch_bounds__(kQueryThreads) __attribute__((amdgpu_waves_per_eu(8, 8)))
k_query(DevHand H, const uint32_t *__restrict__ merged, const float *__restrict__ pts,
        const float *__restrict__ nrm, int N, const float *__restrict__ poses, const float4 *__restrict__ bounds,
        uint32_t *__restrict__ dom_bits, uint32_t *__restrict__ dom_count)
{
    __shared__ QueryLds<FM, LAT> L;
    query_pose<W, FM, LAT>(L, H, merged, pts, nrm, N, poses, bounds, dom_bits, dom_count, blockIdx.x);
}

// The same over the poses of several chunks (one block per pose).
template <int W, int FM, bool LAT>
__global__ void __launch_bounds__(kQueryThreads) __attribute__((amdgpu_waves_per_eu(8, 8)))
k_query_batch(const ChunkDesc *__restrict__ d, const uint16_t *__restrict__ idx, const uint32_t *__restrict__ first,
              int n)
{
    __shared__ QueryLds<FM, LAT> L;
    const int j = batch_member(first, n, blockIdx.x);
    const ChunkDesc &c = d[idx[j]];
    query_pose<W, FM, LAT>(L, c.H, c.merged, c.pts, c.nrm, c.N, c.poses, c.bounds, c.dom_bits, c.dom_count,
                           (int)(blockIdx.x - first[j]));
}

// Cone query (Sec. 4.3's theta_hit test): a query (x, -R n) hits finger f if
// a bin b set in the finger's merged word(s) at voxel(x) has c_b . q >= cos_hit.
// Same sweep and block stores as k_query.  Per point the cone is built once as
// a bin mask over the bins of its polar band that some finger's entry holds;
// each finger's test is then one AND with its entry.
template <int W, int FM>
__global__ void __launch_bounds__(kQueryThreads)
k_query_cone(DevHand H, const uint32_t *__restrict__ merged, const float *__restrict__ pts,
             const float *__restrict__ nrm, int N, const float *__restrict__ poses, const float4 *__restrict__ bounds,
             float cos_hit, uint32_t *__restrict__ dom_bits, uint32_t *__restrict__ dom_count)
{
    __shared__ float cb[3 * kMaxBins];
    __shared__ Affine aff[FM];
    __shared__ uint32_t cnt[FM][kQueryWaves];
    const int g = blockIdx.x;
    const float *pose = poses + 12 * (int64_t)g;
    for (int i = threadIdx.x; i < 3 * H.B; i += blockDim.x) cb[i] = H.bin_c[i];
    if (threadIdx.x < H.F) aff[threadIdx.x] = finger_affine(H, pose, threadIdx.x);
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int F = H.F, G = H.G, B = H.B;
    const float sin_hit = sqrtf(fmaxf(0.f, fmaf(-cos_hit, cos_hit, 1.f)));
    const uint32_t GB = (uint32_t)(G >> 2), G3 = (uint32_t)G * G * G;
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
        uint32_t skip[FM];
        const uint32_t skip_all = block_skip<FM, false>(bounds, aff, H, blk, nchunks, lane, skip);
        for (int chunk = blk * 32; chunk < c_end; ++chunk) {
            const uint32_t cbit = 1u << (chunk - blk * 32);
            if (skip_all & cbit) continue;  // no window in reach: its ballot words stay 0
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
            // bins that can lie within the cone: the polar band |phi_b - phi_q| <=
            // theta_hit, a contiguous index range of the Fibonacci lattice (z_b =
            // 1 - (2b + 1) / B decreases with b), widened by one bin for rounding
            const float sq = sqrtf(fmaxf(0.f, fmaf(-qz, qz, 1.f)));
            const float zhi = qz >= cos_hit ? 1.f : fmaf(qz, cos_hit, sq * sin_hit);
            const float zlo = qz <= -cos_hit ? -1.f : fmaf(qz, cos_hit, -sq * sin_hit);
            const int blo = max(0, (int)floorf(0.5f * fmaf((float)B, 1.f - zhi, -1.f)) - 1);
            const int bhi = min(B - 1, (int)ceilf(0.5f * fmaf((float)B, 1.f - zlo, -1.f)) + 1);
            const unsigned long long band = blo > bhi ? 0ull
                                                      : ((bhi - blo == 63 ? ~0ull : ((1ull << (bhi - blo + 1)) - 1ull))
                                                         << blo);
            unsigned long long ent[FM];
#pragma unroll
            for (int f = 0; f < FM; ++f) {
                ent[f] = 0ull;
                if (f < F && !(skip[f] & cbit)) {
                    // biased window coordinates (see window_voxel): inside iff all in [G, 2G)
                    const Affine &a = aff[f];
                    const float ux = fmaf(a.m[0], px, fmaf(a.m[1], py, fmaf(a.m[2], pz, a.m[3])));
                    const float uy = fmaf(a.m[4], px, fmaf(a.m[5], py, fmaf(a.m[6], pz, a.m[7])));
                    const float uz = fmaf(a.m[8], px, fmaf(a.m[9], py, fmaf(a.m[10], pz, a.m[11])));
                    const unsigned ix = (unsigned)((int)ux - G), iy = (unsigned)((int)uy - G),
                                   iz = (unsigned)((int)uz - G);
                    if (valid && max(ix, max(iy, iz)) < (unsigned)G) {
                        const uint32_t *tab = merged + (int64_t)f * W * G3;
                        const uint32_t wv = brick_word(ix, iy, iz, GB);
                        ent[f] = tab[wv];
                        if (W == 2) ent[f] |= (unsigned long long)tab[G3 + wv] << 32;
                    }
                }
            }
            const int j2 = 2 * (chunk - blk * 32);
            // the point's cone as a bin mask over the band's bins that some
            // finger's entry holds (the per-finger test is then one AND)
            unsigned long long cone = 0ull;
            {
                unsigned long long u = 0ull;
#pragma unroll
                for (int f = 0; f < FM; ++f) u |= ent[f];
                unsigned long long m = u & band;
                while (m) {
                    const int b = __ffsll((long long)m) - 1;
                    m &= m - 1ull;
                    if (fmaf(cb[3 * b], qx, fmaf(cb[3 * b + 1], qy, cb[3 * b + 2] * qz)) >= cos_hit) cone |= 1ull << b;
                }
            }
#pragma unroll
            for (int f = 0; f < FM; ++f) {
                if (f >= F) break;
                if (skip[f] & cbit) continue;  // the ballot would be 0
                const bool hit = (ent[f] & cone) != 0ull;
                const unsigned long long bm = __ballot(hit);
                acc[f] = write_lane(acc[f], (uint32_t)bm, j2);
                acc[f] = write_lane(acc[f], (uint32_t)(bm >> 32), j2 + 1);
            }
        }
        const int wi = blk * 64 + lane;
        if (wi < NW) {
#pragma unroll
            for (int f = 0; f < FM; ++f)
                if (f < F) dom_bits[((int64_t)g * F + f) * NW + wi] = acc[f];
        }
#pragma unroll
        for (int f = 0; f < FM; ++f) c[f] += (uint32_t)__popc(acc[f]);
    }
#pragma unroll
    for (int f = 0; f < FM; ++f)
        for (int off = 32; off > 0; off >>= 1) c[f] += __shfl_xor(c[f], off, 64);
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

static lg_status query_domains(const lg_field *field, const float *pts, const float *nrm, int32_t n_points,
                               const float *poses, int32_t n_poses, const float4 *bounds, uint32_t *dom_bits,
                               uint32_t *dom_count, void *stream)
{
    if (!field) return fail(LG_EINVAL, "null field");
    if (n_points < 0 || n_poses < 0) return fail(LG_EINVAL, "negative size");
    if (n_poses == 0) return LG_OK;
    if (!poses || !dom_count || (n_points > 0 && (!pts || !nrm || !dom_bits)))
        return fail(LG_EINVAL, "null device buffer");
    if ((int64_t)n_points * 12 > 0xffffffffLL)
        return fail(LG_EUNSUPPORTED, "n_points above 357,913,941 (32-bit byte offsets into the point rows)");
    hipStream_t s = as_stream(stream);
    const DevHand &H = field->dh;
#define LG_QUERY(W, FM, LAT)                                                                                 \
    hipLaunchKernelGGL((k_query<W, FM, LAT>), dim3(n_poses), dim3(kQueryThreads), 0, s, H, field->d_merged, pts, \
                       nrm, n_points, poses, bounds, dom_bits, dom_count)
#define LG_QUERY_F(W, LAT)                                                                                   \
    if (H.F <= 3) LG_QUERY(W, 3, LAT); else if (H.F <= 4) LG_QUERY(W, 4, LAT);                               \
    else if (H.F <= 5) LG_QUERY(W, 5, LAT); else LG_QUERY(W, 8, LAT)
    if (H.lat) {
        if (H.W == 1) { LG_QUERY_F(1, true); } else { LG_QUERY_F(2, true); }
    } else {
        if (H.W == 1) { LG_QUERY_F(1, false); } else { LG_QUERY_F(2, false); }
    }
#undef LG_QUERY_F
#undef LG_QUERY
    LG_HIP(hipGetLastError());
    return LG_OK;
}

extern "C" lg_status lg_query_domains(const lg_field *field, const float *pts, const float *nrm, int32_t n_points,
                                      const float *poses, int32_t n_poses, uint32_t *dom_bits, uint32_t *dom_count,
                                      void *stream)
{
    return query_domains(field, pts, nrm, n_points, poses, n_poses, nullptr, dom_bits, dom_count, stream);
}

extern "C" lg_status lg_query_domains_bounded(const lg_field *field, const float *pts, const float *nrm,
                                              int32_t n_points, const float *poses, int32_t n_poses,
                                              const float *bounds, uint32_t *dom_bits, uint32_t *dom_count,
                                              void *stream)
{
    if (n_points > 0 && n_poses > 0 && !bounds) return fail(LG_EINVAL, "null chunk bounds");
    if (reinterpret_cast<uintptr_t>(bounds) % 16 != 0) return fail(LG_EINVAL, "chunk bounds must be 16-byte aligned");
    return query_domains(field, pts, nrm, n_points, poses, n_poses, reinterpret_cast<const float4 *>(bounds),
                         dom_bits, dom_count, stream);
}

lg_status lg::query_batch(const BatchLaunch &b, int W, int F, bool lat, hipStream_t s)
{
    if (b.n <= 0 || b.blocks == 0) return LG_OK;
#define LG_QUERY(W_, FM, LAT)                                                                                \
    hipLaunchKernelGGL((k_query_batch<W_, FM, LAT>), dim3(b.blocks), dim3(kQueryThreads), 0, s, b.d, b.idx,  \
                       b.first, b.n)
#define LG_QUERY_F(W_, LAT)                                                                                  \
    if (F <= 3) LG_QUERY(W_, 3, LAT); else if (F <= 4) LG_QUERY(W_, 4, LAT);                                 \
    else if (F <= 5) LG_QUERY(W_, 5, LAT); else LG_QUERY(W_, 8, LAT)
    if (lat) {
        if (W == 1) { LG_QUERY_F(1, true); } else { LG_QUERY_F(2, true); }
    } else {
        if (W == 1) { LG_QUERY_F(1, false); } else { LG_QUERY_F(2, false); }
    }
#undef LG_QUERY_F
#undef LG_QUERY
    LG_HIP(hipGetLastError());
    return LG_OK;
}

extern "C" lg_status lg_chunk_bounds(const float *pts, int32_t n_points, float *bounds, void *stream)
{
    if (n_points < 0) return fail(LG_EINVAL, "negative size");
    if (n_points == 0) return LG_OK;
    if (!pts || !bounds) return fail(LG_EINVAL, "null device buffer");
    if (reinterpret_cast<uintptr_t>(bounds) % 16 != 0) return fail(LG_EINVAL, "chunk bounds must be 16-byte aligned");
    const int nchunks = (n_points + 63) / 64;
    hipLaunchKernelGGL(k_chunk_bounds, dim3((unsigned)((nchunks + 3) / 4)), dim3(256), 0, as_stream(stream), pts,
                       n_points, reinterpret_cast<float4 *>(bounds));
    LG_HIP(hipGetLastError());
    return LG_OK;
}

// Morton (Z-order) permutation of host points: 10 bits per axis over the
// points' bounding cube, bits interleaved x, y, z from the lowest; ties keep
// the input order.
extern "C" lg_status lg_morton_order(const float *pts_host, int32_t n_points, int32_t *perm_host)
{
    if (n_points < 0) return fail(LG_EINVAL, "negative size");
    if (n_points == 0) return LG_OK;
    if (!pts_host || !perm_host) return fail(LG_EINVAL, "null host buffer");
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = 0; i < n_points; ++i)
        for (int a = 0; a < 3; ++a) {
            const double v = pts_host[3 * i + a];
            if (!std::isfinite(v)) return fail(LG_EINVAL, "non-finite point");
            lo[a] = std::min(lo[a], v);
            hi[a] = std::max(hi[a], v);
        }
    const double ext = std::max(std::max(hi[0] - lo[0], hi[1] - lo[1]), std::max(hi[2] - lo[2], 1e-30));
    std::vector<std::pair<uint32_t, int32_t>> key((size_t)n_points);
    for (int i = 0; i < n_points; ++i) {
        uint32_t code = 0;
        for (int a = 0; a < 3; ++a) {
            const uint32_t q = (uint32_t)std::min(1023.0, std::max(0.0, (pts_host[3 * i + a] - lo[a]) / ext * 1023.0));
            for (int b = 0; b < 10; ++b) code |= ((q >> b) & 1u) << (3 * b + a);
        }
        key[(size_t)i] = {code, i};
    }
    std::stable_sort(key.begin(), key.end(),
                     [](const std::pair<uint32_t, int32_t> &x, const std::pair<uint32_t, int32_t> &y) {
                         return x.first < y.first;
                     });
    for (int i = 0; i < n_points; ++i) perm_host[i] = key[(size_t)i].second;
    return LG_OK;
}

extern "C" lg_status lg_query_domains_cone(const lg_field *field, const float *pts, const float *nrm, int32_t n_points,
                                           const float *poses, int32_t n_poses, const float *bounds, float cos_hit,
                                           uint32_t *dom_bits, uint32_t *dom_count, void *stream)
{
    if (!field) return fail(LG_EINVAL, "null field");
    if (reinterpret_cast<uintptr_t>(bounds) % 16 != 0) return fail(LG_EINVAL, "chunk bounds must be 16-byte aligned");
    if (n_points < 0 || n_poses < 0) return fail(LG_EINVAL, "negative size");
    if (!(cos_hit >= -1.0f && cos_hit <= 1.0f)) return fail(LG_EINVAL, "cos_hit outside [-1, 1]");
    if (n_poses == 0) return LG_OK;
    if (!poses || !dom_count || (n_points > 0 && (!pts || !nrm || !dom_bits)))
        return fail(LG_EINVAL, "null device buffer");
    hipStream_t s = as_stream(stream);
    const DevHand &H = field->dh;
#define LG_QCONE(W, FM)                                                                                        \
    hipLaunchKernelGGL((k_query_cone<W, FM>), dim3(n_poses), dim3(kQueryThreads), 0, s, H, field->d_merged, pts, \
                       nrm, n_points, poses, reinterpret_cast<const float4 *>(bounds), cos_hit, dom_bits, dom_count)
    if (H.W == 1) {
        if (H.F <= 3) LG_QCONE(1, 3); else if (H.F <= 4) LG_QCONE(1, 4); else if (H.F <= 5) LG_QCONE(1, 5); else LG_QCONE(1, 8);
    } else {
        if (H.F <= 3) LG_QCONE(2, 3); else if (H.F <= 4) LG_QCONE(2, 4); else if (H.F <= 5) LG_QCONE(2, 5); else LG_QCONE(2, 8);
    }
#undef LG_QCONE
    LG_HIP(hipGetLastError());
    return LG_OK;
}
