// Object preprocessing (Sec. 5.2): drop the object points where a small box
// placed on the surface penetrates the object, so that no contact is drawn
// in a hole or a crease the fingers cannot enter.  One-off per object: a
// thread per point samples a lattice of the box against the trilinear SDF,
// then one workgroup compacts the kept indices in increasing order.
#include <math.h>

#include "lg_internal.h"

namespace lg {

constexpr int kConcaveThreads = 256;
constexpr int kCompactPointThreads = 1024;
constexpr int kMaxLattice = 16;

// Duff et al. (JCGT 2017) orthonormal tangents of unit n (float)
__device__ inline void duff_tangents(float nx, float ny, float nz, float *x, float *y)
{
    const float sign = copysignf(1.0f, nz);
    const float a = -1.0f / (sign + nz);
    const float b = nx * ny * a;
    x[0] = fmaf(sign * nx * nx, a, 1.0f);
    x[1] = sign * b;
    x[2] = -sign * nx;
    y[0] = b;
    y[1] = fmaf(ny * ny, a, sign);
    y[2] = -ny;
}

// Box of edge s on the surface at point i: bottom face centred at p, axes
// (x, y, n); penetration = max over the (m+1)^3 lattice of -SDF.
__global__ void __launch_bounds__(kConcaveThreads)
k_concave_depth(SdfDev S, const float *__restrict__ pts, const float *__restrict__ nrm, int N, float s, int m,
                float max_depth, float *__restrict__ depth, uint8_t *__restrict__ keep)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const float px = pts[i], py = pts[N + i], pz = pts[2 * N + i];
    float nx = nrm[i], ny = nrm[N + i], nz = nrm[2 * N + i];
    const float rn = 1.0f / sqrtf(fmaf(nx, nx, fmaf(ny, ny, nz * nz)));
    nx *= rn;
    ny *= rn;
    nz *= rn;
    float x[3], y[3];
    duff_tangents(nx, ny, nz, x, y);
    const float step = s / (float)m, half = 0.5f * s;
    float worst = -INFINITY;
    for (int ia = 0; ia <= m; ++ia) {
        const float a = fmaf(step, (float)ia, -half);
        const float ax = fmaf(a, x[0], px), ay = fmaf(a, x[1], py), az = fmaf(a, x[2], pz);
        for (int ib = 0; ib <= m; ++ib) {
            const float b = fmaf(step, (float)ib, -half);
            const float bx = fmaf(b, y[0], ax), by = fmaf(b, y[1], ay), bz = fmaf(b, y[2], az);
            for (int ic = 0; ic <= m; ++ic) {
                const float c = step * (float)ic;
                worst = fmaxf(worst, -sdf_trilinear(S, fmaf(c, nx, bx), fmaf(c, ny, by), fmaf(c, nz, bz)));
            }
        }
    }
    depth[i] = worst;
    keep[i] = worst <= max_depth ? 1 : 0;
}

// One workgroup: contiguous runs per thread, an LDS scan of the run counts,
// then each thread writes its run's kept indices in increasing order.
__global__ void __launch_bounds__(kCompactPointThreads)
k_keep_compact(const uint8_t *__restrict__ keep, int N, int32_t *__restrict__ kept_idx, int32_t *__restrict__ n_kept)
{
    __shared__ uint32_t tot[kCompactPointThreads];
    const int tid = threadIdx.x;
    const int per = (N + kCompactPointThreads - 1) / kCompactPointThreads;
    const int beg = min(N, tid * per), end = min(N, beg + per);
    uint32_t c = 0;
    for (int i = beg; i < end; ++i) c += keep[i] ? 1u : 0u;
    tot[tid] = c;
    __syncthreads();
    for (int o = 1; o < kCompactPointThreads; o <<= 1) {
        const uint32_t v = tid >= o ? tot[tid - o] : 0u;
        __syncthreads();
        tot[tid] += v;
        __syncthreads();
    }
    uint32_t off = tot[tid] - c;
    for (int i = beg; i < end; ++i)
        if (keep[i]) kept_idx[off++] = i;
    if (tid == kCompactPointThreads - 1) n_kept[0] = (int32_t)tot[tid];
}

// columns idx[j] of the SoA points/normals; NaN for an index outside [0, N)
__global__ void __launch_bounds__(256)
k_gather_points(const float *__restrict__ pts, const float *__restrict__ nrm, int N, const int32_t *__restrict__ idx,
                int n_out, float *__restrict__ pts_out, float *__restrict__ nrm_out)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_out) return;
    const int i = idx[j];
    const bool in = i >= 0 && i < N;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        pts_out[(int64_t)c * n_out + j] = in ? pts[(int64_t)c * N + i] : __builtin_nanf("");
        nrm_out[(int64_t)c * n_out + j] = in ? nrm[(int64_t)c * N + i] : __builtin_nanf("");
    }
}

}  // namespace lg

using namespace lg;

extern "C" lg_status lg_concave_filter(const lg_sdf *sdf, const float *pts, const float *nrm, int32_t n_points,
                                       float box_edge, int32_t lattice, float max_depth, float *depth,
                                       uint8_t *keep, int32_t *kept_idx, int32_t *n_kept, void *stream)
{
    if (!sdf) return fail(LG_EINVAL, "null sdf");
    if (sdf->dims < 2 || !(sdf->h > 0.f) || !sdf->values) return fail(LG_EINVAL, "bad sdf");
    if (n_points < 0) return fail(LG_EINVAL, "n_points must be >= 0");
    if (!(box_edge > 0.f) || !isfinite(box_edge)) return fail(LG_EINVAL, "need a finite box_edge > 0");
    if (lattice < 1 || lattice > kMaxLattice) return fail(LG_EINVAL, "need 1 <= lattice <= 16");
    if (isnan(max_depth)) return fail(LG_EINVAL, "max_depth is NaN");
    if (!n_kept || (n_points > 0 && (!pts || !nrm || !depth || !keep || !kept_idx)))
        return fail(LG_EINVAL, "null device buffer");
    hipStream_t s = as_stream(stream);
    SdfDev S{sdf->origin[0], sdf->origin[1], sdf->origin[2], sdf->h, 1.0f / sdf->h, sdf->dims, sdf->values};
    if (n_points > 0)
        hipLaunchKernelGGL(k_concave_depth, dim3((unsigned)((n_points + kConcaveThreads - 1) / kConcaveThreads)),
                           dim3(kConcaveThreads), 0, s, S, pts, nrm, n_points, box_edge, lattice, max_depth, depth,
                           keep);
    hipLaunchKernelGGL(k_keep_compact, dim3(1), dim3(kCompactPointThreads), 0, s, keep, n_points, kept_idx, n_kept);
    LG_HIP(hipGetLastError());
    return LG_OK;
}

extern "C" lg_status lg_gather_points(const float *pts, const float *nrm, int32_t n_points, const int32_t *idx,
                                      int32_t n_out, float *pts_out, float *nrm_out, void *stream)
{
    if (n_points < 0 || n_out < 0) return fail(LG_EINVAL, "sizes must be >= 0");
    if (n_out == 0) return LG_OK;
    if (!pts || !nrm || !idx || !pts_out || !nrm_out) return fail(LG_EINVAL, "null device buffer");
    hipLaunchKernelGGL(k_gather_points, dim3((unsigned)((n_out + 255) / 256)), dim3(256), 0, as_stream(stream), pts,
                       nrm, n_points, idx, n_out, pts_out, nrm_out);
    LG_HIP(hipGetLastError());
    return LG_OK;
}
