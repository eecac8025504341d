// Object placement (Sec. 5.1).  Exhaustive: each pose puts a random object
// surface point onto a random contact vector of the field, normals opposed,
// with a random roll about the contact normal; the contact vector comes from
// the field's own joint sampling and forward kinematics.  Static link: with
// some probability a pose instead puts the object against the palm, and is
// rejected when the palm's capsules penetrate the object.  Thread per pose.
#include <math.h>

#include "lg_internal.h"

namespace lg {

constexpr uint32_t kPurposePlace = 11u;
constexpr uint32_t kPurposePalm = 17u;
constexpr int kPlaceThreads = 256;

__device__ inline float dot3p(const float *a, const float *b) { return fmaf(a[0], b[0], fmaf(a[1], b[1], a[2] * b[2])); }

__device__ inline void mat3_mulf(const float *A, const float *B, float *C)
{
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            C[3 * r + c] = fmaf(A[3 * r], B[c], fmaf(A[3 * r + 1], B[3 + c], A[3 * r + 2] * B[6 + c]));
}

// minimal rotation of unit a onto unit b, through the unit quaternion
// (a.h, a x h) of the bisector h = (a + b) / |a + b|: well conditioned in
// float whenever a.b > -0.9999 (|a + b| >= 0.014), unlike I + [v]x + [v]x^2 / (1 + c)
__device__ inline void rot_min(const float *a, const float *b, float *R)
{
    float h[3] = {a[0] + b[0], a[1] + b[1], a[2] + b[2]};
    const float ih = 1.0f / sqrtf(dot3p(h, h));
    h[0] *= ih;
    h[1] *= ih;
    h[2] *= ih;
    const float w = dot3p(a, h);
    const float x = a[1] * h[2] - a[2] * h[1], y = a[2] * h[0] - a[0] * h[2], z = a[0] * h[1] - a[1] * h[0];
    R[0] = 1.0f - 2.0f * (y * y + z * z);
    R[1] = 2.0f * (x * y - z * w);
    R[2] = 2.0f * (x * z + y * w);
    R[3] = 2.0f * (x * y + z * w);
    R[4] = 1.0f - 2.0f * (x * x + z * z);
    R[5] = 2.0f * (y * z - x * w);
    R[6] = 2.0f * (x * z - y * w);
    R[7] = 2.0f * (y * z + x * w);
    R[8] = 1.0f - 2.0f * (x * x + y * y);
}

// rotation taking a onto b; below c = -0.9999 a half-turn about the Duff
// x-axis of a (a -> -a) first, then the minimal rotation of -a onto b
__device__ inline void rot_align(const float *a, const float *b, float *R)
{
    const float c = dot3p(a, b);
    if (c > -0.9999f) {
        rot_min(a, b, R);
        return;
    }
    const float sign = copysignf(1.0f, a[2]);
    const float s = -1.0f / (sign + a[2]), m = a[0] * a[1] * s;
    const float x[3] = {1.0f + sign * a[0] * a[0] * s, sign * m, -sign * a[0]};
    float Rh[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) Rh[3 * r + q] = 2.0f * x[r] * x[q] - (r == q ? 1.0f : 0.0f);
    const float na[3] = {-a[0], -a[1], -a[2]};
    float Rm[9];
    rot_min(na, b, Rm);
    mat3_mulf(Rm, Rh, R);
}

// rotation R taking unit a onto unit b, then rolled by psi about b
__device__ inline void align_and_roll(const float *a, const float *b, float psi, float *R)
{
    float R0[9], Rr[9];
    rot_align(a, b, R0);
    float sn, cs;
    sincosf(psi, &sn, &cs);
    const float K[9] = {0.f, -b[2], b[1], b[2], 0.f, -b[0], -b[1], b[0], 0.f};
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) Rr[3 * r + c] = (r == c ? cs : 0.0f) + sn * K[3 * r + c] + (1.0f - cs) * b[r] * b[c];
    mat3_mulf(Rr, R0, R);
}

__global__ void __launch_bounds__(kPlaceThreads)
k_place(DevHand H, const float *__restrict__ pts, const float *__restrict__ nrm, int N, int n_poses, uint32_t seed_lo,
        uint32_t seed_hi, uint32_t request_id, int64_t pose_offset, float *__restrict__ poses)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_poses) return;
    uint32_t w[8];
    philox4x32_10((uint32_t)(pose_offset + g), 0u, kPurposePlace, request_id, seed_lo, seed_hi, w);
    philox4x32_10((uint32_t)(pose_offset + g), 1u, kPurposePlace, request_id, seed_lo, seed_hi, w + 4);
    const int f = (int)__umulhi(w[0], (uint32_t)H.F);
    const uint32_t s = __umulhi(w[1], (uint32_t)H.samples);
    const int t = (int)__umulhi(w[2], (uint32_t)H.finger_dof[f]);
    const int js = (int)__umulhi(w[3], (uint32_t)H.nsurf);
    const int i = (int)__umulhi(w[4], (uint32_t)N);
    const float psi = 6.283185307179586f * u01f(w[5]);
    // contact vector: chain of finger f up to its link t at joint sample s
    const int first = H.finger_first[f];
    Tf T;
    for (int u = 0; u <= t; ++u) T = joint_frame(H, T, u > 0, first + u, joint_sample(H, f, s, u));
    const int l = first + t;
    const float *sf = H.surf + ((int64_t)l * H.nsurf + js) * 6;
    float x[3], nu[3];
    tf_point(T, sf[0], sf[1], sf[2], x[0], x[1], x[2]);
    tf_dir(T, sf[3], sf[4], sf[5], nu[0], nu[1], nu[2]);
    float a[3] = {nrm[i], nrm[N + i], nrm[2 * N + i]};
    const float ia = 1.0f / sqrtf(dot3p(a, a));
    a[0] *= ia;
    a[1] *= ia;
    a[2] *= ia;
    const float ib = -1.0f / sqrtf(dot3p(nu, nu));
    const float b[3] = {nu[0] * ib, nu[1] * ib, nu[2] * ib};
    float R[9];
    align_and_roll(a, b, psi, R);  // roll psi about b (Rodrigues)
    const float p[3] = {pts[i], pts[N + i], pts[2 * N + i]};
    float *P = poses + 12 * (int64_t)g;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        P[4 * r + 0] = R[3 * r];
        P[4 * r + 1] = R[3 * r + 1];
        P[4 * r + 2] = R[3 * r + 2];
        P[4 * r + 3] = x[r] - fmaf(R[3 * r], p[0], fmaf(R[3 * r + 1], p[1], R[3 * r + 2] * p[2]));
    }
}

// Static-link placement: with probability prob, object point i onto palm
// contact vector js (normals opposed, roll psi); palm_pt = i when no palm
// capsule penetrates the placed object by more than margin, else -2; -1
// (pose untouched) when not selected.
__global__ void __launch_bounds__(kPlaceThreads)
k_place_palm(DevHand H, SdfDev S, const float *__restrict__ pts, const float *__restrict__ nrm, int N, int n_poses,
             float prob, float margin, uint32_t seed_lo, uint32_t seed_hi, uint32_t request_id, int64_t pose_offset,
             float *__restrict__ poses, int32_t *__restrict__ palm_pt)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_poses) return;
    uint32_t w[4];
    philox4x32_10((uint32_t)(pose_offset + g), 0u, kPurposePalm, request_id, seed_lo, seed_hi, w);
    if (!(u01f(w[0]) < prob)) {
        palm_pt[g] = -1;
        return;
    }
    const int js = (int)__umulhi(w[1], (uint32_t)H.n_palm_surf);
    const int i = (int)__umulhi(w[2], (uint32_t)N);
    const float psi = 6.283185307179586f * u01f(w[3]);
    const float *sf = H.palm_surf + 6 * (int64_t)js;
    const float ib = -1.0f / sqrtf(dot3p(sf + 3, sf + 3));
    const float b[3] = {sf[3] * ib, sf[4] * ib, sf[5] * ib};
    float a[3] = {nrm[i], nrm[N + i], nrm[2 * N + i]};
    const float ia = 1.0f / sqrtf(dot3p(a, a));
    a[0] *= ia;
    a[1] *= ia;
    a[2] *= ia;
    float R[9];
    align_and_roll(a, b, psi, R);
    const float p[3] = {pts[i], pts[N + i], pts[2 * N + i]};
    float t[3];
    float *P = poses + 12 * (int64_t)g;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        t[r] = sf[r] - fmaf(R[3 * r], p[0], fmaf(R[3 * r + 1], p[1], R[3 * r + 2] * p[2]));
        P[4 * r + 0] = R[3 * r];
        P[4 * r + 1] = R[3 * r + 1];
        P[4 * r + 2] = R[3 * r + 2];
        P[4 * r + 3] = t[r];
    }
    // the palm's capsules against the placed object (object frame: R^T (x - t))
    float depth = -INFINITY;
    for (int c = 0; c < H.n_palm_caps; ++c) {
        const float *cp = H.palm_caps + 7 * c;
        const int M = H.axis_samples[H.J + c];
        const float inv = 1.0f / (float)(M - 1);
        for (int s = 0; s < M; ++s) {
            const float u = (float)s * inv;
            const float x0 = fmaf(u, cp[3] - cp[0], cp[0]) - t[0];
            const float x1 = fmaf(u, cp[4] - cp[1], cp[1]) - t[1];
            const float x2 = fmaf(u, cp[5] - cp[2], cp[2]) - t[2];
            const float y0 = fmaf(R[0], x0, fmaf(R[3], x1, R[6] * x2));
            const float y1 = fmaf(R[1], x0, fmaf(R[4], x1, R[7] * x2));
            const float y2 = fmaf(R[2], x0, fmaf(R[5], x1, R[8] * x2));
            depth = fmaxf(depth, cp[6] - sdf_trilinear(S, y0, y1, y2));
        }
    }
    palm_pt[g] = depth <= margin ? i : -2;
}

}  // namespace lg

using namespace lg;

extern "C" lg_status lg_place_palm(const lg_field *field, const lg_sdf *sdf, const float *pts, const float *nrm,
                                   int32_t n_points, int32_t n_poses, float prob, float margin, uint64_t seed,
                                   uint32_t request_id, int64_t pose_offset, float *poses, int32_t *palm_pt,
                                   void *stream)
{
    if (!field || !sdf) return fail(LG_EINVAL, "null field or sdf");
    const DevHand &H = field->dh;
    if (H.n_palm_surf <= 0) return fail(LG_EINVAL, "the hand has no palm contact vectors");
    if (sdf->dims < 2 || !(sdf->h > 0.f) || !sdf->values) return fail(LG_EINVAL, "bad sdf");
    if (n_points <= 0 || n_poses < 0) return fail(LG_EINVAL, "need n_points > 0 and n_poses >= 0");
    if (!(prob >= 0.0f && prob <= 1.0f) || isnan(margin)) return fail(LG_EINVAL, "need 0 <= prob <= 1, margin not NaN");
    if (n_poses == 0) return LG_OK;
    if (!pts || !nrm || !poses || !palm_pt) return fail(LG_EINVAL, "null device buffer");
    SdfDev S{sdf->origin[0], sdf->origin[1], sdf->origin[2], sdf->h, 1.0f / sdf->h, sdf->dims, sdf->values};
    hipLaunchKernelGGL(k_place_palm, dim3((unsigned)((n_poses + kPlaceThreads - 1) / kPlaceThreads)),
                       dim3(kPlaceThreads), 0, as_stream(stream), H, S, pts, nrm, n_points, n_poses, prob, margin,
                       (uint32_t)seed, (uint32_t)(seed >> 32), request_id, pose_offset, poses, palm_pt);
    LG_HIP(hipGetLastError());
    return LG_OK;
}

extern "C" lg_status lg_place_exhaustive(const lg_field *field, const float *pts, const float *nrm, int32_t n_points,
                                         int32_t n_poses, uint64_t seed, uint32_t request_id, int64_t pose_offset,
                                         float *poses, void *stream)
{
    if (!field) return fail(LG_EINVAL, "null field");
    if (n_points <= 0 || n_poses < 0) return fail(LG_EINVAL, "need n_points > 0 and n_poses >= 0");
    if (n_poses == 0) return LG_OK;
    if (!pts || !nrm || !poses) return fail(LG_EINVAL, "null device buffer");
    const DevHand &H = field->dh;
    if (H.samples <= 0 || H.samples > 0xffffffffLL) return fail(LG_EUNSUPPORTED, "joint samples must fit 32 bits");
    hipLaunchKernelGGL(k_place, dim3((unsigned)((n_poses + kPlaceThreads - 1) / kPlaceThreads)), dim3(kPlaceThreads),
                       0, as_stream(stream), H, pts, nrm, n_points, n_poses, (uint32_t)seed, (uint32_t)(seed >> 32),
                       request_id, pose_offset, poses);
    LG_HIP(hipGetLastError());
    return LG_OK;
}
