// Kinematics optimisation (Sec. 5.5, Eq. 7-8, Phase I and II) and the
// penetration part of the validity criterion (Sec. 3.2), fused in one kernel.
//
// Lane layout: F lanes per accepted set, lane f realises finger f, so a wave
// covers 64 / F sets (the 64 mod F lanes left over idle) and the set-level
// reductions (max depth, worst contact error / angle) read the set's lanes
// with shuffles.
// Everything per lane lives in registers; the kernel is templated on the
// largest finger DOF so the small dense solves unroll.
#include <math.h>

#include <algorithm>

#include "lg_internal.h"

namespace lg {

constexpr int kRealizeThreads = 256;

constexpr uint32_t kPurposeUnused = 15u;

// distance between segments [p1, q1] and [p2, q2]: the closest parameters
// (s, t) in [0,1]^2 in closed form (Ericson, Real-Time Collision Detection,
// Sec. 5.1.9)
__device__ inline float segment_distance(const float *p1, const float *q1, const float *p2, const float *q2)
{
    const float d1x = q1[0] - p1[0], d1y = q1[1] - p1[1], d1z = q1[2] - p1[2];
    const float d2x = q2[0] - p2[0], d2y = q2[1] - p2[1], d2z = q2[2] - p2[2];
    const float rx = p1[0] - p2[0], ry = p1[1] - p2[1], rz = p1[2] - p2[2];
    const float a = d1x * d1x + d1y * d1y + d1z * d1z, e = d2x * d2x + d2y * d2y + d2z * d2z;
    const float f = d2x * rx + d2y * ry + d2z * rz;
    float s, t;
    if (a <= 1e-20f && e <= 1e-20f) {
        s = t = 0.0f;
    } else if (a <= 1e-20f) {
        s = 0.0f;
        t = fminf(fmaxf(f / e, 0.0f), 1.0f);
    } else {
        const float c = d1x * rx + d1y * ry + d1z * rz;
        if (e <= 1e-20f) {
            t = 0.0f;
            s = fminf(fmaxf(-c / a, 0.0f), 1.0f);
        } else {
            const float b = d1x * d2x + d1y * d2y + d1z * d2z, den = a * e - b * b;
            s = den > 0.0f ? fminf(fmaxf((b * f - c * e) / den, 0.0f), 1.0f) : 0.0f;
            t = (b * s + f) / e;
            if (t < 0.0f) {
                t = 0.0f;
                s = fminf(fmaxf(-c / a, 0.0f), 1.0f);
            } else if (t > 1.0f) {
                t = 1.0f;
                s = fminf(fmaxf((b - c) / a, 0.0f), 1.0f);
            }
        }
    }
    const float x = rx + s * d1x - t * d2x, y = ry + s * d1y - t * d2y, z = rz + s * d1z - t * d2z;
    return sqrtf(x * x + y * y + z * z);
}

__device__ inline float dot3f(float ax, float ay, float az, float bx, float by, float bz)
{
    return fmaf(ax, bx, fmaf(ay, by, az * bz));
}

// unit vector of (x, y, z); a direction perpendicular to the axis if tiny
__device__ inline void unit_or_perp(float &x, float &y, float &z, float ax, float ay, float az)
{
    const float n2 = dot3f(x, y, z, x, y, z);
    if (n2 > 1e-30f) {
        const float r = 1.0f / sqrtf(n2);
        x *= r;
        y *= r;
        z *= r;
    } else {
        // Duff et al. basis, first tangent of the axis
        const float sign = copysignf(1.0f, az);
        const float a = -1.0f / (sign + az);
        x = 1.0f + sign * ax * ax * a;
        y = sign * ax * ay * a;
        z = -sign * ax;
    }
}

// Capsule point closest to (p, n) in |x - p|^2 + beta^2 |nt - n|^2.
__device__ inline void capsule_aligned(const float *A, const float *Bp, float r, const float *p, const float *n,
                                       float beta, float *pt, float *nt)
{
    float ab[3] = {Bp[0] - A[0], Bp[1] - A[1], Bp[2] - A[2]};
    const float L = sqrtf(dot3f(ab[0], ab[1], ab[2], ab[0], ab[1], ab[2]));
    float ax = 0.f, ay = 0.f, az = 1.f;
    if (L > 0.f) {
        ax = ab[0] / L;
        ay = ab[1] / L;
        az = ab[2] / L;
    }
    const float b2 = beta * beta;
    float best;
    {  // cylinder
        float s = dot3f(p[0] - A[0], p[1] - A[1], p[2] - A[2], ax, ay, az);
        s = fminf(fmaxf(s, 0.f), L);
        const float cx = fmaf(s, ax, A[0]), cy = fmaf(s, ay, A[1]), cz = fmaf(s, az, A[2]);
        float vx = fmaf(r, p[0] - cx, b2 * n[0]), vy = fmaf(r, p[1] - cy, b2 * n[1]), vz = fmaf(r, p[2] - cz, b2 * n[2]);
        const float va = dot3f(vx, vy, vz, ax, ay, az);
        vx = fmaf(-va, ax, vx);
        vy = fmaf(-va, ay, vy);
        vz = fmaf(-va, az, vz);
        unit_or_perp(vx, vy, vz, ax, ay, az);
        pt[0] = fmaf(r, vx, cx);
        pt[1] = fmaf(r, vy, cy);
        pt[2] = fmaf(r, vz, cz);
        nt[0] = vx;
        nt[1] = vy;
        nt[2] = vz;
        const float d0 = pt[0] - p[0], d1 = pt[1] - p[1], d2 = pt[2] - p[2];
        const float e0 = vx - n[0], e1 = vy - n[1], e2 = vz - n[2];
        best = dot3f(d0, d1, d2, d0, d1, d2) + b2 * dot3f(e0, e1, e2, e0, e1, e2);
    }
#pragma unroll
    for (int cap = 0; cap < 2; ++cap) {
        const float *c = cap == 0 ? Bp : A;
        const float sg = cap == 0 ? 1.0f : -1.0f;
        float vx = fmaf(r, p[0] - c[0], b2 * n[0]), vy = fmaf(r, p[1] - c[1], b2 * n[1]),
              vz = fmaf(r, p[2] - c[2], b2 * n[2]);
        const float n2 = dot3f(vx, vy, vz, vx, vy, vz);
        if (!(n2 > 1e-30f)) continue;
        const float rn = 1.0f / sqrtf(n2);
        vx *= rn;
        vy *= rn;
        vz *= rn;
        if (sg * dot3f(vx, vy, vz, ax, ay, az) < 0.f) continue;
        const float x0 = fmaf(r, vx, c[0]), x1 = fmaf(r, vy, c[1]), x2 = fmaf(r, vz, c[2]);
        const float d0 = x0 - p[0], d1 = x1 - p[1], d2 = x2 - p[2];
        const float e0 = vx - n[0], e1 = vy - n[1], e2 = vz - n[2];
        const float cost = dot3f(d0, d1, d2, d0, d1, d2) + b2 * dot3f(e0, e1, e2, e0, e1, e2);
        if (cost < best) {
            best = cost;
            pt[0] = x0;
            pt[1] = x1;
            pt[2] = x2;
            nt[0] = vx;
            nt[1] = vy;
            nt[2] = vz;
        }
    }
}

// Plain projection of p onto the capsule surface.
__device__ inline void capsule_project(const float *A, const float *Bp, float r, const float *p, float *pt, float *nt)
{
    const float ab0 = Bp[0] - A[0], ab1 = Bp[1] - A[1], ab2 = Bp[2] - A[2];
    const float L2 = dot3f(ab0, ab1, ab2, ab0, ab1, ab2);
    float t = L2 > 0.f ? dot3f(p[0] - A[0], p[1] - A[1], p[2] - A[2], ab0, ab1, ab2) / L2 : 0.f;
    t = fminf(fmaxf(t, 0.f), 1.f);
    const float c0 = fmaf(t, ab0, A[0]), c1 = fmaf(t, ab1, A[1]), c2 = fmaf(t, ab2, A[2]);
    float ax = 0.f, ay = 0.f, az = 1.f;
    if (L2 > 0.f) {
        const float rl = 1.0f / sqrtf(L2);
        ax = ab0 * rl;
        ay = ab1 * rl;
        az = ab2 * rl;
    }
    float vx = p[0] - c0, vy = p[1] - c1, vz = p[2] - c2;
    unit_or_perp(vx, vy, vz, ax, ay, az);
    nt[0] = vx;
    nt[1] = vy;
    nt[2] = vz;
    pt[0] = fmaf(r, vx, c0);
    pt[1] = fmaf(r, vy, c1);
    pt[2] = fmaf(r, vz, c2);
}


#define LG_REALIZE_ARGS                                                                                         \
    DevHand H, const int32_t *__restrict__ wit, SdfDev S, const float *__restrict__ pts,                        \
        const float *__restrict__ nrm, int N, const float *__restrict__ poses,                                  \
        const int32_t *__restrict__ set_pt, const int8_t *__restrict__ set_link, int k, int D, int64_t n_sets,  \
        const int32_t *__restrict__ acc_list, const int32_t *__restrict__ n_acc_dev, int max_acc, IkDev ik,    \
        float *__restrict__ q_out, float *__restrict__ cerr, float *__restrict__ cang,                          \
        float *__restrict__ depth_out, uint8_t *__restrict__ valid_out
#define LG_REALIZE_PASS                                                                                         \
    H, wit, S, pts, nrm, N, poses, set_pt, set_link, k, D, n_sets, acc_list, n_acc_dev, max_acc, ik, q_out,     \
        cerr, cang, depth_out, valid_out

// cb: bin centres in LDS; caps: capsule axis end points of every lane's finger
// at its final configuration (LDS); block bid of nb (grid-stride)
template <int DM>
__device__ __forceinline__ void realize_sets(
    float *cb, float (*caps)[DM][6], int64_t bid, int64_t nb, const DevHand &H, const int32_t *__restrict__ wit,
    const SdfDev &S, const float *__restrict__ pts, const float *__restrict__ nrm, int N,
    const float *__restrict__ poses, const int32_t *__restrict__ set_pt, const int8_t *__restrict__ set_link, int k,
    int D, int64_t n_sets, const int32_t *__restrict__ acc_list, const int32_t *__restrict__ n_acc_dev, int max_acc,
    const IkDev &ik, float *__restrict__ q_out, float *__restrict__ cerr, float *__restrict__ cang,
    float *__restrict__ depth_out, uint8_t *__restrict__ valid_out)
{
    for (int i = threadIdx.x; i < 3 * H.B; i += kRealizeThreads) cb[i] = H.bin_c[i];
    __syncthreads();
    const int64_t gt = bid * kRealizeThreads + threadIdx.x;
    const int spw = 64 / H.F;                    // sets per wave
    const int lane = threadIdx.x & 63, slot = lane / H.F;
    const int f = lane - slot * H.F;             // this lane's finger
    const int tid = threadIdx.x, base = tid - f;  // the set's first lane in the block
    const int64_t nacc = min((int64_t)*n_acc_dev, (int64_t)max_acc);
    const int64_t stride = ((nb * kRealizeThreads) >> 6) * spw;
    // grid-stride over accepted sets; the F lanes of a set move together, the
    // lanes past spw * F do nothing
    for (int64_t a = slot < spw ? (gt >> 6) * spw + slot : nacc; a < nacc; a += stride) {
        const int64_t id = acc_list[a];
        if (id < 0 || id >= n_sets) {  // not a set id: no reads through it (uniform over the set's lanes)
            if (f < H.F)
                for (int t = 0; t < H.finger_dof[f]; ++t) q_out[a * H.J + H.finger_first[f] + t] = __builtin_nanf("");
            if (f < k) {
                cerr[a * k + f] = INFINITY;
                cang[a * k + f] = INFINITY;
            }
            if (f == 0) {
                depth_out[a] = __builtin_nanf("");
                valid_out[a] = 0;
            }
            continue;
        }
        const int64_t g = id / D;
        const int dr = (int)(id % D);
        float P[12];
#pragma unroll
        for (int i = 0; i < 12; ++i) P[i] = poses[12 * g + i];
        // contact layout: the finger of contact i is that of its link; the set is
        // realisable iff every link is a hand link, every point an object point
        // and the fingers increase strictly with i
        uint32_t used = 0;
        bool ok = true;
        int prev = -1;
        for (int i = 0; i < k; ++i) {
            const int l = set_link[id * k + i], idx = set_pt[id * k + i];
            int fl = -1;
            for (int ff = 0; ff < H.F; ++ff)
                if (l >= H.finger_first[ff] && l < H.finger_first[ff] + H.finger_dof[ff]) fl = ff;
            ok = ok && fl > prev && idx >= 0 && idx < N;
            prev = fl;
            if (fl >= 0) used |= 1u << fl;
        }
        if (!ok) used = 0;
        float dep = -INFINITY, emax = 0.f, amax = 0.f;
        if (f < H.F) {
            const int first = H.finger_first[f], d = H.finger_dof[f];
            const int ci = ((used >> f) & 1u) ? __popc(used & ((1u << f) - 1u)) : -1;  // this finger's contact
            float q[DM];
            int tl = -1;  // link index within the finger of the contact (-1: none)
            float p[3] = {0.f, 0.f, 0.f}, n[3] = {0.f, 0.f, 1.f};
            if (ci >= 0) {
                const int idx = set_pt[id * k + ci];
                const int l = set_link[id * k + ci];
                const float ox = pts[idx], oy = pts[N + idx], oz = pts[2 * N + idx];
                p[0] = fmaf(P[0], ox, fmaf(P[1], oy, fmaf(P[2], oz, P[3])));
                p[1] = fmaf(P[4], ox, fmaf(P[5], oy, fmaf(P[6], oz, P[7])));
                p[2] = fmaf(P[8], ox, fmaf(P[9], oy, fmaf(P[10], oz, P[11])));
                query_dir(P, nrm[idx], nrm[N + idx], nrm[2 * N + idx], n[0], n[1], n[2]);
                // reverse lookup: witness sample of (link, voxel(p), bin(n))
                int32_t w = kNoWitness;
                if (wit) {
                    const int v = finger_window_voxel(H, P, f, ox, oy, oz);
                    const int b = nearest_bin(cb, H.B, n[0], n[1], n[2]);
                    if (v >= 0) w = wit[((int64_t)l * H.G * H.G * H.G + v) * H.B + b];
                }
#pragma unroll
                for (int t = 0; t < DM; ++t) {
                    q[t] = 0.f;
                    if (t < d) {
                        const int j = first + t;
                        q[t] = (w >= 0 && w < H.samples) ? joint_sample(H, f, (uint32_t)w, t)
                                                         : 0.5f * (H.limits[2 * j] + H.limits[2 * j + 1]);
                    }
                }
                tl = l - first;
                const float *cap = H.capsule + 7 * l;
                const float r = cap[6];
                float loc_p[3] = {0.f, 0.f, 0.f}, loc_n[3] = {0.f, 0.f, 1.f};
                for (int it = 0; it < ik.iters; ++it) {
                    float o[DM][3], z[DM][3];
                    Tf T, Tl;
#pragma unroll
                    for (int t = 0; t < DM; ++t) {
                        if (t < d) {
                            const int j = first + t;
                            T = joint_frame(H, T, t > 0, j, q[t]);
                            o[t][0] = T.m[3];
                            o[t][1] = T.m[7];
                            o[t][2] = T.m[11];
                            tf_dir(T, H.axis[3 * j], H.axis[3 * j + 1], H.axis[3 * j + 2], z[t][0], z[t][1], z[t][2]);
                            if (t == tl) Tl = T;
                        }
                    }
                    float pt[3], nt[3];
                    if (it == 0 || it >= ik.phase1) {
                        float A[3], Bq[3];
                        tf_point(Tl, cap[0], cap[1], cap[2], A[0], A[1], A[2]);
                        tf_point(Tl, cap[3], cap[4], cap[5], Bq[0], Bq[1], Bq[2]);
                        capsule_aligned(A, Bq, r, p, n, ik.beta, pt, nt);
                        const float dx = pt[0] - Tl.m[3], dy = pt[1] - Tl.m[7], dz = pt[2] - Tl.m[11];
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            loc_p[c] = fmaf(Tl.m[c], dx, fmaf(Tl.m[4 + c], dy, Tl.m[8 + c] * dz));
                            loc_n[c] = fmaf(Tl.m[c], nt[0], fmaf(Tl.m[4 + c], nt[1], Tl.m[8 + c] * nt[2]));
                        }
                    } else {
                        tf_point(Tl, loc_p[0], loc_p[1], loc_p[2], pt[0], pt[1], pt[2]);
                        tf_dir(Tl, loc_n[0], loc_n[1], loc_n[2], nt[0], nt[1], nt[2]);
                    }
                    float x2[3], e[6];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        x2[c] = fmaf(ik.beta, nt[c], pt[c]);
                        e[c] = p[c] - pt[c];
                        e[3 + c] = fmaf(ik.beta, n[c], p[c]) - x2[c];
                    }
                    float Jc[DM][6];
#pragma unroll
                    for (int t = 0; t < DM; ++t) {
                        const bool on = t < d && t <= tl;
#pragma unroll
                        for (int s = 0; s < 2; ++s) {
                            const float *x = s == 0 ? pt : x2;
                            const float vx = x[0] - o[t][0], vy = x[1] - o[t][1], vz = x[2] - o[t][2];
                            Jc[t][3 * s + 0] = on ? z[t][1] * vz - z[t][2] * vy : 0.f;
                            Jc[t][3 * s + 1] = on ? z[t][2] * vx - z[t][0] * vz : 0.f;
                            Jc[t][3 * s + 2] = on ? z[t][0] * vy - z[t][1] * vx : 0.f;
                        }
                    }
                    // normal equations (J^T J + lambda I) dq = J^T e, Cholesky in place
                    float M[DM][DM], gv[DM];
#pragma unroll
                    for (int i = 0; i < DM; ++i) {
                        float acc = 0.f;
#pragma unroll
                        for (int rr = 0; rr < 6; ++rr) acc = fmaf(Jc[i][rr], e[rr], acc);
                        gv[i] = acc;
#pragma unroll
                        for (int j = 0; j < DM; ++j) {
                            float s2 = 0.f;
#pragma unroll
                            for (int rr = 0; rr < 6; ++rr) s2 = fmaf(Jc[i][rr], Jc[j][rr], s2);
                            M[i][j] = s2 + (i == j ? ik.lambda : 0.f);
                        }
                    }
                    bool ok = true;
#pragma unroll
                    for (int j = 0; j < DM; ++j) {
                        float s2 = M[j][j];
#pragma unroll
                        for (int kk = 0; kk < j; ++kk) s2 = fmaf(-M[j][kk], M[j][kk], s2);
                        ok &= s2 > 0.f;
                        const float dd = sqrtf(fmaxf(s2, 1e-30f));
                        M[j][j] = dd;
                        const float inv = 1.0f / dd;
#pragma unroll
                        for (int i = j + 1; i < DM; ++i) {
                            float t2 = M[i][j];
#pragma unroll
                            for (int kk = 0; kk < j; ++kk) t2 = fmaf(-M[i][kk], M[j][kk], t2);
                            M[i][j] = t2 * inv;
                        }
                    }
                    if (!ok) break;
#pragma unroll
                    for (int i = 0; i < DM; ++i) {
                        float t2 = gv[i];
#pragma unroll
                        for (int kk = 0; kk < i; ++kk) t2 = fmaf(-M[i][kk], gv[kk], t2);
                        gv[i] = t2 / M[i][i];
                    }
#pragma unroll
                    for (int i = DM - 1; i >= 0; --i) {
                        float t2 = gv[i];
#pragma unroll
                        for (int kk = i + 1; kk < DM; ++kk) t2 = fmaf(-M[kk][i], gv[kk], t2);
                        gv[i] = t2 / M[i][i];
                    }
#pragma unroll
                    for (int t = 0; t < DM; ++t) {
                        if (t < d) {
                            const int j = first + t;
                            q[t] = fminf(fmaxf(q[t] + gv[t], H.limits[2 * j]), H.limits[2 * j + 1]);
                        }
                    }
                }
            } else {
                // a finger without contact takes uniform random joint values (Sec. 5.6)
                uint32_t w[8];
                philox4x32_10((uint32_t)(ik.pose_offset + g), (uint32_t)dr, kPurposeUnused | ((uint32_t)(2 * f) << 8),
                              ik.request_id, ik.seed_lo, ik.seed_hi, w);
                if (d > 4)
                    philox4x32_10((uint32_t)(ik.pose_offset + g), (uint32_t)dr,
                                  kPurposeUnused | ((uint32_t)(2 * f + 1) << 8), ik.request_id, ik.seed_lo,
                                  ik.seed_hi, w + 4);
#pragma unroll
                for (int t = 0; t < DM; ++t) {
                    q[t] = 0.f;
                    if (t < d) {
                        const float lo = H.limits[2 * (first + t)], hi = H.limits[2 * (first + t) + 1];
                        q[t] = fmaf(hi - lo, u01f(w[t]), lo);
                    }
                }
            }
            // final configuration: contact quality and penetration of the finger's links
            Tf T;
#pragma unroll
            for (int t = 0; t < DM; ++t) {
                if (t < d) {
                    const int j = first + t;
                    T = joint_frame(H, T, t > 0, j, q[t]);
                    const float *cj = H.capsule + 7 * j;
                    float A[3], Bq[3];
                    tf_point(T, cj[0], cj[1], cj[2], A[0], A[1], A[2]);
                    tf_point(T, cj[3], cj[4], cj[5], Bq[0], Bq[1], Bq[2]);
                    caps[tid][t][0] = A[0];
                    caps[tid][t][1] = A[1];
                    caps[tid][t][2] = A[2];
                    caps[tid][t][3] = Bq[0];
                    caps[tid][t][4] = Bq[1];
                    caps[tid][t][5] = Bq[2];
                    if (t == tl) {
                        float pt[3], nt[3];
                        capsule_project(A, Bq, cj[6], p, pt, nt);
                        const float d0 = p[0] - pt[0], d1 = p[1] - pt[1], d2 = p[2] - pt[2];
                        emax = sqrtf(dot3f(d0, d1, d2, d0, d1, d2));
                        amax = acosf(fminf(fmaxf(dot3f(nt[0], nt[1], nt[2], n[0], n[1], n[2]), -1.f), 1.f));
                    }
                    const int M = H.axis_samples[j];
                    const float inv = 1.0f / (float)(M - 1);
                    for (int s = 0; s < M; ++s) {
                        const float ts = (float)s * inv;
                        const float x0 = fmaf(ts, Bq[0] - A[0], A[0]) - P[3];
                        const float x1 = fmaf(ts, Bq[1] - A[1], A[1]) - P[7];
                        const float x2 = fmaf(ts, Bq[2] - A[2], A[2]) - P[11];
                        // object frame: R^T (x - t)
                        const float y0 = fmaf(P[0], x0, fmaf(P[4], x1, P[8] * x2));
                        const float y1 = fmaf(P[1], x0, fmaf(P[5], x1, P[9] * x2));
                        const float y2 = fmaf(P[2], x0, fmaf(P[6], x1, P[10] * x2));
                        dep = fmaxf(dep, cj[6] - sdf_trilinear(S, y0, y1, y2));
                    }
                    q_out[a * H.J + j] = q[t];
                }
            }
            if (ci >= 0) {
                cerr[a * k + ci] = emax;
                cang[a * k + ci] = amax;
            }
        }
        if (!ok && f < k) {  // not realisable: no contact is met
            cerr[a * k + f] = INFINITY;
            cang[a * k + f] = INFINITY;
            emax = INFINITY;
            amax = INFINITY;
        }
        // hand self-collision: this finger's links against those of the higher
        // fingers of the set (the F lanes of a set are in one wave)
        if (ik.self_collision) {
            __builtin_amdgcn_wave_barrier();
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            if (f < H.F) {
                const int first = H.finger_first[f], d = H.finger_dof[f];
                for (int f2 = f + 1; f2 < H.F; ++f2) {
                    const int first2 = H.finger_first[f2], d2 = H.finger_dof[f2];
                    for (int t = 0; t < d; ++t)
                        for (int t2 = 0; t2 < d2; ++t2) {
                            const float *c1 = caps[tid][t], *c2 = caps[base + f2][t2];
                            const float pen = H.capsule[7 * (first + t) + 6] + H.capsule[7 * (first2 + t2) + 6] -
                                              segment_distance(c1, c1 + 3, c2, c2 + 3);
                            dep = fmaxf(dep, pen);
                        }
                }
            }
            __builtin_amdgcn_wave_barrier();
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
        }
        // set-level reductions over the F lanes of the set (all active: same set)
        {
            const int first_lane = lane - f;
            float d2 = dep, e2 = emax, a2 = amax;
            for (int j = 0; j < H.F; ++j) {
                d2 = fmaxf(d2, __shfl(dep, first_lane + j, 64));
                e2 = fmaxf(e2, __shfl(emax, first_lane + j, 64));
                a2 = fmaxf(a2, __shfl(amax, first_lane + j, 64));
            }
            dep = d2;
            emax = e2;
            amax = a2;
        }
        if (f == 0) {
            depth_out[a] = dep;
            valid_out[a] = (emax <= ik.tol_pos && amax <= ik.tol_ang && dep <= ik.margin) ? 1 : 0;
        }
    }
}

// up to 6 joints per finger: two waves per SIMD (at most 256 registers)
template <int DM>
__global__ void __launch_bounds__(kRealizeThreads) __attribute__((amdgpu_waves_per_eu(2)))
k_realize(LG_REALIZE_ARGS)
{
    __shared__ float cb[3 * kMaxBins];
    __shared__ float caps[kRealizeThreads][DM][6];
    realize_sets<DM>(cb, caps, blockIdx.x, gridDim.x, LG_REALIZE_PASS);
}

// 7 or 8 joints per finger: one wave per SIMD rather than spilling
__global__ void __launch_bounds__(kRealizeThreads) k_realize_wide(LG_REALIZE_ARGS)
{
    __shared__ float cb[3 * kMaxBins];
    __shared__ float caps[kRealizeThreads][8][6];
    realize_sets<8>(cb, caps, blockIdx.x, gridDim.x, LG_REALIZE_PASS);
}

// The same over the accepted sets of several chunks (max_acc = the chunk's
// P * D); DM = 8 takes one wave per SIMD like k_realize_wide.
template <int DM>
__global__ void __launch_bounds__(kRealizeThreads) __attribute__((amdgpu_waves_per_eu(DM <= 6 ? 2 : 1)))
k_realize_batch(const ChunkDesc *__restrict__ d, const uint16_t *__restrict__ idx, const uint32_t *__restrict__ first,
                int n)
{
    __shared__ float cb[3 * kMaxBins];
    __shared__ float caps[kRealizeThreads][DM][6];
    const int j = batch_member(first, n, blockIdx.x);
    const ChunkDesc &c = d[idx[j]];
    const int64_t n_sets = (int64_t)c.P * c.D;
    realize_sets<DM>(cb, caps, blockIdx.x - first[j], first[j + 1] - first[j], c.H, c.wit, c.S, c.pts, c.nrm, c.N,
                     c.poses, c.set_pt, c.set_link, c.k, c.D, n_sets, c.acc, c.n_acc, (int)n_sets, c.ik, c.q, c.err,
                     c.ang, c.depth, c.valid);
}

#undef LG_REALIZE_ARGS
#undef LG_REALIZE_PASS

}  // namespace lg

using namespace lg;

extern "C" lg_status lg_realize(const lg_field *field, const lg_sdf *sdf, const float *pts, const float *nrm,
                                int32_t n_points, const float *poses, int32_t n_poses, const int32_t *set_pt,
                                const int8_t *set_link, int32_t k, int32_t draws, const int32_t *acc_list,
                                const int32_t *n_acc_dev, int32_t max_acc, const lg_ik_params *p, float *q_out,
                                float *contact_err, float *contact_ang, float *depth, uint8_t *valid, void *stream)
{
    if (!field || !sdf || !p) return fail(LG_EINVAL, "null field, sdf or params");
    const DevHand &H = field->dh;
    if (k < 1 || k > H.F) return fail(LG_EINVAL, "need 1 <= k <= number of fingers");
    if (n_points <= 0 || n_poses <= 0 || draws <= 0 || max_acc < 0)
        return fail(LG_EINVAL, "bad sizes");
    if (sdf->dims < 2 || !(sdf->h > 0.f) || !sdf->values) return fail(LG_EINVAL, "bad sdf");
    if (p->iters < 0 || p->phase1 < 0 || !(p->lambda > 0.f)) return fail(LG_EINVAL, "need iters >= 0, lambda > 0");
    if (max_acc == 0) return LG_OK;
    if (!pts || !nrm || !poses || !set_pt || !set_link || !acc_list || !n_acc_dev || !q_out || !contact_err ||
        !contact_ang || !depth || !valid)
        return fail(LG_EINVAL, "null device buffer");
    SdfDev S{sdf->origin[0], sdf->origin[1], sdf->origin[2], sdf->h, 1.0f / sdf->h, sdf->dims, sdf->values};
    IkDev ik{p->iters, p->phase1, p->lambda, p->beta, p->tol_pos, p->tol_ang, p->margin, p->self_collision,
             (uint32_t)p->seed, (uint32_t)(p->seed >> 32), p->request_id, p->pose_offset};
    hipStream_t s = as_stream(stream);
    // grid-stride launch sized to the device, not to the max_acc upper bound
    int dev = 0, n_cu = 0;
    LG_HIP(hipGetDevice(&dev));
    LG_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    const dim3 grid(realize_blocks(max_acc, H.F, n_cu));
    const int32_t *wit = field->has_witness ? field->d_wit : nullptr;
#define LG_REALIZE(KERNEL)                                                                                      \
    hipLaunchKernelGGL(KERNEL, grid, dim3(kRealizeThreads), 0, s, H, wit, S, pts, nrm, n_points, poses,     \
                       set_pt, set_link, k, draws, (int64_t)n_poses * draws, acc_list, n_acc_dev, max_acc, ik,  \
                       q_out, contact_err,                                                                      \
                       contact_ang, depth, valid)
    if (field->max_dof <= 4)
        LG_REALIZE(k_realize<4>);
    else if (field->max_dof <= 6)
        LG_REALIZE(k_realize<6>);
    else
        LG_REALIZE(k_realize_wide);
#undef LG_REALIZE
    LG_HIP(hipGetLastError());
    return LG_OK;
}

uint32_t lg::realize_blocks(int64_t max_acc, int F, int n_cu)
{
    const int64_t spw = 64 / F;  // sets per wave
    const int64_t threads = std::min<int64_t>((max_acc + spw - 1) / spw * 64, (int64_t)n_cu * 16 * kRealizeThreads);
    return (uint32_t)std::max<int64_t>(1, (threads + kRealizeThreads - 1) / kRealizeThreads);
}

lg_status lg::realize_batch(const BatchLaunch &b, int max_dof, hipStream_t s)
{
    if (b.n <= 0 || b.blocks == 0) return LG_OK;
    if (max_dof <= 4)
        hipLaunchKernelGGL(k_realize_batch<4>, dim3(b.blocks), dim3(kRealizeThreads), 0, s, b.d, b.idx, b.first, b.n);
    else if (max_dof <= 6)
        hipLaunchKernelGGL(k_realize_batch<6>, dim3(b.blocks), dim3(kRealizeThreads), 0, s, b.d, b.idx, b.first, b.n);
    else
        hipLaunchKernelGGL(k_realize_batch<8>, dim3(b.blocks), dim3(kRealizeThreads), 0, s, b.d, b.idx, b.first, b.n);
    LG_HIP(hipGetLastError());
    return LG_OK;
}
