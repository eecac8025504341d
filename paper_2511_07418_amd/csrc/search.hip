// Contact-set draws (Sec. 5.3, Alg. 2 initialisation), reverse lookup of the
// hand link (Sec. 5.5), the contact-set criterion (Eq. 1-2 with a linearised
// friction cone, as an LP) and deterministic compaction of accepted sets.
#include <math.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "lg_internal.h"

namespace lg {

constexpr int kDrawThreads = 256;
constexpr int kSuper = 8;           // words per rank superblock
constexpr int kChunkPerThread = 32; // compaction: sets per thread
constexpr int kCompactThreads = 256;
constexpr int kChunk = kChunkPerThread * kCompactThreads;

// select the r-th (0-based) set bit of x
__device__ inline int select_in_word(uint32_t x, uint32_t r)
{
    for (uint32_t i = 0; i < r; ++i) x &= x - 1u;
    return __ffs(x) - 1;
}

constexpr uint32_t kPurposeFingers = 13u;
constexpr uint32_t kPurposeExtFingers = 19u;  // second contact round: fingers
constexpr uint32_t kPurposeExtDraw = 21u;     // second contact round: points and links

// Contact fingers of set d of pose gg (global index) as a bit mask: k picks
// without replacement among the eligible fingers (non-empty domains), pick j
// taking the floor(w_j (c - j) / 2^32)-th remaining one in increasing finger
// order; contact i goes to the i-th lowest bit.  With c == k every eligible
// finger is picked whatever the words, so they are not drawn.
__device__ inline uint32_t choose_fingers(uint32_t elig, int k, uint32_t gg, int d, uint32_t request_id,
                                          uint32_t seed_lo, uint32_t seed_hi, uint32_t purpose = kPurposeFingers)
{
    const int c = __popc(elig);
    if (c <= k) return c == k ? elig : 0u;
    uint32_t w[8];
    philox4x32_10(gg, (uint32_t)d, purpose, request_id, seed_lo, seed_hi, w);
    if (k > 4) philox4x32_10(gg, (uint32_t)d, purpose | (1u << 8), request_id, seed_lo, seed_hi, w + 4);
    uint32_t left = elig, mask = 0;
    for (int j = 0; j < k; ++j) {
        uint32_t x = left;
        for (uint32_t r = __umulhi(w[j], (uint32_t)(c - j)); r > 0; --r) x &= x - 1u;
        const uint32_t bit = x & (0u - x);
        mask |= bit;
        left &= ~bit;
    }
    return mask;
}

// eligible fingers of pose g: those whose domain is non-empty
__device__ inline uint32_t eligible_fingers(const uint32_t *__restrict__ dom_count, int64_t g, int F)
{
    uint32_t e = 0;
    for (int f = 0; f < F; ++f) e |= (dom_count[g * F + f] > 0 ? 1u : 0u) << f;
    return e;
}

// Reverse lookup (Sec. 5.5): among the links of finger i whose own table is
// hit at point idx under the pose, the floor(r * count / 2^32)-th; -1 if none.
__device__ inline int pick_link(const DevHand &H, const uint32_t *__restrict__ bits, const float *cb,
                                const float *__restrict__ pts, const float *__restrict__ nrm, int N,
                                const float *pose, int i, int idx, uint32_t r)
{
    const int64_t G3 = (int64_t)H.G * H.G * H.G;
    const int v = finger_window_voxel(H, pose, i, pts[idx], pts[N + idx], pts[2 * N + idx]);
    float qx, qy, qz;
    query_dir(pose, nrm[idx], nrm[N + idx], nrm[2 * N + idx], qx, qy, qz);
    const int b = nearest_bin(cb, H.B, qx, qy, qz);
    uint32_t mask = 0;
    const int first = H.finger_first[i], dof = H.finger_dof[i];
    if (v >= 0)
        for (int t = 0; t < dof; ++t)
            if (table_bit(bits + (int64_t)(first + t) * G3 * H.W, H.W, v, b)) mask |= 1u << t;
    const uint32_t pc = __popc(mask);
    return pc ? first + select_in_word(mask, __umulhi(r, pc)) : -1;
}

// The j-th (0-based) set bit of a domain of NW words through its superblock
// prefix pf (nsb + 1 exclusive popcounts of kSuper-word superblocks): binary
// search for the last superblock with pf <= j, then a scan of at most kSuper
// words; -1 if the domain has no j-th bit.
__device__ inline int select_domain(const uint32_t *pf, int nsb, const uint32_t *__restrict__ dom, int NW, uint32_t j)
{
    int lo = 0, hi = nsb;  // invariant pf[lo] <= j < pf[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pf[mid] <= j) lo = mid; else hi = mid;
    }
    uint32_t rem = j - pf[lo];
    for (int wi = lo * kSuper; wi < min(NW, (lo + 1) * kSuper); ++wi) {
        const uint32_t x = dom[wi];
        const uint32_t pc = __popc(x);
        if (rem < pc) return wi * 32 + select_in_word(x, rem);
        rem -= pc;
    }
    return -1;
}

// Superblock popcount prefixes of the F domains of one pose into LDS
// (prefix[f * (nsb + 1) + sb]); the caller synchronises after.
__device__ inline void build_prefix(uint32_t *prefix, const uint32_t *__restrict__ dom, int F, int NW, int nsb)
{
    for (int i = threadIdx.x; i < F * nsb; i += blockDim.x) {
        const int f = i / nsb, sb = i % nsb;
        uint32_t c = 0;
        for (int w = sb * kSuper; w < min(NW, (sb + 1) * kSuper); ++w) c += __popc(dom[(int64_t)f * NW + w]);
        prefix[f * (nsb + 1) + sb + 1] = c;
    }
    __syncthreads();
    if ((int)threadIdx.x < F) {
        uint32_t *pf = prefix + threadIdx.x * (nsb + 1);
        pf[0] = 0;
        for (int sb = 1; sb <= nsb; ++sb) pf[sb] += pf[sb - 1];
    }
}

// One workgroup per pose.  Rank structure: exclusive popcount prefix per
// superblock of 8 domain words, in LDS; a draw binary-searches it and scans
// at most 8 words.
// the D sets of pose g (one block); prefix: [F][nsb + 1] words of LDS
__device__ __forceinline__ void draw_pose(uint32_t *prefix, float *cb, uint32_t *counts, const DevHand &H,
                                          const uint32_t *__restrict__ bits, const float *__restrict__ pts,
                                          const float *__restrict__ nrm, int N, const float *__restrict__ poses,
                                          const uint32_t *__restrict__ dom_bits, const uint32_t *__restrict__ dom_count,
                                          const int32_t *__restrict__ palm_pt, int D, int k, uint32_t seed_lo,
                                          uint32_t seed_hi, uint32_t request_id, int64_t pose_offset,
                                          int32_t *__restrict__ set_pt, int8_t *__restrict__ set_link,
                                          uint8_t *__restrict__ pose_valid, uint8_t *__restrict__ verdict,
                                          double *__restrict__ tstar, int g)
{
    const int F = H.F;
    const int NW = (N + 31) >> 5, nsb = (NW + kSuper - 1) / kSuper;
    const uint32_t *dom = dom_bits + (int64_t)g * F * NW;
    for (int i = threadIdx.x; i < 3 * H.B; i += blockDim.x) cb[i] = H.bin_c[i];
    if (threadIdx.x < F) counts[threadIdx.x] = dom_count[(int64_t)g * F + threadIdx.x];
    __syncthreads();
    uint32_t elig = 0;
    for (int f = 0; f < F; ++f) elig |= (counts[f] > 0 ? 1u : 0u) << f;
    // fewer than k usable domains, or a palm placement that was rejected
    const bool empty = __popc(elig) < k || (palm_pt && palm_pt[g] == -2);
    if (threadIdx.x == 0) pose_valid[g] = empty ? 0 : 1;
    if (empty) {
        for (int i = threadIdx.x; i < D * k; i += blockDim.x) {
            set_pt[(int64_t)g * D * k + i] = -1;
            set_link[(int64_t)g * D * k + i] = -1;
        }
        for (int d = threadIdx.x; d < D; d += blockDim.x) {  // no LP for these sets
            verdict[(int64_t)g * D + d] = 0;
            tstar[(int64_t)g * D + d] = __builtin_nan("");
        }
        return;  // uniform over the block
    }
    build_prefix(prefix, dom, F, NW, nsb);
    __syncthreads();
    const float *pose = poses + 12 * (int64_t)g;
    for (int d = threadIdx.x; d < D; d += blockDim.x) {
        uint32_t w[16];
        for (int blk = 0; blk * 4 < 2 * k; ++blk)
            philox4x32_10((uint32_t)(pose_offset + g), (uint32_t)(4 * d + blk), kPurposeDraw, request_id, seed_lo,
                          seed_hi, w + 4 * blk);
        int32_t *sp = set_pt + ((int64_t)g * D + d) * k;
        int8_t *sl = set_link + ((int64_t)g * D + d) * k;
        uint32_t fm = choose_fingers(elig, k, (uint32_t)(pose_offset + g), d, request_id, seed_lo, seed_hi);
        for (int i = 0; i < k; ++i) {
            const int f = __ffs(fm) - 1;  // finger of contact i
            fm &= fm - 1u;
            const int idx = select_domain(prefix + f * (nsb + 1), nsb, dom + (int64_t)f * NW, NW,
                                          __umulhi(w[i], counts[f]));
            sp[i] = idx;
            sl[i] = (int8_t)(idx >= 0 ? pick_link(H, bits, cb, pts, nrm, N, pose, f, idx, w[k + i]) : -1);
        }
    }
}

__global__ void __launch_bounds__(kDrawThreads)
k_draw(DevHand H, const uint32_t *__restrict__ bits, const float *__restrict__ pts, const float *__restrict__ nrm,
       int N, const float *__restrict__ poses, const uint32_t *__restrict__ dom_bits,
       const uint32_t *__restrict__ dom_count, const int32_t *__restrict__ palm_pt, int D, int k, uint32_t seed_lo,
       uint32_t seed_hi, uint32_t request_id, int64_t pose_offset, int32_t *__restrict__ set_pt,
       int8_t *__restrict__ set_link, uint8_t *__restrict__ pose_valid, uint8_t *__restrict__ verdict,
       double *__restrict__ tstar)
{
    extern __shared__ uint32_t prefix[];
    __shared__ float cb[3 * kMaxBins];
    __shared__ uint32_t counts[kMaxFingers];
    draw_pose(prefix, cb, counts, H, bits, pts, nrm, N, poses, dom_bits, dom_count, palm_pt, D, k, seed_lo, seed_hi,
              request_id, pose_offset, set_pt, set_link, pose_valid, verdict, tstar, blockIdx.x);
}

// the same over the poses of several chunks (no palm contacts)
__global__ void __launch_bounds__(kDrawThreads)
k_draw_batch(const ChunkDesc *__restrict__ d, const uint16_t *__restrict__ idx, const uint32_t *__restrict__ first,
             int n)
{
    extern __shared__ uint32_t prefix[];
    __shared__ float cb[3 * kMaxBins];
    __shared__ uint32_t counts[kMaxFingers];
    const int j = batch_member(first, n, blockIdx.x);
    const ChunkDesc &c = d[idx[j]];
    draw_pose(prefix, cb, counts, c.H, c.bits, c.pts, c.nrm, c.N, c.poses, c.dom_bits, c.dom_count, nullptr, c.D,
              c.k, c.seed_lo, c.seed_hi, c.request_id, c.pose_offset, c.set_pt, c.set_link, c.pose_valid, c.verdict,
              c.tstar, (int)(blockIdx.x - first[j]));
}

// ---- force-closure LP ---------------------------------------------------------
// Duff et al. (2017) branchless orthonormal basis of unit n.
__device__ inline double duff_a(double nz) { return -1.0 / (copysign(1.0, nz) + nz); }

// the basis from a = duff_a(nz), computed once per normal by the LP
__device__ inline void duff_basis_a(double nx, double ny, double nz, double a, double *x, double *y)
{
    const double sign = copysign(1.0, nz);
    const double b = nx * ny * a;
    x[0] = 1.0 + sign * nx * nx * a;
    x[1] = sign * b;
    x[2] = -sign * nx;
    y[0] = b;
    y[1] = sign + ny * ny * a;
    y[2] = -ny;
}

__device__ inline void duff_basis(double nx, double ny, double nz, double *x, double *y)
{
    const double sign = copysign(1.0, nz);
    const double a = duff_a(nz);
    const double b = nx * ny * a;
    x[0] = 1.0 + sign * nx * nx * a;
    x[1] = sign * b;
    x[2] = -sign * nx;
    y[0] = b;
    y[1] = sign + ny * ny * a;
    y[2] = -ny;
}

constexpr double kLpTol = 1e-12;  // reduced-cost and ratio-tie tolerance
constexpr double kLpPiv = 1e-9;   // smallest admissible pivot element
constexpr int kBlandAfter = 48;   // pivots priced by Dantzig's rule before Bland's

// ---- force-closure LP, one set per lane -------------------------------------
// Revised simplex with an explicit 7x7 basis inverse per lane.  Reduced
// costs are priced through the duals y = c_B^T B^-1: for wrench column
// (contact i, edge e),
//   y^T a_ie = u_i . d_ie + y_6,  u_i = y_f + (y_m x p_i) / rho,
//   u_i . d_ie = -u_i.n_i + mu (cos_e u_i.x_i + sin_e u_i.y_i),
// so pricing all k*m columns costs O(k) dot products plus 2 FMAs per edge.
// Bland's rule: lowest entering index, ratio ties to the lowest basic
// variable; pivots below kLpPiv are not admissible.  Double precision: the
// verdict is a thresholded decision and the LP is latency-bound.
// At a candidate optimum x_B and y are refined against the original columns
// (one residual correction through the current B^-1) and the pricing is
// repeated, so drift in B^-1 cannot end the search early or bias t*.  (One
// correction keeps t* within 1e-9 of the FP64 oracle's tableau simplex, as
// two did, at a tenth less time in the Alg. 2 criteria.)
// (LpConst: the cone edge directions, shared with the batched launch.)

// t* of the set held in this lane's LDS column (cd[6 i + c][tid]); status
// 0 = optimal, 1 = pivot cap, 2 = unbounded ratio test (not expected).
// MC > 0: the cone has MC edges (m == MC), known at compile time, so the
// pricing's edge loop is unrolled over constant edge directions.
template <int KM, bool WARM = false, int MC = 0>
__device__ inline double lp_lane(float (&cd)[KM * 6][256], int tid, int k, int m, double mu, double rho,
                                 int max_pivots, const LpConst &cs, int &status_out, int (*warm)[256] = nullptr)
{
    const int n = k * m;
    const double inv_rho = 1.0 / rho;
    // the reciprocal of each contact's tangent basis, once per LP (every
    // pricing and column rebuilds the basis); in LDS up to 6 contacts, beyond
    // that recomputed (the LDS would cost the 8-contact kernels occupancy)
    constexpr bool kDa = KM <= 6;
    __shared__ double da[kDa ? KM : 1][256];
    if constexpr (kDa)
        for (int i = 0; i < k; ++i) da[i][tid] = duff_a((double)cd[6 * i + 5][tid]);
    auto basis_of = [&](int ci, double nx, double ny, double nz, double *x, double *y) {
        if constexpr (kDa)
            duff_basis_a(nx, ny, nz, da[ci][tid], x, y);
        else
            duff_basis(nx, ny, nz, x, y);
    };
    // contact i's point and normal (each lane reads only its own column)
    auto contact = [&](int ci, double &px, double &py, double &pz, double &nx, double &ny, double &nz) {
        px = cd[6 * ci + 0][tid];
        py = cd[6 * ci + 1][tid];
        pz = cd[6 * ci + 2][tid];
        nx = cd[6 * ci + 3][tid];
        ny = cd[6 * ci + 4][tid];
        nz = cd[6 * ci + 5][tid];
    };
    // original column j of [W^T -I I; 1 0 0]
    auto column = [&](int j, double *a) {
#pragma unroll
        for (int r = 0; r < 7; ++r) a[r] = 0.0;
        if (j < n) {
            const int mm = MC > 0 ? MC : m;  // a constant divisor for the 8-edge kernels
            const int ci = j / mm, e = j - ci * mm;
            double px, py, pz, nx, ny, nz;
            contact(ci, px, py, pz, nx, ny, nz);
            double x[3], y[3];
            basis_of(ci, nx, ny, nz, x, y);
            const double c = cs.ce[e], s = cs.se[e];
            const double dx = -nx + mu * (c * x[0] + s * y[0]);
            const double dy = -ny + mu * (c * x[1] + s * y[1]);
            const double dz = -nz + mu * (c * x[2] + s * y[2]);
            a[0] = dx;
            a[1] = dy;
            a[2] = dz;
            a[3] = (py * dz - pz * dy) * inv_rho;
            a[4] = (pz * dx - px * dz) * inv_rho;
            a[5] = (px * dy - py * dx) * inv_rho;
            a[6] = 1.0;
        } else if (j < n + 6) {
#pragma unroll
            for (int r = 0; r < 6; ++r) a[r] = (r == j - n) ? -1.0 : 0.0;
        } else {
#pragma unroll
            for (int r = 0; r < 6; ++r) a[r] = (r == j - n - 6) ? 1.0 : 0.0;
        }
    };
    // initial basis: g_0 on the normalisation row, s-_r (w0_r <= 0) or s+_r
    double Bi[7][7], xB[7];
    int basis[7];
#define LG_LP_COLD()                                                                                        \
    do {                                                                                                    \
        double w0[7];                                                                                       \
        column(0, w0);                                                                                      \
        _Pragma("unroll") for (int r = 0; r < 7; ++r) _Pragma("unroll") for (int c = 0; c < 7; ++c) Bi[r][c] = 0.0; \
        _Pragma("unroll") for (int r = 0; r < 6; ++r) {                                                       \
            const double sg = w0[r] <= 0.0 ? 1.0 : -1.0;                                                    \
            basis[r] = w0[r] <= 0.0 ? n + 6 + r : n + r;                                                    \
            Bi[r][r] = sg;                                                                                  \
            Bi[r][6] = -sg * w0[r];                                                                         \
            xB[r] = -sg * w0[r];                                                                            \
        }                                                                                                   \
        Bi[6][6] = 1.0;                                                                                     \
        basis[6] = 0;                                                                                       \
        xB[6] = 1.0;                                                                                        \
    } while (0)
// replace the basic variable of row lr by column e (al = B^-1 a_e)
#define LG_LP_PIVOT(lr, al, e)                                                                              \
    do {                                                                                                    \
        double pv = 1.0, prow[7], px = 0.0;                                                                 \
        _Pragma("unroll") for (int c = 0; c < 7; ++c) prow[c] = 0.0;                                        \
        _Pragma("unroll") for (int r = 0; r < 7; ++r) if (r == (lr)) {                                      \
            pv = (al)[r];                                                                                   \
            px = xB[r];                                                                                     \
            _Pragma("unroll") for (int c = 0; c < 7; ++c) prow[c] = Bi[r][c];                               \
        }                                                                                                   \
        const double inv = 1.0 / pv;                                                                        \
        _Pragma("unroll") for (int c = 0; c < 7; ++c) prow[c] *= inv;                                       \
        px *= inv;                                                                                          \
        _Pragma("unroll") for (int r = 0; r < 7; ++r) {                                                     \
            if (r == (lr)) {                                                                                \
                _Pragma("unroll") for (int c = 0; c < 7; ++c) Bi[r][c] = prow[c];                           \
                xB[r] = px;                                                                                 \
                basis[r] = (e);                                                                             \
            } else {                                                                                        \
                _Pragma("unroll") for (int c = 0; c < 7; ++c) Bi[r][c] -= (al)[r] * prow[c];                \
                xB[r] -= (al)[r] * px;                                                                      \
            }                                                                                               \
        }                                                                                                   \
    } while (0)
    bool need_cold = true;
    // Warm start (the "free lunch" of Sec. 5.4): the optimal basis of a
    // neighbouring problem -- the same column ids, one contact's columns
    // rebuilt from its new point -- is brought into the cold basis column by
    // column, each by a primal pivot with the usual ratio test (so the basis
    // stays feasible; a column without an admissible pivot is left out).  The
    // simplex then continues from that basis, near the optimum when the
    // problems are close.  The optimum, t*, does not depend on the start.
    // warm[r][tid]: the column ids in, the final basis out.
    if constexpr (WARM) {
        if (warm[0][tid] >= 0) {
            LG_LP_COLD();
            need_cold = false;
#pragma unroll 1
            for (int w = 0; w < 7; ++w) {
                const int col = warm[w][tid];
                bool inb = false;
#pragma unroll
                for (int r = 0; r < 7; ++r) inb |= basis[r] == col;
                if (inb) continue;
                double a[7], al[7];
                column(col, a);
#pragma unroll
                for (int r = 0; r < 7; ++r) {
                    double sacc = 0.0;
#pragma unroll
                    for (int c = 0; c < 7; ++c) sacc += Bi[r][c] * a[c];
                    al[r] = sacc;
                }
                int lr = -1;
                double bx = 0.0, ba = 1.0;
#pragma unroll
                for (int r = 0; r < 7; ++r) {
                    if (al[r] > kLpPiv) {
                        const double lhs = xB[r] * ba, rhs = bx * al[r];
                        const double band = kLpTol * (ba + fabs(bx)) * al[r];
                        if (lr < 0 || lhs < rhs - band || (fabs(lhs - rhs) <= band && basis[r] < basis[lr])) {
                            lr = r;
                            bx = xB[r];
                            ba = al[r];
                        }
                    }
                }
                if (lr >= 0) LG_LP_PIVOT(lr, al, col);
            }
        }
    }
    if (need_cold) LG_LP_COLD();
    auto cost = [&](int j) { return j >= n ? 1.0 : 0.0; };
    auto duals = [&](double *y) {
#pragma unroll
        for (int c = 0; c < 7; ++c) {
            double s = 0.0;
#pragma unroll
            for (int r = 0; r < 7; ++r) s += cost(basis[r]) * Bi[r][c];
            y[c] = s;
        }
    };
    // Pricing.  Dantzig (most negative reduced cost, ties to the lowest index)
    // for the first kBlandAfter pivots; Bland (first negative) afterwards,
    // which rules out cycling.  -1 when no reduced cost is below -kLpTol.
    auto price = [&](const double *y, bool bland) {
        int e = -1;
        double best = -kLpTol;
        for (int i = 0; i < k && !(bland && e >= 0); ++i) {
            double px, py, pz, nx, ny, nz;
            contact(i, px, py, pz, nx, ny, nz);
            // u = y_f + (y_m x p) / rho
            const double ux = y[0] + (y[4] * pz - y[5] * py) * inv_rho;
            const double uy = y[1] + (y[5] * px - y[3] * pz) * inv_rho;
            const double uz = y[2] + (y[3] * py - y[4] * px) * inv_rho;
            double x[3], yy[3];
            basis_of(i, nx, ny, nz, x, yy);
            const double an = ux * nx + uy * ny + uz * nz;
            const double bx = ux * x[0] + uy * x[1] + uz * x[2];
            const double by = ux * yy[0] + uy * yy[1] + uz * yy[2];
            if constexpr (MC > 0) {
                bool done = false;
#pragma unroll
                for (int ee = 0; ee < MC; ++ee) {
                    const double d = -(-an + mu * (cs.ce[ee] * bx + cs.se[ee] * by)) - y[6];
                    if (!done && d < best) {
                        best = d;
                        e = i * MC + ee;
                        done = bland;
                    }
                }
            } else {
                for (int ee = 0; ee < m; ++ee) {
                    const double d = -(-an + mu * (cs.ce[ee] * bx + cs.se[ee] * by)) - y[6];
                    if (d < best) {
                        best = d;
                        e = i * m + ee;
                        if (bland) break;
                    }
                }
            }
        }
        for (int r = 0; r < 6 && !(bland && e >= 0); ++r)
            if (1.0 + y[r] < best) {
                best = 1.0 + y[r];
                e = n + r;
            }
        for (int r = 0; r < 6 && !(bland && e >= 0); ++r)
            if (1.0 - y[r] < best) {
                best = 1.0 - y[r];
                e = n + 6 + r;
            }
        return e;
    };
    // residual corrections of x_B (B x = e_6) and y (B^T y = c_B)
    auto refine = [&](double *y) {
        double rx[7] = {0, 0, 0, 0, 0, 0, 1.0}, ry[7];
#pragma unroll 1
        for (int q = 0; q < 7; ++q) {
            double a[7];
            column(basis[q], a);
            double dot = 0.0;
#pragma unroll
            for (int r = 0; r < 7; ++r) {
                rx[r] -= a[r] * xB[q];
                dot += a[r] * y[r];
            }
            ry[q] = cost(basis[q]) - dot;
        }
#pragma unroll
        for (int r = 0; r < 7; ++r) {
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < 7; ++c) s += Bi[r][c] * rx[c];
            xB[r] += s;
        }
#pragma unroll
        for (int c = 0; c < 7; ++c) {
            double s = 0.0;
#pragma unroll
            for (int r = 0; r < 7; ++r) s += ry[r] * Bi[r][c];
            y[c] += s;
        }
    };
    int piv = 0, status = 0, checks = 0;
    for (;;) {
        double y[7];
        duals(y);
        const bool bland = piv >= kBlandAfter;
        int e = price(y, bland);
        if (e < 0) {
            if (checks >= 4) break;
            ++checks;
            refine(y);
            e = price(y, bland);
            if (e < 0) break;
        }
        if (piv >= max_pivots) {
            status = 1;
            break;
        }
        double a[7], al[7];
        column(e, a);
#pragma unroll
        for (int r = 0; r < 7; ++r) {
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < 7; ++c) s += Bi[r][c] * a[c];
            al[r] = s;
        }
        // ratio test min x_B[r] / al[r] without divisions: the current best is
        // kept as the fraction bx / ba (ba > 0) and ratios are compared by
        // cross-multiplication; the tie band is kLpTol (1 + |best|).
        int lr = -1;
        double bx = 0.0, ba = 1.0;
#pragma unroll
        for (int r = 0; r < 7; ++r) {
            if (al[r] > kLpPiv) {
                const double lhs = xB[r] * ba, rhs = bx * al[r];
                const double band = kLpTol * (ba + fabs(bx)) * al[r];
                if (lr < 0 || lhs < rhs - band || (fabs(lhs - rhs) <= band && basis[r] < basis[lr])) {
                    lr = r;
                    bx = xB[r];
                    ba = al[r];
                }
            }
        }
        if (lr < 0) {
            status = 2;
            break;
        }
        LG_LP_PIVOT(lr, al, e);
        ++piv;
    }
#undef LG_LP_PIVOT
#undef LG_LP_COLD
    double ts = 0.0;
#pragma unroll
    for (int r = 0; r < 7; ++r)
        if (basis[r] >= n) ts += xB[r];
    if constexpr (WARM) {
#pragma unroll
        for (int r = 0; r < 7; ++r) warm[r][tid] = basis[r];
    }
    status_out = status;
    return ts;
}

// block bid of nb blocks (grid-stride); cd: contact data of each lane's set
// in LDS, lane-contiguous: cd[6*i + c][tid]
template <int KM, int MC = 0>
__device__ __forceinline__ void verdict_sets(float (&cd)[KM * 6][256], int64_t bid, int64_t nb,
                                             const float *__restrict__ pts, const float *__restrict__ nrm, int N,
                                             const int32_t *__restrict__ set_pt, const int32_t *__restrict__ palm_pt,
                                             const int32_t *__restrict__ valid_poses,
                                             const int32_t *__restrict__ n_valid_poses, int D, int k, int m, double mu,
                                             double rho, double eps, int max_pivots, const LpConst &cs,
                                             uint8_t *__restrict__ verdict, double *__restrict__ tstar)
{
    const int tid = threadIdx.x;
    const int64_t n_work = (int64_t)(*n_valid_poses) * D;
    const int64_t stride = nb * 256;
    // grid-stride over the sets of poses with at least k non-empty domains
    for (int64_t t = bid * 256 + tid; t < n_work; t += stride) {
        const int64_t g = valid_poses[t / D];
        const int64_t sid = g * D + (t % D);
        const int32_t *sp = set_pt + sid * k;
        // a palm contact (Sec. 5.1 static link) is one more, fixed, contact
        const int pc = palm_pt ? palm_pt[g] : -1;
        const int kc = pc >= 0 ? k + 1 : k;
        bool valid = true;
        for (int i = 0; i < kc; ++i) {
            const int idx = i < k ? sp[i] : pc;
            valid &= idx >= 0 && idx < N;
            const int ii = (idx >= 0 && idx < N) ? idx : 0;
            cd[6 * i + 0][tid] = pts[ii];
            cd[6 * i + 1][tid] = pts[N + ii];
            cd[6 * i + 2][tid] = pts[2 * N + ii];
            cd[6 * i + 3][tid] = nrm[ii];
            cd[6 * i + 4][tid] = nrm[N + ii];
            cd[6 * i + 5][tid] = nrm[2 * N + ii];
        }
        if (!valid) {
            verdict[sid] = 0;
            tstar[sid] = __builtin_nan("");
            continue;
        }
        int status = 0;
        const double ts = lp_lane<KM, false, MC>(cd, tid, kc, m, mu, rho, max_pivots, cs, status);
        verdict[sid] = (status == 0 && ts <= eps) ? 1 : 0;
        tstar[sid] = status == 0 ? ts : __builtin_nan("");
    }
}

template <int KM, int MC>
__global__ void __launch_bounds__(256)
k_verdict_lane(const float *__restrict__ pts, const float *__restrict__ nrm, int N, const int32_t *__restrict__ set_pt,
               const int32_t *__restrict__ palm_pt, const int32_t *__restrict__ valid_poses,
               const int32_t *__restrict__ n_valid_poses, int D, int k, int m, double mu, double rho, double eps,
               int max_pivots, LpConst cs, uint8_t *__restrict__ verdict, double *__restrict__ tstar)
{
    __shared__ float cd[KM * 6][256];
    verdict_sets<KM, MC>(cd, blockIdx.x, gridDim.x, pts, nrm, N, set_pt, palm_pt, valid_poses, n_valid_poses, D, k, m,
                         mu, rho, eps, max_pivots, cs, verdict, tstar);
}

template <int KM, int MC>
__global__ void __launch_bounds__(256)
k_verdict_batch(const ChunkDesc *__restrict__ d, const uint16_t *__restrict__ idx, const uint32_t *__restrict__ first,
                int n)
{
    __shared__ float cd[KM * 6][256];
    const int j = batch_member(first, n, blockIdx.x);
    const ChunkDesc &c = d[idx[j]];
    verdict_sets<KM, MC>(cd, blockIdx.x - first[j], first[j + 1] - first[j], c.pts, c.nrm, c.N, c.set_pt, nullptr,
                     c.valid_poses, c.n_valid_poses, c.D, c.k, c.m, c.mu, c.rho, c.eps, c.max_pivots, c.cs, c.verdict,
                     c.tstar);
}

// ---- contact-point optimisation (Sec. 5.4, Alg. 2) ---------------------------
// A uniform cell grid over the object's points serves the projection of a
// candidate onto a contact domain (nearest domain point).  Cells are cubes of
// edge c = max(sigma, extent / kGridMax); points are bucketed by a counting
// sort.  The search scans shells of cells at Chebyshev distance R = 0, 1, ...
// around the candidate's cell; points in unscanned cells are at least R c away,
// so once the best distance is below R c (less a rounding margin) it is exact
// (project_domain_wave).  Distances are FP64, ties go to the lowest point index.
constexpr int kGridMax = 64;
constexpr uint32_t kPurposeOpt = 5u;
constexpr double kOptTau = 1e-9;  // candidates within kOptTau of the best criterion value tie

struct GridDev {
    float lo[3];
    float cell, inv_cell;
    int dims[3];
};

__global__ void __launch_bounds__(1024)
k_grid_setup(const float *__restrict__ pts, int N, float sigma, GridDev *__restrict__ gd)
{
    __shared__ float red[6][1024];
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = threadIdx.x; i < N; i += blockDim.x)
        for (int a = 0; a < 3; ++a) {
            mn[a] = fminf(mn[a], pts[a * N + i]);
            mx[a] = fmaxf(mx[a], pts[a * N + i]);
        }
    for (int a = 0; a < 3; ++a) {
        red[a][threadIdx.x] = mn[a];
        red[3 + a][threadIdx.x] = mx[a];
    }
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int a = 0; a < 3; ++a) {
                red[a][threadIdx.x] = fminf(red[a][threadIdx.x], red[a][threadIdx.x + w]);
                red[3 + a][threadIdx.x] = fmaxf(red[3 + a][threadIdx.x], red[3 + a][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        float ext = 0.0f;
        for (int a = 0; a < 3; ++a) ext = fmaxf(ext, red[3 + a][0] - red[a][0]);
        const float c = fmaxf(fmaxf(sigma, ext / (float)kGridMax), 1e-4f);
        GridDev g;
        g.cell = c;
        g.inv_cell = 1.0f / c;
        for (int a = 0; a < 3; ++a) {
            g.lo[a] = red[a][0];
            g.dims[a] = min(kGridMax + 1, (int)((red[3 + a][0] - red[a][0]) * g.inv_cell) + 1);
        }
        *gd = g;
    }
}

__device__ inline int grid_coord(const GridDev &g, int a, float x)
{
    return (int)floorf((x - g.lo[a]) * g.inv_cell);
}

__device__ inline int point_cell(const GridDev &g, const float *pts, int N, int i)
{
    int c[3];
    for (int a = 0; a < 3; ++a) c[a] = min(max(grid_coord(g, a, pts[a * N + i]), 0), g.dims[a] - 1);
    return (c[2] * g.dims[1] + c[1]) * g.dims[0] + c[0];
}

__global__ void k_fill_u32(uint32_t *__restrict__ a, int64_t n, uint32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

__global__ void k_grid_count(const float *__restrict__ pts, int N, const GridDev *__restrict__ gd,
                             uint32_t *__restrict__ cell_count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) atomicAdd(&cell_count[point_cell(*gd, pts, N, i)], 1u);
}

// single workgroup: exclusive scan of the cell counts (cell_start[n_cells] = N)
__global__ void __launch_bounds__(1024)
k_grid_scan(uint32_t *__restrict__ cell_count, const GridDev *__restrict__ gd, uint32_t *__restrict__ cell_start)
{
    __shared__ uint32_t tot[1024];
    const int nc = gd->dims[0] * gd->dims[1] * gd->dims[2];
    const int per = (nc + 1023) / 1024, b0 = threadIdx.x * per;
    uint32_t s = 0;
    for (int i = b0; i < min(nc, b0 + per); ++i) s += cell_count[i];
    tot[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int t = 0; t < 1024; ++t) {
            const uint32_t v = tot[t];
            tot[t] = run;
            run += v;
        }
        cell_start[nc] = run;
    }
    __syncthreads();
    uint32_t run = tot[threadIdx.x];
    for (int i = b0; i < min(nc, b0 + per); ++i) {
        const uint32_t v = cell_count[i];
        cell_start[i] = run;
        cell_count[i] = run;  // becomes the scatter cursor
        run += v;
    }
}

// the points of each cell, contiguous: (x, y, z, point index as bits)
__global__ void k_grid_scatter(const float *__restrict__ pts, int N, const GridDev *__restrict__ gd,
                               uint32_t *__restrict__ cursor, float4 *__restrict__ cell_pts)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N)
        cell_pts[atomicAdd(&cursor[point_cell(*gd, pts, N, i)], 1u)] =
            make_float4(pts[i], pts[N + i], pts[2 * N + i], __int_as_float(i));
}

__device__ inline bool dom_has(const uint32_t *dom, int i) { return (dom[i >> 5] >> (i & 31)) & 1u; }

// Nearest domain point to y given a domain point `inc` (the contact's current
// point): FP64 distances, lowest index on ties, with inc as the incumbent.
// The 64 lanes of a wave project one candidate together (all arguments are
// wave-uniform), so the lanes never wait on each other's scans.  Shells of
// cells at Chebyshev distance R = 0, 1, ... around y's cell are scanned while
// R - 1 cell edges can still beat the best distance (the scan ends by R =
// ceil(|y - inc| / c) + 1; the whole domain is scanned only past
// kProjShellsInc shells).  In one pass each lane takes one cell position of
// the shell and keeps it if its box lies within the best distance; the kept
// cells' points are then spread over the lanes, 64 points per step, in the
// order of the lanes' running counts (a DPP scan).  A step's points that beat
// the best are checked against the domain bits and the wave takes their
// minimum (distance, then index) by DPP.  The box and shell tests run in
// float, in cell units, against lim = (sqrt(best) + 1e-6 m) / c rounded up by
// a relative 1e-5: points are binned in float, and the 1e-6 m of slack covers
// both that binning and the float tests, so a skipped cell never holds a
// point that could win.  The incumbent's distance and the centre cell's range
// come in with the candidate (each lane reads them for its own candidate).
constexpr int kProjShellsInc = 8;

__device__ inline double wave_bcast(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// DPP move of both halves of a double; lanes without a source keep v
template <int C, int RM = 0xf>
__device__ inline double dpp_d(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = (int)(uint32_t)b, hi = (int)(b >> 32);
    const int nlo = __builtin_amdgcn_update_dpp(lo, lo, C, RM, 0xf, false);
    const int nhi = __builtin_amdgcn_update_dpp(hi, hi, C, RM, 0xf, false);
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)nhi << 32) | (uint32_t)nlo));
}

// minimum over the wave, valid in lane 63: quad swaps, row rotations by 4
// and 8, then rows 0+1 and 2+3 and the halves joined by the row broadcasts
__device__ inline double wave_min63(double v)
{
    v = fmin(v, dpp_d<0xB1>(v));        // quad_perm [1, 0, 3, 2]
    v = fmin(v, dpp_d<0x4E>(v));        // quad_perm [2, 3, 0, 1]
    v = fmin(v, dpp_d<0x124>(v));       // row_ror:4
    v = fmin(v, dpp_d<0x128>(v));       // row_ror:8
    v = fmin(v, dpp_d<0x142, 0xA>(v));  // row_bcast:15 into rows 1 and 3
    v = fmin(v, dpp_d<0x143, 0xC>(v));  // row_bcast:31 into rows 2 and 3
    return v;
}

// inclusive prefix sum over the lanes (row shifts by 1, 2, 4, 8, then the row
// broadcasts); lanes without a source add 0
__device__ inline uint32_t wave_scan_incl(uint32_t x)
{
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);  // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);  // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);  // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);  // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return x;
}

// the minimum of (d2, i) over the lanes with `take` (lexicographic), folded
// into (best, bi); every lane returns the same result
__device__ inline void wave_lexmin(bool take, double d2, int i, double &best, int &bi)
{
    const unsigned long long m = __ballot(take);
    if (!m) return;
    double v;
    int ib;
    if (__popcll(m) == 1) {
        const int l = __builtin_ctzll(m);
        v = wave_bcast(d2, l);
        ib = __builtin_amdgcn_readlane(i, l);
    } else {
        v = wave_bcast(wave_min63(take ? d2 : INFINITY), 63);
        const unsigned long long t = __ballot(take && d2 == v);
        ib = __builtin_amdgcn_readlane(i, __builtin_ctzll(t));
        for (unsigned long long r = t & (t - 1); r; r &= r - 1)  // equal distances: the lowest index
            ib = min(ib, __builtin_amdgcn_readlane(i, __builtin_ctzll(r)));
    }
    if (v < best || (v == best && ib < bi)) {
        best = v;
        bi = ib;
    }
}

// position p of the shell at Chebyshev distance R >= 1 (side s = 2R + 1):
// the two z faces (s^2 each), then a ring of 4(s - 1) cells per inner z slab
__device__ inline void shell_pos(int R, int p, int &dx, int &dy, int &dz)
{
    const int s = 2 * R + 1, s2 = s * s;
    if (p < 2 * s2) {
        const bool hi = p >= s2;
        dz = hi ? R : -R;
        const int r = p - (hi ? s2 : 0), ry = r / s;
        dy = ry - R;
        dx = r - ry * s - R;
    } else {
        const int q = p - 2 * s2, ring = 4 * (s - 1), sl = q / ring, t = q - sl * ring, e = t / (s - 1),
                  o = t - e * (s - 1);
        dz = sl - R + 1;
        dx = e == 0 ? o - R : (e == 1 ? R : (e == 2 ? R - o : -R));
        dy = e == 0 ? -R : (e == 1 ? o - R : (e == 2 ? R : R - o));
    }
}

// best: the incumbent's squared distance; [cq0, cq0 + ccnt): the records of
// y's own cell (empty when y lies outside the grid)
__device__ int project_domain_wave(const GridDev &g, const uint32_t *__restrict__ cell_start,
                                   const float4 *__restrict__ cell_pts, const float *__restrict__ pts, int N,
                                   const uint32_t *__restrict__ dom, double yx, double yy, double yz, int inc,
                                   double best, uint32_t cq0, uint32_t ccnt, int lane)
{
    const double fx = (yx - g.lo[0]) * (double)g.inv_cell, fy = (yy - g.lo[1]) * (double)g.inv_cell,
                 fz = (yz - g.lo[2]) * (double)g.inv_cell;
    const int cx = (int)floor(fx), cy = (int)floor(fy), cz = (int)floor(fz);
    // y inside its cell, in cell units
    const float rx = (float)(fx - (double)cx), ry = (float)(fy - (double)cy), rz = (float)(fz - (double)cz);
    int bi = inc;
    float lim, lim2;
    auto set_lim = [&]() {
        lim = (float)((sqrt(best) + 1e-6) * (double)g.inv_cell) * 1.00001f;
        lim2 = lim * lim;
    };
    set_lim();
    // distance (cell units) from y to the slab of cells at offset o on one axis
    auto slab = [](int o, float r) { return o > 0 ? (float)o - r : (o < 0 ? (float)(-o - 1) + r : 0.0f); };
    for (int R = 0; R <= kProjShellsInc; ++R) {
        if (R > 0 && lim < (float)(R - 1)) return bi;  // shell R cannot hold a closer point
        const int s = 2 * R + 1, n_pos = R == 0 ? 1 : s * s * s - (s - 2) * (s - 2) * (s - 2);
        for (int p0 = 0; p0 < n_pos; p0 += 64) {
            // this lane's cell position: kept if inside the grid and within lim
            uint32_t q0 = 0, cnt = 0;
            if (R == 0) {
                if (lane == 0) {
                    q0 = cq0;
                    cnt = ccnt;
                }
            } else if (p0 + lane < n_pos) {
                int dx, dy, dz;
                if (R == 1) {  // the 26 neighbours: the 3 x 3 x 3 block less its centre (constant divisors)
                    const int q = lane + (lane >= 13 ? 1 : 0);
                    dx = q % 3 - 1;
                    dy = (q / 3) % 3 - 1;
                    dz = q / 9 - 1;
                } else {
                    shell_pos(R, p0 + lane, dx, dy, dz);
                }
                const int x = cx + dx, yv = cy + dy, z = cz + dz;
                const float bx = slab(dx, rx), by = slab(dy, ry), bz = slab(dz, rz);
                if (x >= 0 && x < g.dims[0] && yv >= 0 && yv < g.dims[1] && z >= 0 && z < g.dims[2] &&
                    bx * bx + by * by + bz * bz <= lim2) {
                    const int cc = (z * g.dims[1] + yv) * g.dims[0] + x;
                    q0 = cell_start[cc];
                    cnt = cell_start[cc + 1] - q0;
                }
            }
            // lane l's points are [ex, ex + cnt) of the pass's running count
            const uint32_t incl = wave_scan_incl(cnt), ex = incl - cnt;
            const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
            for (uint32_t b0 = 0; b0 < total; b0 += 64) {
                const uint32_t f = b0 + (uint32_t)lane;
                // the record of point f: the kept cells whose ranges meet this
                // step, in lane order (the last one starting at or before f owns it)
                uint32_t rec = 0;
                for (unsigned long long km = __ballot(cnt > 0 && ex < b0 + 64u && incl > b0); km; km &= km - 1) {
                    const int l = __builtin_ctzll(km);
                    const uint32_t lex = (uint32_t)__builtin_amdgcn_readlane((int)ex, l);
                    const uint32_t lq0 = (uint32_t)__builtin_amdgcn_readlane((int)q0, l);
                    if (f >= lex) rec = lq0 + (f - lex);
                }
                bool take = false;
                double d2 = INFINITY;
                int i = INT_MAX;
                if (f < total) {
                    const float4 v = cell_pts[rec];
                    i = __float_as_int(v.w);
                    const double ex3 = (double)v.x - yx, ey3 = (double)v.y - yy, ez3 = (double)v.z - yz;
                    d2 = ex3 * ex3 + ey3 * ey3 + ez3 * ez3;
                    take = (d2 < best || (d2 == best && i < bi)) && dom_has(dom, i);
                }
                const double old = best;
                wave_lexmin(take, d2, i, best, bi);
                if (best != old) set_lim();
            }
        }
    }
    if (sqrt(best) < (double)kProjShellsInc * g.cell - 1e-6) return bi;
    // beyond the shells: every domain point, words spread over the lanes
    const int NW = (N + 31) >> 5;
    double lb = INFINITY;
    int li = INT_MAX;
    for (int w = lane; w < NW; w += 64) {
        uint32_t x = dom[w];
        while (x) {
            const int b = __ffs(x) - 1;
            x &= x - 1u;
            const int i = w * 32 + b;
            const double ex3 = (double)pts[i] - yx, ey3 = (double)pts[N + i] - yy, ez3 = (double)pts[2 * N + i] - yz;
            const double d2 = ex3 * ex3 + ey3 * ey3 + ez3 * ez3;
            if (d2 < lb || (d2 == lb && i < li)) {
                lb = d2;
                li = i;
            }
        }
    }
    wave_lexmin(li != INT_MAX, lb, li, best, bi);
    return bi;
}


// Alg. 2, the candidates of one round (Sec. 5.4): one candidate per
// (set, contact i, candidate j).  Contact i's candidates are drawn around its
// point at the start of the round (contact i moves only at its own step), so
// a round's projections are independent of its criterion evaluations and run
// here, before them: y = p_i + dx x_i + dy y_i with (dx, dy) = sigma *
// Box-Muller of Philox block (g + pose_offset, d, 5 | step << 8, request_id),
// step = (round k + i) n_inner + j, and cand = the nearest point of contact
// i's domain (incumbent p_i).  cands[((t k + i) n_inner + j)], t = the set's
// rank among the sets of valid poses; -1 for sets not drawn.  Each lane draws
// one candidate; the wave then projects its 64 candidates one after another,
// all lanes together (project_domain_wave).  Eight waves per SIMD (64 VGPRs;
// the candidate set-up spills a few) hide more of the scans' load latency.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8)))
k_opt_project(const float *__restrict__ pts, const float *__restrict__ nrm, int N,
              const int32_t *__restrict__ valid_poses, const int32_t *__restrict__ n_valid_poses,
              const uint32_t *__restrict__ dom_bits, const uint32_t *__restrict__ dom_count,
              const int32_t *__restrict__ palm_pt, int F, int D, int k, int round, int n_inner, double sigma,
              uint32_t seed_lo, uint32_t seed_hi, uint32_t request_id, int64_t pose_offset,
              const GridDev *__restrict__ gdp, const uint32_t *__restrict__ cell_start,
              const float4 *__restrict__ cell_pts, const int32_t *__restrict__ set_pt, int32_t *__restrict__ cands)
{
    const GridDev g = *gdp;
    const int NW = (N + 31) >> 5;
    const int lane = threadIdx.x & 63;
    const int64_t per_set = (int64_t)k * n_inner;
    const int64_t n_total = (int64_t)(*n_valid_poses) * D * per_set;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // the loop bound is uniform over the wave (u - lane is the wave's first candidate)
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u - lane < n_total; u += stride) {
        bool live = false;
        double yx = 0.0, yy = 0.0, yz = 0.0, best0 = 0.0;
        int inc = 0;
        int64_t dom_off = 0;
        uint32_t cq0 = 0, ccnt = 0;  // the records of y's own cell
        if (u < n_total) {
            const int64_t t = u / per_set;
            const int rem = (int)(u - t * per_set), i = rem / n_inner, j = rem - i * n_inner;
            const int64_t pg = valid_poses[t / D];
            const int d = (int)(t % D);
            const int32_t *sp = set_pt + (pg * D + d) * k;
            const uint32_t fm = choose_fingers(eligible_fingers(dom_count, pg, F), k, (uint32_t)(pose_offset + pg),
                                               d, request_id, seed_lo, seed_hi);
            const int pc = palm_pt ? palm_pt[pg] : -1;
            bool drawn = fm != 0 && pc < N;
            for (int q = 0; q < k; ++q) drawn &= sp[q] >= 0 && sp[q] < N;
            if (!drawn) {
                cands[u] = -1;
            } else {
                live = true;
                inc = sp[i];
                const double px = pts[inc], py = pts[N + inc], pz = pts[2 * N + inc];
                double tx[3], ty[3];
                duff_basis(nrm[inc], nrm[N + inc], nrm[2 * N + inc], tx, ty);
                uint32_t w[4];
                const uint32_t step = (uint32_t)((round * k + i) * n_inner + j);
                philox4x32_10((uint32_t)(pose_offset + pg), (uint32_t)d, kPurposeOpt | (step << 8), request_id,
                              seed_lo, seed_hi, w);
                const double u1 = ((double)(w[0] >> 8) + 1.0) * (1.0 / 16777216.0);
                const double u2 = (double)(w[1] >> 8) * (1.0 / 16777216.0);
                const double rr = sqrt(-2.0 * log(u1));
                const double dx = sigma * rr * cos(2.0 * M_PI * u2), dy = sigma * rr * sin(2.0 * M_PI * u2);
                yx = px + dx * tx[0] + dy * ty[0];
                yy = py + dx * tx[1] + dy * ty[1];
                yz = pz + dx * tx[2] + dy * ty[2];
                dom_off = (pg * F + select_in_word(fm, (uint32_t)i)) * NW;  // contact i's finger
                {
                    const double ex = px - yx, ey = py - yy, ez = pz - yz;
                    best0 = ex * ex + ey * ey + ez * ez;
                }
                const int cx = (int)floor((yx - g.lo[0]) * (double)g.inv_cell),
                          cy = (int)floor((yy - g.lo[1]) * (double)g.inv_cell),
                          cz = (int)floor((yz - g.lo[2]) * (double)g.inv_cell);
                if (cx >= 0 && cx < g.dims[0] && cy >= 0 && cy < g.dims[1] && cz >= 0 && cz < g.dims[2]) {
                    const int cc = (cz * g.dims[1] + cy) * g.dims[0] + cx;
                    cq0 = cell_start[cc];
                    ccnt = cell_start[cc + 1] - cq0;
                }
            }
        }
        int res = -1;
        for (unsigned long long todo = __ballot(live); todo; todo &= todo - 1) {
            const int c = __builtin_ctzll(todo);
            const int64_t off = ((int64_t)__builtin_amdgcn_readlane((int)(dom_off >> 32), c) << 32) |
                                (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)dom_off, c);
            const int r = project_domain_wave(
                g, cell_start, cell_pts, pts, N, dom_bits + off, wave_bcast(yx, c), wave_bcast(yy, c),
                wave_bcast(yz, c), __builtin_amdgcn_readlane(inc, c), wave_bcast(best0, c),
                (uint32_t)__builtin_amdgcn_readlane((int)cq0, c), (uint32_t)__builtin_amdgcn_readlane((int)ccnt, c),
                lane);
            if (lane == c) res = r;
        }
        if (live) cands[u] = res;
    }
}

// Alg. 2, the criterion side of one round: a group of GS = pow2 >= n_inner
// lanes per set (lane = candidate), grid-stride over the sets of poses with
// non-empty domains.  Contacts i = 0..k-1 in turn: each lane evaluates the LP
// of the set with contact i at its candidate (cands of k_opt_project), the
// group takes the minimum by xor-shuffles and the first lane within kOptTau
// of it by one ballot; contact i moves there.  The set's points are written
// back after the round; tstar (the last step's J) and, after the last round,
// the verdict.
template <int KM, int GS, int MC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_optimize(const float *__restrict__ pts, const float *__restrict__ nrm, int N, const int32_t *__restrict__ valid_poses,
           const int32_t *__restrict__ n_valid_poses, const uint32_t *__restrict__ dom_count,
           const int32_t *__restrict__ palm_pt, int F, int D, int k, int m, double mu, double rho, double eps,
           int max_pivots, LpConst cs, int n_inner, bool last, uint32_t seed_lo, uint32_t seed_hi,
           uint32_t request_id, int64_t pose_offset, const int32_t *__restrict__ cands, int32_t *__restrict__ set_pt,
           uint8_t *__restrict__ verdict, double *__restrict__ tstar)
{
    __shared__ float cd[KM * 6][256];
    __shared__ int cur[KM][256];  // the set's current point indices (every lane of a group holds them)
    __shared__ int wbs[7][256];   // per lane: the warm basis of its LP in, its final basis out
    __shared__ int cbs[7][256];   // per lane: the current set's optimal basis (the last pick's)
    const int tid = threadIdx.x, lane = tid & 63, j = tid % GS, gbase = lane - j;
    const int wbase = tid - lane;  // first thread of this wave
    const int64_t n_work = (int64_t)(*n_valid_poses) * D;
    const int64_t groups = ((int64_t)gridDim.x * blockDim.x) / GS;
    auto load = [&](int ci, int idx) {
        cd[6 * ci + 0][tid] = pts[idx];
        cd[6 * ci + 1][tid] = pts[N + idx];
        cd[6 * ci + 2][tid] = pts[2 * N + idx];
        cd[6 * ci + 3][tid] = nrm[idx];
        cd[6 * ci + 4][tid] = nrm[N + idx];
        cd[6 * ci + 5][tid] = nrm[2 * N + idx];
    };
    for (int64_t t = ((int64_t)blockIdx.x * blockDim.x + tid) / GS; t < n_work; t += groups) {
        const int64_t pg = valid_poses[t / D];
        const int d = (int)(t % D);
        const int64_t sid = pg * D + d;
        int32_t *sp = set_pt + sid * k;
        const uint32_t fm = choose_fingers(eligible_fingers(dom_count, pg, F), k, (uint32_t)(pose_offset + pg), d,
                                           request_id, seed_lo, seed_hi);
        const int pc = palm_pt ? palm_pt[pg] : -1;  // fixed palm contact (-1: none)
        const int kc = pc >= 0 ? k + 1 : k;
        bool drawn = fm != 0 && pc < N;
        for (int i = 0; i < k; ++i) drawn &= sp[i] >= 0 && sp[i] < N;
        if (!drawn) {  // not a drawn set (inconsistent domain sizes): no criterion
            if (j == 0) {
                verdict[sid] = 0;
                tstar[sid] = __builtin_nan("");
            }
            continue;  // uniform over the group
        }
        for (int i = 0; i < k; ++i) {
            cur[i][tid] = sp[i];
            load(i, sp[i]);
        }
        if (pc >= 0) load(k, pc);
        double J = INFINITY;
        // optimal basis of the current set (the last pick's), the warm start of
        // the next contact's candidates; none before the round's first pick
        cbs[0][tid] = -1;
        for (int i = 0; i < k; ++i) {
            int cand = -1;
            double Jc = INFINITY;
#pragma unroll
            for (int r = 0; r < 7; ++r) wbs[r][tid] = cbs[r][tid];
            if (j < n_inner) {
                cand = cands[(t * k + i) * n_inner + j];
                if (cand >= 0) {  // always, for a drawn set (its domains are non-empty)
                    load(i, cand);
                    int st = 0;
                    Jc = lp_lane<KM, true, MC>(cd, tid, kc, m, mu, rho, max_pivots, cs, st, wbs);
                    if (st != 0) Jc = INFINITY;
                }
            }
            double mn = Jc;
            for (int off = GS >> 1; off > 0; off >>= 1) mn = fmin(mn, __shfl_xor(mn, off, GS));
            const unsigned long long ok = __ballot(Jc <= mn + kOptTau);
            const int js = __ffsll((long long)((ok >> gbase) & ((GS == 64) ? ~0ull : ((1ull << GS) - 1)))) - 1;
            const int pick = __shfl(cand, gbase + js, 64);
            const double Jp = __shfl(Jc, gbase + js, 64);
            if (pick >= 0) {
                J = Jp;
                cur[i][tid] = pick;
                // the picked lane's final basis (written by that lane of this wave)
                if (!isinf(Jp)) {
#pragma unroll
                    for (int r = 0; r < 7; ++r) cbs[r][tid] = wbs[r][wbase + gbase + js];
                }
            }
            load(i, cur[i][tid]);
        }
        if (j == 0) {
            for (int i = 0; i < k; ++i) sp[i] = cur[i][tid];
            tstar[sid] = isinf(J) ? __builtin_nan("") : J;
            if (last) verdict[sid] = J <= eps ? 1 : 0;
        }
    }
}

// ---- Alg. 2 criteria with the slow LPs gathered into their own waves --------
// k_optimize runs a contact step's candidate LPs side by side, so each wave
// waits for the slowest of its 64 LPs at every step.  Most warm-started LPs
// end within a pivot or two of the warm basis, but about a third need many
// more.  With a workspace that holds a step's candidate results, each
// contact step takes three launches instead: every candidate's LP stopped
// after kOptEasyPivots simplex pivots (kOptColdPivots at a round's first
// step, which has no warm basis) (k_opt_try); the LPs not finished by then
// queued and solved again from the same start with the full pivot cap, in
// waves of slow LPs only (k_opt_hard); then each set's pick (k_opt_pick).
// A capped run is a prefix of the full run from the same start, so t*, the
// final bases and the picks are those of k_optimize.  (Caps measured at c3,
// search stage: 1, 2, 4, 8, 12, 16 warm pivots 119, 117, 112, 110, 113,
// 117 ms with the cold step uncapped; with 8 warm, 10, 14, 20 cold pivots
// 108.6, 107.5, 109.7 ms.)
constexpr int kOptEasyPivots = 8;
constexpr int kOptColdPivots = 14;

struct OptSplit {
    double *sJ;          // per set: criterion value of its last pick (INF before any)
    int32_t *sB;         // per set: 7 basis column ids of its last finite pick (-1: none yet)
    double *cJ;          // per candidate (set t, candidate j at t * n_inner + j): t*, INF if unsolved
    int32_t *cB;         // per candidate: the 7 column ids of its final basis
    int32_t *queue;      // candidates whose LP needs more than kOptEasyPivots pivots
    uint32_t *n_queue;   // queue length, one counter per contact step
};

// Set t of the sets of poses with non-empty domains: its set id and whether it
// was drawn (the drawn-set test of k_optimize); kc = contacts with the palm's.
__device__ inline bool opt_set(int64_t t, const int32_t *__restrict__ valid_poses, const uint32_t *__restrict__ dom_count,
                               const int32_t *__restrict__ palm_pt, const int32_t *__restrict__ set_pt, int N, int F,
                               int D, int k, uint32_t seed_lo, uint32_t seed_hi, uint32_t request_id,
                               int64_t pose_offset, int64_t &sid, int &pc)
{
    const int64_t pg = valid_poses[t / D];
    const int d = (int)(t % D);
    sid = pg * D + d;
    const int32_t *sp = set_pt + sid * k;
    const uint32_t fm = choose_fingers(eligible_fingers(dom_count, pg, F), k, (uint32_t)(pose_offset + pg), d,
                                       request_id, seed_lo, seed_hi);
    pc = palm_pt ? palm_pt[pg] : -1;
    bool drawn = fm != 0 && pc < N;
    for (int i = 0; i < k; ++i) drawn &= sp[i] >= 0 && sp[i] < N;
    return drawn;
}

// LP of candidate j of set t at contact step i, from the set's current points
// (its own column of cd), warm-started from the set's last pick's basis
// (none at the round's first step); cap: the pivot cap of this run.
template <int KM, int MC>
__device__ inline double opt_cand_lp(float (&cd)[KM * 6][256], int (&wb)[7][256], int tid, int64_t t, int j, int i,
                                     const float *__restrict__ pts, const float *__restrict__ nrm, int N,
                                     const int32_t *__restrict__ valid_poses, const uint32_t *__restrict__ dom_count,
                                     const int32_t *__restrict__ palm_pt, int F, int D, int k, int m, double mu,
                                     double rho, int cap, const LpConst &cs, int n_inner, uint32_t seed_lo,
                                     uint32_t seed_hi, uint32_t request_id, int64_t pose_offset,
                                     const int32_t *__restrict__ cands, const int32_t *__restrict__ set_pt,
                                     const OptSplit &os, int &st)
{
    st = 3;  // no LP (not a drawn set, or no candidate)
    int64_t sid;
    int pc;
    if (!opt_set(t, valid_poses, dom_count, palm_pt, set_pt, N, F, D, k, seed_lo, seed_hi, request_id, pose_offset,
                 sid, pc))
        return INFINITY;
    const int cand = cands[(t * k + i) * n_inner + j];
    if (cand < 0) return INFINITY;
    auto load = [&](int ci, int idx) {
        cd[6 * ci + 0][tid] = pts[idx];
        cd[6 * ci + 1][tid] = pts[N + idx];
        cd[6 * ci + 2][tid] = pts[2 * N + idx];
        cd[6 * ci + 3][tid] = nrm[idx];
        cd[6 * ci + 4][tid] = nrm[N + idx];
        cd[6 * ci + 5][tid] = nrm[2 * N + idx];
    };
    const int32_t *sp = set_pt + sid * k;
    for (int c = 0; c < k; ++c) load(c, c == i ? cand : sp[c]);
    if (pc >= 0) load(k, pc);
#pragma unroll
    for (int r = 0; r < 7; ++r) wb[r][tid] = i == 0 ? -1 : os.sB[t * 7 + r];
    return lp_lane<KM, true, MC>(cd, tid, pc >= 0 ? k + 1 : k, m, mu, rho, cap, cs, st, wb);
}

template <int KM, int MC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_opt_try(const float *__restrict__ pts, const float *__restrict__ nrm, int N,
          const int32_t *__restrict__ valid_poses, const int32_t *__restrict__ n_valid_poses,
          const uint32_t *__restrict__ dom_count, const int32_t *__restrict__ palm_pt, int F, int D, int k, int m,
          double mu, double rho, int max_pivots, LpConst cs, int n_inner, int i, uint32_t seed_lo, uint32_t seed_hi,
          uint32_t request_id, int64_t pose_offset, const int32_t *__restrict__ cands,
          const int32_t *__restrict__ set_pt, OptSplit os)
{
    __shared__ float cd[KM * 6][256];
    __shared__ int wb[7][256];
    const int tid = threadIdx.x, lane = tid & 63;
    const int64_t n_cand = (int64_t)(*n_valid_poses) * D * n_inner;
    const int cap = min(max_pivots, i == 0 ? kOptColdPivots : kOptEasyPivots);
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + tid; g < n_cand; g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = g / n_inner;
        const int j = (int)(g - t * n_inner);
        int st;
        const double Jc = opt_cand_lp<KM, MC>(cd, wb, tid, t, j, i, pts, nrm, N, valid_poses, dom_count, palm_pt, F,
                                              D, k, m, mu, rho, cap, cs, n_inner, seed_lo, seed_hi, request_id,
                                              pose_offset, cands, set_pt, os, st);
        const bool slow = st == 1 && cap < max_pivots;
        if (!slow) {
            os.cJ[g] = st == 0 ? Jc : INFINITY;
#pragma unroll
            for (int r = 0; r < 7; ++r) os.cB[g * 7 + r] = wb[r][tid];
        }
        // one queue reservation per wave
        const unsigned long long sb = __ballot(slow);
        if (sb) {
            const int leader = __ffsll((long long)sb) - 1;
            uint32_t base = 0;
            if (lane == leader) base = atomicAdd(os.n_queue + i, (uint32_t)__popcll(sb));
            base = __shfl(base, leader, 64);
            if (slow) os.queue[base + __popcll(sb & ((1ull << lane) - 1))] = (int32_t)g;
        }
    }
}

template <int KM, int MC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_opt_hard(const float *__restrict__ pts, const float *__restrict__ nrm, int N,
           const int32_t *__restrict__ valid_poses, const uint32_t *__restrict__ dom_count,
           const int32_t *__restrict__ palm_pt, int F, int D, int k, int m, double mu, double rho, int max_pivots,
           LpConst cs, int n_inner, int i, uint32_t seed_lo, uint32_t seed_hi, uint32_t request_id,
           int64_t pose_offset, const int32_t *__restrict__ cands, const int32_t *__restrict__ set_pt, OptSplit os)
{
    __shared__ float cd[KM * 6][256];
    __shared__ int wb[7][256];
    const int tid = threadIdx.x;
    const int64_t n = os.n_queue[i];
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + tid; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t g = os.queue[q];
        const int64_t t = g / n_inner;
        const int j = (int)(g - t * n_inner);
        int st;
        const double Jc = opt_cand_lp<KM, MC>(cd, wb, tid, t, j, i, pts, nrm, N, valid_poses, dom_count, palm_pt, F,
                                              D, k, m, mu, rho, max_pivots, cs, n_inner, seed_lo, seed_hi,
                                              request_id, pose_offset, cands, set_pt, os, st);
        os.cJ[g] = st == 0 ? Jc : INFINITY;
#pragma unroll
        for (int r = 0; r < 7; ++r) os.cB[g * 7 + r] = wb[r][tid];
    }
}

// Each set's pick at contact step i: the lowest candidate within kOptTau of
// the best t* (the first candidate when none is finite), its point into the
// set, its basis the warm start of the next step when its t* is finite.
__global__ void k_opt_pick(const int32_t *__restrict__ valid_poses, const int32_t *__restrict__ n_valid_poses,
                           const uint32_t *__restrict__ dom_count, const int32_t *__restrict__ palm_pt, int N, int F,
                           int D, int k, int n_inner, int i, bool last, double eps, uint32_t seed_lo,
                           uint32_t seed_hi, uint32_t request_id, int64_t pose_offset,
                           const int32_t *__restrict__ cands, int32_t *__restrict__ set_pt,
                           uint8_t *__restrict__ verdict, double *__restrict__ tstar, OptSplit os)
{
    const int64_t n_work = (int64_t)(*n_valid_poses) * D;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_work;
         t += (int64_t)gridDim.x * blockDim.x) {
        int64_t sid;
        int pc;
        if (!opt_set(t, valid_poses, dom_count, palm_pt, set_pt, N, F, D, k, seed_lo, seed_hi, request_id,
                     pose_offset, sid, pc)) {
            verdict[sid] = 0;  // not a drawn set: no criterion
            tstar[sid] = __builtin_nan("");
            continue;
        }
        const double *cj = os.cJ + t * n_inner;
        double mn = INFINITY;
        for (int j = 0; j < n_inner; ++j) mn = fmin(mn, cj[j]);
        int js = -1;
        for (int j = n_inner - 1; j >= 0; --j)
            if (cj[j] <= mn + kOptTau) js = j;
        const int pick = js >= 0 ? cands[(t * k + i) * n_inner + js] : -1;
        double J = i == 0 ? INFINITY : os.sJ[t];
        if (i == 0) os.sB[t * 7] = -1;
        if (pick >= 0) {
            J = cj[js];
            set_pt[sid * k + i] = pick;
            if (!isinf(J)) {
#pragma unroll
                for (int r = 0; r < 7; ++r) os.sB[t * 7 + r] = os.cB[(t * n_inner + js) * 7 + r];
            }
        }
        os.sJ[t] = J;
        if (i == k - 1) {
            tstar[sid] = isinf(J) ? __builtin_nan("") : J;
            if (last) verdict[sid] = J <= eps ? 1 : 0;
        }
    }
}

// links of the (moved) contacts of every set of a pose with non-empty domains,
// picked with the set's draw words exactly as k_draw does
__global__ void k_relink(DevHand H, const uint32_t *__restrict__ bits, const float *__restrict__ pts,
                         const float *__restrict__ nrm, int N, const float *__restrict__ poses,
                         const int32_t *__restrict__ valid_poses, const int32_t *__restrict__ n_valid_poses,
                         const uint32_t *__restrict__ dom_count, int D, int k, uint32_t seed_lo, uint32_t seed_hi,
                         uint32_t request_id, int64_t pose_offset, const int32_t *__restrict__ set_pt,
                         int8_t *__restrict__ set_link)
{
    const int64_t n_work = (int64_t)(*n_valid_poses) * D;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_work;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t g = valid_poses[t / D];
        const int d = (int)(t % D);
        uint32_t w[16];
        for (int blk = 0; blk * 4 < 2 * k; ++blk)
            philox4x32_10((uint32_t)(pose_offset + g), (uint32_t)(4 * d + blk), kPurposeDraw, request_id, seed_lo,
                          seed_hi, w + 4 * blk);
        const int32_t *sp = set_pt + (g * D + d) * k;
        int8_t *sl = set_link + (g * D + d) * k;
        uint32_t fm = choose_fingers(eligible_fingers(dom_count, g, H.F), k, (uint32_t)(pose_offset + g), d,
                                     request_id, seed_lo, seed_hi);
        for (int i = 0; i < k; ++i) {
            const int f = __ffs(fm) - 1;
            fm &= fm - 1u;
            const int idx = sp[i];
            sl[i] = (int8_t)((f >= 0 && idx >= 0 && idx < N)
                                 ? pick_link(H, bits, H.bin_c, pts, nrm, N, poses + 12 * g, f, idx, w[k + i])
                                 : -1);
        }
    }
}

// ---- second contact round (Sec. 5.3, additional search phase; Sec. 5.6) -------
// Finger of link l (its joint's finger).
__device__ inline int link_finger(const DevHand &H, int l)
{
    for (int f = 0; f < H.F; ++f)
        if (l >= H.finger_first[f] && l < H.finger_first[f] + H.finger_dof[f]) return f;
    return -1;
}

// One workgroup per pose.  A round-1 set (k1 contacts) is extended when it is
// listed (list: sorted set ids, list_ok[i] != 0 if given) or, without a list,
// when its draw is whole and its verdict 0; its contacts must all have a
// point and a link.  It gets k_add contacts on unused fingers with non-empty
// domains: the fingers by choose_fingers over them (Philox purpose 19), the
// points as the floor(w * count / 2^32)-th domain bit and the links by the
// reverse lookup (purpose 21: word i and k_add + i for the i-th new finger).
// The extended set lists its k1 + k_add contacts in increasing finger order.
// Sets not extended get set_pt -1, verdict 0, t* NaN; pose_valid[g] = some
// set of the pose was extended (its verdicts are computed next).
__global__ void __launch_bounds__(kDrawThreads)
k_extend(DevHand H, const uint32_t *__restrict__ bits, const float *__restrict__ pts, const float *__restrict__ nrm,
         int N, const float *__restrict__ poses, const uint32_t *__restrict__ dom_bits,
         const uint32_t *__restrict__ dom_count, int D, int k1, int k_add, const int32_t *__restrict__ set_pt1,
         const int8_t *__restrict__ set_link1, const uint8_t *__restrict__ verdict1, const int32_t *__restrict__ list,
         const int32_t *__restrict__ list_n, const uint8_t *__restrict__ list_ok, uint32_t seed_lo, uint32_t seed_hi,
         uint32_t request_id, int64_t pose_offset, int32_t *__restrict__ set_pt2, int8_t *__restrict__ set_link2,
         uint8_t *__restrict__ pose_valid, uint8_t *__restrict__ verdict2, double *__restrict__ tstar2)
{
    extern __shared__ uint32_t prefix[];  // [F][nsb + 1]
    __shared__ float cb[3 * kMaxBins];
    __shared__ uint32_t counts[kMaxFingers];
    __shared__ int32_t range[2];
    __shared__ uint32_t any;
    const int g = blockIdx.x, F = H.F, k2 = k1 + k_add;
    const int NW = (N + 31) >> 5, nsb = (NW + kSuper - 1) / kSuper;
    const uint32_t *dom = dom_bits + (int64_t)g * F * NW;
    for (int i = threadIdx.x; i < 3 * H.B; i += blockDim.x) cb[i] = H.bin_c[i];
    if ((int)threadIdx.x < F) counts[threadIdx.x] = dom_count[(int64_t)g * F + threadIdx.x];
    if (threadIdx.x == 0) {
        any = 0;
        range[0] = range[1] = 0;
        if (list) {  // this pose's entries: ids in [g D, (g + 1) D) of the sorted list
            const int n = *list_n;
            int lo = 0, hi = n;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if ((int64_t)list[mid] < (int64_t)g * D) lo = mid + 1; else hi = mid;
            }
            range[0] = lo;
            hi = n;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if ((int64_t)list[mid] < (int64_t)(g + 1) * D) lo = mid + 1; else hi = mid;
            }
            range[1] = lo;
        }
    }
    build_prefix(prefix, dom, F, NW, nsb);
    __syncthreads();
    const float *pose = poses + 12 * (int64_t)g;
    const uint32_t gg = (uint32_t)(pose_offset + g);
    for (int d = threadIdx.x; d < D; d += blockDim.x) {
        const int64_t sid = (int64_t)g * D + d;
        const int32_t *sp1 = set_pt1 + sid * k1;
        const int8_t *sl1 = set_link1 + sid * k1;
        int32_t *sp2 = set_pt2 + sid * k2;
        int8_t *sl2 = set_link2 + sid * k2;
        bool take;
        if (list) {
            int lo = range[0], hi = range[1];
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if ((int64_t)list[mid] < sid) lo = mid + 1; else hi = mid;
            }
            take = lo < range[1] && (int64_t)list[lo] == sid && (!list_ok || list_ok[lo] != 0);
        } else {
            take = verdict1[sid] == 0;
        }
        uint32_t used = 0;
        int fin1[8];
        for (int i = 0; i < k1 && take; ++i) {
            const int l = sl1[i];
            const int f = (l >= 0 && sp1[i] >= 0 && sp1[i] < N) ? link_finger(H, l) : -1;
            if (f < 0) take = false; else { fin1[i] = f; used |= 1u << f; }
        }
        uint32_t fm = 0;
        if (take) {
            uint32_t elig = 0;
            for (int f = 0; f < F; ++f) elig |= (counts[f] > 0 && !((used >> f) & 1u) ? 1u : 0u) << f;
            fm = choose_fingers(elig, k_add, gg, d, request_id, seed_lo, seed_hi, kPurposeExtFingers);
            take = fm != 0u;
        }
        if (!take) {
            for (int i = 0; i < k2; ++i) {
                sp2[i] = -1;
                sl2[i] = -1;
            }
            verdict2[sid] = 0;
            tstar2[sid] = __builtin_nan("");
            continue;
        }
        any = 1u;  // benign race: every writer stores 1
        uint32_t w[16];
        for (int blk = 0; blk * 4 < 2 * k_add; ++blk)
            philox4x32_10(gg, (uint32_t)(4 * d + blk), kPurposeExtDraw, request_id, seed_lo, seed_hi, w + 4 * blk);
        int np[8], nl[8], nf[8];
        for (int i = 0; i < k_add; ++i) {
            const int f = __ffs(fm) - 1;  // the i-th smallest new finger
            fm &= fm - 1u;
            const int idx = select_domain(prefix + f * (nsb + 1), nsb, dom + (int64_t)f * NW, NW,
                                          __umulhi(w[i], counts[f]));
            nf[i] = f;
            np[i] = idx;
            nl[i] = idx >= 0 ? pick_link(H, bits, cb, pts, nrm, N, pose, f, idx, w[k_add + i]) : -1;
        }
        // union in increasing finger order (both groups sorted)
        int a = 0, b = 0;
        for (int o = 0; o < k2; ++o) {
            if (b >= k_add || (a < k1 && fin1[a] < nf[b])) {
                sp2[o] = sp1[a];
                sl2[o] = sl1[a];
                ++a;
            } else {
                sp2[o] = np[b];
                sl2[o] = (int8_t)nl[b];
                ++b;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) pose_valid[g] = any ? 1 : 0;
}

// flag[s] = set s has every point and link and verdict 0 (an unstable set)
__global__ void k_flag_unstable(const int32_t *__restrict__ set_pt, const int8_t *__restrict__ set_link,
                                const uint8_t *__restrict__ verdict, int64_t n_sets, int k, uint8_t *__restrict__ flag)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_sets) return;
    bool ok = verdict[s] == 0;
    for (int i = 0; i < k; ++i) ok &= set_pt[s * k + i] >= 0 && set_link[s * k + i] >= 0;
    flag[s] = ok ? 1 : 0;
}

// ---- compaction ------------------------------------------------------------
// block bid: the number of nonzero flags in its kChunk flags
__device__ __forceinline__ void chunk_count_block(uint32_t *part, int64_t bid, const uint8_t *__restrict__ flag,
                                                  int64_t n, uint32_t *__restrict__ chunk_count)
{
    const int64_t base = bid * kChunk + (int64_t)threadIdx.x * kChunkPerThread;
    uint32_t c = 0;
    for (int i = 0; i < kChunkPerThread; ++i)
        if (base + i < n) c += flag[base + i] != 0;
    for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int w = 0; w < kCompactThreads / 64; ++w) s += part[w];
        chunk_count[bid] = s;
    }
}

// one block: exclusive scan of chunk counts, total into n_acc
__device__ __forceinline__ void chunk_scan_block(uint32_t *tot, const uint32_t *__restrict__ chunk_count,
                                                 int64_t n_chunks, uint32_t *__restrict__ chunk_off,
                                                 int32_t *__restrict__ n_acc)
{
    const int64_t per = (n_chunks + kCompactThreads - 1) / kCompactThreads;
    const int64_t b0 = threadIdx.x * per;
    uint32_t s = 0;
    for (int64_t i = b0; i < min(n_chunks, b0 + per); ++i) s += chunk_count[i];
    tot[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int t = 0; t < kCompactThreads; ++t) {
            const uint32_t v = tot[t];
            tot[t] = run;
            run += v;
        }
        *n_acc = (int32_t)run;
    }
    __syncthreads();
    uint32_t run = tot[threadIdx.x];
    for (int64_t i = b0; i < min(n_chunks, b0 + per); ++i) {
        chunk_off[i] = run;
        run += chunk_count[i];
    }
}

// block bid: the indices of its nonzero flags, in order, from chunk_off[bid]
__device__ __forceinline__ void chunk_scatter_block(uint32_t *pre, int64_t bid, const uint8_t *__restrict__ flag,
                                                    int64_t n, const uint32_t *__restrict__ chunk_off,
                                                    int32_t *__restrict__ list)
{
    const int64_t base = bid * kChunk + (int64_t)threadIdx.x * kChunkPerThread;
    uint32_t c = 0;
    for (int i = 0; i < kChunkPerThread; ++i)
        if (base + i < n) c += flag[base + i] != 0;
    pre[threadIdx.x] = c;
    __syncthreads();
    // Hillis-Steele inclusive scan over the block
    for (int off = 1; off < kCompactThreads; off <<= 1) {
        const uint32_t v = threadIdx.x >= off ? pre[threadIdx.x - off] : 0u;
        __syncthreads();
        pre[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t pos = chunk_off[bid] + pre[threadIdx.x] - c;
    for (int i = 0; i < kChunkPerThread; ++i)
        if (base + i < n && flag[base + i]) list[pos++] = (int32_t)(base + i);
}

__global__ void __launch_bounds__(kCompactThreads)
k_chunk_count(const uint8_t *__restrict__ verdict, int64_t n, uint32_t *__restrict__ chunk_count)
{
    __shared__ uint32_t part[kCompactThreads / 64];
    chunk_count_block(part, blockIdx.x, verdict, n, chunk_count);
}

__global__ void __launch_bounds__(kCompactThreads)
k_chunk_scan(const uint32_t *__restrict__ chunk_count, int64_t n_chunks, uint32_t *__restrict__ chunk_off,
             int32_t *__restrict__ n_acc)
{
    __shared__ uint32_t tot[kCompactThreads];
    chunk_scan_block(tot, chunk_count, n_chunks, chunk_off, n_acc);
}

__global__ void __launch_bounds__(kCompactThreads)
k_chunk_scatter(const uint8_t *__restrict__ verdict, int64_t n, const uint32_t *__restrict__ chunk_off,
                int32_t *__restrict__ acc_list)
{
    __shared__ uint32_t pre[kCompactThreads];
    chunk_scatter_block(pre, blockIdx.x, verdict, n, chunk_off, acc_list);
}

// Batched compaction: POSES = the chunk's poses with a usable draw (the
// verdict launch's work list), else its accepted sets.
struct CompactView {
    const uint8_t *flag;
    int64_t n;
    uint32_t *count, *off;
    int32_t *total, *list;
};

template <bool POSES>
__device__ __forceinline__ CompactView compact_view(const ChunkDesc &c)
{
    if (POSES) return {c.pose_valid, (int64_t)c.P, c.pchunk_count, c.pchunk_off, c.n_valid_poses, c.valid_poses};
    return {c.verdict, (int64_t)c.P * c.D, c.chunk_count, c.chunk_off, c.n_acc, c.acc};
}

template <bool POSES>
__global__ void __launch_bounds__(kCompactThreads)
k_count_batch(const ChunkDesc *__restrict__ d, const uint16_t *__restrict__ idx, const uint32_t *__restrict__ first,
              int n)
{
    __shared__ uint32_t part[kCompactThreads / 64];
    const int j = batch_member(first, n, blockIdx.x);
    const CompactView v = compact_view<POSES>(d[idx[j]]);
    chunk_count_block(part, blockIdx.x - first[j], v.flag, v.n, v.count);
}

template <bool POSES>
__global__ void __launch_bounds__(kCompactThreads)
k_scan_batch(const ChunkDesc *__restrict__ d, const uint16_t *__restrict__ idx, const uint32_t *__restrict__ first,
             int n)
{
    __shared__ uint32_t tot[kCompactThreads];
    const int j = batch_member(first, n, blockIdx.x);
    const CompactView v = compact_view<POSES>(d[idx[j]]);
    chunk_scan_block(tot, v.count, (v.n + kChunk - 1) / kChunk, v.off, v.total);
}

template <bool POSES>
__global__ void __launch_bounds__(kCompactThreads)
k_scatter_batch(const ChunkDesc *__restrict__ d, const uint16_t *__restrict__ idx, const uint32_t *__restrict__ first,
                int n)
{
    __shared__ uint32_t pre[kCompactThreads];
    const int j = batch_member(first, n, blockIdx.x);
    const CompactView v = compact_view<POSES>(d[idx[j]]);
    chunk_scatter_block(pre, blockIdx.x - first[j], v.flag, v.n, v.off, v.list);
}

}  // namespace lg

using namespace lg;

extern "C" {

// workspace: [set chunks: count, offset] [pose chunks: count, offset]
//            [valid pose list P] [n_valid_poses] [pose_valid P bytes]
//            and, for the contact-point optimisation, [grid params]
//            [cell counts/cursor (kGridMax+1)^3] [cell starts +1] [cell points N: xyz + index]
//            [a round's candidates P D k n_inner]
struct SearchWs {
    uint32_t *chunk_count, *chunk_off, *pchunk_count, *pchunk_off;
    int32_t *valid_poses, *n_valid_poses;
    uint8_t *pose_valid;
    GridDev *grid;
    uint32_t *cell_count, *cell_start;
    float4 *cell_pts;
    int32_t *cands;
    OptSplit split;   // arrays of the gathered-slow-LP criteria (null when not laid out)
    size_t bytes;
};

static SearchWs search_ws(void *base, int64_t n_points, int64_t n_poses, int64_t draws, bool opt, int64_t k = 0,
                          int64_t n_inner = 0, bool split = false)
{
    const int64_t n_sets = n_poses * draws;
    const int64_t nc = (n_sets + kChunk - 1) / kChunk, npc = (n_poses + kChunk - 1) / kChunk;
    SearchWs w;
    uint32_t *u = static_cast<uint32_t *>(base);
    w.chunk_count = u;
    w.chunk_off = u + nc;
    w.pchunk_count = u + 2 * nc;
    w.pchunk_off = u + 2 * nc + npc;
    w.valid_poses = reinterpret_cast<int32_t *>(u + 2 * nc + 2 * npc);
    w.n_valid_poses = w.valid_poses + n_poses;
    w.pose_valid = reinterpret_cast<uint8_t *>(w.n_valid_poses + 1);
    size_t off = ((size_t)(2 * nc + 2 * npc + n_poses + 1) * 4 + (size_t)n_poses + 255) & ~(size_t)255;
    w.grid = nullptr;
    w.cell_count = w.cell_start = nullptr;
    w.cell_pts = nullptr;
    w.cands = nullptr;
    w.split = OptSplit{};
    if (opt) {
        const int64_t ncell = (int64_t)(kGridMax + 1) * (kGridMax + 1) * (kGridMax + 1);
        char *b = static_cast<char *>(base);
        w.grid = reinterpret_cast<GridDev *>(b + off);
        off += 256;
        w.cell_count = reinterpret_cast<uint32_t *>(b + off);
        off += (size_t)ncell * 4;
        w.cell_start = reinterpret_cast<uint32_t *>(b + off);
        off += (size_t)(ncell + 1) * 4;
        off = (off + 255) & ~(size_t)255;
        w.cell_pts = reinterpret_cast<float4 *>(b + off);
        off += ((size_t)n_points * 16 + 255) & ~(size_t)255;
        w.cands = reinterpret_cast<int32_t *>(b + off);
        off += (size_t)n_sets * k * n_inner * 4;
        if (split) {
            const size_t nc_ = (size_t)n_sets * n_inner;
            auto take = [&](size_t bytes) {
                off = (off + 255) & ~(size_t)255;
                char *q = b + off;
                off += bytes;
                return q;
            };
            w.split.sJ = reinterpret_cast<double *>(take((size_t)n_sets * 8));
            w.split.sB = reinterpret_cast<int32_t *>(take((size_t)n_sets * 28));
            w.split.cJ = reinterpret_cast<double *>(take(nc_ * 8));
            w.split.cB = reinterpret_cast<int32_t *>(take(nc_ * 28));
            w.split.queue = reinterpret_cast<int32_t *>(take(nc_ * 4));
            w.split.n_queue = reinterpret_cast<uint32_t *>(take((size_t)std::max<int64_t>(k, 1) * 4));
        }
    }
    w.bytes = off + 256;
    return w;
}

// Alg. 2 criteria with the slow LPs gathered need candidate ids below 2^31.
static bool split_fits(int64_t n_poses, int64_t draws, const lg_search_params *p)
{
    return p->opt_outer > 0 && n_poses * draws * p->opt_inner < 0x7fffffffLL;
}

// Workspace of the search: with split, the arrays of the gathered-slow-LP
// criteria too (what lg_search_workspace_bytes asks for); without, the least
// a search runs in (Alg. 2 then runs its criteria in one launch per round).
static size_t search_ws_bytes(int32_t n_points, int32_t n_poses, const lg_search_params *p, bool split)
{
    if (!p || n_poses <= 0 || p->draws <= 0) return 256;
    return search_ws(nullptr, std::max(n_points, 0), n_poses, p->draws, p->opt_outer > 0, p->k,
                     p->opt_outer > 0 ? p->opt_inner : 0, split && split_fits(n_poses, p->draws, p)).bytes;
}

size_t lg_search_workspace_bytes(int32_t n_points, int32_t n_poses, const lg_search_params *p)
{
    return search_ws_bytes(n_points, n_poses, p, true);
}

// One round of Alg. 2 criteria with the slow LPs gathered: per contact step
// the capped LPs of every candidate, the queued slow ones, the picks.
static lg_status opt_split_round(const float *pts, const float *nrm, int n_points, const SearchWs &ws,
                                 const uint32_t *dom_count, const int32_t *palm, int F, const lg_search_params *p,
                                 int kk, bool m8, const LpConst &cs, dim3 sgrid, dim3 cgrid, bool last,
                                 int32_t *set_pt, uint8_t *verdict, double *tstar, hipStream_t s)
{
    const uint32_t slo = (uint32_t)p->seed, shi = (uint32_t)(p->seed >> 32);
    const double mu = p->mu, rho = p->moment_scale;
    // queue counters cleared by a kernel, not a memset node (the stream may be captured)
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, s, ws.split.n_queue, (int64_t)p->k, 0u);
    for (int i = 0; i < p->k; ++i) {
#define LG_SPLIT_M(KM, MC)                                                                                       \
    do {                                                                                                         \
        hipLaunchKernelGGL((k_opt_try<KM, MC>), cgrid, dim3(256), 0, s, pts, nrm, n_points, ws.valid_poses,     \
                           ws.n_valid_poses, dom_count, palm, F, p->draws, p->k, p->m_edges, mu, rho,           \
                           p->max_pivots, cs, p->opt_inner, i, slo, shi, p->request_id, p->pose_offset,          \
                           ws.cands, set_pt, ws.split);                                                          \
        hipLaunchKernelGGL((k_opt_hard<KM, MC>), cgrid, dim3(256), 0, s, pts, nrm, n_points, ws.valid_poses,    \
                           dom_count, palm, F, p->draws, p->k, p->m_edges, mu, rho, p->max_pivots, cs,           \
                           p->opt_inner, i, slo, shi, p->request_id, p->pose_offset, ws.cands, set_pt,           \
                           ws.split);                                                                            \
    } while (0)
#define LG_SPLIT(KM) if (m8) LG_SPLIT_M(KM, 8); else LG_SPLIT_M(KM, 0)
        if (kk <= 3) { LG_SPLIT(3); } else if (kk <= 4) { LG_SPLIT(4); } else if (kk <= 5) { LG_SPLIT(5); }
        else if (kk <= 6) { LG_SPLIT(6); } else { LG_SPLIT(8); }
#undef LG_SPLIT
#undef LG_SPLIT_M
        hipLaunchKernelGGL(k_opt_pick, sgrid, dim3(256), 0, s, ws.valid_poses, ws.n_valid_poses, dom_count, palm,
                           n_points, F, p->draws, p->k, p->opt_inner, i, last, (double)p->eps, slo, shi,
                           p->request_id, p->pose_offset, ws.cands, set_pt, verdict, tstar, ws.split);
    }
    LG_HIP(hipGetLastError());
    return LG_OK;
}

}  // extern "C"

LpConst lg::lp_const(int m)
{
    LpConst cs;
    for (int e = 0; e < 16; ++e) {
        const double th = 2.0 * M_PI * e / m;
        cs.ce[e] = e < m ? cos(th) : 0.0;
        cs.se[e] = e < m ? sin(th) : 0.0;
    }
    return cs;
}

uint32_t lg::verdict_blocks(int64_t n_sets, int n_cu)
{
    return (uint32_t)std::max<int64_t>(1, std::min<int64_t>((n_sets + 255) / 256, (int64_t)n_cu * 8));
}

void lg::chunk_workspace(void *ws, int64_t n_points, int64_t n_poses, int64_t draws, ChunkDesc &c)
{
    const SearchWs w = search_ws(ws, n_points, n_poses, draws, false);
    c.pose_valid = w.pose_valid;
    c.pchunk_count = w.pchunk_count;
    c.pchunk_off = w.pchunk_off;
    c.valid_poses = w.valid_poses;
    c.n_valid_poses = w.n_valid_poses;
    c.chunk_count = w.chunk_count;
    c.chunk_off = w.chunk_off;
}

// the whole search on a given workspace (the caller's, or the static scratch
// array of lg_search_noalloc); allocates nothing
static lg_status search_impl(const lg_field *field, const float *pts, const float *nrm, int32_t n_points,
                             const float *poses, int32_t n_poses, const uint32_t *dom_bits, const uint32_t *dom_count,
                             const lg_search_params *p, int32_t *set_pt, int8_t *set_link, uint8_t *verdict,
                             double *tstar, int32_t *acc_list, int32_t *n_acc, void *workspace,
                             size_t workspace_bytes, void *stream)
{
    if (!field || !p) return fail(LG_EINVAL, "null field or params");
    const DevHand &H = field->dh;
    if (n_points <= 0 || n_poses < 0) return fail(LG_EINVAL, "n_points must be > 0 and n_poses >= 0");
    if (p->k < 1 || p->k > H.F) return fail(LG_EINVAL, "need 1 <= k <= number of fingers (one contact per finger)");
    const int32_t *palm = p->palm_pt;
    const int kk = p->k + (palm ? 1 : 0);  // contacts of the largest set (with a palm contact)
    if (p->draws <= 0 || p->m_edges < 3 || p->m_edges > 16 || kk > 8)
        return fail(LG_EINVAL, "need draws > 0, 3 <= m_edges <= 16, k <= 8 (k <= 7 with palm contacts)");
    if (!(p->mu >= 0.0f) || !(p->moment_scale > 0.0f) || p->max_pivots < 0)
        return fail(LG_EINVAL, "need mu >= 0, moment_scale > 0, max_pivots >= 0");
    if ((int64_t)n_poses * p->draws > 0x7fffffffLL) return fail(LG_EINVAL, "P * D must be < 2^31");
    if (n_poses == 0) return LG_OK;
    if (!pts || !nrm || !poses || !dom_bits || !dom_count || !set_pt || !set_link || !verdict || !tstar ||
        !acc_list || !n_acc || !workspace)
        return fail(LG_EINVAL, "null device buffer");
    if (p->opt_outer < 0 || p->opt_outer > 64 || (p->opt_outer > 0 && (p->opt_inner < 1 || p->opt_inner > 16)) ||
        !(p->opt_sigma >= 0.0f) || (int64_t)p->opt_outer * p->k * p->opt_inner >= (1 << 24))
        return fail(LG_EINVAL, "need 0 <= opt_outer <= 64, 1 <= opt_inner <= 16, opt_sigma >= 0");
    if (workspace_bytes < search_ws_bytes(n_points, n_poses, p, false)) return fail(LG_EINVAL, "workspace too small");
    const int NW = (n_points + 31) / 32, nsb = (NW + kSuper - 1) / kSuper;
    const size_t lds = (size_t)H.F * (nsb + 1) * sizeof(uint32_t);
    if (lds > 48 * 1024) return fail(LG_EUNSUPPORTED, "too many points for the draw rank structure");
    hipStream_t s = as_stream(stream);
    const bool opt = p->opt_outer > 0;
    // Alg. 2 criteria with the slow LPs gathered when the workspace holds their arrays
    const bool split = opt && split_fits(n_poses, p->draws, p) &&
                       workspace_bytes >= search_ws_bytes(n_points, n_poses, p, true);
    const SearchWs ws = search_ws(workspace, n_points, n_poses, p->draws, opt, p->k, opt ? p->opt_inner : 0, split);
    hipLaunchKernelGGL(k_draw, dim3(n_poses), dim3(kDrawThreads), lds, s, H, field->d_bits, pts, nrm, n_points,
                       poses, dom_bits, dom_count, palm, p->draws, p->k, (uint32_t)p->seed, (uint32_t)(p->seed >> 32),
                       p->request_id, p->pose_offset, set_pt, set_link, ws.pose_valid, verdict, tstar);
    LG_HIP(hipGetLastError());
    // list of poses with at least k non-empty domains (ordered)
    const int64_t npc = (n_poses + kChunk - 1) / kChunk;
    hipLaunchKernelGGL(k_chunk_count, dim3((unsigned)npc), dim3(kCompactThreads), 0, s, ws.pose_valid,
                       (int64_t)n_poses, ws.pchunk_count);
    hipLaunchKernelGGL(k_chunk_scan, dim3(1), dim3(kCompactThreads), 0, s, ws.pchunk_count, npc, ws.pchunk_off,
                       ws.n_valid_poses);
    hipLaunchKernelGGL(k_chunk_scatter, dim3((unsigned)npc), dim3(kCompactThreads), 0, s, ws.pose_valid,
                       (int64_t)n_poses, ws.pchunk_off, ws.valid_poses);
    LG_HIP(hipGetLastError());
    const int64_t n_sets = (int64_t)n_poses * p->draws;
    const LpConst cs = lp_const(p->m_edges);
    // grid-stride LP launch sized to the device (the valid count is on the device)
    int dev = 0, n_cu = 0;
    LG_HIP(hipGetDevice(&dev));
    LG_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    const dim3 lgrid(verdict_blocks(n_sets, n_cu));
    // the common 8-edge cone gets kernels with the edge loop unrolled
    const bool m8 = p->m_edges == 8;
#define LG_VERDICT_M(KM, MC)                                                                                    \
    hipLaunchKernelGGL((k_verdict_lane<KM, MC>), lgrid, dim3(256), 0, s, pts, nrm, n_points, set_pt, palm,       \
                       ws.valid_poses,                                                                          \
                       ws.n_valid_poses, p->draws, p->k, p->m_edges, (double)p->mu, (double)p->moment_scale,     \
                       (double)p->eps, p->max_pivots, cs, verdict, tstar)
#define LG_VERDICT(KM) if (m8) LG_VERDICT_M(KM, 8); else LG_VERDICT_M(KM, 0)
    if (!opt) {
        if (kk <= 3) { LG_VERDICT(3); } else if (kk <= 4) { LG_VERDICT(4); } else if (kk <= 5) { LG_VERDICT(5); }
        else if (kk <= 6) { LG_VERDICT(6); } else { LG_VERDICT(8); }
    } else {
        // cell grid of the object, then Alg. 2 on the drawn sets, then the links of the moved contacts
        const int64_t ncell = (int64_t)(kGridMax + 1) * (kGridMax + 1) * (kGridMax + 1);
        hipLaunchKernelGGL(k_grid_setup, dim3(1), dim3(1024), 0, s, pts, n_points, p->opt_sigma, ws.grid);
        // zeroed by a kernel, not a memset node (callers may capture the stream in a graph)
        hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((ncell + 255) / 256)), dim3(256), 0, s, ws.cell_count,
                           ncell, 0u);
        const unsigned pb = (unsigned)((n_points + 255) / 256);
        hipLaunchKernelGGL(k_grid_count, dim3(pb), dim3(256), 0, s, pts, n_points, ws.grid, ws.cell_count);
        hipLaunchKernelGGL(k_grid_scan, dim3(1), dim3(1024), 0, s, ws.cell_count, ws.grid, ws.cell_start);
        hipLaunchKernelGGL(k_grid_scatter, dim3(pb), dim3(256), 0, s, pts, n_points, ws.grid, ws.cell_count,
                           ws.cell_pts);
        const int gs = p->opt_inner <= 1 ? 1 : p->opt_inner <= 2 ? 2 : p->opt_inner <= 4 ? 4 : p->opt_inner <= 8 ? 8 : 16;
        const dim3 ogrid((unsigned)std::max<int64_t>(
            1, std::min<int64_t>((n_sets * gs + 255) / 256, (int64_t)n_cu * 8)));
        const dim3 pgrid((unsigned)std::max<int64_t>(
            1, std::min<int64_t>((n_sets * p->k * p->opt_inner + 255) / 256, (int64_t)n_cu * 32)));
        // grid-stride grids of the gathered-slow-LP criteria (candidates; sets)
        const dim3 cgrid((unsigned)std::max<int64_t>(
            1, std::min<int64_t>((n_sets * p->opt_inner + 255) / 256, (int64_t)n_cu * 8)));
        const dim3 sgrid((unsigned)std::max<int64_t>(1, std::min<int64_t>((n_sets + 255) / 256, (int64_t)n_cu * 8)));
#define LG_OPT_M(KM, GS, MC)                                                                                     \
    hipLaunchKernelGGL((k_optimize<KM, GS, MC>), ogrid, dim3(256), 0, s, pts, nrm, n_points, ws.valid_poses,       \
                       ws.n_valid_poses, dom_count, palm, H.F, p->draws, p->k, p->m_edges, (double)p->mu,         \
                       (double)p->moment_scale, (double)p->eps, p->max_pivots, cs, p->opt_inner,                  \
                       r == p->opt_outer - 1, (uint32_t)p->seed, (uint32_t)(p->seed >> 32), p->request_id,        \
                       p->pose_offset, ws.cands, set_pt, verdict, tstar)
#define LG_OPT(KM, GS) LG_OPT_M(KM, GS, 0)
#define LG_OPT_K(GS)                                                                                             \
    if (kk <= 3) LG_OPT(3, GS); else if (kk <= 4) LG_OPT(4, GS); else if (kk <= 5) LG_OPT(5, GS);              \
    else if (kk <= 6) LG_OPT(6, GS); else LG_OPT(8, GS)
#define LG_OPT_K8                                                                                                \
    if (kk <= 3) LG_OPT_M(3, 8, 8); else if (kk <= 4) LG_OPT_M(4, 8, 8); else if (kk <= 5) LG_OPT_M(5, 8, 8);  \
    else if (kk <= 6) LG_OPT_M(6, 8, 8); else LG_OPT_M(8, 8, 8)
        for (int r = 0; r < p->opt_outer; ++r) {
            hipLaunchKernelGGL(k_opt_project, pgrid, dim3(256), 0, s, pts, nrm, n_points, ws.valid_poses,
                               ws.n_valid_poses, dom_bits, dom_count, palm, H.F, p->draws, p->k, r, p->opt_inner,
                               (double)p->opt_sigma, (uint32_t)p->seed, (uint32_t)(p->seed >> 32), p->request_id,
                               p->pose_offset, ws.grid, ws.cell_start, ws.cell_pts, set_pt, ws.cands);
            if (split) {
                const lg_status so = opt_split_round(pts, nrm, n_points, ws, dom_count, palm, H.F, p, kk, m8, cs,
                                                     sgrid, cgrid, r == p->opt_outer - 1, set_pt, verdict, tstar, s);
                if (so != LG_OK) return so;
                continue;
            }
            if (gs == 1) { LG_OPT_K(1); } else if (gs == 2) { LG_OPT_K(2); } else if (gs == 4) { LG_OPT_K(4); }
            else if (gs == 8 && m8) { LG_OPT_K8; } else if (gs == 8) { LG_OPT_K(8); } else { LG_OPT_K(16); }
        }
#undef LG_OPT_K8
#undef LG_OPT_K
#undef LG_OPT
#undef LG_OPT_M
        LG_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_relink, lgrid, dim3(256), 0, s, H, field->d_bits, pts, nrm, n_points, poses,
                           ws.valid_poses, ws.n_valid_poses, dom_count, p->draws, p->k, (uint32_t)p->seed,
                           (uint32_t)(p->seed >> 32), p->request_id, p->pose_offset, set_pt, set_link);
    }
#undef LG_VERDICT
#undef LG_VERDICT_M
    LG_HIP(hipGetLastError());
    const int64_t n_chunks = (n_sets + kChunk - 1) / kChunk;
    uint32_t *chunk_count = ws.chunk_count;
    uint32_t *chunk_off = ws.chunk_off;
    hipLaunchKernelGGL(k_chunk_count, dim3((unsigned)n_chunks), dim3(kCompactThreads), 0, s, verdict, n_sets,
                       chunk_count);
    hipLaunchKernelGGL(k_chunk_scan, dim3(1), dim3(kCompactThreads), 0, s, chunk_count, n_chunks, chunk_off, n_acc);
    hipLaunchKernelGGL(k_chunk_scatter, dim3((unsigned)n_chunks), dim3(kCompactThreads), 0, s, verdict, n_sets,
                       chunk_off, acc_list);
    LG_HIP(hipGetLastError());
    return LG_OK;
}

// Bytes of device workspace of lg_compact_unstable: set flags, chunk counts and offsets.
static size_t unstable_ws_bytes(int64_t n_sets)
{
    const int64_t nc = (n_sets + kChunk - 1) / kChunk;
    return (((size_t)n_sets + 255) & ~(size_t)255) + (size_t)(2 * nc) * 4 + 256;
}

extern "C" {

size_t lg_compact_unstable_workspace_bytes(int32_t n_poses, int32_t draws)
{
    if (n_poses <= 0 || draws <= 0) return 256;
    return unstable_ws_bytes((int64_t)n_poses * draws);
}

lg_status lg_compact_unstable(const int32_t *set_pt, const int8_t *set_link, const uint8_t *verdict, int32_t n_poses,
                              int32_t draws, int32_t k, int32_t *list, int32_t *n_list, void *workspace,
                              size_t workspace_bytes, void *stream)
{
    if (n_poses < 0 || draws <= 0 || k < 1 || k > 8) return fail(LG_EINVAL, "need n_poses >= 0, draws > 0, 1 <= k <= 8");
    if ((int64_t)n_poses * draws > 0x7fffffffLL) return fail(LG_EINVAL, "P * D must be < 2^31");
    if (!n_list) return fail(LG_EINVAL, "null n_list");
    hipStream_t s = as_stream(stream);
    const int64_t n_sets = (int64_t)n_poses * draws;
    if (n_sets == 0) {  // a count of 0 (a kernel, not a memset node, for callers that capture the stream)
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, reinterpret_cast<uint32_t *>(n_list), (int64_t)1, 0u);
        LG_HIP(hipGetLastError());
        return LG_OK;
    }
    if (!set_pt || !set_link || !verdict || !list || !workspace) return fail(LG_EINVAL, "null device buffer");
    if (workspace_bytes < unstable_ws_bytes(n_sets)) return fail(LG_EINVAL, "workspace too small");
    uint8_t *flag = static_cast<uint8_t *>(workspace);
    uint32_t *cc = reinterpret_cast<uint32_t *>(flag + (((size_t)n_sets + 255) & ~(size_t)255));
    const int64_t nc = (n_sets + kChunk - 1) / kChunk;
    hipLaunchKernelGGL(k_flag_unstable, dim3((unsigned)((n_sets + 255) / 256)), dim3(256), 0, s, set_pt, set_link,
                       verdict, n_sets, k, flag);
    hipLaunchKernelGGL(k_chunk_count, dim3((unsigned)nc), dim3(kCompactThreads), 0, s, flag, n_sets, cc);
    hipLaunchKernelGGL(k_chunk_scan, dim3(1), dim3(kCompactThreads), 0, s, cc, nc, cc + nc, n_list);
    hipLaunchKernelGGL(k_chunk_scatter, dim3((unsigned)nc), dim3(kCompactThreads), 0, s, flag, n_sets, cc + nc, list);
    LG_HIP(hipGetLastError());
    return LG_OK;
}

lg_status lg_search_extend(const lg_field *field, const float *pts, const float *nrm, int32_t n_points,
                           const float *poses, int32_t n_poses, const uint32_t *dom_bits, const uint32_t *dom_count,
                           const lg_search_params *p, const int32_t *set_pt1, const int8_t *set_link1,
                           const uint8_t *verdict1, const lg_extend_params *ep, int32_t *set_pt2, int8_t *set_link2,
                           uint8_t *verdict2, double *tstar2, int32_t *acc_list2, int32_t *n_acc2, void *workspace,
                           size_t workspace_bytes, void *stream)
{
    if (!field || !p || !ep) return fail(LG_EINVAL, "null field or params");
    const DevHand &H = field->dh;
    if (n_points <= 0 || n_poses < 0) return fail(LG_EINVAL, "n_points must be > 0 and n_poses >= 0");
    const int k1 = p->k, k2 = p->k + ep->k_add;
    if (k1 < 1 || ep->k_add < 1 || k2 > H.F || k2 > 8)
        return fail(LG_EINVAL, "need k >= 1, k_add >= 1 and k + k_add <= number of fingers (and <= 8)");
    if (p->palm_pt) return fail(LG_EUNSUPPORTED, "the second contact round takes no palm contacts");
    if (p->draws <= 0 || p->m_edges < 3 || p->m_edges > 16 || !(p->mu >= 0.0f) || !(p->moment_scale > 0.0f) ||
        p->max_pivots < 0)
        return fail(LG_EINVAL, "need draws > 0, 3 <= m_edges <= 16, mu >= 0, moment_scale > 0, max_pivots >= 0");
    if ((int64_t)n_poses * p->draws > 0x7fffffffLL) return fail(LG_EINVAL, "P * D must be < 2^31");
    if (n_poses == 0) return LG_OK;
    if (!pts || !nrm || !poses || !dom_bits || !dom_count || !set_pt1 || !set_link1 || !verdict1 || !set_pt2 ||
        !set_link2 || !verdict2 || !tstar2 || !acc_list2 || !n_acc2 || !workspace)
        return fail(LG_EINVAL, "null device buffer");
    if (ep->list && !ep->list_n) return fail(LG_EINVAL, "a set list needs its device count");
    lg_search_params p2 = *p;
    p2.k = k2;
    p2.opt_outer = 0;
    if (workspace_bytes < lg_search_workspace_bytes(n_points, n_poses, &p2)) return fail(LG_EINVAL, "workspace too small");
    const int NW = (n_points + 31) / 32, nsb = (NW + kSuper - 1) / kSuper;
    const size_t lds = (size_t)H.F * (nsb + 1) * sizeof(uint32_t);
    if (lds > 48 * 1024) return fail(LG_EUNSUPPORTED, "too many points for the draw rank structure");
    hipStream_t s = as_stream(stream);
    const SearchWs ws = search_ws(workspace, n_points, n_poses, p->draws, false);
    hipLaunchKernelGGL(k_extend, dim3(n_poses), dim3(kDrawThreads), lds, s, H, field->d_bits, pts, nrm, n_points,
                       poses, dom_bits, dom_count, p->draws, k1, ep->k_add, set_pt1, set_link1, verdict1, ep->list,
                       ep->list_n, ep->list_ok, (uint32_t)p->seed, (uint32_t)(p->seed >> 32), ep->request_id,
                       p->pose_offset, set_pt2, set_link2, ws.pose_valid, verdict2, tstar2);
    LG_HIP(hipGetLastError());
    const int64_t npc = (n_poses + kChunk - 1) / kChunk;
    hipLaunchKernelGGL(k_chunk_count, dim3((unsigned)npc), dim3(kCompactThreads), 0, s, ws.pose_valid,
                       (int64_t)n_poses, ws.pchunk_count);
    hipLaunchKernelGGL(k_chunk_scan, dim3(1), dim3(kCompactThreads), 0, s, ws.pchunk_count, npc, ws.pchunk_off,
                       ws.n_valid_poses);
    hipLaunchKernelGGL(k_chunk_scatter, dim3((unsigned)npc), dim3(kCompactThreads), 0, s, ws.pose_valid,
                       (int64_t)n_poses, ws.pchunk_off, ws.valid_poses);
    const int64_t n_sets = (int64_t)n_poses * p->draws;
    LpConst cs;
    for (int e = 0; e < 16; ++e) {
        const double th = 2.0 * M_PI * e / p->m_edges;
        cs.ce[e] = e < p->m_edges ? cos(th) : 0.0;
        cs.se[e] = e < p->m_edges ? sin(th) : 0.0;
    }
    int dev = 0, n_cu = 0;
    LG_HIP(hipGetDevice(&dev));
    LG_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    const dim3 lgrid((unsigned)std::max<int64_t>(1, std::min<int64_t>((n_sets + 255) / 256, (int64_t)n_cu * 8)));
    const bool m8 = p->m_edges == 8;
#define LG_VERDICT2_M(KM, MC)                                                                                   \
    hipLaunchKernelGGL((k_verdict_lane<KM, MC>), lgrid, dim3(256), 0, s, pts, nrm, n_points, set_pt2, nullptr,    \
                       ws.valid_poses, ws.n_valid_poses, p->draws, k2, p->m_edges, (double)p->mu,                \
                       (double)p->moment_scale, (double)p->eps, p->max_pivots, cs, verdict2, tstar2)
#define LG_VERDICT2(KM) if (m8) LG_VERDICT2_M(KM, 8); else LG_VERDICT2_M(KM, 0)
    if (k2 <= 3) { LG_VERDICT2(3); } else if (k2 <= 4) { LG_VERDICT2(4); } else if (k2 <= 5) { LG_VERDICT2(5); }
    else if (k2 <= 6) { LG_VERDICT2(6); } else { LG_VERDICT2(8); }
#undef LG_VERDICT2
#undef LG_VERDICT2_M
    LG_HIP(hipGetLastError());
    const int64_t n_chunks = (n_sets + kChunk - 1) / kChunk;
    hipLaunchKernelGGL(k_chunk_count, dim3((unsigned)n_chunks), dim3(kCompactThreads), 0, s, verdict2, n_sets,
                       ws.chunk_count);
    hipLaunchKernelGGL(k_chunk_scan, dim3(1), dim3(kCompactThreads), 0, s, ws.chunk_count, n_chunks, ws.chunk_off,
                       n_acc2);
    hipLaunchKernelGGL(k_chunk_scatter, dim3((unsigned)n_chunks), dim3(kCompactThreads), 0, s, verdict2, n_sets,
                       ws.chunk_off, acc_list2);
    LG_HIP(hipGetLastError());
    return LG_OK;
}

}  // extern "C"

// Scratch of lg_search_noalloc: one array per device, held until the process
// ends.  Host code never passes the array's name to a kernel (on the host it
// is only a stand-in symbol); it uses the device address that
// hipGetSymbolAddress returns, looked up once per device.
constexpr size_t kStaticScratchBytes = (size_t)8 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

static lg_status scratch_address(void **out)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    LG_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(LG_EUNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *ptr = nullptr;
        LG_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(LG_EDEVICE, "no device address for the static scratch array");
        addr[dev] = ptr;
    }
    *out = addr[dev];
    return LG_OK;
}

extern "C" {

size_t lg_search_noalloc_max_bytes(void) { return kStaticScratchBytes; }

lg_status lg_search(const lg_field *field, const float *pts, const float *nrm, int32_t n_points, const float *poses,
                    int32_t n_poses, const uint32_t *dom_bits, const uint32_t *dom_count,
                    const lg_search_params *p, int32_t *set_pt, int8_t *set_link, uint8_t *verdict, double *tstar,
                    int32_t *acc_list, int32_t *n_acc, void *workspace, size_t workspace_bytes, void *stream)
{
    return search_impl(field, pts, nrm, n_points, poses, n_poses, dom_bits, dom_count, p, set_pt, set_link, verdict,
                       tstar, acc_list, n_acc, workspace, workspace_bytes, stream);
}

lg_status lg_search_noalloc(const lg_field *field, const float *pts, const float *nrm, int32_t n_points,
                            const float *poses, int32_t n_poses, const uint32_t *dom_bits, const uint32_t *dom_count,
                            const lg_search_params *p, int32_t *set_pt, int8_t *set_link, uint8_t *verdict,
                            double *tstar, int32_t *acc_list, int32_t *n_acc, void *stream)
{
    if (!p) return fail(LG_EINVAL, "null params");
    const size_t need = search_ws_bytes(n_points, n_poses, p, false);  // the least a search runs in
    if (need > kStaticScratchBytes)
        return fail(LG_EINVAL, "search needs " + std::to_string(need) + " bytes of workspace, above the " +
                                   std::to_string(kStaticScratchBytes) + "-byte static scratch");
    void *ws = nullptr;
    const lg_status st = scratch_address(&ws);
    if (st != LG_OK) return st;
    return search_impl(field, pts, nrm, n_points, poses, n_poses, dom_bits, dom_count, p, set_pt, set_link, verdict,
                       tstar, acc_list, n_acc, ws, kStaticScratchBytes, stream);
}

}  // extern "C"

// ---- batched launches over the chunks of several requests -------------------
size_t lg::draw_lds_bytes(int F, int N)
{
    const int NW = (N + 31) / 32, nsb = (NW + kSuper - 1) / kSuper;
    return (size_t)F * (nsb + 1) * sizeof(uint32_t);
}

uint32_t lg::compact_blocks(int64_t n) { return (uint32_t)((n + kChunk - 1) / kChunk); }

lg_status lg::draw_batch(const BatchLaunch &b, size_t lds, hipStream_t s)
{
    if (b.n <= 0 || b.blocks == 0) return LG_OK;
    if (lds > 48 * 1024) return fail(LG_EUNSUPPORTED, "too many points for the draw rank structure");
    hipLaunchKernelGGL(k_draw_batch, dim3(b.blocks), dim3(kDrawThreads), lds, s, b.d, b.idx, b.first, b.n);
    LG_HIP(hipGetLastError());
    return LG_OK;
}

lg_status lg::compact_count_batch(const BatchLaunch &b, bool poses, hipStream_t s)
{
    if (b.n <= 0 || b.blocks == 0) return LG_OK;
    if (poses)
        hipLaunchKernelGGL(k_count_batch<true>, dim3(b.blocks), dim3(kCompactThreads), 0, s, b.d, b.idx, b.first, b.n);
    else
        hipLaunchKernelGGL(k_count_batch<false>, dim3(b.blocks), dim3(kCompactThreads), 0, s, b.d, b.idx, b.first, b.n);
    LG_HIP(hipGetLastError());
    return LG_OK;
}

lg_status lg::compact_scan_batch(const BatchLaunch &b, bool poses, hipStream_t s)
{
    if (b.n <= 0 || b.blocks == 0) return LG_OK;
    if (poses)
        hipLaunchKernelGGL(k_scan_batch<true>, dim3(b.blocks), dim3(kCompactThreads), 0, s, b.d, b.idx, b.first, b.n);
    else
        hipLaunchKernelGGL(k_scan_batch<false>, dim3(b.blocks), dim3(kCompactThreads), 0, s, b.d, b.idx, b.first, b.n);
    LG_HIP(hipGetLastError());
    return LG_OK;
}

lg_status lg::compact_scatter_batch(const BatchLaunch &b, bool poses, hipStream_t s)
{
    if (b.n <= 0 || b.blocks == 0) return LG_OK;
    if (poses)
        hipLaunchKernelGGL(k_scatter_batch<true>, dim3(b.blocks), dim3(kCompactThreads), 0, s, b.d, b.idx, b.first,
                           b.n);
    else
        hipLaunchKernelGGL(k_scatter_batch<false>, dim3(b.blocks), dim3(kCompactThreads), 0, s, b.d, b.idx, b.first,
                           b.n);
    LG_HIP(hipGetLastError());
    return LG_OK;
}

lg_status lg::verdict_batch(const BatchLaunch &b, int km, bool m8, hipStream_t s)
{
    if (b.n <= 0 || b.blocks == 0) return LG_OK;
#define LG_VB_M(KM, MC)                                                                                          \
    hipLaunchKernelGGL((k_verdict_batch<KM, MC>), dim3(b.blocks), dim3(256), 0, s, b.d, b.idx, b.first, b.n)
#define LG_VB(KM) if (m8) LG_VB_M(KM, 8); else LG_VB_M(KM, 0)
    if (km <= 3) { LG_VB(3); } else if (km <= 4) { LG_VB(4); } else if (km <= 5) { LG_VB(5); }
    else if (km <= 6) { LG_VB(6); } else { LG_VB(8); }
#undef LG_VB
#undef LG_VB_M
    LG_HIP(hipGetLastError());
    return LG_OK;
}
