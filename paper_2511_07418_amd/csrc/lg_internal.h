// Internal declarations of the gfx950 Contact-Field library: the field
// object, the device-side hand description and the device helpers shared by
// the kernels.  Arithmetic that decides a discrete outcome (voxel, normal
// bin) is written with explicit fmaf chains so that every kernel that
// evaluates it (query, draw, realize) gets bit-identical results.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/lg.h"

namespace lg {

constexpr int kMaxFingers = 8;
constexpr int kMaxJoints = 64;
constexpr int kMaxDof = 8;
constexpr int kMaxBins = 64;
constexpr uint32_t kPurposeJoint = 1u;
constexpr uint32_t kPurposeDraw = 3u;
constexpr int32_t kNoWitness = 0x7fffffff;
constexpr int kLutRes = 28;  // cube-map cells per face edge of the bin table (18.4 KiB in LDS)

// Device-side description of a hand and its field window (kernel argument).
struct DevHand {
    int F, J, G, B, W;   // W = 32-bit words per voxel (B / 32)
    int nsurf;
    float h, inv_h;
    uint32_t seed_lo, seed_hi;
    int64_t samples;
    const float *origin;      // [J][12]
    const float *axis;        // [J][3]
    const float *capsule;     // [J][7]
    const float *limits;      // [J][2]
    const float *surf;        // [J][nsurf][6]
    const float *grid_frame;  // [F][12]
    const float *bin_c;       // [B][3]
    const uint32_t *bin_lut;  // [6][kLutRes][kLutRes] 4 candidate bins (8 bit each, absent ones repeat the
                              // first), 0xffffffff = more than four: every bin
    const int32_t *axis_samples;  // [J + n_palm_caps]: links, then the palm's capsules
    int n_palm_surf, n_palm_caps; // static link (palm): contact vectors and capsules, base frame
    const float *palm_surf;       // [n_palm_surf][6]
    const float *palm_caps;       // [n_palm_caps][7]
    int finger_first[kMaxFingers];
    int finger_dof[kMaxFingers];
    // Lattice form of the windows (lat != 0): every finger's window has the
    // rotation of finger 0's and its origin lies a whole number of 4-voxel
    // bricks from the others, G is a power of two.  Lattice coordinates are
    // finger 0's window coordinates shifted by lat_o[0]; finger f's window is
    // the lattice box [lat_o[f], lat_o[f] + G)^3, with G <= lat_o <= 1024 - 2G.
    int lat;
    int lat_o[kMaxFingers][3];
    uint32_t lat_pk[kMaxFingers];  // lat_o packed as x | y << 10 | z << 20
    uint32_t lat_idx[kMaxFingers]; // brick_word(lat_o) (its in-brick part is 0)
    uint32_t lat_hi;               // bits of a packed difference that must be 0 inside a window
};

}  // namespace lg

// The opaque handle of the C ABI.
struct lg_field {
    lg::DevHand dh;
    int device;
    int max_dof;
    bool has_witness;
    int64_t vectors, dropped;
    double build_kernel_ms = 0.0;  // k_field_build's duration (0 for imported fields)
    uint64_t bits_set;
    uint64_t device_bytes;
    // host copies
    std::vector<int32_t> joint_finger, joint_parent, axis_samples;
    std::vector<float> origin, axis, capsule, limits, surf, grid_frame, bin_c, palm_surf, palm_caps;
    // device allocations
    float *d_params = nullptr;     // packed float arrays (origin..bin_c)
    int32_t *d_axis_samples = nullptr;
    uint32_t *d_bits = nullptr;    // per-link tables [J][G^3][W]
    uint32_t *d_merged = nullptr;  // per-finger OR of its links [F][G^3][W]
    int32_t *d_wit = nullptr;      // [J][G^3][B], kNoWitness = none
};

namespace lg {

// ---- error reporting -------------------------------------------------------
lg_status fail(lg_status s, const std::string &msg);
lg_status hip_fail(hipError_t e, const char *what);
#define LG_HIP(call)                                   \
    do {                                               \
        hipError_t _e = (call);                        \
        if (_e != hipSuccess) return lg::hip_fail(_e, #call); \
    } while (0)

lg_status validate_hand(const lg_hand_desc *hand, const lg_field_params *p);
lg_status make_field_shell(const lg_hand_desc *hand, const lg_field_params *p, lg_field **out);
void free_field(lg_field *f);

// ---- Philox4x32-10 (Salmon et al., SC'11) -----------------------------------
__host__ __device__ inline void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t out[4])
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t m0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t m1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(m1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(m0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)m1;
        c3 = (uint32_t)m0;
        c0 = n0;
        c2 = n2;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

__device__ inline float u01f(uint32_t w) { return (float)(w >> 8) * (1.0f / 16777216.0f); }

// Joint t of finger f for joint sample s (q = lo + (hi - lo) u).
__device__ inline float joint_sample(const DevHand &H, int f, uint32_t s, int t)
{
    uint32_t w[4];
    philox4x32_10(s, (uint32_t)(8 * f + t / 4), kPurposeJoint, 0u, H.seed_lo, H.seed_hi, w);
    const int j = H.finger_first[f] + t;
    const float lo = H.limits[2 * j], hi = H.limits[2 * j + 1];
    return fmaf(hi - lo, u01f(w[t & 3]), lo);
}

// ---- rigid transforms (3x4 row-major) -------------------------------------
struct Tf {
    float m[12];
};

__device__ inline Tf tf_load(const float *p)
{
    Tf t;
#pragma unroll
    for (int i = 0; i < 12; ++i) t.m[i] = p[i];
    return t;
}

__device__ inline Tf tf_mul(const Tf &A, const Tf &B)
{
    Tf C;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
            C.m[4 * i + j] = fmaf(A.m[4 * i], B.m[j], fmaf(A.m[4 * i + 1], B.m[4 + j], A.m[4 * i + 2] * B.m[8 + j]));
        C.m[4 * i + 3] = fmaf(A.m[4 * i], B.m[3], fmaf(A.m[4 * i + 1], B.m[7], fmaf(A.m[4 * i + 2], B.m[11], A.m[4 * i + 3])));
    }
    return C;
}

// rotation by angle q about unit axis a (Rodrigues)
__device__ inline Tf tf_axis_angle(float ax, float ay, float az, float q)
{
    float s, c;
    sincosf(q, &s, &c);
    const float v = 1.0f - c;
    Tf T;
    T.m[0] = fmaf(ax * ax, v, c);      T.m[1] = fmaf(ax * ay, v, -az * s); T.m[2] = fmaf(ax * az, v, ay * s);  T.m[3] = 0.f;
    T.m[4] = fmaf(ay * ax, v, az * s); T.m[5] = fmaf(ay * ay, v, c);      T.m[6] = fmaf(ay * az, v, -ax * s); T.m[7] = 0.f;
    T.m[8] = fmaf(az * ax, v, -ay * s); T.m[9] = fmaf(az * ay, v, ax * s); T.m[10] = fmaf(az * az, v, c);     T.m[11] = 0.f;
    return T;
}

__device__ inline void tf_point(const Tf &T, float px, float py, float pz, float &x, float &y, float &z)
{
    x = fmaf(T.m[0], px, fmaf(T.m[1], py, fmaf(T.m[2], pz, T.m[3])));
    y = fmaf(T.m[4], px, fmaf(T.m[5], py, fmaf(T.m[6], pz, T.m[7])));
    z = fmaf(T.m[8], px, fmaf(T.m[9], py, fmaf(T.m[10], pz, T.m[11])));
}

__device__ inline void tf_dir(const Tf &T, float px, float py, float pz, float &x, float &y, float &z)
{
    x = fmaf(T.m[0], px, fmaf(T.m[1], py, T.m[2] * pz));
    y = fmaf(T.m[4], px, fmaf(T.m[5], py, T.m[6] * pz));
    z = fmaf(T.m[8], px, fmaf(T.m[9], py, T.m[10] * pz));
}

// Frame of joint j given its parent frame P and joint value q.
__device__ inline Tf joint_frame(const DevHand &H, const Tf &P, bool has_parent, int j, float q)
{
    Tf O = tf_load(H.origin + 12 * j);
    Tf base = has_parent ? tf_mul(P, O) : O;
    Tf R = tf_axis_angle(H.axis[3 * j], H.axis[3 * j + 1], H.axis[3 * j + 2], q);
    return tf_mul(base, R);
}

// ---- window coordinates and normal bins -------------------------------------
// Affine map u = A p + c from object-frame points to the voxel coordinates of
// finger f's window under pose P: A = R_f^T R_P / h, c = R_f^T (t_P - o_f) / h
// + G.  The +G bias makes every coordinate of interest positive, so a plain
// truncation is the floor (see window_voxel).
struct Affine {
    float m[12];
};

__device__ inline Affine finger_affine(const DevHand &H, const float *pose, int f)
{
    const float *g = H.grid_frame + 12 * f;
    Affine a;
    const float dx = pose[3] - g[3], dy = pose[7] - g[7], dz = pose[11] - g[11];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
            a.m[4 * r + c] = fmaf(g[r], pose[c], fmaf(g[4 + r], pose[4 + c], g[8 + r] * pose[8 + c])) * H.inv_h;
        a.m[4 * r + 3] = fmaf(fmaf(g[r], dx, fmaf(g[4 + r], dy, g[8 + r] * dz)), H.inv_h, (float)H.G);
    }
    return a;
}

// Linear voxel index (iz G + iy) G + ix of object point p in the window, -1
// outside.  The affine map carries a +G bias (u' = u + G): for u' >= 0 the
// truncation equals floor, and u' < 0 (u < -G) truncates to a value <= 0,
// which the unsigned range test rejects like any other outside point.
__device__ inline int window_voxel(const Affine &a, int G, float px, float py, float pz)
{
    const float ux = fmaf(a.m[0], px, fmaf(a.m[1], py, fmaf(a.m[2], pz, a.m[3])));
    const float uy = fmaf(a.m[4], px, fmaf(a.m[5], py, fmaf(a.m[6], pz, a.m[7])));
    const float uz = fmaf(a.m[8], px, fmaf(a.m[9], py, fmaf(a.m[10], pz, a.m[11])));
    const unsigned ix = (unsigned)((int)ux - G), iy = (unsigned)((int)uy - G), iz = (unsigned)((int)uz - G);
    const bool in = max(ix, max(iy, iz)) < (unsigned)G;
    return in ? (int)__umul24(__umul24(iz, G) + iy, G) + (int)ix : -1;
}

// Lattice map of pose P: finger 0's affine map with the bias lat_o[0]
// instead of G (same fmaf chains as finger_affine).
__device__ inline Affine lattice_affine(const DevHand &H, const float *pose)
{
    const float *g = H.grid_frame;
    Affine a;
    const float dx = pose[3] - g[3], dy = pose[7] - g[7], dz = pose[11] - g[11];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
            a.m[4 * r + c] = fmaf(g[r], pose[c], fmaf(g[4 + r], pose[4 + c], g[8 + r] * pose[8 + c])) * H.inv_h;
        a.m[4 * r + 3] = fmaf(fmaf(g[r], dx, fmaf(g[4 + r], dy, g[8 + r] * dz)), H.inv_h, (float)H.lat_o[0][r]);
    }
    return a;
}

// Lattice cell of object point p (truncation; every window lies at lattice
// coordinates >= G, so a truncated negative value is outside all of them).
__device__ inline void lattice_cell(const Affine &a, float px, float py, float pz, int &Ix, int &Iy, int &Iz)
{
    Ix = (int)fmaf(a.m[0], px, fmaf(a.m[1], py, fmaf(a.m[2], pz, a.m[3])));
    Iy = (int)fmaf(a.m[4], px, fmaf(a.m[5], py, fmaf(a.m[6], pz, a.m[7])));
    Iz = (int)fmaf(a.m[8], px, fmaf(a.m[9], py, fmaf(a.m[10], pz, a.m[11])));
}

// a * b + c on the 24-bit multiplier (a, b < 2^24; b uniform)
__device__ inline uint32_t mad_u24(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c));
    return r;
}

// Word of voxel (ix, iy, iz) in a plane of a merged finger table: 4x4x4
// bricks in (z, y, x) order, voxels in a brick in (z, y, x) order.  The map is
// linear in the brick and in-brick coordinates, so for a brick-aligned offset
// O, brick_word(I - O) = brick_word(I) - brick_word(O).
__host__ __device__ inline uint32_t brick_word(uint32_t ix, uint32_t iy, uint32_t iz, uint32_t GB)
{
    return ((((iz >> 2) * GB + (iy >> 2)) * GB + (ix >> 2)) << 6) | ((iz & 3u) << 4) | ((iy & 3u) << 2) | (ix & 3u);
}

// brick_word on the 24-bit multiplier (coordinates below 2^22, GB uniform)
__device__ inline uint32_t brick_word_u24(uint32_t ix, uint32_t iy, uint32_t iz, uint32_t GB)
{
    const uint32_t blk = mad_u24(mad_u24(iz >> 2, GB, iy >> 2), GB, ix >> 2);
    return (blk << 6) | ((iz & 3u) << 4) | ((iy & 3u) << 2) | (ix & 3u);
}

// Voxel of object point p in finger f's window under pose P (-1 outside):
// window_voxel of finger_affine, or, for lattice windows, the lattice cell
// less the finger's offset (the query takes the same decisions).
__device__ inline int finger_window_voxel(const DevHand &H, const float *pose, int f, float px, float py, float pz)
{
    if (H.lat) {
        const Affine a = lattice_affine(H, pose);
        int Ix, Iy, Iz;
        lattice_cell(a, px, py, pz, Ix, Iy, Iz);
        const unsigned ix = (unsigned)(Ix - H.lat_o[f][0]), iy = (unsigned)(Iy - H.lat_o[f][1]),
                       iz = (unsigned)(Iz - H.lat_o[f][2]);
        const bool in = max(ix, max(iy, iz)) < (unsigned)H.G;
        return in ? (int)__umul24(__umul24(iz, H.G) + iy, H.G) + (int)ix : -1;
    }
    return window_voxel(finger_affine(H, pose, f), H.G, px, py, pz);
}

// Query direction of object normal n under pose P: q = -R_P n.
__device__ inline void query_dir(const float *pose, float nx, float ny, float nz, float &qx, float &qy, float &qz)
{
    qx = -fmaf(pose[0], nx, fmaf(pose[1], ny, pose[2] * nz));
    qy = -fmaf(pose[4], nx, fmaf(pose[5], ny, pose[6] * nz));
    qz = -fmaf(pose[8], nx, fmaf(pose[9], ny, pose[10] * nz));
}

// argmax_b <d, c_b>, ties to the lowest b; c is [B][3] (LDS or global).
__device__ inline int nearest_bin(const float *c, int B, float dx, float dy, float dz)
{
    float best = -3.0e38f;
    int bi = 0;
    for (int b = 0; b < B; ++b) {
        const float s = fmaf(c[3 * b], dx, fmaf(c[3 * b + 1], dy, c[3 * b + 2] * dz));
        if (s > best) {
            best = s;
            bi = b;
        }
    }
    return bi;
}

__device__ inline bool table_bit(const uint32_t *tab, int W, int64_t voxel, int b)
{
    return (tab[voxel * W + (b >> 5)] >> (b & 31)) & 1u;
}

// Object signed-distance grid (object frame), [iz][iy][ix] node values.
struct SdfDev {
    float ox, oy, oz, h, inv_h;
    int G;
    const float *v;
};

// Trilinear SDF at object-frame point y; +inf outside the grid.
__device__ inline float sdf_trilinear(const SdfDev &S, float yx, float yy, float yz)
{
    const float ux = (yx - S.ox) * S.inv_h, uy = (yy - S.oy) * S.inv_h, uz = (yz - S.oz) * S.inv_h;
    const float gm = (float)(S.G - 1);
    if (!((ux >= 0.f) & (ux <= gm) & (uy >= 0.f) & (uy <= gm) & (uz >= 0.f) & (uz <= gm))) return INFINITY;
    const int ix = min((int)ux, S.G - 2), iy = min((int)uy, S.G - 2), iz = min((int)uz, S.G - 2);
    const float fx = ux - ix, fy = uy - iy, fz = uz - iz;
    const int64_t G = S.G;
    const float *v = S.v + (iz * G + iy) * G + ix;
    const float c00 = fmaf(fx, v[1] - v[0], v[0]);
    const float c10 = fmaf(fx, v[G + 1] - v[G], v[G]);
    const float c01 = fmaf(fx, v[G * G + 1] - v[G * G], v[G * G]);
    const float c11 = fmaf(fx, v[G * G + G + 1] - v[G * G + G], v[G * G + G]);
    const float c0 = fmaf(fy, c10 - c00, c00), c1 = fmaf(fy, c11 - c01, c01);
    return fmaf(fz, c1 - c0, c0);
}

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// cos, sin of 2 pi e / m for the m edges of the linearised friction cone
struct LpConst {
    double ce[16], se[16];
};

// IK and penetration parameters of lg_realize on the device
struct IkDev {
    int iters, phase1;
    float lambda, beta, tol_pos, tol_ang, margin;
    int self_collision;
    uint32_t seed_lo, seed_hi, request_id;
    int64_t pose_offset;
};

// ---- batched chunks ---------------------------------------------------------
// A server runs the chunks of several requests through one launch per stage
// (query, draws, pose compaction, verdicts, set compaction, realize,
// counters).  A ChunkDesc holds every argument of one chunk's kernels; its
// buffers are the request's own, so chunks of a batch share nothing.
struct ChunkDesc {
    DevHand H;
    const uint32_t *merged, *bits;
    const int32_t *wit;  // witness table, or null
    const float *pts, *nrm, *poses;  // poses: the chunk's first pose
    const float4 *bounds;
    int N, P, D, k, m, max_pivots;
    uint32_t seed_lo, seed_hi, request_id;
    int64_t pose_offset;  // the chunk's first pose within its request
    double mu, rho, eps;
    LpConst cs;
    uint32_t *dom_bits, *dom_count;
    int32_t *set_pt;
    int8_t *set_link;
    uint8_t *verdict;
    double *tstar;
    uint8_t *pose_valid;
    uint32_t *pchunk_count, *pchunk_off;
    int32_t *valid_poses, *n_valid_poses;
    uint32_t *chunk_count, *chunk_off;
    int32_t *acc, *n_acc;
    int realize;
    SdfDev S;
    IkDev ik;
    float *q, *err, *ang, *depth;
    uint8_t *valid;
    unsigned long long *counters;
};

// One launch over some chunks of a batch (all pointers on the device):
// member j is table entry idx[j] and owns blocks [first[j], first[j + 1]);
// first[0] = 0, first[n] = blocks; a member may own no block.
struct BatchLaunch {
    const ChunkDesc *d;
    const uint16_t *idx;
    const uint32_t *first;
    int n;
    uint32_t blocks;
};

// the member that owns block b (first[lo] <= b < first[lo + 1])
__device__ inline int batch_member(const uint32_t *__restrict__ first, int n, uint32_t b)
{
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (first[mid] <= b)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Batched launchers (one kernel launch each; the member's blocks follow the
// single-chunk kernel's grid).  Blocks per member:
//   query, draws: P;  compaction count/scatter: compact_blocks(n);
//   compaction scan: 1;  verdicts: verdict_blocks;  realize: realize_blocks.
lg_status query_batch(const BatchLaunch &b, int W, int F, bool lat, hipStream_t s);
size_t draw_lds_bytes(int F, int N);
lg_status draw_batch(const BatchLaunch &b, size_t lds, hipStream_t s);
uint32_t compact_blocks(int64_t n);
// poses = true: the pose list of the draws; false: the accepted set list
lg_status compact_count_batch(const BatchLaunch &b, bool poses, hipStream_t s);
lg_status compact_scan_batch(const BatchLaunch &b, bool poses, hipStream_t s);
lg_status compact_scatter_batch(const BatchLaunch &b, bool poses, hipStream_t s);
uint32_t verdict_blocks(int64_t n_sets, int n_cu);
LpConst lp_const(int m);
// the search workspace's lists of a chunk of P poses (no contact optimisation)
void chunk_workspace(void *ws, int64_t n_points, int64_t n_poses, int64_t draws, ChunkDesc &c);
lg_status verdict_batch(const BatchLaunch &b, int km, bool m8, hipStream_t s);  // m8: every chunk has an 8-edge cone
uint32_t realize_blocks(int64_t max_acc, int F, int n_cu);
lg_status realize_batch(const BatchLaunch &b, int max_dof, hipStream_t s);

}  // namespace lg
