// Contact-field construction (Sec. 4.3, Alg. 1; fine-grained per-patch
// fields of Sec. 4.4) and the field object's life cycle.
//
// Alg. 1 organises sampled contact vectors in a box cover of width w and a
// BVH, with the normals of each box stored in its leaf.  On gfx950 the cover
// is a dense G^3 window per finger (O(1) addressing, no BVH traversal) and a
// leaf's normal list is a B-bit mask over a spherical Fibonacci lattice (the
// quantised normals of Sec. 4.4), so one 4- or 8-byte word answers a query.
// All links of a finger share the finger's window, so the finger-level OR of
// the link tables (the merged domain of a dependency group, Sec. 5.3) is a
// table of its own and the query reads one word per finger.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "lg_internal.h"

namespace lg {

static thread_local std::string g_last_error;

lg_status fail(lg_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

lg_status hip_fail(hipError_t e, const char *what)
{
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? LG_ENOMEM : LG_EDEVICE;
}

lg_status validate_hand(const lg_hand_desc *hand, const lg_field_params *p)
{
    if (!hand || !p) return fail(LG_EINVAL, "null hand or params");
    const int F = hand->n_fingers, J = hand->n_joints;
    if (F < 1 || F > kMaxFingers) return fail(LG_EINVAL, "n_fingers must be 1..8");
    if (J < F || J > kMaxJoints) return fail(LG_EINVAL, "n_joints must be F..64");
    if (!hand->joint_finger || !hand->joint_parent || !hand->joint_origin || !hand->joint_axis ||
        !hand->capsule || !hand->limits || !hand->surf)
        return fail(LG_EINVAL, "null hand array");
    if (hand->n_surf < 1 || hand->n_surf > 65536) return fail(LG_EINVAL, "n_surf must be 1..65536");
    int prev_f = -1, dof = 0;
    for (int j = 0; j < J; ++j) {
        const int f = hand->joint_finger[j];
        if (f < 0 || f >= F) return fail(LG_EINVAL, "joint_finger out of range");
        if (f != prev_f) {
            if (f != prev_f + 1) return fail(LG_EINVAL, "fingers must be stored contiguously in order");
            if (hand->joint_parent[j] != -1) return fail(LG_EINVAL, "first joint of a finger must have parent -1");
            dof = 0;
            prev_f = f;
        } else if (hand->joint_parent[j] != j - 1) {
            return fail(LG_EINVAL, "a finger must be a serial chain (parent = j - 1)");
        }
        if (++dof > kMaxDof) return fail(LG_EINVAL, "at most 8 joints per finger");
        if (!(hand->limits[2 * j] <= hand->limits[2 * j + 1])) return fail(LG_EINVAL, "limits lo > hi");
    }
    if (prev_f != F - 1) return fail(LG_EINVAL, "every finger needs at least one joint");
    if (hand->n_palm_surf < 0 || hand->n_palm_caps < 0 || (hand->n_palm_surf > 0 && !hand->palm_surf) ||
        (hand->n_palm_caps > 0 && !hand->palm_caps) || hand->n_palm_surf > (1 << 20) || hand->n_palm_caps > 1024)
        return fail(LG_EINVAL, "palm: need 0 <= n_palm_surf <= 2^20, 0 <= n_palm_caps <= 1024 and their arrays");
    for (int c = 0; c < hand->n_palm_caps; ++c)
        if (!(hand->palm_caps[7 * c + 6] >= 0.0f)) return fail(LG_EINVAL, "palm capsule radius must be >= 0");
    if (p->bins != 32 && p->bins != 64) return fail(LG_EINVAL, "bins must be 32 or 64");
    if (p->grid < 4 || p->grid > 128 || p->grid % 4 != 0) return fail(LG_EINVAL, "grid must be a multiple of 4 in 4..128");
    if (!(p->h > 0.0f)) return fail(LG_EINVAL, "h must be > 0");
    if (p->samples < 1 || p->samples > 0x7fffffffLL) return fail(LG_EINVAL, "samples must be 1..2^31-1");
    if (!p->grid_frame) return fail(LG_EINVAL, "null grid_frame");
    return LG_OK;
}

void free_field(lg_field *f)
{
    if (!f) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(f->device);
    (void)hipFree(f->d_params);
    (void)hipFree(f->d_axis_samples);
    (void)hipFree(f->d_bits);
    (void)hipFree(f->d_merged);
    (void)hipFree(f->d_wit);
    (void)hipSetDevice(cur);
    delete f;
}

__global__ void k_fill_i32(int32_t *__restrict__ p, int64_t n, int32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// Candidate table of the normal bins over a cube map of directions, in the
// GPU's own cube-map convention (the v_cube* instructions the query uses): a
// direction d goes to face f = 0..5 (+x, -x, +y, -y, +z, -z; on ties z before
// y before x) and face coordinates (s, t) in [-1, 1]^2, s = sc / |d_major|,
// t = tc / |d_major|, with
//   +x: d ~ (1, -t, -s)   -x: d ~ (-1, -t, s)   +y: d ~ (s, 1, t)
//   -y: d ~ (s, -1, -t)   +z: d ~ (s, -t, 1)    -z: d ~ (-s, -t, -1),
// and to cell (is, it) of a kLutRes x kLutRes grid over (s, t).  A cell lists,
// in increasing order, every bin whose dot product can come within kLutMargin
// of the best one anywhere in the closed cell (checked on a dense sub-grid of
// the cell; the margin exceeds the dot-product variation between sub-grid
// points), so the argmax over the candidates equals the argmax over all bins,
// also for a direction on a cell or face boundary.  Cells with more than four
// candidates are marked for the full search (0xffffffff).
static void cube_direction(int face, double s, double t, double *d)
{
    switch (face) {
    case 0: d[0] = 1.0; d[1] = -t; d[2] = -s; break;
    case 1: d[0] = -1.0; d[1] = -t; d[2] = s; break;
    case 2: d[0] = s; d[1] = 1.0; d[2] = t; break;
    case 3: d[0] = s; d[1] = -1.0; d[2] = -t; break;
    case 4: d[0] = s; d[1] = -t; d[2] = 1.0; break;
    default: d[0] = -s; d[1] = -t; d[2] = -1.0; break;
    }
}

static void build_bin_lut(const std::vector<float> &bc, int B, std::vector<uint32_t> &lut)
{
    const int R = kLutRes, SUB = 9;
    lut.assign(6 * R * R, 0xffffffffu);
    const double sub_step = 2.0 / R / (SUB - 1);           // in face coordinates
    const double margin = 2.0 * sub_step + 1e-4;            // angular spacing <= coordinate spacing
    for (int face = 0; face < 6; ++face) {
        for (int it = 0; it < R; ++it)
            for (int is = 0; is < R; ++is) {
                std::vector<int> cand;
                for (int st = 0; st < SUB; ++st)
                    for (int ss = 0; ss < SUB; ++ss) {
                        const double sv = -1.0 + 2.0 * (is + (double)ss / (SUB - 1)) / R;
                        const double tv = -1.0 + 2.0 * (it + (double)st / (SUB - 1)) / R;
                        double d[3];
                        cube_direction(face, sv, tv, d);
                        const double nd = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                        double best = -1e300, dots[kMaxBins];
                        for (int b = 0; b < B; ++b) {
                            dots[b] = (bc[3 * b] * d[0] + bc[3 * b + 1] * d[1] + bc[3 * b + 2] * d[2]) / nd;
                            best = std::max(best, dots[b]);
                        }
                        for (int b = 0; b < B; ++b)
                            if (dots[b] >= best - margin && std::find(cand.begin(), cand.end(), b) == cand.end())
                                cand.push_back(b);
                    }
                std::sort(cand.begin(), cand.end());
                if (cand.size() <= 4) {
                    // absent slots repeat the first candidate (the kernel evaluates all four)
                    uint32_t e = 0;
                    for (size_t i = 0; i < 4; ++i) e |= (uint32_t)cand[i < cand.size() ? i : 0] << (8 * i);
                    lut[(face * R + it) * R + is] = e;
                }
            }
    }
}

// Lattice form of the windows (see DevHand::lat): every frame has finger 0's
// rotation (same floats), G is a power of two, and each origin is a whole
// number of 4-voxel bricks from finger 0's, within 1e-4 voxel (a few float
// ulps of the origins; the window faces move by far less than the 1e-6 m
// bands in which the oracle flags voxel decisions).  Otherwise lat = 0 and
// every kernel maps each finger's window on its own.
static void set_lattice(DevHand &H, const float *gf)
{
    H.lat = 0;
    const int F = H.F, G = H.G;
    if (G < 4 || (G & (G - 1)) != 0) return;
    for (int f = 1; f < F; ++f)
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c)
                if (gf[12 * f + 4 * r + c] != gf[4 * r + c]) return;
    long k[kMaxFingers][3];
    long lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int f = 0; f < F; ++f) {
        const double d[3] = {(double)gf[12 * f + 3] - gf[3], (double)gf[12 * f + 7] - gf[7],
                             (double)gf[12 * f + 11] - gf[11]};
        for (int a = 0; a < 3; ++a) {
            // a-th coordinate in finger 0's frame: column a of its rotation
            const double u = (gf[a] * d[0] + gf[4 + a] * d[1] + gf[8 + a] * d[2]) / (double)H.h;
            const double r = 4.0 * std::nearbyint(u / 4.0);
            if (!(std::fabs(u - r) <= 1e-4) || std::fabs(r) > 4096.0) return;
            k[f][a] = (long)r;
            lo[a] = std::min(lo[a], k[f][a]);
            hi[a] = std::max(hi[a], k[f][a]);
        }
    }
    for (int a = 0; a < 3; ++a)
        if (hi[a] - lo[a] + 3L * G > 1024L) return;
    const uint32_t GB = (uint32_t)(G / 4), m = (uint32_t)(G - 1);
    for (int f = 0; f < F; ++f) {
        for (int a = 0; a < 3; ++a) H.lat_o[f][a] = (int)(k[f][a] - lo[a] + G);
        H.lat_pk[f] = (uint32_t)H.lat_o[f][0] | (uint32_t)H.lat_o[f][1] << 10 | (uint32_t)H.lat_o[f][2] << 20;
        H.lat_idx[f] = brick_word((uint32_t)H.lat_o[f][0], (uint32_t)H.lat_o[f][1], (uint32_t)H.lat_o[f][2], GB);
    }
    H.lat_hi = ~(m | m << 10 | m << 20);
    H.lat = 1;
}

// Copy the hand, compute bin centres and axis sample counts on the host,
// upload them and allocate the (zeroed) tables.
lg_status make_field_shell(const lg_hand_desc *hand, const lg_field_params *p, lg_field **out)
{
    lg_status st = validate_hand(hand, p);
    if (st != LG_OK) return st;
    if (!out) return fail(LG_EINVAL, "null out");
    lg_field *f = new lg_field();
    const int F = hand->n_fingers, J = hand->n_joints, G = p->grid, B = p->bins, S = hand->n_surf;
    (void)hipGetDevice(&f->device);
    f->joint_finger.assign(hand->joint_finger, hand->joint_finger + J);
    f->joint_parent.assign(hand->joint_parent, hand->joint_parent + J);
    f->origin.assign(hand->joint_origin, hand->joint_origin + 12 * J);
    f->axis.assign(hand->joint_axis, hand->joint_axis + 3 * J);
    f->capsule.assign(hand->capsule, hand->capsule + 7 * J);
    f->limits.assign(hand->limits, hand->limits + 2 * J);
    f->surf.assign(hand->surf, hand->surf + (size_t)6 * J * S);
    f->grid_frame.assign(p->grid_frame, p->grid_frame + 12 * F);
    const int PS = hand->n_palm_surf, PC = hand->n_palm_caps;
    if (PS > 0) f->palm_surf.assign(hand->palm_surf, hand->palm_surf + (size_t)6 * PS);
    if (PC > 0) f->palm_caps.assign(hand->palm_caps, hand->palm_caps + (size_t)7 * PC);
    // spherical Fibonacci lattice, evaluated in double and rounded once
    f->bin_c.resize(3 * B);
    const double golden = M_PI * (3.0 - sqrt(5.0));
    for (int b = 0; b < B; ++b) {
        const double z = 1.0 - (2.0 * b + 1.0) / B, r = sqrt(1.0 - z * z), ph = b * golden;
        f->bin_c[3 * b] = (float)(r * cos(ph));
        f->bin_c[3 * b + 1] = (float)(r * sin(ph));
        f->bin_c[3 * b + 2] = (float)z;
    }
    std::vector<uint32_t> lut;
    build_bin_lut(f->bin_c, B, lut);
    // capsule axis samples for the penetration test: one per mm, ends included
    // (links, then the palm's capsules, which take at least their two ends)
    f->axis_samples.resize(J + PC);
    for (int j = 0; j < J + PC; ++j) {
        const float *c = j < J ? hand->capsule + 7 * j : hand->palm_caps + 7 * (j - J);
        const double dx = (double)c[3] - c[0], dy = (double)c[4] - c[1], dz = (double)c[5] - c[2];
        const double L = sqrt((dx * dx + dy * dy) + dz * dz);
        f->axis_samples[j] = std::max((int32_t)ceil(L / 1e-3) + 1, j < J ? 1 : 2);
    }
    DevHand &H = f->dh;
    memset(&H, 0, sizeof H);
    H.F = F;
    H.J = J;
    H.G = G;
    H.B = B;
    H.W = B / 32;
    H.nsurf = S;
    H.h = p->h;
    H.inv_h = 1.0f / p->h;
    H.seed_lo = (uint32_t)p->seed;
    H.seed_hi = (uint32_t)(p->seed >> 32);
    H.samples = p->samples;
    int maxd = 0;
    for (int fi = 0; fi < F; ++fi) {
        int first = -1, d = 0;
        for (int j = 0; j < J; ++j)
            if (hand->joint_finger[j] == fi) {
                if (first < 0) first = j;
                ++d;
            }
        H.finger_first[fi] = first;
        H.finger_dof[fi] = d;
        maxd = std::max(maxd, d);
    }
    f->max_dof = maxd;
    set_lattice(H, p->grid_frame);
    // packed float parameters
    const size_t n_origin = f->origin.size(), n_axis = f->axis.size(), n_cap = f->capsule.size(),
                 n_lim = f->limits.size(), n_surf = f->surf.size(), n_gf = f->grid_frame.size(),
                 n_bc = f->bin_c.size(), n_ps = f->palm_surf.size(), n_pc = f->palm_caps.size();
    const size_t n_lut = lut.size();
    const size_t n_all = n_origin + n_axis + n_cap + n_lim + n_surf + n_gf + n_bc + n_ps + n_pc + n_lut;
    std::vector<float> packed;
    packed.reserve(n_all);
    for (auto *v : {&f->origin, &f->axis, &f->capsule, &f->limits, &f->surf, &f->grid_frame, &f->bin_c,
                    &f->palm_surf, &f->palm_caps})
        packed.insert(packed.end(), v->begin(), v->end());
    packed.resize(n_all);
    memcpy(packed.data() + (n_all - n_lut), lut.data(), n_lut * sizeof(uint32_t));
    const int64_t G3 = (int64_t)G * G * G;
    hipError_t e = hipMalloc(&f->d_params, n_all * sizeof(float));
    if (e == hipSuccess) e = hipMemcpy(f->d_params, packed.data(), n_all * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&f->d_axis_samples, (J + PC) * sizeof(int32_t));
    if (e == hipSuccess)
        e = hipMemcpy(f->d_axis_samples, f->axis_samples.data(), (J + PC) * sizeof(int32_t), hipMemcpyHostToDevice);
    const size_t bits_bytes = (size_t)J * G3 * H.W * 4, merged_bytes = (size_t)F * G3 * H.W * 4;
    if (e == hipSuccess) e = hipMalloc(&f->d_bits, bits_bytes);
    if (e == hipSuccess) e = hipMalloc(&f->d_merged, merged_bytes);
    if (e == hipSuccess) e = hipMemset(f->d_bits, 0, bits_bytes);
    if (e == hipSuccess) e = hipMemset(f->d_merged, 0, merged_bytes);
    size_t wit_bytes = 0;
    if (e == hipSuccess && p->keep_witness) {
        wit_bytes = (size_t)J * G3 * B * 4;
        e = hipMalloc(&f->d_wit, wit_bytes);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_fill_i32, dim3(2048), dim3(256), 0, nullptr, f->d_wit, (int64_t)J * G3 * B, kNoWitness);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipDeviceSynchronize();
        f->has_witness = true;
    }
    if (e != hipSuccess) {
        st = hip_fail(e, "field allocation");
        free_field(f);
        return st;
    }
    f->device_bytes = n_all * 4 + (J + PC) * 4 + bits_bytes + merged_bytes + wit_bytes;
    float *base = f->d_params;
    H.origin = base;
    base += n_origin;
    H.axis = base;
    base += n_axis;
    H.capsule = base;
    base += n_cap;
    H.limits = base;
    base += n_lim;
    H.surf = base;
    base += n_surf;
    H.grid_frame = base;
    base += n_gf;
    H.bin_c = base;
    base += n_bc;
    H.palm_surf = n_ps ? base : nullptr;
    base += n_ps;
    H.palm_caps = n_pc ? base : nullptr;
    base += n_pc;
    H.bin_lut = reinterpret_cast<const uint32_t *>(base);
    H.axis_samples = f->d_axis_samples;
    H.n_palm_surf = PS;
    H.n_palm_caps = PC;
    *out = f;
    return LG_OK;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
constexpr int kBuildThreads = 256;

// One thread per (finger, joint sample): sample q, walk the chain, and bin
// every surface sample of every link of the finger.  The check-before-atomic
// is safe because table bits only ever go 0 -> 1 and witnesses only decrease:
// a stale read can only cause a redundant atomic, never a lost update.
__global__ void __launch_bounds__(kBuildThreads)
k_field_build(DevHand H, uint32_t *__restrict__ bits, int32_t *__restrict__ wit,
              unsigned long long *__restrict__ dropped)
{
    __shared__ float cb[3 * kMaxBins];
    for (int i = threadIdx.x; i < 3 * H.B; i += blockDim.x) cb[i] = H.bin_c[i];
    __syncthreads();
    const int f = blockIdx.y;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = s < H.samples;
    const int first = H.finger_first[f], d = H.finger_dof[f];
    const int G = H.G, W = H.W, B = H.B;
    const int64_t G3 = (int64_t)G * G * G;
    const float *gf = H.grid_frame + 12 * f;
    unsigned int n_drop = 0;
    Tf T;
    for (int t = 0; t < d; ++t) {
        const int j = first + t;
        const float q = active ? joint_sample(H, f, (uint32_t)s, t) : 0.0f;
        T = joint_frame(H, T, t > 0, j, q);
        // composite link -> window map: u = R_f^T (T x - o_f) / h + G (biased, see window_voxel)
        Affine a;
        {
            const float dx = T.m[3] - gf[3], dy = T.m[7] - gf[7], dz = T.m[11] - gf[11];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    a.m[4 * r + c] = fmaf(gf[r], T.m[c], fmaf(gf[4 + r], T.m[4 + c], gf[8 + r] * T.m[8 + c])) * H.inv_h;
                a.m[4 * r + 3] = fmaf(fmaf(gf[r], dx, fmaf(gf[4 + r], dy, gf[8 + r] * dz)), H.inv_h, (float)G);
            }
        }
        if (!active) continue;
        const float *sp = H.surf + (size_t)j * H.nsurf * 6;
        uint32_t *tab = bits + (size_t)j * G3 * W;
        int32_t *wtab = wit ? wit + (size_t)j * G3 * B : nullptr;
        int last_v = -2, last_b = -1;
        for (int i = 0; i < H.nsurf; ++i) {
            const float px = sp[6 * i], py = sp[6 * i + 1], pz = sp[6 * i + 2];
            const int v = window_voxel(a, G, px, py, pz);
            if (v < 0) {
                ++n_drop;
                continue;
            }
            float nx, ny, nz;
            tf_dir(T, sp[6 * i + 3], sp[6 * i + 4], sp[6 * i + 5], nx, ny, nz);
            const int b = nearest_bin(cb, B, nx, ny, nz);
            if (v == last_v && b == last_b) continue;  // same cell as the previous sample
            last_v = v;
            last_b = b;
            uint32_t *wp = tab + (size_t)v * W + (b >> 5);
            const uint32_t m = 1u << (b & 31);
            if (!(__atomic_load_n(wp, __ATOMIC_RELAXED) & m)) atomicOr(wp, m);
            if (wtab) {
                int32_t *ww = wtab + (size_t)v * B + b;
                if (__atomic_load_n(ww, __ATOMIC_RELAXED) > (int32_t)s) atomicMin(ww, (int32_t)s);
            }
        }
    }
    // wave-level sum of dropped vectors, one atomic per wave
    unsigned long long c = n_drop;
    for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(dropped, c);
}

// Merged finger tables: OR over the links of finger f of their words, laid
// out as merged[f][w][brick_word(v)] (one plane per 32-bin word w, 4x4x4
// voxel bricks), from the canonical per-link tables bits[l][v][w].
__global__ void k_field_merge(DevHand H, const uint32_t *__restrict__ bits, uint32_t *__restrict__ merged)
{
    const int G = H.G, W = H.W;
    const int64_t G3 = (int64_t)G * G * G, G3W = G3 * W;
    const int f = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < G3W; i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t acc = 0;
        const int first = H.finger_first[f], d = H.finger_dof[f];
        for (int t = 0; t < d; ++t) acc |= bits[(int64_t)(first + t) * G3W + i];
        const int64_t v = i / W;
        const int w = (int)(i - v * W);
        const uint32_t ix = (uint32_t)(v % G), iy = (uint32_t)((v / G) % G), iz = (uint32_t)(v / ((int64_t)G * G));
        merged[((int64_t)f * W + w) * G3 + brick_word(ix, iy, iz, (uint32_t)(G / 4))] = acc;
    }
}

__global__ void k_popcount(const uint32_t *__restrict__ w, int64_t n, unsigned long long *__restrict__ out)
{
    unsigned long long c = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        c += __popc(w[i]);
    for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, c);
}

static lg_status merge_and_count(lg_field *f, hipStream_t st)
{
    const DevHand &H = f->dh;
    const int64_t G3W = (int64_t)H.G * H.G * H.G * H.W;
    dim3 grid((unsigned)std::min<int64_t>((G3W + 255) / 256, 4096), H.F);
    hipLaunchKernelGGL(k_field_merge, grid, dim3(256), 0, st, H, f->d_bits, f->d_merged);
    LG_HIP(hipGetLastError());
    unsigned long long *d_cnt = nullptr;
    LG_HIP(hipMalloc(&d_cnt, sizeof(unsigned long long)));
    (void)hipMemsetAsync(d_cnt, 0, sizeof(unsigned long long), st);
    hipLaunchKernelGGL(k_popcount, dim3(1024), dim3(256), 0, st, f->d_bits, (int64_t)H.J * G3W, d_cnt);
    unsigned long long cnt = 0;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&cnt, d_cnt, sizeof cnt, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d_cnt);
    if (e != hipSuccess) return hip_fail(e, "field merge");
    f->bits_set = cnt;
    return LG_OK;
}

}  // namespace lg

using namespace lg;

extern "C" {

const char *lg_status_str(lg_status s)
{
    switch (s) {
    case LG_OK: return "LG_OK";
    case LG_EINVAL: return "LG_EINVAL";
    case LG_ENOMEM: return "LG_ENOMEM";
    case LG_EDEVICE: return "LG_EDEVICE";
    case LG_EUNSUPPORTED: return "LG_EUNSUPPORTED";
    case LG_EINTERNAL: return "LG_EINTERNAL";
    default: return "LG_UNKNOWN";
    }
}

const char *lg_last_error(void) { return g_last_error.c_str(); }

const char *lg_version(void) { return "lg-gfx950 0.1.0"; }

lg_status lg_build_field(const lg_hand_desc *hand, const lg_field_params *params, void *stream, lg_field **out)
{
    lg_field *f = nullptr;
    lg_status st = make_field_shell(hand, params, &f);
    if (st != LG_OK) return st;
    hipStream_t s = as_stream(stream);
    const DevHand &H = f->dh;
    unsigned long long *d_drop = nullptr;
    hipError_t e = hipMalloc(&d_drop, sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMemsetAsync(d_drop, 0, sizeof(unsigned long long), s);
    if (e != hipSuccess) {
        free_field(f);
        return hip_fail(e, "build scratch");
    }
    dim3 grid((unsigned)((H.samples + kBuildThreads - 1) / kBuildThreads), H.F);
    // the build kernel's own duration (events on the build stream), reported by lg_field_info
    hipEvent_t ev[2] = {nullptr, nullptr};
    if (e == hipSuccess) e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    if (e == hipSuccess) e = hipEventRecord(ev[0], s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_field_build, grid, dim3(kBuildThreads), 0, s, H, f->d_bits, f->d_wit, d_drop);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(ev[1], s);
    unsigned long long drop = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&drop, d_drop, sizeof drop, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    float build_ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&build_ms, ev[0], ev[1]);
    f->build_kernel_ms = build_ms;
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    (void)hipFree(d_drop);
    if (e != hipSuccess) {
        free_field(f);
        return hip_fail(e, "k_field_build");
    }
    // dropped counts every (sample, surface point) outside the window
    f->dropped = (int64_t)drop;
    f->vectors = H.samples * (int64_t)H.J * H.nsurf;
    st = merge_and_count(f, s);
    if (st != LG_OK) {
        free_field(f);
        return st;
    }
    *out = f;
    return LG_OK;
}

lg_status lg_field_import(const lg_hand_desc *hand, const lg_field_params *params, const uint32_t *bits_host,
                          const int32_t *witness_host, lg_field **out)
{
    if (!bits_host) return fail(LG_EINVAL, "null bits_host");
    lg_field_params p = *params;
    p.keep_witness = witness_host != nullptr;
    lg_field *f = nullptr;
    lg_status st = make_field_shell(hand, &p, &f);
    if (st != LG_OK) return st;
    const DevHand &H = f->dh;
    const int64_t G3 = (int64_t)H.G * H.G * H.G;
    hipError_t e = hipMemcpy(f->d_bits, bits_host, (size_t)H.J * G3 * H.W * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess && witness_host) {
        const size_t n = (size_t)H.J * G3 * H.B;
        std::vector<int32_t> w(witness_host, witness_host + n);
        for (auto &x : w)
            if (x < 0) x = kNoWitness;
        e = hipMemcpy(f->d_wit, w.data(), n * 4, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        free_field(f);
        return hip_fail(e, "field import");
    }
    f->vectors = 0;
    f->dropped = 0;
    st = merge_and_count(f, nullptr);
    if (st != LG_OK) {
        free_field(f);
        return st;
    }
    *out = f;
    return LG_OK;
}

lg_status lg_field_export(const lg_field *f, uint32_t *bits_host, int32_t *witness_host)
{
    if (!f || !bits_host) return fail(LG_EINVAL, "null field or bits_host");
    const DevHand &H = f->dh;
    const int64_t G3 = (int64_t)H.G * H.G * H.G;
    LG_HIP(hipDeviceSynchronize());
    LG_HIP(hipMemcpy(bits_host, f->d_bits, (size_t)H.J * G3 * H.W * 4, hipMemcpyDeviceToHost));
    if (witness_host) {
        const size_t n = (size_t)H.J * G3 * H.B;
        if (!f->d_wit) {
            memset(witness_host, 0xff, n * 4);
        } else {
            LG_HIP(hipMemcpy(witness_host, f->d_wit, n * 4, hipMemcpyDeviceToHost));
            for (size_t i = 0; i < n; ++i)
                if (witness_host[i] < 0 || witness_host[i] >= (int32_t)H.samples) witness_host[i] = -1;
        }
    }
    return LG_OK;
}

lg_status lg_field_info(const lg_field *f, lg_field_info_t *info)
{
    if (!f || !info) return fail(LG_EINVAL, "null field or info");
    info->n_fingers = f->dh.F;
    info->n_joints = f->dh.J;
    info->grid = f->dh.G;
    info->bins = f->dh.B;
    info->samples = f->dh.samples;
    info->device_bytes = f->device_bytes;
    info->bits_set = f->bits_set;
    info->vectors = f->vectors;
    info->dropped = f->dropped;
    info->has_witness = f->has_witness ? 1 : 0;
    info->lattice = f->dh.lat;
    info->build_kernel_ms = f->build_kernel_ms;
    return LG_OK;
}

lg_status lg_field_release(lg_field *f)
{
    free_field(f);
    return LG_OK;
}

}  // extern "C"
