/*
 * FP64 CPU oracle of the Contact-Field pipeline (Lightning Grasp,
 * arXiv 2511.07418).  TEST INFRASTRUCTURE ONLY: it is loaded by the tests,
 * by the smoke check and by the CPU-baseline leg of the benchmark, never by
 * the product path.  It shares no code with the HIP library.
 *
 * Plain, slow, obviously-correct C11 in double precision.  Inputs arrive as
 * float32 arrays (the library's formats) and are promoted exactly.  Every
 * discrete decision (voxel, normal bin, LP verdict, acceptance thresholds) is
 * also reported with a boundary flag so that a float32 implementation can be
 * compared bit-exactly on everything that is not within the stated bands:
 *   - voxel: a coordinate within 1e-6 m of a voxel face,
 *   - bin:   a direction within 1e-6 rad of a bin (Voronoi) boundary,
 *            measured as (theta2 - theta1)/2,
 *   - verdict / thresholds: within 1e-6 of the threshold.
 *
 * Build: gcc -O2 -std=c11 -fopenmp -ffp-contract=off -shared -fPIC.
 */
#define _DEFAULT_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>

/* threads of the parallel loops (timing at one thread and at all cores) */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_get_threads(void) { return omp_get_max_threads(); }
#endif

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2

#define BAND_POS 1e-6   /* m   */
#define BAND_ANG 1e-6   /* rad */
#define BAND_VAL 1e-6   /* thresholds (t*, contact error, angle, depth) */
#define BAND_CHOICE 1e-6 /* m: IK contact-point choice between two distant capsule candidates */
/* causes of a realize flag (bit mask) */
#define RF_THRESHOLD 1u /* contact error, angle or depth within BAND_VAL of its threshold */
#define RF_LOOKUP 2u    /* reverse lookup: voxel face within BAND_POS or bin boundary within BAND_ANG */
#define RF_CHOICE 4u    /* an IK contact-point choice within BAND_CHOICE of a tie */

#define PURPOSE_JOINT 1u
#define PURPOSE_DRAW 3u
#define PURPOSE_OPT 5u
#define PURPOSE_PLACE 11u
#define PURPOSE_FINGERS 13u
#define PURPOSE_UNUSED 15u
#define PURPOSE_PALM 17u
#define PURPOSE_EXT_FINGERS 19u
#define PURPOSE_EXT_DRAW 21u
#define OPT_TAU 1e-9    /* candidates within OPT_TAU of the best criterion value tie */
#define OPT_BAND 1e-7   /* m: projection near-tie band (FP32 candidate positions err by ~1e-8 m) */

/* ------------------------------------------------------------------------ */
/* Hand description (host arrays, float32 as in the library ABI)             */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t n_fingers;
    int32_t n_joints;
    const int32_t *joint_finger;  /* [J] */
    const int32_t *joint_parent;  /* [J] -1 = hand base */
    const float *joint_origin;    /* [J][12] parent->joint 3x4 row-major */
    const float *joint_axis;      /* [J][3] */
    const float *capsule;         /* [J][7] a, b, r (link frame) */
    const float *limits;          /* [J][2] */
    int32_t n_surf;
    const float *surf;            /* [J][n_surf][6] link-frame point, normal */
} orc_hand;

typedef struct {
    int64_t samples;      /* S per finger */
    uint64_t seed;        /* Philox key */
    int32_t grid;         /* G */
    double h;             /* voxel edge */
    int32_t bins;         /* B: 32 or 64 */
    const float *grid_frame; /* [F][12] [R | o]: u = R^T (x - o) / h */
} orc_field_params;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as    */
/* easy as 1, 2, 3", SC'11).  Counter-based: four 32-bit counter words, two   */
/* 32-bit key words, ten rounds of two 32x32->64 multiplies, the key bumped   */
/* by the Weyl constants between rounds.                                      */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t m0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t m1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(m1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)m1;
        uint32_t y2 = (uint32_t)(m0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)m0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static double u01(uint32_t w) { return (double)(w >> 8) * (1.0 / 16777216.0); }

static int finger_first_joint(const orc_hand *H, int f)
{
    for (int j = 0; j < H->n_joints; ++j)
        if (H->joint_finger[j] == f) return j;
    return -1;
}

static int finger_dof(const orc_hand *H, int f)
{
    int n = 0;
    for (int j = 0; j < H->n_joints; ++j) n += (H->joint_finger[j] == f);
    return n;
}

/* Joint sample s of finger f (Sec. 4.3: random joint configurations).
 * Joint t of the finger uses word t%4 of the block with counter
 * (s, 8f + t/4, JOINT, 0); q = lo + (hi - lo) * u01.                         */
void orc_joint_sample(const orc_hand *H, uint64_t seed, int f, int64_t s, double *q_out)
{
    int j0 = finger_first_joint(H, f), d = finger_dof(H, f);
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int t = 0; t < d; ++t) {
        uint32_t ctr[4] = {(uint32_t)s, (uint32_t)(8 * f + t / 4), PURPOSE_JOINT, 0u};
        uint32_t w[4];
        orc_philox4x32_10(ctr, key, w);
        double lo = H->limits[2 * (j0 + t)], hi = H->limits[2 * (j0 + t) + 1];
        q_out[t] = lo + (hi - lo) * u01(w[t % 4]);
    }
}

/* ------------------------------------------------------------------------ */
/* Rigid transforms: 3x4 row-major [R | t]                                   */
/* ------------------------------------------------------------------------ */
static void tf_load(const float *src, double *T)
{
    for (int i = 0; i < 12; ++i) T[i] = src[i];
}

static void tf_mul(const double *A, const double *B, double *C)
{
    double R[12];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j)
            R[4 * i + j] = A[4 * i] * B[j] + A[4 * i + 1] * B[4 + j] + A[4 * i + 2] * B[8 + j];
        R[4 * i + 3] = A[4 * i] * B[3] + A[4 * i + 1] * B[7] + A[4 * i + 2] * B[11] + A[4 * i + 3];
    }
    memcpy(C, R, sizeof R);
}

static void tf_point(const double *T, const double *p, double *x)
{
    for (int i = 0; i < 3; ++i)
        x[i] = T[4 * i] * p[0] + T[4 * i + 1] * p[1] + T[4 * i + 2] * p[2] + T[4 * i + 3];
}

static void tf_dir(const double *T, const double *p, double *x)
{
    for (int i = 0; i < 3; ++i)
        x[i] = T[4 * i] * p[0] + T[4 * i + 1] * p[1] + T[4 * i + 2] * p[2];
}

/* Rotation by angle q about unit axis a (Rodrigues' formula). */
static void tf_axis_angle(const double *a, double q, double *T)
{
    double c = cos(q), s = sin(q), v = 1.0 - c;
    double x = a[0], y = a[1], z = a[2];
    T[0] = c + x * x * v;     T[1] = x * y * v - z * s; T[2] = x * z * v + y * s;  T[3] = 0;
    T[4] = y * x * v + z * s; T[5] = c + y * y * v;     T[6] = y * z * v - x * s;  T[7] = 0;
    T[8] = z * x * v - y * s; T[9] = z * y * v + x * s; T[10] = c + z * z * v;     T[11] = 0;
}

/* Forward kinematics F of Sec. 3.1 for the joints of finger f:
 * T_j = T_parent * origin_j * Rot(axis_j, q_j).  q_f holds the finger's
 * joints in chain order; frames are written for those joints only (index by
 * global joint id).                                                          */
void orc_fk_finger(const orc_hand *H, int f, const double *q_f, double *T /*[J][12]*/)
{
    int t = 0;
    for (int j = 0; j < H->n_joints; ++j) {
        if (H->joint_finger[j] != f) continue;
        double O[12], Rq[12], P[12];
        tf_load(H->joint_origin + 12 * j, O);
        if (H->joint_parent[j] >= 0)
            tf_mul(T + 12 * H->joint_parent[j], O, P);
        else
            memcpy(P, O, sizeof P);
        double ax[3] = {H->joint_axis[3 * j], H->joint_axis[3 * j + 1], H->joint_axis[3 * j + 2]};
        tf_axis_angle(ax, q_f[t], Rq);
        tf_mul(P, Rq, T + 12 * j);
        ++t;
    }
}

/* All fingers: q holds all J joints in joint order. */
void orc_fk(const orc_hand *H, const double *q, double *T)
{
    for (int f = 0; f < H->n_fingers; ++f) {
        int j0 = finger_first_joint(H, f);
        orc_fk_finger(H, f, q + j0, T);
    }
}

/* ------------------------------------------------------------------------ */
/* Normal bins: spherical Fibonacci lattice, nearest centre = argmax dot      */
/* (the paper quantises normals onto a compact unit sphere, Sec. 4.4).        */
/* ------------------------------------------------------------------------ */
void orc_bin_centers(int B, double *c)
{
    const double golden = M_PI * (3.0 - sqrt(5.0));
    for (int b = 0; b < B; ++b) {
        double z = 1.0 - (2.0 * b + 1.0) / B;
        double r = sqrt(1.0 - z * z);
        double ph = b * golden;
        c[3 * b] = r * cos(ph);
        c[3 * b + 1] = r * sin(ph);
        c[3 * b + 2] = z;
    }
}

/* Best bin of direction d (not necessarily unit) with ties to the lowest
 * index; second best bin; half the angular gap (theta2 - theta1)/2.          */
static int bin_of(int B, const double *c, const double *d, int *second, double *half_gap)
{
    double nd = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    int b1 = -1, b2 = -1;
    double s1 = -1e300, s2 = -1e300;
    for (int b = 0; b < B; ++b) {
        double s = c[3 * b] * d[0] + c[3 * b + 1] * d[1] + c[3 * b + 2] * d[2];
        if (s > s1) { s2 = s1; b2 = b1; s1 = s; b1 = b; }
        else if (s > s2) { s2 = s; b2 = b; }
    }
    if (second) *second = b2;
    if (half_gap) {
        double c1 = s1 / nd, c2 = s2 / nd;
        if (c1 > 1) c1 = 1;
        if (c2 > 1) c2 = 1;
        if (c1 < -1) c1 = -1;
        if (c2 < -1) c2 = -1;
        *half_gap = 0.5 * (acos(c2) - acos(c1));
    }
    return b1;
}

int orc_bin(int B, const double *d, int *second, double *half_gap)
{
    double c[3 * 256];
    if (B <= 0 || B > 256) return -1;
    orc_bin_centers(B, c);
    return bin_of(B, c, d, second, half_gap);
}

/* Voxel coordinates of hand-frame point x in finger window f:
 * u = R^T (x - o) / h.  Returns 1 if inside [0, G)^3.                        */
static int voxel_coords(const orc_field_params *fp, int f, const double *x, double *u)
{
    const float *F = fp->grid_frame + 12 * f;
    double d[3] = {x[0] - F[3], x[1] - F[7], x[2] - F[11]};
    int in = 1;
    for (int a = 0; a < 3; ++a) {
        u[a] = (F[a] * d[0] + F[4 + a] * d[1] + F[8 + a] * d[2]) / fp->h;
        if (!(u[a] >= 0.0 && u[a] < (double)fp->grid)) in = 0;
    }
    return in;
}

/* distance (m) of coordinate u (voxel units) to the nearest voxel face
 * (integer), including the window faces 0 and G                             */
static double face_dist(double u, double h)
{
    double r = u - floor(u);
    double d = r < 0.5 ? r : 1.0 - r;
    return d * h;
}

/* ------------------------------------------------------------------------ */
/* Field construction (Sec. 4.3, Algorithm 1, and Sec. 4.4):                  */
/* for every finger f, joint sample s, link l of f and surface sample (p, n)  */
/* of l: contact vector x = T_l(q_s) p, nu = R_l(q_s) n; the grid cover of    */
/* width h assigns x to voxel floor(u) (dropped if outside the window) and    */
/* the normal is quantised to bin argmax_b <nu, c_b>; the bit of (l, voxel,   */
/* bin) is set and the smallest sample index s reaching it is kept as the     */
/* witness used by the reverse lookup of Sec. 5.5.                             */
/*                                                                            */
/* Outputs (canonical layout, voxel v = (iz*G + iy)*G + ix, word = b/32,      */
/* bit = b%32):                                                               */
/*   bits  [L][G^3][B/32]   every vector at its float64 voxel/bin              */
/*   sure  [L][G^3][B/32]   cells set by at least one unflagged vector         */
/*   maybe [L][G^3][B/32]   cells a flagged vector may reach (its cell, the    */
/*                          neighbour across each near face, the 2nd bin)     */
/*   wit   [L][G^3][B]      min s over `bits` contributions (optional)         */
/*   wit_lo[L][G^3][B]      min s over any possible contribution (optional)   */
/*   wit_hi[L][G^3][B]      min s over unflagged contributions (optional)     */
/*   stats [4]: vectors, in-window vectors, dropped, flagged                  */
/* ------------------------------------------------------------------------ */
static inline void set_bit(uint32_t *w, int64_t v, int nw, int b)
{
    w[v * nw + (b >> 5)] |= 1u << (b & 31);
}

static inline void wmin(int32_t *w, int64_t idx, int32_t s)
{
    if (w[idx] < 0 || s < w[idx]) w[idx] = s;
}

int orc_build_field(const orc_hand *H, const orc_field_params *fp,
                    uint32_t *bits, uint32_t *sure, uint32_t *maybe,
                    int32_t *wit, int32_t *wit_lo, int32_t *wit_hi, int64_t *stats,
                    const int64_t *sample_ids /* NULL: samples 0..S-1 */, int64_t n_ids)
{
    const int G = fp->grid, B = fp->bins, J = H->n_joints;
    if (G <= 0 || (B != 32 && B != 64) || fp->h <= 0 || fp->samples <= 0) return ORC_EINVAL;
    const int nw = B / 32;
    const int64_t G3 = (int64_t)G * G * G;
    const int64_t words = (int64_t)J * G3 * nw;
    if (bits) memset(bits, 0, words * 4);
    if (sure) memset(sure, 0, words * 4);
    if (maybe) memset(maybe, 0, words * 4);
    int32_t *wits[3] = {wit, wit_lo, wit_hi};
    for (int i = 0; i < 3; ++i)
        if (wits[i]) memset(wits[i], 0xff, (size_t)J * G3 * B * 4); /* -1 = none */
    double cb[3 * 64];
    orc_bin_centers(B, cb);
    int64_t n_vec = 0, n_in = 0, n_flag = 0;

    /* one link per task: each task owns its link's tables (no races) */
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : n_vec, n_in, n_flag)
    for (int l = 0; l < J; ++l) {
        const int f = H->joint_finger[l];
        const int j0 = finger_first_joint(H, f);
        double q[32], T[12 * 64];
        const int64_t lbase = (int64_t)l * G3;
        const int64_t n_s = sample_ids ? n_ids : fp->samples;
        for (int64_t si = 0; si < n_s; ++si) {
            const int64_t s = sample_ids ? sample_ids[si] : si;
            orc_joint_sample(H, fp->seed, f, s, q);
            orc_fk_finger(H, f, q, T);
            (void)j0;
            const double *Tl = T + 12 * l;
            for (int i = 0; i < H->n_surf; ++i) {
                const float *sp = H->surf + ((int64_t)l * H->n_surf + i) * 6;
                double p[3] = {sp[0], sp[1], sp[2]}, n[3] = {sp[3], sp[4], sp[5]};
                double x[3], nu[3], u[3];
                tf_point(Tl, p, x);
                tf_dir(Tl, n, nu);
                ++n_vec;
                int in = voxel_coords(fp, f, x, u);
                int b2;
                double gap;
                int b = bin_of(B, cb, nu, &b2, &gap);
                int near_face[3];
                int flagged = gap < BAND_ANG;
                for (int a = 0; a < 3; ++a) {
                    near_face[a] = face_dist(u[a], fp->h) < BAND_POS;
                    flagged |= near_face[a];
                }
                /* a vector just outside the window can be inside at float32 */
                int ix[3];
                for (int a = 0; a < 3; ++a) ix[a] = (int)floor(u[a]);
                if (in) {
                    ++n_in;
                    int64_t v = lbase + ((int64_t)ix[2] * G + ix[1]) * G + ix[0];
                    if (bits) set_bit(bits, v, nw, b);
                    if (wit) wmin(wit, v * B + b, (int32_t)s);
                    if (!flagged) {
                        if (sure) set_bit(sure, v, nw, b);
                        if (wit_hi) wmin(wit_hi, v * B + b, (int32_t)s);
                    }
                }
                if (!flagged) {
                    if (in && wit_lo) {
                        int64_t v = lbase + ((int64_t)ix[2] * G + ix[1]) * G + ix[0];
                        wmin(wit_lo, v * B + b, (int32_t)s);
                    }
                    continue;
                }
                ++n_flag;
                /* enumerate alternative voxels (+-1 across near faces) and bins */
                int lo3[3], hi3[3];
                for (int a = 0; a < 3; ++a) {
                    lo3[a] = hi3[a] = ix[a];
                    if (near_face[a]) {
                        double r = u[a] - floor(u[a]);
                        if (r < 0.5) lo3[a] = ix[a] - 1; else hi3[a] = ix[a] + 1;
                    }
                }
                int nb = gap < BAND_ANG ? 2 : 1;
                int bb[2] = {b, b2};
                for (int zz = lo3[2]; zz <= hi3[2]; ++zz)
                    for (int yy = lo3[1]; yy <= hi3[1]; ++yy)
                        for (int xx = lo3[0]; xx <= hi3[0]; ++xx) {
                            if (xx < 0 || yy < 0 || zz < 0 || xx >= G || yy >= G || zz >= G) continue;
                            int64_t v = lbase + ((int64_t)zz * G + yy) * G + xx;
                            for (int k = 0; k < nb; ++k) {
                                if (maybe) set_bit(maybe, v, nw, bb[k]);
                                if (wit_lo) wmin(wit_lo, v * B + bb[k], (int32_t)s);
                            }
                        }
            }
        }
    }
    if (stats) {
        stats[0] = n_vec;
        stats[1] = n_in;
        stats[2] = n_vec - n_in;
        stats[3] = n_flag;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Object contact query (Sec. 4.2-4.3, Def. 4.3, Sec. 5.3).                  */
/* For pose (R, t) and object point (p, n): x = R p + t, nu = R n; the query  */
/* vector is (x, -nu) (the contact surface representation negates the         */
/* normal).  Link l hits if bit bin(-nu) of its table at voxel(x) is set      */
/* (0 outside the window); the domain of finger f (a dependency group) is the */
/* OR over its links.  dom_bits[g][f][w] bit i%32 of word i/32 is point i.    */
/* dom_flag marks (g, f, i) whose value could change under the float32        */
/* rounding bands (some alternative voxel/bin gives a different OR).          */
/* ------------------------------------------------------------------------ */
static int link_hits_at(const orc_hand *H, const orc_field_params *fp, const uint32_t *bits,
                        int f, const int *vox, int in, int b, uint32_t *mask)
{
    const int G = fp->grid, nw = fp->bins / 32;
    const int64_t G3 = (int64_t)G * G * G;
    uint32_t m = 0;
    int t = 0, any = 0;
    for (int l = 0; l < H->n_joints; ++l) {
        if (H->joint_finger[l] != f) continue;
        if (in) {
            int64_t v = (int64_t)l * G3 + ((int64_t)vox[2] * G + vox[1]) * G + vox[0];
            if ((bits[v * nw + (b >> 5)] >> (b & 31)) & 1u) {
                m |= 1u << t;
                any = 1;
            }
        }
        ++t;
    }
    if (mask) *mask = m;
    return any;
}

/* transform + voxel + bin for one (pose, point, finger); returns in-window */
static int query_lookup(const orc_field_params *fp, const double *cb, const float *pose,
                        const float *pt, const float *nm, int f,
                        double *x, double *u, int *vox, int *b, int *b2, double *gap)
{
    double p[3] = {pt[0], pt[1], pt[2]}, n[3] = {nm[0], nm[1], nm[2]};
    double T[12];
    tf_load(pose, T);
    double nu[3], q[3];
    tf_point(T, p, x);
    tf_dir(T, n, nu);
    q[0] = -nu[0]; q[1] = -nu[1]; q[2] = -nu[2];
    *b = bin_of(fp->bins, cb, q, b2, gap);
    int in = voxel_coords(fp, f, x, u);
    for (int a = 0; a < 3; ++a) vox[a] = (int)floor(u[a]);
    return in;
}

int orc_query(const orc_hand *H, const orc_field_params *fp, const uint32_t *bits,
              const float *pts /*[N][3]*/, const float *nrm /*[N][3]*/, int32_t n_points,
              const float *poses /*[P][12]*/, int32_t n_poses,
              uint32_t *dom_bits, uint32_t *dom_count, uint32_t *dom_flag, int64_t *lookups)
{
    const int F = H->n_fingers, G = fp->grid;
    const int64_t NW = (n_points + 31) / 32;
    if (n_points < 0 || n_poses < 0) return ORC_EINVAL;
    double cb[3 * 64];
    orc_bin_centers(fp->bins, cb);
    int64_t n_lookup = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : n_lookup)
    for (int g = 0; g < n_poses; ++g) {
        for (int f = 0; f < F; ++f) {
            uint32_t *db = dom_bits + ((int64_t)g * F + f) * NW;
            uint32_t *df = dom_flag ? dom_flag + ((int64_t)g * F + f) * NW : NULL;
            memset(db, 0, NW * 4);
            if (df) memset(df, 0, NW * 4);
            uint32_t cnt = 0;
            for (int i = 0; i < n_points; ++i) {
                double x[3], u[3];
                int vox[3], b, b2;
                double gap;
                int in = query_lookup(fp, cb, poses + 12 * (int64_t)g, pts + 3 * (int64_t)i,
                                      nrm + 3 * (int64_t)i, f, x, u, vox, &b, &b2, &gap);
                if (in) n_lookup += finger_dof(H, f);
                int hit = link_hits_at(H, fp, bits, f, vox, in, b, NULL);
                if (hit) {
                    db[i >> 5] |= 1u << (i & 31);
                    ++cnt;
                }
                if (!df) continue;
                /* boundary flag: does any alternative outcome differ? */
                int near[3], any_near = 0;
                for (int a = 0; a < 3; ++a) {
                    near[a] = face_dist(u[a], fp->h) < BAND_POS;
                    any_near |= near[a];
                }
                int bin_near = gap < BAND_ANG;
                if (!any_near && !bin_near) continue;
                int lo3[3], hi3[3];
                for (int a = 0; a < 3; ++a) {
                    lo3[a] = hi3[a] = vox[a];
                    if (near[a]) {
                        double r = u[a] - floor(u[a]);
                        if (r < 0.5) lo3[a] = vox[a] - 1; else hi3[a] = vox[a] + 1;
                    }
                }
                int bb[2] = {b, b2}, nb = bin_near ? 2 : 1, differs = 0;
                for (int zz = lo3[2]; zz <= hi3[2] && !differs; ++zz)
                    for (int yy = lo3[1]; yy <= hi3[1] && !differs; ++yy)
                        for (int xx = lo3[0]; xx <= hi3[0] && !differs; ++xx) {
                            int v3[3] = {xx, yy, zz};
                            int in2 = xx >= 0 && yy >= 0 && zz >= 0 && xx < G && yy < G && zz < G;
                            for (int k = 0; k < nb; ++k)
                                if (link_hits_at(H, fp, bits, f, v3, in2, bb[k], NULL) != hit)
                                    differs = 1;
                        }
                if (differs) df[i >> 5] |= 1u << (i & 31);
            }
            dom_count[(int64_t)g * F + f] = cnt;
        }
    }
    if (lookups) *lookups = n_lookup;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Cone query (Sec. 4.3, the theta_hit test of the object contact query): a   */
/* query (x, -nu) hits link l if some normal of l's field at voxel(x), i.e.   */
/* a bin centre c_b whose bit is set, satisfies c_b . (-nu) >= cos_hit.  The  */
/* domain of finger f is the OR over its links.  dom_flag marks points whose  */
/* outcome could change under the float32 bands: a voxel face within 1e-6 m  */
/* (as in orc_query) or a set bin whose dot product is within 1e-6 of        */
/* cos_hit.                                                                   */
/* ------------------------------------------------------------------------ */
static int cone_hit(const orc_hand *H, const orc_field_params *fp, const uint32_t *bits, const double *cb, int f,
                    const int *vox, int in, const double *q, double cos_hit, int *near)
{
    if (!in) return 0;
    const int G = fp->grid, B = fp->bins, nw = B / 32;
    const int64_t G3 = (int64_t)G * G * G;
    int hit = 0;
    for (int l = 0; l < H->n_joints; ++l) {
        if (H->joint_finger[l] != f) continue;
        const int64_t v = (int64_t)l * G3 + ((int64_t)vox[2] * G + vox[1]) * G + vox[0];
        for (int b = 0; b < B; ++b) {
            if (!((bits[v * nw + (b >> 5)] >> (b & 31)) & 1u)) continue;
            const double d = cb[3 * b] * q[0] + cb[3 * b + 1] * q[1] + cb[3 * b + 2] * q[2];
            if (d >= cos_hit) hit = 1;
            if (near && fabs(d - cos_hit) <= BAND_VAL) *near = 1;
        }
    }
    return hit;
}

int orc_query_cone(const orc_hand *H, const orc_field_params *fp, const uint32_t *bits,
                   const float *pts /*[N][3]*/, const float *nrm /*[N][3]*/, int32_t n_points,
                   const float *poses /*[P][12]*/, int32_t n_poses, double cos_hit,
                   uint32_t *dom_bits, uint32_t *dom_count, uint32_t *dom_flag)
{
    const int F = H->n_fingers, G = fp->grid;
    const int64_t NW = (n_points + 31) / 32;
    if (n_points < 0 || n_poses < 0) return ORC_EINVAL;
    double cb[3 * 64];
    orc_bin_centers(fp->bins, cb);
#pragma omp parallel for schedule(dynamic, 1)
    for (int g = 0; g < n_poses; ++g) {
        for (int f = 0; f < F; ++f) {
            uint32_t *db = dom_bits + ((int64_t)g * F + f) * NW;
            uint32_t *df = dom_flag ? dom_flag + ((int64_t)g * F + f) * NW : NULL;
            memset(db, 0, NW * 4);
            if (df) memset(df, 0, NW * 4);
            uint32_t cnt = 0;
            for (int i = 0; i < n_points; ++i) {
                double x[3], u[3], gap;
                int vox[3], b, b2;
                int in = query_lookup(fp, cb, poses + 12 * (int64_t)g, pts + 3 * (int64_t)i,
                                      nrm + 3 * (int64_t)i, f, x, u, vox, &b, &b2, &gap);
                double T[12], nu[3], q[3];
                tf_load(poses + 12 * (int64_t)g, T);
                const double n[3] = {nrm[3 * (int64_t)i], nrm[3 * (int64_t)i + 1], nrm[3 * (int64_t)i + 2]};
                tf_dir(T, n, nu);
                for (int c = 0; c < 3; ++c) q[c] = -nu[c];
                int near_ang = 0;
                const int hit = cone_hit(H, fp, bits, cb, f, vox, in, q, cos_hit, &near_ang);
                if (hit) {
                    db[i >> 5] |= 1u << (i & 31);
                    ++cnt;
                }
                if (!df) continue;
                int near[3], any_near = 0;
                for (int a = 0; a < 3; ++a) {
                    near[a] = face_dist(u[a], fp->h) < BAND_POS;
                    any_near |= near[a];
                }
                int differs = near_ang;
                if (any_near && !differs) {
                    int lo3[3], hi3[3];
                    for (int a = 0; a < 3; ++a) {
                        lo3[a] = hi3[a] = vox[a];
                        if (near[a]) {
                            double r = u[a] - floor(u[a]);
                            if (r < 0.5) lo3[a] = vox[a] - 1; else hi3[a] = vox[a] + 1;
                        }
                    }
                    for (int zz = lo3[2]; zz <= hi3[2] && !differs; ++zz)
                        for (int yy = lo3[1]; yy <= hi3[1] && !differs; ++yy)
                            for (int xx = lo3[0]; xx <= hi3[0] && !differs; ++xx) {
                                int v3[3] = {xx, yy, zz};
                                int in2 = xx >= 0 && yy >= 0 && zz >= 0 && xx < G && yy < G && zz < G;
                                if (cone_hit(H, fp, bits, cb, f, v3, in2, q, cos_hit, NULL) != hit) differs = 1;
                            }
                }
                if (differs) df[i >> 5] |= 1u << (i & 31);
            }
            dom_count[(int64_t)g * F + f] = cnt;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Contact-set draws (Sec. 5.3: one domain per dependency group, then one     */
/* point per domain, Alg. 2 initialisation) and the reverse lookup of the     */
/* hand link (Sec. 5.5: pick one of the active patch fields at random).       */
/* Contact i lies on finger i (k == F).  Philox block (g, 4d + blk, DRAW,     */
/* request_id); words 0..k-1 pick points, words k..2k-1 pick links.  The      */
/* j-th set bit is selected with j = floor(r * count / 2^32).                 */
/* ------------------------------------------------------------------------ */
static int64_t select1(const uint32_t *words, int64_t nw, uint32_t j)
{
    uint32_t seen = 0;
    for (int64_t w = 0; w < nw; ++w) {
        uint32_t x = words[w];
        for (int b = 0; b < 32; ++b) {
            if ((x >> b) & 1u) {
                if (seen == j) return w * 32 + b;
                ++seen;
            }
        }
    }
    return -1;
}

static uint32_t popcount32(uint32_t x)
{
    uint32_t c = 0;
    for (int b = 0; b < 32; ++b) c += (x >> b) & 1u;
    return c;
}

static void draw_words(uint64_t seed, uint32_t request_id, int64_t g, int d, int n, uint32_t *w)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int blk = 0; blk * 4 < n; ++blk) {
        uint32_t ctr[4] = {(uint32_t)g, (uint32_t)(4 * d + blk), PURPOSE_DRAW, request_id};
        orc_philox4x32_10(ctr, key, w + 4 * blk);
    }
}

/* the floor(r * popcount(mask) / 2^32)-th link of finger f in mask (bit t =
 * the finger's t-th link); -1 for an empty mask */
static int link_of_mask(const orc_hand *H, int f, uint32_t mask, uint32_t r)
{
    uint32_t pc = popcount32(mask);
    if (pc == 0) return -1;
    uint32_t jj = (uint32_t)(((uint64_t)r * pc) >> 32);
    uint32_t seen = 0;
    int t = 0;
    for (int l = 0; l < H->n_joints; ++l) {
        if (H->joint_finger[l] != f) continue;
        if ((mask >> t) & 1u) {
            if (seen == jj) return l;
            ++seen;
        }
        ++t;
    }
    return -1;
}

/* Reverse lookup of the link (Sec. 5.5): among the links of finger f whose
 * table bit is set at point idx under the pose, the floor(r * count / 2^32)-th;
 * -1 if none.  *flag (optional) is set when the voxel lies within 1e-6 m of a
 * face or the bin within 1e-6 rad of a boundary and a cell on the other side
 * gives another link (an implementation in float32 may take either). */
static int pick_link(const orc_hand *H, const orc_field_params *fp, const uint32_t *bits, const double *cb,
                     const float *pts, const float *nrm, const float *pose, int f, int64_t idx, uint32_t r,
                     int *flag)
{
    double x[3], u[3], gap;
    int vox[3], b, b2;
    int in = query_lookup(fp, cb, pose, pts + 3 * idx, nrm + 3 * idx, f, x, u, vox, &b, &b2, &gap);
    uint32_t mask = 0;
    link_hits_at(H, fp, bits, f, vox, in, b, &mask);
    const int link = link_of_mask(H, f, mask, r);
    if (!flag) return link;
    *flag = 0;
    const int G = fp->grid;
    int near[3], any_near = 0;
    for (int a = 0; a < 3; ++a) {
        near[a] = face_dist(u[a], fp->h) < BAND_POS;
        any_near |= near[a];
    }
    const int bin_near = gap < BAND_ANG;
    if (!any_near && !bin_near) return link;
    int lo3[3], hi3[3];
    for (int a = 0; a < 3; ++a) {
        lo3[a] = hi3[a] = vox[a];
        if (near[a]) {
            double rr = u[a] - floor(u[a]);
            if (rr < 0.5) lo3[a] = vox[a] - 1; else hi3[a] = vox[a] + 1;
        }
    }
    int bb[2] = {b, b2}, nb = bin_near ? 2 : 1;
    for (int zz = lo3[2]; zz <= hi3[2]; ++zz)
        for (int yy = lo3[1]; yy <= hi3[1]; ++yy)
            for (int xx = lo3[0]; xx <= hi3[0]; ++xx) {
                int v3[3] = {xx, yy, zz};
                int in2 = xx >= 0 && yy >= 0 && zz >= 0 && xx < G && yy < G && zz < G;
                for (int kk = 0; kk < nb; ++kk) {
                    uint32_t m2 = 0;
                    link_hits_at(H, fp, bits, f, v3, in2, bb[kk], &m2);
                    if (link_of_mask(H, f, m2, r) != link) *flag = 1;
                }
            }
    return link;
}

/* The k contact fingers of set d of pose g (Sec. 5.3: k contact domains
 * chosen at random among the fingers' domains).  Eligible fingers are those
 * with a non-empty domain; with c of them, k picks without replacement: pick
 * j takes the floor(w_j (c - j) / 2^32)-th (0-based, increasing finger order)
 * of the eligible fingers not yet picked, w = Philox blocks (g, d,
 * PURPOSE_FINGERS | blk << 8, request_id), blk = 0, 1.  Contact i goes to the
 * i-th smallest picked finger.  Returns 0 when fewer than k are eligible.  */
int orc_choose_fingers(int F, const uint32_t *count /*[F]*/, int k, uint64_t seed, uint32_t request_id,
                       int64_t g, int d, int32_t *fing /*[k]*/)
{
    int left[8], c = 0;
    for (int f = 0; f < F; ++f)
        if (count[f] > 0) left[c++] = f;
    if (k < 1 || c < k) return 0;
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[8];
    for (int blk = 0; blk < 2; ++blk) {
        uint32_t ctr[4] = {(uint32_t)g, (uint32_t)d, PURPOSE_FINGERS | ((uint32_t)blk << 8), request_id};
        orc_philox4x32_10(ctr, key, w + 4 * blk);
    }
    int picked[8];
    for (int j = 0; j < k; ++j) {
        int r = (int)(((uint64_t)w[j] * (uint32_t)(c - j)) >> 32);
        picked[j] = left[r];
        for (int t = r; t + 1 < c - j; ++t) left[t] = left[t + 1];  /* remove it, keep the order */
    }
    /* increasing finger order */
    for (int a = 1; a < k; ++a)
        for (int b = a; b > 0 && picked[b - 1] > picked[b]; --b) {
            int t = picked[b];
            picked[b] = picked[b - 1];
            picked[b - 1] = t;
        }
    for (int j = 0; j < k; ++j) fing[j] = picked[j];
    return 1;
}

int orc_draw(const orc_hand *H, const orc_field_params *fp, const uint32_t *bits,
             const float *pts, const float *nrm, int32_t n_points,
             const float *poses, int32_t n_poses,
             const uint32_t *dom_bits, const uint32_t *dom_count,
             int32_t draws, int32_t k, uint64_t seed, uint32_t request_id, int64_t pose_offset,
             const int32_t *palm_pt /*[P] or NULL: -2 = rejected placement, no sets*/,
             int32_t *set_pt /*[P][D][k]*/, int32_t *set_link /*[P][D][k]*/,
             uint8_t *link_flag /*[P][D][k] or NULL: link decided inside a band (see pick_link)*/)
{
    const int F = H->n_fingers;
    const int64_t NW = (n_points + 31) / 32;
    if (k < 1 || k > F || k > 8 || draws <= 0) return ORC_EINVAL;
    double cb[3 * 64];
    orc_bin_centers(fp->bins, cb);
#pragma omp parallel for schedule(dynamic, 4)
    for (int g = 0; g < n_poses; ++g) {
        for (int d = 0; d < draws; ++d) {
            uint32_t w[16];
            draw_words(seed, request_id, pose_offset + g, d, 2 * k, w);
            int32_t *sp = set_pt + ((int64_t)g * draws + d) * k;
            int32_t *sl = set_link + ((int64_t)g * draws + d) * k;
            int32_t fing[8];
            uint8_t *lf = link_flag ? link_flag + ((int64_t)g * draws + d) * k : NULL;
            for (int i = 0; i < k; ++i) { sp[i] = -1; sl[i] = -1; if (lf) lf[i] = 0; }
            if (palm_pt && palm_pt[g] == -2) continue;
            if (!orc_choose_fingers(F, dom_count + (int64_t)g * F, k, seed, request_id, pose_offset + g, d, fing))
                continue;
            for (int i = 0; i < k; ++i) {
                const int f = fing[i];
                uint32_t cnt = dom_count[(int64_t)g * F + f];
                uint32_t j = (uint32_t)(((uint64_t)w[i] * cnt) >> 32);
                int64_t idx = select1(dom_bits + ((int64_t)g * F + f) * NW, NW, j);
                sp[i] = (int32_t)idx;
                int fl = 0;
                sl[i] = idx < 0 ? -1
                                : pick_link(H, fp, bits, cb, pts, nrm, poses + 12 * (int64_t)g, f, idx, w[k + i],
                                            lf ? &fl : NULL);
                if (lf) lf[i] = (uint8_t)fl;
            }
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Second contact round on the unused fingers (Sec. 5.3's additional search   */
/* phase, named the general form in Sec. 5.6).  A round-1 set (k1 contacts on */
/* k1 fingers) marked in take[] gets k_add more contacts on fingers that it   */
/* does not use and whose domain is non-empty:                                */
/*  - fingers: with c such fingers (c >= k_add, else the set is not          */
/*    extended), pick j takes the floor(w_j (c - j) / 2^32)-th remaining one  */
/*    in increasing finger order, w = Philox blocks (g, d,                    */
/*    PURPOSE_EXT_FINGERS | blk << 8, request_id), blk = 0, 1;                */
/*  - points and links: Philox blocks (g, 4d + blk, PURPOSE_EXT_DRAW,         */
/*    request_id): word i picks the point of the i-th smallest new finger as  */
/*    the floor(w * count / 2^32)-th domain point, word k_add + i its link by */
/*    the reverse lookup;                                                     */
/*  - the extended set lists all k1 + k_add contacts in increasing finger     */
/*    order (its verdict is that of the larger set, orc_verdicts).            */
/* A round-1 set whose contacts lack a point or a link is not extended.  Not  */
/* extended: every entry -1.  g is the global pose index (pose_offset + local). */
/* ------------------------------------------------------------------------ */
int orc_extend(const orc_hand *H, const orc_field_params *fp, const uint32_t *bits,
               const float *pts, const float *nrm, int32_t n_points, const float *poses, int32_t n_poses,
               const uint32_t *dom_bits, const uint32_t *dom_count, int32_t draws, int32_t k1,
               const int32_t *set_pt1 /*[P][D][k1]*/, const int32_t *set_link1, const uint8_t *take /*[P][D]*/,
               int32_t k_add, uint64_t seed, uint32_t request_id, int64_t pose_offset,
               int32_t *set_pt2 /*[P][D][k1 + k_add]*/, int32_t *set_link2,
               uint8_t *link_flag /*[P][D][k1 + k_add] or NULL*/)
{
    const int F = H->n_fingers, k2 = k1 + k_add;
    const int64_t NW = (n_points + 31) / 32;
    if (k1 < 1 || k_add < 1 || k2 > F || k2 > 8 || draws <= 0) return ORC_EINVAL;
    double cb[3 * 64];
    orc_bin_centers(fp->bins, cb);
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
#pragma omp parallel for schedule(dynamic, 4)
    for (int g = 0; g < n_poses; ++g) {
        const int64_t gg = pose_offset + g;
        for (int d = 0; d < draws; ++d) {
            const int64_t s = (int64_t)g * draws + d;
            int32_t *sp2 = set_pt2 + s * k2;
            int32_t *sl2 = set_link2 + s * k2;
            uint8_t *lf = link_flag ? link_flag + s * k2 : NULL;
            for (int i = 0; i < k2; ++i) { sp2[i] = -1; sl2[i] = -1; if (lf) lf[i] = 0; }
            if (!take[s]) continue;
            const int32_t *sp1 = set_pt1 + s * k1, *sl1 = set_link1 + s * k1;
            int used[8] = {0}, fin1[8], ok = 1;
            for (int i = 0; i < k1; ++i) {
                if (sp1[i] < 0 || sl1[i] < 0 || sl1[i] >= H->n_joints) { ok = 0; break; }
                fin1[i] = H->joint_finger[sl1[i]];
                used[fin1[i]] = 1;
            }
            if (!ok) continue;
            int left[8], c = 0;
            for (int f = 0; f < F; ++f)
                if (!used[f] && dom_count[(int64_t)g * F + f] > 0) left[c++] = f;
            if (c < k_add) continue;
            uint32_t wf[8];
            for (int blk = 0; blk < 2; ++blk) {
                uint32_t ctr[4] = {(uint32_t)gg, (uint32_t)d, PURPOSE_EXT_FINGERS | ((uint32_t)blk << 8), request_id};
                orc_philox4x32_10(ctr, key, wf + 4 * blk);
            }
            int newf[8];
            for (int j = 0; j < k_add; ++j) {
                int r = (int)(((uint64_t)wf[j] * (uint32_t)(c - j)) >> 32);
                newf[j] = left[r];
                for (int t = r; t + 1 < c - j; ++t) left[t] = left[t + 1];
            }
            for (int a = 1; a < k_add; ++a)
                for (int b = a; b > 0 && newf[b - 1] > newf[b]; --b) {
                    int t = newf[b];
                    newf[b] = newf[b - 1];
                    newf[b - 1] = t;
                }
            uint32_t w[16];
            for (int blk = 0; blk * 4 < 2 * k_add; ++blk) {
                uint32_t ctr[4] = {(uint32_t)gg, (uint32_t)(4 * d + blk), PURPOSE_EXT_DRAW, request_id};
                orc_philox4x32_10(ctr, key, w + 4 * blk);
            }
            int32_t np[8], nl[8];
            int nf[8];
            for (int i = 0; i < k_add; ++i) {
                const int f = newf[i];
                const uint32_t cnt = dom_count[(int64_t)g * F + f];
                const uint32_t j = (uint32_t)(((uint64_t)w[i] * cnt) >> 32);
                const int64_t idx = select1(dom_bits + ((int64_t)g * F + f) * NW, NW, j);
                int fl = 0;
                np[i] = (int32_t)idx;
                nl[i] = idx < 0 ? -1 : pick_link(H, fp, bits, cb, pts, nrm, poses + 12 * (int64_t)g, f, idx,
                                                 w[k_add + i], &fl);
                nf[i] = fl;
            }
            /* union in increasing finger order (both groups are sorted) */
            int a = 0, b = 0;
            for (int o = 0; o < k2; ++o) {
                const int take_old = b >= k_add || (a < k1 && fin1[a] < newf[b]);
                if (take_old) {
                    sp2[o] = sp1[a];
                    sl2[o] = sl1[a];
                    ++a;
                } else {
                    sp2[o] = np[b];
                    sl2[o] = nl[b];
                    if (lf) lf[o] = (uint8_t)nf[b];
                    ++b;
                }
            }
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Contact-set criterion (Sec. 3.2, Eq. 1-2) as a linear program.             */
/* Friction cones are linearised with m edges around the contact normal:     */
/*   d_ie = -n_i + mu (cos(2 pi e/m) x_i + sin(2 pi e/m) y_i),                */
/* with (x_i, y_i) the branchless orthonormal tangent basis of Duff et al.    */
/* (JCGT 2017) and the moment rows scaled by 1/rho:                           */
/*   w_ie = [d_ie ; (p_i x d_ie) / rho].                                       */
/* t* = min sum_r |(W g)_r|  s.t. g >= 0, sum g = 1, solved exactly by a      */
/* dense Phase-1 simplex with Bland's rule.  t* = 0 iff a non-trivial         */
/* self-balancing combination of contact forces exists.                       */
/* status: 0 optimal, 1 pivot cap reached (undecided).                         */
/* ------------------------------------------------------------------------ */
static void duff_basis(const double *n, double *x, double *y)
{
    double sign = copysign(1.0, n[2]);
    double a = -1.0 / (sign + n[2]);
    double b = n[0] * n[1] * a;
    x[0] = 1.0 + sign * n[0] * n[0] * a;
    x[1] = sign * b;
    x[2] = -sign * n[0];
    y[0] = b;
    y[1] = sign + n[1] * n[1] * a;
    y[2] = -n[1];
}

void orc_tangent_basis(const double *n, double *x, double *y) { duff_basis(n, x, y); }

/* wrench columns, W[c][6] with c = i*m + e */
void orc_wrench_matrix(int k, const double *p, const double *n, double mu, int m, double rho,
                       double *W)
{
    for (int i = 0; i < k; ++i) {
        double x[3], y[3];
        duff_basis(n + 3 * i, x, y);
        for (int e = 0; e < m; ++e) {
            double th = 2.0 * M_PI * e / m;
            double ce = cos(th), se = sin(th);
            double d[3];
            for (int a = 0; a < 3; ++a) d[a] = -n[3 * i + a] + mu * (ce * x[a] + se * y[a]);
            const double *pi = p + 3 * i;
            double *w = W + 6 * (i * m + e);
            w[0] = d[0]; w[1] = d[1]; w[2] = d[2];
            w[3] = (pi[1] * d[2] - pi[2] * d[1]) / rho;
            w[4] = (pi[2] * d[0] - pi[0] * d[2]) / rho;
            w[5] = (pi[0] * d[1] - pi[1] * d[0]) / rho;
        }
    }
}

#define LP_TOL 1e-12   /* reduced-cost and ratio-tie tolerance */
#define LP_PIV 1e-9    /* smallest admissible pivot element */

/* column j of the constraint matrix [W^T -I I; 1 0 0] (7 rows) */
static void lp_column(int n, const double *W, int j, double *a)
{
    for (int r = 0; r < 7; ++r) a[r] = 0.0;
    if (j < n) {
        for (int r = 0; r < 6; ++r) a[r] = W[6 * j + r];
        a[6] = 1.0;
    } else if (j < n + 6) {
        a[j - n] = -1.0;
    } else {
        a[j - n - 6] = 1.0;
    }
}

/* Rebuild the tableau B^-1 [A | b] of `basis` from the original columns
 * (Gauss-Jordan with partial pivoting).  Returns -1 if B is singular.       */
static int lp_reinvert(int n, const double *W, const int *basis, double *T)
{
    const int nv = n + 12;
    double M[7][14];
    for (int r = 0; r < 7; ++r) {
        double a[7];
        lp_column(n, W, basis[r], a);
        for (int i = 0; i < 7; ++i) M[i][r] = a[i];
        for (int i = 0; i < 7; ++i) M[r][7 + i] = 0.0;
    }
    for (int r = 0; r < 7; ++r) M[r][7 + r] = 1.0;
    for (int c = 0; c < 7; ++c) {
        int p = c;
        for (int r = c + 1; r < 7; ++r)
            if (fabs(M[r][c]) > fabs(M[p][c])) p = r;
        if (fabs(M[p][c]) < 1e-300) return -1;
        if (p != c)
            for (int i = 0; i < 14; ++i) {
                double t = M[c][i];
                M[c][i] = M[p][i];
                M[p][i] = t;
            }
        double pv = M[c][c];
        for (int i = 0; i < 14; ++i) M[c][i] /= pv;
        for (int r = 0; r < 7; ++r) {
            if (r == c || M[r][c] == 0.0) continue;
            double f = M[r][c];
            for (int i = 0; i < 14; ++i) M[r][i] -= f * M[c][i];
        }
    }
    /* T_j = B^-1 A_j; rhs = B^-1 e_6 (row r of the tableau belongs to basis[r]) */
    for (int j = 0; j < nv; ++j) {
        double a[7];
        lp_column(n, W, j, a);
        for (int r = 0; r < 7; ++r) {
            double s = 0.0;
            for (int i = 0; i < 7; ++i) s += M[r][7 + i] * a[i];
            T[r * (nv + 1) + j] = s;
        }
    }
    for (int r = 0; r < 7; ++r) T[r * (nv + 1) + nv] = M[r][7 + 6];
    return 0;
}

/* Phase-1 LP on n columns (6 numbers each).  Variables: g_0..g_{n-1},
 * s+_0..s+_5, s-_0..s-_5 (column index order used by Bland's rule).  When
 * no reduced cost is negative the tableau is rebuilt from the original
 * columns of the final basis and optimality is checked again, so rounding
 * accumulated over long degenerate pivot sequences cannot end the search
 * early or bias t*.                                                          */
double orc_lp_solve(int n, const double *W, int max_pivots, int *status, int *pivots)
{
    const int nv = n + 12, rows = 7;
    double *T = (double *)calloc((size_t)rows * (nv + 1), sizeof(double));
    double *red = (double *)calloc((size_t)nv, sizeof(double));
    int basis[7];
    if (!T || !red) {
        free(T); free(red);
        if (status) *status = -1;
        return NAN;
    }
#define TA(r, c) T[(r) * (nv + 1) + (c)]
    for (int r = 0; r < 6; ++r) {
        for (int c = 0; c < n; ++c) TA(r, c) = W[6 * c + r];
        TA(r, n + r) = -1.0;    /* s+ */
        TA(r, n + 6 + r) = 1.0; /* s- */
        TA(r, nv) = 0.0;
    }
    for (int c = 0; c < n; ++c) TA(6, c) = 1.0;
    TA(6, nv) = 1.0;
    /* initial basis: g_0 for the normalisation row, one slack per wrench row */
    for (int r = 0; r < 6; ++r) {
        double f = TA(r, 0);
        for (int c = 0; c <= nv; ++c) TA(r, c) -= f * TA(6, c);
        if (TA(r, nv) >= 0.0) {
            basis[r] = n + 6 + r;
        } else {
            for (int c = 0; c <= nv; ++c) TA(r, c) = -TA(r, c);
            basis[r] = n + r;
        }
    }
    basis[6] = 0;
    int piv = 0, st = 0, checks = 0;
    for (;;) {
        /* reduced costs d_j = c_j - c_B^T T_j */
        for (int j = 0; j < nv; ++j) {
            double z = 0.0;
            for (int r = 0; r < rows; ++r)
                if (basis[r] >= n) z += TA(r, j);
            red[j] = (j >= n ? 1.0 : 0.0) - z;
        }
        int e = -1;
        for (int j = 0; j < nv; ++j)
            if (red[j] < -LP_TOL) { e = j; break; }
        if (e < 0) {
            /* candidate optimum: verify on a freshly inverted basis */
            if (checks >= 4 || lp_reinvert(n, W, basis, T) != 0) break;
            ++checks;
            int again = 0;
            for (int j = 0; j < nv && !again; ++j) {
                double z = 0.0;
                for (int r = 0; r < rows; ++r)
                    if (basis[r] >= n) z += TA(r, j);
                if ((j >= n ? 1.0 : 0.0) - z < -LP_TOL) again = 1;
            }
            if (!again) break;
            continue;
        }
        if (piv >= max_pivots) { st = 1; break; }
        int lr = -1;
        double best = 0.0;
        for (int r = 0; r < rows; ++r) {
            if (TA(r, e) > LP_PIV) {
                double ratio = TA(r, nv) / TA(r, e);
                if (lr < 0 || ratio < best - LP_TOL * (1.0 + fabs(best)) ||
                    (fabs(ratio - best) <= LP_TOL * (1.0 + fabs(best)) && basis[r] < basis[lr])) {
                    lr = r;
                    best = ratio;
                }
            }
        }
        if (lr < 0) { st = 2; break; } /* unbounded: impossible for this LP */
        double pv = TA(lr, e);
        for (int c = 0; c <= nv; ++c) TA(lr, c) /= pv;
        for (int r = 0; r < rows; ++r) {
            if (r == lr) continue;
            double f = TA(r, e);
            if (f != 0.0)
                for (int c = 0; c <= nv; ++c) TA(r, c) -= f * TA(lr, c);
        }
        basis[lr] = e;
        ++piv;
    }
    double t = 0.0;
    for (int r = 0; r < rows; ++r)
        if (basis[r] >= n) t += TA(r, nv);
#undef TA
    free(T);
    free(red);
    if (status) *status = st;
    if (pivots) *pivots = piv;
    return t;
}

/* t* for one contact set given object-frame points/normals */
double orc_set_tstar(int k, const double *p, const double *n, double mu, int m, double rho,
                     int max_pivots, int *status, int *pivots)
{
    double *W = (double *)malloc(sizeof(double) * 6 * k * m);
    orc_wrench_matrix(k, p, n, mu, m, rho, W);
    double t = orc_lp_solve(k * m, W, max_pivots, status, pivots);
    free(W);
    return t;
}

/* Batch verdicts for drawn sets.  verdict = valid set and t* <= eps;
 * vflag marks |t* - eps| <= 1e-6.                                           */
int orc_verdicts(const float *pts, const float *nrm, int32_t n_sets, int32_t k,
                 const int32_t *set_pt, double mu, int32_t m_edges, double rho, double eps,
                 int32_t max_pivots, uint8_t *verdict, double *tstar, uint8_t *vflag, int32_t *status)
{
    if (k <= 0 || k * m_edges + 12 > 4096 || rho <= 0) return ORC_EINVAL;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t s = 0; s < n_sets; ++s) {
        const int32_t *sp = set_pt + s * k;
        int valid = 1;
        for (int i = 0; i < k; ++i) valid &= sp[i] >= 0;
        if (!valid) {
            verdict[s] = 0;
            if (tstar) tstar[s] = NAN;
            if (vflag) vflag[s] = 0;
            if (status) status[s] = 0;
            continue;
        }
        double p[3 * 16], n[3 * 16];
        for (int i = 0; i < k; ++i)
            for (int a = 0; a < 3; ++a) {
                p[3 * i + a] = pts[3 * (int64_t)sp[i] + a];
                n[3 * i + a] = nrm[3 * (int64_t)sp[i] + a];
            }
        int st, pv;
        double t = orc_set_tstar(k, p, n, mu, m_edges, rho, max_pivots, &st, &pv);
        verdict[s] = (st == 0 && t <= eps);
        if (tstar) tstar[s] = t;
        if (vflag) vflag[s] = fabs(t - eps) <= BAND_VAL;
        if (status) status[s] = st;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Exhaustive placement (Sec. 5.1): a random contact vector of the field      */
/* (finger f, joint sample s, link l of f, surface sample j: hand-frame point */
/* x and outward normal nu after FK) receives a random object point (p, n):   */
/* the pose maps n onto -nu (the minimal rotation, then a roll psi about -nu) */
/* and p onto x.  Pose g draws Philox blocks (g + pose_offset, b, PLACE,      */
/* request_id), b = 0, 1: f, s, t (link index within f), j from words 0-3 as  */
/* floor(w * count / 2^32); the object point from word 4; psi = 2 pi u(w5).   */
/* The minimal rotation of unit a onto unit b: I + [v]x + [v]x^2 / (1 + c),   */
/* v = a x b, c = a.b; for c <= -0.9999 a half-turn about the Duff x-axis of  */
/* a first (a -> -a), then the minimal rotation of -a onto b.  pflag marks    */
/* |c + 0.9999| <= 1e-5 (the branch is a float decision on the GPU).          */
/* ------------------------------------------------------------------------ */
static double dot3(const double *a, const double *b);

static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static void mat3_mul(const double *A, const double *B, double *C)
{
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) C[3 * r + c] = A[3 * r] * B[c] + A[3 * r + 1] * B[3 + c] + A[3 * r + 2] * B[6 + c];
}

static void rot_min(const double *a, const double *b, double *R)
{
    double v[3];
    cross3(a, b, v);
    const double c = a[0] * b[0] + a[1] * b[1] + a[2] * b[2], k = 1.0 / (1.0 + c);
    const double K[9] = {0, -v[2], v[1], v[2], 0, -v[0], -v[1], v[0], 0};
    double K2[9];
    mat3_mul(K, K, K2);
    for (int i = 0; i < 9; ++i) R[i] = (i % 4 == 0 ? 1.0 : 0.0) + K[i] + K2[i] * k;
}

/* flip = 1 takes the other branch of a rotation whose cosine is inside the
 * branch band (an implementation in other precision may take it) */
static void rot_align_pick(const double *a_in, const double *b_in, double *R, int *flag, int flip)
{
    double a[3], b[3];
    const double na = sqrt(dot3(a_in, a_in)), nb = sqrt(dot3(b_in, b_in));
    for (int i = 0; i < 3; ++i) {
        a[i] = a_in[i] / na;
        b[i] = b_in[i] / nb;
    }
    const double c = dot3(a, b);
    const int band = fabs(c + 0.9999) <= 1e-5;
    if (flag) *flag = band;
    if ((c > -0.9999) != (flip && band)) {
        rot_min(a, b, R);
        return;
    }
    double x[3], y[3];
    duff_basis(a, x, y);
    double Rh[9];
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) Rh[3 * r + q] = 2.0 * x[r] * x[q] - (r == q ? 1.0 : 0.0);
    const double na2[3] = {-a[0], -a[1], -a[2]};
    double Rm[9];
    rot_min(na2, b, Rm);
    mat3_mul(Rm, Rh, R);
}

void orc_rot_align(const double *a_in, const double *b_in, double *R, int *flag)
{
    rot_align_pick(a_in, b_in, R, flag, 0);
}

int orc_place_exhaustive(const orc_hand *H, const orc_field_params *fp, const float *pts, const float *nrm,
                         int32_t n_points, int32_t n_poses, uint64_t seed, uint32_t request_id, int64_t pose_offset,
                         double *poses /*[P][12]*/, uint8_t *pflag)
{
    if (n_points <= 0 || n_poses < 0 || fp->samples <= 0 || fp->samples > 0xffffffffLL) return ORC_EINVAL;
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
#pragma omp parallel for schedule(static)
    for (int g = 0; g < n_poses; ++g) {
        uint32_t w[8];
        for (int b = 0; b < 2; ++b) {
            uint32_t ctr[4] = {(uint32_t)(pose_offset + g), (uint32_t)b, PURPOSE_PLACE, request_id};
            orc_philox4x32_10(ctr, key, w + 4 * b);
        }
        const int f = (int)(((uint64_t)w[0] * (uint64_t)H->n_fingers) >> 32);
        const int64_t smp = (int64_t)(((uint64_t)w[1] * (uint64_t)fp->samples) >> 32);
        const int j0 = finger_first_joint(H, f), d = finger_dof(H, f);
        const int l = j0 + (int)(((uint64_t)w[2] * (uint64_t)d) >> 32);
        const int js = (int)(((uint64_t)w[3] * (uint64_t)H->n_surf) >> 32);
        const int64_t i = (int64_t)(((uint64_t)w[4] * (uint64_t)n_points) >> 32);
        const double psi = 2.0 * M_PI * u01(w[5]);
        double q[16];
        orc_joint_sample(H, fp->seed, f, smp, q);
        double *T = (double *)malloc(sizeof(double) * 12 * H->n_joints);
        orc_fk_finger(H, f, q, T);
        const float *sf = H->surf + ((int64_t)l * H->n_surf + js) * 6;
        const double ps[3] = {sf[0], sf[1], sf[2]}, ns[3] = {sf[3], sf[4], sf[5]};
        double x[3], nu[3];
        tf_point(T + 12 * l, ps, x);
        tf_dir(T + 12 * l, ns, nu);
        free(T);
        const double a[3] = {nrm[3 * i], nrm[3 * i + 1], nrm[3 * i + 2]};
        double b[3] = {-nu[0], -nu[1], -nu[2]};
        const double nb = sqrt(dot3(b, b));
        for (int c = 0; c < 3; ++c) b[c] /= nb;
        double R0[9], Rr[9], R[9];
        int fl = 0;
        orc_rot_align(a, b, R0, &fl);
        /* roll psi about b (Rodrigues) */
        const double cs = cos(psi), sn = sin(psi);
        const double K[9] = {0, -b[2], b[1], b[2], 0, -b[0], -b[1], b[0], 0};
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c)
                Rr[3 * r + c] = (r == c ? cs : 0.0) + sn * K[3 * r + c] + (1.0 - cs) * b[r] * b[c];
        mat3_mul(Rr, R0, R);
        const double p[3] = {pts[3 * i], pts[3 * i + 1], pts[3 * i + 2]};
        double *P = poses + 12 * (int64_t)g;
        for (int r = 0; r < 3; ++r) {
            P[4 * r + 0] = R[3 * r];
            P[4 * r + 1] = R[3 * r + 1];
            P[4 * r + 2] = R[3 * r + 2];
            P[4 * r + 3] = x[r] - (R[3 * r] * p[0] + R[3 * r + 1] * p[1] + R[3 * r + 2] * p[2]);
        }
        if (pflag) pflag[g] = (uint8_t)fl;
    }
    return ORC_OK;
}

/* Object signed-distance grid (object frame): trilinear between nodes, +inf
 * outside the grid (orc_sdf_eval below). */
typedef struct {
    double origin[3];
    double h;
    int32_t dims;
    const float *values; /* [G][G][G] as [iz][iy][ix] */
} orc_sdf;
double orc_sdf_eval(const orc_sdf *S, const double *y);

/* Static-link (palm) placement, Sec. 5.1: with probability prob, pose g is
 * replaced by one that puts object point i onto a palm contact vector (x, nu)
 * with normals opposed and a random roll about the contact normal (the
 * alignment of orc_place_exhaustive), and is kept only if no palm capsule
 * penetrates the object by more than margin: axis samples one per mm, ends
 * included (at least 2), depth = max (r - SDF(R^T (x - t))).  Philox blocks
 * (g, b, PURPOSE_PALM, request_id), b = 0, 1, key = seed: u01(w0) < prob
 * selects the pose, w1 the palm sample, w2 the object point, w3 the roll
 * psi = 2 pi u01(w3).  palm_pt[g] = i (accepted), -1 (pose left unchanged),
 * -2 (rejected; its palm pose is still written); sel_pt[g] (optional) = i
 * for a selected pose, else -1.  flag bits: 1 = the rotation's cosine in its
 * branch band, 2 = a penetration within BAND_VAL of margin.  The selection
 * u01(w0) < prob is exact in float32 and double alike (u01 has 24 bits and
 * prob arrives as float32), so it carries no band.  flip = 1 takes the other
 * rotation branch on the poses of flag bit 1. */
int orc_place_palm(const orc_sdf *S, const float *palm_surf, int32_t n_surf, const float *palm_caps, int32_t n_caps,
                   const float *pts, const float *nrm, int32_t n_points, int32_t n_poses, double prob, double margin,
                   uint64_t seed, uint32_t request_id, int64_t pose_offset, double *poses /*[P][12] in/out*/,
                   int32_t *palm_pt, uint8_t *flag, int32_t *sel_pt, int32_t flip)
{
    if (n_points <= 0 || n_poses < 0 || n_surf <= 0 || n_caps < 0 || !(prob >= 0.0)) return ORC_EINVAL;
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
#pragma omp parallel for schedule(static)
    for (int g = 0; g < n_poses; ++g) {
        uint32_t w[8];
        for (int b = 0; b < 2; ++b) {
            uint32_t ctr[4] = {(uint32_t)(pose_offset + g), (uint32_t)b, PURPOSE_PALM, request_id};
            orc_philox4x32_10(ctr, key, w + 4 * b);
        }
        int fl = 0;
        if (sel_pt) sel_pt[g] = -1;
        if (!(u01(w[0]) < prob)) {
            palm_pt[g] = -1;
            if (flag) flag[g] = (uint8_t)fl;
            continue;
        }
        const int js = (int)(((uint64_t)w[1] * (uint64_t)n_surf) >> 32);
        const int64_t i = (int64_t)(((uint64_t)w[2] * (uint64_t)n_points) >> 32);
        const double psi = 2.0 * M_PI * u01(w[3]);
        const float *sf = palm_surf + 6 * (int64_t)js;
        const double x[3] = {sf[0], sf[1], sf[2]};
        double b[3] = {-sf[3], -sf[4], -sf[5]};
        const double nb = sqrt(dot3(b, b));
        for (int c = 0; c < 3; ++c) b[c] /= nb;
        const double a[3] = {nrm[3 * i], nrm[3 * i + 1], nrm[3 * i + 2]};
        double R0[9], Rr[9], R[9];
        int rf = 0;
        rot_align_pick(a, b, R0, &rf, flip);
        fl |= rf ? 1 : 0;
        if (sel_pt) sel_pt[g] = (int32_t)i;
        const double cs = cos(psi), sn = sin(psi);
        const double K[9] = {0, -b[2], b[1], b[2], 0, -b[0], -b[1], b[0], 0};
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c)
                Rr[3 * r + c] = (r == c ? cs : 0.0) + sn * K[3 * r + c] + (1.0 - cs) * b[r] * b[c];
        mat3_mul(Rr, R0, R);
        const double p[3] = {pts[3 * i], pts[3 * i + 1], pts[3 * i + 2]};
        double *P = poses + 12 * (int64_t)g;
        double t[3];
        for (int r = 0; r < 3; ++r) {
            t[r] = x[r] - (R[3 * r] * p[0] + R[3 * r + 1] * p[1] + R[3 * r + 2] * p[2]);
            P[4 * r + 0] = R[3 * r];
            P[4 * r + 1] = R[3 * r + 1];
            P[4 * r + 2] = R[3 * r + 2];
            P[4 * r + 3] = t[r];
        }
        /* the palm's capsules against the placed object */
        double depth = -INFINITY;
        for (int c = 0; c < n_caps; ++c) {
            const float *cp = palm_caps + 7 * (int64_t)c;
            const double A[3] = {cp[0], cp[1], cp[2]}, Bq[3] = {cp[3], cp[4], cp[5]};
            const double L = sqrt((Bq[0] - A[0]) * (Bq[0] - A[0]) + (Bq[1] - A[1]) * (Bq[1] - A[1]) +
                                  (Bq[2] - A[2]) * (Bq[2] - A[2]));
            int M = (int)ceil(L / 1e-3) + 1;
            if (M < 2) M = 2;
            for (int s = 0; s < M; ++s) {
                const double u = (double)s / (double)(M - 1);
                double d[3], y[3];
                for (int e = 0; e < 3; ++e) d[e] = A[e] + u * (Bq[e] - A[e]) - t[e];
                for (int e = 0; e < 3; ++e) y[e] = R[e] * d[0] + R[3 + e] * d[1] + R[6 + e] * d[2];
                const double v = (double)cp[6] - orc_sdf_eval(S, y);
                if (v > depth) depth = v;
            }
        }
        fl |= fabs(depth - margin) <= BAND_VAL ? 2 : 0;
        palm_pt[g] = depth <= margin ? (int32_t)i : -2;
        if (flag) flag[g] = (uint8_t)fl;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Blockwise zeroth-order contact-point optimisation (Sec. 5.4, Alg. 2).       */
/* A drawn set (Alg. 2's random start) is refined in n_outer rounds; in each   */
/* round every contact i in turn gets n_inner candidates: its point moved in   */
/* the tangent plane of its object normal (Duff basis x_i, y_i) by            */
/* (dx, dy) ~ N(0, sigma^2) each, then projected onto its contact domain D_i  */
/* (the nearest domain point, lowest index on ties).  Each candidate set      */
/* (contact i replaced, the others fixed) is scored by the criterion J = t*   */
/* (the LP above) and contact i moves to the best candidate: the first whose  */
/* J is within OPT_TAU of the minimum over the candidates.                     */
/* Noise of candidate j of step s = (round * k + i) * n_inner + j: Philox     */
/* block (g, d, PURPOSE_OPT | s << 8, request_id), key = seed; Box-Muller of  */
/* u1 = ((w0 >> 8) + 1) / 2^24 and u2 = (w1 >> 8) / 2^24.                     */
/* oflag marks sets with a decision inside a band: a runner-up domain point   */
/* within OPT_BAND of the nearest, or a candidate J within 1e-10 of the tie  */
/* threshold.  tstar receives J of the final set (its verdict: J <= eps).     */
/* ------------------------------------------------------------------------ */
static void opt_noise(uint64_t seed, uint32_t request_id, int64_t g, int d, uint32_t step, double sigma,
                      double *dx, double *dy)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {(uint32_t)g, (uint32_t)d, PURPOSE_OPT | (step << 8), request_id};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    double u1 = ((double)(w[0] >> 8) + 1.0) * (1.0 / 16777216.0);
    double u2 = (double)(w[1] >> 8) * (1.0 / 16777216.0);
    double r = sqrt(-2.0 * log(u1));
    *dx = sigma * r * cos(2.0 * M_PI * u2);
    *dy = sigma * r * sin(2.0 * M_PI * u2);
}

void orc_opt_noise(uint64_t seed, uint32_t request_id, int64_t g, int d, uint32_t step, double sigma,
                   double *dxdy)
{
    opt_noise(seed, request_id, g, d, step, sigma, dxdy, dxdy + 1);
}

/* nearest point of the domain (bitset over the N points) to y */
int64_t orc_project_domain(const float *pts, int32_t n_points, const uint32_t *dom, const double *y, int *flag)
{
    const int64_t NW = (n_points + 31) / 32;
    int64_t best = -1;
    double bd = INFINITY, second = INFINITY;
    for (int64_t w = 0; w < NW; ++w) {
        for (int b = 0; b < 32; ++b) {
            if (!((dom[w] >> b) & 1u)) continue;
            int64_t i = w * 32 + b;
            if (i >= n_points) break;
            double dd = 0.0;
            for (int a = 0; a < 3; ++a) {
                double e = (double)pts[3 * i + a] - y[a];
                dd += e * e;
            }
            double dist = sqrt(dd);
            if (dist < bd) {
                second = bd;
                bd = dist;
                best = i;
            } else if (dist < second) {
                second = dist;
            }
        }
    }
    if (flag) *flag = (second - bd) <= OPT_BAND;
    return best;
}

int orc_optimize(const float *pts, const float *nrm, int32_t n_points, const uint32_t *dom_bits /*[P][F][NW]*/,
                 const uint32_t *dom_count /*[P][F]*/, const int32_t *palm_pt /*[P] or NULL*/,
                 int32_t n_poses, int32_t F, int32_t draws, int32_t k, int32_t *set_pt /*[P][D][k] in/out*/,
                 double mu, int32_t m_edges, double rho, int32_t n_outer, int32_t n_inner, double sigma,
                 uint64_t seed, uint32_t request_id, int64_t pose_offset, int32_t max_pivots,
                 double *tstar /*[P][D]*/, uint8_t *oflag /*[P][D]*/)
{
    const int64_t NW = (n_points + 31) / 32;
    if (k <= 0 || k > 8 || k > F || n_outer < 0 || n_inner < 1 || n_inner > 64 || !(sigma >= 0.0))
        return ORC_EINVAL;
    /* a palm contact (Sec. 5.1 static link) is one more, fixed, contact of every set of its pose */
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t s = 0; s < (int64_t)n_poses * draws; ++s) {
        const int64_t g = s / draws;
        const int d = (int)(s % draws);
        int32_t *sp = set_pt + s * k;
        int valid = 1;
        for (int i = 0; i < k; ++i) valid &= sp[i] >= 0;
        int32_t fing[8];
        if (valid && k <= 8)
            valid = orc_choose_fingers(F, dom_count + g * F, k, seed, request_id, pose_offset + g, d, fing);
        if (!valid) {
            tstar[s] = NAN;
            oflag[s] = 0;
            continue;
        }
        const int kc = k + ((palm_pt && palm_pt[g] >= 0) ? 1 : 0);
        double p[3 * 16], n[3 * 16];
        for (int i = 0; i < kc; ++i) {
            const int64_t idx = i < k ? sp[i] : palm_pt[g];
            for (int a = 0; a < 3; ++a) {
                p[3 * i + a] = pts[3 * idx + a];
                n[3 * i + a] = nrm[3 * idx + a];
            }
        }
        int st, pv, fl = 0;
        double J = orc_set_tstar(kc, p, n, mu, m_edges, rho, max_pivots, &st, &pv);
        if (st != 0) J = INFINITY;
        for (int r = 0; r < n_outer; ++r) {
            for (int i = 0; i < k; ++i) {
                double tx[3], ty[3];
                duff_basis(n + 3 * i, tx, ty);
                double Jc[64] = {0};
                int64_t idx[64];
                const uint32_t *dom = dom_bits + (g * F + fing[i]) * NW;
                for (int j = 0; j < n_inner; ++j) {
                    double dx, dy, y[3];
                    opt_noise(seed, request_id, pose_offset + g, d, (uint32_t)((r * k + i) * n_inner + j), sigma,
                              &dx, &dy);
                    for (int a = 0; a < 3; ++a) y[a] = p[3 * i + a] + dx * tx[a] + dy * ty[a];
                    int pf = 0;
                    idx[j] = orc_project_domain(pts, n_points, dom, y, &pf);
                    fl |= pf;
                    double pc[3 * 16], nc[3 * 16];
                    memcpy(pc, p, sizeof(double) * 3 * kc);
                    memcpy(nc, n, sizeof(double) * 3 * kc);
                    for (int a = 0; a < 3; ++a) {
                        pc[3 * i + a] = pts[3 * idx[j] + a];
                        nc[3 * i + a] = nrm[3 * idx[j] + a];
                    }
                    Jc[j] = orc_set_tstar(kc, pc, nc, mu, m_edges, rho, max_pivots, &st, &pv);
                    if (st != 0) Jc[j] = INFINITY;
                }
                double mn = INFINITY;
                for (int j = 0; j < n_inner; ++j) mn = fmin(mn, Jc[j]);
                int js = 0;
                for (int j = 0; j < n_inner; ++j)
                    if (Jc[j] <= mn + OPT_TAU) { js = j; break; }
                for (int j = 0; j < n_inner; ++j)
                    if (isfinite(mn) && fabs(Jc[j] - (mn + OPT_TAU)) <= 1e-10) fl = 1;
                sp[i] = (int32_t)idx[js];
                for (int a = 0; a < 3; ++a) {
                    p[3 * i + a] = pts[3 * idx[js] + a];
                    n[3 * i + a] = nrm[3 * idx[js] + a];
                }
                J = Jc[js];
            }
        }
        tstar[s] = J;
        oflag[s] = (uint8_t)fl;
    }
    return ORC_OK;
}

/* Every outcome of Alg. 2 on one set that the rounding bands admit.  Where   */
/* orc_optimize takes a decision inside a band (a runner-up domain point      */
/* within OPT_BAND of the nearest, or a candidate whose J lies within 1e-10   */
/* of the tie threshold min + OPT_TAU), an implementation in other precision  */
/* may take the other side; this walks every such side: each admissible      */
/* projection of each candidate, and each candidate that can be the first     */
/* within the threshold.  The outcomes (final points and J) are collected,    */
/* duplicates removed.  orc_optimize's own result is one of them; for a set   */
/* it does not flag it is the only one.                                       */
typedef struct {
    const float *pts, *nrm;
    int32_t n_points;
    const uint32_t *dom_bits;
    const int32_t *fing;
    int64_t g, gpose;
    int d, k, kc, n_outer, n_inner, m_edges, max_pivots;
    double mu, rho, sigma;
    uint64_t seed;
    uint32_t request_id;
    int max_out, n_out, overflow;
    int32_t *out_pt;
    double *out_t;
} opt_walk;

/* admissible projections of y onto the domain: the nearest point and every
 * other within OPT_BAND of its distance, nearest first; returns the count */
static int project_admissible(const float *pts, int32_t n_points, const uint32_t *dom, const double *y,
                              int64_t *idx, int max_idx)
{
    const int64_t NW = (n_points + 31) / 32;
    double bd = INFINITY;
    int64_t best = -1;
    for (int64_t w = 0; w < NW; ++w)
        for (int b = 0; b < 32; ++b) {
            if (!((dom[w] >> b) & 1u)) continue;
            const int64_t i = w * 32 + b;
            if (i >= n_points) break;
            double dd = 0.0;
            for (int a = 0; a < 3; ++a) dd += ((double)pts[3 * i + a] - y[a]) * ((double)pts[3 * i + a] - y[a]);
            if (sqrt(dd) < bd) { bd = sqrt(dd); best = i; }
        }
    if (best < 0) return 0;
    int n = 0;
    idx[n++] = best;
    for (int64_t w = 0; w < NW; ++w)
        for (int b = 0; b < 32; ++b) {
            if (!((dom[w] >> b) & 1u)) continue;
            const int64_t i = w * 32 + b;
            if (i >= n_points) break;
            if (i == best) continue;
            double dd = 0.0;
            for (int a = 0; a < 3; ++a) dd += ((double)pts[3 * i + a] - y[a]) * ((double)pts[3 * i + a] - y[a]);
            if (sqrt(dd) - bd <= OPT_BAND && n < max_idx) idx[n++] = i;
        }
    return n;
}

static void opt_walk_step(opt_walk *W, int r, int i, int32_t *sp, double *p, double *n, double J)
{
    if (W->overflow) return;
    if (r == W->n_outer) {
        for (int o = 0; o < W->n_out; ++o) {
            int same = 1;
            for (int c = 0; c < W->k; ++c) same &= W->out_pt[o * W->k + c] == sp[c];
            if (same && W->out_t[o] == J) return;
        }
        if (W->n_out == W->max_out) { W->overflow = 1; return; }
        memcpy(W->out_pt + W->n_out * W->k, sp, sizeof(int32_t) * W->k);
        W->out_t[W->n_out++] = J;
        return;
    }
    const int nr = i + 1 == W->k ? r + 1 : r, ni = i + 1 == W->k ? 0 : i + 1;
    const int64_t NW = (W->n_points + 31) / 32;
    const uint32_t *dom = W->dom_bits + (int64_t)W->fing[i] * NW; /* dom_bits starts at pose g */
    double tx[3], ty[3];
    duff_basis(n + 3 * i, tx, ty);
    /* candidates with their admissible projections and criterion values */
    enum { MAXALT = 4 };
    int64_t alt[64][MAXALT];
    double Jalt[64][MAXALT];
    int nalt[64];
    for (int j = 0; j < W->n_inner; ++j) {
        double dx, dy, y[3];
        opt_noise(W->seed, W->request_id, W->gpose, W->d, (uint32_t)((r * W->k + i) * W->n_inner + j), W->sigma,
                  &dx, &dy);
        for (int a = 0; a < 3; ++a) y[a] = p[3 * i + a] + dx * tx[a] + dy * ty[a];
        nalt[j] = project_admissible(W->pts, W->n_points, dom, y, alt[j], MAXALT);
        if (nalt[j] == 0) { W->overflow = 1; return; } /* an empty domain: not a valid set */
        for (int v = 0; v < nalt[j]; ++v) {
            double pc[3 * 16], nc[3 * 16];
            memcpy(pc, p, sizeof(double) * 3 * W->kc);
            memcpy(nc, n, sizeof(double) * 3 * W->kc);
            for (int a = 0; a < 3; ++a) {
                pc[3 * i + a] = W->pts[3 * alt[j][v] + a];
                nc[3 * i + a] = W->nrm[3 * alt[j][v] + a];
            }
            int st, pv;
            Jalt[j][v] = orc_set_tstar(W->kc, pc, nc, W->mu, W->m_edges, W->rho, W->max_pivots, &st, &pv);
            if (st != 0) Jalt[j][v] = INFINITY;
        }
    }
    /* every combination of projections (an odometer over the candidates) */
    int pick[64] = {0};
    for (;;) {
        double mn = INFINITY;
        for (int j = 0; j < W->n_inner; ++j) mn = fmin(mn, Jalt[j][pick[j]]);
        const double thr = mn + OPT_TAU;
        for (int j = 0; j < W->n_inner; ++j) {
            const double v = Jalt[j][pick[j]];
            /* j may be chosen if it can fall within the threshold and every earlier
             * candidate can fall outside it */
            if (!(v <= thr || (isfinite(mn) && fabs(v - thr) <= 1e-10))) continue;
            const int64_t q = alt[j][pick[j]];
            int32_t sp2[16];
            double p2[3 * 16], n2[3 * 16];
            memcpy(sp2, sp, sizeof(int32_t) * W->k);
            memcpy(p2, p, sizeof(double) * 3 * W->kc);
            memcpy(n2, n, sizeof(double) * 3 * W->kc);
            sp2[i] = (int32_t)q;
            for (int a = 0; a < 3; ++a) {
                p2[3 * i + a] = W->pts[3 * q + a];
                n2[3 * i + a] = W->nrm[3 * q + a];
            }
            opt_walk_step(W, nr, ni, sp2, p2, n2, v);
            if (!(v > thr || (isfinite(mn) && fabs(v - thr) <= 1e-10))) break; /* j is surely within: no later pick */
        }
        int j = 0;
        while (j < W->n_inner && ++pick[j] == nalt[j]) pick[j++] = 0;
        if (j == W->n_inner) break;
    }
    (void)J;
}

/* Outcomes of Alg. 2 for set (g, d) started from set_pt0 [k] (the draw).  */
/* Returns the number of outcomes written to out_pt [max_out][k] and out_t  */
/* [max_out], 0 for a set that is not valid, -1 when more than max_out.     */
int orc_optimize_outcomes(const float *pts, const float *nrm, int32_t n_points, const uint32_t *dom_bits,
                          const uint32_t *dom_count, const int32_t *palm_pt, int32_t F, int32_t k, int64_t g,
                          int32_t d, const int32_t *set_pt0, double mu, int32_t m_edges, double rho, int32_t n_outer,
                          int32_t n_inner, double sigma, uint64_t seed, uint32_t request_id, int64_t pose_offset,
                          int32_t max_pivots, int32_t max_out, int32_t *out_pt, double *out_t)
{
    const int64_t NW = (n_points + 31) / 32;
    if (k <= 0 || k > 8 || k > F || n_outer < 0 || n_inner < 1 || n_inner > 64 || !(sigma >= 0.0) || max_out < 1)
        return -2;
    int valid = 1;
    for (int i = 0; i < k; ++i) valid &= set_pt0[i] >= 0;
    int32_t fing[8];
    if (valid) valid = orc_choose_fingers(F, dom_count + g * F, k, seed, request_id, pose_offset + g, d, fing);
    if (!valid) return 0;
    opt_walk W = {pts, nrm, n_points, dom_bits + g * F * NW, fing, g, pose_offset + g, d, k,
                  k + ((palm_pt && palm_pt[g] >= 0) ? 1 : 0), n_outer, n_inner, m_edges, max_pivots, mu, rho, sigma,
                  seed, request_id, max_out, 0, 0, out_pt, out_t};
    double p[3 * 16], n[3 * 16];
    int32_t sp[16];
    for (int i = 0; i < W.kc; ++i) {
        const int64_t idx = i < k ? set_pt0[i] : palm_pt[g];
        if (i < k) sp[i] = set_pt0[i];
        for (int a = 0; a < 3; ++a) {
            p[3 * i + a] = pts[3 * idx + a];
            n[3 * i + a] = nrm[3 * idx + a];
        }
    }
    int st, pv;
    double J = orc_set_tstar(W.kc, p, n, mu, m_edges, rho, max_pivots, &st, &pv);
    if (st != 0) J = INFINITY;
    if (n_outer == 0) {
        out_t[0] = J;
        memcpy(out_pt, sp, sizeof(int32_t) * k);
        return 1;
    }
    opt_walk_step(&W, 0, 0, sp, p, n, J);
    return W.overflow ? -1 : W.n_out;
}

/* Link of every contact of every valid set, picked as in orc_draw with the  */
/* set's draw words (for sets whose points the optimisation moved).           */
int orc_relink(const orc_hand *H, const orc_field_params *fp, const uint32_t *bits, const float *pts,
               const float *nrm, const float *poses, int32_t n_poses, int32_t draws, int32_t k,
               const uint32_t *dom_count /*[P][F]*/, const int32_t *set_pt, uint64_t seed, uint32_t request_id,
               int64_t pose_offset, int32_t *set_link, uint8_t *link_flag /*[P][D][k] or NULL*/)
{
    const int F = H->n_fingers;
    if (k < 1 || k > F || k > 8 || draws <= 0) return ORC_EINVAL;
    double cb[3 * 64];
    orc_bin_centers(fp->bins, cb);
#pragma omp parallel for schedule(dynamic, 4)
    for (int g = 0; g < n_poses; ++g) {
        for (int d = 0; d < draws; ++d) {
            uint32_t w[16];
            draw_words(seed, request_id, pose_offset + g, d, 2 * k, w);
            const int32_t *sp = set_pt + ((int64_t)g * draws + d) * k;
            int32_t *sl = set_link + ((int64_t)g * draws + d) * k;
            int32_t fing[8];
            const int ok = orc_choose_fingers(F, dom_count + (int64_t)g * F, k, seed, request_id, pose_offset + g,
                                              d, fing);
            uint8_t *lf = link_flag ? link_flag + ((int64_t)g * draws + d) * k : NULL;
            for (int i = 0; i < k; ++i) {
                int fl = 0;
                sl[i] = (!ok || sp[i] < 0) ? -1
                                           : pick_link(H, fp, bits, cb, pts, nrm, poses + 12 * (int64_t)g, fing[i],
                                                       sp[i], w[k + i], lf ? &fl : NULL);
                if (lf) lf[i] = (uint8_t)fl;
            }
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Kinematics optimisation (Sec. 5.5, Eq. 7-8, Phase I and Phase II).          */
/* Contact i (object point p_i, contact-surface normal n_i = -R n_obj) is     */
/* realised by link l_i of finger i.  The hand contact point (p~, n~) is the  */
/* capsule surface point closest to (p, n) in the combined metric             */
/*   |x - p|^2 + beta^2 |n~ - n|^2                                            */
/* (the closest aligned contact vector of the reverse lookup, taken on the    */
/* analytic capsule surface).  Phase I keeps the point chosen at q0 fixed to  */
/* the link; Phase II re-selects it on the current link every iteration.      */
/* Each iteration: forward kinematics; residuals of the two matched points    */
/* p~ -> p and p~ + beta n~ -> p + beta n; point Jacobians z_j x (x - o_j) of */
/* the joints on the chain up to l_i (Eq. 8 written in the base frame); the   */
/* damped least-squares step dq = (J^T J + lambda I)^-1 J^T e (Eq. 7); clamp  */
/* to the joint limits.  Final contact error and angle use the plain          */
/* projection of p onto the capsule (nearest surface point and its normal).   */
/* ------------------------------------------------------------------------ */
static void capsule_world(const orc_hand *H, const double *T, int l, double *A, double *Bp, double *r)
{
    const float *c = H->capsule + 7 * l;
    double a[3] = {c[0], c[1], c[2]}, b[3] = {c[3], c[4], c[5]};
    tf_point(T + 12 * l, a, A);
    tf_point(T + 12 * l, b, Bp);
    *r = c[6];
}

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void normalize_or(double *v, const double *axis)
{
    double nv = sqrt(dot3(v, v));
    if (nv > 1e-300) {
        for (int a = 0; a < 3; ++a) v[a] /= nv;
    } else {
        double y[3];
        duff_basis(axis, v, y); /* any direction perpendicular to the axis */
    }
}

/* plain projection of p onto the capsule surface: point pt, outward normal nt */
static void capsule_project(const double *A, const double *Bp, double r, const double *p,
                            double *pt, double *nt)
{
    double ab[3] = {Bp[0] - A[0], Bp[1] - A[1], Bp[2] - A[2]};
    double ap[3] = {p[0] - A[0], p[1] - A[1], p[2] - A[2]};
    double L2 = dot3(ab, ab);
    double t = L2 > 0 ? dot3(ap, ab) / L2 : 0.0;
    if (t < 0) t = 0;
    if (t > 1) t = 1;
    double c[3] = {A[0] + t * ab[0], A[1] + t * ab[1], A[2] + t * ab[2]};
    double ax[3] = {0, 0, 1};
    if (L2 > 0) for (int a = 0; a < 3; ++a) ax[a] = ab[a] / sqrt(L2);
    for (int a = 0; a < 3; ++a) nt[a] = p[a] - c[a];
    normalize_or(nt, ax);
    for (int a = 0; a < 3; ++a) pt[a] = c[a] + r * nt[a];
}

/* capsule surface point minimising |x - p|^2 + beta^2 |nt - n|^2.
 * Cylinder: axis point c = clamped projection of p; nt = unit part of
 * r (p - c) + beta^2 n perpendicular to the axis.  Caps (centres A, B):
 * nt = unit r (p - centre) + beta^2 n when it points into the cap's half
 * space.  The candidate of least cost wins (cylinder, then end cap, then
 * start cap on exact ties).
 * gap (optional): how close the choice is to a tie between two candidates
 * that are far apart: sqrt(runner-up cost) - sqrt(best cost) in metres, or
 * +inf when no other candidate lies more than BAND_POS away from the chosen
 * one in the same metric (a flip between two candidates that nearly coincide
 * moves the point by less than that).                                      */
static void capsule_aligned_point(const double *A, const double *Bp, double r, const double *p,
                                  const double *n, double beta, double *pt, double *nt, double *gap)
{
    double ab[3] = {Bp[0] - A[0], Bp[1] - A[1], Bp[2] - A[2]};
    double L = sqrt(dot3(ab, ab));
    double ax[3] = {0, 0, 1};
    if (L > 0) for (int a = 0; a < 3; ++a) ax[a] = ab[a] / L;
    double b2 = beta * beta;
    double cx[3][3], cv[3][3], cc[3];
    int ok[3] = {1, 0, 0};
    /* cylinder */
    {
        double ap[3] = {p[0] - A[0], p[1] - A[1], p[2] - A[2]};
        double s = dot3(ap, ax);
        if (s < 0) s = 0;
        if (s > L) s = L;
        double c[3], v[3];
        for (int a = 0; a < 3; ++a) c[a] = A[a] + s * ax[a];
        for (int a = 0; a < 3; ++a) v[a] = r * (p[a] - c[a]) + b2 * n[a];
        double va = dot3(v, ax);
        for (int a = 0; a < 3; ++a) v[a] -= va * ax[a];
        normalize_or(v, ax);
        cc[0] = 0;
        for (int a = 0; a < 3; ++a) {
            cx[0][a] = c[a] + r * v[a];
            cv[0][a] = v[a];
            cc[0] += (cx[0][a] - p[a]) * (cx[0][a] - p[a]) + b2 * (v[a] - n[a]) * (v[a] - n[a]);
        }
    }
    /* end cap (centre B, half space ax . nt >= 0), then start cap (centre A) */
    for (int cap = 0; cap < 2; ++cap) {
        const double *c = cap == 0 ? Bp : A;
        double sg = cap == 0 ? 1.0 : -1.0;
        double v[3];
        for (int a = 0; a < 3; ++a) v[a] = r * (p[a] - c[a]) + b2 * n[a];
        double nv = sqrt(dot3(v, v));
        if (!(nv > 1e-300)) continue;
        for (int a = 0; a < 3; ++a) v[a] /= nv;
        if (sg * dot3(v, ax) < 0) continue;
        ok[1 + cap] = 1;
        cc[1 + cap] = 0;
        for (int a = 0; a < 3; ++a) {
            cx[1 + cap][a] = c[a] + r * v[a];
            cv[1 + cap][a] = v[a];
            cc[1 + cap] += (cx[1 + cap][a] - p[a]) * (cx[1 + cap][a] - p[a]) + b2 * (v[a] - n[a]) * (v[a] - n[a]);
        }
    }
    int w = 0;
    for (int i = 1; i < 3; ++i)
        if (ok[i] && cc[i] < cc[w]) w = i;
    memcpy(pt, cx[w], sizeof cx[w]);
    memcpy(nt, cv[w], sizeof cv[w]);
    if (gap) {
        double g = INFINITY;
        for (int i = 0; i < 3; ++i) {
            if (i == w || !ok[i]) continue;
            double sep = 0;
            for (int a = 0; a < 3; ++a)
                sep += (cx[i][a] - cx[w][a]) * (cx[i][a] - cx[w][a]) + b2 * (cv[i][a] - cv[w][a]) * (cv[i][a] - cv[w][a]);
            if (sqrt(sep) > BAND_POS) g = fmin(g, sqrt(cc[i]) - sqrt(cc[w]));
        }
        *gap = g;
    }
}

/* exported for the tests: the capsule point of least |x - p|^2 + beta^2 |nt - n|^2 */
void orc_capsule_aligned_point(const double *A, const double *Bp, double r, const double *p, const double *n,
                               double beta, double *pt, double *nt, double *gap)
{
    capsule_aligned_point(A, Bp, r, p, n, beta, pt, nt, gap);
}

/* Position Jacobian (3 x d_f, row-major) of a point x fixed to link `link`
 * of finger f (Eq. 8 in the base frame): column t is z_j x (x - o_j) for the
 * finger's joint j = first + t on the chain up to `link`, else zero.  T holds
 * the finger's link frames.                                                  */
void orc_point_jacobian(const orc_hand *H, int f, int link, const double *T, const double *x,
                        double *Jm)
{
    const int j0 = finger_first_joint(H, f), d = finger_dof(H, f);
    for (int i = 0; i < 3 * d; ++i) Jm[i] = 0.0;
    for (int t = 0; t < d; ++t) {
        int j = j0 + t;
        if (j > link) break;
        const double *Tj = T + 12 * j;
        double o[3] = {Tj[3], Tj[7], Tj[11]};
        double al[3] = {H->joint_axis[3 * j], H->joint_axis[3 * j + 1], H->joint_axis[3 * j + 2]};
        double z[3];
        tf_dir(Tj, al, z);
        double v[3] = {x[0] - o[0], x[1] - o[1], x[2] - o[2]};
        Jm[0 * d + t] = z[1] * v[2] - z[2] * v[1];
        Jm[1 * d + t] = z[2] * v[0] - z[0] * v[2];
        Jm[2 * d + t] = z[0] * v[1] - z[1] * v[0];
    }
}

static int cholesky_solve(int n, double *A, double *b)
{
    for (int j = 0; j < n; ++j) {
        double s = A[j * n + j];
        for (int k = 0; k < j; ++k) s -= A[j * n + k] * A[j * n + k];
        if (s <= 0) return -1;
        double d = sqrt(s);
        A[j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double t = A[i * n + j];
            for (int k = 0; k < j; ++k) t -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = t / d;
        }
    }
    for (int i = 0; i < n; ++i) {
        double t = b[i];
        for (int k = 0; k < i; ++k) t -= A[i * n + k] * b[k];
        b[i] = t / A[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double t = b[i];
        for (int k = i + 1; k < n; ++k) t -= A[k * n + i] * b[k];
        b[i] = t / A[i * n + i];
    }
    return 0;
}

typedef struct {
    int32_t iters;     /* total DLS iterations */
    int32_t phase1;    /* leading iterations with the contact point fixed to the link */
    double lambda;
    double beta;
    double tol_pos;
    double tol_ang;
    double margin;
    int32_t self_collision; /* also require no hand self-penetration deeper than margin */
} orc_ik_params;

/* One finger's IK towards one contact.  q_f in/out (finger joints).       */
void orc_ik_finger(const orc_hand *H, int f, int link, const double *p, const double *n,
                   const orc_ik_params *ik, double *q_f, double *err, double *ang,
                   double *pt_out, double *nt_out, double *sel_gap)
{
    const int J = H->n_joints, j0 = finger_first_joint(H, f), d = finger_dof(H, f);
    double *T = (double *)malloc(sizeof(double) * 12 * J);
    double pt[3], nt[3], loc_p[3] = {0, 0, 0}, loc_n[3] = {0, 0, 1};
    double min_gap = INFINITY; /* closest tie of the contact-point choices made */
    for (int it = 0; it < ik->iters; ++it) {
        orc_fk_finger(H, f, q_f, T);
        const double *Tl = T + 12 * link;
        double A[3], Bp[3], r;
        capsule_world(H, T, link, A, Bp, &r);
        if (it >= ik->phase1 || it == 0) {
            double gap;
            capsule_aligned_point(A, Bp, r, p, n, ik->beta, pt, nt, &gap);
            if (gap < min_gap) min_gap = gap;
            /* link-frame copy: R^T (x - t), R^T n */
            double dx[3] = {pt[0] - Tl[3], pt[1] - Tl[7], pt[2] - Tl[11]};
            for (int a = 0; a < 3; ++a) {
                loc_p[a] = Tl[a] * dx[0] + Tl[4 + a] * dx[1] + Tl[8 + a] * dx[2];
                loc_n[a] = Tl[a] * nt[0] + Tl[4 + a] * nt[1] + Tl[8 + a] * nt[2];
            }
        } else {
            tf_point(Tl, loc_p, pt);
            tf_dir(Tl, loc_n, nt);
        }
        double x2[3], e[6];
        for (int a = 0; a < 3; ++a) {
            x2[a] = pt[a] + ik->beta * nt[a];
            e[a] = p[a] - pt[a];
            e[3 + a] = (p[a] + ik->beta * n[a]) - x2[a];
        }
        double Jm[6 * 16];
        orc_point_jacobian(H, f, link, T, pt, Jm);
        orc_point_jacobian(H, f, link, T, x2, Jm + 3 * d);
        double M[16 * 16], g[16];
        for (int a = 0; a < d; ++a) {
            g[a] = 0.0;
            for (int rr = 0; rr < 6; ++rr) g[a] += Jm[rr * d + a] * e[rr];
            for (int b = 0; b < d; ++b) {
                double s = 0.0;
                for (int rr = 0; rr < 6; ++rr) s += Jm[rr * d + a] * Jm[rr * d + b];
                M[a * d + b] = s + (a == b ? ik->lambda : 0.0);
            }
        }
        if (cholesky_solve(d, M, g) != 0) break;
        for (int t = 0; t < d; ++t) {
            double lo = H->limits[2 * (j0 + t)], hi = H->limits[2 * (j0 + t) + 1];
            double v = q_f[t] + g[t];
            q_f[t] = v < lo ? lo : (v > hi ? hi : v);
        }
    }
    orc_fk_finger(H, f, q_f, T);
    {
        double A[3], Bp[3], r;
        capsule_world(H, T, link, A, Bp, &r);
        capsule_project(A, Bp, r, p, pt, nt);
    }
    double dx[3] = {p[0] - pt[0], p[1] - pt[1], p[2] - pt[2]};
    *err = sqrt(dot3(dx, dx));
    double c = dot3(nt, n);
    if (c > 1) c = 1;
    if (c < -1) c = -1;
    *ang = acos(c);
    if (pt_out) memcpy(pt_out, pt, sizeof pt);
    if (nt_out) memcpy(nt_out, nt, sizeof nt);
    if (sel_gap) *sel_gap = min_gap;
    free(T);
}

/* Object SDF on a G^3 node grid (object frame), trilinear interpolation,
 * +inf outside the grid.                                                    */

double orc_sdf_eval(const orc_sdf *S, const double *y)
{
    const int G = S->dims;
    double u[3];
    int i0[3];
    for (int a = 0; a < 3; ++a) {
        u[a] = (y[a] - S->origin[a]) / S->h;
        if (!(u[a] >= 0.0 && u[a] <= (double)(G - 1))) return INFINITY;
        int i = (int)floor(u[a]);
        if (i > G - 2) i = G - 2;
        if (i < 0) i = 0;
        i0[a] = i;
        u[a] -= i;
    }
    double acc = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                double w = (dx ? u[0] : 1 - u[0]) * (dy ? u[1] : 1 - u[1]) * (dz ? u[2] : 1 - u[2]);
                int64_t idx = ((int64_t)(i0[2] + dz) * G + (i0[1] + dy)) * G + (i0[0] + dx);
                acc += w * S->values[idx];
            }
    return acc;
}

/* Object preprocessing (Sec. 5.2): penetration of a small box placed at each
 * object point.  The box is a cube of edge s whose bottom face is centred at
 * the point p, with axes (x, y, n): the Duff basis of the unit outward normal
 * n, and n itself, so the cube stands on the surface outside the object.  Its
 * penetration is the largest -SDF over the lattice p + a x + b y + c n,
 * a, b in {-s/2 + s i / m}, c in {s i / m}, i = 0..m (corners included); a
 * lattice point outside the SDF grid counts as outside the object.  The point
 * is kept iff the penetration is at most max_depth; flag marks penetrations
 * within BAND_VAL of max_depth. */
int orc_concave_filter(const orc_sdf *S, const float *pts, const float *nrm, int32_t n_points, double s, int32_t m,
                       double max_depth, double *depth, uint8_t *keep, uint8_t *flag)
{
    if (n_points < 0 || !(s > 0.0) || m < 1) return ORC_EINVAL;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n_points; ++i) {
        double p[3] = {pts[3 * i], pts[3 * i + 1], pts[3 * i + 2]};
        double n[3] = {nrm[3 * i], nrm[3 * i + 1], nrm[3 * i + 2]};
        const double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        for (int c = 0; c < 3; ++c) n[c] /= nn;
        double x[3], y[3];
        duff_basis(n, x, y);
        double worst = -INFINITY;
        for (int ia = 0; ia <= m; ++ia)
            for (int ib = 0; ib <= m; ++ib)
                for (int ic = 0; ic <= m; ++ic) {
                    const double a = -0.5 * s + s * ia / m, b = -0.5 * s + s * ib / m, c = s * ic / m;
                    double q[3];
                    for (int e = 0; e < 3; ++e) q[e] = p[e] + a * x[e] + b * y[e] + c * n[e];
                    const double d = -orc_sdf_eval(S, q);
                    if (d > worst) worst = d;
                }
        depth[i] = worst;
        keep[i] = worst <= max_depth;
        flag[i] = fabs(worst - max_depth) <= BAND_VAL;
    }
    return ORC_OK;
}

/* number of axis samples of a capsule: one per millimetre of axis, ends included */
int orc_axis_samples(const orc_hand *H, int l)
{
    const float *c = H->capsule + 7 * l;
    double dx = (double)c[3] - c[0], dy = (double)c[4] - c[1], dz = (double)c[5] - c[2];
    double L = sqrt((dx * dx + dy * dy) + dz * dz);
    return (int)ceil(L / 1e-3) + 1;
}

/* Penetration of the hand's capsules into the object (Sec. 3.2 criterion 1
 * with a margin; the capsule axis samples are tested against the object's
 * SDF): depth = max over links and axis samples of (r - SDF(x)).            */
double orc_penetration(const orc_hand *H, const double *T, const orc_sdf *S, const float *pose)
{
    double P[12];
    tf_load(pose, P);
    double depth = -INFINITY;
    for (int l = 0; l < H->n_joints; ++l) {
        double A[3], Bp[3], r;
        capsule_world(H, T, l, A, Bp, &r);
        int M = orc_axis_samples(H, l);
        for (int s = 0; s < M; ++s) {
            double t = (double)s / (double)(M - 1);
            double x[3], d[3], y[3];
            for (int a = 0; a < 3; ++a) {
                x[a] = A[a] + t * (Bp[a] - A[a]);
                d[a] = x[a] - P[4 * a + 3];
            }
            /* object frame: y = R^T (x - t) */
            for (int a = 0; a < 3; ++a) y[a] = P[a] * d[0] + P[4 + a] * d[1] + P[8 + a] * d[2];
            double v = r - orc_sdf_eval(S, y);
            if (v > depth) depth = v;
        }
    }
    return depth;
}

/* Realise accepted sets: witness seed, IK per finger, penetration, acceptance.
 * wit [L][G^3][B] may be NULL (then q0 = mid-limits).                        */
/* ------------------------------------------------------------------------ */
/* Hand self-collision (Sec. 5.6 postprocessing: hand-to-hand collisions),    */
/* for capsule links in closed form: the distance between two axis segments   */
/* is minimised over (s, t) in [0,1]^2 (Ericson, Real-Time Collision          */
/* Detection, Sec. 5.1.9); two capsules of different fingers penetrate by     */
/* r1 + r2 - dist.  Links of one finger are excluded (consecutive links meet  */
/* at their joints).                                                          */
/* ------------------------------------------------------------------------ */
double orc_segment_distance(const double *p1, const double *q1, const double *p2, const double *q2)
{
    double d1[3], d2[3], r[3];
    for (int c = 0; c < 3; ++c) {
        d1[c] = q1[c] - p1[c];
        d2[c] = q2[c] - p2[c];
        r[c] = p1[c] - p2[c];
    }
    const double a = dot3(d1, d1), e = dot3(d2, d2), f = dot3(d2, r);
    double s, t;
    if (a <= 1e-30 && e <= 1e-30) {
        s = t = 0.0;
    } else if (a <= 1e-30) {
        s = 0.0;
        t = fmin(fmax(f / e, 0.0), 1.0);
    } else {
        const double c = dot3(d1, r);
        if (e <= 1e-30) {
            t = 0.0;
            s = fmin(fmax(-c / a, 0.0), 1.0);
        } else {
            const double b = dot3(d1, d2), den = a * e - b * b;
            s = den > 0.0 ? fmin(fmax((b * f - c * e) / den, 0.0), 1.0) : 0.0;
            t = (b * s + f) / e;
            if (t < 0.0) {
                t = 0.0;
                s = fmin(fmax(-c / a, 0.0), 1.0);
            } else if (t > 1.0) {
                t = 1.0;
                s = fmin(fmax((b - c) / a, 0.0), 1.0);
            }
        }
    }
    double dd = 0.0;
    for (int c = 0; c < 3; ++c) {
        const double x = p1[c] + s * d1[c] - (p2[c] + t * d2[c]);
        dd += x * x;
    }
    return sqrt(dd);
}

/* deepest penetration between capsules of different fingers (-inf if none) */
double orc_self_penetration(const orc_hand *H, const double *T /*[J][12]*/)
{
    double worst = -INFINITY;
    for (int l1 = 0; l1 < H->n_joints; ++l1)
        for (int l2 = l1 + 1; l2 < H->n_joints; ++l2) {
            if (H->joint_finger[l1] == H->joint_finger[l2]) continue;
            double A1[3], B1[3], r1, A2[3], B2[3], r2;
            capsule_world(H, T, l1, A1, B1, &r1);
            capsule_world(H, T, l2, A2, B2, &r2);
            worst = fmax(worst, r1 + r2 - orc_segment_distance(A1, B1, A2, B2));
        }
    return worst;
}

/* Uniform joint values of an unused finger f of set (g, d) (Sec. 5.6: joints
 * not fixed by a contact take random values): joint t of the finger is
 * lo + (hi - lo) u, u = (w_t >> 8) / 2^24, w = Philox blocks (g, d,
 * PURPOSE_UNUSED | (2 f + blk) << 8, request_id), blk = 0, 1. */
void orc_unused_joints(const orc_hand *H, int f, uint64_t seed, uint32_t request_id, int64_t g, int d,
                       double *q /*[J]*/)
{
    const int j0 = finger_first_joint(H, f), dof = finger_dof(H, f);
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[8];
    for (int blk = 0; blk < 2; ++blk) {
        uint32_t ctr[4] = {(uint32_t)g, (uint32_t)d, PURPOSE_UNUSED | ((uint32_t)(2 * f + blk) << 8), request_id};
        orc_philox4x32_10(ctr, key, w + 4 * blk);
    }
    for (int t = 0; t < dof; ++t) {
        const double lo = H->limits[2 * (j0 + t)], hi = H->limits[2 * (j0 + t) + 1];
        q[j0 + t] = lo + (hi - lo) * u01(w[t]);
    }
}

/* Accepted set -> grasp.  The finger of contact i is that of its link; a set
 * is realisable iff every link is a hand link, every point an object point and
 * the fingers increase strictly with i.  Fingers carrying a contact start at
 * the witness sample and run the IK; every other finger (all of them for a set
 * that is not realisable, whose contact errors and angles are +inf) takes
 * random joint values.  The penetration covers every link of the hand. */
int orc_realize(const orc_hand *H, const orc_field_params *fp, const int32_t *wit,
                const orc_sdf *S, const float *pts, const float *nrm, int32_t n_points,
                const float *poses, int32_t n_poses,
                const int32_t *set_pt, const int32_t *set_link, int32_t k, int32_t draws,
                const int32_t *acc_list, int32_t n_acc, const orc_ik_params *ik,
                uint64_t seed, uint32_t request_id, int64_t pose_offset,
                double *q_out /*[n_acc][J]*/, double *q0_out /*[n_acc][J] opt*/,
                double *contact_err /*[n_acc][k]*/, double *contact_ang /*[n_acc][k]*/,
                double *depth, uint8_t *valid, uint8_t *rflag, double *rmargin /*[n_acc][3] opt*/)
{
    const int J = H->n_joints, F = H->n_fingers, G = fp->grid, B = fp->bins;
    const int64_t G3 = (int64_t)G * G * G;
    if (k < 1 || k > F || k > 8 || draws <= 0) return ORC_EINVAL;
    for (int a = 0; a < n_acc; ++a)
        if (acc_list[a] < 0 || acc_list[a] >= (int64_t)n_poses * draws) return ORC_EINVAL;
    double cb[3 * 64];
    orc_bin_centers(B, cb);
#pragma omp parallel for schedule(dynamic, 4)
    for (int a = 0; a < n_acc; ++a) {
        const int64_t sid = acc_list[a]; /* set id g*D + d */
        const int64_t g = sid / draws;
        const int d = (int)(sid % draws);
        const float *pose = poses + 12 * g;
        double Tp[12];
        tf_load(pose, Tp);
        double *q = q_out + (int64_t)a * J;
        double q0[64];
        int fl = 0;
        double worst_err = 0, worst_ang = 0;
        double m_face = INFINITY, m_bin = INFINITY, m_gap = INFINITY;
        /* contact of each finger (-1: none) */
        int contact_of[8];
        for (int f = 0; f < F; ++f) contact_of[f] = -1;
        int ok = 1, prev = -1;
        for (int i = 0; i < k; ++i) {
            const int l = set_link[sid * k + i], idx = set_pt[sid * k + i];
            if (l < 0 || l >= J || idx < 0 || idx >= n_points || H->joint_finger[l] <= prev) {
                ok = 0;
                break;
            }
            prev = H->joint_finger[l];
            contact_of[prev] = i;
        }
        if (!ok)
            for (int f = 0; f < F; ++f) contact_of[f] = -1;
        for (int f = 0; f < F; ++f) {
            const int i = contact_of[f];
            const int j0 = finger_first_joint(H, f), dof = finger_dof(H, f);
            if (i < 0) {
                orc_unused_joints(H, f, seed, request_id, pose_offset + g, d, q);
                for (int t = 0; t < dof; ++t) q0[j0 + t] = q[j0 + t];
                continue;
            }
            const int l = set_link[sid * k + i], idx = set_pt[sid * k + i];
            double pl[3] = {pts[3 * idx], pts[3 * idx + 1], pts[3 * idx + 2]};
            double nl[3] = {nrm[3 * idx], nrm[3 * idx + 1], nrm[3 * idx + 2]};
            double p[3], nu[3], n[3];
            tf_point(Tp, pl, p);
            tf_dir(Tp, nl, nu);
            for (int c = 0; c < 3; ++c) n[c] = -nu[c];
            /* reverse lookup: witness sample of (l, voxel(p), bin(n)) */
            int32_t w = -1;
            if (wit) {
                double u[3], half_gap;
                int in = voxel_coords(fp, f, p, u);
                int b = bin_of(B, cb, n, NULL, &half_gap);
                /* the lookup's discrete choices: a voxel face (window faces
                 * included) within BAND_POS, a bin boundary within BAND_ANG */
                for (int c = 0; c < 3; ++c) m_face = fmin(m_face, face_dist(u[c], fp->h));
                m_bin = fmin(m_bin, half_gap);
                if (in) {
                    int64_t v = ((int64_t)(int)floor(u[2]) * G + (int)floor(u[1])) * G + (int)floor(u[0]);
                    w = wit[((int64_t)l * G3 + v) * B + b];
                }
            }
            if (w >= 0) {
                orc_joint_sample(H, fp->seed, f, w, q + j0);
            } else {
                for (int t = 0; t < dof; ++t)
                    q[j0 + t] = 0.5 * ((double)H->limits[2 * (j0 + t)] + H->limits[2 * (j0 + t) + 1]);
            }
            for (int t = 0; t < dof; ++t) q0[j0 + t] = q[j0 + t];
            double err, ang, gap;
            orc_ik_finger(H, f, l, p, n, ik, q + j0, &err, &ang, NULL, NULL, &gap);
            contact_err[(int64_t)a * k + i] = err;
            contact_ang[(int64_t)a * k + i] = ang;
            m_gap = fmin(m_gap, gap);
            fl |= (fabs(err - ik->tol_pos) <= BAND_VAL || fabs(ang - ik->tol_ang) <= BAND_VAL) ? RF_THRESHOLD : 0;
            if (err > worst_err) worst_err = err;
            if (ang > worst_ang) worst_ang = ang;
        }
        if (!ok) {
            for (int i = 0; i < k; ++i) {
                contact_err[(int64_t)a * k + i] = INFINITY;
                contact_ang[(int64_t)a * k + i] = INFINITY;
            }
            worst_err = worst_ang = INFINITY;
        }
        if (q0_out) memcpy(q0_out + (int64_t)a * J, q0, sizeof(double) * J);
        double *T = (double *)malloc(sizeof(double) * 12 * J);
        orc_fk(H, q, T);
        double dp = orc_penetration(H, T, S, pose);
        if (ik->self_collision) dp = fmax(dp, orc_self_penetration(H, T));
        free(T);
        depth[a] = dp;
        fl |= fabs(dp - ik->margin) <= BAND_VAL ? RF_THRESHOLD : 0;
        fl |= (m_face < BAND_POS || m_bin < BAND_ANG) ? RF_LOOKUP : 0;
        fl |= m_gap <= BAND_CHOICE ? RF_CHOICE : 0;
        valid[a] = worst_err <= ik->tol_pos && worst_ang <= ik->tol_ang && dp <= ik->margin;
        if (rflag) rflag[a] = (uint8_t)fl;
        if (rmargin) {
            rmargin[3 * a + 0] = m_face;
            rmargin[3 * a + 1] = m_bin;
            rmargin[3 * a + 2] = m_gap;
        }
    }
    return ORC_OK;
}
