/*
 * lg.h -- C ABI of the MI355X (gfx950) Contact-Field library.
 *
 * The library implements the data-parallel hot path of Lightning Grasp
 * (Yin & Abbeel, arXiv 2511.07418): a sampled contact field of a hand
 * (Sec. 4, Alg. 1, Sec. 4.4), contact-domain queries of an object under many
 * palm poses (Sec. 4.3, Sec. 5.3), seeded contact-set draws scored by a
 * force-closure criterion (Eq. 1-2, Sec. 5.3-5.4), and the realisation of
 * accepted sets by damped-least-squares IK (Sec. 5.5, Eq. 7-8) followed by a
 * penetration check (Sec. 3.2).  The four calls follow the paper's problem
 * statement: hand in (build), object + poses in (query), sets out (search),
 * grasps (P, q) out (realize).
 *
 * Conventions for every call:
 *  - Pointers are DEVICE pointers (HIP, on the current device) unless the
 *    comment says "host".  The caller owns every buffer it passes; the
 *    library owns only the lg_field it returns from lg_build_field /
 *    lg_field_import, which stays resident in HBM until lg_field_release.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued
 *    asynchronously; arguments are validated synchronously before anything is
 *    enqueued, so an LG_EINVAL return leaves all outputs untouched.
 *  - Every call returns an lg_status; no C++ exception crosses the ABI.
 *    lg_last_error() gives a thread-local human-readable detail of the last
 *    failure.  Asynchronous device faults surface at the caller's next
 *    synchronisation of the stream.
 *  - Sizes are int32 (N, P < 2^31); counts of sets are P*D < 2^31.
 *  - Units are SI (m, rad).  Rigid transforms are 3x4 row-major [R | t]
 *    (12 floats) mapping local to parent coordinates.
 */
#ifndef LG_H
#define LG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lg_status;
#define LG_OK 0
#define LG_EINVAL (-1)       /* invalid argument (nothing enqueued) */
#define LG_ENOMEM (-2)       /* device allocation failed */
#define LG_EDEVICE (-3)      /* HIP runtime error */
#define LG_EBUDGET (-4)      /* request can never fit the server's HBM budget */
#define LG_EUNSUPPORTED (-5) /* valid but unsupported configuration */
#define LG_EINTERNAL (-6)

/* Name of a status code (static string). */
const char *lg_status_str(lg_status s);
/* Detail of the last failing call on this thread (static per-thread buffer). */
const char *lg_last_error(void);
/* Library version string. */
const char *lg_version(void);

/* ------------------------------------------------------------------------ */
/* Hand: H = (H_M, C, F) of Sec. 3.1 as a capsule-chain hand.                */
/* One link (capsule) per revolute joint.  Joints are grouped by finger; a    */
/* finger is a dependency group of Sec. 5.3 (a connected component of the     */
/* kinematic tree without static links) and must be a serial chain stored     */
/* contiguously: joint_parent[j] is -1 (hand base) for the first joint of a   */
/* finger and j-1 otherwise.  Frame of joint j:                               */
/*   T_j = T_parent * joint_origin_j * Rot(joint_axis_j, q_j).                */
/* All arrays are HOST memory and are copied by the library.                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t n_fingers;            /* F, 1..8 */
    int32_t n_joints;             /* J = number of links, <= 64, <= 8 per finger */
    const int32_t *joint_finger;  /* host [J] finger of each joint */
    const int32_t *joint_parent;  /* host [J] -1 or j-1 */
    const float *joint_origin;    /* host [J][12] parent -> joint at q = 0 */
    const float *joint_axis;      /* host [J][3] unit axis in the joint frame */
    const float *capsule;         /* host [J][7] a(3), b(3), radius, link frame */
    const float *limits;          /* host [J][2] lo, hi */
    int32_t n_surf;               /* surface samples per link (patch points) */
    const float *surf;            /* host [J][n_surf][6] link-frame point, outward normal */
    /* static link (the palm, Sec. 5.1 static-link contacts); 0 / NULL = none */
    int32_t n_palm_surf;          /* palm contact vectors */
    const float *palm_surf;       /* host [n_palm_surf][6] base-frame point, outward normal */
    int32_t n_palm_caps;          /* palm capsules (penetration test) */
    const float *palm_caps;       /* host [n_palm_caps][7] a(3), b(3), radius, base frame */
} lg_hand_desc;

/* Field construction parameters (Sec. 4.3, Alg. 1 as a dense grid cover). */
typedef struct {
    int64_t samples;          /* S joint samples per finger, 1..2^31-1 */
    uint64_t seed;            /* Philox4x32-10 key (low word, high word) */
    int32_t grid;             /* G: each finger's window has G^3 voxels, 4..128 */
    float h;                  /* voxel edge (m) */
    int32_t bins;             /* B normal bins: 32 or 64 (spherical Fibonacci lattice) */
    const float *grid_frame;  /* host [F][12] [R | o]: voxel coords u = R^T (x - o) / h */
    int32_t keep_witness;     /* 1: keep the smallest sample id per (link, voxel, bin) */
} lg_field_params;

typedef struct lg_field lg_field;

typedef struct {
    int32_t n_fingers, n_joints, grid, bins;
    int64_t samples;
    uint64_t device_bytes;    /* HBM held by the field */
    uint64_t bits_set;        /* set bits over all per-link tables */
    int64_t vectors;          /* contact vectors generated (S * sum_l n_surf) */
    int64_t dropped;          /* vectors outside their finger's window */
    int32_t has_witness;
    int32_t lattice;          /* 1: the windows share one rotation and lie whole 4-voxel bricks
                                 apart (G a power of two), so the query maps each point once for
                                 all fingers; 0: each finger's window is mapped on its own */
    double build_kernel_ms;   /* duration of the sampling + binning kernel of lg_build_field (HIP
                                 events on its stream); 0 for an imported field */
} lg_field_info_t;

/*
 * lg_build_field -- sample the contact field of a hand (Sec. 4.3-4.4).
 * For every finger f and sample s: q = lo + (hi - lo) u with u from Philox
 * block (s, 8f + t/4, 1, 0) word t%4 (t = joint index within the finger),
 * u = (word >> 8) 2^-24; forward kinematics; every surface sample (p, n) of
 * every link l of f gives a contact vector x = T_l p, nu = R_l n that sets
 * bit bin(nu) of voxel floor(R_f^T (x - o_f) / h) in link l's table (vectors
 * outside the window are dropped and counted); bin(nu) = argmax_b <nu, c_b>
 * over the Fibonacci lattice c_b = (sqrt(1-z^2) cos phi, sqrt(1-z^2) sin phi,
 * z), z = 1 - (2b+1)/B, phi = b pi (3 - sqrt 5), ties to the lowest b.
 * The call blocks until the field is built (it returns a usable handle).
 * Errors: LG_EINVAL (bad sizes, non-chain hand, B not 32/64), LG_ENOMEM.
 */
lg_status lg_build_field(const lg_hand_desc *hand, const lg_field_params *params, void *stream,
                         lg_field **out);

/* Build a field from canonical host tables instead of sampling:
 * bits_host [J][G^3][B/32] (voxel v = (iz G + iy) G + ix, bit b of word b/32 is
 * bin b), witness_host [J][G^3][B] (-1 = none) or NULL.  Used to run the
 * query/search/realize stages on an externally computed field. */
lg_status lg_field_import(const lg_hand_desc *hand, const lg_field_params *params,
                          const uint32_t *bits_host, const int32_t *witness_host,
                          lg_field **out);

/* Copy the per-link tables to host memory in the canonical layout above
 * (witness_host may be NULL; -1 marks cells without a witness).  Blocking. */
lg_status lg_field_export(const lg_field *field, uint32_t *bits_host, int32_t *witness_host);

lg_status lg_field_info(const lg_field *field, lg_field_info_t *info);

/* Free the field's device memory (NULL is a no-op). */
lg_status lg_field_release(lg_field *field);

/*
 * lg_query_domains -- contact domains of an object under P poses
 * (Sec. 4.2-4.3, Def. 4.3, Sec. 5.3).
 * pts, nrm: device [3][N] float (structure of arrays, object frame, outward
 *           unit normals).
 * poses:    device [P][12] object pose in the hand frame.
 * For pose g, point i: x = R p + t, query normal -R n (the contact surface
 * representation negates the normal); finger f's domain bit is the OR over
 * its links of the table bit at (voxel_f(x), bin(-R n)), 0 outside the window.
 * dom_bits:  device [P][F][ceil(N/32)] uint32, bit i%32 of word i/32 = point i
 *            (bits past N are zero).
 * dom_count: device [P][F] uint32, set bits per (pose, finger).
 * Errors: LG_EINVAL on null pointers or negative sizes.  N = 0 or P = 0 is a
 * valid no-op (counts are still written for P > 0).
 */
lg_status lg_query_domains(const lg_field *field, const float *pts, const float *nrm,
                           int32_t n_points, const float *poses, int32_t n_poses,
                           uint32_t *dom_bits, uint32_t *dom_count, void *stream);

/*
 * lg_query_domains_cone -- the theta_hit form of the object contact query
 * (Sec. 4.3): point i is in finger f's domain at pose g if some normal-bin
 * centre c_b set in the finger's field at voxel(R p_i + t) satisfies
 * c_b . (-R n_i) >= cos_hit (cos_hit in [-1, 1]; the paper's test over the
 * quantised normals of the leaf).  Same buffers, layout and errors as
 * lg_query_domains; the domains contain lg_query_domains' once the cone is
 * wider than the bins' covering radius.  bounds: NULL or the chunk bounds of
 * lg_chunk_bounds (below) for the same points, which skip (chunk, finger)
 * pairs out of a window's reach without changing the output.
 */
lg_status lg_query_domains_cone(const lg_field *field, const float *pts, const float *nrm, int32_t n_points,
                                const float *poses, int32_t n_poses, const float *bounds, float cos_hit,
                                uint32_t *dom_bits, uint32_t *dom_count, void *stream);

/*
 * lg_chunk_bounds -- bounding spheres of the object's chunks of 64 consecutive
 * points (a one-level bounding-volume hierarchy over the object, as the
 * paper's BVH over contact patches in Alg. 1): bounds DEVICE [ceil(N/64)][4]
 * float (centre of the chunk's box, radius padded by 1e-5 relative + 1e-7 m),
 * 16-byte aligned.  pts DEVICE SoA [3][N].  Compute once per object.
 * lg_query_domains_bounded -- lg_query_domains with those bounds: a (chunk,
 * finger) pair whose sphere (plus 1e-3 voxel) misses the finger's window is
 * skipped (its domain bits are 0, as the lookups would give), and a chunk
 * missing every window is not read.  Outputs are identical to
 * lg_query_domains'; the saving depends on spatially compact chunks, e.g.
 * points in the order of lg_morton_order.  LG_EINVAL on null or misaligned
 * bounds, plus lg_query_domains' errors.
 */
lg_status lg_chunk_bounds(const float *pts, int32_t n_points, float *bounds, void *stream);
lg_status lg_query_domains_bounded(const lg_field *field, const float *pts, const float *nrm, int32_t n_points,
                                   const float *poses, int32_t n_poses, const float *bounds, uint32_t *dom_bits,
                                   uint32_t *dom_count, void *stream);
/* lg_morton_order -- perm_host[j] = index of the j-th point in Morton order
 * (10 bits per axis over the points' bounding cube, x lowest; stable).
 * pts_host: HOST [N][3].  Reorder points and normals with it once per object
 * (e.g. lg_gather_points); domain bits then index the reordered points.
 * LG_EINVAL on null buffers or non-finite points. */
lg_status lg_morton_order(const float *pts_host, int32_t n_points, int32_t *perm_host);

/* Search parameters (Sec. 5.3 draws, Eq. 1-2 criterion). */
typedef struct {
    int32_t draws;        /* D sets per pose */
    int32_t k;            /* contacts per set, 1..F: one per finger, on k fingers drawn per set */
    int32_t m_edges;      /* linearised cone edges, 3..16 */
    int32_t max_pivots;   /* simplex pivot cap (status UNDECIDED when hit) */
    float mu;             /* friction coefficient >= 0 */
    float eps;            /* stability threshold on t* */
    float moment_scale;   /* rho > 0: moment rows are divided by rho */
    uint64_t seed;        /* Philox key */
    uint32_t request_id;  /* 4th Philox counter word */
    int64_t pose_offset;  /* global index of pose 0 (RNG counters use it) */
    int32_t opt_outer;    /* rounds of contact-point optimisation (Sec. 5.4, Alg. 2); 0 = none */
    int32_t opt_inner;    /* candidates per contact and round, 1..16 */
    float opt_sigma;      /* std of the tangent-plane mutations (m) */
    const int32_t *palm_pt; /* DEVICE [P] or NULL: static-link contacts of lg_place_palm.  >= 0: that
                               object point is one more, fixed, contact of every set of the pose (in the
                               verdict and in Alg. 2; k <= 7); -1: none; -2: rejected placement, the pose
                               draws no sets.  Not supported by the server (must be NULL there). */
} lg_search_params;

/* Bytes of device workspace lg_search asks for with n_points points and n_poses
 * poses.  With opt_outer > 0 this includes per-candidate arrays that let the
 * criteria of Alg. 2 gather their slow LPs into launches of their own; lg_search
 * also accepts a workspace without them (down to the size with opt_outer = 0
 * plus Alg. 2's cell grid and candidate ids) and then solves each step's LPs in
 * one launch per round, with the same outputs.  A smaller workspace fails with
 * LG_EINVAL. */
size_t lg_search_workspace_bytes(int32_t n_points, int32_t n_poses, const lg_search_params *params);

/*
 * lg_search -- seeded contact-set draws, force-closure verdicts, compaction.
 * Fingers (Sec. 5.3, k contact domains chosen at random): with c fingers of
 * pose g having a non-empty domain (dom_count > 0) and c >= k, set d picks k
 * of them without replacement, pick j taking the floor(w_j (c - j) / 2^32)-th
 * remaining one in increasing finger order, w = Philox blocks (g +
 * pose_offset, d, 13 | blk << 8, request_id), blk = 0, 1; contact i goes to
 * the i-th smallest picked finger (k = F: contact i on finger i).  Draw d of
 * pose g uses Philox blocks (g + pose_offset, 4d + blk, 3, request_id), blk =
 * 0, 1, ...: word i picks the point of contact i as the floor(w * count /
 * 2^32)-th set bit of its finger's domain; word k+i picks one of the finger's
 * links whose own table is hit at that point (reverse lookup of Sec. 5.5; -1
 * if none is, e.g. for domains of lg_query_domains_cone).  A pose with fewer
 * than k non-empty domains gives set_pt = -1, set_link = -1.
 * Verdict (object frame): wrench columns w_ie = [d_ie; p_i x d_ie / rho],
 * d_ie = -n_i + mu (cos(2 pi e/m) x_i + sin(2 pi e/m) y_i) with the Duff et
 * al. (2017) tangent basis; t* = min sum_r |(W g)_r| over g >= 0, sum g = 1
 * (double-precision Phase-1 simplex, Bland's rule); verdict = t* <= eps.
 * With opt_outer > 0 the drawn sets are first refined by Alg. 2 of Sec. 5.4:
 * for opt_outer rounds, each contact i in turn gets opt_inner candidates, its
 * point moved in the tangent plane of its object normal (Duff basis x_i, y_i)
 * by (dx, dy) ~ N(0, opt_sigma^2) and projected onto its finger's domain
 * (nearest domain point, lowest index on ties); contact i moves to the first candidate whose t* is within 1e-9 of the
 * candidates' minimum.  Candidate j of step s = (round * k + i) * opt_inner + j
 * uses Philox block (g + pose_offset, d, 5 | s << 8, request_id): Box-Muller of
 * u1 = ((w0 >> 8) + 1) / 2^24, u2 = (w1 >> 8) / 2^24.  tstar and verdict are
 * those of the final set; its links are picked again with the draw's words.
 * Outputs (device): set_pt [P][D][k] int32, set_link [P][D][k] int8 (global
 * joint/link index), verdict [P][D] uint8, tstar [P][D] double (NaN for
 * invalid sets), acc_list [P*D] int32 accepted set ids g*D + d in increasing
 * order, n_acc [1] int32.  workspace: device, lg_search_workspace_bytes().
 */
lg_status lg_search(const lg_field *field, const float *pts, const float *nrm, int32_t n_points,
                    const float *poses, int32_t n_poses, const uint32_t *dom_bits,
                    const uint32_t *dom_count, const lg_search_params *params, int32_t *set_pt,
                    int8_t *set_link, uint8_t *verdict, double *tstar, int32_t *acc_list,
                    int32_t *n_acc, void *workspace, size_t workspace_bytes, void *stream);

/*
 * lg_search_noalloc -- lg_search without a caller workspace, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, kernels and outputs
 * as lg_search, minus workspace/workspace_bytes: the workspace is a static
 * device array of lg_search_noalloc_max_bytes() bytes (8 MiB) per GPU, held
 * until the process ends; its device address is looked up once per device on
 * the first call there.  The per-candidate arrays of Alg. 2's gathered slow
 * LPs are used only when they fit; calls whose least workspace (see
 * lg_search_workspace_bytes) exceeds that size fail with LG_EINVAL before
 * anything is enqueued.  No call allocates:
 * no hipMalloc, hipFree or allocating library routine, and no memset node
 * (the cell counts of Alg. 2 are cleared by a kernel).  Every call on a GPU
 * shares that GPU's array, and each call rewrites what it reads from it:
 * calls that overlap in time on one GPU (different streams or threads) race
 * and give undefined results; serialise them.
 */
size_t lg_search_noalloc_max_bytes(void);
lg_status lg_search_noalloc(const lg_field *field, const float *pts, const float *nrm, int32_t n_points,
                            const float *poses, int32_t n_poses, const uint32_t *dom_bits,
                            const uint32_t *dom_count, const lg_search_params *params, int32_t *set_pt,
                            int8_t *set_link, uint8_t *verdict, double *tstar, int32_t *acc_list,
                            int32_t *n_acc, void *stream);

/*
 * lg_compact_unstable -- the ids (g * draws + d, increasing) of the sets of a
 * search whose draw is whole (every point and link >= 0) and whose verdict
 * is 0: the candidates of the second contact round once realised.  set_pt
 * [P][D][k] int32, set_link int8, verdict [P][D] uint8 (device); outputs list
 * [P*D] int32 and n_list [1] int32 (device).  workspace: device,
 * lg_compact_unstable_workspace_bytes().
 */
size_t lg_compact_unstable_workspace_bytes(int32_t n_poses, int32_t draws);
lg_status lg_compact_unstable(const int32_t *set_pt, const int8_t *set_link, const uint8_t *verdict,
                              int32_t n_poses, int32_t draws, int32_t k, int32_t *list, int32_t *n_list,
                              void *workspace, size_t workspace_bytes, void *stream);

/* Second contact round parameters. */
typedef struct {
    int32_t k_add;           /* contacts added on unused fingers, k + k_add <= fingers, <= 8 */
    uint32_t request_id;     /* 4th Philox counter word of this round's draws */
    const int32_t *list;     /* DEVICE, increasing set ids to extend, or NULL: every round-1 set with a
                                whole draw and verdict 0 */
    const int32_t *list_n;   /* DEVICE [1]: entries of list (required with a list) */
    const uint8_t *list_ok;  /* DEVICE, aligned with list, or NULL: only entries != 0 are extended
                                (e.g. lg_realize's valid of the listed sets: collision-free, contacts met) */
} lg_extend_params;

/*
 * lg_search_extend -- the second contact round on the unused fingers
 * (Sec. 5.3: an additional search phase adds contacts; Sec. 5.6: grasps that
 * are collision-free but not stable get an additional contact search on the
 * unused fingers, the general form of the method).  Round-1 sets are those
 * of lg_search with params (k contacts, draws, seed, pose_offset) on the same
 * domains.  Each set taken (see lg_extend_params) whose contacts all have a
 * point and a link gets k_add more: with c fingers unused by the set and with
 * a non-empty domain (c >= k_add, else the set is not extended), pick j takes
 * the floor(w_j (c - j) / 2^32)-th remaining one in increasing finger order,
 * w = Philox blocks (g + pose_offset, d, 19 | blk << 8, request_id); the
 * i-th smallest new finger's point is the floor(w * count / 2^32)-th bit of
 * its domain and its link the reverse lookup, w = word i and k_add + i of
 * Philox blocks (g + pose_offset, 4d + blk, 21, request_id).  The extended
 * set lists its k + k_add contacts in increasing finger order; its verdict
 * and t* are the criterion of lg_search on all of them; acc_list2 holds the
 * accepted extended sets.  Sets not extended: set_pt2 -1, verdict 0, t* NaN.
 * Outputs (device): set_pt2 [P][D][k + k_add] int32, set_link2 int8, verdict2
 * [P][D] uint8, tstar2 double, acc_list2 [P*D] int32, n_acc2 [1] int32.
 * workspace: device, lg_search_workspace_bytes() of params with k + k_add.
 * No palm contacts (params->palm_pt must be NULL).  Realize the extended sets
 * with lg_realize and k = k + k_add.
 */
lg_status lg_search_extend(const lg_field *field, const float *pts, const float *nrm, int32_t n_points,
                           const float *poses, int32_t n_poses, const uint32_t *dom_bits,
                           const uint32_t *dom_count, const lg_search_params *params, const int32_t *set_pt1,
                           const int8_t *set_link1, const uint8_t *verdict1, const lg_extend_params *ext,
                           int32_t *set_pt2, int8_t *set_link2, uint8_t *verdict2, double *tstar2,
                           int32_t *acc_list2, int32_t *n_acc2, void *workspace, size_t workspace_bytes,
                           void *stream);

/* Kinematics optimisation parameters (Sec. 5.5). */
typedef struct {
    int32_t iters;    /* DLS iterations (Eq. 7) */
    int32_t phase1;   /* leading iterations with the hand contact point fixed to the link */
    float lambda;     /* damping */
    float beta;       /* normal offset of the second matched point (m) */
    float tol_pos;    /* acceptance: contact error <= tol_pos (m) */
    float tol_ang;    /* acceptance: normal angle <= tol_ang (rad) */
    float margin;     /* acceptance: penetration depth <= margin (m) */
    int32_t self_collision; /* 1: depth also covers capsules of different fingers (Sec. 5.6
                               hand-to-hand check, closed-form segment distance); 0: object only */
    uint64_t seed;          /* Philox key of the random joint values of fingers without contact
                               (pass the search's seed) */
    uint32_t request_id;    /* 4th Philox counter word of those values (the search's request_id) */
    int64_t pose_offset;    /* global index of pose 0 (the search's pose_offset) */
} lg_ik_params;

/* Object signed-distance grid (object frame). */
typedef struct {
    float origin[3];      /* position of node (0,0,0) */
    float h;              /* node spacing */
    int32_t dims;         /* G nodes per axis, >= 2 */
    const float *values;  /* device [G][G][G] as [iz][iy][ix] */
} lg_sdf;

/*
 * lg_realize -- turn accepted sets into grasps (P, q) (Sec. 5.5, Sec. 3.2,
 * Sec. 5.6).  For accepted set a (id = acc_list[a], pose g = id / draws,
 * draw d = id % draws), contact i is on the finger of link set_link[id][i].
 * The set is realisable iff every link is a hand link, every point an object
 * point and the fingers increase strictly with i (as lg_search writes them);
 * otherwise its contact errors and angles are +inf and valid = 0.  A finger
 * without contact (k < F, or every finger of a set that is not realisable)
 * takes uniform joint values lo + (hi - lo) u, u = (w_t >> 8) / 2^24, w =
 * Philox blocks (g + pose_offset, d, 15 | (2 f + blk) << 8, request_id), blk
 * = 0, 1, key = seed (params).  An id outside [0, n_poses * draws) gives NaN
 * joints and depth, +inf errors, valid = 0, and is not read through.
 * For a finger with a contact, q0 is the field's witness
 * joint sample of (link, voxel(p), bin(n)) (mid-limits without witness);
 * `iters` DLS steps (Eq. 7-8) match the hand contact point -- the capsule
 * point closest to (p, n) in |x-p|^2 + beta^2 |n~-n|^2, held fixed for
 * `phase1` steps then re-selected -- and its beta-offset to p and p + beta n;
 * q is clamped to the limits.  Then every link's capsule axis (one sample per
 * mm, ends included) is tested against the trilinear SDF (+inf outside the
 * grid): depth = max (radius - SDF).  valid = all contact errors <= tol_pos,
 * all normal angles <= tol_ang, depth <= margin.
 * n_acc_dev: device [1] number of accepted sets (<= max_acc); entries past it
 * are not written.  Outputs (device, max_acc rows): q_out [J] float,
 * contact_err [k] float, contact_ang [k] float, depth float, valid uint8.
 */
lg_status lg_realize(const lg_field *field, const lg_sdf *sdf, const float *pts, const float *nrm,
                     int32_t n_points, const float *poses, int32_t n_poses,
                     const int32_t *set_pt, const int8_t *set_link, int32_t k, int32_t draws,
                     const int32_t *acc_list, const int32_t *n_acc_dev, int32_t max_acc,
                     const lg_ik_params *params, float *q_out, float *contact_err,
                     float *contact_ang, float *depth, uint8_t *valid, void *stream);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of grasp requests over resident fields.       */
/* The paper caches each stage's output for reuse across forward passes       */
/* (Fig. 6) and reuses search results (Sec. 5.7); a server keeps the fields   */
/* resident and interleaves many requests on one GPU.  A request (object +    */
/* palm poses + search parameters) is admitted when its device memory fits   */
/* the HBM budget (FIFO); its poses are processed in chunks of `chunk_poses`, */
/* chunks of different requests run concurrently, and a request's RNG        */
/* counters depend only on (request_id, pose index within the request,        */
/* draw), so its result is the same alone and in any mix.                     */
/* Two ways to run the chunks:                                                */
/*  - batched = 0: each request's chunk launches its own kernels on the       */
/*    request's stream (up to `max_active` streams);                          */
/*  - batched = 1: the next chunk of every idle request is described in a     */
/*    per-chunk descriptor table (its field, buffers, sizes and parameters)   */
/*    and the batch runs as one launch per stage: query, draws, pose list,    */
/*    verdicts, accepted-set list, IK + penetration, counters.  Chunks of     */
/*    uneven size share a launch (each owns the blocks its size needs); the   */
/*    kernels with a size template (fingers, contacts, joints per finger)     */
/*    take one launch per size class present.  Up to `batch_slots` batches   */
/*    are in flight, one stream each; when several slots are free, the idle   */
/*    chunks, in ascending size (poses x points), are cut into that many      */
/*    batches of about equal work, so small chunks do not wait behind large   */
/*    ones.  A request joins batches once its upload has finished; one of    */
/*    two chunks or more holds two copies of the chunk buffers, so two of its */
/*    chunks can be in flight at once, in two batches.  Requests              */
/*    with the contact-point optimisation (opt_outer > 0) run on their own    */
/*    streams in either mode.                                                 */
/* Host API, thread-safe; work runs on a server thread.                       */
/* ------------------------------------------------------------------------ */
typedef struct lg_server lg_server;

typedef struct {
    uint64_t budget_bytes;  /* device memory reserved for admitted requests */
    int32_t max_active;     /* requests in flight at once, 1..64 */
    int32_t chunk_poses;    /* poses per scheduling quantum, >= 1 */
    int32_t batched;        /* 1: batched launches over a descriptor table (see above) */
    int32_t batch_slots;    /* batched mode: batches in flight at once, 1..8 (0: 4) */
} lg_server_params;

typedef struct {
    const lg_field *field;    /* resident field of the hand; must outlive the request */
    const float *pts;         /* host [N][3] object points (object frame); copied at submit */
    const float *nrm;         /* host [N][3] outward unit normals */
    int32_t n_points;
    const float *poses;       /* host [P][12] palm poses */
    int32_t n_poses;
    lg_search_params search;  /* request_id and pose_offset are ignored (set per chunk) */
    uint32_t request_id;      /* RNG stream of the request */
    int32_t realize;          /* 1: run IK + penetration (needs ik and sdf) */
    lg_ik_params ik;
    const float *sdf_values;  /* host [G][G][G], used when realize = 1 */
    float sdf_origin[3];
    float sdf_h;
    int32_t sdf_dims;
} lg_request;

#define LG_REQ_QUEUED 0
#define LG_REQ_RUNNING 1
#define LG_REQ_DONE 2
#define LG_REQ_CANCELLED 3
#define LG_REQ_FAILED 4

typedef struct {
    int32_t state;          /* LG_REQ_* */
    int32_t status;         /* lg_status of a failed request */
    int64_t n_acc;          /* accepted sets (verdict true) */
    int64_t n_valid;        /* valid grasps (= n_acc without realize) */
    uint64_t acc_hash;      /* order-independent hash of the accepted (pose, draw) ids */
    double t_submit, t_admit, t_done;  /* seconds on the server's clock */
    uint64_t bytes;         /* device memory reserved for the request */
} lg_result;

typedef struct {
    int64_t submitted, admitted, completed, cancelled, rejected, failed;
    uint64_t budget_bytes, bytes_in_use, peak_bytes;
    int32_t queued, active;
    int64_t batches, batched_chunks;  /* batched launches so far and the chunks they held */
} lg_server_stats;

/* Device bytes a request reserves while admitted (inputs + one chunk of
 * working buffers).  Requests larger than the budget are rejected. */
uint64_t lg_serve_request_bytes(const lg_server_params *params, const lg_request *req);
/* Create a server on the current device (allocates the budget slab). */
lg_status lg_serve_create(const lg_server_params *params, lg_server **out);
/* Copy the request's host data and queue it; LG_EBUDGET if it can never fit. */
lg_status lg_serve_submit(lg_server *srv, const lg_request *req, uint64_t *ticket);
/* Current state / result of a ticket (LG_EINVAL for an unknown ticket). */
lg_status lg_serve_poll(lg_server *srv, uint64_t ticket, lg_result *out);
/* Block until the ticket is DONE/CANCELLED/FAILED or timeout_s elapses. */
lg_status lg_serve_wait(lg_server *srv, uint64_t ticket, double timeout_s, lg_result *out);
/* Cancel: a queued request is dropped; a running one stops after its chunk. */
lg_status lg_serve_cancel(lg_server *srv, uint64_t ticket);
lg_status lg_serve_stats(lg_server *srv, lg_server_stats *out);
/* Seconds on the server's clock (the clock of t_submit/t_admit/t_done). */
double lg_serve_clock(lg_server *srv);
/* Finish in-flight chunks, cancel the rest, free everything. */
lg_status lg_serve_destroy(lg_server *srv);

/* ---- object preprocessing ----------------------------------------------------
 * lg_concave_filter -- concave-point removal of Sec. 5.2: a point is dropped
 * when a small box placed at it penetrates the object.  The box is a cube of
 * edge box_edge (m) standing on the surface: bottom face centred at the point
 * p, axes (x, y, n) with n the unit outward normal and (x, y) its Duff et al.
 * (2017) tangents.  depth = max of -SDF (trilinear, +inf outside the grid)
 * over the lattice p + a x + b y + c n, a, b = -s/2 + s i / m, c = s i / m,
 * i = 0..m (m = lattice, 1..16); keep = depth <= max_depth.
 * Inputs: sdf (device grid), pts/nrm DEVICE SoA [3][N].  Outputs (device):
 * depth [N] float, keep [N] uint8, kept_idx [N] int32 (kept point indices in
 * increasing order; entries past n_kept are not written), n_kept [1] int32.
 * LG_EINVAL on a bad sdf, box_edge <= 0, lattice outside 1..16, NaN max_depth
 * or null buffers.  N = 0 writes n_kept = 0 only.
 */
lg_status lg_concave_filter(const lg_sdf *sdf, const float *pts, const float *nrm, int32_t n_points,
                            float box_edge, int32_t lattice, float max_depth, float *depth, uint8_t *keep,
                            int32_t *kept_idx, int32_t *n_kept, void *stream);

/* lg_gather_points -- pts_out/nrm_out DEVICE SoA [3][n_out] = the columns
 * idx[0..n_out) of pts/nrm DEVICE SoA [3][N] (e.g. the points lg_concave_filter
 * kept, n_out read back from n_kept).  An index outside [0, N) gives NaN
 * columns.  LG_EINVAL on negative sizes or null buffers. */
lg_status lg_gather_points(const float *pts, const float *nrm, int32_t n_points, const int32_t *idx, int32_t n_out,
                           float *pts_out, float *nrm_out, void *stream);

/* ---- exhaustive placement ----------------------------------------------------
 * lg_place_exhaustive -- object poses of the exhaustive placement of Sec. 5.1:
 * pose g puts a random object surface point onto a random contact vector of
 * the field with opposite normals.  Philox blocks (g + pose_offset, b, 11,
 * request_id), b = 0, 1, key = seed, select as floor(w * count / 2^32): word 0
 * the finger f, word 1 the joint sample s (the field's own FK of finger f at
 * sample s), word 2 the link of f, word 3 the link surface sample (point x,
 * outward normal nu), word 4 the object point i; word 5 a roll psi = 2 pi u.
 * R takes n_i onto -nu (the minimal rotation; below a cosine of -0.9999 a
 * half-turn about the Duff x-axis of n_i first), then rolls it by psi about
 * -nu; t = x - R p_i.  pts/nrm: DEVICE SoA [3][N]; poses: DEVICE [P][12] out.
 * LG_EINVAL on null buffers or n_points <= 0.
 */
lg_status lg_place_exhaustive(const lg_field *field, const float *pts, const float *nrm, int32_t n_points,
                              int32_t n_poses, uint64_t seed, uint32_t request_id, int64_t pose_offset,
                              float *poses, void *stream);

/* lg_place_palm -- static-link (palm) placements of Sec. 5.1, in place over
 * `poses` (DEVICE [P][12]): with probability prob (u01(w0) < prob), pose g is
 * replaced by one that puts object point i onto palm contact vector js (the
 * field's hand desc), normals opposed, rolled by psi about the contact normal
 * (the alignment of lg_place_exhaustive); Philox block (g + pose_offset, 0,
 * 17, request_id), key = seed: word 0 the selection, word 1 js, word 2 i,
 * word 3 psi = 2 pi u.  The placement is kept when no palm capsule (axis
 * samples one per mm, ends included) penetrates the object's trilinear SDF by
 * more than margin.  palm_pt (DEVICE [P] int32 out): i (kept), -1 (pose not
 * selected, left untouched), -2 (rejected; the palm pose is still written).
 * Feed palm_pt to lg_search through lg_search_params.palm_pt.
 * LG_EINVAL without palm contact vectors in the hand, on a bad sdf,
 * n_points <= 0, prob outside [0, 1], NaN margin or null buffers.
 */
lg_status lg_place_palm(const lg_field *field, const lg_sdf *sdf, const float *pts, const float *nrm,
                        int32_t n_points, int32_t n_poses, float prob, float margin, uint64_t seed,
                        uint32_t request_id, int64_t pose_offset, float *poses, int32_t *palm_pt, void *stream);

/* ---- learned palm-pose proposer ------------------------------------------------
 * Data-driven search (Sec. 5.7) names learning where to search as a way to skip
 * unproductive regions of the pose space; the paper leaves it unimplemented.
 * This is the project's proposer: a PointNet-style encoder (shared MLP 6 -> 128
 * -> 256 with ReLU, max-pool over the points) and a head 256 -> 256 -> 256
 * (ReLU) -> 152 = 8 x (logit, 9 means, 9 log-sigmas) of a diagonal Gaussian
 * mixture over y = (R[:,0], R[:,1], t / 0.1 m) of a palm pose [R | t]; the
 * rotation is recovered by Gram-Schmidt.  Matrix products run on BF16 MFMA
 * with FP32 accumulation; training keeps FP32 master weights and Adam state.
 * Proposed poses go through lg_query_domains / lg_search / lg_realize
 * unchanged; uniform poses remain the fallback (uniform_frac below).
 *
 * Inputs x are DEVICE [B][Np][6] float32 rows (p in m, unit outward normal n),
 * typically a seeded subsample of the object's points; the network scales p
 * by 1 / 0.1 m.  The library owns each lg_prop: its weights, Adam state and the
 * activations of one batch of at most max_batch objects x max_points points
 * and max_targets targets.  Calls on one lg_prop must not overlap: they share
 * its activation buffers.
 */
typedef struct lg_prop lg_prop;

typedef struct {
    int32_t max_batch;    /* objects per forward / training call, [1, 4096] */
    int32_t max_points;   /* points per object, [1, 2^24] */
    int32_t max_targets;  /* target poses per training call, [1, 2^26] */
    uint64_t seed;        /* Philox key of the He-uniform initialisation */
} lg_prop_params;

/* Number of FP32 parameters (204,568); the flat layout is, per layer
 * W1 [6][128], b1, W2 [128][256], b2, Wa [256][256], ba, Wb [256][256], bb,
 * Wc [256][152], bc, each weight row-major [in][out]. */
int64_t lg_prop_num_params(void);

/* Allocates and initialises a proposer on the current device (synchronises
 * `stream`).  LG_EINVAL on limits outside the ranges above, LG_ENOMEM. */
lg_status lg_prop_create(const lg_prop_params *params, void *stream, lg_prop **out);
lg_status lg_prop_release(lg_prop *p);

/* Host copies of the FP32 master weights [lg_prop_num_params()] (checkpoints).
 * set also refreshes the BF16 copies and resets the Adam state; both calls
 * synchronise the device. */
lg_status lg_prop_get_params(const lg_prop *p, float *host_out);
lg_status lg_prop_set_params(lg_prop *p, const float *host_in);

/* Forward pass of B objects with Np points each.  Optional outputs (NULL =
 * skip): out [B][152] mixture parameters, feat [B][256] pooled features,
 * arg [B][256] the point index of each channel's maximum: the point with the
 * largest FP32 layer-2 sum before the bias (lowest index among equal sums),
 * or 0 for a channel cut to zero by the ReLU (every point then ties at 0).
 * LG_EINVAL if B or Np is outside the proposer's limits. */
lg_status lg_prop_forward(lg_prop *p, const float *x, int32_t B, int32_t Np, float *out, float *feat,
                          int32_t *arg, void *stream);

/* Mean mixture negative log-likelihood over T targets and its gradient.
 * targets [T][9] are y vectors; object b owns targets offsets[b] ..
 * offsets[b+1]-1 (offsets [B+1], offsets[0] = 0, offsets[B] = T, both DEVICE).
 * Writes loss [1] and grad [lg_prop_num_params()] when non-NULL; the gradient
 * also stays in the proposer for lg_prop_adam. */
lg_status lg_prop_backward(lg_prop *p, const float *x, int32_t B, int32_t Np, const float *targets,
                           const int32_t *offsets, int32_t T, float *loss, float *grad, void *stream);

/* One Adam step (Kingma & Ba 2015, bias-corrected step size) with the last
 * gradient; refreshes the BF16 weight copies. */
lg_status lg_prop_adam(lg_prop *p, float lr, float beta1, float beta2, float eps, void *stream);

/* lg_prop_backward followed by lg_prop_adam(lr, 0.9, 0.999, 1e-8). */
lg_status lg_prop_train_step(lg_prop *p, const float *x, int32_t B, int32_t Np, const float *targets,
                             const int32_t *offsets, int32_t T, float lr, float *loss, void *stream);

/* n_poses palm poses [n_poses][12] from one mixture row mix [152].  Pose i
 * uses Philox4x32-10 blocks (i, j, 7, 0), j = 0..2, key (seed lo, seed hi):
 * with probability uniform_frac a uniform pose (Shoemake rotation, object
 * origin at distance U[d_lo, d_hi] along a direction uniform on the +z
 * hemisphere), else a draw of the mixture (component by inversion of the
 * cumulative softmax, Box-Muller normals, log-sigma clamped to [-5, 2]). */
lg_status lg_prop_sample_mixture(const float *mix, int32_t n_poses, uint64_t seed, float uniform_frac, float d_lo,
                                 float d_hi, float *poses, void *stream);

/* Forward pass of one object (x [Np][6]) and n_poses samples of its mixture. */
lg_status lg_prop_sample(lg_prop *p, const float *x, int32_t Np, int32_t n_poses, uint64_t seed, float uniform_frac,
                         float d_lo, float d_hi, float *poses, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* LG_H */
