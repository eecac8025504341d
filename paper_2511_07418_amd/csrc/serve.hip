// Serving: continuous batching of grasp requests over resident contact fields.
//
// The paper builds a field once per hand and caches stage outputs for later
// forward passes (Fig. 6, Sec. 5.7).  A server keeps the fields resident and
// runs many requests' searches on one GPU at once:
//  * admission: one device slab of `budget_bytes` is sub-allocated first-fit;
//    a request is admitted (FIFO) when its inputs and one chunk of working
//    buffers fit, and its block is returned when it completes;
//  * interleaving: the server thread runs one chunk of `chunk_poses` poses
//    per request at a time (query -> draws/verdicts/compaction -> optional
//    IK + penetration -> counters), so a long request never blocks a short
//    one behind it.  Per-stream mode: every admitted request owns a stream
//    (default priority) and its chunk launches its own kernels.  Batched
//    mode: the next chunks of all idle requests are written into a
//    descriptor table (one ChunkDesc each) and run as one launch per stage,
//    each chunk owning the blocks its size needs; `batch_slots` batches can
//    be in flight, one stream each, so batches are assembled while others
//    run; a request joins batches once its admission upload has finished;
//  * determinism: RNG counters depend on (request_id, pose index within the
//    request, draw) only, so results are identical alone and in any mix.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "lg_internal.h"

namespace lg {

constexpr uint64_t kAlign = 256;

static constexpr uint64_t align_up(uint64_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// splitmix64 finaliser (Steele, Lea, Flood 2014) of (request, set id)
__device__ inline uint64_t mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

constexpr int kAccThreads = 256;

// counters[0] += n_acc, counters[1] += valid, counters[2] += sum of mix64(id);
// block bid of nb (grid-stride)
__device__ __forceinline__ void accumulate_block(int bid, int nb, const int32_t *__restrict__ acc_list,
                                                 const int32_t *__restrict__ n_acc_dev,
                                                 const uint8_t *__restrict__ valid, int64_t set_base,
                                                 uint32_t request_id, unsigned long long *__restrict__ counters)
{
    const int n = *n_acc_dev;
    unsigned long long c = 0, v = 0, h = 0;
    for (int i = bid * kAccThreads + threadIdx.x; i < n; i += nb * kAccThreads) {
        const uint64_t id = (uint64_t)(set_base + acc_list[i]);
        c += 1;
        v += valid ? (valid[i] != 0) : 1;
        h += mix64(((uint64_t)request_id << 40) ^ id);
    }
    for (int off = 32; off > 0; off >>= 1) {
        c += __shfl_down(c, off, 64);
        v += __shfl_down(v, off, 64);
        h += __shfl_down(h, off, 64);
    }
    if ((threadIdx.x & 63) == 0 && c) {
        atomicAdd(counters, c);
        atomicAdd(counters + 1, v);
        atomicAdd(counters + 2, h);
    }
}

__global__ void __launch_bounds__(kAccThreads)
k_serve_accumulate(const int32_t *__restrict__ acc_list, const int32_t *__restrict__ n_acc_dev,
                   const uint8_t *__restrict__ valid, int64_t set_base, uint32_t request_id,
                   unsigned long long *__restrict__ counters)
{
    accumulate_block(blockIdx.x, gridDim.x, acc_list, n_acc_dev, valid, set_base, request_id, counters);
}

__global__ void __launch_bounds__(kAccThreads)
k_accumulate_batch(const ChunkDesc *__restrict__ d, const uint16_t *__restrict__ idx,
                   const uint32_t *__restrict__ first, int n)
{
    const int j = batch_member(first, n, blockIdx.x);
    const ChunkDesc &c = d[idx[j]];
    accumulate_block(blockIdx.x - first[j], first[j + 1] - first[j], c.acc, c.n_acc, c.realize ? c.valid : nullptr,
                     c.pose_offset * c.D, c.request_id, c.counters);
}

// First-fit sub-allocator over one device slab (host-side bookkeeping only).
class Slab {
  public:
    uint64_t size = 0;
    char *base = nullptr;
    bool alloc(uint64_t n, uint64_t &off)
    {
        n = align_up(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                off = it->first;
                const uint64_t rest = it->second - n;
                const uint64_t roff = it->first + n;
                free_.erase(it);
                if (rest) free_[roff] = rest;
                used_ += n;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t n)
    {
        n = align_up(n);
        used_ -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    void reset(uint64_t n)
    {
        size = n;
        free_.clear();
        free_[0] = n;
        used_ = 0;
    }
    uint64_t used() const { return used_; }

  private:
    std::map<uint64_t, uint64_t> free_;
    uint64_t used_ = 0;
};

// Sizes of one request's device buffers: its inputs and counters, then
// `nbuf` copies of one chunk's working buffers (the offsets are those of copy
// 0; copy j lies j * buf_bytes further).  Batched requests of two chunks or
// more get two copies, so that two of their chunks can be in flight, in two
// batches, unless two copies exceed the server's budget; the others get one.
struct ReqLayout {
    uint64_t pts, nrm, bounds, poses, sdf, counters;
    uint64_t dom_bits, dom_count, set_pt, set_link, verdict, tstar, acc, n_acc, ws, ws_bytes;
    uint64_t q, err, ang, depth, valid;
    uint64_t buf_bytes;
    int nbuf;
    uint64_t total;
};

static bool batched_request(const lg_server_params &sp, const lg_request &r)
{
    return sp.batched && r.search.opt_outer == 0;
}

static ReqLayout layout_of(const lg_server_params &sp, const lg_request &r)
{
    const lg_field *f = r.field;
    const int F = f->dh.F, J = f->dh.J, k = r.search.k, D = r.search.draws;
    const int64_t N = r.n_points, chunk = std::min<int64_t>(sp.chunk_poses, r.n_poses);
    const int64_t NW = (N + 31) / 32, sets = chunk * D;
    ReqLayout L;
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t o = off;
        off += align_up(bytes);
        return o;
    };
    L.pts = take(12 * N);
    L.nrm = take(12 * N);
    L.bounds = take(16 * (uint64_t)((N + 63) / 64));  // chunk bounding spheres of the object
    L.poses = take(48 * (uint64_t)r.n_poses);
    const int64_t G = r.realize ? r.sdf_dims : 0;
    L.sdf = take(4 * (uint64_t)(G * G * G));
    L.counters = take(3 * 8);
    const uint64_t work0 = off;
    L.dom_bits = take(4 * (uint64_t)(chunk * F * NW));
    L.dom_count = take(4 * (uint64_t)(chunk * F));
    L.set_pt = take(4 * (uint64_t)(sets * k));
    L.set_link = take((uint64_t)(sets * k));
    L.verdict = take((uint64_t)sets);
    L.tstar = take(8 * (uint64_t)sets);
    L.acc = take(4 * (uint64_t)sets);
    L.n_acc = take(4);
    lg_search_params p = r.search;
    L.ws_bytes = lg_search_workspace_bytes((int32_t)N, (int32_t)chunk, &p);
    L.ws = take(L.ws_bytes);
    const int64_t ra = r.realize ? sets : 0;
    L.q = take(4 * (uint64_t)(ra * J));
    L.err = take(4 * (uint64_t)(ra * k));
    L.ang = take(4 * (uint64_t)(ra * k));
    L.depth = take(4 * (uint64_t)ra);
    L.valid = take((uint64_t)ra);
    L.buf_bytes = off - work0;
    L.nbuf = batched_request(sp, r) && r.n_poses > chunk ? 2 : 1;
    if (work0 + L.nbuf * L.buf_bytes > sp.budget_bytes) L.nbuf = 1;  // one copy if two cannot fit
    L.total = work0 + L.nbuf * L.buf_bytes;
    return L;
}

struct Req {
    uint64_t ticket = 0;
    lg_request r{};
    std::vector<float> pts, nrm, poses, sdf;  // host copies (SoA for pts/nrm)
    ReqLayout L{};
    uint64_t off = 0;
    int slot = -1;
    int32_t state = LG_REQ_QUEUED;
    int32_t status = LG_OK;
    bool cancel = false;
    int inflight = 0;      // chunks enqueued and not yet complete
    uint32_t buf_busy = 0; // working-buffer copies held by chunks in flight (bit per copy)
    bool batched = false;  // chunks go through the batched launches
    bool fresh = false;    // admission copies not yet waited for by a batch
    int64_t next_pose = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    unsigned long long counters[3] = {0, 0, 0};
    hipEvent_t ev = nullptr;
};

// Batched launches: one descriptor table per batch slot, staged in pinned
// host memory and copied to the device ahead of the batch's kernels.  A table
// holds kMaxBatch chunk descriptors and up to kMaxLaunch member lists.
constexpr int kMaxBatch = 64;
constexpr int kMaxLaunch = 48;
constexpr int kMaxBatchSlots = 8;
constexpr size_t kListBytes = align_up(2 * kMaxBatch) + align_up(4 * (kMaxBatch + 1));
constexpr size_t kTableBytes = align_up(sizeof(ChunkDesc) * kMaxBatch) + kMaxLaunch * kListBytes;

struct BatchSlot {
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;
    char *dev = nullptr;   // device table
    char *host = nullptr;  // pinned staging copy
    std::vector<Req *> members;
    std::vector<int> bufs;  // the working-buffer copy of each member's chunk
    bool busy = false;
};

}  // namespace lg

struct lg_server {
    lg_server_params p{};
    int device = 0;
    lg::Slab slab;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    std::vector<int> free_slots;
    std::vector<lg::BatchSlot> batch;
    int n_cu = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::thread worker;
    bool stop = false;
    std::deque<lg::Req *> queued;
    std::vector<lg::Req *> active;
    std::unordered_map<uint64_t, std::unique_ptr<lg::Req>> all;
    uint64_t next_ticket = 1;
    lg_server_stats st{};
    std::chrono::steady_clock::time_point t0;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace lg {

static lg_status validate_request(const lg_server_params &sp, const lg_request *r)
{
    if (!r || !r->field) return fail(LG_EINVAL, "null request or field");
    if (r->n_points <= 0 || r->n_poses <= 0 || !r->pts || !r->nrm || !r->poses)
        return fail(LG_EINVAL, "request needs points, normals and poses");
    if (r->search.k < 1 || r->search.k > r->field->dh.F)
        return fail(LG_EINVAL, "need 1 <= k <= the field's number of fingers");
    if (r->search.palm_pt) return fail(LG_EINVAL, "palm contacts are not served (search.palm_pt must be NULL)");
    if (r->search.draws <= 0 || r->search.m_edges < 3 || r->search.m_edges > 16)
        return fail(LG_EINVAL, "bad search parameters");
    if ((int64_t)std::min<int64_t>(sp.chunk_poses, r->n_poses) * r->search.draws > 0x7fffffffLL)
        return fail(LG_EINVAL, "chunk_poses * draws must be < 2^31");
    if (r->realize && (!r->sdf_values || r->sdf_dims < 2 || !(r->sdf_h > 0.f) || !(r->ik.lambda > 0.f) ||
                       r->ik.iters < 0 || r->ik.phase1 < 0))
        return fail(LG_EINVAL, "realize needs an SDF and IK parameters");
    // what the search and the query refuse at launch is refused here, in either mode
    const lg_search_params &p = r->search;
    if (p.k > 8 || !(p.mu >= 0.0f) || !(p.moment_scale > 0.0f) || p.max_pivots < 0)
        return fail(LG_EINVAL, "need k <= 8, mu >= 0, moment_scale > 0, max_pivots >= 0");
    if (p.opt_outer < 0 || p.opt_outer > 64 || (p.opt_outer > 0 && (p.opt_inner < 1 || p.opt_inner > 16)) ||
        !(p.opt_sigma >= 0.0f) || (int64_t)p.opt_outer * p.k * p.opt_inner >= (1 << 24))
        return fail(LG_EINVAL, "need 0 <= opt_outer <= 64, 1 <= opt_inner <= 16, opt_sigma >= 0");
    if ((int64_t)r->n_points * 12 > 0xffffffffLL || draw_lds_bytes(r->field->dh.F, r->n_points) > 48 * 1024)
        return fail(LG_EUNSUPPORTED, "too many points for the query offsets or the draw rank structure");
    return LG_OK;
}

// enqueue the next chunk of request q on its stream (server lock held)
static lg_status launch_chunk(lg_server *S, Req *q)
{
    hipStream_t s = S->streams[q->slot];
    const lg_request &r = q->r;
    char *base = S->slab.base + q->off;
    const ReqLayout &L = q->L;
    const int64_t g0 = q->next_pose;
    const int32_t P = (int32_t)std::min<int64_t>(S->p.chunk_poses, r.n_poses - g0);
    const float *pts = reinterpret_cast<const float *>(base + L.pts);
    const float *nrm = reinterpret_cast<const float *>(base + L.nrm);
    const float *poses = reinterpret_cast<const float *>(base + L.poses) + 12 * g0;
    uint32_t *db = reinterpret_cast<uint32_t *>(base + L.dom_bits);
    uint32_t *dc = reinterpret_cast<uint32_t *>(base + L.dom_count);
    lg_status st = lg_query_domains_bounded(r.field, pts, nrm, r.n_points, poses, P,
                                            reinterpret_cast<const float *>(base + L.bounds), db, dc, s);
    if (st != LG_OK) return st;
    lg_search_params sp = r.search;
    sp.request_id = r.request_id;
    sp.pose_offset = g0;
    int32_t *set_pt = reinterpret_cast<int32_t *>(base + L.set_pt);
    int8_t *set_link = reinterpret_cast<int8_t *>(base + L.set_link);
    int32_t *acc = reinterpret_cast<int32_t *>(base + L.acc);
    int32_t *n_acc = reinterpret_cast<int32_t *>(base + L.n_acc);
    st = lg_search(r.field, pts, nrm, r.n_points, poses, P, db, dc, &sp, set_pt, set_link,
                   reinterpret_cast<uint8_t *>(base + L.verdict), reinterpret_cast<double *>(base + L.tstar), acc,
                   n_acc, base + L.ws, L.ws_bytes, s);
    if (st != LG_OK) return st;
    uint8_t *valid = nullptr;
    if (r.realize) {
        lg_sdf sdf;
        memcpy(sdf.origin, r.sdf_origin, sizeof sdf.origin);
        sdf.h = r.sdf_h;
        sdf.dims = r.sdf_dims;
        sdf.values = reinterpret_cast<const float *>(base + L.sdf);
        valid = reinterpret_cast<uint8_t *>(base + L.valid);
        lg_ik_params ik = r.ik;  // random joints of fingers without contact: keyed like the search
        ik.seed = sp.seed;
        ik.request_id = sp.request_id;
        ik.pose_offset = sp.pose_offset;
        st = lg_realize(r.field, &sdf, pts, nrm, r.n_points, poses, P, set_pt, set_link, sp.k, sp.draws, acc, n_acc,
                        P * sp.draws, &ik, reinterpret_cast<float *>(base + L.q),
                        reinterpret_cast<float *>(base + L.err), reinterpret_cast<float *>(base + L.ang),
                        reinterpret_cast<float *>(base + L.depth), valid, s);
        if (st != LG_OK) return st;
    }
    hipLaunchKernelGGL(k_serve_accumulate, dim3(64), dim3(256), 0, s, acc, n_acc, valid, g0 * (int64_t)sp.draws,
                       r.request_id, reinterpret_cast<unsigned long long *>(base + L.counters));
    LG_HIP(hipGetLastError());
    LG_HIP(hipEventRecord(q->ev, s));
    q->next_pose = g0 + P;
    q->inflight = 1;
    return LG_OK;
}

// ---- batched launches ----------------------------------------------------------
// The next chunk of each member goes through one launch per stage; members
// are grouped by the template bucket of the kernels that have one.
static int fm_bucket(int F) { return F <= 3 ? 3 : F <= 4 ? 4 : F <= 5 ? 5 : 8; }
static int km_bucket(int k) { return k <= 3 ? 3 : k <= 4 ? 4 : k <= 5 ? 5 : k <= 6 ? 6 : 8; }
static int dm_bucket(int d) { return d <= 4 ? 4 : d <= 6 ? 6 : 8; }

// host view of a slot's table while it is filled
struct TableWriter {
    char *host, *dev;
    int n_lists = 0;
    static constexpr size_t kListBase = align_up(sizeof(ChunkDesc) * kMaxBatch);
    ChunkDesc *descs() { return reinterpret_cast<ChunkDesc *>(host); }
    // member list `who` (table entries) owning nb[j] blocks each
    lg_status list(const std::vector<int> &who, const std::vector<uint32_t> &nb, BatchLaunch &out)
    {
        if (n_lists >= kMaxLaunch) return fail(LG_EINVAL, "batch needs more member lists than its table holds");
        const size_t off = kListBase + (size_t)n_lists * kListBytes, foff = off + align_up(2 * kMaxBatch);
        uint16_t *idx = reinterpret_cast<uint16_t *>(host + off);
        uint32_t *first = reinterpret_cast<uint32_t *>(host + foff);
        uint64_t t = 0;
        first[0] = 0;
        for (size_t j = 0; j < who.size(); ++j) {
            idx[j] = (uint16_t)who[j];
            t += nb[j];
            first[j + 1] = (uint32_t)t;
        }
        if (t > 0x7fffffffull) return fail(LG_EINVAL, "batched launch above 2^31 - 1 blocks");
        out.d = reinterpret_cast<const ChunkDesc *>(dev);
        out.idx = reinterpret_cast<const uint16_t *>(dev + off);
        out.first = reinterpret_cast<const uint32_t *>(dev + foff);
        out.n = (int)who.size();
        out.blocks = (uint32_t)t;
        ++n_lists;
        return LG_OK;
    }
};

// every argument of request q's next chunk of P poses, in working-buffer copy buf
static void fill_desc(const lg_server *S, const Req *q, int32_t P, int buf, ChunkDesc &c)
{
    const lg_request &r = q->r;
    const lg_field *f = r.field;
    char *in = S->slab.base + q->off;                    // inputs and counters
    char *base = in + (uint64_t)buf * q->L.buf_bytes;  // this chunk's working buffers
    const ReqLayout &L = q->L;
    const int64_t g0 = q->next_pose;
    memset(&c, 0, sizeof c);
    c.H = f->dh;
    c.merged = f->d_merged;
    c.bits = f->d_bits;
    c.wit = f->has_witness ? f->d_wit : nullptr;
    c.pts = reinterpret_cast<const float *>(in + L.pts);
    c.nrm = reinterpret_cast<const float *>(in + L.nrm);
    c.poses = reinterpret_cast<const float *>(in + L.poses) + 12 * g0;
    c.bounds = reinterpret_cast<const float4 *>(in + L.bounds);
    c.N = r.n_points;
    c.P = P;
    c.D = r.search.draws;
    c.k = r.search.k;
    c.m = r.search.m_edges;
    c.max_pivots = r.search.max_pivots;
    c.seed_lo = (uint32_t)r.search.seed;
    c.seed_hi = (uint32_t)(r.search.seed >> 32);
    c.request_id = r.request_id;
    c.pose_offset = g0;
    c.mu = (double)r.search.mu;
    c.rho = (double)r.search.moment_scale;
    c.eps = (double)r.search.eps;
    c.cs = lp_const(c.m);
    c.dom_bits = reinterpret_cast<uint32_t *>(base + L.dom_bits);
    c.dom_count = reinterpret_cast<uint32_t *>(base + L.dom_count);
    c.set_pt = reinterpret_cast<int32_t *>(base + L.set_pt);
    c.set_link = reinterpret_cast<int8_t *>(base + L.set_link);
    c.verdict = reinterpret_cast<uint8_t *>(base + L.verdict);
    c.tstar = reinterpret_cast<double *>(base + L.tstar);
    c.acc = reinterpret_cast<int32_t *>(base + L.acc);
    c.n_acc = reinterpret_cast<int32_t *>(base + L.n_acc);
    chunk_workspace(base + L.ws, r.n_points, P, r.search.draws, c);
    c.realize = r.realize ? 1 : 0;
    if (r.realize) {
        c.S = SdfDev{r.sdf_origin[0], r.sdf_origin[1], r.sdf_origin[2], r.sdf_h, 1.0f / r.sdf_h, r.sdf_dims,
                     reinterpret_cast<const float *>(in + L.sdf)};
        const lg_ik_params &p = r.ik;  // random joints of fingers without contact: keyed like the search
        c.ik = IkDev{p.iters, p.phase1, p.lambda, p.beta, p.tol_pos, p.tol_ang, p.margin, p.self_collision,
                     c.seed_lo, c.seed_hi, r.request_id, g0};
        c.q = reinterpret_cast<float *>(base + L.q);
        c.err = reinterpret_cast<float *>(base + L.err);
        c.ang = reinterpret_cast<float *>(base + L.ang);
        c.depth = reinterpret_cast<float *>(base + L.depth);
        c.valid = reinterpret_cast<uint8_t *>(base + L.valid);
    }
    c.counters = reinterpret_cast<unsigned long long *>(in + L.counters);
}

// members with the same bucket value, in member order
template <class Key>
static std::vector<std::vector<int>> buckets(const std::vector<int> &who, Key key)
{
    std::vector<std::vector<int>> out;
    std::vector<int> keys;
    for (int m : who) {
        const int kv = key(m);
        size_t b = std::find(keys.begin(), keys.end(), kv) - keys.begin();
        if (b == keys.size()) {
            keys.push_back(kv);
            out.emplace_back();
        }
        out[b].push_back(m);
    }
    return out;
}

// Fill slot B's table with the next chunk of each member and enqueue the
// batch (server lock held).  Members are marked in flight even when a launch
// fails part-way: the slot's event still ends what was enqueued.
static lg_status launch_batch(lg_server *S, BatchSlot &B)
{
    const int n = (int)B.members.size();
    B.bufs.assign(n, 0);
    TableWriter T{B.host, B.dev};
    ChunkDesc *cd = T.descs();
    std::vector<int> all(n);
    for (int j = 0; j < n; ++j) {
        Req *q = B.members[j];
        const int32_t P = (int32_t)std::min<int64_t>(S->p.chunk_poses, q->r.n_poses - q->next_pose);
        const int buf = __builtin_ctz(~q->buf_busy);  // a free working-buffer copy (inflight < nbuf)
        fill_desc(S, q, P, buf, cd[j]);
        B.bufs[j] = buf;
        q->buf_busy |= 1u << buf;
        all[j] = j;
        q->next_pose += P;
        ++q->inflight;
    }
    auto blocks = [&](const std::vector<int> &who, auto per) {
        std::vector<uint32_t> nb;
        for (int m : who) nb.push_back((uint32_t)per(cd[m]));
        return nb;
    };
    // member lists of every stage, then one copy of the table
    struct Keyed {
        BatchLaunch b;
        int rep;  // a member: its field and parameters give the bucket
    };
    std::vector<Keyed> lq, lv, lr;
    BatchLaunch ld, pc, ps, sc, ss, la;
    lg_status st;
    auto one = [](const ChunkDesc &) { return 1u; };
    auto poses = [](const ChunkDesc &c) { return (uint32_t)c.P; };
    auto pose_chunks = [](const ChunkDesc &c) { return compact_blocks(c.P); };
    auto set_chunks = [](const ChunkDesc &c) { return compact_blocks((int64_t)c.P * c.D); };
    const int ncu = S->n_cu;
    auto lp_blocks = [ncu](const ChunkDesc &c) { return verdict_blocks((int64_t)c.P * c.D, ncu); };
    auto ik_blocks = [ncu](const ChunkDesc &c) { return realize_blocks((int64_t)c.P * c.D, c.H.F, ncu); };
    auto acc_blocks = [](const ChunkDesc &c) {
        return (uint32_t)std::max<int64_t>(1, std::min<int64_t>(64, ((int64_t)c.P * c.D + 4095) / 4096));
    };
    for (auto &g : buckets(all, [&](int m) { return (cd[m].H.W << 16) | (fm_bucket(cd[m].H.F) << 1) | cd[m].H.lat; })) {
        lq.push_back({BatchLaunch{}, g[0]});
        if ((st = T.list(g, blocks(g, poses), lq.back().b)) != LG_OK) return st;
    }
    if ((st = T.list(all, blocks(all, poses), ld)) != LG_OK) return st;
    if ((st = T.list(all, blocks(all, pose_chunks), pc)) != LG_OK) return st;
    if ((st = T.list(all, blocks(all, one), ps)) != LG_OK) return st;
    // verdict launches by contact-count class and by whether the cone has 8 edges
    for (auto &g : buckets(all, [&](int m) { return (km_bucket(cd[m].k) << 1) | (cd[m].m == 8 ? 1 : 0); })) {
        lv.push_back({BatchLaunch{}, g[0]});
        if ((st = T.list(g, blocks(g, lp_blocks), lv.back().b)) != LG_OK) return st;
    }
    if ((st = T.list(all, blocks(all, set_chunks), sc)) != LG_OK) return st;
    if ((st = T.list(all, blocks(all, one), ss)) != LG_OK) return st;
    std::vector<int> rz;
    for (int m : all)
        if (cd[m].realize) rz.push_back(m);
    auto max_dof = [&](int m) { return B.members[m]->r.field->max_dof; };
    for (auto &g : buckets(rz, [&](int m) { return dm_bucket(max_dof(m)); })) {
        lr.push_back({BatchLaunch{}, g[0]});
        if ((st = T.list(g, blocks(g, ik_blocks), lr.back().b)) != LG_OK) return st;
    }
    if ((st = T.list(all, blocks(all, acc_blocks), la)) != LG_OK) return st;
    size_t lds = 0;
    for (int m : all) lds = std::max(lds, draw_lds_bytes(cd[m].H.F, cd[m].N));
    LG_HIP(hipMemcpyAsync(B.dev, B.host, sizeof(ChunkDesc) * n, hipMemcpyHostToDevice, B.s));
    LG_HIP(hipMemcpyAsync(B.dev + TableWriter::kListBase, B.host + TableWriter::kListBase,
                          (size_t)T.n_lists * kListBytes, hipMemcpyHostToDevice, B.s));
    // the stages, in the order of the single-chunk path
    for (const Keyed &g : lq) {
        const DevHand &H = cd[g.rep].H;
        if ((st = query_batch(g.b, H.W, H.F, H.lat != 0, B.s)) != LG_OK) return st;
    }
    if ((st = draw_batch(ld, lds, B.s)) != LG_OK) return st;
    if ((st = compact_count_batch(pc, true, B.s)) != LG_OK) return st;
    if ((st = compact_scan_batch(ps, true, B.s)) != LG_OK) return st;
    if ((st = compact_scatter_batch(pc, true, B.s)) != LG_OK) return st;
    for (const Keyed &g : lv)
        if ((st = verdict_batch(g.b, cd[g.rep].k, cd[g.rep].m == 8, B.s)) != LG_OK) return st;
    if ((st = compact_count_batch(sc, false, B.s)) != LG_OK) return st;
    if ((st = compact_scan_batch(ss, false, B.s)) != LG_OK) return st;
    if ((st = compact_scatter_batch(sc, false, B.s)) != LG_OK) return st;
    for (const Keyed &g : lr)
        if ((st = realize_batch(g.b, max_dof(g.rep), B.s)) != LG_OK) return st;
    if (la.blocks) {
        hipLaunchKernelGGL(k_accumulate_batch, dim3(la.blocks), dim3(kAccThreads), 0, B.s, la.d, la.idx, la.first, la.n);
        LG_HIP(hipGetLastError());
    }
    return LG_OK;
}

static void finish(lg_server *S, Req *q, int32_t state)
{
    if (q->slot >= 0) {
        // Work of the request may still be queued on its stream when admit() or a
        // launch failed part-way (its event then does not cover it): drain the
        // stream before the block can be handed to another request.  After a
        // normal completion the last event fired and this returns at once.
        (void)hipStreamSynchronize(S->streams[q->slot]);
        char *base = S->slab.base + q->off;
        if (state == LG_REQ_DONE)
            (void)hipMemcpy(q->counters, base + q->L.counters, sizeof q->counters, hipMemcpyDeviceToHost);
        S->slab.release(q->off, q->L.total);
        S->free_slots.push_back(q->slot);
        q->slot = -1;
    }
    // the host copies are no longer read (the stream above has drained)
    std::vector<float>().swap(q->pts);
    std::vector<float>().swap(q->nrm);
    std::vector<float>().swap(q->poses);
    std::vector<float>().swap(q->sdf);
    q->state = state;
    q->t_done = S->now();
    if (state == LG_REQ_DONE) ++S->st.completed;
    if (state == LG_REQ_CANCELLED) ++S->st.cancelled;
    if (state == LG_REQ_FAILED) ++S->st.failed;
}

static lg_status admit(lg_server *S, Req *q)
{
    char *base = S->slab.base + q->off;
    hipStream_t s = S->streams[q->slot];
    const ReqLayout &L = q->L;
    const int64_t N = q->r.n_points;
    LG_HIP(hipMemcpyAsync(base + L.pts, q->pts.data(), 12 * N, hipMemcpyHostToDevice, s));
    LG_HIP(hipMemcpyAsync(base + L.nrm, q->nrm.data(), 12 * N, hipMemcpyHostToDevice, s));
    LG_HIP(hipMemcpyAsync(base + L.poses, q->poses.data(), 48 * (size_t)q->r.n_poses, hipMemcpyHostToDevice, s));
    const lg_status st = lg_chunk_bounds(reinterpret_cast<const float *>(base + L.pts), (int32_t)N,
                                         reinterpret_cast<float *>(base + L.bounds), s);
    if (st != LG_OK) return st;
    if (q->r.realize)
        LG_HIP(hipMemcpyAsync(base + L.sdf, q->sdf.data(), 4 * q->sdf.size(), hipMemcpyHostToDevice, s));
    LG_HIP(hipMemsetAsync(base + L.counters, 0, 24, s));
    if (q->batched) {  // the first batch with this request waits for these copies
        LG_HIP(hipEventRecord(q->ev, s));
        q->fresh = true;
    }
    return LG_OK;
}

// free the server's device resources (streams, events, tables, slab)
static void release(lg_server *S)
{
    for (auto s : S->streams) (void)hipStreamDestroy(s);
    for (auto e : S->events) (void)hipEventDestroy(e);
    S->streams.clear();
    S->events.clear();
    for (BatchSlot &B : S->batch) {
        if (B.s) (void)hipStreamDestroy(B.s);
        if (B.ev) (void)hipEventDestroy(B.ev);
        if (B.dev) (void)hipFree(B.dev);
        if (B.host) (void)hipHostFree(B.host);
    }
    S->batch.clear();
    if (S->slab.base) (void)hipFree(S->slab.base);
    S->slab.base = nullptr;
}

static void worker_loop(lg_server *S)
{
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    while (true) {
        bool progressed = false;
        // completions: batches, then requests
        for (BatchSlot &B : S->batch) {
            if (B.busy && hipEventQuery(B.ev) == hipSuccess) {
                for (size_t j = 0; j < B.members.size(); ++j) {
                    --B.members[j]->inflight;
                    B.members[j]->buf_busy &= ~(1u << B.bufs[j]);
                }
                B.members.clear();
                B.busy = false;
                progressed = true;
            }
        }
        for (size_t i = 0; i < S->active.size();) {
            Req *q = S->active[i];
            if (q->inflight && !q->batched && hipEventQuery(q->ev) == hipSuccess) {
                q->inflight = 0;
                progressed = true;
            }
            if (!q->inflight && (q->cancel || q->next_pose >= q->r.n_poses || q->status != LG_OK)) {
                finish(S, q, q->status != LG_OK ? LG_REQ_FAILED : (q->cancel ? LG_REQ_CANCELLED : LG_REQ_DONE));
                S->active.erase(S->active.begin() + i);
                S->st.active = (int32_t)S->active.size();
                S->cv.notify_all();
                progressed = true;
                continue;
            }
            ++i;
        }
        if (S->stop && S->active.empty()) break;
        // admission, FIFO: the head waits until its block fits
        while (!S->stop && !S->queued.empty() && !S->free_slots.empty()) {
            Req *q = S->queued.front();
            uint64_t off = 0;
            if (!S->slab.alloc(q->L.total, off)) break;
            S->queued.pop_front();
            q->off = off;
            q->slot = S->free_slots.back();
            S->free_slots.pop_back();
            q->ev = S->events[q->slot];
            q->batched = batched_request(S->p, q->r);
            q->state = LG_REQ_RUNNING;
            q->t_admit = S->now();
            lg_status st = admit(S, q);
            if (st != LG_OK) q->status = st;
            S->active.push_back(q);
            ++S->st.admitted;
            S->st.queued = (int32_t)S->queued.size();
            S->st.active = (int32_t)S->active.size();
            S->st.peak_bytes = std::max<uint64_t>(S->st.peak_bytes, S->slab.used());
            progressed = true;
        }
        // one chunk per idle active request: on the request's own stream, or
        // in a batch (batched requests, when a batch slot is free)
        std::vector<Req *> idle;
        for (Req *q : S->active) {
            if (q->cancel || q->status != LG_OK || q->next_pose >= q->r.n_poses) continue;
            if (q->batched) {
                if (q->inflight >= q->L.nbuf) continue;
                // a request joins a batch once its admission copies are done, so
                // that no batch waits for another request's upload
                if (q->fresh) {
                    if (hipEventQuery(q->ev) != hipSuccess) continue;
                    q->fresh = false;
                }
                idle.push_back(q);
                continue;
            }
            if (q->inflight) continue;
            lg_status st = launch_chunk(S, q);
            if (st != LG_OK) q->status = st;
            progressed = true;
        }
        std::vector<BatchSlot *> free_slots;
        for (BatchSlot &B : S->batch)
            if (!B.busy) free_slots.push_back(&B);
        if (!idle.empty() && !free_slots.empty()) {
            // Idle chunks in ascending size (poses x points), cut into as many
            // batches as there are free slots, of about equal size: small
            // chunks share a batch instead of waiting behind large ones.
            auto work = [&](const Req *q) {
                return (double)std::min<int64_t>(S->p.chunk_poses, q->r.n_poses - q->next_pose) * q->r.n_points;
            };
            std::stable_sort(idle.begin(), idle.end(), [&](const Req *x, const Req *y) { return work(x) < work(y); });
            double total = 0;
            for (const Req *q : idle) total += work(q);
            const size_t nb = std::min(free_slots.size(), idle.size());
            size_t b = 0;
            double acc = 0;
            for (Req *q : idle) {
                BatchSlot *B = free_slots[b];
                B->members.push_back(q);
                acc += work(q);
                if (b + 1 < nb && acc >= total * (double)(b + 1) / (double)nb) ++b;
            }
            for (size_t i = 0; i < nb; ++i) {
                BatchSlot *B = free_slots[i];
                if (B->members.empty()) continue;
                const lg_status st = launch_batch(S, *B);
                if (st != LG_OK)
                    for (Req *q : B->members) q->status = st;
                // the event ends whatever was enqueued, also after a failure
                if (hipEventRecord(B->ev, B->s) != hipSuccess) (void)hipStreamSynchronize(B->s);
                B->busy = true;
                ++S->st.batches;
                S->st.batched_chunks += (int64_t)B->members.size();
                progressed = true;
            }
        }
        S->st.bytes_in_use = S->slab.used();
        if (!progressed) {
            S->cv.wait_for(lk, std::chrono::microseconds(S->active.empty() ? 2000 : 50));
        } else {
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        }
    }
}

}  // namespace lg

using namespace lg;

extern "C" {

uint64_t lg_serve_request_bytes(const lg_server_params *params, const lg_request *req)
{
    if (!params || !req || !req->field || params->chunk_poses <= 0) return 0;
    return layout_of(*params, *req).total;
}

lg_status lg_serve_create(const lg_server_params *params, lg_server **out)
{
    if (!params || !out) return fail(LG_EINVAL, "null params or out");
    if (params->max_active < 1 || params->max_active > kMaxBatch || params->chunk_poses < 1 ||
        params->budget_bytes < kAlign || params->batch_slots < 0 || params->batch_slots > kMaxBatchSlots)
        return fail(LG_EINVAL, "need 1 <= max_active <= 64, chunk_poses >= 1, budget >= 256 B, 0 <= batch_slots <= 8");
    auto S = std::make_unique<lg_server>();
    S->p = *params;
    S->t0 = std::chrono::steady_clock::now();
    // device resources; what was made before a failure is freed again
    auto init = [&]() -> lg_status {
        LG_HIP(hipGetDevice(&S->device));
        void *slab = nullptr;
        LG_HIP(hipMalloc(&slab, params->budget_bytes));
        S->slab.base = static_cast<char *>(slab);
        S->slab.reset(params->budget_bytes);
        S->st.budget_bytes = params->budget_bytes;
        for (int i = 0; i < params->max_active; ++i) {
            hipStream_t s;
            hipEvent_t e;
            LG_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
            S->streams.push_back(s);
            LG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            S->events.push_back(e);
            S->free_slots.push_back(params->max_active - 1 - i);
        }
        if (params->batched) {
            LG_HIP(hipDeviceGetAttribute(&S->n_cu, hipDeviceAttributeMultiprocessorCount, S->device));
            S->batch.resize(params->batch_slots > 0 ? params->batch_slots : 4);
            for (BatchSlot &B : S->batch) {
                LG_HIP(hipStreamCreateWithFlags(&B.s, hipStreamNonBlocking));
                LG_HIP(hipEventCreateWithFlags(&B.ev, hipEventDisableTiming));
                LG_HIP(hipMalloc(&B.dev, kTableBytes));
                LG_HIP(hipHostMalloc(&B.host, kTableBytes, hipHostMallocDefault));
            }
        }
        return LG_OK;
    };
    const lg_status st = init();
    if (st != LG_OK) {
        release(S.get());
        return st;
    }
    lg_server *raw = S.release();
    raw->worker = std::thread(worker_loop, raw);
    *out = raw;
    return LG_OK;
}

lg_status lg_serve_submit(lg_server *S, const lg_request *r, uint64_t *ticket)
{
    if (!S || !ticket) return fail(LG_EINVAL, "null server or ticket");
    lg_status st = validate_request(S->p, r);
    if (st != LG_OK) return st;
    auto q = std::make_unique<Req>();
    q->r = *r;
    q->L = layout_of(S->p, *r);
    const int64_t N = r->n_points;
    q->pts.resize(3 * N);
    q->nrm.resize(3 * N);
    for (int64_t i = 0; i < N; ++i)
        for (int a = 0; a < 3; ++a) {
            q->pts[a * N + i] = r->pts[3 * i + a];
            q->nrm[a * N + i] = r->nrm[3 * i + a];
        }
    q->poses.assign(r->poses, r->poses + 12 * (size_t)r->n_poses);
    if (r->realize) {
        const size_t G = r->sdf_dims;
        q->sdf.assign(r->sdf_values, r->sdf_values + G * G * G);
    }
    q->r.pts = q->r.nrm = q->r.poses = q->r.sdf_values = nullptr;  // host copies live in q
    std::lock_guard<std::mutex> lk(S->mu);
    ++S->st.submitted;
    if (q->L.total > S->p.budget_bytes) {
        ++S->st.rejected;
        return fail(LG_EBUDGET, "request needs more device memory than the server's budget");
    }
    q->ticket = S->next_ticket++;
    q->t_submit = S->now();
    *ticket = q->ticket;
    S->queued.push_back(q.get());
    S->all.emplace(q->ticket, std::move(q));
    S->st.queued = (int32_t)S->queued.size();
    S->cv.notify_all();
    return LG_OK;
}

static void fill_result(const Req *q, lg_result *o)
{
    o->state = q->state;
    o->status = q->status;
    o->n_acc = (int64_t)q->counters[0];
    o->n_valid = (int64_t)q->counters[1];
    o->acc_hash = q->counters[2];
    o->t_submit = q->t_submit;
    o->t_admit = q->t_admit;
    o->t_done = q->t_done;
    o->bytes = q->L.total;
}

lg_status lg_serve_poll(lg_server *S, uint64_t ticket, lg_result *out)
{
    if (!S || !out) return fail(LG_EINVAL, "null server or out");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return fail(LG_EINVAL, "unknown ticket");
    fill_result(it->second.get(), out);
    return LG_OK;
}

lg_status lg_serve_wait(lg_server *S, uint64_t ticket, double timeout_s, lg_result *out)
{
    if (!S || !out) return fail(LG_EINVAL, "null server or out");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return fail(LG_EINVAL, "unknown ticket");
    Req *q = it->second.get();
    const auto deadline = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s);
    while (q->state == LG_REQ_QUEUED || q->state == LG_REQ_RUNNING) {
        if (S->cv.wait_until(lk, deadline) == std::cv_status::timeout) break;
    }
    fill_result(q, out);
    return LG_OK;
}

lg_status lg_serve_cancel(lg_server *S, uint64_t ticket)
{
    if (!S) return fail(LG_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return fail(LG_EINVAL, "unknown ticket");
    Req *q = it->second.get();
    if (q->state == LG_REQ_QUEUED) {
        S->queued.erase(std::find(S->queued.begin(), S->queued.end(), q));
        S->st.queued = (int32_t)S->queued.size();
        finish(S, q, LG_REQ_CANCELLED);
        S->cv.notify_all();
    } else if (q->state == LG_REQ_RUNNING) {
        q->cancel = true;
    }
    return LG_OK;
}

lg_status lg_serve_stats(lg_server *S, lg_server_stats *out)
{
    if (!S || !out) return fail(LG_EINVAL, "null server or out");
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->st;
    out->bytes_in_use = S->slab.used();
    return LG_OK;
}

double lg_serve_clock(lg_server *S) { return S ? S->now() : 0.0; }

lg_status lg_serve_destroy(lg_server *S)
{
    if (!S) return LG_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        for (Req *q : S->queued) finish(S, q, LG_REQ_CANCELLED);
        S->queued.clear();
        for (Req *q : S->active) q->cancel = true;
        S->cv.notify_all();
    }
    if (S->worker.joinable()) S->worker.join();
    release(S);
    delete S;
    return LG_OK;
}

}  // extern "C"
