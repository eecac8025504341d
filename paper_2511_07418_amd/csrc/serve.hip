// Serving: continuous batching of grasp requests over resident contact fields.
//
// The paper builds a field once per hand and caches stage outputs for later
// forward passes (Fig. 6, Sec. 5.7).  A server keeps the fields resident and
// runs many requests' searches on one GPU at once:
//  * admission: one device slab of `budget_bytes` is sub-allocated first-fit;
//    a request is admitted (FIFO) when its inputs and one chunk of working
//    buffers fit, and its block is returned when it completes;
//  * interleaving: every admitted request owns a stream (default priority);
//    the server thread enqueues one chunk of `chunk_poses` poses per request
//    at a time (query -> draws/verdicts/compaction -> optional IK +
//    penetration -> counters), so chunks of different requests overlap on the
//    device and a long request never blocks a short one behind it;
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

static uint64_t align_up(uint64_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// splitmix64 finaliser (Steele, Lea, Flood 2014) of (request, set id)
__device__ inline uint64_t mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// counters[0] += n_acc, counters[1] += valid, counters[2] += sum of mix64(id)
__global__ void k_serve_accumulate(const int32_t *__restrict__ acc_list, const int32_t *__restrict__ n_acc_dev,
                                   const uint8_t *__restrict__ valid, int64_t set_base, uint32_t request_id,
                                   unsigned long long *__restrict__ counters)
{
    const int n = *n_acc_dev;
    unsigned long long c = 0, v = 0, h = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
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

// Sizes of one request's device buffers (inputs + one chunk of work).
struct ReqLayout {
    uint64_t pts, nrm, bounds, poses, sdf, dom_bits, dom_count, set_pt, set_link, verdict, tstar, acc, n_acc, ws;
    uint64_t q, err, ang, depth, valid, counters, total;
};

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
    L.dom_bits = take(4 * (uint64_t)(chunk * F * NW));
    L.dom_count = take(4 * (uint64_t)(chunk * F));
    L.set_pt = take(4 * (uint64_t)(sets * k));
    L.set_link = take((uint64_t)(sets * k));
    L.verdict = take((uint64_t)sets);
    L.tstar = take(8 * (uint64_t)sets);
    L.acc = take(4 * (uint64_t)sets);
    L.n_acc = take(4);
    lg_search_params p = r.search;
    L.ws = take(lg_search_workspace_bytes((int32_t)N, (int32_t)chunk, &p));
    const int64_t ra = r.realize ? sets : 0;
    L.q = take(4 * (uint64_t)(ra * J));
    L.err = take(4 * (uint64_t)(ra * k));
    L.ang = take(4 * (uint64_t)(ra * k));
    L.depth = take(4 * (uint64_t)ra);
    L.valid = take((uint64_t)ra);
    L.counters = take(3 * 8);
    L.total = off;
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
    bool cancel = false, in_flight = false;
    int64_t next_pose = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    unsigned long long counters[3] = {0, 0, 0};
    hipEvent_t ev = nullptr;
};

}  // namespace lg

struct lg_server {
    lg_server_params p{};
    int device = 0;
    lg::Slab slab;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    std::vector<int> free_slots;
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
    if (r->realize && (!r->sdf_values || r->sdf_dims < 2 || !(r->sdf_h > 0.f) || !(r->ik.lambda > 0.f)))
        return fail(LG_EINVAL, "realize needs an SDF and IK parameters");
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
                   n_acc, base + L.ws, L.q - L.ws, s);
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
    q->in_flight = true;
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
    return LG_OK;
}

static void worker_loop(lg_server *S)
{
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    while (true) {
        bool progressed = false;
        // completions
        for (size_t i = 0; i < S->active.size();) {
            Req *q = S->active[i];
            if (q->in_flight && hipEventQuery(q->ev) == hipSuccess) {
                q->in_flight = false;
                progressed = true;
            }
            if (!q->in_flight && (q->cancel || q->next_pose >= q->r.n_poses || q->status != LG_OK)) {
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
        // one chunk per idle active request, round-robin by admission order
        for (Req *q : S->active) {
            if (q->in_flight || q->cancel || q->status != LG_OK || q->next_pose >= q->r.n_poses) continue;
            lg_status st = launch_chunk(S, q);
            if (st != LG_OK) q->status = st;
            progressed = true;
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
    if (params->max_active < 1 || params->max_active > 64 || params->chunk_poses < 1 || params->budget_bytes < kAlign)
        return fail(LG_EINVAL, "need 1 <= max_active <= 64, chunk_poses >= 1, budget >= 256 B");
    auto S = std::make_unique<lg_server>();
    S->p = *params;
    S->t0 = std::chrono::steady_clock::now();
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
        LG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        S->streams.push_back(s);
        S->events.push_back(e);
        S->free_slots.push_back(params->max_active - 1 - i);
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
    for (auto s : S->streams) (void)hipStreamDestroy(s);
    for (auto e : S->events) (void)hipEventDestroy(e);
    (void)hipFree(S->slab.base);
    delete S;
    return LG_OK;
}

}  // extern "C"
