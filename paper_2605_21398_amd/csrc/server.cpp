// Serving loop: registrations are submitted from any thread, admitted in
// arrival order as device memory and worker slots free up, and run
// concurrently on one HIP stream per slot, so the work of requests that
// arrive while others are on the GPU overlaps on the device (continuous
// batching).  Object spectra stay resident in a cache keyed by the mesh's
// contents (a 64-bit hash, confirmed byte for byte on a hit), the canvas and
// the object-grid thresholds.  In serial mode a single slot gives the plain
// one-request-at-a-time path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "regdock.h"
#include "runtime.h"

namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

thread_local std::string t_err;

int sfail(int code, const std::string& msg) {
    t_err = msg;
    return code;
}

// FNV-1a over a byte range, continuing from h
uint64_t fnv1a(const void* p, size_t n, uint64_t h) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

// the mesh of a request, kept by the cache to confirm a hash hit exactly
struct MeshBytes {
    std::vector<float> vertices;
    std::vector<int32_t> faces;
    std::vector<uint8_t> touchable;
    uint64_t hash = 0;
    bool same(const MeshBytes& o) const {
        return hash == o.hash && vertices == o.vertices && faces == o.faces && touchable == o.touchable;
    }
};

// a request's inputs, copied at submission
struct Job {
    reg_ticket ticket = 0;
    std::shared_ptr<MeshBytes> mesh;
    std::vector<float> poses, so3;
    int64_t object_id = -1;
    reg_probe probe{};
    reg_grid_spec grid{};
    reg_params params{};
    int32_t top_k = 16, refine = 1;
    size_t footprint = 0, object_part = 0;
    bool done = false;
    reg_result result{};
};

// mesh hash, canvas edge, voxel size and the object-grid thresholds
using ObjKey = std::tuple<uint64_t, int, double, double, double, double>;

struct CacheEntry {
    ObjKey key;
    std::shared_ptr<const MeshBytes> mesh;
    std::shared_ptr<ObjectData> obj;
};

}  // namespace

struct reg_server {
    reg_server_cfg cfg{};
    std::mutex mu;
    std::condition_variable cv_dispatch, cv_done, cv_work;
    std::deque<std::shared_ptr<Job>> queue;
    std::map<reg_ticket, std::shared_ptr<Job>> jobs;
    std::vector<std::shared_ptr<Job>> slot_job;  // per worker: assigned job or null
    std::vector<std::thread> workers;
    std::thread dispatcher;
    std::vector<hipStream_t> streams;
    bool stopping = false;
    reg_ticket next_ticket = 1;
    size_t in_use = 0;
    int64_t n_done = 0, hits = 0, misses = 0;
    // object cache, least recently used first
    std::mutex cache_mu;
    std::list<CacheEntry> cache;
    size_t cache_bytes = 0;

    std::shared_ptr<ObjectData> cache_get(const ObjKey& k, const MeshBytes& mesh) {
        std::lock_guard<std::mutex> lk(cache_mu);
        for (auto it = cache.begin(); it != cache.end(); ++it)
            if (it->key == k && it->mesh->same(mesh)) {
                cache.splice(cache.end(), cache, it);
                ++hits;
                return it->obj;
            }
        ++misses;
        return nullptr;
    }
    // An object is published once its build is queued: its ready event orders
    // every later user's stream after the build.
    void cache_put(const ObjKey& k, std::shared_ptr<const MeshBytes> mesh, std::shared_ptr<ObjectData> o) {
        std::lock_guard<std::mutex> lk(cache_mu);
        for (auto& e : cache)
            if (e.key == k && e.mesh->same(*mesh)) return;
        cache_bytes += regdock_rt::object_bytes(o.get());
        cache.push_back(CacheEntry{k, std::move(mesh), std::move(o)});
        // evict least recently used objects no registration holds any more
        for (auto it = cache.begin(); it != cache.end() && cache_bytes > (size_t)cfg.cache_bytes;) {
            if (it->obj.use_count() == 1) {
                cache_bytes -= regdock_rt::object_bytes(it->obj.get());
                it = cache.erase(it);
            } else {
                ++it;
            }
        }
    }

    void run_fake(Job& j) {
        // test executor: no device work, a duration proportional to the rotations
        const double us = cfg.fake_us_per_rotation * j.so3.size() / 4.0;
        std::this_thread::sleep_for(std::chrono::microseconds((int64_t)us));
        j.result.status = REG_OK;
        j.result.n_top = std::min<int32_t>(j.top_k, (int32_t)(j.so3.size() / 4));
        j.result.best_score = (float)(j.so3.size() / 4);
    }

    int run_gpu(Job& j, hipStream_t s);
    void worker_loop(int w);
    void dispatch_loop();
};

// One registration on the worker's stream: stage the inputs, build (or take
// from the cache) the object, score every rotation, take the top K and refine.
int reg_server::run_gpu(Job& j, hipStream_t s) {
    const MeshBytes& mb = *j.mesh;
    const int32_t nv = (int32_t)(mb.vertices.size() / 3), nf = (int32_t)(mb.faces.size() / 3);
    const int32_t N = (int32_t)(j.poses.size() / 7), M = (int32_t)(j.so3.size() / 4);
    std::vector<void*> dev;
    struct Free {
        std::vector<void*>& d;
        hipStream_t s;
        ~Free() {
            (void)hipStreamSynchronize(s);
            for (void* p : d) regdock_rt::dev_release(p);
        }
    } fr{dev, s};
    auto dalloc = [&](size_t bytes) -> void* {
        void* p = nullptr;
        if (regdock_rt::dev_alloc(&p, bytes ? bytes : 1) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        dev.push_back(p);
        return p;
    };
    float* dV = (float*)dalloc(mb.vertices.size() * 4);
    int32_t* dF = (int32_t*)dalloc(mb.faces.size() * 4);
    uint8_t* dT = mb.touchable.empty() ? nullptr : (uint8_t*)dalloc(mb.touchable.size());
    float* dP = (float*)dalloc(j.poses.size() * 4);
    float* dQ = (float*)dalloc(j.so3.size() * 4);
    float* dS = (float*)dalloc((size_t)M * 4);
    double* dPose = (double*)dalloc((size_t)M * 56);
    const int K = std::max(1, std::min(j.top_k, std::min<int32_t>(16, M)));
    int32_t* dTop = (int32_t*)dalloc((size_t)K * 4);
    double* dInit = (double*)dalloc((size_t)K * 56);
    double* dOut = (double*)dalloc((size_t)K * 56);
    double* dJ = (double*)dalloc((size_t)K * 8);
    if (!dV || !dF || (!dT && !mb.touchable.empty()) || !dP || !dQ || !dS || !dPose || !dTop || !dInit || !dOut || !dJ)
        return sfail(REG_ENOMEM, "device staging allocation failed");
    auto up = [&](void* d, const void* hsrc, size_t bytes) {
        return hipMemcpyAsync(d, hsrc, bytes, hipMemcpyHostToDevice, s) == hipSuccess;
    };
    if (!up(dV, mb.vertices.data(), mb.vertices.size() * 4) || !up(dF, mb.faces.data(), mb.faces.size() * 4) ||
        (dT && !up(dT, mb.touchable.data(), mb.touchable.size())) || !up(dP, j.poses.data(), j.poses.size() * 4) ||
        !up(dQ, j.so3.data(), j.so3.size() * 4))
        return sfail(REG_EDEVICE, "staging copy failed");

    const ObjKey key{mb.hash, j.grid.n, j.grid.h_mm, j.params.tau_out1, j.params.tau_in1, j.params.rho};
    std::shared_ptr<ObjectData> cached = j.object_id >= 0 ? cache_get(key, mb) : nullptr;
    reg_mesh mesh{dV, nv, dF, nf, dT};
    reg_handle* h = nullptr;
    int rc = regdock_rt::init_shared(&mesh, &j.probe, dP, N, dQ, M, &j.grid, &j.params, (void*)s, cached, &h);
    if (rc) return sfail(rc, regdock_rt::last_error());
    struct HFree {
        reg_handle* h;
        ~HFree() { register_free(h); }
    } hf{h};
    if (!cached && j.object_id >= 0) cache_put(key, j.mesh, regdock_rt::object_of(h));

    rc = score_rotations(h, 0, M, dS, nullptr, dPose);
    if (rc) return sfail(rc, regdock_rt::last_error());
    rc = register_top_k(h, dS, M, K, dTop);
    if (rc) return sfail(rc, regdock_rt::last_error());
    std::vector<int32_t> top(K);
    std::vector<float> sc(M);
    std::vector<double> pose((size_t)M * 7);
    if (hipMemcpyAsync(top.data(), dTop, K * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(sc.data(), dS, (size_t)M * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(pose.data(), dPose, (size_t)M * 56, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return sfail(REG_EDEVICE, "result copy failed");
    reg_result& r = j.result;
    r.n_top = K;
    for (int k = 0; k < K; ++k) {
        r.top_rot[k] = top[k];
        r.top_score[k] = sc[top[k]];
        for (int c = 0; c < 7; ++c) r.top_pose[7 * k + c] = pose[(size_t)top[k] * 7 + c];
    }
    r.best_score = r.top_score[0];
    for (int c = 0; c < 7; ++c) r.best_pose[c] = r.top_pose[c];
    r.best_J = 0.0;
    if (j.refine) {
        if (hipMemcpyAsync(dInit, r.top_pose, (size_t)K * 56, hipMemcpyHostToDevice, s) != hipSuccess)
            return sfail(REG_EDEVICE, "start copy failed");
        rc = j.refine == 2 ? refine_se3_lbfgsb(h, dInit, K, dOut, dJ, nullptr) : refine_se3(h, dInit, K, dOut, dJ, nullptr);
        if (rc) return sfail(rc, regdock_rt::last_error());
        if (hipMemcpyAsync(r.refined_pose, dOut, (size_t)K * 56, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(r.refined_J, dJ, (size_t)K * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return sfail(REG_EDEVICE, "refinement copy failed");
        int best = 0;
        for (int k = 1; k < K; ++k)
            if (r.refined_J[k] < r.refined_J[best]) best = k;
        r.best_J = r.refined_J[best];
        for (int c = 0; c < 7; ++c) r.best_pose[c] = r.refined_pose[7 * best + c];
    }
    return REG_OK;
}

void reg_server::worker_loop(int w) {
    for (;;) {
        std::shared_ptr<Job> j;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return stopping || slot_job[w] != nullptr; });
            if (!slot_job[w]) return;  // stopping with nothing assigned
            j = slot_job[w];
        }
        j->result.t_start_ns = now_ns();
        int rc = REG_OK;
        if (cfg.fake) {
            run_fake(*j);
        } else {
            rc = run_gpu(*j, streams[w]);
        }
        j->result.t_end_ns = now_ns();
        {
            std::lock_guard<std::mutex> lk(mu);
            j->result.status = rc;
            if (rc) std::snprintf(j->result.error, sizeof j->result.error, "%s", t_err.c_str());
            j->done = true;
            in_use -= j->footprint;
            slot_job[w] = nullptr;
            ++n_done;
        }
        cv_done.notify_all();
        cv_dispatch.notify_all();
    }
}

// Admission in arrival order: the head of the queue starts when a slot is free
// and its footprint fits beside the registrations in flight.
void reg_server::dispatch_loop() {
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        cv_dispatch.wait(lk, [&] {
            if (stopping) return true;
            if (queue.empty()) return false;
            const bool slot = std::find(slot_job.begin(), slot_job.end(), nullptr) != slot_job.end();
            return slot && in_use + queue.front()->footprint <= (size_t)cfg.hbm_budget_bytes;
        });
        if (stopping) return;
        std::shared_ptr<Job> j = queue.front();
        queue.pop_front();
        const int w = (int)(std::find(slot_job.begin(), slot_job.end(), nullptr) - slot_job.begin());
        in_use += j->footprint;
        j->result.t_admit_ns = now_ns();
        slot_job[w] = j;
        cv_work.notify_all();
    }
}

extern "C" {

const char* register_server_last_error(void) { return t_err.c_str(); }

int register_server_create(const reg_server_cfg* cfg, reg_server** out) {
    if (!out) return sfail(REG_EINVAL, "out is NULL");
    *out = nullptr;
    auto srv = std::make_unique<reg_server>();
    if (cfg) srv->cfg = *cfg;
    reg_server_cfg& c = srv->cfg;
    if (c.max_inflight <= 0) c.max_inflight = 4;
    if (c.mode == 1) c.max_inflight = 1;
    if (c.max_inflight > 64) return sfail(REG_EINVAL, "max_inflight must be <= 64");
    if (c.cache_bytes <= 0) c.cache_bytes = (int64_t)4 << 30;
    if (c.hbm_budget_bytes <= 0) {
        if (c.fake) {
            c.hbm_budget_bytes = (int64_t)64 << 30;
        } else {
            size_t fr = 0, tot = 0;
            if (hipMemGetInfo(&fr, &tot) != hipSuccess) return sfail(REG_EDEVICE, "hipMemGetInfo failed");
            c.hbm_budget_bytes = (int64_t)(fr / 4 * 3) - c.cache_bytes;
            if (c.hbm_budget_bytes <= 0) return sfail(REG_ENOMEM, "no device memory left for registrations");
        }
    }
    if (!c.fake) {
        srv->streams.resize(c.max_inflight, nullptr);
        for (auto& s : srv->streams)
            if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
                for (auto& t : srv->streams)
                    if (t) (void)hipStreamDestroy(t);
                return sfail(REG_EDEVICE, "hipStreamCreate failed");
            }
    }
    srv->slot_job.resize(c.max_inflight);
    reg_server* s = srv.get();
    for (int w = 0; w < c.max_inflight; ++w) s->workers.emplace_back([s, w] { s->worker_loop(w); });
    s->dispatcher = std::thread([s] { s->dispatch_loop(); });
    *out = srv.release();
    return REG_OK;
}

void register_server_destroy(reg_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (auto& j : s->queue) {
            j->result.status = REG_ECANCELED;
            std::snprintf(j->result.error, sizeof j->result.error, "server destroyed before admission");
            j->done = true;
        }
        s->queue.clear();
        s->stopping = true;
    }
    s->cv_dispatch.notify_all();
    s->dispatcher.join();
    s->cv_work.notify_all();
    for (auto& t : s->workers) t.join();  // running registrations finish first
    s->cv_done.notify_all();
    for (auto& st : s->streams) (void)hipStreamDestroy(st);
    s->cache.clear();
    delete s;
}

int register_submit(reg_server* s, const reg_request* rq, reg_ticket* out) {
    if (!s || !rq || !out) return sfail(REG_EINVAL, "NULL argument");
    const reg_mesh& m = rq->mesh;
    if (!m.vertices || !m.faces || m.n_vertices < 3 || m.n_faces < 1 || !rq->poses || rq->n_poses < 1 || !rq->so3 ||
        rq->n_rot < 1)
        return sfail(REG_EINVAL, "request needs a mesh, >= 1 pose and >= 1 rotation");
    if (rq->top_k < 0 || rq->top_k > 16) return sfail(REG_EINVAL, "top_k must be in [0, 16]");
    if (rq->refine < 0 || rq->refine > 2) return sfail(REG_EINVAL, "refine must be 0, 1 or 2");
    auto j = std::make_shared<Job>();
    auto mesh = std::make_shared<MeshBytes>();
    mesh->vertices.assign(m.vertices, m.vertices + 3 * (size_t)m.n_vertices);
    mesh->faces.assign(m.faces, m.faces + 3 * (size_t)m.n_faces);
    if (m.touchable) mesh->touchable.assign(m.touchable, m.touchable + (size_t)m.n_faces);
    {
        uint64_t hh = 0xcbf29ce484222325ull;
        const int64_t sizes[3] = {m.n_vertices, m.n_faces, m.touchable ? 1 : 0};
        hh = fnv1a(sizes, sizeof sizes, hh);
        hh = fnv1a(mesh->vertices.data(), mesh->vertices.size() * 4, hh);
        hh = fnv1a(mesh->faces.data(), mesh->faces.size() * 4, hh);
        hh = fnv1a(mesh->touchable.data(), mesh->touchable.size(), hh);
        mesh->hash = hh;
    }
    j->mesh = std::move(mesh);
    j->poses.assign(rq->poses, rq->poses + 7 * (size_t)rq->n_poses);
    j->so3.assign(rq->so3, rq->so3 + 4 * (size_t)rq->n_rot);
    j->object_id = rq->object_id;
    j->probe = rq->probe;
    j->grid = rq->grid;
    j->params = rq->params;
    // the thresholds that key the object cache take their defaults here
    if (j->params.tau_out1 <= 0) j->params.tau_out1 = 0.5;
    if (j->params.tau_in1 <= 0) j->params.tau_in1 = 0.2;
    if (j->params.rho <= 0) j->params.rho = 50.0;
    j->top_k = rq->top_k > 0 ? rq->top_k : 16;
    j->refine = rq->refine;
    const int batch = j->params.batch > 0 ? (j->params.batch + 7) / 8 * 8
                                          : regdock_rt::default_batch_for(rq->grid.n, rq->n_rot);
    const auto fp = regdock_rt::footprint(rq->grid.n, rq->n_rot, rq->n_poses, m.n_vertices, m.n_faces, batch,
                                          rq->refine ? j->top_k : 0);
    const size_t staging = j->mesh->vertices.size() * 4 + j->mesh->faces.size() * 4 + j->mesh->touchable.size() + j->poses.size() * 4 +
                           j->so3.size() * 4 + (size_t)rq->n_rot * 60 + 16 * 200;
    j->object_part = fp.object;
    j->footprint = fp.request + fp.object + staging;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) return sfail(REG_ECANCELED, "server is stopping");
    if (j->footprint > (size_t)s->cfg.hbm_budget_bytes)
        return sfail(REG_EBUSY, "request needs " + std::to_string(j->footprint) + " device bytes, more than the budget");
    j->ticket = s->next_ticket++;
    j->result.t_submit_ns = now_ns();
    j->result.footprint_bytes = (int64_t)j->footprint;
    s->jobs[j->ticket] = j;
    s->queue.push_back(j);
    *out = j->ticket;
    s->cv_dispatch.notify_all();
    return REG_OK;
}

static int take_result(reg_server* s, reg_ticket t, reg_result* out, std::unique_lock<std::mutex>& lk,
                       int64_t timeout_ms) {
    auto it = s->jobs.find(t);
    if (it == s->jobs.end()) return sfail(REG_EINVAL, "unknown ticket");
    std::shared_ptr<Job> j = it->second;
    if (timeout_ms != 0 && !j->done) {
        auto ready = [&] { return j->done; };
        if (timeout_ms < 0) s->cv_done.wait(lk, ready);
        else s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready);
    }
    if (!j->done) return REG_EAGAIN;
    if (out) *out = j->result;
    s->jobs.erase(t);
    return j->result.status == REG_OK ? REG_OK : sfail(j->result.status, j->result.error);
}

int register_poll(reg_server* s, reg_ticket t, reg_result* out) {
    if (!s) return sfail(REG_EINVAL, "NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    return take_result(s, t, out, lk, 0);
}

int register_wait(reg_server* s, reg_ticket t, int64_t timeout_ms, reg_result* out) {
    if (!s) return sfail(REG_EINVAL, "NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    return take_result(s, t, out, lk, timeout_ms);
}

int register_server_stats(reg_server* s, reg_server_stats* out) {
    if (!s || !out) return sfail(REG_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    out->queued = (int64_t)s->queue.size();
    out->running = (int64_t)std::count_if(s->slot_job.begin(), s->slot_job.end(), [](auto& j) { return j != nullptr; });
    out->done = s->n_done;
    out->in_use_bytes = (int64_t)s->in_use;
    out->budget_bytes = s->cfg.hbm_budget_bytes;
    {
        std::lock_guard<std::mutex> lc(s->cache_mu);
        out->cache_hits = s->hits;
        out->cache_misses = s->misses;
        out->cache_bytes = (int64_t)s->cache_bytes;
        out->cached_objects = (int64_t)s->cache.size();
    }
    return REG_OK;
}

}  // extern "C"
