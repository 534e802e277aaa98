// Serving loop: registrations are submitted from any thread and admitted in
// arrival order as device memory and worker slots free up.
//
// Serial mode (one slot) is the plain path: each registration runs whole on
// one stream, one after the other.
//
// Continuous mode splits each admitted registration into work items.  Its
// worker thread stages the inputs and builds the handle (object grid and
// spectrum, or the cached object; swept lattice) on the worker's stream; a
// scheduler thread then issues the registration's rotation batches (three
// search passes and candidate selection each) onto two shared search
// streams, always taking the next batch of the admitted registration with the
// least search work left, so a small request is not stuck behind a large one;
// once its last batch is issued, the worker certifies the scores, takes the
// top K and refines them on its own stream while the search streams serve
// other registrations.  Results equal the serial path's bit for bit: every
// item runs the same kernels on the same data.
//
// Object spectra stay resident in a cache keyed by the mesh's contents (a
// 64-bit hash, confirmed byte for byte on a hit), the canvas and the
// object-grid thresholds.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
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

// a registration's search in continuous mode, shared by its worker and the
// scheduler (guarded by reg_server::mu)
struct SearchTask {
    reg_handle* h = nullptr;
    int M = 0, B = 0, nb = 0, sets = 1;
    int next = 0;                 // next batch to issue
    double cost = 0;              // model bytes of one batch (4 half-spectra per rotation)
    hipEvent_t ready = nullptr;   // the handle is built (recorded on the worker's stream)
    hipEvent_t set_ev[2] = {nullptr, nullptr};  // last batch issued on each pass-buffer set
    bool issued_all = false;
    int error = 0;
};

}  // namespace

struct reg_server {
    reg_server_cfg cfg{};
    std::mutex mu;
    std::condition_variable cv_dispatch, cv_done, cv_work, cv_sched, cv_issued;
    std::deque<std::shared_ptr<Job>> queue;
    std::map<reg_ticket, std::shared_ptr<Job>> jobs;
    std::vector<std::shared_ptr<Job>> slot_job;  // per worker: assigned job or null
    std::vector<std::thread> workers;
    std::thread dispatcher;
    std::vector<hipStream_t> streams;
    // continuous mode: registrations searching, the shared search streams and
    // the batches in flight on them (completion events, oldest first)
    std::vector<std::shared_ptr<SearchTask>> tasks;
    std::thread scheduler;
    hipStream_t sstream[2] = {nullptr, nullptr};
    std::deque<hipEvent_t> inflight[2];
    std::vector<hipEvent_t> ev_pool;
    int64_t batches_issued = 0;
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
    void schedule_loop();
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

    if (cfg.mode == 1) {
        rc = score_rotations(h, 0, M, dS, nullptr, dPose);
        if (rc) return sfail(rc, regdock_rt::last_error());
    } else {
        // hand the search to the scheduler, then certify on this stream
        auto t = std::make_shared<SearchTask>();
        t->h = h;
        t->M = M;
        t->B = regdock_rt::handle_batch(h);
        t->nb = (M + t->B - 1) / t->B;
        t->sets = regdock_rt::handle_buffer_sets(h);
        t->cost = 4.0 * (double)t->B * (double)j.grid.n * j.grid.n * (j.grid.n / 2 + 1) * 8.0;
        struct FreeEv {
            SearchTask* t;
            hipStream_t s;
            ~FreeEv() {
                (void)hipStreamSynchronize(s);  // every batch is done once the stream's later work is
                for (hipEvent_t e : {t->ready, t->set_ev[0], t->set_ev[1]})
                    if (e) (void)hipEventDestroy(e);
            }
        } fe{t.get(), s};
        for (hipEvent_t* e : {&t->ready, &t->set_ev[0], &t->set_ev[1]})
            if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) return sfail(REG_EDEVICE, "event");
        if (hipEventRecord(t->ready, s) != hipSuccess) return sfail(REG_EDEVICE, "event record");
        {
            std::unique_lock<std::mutex> lk(mu);
            tasks.push_back(t);
            cv_sched.notify_all();
            cv_issued.wait(lk, [&] { return t->issued_all; });
            tasks.erase(std::find(tasks.begin(), tasks.end(), t));
        }
        if (t->error) return sfail(t->error, "search batch failed");
        for (int k = 0; k < t->sets; ++k)
            if (hipStreamWaitEvent(s, t->set_ev[k], 0) != hipSuccess) return sfail(REG_EDEVICE, "wait");
        rc = regdock_rt::enqueue_search_finish(h, dS, nullptr, dPose, s);
        if (rc) return sfail(rc, regdock_rt::last_error());
    }
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

// Continuous mode: issue rotation batches of the registrations whose handle is
// built, the one with the least search work left first, onto the two search
// streams, keeping at most two batches in flight per stream.  A batch waits
// on the device for its handle's build and for the previous batch that used
// its pass-buffer set.
void reg_server::schedule_loop() {
    constexpr int PER_STREAM = 2;
    int rr = 0;
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        for (int k = 0; k < 2; ++k)
            while (!inflight[k].empty() && hipEventQuery(inflight[k].front()) == hipSuccess) {
                ev_pool.push_back(inflight[k].front());
                inflight[k].pop_front();
            }
        SearchTask* pick = nullptr;
        double least = INFINITY;
        for (auto& t : tasks) {
            if (t->issued_all) continue;
            const double left = (double)(t->nb - t->next) * t->cost;
            if (left < least) {
                least = left;
                pick = t.get();
            }
        }
        const int slot = inflight[rr].size() < PER_STREAM ? rr : inflight[1 - rr].size() < PER_STREAM ? 1 - rr : -1;
        if (pick && slot >= 0) {
            hipStream_t ss = sstream[slot];
            const int b = pick->next++;
            const int set = pick->sets == 2 ? (b & 1) : 0;
            const int b0 = b * pick->B, cnt = std::min(pick->B, pick->M - b0);
            hipEvent_t done = nullptr;
            if (!ev_pool.empty()) {
                done = ev_pool.back();
                ev_pool.pop_back();
            } else if (hipEventCreateWithFlags(&done, hipEventDisableTiming) != hipSuccess) {
                done = nullptr;
            }
            int rc = REG_OK;
            if (!done || hipStreamWaitEvent(ss, pick->ready, 0) != hipSuccess ||
                (b >= pick->sets && hipStreamWaitEvent(ss, pick->set_ev[set], 0) != hipSuccess))
                rc = REG_EDEVICE;
            if (!rc) rc = regdock_rt::enqueue_search_batch(pick->h, b0, cnt, set, ss);
            if (!rc && (hipEventRecord(pick->set_ev[set], ss) != hipSuccess || hipEventRecord(done, ss) != hipSuccess))
                rc = REG_EDEVICE;
            if (rc) {
                pick->error = rc;
                pick->issued_all = true;
                if (done) ev_pool.push_back(done);
                cv_issued.notify_all();
                continue;
            }
            inflight[slot].push_back(done);
            ++batches_issued;
            rr = 1 - slot;
            if (pick->next == pick->nb) {
                pick->issued_all = true;
                cv_issued.notify_all();
            }
            continue;
        }
        if (stopping && tasks.empty()) break;
        // wait for a new registration, or poll the batches in flight
        cv_sched.wait_for(lk, std::chrono::microseconds(100));
    }
    lk.unlock();
    for (int k = 0; k < 2; ++k) {
        for (hipEvent_t e : inflight[k]) {
            (void)hipEventSynchronize(e);
            (void)hipEventDestroy(e);
        }
        inflight[k].clear();
    }
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    ev_pool.clear();
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
    if (!c.fake && c.mode != 1)
        for (auto& st : srv->sstream)
            if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
                for (auto& t : srv->streams) (void)hipStreamDestroy(t);
                for (auto& t : srv->sstream)
                    if (t) (void)hipStreamDestroy(t);
                return sfail(REG_EDEVICE, "hipStreamCreate failed");
            }
    srv->slot_job.resize(c.max_inflight);
    reg_server* s = srv.get();
    for (int w = 0; w < c.max_inflight; ++w) s->workers.emplace_back([s, w] { s->worker_loop(w); });
    s->dispatcher = std::thread([s] { s->dispatch_loop(); });
    if (!c.fake && c.mode != 1) s->scheduler = std::thread([s] { s->schedule_loop(); });
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
    if (s->scheduler.joinable()) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->cv_sched.notify_all();
        }
        s->scheduler.join();
    }
    s->cv_done.notify_all();
    for (auto& st : s->streams) (void)hipStreamDestroy(st);
    for (auto& st : s->sstream)
        if (st) (void)hipStreamDestroy(st);
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
                                          rq->refine ? j->top_k : 0, j->params.rotate_object, j->params.split_plane);
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
