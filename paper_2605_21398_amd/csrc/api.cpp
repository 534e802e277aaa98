// C ABI of libregdock: handles, validation, device buffers and the batched
// launch sequence of the global search.  See include/regdock.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <future>
#include <mutex>
#include <unordered_map>
#include <string>
#include <vector>

#include "refine_kernels.h"
#include "regdock.h"
#include "runtime.h"
#include "search_kernels.h"
#include "so3_sampling.h"

using namespace regdock;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int lattice_edge(int n) { return 2 * (int)std::ceil((std::sqrt(3.0) * n + 2.0) / 2.0); }

}  // namespace

// Everything derived from the object alone (mesh, canvas edge and spacing,
// and the object-grid thresholds): the mesh, its anchor, the object grid O,
// its spectrum conj(F(O))/n^3 with the exact low-frequency block, the nonzero
// list of O, the twiddles and the refinement's bounding-sphere hierarchy.
// Handles share it, so a serving cache keeps object spectra resident.
// ------------------------------------------------------ device memory cache

namespace {
struct DevCache {
    std::mutex mu;
    std::map<std::pair<int, size_t>, std::vector<void*>> free_blocks;  // (device, size) -> blocks
    std::unordered_map<void*, std::pair<int, size_t>> live;             // block -> (device, size)
    size_t cached = 0;
    size_t cap = (size_t)32 << 30;  // cached bytes beyond this go back to HIP
};
// never destroyed: blocks still cached at exit go with the process
DevCache& dev_cache() {
    static DevCache* c = new DevCache;
    return *c;
}
size_t round_block(size_t b) {
    const size_t small = 512, big = (size_t)2 << 20;
    return b <= ((size_t)1 << 20) ? (b + small - 1) / small * small : (b + big - 1) / big * big;
}
void trim_device(int dev) {
    std::vector<void*> out;
    {
        DevCache& c = dev_cache();
        std::lock_guard<std::mutex> g(c.mu);
        for (auto it = c.free_blocks.begin(); it != c.free_blocks.end();) {
            if (dev < 0 || it->first.first == dev) {
                for (void* q : it->second) out.push_back(q);
                c.cached -= it->first.second * it->second.size();
                it = c.free_blocks.erase(it);
            } else {
                ++it;
            }
        }
    }
    for (void* q : out) (void)hipFree(q);
}
}  // namespace

namespace regdock_rt {
hipError_t dev_alloc(void** p, size_t bytes) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    const size_t rb = round_block(bytes ? bytes : 1);
    DevCache& c = dev_cache();
    {
        std::lock_guard<std::mutex> g(c.mu);
        auto it = c.free_blocks.find({dev, rb});
        if (it != c.free_blocks.end() && !it->second.empty()) {
            *p = it->second.back();
            it->second.pop_back();
            c.cached -= rb;
            c.live[*p] = {dev, rb};
            return hipSuccess;
        }
    }
    hipError_t e = hipMalloc(p, rb);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        trim_device(dev);
        e = hipMalloc(p, rb);
        if (e != hipSuccess) return e;
    }
    std::lock_guard<std::mutex> g(c.mu);
    c.live[*p] = {dev, rb};
    return hipSuccess;
}
void dev_release(void* p) {
    if (!p) return;
    DevCache& c = dev_cache();
    {
        std::lock_guard<std::mutex> g(c.mu);
        auto it = c.live.find(p);
        if (it != c.live.end()) {
            const auto key = it->second;
            c.live.erase(it);
            if (c.cached + key.second <= c.cap) {
                c.free_blocks[key].push_back(p);
                c.cached += key.second;
                return;
            }
        }
    }
    (void)hipFree(p);
}
size_t dev_cached_bytes() {
    DevCache& c = dev_cache();
    std::lock_guard<std::mutex> g(c.mu);
    return c.cached;
}
void dev_trim() { trim_device(-1); }
}  // namespace regdock_rt

// Refinement hierarchy on the host (built off the device path, uploaded once).
struct HostGeometry {
    std::vector<float4> face, cl, top;
    std::vector<int2> cl_range, top_range;
    std::vector<int> slot_of;
};

// Launch schedule of a handle's search: rotations per batch, streams the
// batches alternate over, and the workgroup variants of the three passes.
struct Schedule {
    int batch = 0, lanes = 2, pv1 = -1, pv3 = -1, zv = -1;
    double us1 = 0, usz = 0, us3 = 0, ns_rot = 0;  // tuned timings (us per rotation per pass, ns per rotation)
};

struct ObjectData {
    int n = 0, nv = 0, nf = 0;
    double h = 0, tau_out1 = 0, tau_in1 = 0, rho = 0;
    float* V = nullptr;
    int32_t* F = nullptr;
    uint8_t* touch = nullptr;
    double* anchor = nullptr;
    float* O = nullptr;
    float* fo = nullptr;
    float2* W = nullptr;
    double2* Wlow = nullptr;
    uint32_t* nz_idx = nullptr;
    float* nz_val = nullptr;
    int* nz_count = nullptr;
    int* nz_bcount = nullptr;
    int* nz_boff = nullptr;
    float2* tw = nullptr;
    double2* tw64 = nullptr;
    bool geo_ready = false;
    RefineGeometry geo{};
    std::mutex geo_mu;                        // the first refinement of the object builds geo
    std::future<HostGeometry> geo_job;  // host part of geo, started when the object is built
    size_t bytes = 0;
    std::vector<void*> owned;
    // recorded on the building stream once the grid, spectrum and nonzero list
    // are written; a handle that takes the object from a cache waits for it
    hipEvent_t ready = nullptr;
    template <class T>
    hipError_t alloc(T** p, size_t count) {
        void* q = nullptr;
        const size_t b = count * sizeof(T) > 0 ? count * sizeof(T) : 1;
        hipError_t e = regdock_rt::dev_alloc(&q, b);
        if (e == hipSuccess) {
            owned.push_back(q);
            bytes += b;
            *p = (T*)q;
        }
        return e;
    }
    bool matches(int n_, double h_, const reg_params& p) const {
        return n == n_ && h == h_ && tau_out1 == p.tau_out1 && tau_in1 == p.tau_in1 && rho == p.rho;
    }
    // the last handle using the object has synchronised its stream
    ~ObjectData() {
        if (geo_job.valid()) geo_job.wait();
        if (ready) (void)hipEventDestroy(ready);
        for (void* q : owned) regdock_rt::dev_release(q);
    }
};

struct reg_handle {
    std::shared_ptr<ObjectData> obj;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool poisoned = false;
    int n = 0, m = 0, mp = 0, n_rot = 0, n_poses = 0, nv = 0, nf = 0, batch = 0;
    Schedule sched;  // lanes and kernel variants (batch is the field above)
    int rot_cap = 0;     // rotations the per-rotation buffers hold
    int in_batches = 0;  // live batches whose captured graph holds this handle's buffers
    size_t H = 0;
    double h = 0, wc[3] = {0, 0, 0};
    reg_probe probe{};
    reg_params prm{};
    // device buffers
    float* V = nullptr;
    int32_t* F = nullptr;
    uint8_t* touch = nullptr;
    float* poses = nullptr;
    float* so3 = nullptr;
    double* rots = nullptr;
    double* pose_prep = nullptr;
    double* anchor = nullptr;
    float* O = nullptr;
    float* fo = nullptr;
    unsigned long long* od2 = nullptr;
    unsigned long long* odt2 = nullptr;
    uint32_t* opar = nullptr;
    float2* W = nullptr;
    float2* spec = nullptr;
    unsigned long long* ptop = nullptr;
    double* pssq = nullptr;
    int32_t* cand_idx = nullptr;
    int32_t* cand_n = nullptr;
    double* cand_part = nullptr;
    int* stats = nullptr;
    double* window = nullptr;
    uint8_t* ovf = nullptr;
    double* best_val = nullptr;
    int32_t* best_flat = nullptr;
    int32_t* need_list = nullptr;
    int* need_count = nullptr;
    uint32_t* nz_idx = nullptr;
    float* nz_val = nullptr;
    int* nz_count = nullptr;
    int* nz_bcount = nullptr;
    int* nz_boff = nullptr;
    uint8_t* Sw = nullptr;
    uint8_t* cm = nullptr;
    // rotated-object search (params.rotate_object): cell classes and corner
    // records of O on the body lattice, and the fixed swept canvas S, whose
    // spectrum and nonzero list replace O's (W, Wlow, nz_* then point to
    // buffers of the handle)
    bool rotobj = false;
    uint8_t* ocls = nullptr;
    float4* orec = nullptr;
    float* Sc = nullptr;
    // split plane passes (edges above 180, or params.split_plane): the plane
    // buffer and the rows' low-block x sums of each lane; units = peak records
    // per rotation (n for the fused passes)
    bool split = false;
    int units = 0;
    float2* xbuf = nullptr;
    float2* xbuf2 = nullptr;
    double2* lowrow = nullptr;
    double2* lowrow2 = nullptr;
    unsigned long long* reach4 = nullptr;  // the swept lattice's reach (S_r beyond it is skipped)
    float2* tw = nullptr;
    double2* tw64 = nullptr;
    double2* lowT = nullptr;
    double2* Wlow = nullptr;
    double2* Plow = nullptr;
    // the second lane of the search pipeline: the odd batches of a call run on
    // stream2 with pass buffers of their own, so that one batch's HBM-bound z
    // pass overlaps the VALU-bound plane passes of the next
    hipStream_t stream2 = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    float2* spec2 = nullptr;
    unsigned long long* ptop2 = nullptr;
    double* pssq2 = nullptr;
    double2* lowT2 = nullptr;
    double2* Plow2 = nullptr;
    int* err = nullptr;
    // refinement solver state (the mesh hierarchy lives in the object)
    RefineState* rst = nullptr;
    RefineTrial* rtr = nullptr;
    RefineEval* rev = nullptr;
    LbfgsState* rlb = nullptr;  // L-BFGS-B state per start
    bool r_lbfgsb = false;      // the solver of the refinement in progress
    RefineHit* rhits = nullptr;
    RefineScratch rw{};
    int r_cap = 0;
    int* r_active = nullptr;       // [unfinished starts, evaluations]
    int* r_active_host = nullptr;  // pinned copy of r_active
    int64_t r_rounds = 0, r_evals = 0;  // of the last refine_se3 call
    std::vector<void*> owned;
    // optional per-kernel timing with HIP events on the handle's stream
    bool timing = false;
    struct Timed {
        hipEvent_t a, b;
        int kernel;
        int rotations;
    };
    std::vector<Timed> timed;
    std::vector<hipEvent_t> event_pool;
    size_t pool_used = 0;
    hipEvent_t next_event() {
        if (pool_used == event_pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            event_pool.push_back(e);
        }
        return event_pool[pool_used++];
    }

    template <class T>
    hipError_t alloc(T** p, size_t count) {
        void* q = nullptr;
        hipError_t e = regdock_rt::dev_alloc(&q, count * sizeof(T) > 0 ? count * sizeof(T) : 1);
        if (e == hipSuccess) {
            owned.push_back(q);
            *p = (T*)q;
        }
        return e;
    }
    // give one owned block back (the stream has no queued work using it)
    void release(void* p) {
        for (size_t i = 0; i < owned.size(); ++i)
            if (owned[i] == p) {
                owned.erase(owned.begin() + i);
                regdock_rt::dev_release(p);
                return;
            }
    }
    ~reg_handle() {
        // queued work must finish before the blocks (and the object, released
        // after this body) can serve anyone else
        if (stream) (void)hipStreamSynchronize(stream);
        if (stream2) (void)hipStreamSynchronize(stream2);
        if (stream2) (void)hipStreamDestroy(stream2);
        if (fork_ev) (void)hipEventDestroy(fork_ev);
        if (join_ev) (void)hipEventDestroy(join_ev);
        for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
        for (void* p : owned) regdock_rt::dev_release(p);
        if (r_active_host) (void)hipHostFree(r_active_host);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
};

#define DEV_TRY(hd, expr)                                                                        \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess) {                                                                  \
            if (hd) (hd)->poisoned = true;                                                       \
            return fail(REG_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));            \
        }                                                                                        \
    } while (0)

#define ALLOC_TRY(hd, ptr, count)                                                                \
    do {                                                                                         \
        hipError_t e_ = (hd)->alloc(&(ptr), (count));                                            \
        if (e_ != hipSuccess) {                                                                  \
            (void)hipGetLastError();                                                             \
            return fail(REG_ENOMEM, "device allocation of %zu elements for %s failed: %s",       \
                        (size_t)(count), #ptr, hipGetErrorString(e_));                           \
        }                                                                                        \
    } while (0)

#define OBJ_ALLOC_TRY(ob, ptr, count)                                                            \
    do {                                                                                         \
        hipError_t e_ = (ob)->alloc(&(ptr), (count));                                            \
        if (e_ != hipSuccess) {                                                                  \
            (void)hipGetLastError();                                                             \
            return fail(REG_ENOMEM, "device allocation of %zu elements for %s failed: %s",       \
                        (size_t)(count), #ptr, hipGetErrorString(e_));                           \
        }                                                                                        \
    } while (0)

static void fill_defaults(reg_params& p) {
    if (p.tau_out1 <= 0) p.tau_out1 = 0.5;
    if (p.tau_in1 <= 0) p.tau_in1 = 0.2;
    if (p.rho <= 0) p.rho = 50.0;
    if (p.tau_out2 <= 0) p.tau_out2 = 0.2;
    if (p.tau_in2 <= 0) p.tau_in2 = 0.03;
    if (p.k <= 0) p.k = 15.0;
    if (p.lambda <= 0) p.lambda = 1e-3;
    if (p.b_t <= 0) p.b_t = 0.5;
    if (p.b_r <= 0) p.b_r = 0.2;
    if (p.eps <= 0) p.eps = 0.25;
    if (p.max_iters <= 0) p.max_iters = 200;
}

// schedules per canvas edge recorded by the autotuner
static std::mutex g_tune_mu;
static std::map<int, Schedule> g_tuned;

static int default_batch(int n, size_t H, int n_rot) {
    size_t need = ((size_t)n_rot + 7) / 8 * 8;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(n);
        if (it != g_tuned.end() && it->second.batch > 0) return (int)std::min<size_t>((size_t)it->second.batch, need);
    }
    // about 256 MB of spectrum work buffer, a multiple of 8 for the XCD mapping
    size_t b = (256u << 20) / (H * sizeof(float2));
    if (b < 8) b = 8;
    if (b > 4096) b = 4096;
    if (b > need) b = need;
    b = (b + 7) / 8 * 8;
    return (int)b;
}

// the handle's lanes and kernel variants: the params where set, else the
// recorded schedule for the edge, else the defaults
static int resolve_schedule(int n, const reg_params& p, Schedule& s, bool split = false) {
    Schedule t;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(n);
        if (it != g_tuned.end()) t = it->second;
    }
    s.lanes = p.lanes > 0 ? p.lanes : t.lanes > 0 ? t.lanes : 2;
    if (s.lanes > 2) return fail(REG_EINVAL, "lanes must be 1 or 2");
    const int dpv = default_plane_variant(n), dzv = default_z_variant(n);
    s.pv1 = p.plane_variant > 0 ? p.plane_variant - 1 : t.pv1 >= 0 ? t.pv1 : dpv;
    s.pv3 = p.plane_variant > 0 ? p.plane_variant - 1 : t.pv3 >= 0 ? t.pv3 : dpv;
    s.zv = p.z_variant > 0 ? p.z_variant - 1 : t.zv >= 0 ? t.zv : dzv;
    if (!split && (!plane_variant_ok(n, s.pv1) || !plane_variant_ok(n, s.pv3)))
        return fail(REG_EINVAL, "plane_variant %d is not valid for edge %d", p.plane_variant, n);
    if (!z_variant_ok(n, s.zv)) return fail(REG_EINVAL, "z_variant %d is not valid for edge %d", p.z_variant, n);
    return REG_OK;
}

// spectrum conj(F(O))/n^3 and the nonzero list of O, both derived from h->O
// The rotated-object search (the paper's variant of Sec. IV-D): O on the body
// lattice a + h (j - m/2) (the object-grid build at edge m), reduced to cell
// classes and corner records, and the swept canvas S (the central n^3 block of
// the swept lattice) with its spectrum conj(F(S))/n^3 and nonzero list, which
// take the places of the swept corner masks and of O's spectrum.  The lattice
// build's scratch is released before returning.
static int build_rotated_object(reg_handle* h) {
    hipStream_t s = h->stream;
    const size_t n3 = (size_t)h->n * h->n * h->n, m3 = (size_t)h->m * h->m * h->m;
    const size_t mp3 = (size_t)h->mp * h->mp * h->mp;
    const size_t words = (size_t)h->m * h->m * ((h->m + 31) / 32);
    float *Ow = nullptr, *fow = nullptr;
    unsigned long long *d2 = nullptr, *dt2 = nullptr;
    uint32_t* par = nullptr;
    ALLOC_TRY(h, Ow, m3);
    ALLOC_TRY(h, fow, m3);
    ALLOC_TRY(h, d2, m3);
    ALLOC_TRY(h, dt2, m3);
    ALLOC_TRY(h, par, words);
    ALLOC_TRY(h, h->ocls, mp3);
    ALLOC_TRY(h, h->orec, 2 * mp3);
    ALLOC_TRY(h, h->Sc, n3);
    ALLOC_TRY(h, h->W, h->H);
    ALLOC_TRY(h, h->Wlow, (size_t)NLOW3);
    ALLOC_TRY(h, h->nz_idx, n3);
    ALLOC_TRY(h, h->nz_val, n3);
    ALLOC_TRY(h, h->nz_count, 1);
    ALLOC_TRY(h, h->nz_bcount, (n3 + 255) / 256);
    ALLOC_TRY(h, h->nz_boff, (n3 + 255) / 256);
    DEV_TRY(h, setup_object_grid(h->V, h->F, h->touch, h->nf, h->m, h->h, h->anchor, h->prm.tau_out1, h->prm.tau_in1,
                                 h->prm.rho, Ow, fow, ObjectScratch{d2, dt2, par}, s));
    DEV_TRY(h, setup_object_cells(Ow, h->m, h->mp, (float)(-h->prm.rho), h->ocls, h->orec, s));
    DEV_TRY(h, swept_canvas(h->Sw, h->m, h->n, h->Sc, s));
    DEV_TRY(h, object_spectrum(h->n, h->Sc, h->spec, h->W, h->tw, h->tw64, h->lowT, h->Wlow, s));
    DEV_TRY(h, build_nonzero_list(h->Sc, h->n, h->nz_bcount, h->nz_boff, h->nz_idx, h->nz_val, h->nz_count, s));
    DEV_TRY(h, hipStreamSynchronize(s));
    for (void* p : {(void*)Ow, (void*)fow, (void*)d2, (void*)dt2, (void*)par}) h->release(p);
    return REG_OK;
}

static int build_object_derived(reg_handle* h) {
    DEV_TRY(h, object_spectrum(h->n, h->O, h->spec, h->W, h->tw, h->tw64, h->lowT, h->Wlow, h->stream, h->xbuf,
                               h->lowrow));
    DEV_TRY(h, build_nonzero_list(h->O, h->n, h->nz_bcount, h->nz_boff, h->nz_idx, h->nz_val, h->nz_count, h->stream));
    return REG_OK;
}

// Bounding-sphere hierarchy for the refinement's distance queries: faces in
// Morton order of their centroids, REF_FANOUT faces per cluster and
// REF_FANOUT clusters per top node.  A node's radius bounds the distance from
// its centre to every point of its faces (centroid distance plus the face's
// own radius), widened by 1e-5 mm so that float32 evaluation stays
// conservative.  Face centroid and radius follow the body-frame definition of
// the bounding-sphere test (mean of the three vertices, largest vertex distance).
// Faces in Morton order of their centroids with clusters of REF_FANOUT faces
// and top nodes of REF_FANOUT clusters (pure host work on copies of the mesh).
static HostGeometry host_refine_geometry(std::vector<float> V, std::vector<int32_t> F, int nv, int nf) {
    (void)nv;
    std::vector<double> fc(3 * (size_t)nf), fr(nf);
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int f = 0; f < nf; ++f) {
        const float* v[3] = {&V[3 * (size_t)F[3 * f]], &V[3 * (size_t)F[3 * f + 1]], &V[3 * (size_t)F[3 * f + 2]]};
        for (int a = 0; a < 3; ++a) {
            fc[3 * f + a] = ((double)v[0][a] + (double)v[1][a] + (double)v[2][a]) / 3.0;
            lo[a] = std::min(lo[a], fc[3 * f + a]);
            hi[a] = std::max(hi[a], fc[3 * f + a]);
        }
        double r = 0;
        for (int k = 0; k < 3; ++k) {
            double d2 = 0;
            for (int a = 0; a < 3; ++a) d2 += ((double)v[k][a] - fc[3 * f + a]) * ((double)v[k][a] - fc[3 * f + a]);
            r = std::max(r, std::sqrt(d2));
        }
        fr[f] = r;
    }
    auto spread = [](uint32_t x) {
        x &= 0x3ff;
        x = (x | (x << 16)) & 0x030000ff;
        x = (x | (x << 8)) & 0x0300f00f;
        x = (x | (x << 4)) & 0x030c30c3;
        x = (x | (x << 2)) & 0x09249249;
        return x;
    };
    std::vector<std::pair<uint32_t, int>> key(nf);
    for (int f = 0; f < nf; ++f) {
        uint32_t q[3];
        for (int a = 0; a < 3; ++a) {
            const double ext = hi[a] - lo[a];
            const double u = ext > 0 ? (fc[3 * f + a] - lo[a]) / ext : 0.0;
            q[a] = (uint32_t)std::min(1023.0, std::max(0.0, std::floor(u * 1024.0)));
        }
        key[f] = {spread(q[0]) | (spread(q[1]) << 1) | (spread(q[2]) << 2), f};
    }
    std::sort(key.begin(), key.end());
    const int n_cl = (nf + REF_FANOUT - 1) / REF_FANOUT;
    const int n_top = (n_cl + REF_FANOUT - 1) / REF_FANOUT;
    std::vector<float4> face(4 * (size_t)nf), cl(n_cl), top(n_top);
    std::vector<int2> cl_range(n_cl), top_range(n_top);
    std::vector<double> clc(3 * (size_t)n_cl), clr(n_cl);
    std::vector<int> slot_of(nf);
    for (int slot = 0; slot < nf; ++slot) {
        const int f = key[slot].second;
        slot_of[f] = slot;
        const float* v[3] = {&V[3 * (size_t)F[3 * f]], &V[3 * (size_t)F[3 * f + 1]], &V[3 * (size_t)F[3 * f + 2]]};
        float idx_bits;
        std::memcpy(&idx_bits, &f, 4);
        face[4 * (size_t)slot] = make_float4(v[0][0], v[0][1], v[0][2], v[1][0]);
        face[4 * (size_t)slot + 1] = make_float4(v[1][1], v[1][2], v[2][0], v[2][1]);
        face[4 * (size_t)slot + 2] = make_float4(v[2][2], (float)fc[3 * f], (float)fc[3 * f + 1], (float)fc[3 * f + 2]);
        face[4 * (size_t)slot + 3] = make_float4((float)fr[f], idx_bits, 0.0f, 0.0f);
    }
    const double slack = 1e-5;
    for (int c = 0; c < n_cl; ++c) {
        const int s0 = c * REF_FANOUT, s1 = std::min(nf, s0 + REF_FANOUT);
        double blo[3] = {INFINITY, INFINITY, INFINITY}, bhi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int slot = s0; slot < s1; ++slot) {
            const int f = key[slot].second;
            for (int a = 0; a < 3; ++a) {
                blo[a] = std::min(blo[a], fc[3 * f + a] - fr[f]);
                bhi[a] = std::max(bhi[a], fc[3 * f + a] + fr[f]);
            }
        }
        double r = 0;
        for (int a = 0; a < 3; ++a) clc[3 * c + a] = 0.5 * (blo[a] + bhi[a]);
        for (int slot = s0; slot < s1; ++slot) {
            const int f = key[slot].second;
            double d2 = 0;
            for (int a = 0; a < 3; ++a) d2 += (fc[3 * f + a] - clc[3 * c + a]) * (fc[3 * f + a] - clc[3 * c + a]);
            r = std::max(r, std::sqrt(d2) + fr[f]);
        }
        clr[c] = r * (1 + 1e-6) + slack;
        cl[c] = make_float4((float)clc[3 * c], (float)clc[3 * c + 1], (float)clc[3 * c + 2], (float)clr[c]);
        cl_range[c] = make_int2(s0, s1 - s0);
    }
    for (int t = 0; t < n_top; ++t) {
        const int c0 = t * REF_FANOUT, c1 = std::min(n_cl, c0 + REF_FANOUT);
        double blo[3] = {INFINITY, INFINITY, INFINITY}, bhi[3] = {-INFINITY, -INFINITY, -INFINITY}, tc[3];
        for (int c = c0; c < c1; ++c)
            for (int a = 0; a < 3; ++a) {
                blo[a] = std::min(blo[a], clc[3 * c + a] - clr[c]);
                bhi[a] = std::max(bhi[a], clc[3 * c + a] + clr[c]);
            }
        for (int a = 0; a < 3; ++a) tc[a] = 0.5 * (blo[a] + bhi[a]);
        double r = 0;
        for (int c = c0; c < c1; ++c) {
            double d2 = 0;
            for (int a = 0; a < 3; ++a) d2 += (clc[3 * c + a] - tc[a]) * (clc[3 * c + a] - tc[a]);
            r = std::max(r, std::sqrt(d2) + clr[c]);
        }
        top[t] = make_float4((float)tc[0], (float)tc[1], (float)tc[2], (float)(r * (1 + 1e-6) + slack));
        top_range[t] = make_int2(c0, c1 - c0);
    }
    HostGeometry g;
    g.face = std::move(face);
    g.cl = std::move(cl);
    g.top = std::move(top);
    g.cl_range = std::move(cl_range);
    g.top_range = std::move(top_range);
    g.slot_of = std::move(slot_of);
    return g;
}

// Starts the host part of the hierarchy on a thread of its own (the mesh is
// on the device and the stream idle); the first refinement uploads it.
static int start_refine_geometry(reg_handle* h) {
    std::vector<float> V(3 * (size_t)h->nv);
    std::vector<int32_t> F(3 * (size_t)h->nf);
    DEV_TRY(h, hipMemcpyAsync(V.data(), h->V, V.size() * 4, hipMemcpyDeviceToHost, h->stream));
    DEV_TRY(h, hipMemcpyAsync(F.data(), h->F, F.size() * 4, hipMemcpyDeviceToHost, h->stream));
    DEV_TRY(h, hipStreamSynchronize(h->stream));
    h->obj->geo_job = std::async(std::launch::async, host_refine_geometry, std::move(V), std::move(F), h->nv, h->nf);
    return REG_OK;
}

// The hierarchy on the device (called with the object's geo_mu held).
static int build_refine_geometry(reg_handle* h) {
    ObjectData* o = h->obj.get();
    if (!o->geo_job.valid()) {
        const int rc = start_refine_geometry(h);
        if (rc) return rc;
    }
    HostGeometry g;
    try {
        g = o->geo_job.get();
    } catch (const std::exception& e) {
        return fail(REG_ENOMEM, "refinement hierarchy: %s", e.what());
    }
    const int n_cl = (int)g.cl.size(), n_top = (int)g.top.size();
    float4 *d_face, *d_cl, *d_top;
    int2 *d_clr, *d_topr;
    int* d_slot;
    OBJ_ALLOC_TRY(o, d_slot, g.slot_of.size());
    OBJ_ALLOC_TRY(o, d_face, g.face.size());
    OBJ_ALLOC_TRY(o, d_cl, g.cl.size());
    OBJ_ALLOC_TRY(o, d_top, g.top.size());
    OBJ_ALLOC_TRY(o, d_clr, g.cl_range.size());
    OBJ_ALLOC_TRY(o, d_topr, g.top_range.size());
    hipStream_t s = h->stream;
    DEV_TRY(h, hipMemcpyAsync(d_face, g.face.data(), g.face.size() * sizeof(float4), hipMemcpyHostToDevice, s));
    DEV_TRY(h, hipMemcpyAsync(d_cl, g.cl.data(), g.cl.size() * sizeof(float4), hipMemcpyHostToDevice, s));
    DEV_TRY(h, hipMemcpyAsync(d_top, g.top.data(), g.top.size() * sizeof(float4), hipMemcpyHostToDevice, s));
    DEV_TRY(h, hipMemcpyAsync(d_clr, g.cl_range.data(), g.cl_range.size() * sizeof(int2), hipMemcpyHostToDevice, s));
    DEV_TRY(h, hipMemcpyAsync(d_topr, g.top_range.data(), g.top_range.size() * sizeof(int2), hipMemcpyHostToDevice, s));
    DEV_TRY(h, hipMemcpyAsync(d_slot, g.slot_of.data(), g.slot_of.size() * sizeof(int), hipMemcpyHostToDevice, s));
    DEV_TRY(h, hipStreamSynchronize(s));
    o->geo = RefineGeometry{d_top, d_topr, d_cl, d_clr, d_face, d_slot, n_top, n_cl, (int)g.slot_of.size()};
    o->geo_ready = true;
    return REG_OK;
}

// solver constants: Table I values, the box, and the device-side stopping rule
static RefineConst refine_const(const reg_handle* h) {
    RefineConst c{};
    c.r = (float)h->probe.radius_mm;
    c.L = (float)h->probe.length_mm;
    c.r64 = h->probe.radius_mm;
    c.L64 = h->probe.length_mm;
    // faces farther than tau_out2 cannot change s, s' or s''; cull at the
    // smaller of the cutoff and tau_out2
    c.cull = (float)std::min(h->prm.eps, h->prm.tau_out2);
    c.eps = (float)h->prm.eps;
    c.tau_out2 = h->prm.tau_out2;
    c.tau_in2 = h->prm.tau_in2;
    c.k = h->prm.k;
    c.lambda = h->prm.lambda;
    c.b_t = h->prm.b_t;
    c.b_r = h->prm.b_r;
    c.tol_pg = 1e-6;
    // an accepted, nearly undamped step (mu <= 10 mu0) below 1e-7 (mm, rad)
    // ends a start: with a linear rate rho of the last iterations the iterate
    // is then step * rho / (1 - rho) from the limit, within 1e-3 mm and 1e-3 deg
    // for rho up to 0.99
    c.tol_step = 1e-7;
    c.mu0 = 1e-3;
    c.max_iters = h->prm.max_iters;
    return c;
}

static int ensure_refine_buffers(reg_handle* h, int K) {
    {
        std::lock_guard<std::mutex> g(h->obj->geo_mu);
        if (!h->obj->geo_ready) {
            int rc = build_refine_geometry(h);
            if (rc) return rc;
        }
    }
    if (!h->r_active_host) {
        if (hipHostMalloc((void**)&h->r_active_host, 2 * sizeof(int), hipHostMallocDefault) != hipSuccess) {
            h->r_active_host = nullptr;
            (void)hipGetLastError();
            return fail(REG_ENOMEM, "pinned host allocation failed");
        }
        ALLOC_TRY(h, h->r_active, 2);
    }
    if (K > h->r_cap) {
        const int cap = std::max(K, 16);
        ALLOC_TRY(h, h->rst, (size_t)cap);
        ALLOC_TRY(h, h->rtr, (size_t)cap * REF_TMAX);
        ALLOC_TRY(h, h->rev, (size_t)cap * REF_TMAX * REF_EVAL_PARTS);
        ALLOC_TRY(h, h->rlb, (size_t)cap);
        ALLOC_TRY(h, h->rhits, (size_t)cap * REF_TMAX * h->n_poses);
        // pairs: 16 per query on average (about 3 are needed); a query whose
        // pairs do not fit is searched by itself
        const size_t nq = (size_t)cap * REF_TMAX * h->n_poses;
        ALLOC_TRY(h, h->rw.xf, 12 * nq);
        ALLOC_TRY(h, h->rw.qkey, nq);
        ALLOC_TRY(h, h->rw.qflag, nq);
        ALLOC_TRY(h, h->rw.qst, nq);
        ALLOC_TRY(h, h->rw.pairs, 16 * nq);
        ALLOC_TRY(h, h->rw.pres, 16 * nq);
        ALLOC_TRY(h, h->rw.nest, 16 * nq);
        if (!h->rw.pair_count) ALLOC_TRY(h, h->rw.pair_count, REF_COUNTERS);
        h->rw.pair_cap = (int)(std::min<size_t>(16 * nq, 1u << 30) / REF_SEGS * REF_SEGS);
        h->r_cap = cap;
    }
    return REG_OK;
}

// register_init with an optional object already built for the same mesh,
// canvas and object-grid thresholds (the serving cache): then the mesh copy,
// the object grid, its spectrum and nonzero list are taken from it.
// Per-rotation buffers for `count` rotations (the old ones, if any, are
// released first; the handle's stream has no queued work using them).
static int alloc_rotation_buffers(reg_handle* h, int count) {
    for (void* p : {(void*)h->so3, (void*)h->rots, (void*)h->cand_idx, (void*)h->cand_n, (void*)h->cand_part,
                    (void*)h->window, (void*)h->ovf, (void*)h->best_val, (void*)h->best_flat, (void*)h->need_list})
        if (p) h->release(p);
    h->rot_cap = 0;
    const size_t M = (size_t)count;
    ALLOC_TRY(h, h->so3, 4 * M);
    ALLOC_TRY(h, h->rots, 9 * M);
    ALLOC_TRY(h, h->cand_idx, M * CMAX);
    ALLOC_TRY(h, h->cand_n, M);
    ALLOC_TRY(h, h->cand_part, M * CMAX * rescore_slices(h->n));
    ALLOC_TRY(h, h->window, M);
    ALLOC_TRY(h, h->ovf, M);
    ALLOC_TRY(h, h->best_val, M);
    ALLOC_TRY(h, h->best_flat, M);
    ALLOC_TRY(h, h->need_list, M);
    h->rot_cap = count;
    return REG_OK;
}

static int init_impl(const reg_mesh* mesh, const reg_probe* probe, const float* poses, int32_t n_poses,
                     const float* so3, int32_t n_rot, const reg_grid_spec* grid, const reg_params* params,
                     void* hip_stream, std::shared_ptr<ObjectData> cached, reg_handle** out) {
    g_err.clear();
    if (!out) return fail(REG_EINVAL, "out is NULL");
    *out = nullptr;
    if (!mesh || !probe || !poses || !so3 || !grid) return fail(REG_EINVAL, "NULL argument");
    if (!mesh->vertices || !mesh->faces || mesh->n_vertices < 3 || mesh->n_faces < 1)
        return fail(REG_EINVAL, "mesh needs >= 3 vertices and >= 1 face");
    if (n_poses < 1 || n_rot < 1) return fail(REG_EINVAL, "n_poses and n_rot must be >= 1");
    if (!(probe->radius_mm > 0) || !(probe->length_mm > 0) || !std::isfinite(probe->radius_mm) ||
        !std::isfinite(probe->length_mm))
        return fail(REG_EINVAL, "probe radius and length must be finite and > 0");
    if (!(grid->h_mm > 0) || !std::isfinite(grid->h_mm)) return fail(REG_EINVAL, "grid h must be finite and > 0");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(grid->center_world[a])) return fail(REG_EINVAL, "grid center must be finite");
    if (!canvas_supported(grid->n)) return fail(REG_ENOTSUP, "canvas edge n=%d has no compiled plan", grid->n);

    reg_handle* h = new reg_handle();
    struct Guard {
        reg_handle*& p;
        ~Guard() { delete p; }
    } guard{h};

    h->n = grid->n;
    h->h = grid->h_mm;
    for (int a = 0; a < 3; ++a) h->wc[a] = grid->center_world[a];
    h->m = lattice_edge(h->n);
    h->mp = (h->m + 3) / 4 * 4;
    h->probe = *probe;
    if (params) h->prm = *params;
    fill_defaults(h->prm);
    h->rotobj = h->prm.rotate_object != 0;
    h->split = !fused_supported(grid->n) || h->prm.split_plane != 0;
    if (h->split && !split_supported(grid->n))
        return fail(REG_ENOTSUP, "no split plane passes are compiled for edge %d", grid->n);
    if (h->split && h->rotobj)
        return fail(REG_ENOTSUP, "the rotated-object search runs on the fused plane passes only (edges up to 180)");
    h->units = h->split ? split_units(grid->n) : grid->n;
    h->n_rot = n_rot;
    h->n_poses = n_poses;
    h->nv = mesh->n_vertices;
    h->nf = mesh->n_faces;
    h->H = spectrum_elems(h->n);
    h->batch = h->prm.batch > 0 ? (h->prm.batch + 7) / 8 * 8 : default_batch(h->n, h->H, n_rot);
    {
        const int rc = resolve_schedule(h->n, h->prm, h->sched, h->split);
        if (rc) return rc;
    }
    h->stream = (hipStream_t)hip_stream;  // NULL: the null stream
    const size_t n3 = (size_t)h->n * h->n * h->n;
    const size_t m3 = (size_t)h->m * h->m * h->m;
    const size_t mp3 = (size_t)h->mp * h->mp * h->mp;
    hipStream_t s = h->stream;

    const bool build = !cached;
    if (cached) {
        if (!cached->matches(h->n, h->h, h->prm) || cached->nv != h->nv || cached->nf != h->nf)
            return fail(REG_EINVAL, "cached object does not match the mesh, canvas or thresholds");
        h->obj = cached;
        // the object may still be in the making on the stream that built it
        if (cached->ready) DEV_TRY(h, hipStreamWaitEvent(s, cached->ready, 0));
    } else {
        auto o = std::make_shared<ObjectData>();
        o->n = h->n;
        o->h = h->h;
        o->nv = h->nv;
        o->nf = h->nf;
        o->tau_out1 = h->prm.tau_out1;
        o->tau_in1 = h->prm.tau_in1;
        o->rho = h->prm.rho;
        OBJ_ALLOC_TRY(o, o->V, 3 * (size_t)h->nv);
        OBJ_ALLOC_TRY(o, o->F, 3 * (size_t)h->nf);
        OBJ_ALLOC_TRY(o, o->touch, (size_t)h->nf);
        OBJ_ALLOC_TRY(o, o->anchor, 3);
        OBJ_ALLOC_TRY(o, o->O, n3);
        OBJ_ALLOC_TRY(o, o->fo, n3);
        OBJ_ALLOC_TRY(o, o->W, h->H);
        OBJ_ALLOC_TRY(o, o->Wlow, (size_t)NLOW3);
        OBJ_ALLOC_TRY(o, o->nz_idx, n3);
        OBJ_ALLOC_TRY(o, o->nz_val, n3);
        OBJ_ALLOC_TRY(o, o->nz_count, 1);
        OBJ_ALLOC_TRY(o, o->nz_bcount, (n3 + 255) / 256);
        OBJ_ALLOC_TRY(o, o->nz_boff, (n3 + 255) / 256);
        OBJ_ALLOC_TRY(o, o->tw, (size_t)h->n);
        OBJ_ALLOC_TRY(o, o->tw64, (size_t)h->n);
        h->obj = o;
    }
    ObjectData* o = h->obj.get();
    h->V = o->V;
    h->F = o->F;
    h->touch = o->touch;
    h->anchor = o->anchor;
    h->O = o->O;
    h->fo = o->fo;
    h->W = o->W;
    h->Wlow = o->Wlow;
    h->nz_idx = o->nz_idx;
    h->nz_val = o->nz_val;
    h->nz_count = o->nz_count;
    h->nz_bcount = o->nz_bcount;
    h->nz_boff = o->nz_boff;
    h->tw = o->tw;
    h->tw64 = o->tw64;

    ALLOC_TRY(h, h->poses, 7 * (size_t)n_poses);
    {
        const int rc = alloc_rotation_buffers(h, n_rot);
        if (rc) return rc;
    }
    ALLOC_TRY(h, h->pose_prep, 12 * (size_t)n_poses);
    if (build) {
        ALLOC_TRY(h, h->od2, n3);
        ALLOC_TRY(h, h->odt2, n3);
        ALLOC_TRY(h, h->opar, (size_t)h->n * h->n * ((h->n + 31) / 32));
    }
    ALLOC_TRY(h, h->spec, h->H * (size_t)h->batch);
    ALLOC_TRY(h, h->ptop, (size_t)h->batch * h->units * KREC);
    ALLOC_TRY(h, h->pssq, (size_t)h->batch * h->units);
    if (h->split) {
        ALLOC_TRY(h, h->xbuf, split_plane_elems(h->n) * (size_t)h->batch);
        ALLOC_TRY(h, h->lowrow, (size_t)h->n * h->n * NLX * (size_t)h->batch);
    }
    if (!h->rotobj) ALLOC_TRY(h, h->reach4, 1);
    ALLOC_TRY(h, h->stats, 5);
    ALLOC_TRY(h, h->need_count, 1);
    ALLOC_TRY(h, h->Sw, m3);
    ALLOC_TRY(h, h->cm, mp3);
    ALLOC_TRY(h, h->lowT, (size_t)h->batch * h->n * NLOW2);
    ALLOC_TRY(h, h->Plow, (size_t)h->batch * NLOW3);
    if (n_rot > h->batch && h->sched.lanes > 1) {  // a call can span two batches: the second lane
        ALLOC_TRY(h, h->spec2, h->H * (size_t)h->batch);
        ALLOC_TRY(h, h->ptop2, (size_t)h->batch * h->units * KREC);
        ALLOC_TRY(h, h->pssq2, (size_t)h->batch * h->units);
        if (h->split) {
            ALLOC_TRY(h, h->xbuf2, split_plane_elems(h->n) * (size_t)h->batch);
            ALLOC_TRY(h, h->lowrow2, (size_t)h->n * h->n * NLX * (size_t)h->batch);
        }
        ALLOC_TRY(h, h->lowT2, (size_t)h->batch * h->n * NLOW2);
        ALLOC_TRY(h, h->Plow2, (size_t)h->batch * NLOW3);
        DEV_TRY(h, hipStreamCreateWithFlags(&h->stream2, hipStreamNonBlocking));
        DEV_TRY(h, hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming));
        DEV_TRY(h, hipEventCreateWithFlags(&h->join_ev, hipEventDisableTiming));
    }
    ALLOC_TRY(h, h->err, 1);

    if (build) {
        DEV_TRY(h, hipMemcpyAsync(h->V, mesh->vertices, 12 * (size_t)h->nv, hipMemcpyDeviceToDevice, s));
        DEV_TRY(h, hipMemcpyAsync(h->F, mesh->faces, 12 * (size_t)h->nf, hipMemcpyDeviceToDevice, s));
        if (mesh->touchable)
            DEV_TRY(h, hipMemcpyAsync(h->touch, mesh->touchable, (size_t)h->nf, hipMemcpyDeviceToDevice, s));
        else
            DEV_TRY(h, hipMemsetAsync(h->touch, 1, (size_t)h->nf, s));
        // twiddles exp(-2 pi i t / n) in double, rounded to float
        std::vector<float2> tw(h->n);
        std::vector<double2> tw64(h->n);
        for (int t = 0; t < h->n; ++t) {
            const double ang = -2.0 * M_PI * (double)t / (double)h->n;
            tw64[t] = make_double2(std::cos(ang), std::sin(ang));
            tw[t] = make_float2((float)tw64[t].x, (float)tw64[t].y);
        }
        DEV_TRY(h, hipMemcpyAsync(h->tw, tw.data(), sizeof(float2) * h->n, hipMemcpyHostToDevice, s));
        DEV_TRY(h, hipMemcpyAsync(h->tw64, tw64.data(), sizeof(double2) * h->n, hipMemcpyHostToDevice, s));
    }
    DEV_TRY(h, hipMemcpyAsync(h->poses, poses, 28 * (size_t)n_poses, hipMemcpyDeviceToDevice, s));
    DEV_TRY(h, hipMemcpyAsync(h->so3, so3, 16 * (size_t)n_rot, hipMemcpyDeviceToDevice, s));

    // input checks on the device, then wait for them
    DEV_TRY(h, hipMemsetAsync(h->err, 0, sizeof(int), s));
    DEV_TRY(h, hipMemsetAsync(h->stats, 0, 5 * sizeof(int), s));
    DEV_TRY(h, validate_inputs(h->V, h->nv, h->F, h->nf, h->poses, n_poses, h->err, s));
    DEV_TRY(h, setup_rotations(h->so3, n_rot, h->rots, h->err, s, h->rotobj ? 1 : 0));
    int herr = 0;
    DEV_TRY(h, hipMemcpyAsync(&herr, h->err, sizeof(int), hipMemcpyDeviceToHost, s));
    DEV_TRY(h, hipStreamSynchronize(s));
    if (herr & REGK_ERR_NONFINITE) return fail(REG_EINVAL, "non-finite vertex or pose value");
    if (herr & REGK_ERR_FACE) return fail(REG_EINVAL, "face vertex index out of range");
    if (herr & REGK_ERR_QUAT) return fail(REG_EINVAL, "quaternion norm outside 1 +- 1e-3 (or not finite)");

    // object grid and spectrum (per object), swept occupancy (per request);
    // the refinement hierarchy is built on the host meanwhile
    if (build) {
        const int grc = start_refine_geometry(h);
        if (grc) return grc;
        DEV_TRY(h, setup_anchor(h->V, h->nv, h->anchor, s));
        DEV_TRY(h, setup_object_grid(h->V, h->F, h->touch, h->nf, h->n, h->h, h->anchor, h->prm.tau_out1,
                                     h->prm.tau_in1, h->prm.rho, h->O, h->fo,
                                     ObjectScratch{h->od2, h->odt2, h->opar}, s));
        int rc = build_object_derived(h);
        if (rc) return rc;
        DEV_TRY(h, hipEventCreateWithFlags(&h->obj->ready, hipEventDisableTiming));
        DEV_TRY(h, hipEventRecord(h->obj->ready, s));
    }
    DEV_TRY(h, setup_swept(h->poses, n_poses, probe->radius_mm, probe->length_mm, h->m, h->mp, h->h, h->wc,
                           h->pose_prep, h->Sw, h->cm, s));
    if (h->reach4) DEV_TRY(h, swept_reach(h->Sw, h->m, h->reach4, s));
    if (h->rotobj) {
        const int rc = build_rotated_object(h);
        if (rc) return rc;
    }
    *out = h;
    h = nullptr;  // release the guard
    return REG_OK;
}

// Refinement rounds on the handle's stream until no start is left (checked
// every 4 rounds), then the results.  Every round evaluates the next trials
// of each unfinished start and settles at least one of its trial steps; a
// start takes at most max_iters accepted steps and the damping can grow 3x at
// most 51 times in a row, which bounds the rounds.
static int refine_continue(reg_handle* h, int K, double* out_poses, double* out_J, int32_t* out_iters) {
    const RefineConst c = refine_const(h);
    hipStream_t s = h->stream;
    // Gauss-Newton: at most 51 rejections in a row; L-BFGS-B: at most 9
    // backtracking rounds per iteration and one restart from steepest descent
    const long max_rounds = 1 + (long)(c.max_iters + 1) * (h->r_lbfgsb ? 20 : 52);
    DEV_TRY(h, hipMemcpyAsync(h->r_active_host, h->r_active, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    DEV_TRY(h, hipStreamSynchronize(s));
    long round = h->r_rounds;
    while (h->r_active_host[0] > 0 && round < max_rounds) {
        if (h->r_lbfgsb)
            DEV_TRY(h, refine_round_lbfgsb(h->rst, h->rlb, h->rtr, K, h->obj->geo, h->poses, h->n_poses, c, h->rw,
                                           h->rhits, h->rev, h->r_active, s));
        else
            DEV_TRY(h, refine_round(h->rst, h->rtr, K, h->obj->geo, h->poses, h->n_poses, c, h->rw, h->rhits, h->rev,
                                    h->r_active, s));
        ++round;
        if (round % 4 == 0 || round == max_rounds) {
            DEV_TRY(h, hipMemcpyAsync(h->r_active_host, h->r_active, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
            DEV_TRY(h, hipStreamSynchronize(s));
        }
    }
    DEV_TRY(h, refine_finish(h->rst, K, out_poses, out_J, out_iters, s));
    DEV_TRY(h, hipMemcpyAsync(h->r_active_host, h->r_active, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    DEV_TRY(h, hipStreamSynchronize(s));
    h->r_rounds = round;
    h->r_evals = h->r_active_host[1];
    return REG_OK;
}

// ------------------------------------------------------------- batching
//
// Many registrations of uneven canvases in one captured hipGraph: the search
// over every rotation, the top K and a fixed budget of refinement rounds of
// each handle go onto one of a few parallel branches (streams forked from and
// joined to the launch stream), balanced by their model HBM bytes.  Rounds
// after a start has finished are no-ops, so the captured budget gives the
// same result as the host-driven loop; a start still running afterwards is
// continued on its handle's stream.
struct reg_batch {
    struct Out {
        float* score = nullptr;
        double* pose = nullptr;
        int32_t* top = nullptr;
        double* init = nullptr;
        double* refined = nullptr;
        double* J = nullptr;
        int32_t* iters = nullptr;
    };
    std::vector<reg_handle*> hs;
    std::vector<int> K, branch_of;
    std::vector<Out> out;
    int rounds = 0, refine = 1;  // refine: 0 none, 1 Gauss-Newton, 2 L-BFGS-B
    hipStream_t main = nullptr;
    std::vector<hipStream_t> br;
    std::vector<hipEvent_t> ev;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<void*> owned;
    ~reg_batch() {
        // replays still queued must finish before the blocks are reused
        if (main) (void)hipStreamSynchronize(main);
        for (auto s : br) (void)hipStreamSynchronize(s);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (auto e : ev) (void)hipEventDestroy(e);
        for (auto s : br) (void)hipStreamDestroy(s);
        if (main) (void)hipStreamDestroy(main);
        for (void* p : owned) regdock_rt::dev_release(p);
        for (reg_handle* h : hs) --h->in_batches;
    }
    template <class T>
    bool alloc(T** p, size_t count) {
        void* q = nullptr;
        if (regdock_rt::dev_alloc(&q, count * sizeof(T) > 0 ? count * sizeof(T) : 1) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        owned.push_back(q);
        *p = (T*)q;
        return true;
    }
};

static int run_batches(reg_handle* h, int first, int count, float* out_score, int32_t* out_shift, double* out_pose,
                       float* corr_out);

// enqueue one handle's registration on stream s (captured)
static int batch_enqueue(reg_batch* b, int i, hipStream_t s) {
    reg_handle* h = b->hs[i];
    const reg_batch::Out& o = b->out[i];
    hipStream_t saved = h->stream;
    h->stream = s;
    struct Restore {
        reg_handle* h;
        hipStream_t s;
        ~Restore() { h->stream = s; }
    } rs{h, saved};
    int rc = run_batches(h, 0, h->n_rot, o.score, nullptr, o.pose, nullptr);
    if (rc) return rc;
    const int K = b->K[i];
    DEV_TRY(h, top_k(o.score, h->n_rot, K, o.top, s));
    if (!b->refine) return REG_OK;
    DEV_TRY(h, gather_poses(o.top, o.pose, K, o.init, s));
    const RefineConst c = refine_const(h);
    DEV_TRY(h, refine_start(o.init, K, h->anchor, c, h->rst, h->rtr, h->r_active, h->rw, s));
    for (int r = 0; r < b->rounds; ++r) {
        if (b->refine == 2)
            DEV_TRY(h, refine_round_lbfgsb(h->rst, h->rlb, h->rtr, K, h->obj->geo, h->poses, h->n_poses, c, h->rw,
                                           h->rhits, h->rev, h->r_active, s));
        else
            DEV_TRY(h, refine_round(h->rst, h->rtr, K, h->obj->geo, h->poses, h->n_poses, c, h->rw, h->rhits, h->rev,
                                    h->r_active, s));
    }
    DEV_TRY(h, refine_finish(h->rst, K, o.refined, o.J, o.iters, s));
    return REG_OK;
}

// The schedule timed on the handle's own problem (its first M rotations):
// each pass's workgroup variants alone (event-timed launches, one lane), then
// rotation batches on one and two lanes with the chosen kernels (the whole
// search, event-timed on the handle's stream).  The fastest is recorded for
// the handle's canvas edge.
static int autotune_impl(reg_handle* h, int max_rotations, int* out_batch) {
    const int M = std::max(8, std::min(h->n_rot, max_rotations > 0 ? max_rotations : 512));
    float* score = nullptr;
    if (hipMalloc((void**)&score, (size_t)M * 4) != hipSuccess) {
        (void)hipGetLastError();
        return fail(REG_ENOMEM, "autotune score buffer");
    }
    struct FreeS {
        float* p;
        ~FreeS() { (void)hipFree(p); }
    } fs{score};
    hipEvent_t e0, e1;
    DEV_TRY(h, hipEventCreate(&e0));
    DEV_TRY(h, hipEventCreate(&e1));
    struct FreeE {
        hipEvent_t a, b;
        ~FreeE() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } fe{e0, e1};
    reg_mesh mesh{h->V, h->nv, h->F, h->nf, h->touch};
    reg_grid_spec grid{h->n, h->h, {h->wc[0], h->wc[1], h->wc[2]}};
    struct FreeH {
        reg_handle* t = nullptr;
        ~FreeH() {
            if (t) register_free(t);
        }
    };
    auto make = [&](int B, int lanes, FreeH& fh) -> int {
        reg_params prm = h->prm;
        prm.batch = B;
        prm.lanes = lanes;
        prm.plane_variant = 0;
        prm.z_variant = 0;
        return init_impl(&mesh, &h->probe, h->poses, h->n_poses, h->so3, M, &grid, &prm, (void*)h->stream, h->obj,
                         &fh.t);
    };
    // per-pass time (us per rotation) of the timed launches of t
    auto pass_us = [&](reg_handle* t, double* us) -> int {
        double ms[3] = {0, 0, 0};
        long rot[3] = {0, 0, 0};
        DEV_TRY(t, hipStreamSynchronize(t->stream));
        for (const auto& x : t->timed) {
            float e = 0;
            DEV_TRY(t, hipEventElapsedTime(&e, x.a, x.b));
            ms[x.kernel] += e;
            rot[x.kernel] += x.rotations;
        }
        for (int k = 0; k < 3; ++k) us[k] = rot[k] ? 1e3 * ms[k] / (double)rot[k] : INFINITY;
        return REG_OK;
    };
    Schedule best;
    best.us1 = best.usz = best.us3 = INFINITY;
    {
        // kernel variants on a batch of the default size, one lane
        const int B0 = std::min(default_batch(h->n, h->H, M), ((M + 7) / 8) * 8);
        FreeH fh;
        int rc = make(B0, 1, fh);
        if (rc) return rc;
        reg_handle* t = fh.t;
        const int cnt = std::min(M, 2 * t->batch);
        best.pv1 = best.pv3 = t->sched.pv1;
        best.zv = t->sched.zv;
        for (int v = 0; v < PLANE_VARIANTS; ++v) {
            if (!plane_variant_ok(h->n, v)) continue;
            t->sched.pv1 = t->sched.pv3 = v;
            t->timing = false;
            rc = run_batches(t, 0, cnt, score, nullptr, nullptr, nullptr);  // warm-up
            if (rc) return rc;
            DEV_TRY(t, hipStreamSynchronize(t->stream));
            t->timing = true;
            t->timed.clear();
            t->pool_used = 0;
            for (int rep = 0; rep < 2 && !rc; ++rep) rc = run_batches(t, 0, cnt, score, nullptr, nullptr, nullptr);
            if (rc) return rc;
            double us[3];
            rc = pass_us(t, us);
            if (rc) return rc;
            if (us[0] < best.us1) {
                best.us1 = us[0];
                best.pv1 = v;
            }
            if (us[2] < best.us3) {
                best.us3 = us[2];
                best.pv3 = v;
            }
        }
        t->sched.pv1 = best.pv1;
        t->sched.pv3 = best.pv3;
        for (int v = 0; v < Z_VARIANTS; ++v) {
            if (!z_variant_ok(h->n, v)) continue;
            t->sched.zv = v;
            t->timing = false;
            rc = run_batches(t, 0, cnt, score, nullptr, nullptr, nullptr);
            if (rc) return rc;
            DEV_TRY(t, hipStreamSynchronize(t->stream));
            t->timing = true;
            t->timed.clear();
            t->pool_used = 0;
            for (int rep = 0; rep < 2 && !rc; ++rep) rc = run_batches(t, 0, cnt, score, nullptr, nullptr, nullptr);
            if (rc) return rc;
            double us[3];
            rc = pass_us(t, us);
            if (rc) return rc;
            if (us[1] < best.usz) {
                best.usz = us[1];
                best.zv = v;
            }
        }
        t->timing = false;
    }
    // rotation batch and lanes with the chosen kernels
    double best_t = INFINITY;
    for (int B : {8, 16, 32, 64, 128, 256, 512}) {
        if ((size_t)B * h->H * sizeof(float2) > ((size_t)2 << 30) || B > ((M + 7) / 8) * 8) continue;
        for (int lanes = 1; lanes <= 2; ++lanes) {
            if (lanes == 2 && B >= M) continue;
            FreeH fh;
            int rc = make(B, lanes, fh);
            if (rc == REG_ENOMEM) continue;
            if (rc) return rc;
            reg_handle* t = fh.t;
            t->sched.pv1 = best.pv1;
            t->sched.pv3 = best.pv3;
            t->sched.zv = best.zv;
            rc = run_batches(t, 0, M, score, nullptr, nullptr, nullptr);  // warm-up
            if (!rc) {
                DEV_TRY(h, hipEventRecord(e0, h->stream));
                for (int rep = 0; rep < 2 && !rc; ++rep) rc = run_batches(t, 0, M, score, nullptr, nullptr, nullptr);
                DEV_TRY(h, hipEventRecord(e1, h->stream));
                DEV_TRY(h, hipEventSynchronize(e1));
            }
            if (rc) return rc;
            float ms = 0;
            DEV_TRY(h, hipEventElapsedTime(&ms, e0, e1));
            if (ms < best_t) {
                best_t = ms;
                best.batch = B;
                best.lanes = lanes;
            }
        }
    }
    if (!best.batch) return fail(REG_ENOMEM, "no rotation batch fits in device memory");
    best.ns_rot = 1e6 * best_t / (2.0 * M);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[h->n] = best;
    }
    *out_batch = best.batch;
    return REG_OK;
}

extern "C" {

const char* register_last_error(void) { return g_err.c_str(); }

int register_init(const reg_mesh* mesh, const reg_probe* probe, const float* poses, int32_t n_poses, const float* so3,
                  int32_t n_rot, const reg_grid_spec* grid, const reg_params* params, void* hip_stream, reg_handle** out) {
    return init_impl(mesh, probe, poses, n_poses, so3, n_rot, grid, params, hip_stream, nullptr, out);
}

void register_free(reg_handle* h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    delete h;
}

// ------------------------------------------------------ linear correlation

// Both supports are bounded by spheres about the canvas centre: the object's
// by the vertex radius about the anchor plus tau_out1 (O vanishes farther out
// of the mesh), the rotated swept occupancy's by the trajectory's farthest
// probe point from center_world plus sqrt(3) h, the reach of its trilinear
// resampling.  A sphere of radius R holds 2 floor(R / h) + 1 grid points along
// an axis, and the circular correlation of the canvas equals the linear one
// once n >= n_o + n_s - 1 (Sec. IV-B).
int register_linear_edge(const float* vertices, int32_t n_vertices, const reg_probe* probe, const float* poses,
                         int32_t n_poses, const double* center_world, double h_mm, double tau_out1, int32_t* needed,
                         int32_t* edge) {
    g_err.clear();
    if (!vertices || n_vertices < 1 || !probe || !poses || n_poses < 1 || !center_world || !needed || !edge)
        return fail(REG_EINVAL, "register_linear_edge: NULL argument or empty mesh/trajectory");
    if (!(h_mm > 0) || !std::isfinite(h_mm) || !(probe->radius_mm > 0) || !(probe->length_mm > 0) ||
        !std::isfinite(probe->radius_mm) || !std::isfinite(probe->length_mm))
        return fail(REG_EINVAL, "register_linear_edge: h and the probe dimensions must be finite and > 0");
    if (!(tau_out1 > 0)) tau_out1 = 0.5;
    double a[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < n_vertices; ++i)
        for (int k = 0; k < 3; ++k) {
            if (!std::isfinite(vertices[3 * i + k])) return fail(REG_EINVAL, "vertex %d is not finite", i);
            a[k] += vertices[3 * i + k];
        }
    for (int k = 0; k < 3; ++k) a[k] /= n_vertices;
    double ro = 0.0;
    for (int i = 0; i < n_vertices; ++i) {
        const double dx = vertices[3 * i] - a[0], dy = vertices[3 * i + 1] - a[1], dz = vertices[3 * i + 2] - a[2];
        ro = std::max(ro, std::sqrt(dx * dx + dy * dy + dz * dz));
    }
    const double r = probe->radius_mm, L = probe->length_mm;
    double rs = 0.0;
    for (int i = 0; i < n_poses; ++i) {
        const float* P = poses + 7 * i;
        for (int k = 0; k < 7; ++k)
            if (!std::isfinite(P[k])) return fail(REG_EINVAL, "pose %d is not finite", i);
        const double qn = std::sqrt((double)P[0] * P[0] + (double)P[1] * P[1] + (double)P[2] * P[2] + (double)P[3] * P[3]);
        if (!(qn > 0)) return fail(REG_EINVAL, "pose %d has a zero quaternion", i);
        const double w = P[0] / qn, x = P[1] / qn, y = P[2] / qn, z = P[3] / qn;
        const double ax[3] = {2 * (x * z + w * y), 2 * (y * z - w * x), 1 - 2 * (x * x + y * y)};  // probe axis
        for (int e = 0; e < 2; ++e) {  // tip disk and far disk: the farthest point is on a rim
            double v[3];
            for (int k = 0; k < 3; ++k) v[k] = P[4 + k] + e * L * ax[k] - center_world[k];
            const double al = v[0] * ax[0] + v[1] * ax[1] + v[2] * ax[2];
            double pr2 = 0.0;
            for (int k = 0; k < 3; ++k) pr2 += (v[k] - al * ax[k]) * (v[k] - al * ax[k]);
            const double b = std::sqrt(pr2) + r;
            rs = std::max(rs, std::sqrt(al * al + b * b));
        }
    }
    const double no = 2.0 * std::floor((ro + tau_out1) / h_mm) + 1.0;
    const double ns = 2.0 * std::floor(rs / h_mm + std::sqrt(3.0)) + 1.0;
    const double need = no + ns - 1.0;
    *needed = need > 2147483647.0 ? 2147483647 : (int32_t)need;
    *edge = 0;
    constexpr int kMaxEdge = 1024;  // above every supported edge
    for (int n = (int)std::min(need, (double)kMaxEdge + 1); n <= kMaxEdge; ++n)
        if (canvas_supported(n)) {
            *edge = n;
            break;
        }
    if (*edge == 0)
        return fail(REG_ENOTSUP, "the linear correlation needs a canvas edge >= %d, above every supported edge",
                    (int)*needed);
    return REG_OK;
}

// ------------------------------------------------------ orientation samplers

int so3_super_fibonacci(int32_t n, float* out, void* hip_stream) {
    if (n < 1 || !out) return fail(REG_EINVAL, "n >= 1 and an output buffer are required");
    if (n > SO3_SAMPLER_MAX_N) return fail(REG_EINVAL, "n = %d exceeds SO3_SAMPLER_MAX_N", n);
    hipStream_t s = (hipStream_t)hip_stream;
    reg_handle* none = nullptr;
    DEV_TRY(none, super_fibonacci(n, out, s));
    DEV_TRY(none, hipStreamSynchronize(s));
    return REG_OK;
}

int so3_geoball_sf(int32_t n, const double* q0, double theta, double gamma, float* out, void* hip_stream) {
    if (n < 1 || !out || !q0) return fail(REG_EINVAL, "n >= 1, q0 and an output buffer are required");
    if (n > SO3_SAMPLER_MAX_N) return fail(REG_EINVAL, "n = %d exceeds SO3_SAMPLER_MAX_N", n);
    double qn = 0.0;
    for (int j = 0; j < 4; ++j) {
        if (!std::isfinite(q0[j])) return fail(REG_EINVAL, "non-finite q0");
        qn += q0[j] * q0[j];
    }
    if (!(qn > 1e-12)) return fail(REG_EINVAL, "q0 has zero norm");
    if (!(theta > 0.0 && theta <= 0.5 * M_PI)) return fail(REG_EINVAL, "theta must lie in (0, pi/2]");
    if (!(gamma >= 0.0) || !std::isfinite(gamma)) return fail(REG_EINVAL, "gamma must be >= 0 (0: gamma = n)");
    reg_handle* none = nullptr;
    DEV_TRY(none, geoball_sf(n, q0, theta, gamma, out, (hipStream_t)hip_stream));
    return REG_OK;
}

int so3_geoball_sf_noalloc(int32_t n, const double* q0, double theta, double gamma, float* out, void* hip_stream) {
    if (n < 1 || !out || !q0) return fail(REG_EINVAL, "n >= 1, q0 and an output buffer are required");
    double qn = 0.0;
    for (int j = 0; j < 4; ++j) {
        if (!std::isfinite(q0[j])) return fail(REG_EINVAL, "non-finite q0");
        qn += q0[j] * q0[j];
    }
    if (!(qn > 1e-12)) return fail(REG_EINVAL, "q0 has zero norm");
    if (!(theta > 0.0 && theta <= 0.5 * M_PI)) return fail(REG_EINVAL, "theta must lie in (0, pi/2]");
    if (!(gamma >= 0.0) || !std::isfinite(gamma)) return fail(REG_EINVAL, "gamma must be >= 0 (0: gamma = n)");
    if (n > SO3_SAMPLER_MAX_N) return fail(REG_EINVAL, "n = %d exceeds SO3_SAMPLER_MAX_N", n);
    reg_handle* none = nullptr;
    DEV_TRY(none, geoball_sf_noalloc(n, q0, theta, gamma, out, (hipStream_t)hip_stream));
    return REG_OK;
}

int register_set_rotations(reg_handle* h, const float* so3, int32_t n_rot) {
    if (!h || !so3) return fail(REG_EINVAL, "NULL argument");
    if (h->poisoned) return fail(REG_EDEVICE, "handle unusable after a device error");
    if (n_rot < 1) return fail(REG_EINVAL, "n_rot must be >= 1");
    if (h->in_batches > 0)
        return fail(REG_EBUSY, "a live batch captured this handle's rotation set; free the batch first");
    hipStream_t s = h->stream;
    DEV_TRY(h, hipStreamSynchronize(s));
    if (n_rot > h->rot_cap) {
        const int rc = alloc_rotation_buffers(h, n_rot);
        if (rc) return rc;
    }
    DEV_TRY(h, hipMemcpyAsync(h->so3, so3, 16 * (size_t)n_rot, hipMemcpyDeviceToDevice, s));
    DEV_TRY(h, hipMemsetAsync(h->err, 0, sizeof(int), s));
    DEV_TRY(h, setup_rotations(h->so3, n_rot, h->rots, h->err, s, h->rotobj ? 1 : 0));
    int herr = 0;
    DEV_TRY(h, hipMemcpyAsync(&herr, h->err, sizeof(int), hipMemcpyDeviceToHost, s));
    DEV_TRY(h, hipStreamSynchronize(s));
    h->n_rot = 0;  // unusable until the new set is known to be valid
    if (herr & REGK_ERR_QUAT) return fail(REG_EINVAL, "quaternion norm outside 1 +- 1e-3 (or not finite)");
    h->n_rot = n_rot;
    return REG_OK;
}

int64_t register_cached_bytes(void) { return (int64_t)regdock_rt::dev_cached_bytes(); }

void register_release_cached(void) { regdock_rt::dev_trim(); }

int register_info(const reg_handle* h, int32_t* n, int32_t* m, int64_t* spectrum_elems_out, int32_t* batch, int32_t* n_rot) {
    if (!h) return fail(REG_EINVAL, "NULL handle");
    if (n) *n = h->n;
    if (m) *m = h->m;
    if (spectrum_elems_out) *spectrum_elems_out = (int64_t)h->H;
    if (batch) *batch = h->batch;
    if (n_rot) *n_rot = h->n_rot;
    return REG_OK;
}

static PeakArrays peak_arrays(reg_handle* h) {
    return PeakArrays{h->cand_idx, h->cand_n, h->window, h->ovf, h->best_val, h->best_flat,
                      h->need_list, h->need_count, h->cand_part, h->stats};
}

// One rotation batch [b0, b0 + cnt) of the handle's set through the three
// search passes and the per-rotation candidate selection, on stream ls with
// pass-buffer set `lane` (1: the second set, which exists when the set spans
// more than one batch).  after_plane_pass, when given, is recorded on ls once
// the batch's first pass is enqueued.
static int enqueue_batch(reg_handle* h, int b0, int cnt, int lane, hipStream_t ls, float* corr_out,
                         hipEvent_t after_plane_pass = nullptr) {
    const bool odd = lane == 1;
    SearchBatchArgs a{};
    a.cmask = h->rotobj ? h->ocls : h->cm;
    a.crec = h->orec;
    a.cval = (float)(-h->prm.rho);
    a.m = h->m;
    a.mp = h->mp;
    a.rots = h->rots + 9 * (size_t)b0;
    a.count = cnt;
    a.tw = h->tw;
    a.spec = odd ? h->spec2 : h->spec;
    a.W = h->W;
    a.tw64 = h->tw64;
    a.lowT = odd ? h->lowT2 : h->lowT;
    a.Wlow = h->Wlow;
    a.Plow = odd ? h->Plow2 : h->Plow;
    a.ptop = odd ? h->ptop2 : h->ptop;
    a.pssq = odd ? h->pssq2 : h->pssq;
    a.units = h->units;
    a.xbuf = odd ? h->xbuf2 : h->xbuf;
    a.lowrow = odd ? h->lowrow2 : h->lowrow;
    a.reach4 = h->reach4;
    a.corr_out = corr_out;
    a.pv1 = h->sched.pv1;
    a.pv3 = h->sched.pv3;
    a.zv = h->sched.zv;
    a.stream = ls;
    for (int pass = 0; pass < 3; ++pass) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (h->timing) {
            e0 = h->next_event();
            e1 = h->next_event();
            if (!e0 || !e1) return fail(REG_EDEVICE, "hipEventCreate failed");
            DEV_TRY(h, hipEventRecord(e0, ls));
        }
        DEV_TRY(h, search_pass(h->n, pass, a));
        if (h->timing) {
            DEV_TRY(h, hipEventRecord(e1, ls));
            h->timed.push_back({e0, e1, pass, cnt});
        }
        if (pass == 0 && after_plane_pass) DEV_TRY(h, hipEventRecord(after_plane_pass, ls));
    }
    DEV_TRY(h, select_batch(h->n, a, b0, peak_arrays(h)));
    return REG_OK;
}

// certification, exact re-scoring and the outputs of rotations [first, first + count)
static int enqueue_finish(reg_handle* h, int first, int count, float* out_score, int32_t* out_shift, double* out_pose,
                          hipStream_t s) {
    const RescoreInputs ri{h->nz_idx,  h->nz_val, h->nz_count,          h->rotobj ? h->ocls : h->cm, h->m, h->mp,
                           h->rots,    h->orec,   (float)(-h->prm.rho)};
    DEV_TRY(h, finish_call(h->n, first, count, h->prm.rescore != 0, peak_arrays(h), ri, h->so3 + 4 * (size_t)first,
                           h->h, h->anchor, h->wc, out_score, out_shift, out_pose, s));
    return REG_OK;
}

static int run_batches(reg_handle* h, int first, int count, float* out_score, int32_t* out_shift, double* out_pose,
                       float* corr_out) {
    // two lanes when the schedule asks for them and the call spans more than
    // one batch: even batches on the handle's stream, odd ones on stream2
    // (forked from it here and joined back before the call's last step); each
    // lane keeps its own pass buffers.  Not under graph capture, whose batches
    // already run on parallel branches (a fork of stream2 inside the capture
    // crashed register_batch_create).
    hipStreamCaptureStatus capture = hipStreamCaptureStatusNone;
    DEV_TRY(h, hipStreamIsCapturing(h->stream, &capture));
    const bool two = h->stream2 && h->sched.lanes > 1 && count > h->batch && capture == hipStreamCaptureStatusNone;
    for (int b0 = 0, j = 0; b0 < count; b0 += h->batch, ++j) {
        const int cnt = count - b0 < h->batch ? count - b0 : h->batch;
        const bool odd = two && (j & 1);
        // the second lane starts once the first batch's plane pass is done,
        // half a batch out of phase: its plane passes then meet the first
        // lane's z pass more often than its plane passes
        const int rc = enqueue_batch(h, first + b0, cnt, odd ? 1 : 0, odd ? h->stream2 : h->stream, corr_out,
                                     two && j == 0 ? h->fork_ev : nullptr);
        if (rc) return rc;
        if (two && j == 0) DEV_TRY(h, hipStreamWaitEvent(h->stream2, h->fork_ev, 0));
    }
    if (two) {
        DEV_TRY(h, hipEventRecord(h->join_ev, h->stream2));
        DEV_TRY(h, hipStreamWaitEvent(h->stream, h->join_ev, 0));
    }
    return enqueue_finish(h, first, count, out_score, out_shift, out_pose, h->stream);
}

int score_rotations(reg_handle* h, int32_t first, int32_t count, float* out_score, int32_t* out_shift, double* out_pose) {
    g_err.clear();
    if (!h) return fail(REG_EINVAL, "NULL handle");
    if (h->poisoned) return fail(REG_EDEVICE, "handle poisoned by an earlier device error");
    if (!out_score) return fail(REG_EINVAL, "out_score is NULL");
    if (first < 0 || count < 0 || (int64_t)first + count > h->n_rot)
        return fail(REG_EINVAL, "rotation range [%d, %d) outside [0, %d)", first, first + count, h->n_rot);
    if (count == 0) return REG_OK;
    return run_batches(h, first, count, out_score, out_shift, out_pose, nullptr);
}

int register_set_timing(reg_handle* h, int32_t enable) {
    if (!h) return fail(REG_EINVAL, "NULL handle");
    DEV_TRY(h, hipStreamSynchronize(h->stream));
    h->timing = enable != 0;
    h->timed.clear();
    h->pool_used = 0;
    return REG_OK;
}

int register_get_timing(reg_handle* h, double* ms, int64_t* launches, int64_t* rotations) {
    if (!h || !ms || !launches || !rotations) return fail(REG_EINVAL, "NULL argument");
    DEV_TRY(h, hipStreamSynchronize(h->stream));
    for (int k = 0; k < 3; ++k) {
        ms[k] = 0;
        launches[k] = 0;
        rotations[k] = 0;
    }
    for (const auto& t : h->timed) {
        float e = 0;
        DEV_TRY(h, hipEventElapsedTime(&e, t.a, t.b));
        ms[t.kernel] += e;
        launches[t.kernel] += 1;
        rotations[t.kernel] += t.rotations;
    }
    return REG_OK;
}

int register_search_stats(reg_handle* h, int64_t* rotations, int64_t* candidates, int64_t* overflows,
                          int64_t* uncertain, int64_t* rescored) {
    if (!h || !rotations || !candidates || !overflows || !uncertain || !rescored)
        return fail(REG_EINVAL, "NULL argument");
    if (h->poisoned) return fail(REG_EDEVICE, "handle poisoned by an earlier device error");
    int st[5] = {0, 0, 0, 0, 0};
    DEV_TRY(h, hipMemcpyAsync(st, h->stats, sizeof st, hipMemcpyDeviceToHost, h->stream));
    DEV_TRY(h, hipStreamSynchronize(h->stream));
    *rotations = st[0];
    *candidates = st[1];
    *overflows = st[2];
    *uncertain = st[3];
    *rescored = st[4];
    return REG_OK;
}

int register_top_k(reg_handle* h, const float* scores, int32_t count, int32_t K, int32_t* out_idx) {
    g_err.clear();
    if (!h) return fail(REG_EINVAL, "NULL handle");
    if (h->poisoned) return fail(REG_EDEVICE, "handle poisoned by an earlier device error");
    if (!scores || !out_idx || count < 1 || K < 1) return fail(REG_EINVAL, "bad top-k arguments");
    DEV_TRY(h, top_k(scores, count, K, out_idx, h->stream));
    return REG_OK;
}

int register_debug_object_grid(reg_handle* h, float* out_O, float* out_fo) {
    if (!h || !out_O) return fail(REG_EINVAL, "NULL argument");
    if (h->poisoned) return fail(REG_EDEVICE, "handle poisoned by an earlier device error");
    const size_t n3 = (size_t)h->n * h->n * h->n;
    DEV_TRY(h, hipMemcpyAsync(out_O, h->O, n3 * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    if (out_fo) DEV_TRY(h, hipMemcpyAsync(out_fo, h->fo, n3 * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    return REG_OK;
}

int register_debug_swept(reg_handle* h, uint8_t* out_Sw) {
    if (!h || !out_Sw) return fail(REG_EINVAL, "NULL argument");
    if (h->poisoned) return fail(REG_EDEVICE, "handle poisoned by an earlier device error");
    const size_t m3 = (size_t)h->m * h->m * h->m;
    DEV_TRY(h, hipMemcpyAsync(out_Sw, h->Sw, m3, hipMemcpyDeviceToDevice, h->stream));
    return REG_OK;
}

int register_debug_swept_reach(reg_handle* h, int64_t* out_reach4) {
    if (!h || !out_reach4) return fail(REG_EINVAL, "NULL argument");
    if (h->poisoned) return fail(REG_EDEVICE, "handle poisoned by an earlier device error");
    if (!h->reach4) return fail(REG_ENOTSUP, "the rotated-object search does not compute the swept lattice's reach");
    unsigned long long v = 0;
    DEV_TRY(h, hipMemcpyAsync(&v, h->reach4, sizeof(v), hipMemcpyDeviceToHost, h->stream));
    DEV_TRY(h, hipStreamSynchronize(h->stream));
    *out_reach4 = (int64_t)v;
    return REG_OK;
}

int register_debug_correlation(reg_handle* h, int32_t rot, float* out_C) {
    if (!h || !out_C) return fail(REG_EINVAL, "NULL argument");
    if (h->poisoned) return fail(REG_EDEVICE, "handle poisoned by an earlier device error");
    if (rot < 0 || rot >= h->n_rot) return fail(REG_EINVAL, "rotation %d outside [0, %d)", rot, h->n_rot);
    return run_batches(h, rot, 1, nullptr, nullptr, nullptr, out_C);
}

int register_set_grids(reg_handle* h, const float* O, const uint8_t* Sw) {
    if (!h) return fail(REG_EINVAL, "NULL handle");
    if (h->poisoned) return fail(REG_EDEVICE, "handle poisoned by an earlier device error");
    if (h->rotobj) return fail(REG_ENOTSUP, "grid injection is not offered for the rotated-object search");
    if (O) {
        const size_t n3 = (size_t)h->n * h->n * h->n;
        DEV_TRY(h, hipMemcpyAsync(h->O, O, n3 * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
        int rc = build_object_derived(h);
        if (rc) return rc;
    }
    if (Sw) {
        const size_t m3 = (size_t)h->m * h->m * h->m;
        DEV_TRY(h, hipMemcpyAsync(h->Sw, Sw, m3, hipMemcpyDeviceToDevice, h->stream));
        DEV_TRY(h, setup_cellmask(h->Sw, h->m, h->mp, h->cm, h->stream));
        if (h->reach4) DEV_TRY(h, swept_reach(h->Sw, h->m, h->reach4, h->stream));
    }
    return REG_OK;
}

static int refine_impl(reg_handle* h, const double* init_poses, int32_t K, double* out_poses, double* out_J,
                       int32_t* out_iters, bool lbfgsb) {
    g_err.clear();
    if (!h) return fail(REG_EINVAL, "NULL handle");
    if (h->poisoned) return fail(REG_EDEVICE, "handle poisoned by an earlier device error");
    if (!init_poses || !out_poses || K < 1) return fail(REG_EINVAL, "refine_se3 needs K >= 1 and non-NULL poses");
    std::vector<double> init(7 * (size_t)K);
    DEV_TRY(h, hipMemcpyAsync(init.data(), init_poses, init.size() * 8, hipMemcpyDeviceToHost, h->stream));
    DEV_TRY(h, hipStreamSynchronize(h->stream));
    for (int k = 0; k < K; ++k) {
        const double* q = &init[7 * (size_t)k];
        for (int j = 0; j < 7; ++j)
            if (!std::isfinite(q[j])) return fail(REG_EINVAL, "initial pose %d is not finite", k);
        const double nq = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        if (std::fabs(nq - 1.0) > 1e-3) return fail(REG_EINVAL, "initial pose %d: quaternion norm %g", k, nq);
    }
    int rc = ensure_refine_buffers(h, K);
    if (rc) return rc;
    DEV_TRY(h, refine_start(init_poses, K, h->anchor, refine_const(h), h->rst, h->rtr, h->r_active, h->rw, h->stream));
    h->r_rounds = 0;
    h->r_lbfgsb = lbfgsb;
    const int rc2 = refine_continue(h, K, out_poses, out_J, out_iters);
    h->r_lbfgsb = false;
    return rc2;
}

int refine_se3(reg_handle* h, const double* init_poses, int32_t K, double* out_poses, double* out_J,
               int32_t* out_iters) {
    return refine_impl(h, init_poses, K, out_poses, out_J, out_iters, false);
}

int refine_se3_lbfgsb(reg_handle* h, const double* init_poses, int32_t K, double* out_poses, double* out_J,
                      int32_t* out_iters) {
    return refine_impl(h, init_poses, K, out_poses, out_J, out_iters, true);
}

int register_refine_stats(reg_handle* h, int64_t* rounds, int64_t* evaluations) {
    if (!h || !rounds || !evaluations) return fail(REG_EINVAL, "NULL argument");
    *rounds = h->r_rounds;
    *evaluations = h->r_evals;
    return REG_OK;
}

int register_batch_create(reg_handle* const* handles, int32_t count, int32_t top_k, int32_t refine,
                          int32_t graph_rounds, int32_t branches, reg_batch** out) {
    g_err.clear();
    if (!handles || !out || count < 1) return fail(REG_EINVAL, "register_batch_create needs >= 1 handle");
    *out = nullptr;
    if (top_k < 1 || top_k > 16) return fail(REG_EINVAL, "top_k must be in [1, 16]");
    auto b = std::make_unique<reg_batch>();
    if (refine < 0 || refine > 2) return fail(REG_EINVAL, "refine must be 0, 1 or 2");
    b->refine = refine;
    b->rounds = graph_rounds > 0 ? graph_rounds : 64;
    const int nb = std::max(1, std::min<int>(branches > 0 ? branches : 4, count));
    for (int i = 0; i < count; ++i) {
        reg_handle* h = handles[i];
        if (!h) return fail(REG_EINVAL, "handle %d is NULL", i);
        if (h->poisoned) return fail(REG_EDEVICE, "handle %d is poisoned", i);
        if (h->timing) return fail(REG_EINVAL, "handle %d has event timing on (not capturable)", i);
        for (int j = 0; j < i; ++j)
            if (handles[j] == h) return fail(REG_EINVAL, "handle %d appears twice", i);
        b->hs.push_back(h);
        ++h->in_batches;  // released by ~reg_batch
        const int K = std::min<int>(top_k, h->n_rot);
        b->K.push_back(K);
        if (b->refine) {
            int rc = ensure_refine_buffers(h, K);
            if (rc) return rc;
        }
        reg_batch::Out o;
        if (!b->alloc(&o.score, h->n_rot) || !b->alloc(&o.pose, 7 * (size_t)h->n_rot) || !b->alloc(&o.top, K) ||
            !b->alloc(&o.init, 7 * (size_t)K) || !b->alloc(&o.refined, 7 * (size_t)K) || !b->alloc(&o.J, K) ||
            !b->alloc(&o.iters, K))
            return fail(REG_ENOMEM, "batch output allocation failed");
        b->out.push_back(o);
        DEV_TRY(h, hipStreamSynchronize(h->stream));
    }
    // longest-processing-time assignment of the handles to the branches by
    // their model bytes (4 half-spectra per rotation)
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    auto cost = [&](int i) { return (double)b->hs[i]->H * b->hs[i]->n_rot; };
    std::sort(order.begin(), order.end(), [&](int x, int y) { return cost(x) > cost(y); });
    std::vector<double> load(nb, 0.0);
    b->branch_of.assign(count, 0);
    for (int i : order) {
        const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        b->branch_of[i] = k;
        load[k] += cost(i);
    }
    reg_handle* h0 = b->hs[0];
    DEV_TRY(h0, hipStreamCreateWithFlags(&b->main, hipStreamNonBlocking));
    b->br.assign(nb, nullptr);
    for (auto& s : b->br) DEV_TRY(h0, hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    b->ev.assign(nb + 1, nullptr);
    for (auto& e : b->ev) DEV_TRY(h0, hipEventCreateWithFlags(&e, hipEventDisableTiming));

    DEV_TRY(h0, hipStreamBeginCapture(b->main, hipStreamCaptureModeRelaxed));
    int rc = REG_OK;
    if (hipEventRecord(b->ev[0], b->main) != hipSuccess) rc = fail(REG_EDEVICE, "fork event");
    for (int k = 0; k < nb && !rc; ++k)
        if (hipStreamWaitEvent(b->br[k], b->ev[0], 0) != hipSuccess) rc = fail(REG_EDEVICE, "fork wait");
    for (int i : order) {
        if (rc) break;
        rc = batch_enqueue(b.get(), i, b->br[b->branch_of[i]]);
    }
    for (int k = 0; k < nb && !rc; ++k)
        if (hipEventRecord(b->ev[1 + k], b->br[k]) != hipSuccess || hipStreamWaitEvent(b->main, b->ev[1 + k], 0) != hipSuccess)
            rc = fail(REG_EDEVICE, "join");
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(b->main, &g);
    b->graph = g;
    if (rc) return rc;
    if (ec != hipSuccess) return fail(REG_EDEVICE, "hipStreamEndCapture failed: %s", hipGetErrorString(ec));
    DEV_TRY(h0, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    *out = b.release();
    return REG_OK;
}

int register_batch_run(reg_batch* b) {
    g_err.clear();
    if (!b) return fail(REG_EINVAL, "NULL batch");
    reg_handle* h0 = b->hs[0];
    DEV_TRY(h0, hipGraphLaunch(b->exec, b->main));
    DEV_TRY(h0, hipStreamSynchronize(b->main));
    if (!b->refine) return REG_OK;
    for (size_t i = 0; i < b->hs.size(); ++i) {
        reg_handle* h = b->hs[i];
        h->r_rounds = b->rounds;
        const reg_batch::Out& o = b->out[i];
        h->r_lbfgsb = b->refine == 2;
        int rc = refine_continue(h, b->K[i], o.refined, o.J, o.iters);
        h->r_lbfgsb = false;
        if (rc) return rc;
    }
    return REG_OK;
}

int register_batch_outputs(reg_batch* b, int32_t i, float* scores, double* poses, int32_t* top, double* refined,
                           double* J) {
    g_err.clear();
    if (!b || i < 0 || i >= (int32_t)b->hs.size()) return fail(REG_EINVAL, "bad batch index");
    const reg_batch::Out& o = b->out[i];
    reg_handle* h = b->hs[i];
    const size_t M = (size_t)h->n_rot, K = (size_t)b->K[i];
    const hipMemcpyKind d2d = hipMemcpyDeviceToDevice;
    if (scores) DEV_TRY(h, hipMemcpyAsync(scores, o.score, M * 4, d2d, b->main));
    if (poses) DEV_TRY(h, hipMemcpyAsync(poses, o.pose, M * 56, d2d, b->main));
    if (top) DEV_TRY(h, hipMemcpyAsync(top, o.top, K * 4, d2d, b->main));
    if (refined) DEV_TRY(h, hipMemcpyAsync(refined, o.refined, K * 56, d2d, b->main));
    if (J) DEV_TRY(h, hipMemcpyAsync(J, o.J, K * 8, d2d, b->main));
    DEV_TRY(h, hipStreamSynchronize(b->main));
    return REG_OK;
}

void register_batch_free(reg_batch* b) {
    if (!b) return;
    if (b->main) (void)hipStreamSynchronize(b->main);
    delete b;
}

int register_autotune(reg_handle* h, int32_t max_rotations, int32_t* out_batch) {
    g_err.clear();
    if (!h || !out_batch) return fail(REG_EINVAL, "NULL argument");
    if (h->poisoned) return fail(REG_EDEVICE, "handle poisoned by an earlier device error");
    if (h->split) return fail(REG_ENOTSUP, "the split plane passes have no workgroup variants to tune");
    int b = 0;
    int rc = autotune_impl(h, max_rotations, &b);
    if (rc) return rc;
    *out_batch = b;
    return REG_OK;
}

int register_tuned_batch(int32_t n) { return regdock_rt::tuned_batch(n); }

int register_tuned_schedule(int32_t n, double* out) {
    g_err.clear();
    if (!out || !canvas_supported(n)) return fail(REG_EINVAL, "NULL output or unsupported edge %d", n);
    Schedule s;
    bool have = false;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(n);
        if (it != g_tuned.end()) {
            s = it->second;
            have = true;
        }
    }
    if (s.pv1 < 0) s.pv1 = default_plane_variant(n);
    if (s.pv3 < 0) s.pv3 = default_plane_variant(n);
    if (s.zv < 0) s.zv = default_z_variant(n);
    if (s.batch <= 0) s.batch = default_batch(n, spectrum_elems(n), 1 << 30);
    const double v[9] = {(double)s.batch, (double)s.lanes, (double)s.pv1, (double)s.pv3, (double)s.zv,
                         s.us1, s.usz, s.us3, s.ns_rot};
    for (int k = 0; k < 9; ++k) out[k] = v[k];
    return have ? 1 : 0;
}

int register_tune_save(const char* path) {
    g_err.clear();
    if (!path) return fail(REG_EINVAL, "NULL path");
    std::map<int, Schedule> snap;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        snap = g_tuned;
    }
    FILE* f = std::fopen(path, "w");
    if (!f) return fail(REG_EINVAL, "cannot write %s", path);
    std::fprintf(f, "[\n");
    size_t k = 0;
    for (const auto& e : snap) {
        const Schedule& s = e.second;
        std::fprintf(f,
                     "  {\"n\": %d, \"batch\": %d, \"lanes\": %d, \"pv1\": %d, \"pv3\": %d, \"zv\": %d, "
                     "\"us1\": %.4f, \"usz\": %.4f, \"us3\": %.4f, \"ns_rot\": %.2f}%s\n",
                     e.first, s.batch, s.lanes, s.pv1, s.pv3, s.zv, std::isfinite(s.us1) ? s.us1 : 0.0,
                     std::isfinite(s.usz) ? s.usz : 0.0, std::isfinite(s.us3) ? s.us3 : 0.0, s.ns_rot,
                     ++k < snap.size() ? "," : "");
    }
    std::fprintf(f, "]\n");
    const bool ok = std::fclose(f) == 0;
    return ok ? REG_OK : fail(REG_EINVAL, "write of %s failed", path);
}

int register_tune_load(const char* path) {
    g_err.clear();
    if (!path) return fail(REG_EINVAL, "NULL path");
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(REG_EINVAL, "cannot read %s", path);
    std::string txt;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, got);
    std::fclose(f);
    // one object per edge: {"n": .., "batch": .., "lanes": .., "pv1": .., "pv3": .., "zv": .., ...}
    auto field = [](const std::string& obj, const char* key, double& v) {
        const std::string k = std::string("\"") + key + "\"";
        const size_t p = obj.find(k);
        if (p == std::string::npos) return false;
        const size_t c = obj.find(':', p + k.size());
        if (c == std::string::npos) return false;
        char* end = nullptr;
        v = std::strtod(obj.c_str() + c + 1, &end);
        return end != obj.c_str() + c + 1;
    };
    std::map<int, Schedule> add;
    size_t pos = 0;
    while ((pos = txt.find('{', pos)) != std::string::npos) {
        const size_t e = txt.find('}', pos);
        if (e == std::string::npos) return fail(REG_EINVAL, "malformed schedule file %s", path);
        const std::string obj = txt.substr(pos, e - pos + 1);
        pos = e + 1;
        double n, b, l, p1, p3, z;
        if (!field(obj, "n", n) || !field(obj, "batch", b) || !field(obj, "lanes", l) || !field(obj, "pv1", p1) ||
            !field(obj, "pv3", p3) || !field(obj, "zv", z))
            return fail(REG_EINVAL, "malformed schedule entry in %s", path);
        const int ni = (int)n;
        if (!canvas_supported(ni) || !plane_variant_ok(ni, (int)p1) || !plane_variant_ok(ni, (int)p3) ||
            !z_variant_ok(ni, (int)z) || b < 8 || (l != 1 && l != 2))
            continue;
        Schedule s;
        s.batch = ((int)b + 7) / 8 * 8;
        s.lanes = (int)l;
        s.pv1 = (int)p1;
        s.pv3 = (int)p3;
        s.zv = (int)z;
        double x;
        if (field(obj, "us1", x)) s.us1 = x;
        if (field(obj, "usz", x)) s.usz = x;
        if (field(obj, "us3", x)) s.us3 = x;
        if (field(obj, "ns_rot", x)) s.ns_rot = x;
        add[ni] = s;
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto& e : add) g_tuned[e.first] = e.second;
    return REG_OK;
}

int register_debug_distance(reg_handle* h, const double* R, const double* p, float* out) {
    g_err.clear();
    if (!h || !R || !p || !out) return fail(REG_EINVAL, "NULL argument");
    if (h->poisoned) return fail(REG_EDEVICE, "handle poisoned by an earlier device error");
    int rc = ensure_refine_buffers(h, 1);
    if (rc) return rc;
    RefineTrial tr{};
    for (int j = 0; j < 9; ++j) tr.R[j] = R[j];
    for (int j = 0; j < 3; ++j) tr.p[j] = p[j];
    tr.valid = 1;
    const RefineConst c = refine_const(h);
    DEV_TRY(h, hipMemcpyAsync(h->rtr, &tr, sizeof tr, hipMemcpyHostToDevice, h->stream));
    DEV_TRY(h, refine_query_only(h->rtr, h->obj->geo, h->poses, h->n_poses, c, h->rw, h->rhits, h->r_active, h->stream));
    DEV_TRY(h, hipMemcpyAsync(out, h->rhits, sizeof(RefineHit) * h->n_poses, hipMemcpyDeviceToDevice, h->stream));
    DEV_TRY(h, hipStreamSynchronize(h->stream));
    return REG_OK;
}

}  // extern "C"

namespace regdock_rt {

int init_shared(const reg_mesh* mesh, const reg_probe* probe, const float* poses, int32_t n_poses, const float* so3,
                int32_t n_rot, const reg_grid_spec* grid, const reg_params* params, void* hip_stream,
                std::shared_ptr<ObjectData> cached, reg_handle** out) {
    return init_impl(mesh, probe, poses, n_poses, so3, n_rot, grid, params, hip_stream, std::move(cached), out);
}

std::shared_ptr<ObjectData> object_of(reg_handle* h) { return h ? h->obj : nullptr; }

int handle_batch(const reg_handle* h) { return h->batch; }

int handle_buffer_sets(const reg_handle* h) { return h->spec2 ? 2 : 1; }

int enqueue_search_batch(reg_handle* h, int b0, int cnt, int set, hipStream_t s) {
    if (set == 1 && !h->spec2) return fail(REG_EINVAL, "the handle has one pass-buffer set");
    return enqueue_batch(h, b0, cnt, set, s, nullptr);
}

int enqueue_search_finish(reg_handle* h, float* out_score, int32_t* out_shift, double* out_pose, hipStream_t s) {
    return enqueue_finish(h, 0, h->n_rot, out_score, out_shift, out_pose, s);
}

size_t object_bytes(const ObjectData* o) { return o ? o->bytes : 0; }

Footprint footprint(int n, int n_rot, int n_poses, int nv, int nf, int batch, int refine_starts, int rotate_object,
                    int split_plane) {
    const size_t n3 = (size_t)n * n * n, H = spectrum_elems(n);
    const size_t m = (size_t)lattice_edge(n), mp = (m + 3) / 4 * 4;
    const size_t B = (size_t)batch, M = (size_t)n_rot, N = (size_t)n_poses;
    Footprint f;
    f.object = 16 * n3 + 8 * H + 16 * (size_t)NLOW3 + 12 * (size_t)nv + 13 * (size_t)nf + 24 * (size_t)n +
               8 * ((n3 + 255) / 256) + 68 * (size_t)nf + 2048;
    const size_t per_rot = 4 * 4 + 4 + 12 + 8 + 4 + 8 + 1 + 8 + 4 + 4 + CMAX * 4 + CMAX * 8 * (size_t)rescore_slices(n);
    // refinement buffers are allocated for at least 16 starts (ensure_refine_buffers)
    const size_t K = refine_starts > 0 ? (size_t)std::max(refine_starts, 16) : 1, nq = K * REF_TMAX * N;
    const size_t lanes = M > B ? 2 : 1;  // the second lane's pass buffers
    f.request = lanes * (H * B * 8 + B * n * KREC * 8 + B * n * 8 + B * n * NLOW2 * 16 + B * NLOW3 * 16) + M * per_rot +
                M * (4 + 56) + 28 * N + 96 * N + m * m * m + mp * mp * mp + 16 * n3 + n * n * ((n + 31) / 32) * 4 +
                K * (sizeof(RefineState) + sizeof(LbfgsState) +
                     REF_TMAX * (sizeof(RefineTrial) + REF_EVAL_PARTS * sizeof(RefineEval))) +
                nq * (sizeof(RefineHit) + 48 + 8 + 4 + 8 + 16 * (8 + 16 + 4)) + 4096;
    if (split_plane || !fused_supported(n)) {  // the plane buffers and row sums of each lane; more peak records
        const size_t units = (size_t)split_units(n);
        f.request += lanes * B * (split_plane_elems(n) * 8 + (size_t)n * n * NLX * 16 + (units - n) * (KREC * 8 + 8));
    }
    if (rotate_object)  // build_rotated_object: classes, records, S and its spectrum, the lattice build's scratch
        f.request += 33 * mp * mp * mp + 4 * n3 + 8 * H + 16 * (size_t)NLOW3 + 8 * n3 + 8 * ((n3 + 255) / 256) +
                     24 * m * m * m + m * m * ((m + 31) / 32) * 4;
    return f;
}

int default_batch_for(int n, int n_rot) { return default_batch(n, spectrum_elems(n), n_rot); }

std::string last_error() { return g_err; }

int tuned_batch(int n) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(n);
    return it == g_tuned.end() ? 0 : it->second.batch;
}

void set_tuned_batch(int n, int batch) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[n].batch = batch;
}

}  // namespace regdock_rt
