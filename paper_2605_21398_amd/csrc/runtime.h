// Internal interface between the handle layer (api.cpp) and the serving and
// batching runtime: registrations that share one device-resident object
// (mesh, object grid, spectrum), and the device footprint used for admission.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <memory>
#include <string>

#include "regdock.h"

struct ObjectData;

namespace regdock_rt {

// register_init, reusing `cached` (built for the same mesh, canvas and
// object-grid thresholds) when it is not null.
int init_shared(const reg_mesh* mesh, const reg_probe* probe, const float* poses, int32_t n_poses, const float* so3,
                int32_t n_rot, const reg_grid_spec* grid, const reg_params* params, void* hip_stream,
                std::shared_ptr<ObjectData> cached, reg_handle** out);

std::shared_ptr<ObjectData> object_of(reg_handle* h);

// The search of a handle as separate work items, for a scheduler that
// interleaves items of several handles on its own streams: the rotation batch
// [b0, b0 + cnt) through the three passes and the candidate selection with
// pass-buffer set `set` (0, or 1 when handle_buffer_sets is 2) on stream s;
// then, once every batch is done, the certification, re-scoring and outputs
// of all rotations (as score_rotations over the whole set).  The caller
// orders items that share a buffer set and the finish after every batch.
int handle_batch(const reg_handle* h);
int handle_buffer_sets(const reg_handle* h);
int enqueue_search_batch(reg_handle* h, int b0, int cnt, int set, hipStream_t s);
int enqueue_search_finish(reg_handle* h, float* out_score, int32_t* out_shift, double* out_pose, hipStream_t s);
size_t object_bytes(const ObjectData* o);

// Device bytes of one registration: the object part (grid, spectrum, lists,
// mesh and its hierarchy) and the request part (swept lattice, spectrum work
// buffer of one batch, per-rotation arrays, refinement buffers, and with
// rotate_object the rotated-object search's lattice records and spectra).
struct Footprint {
    size_t object = 0, request = 0;
};
Footprint footprint(int n, int n_rot, int n_poses, int n_vertices, int n_faces, int batch, int refine_starts,
                    int rotate_object = 0, int split_plane = 0);
int default_batch_for(int n, int n_rot);

// the calling thread's last error message
std::string last_error();

// Device memory cache: blocks released by handles, objects, batches and
// server requests are kept per device and rounded size for the next ones
// (hipMalloc and hipFree cost milliseconds, and hipFree waits for the whole
// device).  A block may be released only once no queued work uses it (the
// releasing side synchronises its stream first).  A failed allocation returns
// every cached block of the device to HIP and tries once more.
hipError_t dev_alloc(void** p, size_t bytes);
void dev_release(void* p);
size_t dev_cached_bytes();
void dev_trim();

// Rotation batch per canvas edge chosen by the autotuner (0: none recorded).
int tuned_batch(int n);
void set_tuned_batch(int n, int batch);

}  // namespace regdock_rt
