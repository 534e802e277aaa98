/*
 * regdock -- probe-aware contact registration by complementary-shape docking,
 * global grid-correlation search on AMD MI355X (gfx950).
 *
 * Problem (Sec. III of the paper): a rigid probe of known shape is swept along
 * a trajectory of N poses T_i in SE(3) near an object whose mesh is known; some
 * poses touch the surface, none is known to.  Find the object pose T = (R, t)
 * (body -> world) that best docks the object against the probe's swept volume.
 *
 * The search (Sec. IV): the object grid O = min(O_t, O_m) rewards voxels near
 * the touchable surface, tolerates shallow penetration and penalises deep
 * penetration; the swept occupancy S marks every voxel the probe covered.  For
 * each SO(3) sample the swept grid is rotated by trilinear resampling, the
 * circular correlation C[d] = sum_k O[k] S[k + d] (Eq. xcorr) is evaluated by
 * 3D FFTs, and its maximum gives the best translation for that rotation.
 *
 * Conventions
 *   - Every array argument is a DEVICE pointer (HBM) unless stated otherwise;
 *     the caller owns it and may free it as soon as the call has returned and
 *     the given stream has reached the call.  The library copies what it keeps.
 *   - Quaternions are (w, x, y, z), scalar first.  Poses are rows
 *     (qw, qx, qy, qz, tx, ty, tz) in millimetres.
 *   - Grids are [z][y][x], x fastest; a canvas flat index is (kz*n + ky)*n + kx.
 *   - Calls are enqueued on the handle's HIP stream; results are ready when the
 *     stream reaches them.  A handle must not be used by two threads at once.
 *   - Errors return a negative reg_status; register_last_error() gives a
 *     thread-local message.  After REG_EDEVICE the handle is poisoned: every
 *     later call on it returns REG_EDEVICE.
 */
#ifndef REGDOCK_H
#define REGDOCK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    REG_OK = 0,
    REG_EINVAL = -1,    /* bad argument: null pointer, size, non-finite value, non-unit quaternion */
    REG_ENOMEM = -2,    /* device allocation failed */
    REG_EDEVICE = -3,   /* a HIP call failed; the handle is poisoned */
    REG_EBUSY = -4,     /* admission refused (server) */
    REG_ENOTSUP = -5,   /* canvas edge n without a compiled plan */
    REG_EAGAIN = -6,    /* result not ready (server poll) */
    REG_ECANCELED = -7  /* request cancelled or timed out (server) */
} reg_status;

typedef struct reg_handle reg_handle;

/* Object mesh in its body frame (Sec. IV-A: a watertight mesh for
 * inside/outside and a touchable subset for the surface mask).
 * vertices: n_vertices x 3 float (mm).  faces: n_faces x 3 int32 vertex ids,
 * counter-clockwise seen from outside.  touchable: n_faces uint8 flags, NULL
 * meaning every face is touchable. */
typedef struct {
    const float* vertices;
    int32_t n_vertices;
    const int32_t* faces;
    int32_t n_faces;
    const uint8_t* touchable;
} reg_mesh;

/* Flat-ended cylindrical probe (Sec. VI: cylindrical probe / bur).  In the
 * probe frame the tip disk is centred at the origin and the axis is +z. */
typedef struct {
    double radius_mm;
    double length_mm;
} reg_probe;

/* Common canvas of edge n at spacing h (Sec. IV-A/B).  The object canvas is
 * x_k = a + h (k - n/2) with a the mean of the mesh vertices; the swept
 * lattice is y_j = center_world + h (j - m/2), m = 2 ceil((sqrt(3) n + 2)/2).
 * n must be one of 16, 32, 48, 60, 64, 80, 96, 120, 128, 160, 180 (plane
 * passes in one workgroup per plane) or 192, 256, 360 (split plane passes). */
typedef struct {
    int32_t n;
    double h_mm;
    double center_world[3];
} reg_grid_spec;

/* Zero (or a NULL params pointer) selects the default, Table I of the paper:
 * tau_out1 0.5 mm, tau_in1 0.2 mm, deep-penetration penalty rho 50 (a deep voxel
 * gets -rho), tau_out2 0.2 mm, tau_in2 0.03 mm, k 15, lambda 1e-3; bounds
 * b_t 0.5 mm and b_r 0.2 rad and the query cutoff eps 0.25 mm are not given by
 * the paper.  batch = rotations per batched launch (0: the autotuner's choice
 * for n, else chosen from n).  rescore = 1 re-scores the candidates of every
 * rotation exactly; 0 only those whose float32 error window exceeds the score
 * tolerance (see register_search_stats).  The launch schedule (0: the
 * autotuner's choice for n, else the default): lanes = streams a call's
 * batches alternate over (1 or 2); plane_variant = workgroup of the two plane
 * passes, k selecting variant k - 1 of (threads, waves per SIMD) = (256, 1),
 * (256, 2), (512, 4), (1024, 4) (edges up to 80 take the first three, edges
 * up to 128 the last three, larger edges the last); z_variant = threads of the z-pencil workgroup, k
 * selecting 128, 256 or 512.
 * rotate_object = 1 selects the paper's own search variant (Sec. IV-D as
 * printed): for each sample the object grid O is rotated about the anchor a
 * and resampled trilinearly onto the canvas z_k = center_world + h (k - n/2),
 * from O on the body lattice a + h (j - m/2), and correlated with the swept
 * occupancy S on that canvas, which stays fixed.  0 (the default) rotates S
 * instead, against the fixed object canvas.  The variant keeps an m^3
 * lattice of cell classes and 32-byte corner records per cell (360 MB at
 * n = 128, 1 GB at 180); pass 1 then runs with the default workgroup.
 * split_plane = 1 runs the search's plane passes as split row and column
 * passes through an HBM plane buffer (n^2 n/2 complex per rotation of a
 * batch) instead of one workgroup per plane; edges above 180, whose plane does
 * not fit the LDS, always do.  Compiled for 64, 128, 192, 256 and 360
 * (REG_ENOTSUP otherwise, and with rotate_object). */
typedef struct {
    double tau_out1, tau_in1, rho;
    double tau_out2, tau_in2, k, lambda;
    double b_t, b_r, eps;
    int32_t max_iters;
    int32_t batch;
    int32_t rescore;
    int32_t lanes;
    int32_t plane_variant;
    int32_t z_variant;
    int32_t rotate_object;
    int32_t split_plane;
} reg_params;

/* Build a registration problem (Sec. IV-A): the object grid O and its spectrum
 * conj(F(O))/n^3 (kept resident), the swept occupancy S_w of the trajectory on
 * the world lattice, and the rotation matrices of the n_rot SO(3) samples.
 *   poses: n_poses x 7 float, probe-local -> world.  so3: n_rot x 4 float unit
 *   quaternions, object body -> world.  hip_stream: the hipStream_t every call
 *   on the handle is enqueued on (NULL: the null stream); the caller keeps it
 *   alive for the handle's lifetime.  On success *out receives a new handle.
 * Blocks until the input checks (finite values, face ids in range, quaternion
 * norms within 1 +- 1e-3) have run on the device.
 * Errors: REG_EINVAL, REG_ENOTSUP, REG_ENOMEM, REG_EDEVICE. */
int register_init(const reg_mesh* mesh, const reg_probe* probe, const float* poses, int32_t n_poses,
                  const float* so3, int32_t n_rot, const reg_grid_spec* grid, const reg_params* params,
                  void* hip_stream, reg_handle** out);

/* Canvas edge for the padded, linear correlation of Sec. IV-B: the search's
 * correlation is circular on the n^3 canvas, and it equals the linear
 * (zero-padded) correlation once n >= n_o + n_s - 1, where n_o and n_s are the
 * grid extents of the object and of the rotated swept occupancy.  Both are
 * bounded by spheres about the canvas centre: the vertex radius about the
 * vertex mean plus tau_out1 (the object grid vanishes farther from the mesh;
 * <= 0 selects 0.5 mm), and the farthest probe point of the trajectory from
 * center_world (grid spec) plus sqrt(3) h (the reach of the trilinear
 * resampling); a radius R covers 2 floor(R/h) + 1 grid points.
 *   vertices: n_vertices x 3 float, poses: n_poses x 7 float, both HOST
 *   memory (this is a planning call, before register_init).
 *   *needed = n_o + n_s - 1; *edge = the smallest supported edge >= *needed.
 * Passing *edge as grid.n (same h and centre) gives a wrap-free search.
 * Errors: REG_EINVAL (NULL or non-finite input, h or probe size <= 0),
 * REG_ENOTSUP (*needed above 360; *needed is still set, *edge = 0). */
int register_linear_edge(const float* vertices, int32_t n_vertices, const reg_probe* probe, const float* poses,
                         int32_t n_poses, const double* center_world, double h_mm, double tau_out1, int32_t* needed,
                         int32_t* edge);

/* Score SO(3) samples [first, first + count) (Sec. IV-B and IV-D).  For each
 * rotation R: S_r[k] = trilinear S_w at R (x_k - a) + center_world; C = circular
 * correlation of O with S_r; score = max C; d* = the lowest flat index among
 * the maxima; shift = d* with components >= n/2 reduced by n.  The maximum is
 * found by float32 FFTs and confirmed by exact re-scoring of every shift the
 * float32 error could hide it behind (see register_search_stats).
 *   out_score: count float.  out_shift: count x 3 int32 (x, y, z) or NULL.
 *   out_pose: count x 7 double (unit quaternion, t) or NULL, with
 *   t = center_world - R a + h R shift, so that x -> R x + t maps the object
 *   body frame to world.  Asynchronous on the handle's stream.
 * With params.rotate_object: O_q[k] = trilinear O at a + R^T (z_k - center_world);
 * the field is C'[e] = sum_k S[k] O_q[k + e] (circular), whose lowest-index
 * maximum e* gives the shift of Eq. (xcorr), shift = -e* (components of e*
 * >= n/2 reduced by n first), and t = center_world - R a + h shift.
 * Errors: REG_EINVAL (range or null out_score), REG_EDEVICE. */
int score_rotations(reg_handle* h, int32_t first, int32_t count, float* out_score, int32_t* out_shift,
                    double* out_pose);

/* How the peaks were found.  The field is float32 FFTs plus an exact double
 * low-frequency block; eps = 6 * 2^-24 * rms(C_high) * log2(n^3) bounds its
 * error.  Per rotation, every shift within 2 eps of the field maximum is a
 * candidate (4 kept per plane, 16 per rotation).  After all rotations of a
 * call, tol = 1e-4 * max |score|: a rotation with 2 eps <= tol keeps the field
 * maximum (value within eps, index within tol of the best); the others (all,
 * with params.rescore) have their candidates re-scored exactly -- a direct sum
 * over the nonzero voxels of O in double -- and the best exact score wins.
 * Counters since register_init: scored rotations, candidates, rotations whose
 * window held more candidates than were kept (exact-tie plateaus), "uncertain"
 * rotations (re-scored, overflowed, and 2 eps > tol), and re-scored rotations.
 * Host pointers; synchronises the stream. */
int register_search_stats(reg_handle* h, int64_t* rotations, int64_t* candidates, int64_t* overflows,
                          int64_t* uncertain, int64_t* rescored);

/* The K best rotations of a score vector (score descending, index ascending),
 * computed on the device.  scores: count float; out_idx: K int32.
 * Errors: REG_EINVAL, REG_EDEVICE. */
int register_top_k(reg_handle* h, const float* scores, int32_t count, int32_t K, int32_t* out_idx);

/* Release a handle and every device buffer it owns (NULL is a no-op).  Waits
 * for the handle's stream; the buffers go to the library's device memory
 * cache, where the next handles, batches and server requests of the same sizes
 * take them without hipMalloc (the cache holds at most 32 GiB per process, and
 * an allocation that fails first returns the device's cached blocks to HIP). */
void register_free(reg_handle* h);

/* ------------------------------------------------ orientation samplers
 * (Sec. IV-C).  Unit quaternions, scalar first, written as n x 4 float32 to
 * the device buffer `out` on hip_stream (NULL: the null stream); the call
 * returns when they are written.  Errors: REG_EINVAL, REG_EDEVICE. */

/* Super-Fibonacci sequence (the global sampler the paper adopts): for
 * s = i + 1/2, r = sqrt(s/n), R = sqrt(1 - s/n), a = 2 pi s / sqrt 2,
 * b = 2 pi s / psi (psi^4 = psi + 4): q = (r sin a, r cos a, R sin b, R cos b). */
int so3_super_fibonacci(int32_t n, float* out, void* hip_stream);

/* GeoBall-SF (Alg. geoball-sf): n low-discrepancy samples uniform in the
 * geodesic ball {q : arccos |<q, q0>| <= theta} (rotations within 2 theta of
 * q0).  q0: 4 host doubles (normalised here); theta in (0, pi/2]; gamma: the
 * divisor of the radial coordinate u1 = (i + 1/2) / gamma mod 1, 0 meaning
 * gamma = n (the paper leaves it undefined).  The radial law r L(r),
 * L(r) = 2 arccos(cos theta / sqrt(1 - r^2)), is tabulated at 4096 points and
 * inverted by linear interpolation. */
int so3_geoball_sf(int32_t n, const double* q0, double theta, double gamma, float* out, void* hip_stream);

/* Largest n of the samplers: (n + 255) / 256 blocks of 256 threads must be
 * indexable in int32. */
#define SO3_SAMPLER_MAX_N 2147483392

/* so3_geoball_sf for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same samples, with no allocation, no host copy and no synchronisation.
 * Its only scratch is the radial table (radii and distribution function,
 * 2 x 4096 doubles = 64 KiB), built on the device by a kernel into a static
 * device array that each GPU holds for the life of the process; its size does
 * not depend on n.  Arguments as so3_geoball_sf; out: n x 4 float32 on the
 * device, written asynchronously on hip_stream (NULL: the null stream).  The
 * table keeps the last call's contents and is rebuilt by every call: calls
 * that overlap on one GPU (different streams, or threads) race on it and must
 * be serialised by the caller.  The samples agree with so3_geoball_sf's to
 * float32 rounding (both tabulate the same function in the same order).
 * Errors: REG_EINVAL (as so3_geoball_sf, or n > SO3_SAMPLER_MAX_N),
 * REG_EDEVICE. */
int so3_geoball_sf_noalloc(int32_t n, const double* q0, double theta, double gamma, float* out, void* hip_stream);

/* Replace the handle's SO(3) sample set (M x 4 float32 on the device, copied)
 * so that score_rotations scores it against the same object grid and swept
 * lattice, e.g. the local GeoBall-SF set around the global maximum (Sec.
 * IV-D).  Synchronises the handle's stream.  Errors: REG_EINVAL (NULL, M < 1,
 * a quaternion norm outside 1 +- 1e-3: the handle then has no rotations until
 * a valid set is given), REG_EBUSY (the handle is in a live batch, whose graph
 * captured its rotation set), REG_ENOMEM, REG_EDEVICE. */
int register_set_rotations(reg_handle* h, const float* so3, int32_t n_rot);

/* Memory management (not an operation of the method): bytes held by the
 * device memory cache, and the release of every cached block back to HIP. */
int64_t register_cached_bytes(void);
void register_release_cached(void);

/* Thread-local description of the last error on this thread ("" if none). */
const char* register_last_error(void);

/* Canvas edge, swept-lattice edge, spectrum elements per rotation, rotations
 * per batched launch and number of rotations of a handle (any pointer may be
 * NULL).  Host pointers. */
int register_info(const reg_handle* h, int32_t* n, int32_t* m, int64_t* spectrum_elems, int32_t* batch, int32_t* n_rot);

/* ---- measurement: per-kernel durations from HIP events ---- */

/* enable != 0 records a HIP event pair around every launch of the three
 * per-rotation kernels (0: rotate + voxelise + forward FFT in x and y;
 * 1: z FFT, spectral product, inverse z FFT; 2: inverse FFT in y and x +
 * argmax) on the handle's stream; any call resets the record.  Host call,
 * synchronises the stream. */
int register_set_timing(reg_handle* h, int32_t enable);

/* Sums over the recorded launches since register_set_timing: ms[k] total
 * milliseconds, launches[k] launch count, rotations[k] rotations processed, for
 * k = 0, 1, 2 (host arrays of 3).  Synchronises the stream. */
int register_get_timing(reg_handle* h, double* ms, int64_t* launches, int64_t* rotations);

/* ---- test hooks: inspect or replace the per-problem grids ---- */

/* Copy the object grid O (n^3 float) and its signed distance f_o (n^3 float,
 * may be NULL) to device buffers. */
int register_debug_object_grid(reg_handle* h, float* out_O, float* out_fo);

/* Copy the swept occupancy S_w (m^3 uint8, 0/1) to a device buffer. */
int register_debug_swept(reg_handle* h, uint8_t* out_Sw);

/* The swept lattice's reach as the search holds it: the largest
 * (2x - m)^2 + (2y - m)^2 + (2z - m)^2 over the occupied points of S_w (0 for
 * an empty lattice).  Rows and planes of S_r farther than sqrt(reach4) / 2 +
 * sqrt(3) voxels from the canvas centre are zero; the split plane passes write
 * such row blocks and planes unsampled, the fused pass 1 such planes.  Host
 * pointer; synchronises the stream.  REG_ENOTSUP for the rotated-object
 * search, which does not compute it. */
int register_debug_swept_reach(reg_handle* h, int64_t* out_reach4);

/* Full correlation C (n^3 float) of SO(3) sample `rot` into a device buffer
 * (C' of the rotated-object search, indexed by e). */
int register_debug_correlation(reg_handle* h, int32_t rot, float* out_C);

/* Replace O (n^3 float, device) and/or S_w (m^3 uint8 0/1, device) of a
 * handle by given grids (NULL keeps the current one); the spectrum and the
 * corner masks are rebuilt.  Isolates the per-rotation path from threshold
 * decisions taken while building the grids.  REG_ENOTSUP on a handle of the
 * rotated-object search (params.rotate_object). */
int register_set_grids(reg_handle* h, const float* O, const uint8_t* Sw);

/* Continuous SE(3) refinement of K initial object poses (Sec. V).  Each start
 * (R0, p0) is refined over the twist xi = (v, w) with |v|_inf <= b_t and
 * |w|_inf <= b_r, the left perturbation about the anchor a (Eq. se3-exp and
 * the left pose updates): R = exp(w^) R0, p = p0 + V(w) v + (I - exp(w^)) R0 a.
 * It minimises J = -sum_i s(d_i) + lambda |xi|^2 (Eq. objective), s the
 * proximity score of Sec. V-A and d_i the smallest signed probe-mesh distance
 * at probe pose i (Sec. V-B: faces kept by the bounding-sphere test with the
 * cutoff eps, d_i = eps when none is), with the analytic contact sensitivities
 * of Sec. V-C.  Solver: damped Gauss-Newton from xi = 0 with curvature
 * sum_i max(0, -s''(d_i)) g_i g_i^T + 2 lambda I and an FP64 6x6 Cholesky solve
 * of (H + mu diag H + 1e-12 I) step = -grad J; a step is kept when J
 * decreases (mu /= 3), else mu *= 3.  Stops when the projected gradient is
 * <= 1e-6, a step is <= 1e-9, mu reaches 1e12 or after params.max_iters steps.
 * Distances are float32, the objective, its derivatives and the solve FP64.
 *   init_poses: K x 7 double (qw qx qy qz tx ty tz, object body -> world, the
 *   pose format of score_rotations), device memory; the quaternion norm must be
 *   within 1 +- 1e-3.  out_poses: K x 7 double (w >= 0), out_J: K double or
 *   NULL, out_iters: K int32 accepted-step counts or NULL; device memory.
 * Synchronous: returns when the results are written.
 * Errors: REG_EINVAL (K < 1, NULL poses, non-finite or non-unit start),
 * REG_ENOMEM, REG_EDEVICE. */
int refine_se3(reg_handle* h, const double* init_poses, int32_t K, double* out_poses, double* out_J,
               int32_t* out_iters);

/* The same refinement with the paper's solver, L-BFGS-B (Sec. V-C), on the
 * same objective, gradient and box: generalised Cauchy point and subspace step
 * on the limited-memory matrix of the last 10 correction pairs, backtracking
 * line search with sufficient decrease.  Stops on a projected gradient below
 * 1e-6, a relative decrease of J below 1e-10, max_iters steps, or no decrease
 * found even along the projected steepest descent.  out_iters: accepted steps.
 * Arguments, ownership and errors as refine_se3. */
int refine_se3_lbfgsb(reg_handle* h, const double* init_poses, int32_t K, double* out_poses, double* out_J,
                      int32_t* out_iters);

/* Work of the last refine_se3 call on the handle: evaluation rounds launched
 * (all unfinished starts are evaluated together in a round) and evaluations
 * made (one per unfinished start per round: a trial step, or the start
 * itself).  Host pointers. */
int register_refine_stats(reg_handle* h, int64_t* rounds, int64_t* evaluations);

/* Test hook: the refinement's distance query (Sec. V-B) of every probe pose
 * against the object mesh placed by x -> R x + p.  R: 9 double row-major, p: 3
 * double, host memory.  out: n_poses x 8 float, device memory: d, the witness
 * x* (world), the unit normal n of the probe SDF there (world) and the index of
 * the face that holds x* (int32 bits; -1 with d = eps when no face was kept).
 * Faces farther than min(eps, tau_out2) may be skipped, since they cannot
 * change s, s' or s''.  Synchronous. */
int register_debug_distance(reg_handle* h, const double* R, const double* p, float* out);

/* ----------------------------------------------------------------- batching
 *
 * Many registrations of uneven canvases as one captured hipGraph: for each
 * handle, the global search over all its rotations (Sec. IV), its top_k peaks
 * and graph_rounds rounds of their SE(3) refinement (Sec. V), on a few
 * parallel branches balanced by model HBM bytes.  A replay recomputes
 * everything from the handles' inputs; refinements still running after the
 * captured rounds are continued by register_batch_run, so the results equal
 * those of score_rotations / register_top_k / refine_se3 (or refine_se3_lbfgsb)
 * on each handle.
 * The handles must stay alive and must not be used elsewhere while the batch
 * runs; their event timing must be off.
 */
typedef struct reg_batch reg_batch;

/* handles: count handle pointers (host array).  top_k in [1, 16]; refine 0
 * (none), 1 (Gauss-Newton, as refine_se3) or 2 (L-BFGS-B, as refine_se3_lbfgsb);
 * graph_rounds: refinement rounds captured (0: 64); branches: parallel
 * streams (0: 4).  Errors: REG_EINVAL, REG_ENOMEM, REG_EDEVICE. */
int register_batch_create(reg_handle* const* handles, int32_t count, int32_t top_k, int32_t refine,
                          int32_t graph_rounds, int32_t branches, reg_batch** out);
/* Replays the graph and waits for it (and any continued refinement). */
int register_batch_run(reg_batch* b);
/* Copies handle i's outputs of the last run into the given device buffers:
 * scores (n_rot float), search poses (n_rot x 7 double), top (K int32), refined
 * poses (K x 7 double) and J (K double), K = min(top_k, n_rot).  Any pointer
 * may be NULL.  Synchronous. */
int register_batch_outputs(reg_batch* b, int32_t i, float* scores, double* poses, int32_t* top, double* refined,
                           double* J);
void register_batch_free(reg_batch* b);

/* Autotuner of the search schedule for the handle's canvas edge, timed on
 * the handle's own problem (its first max_rotations rotations, 0: 512) with
 * HIP events: every valid plane-workgroup variant for pass 1 and for pass 3
 * and every z-workgroup variant (each pass timed alone), then rotation
 * batches of 8..512 (up to the rotations timed, within 4 GB of work buffers)
 * on one and on two lanes with the chosen kernels, the whole search timed.
 * The fastest schedule is recorded for the edge; later register_init calls
 * whose params leave a field at 0 take it.  *out_batch receives the batch.
 * Synchronous.  Errors: REG_EINVAL, REG_ENOMEM, REG_EDEVICE. */
int register_autotune(reg_handle* h, int32_t max_rotations, int32_t* out_batch);
/* the recorded batch for canvas edge n, 0 if none */
int register_tuned_batch(int32_t n);
/* The recorded schedule for edge n: out[0] batch, out[1] lanes, out[2] pass-1
 * plane variant, out[3] pass-3 plane variant, out[4] z variant (variants
 * numbered from 0 as in reg_params, less one); out[5..7] the best times (us
 * per rotation) of pass 1, the z pass and pass 3; out[8] the whole search (ns
 * per rotation).  Returns 1 if a schedule is recorded, 0 if not (out is then
 * filled with the defaults), or REG_EINVAL. */
int register_tuned_schedule(int32_t n, double* out);
/* Save every recorded schedule to a JSON file (one object per edge), or load
 * such a file (entries for unsupported edges or invalid variants are
 * skipped).  Errors: REG_EINVAL (NULL path, unreadable or malformed file). */
int register_tune_save(const char* path);
int register_tune_load(const char* path);

/* ------------------------------------------------------------------ serving
 *
 * A server runs whole registrations -- object grid and spectrum, swept
 * occupancy, the global search over every SO(3) sample (Sec. IV), the top-K
 * peaks and their SE(3) refinement (Sec. V) -- for requests submitted from
 * any thread.  Requests are admitted in arrival order when a worker slot is
 * free and their device footprint fits beside the registrations in flight;
 * each slot has its own HIP stream, so admitted registrations overlap on the
 * device and a request arriving while others run starts as soon as a slot and
 * memory free up.  Objects (mesh + canvas + object-grid thresholds) stay
 * resident in a cache keyed by the mesh's contents (a hash of the vertex,
 * face and touchable arrays, confirmed byte for byte on a hit), the canvas and
 * the thresholds: a later request for the same object skips the object grid
 * and its spectrum.  A registration's results do not depend on what else runs
 * beside it.
 */
typedef struct reg_server reg_server;
typedef uint64_t reg_ticket;

typedef struct {
    int64_t hbm_budget_bytes;   /* device bytes for registrations in flight; 0: 3/4 of free memory minus the cache */
    int32_t max_inflight;       /* worker slots (concurrent registrations); 0: 4 */
    int32_t mode;               /* 0: continuous, 1: serial (one registration at a time) */
    int64_t cache_bytes;        /* object cache budget (least recently used objects evicted); 0: 4 GiB */
    int32_t fake;               /* test hook: 1 = no device work, a registration takes fake_us_per_rotation per rotation */
    double fake_us_per_rotation;
} reg_server_cfg;

/* All arrays in HOST memory; they are copied before register_submit returns. */
typedef struct {
    reg_mesh mesh;
    int64_t object_id;          /* >= 0: the object may be cached and taken from the cache; -1: built afresh, not cached */
    reg_probe probe;
    const float* poses;         /* n_poses x 7 */
    int32_t n_poses;
    const float* so3;           /* n_rot x 4 */
    int32_t n_rot;
    reg_grid_spec grid;
    reg_params params;          /* zero fields take the defaults */
    int32_t top_k;              /* peaks kept, 1..16 (0: 16) */
    int32_t refine;             /* 0: no refinement; 1: the top_k peaks by Gauss-Newton (refine_se3);
                                   2: by L-BFGS-B (refine_se3_lbfgsb); other values: REG_EINVAL */
} reg_request;

typedef struct {
    int32_t status;             /* REG_OK or the error of the registration */
    int32_t n_top;
    float best_score;           /* the largest search score */
    double best_pose[7];        /* refined pose of lowest J (refine = 1), else the best search pose */
    double best_J;
    int32_t top_rot[16];        /* rotation indices of the peaks, score descending */
    float top_score[16];
    double top_pose[16 * 7];    /* search poses of the peaks */
    double refined_pose[16 * 7];
    double refined_J[16];
    int64_t t_submit_ns, t_admit_ns, t_start_ns, t_end_ns;  /* steady clock */
    int64_t footprint_bytes;    /* device bytes reserved for the registration */
    char error[128];
} reg_result;

typedef struct {
    int64_t queued, running, done;
    int64_t in_use_bytes, budget_bytes;
    int64_t cache_hits, cache_misses, cache_bytes, cached_objects;
} reg_server_stats;

/* Errors: REG_EINVAL, REG_EDEVICE (stream creation), REG_ENOMEM. */
int register_server_create(const reg_server_cfg* cfg, reg_server** out);
/* Cancels queued requests (REG_ECANCELED), waits for running ones, frees all. */
void register_server_destroy(reg_server* s);
/* Queues a registration.  Errors: REG_EINVAL, REG_EBUSY (needs more than the
 * whole budget), REG_ECANCELED (server stopping). */
int register_submit(reg_server* s, const reg_request* request, reg_ticket* out);
/* The result if the registration has finished (the ticket is then released),
 * else REG_EAGAIN.  Returns the registration's own status when it failed. */
int register_poll(reg_server* s, reg_ticket t, reg_result* out);
/* As register_poll, waiting up to timeout_ms (< 0: without limit). */
int register_wait(reg_server* s, reg_ticket t, int64_t timeout_ms, reg_result* out);
int register_server_stats(reg_server* s, reg_server_stats* out);
/* message of the calling thread's last failing server call */
const char* register_server_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* REGDOCK_H */
