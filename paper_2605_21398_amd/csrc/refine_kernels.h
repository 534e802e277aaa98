// Device side of the continuous SE(3) refinement (Sec. V): distance queries of
// the probe poses against the moved object mesh (Sec. V-B), the objective with
// its analytic contact sensitivities (Sec. V-A, V-C) and a damped Gauss-Newton
// (Levenberg-Marquardt) step on the box-bounded twist with an FP64 6x6 solve.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

// Bounding-sphere hierarchy of the body-frame mesh (Sec. V-B keeps a node when
// the probe SDF at its centre is below its radius plus the cutoff): top-level
// nodes hold up to REF_FANOUT clusters, clusters hold up to REF_FANOUT faces
// (faces in Morton order of their centroids).
constexpr int REF_FANOUT = 32;

// The pair queue is cut into REF_SEGS segments of pair_cap / REF_SEGS slots,
// each with its own counter on a cache line of its own, so that the queries'
// appends do not all serialise on one atomic.
constexpr int REF_SEGS = 64;
constexpr int REF_SEG_STRIDE = 16;                              // ints between counters
constexpr int REF_NESTED_AT = REF_SEGS * REF_SEG_STRIDE;        // the nested pairs count
constexpr int REF_COUNTERS = REF_NESTED_AT + REF_SEG_STRIDE;

struct RefineGeometry {
    const float4* top;        // n_top spheres (centre, radius)
    const int2* top_range;    // first cluster, cluster count
    const float4* cluster;    // n_cluster spheres
    const int2* cluster_range;  // first face slot, face count
    const float4* face;       // 4 float4 per face slot: v0 v1 v2 (body), centroid, radius, original index
    const int* slot_of;       // original face index -> slot
    int n_top;
    int n_cluster;
    int n_faces;              // entries of slot_of
};

// Work buffers of the distance query, per (start, probe pose) query q.
struct RefineScratch {
    float* xf;                  // 12 floats per query: body -> probe frame (A row-major, c)
    unsigned long long* qkey;   // best (value, face index) key
    int* qflag;                 // 0: no face kept, 1: key valid, 2: pair list overflowed
    float2* qst;                // barycentric witness of the winning search (-1: a vertex won)
    int2* pairs;                // (query, face slot) pairs for a face search
    float4* pres;               // per pair: minimum, s, t
    int* nest;                  // pairs left to the nested search (indices into pairs)
    int* pair_count;            // REF_COUNTERS ints: the segment counters, then the nested count
    int pair_cap;               // capacity of pairs, pres and nest (a multiple of REF_SEGS)
};

struct RefineConst {
    float r, L;               // probe radius and length (mm)
    float cull;               // cutoff margin of the node/face test (mm)
    float eps;                // d reported when no face is kept
    double r64, L64;          // the same in FP64 (witness polish)
    double tau_out2, tau_in2, k, lambda, b_t, b_r;
    double tol_pg, tol_step, mu0;
    int max_iters;
};

// Per-start solver state, FP64.  status: 0 = evaluation at xi = 0 pending,
// 1 = trial steps pending, 2 = finished.
struct RefineState {
    double R0[9], p0[3], a[3];
    double xi[6];
    double J, g[6], H[36];
    double mu;
    int it, status, pad0, pad1;
};

// Trial slots per start: one round evaluates the trial steps the damped
// Gauss-Newton iteration would try next (damping mu, 3 mu, 9 mu, ...), so a
// rejected step does not cost a round of its own.
constexpr int REF_TMAX = 4;

// L-BFGS-B per start (the paper's solver, Sec. V-C): the last LBFGS_M
// correction pairs, the search direction of the current iteration and the
// step lengths of its line-search trials.
constexpr int LBFGS_M = 10;
struct LbfgsState {
    double S[LBFGS_M][6], Y[LBFGS_M][6];
    double p[6];    // direction x_bar - x (x_bar from the Cauchy point and the subspace step)
    double gp;      // g . p
    double lam0;    // largest step length of the trials in flight (trial j: lam0 / 2^j)
    double fprev;   // J before the last accepted step
    int npairs, head, nback;  // nback: halvings of the current line search
    int ntr;                  // step lengths evaluated in the last round
};
// One trial point of a start, FP64: twist, step, damping, pose and Jacobians.
struct RefineTrial {
    double xe[6], step[6], mu;
    double R[9], p[3], V[9], D[9], c[3];
    int valid, pad;
};

// Objective, gradient and Gauss-Newton curvature at a trial (upper triangle of H).
struct RefineEval {
    double J, g[6], H[21];
};
// the evaluation of a trial is summed by REF_EVAL_PARTS blocks over fixed
// ranges of probe poses; the partial sums (ev holds REF_EVAL_PARTS per trial
// slot) are added in part order by k_ref_decide
constexpr int REF_EVAL_PARTS = 16;

// One distance-query result: {d, x*} and {n, face index bits}.
struct RefineHit {
    float4 dx, nf;
};

// counters[0]: unfinished starts, counters[1]: evaluations so far (device)
hipError_t refine_start(const double* init_poses, int K, const double* anchor, const RefineConst& c,
                        RefineState* st, RefineTrial* tr, int* counters, const RefineScratch& w, hipStream_t s);
// One evaluation round for every unfinished start: distance queries at its
// trial poses, FP64 assembly, the damped Gauss-Newton decision and the next
// trials; updates counters.
hipError_t refine_round(RefineState* st, RefineTrial* tr, int K, const RefineGeometry& geo, const float* poses,
                        int n_poses, const RefineConst& c, const RefineScratch& w, RefineHit* hits, RefineEval* ev,
                        int* counters, hipStream_t s);
// one round of the L-BFGS-B iteration: the queries and evaluations of the
// trials in flight, then the line-search decision and the next direction
hipError_t refine_round_lbfgsb(RefineState* st, LbfgsState* lb, RefineTrial* tr, int K, const RefineGeometry& geo,
                               const float* poses, int n_poses, const RefineConst& c, const RefineScratch& w,
                               RefineHit* hits, RefineEval* ev, int* counters, hipStream_t s);
hipError_t refine_finish(const RefineState* st, int K, double* out_poses, double* out_J, int32_t* out_iters,
                         hipStream_t s);
// Distance queries of all poses at the object pose of trial slot 0 (R, p set, valid).
hipError_t refine_query_only(const RefineTrial* tr, const RefineGeometry& geo, const float* poses, int n_poses,
                             const RefineConst& c, const RefineScratch& w, RefineHit* hits, int* counters,
                             hipStream_t s);
// dst[k] = src[idx[k]] for K rows of 7 doubles (search poses -> starts)
hipError_t gather_poses(const int32_t* idx, const double* src, int K, double* dst, hipStream_t s);
