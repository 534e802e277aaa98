// Host-side launchers of the global-search kernels (internal to libregdock).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace regdock {

// per-plane candidates kept by pass 3 (plus one bound per plane), candidates
// re-scored per rotation
constexpr int KTOP = 4;
constexpr int KREC = KTOP + 1;
constexpr int CMAX = 16;
// Exact low-frequency block: frequencies with max(|kx|, |ky|, |kz|) <= KLOW are
// taken out of the float32 FFT path and carried in double (they hold nearly all
// of the correlation's energy, which the -50 penalty makes huge).
constexpr int KLOW = 3;
constexpr int NLX = KLOW + 1;        // kx in [0, KLOW]
constexpr int NLY = 2 * KLOW + 1;    // ky, kz in [-KLOW, KLOW]
constexpr int NLOW2 = NLX * NLY;     // (kx, ky) pairs of a plane
constexpr int NLOW3 = NLOW2 * NLY;   // (kx, ky, kz) of a rotation
// Window half-width eps = REGK_EPS_SCALE * 2^-24 * rms(C_high) * log2(n^3)
// bounds the float32 error of the remaining (high-frequency) field.
constexpr double REGK_EPS_SCALE = 6.0;

enum : int {
    REGK_ERR_NONFINITE = 1,
    REGK_ERR_QUAT = 2,
    REGK_ERR_FACE = 4,
};

struct SearchBatchArgs {
    const uint8_t* cmask;      // bricked corner masks, mp^3 bytes
    int m, mp;                 // lattice edge and its multiple-of-4 padding
    const double* rots;        // [count][9] rotation matrices of this batch (double)
    int count;                 // rotations in this batch
    const float2* tw;          // twiddles w[t] = exp(-2 pi i t / n), n entries
    float2* spec;              // [count][H] spectrum work buffer
    const float2* W;           // conj(F(O)) / n^3 in the tiled layout, H entries
    const double2* tw64;       // exp(-2 pi i t / n) in double, n entries
    double2* lowT;             // [count][n][NLOW2] per-plane low 2D DFT of S_r (double)
    const double2* Wlow;       // [NLOW3] conj(F(O)) / n^3 on the low block (double)
    double2* Plow;             // [count][NLOW3] exact product on the low block
    unsigned long long* ptop;  // [count][n][KREC] per plane: best keys (score bits, ~flat), then the bound (double bits)
    double* pssq;              // [count][n] per-plane sums of squares of the field
    float* corr_out;           // optional: full float32 field of a 1-rotation batch
    int pv1, pv3, zv;          // schedule variants of pass 1, pass 3 and the z pass
    hipStream_t stream;
    // rotated-object search: the rotated grid is a real lattice whose cell
    // classes sit in cmask and whose mixed cells' corner values sit in crec
    // (two float4 per cell, bricked as cmask), class 1 standing for cval;
    // rots then hold R^T.  NULL: corner masks of the binary swept lattice.
    const float4* crec = nullptr;
    float cval = 0.0f;
    // peak records per rotation in ptop / pssq (0: n, one per plane)
    int units = 0;
    // split plane passes: the plane buffer [count][n][n][n/2] and the rows'
    // x sums of the low block [count][n][n][NLX]; NULL selects the fused passes
    float2* xbuf = nullptr;
    double2* lowrow = nullptr;
    // the swept lattice's reach (swept_reach): the split passes write row
    // blocks and planes of S_r beyond it as zeros unsampled, the fused pass 1
    // such planes.  NULL: no skip
    const unsigned long long* reach4 = nullptr;
};

// Schedule variants (threads and waves per SIMD of the plane workgroups;
// threads of the z-pencil workgroups), valid per canvas edge.
constexpr int PLANE_VARIANTS = 4;
constexpr int Z_VARIANTS = 3;
bool plane_variant_ok(int n, int v);
bool z_variant_ok(int n, int v);
int default_plane_variant(int n);
int default_z_variant(int n);
int plane_variant_threads(int v);
int z_variant_threads(int v);

bool canvas_supported(int n);
bool fused_supported(int n);   // the plane fits one workgroup's LDS (edges up to 180)
bool split_supported(int n);   // split plane passes compiled (64, 128, 192, 256, 360)
int split_units(int n);        // peak records per rotation of the split passes
size_t split_plane_elems(int n);  // complex per rotation of the split passes' plane buffer
int rescore_slices(int n);
size_t spectrum_elems(int n);
int tile_width(int n);

// pass 0: rotate+voxelise+FFT xy; 1: z FFT * W * z IFFT; 2: IFFT yx + argmax
hipError_t search_pass(int n, int pass, const SearchBatchArgs& a);
hipError_t object_spectrum(int n, const float* O, float2* spec_tmp, float2* W, const float2* tw, const double2* tw64,
                           double2* lowT_tmp, double2* Wlow, hipStream_t s, float2* xbuf = nullptr,
                           double2* lowrow = nullptr);
hipError_t setup_anchor(const float* V, int nv, double* anchor, hipStream_t s);
// scratch of the object-grid build: squared distances (double bits, n^3 each)
// and the inside-parity bit words of every column (n^2 * ceil(n/32))
struct ObjectScratch {
    unsigned long long* d2;
    unsigned long long* dt2;
    uint32_t* par;
};
hipError_t setup_object_grid(const float* V, const int32_t* F, const uint8_t* touch, int nf, int n, double h,
                             const double* anchor, double tau_out1, double tau_in1, double rho, float* O, float* fo,
                             const ObjectScratch& w, hipStream_t s);
hipError_t setup_swept(const float* poses, int np, double r, double L, int m, int mp, double h, const double* wc,
                       double* pose_tmp, uint8_t* Sw, uint8_t* cm, hipStream_t s);
hipError_t setup_cellmask(const uint8_t* Sw, int m, int mp, uint8_t* cm, hipStream_t s);
// the swept lattice's reach: max over occupied points of (2x-m)^2 + (2y-m)^2 +
// (2z-m)^2 into *reach4 (one device word, cleared first)
hipError_t swept_reach(const uint8_t* Sw, int m, unsigned long long* reach4, hipStream_t s);
hipError_t setup_rotations(const float* so3, int M, double* rots, int* err, hipStream_t s, int transpose = 0);
// rotated-object search: cell classes (mp^3 bytes, bricked) and corner records
// (2 mp^3 float4) of the object grid on the body lattice; the fixed grid S
// (n^3 float) from the swept lattice
hipError_t setup_object_cells(const float* G, int m, int mp, float cval, uint8_t* cls, float4* rec, hipStream_t s);
hipError_t swept_canvas(const uint8_t* Sw, int m, int n, float* S, hipStream_t s);
hipError_t validate_inputs(const float* V, int nv, const int32_t* F, int nf, const float* poses, int np, int* err,
                           hipStream_t s);
// per-rotation peak bookkeeping, indexed by absolute rotation
struct PeakArrays {
    int32_t* cand_idx;   // [n_rot][CMAX] candidate flat indices
    int32_t* cand_n;     // [n_rot]
    double* window;      // [n_rot] 2 eps
    uint8_t* ovf;        // [n_rot] window overflowed
    double* best_val;    // [n_rot] field maximum (double)
    int32_t* best_flat;  // [n_rot] its flat index
    int32_t* need_list;  // [n_rot] rotations (relative to the call) to re-score
    int* need_count;     // [1]
    double* cand_part;   // [n_rot][CMAX][rescore_slices(n)] slice sums
    int* stats;          // [5] rotations, candidates, overflowed, uncertain, re-scored
};
// what the exact re-score reads
struct RescoreInputs {
    const uint32_t* nz_idx;  // nonzero voxels of the fixed grid (O; S when O rotates): kx | ky << 10 | kz << 20
    const float* nz_val;
    const int* nz_count;
    const uint8_t* cmask;
    int m, mp;
    const double* rots;      // all rotations
    const float4* crec;      // rotated-object search (as in SearchBatchArgs), else NULL
    float cval;
};
hipError_t select_batch(int n, const SearchBatchArgs& a, int base, const PeakArrays& pk);
hipError_t finish_call(int n, int first, int count, int always, const PeakArrays& pk, const RescoreInputs& ri,
                       const float* quats, double h, const double* anchor, const double* wc, float* out_score,
                       int32_t* out_shift, double* out_pose, hipStream_t s);
hipError_t build_nonzero_list(const float* O, int n, int* bcount, int* boff, uint32_t* idx, float* val, int* nnz,
                              hipStream_t s);

}  // namespace regdock

namespace regdock {
hipError_t top_k(const float* scores, int count, int K, int32_t* out, hipStream_t s);
}

