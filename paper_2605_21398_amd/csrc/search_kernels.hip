// HIP kernels of the global grid-correlation search (Sec. IV), for gfx950.
//
// Per registration problem (setup, off the per-rotation path):
//   k_anchor         geometry centre a = mean of the mesh vertices (FP64)
//   k_object_grid    O[k] = min(O_t, O_m) on the n^3 canvas x_k = a + h(k - n/2)
//                    (Sec. IV-A: banded template of the signed distance, surface
//                    mask of the touchable distance, element-wise minimum)
//   k_pose_prep      probe poses -> rotation matrix + position (double)
//   k_swept          S_w[j] = 1 iff min_i f_p(T_i^{-1} y_j) <= 0 on the m^3 world
//                    lattice y_j = wc + h(j - m/2) (Sec. IV-A, swept occupancy)
//   k_cellmask       8-bit corner masks of S_w, 4x4x4-bricked, so one byte load
//                    gives all eight trilinear taps of a cell
//   k_rot_prep       SO(3) samples -> rotation matrices; input validation
//   pass1 + pass2(spectrum mode) on O   -> W = conj(F(O)) / n^3, kept resident
//
// Per rotation (the hot path; Sec. IV-B and IV-D):
//   pass1  k_rotvox_fwd_xy   per (rotation, z-plane): rotate-and-voxelise the
//                            swept grid by trilinear resampling, real-to-complex
//                            FFT along x (half-length complex trick), complex FFT
//                            along y, all in LDS; writes the plane into the
//                            pencil-tiled spectrum layout
//   pass2  k_zpass           per (rotation, tile of T z-pencils): FFT along z,
//                            multiply by W, inverse FFT along z, in LDS
//   pass3  k_inv_xy_argmax   per (rotation, z-plane): inverse FFT along y,
//                            complex-to-real along x, the exact low block added
//                            in double; the plane's four best column maxima
//                            as keys (orderable score bits, ~index) and a bound
//                            on every other voxel of the plane
//   k_select, k_certify,     candidates within the float32 error of each
//   k_rescore, k_finalize    rotation's maximum, exact re-scoring where that
//                            error exceeds the tolerance; score, shift, pose
//
// The paper's own form of the search rotates O instead (Sec. IV-D as printed):
// k_objcells turns O on the body lattice into cell classes and corner records,
// k_swept_canvas cuts the fixed swept canvas S out of S_w and S takes O's place
// in the spectrum; pass 1 then resamples the rotated object grid
// (k_rotvox_fwd_xy with REC), and the shift and pose follow from the reversed
// correlation (write_peak).
//
// Spectrum layout of one rotation (complex64, H = n (n/2 + 1) n elements):
//   tile t in [0, n * (n/2)/T): ky = t / (n/2/T), kx in [(t % (n/2/T)) T, +T)
//   tile t in [n (n/2)/T, +n/T): the Nyquist column kx = n/2, ky in a T-range
//   inside a tile: [z][T] -- T consecutive complex per z (one 128-byte segment
//   at T = 16), so pass 2 reads and writes whole tiles contiguously while pass 1
//   and pass 3 move T-element segments per (row, plane).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "fft_device.h"
#include "search_kernels.h"

namespace regdock {

// ------------------------------------------------------------ canvas traits

// index field of the peak keys (see key64): canvases up to 2^26 voxels
constexpr int FLAT_BITS_MAX = 26;

__host__ __device__ constexpr int largest_divisor_le(int v, int cap) {
    for (int d = cap; d >= 1; --d)
        if (v % d == 0) return d;
    return 1;
}

// lattice edge m = 2 ceil((sqrt(3) n + 2) / 2): the smallest even m with
// m - 2 >= sqrt(3) n, i.e. (m - 2)^2 >= 3 n^2 (exact in integers)
__host__ __device__ constexpr int lattice_edge_of(int n) {
    int m = 2;
    while ((long long)(m - 2) * (m - 2) < 3ll * n * n) m += 2;
    return m;
}

// Sizes of an edge-N canvas shared by every search path: the half spectrum,
// its pencil tiles and the swept lattice.
template <int N> struct Dims {
    static constexpr int N2 = N / 2;
    static constexpr int M = lattice_edge_of(N);          // swept lattice edge
    static constexpr int P = N2 + 1;                      // row pitch (complex)
    static constexpr int T = largest_divisor_le(N2, 16);  // tile width (complex)
    static constexpr int NT2 = N2 / T;                    // main tiles per ky row
    static constexpr int TILES = N * NT2 + N / T;         // tiles per rotation
    static constexpr size_t H = (size_t)N * P * N;        // complex per rotation
    static_assert(N % 2 == 0 && N % T == 0, "canvas edge must be even and tile the Nyquist column");
    static_assert(fft_supported(N) && fft_supported(N2), "edge must be 2^a 3^b 5^c");
    static_assert((size_t)N * N * N <= (1u << FLAT_BITS_MAX),
                  "flat indices must fit the index field of the peak keys");
};

// The fused plane passes: a whole plane in the LDS of one workgroup.
template <int N> struct Canvas : Dims<N> {
    using D = Dims<N>;
    using D::N2;
    using D::M;
    using D::P;
    using D::T;
    using D::NT2;
    using D::TILES;
    using D::H;
    // threads of a plane workgroup: from 96^3 up the plane fills enough LDS
    // that only one to three workgroups fit per CU, and workgroups of 8 (16
    // above 128^3, where one fits) waves give each SIMD more waves to hide LDS
    // and barrier latency
    static constexpr int NT = N > 128 ? 1024 : N >= 96 ? 512 : 256;
    static constexpr int WPE = N >= 96 ? 4 : 1;  // waves per SIMD asked of the compiler
    static_assert((size_t)N * P * 8 <= 160 * 1024, "plane must fit in LDS");
};

// Workgroup -> (rotation, plane).  Workgroups are dealt round-robin to the 8
// XCDs; when the batch is a multiple of 8, every plane of a rotation lands on
// the same XCD so its L2 keeps that rotation's lattice footprint.
__device__ __forceinline__ void map_plane_block(int bid, int count, int n, int& rot, int& z) {
    if ((count & 7) == 0) {
        const int xcd = bid & 7, local = bid >> 3;
        rot = (local / n) * 8 + xcd;
        z = local % n;
    } else {
        rot = bid / n;
        z = bid % n;
    }
}

// float -> unsigned bits whose unsigned order is the float order
__device__ __forceinline__ uint32_t ordered_bits(float f) {
    uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__host__ __device__ __forceinline__ float unordered_float(uint32_t o) {
    uint32_t b = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
#ifdef __HIP_DEVICE_COMPILE__
    return __uint_as_float(b);
#else
    float f;
    __builtin_memcpy(&f, &b, 4);
    return f;
#endif
}

__device__ __forceinline__ size_t brick_index(int ix, int iy, int iz, int mb) {
    return ((((size_t)(iz >> 2) * mb + (iy >> 2)) * mb + (ix >> 2)) << 6) + ((iz & 3) << 4) + ((iy & 3) << 2) + (ix & 3);
}


// Trilinear value of a binary lattice from the corner mask of the cell
// (bit cx + 2 cy + 4 cz is the lattice value at (i + cx, j + cy, k + cz)).
__device__ __forceinline__ float trilinear_mask(uint32_t mk, float fx, float fy, float fz) {
    const float gx = 1.0f - fx, gy = 1.0f - fy, gz = 1.0f - fz;
    const float b0 = (float)(mk & 1u), b1 = (float)((mk >> 1) & 1u), b2 = (float)((mk >> 2) & 1u), b3 = (float)((mk >> 3) & 1u);
    const float b4 = (float)((mk >> 4) & 1u), b5 = (float)((mk >> 5) & 1u), b6 = (float)((mk >> 6) & 1u), b7 = (float)((mk >> 7) & 1u);
    const float c00 = b0 * gx + b1 * fx, c10 = b2 * gx + b3 * fx;
    const float c01 = b4 * gx + b5 * fx, c11 = b6 * gx + b7 * fx;
    const float c0 = c00 * gy + c10 * fy, c1 = c01 * gy + c11 * fy;
    return c0 * gz + c1 * fz;
}

// Trilinear value of a real lattice from the eight corner values of a cell,
// held as two float4 (corner c = cx + 2 cy + 4 cz is component c % 4 of
// record c / 4): lerps along x, then y, then z.
__device__ __forceinline__ float trilinear_rec(float4 a, float4 b, float fx, float fy, float fz) {
    const float c00 = fmaf(fx, a.y - a.x, a.x), c10 = fmaf(fx, a.w - a.z, a.z);
    const float c01 = fmaf(fx, b.y - b.x, b.x), c11 = fmaf(fx, b.w - b.z, b.z);
    const float c0 = fmaf(fy, c10 - c00, c00), c1 = fmaf(fy, c11 - c01, c01);
    return fmaf(fz, c1 - c0, c0);
}

// Cell classes of a real lattice (the object grid of the rotated-object
// search): every corner 0, every corner the constant of the class (the deep
// penalty -rho), or mixed, with its corner values in a record.
constexpr uint8_t CELL_ZERO = 0, CELL_CONST = 1, CELL_MIXED = 2;

// Global -> LDS copy of COUNT elements by NTH threads with every thread's
// loads issued before the first is waited for (a loop that stores each load
// to LDS before issuing the next pays one memory latency per element):
// dst(e, src(e)) for e in [0, COUNT).
template <int COUNT, int NTH, class Src, class Dst>
__device__ __forceinline__ void batched_copy(Src src, Dst dst) {
    constexpr int PER = (COUNT + NTH - 1) / NTH;
    float2 v[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int e = threadIdx.x + i * NTH;
        if (COUNT % NTH == 0 || e < COUNT) v[i] = src(e);
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int e = threadIdx.x + i * NTH;
        if (COUNT % NTH == 0 || e < COUNT) dst(e, v[i]);
    }
}

// The same copy split in two: load() issues the global loads into registers
// and store() writes them to LDS later, so other loads can go out in between.
template <int COUNT, int NTH>
struct RegStage {
    static constexpr int PER = (COUNT + NTH - 1) / NTH;
    float2 v[PER];
    template <class Src>
    __device__ __forceinline__ void load(Src src) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = threadIdx.x + i * NTH;
            if (COUNT % NTH == 0 || e < COUNT) v[i] = src(e);
        }
    }
    template <class Dst>
    __device__ __forceinline__ void store(Dst dst) const {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = threadIdx.x + i * NTH;
            if (COUNT % NTH == 0 || e < COUNT) dst(e, v[i]);
        }
    }
};

// ------------------------------------------------------------- plane FFTs
// The plane lives in LDS as [y][kx] with pitch P = N/2 + 1 complex.

// Rows hold z[j] = s[2j] + i s[2j+1]; after the length-N/2 FFT, turn each row
// into X[k], k in [0, N/2], of the length-N real FFT:
//   X[k] = ((Z[k] + conj Z[N/2-k]) - i w^k (Z[k] - conj Z[N/2-k])) / 2.
// X[0] and X[N/2] are real; both go to slot 0 as X[0] + i X[N/2], so that the
// y transform runs over n/2 columns (unpack_nyquist splits the result).
template <int N, int NT, int ROWS = N>
__device__ __forceinline__ void r2c_post(float2* plane, const float2* tw) {
    using C = Dims<N>;
    constexpr int Q = C::N2 / 2 + 1;  // pairs (k, N/2 - k), k in [0, N/4]
    constexpr int R = NT / Q;         // rows per step: thread t keeps k = t % Q and its twiddles
    static_assert(R >= 1, "a plane workgroup covers the pairs of a row");
    const int t = threadIdx.x;
    if (t < R * Q) {
        const int k = t % Q, kk = C::N2 - k;
        const float2 wk = tw[k], wkk = tw[kk];
        for (int y = t / Q; y < ROWS; y += R) {
            float2* row = plane + y * C::P;
            if (k == 0) {
                const float2 z0 = row[0];
                row[0] = make_float2(z0.x + z0.y, z0.x - z0.y);
            } else {
                const float2 a = row[k], b = row[kk];
                // pair k
                float2 s = cadd(a, cconj(b)), d = csub(a, cconj(b));
                float2 wd = cmul(wk, d);
                float2 xk = make_float2(0.5f * (s.x + wd.y), 0.5f * (s.y - wd.x));
                // pair N/2 - k
                float2 s2 = cadd(b, cconj(a)), d2 = csub(b, cconj(a));
                float2 wd2 = cmul(wkk, d2);
                float2 xkk = make_float2(0.5f * (s2.x + wd2.y), 0.5f * (s2.y - wd2.x));
                row[k] = xk;
                row[kk] = xkk;
            }
        }
    }
    __syncthreads();
}

// Inverse of r2c_post (up to the factor 2 that makes the length-N/2 inverse
// FFT below equal the unnormalised length-N inverse real FFT):
//   Z[k] = (X[k] + conj X[N/2-k]) + i conj(w^k) (X[k] - conj X[N/2-k]).
// Slot 0 holds x[0] + i x[N/2] (pack_nyquist before the y transform), both
// real after it.
template <int N, int NT, int ROWS = N>
__device__ __forceinline__ void c2r_pre(float2* plane, const float2* tw) {
    using C = Dims<N>;
    constexpr int Q = C::N2 / 2 + 1;
    constexpr int R = NT / Q;
    static_assert(R >= 1, "a plane workgroup covers the pairs of a row");
    const int t = threadIdx.x;
    if (t < R * Q) {
        const int k = t % Q, kk = C::N2 - k;
        const float2 wk = tw[k], wkk = tw[kk];
        for (int y = t / Q; y < ROWS; y += R) {
            float2* row = plane + y * C::P;
            const float2 a = k == 0 ? make_float2(row[0].x, 0.0f) : row[k];
            const float2 b = k == 0 ? make_float2(row[0].y, 0.0f) : row[kk];
            float2 s = cadd(a, cconj(b)), d = csub(a, cconj(b));
            float2 wd = cmulc(d, wk);
            float2 zk = make_float2(s.x - wd.y, s.y + wd.x);
            if (k == 0) {
                row[0] = zk;
            } else {
                float2 s2 = cadd(b, cconj(a)), d2 = csub(b, cconj(a));
                float2 wd2 = cmulc(d2, wkk);
                row[kk] = make_float2(s2.x - wd2.y, s2.y + wd2.x);
                row[k] = zk;
            }
        }
    }
    __syncthreads();
}

// After the y transform of slot 0 (holding X0 + i XN, both real along y):
// Z[k] -> A[k] = (Z[k] + conj Z[-k]) / 2 in column 0 and B[k] = (Z[k] - conj
// Z[-k]) / 2i in column n/2, the transforms of X0 and XN.  One thread per pair
// (k, n - k), k in [0, n/2].
template <int N, int NT>
__device__ __forceinline__ void unpack_nyquist(float2* plane) {
    using C = Canvas<N>;
    for (int k = threadIdx.x; k <= N / 2; k += NT) {
        const int kk = (N - k) % N;
        const float2 z = plane[k * C::P], zz = plane[kk * C::P];
        const float2 a = make_float2(0.5f * (z.x + zz.x), 0.5f * (z.y - zz.y));
        const float2 b = make_float2(0.5f * (z.y + zz.y), 0.5f * (zz.x - z.x));
        plane[k * C::P] = a;
        plane[k * C::P + C::N2] = b;
        if (kk != k) {
            plane[kk * C::P] = cconj(a);
            plane[kk * C::P + C::N2] = cconj(b);
        }
    }
    __syncthreads();
}

// Before the inverse y transform: column 0 (A) and column n/2 (B) of each row
// become A + i B in column 0; after the transform its real and imaginary parts
// are the two real columns.
template <int N, int NT>
__device__ __forceinline__ void pack_nyquist(float2* plane) {
    using C = Canvas<N>;
    for (int k = threadIdx.x; k < N; k += NT) {
        const float2 a = plane[k * C::P], b = plane[k * C::P + C::N2];
        plane[k * C::P] = make_float2(a.x - b.y, a.y + b.x);
    }
    __syncthreads();
}

// forward 2D real FFT of the packed plane (x then y) and write to the tiled spectrum
template <int N, int NT>
__device__ __forceinline__ void plane_forward_and_store(float2* plane, const float2* tw, float2* __restrict__ spec_rot, int z) {
    using C = Canvas<N>;
    fft_lds<C::N2, false, N, NT, true, N>(plane, 1, C::P, tw);
    r2c_post<N, NT>(plane, tw);
    fft_lds<N, false, C::N2, NT, true, N>(plane, C::P, 1, tw);
    unpack_nyquist<N, NT>(plane);
    // LDS reads first, then the global stores
    batched_copy<N * C::N2, NT>([&](int e) { return plane[(e / C::N2) * C::P + e % C::N2]; },
                                   [&](int e, float2 v) {
                                       const int ky = e / C::N2, kx = e % C::N2;
                                       spec_rot[((size_t)(ky * C::NT2 + kx / C::T) * N + z) * C::T + (kx % C::T)] = v;
                                   });
    float2* nyq = spec_rot + (size_t)N * C::N2 * N;
    for (int ky = threadIdx.x; ky < N; ky += NT)
        nyq[((size_t)(ky / C::T) * N + z) * C::T + (ky % C::T)] = plane[ky * C::P + C::N2];
}

// ---------------------------------------------------- exact low-frequency block
// The correlation field's energy sits almost entirely in the lowest
// frequencies (the smooth, huge overlap with the -50 interior).  Those
// frequencies, max(|kx|, |ky|, |kz|) <= KLOW, are carried in double: pass 1 adds
// a double-precision 2D DFT of each plane at (kx in [0, KLOW], ky in [-KLOW,
// KLOW]); k_low_combine finishes the z direction and multiplies by the object's
// double-precision low block; pass 2 removes the block from the float32
// product; pass 3 adds the block's field back in double at every voxel.

__host__ __device__ constexpr int pow2floor(int v) {
    int p = 1;
    while (p * 2 <= v) p *= 2;
    return p;
}

__device__ __forceinline__ double2 dcmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ double2 dcmulc(double2 a, double2 b) {
    return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ int mod_n(int v, int n) {
    const int r = v % n;
    return r < 0 ? r + n : r;
}

// plane holds z[j] = s[2j] + i s[2j+1] per row; out[kx * NLY + ky + KLOW] =
// sum_{x,y} s[x,y] exp(-2 pi i (kx x + ky y) / N) in double.  tw64 is the
// double twiddle table in LDS.  Row sums over x run as second-order Goertzel
// recurrences per kx (one FMA and one subtraction per sample and frequency, no
// table reads); each row is split into CH contiguous chunks on CH lanes.  The
// row sums go to rbuf[y][kx] with kx rotated by y / 4 inside the row
// (low_slot), so that the 16 consecutive rows that the lanes of a wave read
// together in the y pass fall in distinct banks.
__device__ __forceinline__ int low_slot(int y, int kx) {
    static_assert(NLX == 4, "the rotation assumes four kx entries per row");
    return y * NLX + ((kx + (y >> 2)) & 3);
}
// x direction for ROWS rows of pitch N/2 + 1 (rbuf rows local to the block)
template <int N, int NT, int ROWS>
__device__ __forceinline__ void low_rows_x(const float2* plane, const double2* tw64, double2* rbuf) {
    using C = Dims<N>;
    static_assert(ROWS <= NT, "one row task set per pass");
    constexpr int CH = pow2floor(NT / ROWS) < 64 ? pow2floor(NT / ROWS) : 64;  // lanes per row, a power of two
    constexpr int JC = (C::N2 + CH - 1) / CH;
    // A wave takes RPW consecutive rows: lane l reads row l % RPW, chunk
    // l / RPW.  The lanes that read together (a half wave) then take distinct
    // rows, whose offsets 2 P y fall in distinct banks, rather than the chunks
    // of one row, which at n = 128 start 16 elements (32 banks of 4 bytes)
    // apart and hit the same banks.
    constexpr int RPW = 64 / CH;
    static_assert(CH <= 64 && ((ROWS + RPW - 1) / RPW) * 64 <= NT, "low-block x pass layout");
    const int t = threadIdx.x;
    const int y = (t >> 6) * RPW + (t & 63) % RPW, c = (t & 63) / RPW;
    if (y < ROWS) {
        const int j0 = c * JC, j1 = min(C::N2, j0 + JC);
        double coef[NLX], s1[NLX], s2[NLX];
        double sum0 = 0.0;
#pragma unroll
        for (int k = 1; k < NLX; ++k) {
            coef[k] = 2.0 * tw64[k].x;
            s1[k] = 0.0;
            s2[k] = 0.0;
        }
        for (int j = j0; j < j1; ++j) {
            const float2 v = plane[y * C::P + j];
            const double a = (double)v.x, b = (double)v.y;
            sum0 += a + b;
#pragma unroll
            for (int k = 1; k < NLX; ++k) {
                const double u0 = fma(coef[k], s1[k], a - s2[k]);
                const double u1 = fma(coef[k], u0, b - s1[k]);
                s2[k] = u0;
                s1[k] = u1;
            }
        }
        double2 acc[NLX];
        acc[0] = make_double2(sum0, 0.0);
        const int xl = 2 * j1 - 1;  // last sample of the chunk
#pragma unroll
        for (int k = 1; k < NLX; ++k) {
            // y = s1 - e^{-i w} s2 equals e^{+i w xl} * sum_x s[x] e^{-i w x}
            const double2 e1 = tw64[k];  // (cos w, -sin w)
            const double2 yk = make_double2(s1[k] - e1.x * s2[k], -e1.y * s2[k]);
            acc[k] = dcmul(yk, tw64[(k * xl) % N]);
            if (j1 <= j0) acc[k] = make_double2(0.0, 0.0);
        }
        // the CH chunks of a row sit RPW lanes apart
#pragma unroll
        for (int off = 32; off >= RPW; off >>= 1)
#pragma unroll
            for (int k = 0; k < NLX; ++k) {
                acc[k].x += __shfl_xor(acc[k].x, off, 64);
                acc[k].y += __shfl_xor(acc[k].y, off, 64);
            }
        if (c == 0)
#pragma unroll
            for (int k = 0; k < NLX; ++k) rbuf[low_slot(y, k)] = acc[k];
    }
}

// y direction from the row sums of all N rows of a plane
template <int N, int NT>
__device__ __forceinline__ void low_cols_y(const double2* rbuf, const double2* tw64, double2* __restrict__ out) {
    const int t = threadIdx.x;
    // y direction: CB lanes per (kx, ky) (CB a power of two, at most 16, with
    // NLOW2 CB <= NT), lane c taking rows c, c + CB, ...; a shuffle tree adds
    // the CB parts
    constexpr int CB = pow2floor(NT / NLOW2) < 16 ? pow2floor(NT / NLOW2) : 16;
    static_assert(CB >= 1 && NLOW2 * CB <= NT && 64 % CB == 0, "low-block y pass layout");
    double2 part = make_double2(0.0, 0.0);
    if (t < NLOW2 * CB) {
        const int o = t / CB, c = t % CB;
        const int kx = o / NLY, ky = o % NLY - KLOW;
        int idx = mod_n(ky * c, N);
        const int step = mod_n(ky * CB, N);
        for (int y = c; y < N; y += CB) {
            const double2 r = rbuf[low_slot(y, kx)], w = tw64[idx];
            part.x = fma(r.x, w.x, fma(-r.y, w.y, part.x));
            part.y = fma(r.x, w.y, fma(r.y, w.x, part.y));
            idx += step;
            idx -= idx >= N ? N : 0;
        }
    }
#pragma unroll
    for (int off = CB / 2; off >= 1; off >>= 1) {
        part.x += __shfl_xor(part.x, off, 64);
        part.y += __shfl_xor(part.y, off, 64);
    }
    if (t < NLOW2 * CB && (t % CB) == 0) out[t / CB] = part;
}

// the whole plane: x sums of every row, then the y direction
template <int N, int NT>
__device__ __forceinline__ void plane_low_dft(const float2* plane, const double2* tw64, double2* rbuf,
                                              double2* __restrict__ out) {
    low_rows_x<N, NT, N>(plane, tw64, rbuf);
    __syncthreads();
    low_cols_y<N, NT>(rbuf, tw64, out);
}

// S_r at canvas voxel (x, y, z) for rotation R: u = R (k - N/2) + m/2 in double
// (the lattice spans ~2N voxels, where float32 would leave ~1e-5 voxel of
// position error), then trilinear weights in float from the corner mask.
// Squared canvas radius (in voxels^2) beyond which S_r is zero, from the swept
// lattice's reach4 (k_lattice_reach): a rotated canvas voxel k samples a cell
// with an occupied corner only if |k - n/2| <= sqrt(reach4) / 2 + sqrt(3).  The
// small slack covers the rounding of the double rotation and of the
// generator's fixed-point walk.
__device__ __forceinline__ double canvas_reach2(const unsigned long long* reach4) {
    const double r = 0.5 * sqrt((double)*reach4) + 1.7320508075688772 + 1e-6;
    return r * r;
}

struct RotSampler {
    double r00, r01, r02, r10, r11, r12, r20, r21, r22;
    double hm, hn;
    __device__ __forceinline__ void load(const double* R, int m, int n) {
        r00 = R[0]; r01 = R[1]; r02 = R[2];
        r10 = R[3]; r11 = R[4]; r12 = R[5];
        r20 = R[6]; r21 = R[7]; r22 = R[8];
        hm = 0.5 * m;
        hn = 0.5 * n;
    }
    // lattice cell (brick address, or -1 outside) and the fractional position
    __device__ __forceinline__ long locate(int m, int mb, int x, int y, int z, float& fx, float& fy, float& fz) const {
        const double xc = (double)x - hn, yc = (double)y - hn, zc = (double)z - hn;
        const double ux = fma(r00, xc, fma(r01, yc, fma(r02, zc, hm)));
        const double uy = fma(r10, xc, fma(r11, yc, fma(r12, zc, hm)));
        const double uz = fma(r20, xc, fma(r21, yc, fma(r22, zc, hm)));
        const double fx0 = floor(ux), fy0 = floor(uy), fz0 = floor(uz);
        const int ix = (int)fx0, iy = (int)fy0, iz = (int)fz0;
        fx = (float)(ux - fx0);
        fy = (float)(uy - fy0);
        fz = (float)(uz - fz0);
        if (ix < 0 || iy < 0 || iz < 0 || ix >= m || iy >= m || iz >= m) return -1;
        return (long)brick_index(ix, iy, iz, mb);
    }
    __device__ __forceinline__ float sample(const uint8_t* __restrict__ cmask, int m, int mb, int x, int y, int z) const {
        float fx, fy, fz;
        const long a = locate(m, mb, x, y, z, fx, fy, fz);
        if (a < 0) return 0.0f;
        const uint32_t mk = cmask[a];
        return mk ? trilinear_mask(mk, fx, fy, fz) : 0.0f;
    }
    // the same on a real lattice given by cell classes and corner records
    __device__ __forceinline__ float sample_rec(const uint8_t* __restrict__ cls, const float4* __restrict__ rec, float cval,
                                                int m, int mb, int x, int y, int z) const {
        float fx, fy, fz;
        const long a = locate(m, mb, x, y, z, fx, fy, fz);
        if (a < 0) return 0.0f;
        const uint32_t c = cls[a];
        if (c == CELL_MIXED) return trilinear_rec(rec[2 * a], rec[2 * a + 1], fx, fy, fz);
        return c == CELL_CONST ? cval : 0.0f;
    }
};

// Trilinear value of a binary lattice cell as a polynomial in the fractions:
// with bit c = cx + 2 cy + 4 cz of the corner mask holding the lattice value
// b_c, sum_c b_c prod_axes (c ? f : 1 - f) expands to
//   c0 + c1 fx + c2 fy + c3 fz + c4 fx fy + c5 fx fz + c6 fy fz + c7 fx fy fz
// with c0 = b0, c1 = b1 - b0, c2 = b2 - b0, c3 = b4 - b0,
// c4 = b3 - b1 - b2 + b0, c5 = b5 - b1 - b4 + b0, c6 = b6 - b2 - b4 + b0,
// c7 = b7 - b3 - b5 - b6 + b1 + b2 + b4 - b0 (small integers).  The table
// holds them per mask, each scaled by 2^(-32 per fraction factor), so the
// fractions enter as their raw 32-bit fixed-point words converted to float
// (powers of two scale exactly).  Entry e: lut[2e] = (c0, c1, c2, c3),
// lut[2e + 1] = (c4, c5, c6, c7).
constexpr int TRI_LUT = 2 * 256;  // float4 entries

template <int NT>
__device__ __forceinline__ void build_trilinear_lut(float4* lut) {
    const float s1 = 2.3283064365386963e-10f;  // 2^-32
    const float s2 = s1 * s1, s3 = s2 * s1;
    for (int e = threadIdx.x; e < 256; e += NT) {
        int b[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) b[c] = (e >> c) & 1;
        lut[2 * e] = make_float4((float)b[0], (float)(b[1] - b[0]) * s1, (float)(b[2] - b[0]) * s1,
                                 (float)(b[4] - b[0]) * s1);
        lut[2 * e + 1] = make_float4((float)(b[3] - b[1] - b[2] + b[0]) * s2, (float)(b[5] - b[1] - b[4] + b[0]) * s2,
                                     (float)(b[6] - b[2] - b[4] + b[0]) * s2,
                                     (float)(b[7] - b[3] - b[5] - b[6] + b[1] + b[2] + b[4] - b[0]) * s3);
    }
}

// Per-axis parts of brick_index on a lattice of edge m (padded to mb bricks of
// 4 per axis): the brick coordinate times its stride in bytes, plus the
// position inside the brick.  The three parts of a cell occupy disjoint bits
// inside the brick and add up across bricks, so their sum is the address
// (below 2^31: mp^3 < 2^31 for every supported canvas).
template <int NT>
__device__ __forceinline__ void build_brick_tables(uint32_t* bax, uint32_t* bay, uint32_t* baz, int m, int mb) {
    for (int i = threadIdx.x; i < m; i += NT) {
        const uint32_t b = (uint32_t)i >> 2, r = (uint32_t)i & 3u;
        bax[i] = (b << 6) | r;
        bay[i] = ((b * (uint32_t)mb) << 6) | (r << 2);
        baz[i] = ((b * (uint32_t)mb * (uint32_t)mb) << 6) | (r << 4);
    }
}

// the polynomial at raw fraction words X, Y, Z (floats of the 32-bit words)
__device__ __forceinline__ float trilinear_poly(const float4* lut, uint32_t mk, float X, float Y, float Z) {
    const float4 a = lut[2 * mk], b = lut[2 * mk + 1];
    const float yz = fmaf(b.w, X, b.z);
    const float zc = fmaf(b.y, X, a.w);
    const float yc = fmaf(b.x, X, a.z);
    const float c0 = fmaf(a.y, X, a.x);
    return fmaf(fmaf(yz, Y, zc), Z, fmaf(yc, Y, c0));
}

// Fill the LDS plane with z[j] = S_r[2j] + i S_r[2j+1] for plane z (rows
// ybase .. ybase + ROWS - 1 of it, local row r at plane[r (n/2 + 1)]).  The
// corner-mask loads of several elements are issued together before any is
// used, so each lane keeps many gathers in flight.
//
// Every working lane owns fixed columns x = 2j, 2j+1 (the first YS n/2 lanes,
// YS = workgroup / (n/2); the other few are idle), so its lattice coordinates
// advance by a constant step per row: they are kept in 64-bit fixed point with
// 32 fractional bits (the integer cell is the high word, the trilinear
// fraction the low word), so a sample costs three integer additions instead of
// a double-precision matrix product.  The start and the step are rounded from
// double once: after n rows the drift is below 1e-8 voxel.  No bounds test is
// needed: rotations are orthonormal (checked and
// normalised in double at set-up) and |k - n/2| <= n sqrt(3) / 2, so with
// m = 2 ceil((sqrt(3) n + 2) / 2) every sample lies in [1, m - 1] on each axis
// (the launcher checks m).  Eight rows per batch keep 16 gathers in flight.
// Each value is the trilinear polynomial of its cell (table in LDS), with no
// branch on the mask.  The brick address of cell (ix, iy, iz) is the sum of
// three per-axis table entries (bax[ix] + bay[iy] + baz[iz], see
// build_brick_tables), three LDS reads in place of the shifts, masks and
// multiplies of brick_index.
template <int N, int NT, int ROWS = N>
__device__ __forceinline__ void generate_plane(float2* plane, const float4* lut, const uint32_t* bax,
                                               const uint32_t* bay, const uint32_t* baz, const RotSampler& rs,
                                               const uint8_t* __restrict__ cmask, int z, int ybase = 0) {
    using C = Dims<N>;
    static_assert(C::N2 <= NT, "a plane workgroup covers every column pair");
    constexpr int YS = NT / C::N2;  // row step of a lane (YS * N2 lanes work, the rest idle)
    constexpr int G = 8;               // rows per batch of loads
    const int j = threadIdx.x % C::N2, y0 = threadIdx.x / C::N2;
    if (threadIdx.x >= YS * C::N2 || y0 >= ROWS) return;
    const double two32 = 4294967296.0;
    long long U[2][3], D[3];
    {
        const double yc = (double)(ybase + y0) - rs.hn, zc = (double)z - rs.hn;
        for (int s2 = 0; s2 < 2; ++s2) {
            const double xc = (double)(2 * j + s2) - rs.hn;
            U[s2][0] = __double2ll_rn(fma(rs.r00, xc, fma(rs.r01, yc, fma(rs.r02, zc, rs.hm))) * two32);
            U[s2][1] = __double2ll_rn(fma(rs.r10, xc, fma(rs.r11, yc, fma(rs.r12, zc, rs.hm))) * two32);
            U[s2][2] = __double2ll_rn(fma(rs.r20, xc, fma(rs.r21, yc, fma(rs.r22, zc, rs.hm))) * two32);
        }
        D[0] = __double2ll_rn((double)YS * rs.r01 * two32);
        D[1] = __double2ll_rn((double)YS * rs.r11 * two32);
        D[2] = __double2ll_rn((double)YS * rs.r21 * two32);
    }
    for (int y = y0; y < ROWS; y += YS * G) {
        uint32_t addr[2 * G];
        float fx[2 * G], fy[2 * G], fz[2 * G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2) {
                const int q = 2 * g + s2;
                const uint32_t ix = (uint32_t)(U[s2][0] >> 32), iy = (uint32_t)(U[s2][1] >> 32),
                               iz = (uint32_t)(U[s2][2] >> 32);
                fx[q] = (float)(uint32_t)U[s2][0];
                fy[q] = (float)(uint32_t)U[s2][1];
                fz[q] = (float)(uint32_t)U[s2][2];
                addr[q] = bax[ix] + bay[iy] + baz[iz];
                U[s2][0] += D[0];
                U[s2][1] += D[1];
                U[s2][2] += D[2];
            }
        }
        uint32_t mk[2 * G];
#pragma unroll
        for (int q = 0; q < 2 * G; ++q) {
            const bool live = (ROWS % (YS * G) == 0) || y + (q / 2) * YS < ROWS;
            mk[q] = live ? (uint32_t)cmask[addr[q]] : 0u;
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int yy = y + g * YS;
            if ((ROWS % (YS * G) == 0) || yy < ROWS)
                plane[yy * C::P + j] = make_float2(trilinear_poly(lut, mk[2 * g], fx[2 * g], fy[2 * g], fz[2 * g]),
                                                   trilinear_poly(lut, mk[2 * g + 1], fx[2 * g + 1], fy[2 * g + 1],
                                                                  fz[2 * g + 1]));
        }
    }
}

// The plane of the rotated object grid (the search that rotates O, Sec.
// IV-D): the fixed-point walk of generate_plane over a real lattice held as
// cell classes (bricked bytes, as the corner masks) and corner records.  The
// class bytes of a batch are gathered first, then the records of its mixed
// cells; two rows per batch keep the four samples' records in 32
// registers.
template <int N, int NT>
__device__ __forceinline__ void generate_plane_rec(float2* plane, const uint32_t* bax, const uint32_t* bay,
                                                   const uint32_t* baz, const RotSampler& rs,
                                                   const uint8_t* __restrict__ cls, const float4* __restrict__ rec,
                                                   float cval, int z) {
    using C = Canvas<N>;
    static_assert(C::N2 <= NT, "a plane workgroup covers every column pair");
    constexpr int YS = NT / C::N2;
    constexpr int G = 2;
    const int j = threadIdx.x % C::N2, y0 = threadIdx.x / C::N2;
    if (threadIdx.x >= YS * C::N2 || y0 >= N) return;
    const double two32 = 4294967296.0;
    const float inv32 = 2.3283064365386963e-10f;  // 2^-32
    long long U[2][3], D[3];
    {
        const double yc = (double)y0 - rs.hn, zc = (double)z - rs.hn;
        for (int s2 = 0; s2 < 2; ++s2) {
            const double xc = (double)(2 * j + s2) - rs.hn;
            U[s2][0] = __double2ll_rn(fma(rs.r00, xc, fma(rs.r01, yc, fma(rs.r02, zc, rs.hm))) * two32);
            U[s2][1] = __double2ll_rn(fma(rs.r10, xc, fma(rs.r11, yc, fma(rs.r12, zc, rs.hm))) * two32);
            U[s2][2] = __double2ll_rn(fma(rs.r20, xc, fma(rs.r21, yc, fma(rs.r22, zc, rs.hm))) * two32);
        }
        D[0] = __double2ll_rn((double)YS * rs.r01 * two32);
        D[1] = __double2ll_rn((double)YS * rs.r11 * two32);
        D[2] = __double2ll_rn((double)YS * rs.r21 * two32);
    }
    for (int y = y0; y < N; y += YS * G) {
        uint32_t addr[2 * G];
        float fx[2 * G], fy[2 * G], fz[2 * G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2) {
                const int q = 2 * g + s2;
                const uint32_t ix = (uint32_t)(U[s2][0] >> 32), iy = (uint32_t)(U[s2][1] >> 32),
                               iz = (uint32_t)(U[s2][2] >> 32);
                fx[q] = (float)(uint32_t)U[s2][0] * inv32;
                fy[q] = (float)(uint32_t)U[s2][1] * inv32;
                fz[q] = (float)(uint32_t)U[s2][2] * inv32;
                addr[q] = bax[ix] + bay[iy] + baz[iz];
                U[s2][0] += D[0];
                U[s2][1] += D[1];
                U[s2][2] += D[2];
            }
        }
        uint32_t cl[2 * G];
#pragma unroll
        for (int q = 0; q < 2 * G; ++q) {
            const bool live = (N % (YS * G) == 0) || y + (q / 2) * YS < N;
            cl[q] = live ? (uint32_t)cls[addr[q]] : (uint32_t)CELL_ZERO;
        }
        float4 ra[2 * G], rb[2 * G];
#pragma unroll
        for (int q = 0; q < 2 * G; ++q) {
            ra[q] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            rb[q] = ra[q];
            if (cl[q] == CELL_MIXED) {
                ra[q] = rec[2 * (size_t)addr[q]];
                rb[q] = rec[2 * (size_t)addr[q] + 1];
            }
        }
        float v[2 * G];
#pragma unroll
        for (int q = 0; q < 2 * G; ++q)
            v[q] = cl[q] == CELL_MIXED ? trilinear_rec(ra[q], rb[q], fx[q], fy[q], fz[q])
                                       : (cl[q] == CELL_CONST ? cval : 0.0f);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int yy = y + g * YS;
            if ((N % (YS * G) == 0) || yy < N) plane[yy * C::P + j] = make_float2(v[2 * g], v[2 * g + 1]);
        }
    }
}

// ------------------------------------------------------------------ pass 1

// REC: the rotated grid is a real lattice (cell classes in cmask, corner
// records in crec, the class constant cval) instead of corner masks.
template <int N, int NT, int WPE, bool REC>
__global__ __launch_bounds__(NT, WPE) void k_rotvox_fwd_xy(const uint8_t* __restrict__ cmask, int m, int mb,
                                                       const double* __restrict__ rots, int count,
                                                       const float2* __restrict__ twg, const double2* __restrict__ tw64,
                                                       float2* __restrict__ spec, double2* __restrict__ lowT,
                                                       const float4* __restrict__ crec, float cval,
                                                       const unsigned long long* __restrict__ reach4) {
    using C = Canvas<N>;
    __shared__ float2 plane[N * C::P];
    __shared__ float2 tw[N];
    __shared__ double2 tws[N];
    // the trilinear table is used only while the plane is generated, the
    // low-block row sums only afterwards: they share one buffer
    constexpr int RB = N * NLX * (int)sizeof(double2), LB = TRI_LUT * (int)sizeof(float4);
    __shared__ __align__(16) unsigned char scratch_lds[RB > LB ? RB : LB];
    __shared__ uint32_t bax[C::M], bay[C::M], baz[C::M];
    double2* rbuf = reinterpret_cast<double2*>(scratch_lds);
    float4* lut = reinterpret_cast<float4*>(scratch_lds);
    static_assert(N <= NT, "one twiddle per thread at most");
    int rot, z;
    map_plane_block(blockIdx.x, count, N, rot, z);
    if (!REC && reach4) {
        // a plane beyond the swept lattice's reach (on a padded canvas): S_r is
        // zero there, and so are its spectrum slices and low-block sums
        const double dz = z - N / 2;
        if (dz * dz > canvas_reach2(reach4)) {
            float2* spec_rot = spec + (size_t)rot * C::H;
            for (int e = threadIdx.x; e < N * C::N2; e += NT) {
                const int ky = e / C::N2, kx = e % C::N2;
                spec_rot[((size_t)(ky * C::NT2 + kx / C::T) * N + z) * C::T + (kx % C::T)] = make_float2(0.0f, 0.0f);
            }
            float2* nyq = spec_rot + (size_t)N * C::N2 * N;
            for (int ky = threadIdx.x; ky < N; ky += NT)
                nyq[((size_t)(ky / C::T) * N + z) * C::T + (ky % C::T)] = make_float2(0.0f, 0.0f);
            double2* lo = lowT + ((size_t)rot * N + z) * NLOW2;
            for (int e = threadIdx.x; e < NLOW2; e += NT) lo[e] = make_double2(0.0, 0.0);
            return;
        }
    }
    // the global loads (twiddles, rotation) go out first; the tables are built
    // while they are in flight
    const int tid = threadIdx.x;
    float2 twv;
    double2 tw64v;
    if (tid < N) {
        twv = twg[tid];
        tw64v = tw64[tid];
    }
    RotSampler rs;
    rs.load(rots + rot * 9, m, N);
    if (!REC) build_trilinear_lut<NT>(lut);
    build_brick_tables<NT>(bax, bay, baz, C::M, mb);
    if (tid < N) {
        tw[tid] = twv;
        tws[tid] = tw64v;
    }
    __syncthreads();
    if (REC)
        generate_plane_rec<N, NT>(plane, bax, bay, baz, rs, cmask, crec, cval, z);
    else
        generate_plane<N, NT>(plane, lut, bax, bay, baz, rs, cmask, z);
    __syncthreads();
    plane_low_dft<N, NT>(plane, tws, rbuf, lowT + ((size_t)rot * N + z) * NLOW2);
    plane_forward_and_store<N, NT>(plane, tw, spec + (size_t)rot * C::H, z);
}

// pass 1 on a real grid (the object grid O): same transform, no rotation
template <int N>
__global__ __launch_bounds__(Canvas<N>::NT, Canvas<N>::WPE) void k_grid_fwd_xy(const float* __restrict__ grid, const float2* __restrict__ twg,
                                                     const double2* __restrict__ tw64, float2* __restrict__ spec,
                                                     double2* __restrict__ lowT) {
    using C = Canvas<N>;
    __shared__ float2 plane[N * C::P];
    __shared__ float2 tw[N];
    __shared__ double2 tws[N];
    __shared__ double2 rbuf[N * NLX];
    const int z = blockIdx.x;
    for (int i = threadIdx.x; i < N; i += C::NT) {
        tw[i] = twg[i];
        tws[i] = tw64[i];
    }
    for (int e = threadIdx.x; e < N * C::N2; e += C::NT) {
        const int y = e / C::N2, j = e % C::N2;
        const float* row = grid + ((size_t)z * N + y) * N;
        plane[y * C::P + j] = make_float2(row[2 * j], row[2 * j + 1]);
    }
    __syncthreads();
    plane_low_dft<N, Canvas<N>::NT>(plane, tws, rbuf, lowT + (size_t)z * NLOW2);
    plane_forward_and_store<N, Canvas<N>::NT>(plane, tw, spec, z);
}

// ------------------------------------------------------------------ pass 2
// MODE 0: x <- IFFT_z(FFT_z(x) * W);  MODE 1: W <- conj(FFT_z(x)) * scale

template <int N, int MODE, int ZT>
__global__ __launch_bounds__(ZT) void k_zpass(float2* __restrict__ spec, const float2* __restrict__ W, float2* __restrict__ wout,
                                               const float2* __restrict__ twg, float scale) {
    using C = Dims<N>;
    constexpr int E = N * C::T;
    constexpr int PER = (E + ZT - 1) / ZT;
    __shared__ float2 buf[E];
    __shared__ float2 tw[N];
    // Block -> (tile, rotation).  Blocks are dealt round-robin to the 8 XCDs;
    // with a batch that is a multiple of 8, each XCD takes rotations xcd,
    // xcd + 8, ... of one tile in a row, so its L2 reads the tile of W once.
    const int count = gridDim.x / C::TILES;
    int tile, rot;
    if (MODE == 0 && (count & 7) == 0) {
        const int xcd = blockIdx.x & 7, local = blockIdx.x >> 3, per = count >> 3;
        tile = local / per;
        rot = (local % per) * 8 + xcd;
    } else {
        tile = blockIdx.x % C::TILES;
        rot = blockIdx.x / C::TILES;
    }
    float2* src = spec + (size_t)rot * C::H + (size_t)tile * E;
    // the twiddles and the tile go out together; the tile of W is loaded into
    // registers after them and arrives while the forward FFT runs
    RegStage<N, ZT> st_tw;
    RegStage<E, ZT> st_tile;
    st_tw.load([&](int i) { return twg[i]; });
    st_tile.load([&](int i) { return src[i]; });
    st_tw.store([&](int i, float2 v) { tw[i] = v; });
    st_tile.store([&](int i, float2 v) { buf[i] = v; });
    float2 wv[PER];
    if (MODE == 0) {
        const float2* w = W + (size_t)tile * E;
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int i = threadIdx.x + r * ZT;
            wv[r] = (E % ZT == 0 || i < E) ? w[i] : make_float2(0.0f, 0.0f);
        }
    }
    __syncthreads();
    fft_lds<N, false, C::T, ZT, true, N>(buf, C::T, 1, tw);
    if (MODE == 0) {
        // the low block (max(|kx|,|ky|,|kz|) <= KLOW) is carried exactly elsewhere
        const int ky = tile / C::NT2;
        const bool low_tile = tile < N * C::NT2 && (tile % C::NT2) == 0 && (ky <= KLOW || ky >= N - KLOW);
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int i = threadIdx.x + r * ZT;
            if (E % ZT != 0 && i >= E) break;
            const int kz = i / C::T, kx = i % C::T;
            const bool low = low_tile && kx <= KLOW && (kz <= KLOW || kz >= N - KLOW);
            buf[i] = low ? make_float2(0.0f, 0.0f) : cmul(buf[i], wv[r]);
        }
        __syncthreads();
        fft_lds<N, true, C::T, ZT, true, N>(buf, C::T, 1, tw);
        for (int i = threadIdx.x; i < E; i += ZT) src[i] = buf[i];
    } else {
        float2* dst = wout + (size_t)tile * E;
        for (int i = threadIdx.x; i < E; i += ZT) dst[i] = cscale(cconj(buf[i]), scale);
    }
}

// ------------------------------------------------------------------ pass 3
// Per (rotation, plane): inverse FFT along y, complex-to-real along x, then the
// plane's four best column maxima as keys (orderable score bits, ~flat index),
// a bound on its other voxels and its sum of squares.  The float32 field only
// locates candidates; their scores are recomputed exactly by k_rescore where
// its error could exceed the tolerance.

// key = orderable bits of a double, low FLAT_BITS bits replaced by ~flat
// (flat < 2^FLAT_BITS = 67,108,864 > 400^3); the value keeps 52 - FLAT_BITS
// mantissa bits (relative truncation below 2^-26, under float32's rounding)
constexpr int FLAT_BITS = FLAT_BITS_MAX;
constexpr unsigned long long FLAT_MASK = (1ull << FLAT_BITS) - 1;
__device__ __forceinline__ unsigned long long key64(double v, uint32_t flat) {
    unsigned long long b = (unsigned long long)__double_as_longlong(v);
    b = (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
    return (b & ~FLAT_MASK) | (FLAT_MASK - flat);
}
__device__ __forceinline__ double key_value(unsigned long long k) {
    unsigned long long b = k & ~FLAT_MASK;
    b = (b & 0x8000000000000000ull) ? (b & 0x7fffffffffffffffull) : ~b;
    return __longlong_as_double((long long)b);
}
__device__ __forceinline__ uint32_t key_flat(unsigned long long k) { return (uint32_t)(FLAT_MASK - (k & FLAT_MASK)); }

// Scan of ROWS field rows (rows y0 .. y0 + ROWS - 1 of plane z; local row r
// at rows[r * (n/2 + 1)], its low-block row at btab[r * NLX]) and the merges
// of the lanes' and waves' maxima: one record of KTOP keys and the bound to
// o, the rows' sum of squares to ss_out.
template <int N, int NT, int ROWS>
__device__ __forceinline__ void scan_rows(const float2* rows, const double2* btab, const double2* tws, int z, int y0,
                                          unsigned long long (*wtop)[KTOP + 1], double* wss, double* wsec,
                                          unsigned long long* __restrict__ o, double* __restrict__ ss_out,
                                          float* __restrict__ corr_out) {
    // Every working lane keeps the same columns x = 2j, 2j+1 (YS n/2 lanes
    // work, the rest idle), so its low-block phases live in registers.  Each
    // column of a lane ("virtual lane": x fixed, rows y0, y0 + YS, ...) keeps
    // its largest value with the lowest row holding it, and the largest value
    // below that (or equal to it at another row).  The plane then reports the
    // four best virtual-lane maxima as keys and a bound: the larger of the
    // fifth-best virtual-lane maximum and every virtual lane's second value.
    // No voxel outside the four keys exceeds the bound, so a candidate window
    // that the bound does not reach holds only those keys.
    using C = Dims<N>;
    constexpr int NW = NT / 64;
    static_assert(C::N2 <= NT, "a plane workgroup covers every column pair");
    constexpr int YS = NT / C::N2;
    const int j = threadIdx.x % C::N2;
    double2 w0[NLX], w1[NLX];
#pragma unroll
    for (int k = 1; k < NLX; ++k) {
        w0[k] = tws[(k * 2 * j) % N];
        w1[k] = tws[(k * (2 * j + 1)) % N];
    }
    double m1a = -INFINITY, m2a = -INFINITY, m1b = -INFINITY, m2b = -INFINITY;
    int ya = -1, yb = -1;
    float ss = 0.0f;
    const int ystart = threadIdx.x < YS * C::N2 ? threadIdx.x / C::N2 : ROWS;
    for (int yl = ystart; yl < ROWS; yl += YS) {
        const int y = y0 + yl;
        const float2 v = rows[yl * C::P + j];
        const double2* b = btab + yl * NLX;
        double c0 = b[0].x, c1 = b[0].x;
#pragma unroll
        for (int k = 1; k < NLX; ++k) {
            const double2 bk = b[k];
            c0 = fma(bk.x, w0[k].x, fma(bk.y, w0[k].y, c0));
            c1 = fma(bk.x, w1[k].x, fma(bk.y, w1[k].y, c1));
        }
        const double v0 = (double)v.x + c0, v1 = (double)v.y + c1;
        // rows ascend, so a strict test keeps the lowest row of a tie, and a
        // tie becomes the second value
        ya = v0 > m1a ? y : ya;
        m2a = fmax(m2a, fmin(v0, m1a));
        m1a = fmax(m1a, v0);
        yb = v1 > m1b ? y : yb;
        m2b = fmax(m2b, fmin(v1, m1b));
        m1b = fmax(m1b, v1);
        ss = fmaf(v.x, v.x, fmaf(v.y, v.y, ss));
        if (corr_out) {
            const uint32_t flat0 = (uint32_t)(((z * N) + y) * N + 2 * j);
            corr_out[flat0] = (float)v0;
            corr_out[flat0 + 1] = (float)v1;
        }
    }
    // each lane: its two virtual-lane maxima as keys, sorted
    const uint32_t rowbase = (uint32_t)(z * N) * N;
    unsigned long long ka = ya >= 0 ? key64(m1a, rowbase + (uint32_t)(ya * N + 2 * j)) : 0ull;
    unsigned long long kb = yb >= 0 ? key64(m1b, rowbase + (uint32_t)(yb * N + 2 * j + 1)) : 0ull;
    unsigned long long t0 = ka > kb ? ka : kb, t1 = ka > kb ? kb : ka;
    double sec = fmax(m2a, m2b);
    // wave: five rounds of a wave maximum over the lanes' list heads; the lane
    // holding the maximum (keys are unique) shifts its list up
    unsigned long long wt[KTOP + 1];
#pragma unroll
    for (int r = 0; r < KTOP + 1; ++r) {
        unsigned long long mx = t0;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const unsigned long long o = __shfl_xor(mx, off, 64);
            mx = o > mx ? o : mx;
        }
        const bool mine = t0 == mx && mx != 0ull;
        t0 = mine ? t1 : t0;
        t1 = mine ? 0ull : t1;
        wt[r] = mx;
    }
    double ds = (double)ss;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        ds += __shfl_xor(ds, off, 64);
        sec = fmax(sec, __shfl_xor(sec, off, 64));
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int r = 0; r < KTOP + 1; ++r) wtop[wave][r] = wt[r];
        wss[wave] = ds;
        wsec[wave] = sec;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        // the plane, in wave 0: five rounds of a maximum over the waves' sorted
        // lists (lane w < NW holds wave w's list and pops its head when it
        // wins), then the sums of squares and the bounds of the waves
        static_assert(NW <= 64, "one lane per wave of the workgroup");
        constexpr int SPAN = pow2floor(2 * NW - 1);  // lanes holding lists, rounded up to a power of two
        const int l = threadIdx.x;
        unsigned long long L[KTOP + 1], b[KTOP + 1];
#pragma unroll
        for (int r = 0; r < KTOP + 1; ++r) L[r] = l < NW ? wtop[l][r] : 0ull;
#pragma unroll
        for (int r = 0; r < KTOP + 1; ++r) {
            unsigned long long mx = L[0];
#pragma unroll
            for (int off = SPAN / 2; off >= 1; off >>= 1) {
                const unsigned long long o = __shfl_xor(mx, off, 64);
                mx = o > mx ? o : mx;
            }
            const bool mine = L[0] == mx && mx != 0ull;
#pragma unroll
            for (int q = 0; q < KTOP; ++q) L[q] = mine ? L[q + 1] : L[q];
            L[KTOP] = mine ? 0ull : L[KTOP];
            b[r] = mx;
        }
        double tot = l < NW ? wss[l] : 0.0, bound = l < NW ? wsec[l] : -INFINITY;
#pragma unroll
        for (int off = SPAN / 2; off >= 1; off >>= 1) {
            tot += __shfl_xor(tot, off, 64);
            bound = fmax(bound, __shfl_xor(bound, off, 64));
        }
        if (l == 0) {
            if (b[KTOP]) bound = fmax(bound, key_value(b[KTOP]));
#pragma unroll
            for (int r = 0; r < KTOP; ++r) o[r] = b[r];
            o[KTOP] = (unsigned long long)__double_as_longlong(bound);
            *ss_out = tot;
        }
    }
}

template <int N, int NT, int WPE>
__global__ __launch_bounds__(NT, WPE) void k_inv_xy_argmax(const float2* __restrict__ spec, int count, const float2* __restrict__ twg,
                                                       const double2* __restrict__ tw64, const double2* __restrict__ Plow,
                                                       unsigned long long* __restrict__ ptop, double* __restrict__ pssq,
                                                       float* __restrict__ corr_out) {
    using C = Canvas<N>;
    constexpr int NW = NT / 64;
    __shared__ float2 plane[N * C::P];
    __shared__ float2 tw[N];
    __shared__ double2 btab[N * NLX];
    __shared__ double2 az[NLOW2];
    __shared__ double2 tws[N];
    __shared__ unsigned long long wtop[NW][KTOP + 1];
    __shared__ double wss[NW];
    __shared__ double wsec[NW];
    static_assert(N <= NT && NLOW2 <= NT, "one twiddle and one low-block row per thread at most");
    int rot, z;
    map_plane_block(blockIdx.x, count, N, rot, z);
    // every global load of the plane is issued before the first is waited for:
    // the twiddles, this thread's row of the low-block product, the spectrum
    const int tid = threadIdx.x;
    float2 twv;
    double2 tw64v;
    if (tid < N) {
        twv = twg[tid];
        tw64v = tw64[tid];
    }
    double2 pz[NLY];
    if (tid < NLOW2) {
        const double2* P = Plow + (size_t)rot * NLOW3 + tid * NLY;
#pragma unroll
        for (int kzi = 0; kzi < NLY; ++kzi) pz[kzi] = P[kzi];
    }
    const float2* spec_rot = spec + (size_t)rot * C::H;
    RegStage<N * C::N2, NT> st_main;
    RegStage<N, NT> st_nyq;
    st_main.load([&](int e) {
        const int ky = e / C::N2, kx = e % C::N2;
        return spec_rot[((size_t)(ky * C::NT2 + kx / C::T) * N + z) * C::T + (kx % C::T)];
    });
    const float2* nyq = spec_rot + (size_t)N * C::N2 * N;
    st_nyq.load([&](int ky) { return nyq[((size_t)(ky / C::T) * N + z) * C::T + (ky % C::T)]; });
    if (tid < N) {
        tw[tid] = twv;
        tws[tid] = tw64v;
    }
    st_main.store([&](int e, float2 v) { plane[(e / C::N2) * C::P + e % C::N2] = v; });
    st_nyq.store([&](int ky, float2 v) { plane[ky * C::P + C::N2] = v; });
    __syncthreads();
    // low block of this plane: az[kx][ky] = sum_kz P[kx][ky][kz] e^{+2 pi i kz z / N}
    if (tid < NLOW2) {
        double2 acc = make_double2(0.0, 0.0);
#pragma unroll
        for (int kzi = 0; kzi < NLY; ++kzi) {
            const double2 t = dcmulc(pz[kzi], tws[mod_n((kzi - KLOW) * z, N)]);
            acc.x += t.x;
            acc.y += t.y;
        }
        az[tid] = acc;
    }
    // az is complete before the barrier that ends pack_nyquist and is read
    // only after it
    pack_nyquist<N, NT>(plane);
    fft_lds<N, true, C::N2, NT, true, N>(plane, C::P, 1, tw);
    // btab[y][kx] = sum_ky az[kx][ky] e^{+2 pi i ky y / N}, doubled for kx > 0
    // (the field sums Re b_0 + 2 sum_kx Re(b_kx e^{+2 pi i kx x / N}))
    for (int t = threadIdx.x; t < N * NLX; t += NT) {
        const int y = t / NLX, kx = t % NLX;
        double2 acc = make_double2(0.0, 0.0);
#pragma unroll
        for (int kyi = 0; kyi < NLY; ++kyi) {
            const double2 v = dcmulc(az[kx * NLY + kyi], tws[mod_n((kyi - KLOW) * y, N)]);
            acc.x += v.x;
            acc.y += v.y;
        }
        btab[t] = kx > 0 ? make_double2(2.0 * acc.x, 2.0 * acc.y) : acc;
    }
    c2r_pre<N, NT>(plane, tw);
    fft_lds<C::N2, true, N, NT, true, N>(plane, 1, C::P, tw);
    scan_rows<N, NT, N>(plane, btab, tws, z, 0, wtop, wss, wsec, ptop + ((size_t)rot * N + z) * KREC,
                        pssq + (size_t)rot * N + z, corr_out);
}

// Per rotation (absolute index base + block): the field maximum v (double,
// from the keys), the RMS of the float32 part (from the plane sums of squares),
// the window 2 eps with eps = REGK_EPS_SCALE * 2^-24 * rms * log2(n^3) bounding
// the float32 error, and every key inside [v - 2 eps, v] as a candidate (at
// most CMAX, in descending key order).  If a plane's bound (no voxel of the
// plane besides its keys exceeds it) reaches the window, the plane may hold
// more: the rotation is marked as overflowed.
__global__ __launch_bounds__(256) void k_select(const unsigned long long* __restrict__ ptop, const double* __restrict__ pssq,
                                                int n, int units, double eps_per_rms, int base, int32_t* __restrict__ cand_idx,
                                                int32_t* __restrict__ cand_n, double* __restrict__ window,
                                                uint8_t* __restrict__ ovf, double* __restrict__ best_val,
                                                int32_t* __restrict__ best_flat, int* __restrict__ stats) {
    __shared__ unsigned long long red[4];
    __shared__ double red_ss[4];
    __shared__ double thr_s;
    __shared__ int cnt;
    __shared__ unsigned long long list[CMAX];
    __shared__ int overflow;
    const int rot = blockIdx.x, r = base + blockIdx.x;
    const unsigned long long* T = ptop + (size_t)rot * units * KREC;
    // the best key and the sum of the units' (planes' or row blocks') sums of
    // squares (a fixed shuffle tree per wave, then the four waves in order)
    unsigned long long mx = 0;
    double ss = 0.0;
    for (int zz = threadIdx.x; zz < units; zz += 256) {
        mx = T[zz * KREC] > mx ? T[zz * KREC] : mx;
        ss += pssq[(size_t)rot * units + zz];
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(mx, off, 64);
        mx = o > mx ? o : mx;
        ss += __shfl_xor(ss, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = mx;
        red_ss[threadIdx.x >> 6] = ss;
    }
    if (threadIdx.x == 0) {
        cnt = 0;
        overflow = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long b = red[0];
        double ssq = red_ss[0];
        for (int w = 1; w < 4; ++w) {
            b = red[w] > b ? red[w] : b;
            ssq += red_ss[w];
        }
        const double rms = sqrt(ssq / ((double)n * n * n));
        const double v = key_value(b);
        thr_s = v - 2.0 * eps_per_rms * rms;
        window[r] = 2.0 * eps_per_rms * rms;
        best_val[r] = v;
        best_flat[r] = (int32_t)key_flat(b);
    }
    __syncthreads();
    const double thr = thr_s;
    for (int i = threadIdx.x; i < units * KREC; i += 256) {
        const unsigned long long k = T[i];
        if (i % KREC == KTOP) {
            if (__longlong_as_double((long long)k) >= thr) overflow = 1;
        } else if (k != 0ull && key_value(k) >= thr) {
            const int slot = atomicAdd(&cnt, 1);
            if (slot < CMAX) list[slot] = k;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int c = cnt;
        if (c > CMAX) {
            overflow = 1;
            c = CMAX;
        }
        // descending key order (insertion sort of at most CMAX keys)
        for (int q = 1; q < c; ++q) {
            const unsigned long long k = list[q];
            int b = q - 1;
            while (b >= 0 && list[b] < k) {
                list[b + 1] = list[b];
                --b;
            }
            list[b + 1] = k;
        }
        for (int q = 0; q < c; ++q) cand_idx[(size_t)r * CMAX + q] = (int32_t)key_flat(list[q]);
        cand_n[r] = c;
        ovf[r] = overflow ? 1 : 0;
        atomicAdd(stats + 0, 1);
        atomicAdd(stats + 1, c);
        if (overflow) atomicAdd(stats + 2, 1);
    }
}

// Which rotations need exact re-scoring.  tol = 1e-4 * max |v| over the call's
// rotations.  A rotation whose window 2 eps is within tol is settled by the
// field maximum (value within eps, index within 2 eps <= tol of the best); the
// others (or all, when asked) are listed, in rotation order, for k_rescore.
// Listed rotations whose window also overflowed are counted as uncertain.
__global__ __launch_bounds__(1024) void k_certify(const double* __restrict__ best_val, const double* __restrict__ window,
                                                  const uint8_t* __restrict__ ovf, int count, int always,
                                                  int32_t* __restrict__ need_list, int* __restrict__ need_count,
                                                  int* __restrict__ stats) {
    __shared__ double red[16];
    __shared__ int part[1024];
    double mx = 0.0;
    for (int i = threadIdx.x; i < count; i += 1024) mx = fmax(mx, fabs(best_val[i]));
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = red[0];
        for (int w = 1; w < 16; ++w) b = fmax(b, red[w]);
        red[0] = b;
    }
    __syncthreads();
    const double tol = 1e-4 * red[0];
    // contiguous chunk per thread, exclusive scan of the chunk counts
    const int per = (count + 1023) / 1024;
    const int i0 = threadIdx.x * per, i1 = min(count, i0 + per);
    int c = 0, bad = 0;
    for (int i = i0; i < i1; ++i) {
        const bool wide = window[i] > tol;
        c += (always || wide) ? 1 : 0;
        bad += (wide && ovf[i]) ? 1 : 0;
    }
    part[threadIdx.x] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int t = 0; t < 1024; ++t) {
            const int v = part[t];
            part[t] = run;
            run += v;
        }
        *need_count = run;
        atomicAdd(stats + 4, run);
    }
    __syncthreads();
    int pos = part[threadIdx.x];
    for (int i = i0; i < i1; ++i)
        if (always || window[i] > tol) need_list[pos++] = i;
    if (bad) atomicAdd(stats + 3, bad);
}

// Exact score of one candidate shift d of one rotation:
//   sum over the nonzero voxels k of O of O[k] * S_r[(k + d) mod n]
// with S_r resampled exactly as in pass 1 and the sum accumulated in double.
// The nonzero list is cut into `nslice` slices; a grid-stride loop runs over
// (listed rotation, candidate, slice) items, skipping empty candidate slots,
// and each item writes its slice sum; k_apply adds the slices in a fixed order.
__global__ __launch_bounds__(256) void k_rescore(const uint32_t* __restrict__ nz_idx, const float* __restrict__ nz_val,
                                                 const int* __restrict__ nz_count, int n, int nslice,
                                                 const uint8_t* __restrict__ cmask, int m, int mb,
                                                 const float4* __restrict__ crec, float cval,
                                                 const double* __restrict__ rots, const int32_t* __restrict__ need_list,
                                                 const int* __restrict__ need_count, const int32_t* __restrict__ cand_idx,
                                                 const int32_t* __restrict__ cand_n, double* __restrict__ cand_part) {
    __shared__ double red[4];
    const int nnz = *nz_count;
    const int per = (nnz + nslice - 1) / nslice;
    const int items = (*need_count) * CMAX * nslice;
    for (int it = blockIdx.x; it < items; it += gridDim.x) {
        const int sl = it % nslice, pc = it / nslice;
        const int pos = pc / CMAX, c = pc % CMAX;
        const int rot = need_list[pos];
        if (c >= cand_n[rot]) continue;  // uniform across the workgroup
        const uint32_t flat = (uint32_t)cand_idx[(size_t)rot * CMAX + c];
        const int dx = (int)(flat % n), dy = (int)((flat / n) % n), dz = (int)(flat / ((uint32_t)n * n));
        RotSampler rs;
        rs.load(rots + rot * 9, m, n);
        const int j0 = sl * per, j1 = min(nnz, j0 + per);
        double acc = 0.0;
        for (int j = j0 + threadIdx.x; j < j1; j += 256) {
            const uint32_t k = nz_idx[j];
            int x = (int)(k & 0x3ffu) + dx, y = (int)((k >> 10) & 0x3ffu) + dy, zz = (int)(k >> 20) + dz;
            x -= x >= n ? n : 0;
            y -= y >= n ? n : 0;
            zz -= zz >= n ? n : 0;
            const float sv = crec ? rs.sample_rec(cmask, crec, cval, m, mb, x, y, zz) : rs.sample(cmask, m, mb, x, y, zz);
            if (sv != 0.0f) acc += (double)nz_val[j] * (double)sv;
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) cand_part[(size_t)pc * nslice + sl] = ((red[0] + red[1]) + red[2]) + red[3];
        __syncthreads();
    }
}

// Finish the low block along z: L[kx][ky][kz] = sum_z lowT[z][kx][ky] e^{-2 pi i kz z / n},
// summed in a fixed order (independent of scheduling).
// MODE 0 (per rotation): out = L * Wlow.  MODE 1 (object): out = conj(L) * scale.
template <int MODE, int N>
__global__ __launch_bounds__(256) void k_low_combine(const double2* __restrict__ lowT, const double2* __restrict__ tw64,
                                                     const double2* __restrict__ Wlow, double scale, double2* __restrict__ out) {
    // One block per rotation.  Lane l < NLOW2 of each half wave owns the
    // (kx, ky) pair l; the 8 half waves take the planes z = h, h + 8, ... (the
    // 28 pairs of a plane are contiguous, so each half wave reads them in one
    // coalesced load), then the 8 partial sums are added per output.  All
    // loads of a lane are issued before the first is used, and the twiddles
    // are read from LDS.
    constexpr int HW = 256 / 32;
    constexpr int ZI = (N + HW - 1) / HW;  // planes per half wave
    constexpr int ZC = ZI < 16 ? ZI : 16;  // planes of a half wave loaded at once
    static_assert(NLOW2 <= 32, "one (kx, ky) pair per lane of a half wave");
    __shared__ double2 red[HW][NLOW2][NLY];
    __shared__ double2 tws[N];
    const int rot = blockIdx.x, h = threadIdx.x >> 5, l = threadIdx.x & 31;
    const double2* T = lowT + (size_t)rot * N * NLOW2 + l;
    double2 acc[NLY];
#pragma unroll
    for (int k = 0; k < NLY; ++k) acc[k] = make_double2(0.0, 0.0);
    for (int c0 = 0; c0 < ZI; c0 += ZC) {
        double2 v[ZC];
        if (l < NLOW2) {
#pragma unroll
            for (int i = 0; i < ZC; ++i) {
                const int zz = h + (c0 + i) * HW;
                v[i] = (N % HW == 0 && ZI % ZC == 0) || zz < N ? T[(size_t)zz * NLOW2] : make_double2(0.0, 0.0);
            }
        }
        if (c0 == 0) {
            for (int i = threadIdx.x; i < N; i += 256) tws[i] = tw64[i];
            __syncthreads();
        }
        if (l < NLOW2) {
#pragma unroll
            for (int i = 0; i < ZC; ++i) {
                const int zz = h + (c0 + i) * HW;
                if (!(N % HW == 0 && ZI % ZC == 0) && zz >= N) break;
#pragma unroll
                for (int k = 0; k < NLY; ++k) {
                    const double2 t = dcmul(v[i], tws[mod_n((k - KLOW) * zz, N)]);
                    acc[k].x += t.x;
                    acc[k].y += t.y;
                }
            }
        }
    }
    if (l < NLOW2) {
#pragma unroll
        for (int k = 0; k < NLY; ++k) red[h][l][k] = acc[k];
    }
    __syncthreads();
    for (int o = threadIdx.x; o < NLOW3; o += 256) {
        const int kxy = o / NLY, k = o % NLY;
        double2 L = red[0][kxy][k];
#pragma unroll
        for (int w = 1; w < HW; ++w) {
            L.x += red[w][kxy][k].x;
            L.y += red[w][kxy][k].y;
        }
        out[(size_t)rot * NLOW3 + o] = MODE == 0 ? dcmul(L, Wlow[o]) : make_double2(L.x * scale, -L.y * scale);
    }
}

// ------------------------------------------------------------- finalize
// score, signed shift and FP64 pose of a peak: t = wc - R a + h R shift

// rotobj: the field is C'[e] = sum_j S[j] O_q[j + e] of the rotated-object
// search, whose shift of Eq. (xcorr) is dk = -e, and the pose is
// t = center_world - R a + h dk (the object is rotated about its anchor, which
// sits at the canvas centre); otherwise t = center_world - R a + h R d.
__device__ __forceinline__ void write_peak(int i, double score, uint32_t flat, const float* __restrict__ quats, int n, double h,
                                           const double* __restrict__ anchor, const double* wc, int rotobj,
                                           float* __restrict__ out_score, int32_t* __restrict__ out_shift,
                                           double* __restrict__ out_pose) {
    int d[3] = {(int)(flat % n), (int)((flat / n) % n), (int)(flat / ((uint32_t)n * n))};
    for (int a = 0; a < 3; ++a) {
        if (d[a] >= n / 2) d[a] -= n;
        if (rotobj) d[a] = -d[a];
    }
    if (out_score) out_score[i] = (float)score;
    if (out_shift) {
        out_shift[3 * i] = d[0];
        out_shift[3 * i + 1] = d[1];
        out_shift[3 * i + 2] = d[2];
    }
    if (out_pose) {
        double q[4] = {quats[4 * i], quats[4 * i + 1], quats[4 * i + 2], quats[4 * i + 3]};
        const double nq = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        for (int a = 0; a < 4; ++a) q[a] /= nq;
        const double w = q[0], x = q[1], y = q[2], zq = q[3];
        const double Rm[9] = {1 - 2 * (y * y + zq * zq), 2 * (x * y - w * zq), 2 * (x * zq + w * y),
                              2 * (x * y + w * zq), 1 - 2 * (x * x + zq * zq), 2 * (y * zq - w * x),
                              2 * (x * zq - w * y), 2 * (y * zq + w * x), 1 - 2 * (x * x + y * y)};
        double* o = out_pose + 7 * i;
        for (int a = 0; a < 4; ++a) o[a] = q[a];
        for (int r = 0; r < 3; ++r) {
            double ra = 0, rd = 0;
            for (int c = 0; c < 3; ++c) {
                ra += Rm[3 * r + c] * anchor[c];
                rd += Rm[3 * r + c] * (double)d[c];
            }
            o[4 + r] = wc[r] - ra + h * (rotobj ? (double)d[r] : rd);
        }
    }
}

// field maxima of a call's rotations -> outputs (arrays offset to the call)
__global__ void k_finalize(const double* __restrict__ best_val, const int32_t* __restrict__ best_flat, int count,
                           const float* __restrict__ quats, int n, double h, const double* __restrict__ anchor, double wc0,
                           double wc1, double wc2, int rotobj, float* __restrict__ out_score, int32_t* __restrict__ out_shift,
                           double* __restrict__ out_pose) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const double wc[3] = {wc0, wc1, wc2};
    write_peak(i, best_val[i], (uint32_t)best_flat[i], quats, n, h, anchor, wc, rotobj, out_score, out_shift, out_pose);
}

// re-scored rotations: the best exact candidate (ties: lowest flat index)
// replaces the field maximum
__global__ void k_apply(const int32_t* __restrict__ need_list, const int* __restrict__ need_count,
                        const int32_t* __restrict__ cand_idx, const int32_t* __restrict__ cand_n,
                        const double* __restrict__ cand_part, int nslice, const float* __restrict__ quats, int n, double h,
                        const double* __restrict__ anchor, double wc0, double wc1, double wc2, int rotobj,
                        float* __restrict__ out_score, int32_t* __restrict__ out_shift, double* __restrict__ out_pose) {
    const int nc = *need_count;
    const double wc[3] = {wc0, wc1, wc2};
    for (int pos = blockIdx.x * blockDim.x + threadIdx.x; pos < nc; pos += gridDim.x * blockDim.x) {
        const int i = need_list[pos];
        const int cn = cand_n[i];
        double best = -1.0e308;
        uint32_t flat = 0xffffffffu;
        for (int c = 0; c < cn; ++c) {
            const double* part = cand_part + ((size_t)pos * CMAX + c) * nslice;
            double v = 0.0;
            for (int sl = 0; sl < nslice; ++sl) v += part[sl];
            const uint32_t f = (uint32_t)cand_idx[(size_t)i * CMAX + c];
            if (v > best || (v == best && f < flat)) {
                best = v;
                flat = f;
            }
        }
        if (cn > 0) write_peak(i, best, flat, quats, n, h, anchor, wc, rotobj, out_score, out_shift, out_pose);
    }
}

// ------------------------------------------- nonzero list of the object grid
// (ascending flat index, so the exact sums run in a fixed order)

__global__ void k_nz_count(const float* __restrict__ O, size_t n3, int* __restrict__ bcount) {
    __shared__ int wc[4];
    const size_t id = (size_t)blockIdx.x * 256 + threadIdx.x;
    const bool nz = id < n3 && O[id] != 0.0f;
    const unsigned long long b = __ballot(nz);
    if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = __popcll(b);
    __syncthreads();
    if (threadIdx.x == 0) bcount[blockIdx.x] = wc[0] + wc[1] + wc[2] + wc[3];
}

__global__ __launch_bounds__(1024) void k_nz_scan(const int* __restrict__ bcount, int nb, int* __restrict__ boff,
                                                  int* __restrict__ total) {
    __shared__ int part[1024];
    const int per = (nb + 1023) / 1024;
    const int b0 = threadIdx.x * per, b1 = min(nb, b0 + per);
    int s = 0;
    for (int b = b0; b < b1; ++b) s += bcount[b];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int t = 0; t < 1024; ++t) {
            const int v = part[t];
            part[t] = run;
            run += v;
        }
        *total = run;
    }
    __syncthreads();
    int run = part[threadIdx.x];
    for (int b = b0; b < b1; ++b) {
        boff[b] = run;
        run += bcount[b];
    }
}

__global__ void k_nz_write(const float* __restrict__ O, size_t n3, int n, const int* __restrict__ boff,
                           uint32_t* __restrict__ idx, float* __restrict__ val) {
    __shared__ int wc[4];
    const size_t id = (size_t)blockIdx.x * 256 + threadIdx.x;
    const float v = id < n3 ? O[id] : 0.0f;
    const bool nz = v != 0.0f;
    const unsigned long long b = __ballot(nz);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) wc[wave] = __popcll(b);
    __syncthreads();
    int base = boff[blockIdx.x];
    for (int w = 0; w < wave; ++w) base += wc[w];
    if (nz) {
        const int r = base + __popcll(b & ((1ull << lane) - 1ull));
        const uint32_t kx = (uint32_t)(id % n), ky = (uint32_t)((id / n) % n), kz = (uint32_t)(id / ((size_t)n * n));
        idx[r] = kx | (ky << 10) | (kz << 20);
        val[r] = v;
    }
}

// ----------------------------------------------------------- setup kernels

// a = mean of the vertices, one workgroup, fixed-order reduction in double
__global__ __launch_bounds__(256) void k_anchor(const float* __restrict__ V, int nv, double* __restrict__ anchor) {
    __shared__ double acc[3][256];
    double s[3] = {0, 0, 0};
    for (int i = threadIdx.x; i < nv; i += 256)
        for (int a = 0; a < 3; ++a) s[a] += (double)V[3 * i + a];
    for (int a = 0; a < 3; ++a) acc[a][threadIdx.x] = s[a];
    __syncthreads();
    for (int st = 128; st >= 1; st >>= 1) {
        if (threadIdx.x < st)
            for (int a = 0; a < 3; ++a) acc[a][threadIdx.x] += acc[a][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x < 3) anchor[threadIdx.x] = acc[threadIdx.x][0] / (double)nv;
}

// squared distance from p to triangle abc (closest-point case analysis of
// Ericson, Real-Time Collision Detection, Sec. 5.1.5), in double: the object
// grid's jump at f_o = -tau_in1 is then decided on the same side as an FP64
// evaluation up to rounding order
struct d3 {
    double x, y, z;
};
__device__ __forceinline__ d3 d3sub(d3 a, d3 b) { return d3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ double d3dot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ d3 d3axpy(d3 a, double v, d3 u) { return d3{a.x + v * u.x, a.y + v * u.y, a.z + v * u.z}; }

__device__ __forceinline__ double tri_dist2(d3 p, d3 a, d3 b, d3 c) {
    const d3 ab = d3sub(b, a), ac = d3sub(c, a), ap = d3sub(p, a);
    const double d1 = d3dot(ab, ap), d2 = d3dot(ac, ap);
    d3 q;
    if (d1 <= 0.0 && d2 <= 0.0) {
        q = a;
    } else {
        const d3 bp = d3sub(p, b), cp = d3sub(p, c);
        const double d3v = d3dot(ab, bp), d4 = d3dot(ac, bp);
        const double d5 = d3dot(ab, cp), d6 = d3dot(ac, cp);
        const double vc = d1 * d4 - d3v * d2;
        const double vb = d5 * d2 - d1 * d6;
        const double va = d3v * d6 - d5 * d4;
        if (d3v >= 0.0 && d4 <= d3v) {
            q = b;
        } else if (vc <= 0.0 && d1 >= 0.0 && d3v <= 0.0) {
            q = d3axpy(a, d1 / (d1 - d3v), ab);
        } else if (d6 >= 0.0 && d5 <= d6) {
            q = c;
        } else if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
            q = d3axpy(a, d2 / (d2 - d6), ac);
        } else if (va <= 0.0 && (d4 - d3v) >= 0.0 && (d5 - d6) >= 0.0) {
            q = d3axpy(b, (d4 - d3v) / ((d4 - d3v) + (d5 - d6)), d3sub(c, b));
        } else {
            const double den = 1.0 / (va + vb + vc);
            q = d3axpy(d3axpy(a, vb * den, ab), vc * den, ac);
        }
    }
    const d3 d = d3sub(p, q);
    return d3dot(d, d);
}

// banded template, surface mask and their minimum (Sec. IV-A)
__device__ __forceinline__ double object_value(double fo, double dt, double tau_out1, double tau_in1, double rho) {
    double ot;
    if (fo >= 0.0 && fo < tau_out1) ot = 1.0 - fo / tau_out1;
    else if (fo < 0.0 && fo > -tau_in1) ot = 1.0 + fo / tau_in1;
    else if (fo <= -tau_in1) ot = -rho;
    else ot = 0.0;
    const double om = fmax(0.0, 1.0 - fabs(dt) / tau_out1);
    return fmin(ot, om);
}

// capped-cylinder SDF of the probe (tip disk at the origin, axis +z), in
// double so that the swept occupancy switches at f_p = 0 where an FP64
// evaluation does
__device__ __forceinline__ double probe_sdf(double x, double y, double z, double r, double L) {
    const double q1 = sqrt(x * x + y * y) - r;
    const double q2 = fabs(z - 0.5 * L) - 0.5 * L;
    const double a = fmax(q1, 0.0), b = fmax(q2, 0.0);
    return fmin(fmax(q1, q2), 0.0) + sqrt(a * a + b * b);
}

// ---- object grid by scatter (per object) ----------------------------------
// Distances matter only inside the band (tau_out1 + h): every face updates
// the voxels of its bounding box grown by the band with atomicMin on double
// bits (non-negative doubles order like their bits), so the minimum is exact there
// and independent of the order.  Inside/outside comes from +z ray crossing
// parity: every face toggles, in each column its projection covers, the bits of
// the voxels below the crossing (atomicXor on per-column bit words), with the
// same simulation-of-simplicity tie rule at shared edges as the FP64 oracle.

constexpr unsigned long long DBL_MAX_BITS = 0x7fefffffffffffffull;

__global__ void k_obj_init(unsigned long long* __restrict__ d2, unsigned long long* __restrict__ dt2, size_t n3,
                           uint32_t* __restrict__ par, size_t nwords) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n3) {
        d2[i] = DBL_MAX_BITS;
        dt2[i] = DBL_MAX_BITS;
    }
    if (i < nwords) par[i] = 0u;
}

__device__ __forceinline__ void face_box(const double* lo_w, const double* hi_w, const double* anchor, double h, int n,
                                         int* lo, int* hi) {
    const double half = 0.5 * n;
    for (int j = 0; j < 3; ++j) {
        lo[j] = (int)ceil((lo_w[j] - anchor[j]) / h + half);
        hi[j] = (int)floor((hi_w[j] - anchor[j]) / h + half);
        lo[j] = lo[j] < 0 ? 0 : lo[j];
        hi[j] = hi[j] > n - 1 ? n - 1 : hi[j];
    }
}

__global__ __launch_bounds__(256) void k_obj_faces(const float* __restrict__ V, const int32_t* __restrict__ F,
                                                   const uint8_t* __restrict__ touch, int n, double h,
                                                   const double* __restrict__ anchor, double band,
                                                   unsigned long long* __restrict__ d2, unsigned long long* __restrict__ dt2) {
    const int f = blockIdx.x;
    const int i0 = F[3 * f], i1 = F[3 * f + 1], i2 = F[3 * f + 2];
    const d3 a{V[3 * i0], V[3 * i0 + 1], V[3 * i0 + 2]};
    const d3 b{V[3 * i1], V[3 * i1 + 1], V[3 * i1 + 2]};
    const d3 c{V[3 * i2], V[3 * i2 + 1], V[3 * i2 + 2]};
    const bool tf = touch[f] != 0;
    const double an[3] = {anchor[0], anchor[1], anchor[2]};
    double lo_w[3] = {fmin(a.x, fmin(b.x, c.x)) - band, fmin(a.y, fmin(b.y, c.y)) - band, fmin(a.z, fmin(b.z, c.z)) - band};
    double hi_w[3] = {fmax(a.x, fmax(b.x, c.x)) + band, fmax(a.y, fmax(b.y, c.y)) + band, fmax(a.z, fmax(b.z, c.z)) + band};
    int lo[3], hi[3];
    face_box(lo_w, hi_w, an, h, n, lo, hi);
    const int ex = hi[0] - lo[0] + 1, ey = hi[1] - lo[1] + 1, ez = hi[2] - lo[2] + 1;
    if (ex <= 0 || ey <= 0 || ez <= 0) return;
    const int cnt = ex * ey * ez;
    const double band2 = band * band;
    const double hn = 0.5 * n;
    for (int q = threadIdx.x; q < cnt; q += 256) {
        const int kx = lo[0] + q % ex, ky = lo[1] + (q / ex) % ey, kz = lo[2] + q / (ex * ey);
        const d3 p{an[0] + h * (kx - hn), an[1] + h * (ky - hn), an[2] + h * (kz - hn)};
        const double dd = tri_dist2(p, a, b, c);
        if (dd < band2) {
            const size_t id = ((size_t)kz * n + ky) * n + kx;
            const unsigned long long bits = (unsigned long long)__double_as_longlong(dd);
            atomicMin(d2 + id, bits);
            if (tf) atomicMin(dt2 + id, bits);
        }
    }
}

__device__ __forceinline__ int orient_sos(double ax, double ay, double bx, double by, double px, double py) {
    const double o = (bx - ax) * (py - ay) - (by - ay) * (px - ax);
    if (o > 0) return 1;
    if (o < 0) return -1;
    if (by != ay) return (ay - by) > 0 ? 1 : -1;
    if (bx != ax) return (bx - ax) > 0 ? 1 : -1;
    return 0;
}

__global__ __launch_bounds__(64) void k_obj_parity(const float* __restrict__ V, const int32_t* __restrict__ F, int n, double h,
                                                   const double* __restrict__ anchor, int W, uint32_t* __restrict__ par) {
    const int f = blockIdx.x;
    const int i0 = F[3 * f], i1 = F[3 * f + 1], i2 = F[3 * f + 2];
    const double a[3] = {V[3 * i0], V[3 * i0 + 1], V[3 * i0 + 2]};
    const double b[3] = {V[3 * i1], V[3 * i1 + 1], V[3 * i1 + 2]};
    const double c[3] = {V[3 * i2], V[3 * i2 + 1], V[3 * i2 + 2]};
    const double an[3] = {anchor[0], anchor[1], anchor[2]};
    const double hn = 0.5 * n;
    int clo[2], chi[2];
    for (int j = 0; j < 2; ++j) {
        const double mn = fmin(a[j], fmin(b[j], c[j])), mx = fmax(a[j], fmax(b[j], c[j]));
        clo[j] = (int)floor((mn - an[j]) / h + hn);
        chi[j] = (int)ceil((mx - an[j]) / h + hn);
        clo[j] = clo[j] < 0 ? 0 : clo[j];
        chi[j] = chi[j] > n - 1 ? n - 1 : chi[j];
    }
    const int ex = chi[0] - clo[0] + 1, ey = chi[1] - clo[1] + 1;
    if (ex <= 0 || ey <= 0) return;
    for (int q = threadIdx.x; q < ex * ey; q += 64) {
        const int kx = clo[0] + q % ex, ky = clo[1] + q / ex;
        const double px = an[0] + h * (kx - hn), py = an[1] + h * (ky - hn);
        const int s1 = orient_sos(a[0], a[1], b[0], b[1], px, py);
        const int s2 = orient_sos(b[0], b[1], c[0], c[1], px, py);
        const int s3 = orient_sos(c[0], c[1], a[0], a[1], px, py);
        if (!((s1 > 0 && s2 > 0 && s3 > 0) || (s1 < 0 && s2 < 0 && s3 < 0))) continue;
        const double w1 = (b[0] - a[0]) * (py - a[1]) - (b[1] - a[1]) * (px - a[0]);
        const double w2 = (c[0] - b[0]) * (py - b[1]) - (c[1] - b[1]) * (px - b[0]);
        const double w3 = (a[0] - c[0]) * (py - c[1]) - (a[1] - c[1]) * (px - c[0]);
        const double zi = (w2 * a[2] + w3 * b[2] + w1 * c[2]) / (w1 + w2 + w3);
        int below = 0;  // voxels of the column with z < zi
        while (below < n && an[2] + h * (below - hn) < zi) ++below;
        uint32_t* col = par + ((size_t)ky * n + kx) * W;
        for (int w = 0; w < W && 32 * w < below; ++w) {
            const int top = below - 32 * w;
            atomicXor(col + w, top >= 32 ? 0xffffffffu : ((1u << top) - 1u));
        }
    }
}

__global__ void k_obj_finalize(const unsigned long long* __restrict__ d2, const unsigned long long* __restrict__ dt2,
                               const uint32_t* __restrict__ par, int W, int n, double tau_out1, double tau_in1, double rho,
                               float* __restrict__ O, float* __restrict__ fo_out) {
    const size_t n3 = (size_t)n * n * n;
    const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n3) return;
    const int kx = (int)(id % n), ky = (int)((id / n) % n), kz = (int)(id / ((size_t)n * n));
    const bool inside = (par[((size_t)ky * n + kx) * W + (kz >> 5)] >> (kz & 31)) & 1u;
    const double dm = d2[id] == DBL_MAX_BITS ? INFINITY : sqrt(__longlong_as_double((long long)d2[id]));
    const double dt = dt2[id] == DBL_MAX_BITS ? INFINITY : sqrt(__longlong_as_double((long long)dt2[id]));
    const double fo = inside ? -dm : dm;
    O[id] = (float)object_value(fo, dt, tau_out1, tau_in1, rho);
    if (fo_out) fo_out[id] = (float)fo;
}

// ---- swept occupancy by scatter (per request) -----------------------------
// Each pose visits the lattice points of its cylinder's bounding box (grown by
// a small margin) and stores 1 where f_p <= 0; stores are idempotent, so the
// result does not depend on the order of the poses.

__global__ void k_fill_u8(uint8_t* __restrict__ p, size_t cnt, uint8_t v) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) p[i] = v;
}

__global__ __launch_bounds__(256) void k_swept_pose(const double* __restrict__ pz, double r, double L, int m, double h,
                                                    double wc0, double wc1, double wc2, uint8_t* __restrict__ Sw) {
    const double* P = pz + 12 * blockIdx.x;
    const double wc[3] = {wc0, wc1, wc2};
    const double ax[3] = {P[2], P[5], P[8]};  // probe axis in world
    const double hm = 0.5 * m;
    int lo[3], hi[3];
    for (int j = 0; j < 3; ++j) {
        const double e = r * sqrt(fmax(0.0, 1.0 - ax[j] * ax[j])) + 1e-3;
        const double c0 = P[9 + j], c1 = P[9 + j] + L * ax[j];
        lo[j] = (int)ceil((fmin(c0, c1) - e - wc[j]) / h + hm);
        hi[j] = (int)floor((fmax(c0, c1) + e - wc[j]) / h + hm);
        lo[j] = lo[j] < 0 ? 0 : lo[j];
        hi[j] = hi[j] > m - 1 ? m - 1 : hi[j];
    }
    const int ex = hi[0] - lo[0] + 1, ey = hi[1] - lo[1] + 1, ez = hi[2] - lo[2] + 1;
    if (ex <= 0 || ey <= 0 || ez <= 0) return;
    const int cnt = ex * ey * ez;
    for (int q = threadIdx.x; q < cnt; q += 256) {
        const int jx = lo[0] + q % ex, jy = lo[1] + (q / ex) % ey, jz = lo[2] + q / (ex * ey);
        const double dx = wc0 + h * (jx - hm) - P[9], dy = wc1 + h * (jy - hm) - P[10], dz = wc2 + h * (jz - hm) - P[11];
        const double lx = P[0] * dx + P[3] * dy + P[6] * dz;
        const double ly = P[1] * dx + P[4] * dy + P[7] * dz;
        const double lz = P[2] * dx + P[5] * dy + P[8] * dz;
        if (probe_sdf(lx, ly, lz, r, L) <= 0.0) Sw[((size_t)jz * m + jy) * m + jx] = 1;
    }
}

// poses (qw qx qy qz tx ty tz) -> R (row-major, from the normalised quaternion)
// and p, 12 doubles per pose
__global__ void k_pose_prep(const float* __restrict__ poses, int np, double* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    double q[4] = {poses[7 * i], poses[7 * i + 1], poses[7 * i + 2], poses[7 * i + 3]};
    const double nq = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const double w = q[0] / nq, x = q[1] / nq, y = q[2] / nq, z = q[3] / nq;
    double* o = out + 12 * i;
    o[0] = 1 - 2 * (y * y + z * z); o[1] = 2 * (x * y - w * z); o[2] = 2 * (x * z + w * y);
    o[3] = 2 * (x * y + w * z); o[4] = 1 - 2 * (x * x + z * z); o[5] = 2 * (y * z - w * x);
    o[6] = 2 * (x * z - w * y); o[7] = 2 * (y * z + w * x); o[8] = 1 - 2 * (x * x + y * y);
    o[9] = poses[7 * i + 4]; o[10] = poses[7 * i + 5]; o[11] = poses[7 * i + 6];
}

// corner masks over the padded, bricked lattice; taps beyond the lattice are 0
__global__ void k_cellmask(const uint8_t* __restrict__ Sw, int m, int mp, uint8_t* __restrict__ cm) {
    const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t mp3 = (size_t)mp * mp * mp;
    if (id >= mp3) return;
    const int ix = (int)(id % mp), iy = (int)((id / mp) % mp), iz = (int)(id / ((size_t)mp * mp));
    uint32_t mk = 0;
    for (int c = 0; c < 8; ++c) {
        const int x = ix + (c & 1), y = iy + ((c >> 1) & 1), z = iz + ((c >> 2) & 1);
        if (x < m && y < m && z < m && Sw[((size_t)z * m + y) * m + x]) mk |= 1u << c;
    }
    cm[brick_index(ix, iy, iz, mp / 4)] = (uint8_t)mk;
}

// Reach of the swept lattice: the largest (2x - m)^2 + (2y - m)^2 + (2z - m)^2
// over its occupied points, i.e. four times the squared distance from the
// lattice centre.  A rotated canvas voxel k samples a cell with an occupied
// corner only if |k - n/2| <= sqrt(reach4) / 2 + sqrt(3) (rotations keep
// distances from the centre, and a cell's corners lie within sqrt(3) of any
// point in it), so rows and planes of the canvas beyond that radius hold
// exact zeros.  One workgroup per (z, block of 16 rows); reach4 starts at 0.
__global__ __launch_bounds__(256) void k_lattice_reach(const uint8_t* __restrict__ Sw, int m,
                                                       unsigned long long* __restrict__ reach4) {
    const int yb = blockIdx.x % ((m + 15) / 16), z = blockIdx.x / ((m + 15) / 16);
    const long long dz = 2LL * z - m;
    unsigned long long best = 0;
    for (int y = yb * 16; y < m && y < yb * 16 + 16; ++y) {
        const long long dy = 2LL * y - m, dyz = dy * dy + dz * dz;
        const uint8_t* row = Sw + ((size_t)z * m + y) * m;
        for (int x = threadIdx.x; x < m; x += 256) {
            const long long dx = 2LL * x - m;
            if (row[x]) best = max(best, (unsigned long long)(dyz + dx * dx));
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) best = max(best, (unsigned long long)__shfl_xor(best, off, 64));
    __shared__ unsigned long long wbest[4];
    if ((threadIdx.x & 63) == 0) wbest[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long b = max(max(wbest[0], wbest[1]), max(wbest[2], wbest[3]));
        if (b) atomicMax(reach4, b);
    }
}

// SO(3) samples -> rotation matrices (double math, float storage) + checks
// transpose: store R^T, the map from canvas offsets to body-lattice offsets of
// the rotated-object search
__global__ void k_rot_prep(const float* __restrict__ so3, int M, int transpose, double* __restrict__ rots,
                           int* __restrict__ err) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    double q[4] = {so3[4 * i], so3[4 * i + 1], so3[4 * i + 2], so3[4 * i + 3]};
    const double n2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    const double nq = sqrt(n2);
    if (!(nq >= 1.0 - 1e-3 && nq <= 1.0 + 1e-3)) atomicOr(err, REGK_ERR_QUAT);
    const double w = q[0] / nq, x = q[1] / nq, y = q[2] / nq, z = q[3] / nq;
    double* o = rots + 9 * i;
    o[0] = 1 - 2 * (y * y + z * z); o[1] = 2 * (x * y - w * z); o[2] = 2 * (x * z + w * y);
    o[3] = 2 * (x * y + w * z); o[4] = 1 - 2 * (x * x + z * z); o[5] = 2 * (y * z - w * x);
    o[6] = 2 * (x * z - w * y); o[7] = 2 * (y * z + w * x); o[8] = 1 - 2 * (x * x + y * y);
    if (transpose) {
        double t = o[1]; o[1] = o[3]; o[3] = t;
        t = o[2]; o[2] = o[6]; o[6] = t;
        t = o[5]; o[5] = o[7]; o[7] = t;
    }
}

// Cell classes and corner records of a real lattice over the padded, bricked
// lattice (the object grid on the body lattice, for the rotated-object
// search); taps beyond the lattice are 0.  Records are written for mixed
// cells only.
__global__ void k_objcells(const float* __restrict__ G, int m, int mp, float cval, uint8_t* __restrict__ cls,
                           float4* __restrict__ rec) {
    const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t mp3 = (size_t)mp * mp * mp;
    if (id >= mp3) return;
    const int ix = (int)(id % mp), iy = (int)((id / mp) % mp), iz = (int)(id / ((size_t)mp * mp));
    float v[8];
    bool zero = true, cst = true;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int x = ix + (c & 1), y = iy + ((c >> 1) & 1), z = iz + ((c >> 2) & 1);
        v[c] = (x < m && y < m && z < m) ? G[((size_t)z * m + y) * m + x] : 0.0f;
        zero = zero && v[c] == 0.0f;
        cst = cst && v[c] == cval;
    }
    const size_t b = brick_index(ix, iy, iz, mp / 4);
    cls[b] = zero ? CELL_ZERO : cst ? CELL_CONST : CELL_MIXED;
    if (!zero && !cst) {
        rec[2 * b] = make_float4(v[0], v[1], v[2], v[3]);
        rec[2 * b + 1] = make_float4(v[4], v[5], v[6], v[7]);
    }
}

// S[k] = S_w at center_world + h (k - n/2): the central n^3 block of the swept
// lattice, the fixed grid of the rotated-object search
__global__ void k_swept_canvas(const uint8_t* __restrict__ Sw, int m, int n, float* __restrict__ S) {
    const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t n3 = (size_t)n * n * n;
    if (id >= n3) return;
    const int o = (m - n) / 2;
    const int kx = (int)(id % n), ky = (int)((id / n) % n), kz = (int)(id / ((size_t)n * n));
    S[id] = Sw[((size_t)(kz + o) * m + (ky + o)) * m + (kx + o)] ? 1.0f : 0.0f;
}

// finite vertices and poses, face indices in range, pose quaternions near unit
__global__ void k_validate(const float* __restrict__ V, int nv, const int32_t* __restrict__ F, int nf,
                           const float* __restrict__ poses, int np, int* __restrict__ err) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nv)
        for (int a = 0; a < 3; ++a)
            if (!isfinite(V[3 * i + a])) atomicOr(err, REGK_ERR_NONFINITE);
    if (i < nf)
        for (int a = 0; a < 3; ++a)
            if (F[3 * i + a] < 0 || F[3 * i + a] >= nv) atomicOr(err, REGK_ERR_FACE);
    if (i < np) {
        double s = 0;
        for (int a = 0; a < 7; ++a) {
            if (!isfinite(poses[7 * i + a])) atomicOr(err, REGK_ERR_NONFINITE);
            if (a < 4) s += (double)poses[7 * i + a] * poses[7 * i + a];
        }
        const double nq = sqrt(s);
        if (!(nq >= 1.0 - 1e-3 && nq <= 1.0 + 1e-3)) atomicOr(err, REGK_ERR_QUAT);
    }
}

// ------------------------------------------------------ split plane passes
//
// For canvases whose plane does not fit the LDS of one workgroup (above 180^3;
// also available at smaller edges, reg_params.split_plane), passes 1 and 3
// each become a row pass and a column pass that meet in an HBM plane buffer
// X (per rotation n planes of n rows of n/2 complex; slot 0 of a row holds
// X0 + i X_{n/2} as in the fused passes):
//   k_split_rows_fwd   per (rotation, plane, block of RB rows): the rows of
//                      S_r (or of a real grid), their x sums of the exact low
//                      block, the real-to-complex x FFT -> X
//   k_split_cols_fwd   per (rotation, plane, tile of T columns): the y FFT of
//                      the tile's columns -> the tiled spectrum; the tile of
//                      column 0 splits X0 and X_{n/2}
//   k_split_low_y      per (rotation, plane): the plane's low block along y
//   k_split_cols_inv   per (rotation, plane, tile): inverse y FFT -> X
//   k_split_rows_inv   per (rotation, plane, block of RB rows): complex-to-
//                      real x FFT, the exact low field, the block's peak keys
// The z pass, the low-block combine and the candidate selection are the fused
// path's (one record of keys per row block instead of per plane).  A rotation
// moves 8 H8 through HBM instead of 4 H8: each split pass writes and reads
// the plane buffer once more.  Given the swept lattice's reach
// (k_lattice_reach), the forward row pass writes row blocks beyond it as
// zeros unsampled, and the forward column pass does the same for planes.
template <int N> struct Split : Dims<N> {
    using D = Dims<N>;
    using D::N2;
    using D::M;
    using D::P;
    using D::T;
    using D::NT2;
    // rows per row-pass workgroup: above 180 at most 16, which keeps a row
    // workgroup's LDS low enough for three (forward) or more (inverse) per CU
    // (at 360^3: 15 rows against 30 gave 1.2x the rotations/s)
    static constexpr int RB = largest_divisor_le(N, N > 180 ? 16 : 32);
    static constexpr int NB = N / RB;  // row blocks per plane
    // threads of a row-pass workgroup: every column pair busy, two rows at a time
    static constexpr int RT = 2 * ((N2 + 63) / 64) * 64 < 128 ? 128 : 2 * ((N2 + 63) / 64) * 64;
    // threads of a column-pass workgroup: 512 above 180, where the T columns'
    // transforms are long enough to keep them busy (at 360^3 1.06x against 256)
    static constexpr int CT = N > 180 ? 512 : 256;
    static constexpr size_t XH = (size_t)N * N * N2;      // complex of X per rotation
    static_assert(RT <= 512 && N2 <= RT && N2 / 2 + 1 <= RT, "row pass layout");
};

// SRC 0: the rotated swept grid from its corner masks; SRC 1: rows of a real
// grid (the object grid O, no rotation)
template <int N, int SRC>
__global__ __launch_bounds__(Split<N>::RT) void k_split_rows_fwd(const uint8_t* __restrict__ cmask, int m, int mb,
                                                             const double* __restrict__ rots,
                                                             const float* __restrict__ grid,
                                                             const float2* __restrict__ twg,
                                                             const double2* __restrict__ tw64,
                                                             float2* __restrict__ xb, double2* __restrict__ lowrow,
                                                             const unsigned long long* __restrict__ reach4) {
    using C = Split<N>;
    constexpr int NT = C::RT, RB = C::RB;
    __shared__ float2 rows[RB * C::P];
    __shared__ float2 tw[N];
    __shared__ double2 tws[N];
    constexpr int RBB = RB * NLX * (int)sizeof(double2), LB = TRI_LUT * (int)sizeof(float4);
    __shared__ __align__(16) unsigned char scratch_lds[SRC == 0 ? (RBB > LB ? RBB : LB) : RBB];
    __shared__ uint32_t bax[SRC == 0 ? C::M : 1], bay[SRC == 0 ? C::M : 1], baz[SRC == 0 ? C::M : 1];
    double2* rbuf = reinterpret_cast<double2*>(scratch_lds);
    float4* lut = reinterpret_cast<float4*>(scratch_lds);
    const int blk = blockIdx.x % C::NB, pl = blockIdx.x / C::NB;  // pl = rot * N + z
    const int rot = pl / N, z = pl % N, y0 = blk * RB;
    if (SRC == 0 && reach4) {
        // every row of the block beyond the swept lattice's reach: zero rows
        // and zero low-block sums, without sampling or transforming them
        const int yc = N / 2 < y0 ? y0 : N / 2 > y0 + RB - 1 ? y0 + RB - 1 : N / 2;
        const double dy = yc - N / 2, dz = z - N / 2;
        if (dy * dy + dz * dz > canvas_reach2(reach4)) {
            float2* dst = xb + ((size_t)pl * N + y0) * C::N2;
            for (int e = threadIdx.x; e < RB * C::N2; e += NT) dst[e] = make_float2(0.0f, 0.0f);
            double2* lr = lowrow + ((size_t)pl * N + y0) * NLX;
            for (int e = threadIdx.x; e < RB * NLX; e += NT) lr[e] = make_double2(0.0, 0.0);
            return;
        }
    }
    for (int i = threadIdx.x; i < N; i += NT) {
        tw[i] = twg[i];
        tws[i] = tw64[i];
    }
    if constexpr (SRC == 0) {
        RotSampler rs;
        rs.load(rots + rot * 9, m, N);
        build_trilinear_lut<NT>(lut);
        build_brick_tables<NT>(bax, bay, baz, C::M, mb);
        __syncthreads();
        generate_plane<N, NT, RB>(rows, lut, bax, bay, baz, rs, cmask, z, y0);
    } else {
        for (int e = threadIdx.x; e < RB * C::N2; e += NT) {
            const int yl = e / C::N2, j = e % C::N2;
            const float* row = grid + ((size_t)z * N + y0 + yl) * N;
            rows[yl * C::P + j] = make_float2(row[2 * j], row[2 * j + 1]);
        }
    }
    __syncthreads();
    low_rows_x<N, NT, RB>(rows, tws, rbuf);
    fft_lds<C::N2, false, RB, NT, true, N>(rows, 1, C::P, tw);
    r2c_post<N, NT, RB>(rows, tw);
    float2* dst = xb + ((size_t)pl * N + y0) * C::N2;
    for (int e = threadIdx.x; e < RB * C::N2; e += NT) dst[e] = rows[(e / C::N2) * C::P + e % C::N2];
    double2* lr = lowrow + ((size_t)pl * N + y0) * NLX;
    for (int e = threadIdx.x; e < RB * NLX; e += NT) lr[e] = rbuf[low_slot(e / NLX, e % NLX)];
}

template <int N>
__global__ __launch_bounds__(Split<N>::CT) void k_split_cols_fwd(const float2* __restrict__ xb,
                                                             const float2* __restrict__ twg,
                                                             float2* __restrict__ spec,
                                                             const unsigned long long* __restrict__ reach4) {
    using C = Split<N>;
    constexpr int NT = C::CT, TT = C::T;
    __shared__ float2 buf[N * TT];  // [y][c]
    __shared__ float2 tw[N];
    __shared__ float2 nyqb[N];
    const int t = blockIdx.x % C::NT2, pl = blockIdx.x / C::NT2;
    const int rot = pl / N, z = pl % N;
    if (reach4) {
        // a plane beyond the swept lattice's reach: its X rows are zero, so is
        // its spectrum tile (and, for the tile of column 0, its Nyquist column)
        const double dz = z - N / 2;
        if (dz * dz > canvas_reach2(reach4)) {
            float2* spec_rot = spec + (size_t)rot * C::H;
            for (int e = threadIdx.x; e < N * TT; e += NT) {
                const int ky = e / TT, c = e % TT;
                spec_rot[((size_t)(ky * C::NT2 + t) * N + z) * C::T + c] = make_float2(0.0f, 0.0f);
            }
            if (t == 0) {
                float2* nyq = spec_rot + (size_t)N * C::N2 * N;
                for (int ky = threadIdx.x; ky < N; ky += NT)
                    nyq[((size_t)(ky / C::T) * N + z) * C::T + (ky % C::T)] = make_float2(0.0f, 0.0f);
            }
            return;
        }
    }
    for (int i = threadIdx.x; i < N; i += NT) tw[i] = twg[i];
    const float2* src = xb + (size_t)pl * N * C::N2 + t * TT;
    for (int e = threadIdx.x; e < N * TT; e += NT) buf[e] = src[(size_t)(e / TT) * C::N2 + e % TT];
    __syncthreads();
    fft_lds<N, false, TT, NT, true, N>(buf, TT, 1, tw);
    float2* spec_rot = spec + (size_t)rot * C::H;
    if (t == 0) {
        // column 0 holds Z = X0 + i X_{n/2} transformed along y (see unpack_nyquist)
        for (int k = threadIdx.x; k <= N / 2; k += NT) {
            const int kk = (N - k) % N;
            const float2 zk = buf[k * TT], zz = buf[kk * TT];
            const float2 a = make_float2(0.5f * (zk.x + zz.x), 0.5f * (zk.y - zz.y));
            const float2 b = make_float2(0.5f * (zk.y + zz.y), 0.5f * (zz.x - zk.x));
            buf[k * TT] = a;
            nyqb[k] = b;
            if (kk != k) {
                buf[kk * TT] = cconj(a);
                nyqb[kk] = cconj(b);
            }
        }
        __syncthreads();
        float2* nyq = spec_rot + (size_t)N * C::N2 * N;
        for (int ky = threadIdx.x; ky < N; ky += NT) nyq[((size_t)(ky / C::T) * N + z) * C::T + (ky % C::T)] = nyqb[ky];
    }
    for (int e = threadIdx.x; e < N * TT; e += NT) {
        const int ky = e / TT, c = e % TT;
        spec_rot[((size_t)(ky * C::NT2 + t) * N + z) * C::T + c] = buf[e];
    }
}

// per (rotation, plane): the y direction of the plane's exact low block from
// the row pass's x sums (kept out of the column pass, whose LDS it would
// double for one tile in NT2)
template <int N>
__global__ __launch_bounds__(256) void k_split_low_y(const double2* __restrict__ lowrow,
                                                     const double2* __restrict__ tw64, double2* __restrict__ lowT) {
    constexpr int NT = 256;
    __shared__ double2 tws[N];
    __shared__ double2 rbuf[N * NLX];
    const int pl = blockIdx.x;
    for (int i = threadIdx.x; i < N; i += NT) tws[i] = tw64[i];
    const double2* lr = lowrow + (size_t)pl * N * NLX;
    for (int e = threadIdx.x; e < N * NLX; e += NT) rbuf[low_slot(e / NLX, e % NLX)] = lr[e];
    __syncthreads();
    low_cols_y<N, NT>(rbuf, tws, lowT + (size_t)pl * NLOW2);
}

template <int N>
__global__ __launch_bounds__(Split<N>::CT) void k_split_cols_inv(const float2* __restrict__ spec,
                                                             const float2* __restrict__ twg, float2* __restrict__ xb) {
    using C = Split<N>;
    constexpr int NT = C::CT, TT = C::T;
    __shared__ float2 buf[N * TT];
    __shared__ float2 tw[N];
    const int t = blockIdx.x % C::NT2, pl = blockIdx.x / C::NT2;
    const int rot = pl / N, z = pl % N;
    for (int i = threadIdx.x; i < N; i += NT) tw[i] = twg[i];
    const float2* spec_rot = spec + (size_t)rot * C::H;
    for (int e = threadIdx.x; e < N * TT; e += NT) {
        const int ky = e / TT, c = e % TT;
        buf[e] = spec_rot[((size_t)(ky * C::NT2 + t) * N + z) * C::T + c];
    }
    __syncthreads();
    if (t == 0) {
        // column 0 (A) and the Nyquist column (B) become A + i B (see pack_nyquist)
        const float2* nyq = spec_rot + (size_t)N * C::N2 * N;
        for (int ky = threadIdx.x; ky < N; ky += NT) {
            const float2 a = buf[ky * TT], b = nyq[((size_t)(ky / C::T) * N + z) * C::T + (ky % C::T)];
            buf[ky * TT] = make_float2(a.x - b.y, a.y + b.x);
        }
        __syncthreads();
    }
    fft_lds<N, true, TT, NT, true, N>(buf, TT, 1, tw);
    float2* dst = xb + (size_t)pl * N * C::N2 + t * TT;
    for (int e = threadIdx.x; e < N * TT; e += NT) dst[(size_t)(e / TT) * C::N2 + e % TT] = buf[e];
}

template <int N>
__global__ __launch_bounds__(Split<N>::RT) void k_split_rows_inv(const float2* __restrict__ xb,
                                                             const float2* __restrict__ twg,
                                                             const double2* __restrict__ tw64,
                                                             const double2* __restrict__ Plow,
                                                             unsigned long long* __restrict__ ptop,
                                                             double* __restrict__ pssq, float* __restrict__ corr_out) {
    using C = Split<N>;
    constexpr int NT = C::RT, RB = C::RB, NW = NT / 64;
    __shared__ float2 rows[RB * C::P];
    __shared__ float2 tw[N];
    __shared__ double2 tws[N];
    __shared__ double2 btab[RB * NLX];
    __shared__ double2 az[NLOW2];
    __shared__ unsigned long long wtop[NW][KTOP + 1];
    __shared__ double wss[NW];
    __shared__ double wsec[NW];
    static_assert(NLOW2 <= NT, "one low-block row per thread");
    const int blk = blockIdx.x % C::NB, pl = blockIdx.x / C::NB;
    const int rot = pl / N, z = pl % N, y0 = blk * RB;
    const int tid = threadIdx.x;
    double2 pz[NLY];
    if (tid < NLOW2) {
        const double2* Pr = Plow + (size_t)rot * NLOW3 + tid * NLY;
#pragma unroll
        for (int kzi = 0; kzi < NLY; ++kzi) pz[kzi] = Pr[kzi];
    }
    for (int i = tid; i < N; i += NT) {
        tw[i] = twg[i];
        tws[i] = tw64[i];
    }
    const float2* src = xb + ((size_t)pl * N + y0) * C::N2;
    for (int e = tid; e < RB * C::N2; e += NT) rows[(e / C::N2) * C::P + e % C::N2] = src[e];
    __syncthreads();
    if (tid < NLOW2) {
        double2 acc = make_double2(0.0, 0.0);
#pragma unroll
        for (int kzi = 0; kzi < NLY; ++kzi) {
            const double2 t = dcmulc(pz[kzi], tws[mod_n((kzi - KLOW) * z, N)]);
            acc.x += t.x;
            acc.y += t.y;
        }
        az[tid] = acc;
    }
    __syncthreads();
    for (int t = tid; t < RB * NLX; t += NT) {
        const int y = y0 + t / NLX, kx = t % NLX;
        double2 acc = make_double2(0.0, 0.0);
#pragma unroll
        for (int kyi = 0; kyi < NLY; ++kyi) {
            const double2 v = dcmulc(az[kx * NLY + kyi], tws[mod_n((kyi - KLOW) * y, N)]);
            acc.x += v.x;
            acc.y += v.y;
        }
        btab[t] = kx > 0 ? make_double2(2.0 * acc.x, 2.0 * acc.y) : acc;
    }
    c2r_pre<N, NT, RB>(rows, tw);
    fft_lds<C::N2, true, RB, NT, true, N>(rows, 1, C::P, tw);
    const size_t unit = (size_t)pl * C::NB + blk;
    scan_rows<N, NT, RB>(rows, btab, tws, z, y0, wtop, wss, wsec, ptop + unit * KREC, pssq + unit, corr_out);
}

// ------------------------------------------------------------- launchers

// Schedule variants of the search kernels, chosen per canvas edge by the
// autotuner.  Plane workgroups (passes 1 and 3): (threads, waves per SIMD asked
// of the compiler) = (256, 1), (256, 2), (512, 4), (1024, 4); edges up to 80
// take the first three, edges up to 128 the last three, larger edges the last.
// z-pencil workgroups: 128, 256 or 512 threads per tile of T pencils.
template <int V> struct PlaneVariant;
template <> struct PlaneVariant<0> { static constexpr int NT = 256, WPE = 1; };
template <> struct PlaneVariant<1> { static constexpr int NT = 256, WPE = 2; };
template <> struct PlaneVariant<2> { static constexpr int NT = 512, WPE = 4; };
template <> struct PlaneVariant<3> { static constexpr int NT = 1024, WPE = 4; };
__host__ __device__ constexpr int z_threads_of(int v) { return v == 0 ? 128 : v == 1 ? 256 : 512; }

__host__ __device__ constexpr int default_plane_variant_of(int N) { return N > 128 ? 3 : N >= 96 ? 2 : 0; }

__host__ __device__ constexpr bool plane_variant_valid(int N, int v) {
    // above 128 a plane fills more than half of the LDS, so one workgroup per
    // CU holds the whole plane: only the widest workgroup is offered
    return v >= 0 && v < PLANE_VARIANTS && (N <= 80 ? v <= 2 : N <= 128 ? v >= 1 : v == 3);
}
template <int N>
constexpr bool z_variant_valid(int v) {
    return v >= 0 && v < Z_VARIANTS && (v == 1 || z_threads_of(v) <= N * Dims<N>::T);
}

template <int N, int V>
static void launch_plane(int pass, const SearchBatchArgs& a) {
    if constexpr (plane_variant_valid(N, V)) {
        constexpr int NT = PlaneVariant<V>::NT, WPE = PlaneVariant<V>::WPE;
        if (pass == 0 && a.crec) {
            // the rotated-object search compiles pass 1 for the default workgroup only
            if constexpr (V == default_plane_variant_of(N))
                hipLaunchKernelGGL((k_rotvox_fwd_xy<N, NT, WPE, true>), dim3(a.count * N), dim3(NT), 0, a.stream, a.cmask,
                                   a.m, a.mp / 4, a.rots, a.count, a.tw, a.tw64, a.spec, a.lowT, a.crec, a.cval, nullptr);
        } else if (pass == 0)
            hipLaunchKernelGGL((k_rotvox_fwd_xy<N, NT, WPE, false>), dim3(a.count * N), dim3(NT), 0, a.stream, a.cmask,
                               a.m, a.mp / 4, a.rots, a.count, a.tw, a.tw64, a.spec, a.lowT, nullptr, 0.0f, a.reach4);
        else
            hipLaunchKernelGGL((k_inv_xy_argmax<N, NT, WPE>), dim3(a.count * N), dim3(NT), 0, a.stream, a.spec, a.count,
                               a.tw, a.tw64, a.Plow, a.ptop, a.pssq, a.corr_out);
    }
}

template <int N, int V>
static void launch_z(const SearchBatchArgs& a) {
    if constexpr (z_variant_valid<N>(V)) {
        constexpr int ZT = z_threads_of(V);
        hipLaunchKernelGGL((k_zpass<N, 0, ZT>), dim3(a.count * Dims<N>::TILES), dim3(ZT), 0, a.stream, a.spec, a.W,
                           nullptr, a.tw, 1.0f);
    }
}

// pass 2 of either path: the low block along z, then the z pencils
template <int N>
static hipError_t launch_z_pass(const SearchBatchArgs& a) {
    if (!z_variant_valid<N>(a.zv)) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_low_combine<0, N>), dim3(a.count), dim3(256), 0, a.stream, a.lowT, a.tw64, a.Wlow, 1.0, a.Plow);
    switch (a.zv) {
        case 0: launch_z<N, 0>(a); break;
        case 1: launch_z<N, 1>(a); break;
        default: launch_z<N, 2>(a); break;
    }
    return hipGetLastError();
}

template <int N>
static hipError_t launch_split_pass(int pass, const SearchBatchArgs& a) {
    using C = Split<N>;
    // the row pass's sampler needs every rotated canvas point inside the
    // lattice (edge m) and brick tables of m entries; the split passes take
    // the corner masks of the swept grid only
    if (a.m != C::M || a.mp < a.m || a.mp % 4 || !a.xbuf || !a.lowrow || a.crec) return hipErrorInvalidValue;
    if (pass == 1) return launch_z_pass<N>(a);
    const unsigned rb = (unsigned)((size_t)a.count * N * C::NB), cb = (unsigned)((size_t)a.count * N * C::NT2);
    if (pass == 0) {
        hipLaunchKernelGGL((k_split_rows_fwd<N, 0>), dim3(rb), dim3(C::RT), 0, a.stream, a.cmask, a.m, a.mp / 4, a.rots,
                           nullptr, a.tw, a.tw64, a.xbuf, a.lowrow, a.reach4);
        hipLaunchKernelGGL(k_split_cols_fwd<N>, dim3(cb), dim3(C::CT), 0, a.stream, a.xbuf, a.tw, a.spec, a.reach4);
        hipLaunchKernelGGL(k_split_low_y<N>, dim3((unsigned)a.count * N), dim3(256), 0, a.stream, a.lowrow, a.tw64,
                           a.lowT);
    } else {
        hipLaunchKernelGGL(k_split_cols_inv<N>, dim3(cb), dim3(C::CT), 0, a.stream, a.spec, a.tw, a.xbuf);
        hipLaunchKernelGGL(k_split_rows_inv<N>, dim3(rb), dim3(C::RT), 0, a.stream, a.xbuf, a.tw, a.tw64, a.Plow, a.ptop,
                           a.pssq, a.corr_out);
    }
    return hipGetLastError();
}

template <int N>
static hipError_t launch_object_spectrum_split(const float* O, float2* spec_tmp, float2* W, const float2* tw,
                                               const double2* tw64, double2* lowT_tmp, double2* Wlow, float2* xbuf,
                                               double2* lowrow, hipStream_t s) {
    using C = Split<N>;
    if (!xbuf || !lowrow) return hipErrorInvalidValue;
    const double scale = 1.0 / ((double)N * N * N);
    hipLaunchKernelGGL((k_split_rows_fwd<N, 1>), dim3(N * C::NB), dim3(C::RT), 0, s, nullptr, 0, 0, nullptr, O, tw, tw64,
                       xbuf, lowrow, nullptr);
    hipLaunchKernelGGL(k_split_cols_fwd<N>, dim3(N * C::NT2), dim3(C::CT), 0, s, xbuf, tw, spec_tmp, nullptr);
    hipLaunchKernelGGL(k_split_low_y<N>, dim3(N), dim3(256), 0, s, lowrow, tw64, lowT_tmp);
    hipLaunchKernelGGL((k_zpass<N, 1, 256>), dim3(C::TILES), dim3(256), 0, s, spec_tmp, nullptr, W, tw, (float)scale);
    hipLaunchKernelGGL((k_low_combine<1, N>), dim3(1), dim3(256), 0, s, lowT_tmp, tw64, nullptr, scale, Wlow);
    return hipGetLastError();
}

template <int N>
static hipError_t launch_search_pass(int pass, const SearchBatchArgs& a) {
    // the sample generator relies on every rotated canvas point lying inside
    // the lattice (edge m = 2 ceil((sqrt(3) n + 2) / 2)),
    // with a one-cell margin, and its brick-address tables hold m entries
    if (a.m != Canvas<N>::M || a.mp < a.m || a.mp % 4) return hipErrorInvalidValue;
    if (pass == 1) return launch_z_pass<N>(a);
    const int v = pass == 0 ? (a.crec ? default_plane_variant_of(N) : a.pv1) : a.pv3;
    if (!plane_variant_valid(N, v)) return hipErrorInvalidValue;
    switch (v) {
        case 0: launch_plane<N, 0>(pass, a); break;
        case 1: launch_plane<N, 1>(pass, a); break;
        case 2: launch_plane<N, 2>(pass, a); break;
        default: launch_plane<N, 3>(pass, a); break;
    }
    return hipGetLastError();
}

template <int N>
static hipError_t launch_object_spectrum(const float* O, float2* spec_tmp, float2* W, const float2* tw,
                                         const double2* tw64, double2* lowT_tmp, double2* Wlow, hipStream_t s) {
    using C = Canvas<N>;
    const double scale = 1.0 / ((double)N * N * N);
    hipLaunchKernelGGL(k_grid_fwd_xy<N>, dim3(N), dim3(C::NT), 0, s, O, tw, tw64, spec_tmp, lowT_tmp);
    hipLaunchKernelGGL((k_zpass<N, 1, 256>), dim3(C::TILES), dim3(256), 0, s, spec_tmp, nullptr, W, tw, (float)scale);
    hipLaunchKernelGGL((k_low_combine<1, N>), dim3(1), dim3(256), 0, s, lowT_tmp, tw64, nullptr, scale, Wlow);
    return hipGetLastError();
}

// edges of the fused plane passes, edges with split passes compiled, and
// the edges that only the split passes serve (planes above the LDS)
#define REGDOCK_FOR_EACH_N(X) X(16) X(32) X(48) X(60) X(64) X(80) X(96) X(120) X(128) X(160) X(180)
#define REGDOCK_FOR_EACH_SPLIT_N(X) X(64) X(128) X(192) X(256) X(360)
#define REGDOCK_FOR_EACH_SPLIT_ONLY_N(X) X(192) X(256) X(360)

bool canvas_supported(int n) { return fused_supported(n) || split_supported(n); }

bool fused_supported(int n) {
    switch (n) {
#define CASE(N) case N: return true;
        REGDOCK_FOR_EACH_N(CASE)
#undef CASE
        default: return false;
    }
}

bool split_supported(int n) {
    switch (n) {
#define CASE(N) case N: return true;
        REGDOCK_FOR_EACH_SPLIT_N(CASE)
#undef CASE
        default: return false;
    }
}

size_t spectrum_elems(int n) {
    switch (n) {
#define CASE(N) case N: return Dims<N>::H;
        REGDOCK_FOR_EACH_N(CASE)
        REGDOCK_FOR_EACH_SPLIT_ONLY_N(CASE)
#undef CASE
        default: return 0;
    }
}

int tile_width(int n) {
    switch (n) {
#define CASE(N) case N: return Dims<N>::T;
        REGDOCK_FOR_EACH_N(CASE)
        REGDOCK_FOR_EACH_SPLIT_ONLY_N(CASE)
#undef CASE
        default: return 0;
    }
}

int split_units(int n) {
    switch (n) {
#define CASE(N) case N: return N * Split<N>::NB;
        REGDOCK_FOR_EACH_SPLIT_N(CASE)
#undef CASE
        default: return 0;
    }
}

size_t split_plane_elems(int n) {
    switch (n) {
#define CASE(N) case N: return Split<N>::XH;
        REGDOCK_FOR_EACH_SPLIT_N(CASE)
#undef CASE
        default: return 0;
    }
}

bool plane_variant_ok(int n, int v) {
    switch (n) {
#define CASE(N) case N: return plane_variant_valid(N, v);
        REGDOCK_FOR_EACH_N(CASE)
#undef CASE
        default: return false;
    }
}

bool z_variant_ok(int n, int v) {
    switch (n) {
#define CASE(N) case N: return z_variant_valid<N>(v);
        REGDOCK_FOR_EACH_N(CASE)
        REGDOCK_FOR_EACH_SPLIT_ONLY_N(CASE)
#undef CASE
        default: return false;
    }
}

int default_plane_variant(int n) { return default_plane_variant_of(n); }
int default_z_variant(int) { return 1; }
int plane_variant_threads(int v) { return v == 0 || v == 1 ? 256 : v == 2 ? 512 : 1024; }
int z_variant_threads(int v) { return z_threads_of(v); }

hipError_t search_pass(int n, int pass, const SearchBatchArgs& a) {
    if (a.xbuf) {
        switch (n) {
#define CASE(N) case N: return launch_split_pass<N>(pass, a);
            REGDOCK_FOR_EACH_SPLIT_N(CASE)
#undef CASE
            default: return hipErrorInvalidValue;
        }
    }
    switch (n) {
#define CASE(N) case N: return launch_search_pass<N>(pass, a);
        REGDOCK_FOR_EACH_N(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t object_spectrum(int n, const float* O, float2* spec_tmp, float2* W, const float2* tw, const double2* tw64,
                           double2* lowT_tmp, double2* Wlow, hipStream_t s, float2* xbuf, double2* lowrow) {
    if (xbuf) {
        switch (n) {
#define CASE(N) \
    case N: return launch_object_spectrum_split<N>(O, spec_tmp, W, tw, tw64, lowT_tmp, Wlow, xbuf, lowrow, s);
            REGDOCK_FOR_EACH_SPLIT_N(CASE)
#undef CASE
            default: return hipErrorInvalidValue;
        }
    }
    switch (n) {
#define CASE(N) case N: return launch_object_spectrum<N>(O, spec_tmp, W, tw, tw64, lowT_tmp, Wlow, s);
        REGDOCK_FOR_EACH_N(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t setup_object_grid(const float* V, const int32_t* F, const uint8_t* touch, int nf, int n, double h,
                             const double* anchor, double tau_out1, double tau_in1, double rho, float* O, float* fo,
                             const ObjectScratch& w, hipStream_t s) {
    const size_t n3 = (size_t)n * n * n;
    const int W = (n + 31) / 32;
    const size_t nwords = (size_t)n * n * W;
    const size_t mx = n3 > nwords ? n3 : nwords;
    hipLaunchKernelGGL(k_obj_init, dim3((unsigned)((mx + 255) / 256)), dim3(256), 0, s, w.d2, w.dt2, n3, w.par, nwords);
    hipLaunchKernelGGL(k_obj_faces, dim3(nf), dim3(256), 0, s, V, F, touch, n, h, anchor, (double)tau_out1 + h, w.d2, w.dt2);
    hipLaunchKernelGGL(k_obj_parity, dim3(nf), dim3(64), 0, s, V, F, n, h, anchor, W, w.par);
    hipLaunchKernelGGL(k_obj_finalize, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, s, w.d2, w.dt2, w.par, W, n, tau_out1,
                       tau_in1, rho, O, fo);
    return hipGetLastError();
}

hipError_t setup_anchor(const float* V, int nv, double* anchor, hipStream_t s) {
    hipLaunchKernelGGL(k_anchor, dim3(1), dim3(256), 0, s, V, nv, anchor);
    return hipGetLastError();
}

hipError_t setup_swept(const float* poses, int np, double r, double L, int m, int mp, double h, const double* wc,
                       double* pose_tmp, uint8_t* Sw, uint8_t* cm, hipStream_t s) {
    hipLaunchKernelGGL(k_pose_prep, dim3((np + 255) / 256), dim3(256), 0, s, poses, np, pose_tmp);
    const size_t m3 = (size_t)m * m * m;
    hipLaunchKernelGGL(k_fill_u8, dim3((unsigned)((m3 + 255) / 256)), dim3(256), 0, s, Sw, m3, (uint8_t)0);
    hipLaunchKernelGGL(k_swept_pose, dim3(np), dim3(256), 0, s, pose_tmp, r, L, m, h, wc[0], wc[1], wc[2], Sw);
    const size_t mp3 = (size_t)mp * mp * mp;
    hipLaunchKernelGGL(k_cellmask, dim3((unsigned)((mp3 + 255) / 256)), dim3(256), 0, s, Sw, m, mp, cm);
    return hipGetLastError();
}

hipError_t setup_cellmask(const uint8_t* Sw, int m, int mp, uint8_t* cm, hipStream_t s) {
    const size_t mp3 = (size_t)mp * mp * mp;
    hipLaunchKernelGGL(k_cellmask, dim3((unsigned)((mp3 + 255) / 256)), dim3(256), 0, s, Sw, m, mp, cm);
    return hipGetLastError();
}

hipError_t swept_reach(const uint8_t* Sw, int m, unsigned long long* reach4, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u8, dim3(1), dim3(256), 0, s, reinterpret_cast<uint8_t*>(reach4), sizeof(*reach4),
                       (uint8_t)0);
    hipLaunchKernelGGL(k_lattice_reach, dim3((unsigned)m * (unsigned)((m + 15) / 16)), dim3(256), 0, s, Sw, m, reach4);
    return hipGetLastError();
}

hipError_t setup_rotations(const float* so3, int M, double* rots, int* err, hipStream_t s, int transpose) {
    hipLaunchKernelGGL(k_rot_prep, dim3((M + 255) / 256), dim3(256), 0, s, so3, M, transpose, rots, err);
    return hipGetLastError();
}

hipError_t setup_object_cells(const float* G, int m, int mp, float cval, uint8_t* cls, float4* rec, hipStream_t s) {
    const size_t mp3 = (size_t)mp * mp * mp;
    hipLaunchKernelGGL(k_objcells, dim3((unsigned)((mp3 + 255) / 256)), dim3(256), 0, s, G, m, mp, cval, cls, rec);
    return hipGetLastError();
}

hipError_t swept_canvas(const uint8_t* Sw, int m, int n, float* S, hipStream_t s) {
    const size_t n3 = (size_t)n * n * n;
    hipLaunchKernelGGL(k_swept_canvas, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, s, Sw, m, n, S);
    return hipGetLastError();
}

hipError_t validate_inputs(const float* V, int nv, const int32_t* F, int nf, const float* poses, int np, int* err,
                           hipStream_t s) {
    const int mx = nv > nf ? (nv > np ? nv : np) : (nf > np ? nf : np);
    hipLaunchKernelGGL(k_validate, dim3((mx + 255) / 256), dim3(256), 0, s, V, nv, F, nf, poses, np, err);
    return hipGetLastError();
}

int rescore_slices(int n) {
    const size_t n3 = (size_t)n * n * n;
    return (int)((n3 + 65535) / 65536);
}

hipError_t select_batch(int n, const SearchBatchArgs& a, int base, const PeakArrays& pk) {
    const double eps_per_rms = REGK_EPS_SCALE * std::ldexp(1.0, -24) * std::log2((double)n * n * n);
    hipLaunchKernelGGL(k_select, dim3(a.count), dim3(256), 0, a.stream, a.ptop, a.pssq, n, a.units > 0 ? a.units : n, eps_per_rms,
                       base, pk.cand_idx,
                       pk.cand_n, pk.window, pk.ovf, pk.best_val, pk.best_flat, pk.stats);
    return hipGetLastError();
}

hipError_t finish_call(int n, int first, int count, int always, const PeakArrays& pk, const RescoreInputs& ri,
                       const float* quats, double h, const double* anchor, const double* wc, float* out_score,
                       int32_t* out_shift, double* out_pose, hipStream_t s) {
    const int rotobj = ri.crec != nullptr;
    hipLaunchKernelGGL(k_finalize, dim3((count + 127) / 128), dim3(128), 0, s, pk.best_val + first, pk.best_flat + first,
                       count, quats, n, h, anchor, wc[0], wc[1], wc[2], rotobj, out_score, out_shift, out_pose);
    hipLaunchKernelGGL(k_certify, dim3(1), dim3(1024), 0, s, pk.best_val + first, pk.window + first, pk.ovf + first, count,
                       always, pk.need_list, pk.need_count, pk.stats);
    const int nslice = rescore_slices(n);
    hipLaunchKernelGGL(k_rescore, dim3(2048), dim3(256), 0, s, ri.nz_idx, ri.nz_val, ri.nz_count, n, nslice, ri.cmask, ri.m,
                       ri.mp / 4, ri.crec, ri.cval, ri.rots + 9 * (size_t)first, pk.need_list, pk.need_count,
                       pk.cand_idx + (size_t)first * CMAX, pk.cand_n + first, pk.cand_part);
    hipLaunchKernelGGL(k_apply, dim3(16), dim3(256), 0, s, pk.need_list, pk.need_count, pk.cand_idx + (size_t)first * CMAX,
                       pk.cand_n + first, pk.cand_part, nslice, quats, n, h, anchor, wc[0], wc[1], wc[2], rotobj, out_score,
                       out_shift, out_pose);
    return hipGetLastError();
}

hipError_t build_nonzero_list(const float* O, int n, int* bcount, int* boff, uint32_t* idx, float* val, int* nnz,
                              hipStream_t s) {
    const size_t n3 = (size_t)n * n * n;
    const int nb = (int)((n3 + 255) / 256);
    hipLaunchKernelGGL(k_nz_count, dim3(nb), dim3(256), 0, s, O, n3, bcount);
    hipLaunchKernelGGL(k_nz_scan, dim3(1), dim3(1024), 0, s, bcount, nb, boff, nnz);
    hipLaunchKernelGGL(k_nz_write, dim3(nb), dim3(256), 0, s, O, n3, n, boff, idx, val);
    return hipGetLastError();
}

}  // namespace regdock

namespace regdock {

// K best of a score vector: K rounds of a block-wide maximum over packed keys
// (orderable score bits, ~index), each round taking the largest key below the
// previous one.  Keys are unique, so the order is score descending, index
// ascending.  Slots beyond count receive -1.
__global__ __launch_bounds__(1024) void k_topk(const float* __restrict__ scores, int count, int K, int32_t* __restrict__ out) {
    __shared__ unsigned long long wb[16];
    __shared__ unsigned long long sel;
    unsigned long long last = ~0ull;
    for (int r = 0; r < K; ++r) {
        unsigned long long best = 0ull;
        for (int i = threadIdx.x; i < count; i += 1024) {
            const unsigned long long key = ((unsigned long long)ordered_bits(scores[i]) << 32) | (0xffffffffu - (uint32_t)i);
            if (key < last && key > best) best = key;
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const unsigned long long o = __shfl_xor(best, off, 64);
            best = o > best ? o : best;
        }
        if ((threadIdx.x & 63) == 0) wb[threadIdx.x >> 6] = best;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long b = wb[0];
            for (int w = 1; w < 16; ++w) b = wb[w] > b ? wb[w] : b;
            sel = b;
            out[r] = (r < count) ? (int32_t)(0xffffffffu - (uint32_t)(b & 0xffffffffu)) : -1;
        }
        __syncthreads();
        last = sel;
    }
}

hipError_t top_k(const float* scores, int count, int K, int32_t* out, hipStream_t s) {
    hipLaunchKernelGGL(k_topk, dim3(1), dim3(1024), 0, s, scores, count, K, out);
    return hipGetLastError();
}

}  // namespace regdock

