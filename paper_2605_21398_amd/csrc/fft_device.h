// Mixed-radix (2, 3, 4, 5, 8, 16 and the composites 6, 9, 10, 12, 15) complex
// FFTs on LDS-resident batches, for gfx950.
//
// The docking score of Sec. IV-B is a circular cross-correlation evaluated
// through 3D FFTs (Eq. xcorr and the FFT identity that follows it).  This
// header holds the building blocks: radix codelets in registers and a
// Stockham autosort pass over a batch of transforms that live in LDS.
//
// A pass reads every butterfly input of the thread into registers, applies the
// twiddles and the radix-R DFT, waits at a barrier and writes the outputs back
// to the same LDS buffer, so a transform needs no second buffer.  All sizes are
// compile-time constants; the per-thread butterfly loop is fully unrolled.
//
// Twiddles come from one table per canvas edge N: w[t] = exp(-2 pi i t / N),
// t in [0, N), computed in double on the host and rounded to float.  A length
// L that divides N reads w[t * (N / L)].
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace regdock {

__host__ __device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__host__ __device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__host__ __device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__host__ __device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__host__ __device__ __forceinline__ float2 mul_mi(float2 a) {
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// ---------------------------------------------------------------- codelets
// DFT_R: X[k] = sum_r x[r] exp(-+2 pi i r k / R), sign - forward, + inverse.

template <int R, bool INV> struct Dft;

template <bool INV> struct Dft<2, INV> {
    __host__ __device__ __forceinline__ static void run(float2* v) {
        float2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <bool INV> struct Dft<3, INV> {
    __host__ __device__ __forceinline__ static void run(float2* v) {
        const float s3 = 0.866025403784438647f;  // sin(2 pi / 3)
        float2 t1 = cadd(v[1], v[2]);
        float2 t2 = csub(v[1], v[2]);
        float2 x0 = v[0];
        v[0] = cadd(x0, t1);
        float2 m1 = make_float2(x0.x - 0.5f * t1.x, x0.y - 0.5f * t1.y);
        float2 m2 = mul_mi<INV>(cscale(t2, s3));
        v[1] = cadd(m1, m2);
        v[2] = csub(m1, m2);
    }
};

template <bool INV> struct Dft<4, INV> {
    __host__ __device__ __forceinline__ static void run(float2* v) {
        float2 t0 = cadd(v[0], v[2]);
        float2 t1 = csub(v[0], v[2]);
        float2 t2 = cadd(v[1], v[3]);
        float2 t3 = mul_mi<INV>(csub(v[1], v[3]));
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, t3);
        v[3] = csub(t1, t3);
    }
};

template <bool INV> struct Dft<5, INV> {
    __host__ __device__ __forceinline__ static void run(float2* v) {
        const float c1 = 0.309016994374947424f;   // cos(2 pi / 5)
        const float c2 = -0.809016994374947424f;  // cos(4 pi / 5)
        const float s1 = 0.951056516295153572f;   // sin(2 pi / 5)
        const float s2 = 0.587785252292473129f;   // sin(4 pi / 5)
        float2 x0 = v[0];
        float2 t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
        float2 t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
        float2 a1 = make_float2(x0.x + c1 * t1.x + c2 * t2.x, x0.y + c1 * t1.y + c2 * t2.y);
        float2 a2 = make_float2(x0.x + c2 * t1.x + c1 * t2.x, x0.y + c2 * t1.y + c1 * t2.y);
        float2 b1 = make_float2(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y);
        float2 b2 = make_float2(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y);
        float2 ib1 = mul_mi<INV>(b1), ib2 = mul_mi<INV>(b2);
        v[0] = cadd(x0, cadd(t1, t2));
        v[1] = cadd(a1, ib1);
        v[4] = csub(a1, ib1);
        v[2] = cadd(a2, ib2);
        v[3] = csub(a2, ib2);
    }
};

template <bool INV> struct Dft<8, INV> {
    // radix-2 butterflies on (x_j, x_{j+4}), twiddle W8^j on the differences,
    // then a radix-4 DFT on each half: sums give even outputs, differences odd.
    __host__ __device__ __forceinline__ static void run(float2* v) {
        const float h = 0.707106781186547524f;
        float2 a[4], b[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            a[j] = cadd(v[j], v[j + 4]);
            b[j] = csub(v[j], v[j + 4]);
        }
        // W8^1 = h (1 -+ i), W8^2 = -+ i, W8^3 = h (-1 -+ i)
        b[1] = INV ? make_float2(h * (b[1].x - b[1].y), h * (b[1].x + b[1].y))
                   : make_float2(h * (b[1].x + b[1].y), h * (b[1].y - b[1].x));
        b[2] = mul_mi<INV>(b[2]);
        b[3] = INV ? make_float2(-h * (b[3].x + b[3].y), h * (b[3].x - b[3].y))
                   : make_float2(h * (b[3].y - b[3].x), -h * (b[3].x + b[3].y));
        Dft<4, INV>::run(a);
        Dft<4, INV>::run(b);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[2 * k] = a[k];
            v[2 * k + 1] = b[k];
        }
    }
};

template <bool INV> struct Dft<16, INV> {
    // 4 x 4: radix-4 DFTs over the residues n2 = j mod 4 (inputs j = 4 n1 + n2),
    // twiddles W16^(n2 k1), radix-4 DFTs over n2; output k = k1 + 4 k2
    __host__ __device__ __forceinline__ static void run(float2* v) {
        const float h = 0.707106781186547524f;   // cos(pi/4)
        const float c1 = 0.923879532511286756f;  // cos(pi/8)
        const float s1 = 0.382683432365089772f;  // sin(pi/8)
        float2 a[4][4];
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
            for (int n1 = 0; n1 < 4; ++n1) a[n2][n1] = v[4 * n1 + n2];
            Dft<4, INV>::run(a[n2]);
        }
        // forward W16^m = exp(-2 pi i m / 16); the inverse conjugates
        auto tw = [](float2 x, float wr, float wi) {
            const float si = INV ? -wi : wi;
            return make_float2(x.x * wr - x.y * si, x.x * si + x.y * wr);
        };
        a[1][1] = tw(a[1][1], c1, -s1);   // m = 1
        a[1][2] = INV ? make_float2(h * (a[1][2].x - a[1][2].y), h * (a[1][2].x + a[1][2].y))
                      : make_float2(h * (a[1][2].x + a[1][2].y), h * (a[1][2].y - a[1][2].x));  // m = 2
        a[1][3] = tw(a[1][3], s1, -c1);   // m = 3
        a[2][1] = INV ? make_float2(h * (a[2][1].x - a[2][1].y), h * (a[2][1].x + a[2][1].y))
                      : make_float2(h * (a[2][1].x + a[2][1].y), h * (a[2][1].y - a[2][1].x));  // m = 2
        a[2][2] = mul_mi<INV>(a[2][2]);    // m = 4
        a[2][3] = INV ? make_float2(-h * (a[2][3].x + a[2][3].y), h * (a[2][3].x - a[2][3].y))
                      : make_float2(h * (a[2][3].y - a[2][3].x), -h * (a[2][3].x + a[2][3].y));  // m = 6
        a[3][1] = tw(a[3][1], s1, -c1);   // m = 3
        a[3][2] = INV ? make_float2(-h * (a[3][2].x + a[3][2].y), h * (a[3][2].x - a[3][2].y))
                      : make_float2(h * (a[3][2].y - a[3][2].x), -h * (a[3][2].x + a[3][2].y));  // m = 6
        a[3][3] = tw(a[3][3], -c1, s1);   // m = 9
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            float2 b[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
            Dft<4, INV>::run(b);
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = b[k2];
        }
    }
};

// Composite codelets DFT_{PQ} from DFT_P and DFT_Q: inputs j = Q n1 + n2,
// DFT_P over n1 for each n2, twiddles W_PQ^(n2 k1), DFT_Q over n2 for each k1;
// output k = k1 + P k2.  The twiddles are compile-time constants (cosine and
// sine by their Taylor series in double, rounded to float); multiples of a
// quarter turn become sign changes and swaps.
struct CTw {
    double c, s;
};
__host__ __device__ constexpr CTw ct_twiddle(int m, int R) {
    // cos and sin of 2 pi m / R, the angle reduced to [-pi, pi]
    int mm = m % R;
    if (2 * mm > R) mm -= R;
    const double x = 2.0 * 3.14159265358979323846 * (double)mm / (double)R;
    double c = 1.0, s = x, tc = 1.0, ts = x;
    for (int k = 1; k < 30; ++k) {
        tc *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
        ts *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
        c += tc;
        s += ts;
    }
    return CTw{c, s};
}

// x * W_R^M, W_R = exp(-+2 pi i / R) (forward, inverse)
template <int R, int M, bool INV>
__host__ __device__ __forceinline__ float2 ct_rot(float2 x) {
    constexpr int m = M % R;
    if constexpr (m == 0) {
        return x;
    } else if constexpr (4 * m == R) {
        return mul_mi<INV>(x);
    } else if constexpr (2 * m == R) {
        return make_float2(-x.x, -x.y);
    } else if constexpr (4 * m == 3 * R) {
        return mul_mi<!INV>(x);
    } else {
        constexpr CTw t = ct_twiddle(m, R);
        constexpr float c = (float)t.c, sn = INV ? (float)t.s : -(float)t.s;
        return make_float2(x.x * c - x.y * sn, x.x * sn + x.y * c);
    }
}

template <int P, int Q, bool INV>
struct DftPQ {
    template <int I>
    __host__ __device__ __forceinline__ static void twiddle_all(float2 (&a)[Q][P]) {
        if constexpr (I < P * Q) {
            constexpr int n2 = I / P, k1 = I % P;
            a[n2][k1] = ct_rot<P * Q, n2 * k1, INV>(a[n2][k1]);
            twiddle_all<I + 1>(a);
        }
    }
    __host__ __device__ __forceinline__ static void run(float2* v) {
        float2 a[Q][P];
#pragma unroll
        for (int n2 = 0; n2 < Q; ++n2) {
#pragma unroll
            for (int n1 = 0; n1 < P; ++n1) a[n2][n1] = v[Q * n1 + n2];
            Dft<P, INV>::run(a[n2]);
        }
        twiddle_all<0>(a);
#pragma unroll
        for (int k1 = 0; k1 < P; ++k1) {
            float2 b[Q];
#pragma unroll
            for (int n2 = 0; n2 < Q; ++n2) b[n2] = a[n2][k1];
            Dft<Q, INV>::run(b);
#pragma unroll
            for (int k2 = 0; k2 < Q; ++k2) v[k1 + P * k2] = b[k2];
        }
    }
};

template <bool INV> struct Dft<6, INV> : DftPQ<3, 2, INV> {};
template <bool INV> struct Dft<9, INV> : DftPQ<3, 3, INV> {};
template <bool INV> struct Dft<10, INV> : DftPQ<5, 2, INV> {};
template <bool INV> struct Dft<12, INV> : DftPQ<4, 3, INV> {};
template <bool INV> struct Dft<15, INV> : DftPQ<5, 3, INV> {};

// ------------------------------------------------------- factorisation plan

__host__ __device__ constexpr int pow2_exponent(int L) {
    int e = 0;
    while (L > 1 && L % 2 == 0) {
        L /= 2;
        ++e;
    }
    return e;
}

__host__ __device__ constexpr int greedy_radix(int L, int p) {
    // greedy: 8s, then a 4, then a 2, then 5s, then 3s; when the power of two
    // in L is 2^(3k + 1) (k >= 1) one radix-16 stage replaces an 8 and a 2,
    // saving a pass
    bool use16 = pow2_exponent(L) >= 4 && pow2_exponent(L) % 3 == 1;
    int i = 0;
    while (L > 1) {
        int r = (use16 && L % 16 == 0) ? 16
              : (L % 8 == 0) ? 8 : (L % 4 == 0) ? 4 : (L % 2 == 0) ? 2 : (L % 5 == 0) ? 5 : (L % 3 == 0) ? 3 : 0;
        if (r == 0) return 0;
        if (r == 16) use16 = false;
        if (i == p) return r;
        L /= r;
        ++i;
    }
    return 1;
}

__host__ __device__ constexpr int greedy_npass(int L) {
    int n = 0;
    while (greedy_radix(L, n) > 1) ++n;
    return n;
}

__host__ __device__ constexpr bool is_codelet(int r) {
    return r == 2 || r == 3 || r == 4 || r == 5 || r == 6 || r == 8 || r == 9 || r == 10 || r == 12 || r == 15 ||
           r == 16;
}

// first radix of a two-pass plan L = R1 R2 of codelets, the most balanced
// (largest min(R1, R2)), the larger R1 among equals; 0 if there is none
__host__ __device__ constexpr int two_pass_first(int L) {
    int best = 0, bmin = 0;
    for (int r1 = 16; r1 >= 2; --r1)
        if (is_codelet(r1) && L % r1 == 0 && is_codelet(L / r1)) {
            const int mn = r1 < L / r1 ? r1 : L / r1;
            if (mn > bmin) {
                bmin = mn;
                best = r1;
            }
        }
    return best;
}

// first two radices of a three-pass plan L = R1 R2 R3 of codelets, the most
// balanced (largest min(R1, R2, R3)), the larger R1, then R2, among equals;
// 0 if there is none.  which = 0 gives R1, 1 gives R2.
__host__ __device__ constexpr int three_pass_radix(int L, int which) {
    int b1 = 0, b2 = 0, bmin = 0;
    for (int r1 = 16; r1 >= 2; --r1) {
        if (!is_codelet(r1) || L % r1) continue;
        for (int r2 = 16; r2 >= 2; --r2) {
            if (!is_codelet(r2) || (L / r1) % r2 || !is_codelet(L / r1 / r2)) continue;
            const int r3 = L / r1 / r2;
            const int mn = r1 < r2 ? (r1 < r3 ? r1 : r3) : (r2 < r3 ? r2 : r3);
            if (mn > bmin) {
                bmin = mn;
                b1 = r1;
                b2 = r2;
            }
        }
    }
    return which == 0 ? b1 : b2;
}

// Radix of pass p of a length-L transform (1 past the last pass, 0 if L has
// another prime factor): the greedy plan where it takes at most two passes,
// else a two-pass plan through a composite codelet where one exists (60 =
// 10 x 6, 96 = 12 x 8, 120 = 12 x 10, 160 = 16 x 10, 180 = 15 x 12, 30 = 6 x 5,
// 90 = 10 x 9), else a three-pass plan of codelets where the greedy one
// takes more passes (360 = 10 x 6 x 6 against 8 x 5 x 3 x 3), else the
// greedy plan.
__host__ __device__ constexpr int fft_radix(int L, int p) {
    if (greedy_npass(L) <= 2) return greedy_radix(L, p);
    if (two_pass_first(L) != 0) {
        const int r1 = two_pass_first(L);
        return p == 0 ? r1 : p == 1 ? L / r1 : 1;
    }
    if (greedy_npass(L) > 3 && three_pass_radix(L, 0) != 0) {
        const int r1 = three_pass_radix(L, 0), r2 = three_pass_radix(L, 1);
        return p == 0 ? r1 : p == 1 ? r2 : p == 2 ? L / (r1 * r2) : 1;
    }
    return greedy_radix(L, p);
}

__host__ __device__ constexpr int fft_npass(int L) {
    int n = 0;
    while (fft_radix(L, n) > 1) ++n;
    return n;
}

__host__ __device__ constexpr bool fft_supported(int L) {
    int n = 0;
    while (L > 1) {
        int r = fft_radix(L, 0);
        if (r == 0) return false;
        L /= r;
        if (++n > 16) return false;
    }
    return true;
}

// ------------------------------------------------------------ Stockham pass
//
// Batch of NB transforms of length L in LDS: element e of transform b is at
// buf[b * BS + e * ES].  Pass p (radix R, span NS = product of earlier radices)
// maps butterfly j in [0, L/R):
//   v[r] = x[j + r L/R] * w_{NS R}^{(j mod NS) r}
//   v = DFT_R(v)
//   x[(j / NS) NS R + (j mod NS) + r NS] = v[r]
// BATCH_FAST selects which index varies fastest across consecutive threads:
// the batch (columns of a row-major plane) or the butterfly (rows).

template <int L, int R, int NS, bool INV, int NB, int NT, bool BATCH_FAST, int TWN>
__device__ __forceinline__ void stockham_pass(float2* buf, int ES, int BS, const float2* __restrict__ tw) {
    constexpr int NBF = L / R;
    constexpr int TOT = NB * NBF;
    constexpr int PER = (TOT + NT - 1) / NT;
    constexpr int TWSTEP = (TWN / L) * (L / (NS * R));  // table stride per (j mod NS) * r
    float2 v[PER][R];
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int b = tid + i * NT;
        if (PER * NT == TOT || b < TOT) {
            const int bat = BATCH_FAST ? (b % NB) : (b / NBF);
            const int j = BATCH_FAST ? (b / NB) : (b % NBF);
            const float2* src = buf + bat * BS;
            const int jm = j % NS;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float2 x = src[(j + r * NBF) * ES];
                if (NS > 1 && r > 0) {
                    const float2 w = tw[(jm * r * TWSTEP) % TWN];
                    x = INV ? cmulc(x, w) : cmul(x, w);
                }
                v[i][r] = x;
            }
            Dft<R, INV>::run(v[i]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int b = tid + i * NT;
        if (PER * NT == TOT || b < TOT) {
            const int bat = BATCH_FAST ? (b % NB) : (b / NBF);
            const int j = BATCH_FAST ? (b / NB) : (b % NBF);
            float2* dst = buf + bat * BS;
            const int jm = j % NS;
            const int base = (j / NS) * NS * R + jm;
#pragma unroll
            for (int r = 0; r < R; ++r) dst[(base + r * NS) * ES] = v[i][r];
        }
    }
    __syncthreads();
}

template <int L, bool INV, int NB, int NT, bool BATCH_FAST, int TWN, int P = 0, int NS = 1>
__device__ __forceinline__ void fft_lds(float2* buf, int ES, int BS, const float2* __restrict__ tw) {
    if constexpr (P < fft_npass(L)) {
        constexpr int R = fft_radix(L, P);
        stockham_pass<L, R, NS, INV, NB, NT, BATCH_FAST, TWN>(buf, ES, BS, tw);
        fft_lds<L, INV, NB, NT, BATCH_FAST, TWN, P + 1, NS * R>(buf, ES, BS, tw);
    }
}

}  // namespace regdock
