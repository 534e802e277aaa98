// Continuous SE(3) refinement (Sec. V) on the device.
//
// Every start (an initial object pose from the global search) is refined by a
// damped Gauss-Newton iteration on the twist xi = (v, w), one evaluation round
// per trial step for all unfinished starts at once:
//   k_ref_pose    FP64: R = exp(w^) R0, p = p0 + V(w) v + (I - exp(w^)) R0 a
//                 (Eq. se3-exp and the left updates), V(w), D = d(V v)/dw and
//                 the pivot c = p0 + V v + R0 a;
//   k_ref_query   FP32: per (start, probe pose) the smallest signed distance d,
//                 its witness x* and the probe normal n (Sec. V-B);
//   k_ref_reduce  FP64: J = -sum s(d) + lambda |xi|^2, grad J and the
//                 curvature sum max(0, -s'') g g^T + 2 lambda I, g the contact
//                 sensitivities (Sec. V-C), in a fixed summation order;
//   k_ref_step    FP64: accept or reject the trial, update the damping and
//                 solve (H + mu diag H + 1e-12 I) step = -grad by Cholesky.
#include "refine_kernels.h"

#include <cmath>

namespace {

constexpr float GOLD_TOL = 1e-5f;         // barycentric bracket width of the face minimisation
constexpr float RIDGE_TOL = 1e-4f;        // |q1 - q2| below which a witness is on the side/cap ridge
constexpr float EDGE_TOL = 1e-4f;         // barycentric distance below which a witness is on an edge
constexpr float INVPHI_F = 0.618033988749894848f;

// ------------------------------------------------------------ FP64 rotations

__device__ void quat_mat(double w, double x, double y, double z, double* R) {
    const double n = sqrt(w * w + x * x + y * y + z * z);
    w /= n; x /= n; y /= n; z /= n;
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z); R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z); R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y); R[7] = 2 * (y * z + w * x); R[8] = 1 - 2 * (x * x + y * y);
}

__device__ void mat3_mul(const double* A, const double* B, double* C) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

__device__ void mat3_vec(const double* A, const double* v, double* o) {
    for (int i = 0; i < 3; ++i) o[i] = A[3 * i] * v[0] + A[3 * i + 1] * v[1] + A[3 * i + 2] * v[2];
}

// I + c1 W + c2 W^2 with W = w^
__device__ void so3_poly(const double* w, double c1, double c2, double* M) {
    const double W[9] = {0, -w[2], w[1], w[2], 0, -w[0], -w[1], w[0], 0};
    double W2[9];
    mat3_mul(W, W, W2);
    for (int i = 0; i < 9; ++i) M[i] = (i % 4 == 0 ? 1.0 : 0.0) + c1 * W[i] + c2 * W2[i];
}

// Rodrigues' formula exp(w^)
__device__ void so3_exp(const double* w, double* M) {
    const double th = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    if (th < 1e-8) so3_poly(w, 1.0, 0.5, M);
    else so3_poly(w, sin(th) / th, (1 - cos(th)) / (th * th), M);
}

// left Jacobian V(w) = I + (1 - cos t)/t^2 W + (t - sin t)/t^3 W^2 (series below 1e-4)
__device__ void left_jac(const double* w, double* M) {
    const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    const double th = sqrt(th2);
    if (th < 1e-4) {
        so3_poly(w, 0.5 - th2 / 24.0, 1.0 / 6.0 - th2 / 120.0, M);
    } else {
        so3_poly(w, (1 - cos(th)) / th2, (th - sin(th)) / (th2 * th), M);
    }
}

__device__ double clampd(double x, double b) { return fmin(b, fmax(-b, x)); }

// ------------------------------------------------------------ FP32 probe SDF

// capped cylinder, tip disk at the origin, axis +z, length L (negative inside)
__device__ __forceinline__ float sdf_f(float x, float y, float z, float r, float L) {
    const float q1 = sqrtf(x * x + y * y) - r;
    const float q2 = fabsf(z - 0.5f * L) - 0.5f * L;
    const float in = fminf(fmaxf(q1, q2), 0.0f);
    const float a = fmaxf(q1, 0.0f), b = fmaxf(q2, 0.0f);
    return in + sqrtf(a * a + b * b);
}

struct Xf {  // body -> probe frame, u = A b + c
    float a[9], c[3];
    __device__ float3 apply(float bx, float by, float bz) const {
        return make_float3(a[0] * bx + a[1] * by + a[2] * bz + c[0], a[3] * bx + a[4] * by + a[5] * bz + c[1],
                           a[6] * bx + a[7] * by + a[8] * bz + c[2]);
    }
};

struct Tri {
    float3 p0, e1, e2;
    float r, L;
    __device__ float at(float s, float t) const {
        return sdf_f(p0.x + s * e1.x + t * e2.x, p0.y + s * e1.y + t * e2.y, p0.z + s * e1.z + t * e2.z, r, L);
    }
};

// min over t in [0, tmax] of f(s, t): golden section, then the bracket's ends
__device__ float inner_min(const Tri& T, float s, float tmax, float& t_out) {
    float a = 0.0f, b = tmax;
    float c = b - INVPHI_F * (b - a), d = a + INVPHI_F * (b - a);
    float fc = T.at(s, c), fd = T.at(s, d);
    while (b - a > GOLD_TOL) {
        if (fc <= fd) {
            b = d; d = c; fd = fc; c = b - INVPHI_F * (b - a); fc = T.at(s, c);
        } else {
            a = c; c = d; fc = fd; d = a + INVPHI_F * (b - a); fd = T.at(s, d);
        }
    }
    float tm = 0.5f * (a + b), fm = T.at(s, tm);
    const float f0 = T.at(s, 0.0f), f1 = T.at(s, tmax);
    if (f0 < fm) { fm = f0; tm = 0.0f; }
    if (f1 < fm) { fm = f1; tm = tmax; }
    t_out = tm;
    return fm;
}

// min of the probe SDF over the triangle p0 + s e1 + t e2 (s, t >= 0, s + t <= 1).
// f is convex, so is its partial minimum over t; nested golden sections.
__device__ float face_min(const Tri& T, float& s_out, float& t_out) {
    float a = 0.0f, b = 1.0f, tt;
    float c = b - INVPHI_F * (b - a), d = a + INVPHI_F * (b - a);
    float fc = inner_min(T, c, 1.0f - c, tt), fd = inner_min(T, d, 1.0f - d, tt);
    while (b - a > GOLD_TOL) {
        if (fc <= fd) {
            b = d; d = c; fd = fc; c = b - INVPHI_F * (b - a); fc = inner_min(T, c, 1.0f - c, tt);
        } else {
            a = c; c = d; fc = fd; d = a + INVPHI_F * (b - a); fd = inner_min(T, d, 1.0f - d, tt);
        }
    }
    float sm = 0.5f * (a + b), tm;
    float fm = inner_min(T, sm, 1.0f - sm, tm);
    float t0, t1;
    const float f0 = inner_min(T, 0.0f, 1.0f, t0), f1 = inner_min(T, 1.0f, 0.0f, t1);
    if (f0 < fm) { fm = f0; sm = 0.0f; tm = t0; }
    if (f1 < fm) { fm = f1; sm = 1.0f; tm = t1; }
    s_out = sm;
    t_out = tm;
    return fm;
}

__device__ float dot3(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// Gradient of the face minimum with respect to a motion of the face, at the
// witness u = p0 + s e1 + t e2: grad f_p where it is differentiable; on the
// inner ridge between the side wall (q1) and a cap (q2) the minimum is a
// min-max of the branches and the derivative is a grad q1 + (1 - a) grad q2
// with a in [0, 1] leaving no component along the directions the witness can
// move in (the face plane, or the edge it lies on).
__device__ float3 witness_gradient(float3 u, const Tri& T, float s, float t) {
    const float rho = sqrtf(u.x * u.x + u.y * u.y);
    const float q1 = rho - T.r, q2 = fabsf(u.z - 0.5f * T.L) - 0.5f * T.L;
    const float sz = u.z >= 0.5f * T.L ? 1.0f : -1.0f;
    const float3 g1 = rho > 0 ? make_float3(u.x / rho, u.y / rho, 0.0f) : make_float3(1.0f, 0.0f, 0.0f);
    const float3 g2 = make_float3(0.0f, 0.0f, sz);
    float3 g;
    if (q1 <= 0 && q2 <= 0) {
        g = q1 >= q2 ? g1 : g2;
    } else {
        const float a = fmaxf(q1, 0.0f), b = fmaxf(q2, 0.0f);
        const float n = sqrtf(a * a + b * b);
        return make_float3(a * g1.x / n, a * g1.y / n, b * sz / n);
    }
    if (!(fabsf(q1 - q2) <= RIDGE_TOL && rho > 0)) return g;
    const bool on_s = s <= EDGE_TOL, on_t = t <= EDGE_TOL, on_st = (1.0f - s) - t <= EDGE_TOL;
    const int active = (int)on_s + (int)on_t + (int)on_st;
    if (active >= 2) return g;
    const float3 db = make_float3(g1.x - g2.x, g1.y - g2.y, g1.z - g2.z);
    float3 pa, pb;
    if (active == 0) {
        const float3 e1 = T.e1, e2 = T.e2;
        const float3 N = make_float3(e1.y * e2.z - e1.z * e2.y, e1.z * e2.x - e1.x * e2.z, e1.x * e2.y - e1.y * e2.x);
        const float nn = dot3(N, N);
        if (!(nn > 0)) return g;
        const float ga = dot3(g2, N) / nn, gb = dot3(db, N) / nn;
        pa = make_float3(g2.x - ga * N.x, g2.y - ga * N.y, g2.z - ga * N.z);
        pb = make_float3(db.x - gb * N.x, db.y - gb * N.y, db.z - gb * N.z);
    } else {
        const float3 e = on_s ? T.e2 : on_t ? T.e1 : make_float3(T.e2.x - T.e1.x, T.e2.y - T.e1.y, T.e2.z - T.e1.z);
        const float ee = dot3(e, e);
        if (!(ee > 0)) return g;
        const float ga = dot3(g2, e) / ee, gb = dot3(db, e) / ee;
        pa = make_float3(ga * e.x, ga * e.y, ga * e.z);
        pb = make_float3(gb * e.x, gb * e.y, gb * e.z);
    }
    const float bb = dot3(pb, pb);
    if (!(bb > 1e-20f)) return g;
    const float alpha = fminf(1.0f, fmaxf(0.0f, -dot3(pa, pb) / bb));
    return make_float3(g2.x + alpha * db.x, g2.y + alpha * db.y, g2.z + alpha * db.z);
}

// ------------------------------------------------------------------ kernels

__global__ void k_ref_start(const double* __restrict__ init, int K, const double* __restrict__ anchor, double mu0,
                            RefineState* __restrict__ st) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    RefineState& S = st[k];
    const double* P = init + 7 * k;
    quat_mat(P[0], P[1], P[2], P[3], S.R0);
    for (int a = 0; a < 3; ++a) {
        S.p0[a] = P[4 + a];
        S.a[a] = anchor[a];
    }
    for (int j = 0; j < 6; ++j) S.xi[j] = S.xe[j] = S.step[j] = 0.0;
    S.mu = mu0;
    S.it = 0;
    S.status = 0;
}

// pose of the twist xe and the Jacobians the sensitivities need
__device__ void pose_at(RefineState& S, const double* x) {
    const double v[3] = {x[0], x[1], x[2]}, w[3] = {x[3], x[4], x[5]};
    double dR[9], V[9], Ra[3], Vv[3];
    so3_exp(w, dR);
    left_jac(w, V);
    mat3_mul(dR, S.R0, S.R);
    mat3_vec(S.R0, S.a, Ra);
    mat3_vec(V, v, Vv);
    double dRa[3];
    mat3_vec(dR, Ra, dRa);
    for (int i = 0; i < 3; ++i) {
        S.p[i] = S.p0[i] + Vv[i] + Ra[i] - dRa[i];
        S.c[i] = S.p0[i] + Vv[i] + Ra[i];
    }
    for (int i = 0; i < 9; ++i) S.V[i] = V[i];
    // D = d(V(w) v)/dw by central differences (step 1e-7)
    const double hh = 1e-7;
    for (int j = 0; j < 3; ++j) {
        double wp[3] = {w[0], w[1], w[2]}, wm[3] = {w[0], w[1], w[2]};
        wp[j] += hh;
        wm[j] -= hh;
        double Vp[9], Vm[9], a[3], b[3];
        left_jac(wp, Vp);
        left_jac(wm, Vm);
        mat3_vec(Vp, v, a);
        mat3_vec(Vm, v, b);
        for (int i = 0; i < 3; ++i) S.D[3 * i + j] = (a[i] - b[i]) / (2 * hh);
    }
}

__global__ void k_ref_pose(RefineState* __restrict__ st, int K) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K || st[k].status == 2) return;
    pose_at(st[k], st[k].xe);
}

// One thread per (start, probe pose): smallest signed distance over the faces
// kept by the bounding-sphere test, by branch and bound (a face whose lower
// bound f_p(centroid) - radius exceeds the best vertex value cannot hold the
// minimum), ties to the lowest face index.
__global__ __launch_bounds__(64) void k_ref_query(const RefineState* __restrict__ st, int K, RefineGeometry geo,
                                                  const float* __restrict__ poses, int N, RefineConst c,
                                                  RefineHit* __restrict__ hits) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= K * N) return;
    const int k = q / N, i = q - k * N;
    const RefineState& S = st[k];
    if (S.status == 2) return;
    const float* P = poses + 7 * i;
    double Ri[9];
    quat_mat(P[0], P[1], P[2], P[3], Ri);
    const double pi[3] = {P[4], P[5], P[6]};
    Xf X;
    for (int a = 0; a < 3; ++a) {
        for (int b = 0; b < 3; ++b)
            X.a[3 * a + b] = (float)(Ri[a] * S.R[b] + Ri[3 + a] * S.R[3 + b] + Ri[6 + a] * S.R[6 + b]);
        X.c[a] = (float)(Ri[a] * (S.p[0] - pi[0]) + Ri[3 + a] * (S.p[1] - pi[1]) + Ri[6 + a] * (S.p[2] - pi[2]));
    }
    const float r = c.r, L = c.L, cull = c.cull;
    auto sdf_body = [&](float bx, float by, float bz) {
        const float3 u = X.apply(bx, by, bz);
        return sdf_f(u.x, u.y, u.z, r, L);
    };

    // pass 1: best vertex value over the kept faces
    float best_ub = INFINITY;
    int kept = 0;
    for (int tn = 0; tn < geo.n_top; ++tn) {
        const float4 sp = geo.top[tn];
        if (!(sdf_body(sp.x, sp.y, sp.z) < sp.w + cull)) continue;
        const int2 cr = geo.top_range[tn];
        for (int cl = cr.x; cl < cr.x + cr.y; ++cl) {
            const float4 cs = geo.cluster[cl];
            if (!(sdf_body(cs.x, cs.y, cs.z) < cs.w + cull)) continue;
            const int2 fr = geo.cluster_range[cl];
            for (int f = fr.x; f < fr.x + fr.y; ++f) {
                const float4 a0 = geo.face[4 * f], a1 = geo.face[4 * f + 1], a2 = geo.face[4 * f + 2],
                             a3 = geo.face[4 * f + 3];
                if (!(sdf_body(a2.y, a2.z, a2.w) < a3.x + cull)) continue;
                ++kept;
                const float v = fminf(sdf_body(a0.x, a0.y, a0.z),
                                      fminf(sdf_body(a0.w, a1.x, a1.y), sdf_body(a1.z, a1.w, a2.x)));
                best_ub = fminf(best_ub, v);
            }
        }
    }
    RefineHit out;
    if (kept == 0) {
        out.dx = make_float4(c.eps, 0.0f, 0.0f, 0.0f);
        out.nf = make_float4(0.0f, 0.0f, 0.0f, __int_as_float(-1));
        hits[q] = out;
        return;
    }

    // pass 2: minimise the faces whose lower bound does not exceed best_ub
    float best = INFINITY, bs = 0.0f, bt = 0.0f;
    int bidx = 0x7fffffff;
    Tri BT{};
    BT.r = r;
    BT.L = L;
    for (int tn = 0; tn < geo.n_top; ++tn) {
        const float4 sp = geo.top[tn];
        if (!(sdf_body(sp.x, sp.y, sp.z) < sp.w + cull)) continue;
        const int2 cr = geo.top_range[tn];
        for (int cl = cr.x; cl < cr.x + cr.y; ++cl) {
            const float4 cs = geo.cluster[cl];
            if (!(sdf_body(cs.x, cs.y, cs.z) < cs.w + cull)) continue;
            const int2 fr = geo.cluster_range[cl];
            for (int f = fr.x; f < fr.x + fr.y; ++f) {
                const float4 a0 = geo.face[4 * f], a1 = geo.face[4 * f + 1], a2 = geo.face[4 * f + 2],
                             a3 = geo.face[4 * f + 3];
                const float fc = sdf_body(a2.y, a2.z, a2.w);
                if (!(fc < a3.x + cull)) continue;
                if (fc - a3.x > best_ub + 1e-5f) continue;
                const int idx = __float_as_int(a3.y);
                const float3 u0 = X.apply(a0.x, a0.y, a0.z), u1 = X.apply(a0.w, a1.x, a1.y),
                             u2 = X.apply(a1.z, a1.w, a2.x);
                Tri T;
                T.p0 = u0;
                T.e1 = make_float3(u1.x - u0.x, u1.y - u0.y, u1.z - u0.z);
                T.e2 = make_float3(u2.x - u0.x, u2.y - u0.y, u2.z - u0.z);
                T.r = r;
                T.L = L;
                float s, t;
                const float m = face_min(T, s, t);
                if (m < best || (m == best && idx < bidx)) {
                    best = m;
                    bidx = idx;
                    bs = s;
                    bt = t;
                    BT = T;
                }
            }
        }
    }
    const float3 u = make_float3(BT.p0.x + bs * BT.e1.x + bt * BT.e2.x, BT.p0.y + bs * BT.e1.y + bt * BT.e2.y,
                                 BT.p0.z + bs * BT.e1.z + bt * BT.e2.z);
    const float3 gl = witness_gradient(u, BT, bs, bt);
    double xw[3], nw[3];
    for (int a = 0; a < 3; ++a) {
        xw[a] = Ri[3 * a] * u.x + Ri[3 * a + 1] * u.y + Ri[3 * a + 2] * u.z + pi[a];
        nw[a] = Ri[3 * a] * gl.x + Ri[3 * a + 1] * gl.y + Ri[3 * a + 2] * gl.z;
    }
    out.dx = make_float4(best, (float)xw[0], (float)xw[1], (float)xw[2]);
    out.nf = make_float4((float)nw[0], (float)nw[1], (float)nw[2], __int_as_float(bidx));
    hits[q] = out;
}

// proximity score s(d) (Sec. V-A) with ds/dd and d2s/dd2, one-sided at the joints
__device__ void proximity(double d, const RefineConst& c, double& s, double& ds, double& d2) {
    const double tau = c.tau_out2, r = c.tau_in2 / c.tau_out2, k = c.k;
    const double A = k / (r * r) - 2.0 / (r * r * r), B = k / r - 3.0 / (r * r);
    const double t = d / tau;
    s = ds = d2 = 0.0;
    if (t > 0 && t <= 1) {
        const double cs = cos(0.5 * M_PI * t);
        s = cs * cs;
        ds = -0.5 * M_PI * sin(M_PI * t);
        d2 = -0.5 * M_PI * M_PI * cos(M_PI * t);
    } else if (t > -r && t <= 0) {
        s = A * t * t * t + B * t * t + 1.0;
        ds = 3 * A * t * t + 2 * B * t;
        d2 = 6 * A * t + 2 * B;
    } else if (t <= -r) {
        s = k * (t + r);
        ds = k;
    }
    ds /= tau;
    d2 /= tau * tau;
}

constexpr int RED_T = 128;
constexpr int NACC = 28;  // J, grad (6), H upper triangle (21)

__global__ __launch_bounds__(RED_T) void k_ref_reduce(const RefineState* __restrict__ st, const RefineHit* __restrict__ hits,
                                                     int N, RefineConst c, RefineEval* __restrict__ ev) {
    const int k = blockIdx.x;
    const RefineState& S = st[k];
    if (S.status == 2) return;
    __shared__ double red[NACC][RED_T];
    double V[9], D[9], cc[3];
    for (int j = 0; j < 9; ++j) {
        V[j] = S.V[j];
        D[j] = S.D[j];
    }
    for (int j = 0; j < 3; ++j) cc[j] = S.c[j];
    double acc[NACC];
    for (int j = 0; j < NACC; ++j) acc[j] = 0.0;
    for (int i = threadIdx.x; i < N; i += RED_T) {
        const RefineHit hv = hits[(size_t)k * N + i];
        double s, ds, d2;
        proximity((double)hv.dx.x, c, s, ds, d2);
        if (s == 0.0 && ds == 0.0 && d2 == 0.0) continue;
        const double n[3] = {hv.nf.x, hv.nf.y, hv.nf.z};
        const double r[3] = {hv.dx.y - cc[0], hv.dx.z - cc[1], hv.dx.w - cc[2]};
        const double rn[3] = {r[1] * n[2] - r[2] * n[1], r[2] * n[0] - r[0] * n[2], r[0] * n[1] - r[1] * n[0]};
        double g[6];
        for (int j = 0; j < 3; ++j) {
            g[j] = V[j] * n[0] + V[3 + j] * n[1] + V[6 + j] * n[2];
            g[3 + j] = V[j] * rn[0] + V[3 + j] * rn[1] + V[6 + j] * rn[2] + D[j] * n[0] + D[3 + j] * n[1] +
                       D[6 + j] * n[2];
        }
        acc[0] -= s;
        for (int j = 0; j < 6; ++j) acc[1 + j] -= ds * g[j];
        const double w = fmax(0.0, -d2);
        int o = 7;
        for (int a = 0; a < 6; ++a)
            for (int b = a; b < 6; ++b) acc[o++] += w * g[a] * g[b];
    }
    for (int j = 0; j < NACC; ++j) red[j][threadIdx.x] = acc[j];
    __syncthreads();
    for (int stride = RED_T / 2; stride > 0; stride >>= 1) {
        if (threadIdx.x < stride)
            for (int j = 0; j < NACC; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + stride];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        RefineEval& E = ev[k];
        double xx = 0;
        for (int j = 0; j < 6; ++j) xx += S.xe[j] * S.xe[j];
        E.J = red[0][0] + c.lambda * xx;
        for (int j = 0; j < 6; ++j) E.g[j] = red[1 + j][0] + 2 * c.lambda * S.xe[j];
        int o = 0;
        for (int a = 0; a < 6; ++a)
            for (int b = a; b < 6; ++b, ++o) E.H[o] = red[7 + o][0] + (a == b ? 2 * c.lambda : 0.0);
    }
}

// Cholesky solve of the SPD 6x6 system A x = b; false if A is not positive definite
__device__ bool chol6(double* A, const double* b, double* x) {
    for (int j = 0; j < 6; ++j) {
        double s = A[6 * j + j];
        for (int k = 0; k < j; ++k) s -= A[6 * j + k] * A[6 * j + k];
        if (!(s > 0)) return false;
        const double l = sqrt(s);
        A[6 * j + j] = l;
        for (int i = j + 1; i < 6; ++i) {
            double t = A[6 * i + j];
            for (int k = 0; k < j; ++k) t -= A[6 * i + k] * A[6 * j + k];
            A[6 * i + j] = t / l;
        }
    }
    double y[6];
    for (int i = 0; i < 6; ++i) {
        double t = b[i];
        for (int k = 0; k < i; ++k) t -= A[6 * i + k] * y[k];
        y[i] = t / A[6 * i + i];
    }
    for (int i = 5; i >= 0; --i) {
        double t = y[i];
        for (int k = i + 1; k < 6; ++k) t -= A[6 * k + i] * x[k];
        x[i] = t / A[6 * i + i];
    }
    return true;
}

__device__ double maxabs6(const double* v) {
    double m = 0;
    for (int j = 0; j < 6; ++j) m = fmax(m, fabs(v[j]));
    return m;
}

// next trial from (xi, g, H, mu); false when no positive-definite system is left
__device__ bool make_trial(RefineState& S, const RefineConst& c) {
    while (S.mu < 1e12) {
        double A[36], rhs[6], step[6];
        for (int a = 0; a < 6; ++a) {
            for (int b = 0; b < 6; ++b) A[6 * a + b] = S.H[6 * a + b];
            A[6 * a + a] += S.mu * S.H[6 * a + a] + 1e-12;
            rhs[a] = -S.g[a];
        }
        if (chol6(A, rhs, step)) {
            for (int j = 0; j < 6; ++j) {
                S.step[j] = step[j];
                S.xe[j] = clampd(S.xi[j] + step[j], j < 3 ? c.b_t : c.b_r);
            }
            S.status = 1;
            return true;
        }
        S.mu *= 3.0;
    }
    return false;
}

// continue from an accepted point: projected-gradient test, iteration cap, trial
__device__ void next_iteration(RefineState& S, const RefineConst& c) {
    double pg = 0;
    for (int j = 0; j < 6; ++j) {
        const double b = j < 3 ? c.b_t : c.b_r;
        pg = fmax(pg, fabs(S.xi[j] - clampd(S.xi[j] - S.g[j], b)));
    }
    if (pg <= c.tol_pg || S.it >= c.max_iters) {
        S.status = 2;
        return;
    }
    S.it += 1;
    if (!make_trial(S, c)) S.status = 2;
}

__global__ void k_ref_step(RefineState* __restrict__ st, int K, const RefineEval* __restrict__ ev, RefineConst c,
                           int* __restrict__ active) {
    int mine = 0;
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        RefineState& S = st[k];
        if (S.status != 2) {
            const RefineEval& E = ev[k];
            bool take = S.status == 0 || E.J < S.J;
            if (take) {
                const bool first = S.status == 0;
                for (int j = 0; j < 6; ++j) {
                    S.xi[j] = S.xe[j];
                    S.g[j] = E.g[j];
                }
                S.J = E.J;
                int o = 0;
                for (int a = 0; a < 6; ++a)
                    for (int b = a; b < 6; ++b, ++o) S.H[6 * a + b] = S.H[6 * b + a] = E.H[o];
                if (!first) S.mu = fmax(S.mu / 3.0, 1e-12);
                if (!first && maxabs6(S.step) <= c.tol_step) S.status = 2;
                else next_iteration(S, c);
            } else {
                S.mu *= 3.0;
                if (S.mu >= 1e12 || maxabs6(S.step) <= c.tol_step || !make_trial(S, c)) S.status = 2;
            }
        }
        mine += S.status != 2;
    }
    // the number of unfinished starts, summed over the block (blockDim.x <= 1024)
    __shared__ int part[16];
    int v = mine;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int sum = 0;
        for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) sum += part[w];
        *active = sum;
    }
}

__global__ void k_ref_finish(const RefineState* __restrict__ st, int K, double* __restrict__ out_poses,
                             double* __restrict__ out_J, int32_t* __restrict__ out_iters) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    RefineState S = st[k];
    pose_at(S, S.xi);
    const double* R = S.R;
    double w, x, y, z;
    const double tr = R[0] + R[4] + R[8];
    if (tr > 0) {
        const double q = 2 * sqrt(tr + 1);
        w = 0.25 * q; x = (R[7] - R[5]) / q; y = (R[2] - R[6]) / q; z = (R[3] - R[1]) / q;
    } else if (R[0] > R[4] && R[0] > R[8]) {
        const double q = 2 * sqrt(1 + R[0] - R[4] - R[8]);
        w = (R[7] - R[5]) / q; x = 0.25 * q; y = (R[1] + R[3]) / q; z = (R[2] + R[6]) / q;
    } else if (R[4] > R[8]) {
        const double q = 2 * sqrt(1 + R[4] - R[0] - R[8]);
        w = (R[2] - R[6]) / q; x = (R[1] + R[3]) / q; y = 0.25 * q; z = (R[5] + R[7]) / q;
    } else {
        const double q = 2 * sqrt(1 + R[8] - R[0] - R[4]);
        w = (R[3] - R[1]) / q; x = (R[2] + R[6]) / q; y = (R[5] + R[7]) / q; z = 0.25 * q;
    }
    const double sg = w < 0 ? -1.0 : 1.0;
    double* o = out_poses + 7 * k;
    o[0] = sg * w; o[1] = sg * x; o[2] = sg * y; o[3] = sg * z;
    o[4] = S.p[0]; o[5] = S.p[1]; o[6] = S.p[2];
    if (out_J) out_J[k] = S.J;
    if (out_iters) out_iters[k] = S.it;
}

}  // namespace

hipError_t refine_start(const double* init_poses, int K, const double* anchor, const RefineConst& c, RefineState* st,
                        hipStream_t s) {
    k_ref_start<<<(K + 63) / 64, 64, 0, s>>>(init_poses, K, anchor, c.mu0, st);
    return hipGetLastError();
}

hipError_t refine_round(RefineState* st, int K, const RefineGeometry& geo, const float* poses, int n_poses,
                        const RefineConst& c, RefineHit* hits, RefineEval* ev, int* active, hipStream_t s) {
    k_ref_pose<<<(K + 63) / 64, 64, 0, s>>>(st, K);
    const long long q = (long long)K * n_poses;
    k_ref_query<<<(unsigned)((q + 63) / 64), 64, 0, s>>>(st, K, geo, poses, n_poses, c, hits);
    k_ref_reduce<<<K, RED_T, 0, s>>>(st, hits, n_poses, c, ev);
    k_ref_step<<<1, 256, 0, s>>>(st, K, ev, c, active);
    return hipGetLastError();
}

hipError_t refine_finish(const RefineState* st, int K, double* out_poses, double* out_J, int32_t* out_iters,
                         hipStream_t s) {
    k_ref_finish<<<(K + 63) / 64, 64, 0, s>>>(st, K, out_poses, out_J, out_iters);
    return hipGetLastError();
}

hipError_t refine_query_only(RefineState* st, const RefineGeometry& geo, const float* poses, int n_poses,
                             const RefineConst& c, RefineHit* hits, hipStream_t s) {
    k_ref_query<<<(n_poses + 63) / 64, 64, 0, s>>>(st, 1, geo, poses, n_poses, c, hits);
    return hipGetLastError();
}
