// Continuous SE(3) refinement (Sec. V) on the device.
//
// Every start (an initial object pose from the global search) is refined by a
// damped Gauss-Newton iteration on the twist xi = (v, w), one evaluation round
// per trial step for all unfinished starts at once:
//   k_ref_cull, k_ref_pairs, k_ref_nested, k_ref_winner, k_ref_resolve
//                 per (start, probe pose) the smallest signed distance d, its
//                 witness x* and the probe normal n (Sec. V-B): the face
//                 searches in FP32, the winning face's minimiser polished and
//                 evaluated in FP64;
//   k_ref_eval    FP64, REF_EVAL_PARTS blocks per trial: J = -sum s(d) + lambda |xi|^2,
//                 grad J and the curvature sum max(0, -s'') g g^T + 2 lambda I
//                 with g the contact sensitivities (Sec. V-C), in a fixed
//                 summation order;
//   k_ref_decide  FP64, one block per start: accept or reject the trials in
//                 the order the sequential iteration tries them, update the
//                 damping, solve (H + mu diag H + 1e-12 I) step = -grad by
//                 Cholesky for the next trials, and set up their poses
//                 R = exp(w^) R0, p = p0 + V(w) v + (I - exp(w^)) R0 a
//                 (Eq. se3-exp and the left updates) with V(w), the coupling
//                 D = d(V v)/dw and the pivot c = p0 + V v + R0 a.
// The L-BFGS-B variant (the paper's solver) replaces k_ref_decide by
// k_ref_decide_lbfgsb on the same queries and evaluations.
#include "refine_kernels.h"

#include <algorithm>
#include <cmath>

namespace {

constexpr float GOLD_TOL = 1e-5f;         // barycentric bracket width of the face minimisation
constexpr float RIDGE_TOL = 1e-4f;        // |q1 - q2| below which a witness is on the side/cap ridge
constexpr float EDGE_TOL = 1e-4f;         // barycentric distance below which a witness is on an edge
constexpr float INVPHI_F = 0.618033988749894848f;
constexpr float BOUND_SLACK = 1e-5f;      // float32 rounding allowance of the face bounds (mm)
constexpr float VERTEX_GAP = 2e-6f;       // bounds this close: the best vertex is the face minimum (mm)
constexpr float CERT_TOL = 4e-6f;         // a boundary point this close to a lower bound is the face minimum (mm)
constexpr int RIM_NEWTON = 3;             // Newton steps of the FP64 witness polish (rim edge)
constexpr int RIDGE_NEWTON = 4;           // and (inner ridge inside a face)

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

// hardware square root (v_sqrt_f32, about 1 ulp): the correctly rounded
// sqrtf adds a dozen dependent instructions, which the sequential face
// searches pay on every evaluation; 1 ulp of a radius is ~1e-7 of it
__device__ __forceinline__ float hw_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// capped cylinder, tip disk at the origin, axis +z, length L (negative inside)
__device__ __forceinline__ float sdf_f(float x, float y, float z, float r, float L) {
    const float q1 = hw_sqrt(x * x + y * y) - r;
    const float q2 = fabsf(z - 0.5f * L) - 0.5f * L;
    const float in = fminf(fmaxf(q1, q2), 0.0f);
    const float a = fmaxf(q1, 0.0f), b = fmaxf(q2, 0.0f);
    return in + hw_sqrt(a * a + b * b);
}

// hardware reciprocal (v_rcp_f32, about 1 ulp): the gradients feed bounds
// and slope tests whose allowances are far above float32 rounding
__device__ __forceinline__ float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// f_p and a subgradient (the gradient where f_p is differentiable; on the
// inner ridge the gradient of the larger branch)
__device__ __forceinline__ float sdf_grad_f(float3 u, float r, float L, float3& g) {
    const float rho = hw_sqrt(u.x * u.x + u.y * u.y);
    const float q1 = rho - r, q2 = fabsf(u.z - 0.5f * L) - 0.5f * L;
    const float sz = u.z >= 0.5f * L ? 1.0f : -1.0f;
    const bool off_axis = rho > 1e-30f;
    const float ir = off_axis ? hw_rcp(rho) : 0.0f;
    const float ex = off_axis ? u.x * ir : 1.0f, ey = off_axis ? u.y * ir : 0.0f;
    if (q1 <= 0 && q2 <= 0) {
        if (q1 >= q2) {
            g = make_float3(ex, ey, 0.0f);
            return q1;
        }
        g = make_float3(0.0f, 0.0f, sz);
        return q2;
    }
    const float a = fmaxf(q1, 0.0f), b = fmaxf(q2, 0.0f);
    const float n = hw_sqrt(a * a + b * b);
    const float in = n > 0.0f ? hw_rcp(n) : 0.0f;
    g = make_float3(a * in * ex, a * in * ey, b * in * sz);
    return n;
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
__device__ float face_min_nested(const Tri& T, float& s_out, float& t_out) {
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

__device__ __forceinline__ float3 f3sub(float3 a, float3 b) { return make_float3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ float3 f3add(float3 a, float3 b) { return make_float3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ float3 f3scale(float3 a, float k) { return make_float3(k * a.x, k * a.y, k * a.z); }

// the probe's point farthest along m (its support point): the rim in the
// direction of m's xy part, on the cap m.z points to
__device__ __forceinline__ float3 probe_support(float3 m, float r, float L) {
    const float h = hw_sqrt(m.x * m.x + m.y * m.y);
    const float k = h > 0.0f ? r / h : 0.0f;
    return make_float3(k * m.x, k * m.y, m.z > 0.0f ? L : 0.0f);
}

// min of f_p over the segment P + l D, l in [0, 1], given the values and
// subgradients at its ends.  f_p is convex: an end whose subgradient does not
// descend into the segment holds the minimum; otherwise golden section over
// l, then the ends.
__device__ float seg_min(float3 P, float3 D, float f0, float3 g0, float f1, float3 g1, float r, float L,
                         float& l_out) {
    if (dot3(g0, D) >= 0.0f) {
        l_out = 0.0f;
        return f0;
    }
    if (dot3(g1, D) <= 0.0f) {
        l_out = 1.0f;
        return f1;
    }
    auto at = [&](float l) { return sdf_f(P.x + l * D.x, P.y + l * D.y, P.z + l * D.z, r, L); };
    float a = 0.0f, b = 1.0f;
    float c = b - INVPHI_F * (b - a), d = a + INVPHI_F * (b - a);
    float fc = at(c), fd = at(d);
    while (b - a > GOLD_TOL) {
        if (fc <= fd) {
            b = d; d = c; fd = fc; c = b - INVPHI_F * (b - a); fc = at(c);
        } else {
            a = c; c = d; fc = fd; d = a + INVPHI_F * (b - a); fd = at(d);
        }
    }
    float lm = 0.5f * (a + b), fm = at(lm);
    if (f0 < fm) { fm = f0; lm = 0.0f; }
    if (f1 < fm) { fm = f1; lm = 1.0f; }
    l_out = lm;
    return fm;
}

// Lower bound of f_p over the triangle with vertices xb + w_j from the
// supporting half-space of the probe with unit normal m: f_p(y) >= m . y -
// max_C m . x for every y (inside the probe too), minimised over the vertices.
__device__ __forceinline__ float plane_lb(float3 m, float3 xb, float3 w0, float3 w1, float3 w2, float r, float L) {
    const float3 sp = probe_support(m, r, L);
    return fminf(dot3(m, w0), fminf(dot3(m, w1), dot3(m, w2))) + dot3(m, f3sub(xb, sp));
}

// Lower bound of f_p over the triangle from the two branches at xb:
// f_p >= max(q1, q2) >= a q1 + (1 - a) q2 for a in [0, 1], with q1 = rho - r
// and q2 = |z - L/2| - L/2 convex and bounded below by their tangent planes at
// xb.  Over the triangle this is min_j (c_j + a d_j), maximised over a at 0,
// 1 and the crossings of the three lines.
__device__ float ridge_lb(float3 xb, float3 w0, float3 w1, float3 w2, float r, float L) {
    const float rho = hw_sqrt(xb.x * xb.x + xb.y * xb.y);
    if (!(rho > 0.0f)) return -INFINITY;
    const float q1 = rho - r, q2 = fabsf(xb.z - 0.5f * L) - 0.5f * L;
    const float sz = xb.z >= 0.5f * L ? 1.0f : -1.0f;
    const float ex = xb.x / rho, ey = xb.y / rho;
    // c_j = q2 + g2 . w_j, d_j = (q1 - q2) + (g1 - g2) . w_j
    const float c0 = q2 + sz * w0.z, c1 = q2 + sz * w1.z, c2 = q2 + sz * w2.z;
    const float d0 = (q1 - q2) + ex * w0.x + ey * w0.y - sz * w0.z;
    const float d1 = (q1 - q2) + ex * w1.x + ey * w1.y - sz * w1.z;
    const float d2 = (q1 - q2) + ex * w2.x + ey * w2.y - sz * w2.z;
    auto env = [&](float a) { return fminf(c0 + a * d0, fminf(c1 + a * d1, c2 + a * d2)); };
    float best = fmaxf(env(0.0f), env(1.0f));
    auto cross_at = [&](float ci, float di, float cj, float dj) {
        if (di != dj) {
            const float a = (cj - ci) / (di - dj);
            if (a > 0.0f && a < 1.0f) best = fmaxf(best, env(a));
        }
    };
    cross_at(c0, d0, c1, d1);
    cross_at(c0, d0, c2, d2);
    cross_at(c1, d1, c2, d2);
    return best;
}

// Minimum of the probe SDF over the triangle p0 + s e1 + t e2 (s, t >= 0,
// s + t <= 1), exact up to the golden-section bracket:
//  * the least of the three edge minima is the boundary minimum;
//  * if the probe lies strictly on one side of the face plane, f_p on the
//    plane is the distance to the probe and its minimum is the projection of
//    the probe's nearest (support) point: the face minimum if inside the
//    face, else the minimum lies on the boundary;
//  * otherwise the boundary minimum is the face minimum when a lower bound of
//    f_p over the face (supporting half-spaces of the probe at the witness'
//    normal, and the branch bound) comes within CERT_TOL of it;
//  * else (a minimum inside the face on the side/cap ridge of a penetrating
//    face) nested golden sections.
// face_min_bounded stops before the last step and clears `done` instead.
__device__ float face_min_bounded(const Tri& T, float& s_out, float& t_out, bool& done) {
    done = true;
    const float r = T.r, L = T.L;
    const float3 p0 = T.p0, p1 = f3add(T.p0, T.e1), p2 = f3add(T.p0, T.e2), e12 = f3sub(T.e2, T.e1);
    float3 g0, g1, g2;
    const float f0 = sdf_grad_f(p0, r, L, g0), f1 = sdf_grad_f(p1, r, L, g1), f2 = sdf_grad_f(p2, r, L, g2);
    float l, best, bs, bt;
    float3 edge = T.e1;
    best = seg_min(p0, T.e1, f0, g0, f1, g1, r, L, l);
    bs = l;
    bt = 0.0f;
    bool inner = l > 0.0f && l < 1.0f;
    float m = seg_min(p0, T.e2, f0, g0, f2, g2, r, L, l);
    if (m < best) {
        best = m; bs = 0.0f; bt = l; edge = T.e2; inner = l > 0.0f && l < 1.0f;
    }
    m = seg_min(p1, e12, f1, g1, f2, g2, r, L, l);
    if (m < best) {
        best = m; bs = 1.0f - l; bt = l; edge = e12; inner = l > 0.0f && l < 1.0f;
    }
    s_out = bs;
    t_out = bt;
    const float3 N = make_float3(T.e1.y * T.e2.z - T.e1.z * T.e2.y, T.e1.z * T.e2.x - T.e1.x * T.e2.z,
                                 T.e1.x * T.e2.y - T.e1.y * T.e2.x);
    const float nn = dot3(N, N);
    if (!(nn > 0.0f)) return best;  // a degenerate face is the union of its edges
    const float3 n = f3scale(N, 1.0f / hw_sqrt(nn));
    const float3 sh = probe_support(n, r, L), sl = probe_support(make_float3(-n.x, -n.y, -n.z), r, L);
    const float top = dot3(n, f3sub(sh, p0)), bot = dot3(n, f3sub(sl, p0));
    if (bot > 0.0f || top < 0.0f) {
        const float h = bot > 0.0f ? bot : top;
        const float3 x = f3sub(f3sub(bot > 0.0f ? sl : sh, f3scale(n, h)), p0);
        const float a11 = dot3(T.e1, T.e1), a12 = dot3(T.e1, T.e2), a22 = dot3(T.e2, T.e2);
        const float b1 = dot3(x, T.e1), b2 = dot3(x, T.e2), det = a11 * a22 - a12 * a12;
        const float s = (b1 * a22 - b2 * a12) / det, t = (b2 * a11 - b1 * a12) / det;
        if (s >= 0.0f && t >= 0.0f && s + t <= 1.0f) {
            const float v = T.at(s, t);
            if (v < best) {
                s_out = s;
                t_out = t;
                return v;
            }
        }
        return best;
    }
    const float3 xb = make_float3(p0.x + bs * T.e1.x + bt * T.e2.x, p0.y + bs * T.e1.y + bt * T.e2.y,
                                  p0.z + bs * T.e1.z + bt * T.e2.z);
    const float3 w0 = f3sub(p0, xb), w1 = f3sub(p1, xb), w2 = f3sub(p2, xb);
    float3 gm;
    (void)sdf_grad_f(xb, r, L, gm);
    float lb = fmaxf(plane_lb(gm, xb, w0, w1, w2, r, L), ridge_lb(xb, w0, w1, w2, r, L));
    if (inner && lb < best - CERT_TOL) {
        // at a minimum inside an edge the normal is orthogonal to the edge:
        // drop the component the bracket error leaves along it
        const float3 pm = f3sub(gm, f3scale(edge, dot3(gm, edge) / dot3(edge, edge)));
        const float pn = dot3(pm, pm);
        if (pn > 0.0f) lb = fmaxf(lb, plane_lb(f3scale(pm, 1.0f / hw_sqrt(pn)), xb, w0, w1, w2, r, L));
    }
    done = lb >= best - CERT_TOL;
    return best;
}

__device__ float face_min(const Tri& T, float& s_out, float& t_out) {
    bool done;
    const float m = face_min_bounded(T, s_out, t_out, done);
    return done ? m : face_min_nested(T, s_out, t_out);
}


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

// ------------------------------------------------------ FP64 witness polish
//
// The float32 searches place a smooth face minimum only to about
// sqrt(2 e / k) (e the float32 rounding of f_p, k its curvature along the
// face): up to ~1e-3 mm where the probe wall runs close to an edge, and a
// minimum where f_p is nearly constant (a face almost parallel to the tip
// disk) anywhere in that flat part.  The witness sets d, the contact normal and
// the moment arm of the sensitivities, so the winning face of every live query
// is placed by the FP64 pose and minimised again in FP64 over a few candidate
// points that hold the exact minimiser: f_p of the capped cylinder along a line
// or over a plane is made of pieces (wall: rho - r, cap: a linear q2, rim:
// sqrt(q1^2 + q2^2), inside: max(q1, q2)), so its minimum is at a stationary
// point of a smooth piece, on the inner side/cap ridge where max(q1, q2)
// kinks, or at an end.  The candidate with the least f_p wins; the search's own
// point is one of them, so the polish never raises f_p.
//  * On an edge: both ends; the wall's stationary point (rho^2 is quadratic
//    along the edge, closed form); the rim's (Newton on q1^2 + q2^2 from the
//    search's point); the two crossings of the ridge rho = r + q2 (a quadratic
//    equation, q2 being linear along the edge; one Newton step polishes each).
//  * Inside the face: the projection of the probe's support point (exact when
//    the probe lies strictly on one side of the plane); the minimiser on the
//    inner ridge (Newton on a grad q1 + (1 - a) grad q2 = 0, q1 = q2 in the
//    face coordinates, from the better of the search's point and that
//    projection: a face grazing the rim circle cuts the probe by a hair); the
//    crossing of the axis (rho = 0).
__device__ __forceinline__ void sdf_q64(const double* u, double r, double L, double& rho, double& q1, double& q2) {
    rho = sqrt(u[0] * u[0] + u[1] * u[1]);
    q1 = rho - r;
    q2 = fabs(u[2] - 0.5 * L) - 0.5 * L;
}

__device__ double sdf64(const double* u, double r, double L) {
    double rho, q1, q2;
    sdf_q64(u, r, L, rho, q1, q2);
    const double a = fmax(q1, 0.0), b = fmax(q2, 0.0);
    return fmin(fmax(q1, q2), 0.0) + sqrt(a * a + b * b);
}

__device__ __forceinline__ double seg_f64(const double* Q, const double* D, double l, double r, double L) {
    const double u[3] = {Q[0] + l * D[0], Q[1] + l * D[1], Q[2] + l * D[2]};
    return sdf64(u, r, L);
}

// minimiser of f_p on the segment Q + l D, l in [0, 1]: l_best / f_best hold
// the search's point on entry and the best candidate on return
__device__ void polish_edge(const double* Q, const double* D, double r, double L, double& l_best, double& f_best) {
    const double l0 = l_best;
    auto consider = [&](double l) {
        if (!(l >= 0.0 && l <= 1.0)) return;
        const double f = seg_f64(Q, D, l, r, L);
        if (f < f_best) {
            f_best = f;
            l_best = l;
        }
    };
    consider(0.0);
    consider(1.0);
    const double dd = D[0] * D[0] + D[1] * D[1];
    if (dd > 0.0) consider(-(Q[0] * D[0] + Q[1] * D[1]) / dd);  // wall
    const double sz = Q[2] + l0 * D[2] >= 0.5 * L ? 1.0 : -1.0;
    {   // rim
        double l = l0;
        bool ok = true;
        for (int it = 0; it < RIM_NEWTON && ok; ++it) {
            const double ux = Q[0] + l * D[0], uy = Q[1] + l * D[1], uz = Q[2] + l * D[2];
            const double rho = sqrt(ux * ux + uy * uy);
            ok = rho > 0.0;
            if (!ok) break;
            const double ir = 1.0 / rho;
            const double rp = (ux * D[0] + uy * D[1]) * ir, rpp = (dd - rp * rp) * ir;
            const double a1 = rho - r, a2 = sz * (uz - 0.5 * L) - 0.5 * L;
            const double g2 = rp * rp + a1 * rpp + D[2] * D[2];
            ok = g2 > 0.0;
            if (ok) l -= (a1 * rp + a2 * sz * D[2]) / g2;
        }
        if (ok) consider(l);
    }
    {   // ridge crossings: (Qx + l Dx)^2 + (Qy + l Dy)^2 = (r + q2)^2, q2 = b0 + b1 l
        const double b1 = sz * D[2], g0 = r + sz * (Q[2] - 0.5 * L) - 0.5 * L;
        const double qa = dd - b1 * b1, qb = Q[0] * D[0] + Q[1] * D[1] - g0 * b1;
        const double qc = Q[0] * Q[0] + Q[1] * Q[1] - g0 * g0;
        const double disc = qb * qb - qa * qc;
        if (disc >= 0.0) {
            const double qq = -(qb + copysign(sqrt(disc), qb));
            const double roots[2] = {qa != 0.0 ? qq / qa : INFINITY, qq != 0.0 ? qc / qq : INFINITY};
            for (int j = 0; j < 2; ++j) {
                double l = roots[j];
                if (!(l >= -1e-3 && l <= 1.0 + 1e-3)) continue;
                const double ux = Q[0] + l * D[0], uy = Q[1] + l * D[1], rh = sqrt(ux * ux + uy * uy);
                if (rh > 0.0) {  // one Newton step on rho - r - q2
                    const double dphi = (ux * D[0] + uy * D[1]) / rh - b1;
                    if (dphi != 0.0) l -= (rh - g0 - b1 * l) / dphi;
                }
                consider(l);
            }
        }
    }
}

// interior candidate: the projection of the probe's support point onto the
// face plane (the minimiser when the probe lies strictly on one side)
__device__ bool polish_support(const double* P0, const double* E1, const double* E2, double r, double L, double& s_out,
                               double& t_out) {
    double N[3] = {E1[1] * E2[2] - E1[2] * E2[1], E1[2] * E2[0] - E1[0] * E2[2], E1[0] * E2[1] - E1[1] * E2[0]};
    const double nn = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
    if (!(nn > 0.0)) return false;
    for (int a = 0; a < 3; ++a) N[a] /= nn;
    auto support = [&](double sg, double* o) {
        const double mx = sg * N[0], my = sg * N[1], h = sqrt(mx * mx + my * my);
        const double k = h > 0.0 ? r / h : 0.0;
        o[0] = k * mx;
        o[1] = k * my;
        o[2] = sg * N[2] > 0.0 ? L : 0.0;
    };
    double sh[3], sl[3];
    support(1.0, sh);
    support(-1.0, sl);
    double top = 0.0, bot = 0.0;
    for (int a = 0; a < 3; ++a) {
        top += N[a] * (sh[a] - P0[a]);
        bot += N[a] * (sl[a] - P0[a]);
    }
    // the probe's nearest point to the plane, or where it cuts the plane the
    // support point of the shallower side (a face grazing the rim circle)
    const bool low = bot > 0.0 || (!(top < 0.0) && fabs(bot) <= fabs(top));
    const double h = low ? bot : top;
    const double* sp = low ? sl : sh;
    double x[3];
    for (int a = 0; a < 3; ++a) x[a] = sp[a] - N[a] * h - P0[a];
    const double a11 = E1[0] * E1[0] + E1[1] * E1[1] + E1[2] * E1[2];
    const double a12 = E1[0] * E2[0] + E1[1] * E2[1] + E1[2] * E2[2];
    const double a22 = E2[0] * E2[0] + E2[1] * E2[1] + E2[2] * E2[2];
    const double b1 = x[0] * E1[0] + x[1] * E1[1] + x[2] * E1[2], b2 = x[0] * E2[0] + x[1] * E2[1] + x[2] * E2[2];
    const double det = a11 * a22 - a12 * a12;
    if (!(det > 0.0)) return false;
    const double s = (b1 * a22 - b2 * a12) / det, t = (b2 * a11 - b1 * a12) / det;
    if (!(s >= 0.0 && t >= 0.0 && s + t <= 1.0)) return false;
    s_out = s;
    t_out = t;
    return true;
}

// interior witness on the inner ridge; (s, t) and the branch weight a by Newton
__device__ bool polish_ridge(const double* P0, const double* E1, const double* E2, double s0, double t0, double r,
                             double L, double& s_out, double& t_out) {
    double u0[3];
    for (int a = 0; a < 3; ++a) u0[a] = P0[a] + s0 * E1[a] + t0 * E2[a];
    double rho, q1, q2;
    sdf_q64(u0, r, L, rho, q1, q2);
    if (!(q1 <= 0.0 && q2 <= 0.0 && fabs(q1 - q2) <= (double)RIDGE_TOL && rho > 0.0)) return false;
    const double sz = u0[2] >= 0.5 * L ? 1.0 : -1.0;
    const double c1 = sz * E1[2], c2 = sz * E2[2];  // grad q2 in (s, t)
    double s = s0, t = t0, wa = -1.0;
    const double m11 = E1[0] * E1[0] + E1[1] * E1[1], m12 = E1[0] * E2[0] + E1[1] * E2[1];
    const double m22 = E2[0] * E2[0] + E2[1] * E2[1];
    // quadratic convergence from the search's point (~1e-3 of the face off)
    for (int it = 0; it < RIDGE_NEWTON; ++it) {
        const double wx = P0[0] + s * E1[0] + t * E2[0], wy = P0[1] + s * E1[1] + t * E2[1];
        rho = sqrt(wx * wx + wy * wy);
        if (!(rho > 0.0)) return false;
        const double ir = 1.0 / rho;
        const double g1 = (E1[0] * wx + E1[1] * wy) * ir, g2 = (E2[0] * wx + E2[1] * wy) * ir;  // grad q1
        const double h11 = (m11 - g1 * g1) * ir, h12 = (m12 - g1 * g2) * ir, h22 = (m22 - g2 * g2) * ir;
        const double d1 = g1 - c1, d2 = g2 - c2;
        if (wa < 0.0) {  // the weight that best cancels the two gradients
            const double dd = d1 * d1 + d2 * d2;
            if (!(dd > 0.0)) return false;
            wa = fmin(1.0, fmax(0.0, -(c1 * d1 + c2 * d2) / dd));
        }
        const double zq2 = sz * (P0[2] + s * E1[2] + t * E2[2] - 0.5 * L) - 0.5 * L;
        const double F1 = c1 + wa * d1, F2 = c2 + wa * d2, F3 = (rho - r) - zq2;
        // [[a H, d], [d^T, 0]] (ds, dt, da) = -(F1, F2, F3)
        const double A11 = wa * h11, A12 = wa * h12, A22 = wa * h22;
        const double det = -A11 * d2 * d2 + A12 * d1 * d2 + d1 * (A12 * d2 - A22 * d1);
        if (!(fabs(det) > 1e-300)) return false;
        const double idet = 1.0 / det;
        const double b1 = -F1, b2 = -F2, b3 = -F3;
        // Cramer's rule
        const double ds = (-b1 * d2 * d2 + A12 * d2 * b3 + d1 * (b2 * d2 - A22 * b3)) * idet;
        const double dt = (-A11 * d2 * b3 + b1 * d1 * d2 + d1 * (A12 * b3 - b2 * d1)) * idet;
        const double da = (A11 * (A22 * b3 - b2 * d2) - A12 * (A12 * b3 - b2 * d1) + b1 * (A12 * d2 - A22 * d1)) * idet;
        s += ds;
        t += dt;
        wa += da;
    }
    if (!(wa >= 0.0 && wa <= 1.0)) return false;
    s_out = s;
    t_out = t;
    return true;
}

// witness_gradient in FP64: grad f_p, or on the inner ridge the branch mix
// with no component along the face (interior witness) or the edge it is on
__device__ void witness_gradient64(const double* u, const double* E1, const double* E2, double s, double t, double r,
                                   double L, double* g) {
    double rho, q1, q2;
    sdf_q64(u, r, L, rho, q1, q2);
    const double ex = rho > 0.0 ? u[0] / rho : 1.0, ey = rho > 0.0 ? u[1] / rho : 0.0;
    const double sz = u[2] >= 0.5 * L ? 1.0 : -1.0;
    if (!(q1 <= 0.0 && q2 <= 0.0)) {
        const double a = fmax(q1, 0.0), b = fmax(q2, 0.0), n = sqrt(a * a + b * b);
        g[0] = a * ex / n;
        g[1] = a * ey / n;
        g[2] = b * sz / n;
        return;
    }
    g[0] = q1 >= q2 ? ex : 0.0;
    g[1] = q1 >= q2 ? ey : 0.0;
    g[2] = q1 >= q2 ? 0.0 : sz;
    if (!(fabs(q1 - q2) <= (double)RIDGE_TOL && rho > 0.0)) return;
    const bool on_s = s <= (double)EDGE_TOL, on_t = t <= (double)EDGE_TOL, on_st = 1.0 - s - t <= (double)EDGE_TOL;
    const int active = (int)on_s + (int)on_t + (int)on_st;
    if (active >= 2) return;
    const double g2v[3] = {0.0, 0.0, sz}, db[3] = {ex, ey, -sz};
    double pa[3], pb[3];
    if (active == 0) {
        const double N[3] = {E1[1] * E2[2] - E1[2] * E2[1], E1[2] * E2[0] - E1[0] * E2[2],
                             E1[0] * E2[1] - E1[1] * E2[0]};
        const double nn = N[0] * N[0] + N[1] * N[1] + N[2] * N[2];
        if (!(nn > 0.0)) return;
        const double ga = (g2v[0] * N[0] + g2v[1] * N[1] + g2v[2] * N[2]) / nn;
        const double gb = (db[0] * N[0] + db[1] * N[1] + db[2] * N[2]) / nn;
        for (int a = 0; a < 3; ++a) {
            pa[a] = g2v[a] - ga * N[a];
            pb[a] = db[a] - gb * N[a];
        }
    } else {
        double e[3];
        for (int a = 0; a < 3; ++a) e[a] = on_s ? E2[a] : on_t ? E1[a] : E2[a] - E1[a];
        const double ee = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
        if (!(ee > 0.0)) return;
        const double ga = (g2v[0] * e[0] + g2v[1] * e[1] + g2v[2] * e[2]) / ee;
        const double gb = (db[0] * e[0] + db[1] * e[1] + db[2] * e[2]) / ee;
        for (int a = 0; a < 3; ++a) {
            pa[a] = ga * e[a];
            pb[a] = gb * e[a];
        }
    }
    const double bb = pb[0] * pb[0] + pb[1] * pb[1] + pb[2] * pb[2];
    if (!(bb > 1e-24)) return;
    const double al = fmin(1.0, fmax(0.0, -(pa[0] * pb[0] + pa[1] * pb[1] + pa[2] * pb[2]) / bb));
    for (int a = 0; a < 3; ++a) g[a] = g2v[a] + al * db[a];
}

// The winner's witness on its face in FP64 from the search's point (bs, bt):
// u (probe frame), f_p there and its gradient.  A (row-major) and c place body
// points in the probe frame.
__device__ void polish_witness(const double* A, const double* c, const float4& a0, const float4& a1, const float4& a2,
                               float bs, float bt, double r, double L, double* u, double& f, double* g) {
    const double b[3][3] = {{a0.x, a0.y, a0.z}, {a0.w, a1.x, a1.y}, {a1.z, a1.w, a2.x}};
    double P[3][3];
    for (int v = 0; v < 3; ++v)
        for (int a = 0; a < 3; ++a) P[v][a] = A[3 * a] * b[v][0] + A[3 * a + 1] * b[v][1] + A[3 * a + 2] * b[v][2] + c[a];
    double E1[3], E2[3], E12[3];
    for (int a = 0; a < 3; ++a) {
        E1[a] = P[1][a] - P[0][a];
        E2[a] = P[2][a] - P[0][a];
        E12[a] = P[2][a] - P[1][a];
    }
    double s = bs, t = bt;
    for (int a = 0; a < 3; ++a) u[a] = P[0][a] + s * E1[a] + t * E2[a];
    double fb = sdf64(u, r, L);
    auto take = [&](double sc, double tc) {
        if (!(sc >= 0.0 && tc >= 0.0 && sc + tc <= 1.0)) return;
        double uc[3];
        for (int a = 0; a < 3; ++a) uc[a] = P[0][a] + sc * E1[a] + tc * E2[a];
        const double fc = sdf64(uc, r, L);
        if (fc < fb) {
            fb = fc;
            s = sc;
            t = tc;
        }
    };
    if (bt == 0.0f && bs > 0.0f && bs < 1.0f) {
        double l = bs, fl = fb;
        polish_edge(P[0], E1, r, L, l, fl);
        if (fl < fb) { fb = fl; s = l; t = 0.0; }
    } else if (bs == 0.0f && bt > 0.0f && bt < 1.0f) {
        double l = bt, fl = fb;
        polish_edge(P[0], E2, r, L, l, fl);
        if (fl < fb) { fb = fl; s = 0.0; t = l; }
    } else if (bt > 0.0f && bt < 1.0f && fabsf(1.0f - bs - bt) <= 1e-6f) {
        double l = bt, fl = fb;
        polish_edge(P[1], E12, r, L, l, fl);
        if (fl < fb) { fb = fl; s = 1.0 - l; t = l; }
    } else if (bs > 0.0f && bt > 0.0f) {
        double sc, tc;
        if (polish_support(P[0], E1, E2, r, L, sc, tc)) take(sc, tc);
        // Newton on the ridge from the better of the two
        if (polish_ridge(P[0], E1, E2, s, t, r, L, sc, tc)) take(sc, tc);
        const double det = E1[0] * E2[1] - E2[0] * E1[1];  // the axis crossing the face
        if (det != 0.0) take((E2[0] * P[0][1] - P[0][0] * E2[1]) / det, (P[0][0] * E1[1] - E1[0] * P[0][1]) / det);
    }
    for (int a = 0; a < 3; ++a) u[a] = P[0][a] + s * E1[a] + t * E2[a];
    f = sdf64(u, r, L);
    witness_gradient64(u, E1, E2, s, t, r, L, g);
}

// ------------------------------------------------------------------ kernels

// zero the pair-queue counters; called by threads t = 0..63 of one block
__device__ __forceinline__ void clear_pair_counters(int* __restrict__ pair_count, int t) {
    if (t < REF_SEGS) pair_count[t * REF_SEG_STRIDE] = 0;
    if (t == 0) pair_count[REF_NESTED_AT] = 0;
}

// pose of the twist x about the start's anchor and the Jacobians the
// sensitivities need, into the trial T
__device__ void pose_at(const RefineState& S, const double* x, RefineTrial& T) {
    const double v[3] = {x[0], x[1], x[2]}, w[3] = {x[3], x[4], x[5]};
    double dR[9], V[9], Ra[3], Vv[3];
    so3_exp(w, dR);
    left_jac(w, V);
    mat3_mul(dR, S.R0, T.R);
    mat3_vec(S.R0, S.a, Ra);
    mat3_vec(V, v, Vv);
    double dRa[3];
    mat3_vec(dR, Ra, dRa);
    for (int i = 0; i < 3; ++i) {
        T.p[i] = S.p0[i] + Vv[i] + Ra[i] - dRa[i];
        T.c[i] = S.p0[i] + Vv[i] + Ra[i];
    }
    for (int i = 0; i < 9; ++i) T.V[i] = V[i];
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
        for (int i = 0; i < 3; ++i) T.D[3 * i + j] = (a[i] - b[i]) / (2 * hh);
    }
}

__global__ void k_ref_start(const double* __restrict__ init, int K, const double* __restrict__ anchor, double mu0,
                            RefineState* __restrict__ st, RefineTrial* __restrict__ tr, int* __restrict__ counters,
                            int* __restrict__ pair_count) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k == 0) {
        counters[0] = K;
        counters[1] = 0;
    }
    if (blockIdx.x == 0) clear_pair_counters(pair_count, threadIdx.x);
    if (k >= K) return;
    RefineState& S = st[k];
    const double* P = init + 7 * k;
    quat_mat(P[0], P[1], P[2], P[3], S.R0);
    for (int a = 0; a < 3; ++a) {
        S.p0[a] = P[4 + a];
        S.a[a] = anchor[a];
    }
    for (int j = 0; j < 6; ++j) S.xi[j] = 0.0;
    S.mu = mu0;
    S.it = 0;
    S.status = 0;
    // the first round evaluates xi = 0 alone
    for (int j = 0; j < REF_TMAX; ++j) tr[k * REF_TMAX + j].valid = 0;
    RefineTrial& T = tr[k * REF_TMAX];
    for (int j = 0; j < 6; ++j) T.xe[j] = T.step[j] = 0.0;
    T.mu = mu0;
    pose_at(S, T.xe, T);
    T.valid = 1;
}

// ------------------------------------------------- distance query (Sec. V-B)
//
// Per round, for every (start, trial, probe pose) query:
//   k_ref_cull     one wavefront per query: the body -> probe frame, the
//                  bounding-sphere tests down to the faces, one level of the
//                  hierarchy at a time, and per kept face the bounds ub (best
//                  vertex value) and lb (supporting planes of the convex f_p).
//                  Faces with lb above the best ub cannot hold the minimum;
//                  faces whose bounds meet are settled at their best vertex;
//                  the rest go to a pair list.
//   k_ref_pairs    one thread per (query, face) pair: the face minimum by edge
//                  searches, the support point and a lower-bound certificate,
//                  folded into the query's key (value, face index) by
//                  atomicMin, so the order of the pairs does not matter; pairs
//                  the certificate cannot settle are handed on.
//   k_ref_nested   one wavefront per handed-on pair: a parallel nested search.
//   k_ref_winner   the winning pair's witness to its query.
//   k_ref_resolve  one thread per query: the winning face placed by the FP64
//                  pose, the witness polished in FP64, the normal and the
//                  world coordinates.

// orderable 64-bit key: float value bits (monotone), then the face index
__device__ unsigned long long face_key(float v, int idx) {
    unsigned int b = __float_as_uint(v);
    b = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
    return ((unsigned long long)b << 32) | (unsigned int)idx;
}

__device__ float key_value(unsigned long long key) {
    unsigned int b = (unsigned int)(key >> 32);
    b = (b & 0x80000000u) ? (b & 0x7fffffffu) : ~b;
    return __uint_as_float(b);
}

struct FaceBounds {
    float3 u0, u1, u2;
    float lb, ub;
    int vbest;
};

// ub: the best vertex value; lb = max_j [f(v_j) + min_k g_j . (v_k - v_j)]
// (exact where f_p is linear on the face, e.g. under the flat tip disk)
__device__ FaceBounds face_bounds(const Xf& X, const float4& a0, const float4& a1, const float4& a2, float r, float L) {
    FaceBounds B;
    B.u0 = X.apply(a0.x, a0.y, a0.z);
    B.u1 = X.apply(a0.w, a1.x, a1.y);
    B.u2 = X.apply(a1.z, a1.w, a2.x);
    float3 g0, g1, g2;
    const float f0 = sdf_grad_f(B.u0, r, L, g0), f1 = sdf_grad_f(B.u1, r, L, g1), f2 = sdf_grad_f(B.u2, r, L, g2);
    const float3 d01 = make_float3(B.u1.x - B.u0.x, B.u1.y - B.u0.y, B.u1.z - B.u0.z);
    const float3 d02 = make_float3(B.u2.x - B.u0.x, B.u2.y - B.u0.y, B.u2.z - B.u0.z);
    const float3 d12 = make_float3(B.u2.x - B.u1.x, B.u2.y - B.u1.y, B.u2.z - B.u1.z);
    const float l0 = f0 + fminf(0.0f, fminf(dot3(g0, d01), dot3(g0, d02)));
    const float l1 = f1 + fminf(0.0f, fminf(-dot3(g1, d01), dot3(g1, d12)));
    const float l2 = f2 + fminf(0.0f, fminf(-dot3(g2, d02), -dot3(g2, d12)));
    B.lb = fmaxf(l0, fmaxf(l1, l2));
    B.ub = f0;
    B.vbest = 0;
    if (f1 < B.ub) { B.ub = f1; B.vbest = 1; }
    if (f2 < B.ub) { B.ub = f2; B.vbest = 2; }
    return B;
}

__device__ Tri make_tri(const FaceBounds& B, float r, float L) {
    Tri T;
    T.p0 = B.u0;
    T.e1 = make_float3(B.u1.x - B.u0.x, B.u1.y - B.u0.y, B.u1.z - B.u0.z);
    T.e2 = make_float3(B.u2.x - B.u0.x, B.u2.y - B.u0.y, B.u2.z - B.u0.z);
    T.r = r;
    T.L = L;
    return T;
}

// minimum over one face: the best vertex when the bounds meet, else golden
__device__ float face_minimum(const FaceBounds& B, const Tri& T, float& s, float& t) {
    if (B.ub - B.lb <= VERTEX_GAP) {
        s = B.vbest == 1 ? 1.0f : 0.0f;
        t = B.vbest == 2 ? 1.0f : 0.0f;
        return B.ub;
    }
    return face_min(T, s, t);
}

__device__ Xf load_xf(const float* __restrict__ xf, int q) {
    Xf X;
    for (int j = 0; j < 9; ++j) X.a[j] = xf[12 * q + j];
    for (int j = 0; j < 3; ++j) X.c[j] = xf[12 * q + 9 + j];
    return X;
}

__device__ __forceinline__ bool sphere_kept(const Xf& X, const float4& sp, float r, float L, float cull) {
    const float3 u = X.apply(sp.x, sp.y, sp.z);
    return sdf_f(u.x, u.y, u.z, r, L) < sp.w + cull;
}

// every kept face in hierarchy order: fn(slot, a0, a1, a2, a3)
template <class Fn>
__device__ void for_kept_faces(const Xf& X, const RefineGeometry& geo, float r, float L, float cull, Fn&& fn) {
    for (int tn = 0; tn < geo.n_top; ++tn) {
        if (!sphere_kept(X, geo.top[tn], r, L, cull)) continue;
        const int2 cr = geo.top_range[tn];
        for (int cl = cr.x; cl < cr.x + cr.y; ++cl) {
            if (!sphere_kept(X, geo.cluster[cl], r, L, cull)) continue;
            const int2 fr = geo.cluster_range[cl];
            for (int f = fr.x; f < fr.x + fr.y; ++f) {
                const float4 a2 = geo.face[4 * f + 2], a3 = geo.face[4 * f + 3];
                const float3 u = X.apply(a2.y, a2.z, a2.w);
                if (!(sdf_f(u.x, u.y, u.z, r, L) < a3.x + cull)) continue;
                fn(f, geo.face[4 * f], geo.face[4 * f + 1], a2, a3);
            }
        }
    }
}

__device__ void probe_frame(const float* __restrict__ poses, int i, double* Ri, double* pi) {
    const float* P = poses + 7 * i;
    quat_mat(P[0], P[1], P[2], P[3], Ri);
    pi[0] = P[4];
    pi[1] = P[5];
    pi[2] = P[6];
}

__global__ void k_ref_reset(int* __restrict__ pair_count) { clear_pair_counters(pair_count, threadIdx.x); }

// Flat view of the segmented pair queue: pre[s] = pairs in segments below s
// (each count clamped to the segment's capacity).  Every thread of the block
// must call it; the first wavefront scans.
__device__ int pair_prefix(const RefineScratch& w, int* pre) {
    if (threadIdx.x < 64) {
        const int t = threadIdx.x;
        int x = min(w.pair_count[t * REF_SEG_STRIDE], w.pair_cap / REF_SEGS);
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o, 64);
            if (t >= o) x += y;
        }
        pre[t + 1] = x;
        if (t == 0) pre[0] = 0;
    }
    __syncthreads();
    return pre[REF_SEGS];
}

// queue slot of flat index e < pre[REF_SEGS]: the segment s with pre[s] <= e < pre[s + 1]
__device__ __forceinline__ int pair_slot(const int* pre, int e, int seg_cap) {
    int lo = 0, hi = REF_SEGS;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] <= e) lo = mid;
        else hi = mid;
    }
    return lo * seg_cap + (e - pre[lo]);
}

// refinement starts from search results: rows idx[k] of a count x 7 pose array
__global__ void k_gather_poses(const int32_t* __restrict__ idx, const double* __restrict__ src, int K,
                               double* __restrict__ dst) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 7 * K) return;
    const int k = t / 7, c = t - 7 * k;
    dst[t] = src[7 * (size_t)idx[k] + c];
}

__device__ __forceinline__ float wave_min_f(float v) {
    for (int off = 32; off > 0; off >>= 1) v = fminf(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned lo = __shfl_xor((unsigned)(v & 0xffffffffu), off, 64);
        const unsigned hi = __shfl_xor((unsigned)(v >> 32), off, 64);
        const unsigned long long o = ((unsigned long long)hi << 32) | lo;
        v = o < v ? o : v;
    }
    return v;
}

constexpr int CULL_WAVES = 4;   // queries per 256-thread block, one wavefront each
constexpr int CULL_LIST = 256;  // kept faces a wavefront holds in LDS between its two passes

// LDS written by one lane of a wavefront and read by another afterwards
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// wavefront-wide list append: lanes with `keep` take consecutive positions
__device__ __forceinline__ int wave_append(bool keep, int lane, int& count) {
    const unsigned long long m = __ballot(keep);
    const int pos = count + __popcll(m & ((1ull << lane) - 1));
    count += __popcll(m);
    return pos;
}

// Kept faces of one query, spread over the lanes of its wavefront, one level
// of the hierarchy at a time: the top spheres are tested 64 at a time, the
// kept ones listed in LDS (ktop); their clusters are enumerated flat, one per
// lane, and the kept ones listed (kcl, at most 64 per step); their faces are
// enumerated flat and tested.  Each level costs one round of independent loads
// instead of one per node.  fn(lane_has_face, slot) is called by every lane at
// the same points (uniform control flow).
template <class Fn>
__device__ void wave_kept_faces(const Xf& X, const RefineGeometry& geo, float r, float L, float cull, int lane,
                                int* ktop, int* kcl, Fn&& fn) {
    for (int t0 = 0; t0 < geo.n_top; t0 += 64) {
        const int tn = t0 + lane;
        const bool tk = tn < geo.n_top && sphere_kept(X, geo.top[tn], r, L, cull);
        int nt = 0;
        const int tp = wave_append(tk, lane, nt);
        if (tk) ktop[tp] = tn;
        if (nt == 0) continue;
        wave_lds_sync();
        for (int e0 = 0; e0 < REF_FANOUT * nt; e0 += 64) {
            const int e = e0 + lane;
            int cl = -1;
            if (e < REF_FANOUT * nt) {
                const int2 cr = geo.top_range[ktop[e / REF_FANOUT]];
                const int j = e % REF_FANOUT;
                if (j < cr.y && sphere_kept(X, geo.cluster[cr.x + j], r, L, cull)) cl = cr.x + j;
            }
            int nc = 0;
            const int cp = wave_append(cl >= 0, lane, nc);
            if (cl >= 0) kcl[cp] = cl;
            if (nc == 0) continue;
            wave_lds_sync();
            for (int f0 = 0; f0 < REF_FANOUT * nc; f0 += 64) {
                const int fe = f0 + lane;
                bool has = false;
                int f = 0;
                if (fe < REF_FANOUT * nc) {
                    const int2 fr = geo.cluster_range[kcl[fe / REF_FANOUT]];
                    const int j = fe % REF_FANOUT;
                    if (j < fr.y) {
                        f = fr.x + j;
                        const float4 a2 = geo.face[4 * f + 2], a3 = geo.face[4 * f + 3];
                        const float3 u = X.apply(a2.y, a2.z, a2.w);
                        has = sdf_f(u.x, u.y, u.z, r, L) < a3.x + cull;
                    }
                }
                fn(has, f);
            }
            wave_lds_sync();  // kcl is rewritten by the next step
        }
        wave_lds_sync();      // and ktop by the next chunk of top nodes
    }
}

// queue pair (q, f) for lanes with `need` in segment seg (one atomic per wavefront)
__device__ __forceinline__ void push_pairs(bool need, int lane, int q, int f, int seg, const RefineScratch& w,
                                           bool& overflow) {
    const unsigned long long nm = __ballot(need);
    if (!nm) return;
    const int leader = __ffsll((long long)nm) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(&w.pair_count[seg * REF_SEG_STRIDE], __popcll(nm));
    base = __shfl(base, leader, 64);
    if (need) {
        const int seg_cap = w.pair_cap / REF_SEGS;
        const int off = base + __popcll(nm & ((1ull << lane) - 1));
        if (off < seg_cap) w.pairs[seg * seg_cap + off] = make_int2(q, f);
        else overflow = true;
    }
}

__global__ __launch_bounds__(64 * CULL_WAVES) void k_ref_cull(const RefineTrial* __restrict__ tr, int K,
                                                              RefineGeometry geo, const float* __restrict__ poses,
                                                              int N, RefineConst c, RefineScratch w,
                                                              int* __restrict__ active) {
    __shared__ int l_slot[CULL_WAVES][CULL_LIST], l_idx[CULL_WAVES][CULL_LIST];
    __shared__ float l_lb[CULL_WAVES][CULL_LIST], l_ub[CULL_WAVES][CULL_LIST];
    __shared__ int l_queue[CULL_WAVES][128];
    __shared__ int l_ktop[CULL_WAVES][64], l_kcl[CULL_WAVES][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int q = blockIdx.x * CULL_WAVES + wv;
    if (blockIdx.x == 0 && threadIdx.x == 0) active[0] = 0;  // counted again by k_ref_decide
    if (q >= K * N) return;  // whole wavefronts
    const int k = q / N, i = q - k * N;
    const RefineTrial& S = tr[k];
    if (!S.valid) return;
    const int seg = blockIdx.x % REF_SEGS;
    double Ri[9], pi[3];
    probe_frame(poses, i, Ri, pi);
    Xf X;
    for (int a = 0; a < 3; ++a) {
        for (int b = 0; b < 3; ++b)
            X.a[3 * a + b] = (float)(Ri[a] * S.R[b] + Ri[3 + a] * S.R[3 + b] + Ri[6 + a] * S.R[6 + b]);
        X.c[a] = (float)(Ri[a] * (S.p[0] - pi[0]) + Ri[3 + a] * (S.p[1] - pi[1]) + Ri[6 + a] * (S.p[2] - pi[2]));
    }
    float xv = 0.0f;  // constant indices keep X in registers
#pragma unroll
    for (int j = 0; j < 12; ++j)
        if (lane == j) xv = j < 9 ? X.a[j] : X.c[j - 9];
    if (lane < 12) w.xf[12 * q + lane] = xv;
    if (lane == 0) w.qst[q] = make_float2(-1.0f, -1.0f);
    const float r = c.r, L = c.L;

    // pass 1: the bounds of every kept face; the best vertex value.  Kept
    // faces queue up in LDS and their bounds are taken 64 at a time, one per
    // lane.  A face whose lb exceeds its lane's best ub so far (never below
    // the final best) cannot hold the minimum; the others are listed for
    // pass 2.
    float run_ub = INFINITY;
    bool any = false;
    int n_list = 0, n_q = 0;
    auto bounds_of_queue = [&](int count) {
        FaceBounds B{};
        bool keep = false;
        int f = 0, idx = 0;
        if (lane < count) {
            f = l_queue[wv][lane];
            const float4 a0 = geo.face[4 * f], a1 = geo.face[4 * f + 1], a2 = geo.face[4 * f + 2];
            idx = __float_as_int(geo.face[4 * f + 3].y);
            B = face_bounds(X, a0, a1, a2, r, L);
            run_ub = fminf(run_ub, B.ub);
            keep = B.lb <= run_ub + BOUND_SLACK;
        }
        const int pos = wave_append(keep, lane, n_list);
        if (keep && pos < CULL_LIST) {
            l_slot[wv][pos] = f;
            l_idx[wv][pos] = idx;
            l_lb[wv][pos] = B.lb;
            l_ub[wv][pos] = B.ub;
        }
    };
    wave_kept_faces(X, geo, r, L, c.cull, lane, l_ktop[wv], l_kcl[wv], [&](bool has, int f) {
        any |= has;
        const int pos = wave_append(has, lane, n_q);  // n_q < 128 after the append
        if (has) l_queue[wv][pos] = f;
        if (n_q >= 64) {
            wave_lds_sync();
            bounds_of_queue(64);
            const int rest = n_q - 64;
            const int mv = lane < rest ? l_queue[wv][64 + lane] : 0;
            wave_lds_sync();
            if (lane < rest) l_queue[wv][lane] = mv;
            n_q = rest;
        }
    });
    if (n_q > 0) {
        wave_lds_sync();
        bounds_of_queue(n_q);
    }
    if (!__ballot(any)) {
        if (lane == 0) {
            w.qkey[q] = ~0ull;
            w.qflag[q] = 0;
        }
        return;
    }
    const float best_ub = wave_min_f(run_ub);

    // pass 2: settle faces whose bounds meet; queue the others for a search
    unsigned long long best = ~0ull;
    bool overflow = false;
    if (n_list <= CULL_LIST) {
        wave_lds_sync();
        for (int j0 = 0; j0 < n_list; j0 += 64) {
            const int j = j0 + lane;
            bool need = false;
            int f = 0;
            if (j < n_list) {
                const float lb = l_lb[wv][j], ub = l_ub[wv][j];
                f = l_slot[wv][j];
                if (lb <= best_ub + BOUND_SLACK) {
                    if (ub - lb <= VERTEX_GAP) {
                        const unsigned long long key = face_key(ub, l_idx[wv][j]);
                        best = key < best ? key : best;
                    } else {
                        need = true;
                    }
                }
            }
            push_pairs(need, lane, q, f, seg, w, overflow);
        }
    } else {
        // the list overflowed: walk the kept faces again
        wave_kept_faces(X, geo, r, L, c.cull, lane, l_ktop[wv], l_kcl[wv], [&](bool has, int f) {
                            bool need = false;
                            if (has) {
                                const FaceBounds B = face_bounds(X, geo.face[4 * f], geo.face[4 * f + 1],
                                                                 geo.face[4 * f + 2], r, L);
                                if (B.lb <= best_ub + BOUND_SLACK) {
                                    if (B.ub - B.lb <= VERTEX_GAP) {
                                        const unsigned long long key =
                                            face_key(B.ub, __float_as_int(geo.face[4 * f + 3].y));
                                        best = key < best ? key : best;
                                    } else {
                                        need = true;
                                    }
                                }
                            }
                            push_pairs(need, lane, q, f, seg, w, overflow);
                        });
    }
    best = wave_min_u64(best);
    const bool ovf = __ballot(overflow) != 0;
    if (lane == 0) {
        w.qkey[q] = best;
        w.qflag[q] = ovf ? 2 : 1;
    }
}

__global__ __launch_bounds__(256) void k_ref_pairs(RefineGeometry geo, RefineConst c, RefineScratch w) {
    __shared__ int pre[REF_SEGS + 1];
    const int n = pair_prefix(w, pre), seg_cap = w.pair_cap / REF_SEGS;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const int j = pair_slot(pre, e, seg_cap);
        const int2 pr = w.pairs[j];
        const Xf X = load_xf(w.xf, pr.x);
        const int f = pr.y;
        const FaceBounds B = face_bounds(X, geo.face[4 * f], geo.face[4 * f + 1], geo.face[4 * f + 2], c.r, c.L);
        float s, t;
        bool done;
        const float m = face_min_bounded(make_tri(B, c.r, c.L), s, t, done);
        w.pres[j] = make_float4(m, s, t, 0.0f);
        if (done) {
            atomicMin(&w.qkey[pr.x], face_key(m, __float_as_int(geo.face[4 * f + 3].y)));
        } else {
            // a few percent of the pairs, left to k_ref_nested with the
            // boundary minimum in pres
            w.nest[atomicAdd(&w.pair_count[REF_NESTED_AT], 1)] = j;
        }
    }
}

// (v, i) of the least v over aligned groups of `width` lanes, the lowest i on ties
__device__ __forceinline__ void group_argmin(float& v, int& i, int first_mask, int width) {
    for (int m = first_mask; m < first_mask * width; m <<= 1) {
        const float ov = __shfl_xor(v, m, 64);
        const int oi = __shfl_xor(i, m, 64);
        if (ov < v || (ov == v && oi < i)) {
            v = ov;
            i = oi;
        }
    }
}

constexpr int NSEC = 8;     // points per bracket of the parallel searches
constexpr int NSEC_IT = 8;  // (2 / (NSEC + 1))^NSEC_IT = 6e-6 of the bracket is left

// The face minimum of a deferred pair inside the face, one wavefront per
// pair: f is convex, so is its partial minimum over t.  Eight groups of eight
// lanes evaluate the partial minimum at NSEC points of the s bracket, each by
// NSEC-section over t; the bracket then shrinks to the neighbours of the best
// point (for a unimodal function the minimum lies between them).  The best
// point evaluated is folded with the boundary minimum k_ref_pairs left in
// pres.
__global__ __launch_bounds__(64) void k_ref_nested(RefineGeometry geo, RefineConst c, RefineScratch w) {
    const int n = w.pair_count[REF_NESTED_AT];
    const int lane = threadIdx.x, grp = lane >> 3, sub = lane & 7;
    for (int e = blockIdx.x; e < n; e += gridDim.x) {
        const int j = w.nest[e];
        const int2 pr = w.pairs[j];
        const Xf X = load_xf(w.xf, pr.x);
        const int f = pr.y;
        const FaceBounds B = face_bounds(X, geo.face[4 * f], geo.face[4 * f + 1], geo.face[4 * f + 2], c.r, c.L);
        const Tri T = make_tri(B, c.r, c.L);
        float bv = INFINITY, bs = 0.0f, bt = 0.0f;  // this lane's best evaluation
        float sa = 0.0f, sb = 1.0f;
        for (int io = 0; io < NSEC_IT; ++io) {
            const float hs = (sb - sa) * (1.0f / (NSEC + 1));
            const float sv = sa + hs * (float)(grp + 1);
            float ta = 0.0f, tb = 1.0f - sv, phi = INFINITY;
            for (int ii = 0; ii < NSEC_IT; ++ii) {
                const float ht = (tb - ta) * (1.0f / (NSEC + 1));
                const float tv = ta + ht * (float)(sub + 1);
                float v = T.at(sv, tv);
                if (v < bv) {
                    bv = v; bs = sv; bt = tv;
                }
                int im = sub;
                group_argmin(v, im, 1, NSEC);
                phi = fminf(phi, v);
                ta = ta + ht * (float)im;
                tb = ta + 2.0f * ht;
            }
            int ig = grp;
            group_argmin(phi, ig, NSEC, 64 / NSEC);
            sa = sa + hs * (float)ig;
            sb = sa + 2.0f * hs;
        }
        int il = lane;
        float v = bv;
        group_argmin(v, il, 1, 64);
        const float ws = __shfl(bs, il, 64), wt = __shfl(bt, il, 64);
        if (lane == 0) {
            float4 cur = w.pres[j];  // the boundary minimum
            if (v < cur.x) cur = make_float4(v, ws, wt, 0.0f);
            w.pres[j] = cur;
            atomicMin(&w.qkey[pr.x], face_key(cur.x, __float_as_int(geo.face[4 * f + 3].y)));
        }
    }
}

// the pair that holds its query's minimum hands over its barycentric witness
__global__ __launch_bounds__(256) void k_ref_winner(RefineGeometry geo, RefineScratch w) {
    __shared__ int pre[REF_SEGS + 1];
    const int n = pair_prefix(w, pre), seg_cap = w.pair_cap / REF_SEGS;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const int j = pair_slot(pre, e, seg_cap);
        const int2 pr = w.pairs[j];
        const float4 res = w.pres[j];
        if (face_key(res.x, __float_as_int(geo.face[4 * pr.y + 3].y)) == w.qkey[pr.x])
            w.qst[pr.x] = make_float2(res.y, res.z);
    }
}

__global__ __launch_bounds__(64) void k_ref_resolve(const RefineTrial* __restrict__ tr, int K, RefineGeometry geo,
                                                    const float* __restrict__ poses, int N, RefineConst c,
                                                    RefineScratch w, RefineHit* __restrict__ hits) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= K * N) return;
    const int k = q / N, i = q - k * N;
    if (!tr[k].valid) return;
    RefineHit out;
    // the face that holds the best vertex value always passes the bounds test,
    // so a query with kept faces has a key; an empty key is treated as none kept
    const int flag = w.qflag[q] == 1 && w.qkey[q] == ~0ull ? 0 : w.qflag[q];
    if (flag == 0) {
        out.dx = make_float4(c.eps, 0.0f, 0.0f, 0.0f);
        out.nf = make_float4(0.0f, 0.0f, 0.0f, __int_as_float(-1));
        hits[q] = out;
        return;
    }
    const Xf X = load_xf(w.xf, q);
    const float r = c.r, L = c.L;
    float best = INFINITY, bs = 0.0f, bt = 0.0f;
    int bidx = 0x7fffffff;
    Tri BT{};
    if (flag == 2) {
        // the pair list overflowed: search this query's faces here
        float best_ub = INFINITY;
        for_kept_faces(X, geo, r, L, c.cull, [&](int, const float4& a0, const float4& a1, const float4& a2, const float4&) {
            best_ub = fminf(best_ub, face_bounds(X, a0, a1, a2, r, L).ub);
        });
        for_kept_faces(X, geo, r, L, c.cull, [&](int, const float4& a0, const float4& a1, const float4& a2, const float4& a3) {
            const FaceBounds B = face_bounds(X, a0, a1, a2, r, L);
            if (B.lb > best_ub + BOUND_SLACK) return;
            const Tri T = make_tri(B, r, L);
            float s, t;
            const float m = face_minimum(B, T, s, t);
            const int idx = __float_as_int(a3.y);
            if (m < best || (m == best && idx < bidx)) {
                best = m; bidx = idx; bs = s; bt = t; BT = T;
            }
        });
    } else {
        const unsigned long long key = w.qkey[q];
        bidx = (int)(unsigned int)(key & 0xffffffffu);
        best = key_value(key);
        const int f = geo.slot_of[bidx];
        const FaceBounds B = face_bounds(X, geo.face[4 * f], geo.face[4 * f + 1], geo.face[4 * f + 2], r, L);
        BT = make_tri(B, r, L);
        const float2 st2 = w.qst[q];
        if (st2.x >= 0.0f) {  // found by a golden-section search
            bs = st2.x;
            bt = st2.y;
        } else {              // settled at the face's best vertex
            bs = B.vbest == 1 ? 1.0f : 0.0f;
            bt = B.vbest == 2 ? 1.0f : 0.0f;
        }
    }
    double Ri[9], pi[3];
    probe_frame(poses, i, Ri, pi);
    double u64[3], f64;
    double xw[3], nw[3];
    // beyond tau_out2 s, s' and s'' vanish: the float32 witness serves
    const bool found = bidx >= 0 && bidx < geo.n_faces && best < (float)c.tau_out2 + 1e-4f;
    const int fs = found ? geo.slot_of[bidx] : 0;
    double g[3];
    if (found) {
        // body -> probe frame in FP64
        const RefineTrial& P = tr[k];
        double A[9], cc[3];
        for (int a = 0; a < 3; ++a) {
            for (int b = 0; b < 3; ++b) A[3 * a + b] = Ri[a] * P.R[b] + Ri[3 + a] * P.R[3 + b] + Ri[6 + a] * P.R[6 + b];
            cc[a] = Ri[a] * (P.p[0] - pi[0]) + Ri[3 + a] * (P.p[1] - pi[1]) + Ri[6 + a] * (P.p[2] - pi[2]);
        }
        polish_witness(A, cc, geo.face[4 * fs], geo.face[4 * fs + 1], geo.face[4 * fs + 2], bs, bt, c.r64, c.L64, u64,
                       f64, g);
        for (int a = 0; a < 3; ++a) {
            xw[a] = Ri[3 * a] * u64[0] + Ri[3 * a + 1] * u64[1] + Ri[3 * a + 2] * u64[2] + pi[a];
            nw[a] = Ri[3 * a] * g[0] + Ri[3 * a + 1] * g[1] + Ri[3 * a + 2] * g[2];
        }
        best = (float)f64;
    } else {
        const float3 u = make_float3(BT.p0.x + bs * BT.e1.x + bt * BT.e2.x, BT.p0.y + bs * BT.e1.y + bt * BT.e2.y,
                                     BT.p0.z + bs * BT.e1.z + bt * BT.e2.z);
        const float3 gl = witness_gradient(u, BT, bs, bt);
        for (int a = 0; a < 3; ++a) {
            xw[a] = Ri[3 * a] * u.x + Ri[3 * a + 1] * u.y + Ri[3 * a + 2] * u.z + pi[a];
            nw[a] = Ri[3 * a] * gl.x + Ri[3 * a + 1] * gl.y + Ri[3 * a + 2] * gl.z;
        }
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

constexpr int RED_T = 64;
constexpr int NACC = 28;  // J, grad (6), H upper triangle (21)

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

// REF_EVAL_PARTS blocks per valid trial slot, each a fixed range of probe
// poses: -sum s, -sum s' g and the curvature sum max(0, -s'') g g^T in FP64,
// lane sums added in lane order.  counters[1] counts the evaluations.
__global__ __launch_bounds__(RED_T) void k_ref_eval(const RefineTrial* __restrict__ tr, const RefineHit* __restrict__ hits,
                                                   int N, RefineConst c, RefineEval* __restrict__ ev,
                                                   int* __restrict__ counters) {
    const int k = blockIdx.x / REF_EVAL_PARTS, part = blockIdx.x % REF_EVAL_PARTS;
    const RefineTrial& S = tr[k];
    if (!S.valid) return;
    __shared__ double red[NACC][RED_T];
    double V[9], D[9], cc[3];
    for (int j = 0; j < 9; ++j) {
        V[j] = S.V[j];
        D[j] = S.D[j];
    }
    for (int j = 0; j < 3; ++j) cc[j] = S.c[j];
    double acc[NACC];
    for (int j = 0; j < NACC; ++j) acc[j] = 0.0;
    const int chunk = (N + REF_EVAL_PARTS - 1) / REF_EVAL_PARTS;
    const int i1 = min(N, (part + 1) * chunk);
    for (int i = part * chunk + threadIdx.x; i < i1; i += RED_T) {
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
    if (threadIdx.x < NACC) {
        double t = 0.0;
        for (int l = 0; l < RED_T; ++l) t += red[threadIdx.x][l];
        reinterpret_cast<double*>(&ev[blockIdx.x])[threadIdx.x] = t;
    }
    if (part == 0 && threadIdx.x == 0) atomicAdd(&counters[1], 1);
}

// The evaluations of start k's trials: their partial sums in part order, plus
// lambda |xi|^2 and its derivatives (all threads of the block take part).
__device__ void gather_trial_evals(const RefineTrial* __restrict__ tr, const RefineEval* __restrict__ ev, int k,
                                   const RefineConst& c, RefineEval* Es) {
    for (int t = threadIdx.x; t < REF_TMAX * NACC; t += blockDim.x) {
        const int j = t / NACC, a = t % NACC;
        const RefineTrial& T = tr[k * REF_TMAX + j];
        if (!T.valid) continue;
        double v = 0.0;
        for (int p = 0; p < REF_EVAL_PARTS; ++p)
            v += reinterpret_cast<const double*>(&ev[(k * REF_TMAX + j) * REF_EVAL_PARTS + p])[a];
        if (a == 0) {
            double xx = 0.0;
            for (int q = 0; q < 6; ++q) xx += T.xe[q] * T.xe[q];
            v += c.lambda * xx;
        } else if (a < 7) {
            v += 2 * c.lambda * T.xe[a - 1];
        } else {
            int o = a - 7, r = 0;  // upper-triangle index o -> row r, diagonal when o hits its start
            while (o >= 6 - r) {
                o -= 6 - r;
                ++r;
            }
            if (o == 0) v += 2 * c.lambda;
        }
        reinterpret_cast<double*>(&Es[j])[a] = v;
    }
}

// Trial step with damping mu from (xi, g, H): a coordinate at its bound whose
// gradient points out of the box is held there (its row and column replaced
// by the identity, its right-hand side zero); false if the system is not
// positive definite.
__device__ bool trial_step(const RefineState& S, double mu, const RefineConst& c, RefineTrial& T) {
    bool act[6];
    for (int j = 0; j < 6; ++j) {
        const double b = j < 3 ? c.b_t : c.b_r;
        act[j] = (S.xi[j] >= b - 1e-12 && S.g[j] < 0) || (S.xi[j] <= -b + 1e-12 && S.g[j] > 0);
    }
    double A[36], rhs[6], step[6];
    for (int a = 0; a < 6; ++a) {
        for (int b = 0; b < 6; ++b) A[6 * a + b] = (act[a] || act[b]) ? 0.0 : S.H[6 * a + b];
        A[6 * a + a] = act[a] ? 1.0 : A[6 * a + a] + mu * S.H[6 * a + a] + 1e-12;
        rhs[a] = act[a] ? 0.0 : -S.g[a];
    }
    if (!chol6(A, rhs, step)) return false;
    for (int j = 0; j < 6; ++j) {
        T.step[j] = step[j];
        T.xe[j] = clampd(S.xi[j] + step[j], j < 3 ? c.b_t : c.b_r);
    }
    T.mu = mu;
    return true;
}

// One block per start (REF_TMAX or more threads).  Thread 0 replays the
// damped Gauss-Newton decisions over the evaluated trials in the order the
// sequential iteration would try them: the first trial that lowers J is
// taken (mu = max(mu / 3, 1e-12)); a rejected trial multiplies mu by 3 and
// ends the start when mu reaches 1e12 or its step was below tol_step.  An
// accepted step below tol_step taken with a damping of at most 10 mu0 ends the
// start; otherwise the projected-gradient test and the iteration cap apply.
// Then the block's threads set up the next round's trials in parallel: one
// after a first-try acceptance, two after an acceptance that needed a
// rejection, REF_TMAX after a round of rejections.
__global__ void k_ref_decide(RefineState* __restrict__ st, RefineTrial* __restrict__ tr,
                             const RefineEval* __restrict__ ev, RefineConst c, int* __restrict__ pair_count,
                             int* __restrict__ counters) {
    const int k = blockIdx.x;
    if (k == 0) clear_pair_counters(pair_count, threadIdx.x);  // for the next round's queries
    RefineState& S = st[k];
    if (S.status == 2) return;
    __shared__ int ntrial;
    __shared__ RefineEval Es[REF_TMAX];
    gather_trial_evals(tr, ev, k, c, Es);
    __syncthreads();
    if (threadIdx.x == 0) {
        int next = 0;
        int taken = -1;
        bool stop = false;
        double mu_next = S.mu;
        for (int j = 0; j < REF_TMAX; ++j) {
            const RefineTrial& T = tr[k * REF_TMAX + j];
            if (!T.valid) break;
            const RefineEval& E = Es[j];
            if (S.status == 0 || E.J < S.J) {
                taken = j;
                break;
            }
            mu_next = 3.0 * T.mu;
            if (mu_next >= 1e12 || maxabs6(T.step) <= c.tol_step) {
                stop = true;
                break;
            }
        }
        if (taken >= 0) {
            const RefineTrial& T = tr[k * REF_TMAX + taken];
            const RefineEval& E = Es[taken];
            const bool first = S.status == 0;
            for (int j = 0; j < 6; ++j) {
                S.xi[j] = T.xe[j];
                S.g[j] = E.g[j];
            }
            S.J = E.J;
            int o = 0;
            for (int a = 0; a < 6; ++a)
                for (int b = a; b < 6; ++b, ++o) S.H[6 * a + b] = S.H[6 * b + a] = E.H[o];
            if (!first) S.mu = fmax(T.mu / 3.0, 1e-12);
            S.status = 1;
            // a small step ends the start only when it was taken with little
            // damping: a heavily damped step is small because mu is large,
            // not because the iterate is near the minimum
            if (!first && maxabs6(T.step) <= c.tol_step && T.mu <= 10.0 * c.mu0) {
                S.status = 2;
            } else {
                double pg = 0;
                for (int j = 0; j < 6; ++j) {
                    const double b = j < 3 ? c.b_t : c.b_r;
                    pg = fmax(pg, fabs(S.xi[j] - clampd(S.xi[j] - S.g[j], b)));
                }
                if (pg <= c.tol_pg || S.it >= c.max_iters) {
                    S.status = 2;
                } else {
                    S.it += 1;
                    next = taken == 0 ? 1 : 2;
                }
            }
        } else if (stop || !tr[k * REF_TMAX].valid) {
            S.status = 2;    // (no valid trial: no positive-definite system was left)
        } else {
            S.mu = mu_next;  // every trial of the round was rejected
            next = REF_TMAX;
        }
        ntrial = next;
        if (next > 0) atomicAdd(&counters[0], 1);
    }
    __syncthreads();
    if (threadIdx.x < REF_TMAX) {
        RefineTrial& T = tr[k * REF_TMAX + threadIdx.x];
        T.valid = 0;
        if ((int)threadIdx.x < ntrial) {
            double mu = S.mu;
            for (unsigned j = 0; j < threadIdx.x; ++j) mu *= 3.0;
            if (mu < 1e12 && trial_step(S, mu, c, T)) {
                pose_at(S, T.xe, T);
                T.valid = 1;
            }
        }
    }
}

// ------------------------------------------------- L-BFGS-B (Sec. V-C)
//
// The paper's solver on the same objective and gradient.  With six variables
// the limited-memory matrix is formed explicitly: B = theta I updated by the
// BFGS formula with the stored pairs, oldest first (theta = y'y / s'y of the
// newest pair).  An iteration takes the generalised Cauchy point of the
// quadratic model along the projected-gradient path x(t) = P(x - t g), then
// minimises the model over the variables still free there (Cholesky of their
// block of B) and truncates that step to the box; the direction is
// p = x_bar - x.  The line search backtracks from step 1 (1/|p| at the first
// iteration) by halving and takes the first step length that meets the
// sufficient decrease J <= J0 + 1e-4 lam g.p.  After an accepted step the
// next round evaluates the unit step alone (taken most of the time); once a
// round finds no decrease, the following ones evaluate four halvings each.
// A pair enters the memory when s'y > eps y'y.  The iteration stops on a
// projected gradient below tol_pg, a relative decrease of J below 1e-10,
// max_iters steps, or a line search that finds no decrease (32 halvings) even
// from steepest descent.

__device__ __forceinline__ double dot6(const double* a, const double* b) {
    double t = 0.0;
    for (int j = 0; j < 6; ++j) t += a[j] * b[j];
    return t;
}

__device__ __forceinline__ void matvec6(const double* A, const double* v, double* o) {
    for (int i = 0; i < 6; ++i) o[i] = dot6(A + 6 * i, v);
}

__device__ double projected_gradient(const RefineState& S, const RefineConst& c) {
    double pg = 0;
    for (int j = 0; j < 6; ++j) {
        const double b = j < 3 ? c.b_t : c.b_r;
        pg = fmax(pg, fabs(S.xi[j] - clampd(S.xi[j] - S.g[j], b)));
    }
    return pg;
}

__device__ void lbfgsb_direction(const RefineState& S, LbfgsState& L, const RefineConst& c) {
    const double* x = S.xi;
    const double* g = S.g;
    double lo[6], hi[6];
    for (int j = 0; j < 6; ++j) {
        hi[j] = j < 3 ? c.b_t : c.b_r;
        lo[j] = -hi[j];
    }
    // the limited-memory matrix
    double B[36];
    double theta = 1.0;
    if (L.npairs > 0) {
        const int nw = (L.head + LBFGS_M - 1) % LBFGS_M;
        theta = dot6(L.Y[nw], L.Y[nw]) / dot6(L.S[nw], L.Y[nw]);
    }
    for (int i = 0; i < 36; ++i) B[i] = (i % 7 == 0) ? theta : 0.0;
    for (int q = 0; q < L.npairs; ++q) {
        const int idx = (L.head - L.npairs + q + 2 * LBFGS_M) % LBFGS_M;
        const double* sv = L.S[idx];
        const double* yv = L.Y[idx];
        double Bs[6];
        matvec6(B, sv, Bs);
        const double sBs = dot6(sv, Bs), ys = dot6(yv, sv);
        if (!(sBs > 0.0 && ys > 0.0)) continue;
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j) B[6 * i + j] += yv[i] * yv[j] / ys - Bs[i] * Bs[j] / sBs;
    }
    // generalised Cauchy point: breakpoints of the projected path in order
    double tb[6], d[6], z[6];
    int ord[6];
    for (int i = 0; i < 6; ++i) {
        tb[i] = g[i] < 0.0 ? (x[i] - hi[i]) / g[i] : g[i] > 0.0 ? (x[i] - lo[i]) / g[i] : INFINITY;
        d[i] = tb[i] > 0.0 ? -g[i] : 0.0;
        z[i] = 0.0;
        ord[i] = i;
    }
    for (int i = 1; i < 6; ++i)
        for (int j = i; j > 0 && tb[ord[j]] < tb[ord[j - 1]]; --j) {
            const int t = ord[j];
            ord[j] = ord[j - 1];
            ord[j - 1] = t;
        }
    double tprev = 0.0;
    for (int q = 0; q <= 6; ++q) {
        if (q < 6 && d[ord[q]] == 0.0) continue;  // at its bound from the start (or g = 0)
        double Bz[6], Bd[6];
        matvec6(B, z, Bz);
        matvec6(B, d, Bd);
        const double fp = dot6(g, d) + dot6(d, Bz), fpp = dot6(d, Bd);
        if (!(fp < 0.0)) break;  // the model no longer decreases along the path
        const double tnext = q < 6 ? tb[ord[q]] : INFINITY;
        const double dtmin = fpp > 0.0 ? -fp / fpp : INFINITY;
        if (dtmin < tnext - tprev) {
            for (int i = 0; i < 6; ++i) z[i] += dtmin * d[i];
            break;
        }
        if (!(tnext < INFINITY)) break;
        for (int i = 0; i < 6; ++i) z[i] += (tnext - tprev) * d[i];
        const int b = ord[q];
        z[b] = (d[b] > 0.0 ? hi[b] : lo[b]) - x[b];
        d[b] = 0.0;
        tprev = tnext;
    }
    // subspace step on the variables free at the Cauchy point
    double xc[6], r[6], A[36], rhs[6], du[6];
    bool fr[6];
    for (int i = 0; i < 6; ++i) {
        xc[i] = fmin(hi[i], fmax(lo[i], x[i] + z[i]));
        fr[i] = xc[i] > lo[i] && xc[i] < hi[i];
        z[i] = xc[i] - x[i];
    }
    matvec6(B, z, r);
    for (int i = 0; i < 6; ++i) {
        r[i] += g[i];
        rhs[i] = fr[i] ? -r[i] : 0.0;
        for (int j = 0; j < 6; ++j) A[6 * i + j] = (fr[i] && fr[j]) ? B[6 * i + j] : (i == j ? 1.0 : 0.0);
    }
    double xbar[6];
    for (int i = 0; i < 6; ++i) xbar[i] = xc[i];
    if (chol6(A, rhs, du)) {
        double alpha = 1.0;
        for (int i = 0; i < 6; ++i) {
            if (!fr[i]) continue;
            if (du[i] > 0.0) alpha = fmin(alpha, (hi[i] - xc[i]) / du[i]);
            else if (du[i] < 0.0) alpha = fmin(alpha, (lo[i] - xc[i]) / du[i]);
        }
        for (int i = 0; i < 6; ++i)
            if (fr[i]) xbar[i] = xc[i] + alpha * du[i];
    }
    for (int i = 0; i < 6; ++i) L.p[i] = xbar[i] - x[i];
    L.gp = dot6(g, L.p);
    if (!(L.gp < 0.0)) {
        // not a descent direction: drop the memory, projected steepest descent
        L.npairs = 0;
        for (int i = 0; i < 6; ++i) L.p[i] = fmin(hi[i], fmax(lo[i], x[i] - g[i])) - x[i];
        L.gp = dot6(g, L.p);
    }
}

__global__ void k_ref_decide_lbfgsb(RefineState* __restrict__ st, LbfgsState* __restrict__ lb,
                                    RefineTrial* __restrict__ tr, const RefineEval* __restrict__ ev, RefineConst c,
                                    int* __restrict__ pair_count, int* __restrict__ counters) {
    const int k = blockIdx.x;
    if (k == 0) clear_pair_counters(pair_count, threadIdx.x);  // for the next round's queries
    RefineState& S = st[k];
    if (S.status == 2) return;
    __shared__ RefineEval Es[REF_TMAX];
    __shared__ int ntrial;
    gather_trial_evals(tr, ev, k, c, Es);
    __syncthreads();
    LbfgsState& L = lb[k];
    if (threadIdx.x == 0) {
        constexpr double C1 = 1e-4, FTOL = 1e-10;
        constexpr int MAX_HALVINGS = 32;
        bool stop = false;
        int next = REF_TMAX;  // step lengths for the next round
        if (S.status == 0) {
            // the start's evaluation at xi = 0
            S.J = Es[0].J;
            for (int j = 0; j < 6; ++j) S.g[j] = Es[0].g[j];
            S.it = 0;
            L.npairs = 0;
            L.head = 0;
            L.nback = 0;
            L.fprev = INFINITY;
            if (projected_gradient(S, c) <= c.tol_pg) {
                stop = true;
            } else {
                lbfgsb_direction(S, L, c);
                L.lam0 = fmin(1.0, 1.0 / sqrt(dot6(L.p, L.p)));
            }
        } else {
            int taken = -1;
            for (int j = 0; j < REF_TMAX; ++j) {
                const RefineTrial& T = tr[k * REF_TMAX + j];
                if (!T.valid) break;
                if (Es[j].J <= S.J + C1 * T.mu * L.gp) {
                    taken = j;
                    break;
                }
            }
            if (taken >= 0) {
                const RefineTrial& T = tr[k * REF_TMAX + taken];
                double sv[6], yv[6];
                for (int j = 0; j < 6; ++j) {
                    sv[j] = T.xe[j] - S.xi[j];
                    yv[j] = Es[taken].g[j] - S.g[j];
                }
                if (dot6(sv, yv) > 2.220446049250313e-16 * dot6(yv, yv)) {
                    for (int j = 0; j < 6; ++j) {
                        L.S[L.head][j] = sv[j];
                        L.Y[L.head][j] = yv[j];
                    }
                    L.head = (L.head + 1) % LBFGS_M;
                    L.npairs = min(L.npairs + 1, LBFGS_M);
                }
                L.fprev = S.J;
                S.J = Es[taken].J;
                for (int j = 0; j < 6; ++j) {
                    S.xi[j] = T.xe[j];
                    S.g[j] = Es[taken].g[j];
                }
                S.it += 1;
                L.nback = 0;
                if (projected_gradient(S, c) <= c.tol_pg ||
                    L.fprev - S.J <= FTOL * fmax(fmax(fabs(L.fprev), fabs(S.J)), 1.0) || S.it >= c.max_iters) {
                    stop = true;
                } else {
                    lbfgsb_direction(S, L, c);
                    L.lam0 = 1.0;
                    // the unit step is taken most of the time: try it alone,
                    // and four halvings only once it fails
                    next = 1;
                }
            } else {
                for (int j = 0; j < L.ntr; ++j) L.lam0 *= 0.5;  // continue the halving
                L.nback += L.ntr;
                if (L.nback > MAX_HALVINGS) {
                    if (L.npairs > 0) {
                        L.npairs = 0;
                        lbfgsb_direction(S, L, c);
                        L.lam0 = fmin(1.0, 1.0 / sqrt(dot6(L.p, L.p)));
                        L.nback = 0;
                    } else {
                        stop = true;
                    }
                }
            }
        }
        S.status = stop ? 2 : 1;
        ntrial = stop ? 0 : next;
        L.ntr = stop ? 0 : next;
        if (!stop) atomicAdd(&counters[0], 1);
    }
    __syncthreads();
    if (threadIdx.x < REF_TMAX) {
        RefineTrial& T = tr[k * REF_TMAX + threadIdx.x];
        T.valid = 0;
        if ((int)threadIdx.x < ntrial) {
            double lam = L.lam0;
            for (unsigned j = 0; j < threadIdx.x; ++j) lam *= 0.5;
            for (int j = 0; j < 6; ++j) {
                const double b = j < 3 ? c.b_t : c.b_r;
                T.xe[j] = clampd(S.xi[j] + lam * L.p[j], b);
                T.step[j] = T.xe[j] - S.xi[j];
            }
            T.mu = lam;
            pose_at(S, T.xe, T);
            T.valid = 1;
        }
    }
}

__global__ void k_ref_finish(const RefineState* __restrict__ st, int K, double* __restrict__ out_poses,
                             double* __restrict__ out_J, int32_t* __restrict__ out_iters) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    const RefineState& S = st[k];
    RefineTrial T;
    pose_at(S, S.xi, T);
    const double* R = T.R;
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
    o[4] = T.p[0]; o[5] = T.p[1]; o[6] = T.p[2];
    if (out_J) out_J[k] = S.J;
    if (out_iters) out_iters[k] = S.it;
}

}  // namespace

hipError_t refine_start(const double* init_poses, int K, const double* anchor, const RefineConst& c, RefineState* st,
                        RefineTrial* tr, int* counters, const RefineScratch& w, hipStream_t s) {
    k_ref_start<<<(K + 63) / 64, 64, 0, s>>>(init_poses, K, anchor, c.mu0, st, tr, counters, w.pair_count);
    return hipGetLastError();
}

// distance queries of `slots` trial poses x N probe poses: cull, pair
// searches, winners, resolve
static void launch_queries(const RefineTrial* tr, int slots, const RefineGeometry& geo, const float* poses, int N,
                           const RefineConst& c, const RefineScratch& w, RefineHit* hits, int* counters,
                           hipStream_t s) {
    const long long q = (long long)slots * N;
    k_ref_cull<<<(unsigned)((q + CULL_WAVES - 1) / CULL_WAVES), 64 * CULL_WAVES, 0, s>>>(tr, slots, geo, poses, N, c,
                                                                                      w, counters);
    // about 3 searches per query are needed; the kernels stride over the rest
    const unsigned pb = (unsigned)std::min<long long>(2048, std::max<long long>(1, (4 * q + 255) / 256));
    k_ref_pairs<<<pb, 256, 0, s>>>(geo, c, w);
    k_ref_nested<<<4096, 64, 0, s>>>(geo, c, w);
    k_ref_winner<<<pb, 256, 0, s>>>(geo, w);
    k_ref_resolve<<<(unsigned)((q + 63) / 64), 64, 0, s>>>(tr, slots, geo, poses, N, c, w, hits);
}

hipError_t refine_round(RefineState* st, RefineTrial* tr, int K, const RefineGeometry& geo, const float* poses,
                        int n_poses, const RefineConst& c, const RefineScratch& w, RefineHit* hits, RefineEval* ev,
                        int* counters, hipStream_t s) {
    const int slots = K * REF_TMAX;
    launch_queries(tr, slots, geo, poses, n_poses, c, w, hits, counters, s);
    k_ref_eval<<<slots * REF_EVAL_PARTS, RED_T, 0, s>>>(tr, hits, n_poses, c, ev, counters);
    k_ref_decide<<<K, 64, 0, s>>>(st, tr, ev, c, w.pair_count, counters);
    return hipGetLastError();
}

hipError_t refine_round_lbfgsb(RefineState* st, LbfgsState* lb, RefineTrial* tr, int K, const RefineGeometry& geo,
                               const float* poses, int n_poses, const RefineConst& c, const RefineScratch& w,
                               RefineHit* hits, RefineEval* ev, int* counters, hipStream_t s) {
    const int slots = K * REF_TMAX;
    launch_queries(tr, slots, geo, poses, n_poses, c, w, hits, counters, s);
    k_ref_eval<<<slots * REF_EVAL_PARTS, RED_T, 0, s>>>(tr, hits, n_poses, c, ev, counters);
    k_ref_decide_lbfgsb<<<K, 64, 0, s>>>(st, lb, tr, ev, c, w.pair_count, counters);
    return hipGetLastError();
}

hipError_t refine_finish(const RefineState* st, int K, double* out_poses, double* out_J, int32_t* out_iters,
                         hipStream_t s) {
    k_ref_finish<<<(K + 63) / 64, 64, 0, s>>>(st, K, out_poses, out_J, out_iters);
    return hipGetLastError();
}

hipError_t refine_query_only(const RefineTrial* tr, const RefineGeometry& geo, const float* poses, int n_poses,
                             const RefineConst& c, const RefineScratch& w, RefineHit* hits, int* counters,
                             hipStream_t s) {
    k_ref_reset<<<1, 64, 0, s>>>(w.pair_count);
    launch_queries(tr, 1, geo, poses, n_poses, c, w, hits, counters, s);
    return hipGetLastError();
}

hipError_t gather_poses(const int32_t* idx, const double* src, int K, double* dst, hipStream_t s) {
    k_gather_poses<<<(7 * K + 63) / 64, 64, 0, s>>>(idx, src, K, dst);
    return hipGetLastError();
}
