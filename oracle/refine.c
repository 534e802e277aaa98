/*
 * FP64 reference distance queries for the SE(3) refinement (Sec. V-B).
 *
 * TEST INFRASTRUCTURE ONLY: part of the CPU oracle, loaded by the tests, the
 * smoke check and the benchmark's CPU-baseline leg; it shares no code with the
 * HIP path.
 *
 * For every probe pose T_i the query returns the smallest signed distance d_i
 * between the probe (SDF f_p in its frame) and the object mesh placed by
 * (R, p), the witness point x* on the object (world) and the outward unit
 * normal n_i of f_p there (world).  Faces are kept when f_p at their
 * centroid is below their bounding radius plus eps (the paper's bounding-sphere
 * test); with no face left, d_i = eps.  On each kept face f_p is minimised
 * exactly up to a parameter tolerance: f_p is convex (the SDF of a convex
 * body) and so is its restriction to the triangle, whose partial minimum over
 * one barycentric coordinate is convex in the other -- nested golden-section
 * searches converge to the minimum.  Ties keep the lowest face index.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

static double probe_sdf(const double *u, double r, double L)
{
    double q1 = sqrt(u[0] * u[0] + u[1] * u[1]) - r;
    double q2 = fabs(u[2] - 0.5 * L) - 0.5 * L;
    double in = fmin(fmax(q1, q2), 0.0);
    double a = fmax(q1, 0.0), b = fmax(q2, 0.0);
    return in + sqrt(a * a + b * b);
}

/* gradient of the capped-cylinder SDF (a subgradient on its ridges) */
static void probe_grad(const double *u, double r, double L, double *g)
{
    double rho = sqrt(u[0] * u[0] + u[1] * u[1]);
    double q1 = rho - r, q2 = fabs(u[2] - 0.5 * L) - 0.5 * L;
    double e1[3] = {1.0, 0.0, 0.0};
    if (rho > 0) { e1[0] = u[0] / rho; e1[1] = u[1] / rho; }
    double sz = u[2] >= 0.5 * L ? 1.0 : -1.0;
    if (q1 <= 0 && q2 <= 0) {
        if (q1 >= q2) { g[0] = e1[0]; g[1] = e1[1]; g[2] = 0; }
        else { g[0] = 0; g[1] = 0; g[2] = sz; }
        return;
    }
    double a = fmax(q1, 0.0), b = fmax(q2, 0.0);
    double n = sqrt(a * a + b * b);
    g[0] = a * e1[0] / n; g[1] = a * e1[1] / n; g[2] = b * sz / n;
}

/* Sensitivity direction at the witness u = p0 + s (p1 - p0) + t (p2 - p0).
 * Where f_p is differentiable it is grad f_p.  Inside the probe, on the ridge
 * where the side wall and an end cap are equally near (q1 = q2 within
 * RIDGE_TOL), the face minimum is a min-max of the two branches and its
 * derivative is g = a grad q1 + (1 - a) grad q2, with a in [0, 1] chosen so
 * that g has no component along the directions in which the witness can move
 * (the face plane for an interior witness, the edge for an edge witness).  At a
 * vertex witness, or when those directions do not fix a, the one-sided
 * gradient is kept.  A witness within EDGE_TOL (barycentric) of an edge counts
 * as on it: at an interior minimum the combination has no component along any
 * face direction, the edge's included, so the edge gives the same a. */
#define RIDGE_TOL 1e-4
#define EDGE_TOL 1e-4
static void witness_gradient(const double *u, const double *p0, const double *p1, const double *p2, double s,
                             double t, double r, double L, double *g)
{
    double rho = sqrt(u[0] * u[0] + u[1] * u[1]);
    double q1 = rho - r, q2 = fabs(u[2] - 0.5 * L) - 0.5 * L;
    probe_grad(u, r, L, g);
    if (!(q1 <= 0 && q2 <= 0 && fabs(q1 - q2) <= RIDGE_TOL && rho > 0)) return;
    int on_s = s <= EDGE_TOL, on_t = t <= EDGE_TOL, on_st = 1.0 - s - t <= EDGE_TOL;
    int active = on_s + on_t + on_st;
    if (active >= 2) return;
    double g1[3] = {u[0] / rho, u[1] / rho, 0.0};
    double g2[3] = {0.0, 0.0, u[2] >= 0.5 * L ? 1.0 : -1.0};
    double db[3] = {g1[0] - g2[0], g1[1] - g2[1], g1[2] - g2[2]};
    double e1[3], e2[3], a[3], b[3];
    for (int k = 0; k < 3; k++) { e1[k] = p1[k] - p0[k]; e2[k] = p2[k] - p0[k]; }
    if (active == 0) {
        /* project onto the face plane */
        double N[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        double nn = N[0] * N[0] + N[1] * N[1] + N[2] * N[2];
        if (!(nn > 0)) return;
        double ga = (g2[0] * N[0] + g2[1] * N[1] + g2[2] * N[2]) / nn;
        double gb = (db[0] * N[0] + db[1] * N[1] + db[2] * N[2]) / nn;
        for (int k = 0; k < 3; k++) { a[k] = g2[k] - ga * N[k]; b[k] = db[k] - gb * N[k]; }
    } else {
        /* project onto the active edge */
        double e[3];
        for (int k = 0; k < 3; k++) e[k] = on_s ? e2[k] : on_t ? e1[k] : e2[k] - e1[k];
        double ee = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
        if (!(ee > 0)) return;
        double ga = (g2[0] * e[0] + g2[1] * e[1] + g2[2] * e[2]) / ee;
        double gb = (db[0] * e[0] + db[1] * e[1] + db[2] * e[2]) / ee;
        for (int k = 0; k < 3; k++) { a[k] = ga * e[k]; b[k] = gb * e[k]; }
    }
    double bb = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    if (!(bb > 1e-24)) return;
    double alpha = -(a[0] * b[0] + a[1] * b[1] + a[2] * b[2]) / bb;
    alpha = fmin(1.0, fmax(0.0, alpha));
    for (int k = 0; k < 3; k++) g[k] = g2[k] + alpha * db[k];
}

static const double INVPHI = 0.6180339887498949;   /* (sqrt 5 - 1) / 2 */

typedef struct { double p0[3], e1[3], e2[3], r, L; } Tri;

static double tri_f(const Tri *T, double s, double t)
{
    double u[3];
    for (int k = 0; k < 3; k++) u[k] = T->p0[k] + s * T->e1[k] + t * T->e2[k];
    return probe_sdf(u, T->r, T->L);
}

/* min over t in [0, tmax] of f(s, t) by golden section; returns the value and t */
static double inner_min(const Tri *T, double s, double tmax, double tol, double *t_out)
{
    double a = 0.0, b = tmax;
    double c = b - INVPHI * (b - a), d = a + INVPHI * (b - a);
    double fc = tri_f(T, s, c), fd = tri_f(T, s, d);
    while (b - a > tol) {
        if (fc <= fd) { b = d; d = c; fd = fc; c = b - INVPHI * (b - a); fc = tri_f(T, s, c); }
        else { a = c; c = d; fc = fd; d = a + INVPHI * (b - a); fd = tri_f(T, s, d); }
    }
    /* the bracket's ends are candidates too (minimum on the boundary) */
    double tm = 0.5 * (a + b), fm = tri_f(T, s, tm);
    double f0 = tri_f(T, s, 0.0), f1 = tri_f(T, s, tmax);
    if (f0 < fm) { fm = f0; tm = 0.0; }
    if (f1 < fm) { fm = f1; tm = tmax; }
    *t_out = tm;
    return fm;
}

/* min over the triangle p0 + s e1 + t e2 (s, t >= 0, s + t <= 1) */
double orc_face_min(const double *p0, const double *p1, const double *p2, double r, double L, double tol,
                    double *s_out, double *t_out)
{
    Tri T;
    for (int k = 0; k < 3; k++) { T.p0[k] = p0[k]; T.e1[k] = p1[k] - p0[k]; T.e2[k] = p2[k] - p0[k]; }
    T.r = r; T.L = L;
    double a = 0.0, b = 1.0, tt;
    double c = b - INVPHI * (b - a), d = a + INVPHI * (b - a);
    double fc = inner_min(&T, c, 1.0 - c, tol, &tt), fd = inner_min(&T, d, 1.0 - d, tol, &tt);
    while (b - a > tol) {
        if (fc <= fd) { b = d; d = c; fd = fc; c = b - INVPHI * (b - a); fc = inner_min(&T, c, 1.0 - c, tol, &tt); }
        else { a = c; c = d; fc = fd; d = a + INVPHI * (b - a); fd = inner_min(&T, d, 1.0 - d, tol, &tt); }
    }
    double sm = 0.5 * (a + b), tm;
    double fm = inner_min(&T, sm, 1.0 - sm, tol, &tm);
    double t0, t1;
    double f0 = inner_min(&T, 0.0, 1.0, tol, &t0), f1 = inner_min(&T, 1.0, 0.0, tol, &t1);
    if (f0 < fm) { fm = f0; sm = 0.0; tm = t0; }
    if (f1 < fm) { fm = f1; sm = 1.0; tm = t1; }
    *s_out = sm;
    *t_out = tm;
    return fm;
}

/* Distance queries of all poses for the object at (R, p).  R row-major.
 * face_c: body-frame centroids (nf x 3), face_r: bounding radii about them. */
void orc_distance_query(const float *V, const int32_t *F, int nf, const double *face_c, const double *face_r,
                        const double *R, const double *p, const float *poses, int np, double r, double L,
                        double eps, double tol, double *d_out, double *x_out, double *n_out, int32_t *face_out)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < np; i++) {
        const float *P = poses + 7 * i;
        double qn = sqrt((double)P[0] * P[0] + (double)P[1] * P[1] + (double)P[2] * P[2] + (double)P[3] * P[3]);
        double w = P[0] / qn, x = P[1] / qn, y = P[2] / qn, z = P[3] / qn;
        double Ri[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                        2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                        2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
        double pi[3] = {P[4], P[5], P[6]};
        /* body point b -> probe frame: Ri^T (R b + p - pi) = A b + c */
        double A[9], c[3];
        for (int a = 0; a < 3; a++) {
            for (int bb = 0; bb < 3; bb++) {
                double s = 0;
                for (int k = 0; k < 3; k++) s += Ri[3 * k + a] * R[3 * k + bb];
                A[3 * a + bb] = s;
            }
            double s = 0;
            for (int k = 0; k < 3; k++) s += Ri[3 * k + a] * (p[k] - pi[k]);
            c[a] = s;
        }
        double best = INFINITY, bs = 0, bt = 0;
        int bf = -1;
        double bu[3][3];
        for (int f = 0; f < nf; f++) {
            double cu[3];
            for (int a = 0; a < 3; a++)
                cu[a] = A[3 * a] * face_c[3 * f] + A[3 * a + 1] * face_c[3 * f + 1] + A[3 * a + 2] * face_c[3 * f + 2] + c[a];
            if (!(probe_sdf(cu, r, L) < face_r[f] + eps)) continue;
            double u[3][3];
            for (int v = 0; v < 3; v++) {
                int vi = F[3 * f + v];
                double b0 = V[3 * vi], b1 = V[3 * vi + 1], b2 = V[3 * vi + 2];
                for (int a = 0; a < 3; a++) u[v][a] = A[3 * a] * b0 + A[3 * a + 1] * b1 + A[3 * a + 2] * b2 + c[a];
            }
            double s, t;
            double m = orc_face_min(u[0], u[1], u[2], r, L, tol, &s, &t);
            if (m < best) {
                best = m; bf = f; bs = s; bt = t;
                for (int v = 0; v < 3; v++)
                    for (int a = 0; a < 3; a++) bu[v][a] = u[v][a];
            }
        }
        face_out[i] = bf;
        if (bf < 0) {
            d_out[i] = eps;
            for (int a = 0; a < 3; a++) { x_out[3 * i + a] = 0; n_out[3 * i + a] = 0; }
            continue;
        }
        d_out[i] = best;
        double u[3], g[3];
        for (int a = 0; a < 3; a++) u[a] = bu[0][a] + bs * (bu[1][a] - bu[0][a]) + bt * (bu[2][a] - bu[0][a]);
        witness_gradient(u, bu[0], bu[1], bu[2], bs, bt, r, L, g);
        for (int a = 0; a < 3; a++) {
            /* world = Ri u + pi ; normal = Ri g */
            x_out[3 * i + a] = Ri[3 * a] * u[0] + Ri[3 * a + 1] * u[1] + Ri[3 * a + 2] * u[2] + pi[a];
            n_out[3 * i + a] = Ri[3 * a] * g[0] + Ri[3 * a + 1] * g[1] + Ri[3 * a + 2] * g[2];
        }
    }
}
