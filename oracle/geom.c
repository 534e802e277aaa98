/*
 * FP64 reference geometry for the swept-contact docking search.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is part of the CPU oracle: only the
 * test-suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it.  It shares no code with the HIP path.
 *
 * Plain loops in double precision; every function states the passage of the
 * paper it follows.  Geometry arrives as float32 (vertices, poses) and is
 * widened to double before any arithmetic.
 *
 *   orc_probe_sdf        probe SDF f_p of a flat-ended cylinder (Sec. IV-A,
 *                        swept occupancy; Sec. V-B distance queries)
 *   orc_object_points    object grid value O(x) = min(O_t, O_m) at arbitrary
 *                        points, brute force over every face (Sec. IV-A,
 *                        banded template, surface mask, element-wise min)
 *   orc_object_grid      the same values on the n^3 canvas, with the face loop
 *                        restricted to faces whose box, grown by the band,
 *                        contains the point (exact inside the band) and the
 *                        inside test done by +z ray crossing parity
 *   orc_swept_points     min_i f_p(T_i^{-1} y) at arbitrary points (Sec. IV-A,
 *                        swept occupancy S = max_i H(.)), brute force
 *   orc_swept_lattice    the same on the m^3 world lattice, each pose visiting
 *                        only the lattice points of its grown bounding box
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_INF (1.0 / 0.0)

/* ---------------------------------------------------------------- probe */

/* Exact Euclidean SDF of the capped cylinder {x^2+y^2 <= r^2, 0 <= z <= L},
 * negative inside.  The tip disk is centred at the local origin, axis +z. */
double orc_probe_sdf(double x, double y, double z, double r, double L)
{
    double q1 = sqrt(x * x + y * y) - r;
    double q2 = fabs(z - 0.5 * L) - 0.5 * L;
    double in = fmin(fmax(q1, q2), 0.0);
    double a = fmax(q1, 0.0), b = fmax(q2, 0.0);
    return in + sqrt(a * a + b * b);
}

/* Rotation matrix (row-major) of the normalised quaternion (w,x,y,z). */
static void quat_mat(const double q_in[4], double R[9])
{
    double n = sqrt(q_in[0] * q_in[0] + q_in[1] * q_in[1] + q_in[2] * q_in[2] + q_in[3] * q_in[3]);
    double w = q_in[0] / n, x = q_in[1] / n, y = q_in[2] / n, z = q_in[3] / n;
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* f_p(T^{-1} y) for the pose T = (R(q), p). */
static double probe_sdf_world(const double R[9], const double p[3], double r, double L,
                              double yx, double yy, double yz)
{
    double dx = yx - p[0], dy = yy - p[1], dz = yz - p[2];
    /* local = R^T (y - p) */
    double lx = R[0] * dx + R[3] * dy + R[6] * dz;
    double ly = R[1] * dx + R[4] * dy + R[7] * dz;
    double lz = R[2] * dx + R[5] * dy + R[8] * dz;
    return orc_probe_sdf(lx, ly, lz, r, L);
}

/* --------------------------------------------------------------- meshes */

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void sub3(const double *a, const double *b, double *o) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }
static void cross3(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/* Squared distance from p to the closest point of triangle abc, by the
 * Voronoi-region case analysis of Ericson, "Real-Time Collision Detection",
 * Sec. 5.1.5. */
double orc_point_tri_dist2(const double *p, const double *a, const double *b, const double *c)
{
    double ab[3], ac[3], ap[3], bp[3], cp[3], q[3], d[3];
    sub3(b, a, ab); sub3(c, a, ac); sub3(p, a, ap);
    double d1 = dot3(ab, ap), d2 = dot3(ac, ap);
    if (d1 <= 0 && d2 <= 0) { sub3(p, a, d); return dot3(d, d); }
    sub3(p, b, bp);
    double d3 = dot3(ab, bp), d4 = dot3(ac, bp);
    if (d3 >= 0 && d4 <= d3) { sub3(p, b, d); return dot3(d, d); }
    double vc = d1 * d4 - d3 * d2;
    if (vc <= 0 && d1 >= 0 && d3 <= 0) {
        double v = d1 / (d1 - d3);
        for (int i = 0; i < 3; i++) q[i] = a[i] + v * ab[i];
        sub3(p, q, d); return dot3(d, d);
    }
    sub3(p, c, cp);
    double d5 = dot3(ab, cp), d6 = dot3(ac, cp);
    if (d6 >= 0 && d5 <= d6) { sub3(p, c, d); return dot3(d, d); }
    double vb = d5 * d2 - d1 * d6;
    if (vb <= 0 && d2 >= 0 && d6 <= 0) {
        double w = d2 / (d2 - d6);
        for (int i = 0; i < 3; i++) q[i] = a[i] + w * ac[i];
        sub3(p, q, d); return dot3(d, d);
    }
    double va = d3 * d6 - d5 * d4;
    if (va <= 0 && (d4 - d3) >= 0 && (d5 - d6) >= 0) {
        double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
        for (int i = 0; i < 3; i++) q[i] = b[i] + w * (c[i] - b[i]);
        sub3(p, q, d); return dot3(d, d);
    }
    double den = 1.0 / (va + vb + vc);
    double v = vb * den, w = vc * den;
    for (int i = 0; i < 3; i++) q[i] = a[i] + ab[i] * v + ac[i] * w;
    sub3(p, q, d);
    return dot3(d, d);
}

/* Signed solid angle of triangle abc seen from p (Van Oosterom & Strackee,
 * IEEE TBME 1983).  Summed over a closed outward mesh it is 4*pi inside and 0
 * outside: the generalised winding number times 4*pi. */
double orc_solid_angle(const double *p, const double *a, const double *b, const double *c)
{
    double ra[3], rb[3], rc[3], x[3];
    sub3(a, p, ra); sub3(b, p, rb); sub3(c, p, rc);
    double la = sqrt(dot3(ra, ra)), lb = sqrt(dot3(rb, rb)), lc = sqrt(dot3(rc, rc));
    cross3(rb, rc, x);
    double num = dot3(ra, x);
    double den = la * lb * lc + dot3(ra, rb) * lc + dot3(ra, rc) * lb + dot3(rb, rc) * la;
    return 2.0 * atan2(num, den);
}

/* The banded template O_t of the signed distance f_o, the surface mask O_m
 * of the touchable distance d, and their element-wise minimum (Sec. IV-A).
 * rho is the magnitude of the deep-penetration penalty: deep points get -rho. */
static double object_value(double fo, double dt, double tau_out1, double tau_in1, double rho)
{
    double ot;
    if (fo >= 0 && fo < tau_out1) ot = 1.0 - fo / tau_out1;
    else if (fo < 0 && fo > -tau_in1) ot = 1.0 + fo / tau_in1;
    else if (fo <= -tau_in1) ot = -rho;
    else ot = 0.0;
    double om = fmax(0.0, 1.0 - fabs(dt) / tau_out1);
    return fmin(ot, om);
}

static void vert(const float *V, int i, double *o) { o[0] = V[3 * i]; o[1] = V[3 * i + 1]; o[2] = V[3 * i + 2]; }

/* Brute force over every face: O(x), f_o(x) and d(x) at each point.
 * The inside test is the generalised winding number >= 1/2. */
void orc_object_points(const float *V, int nv, const int32_t *F, int nf, const uint8_t *touch,
                       const double *pts, int npts, double tau_out1, double tau_in1, double rho,
                       double *out_O, double *out_fo, double *out_d)
{
    (void)nv;
    for (int i = 0; i < npts; i++) {
        const double *p = pts + 3 * i;
        double dmin = ORC_INF, dtmin = ORC_INF, omega = 0.0;
        for (int f = 0; f < nf; f++) {
            double a[3], b[3], c[3];
            vert(V, F[3 * f], a); vert(V, F[3 * f + 1], b); vert(V, F[3 * f + 2], c);
            double d2 = orc_point_tri_dist2(p, a, b, c);
            if (d2 < dmin) dmin = d2;
            if ((!touch || touch[f]) && d2 < dtmin) dtmin = d2;
            omega += orc_solid_angle(p, a, b, c);
        }
        dmin = sqrt(dmin);
        dtmin = sqrt(dtmin);
        int inside = omega / (4.0 * M_PI) >= 0.5;
        double fo = inside ? -dmin : dmin;
        if (out_fo) out_fo[i] = fo;
        if (out_d) out_d[i] = dtmin;
        out_O[i] = object_value(fo, dtmin, tau_out1, tau_in1, rho);
    }
}

/* 2D orientation of p against the directed edge a->b, with p displaced by
 * (eps, eps^2) for an infinitesimal eps (simulation of simplicity), so that a
 * ray through a shared edge or vertex is counted by exactly one face. */
static int orient_sos(double ax, double ay, double bx, double by, double px, double py)
{
    double o = (bx - ax) * (py - ay) - (by - ay) * (px - ax);
    if (o > 0) return 1;
    if (o < 0) return -1;
    if (by != ay) return (ay - by) > 0 ? 1 : -1;
    if (bx != ax) return (bx - ax) > 0 ? 1 : -1;
    return 0;
}

/* Full canvas x_k = a + h (k - n/2), flat index (kz*n + ky)*n + kx.
 * Distances are exact wherever they are below `band`; elsewhere they are
 * reported as +inf.  Inside/outside by +z ray crossing parity, which equals the
 * winding-number test for a closed, consistently oriented mesh. */
void orc_object_grid(const float *V, int nv, const int32_t *F, int nf, const uint8_t *touch,
                     int n, double h, const double *anchor, double tau_out1, double tau_in1,
                     double rho, double band, double *out_O, double *out_fo, double *out_d)
{
    (void)nv;
    size_t N3 = (size_t)n * n * n;
    double *dmin = (double *)malloc(N3 * sizeof(double));
    double *dtmin = (double *)malloc(N3 * sizeof(double));
    uint8_t *par = (uint8_t *)calloc(N3, 1);
    for (size_t i = 0; i < N3; i++) { dmin[i] = ORC_INF; dtmin[i] = ORC_INF; }
    double half = 0.5 * n;
    for (int f = 0; f < nf; f++) {
        double a[3], b[3], c[3];
        vert(V, F[3 * f], a); vert(V, F[3 * f + 1], b); vert(V, F[3 * f + 2], c);
        int lo[3], hi[3];
        for (int j = 0; j < 3; j++) {
            double mn = fmin(a[j], fmin(b[j], c[j])) - band, mx = fmax(a[j], fmax(b[j], c[j])) + band;
            lo[j] = (int)ceil((mn - anchor[j]) / h + half);
            hi[j] = (int)floor((mx - anchor[j]) / h + half);
            if (lo[j] < 0) lo[j] = 0;
            if (hi[j] > n - 1) hi[j] = n - 1;
        }
        int tf = !touch || touch[f];
        for (int kz = lo[2]; kz <= hi[2]; kz++)
            for (int ky = lo[1]; ky <= hi[1]; ky++)
                for (int kx = lo[0]; kx <= hi[0]; kx++) {
                    double p[3] = {anchor[0] + h * (kx - half), anchor[1] + h * (ky - half), anchor[2] + h * (kz - half)};
                    double d2 = orc_point_tri_dist2(p, a, b, c);
                    size_t id = ((size_t)kz * n + ky) * n + kx;
                    if (d2 < dmin[id]) dmin[id] = d2;
                    if (tf && d2 < dtmin[id]) dtmin[id] = d2;
                }
        /* crossing parity: every column whose (x,y) falls in the projected face */
        int clo[2], chi[2];
        for (int j = 0; j < 2; j++) {
            double mn = fmin(a[j], fmin(b[j], c[j])), mx = fmax(a[j], fmax(b[j], c[j]));
            clo[j] = (int)floor((mn - anchor[j]) / h + half);
            chi[j] = (int)ceil((mx - anchor[j]) / h + half);
            if (clo[j] < 0) clo[j] = 0;
            if (chi[j] > n - 1) chi[j] = n - 1;
        }
        for (int ky = clo[1]; ky <= chi[1]; ky++)
            for (int kx = clo[0]; kx <= chi[0]; kx++) {
                double px = anchor[0] + h * (kx - half), py = anchor[1] + h * (ky - half);
                int s1 = orient_sos(a[0], a[1], b[0], b[1], px, py);
                int s2 = orient_sos(b[0], b[1], c[0], c[1], px, py);
                int s3 = orient_sos(c[0], c[1], a[0], a[1], px, py);
                if (!((s1 > 0 && s2 > 0 && s3 > 0) || (s1 < 0 && s2 < 0 && s3 < 0))) continue;
                double w1 = (b[0] - a[0]) * (py - a[1]) - (b[1] - a[1]) * (px - a[0]); /* weight of c */
                double w2 = (c[0] - b[0]) * (py - b[1]) - (c[1] - b[1]) * (px - b[0]); /* weight of a */
                double w3 = (a[0] - c[0]) * (py - c[1]) - (a[1] - c[1]) * (px - c[0]); /* weight of b */
                double tot = w1 + w2 + w3;
                double zi = (w2 * a[2] + w3 * b[2] + w1 * c[2]) / tot;
                for (int kz = 0; kz < n; kz++) {
                    double pz = anchor[2] + h * (kz - half);
                    if (pz < zi) par[((size_t)kz * n + ky) * n + kx] ^= 1;
                }
            }
    }
    for (size_t i = 0; i < N3; i++) {
        double dm = sqrt(dmin[i]), dt = sqrt(dtmin[i]);
        double fo = par[i] ? -dm : dm;
        if (out_fo) out_fo[i] = fo;
        if (out_d) out_d[i] = dt;
        out_O[i] = object_value(fo, dt, tau_out1, tau_in1, rho);
    }
    free(dmin); free(dtmin); free(par);
}

/* ------------------------------------------------------- swept volume */

/* min_i f_p(T_i^{-1} y) over all poses, at arbitrary points. Poses are rows
 * (qw qx qy qz tx ty tz) mapping probe-local coordinates to world. */
void orc_swept_points(const float *poses, int N, double r, double L,
                      const double *pts, int npts, double *out_minf)
{
    double *Rs = (double *)malloc((size_t)N * 9 * sizeof(double));
    for (int i = 0; i < N; i++) {
        double q[4] = {poses[7 * i], poses[7 * i + 1], poses[7 * i + 2], poses[7 * i + 3]};
        quat_mat(q, Rs + 9 * i);
    }
    for (int k = 0; k < npts; k++) {
        double best = ORC_INF;
        for (int i = 0; i < N; i++) {
            double p[3] = {poses[7 * i + 4], poses[7 * i + 5], poses[7 * i + 6]};
            double f = probe_sdf_world(Rs + 9 * i, p, r, L, pts[3 * k], pts[3 * k + 1], pts[3 * k + 2]);
            if (f < best) best = f;
        }
        out_minf[k] = best;
    }
    free(Rs);
}

/* The world lattice y_j = wc + h (j - m/2), flat index (jz*m + jy)*m + jx.
 * Each pose visits the lattice points of the cylinder's bounding box grown by
 * `margin`; points outside every box keep +inf (f_p > margin there). */
void orc_swept_lattice(const float *poses, int N, double r, double L, int m, double h,
                       const double *wc, double margin, double *out_minf)
{
    size_t M3 = (size_t)m * m * m;
    for (size_t i = 0; i < M3; i++) out_minf[i] = ORC_INF;
    double half = 0.5 * m;
    for (int i = 0; i < N; i++) {
        double q[4] = {poses[7 * i], poses[7 * i + 1], poses[7 * i + 2], poses[7 * i + 3]};
        double R[9];
        quat_mat(q, R);
        double p[3] = {poses[7 * i + 4], poses[7 * i + 5], poses[7 * i + 6]};
        double ax[3] = {R[2], R[5], R[8]}; /* probe axis in world */
        int lo[3], hi[3];
        for (int j = 0; j < 3; j++) {
            double e = r * sqrt(fmax(0.0, 1.0 - ax[j] * ax[j])) + margin;
            double c0 = p[j], c1 = p[j] + L * ax[j];
            double mn = fmin(c0, c1) - e, mx = fmax(c0, c1) + e;
            lo[j] = (int)ceil((mn - wc[j]) / h + half);
            hi[j] = (int)floor((mx - wc[j]) / h + half);
            if (lo[j] < 0) lo[j] = 0;
            if (hi[j] > m - 1) hi[j] = m - 1;
        }
        for (int jz = lo[2]; jz <= hi[2]; jz++)
            for (int jy = lo[1]; jy <= hi[1]; jy++)
                for (int jx = lo[0]; jx <= hi[0]; jx++) {
                    double f = probe_sdf_world(R, p, r, L, wc[0] + h * (jx - half),
                                               wc[1] + h * (jy - half), wc[2] + h * (jz - half));
                    size_t id = ((size_t)jz * m + jy) * m + jx;
                    if (f < out_minf[id]) out_minf[id] = f;
                }
    }
}
