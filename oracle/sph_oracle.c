/*
 * sph_oracle.c -- plain FP64 CPU oracle of the SPHaptics SPH step.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this file.  It shares no code, header,
 * table or constant with the HIP library; the two meet only in the seeded
 * scene arrays.
 *
 * What it computes (arXiv 2511.15908, Sec. 3.1 Alg. 1, Eqs. kernel / density /
 * pressure / euler; Sec. 3.2 typed particles, rigid point forces and springs;
 * Sec. 3.3 grabbed body and rolling average), written as the plain
 * definitions: every neighbour set is explicit, every sum runs over the
 * neighbours in ascending particle id, all physics arithmetic is binary64.
 * The only binary32 arithmetic is the pair of integer decisions (the cell
 * coordinate of a particle and the neighbour predicate) when the run is an
 * FP32 run: those are evaluated in binary32 exactly as defined below so that
 * both sides of a comparison take the same decision in the same precision.
 *
 * Readings of points the paper leaves open (each is listed in the design
 * notes): support radius 2h (the kernel equation), alpha_3 = 3/(2 pi h^3),
 * symmetric (Monaghan) pressure term, Brookshaw/Morris viscosity with
 * eps = 0.01 h^2, boundary volumes psi_b = rho0 / sum_same_object W (Akinci
 * style, cited in Sec. 2.1), pressure mirroring at boundaries, no force
 * between two boundary particles.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fno-fast-math -shared -fPIC
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_FLUID 0
#define ORC_SOFT 1
#define ORC_BOUNDARY 2

#define ORC_CLAMP_NEG_PRESSURE 1u
#define ORC_BOUNDARY_SINGLE_TERM 2u
#define ORC_NO_BOUNDARY_VISCOSITY 4u
#define ORC_UNIFIED_BOUNDARY 8u

typedef struct {
    int32_t precision; /* 0: decisions in binary32, 1: decisions in binary64 */
    uint32_t flags;
    double h, rho0, k, nu;
    double g[3];
    double dt;
    double lo[3], hi[3];
} orc_params;

typedef struct {
    int32_t dims[3];
    int32_t bits;      /* Morton bits per axis */
    double cs;         /* cell size */
    double inv_cs64;
    float inv_cs32;
    float lo32[3];
    float R2_32;
    double R2_64;
} orc_grid;

/* ------------------------------------------------------------------ */
/* Cubic spline kernel (Eq. kernel), support 2h, 3-D normalisation.     */
/* ------------------------------------------------------------------ */

double orc_alpha3(double h) { return 3.0 / (2.0 * M_PI * h * h * h); }

double orc_W(double r, double h)
{
    double q = r / h;
    double a = orc_alpha3(h);
    if (q < 1.0) return a * (2.0 / 3.0 - q * q + 0.5 * q * q * q);
    if (q < 2.0) {
        double t = 2.0 - q;
        return a * t * t * t / 6.0;
    }
    return 0.0;
}

/* dW/dr of the same kernel */
double orc_dWdr(double r, double h)
{
    double q = r / h;
    double a = orc_alpha3(h);
    if (q < 1.0) return a / h * (-2.0 * q + 1.5 * q * q);
    if (q < 2.0) {
        double t = 2.0 - q;
        return -a / h * 0.5 * t * t;
    }
    return 0.0;
}

/* ------------------------------------------------------------------ */
/* Uniform grid (Alg. 2, spatial hash over a uniform grid; Sec. 3.1).  */
/* Cell size = 2h (1 + 2^-10); cell coordinate                         */
/*   c = clamp(floor((x - lo) * inv_cs), 0, D - 1)                     */
/* with both roundings in the run's precision.                         */
/* ------------------------------------------------------------------ */

void orc_grid_setup(const orc_params *p, orc_grid *g)
{
    double R = 2.0 * p->h;
    g->cs = R * (1.0 + 1.0 / 1024.0);
    int maxd = 1;
    for (int a = 0; a < 3; ++a) {
        double span = p->hi[a] - p->lo[a];
        int d = (int)ceil(span / g->cs);
        if (d < 1) d = 1;
        g->dims[a] = d;
        if (d > maxd) maxd = d;
        g->lo32[a] = (float)p->lo[a];
    }
    int b = 0;
    while ((1 << b) < maxd) ++b;
    g->bits = b;
    g->inv_cs64 = 1.0 / g->cs;
    g->inv_cs32 = (float)g->inv_cs64;
    float Rf = (float)R;
    g->R2_32 = Rf * Rf;
    g->R2_64 = R * R;
}

static int clampi(double t, int d)
{
    if (!(t >= 0.0)) return 0; /* also NaN */
    if (t >= (double)d) return d - 1;
    return (int)t;
}

static void cell_coord(const orc_params *p, const orc_grid *g, const double *x, int c[3])
{
    for (int a = 0; a < 3; ++a) {
        double t;
        if (p->precision == 0) {
            float xf = (float)x[a];
            float d = xf - g->lo32[a];
            float s = d * g->inv_cs32;
            t = (double)floorf(s);
        } else {
            double d = x[a] - p->lo[a];
            double s = d * g->inv_cs64;
            t = floor(s);
        }
        c[a] = clampi(t, g->dims[a]);
    }
}

/* Morton code: bit b of x, y, z goes to bits 3b, 3b+1, 3b+2. */
uint32_t orc_morton3(int cx, int cy, int cz, int bits)
{
    uint32_t k = 0;
    for (int b = 0; b < bits; ++b) {
        k |= (uint32_t)((cx >> b) & 1) << (3 * b);
        k |= (uint32_t)((cy >> b) & 1) << (3 * b + 1);
        k |= (uint32_t)((cz >> b) & 1) << (3 * b + 2);
    }
    return k;
}

void orc_cell_keys(const orc_params *p, int64_t n, const double *x, uint32_t *keys)
{
    orc_grid g;
    orc_grid_setup(p, &g);
    for (int64_t i = 0; i < n; ++i) {
        int c[3];
        cell_coord(p, &g, x + 3 * i, c);
        keys[i] = orc_morton3(c[0], c[1], c[2], g.bits);
    }
}

/* Neighbour predicate: j is a neighbour of i iff r^2 < R^2 with
 *   d = x_j - x_i (per axis), r^2 = fma(dz, dz, fma(dy, dy, dx*dx))
 * in the run's precision, R^2 rounded to that precision. */
static int is_nbr(const orc_params *p, const orc_grid *g, const double *xi, const double *xj)
{
    if (p->precision == 0) {
        float dx = (float)xj[0] - (float)xi[0];
        float dy = (float)xj[1] - (float)xi[1];
        float dz = (float)xj[2] - (float)xi[2];
        float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        return r2 < g->R2_32;
    } else {
        double dx = xj[0] - xi[0];
        double dy = xj[1] - xi[1];
        double dz = xj[2] - xi[2];
        double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        return r2 < g->R2_64;
    }
}

static double dist(const double *a, const double *b, double d[3])
{
    d[0] = a[0] - b[0];
    d[1] = a[1] - b[1];
    d[2] = a[2] - b[2];
    return sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
}

/* ------------------------------------------------------------------ */
/* Neighbour lists N(i) = { j : predicate(i, j) }, self included,       */
/* each list in ascending id.                                           */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t n;
    int32_t *cell_of;   /* linear cell index per particle */
    int64_t *start;     /* per linear cell, size ncell+1 */
    int64_t *items;     /* particle ids sorted by cell, ascending id inside a cell */
    int64_t ncell;
} cell_list;

static void cl_build(const orc_params *p, const orc_grid *g, int64_t n, const double *x, cell_list *cl)
{
    int64_t nc = (int64_t)g->dims[0] * g->dims[1] * g->dims[2];
    cl->n = n;
    cl->ncell = nc;
    cl->cell_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    cl->start = (int64_t *)calloc((size_t)nc + 1, sizeof(int64_t));
    cl->items = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        int c[3];
        cell_coord(p, g, x + 3 * i, c);
        int32_t lin = (int32_t)(((int64_t)c[2] * g->dims[1] + c[1]) * g->dims[0] + c[0]);
        cl->cell_of[i] = lin;
        cl->start[lin + 1]++;
    }
    for (int64_t c = 0; c < nc; ++c) cl->start[c + 1] += cl->start[c];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nc + 1));
    memcpy(fill, cl->start, sizeof(int64_t) * (size_t)(nc + 1));
    for (int64_t i = 0; i < n; ++i) cl->items[fill[cl->cell_of[i]]++] = i;
    free(fill);
}

static void cl_free(cell_list *cl)
{
    free(cl->cell_of);
    free(cl->start);
    free(cl->items);
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* one target's list through the cell list: the 27 cells around its cell */
static int64_t nbr_grid_one(const orc_params *p, const orc_grid *g, const cell_list *cl,
                            const double *x, int64_t i, int64_t *buf, int64_t cap)
{
    int c[3];
    cell_coord(p, g, x + 3 * i, c);
    int64_t m = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int a = c[0] + dx, b = c[1] + dy, d = c[2] + dz;
                if (a < 0 || b < 0 || d < 0 || a >= g->dims[0] || b >= g->dims[1] || d >= g->dims[2])
                    continue;
                int64_t lin = ((int64_t)d * g->dims[1] + b) * g->dims[0] + a;
                for (int64_t t = cl->start[lin]; t < cl->start[lin + 1]; ++t) {
                    int64_t j = cl->items[t];
                    if (is_nbr(p, g, x + 3 * i, x + 3 * j)) {
                        if (m < cap) buf[m] = j;
                        ++m;
                    }
                }
            }
    if (m <= cap) qsort(buf, (size_t)m, sizeof(int64_t), cmp_i64);
    return m;
}

/*
 * Neighbour lists of the targets (all particles when targets == NULL).
 * use_grid = 0: brute force over all n particles (O(n^2)); 1: cell list.
 * counts[t] receives |N(target t)|; the lists are written back to back into
 * ids (capacity cap entries).  Returns the total count (the lists are only
 * written when it fits).
 */
int64_t orc_neighbors(const orc_params *p, int64_t n, const double *x, int64_t nt,
                      const int64_t *targets, int use_grid, int64_t *counts, int64_t *ids, int64_t cap)
{
    orc_grid g;
    orc_grid_setup(p, &g);
    int64_t NT = targets ? nt : n;
    cell_list cl;
    if (use_grid) cl_build(p, &g, n, x, &cl);
    /* pass 1: counts */
#pragma omp parallel
    {
        int64_t bcap = 4096;
        int64_t *buf = (int64_t *)malloc(sizeof(int64_t) * (size_t)bcap);
#pragma omp for schedule(dynamic, 256)
        for (int64_t t = 0; t < NT; ++t) {
            int64_t i = targets ? targets[t] : t;
            int64_t m = 0;
            if (use_grid) {
                m = nbr_grid_one(p, &g, &cl, x, i, buf, 0);
            } else {
                for (int64_t j = 0; j < n; ++j) m += is_nbr(p, &g, x + 3 * i, x + 3 * j);
            }
            counts[t] = m;
        }
        free(buf);
    }
    int64_t total = 0;
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(NT + 1));
    for (int64_t t = 0; t < NT; ++t) {
        off[t] = total;
        total += counts[t];
    }
    off[NT] = total;
    if (ids && total <= cap) {
#pragma omp parallel
        {
            int64_t bcap = 8192;
            int64_t *buf = (int64_t *)malloc(sizeof(int64_t) * (size_t)bcap);
#pragma omp for schedule(dynamic, 256)
            for (int64_t t = 0; t < NT; ++t) {
                int64_t i = targets ? targets[t] : t;
                if (use_grid) {
                    int64_t m = nbr_grid_one(p, &g, &cl, x, i, buf, bcap);
                    if (m > bcap) {
                        free(buf);
                        bcap = m;
                        buf = (int64_t *)malloc(sizeof(int64_t) * (size_t)bcap);
                        m = nbr_grid_one(p, &g, &cl, x, i, buf, bcap);
                    }
                    memcpy(ids + off[t], buf, sizeof(int64_t) * (size_t)m);
                } else {
                    int64_t m = 0;
                    for (int64_t j = 0; j < n; ++j)
                        if (is_nbr(p, &g, x + 3 * i, x + 3 * j)) ids[off[t] + m++] = j;
                }
            }
            free(buf);
        }
    }
    free(off);
    if (use_grid) cl_free(&cl);
    return total;
}

/* ------------------------------------------------------------------ */
/* Boundary particle volumes (Sec. 3.2 boundary particles, Akinci et   */
/* al. 2012 cited in Sec. 2.1): V_b = 1 / sum_{k in N(b), same object} */
/* W(r_bk), psi_b = rho0 V_b, from the configuration given.            */
/* ------------------------------------------------------------------ */

void orc_boundary_psi(const orc_params *p, int64_t n, const double *x, const uint8_t *type,
                      const int32_t *object, const int64_t *counts, const int64_t *offsets,
                      const int64_t *ids, double *psi)
{
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        psi[i] = 0.0;
        if (type[i] != ORC_BOUNDARY) continue;
        double s = 0.0;
        for (int64_t t = 0; t < counts[i]; ++t) {
            int64_t k = ids[offsets[i] + t];
            if (type[k] != ORC_BOUNDARY || object[k] != object[i]) continue;
            double d[3];
            s += orc_W(dist(x + 3 * i, x + 3 * k, d), p->h);
        }
        psi[i] = p->rho0 / s;
    }
}

/* ------------------------------------------------------------------ */
/* Rigid bodies (Sec. 3.2: constant offsets from the parent transform). */
/* ------------------------------------------------------------------ */

/* rotation matrix of a unit quaternion q = (w, x, y, z) */
void orc_quat_to_R(const double q[4], double R[9])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

static void quat_unit(const double *q, double out[4])
{
    double s = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int a = 0; a < 4; ++a) out[a] = q[a] / s;
}

/* body-frame offsets r_loc = R(q0)^T (x - c0) of the particles of object o */
void orc_body_frame(int64_t n, const double *x, const int32_t *object, int32_t o,
                    const double pose0[7], double *r_loc)
{
    double q[4], R[9];
    quat_unit(pose0 + 3, q);
    orc_quat_to_R(q, R);
    for (int64_t i = 0; i < n; ++i) {
        if (object[i] != o) continue;
        double d[3] = {x[3 * i] - pose0[0], x[3 * i + 1] - pose0[1], x[3 * i + 2] - pose0[2]};
        for (int a = 0; a < 3; ++a) r_loc[3 * i + a] = R[a] * d[0] + R[3 + a] * d[1] + R[6 + a] * d[2];
    }
}

/* placement: x_b = c + R(q) r_loc, v_b = v + w x (R(q) r_loc) */
void orc_body_place(int64_t n, const int32_t *object, int32_t o, const double c[3],
                    const double q_in[4], const double vc[3], const double w[3],
                    const double *r_loc, double *x, double *v)
{
    double q[4], R[9];
    quat_unit(q_in, q);
    orc_quat_to_R(q, R);
    for (int64_t i = 0; i < n; ++i) {
        if (object[i] != o) continue;
        const double *r = r_loc + 3 * i;
        double rw[3];
        for (int a = 0; a < 3; ++a) rw[a] = R[3 * a] * r[0] + R[3 * a + 1] * r[1] + R[3 * a + 2] * r[2];
        for (int a = 0; a < 3; ++a) x[3 * i + a] = c[a] + rw[a];
        v[3 * i + 0] = vc[0] + (w[1] * rw[2] - w[2] * rw[1]);
        v[3 * i + 1] = vc[1] + (w[2] * rw[0] - w[0] * rw[2]);
        v[3 * i + 2] = vc[2] + (w[0] * rw[1] - w[1] * rw[0]);
    }
}

/* pose advance over dt: c += v dt, q <- normalise(q + dt/2 (0, w) q) */
void orc_pose_advance(double c[3], double q[4], const double v[3], const double w[3], double dt)
{
    for (int a = 0; a < 3; ++a) c[a] += v[a] * dt;
    double wq[4] = {-w[0] * q[1] - w[1] * q[2] - w[2] * q[3],
                    w[0] * q[0] + w[1] * q[3] - w[2] * q[2],
                    w[1] * q[0] + w[2] * q[1] - w[0] * q[3],
                    w[2] * q[0] + w[0] * q[2] - w[1] * q[1]};
    double t[4];
    for (int a = 0; a < 4; ++a) t[a] = q[a] + 0.5 * dt * wq[a];
    quat_unit(t, q);
}

/* ------------------------------------------------------------------ */
/* Free rigid bodies (Sec. 3.2: a rigid body takes the summed point      */
/* forces of its particles; Sec. 3.3: a released body moves under them). */
/* Mass properties from the body's particles: m = sum m_i, centre of     */
/* mass, inertia about it in the body frame I = sum m_i (|r|^2 1 - r r^T) */
/* with r = R(q0)^T (x_i - com).  Velocity step (semi-implicit Euler, as */
/* Eq. euler for particles): v += dt (F/m + g); with the world inertia   */
/* I_w = R I R^T, w += dt I_w^{-1} (T - w x (I_w w)) (Euler's equations). */
/* ------------------------------------------------------------------ */

void orc_body_mass_props(int64_t n, const double *x, const double *mass, const int32_t *object, int32_t o,
                         const double q0[4], double com[3], double *m_out, double I_body[9])
{
    double m = 0.0, s[3] = {0.0, 0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) {
        if (object[i] != o) continue;
        m += mass[i];
        for (int a = 0; a < 3; ++a) s[a] += mass[i] * x[3 * i + a];
    }
    for (int a = 0; a < 3; ++a) com[a] = s[a] / m;
    *m_out = m;
    double q[4], R[9];
    quat_unit(q0, q);
    orc_quat_to_R(q, R);
    for (int k = 0; k < 9; ++k) I_body[k] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (object[i] != o) continue;
        double d[3] = {x[3 * i] - com[0], x[3 * i + 1] - com[1], x[3 * i + 2] - com[2]};
        double r[3];
        for (int a = 0; a < 3; ++a) r[a] = R[a] * d[0] + R[3 + a] * d[1] + R[6 + a] * d[2];
        double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) I_body[3 * a + b] += mass[i] * ((a == b ? rr : 0.0) - r[a] * r[b]);
    }
}

/* inverse of a 3x3 matrix by cofactors */
static void inv3(const double A[9], double B[9])
{
    double c00 = A[4] * A[8] - A[5] * A[7], c01 = A[5] * A[6] - A[3] * A[8], c02 = A[3] * A[7] - A[4] * A[6];
    double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
    B[0] = c00 / det;
    B[1] = (A[2] * A[7] - A[1] * A[8]) / det;
    B[2] = (A[1] * A[5] - A[2] * A[4]) / det;
    B[3] = c01 / det;
    B[4] = (A[0] * A[8] - A[2] * A[6]) / det;
    B[5] = (A[2] * A[3] - A[0] * A[5]) / det;
    B[6] = c02 / det;
    B[7] = (A[1] * A[6] - A[0] * A[7]) / det;
    B[8] = (A[0] * A[4] - A[1] * A[3]) / det;
}

void orc_body_velocity_step(const double F[3], const double T[3], double m, const double I_body[9],
                            const double q_in[4], const double g[3], double dt, double v[3], double w[3])
{
    double q[4], R[9], Iw[9], Iwi[9], tmp[9];
    quat_unit(q_in, q);
    orc_quat_to_R(q, R);
    /* I_w = R I R^T */
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double t = 0.0;
            for (int k = 0; k < 3; ++k) t += R[3 * a + k] * I_body[3 * k + b];
            tmp[3 * a + b] = t;
        }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double t = 0.0;
            for (int k = 0; k < 3; ++k) t += tmp[3 * a + k] * R[3 * b + k];
            Iw[3 * a + b] = t;
        }
    inv3(Iw, Iwi);
    double L[3];
    for (int a = 0; a < 3; ++a) L[a] = Iw[3 * a] * w[0] + Iw[3 * a + 1] * w[1] + Iw[3 * a + 2] * w[2];
    double rhs[3] = {T[0] - (w[1] * L[2] - w[2] * L[1]), T[1] - (w[2] * L[0] - w[0] * L[2]),
                     T[2] - (w[0] * L[1] - w[1] * L[0])};
    double wd[3];
    for (int a = 0; a < 3; ++a) wd[a] = Iwi[3 * a] * rhs[0] + Iwi[3 * a + 1] * rhs[1] + Iwi[3 * a + 2] * rhs[2];
    for (int a = 0; a < 3; ++a) {
        v[a] += dt * (F[a] / m + g[a]);
        w[a] += dt * wd[a];
    }
}

/* ------------------------------------------------------------------ */
/* Density and pressure (Eqs. density, pressure; Alg. 1 first pass).    */
/* rho_i = sum_{j in N(i)} mass_j W_ij, boundary mass = psi_b.          */
/* ------------------------------------------------------------------ */

void orc_density(const orc_params *p, int64_t n, const double *x, const double *mass,
                 const uint8_t *type, const double *psi, int64_t nt, const int64_t *targets,
                 const int64_t *counts, const int64_t *offsets, const int64_t *ids,
                 double *rho, double *press)
{
    (void)n;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t i = targets[t];
        double s = 0.0;
        for (int64_t u = 0; u < counts[t]; ++u) {
            int64_t j = ids[offsets[t] + u];
            double d[3];
            double mj = type[j] == ORC_BOUNDARY ? psi[j] : mass[j];
            s += mj * orc_W(dist(x + 3 * i, x + 3 * j, d), p->h);
        }
        double pr = p->k * (s - p->rho0);
        if ((p->flags & ORC_CLAMP_NEG_PRESSURE) && pr < 0.0) pr = 0.0;
        rho[t] = s;
        press[t] = pr;
    }
}

/* ------------------------------------------------------------------ */
/* Density probes: the summation of Eq. density evaluated at a free point */
/* (Sec. 3.4 reads the fluid density field of the tank), over fluid and   */
/* soft particles only.  The point is first rounded to the run precision */
/* (the precision particle positions are stored in), then every particle */
/* is tested with the same support predicate as a particle pair.         */
/* Brute force over all particles: no grid involved.                    */
/* ------------------------------------------------------------------ */

void orc_probe_density(const orc_params *p, int64_t n, const double *x, const double *mass,
                       const uint8_t *type, int64_t np, const double *pts, double *out)
{
    orc_grid g;
    orc_grid_setup(p, &g);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < np; ++t) {
        double q[3];
        for (int a = 0; a < 3; ++a) q[a] = p->precision == 0 ? (double)(float)pts[3 * t + a] : pts[3 * t + a];
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (type[j] == ORC_BOUNDARY) continue;
            if (!is_nbr(p, &g, q, x + 3 * j)) continue;
            double d[3];
            s += mass[j] * orc_W(dist(q, x + 3 * j, d), p->h);
        }
        out[t] = s;
    }
}

/* ------------------------------------------------------------------ */
/* Springs of the soft bodies (Sec. 3.2 mass-spring, Alg. 2).            */
/* f_i += -[k (|x_ij| - L0) + c (v_ij . e_ij)] e_ij, e_ij = x_ij/|x_ij| */
/* ------------------------------------------------------------------ */

void orc_springs(int64_t n, const double *x, const double *v, int64_t ns, const uint32_t *ij,
                 const double *L0, const double *ks, const double *cs, double *f)
{
    memset(f, 0, sizeof(double) * 3 * (size_t)n);
    for (int64_t s = 0; s < ns; ++s) {
        int64_t i = ij[2 * s], j = ij[2 * s + 1];
        double d[3];
        double r = dist(x + 3 * i, x + 3 * j, d);
        double e[3] = {d[0] / r, d[1] / r, d[2] / r};
        double vr = (v[3 * i] - v[3 * j]) * e[0] + (v[3 * i + 1] - v[3 * j + 1]) * e[1] +
                    (v[3 * i + 2] - v[3 * j + 2]) * e[2];
        double mag = ks[s] * (r - L0[s]) + cs[s] * vr;
        for (int a = 0; a < 3; ++a) {
            f[3 * i + a] -= mag * e[a];
            f[3 * j + a] += mag * e[a];
        }
    }
}

/* ------------------------------------------------------------------ */
/* Pair forces (Alg. 1 second pass: pressure and viscosity forces).      */
/* f_ij for i a fluid/soft particle:                                    */
/*   j fluid/soft: -m_i m_j (p_i/rho_i^2 + p_j/rho_j^2) gradW_ij         */
/*                 + 2 nu m_i m_j [2/(rho_i+rho_j)] (x_ij.gradW)/(r^2+eps) v_ij */
/*   j boundary b: the same with m_j = psi_b, p_j = p_i, rho_j = rho_i   */
/*   (pressure mirrored into the boundary particle); with the unified   */
/*   reading (every typed particle an SPH particle, Sec. 3.2) the same   */
/*   with m_j = psi_b and the boundary particle's own rho_b and p_b.      */
/* gradW_ij = dW/dr(r) x_ij / r (0 at r = 0).                           */
/* ------------------------------------------------------------------ */

static void pair_force(const orc_params *p, int64_t i, int64_t j, const double *x, const double *v,
                       const double *mass, const uint8_t *type, const double *psi, double rhoi,
                       double pi, double rhoj, double pj, double out[3])
{
    double d[3];
    double r = dist(x + 3 * i, x + 3 * j, d);
    out[0] = out[1] = out[2] = 0.0;
    if (r == 0.0) return;
    double dw = orc_dWdr(r, p->h);
    double gw[3] = {dw * d[0] / r, dw * d[1] / r, dw * d[2] / r};
    double eps = 0.01 * p->h * p->h;
    double vij[3] = {v[3 * i] - v[3 * j], v[3 * i + 1] - v[3 * j + 1], v[3 * i + 2] - v[3 * j + 2]};
    double xg = d[0] * gw[0] + d[1] * gw[1] + d[2] * gw[2];
    double mi = mass[i];
    if (type[j] == ORC_BOUNDARY && (p->flags & ORC_UNIFIED_BOUNDARY)) {
        double mj = psi[j];
        double pterm = pi / (rhoi * rhoi) + pj / (rhoj * rhoj);
        double visc = (p->flags & ORC_NO_BOUNDARY_VISCOSITY)
                          ? 0.0
                          : 2.0 * p->nu * mi * mj * (2.0 / (rhoi + rhoj)) * xg / (r * r + eps);
        for (int a = 0; a < 3; ++a) out[a] = -mi * mj * pterm * gw[a] + visc * vij[a];
    } else if (type[j] == ORC_BOUNDARY) {
        double psib = psi[j];
        double pterm = (p->flags & ORC_BOUNDARY_SINGLE_TERM) ? pi / (rhoi * rhoi) : 2.0 * pi / (rhoi * rhoi);
        double visc = (p->flags & ORC_NO_BOUNDARY_VISCOSITY) ? 0.0 : 2.0 * p->nu * mi * psib * (1.0 / rhoi) * xg / (r * r + eps);
        for (int a = 0; a < 3; ++a) out[a] = -mi * psib * pterm * gw[a] + visc * vij[a];
    } else {
        double mj = mass[j];
        double pterm = pi / (rhoi * rhoi) + pj / (rhoj * rhoj);
        double visc = 2.0 * p->nu * mi * mj * (2.0 / (rhoi + rhoj)) * xg / (r * r + eps);
        for (int a = 0; a < 3; ++a) out[a] = -mi * mj * pterm * gw[a] + visc * vij[a];
    }
}

/*
 * Force on each target.  rho/press are indexed by particle id (entries of
 * boundary particles unused).  fluid/soft: sum_{j in N(i), j != i, not both
 * boundary} f_ij + m_i g + f_i^spring.  boundary b: f_b = -sum_{i in N(b),
 * i fluid/soft} f_ib (Newton's third law, the point forces on the body).
 */
void orc_forces(const orc_params *p, int64_t n, const double *x, const double *v, const double *mass,
                const uint8_t *type, const double *psi, const double *rho, const double *press,
                const double *fspring, int64_t nt, const int64_t *targets, const int64_t *counts,
                const int64_t *offsets, const int64_t *ids, double *f)
{
    (void)n;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t i = targets[t];
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t u = 0; u < counts[t]; ++u) {
            int64_t j = ids[offsets[t] + u];
            if (j == i) continue;
            double fij[3];
            if (type[i] != ORC_BOUNDARY) {
                pair_force(p, i, j, x, v, mass, type, psi, rho[i], press[i], rho[j], press[j], fij);
                for (int a = 0; a < 3; ++a) acc[a] += fij[a];
            } else if (type[j] != ORC_BOUNDARY) {
                pair_force(p, j, i, x, v, mass, type, psi, rho[j], press[j], rho[i], press[i], fij);
                for (int a = 0; a < 3; ++a) acc[a] -= fij[a];
            }
        }
        if (type[i] != ORC_BOUNDARY) {
            for (int a = 0; a < 3; ++a) acc[a] += mass[i] * p->g[a] + (fspring ? fspring[3 * i + a] : 0.0);
        }
        for (int a = 0; a < 3; ++a) f[3 * t + a] = acc[a];
    }
}

/* ------------------------------------------------------------------ */
/* Body wrench (Sec. 3.2 point forces summed into the parent; Sec. 3.3   */
/* the grabbed body's force goes to the device): F = sum f_b,           */
/* T = sum (R(q) r_loc_b) x f_b about the body reference point c.       */
/* ------------------------------------------------------------------ */

void orc_wrench(int64_t n, const int32_t *object, int32_t o, const double q_in[4],
                const double *r_loc, const double *f, double F[3], double T[3])
{
    double q[4], R[9];
    quat_unit(q_in, q);
    orc_quat_to_R(q, R);
    F[0] = F[1] = F[2] = T[0] = T[1] = T[2] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (object[i] != o) continue;
        const double *r = r_loc + 3 * i;
        const double *fb = f + 3 * i;
        double rw[3];
        for (int a = 0; a < 3; ++a) rw[a] = R[3 * a] * r[0] + R[3 * a + 1] * r[1] + R[3 * a + 2] * r[2];
        for (int a = 0; a < 3; ++a) F[a] += fb[a];
        T[0] += rw[1] * fb[2] - rw[2] * fb[1];
        T[1] += rw[2] * fb[0] - rw[0] * fb[2];
        T[2] += rw[0] * fb[1] - rw[1] * fb[0];
    }
}

/* ------------------------------------------------------------------ */
/* Semi-implicit Euler (Eq. euler) for fluid and soft particles.        */
/* ------------------------------------------------------------------ */

void orc_integrate(const orc_params *p, int64_t n, const uint8_t *type, const double *mass,
                   const double *f, double *x, double *v)
{
    for (int64_t i = 0; i < n; ++i) {
        if (type[i] == ORC_BOUNDARY) continue;
        for (int a = 0; a < 3; ++a) {
            v[3 * i + a] = v[3 * i + a] + (f[3 * i + a] / mass[i]) * p->dt;
            x[3 * i + a] = x[3 * i + a] + v[3 * i + a] * p->dt;
        }
    }
}
