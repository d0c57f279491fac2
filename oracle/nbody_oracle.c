/*
 * nbody_oracle.c -- plain, slow FP64 CPU oracle for the gravity-centred binary-star element model
 * (Goderya et al., "N-body simulation of binary star mass transfer using NVIDIA GPUs").
 *
 * TEST INFRASTRUCTURE ONLY. The tests, the smoke check and the benchmark's CPU-baseline leg are
 * the only callers. It shares no code, header, table or helper with the GPU library, and the GPU
 * library never calls it.
 *
 * What it computes, and where each piece comes from:
 *  - all-pairs acceleration: the state of each element changes only through the sum of every
 *    pairwise element-element interaction (Methodology). Direct double loop, j in index order,
 *    no cut-off, no tiling.
 *  - pair law: elements always attract and elements in contact also repel (Methodology, the
 *    description of the interactions). The law used is the conservative contact law:
 *      f(r) = G mi mj / r^2                        for r >= D
 *      f(r) = G mi mj r / D^3 - K (1 - r/D)        for r <  D,   K = 10 G mi mj / D^2
 *    with f > 0 meaning attraction, D the element diameter of the pair (per star; the mean of
 *    the two stars' diameters across stars).
 *  - pair potential U(r) with dU/dr = f(r) and U continuous at D (its derivative is the law).
 *  - leap-frog integrator (Methodology) in kick-drift-kick form, x and v synchronous.
 *  - donor growth: the donor's element diameter grows by a fixed factor per step while the
 *    donor's nominal radius stays inside its Roche lobe (Methodology: element radius grows to
 *    turn a main-sequence star into a red giant; eq. 3 for the lobe radius).
 *  - eq. (3): Roche-lobe radius r_L(q) / a as printed, coefficient 0.69.
 *  - L1: inner Lagrange point of the normalised Roche potential (the equipotential discussion
 *    around eq. 2), found by bisection of the axial derivative.
 *  - FP64 diagnostics: centre of mass, linear and angular momentum, kinetic, potential and total
 *    energy.
 *  - the paper's own element law, eqs. (4)-(6), as a second law: softened attraction
 *    G mi mj / (r + eps)^2 everywhere; for elements in contact (r < 2R) minus a repulsion
 *    gamma V(r) proportional to the overlap volume V of two spheres of radius R, at full strength
 *    while the pair converges ((v_j - v_i).(r_j - r_i) < 0) and reduced by the factor beta
 *    otherwise. The printed volume term r^2/12 is read as r^3/12, so that V vanishes at r = 2R.
 *    R is half the pair's element diameter.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- threads */

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------- pair law */

/* Attractive magnitude of the force between two elements at centre distance r (negative values
 * are net repulsion). */
double orc_pair_force(double r, double D, double G, double mi, double mj)
{
    if (r >= D) {
        return G * mi * mj / (r * r);
    }
    double K = 10.0 * G * mi * mj / (D * D);
    return G * mi * mj * r / (D * D * D) - K * (1.0 - r / D);
}

/* Pair potential energy whose radial derivative is orc_pair_force. */
double orc_pair_potential(double r, double D, double G, double mi, double mj)
{
    if (r >= D) {
        return -G * mi * mj / r;
    }
    double K = 10.0 * G * mi * mj / (D * D);
    return -(G * mi * mj / (2.0 * D * D * D)) * (3.0 * D * D - r * r)
           + K * (D - r) * (D - r) / (2.0 * D);
}

/* Element diameter that governs the pair (i, j): star 1 owns indices [0, n1), star 2 the rest. */
static double pair_diameter(int64_t i, int64_t j, int64_t n1, double D1, double D2)
{
    int si = (i >= n1);
    int sj = (j >= n1);
    if (si != sj) {
        return 0.5 * (D1 + D2);
    }
    return si ? D2 : D1;
}

/* ---------------------------------------------------------------- paper's law, eqs. (4)-(6) */

static const double ORC_PI = 3.14159265358979323846;

/* Overlap volume of two spheres of radius R whose centres are r apart (0 for r >= 2R):
 * pi (4/3 R^3 - R^2 r + r^3 / 12). */
double orc_overlap_volume(double r, double R)
{
    if (r >= 2.0 * R) return 0.0;
    return ORC_PI * (4.0 / 3.0 * R * R * R - R * R * r + r * r * r / 12.0);
}

/* Attractive magnitude of eqs. (4)-(6). vr is the radial relative velocity
 * (v_j - v_i).(r_j - r_i) / r; the pair converges when vr < 0. */
double orc_paper_force(double r, double vr, double R, double G, double mi, double mj, double eps,
                       double gamma, double beta)
{
    double f = G * mi * mj / ((r + eps) * (r + eps));
    if (r < 2.0 * R) {
        double g = vr < 0.0 ? gamma : gamma * beta;
        f -= g * orc_overlap_volume(r, R);
    }
    return f;
}

/* Potential of the converging branch (beta = 1): softened gravity plus the primitive of the
 * overlap repulsion, gamma pi (R^4 - 4/3 R^3 r + R^2 r^2 / 2 - r^4 / 48) for r < 2R. */
double orc_paper_potential(double r, double R, double G, double mi, double mj, double eps,
                           double gamma)
{
    double u = -G * mi * mj / (r + eps);
    if (r < 2.0 * R) {
        u += gamma * ORC_PI * (R * R * R * R - 4.0 / 3.0 * R * R * R * r + R * R * r * r / 2.0
                             - r * r * r * r / 48.0);
    }
    return u;
}

/* ---------------------------------------------------------------- all-pairs acceleration */

/* a_i = sum_{j != i, r_ij > 0} (f(r_ij) / m) (r_j - r_i) / r_ij for the requested rows.
 * rows == NULL means rows 0..nrows-1. Output k belongs to row rows[k]. */
void orc_accel_rows(const double *x, const double *y, const double *z, int64_t n, int64_t n1,
                    double G, double m, double D1, double D2, const int64_t *rows, int64_t nrows,
                    double *ax, double *ay, double *az)
{
    int64_t k;
#pragma omp parallel for schedule(dynamic, 8)
    for (k = 0; k < nrows; ++k) {
        int64_t i = rows ? rows[k] : k;
        double sx = 0.0, sy = 0.0, sz = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = x[j] - x[i];
            double dy = y[j] - y[i];
            double dz = z[j] - z[i];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            if (r == 0.0) continue;
            double f = orc_pair_force(r, pair_diameter(i, j, n1, D1, D2), G, m, m);
            double g = (f / m) / r;
            sx += g * dx;
            sy += g * dy;
            sz += g * dz;
        }
        ax[k] = sx;
        ay[k] = sy;
        az[k] = sz;
    }
}

/* a_i under eqs. (4)-(6): like orc_accel_rows, with the pair radius R = D_ij / 2 and the radial
 * relative velocity taken from vx, vy, vz. */
void orc_accel_rows_paper(const double *x, const double *y, const double *z, const double *vx,
                          const double *vy, const double *vz, int64_t n, int64_t n1, double G,
                          double m, double D1, double D2, double eps, double gamma, double beta,
                          const int64_t *rows, int64_t nrows, double *ax, double *ay, double *az)
{
    int64_t k;
#pragma omp parallel for schedule(dynamic, 8)
    for (k = 0; k < nrows; ++k) {
        int64_t i = rows ? rows[k] : k;
        double sx = 0.0, sy = 0.0, sz = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = x[j] - x[i];
            double dy = y[j] - y[i];
            double dz = z[j] - z[i];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            if (r == 0.0) continue;
            double vr = ((vx[j] - vx[i]) * dx + (vy[j] - vy[i]) * dy + (vz[j] - vz[i]) * dz) / r;
            double R = 0.5 * pair_diameter(i, j, n1, D1, D2);
            double f = orc_paper_force(r, vr, R, G, m, m, eps, gamma, beta);
            double g = (f / m) / r;
            sx += g * dx;
            sy += g * dy;
            sz += g * dz;
        }
        ax[k] = sx;
        ay[k] = sy;
        az[k] = sz;
    }
}

/* Potential energy sum_{i<j} of the converging-branch potential of eqs. (4)-(6). */
double orc_paper_pe(const double *x, const double *y, const double *z, int64_t n, int64_t n1,
                    double G, double m, double D1, double D2, double eps, double gamma)
{
    double *row = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    int64_t i;
#pragma omp parallel for schedule(dynamic, 8)
    for (i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t j = i + 1; j < n; ++j) {
            double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            if (r == 0.0) continue;
            s += orc_paper_potential(r, 0.5 * pair_diameter(i, j, n1, D1, D2), G, m, m, eps, gamma);
        }
        row[i] = s;
    }
    double pe = 0.0;
    for (i = 0; i < n; ++i) pe += row[i];
    free(row);
    return pe;
}

/* Force on element i from element j alone (f_ij as a vector), for antisymmetry checks. */
void orc_pair_vector(const double *x, const double *y, const double *z, int64_t n1, double G,
                     double m, double D1, double D2, int64_t i, int64_t j, double out[3])
{
    double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    out[0] = out[1] = out[2] = 0.0;
    if (i == j || r == 0.0) return;
    double f = orc_pair_force(r, pair_diameter(i, j, n1, D1, D2), G, m, m);
    out[0] = f * dx / r;
    out[1] = f * dy / r;
    out[2] = f * dz / r;
}

/* ---------------------------------------------------------------- eq. (3) and L1 */

/* eq. (3): Roche-lobe radius of the star of mass ratio q, in units of the separation. */
double orc_roche_lobe(double q)
{
    double q13 = cbrt(q);
    double q23 = q13 * q13;
    return 0.49 * q23 / (0.69 * q23 + log(1.0 + q13));
}

/* Distance of L1 from the accretor (mass 1) towards the donor (mass q), separation 1. In the
 * co-rotating frame with unit separation and G (M1 + M2) = 1, the axial derivative of the Roche
 * potential between the stars is mu1 / x^2 - mu2 / (1 - x)^2 - (x - mu2), mu1 = 1/(1+q),
 * mu2 = q/(1+q); it falls strictly from +inf to -inf on (0, 1), and L1 is its zero. */
double orc_l1_point(double q)
{
    double mu1 = 1.0 / (1.0 + q);
    double mu2 = q / (1.0 + q);
    double lo = 0.0, hi = 1.0;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double g = mu1 / (mid * mid) - mu2 / ((1.0 - mid) * (1.0 - mid)) - (mid - mu2);
        if (g > 0.0) {
            lo = mid;
        } else {
            hi = mid;
        }
    }
    return 0.5 * (lo + hi);
}

/* Centres of mass of the two stars (equal element masses: plain means over index ranges),
 * sequential sums in index order. */
static void star_centres(const double *x, const double *y, const double *z, int64_t n,
                         int64_t n1, double c1[3], double c2[3])
{
    double s1[3] = {0.0, 0.0, 0.0}, s2[3] = {0.0, 0.0, 0.0};
    for (int64_t i = 0; i < n1; ++i) {
        s1[0] += x[i];
        s1[1] += y[i];
        s1[2] += z[i];
    }
    for (int64_t i = n1; i < n; ++i) {
        s2[0] += x[i];
        s2[1] += y[i];
        s2[2] += z[i];
    }
    for (int d = 0; d < 3; ++d) {
        c1[d] = n1 > 0 ? s1[d] / (double)n1 : 0.0;
        c2[d] = (n - n1) > 0 ? s2[d] / (double)(n - n1) : 0.0;
    }
}

/* Donor elements past the L1 plane: the plane through L1 perpendicular to the line joining the
 * two stars' centres of mass, with L1 at l1_point(q) times the measured centre distance from the
 * accretor's centre. side[] (optional) holds each donor element's previous side (1 = past L1);
 * with init != 0 it is only set. out = {n_past, forward crossings, backward crossings}. */
void orc_l1_count(const double *x, const double *y, const double *z, int64_t n, int64_t n1,
                  double q, int8_t *side, int init, int32_t out[3])
{
    double c1[3], c2[3];
    star_centres(x, y, z, n, n1, c1, c2);
    double e[3] = {c2[0] - c1[0], c2[1] - c1[1], c2[2] - c1[2]};
    double d = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    int32_t past = 0, fwd = 0, bwd = 0;
    if (d > 0.0) {
        e[0] /= d;
        e[1] /= d;
        e[2] /= d;
        double xi_l1 = orc_l1_point(q) * d;
        for (int64_t i = n1; i < n; ++i) {
            double xi = (x[i] - c1[0]) * e[0] + (y[i] - c1[1]) * e[1] + (z[i] - c1[2]) * e[2];
            int p = xi < xi_l1;
            past += p;
            if (side) {
                if (!init) {
                    if (p && !side[i]) fwd++;
                    if (!p && side[i]) bwd++;
                }
                side[i] = (int8_t)p;
            }
        }
    }
    out[0] = past;
    out[1] = fwd;
    out[2] = bwd;
}

/* Accretor-side retention of transferred elements. A donor element counts as transferred when it
 * is past the L1 plane (the test of orc_l1_count), and as retained when it is also bound to the
 * accretor taken as a point mass M1 = n1 m at its centre of mass C1 moving with its mean velocity
 * V1: |v - V1|^2 / 2 - G M1 / |r - C1| < 0. out = {n_past, n_bound}. */
void orc_retention(const double *x, const double *y, const double *z, const double *vx,
                   const double *vy, const double *vz, int64_t n, int64_t n1, double G,
                   double m, double q, int32_t out[2])
{
    double c1[3], c2[3], v1[3], v2[3];
    star_centres(x, y, z, n, n1, c1, c2);
    star_centres(vx, vy, vz, n, n1, v1, v2); /* mean velocities, same index-order sums */
    double e[3] = {c2[0] - c1[0], c2[1] - c1[1], c2[2] - c1[2]};
    double d = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    int32_t past = 0, bound = 0;
    if (n1 > 0 && n > n1 && d > 0.0) {
        e[0] /= d;
        e[1] /= d;
        e[2] /= d;
        double xi_l1 = orc_l1_point(q) * d;
        double gm1 = G * m * (double)n1;
        for (int64_t i = n1; i < n; ++i) {
            double rx = x[i] - c1[0], ry = y[i] - c1[1], rz = z[i] - c1[2];
            if (!(rx * e[0] + ry * e[1] + rz * e[2] < xi_l1)) continue;
            past++;
            double ux = vx[i] - v1[0], uy = vy[i] - v1[1], uz = vz[i] - v1[2];
            double r = sqrt(rx * rx + ry * ry + rz * rz);
            double energy = 0.5 * (ux * ux + uy * uy + uz * uz) - gm1 / r;
            if (energy < 0.0) bound++;
        }
    }
    out[0] = past;
    out[1] = bound;
}

/* ---------------------------------------------------------------- diagnostics */

/* out = {com[3], P[3], L[3], KE, PE, E}. PE = sum_{i<j} U(r_ij) when with_pe, else 0. */
void orc_diag(const double *x, const double *y, const double *z, const double *vx,
              const double *vy, const double *vz, int64_t n, int64_t n1, double G, double m,
              double D1, double D2, int with_pe, double out[12])
{
    double com[3] = {0, 0, 0}, P[3] = {0, 0, 0}, L[3] = {0, 0, 0}, KE = 0.0, PE = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        com[0] += m * x[i];
        com[1] += m * y[i];
        com[2] += m * z[i];
        P[0] += m * vx[i];
        P[1] += m * vy[i];
        P[2] += m * vz[i];
        L[0] += m * (y[i] * vz[i] - z[i] * vy[i]);
        L[1] += m * (z[i] * vx[i] - x[i] * vz[i]);
        L[2] += m * (x[i] * vy[i] - y[i] * vx[i]);
        KE += 0.5 * m * (vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]);
    }
    double M = m * (double)n;
    for (int d = 0; d < 3; ++d) com[d] = M > 0.0 ? com[d] / M : 0.0;
    if (with_pe && n > 1) {
        double *row = (double *)calloc((size_t)n, sizeof(double));
        int64_t i;
#pragma omp parallel for schedule(dynamic, 8)
        for (i = 0; i < n; ++i) {
            double s = 0.0;
            for (int64_t j = i + 1; j < n; ++j) {
                double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
                double r = sqrt(dx * dx + dy * dy + dz * dz);
                if (r == 0.0) continue;
                s += orc_pair_potential(r, pair_diameter(i, j, n1, D1, D2), G, m, m);
            }
            row[i] = s;
        }
        for (i = 0; i < n; ++i) PE += row[i];
        free(row);
    }
    memcpy(out, com, sizeof com);
    memcpy(out + 3, P, sizeof P);
    memcpy(out + 6, L, sizeof L);
    out[9] = KE;
    out[10] = PE;
    out[11] = KE + PE;
}

/* ---------------------------------------------------------------- time stepping */

typedef struct {
    int64_t n, n1;
    double G, m, dt;
    double D1, D2;       /* current diameters; D2 is updated by the growth rule */
    double q, a;         /* mass ratio (eq. 3, L1) and nominal separation */
    double R2_0, D2_0;   /* donor radius and element diameter at t = 0 */
    double growth_rate;  /* D2 <- D2 (1 + growth_rate) per growing step */
    int32_t growth_on;
    int32_t growth_stopped;
    int64_t step;        /* completed steps */
    int32_t law;         /* 0: conservative contact law; 1: eqs. (4)-(6) */
    int32_t pad;
    double eps, gamma, beta;  /* parameters of eqs. (4)-(6) */
} orc_state;

/* Accelerations of every element under the state's law (velocity-dependent for law 1). */
static void accel_all(const orc_state *s, const double *x, const double *y, const double *z,
                      const double *vx, const double *vy, const double *vz, double *ax,
                      double *ay, double *az)
{
    if (s->law == 1) {
        orc_accel_rows_paper(x, y, z, vx, vy, vz, s->n, s->n1, s->G, s->m, s->D1, s->D2, s->eps,
                             s->gamma, s->beta, NULL, s->n, ax, ay, az);
    } else {
        orc_accel_rows(x, y, z, s->n, s->n1, s->G, s->m, s->D1, s->D2, NULL, s->n, ax, ay, az);
    }
}

/* Donor growth after a step: while the donor's nominal radius R2_0 D2 / D2_0 is at most
 * r_L(q) a, its element diameter grows by (1 + rate); the first time it exceeds the lobe, growth
 * stops for good. */
static void growth_update(orc_state *s)
{
    if (!s->growth_on || s->growth_stopped) return;
    double R2 = s->R2_0 * s->D2 / s->D2_0;
    if (R2 <= orc_roche_lobe(s->q) * s->a) {
        s->D2 = s->D2 * (1.0 + s->growth_rate);
    } else {
        s->growth_stopped = 1;
    }
}

/* Advance `steps` kick-drift-kick leap-frog steps. x, v (inout) are FP64; side (inout, n bytes,
 * only donor entries used) carries L1 sides; when init_side != 0 the sides are first set from the
 * initial positions. ax, ay, az (inout, n each) hold the acceleration of the current state: with
 * have_accel == 0 it is evaluated first (a(x, v) of the given state), otherwise the values from
 * the previous call are used, so that runs split over several calls equal one long run (under
 * law 1 the acceleration at the end of a step was evaluated with the half-step velocities).
 * counts (optional, steps x 3) receives the per-step L1 counts; d2_log (optional, steps) the
 * donor diameter after each step's growth update. */
void orc_run(orc_state *s, double *x, double *y, double *z, double *vx, double *vy, double *vz,
             int8_t *side, int init_side, double *ax, double *ay, double *az, int have_accel,
             int64_t steps, int32_t *counts, double *d2_log)
{
    int64_t n = s->n;
    int32_t c[3];
    if (init_side && side) orc_l1_count(x, y, z, n, s->n1, s->q, side, 1, c);
    if (!have_accel) accel_all(s, x, y, z, vx, vy, vz, ax, ay, az);
    double h = 0.5 * s->dt;
    for (int64_t st = 0; st < steps; ++st) {
        for (int64_t i = 0; i < n; ++i) {
            vx[i] += h * ax[i];
            vy[i] += h * ay[i];
            vz[i] += h * az[i];
            x[i] += s->dt * vx[i];
            y[i] += s->dt * vy[i];
            z[i] += s->dt * vz[i];
        }
        /* for law 1 the velocities seen by the force are the half-step ones */
        accel_all(s, x, y, z, vx, vy, vz, ax, ay, az);
        for (int64_t i = 0; i < n; ++i) {
            vx[i] += h * ax[i];
            vy[i] += h * ay[i];
            vz[i] += h * az[i];
        }
        growth_update(s);
        orc_l1_count(x, y, z, n, s->n1, s->q, side, 0, c);
        if (counts) {
            counts[3 * st + 0] = c[0];
            counts[3 * st + 1] = c[1];
            counts[3 * st + 2] = c[2];
        }
        if (d2_log) d2_log[st] = s->D2;
        s->step++;
    }
}
