/*
 * tril_oracle.c -- plain FP64 CPU oracle for photon-photon (Breit-Wheeler)
 * collision detection between two beams.
 *
 * TEST INFRASTRUCTURE ONLY.  The product library never links, loads or calls
 * this file; only the test suite, the smoke check and the benchmark's CPU
 * baseline do.  It shares no source, header, table or constant generator with
 * the GPU library.
 *
 * What it computes is the plain definition, with no tree and no pruning that
 * could change a result: for every query photon i (beam A), every target photon
 * j (beam B) and every time step k, the pair collides in step k when
 *
 *   (1) it lies above the Breit-Wheeler threshold, s_ij > 1, where
 *       s = E_i E_j (1 - cos Phi_B) / (2 m_e^2 c^4)          (Sec. 1, Eq. 1 and
 *       the threshold condition Eq. 2; sigma(s = 1) = 0, so the boundary case
 *       s = 1 is not a collision), and
 *
 *   (2) the smallest distance between the two photons over the step's time
 *       window [k dt, (k+1) dt] -- both photons moving on straight lines at c,
 *       positions compared at the same instant -- is at most the collision
 *       radius r_ij, with
 *           r_ij^2 = sqrt(w_i w_j) * sigma_BW(s_ij) / pi
 *       (total cross-section Eq. 1; weights are the macro-particle photon
 *       counts of Sec. 2.2; the boxes of Sec. 2.1 are enlarged by one step's
 *       travel so that collisions inside a step are found in advance).
 *
 * Conventions the paper leaves open (units um, um/c, MeV with c = 1):
 *   * direction u = p / E, componentwise IEEE division, not renormalised;
 *   * photon position at time t: X(t) = x0 + t * u;
 *   * sigma is evaluated in the algebraically identical form
 *       sigma = (pi r_e^2 / 2) / s * [ (3 - b^4) L - 2 b (2 - b^2) ],
 *       b^2 = (s - 1)/s,  L = ln((1+b)/(1-b)) = 2 log1p(b) + ln(s),
 *     using 1 - beta^2 = 1/s; the literal form loses digits to cancellation
 *     near threshold and at large s;
 *   * constants: m_e c^2 = 0.51099895000 MeV, r_e = 2.8179403262e-9 um
 *     (CODATA 2018; the paper quotes none);
 *   * the closest-approach time inside a step is clamped to [0, dt] and both
 *     ends of the distance test are closed (d^2 <= r^2).
 *
 * Every expression below is written in the evaluation order it is computed in;
 * the file is compiled without floating-point contraction or fast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_ME 0.51099895000           /* electron rest energy, MeV */
#define ORC_RE 2.8179403262e-9         /* classical electron radius, um */

typedef struct {
    int64_t n;
    const double *x, *y, *z, *px, *py, *pz, *E, *w;
} orc_beam;

typedef struct {
    int64_t cap;
    int64_t count;        /* number of hits found (may exceed cap) */
    int32_t *i, *j, *k;   /* query row, target row, step */
    double *margin;       /* (r^2 - d^2) / r^2 of the hit */
    int64_t knife_margin; /* pair-steps with |r^2 - d^2| < 2^-40 r^2 */
    int64_t knife_s;      /* pairs with |s - 1| < 2^-40 */
    int64_t pairs_tested; /* pairs (i, j) evaluated, above or below threshold */
    int64_t pairs_full;   /* pairs whose every step was evaluated */
} orc_out;

/* ---- physics of one pair -------------------------------------------------- */

/* Breit-Wheeler total cross-section sigma(s) in um^2 (Sec. 1, Eq. 1). Zero for s <= 1. */
double orc_sigma(double s)
{
    if (!(s > 1.0)) return 0.0;
    const double k_sig = (0.5 * M_PI) * (ORC_RE * ORC_RE);
    double b2 = (s - 1.0) / s;                 /* beta^2 = 1 - 1/s */
    double b = sqrt(b2);
    double L = 2.0 * log1p(b) + log(s);        /* ln((1+b)/(1-b)) */
    double bracket = (3.0 - b2 * b2) * L - (2.0 * b) * (2.0 - b2);
    return (k_sig / s) * bracket;
}

/* Invariant s of two photons (Sec. 1, below Eq. 1): E_i E_j (1 - u_i.u_j) / (2 m_e^2). */
double orc_invariant(double Ei, double uix, double uiy, double uiz,
                     double Ej, double ujx, double ujy, double ujz)
{
    double c = (uix * ujx + uiy * ujy) + uiz * ujz;
    double q = 1.0 - c;
    double two_me2 = 2.0 * ORC_ME * ORC_ME;
    return ((Ei * Ej) * q) / two_me2;
}

/* Smallest squared distance of two photons over [t, t + dt] (positions at equal time).
   Xi(t) = xi + t ui, Xj(t) = xj + t uj; the minimum of |Xi - Xj|^2 over the window is at
   tau* = -(Delta . v)/(v . v) clamped to [0, dt], Delta = Xi(t) - Xj(t), v = ui - uj.
   orc_step_closest gives both; *tau_out receives tau*, the time of closest approach
   measured from t. */
static double orc_step_closest(double t, double dt,
                               double xi, double yi, double zi, double uix, double uiy,
                               double uiz, double xj, double yj, double zj, double ujx,
                               double ujy, double ujz, double *tau_out)
{
    double Xix = xi + t * uix, Xiy = yi + t * uiy, Xiz = zi + t * uiz;
    double Xjx = xj + t * ujx, Xjy = yj + t * ujy, Xjz = zj + t * ujz;
    double dx = Xix - Xjx, dy = Xiy - Xjy, dz = Xiz - Xjz;
    double vx = uix - ujx, vy = uiy - ujy, vz = uiz - ujz;
    double vv = (vx * vx + vy * vy) + vz * vz;
    double dv = (dx * vx + dy * vy) + dz * vz;
    double tau = -dv / vv;
    if (!(tau > 0.0)) tau = 0.0;   /* also catches vv == 0 (NaN / -inf) */
    if (tau > dt) tau = dt;
    double px = dx + tau * vx, py = dy + tau * vy, pz = dz + tau * vz;
    *tau_out = tau;
    return (px * px + py * py) + pz * pz;
}

double orc_step_d2(double t, double dt,
                   double xi, double yi, double zi, double uix, double uiy, double uiz,
                   double xj, double yj, double zj, double ujx, double ujy, double ujz)
{
    double tau;
    return orc_step_closest(t, dt, xi, yi, zi, uix, uiy, uiz, xj, yj, zj, ujx, ujy, ujz, &tau);
}

double orc_step_tau(double t, double dt,
                    double xi, double yi, double zi, double uix, double uiy, double uiz,
                    double xj, double yj, double zj, double ujx, double ujy, double ujz)
{
    double tau;
    (void)orc_step_closest(t, dt, xi, yi, zi, uix, uiy, uiz, xj, yj, zj, ujx, ujy, ujz, &tau);
    return tau;
}

/* Largest value of sigma over all s, found by golden-section search on orc_sigma
   (sigma rises from 0 at threshold to one maximum near s = 2, then falls). */
double orc_sigma_max(void)
{
    double a = 1.0, b = 10.0;
    const double g = 0.6180339887498949;
    double c = b - g * (b - a), d = a + g * (b - a);
    for (int it = 0; it < 200; ++it) {
        if (orc_sigma(c) > orc_sigma(d)) b = d; else a = c;
        c = b - g * (b - a);
        d = a + g * (b - a);
    }
    double m = orc_sigma(0.5 * (a + b));
    /* neighbourhood scan guards the search */
    for (int t = -50; t <= 50; ++t) {
        double v = orc_sigma(0.5 * (a + b) * (1.0 + 1e-4 * t));
        if (v > m) m = v;
    }
    return m;
}

/* ---- all pairs ---------------------------------------------------------- */

static void orc_record(orc_out *o, int32_t i, int32_t j, int32_t k, double margin)
{
    int64_t pos;
#pragma omp atomic capture
    pos = o->count++;
    if (pos < o->cap) {
        o->i[pos] = i;
        o->j[pos] = j;
        o->k[pos] = k;
        o->margin[pos] = margin;
    }
}

/*
 * Evaluate rows `rows[0..n_rows)` of beam A (all rows when rows == NULL) against
 * every photon of B, for steps k0 .. k0+n_steps-1 with step length dt.
 *
 * strict != 0: every pair above threshold is evaluated at every step.
 * strict == 0: a pair above threshold first gets a necessary-condition check:
 *   the distance curve |Xi(t) - Xj(t)| is convex in t, so its minimum over the whole
 *   window [k0 dt, (k0+n_steps) dt] bounds every step's minimum from below; if that
 *   global minimum exceeds an upper bound of r_ij (sigma <= sigma_max) by more than
 *   a rounding slack far above FP64 error, no step can collide and the steps are
 *   skipped. Strict and non-strict runs produce identical hits (checked by tests).
 */
void orc_collide(const orc_beam *A, const orc_beam *B,
                 const int64_t *rows, int64_t n_rows,
                 double dt, int32_t k0, int32_t n_steps, int32_t strict,
                 orc_out *o)
{
    const int64_t nr = rows ? n_rows : A->n;
    const double sig_max = orc_sigma_max() * (1.0 + 1e-6);
    const double t_lo = (double)k0 * dt;
    const double t_hi = (double)(k0 + n_steps) * dt;

    /* coordinate scale for the rounding slack of the pruning test */
    double scale = 1.0;
    for (int64_t a = 0; a < A->n; ++a) {
        double m = fabs(A->x[a]) + fabs(A->y[a]) + fabs(A->z[a]);
        if (m > scale) scale = m;
    }
    for (int64_t b = 0; b < B->n; ++b) {
        double m = fabs(B->x[b]) + fabs(B->y[b]) + fabs(B->z[b]);
        if (m > scale) scale = m;
    }
    scale += fabs(t_hi) + fabs(t_lo);
    const double slack = 1e-9 * scale;

    int64_t knife_m = 0, knife_s = 0, tested = 0, full = 0;

#pragma omp parallel for schedule(dynamic, 16) reduction(+ : knife_m, knife_s, tested, full)
    for (int64_t r = 0; r < nr; ++r) {
        const int64_t i = rows ? rows[r] : r;
        const double Ei = A->E[i];
        const double uix = A->px[i] / Ei, uiy = A->py[i] / Ei, uiz = A->pz[i] / Ei;
        const double xi = A->x[i], yi = A->y[i], zi = A->z[i];
        const double wi = A->w[i];
        for (int64_t j = 0; j < B->n; ++j) {
            const double Ej = B->E[j];
            const double ujx = B->px[j] / Ej, ujy = B->py[j] / Ej, ujz = B->pz[j] / Ej;
            ++tested;
            double s = orc_invariant(Ei, uix, uiy, uiz, Ej, ujx, ujy, ujz);
            if (fabs(s - 1.0) < 0x1p-40) ++knife_s;
            if (!(s > 1.0)) continue;                       /* below threshold */
            const double xj = B->x[j], yj = B->y[j], zj = B->z[j];
            const double wij = sqrt(A->w[i] * B->w[j]);
            (void)wi;
            if (!strict) {
                /* global closest approach over the whole window */
                double r_up = sqrt((wij * sig_max) / M_PI);
                double d2g = orc_step_d2(t_lo, t_hi - t_lo, xi, yi, zi, uix, uiy, uiz,
                                         xj, yj, zj, ujx, ujy, ujz);
                if (sqrt(d2g) > r_up * (1.0 + 1e-9) + slack) continue;
            }
            ++full;
            const double sig = orc_sigma(s);
            const double r2 = (wij * sig) / M_PI;
            for (int32_t kk = 0; kk < n_steps; ++kk) {
                const int32_t k = k0 + kk;
                const double t = (double)k * dt;
                double d2 = orc_step_d2(t, dt, xi, yi, zi, uix, uiy, uiz,
                                        xj, yj, zj, ujx, ujy, ujz);
                double diff = r2 - d2;
                if (fabs(diff) < 0x1p-40 * r2) ++knife_m;
                if (d2 <= r2) orc_record(o, (int32_t)i, (int32_t)j, k, diff / r2);
            }
        }
    }
    o->knife_margin += knife_m;
    o->knife_s += knife_s;
    o->pairs_tested += tested;
    o->pairs_full += full;
}

/* ---- statistical (cloud) regime ------------------------------------------------
 *
 * Each macro-particle is a uniform cloud filling a box of edges cell[0..2] about its
 * position, with number density w / V, V = cell[0] cell[1] cell[2] (the paper's rate
 * picture of Sec. 2.2: rate n_I n_II <sigma v> between two clouds, <sigma v> for two
 * photons carrying the factor (1 - cos phi) c). Over step k the pair (i, j) yields
 *   Y = n_i n_j sigma(s) (1 - u_i.u_j) dt V_ov,
 * V_ov the volume common to the two clouds at the middle of the step, t = k dt + dt/2.
 * out[a * nB + j] receives Y summed over steps k0 .. k0+n_steps-1 for query row
 * rows[a] (all rows of A when rows is NULL, then a = i). */
static double orc_cloud_overlap(double dx, double dy, double dz, const double cell[3])
{
    double ov = 1.0;
    const double d[3] = {dx, dy, dz};
    for (int a = 0; a < 3; ++a) {
        const double len = cell[a] - fabs(d[a]);
        if (!(len > 0.0))
            return 0.0;
        ov *= len;
    }
    return ov;
}

void orc_st_pairs(const orc_beam *A, const orc_beam *B, const int64_t *rows, int64_t n_rows,
                  double dt, int32_t k0, int32_t n_steps, const double *cell, double *out)
{
    const int64_t nr = rows ? n_rows : A->n;
    const double vol = cell[0] * cell[1] * cell[2];
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4)
#endif
    for (int64_t a = 0; a < nr; ++a) {
        const int64_t i = rows ? rows[a] : a;
        const double Ei = A->E[i];
        const double ui[3] = {A->px[i] / Ei, A->py[i] / Ei, A->pz[i] / Ei};
        for (int64_t j = 0; j < B->n; ++j) {
            const double Ej = B->E[j];
            const double uj[3] = {B->px[j] / Ej, B->py[j] / Ej, B->pz[j] / Ej};
            const double s = orc_invariant(Ei, ui[0], ui[1], ui[2], Ej, uj[0], uj[1], uj[2]);
            double y = 0.0;
            if (s > 1.0) {
                const double dens2 = (A->w[i] * B->w[j]) / (vol * vol);
                const double rate = dens2 * orc_sigma(s);
                const double cosphi = (ui[0] * uj[0] + ui[1] * uj[1]) + ui[2] * uj[2];
                for (int32_t k = k0; k < k0 + n_steps; ++k) {
                    const double tm = (double)k * dt + 0.5 * dt;
                    const double dx = (A->x[i] + tm * ui[0]) - (B->x[j] + tm * uj[0]);
                    const double dy = (A->y[i] + tm * ui[1]) - (B->y[j] + tm * uj[1]);
                    const double dz = (A->z[i] + tm * ui[2]) - (B->z[j] + tm * uj[2]);
                    const double ov = orc_cloud_overlap(dx, dy, dz, cell);
                    if (ov > 0.0)
                        y += ((rate * (1.0 - cosphi)) * dt) * ov;
                }
            }
            out[a * B->n + j] = y;
        }
    }
}

/* Exposure of every cloud pair for the depletion picture (Sec. 2.2, the rate equation
 * integrated with the loss of collision partners): per pair, summed over steps k0 ..
 * k0+n_steps-1 at mid-step,
 *   S = sum_k sigma(s) (1 - u_i.u_j) dt V_ov / V,
 * i.e. k tau of the closed forms with k = sigma c (1 - cos phi) and the time weighted by the
 * fraction of a cloud's volume the two clouds share. out[a * nB + j] as in orc_st_pairs. */
void orc_st_exposure(const orc_beam *A, const orc_beam *B, const int64_t *rows, int64_t n_rows,
                     double dt, int32_t k0, int32_t n_steps, const double *cell, double *out)
{
    const int64_t nr = rows ? n_rows : A->n;
    const double vol = cell[0] * cell[1] * cell[2];
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4)
#endif
    for (int64_t a = 0; a < nr; ++a) {
        const int64_t i = rows ? rows[a] : a;
        const double Ei = A->E[i];
        const double ui[3] = {A->px[i] / Ei, A->py[i] / Ei, A->pz[i] / Ei};
        for (int64_t j = 0; j < B->n; ++j) {
            const double Ej = B->E[j];
            const double uj[3] = {B->px[j] / Ej, B->py[j] / Ej, B->pz[j] / Ej};
            const double s = orc_invariant(Ei, ui[0], ui[1], ui[2], Ej, uj[0], uj[1], uj[2]);
            double x = 0.0;
            if (s > 1.0) {
                const double sig = orc_sigma(s);
                const double cosphi = (ui[0] * uj[0] + ui[1] * uj[1]) + ui[2] * uj[2];
                for (int32_t k = k0; k < k0 + n_steps; ++k) {
                    const double tm = (double)k * dt + 0.5 * dt;
                    const double dx = (A->x[i] + tm * ui[0]) - (B->x[j] + tm * uj[0]);
                    const double dy = (A->y[i] + tm * ui[1]) - (B->y[j] + tm * uj[1]);
                    const double dz = (A->z[i] + tm * ui[2]) - (B->z[j] + tm * uj[2]);
                    const double ov = orc_cloud_overlap(dx, dy, dz, cell);
                    if (ov > 0.0)
                        x += (((sig * (1.0 - cosphi)) * dt) * ov) / vol;
                }
            }
            out[a * B->n + j] = x;
        }
    }
}

/* ---- individual-particle (IP) regime: swarms --------------------------------------
 *
 * Sec. 2.2: when two macro-particles meet, each is split into a swarm of real photons with
 * its momentum, placed as evenly as possible over its volume and held in an octree. Here a
 * macro-particle of weight w is floor(w + 1/2) real photons filling its cloud box (edges
 * cell[0..2] about its position). Real photon k sits at the centre of the level-L octree
 * cell (8^L >= n, L smallest) whose octant at level l is base-8 digit l of k (lowest digit =
 * top level; bits 2, 1, 0 of a digit pick the upper half along x, y, z), so that the first 8
 * photons take one octant each, the first 64 one sub-octant each, and so on. Two real
 * photons collide when their time-synchronous distance over the run window
 * [k0 dt, (k0 + n_steps) dt] comes within r, r^2 = sigma(s) / pi (weight 1 each), s that of
 * their macro-particles. out[a * nB + j] = colliding real pairs of macro-particle pair
 * (rows[a], j); *knife counts real pairs with |d^2 - r^2| < 2^-40 r^2. */
static int orc_swarm_level(int64_t n)
{
    int L = 0;
    int64_t cells = 1;
    while (cells < n) {
        cells *= 8;
        ++L;
    }
    return L;
}

static void orc_swarm_offset(int64_t k, int L, const double *cell, double o[3])
{
    int64_t c[3] = {0, 0, 0};
    for (int l = 0; l < L; ++l) {
        const int d = (int)((k >> (3 * l)) & 7);
        c[0] = 2 * c[0] + ((d >> 2) & 1);
        c[1] = 2 * c[1] + ((d >> 1) & 1);
        c[2] = 2 * c[2] + (d & 1);
    }
    const double cells = (double)((int64_t)1 << L);
    for (int a = 0; a < 3; ++a) {
        const double h = cell[a] / cells;
        o[a] = ((double)c[a] + 0.5) * h - 0.5 * cell[a];
    }
}

void orc_swarm_offsets(int64_t n, const double *cell, double *out)
{
    const int L = orc_swarm_level(n);
    for (int64_t k = 0; k < n; ++k) orc_swarm_offset(k, L, cell, out + 3 * k);
}

void orc_swarm_pairs(const orc_beam *A, const orc_beam *B, const int64_t *rows, int64_t n_rows,
                     double dt, int32_t k0, int32_t n_steps, const double *cell, int64_t *out,
                     int64_t *knife)
{
    const int64_t nr = rows ? n_rows : A->n;
    const double T0 = (double)k0 * dt, Tw = (double)n_steps * dt;
    int64_t kn = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : kn)
#endif
    for (int64_t a = 0; a < nr; ++a) {
        const int64_t i = rows ? rows[a] : a;
        const double Ei = A->E[i];
        const double ui[3] = {A->px[i] / Ei, A->py[i] / Ei, A->pz[i] / Ei};
        const int64_t ni = (int64_t)floor(A->w[i] + 0.5);
        const int Li = orc_swarm_level(ni);
        for (int64_t j = 0; j < B->n; ++j) {
            const double Ej = B->E[j];
            const double uj[3] = {B->px[j] / Ej, B->py[j] / Ej, B->pz[j] / Ej};
            const double s = orc_invariant(Ei, ui[0], ui[1], ui[2], Ej, uj[0], uj[1], uj[2]);
            int64_t cnt = 0;
            const int64_t nj = (int64_t)floor(B->w[j] + 0.5);
            if (s > 1.0 && ni > 0 && nj > 0) {
                const double r2 = orc_sigma(s) / M_PI;
                const int Lj = orc_swarm_level(nj);
                for (int64_t p = 0; p < ni; ++p) {
                    double op[3];
                    orc_swarm_offset(p, Li, cell, op);
                    for (int64_t q = 0; q < nj; ++q) {
                        double oq[3], tau;
                        orc_swarm_offset(q, Lj, cell, oq);
                        const double d2 = orc_step_closest(
                            T0, Tw, A->x[i] + op[0], A->y[i] + op[1], A->z[i] + op[2], ui[0],
                            ui[1], ui[2], B->x[j] + oq[0], B->y[j] + oq[1], B->z[j] + oq[2],
                            uj[0], uj[1], uj[2], &tau);
                        if (fabs(r2 - d2) < 0x1p-40 * r2) ++kn;
                        if (d2 <= r2) ++cnt;
                    }
                }
            }
            out[a * B->n + j] = cnt;
        }
    }
    *knife = kn;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
