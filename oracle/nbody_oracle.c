/*
 * nbody_oracle.c -- FP64 CPU oracle of the direct-summation Hermite block-step scheme of
 * Portegies Zwart, Belleman & Geldof (2007), "High Performance Direct Gravitational N-body
 * Simulations on Graphics Processing Units".
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call this file;
 * only the test suite, the smoke check and the CPU-baseline leg of the benchmark do.
 * It shares no code, header or constant with the HIP library.
 *
 * Everything is IEEE double precision (no -ffast-math).  Force and energy sums are
 * accumulated in `long double` (x87 80-bit on x86-64) so that the oracle's own rounding error
 * stays far below the 1e-11 tolerance the double-single GPU form is checked against.
 *
 * Layout: positions, velocities, accelerations and jerks are AoS, n x 3 doubles.
 * Time is counted in integer ticks of 2^-lmax (lmax = 26 by default, the paper's minimum
 * time step); a particle on level l has time step 2^-l = 2^(lmax-l) ticks.
 *
 * Readings of the paper that this code takes (each listed with its reason in the design notes):
 *  - Eq. Force is printed with r_i - r_j in the numerator; gravity is attractive, and the
 *    App. A kernel uses the separation d = r_j - r_i, which is what is computed here.
 *  - The softened form of App. A is used: s = |d|^2 + eps^2, G = 1.
 *  - j = i is excluded from all sums (Eq. Force), including the potential.
 *  - In the corrector, Delta a = a - a_p = (old acceleration) - (new acceleration).
 *  - The time-step criterion (Eq. timestep) uses magnitudes: the new acceleration a_1, the
 *    new jerk k_1, a2_p = a2 + a3 dt and a3 from the corrector; the initial step
 *    (Eq. initTimestep) is nu |a| / |k|.
 *  - Block steps: levels are powers of two (Sec. 2, integration-step list).  A step may
 *    shrink by any power of two, and may double only when the particle's time is a multiple
 *    of the doubled step (the commensurability rule of the block scheme the paper cites).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef long double acc_t;

/* Number of threads the parallel loops below use. */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------------------------
 * Sec. 2 Eq. Force with the softening of App. A.  For each listed i: the acceleration
 *   a_i = sum_{j != i} m_j d s^{-3/2},
 * its time derivative (the jerk) along the current velocities
 *   k_i = sum_{j != i} m_j [ u s^{-3/2} - 3 (d.u) d s^{-5/2} ],
 * and the potential  phi_i = - sum_{j != i} m_j s^{-1/2},
 * with d = x_j - x_i, u = v_j - v_i, s = |d|^2 + eps2.  The i-particle's own position and
 * velocity are row idx[q] of x and v.  Outputs are n_i x 3 (acc, jerk) and n_i (pot).
 * ------------------------------------------------------------------------------------------ */
void orc_force(int64_t n_i, const int64_t *idx, int64_t n, const double *x, const double *v,
               const double *m, double eps2, double *acc, double *jerk, double *pot)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < n_i; ++q) {
        const int64_t i = idx[q];
        acc_t ax = 0, ay = 0, az = 0, jx = 0, jy = 0, jz = 0, p = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const double dx = x[3 * j + 0] - x[3 * i + 0];
            const double dy = x[3 * j + 1] - x[3 * i + 1];
            const double dz = x[3 * j + 2] - x[3 * i + 2];
            const double ux = v[3 * j + 0] - v[3 * i + 0];
            const double uy = v[3 * j + 1] - v[3 * i + 1];
            const double uz = v[3 * j + 2] - v[3 * i + 2];
            const double s = dx * dx + dy * dy + dz * dz + eps2;
            const double r = sqrt(s);
            const double inv_r = 1.0 / r;          /* s^{-1/2} */
            const double inv_r3 = inv_r / s;       /* s^{-3/2} */
            const double inv_r5 = inv_r3 / s;      /* s^{-5/2} */
            const double du = dx * ux + dy * uy + dz * uz;
            const double mj = m[j];
            ax += mj * dx * inv_r3;
            ay += mj * dy * inv_r3;
            az += mj * dz * inv_r3;
            jx += mj * (ux * inv_r3 - 3.0 * du * dx * inv_r5);
            jy += mj * (uy * inv_r3 - 3.0 * du * dy * inv_r5);
            jz += mj * (uz * inv_r3 - 3.0 * du * dz * inv_r5);
            p -= mj * inv_r;
        }
        acc[3 * q + 0] = (double)ax;
        acc[3 * q + 1] = (double)ay;
        acc[3 * q + 2] = (double)az;
        jerk[3 * q + 0] = (double)jx;
        jerk[3 * q + 1] = (double)jy;
        jerk[3 * q + 2] = (double)jz;
        pot[q] = (double)p;
    }
}

/* ------------------------------------------------------------------------------------------
 * Size of the terms of Eq. Force on each listed i, the scale against which the rounding of a
 * sum of those terms is measured (a sum of terms rounded to relative u has an error of at most
 * about u times the sum of the terms' magnitudes, however much the terms cancel):
 *   sa_i = sum_{j != i} m_j |d| s^{-3/2}                                (the pulls' sizes)
 *   sk_i = sum_{j != i} m_j ( |u| s^{-3/2} + 3 |d.u| |d| s^{-5/2} )    (both jerk parts)
 * with d, u, s as in orc_force.
 * ------------------------------------------------------------------------------------------ */
void orc_force_scale(int64_t n_i, const int64_t *idx, int64_t n, const double *x,
                     const double *v, const double *m, double eps2, double *sa, double *sk)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < n_i; ++q) {
        const int64_t i = idx[q];
        acc_t a = 0, k = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const double dx = x[3 * j + 0] - x[3 * i + 0];
            const double dy = x[3 * j + 1] - x[3 * i + 1];
            const double dz = x[3 * j + 2] - x[3 * i + 2];
            const double ux = v[3 * j + 0] - v[3 * i + 0];
            const double uy = v[3 * j + 1] - v[3 * i + 1];
            const double uz = v[3 * j + 2] - v[3 * i + 2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double s = r2 + eps2;
            const double inv_r3 = 1.0 / (s * sqrt(s));
            const double dist = sqrt(r2), speed = sqrt(ux * ux + uy * uy + uz * uz);
            const double du = fabs(dx * ux + dy * uy + dz * uz);
            a += m[j] * dist * inv_r3;
            k += m[j] * (speed * inv_r3 + 3.0 * du * dist * inv_r3 / s);
        }
        sa[q] = (double)a;
        sk[q] = (double)k;
    }
}

/* ------------------------------------------------------------------------------------------
 * Sec. 4.2 energy diagnostic: kinetic energy sum_i m_i |v_i|^2 / 2 and potential energy
 * -1/2 sum_i sum_{j != i} m_i m_j s^{-1/2} (softened, the same potential the force derives
 * from).  Written to ekin and epot.
 * ------------------------------------------------------------------------------------------ */
void orc_energy(int64_t n, const double *x, const double *v, const double *m, double eps2,
                double *ekin, double *epot)
{
    acc_t t = 0;
    for (int64_t i = 0; i < n; ++i)
        t += 0.5L * m[i] * ((acc_t)v[3 * i] * v[3 * i] + (acc_t)v[3 * i + 1] * v[3 * i + 1] +
                            (acc_t)v[3 * i + 2] * v[3 * i + 2]);
    double *part = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        acc_t w = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const double dx = x[3 * j + 0] - x[3 * i + 0];
            const double dy = x[3 * j + 1] - x[3 * i + 1];
            const double dz = x[3 * j + 2] - x[3 * i + 2];
            w += m[j] / sqrt(dx * dx + dy * dy + dz * dz + eps2);
        }
        part[i] = (double)(m[i] * w);
    }
    acc_t w = 0;
    for (int64_t i = 0; i < n; ++i) w += part[i];
    free(part);
    *ekin = (double)t;
    *epot = (double)(-0.5L * w);
}

/* ------------------------------------------------------------------------------------------
 * Sec. 2 predictor: third-order Taylor step of position and second-order of velocity,
 *   x_p = x + v D + a D^2/2 + k D^3/6,   v_p = v + a D + k D^2/2,
 * for every particle, D = (t_target - t_i) * tick.
 * ------------------------------------------------------------------------------------------ */
static void predict_one(double D, const double *x, const double *v, const double *a,
                        const double *k, double *xp, double *vp)
{
    for (int c = 0; c < 3; ++c) {
        xp[c] = x[c] + v[c] * D + a[c] * D * D / 2.0 + k[c] * D * D * D / 6.0;
        vp[c] = v[c] + a[c] * D + k[c] * D * D / 2.0;
    }
}

void orc_predict(int64_t n, const double *x, const double *v, const double *a, const double *k,
                 const int64_t *tick, int64_t t_target, double tick_len, double *xp, double *vp)
{
    for (int64_t i = 0; i < n; ++i)
        predict_one((double)(t_target - tick[i]) * tick_len, x + 3 * i, v + 3 * i, a + 3 * i,
                    k + 3 * i, xp + 3 * i, vp + 3 * i);
}

/* ------------------------------------------------------------------------------------------
 * Sec. 2 corrector for one particle (the rows q of the n_act-long arrays):
 *   a2 = -6 (a0 - a1)/dt^2 - (4 k0 + 2 k1)/dt,
 *   a3 = 12 (a0 - a1)/dt^3 + 6 (k0 + k1)/dt^2,
 *   x  = x_p + a2 dt^4/24 + a3 dt^5/120,   v = v_p + a2 dt^3/6 + a3 dt^4/24,
 * then the quantities the time-step criterion (Eq. timestep) needs:
 *   a2p = a2 + a3 dt,
 *   crit_num = |a1| |a2p| + |k1|^2,  crit_den = |k1| |a3| + |a2p|^2.
 * x, v are overwritten with the corrected values; a0, k0 are replaced by a1, k1.
 * ------------------------------------------------------------------------------------------ */
static void correct_one(double dt, const double *xp, const double *vp, double *x, double *v,
                        double *a0, double *k0, const double *a1, const double *k1,
                        double *crit_num, double *crit_den)
{
    double a2[3], a3[3], a2p[3];
    for (int c = 0; c < 3; ++c) {
        const double da = a0[c] - a1[c];
        a2[c] = -6.0 * da / (dt * dt) - (4.0 * k0[c] + 2.0 * k1[c]) / dt;
        a3[c] = 12.0 * da / (dt * dt * dt) + 6.0 * (k0[c] + k1[c]) / (dt * dt);
    }
    for (int c = 0; c < 3; ++c) {
        x[c] = xp[c] + a2[c] * dt * dt * dt * dt / 24.0 + a3[c] * dt * dt * dt * dt * dt / 120.0;
        v[c] = vp[c] + a2[c] * dt * dt * dt / 6.0 + a3[c] * dt * dt * dt * dt / 24.0;
        a2p[c] = a2[c] + a3[c] * dt;
        a0[c] = a1[c];
        k0[c] = k1[c];
    }
    const double na1 = sqrt(a1[0] * a1[0] + a1[1] * a1[1] + a1[2] * a1[2]);
    const double nk1 = sqrt(k1[0] * k1[0] + k1[1] * k1[1] + k1[2] * k1[2]);
    const double na2p = sqrt(a2p[0] * a2p[0] + a2p[1] * a2p[1] + a2p[2] * a2p[2]);
    const double na3 = sqrt(a3[0] * a3[0] + a3[1] * a3[1] + a3[2] * a3[2]);
    *crit_num = na1 * na2p + nk1 * nk1;
    *crit_den = nk1 * na3 + na2p * na2p;
}

/* Correct the listed particles (block of n_act, indices idx) over their step dt_q = 2^-level.
 * xp, vp are the predicted state of all particles (n x 3); a1, k1, pot1 are n_act-long.
 * The criterion inputs are written to crit (n_act x 2: numerator, denominator). */
void orc_correct(int64_t n_act, const int64_t *idx, const int32_t *level, const double *xp,
                 const double *vp, const double *a1, const double *k1, const double *pot1,
                 double *x, double *v, double *a, double *k, double *pot, double *crit)
{
    for (int64_t q = 0; q < n_act; ++q) {
        const int64_t i = idx[q];
        const double dt = ldexp(1.0, -level[i]);
        correct_one(dt, xp + 3 * i, vp + 3 * i, x + 3 * i, v + 3 * i, a + 3 * i, k + 3 * i,
                    a1 + 3 * q, k1 + 3 * q, crit + 2 * q, crit + 2 * q + 1);
        pot[i] = pot1[q];
    }
}

/* Eq. timestep: dt = ( nu * crit_num / crit_den )^{1/2}.  A zero denominator means no
 * constraint (infinite step). */
double orc_aarseth_dt(double nu, double crit_num, double crit_den)
{
    if (!(crit_den > 0.0)) return INFINITY;
    return sqrt(nu * crit_num / crit_den);
}

/* Eq. initTimestep: dt = nu |a| / |k|. */
double orc_initial_dt(double nu, const double *a, const double *k)
{
    const double na = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    const double nk = sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
    if (!(nk > 0.0)) return INFINITY;
    return nu * na / nk;
}

/* Power-of-two quantisation of a fresh step (Sec. 2, block steps): the largest 2^-l with
 * lmin <= l <= lmax and 2^-l <= dt_raw; l = lmax if even 2^-lmax exceeds dt_raw. */
int32_t orc_level_from_dt(double dt_raw, int32_t lmin, int32_t lmax)
{
    int32_t l = lmin;
    while (l < lmax && ldexp(1.0, -l) > dt_raw) ++l;
    return l;
}

/* New level of a particle just advanced to tick t (on level l_old): shrink by halving until
 * the step is no longer above dt_raw; otherwise double once if dt_raw allows twice the old
 * step, the doubled step does not exceed 2^-lmin, and t is a multiple of the doubled step. */
int32_t orc_next_level(double dt_raw, int32_t l_old, int64_t t, int32_t lmin, int32_t lmax)
{
    int32_t l = l_old;
    if (dt_raw < ldexp(1.0, -l)) {
        while (l < lmax && ldexp(1.0, -l) > dt_raw) ++l;
        return l;
    }
    if (l > lmin && dt_raw >= ldexp(1.0, -(l - 1))) {
        const int64_t two_dt = (int64_t)1 << (lmax - l + 1);
        if (t % two_dt == 0) return l - 1;
    }
    return l;
}

/* Sec. 2 block selection: t_next = min_i (t_i + dt_i), and the block is every i with
 * t_i + dt_i == t_next, listed in ascending index.  Returns t_next, writes n_act. */
int64_t orc_select_block(int64_t n, const int64_t *tick, const int32_t *level, int32_t lmax,
                         int64_t *idx, int64_t *n_act)
{
    int64_t t_next = INT64_MAX;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t tn = tick[i] + ((int64_t)1 << (lmax - level[i]));
        if (tn < t_next) t_next = tn;
    }
    int64_t c = 0;
    for (int64_t i = 0; i < n; ++i)
        if (tick[i] + ((int64_t)1 << (lmax - level[i])) == t_next) idx[c++] = i;
    *n_act = c;
    return t_next;
}

/* ------------------------------------------------------------------------------------------
 * Start of a run (Sec. 2): full force on every particle at t = 0, initial step from
 * Eq. initTimestep, every particle's time set to 0.
 * ------------------------------------------------------------------------------------------ */
void orc_init(int64_t n, const double *x, const double *v, const double *m, double eps2,
              double nu, int32_t lmin, int32_t lmax, double *a, double *k, double *pot,
              int64_t *tick, int32_t *level)
{
    int64_t *all = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) all[i] = i;
    orc_force(n, all, n, x, v, m, eps2, a, k, pot);
    for (int64_t i = 0; i < n; ++i) {
        tick[i] = 0;
        level[i] = orc_level_from_dt(orc_initial_dt(nu, a + 3 * i, k + 3 * i), lmin, lmax);
    }
    free(all);
}

/* ------------------------------------------------------------------------------------------
 * One integration step of Sec. 2, in the paper's order:
 *  1. choose the block: the particles with the smallest t_i + dt_i;
 *  2. predict all particles to that time;
 *  3. recompute acceleration and jerk (and potential) of the block from the predicted
 *     positions and velocities of all particles;
 *  4. correct the block and give each particle of the block its new step (Eq. timestep).
 * Returns t_next; the block is left in idx[0..*n_act).  dt_raw (n-long, may be NULL)
 * receives the unquantised criterion value of each corrected particle.
 * *n_dtmin counts particles that wanted a step below 2^-lmax (clamped).
 * ------------------------------------------------------------------------------------------ */
int64_t orc_block_step(int64_t n, double *x, double *v, double *a, double *k, const double *m,
                       double *pot, int64_t *tick, int32_t *level, double eps2, double nu,
                       int32_t lmin, int32_t lmax, int64_t *idx, int64_t *n_act, double *dt_raw,
                       int64_t *n_dtmin)
{
    const double tick_len = ldexp(1.0, -lmax);
    const int64_t t_next = orc_select_block(n, tick, level, lmax, idx, n_act);
    const int64_t na = *n_act;

    double *xp = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *vp = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *a1 = (double *)malloc(sizeof(double) * 3 * (size_t)na);
    double *k1 = (double *)malloc(sizeof(double) * 3 * (size_t)na);
    double *p1 = (double *)malloc(sizeof(double) * (size_t)na);
    double *crit = (double *)malloc(sizeof(double) * 2 * (size_t)na);

    orc_predict(n, x, v, a, k, tick, t_next, tick_len, xp, vp);
    orc_force(na, idx, n, xp, vp, m, eps2, a1, k1, p1);
    orc_correct(na, idx, level, xp, vp, a1, k1, p1, x, v, a, k, pot, crit);
    for (int64_t q = 0; q < na; ++q) {
        const int64_t i = idx[q];
        const double dr = orc_aarseth_dt(nu, crit[2 * q], crit[2 * q + 1]);
        if (dt_raw) dt_raw[i] = dr;
        if (n_dtmin && dr < tick_len) ++*n_dtmin;
        tick[i] = t_next;
        level[i] = orc_next_level(dr, level[i], t_next, lmin, lmax);
    }
    free(xp); free(vp); free(a1); free(k1); free(p1); free(crit);
    return t_next;
}

/* Shared-step mode: every particle advanced together by the fixed step dt (the same
 * predictor, force and corrector; no time-step criterion). */
void orc_shared_step(int64_t n, double *x, double *v, double *a, double *k, const double *m,
                     double *pot, double eps2, double dt)
{
    double *xp = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *vp = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *a1 = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *k1 = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *p1 = (double *)malloc(sizeof(double) * (size_t)n);
    int64_t *all = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) all[i] = i;
    for (int64_t i = 0; i < n; ++i)
        predict_one(dt, x + 3 * i, v + 3 * i, a + 3 * i, k + 3 * i, xp + 3 * i, vp + 3 * i);
    orc_force(n, all, n, xp, vp, m, eps2, a1, k1, p1);
    for (int64_t i = 0; i < n; ++i) {
        double cn, cd;
        correct_one(dt, xp + 3 * i, vp + 3 * i, x + 3 * i, v + 3 * i, a + 3 * i, k + 3 * i,
                    a1 + 3 * i, k1 + 3 * i, &cn, &cd);
        pot[i] = p1[i];
    }
    free(xp); free(vp); free(a1); free(k1); free(p1); free(all);
}
