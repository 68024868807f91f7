/*
 * nbody_oracle.c -- CPU FP64 reference for the direct-sum (particle-particle)
 * N-body step.  TEST INFRASTRUCTURE ONLY: this file is the checker that the
 * GPU library is compared against.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it; the product never does.
 *
 * It is deliberately plain: scalar double arithmetic, IEEE sqrt and
 * division, no blocking, no fused multiply-add (built with
 * -ffp-contract=off), the j sum taken in index order.  Parallelism is over
 * target particles i only, so every result is independent of the thread
 * count.  It shares no source with the GPU kernels.
 *
 * Paper: Khrapov, Khoperskov & Khoperskov, "New features of parallel
 * implementation of N-body problems on GPU" (2018).
 *
 * Readings taken where the paper is silent or garbled:
 *  - Eq. (2)'s denominator |r_i - r_j + delta| is the Plummer-softened
 *    distance sqrt(|r_i - r_j|^2 + delta^2), as the text under Eq. (2) defines.
 *  - A pair whose softened distance is exactly zero (delta = 0 and coincident
 *    particles) contributes nothing.
 *  - Eq. (8) prints the potential term with a plus sign; gravity needs a minus.
 *  - Eq. (10) is the z-component of L; the full vector is returned.
 *  - The fixed halo is not in the paper (its disk is fully self-gravitating);
 *    it is an optional external field: a cored isothermal sphere.
 *  - The "fourth-order scheme" of the abstract is not named; the triple-jump
 *    composition of the leapfrog step (Yoshida 1990; Forest & Ruth 1990) is used,
 *    and the fourth-order Hermite scheme and classical RK4 are provided too.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int on;       /* 0: no external field */
    double v2;    /* asymptotic circular speed squared V_inf^2 */
    double rc;    /* core radius */
} orc_halo;

static void set_threads(int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Eqs. (1)-(2): a_i = sum_{j != i} f_ij with
 *   f_ij = -G m_j (r_i - r_j) / (|r_i - r_j|^2 + delta^2)^{3/2}.
 * Also, when requested:
 *   phi_i = -sum_{j != i} G m_j / sqrt(|r_i - r_j|^2 + delta^2)   (potential)
 *   A_i   =  sum_{j != i} |f_ij|                                 (force scale)
 * rows == NULL evaluates every i (outputs of length n); otherwise the nrows
 * listed targets (outputs of length nrows).  reverse_j sums j from n-1 down.
 */
static void accel_one(int64_t n, const double *x, const double *y, const double *z,
                      const double *m, double G, double eps, int64_t i, int reverse_j,
                      double *oax, double *oay, double *oaz, double *ophi, double *oA) {
    const double d2 = eps * eps;
    double ax = 0.0, ay = 0.0, az = 0.0, phi = 0.0, A = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        const int64_t j = reverse_j ? (n - 1 - k) : k;
        if (j == i) continue;                       /* Eq. (1): j != i */
        const double dx = x[i] - x[j];
        const double dy = y[i] - y[j];
        const double dz = z[i] - z[j];
        const double r2 = dx * dx + dy * dy + dz * dz + d2;
        if (r2 == 0.0) continue;                    /* zero softened distance */
        const double r = sqrt(r2);
        const double r3 = r2 * r;
        const double s = G * m[j] / r3;
        ax -= s * dx;                               /* f_ij = -G m_j (r_i - r_j) / r^3 */
        ay -= s * dy;
        az -= s * dz;
        phi -= G * m[j] / r;
        A += s * sqrt(dx * dx + dy * dy + dz * dz);
    }
    *oax = ax; *oay = ay; *oaz = az;
    if (ophi) *ophi = phi;
    if (oA) *oA = A;
}

void orc_accel(int64_t n, const double *x, const double *y, const double *z, const double *m,
               double G, double eps, const int64_t *rows, int64_t nrows, int reverse_j,
               double *ax, double *ay, double *az, double *phi, double *A, int nthreads) {
    set_threads(nthreads);
    const int64_t cnt = rows ? nrows : n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < cnt; ++q) {
        const int64_t i = rows ? rows[q] : q;
        accel_one(n, x, y, z, m, G, eps, i, reverse_j, &ax[q], &ay[q], &az[q],
                  phi ? &phi[q] : NULL, A ? &A[q] : NULL);
    }
}

/* ------------------------------------------------------------------------ */
/* Cored isothermal halo, density rho0 / (1 + r^2/rc^2), V_inf^2 = 4 pi G rho0 rc^2.
 * Enclosed mass G M(<r) = V_inf^2 (r - rc atan(r/rc)), so with s = r/rc
 *   a_h = -(G M(<r) / r^3) r_vec = -V_inf^2 (1 - atan(s)/s) r_vec / r^2.
 * The potential diverges logarithmically at infinity, so its constant is
 * chosen to give Phi(r) = V_inf^2 [atan(s)/s + ln(1 + s^2)/2], which has
 * dPhi/dr = V_c^2 / r and Phi(0) = V_inf^2.
 * 1 - atan(s)/s cancels for small s, so below s = 1/2 it is summed from its
 * Taylor series sum_{k>=1} (-1)^{k+1} s^{2k} / (2k + 1) instead. */
static double halo_series_over_s2(double s) {
    /* (1 - atan(s)/s) / s^2 = 1/3 - s^2/5 + s^4/7 - ... for s < 1/2 */
    const double s2 = s * s;
    double term = 1.0, sum = 0.0;
    for (int k = 1; k <= 40; ++k) {
        sum += ((k % 2) ? term : -term) / (2.0 * k + 1.0);
        term *= s2;
    }
    return sum;
}

static double halo_g_over_r(double r, double v2, double rc) {
    /* returns G M(<r) / r^3 */
    const double s = r / rc;
    if (s < 0.5) return v2 / (rc * rc) * halo_series_over_s2(s);
    return v2 * (1.0 - atan(s) / s) / (r * r);
}

static double halo_phi(double r, double v2, double rc) {
    const double s = r / rc;
    const double atan_over_s = (s < 0.5) ? 1.0 - s * s * halo_series_over_s2(s) : atan(s) / s;
    return v2 * (atan_over_s + 0.5 * log1p(s * s));
}

void orc_halo_accel(int64_t n, const double *x, const double *y, const double *z, double v2,
                    double rc, double *ax, double *ay, double *az, double *phi) {
    for (int64_t i = 0; i < n; ++i) {
        const double r = sqrt(x[i] * x[i] + y[i] * y[i] + z[i] * z[i]);
        const double g = halo_g_over_r(r, v2, rc);
        ax[i] = -g * x[i];
        ay[i] = -g * y[i];
        az[i] = -g * z[i];
        if (phi) phi[i] = halo_phi(r, v2, rc);
    }
}

/* total acceleration: self-gravity plus the optional halo */
static void total_accel(int64_t n, const double *x, const double *y, const double *z,
                        const double *m, double G, double eps, const orc_halo *h,
                        int reverse_j, double *ax, double *ay, double *az, int nthreads) {
    orc_accel(n, x, y, z, m, G, eps, NULL, 0, reverse_j, ax, ay, az, NULL, NULL, nthreads);
    if (h && h->on) {
        for (int64_t i = 0; i < n; ++i) {
            const double r = sqrt(x[i] * x[i] + y[i] * y[i] + z[i] * z[i]);
            const double g = halo_g_over_r(r, h->v2, h->rc);
            ax[i] += -g * x[i];
            ay[i] += -g * y[i];
            az[i] += -g * z[i];
        }
    }
}

static int64_t g_force_evals = 0;
int64_t orc_force_evals(void) { return g_force_evals; }
void orc_reset_force_evals(void) { g_force_evals = 0; }

/* ------------------------------------------------------------------------ */
/* Section 1, Eqs. (5)-(7): leapfrog kick-drift-kick with one force
 * evaluation per step.  On entry a must hold the acceleration at r; on
 * return it holds the acceleration at the final r.
 *
 * paper_form = 1 follows the printed predictor / drift / corrector:
 *   v~ = v + dt a(t);  r += dt/2 (v~ + v);  a(t+dt);  v = (v + v~)/2 + dt/2 a(t+dt)
 * paper_form = 0 uses the algebraically identical half-kick form:
 *   v += dt/2 a;  r += dt v;  a(t+dt);  v += dt/2 a(t+dt)
 */
static void kdk_once(int64_t n, double *x, double *y, double *z, double *vx, double *vy,
                     double *vz, const double *m, double *ax, double *ay, double *az, double G,
                     double eps, const orc_halo *h, double dt, int paper_form, int reverse_j,
                     int nthreads) {
    if (paper_form) {
        for (int64_t i = 0; i < n; ++i) {
            const double wx = vx[i] + dt * ax[i];
            const double wy = vy[i] + dt * ay[i];
            const double wz = vz[i] + dt * az[i];
            x[i] += dt / 2.0 * (wx + vx[i]);
            y[i] += dt / 2.0 * (wy + vy[i]);
            z[i] += dt / 2.0 * (wz + vz[i]);
            /* keep (v + v~)/2 in v until the new force is known */
            vx[i] = (vx[i] + wx) / 2.0;
            vy[i] = (vy[i] + wy) / 2.0;
            vz[i] = (vz[i] + wz) / 2.0;
        }
    } else {
        for (int64_t i = 0; i < n; ++i) {
            vx[i] += dt / 2.0 * ax[i];
            vy[i] += dt / 2.0 * ay[i];
            vz[i] += dt / 2.0 * az[i];
            x[i] += dt * vx[i];
            y[i] += dt * vy[i];
            z[i] += dt * vz[i];
        }
    }
    total_accel(n, x, y, z, m, G, eps, h, reverse_j, ax, ay, az, nthreads);
    ++g_force_evals;
    for (int64_t i = 0; i < n; ++i) {
        vx[i] += dt / 2.0 * ax[i];
        vy[i] += dt / 2.0 * ay[i];
        vz[i] += dt / 2.0 * az[i];
    }
}

void orc_step_kdk(int64_t n, double *x, double *y, double *z, double *vx, double *vy, double *vz,
                  const double *m, double *ax, double *ay, double *az, double G, double eps,
                  const orc_halo *h, double dt, int64_t nsteps, int paper_form, int reverse_j,
                  int nthreads) {
    for (int64_t s = 0; s < nsteps; ++s)
        kdk_once(n, x, y, z, vx, vy, vz, m, ax, ay, az, G, eps, h, dt, paper_form, reverse_j,
                 nthreads);
}

/* Fourth order: S4(dt) = S2(w1 dt) S2(w0 dt) S2(w1 dt) where S2 is the
 * leapfrog step above and (w1, w0) satisfy 2 w1 + w0 = 1, 2 w1^3 + w0^3 = 0
 * (the caller passes them).  Three force evaluations per step. */
void orc_step_o4(int64_t n, double *x, double *y, double *z, double *vx, double *vy, double *vz,
                 const double *m, double *ax, double *ay, double *az, double G, double eps,
                 const orc_halo *h, double dt, int64_t nsteps, double w1, double w0,
                 int reverse_j, int nthreads) {
    for (int64_t s = 0; s < nsteps; ++s) {
        kdk_once(n, x, y, z, vx, vy, vz, m, ax, ay, az, G, eps, h, w1 * dt, 0, reverse_j, nthreads);
        kdk_once(n, x, y, z, vx, vy, vz, m, ax, ay, az, G, eps, h, w0 * dt, 0, reverse_j, nthreads);
        kdk_once(n, x, y, z, vx, vy, vz, m, ax, ay, az, G, eps, h, w1 * dt, 0, reverse_j, nthreads);
    }
}

/* ------------------------------------------------------------------------ */
/* Other fourth-order schemes (the abstract names fourth-order schemes
 * without fixing one; Section 1 compares the leapfrog with Runge-Kutta).
 *
 * Jerk: the time derivative of Eq. (1)'s acceleration when every particle
 * moves with its own velocity.  With r_ji = r_j - r_i, v_ji = v_j - v_i and
 * the softened R^2 = |r_ji|^2 + delta^2,
 *   d/dt [G m_j r_ji / R^3] = G m_j [v_ji / R^3 - 3 (r_ji . v_ji) r_ji / R^5].
 * Halo: a_h = -g(r) r_vec with g = G M(<r) / r^3, so
 *   j_h = -g v - g'(r) (r_vec . v / r) r_vec.
 * With s = r/rc and F(s) = (1 - atan(s)/s) / s^2 (so g = V^2 F / rc^2),
 * g'(r) / r = V^2 H(s) / rc^4 where H(s) = F'(s) / s
 *   = 1/(s^2 (1 + s^2)) - 3/s^4 + 3 atan(s)/s^5,
 * summed below s = 1/2 from its series sum_{k>=2} (-1)^{k+1} (2k-2) s^{2k-4} / (2k+1). */
static double halo_h_series(double s) {
    const double s2 = s * s;
    double term = 1.0, sum = 0.0;
    for (int k = 2; k <= 41; ++k) {
        sum += ((k % 2) ? term : -term) * (2.0 * k - 2.0) / (2.0 * k + 1.0);
        term *= s2;
    }
    return sum;
}

static double halo_h(double s) {
    if (s < 0.5) return halo_h_series(s);
    const double s2 = s * s;
    return 1.0 / (s2 * (1.0 + s2)) - 3.0 / (s2 * s2) + 3.0 * atan(s) / (s2 * s2 * s);
}

/* o[0..5] = a, j of particle i; o[6] = sum |a term|, o[7] = sum of the
 * jerk terms' magnitude bounds G m_j (|u| / R^3 + 3 |r . u| |r| / R^5). */
static void jerk_one(int64_t n, const double *x, const double *y, const double *z,
                     const double *vx, const double *vy, const double *vz, const double *m,
                     double G, double eps, int64_t i, double *o) {
    const double d2 = eps * eps;
    double ax = 0, ay = 0, az = 0, jx = 0, jy = 0, jz = 0, sa = 0, sj = 0;
    for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        const double rx = x[j] - x[i], ry = y[j] - y[i], rz = z[j] - z[i];
        const double ux = vx[j] - vx[i], uy = vy[j] - vy[i], uz = vz[j] - vz[i];
        const double R2 = rx * rx + ry * ry + rz * rz + d2;
        if (R2 == 0.0) continue;
        const double R = sqrt(R2);
        const double R3 = R2 * R;
        const double R5 = R3 * R2;
        const double rv = rx * ux + ry * uy + rz * uz;
        ax += G * m[j] * rx / R3;
        ay += G * m[j] * ry / R3;
        az += G * m[j] * rz / R3;
        jx += G * m[j] * (ux / R3 - 3.0 * rv * rx / R5);
        jy += G * m[j] * (uy / R3 - 3.0 * rv * ry / R5);
        jz += G * m[j] * (uz / R3 - 3.0 * rv * rz / R5);
        const double rl = sqrt(rx * rx + ry * ry + rz * rz);
        sa += G * m[j] * rl / R3;
        sj += G * m[j] * (sqrt(ux * ux + uy * uy + uz * uz) / R3 + 3.0 * fabs(rv) * rl / R5);
    }
    o[0] = ax; o[1] = ay; o[2] = az; o[3] = jx; o[4] = jy; o[5] = jz; o[6] = sa; o[7] = sj;
}

/* acceleration and jerk (plus the halo's when h->on) of every particle, or of
 * the nrows targets listed in rows (outputs of length nrows); sa, sj
 * (nullable): the sums of the self-gravity terms' magnitudes, scales for
 * conditioned error measures. */
void orc_accel_jerk(int64_t n, const double *x, const double *y, const double *z, const double *vx,
                    const double *vy, const double *vz, const double *m, double G, double eps,
                    const orc_halo *h, const int64_t *rows, int64_t nrows, double *ax, double *ay,
                    double *az, double *jx, double *jy, double *jz, double *sa, double *sj, int nthreads) {
    set_threads(nthreads);
    const int64_t cnt = rows ? nrows : n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < cnt; ++q) {
        const int64_t i = rows ? rows[q] : q;
        double o[8];
        jerk_one(n, x, y, z, vx, vy, vz, m, G, eps, i, o);
        if (h && h->on) {
            const double r = sqrt(x[i] * x[i] + y[i] * y[i] + z[i] * z[i]);
            const double g = halo_g_over_r(r, h->v2, h->rc);
            const double hh = h->v2 * halo_h(r / h->rc) / (h->rc * h->rc * h->rc * h->rc);
            const double rv = x[i] * vx[i] + y[i] * vy[i] + z[i] * vz[i];
            o[0] -= g * x[i];
            o[1] -= g * y[i];
            o[2] -= g * z[i];
            o[3] -= g * vx[i] + hh * rv * x[i];
            o[4] -= g * vy[i] + hh * rv * y[i];
            o[5] -= g * vz[i] + hh * rv * z[i];
        }
        ax[q] = o[0]; ay[q] = o[1]; az[q] = o[2]; jx[q] = o[3]; jy[q] = o[4]; jz[q] = o[5];
        if (sa) sa[q] = o[6];
        if (sj) sj[q] = o[7];
    }
}

/* Fourth-order Hermite scheme (Makino & Aarseth 1992), shared step dt:
 * predict r_p = r + v dt + a dt^2/2 + j dt^3/6, v_p = v + a dt + j dt^2/2;
 * evaluate a1, j1 at (r_p, v_p); correct
 *   v' = v + (a + a1) dt/2 + (j - j1) dt^2/12,
 *   r' = r + (v + v') dt/2 + (a - a1) dt^2/12;
 * a, j <- a1, j1.  On entry a and j must hold the values at (r, v); on return
 * they hold those of the predicted state, as the scheme carries them. */
void orc_step_hermite(int64_t n, double *x, double *y, double *z, double *vx, double *vy, double *vz,
                      const double *m, double *ax, double *ay, double *az, double *jx, double *jy,
                      double *jz, double G, double eps, const orc_halo *h, double dt, int64_t nsteps,
                      int nthreads) {
    const size_t bytes = (size_t)(n > 0 ? n : 1) * sizeof(double);
    double *buf[12];
    for (int k = 0; k < 12; ++k) buf[k] = (double *)malloc(bytes);
    double *px = buf[0], *py = buf[1], *pz = buf[2], *pvx = buf[3], *pvy = buf[4], *pvz = buf[5];
    double *bx = buf[6], *by = buf[7], *bz = buf[8], *kx = buf[9], *ky = buf[10], *kz = buf[11];
    for (int64_t s = 0; s < nsteps; ++s) {
        for (int64_t i = 0; i < n; ++i) {
            px[i] = x[i] + vx[i] * dt + ax[i] * dt * dt / 2.0 + jx[i] * dt * dt * dt / 6.0;
            py[i] = y[i] + vy[i] * dt + ay[i] * dt * dt / 2.0 + jy[i] * dt * dt * dt / 6.0;
            pz[i] = z[i] + vz[i] * dt + az[i] * dt * dt / 2.0 + jz[i] * dt * dt * dt / 6.0;
            pvx[i] = vx[i] + ax[i] * dt + jx[i] * dt * dt / 2.0;
            pvy[i] = vy[i] + ay[i] * dt + jy[i] * dt * dt / 2.0;
            pvz[i] = vz[i] + az[i] * dt + jz[i] * dt * dt / 2.0;
        }
        orc_accel_jerk(n, px, py, pz, pvx, pvy, pvz, m, G, eps, h, NULL, 0, bx, by, bz, kx, ky, kz, NULL,
                       NULL, nthreads);
        ++g_force_evals;
        for (int64_t i = 0; i < n; ++i) {
            const double wx = vx[i] + (ax[i] + bx[i]) * dt / 2.0 + (jx[i] - kx[i]) * dt * dt / 12.0;
            const double wy = vy[i] + (ay[i] + by[i]) * dt / 2.0 + (jy[i] - ky[i]) * dt * dt / 12.0;
            const double wz = vz[i] + (az[i] + bz[i]) * dt / 2.0 + (jz[i] - kz[i]) * dt * dt / 12.0;
            x[i] += (vx[i] + wx) * dt / 2.0 + (ax[i] - bx[i]) * dt * dt / 12.0;
            y[i] += (vy[i] + wy) * dt / 2.0 + (ay[i] - by[i]) * dt * dt / 12.0;
            z[i] += (vz[i] + wz) * dt / 2.0 + (az[i] - bz[i]) * dt * dt / 12.0;
            vx[i] = wx; vy[i] = wy; vz[i] = wz;
            ax[i] = bx[i]; ay[i] = by[i]; az[i] = bz[i];
            jx[i] = kx[i]; jy[i] = ky[i]; jz[i] = kz[i];
        }
    }
    for (int k = 0; k < 12; ++k) free(buf[k]);
}

/* Classical fourth-order Runge-Kutta on the first-order system r' = v,
 * v' = a(r):
 *   k1 = (v, a(r)),
 *   k2 = (v + dt/2 k1v, a(r + dt/2 k1r)),
 *   k3 = (v + dt/2 k2v, a(r + dt/2 k2r)),
 *   k4 = (v + dt k3v, a(r + dt k3r)),
 *   (r, v) += dt/6 (k1 + 2 k2 + 2 k3 + k4).
 * On entry a must hold a(r); on return a(r') is evaluated, so there are four
 * force evaluations per step. */
void orc_step_rk4(int64_t n, double *x, double *y, double *z, double *vx, double *vy, double *vz,
                  const double *m, double *ax, double *ay, double *az, double G, double eps,
                  const orc_halo *h, double dt, int64_t nsteps, int nthreads) {
    const size_t bytes = (size_t)(n > 0 ? n : 1) * sizeof(double);
    double *buf[24];
    for (int k = 0; k < 24; ++k) buf[k] = (double *)malloc(bytes);
    double *sx = buf[0], *sy = buf[1], *sz = buf[2];                         /* stage position */
    double *k1rx = buf[3], *k1ry = buf[4], *k1rz = buf[5];
    double *k2rx = buf[6], *k2ry = buf[7], *k2rz = buf[8];
    double *k3rx = buf[9], *k3ry = buf[10], *k3rz = buf[11];
    double *k4rx = buf[12], *k4ry = buf[13], *k4rz = buf[14];
    double *k2vx = buf[15], *k2vy = buf[16], *k2vz = buf[17];
    double *k3vx = buf[18], *k3vy = buf[19], *k3vz = buf[20];
    double *k4vx = buf[21], *k4vy = buf[22], *k4vz = buf[23];
    for (int64_t s = 0; s < nsteps; ++s) {
        /* k1 = (v, a) */
        for (int64_t i = 0; i < n; ++i) {
            k1rx[i] = vx[i]; k1ry[i] = vy[i]; k1rz[i] = vz[i];
            sx[i] = x[i] + dt / 2.0 * k1rx[i];
            sy[i] = y[i] + dt / 2.0 * k1ry[i];
            sz[i] = z[i] + dt / 2.0 * k1rz[i];
        }
        total_accel(n, sx, sy, sz, m, G, eps, h, 0, k2vx, k2vy, k2vz, nthreads);
        ++g_force_evals;
        for (int64_t i = 0; i < n; ++i) {
            k2rx[i] = vx[i] + dt / 2.0 * ax[i];
            k2ry[i] = vy[i] + dt / 2.0 * ay[i];
            k2rz[i] = vz[i] + dt / 2.0 * az[i];
            sx[i] = x[i] + dt / 2.0 * k2rx[i];
            sy[i] = y[i] + dt / 2.0 * k2ry[i];
            sz[i] = z[i] + dt / 2.0 * k2rz[i];
        }
        total_accel(n, sx, sy, sz, m, G, eps, h, 0, k3vx, k3vy, k3vz, nthreads);
        ++g_force_evals;
        for (int64_t i = 0; i < n; ++i) {
            k3rx[i] = vx[i] + dt / 2.0 * k2vx[i];
            k3ry[i] = vy[i] + dt / 2.0 * k2vy[i];
            k3rz[i] = vz[i] + dt / 2.0 * k2vz[i];
            sx[i] = x[i] + dt * k3rx[i];
            sy[i] = y[i] + dt * k3ry[i];
            sz[i] = z[i] + dt * k3rz[i];
        }
        total_accel(n, sx, sy, sz, m, G, eps, h, 0, k4vx, k4vy, k4vz, nthreads);
        ++g_force_evals;
        for (int64_t i = 0; i < n; ++i) {
            k4rx[i] = vx[i] + dt * k3vx[i];
            k4ry[i] = vy[i] + dt * k3vy[i];
            k4rz[i] = vz[i] + dt * k3vz[i];
            x[i] += dt / 6.0 * (k1rx[i] + 2.0 * k2rx[i] + 2.0 * k3rx[i] + k4rx[i]);
            y[i] += dt / 6.0 * (k1ry[i] + 2.0 * k2ry[i] + 2.0 * k3ry[i] + k4ry[i]);
            z[i] += dt / 6.0 * (k1rz[i] + 2.0 * k2rz[i] + 2.0 * k3rz[i] + k4rz[i]);
            vx[i] += dt / 6.0 * (ax[i] + 2.0 * k2vx[i] + 2.0 * k3vx[i] + k4vx[i]);
            vy[i] += dt / 6.0 * (ay[i] + 2.0 * k2vy[i] + 2.0 * k3vy[i] + k4vy[i]);
            vz[i] += dt / 6.0 * (az[i] + 2.0 * k2vz[i] + 2.0 * k3vz[i] + k4vz[i]);
        }
        total_accel(n, x, y, z, m, G, eps, h, 0, ax, ay, az, nthreads);
        ++g_force_evals;
    }
    for (int k = 0; k < 24; ++k) free(buf[k]);
}

/* ------------------------------------------------------------------------ */
/* Section 3, Eqs. (8)-(10) and the centre of mass.
 * out[0]  K    = sum m |v|^2 / 2
 * out[1]  W    = -(1/2) sum_i sum_{j != i} G m_i m_j / sqrt(|r_i - r_j|^2 + delta^2)
 * out[2]  Wext = sum m_i Phi_h(r_i)            (0 without halo)
 * out[3]  E    = K + W + Wext
 * out[4..6]   P = sum m v
 * out[7..9]   L = sum m r x v   (Eq. (10) is out[9])
 * out[10..12] centre of mass sum m r / M
 * out[13] M    = sum m
 * Per-particle terms are formed in parallel and summed serially in index
 * order. */
void orc_diag(int64_t n, const double *x, const double *y, const double *z, const double *vx,
              const double *vy, const double *vz, const double *m, double G, double eps,
              const orc_halo *h, double *out, int nthreads) {
    set_threads(nthreads);
    double *w = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    const double d2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const double dx = x[i] - x[j];
            const double dy = y[i] - y[j];
            const double dz = z[i] - z[j];
            const double r2 = dx * dx + dy * dy + dz * dz + d2;
            if (r2 == 0.0) continue;
            s += G * m[i] * m[j] / sqrt(r2);
        }
        w[i] = s;
    }
    double K = 0, W = 0, Wext = 0, P[3] = {0, 0, 0}, L[3] = {0, 0, 0}, C[3] = {0, 0, 0}, M = 0;
    for (int64_t i = 0; i < n; ++i) {
        K += m[i] * (vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]) / 2.0;
        W -= w[i] / 2.0;
        if (h && h->on) {
            const double r = sqrt(x[i] * x[i] + y[i] * y[i] + z[i] * z[i]);
            Wext += m[i] * halo_phi(r, h->v2, h->rc);
        }
        P[0] += m[i] * vx[i];
        P[1] += m[i] * vy[i];
        P[2] += m[i] * vz[i];
        L[0] += m[i] * (y[i] * vz[i] - z[i] * vy[i]);
        L[1] += m[i] * (z[i] * vx[i] - x[i] * vz[i]);
        L[2] += m[i] * (x[i] * vy[i] - y[i] * vx[i]);
        C[0] += m[i] * x[i];
        C[1] += m[i] * y[i];
        C[2] += m[i] * z[i];
        M += m[i];
    }
    free(w);
    out[0] = K; out[1] = W; out[2] = Wext; out[3] = K + W + Wext;
    out[4] = P[0]; out[5] = P[1]; out[6] = P[2];
    out[7] = L[0]; out[8] = L[1]; out[9] = L[2];
    out[10] = M > 0 ? C[0] / M : 0.0;
    out[11] = M > 0 ? C[1] / M : 0.0;
    out[12] = M > 0 ? C[2] / M : 0.0;
    out[13] = M;
}

/* Surface-density map on the x-y plane, the quantity whose single- and
 * double-precision versions Section 3 (Fig. 7) compares.  For each particle:
 * ix = floor((x - x0) * sx), iy = floor((y - y0) * sy), each decided in
 * float64 by one subtraction and one multiplication; particles with
 * 0 <= ix < nx and 0 <= iy < ny are counted in counts[iy * nx + ix], others
 * (and NaN coordinates) are not.  Serial, in index order. */
void orc_surface_density(int64_t n, const double *x, const double *y, int32_t nx, int32_t ny, double x0,
                         double y0, double sx, double sy, uint32_t *counts) {
    memset(counts, 0, (size_t)nx * (size_t)ny * sizeof(uint32_t));
    for (int64_t i = 0; i < n; ++i) {
        const double fx = floor((x[i] - x0) * sx);
        const double fy = floor((y[i] - y0) * sy);
        if (!(fx >= 0.0 && fx < (double)nx && fy >= 0.0 && fy < (double)ny)) continue;
        counts[(int64_t)fy * nx + (int64_t)fx] += 1u;
    }
}
