/*
 * Oracle for the trapped-ion Coulomb + linear-Paul-trap + velocity-Verlet path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, FP64 CPU statement of
 * what the GPU path computes.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header or constant
 * with the GPU library and the GPU library never calls it.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math), so every
 * product and sum below is rounded as written.
 *
 * Physics followed (paper: "Dynamics of trapped ions", eq. (field), eq. (Mathieuaq),
 * eq. (fullPotential); "Implementation details": units si, coul/cut, nve):
 *   E_ext(r, t) = (V0/R0^2) cos(Omega t) (x, -y, 0) + (kappa U0/Z0^2) (x, y, -2z)
 *     The dc term is read as axially confining, i.e. minus the gradient of
 *     (kappa U0/Z0^2)(z^2 - (x^2+y^2)/2); this is the only sign consistent with
 *     eq. (Mathieuaq) (a_x = -a_z/2 = -4 Q kappa U0/(M Z0^2 Omega^2)).
 *   E_c,i = k_e sum_{j != i} Q_j (r_i - r_j) / |r_i - r_j|^3   (unscreened, no cutoff;
 *     the paper's 10 m cutoff never acts on a trapped cloud)
 *   a_i = (Q_i / M_i) (E_c,i + E_ext(r_i, t))
 *   Step (velocity Verlet as LAMMPS nve, with laser-cooling damping applied as exact
 *   exp(-gamma dt/2) velocity scalings before and after):
 *     v <- f v;  v <- v + (dt/2) a;  x <- x + dt v;  t_{k+1} = t_start + (k+1) dt;
 *     a <- accel(x, t_{k+1});  v <- v + (dt/2) a;  v <- f v,   f = exp(-gamma dt / 2).
 *
 * Pair sums use Neumaier's compensated summation (Neumaier 1974) in ascending j, so
 * the oracle's own rounding error is far below the GPU tolerances it checks.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* CODATA 2018 / SI 2019 values, written out here independently of the GPU library. */
#define OR_ECHARGE 1.602176634e-19
#define OR_EPS0 8.8541878128e-12
#define OR_PI 3.14159265358979323846
#define OR_KB 1.380649e-23

typedef struct {
    double V0;     /* rf amplitude (V) */
    double Omega;  /* rf angular frequency (rad/s) */
    double U0;     /* end-cap dc voltage (V) */
    double R0;     /* radial length scale (m) */
    double Z0;     /* axial length scale (m) */
    double kappa;  /* geometric factor */
    int32_t pseudo; /* 1: pseudopotential approximation of the rf (eq. (pseudopot)) */
    int32_t pad;
} oracle_trap;

double oracle_coulomb_constant(void) { return 1.0 / (4.0 * OR_PI * OR_EPS0); }

/* Threads the OpenMP loops of this library use. */
int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the thread count of later OpenMP loops (for timing the oracle on one
 * core); n < 1 is ignored. */
void oracle_set_num_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Neumaier running sum: value s, compensation c. */
typedef struct { double s, c; } nsum;

static void nsum_add(nsum *a, double t) {
    double u = a->s + t;
    if (fabs(a->s) >= fabs(t))
        a->c += (a->s - u) + t;
    else
        a->c += (t - u) + a->s;
    a->s = u;
}

static double nsum_get(const nsum *a) { return a->s + a->c; }

/* External field of eq. (field) at one point, dc sign read as confining. */
/* Strength A_rf^2 / (2 Omega^2) of the pseudopotential's radial term (0 for
 * the full rf field).  With eq. (Mathieuaq) in eq. (pseudopot),
 * omega_x^2 = (Omega^2/4)(a_x + q_x^2/2) = (Q/M)^2 A_rf^2/(2 Omega^2) - (Q/M) A_dc and
 * omega_z^2 = 2 (Q/M) A_dc: the dc field stays as it is and the rf becomes the
 * static radial field -(Q/M) A_rf^2/(2 Omega^2) (x, y, 0), whose strength
 * depends on the ion's own Q/M. */
static double pseudo_strength(const oracle_trap *tp) {
    if (!tp->pseudo) return 0.0;
    double a_rf = tp->V0 / (tp->R0 * tp->R0);
    return (a_rf * a_rf) / (2.0 * tp->Omega * tp->Omega);
}

/* External field E_ext on an ion of charge-to-mass ratio qm at (x, y, z). */
static void trap_field(const oracle_trap *tp, double t, double qm, double x, double y, double z,
                       double *ex, double *ey, double *ez) {
    double a_rf = tp->V0 / (tp->R0 * tp->R0);
    double a_dc = tp->kappa * tp->U0 / (tp->Z0 * tp->Z0);
    if (tp->pseudo) {
        double k = qm * pseudo_strength(tp);
        *ex = a_dc * x - k * x;
        *ey = a_dc * y - k * y;
        *ez = -2.0 * a_dc * z;
        return;
    }
    double c = cos(tp->Omega * t);
    *ex = a_rf * c * x + a_dc * x;
    *ey = -a_rf * c * y + a_dc * y;
    *ez = -2.0 * a_dc * z;
}

/* Magnitude of the radial (rf or pseudopotential) field on an ion, for the
 * force scale. */
static double radial_scale(const oracle_trap *tp, double t, double qm, double x, double y) {
    double rho = sqrt(x * x + y * y);
    if (tp->pseudo) return fabs(qm * pseudo_strength(tp)) * rho;
    double a_rf = tp->V0 / (tp->R0 * tp->R0);
    return fabs(a_rf * cos(tp->Omega * t)) * rho;
}

/* Coulomb field E_c,i (V/m) on every ion of one cloud.  Returns the number of
 * exactly coincident pairs met (they contribute zero). */
int64_t oracle_coulomb_field(int64_t n, const double *x, const double *y, const double *z,
                             const double *charge, double *ex, double *ey, double *ez) {
    const double ke = oracle_coulomb_constant();
    int64_t coincident = 0;
#pragma omp parallel for schedule(static) reduction(+ : coincident) if (n >= 256)
    for (int64_t i = 0; i < n; ++i) {
        nsum sx = {0, 0}, sy = {0, 0}, sz = {0, 0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) {
                ++coincident;
                continue;
            }
            double s = charge[j] * (1.0 / (r2 * sqrt(r2)));
            nsum_add(&sx, s * dx);
            nsum_add(&sy, s * dy);
            nsum_add(&sz, s * dz);
        }
        ex[i] = ke * nsum_get(&sx);
        ey[i] = ke * nsum_get(&sy);
        ez[i] = ke * nsum_get(&sz);
    }
    return coincident;
}

/* Acceleration a_i = (Q_i/M_i)(E_c,i + E_ext(r_i, t)) for one cloud in one trap. */
int64_t oracle_accel(int64_t n, const double *x, const double *y, const double *z,
                     const double *charge, const double *mass, const oracle_trap *tp,
                     double t, double *ax, double *ay, double *az) {
    int64_t coincident = oracle_coulomb_field(n, x, y, z, charge, ax, ay, az);
    for (int64_t i = 0; i < n; ++i) {
        double ex, ey, ez;
        double qm = charge[i] / mass[i];
        trap_field(tp, t, qm, x[i], y[i], z[i], &ex, &ey, &ez);
        ax[i] = qm * (ax[i] + ex);
        ay[i] = qm * (ay[i] + ey);
        az[i] = qm * (az[i] + ez);
    }
    return coincident;
}

/* Acceleration of the selected targets idx[0..m) only (same definition as
 * oracle_accel); used to check very large clouds on a sample of ions. */
void oracle_accel_at(int64_t n, const double *x, const double *y, const double *z,
                     const double *charge, const double *mass, const oracle_trap *tp, double t,
                     int64_t m, const int64_t *idx, double *ax, double *ay, double *az,
                     double *scale) {
    const double ke = oracle_coulomb_constant();
    double a_dc = tp->kappa * tp->U0 / (tp->Z0 * tp->Z0);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < m; ++k) {
        int64_t i = idx[k];
        nsum sx = {0, 0}, sy = {0, 0}, sz = {0, 0}, sm = {0, 0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) continue;
            double s = charge[j] * (1.0 / (r2 * sqrt(r2)));
            nsum_add(&sx, s * dx);
            nsum_add(&sy, s * dy);
            nsum_add(&sz, s * dz);
            nsum_add(&sm, fabs(charge[j]) / r2);
        }
        double ex, ey, ez;
        double qm = charge[i] / mass[i];
        trap_field(tp, t, qm, x[i], y[i], z[i], &ex, &ey, &ez);
        ax[k] = qm * (ke * nsum_get(&sx) + ex);
        ay[k] = qm * (ke * nsum_get(&sy) + ey);
        az[k] = qm * (ke * nsum_get(&sz) + ez);
        double erf = radial_scale(tp, t, charge[i] / mass[i], x[i], y[i]);
        double edc = fabs(a_dc) * sqrt(x[i] * x[i] + y[i] * y[i] + 4.0 * z[i] * z[i]);
        scale[k] = fabs(charge[i]) / mass[i] * (ke * nsum_get(&sm) + erf + edc);
    }
}

/* Acceleration with pairs inside rigid bodies left out (section "Charged rigid
 * body": ions of one group are bound together, so their mutual forces are
 * internal to the body).  body[i] >= 0 names the body of ion i, -1 a free ion;
 * pairs with body[i] == body[j] >= 0 are skipped.  Also returns the rounding
 * scale of each a_i over the pairs that remain (as oracle_accel_scale). */
int64_t oracle_accel_bodies(int64_t n, const double *x, const double *y, const double *z,
                            const double *charge, const double *mass, const int32_t *body,
                            const oracle_trap *tp, double t, double *ax, double *ay, double *az,
                            double *scale) {
    const double ke = oracle_coulomb_constant();
    double a_dc = tp->kappa * tp->U0 / (tp->Z0 * tp->Z0);
    int64_t coincident = 0;
#pragma omp parallel for schedule(static) reduction(+ : coincident) if (n >= 256)
    for (int64_t i = 0; i < n; ++i) {
        nsum sx = {0, 0}, sy = {0, 0}, sz = {0, 0}, sm = {0, 0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            if (body[i] >= 0 && body[j] == body[i]) continue;
            double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) {
                ++coincident;
                continue;
            }
            double s = charge[j] * (1.0 / (r2 * sqrt(r2)));
            nsum_add(&sx, s * dx);
            nsum_add(&sy, s * dy);
            nsum_add(&sz, s * dz);
            nsum_add(&sm, fabs(charge[j]) / r2);
        }
        double ex, ey, ez;
        double qm = charge[i] / mass[i];
        trap_field(tp, t, qm, x[i], y[i], z[i], &ex, &ey, &ez);
        ax[i] = qm * (ke * nsum_get(&sx) + ex);
        ay[i] = qm * (ke * nsum_get(&sy) + ey);
        az[i] = qm * (ke * nsum_get(&sz) + ez);
        double erf = radial_scale(tp, t, charge[i] / mass[i], x[i], y[i]);
        double edc = fabs(a_dc) * sqrt(x[i] * x[i] + y[i] * y[i] + 4.0 * z[i] * z[i]);
        scale[i] = fabs(charge[i]) / mass[i] * (ke * nsum_get(&sm) + erf + edc);
    }
    return coincident;
}

/* oracle_accel_bodies for the selected targets idx[0..m) only (every source
 * still counts); used to check very large clouds on a sample of ions. */
void oracle_accel_bodies_at(int64_t n, const double *x, const double *y, const double *z,
                            const double *charge, const double *mass, const int32_t *body,
                            const oracle_trap *tp, double t, int64_t m, const int64_t *idx,
                            double *ax, double *ay, double *az, double *scale) {
    const double ke = oracle_coulomb_constant();
    double a_dc = tp->kappa * tp->U0 / (tp->Z0 * tp->Z0);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < m; ++k) {
        int64_t i = idx[k];
        nsum sx = {0, 0}, sy = {0, 0}, sz = {0, 0}, sm = {0, 0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            if (body[i] >= 0 && body[j] == body[i]) continue;
            double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) continue;
            double s = charge[j] * (1.0 / (r2 * sqrt(r2)));
            nsum_add(&sx, s * dx);
            nsum_add(&sy, s * dy);
            nsum_add(&sz, s * dz);
            nsum_add(&sm, fabs(charge[j]) / r2);
        }
        double ex, ey, ez;
        double qm = charge[i] / mass[i];
        trap_field(tp, t, qm, x[i], y[i], z[i], &ex, &ey, &ez);
        ax[k] = qm * (ke * nsum_get(&sx) + ex);
        ay[k] = qm * (ke * nsum_get(&sy) + ey);
        az[k] = qm * (ke * nsum_get(&sz) + ez);
        double erf = radial_scale(tp, t, charge[i] / mass[i], x[i], y[i]);
        double edc = fabs(a_dc) * sqrt(x[i] * x[i] + y[i] * y[i] + 4.0 * z[i] * z[i]);
        scale[k] = fabs(charge[i]) / mass[i] * (ke * nsum_get(&sm) + erf + edc);
    }
}

/* Rounding scale of a_i: (|Q_i|/M_i)(k_e sum_j |Q_j|/r_ij^2 + |E_rf,i| + |E_dc,i|),
 * the sum of the magnitudes of every contribution to a_i. */
void oracle_accel_scale(int64_t n, const double *x, const double *y, const double *z,
                        const double *charge, const double *mass, const oracle_trap *tp,
                        double t, double *scale) {
    const double ke = oracle_coulomb_constant();
    double a_dc = tp->kappa * tp->U0 / (tp->Z0 * tp->Z0);
#pragma omp parallel for schedule(static) if (n >= 256)
    for (int64_t i = 0; i < n; ++i) {
        nsum s = {0, 0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) continue;
            nsum_add(&s, fabs(charge[j]) / r2);
        }
        double erf = radial_scale(tp, t, charge[i] / mass[i], x[i], y[i]);
        double edc = fabs(a_dc) * sqrt(x[i] * x[i] + y[i] * y[i] + 4.0 * z[i] * z[i]);
        scale[i] = fabs(charge[i]) / mass[i] * (ke * nsum_get(&s) + erf + edc);
    }
}

/* nsteps velocity-Verlet steps with damping, starting at t_start.  On entry
 * (ax, ay, az) must hold accel(x, t_start); on exit they hold accel at the end
 * time t_start + nsteps dt, which is returned through *t_end. */
int64_t oracle_step(int64_t n, double *x, double *y, double *z, double *vx, double *vy,
                    double *vz, double *ax, double *ay, double *az, const double *charge,
                    const double *mass, const oracle_trap *tp, double gamma, double t_start,
                    double dt, int64_t nsteps, double *t_end) {
    const double f = exp(-(gamma * dt) * 0.5);
    const double h = 0.5 * dt;
    int64_t coincident = 0;
    for (int64_t k = 0; k < nsteps; ++k) {
        for (int64_t i = 0; i < n; ++i) {
            vx[i] = f * vx[i];
            vy[i] = f * vy[i];
            vz[i] = f * vz[i];
            vx[i] = vx[i] + h * ax[i];
            vy[i] = vy[i] + h * ay[i];
            vz[i] = vz[i] + h * az[i];
            x[i] = x[i] + dt * vx[i];
            y[i] = y[i] + dt * vy[i];
            z[i] = z[i] + dt * vz[i];
        }
        double t = t_start + (double)(k + 1) * dt;
        coincident += oracle_accel(n, x, y, z, charge, mass, tp, t, ax, ay, az);
        for (int64_t i = 0; i < n; ++i) {
            vx[i] = vx[i] + h * ax[i];
            vy[i] = vy[i] + h * ay[i];
            vz[i] = vz[i] + h * az[i];
            vx[i] = f * vx[i];
            vy[i] = f * vy[i];
            vz[i] = f * vz[i];
        }
    }
    *t_end = t_start + (double)nsteps * dt;
    return coincident;
}

/* Kinetic energy sum 1/2 M v^2, Coulomb energy sum_{i<j} k_e Q_i Q_j / r_ij
 * (eq. (fullPotential), each pair once), and the dc-trap energy
 * sum Q_i (kappa U0/Z0^2)(z^2 - (x^2+y^2)/2).  Joules. */
void oracle_energy(int64_t n, const double *x, const double *y, const double *z,
                   const double *vx, const double *vy, const double *vz, const double *charge,
                   const double *mass, const oracle_trap *tp, double *kinetic, double *coulomb,
                   double *dc_trap) {
    const double ke = oracle_coulomb_constant();
    double a_dc = tp->kappa * tp->U0 / (tp->Z0 * tp->Z0);
    nsum k = {0, 0}, c = {0, 0}, d = {0, 0};
    for (int64_t i = 0; i < n; ++i) {
        nsum_add(&k, 0.5 * mass[i] * (vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]));
        nsum_add(&d, charge[i] * a_dc * (z[i] * z[i] - 0.5 * (x[i] * x[i] + y[i] * y[i])));
        if (tp->pseudo) /* potential of the radial pseudopotential field */
            nsum_add(&d, 0.5 * charge[i] * (charge[i] / mass[i]) * pseudo_strength(tp) *
                             (x[i] * x[i] + y[i] * y[i]));
        for (int64_t j = i + 1; j < n; ++j) {
            double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            if (r == 0.0) continue;
            nsum_add(&c, ke * charge[i] * charge[j] / r);
        }
    }
    *kinetic = nsum_get(&k);
    *coulomb = nsum_get(&c);
    *dc_trap = nsum_get(&d);
}

/* Independent traps concatenated in trap order: trap k owns ions
 * [offset[k], offset[k+1]).  Each trap is one oracle_step call with its own
 * parameters, damping rate and step size; no force crosses traps. */
int64_t oracle_step_batch(int32_t n_traps, const int64_t *offset, double *x, double *y,
                          double *z, double *vx, double *vy, double *vz, double *ax, double *ay,
                          double *az, const double *charge, const double *mass,
                          const oracle_trap *traps, const double *gamma, const double *t_start,
                          const double *dt, int64_t nsteps, double *t_end) {
    int64_t coincident = 0;
    for (int32_t k = 0; k < n_traps; ++k) {
        int64_t o = offset[k], m = offset[k + 1] - offset[k];
        coincident += oracle_step(m, x + o, y + o, z + o, vx + o, vy + o, vz + o, ax + o, ay + o,
                                  az + o, charge + o, mass + o, &traps[k], gamma[k], t_start[k],
                                  dt[k], nsteps, &t_end[k]);
    }
    return coincident;
}

int64_t oracle_accel_batch(int32_t n_traps, const int64_t *offset, const double *x,
                           const double *y, const double *z, const double *charge,
                           const double *mass, const oracle_trap *traps, const double *t,
                           double *ax, double *ay, double *az) {
    int64_t coincident = 0;
    for (int32_t k = 0; k < n_traps; ++k) {
        int64_t o = offset[k], m = offset[k + 1] - offset[k];
        coincident += oracle_accel(m, x + o, y + o, z + o, charge + o, mass + o, &traps[k], t[k],
                                   ax + o, ay + o, az + o);
    }
    return coincident;
}

/* ------------------------------------------------------------------------
 * Cooling beams and Langevin baths (section "Cooling the motion of ions").
 *
 * A beam acts on ions of one species (-1: every species) along unit direction
 * k with rate gamma: viscous force -M gamma (k.v) k, applied in each velocity
 * half-step as the exact decay v <- v - (1 - exp(-gamma dt/2)) (k.v) k.
 * A bath (temperature T, 1/e velocity relaxation time tau) acts on ions of one
 * species in each half-step as the exact Ornstein-Uhlenbeck update
 *   v <- c v + sqrt(k_B T / M (1 - c^2)) xi,   c = exp(-dt / (2 tau)),
 * with xi three standard normal numbers.  The normals come from Philox4x32-10
 * (Salmon, Moraes, Dror, Shaw, SC'11) keyed by the bath's 64-bit seed, with
 * counter (ion, step low word, step high word, bath << 8 | half-step), and the
 * Box-Muller transform of its four outputs (uniforms (r + 1/2) 2^-32).
 * Order inside one half-step: isotropic damping, beams in index order, baths in
 * index order.  Steps are numbered from 1 over the whole run: step_base is the
 * number of steps done before this call.
 * ---------------------------------------------------------------------- */

typedef struct {
    double kx, ky, kz, gamma;
    int32_t species, pad;
} oracle_beam;

typedef struct {
    double temperature, tau;
    uint64_t seed;
    int32_t species, pad;
} oracle_bath;

static uint32_t mulhilo32(uint32_t a, uint32_t b, uint32_t *hi) {
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    return (uint32_t)p;
}

void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        uint32_t hi0, hi1;
        uint32_t lo0 = mulhilo32(0xD2511F53u, c0, &hi0);
        uint32_t lo1 = mulhilo32(0xCD9E8D57u, c2, &hi1);
        uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* Three standard normals for (seed, ion, step, bath, half-step). */
void oracle_normals3(uint64_t seed, int64_t ion, int64_t step, int32_t bath, int32_t half,
                     double z[3]) {
    uint32_t ctr[4] = {(uint32_t)ion, (uint32_t)((uint64_t)step & 0xffffffffu),
                       (uint32_t)((uint64_t)step >> 32), ((uint32_t)bath << 8) | (uint32_t)half};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t r[4];
    oracle_philox4x32_10(ctr, key, r);
    const double two32 = 1.0 / 4294967296.0;
    double u1 = ((double)r[0] + 0.5) * two32, u2 = ((double)r[1] + 0.5) * two32;
    double u3 = ((double)r[2] + 0.5) * two32, u4 = ((double)r[3] + 0.5) * two32;
    double rad1 = sqrt(-2.0 * log(u1)), rad2 = sqrt(-2.0 * log(u3));
    z[0] = rad1 * cos(2.0 * OR_PI * u2);
    z[1] = rad1 * sin(2.0 * OR_PI * u2);
    z[2] = rad2 * cos(2.0 * OR_PI * u4);
}

static void velocity_half(int64_t i, double *vx, double *vy, double *vz, double f, double h,
                          double mass, int32_t species, int nbeams, const oracle_beam *beams,
                          int nbaths, const oracle_bath *baths, int64_t step, int half) {
    double u = f * *vx, v = f * *vy, w = f * *vz;
    for (int b = 0; b < nbeams; ++b) {
        const oracle_beam *B = &beams[b];
        if (B->gamma <= 0.0 || (B->species >= 0 && B->species != species)) continue;
        double fb = exp(-(B->gamma * h));
        double d = (1.0 - fb) * (B->kx * u + B->ky * v + B->kz * w);
        u = u - d * B->kx;
        v = v - d * B->ky;
        w = w - d * B->kz;
    }
    for (int c = 0; c < nbaths; ++c) {
        const oracle_bath *T = &baths[c];
        if (T->tau <= 0.0 || (T->species >= 0 && T->species != species)) continue;
        double c1 = exp(-(h / T->tau));
        double sig = sqrt(OR_KB * T->temperature / mass * (1.0 - c1 * c1));
        double z[3];
        oracle_normals3(T->seed, i, step, c, half, z);
        u = c1 * u + sig * z[0];
        v = c1 * v + sig * z[1];
        w = c1 * w + sig * z[2];
    }
    *vx = u;
    *vy = v;
    *vz = w;
}

/* oracle_step with cooling beams and Langevin baths.  The beam directions are
 * used as given (the caller normalises them).  Ion i of this trap draws its bath
 * normals as ion ion_base + i of the run (a trap inside a batch passes the
 * index of its first ion).  With nbeams = nbaths = 0 this is oracle_step
 * exactly. */
int64_t oracle_step_cooled(int64_t n, double *x, double *y, double *z, double *vx, double *vy,
                           double *vz, double *ax, double *ay, double *az, const double *charge,
                           const double *mass, const int32_t *species, const oracle_trap *tp,
                           double gamma, int nbeams, const oracle_beam *beams, int nbaths,
                           const oracle_bath *baths, int64_t ion_base, int64_t step_base,
                           double t_start, double dt, int64_t nsteps, double *t_end) {
    const double f = exp(-(gamma * dt) * 0.5);
    const double h = 0.5 * dt;
    int64_t coincident = 0;
    for (int64_t k = 0; k < nsteps; ++k) {
        const int64_t s = step_base + k + 1;
        for (int64_t i = 0; i < n; ++i) {
            velocity_half(ion_base + i, &vx[i], &vy[i], &vz[i], f, h, mass[i], species[i],
                          nbeams, beams, nbaths, baths, s, 0);
            vx[i] = vx[i] + h * ax[i];
            vy[i] = vy[i] + h * ay[i];
            vz[i] = vz[i] + h * az[i];
            x[i] = x[i] + dt * vx[i];
            y[i] = y[i] + dt * vy[i];
            z[i] = z[i] + dt * vz[i];
        }
        double t = t_start + (double)(k + 1) * dt;
        coincident += oracle_accel(n, x, y, z, charge, mass, tp, t, ax, ay, az);
        for (int64_t i = 0; i < n; ++i) {
            vx[i] = vx[i] + h * ax[i];
            vy[i] = vy[i] + h * ay[i];
            vz[i] = vz[i] + h * az[i];
            velocity_half(ion_base + i, &vx[i], &vy[i], &vz[i], f, h, mass[i], species[i],
                          nbeams, beams, nbaths, baths, s, 1);
        }
    }
    *t_end = t_start + (double)nsteps * dt;
    return coincident;
}

/* Time average of a per-ion quantity (section "Writing/reading data": timeAvg
 * averages a variable over a duration, e.g. one rf period).  samples holds
 * nsamples rows of n values; row k was taken at the end of run-wide step
 * first_step + k.  Averaging windows of W steps close at steps origin + m W
 * (m = 1, 2, ...); window m covers the W steps origin + (m-1) W + 1 .. origin + m W.
 * Every window whose steps all lie among the samples is written, in order: its
 * mean (plain sum in step order, divided by W) to a row of `means` and its
 * closing step to end_steps.  Returns the number of windows written (at most
 * max_windows). */
int64_t oracle_time_average(int64_t n, int64_t nsamples, const double *samples,
                            int64_t first_step, int64_t origin, int64_t W, int64_t max_windows,
                            double *means, int64_t *end_steps) {
    int64_t count = 0;
    if (W < 1) return 0;
    const int64_t last_step = first_step + nsamples - 1;
    for (int64_t m = 1; count < max_windows; ++m) {
        const int64_t end = origin + m * W;
        const int64_t start = end - W + 1;
        if (end > last_step) break;
        if (start < first_step) continue;
        for (int64_t i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int64_t s = start; s < start + W; ++s) acc = acc + samples[(s - first_step) * n + i];
            means[count * n + i] = acc / (double)W;
        }
        end_steps[count] = end;
        ++count;
    }
    return count;
}

/* ------------------------------------------------------------ rigid bodies
 *
 * Rigid clusters of ions (sections "Charged rigid body" and "Integration": the
 * ions of a rigid group keep their relative positions and the group moves and
 * rotates under the sum of the forces on its ions).  Each body b carries its
 * mass M, centre of mass R, COM velocity V, angular momentum L about R (space
 * frame), orientation quaternion q = (w, x, y, z) that turns body-frame vectors
 * into space-frame ones, and inverse principal moments 1/I_k (0 for a moment
 * that vanishes, e.g. along a rod).  Member i sits at R + A(q) d_i with d_i
 * fixed in the body frame, and moves with V + omega x A(q) d_i where
 * omega = A diag(1/I) A^T L.
 *
 * One step is the velocity-Verlet scheme for rigid bodies, with the damping
 * half-steps of the free ions applied to V and L (scaling every member
 * velocity by f scales both):
 *   V <- f V, L <- f L;  V <- V + (dt/2) F/M,  L <- L + (dt/2) tau;  R <- R + dt V;
 *   q advanced over dt with L held fixed (below);  members placed;
 *   forces at t_{k+1} (pairs inside one body left out);
 *   F = sum m_i a_i,  tau = sum A(q) d_i x m_i a_i;
 *   V <- V + (dt/2) F/M,  L <- L + (dt/2) tau;  V <- f V, L <- f L.
 * The orientation follows dq/dt = (1/2) (0, omega(q)) q (Hamilton product).  It
 * is advanced by Richardson extrapolation of normalised Euler steps: one step
 * of dt and two of dt/2 (omega re-evaluated at the midpoint), combined as
 * 2 q_half - q_full and normalised.  This uses only the space-frame inertia
 * tensor, so the result does not depend on how principal axes are chosen
 * inside a degenerate eigenspace. */

static void quat_matrix(const double q[4], double A[9]) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    A[0] = 1.0 - 2.0 * (y * y + z * z);
    A[1] = 2.0 * (x * y - w * z);
    A[2] = 2.0 * (x * z + w * y);
    A[3] = 2.0 * (x * y + w * z);
    A[4] = 1.0 - 2.0 * (x * x + z * z);
    A[5] = 2.0 * (y * z - w * x);
    A[6] = 2.0 * (x * z - w * y);
    A[7] = 2.0 * (y * z + w * x);
    A[8] = 1.0 - 2.0 * (x * x + y * y);
}

/* omega = A diag(inv_i) A^T L */
static void body_omega(const double q[4], const double inv_i[3], const double L[3],
                       double w[3]) {
    double A[9], p[3];
    quat_matrix(q, A);
    for (int k = 0; k < 3; ++k) p[k] = (A[k] * L[0] + A[3 + k] * L[1] + A[6 + k] * L[2]) * inv_i[k];
    for (int r = 0; r < 3; ++r) w[r] = A[3 * r] * p[0] + A[3 * r + 1] * p[1] + A[3 * r + 2] * p[2];
}

/* q + s (0, w) q, normalised */
static void quat_euler(const double q[4], const double w[3], double s, double out[4]) {
    const double dw = -(w[0] * q[1] + w[1] * q[2] + w[2] * q[3]);
    const double dx = w[0] * q[0] + (w[1] * q[3] - w[2] * q[2]);
    const double dy = w[1] * q[0] + (w[2] * q[1] - w[0] * q[3]);
    const double dz = w[2] * q[0] + (w[0] * q[2] - w[1] * q[1]);
    double r[4] = {q[0] + s * dw, q[1] + s * dx, q[2] + s * dy, q[3] + s * dz};
    double nrm = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3]);
    for (int k = 0; k < 4; ++k) out[k] = r[k] / nrm;
}

static void rotate_richardson(double q[4], const double L[3], const double inv_i[3], double dt) {
    double w0[3], w1[3], qf[4], qh[4], qh2[4];
    body_omega(q, inv_i, L, w0);
    quat_euler(q, w0, 0.5 * dt, qf);
    quat_euler(q, w0, 0.25 * dt, qh);
    body_omega(qh, inv_i, L, w1);
    quat_euler(qh, w1, 0.25 * dt, qh2);
    double r[4];
    for (int k = 0; k < 4; ++k) r[k] = 2.0 * qh2[k] - qf[k];
    double nrm = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3]);
    for (int k = 0; k < 4; ++k) q[k] = r[k] / nrm;
}

/* Space-frame offset A(q) d of member i. */
static void member_offset(const double *q, const double *dbody, int64_t i, double o[3]) {
    double A[9];
    quat_matrix(q, A);
    const double *d = dbody + 3 * i;
    for (int r = 0; r < 3; ++r) o[r] = A[3 * r] * d[0] + A[3 * r + 1] * d[1] + A[3 * r + 2] * d[2];
}

/* F_b = sum m_i a_i, tau_b = sum A d_i x m_i a_i over the members, ascending i. */
static void body_wrench(int64_t n, const double *ax, const double *ay, const double *az,
                        const double *mass, const int32_t *rb, const double *dbody,
                        int32_t nb, const double *q, double *F, double *T) {
    for (int32_t b = 0; b < nb; ++b)
        for (int k = 0; k < 3; ++k) F[3 * b + k] = T[3 * b + k] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const int32_t b = rb[i];
        if (b < 0) continue;
        double o[3];
        member_offset(q + 4 * b, dbody, i, o);
        const double fx = mass[i] * ax[i], fy = mass[i] * ay[i], fz = mass[i] * az[i];
        F[3 * b] += fx;
        F[3 * b + 1] += fy;
        F[3 * b + 2] += fz;
        T[3 * b] += o[1] * fz - o[2] * fy;
        T[3 * b + 1] += o[2] * fx - o[0] * fz;
        T[3 * b + 2] += o[0] * fy - o[1] * fx;
    }
}

static void place_members(int64_t n, double *x, double *y, double *z, double *vx, double *vy,
                          double *vz, const int32_t *rb, const double *dbody, const double *R,
                          const double *V, const double *L, const double *q,
                          const double *inv_i) {
    for (int64_t i = 0; i < n; ++i) {
        const int32_t b = rb[i];
        if (b < 0) continue;
        double o[3], w[3];
        member_offset(q + 4 * b, dbody, i, o);
        body_omega(q + 4 * b, inv_i + 3 * b, L + 3 * b, w);
        x[i] = R[3 * b] + o[0];
        y[i] = R[3 * b + 1] + o[1];
        z[i] = R[3 * b + 2] + o[2];
        vx[i] = V[3 * b] + (w[1] * o[2] - w[2] * o[1]);
        vy[i] = V[3 * b + 1] + (w[2] * o[0] - w[0] * o[2]);
        vz[i] = V[3 * b + 2] + (w[0] * o[1] - w[1] * o[0]);
    }
}

/* nsteps steps with rigid bodies.  rb[i] is the body index (0..nb-1) of ion i,
 * or -1 for a free ion; body[i] the exclusion id passed to the force (pairs of
 * ions with equal body[i] >= 0 are left out).  ax..az hold the accelerations
 * at the starting state and t_start; member positions and velocities are
 * written from the body state after every step.  Returns the number of
 * coincident pairs met. */
int64_t oracle_step_rigid(int64_t n, double *x, double *y, double *z, double *vx, double *vy,
                          double *vz, double *ax, double *ay, double *az, const double *charge,
                          const double *mass, const int32_t *body, const int32_t *rb,
                          const double *dbody, int32_t nb, const double *Mb, const double *inv_i,
                          double *q, double *R, double *V, double *L, const oracle_trap *tp,
                          double gamma, double t_start, double dt, int64_t nsteps,
                          double *t_end) {
    const double f = exp(-(gamma * dt) * 0.5);
    const double h = 0.5 * dt;
    int64_t coincident = 0;
    double *F = (double *)malloc(sizeof(double) * 3 * (size_t)(nb > 0 ? nb : 1));
    double *T = (double *)malloc(sizeof(double) * 3 * (size_t)(nb > 0 ? nb : 1));
    double *sc = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    body_wrench(n, ax, ay, az, mass, rb, dbody, nb, q, F, T);
    for (int64_t k = 0; k < nsteps; ++k) {
        for (int64_t i = 0; i < n; ++i) {
            if (rb[i] >= 0) continue;
            vx[i] = f * vx[i];
            vy[i] = f * vy[i];
            vz[i] = f * vz[i];
            vx[i] = vx[i] + h * ax[i];
            vy[i] = vy[i] + h * ay[i];
            vz[i] = vz[i] + h * az[i];
            x[i] = x[i] + dt * vx[i];
            y[i] = y[i] + dt * vy[i];
            z[i] = z[i] + dt * vz[i];
        }
        for (int32_t b = 0; b < nb; ++b) {
            for (int c = 0; c < 3; ++c) {
                V[3 * b + c] = f * V[3 * b + c];
                L[3 * b + c] = f * L[3 * b + c];
                V[3 * b + c] = V[3 * b + c] + h * (F[3 * b + c] / Mb[b]);
                L[3 * b + c] = L[3 * b + c] + h * T[3 * b + c];
                R[3 * b + c] = R[3 * b + c] + dt * V[3 * b + c];
            }
            rotate_richardson(q + 4 * b, L + 3 * b, inv_i + 3 * b, dt);
        }
        place_members(n, x, y, z, vx, vy, vz, rb, dbody, R, V, L, q, inv_i);
        double t = t_start + (double)(k + 1) * dt;
        coincident += oracle_accel_bodies(n, x, y, z, charge, mass, body, tp, t, ax, ay, az, sc);
        for (int64_t i = 0; i < n; ++i) {
            if (rb[i] >= 0) continue;
            vx[i] = vx[i] + h * ax[i];
            vy[i] = vy[i] + h * ay[i];
            vz[i] = vz[i] + h * az[i];
            vx[i] = f * vx[i];
            vy[i] = f * vy[i];
            vz[i] = f * vz[i];
        }
        body_wrench(n, ax, ay, az, mass, rb, dbody, nb, q, F, T);
        for (int32_t b = 0; b < nb; ++b) {
            for (int c = 0; c < 3; ++c) {
                V[3 * b + c] = V[3 * b + c] + h * (F[3 * b + c] / Mb[b]);
                L[3 * b + c] = L[3 * b + c] + h * T[3 * b + c];
                V[3 * b + c] = f * V[3 * b + c];
                L[3 * b + c] = f * L[3 * b + c];
            }
        }
        place_members(n, x, y, z, vx, vy, vz, rb, dbody, R, V, L, q, inv_i);
    }
    free(F);
    free(T);
    free(sc);
    *t_end = t_start + (double)nsteps * dt;
    return coincident;
}

/* ------------------------------------------------------------ minimisation
 *
 * Energy minimisation (section "Minimisation": damped dynamics that extract
 * energy and cap how far each ion moves in one step; meaningful only in a
 * time-independent trap, i.e. the pseudopotential trap or no rf).  Each
 * iteration, with F_i = M_i a_i at the current positions (trap field at the
 * fixed time t):
 *   stop if max_i |F_i| <= ftol;
 *   P = sum_i v_i . F_i;  v <- (P / sum_i F_i . F_i) F  if P > 0, else v <- 0
 *     (the 3N-velocity keeps only its component along the 3N-force);
 *   v <- v + dt a;
 *   for every ion with dt |v_i| > dmax: v_i <- v_i dmax / (dt |v_i|);
 *   x <- x + dt v;  forces at the new positions.
 * Velocities start from the values passed in.  Returns the number of
 * iterations that moved the ions; *fmax gets max_i |F_i| at the final
 * positions and (ax, ay, az) the final accelerations. */
int64_t oracle_minimize(int64_t n, double *x, double *y, double *z, double *vx, double *vy,
                        double *vz, double *ax, double *ay, double *az, const double *charge,
                        const double *mass, const oracle_trap *tp, double t, double dt,
                        double dmax, double ftol, int64_t max_iter, double *fmax) {
    int64_t it = 0;
    oracle_accel(n, x, y, z, charge, mass, tp, t, ax, ay, az);
    for (;;) {
        double P = 0.0, FF = 0.0, fm = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            const double fx = mass[i] * ax[i], fy = mass[i] * ay[i], fz = mass[i] * az[i];
            P += vx[i] * fx + vy[i] * fy + vz[i] * fz;
            const double f2 = fx * fx + fy * fy + fz * fz;
            FF += f2;
            if (sqrt(f2) > fm) fm = sqrt(f2);
        }
        *fmax = fm;
        if (fm <= ftol || it >= max_iter) break;
        const double coef = (P > 0.0 && FF > 0.0) ? P / FF : 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double u = coef * (mass[i] * ax[i]), v = coef * (mass[i] * ay[i]),
                   w = coef * (mass[i] * az[i]);
            u = u + dt * ax[i];
            v = v + dt * ay[i];
            w = w + dt * az[i];
            const double s = dt * sqrt(u * u + v * v + w * w);
            if (s > dmax) {
                const double r = dmax / s;
                u = u * r;
                v = v * r;
                w = w * r;
            }
            vx[i] = u;
            vy[i] = v;
            vz[i] = w;
            x[i] = x[i] + dt * u;
            y[i] = y[i] + dt * v;
            z[i] = z[i] + dt * w;
        }
        ++it;
        oracle_accel(n, x, y, z, charge, mass, tp, t, ax, ay, az);
    }
    return it;
}

/* ------------------------------------------------------------ normal modes
 *
 * Mass-weighted Hessian of the static potential (section "Normal modes of
 * motion": mode frequencies are eigenvalues of the Hessian of
 * eq. (fullPotential); the trap part is the pseudopotential's, or the dc alone
 * when there is no rf).  D[3i+a][3j+b] = d^2 V / dx_ia dx_jb / sqrt(M_i M_j):
 *   i != j: k_e Q_i Q_j (delta_ab / r^3 - 3 r_a r_b / r^5),  r = x_i - x_j;
 *   i == j: minus the sum of those blocks over j, plus the trap curvature
 *           Q_i (Q_i/M_i) A_rf^2/(2 Omega^2) - Q_i A_dc on x and y (the first
 *           term only for the pseudopotential trap) and 2 Q_i A_dc on z.
 * D is written row-major, (3n)^2 doubles.  The eigenvalues of D are the
 * squared angular frequencies of the normal modes. */
void oracle_hessian(int64_t n, const double *x, const double *y, const double *z,
                    const double *charge, const double *mass, const oracle_trap *tp, double *D) {
    const double ke = oracle_coulomb_constant();
    const double a_dc = tp->kappa * tp->U0 / (tp->Z0 * tp->Z0);
    const double ps = pseudo_strength(tp);
    const int64_t m = 3 * n;
    for (int64_t k = 0; k < m * m; ++k) D[k] = 0.0;
#pragma omp parallel for schedule(static) if (n >= 64)
    for (int64_t i = 0; i < n; ++i) {
        double diag[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const double r[3] = {x[i] - x[j], y[i] - y[j], z[i] - z[j]};
            const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            if (r2 == 0.0) continue;
            const double inv_r = 1.0 / sqrt(r2);
            const double inv_r3 = inv_r * inv_r * inv_r, inv_r5 = inv_r3 * inv_r * inv_r;
            const double c = ke * charge[i] * charge[j];
            const double w = 1.0 / sqrt(mass[i] * mass[j]);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    const double h = c * ((a == b ? inv_r3 : 0.0) - 3.0 * r[a] * r[b] * inv_r5);
                    D[(3 * i + a) * m + 3 * j + b] = h * w;
                    diag[a][b] -= h;
                }
        }
        const double qm = charge[i] / mass[i];
        diag[0][0] += charge[i] * qm * ps - charge[i] * a_dc;
        diag[1][1] += charge[i] * qm * ps - charge[i] * a_dc;
        diag[2][2] += 2.0 * charge[i] * a_dc;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) D[(3 * i + a) * m + 3 * i + b] = diag[a][b] / mass[i];
    }
}
