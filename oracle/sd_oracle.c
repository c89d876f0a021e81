/*
 * sd_oracle.c -- plain FP64 CPU oracle for the all-pairs mobility product of
 * leading-order Stokesian dynamics (Kopp & Hoefling, "GPU-accelerated
 * simulation of colloidal suspensions with direct hydrodynamic interactions",
 * Eur. Phys. J. Special Topics 2012).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never does.  It shares no code, header or constant with the
 * HIP library.
 *
 * Everything is double precision.  Loops are the plain definitions: no
 * blocking, no symmetry exploitation, no reordering.  The outer loop over
 * particles may run on several threads (OpenMP); each output element is still
 * produced by one thread in a fixed order, so results are deterministic.
 *
 * Readings where the paper is silent (documented next to the code that uses
 * them):
 *   - overlap form of the pair tensor for r < 2a (not in the paper; the
 *     Rotne-Prager-Yamakawa regularisation), continuous at r = 2a;
 *   - coincident distinct particles (r = 0): mu0*I with the overlap form,
 *     zero contribution otherwise;
 *   - AB2 integrator (the paper only suggests higher-order schemes), first
 *     step explicit Euler;
 *   - the velocity at step n is computed from the positions at step n before
 *     the positions move (standard explicit Euler);
 *   - lubrication (Eq. 8): the surface separation s = r/a - 2 is clamped below
 *     at s_min (the paper does not say what happens at contact or overlap),
 *     and the previous step's velocities are supplied by the caller (zero or
 *     any other initial guess before the first step);
 *   - periodic box (footnote of Sec. 3.1): only the nearest image interacts;
 *     a difference of exactly half a box rounds half to even (nearbyint).
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double a;      /* sphere radius */
    double eta;    /* shear viscosity */
    int tensor;    /* 0 = Rotne-Prager (Eq. 7b), 1 = Oseen (Eq. 4) */
    int overlap;   /* 0 = far form at every r > 0, 1 = overlap form for r < 2a */
    double box[3]; /* periodic box sides; 0 = free space along that axis */
} oracle_params;

enum { OR_RPY = 0, OR_OSEEN = 1 };

/* Number of threads the parallel loops below run on (1 without OpenMP). */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the number of threads of the parallel loops (no effect without OpenMP). */
void oracle_set_threads(int k)
{
#ifdef _OPENMP
    if (k > 0) omp_set_num_threads(k);
#else
    (void)k;
#endif
}

/* Nearest image (footnote of Sec. 3.1): in a periodic box only the nearest
 * image of each particle interacts.  r = r_i - r_j is replaced by the
 * periodic copy of least length along every periodic axis (ties at exactly
 * half a box side round to even, a measure-zero reading). */
static void nearest_image(const oracle_params* p, double r[3])
{
    for (int k = 0; k < 3; ++k)
        if (p->box[k] > 0.0) r[k] -= p->box[k] * nearbyint(r[k] / p->box[k]);
}

/* Stokes mobility of a single sphere, mu0 = 1/(6 pi eta a): Eq. (7a), Sec. 2.2. */
static double stokes_mobility(const oracle_params* p)
{
    return 1.0 / (6.0 * M_PI * p->eta * p->a);
}

/*
 * 3x3 pair block T(r) of the mobility matrix for r = r_i - r_j, i != j,
 * row-major into T[9].
 *
 *  Oseen, Eq. (4), Sec. 2.2:   G(r) = (I + rhat rhat) / (8 pi eta r)
 *  Rotne-Prager, Eq. (7b):     T(r) = mu0 (3a/4r)(I + rhat rhat)
 *                                   + mu0 (a^3/2r^3)(I - 3 rhat rhat)
 *  Overlap (r < 2a, reading; not in the paper):
 *                              T(r) = mu0 [(1 - 9r/32a) I + (3r/32a) rhat rhat]
 *  Coincident distinct particles (r = 0, reading): mu0 I with the overlap form,
 *  zero otherwise (the far forms are singular there).
 */
void oracle_pair_tensor(const oracle_params* p, const double r[3], double T[9])
{
    const double mu0 = stokes_mobility(p);
    const double a = p->a;
    const double rr = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    double cI, cP;  /* T = cI * I + cP * rhat rhat */

    if (rr == 0.0) {
        for (int k = 0; k < 9; ++k) T[k] = 0.0;
        if (p->overlap && p->tensor == OR_RPY) T[0] = T[4] = T[8] = mu0;
        return;
    }
    if (p->tensor == OR_OSEEN) {
        const double g = 1.0 / (8.0 * M_PI * p->eta * rr);
        cI = g;
        cP = g;
    } else if (p->overlap && rr < 2.0 * a) {
        cI = mu0 * (1.0 - 9.0 * rr / (32.0 * a));
        cP = mu0 * (3.0 * rr / (32.0 * a));
    } else {
        const double t1 = mu0 * 3.0 * a / (4.0 * rr);            /* (I + rr) part */
        const double t3 = mu0 * a * a * a / (2.0 * rr * rr * rr); /* (I - 3rr) part */
        cI = t1 + t3;
        cP = t1 - 3.0 * t3;
    }
    double h[3] = { r[0] / rr, r[1] / rr, r[2] / rr };
    for (int al = 0; al < 3; ++al)
        for (int be = 0; be < 3; ++be)
            T[3 * al + be] = (al == be ? cI : 0.0) + cP * h[al] * h[be];
}

/* velocity of one particle i: v_i = mu0 F_i + sum_{j != i} T(r_i - r_j) F_j, Eq. (7a) */
static void velocity_of(const oracle_params* p, int64_t n, const double* x, const double* f,
                        int64_t i, double out[3])
{
    const double mu0 = stokes_mobility(p);
    double v[3] = { mu0 * f[3 * i + 0], mu0 * f[3 * i + 1], mu0 * f[3 * i + 2] };
    for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        double r[3] = { x[3 * i + 0] - x[3 * j + 0], x[3 * i + 1] - x[3 * j + 1],
                        x[3 * i + 2] - x[3 * j + 2] };
        nearest_image(p, r);
        double T[9];
        oracle_pair_tensor(p, r, T);
        for (int al = 0; al < 3; ++al)
            v[al] += T[3 * al + 0] * f[3 * j + 0] + T[3 * al + 1] * f[3 * j + 1]
                   + T[3 * al + 2] * f[3 * j + 2];
    }
    out[0] = v[0]; out[1] = v[1]; out[2] = v[2];
}

/* Pairs that break the premise of the far-field tensor: the Rotne-Prager
 * tensor of Eq. (4) keeps the mobility matrix positive definite only while
 * every pair distance is r >= 2a (Sec. 2.2).  Counts the unordered pairs
 * i < j with 0 < r < 2a (out[0]) and with r = 0 (out[1]), r the nearest-image
 * distance; r < 2a is tested as r^2 < 4 a^2. */
void oracle_premise_counts(const oracle_params* p, int64_t n, const double* x, int64_t out[2])
{
    int64_t sub = 0, co = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j) {
            double r[3] = { x[3 * i + 0] - x[3 * j + 0], x[3 * i + 1] - x[3 * j + 1],
                            x[3 * i + 2] - x[3 * j + 2] };
            nearest_image(p, r);
            const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            if (r2 == 0.0)
                ++co;
            else if (r2 < 4.0 * p->a * p->a)
                ++sub;
        }
    out[0] = sub;
    out[1] = co;
}

/* All-pairs mobility product, Eq. (7a), step 3 of the algorithm of Sec. 3.1.
 * x, f, v: n x 3 row-major (AoS). */
void oracle_mobility(const oracle_params* p, int64_t n, const double* x, const double* f, double* v)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) velocity_of(p, n, x, f, i, v + 3 * i);
}

/* The same product for a subset of rows (used for sampled checks at large n). */
void oracle_mobility_rows(const oracle_params* p, int64_t n, const double* x, const double* f,
                          int64_t nrows, const int64_t* rows, double* v_rows)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < nrows; ++q) velocity_of(p, n, x, f, rows[q], v_rows + 3 * q);
}

/* Dense 3n x 3n mobility matrix with blocks mu_ij (Eq. 7a): mu_ii = mu0 I,
 * mu_ij = T(r_i - r_j).  Row-major, M[(3i+al)*(3n) + 3j+be].  Tiny n only. */
void oracle_dense_mobility(const oracle_params* p, int64_t n, const double* x, double* M)
{
    const double mu0 = stokes_mobility(p);
    const int64_t ld = 3 * n;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double T[9];
            if (i == j) {
                for (int k = 0; k < 9; ++k) T[k] = 0.0;
                T[0] = T[4] = T[8] = mu0;
            } else {
                double r[3] = { x[3 * i] - x[3 * j], x[3 * i + 1] - x[3 * j + 1],
                                x[3 * i + 2] - x[3 * j + 2] };
                nearest_image(p, r);
                oracle_pair_tensor(p, r, T);
            }
            for (int al = 0; al < 3; ++al)
                for (int be = 0; be < 3; ++be) M[(3 * i + al) * ld + 3 * j + be] = T[3 * al + be];
        }
}

/*
 * Time integration of dx/dt = M(x) F with constant forces (Sec. 3.1, step 1
 * "update particle positions" with the velocities of step 3).
 *   integrator 0: explicit Euler,  x_{k+1} = x_k + dt v_k            (Sec. 3.1)
 *   integrator 1: Adams-Bashforth 2, x_{k+1} = x_k + dt (3/2 v_k - 1/2 v_{k-1})
 *                 (reading: not in the paper; the step with global index 0 is
 *                 an Euler step)
 * v_k = M(x_k) F.  step0 is the global index of the first step taken, so a run
 * can be resumed; v_prev holds v_{k-1} on entry (ignored when step0 == 0) and
 * v_{last} on exit.  If traj != NULL, x is copied to traj every `stride` steps,
 * starting with the initial state: traj holds floor(steps/stride)+1 frames.
 */
int oracle_run(const oracle_params* p, int64_t n, double* x, const double* f, double dt,
               int64_t steps, int64_t step0, int integrator, double* v_prev, double* traj,
               int64_t stride)
{
    double* v = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    if (!v) return 1;
    int64_t frame = 0;
    if (traj) memcpy(traj + 3 * n * frame++, x, sizeof(double) * 3 * (size_t)n);
    for (int64_t s = 0; s < steps; ++s) {
        oracle_mobility(p, n, x, f, v);
        const int euler = (integrator == 0) || (step0 + s == 0);
        for (int64_t k = 0; k < 3 * n; ++k) {
            if (euler) x[k] = x[k] + dt * v[k];
            else x[k] = x[k] + dt * (1.5 * v[k] - 0.5 * v_prev[k]);
        }
        if (v_prev) memcpy(v_prev, v, sizeof(double) * 3 * (size_t)n);
        if (traj && stride > 0 && (s + 1) % stride == 0)
            memcpy(traj + 3 * n * frame++, x, sizeof(double) * 3 * (size_t)n);
    }
    free(v);
    return 0;
}

/*
 * Gradient with respect to r of the bilinear form u . T(r) w, for r != 0.
 * With T = cI(r) I + cP(r) rhat rhat written as  A(r) I + Bt(r) r r  (Bt = cP/r^2):
 *   grad_r [u.T.w] = A'(r) (u.w) rhat + Bt'(r) (u.r)(w.r) rhat + Bt(r) [(w.r) u + (u.r) w]
 * Derivatives of the three forms of oracle_pair_tensor:
 *   Rotne-Prager far:  A = mu0(3a/4r + a^3/2r^3),  Bt = mu0(3a/4r^3 - 3a^3/2r^5)
 *   Oseen:             A = 1/(8 pi eta r),         Bt = 1/(8 pi eta r^3)
 *   overlap (r < 2a):  A = mu0(1 - 9r/32a),        Bt = mu0 3/(32 a r)
 * At r = 0 the gradient is defined as zero (measure-zero set).  At r = 2a the
 * far form is used (one-sided derivative), matching oracle_pair_tensor.
 */
void oracle_pair_grad(const oracle_params* p, const double r[3], const double u[3],
                      const double w[3], double g[3])
{
    const double mu0 = stokes_mobility(p);
    const double a = p->a;
    const double rr = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    g[0] = g[1] = g[2] = 0.0;
    if (rr == 0.0) return;
    double Bt, dA, dBt;
    if (p->tensor == OR_OSEEN) {
        const double c = 1.0 / (8.0 * M_PI * p->eta);
        Bt = c / (rr * rr * rr);
        dA = -c / (rr * rr);
        dBt = -3.0 * c / (rr * rr * rr * rr);
    } else if (p->overlap && rr < 2.0 * a) {
        Bt = mu0 * 3.0 / (32.0 * a * rr);
        dA = -mu0 * 9.0 / (32.0 * a);
        dBt = -mu0 * 3.0 / (32.0 * a * rr * rr);
    } else {
        const double r2 = rr * rr, r3 = r2 * rr, r4 = r2 * r2, r5 = r4 * rr, r6 = r3 * r3;
        const double a3 = a * a * a;
        Bt = mu0 * (3.0 * a / (4.0 * r3) - 3.0 * a3 / (2.0 * r5));
        dA = mu0 * (-3.0 * a / (4.0 * r2) - 3.0 * a3 / (2.0 * r4));
        dBt = mu0 * (-9.0 * a / (4.0 * r4) + 15.0 * a3 / (2.0 * r6));
    }
    const double uw = u[0] * w[0] + u[1] * w[1] + u[2] * w[2];
    const double ur = u[0] * r[0] + u[1] * r[1] + u[2] * r[2];
    const double wr = w[0] * r[0] + w[1] * r[1] + w[2] * r[2];
    for (int k = 0; k < 3; ++k)
        g[k] = (dA * uw + dBt * ur * wr) * r[k] / rr + Bt * (wr * u[k] + ur * w[k]);
}

/* Transposed mobility product (M^T y)_i = mu0 y_i + sum_{j != i} T(r_j - r_i)^T y_j.
 * Written from the definition of the transpose; that it equals M y is a
 * property the tests check, not an assumption made here. */
void oracle_mobility_transpose(const oracle_params* p, int64_t n, const double* x, const double* y,
                               double* out)
{
    const double mu0 = stokes_mobility(p);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        double acc[3] = { mu0 * y[3 * i], mu0 * y[3 * i + 1], mu0 * y[3 * i + 2] };
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double r[3] = { x[3 * j] - x[3 * i], x[3 * j + 1] - x[3 * i + 1],
                            x[3 * j + 2] - x[3 * i + 2] };
            nearest_image(p, r);
            double T[9];
            oracle_pair_tensor(p, r, T);
            for (int be = 0; be < 3; ++be)  /* column be of block mu_ji = row be of its transpose */
                acc[be] += T[0 * 3 + be] * y[3 * j] + T[1 * 3 + be] * y[3 * j + 1]
                         + T[2 * 3 + be] * y[3 * j + 2];
        }
        out[3 * i] = acc[0]; out[3 * i + 1] = acc[1]; out[3 * i + 2] = acc[2];
    }
}

/*
 * Position gradient of the scalar  s(x) = sum_k lam_k . v_k(x),  v = M(x) F:
 *   d s / d x_i = sum_{j != i} d/dx_i [ lam_i . T(x_i - x_j) F_j ]
 *               + sum_{j != i} d/dx_i [ lam_j . T(x_j - x_i) F_i ]
 * (x_i enters v_i through every T(x_i - x_j) and v_j through T(x_j - x_i)).
 * The chain rule gives +grad_r at r = x_i - x_j for the first term and
 * -grad_r at r = x_j - x_i for the second.
 */
void oracle_mobility_vjp_x(const oracle_params* p, int64_t n, const double* x, const double* f,
                           const double* lam, double* gx)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        double acc[3] = { 0.0, 0.0, 0.0 };
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double rij[3] = { x[3 * i] - x[3 * j], x[3 * i + 1] - x[3 * j + 1],
                              x[3 * i + 2] - x[3 * j + 2] };
            double rji[3] = { x[3 * j] - x[3 * i], x[3 * j + 1] - x[3 * i + 1],
                              x[3 * j + 2] - x[3 * i + 2] };
            nearest_image(p, rij);
            nearest_image(p, rji);
            double g1[3], g2[3];
            oracle_pair_grad(p, rij, lam + 3 * i, f + 3 * j, g1);
            oracle_pair_grad(p, rji, lam + 3 * j, f + 3 * i, g2);
            for (int k = 0; k < 3; ++k) acc[k] += g1[k] - g2[k];
        }
        gx[3 * i] = acc[0]; gx[3 * i + 1] = acc[1]; gx[3 * i + 2] = acc[2];
    }
}

/*
 * Discrete adjoint of `steps` explicit-Euler steps x_{k+1} = x_k + dt M(x_k) F
 * for a loss L(x_steps) whose gradient lam_N = dL/dx_steps is given.
 *   lam_k = lam_{k+1} + dt * d/dx [lam_{k+1} . M(x_k) F]
 *   dL/dF += dt * M(x_k)^T lam_{k+1}
 *   dL/dx_0 = lam_0
 * The forward trajectory is recomputed and kept whole (plain, not checkpointed).
 */
int oracle_run_adjoint_euler(const oracle_params* p, int64_t n, const double* x0, const double* f,
                             double dt, int64_t steps, const double* lam_final, double* grad_x0,
                             double* grad_f)
{
    const size_t m = 3 * (size_t)n;
    double* xs = (double*)malloc(sizeof(double) * m * (size_t)(steps + 1));
    double* lam = (double*)malloc(sizeof(double) * m);
    double* tmp = (double*)malloc(sizeof(double) * m);
    double* v = (double*)malloc(sizeof(double) * m);
    if (!xs || !lam || !tmp || !v) { free(xs); free(lam); free(tmp); free(v); return 1; }
    memcpy(xs, x0, sizeof(double) * m);
    for (int64_t s = 0; s < steps; ++s) {
        oracle_mobility(p, n, xs + m * s, f, v);
        for (size_t k = 0; k < m; ++k) xs[m * (s + 1) + k] = xs[m * s + k] + dt * v[k];
    }
    memcpy(lam, lam_final, sizeof(double) * m);
    for (size_t k = 0; k < m; ++k) grad_f[k] = 0.0;
    for (int64_t s = steps - 1; s >= 0; --s) {
        const double* xk = xs + m * s;
        oracle_mobility_transpose(p, n, xk, lam, tmp);
        for (size_t k = 0; k < m; ++k) grad_f[k] += dt * tmp[k];
        oracle_mobility_vjp_x(p, n, xk, f, lam, tmp);
        for (size_t k = 0; k < m; ++k) lam[k] += dt * tmp[k];
    }
    memcpy(grad_x0, lam, sizeof(double) * m);
    free(xs); free(lam); free(tmp); free(v);
    return 0;
}

/* ------------------------------------------------------------ lubrication */

typedef struct {
    double s_cut;   /* truncation: pairs with s = r/a - 2 < s_cut (Sec. 2.3: s_cut = 1) */
    double s_min;   /* s is clamped to >= s_min (reading: contact / overlap) */
} oracle_lub;

/*
 * Singular lubrication friction of one pair, Eq. (8), Sec. 2.3:
 *   mu0 zeta(r) = [1/(4s) - 9/40 log s] rhat rhat - 1/6 log s (I - rhat rhat),
 *   s = r/a - 2, for s < s_cut; zero otherwise.  3x3 row-major, physical units.
 */
void oracle_lub_tensor(const oracle_params* p, const oracle_lub* lub, const double r[3],
                       double Z[9])
{
    const double mu0 = stokes_mobility(p);
    const double rr = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    for (int k = 0; k < 9; ++k) Z[k] = 0.0;
    if (rr == 0.0) return;
    double s = rr / p->a - 2.0;
    if (s >= lub->s_cut) return;
    if (s < lub->s_min) s = lub->s_min;
    const double ls = log(s);
    const double cP = (1.0 / (4.0 * s) - 9.0 / 40.0 * ls) / mu0;  /* rhat rhat part */
    const double cT = (-1.0 / 6.0 * ls) / mu0;                   /* (I - rhat rhat) part */
    const double h[3] = { r[0] / rr, r[1] / rr, r[2] / rr };
    for (int al = 0; al < 3; ++al)
        for (int be = 0; be < 3; ++be) {
            const double P = h[al] * h[be];
            Z[3 * al + be] = cP * P + cT * ((al == be ? 1.0 : 0.0) - P);
        }
}

/*
 * Lubrication forces of step 2 of the algorithm of Sec. 3.1:
 *   f_i = - sum_{j != i} zeta(r_i - r_j) (v_i - v_j)
 * over all pairs (plain double loop; the primed sum of the paper runs over the
 * close pairs, which are exactly the pairs with a non-zero zeta).
 */
void oracle_lubrication_force(const oracle_params* p, const oracle_lub* lub, int64_t n,
                              const double* x, const double* v, double* f)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        double acc[3] = { 0.0, 0.0, 0.0 };
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double r[3] = { x[3 * i] - x[3 * j], x[3 * i + 1] - x[3 * j + 1],
                            x[3 * i + 2] - x[3 * j + 2] };
            nearest_image(p, r);
            double Z[9];
            oracle_lub_tensor(p, lub, r, Z);
            const double dv[3] = { v[3 * i] - v[3 * j], v[3 * i + 1] - v[3 * j + 1],
                                   v[3 * i + 2] - v[3 * j + 2] };
            for (int al = 0; al < 3; ++al)
                acc[al] -= Z[3 * al] * dv[0] + Z[3 * al + 1] * dv[1] + Z[3 * al + 2] * dv[2];
        }
        f[3 * i] = acc[0];
        f[3 * i + 1] = acc[1];
        f[3 * i + 2] = acc[2];
    }
}

/*
 * The three-step loop of Sec. 3.1 with lubrication: at every step
 *   F_k = F_ext - sum' zeta(x_k) (v_i - v_j) with the previous velocities v_{k-1},
 *   v_k = M(x_k) F_k,  x_{k+1} = x_k + dt v_k  (Euler; AB2 as oracle_run).
 * v_prev: in = the velocities before the first step, out = v of the last step.
 * traj as in oracle_run.
 */
int oracle_run_lub(const oracle_params* p, const oracle_lub* lub, int64_t n, double* x,
                   const double* f_ext, double dt, int64_t steps, int64_t step0, int integrator,
                   double* v_prev, double* traj, int64_t stride)
{
    const size_t m = 3 * (size_t)n;
    double* v = (double*)malloc(sizeof(double) * m);
    double* F = (double*)malloc(sizeof(double) * m);
    if (!v || !F) { free(v); free(F); return 1; }
    int64_t frame = 0;
    if (traj) memcpy(traj + m * frame++, x, sizeof(double) * m);
    for (int64_t s = 0; s < steps; ++s) {
        oracle_lubrication_force(p, lub, n, x, v_prev, F);
        for (size_t k = 0; k < m; ++k) F[k] += f_ext[k];
        oracle_mobility(p, n, x, F, v);
        const int euler = (integrator == 0) || (step0 + s == 0);
        for (size_t k = 0; k < m; ++k) {
            if (euler) x[k] = x[k] + dt * v[k];
            else x[k] = x[k] + dt * (1.5 * v[k] - 0.5 * v_prev[k]);
        }
        memcpy(v_prev, v, sizeof(double) * m);
        if (traj && stride > 0 && (s + 1) % stride == 0)
            memcpy(traj + m * frame++, x, sizeof(double) * m);
    }
    free(v);
    free(F);
    return 0;
}
