/*
 * Reference oracle for truncated Lennard-Jones molecular dynamics.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, plain, FP64 definition of
 * what the GPU library computes. Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it. It shares no code, header or
 * constant with the GPU library, and the GPU library never calls it.
 *
 * What it computes (van Meel, Arnold, Frenkel, Portegies Zwart, Belleman,
 * "Harvesting graphics power for MD simulations"):
 *   - the force on particle i is a sum over all other particles j of the
 *     pair force magnitude f(r_ij) along the unit vector from j to i
 *     (section 2, equation for f_i; positive f is repulsive);
 *   - the pair force is the LJ force truncated at r_c = 2.5 sigma and shifted
 *     so that it vanishes at the cutoff (section 2, equations for f_LJ and
 *     f(r));
 *   - time integration is velocity Verlet (section 2, last sentence before
 *     the implementation details).
 * The cell list of section 3 prunes this same sum without dropping any pair
 * ("care was taken not to neglect any interactions"), so the oracle is the
 * brute-force O(N^2) sum over all pairs, with no cells at all.
 *
 * Readings where the paper is silent or inconsistent (each one is listed in
 * the design notes of the repository):
 *   - f_LJ as printed lacks a factor 1/sigma; we use f_LJ = -du_LJ/dr, i.e.
 *     (24 eps / r) [2 (sigma/r)^12 - (sigma/r)^6].
 *   - The paper prints no energy. The energy consistent with the shifted force
 *     (phi = -du/dr, u(r_c) = 0) is
 *     u_sf(r) = u_LJ(r) - u_LJ(r_c) + (r - r_c) f_LJ(r_c).
 *     shift_mode = 1 selects the energy-shift alternative instead:
 *     phi = f_LJ, u = u_LJ(r) - u_LJ(r_c).
 *   - Boundary conditions are cubic periodic with the minimum-image
 *     convention, d -= L * rint(d / L) per component; the box must satisfy
 *     L >= 2 r_c so at most one image lies inside the cutoff.
 *   - The cutoff is strict: pairs with r^2 < r_c^2 interact.
 *   - The virial is W = sum over pairs of r * phi(r) (positive = repulsive),
 *     kinetic energy K = m/2 sum v^2.
 *   - Velocity Verlet is kick(dt/2) - drift(dt) - wrap into [0, L) - force -
 *     kick(dt/2).
 *
 * Derivatives for the adjoint (force-shift mode only; with the energy shift
 * the truncated force jumps at r_c and has no derivative there):
 *   - oracle_hvp: the Jacobian of the force sum applied to a vector,
 *     (J u)_i = sum_j [g (u_i - u_j) + B d (d . (u_i - u_j))], g = phi/r,
 *     B = (phi' - g)/r^2, d = r_i - r_j (minimum image);
 *   - oracle_dforce_dparams: sum_i a_i . dF_i/d(eps) and sum_i a_i . dF_i/d(sigma),
 *     with r_c = 2.5 sigma moving with sigma (no boundary term since phi(r_c) = 0);
 *   - oracle_virial_grad: the gradient of W with respect to the positions and
 *     dW/d(eps), dW/d(sigma).
 *
 * Parity status: every function below is pinned by CPU tests against closed
 * forms, textbook lattice sums, finite differences, invariances and brute
 * force on tiny inputs (tests/test_oracle.py, tests/test_oracle_adjoint.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double box;       /* cubic periodic box side L */
    double epsilon;   /* LJ well depth */
    double sigma;     /* LJ length */
    double rc;        /* cutoff radius (2.5 sigma in the paper) */
    double mass;      /* particle mass */
    double dt;        /* time step */
    int32_t shift_mode; /* 0: force shift (paper), 1: energy shift */
    int32_t pad;
} oracle_params;

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Full LJ pair force magnitude, -du_LJ/dr. */
static double f_lj(const oracle_params* p, double r) {
    double sr = p->sigma / r;
    double sr6 = sr * sr * sr * sr * sr * sr;
    return 24.0 * p->epsilon / r * (2.0 * sr6 * sr6 - sr6);
}

/* Full LJ pair energy. */
static double u_lj(const oracle_params* p, double r) {
    double sr = p->sigma / r;
    double sr6 = sr * sr * sr * sr * sr * sr;
    return 4.0 * p->epsilon * (sr6 * sr6 - sr6);
}

/* Truncated, shifted pair force magnitude phi(r) and energy u(r) for r < rc. */
static void pair_terms(const oracle_params* p, double r, double* phi, double* u) {
    if (!(r < p->rc)) {
        *phi = 0.0;
        *u = 0.0;
        return;
    }
    if (p->shift_mode == 0) {
        double fc = f_lj(p, p->rc);
        *phi = f_lj(p, r) - fc;
        *u = u_lj(p, r) - u_lj(p, p->rc) + (r - p->rc) * fc;
    } else {
        *phi = f_lj(p, r);
        *u = u_lj(p, r) - u_lj(p, p->rc);
    }
}

/* Public pair evaluation (used by the closed-form tests). */
void oracle_pair(const oracle_params* p, double r, double* phi, double* u) {
    pair_terms(p, r, phi, u);
}

/* Minimum-image displacement d = r_i - r_j. */
static void min_image(const oracle_params* p, const double* ri, const double* rj, double* d) {
    for (int k = 0; k < 3; ++k) {
        double x = ri[k] - rj[k];
        x -= p->box * rint(x / p->box);
        d[k] = x;
    }
}

/*
 * Forces, energy and virial for the listed rows i (all other j considered).
 * pos: n x 3 doubles. rows: nrows indices, or NULL for all n rows in order.
 * force: nrows x 3 out. u_row, w_row: per-row halves of the pair sums
 * (nullable), so that summing them over all rows gives U and W.
 * Returns 0, or -1 on invalid arguments.
 */
int oracle_forces_rows(const oracle_params* p, int64_t n, const double* pos, int64_t nrows,
                       const int64_t* rows, double* force, double* u_row, double* w_row) {
    if (n < 0 || nrows < 0 || !(p->box >= 2.0 * p->rc)) return -1;
    const double rc2 = p->rc * p->rc;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nrows; ++k) {
        int64_t i = rows ? rows[k] : k;
        double f[3] = {0.0, 0.0, 0.0};
        double usum = 0.0, wsum = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3];
            min_image(p, pos + 3 * i, pos + 3 * j, d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (!(r2 < rc2)) continue;
            double r = sqrt(r2);
            double phi, u;
            pair_terms(p, r, &phi, &u);
            /* f_i = -sum f(r) (r_j - r_i)/r = sum f(r) d / r, d = r_i - r_j */
            for (int c = 0; c < 3; ++c) f[c] += phi * d[c] / r;
            usum += u;
            wsum += r * phi;
        }
        for (int c = 0; c < 3; ++c) force[3 * k + c] = f[c];
        if (u_row) u_row[k] = 0.5 * usum;
        if (w_row) w_row[k] = 0.5 * wsum;
    }
    return 0;
}

/* All forces plus totals uw[0] = U, uw[1] = W. */
int oracle_forces(const oracle_params* p, int64_t n, const double* pos, double* force, double* uw) {
    double* ur = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* wr = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!ur || !wr) {
        free(ur);
        free(wr);
        return -2;
    }
    int rc = oracle_forces_rows(p, n, pos, n, NULL, force, ur, wr);
    if (rc == 0 && uw) {
        double U = 0.0, W = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            U += ur[i];
            W += wr[i];
        }
        uw[0] = U;
        uw[1] = W;
    }
    free(ur);
    free(wr);
    return rc;
}

/* Kinetic energy K = m/2 sum |v|^2. */
double oracle_kinetic(const oracle_params* p, int64_t n, const double* vel) {
    double k = 0.0;
    for (int64_t i = 0; i < 3 * n; ++i) k += vel[i] * vel[i];
    return 0.5 * p->mass * k;
}

/*
 * Brute-force neighbour sets {j != i : r_ij^2 < rc^2} in CSR form.
 * counts: n out. idx: flat list in row order, ascending j within a row.
 * cap: capacity of idx. guard: number of ordered pairs whose r^2 lies within
 * a relative band `band` of rc^2 (those pairs are where FP32 and FP64 cutoff
 * tests may legitimately disagree). Returns the total number of entries, or
 * -1 if cap is too small (counts are still filled).
 */
int64_t oracle_neighbors(const oracle_params* p, int64_t n, const double* pos, int32_t* counts,
                         int32_t* idx, int64_t cap, double band, int64_t* guard) {
    const double rc2 = p->rc * p->rc;
    int64_t g = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : g)
    for (int64_t i = 0; i < n; ++i) {
        int32_t c = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3];
            min_image(p, pos + 3 * i, pos + 3 * j, d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (fabs(r2 - rc2) < band * rc2) ++g;
            if (r2 < rc2) ++c;
        }
        counts[i] = c;
    }
    if (guard) *guard = g;
    int64_t total = 0;
    for (int64_t i = 0; i < n; ++i) total += counts[i];
    if (total > cap) return -1;
    int64_t off = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3];
            min_image(p, pos + 3 * i, pos + 3 * j, d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 < rc2) idx[off++] = (int32_t)j;
        }
    }
    return total;
}

/* Bring one coordinate into [0, L). */
static double wrap_coord(double x, double L) {
    x -= L * floor(x / L);
    if (x >= L) x -= L;
    if (x < 0.0 || x >= L) x = 0.0;
    return x;
}

/*
 * Velocity Verlet, nsteps full steps, in place on pos and vel (n x 3 each).
 * Each step: v += dt/(2m) F; r += dt v; wrap; F = F(r); v += dt/(2m) F.
 * thermo: (nsteps + 1) x 3 doubles (U, K, W) at steps 0..nsteps, nullable.
 * Returns 0, or a negative code on failure.
 */
int oracle_run(const oracle_params* p, int64_t n, double* pos, double* vel, int32_t nsteps,
               double* thermo) {
    double* f = (double*)malloc(sizeof(double) * (size_t)(3 * (n > 0 ? n : 1)));
    if (!f) return -2;
    double uw[2];
    int rc = oracle_forces(p, n, pos, f, uw);
    if (rc) {
        free(f);
        return rc;
    }
    if (thermo) {
        thermo[0] = uw[0];
        thermo[1] = oracle_kinetic(p, n, vel);
        thermo[2] = uw[1];
    }
    const double h = 0.5 * p->dt / p->mass;
    for (int32_t s = 1; s <= nsteps; ++s) {
        for (int64_t i = 0; i < 3 * n; ++i) {
            vel[i] += h * f[i];
            pos[i] = wrap_coord(pos[i] + p->dt * vel[i], p->box);
        }
        rc = oracle_forces(p, n, pos, f, uw);
        if (rc) break;
        for (int64_t i = 0; i < 3 * n; ++i) vel[i] += h * f[i];
        if (thermo) {
            thermo[3 * s + 0] = uw[0];
            thermo[3 * s + 1] = oracle_kinetic(p, n, vel);
            thermo[3 * s + 2] = uw[1];
        }
    }
    free(f);
    return rc;
}

/* phi'(r) = f_LJ'(r) = (24 eps / r^2) [-26 (sigma/r)^12 + 7 (sigma/r)^6]; the shift is constant in r. */
static double dphi_dr(const oracle_params* p, double r) {
    double sr = p->sigma / r;
    double sr6 = sr * sr * sr * sr * sr * sr;
    return 24.0 * p->epsilon / (r * r) * (-26.0 * sr6 * sr6 + 7.0 * sr6);
}

/* d phi / d sigma at fixed r, with r_c = rc_over_sigma * sigma moving along:
 * d f_LJ(r)/d sigma = (24 eps / (r sigma)) [24 (sigma/r)^12 - 6 (sigma/r)^6],
 * and f_LJ(r_c(sigma); sigma) is proportional to eps / sigma, so its total
 * derivative is -f_LJ(r_c)/sigma. */
static double dphi_dsigma(const oracle_params* p, double r) {
    double sr = p->sigma / r;
    double sr6 = sr * sr * sr * sr * sr * sr;
    double d = 24.0 * p->epsilon / (r * p->sigma) * (24.0 * sr6 * sr6 - 6.0 * sr6);
    if (p->shift_mode == 0) d += f_lj(p, p->rc) / p->sigma;
    return d;
}

/* out = J u with J = dF/dr (force-shift mode). u, out: n x 3. */
int oracle_hvp(const oracle_params* p, int64_t n, const double* pos, const double* u, double* out) {
    if (p->shift_mode != 0 || !(p->box >= 2.0 * p->rc)) return -1;
    const double rc2 = p->rc * p->rc;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3];
            min_image(p, pos + 3 * i, pos + 3 * j, d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (!(r2 < rc2)) continue;
            double r = sqrt(r2);
            double phi, uu;
            pair_terms(p, r, &phi, &uu);
            double g = phi / r;
            double B = (dphi_dr(p, r) - g) / r2;
            double du[3], dd = 0.0;
            for (int c = 0; c < 3; ++c) {
                du[c] = u[3 * i + c] - u[3 * j + c];
                dd += d[c] * du[c];
            }
            for (int c = 0; c < 3; ++c) acc[c] += g * du[c] + B * d[c] * dd;
        }
        for (int c = 0; c < 3; ++c) out[3 * i + c] = acc[c];
    }
    return 0;
}

/* out2[0] = sum_i a_i . dF_i/d eps, out2[1] = sum_i a_i . dF_i/d sigma. */
int oracle_dforce_dparams(const oracle_params* p, int64_t n, const double* pos, const double* a, double* out2) {
    if (p->shift_mode != 0 || !(p->box >= 2.0 * p->rc)) return -1;
    const double rc2 = p->rc * p->rc;
    double se = 0.0, ss = 0.0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : se, ss)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3];
            min_image(p, pos + 3 * i, pos + 3 * j, d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (!(r2 < rc2)) continue;
            double r = sqrt(r2);
            double phi, uu;
            pair_terms(p, r, &phi, &uu);
            double da = d[0] * a[3 * i] + d[1] * a[3 * i + 1] + d[2] * a[3 * i + 2];
            se += phi / p->epsilon / r * da; /* phi is linear in eps, shift included */
            ss += dphi_dsigma(p, r) / r * da;
        }
    }
    out2[0] = se;
    out2[1] = ss;
    return 0;
}

/* grad: n x 3 gradient of W = sum over pairs r phi(r); dw2 = {dW/d eps, dW/d sigma}. */
int oracle_virial_grad(const oracle_params* p, int64_t n, const double* pos, double* grad, double* dw2) {
    if (p->shift_mode != 0 || !(p->box >= 2.0 * p->rc)) return -1;
    const double rc2 = p->rc * p->rc;
    double we = 0.0, ws = 0.0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : we, ws)
    for (int64_t i = 0; i < n; ++i) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3];
            min_image(p, pos + 3 * i, pos + 3 * j, d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (!(r2 < rc2)) continue;
            double r = sqrt(r2);
            double phi, uu;
            pair_terms(p, r, &phi, &uu);
            /* d(r phi)/dr = phi + r phi', along the unit vector d/r */
            double s = (phi + r * dphi_dr(p, r)) / r;
            for (int c = 0; c < 3; ++c) acc[c] += s * d[c];
            we += 0.5 * r * phi / p->epsilon;
            ws += 0.5 * r * dphi_dsigma(p, r);
        }
        for (int c = 0; c < 3; ++c) grad[3 * i + c] = acc[c];
    }
    dw2[0] = we;
    dw2[1] = ws;
    return 0;
}
