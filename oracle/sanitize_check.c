/*
 * TEST INFRASTRUCTURE ONLY: a driver that runs every entry point of the FP64
 * oracle (hsref.c, compiled into the same program) on small grids, for builds
 * with the address and undefined-behaviour sanitizers
 * (tests/test_oracle_sanitize.py).  It checks nothing numerically: the pins
 * live in the Python tests; here a sanitizer report or a failing call ends the
 * program with a nonzero status.
 *
 * Cases: slits and periodic boxes for sigma 2..8 (odd sigma included), the
 * Carnahan-Starling closure, the attraction, a solid mask, the supplied-force
 * step, and the 39-velocity lattice with and without the non-isothermal terms.
 */
#include "hsref.c"

#include <stdio.h>

static unsigned long long rng_state = 88172645463325252ull;

static double urand(void)
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

static int run_case(int nx, int ny, int nz, int walls, int sigma, int lattice, int thermal, int g2_model,
                    double att_eps, int mask)
{
    hsref_params p;
    memset(&p, 0, sizeof(p));
    p.nx = nx, p.ny = ny, p.nz = nz;
    p.wall_lo = walls, p.wall_hi = walls;
    p.sigma = sigma;
    p.tau = 0.9;
    p.accel[0] = 1e-5;
    p.g2_model = g2_model;
    p.wall_reg = 1;
    p.att_eps = att_eps;
    p.att_range = att_eps != 0.0 ? 1.5 : 0.0;
    p.lattice = lattice;
    p.thermal = thermal;
    hsref_ctx *c = hsref_create(&p);
    if (!c) {
        fprintf(stderr, "create failed: %dx%dx%d sigma %d lattice %d\n", nx, ny, nz, sigma, lattice);
        return 1;
    }
    const int N = nx * ny * nz;
    const int q = hsref_q(c);
    double *n = malloc(sizeof(double) * N), *u = malloc(sizeof(double) * 3 * N);
    double *T = malloc(sizeof(double) * N), *F = malloc(sizeof(double) * 3 * N);
    double *f = malloc(sizeof(double) * (size_t)q * N), *pz = malloc(sizeof(double) * 4 * nz);
    uint8_t *sol = calloc(N, 1);
    const double nb = 6.0 * 0.2 / (M_PI * sigma * sigma * sigma);
    for (int k = 0; k < N; ++k) {
        n[k] = nb * (1.0 + 0.05 * (2.0 * urand() - 1.0));
        T[k] = (2.0 / 3.0) * (1.0 + 0.02 * (2.0 * urand() - 1.0));
    }
    for (int k = 0; k < 3 * N; ++k) u[k] = 1e-3 * (2.0 * urand() - 1.0);
    int rc = 0;
    if (mask) {
        sol[(nz / 2) * nx * ny + (ny / 2) * nx + nx / 2] = 1;
        rc |= hsref_set_solid(c, sol);
    }
    rc |= thermal ? hsref_init_thermal(c, n, u, T) : hsref_init(c, n, u);
    rc |= hsref_step(c, 3);
    rc |= hsref_force(c, F);
    rc |= hsref_eta_bar(c, n);
    rc |= hsref_moments(c, n, u);
    rc |= hsref_profiles(c, pz, pz + nz);
    rc |= hsref_attraction_potential(c, T);
    rc |= hsref_get_populations(c, f);
    rc |= hsref_set_populations(c, f);
    if (lattice != 39) {
        for (int k = 0; k < 3 * N; ++k) F[k] *= 0.5;
        rc |= hsref_step_with_force(c, F);
    }
    if (thermal) rc |= hsref_thermal_fields(c, T, F);
    rc |= hsref_step(c, 2);
    hsref_destroy(c);
    free(n), free(u), free(T), free(F), free(f), free(pz), free(sol);
    if (rc) fprintf(stderr, "a call failed: %dx%dx%d sigma %d lattice %d\n", nx, ny, nz, sigma, lattice);
    return rc != 0;
}

int main(void)
{
    int bad = 0;
    hsref_set_threads(2);
    for (int sigma = 2; sigma <= 8; ++sigma) {
        const int w = (sigma + 1) / 2;
        bad |= run_case(sigma + 3, sigma + 2, 2 * w + 5, w, sigma, 19, 0, sigma & 1, 0.0, 0);
        bad |= run_case(sigma + 2, sigma + 3, sigma + 4, 0, sigma, 19, 0, 0, 0.0, 0);
    }
    bad |= run_case(8, 7, 14, 2, 4, 19, 0, 0, 1e-3, 1);
    bad |= run_case(7, 6, 12, 2, 3, 39, 0, 0, 0.0, 0);
    bad |= run_case(6, 6, 8, 0, 4, 39, 1, 0, 0.0, 0);
    bad |= run_case(6, 7, 13, 2, 4, 39, 1, 1, 0.0, 0);
    for (int sigma = 2; sigma <= 8; ++sigma) {
        double W[18], s[54], alpha[72];
        int ncorner[18], d[216];
        bad |= hsref_shell_table(sigma, W, s, ncorner, d, alpha) < 0;
        bad |= hsref_ball_count(sigma) < 1;
    }
    if (bad) return 1;
    printf("oracle sanitizer driver: all cases ran\n");
    return 0;
}
