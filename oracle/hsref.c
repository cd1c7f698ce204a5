/*
 * hsref.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU oracle for the time step of the lattice Boltzmann
 * method for inhomogeneous hard-sphere fluids of Melchionna and Marini Bettolo
 * Marconi ("Lattice Boltzmann method for inhomogeneous fluids", EPL).
 *
 * Only the test suite, the package smoke check and the benchmark's CPU-baseline
 * leg load this library.  The GPU library never includes, links or calls it, and
 * it shares no source with it.
 *
 * Equation numbers are the paper's printed ones:
 *   (3)  Dufty-Santos-Brey kinetic equation: BGK relaxation plus the Hermite
 *        sources C^(1) (momentum transfer) and C^(2) (energy transfer);
 *   (8)  hydrodynamic moments as lattice sums over the populations;
 *   (10) first-order forward-Euler propagation with the Hermite source;
 *   (11) second-order (low-Mach) local equilibrium;
 *   (12) C^(1) as a surface integral over the sphere of radius sigma with the
 *        density-current coupling term.
 * Section "Methods and Results" also fixes: the isothermal restriction (T const,
 * so C^(2) and all temperature differences drop out), the coarse-grained density
 * (uniform smearing over a ball of radius sigma/2, packing fraction
 * eta = pi sigma^3 n / 6), the contact-value closure for g2 evaluated at the pair
 * midpoint, the 18-point spherical quadrature with 6 on-lattice and 12
 * interpolated points, and the wall factor (1 - exp(-|r - r_w|/sigma)) on the
 * density-current term.  Subsection "Numerical validation" fixes the halfway
 * bounce-back walls and the uniform driving field parallel to the walls.
 *
 * Readings where the paper is silent or garbled (all listed in the design notes):
 *   - m = 1, v_T^2 = k_B T = 1/3 and the standard D3Q19 weights 1/3, 1/18, 1/36;
 *   - the surface integral is sigma^2 * 4 pi * sum_q W_q (...), with the 18-point
 *     rule W = 1/30 on the 6 axis points and 1/15 on the 12 face diagonals;
 *   - the "linear interpolation" of an off-lattice point interpolates the pair
 *     elements (g2 * n * [...] of each lattice pair) bilinearly over the four
 *     in-plane lattice corners around the point;
 *   - g2 is evaluated at the midpoint of each actual lattice pair; at a
 *     half-integer midpoint the coarse-grained packing fraction is the mean over
 *     the 2^h lattice nodes nearest to it (h = number of half-integer coordinates);
 *   - the closure is the printed one, (1 - eta/2 + eta^2/4)/(1 - eta)^3, with the
 *     Carnahan-Starling contact value (1 - eta/2)/(1 - eta)^3 as a switch;
 *   - the velocity in the equilibrium and in the current term is u = j/n, with
 *     the force added as the first-order source 3 w_i c_i . F;
 *   - the external field is a force per particle g, so its momentum source is n g;
 *   - solid nodes and points beyond the array carry n = j = 0;
 *   - the wall factor multiplies only the current term, is evaluated at the
 *     receiving node, and uses the distance to the nearest halfway wall plane.
 *
 * Optional mean-field attraction (the generalisation to attractive forces the
 * paper's conclusions name; off unless att_eps != 0).  In equilibrium the
 * paper ties C^(1) to density functional theory, C^(1) = -n grad dF_exc/dn
 * (m = 1); a mean-field attractive functional (1/2) sum sum n n' phi adds
 * dF/dn = (phi * n), so the attraction enters the force as
 *   Phi(r)    = -att_eps sum_{o: |o_x|,|o_y|,|o_z| <= R} exp(-|o|^2/att_range^2) n(r+o),
 *   C1_att(r) = -n(r) [Phi(r + e_a) - Phi(r - e_a)] / 2   (each axis a),
 * with R = ceil(3 att_range), the same n = 0 on solid nodes and beyond the
 * array, and periodic images along periodic axes.  Written here as the plain
 * triple sum.
 *
 * Optional third-order lattice (lattice = 39; the higher-order Hermite basis the
 * paper names in its discussion of the wall regulariser and in its conclusions,
 * as the way to high Knudsen numbers).  Readings, all in the design notes:
 *   - the 39-velocity quadrature of degree 7 with integer velocities: the rest
 *     vector (weight 1/12), the 6 axis vectors of length 1 (1/12), the 8 cube
 *     diagonals (1, 1, 1) (1/27), the 6 axis vectors of length 2 (2/135), the 12
 *     vectors (2, 2, 0) (1/432) and the 6 axis vectors of length 3 (1/1620); its
 *     second moment fixes v_T^2 = k_B T = 2/3 in lattice units, which also enters
 *     the force's k_B T and its current-term coefficient;
 *   - the local equilibrium (11) carried to third order in u, the Hermite
 *     expansion of the Maxwellian through h^(3);
 *   - "removing the off-basis contributions": before relaxation the
 *     non-equilibrium part f - f_eq is replaced by its projection on h^(2) and
 *     h^(3), f_neq -> w_i [h2(c_i) : a2 / (2 v_T^4) + h3(c_i) : a3 / (6 v_T^6)],
 *     a_l = sum_i h_l(c_i) (f_i - f_eq,i); post-collision
 *     f = f_eq + (1 - 1/tau) f_neq + w_i c_i . F / v_T^2 (the same first-order
 *     source as on the 19-velocity lattice);
 *   - halfway bounce-back for the longer links: a population that would cross
 *     a wall plane is reversed where it meets the plane and travels the rest of
 *     the step back, landing on a lattice node (every link of this set that
 *     crosses a z plane has |c_x|, |c_y| equal to 0 or |c_z|); the slit needs at
 *     least 3 fluid layers so that no link crosses both walls; solid masks are
 *     not available on this lattice.
 *
 * Optional non-isothermal terms (thermal = 1, on the third-order lattice only):
 * the temperature term of C^(1) and the energy source C^(2) that the paper
 * derives next to equation (12) and then drops by taking T constant.  Readings,
 * all in the design notes:
 *   - k_B = m = 1; n T = (1/3) sum_i f_i |c_i - u|^2; solid nodes carry T = 0;
 *   - v_T^2 = T(r), the receiving node's temperature, in C^(1)'s prefactor, in
 *     kappa = 2/(v_T sqrt(pi)), and in both temperature terms; the garbled
 *     T(r + s_hat) is T(r + sigma s_hat), the partner of the pair;
 *   - C^(1) = -v_T^2 sigma^2 4 pi n sum_q W_q s_q sum_k alpha_k G_k
 *             [n' - chi kappa s.(j' - n' u) + n' (T' - T) / (2 v_T^2)],
 *     C^(2) = v_T^2 sigma^2 4 pi n sum_q W_q sum_k alpha_k G_k
 *             [-s.(j' - n' u) / 2 + n' (T' - T) / (sqrt(pi) v_T)],
 *     with the same quadrature, interpolation and midpoint closure as C^(1)
 *     (the wall factor only on C^(1)'s current term, as before); C^(2) is the
 *     energy gained per unit volume and step;
 *   - the equilibrium is the third-order Hermite expansion of the Maxwellian at
 *     (n, u, T) about the lattice temperature T0 = 2/3 (xi = c/sqrt(T0),
 *     theta = T/T0): w n [1 + xi.u~ + ((xi.u~)^2 - u~^2 + (theta - 1)(xi^2 - 3))/2
 *     + (xi.u~)((xi.u~)^2 - 3 u~^2 + 3 (theta - 1)(xi^2 - 5))/6], u~ = u/sqrt(T0);
 *   - the sources are the force's Hermite terms through second order and the
 *     energy source on the trace of h^(2):
 *     w_i [c.F/T0 + ((c.F)(c.u) - T0 F.u)/T0^2 + C2 (c^2 - 3 T0)/(3 T0^2)],
 *     so that momentum gains F and energy gains F.u + C2;
 *   - the same regularised collision; bounce-back walls are adiabatic.
 *
 * Optional solid mask (hsref_set_solid): any node may be solid, beyond the wall
 * layers.  Solid nodes carry n = j = 0 and take part in nothing; a population
 * heading into a solid node returns reversed (halfway bounce-back), as at the
 * walls; the wall factor of a fluid node uses the distance to the nearest
 * solid surface, read as the distance to the nearest solid node centre (wall
 * layers included, periodic images along periodic axes) minus half a lattice
 * spacing, which is the halfway-plane distance of the flat walls.  Found here
 * by brute force over all solid nodes.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NQ 19
#define QMAX 39
/* grids below this size run on one thread: the fork/join of four phases per
 * step would cost more than the work */
#define PAR_MIN_NODES 32768
#define NSHELL 18

typedef struct {
    int32_t nx, ny, nz;
    int32_t wall_lo, wall_hi; /* solid layers at each z end; both 0 -> z periodic */
    int32_t sigma;            /* hard-sphere diameter in lattice units (>= 2) */
    double tau;               /* BGK relaxation time */
    double accel[3];          /* external force per particle (m = 1) */
    int32_t g2_model;         /* 0: printed closure, 1: Carnahan-Starling */
    int32_t wall_reg;         /* 1: wall factor on the current term */
    int32_t force_mode;       /* 0: hard-sphere term on, 2: off */
    double att_eps;           /* depth of the Gaussian attraction (0: off) */
    double att_range;         /* its range in lattice units */
    int32_t lattice;          /* 19 (or 0): D3Q19; 39: the third-order lattice */
    int32_t thermal;          /* 1: temperature field and energy source (lattice 39) */
} hsref_params;

/* D3Q19 velocities, the discrete set of section "Methods and Results". */
static const int CV[NQ][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

/* The 39-velocity third-order lattice; each velocity is followed by its
 * opposite.  Weights by shell: |c|^2 = 0, 1: 1/12; 3: 1/27; 4: 2/135; 8: 1/432;
 * 9: 1/1620. */
static const int CV39[QMAX][3] = {
    {0, 0, 0},
    {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},   {0, -1, 0},  {0, 0, 1},   {0, 0, -1},
    {1, 1, 1},   {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1}, {1, -1, 1},  {-1, 1, -1},
    {-1, 1, 1},  {1, -1, -1},
    {2, 0, 0},   {-2, 0, 0},  {0, 2, 0},   {0, -2, 0},  {0, 0, 2},   {0, 0, -2},
    {2, 2, 0},   {-2, -2, 0}, {2, -2, 0},  {-2, 2, 0},  {2, 0, 2},   {-2, 0, -2},
    {2, 0, -2},  {-2, 0, 2},  {0, 2, 2},   {0, -2, -2}, {0, 2, -2},  {0, -2, 2},
    {3, 0, 0},   {-3, 0, 0},  {0, 3, 0},   {0, -3, 0},  {0, 0, 3},   {0, 0, -3}};

static double weight39_of(const int *v)
{
    switch (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) {
    case 0:
    case 1: return 1.0 / 12.0;
    case 3: return 1.0 / 27.0;
    case 4: return 2.0 / 135.0;
    case 8: return 1.0 / 432.0;
    default: return 1.0 / 1620.0;
    }
}

static double weight_of(int i)
{
    int s = abs(CV[i][0]) + abs(CV[i][1]) + abs(CV[i][2]);
    if (s == 0) return 1.0 / 3.0;
    if (s == 1) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

/* One of the 18 quadrature directions on the sphere of radius sigma. */
typedef struct {
    double W;         /* quadrature weight (sums to 1 over the 18 points) */
    double s[3];      /* unit vector s_hat */
    int ncorner;      /* 1 for an on-lattice point, 4 for an interpolated one */
    int d[4][3];      /* lattice offsets of the corners */
    double alpha[4];  /* interpolation weights of the corners */
} shell_dir;

struct hsref_ctx {
    hsref_params p;
    int64_t N;
    int zperiodic;
    int q;                /* number of velocities, 19 or 39 */
    int cv[QMAX][3];
    double cs2;           /* v_T^2 of the lattice: 1/3 or 2/3 */
    double w[QMAX];
    int opp[QMAX];
    shell_dir shell[NSHELL];
    int nball;
    int (*ball)[3];
    double *chi;     /* [nz] wall factor of the receiving layer */
    double *f;       /* [q][N] populations after streaming */
    double *fs;      /* [q][N] scratch for the streamed populations */
    double *n;       /* [N] */
    double *j;       /* [3][N] */
    double *u;       /* [3][N] */
    double *eb;      /* [N] coarse-grained packing fraction */
    double *F;       /* [3][N] total force */
    double *phi;     /* [N] mean-field attraction potential (att_eps != 0) */
    double *T;       /* [N] temperature (thermal) */
    double *Q;       /* [N] energy source C^(2) (thermal) */
    int att_R;       /* its cube half-width, ceil(3 att_range) */
    uint8_t *solid;  /* [N] solid mask (NULL: only the wall layers are solid) */
    double *chi_n;   /* [N] per-node wall factor when a mask is set */
};

typedef struct hsref_ctx hsref_ctx;

/* ---------------------------------------------------------------- tables */

/* The 18-point rule: the 6 axis points +-sigma e_a lie on the lattice; each of
 * the 12 face-diagonal points sigma (s_a e_a + s_b e_b)/sqrt(2) is replaced by
 * the 4 lattice corners of its in-plane cell with bilinear weights. */
static void build_shell(int sigma, shell_dir *sh)
{
    int q = 0;
    for (int a = 0; a < 3; ++a) {
        for (int sgn = 1; sgn >= -1; sgn -= 2) {
            shell_dir *e = &sh[q++];
            memset(e, 0, sizeof(*e));
            e->W = 1.0 / 30.0;
            e->s[a] = (double)sgn;
            e->ncorner = 1;
            e->d[0][a] = sgn * sigma;
            e->alpha[0] = 1.0;
        }
    }
    const double A = (double)sigma / sqrt(2.0);
    const int l = (int)floor(A);
    const double th = A - (double)l;
    const int planes[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (int pl = 0; pl < 3; ++pl) {
        int a = planes[pl][0], b = planes[pl][1];
        const int sab[2][2] = {{1, 1}, {1, -1}};
        for (int v = 0; v < 2; ++v) {
            /* the direction and its negation, as a pair */
            for (int neg = 0; neg < 2; ++neg) {
                int sa = neg ? -sab[v][0] : sab[v][0];
                int sb = neg ? -sab[v][1] : sab[v][1];
                shell_dir *e = &sh[q++];
                memset(e, 0, sizeof(*e));
                e->W = 1.0 / 15.0;
                e->s[a] = sa / sqrt(2.0);
                e->s[b] = sb / sqrt(2.0);
                e->ncorner = 4;
                int k = 0;
                for (int ia = 0; ia < 2; ++ia) {
                    for (int ib = 0; ib < 2; ++ib) {
                        e->d[k][a] = sa * (l + ia);
                        e->d[k][b] = sb * (l + ib);
                        double wa = ia ? th : 1.0 - th;
                        double wb = ib ? th : 1.0 - th;
                        e->alpha[k] = wa * wb;
                        ++k;
                    }
                }
            }
        }
    }
}

/* All integer offsets inside the closed ball of radius sigma/2. */
static int build_ball(int sigma, int (*out)[3])
{
    int r = sigma / 2 + 1, cnt = 0;
    for (int z = -r; z <= r; ++z)
        for (int y = -r; y <= r; ++y)
            for (int x = -r; x <= r; ++x)
                if (4 * (x * x + y * y + z * z) <= sigma * sigma) {
                    if (out) {
                        out[cnt][0] = x;
                        out[cnt][1] = y;
                        out[cnt][2] = z;
                    }
                    ++cnt;
                }
    return cnt;
}

/* Contact value of the pair correlation as a function of the coarse-grained
 * packing fraction (section "Methods and Results", Fischer-Methfessel
 * prescription). */
double hsref_g2(int model, double eta)
{
    double om = 1.0 - eta;
    if (model == 1) return (1.0 - 0.5 * eta) / (om * om * om);
    return (1.0 - 0.5 * eta + 0.25 * eta * eta) / (om * om * om);
}

/* ---------------------------------------------------------------- helpers */

static int wrapi(int v, int n)
{
    int m = v % n;
    return m < 0 ? m + n : m;
}

static int is_solid_z(const hsref_ctx *c, int z)
{
    return z < c->p.wall_lo || z >= c->p.nz - c->p.wall_hi;
}

/* Lattice node at (x,y,z) after periodic wrapping; -1 when the point lies
 * beyond a non-periodic end of the array. */
static int64_t node_at(const hsref_ctx *c, int x, int y, int z)
{
    x = wrapi(x, c->p.nx);
    y = wrapi(y, c->p.ny);
    if (c->zperiodic)
        z = wrapi(z, c->p.nz);
    else if (z < 0 || z >= c->p.nz)
        return -1;
    return (int64_t)x + (int64_t)c->p.nx * ((int64_t)y + (int64_t)c->p.ny * z);
}

static int fluid_node(const hsref_ctx *c, int64_t id)
{
    if (id < 0) return 0;
    int z = (int)(id / ((int64_t)c->p.nx * c->p.ny));
    if (is_solid_z(c, z)) return 0;
    return !(c->solid && c->solid[id]);
}

/* Wall factor of the receiving node. */
static double chi_at(const hsref_ctx *c, int64_t id, int z)
{
    return c->chi_n ? c->chi_n[id] : c->chi[z];
}

/* ---------------------------------------------------------------- create */

void hsref_set_threads(int nt)
{
#ifdef _OPENMP
    if (nt > 0) omp_set_num_threads(nt);
#else
    (void)nt;
#endif
}

int hsref_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

hsref_ctx *hsref_create(const hsref_params *p)
{
    if (!p) return NULL;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return NULL;
    if (p->wall_lo < 0 || p->wall_hi < 0) return NULL;
    if ((p->wall_lo == 0) != (p->wall_hi == 0)) return NULL;
    if (p->wall_lo + p->wall_hi >= p->nz) return NULL;
    if (p->force_mode != 2 && p->sigma < 2) return NULL;
    if (!(p->tau > 0.5)) return NULL;
    if (!isfinite(p->att_eps) || (p->att_eps != 0.0 && !(p->att_range > 0.0 && p->att_range <= 10.0)))
        return NULL;
    if (p->lattice != 0 && p->lattice != 19 && p->lattice != 39) return NULL;
    /* no link of the third-order lattice may cross both walls */
    if (p->lattice == 39 && p->wall_lo > 0 && p->nz - p->wall_lo - p->wall_hi < 3) return NULL;
    if (p->thermal != 0 && (p->thermal != 1 || p->lattice != 39)) return NULL;
    hsref_ctx *c = (hsref_ctx *)calloc(1, sizeof(hsref_ctx));
    if (!c) return NULL;
    c->p = *p;
    c->N = (int64_t)p->nx * p->ny * p->nz;
    c->zperiodic = (p->wall_lo == 0 && p->wall_hi == 0);
    c->q = p->lattice == 39 ? 39 : NQ;
    c->cs2 = p->lattice == 39 ? 2.0 / 3.0 : 1.0 / 3.0;
    for (int i = 0; i < c->q; ++i) {
        for (int a = 0; a < 3; ++a) c->cv[i][a] = c->q == 39 ? CV39[i][a] : CV[i][a];
        c->w[i] = c->q == 39 ? weight39_of(CV39[i]) : weight_of(i);
    }
    for (int i = 0; i < c->q; ++i)
        for (int k = 0; k < c->q; ++k)
            if (c->cv[k][0] == -c->cv[i][0] && c->cv[k][1] == -c->cv[i][1] && c->cv[k][2] == -c->cv[i][2])
                c->opp[i] = k;
    int sig = p->sigma >= 2 ? p->sigma : 2;
    build_shell(sig, c->shell);
    c->nball = build_ball(sig, NULL);
    c->ball = malloc(sizeof(int[3]) * (size_t)c->nball);
    build_ball(sig, c->ball);
    c->chi = malloc(sizeof(double) * (size_t)p->nz);
    for (int z = 0; z < p->nz; ++z) {
        double chi = 1.0;
        if (!c->zperiodic && p->wall_reg) {
            double za = p->wall_lo - 0.5, zb = p->nz - p->wall_hi - 0.5;
            double dw = fmin((double)z - za, zb - (double)z);
            chi = 1.0 - exp(-dw / (double)sig);
        }
        c->chi[z] = chi;
    }
    size_t N = (size_t)c->N;
    c->f = calloc((size_t)c->q * N, sizeof(double));
    c->fs = calloc((size_t)c->q * N, sizeof(double));
    c->n = calloc(N, sizeof(double));
    c->j = calloc(3 * N, sizeof(double));
    c->u = calloc(3 * N, sizeof(double));
    c->eb = calloc(N, sizeof(double));
    c->F = calloc(3 * N, sizeof(double));
    c->phi = calloc(N, sizeof(double));
    c->T = calloc(N, sizeof(double));
    c->Q = calloc(N, sizeof(double));
    c->att_R = p->att_eps != 0.0 ? (int)ceil(3.0 * p->att_range) : 0;
    if (!c->ball || !c->chi || !c->f || !c->fs || !c->n || !c->j || !c->u || !c->eb || !c->F || !c->phi ||
        !c->T || !c->Q) {
        free(c->ball); free(c->chi); free(c->f); free(c->fs); free(c->n); free(c->j);
        free(c->u); free(c->eb); free(c->F); free(c->phi); free(c->T); free(c->Q); free(c);
        return NULL;
    }
    return c;
}

void hsref_destroy(hsref_ctx *c)
{
    if (!c) return;
    free(c->ball); free(c->chi); free(c->f); free(c->fs); free(c->n); free(c->j);
    free(c->u); free(c->eb); free(c->F); free(c->phi); free(c->solid); free(c->chi_n);
    free(c->T); free(c->Q);
    free(c);
}

/* ---------------------------------------------------------------- phases */

/* Equation (8): n = sum_i f_i, n u = sum_i c_i f_i.  Solid nodes carry nothing. */
static void phase_moments(hsref_ctx *c)
{
    const int64_t N = c->N;
    const int64_t plane = (int64_t)c->p.nx * c->p.ny;
#pragma omp parallel for schedule(static) if (c->N >= PAR_MIN_NODES)
    for (int z = 0; z < c->p.nz; ++z) {
        for (int64_t id = z * plane; id < (z + 1) * plane; ++id) {
            double n = 0.0, j[3] = {0.0, 0.0, 0.0}, e = 0.0;
            if (fluid_node(c, id)) {
                for (int i = 0; i < c->q; ++i) {
                    double fi = c->f[(int64_t)i * N + id];
                    n += fi;
                    j[0] += c->cv[i][0] * fi;
                    j[1] += c->cv[i][1] * fi;
                    j[2] += c->cv[i][2] * fi;
                    e += (c->cv[i][0] * c->cv[i][0] + c->cv[i][1] * c->cv[i][1] + c->cv[i][2] * c->cv[i][2]) * fi;
                }
            }
            c->n[id] = n;
            double uu = 0.0;
            for (int a = 0; a < 3; ++a) {
                c->j[a * N + id] = j[a];
                c->u[a * N + id] = n != 0.0 ? j[a] / n : 0.0;
                uu += c->u[a * N + id] * c->u[a * N + id];
            }
            /* n T = (1/3) sum f |c - u|^2 = (sum f c^2 - n u^2) / 3 */
            if (c->p.thermal) c->T[id] = n != 0.0 ? (e / n - uu) / 3.0 : 0.0;
        }
    }
}

/* Coarse-grained packing fraction: the density averaged over the lattice nodes
 * of the ball of radius sigma/2, times pi sigma^3 / 6. */
static void phase_eta_bar(hsref_ctx *c)
{
    const int64_t plane = (int64_t)c->p.nx * c->p.ny;
    const double sig = (double)c->p.sigma;
    const double pref = M_PI * sig * sig * sig / 6.0 / (double)c->nball;
#pragma omp parallel for schedule(static) if (c->N >= PAR_MIN_NODES)
    for (int z = 0; z < c->p.nz; ++z) {
        for (int y = 0; y < c->p.ny; ++y) {
            for (int x = 0; x < c->p.nx; ++x) {
                double s = 0.0;
                for (int b = 0; b < c->nball; ++b) {
                    int64_t id = node_at(c, x + c->ball[b][0], y + c->ball[b][1], z + c->ball[b][2]);
                    if (id >= 0) s += c->n[id];
                }
                c->eb[z * plane + (int64_t)y * c->p.nx + x] = pref * s;
            }
        }
    }
}

/* Coarse-grained packing fraction at the midpoint of the pair (r, r+d): the mean
 * over the 2^h lattice nodes nearest to r + d/2.  Returns 0 when one of them lies
 * beyond the array (such pairs carry no density and are never used). */
static int eta_mid(const hsref_ctx *c, int x, int y, int z, const int d[3], double *out)
{
    int lo[3], hi[3];
    const int r[3] = {x, y, z};
    for (int a = 0; a < 3; ++a) {
        /* floor(d/2) and ceil(d/2) for either sign */
        int fl = (d[a] >= 0) ? d[a] / 2 : -((-d[a] + 1) / 2);
        lo[a] = r[a] + fl;
        hi[a] = r[a] + d[a] - fl;
    }
    double s = 0.0;
    int cnt = 0;
    for (int zz = lo[2]; zz <= hi[2]; ++zz)
        for (int yy = lo[1]; yy <= hi[1]; ++yy)
            for (int xx = lo[0]; xx <= hi[0]; ++xx) {
                int64_t id = node_at(c, xx, yy, zz);
                if (id < 0) return 0;
                s += c->eb[id];
                ++cnt;
            }
    *out = s / (double)cnt;
    return 1;
}

/* Mean-field attraction potential at every node (see the header):
 *   Phi(r) = -att_eps sum_o exp(-|o|^2 / att_range^2) n(r + o),
 * o over the cube |o_a| <= R, as a plain triple sum. */
static void phase_attraction(hsref_ctx *c)
{
    const int64_t plane = (int64_t)c->p.nx * c->p.ny;
    const int R = c->att_R;
    const double l2 = c->p.att_range * c->p.att_range;
#pragma omp parallel for schedule(static) if (c->N >= PAR_MIN_NODES)
    for (int z = 0; z < c->p.nz; ++z) {
        for (int y = 0; y < c->p.ny; ++y) {
            for (int x = 0; x < c->p.nx; ++x) {
                double s = 0.0;
                for (int oz = -R; oz <= R; ++oz)
                    for (int oy = -R; oy <= R; ++oy)
                        for (int ox = -R; ox <= R; ++ox) {
                            int64_t id = node_at(c, x + ox, y + oy, z + oz);
                            if (id < 0) continue;
                            s += exp(-(double)(ox * ox + oy * oy + oz * oz) / l2) * c->n[id];
                        }
                c->phi[z * plane + (int64_t)y * c->p.nx + x] = -c->p.att_eps * s;
            }
        }
    }
}

/* Equation (12) with the isothermal restriction, plus the external field:
 *   C1(r) = -v_T^2 sigma^2 4pi n(r) sum_q W_q s_q sum_k alpha_qk G_qk
 *           [ n(r+d) - chi(r) kappa s_q . (j(r+d) - n(r+d) u(r)) ],
 *   kappa = 2/(v_T sqrt(pi)),  G_qk = g2(eta_bar at the pair midpoint),
 *   F = C1 + n(r) g.
 * Directions are summed as (q, -q) pairs, pairs in table order. */
static void phase_force(hsref_ctx *c)
{
    const int64_t N = c->N;
    const int64_t plane = (int64_t)c->p.nx * c->p.ny;
    const double vt2 = c->cs2;
    const double kappa = 2.0 / (sqrt(vt2) * sqrt(M_PI));
    const double sig = (double)c->p.sigma;
    const double pref = -vt2 * sig * sig * 4.0 * M_PI;
    const int hs_on = (c->p.force_mode != 2);
    const int th = c->p.thermal;
#pragma omp parallel for schedule(static) if (c->N >= PAR_MIN_NODES)
    for (int z = 0; z < c->p.nz; ++z) {
        for (int y = 0; y < c->p.ny; ++y) {
            for (int x = 0; x < c->p.nx; ++x) {
                int64_t id = z * plane + (int64_t)y * c->p.nx + x;
                double Fv[3] = {0.0, 0.0, 0.0};
                double Qv = 0.0;
                if (fluid_node(c, id)) {
                    double nr = c->n[id];
                    double ur[3] = {c->u[id], c->u[N + id], c->u[2 * N + id]};
                    double S[3] = {0.0, 0.0, 0.0}, Qs = 0.0;
                    /* thermal: v_T^2 = T(r) in the prefactor, kappa and the temperature terms */
                    const double Tr = th ? c->T[id] : 0.0;
                    const double kap = th ? 2.0 / (sqrt(Tr) * sqrt(M_PI)) : kappa;
                    const double prf = th ? -Tr * sig * sig * 4.0 * M_PI : pref;
                    if (hs_on) {
                        for (int pr = 0; pr < NSHELL / 2; ++pr) {
                            double Sp[3] = {0.0, 0.0, 0.0}, Qp = 0.0;
                            for (int m = 0; m < 2; ++m) {
                                const shell_dir *e = &c->shell[2 * pr + m];
                                double acc = 0.0, accq = 0.0;
                                for (int k = 0; k < e->ncorner; ++k) {
                                    int64_t id2 = node_at(c, x + e->d[k][0], y + e->d[k][1], z + e->d[k][2]);
                                    if (!fluid_node(c, id2)) continue; /* n = j = 0 there */
                                    double etam;
                                    if (!eta_mid(c, x, y, z, e->d[k], &etam)) continue;
                                    double G = hsref_g2(c->p.g2_model, etam);
                                    double n2 = c->n[id2];
                                    double cur = 0.0;
                                    for (int a = 0; a < 3; ++a)
                                        cur += e->s[a] * (c->j[a * N + id2] - n2 * ur[a]);
                                    if (!th) {
                                        acc += e->alpha[k] * G * (n2 - chi_at(c, id, z) * kappa * cur);
                                    } else {
                                        const double dT = c->T[id2] - Tr;
                                        acc += e->alpha[k] * G *
                                               (n2 - chi_at(c, id, z) * kap * cur + n2 * dT / (2.0 * Tr));
                                        accq += e->alpha[k] * G * (-0.5 * cur + n2 * dT / (sqrt(M_PI) * sqrt(Tr)));
                                    }
                                }
                                for (int a = 0; a < 3; ++a) Sp[a] += e->W * e->s[a] * acc;
                                Qp += e->W * accq;
                            }
                            for (int a = 0; a < 3; ++a) S[a] += Sp[a];
                            Qs += Qp;
                        }
                    }
                    Qv = -prf * nr * Qs;  /* C^(2) = v_T^2 sigma^2 4 pi n sum ... */
                    double Fa[3] = {0.0, 0.0, 0.0};
                    if (c->att_R > 0) {
                        /* central differences of Phi; r +- e_a lies inside the array at a fluid node */
                        for (int a = 0; a < 3; ++a) {
                            int e[3] = {0, 0, 0};
                            e[a] = 1;
                            int64_t ip = node_at(c, x + e[0], y + e[1], z + e[2]);
                            int64_t im = node_at(c, x - e[0], y - e[1], z - e[2]);
                            Fa[a] = -nr * (c->phi[ip] - c->phi[im]) / 2.0;
                        }
                    }
                    for (int a = 0; a < 3; ++a) Fv[a] = prf * nr * S[a] + Fa[a] + nr * c->p.accel[a];
                }
                for (int a = 0; a < 3; ++a) c->F[a * N + id] = Fv[a];
                c->Q[id] = th ? Qv : 0.0;
            }
        }
    }
}

/* Third-order lattice: the local equilibrium (11) carried through h^(3),
 * w n [1 + h1.u/v_T^2 + h2:uu/(2 v_T^4) + h3:uuu/(6 v_T^6)], written out as
 * w n [1 + xi + xi^2/2 - u^2/(2 v_T^2) + xi^3/6 - xi u^2/(2 v_T^2)], xi = c.u / v_T^2. */
static double feq39(const hsref_ctx *c, int i, double n, const double u[3])
{
    const double cs2 = c->cs2;
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const double xi = (c->cv[i][0] * u[0] + c->cv[i][1] * u[1] + c->cv[i][2] * u[2]) / cs2;
    return c->w[i] * n * (1.0 + xi + 0.5 * xi * xi - uu / (2.0 * cs2) + xi * xi * xi / 6.0 - xi * uu / (2.0 * cs2));
}

/* Thermal: the Maxwellian at (n, u, T) expanded through h^(3) about T0 = v_T^2
 * of the lattice (xi = c/sqrt(T0), u~ = u/sqrt(T0), theta = T/T0):
 * w n [1 + xi.u~ + ((xi.u~)^2 - u~^2 + (theta - 1)(xi^2 - 3))/2
 *      + (xi.u~)((xi.u~)^2 - 3 u~^2 + 3 (theta - 1)(xi^2 - 5))/6]. */
static double feq39_thermal(const hsref_ctx *c, int i, double n, const double u[3], double T)
{
    const double T0 = c->cs2;
    const int *v = c->cv[i];
    const double xu = (v[0] * u[0] + v[1] * u[1] + v[2] * u[2]) / T0;          /* xi.u~ */
    const double uu = (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) / T0;          /* u~^2 */
    const double xx = (double)(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) / T0;  /* xi^2 */
    const double th1 = T / T0 - 1.0;
    return c->w[i] * n *
           (1.0 + xu + 0.5 * (xu * xu - uu + th1 * (xx - 3.0)) +
            xu * (xu * xu - 3.0 * uu + 3.0 * th1 * (xx - 5.0)) / 6.0);
}

/* Hermite tensors of velocity i: h2_ab = c_a c_b - v_T^2 d_ab and
 * h3_abc = c_a c_b c_c - v_T^2 (c_a d_bc + c_b d_ac + c_c d_ab). */
static double herm2(const hsref_ctx *c, int i, int a, int b)
{
    return c->cv[i][a] * c->cv[i][b] - (a == b ? c->cs2 : 0.0);
}

static double herm3(const hsref_ctx *c, int i, int a, int b, int g)
{
    const int *v = c->cv[i];
    return (double)(v[a] * v[b] * v[g]) -
           c->cs2 * ((b == g ? v[a] : 0) + (a == g ? v[b] : 0) + (a == b ? v[g] : 0));
}

/* Collision on the third-order lattice (readings in the header): the
 * non-equilibrium part is projected on h^(2) and h^(3), relaxed, and the
 * first-order source added; then propagation, with the longer links reversed
 * at the wall planes. */
static void phase_collide_stream39(hsref_ctx *c)
{
    const int64_t N = c->N;
    const int64_t plane = (int64_t)c->p.nx * c->p.ny;
    const double tau = c->p.tau, cs2 = c->cs2;
    const int q = c->q;
    memset(c->fs, 0, sizeof(double) * (size_t)q * (size_t)N);
#pragma omp parallel for schedule(static) if (c->N >= PAR_MIN_NODES)
    for (int z = 0; z < c->p.nz; ++z) {
        if (is_solid_z(c, z)) continue;
        for (int y = 0; y < c->p.ny; ++y) {
            for (int x = 0; x < c->p.nx; ++x) {
                int64_t id = z * plane + (int64_t)y * c->p.nx + x;
                double n = c->n[id];
                double u[3] = {c->u[id], c->u[N + id], c->u[2 * N + id]};
                double F[3] = {c->F[id], c->F[N + id], c->F[2 * N + id]};
                double feq[QMAX], a2[3][3] = {{0.0}}, a3[3][3][3] = {{{0.0}}};
                const int th = c->p.thermal;
                const double Tn = th ? c->T[id] : 0.0, Qn = th ? c->Q[id] : 0.0;
                const double Fu = F[0] * u[0] + F[1] * u[1] + F[2] * u[2];
                for (int i = 0; i < q; ++i) {
                    feq[i] = th ? feq39_thermal(c, i, n, u, Tn) : feq39(c, i, n, u);
                    double fneq = c->f[(int64_t)i * N + id] - feq[i];
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) {
                            a2[a][b] += herm2(c, i, a, b) * fneq;
                            for (int g = 0; g < 3; ++g) a3[a][b][g] += herm3(c, i, a, b, g) * fneq;
                        }
                }
                for (int i = 0; i < q; ++i) {
                    double p2 = 0.0, p3 = 0.0;
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) {
                            p2 += herm2(c, i, a, b) * a2[a][b];
                            for (int g = 0; g < 3; ++g) p3 += herm3(c, i, a, b, g) * a3[a][b][g];
                        }
                    double fneq_reg = c->w[i] * (p2 / (2.0 * cs2 * cs2) + p3 / (6.0 * cs2 * cs2 * cs2));
                    double cF = c->cv[i][0] * F[0] + c->cv[i][1] * F[1] + c->cv[i][2] * F[2];
                    double src = cF / cs2;
                    if (th) {
                        /* the force's second Hermite order and the energy source on the trace of h^(2) */
                        const int *v = c->cv[i];
                        const double cu = v[0] * u[0] + v[1] * u[1] + v[2] * u[2];
                        const double c2 = (double)(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                        src += (cF * cu - cs2 * Fu) / (cs2 * cs2) + Qn * (c2 - 3.0 * cs2) / (3.0 * cs2 * cs2);
                    }
                    double fpost = feq[i] + (1.0 - 1.0 / tau) * fneq_reg + c->w[i] * src;
                    const int *v = c->cv[i];
                    int xt = x + v[0], yt = y + v[1], zt = z + v[2], k = i;
                    if (!c->zperiodic) {
                        const int lo = c->p.wall_lo, hi = c->p.nz - c->p.wall_hi;  /* fluid layers [lo, hi) */
                        int run = 0;   /* signed lateral distance travelled in units of c_a / |c_z| */
                        if (zt < lo) {
                            run = 2 * (z - lo) + 1 + v[2];       /* 2 d - |c_z| with d = z - lo + 1/2 */
                            zt = 2 * lo - 1 - zt;
                        } else if (zt >= hi) {
                            run = 2 * (hi - 1 - z) + 1 - v[2];
                            zt = 2 * hi - 1 - zt;
                        }
                        if (zt != z + v[2]) {
                            const int az = abs(v[2]);
                            xt = x + v[0] / az * run;
                            yt = y + v[1] / az * run;
                            k = c->opp[i];
                        }
                    }
                    int64_t id2 = node_at(c, xt, yt, zt);
                    c->fs[(int64_t)k * N + id2] = fpost;
                }
            }
        }
    }
    double *t = c->f;
    c->f = c->fs;
    c->fs = t;
}

/* Equations (10) and (11): BGK relaxation toward the second-order equilibrium
 * with the first-order source 3 w_i c_i . F, then propagation to r + c_i, with
 * halfway bounce-back (the population returns reversed to r) when r + c_i is
 * solid. */
static void phase_collide_stream(hsref_ctx *c)
{
    if (c->q == 39) {
        phase_collide_stream39(c);
        return;
    }
    const int64_t N = c->N;
    const int64_t plane = (int64_t)c->p.nx * c->p.ny;
    const double tau = c->p.tau;
    memset(c->fs, 0, sizeof(double) * (size_t)NQ * (size_t)N);
#pragma omp parallel for schedule(static) if (c->N >= PAR_MIN_NODES)
    for (int z = 0; z < c->p.nz; ++z) {
        if (is_solid_z(c, z)) continue;
        for (int y = 0; y < c->p.ny; ++y) {
            for (int x = 0; x < c->p.nx; ++x) {
                int64_t id = z * plane + (int64_t)y * c->p.nx + x;
                if (!fluid_node(c, id)) continue;
                double n = c->n[id];
                double u[3] = {c->u[id], c->u[N + id], c->u[2 * N + id]};
                double F[3] = {c->F[id], c->F[N + id], c->F[2 * N + id]};
                double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
                for (int i = 0; i < NQ; ++i) {
                    double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
                    double cF = CV[i][0] * F[0] + CV[i][1] * F[1] + CV[i][2] * F[2];
                    double feq = c->w[i] * n * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
                    double fi = c->f[(int64_t)i * N + id];
                    double fpost = fi - (fi - feq) / tau + 3.0 * c->w[i] * cF;
                    int64_t id2 = node_at(c, x + CV[i][0], y + CV[i][1], z + CV[i][2]);
                    if (fluid_node(c, id2))
                        c->fs[(int64_t)i * N + id2] = fpost;
                    else
                        c->fs[(int64_t)c->opp[i] * N + id] = fpost;
                }
            }
        }
    }
    double *t = c->f;
    c->f = c->fs;
    c->fs = t;
}

/* ---------------------------------------------------------------- API */

static int check_fields(const hsref_ctx *c, const double *n, const double *u)
{
    const int64_t N = c->N;
    for (int64_t id = 0; id < N; ++id) {
        if (!fluid_node(c, id)) continue;
        if (!isfinite(n[id]) || n[id] < 0.0) return -1;
        if (u)
            for (int a = 0; a < 3; ++a)
                if (!isfinite(u[a * N + id])) return -1;
    }
    return 0;
}

static int init_fields(hsref_ctx *c, const double *n, const double *u, const double *T);

/* Initial populations: the local equilibrium (11) of the given fields. */
int hsref_init(hsref_ctx *c, const double *n, const double *u)
{
    return init_fields(c, n, u, NULL);
}

/* Thermal contexts: the equilibrium at (n, u, T); T NULL means T0 everywhere. */
int hsref_init_thermal(hsref_ctx *c, const double *n, const double *u, const double *T)
{
    if (!c || !c->p.thermal) return -1;
    return init_fields(c, n, u, T);
}

static int init_fields(hsref_ctx *c, const double *n, const double *u, const double *T)
{
    if (!c || !n) return -1;
    if (check_fields(c, n, u)) return -1;
    if (T)
        for (int64_t id = 0; id < c->N; ++id)
            if (fluid_node(c, id) && !(isfinite(T[id]) && T[id] > 0.0)) return -1;
    const int64_t N = c->N;
    memset(c->f, 0, sizeof(double) * (size_t)c->q * (size_t)N);
    for (int64_t id = 0; id < N; ++id) {
        if (!fluid_node(c, id)) continue;
        double uu[3] = {0.0, 0.0, 0.0};
        if (u)
            for (int a = 0; a < 3; ++a) uu[a] = u[a * N + id];
        if (c->q == 39) {
            for (int i = 0; i < c->q; ++i)
                c->f[(int64_t)i * N + id] = c->p.thermal ? feq39_thermal(c, i, n[id], uu, T ? T[id] : c->cs2)
                                                         : feq39(c, i, n[id], uu);
            continue;
        }
        double u2 = uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2];
        for (int i = 0; i < NQ; ++i) {
            double cu = CV[i][0] * uu[0] + CV[i][1] * uu[1] + CV[i][2] * uu[2];
            c->f[(int64_t)i * N + id] = c->w[i] * n[id] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * u2);
        }
    }
    phase_moments(c);
    return 0;
}

int hsref_step(hsref_ctx *c, int64_t nsteps)
{
    if (!c || nsteps < 0) return -1;
    for (int64_t s = 0; s < nsteps; ++s) {
        phase_moments(c);
        if (c->p.force_mode != 2) phase_eta_bar(c);
        if (c->att_R > 0) phase_attraction(c);
        phase_force(c);
        phase_collide_stream(c);
    }
    phase_moments(c);
    return 0;
}

int hsref_moments(hsref_ctx *c, double *n, double *u)
{
    if (!c) return -1;
    phase_moments(c);
    const size_t N = (size_t)c->N;
    if (n) memcpy(n, c->n, sizeof(double) * N);
    if (u) memcpy(u, c->u, sizeof(double) * 3 * N);
    return 0;
}

/* Layer profiles: n(z) is the layer mean of n, u(z) = sum j / sum n. */
int hsref_profiles(hsref_ctx *c, double *nz_out, double *uz_out)
{
    if (!c) return -1;
    phase_moments(c);
    const int64_t N = c->N, plane = (int64_t)c->p.nx * c->p.ny;
    for (int z = 0; z < c->p.nz; ++z) {
        double sn = 0.0, sj[3] = {0.0, 0.0, 0.0};
        for (int64_t id = z * plane; id < (z + 1) * plane; ++id) {
            sn += c->n[id];
            for (int a = 0; a < 3; ++a) sj[a] += c->j[a * N + id];
        }
        if (nz_out) nz_out[z] = sn / (double)plane;
        if (uz_out)
            for (int a = 0; a < 3; ++a) uz_out[a * c->p.nz + z] = sn != 0.0 ? sj[a] / sn : 0.0;
    }
    return 0;
}

/* Total force F = C1 + n g at the current state, [3][N]. */
/* One step whose interaction force is given per node instead of computed:
 * F = C1 + n g at fluid nodes, then the collision (10)-(11) and propagation as
 * in hsref_step.  C1 is [3][N]; its solid-node values are ignored.  (The
 * learned force replaces C1 this way between exact steps.) */
int hsref_step_with_force(hsref_ctx *c, const double *C1)
{
    if (!c || !C1) return -1;
    const int64_t N = c->N;
    phase_moments(c);
    for (int64_t id = 0; id < N; ++id) {
        const int fl = fluid_node(c, id);
        for (int a = 0; a < 3; ++a) c->F[a * N + id] = fl ? C1[a * N + id] + c->n[id] * c->p.accel[a] : 0.0;
    }
    phase_collide_stream(c);
    phase_moments(c);
    return 0;
}

int hsref_force(hsref_ctx *c, double *F)
{
    if (!c || !F) return -1;
    phase_moments(c);
    if (c->p.force_mode != 2) phase_eta_bar(c);
    if (c->att_R > 0) phase_attraction(c);
    phase_force(c);
    memcpy(F, c->F, sizeof(double) * 3 * (size_t)c->N);
    return 0;
}

/* Solid mask solid[N] (nonzero: solid), before hsref_init.  Rebuilds the
 * per-node wall factor by brute force over the solid nodes. */
int hsref_set_solid(hsref_ctx *c, const uint8_t *solid)
{
    if (!c || !solid || c->q != NQ) return -1;
    const int64_t N = c->N, plane = (int64_t)c->p.nx * c->p.ny;
    if (!c->solid) c->solid = malloc((size_t)N);
    if (!c->chi_n) c->chi_n = malloc(sizeof(double) * (size_t)N);
    if (!c->solid || !c->chi_n) return -1;
    for (int64_t id = 0; id < N; ++id) c->solid[id] = solid[id] ? 1 : 0;
    /* solid node centres: mask and wall layers */
    int64_t ns = 0;
    for (int64_t id = 0; id < N; ++id)
        if (!fluid_node(c, id)) ++ns;
    int (*sp)[3] = malloc(sizeof(int[3]) * (size_t)(ns ? ns : 1));
    if (!sp) return -1;
    ns = 0;
    for (int64_t id = 0; id < N; ++id)
        if (!fluid_node(c, id)) {
            sp[ns][2] = (int)(id / plane);
            sp[ns][1] = (int)((id % plane) / c->p.nx);
            sp[ns][0] = (int)(id % c->p.nx);
            ++ns;
        }
    const int sig = c->p.sigma >= 2 ? c->p.sigma : 2;
    const int dims[3] = {c->p.nx, c->p.ny, c->p.nz};
    const int per[3] = {1, 1, c->zperiodic};
#pragma omp parallel for schedule(static) if (N >= PAR_MIN_NODES)
    for (int64_t id = 0; id < N; ++id) {
        double chi = 1.0;
        if (c->p.wall_reg && ns > 0 && fluid_node(c, id)) {
            const int r[3] = {(int)(id % c->p.nx), (int)((id % plane) / c->p.nx), (int)(id / plane)};
            int64_t best = -1;
            for (int64_t k = 0; k < ns; ++k) {
                int64_t d2 = 0;
                for (int a = 0; a < 3; ++a) {
                    int d = abs(r[a] - sp[k][a]);
                    if (per[a] && dims[a] - d < d) d = dims[a] - d;   /* nearest periodic image */
                    d2 += (int64_t)d * d;
                }
                if (best < 0 || d2 < best) best = d2;
            }
            chi = 1.0 - exp(-(sqrt((double)best) - 0.5) / (double)sig);
        }
        c->chi_n[id] = chi;
    }
    free(sp);
    return 0;
}

/* Mean-field attraction potential Phi[N] at the current state (0 when the
 * attraction is off). */
int hsref_attraction_potential(hsref_ctx *c, double *phi)
{
    if (!c || !phi) return -1;
    phase_moments(c);
    if (c->att_R > 0) phase_attraction(c);
    memcpy(phi, c->phi, sizeof(double) * (size_t)c->N);
    return 0;
}

int hsref_eta_bar(hsref_ctx *c, double *eb)
{
    if (!c || !eb) return -1;
    phase_moments(c);
    phase_eta_bar(c);
    memcpy(eb, c->eb, sizeof(double) * (size_t)c->N);
    return 0;
}

int hsref_get_populations(hsref_ctx *c, double *f)
{
    if (!c || !f) return -1;
    memcpy(f, c->f, sizeof(double) * c->q * (size_t)c->N);
    return 0;
}

int hsref_set_populations(hsref_ctx *c, const double *f)
{
    if (!c || !f) return -1;
    memcpy(c->f, f, sizeof(double) * c->q * (size_t)c->N);
    for (int64_t id = 0; id < c->N; ++id)
        if (!fluid_node(c, id))
            for (int i = 0; i < c->q; ++i) c->f[(int64_t)i * c->N + id] = 0.0;
    phase_moments(c);
    return 0;
}

/* The 18-direction table for sigma: W[18], s[18][3], ncorner[18], d[18][4][3],
 * alpha[18][4] (unused corners are zero). */
int hsref_shell_table(int sigma, double *W, double *s, int *ncorner, int *d, double *alpha)
{
    if (sigma < 1) return -1;
    shell_dir sh[NSHELL];
    build_shell(sigma, sh);
    for (int q = 0; q < NSHELL; ++q) {
        if (W) W[q] = sh[q].W;
        for (int a = 0; a < 3; ++a)
            if (s) s[3 * q + a] = sh[q].s[a];
        if (ncorner) ncorner[q] = sh[q].ncorner;
        for (int k = 0; k < 4; ++k) {
            if (alpha) alpha[4 * q + k] = k < sh[q].ncorner ? sh[q].alpha[k] : 0.0;
            for (int a = 0; a < 3; ++a)
                if (d) d[12 * q + 3 * k + a] = k < sh[q].ncorner ? sh[q].d[k][a] : 0;
        }
    }
    return 0;
}

int hsref_ball_count(int sigma) { return build_ball(sigma, NULL); }

/* D3Q19 velocities [19][3] and weights [19]. */
int hsref_lattice(int *c, double *w)
{
    for (int i = 0; i < NQ; ++i) {
        if (w) w[i] = weight_of(i);
        for (int a = 0; a < 3; ++a)
            if (c) c[3 * i + a] = CV[i][a];
    }
    return 0;
}

/* Velocities [q][3] and weights [q] of the lattice with q = 19 or 39; returns
 * q, or -1 for another count. */
int hsref_lattice_q(int q, int *c, double *w)
{
    if (q != 19 && q != 39) return -1;
    for (int i = 0; i < q; ++i) {
        const int *v = q == 39 ? CV39[i] : CV[i];
        if (w) w[i] = q == 39 ? weight39_of(v) : weight_of(i);
        for (int a = 0; a < 3; ++a)
            if (c) c[3 * i + a] = v[a];
    }
    return q;
}

/* Number of velocities of the context's lattice. */
int hsref_q(const hsref_ctx *c) { return c ? c->q : -1; }

/* Temperature T[N] and energy source C^(2) Q[N] at the current state (thermal
 * contexts; Q needs the force phase, run here). */
int hsref_thermal_fields(hsref_ctx *c, double *T, double *Q)
{
    if (!c || !c->p.thermal) return -1;
    phase_moments(c);
    if (c->p.force_mode != 2) phase_eta_bar(c);
    if (c->att_R > 0) phase_attraction(c);
    phase_force(c);
    if (T) memcpy(T, c->T, sizeof(double) * (size_t)c->N);
    if (Q) memcpy(Q, c->Q, sizeof(double) * (size_t)c->N);
    return 0;
}
