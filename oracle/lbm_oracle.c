/*
 * Oracle for the D3Q19 BGK + Smagorinsky lattice-Boltzmann update.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, double-precision
 * CPU reference that the HIP library is checked against.  Only the tests,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * library never does.  It shares no code, header, table or helper with the
 * HIP path: the lattice table, the noise generator and every formula below
 * are written out here from the paper (arXiv 2607.04516, Appendix D
 * "Lattice Boltzmann method in FluidX3D") and from the boundary readings
 * listed in the design notes.
 *
 * Scheme: two lattices, pull streaming.  The state f[i][n] is the set of
 * pre-collision (post-stream) populations f_i(x, t), unshifted, double
 * precision, cell index n = x + nx*(y + ny*z), direction index slowest.
 *
 * One step t -> t+1 (App. D, BGK collision equation and streaming equation):
 *   1. every fluid cell collides:  f*_i = f_i - (f_i - feq_i)/tau_eff
 *      (+ Guo source for a uniform body force), with tau_eff from the local
 *      Smagorinsky closure (App. D, closed-form tau_eff equation);
 *      every inflow cell takes f*_i = feq_i(rho0, u_in);
 *   2. every non-solid destination pulls f_i(x, t+1) = f*_i(x - c_i) with
 *      the boundary rules of pull_resolve() below.
 * Nothing here is blocked, fused or reordered.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NQ 19

/* D3Q19 velocity set (App. D: 19 discrete velocities on the cubic lattice).
 * Order: rest, 6 faces, 12 edges; each pair (2k-1, 2k) is an opposite pair. */
static const int CV[NQ][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0},
    {0, 1, 0},  {0, -1, 0},
    {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0},
    {1, 0, 1},  {-1, 0, -1},
    {0, 1, 1},  {0, -1, -1},
    {1, -1, 0}, {-1, 1, 0},
    {1, 0, -1}, {-1, 0, 1},
    {0, 1, -1}, {0, -1, 1},
};

/* Weights: the isotropy constraints of App. D fix them as 1/3 (rest),
 * 1/18 (face neighbours) and 1/36 (edge neighbours). */
static double weight(int i)
{
    if (i == 0) return 1.0 / 3.0;
    if (i <= 6) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

static int opposite(int i)
{
    if (i == 0) return 0;
    return (i % 2 == 1) ? i + 1 : i - 1;
}

/* Direction with component a of c_i negated (specular reflection). */
static int mirror(int i, int a)
{
    int want[3] = {CV[i][0], CV[i][1], CV[i][2]};
    want[a] = -want[a];
    for (int j = 0; j < NQ; j++)
        if (CV[j][0] == want[0] && CV[j][1] == want[1] && CV[j][2] == want[2])
            return j;
    return -1;
}

/* Face kinds; faces are numbered x-, x+, y-, y+, z-, z+. */
enum { OR_PERIODIC = 0, OR_INFLOW_EQ = 1, OR_OUTFLOW_ZG = 2, OR_FREESLIP = 3, OR_WALL = 4 };

typedef struct {
    int32_t nx, ny, nz;
    int32_t face[6];
    double tau0;    /* molecular relaxation time, > 1/2 */
    double c_smag;  /* Smagorinsky constant C */
    double delta;   /* filter width Delta in lattice units */
    double rho0;    /* reference density of inflow cells */
    double force[3];/* uniform body force per unit volume (Guo scheme) */
    double omega[3];/* Earth rotation vector in lattice units (App. E), ENU frame */
    const double *inflow_field; /* optional [N][3] velocity of every inflow cell (App. F:
                                   the boundary velocity array); NULL: per-height profiles */
    double sponge_strength;     /* s_max of the sponge / buffer nudging (Sec. 2.2); 0: off */
    int32_t sponge_width;       /* W, layers next to each nudged face */
    int32_t pad_;
    const double *face_base[6]; /* optional per-cell boundary velocity of each face (the
                                   face-wise mapped boundary state, Sec. 2.3; App. F's U_b,i):
                                   [n2][n1][3] over the face's cells, n1 = ny for x faces and nx
                                   otherwise, n2 = ny for z faces and nz otherwise; NULL: the
                                   face's per-height profile */
} or_cfg;

/* Error state of the last call (0 = fine). */
static int g_err = 0;
int or_last_error(void) { return g_err; }

/* ------------------------------------------------------------------ */
/* Lattice table export, for the tests that pin it.                    */
void or_lattice(int32_t *c, double *w, int32_t *opp)
{
    for (int i = 0; i < NQ; i++) {
        for (int a = 0; a < 3; a++) c[3 * i + a] = CV[i][a];
        w[i] = weight(i);
        opp[i] = opposite(i);
    }
}

/* ------------------------------------------------------------------ */
/* Equilibrium (App. D, second-order Hermite equilibrium, cs^2 = 1/3):
 *   feq_i = w_i rho [1 + (c.u)/cs^2 + (c.u)^2/(2 cs^4) - (u.u)/(2 cs^2)]  */
void or_equilibrium(double rho, const double *u, double *feq)
{
    const double cs2 = 1.0 / 3.0;
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < NQ; i++) {
        double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
        feq[i] = weight(i) * rho *
                 (1.0 + cu / cs2 + (cu * cu) / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
    }
}

/* Total body force on a cell: the uniform force plus the Coriolis force
 * (App. E) F_c = -2 rho Omega x u0, with u0 = (sum c f)/rho the velocity
 * recovered from the populations before the force enters.  The paper
 * prints +2 Omega x v; the rotating-frame acceleration is -2 Omega x v,
 * which is the reading taken here. */
static void body_force(const or_cfg *g, double rho, const double *m, double *F)
{
    double u0[3] = {m[0] / rho, m[1] / rho, m[2] / rho};
    const double *w = g->omega;
    double wxu[3] = {w[1] * u0[2] - w[2] * u0[1], w[2] * u0[0] - w[0] * u0[2], w[0] * u0[1] - w[1] * u0[0]};
    for (int a = 0; a < 3; a++) F[a] = g->force[a] - 2.0 * rho * wxu[a];
}

/* Moments (App. D, zeroth and first moment equation):
 *   rho = sum_i f_i,  rho u = sum_i c_i f_i  (+ F/2 with a body force, Guo). */
void or_moments(const or_cfg *g, const double *f, double *rho, double *u)
{
    double r = 0.0, m[3] = {0.0, 0.0, 0.0}, F[3];
    for (int i = 0; i < NQ; i++) {
        r += f[i];
        for (int a = 0; a < 3; a++) m[a] += CV[i][a] * f[i];
    }
    *rho = r;
    body_force(g, r, m, F);
    for (int a = 0; a < 3; a++) u[a] = (m[a] + 0.5 * F[a]) / r;
}

/* Effective relaxation time (App. D, closed-form tau_eff equation):
 *   tau_eff = 1/2 [tau + sqrt(tau^2 + 2 (C Delta)^2 Q / (rho cs^4))]      */
double or_tau_eff(double tau0, double c_smag, double delta, double q, double rho)
{
    const double cs2 = 1.0 / 3.0;
    double cd = c_smag * delta;
    return 0.5 * (tau0 + sqrt(tau0 * tau0 + 2.0 * cd * cd * q / (rho * cs2 * cs2)));
}

/* Non-equilibrium momentum flux (App. D, Pi^(1) definition) and its
 * invariant Q = sqrt(2 Pi:Pi) (App. D, Q definition). */
double or_q_invariant(const double *f, const double *feq, double *pi /* [3][3] or NULL */)
{
    double p[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double s = 0.0;
            for (int i = 0; i < NQ; i++) s += CV[i][a] * CV[i][b] * (f[i] - feq[i]);
            p[a][b] = s;
        }
    double pp = 0.0;
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) pp += p[a][b] * p[a][b];
    if (pi)
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) pi[3 * a + b] = p[a][b];
    return sqrt(2.0 * pp);
}

/* Collision of one cell (App. D, BGK collision equation with tau_eff; Guo
 * forcing as cited in App. E).  Returns tau_eff. */
double or_collide(const or_cfg *g, const double *f, double *fstar, double *rho_out, double *u_out)
{
    double rho, u[3], feq[NQ], F[3], m[3];
    or_moments(g, f, &rho, u);
    for (int a = 0; a < 3; a++) {
        m[a] = 0.0;
        for (int i = 0; i < NQ; i++) m[a] += CV[i][a] * f[i];
    }
    body_force(g, rho, m, F);
    or_equilibrium(rho, u, feq);
    double q = or_q_invariant(f, feq, NULL);
    double tau = or_tau_eff(g->tau0, g->c_smag, g->delta, q, rho);
    double omega = 1.0 / tau;
    for (int i = 0; i < NQ; i++) {
        /* Guo et al. (2002) source: (1 - 1/(2 tau)) w_i [3(c_i - u) + 9 (c_i.u) c_i] . F */
        double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
        double src = 0.0;
        for (int a = 0; a < 3; a++)
            src += (3.0 * (CV[i][a] - u[a]) + 9.0 * cu * CV[i][a]) * F[a];
        src *= (1.0 - 0.5 * omega) * weight(i);
        fstar[i] = f[i] - omega * (f[i] - feq[i]) + src;
    }
    if (rho_out) *rho_out = rho;
    if (u_out)
        for (int a = 0; a < 3; a++) u_out[a] = u[a];
    return tau;
}

/* ------------------------------------------------------------------ */
/* Cell classification.  Precedence: solid > inflow cell > fluid.       */
#define IDX(g, x, y, z) ((int64_t)(x) + (int64_t)(g)->nx * ((int64_t)(y) + (int64_t)(g)->ny * (int64_t)(z)))

static int dim(const or_cfg *g, int a) { return a == 0 ? g->nx : (a == 1 ? g->ny : g->nz); }

/* Returns the lowest-numbered INFLOW_EQ face whose layer holds the cell, or -1. */
static int inflow_face(const or_cfg *g, const int *p)
{
    for (int a = 0; a < 3; a++) {
        if (g->face[2 * a] == OR_INFLOW_EQ && p[a] == 0) return 2 * a;
        if (g->face[2 * a + 1] == OR_INFLOW_EQ && p[a] == dim(g, a) - 1) return 2 * a + 1;
    }
    return -1;
}

static int is_solid(const or_cfg *g, const uint8_t *solid, const int *p)
{
    return solid[IDX(g, p[0], p[1], p[2])] != 0;
}

/* Boundary state of face `face` at the face cell with the transverse
 * coordinates of p (its coordinate along the face normal is ignored): the
 * per-cell face array when given, else the face's profile at the cell's
 * height (the top row for the z+ face). */
static const double *face_value(const or_cfg *g, const double *inflow, int face, const int *p)
{
    if (g->face_base[face]) {
        int a = face / 2;
        int64_t j = a == 0 ? p[1] + (int64_t)g->ny * p[2]
                  : a == 1 ? p[0] + (int64_t)g->nx * p[2] : p[0] + (int64_t)g->nx * p[1];
        return g->face_base[face] + 3 * j;
    }
    return inflow + ((int64_t)face * g->nz + (face == 5 ? g->nz - 1 : p[2])) * 3;
}

/* Inflow velocity of an inflow cell: the instantaneous per-cell field when
 * given, else the boundary state of its face. */
static void inflow_velocity(const or_cfg *g, const double *inflow, int face, const int *p, double *u)
{
    const double *v = g->inflow_field ? g->inflow_field + 3 * IDX(g, p[0], p[1], p[2]) : face_value(g, inflow, face, p);
    u[0] = v[0];
    u[1] = v[1];
    u[2] = v[2];
}

/* ------------------------------------------------------------------ */
/* Streaming resolution: the post-collision slot (j, s) whose value f*_j(s)
 * becomes f_i at the non-solid, non-inflow cell p after streaming, returned
 * as the flat index j*N + n(s), or -1 if the rules are violated.        */
static int64_t source_plain(const or_cfg *g, const uint8_t *solid, int i, const int *p)
{
    int64_t N = (int64_t)g->nx * g->ny * g->nz;
    int64_t n = IDX(g, p[0], p[1], p[2]);
    int s[3], j = i;
    for (int a = 0; a < 3; a++) s[a] = p[a] - CV[i][a];
    for (int a = 0; a < 3; a++) {
        if (s[a] >= 0 && s[a] < dim(g, a)) continue;
        int kind = g->face[s[a] < 0 ? 2 * a : 2 * a + 1];
        if (kind == OR_WALL) {
            /* halfway bounce-back at the face plane (App. D, bounce-back) */
            return opposite(i) * N + n;
        } else if (kind == OR_PERIODIC) {
            s[a] = (s[a] + dim(g, a)) % dim(g, a);
        } else if (kind == OR_FREESLIP) {
            /* specular reflection at the face plane */
            j = mirror(j, a);
            s[a] = p[a];
        } else {
            /* an inflow or outflow face is never crossed by a pull from here */
            g_err = 2;
            return -1;
        }
    }
    if (is_solid(g, solid, s)) return opposite(i) * N + n; /* halfway bounce-back */
    return j * N + IDX(g, s[0], s[1], s[2]);
}

static int64_t source_of(const or_cfg *g, const uint8_t *solid, int i, const int *p)
{
    int64_t N = (int64_t)g->nx * g->ny * g->nz;
    int64_t n = IDX(g, p[0], p[1], p[2]);
    /* zero-gradient outflow: a population entering through an outflow face
     * copies what the cell one layer inward (along every such face) receives */
    int q[3] = {p[0], p[1], p[2]}, moved = 0;
    for (int a = 0; a < 3; a++) {
        if (g->face[2 * a] == OR_OUTFLOW_ZG && p[a] == 0 && CV[i][a] == 1) {
            q[a] = 1;
            moved = 1;
        }
        if (g->face[2 * a + 1] == OR_OUTFLOW_ZG && p[a] == dim(g, a) - 1 && CV[i][a] == -1) {
            q[a] = dim(g, a) - 2;
            moved = 1;
        }
    }
    if (moved) {
        if (is_solid(g, solid, q)) return opposite(i) * N + n;
        return source_plain(g, solid, i, q);
    }
    return source_plain(g, solid, i, p);
}

static double pull_resolve(const or_cfg *g, const uint8_t *solid, const double *fs, int i, const int *p)
{
    int64_t k = source_of(g, solid, i, p);
    return k < 0 ? NAN : fs[k];
}

/* ------------------------------------------------------------------ */
/* splitmix64 (Steele, Lea & Flood 2014): state advanced by the golden gamma,
 * then the published 64-bit finaliser. */
uint64_t or_splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Uniform noise in [-amp, amp) for component c of cell n. */
static double noise(uint64_t seed, int64_t n, int c, double amp)
{
    uint64_t r = or_splitmix64(seed + 3ull * (uint64_t)n + (uint64_t)c);
    double unit = (double)(r >> 11) * (1.0 / 9007199254740992.0); /* 2^-53 */
    return amp * (2.0 * unit - 1.0);
}

/* ------------------------------------------------------------------ */
static int check_cfg(const or_cfg *g)
{
    if (g->nx < 3 || g->ny < 3 || g->nz < 3) return 1;
    if (!(g->tau0 > 0.5)) return 1;
    for (int a = 0; a < 3; a++) {
        int lo = g->face[2 * a], hi = g->face[2 * a + 1];
        if ((lo == OR_PERIODIC) != (hi == OR_PERIODIC)) return 1;
        if (lo < 0 || lo > 4 || hi < 0 || hi > 4) return 1;
    }
    return 0;
}

/* Initial state: feq(rho0, u0(z) + noise) in fluid cells, feq(rho0, u_in) in
 * inflow cells, feq(rho0, 0) = w_i rho0 in solid cells.
 * u0: [nz][3]; inflow: [6][nz][3]. */
int or_init(const or_cfg *g, const uint8_t *solid, const double *inflow, const double *u0,
            double amp, uint64_t seed, double *f)
{
    g_err = check_cfg(g);
    if (g_err) return g_err;
    int64_t N = (int64_t)g->nx * g->ny * g->nz;
    for (int z = 0; z < g->nz; z++)
        for (int y = 0; y < g->ny; y++)
            for (int x = 0; x < g->nx; x++) {
                int p[3] = {x, y, z};
                int64_t n = IDX(g, x, y, z);
                double u[3] = {0.0, 0.0, 0.0}, feq[NQ];
                int face = inflow_face(g, p);
                if (is_solid(g, solid, p)) {
                    /* at rest */
                } else if (face >= 0) {
                    inflow_velocity(g, inflow, face, p, u);
                } else {
                    for (int c = 0; c < 3; c++) u[c] = u0[3 * z + c] + noise(seed, n, c, amp);
                }
                or_equilibrium(g->rho0, u, feq);
                for (int i = 0; i < NQ; i++) f[i * N + n] = feq[i];
            }
    return 0;
}

/* Sponge and buffer nudging (Sec. 2.2; widths and rates are not printed, so
 * these are readings): next to every INFLOW_EQ face except the ground, a cell
 * at distance d = 1..W from the face layer has strength
 * s = s_max ((W + 1 - d) / W)^2; near several faces the largest strength
 * wins (lower-numbered face on ties).  Returns s and the face. */
static double sponge_at(const or_cfg *g, const int *p, int *face)
{
    static const int nudged[5] = {0, 1, 2, 3, 5};
    int dist[6] = {p[0], g->nx - 1 - p[0], p[1], g->ny - 1 - p[1], p[2], g->nz - 1 - p[2]};
    double best = 0.0;
    *face = -1;
    if (g->sponge_width <= 0 || !(g->sponge_strength > 0.0)) return 0.0;
    for (int k = 0; k < 5; k++) {
        int f = nudged[k];
        if (g->face[f] != OR_INFLOW_EQ) continue;
        int d = dist[f];
        if (d < 1 || d > g->sponge_width) continue;
        double r = (double)(g->sponge_width + 1 - d) / g->sponge_width;
        double sv = g->sponge_strength * r * r;
        if (sv > best) {
            best = sv;
            *face = f;
        }
    }
    return best;
}

/* Post-collision populations of one non-solid, non-inflow cell: the
 * collision, then the nudging toward the equilibrium of the face's target
 * velocity at the cell's density, f* += s (feq(rho, u_t) - feq(rho, u)),
 * with u_t the face's boundary state at the cell's projection onto the face
 * (per-height profile: its value at the cell's height, the top row for z+). */
void or_collide_cell(const or_cfg *g, const double *inflow, const double *fc, int x, int y, int z, double *fo)
{
    double rho, u[3];
    or_collide(g, fc, fo, &rho, u);
    int p[3] = {x, y, z}, face;
    double s = sponge_at(g, p, &face);
    if (s > 0.0) {
        const double *ut = face_value(g, inflow, face, p);
        double et[NQ], e[NQ];
        or_equilibrium(rho, ut, et);
        or_equilibrium(rho, u, e);
        for (int i = 0; i < NQ; i++) fo[i] += s * (et[i] - e[i]);
    }
}

/* One step.  f: state at t; fnext: state at t+1; fs: work array [19][N]. */
int or_step(const or_cfg *g, const uint8_t *solid, const double *inflow,
            const double *f, double *fnext, double *fs)
{
    g_err = check_cfg(g);
    if (g_err) return g_err;
    int64_t N = (int64_t)g->nx * g->ny * g->nz;
    /* 1. collision (z planes are independent: the OpenMP build of the
     * oracle, used only to time it on all host cores, splits them) */
#pragma omp parallel for schedule(static)
    for (int z = 0; z < g->nz; z++)
        for (int y = 0; y < g->ny; y++)
            for (int x = 0; x < g->nx; x++) {
                int p[3] = {x, y, z};
                int64_t n = IDX(g, x, y, z);
                double fc[NQ], fo[NQ];
                if (is_solid(g, solid, p)) {
                    for (int i = 0; i < NQ; i++) fs[i * N + n] = f[i * N + n];
                    continue;
                }
                int face = inflow_face(g, p);
                if (face >= 0) {
                    double u[3];
                    inflow_velocity(g, inflow, face, p, u);
                    or_equilibrium(g->rho0, u, fo);
                } else {
                    for (int i = 0; i < NQ; i++) fc[i] = f[i * N + n];
                    or_collide_cell(g, inflow, fc, x, y, z, fo);
                }
                for (int i = 0; i < NQ; i++) fs[i * N + n] = fo[i];
            }
    /* 2. streaming */
#pragma omp parallel for schedule(static)
    for (int z = 0; z < g->nz; z++)
        for (int y = 0; y < g->ny; y++)
            for (int x = 0; x < g->nx; x++) {
                int p[3] = {x, y, z};
                int64_t n = IDX(g, x, y, z);
                if (is_solid(g, solid, p)) {
                    for (int i = 0; i < NQ; i++) fnext[i * N + n] = f[i * N + n];
                    continue;
                }
                if (inflow_face(g, p) >= 0) {
                    for (int i = 0; i < NQ; i++) fnext[i * N + n] = fs[i * N + n];
                    continue;
                }
                for (int i = 0; i < NQ; i++) fnext[i * N + n] = pull_resolve(g, solid, fs, i, p);
            }
    return g_err;
}

/* n steps, ping-ponging between f and a work lattice; result left in f. */
int or_run(const or_cfg *g, const uint8_t *solid, const double *inflow, double *f, int64_t steps)
{
    int64_t N = (int64_t)g->nx * g->ny * g->nz;
    double *b = (double *)malloc(sizeof(double) * NQ * N);
    double *fs = (double *)malloc(sizeof(double) * NQ * N);
    if (!b || !fs) {
        free(b);
        free(fs);
        return 3;
    }
    int rc = 0;
    for (int64_t t = 0; t < steps && rc == 0; t++) {
        rc = or_step(g, solid, inflow, f, b, fs);
        memcpy(f, b, sizeof(double) * NQ * N);
    }
    free(b);
    free(fs);
    return rc;
}

/* Macroscopic fields of a state: rho, u ([3][N]) and nu_t = (tau_eff - tau0)/3
 * (App. D: nu_eff = cs^2 (tau_eff - 1/2) = nu_0 + nu_t).  Inflow cells report
 * (rho0, u_in, 0), solid cells (rho0, 0, 0). */
void or_macros(const or_cfg *g, const uint8_t *solid, const double *inflow, const double *f,
               double *rho, double *u, double *nu_t)
{
    int64_t N = (int64_t)g->nx * g->ny * g->nz;
    for (int z = 0; z < g->nz; z++)
        for (int y = 0; y < g->ny; y++)
            for (int x = 0; x < g->nx; x++) {
                int p[3] = {x, y, z};
                int64_t n = IDX(g, x, y, z);
                double r = g->rho0, v[3] = {0.0, 0.0, 0.0}, nt = 0.0;
                int face = inflow_face(g, p);
                if (is_solid(g, solid, p)) {
                } else if (face >= 0) {
                    inflow_velocity(g, inflow, face, p, v);
                } else {
                    double fc[NQ], fo[NQ];
                    for (int i = 0; i < NQ; i++) fc[i] = f[i * N + n];
                    double tau = or_collide(g, fc, fo, &r, v);
                    nt = (tau - g->tau0) / 3.0;
                }
                rho[n] = r;
                for (int a = 0; a < 3; a++) u[a * N + n] = v[a];
                nu_t[n] = nt;
            }
}

/* Mass sum(rho) and kinetic energy sum(rho |u|^2 / 2) over fluid cells
 * (solid and inflow cells excluded). */
void or_mass(const or_cfg *g, const uint8_t *solid, const double *f, double *mass, double *energy)
{
    int64_t N = (int64_t)g->nx * g->ny * g->nz;
    double m = 0.0, e = 0.0;
    for (int z = 0; z < g->nz; z++)
        for (int y = 0; y < g->ny; y++)
            for (int x = 0; x < g->nx; x++) {
                int p[3] = {x, y, z};
                int64_t n = IDX(g, x, y, z);
                if (is_solid(g, solid, p) || inflow_face(g, p) >= 0) continue;
                double fc[NQ], r, v[3];
                for (int i = 0; i < NQ; i++) fc[i] = f[i * N + n];
                or_moments(g, fc, &r, v);
                m += r;
                e += 0.5 * r * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            }
    *mass = m;
    *energy = e;
}

/* ------------------------------------------------------------------ */
/* Discrete adjoint (test infrastructure for the adjoint kernel).
 *
 * Forward step, written as a map of the state: f(t+1) = S(C(f(t)), u_in),
 * with C the local collision of every fluid cell and S the streaming with
 * its boundary rules, inflow cells supplying feq(rho0, u_in).  Its
 * transpose applied to lam_next = dL/df(t+1) is computed literally:
 *   1. scatter-add: every pull (x, i) <- (j, s) adds lam_next[i][x] into
 *      lam_star[j][s] (the outflow copy adds twice into one source);
 *   2. lam[.][s] = J(f_t(s))^T lam_star[.][s] with J the explicit 19x19
 *      Jacobian of the collision, for every fluid cell;
 *   3. inflow cells turn lam_star into the gradient of their profile:
 *      g[face][z] += sum_j lam_star[j] d feq_j(rho0, u)/du;
 *   4. probe cells add dL/du(x_p, t) . du/df_j = src . (c_j - u)/rho.
 * Solid and inflow cells get lam = 0.                                    */

/* J[i*19 + j] = d f*_i / d f_j of or_collide, term by term. */
void or_collide_jacobian(const or_cfg *g, const double *f, double *J)
{
    const double cs2 = 1.0 / 3.0;
    double rho, u[3], feq[NQ], pi[9], m[3] = {0.0, 0.0, 0.0}, F[3];
    or_moments(g, f, &rho, u);
    for (int a = 0; a < 3; a++)
        for (int i = 0; i < NQ; i++) m[a] += CV[i][a] * f[i];
    body_force(g, rho, m, F);
    or_equilibrium(rho, u, feq);
    double q = or_q_invariant(f, feq, pi);
    double tau = or_tau_eff(g->tau0, g->c_smag, g->delta, q, rho);
    double omega = 1.0 / tau;
    double cd = g->c_smag * g->delta;
    double K = 2.0 * cd * cd / (cs2 * cs2);
    double D = g->tau0 * g->tau0 + K * q / rho;

    /* The Coriolis part of F is -2 Omega x m with m = sum c f, so
     * d F_a / d f_j = -2 (Omega x c_j)_a, and with rho u = m + F/2:
     * d u_a / d f_j = (c_ja + dF_a/df_j / 2 - u_a) / rho */
    double dF[3][NQ], du[3][NQ];
    const double *w = g->omega;
    for (int j = 0; j < NQ; j++) {
        dF[0][j] = -2.0 * (w[1] * CV[j][2] - w[2] * CV[j][1]);
        dF[1][j] = -2.0 * (w[2] * CV[j][0] - w[0] * CV[j][2]);
        dF[2][j] = -2.0 * (w[0] * CV[j][1] - w[1] * CV[j][0]);
    }
    for (int a = 0; a < 3; a++)
        for (int j = 0; j < NQ; j++) du[a][j] = (CV[j][a] + 0.5 * dF[a][j] - u[a]) / rho;

    /* d feq_i / d f_j = feq_i / rho + sum_a (d feq_i / d u_a) (d u_a / d f_j) */
    double dfeq[NQ][NQ];
    for (int i = 0; i < NQ; i++) {
        double e = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
        double dfdu[3];
        for (int a = 0; a < 3; a++)
            dfdu[a] = weight(i) * rho * (CV[i][a] / cs2 + e * CV[i][a] / (cs2 * cs2) - u[a] / cs2);
        for (int j = 0; j < NQ; j++) {
            double v = feq[i] / rho;
            for (int a = 0; a < 3; a++) v += dfdu[a] * du[a][j];
            dfeq[i][j] = v;
        }
    }

    /* d Pi_ab / d f_j = c_ja c_jb - sum_i c_ia c_ib d feq_i / d f_j;
     * d Q / d f_j = 2 Pi:dPi / Q (taken as 0 at Q = 0) */
    double dq[NQ];
    for (int j = 0; j < NQ; j++) {
        double s = 0.0;
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                double dp = CV[j][a] * CV[j][b];
                for (int i = 0; i < NQ; i++) dp -= CV[i][a] * CV[i][b] * dfeq[i][j];
                s += pi[3 * a + b] * dp;
            }
        dq[j] = q > 0.0 ? 2.0 * s / q : 0.0;
    }

    /* tau = (tau0 + sqrt(D))/2, D = tau0^2 + K Q / rho, d rho / d f_j = 1 */
    double domega[NQ];
    for (int j = 0; j < NQ; j++) {
        double dD = K * (dq[j] / rho - q / (rho * rho));
        double dtau = 0.25 * dD / sqrt(D);
        domega[j] = -dtau / (tau * tau);
    }

    for (int i = 0; i < NQ; i++) {
        double e = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
        double B = 0.0;
        for (int a = 0; a < 3; a++) B += (3.0 * (CV[i][a] - u[a]) + 9.0 * e * CV[i][a]) * F[a];
        for (int j = 0; j < NQ; j++) {
            double dB = 0.0;
            double cdu = CV[i][0] * du[0][j] + CV[i][1] * du[1][j] + CV[i][2] * du[2][j];
            for (int a = 0; a < 3; a++)
                dB += F[a] * (-3.0 * du[a][j] + 9.0 * CV[i][a] * cdu) +
                      (3.0 * (CV[i][a] - u[a]) + 9.0 * e * CV[i][a]) * dF[a][j];
            double dS = -0.5 * domega[j] * weight(i) * B + (1.0 - 0.5 * omega) * weight(i) * dB;
            double kd = (i == j) ? 1.0 : 0.0;
            J[i * NQ + j] = kd - domega[j] * (f[i] - feq[i]) - omega * (kd - dfeq[i][j]) + dS;
        }
    }
}

int or_adjoint_step(const or_cfg *g, const uint8_t *solid, const double *inflow, const double *f_t,
                    const double *lam_next, double *lam, const int32_t *probes, int32_t np,
                    const double *probe_src, double *g_inflow, double *work)
{
    g_err = check_cfg(g);
    if (g_err) return g_err;
    if (g->sponge_width > 0 && g->sponge_strength > 0.0) return g_err = 6; /* not differentiated */
    int64_t N = (int64_t)g->nx * g->ny * g->nz;
    double *lam_star = work;
    for (int64_t k = 0; k < NQ * N; k++) lam_star[k] = 0.0;

    /* 1. transpose of the streaming: scatter-add over every pull */
    for (int z = 0; z < g->nz; z++)
        for (int y = 0; y < g->ny; y++)
            for (int x = 0; x < g->nx; x++) {
                int p[3] = {x, y, z};
                int64_t n = IDX(g, x, y, z);
                if (is_solid(g, solid, p) || inflow_face(g, p) >= 0) continue;
                for (int i = 0; i < NQ; i++) {
                    int64_t k = source_of(g, solid, i, p);
                    if (k < 0) return g_err;
                    lam_star[k] += lam_next[i * N + n];
                }
            }

    /* 2./3. transpose of the collision; inflow parameter sources */
    for (int z = 0; z < g->nz; z++)
        for (int y = 0; y < g->ny; y++)
            for (int x = 0; x < g->nx; x++) {
                int p[3] = {x, y, z};
                int64_t n = IDX(g, x, y, z);
                for (int j = 0; j < NQ; j++) lam[j * N + n] = 0.0;
                if (is_solid(g, solid, p)) continue;
                int face = inflow_face(g, p);
                if (face >= 0) {
                    double u[3];
                    inflow_velocity(g, inflow, face, p, u);
                    double *gz = g_inflow + ((int64_t)face * g->nz + z) * 3;
                    for (int j = 0; j < NQ; j++) {
                        double e = CV[j][0] * u[0] + CV[j][1] * u[1] + CV[j][2] * u[2];
                        for (int a = 0; a < 3; a++)
                            gz[a] += lam_star[j * N + n] * weight(j) * g->rho0 *
                                     (3.0 * CV[j][a] + 9.0 * e * CV[j][a] - 3.0 * u[a]);
                    }
                    continue;
                }
                double fc[NQ], J[NQ * NQ];
                for (int i = 0; i < NQ; i++) fc[i] = f_t[i * N + n];
                or_collide_jacobian(g, fc, J);
                for (int j = 0; j < NQ; j++) {
                    double s = 0.0;
                    for (int i = 0; i < NQ; i++) s += J[i * NQ + j] * lam_star[i * N + n];
                    lam[j * N + n] = s;
                }
            }

    /* 4. probe sources dL/du(x_p, t) . du/df */
    for (int k = 0; k < np && probe_src; k++) {
        int p[3] = {probes[3 * k], probes[3 * k + 1], probes[3 * k + 2]};
        if (is_solid(g, solid, p) || inflow_face(g, p) >= 0) continue;
        int64_t n = IDX(g, p[0], p[1], p[2]);
        double fc[NQ], rho, u[3];
        for (int i = 0; i < NQ; i++) fc[i] = f_t[i * N + n];
        or_moments(g, fc, &rho, u);
        const double *w = g->omega;
        for (int j = 0; j < NQ; j++) {
            /* d u / d f_j = (c_j - Omega x c_j - u) / rho (Coriolis part of F/2) */
            double oc[3] = {w[1] * CV[j][2] - w[2] * CV[j][1], w[2] * CV[j][0] - w[0] * CV[j][2],
                            w[0] * CV[j][1] - w[1] * CV[j][0]};
            for (int a = 0; a < 3; a++)
                lam[j * N + n] += probe_src[3 * k + a] * (CV[j][a] - oc[a] - u[a]) / rho;
        }
    }
    return 0;
}

/* f(x, t+1) at one non-solid cell x from a 5x5x5 window of f(t) centred on
 * x (window index [i][dz+2][dy+2][dx+2], periodic coordinates wrapped), by
 * colliding on demand the cells the pulls reach.  Used to check single
 * cells of grids too large for a full oracle step. */
int or_step_cell(const or_cfg *g, const uint8_t *solid, const double *inflow, const double *win,
                 int x, int y, int z, double *out)
{
    g_err = check_cfg(g);
    if (g_err) return g_err;
    int64_t N = (int64_t)g->nx * g->ny * g->nz;
    int p[3] = {x, y, z};
    if (is_solid(g, solid, p)) return 4;
    int face = inflow_face(g, p);
    if (face >= 0) {
        double u[3];
        inflow_velocity(g, inflow, face, p, u);
        or_equilibrium(g->rho0, u, out);
        return 0;
    }
    for (int i = 0; i < NQ; i++) {
        int64_t k = source_of(g, solid, i, p);
        if (k < 0) return g_err;
        int j = (int)(k / N);
        int64_t n = k % N;
        int s[3] = {(int)(n % g->nx), (int)((n / g->nx) % g->ny), (int)(n / ((int64_t)g->nx * g->ny))};
        int sf = inflow_face(g, s);
        double fo[NQ];
        if (sf >= 0) {
            double u[3];
            inflow_velocity(g, inflow, sf, s, u);
            or_equilibrium(g->rho0, u, fo);
        } else {
            int d[3];
            for (int a = 0; a < 3; a++) {
                int n_a = dim(g, a);
                d[a] = s[a] - p[a];
                if (d[a] > n_a / 2) d[a] -= n_a;   /* periodic wrap back to the nearest image */
                if (d[a] < -n_a / 2) d[a] += n_a;
                if (d[a] < -2 || d[a] > 2) return 5;
            }
            double fc[NQ];
            for (int m = 0; m < NQ; m++)
                fc[m] = win[(((int64_t)m * 5 + (d[2] + 2)) * 5 + (d[1] + 2)) * 5 + (d[0] + 2)];
            or_collide_cell(g, inflow, fc, s[0], s[1], s[2], fo);
        }
        out[i] = fo[j];
    }
    return 0;
}
