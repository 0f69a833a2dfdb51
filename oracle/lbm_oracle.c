/*
 * lbm_oracle.c -- plain CPU FP64 reference of the D3Q19 BGK lattice Boltzmann
 * recurrence (Feichtinger et al., "A Flexible Patch-Based Lattice Boltzmann
 * Parallelization Approach for Heterogeneous GPU-CPU Clusters", Sec. 2.1).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  It is slow and simple on purpose: one global grid, no
 * blocks, no ghost layers, a fixed z,y,x,i loop order and FP64 throughout.  It
 * shares no code, header, table or constant with the HIP library; only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg call it.
 *
 * What it computes, per time step and fluid cell x (pull scheme, two grids,
 * Sec. 2.1, last two paragraphs):
 *   1. pull   f_i(x) = g_i(x - e_i) from the previous post-collision grid g,
 *             periodic axes wrapped;
 *   2. walls  if x - e_i lies beyond a wall face or in a solid cell the link
 *             is a half-way bounce-back link (Sec. 2.1, bounce-back rule):
 *             f_i(x) = g_ibar(x) + 6 w_i rho0 (e_i . u_w), e_i being the
 *             direction that ARRIVES at x and u_w the wall velocity (this is
 *             the standard sign; the printed formula, read literally, has the
 *             opposite sign and would drive the fluid against a moving lid);
 *   3. moments  drho = sum_i f_i, j = sum_i e_i f_i, u = j/rho0 + g/2
 *             (velocity normalised by the constant rho0, Sec. 2.1; the g/2
 *             half-force shift is the Guo forcing reading, which the paper
 *             does not cover because its cavities have no body force);
 *   4. collide  BGK with the incompressible equilibrium of Eq. (2) written
 *             for shifted populations f~ = f - w_i rho0 (Sec. 2.1, shift):
 *             feq~_i = w_i [drho + rho0 (3 e.u + 4.5 (e.u)^2 - 1.5 u.u)],
 *             F_i    = w_i rho0 [3 (e_i - u).g + 9 (e_i.u)(e_i.g)],
 *             g'_i(x) = f_i - (1/tau)(f_i - feq~_i) + (1 - 1/(2 tau)) F_i.
 *   Solid cells are never updated and always hold 0; they report rho0 and 0.
 *
 * Open faces (an extension: the paper names boundary conditions computed
 * on the GPU as future work, Sec. 5.1 and the conclusion), on the two faces
 * of one axis: a VELOCITY or PRESSURE face replaces the wall or the periodic
 * image by a boundary node one cell outside, whose post-collision
 * populations follow the non-equilibrium extrapolation rule of Guo, Zheng
 * and Shi (2002):
 *     g_i(x_b) = feq~_i(drho_b, u_b) + [ g_i(x_f) - feq~_i(drho_f, u_f) ],
 * x_f the domain cell next to x_b (the same position along the two other
 * axes, wrapped on a periodic one), drho_f and u_f the moments of
 * x_f rebuilt from its post-collision populations (drho = sum g,
 * u = sum e g / rho0 - g/2: the collision keeps drho and adds rho0 g to the
 * momentum).  A velocity face prescribes u_b and takes drho_b = drho_f; a
 * pressure face prescribes drho_b = rho_b - rho0 and takes u_b = u_f.  A link
 * whose source lies beyond a wall face as well bounces back (walls take
 * precedence).  Solid cells must not lie on an open face.
 *
 * Readings of points the paper leaves open (each stated where it is used):
 *   - 19 directions i = 0..18 (the equation's index range printed as 0..19
 *     is taken as a typo; the text speaks of 19 PDFs);
 *   - direction order: rest, 6 faces (+x,-x,+y,-y,+z,-z), then the 12 edges
 *     in opposite pairs (see E below);
 *   - walls sit half a cell outside the outermost listed cells;
 *   - a bounce-back link whose source lies beyond several faces takes the
 *     velocity of the first MOVING face among them in the order
 *     -x,+x,-y,+y,-z,+z (so the lid wins on lid/side-wall edges);
 *   - "macroscopic" rho,u are those used by the most recent collision; before
 *     any step they are the initial values;
 *   - residual r_n = ||u^n - u^(n-1)||_2 / ||u^n||_2 over fluid cells.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC lbm_oracle.c -o liblbm_oracle.so
 * OpenMP only splits the z loop of the step; every cell is computed by the
 * same serial code, so the result does not depend on the thread count.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define Q 19

/* D3Q19 velocity set (Sec. 2.1: a 19-point stencil). */
static const int E[Q][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

enum { ORC_PERIODIC = 0, ORC_WALL = 1, ORC_VELOCITY = 2, ORC_PRESSURE = 3 };

typedef struct {
    int n[3];          /* nx, ny, nz */
    int wall[3];       /* per axis: 0 periodic, 1 half-way bounce-back walls */
    int kind[6];       /* per face -x,+x,-y,+y,-z,+z: ORC_* */
    double ob_u[6][3]; /* prescribed velocity of an open face */
    double ob_rho[6];  /* prescribed density of an open face */
    double uw[6][3];   /* wall velocity of faces -x,+x,-y,+y,-z,+z */
    double tau, rho0;
    double g[3];       /* body force per unit mass, lattice units */
    double w[Q];
    int opp[Q];
    size_t ncell;
    uint8_t *solid;    /* [z][y][x], 1 = solid */
    double *f, *fnew;  /* post-collision shifted populations [i][z][y][x] */
    double *rho, *u;   /* macroscopic of the last collision: rho[c], u[3][c] */
    double *uprev;     /* u of the step before (residual) */
    long steps;        /* steps since the last (re)initialisation */
} orc_lbm;

/* Lattice weight from |e_i|^2: 1/3 rest, 1/18 faces, 1/36 edges (Sec. 2.1). */
static double weight_of(int i) {
    int s = E[i][0] * E[i][0] + E[i][1] * E[i][1] + E[i][2] * E[i][2];
    if (s == 0) return 1.0 / 3.0;
    if (s == 1) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

/* ibar: the direction with e_ibar = -e_i (bounce-back rule, Sec. 2.1). */
static int opposite_of(int i) {
    for (int j = 0; j < Q; ++j)
        if (E[j][0] == -E[i][0] && E[j][1] == -E[i][1] && E[j][2] == -E[i][2]) return j;
    return -1;
}

static size_t cidx(const orc_lbm *L, int x, int y, int z) {
    return ((size_t)z * L->n[1] + y) * L->n[0] + x;
}

void orc_destroy(orc_lbm *L) {
    if (!L) return;
    free(L->solid); free(L->f); free(L->fnew); free(L->rho); free(L->u); free(L->uprev);
    free(L);
}

/* Reset every population to f~ = 0, i.e. f = feq(rho0, 0) (Sec. 2.1: the usual
 * initialisation), and the macroscopic record to rho0, 0. */
static void reset_rest(orc_lbm *L) {
    memset(L->f, 0, sizeof(double) * Q * L->ncell);
    memset(L->fnew, 0, sizeof(double) * Q * L->ncell);
    for (size_t c = 0; c < L->ncell; ++c) L->rho[c] = L->rho0;
    memset(L->u, 0, sizeof(double) * 3 * L->ncell);
    memset(L->uprev, 0, sizeof(double) * 3 * L->ncell);
    L->steps = 0;
}

/* dims[3]; wall_axis[3] (0 periodic, 1 walls on both faces of that axis);
 * wall_u[18] = faces -x,+x,-y,+y,-z,+z times (ux,uy,uz); g[3]. */
orc_lbm *orc_create(const int *dims, const int *wall_axis, const double *wall_u,
                    double tau, double rho0, const double *g) {
    if (dims[0] <= 0 || dims[1] <= 0 || dims[2] <= 0 || !(tau > 0.5)) return NULL;
    orc_lbm *L = (orc_lbm *)calloc(1, sizeof(orc_lbm));
    if (!L) return NULL;
    for (int a = 0; a < 3; ++a) {
        L->n[a] = dims[a];
        L->wall[a] = wall_axis[a] ? 1 : 0;
        L->kind[2 * a] = L->kind[2 * a + 1] = L->wall[a] ? ORC_WALL : ORC_PERIODIC;
        L->g[a] = g ? g[a] : 0.0;
    }
    for (int f = 0; f < 6; ++f)
        for (int a = 0; a < 3; ++a) L->uw[f][a] = wall_u ? wall_u[3 * f + a] : 0.0;
    L->tau = tau;
    L->rho0 = rho0;
    for (int i = 0; i < Q; ++i) {
        L->w[i] = weight_of(i);
        L->opp[i] = opposite_of(i);
    }
    L->ncell = (size_t)dims[0] * dims[1] * dims[2];
    L->solid = (uint8_t *)calloc(L->ncell, 1);
    L->f = (double *)malloc(sizeof(double) * Q * L->ncell);
    L->fnew = (double *)malloc(sizeof(double) * Q * L->ncell);
    L->rho = (double *)malloc(sizeof(double) * L->ncell);
    L->u = (double *)malloc(sizeof(double) * 3 * L->ncell);
    L->uprev = (double *)malloc(sizeof(double) * 3 * L->ncell);
    if (!L->solid || !L->f || !L->fnew || !L->rho || !L->u || !L->uprev) {
        orc_destroy(L);
        return NULL;
    }
    reset_rest(L);
    return L;
}

/* Make face `face` (0..5: -x, +x, -y, +y, -z, +z) open: kind ORC_VELOCITY
 * with velocity u[3], or ORC_PRESSURE with density rho; ORC_WALL or
 * ORC_PERIODIC restore those (a periodic axis needs both faces periodic).
 * Open faces lie on one axis only.  Returns 0, or -1 on a bad argument. */
int orc_set_face(orc_lbm *L, int face, int kind, const double *u, double rho) {
    if (face < 0 || face > 5 || kind < ORC_PERIODIC || kind > ORC_PRESSURE) return -1;
    if (kind == ORC_VELOCITY || kind == ORC_PRESSURE)
        for (int f = 0; f < 6; ++f)
            if (f / 2 != face / 2 && (L->kind[f] == ORC_VELOCITY || L->kind[f] == ORC_PRESSURE)) return -1;
    L->kind[face] = kind;
    for (int a = 0; a < 3; ++a) L->ob_u[face][a] = (kind == ORC_VELOCITY && u) ? u[a] : 0.0;
    L->ob_rho[face] = kind == ORC_PRESSURE ? rho : L->rho0;
    const int a = face / 2;
    L->wall[a] = L->kind[2 * a] != ORC_PERIODIC || L->kind[2 * a + 1] != ORC_PERIODIC;
    return 0;
}

/* The same for the x faces (side 0: -x, 1: +x). */
int orc_set_xface(orc_lbm *L, int side, int kind, const double *u, double rho) {
    if (side < 0 || side > 1) return -1;
    return orc_set_face(L, side, kind, u, rho);
}

/* Solid mask [z][y][x] (1 = solid), NULL = all fluid; resets to rest. */
void orc_set_geometry(orc_lbm *L, const uint8_t *solid) {
    for (size_t c = 0; c < L->ncell; ++c) L->solid[c] = solid ? (solid[c] != 0) : 0;
    reset_rest(L);
}

/* Equilibrium of Eq. (2), shifted by w_i rho0 (Sec. 2.1):
 * feq~_i = w_i [drho + rho0 (3 e.u + 4.5 (e.u)^2 - 1.5 u.u)]. */
static double feq_shifted(const orc_lbm *L, int i, double drho, const double u[3]) {
    double eu = E[i][0] * u[0] + E[i][1] * u[1] + E[i][2] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return L->w[i] * (drho + L->rho0 * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu));
}

/* Warm start: f~ = feq~(rho - rho0, u) per fluid cell, 0 in solid cells.
 * rho[c], u[3][c] with c = (z*ny + y)*nx + x. */
void orc_set_equilibrium(orc_lbm *L, const double *rho, const double *u) {
    for (size_t c = 0; c < L->ncell; ++c) {
        double uc[3] = {u[c], u[L->ncell + c], u[2 * L->ncell + c]};
        for (int i = 0; i < Q; ++i)
            L->f[(size_t)i * L->ncell + c] = L->solid[c] ? 0.0 : feq_shifted(L, i, rho[c] - L->rho0, uc);
        L->rho[c] = L->solid[c] ? L->rho0 : rho[c];
        for (int a = 0; a < 3; ++a) {
            L->u[(size_t)a * L->ncell + c] = L->solid[c] ? 0.0 : uc[a];
            L->uprev[(size_t)a * L->ncell + c] = L->u[(size_t)a * L->ncell + c];
        }
    }
    memcpy(L->fnew, L->f, sizeof(double) * Q * L->ncell);
    L->steps = 0;
}

/* Post-collision population i of the boundary node one cell beyond open
 * face `side`, next to the domain cell xf (non-equilibrium extrapolation,
 * see the file header). */
static double open_node(const orc_lbm *L, int side, int i, size_t xf) {
    const size_t N = L->ncell;
    double drho_f = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < Q; ++k) {
        const double v = L->f[(size_t)k * N + xf];
        drho_f += v;
        for (int a = 0; a < 3; ++a) j[a] += E[k][a] * v;
    }
    double u_f[3], u_b[3], drho_b;
    for (int a = 0; a < 3; ++a) u_f[a] = j[a] / L->rho0 - 0.5 * L->g[a];
    if (L->kind[side] == ORC_VELOCITY) {
        for (int a = 0; a < 3; ++a) u_b[a] = L->ob_u[side][a];
        drho_b = drho_f;
    } else {
        for (int a = 0; a < 3; ++a) u_b[a] = u_f[a];
        drho_b = L->ob_rho[side] - L->rho0;
    }
    return feq_shifted(L, i, drho_b, u_b) + L->f[(size_t)i * N + xf] - feq_shifted(L, i, drho_f, u_f);
}

/* One cell update; see the file header for the five parts. */
static void update_cell(orc_lbm *L, int x, int y, int z) {
    const size_t c = cidx(L, x, y, z);
    const size_t N = L->ncell;
    if (L->solid[c]) return;
    const int p[3] = {x, y, z};
    double f[Q];
    for (int i = 0; i < Q; ++i) {
        int s[3];
        int beyond[3] = {0, 0, 0}; /* -1: beyond the low face, +1: beyond the high face */
        int wall_link = 0, ofc = -1;
        for (int a = 0; a < 3; ++a) {
            s[a] = p[a] - E[i][a];
            if (s[a] < 0 || s[a] >= L->n[a]) {
                const int face = 2 * a + (s[a] < 0 ? 0 : 1);
                if (L->kind[face] == ORC_WALL) {
                    wall_link = 1;
                    beyond[a] = s[a] < 0 ? -1 : 1;
                } else if (L->kind[face] == ORC_PERIODIC) {
                    s[a] = (s[a] + L->n[a]) % L->n[a]; /* periodic image */
                } else {
                    ofc = face; /* open faces lie on one axis */
                }
            }
        }
        if (!wall_link && ofc >= 0) {
            /* boundary node beyond an open face; x_f next to it inside */
            int q[3] = {s[0], s[1], s[2]};
            q[ofc / 2] = ofc % 2 == 0 ? 0 : L->n[ofc / 2] - 1;
            f[i] = open_node(L, ofc, i, cidx(L, q[0], q[1], q[2]));
            continue;
        }
        if (!wall_link && L->solid[cidx(L, s[0], s[1], s[2])]) {
            /* obstacle link: half-way bounce-back from a resting wall */
            f[i] = L->f[(size_t)L->opp[i] * N + c];
        } else if (wall_link) {
            /* first moving face in the order -x,+x,-y,+y,-z,+z */
            const double *uw = NULL;
            for (int face = 0; face < 6 && !uw; ++face) {
                int a = face / 2, side = (face % 2) ? 1 : -1;
                const double *v = L->uw[face];
                if (beyond[a] == side && (v[0] != 0.0 || v[1] != 0.0 || v[2] != 0.0)) uw = v;
            }
            double eu = uw ? (E[i][0] * uw[0] + E[i][1] * uw[1] + E[i][2] * uw[2]) : 0.0;
            f[i] = L->f[(size_t)L->opp[i] * N + c] + 6.0 * L->w[i] * L->rho0 * eu;
        } else {
            f[i] = L->f[(size_t)i * N + cidx(L, s[0], s[1], s[2])];
        }
    }
    /* moments (Sec. 2.1): drho = sum f~, rho0 u = sum e f~ (+ half force) */
    double drho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
        drho += f[i];
        for (int a = 0; a < 3; ++a) j[a] += E[i][a] * f[i];
    }
    double u[3];
    for (int a = 0; a < 3; ++a) u[a] = j[a] / L->rho0 + 0.5 * L->g[a];
    const double omega = 1.0 / L->tau;
    for (int i = 0; i < Q; ++i) {
        double eu = E[i][0] * u[0] + E[i][1] * u[1] + E[i][2] * u[2];
        double eg = E[i][0] * L->g[0] + E[i][1] * L->g[1] + E[i][2] * L->g[2];
        double ug = u[0] * L->g[0] + u[1] * L->g[1] + u[2] * L->g[2];
        double F = L->w[i] * L->rho0 * (3.0 * (eg - ug) + 9.0 * eu * eg);
        double fe = feq_shifted(L, i, drho, u);
        L->fnew[(size_t)i * N + c] = f[i] - omega * (f[i] - fe) + (1.0 - 0.5 * omega) * F;
    }
    L->rho[c] = L->rho0 + drho;
    for (int a = 0; a < 3; ++a) L->u[(size_t)a * N + c] = u[a];
}

void orc_step(orc_lbm *L, long nsteps) {
    for (long t = 0; t < nsteps; ++t) {
        memcpy(L->uprev, L->u, sizeof(double) * 3 * L->ncell);
#pragma omp parallel for schedule(static)
        for (int z = 0; z < L->n[2]; ++z)
            for (int y = 0; y < L->n[1]; ++y)
                for (int x = 0; x < L->n[0]; ++x) update_cell(L, x, y, z);
        double *tmp = L->f;
        L->f = L->fnew;
        L->fnew = tmp;
        L->steps += 1;
    }
}

/* rho[c], u[3][c] of the most recent collision; solid cells: rho0 and 0. */
void orc_macroscopic(const orc_lbm *L, double *rho, double *u) {
    memcpy(rho, L->rho, sizeof(double) * L->ncell);
    memcpy(u, L->u, sizeof(double) * 3 * L->ncell);
}

/* Neumaier-compensated running sum in the fixed cell order. */
typedef struct { double s, c; } ksum;
static void kadd(ksum *k, double v) {
    double t = k->s + v;
    if (fabs(k->s) >= fabs(v)) k->c += (k->s - t) + v;
    else k->c += (v - t) + k->s;
    k->s = t;
}
static double kval(const ksum *k) { return k->s + k->c; }

/* Total mass M = N_f rho0 + sum drho and momentum P = sum rho0 u over fluid cells. */
void orc_sums(const orc_lbm *L, double *mass, double *mom) {
    ksum m = {0, 0}, p[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (size_t c = 0; c < L->ncell; ++c) {
        if (L->solid[c]) continue;
        kadd(&m, L->rho[c]);
        for (int a = 0; a < 3; ++a) kadd(&p[a], L->rho0 * L->u[(size_t)a * L->ncell + c]);
    }
    *mass = kval(&m);
    for (int a = 0; a < 3; ++a) mom[a] = kval(&p[a]);
}

/* r = ||u^n - u^(n-1)||_2 / ||u^n||_2 over fluid cells; -1 before the first step. */
double orc_residual(const orc_lbm *L) {
    if (L->steps < 1) return -1.0;
    ksum d = {0, 0}, n = {0, 0};
    for (size_t c = 0; c < L->ncell; ++c) {
        if (L->solid[c]) continue;
        for (int a = 0; a < 3; ++a) {
            double un = L->u[(size_t)a * L->ncell + c], up = L->uprev[(size_t)a * L->ncell + c];
            kadd(&d, (un - up) * (un - up));
            kadd(&n, un * un);
        }
    }
    return sqrt(kval(&d)) / sqrt(kval(&n));
}

/* Post-collision shifted populations, 19 x ncell in [i][z][y][x]. */
void orc_get_state(const orc_lbm *L, double *f) {
    memcpy(f, L->f, sizeof(double) * Q * L->ncell);
}

/* Restore a state taken by orc_get_state (solid entries are forced to 0) and
 * the macroscopic record that goes with it. */
void orc_set_state(orc_lbm *L, const double *f, const double *rho, const double *u) {
    for (int i = 0; i < Q; ++i)
        for (size_t c = 0; c < L->ncell; ++c)
            L->f[(size_t)i * L->ncell + c] = L->solid[c] ? 0.0 : f[(size_t)i * L->ncell + c];
    memcpy(L->fnew, L->f, sizeof(double) * Q * L->ncell);
    if (rho) memcpy(L->rho, rho, sizeof(double) * L->ncell);
    if (u) {
        memcpy(L->u, u, sizeof(double) * 3 * L->ncell);
        memcpy(L->uprev, u, sizeof(double) * 3 * L->ncell);
    }
    L->steps = 0;
}

long orc_steps(const orc_lbm *L) { return L->steps; }
int orc_q(void) { return Q; }
void orc_velocity(int i, int *e) { e[0] = E[i][0]; e[1] = E[i][1]; e[2] = E[i][2]; }
double orc_weight(int i) { return weight_of(i); }

/* Threads of the OpenMP z loop (timing of the baseline on 1 and all cores). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_max_threads(void) { return omp_get_max_threads(); }
