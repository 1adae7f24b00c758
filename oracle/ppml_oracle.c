/*
 * ppml_oracle.c -- plain, slow, FP64 CPU oracle of the operator-splitting
 * PPML update of Kulikov & Vorobyov, "Using the PPML approach for
 * constructing a low-dissipation, operator-splitting scheme for numerical
 * simulations of hydrodynamic flows" (arXiv:1607.01105).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  The GPU product path
 * never calls it and shares no code with it.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (no fast-math), so
 * every floating-point operation below is one IEEE-754 double operation in
 * the order written.  OpenMP only distributes independent lines over threads;
 * results are bit-identical to a one-thread run.
 *
 * What it follows, section by section of the paper:
 *   - state and equation of state p = (gamma-1) rho eps        : Sec. 2, eqs. (1)-(4)
 *   - operator split: Eulerian stage (no advection), then
 *     Lagrangian stage (advection only)                         : Sec. 2, text after eq. (4)
 *   - Eulerian finite-difference update of rho v, rho E, rho eps: Sec. 2.1, scheme for eqs. (23)-(25)
 *   - modified Roe averages of density and pressure             : Sec. 2.1
 *   - acoustic Riemann solution V, P on parabolas               : Sec. 2.2, eqs. (lowriemannvelocity/pressure)
 *   - CFL time step                                             : Sec. 2.1, CFL condition
 *   - Lagrangian upwind flux on parabolas                       : Sec. 2.3, eq. (fluxonlagrangestage)
 *   - density-weighted interface velocity, 9-point transverse
 *     velocity template, unsplit 3-D Lagrangian update          : Sec. 2.3, detailed algorithm
 *   - total-energy correction (dual energy)                     : Sec. 2.4
 *   - self-gravity potential (27-point Poisson equation)        : Sec. 2.5
 *   - isothermal variant (gamma = 1, p = cs^2 rho)               : Sec. 4, first paragraph
 *   - parabola construction and characteristic averages         : Appendix, steps 1-3
 *
 * Readings where the paper is silent or inconsistent (each listed in the
 * design notes): the parabola jump is taken as qR - qL (Colella-Woodward);
 * the state right of an interface is cell i+1's parabola; Roe-type
 * averages use cell-centre values; both stages are unsplit (directional
 * increments from one stage input, summed x, y, z); 3 ghost layers refreshed
 * before each stage; transverse template is (1/4,1/2,1/4) per transverse axis;
 * the energy correction runs after every Lagrangian stage with the initial
 * mean density and never changes rho E.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define NF 6
enum { F_RHO = 0, F_MX = 1, F_MY = 2, F_MZ = 3, F_ET = 4, F_E = 5 };
enum { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_REFLECT = 2, BC_INFLOW = 3 };
enum { POT_NONE = 0, POT_LOG = 1, POT_UNIFORM = 2, POT_HALO = 3 };
#define GH 3 /* ghost layers on each side of an active axis */

typedef struct {
    int ndim;
    long n[3];   /* interior cells per axis (1 for an unused axis)      */
    long g[3];   /* ghost layers per axis (GH when active, else 0)      */
    long N[3];   /* n + 2 g                                              */
    double lo[3], h[3];
    double gamma, cfl, vacuum_ratio, rho_mean0;
    int bc_lo[3], bc_hi[3];
    int potential;
    double pot[8]; /* POT_LOG: v0, rc, q, cx, cy, cz ; POT_UNIFORM: gx, gy, gz ;
                      POT_HALO: G rho0, r0, rh, cx, cy, cz */
    int first_order; /* 1: piecewise-constant states instead of parabolas */
    double inflow[6][NF]; /* conserved state of the ghost cells of inflow face
                             2*axis + side (0 low, 1 high)                 */
    double t;
    long steps;
    double *U[NF];   /* state U^n, ghosted                                 */
    double *W[NF];   /* Eulerian-stage output U^{n+1/2}, ghosted           */
    double *acc[NF]; /* per-cell sums of directional differences           */
    double last_max_z_euler, last_max_z_lagr;
    int iso;         /* 1: isothermal variant, p = cs^2 rho                 */
    double cs;       /* its sound speed                                      */
    int self_grav;   /* 1: the self-gravity potential enters the force      */
    double grav_G;   /* gravitational constant of Delta Phi = 4 pi G rho    */
    double *phi;     /* potential on the interior plus a one-cell shell     */
} og_grid;

static long ncell_ghosted(const og_grid *g) { return g->N[0] * g->N[1] * g->N[2]; }
static long gidx(const og_grid *g, long i, long j, long k) { return (k * g->N[1] + j) * g->N[0] + i; }
static long stride_of(const og_grid *g, int a) { return a == 0 ? 1 : (a == 1 ? g->N[0] : g->N[0] * g->N[1]); }

/* ------------------------------------------------------------------------ */
/* Parabola construction on one line (Appendix, steps 1-3).                 */
/* Input q[0..n); output for cells j = 2 .. n-3 (the others untouched).     */
/* The jump inside the cell is dq = qR - qL (reading of the Appendix's       */
/* Delta q; with it the parabola q(xi) = qL + xi (dq + q6 (1 - xi)) takes   */
/* the values qL and qR at the cell edges and has mean q).                  */
/* ------------------------------------------------------------------------ */
void og_reconstruct_line(const double *q, long n, double *qL, double *qR, double *q6, double *dm, double *qI)
{
    /* step 1: limited slope at cells 1 .. n-2 */
    for (long j = 1; j <= n - 2; j++) {
        double dq = 0.5 * (q[j + 1] - q[j - 1]);
        double dplus = q[j + 1] - q[j];
        double dminus = q[j] - q[j - 1];
        if (dplus * dminus > 0.0) {
            double a = fabs(dq), b = 2.0 * fabs(dplus), c = 2.0 * fabs(dminus);
            double m = a;
            if (b < m) m = b;
            if (c < m) m = c;
            dm[j] = copysign(m, dq);
        } else {
            dm[j] = 0.0;
        }
    }
    /* step 1 (cont.): fourth-order interface value q_{j+1/2}, j = 1 .. n-3 */
    for (long j = 1; j <= n - 3; j++)
        qI[j] = 0.5 * (q[j] + q[j + 1]) - (dm[j + 1] - dm[j]) / 6.0;
    /* steps 2 and 3: monotonize each parabola, then recompute dq and q6 */
    for (long j = 2; j <= n - 3; j++) {
        double c = q[j];
        double l = qI[j - 1];
        double r = qI[j];
        if ((r - c) * (c - l) <= 0.0) {
            l = c;
            r = c;
        } else {
            double d = r - l;
            double s6 = 6.0 * (c - 0.5 * (l + r));
            if (d * s6 > d * d)
                l = 3.0 * c - 2.0 * r;
            else if (d * s6 < -(d * d))
                r = 3.0 * c - 2.0 * l;
        }
        qL[j] = l;
        qR[j] = r;
        q6[j] = 6.0 * (c - 0.5 * (l + r));
    }
}

/* Piecewise-constant states (the first-order scheme of Sec. 2.1). */
static void constant_line(const double *q, long n, double *qL, double *qR, double *q6)
{
    for (long j = 2; j <= n - 3; j++) {
        qL[j] = q[j];
        qR[j] = q[j];
        q6[j] = 0.0;
    }
}

/* Average of cell i's parabola over the strip of width z*h that ends at its
 * right edge (Appendix, q_L(-lambda t)), z = lambda t / h. */
double og_avg_left(double qL, double qR, double q6, double z)
{
    double d = qR - qL;
    double w = 1.0 - (2.0 * z) / 3.0;
    return qR - (0.5 * z) * (d - q6 * w);
}

/* Average of cell i+1's parabola over the strip of width z*h that starts at
 * its left edge (Appendix, q_R(lambda t)). */
double og_avg_right(double qL, double qR, double q6, double z)
{
    double d = qR - qL;
    double w = 1.0 - (2.0 * z) / 3.0;
    return qL + (0.5 * z) * (d + q6 * w);
}

/* ------------------------------------------------------------------------ */
/* Boundary conditions: ghost layer source index along one axis.           */
/* ------------------------------------------------------------------------ */
static long ghost_src(long i, long G, long n, int bc_lo, int bc_hi, int *flip)
{
    *flip = 0;
    if (i < G) {
        if (bc_lo == BC_PERIODIC) return G + ((((i - G) % n) + n) % n);
        if (bc_lo == BC_OUTFLOW) return G;
        if (bc_lo == BC_INFLOW) return -1; /* prescribed state */
        *flip = 1;
        return 2 * G - 1 - i; /* mirror */
    }
    if (i >= G + n) {
        if (bc_hi == BC_PERIODIC) return G + ((((i - G) % n) + n) % n);
        if (bc_hi == BC_OUTFLOW) return G + n - 1;
        if (bc_hi == BC_INFLOW) return -1;
        *flip = 1;
        return 2 * (G + n) - 1 - i;
    }
    return i;
}

/* Fill the ghost layers of V, axis by axis (x, then y, then z), each pass over
 * the full extent of the other axes so that edges and corners are filled.
 * Periodic: wrap; outflow: copy the nearest interior cell; reflect: mirror
 * and negate the momentum normal to the wall; inflow: the prescribed state
 * (the same in both stages). */
static void fill_ghosts(og_grid *g, double **V)
{
    for (int a = 0; a < 3; a++) {
        if (g->g[a] == 0) continue;
        long G = g->g[a], n = g->n[a];
        long s = stride_of(g, a);
        long n_other1 = (a == 0) ? g->N[1] : g->N[0];
        long n_other2 = (a == 2) ? g->N[1] : g->N[2];
        for (long o2 = 0; o2 < n_other2; o2++)
            for (long o1 = 0; o1 < n_other1; o1++) {
                long base;
                if (a == 0) base = gidx(g, 0, o1, o2);
                else if (a == 1) base = gidx(g, o1, 0, o2);
                else base = gidx(g, o1, o2, 0);
                for (long i = 0; i < g->N[a]; i++) {
                    if (i >= G && i < G + n) continue;
                    int flip;
                    long src = ghost_src(i, G, n, g->bc_lo[a], g->bc_hi[a], &flip);
                    if (src < 0) {
                        const double *st = g->inflow[2 * a + (i >= G + n ? 1 : 0)];
                        for (int f = 0; f < NF; f++) V[f][base + i * s] = st[f];
                        continue;
                    }
                    for (int f = 0; f < NF; f++) V[f][base + i * s] = V[f][base + src * s];
                    if (flip) V[F_MX + a][base + i * s] = -V[F_MX + a][base + i * s];
                }
            }
    }
}

/* ------------------------------------------------------------------------ */
/* Creation and state setting.                                              */
/* ------------------------------------------------------------------------ */
og_grid *og_create(int ndim, const long *n, const double *lo, const double *hi, double gamma, double cfl,
                   const int *bc_lo, const int *bc_hi, double vacuum_ratio, int potential, const double *pot,
                   int first_order)
{
    if (ndim < 1 || ndim > 3) return NULL;
    og_grid *g = (og_grid *)calloc(1, sizeof(og_grid));
    g->ndim = ndim;
    for (int a = 0; a < 3; a++) {
        g->n[a] = (a < ndim) ? n[a] : 1;
        g->g[a] = (a < ndim) ? GH : 0;
        g->N[a] = g->n[a] + 2 * g->g[a];
        g->lo[a] = lo[a];
        g->h[a] = (hi[a] - lo[a]) / (double)g->n[a];
        g->bc_lo[a] = bc_lo[a];
        g->bc_hi[a] = bc_hi[a];
    }
    g->gamma = gamma;
    g->cfl = cfl;
    g->vacuum_ratio = vacuum_ratio;
    g->potential = potential;
    for (int i = 0; i < 8; i++) g->pot[i] = pot ? pot[i] : 0.0;
    g->first_order = first_order;
    long nc = ncell_ghosted(g);
    for (int f = 0; f < NF; f++) {
        g->U[f] = (double *)calloc((size_t)nc, sizeof(double));
        g->W[f] = (double *)calloc((size_t)nc, sizeof(double));
        g->acc[f] = (double *)calloc((size_t)nc, sizeof(double));
    }
    return g;
}

void og_destroy(og_grid *g)
{
    if (!g) return;
    for (int f = 0; f < NF; f++) {
        free(g->U[f]);
        free(g->W[f]);
        free(g->acc[f]);
    }
    free(g->phi);
    free(g);
}

static void compute_rho_mean0(og_grid *g)
{
    double s = 0.0;
    for (long k = 0; k < g->n[2]; k++)
        for (long j = 0; j < g->n[1]; j++)
            for (long i = 0; i < g->n[0]; i++) s += g->U[F_RHO][gidx(g, i + g->g[0], j + g->g[1], k + g->g[2])];
    g->rho_mean0 = s / (double)(g->n[0] * g->n[1] * g->n[2]);
}

/* Primitive (rho, v, p) at cell centres -> conserved densities, using
 * p = (gamma-1) rho eps and rho E = rho eps + rho |v|^2 / 2 (Sec. 2).
 * Arrays are interior-only, C order [z][y][x]; vy, vz may be NULL. */
void og_set_primitive(og_grid *g, const double *rho, const double *vx, const double *vy, const double *vz,
                      const double *p)
{
    long c = 0;
    for (long k = 0; k < g->n[2]; k++)
        for (long j = 0; j < g->n[1]; j++)
            for (long i = 0; i < g->n[0]; i++, c++) {
                long q = gidx(g, i + g->g[0], j + g->g[1], k + g->g[2]);
                double r = rho[c];
                /* velocity components of unused axes are not part of the state */
                double ux = vx ? vx[c] : 0.0;
                double uy = (vy && g->ndim >= 2) ? vy[c] : 0.0;
                double uz = (vz && g->ndim >= 3) ? vz[c] : 0.0;
                double e = p[c] / (g->gamma - 1.0);
                double ke = 0.5 * r * (ux * ux + uy * uy + uz * uz);
                g->U[F_RHO][q] = r;
                g->U[F_MX][q] = r * ux;
                g->U[F_MY][q] = r * uy;
                g->U[F_MZ][q] = r * uz;
                g->U[F_ET][q] = e + ke;
                g->U[F_E][q] = e;
            }
    compute_rho_mean0(g);
    g->t = 0.0;
    g->steps = 0;
}

/* State of the ghost cells of an inflow face (face = 2*axis + side, side 0
 * low, 1 high) from primitives, with the conversion of og_set_primitive. */
void og_set_inflow(og_grid *g, int face, double rho, double vx, double vy, double vz, double p)
{
    if (face < 0 || face >= 6) return;
    double ux = vx;
    double uy = g->ndim >= 2 ? vy : 0.0;
    double uz = g->ndim >= 3 ? vz : 0.0;
    double e = p / (g->gamma - 1.0);
    double ke = 0.5 * rho * (ux * ux + uy * uy + uz * uz);
    double *st = g->inflow[face];
    st[F_RHO] = rho;
    st[F_MX] = rho * ux;
    st[F_MY] = rho * uy;
    st[F_MZ] = rho * uz;
    st[F_ET] = e + ke;
    st[F_E] = e;
}

/* Conserved fields directly (checkpoint restore); f[6] interior arrays. */
void og_set_conserved(og_grid *g, const double *const *f, double rho_mean0, double t)
{
    long c = 0;
    for (long k = 0; k < g->n[2]; k++)
        for (long j = 0; j < g->n[1]; j++)
            for (long i = 0; i < g->n[0]; i++, c++) {
                long q = gidx(g, i + g->g[0], j + g->g[1], k + g->g[2]);
                for (int m = 0; m < NF; m++) g->U[m][q] = f[m] ? f[m][c] : 0.0;
            }
    if (rho_mean0 > 0.0) g->rho_mean0 = rho_mean0;
    else compute_rho_mean0(g);
    g->t = t;
}

void og_get(const og_grid *g, int field, double *out)
{
    long c = 0;
    for (long k = 0; k < g->n[2]; k++)
        for (long j = 0; j < g->n[1]; j++)
            for (long i = 0; i < g->n[0]; i++, c++) out[c] = g->U[field][gidx(g, i + g->g[0], j + g->g[1], k + g->g[2])];
}

/* Plain sequential FP64 sums of each conserved density over interior cells. */
void og_totals(const og_grid *g, double *out)
{
    for (int f = 0; f < NF; f++) {
        double s = 0.0;
        for (long k = 0; k < g->n[2]; k++)
            for (long j = 0; j < g->n[1]; j++)
                for (long i = 0; i < g->n[0]; i++) s += g->U[f][gidx(g, i + g->g[0], j + g->g[1], k + g->g[2])];
        out[f] = s;
    }
}

double og_time(const og_grid *g) { return g->t; }
double og_rho_mean0(const og_grid *g) { return g->rho_mean0; }
double og_last_max_z_euler(const og_grid *g) { return g->last_max_z_euler; }
double og_last_max_z_lagr(const og_grid *g) { return g->last_max_z_lagr; }

/* ------------------------------------------------------------------------ */
/* CFL time step (Sec. 2.1): tau (|v|_max + c_max) / h = CFL, with the two   */
/* maxima taken separately over interior cells of U^n, |v| the vector norm, */
/* c = sqrt(gamma p / rho) and h the smallest cell size of the active axes. */
/* ------------------------------------------------------------------------ */
void og_max_speeds(const og_grid *g, double *vmax, double *cmax)
{
    double vm = 0.0, cm = 0.0;
    for (long k = 0; k < g->n[2]; k++)
        for (long j = 0; j < g->n[1]; j++)
            for (long i = 0; i < g->n[0]; i++) {
                long q = gidx(g, i + g->g[0], j + g->g[1], k + g->g[2]);
                double r = g->U[F_RHO][q];
                double ux = g->U[F_MX][q] / r, uy = g->U[F_MY][q] / r, uz = g->U[F_MZ][q] / r;
                double v = sqrt(ux * ux + uy * uy + uz * uz);
                double p = g->iso ? (g->cs * g->cs) * r : (g->gamma - 1.0) * g->U[F_E][q];
                double c = sqrt((g->iso ? 1.0 : g->gamma) * p / r);
                if (v > vm) vm = v;
                if (c > cm) cm = c;
            }
    *vmax = vm;
    *cmax = cm;
}

double og_dt(const og_grid *g)
{
    double vm, cm;
    og_max_speeds(g, &vm, &cm);
    double h = g->h[0];
    for (int a = 1; a < g->ndim; a++)
        if (g->h[a] < h) h = g->h[a];
    return g->cfl * h / (vm + cm);
}

/* Gradient of the fixed external potential at a cell centre (eqs. (2)-(3)
 * force terms).  POT_LOG: Phi = v0^2/2 ln(rc^2 + X^2 + Y^2 + Z^2/q^2);
 * POT_UNIFORM: Phi = g . x; POT_HALO: the dark-matter halo of Sec. 4,
 * rho_DM = rho0 / (1 + (r/r0)^2) out to the halo radius rh, whose field is
 * G M(r) / r^2 towards the centre with the enclosed mass
 * M(r) = 4 pi rho0 r0^3 (u - atan u), u = min(r, rh) / r0. */
static void potential_grad(const og_grid *g, long i, long j, long k, double *gr)
{
    double x = g->lo[0] + ((double)i + 0.5) * g->h[0];
    double y = g->lo[1] + ((double)j + 0.5) * g->h[1];
    double z = g->lo[2] + ((double)k + 0.5) * g->h[2];
    if (g->potential == POT_LOG) {
        double v0 = g->pot[0], rc = g->pot[1], q = g->pot[2];
        double X = x - g->pot[3], Y = y - g->pot[4], Z = z - g->pot[5];
        double q2 = q * q;
        double den = rc * rc + X * X + Y * Y + Z * Z / q2;
        double a = v0 * v0 / den;
        gr[0] = a * X;
        gr[1] = a * Y;
        gr[2] = a * (Z / q2);
    } else if (g->potential == POT_UNIFORM) {
        gr[0] = g->pot[0];
        gr[1] = g->pot[1];
        gr[2] = g->pot[2];
    } else if (g->potential == POT_HALO) {
        double X = x - g->pot[3], Y = y - g->pot[4], Z = z - g->pot[5];
        double r = sqrt(X * X + Y * Y + Z * Z);
        if (r > 0.0) {
            double r0 = g->pot[1];
            double u = (r < g->pot[2] ? r : g->pot[2]) / r0;
            double m = 4.0 * M_PI * g->pot[0] * (r0 * r0 * r0) * (u - atan(u));
            double a = m / (r * r * r);
            gr[0] = a * X;
            gr[1] = a * Y;
            gr[2] = a * Z;
        } else {
            gr[0] = gr[1] = gr[2] = 0.0;
        }
    } else {
        gr[0] = gr[1] = gr[2] = 0.0;
    }
}

/* ------------------------------------------------------------------------ */
/* Self-gravity (Sec. 2.5, the Poisson solver).                             */
/* The potential solves the 27-point finite-difference form of             */
/* Delta Phi = 4 pi G rho (weights -38/9 at the centre, 4/9 on the 6 face   */
/* neighbours, 1/9 on the 12 edge neighbours, 1/36 on the 8 corners;       */
/* right-hand side 4 pi G h^2 rho) on the interior cells.  Stage 1: the    */
/* cells of the one-cell shell around the box take the two-term multipole  */
/* expansion of the mass about the coordinate origin, and every shell      */
/* value the stencil of an interior cell touches moves to the right-hand   */
/* side.  Stages 2-3: the Dirichlet problem is diagonal in the sine basis  */
/* sin(pi j k / (N+1)) of each axis (the Fourier basis of the odd          */
/* extension, period 2(N+1)); the amplitudes are divided by the stencil's  */
/* eigenvalue and transformed back.  Cells must be cubes; 3-D only.        */
/* Readings: the multipole is taken about the coordinate origin; its       */
/* quadrupole term carries the factor 1/2 of MacCullagh's formula; the     */
/* eigenvalue is -6 (1 - prod_a (1 - (2/3) sin^2(pi j_a / (2 (N_a+1)))))   */
/* (negative: the potential of a positive mass is negative); the force     */
/* uses the central difference of Phi across each cell.                    */
/* ------------------------------------------------------------------------ */
static long pidx(const og_grid *g, long i, long j, long k)
{
    return ((k + 1) * (g->n[1] + 2) + (j + 1)) * (g->n[0] + 2) + (i + 1);
}

/* Isothermal variant (Sec. 4 adopts the isothermal approximation, gamma = 1):
 * the pressure is cs^2 rho and the sound speed cs, in the Riemann problem and
 * the CFL step.  The isothermal model has no energy equation; rho E and
 * rho eps are carried along by the same updates (with gamma = 1 the eps
 * equation loses its work term) but feed nothing back, and the vacuum branch
 * of Sec. 2.4, which acts on them, is off.  0 or -1. */
int og_set_isothermal(og_grid *g, double cs)
{
    if (!(cs > 0.0)) return -1;
    g->iso = 1;
    g->cs = cs;
    g->vacuum_ratio = 0.0;
    return 0;
}

/* Enable self-gravity with constant G (3-D, cubic cells).  0 or -1. */
int og_set_self_gravity(og_grid *g, double G)
{
    if (g->ndim != 3) return -1;
    double h = g->h[0];
    if (fabs(g->h[1] - h) > 1e-12 * h || fabs(g->h[2] - h) > 1e-12 * h) return -1;
    /* the expansion about the origin is undefined at the origin itself */
    int on_grid = 1, on_shell = 0;
    for (int a = 0; a < 3; a++) {
        double u = (0.0 - g->lo[a]) / h - 0.5, ur = nearbyint(u);
        if (fabs(u - ur) > 1e-9 || ur < -1.0 || ur > (double)g->n[a]) on_grid = 0;
        if (ur == -1.0 || ur == (double)g->n[a]) on_shell = 1;
    }
    if (on_grid && on_shell) return -1;
    if (!g->phi) g->phi = (double *)calloc((size_t)((g->n[0] + 2) * (g->n[1] + 2) * (g->n[2] + 2)), sizeof(double));
    g->self_grav = 1;
    g->grav_G = G;
    return 0;
}

/* Mass and second moments of the cell masses m = rho h^3 (cell centres,
 * coordinate origin): mom = {M, Ix, Iy, Iz, Ixy, Ixz, Iyz} with
 * Ix = sum (y^2 + z^2) m, Iy = sum (x^2 + z^2) m, Iz = sum (x^2 + y^2) m,
 * Ixy = sum x y m, Ixz = sum x z m, Iyz = sum y z m (stage 1). */
void og_multipole_moments(const og_grid *g, double *mom)
{
    double vol = g->h[0] * g->h[1] * g->h[2];
    for (int q = 0; q < 7; q++) mom[q] = 0.0;
    for (long k = 0; k < g->n[2]; k++)
        for (long j = 0; j < g->n[1]; j++)
            for (long i = 0; i < g->n[0]; i++) {
                double x = g->lo[0] + ((double)i + 0.5) * g->h[0];
                double y = g->lo[1] + ((double)j + 0.5) * g->h[1];
                double z = g->lo[2] + ((double)k + 0.5) * g->h[2];
                double m = g->U[F_RHO][gidx(g, i + g->g[0], j + g->g[1], k + g->g[2])] * vol;
                mom[0] += m;
                mom[1] += (y * y + z * z) * m;
                mom[2] += (x * x + z * z) * m;
                mom[3] += (x * x + y * y) * m;
                mom[4] += x * y * m;
                mom[5] += x * z * m;
                mom[6] += y * z * m;
            }
}

/* Two-term multipole potential at (x, y, z) (stage 1):
 * -G M / r - G (Ix + Iy + Iz - 3 I0) / (2 r^3), where I0 is the moment of
 * inertia about the line from the origin through the point. */
double og_multipole_value(const double *mom, double G, double x, double y, double z)
{
    double r2 = x * x + y * y + z * z;
    double r = sqrt(r2);
    double I0 = ((x * x * mom[1] + y * y * mom[2] + z * z * mom[3]) -
                 2.0 * (x * y * mom[4] + x * z * mom[5] + y * z * mom[6])) / r2;
    return -G * mom[0] / r - G * (mom[1] + mom[2] + mom[3] - 3.0 * I0) / (2.0 * r2 * r);
}

/* Sine transform of one line of n values: y_j = sum_k x_k sin(pi j k / (n+1)),
 * j, k = 1..n (x[k-1], y[j-1]); the same sum transforms back up to the
 * factor 2 / (n+1). */
void og_sine_transform(const double *x, long n, double *y)
{
    for (long j = 1; j <= n; j++) {
        double s = 0.0;
        for (long k = 1; k <= n; k++) s += x[k - 1] * sin(M_PI * (double)(j * k) / (double)(n + 1));
        y[j - 1] = s;
    }
}

/* Sine transform of every line of axis a of the interior array A (C order
 * [k][j][i], extents n[0..2]) into B. */
static void transform_axis(const og_grid *g, int a, const double *A, double *B)
{
    long n0 = g->n[0], n1 = g->n[1], n2 = g->n[2];
    long n = g->n[a];
    long s = a == 0 ? 1 : (a == 1 ? n0 : n0 * n1);
    long nl = n0 * n1 * n2 / n;
    /* sine table of this axis (the definition above, tabulated) */
    double *S = (double *)malloc((size_t)(n * n) * sizeof(double));
    for (long j = 1; j <= n; j++)
        for (long k = 1; k <= n; k++) S[(j - 1) * n + (k - 1)] = sin(M_PI * (double)(j * k) / (double)(n + 1));
#pragma omp parallel for schedule(static)
    for (long l = 0; l < nl; l++) {
        long base;
        if (a == 0) base = l * n0;
        else if (a == 1) base = (l / n0) * n0 * n1 + (l % n0);
        else base = l;
        for (long j = 0; j < n; j++) {
            double acc = 0.0;
            for (long k = 0; k < n; k++) acc += A[base + k * s] * S[j * n + k];
            B[base + j * s] = acc;
        }
    }
    free(S);
}

static double stencil_weight(int nd) { return nd == 1 ? 4.0 / 9.0 : (nd == 2 ? 1.0 / 9.0 : 1.0 / 36.0); }

/* Potential of the current density on the interior and the shell. */
static void poisson(og_grid *g)
{
    long n0 = g->n[0], n1 = g->n[1], n2 = g->n[2];
    double h = g->h[0], G = g->grav_G;
    double mom[7];
    og_multipole_moments(g, mom);
    /* stage 1: shell values */
    for (long k = -1; k <= n2; k++)
        for (long j = -1; j <= n1; j++)
            for (long i = -1; i <= n0; i++) {
                if (i >= 0 && i < n0 && j >= 0 && j < n1 && k >= 0 && k < n2) continue;
                double x = g->lo[0] + ((double)i + 0.5) * h;
                double y = g->lo[1] + ((double)j + 0.5) * h;
                double z = g->lo[2] + ((double)k + 0.5) * h;
                g->phi[pidx(g, i, j, k)] = og_multipole_value(mom, G, x, y, z);
            }
    /* right-hand side: 4 pi G h^2 rho minus the stencil's shell terms */
    long nc = n0 * n1 * n2;
    double *A = (double *)malloc((size_t)nc * sizeof(double));
    double *B = (double *)malloc((size_t)nc * sizeof(double));
    for (long k = 0; k < n2; k++)
        for (long j = 0; j < n1; j++)
            for (long i = 0; i < n0; i++) {
                double b = 4.0 * M_PI * G * h * h * g->U[F_RHO][gidx(g, i + g->g[0], j + g->g[1], k + g->g[2])];
                for (int dz = -1; dz <= 1; dz++)
                    for (int dy = -1; dy <= 1; dy++)
                        for (int dx = -1; dx <= 1; dx++) {
                            long ii = i + dx, jj = j + dy, kk = k + dz;
                            if (ii >= 0 && ii < n0 && jj >= 0 && jj < n1 && kk >= 0 && kk < n2) continue;
                            int nd = abs(dx) + abs(dy) + abs(dz);
                            b -= stencil_weight(nd) * g->phi[pidx(g, ii, jj, kk)];
                        }
                A[(k * n1 + j) * n0 + i] = b;
            }
    /* stage 2: forward transform */
    transform_axis(g, 0, A, B);
    transform_axis(g, 1, B, A);
    transform_axis(g, 2, A, B);
    /* stage 3: divide by the eigenvalue (and the inverse transform's factors) */
    double norm = (2.0 / (double)(n0 + 1)) * (2.0 / (double)(n1 + 1)) * (2.0 / (double)(n2 + 1));
    for (long k = 0; k < n2; k++)
        for (long j = 0; j < n1; j++)
            for (long i = 0; i < n0; i++) {
                double sx = sin(M_PI * (double)(i + 1) / (2.0 * (double)(n0 + 1)));
                double sy = sin(M_PI * (double)(j + 1) / (2.0 * (double)(n1 + 1)));
                double sz = sin(M_PI * (double)(k + 1) / (2.0 * (double)(n2 + 1)));
                double prod = (1.0 - 2.0 * sx * sx / 3.0) * (1.0 - 2.0 * sy * sy / 3.0) * (1.0 - 2.0 * sz * sz / 3.0);
                double lam = -6.0 * (1.0 - prod);
                B[(k * n1 + j) * n0 + i] = B[(k * n1 + j) * n0 + i] / lam * norm;
            }
    /* back to physical space */
    transform_axis(g, 0, B, A);
    transform_axis(g, 1, A, B);
    transform_axis(g, 2, B, A);
    for (long k = 0; k < n2; k++)
        for (long j = 0; j < n1; j++)
            for (long i = 0; i < n0; i++) g->phi[pidx(g, i, j, k)] = A[(k * n1 + j) * n0 + i];
    free(A);
    free(B);
}

/* Solve for the potential of the current state and copy it out with its
 * shell: (n0+2)(n1+2)(n2+2) values, C order, shell included.  -1 if
 * self-gravity is off. */
int og_potential(og_grid *g, double *out)
{
    if (!g->self_grav) return -1;
    poisson(g);
    long np = (g->n[0] + 2) * (g->n[1] + 2) * (g->n[2] + 2);
    memcpy(out, g->phi, (size_t)np * sizeof(double));
    return 0;
}

/* Gradient of the self-gravity potential at interior cell (i, j, k): central
 * differences across the cell. */
static void self_gravity_grad(const og_grid *g, long i, long j, long k, double *gr)
{
    double h2 = 2.0 * g->h[0];
    gr[0] = (g->phi[pidx(g, i + 1, j, k)] - g->phi[pidx(g, i - 1, j, k)]) / h2;
    gr[1] = (g->phi[pidx(g, i, j + 1, k)] - g->phi[pidx(g, i, j - 1, k)]) / h2;
    gr[2] = (g->phi[pidx(g, i, j, k + 1)] - g->phi[pidx(g, i, j, k - 1)]) / h2;
}

/* ------------------------------------------------------------------------ */
/* Line buffers (one set per thread).                                       */
/* ------------------------------------------------------------------------ */
typedef struct {
    double *q[NF + 4];
    double *qL[NF + 2], *qR[NF + 2], *q6[NF + 2];
    double *dm, *qI;
    double *A, *B, *C, *D; /* interface quantities */
    double *F[NF];
} linebuf;

static void lb_alloc(linebuf *b, long n)
{
    for (int i = 0; i < NF + 4; i++) b->q[i] = (double *)calloc((size_t)n, sizeof(double));
    for (int i = 0; i < NF + 2; i++) {
        b->qL[i] = (double *)calloc((size_t)n, sizeof(double));
        b->qR[i] = (double *)calloc((size_t)n, sizeof(double));
        b->q6[i] = (double *)calloc((size_t)n, sizeof(double));
    }
    b->dm = (double *)calloc((size_t)n, sizeof(double));
    b->qI = (double *)calloc((size_t)n, sizeof(double));
    b->A = (double *)calloc((size_t)n, sizeof(double));
    b->B = (double *)calloc((size_t)n, sizeof(double));
    b->C = (double *)calloc((size_t)n, sizeof(double));
    b->D = (double *)calloc((size_t)n, sizeof(double));
    for (int i = 0; i < NF; i++) b->F[i] = (double *)calloc((size_t)n, sizeof(double));
}

static void lb_free(linebuf *b)
{
    for (int i = 0; i < NF + 4; i++) free(b->q[i]);
    for (int i = 0; i < NF + 2; i++) {
        free(b->qL[i]);
        free(b->qR[i]);
        free(b->q6[i]);
    }
    free(b->dm);
    free(b->qI);
    free(b->A);
    free(b->B);
    free(b->C);
    free(b->D);
    for (int i = 0; i < NF; i++) free(b->F[i]);
}

static void recon(const og_grid *g, linebuf *b, int slot, long n)
{
    if (g->first_order) constant_line(b->q[slot], n, b->qL[slot], b->qR[slot], b->q6[slot]);
    else og_reconstruct_line(b->q[slot], n, b->qL[slot], b->qR[slot], b->q6[slot], b->dm, b->qI);
}

/* Number of lines along axis a and the base index of line number `l`. */
static long nlines(const og_grid *g, int a)
{
    if (a == 0) return g->n[1] * g->n[2];
    if (a == 1) return g->n[0] * g->n[2];
    return g->n[0] * g->n[1];
}

static long line_base(const og_grid *g, int a, long l, long *ci, long *cj, long *ck)
{
    long i = 0, j = 0, k = 0;
    if (a == 0) {
        j = l % g->n[1];
        k = l / g->n[1];
    } else if (a == 1) {
        i = l % g->n[0];
        k = l / g->n[0];
    } else {
        i = l % g->n[0];
        j = l / g->n[0];
    }
    /* ghosted coordinates of the line's transverse position, line index 0 */
    long gi = (a == 0) ? 0 : i + g->g[0];
    long gj = (a == 1) ? 0 : j + g->g[1];
    long gk = (a == 2) ? 0 : k + g->g[2];
    *ci = gi;
    *cj = gj;
    *ck = gk;
    return gidx(g, gi, gj, gk);
}

/* ------------------------------------------------------------------------ */
/* Eulerian stage (Sec. 2.1, 2.2): U -> W.                                   */
/* For each active axis d and every line along d: reconstruct v_d and p,     */
/* solve the acoustic Riemann problem on parabolas at every interface, and   */
/* accumulate the directional differences.  Then update m, rho E, rho eps    */
/* from the same stage input (unsplit), add the external force, rho fixed.   */
/* ------------------------------------------------------------------------ */
static void eulerian_stage(og_grid *g, double tau)
{
    /* isothermal variant: sound speeds and Riemann averages with gamma = 1,
     * so the work term of the eps equation, (gamma - 1) rho eps div v, is 0 */
    const double gam = g->iso ? 1.0 : g->gamma;
    long nc = ncell_ghosted(g);
    double **U = g->U;
    /* acc[0..2]: D^P_d per axis; acc[3]: sum_d D^{PV}_d; acc[4]: sum_d D^V_d */
    for (int f = 0; f < 5; f++) memset(g->acc[f], 0, (size_t)nc * sizeof(double));
    double maxz = 0.0;
    for (int a = 0; a < g->ndim; a++) {
        long L = g->N[a], s = stride_of(g, a), G = g->g[a], n = g->n[a];
        double h = g->h[a];
        long nl = nlines(g, a);
#pragma omp parallel reduction(max : maxz)
        {
            linebuf b;
            lb_alloc(&b, L);
#pragma omp for schedule(static)
            for (long l = 0; l < nl; l++) {
                long ci, cj, ck;
                long base = line_base(g, a, l, &ci, &cj, &ck);
                double *qv = b.q[0], *qp = b.q[1], *qr = b.q[2], *qs = b.q[3];
                for (long m = 0; m < L; m++) {
                    long q = base + m * s;
                    double r = U[F_RHO][q];
                    qr[m] = r;
                    qs[m] = sqrt(r);
                    qv[m] = U[F_MX + a][q] / r;
                    qp[m] = g->iso ? (g->cs * g->cs) * r : (gam - 1.0) * U[F_E][q];
                }
                recon(g, &b, 0, L); /* velocity parabolas */
                recon(g, &b, 1, L); /* pressure parabolas */
                /* interfaces j+1/2 between cells j and j+1, j = G-1 .. G+n-1 */
                double *Vi = b.A, *Pi = b.B;
                for (long j = G - 1; j <= G + n - 1; j++) {
                    double sL = qs[j], sR = qs[j + 1];
                    double A = qr[j] * sL + qr[j + 1] * sR;
                    double B = sL + sR;
                    double C = qp[j] * sL + qp[j + 1] * sR;
                    double lam = sqrt(gam * C / A);
                    double Z = sqrt(gam * A * C) / B;
                    double z = lam * tau / h;
                    if (z > maxz) maxz = z;
                    double vm = og_avg_left(b.qL[0][j], b.qR[0][j], b.q6[0][j], z);
                    double vp = og_avg_right(b.qL[0][j + 1], b.qR[0][j + 1], b.q6[0][j + 1], z);
                    double pm = og_avg_left(b.qL[1][j], b.qR[1][j], b.q6[1][j], z);
                    double pp = og_avg_right(b.qL[1][j + 1], b.qR[1][j + 1], b.q6[1][j + 1], z);
                    Vi[j] = 0.5 * (vm + vp) + (pm - pp) / (2.0 * Z);
                    Pi[j] = 0.5 * (pm + pp) + (0.5 * Z) * (vm - vp);
                }
                for (long j = G; j < G + n; j++) {
                    long q = base + j * s;
                    g->acc[a][q] = (Pi[j] - Pi[j - 1]) / h;
                    g->acc[3][q] += (Pi[j] * Vi[j] - Pi[j - 1] * Vi[j - 1]) / h;
                    g->acc[4][q] += (Vi[j] - Vi[j - 1]) / h;
                }
            }
            lb_free(&b);
        }
    }
    g->last_max_z_euler = maxz;
    /* stage update (rho unchanged) */
    for (long k = 0; k < g->n[2]; k++)
        for (long j = 0; j < g->n[1]; j++)
            for (long i = 0; i < g->n[0]; i++) {
                long q = gidx(g, i + g->g[0], j + g->g[1], k + g->g[2]);
                double r = U[F_RHO][q];
                g->W[F_RHO][q] = r;
                for (int a = 0; a < 3; a++) {
                    double m = U[F_MX + a][q];
                    if (a < g->ndim) m = m - tau * g->acc[a][q];
                    g->W[F_MX + a][q] = m;
                }
                g->W[F_ET][q] = U[F_ET][q] - tau * g->acc[3][q];
                g->W[F_E][q] = U[F_E][q] - ((tau * (gam - 1.0)) * U[F_E][q]) * g->acc[4][q];
                if (g->potential != POT_NONE || g->self_grav) {
                    double gr[3];
                    potential_grad(g, i, j, k, gr);
                    if (g->self_grav) {
                        double gs[3];
                        self_gravity_grad(g, i, j, k, gs);
                        for (int a = 0; a < 3; a++) gr[a] += gs[a];
                    }
                    /* force along the active axes only */
                    for (int a = g->ndim; a < 3; a++) gr[a] = 0.0;
                    double work = U[F_MX][q] * gr[0] + U[F_MY][q] * gr[1] + U[F_MZ][q] * gr[2];
                    for (int a = 0; a < g->ndim; a++) g->W[F_MX + a][q] = g->W[F_MX + a][q] - (tau * r) * gr[a];
                    g->W[F_ET][q] = g->W[F_ET][q] - tau * work;
                }
            }
}

/* Transverse velocity template (Sec. 2.3, 9-point formula): weights 1/16 on
 * the four transverse corners, 1/8 on the four transverse edges and 1/4 at
 * the centre in 3-D; the same (1/4,1/2,1/4) rule on one transverse axis in
 * 2-D; the cell's own velocity in 1-D.  V holds the velocity component along
 * axis a on the whole ghosted grid. */
static double transverse_avg(const og_grid *g, const double *V, int a, long q)
{
    if (g->ndim == 1) return V[q];
    /* transverse axes in increasing order */
    int t1 = (a == 0) ? 1 : 0;
    int t2 = (a == 2) ? 1 : 2;
    long s1 = stride_of(g, t1);
    if (g->ndim == 2) {
        /* the single transverse axis is t1 (axis 0 or 1) */
        return 0.25 * (V[q + s1] + V[q - s1]) + 0.5 * V[q];
    }
    long s2 = stride_of(g, t2);
    double corners = V[q + s1 + s2] + V[q + s1 - s2] + V[q - s1 + s2] + V[q - s1 - s2];
    double edges = V[q + s1] + V[q - s1] + V[q + s2] + V[q - s2];
    return 0.0625 * corners + 0.125 * edges + 0.25 * V[q];
}

/* ------------------------------------------------------------------------ */
/* Lagrangian stage (Sec. 2.3): W -> U.  Unsplit advective transport of      */
/* every conserved density with upwind parabolic fluxes F = vhat * f.        */
/* ------------------------------------------------------------------------ */
static void lagrangian_stage(og_grid *g, double tau)
{
    long nc = ncell_ghosted(g);
    double **W = g->W;
    for (int f = 0; f < NF; f++) memset(g->acc[f], 0, (size_t)nc * sizeof(double));
    /* velocity component along each axis, on the whole ghosted grid */
    double *vel = (double *)calloc((size_t)nc, sizeof(double));
    double maxz = 0.0;
    for (int a = 0; a < g->ndim; a++) {
        for (long q = 0; q < nc; q++) vel[q] = W[F_MX + a][q] / W[F_RHO][q];
        long L = g->N[a], s = stride_of(g, a), G = g->g[a], n = g->n[a];
        double h = g->h[a];
        long nl = nlines(g, a);
#pragma omp parallel reduction(max : maxz)
        {
            linebuf b;
            lb_alloc(&b, L);
#pragma omp for schedule(static)
            for (long l = 0; l < nl; l++) {
                long ci, cj, ck;
                long base = line_base(g, a, l, &ci, &cj, &ck);
                double *vt = b.q[NF], *sq = b.q[NF + 1], *vh = b.A;
                for (long m = 0; m < L; m++) {
                    long q = base + m * s;
                    for (int f = 0; f < NF; f++) b.q[f][m] = W[f][q];
                    sq[m] = sqrt(W[F_RHO][q]);
                }
                for (long m = G - 1; m <= G + n; m++) vt[m] = transverse_avg(g, vel, a, base + m * s);
                for (int f = 0; f < NF; f++) recon(g, &b, f, L);
                for (long j = G - 1; j <= G + n - 1; j++) {
                    double v = (vt[j] * sq[j] + vt[j + 1] * sq[j + 1]) / (sq[j] + sq[j + 1]);
                    vh[j] = v;
                    double z = fabs(v) * tau / h;
                    if (z > maxz) maxz = z;
                    for (int f = 0; f < NF; f++) {
                        double fs;
                        if (v >= 0.0) fs = og_avg_left(b.qL[f][j], b.qR[f][j], b.q6[f][j], z);
                        else fs = og_avg_right(b.qL[f][j + 1], b.qR[f][j + 1], b.q6[f][j + 1], z);
                        b.F[f][j] = v * fs;
                    }
                }
                for (long j = G; j < G + n; j++) {
                    long q = base + j * s;
                    for (int f = 0; f < NF; f++) g->acc[f][q] += (b.F[f][j] - b.F[f][j - 1]) / h;
                }
            }
            lb_free(&b);
        }
    }
    free(vel);
    g->last_max_z_lagr = maxz;
    for (long k = 0; k < g->n[2]; k++)
        for (long j = 0; j < g->n[1]; j++)
            for (long i = 0; i < g->n[0]; i++) {
                long q = gidx(g, i + g->g[0], j + g->g[1], k + g->g[2]);
                for (int f = 0; f < NF; f++) g->U[f][q] = W[f][q] - tau * g->acc[f][q];
            }
}

/* ------------------------------------------------------------------------ */
/* Total-energy correction (Sec. 2.4), on interior cells of U^{n+1}.        */
/* rho < vacuum_ratio * mean: rescale |v| to sqrt(2 (E - eps)) keeping its   */
/* direction (or stop the gas and put all energy in eps when E <= eps).     */
/* Elsewhere: rho eps := rho E - |rho v|^2 / (2 rho) when that is positive.  */
/* rho E is never changed.                                                  */
/* ------------------------------------------------------------------------ */
static void energy_correction(og_grid *g)
{
    double thr = g->vacuum_ratio * g->rho_mean0;
    for (long k = 0; k < g->n[2]; k++)
        for (long j = 0; j < g->n[1]; j++)
            for (long i = 0; i < g->n[0]; i++) {
                long q = gidx(g, i + g->g[0], j + g->g[1], k + g->g[2]);
                double r = g->U[F_RHO][q];
                double mx = g->U[F_MX][q], my = g->U[F_MY][q], mz = g->U[F_MZ][q];
                double Et = g->U[F_ET][q], e = g->U[F_E][q];
                if (r < thr) {
                    double E = Et / r, eps = e / r;
                    double w = sqrt(mx * mx + my * my + mz * mz) / r;
                    if (E > eps && w > 0.0) {
                        double sc = sqrt(2.0 * (E - eps)) / w;
                        g->U[F_MX][q] = mx * sc;
                        g->U[F_MY][q] = my * sc;
                        g->U[F_MZ][q] = mz * sc;
                    } else {
                        g->U[F_MX][q] = 0.0;
                        g->U[F_MY][q] = 0.0;
                        g->U[F_MZ][q] = 0.0;
                        g->U[F_E][q] = Et;
                    }
                } else {
                    double kin = (mx * mx + my * my + mz * mz) / (2.0 * r);
                    double d = Et - kin;
                    if (d > 0.0) g->U[F_E][q] = d;
                }
            }
}

/* One full step U^n -> U^{n+1} with time step tau. */
void og_step(og_grid *g, double tau)
{
    if (g->self_grav) poisson(g);
    fill_ghosts(g, g->U);
    eulerian_stage(g, tau);
    fill_ghosts(g, g->W);
    lagrangian_stage(g, tau);
    energy_correction(g);
    g->t += tau;
    g->steps += 1;
}

/* Run up to nsteps steps.  dt_fixed > 0 uses that time step, otherwise the
 * CFL step of the current state; t_stop > 0 clips the step so the run ends
 * exactly at t_stop and stops there.  taus (may be NULL) receives the time
 * steps taken.  Returns the number of steps taken. */
long og_run(og_grid *g, long nsteps, double dt_fixed, double t_stop, double *taus)
{
    long taken = 0;
    for (long s = 0; s < nsteps; s++) {
        double tau = dt_fixed > 0.0 ? dt_fixed : og_dt(g);
        if (t_stop > 0.0) {
            double rem = t_stop - g->t;
            if (rem <= 0.0) break;
            if (tau > rem) tau = rem;
        }
        og_step(g, tau);
        if (taus) taus[taken] = tau;
        taken++;
    }
    return taken;
}

/* Threads the oracle's parallel loops use (for reporting), and a setter for
 * timing it on a given number of cores (results do not depend on it: the
 * only reduction is an exact maximum). */
#ifdef _OPENMP
#include <omp.h>
int og_max_threads(void) { return omp_get_max_threads(); }
void og_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
#else
int og_max_threads(void) { return 1; }
void og_set_threads(int n) { (void)n; }
#endif
