/* Drives every mode of the CPU oracle (test infrastructure) on small grids,
 * for a build with AddressSanitizer and UndefinedBehaviorSanitizer: 1-, 2-
 * and 3-D grids with every boundary kind (inflow included), the first-order
 * and isothermal variants, the three fixed potentials, a vacuum region (the
 * vacuum branch of the energy correction), self-gravity with its potential
 * solve, and the line, strip-mean, sine-transform and multipole helpers.
 * Exits 0 when every run keeps its state finite; a sanitizer finding aborts. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct og_grid og_grid;
og_grid *og_create(int ndim, const long *n, const double *lo, const double *hi, double gamma, double cfl,
                   const int *bc_lo, const int *bc_hi, double vacuum_ratio, int potential, const double *pot,
                   int first_order);
void og_destroy(og_grid *g);
void og_set_primitive(og_grid *g, const double *rho, const double *vx, const double *vy, const double *vz,
                      const double *p);
void og_set_inflow(og_grid *g, int face, double rho, double vx, double vy, double vz, double p);
void og_get(const og_grid *g, int field, double *out);
void og_totals(const og_grid *g, double *out);
long og_run(og_grid *g, long nsteps, double dt_fixed, double t_stop, double *taus);
double og_dt(const og_grid *g);
void og_max_speeds(const og_grid *g, double *vmax, double *cmax);
int og_set_isothermal(og_grid *g, double cs);
int og_set_self_gravity(og_grid *g, double G);
int og_potential(og_grid *g, double *out);
void og_reconstruct_line(const double *q, long n, double *qL, double *qR, double *q6, double *dm, double *qI);
double og_avg_left(double qL, double qR, double q6, double z);
double og_avg_right(double qL, double qR, double q6, double z);
void og_sine_transform(const double *x, long n, double *y);
void og_multipole_moments(const og_grid *g, double *mom);
double og_multipole_value(const double *mom, double G, double x, double y, double z);

enum { PER = 0, OUT = 1, REF = 2, INF = 3 };
enum { POT_NONE = 0, POT_LOG = 1, POT_UNIFORM = 2, POT_HALO = 3 };

static int failures = 0;

static void check_finite(const og_grid *g, long nc, const char *name)
{
    double *buf = (double *)malloc((size_t)nc * sizeof(double));
    for (int f = 0; f < 6; f++) {
        og_get(g, f, buf);
        for (long c = 0; c < nc; c++)
            if (!isfinite(buf[c])) {
                printf("%s: field %d cell %ld not finite\n", name, f, c);
                failures++;
                free(buf);
                return;
            }
    }
    free(buf);
    double tot[6];
    og_totals(g, tot);
    for (int f = 0; f < 6; f++)
        if (!isfinite(tot[f])) failures++;
}

/* A smooth state with a dense blob and, optionally, a near-vacuum corner. */
static og_grid *make(int ndim, const long *n, const int *bl, const int *bh, int pot, const double *pp, int fo,
                     int vacuum, double lo0)
{
    double lo[3] = {lo0, lo0, lo0}, hi[3] = {lo0 + 1.0, lo0 + 1.0, lo0 + 1.0};
    og_grid *g = og_create(ndim, n, lo, hi, 5.0 / 3.0, 0.3, bl, bh, 1e-5, pot, pp, fo);
    if (!g) {
        failures++;
        return NULL;
    }
    long nc = n[0] * (ndim > 1 ? n[1] : 1) * (ndim > 2 ? n[2] : 1);
    double *r = malloc(nc * sizeof(double)), *u = malloc(nc * sizeof(double)), *v = malloc(nc * sizeof(double));
    double *w = malloc(nc * sizeof(double)), *p = malloc(nc * sizeof(double));
    long c = 0;
    for (long k = 0; k < (ndim > 2 ? n[2] : 1); k++)
        for (long j = 0; j < (ndim > 1 ? n[1] : 1); j++)
            for (long i = 0; i < n[0]; i++, c++) {
                double x = (i + 0.5) / n[0], y = (j + 0.5) / (ndim > 1 ? n[1] : 1), z = (k + 0.5) / (ndim > 2 ? n[2] : 1);
                double d2 = (x - 0.5) * (x - 0.5) + (y - 0.5) * (y - 0.5) + (z - 0.5) * (z - 0.5);
                r[c] = 1.0 + 2.0 * exp(-20.0 * d2);
                if (vacuum && x < 0.3 && y < 0.3) r[c] = 1e-8;
                u[c] = 0.3 * sin(6.283 * y);
                v[c] = -0.2 * cos(6.283 * x);
                w[c] = 0.1 * sin(6.283 * z);
                p[c] = 1.0 + (d2 < 0.02 ? 20.0 : 0.0);
            }
    og_set_primitive(g, r, u, v, w, p);
    free(r);
    free(u);
    free(v);
    free(w);
    free(p);
    return g;
}

static void run(og_grid *g, long nc, long steps, const char *name)
{
    if (!g) return;
    double taus[16];
    double vm, cm;
    og_max_speeds(g, &vm, &cm);
    if (!(og_dt(g) > 0.0)) failures++;
    long done = og_run(g, steps, 0.0, 0.0, taus);
    if (done != steps) {
        printf("%s: %ld of %ld steps\n", name, done, steps);
        failures++;
    }
    check_finite(g, nc, name);
    og_destroy(g);
}

int main(void)
{
    const double none[8] = {0};
    /* 1-D: periodic, reflect/outflow, inflow/outflow, first order */
    {
        long n[3] = {40, 1, 1};
        int bl[3] = {PER, PER, PER}, bh[3] = {PER, PER, PER};
        run(make(1, n, bl, bh, POT_NONE, none, 0, 0, 0.0), 40, 6, "1d periodic");
        int bl2[3] = {REF, PER, PER}, bh2[3] = {OUT, PER, PER};
        run(make(1, n, bl2, bh2, POT_NONE, none, 1, 0, 0.0), 40, 6, "1d reflect/outflow first order");
        int bl3[3] = {INF, PER, PER}, bh3[3] = {OUT, PER, PER};
        og_grid *g = make(1, n, bl3, bh3, POT_NONE, none, 0, 0, 0.0);
        og_set_inflow(g, 0, 1.5, 0.8, 0.0, 0.0, 2.0);
        run(g, 40, 6, "1d inflow");
    }
    /* 2-D: mixed faces with a uniform field, the isothermal variant, inflow */
    {
        long n[3] = {20, 16, 1};
        int bl[3] = {PER, REF, PER}, bh[3] = {PER, OUT, PER};
        double pu[8] = {0.0, -0.5, 0.0};
        run(make(2, n, bl, bh, POT_UNIFORM, pu, 0, 0, 0.0), 320, 5, "2d uniform field");
        og_grid *g = make(2, n, bl, bh, POT_NONE, none, 0, 0, 0.0);
        if (og_set_isothermal(g, 0.7) != 0) failures++;
        run(g, 320, 5, "2d isothermal");
        int bl2[3] = {INF, OUT, PER}, bh2[3] = {OUT, INF, PER};
        g = make(2, n, bl2, bh2, POT_NONE, none, 0, 0, 0.0);
        og_set_inflow(g, 0, 1.2, 0.5, 0.1, 0.0, 1.0);
        og_set_inflow(g, 3, 0.8, 0.0, -0.4, 0.0, 0.7);
        run(g, 320, 5, "2d inflow");
    }
    /* 3-D: every face kind, the logarithmic and halo potentials, a vacuum corner */
    {
        long n[3] = {10, 9, 8};
        int bl[3] = {PER, REF, OUT}, bh[3] = {PER, OUT, REF};
        double plog[8] = {0.3, 0.05, 0.9};
        run(make(3, n, bl, bh, POT_LOG, plog, 0, 1, -0.5), 720, 4, "3d log potential, vacuum");
        double phalo[8] = {0.5, 0.1, 0.3, 1.0, 0.2};
        run(make(3, n, bl, bh, POT_HALO, phalo, 0, 0, -0.5), 720, 4, "3d halo potential");
        int bl2[3] = {INF, REF, OUT}, bh2[3] = {OUT, REF, INF};
        og_grid *g = make(3, n, bl2, bh2, POT_NONE, none, 1, 0, 0.0);
        og_set_inflow(g, 0, 1.1, 0.4, 0.0, 0.1, 1.3);
        og_set_inflow(g, 5, 0.9, 0.0, 0.0, -0.3, 0.8);
        run(g, 720, 4, "3d inflow first order");
    }
    /* 3-D self-gravity: cubic cells, the origin off the shell cell centres */
    {
        long n[3] = {8, 8, 8};
        int bl[3] = {OUT, OUT, OUT}, bh[3] = {OUT, OUT, OUT};
        og_grid *g = make(3, n, bl, bh, POT_NONE, none, 0, 0, -0.53);
        if (og_set_self_gravity(g, 1.0) != 0) failures++;
        double *phi = malloc(10 * 10 * 10 * sizeof(double));
        if (og_potential(g, phi) != 0) failures++;
        for (int c = 0; c < 1000; c++)
            if (!isfinite(phi[c])) failures++;
        double mom[7];
        og_multipole_moments(g, mom);
        if (!isfinite(og_multipole_value(mom, 1.0, 2.0, 0.3, -0.1))) failures++;
        free(phi);
        run(g, 512, 3, "3d self-gravity");
    }
    /* helpers */
    {
        double q[12], qL[12], qR[12], q6[12], dm[12], qI[12], y[12];
        for (int j = 0; j < 12; j++) q[j] = sin(0.7 * j) + (j > 6 ? 1.0 : 0.0);
        og_reconstruct_line(q, 12, qL, qR, q6, dm, qI);
        for (int j = 2; j <= 9; j++)
            if (!isfinite(og_avg_left(qL[j], qR[j], q6[j], 0.3) + og_avg_right(qL[j], qR[j], q6[j], 0.3))) failures++;
        og_sine_transform(q, 12, y);
        for (int j = 0; j < 12; j++)
            if (!isfinite(y[j])) failures++;
    }
    printf("oracle sanitizer driver: %d failure(s)\n", failures);
    return failures ? 1 : 0;
}
