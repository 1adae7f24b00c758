// ppml_api.hip -- host implementation of the C ABI declared in include/ppml.h.
// Argument checking, launch geometry, and the enqueueing of the kernels of
// ppml_kernels.hip on the caller's stream.  No computation of the method
// happens on the host.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/ppml.h"
#include "ppml_kernels.hpp"

using namespace ppml;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

#define HIPCHK(expr)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return fail(PPML_EHIP, "%s: %s", #expr, hipGetErrorString(e_));          \
    } while (0)

// Tile shapes per dimensionality (x extent, y extent, z chunk).
constexpr int T1X = 256;
constexpr int T2X = 32, T2Y = 8;
constexpr int T3X = 32, T3Y = 8;

// Fields per LDS pass of the Lagrangian kernel (all six in FP32; FP64 in
// two passes to keep two work groups per CU).
template <typename T> struct LG {
    static constexpr int g = sizeof(T) == 4 ? 6 : 3;
};

int nfields(const ppml_desc *d) { return 3 + d->ndim; }

size_t elem(const ppml_desc *d) { return d->prec == PPML_FP64 ? sizeof(double) : sizeof(float); }

long long ncells(const ppml_desc *d)
{
    return (long long)d->n[0] * (long long)d->n[1] * (long long)d->n[2];
}

int validate(const ppml_desc *d)
{
    if (!d) return fail(PPML_EINVAL, "descriptor is NULL");
    if (d->ndim < 1 || d->ndim > 3) return fail(PPML_EINVAL, "ndim must be 1, 2 or 3 (got %d)", d->ndim);
    if (d->prec != PPML_FP32 && d->prec != PPML_FP64) return fail(PPML_EINVAL, "prec must be PPML_FP32 or PPML_FP64");
    for (int a = 0; a < 3; a++) {
        if (a < d->ndim) {
            if (d->n[a] < 1 || d->n[a] > (1 << 20)) return fail(PPML_EINVAL, "n[%d] out of range", a);
            if (!(d->hi[a] > d->lo[a])) return fail(PPML_EINVAL, "hi[%d] must exceed lo[%d]", a, a);
            for (int s = 0; s < 2; s++) {
                int b = s ? d->bc_hi[a] : d->bc_lo[a];
                if (b != PPML_PERIODIC && b != PPML_OUTFLOW && b != PPML_REFLECT)
                    return fail(PPML_EINVAL, "bad boundary code on axis %d", a);
                if (b == PPML_REFLECT && d->n[a] < 3) return fail(PPML_EINVAL, "reflecting axis %d needs n >= 3", a);
            }
            if ((d->bc_lo[a] == PPML_PERIODIC) != (d->bc_hi[a] == PPML_PERIODIC))
                return fail(PPML_EINVAL, "axis %d: periodic must be set on both faces", a);
        } else if (d->n[a] != 1) {
            return fail(PPML_EINVAL, "n[%d] must be 1 for an unused axis", a);
        }
    }
    if (ncells(d) > (1ll << 31) - 1) return fail(PPML_EINVAL, "grid too large (%lld cells)", ncells(d));
    if (!(d->gamma > 1.0) || !std::isfinite(d->gamma)) return fail(PPML_EINVAL, "gamma must be > 1");
    if (!(d->cfl > 0.0 && d->cfl < 1.0)) return fail(PPML_EINVAL, "cfl must lie in (0, 1)");
    if (!(d->vacuum_ratio >= 0.0)) return fail(PPML_EINVAL, "vacuum_ratio must be >= 0");
    if (d->potential != PPML_POT_NONE && d->potential != PPML_POT_LOG && d->potential != PPML_POT_UNIFORM)
        return fail(PPML_EINVAL, "bad potential code");
    if (d->potential == PPML_POT_LOG && !(d->pot[2] > 0.0)) return fail(PPML_EINVAL, "log potential needs q > 0");
    if (d->reserved != 0) return fail(PPML_EINVAL, "reserved must be 0");
    return PPML_OK;
}

constexpr size_t ALIGN = 256;
size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

// Totals reduction: fixed number of blocks so the summation order is fixed.
int totals_blocks(long long n) { return (int)std::min<long long>(1024, (n + 4095) / 4096 > 0 ? (n + 4095) / 4096 : 1); }

struct ScratchLayout {
    size_t half, ctrl, partial, totals, total;
};

ScratchLayout layout(const ppml_desc *d)
{
    ScratchLayout L;
    L.half = 0;
    size_t sz = align_up((size_t)nfields(d) * (size_t)ncells(d) * elem(d));
    L.ctrl = sz;
    sz += align_up(sizeof(Ctrl));
    L.partial = sz;
    sz += align_up((size_t)totals_blocks(ncells(d)) * 6 * sizeof(double));
    L.totals = sz;
    sz += align_up(8 * sizeof(double));
    L.total = sz;
    return L;
}

}  // namespace

struct ppml_grid {
    ppml_desc d;
    GridParams gp;
    hipStream_t stream;
    int device;
    void *state;
    void *half;
    Ctrl *ctrl;
    double *partial;
    double *totals;
    long long step_count;  // steps enqueued (selects the CFL slot)
    bool has_state;
    std::vector<hipEvent_t> ev;  // 3 events per timed step
    long long timed;             // steps recorded since the last read
};

namespace {

template <typename T> void launch_speeds(ppml_grid *g, int slot)
{
    const T *U = (const T *)g->state;
    int nb = (int)std::min<long long>(4096, (g->gp.ncell + 255) / 256);
    switch (g->d.ndim) {
    case 1: k_speeds<T, 1><<<nb, 256, 0, g->stream>>>(U, g->gp, g->ctrl, slot); break;
    case 2: k_speeds<T, 2><<<nb, 256, 0, g->stream>>>(U, g->gp, g->ctrl, slot); break;
    default: k_speeds<T, 3><<<nb, 256, 0, g->stream>>>(U, g->gp, g->ctrl, slot); break;
    }
}

template <typename T> void launch_step(ppml_grid *g, const StepArgs &sa, hipEvent_t *ev)
{
    // ev (may be NULL): events recorded before, between and after the kernels
    const T *U = (const T *)g->state;
    T *Us = (T *)g->state;
    T *W = (T *)g->half;
    const GridParams &gp = g->gp;
    const int nb = gp.tiles[0] * gp.tiles[1] * gp.tiles[2];
    if (ev) (void)hipEventRecord(ev[0], g->stream);
    switch (g->d.ndim) {
    case 1: k_euler<T, 1, T1X, 1><<<nb, T1X, 0, g->stream>>>(U, W, gp, g->ctrl, sa); break;
    case 2: k_euler<T, 2, T2X, T2Y><<<nb, T2X * T2Y, 0, g->stream>>>(U, W, gp, g->ctrl, sa); break;
    default: k_euler<T, 3, T3X, T3Y><<<nb, T3X * T3Y, 0, g->stream>>>(U, W, gp, g->ctrl, sa); break;
    }
    if (ev) (void)hipEventRecord(ev[1], g->stream);
    switch (g->d.ndim) {
    case 1: k_lagr<T, 1, T1X, 1, LG<T>::g><<<nb, T1X, 0, g->stream>>>(W, Us, gp, g->ctrl, sa); break;
    case 2: k_lagr<T, 2, T2X, T2Y, LG<T>::g><<<nb, T2X * T2Y, 0, g->stream>>>(W, Us, gp, g->ctrl, sa); break;
    default: k_lagr<T, 3, T3X, T3Y, LG<T>::g><<<nb, T3X * T3Y, 0, g->stream>>>(W, Us, gp, g->ctrl, sa); break;
    }
    if (ev) (void)hipEventRecord(ev[2], g->stream);
}

template <typename T> void launch_totals(ppml_grid *g, double mean_cells)
{
    const long long N = g->gp.ncell;
    int nb = totals_blocks(N);
    long long chunk = (N + nb - 1) / nb;
    k_totals_partial<T><<<nb, TOT_THREADS, 0, g->stream>>>((const T *)g->state, N, nfields(&g->d), chunk, g->partial);
    k_totals_final<<<1, TOT_THREADS, 0, g->stream>>>(g->partial, nb, nfields(&g->d), g->d.ndim, g->totals, g->ctrl,
                                                      mean_cells);
}

int check_err(ppml_grid *g)
{
    int err = 0;
    HIPCHK(hipMemcpyAsync(&err, &g->ctrl->err, sizeof(int), hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
    if (err) return fail(PPML_ENONFINITE, "a step produced rho <= 0, eps <= 0 or a non-finite value");
    return PPML_OK;
}

int grid_ok(ppml_grid *g)
{
    if (!g) return fail(PPML_EINVAL, "grid is NULL");
    return PPML_OK;
}

// After the state is set: reset the control block, record the mean density,
// compute the CFL maxima of the state into slot 0.
int finish_set(ppml_grid *g, double t, double rho_mean0)
{
    k_ctrl_reset<<<1, 1, 0, g->stream>>>(g->ctrl, t);
    HIPCHK(hipGetLastError());
    if (g->d.prec == PPML_FP64) {
        launch_totals<double>(g, rho_mean0 > 0.0 ? 0.0 : (double)g->gp.ncell);
        launch_speeds<double>(g, 0);
    } else {
        launch_totals<float>(g, rho_mean0 > 0.0 ? 0.0 : (double)g->gp.ncell);
        launch_speeds<float>(g, 0);
    }
    HIPCHK(hipGetLastError());
    if (rho_mean0 > 0.0)
        HIPCHK(hipMemcpyAsync(&g->ctrl->rho_mean0, &rho_mean0, sizeof(double), hipMemcpyHostToDevice, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
    g->step_count = 0;
    g->has_state = true;
    return PPML_OK;
}

bool all_finite_positive(const double *a, long long n)
{
    for (long long i = 0; i < n; i++)
        if (!(a[i] > 0.0) || !std::isfinite(a[i])) return false;
    return true;
}

bool all_finite(const double *a, long long n)
{
    for (long long i = 0; i < n; i++)
        if (!std::isfinite(a[i])) return false;
    return true;
}

}  // namespace

extern "C" {

size_t ppml_state_bytes(const ppml_desc *d)
{
    if (validate(d) != PPML_OK) return 0;
    return (size_t)nfields(d) * (size_t)ncells(d) * elem(d);
}

size_t ppml_scratch_bytes(const ppml_desc *d)
{
    if (validate(d) != PPML_OK) return 0;
    return layout(d).total;
}

int ppml_create(const ppml_desc *d, void *state_dev, void *scratch_dev, void *hip_stream, ppml_grid **out)
{
    int rc = validate(d);
    if (rc != PPML_OK) return rc;
    if (!out) return fail(PPML_EINVAL, "out is NULL");
    if (!state_dev || !scratch_dev) return fail(PPML_EINVAL, "state and scratch pointers must be non-NULL");
    if (((uintptr_t)state_dev % ALIGN) || ((uintptr_t)scratch_dev % ALIGN))
        return fail(PPML_EINVAL, "device pointers must be %zu-byte aligned", ALIGN);
    ppml_grid *g = new (std::nothrow) ppml_grid();
    if (!g) return fail(PPML_ENOMEM, "host allocation failed");
    g->d = *d;
    HIPCHK(hipGetDevice(&g->device));
    g->stream = (hipStream_t)hip_stream;
    g->state = state_dev;
    ScratchLayout L = layout(d);
    char *s = (char *)scratch_dev;
    g->half = s + L.half;
    g->ctrl = (Ctrl *)(s + L.ctrl);
    g->partial = (double *)(s + L.partial);
    g->totals = (double *)(s + L.totals);
    GridParams &gp = g->gp;
    memset(&gp, 0, sizeof gp);
    gp.ndim = d->ndim;
    double hmin = 1e300;
    for (int a = 0; a < 3; a++) {
        gp.n[a] = (int)d->n[a];
        gp.lo[a] = d->lo[a];
        gp.h[a] = (d->hi[a] - d->lo[a]) / (double)d->n[a];
        gp.inv_h[a] = 1.0 / gp.h[a];
        gp.bc_lo[a] = a < d->ndim ? d->bc_lo[a] : PPML_PERIODIC;
        gp.bc_hi[a] = a < d->ndim ? d->bc_hi[a] : PPML_PERIODIC;
        if (a < d->ndim && gp.h[a] < hmin) hmin = gp.h[a];
    }
    gp.ncell = ncells(d);
    gp.gamma = d->gamma;
    gp.cfl_hmin = d->cfl * hmin;
    gp.vacuum_ratio = d->vacuum_ratio;
    gp.potential = d->potential;
    for (int i = 0; i < 8; i++) gp.pot[i] = d->pot[i];
    // tiles of the stage kernels; 3-D: z chunk small enough that the launch
    // has enough work groups to fill 256 CUs several times over
    if (d->ndim == 1) {
        gp.tiles[0] = (gp.n[0] + T1X - 1) / T1X;
        gp.tiles[1] = gp.tiles[2] = 1;
        gp.cz = 1;
    } else if (d->ndim == 2) {
        gp.tiles[0] = (gp.n[0] + T2X - 1) / T2X;
        gp.tiles[1] = (gp.n[1] + T2Y - 1) / T2Y;
        gp.tiles[2] = 1;
        gp.cz = 1;
    } else {
        gp.tiles[0] = (gp.n[0] + T3X - 1) / T3X;
        gp.tiles[1] = (gp.n[1] + T3Y - 1) / T3Y;
        long long tiles = (long long)gp.tiles[0] * gp.tiles[1];
        int cz = gp.n[2];
        while (cz > 16 && tiles * ((gp.n[2] + cz - 1) / cz) < 2048) cz = (cz + 1) / 2;
        gp.cz = cz;
        gp.tiles[2] = (gp.n[2] + cz - 1) / cz;
    }
    g->has_state = false;
    g->step_count = 0;
    g->timed = 0;
    *out = g;
    return PPML_OK;
}

int ppml_set_primitive(ppml_grid *g, const double *rho, const double *vx, const double *vy, const double *vz,
                       const double *p)
{
    int rc = grid_ok(g);
    if (rc) return rc;
    if (!rho || !p) return fail(PPML_EINVAL, "rho and p are required");
    const long long N = g->gp.ncell;
    if (!all_finite_positive(rho, N)) return fail(PPML_EINVAL, "rho must be finite and > 0");
    if (!all_finite_positive(p, N)) return fail(PPML_EINVAL, "p must be finite and > 0");
    const double *v[3] = {vx, vy, vz};
    for (int a = 0; a < g->d.ndim; a++)
        if (v[a] && !all_finite(v[a], N)) return fail(PPML_EINVAL, "velocity %d has non-finite values", a);
    double *prim = nullptr;
    HIPCHK(hipMalloc(&prim, (size_t)5 * N * sizeof(double)));
    const double *src[5] = {rho, vx, vy, vz, p};
    for (int i = 0; i < 5; i++) {
        if (src[i]) {
            hipError_t e = hipMemcpyAsync(prim + (size_t)i * N, src[i], N * sizeof(double), hipMemcpyHostToDevice,
                                          g->stream);
            if (e != hipSuccess) {
                (void)hipFree(prim);
                return fail(PPML_EHIP, "copy of primitive %d: %s", i, hipGetErrorString(e));
            }
        } else {
            hipError_t e = hipMemsetAsync(prim + (size_t)i * N, 0, N * sizeof(double), g->stream);
            if (e != hipSuccess) {
                (void)hipFree(prim);
                return fail(PPML_EHIP, "hipMemsetAsync: %s", hipGetErrorString(e));
            }
        }
    }
    int nb = (int)std::min<long long>(4096, (N + 255) / 256);
    if (g->d.prec == PPML_FP64) k_prim_to_cons<double><<<nb, 256, 0, g->stream>>>(prim, (double *)g->state, g->gp);
    else k_prim_to_cons<float><<<nb, 256, 0, g->stream>>>(prim, (float *)g->state, g->gp);
    hipError_t e = hipGetLastError();
    hipError_t e2 = hipStreamSynchronize(g->stream);
    (void)hipFree(prim);
    if (e != hipSuccess || e2 != hipSuccess)
        return fail(PPML_EHIP, "prim_to_cons: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    return finish_set(g, 0.0, 0.0);
}

int ppml_set_conserved(ppml_grid *g, const double *const *f, double rho_mean0, double t)
{
    int rc = grid_ok(g);
    if (rc) return rc;
    if (!f || !f[PPML_RHO] || !f[PPML_ETOT] || !f[PPML_EINT]) return fail(PPML_EINVAL, "rho, Et and e are required");
    const long long N = g->gp.ncell;
    const int nd = g->d.ndim;
    if (!all_finite_positive(f[PPML_RHO], N)) return fail(PPML_EINVAL, "rho must be finite and > 0");
    if (!all_finite_positive(f[PPML_EINT], N)) return fail(PPML_EINVAL, "rho*eps must be finite and > 0");
    if (!all_finite(f[PPML_ETOT], N)) return fail(PPML_EINVAL, "rho*E must be finite");
    if (!std::isfinite(t) || t < 0.0) return fail(PPML_EINVAL, "t must be finite and >= 0");
    double *tmp = nullptr;
    HIPCHK(hipMalloc(&tmp, (size_t)N * sizeof(double)));
    int nb = (int)std::min<long long>(4096, (N + 255) / 256);
    // stored field s <- ppml_field
    int nfs = nfields(&g->d);
    for (int s = 0; s < nfs; s++) {
        int fld = s == 0 ? PPML_RHO : (s <= nd ? s : (s == nd + 1 ? PPML_ETOT : PPML_EINT));
        hipError_t e;
        if (f[fld]) {
            if (!all_finite(f[fld], N)) {
                (void)hipFree(tmp);
                return fail(PPML_EINVAL, "field %d has non-finite values", fld);
            }
            e = hipMemcpyAsync(tmp, f[fld], N * sizeof(double), hipMemcpyHostToDevice, g->stream);
        } else {
            e = hipMemsetAsync(tmp, 0, N * sizeof(double), g->stream);
        }
        if (e == hipSuccess) {
            if (g->d.prec == PPML_FP64)
                k_from_double<double><<<nb, 256, 0, g->stream>>>(tmp, (double *)g->state + (size_t)s * N, N);
            else
                k_from_double<float><<<nb, 256, 0, g->stream>>>(tmp, (float *)g->state + (size_t)s * N, N);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
        if (e != hipSuccess) {
            (void)hipFree(tmp);
            return fail(PPML_EHIP, "set_conserved: %s", hipGetErrorString(e));
        }
    }
    (void)hipFree(tmp);
    return finish_set(g, t, rho_mean0);
}

int ppml_step(ppml_grid *g, int32_t nsteps, double dt_fixed, double t_stop)
{
    int rc = grid_ok(g);
    if (rc) return rc;
    if (nsteps < 0) return fail(PPML_EINVAL, "nsteps must be >= 0");
    if (!g->has_state) return fail(PPML_ESTATE, "state was never set");
    if (!std::isfinite(dt_fixed) || !std::isfinite(t_stop)) return fail(PPML_EINVAL, "dt_fixed and t_stop must be finite");
    for (int s = 0; s < nsteps; s++) {
        StepArgs sa;
        sa.dt_fixed = dt_fixed;
        sa.t_stop = t_stop;
        sa.slot = (int)(g->step_count & 1);
        hipEvent_t *ev = nullptr;
        if ((size_t)(3 * (g->timed + 1)) <= g->ev.size()) ev = &g->ev[3 * g->timed];
        if (g->d.prec == PPML_FP64) launch_step<double>(g, sa, ev);
        else launch_step<float>(g, sa, ev);
        if (ev) g->timed++;
        g->step_count++;
    }
    HIPCHK(hipGetLastError());
    return PPML_OK;
}

int ppml_get_time(ppml_grid *g, double *t, double *dt_last, int64_t *steps)
{
    int rc = grid_ok(g);
    if (rc) return rc;
    Ctrl c;
    HIPCHK(hipMemcpyAsync(&c, g->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
    if (t) *t = c.t;
    if (dt_last) *dt_last = c.dt_last;
    if (steps) *steps = c.steps;
    if (c.err) return fail(PPML_ENONFINITE, "a step produced rho <= 0, eps <= 0 or a non-finite value");
    return PPML_OK;
}

int ppml_max_speeds(ppml_grid *g, double *vmax, double *cmax)
{
    int rc = grid_ok(g);
    if (rc) return rc;
    Ctrl c;
    HIPCHK(hipMemcpyAsync(&c, g->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
    int slot = (int)(g->step_count & 1);
    double v, cs;
    unsigned long long vb = c.vmax_bits[slot], cb = c.cmax_bits[slot];
    memcpy(&v, &vb, sizeof v);
    memcpy(&cs, &cb, sizeof cs);
    if (vmax) *vmax = v;
    if (cmax) *cmax = cs;
    return PPML_OK;
}

int ppml_get_conserved(ppml_grid *g, int32_t field, double *host_out)
{
    int rc = grid_ok(g);
    if (rc) return rc;
    if (!host_out) return fail(PPML_EINVAL, "host_out is NULL");
    const int nd = g->d.ndim;
    int s;
    switch (field) {
    case PPML_RHO: s = 0; break;
    case PPML_MX: s = 1; break;
    case PPML_MY: s = nd >= 2 ? 2 : -1; break;
    case PPML_MZ: s = nd >= 3 ? 3 : -1; break;
    case PPML_ETOT: s = nd + 1; break;
    case PPML_EINT: s = nd + 2; break;
    default: s = -1;
    }
    if (s < 0) return fail(PPML_EINVAL, "field %d is not stored for ndim=%d", field, nd);
    const long long N = g->gp.ncell;
    double *tmp = nullptr;
    HIPCHK(hipMalloc(&tmp, (size_t)N * sizeof(double)));
    int nb = (int)std::min<long long>(4096, (N + 255) / 256);
    if (g->d.prec == PPML_FP64)
        k_to_double<double><<<nb, 256, 0, g->stream>>>((const double *)g->state + (size_t)s * N, tmp, N);
    else
        k_to_double<float><<<nb, 256, 0, g->stream>>>((const float *)g->state + (size_t)s * N, tmp, N);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(host_out, tmp, N * sizeof(double), hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    (void)hipFree(tmp);
    if (e != hipSuccess) return fail(PPML_EHIP, "get_conserved: %s", hipGetErrorString(e));
    return PPML_OK;
}

int ppml_totals(ppml_grid *g, double out[6])
{
    int rc = grid_ok(g);
    if (rc) return rc;
    if (!out) return fail(PPML_EINVAL, "out is NULL");
    if (!g->has_state) return fail(PPML_ESTATE, "state was never set");
    if (g->d.prec == PPML_FP64) launch_totals<double>(g, 0.0);
    else launch_totals<float>(g, 0.0);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(out, g->totals, 6 * sizeof(double), hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
    return PPML_OK;
}

int ppml_sync(ppml_grid *g)
{
    int rc = grid_ok(g);
    if (rc) return rc;
    return check_err(g);
}

int ppml_set_timing(ppml_grid *g, int32_t cap)
{
    int rc = grid_ok(g);
    if (rc) return rc;
    if (cap < 0 || cap > (1 << 20)) return fail(PPML_EINVAL, "timing capacity out of range");
    HIPCHK(hipStreamSynchronize(g->stream));
    for (hipEvent_t e : g->ev) (void)hipEventDestroy(e);
    g->ev.clear();
    g->timed = 0;
    for (int i = 0; i < 3 * cap; i++) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        g->ev.push_back(e);
    }
    return PPML_OK;
}

int ppml_get_timing(ppml_grid *g, double *ms_euler, double *ms_lagr, int64_t *nsteps)
{
    int rc = grid_ok(g);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(g->stream));
    double me = 0.0, ml = 0.0;
    for (long long s = 0; s < g->timed; s++) {
        float a = 0.f, b = 0.f;
        HIPCHK(hipEventElapsedTime(&a, g->ev[3 * s], g->ev[3 * s + 1]));
        HIPCHK(hipEventElapsedTime(&b, g->ev[3 * s + 1], g->ev[3 * s + 2]));
        me += a;
        ml += b;
    }
    if (ms_euler) *ms_euler = me;
    if (ms_lagr) *ms_lagr = ml;
    if (nsteps) *nsteps = g->timed;
    g->timed = 0;
    return PPML_OK;
}

int ppml_destroy(ppml_grid *g)
{
    if (!g) return fail(PPML_EINVAL, "grid is NULL");
    (void)hipStreamSynchronize(g->stream);
    for (hipEvent_t e : g->ev) (void)hipEventDestroy(e);
    delete g;
    return PPML_OK;
}

const char *ppml_strerror(int status)
{
    switch (status) {
    case PPML_OK: return "ok";
    case PPML_EINVAL: return "invalid argument";
    case PPML_ENOMEM: return "out of memory";
    case PPML_EHIP: return "HIP runtime error";
    case PPML_ENONFINITE: return "non-physical or non-finite state";
    case PPML_EBUDGET: return "memory budget exceeded";
    case PPML_ESTATE: return "invalid object state";
    default: return "unknown status";
    }
}

const char *ppml_last_error(void) { return g_err; }

int ppml_version(void) { return 100; }

}  // extern "C"
