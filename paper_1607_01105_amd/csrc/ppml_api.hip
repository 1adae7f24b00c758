// ppml_api.hip -- host implementation of the C ABI declared in include/ppml.h.
// Argument checking, launch geometry, and the enqueueing of the kernels of
// ppml_kernels.hip on the caller's stream.  No computation of the method
// happens on the host.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <cmath>
#include <cstddef>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/ppml.h"
#include "ppml_gravity.hpp"
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

// Work-group tile shapes (x extent, y extent) per dimensionality; index 0 is
// the default.  Every shape runs the same per-cell arithmetic, so results do
// not depend on the choice; the autotuner picks one per workload.
template <int X, int Y> struct Tile {
    static constexpr int tx = X, ty = Y, nt = X * Y;
};
constexpr int NTILE[4] = {0, 3, 4, 4};
constexpr int TILE_X[4][4] = {{0, 0, 0, 0}, {256, 128, 64, 0}, {32, 64, 16, 32}, {32, 64, 16, 32}};
constexpr int TILE_Y[4][4] = {{0, 0, 0, 0}, {1, 1, 1, 0}, {8, 4, 16, 4}, {8, 4, 16, 4}};

// Calls f(Tile<tx, ty>{}) for tile shape v of dimensionality NDIM (the
// tables above, spelled out as template arguments).
template <int NDIM, typename F> void with_tile(int v, F &&f)
{
    if constexpr (NDIM == 1) {
        switch (v) {
        case 1: f(Tile<128, 1>{}); break;
        case 2: f(Tile<64, 1>{}); break;
        default: f(Tile<256, 1>{}); break;
        }
    } else {
        switch (v) {
        case 1: f(Tile<64, 4>{}); break;
        case 2: f(Tile<16, 16>{}); break;
        case 3: f(Tile<32, 4>{}); break;
        default: f(Tile<32, 8>{}); break;
        }
    }
}

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
                if (b != PPML_PERIODIC && b != PPML_OUTFLOW && b != PPML_REFLECT && b != PPML_INFLOW)
                    return fail(PPML_EINVAL, "bad boundary code on axis %d", a);
                if (b == PPML_REFLECT && d->n[a] < 3) return fail(PPML_EINVAL, "reflecting axis %d needs n >= 3", a);
                if (b == PPML_INFLOW) {
                    const double *st = d->inflow[2 * a + s];
                    for (int q = 0; q < 5; q++)
                        if (!std::isfinite(st[q])) return fail(PPML_EINVAL, "inflow state of face %d is not finite", 2 * a + s);
                    if (!(st[0] > 0.0) || !(st[4] > 0.0))
                        return fail(PPML_EINVAL, "inflow face %d needs rho > 0 and p > 0", 2 * a + s);
                }
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
    if (d->potential != PPML_POT_NONE && d->potential != PPML_POT_LOG && d->potential != PPML_POT_UNIFORM &&
        d->potential != PPML_POT_HALO)
        return fail(PPML_EINVAL, "bad potential code");
    if (d->potential == PPML_POT_LOG && !(d->pot[2] > 0.0)) return fail(PPML_EINVAL, "log potential needs q > 0");
    if (d->potential == PPML_POT_HALO && !(d->pot[1] > 0.0 && d->pot[2] > 0.0))
        return fail(PPML_EINVAL, "halo potential needs r0 > 0 and rh > 0");
    if (d->potential == PPML_POT_HALO && d->ndim != 3) return fail(PPML_EINVAL, "the halo potential needs ndim = 3");
    if (d->flags & ~(PPML_FLAG_FIRST_ORDER | PPML_FLAG_ISOTHERMAL)) return fail(PPML_EINVAL, "unknown flags 0x%x", d->flags);
    if ((d->flags & PPML_FLAG_ISOTHERMAL) && !(d->iso_cs > 0.0 && std::isfinite(d->iso_cs)))
        return fail(PPML_EINVAL, "the isothermal variant needs iso_cs > 0");
    if (d->tile < 0 || d->tile >= NTILE[d->ndim])
        return fail(PPML_EINVAL, "tile %d out of range [0, %d) for ndim %d", d->tile, NTILE[d->ndim], d->ndim);
    if (d->self_gravity != 0 && d->self_gravity != 1) return fail(PPML_EINVAL, "self_gravity must be 0 or 1");
    if (d->self_gravity) {
        if (d->ndim != 3) return fail(PPML_EINVAL, "self-gravity needs ndim = 3");
        const double h0 = (d->hi[0] - d->lo[0]) / (double)d->n[0];
        for (int a = 1; a < 3; a++) {
            const double ha = (d->hi[a] - d->lo[a]) / (double)d->n[a];
            if (std::fabs(ha - h0) > 1e-12 * h0) return fail(PPML_EINVAL, "self-gravity needs cubic cells");
        }
        if (!(d->grav_G > 0.0) || !std::isfinite(d->grav_G)) return fail(PPML_EINVAL, "grav_G must be > 0");
        // the multipole expansion about the origin is undefined at the origin
        int on_grid = 1, on_shell = 0;
        for (int a = 0; a < 3; a++) {
            const double u = (0.0 - d->lo[a]) / h0 - 0.5;  // origin in cell units
            const double ur = std::nearbyint(u);
            if (std::fabs(u - ur) > 1e-9 || ur < -1.0 || ur > (double)d->n[a]) on_grid = 0;
            if (ur == -1.0 || ur == (double)d->n[a]) on_shell = 1;
        }
        if (on_grid && on_shell) return fail(PPML_EINVAL, "the origin (the multipole centre) is a shell cell centre");
    }
    return PPML_OK;
}

constexpr size_t ALIGN = 256;
size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

// Totals reduction: fixed number of blocks so the summation order is fixed.
int totals_blocks(long long n) { return (int)std::min<long long>(1024, (n + 4095) / 4096 > 0 ? (n + 4095) / 4096 : 1); }

struct ScratchLayout {
    size_t half, ctrl, partial, totals;
    // self-gravity: padded potential, two work arrays, sine matrices,
    // eigenvalue factors, moment partials, shell terms of the outer layer
    size_t phi, wx, wy, sx, sy, sz, fx, fy, fz, gpart, gedge;
    size_t total;
};

// Moment reduction of the self-gravity solve: fixed block count (fixed order).
int grav_blocks(long long n) { return (int)std::min<long long>(1024, (n + 2047) / 2048 > 0 ? (n + 2047) / 2048 : 1); }

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
    L.phi = L.wx = L.wy = L.sx = L.sy = L.sz = L.fx = L.fy = L.fz = L.gpart = L.gedge = 0;
    if (d->self_gravity) {
        const size_t e = elem(d);
        const size_t n0 = (size_t)d->n[0], n1 = (size_t)d->n[1], n2 = (size_t)d->n[2];
        L.phi = sz;
        sz += align_up((n0 + 2) * (n1 + 2) * (n2 + 2) * e);
        L.wx = sz;
        sz += align_up(n0 * n1 * n2 * e);
        L.wy = sz;
        sz += align_up(n0 * n1 * n2 * e);
        L.sx = sz;
        sz += align_up(n0 * n0 * e);
        L.sy = sz;
        sz += align_up(n1 * n1 * e);
        L.sz = sz;
        sz += align_up(n2 * n2 * e);
        L.fx = sz;
        sz += align_up(n0 * sizeof(double));
        L.fy = sz;
        sz += align_up(n1 * sizeof(double));
        L.fz = sz;
        sz += align_up(n2 * sizeof(double));
        L.gpart = sz;
        sz += align_up((size_t)grav_blocks(ncells(d)) * GRAV_MOM * sizeof(double));
        L.gedge = sz;
        sz += align_up((size_t)grav_edge_cells(d->n[0], d->n[1], d->n[2]) * e);
    }
    L.total = sz;
    return L;
}

}  // namespace

struct ppml_grid {
    ppml_desc d;
    GridParams gp;         // batch launches and the per-cell kernels
    GridParams gpE, gpL;   // solo launches of the two stage kernels (own z chunks)
    hipStream_t stream;
    int device;
    void *state;
    void *half;
    Ctrl *ctrl;
    double *partial;
    double *totals;
    bool in_batch;         // admitted to a batch: stepped only by the batch
    hipStream_t bstream;   // that batch's stream (the batch kernels write the state there)
    bool has_state;
    std::vector<hipEvent_t> ev;  // 4 events per timed step
    long long timed;             // steps recorded since the last read
    // self-gravity (Sec. 2.5)
    rocblas_handle blas;
    void *phi, *wx, *wy, *sx, *sy, *sz, *gedge;
    double *fx, *fy, *fz, *gpart;
    double grav_coef;      // 4 pi G h^2
    double grav_norm;      // prod_a 2 / (n_a + 1)
    // a captured chunk of STEP_GRAPH steps, replayed by long ppml_step calls
    hipGraphExec_t sexec;
    bool graph_off;        // capture failed once: launch eagerly
};

namespace {

template <typename T> void launch_speeds(ppml_grid *g)
{
    const T *U = (const T *)g->state;
    int nb = (int)std::min<long long>(4096, (g->gp.ncell + 255) / 256);
    switch (g->d.ndim) {
    case 1: k_speeds<T, 1><<<nb, 256, 0, g->stream>>>(U, g->gp, g->ctrl); break;
    case 2: k_speeds<T, 2><<<nb, 256, 0, g->stream>>>(U, g->gp, g->ctrl); break;
    default: k_speeds<T, 3><<<nb, 256, 0, g->stream>>>(U, g->gp, g->ctrl); break;
    }
}

template <typename T, int NDIM> void launch_stages(ppml_grid *g, hipEvent_t *ev)
{
    const T *U = (const T *)g->state;
    T *Us = (T *)g->state;
    T *W = (T *)g->half;
    with_tile<NDIM>(g->d.tile, [&](auto tl) {
        using TL = decltype(tl);
        const GridParams &ge = g->gpE;
        const GridParams &gl = g->gpL;
        const int nbe = ge.tiles[0] * ge.tiles[1] * ge.tiles[2];
        const int nbl = gl.tiles[0] * gl.tiles[1] * gl.tiles[2];
        if (ev) (void)hipEventRecord(ev[1], g->stream);
        if constexpr (NDIM == 3) {
            if (ge.potential == POT_HALO)
                k_euler<T, 3, TL::tx, TL::ty, 2><<<nbe, TL::nt, 0, g->stream>>>(U, W, ge, g->ctrl);
            else if (ge.self_grav)
                k_euler<T, 3, TL::tx, TL::ty, 1><<<nbe, TL::nt, 0, g->stream>>>(U, W, ge, g->ctrl);
            else
                k_euler<T, 3, TL::tx, TL::ty><<<nbe, TL::nt, 0, g->stream>>>(U, W, ge, g->ctrl);
        } else {
            k_euler<T, NDIM, TL::tx, TL::ty><<<nbe, TL::nt, 0, g->stream>>>(U, W, ge, g->ctrl);
        }
        if (ev) (void)hipEventRecord(ev[2], g->stream);
        k_lagr<T, NDIM, TL::tx, TL::ty, LG<T>::g><<<nbl, TL::nt, 0, g->stream>>>(W, Us, gl, g->ctrl);
        if (ev) (void)hipEventRecord(ev[3], g->stream);
    });
}

// GEMMs of the sine transforms (column-major view of the C-order arrays:
// a matrix with leading dimension n0 has the x index as its row).
rocblas_status gemm(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, int m, int n, int k, const float *A,
                    int lda, long long sa, const float *B, int ldb, long long sb, float *C, int ldc, long long sc,
                    int batch)
{
    const float one = 1.0f, zero = 0.0f;
    if (batch == 1) return rocblas_sgemm(h, ta, tb, m, n, k, &one, A, lda, B, ldb, &zero, C, ldc);
    return rocblas_sgemm_strided_batched(h, ta, tb, m, n, k, &one, A, lda, sa, B, ldb, sb, &zero, C, ldc, sc, batch);
}

rocblas_status gemm(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, int m, int n, int k,
                    const double *A, int lda, long long sa, const double *B, int ldb, long long sb, double *C, int ldc,
                    long long sc, int batch)
{
    const double one = 1.0, zero = 0.0;
    if (batch == 1) return rocblas_dgemm(h, ta, tb, m, n, k, &one, A, lda, B, ldb, &zero, C, ldc);
    return rocblas_dgemm_strided_batched(h, ta, tb, m, n, k, &one, A, lda, sa, B, ldb, sb, &zero, C, ldc, sc, batch);
}

// Sine transform of every line of one axis, on data in (sum | difference)
// slots along that axis: the odd modes are So times the sums, the even
// modes Se times the differences (forward); back, the sums are So^T times
// the odd modes and the differences Se^T times the even modes.  Column-major
// views of the C-order arrays: x as rows (C = op(S) A over the n1 n2
// columns), y per plane (C_k = A_k op(S)^T, a strided batch over the n2
// planes), z as columns (C = A op(S)^T over the n0 n1 rows).
template <typename T> int sine_transform(ppml_grid *g, int axis, bool inverse, const T *A, T *C)
{
    const int n[3] = {g->gp.n[0], g->gp.n[1], g->gp.n[2]};
    const int na = n[axis];
    const int no = grav_no(na), ne = grav_ne(na);
    const T *S = (const T *)(axis == 0 ? g->sx : axis == 1 ? g->sy : g->sz);
    const rocblas_operation N_ = rocblas_operation_none, T_ = rocblas_operation_transpose;
    const long long plane = (long long)n[0] * n[1];
    for (int half = 0; half < 2; half++) {
        const int m = half ? ne : no;             // slots of this half
        if (m == 0) continue;
        const T *Sh = S + (half ? (long long)no * no : 0);  // m x m, column major
        const long long off = half ? no : 0;      // first slot of the half
        rocblas_status st;
        if (axis == 0)
            st = gemm(g->blas, inverse ? T_ : N_, N_, m, n[1] * n[2], m, Sh, m, 0, A + off, n[0], 0, C + off, n[0], 0,
                      1);
        else if (axis == 1)
            st = gemm(g->blas, N_, inverse ? N_ : T_, n[0], m, m, A + off * n[0], n[0], plane, Sh, m, 0,
                      C + off * n[0], n[0], plane, n[2]);
        else
            st = gemm(g->blas, N_, inverse ? N_ : T_, (int)plane, m, m, A + off * plane, (int)plane, 0, Sh, m, 0,
                      C + off * plane, (int)plane, 0, 1);
        if (st != rocblas_status_success)
            return fail(PPML_EHIP, "rocBLAS GEMM of the sine transform: status %d", (int)st);
    }
    return PPML_OK;
}

// The self-gravity potential of the current state into g->phi (Sec. 2.5).
template <typename T> int launch_gravity(ppml_grid *g)
{
    const GridParams &gp = g->gp;
    const long long N = gp.ncell;
    const int n0 = gp.n[0], n1 = gp.n[1], n2 = gp.n[2];
    const T *rho = (const T *)g->state;
    T *phi = (T *)g->phi;
    T *X = (T *)g->wx;
    T *Y = (T *)g->wy;
    const int rows = n1 * n2;
    const int nb = grav_blocks(N);
    const int chunk = (rows + nb - 1) / nb;
    k_grav_moments_partial<T><<<nb, GRAV_THREADS, 0, g->stream>>>(rho, gp, chunk, g->gpart);
    k_grav_moments_final<<<1, GRAV_THREADS, 0, g->stream>>>(g->gpart, nb, g->ctrl);
    const long long nshell = (long long)(n0 + 2) * (n1 + 2) * (n2 + 2) - N;
    k_grav_shell<T><<<(unsigned)((nshell + 255) / 256), 256, 0, g->stream>>>(gp, g->ctrl, g->d.grav_G, phi);
    // shell terms of the outer layer, then the right-hand side's sums and
    // differences into Y
    T *E = (T *)g->gedge;
    const long long nedge = grav_edge_cells(n0, n1, n2);
    k_grav_edge_terms<T><<<(unsigned)((nedge + 255) / 256), 256, 0, g->stream>>>(phi, gp, E);
    const long long nrep = (long long)grav_no(n0) * grav_no(n1) * grav_no(n2);
    const unsigned nbr = (unsigned)((nrep + 255) / 256);
    k_grav_butterfly<T><<<nbr, 256, 0, g->stream>>>(rho, E, g->grav_coef, Y, gp);
    HIPCHK(hipGetLastError());
    int rc;
    if ((rc = sine_transform<T>(g, 0, false, Y, X))) return rc;
    if ((rc = sine_transform<T>(g, 1, false, X, Y))) return rc;
    if ((rc = sine_transform<T>(g, 2, false, Y, X))) return rc;
    const dim3 ged((unsigned)((n0 + 255) / 256), (unsigned)std::min((rows + 3) / 4, 4096));
    k_grav_eigdiv<T><<<ged, 256, 0, g->stream>>>(X, g->fx, g->fy, g->fz, gp, g->grav_norm);
    HIPCHK(hipGetLastError());
    if ((rc = sine_transform<T>(g, 2, true, X, Y))) return rc;
    if ((rc = sine_transform<T>(g, 1, true, Y, X))) return rc;
    if ((rc = sine_transform<T>(g, 0, true, X, Y))) return rc;
    k_grav_unbutterfly<T><<<nbr, 256, 0, g->stream>>>(Y, phi, gp);
    HIPCHK(hipGetLastError());
    return PPML_OK;
}

template <typename T> int launch_step(ppml_grid *g, hipEvent_t *ev)
{
    // ev (may be NULL): events recorded before the gravity solve, before,
    // between and after the stage kernels
    if (ev) (void)hipEventRecord(ev[0], g->stream);
    if (g->gp.self_grav) {
        int rc = launch_gravity<T>(g);
        if (rc) return rc;
    }
    switch (g->d.ndim) {
    case 1: launch_stages<T, 1>(g, ev); break;
    case 2: launch_stages<T, 2>(g, ev); break;
    default: launch_stages<T, 3>(g, ev); break;
    }
    return PPML_OK;
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

// A grid in a batch is stepped on the batch's stream: calls that touch its
// state on the grid's own stream first wait for the batch's queued work.
int settle(ppml_grid *g)
{
    if (g->in_batch && g->bstream != g->stream) HIPCHK(hipStreamSynchronize(g->bstream));
    return PPML_OK;
}

// After the state is set: reset the control block, record the mean density
// (the given one, or the mean of the state when rho_mean0 <= 0), compute the
// CFL maxima of the state into slot 0.  Kernels only: nothing is copied from
// the host.
int finish_set_async(ppml_grid *g, double t, double rho_mean0)
{
    k_ctrl_reset<<<1, 1, 0, g->stream>>>(g->ctrl, t, rho_mean0);
    HIPCHK(hipGetLastError());
    if (g->d.prec == PPML_FP64) {
        launch_totals<double>(g, rho_mean0 > 0.0 ? 0.0 : (double)g->gp.ncell);
        launch_speeds<double>(g);
    } else {
        launch_totals<float>(g, rho_mean0 > 0.0 ? 0.0 : (double)g->gp.ncell);
        launch_speeds<float>(g);
    }
    HIPCHK(hipGetLastError());
    g->has_state = true;
    return PPML_OK;
}

int finish_set(ppml_grid *g, double t, double rho_mean0)
{
    int rc = finish_set_async(g, t, rho_mean0);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(g->stream));
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

// Number of z chunks of a 3-D stage launch.  A work group streams cz planes
// after `warm` planes of pipeline start-up (in units of a full plane); the
// launch runs in ceil(groups / slots) rounds of resident work groups, so the
// time is modelled as rounds * (cz + warm) and minimised over the chunk count.
int choose_chunks(long long tiles_xy, int nz, long long slots, double warm)
{
    if (slots < 1) slots = 1;
    int best = 1;
    double best_cost = 1e300;
    for (int c = 1; c <= nz; c++) {
        const int cz = (nz + c - 1) / c;
        if ((long long)(c - 1) * cz >= nz) continue;  // same chunks as a smaller count
        const long long groups = tiles_xy * c;
        if (groups > (1ll << 30)) break;
        const double rounds = (double)((groups + slots - 1) / slots);
        const double cost = rounds * (cz + warm);
        if (cost < best_cost * (1.0 - 1e-9)) {
            best_cost = cost;
            best = c;
        }
    }
    return best;
}

template <typename T> void stage_slots(int device, int tile, int xf, long long &slots_e, long long &slots_l)
{
    int cus = 0, be = 0, bl = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) cus = 0;
    with_tile<3>(tile, [&](auto tl) {
        using TL = decltype(tl);
        hipError_t e =
            xf == 2   ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&be, k_euler<T, 3, TL::tx, TL::ty, 2>, TL::nt, 0)
            : xf == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&be, k_euler<T, 3, TL::tx, TL::ty, 1>, TL::nt, 0)
                      : hipOccupancyMaxActiveBlocksPerMultiprocessor(&be, k_euler<T, 3, TL::tx, TL::ty>, TL::nt, 0);
        if (e != hipSuccess) be = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&bl, k_lagr<T, 3, TL::tx, TL::ty, LG<T>::g>, TL::nt, 0) !=
            hipSuccess)
            bl = 0;
    });
    (void)hipGetLastError();
    if (cus < 1) cus = 256;
    slots_e = (long long)cus * (be > 0 ? be : 2);
    slots_l = (long long)cus * (bl > 0 ? bl : 2);
}

// Work-group tiling of a grid for tile shape v: x/y tiles, and a z chunk
// small enough that a 3-D grid alone gives the launch a few thousand work
// groups (batches then fit the chunks of their 3-D grids together).
void set_tiling(GridParams &gp, int ndim, int v)
{
    const int tx = TILE_X[ndim][v], ty = TILE_Y[ndim][v];
    gp.tiles[0] = (gp.n[0] + tx - 1) / tx;
    gp.tiles[1] = ndim >= 2 ? (gp.n[1] + ty - 1) / ty : 1;
    gp.tiles[2] = 1;
    gp.cz = 1;
    if (ndim == 3) {
        long long tiles = (long long)gp.tiles[0] * gp.tiles[1];
        int cz = gp.n[2];
        while (cz > 16 && tiles * ((gp.n[2] + cz - 1) / cz) < 2048) cz = (cz + 1) / 2;
        gp.cz = cz;
        gp.tiles[2] = (gp.n[2] + cz - 1) / cz;
    }
}

void set_chunks(GridParams &gp, int chunks)
{
    const int nz = gp.n[2];
    gp.cz = (nz + chunks - 1) / chunks;
    gp.tiles[2] = (nz + gp.cz - 1) / gp.cz;
}

// Z chunks shared by the 3-D grids of a batch: every work group of the launch
// streams at most cz planes after its start-up (`warm`, in plane units).  With
// the groups' work spread over the resident slots, the launch takes about
// max(sum of the groups' lengths / slots, the longest group); cz minimises
// that over all the batch's grids at once, where chunks chosen per grid as if
// it ran alone cut every grid into short chunks whose start-up dominates.
int batch_cz3(const std::vector<GridParams *> &gps, long long slots, double warm)
{
    int nzmax = 1;
    for (const GridParams *gp : gps) nzmax = gp->n[2] > nzmax ? gp->n[2] : nzmax;
    if (slots < 1) slots = 1;
    int best = nzmax;
    double best_t = 1e300;
    for (int c = 1; c <= nzmax; c++) {
        const int cz = (nzmax + c - 1) / c;
        if ((long long)(c - 1) * cz >= nzmax) continue;  // same cz as a smaller count
        double work = 0.0, longest = 0.0;
        for (const GridParams *gp : gps) {
            const int nz = gp->n[2];
            const int ch = (nz + cz - 1) / cz;
            const int czg = (nz + ch - 1) / ch;
            work += (double)gp->tiles[0] * gp->tiles[1] * ch * (czg + warm);
            longest = czg + warm > longest ? czg + warm : longest;
        }
        const double t = work / (double)slots > longest ? work / (double)slots : longest;
        if (t < best_t * (1.0 - 1e-9)) {
            best_t = t;
            best = cz;
        }
    }
    return best;
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

}  // extern "C"

namespace {

// Grid parameters, pointers into the scratch area and the inflow ghost states
// of a validated descriptor (everything of ppml_create but the self-gravity
// set-up and the z chunks).  Allocates nothing: g is the caller's object.
int init_grid(ppml_grid *g, const ppml_desc *d, void *state_dev, void *scratch_dev, void *hip_stream)
{
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
    if (d->flags & PPML_FLAG_ISOTHERMAL) {
        gp.pa = d->iso_cs * d->iso_cs;
        gp.pb = 0.0;
        gp.gs = 1.0;
    } else {
        gp.pa = 0.0;
        gp.pb = d->gamma - 1.0;
        gp.gs = d->gamma;
    }
    gp.cfl_hmin = d->cfl * hmin;
    gp.vacuum_ratio = (d->flags & PPML_FLAG_ISOTHERMAL) ? 0.0 : d->vacuum_ratio;
    gp.potential = d->potential;
    gp.first_order = (d->flags & PPML_FLAG_FIRST_ORDER) ? 1 : 0;
    for (int i = 0; i < 8; i++) gp.pot[i] = d->pot[i];
    set_tiling(gp, d->ndim, d->tile);
    // conserved ghost states of inflow faces, converted in FP64 as the state
    // is, into the control block
    double tab[6][6];
    memset(tab, 0, sizeof tab);
    gp.any_inflow = 0;
    for (int a = 0; a < d->ndim; a++)
        for (int s = 0; s < 2; s++) {
            if ((s ? d->bc_hi[a] : d->bc_lo[a]) != PPML_INFLOW) continue;
            const double *st = d->inflow[2 * a + s];
            const double r = st[0];
            const double ux = st[1];
            const double uy = d->ndim >= 2 ? st[2] : 0.0;
            const double uz = d->ndim >= 3 ? st[3] : 0.0;
            const double e = st[4] / (d->gamma - 1.0);
            const double ke = 0.5 * r * (ux * ux + uy * uy + uz * uz);
            double *c = tab[2 * a + s];
            c[0] = r;
            c[1] = r * ux;
            c[2] = r * uy;
            c[3] = r * uz;
            c[4] = e + ke;
            c[5] = e;
            gp.any_inflow = 1;
        }
    if (gp.any_inflow) {
        InflowTable it;
        memcpy(it.v, tab, sizeof tab);
        k_set_inflow<<<1, 64, 0, g->stream>>>(g->ctrl, it);
        HIPCHK(hipGetLastError());
    }
    g->blas = nullptr;
    g->sexec = nullptr;
    g->graph_off = false;
    g->phi = g->wx = g->wy = g->sx = g->sy = g->sz = g->gedge = nullptr;
    g->fx = g->fy = g->fz = g->gpart = nullptr;
    g->has_state = false;
    g->in_batch = false;
    g->bstream = nullptr;
    g->timed = 0;
    return PPML_OK;
}

// Z chunks of the solo stage launches, fitted to the resident work groups of
// each stage kernel (start-up cost: 3 z-only planes in the Eulerian kernel, 6
// in the Lagrangian kernel).  After the self-gravity set-up, which selects
// the Eulerian instantiation.
void init_chunks(ppml_grid *g)
{
    const GridParams &gp = g->gp;
    const ppml_desc *d = &g->d;
    g->gpE = gp;
    g->gpL = gp;
    if (d->ndim == 3) {
        long long se, sl;
        const int xf = gp.potential == POT_HALO ? 2 : (gp.self_grav ? 1 : 0);
        if (d->prec == PPML_FP64) stage_slots<double>(g->device, d->tile, xf, se, sl);
        else stage_slots<float>(g->device, d->tile, xf, se, sl);
        const long long txy = (long long)gp.tiles[0] * gp.tiles[1];
        set_chunks(g->gpE, choose_chunks(txy, gp.n[2], se, 1.5));
        set_chunks(g->gpL, choose_chunks(txy, gp.n[2], sl, 3.0));
    }
}

}  // namespace

extern "C" {

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
    if ((rc = init_grid(g, d, state_dev, scratch_dev, hip_stream))) {
        delete g;
        return rc;
    }
    GridParams &gp = g->gp;
    const ScratchLayout L = layout(d);
    char *s = (char *)scratch_dev;
    if (d->self_gravity) {
        g->phi = s + L.phi;
        g->wx = s + L.wx;
        g->wy = s + L.wy;
        g->sx = s + L.sx;
        g->sy = s + L.sy;
        g->sz = s + L.sz;
        g->fx = (double *)(s + L.fx);
        g->fy = (double *)(s + L.fy);
        g->fz = (double *)(s + L.fz);
        g->gpart = (double *)(s + L.gpart);
        g->gedge = s + L.gedge;
        gp.self_grav = 1;
        gp.phi = g->phi;
        const double h = gp.h[0];
        g->grav_coef = 4.0 * M_PI * d->grav_G * h * h;
        g->grav_norm = (2.0 / (double)(gp.n[0] + 1)) * (2.0 / (double)(gp.n[1] + 1)) * (2.0 / (double)(gp.n[2] + 1));
        if (rocblas_create_handle(&g->blas) != rocblas_status_success) {
            delete g;
            return fail(PPML_EHIP, "rocblas_create_handle failed");
        }
        if (rocblas_set_stream(g->blas, g->stream) != rocblas_status_success) {
            rocblas_destroy_handle(g->blas);
            delete g;
            return fail(PPML_EHIP, "rocblas_set_stream failed");
        }
        const long long nt = grav_table_count(gp.n[0]) + grav_table_count(gp.n[1]) + grav_table_count(gp.n[2]);
        const unsigned nbt = (unsigned)((nt + 255) / 256);
        if (d->prec == PPML_FP64)
            k_grav_tables<double><<<nbt, 256, 0, g->stream>>>((double *)g->sx, (double *)g->sy, (double *)g->sz,
                                                               g->fx, g->fy, g->fz, gp.n[0], gp.n[1], gp.n[2]);
        else
            k_grav_tables<float><<<nbt, 256, 0, g->stream>>>((float *)g->sx, (float *)g->sy, (float *)g->sz, g->fx,
                                                              g->fy, g->fz, gp.n[0], gp.n[1], gp.n[2]);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
        if (e != hipSuccess) {
            rocblas_destroy_handle(g->blas);
            delete g;
            return fail(PPML_EHIP, "self-gravity tables: %s", hipGetErrorString(e));
        }
    }
    init_chunks(g);
    *out = g;
    return PPML_OK;
}

int ppml_set_primitive(ppml_grid *g, const double *rho, const double *vx, const double *vy, const double *vz,
                       const double *p)
{
    int rc = grid_ok(g);
    if (rc) return rc;
    if ((rc = settle(g))) return rc;
    if (!rho || !p) return fail(PPML_EINVAL, "rho and p are required");
    const long long N = g->gp.ncell;
    if (!all_finite_positive(rho, N)) return fail(PPML_EINVAL, "rho must be finite and > 0");
    if (!all_finite_positive(p, N)) return fail(PPML_EINVAL, "p must be finite and > 0");
    const double *v[3] = {vx, vy, vz};
    for (int a = 0; a < g->d.ndim; a++)
        if (v[a] && !all_finite(v[a], N)) return fail(PPML_EINVAL, "velocity %d has non-finite values", a);
    double *prim = nullptr;
    HIPCHK(hipMallocAsync((void **)&prim, (size_t)5 * N * sizeof(double), g->stream));
    const double *src[5] = {rho, vx, vy, vz, p};
    for (int i = 0; i < 5; i++) {
        if (src[i]) {
            hipError_t e = hipMemcpyAsync(prim + (size_t)i * N, src[i], N * sizeof(double), hipMemcpyHostToDevice,
                                          g->stream);
            if (e != hipSuccess) {
                (void)hipFreeAsync(prim, g->stream);
                return fail(PPML_EHIP, "copy of primitive %d: %s", i, hipGetErrorString(e));
            }
        } else {
            hipError_t e = hipMemsetAsync(prim + (size_t)i * N, 0, N * sizeof(double), g->stream);
            if (e != hipSuccess) {
                (void)hipFreeAsync(prim, g->stream);
                return fail(PPML_EHIP, "hipMemsetAsync: %s", hipGetErrorString(e));
            }
        }
    }
    int nb = (int)std::min<long long>(4096, (N + 255) / 256);
    if (g->d.prec == PPML_FP64) k_prim_to_cons<double><<<nb, 256, 0, g->stream>>>(prim, (double *)g->state, g->gp);
    else k_prim_to_cons<float><<<nb, 256, 0, g->stream>>>(prim, (float *)g->state, g->gp);
    hipError_t e = hipGetLastError();
    (void)hipFreeAsync(prim, g->stream);
    hipError_t e2 = hipStreamSynchronize(g->stream);
    if (e != hipSuccess || e2 != hipSuccess)
        return fail(PPML_EHIP, "prim_to_cons: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    return finish_set(g, 0.0, 0.0);
}

int ppml_set_conserved(ppml_grid *g, const double *const *f, double rho_mean0, double t)
{
    int rc = grid_ok(g);
    if (rc) return rc;
    if ((rc = settle(g))) return rc;
    if (!f || !f[PPML_RHO] || !f[PPML_ETOT] || !f[PPML_EINT]) return fail(PPML_EINVAL, "rho, Et and e are required");
    const long long N = g->gp.ncell;
    const int nd = g->d.ndim;
    if (!all_finite_positive(f[PPML_RHO], N)) return fail(PPML_EINVAL, "rho must be finite and > 0");
    if (!all_finite_positive(f[PPML_EINT], N)) return fail(PPML_EINVAL, "rho*eps must be finite and > 0");
    if (!all_finite(f[PPML_ETOT], N)) return fail(PPML_EINVAL, "rho*E must be finite");
    if (!std::isfinite(t) || t < 0.0) return fail(PPML_EINVAL, "t must be finite and >= 0");
    double *tmp = nullptr;
    HIPCHK(hipMallocAsync((void **)&tmp, (size_t)N * sizeof(double), g->stream));
    int nb = (int)std::min<long long>(4096, (N + 255) / 256);
    // stored field s <- ppml_field
    int nfs = nfields(&g->d);
    for (int s = 0; s < nfs; s++) {
        int fld = s == 0 ? PPML_RHO : (s <= nd ? s : (s == nd + 1 ? PPML_ETOT : PPML_EINT));
        hipError_t e;
        if (f[fld]) {
            if (!all_finite(f[fld], N)) {
                (void)hipFreeAsync(tmp, g->stream);
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
            (void)hipFreeAsync(tmp, g->stream);
            return fail(PPML_EHIP, "set_conserved: %s", hipGetErrorString(e));
        }
    }
    (void)hipFreeAsync(tmp, g->stream);
    return finish_set(g, t, rho_mean0);
}

namespace {

// Steps per captured graph of a solo grid.  Every step reads its time step
// and run limits from the control block, so one graph of STEP_GRAPH steps
// serves any call; steps past the run's end are no-ops.
constexpr int STEP_GRAPH = 32;

// Capture STEP_GRAPH steps of the grid into g->sexec (once).  The launches
// are captured on a private non-blocking stream (the grid's own stream may be
// the null stream, which cannot be captured); the graph is then launched on
// the grid's stream, in order with the rest of its work.  False if capture
// fails; the caller then launches eagerly.
bool step_graph(ppml_grid *g)
{
    if (g->sexec) return true;
    if (g->graph_off) return false;
    g->graph_off = true;  // until the capture below succeeds
    // capture on the grid's device, whichever device is current
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != g->device && hipSetDevice(g->device) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    hipStream_t cap = nullptr;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        if (prev >= 0 && prev != g->device) (void)hipSetDevice(prev);
        return false;
    }
    hipGraph_t gr = nullptr;
    hipGraphExec_t ex = nullptr;
    bool ok = false;
    const hipStream_t own = g->stream;
    if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) == hipSuccess) {
        g->stream = cap;
        int rc = PPML_OK;
        for (int s = 0; s < STEP_GRAPH && rc == PPML_OK; s++)
            rc = g->d.prec == PPML_FP64 ? launch_step<double>(g, nullptr) : launch_step<float>(g, nullptr);
        g->stream = own;
        const hipError_t e = hipStreamEndCapture(cap, &gr);
        ok = rc == PPML_OK && e == hipSuccess && gr && hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0) == hipSuccess;
    }
    if (gr) (void)hipGraphDestroy(gr);
    (void)hipStreamDestroy(cap);
    (void)hipGetLastError();
    if (prev >= 0 && prev != g->device) (void)hipSetDevice(prev);
    if (!ok) {
        if (ex) (void)hipGraphExecDestroy(ex);
        return false;
    }
    g->sexec = ex;
    g->graph_off = false;
    return true;
}

}  // namespace

int ppml_step(ppml_grid *g, int32_t nsteps, double dt_fixed, double t_stop)
{
    int rc = grid_ok(g);
    if (rc) return rc;
    if (nsteps < 0) return fail(PPML_EINVAL, "nsteps must be >= 0");
    if (!g->has_state) return fail(PPML_ESTATE, "state was never set");
    if (!std::isfinite(dt_fixed) || !std::isfinite(t_stop)) return fail(PPML_EINVAL, "dt_fixed and t_stop must be finite");
    if (nsteps == 0) return PPML_OK;
    if (g->in_batch) return fail(PPML_ESTATE, "grid is stepped by its batch");
    k_set_run<<<1, 1, 0, g->stream>>>(g->ctrl, dt_fixed, t_stop, (long long)nsteps);
    HIPCHK(hipGetLastError());  // before a capture attempt clears the last error
    // long calls replay the captured chunk (launch overhead once per
    // STEP_GRAPH steps); not while per-step timing is recorded, nor with
    // self-gravity (its library GEMMs stay outside captured graphs)
    const bool timing = (size_t)(4 * (g->timed + 1)) <= g->ev.size();
    int s = 0;
    if (nsteps >= STEP_GRAPH && !timing && !g->gp.self_grav && step_graph(g)) {
        for (; s + STEP_GRAPH <= nsteps; s += STEP_GRAPH) HIPCHK(hipGraphLaunch(g->sexec, g->stream));
    }
    for (; s < nsteps; s++) {
        hipEvent_t *ev = nullptr;
        if ((size_t)(4 * (g->timed + 1)) <= g->ev.size()) ev = &g->ev[4 * g->timed];
        rc = g->d.prec == PPML_FP64 ? launch_step<double>(g, ev) : launch_step<float>(g, ev);
        if (rc) return rc;
        if (ev) g->timed++;
    }
    HIPCHK(hipGetLastError());
    return PPML_OK;
}

}  // extern "C"

// Work area of ppml_step_noalloc: the Eulerian-stage output, the control block
// and the totals partials of one grid, one copy per GPU the library runs on,
// held until the process ends.  Host code never passes the array's name to a
// kernel or a copy (in host code it is only a stand-in for the device
// symbol): its device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[PPML_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int NOALLOC_MAX_DEV = 64;
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[NOALLOC_MAX_DEV];

// Device address of the work area on the current device (looked up on the
// first call on that device, with the device current).
int noalloc_area(int device, void **out)
{
    if (device < 0 || device >= NOALLOC_MAX_DEV) return fail(PPML_EINVAL, "device %d out of range", device);
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(PPML_EHIP, "hipGetSymbolAddress of the work area: %s", hipGetErrorString(e));
        g_noalloc_ptr[device] = ptr;
    }
    *out = g_noalloc_ptr[device];
    return PPML_OK;
}

}  // namespace

extern "C" {

int ppml_step_noalloc(const ppml_desc *d, void *state_dev, double rho_mean0, double t0, int32_t nsteps,
                      double dt_fixed, double t_stop, void *hip_stream, double *t_out, int64_t *steps_out)
{
    int rc = validate(d);
    if (rc != PPML_OK) return rc;
    if (d->self_gravity) return fail(PPML_EINVAL, "self-gravity grids step through ppml_create / ppml_step");
    if (!state_dev) return fail(PPML_EINVAL, "state pointer must be non-NULL");
    if ((uintptr_t)state_dev % ALIGN) return fail(PPML_EINVAL, "the state pointer must be %zu-byte aligned", ALIGN);
    if (nsteps < 0) return fail(PPML_EINVAL, "nsteps must be >= 0");
    if (!std::isfinite(dt_fixed) || !std::isfinite(t_stop) || !std::isfinite(rho_mean0))
        return fail(PPML_EINVAL, "dt_fixed, t_stop and rho_mean0 must be finite");
    if (!std::isfinite(t0) || t0 < 0.0) return fail(PPML_EINVAL, "t0 must be finite and >= 0");
    const size_t need = layout(d).total;
    if (need > (size_t)PPML_NOALLOC_SCRATCH_BYTES)
        return fail(PPML_EINVAL, "the grid needs %zu bytes of work area; the fixed area holds %zu", need,
                    (size_t)PPML_NOALLOC_SCRATCH_BYTES);
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    void *area = nullptr;
    if ((rc = noalloc_area(dev, &area))) return rc;
    ppml_grid g{};  // on the stack: no host allocation
    if ((rc = init_grid(&g, d, state_dev, area, hip_stream))) return rc;
    init_chunks(&g);
    // every value of the work area that a step reads is written first: the
    // control block by the reset, the maxima slots, the mean density and the
    // partials by the kernels below, the stage output by the Eulerian kernel
    if ((rc = finish_set_async(&g, t0, rho_mean0))) return rc;
    if (nsteps > 0) {
        k_set_run<<<1, 1, 0, g.stream>>>(g.ctrl, dt_fixed, t_stop, (long long)nsteps);
        HIPCHK(hipGetLastError());
        for (int s = 0; s < nsteps; s++) {
            rc = d->prec == PPML_FP64 ? launch_step<double>(&g, nullptr) : launch_step<float>(&g, nullptr);
            if (rc) return rc;
        }
    }
    HIPCHK(hipGetLastError());
    if (t_out || steps_out) {
        Ctrl c;
        HIPCHK(hipMemcpyAsync(&c, g.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, g.stream));
        HIPCHK(hipStreamSynchronize(g.stream));
        if (t_out) *t_out = c.t;
        if (steps_out) *steps_out = c.steps;
        if (c.err) return fail(PPML_ENONFINITE, "a step produced rho <= 0, eps <= 0 or a non-finite value");
    }
    return PPML_OK;
}

int ppml_get_time(ppml_grid *g, double *t, double *dt_last, int64_t *steps)
{
    int rc = grid_ok(g);
    if (rc) return rc;
    if ((rc = settle(g))) return rc;
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
    if ((rc = settle(g))) return rc;
    Ctrl c;
    HIPCHK(hipMemcpyAsync(&c, g->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
    int slot = c.slot_cur;
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
    if ((rc = settle(g))) return rc;
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
    HIPCHK(hipMallocAsync((void **)&tmp, (size_t)N * sizeof(double), g->stream));
    int nb = (int)std::min<long long>(4096, (N + 255) / 256);
    if (g->d.prec == PPML_FP64)
        k_to_double<double><<<nb, 256, 0, g->stream>>>((const double *)g->state + (size_t)s * N, tmp, N);
    else
        k_to_double<float><<<nb, 256, 0, g->stream>>>((const float *)g->state + (size_t)s * N, tmp, N);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(host_out, tmp, N * sizeof(double), hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    (void)hipFreeAsync(tmp, g->stream);
    if (e != hipSuccess) return fail(PPML_EHIP, "get_conserved: %s", hipGetErrorString(e));
    return PPML_OK;
}

int ppml_totals(ppml_grid *g, double out[6])
{
    int rc = grid_ok(g);
    if (rc) return rc;
    if ((rc = settle(g))) return rc;
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
    if ((rc = settle(g))) return rc;
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
    for (int i = 0; i < 4 * cap; i++) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        g->ev.push_back(e);
    }
    return PPML_OK;
}

int ppml_get_timing_split(ppml_grid *g, double ms[3], int64_t *nsteps)
{
    int rc = grid_ok(g);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(g->stream));
    double acc[3] = {0.0, 0.0, 0.0};
    for (long long s = 0; s < g->timed; s++)
        for (int q = 0; q < 3; q++) {
            float a = 0.f;
            HIPCHK(hipEventElapsedTime(&a, g->ev[4 * s + q], g->ev[4 * s + q + 1]));
            acc[q] += a;
        }
    if (ms)
        for (int q = 0; q < 3; q++) ms[q] = acc[q];
    if (nsteps) *nsteps = g->timed;
    g->timed = 0;
    return PPML_OK;
}

int ppml_get_timing(ppml_grid *g, double *ms_euler, double *ms_lagr, int64_t *nsteps)
{
    double ms[3];
    int rc = ppml_get_timing_split(g, ms, nsteps);
    if (rc) return rc;
    if (ms_euler) *ms_euler = ms[1];
    if (ms_lagr) *ms_lagr = ms[2];
    return PPML_OK;
}

int ppml_get_potential(ppml_grid *g, double *host_out)
{
    int rc = grid_ok(g);
    if (rc) return rc;
    if (!host_out) return fail(PPML_EINVAL, "host_out is NULL");
    if (!g->gp.self_grav) return fail(PPML_EINVAL, "self-gravity is off for this grid");
    if (!g->has_state) return fail(PPML_ESTATE, "state was never set");
    if (g->in_batch) return fail(PPML_ESTATE, "grid is stepped by its batch");
    rc = g->d.prec == PPML_FP64 ? launch_gravity<double>(g) : launch_gravity<float>(g);
    if (rc) return rc;
    const long long np = (long long)(g->gp.n[0] + 2) * (g->gp.n[1] + 2) * (g->gp.n[2] + 2);
    double *tmp = nullptr;
    HIPCHK(hipMallocAsync((void **)&tmp, (size_t)np * sizeof(double), g->stream));
    int nb = (int)std::min<long long>(4096, (np + 255) / 256);
    if (g->d.prec == PPML_FP64) k_to_double<double><<<nb, 256, 0, g->stream>>>((const double *)g->phi, tmp, np);
    else k_to_double<float><<<nb, 256, 0, g->stream>>>((const float *)g->phi, tmp, np);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(host_out, tmp, np * sizeof(double), hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    (void)hipFreeAsync(tmp, g->stream);
    if (e != hipSuccess) return fail(PPML_EHIP, "get_potential: %s", hipGetErrorString(e));
    return PPML_OK;
}

int ppml_destroy(ppml_grid *g)
{
    if (!g) return fail(PPML_EINVAL, "grid is NULL");
    if (g->in_batch) return fail(PPML_ESTATE, "retire the grid from its batch first");
    (void)hipStreamSynchronize(g->stream);
    for (hipEvent_t e : g->ev) (void)hipEventDestroy(e);
    if (g->sexec) (void)hipGraphExecDestroy(g->sexec);
    if (g->blas) rocblas_destroy_handle(g->blas);
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

int ppml_tile_count(int32_t ndim)
{
    if (ndim < 1 || ndim > 3) return fail(PPML_EINVAL, "ndim must be 1, 2 or 3 (got %d)", ndim);
    return NTILE[ndim];
}

int ppml_tile_shape(int32_t ndim, int32_t variant, int32_t *tx, int32_t *ty)
{
    if (ndim < 1 || ndim > 3) return fail(PPML_EINVAL, "ndim must be 1, 2 or 3 (got %d)", ndim);
    if (variant < 0 || variant >= NTILE[ndim]) return fail(PPML_EINVAL, "tile %d out of range", variant);
    if (tx) *tx = TILE_X[ndim][variant];
    if (ty) *ty = TILE_Y[ndim][variant];
    return PPML_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------
struct ppml_batch {
    hipStream_t stream;
    int device;
    int capacity;
    size_t budget;   // 0: unlimited
    size_t in_use;   // state + scratch bytes of the admitted grids
    int prec;        // precision shared by all admitted grids (-1: none yet)
    std::vector<ppml_grid *> slots;
    BatchEntry *d_ents;   // device table, grouped by dimensionality
    int *d_steps;         // device per-entry step counts
    BatchEntry *h_ents;   // pinned host copies
    int *h_steps;
    std::vector<int> entry_slot;
    int goff[4], gn[4], gtiles[4];
    int tile[4];          // tile shape of the launches per dimensionality
    bool dirty;
    long long version;
    hipGraph_t graph;
    hipGraphExec_t exec;
    int graph_nsteps;
    long long graph_version;
    // grids of different dimensionalities share nothing: their launch chains
    // run as parallel branches (streams forked from and joined to the batch
    // stream, default priority), so the small 1-D launches overlap the 2-D
    // and 3-D ones instead of adding their dispatch time
    hipStream_t side[4];
    hipEvent_t ev_fork, ev_join[4];
};

namespace {

size_t grid_bytes(const ppml_grid *g) { return ppml_state_bytes(&g->d) + ppml_scratch_bytes(&g->d); }

int batch_rebuild(ppml_batch *b)
{
    int n = 0;
    b->entry_slot.clear();
    for (int nd = 1; nd <= 3; nd++) {
        b->goff[nd] = n;
        int tiles = 0;
        for (int s = 0; s < b->capacity; s++) {
            ppml_grid *g = b->slots[s];
            if (!g || g->d.ndim != nd) continue;
            BatchEntry &e = b->h_ents[n];
            e.gp = g->gp;
            set_tiling(e.gp, nd, b->tile[nd]);
            b->entry_slot.push_back(s);
            n++;
        }
        b->gn[nd] = n - b->goff[nd];
        if (nd == 3 && b->gn[3] > 0) {
            // one chunk length for all 3-D grids, fitted to the Lagrangian
            // kernel's resident work groups (its start-up: 6 z-only planes,
            // about 3 full ones)
            std::vector<GridParams *> gps;
            for (int i = b->goff[3]; i < n; i++) gps.push_back(&b->h_ents[i].gp);
            long long se, sl;
            if (b->prec == PPML_FP64) stage_slots<double>(b->device, b->tile[3], 0, se, sl);
            else stage_slots<float>(b->device, b->tile[3], 0, se, sl);
            const int cz = batch_cz3(gps, sl, 3.0);
            for (GridParams *gp : gps) set_chunks(*gp, (gp->n[2] + cz - 1) / cz);
        }
        for (int i = b->goff[nd]; i < n; i++) {
            BatchEntry &e = b->h_ents[i];
            const ppml_grid *g = b->slots[b->entry_slot[i]];
            e.state = g->state;
            e.half = g->half;
            e.ctrl = g->ctrl;
            e.tile0 = tiles;
            e.pad = 0;
            tiles += e.gp.tiles[0] * e.gp.tiles[1] * e.gp.tiles[2];
        }
        b->gtiles[nd] = tiles;
    }
    if (n > 0) {
        HIPCHK(hipMemcpyAsync(b->d_ents, b->h_ents, (size_t)n * sizeof(BatchEntry), hipMemcpyHostToDevice, b->stream));
        HIPCHK(hipStreamSynchronize(b->stream));
    }
    b->dirty = false;
    b->version++;
    return PPML_OK;
}

template <typename T, int NDIM> void batch_stage(ppml_batch *b, bool lagr, hipStream_t st)
{
    if (!b->gn[NDIM]) return;
    with_tile<NDIM>(b->tile[NDIM], [&](auto tl) {
        using TL = decltype(tl);
        const BatchEntry *e = b->d_ents + b->goff[NDIM];
        if (lagr)
            k_lagr_batch<T, NDIM, TL::tx, TL::ty, LG<T>::g><<<b->gtiles[NDIM], TL::nt, 0, st>>>(e, b->gn[NDIM]);
        else
            k_euler_batch<T, NDIM, TL::tx, TL::ty><<<b->gtiles[NDIM], TL::nt, 0, st>>>(e, b->gn[NDIM]);
    });
}

template <typename T, int NDIM> void batch_chain(ppml_batch *b, int nsteps, hipStream_t st)
{
    for (int s = 0; s < nsteps; s++) {
        batch_stage<T, NDIM>(b, false, st);
        batch_stage<T, NDIM>(b, true, st);
    }
}

// nsteps steps of every grid: one chain of stage launches per dimensionality
// present; with more than one, each chain runs on a side stream forked from
// the batch stream and joined back to it.
template <typename T> int batch_enqueue(ppml_batch *b, int nsteps)
{
    int present = 0;
    for (int nd = 1; nd <= 3; nd++) present += b->gn[nd] ? 1 : 0;
    const bool fork = present > 1;
    if (fork) HIPCHK(hipEventRecord(b->ev_fork, b->stream));
    for (int nd = 1; nd <= 3; nd++) {
        if (!b->gn[nd]) continue;
        hipStream_t st = fork ? b->side[nd] : b->stream;
        if (fork) HIPCHK(hipStreamWaitEvent(st, b->ev_fork, 0));
        if (nd == 1) batch_chain<T, 1>(b, nsteps, st);
        else if (nd == 2) batch_chain<T, 2>(b, nsteps, st);
        else batch_chain<T, 3>(b, nsteps, st);
        HIPCHK(hipGetLastError());
        if (fork) {
            HIPCHK(hipEventRecord(b->ev_join[nd], st));
            HIPCHK(hipStreamWaitEvent(b->stream, b->ev_join[nd], 0));
        }
    }
    return PPML_OK;
}

void batch_drop_graph(ppml_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_nsteps = -1;
}

}  // namespace

extern "C" {

int ppml_batch_create(int32_t capacity, size_t budget_bytes, void *hip_stream, ppml_batch **out)
{
    if (!out) return fail(PPML_EINVAL, "out is NULL");
    if (capacity < 1 || capacity > 65536) return fail(PPML_EINVAL, "capacity must be in [1, 65536]");
    int device = 0;
    HIPCHK(hipGetDevice(&device));
    ppml_batch *b = new (std::nothrow) ppml_batch();
    if (!b) return fail(PPML_ENOMEM, "host allocation failed");
    b->stream = (hipStream_t)hip_stream;
    b->device = device;
    b->capacity = capacity;
    b->budget = budget_bytes;
    b->in_use = 0;
    b->prec = -1;
    b->slots.assign(capacity, nullptr);
    b->d_ents = nullptr;
    b->d_steps = nullptr;
    b->h_ents = nullptr;
    b->h_steps = nullptr;
    b->dirty = true;
    for (int nd = 0; nd < 4; nd++) b->tile[nd] = 0;
    b->version = 0;
    b->graph = nullptr;
    b->exec = nullptr;
    b->graph_nsteps = -1;
    b->graph_version = -1;
    for (int nd = 0; nd < 4; nd++) {
        b->side[nd] = nullptr;
        b->ev_join[nd] = nullptr;
    }
    b->ev_fork = nullptr;
    hipError_t e = hipMalloc(&b->d_ents, (size_t)capacity * sizeof(BatchEntry));
    if (e == hipSuccess) e = hipMalloc(&b->d_steps, (size_t)capacity * sizeof(int));
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming);
    for (int nd = 1; nd <= 3 && e == hipSuccess; nd++) {
        e = hipStreamCreateWithFlags(&b->side[nd], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_join[nd], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipHostMalloc(&b->h_ents, (size_t)capacity * sizeof(BatchEntry), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&b->h_steps, (size_t)capacity * sizeof(int), hipHostMallocDefault);
    if (e != hipSuccess) {
        if (b->d_ents) (void)hipFree(b->d_ents);
        if (b->d_steps) (void)hipFree(b->d_steps);
        if (b->h_ents) (void)hipHostFree(b->h_ents);
        if (b->h_steps) (void)hipHostFree(b->h_steps);
        for (int nd = 1; nd <= 3; nd++) {
            if (b->side[nd]) (void)hipStreamDestroy(b->side[nd]);
            if (b->ev_join[nd]) (void)hipEventDestroy(b->ev_join[nd]);
        }
        if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
        delete b;
        return fail(PPML_ENOMEM, "batch tables: %s", hipGetErrorString(e));
    }
    *out = b;
    return PPML_OK;
}

int ppml_batch_admit(ppml_batch *b, ppml_grid *g, int32_t *slot)
{
    if (!b || !g) return fail(PPML_EINVAL, "batch and grid are required");
    if (g->in_batch) return fail(PPML_ESTATE, "grid already belongs to a batch");
    if (!g->has_state) return fail(PPML_ESTATE, "grid state was never set");
    if (g->device != b->device) return fail(PPML_EINVAL, "grid and batch live on different devices");
    if (b->prec >= 0 && g->d.prec != b->prec) return fail(PPML_EINVAL, "all grids of a batch share one precision");
    if (g->gp.self_grav || g->gp.potential == POT_HALO)
        return fail(PPML_EINVAL, "grids with self-gravity or the halo potential step alone, not in a batch");
    const size_t need = grid_bytes(g);
    if (b->budget > 0 && b->in_use + need > b->budget)
        return fail(PPML_EBUDGET, "admitting %zu bytes would exceed the budget (%zu of %zu in use)", need, b->in_use,
                    b->budget);
    int s = -1;
    for (int i = 0; i < b->capacity; i++)
        if (!b->slots[i]) {
            s = i;
            break;
        }
    if (s < 0) return fail(PPML_EBUDGET, "batch is full (%d grids)", b->capacity);
    HIPCHK(hipStreamSynchronize(b->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
    b->slots[s] = g;
    b->in_use += need;
    b->prec = g->d.prec;
    g->in_batch = true;
    g->bstream = b->stream;
    b->dirty = true;
    if (slot) *slot = s;
    return PPML_OK;
}

int ppml_batch_retire(ppml_batch *b, int32_t slot)
{
    if (!b) return fail(PPML_EINVAL, "batch is NULL");
    if (slot < 0 || slot >= b->capacity || !b->slots[slot]) return fail(PPML_EINVAL, "slot %d is not in use", slot);
    HIPCHK(hipStreamSynchronize(b->stream));
    ppml_grid *g = b->slots[slot];
    g->in_batch = false;
    b->in_use -= grid_bytes(g);
    b->slots[slot] = nullptr;
    b->dirty = true;
    bool any = false;
    for (ppml_grid *x : b->slots) any = any || x;
    if (!any) b->prec = -1;
    return PPML_OK;
}

int ppml_batch_step(ppml_batch *b, int32_t nsteps, const int32_t *steps_per_slot, double dt_fixed, double t_stop,
                    int32_t use_graph)
{
    if (!b) return fail(PPML_EINVAL, "batch is NULL");
    if (nsteps < 0) return fail(PPML_EINVAL, "nsteps must be >= 0");
    if (!std::isfinite(dt_fixed) || !std::isfinite(t_stop)) return fail(PPML_EINVAL, "dt_fixed and t_stop must be finite");
    HIPCHK(hipStreamSynchronize(b->stream));  // staging buffers are free again
    if (b->dirty) {
        int rc = batch_rebuild(b);
        if (rc) return rc;
    }
    const int n = (int)b->entry_slot.size();
    if (n == 0 || nsteps == 0) return PPML_OK;
    for (int i = 0; i < n; i++) {
        int s = b->entry_slot[i];
        int k = steps_per_slot ? steps_per_slot[s] : nsteps;
        if (k < 0 || k > nsteps) return fail(PPML_EINVAL, "steps of slot %d must lie in [0, nsteps]", s);
        b->h_steps[i] = k;
    }
    HIPCHK(hipMemcpyAsync(b->d_steps, b->h_steps, (size_t)n * sizeof(int), hipMemcpyHostToDevice, b->stream));
    k_batch_set_run<<<(n + 255) / 256, 256, 0, b->stream>>>(b->d_ents, n, b->d_steps, dt_fixed, t_stop);
    HIPCHK(hipGetLastError());
    const bool fp64 = b->prec == PPML_FP64;
    if (use_graph) {
        if (!b->exec || b->graph_version != b->version || b->graph_nsteps != nsteps) {
            batch_drop_graph(b);
            HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            const int erc = fp64 ? batch_enqueue<double>(b, nsteps) : batch_enqueue<float>(b, nsteps);
            hipGraph_t gr = nullptr;
            const hipError_t ce = hipStreamEndCapture(b->stream, &gr);
            if (erc) {
                if (gr) (void)hipGraphDestroy(gr);
                return erc;
            }
            HIPCHK(ce);
            b->graph = gr;
            HIPCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
            b->graph_nsteps = nsteps;
            b->graph_version = b->version;
        }
        HIPCHK(hipGraphLaunch(b->exec, b->stream));
    } else {
        const int erc = fp64 ? batch_enqueue<double>(b, nsteps) : batch_enqueue<float>(b, nsteps);
        if (erc) return erc;
    }
    return PPML_OK;
}

int ppml_batch_sync(ppml_batch *b)
{
    if (!b) return fail(PPML_EINVAL, "batch is NULL");
    HIPCHK(hipStreamSynchronize(b->stream));
    for (int s = 0; s < b->capacity; s++) {
        ppml_grid *g = b->slots[s];
        if (!g) continue;
        int err = 0;
        HIPCHK(hipMemcpy(&err, &g->ctrl->err, sizeof(int), hipMemcpyDeviceToHost));
        if (err) return fail(PPML_ENONFINITE, "grid in slot %d produced a non-physical or non-finite value", s);
    }
    return PPML_OK;
}

int ppml_batch_info(ppml_batch *b, int32_t *count, size_t *bytes_in_use)
{
    if (!b) return fail(PPML_EINVAL, "batch is NULL");
    int n = 0;
    for (ppml_grid *x : b->slots) n += x ? 1 : 0;
    if (count) *count = n;
    if (bytes_in_use) *bytes_in_use = b->in_use;
    return PPML_OK;
}

int ppml_batch_set_tile(ppml_batch *b, int32_t ndim, int32_t variant)
{
    if (!b) return fail(PPML_EINVAL, "batch is NULL");
    if (ndim < 1 || ndim > 3) return fail(PPML_EINVAL, "ndim must be 1, 2 or 3 (got %d)", ndim);
    if (variant < 0 || variant >= NTILE[ndim]) return fail(PPML_EINVAL, "tile %d out of range", variant);
    for (ppml_grid *x : b->slots)
        if (x && x->d.ndim == ndim) return fail(PPML_ESTATE, "grids of ndim %d are admitted", ndim);
    b->tile[ndim] = variant;
    b->dirty = true;
    return PPML_OK;
}

int ppml_batch_destroy(ppml_batch *b)
{
    if (!b) return fail(PPML_EINVAL, "batch is NULL");
    (void)hipStreamSynchronize(b->stream);
    batch_drop_graph(b);
    for (ppml_grid *g : b->slots)
        if (g) g->in_batch = false;
    (void)hipFree(b->d_ents);
    (void)hipFree(b->d_steps);
    (void)hipHostFree(b->h_ents);
    (void)hipHostFree(b->h_steps);
    for (int nd = 1; nd <= 3; nd++) {
        (void)hipStreamDestroy(b->side[nd]);
        (void)hipEventDestroy(b->ev_join[nd]);
    }
    (void)hipEventDestroy(b->ev_fork);
    delete b;
    return PPML_OK;
}

}  // extern "C"
