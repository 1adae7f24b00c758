// ppml_gravity.hpp -- device kernels of the self-gravity potential (Sec. 2.5,
// the Poisson solver) on gfx950.
//
// Delta Phi = 4 pi G rho in its 27-point finite-difference form (weights
// -38/9, 4/9 on faces, 1/9 on edges, 1/36 on corners; right-hand side
// 4 pi G h^2 rho) on the interior cells of a 3-D grid of cubic cells:
//   1. k_grav_moments_*: mass and second moments of the cell masses about
//      the coordinate origin (FP64, fixed summation order);
//   2. k_grav_shell: the one-cell shell around the box takes the two-term
//      multipole expansion (monopole and quadrupole, MacCullagh's form with
//      its factor 1/2) -- stage 1;
//   3. k_grav_rhs: 4 pi G h^2 rho minus the stencil terms that reach the
//      shell (the boundary values move to the right-hand side);
//   4. sine transforms along x, y, z (stage 2) -- products with the sine
//      matrices sin(pi j k / (N+1)), which diagonalise the Dirichlet problem
//      (the Fourier basis of the odd extension).  The matrix is split by the
//      symmetry sin(pi j (N+1-k) / (N+1)) = -(-1)^j sin(pi j k / (N+1)): the
//      odd modes need only the sums x_k + x_{N+1-k}, the even modes only the
//      differences, so k_grav_butterfly forms sums and differences along all
//      three axes at once and each axis transform is two half-size GEMMs on
//      the matrix cores (half the work of the full product), run by the host
//      code; the modes come out odd first, then even, along each axis;
//   5. k_grav_eigdiv: division by the stencil's eigenvalue
//      -6 (1 - prod_a (1 - (2/3) sin^2(pi j_a / (2 (N_a + 1))))) and the
//      inverse transform's factor prod_a 2 / (N_a + 1) -- stage 3 (the
//      eigenvalue factors are tabulated in the modes' storage order);
//   6. inverse transforms (the transposed half-size products), then
//      k_grav_unbutterfly undoes the sums and differences into the interior
//      of the shell-padded potential, which the Eulerian kernel differences.
// Tables (half-size sine matrices, eigenvalue factors) are built once by
// k_grav_tables.
#pragma once

#include "ppml_device.hpp"

namespace ppml {

constexpr int GRAV_THREADS = 256;
constexpr int GRAV_MOM = 7;  // M, Ix, Iy, Iz, Ixy, Ixz, Iyz

// Modes along an axis of n cells are stored odd first: slot p < no holds
// j = 2p + 1, slot no + p holds j = 2p + 2 (no = (n+1)/2 odd and ne = n/2
// even modes).
__host__ __device__ __forceinline__ int grav_no(int n) { return (n + 1) / 2; }
__host__ __device__ __forceinline__ int grav_ne(int n) { return n / 2; }
__device__ __forceinline__ int grav_mode(int p, int n) { return p < grav_no(n) ? 2 * p + 1 : 2 * (p - grav_no(n)) + 2; }

// Table entries of one axis of n cells: the odd block So (no x no, column
// major, So(a, b) = sin(pi (2a+1)(b+1) / (n+1))), then the even block Se
// (ne x ne, Se(a, b) = sin(pi (2a+2)(b+1) / (n+1))), the argument reduced
// exactly modulo 2 (n+1) before sinpi; entries q >= no^2 + ne^2 are the
// eigenvalue factors f[p] = 1 - (2/3) sin^2(pi j / (2 (n+1))) of slot p.
template <typename T> __device__ void grav_table_entry(T *S, double *f, int n, long long q)
{
    const long long no = grav_no(n), ne = grav_ne(n);
    long long j, k;
    if (q < no * no) {
        const long long a = q % no, b = q / no;
        j = 2 * a + 1, k = b + 1;
    } else if (q < no * no + ne * ne) {
        const long long r = q - no * no;
        const long long a = r % ne, b = r / ne;
        j = 2 * a + 2, k = b + 1;
    } else {
        const int p = (int)(q - no * no - ne * ne);
        const double s = sin(M_PI * (double)grav_mode(p, n) / (2.0 * (double)(n + 1)));
        f[p] = 1.0 - 2.0 * s * s / 3.0;
        return;
    }
    const long long m = (j * k) % (2ll * (n + 1));
    S[q] = (T)sinpi((double)m / (double)(n + 1));
}

__host__ __device__ inline long long grav_table_count(int n)
{
    const long long no = grav_no(n), ne = grav_ne(n);
    return no * no + ne * ne + n;
}

template <typename T>
__global__ void k_grav_tables(T *__restrict__ Sx, T *__restrict__ Sy, T *__restrict__ Sz, double *__restrict__ fx,
                              double *__restrict__ fy, double *__restrict__ fz, int n0, int n1, int n2)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long c0 = grav_table_count(n0), c1 = grav_table_count(n1), c2 = grav_table_count(n2);
    if (t < c0) grav_table_entry<T>(Sx, fx, n0, t);
    else if (t < c0 + c1) grav_table_entry<T>(Sy, fy, n1, t - c0);
    else if (t < c0 + c1 + c2) grav_table_entry<T>(Sz, fz, n2, t - c0 - c1);
}

__device__ __forceinline__ double block_sum(double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = GRAV_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + w];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// Stage 1, moments: block b sums the x rows [b chunk, (b+1) chunk) of the
// grid (row r = j + n1 k; thread t takes columns i = t, t + GRAV_THREADS, ...
// and runs down the block's rows, U loads in flight, then a fixed tree), so
// the order of every sum is fixed by the grid size alone.
template <typename T>
__global__ __launch_bounds__(GRAV_THREADS) void k_grav_moments_partial(const T *__restrict__ rho, GridParams gp,
                                                                       int chunk, double *__restrict__ part)
{
    __shared__ double sh[GRAV_THREADS];
    const int n0 = gp.n[0], n1 = gp.n[1];
    const int rows = n1 * gp.n[2];
    const int r0 = blockIdx.x * chunk;
    const int r1 = r0 + chunk < rows ? r0 + chunk : rows;
    const double vol = gp.h[0] * gp.h[1] * gp.h[2];
    double s[GRAV_MOM] = {0, 0, 0, 0, 0, 0, 0};
    constexpr int U = 8;  // loads in flight per thread
    for (int i = threadIdx.x; i < n0; i += GRAV_THREADS) {
        const double x = gp.lo[0] + ((double)i + 0.5) * gp.h[0];
        for (int rb = r0; rb < r1; rb += U) {
            T v[U];
#pragma unroll
            for (int u = 0; u < U; u++) v[u] = rb + u < r1 ? rho[(long long)(rb + u) * n0 + i] : T(0);
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int row = rb + u;
                if (row >= r1) break;
                const int k = row / n1, j = row - k * n1;
                const double y = gp.lo[1] + ((double)j + 0.5) * gp.h[1];
                const double z = gp.lo[2] + ((double)k + 0.5) * gp.h[2];
                const double m = (double)v[u] * vol;
                s[0] = s[0] + m;
                s[1] = s[1] + (y * y + z * z) * m;
                s[2] = s[2] + (x * x + z * z) * m;
                s[3] = s[3] + (x * x + y * y) * m;
                s[4] = s[4] + x * y * m;
                s[5] = s[5] + x * z * m;
                s[6] = s[6] + y * z * m;
            }
        }
    }
    for (int q = 0; q < GRAV_MOM; q++) {
        const double r = block_sum(s[q], sh);
        if (threadIdx.x == 0) part[(long long)blockIdx.x * GRAV_MOM + q] = r;
    }
}

__global__ __launch_bounds__(GRAV_THREADS) void k_grav_moments_final(const double *__restrict__ part, int nb,
                                                                     Ctrl *ctrl)
{
    __shared__ double sh[GRAV_THREADS];
    for (int q = 0; q < GRAV_MOM; q++) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nb; b += GRAV_THREADS) s = s + part[(long long)b * GRAV_MOM + q];
        const double r = block_sum(s, sh);
        if (threadIdx.x == 0) ctrl->mom[q] = r;
    }
}

__device__ __forceinline__ long long pad_index(const GridParams &gp, int i, int j, int k)
{
    const long long px = gp.n[0] + 2;
    return ((long long)(k + 1) * (gp.n[1] + 2) + (j + 1)) * px + (i + 1);
}

// Stage 1, boundary values: shell cell s -> (i, j, k) (the two z planes,
// then the two y rows of each interior plane, then the two x ends of each
// interior row), value of the multipole expansion at its centre.
template <typename T>
__global__ void k_grav_shell(GridParams gp, const Ctrl *__restrict__ ctrl, double G, T *__restrict__ phi)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int n0 = gp.n[0], n1 = gp.n[1], n2 = gp.n[2];
    const long long P = (long long)(n0 + 2) * (n1 + 2);
    const long long nA = 2 * P, nB = 2ll * n2 * (n0 + 2), nC = 2ll * n1 * n2;
    int i, j, k;
    if (s < nA) {
        k = (s / P) ? n2 : -1;
        const long long r = s % P;
        j = (int)(r / (n0 + 2)) - 1;
        i = (int)(r % (n0 + 2)) - 1;
    } else if (s < nA + nB) {
        const long long t = s - nA;
        const long long row = t / (n0 + 2);
        k = (int)(row / 2);
        j = (row % 2) ? n1 : -1;
        i = (int)(t % (n0 + 2)) - 1;
    } else if (s < nA + nB + nC) {
        const long long t = s - nA - nB;
        k = (int)(t / (2 * n1));
        const long long r = t % (2 * n1);
        j = (int)(r / 2);
        i = (r % 2) ? n0 : -1;
    } else {
        return;
    }
    const double x = gp.lo[0] + ((double)i + 0.5) * gp.h[0];
    const double y = gp.lo[1] + ((double)j + 0.5) * gp.h[1];
    const double z = gp.lo[2] + ((double)k + 0.5) * gp.h[2];
    const double *mo = ctrl->mom;
    const double r2 = x * x + y * y + z * z;
    const double r = sqrt(r2);
    const double I0 = ((x * x * mo[1] + y * y * mo[2] + z * z * mo[3]) -
                       2.0 * (x * y * mo[4] + x * z * mo[5] + y * z * mo[6])) / r2;
    const double v = -G * mo[0] / r - G * (mo[1] + mo[2] + mo[3] - 3.0 * I0) / (2.0 * r2 * r);
    phi[pad_index(gp, i, j, k)] = (T)v;
}

// Right-hand side of the interior cells, first pass: coef rho (coef =
// 4 pi G h^2) everywhere (a plain stream).
template <typename T>
__global__ void k_grav_rhs(const T *__restrict__ rho, GridParams gp, double coef, T *__restrict__ X)
{
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= gp.ncell) return;
    X[c] = (T)(coef * (double)rho[c]);
}

// Second pass over the outer layer of interior cells only (the two z
// planes, the two y rows of the other planes, the two x ends of the other
// rows; a cell listed twice on a grid of extent 1 or 2 gets the same value
// twice): coef rho minus the stencil's weight times every shell value the
// cell's stencil touches, in the stencil's (dz, dy, dx) order.
template <typename T>
__global__ void k_grav_rhs_edge(const T *__restrict__ rho, const T *__restrict__ phi, GridParams gp, double coef,
                                T *__restrict__ X)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int n0 = gp.n[0], n1 = gp.n[1], n2 = gp.n[2];
    const long long P = (long long)n0 * n1;
    const int m2 = n2 > 2 ? n2 - 2 : 0, m1 = n1 > 2 ? n1 - 2 : 0;
    const long long nA = 2 * P, nB = 2ll * m2 * n0, nC = 2ll * m2 * m1;
    int i, j, k;
    if (s < nA) {
        k = (s / P) ? n2 - 1 : 0;
        const long long r = s % P;
        j = (int)(r / n0);
        i = (int)(r % n0);
    } else if (s < nA + nB) {
        const long long t = s - nA;
        const long long row = t / n0;
        k = 1 + (int)(row / 2);
        j = (row % 2) ? n1 - 1 : 0;
        i = (int)(t % n0);
    } else if (s < nA + nB + nC) {
        const long long t = s - nA - nB;
        k = 1 + (int)(t / (2 * m1));
        const long long r = t % (2 * m1);
        j = 1 + (int)(r / 2);
        i = (r % 2) ? n0 - 1 : 0;
    } else {
        return;
    }
    const long long c = ((long long)k * n1 + j) * n0 + i;
    double b = coef * (double)rho[c];
    {
        for (int dz = -1; dz <= 1; dz++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    const int ii = i + dx, jj = j + dy, kk = k + dz;
                    if (ii >= 0 && ii < n0 && jj >= 0 && jj < n1 && kk >= 0 && kk < n2) continue;
                    const int nd = (dx != 0) + (dy != 0) + (dz != 0);
                    const double w = nd == 1 ? 4.0 / 9.0 : (nd == 2 ? 1.0 / 9.0 : 1.0 / 36.0);
                    b = b - w * (double)phi[pad_index(gp, ii, jj, kk)];
                }
    }
    X[c] = (T)b;
}

// Cells of the outer layer listed by k_grav_rhs_edge.
__host__ __device__ inline long long grav_edge_cells(int n0, int n1, int n2)
{
    const long long m2 = n2 > 2 ? n2 - 2 : 0, m1 = n1 > 2 ? n1 - 2 : 0;
    return 2ll * n0 * n1 + 2ll * m2 * n0 + 2ll * m2 * m1;
}

// Representative (i, j, k) of a group of up to eight mirror cells (i or
// n0-1-i, ...), i < no0, j < no1, k < no2.
__device__ __forceinline__ bool grav_rep(const GridParams &gp, long long t, int &i, int &j, int &k)
{
    const unsigned o0 = grav_no(gp.n[0]), o1 = grav_no(gp.n[1]), o2 = grav_no(gp.n[2]);
    if (t >= (long long)o0 * o1 * o2) return false;
    const unsigned tu = (unsigned)t;
    const unsigned r = tu / o0;
    i = (int)(tu - r * o0);
    k = (int)(r / o1);
    j = (int)(r - (unsigned)k * o1);
    return true;
}

// (a, b) -> (a + b, a - b) along x, then y, then z of a group of eight.
__device__ __forceinline__ void grav_pairs(double a[2][2][2])
{
#pragma unroll
    for (int p = 0; p < 2; p++)
#pragma unroll
        for (int q = 0; q < 2; q++) {
            const double u = a[p][q][0] + a[p][q][1], v = a[p][q][0] - a[p][q][1];  // x
            a[p][q][0] = u, a[p][q][1] = v;
        }
#pragma unroll
    for (int p = 0; p < 2; p++)
#pragma unroll
        for (int q = 0; q < 2; q++) {
            const double u = a[p][0][q] + a[p][1][q], v = a[p][0][q] - a[p][1][q];  // y
            a[p][0][q] = u, a[p][1][q] = v;
        }
#pragma unroll
    for (int p = 0; p < 2; p++)
#pragma unroll
        for (int q = 0; q < 2; q++) {
            const double u = a[0][p][q] + a[1][p][q], v = a[0][p][q] - a[1][p][q];  // z
            a[0][p][q] = u, a[1][p][q] = v;
        }
}

// Sums and differences of mirror cells along x, y and z: X in cell order ->
// Y in (sum | difference) slots per axis.  Along an axis the pair (p, n-1-p),
// p < ne, gives slot p the sum and slot no + p the difference; a middle cell
// (n odd) is its own sum.
template <typename T>
__global__ void k_grav_butterfly(const T *__restrict__ X, T *__restrict__ Y, GridParams gp)
{
    int i, j, k;
    if (!grav_rep(gp, (long long)blockIdx.x * blockDim.x + threadIdx.x, i, j, k)) return;
    const int n0 = gp.n[0], n1 = gp.n[1], n2 = gp.n[2];
    const bool hx = i < grav_ne(n0), hy = j < grav_ne(n1), hz = k < grav_ne(n2);
    const int cx[2] = {i, n0 - 1 - i}, cy[2] = {j, n1 - 1 - j}, cz[2] = {k, n2 - 1 - k};
    double a[2][2][2];
#pragma unroll
    for (int mz = 0; mz < 2; mz++)
#pragma unroll
        for (int my = 0; my < 2; my++)
#pragma unroll
            for (int mx = 0; mx < 2; mx++) {
                const bool ok = (!mx || hx) && (!my || hy) && (!mz || hz);
                a[mz][my][mx] = ok ? (double)X[((long long)cz[mz] * n1 + cy[my]) * n0 + cx[mx]] : 0.0;
            }
    grav_pairs(a);
    const int sx[2] = {i, grav_no(n0) + i}, sy[2] = {j, grav_no(n1) + j}, sz[2] = {k, grav_no(n2) + k};
#pragma unroll
    for (int mz = 0; mz < 2; mz++)
#pragma unroll
        for (int my = 0; my < 2; my++)
#pragma unroll
            for (int mx = 0; mx < 2; mx++)
                if ((!mx || hx) && (!my || hy) && (!mz || hz))
                    Y[((long long)sz[mz] * n1 + sy[my]) * n0 + sx[mx]] = (T)a[mz][my][mx];
}

// Inverse of the sums and differences: Y in (sum | difference) slots ->
// the cells of the group, into the interior of the padded potential.
template <typename T>
__global__ void k_grav_unbutterfly(const T *__restrict__ Y, T *__restrict__ phi, GridParams gp)
{
    int i, j, k;
    if (!grav_rep(gp, (long long)blockIdx.x * blockDim.x + threadIdx.x, i, j, k)) return;
    const int n0 = gp.n[0], n1 = gp.n[1], n2 = gp.n[2];
    const bool hx = i < grav_ne(n0), hy = j < grav_ne(n1), hz = k < grav_ne(n2);
    const int sx[2] = {i, grav_no(n0) + i}, sy[2] = {j, grav_no(n1) + j}, sz[2] = {k, grav_no(n2) + k};
    double a[2][2][2];
#pragma unroll
    for (int mz = 0; mz < 2; mz++)
#pragma unroll
        for (int my = 0; my < 2; my++)
#pragma unroll
            for (int mx = 0; mx < 2; mx++) {
                const bool ok = (!mx || hx) && (!my || hy) && (!mz || hz);
                a[mz][my][mx] = ok ? (double)Y[((long long)sz[mz] * n1 + sy[my]) * n0 + sx[mx]] : 0.0;
            }
    // low member = sum + difference, high member = sum - difference
    grav_pairs(a);
    const int cx[2] = {i, n0 - 1 - i}, cy[2] = {j, n1 - 1 - j}, cz[2] = {k, n2 - 1 - k};
#pragma unroll
    for (int mz = 0; mz < 2; mz++)
#pragma unroll
        for (int my = 0; my < 2; my++)
#pragma unroll
            for (int mx = 0; mx < 2; mx++)
                if ((!mx || hx) && (!my || hy) && (!mz || hz))
                    phi[pad_index(gp, cx[mx], cy[my], cz[mz])] = (T)a[mz][my][mx];
}

// Stage 3: amplitude / eigenvalue times the inverse transform's factor.
// Grid: x over blockIdx.x, rows (j + n1 k, uniform per block) strided over
// blockIdx.y.
template <typename T>
__global__ void k_grav_eigdiv(T *__restrict__ Y, const double *__restrict__ fx, const double *__restrict__ fy,
                              const double *__restrict__ fz, GridParams gp, double norm)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int n0 = gp.n[0], n1 = gp.n[1];
    const int rows = n1 * gp.n[2];
    if (i >= n0) return;
    const double f0 = fx[i];
    for (int row = blockIdx.y; row < rows; row += gridDim.y) {
        const int k = row / n1, j = row - k * n1;
        const long long c = (long long)row * n0 + i;
        const double prod = f0 * fy[j] * fz[k];
        const double lam = -6.0 * (1.0 - prod);
        Y[c] = (T)((double)Y[c] / lam * norm);
    }
}

}  // namespace ppml
