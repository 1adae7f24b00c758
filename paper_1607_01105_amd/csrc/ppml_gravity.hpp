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
//   3. right-hand side 4 pi G h^2 rho minus the stencil terms that reach
//      the shell (the boundary values move to the right-hand side):
//      k_grav_edge_terms forms the shell terms of the outer layer of cells,
//      k_grav_butterfly adds them to 4 pi G h^2 rho as it reads the density;
//   4. sine transforms along x, y, z (stage 2) -- products with the sine
//      matrices sin(pi j k / (N+1)), which diagonalise the Dirichlet problem
//      (the Fourier basis of the odd extension).  The matrix is split by the
//      symmetry sin(pi j (N+1-k) / (N+1)) = -(-1)^j sin(pi j k / (N+1)): the
//      odd modes need only the sums x_k + x_{N+1-k}, the even modes only the
//      differences, so k_grav_butterfly forms sums and differences of the
//      right-hand side along all
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

// Stage 1, moments: block b sums the x rows [b chunk, (b+1) chunk) of the
// grid (row r = j + n1 k; thread t takes columns i = t, t + GRAV_THREADS, ...
// and runs down the block's rows, U loads in flight, then a fixed-order
// reduction), so the order of every sum is fixed by the grid size alone.
// x is fixed along a
// thread's column, so the thread sums rho, y rho, z rho, y^2 rho, z^2 rho and
// y z rho and forms the seven moments from them and x once per column; the
// cell volume is applied once per block.
template <typename T>
__global__ __launch_bounds__(GRAV_THREADS) void k_grav_moments_partial(const T *__restrict__ rho, GridParams gp,
                                                                       int chunk, double *__restrict__ part)
{
    const int n0 = gp.n[0], n1 = gp.n[1];
    const int rows = n1 * gp.n[2];
    const int r0 = blockIdx.x * chunk;
    const int r1 = r0 + chunk < rows ? r0 + chunk : rows;
    const double vol = gp.h[0] * gp.h[1] * gp.h[2];
    double s[GRAV_MOM] = {0, 0, 0, 0, 0, 0, 0};
    constexpr int U = 16;  // loads in flight per thread
    for (int i = threadIdx.x; i < n0; i += GRAV_THREADS) {
        const double x = gp.lo[0] + ((double)i + 0.5) * gp.h[0];
        double a0 = 0, ay = 0, az = 0, ayy = 0, azz = 0, ayz = 0;
        // (j, k) of the first row of each group of U, advanced without a
        // division (uniform over the block)
        int k0 = r0 / n1, j0 = r0 - k0 * n1;
        for (int rb = r0; rb < r1; rb += U) {
            T v[U];
#pragma unroll
            for (int u = 0; u < U; u++) v[u] = rb + u < r1 ? rho[(long long)(rb + u) * n0 + i] : T(0);
            int j = j0, k = k0;
#pragma unroll
            for (int u = 0; u < U; u++) {
                if (rb + u >= r1) break;
                const double y = gp.lo[1] + ((double)j + 0.5) * gp.h[1];
                const double z = gp.lo[2] + ((double)k + 0.5) * gp.h[2];
                const double m = (double)v[u];
                const double ym = y * m, zm = z * m;
                a0 = a0 + m;
                ay = ay + ym;
                az = az + zm;
                ayy = ayy + y * ym;
                azz = azz + z * zm;
                ayz = ayz + y * zm;
                if (++j == n1) {
                    j = 0;
                    ++k;
                }
            }
            j0 = j;
            k0 = k;
        }
        const double xx = x * x;
        s[0] = s[0] + a0;
        s[1] = s[1] + (ayy + azz);
        s[2] = s[2] + (xx * a0 + azz);
        s[3] = s[3] + (xx * a0 + ayy);
        s[4] = s[4] + x * ay;
        s[5] = s[5] + x * az;
        s[6] = s[6] + ayz;
    }
    // fixed-order reduction: butterfly within each wave, then the waves'
    // sums in order
    __shared__ double shw[GRAV_THREADS / 64][GRAV_MOM];
#pragma unroll
    for (int q = 0; q < GRAV_MOM; q++) {
        double v = s[q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v = v + __shfl_xor(v, o, 64);
        if ((threadIdx.x & 63) == 0) shw[threadIdx.x >> 6][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < GRAV_MOM) {
        double r = 0.0;
#pragma unroll
        for (int w = 0; w < GRAV_THREADS / 64; w++) r = r + shw[w][threadIdx.x];
        part[(long long)blockIdx.x * GRAV_MOM + threadIdx.x] = r * vol;
    }
}

__global__ __launch_bounds__(GRAV_THREADS) void k_grav_moments_final(const double *__restrict__ part, int nb,
                                                                     Ctrl *ctrl)
{
    // thread t sums the blocks t, t + GRAV_THREADS, ... in order, then the
    // same fixed-order reduction as the partial sums
    double s[GRAV_MOM];
#pragma unroll
    for (int q = 0; q < GRAV_MOM; q++) s[q] = 0.0;
    for (int b = threadIdx.x; b < nb; b += GRAV_THREADS)
#pragma unroll
        for (int q = 0; q < GRAV_MOM; q++) s[q] = s[q] + part[(long long)b * GRAV_MOM + q];
    __shared__ double shw[GRAV_THREADS / 64][GRAV_MOM];
#pragma unroll
    for (int q = 0; q < GRAV_MOM; q++) {
        double v = s[q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v = v + __shfl_xor(v, o, 64);
        if ((threadIdx.x & 63) == 0) shw[threadIdx.x >> 6][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < GRAV_MOM) {
        double r = 0.0;
#pragma unroll
        for (int w = 0; w < GRAV_THREADS / 64; w++) r = r + shw[w][threadIdx.x];
        ctrl->mom[threadIdx.x] = r;
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

// Shell terms of the right-hand side, over the outer layer of interior
// cells only (the two z planes, the two y rows of the other planes, the two
// x ends of the other rows; a cell listed twice on a grid of extent 1 or 2
// gets the same value twice): minus the stencil's weight times every shell
// value the cell's stencil touches, in the stencil's (dz, dy, dx) order,
// into E[s] for the cell's place s in that list.
template <typename T>
__global__ void k_grav_edge_terms(const T *__restrict__ phi, GridParams gp, T *__restrict__ E)
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
    double b = 0.0;
    for (int dz = -1; dz <= 1; dz++)
        for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++) {
                const int ii = i + dx, jj = j + dy, kk = k + dz;
                if (ii >= 0 && ii < n0 && jj >= 0 && jj < n1 && kk >= 0 && kk < n2) continue;
                const int nd = (dx != 0) + (dy != 0) + (dz != 0);
                const double w = nd == 1 ? 4.0 / 9.0 : (nd == 2 ? 1.0 / 9.0 : 1.0 / 36.0);
                b = b - w * (double)phi[pad_index(gp, ii, jj, kk)];
            }
    E[s] = (T)b;
}

// Place of cell (i, j, k) in the outer-layer list of k_grav_edge_terms (its
// first place where listed twice), -1 for a cell inside the layer.
__device__ __forceinline__ long long grav_edge_index(int i, int j, int k, int n0, int n1, int n2)
{
    const long long P = (long long)n0 * n1;
    const long long m2 = n2 > 2 ? n2 - 2 : 0, m1 = n1 > 2 ? n1 - 2 : 0;
    if (k == 0) return (long long)j * n0 + i;
    if (k == n2 - 1) return P + (long long)j * n0 + i;
    if (j == 0 || j == n1 - 1) return 2 * P + (2ll * (k - 1) + (j == 0 ? 0 : 1)) * n0 + i;
    if (i == 0 || i == n0 - 1) return 2 * P + 2 * m2 * n0 + (long long)(k - 1) * 2 * m1 + 2ll * (j - 1) + (i == 0 ? 0 : 1);
    return -1;
}

// Cells of the outer layer listed by k_grav_edge_terms.
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

// Right-hand side of the cells (coef rho, coef = 4 pi G h^2, plus the shell
// terms E of the outer layer) and its sums and differences of mirror cells
// along x, y and z: Y in (sum | difference) slots per axis.  Along an axis
// the pair (p, n-1-p), p < ne, gives slot p the sum and slot no + p the
// difference; a middle cell (n odd) is its own sum.
template <typename T>
__global__ void k_grav_butterfly(const T *__restrict__ rho, const T *__restrict__ E, double coef,
                                 T *__restrict__ Y, GridParams gp)
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
                double b = 0.0;
                if (ok) {
                    b = coef * (double)rho[((long long)cz[mz] * n1 + cy[my]) * n0 + cx[mx]];
                    const long long e = grav_edge_index(cx[mx], cy[my], cz[mz], n0, n1, n2);
                    if (e >= 0) b = b + (double)E[e];
                }
                a[mz][my][mx] = b;
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
// Grid: x over blockIdx.x, groups of four rows (j + n1 k, uniform per
// block) strided over blockIdx.y, the four loads in flight together.
template <typename T>
__global__ void k_grav_eigdiv(T *__restrict__ Y, const double *__restrict__ fx, const double *__restrict__ fy,
                              const double *__restrict__ fz, GridParams gp, double norm)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int n0 = gp.n[0], n1 = gp.n[1];
    const int rows = n1 * gp.n[2];
    if (i >= n0) return;
    const double f0 = fx[i];
    constexpr int U = 4;  // rows in flight per thread
    for (int rb = blockIdx.y * U; rb < rows; rb += gridDim.y * U) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; u++) v[u] = rb + u < rows ? Y[(long long)(rb + u) * n0 + i] : T(0);
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int row = rb + u;
            if (row >= rows) break;
            const int k = row / n1, j = row - k * n1;
            const double prod = f0 * fy[j] * fz[k];
            const double lam = -6.0 * (1.0 - prod);
#ifdef PPML_EXACT
            Y[(long long)row * n0 + i] = (T)((double)v[u] / lam * norm);
#else
            // reciprocal by two Newton steps from the hardware estimate
            // (within an ulp or two of the division)
            double r = __builtin_amdgcn_rcp(lam);
            r = r * (2.0 - lam * r);
            r = r * (2.0 - lam * r);
            Y[(long long)row * n0 + i] = (T)((double)v[u] * (r * norm));
#endif
        }
    }
}

}  // namespace ppml
