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
//   4. sine transforms along x, y, z (stage 2) -- dense products with the
//      sine matrices sin(pi j k / (N+1)), which diagonalise the Dirichlet
//      problem (the Fourier basis of the odd extension); run as GEMMs on the
//      matrix cores by the host code;
//   5. k_grav_eigdiv: division by the stencil's eigenvalue
//      -6 (1 - prod_a (1 - (2/3) sin^2(pi j_a / (2 (N_a + 1))))) and the
//      inverse transform's factor prod_a 2 / (N_a + 1) -- stage 3;
//   6. inverse transforms (the same products) into the interior of the
//      shell-padded potential, which the Eulerian kernel differences.
// Tables (sine matrices, eigenvalue factors) are built once by
// k_grav_tables.
#pragma once

#include "ppml_device.hpp"

namespace ppml {

constexpr int GRAV_THREADS = 256;
constexpr int GRAV_MOM = 7;  // M, Ix, Iy, Iz, Ixy, Ixz, Iyz

// Sine matrices S_a[j][k] = sin(pi (j+1)(k+1) / (n_a + 1)) of the three
// axes (the argument reduced exactly modulo 2 (n_a + 1) before sinpi), and
// the per-axis eigenvalue factors f_a[j] = 1 - (2/3) sin^2(pi (j+1) / (2 (n_a + 1))).
template <typename T>
__global__ void k_grav_tables(T *__restrict__ Sx, T *__restrict__ Sy, T *__restrict__ Sz, double *__restrict__ fx,
                              double *__restrict__ fy, double *__restrict__ fz, int n0, int n1, int n2)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long m0 = (long long)n0 * n0, m1 = (long long)n1 * n1, m2 = (long long)n2 * n2;
    T *S;
    int n;
    long long q;
    if (t < m0) {
        S = Sx, n = n0, q = t;
    } else if (t < m0 + m1) {
        S = Sy, n = n1, q = t - m0;
    } else if (t < m0 + m1 + m2) {
        S = Sz, n = n2, q = t - m0 - m1;
    } else {
        const long long r = t - m0 - m1 - m2;
        double *f;
        int nn, j;
        if (r < n0) f = fx, nn = n0, j = (int)r;
        else if (r < n0 + n1) f = fy, nn = n1, j = (int)(r - n0);
        else if (r < n0 + n1 + n2) f = fz, nn = n2, j = (int)(r - n0 - n1);
        else return;
        const double s = sin(M_PI * (double)(j + 1) / (2.0 * (double)(nn + 1)));
        f[j] = 1.0 - 2.0 * s * s / 3.0;
        return;
    }
    const long long j = q / n + 1, k = q % n + 1;
    const long long per = 2ll * (n + 1);
    const long long m = (j * k) % per;
    S[q] = (T)sinpi((double)m / (double)(n + 1));
}

// Interior cell index -> (i, j, k).  Grids hold fewer than 2^31 cells, so
// 32-bit unsigned division serves (64-bit division is a long software
// sequence on the GPU).
__device__ __forceinline__ void cell_of(const GridParams &gp, long long c, int &i, int &j, int &k)
{
    const unsigned n0 = (unsigned)gp.n[0], n01 = n0 * (unsigned)gp.n[1];
    const unsigned cu = (unsigned)c;
    const unsigned kk = cu / n01;
    const unsigned r = cu - kk * n01;
    const unsigned jj = r / n0;
    k = (int)kk;
    j = (int)jj;
    i = (int)(r - jj * n0);
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

// Stage 1, moments: block b sums cells [b chunk, (b+1) chunk) (thread t
// takes every GRAV_THREADS-th cell from t on, then a fixed tree), so the
// order of every sum is fixed by the grid size alone.
template <typename T>
__global__ __launch_bounds__(GRAV_THREADS) void k_grav_moments_partial(const T *__restrict__ rho, GridParams gp,
                                                                       long long chunk, double *__restrict__ part)
{
    __shared__ double sh[GRAV_THREADS];
    const long long c0 = (long long)blockIdx.x * chunk;
    long long c1 = c0 + chunk;
    if (c1 > gp.ncell) c1 = gp.ncell;
    const double vol = gp.h[0] * gp.h[1] * gp.h[2];
    double s[GRAV_MOM] = {0, 0, 0, 0, 0, 0, 0};
    for (long long c = c0 + threadIdx.x; c < c1; c += GRAV_THREADS) {
        int i, j, k;
        cell_of(gp, c, i, j, k);
        const double x = gp.lo[0] + ((double)i + 0.5) * gp.h[0];
        const double y = gp.lo[1] + ((double)j + 0.5) * gp.h[1];
        const double z = gp.lo[2] + ((double)k + 0.5) * gp.h[2];
        const double m = (double)rho[c] * vol;
        s[0] = s[0] + m;
        s[1] = s[1] + (y * y + z * z) * m;
        s[2] = s[2] + (x * x + z * z) * m;
        s[3] = s[3] + (x * x + y * y) * m;
        s[4] = s[4] + x * y * m;
        s[5] = s[5] + x * z * m;
        s[6] = s[6] + y * z * m;
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
inline long long grav_edge_cells(int n0, int n1, int n2)
{
    const long long m2 = n2 > 2 ? n2 - 2 : 0, m1 = n1 > 2 ? n1 - 2 : 0;
    return 2ll * n0 * n1 + 2ll * m2 * n0 + 2ll * m2 * m1;
}

// Stage 3: amplitude / eigenvalue times the inverse transform's factor.
template <typename T>
__global__ void k_grav_eigdiv(T *__restrict__ Y, const double *__restrict__ fx, const double *__restrict__ fy,
                              const double *__restrict__ fz, GridParams gp, double norm)
{
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= gp.ncell) return;
    int i, j, k;
    cell_of(gp, c, i, j, k);
    const double prod = fx[i] * fy[j] * fz[k];
    const double lam = -6.0 * (1.0 - prod);
    Y[c] = (T)((double)Y[c] / lam * norm);
}

}  // namespace ppml
