// ppml_kernels.hip -- HIP kernels of the PPML operator-splitting update on
// gfx950.  One step is two fused kernels:
//
//   k_euler : Eulerian stage (Sec. 2.1-2.2): reconstruct v_d and p along
//             every axis, acoustic Riemann problem on parabolas at every
//             interface, unsplit update of rho v, rho E, rho eps plus the
//             external force.  U^n -> U^{n+1/2}.
//   k_lagr  : Lagrangian stage (Sec. 2.3): 9-point transverse velocity,
//             density-weighted interface velocity, upwind parabolic fluxes
//             of all conserved densities, unsplit update; then the
//             total-energy correction (Sec. 2.4) and the per-wave maxima of
//             |v| and c for the next CFL step (Sec. 2.1).  U^{n+1/2} -> U^{n+1}.
//
// Work decomposition (3-D): a workgroup owns a TX x TY column tile in (x, y)
// and marches along z over a chunk of planes.  The x and y directions of each
// plane are computed from LDS tiles with a 3-cell halo; the z direction is a
// per-thread register pipeline over the thread's own column (loads run three
// planes ahead), so no z halo is ever staged.  2-D and 1-D grids use the same
// kernels with one plane (and TY = 1 in 1-D).
#include "ppml_device.hpp"

namespace ppml {

template <typename T> __device__ __forceinline__ T ldg(const T *p) { return __builtin_nontemporal_load(p); }

// Job spaces of two kinds (NA x jobs, then NB y jobs) spread over the waves
// of a work group of NT threads: whole wave-rounds of 64 jobs hold one kind
// (wave-rounds 0 .. QA-1 the x jobs, QA .. QA+QB-1 the y jobs), and round r
// of wave w takes wave-round r NW + w.  No wave runs both kinds in one round
// and the partly filled rounds fall on different waves, so the waves of a
// group finish a job phase close together.  job() gives the job of a lane
// (x: 0 .. NA-1, y: NA .. NA+NB-1) or NA + NB for none.
template <int NT, int NA, int NB> struct JobMap {
    static_assert(NT % 64 == 0, "work groups of whole waves");
    static constexpr int NW = NT / 64;
    static constexpr int QA = (NA + 63) / 64;
    static constexpr int QB = (NB + 63) / 64;
    static constexpr int R = (QA + QB + NW - 1) / NW;  // rounds per wave
    static __device__ __forceinline__ int job(int r, int wave, int lane)
    {
        const int q = r * NW + wave;
        if (q < QA) {
            const int j = q * 64 + lane;
            return j < NA ? j : NA + NB;
        }
        const int j = NA + (q - QA) * 64 + lane;
        return j < NA + NB ? j : NA + NB;
    }
    // first wave-round of the y jobs that this wave takes
    static __device__ __forceinline__ int first_b(int wave) { return QA + ((wave - QA % NW) % NW + NW) % NW; }
};

// The value of the previous lane of the 16-lane DPP row (row_shr:1); lane
// 0 of each row, which has no previous lane, gets 0.  Every lane of the row
// must be active.
__device__ __forceinline__ float dpp_prev16(float v)
{
    const int i = __builtin_bit_cast(int, v);
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(i, 0x111, 0xF, 0xF, true));
}

// The wave's index in its work group, as a wave-uniform (scalar) value.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6); }

// s_waitcnt operand that waits for every outstanding vector-memory operation
// of the wave (vmcnt = 0) and leaves the export and LDS/scalar counters
// unconstrained (gfx9 encoding: vmcnt[3:0], expcnt[6:4], lgkmcnt[11:8],
// vmcnt[15:14]).
constexpr int VMCNT0 = 0x0F70;

// ---------------------------------------------------------------------------
// State initialisation and conversion kernels
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_prim_to_cons(const double *__restrict__ prim, T *__restrict__ U, GridParams gp)
{
    const long long N = gp.ncell;
    const int nd = gp.ndim;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (long long)gridDim.x * blockDim.x) {
        double r = prim[c];
        double ux = prim[N + c];
        double uy = nd >= 2 ? prim[2 * N + c] : 0.0;
        double uz = nd >= 3 ? prim[3 * N + c] : 0.0;
        double p = prim[4 * N + c];
        double e = p / (gp.gamma - 1.0);
        double ke = 0.5 * r * (ux * ux + uy * uy + uz * uz);
        U[c] = (T)r;
        U[N + c] = (T)(r * ux);
        if (nd >= 2) U[2 * N + c] = (T)(r * uy);
        if (nd >= 3) U[3 * N + c] = (T)(r * uz);
        U[(1 + nd) * N + c] = (T)(e + ke);
        U[(2 + nd) * N + c] = (T)e;
    }
}

template <typename T> __global__ void k_from_double(const double *__restrict__ src, T *__restrict__ dst, long long n)
{
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (long long)gridDim.x * blockDim.x)
        dst[c] = (T)src[c];
}

template <typename T> __global__ void k_to_double(const T *__restrict__ src, double *__restrict__ dst, long long n)
{
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (long long)gridDim.x * blockDim.x)
        dst[c] = (double)src[c];
}

// Control block of a freshly set state: time t, vacuum reference density
// rho_mean0 (<= 0: left for the totals kernel to fill in).
__global__ void k_ctrl_reset(Ctrl *ctrl, double t, double rho_mean0)
{
    ctrl->t = t;
    ctrl->rho_mean0 = rho_mean0 > 0.0 ? rho_mean0 : 0.0;
    ctrl->tau = 0.0;
    ctrl->dt_last = 0.0;
    ctrl->vmax_bits[0] = ctrl->vmax_bits[1] = 0ull;
    ctrl->cmax_bits[0] = ctrl->cmax_bits[1] = 0ull;
    ctrl->steps = 0;
    ctrl->steps_left = 0;
    ctrl->dt_fixed = 0.0;
    ctrl->t_stop = 0.0;
    ctrl->err = 0;
    ctrl->slot_cur = 0;
    ctrl->slot_l = 0;
}

// Conserved ghost states of the inflow faces into the control block (set
// once per grid; by value, so that no host buffer is involved).
struct InflowTable {
    double v[6][6];
};
__global__ void k_set_inflow(Ctrl *ctrl, InflowTable tab)
{
    const int i = threadIdx.x;
    if (i < 36) ctrl->inflow[i / 6][i % 6] = tab.v[i / 6][i % 6];
}

// Parameters of the next run of steps of one grid.
__global__ void k_set_run(Ctrl *ctrl, double dt_fixed, double t_stop, long long nsteps)
{
    ctrl->dt_fixed = dt_fixed;
    ctrl->t_stop = t_stop;
    ctrl->steps_left = nsteps;
}

// Per-cell speeds |v| and c (Sec. 2.1) of a conserved state.
template <typename T, int NDIM>
__device__ __forceinline__ void cell_speeds(T r, T mx, T my, T mz, T e, T prho, T gam, T gm1, T &v, T &c)
{
#ifdef PPML_EXACT
    T ux = mx / r;
    T uy = NDIM >= 2 ? my / r : T(0);
    T uz = NDIM >= 3 ? mz / r : T(0);
    v = dsqrt(ux * ux + uy * uy + uz * uz);
    T p = prho * r + gm1 * e;
    c = dsqrt(gam * p / r);
#else
    const T ir = fast_rcp(r);
    T ux = mx * ir;
    T uy = NDIM >= 2 ? my * ir : T(0);
    T uz = NDIM >= 3 ? mz * ir : T(0);
    v = dsqrt(ux * ux + uy * uy + uz * uz);
    T p = prho * r + gm1 * e;
    c = dsqrt(gam * p * ir);
#endif
}

__device__ __forceinline__ void publish_max(Ctrl *ctrl, int slot, double v, double c)
{
    v = wave_max(v);
    c = wave_max(c);
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&ctrl->vmax_bits[slot], (unsigned long long)__double_as_longlong(v));
        atomicMax(&ctrl->cmax_bits[slot], (unsigned long long)__double_as_longlong(c));
    }
}

// Maxima of |v| and c over the state into the current slot (first step).
template <typename T, int NDIM>
__global__ void k_speeds(const T *__restrict__ U, GridParams gp, Ctrl *ctrl)
{
    const int slot = ctrl->slot_cur;
    const long long N = gp.ncell;
    const T gam = (T)gp.gs, gm1 = (T)gp.pb, prho = (T)gp.pa;
    double vm = 0.0, cm = 0.0;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (long long)gridDim.x * blockDim.x) {
        T r = U[c];
        T mx = U[N + c];
        T my = NDIM >= 2 ? U[2 * N + c] : T(0);
        T mz = NDIM >= 3 ? U[3 * N + c] : T(0);
        T e = U[(2 + NDIM) * N + c];
        T v, cs;
        cell_speeds<T, NDIM>(r, mx, my, mz, e, prho, gam, gm1, v, cs);
        vm = vm > (double)v ? vm : (double)v;
        cm = cm > (double)cs ? cm : (double)cs;
    }
    publish_max(ctrl, slot, vm, cm);
}

// Deterministic FP64 totals: fixed per-block ranges and fixed tree order.
constexpr int TOT_THREADS = 256;

template <typename T>
__global__ __launch_bounds__(TOT_THREADS) void k_totals_partial(const T *__restrict__ U, long long N, int nfs,
                                                                long long chunk, double *__restrict__ partial)
{
    __shared__ double red[TOT_THREADS];
    long long beg = (long long)blockIdx.x * chunk;
    long long end = beg + chunk < N ? beg + chunk : N;
    for (int f = 0; f < nfs; f++) {
        double s = 0.0;
        for (long long c = beg + threadIdx.x; c < end; c += TOT_THREADS) s += (double)U[f * N + c];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = TOT_THREADS / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[(long long)blockIdx.x * 6 + f] = red[0];
        __syncthreads();
    }
}

__global__ __launch_bounds__(TOT_THREADS) void k_totals_final(const double *__restrict__ partial, int nblocks, int nfs,
                                                              int ndim, double *__restrict__ out, Ctrl *ctrl,
                                                              double ncell_for_mean)
{
    __shared__ double red[TOT_THREADS];
    for (int f = 0; f < nfs; f++) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += TOT_THREADS) s += partial[(long long)b * 6 + f];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = TOT_THREADS / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            // stored field f -> ppml_field slot
            int slot = f == 0 ? 0 : (f <= ndim ? f : (f == ndim + 1 ? 4 : 5));
            out[slot] = red[0];
            if (f == 0 && ncell_for_mean > 0.0) ctrl->rho_mean0 = red[0] / ncell_for_mean;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int a = ndim; a < 3; a++) out[1 + a] = 0.0;
}

// ---------------------------------------------------------------------------
// Eulerian stage
// ---------------------------------------------------------------------------
// XF: 1 for grids with self-gravity, 2 for grids in the halo potential (with
// or without self-gravity); separate instantiations, so the loads of the
// self-gravity potential and the halo's arctangent cost the other grids no
// registers.
template <typename T, int NDIM, int TX, int TY, int XF = 0>
__device__ __forceinline__ void euler_body(const T *__restrict__ U, T *__restrict__ Wst, const GridParams &gp,
                                           Ctrl *ctrl, const int bx, const int by, const int bz, const bool lead)
{
    constexpr int NT = TX * TY;
    constexpr int NF = 3 + NDIM;
    constexpr int HX = GH;
    constexpr int HY = NDIM >= 2 ? GH : 0;
    constexpr int PW = TX + 2 * HX;
    constexpr int PH = TY + 2 * HY;
    constexpr int PS = PW * PH;
    constexpr int NXP = (TX + 2) * TY;
    constexpr int NYP = NDIM >= 2 ? TX * (TY + 2) : 1;
    // parabola jobs: runs of NC cells along x (rows of TX + 2 cells) or y
    // (columns of TY + 2); a line's last run starts early where NC does not
    // divide it, so it recomputes cells of the run before it (same values)
    constexpr int NC = NDIM == 1 ? 2 : 5;
    static_assert(TX + 2 >= NC && (NDIM < 2 || TY + 2 >= NC), "a run fits a line of the tile");
    constexpr int RXN = (TX + 2 + NC - 1) / NC;               // x runs per row
    constexpr int RYN = (TY + 2 + NC - 1) / NC;               // y runs per column
    constexpr int NXR = RXN * TY;                             // x runs of a field
    constexpr int NYR = NDIM >= 2 ? RYN * TX : 0;             // y runs of a field
    constexpr int NXI = (TX + 1) * TY;
    constexpr int NYI = NDIM >= 2 ? TX * (TY + 1) : 1;

    // The velocity and pressure tiles (read by the parabola jobs) and the
    // interface states (written by the Riemann jobs, read by the update) are
    // never live at once.  FP64 3-D overlays them where that lets three
    // waves per SIMD fit the CU's 160 KiB of LDS and keeping them apart does
    // not (16x16: 59.6 -> 50.9 KB), at the price of one barrier per plane
    // before the tiles are rewritten.  LDS is taken as granted in 2 KiB
    // steps: a 4-wave group of 53.9 KB measured two resident groups per CU,
    // not three.  FP32 3-D groups are held to four per CU by their
    // registers already.
    constexpr int NVY = NDIM >= 2 ? PS : 1;
    constexpr size_t B_TILE = ((size_t)(2 * PS + NVY) * sizeof(T) + 15) & ~(size_t)15;
    constexpr size_t B_IFACE = (size_t)(NXI + NYI) * sizeof(VP<T>);
    constexpr size_t B_REST = (size_t)3 * PS * sizeof(T) + (size_t)2 * (NXP + NYP) * sizeof(Profile<T>);
    constexpr size_t GROUPS3 = NT >= 64 ? (size_t)12 / (NT / 64) : 12;  // groups per CU for 3 waves/SIMD
    constexpr size_t B_SEP = (B_TILE + B_IFACE + B_REST + 2047) & ~(size_t)2047;
    constexpr size_t B_OVL = ((B_TILE > B_IFACE ? B_TILE : B_IFACE) + B_REST + 2047) & ~(size_t)2047;
    // 1-D and 2-D kernels hold few registers, so LDS alone decides how many
    // groups fit (up to 32 waves per CU): overlay where that adds a group
    constexpr size_t GMAX = NT >= 64 ? (size_t)32 / (NT / 64) : 32;
    constexpr size_t G_SEP = 163840 / B_SEP < GMAX ? 163840 / B_SEP : GMAX;
    constexpr size_t G_OVL = 163840 / B_OVL < GMAX ? 163840 / B_OVL : GMAX;
    constexpr bool OVERLAY = (sizeof(T) == 8 && GROUPS3 * B_OVL <= 163840 && GROUPS3 * B_SEP > 163840) ||
                             (NDIM <= 2 && G_OVL > G_SEP);
    constexpr size_t B_UNION = OVERLAY ? (B_TILE > B_IFACE ? B_TILE : B_IFACE) : B_TILE + B_IFACE;
    __shared__ __align__(16) unsigned char s_union[B_UNION];
    T *const s_vx = reinterpret_cast<T *>(s_union);
    T *const s_vy = s_vx + PS;
    T *const s_p = s_vy + NVY;
    VP<T> *const xi = reinterpret_cast<VP<T> *>(s_union + (OVERLAY ? 0 : B_TILE));
    VP<T> *const yi = xi + NXI;
    __shared__ T s_s[PS], s_r32[PS], s_ps[PS];
    __shared__ Profile<T> xv[NXP], xp[NXP];
    __shared__ Profile<T> yv[NYP], yp[NYP];

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int wv = wave_id(), ln = tid & 63;  // the wave (scalar) and the lane
    const int x0 = bx * TX, y0 = by * TY;
    const int nx = gp.n[0], ny = gp.n[1], nz = gp.n[2];
    const long long N = gp.ncell;

    const double tau_d = compute_tau(ctrl, gp);
    if (lead) {
        // publish the step for the Lagrangian kernel; a no-op step (tau = 0)
        // leaves the state, its maxima slot and the time unchanged
        const int s = ctrl->slot_cur;
        ctrl->slot_l = s;
        ctrl->tau = tau_d > 0.0 ? tau_d : 0.0;
        if (tau_d > 0.0) {
            ctrl->vmax_bits[s ^ 1] = 0ull;
            ctrl->cmax_bits[s ^ 1] = 0ull;
        }
    }
    if (!(tau_d > 0.0)) return;

    const T gam = (T)gp.gs;
    const T gm1 = (T)gp.pb;
    const T prho = (T)gp.pa;
    const T tau = (T)tau_d;
    const T hx = (T)gp.h[0], hy = (T)gp.h[1], hz = (T)gp.h[2];
    const T ihx = (T)gp.inv_h[0], ihy = (T)gp.inv_h[1], ihz = (T)gp.inv_h[2];
    const T tohx = (T)(tau_d * gp.inv_h[0]), tohy = (T)(tau_d * gp.inv_h[1]), tohz = (T)(tau_d * gp.inv_h[2]);
    (void)hz;
    (void)ihz;
    (void)tohz;
    (void)hy;
    (void)ihy;
    (void)tohy;

    const int gx = x0 + tx, gy = y0 + ty;
    const bool valid = gx < nx && (NDIM < 2 || gy < ny);
    int fdum;
    const int cx_ = map_index(gx, nx, gp.bc_lo[0], gp.bc_hi[0], fdum);
    const int cy_ = NDIM >= 2 ? map_index(gy, ny, gp.bc_lo[1], gp.bc_hi[1], fdum) : 0;

    int z0 = 0, z1 = 1;
    if constexpr (NDIM == 3) {
        z0 = bz * gp.cz;
        z1 = z0 + gp.cz < nz ? z0 + gp.cz : nz;
    }

    // per-field base pointers (uniform) and 32-bit cell offsets
    const T *Uf[NF];
    T *Wf[NF];
#pragma unroll
    for (int f = 0; f < NF; f++) {
        Uf[f] = U + (size_t)f * (size_t)N;
        Wf[f] = Wst + (size_t)f * (size_t)N;
    }
    const int plane = nx * ny;
    const int own_off = cy_ * nx + cx_;

    // Cross-tile cells this thread stages on every plane: (y, x) offset of
    // the boundary-mapped source cell (-1 where nothing is loaded) and the
    // momentum flips, two bits per cell.  Only the plane index changes along
    // z, so the maps are evaluated once.
    constexpr int RC = (PS + NT - 1) / NT;
    static_assert(2 * RC <= 16 && 16 + 3 * RC <= 32, "flip and inflow bits");
    int ccode[RC];
    unsigned flips = 0;
#pragma unroll
    for (int r = 0; r < RC; r++) {
        const int li = tid + r * NT;
        ccode[r] = -1;
        if (li < PS) {
            const int dx = li % PW - HX, dy = li / PW - HY;
            if ((dy >= 0 && dy < TY) || (dx >= 0 && dx < TX)) {
                int fx, fy = 0;
                const int ax = map_index(x0 + dx, nx, gp.bc_lo[0], gp.bc_hi[0], fx);
                const int ay = NDIM >= 2 ? map_index(y0 + dy, ny, gp.bc_lo[1], gp.bc_hi[1], fy) : 0;
                ccode[r] = ay * nx + ax;
                flips |= (unsigned)(fx | (fy << 1)) << (2 * r);
                if (gp.any_inflow) flips |= inflow_code_xy(gp, x0 + dx, y0 + dy, NDIM) << (16 + 3 * r);
            }
        }
    }

    // z pipeline registers (3-D): values of the thread's own column
    T qv0 = 1, qv1 = 1, qv2 = 1, qp0 = 1, qp1 = 1, qp2 = 1;  // q_{m-2}, q_{m-1}, q_m
    T dmv = 0, dmp = 0;                                      // slope at m-2
    T qIv = 1, qIp = 1;                                      // interface value (m-3)+1/2
#ifdef PPML_EXACT
    Profile<T> pv_prev = {1, 1, 0}, pp_prev = {1, 1, 0};     // profile of cell m-3
#else
    Profile<T> pv_prev = {0, 0, 1}, pp_prev = {0, 0, 1};
#endif
    T sr0 = 1, sr1 = 1, sr2 = 1, sr3 = 1;                    // sqrt(rho) at m-3..m
    T rr0 = 1, rr1 = 1, rr2 = 1, rr3 = 1;                    // rho^{3/2}
    T pr0 = 1, pr1 = 1, pr2 = 1, pr3 = 1;                    // p sqrt(rho)
    T Vprev = 0, Pprev = 0;

    const int m_beg = NDIM == 3 ? z0 - 3 : 0;
    const int m_end = NDIM == 3 ? z1 + 3 : 1;
    // FP32 3-D without a halo potential takes two planes per trip with the
    // two pairs of z profiles exchanged (every tile shape, so that they all
    // give the same bits); an odd count of planes starts one plane lower, whose
    // state reaches only warm-up planes.  Tiles of at least eight rows, which
    // hold the extra registers without spilling, also load the own column
    // one plane ahead, so that a plane's z arithmetic need not wait for
    // memory.  Otherwise one plane per trip.
    constexpr bool TWO = NDIM == 3 && sizeof(T) == 4 && XF <= 1;
    constexpr bool ZPRE = TWO && TY >= 8;
    if constexpr (TWO) {
        T zn0 = 1, zn1 = 1, zn2 = 1;  // rho, m_z, rho*eps of the column, one plane ahead
        int fzn = 0;
        auto load_column = [&](const int mm) {
            const int c = map_index(mm, nz, gp.bc_lo[2], gp.bc_hi[2], fzn) * plane + own_off;
            zn0 = Uf[0][c];
            zn1 = Uf[3][c];
            zn2 = Uf[5][c];
        };
        Profile<T> pvB = pv_prev, ppB = pp_prev;
        auto plane_step = [&](const int m, Profile<T> &pv_prev, Profile<T> &pp_prev, Profile<T> &pv_next,
                              Profile<T> &pp_next) __attribute__((always_inline)) {
            do {  // `continue` in the plane's body leaves it
#include "ppml_euler_plane.inc"
            } while (false);
        };
        const int m_first = (m_end - m_beg) & 1 ? m_beg - 1 : m_beg;
        if constexpr (ZPRE) load_column(m_first);
        for (int m = m_first; m < m_end; m += 2) {
            plane_step(m, pv_prev, pp_prev, pvB, ppB);
            plane_step(m + 1, pvB, ppB, pv_prev, pp_prev);
        }
    } else {
        // stand-ins for the names that only the body's two-plane branches use
        T zn0, zn1, zn2;
        int fzn;
        auto load_column = [](int) {};
        Profile<T> pv_next, pp_next;
        for (int m = m_beg; m < m_end; ++m) {
#include "ppml_euler_plane.inc"
        }
    }
}

// Waves per SIMD the register allocator aims for in the Eulerian kernel
// without self-gravity: four (<= 128 VGPRs) for FP32 3-D, three (<= 168)
// for FP64 3-D where its LDS tiles fit that many groups; the compiler's
// choice otherwise.
template <typename T, int NDIM, int XF> constexpr int euler_waves() { return NDIM == 3 && XF == 0 ? (sizeof(T) == 4 ? 4 : 3) : 1; }

template <typename T, int NDIM, int TX, int TY, int XF = 0>
__global__ __launch_bounds__(TX *TY) __attribute__((amdgpu_waves_per_eu(euler_waves<T, NDIM, XF>()))) void k_euler(
    const T *__restrict__ U, T *__restrict__ Wst, GridParams gp, Ctrl *ctrl)
{
    int bx, by, bz;
    block_tile(gp, bx, by, bz);
    euler_body<T, NDIM, TX, TY, XF>(U, Wst, gp, ctrl, bx, by, bz, blockIdx.x == 0 && threadIdx.x == 0);
}

// ---------------------------------------------------------------------------
// Lagrangian stage + energy correction + CFL maxima
// ---------------------------------------------------------------------------
// Transverse template of the interface velocity (Sec. 2.3): weights 1/16
// (corners), 1/8 (edges), 1/4 (centre) in 3-D, (1/4, 1/2, 1/4) in 2-D.
template <typename T>
__device__ __forceinline__ T tmpl9(T c11, T c1m, T cm1, T cmm, T e1a, T ema, T e1b, T emb, T ctr)
{
    T corners = c11 + c1m + cm1 + cmm;
    T edges = e1a + ema + e1b + emb;
    return T(0.0625) * corners + T(0.125) * edges + T(0.25) * ctr;
}
template <typename T> __device__ __forceinline__ T tmpl3(T vp, T vm, T ctr)
{
    return T(0.25) * (vp + vm) + T(0.5) * ctr;
}

template <typename T, int NDIM, int TX, int TY, int G>
__device__ __forceinline__ void lagr_body(const T *__restrict__ Wst, T *__restrict__ U, const GridParams &gp,
                                          Ctrl *ctrl, const int bx, const int by, const int bz, const bool lead)
{
    constexpr int NT = TX * TY;
    constexpr int NF = 3 + NDIM;
    constexpr int NPASS = (NF + G - 1) / G;
    constexpr int HX = GH;
    constexpr int HY = NDIM >= 2 ? GH : 0;
    constexpr int PW = TX + 2 * HX;
    constexpr int PH = TY + 2 * HY;
    constexpr int PS = PW * PH;
    // faces carrying interface values: x faces between tile-rel cells fx-2 and
    // fx-1 (fx = 0 .. TX+2), y faces between rows fy-2 and fy-1
    constexpr int NXQ = (TX + 3) * TY;
    constexpr int NYQ = NDIM >= 2 ? TX * (TY + 3) : 0;
    // flux interfaces: x between cells i-1 and i (i = 0 .. TX), y likewise
    constexpr int NXI = (TX + 1) * TY;
    constexpr int NYI = NDIM >= 2 ? TX * (TY + 1) : 0;
    constexpr int VW = TX + 2;
    constexpr int VH = NDIM >= 2 ? TY + 2 : 1;
    constexpr int VS = VW * VH;
    constexpr int NR = NDIM == 3 ? 3 : 1;

    // FP32 3-D: the cross tile of plane k+1 travels from memory straight to
    // LDS (one transfer per lane and field) while plane k is computed, into
    // the second of two tile buffers
    constexpr bool PIPE = sizeof(T) == 4 && NDIM == 3 && G >= NF;
    constexpr int NBUF = PIPE ? 2 : 1;
    // field slots of the tiles: G per pass, or all NF fields when they are
    // fewer (1-D and 2-D FP32), so that no slot of LDS goes unused
    constexpr int GL = G < NF ? G : NF;
    __shared__ T s_f[NBUF][GL][PS];
    __shared__ T s_qx[GL][NXQ];
    __shared__ T s_qy[GL][NYQ > 0 ? NYQ : 1];
    // fluxes reuse the interface-value arrays once those are consumed
    static_assert(NXI <= NXQ && NYI <= NYQ + 1, "flux arrays must fit in the face arrays");
    T (*s_Fx)[NXQ] = s_qx;
    T (*s_Fy)[NYQ > 0 ? NYQ : 1] = s_qy;
    __shared__ T s_vx[NR][VS];
    __shared__ T s_vy[NDIM >= 2 ? NR : 1][NDIM >= 2 ? VS : 1];
    // v_z is only needed on the newest plane; two slots alternate so that a
    // plane's slot is never rewritten while the previous one is being read
    __shared__ T s_vz[NDIM == 3 ? 2 : 1][NDIM == 3 ? VS : 1];

    const double tau_d = ctrl->tau;
    if (!(tau_d > 0.0)) return;
    const int tid = threadIdx.x;
    const int sl = ctrl->slot_l;
    if (lead) {
        ctrl->t = ctrl->t + tau_d;
        ctrl->dt_last = tau_d;
        ctrl->steps = ctrl->steps + 1;
        ctrl->steps_left = ctrl->steps_left - 1;
        ctrl->slot_cur = sl ^ 1;
    }
    const int tx = tid % TX, ty = tid / TX;
    const int wv = wave_id(), ln = tid & 63;  // the wave (scalar) and the lane
    const int x0 = bx * TX, y0 = by * TY;
    const int nx = gp.n[0], ny = gp.n[1], nz = gp.n[2];
    const long long N = gp.ncell;
    const T gam = (T)gp.gs;
    const T gm1 = (T)gp.pb;
    const T prho = (T)gp.pa;
    const T tau = (T)tau_d;
    const T hx = (T)gp.h[0], hy = (T)gp.h[1], hz = (T)gp.h[2];
    const T ihx = (T)gp.inv_h[0], ihy = (T)gp.inv_h[1], ihz = (T)gp.inv_h[2];
    const T tohx = (T)(tau_d * gp.inv_h[0]), tohy = (T)(tau_d * gp.inv_h[1]), tohz = (T)(tau_d * gp.inv_h[2]);
    (void)hy; (void)ihy; (void)tohy; (void)hz; (void)ihz; (void)tohz; (void)tohx; (void)hx; (void)ihx; (void)tau;
    const double thr = gp.vacuum_ratio * ctrl->rho_mean0;

    const int gx = x0 + tx, gy = y0 + ty;
    const bool valid = gx < nx && (NDIM < 2 || gy < ny);
    int fdum;
    const int cx_ = map_index(gx, nx, gp.bc_lo[0], gp.bc_hi[0], fdum);
    const int cy_ = NDIM >= 2 ? map_index(gy, ny, gp.bc_lo[1], gp.bc_hi[1], fdum) : 0;

    int z0 = 0, z1 = 1;
    if constexpr (NDIM == 3) {
        z0 = bz * gp.cz;
        z1 = z0 + gp.cz < nz ? z0 + gp.cz : nz;
    }

    // per-field base pointers (uniform) and 32-bit cell offsets
    const T *Wf[NF];
#pragma unroll
    for (int f = 0; f < NF; f++) Wf[f] = Wst + (size_t)f * (size_t)N;
    const int plane = nx * ny;
    const int own_off = cy_ * nx + cx_;

    // Tile cells this thread stages on every plane: the (y, x) offset of the
    // boundary-mapped source cell (-1 where nothing is loaded), the momentum
    // flips, two bits per cell (x, y) from bit 0, and the inflow code of the
    // cell, three bits per cell from bit 16.  Only the plane index changes
    // along z, so the maps are evaluated once.
    constexpr int RC = (PS + NT - 1) / NT;
    constexpr int RV = (VS + NT - 1) / NT;
    static_assert(2 * (RC + RV) <= 16 && 16 + 3 * (RC + RV) <= 32, "flip and inflow bits");
    int ccode[RC], vcode[RV];
    unsigned flips = 0;
#pragma unroll
    for (int r = 0; r < RC; r++) {
        const int li = tid + r * NT;
        ccode[r] = -1;
        if (li < PS) {
            const int dx = li % PW - HX, dy = li / PW - HY;
            if ((dy >= 0 && dy < TY) || (dx >= 0 && dx < TX)) {
                int fx, fy = 0;
                const int ax = map_index(x0 + dx, nx, gp.bc_lo[0], gp.bc_hi[0], fx);
                const int ay = NDIM >= 2 ? map_index(y0 + dy, ny, gp.bc_lo[1], gp.bc_hi[1], fy) : 0;
                ccode[r] = ay * nx + ax;
                flips |= (unsigned)(fx | (fy << 1)) << (2 * r);
                if (gp.any_inflow) flips |= inflow_code_xy(gp, x0 + dx, y0 + dy, NDIM) << (16 + 3 * r);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < RV; r++) {
        const int li = tid + r * NT;
        vcode[r] = -1;
        if (li < VS) {
            int fx, fy = 0;
            const int ax = map_index(x0 + li % VW - 1, nx, gp.bc_lo[0], gp.bc_hi[0], fx);
            const int ay = NDIM >= 2 ? map_index(y0 + li / VW - 1, ny, gp.bc_lo[1], gp.bc_hi[1], fy) : 0;
            vcode[r] = ay * nx + ax;
            flips |= (unsigned)(fx | (fy << 1)) << (2 * (RC + r));
            if (gp.any_inflow)
                flips |= inflow_code_xy(gp, x0 + li % VW - 1, y0 + li / VW - 1, NDIM) << (16 + 3 * (RC + r));
        }
    }

    // z pipeline registers (3-D), one set per field.  The profile of the
    // previous cell: its parabola in the exact build, its value and
    // monotonised one-sided jumps in the product build.
    using Prof = Profile<T>;
#ifdef PPML_EXACT
    const Prof prof_one{T(1), T(1), T(0)};
#else
    const Prof prof_one{T(0), T(0), T(1)};
#endif
    T q0[NF], q1[NF], q2[NF], dmq[NF], qI[NF], Fzp[NF];
    Prof pprev[NF];
#pragma unroll
    for (int f = 0; f < NF; f++) {
        q0[f] = q1[f] = q2[f] = T(1);
        dmq[f] = T(0);
        qI[f] = T(1);
        Fzp[f] = T(0);
        pprev[f] = prof_one;
    }
    T sz0 = 1, sz1 = 1, sz2 = 1, sz3 = 1;  // sqrt(rho) of the column at m-3..m
    T vtz_prev = 0;                        // transverse velocity of the column at m-3
    T vmax = T(0), cmax = T(0);  // running maxima (FP64 only once published)

    const int m_beg = NDIM == 3 ? z0 - 3 : 0;
    const int m_end = NDIM == 3 ? z1 + 3 : 1;

    // cross tile of plane kk, every field, from memory into the LDS buffer of
    // plane kk: each wave fills 64 consecutive tile slots per field, lanes
    // without a cross cell do not transfer
    auto dma_cross = [&](int kk) {
        T (*dst)[PS] = s_f[kk & 1];
#pragma unroll
        for (int r = 0; r < RC; r++) {
            if (ccode[r] < 0) continue;
            const int c = kk * plane + ccode[r];
            const int wbase = r * NT + wv * 64;  // the wave's first slot (scalar)
#pragma unroll
            for (int f = 0; f < NF; f++)
                __builtin_amdgcn_global_load_lds((const void *)(Wf[f] + c),
                                                 (__attribute__((address_space(3))) void *)&dst[f][wbase], 4, 0, 0);
        }
    };
    if constexpr (PIPE) dma_cross(z0);
    // the cross tile of plane kk arrived by transfer: once this wave's
    // transfers have landed, each thread mirrors the normal momenta at
    // reflecting faces and writes the state of inflow faces into the slots
    // it owns (every slot it owns was moved by its own wave)
    auto fix_cross = [&](int kk) {
        T (*sf)[PS] = s_f[kk & 1];
        __builtin_amdgcn_s_waitcnt(VMCNT0);
        if (flips & 0xFFFFu) {
#pragma unroll
            for (int r = 0; r < RC; r++) {
                if (ccode[r] < 0) continue;
                const int li = tid + r * NT;
                const unsigned fl = flips >> (2 * r);
                if (fl & 1) sf[1][li] = -sf[1][li];
                if (NDIM >= 2 && (fl & 2)) sf[2][li] = -sf[2][li];
            }
        }
        if (gp.any_inflow) {
            // ghosts of inflow faces take the face's state (after an x face
            // only a y reflection applies)
#pragma unroll 1
            for (int r = 0; r < RC; r++) {
                const unsigned io = (flips >> (16 + 3 * r)) & 7u;
                if (ccode[r] < 0 || io == 0) continue;
                const int li = tid + r * NT;
                const bool fly = io < 3 && ((flips >> (2 * r)) & 2u);
#pragma unroll 1
                for (int f = 0; f < NF; f++) {
                    const T v = inflow_value<T>(ctrl, io - 1, inflow_component<NDIM>(f));
                    sf[f][li] = (f == 2 && fly) ? -v : v;
                }
            }
        }
    };
    (void)fix_cross;

    // FP32 3-D takes two planes per trip with the two sets of profiles of
    // the previous cell exchanged, so that no profile is copied from one
    // plane to the next; an odd count of planes starts one plane lower, whose
    // state reaches only warm-up planes.  Otherwise one plane per trip and a
    // copy of the new profiles.
    constexpr bool TWO = NDIM == 3 && sizeof(T) == 4;
    if constexpr (TWO) {
        Prof pB[NF];
        auto plane_step = [&](const int m, Prof(&pprev)[NF], Prof(&pnew)[NF]) __attribute__((always_inline)) {
            do {  // `continue` in the plane's body leaves it
#include "ppml_lagr_plane.inc"
            } while (false);
        };
        for (int m = (m_end - m_beg) & 1 ? m_beg - 1 : m_beg; m < m_end; m += 2) {
            plane_step(m, pprev, pB);
            plane_step(m + 1, pB, pprev);
        }
    } else {
        for (int m = m_beg; m < m_end; ++m) {
            Prof pnew[NF];
            (void)pnew;
#include "ppml_lagr_plane.inc"
        }
    }
    publish_max(ctrl, sl ^ 1, (double)vmax, (double)cmax);
}

// Waves per SIMD the register allocator aims for in the Lagrangian kernel:
// three 4-wave work groups per CU (<= 168 VGPRs) for the FP32 3-D kernel,
// whose LDS tiles also fit three times; two (<= 256 registers, so that no
// accumulation register halves the occupancy) for the FP64 3-D kernel; the
// compiler's choice otherwise.
template <typename T, int NDIM> constexpr int lagr_waves() { return NDIM == 3 ? (sizeof(T) == 4 ? 3 : 2) : 1; }

template <typename T, int NDIM, int TX, int TY, int G>
__global__ __launch_bounds__(TX *TY) __attribute__((amdgpu_waves_per_eu(lagr_waves<T, NDIM>()))) void k_lagr(const T *__restrict__ Wst, T *__restrict__ U, GridParams gp,
                                                  Ctrl *ctrl)
{
    int bx, by, bz;
    block_tile(gp, bx, by, bz);
    lagr_body<T, NDIM, TX, TY, G>(Wst, U, gp, ctrl, bx, by, bz, blockIdx.x == 0 && threadIdx.x == 0);
}

// ---------------------------------------------------------------------------
// Batched launches: many independent grids of one dimensionality step in the
// same two kernel launches.  Each work group finds its grid in a table sorted
// by first tile; every grid keeps its own control block (time step, time,
// CFL maxima), so a grid's results do not depend on the other grids.
// ---------------------------------------------------------------------------
struct BatchEntry {
    GridParams gp;
    const void *state;
    void *half;
    Ctrl *ctrl;
    int tile0;   // first work group of this grid in the launch
    int pad;
};

__device__ __forceinline__ int batch_entry(const BatchEntry *__restrict__ ents, int ne, int b)
{
    int lo = 0, hi = ne - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ents[mid].tile0 <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <typename T, int NDIM, int TX, int TY>
__global__ __launch_bounds__(TX *TY) __attribute__((amdgpu_waves_per_eu(euler_waves<T, NDIM, 0>()))) void k_euler_batch(
    const BatchEntry *__restrict__ ents, int ne)
{
    const BatchEntry *e = ents + batch_entry(ents, ne, blockIdx.x);
    const int L = blockIdx.x - e->tile0;
    int bx, by, bz;
    tile_decode(e->gp, L, bx, by, bz);
    euler_body<T, NDIM, TX, TY>((const T *)e->state, (T *)e->half, e->gp, e->ctrl, bx, by, bz,
                                L == 0 && threadIdx.x == 0);
}

template <typename T, int NDIM, int TX, int TY, int G>
__global__ __launch_bounds__(TX *TY) __attribute__((amdgpu_waves_per_eu(lagr_waves<T, NDIM>()))) void k_lagr_batch(const BatchEntry *__restrict__ ents, int ne)
{
    const BatchEntry *e = ents + batch_entry(ents, ne, blockIdx.x);
    const int L = blockIdx.x - e->tile0;
    int bx, by, bz;
    tile_decode(e->gp, L, bx, by, bz);
    lagr_body<T, NDIM, TX, TY, G>((const T *)e->half, (T *)e->state, e->gp, e->ctrl, bx, by, bz,
                                  L == 0 && threadIdx.x == 0);
}

// Run parameters of every grid of a batch (steps[i] < 0: same as nsteps).
__global__ void k_batch_set_run(const BatchEntry *__restrict__ ents, int ne, const int *__restrict__ steps,
                                double dt_fixed, double t_stop)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ne) return;
    Ctrl *c = ents[i].ctrl;
    c->dt_fixed = dt_fixed;
    c->t_stop = t_stop;
    c->steps_left = steps[i];
}

}  // namespace ppml
