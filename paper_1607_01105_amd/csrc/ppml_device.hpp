// ppml_device.hpp -- device-side building blocks of the PPML update for
// gfx950 (CDNA4): parameters, boundary index maps, parabola construction
// (Appendix, steps 1-3), characteristic averages (Appendix), the
// modified-Roe acoustic Riemann solver (Sec. 2.1-2.2) and the upwind
// parabolic flux (Sec. 2.3).
//
// Arithmetic notes.  With PPML_EXACT defined the build uses no FMA
// contraction and divides wherever the scheme's formulas divide, in the
// formulas' own operation order, so an FP64 build reproduces an
// IEEE-754 evaluation of the formulas operation by operation.  The normal
// build lets the compiler contract multiply-adds and replaces divisions by
// constants and cell sizes with multiplications by precomputed inverses.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ppml {

enum { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_REFLECT = 2, BC_INFLOW = 3 };
enum { POT_NONE = 0, POT_LOG = 1, POT_UNIFORM = 2, POT_HALO = 3 };
constexpr int GH = 3;  // ghost layers: a cell update reads q[i-3 .. i+3]

// Per-grid constants passed by value to every kernel.
struct GridParams {
    int ndim;
    int n[3];
    long long ncell;
    double h[3], inv_h[3];
    double lo[3];
    double gamma;         // ratio of specific heats (state conversions)
    double pa, pb;        // pressure p = pa rho + pb rho eps: (0, gamma - 1), or
                          // (cs^2, 0) in the isothermal variant; pb is also the
                          // factor of the eps equation's work term
    double gs;            // gamma of the sound speeds (1 in the isothermal variant)
    double cfl_hmin;      // cfl * min over active axes of h
    double vacuum_ratio;  // threshold relative to the initial mean density
    int bc_lo[3], bc_hi[3];
    int potential;
    double pot[8];
    int first_order;  // 1: piecewise-constant states (first-order scheme of Sec. 2.1)
    int tiles[3];  // work-group tiles along x, y and z chunks of the stage kernels
    int cz;        // planes per z chunk (3-D)
    int any_inflow;  // some face has an inflow boundary (states in Ctrl::inflow)
    int self_grav;   // 1: the force includes the gradient of the self-gravity potential
    const void *phi; // that potential (storage type): interior cells plus a one-cell
                     // shell, C order [k+1][j+1][i+1] with extents n+2
};

// Device control block of one grid (lives in the scratch area).  Every
// field is written by one thread of one kernel and read by the next kernel
// on the stream, never by another work group of the kernel that writes it:
// the Eulerian kernel reads slot_cur, t and the run parameters and writes
// tau, slot_l and the other maxima slot; the Lagrangian kernel reads tau and
// slot_l and writes t, the step counters and slot_cur.
struct Ctrl {
    double t;             // simulation time
    double tau;           // time step of the step in flight (0: no-op step)
    double rho_mean0;     // FP64 initial mean density (vacuum reference)
    double dt_last;       // last time step taken
    unsigned long long vmax_bits[2];  // max |v| of a state, as FP64 bits (two slots)
    unsigned long long cmax_bits[2];  // max c, as FP64 bits
    long long steps;      // steps taken
    long long steps_left; // steps the current run may still take
    double dt_fixed;      // run parameter: > 0 fixed time step
    double t_stop;        // run parameter: > 0 end time
    int err;              // sticky error word (bit 0: non-physical state)
    int slot_cur;         // slot holding the maxima of the current state
    int slot_l;           // slot_cur of the step in flight (for the Lagrangian kernel)
    int pad;
    double inflow[6][6];  // conserved ghost state of inflow face 2*axis+side (set once)
    double mom[8];        // mass and second moments of the state (self-gravity boundary values)
};

#ifdef PPML_EXACT
#define PPML_DIV(a, b, inv_b) ((a) / (b))
#else
#define PPML_DIV(a, b, inv_b) ((a) * (inv_b))
#endif

template <typename T> struct K {
    static constexpr T half = T(0.5);
    static constexpr T two = T(2);
    static constexpr T three = T(3);
    static constexpr T six = T(6);
    static constexpr T inv3 = T(1) / T(3);
    static constexpr T inv12 = T(1) / T(12);
};

__device__ __forceinline__ float dsqrt(float x) { return __builtin_sqrtf(x); }
__device__ __forceinline__ double dsqrt(double x) { return __builtin_sqrt(x); }
__device__ __forceinline__ float dabs(float x) { return __builtin_fabsf(x); }
__device__ __forceinline__ double dabs(double x) { return __builtin_fabs(x); }
__device__ __forceinline__ float dcopysign(float m, float s) { return __builtin_copysignf(m, s); }
__device__ __forceinline__ double dcopysign(double m, double s) { return __builtin_copysign(m, s); }
__device__ __forceinline__ float dmin(float a, float b) { return __builtin_fminf(a, b); }
// median of a, b and 0
__device__ __forceinline__ float med0(float a, float b) { return __builtin_amdgcn_fmed3f(a, b, 0.0f); }
__device__ __forceinline__ double med0(double a, double b)
{
    return __builtin_fmax(__builtin_fmin(a, b), __builtin_fmin(__builtin_fmax(a, b), 0.0));
}
__device__ __forceinline__ double dmin(double a, double b) { return __builtin_fmin(a, b); }

// Reciprocal and reciprocal square root of a positive normal value for the
// product build: FP32 the hardware estimates (about 1 ulp, as the build's
// FP32 division and square root); FP64 the hardware estimate refined by two
// Newton steps (within a few ulp; the correctly rounded FP64 division and
// square root cost about three times as many instructions).
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fast_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double fast_rcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
    r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
    return r;
}
__device__ __forceinline__ double fast_rsqrt(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    y = y * __builtin_fma(-hx * y, y, 1.5);
    y = y * __builtin_fma(-hx * y, y, 1.5);
    return y;
}

// Index of the interior cell that supplies the value at index i (which may
// lie in a ghost layer or, for cells of a partial tile, further out) along
// an axis of n cells; flip = 1 when the wall-normal momentum changes sign.
__device__ __forceinline__ int map_index(int i, int n, int bclo, int bchi, int &flip)
{
    flip = 0;
    if (i < 0) {
        if (bclo == BC_PERIODIC) {
            int r = i % n;
            return r < 0 ? r + n : r;
        }
        if (bclo == BC_OUTFLOW || bclo == BC_INFLOW) return 0;  // inflow: value replaced
        flip = 1;
        int r = -1 - i;
        return r < n ? r : n - 1;
    }
    if (i >= n) {
        if (bchi == BC_PERIODIC) return i % n;
        if (bchi == BC_OUTFLOW || bchi == BC_INFLOW) return n - 1;
        flip = 1;
        int r = 2 * n - 1 - i;
        return r >= 0 ? r : 0;
    }
    return i;
}

// Inflow face (2*axis + side) whose prescribed state the ghost index i takes
// along an axis, or -1.  Ghost layers are filled axis by axis (x, y, z), so a
// cell that is a ghost along several axes takes the state of the last inflow
// axis, with the wall-normal momentum of later reflecting axes negated.
__device__ __forceinline__ int inflow_face(int i, int n, int bclo, int bchi, int axis)
{
    if (i < 0 && bclo == BC_INFLOW) return 2 * axis;
    if (i >= n && bchi == BC_INFLOW) return 2 * axis + 1;
    return -1;
}

// Component q (0 rho, 1-3 rho v_x..z, 4 rho E, 5 rho eps) of the prescribed
// state of inflow face `face` (read from the control block only on the rare
// ghost cells of inflow faces).
template <typename T> __device__ __forceinline__ T inflow_value(const Ctrl *ctrl, int face, int q)
{
    return (T)ctrl->inflow[face][q];
}

// Component of the inflow state for stored field f of a grid of NDIM
// dimensions (fields rho, rho v_0 .. rho v_{NDIM-1}, rho E, rho eps).
template <int NDIM> __device__ __forceinline__ int inflow_component(int f) { return f <= NDIM ? f : f + (3 - NDIM); }

// Inflow code of a staged cell (x, y of a plane): 0 none, else 1 + the face
// of the last inflow axis among x and y.
__device__ __forceinline__ unsigned inflow_code_xy(const GridParams &gp, int i, int j, int ndim)
{
    const int fx = inflow_face(i, gp.n[0], gp.bc_lo[0], gp.bc_hi[0], 0);
    const int fy = ndim >= 2 ? inflow_face(j, gp.n[1], gp.bc_lo[1], gp.bc_hi[1], 1) : -1;
    return fy >= 0 ? (unsigned)(fy + 1) : (fx >= 0 ? (unsigned)(fx + 1) : 0u);
}

// Appendix step 1: limited slope delta_m q of the middle value.  The product
// build returns 2 delta_m q, the form interface_value takes there.
template <typename T> __device__ __forceinline__ T limited_slope(T qm, T q0, T qp)
{
#ifdef PPML_EXACT
    T dq = K<T>::half * (qp - qm);
    T dplus = qp - q0;
    T dminus = q0 - qm;
    T m = dmin(dabs(dq), dmin(K<T>::two * dabs(dplus), K<T>::two * dabs(dminus)));
    return (dplus * dminus > T(0)) ? dcopysign(m, dq) : T(0);
#else
    // With d+ = qp - q0, d- = q0 - qm: med(d+, d-, 0) is 0 unless d+ d- > 0,
    // and then the one of the two nearer 0, so 4 med(d+, d-, 0) is the limit
    // 2 min(|d+|, |d-|), doubled and signed; the median of it, 2 dq = qp - qm
    // and 0 is twice the limited slope.  Every scaling is by a power of two,
    // so the result is exactly twice the paper's slope (barring underflow of
    // the product d+ d-).
    return med0(qp - qm, T(4) * med0(qp - q0, q0 - qm));
#endif
}

// Appendix step 1: fourth-order interface value between q0 and q1 from the
// limited slopes of the two cells (product build: twice the slopes).
template <typename T> __device__ __forceinline__ T interface_value(T q0, T q1, T dm0, T dm1)
{
#ifdef PPML_EXACT
    return K<T>::half * (q0 + q1) - (dm1 - dm0) / K<T>::six;
#else
    return K<T>::half * (q0 + q1) - (dm1 - dm0) * K<T>::inv12;
#endif
}

// Appendix steps 2-3: monotonize the parabola of a cell with value c and
// edge values l, r; returns (L, R, Q6) with Q6 = 6 (c - (L + R)/2).  The
// jump across the cell is R - L.
template <typename T> struct Parab {
    T L, R, Q6;
};

template <typename T> __device__ __forceinline__ Parab<T> monotonize(T c, T l, T r)
{
    if ((r - c) * (c - l) <= T(0)) {
        l = c;
        r = c;
    } else {
        T d = r - l;
        T s6 = K<T>::six * (c - K<T>::half * (l + r));
        T ds = d * s6, dd = d * d;
        if (ds > dd)
            l = K<T>::three * c - K<T>::two * r;
        else if (ds < -dd)
            r = K<T>::three * c - K<T>::two * l;
    }
    Parab<T> p;
    p.L = l;
    p.R = r;
    p.Q6 = K<T>::six * (c - K<T>::half * (l + r));
    return p;
}

// The first-order scheme's constant state (Sec. 2.1) in place of the
// parabola p of a cell of value c.  Selected after the parabola is built, so
// that the choice is a select rather than a branch between the fields.
template <typename T> __device__ __forceinline__ Parab<T> pick_profile(int first_order, T c, const Parab<T> &p)
{
    const bool fo = first_order != 0;
    return Parab<T>{fo ? c : p.L, fo ? c : p.R, fo ? T(0) : p.Q6};
}

// Product build: a cell's monotonised profile as its value and its one-sided
// jumps dl = c - L, dr = R - c.  In these terms the rules of monotonize are:
// jumps of different sign, or a zero jump, flatten the cell; otherwise a jump
// larger than twice the other is cut to twice the other.  The median of
// (d, 2 d_other, 0) applies all of them at once: it is 0 when d and d_other
// differ in sign, and otherwise whichever of d and 2 d_other is nearer to 0.
template <typename T> struct Jumps {
    T dl, dr, c;
};
template <typename T> __device__ __forceinline__ Jumps<T> mono_jumps(T c, T l, T r)
{
    const T dl = c - l, dr = r - c;
    return Jumps<T>{med0(dl, dr + dr), med0(dr, dl + dl), c};
}

// State profile of a cell: the monotonised parabola, or the constant cell
// value in the first-order scheme, in the exact build; the value and the
// monotonised jumps in the product build, whose strip means apply the
// first-order scheme through their weights.
#ifdef PPML_EXACT
template <typename T> using Profile = Parab<T>;
#else
template <typename T> using Profile = Jumps<T>;
#endif
template <typename T> __device__ __forceinline__ Profile<T> profile(int first_order, T c, T l, T r)
{
#ifdef PPML_EXACT
    return pick_profile(first_order, c, monotonize(c, l, r));
#else
    (void)first_order;
    return mono_jumps(c, l, r);
#endif
}

// Profiles of NC consecutive cells of a line, q[0], q[S], ..., q[(NC - 1) S]
// (values q[-2 S] .. q[(NC + 1) S]), written to out[0], out[OS], ...: each
// slope and interface value is built once and serves the cells on both of
// its sides, and each profile comes from its cell's three slopes and two
// interface values by the same operations as on its own.
template <int NC, int S, int OS, typename T>
__device__ __forceinline__ void parabola_run(int first_order, const T *q, Profile<T> *out)
{
    T v[NC + 4];  // cells -2 .. NC + 1
#pragma unroll
    for (int i = 0; i < NC + 4; i++) v[i] = q[(i - 2) * S];
    T sl[NC + 2];  // limited slopes of cells -1 .. NC
#pragma unroll
    for (int i = 0; i < NC + 2; i++) sl[i] = limited_slope(v[i], v[i + 1], v[i + 2]);
    T iv[NC + 1];  // interface values between cells i - 1 and i, i = 0 .. NC
#pragma unroll
    for (int i = 0; i <= NC; i++) iv[i] = interface_value(v[i + 1], v[i + 2], sl[i], sl[i + 1]);
#pragma unroll
    for (int i = 0; i < NC; i++) out[i * OS] = profile(first_order, v[i + 2], iv[i], iv[i + 1]);
}

// Appendix: mean of a cell's parabola over the strip of z*h next to its
// right edge (q_L(-lambda t)) and next to its left edge (q_R(lambda t)).
template <typename T> __device__ __forceinline__ T curv_weight(T z)
{
#ifdef PPML_EXACT
    return T(1) - (K<T>::two * z) / K<T>::three;
#else
    return T(1) - (K<T>::two * z) * K<T>::inv3;
#endif
}
template <typename T> __device__ __forceinline__ T avg_left(T L, T R, T Q6, T z)
{
    T d = R - L;
    T w = curv_weight(z);
    return R - (K<T>::half * z) * (d - Q6 * w);
}
template <typename T> __device__ __forceinline__ T avg_right(T L, T R, T Q6, T z)
{
    T d = R - L;
    T w = curv_weight(z);
    return L + (K<T>::half * z) * (d + Q6 * w);
}

// Sec. 2.1-2.2: acoustic Riemann problem at the interface between cells a
// (left) and b (right).  s = sqrt(rho), r32 = rho * s, ps = p * s are the
// cell-centre values; (vL, pL) and (vR, pR) the parabolas of the normal
// velocity and the pressure of the two cells.  Returns V and P.
template <typename T> struct VP {
    T V, P;
};

template <typename T>
__device__ __forceinline__ VP<T> riemann(int first_order, T sa, T sb, T r32a, T r32b, T psa, T psb,
                                         const Profile<T> &va, const Profile<T> &vb, const Profile<T> &pa,
                                         const Profile<T> &pb, T gamma, T tau, T h, T tau_over_h)
{
    T A = r32a + r32b;
    T B = sa + sb;
    T C = psa + psb;
#ifdef PPML_EXACT
    T lam = dsqrt(gamma * C / A);
    T Z = dsqrt(gamma * A * C) / B;
    T z = lam * tau / h;
#else
    // the same quantities from three reciprocal estimates instead of three
    // divisions and two square roots: q = lambda^2 = gamma C / A,
    // lambda = q / sqrt(q), Z = sqrt(gamma A C) / B = A lambda / B, and
    // 1 / Z = B / (A lambda)
    (void)tau;
    (void)h;
    const T iA = fast_rcp(A);
    const T q = gamma * C * iA;
    const T rl = fast_rsqrt(q);
    T lam = q * rl;
    T Z = A * lam * fast_rcp(B);
    const T iZ = B * iA * rl;
    T z = lam * tau_over_h;
#endif
#ifdef PPML_EXACT
    (void)first_order;
    T vm = avg_left(va.L, va.R, va.Q6, z);
    T vp = avg_right(vb.L, vb.R, vb.Q6, z);
    T pm = avg_left(pa.L, pa.R, pa.Q6, z);
    T pp = avg_right(pb.L, pb.R, pb.Q6, z);
#else
    // the strip means in terms of the monotonised jumps (L = c - dl,
    // R = c + dr, Q6 = 3 (dl - dr)): next to the right edge of the left cell
    // c + (1 - z)^2 dr + z (1 - z) dl, next to the left edge of the right
    // cell c - (1 - z)^2 dl - z (1 - z) dr; both weights vanish for the
    // first-order constant states
    const T y = T(1) - z;
    const T wn = first_order != 0 ? T(0) : y * y, wf = first_order != 0 ? T(0) : z * y;
    T vm = va.c + (wn * va.dr + wf * va.dl);
    T vp = vb.c - (wn * vb.dl + wf * vb.dr);
    T pm = pa.c + (wn * pa.dr + wf * pa.dl);
    T pp = pb.c - (wn * pb.dl + wf * pb.dr);
#endif
    VP<T> o;
#ifdef PPML_EXACT
    o.V = K<T>::half * (vm + vp) + (pm - pp) / (K<T>::two * Z);
#else
    o.V = K<T>::half * (vm + vp) + (pm - pp) * (K<T>::half * iZ);
#endif
    o.P = K<T>::half * (pm + pp) + (K<T>::half * Z) * (vm - vp);
    return o;
}

// Sec. 2.3: upwind flux of one field through an interface with velocity vh;
// a is the cell on the left, b on the right.
template <typename T> __device__ __forceinline__ T upwind_flux(T vh, T z, const Parab<T> &a, const Parab<T> &b)
{
    T fs = (vh >= T(0)) ? avg_left(a.L, a.R, a.Q6, z) : avg_right(b.L, b.R, b.Q6, z);
    return vh * fs;
}

// Weights of the upwind flux through a face, vs = v tau / h, z = |vs|.  With
// the strip mean written as c plus the weighted edge offsets (the weights
// (1 - z)^2, z (z - 1), z (3 - 2 z) sum to 1), the flux times tau / h is
//   vs c + a dr + b dl,
// a = z (1 - z)^2, b = z^2 (1 - z) when the upwind cell is on the left, and
// the two swapped when it is on the right.  The first-order scheme's constant
// state has a = b = 0.
template <typename T> struct FaceW {
    T vs, a, b;
};
template <typename T> __device__ __forceinline__ FaceW<T> face_weights(int first_order, bool left, T vs)
{
    const T z = first_order != 0 ? T(0) : dabs(vs);
    const T zy = z * (T(1) - z);
    const T p = zy * (T(1) - z), q = zy * z;
    return FaceW<T>{vs, left ? p : q, left ? q : p};
}
template <typename T> __device__ __forceinline__ T face_flux(const FaceW<T> &w, const Jumps<T> &u)
{
    return w.vs * u.c + (w.a * u.dr + w.b * u.dl);
}

// Density-weighted interface velocity (Sec. 2.3).
template <typename T> __device__ __forceinline__ T interface_velocity(T va, T sa, T vb, T sb)
{
#ifdef PPML_EXACT
    return (va * sa + vb * sb) / (sa + sb);
#else
    return (va * sa + vb * sb) * fast_rcp(sa + sb);
#endif
}

// Gradient of the fixed potential at a cell centre (eqs. (2)-(3) force terms).
// XF = 2: the instantiation for halo grids, the only one that evaluates the
// halo (its arctangent would cost the other grids registers).
template <int XF>
__device__ __forceinline__ void potential_grad(const GridParams &gp, int i, int j, int k, double g[3])
{
    double x = gp.lo[0] + ((double)i + 0.5) * gp.h[0];
    double y = gp.lo[1] + ((double)j + 0.5) * gp.h[1];
    double z = gp.lo[2] + ((double)k + 0.5) * gp.h[2];
    if (gp.potential == POT_LOG) {
        double v0 = gp.pot[0], rc = gp.pot[1], q = gp.pot[2];
        double X = x - gp.pot[3], Y = y - gp.pot[4], Z = z - gp.pot[5];
        double q2 = q * q;
        double den = rc * rc + X * X + Y * Y + Z * Z / q2;
        double a = v0 * v0 / den;
        g[0] = a * X;
        g[1] = a * Y;
        g[2] = a * (Z / q2);
    } else if (gp.potential == POT_UNIFORM) {
        g[0] = gp.pot[0];
        g[1] = gp.pot[1];
        g[2] = gp.pot[2];
    } else if (XF == 2 && gp.potential == POT_HALO) {
        // dark-matter halo rho0 / (1 + (r/r0)^2) out to rh (Sec. 4): field
        // G M(r) / r^2 with M(r) = 4 pi rho0 r0^3 (u - atan u), u = min(r, rh) / r0
        const double X = x - gp.pot[3], Y = y - gp.pot[4], Z = z - gp.pot[5];
        const double r = sqrt(X * X + Y * Y + Z * Z);
        if (r > 0.0) {
            const double r0 = gp.pot[1];
            const double u = (r < gp.pot[2] ? r : gp.pot[2]) / r0;
            const double m = 4.0 * M_PI * gp.pot[0] * (r0 * r0 * r0) * (u - atan(u));
            const double a = m / (r * r * r);
            g[0] = a * X;
            g[1] = a * Y;
            g[2] = a * Z;
        } else {
            g[0] = g[1] = g[2] = 0.0;
        }
    } else {
        g[0] = g[1] = g[2] = 0.0;
    }
    for (int a = gp.ndim; a < 3; a++) g[a] = 0.0;
}

// Adds the gradient of the self-gravity potential at interior cell (i, j, k):
// the central difference across the cell (cubic cells, so h[0] serves
// every axis).
template <typename T>
__device__ __forceinline__ void self_gravity_grad(const GridParams &gp, int i, int j, int k, double g[3])
{
    const T *ph = (const T *)gp.phi;
    const long long px = gp.n[0] + 2;
    const long long pp = px * (gp.n[1] + 2);
    const long long b = (long long)(k + 1) * pp + (long long)(j + 1) * px + (i + 1);
    const double h2 = 2.0 * gp.h[0];
    const double ih2 = 0.5 * gp.inv_h[0];
    g[0] = g[0] + PPML_DIV((double)ph[b + 1] - (double)ph[b - 1], h2, ih2);
    g[1] = g[1] + PPML_DIV((double)ph[b + px] - (double)ph[b - px], h2, ih2);
    g[2] = g[2] + PPML_DIV((double)ph[b + pp] - (double)ph[b - pp], h2, ih2);
}

// Time step of the next step (Sec. 2.1 CFL condition, or the fixed step),
// clipped to end at t_stop; 0 when the run has no steps left.
__device__ __forceinline__ double compute_tau(const Ctrl *c, const GridParams &gp)
{
    if (c->steps_left <= 0) return 0.0;
    double tau;
    if (c->dt_fixed > 0.0) {
        tau = c->dt_fixed;
    } else {
        const int s = c->slot_cur;
        double vm = __longlong_as_double((long long)c->vmax_bits[s]);
        double cm = __longlong_as_double((long long)c->cmax_bits[s]);
        tau = gp.cfl_hmin / (vm + cm);
    }
    if (c->t_stop > 0.0) {
        double rem = c->t_stop - c->t;
        if (rem <= 0.0) tau = 0.0;
        else if (tau > rem) tau = rem;
    }
    return tau;
}

// Tile of this work group.  Work groups are dispatched round-robin over the
// 8 XCDs of the chip by their linear id; giving each XCD a contiguous range
// of tiles (x fastest, then y, then z chunk) keeps the halo planes that
// neighbouring tiles share in that XCD's L2.
__device__ __forceinline__ void tile_decode(const GridParams &gp, int L, int &bx, int &by, int &bz)
{
    bx = L % gp.tiles[0];
    const int t = L / gp.tiles[0];
    by = t % gp.tiles[1];
    bz = t / gp.tiles[1];
}

__device__ __forceinline__ void block_tile(const GridParams &gp, int &bx, int &by, int &bz)
{
    const int nb = gp.tiles[0] * gp.tiles[1] * gp.tiles[2];
    const int b = blockIdx.x;
    const int x = b & 7, q = nb >> 3, r = nb & 7;
    const int L = x * q + (x < r ? x : r) + (b >> 3);
    tile_decode(gp, L, bx, by, bz);
}

// Wave-wide maximum (wave64).
template <typename T> __device__ __forceinline__ T wave_max(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        T w = __shfl_xor(v, o, 64);
        v = v > w ? v : w;
    }
    return v;
}

}  // namespace ppml
