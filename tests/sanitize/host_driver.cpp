// Drives the host-side code of the HIP library without a GPU, for a build
// with AddressSanitizer and UndefinedBehaviorSanitizer on the host code:
// descriptor validation (every rejection and every accepted kind), the
// state and scratch sizing, the tile-shape tables, the status strings, the
// NULL-handle checks of every entry point, and the HIP-error paths that
// creating a grid, a batch or an allocation-free run take when no device
// answers.  Exits 0 when every call returns the expected status; a
// sanitizer finding aborts.
#include <cmath>
#include <cstdio>
#include <cstring>

#include "../../include/ppml.h"

static int failures = 0;

static void expect(bool ok, const char *what)
{
    if (!ok) {
        std::printf("unexpected: %s (last error: %s)\n", what, ppml_last_error());
        failures++;
    }
}

static ppml_desc base(int ndim, int prec)
{
    ppml_desc d;
    std::memset(&d, 0, sizeof d);
    d.ndim = ndim;
    d.prec = prec;
    for (int a = 0; a < 3; a++) {
        d.n[a] = a < ndim ? 24 + 4 * a : 1;
        d.lo[a] = -0.5;
        d.hi[a] = 0.5;
        d.bc_lo[a] = d.bc_hi[a] = PPML_PERIODIC;
    }
    d.gamma = 5.0 / 3.0;
    d.cfl = 0.3;
    d.vacuum_ratio = 1e-5;
    return d;
}

int main()
{
    expect(ppml_version() > 0, "version");
    for (int s = 1; s >= -8; s--) expect(ppml_strerror(s) != nullptr, "strerror");
    // tile tables
    for (int nd = 0; nd <= 4; nd++) {
        const int c = ppml_tile_count(nd);
        if (nd < 1 || nd > 3) {
            expect(c == PPML_EINVAL, "tile count of a bad ndim");
            continue;
        }
        for (int v = -1; v <= c; v++) {
            int tx = 0, ty = 0;
            const int rc = ppml_tile_shape(nd, v, &tx, &ty);
            expect((v >= 0 && v < c) ? (rc == PPML_OK && tx * ty >= 64) : rc == PPML_EINVAL, "tile shape");
        }
    }
    // accepted descriptors: every dimensionality, precision, face kind,
    // potential, variant and tile
    for (int nd = 1; nd <= 3; nd++)
        for (int prec = 0; prec <= 1; prec++)
            for (int v = 0; v < ppml_tile_count(nd); v++) {
                ppml_desc d = base(nd, prec == 0 ? PPML_FP32 : PPML_FP64);
                d.tile = v;
                d.bc_lo[0] = PPML_INFLOW;
                d.bc_hi[0] = PPML_OUTFLOW;
                d.inflow[0][0] = 1.0;
                d.inflow[0][1] = 0.5;
                d.inflow[0][4] = 1.0;
                if (nd >= 2) d.bc_lo[1] = d.bc_hi[1] = PPML_REFLECT;
                d.flags = (v & 1) ? PPML_FLAG_FIRST_ORDER : PPML_FLAG_ISOTHERMAL;
                d.iso_cs = 0.5;
                d.potential = v == 0 ? PPML_POT_UNIFORM : PPML_POT_LOG;
                d.pot[2] = 0.9;
                expect(ppml_state_bytes(&d) > 0 && ppml_scratch_bytes(&d) > 0, "accepted descriptor");
            }
    {
        ppml_desc d = base(3, PPML_FP64);
        d.potential = PPML_POT_HALO;
        d.pot[1] = 0.1;
        d.pot[2] = 0.3;
        expect(ppml_state_bytes(&d) > 0, "halo potential");
        d = base(3, PPML_FP32);
        d.self_gravity = 1;
        d.grav_G = 1.0;
        d.lo[0] = d.lo[1] = d.lo[2] = -0.53;
        d.hi[0] = -0.53 + 24.0 / 24.0;
        d.hi[1] = -0.53 + 28.0 / 24.0;
        d.hi[2] = -0.53 + 32.0 / 24.0;
        const size_t plain = ppml_scratch_bytes(&d);
        expect(plain > 0, "self-gravity descriptor");
    }
    // every rejection
    struct Bad {
        const char *what;
        void (*edit)(ppml_desc &);
    };
    const Bad bad[] = {
        {"ndim 0", [](ppml_desc &d) { d.ndim = 0; }},
        {"ndim 4", [](ppml_desc &d) { d.ndim = 4; }},
        {"prec", [](ppml_desc &d) { d.prec = 7; }},
        {"n 0", [](ppml_desc &d) { d.n[1] = 0; }},
        {"n huge", [](ppml_desc &d) { d.n[0] = (1 << 20) + 1; }},
        {"extent", [](ppml_desc &d) { d.hi[2] = d.lo[2]; }},
        {"face code", [](ppml_desc &d) { d.bc_lo[1] = 9; }},
        {"reflect n < 3", [](ppml_desc &d) { d.n[0] = 2; d.bc_lo[0] = d.bc_hi[0] = PPML_REFLECT; }},
        {"half periodic", [](ppml_desc &d) { d.bc_hi[0] = PPML_OUTFLOW; }},
        {"inflow NaN", [](ppml_desc &d) { d.bc_lo[0] = PPML_INFLOW; d.bc_hi[0] = PPML_OUTFLOW; d.inflow[0][0] = NAN; }},
        {"inflow rho", [](ppml_desc &d) { d.bc_lo[0] = PPML_INFLOW; d.bc_hi[0] = PPML_OUTFLOW; d.inflow[0][4] = 1.0; }},
        {"unused axis n", [](ppml_desc &d) { d.ndim = 2; d.n[2] = 5; }},
        {"too many cells", [](ppml_desc &d) { d.n[0] = d.n[1] = 1 << 20; d.n[2] = 4; }},
        {"gamma", [](ppml_desc &d) { d.gamma = 1.0; }},
        {"cfl", [](ppml_desc &d) { d.cfl = 1.0; }},
        {"vacuum", [](ppml_desc &d) { d.vacuum_ratio = -1.0; }},
        {"potential code", [](ppml_desc &d) { d.potential = 17; }},
        {"log q", [](ppml_desc &d) { d.potential = PPML_POT_LOG; d.pot[2] = 0.0; }},
        {"halo radii", [](ppml_desc &d) { d.potential = PPML_POT_HALO; }},
        {"halo ndim", [](ppml_desc &d) { d.ndim = 2; d.n[2] = 1; d.potential = PPML_POT_HALO; d.pot[1] = d.pot[2] = 1; }},
        {"flags", [](ppml_desc &d) { d.flags = 64; }},
        {"iso cs", [](ppml_desc &d) { d.flags = PPML_FLAG_ISOTHERMAL; d.iso_cs = 0.0; }},
        {"tile", [](ppml_desc &d) { d.tile = 99; }},
        {"self_gravity 2", [](ppml_desc &d) { d.self_gravity = 2; }},
        {"self-gravity ndim", [](ppml_desc &d) { d.ndim = 2; d.n[2] = 1; d.self_gravity = 1; d.grav_G = 1; }},
        {"self-gravity cells", [](ppml_desc &d) { d.self_gravity = 1; d.grav_G = 1; }},
        {"self-gravity G", [](ppml_desc &d) { d.n[0] = d.n[1] = d.n[2] = 24; d.self_gravity = 1; }},
        {"origin on shell", [](ppml_desc &d) {
             d.n[0] = d.n[1] = d.n[2] = 24;
             d.self_gravity = 1;
             d.grav_G = 1;
             const double h = 1.0 / 24.0;
             for (int a = 0; a < 3; a++) { d.lo[a] = 0.5 * h; d.hi[a] = d.lo[a] + 1.0; }
         }},
    };
    for (const Bad &b : bad) {
        ppml_desc d = base(3, PPML_FP32);
        b.edit(d);
        if (ppml_state_bytes(&d) != 0 || ppml_scratch_bytes(&d) != 0) {
            std::printf("accepted: %s\n", b.what);
            failures++;
        }
        ppml_grid *g = nullptr;
        expect(ppml_create(&d, (void *)256, (void *)512, nullptr, &g) == PPML_EINVAL && !g, b.what);
    }
    expect(ppml_state_bytes(nullptr) == 0, "NULL descriptor");
    // argument checks of ppml_create, then its HIP path with no device
    {
        ppml_desc d = base(2, PPML_FP32);
        ppml_grid *g = nullptr;
        expect(ppml_create(nullptr, (void *)256, (void *)512, nullptr, &g) == PPML_EINVAL, "create NULL desc");
        expect(ppml_create(&d, (void *)256, (void *)512, nullptr, nullptr) == PPML_EINVAL, "create NULL out");
        expect(ppml_create(&d, nullptr, (void *)512, nullptr, &g) == PPML_EINVAL, "create NULL state");
        expect(ppml_create(&d, (void *)260, (void *)512, nullptr, &g) == PPML_EINVAL, "create misaligned");
        expect(ppml_create(&d, (void *)256, (void *)512, nullptr, &g) == PPML_EHIP && !g, "create without a device");
    }
    // every entry point rejects a NULL handle
    {
        double x[8];
        int64_t s = 0;
        int32_t c = 0;
        size_t b = 0;
        expect(ppml_set_primitive(nullptr, x, x, x, x, x) == PPML_EINVAL, "set_primitive");
        expect(ppml_set_conserved(nullptr, nullptr, 1.0, 0.0) == PPML_EINVAL, "set_conserved");
        expect(ppml_step(nullptr, 1, 0.0, 0.0) == PPML_EINVAL, "step");
        expect(ppml_get_time(nullptr, x, x, &s) == PPML_EINVAL, "get_time");
        expect(ppml_max_speeds(nullptr, x, x) == PPML_EINVAL, "max_speeds");
        expect(ppml_get_conserved(nullptr, 0, x) == PPML_EINVAL, "get_conserved");
        expect(ppml_get_potential(nullptr, x) == PPML_EINVAL, "get_potential");
        expect(ppml_totals(nullptr, x) == PPML_EINVAL, "totals");
        expect(ppml_sync(nullptr) == PPML_EINVAL, "sync");
        expect(ppml_set_timing(nullptr, 4) == PPML_EINVAL, "set_timing");
        expect(ppml_get_timing(nullptr, x, x, &s) == PPML_EINVAL, "get_timing");
        expect(ppml_get_timing_split(nullptr, x, &s) == PPML_EINVAL, "get_timing_split");
        expect(ppml_destroy(nullptr) == PPML_EINVAL, "destroy");
        expect(ppml_batch_admit(nullptr, nullptr, &c) == PPML_EINVAL, "batch_admit");
        expect(ppml_batch_retire(nullptr, 0) == PPML_EINVAL, "batch_retire");
        expect(ppml_batch_step(nullptr, 1, nullptr, 0.0, 0.0, 1) == PPML_EINVAL, "batch_step");
        expect(ppml_batch_sync(nullptr) == PPML_EINVAL, "batch_sync");
        expect(ppml_batch_info(nullptr, &c, &b) == PPML_EINVAL, "batch_info");
        expect(ppml_batch_set_tile(nullptr, 2, 0) == PPML_EINVAL, "batch_set_tile");
        expect(ppml_batch_destroy(nullptr) == PPML_EINVAL, "batch_destroy");
    }
    // batches and the allocation-free entry point: arguments, then no device
    {
        ppml_batch *b = nullptr;
        expect(ppml_batch_create(0, 1 << 20, nullptr, &b) == PPML_EINVAL, "batch capacity 0");
        expect(ppml_batch_create(4, 1 << 20, nullptr, nullptr) == PPML_EINVAL, "batch NULL out");
        expect(ppml_batch_create(4, 1 << 20, nullptr, &b) == PPML_EHIP && !b, "batch without a device");
        ppml_desc d = base(3, PPML_FP32);
        double t = 0.0;
        int64_t s = 0;
        expect(ppml_step_noalloc(nullptr, (void *)256, 1.0, 0.0, 1, 0.0, 0.0, nullptr, &t, &s) == PPML_EINVAL,
               "noalloc NULL desc");
        expect(ppml_step_noalloc(&d, nullptr, 1.0, 0.0, 1, 0.0, 0.0, nullptr, &t, &s) == PPML_EINVAL,
               "noalloc NULL state");
        expect(ppml_step_noalloc(&d, (void *)256, 1.0, 0.0, -1, 0.0, 0.0, nullptr, &t, &s) == PPML_EINVAL,
               "noalloc negative steps");
        d.self_gravity = 1;
        expect(ppml_step_noalloc(&d, (void *)256, 1.0, 0.0, 1, 0.0, 0.0, nullptr, &t, &s) == PPML_EINVAL,
               "noalloc self-gravity");
        d = base(3, PPML_FP32);
        d.n[0] = d.n[1] = d.n[2] = 1024;
        expect(ppml_step_noalloc(&d, (void *)256, 1.0, 0.0, 1, 0.0, 0.0, nullptr, &t, &s) == PPML_EINVAL,
               "noalloc oversized");
        d = base(3, PPML_FP32);
        expect(ppml_step_noalloc(&d, (void *)256, 1.0, 0.0, 1, 0.0, 0.0, nullptr, &t, &s) == PPML_EHIP,
               "noalloc without a device");
    }
    std::printf("host sanitizer driver: %d failure(s)\n", failures);
    return failures ? 1 : 0;
}
