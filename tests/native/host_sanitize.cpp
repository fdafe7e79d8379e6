// host_sanitize.cpp -- drives the host-side validation and layout code of the
// C ABI (include/mdf.h) with AddressSanitizer and UndefinedBehaviorSanitizer:
// workspace sizes over every lattice, storage and a range of grids (up to the
// 4 GiB plane limit and past it), the refused forms of mdf_init, and every
// entry point with a NULL context.  None of these calls reaches the device,
// so the run needs no GPU.  Built by tests/test_sanitizers_cpu.py with the
// host library source compiled under the sanitizers and the kernels' objects
// linked as they are.  Test infrastructure only.
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "mdf.h"

static int fails = 0;

#define CHECK(cond)                                                                \
    do {                                                                           \
        if (!(cond)) {                                                             \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
            ++fails;                                                               \
        }                                                                          \
    } while (0)

static mdf_case make_case(int d, int nx, int ny, int nz)
{
    mdf_case c;
    std::memset(&c, 0, sizeof c);
    c.nx = nx;
    c.ny = ny;
    c.nz = d == 2 ? 1 : nz;
    c.s0 = 1.0;
    c.s1 = 1.2;
    c.rho0 = 1.0;
    c.bc[2] = c.bc[3] = MDF_WALL;
    c.wall_u[3][0] = 0.1;
    return c;
}

static int dim_of(int lattice)
{
    return (lattice % 2 == 0) ? 2 : 3;
}

int main()
{
    // workspace sizes: every lattice id and storage, valid and refused
    for (int lat = -2; lat <= 15; ++lat) {
        const bool lat_ok = lat >= 0 && lat <= 13;
        for (int st = -1; st <= 4; ++st) {
            const bool st_ok = st >= 0 && st <= 3;
            const int d = dim_of(lat < 0 ? 0 : lat);
            mdf_case cases[3] = {make_case(d, 37, 21, 9), make_case(d, 64, 64, 16), make_case(d, 5, 3, 2)};
            for (int solid = 0; solid <= 1; ++solid) {
                const size_t one = mdf_workspace_size(mdf_lattice(lat), mdf_storage(st), cases, 1, solid);
                const size_t three = mdf_workspace_size(mdf_lattice(lat), mdf_storage(st), cases, 3, solid);
                if (lat_ok && st_ok) {
                    CHECK(three > one);
                } else {
                    CHECK(one == 0 && three == 0);
                }
                CHECK(mdf_last_error(nullptr) != nullptr);
            }
            CHECK(mdf_workspace_size(mdf_lattice(lat), mdf_storage(st), cases, 0, 0) == 0);
            CHECK(mdf_workspace_size(mdf_lattice(lat), mdf_storage(st), cases, -3, 0) == 0);
            CHECK(mdf_workspace_size(mdf_lattice(lat), mdf_storage(st), nullptr, 1, 0) == 0);
        }
    }
    // grid sizes: degenerate, ragged, at and past the per-plane limit
    const int dims[][3] = {{0, 4, 1}, {4, 0, 1}, {1, 1, 1}, {33, 17, 1}, {65536, 16383, 1}, {65536, 16385, 1},
                           {70000, 70000, 1}, {2147483647, 2, 1}, {-5, 4, 1}};
    for (const auto &g : dims) {
        mdf_case c = make_case(2, g[0], g[1], g[2]);
        c.bc[2] = c.bc[3] = MDF_PERIODIC;
        for (int st = 0; st <= 3; ++st) {
            const size_t ws = mdf_workspace_size(MDF_D2Q5, mdf_storage(st), &c, 1, 1);
            if (g[0] <= 0 || g[1] <= 0) CHECK(ws == 0);
            CHECK(mdf_last_error(nullptr) != nullptr);
        }
    }
    // refused case parameters
    for (int k = 0; k < 9; ++k) {   // 8: exercised, not necessarily refused
        mdf_case c = make_case(2, 16, 16, 1);
        switch (k) {
        case 0: c.s1 = 0.0; break;
        case 1: c.s1 = 2.0; break;
        case 2: c.rho0 = 0.0; break;
        case 3: c.bc[0] = MDF_WALL; c.bc[1] = MDF_PERIODIC; break;   // unpaired periodic face
        case 4: c.bc[4] = 7; break;
        case 5: c.forcing = 5; break;
        case 6: c.nz = 3; break;                                    // 2D with nz != 1
        case 7: c.s1 = 0.0 / 0.0; break;                            // NaN rate
        case 8: c.wall_u[3][0] = 1.0 / 0.0; break;                  // infinite wall speed
        }
        const size_t ws = mdf_workspace_size(MDF_D2Q5, MDF_F32, &c, 1, 0);
        if (k < 8) CHECK(ws == 0);
        CHECK(std::strlen(mdf_last_error(nullptr)) > 0);
    }
    // mdf_init refuses before touching the device
    mdf_case c = make_case(2, 16, 16, 1);
    mdf_ctx *ctx = nullptr;
    void *fake = reinterpret_cast<void *>(uintptr_t(256));
    CHECK(mdf_init(nullptr, MDF_D2Q5, MDF_F32, &c, 1, fake, size_t(1) << 30, nullptr, 0, nullptr, nullptr) ==
          MDF_EINVAL);
    CHECK(mdf_init(&ctx, MDF_D2Q5, MDF_F32, &c, 1, nullptr, 0, nullptr, 0, nullptr, nullptr) == MDF_EINVAL);
    CHECK(mdf_init(&ctx, MDF_D2Q5, MDF_F32, &c, 1, reinterpret_cast<void *>(uintptr_t(16)), size_t(1) << 30,
                   nullptr, 0, nullptr, nullptr) == MDF_EINVAL);
    CHECK(mdf_init(&ctx, MDF_D2Q5, MDF_F32, &c, 1, fake, 1024, nullptr, 0, nullptr, nullptr) == MDF_ENOMEM);
    CHECK(mdf_init(&ctx, mdf_lattice(14), MDF_F32, &c, 1, fake, size_t(1) << 30, nullptr, 0, nullptr, nullptr) ==
          MDF_EINVAL);
    CHECK(mdf_init(&ctx, MDF_D2Q5, mdf_storage(9), &c, 1, fake, size_t(1) << 30, nullptr, 0, nullptr, nullptr) ==
          MDF_EINVAL);
    CHECK(mdf_init(&ctx, MDF_D2Q5, MDF_F32, &c, 1, fake, size_t(1) << 30, nullptr, 1, nullptr, nullptr) ==
          MDF_EINVAL);
    CHECK(mdf_init(&ctx, MDF_D2Q5, MDF_F32, &c, 1, fake, size_t(1) << 30, nullptr, 9, nullptr, nullptr) ==
          MDF_EINVAL);
    CHECK(mdf_init(&ctx, MDF_D2Q5, MDF_F32, &c, 0, fake, size_t(1) << 30, nullptr, 0, nullptr, nullptr) ==
          MDF_EINVAL);
    CHECK(ctx == nullptr);
    // every entry point with a NULL context
    double d8[8];
    int32_t i8[8];
    int64_t l8[8];
    const char *msg = nullptr;
    void *ptr = nullptr;
    size_t nbytes = 0;
    CHECK(mdf_step(nullptr, 1, nullptr) == MDF_EINVAL);
    CHECK(mdf_step_emit(nullptr, 1, MDF_FIELD_ALL, nullptr, nullptr) == MDF_EINVAL);
    CHECK(mdf_moments(nullptr, 0, nullptr, nullptr) == MDF_EINVAL);
    CHECK(mdf_gradients(nullptr, 0, MDF_FIELD_ALL, nullptr, nullptr) == MDF_EINVAL);
    CHECK(mdf_populations(nullptr, 0, nullptr, nullptr) == MDF_EINVAL);
    CHECK(mdf_check(nullptr, d8, i8, nullptr) == MDF_EINVAL);
    CHECK(mdf_run_steady(nullptr, 1e-8, 100, 1000, 0, nullptr, i8, l8, d8, nullptr) == MDF_EINVAL);
    CHECK(mdf_invariants(nullptr, 0, d8, nullptr) == MDF_EINVAL);
    CHECK(mdf_set_launch(nullptr, 64, 4, 8, 0) == MDF_EINVAL);
    CHECK(mdf_state_size(nullptr) == 0);
    CHECK(mdf_save(nullptr, nullptr, 0, nullptr) == MDF_EINVAL);
    CHECK(mdf_load(nullptr, nullptr, 0, nullptr) == MDF_EINVAL);
    CHECK(mdf_set_force_field(nullptr, 0, nullptr) == MDF_EINVAL);
    CHECK(mdf_set_active(nullptr, i8) == MDF_EINVAL);
    CHECK(mdf_autotune(nullptr, 3, i8, d8, nullptr) == MDF_EINVAL);
    CHECK(mdf_graph_stats(nullptr, l8, &msg) == MDF_EINVAL);
    CHECK(mdf_population_buffer(nullptr, 0, 0, &ptr, &nbytes) == MDF_EINVAL);
    CHECK(mdf_time(nullptr, 0) == -1);
    CHECK(mdf_last_error(nullptr) != nullptr);
    CHECK(mdf_destroy(nullptr) == MDF_OK);
    std::printf("host sanitizer run: %d failed checks\n", fails);
    return fails != 0;
}
