// Host-side checks of the lbm3d runtime, built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code.  The kernels are not compiled
// into this test program: the launch wrappers below stand in for them and report that
// there is no device, so every path that would launch a kernel takes its
// error branch.  Exercises parameter validation and layout, the stability
// analysis and admission, the batched step's work plans, the autotuner's
// cache files, and the error paths of create / server without a device.
#include "../../include/lbm3d.h"
#include "../../paper_1010_4135_amd/csrc/lbm3d_api_impl.h"
#include "../../paper_1010_4135_amd/csrc/lbm3d_internal.h"

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

namespace lbm3d {
hipError_t launch_init(int, const Grid&, const Model<double>&, const double*, void*, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_step(int, const Grid&, const FaceBC&, const TileCfg&, const Model<double>&, const Model<float>&,
                       const double (*)[5], const void*, void*, uint32_t*, hipStream_t, bool, hipEvent_t,
                       hipEvent_t) { return hipErrorNoDevice; }
hipError_t launch_ghosts(int, const Grid&, const FaceBC&, const Model<double>&, const double (*)[5], bool, void*,
                         hipStream_t, uint32_t) { return hipErrorNoDevice; }
hipError_t launch_moments(int, const Grid&, const Model<double>&, const void*, double*, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_conserved(int, const Grid&, const Model<double>&, const void*, double*, int, double*, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_pack(int, const Grid&, const void*, void*, bool, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_batch_layers(int, const BatchSolve*, const BatchLayerJob*, const int32_t*, int, int, const BatchCount*,
                               hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_batch_count(BatchCount*, int, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_gather_health(const BatchSolve*, int, uint32_t*, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_batch_step(int, int, bool, const BatchSolve*, const BatchTile*, BatchQueue*, int, int, int,
                             const BatchCount*, hipStream_t) { return hipErrorNoDevice; }
}  // namespace lbm3d

extern "C" int32_t lbm3d_stream_copy_rate(int64_t, int32_t, double*) { return LBM3D_E_DEVICE; }

static int failures = 0;
#define EXPECT(c)                                                            \
    do {                                                                     \
        if (!(c)) {                                                          \
            std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            failures++;                                                      \
        }                                                                    \
    } while (0)

static lbm3d_params base(int nx, int ny, int nz, int prec)
{
    lbm3d_params p;
    std::memset(&p, 0, sizeof p);
    p.nx = nx;
    p.ny = ny;
    p.nz = nz;
    p.c1 = 8;
    p.c2 = 24;
    p.eta0 = 8;
    p.gamma = 1.4;
    p.tau = 1e-5;
    p.dt = 1e-5;
    p.dx = 1.0 / 256;
    p.precision = prec;
    return p;
}

// The memory layout of a level (make_grid), for small random grids in both
// plane orders and every precision: each node the kernels address (interior
// and the two layers per face; with dense rows the x layers sit in the
// x-layer block instead), every velocity's sink region and x-layer block lie
// inside the level; no two of them share an element, except that the sink
// regions of different velocities may overlap one another (their contents
// are never read).
static void check_layouts(std::mt19937& rng)
{
    for (int k = 0; k < 240; k++) {
        const int prec = (int)(rng() % 3);
        lbm3d_params p = base(1 + (int)(rng() % 100), 1 + (int)(rng() % 20), 1 + (int)(rng() % 12), prec);
        if (k % 3 == 0) p.nx = 64 * (1 + (int)(rng() % 2));  // dense rows
        const bool vm = rng() % 2;
        if (vm) p.flags = LBM3D_VELOCITY_MAJOR;
        const lbm3d::Grid g = lbm3d::make_grid(&p);
        const int64_t es = prec == LBM3D_FP64 ? 8 : 4;
        const bool dense = lbm3d::dense_rows(p.nx);
        EXPECT(g.plane_major == (vm ? 0 : 1));
        EXPECT((int64_t)lbm3d::f_bytes(g, prec) == g.len * es);
        EXPECT(lbm3d::tiled_fits(prec, g));
        EXPECT(g.sv % (256 / es) == 0 && (g.sv / (256 / es)) % 2 == 1);
        std::vector<int32_t> own((size_t)g.len, 0);
        int32_t id = 0;
        bool ok = true;
        auto claim = [&](int64_t a) {
            ++id;
            if (a < 0 || a >= g.len || own[(size_t)a] != 0) {
                ok = false;
                return;
            }
            own[(size_t)a] = id;
        };
        const int x0 = dense ? 0 : -2, x1 = dense ? p.nx : p.nx + 2;
        for (int i = 0; i < 15; i++)
            for (int z = -2; z < p.nz + 2; z++)
                for (int y = -2; y < p.ny + 2; y++)
                    for (int x = x0; x < x1; x++) claim(i * g.sv + g.org + z * g.sz + y * g.sy + x);
        if (dense) {
            EXPECT(g.xg != 0);
            for (int i = 0; i < 15; i++)
                for (int z = 0; z < p.nz; z++)
                    for (int y = 0; y < p.ny; y++)
                        for (int c = 0; c < 4; c++) claim(i * g.sv + g.xg + (z + 2) * g.xgz + (y + 2) * 4 + c);
        } else {
            EXPECT(g.xg == 0);
        }
        EXPECT(ok);
        // the tiled kernels' clamped loads (x up to nx + 1 with dense rows)
        // stay inside the level
        if (dense) EXPECT(14 * g.sv + g.org + (p.nz + 1) * g.sz + (p.ny + 1) * g.sy + p.nx + 1 < g.len);
        for (int i = 0; i < 15; i++)
            for (int64_t e = 0; e < (int64_t)lbm3d::SINK_ROWS * lbm3d::TILE_X; e++) {
                const int64_t a = i * g.sv + g.sink + e;
                if (a < 0 || a >= g.len || own[(size_t)a] > 0) ok = false;
            }
        EXPECT(ok);
        // every sink element lies past every plane the step writes
        EXPECT(g.sink - g.org - (int64_t)(p.nz - 1) * g.sz >= 0);
    }
}

int main(int argc, char** argv)
{
    const std::string tmp = argc > 1 ? argv[1] : "/tmp";
    std::mt19937 rng(12345);
    // validation and footprint over random parameters, valid or not
    for (int k = 0; k < 4000; k++) {
        lbm3d_params p = base(1 + (int)(rng() % 300), 1 + (int)(rng() % 300), 1 + (int)(rng() % 300), (int)(rng() % 4) - 0);
        for (int f = 0; f < 6; f++) p.bc[f] = (int)(rng() % 5);
        if (rng() % 2) { p.bc[1] = p.bc[0]; p.bc[3] = p.bc[2]; p.bc[5] = p.bc[4]; }
        for (int f = 0; f < 6; f++)
            for (int c = 0; c < 5; c++) p.inflow[f][c] = (rng() % 3) * 0.7;
        if (rng() % 5 == 0) p.dt = 1e-2;
        if (rng() % 7 == 0) p.flags = (uint32_t)(rng() % 16);
        size_t bytes = 0;
        const int32_t rc = lbm3d_footprint(&p, &bytes);
        EXPECT(rc == LBM3D_OK || rc == LBM3D_E_INVAL || rc == LBM3D_E_UNSTABLE);
        if (rc == LBM3D_OK) EXPECT(bytes >= (size_t)2 * 15 * p.nx * p.ny * p.nz * (p.precision == 0 ? 8 : 4));
    }
    check_layouts(rng);
    // stability analysis and admission
    for (int k = 0; k < 20; k++) {
        lbm3d_params p = base(6, 5, 4, 0);
        const double q[5] = {1.0 + 0.1 * k, 0.3 * k, -0.1, 0.2, 0.5 + 0.2 * k};
        double om = 0, kk = 0;
        EXPECT(lbm3d_stability(&p, q, k % 4, 0.0, 3.14159, 9, 0.0, &om, &kk) == LBM3D_OK);
        EXPECT(std::isfinite(om) && om > 0.9);
        const int n = 6 * 5 * 4;
        std::vector<double> f[5];
        for (int c = 0; c < 5; c++) f[c].assign(n, c == 0 || c == 4 ? 1.0 + 0.01 * (k + c) : 0.1 * c);
        const int32_t rc = lbm3d_admit(&p, f[0].data(), f[1].data(), f[2].data(), f[3].data(), f[4].data(), &om);
        EXPECT(rc == LBM3D_OK || rc == LBM3D_E_UNSTABLE);
    }
    // work plans of random batches
    for (int k = 0; k < 60; k++) {
        const int count = 1 + (int)(rng() % 20);
        const int prec = (int)(rng() % 3);
        std::vector<lbm3d_params> ps;
        int64_t nodes = 0;
        for (int j = 0; j < count; j++) {
            ps.push_back(base(1 + (int)(rng() % 200), 1 + (int)(rng() % 100), 1 + (int)(rng() % 100), prec));
            nodes += (int64_t)ps.back().nx * ps.back().ny * ps.back().nz;
        }
        int32_t nt = 0, nl = 0, nb = 0;
        const int32_t tz = (int32_t)(rng() % 140);
        EXPECT(lbm3d_batch_plan(ps.data(), count, tz, 1 + (int)(rng() % 300), &nt, &nl, &nb, nullptr, 0, nullptr) == LBM3D_OK);
        std::vector<int32_t> tiles((size_t)nt * 7);
        int32_t first[9];
        EXPECT(lbm3d_batch_plan(ps.data(), count, tz, 256, nullptr, nullptr, nullptr, tiles.data(), nt, first) == LBM3D_OK);
        int64_t covered = 0;
        for (int32_t t = 0; t < nt; t++) {
            const int32_t* o = &tiles[(size_t)t * 7];
            covered += (int64_t)(o[2] - o[1]) * (o[4] - o[3]) * (o[6] - o[5]);
        }
        EXPECT(covered == nodes);
        if (nt > 1) EXPECT(lbm3d_batch_plan(ps.data(), count, tz, 256, nullptr, nullptr, nullptr, tiles.data(), nt - 1, first) == LBM3D_E_NOMEM);
    }
    // the autotuner's cache files
    const std::string good = tmp + "/tune_good.txt", bad = tmp + "/tune_bad.txt", out = tmp + "/tune_out.txt";
    {
        FILE* fp = std::fopen(good.c_str(), "w");
        std::fprintf(fp, "lbm3d-tune 2 none\ntile 2 256 128 128 2 1 3 3 3 3 8 32 1\nbatch 1 64\n");
        std::fclose(fp);
        fp = std::fopen(bad.c_str(), "w");
        std::fprintf(fp, "lbm3d-tune 2 none\ntile 2 256 128 128 2 1 3 3 3 3 8 32 1 9 9 9 9 9 9 9 9\nbatch 7 1\n");
        std::fclose(fp);
    }
    EXPECT(lbm3d_tune_load(good.c_str()) == LBM3D_OK);
    EXPECT(lbm3d_tune_load(bad.c_str()) == LBM3D_E_INVAL);
    EXPECT(lbm3d_tune_save(out.c_str()) == LBM3D_OK);
    EXPECT(lbm3d_tune_load(out.c_str()) == LBM3D_OK);
    EXPECT(lbm3d_tune_load((tmp + "/missing.txt").c_str()) == LBM3D_E_NOTFOUND);
    // without a device: create and server fail cleanly
    lbm3d_params p = base(32, 16, 8, 1);
    lbm3d_t h = nullptr;
    const int32_t rc = lbm3d_create(&p, &h);
    EXPECT(rc != LBM3D_OK && h == nullptr);
    lbm3d_server_t s = nullptr;
    EXPECT(lbm3d_server_create(1 << 30, 4, &s) != LBM3D_OK && s == nullptr);
    EXPECT(lbm3d_destroy(nullptr) == LBM3D_OK && lbm3d_server_destroy(nullptr) == LBM3D_OK);
    for (int c = 1; c >= -10; c--) EXPECT(lbm3d_strerror(c) != nullptr);
    int32_t count = -1;
    EXPECT(lbm3d_device_count(&count) == LBM3D_OK && count >= 0);
    if (failures) {
        std::fprintf(stderr, "%d host checks failed\n", failures);
        return 1;
    }
    std::printf("host checks passed\n");
    return 0;
}
