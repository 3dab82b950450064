// Host-side layout decisions of the lbm3d library: where each node's
// distributions sit in memory, which kernels and tile shapes take a solve,
// which boundary layers the kernels leave to memory.
#include "lbm3d_api_impl.h"
#include "lbm3d_model.h"

#include <algorithm>
#include <mutex>
#include <vector>

namespace lbm3d {

size_t elem_size(int precision) { return precision == LBM3D_FP64 ? 8 : 4; }

// Padded layout: each x row holds `ox` leading elements (the two boundary
// layers sit just before interior x = 0, which starts on a 128-byte line),
// the nx interior nodes and two boundary layers, rounded up to whole lines.
Grid make_grid(const lbm3d_params* p)
{
    Grid g;
    const int64_t es = (int64_t)elem_size(p->precision);
    const int64_t line = 128 / es;
    g.nx = p->nx;
    g.ny = p->ny;
    g.nz = p->nz;
    const bool dense = dense_rows(p->nx);
    // dense rows: the interior only, rows start on a line (nx is a multiple
    // of 64 elements); otherwise the x layers pad the rows
    const int64_t ox = dense ? 0 : line;
    // one cache line of padding per row, holding the two right layer nodes
    // of the row (its first elements) and the two left layer nodes of the
    // next row (its last elements); interior rows start on a line
    const int64_t mxp = (p->nx + line - 1) / line * line + line;
    const int64_t mx = dense ? p->nx : mxp;
    const int64_t my = p->ny + 2 * NG;
    const int64_t mz = p->nz + 2 * NG;
    const int64_t plane = mx * my;
    const int64_t xrows = dense ? 4 * my : 0;  // x layers of one plane's rows (dense rows)
    const int64_t sinkn = (int64_t)SINK_ROWS * TILE_X;
    g.my = (int32_t)my;
    g.sy = mx;
    // an odd number of 256-byte blocks holding at least n elements
    const int64_t blk = 256 / es;
    auto odd_blocks = [&](int64_t n) {
        int64_t b = (n + blk - 1) / blk;
        if ((b & 1) == 0) b += 1;
        return b * blk;
    };
    // The sink region of the tiled step's stores from lanes outside the grid
    // sits after one spare line past the last plane (the right layer nodes
    // of the last row of a padded plane reach two elements past it), at the
    // same offset from every velocity's base.
    const bool velocity_major = (p->flags & LBM3D_VELOCITY_MAJOR) != 0;
    if (!velocity_major) {
        const int64_t sv = odd_blocks(plane + xrows);
        const int64_t sz = NV * sv;
        const int64_t sink = sz * mz + line;
        const int64_t len = (NV - 1) * sv + sink + sinkn + line;
        if (len * es < ((int64_t)1 << 31)) {
            g.plane_major = 1;
            g.sv = sv;
            g.sz = sz;
            g.sink = sink;
            g.xg = dense ? plane : 0;
            g.xgz = sz;
            g.len = len;
            g.org = NG * g.sz + NG * g.sy + ox;
            return g;
        }
    }
    g.plane_major = 0;
    g.sz = plane;
    g.sink = g.sz * mz + line;
    const int64_t sink_end = g.sink + sinkn;
    // dense rows: the x layers of every row (4 nodes) after the sink region
    g.xg = dense ? sink_end + line : 0;
    g.xgz = xrows;
    const int64_t end = dense ? g.xg + xrows * mz : sink_end + line;
    g.sv = odd_blocks(end);
    g.len = NV * g.sv;
    g.org = NG * g.sz + NG * g.sy + ox;
    return g;
}

size_t f_bytes(const Grid& g, int precision) { return (size_t)g.len * elem_size(precision); }


bool tiled_fits(int mode, const Grid& g)
{
    // the tiled kernels reach everything from a velocity's base (its sink
    // region included) with 32-bit byte offsets: the whole level when it is
    // plane-major, one velocity block when it is velocity-major
    const int64_t es = mode == MODE_FP64 ? 8 : 4;
    return (g.plane_major ? g.len : g.sv) * es < ((int64_t)1 << 31);
}

int device_cus()
{
    static std::mutex mu;
    static std::vector<int> cache;  // per device, 0 until looked up
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) {
        (void)hipGetLastError();
        return 256;
    }
    std::lock_guard<std::mutex> lk(mu);
    if ((size_t)dev >= cache.size()) cache.resize((size_t)dev + 1, 0);
    if (!cache[(size_t)dev]) {
        int cus = 256;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
            cus = prop.multiProcessorCount;
        cache[(size_t)dev] = cus;
    }
    return cache[(size_t)dev];
}

TileCfg default_tile(int mode, const Grid& g)
{
    // Tiles of 64 x BY columns (BY = 8 in the FP32 modes, 4 in FP64, the
    // rows that fit two wavefronts per SIMD) and a z-chunk depth from a
    // simple launch model: the tiles run in rounds of one per compute unit,
    // and a tile takes time in proportion to its planes plus the four
    // planes its z ring loads first; the depth with the lowest cost wins
    // (the longer one on a tie).  When even the shortest useful chunks (8
    // planes) leave more than a quarter of the compute units without a
    // tile, the untiled kernel, whose small blocks spread over all of
    // them, is faster.  These choices match the autotuner's on the grids it
    // was compared on (256x128x128, 192x128x128, 128^3 and the paper's
    // 298x78x78 tile; grids up to 96x64x64 in the FP32 modes and up to 64^3
    // in FP64 untiled), which remains the way to the best shape.
    TileCfg t;
    t.by = 0;
    t.tz = 1;
    if (!tiled_fits(mode, g)) return t;
    const int64_t es = mode == MODE_FP64 ? 8 : 4;
    t.stream = 2 * g.len * es > STREAM_MIN_BYTES;
    const int by = mode == MODE_FP64 ? 4 : 8;
    const int64_t cus = device_cus();
    const int64_t cols = (int64_t)((g.nx + TILE_X - 1) / TILE_X) * ((g.ny + by - 1) / by);
    int best_tz = 0;
    int64_t best_cost = 0, best_tiles = 0;
    for (int64_t tz = 8;; tz *= 2) {
        const int64_t d = std::min<int64_t>(tz, g.nz);
        const int64_t tiles = cols * ((g.nz + d - 1) / d);
        const int64_t cost = ((tiles + cus - 1) / cus) * (d + 4);
        if (best_tz == 0 || cost <= best_cost) {
            best_tz = (int)d;
            best_cost = cost;
            best_tiles = tiles;
        }
        if (d >= g.nz) break;
    }
    if (4 * best_tiles < 3 * cus) return t;  // untiled
    t.by = by;
    t.tz = best_tz;
    return t;
}

bool tile_supported(int mode, const Grid& g, const TileCfg& t)
{
    if (t.tz < 1) return false;
    if (t.by == 0) return true;
    if (!tiled_fits(mode, g)) return false;
    if (t.by == 2 || t.by == 4) return true;
    return t.by == 8 && mode != MODE_FP64;
}

uint32_t ghost_faces(const Grid& g, const FaceBC& bc, bool tiled)
{
    uint32_t m = 0;
    for (int face = 0; face < 6; face++) {
        const int kind = bc.kind[face];
        if (kind == BC_INFLOW) continue;
        // the tiles form the -x layers, and the +x layers unless the last
        // tile holds a single column (see x_forms)
        if (tiled && face == 0) continue;
        if (tiled && face == 1 && g.nx % TILE_X != 1) continue;
        if (tiled && kind == BC_PERIODIC) continue;
        m |= 1u << face;
    }
    return m;
}

void x_fixed_states(const double (*inflow)[5], double (&xin)[2][5])
{
    for (int s = 0; s < 2; s++) {
        const double* st = inflow[s];
        xin[s][0] = st[0];
        xin[s][1] = st[1];
        xin[s][2] = st[2];
        xin[s][3] = st[3];
        xin[s][4] = st[0] > 0.0 ? st[4] / st[0] : 0.0;  // T = p / rho
    }
}

int conserved_blocks(const Grid& g)
{
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    return (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n + RB - 1) / RB));
}

}  // namespace lbm3d
