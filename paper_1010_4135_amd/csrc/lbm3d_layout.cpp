// Host-side layout decisions of the lbm3d library: which kernels and tile
// shapes take a solve, which boundary layers the kernels leave to memory.
#include "lbm3d_model.h"

#include <algorithm>

namespace lbm3d {

bool tiled_fits(int mode, const Grid& g)
{
    // the tiled kernels address a velocity plane with 32-bit byte offsets
    const int64_t es = mode == MODE_FP64 ? 8 : 4;
    return g.sv * es < ((int64_t)1 << 31);
}

TileCfg default_tile(int mode, const Grid& g)
{
    // measured on MI355X at 256x128x128: 64x8x32 tiles (FP32 modes) and
    // 64x4x64 (FP64); a short z extent leaves too few workgroups on small grids
    TileCfg t;
    if (!tiled_fits(mode, g)) {
        t.by = 0;
        t.tz = 1;
        return t;
    }
    t.by = mode == MODE_FP64 ? 4 : 8;
    t.tz = mode == MODE_FP64 ? 64 : 32;
    const int64_t es = mode == MODE_FP64 ? 8 : 4;
    t.stream = 2 * NV * g.sv * es > STREAM_MIN_BYTES;
    if (g.nz < 2 * t.tz) t.tz = std::max(2, g.nz / 4);
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
        const int kind = bc.kind[face], axis = face >> 1;
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
