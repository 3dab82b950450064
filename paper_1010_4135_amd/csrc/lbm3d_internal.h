// Internal declarations shared by the host runtime and the device code of
// the lbm3d library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace lbm3d {

constexpr int NV = 15;  // discrete velocities, Sec. 2, Eq. (vv)
constexpr int NG = 2;   // boundary-node layers per face (NND stencil half-width)

// Model constants of one solve, in one floating type.  The equilibrium of
// Eqs. (eq)/(e18) is written per velocity group as
//   A = a0 + aT T + au u^2,   B = b0 + bT T + bu u^2,   D = d
// (rest: A = aT T, B = D = 0), and f_i^eq = rho (A + B s + D s^2), s = v_i.u.
template <typename T>
struct Model {
    T c1, k;             // axis speed c1 and diagonal component c2/sqrt(3)
    T c1sq, c2sq, e0sq;  // c1^2, c2^2, eta0^2
    T inv_b;             // 1/b
    T r_aT;              // rest:  A = r_aT T
    T x_a0, x_aT, x_au, x_b0, x_bT, x_bu, x_d;   // axis group
    T d_a0, d_aT, d_au, d_b0, d_bT, d_bu, d_d;   // diagonal group
    T k_adv;             // dt/dx
    T k_bgk;             // dt/tau
    T k_lap0, k_lap1;    // lambda_1 dt/dx^2 (rest), lambda_{2..7} dt/dx^2 (axis)
    T a1, ad;            // dt/dx c1 and dt/dx c2/sqrt(3): advection factors per axis
};

// Geometry of one solve's padded distribution array: interior node
// (x, y, z) of velocity i sits at i*sv + org + z*sz + y*sy + x.  Two
// boundary layers pad each face; the y and z layers are rows and planes of
// the array.  The planes are ordered one of two ways:
//  - plane-major, f[mz][15][my][mx] (every level below 2 GiB): the 15
//    velocity planes of one z lie side by side (sv = plane stride,
//    sz = 15 sv), so a tile marching z reads and writes one compact region
//    per plane step rather than 15 regions a velocity block apart, which
//    the memory streams measurably faster;
//  - velocity-major, f[15][mz][my][mx] (larger levels): each velocity's
//    planes form one block (sz = plane, sv = block), so that everything the
//    tiled kernels reach from a velocity's base stays within 32-bit offsets.
// Plane (plane-major) and block (velocity-major) strides are odd numbers of
// 256-byte blocks, so that the 15 streams do not start on the same memory
// channel.  The x layers either sit in the row padding (xg = 0) or, when
// the rows are dense (mx = nx), in a block of their own: layer k (0: x = -2,
// 1: x = -1, 2: x = nx, 3: x = nx+1) of row (y, z) of velocity i at
// i*sv + xg + (z + 2) * xgz + (y + 2) * 4 + k (plane-major: right after each
// velocity plane; velocity-major: after each velocity block's planes).
struct Grid {
    int32_t nx, ny, nz;
    int32_t my;          // rows per plane (ny + 4)
    int64_t sy, sz, sv;  // strides of y, z and velocity (elements)
    int64_t org;         // offset of interior node (0,0,0)
    int64_t sink;        // offset from a velocity's base of a region of SINK_ROWS x TILE_X elements that is never read
    int64_t xg;          // offset from a velocity's base of its x-layer block, 0 if none
    int64_t xgz;         // z stride of the x-layer block
    int64_t len;         // elements of one level (one distribution buffer)
    int32_t plane_major; // 1: plane-major order, 0: velocity-major
};

struct FaceBC {
    int32_t kind[6];        // LBM3D_PERIODIC .. LBM3D_REFLECT per face
};

struct Device;  // per-solve device pointers, defined in lbm3d_api.cpp

// Precision modes (same values as the ABI enum).
enum Mode { MODE_FP64 = 0, MODE_FP32 = 1, MODE_FP32_T64 = 2 };

// One tile of the batched step: a 64 x BY x (z1 - z0) box of one solve.
// (32-bit fields: a solve may have up to 2^20 rows and 65535 planes.)
struct BatchTile {
    int32_t solve;        // index into the solve table
    int32_t txi, tyi;     // tile column (x0 = 64 txi, y0 = BY tyi)
    int32_t z0, z1;       // z range
};

// Work lists of the batched step: the tiles are split into `nlists` lists
// (one per XCD), list l holding tiles [first[l], first[l + 1]); the
// workgroups of a list take its tiles in order from a counter.
constexpr int BATCH_MAX_LISTS = 8;
struct BatchQueue {
    int32_t first[BATCH_MAX_LISTS + 1];
    uint32_t next[BATCH_MAX_LISTS];  // zero between launches
};

// Per-solve entry of the batched step (device memory, read uniformly).
struct BatchSolve {
    Grid g;
    FaceBC bc;
    int32_t cur0;         // buffer holding the current level at batch step 0
    double xin[2][5];     // fixed states of the x faces (rho, ux, uy, uz, T)
    void* f[2];           // the two distribution buffers
    uint32_t* health;
    Model<double> md;
    Model<float> mf;
};

// One solve's share of the batched boundary-layer launch: workgroups
// [first, next job's first) of 64 lines each over the faces in `faces`.
// Step count of a batch member within a run of the batched step: it takes
// part in the launches while done < target, and its current buffer is
// cur0 ^ (done & 1).  A counting launch after each step advances done.
struct BatchCount {
    int32_t done;
    int32_t target;
};

struct BatchLayerJob {
    int32_t solve;
    uint32_t faces;
    int32_t first;
};

// ---- launches (lbm3d_device.hip) ----
hipError_t launch_init(int mode, const Grid& g, const Model<double>& md, const double* q5,
                       void* f, hipStream_t s);
// Launch shape of the fused step: tile height BY (rows of 64 nodes; 0 selects
// the untiled one-node-per-thread kernel) and the z extent TZ of a tile.
struct TileCfg {
    int by = 4;
    int tz = 16;
    bool stream = true;  // non-temporal stores of the new level (tiled kernels)
};
// Stores of the new level: non-temporal (streaming past the caches) when the
// two levels of a solve exceed this many bytes, else plain.  A pair of
// levels that fits the 256 MB memory-side cache is read back from it by the
// next step when stored plainly (the step on the 298x78x78 grid, 240 MB,
// takes 61 us against 85 us streaming); larger ones gain nothing there and
// streaming keeps the L2 for the halo planes.  The autotuner tries both.
constexpr int64_t STREAM_MIN_BYTES = (int64_t)320 << 20;
TileCfg default_tile(int mode, const Grid& g);
// compute units of the current device (256 when it cannot be asked)
int device_cus();
bool tile_supported(int mode, const Grid& g, const TileCfg& t);
// the tiled kernels (single and batched) take this solve
bool tiled_fits(int mode, const Grid& g);
// Faces whose boundary layers the boundary-layer kernel refreshes after
// every step.  Fixed-state layers are written once at init.  The tiled
// kernels form the x layers themselves when 64-wide tiles cover x exactly
// (nx a multiple of 64) and wrap periodic faces, so with `tiled` those
// faces need no layers in memory.
uint32_t ghost_faces(const Grid& g, const FaceBC& bc, bool tiled);
// upwind2: the second-order upwind variant (untiled kernel only: tc.by == 0)
// ev_start / ev_stop (optional): events that the kernel's own dispatch
// records at its start and end (hipExtLaunchKernel), for timing the kernel
// without markers of their own around it.
hipError_t launch_step(int mode, const Grid& g, const FaceBC& bc, const TileCfg& tc, const Model<double>& md,
                       const Model<float>& mf, const double (*inflow)[5], const void* f, void* fn,
                       uint32_t* health, hipStream_t s, bool upwind2 = false, hipEvent_t ev_start = nullptr,
                       hipEvent_t ev_stop = nullptr);
// (rho, ux, uy, uz, T) of the two x faces' fixed states, from the ABI's
// (rho, ux, uy, uz, p)
void x_fixed_states(const double (*inflow)[5], double (&xin)[2][5]);
hipError_t launch_ghosts(int mode, const Grid& g, const FaceBC& bc, const Model<double>& md,
                         const double (*inflow)[5], bool include_fixed, void* f, hipStream_t s,
                         uint32_t face_mask = 0x3fu);
hipError_t launch_moments(int mode, const Grid& g, const Model<double>& md, const void* f,
                          double* q5, hipStream_t s);
hipError_t launch_conserved(int mode, const Grid& g, const Model<double>& md, const void* f,
                            double* partial, int nblocks, double* out5, hipStream_t s);
int conserved_blocks(const Grid& g);
hipError_t launch_pack(int mode, const Grid& g, const void* f, void* dense, bool to_dense,
                       hipStream_t s);
// One step of every solve in `solves` (device table) over the packed tile
// list (device); `parity` selects f[cur0 ^ parity] as the current level.
// Boundary layers of the members of a batch after a step (one launch).
// parity >= 0: every member steps from its buffer of that parity (relative
// to build); parity < 0: each member steps per its BatchCount (see above).
hipError_t launch_batch_layers(int mode, const BatchSolve* solves, const BatchLayerJob* jobs, const int32_t* block_job,
                               int nblocks, int parity, const BatchCount* counts, hipStream_t s);
// done += 1 for each of the n members with done < target.
hipError_t launch_batch_count(BatchCount* counts, int n, hipStream_t s);
// out[k] = the health word of member k (n members).
hipError_t launch_gather_health(const BatchSolve* solves, int n, uint32_t* out, hipStream_t s);
// One step of every member (parity as for launch_batch_layers): `nblocks`
// persistent workgroups (a multiple of `nlists`); workgroup b works on list
// b mod nlists.  `stream`: the store kind of the new level (see
// STREAM_MIN_BYTES).
hipError_t launch_batch_step(int mode, int by, bool stream, const BatchSolve* solves, const BatchTile* tiles,
                             BatchQueue* queue, int nlists, int nblocks, int parity, const BatchCount* counts,
                             hipStream_t s);

// block shape of the untiled step kernel; x extent of a tile of the tiled one;
// block size of the conservation reduction
constexpr int TX = 64, TY = 4;
constexpr int RB = 256;
constexpr int TILE_X = 64;
// Lanes of the tiled step outside the grid store unconditionally into a sink
// region past the array, each to its own element (row y mod SINK_ROWS, its
// lane): stores that all went to one element would queue on one address,
// which on ragged grids (every row's last tile overhangs the face) made the
// tiled step several times slower.
constexpr int SINK_ROWS = 64;

// Rows hold the interior only (mx = nx) when 64-wide tiles cover x exactly:
// the tiles then form the x boundary layers themselves and never read them
// from memory, and the x layers live in a block of their own.  Other rows
// are padded by a cache line that holds the x layers.
__host__ __device__ inline bool dense_rows(int nx) { return nx % TILE_X == 0; }

}  // namespace lbm3d
