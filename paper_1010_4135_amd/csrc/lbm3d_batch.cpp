// Batched stepping: many solves of uneven size advanced by one persistent
// launch per step over a packed tile list, with step runs replayed from a
// captured HIP graph.
#include "lbm3d_batch.h"

#include <algorithm>
#include <cstring>
#include <new>
#include <set>

namespace lbm3d {

static int32_t herr(hipError_t e)
{
    return e == hipSuccess ? LBM3D_OK : (e == hipErrorOutOfMemory ? LBM3D_E_NOMEM : LBM3D_E_DEVICE);
}

// Steps per captured graph of the batched step (even: parities 0,1,...).
constexpr int BATCH_GRAPH_STEPS = 16;
// z extent of a batch tile (build-time tuning knob)
#ifndef LBM3D_BATCH_TZ
#define LBM3D_BATCH_TZ 16
#endif

BatchPlan::~BatchPlan()
{
    release_graph();
    if (capture_stream_) (void)hipStreamDestroy(capture_stream_);
    if (dmem_) (void)hipFree(dmem_);
}

void BatchPlan::release_graph()
{
    if (graph_) (void)hipGraphExecDestroy(graph_);
    graph_ = nullptr;
}

int32_t BatchPlan::build(const std::vector<lbm3d_solver*>& members, hipStream_t s, int tz)
{
    release_graph();
    members_ = members;
    ntiles_ = 0;
    parity_ = 0;
    if (members.empty()) return LBM3D_OK;
    mode_ = members[0]->mode;
    by_ = mode_ == LBM3D_FP64 ? 4 : 8;
    // tile depth: the caller's, else the tuned one, else the build default
    tz_ = tz > 0 ? tz : batch_tile_depth(mode_);
    if (tz_ <= 0) tz_ = LBM3D_BATCH_TZ;

    // packed tile list: each solve's tiles in (z chunk, y, x) order, split
    // into eight contiguous runs interleaved so that run c lands on XCD c
    // (workgroup b runs tiles b, b + G, ... with G a multiple of 8)
    std::vector<BatchTile> order;
    std::vector<BatchSolve> table(members.size());
    ghost_rest_.assign(members.size(), 0u);
    cur0_.assign(members.size(), 0);
    for (size_t k = 0; k < members.size(); k++) {
        lbm3d_solver* h = members[k];
        BatchSolve& d = table[k];
        std::memset(&d, 0, sizeof(d));
        d.g = h->g;
        d.bc = h->bc;
        d.cur0 = h->cur;
        x_fixed_states(h->p.inflow, d.xin);
        d.f[0] = h->f[0];
        d.f[1] = h->f[1];
        d.health = h->health;
        d.md = h->md;
        d.mf = h->mf;
        ghost_rest_[k] = ghost_faces(h->g, h->bc, true);
        cur0_[k] = h->cur;
        const int ntx = (h->g.nx + TILE_X - 1) / TILE_X;
        const int nty = (h->g.ny + by_ - 1) / by_;
        for (int z0 = 0; z0 < h->g.nz; z0 += tz_)
            for (int ty = 0; ty < nty; ty++)
                for (int tx = 0; tx < ntx; tx++) {
                    BatchTile t;
                    t.solve = (int32_t)k;
                    t.txi = (int16_t)tx;
                    t.tyi = (int16_t)ty;
                    t.z0 = (int16_t)z0;
                    t.z1 = (int16_t)std::min(z0 + tz_, h->g.nz);
                    order.push_back(t);
                }
    }
    const int n = (int)order.size();
    std::vector<BatchTile> tiles(n);
    const int per = n / 8, rem = n % 8;
    int pos = 0;
    for (int c = 0; c < 8; c++) {
        // slots c, c+8, c+16, ... (all < n) take run c of the natural order
        const int cnt = per + (c < rem ? 1 : 0);
        for (int j = 0; j < cnt; j++) tiles[8 * j + c] = order[pos + j];
        pos += cnt;
    }
    ntiles_ = n;
    // persistent grid: a multiple of 8 workgroups, about what the GPU holds
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
            cus = prop.multiProcessorCount;
    }
    // (one workgroup per CU is what the LDS of a tile leaves room for)
    nblocks_ = std::min(n, cus);
    if (nblocks_ >= 8) nblocks_ -= nblocks_ % 8;

    // boundary layers left after each step: one launch over all members
    std::vector<BatchLayerJob> ljobs;
    nlblocks_ = 0;
    for (size_t k = 0; k < members.size(); k++) {
        const uint32_t faces = ghost_rest_[k];
        if (!faces) continue;
        const Grid& g = members[k]->g;
        int64_t lines = 0;
        for (int face = 0; face < 6; face++) {
            if (!((faces >> face) & 1)) continue;
            const int axis = face >> 1;
            lines += axis == 0 ? (int64_t)g.ny * g.nz : axis == 1 ? (int64_t)g.nx * g.nz : (int64_t)g.nx * g.ny;
        }
        BatchLayerJob jb;
        jb.solve = (int32_t)k;
        jb.faces = faces;
        jb.first = nlblocks_;
        ljobs.push_back(jb);
        nlblocks_ += (int)((lines + 63) / 64);
    }
    nljobs_ = (int)ljobs.size();
    std::vector<int32_t> block_job((size_t)nlblocks_);
    for (int j = 0; j < nljobs_; j++) {
        const int end = j + 1 < nljobs_ ? ljobs[j + 1].first : nlblocks_;
        for (int b = ljobs[j].first; b < end; b++) block_job[(size_t)b] = j;
    }

    const size_t sb = table.size() * sizeof(BatchSolve);
    const size_t tb = (size_t)n * sizeof(BatchTile);
    const size_t lb = ljobs.size() * sizeof(BatchLayerJob);
    const size_t bb = block_job.size() * sizeof(int32_t);
    const size_t need = ((sb + 255) / 256) * 256 + ((tb + 255) / 256) * 256 + ((lb + 255) / 256) * 256 + bb + 256;
    if (need > dbytes_) {
        if (dmem_) (void)hipFree(dmem_);
        dmem_ = nullptr;
        dbytes_ = 0;
        hipError_t e = hipMalloc(&dmem_, need);
        if (e != hipSuccess) return herr(e);
        dbytes_ = need;
    }
    dsolves_ = (BatchSolve*)dmem_;
    dtiles_ = (BatchTile*)((char*)dmem_ + ((sb + 255) / 256) * 256);
    dlayers_ = (BatchLayerJob*)((char*)dtiles_ + ((tb + 255) / 256) * 256);
    dblockjob_ = (int32_t*)((char*)dlayers_ + ((lb + 255) / 256) * 256);
    hipError_t e = hipMemcpyAsync(dsolves_, table.data(), sb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dtiles_, tiles.data(), tb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && lb) e = hipMemcpyAsync(dlayers_, ljobs.data(), lb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && bb) e = hipMemcpyAsync(dblockjob_, block_job.data(), bb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // host tables die at return
    return herr(e);
}

hipError_t BatchPlan::launch_once(hipStream_t s) { return enqueue(0, s); }

hipError_t BatchPlan::enqueue(int parity, hipStream_t s)
{
    hipError_t e = launch_batch_step(mode_, by_, dsolves_, dtiles_, ntiles_, nblocks_, parity, s);
    if (e != hipSuccess) return e;
    // boundary layers the tiles do not form themselves, all members at once
    return launch_batch_layers(mode_, dsolves_, dlayers_, dblockjob_, nlblocks_, parity, s);
}

int32_t BatchPlan::run(int64_t k, hipStream_t s)
{
    if (members_.empty() || k <= 0) return LBM3D_OK;
    int64_t left = k;
    // align to an even parity so the captured graph (parities 0,1,...) applies
    if (parity_ & 1) {
        hipError_t e = enqueue(1, s);
        if (e != hipSuccess) return herr(e);
        parity_ ^= 1;
        left--;
    }
    while (left >= BATCH_GRAPH_STEPS) {
        if (!graph_) {
            if (!capture_stream_) {
                hipError_t e = hipStreamCreateWithFlags(&capture_stream_, hipStreamNonBlocking);
                if (e != hipSuccess) return herr(e);
            }
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamBeginCapture(capture_stream_, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return herr(e);
            for (int j = 0; j < BATCH_GRAPH_STEPS && e == hipSuccess; j++) e = enqueue(j & 1, capture_stream_);
            hipError_t e2 = hipStreamEndCapture(capture_stream_, &graph);
            if (e != hipSuccess || e2 != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return herr(e != hipSuccess ? e : e2);
            }
            e = hipGraphInstantiate(&graph_, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) return herr(e);
        }
        hipError_t e = hipGraphLaunch(graph_, s);
        if (e != hipSuccess) return herr(e);
        left -= BATCH_GRAPH_STEPS;
    }
    for (; left > 0; left--) {
        hipError_t e = enqueue(parity_, s);
        if (e != hipSuccess) return herr(e);
        parity_ ^= 1;
    }
    // members advance by k steps; their current buffer flips with odd k (the
    // device table keeps the build-time buffers and parity_ the offset)
    for (lbm3d_solver* h : members_) {
        h->steps += k;
        if (k & 1) h->cur ^= 1;
        // a member that steps alone untiled reads every layer from memory:
        // refresh the ones the tiled batch kernel formed itself
        if (h->tile.by == 0) {
            hipError_t e = launch_ghosts(h->mode, h->g, h->bc, h->md, h->p.inflow, false, h->f[h->cur], s);
            if (e != hipSuccess) return herr(e);
        }
    }
    return LBM3D_OK;
}

}  // namespace lbm3d

// ------------------------------------------------------------------- C ABI --
using namespace lbm3d;

extern "C" int32_t lbm3d_batch_step(lbm3d_t* hs, int32_t count, const int64_t* nsteps)
{
    if (!hs || !nsteps || count < 1) return LBM3D_E_INVAL;
    std::set<lbm3d_t> seen;
    for (int32_t k = 0; k < count; k++) {
        if (!hs[k] || nsteps[k] < 0 || !seen.insert(hs[k]).second) return LBM3D_E_INVAL;
        if (!hs[k]->initialised) return LBM3D_E_STATE;
        if (hs[k]->mode != hs[0]->mode) return LBM3D_E_INVAL;
        if (!lbm3d::tiled_fits(hs[k]->mode, hs[k]->g)) return LBM3D_E_INVAL;
    }
    hipStream_t s = hs[0]->stream;
    // work already queued on the other solves' streams precedes the batch
    for (int32_t k = 1; k < count; k++)
        if (hs[k]->stream != s && hipStreamSynchronize(hs[k]->stream) != hipSuccess) return LBM3D_E_DEVICE;
    std::vector<int64_t> left(nsteps, nsteps + count);
    BatchPlan plan;
    for (;;) {
        std::vector<lbm3d_solver*> active;
        int64_t k = 0;
        for (int32_t j = 0; j < count; j++)
            if (left[j] > 0) {
                active.push_back(hs[j]);
                k = (k == 0) ? left[j] : std::min(k, left[j]);
            }
        if (active.empty()) break;
        int32_t rc = plan.build(active, s);
        if (rc) return rc;
        rc = plan.run(k, s);
        if (rc) return rc;
        for (int32_t j = 0; j < count; j++)
            if (left[j] > 0) left[j] -= k;
    }
    return hipStreamSynchronize(s) == hipSuccess ? LBM3D_OK : LBM3D_E_DEVICE;
}
