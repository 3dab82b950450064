// Batched stepping: many solves of uneven size advanced by one persistent
// launch per step over per-XCD tile lists, with step runs replayed from a
// captured HIP graph.
#include "lbm3d_batch.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <set>

namespace lbm3d {

static int32_t herr(hipError_t e)
{
    return e == hipSuccess ? LBM3D_OK : (e == hipErrorOutOfMemory ? LBM3D_E_NOMEM : LBM3D_E_DEVICE);
}

// Steps per captured graph of the batched step (even: parities 0,1,...).
constexpr int BATCH_GRAPH_STEPS = 16;
// Planes a tile marches before its first update (the z prologue), counted
// in the cost that balances the lists.
constexpr double TILE_PROLOGUE_PLANES = 3.0;

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

int32_t plan_tiles(const std::vector<Grid>& grids, int by, int tz, int cus, TilePlan& out)
{
    out = TilePlan();
    if (by < 1 || tz < 1 || cus < 1) return LBM3D_E_INVAL;
    // every member's tiles in natural order: z chunk, then row, then column
    std::vector<BatchTile> all;
    std::vector<double> tcost;
    std::vector<size_t> mbegin(grids.size() + 1, 0);
    for (size_t k = 0; k < grids.size(); k++) {
        const Grid& g = grids[k];
        mbegin[k] = all.size();
        const int64_t ntx = (g.nx + TILE_X - 1) / TILE_X;
        const int64_t nty = (g.ny + by - 1) / by;
        const int64_t ntz = (g.nz + (int64_t)tz - 1) / tz;
        if ((int64_t)all.size() + ntx * nty * ntz > (int64_t)INT32_MAX) return LBM3D_E_INVAL;
        for (int64_t cz = 0; cz < ntz; cz++) {
            const int z0 = (int)(cz * tz);
            const int z1 = (int)std::min<int64_t>((int64_t)z0 + tz, g.nz);
            for (int64_t ty = 0; ty < nty; ty++)
                for (int64_t tx = 0; tx < ntx; tx++) {
                    BatchTile t;
                    t.solve = (int32_t)k;
                    t.txi = (int32_t)tx;
                    t.tyi = (int32_t)ty;
                    t.z0 = z0;
                    t.z1 = z1;
                    all.push_back(t);
                    tcost.push_back((z1 - z0) + TILE_PROLOGUE_PLANES);
                }
        }
    }
    mbegin[grids.size()] = all.size();
    const int n = (int)all.size();
    if (n == 0) return LBM3D_OK;
    int nblocks = std::min(n, cus);
    if (nblocks >= BATCH_MAX_LISTS) nblocks -= nblocks % BATCH_MAX_LISTS;
    const int nlists = std::min(BATCH_MAX_LISTS, nblocks);
    out.nblocks = nblocks;
    out.nlists = nlists;

    // contiguous pieces of each member, at most a quarter of a list's share each
    struct Piece {
        size_t begin, end;
        double cost;
    };
    double total = 0.0;
    for (double c : tcost) total += c;
    const double piece_max = nlists > 1 ? 0.25 * total / nlists : total;
    std::vector<Piece> pieces;
    for (size_t k = 0; k < grids.size(); k++) {
        double ck = 0.0;
        for (size_t j = mbegin[k]; j < mbegin[k + 1]; j++) ck += tcost[j];
        const int np = std::max(1, (int)std::ceil(ck / piece_max - 1e-9));
        size_t b = mbegin[k];
        double acc = 0.0;
        for (int p = 0; p < np; p++) {
            const double upto = ck * (p + 1) / np;
            size_t e = b;
            double pc = 0.0;
            while (e < mbegin[k + 1] && (p == np - 1 || acc + tcost[e] <= upto + 1e-9 || e == b)) {
                acc += tcost[e];
                pc += tcost[e];
                e++;
            }
            if (e > b) pieces.push_back(Piece{b, e, pc});
            b = e;
        }
    }
    // largest piece first onto the least-loaded list
    std::stable_sort(pieces.begin(), pieces.end(), [](const Piece& a, const Piece& b) { return a.cost > b.cost; });
    std::vector<std::vector<const Piece*>> lists((size_t)nlists);
    for (const Piece& p : pieces) {
        int best = 0;
        for (int l = 1; l < nlists; l++)
            if (out.cost[l] < out.cost[best]) best = l;
        lists[(size_t)best].push_back(&p);
        out.cost[best] += p.cost;
    }
    // each list: its pieces' tiles, deepest first (the order within a depth
    // is kept, so neighbouring tiles run together)
    out.tiles.reserve((size_t)n);
    for (int l = 0; l < nlists; l++) {
        out.queue.first[l] = (int32_t)out.tiles.size();
        std::vector<BatchTile> lt;
        for (const Piece* p : lists[(size_t)l])
            for (size_t j = p->begin; j < p->end; j++) lt.push_back(all[j]);
        std::stable_sort(lt.begin(), lt.end(),
                         [](const BatchTile& a, const BatchTile& b) { return (a.z1 - a.z0) > (b.z1 - b.z0); });
        out.tiles.insert(out.tiles.end(), lt.begin(), lt.end());
    }
    for (int l = nlists; l <= BATCH_MAX_LISTS; l++) out.queue.first[l] = (int32_t)out.tiles.size();
    for (int l = 0; l < BATCH_MAX_LISTS; l++) out.queue.next[l] = 0;
    return LBM3D_OK;
}

BatchPlan::~BatchPlan()
{
    if (last_stream_) (void)hipStreamSynchronize(last_stream_);
    release_graph();
    if (capture_stream_) (void)hipStreamDestroy(capture_stream_);
    if (dmem_) (void)hipFree(dmem_);
}

void BatchPlan::release_graph()
{
    // (callers have drained the stream the graph was launched on)
    if (graph_) (void)hipGraphExecDestroy(graph_);
    graph_ = nullptr;
}

// Tile depth from a launch model of a membership: the persistent
// workgroups share the tiles' work (each tile's planes plus the planes its
// z ring loads first), and no launch ends before its longest tile.  The
// depth (16, 32, ... up to whole columns) with the lowest estimate wins,
// the deeper one on a tie: whole columns for a batch as large as the
// 64-solve mix (as the tuner finds), short chunks for a few solves, whose
// whole columns would leave most compute units idle.
static int model_depth(const std::vector<Grid>& grids, int by, int cus)
{
    int maxnz = 1;
    for (const Grid& g : grids) maxnz = std::max(maxnz, g.nz);
    int best = 0;
    double best_t = 0.0;
    for (int d = 16;; d *= 2) {
        const int dd = std::min(d, maxnz);
        double work = 0.0, longest = 0.0;
        for (const Grid& g : grids) {
            const double cols = (double)((g.nx + TILE_X - 1) / TILE_X) * ((g.ny + by - 1) / by);
            const double chunks = (double)((g.nz + dd - 1) / dd);
            work += cols * (g.nz + TILE_PROLOGUE_PLANES * chunks);
            longest = std::max(longest, std::min(dd, g.nz) + TILE_PROLOGUE_PLANES);
        }
        const double t = std::max(work / cus, longest);
        if (best == 0 || t <= best_t) {
            best = dd;
            best_t = t;
        }
        if (dd >= maxnz) break;
    }
    return best;
}

// Tile depth of a plan: tz > 0 as given; 0: the precision's tuned depth,
// else the model's; < 0: the model's (memberships that change from tick to
// tick, whose best depth no earlier tuning knows).
static int plan_depth(int mode, int tz, const std::vector<Grid>& grids, int by, int cus)
{
    if (tz > 0) return tz;
    if (tz == 0) {
        const int t = batch_tile_depth(mode);
        if (t > 0) return t;
    }
    return model_depth(grids, by, cus);
}

// layer jobs of the members (faces the tiles leave to memory)
static void layer_jobs(const std::vector<lbm3d_solver*>& members, std::vector<uint32_t>& rest,
                       std::vector<BatchLayerJob>& ljobs, std::vector<int32_t>& block_job, int& nlblocks)
{
    rest.assign(members.size(), 0u);
    ljobs.clear();
    nlblocks = 0;
    for (size_t k = 0; k < members.size(); k++) {
        const Grid& g = members[k]->g;
        const uint32_t faces = ghost_faces(g, members[k]->bc, true);
        rest[k] = faces;
        if (!faces) continue;
        int64_t lines = 0;
        for (int face = 0; face < 6; face++) {
            if (!((faces >> face) & 1)) continue;
            const int axis = face >> 1;
            lines += axis == 0 ? (int64_t)g.ny * g.nz : axis == 1 ? (int64_t)g.nx * g.nz : (int64_t)g.nx * g.ny;
        }
        BatchLayerJob jb;
        jb.solve = (int32_t)k;
        jb.faces = faces;
        jb.first = nlblocks;
        ljobs.push_back(jb);
        nlblocks += (int)((lines + 63) / 64);
    }
    block_job.assign((size_t)nlblocks, 0);
    for (size_t j = 0; j < ljobs.size(); j++) {
        const int end = j + 1 < ljobs.size() ? ljobs[j + 1].first : nlblocks;
        for (int b = ljobs[j].first; b < end; b++) block_job[(size_t)b] = (int32_t)j;
    }
}

static size_t tables_need(size_t nmembers, size_t ntiles, size_t nljobs, size_t nlblocks)
{
    return align256(nmembers * sizeof(BatchSolve)) + align256(ntiles * sizeof(BatchTile)) +
           align256(sizeof(BatchQueue)) + align256(nljobs * sizeof(BatchLayerJob)) +
           align256(nlblocks * sizeof(int32_t)) + align256(nmembers * sizeof(BatchCount)) +
           nmembers * sizeof(uint32_t) + 256;
}

size_t BatchPlan::table_bytes(const std::vector<lbm3d_solver*>& members, int tz)
{
    if (members.empty()) return 0;
    const int mode = members[0]->mode;
    const int by = mode == LBM3D_FP64 ? 4 : 8;
    std::vector<Grid> grids;
    for (lbm3d_solver* h : members) grids.push_back(h->g);
    TilePlan p;
    const int cus = device_cus();
    if (plan_tiles(grids, by, plan_depth(mode, tz, grids, by, cus), cus, p) != LBM3D_OK) return (size_t)-1;
    std::vector<uint32_t> rest;
    std::vector<BatchLayerJob> lj;
    std::vector<int32_t> bj;
    int nlb = 0;
    layer_jobs(members, rest, lj, bj, nlb);
    return tables_need(members.size(), p.tiles.size(), lj.size(), (size_t)nlb);
}

int32_t BatchPlan::build(const std::vector<lbm3d_solver*>& members, hipStream_t s, int tz, void* dev, size_t cap)
{
    // work still queued may read the old tables or replay the old graph
    if (last_stream_ && hipStreamSynchronize(last_stream_) != hipSuccess) return LBM3D_E_DEVICE;
    last_stream_ = nullptr;
    release_graph();
    members_ = members;
    plan_ = TilePlan();
    hcount_.assign(members.size(), BatchCount{0, 0});
    count_pending_ = false;
    if (members.empty()) return LBM3D_OK;
    mode_ = members[0]->mode;
    by_ = mode_ == LBM3D_FP64 ? 4 : 8;
    // plain stores when the members' levels together fit the memory-side
    // cache, as for a single solve
    int64_t level_bytes = 0;
    for (lbm3d_solver* h : members) level_bytes += 2 * (int64_t)f_bytes(h->g, h->mode);
    stream_ = level_bytes > STREAM_MIN_BYTES;
    std::vector<Grid> grids;
    for (lbm3d_solver* h : members) grids.push_back(h->g);
    const int cus = device_cus();
    tz_ = plan_depth(mode_, tz, grids, by_, cus);
    int32_t rc = plan_tiles(grids, by_, tz_, cus, plan_);
    if (rc) return rc;

    std::vector<BatchSolve> table(members.size());
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
    }
    std::vector<BatchLayerJob> ljobs;
    std::vector<int32_t> block_job;
    layer_jobs(members, ghost_rest_, ljobs, block_job, nlblocks_);
    nljobs_ = (int)ljobs.size();

    const size_t sb = table.size() * sizeof(BatchSolve);
    const size_t tb = plan_.tiles.size() * sizeof(BatchTile);
    const size_t lb = ljobs.size() * sizeof(BatchLayerJob);
    const size_t bb = block_job.size() * sizeof(int32_t);
    const size_t need = tables_need(table.size(), plan_.tiles.size(), ljobs.size(), block_job.size());
    char* base = nullptr;
    if (dev) {
        if (need > cap) return LBM3D_E_NOMEM;
        if (dmem_) {
            (void)hipFree(dmem_);
            dmem_ = nullptr;
            dbytes_ = 0;
        }
        base = (char*)dev;
    } else {
        if (need > dbytes_) {
            if (dmem_) (void)hipFree(dmem_);
            dmem_ = nullptr;
            dbytes_ = 0;
            hipError_t e = hipMalloc(&dmem_, need);
            if (e != hipSuccess) return herr(e);
            dbytes_ = need;
        }
        base = (char*)dmem_;
    }
    dsolves_ = (BatchSolve*)base;
    dtiles_ = (BatchTile*)(base + align256(sb));
    dqueue_ = (BatchQueue*)((char*)dtiles_ + align256(tb));
    dlayers_ = (BatchLayerJob*)((char*)dqueue_ + align256(sizeof(BatchQueue)));
    dblockjob_ = (int32_t*)((char*)dlayers_ + align256(lb));
    const size_t cb = hcount_.size() * sizeof(BatchCount);
    dcount_ = (BatchCount*)((char*)dblockjob_ + align256(bb));
    dhealth_ = (uint32_t*)((char*)dcount_ + align256(cb));
    hipError_t e = hipMemcpyAsync(dsolves_, table.data(), sb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dtiles_, plan_.tiles.data(), tb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dqueue_, &plan_.queue, sizeof(BatchQueue), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && lb) e = hipMemcpyAsync(dlayers_, ljobs.data(), lb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && bb) e = hipMemcpyAsync(dblockjob_, block_job.data(), bb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dcount_, hcount_.data(), cb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // host tables die at return
    last_stream_ = nullptr;
    return herr(e);
}

int32_t BatchPlan::health(std::vector<uint32_t>& out, hipStream_t s)
{
    out.assign(members_.size(), 0u);
    if (members_.empty()) return LBM3D_OK;
    hipError_t e = launch_gather_health(dsolves_, (int)members_.size(), dhealth_, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out.data(), dhealth_, out.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && s == last_stream_) count_pending_ = false;
    return herr(e);
}

hipError_t BatchPlan::launch_at(int parity, hipStream_t s)
{
    last_stream_ = s;
    return enqueue(parity & 1, s);
}

hipError_t BatchPlan::enqueue(int parity, hipStream_t s)
{
    hipError_t e = launch_batch_step(mode_, by_, stream_, dsolves_, dtiles_, dqueue_, plan_.nlists, plan_.nblocks,
                                     parity, dcount_, s);
    if (e != hipSuccess) return e;
    // boundary layers the tiles do not form themselves, all members at once
    e = launch_batch_layers(mode_, dsolves_, dlayers_, dblockjob_, nlblocks_, parity, dcount_, s);
    if (e != hipSuccess || parity >= 0) return e;
    return launch_batch_count(dcount_, (int)members_.size(), s);
}

int32_t BatchPlan::run(int64_t k, hipStream_t s, bool graphs, const std::vector<int64_t>* limit)
{
    if (members_.empty() || k <= 0) return LBM3D_OK;
    if (limit && limit->size() != members_.size()) return LBM3D_E_INVAL;
    // the counts are 32-bit: very long runs go in pieces
    constexpr int64_t PIECE = (int64_t)1 << 30;
    if (k > PIECE) {
        std::vector<int64_t> rest = limit ? *limit : std::vector<int64_t>(members_.size(), k);
        for (int64_t left = k; left > 0;) {
            const int64_t c = std::min(left, PIECE);
            int32_t rc = run(c, s, graphs, &rest);
            if (rc) return rc;
            for (int64_t& r : rest) r = std::max<int64_t>(0, r - c);
            left -= c;
        }
        return LBM3D_OK;
    }
    // the counts of the last run may still be on their way from hcount_
    if (count_pending_ && last_stream_ && hipStreamSynchronize(last_stream_) != hipSuccess) return LBM3D_E_DEVICE;
    count_pending_ = false;
    last_stream_ = s;
    // this run's counts: done restarts at each member's parity since build
    // (so it never grows), target = done + the member's steps
    std::vector<int64_t> steps(members_.size(), k);
    for (size_t m = 0; m < members_.size(); m++) {
        if (limit) steps[m] = std::max<int64_t>(0, std::min<int64_t>(k, (*limit)[m]));
        hcount_[m].done &= 1;
        hcount_[m].target = hcount_[m].done + (int32_t)steps[m];
    }
    hipError_t e = hipMemcpyAsync(dcount_, hcount_.data(), hcount_.size() * sizeof(BatchCount),
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return herr(e);
    count_pending_ = true;
    int64_t left = k;
    // the launches carry nothing step-specific (each member's parity comes
    // from its count), so one captured run of BATCH_GRAPH_STEPS serves all
    while (graphs && left >= BATCH_GRAPH_STEPS) {
        if (!graph_) {
            if (!capture_stream_) {
                e = hipStreamCreateWithFlags(&capture_stream_, hipStreamNonBlocking);
                if (e != hipSuccess) return herr(e);
            }
            hipGraph_t graph = nullptr;
            e = hipStreamBeginCapture(capture_stream_, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return herr(e);
            for (int j = 0; j < BATCH_GRAPH_STEPS && e == hipSuccess; j++) e = enqueue(-1, capture_stream_);
            hipError_t e2 = hipStreamEndCapture(capture_stream_, &graph);
            if (e != hipSuccess || e2 != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return herr(e != hipSuccess ? e : e2);
            }
            e = hipGraphInstantiate(&graph_, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) return herr(e);
        }
        e = hipGraphLaunch(graph_, s);
        if (e != hipSuccess) return herr(e);
        left -= BATCH_GRAPH_STEPS;
    }
    for (; left > 0; left--) {
        e = enqueue(-1, s);
        if (e != hipSuccess) return herr(e);
    }
    // members advance by their steps; their current buffer flips with an
    // odd count (the device table keeps the build-time buffers, and each
    // count's done its parity since build)
    for (size_t m = 0; m < members_.size(); m++) {
        lbm3d_solver* h = members_[m];
        const int64_t n = steps[m];
        hcount_[m].done = (hcount_[m].done + (int32_t)(n & 1)) & 1;
        if (n == 0) continue;
        h->steps += n;
        if (n & 1) h->cur ^= 1;
        // a member that steps alone untiled reads every layer from memory:
        // refresh the ones the tiled batch kernel formed itself
        if (h->tile.by == 0) {
            e = launch_ghosts(h->mode, h->g, h->bc, h->md, h->p.inflow, false, h->f[h->cur], s);
            if (e != hipSuccess) return herr(e);
        }
    }
    return LBM3D_OK;
}

// Checks shared by the batched entry points: non-null distinct handles,
// initialised, one precision, within the tiled kernels' addressing.
int32_t check_batch(lbm3d_t* hs, int32_t count)
{
    if (!hs || count < 1) return LBM3D_E_INVAL;
    std::set<lbm3d_t> seen;
    for (int32_t k = 0; k < count; k++) {
        if (!hs[k] || !seen.insert(hs[k]).second) return LBM3D_E_INVAL;
        if (!hs[k]->initialised) return LBM3D_E_STATE;
        if (hs[k]->mode != hs[0]->mode) return LBM3D_E_INVAL;
        if (!tiled_fits(hs[k]->mode, hs[k]->g)) return LBM3D_E_INVAL;
        if (hs[k]->upwind2) return LBM3D_E_INVAL;  // the batched kernel is NND only
    }
    return LBM3D_OK;
}

// Steps of a batch whose members need different step counts: runs of the
// common count with the members that still have steps to do.
int32_t batch_advance(lbm3d_t* hs, int32_t count, const int64_t* nsteps, hipStream_t s, BatchPlan& plan,
                      void* dev, size_t cap, bool graphs)
{
    std::vector<lbm3d_solver*> active;
    std::vector<int64_t> limit;
    int64_t k = 0;
    for (int32_t j = 0; j < count; j++)
        if (nsteps[j] > 0) {
            active.push_back(hs[j]);
            limit.push_back(nsteps[j]);
            k = std::max(k, nsteps[j]);
        }
    if (!active.empty()) {
        int32_t rc = plan.build(active, s, 0, dev, cap);
        if (rc) return rc;
        rc = plan.run(k, s, graphs, &limit);
        if (rc) return rc;
    }
    return hipStreamSynchronize(s) == hipSuccess ? LBM3D_OK : LBM3D_E_DEVICE;
}

}  // namespace lbm3d

// ------------------------------------------------------------------- C ABI --
using namespace lbm3d;

extern "C" int32_t lbm3d_batch_step(lbm3d_t* hs, int32_t count, const int64_t* nsteps)
{
    int32_t rc = check_batch(hs, count);
    if (rc) return rc;
    if (!nsteps) return LBM3D_E_INVAL;
    for (int32_t k = 0; k < count; k++)
        if (nsteps[k] < 0) return LBM3D_E_INVAL;
    hipStream_t s = hs[0]->stream;
    // work already queued on the other solves' streams precedes the batch
    for (int32_t k = 1; k < count; k++)
        if (hs[k]->stream != s && hipStreamSynchronize(hs[k]->stream) != hipSuccess) return LBM3D_E_DEVICE;
    BatchPlan plan;
    return batch_advance(hs, count, nsteps, s, plan, nullptr, 0, true);
}

// ------------------------------------------------ the allocation-free step --
// The tables of lbm3d_batch_step_noalloc (solve table, tile lists and their
// counters, boundary-layer jobs, health words) live in this array, one copy
// per device, held until the process ends.  In host code its name is only a
// stand-in: the device address of each device's copy comes from
// hipGetSymbolAddress and is kept per device.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)4 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::vector<void*> g_scratch;  // device address of `scratch` per device (nullptr: not looked up yet)
}  // namespace

// The device address of the current device's scratch array (looked up once
// per device, with that device current).
static int32_t scratch_address(void** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return LBM3D_E_DEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((size_t)dev >= g_scratch.size()) g_scratch.resize((size_t)dev + 1, nullptr);
    if (!g_scratch[(size_t)dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return LBM3D_E_DEVICE;
        g_scratch[(size_t)dev] = ptr;
    }
    *out = g_scratch[(size_t)dev];
    return LBM3D_OK;
}

extern "C" int32_t lbm3d_batch_step_noalloc(lbm3d_t* hs, int32_t count, const int64_t* nsteps)
{
    int32_t rc = check_batch(hs, count);
    if (rc) return rc;
    if (!nsteps) return LBM3D_E_INVAL;
    for (int32_t k = 0; k < count; k++)
        if (nsteps[k] < 0) return LBM3D_E_INVAL;
    std::vector<lbm3d_solver*> members(hs, hs + count);
    // the full membership needs the largest tables of the call
    if (BatchPlan::table_bytes(members) > NOALLOC_SCRATCH_BYTES) return LBM3D_E_NOMEM;
    void* ptr = nullptr;
    rc = scratch_address(&ptr);
    if (rc) return rc;
    hipStream_t s = hs[0]->stream;
    for (int32_t k = 1; k < count; k++)
        if (hs[k]->stream != s && hipStreamSynchronize(hs[k]->stream) != hipSuccess) return LBM3D_E_DEVICE;
    BatchPlan plan;  // tables in the scratch array, steps launched directly (no graph)
    return batch_advance(hs, count, nsteps, s, plan, ptr, NOALLOC_SCRATCH_BYTES, false);
}

extern "C" int32_t lbm3d_batch_plan(const lbm3d_params* ps, int32_t count, int32_t tz, int32_t cus,
                                    int32_t* ntiles, int32_t* nlists, int32_t* nblocks, int32_t* tiles,
                                    int64_t cap, int32_t* list_first)
{
    if (!ps || count < 1 || cus < 1) return LBM3D_E_INVAL;
    std::vector<Grid> grids;
    for (int32_t k = 0; k < count; k++) {
        int32_t rc = validate(&ps[k]);
        if (rc) return rc;
        if (ps[k].precision != ps[0].precision || (ps[k].flags & LBM3D_UPWIND2)) return LBM3D_E_INVAL;
        const Grid g = make_grid(&ps[k]);
        if (!tiled_fits(ps[k].precision, g)) return LBM3D_E_INVAL;
        grids.push_back(g);
    }
    const int mode = ps[0].precision;
    const int by = mode == LBM3D_FP64 ? 4 : 8;
    TilePlan p;
    int32_t rc = plan_tiles(grids, by, plan_depth(mode, tz, grids, by, cus), cus, p);
    if (rc) return rc;
    const int64_t n = (int64_t)p.tiles.size();
    if (ntiles) *ntiles = (int32_t)n;
    if (nlists) *nlists = p.nlists;
    if (nblocks) *nblocks = p.nblocks;
    if (list_first)
        for (int l = 0; l <= BATCH_MAX_LISTS; l++) list_first[l] = p.queue.first[l];
    if (tiles) {
        if (cap < n) return LBM3D_E_NOMEM;
        for (int64_t j = 0; j < n; j++) {
            const BatchTile& t = p.tiles[(size_t)j];
            const Grid& g = grids[(size_t)t.solve];
            int32_t* o = tiles + 7 * j;
            o[0] = t.solve;
            o[1] = t.txi * TILE_X;
            o[2] = std::min(o[1] + TILE_X, g.nx);
            o[3] = t.tyi * by;
            o[4] = std::min(o[3] + by, g.ny);
            o[5] = t.z0;
            o[6] = t.z1;
        }
    }
    return LBM3D_OK;
}
