// Batched stepping of many solves with one launch per step (internal).
#pragma once

#include <vector>

#include "lbm3d_api_impl.h"

namespace lbm3d {

// Work plan of a batched step, computed on the host: the tiles of every
// member split into per-XCD lists (see plan_tiles).
struct TilePlan {
    std::vector<BatchTile> tiles;  // list 0's tiles, then list 1's, ...
    BatchQueue queue{};            // list boundaries; counters zero
    int nlists = 0;                // lists (one per XCD, fewer for tiny batches)
    int nblocks = 0;               // persistent workgroups, a multiple of nlists
    double cost[BATCH_MAX_LISTS] = {};  // planes marched per list (balance)
};

// Tiles of 64 x `by` x `tz` nodes (tz >= nz: whole columns) over the grids,
// for `cus` compute units.  Each member's tiles are cut into contiguous
// pieces (row slabs, which share their halo rows through one L2), the pieces
// are dealt to the lists largest first onto the least-loaded list, and each
// list runs its deepest tiles first.  Host only.
int32_t plan_tiles(const std::vector<Grid>& grids, int by, int tz, int cus, TilePlan& out);

// A fixed set of solves (one precision) advanced together: a device table
// of the solves, the tile lists over all of them and a persistent launch
// per step; runs of steps are replayed from a captured graph.
class BatchPlan {
public:
    BatchPlan() = default;
    ~BatchPlan();
    BatchPlan(const BatchPlan&) = delete;
    BatchPlan& operator=(const BatchPlan&) = delete;

    // (Re)build for `members` (all initialised, same precision); each
    // member's current buffer is taken as parity 0.  Enqueued on `s`.
    // `tz` > 0 sets the tile depth; 0 takes the tuned depth of the
    // precision, else the launch model's; < 0 the launch model's.
    // The device tables go into a buffer the plan allocates, or, with
    // `dev` != nullptr, into the caller's `cap` bytes at `dev` (then nothing
    // is allocated and E_NOMEM is returned if they do not fit).
    int32_t build(const std::vector<lbm3d_solver*>& members, hipStream_t s, int tz = 0,
                  void* dev = nullptr, size_t cap = 0);
    // Device bytes the tables of `members` need at tile depth tz (0: the
    // depth as for build).
    static size_t table_bytes(const std::vector<lbm3d_solver*>& members, int tz = 0);
    // One step of every member from its buffer of the given parity
    // (relative to build) into the other one, boundary layers included,
    // without advancing the members' step counters or parity (for timing).
    hipError_t launch_at(int parity, hipStream_t s);
    // Enqueue k launches of the step on `s`, in which member m takes
    // min(k, limit[m]) steps (k each without `limit`; a member that is done
    // sits out the remaining launches), and update the members' buffer
    // parity and step counters; `graphs` = false launches every step
    // directly (no graph is instantiated).
    int32_t run(int64_t k, hipStream_t s, bool graphs = true, const std::vector<int64_t>* limit = nullptr);
    // Health words of the members (in build order) after the work queued
    // on `s`; waits for `s`.
    int32_t health(std::vector<uint32_t>& out, hipStream_t s);
    int ntiles() const { return (int)plan_.tiles.size(); }
    int by() const { return by_; }
    int tz() const { return tz_; }

private:
    hipError_t enqueue(int parity, hipStream_t s);  // parity < 0: by the members' counts
    void release_graph();

    std::vector<lbm3d_solver*> members_;
    int mode_ = 0, by_ = 8, tz_ = 8;
    bool stream_ = true;  // non-temporal stores (the members' levels exceed STREAM_MIN_BYTES)
    TilePlan plan_;
    void* dmem_ = nullptr;  // tables allocated by the plan (nullptr with a caller's buffer)
    size_t dbytes_ = 0;
    BatchSolve* dsolves_ = nullptr;
    BatchTile* dtiles_ = nullptr;
    BatchQueue* dqueue_ = nullptr;
    BatchLayerJob* dlayers_ = nullptr;  // boundary-layer jobs (sorted by first workgroup)
    int32_t* dblockjob_ = nullptr;      // job of each boundary-layer workgroup
    uint32_t* dhealth_ = nullptr;       // gathered health words, one per member
    BatchCount* dcount_ = nullptr;      // step counts of the members in the current run
    std::vector<BatchCount> hcount_;    // their host copy (source of the upload; done = parity since build)
    bool count_pending_ = false;        // hcount_ was uploaded and the stream not waited for since
    int nljobs_ = 0, nlblocks_ = 0;
    std::vector<uint32_t> ghost_rest_;  // per member: faces left to the boundary-layer launch
    hipGraphExec_t graph_ = nullptr;
    hipStream_t capture_stream_ = nullptr;
    hipStream_t last_stream_ = nullptr;  // stream of the last enqueued work (drained before teardown)
};

// Checks shared by the batched entry points (E_INVAL / E_STATE).
int32_t check_batch(lbm3d_t* hs, int32_t count);
// Advance members by their own step counts (one run of the largest count,
// the others sitting out its last launches), then wait for `s`.  Tables go
// into `dev` (cap bytes) when given; `graphs` = false launches every step
// directly.
int32_t batch_advance(lbm3d_t* hs, int32_t count, const int64_t* nsteps, hipStream_t s, BatchPlan& plan,
                      void* dev, size_t cap, bool graphs);

}  // namespace lbm3d
