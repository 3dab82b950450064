// Batched stepping of many solves with one launch per step (internal).
#pragma once

#include <vector>

#include "lbm3d_api_impl.h"

namespace lbm3d {

// A fixed set of solves (one precision) advanced together: a device table
// of the solves, a packed tile list over all of them and a persistent
// launch per step; runs of steps are replayed from a captured graph.
class BatchPlan {
public:
    BatchPlan() = default;
    ~BatchPlan();
    BatchPlan(const BatchPlan&) = delete;
    BatchPlan& operator=(const BatchPlan&) = delete;

    // (Re)build for `members` (all initialised, same precision); each
    // member's current buffer is taken as parity 0.  Enqueued on `s`.
    // `tz` > 0 sets the tile depth, else the tuned or default one is used.
    int32_t build(const std::vector<lbm3d_solver*>& members, hipStream_t s, int tz = 0);
    // One step of every member from the build-time buffers into the other
    // ones, without advancing anything (for timing: repeated launches
    // recompute the same next level).
    hipError_t launch_once(hipStream_t s);
    // Enqueue k steps of every member on `s` and update the members'
    // buffer parity and step counters.
    int32_t run(int64_t k, hipStream_t s);
    int ntiles() const { return ntiles_; }
    int by() const { return by_; }

private:
    hipError_t enqueue(int parity, hipStream_t s);
    void release_graph();

    std::vector<lbm3d_solver*> members_;
    int mode_ = 0, by_ = 8, tz_ = 8, ntiles_ = 0, nblocks_ = 0;
    void* dmem_ = nullptr;  // solve table + tile list
    size_t dbytes_ = 0;
    BatchSolve* dsolves_ = nullptr;
    BatchTile* dtiles_ = nullptr;
    BatchLayerJob* dlayers_ = nullptr;  // boundary-layer jobs (sorted by first workgroup)
    int32_t* dblockjob_ = nullptr;      // job of each boundary-layer workgroup
    int nljobs_ = 0, nlblocks_ = 0;
    std::vector<uint32_t> ghost_rest_;  // per member: faces left to the boundary-layer launch
    std::vector<int> cur0_;             // per member: current buffer at build()
    hipGraphExec_t graph_ = nullptr;
    hipStream_t capture_stream_ = nullptr;
    int parity_ = 0;  // parity of the next step relative to build()
};

}  // namespace lbm3d
