// Host-side solver object shared by the C ABI, the batched step and the
// server (internal).
#pragma once

#include "../../include/lbm3d.h"
#include "lbm3d_internal.h"

struct lbm3d_solver {
    lbm3d_params p{};
    int mode = 0;
    lbm3d::Grid g{};
    lbm3d::FaceBC bc{};
    lbm3d::TileCfg tile{};
    lbm3d::Model<double> md{};
    lbm3d::Model<float> mf{};
    int64_t n = 0;             // interior nodes
    size_t bytes = 0;          // device bytes held
    void* mem = nullptr;       // one allocation for everything below
    void* f[2] = {nullptr, nullptr};
    double* q5 = nullptr;      // 5 x n staging for init / moments
    double* partial = nullptr; // per-block totals
    double* out5 = nullptr;
    uint32_t* health = nullptr;
    int nred = 0;
    bool upwind2 = false;      // the second-order upwind variant (steps untiled)
    int cur = 0;               // buffer holding the current level
    int64_t steps = 0;
    bool initialised = false;
    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
    ~lbm3d_solver();
};

namespace lbm3d {

constexpr int GRAPH_STEPS = 32;  // steps per captured graph (even)

int32_t validate(const lbm3d_params* p);
Model<double> make_model(const lbm3d_params* p);
Model<float> model_to_float(const Model<double>& d);
Grid make_grid(const lbm3d_params* p);
size_t elem_size(int precision);
size_t f_bytes(const Grid& g, int precision);
size_t footprint_of(const lbm3d_params* p);
int32_t solver_create(const lbm3d_params* p, lbm3d_solver** out);
int32_t solver_enqueue_steps(lbm3d_solver* h, int64_t nsteps);
// Stability admission of an initial state (lbm3d_admit): E_UNSTABLE if the
// von Neumann analysis at the state's extremes exceeds 1 + STABILITY_TOL.
constexpr double STABILITY_TOL = 1e-3;
int32_t admission(const lbm3d_params* p, const double* rho, const double* ux, const double* uy, const double* uz,
                  const double* pr, double* worst);
// autotuner results (lbm3d_tune.cpp): the tuned tile of a solve shape, and
// the tuned batch tile depth of a precision (0 if not tuned)
bool cached_tile(int mode, const Grid& g, const FaceBC& bc, TileCfg* out);
int batch_tile_depth(int mode);

}  // namespace lbm3d
