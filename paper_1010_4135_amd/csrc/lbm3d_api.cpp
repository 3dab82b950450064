// Host runtime and C ABI of the lbm3d library: parameter validation, device
// state, step loops replayed from captured HIP graphs, moments, totals,
// checkpoints.  The batched step and the server live in their own files.
#include "lbm3d_api_impl.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

using namespace lbm3d;

namespace lbm3d {

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int32_t validate(const lbm3d_params* p)
{
    if (!p) return LBM3D_E_INVAL;
    const int32_t n[3] = {p->nx, p->ny, p->nz};
    for (int a = 0; a < 3; a++) {
        if (n[a] < 1 || n[a] > (1 << 20)) return LBM3D_E_INVAL;
        const int lo = p->bc[2 * a], hi = p->bc[2 * a + 1];
        if (lo < LBM3D_PERIODIC || lo > LBM3D_REFLECT || hi < LBM3D_PERIODIC || hi > LBM3D_REFLECT)
            return LBM3D_E_INVAL;
        if ((lo == LBM3D_PERIODIC) != (hi == LBM3D_PERIODIC)) return LBM3D_E_INVAL;
        if (lo != LBM3D_PERIODIC && n[a] < 2) return LBM3D_E_INVAL;
    }
    if (p->nz > 65535) return LBM3D_E_INVAL;
    {
        // one velocity plane (with boundary layers and padding) must be
        // addressable with 32-bit element offsets
        const double plane = (double)(p->nx + 64 + NG) * (p->ny + 2 * NG) * (p->nz + 2 * NG);
        if (plane > 2.0e9) return LBM3D_E_INVAL;
    }
    if (!finite_pos(p->c1) || !finite_pos(p->c2) || !finite_pos(p->eta0)) return LBM3D_E_INVAL;
    if (p->c1 == p->c2) return LBM3D_E_INVAL;  // A_i and B_i divide by c1^2 - c2^2
    if (!std::isfinite(p->gamma) || !(p->gamma > 1.0)) return LBM3D_E_INVAL;
    if (!finite_pos(p->tau) || !finite_pos(p->dt) || !finite_pos(p->dx)) return LBM3D_E_INVAL;
    if (p->precision < LBM3D_FP64 || p->precision > LBM3D_FP32_T64) return LBM3D_E_INVAL;
    if (p->flags & ~(uint32_t)(LBM3D_NO_DISSIPATION | LBM3D_UPWIND2 | LBM3D_CHECK_STABILITY | LBM3D_VELOCITY_MAJOR))
        return LBM3D_E_INVAL;
    for (int face = 0; face < 6; face++) {
        if (p->bc[face] != LBM3D_INFLOW) continue;
        const double* s = p->inflow[face];
        if (!finite_pos(s[0]) || !finite_pos(s[4])) return LBM3D_E_INVAL;
        if (!std::isfinite(s[1]) || !std::isfinite(s[2]) || !std::isfinite(s[3])) return LBM3D_E_INVAL;
    }
    // explicit-step admission: Courant number of the diagonal velocities,
    // diffusion number of the rest particle, relaxation factor dt/tau
    const double cfl = std::sqrt(3.0) * p->c2 * p->dt / p->dx;
    const double dif = (p->flags & LBM3D_NO_DISSIPATION) ? 0.0 : 6.0 * p->c1 * p->dt / p->dx;
    if (cfl > 1.0 || dif > 1.0 || p->dt / p->tau > 2.0) return LBM3D_E_UNSTABLE;
    return LBM3D_OK;
}

Model<double> make_model(const lbm3d_params* p)
{
    Model<double> m;
    const double c1 = p->c1, c2 = p->c2, e0 = p->eta0;
    const double b = 2.0 / (p->gamma - 1.0);
    const double c1s = c1 * c1, c2s = c2 * c2, e0s = e0 * e0;
    m.c1 = c1;
    m.k = c2 / std::sqrt(3.0);
    m.c1sq = c1s;
    m.c2sq = c2s;
    m.e0sq = e0s;
    m.inv_b = 1.0 / b;
    // Eq. (e18): rest A_1 = (b-3) T / eta0^2
    m.r_aT = (b - 3.0) / e0s;
    // axis group i = 2..7
    const double ia = 1.0 / (6.0 * (c1s - c2s));
    m.x_a0 = -c2s * ia;
    m.x_aT = ((b - 3.0) * c2s / e0s + 3.0) * ia;
    m.x_au = c2s / c1s * ia;
    const double ib = 1.0 / (2.0 * c1s * (c1s - c2s));
    m.x_b0 = -c2s * ib;
    m.x_bT = (b + 2.0) * ib;
    m.x_bu = ib;
    m.x_d = 1.0 / (2.0 * c1s * c1s);
    // diagonal group i = 8..15
    const double da = 1.0 / (8.0 * (c2s - c1s));
    m.d_a0 = -c1s * da;
    m.d_aT = ((b - 3.0) * c1s / e0s + 3.0) * da;
    m.d_au = (3.0 * c1s - c2s) / (2.0 * c2s) * da;
    const double db = 3.0 / (8.0 * c2s * (c2s - c1s));
    m.d_b0 = -c1s * db;
    m.d_bT = (b + 2.0) * db;
    m.d_bu = db;
    m.d_d = 9.0 / (16.0 * c2s * c2s);
    // time-step factors; lambda_i of Eq. (lp): c1 dx (rest), c1 dx / 10 (axis), 0 (diagonal)
    m.k_adv = p->dt / p->dx;
    m.k_bgk = p->dt / p->tau;
    const bool diss = !(p->flags & LBM3D_NO_DISSIPATION);
    m.k_lap0 = diss ? c1 * p->dx * p->dt / (p->dx * p->dx) : 0.0;
    m.k_lap1 = diss ? c1 * p->dx / 10.0 * p->dt / (p->dx * p->dx) : 0.0;
    m.a1 = m.k_adv * m.c1;
    m.ad = m.k_adv * m.k;
    return m;
}

Model<float> model_to_float(const Model<double>& d)
{
    Model<float> f;
    const double* src = reinterpret_cast<const double*>(&d);
    float* dst = reinterpret_cast<float*>(&f);
    static_assert(sizeof(Model<double>) == 2 * sizeof(Model<float>), "model layout");
    for (size_t i = 0; i < sizeof(Model<float>) / sizeof(float); i++) dst[i] = (float)src[i];
    return f;
}


size_t footprint_of(const lbm3d_params* p)
{
    const Grid g = make_grid(p);
    const size_t n = (size_t)p->nx * p->ny * p->nz;
    return 2 * f_bytes(g, p->precision) + 5 * n * sizeof(double) + 1024 * 5 * sizeof(double) + 4096;
}

}  // namespace lbm3d

// ------------------------------------------------------------------ solver --
static int32_t dev_err(hipError_t e) { return e == hipSuccess ? LBM3D_OK : (e == hipErrorOutOfMemory ? LBM3D_E_NOMEM : LBM3D_E_DEVICE); }

#define HIPCHK(x)                                  \
    do {                                           \
        hipError_t _e = (x);                       \
        if (_e != hipSuccess) return dev_err(_e);  \
    } while (0)

lbm3d_solver::~lbm3d_solver()
{
    for (int k = 0; k < 2; k++)
        if (graph_exec[k]) (void)hipGraphExecDestroy(graph_exec[k]);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    if (own_stream) (void)hipStreamDestroy(own_stream);
    if (mem) (void)hipFree(mem);
}

namespace lbm3d {

int32_t solver_create(const lbm3d_params* p, lbm3d_solver** out)
{
    if (!out) return LBM3D_E_INVAL;
    *out = nullptr;
    int32_t rc = validate(p);
    if (rc) return rc;
    lbm3d_solver* h = new (std::nothrow) lbm3d_solver();
    if (!h) return LBM3D_E_NOMEM;
    h->p = *p;
    h->mode = p->precision;
    h->g = make_grid(p);
    h->md = make_model(p);
    h->mf = model_to_float(h->md);
    for (int f = 0; f < 6; f++) h->bc.kind[f] = p->bc[f];
    h->upwind2 = (p->flags & LBM3D_UPWIND2) != 0;
    h->tile = default_tile(h->mode, h->g);
    TileCfg tuned;
    if (cached_tile(h->mode, h->g, h->bc, &tuned) && tile_supported(h->mode, h->g, tuned)) h->tile = tuned;
    if (h->upwind2) {
        // the variant runs in the untiled kernel
        h->tile.by = 0;
        h->tile.tz = 1;
    }
    h->n = (int64_t)p->nx * p->ny * p->nz;
    const size_t fb = f_bytes(h->g, h->mode);
    h->nred = conserved_blocks(h->g);
    const size_t q5b = (size_t)5 * h->n * sizeof(double);
    const size_t redb = (size_t)h->nred * 5 * sizeof(double) + 8 * sizeof(double);
    h->bytes = 2 * fb + q5b + redb + 256;
    hipError_t e = hipMalloc(&h->mem, h->bytes);
    if (e != hipSuccess) {
        delete h;
        return dev_err(e);
    }
    char* base = (char*)h->mem;
    h->f[0] = base;
    h->f[1] = base + fb;
    h->q5 = (double*)(base + 2 * fb);
    h->partial = (double*)(base + 2 * fb + q5b);
    h->out5 = h->partial + (size_t)h->nred * 5;
    h->health = (uint32_t*)(h->out5 + 5);
    e = hipStreamCreateWithFlags(&h->own_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&h->ev0);
    if (e == hipSuccess) e = hipEventCreate(&h->ev1);
    // zero both buffers once so the unused padding never holds garbage
    if (e == hipSuccess) e = hipMemsetAsync(h->mem, 0, h->bytes, h->own_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->own_stream);
    if (e != hipSuccess) {
        delete h;
        return dev_err(e);
    }
    h->stream = h->own_stream;
    *out = h;
    return LBM3D_OK;
}

// One time step of a solve: fused update f[cur] -> f[cur^1], then the
// boundary layers of the new level.
static hipError_t enqueue_one(lbm3d_solver* h, int cur, hipStream_t s)
{
    hipError_t e = launch_step(h->mode, h->g, h->bc, h->tile, h->md, h->mf, h->p.inflow, h->f[cur], h->f[cur ^ 1],
                               h->health, s, h->upwind2);
    if (e != hipSuccess) return e;
    const uint32_t rest = ghost_faces(h->g, h->bc, h->tile.by != 0);
    if (!rest) return hipSuccess;
    return launch_ghosts(h->mode, h->g, h->bc, h->md, h->p.inflow, false, h->f[cur ^ 1], s, rest);
}

int32_t solver_enqueue_steps(lbm3d_solver* h, int64_t nsteps)
{
    hipStream_t s = h->stream;
    int64_t left = nsteps;
    // runs of GRAPH_STEPS steps are replayed from a graph captured once per
    // starting buffer (the step count is even, so the run ends where it began)
    while (left >= GRAPH_STEPS) {
        hipGraphExec_t& ge = h->graph_exec[h->cur];
        if (!ge) {
            hipGraph_t graph = nullptr;
            hipStream_t cs = h->own_stream;
            HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            hipError_t e = hipSuccess;
            int c = h->cur;
            for (int k = 0; k < GRAPH_STEPS && e == hipSuccess; k++) {
                e = enqueue_one(h, c, cs);
                c ^= 1;
            }
            hipError_t e2 = hipStreamEndCapture(cs, &graph);
            if (e != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return dev_err(e);
            }
            HIPCHK(e2);
            e = hipGraphInstantiate(&ge, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            HIPCHK(e);
        }
        HIPCHK(hipGraphLaunch(ge, s));
        left -= GRAPH_STEPS;
        h->steps += GRAPH_STEPS;
    }
    for (; left > 0; left--) {
        HIPCHK(enqueue_one(h, h->cur, s));
        h->cur ^= 1;
        h->steps++;
    }
    return LBM3D_OK;
}

}  // namespace lbm3d

// ------------------------------------------------------------------- C ABI --
extern "C" {

const char* lbm3d_version(void) { return "lbm3d 0.1 (gfx950)"; }

const char* lbm3d_strerror(int32_t code)
{
    switch (code) {
    case LBM3D_OK: return "ok";
    case LBM3D_E_INVAL: return "invalid argument";
    case LBM3D_E_UNSTABLE: return "explicit step not admitted (Courant, diffusion or relaxation number too large)";
    case LBM3D_E_NOMEM: return "out of memory or over budget";
    case LBM3D_E_DEVICE: return "HIP runtime error";
    case LBM3D_E_STATE: return "call out of order";
    case LBM3D_E_NONFINITE: return "solution is not finite";
    case LBM3D_E_NOTFOUND: return "unknown ticket";
    case LBM3D_E_CANCELLED: return "cancelled";
    default: return "unknown status";
    }
}

int32_t lbm3d_device_count(int32_t* count)
{
    if (!count) return LBM3D_E_INVAL;
    int c = 0;
    hipError_t e = hipGetDeviceCount(&c);
    *count = (e == hipSuccess) ? c : 0;
    return LBM3D_OK;
}

int32_t lbm3d_footprint(const lbm3d_params* p, size_t* bytes)
{
    if (!bytes) return LBM3D_E_INVAL;
    int32_t rc = validate(p);
    if (rc) return rc;
    *bytes = footprint_of(p);
    return LBM3D_OK;
}

int32_t lbm3d_create(const lbm3d_params* p, lbm3d_t* out) { return solver_create(p, out); }

int32_t lbm3d_destroy(lbm3d_t h)
{
    if (!h) return LBM3D_OK;
    (void)hipStreamSynchronize(h->stream);
    delete h;
    return LBM3D_OK;
}

int32_t lbm3d_set_stream(lbm3d_t h, void* hip_stream)
{
    if (!h) return LBM3D_E_INVAL;
    HIPCHK(hipStreamSynchronize(h->stream));
    h->stream = hip_stream ? (hipStream_t)hip_stream : h->own_stream;
    return LBM3D_OK;
}

int32_t lbm3d_init(lbm3d_t h, const double* rho, const double* ux, const double* uy, const double* uz,
                   const double* p)
{
    if (!h || !rho || !ux || !uy || !uz || !p) return LBM3D_E_INVAL;
    for (int64_t k = 0; k < h->n; k++) {
        if (!finite_pos(rho[k]) || !finite_pos(p[k])) return LBM3D_E_INVAL;
        if (!std::isfinite(ux[k]) || !std::isfinite(uy[k]) || !std::isfinite(uz[k])) return LBM3D_E_INVAL;
    }
    if (h->p.flags & LBM3D_CHECK_STABILITY) {
        const int32_t rc = admission(&h->p, rho, ux, uy, uz, p, nullptr);
        if (rc) return rc;
    }
    hipStream_t s = h->stream;
    const double* src[5] = {rho, ux, uy, uz, p};
    for (int c = 0; c < 5; c++)
        HIPCHK(hipMemcpyAsync(h->q5 + (size_t)c * h->n, src[c], (size_t)h->n * sizeof(double),
                              hipMemcpyHostToDevice, s));
    HIPCHK(launch_init(h->mode, h->g, h->md, h->q5, h->f[0], s));
    HIPCHK(launch_ghosts(h->mode, h->g, h->bc, h->md, h->p.inflow, true, h->f[0], s));
    // the fixed-state layers never change: write them into the other buffer too
    HIPCHK(launch_init(h->mode, h->g, h->md, h->q5, h->f[1], s));
    HIPCHK(launch_ghosts(h->mode, h->g, h->bc, h->md, h->p.inflow, true, h->f[1], s));
    HIPCHK(hipMemsetAsync(h->health, 0, sizeof(uint32_t), s));
    HIPCHK(hipStreamSynchronize(s));
    h->cur = 0;
    h->steps = 0;
    h->initialised = true;
    return LBM3D_OK;
}

int32_t lbm3d_step(lbm3d_t h, int64_t nsteps)
{
    if (!h || nsteps < 0) return LBM3D_E_INVAL;
    if (!h->initialised) return LBM3D_E_STATE;
    return solver_enqueue_steps(h, nsteps);
}

int32_t lbm3d_step_timed(lbm3d_t h, int64_t nsteps, double* ms)
{
    if (!h || nsteps < 0) return LBM3D_E_INVAL;
    if (!h->initialised) return LBM3D_E_STATE;
    HIPCHK(hipEventRecord(h->ev0, h->stream));
    int32_t rc = solver_enqueue_steps(h, nsteps);
    if (rc) return rc;
    HIPCHK(hipEventRecord(h->ev1, h->stream));
    HIPCHK(hipEventSynchronize(h->ev1));
    float t = 0.0f;
    HIPCHK(hipEventElapsedTime(&t, h->ev0, h->ev1));
    if (ms) *ms = (double)t;
    return LBM3D_OK;
}

int32_t lbm3d_step_profiled(lbm3d_t h, int64_t nsteps, double* total_ms, double* step_kernel_ms)
{
    if (!h || nsteps < 1) return LBM3D_E_INVAL;
    if (!h->initialised) return LBM3D_E_STATE;
    std::vector<hipEvent_t> ev((size_t)2 * nsteps, nullptr);
    hipError_t e = hipSuccess;
    for (auto& x : ev)
        if (e == hipSuccess) e = hipEventCreate(&x);
    hipStream_t s = h->stream;
    if (e == hipSuccess) e = hipEventRecord(h->ev0, s);
    for (int64_t k = 0; k < nsteps && e == hipSuccess; k++) {
        const int c = h->cur;
        // the step kernel's own dispatch records its start and end (no
        // markers of their own around it, whose overhead would count)
        e = launch_step(h->mode, h->g, h->bc, h->tile, h->md, h->mf, h->p.inflow, h->f[c], h->f[c ^ 1],
                        h->health, s, h->upwind2, ev[2 * k], ev[2 * k + 1]);
        const uint32_t rest = ghost_faces(h->g, h->bc, h->tile.by != 0);
        if (e == hipSuccess && rest)
            e = launch_ghosts(h->mode, h->g, h->bc, h->md, h->p.inflow, false, h->f[c ^ 1], s, rest);
        if (e == hipSuccess) {
            h->cur ^= 1;
            h->steps++;
        }
    }
    if (e == hipSuccess) e = hipEventRecord(h->ev1, s);
    if (e == hipSuccess) e = hipEventSynchronize(h->ev1);
    double ksum = 0.0;
    float t = 0.0f;
    for (int64_t k = 0; k < nsteps && e == hipSuccess; k++) {
        e = hipEventElapsedTime(&t, ev[2 * k], ev[2 * k + 1]);
        ksum += t;
    }
    if (e == hipSuccess) e = hipEventElapsedTime(&t, h->ev0, h->ev1);
    for (auto& x : ev)
        if (x) (void)hipEventDestroy(x);
    if (e != hipSuccess) return dev_err(e);
    if (total_ms) *total_ms = (double)t;
    if (step_kernel_ms) *step_kernel_ms = ksum / (double)nsteps;
    return LBM3D_OK;
}

// A new launch shape (or store kind) for the solve's next steps.
static int32_t set_launch(lbm3d_t h, const TileCfg& t)
{
    if (!tile_supported(h->mode, h->g, t) || (h->upwind2 && t.by != 0)) return LBM3D_E_INVAL;
    HIPCHK(hipStreamSynchronize(h->stream));
    for (int k = 0; k < 2; k++)
        if (h->graph_exec[k]) {
            (void)hipGraphExecDestroy(h->graph_exec[k]);
            h->graph_exec[k] = nullptr;
        }
    h->tile = t;
    // the layers a tiled step forms itself are not kept in memory: refresh
    // them all, so any launch shape can take over
    if (h->initialised) {
        HIPCHK(launch_ghosts(h->mode, h->g, h->bc, h->md, h->p.inflow, true, h->f[h->cur], h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
    }
    return LBM3D_OK;
}

int32_t lbm3d_set_tile(lbm3d_t h, int32_t by, int32_t tz)
{
    if (!h) return LBM3D_E_INVAL;
    TileCfg t = h->tile;  // (the store kind is kept)
    t.by = by;
    t.tz = tz;
    return set_launch(h, t);
}

int32_t lbm3d_set_streaming(lbm3d_t h, int32_t streaming)
{
    if (!h || (streaming != 0 && streaming != 1)) return LBM3D_E_INVAL;
    TileCfg t = h->tile;
    t.stream = streaming == 1;
    return set_launch(h, t);
}

int32_t lbm3d_get_streaming(lbm3d_t h, int32_t* streaming)
{
    if (!h || !streaming) return LBM3D_E_INVAL;
    *streaming = h->tile.stream ? 1 : 0;
    return LBM3D_OK;
}

int32_t lbm3d_get_tile(lbm3d_t h, int32_t* by, int32_t* tz)
{
    if (!h) return LBM3D_E_INVAL;
    if (by) *by = h->tile.by;
    if (tz) *tz = h->tile.tz;
    return LBM3D_OK;
}

int32_t lbm3d_sync(lbm3d_t h)
{
    if (!h) return LBM3D_E_INVAL;
    HIPCHK(hipStreamSynchronize(h->stream));
    return LBM3D_OK;
}

int32_t lbm3d_moments(lbm3d_t h, double* rho, double* ux, double* uy, double* uz, double* p)
{
    if (!h) return LBM3D_E_INVAL;
    if (!h->initialised) return LBM3D_E_STATE;
    hipStream_t s = h->stream;
    HIPCHK(launch_moments(h->mode, h->g, h->md, h->f[h->cur], h->q5, s));
    double* dst[5] = {rho, ux, uy, uz, p};
    for (int c = 0; c < 5; c++)
        if (dst[c])
            HIPCHK(hipMemcpyAsync(dst[c], h->q5 + (size_t)c * h->n, (size_t)h->n * sizeof(double),
                                  hipMemcpyDeviceToHost, s));
    uint32_t hw = 0;
    HIPCHK(hipMemcpyAsync(&hw, h->health, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return (hw & LBM3D_HEALTH_NONFINITE) ? LBM3D_E_NONFINITE : LBM3D_OK;
}

int32_t lbm3d_conserved(lbm3d_t h, double out[5])
{
    if (!h || !out) return LBM3D_E_INVAL;
    if (!h->initialised) return LBM3D_E_STATE;
    hipStream_t s = h->stream;
    HIPCHK(launch_conserved(h->mode, h->g, h->md, h->f[h->cur], h->partial, h->nred, h->out5, s));
    HIPCHK(hipMemcpyAsync(out, h->out5, 5 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return LBM3D_OK;
}

int32_t lbm3d_status(lbm3d_t h, uint32_t* health, int64_t* steps_done)
{
    if (!h) return LBM3D_E_INVAL;
    uint32_t hw = 0;
    HIPCHK(hipMemcpyAsync(&hw, h->health, sizeof(uint32_t), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (health) *health = hw;
    if (steps_done) *steps_done = h->steps;
    return LBM3D_OK;
}

int32_t lbm3d_poison_next(lbm3d_t h)
{
    if (!h) return LBM3D_E_INVAL;
    if (!h->initialised) return LBM3D_E_STATE;
    hipStream_t s = h->stream;
    // all ones is a quiet NaN in both float and double
    HIPCHK(hipMemsetAsync(h->f[h->cur ^ 1], 0xff, f_bytes(h->g, h->mode), s));
    // the fixed-state layers are written once per buffer (at init), not by
    // the steps: restore them
    HIPCHK(launch_ghosts(h->mode, h->g, h->bc, h->md, h->p.inflow, true, h->f[h->cur ^ 1], s, 0u));
    HIPCHK(hipStreamSynchronize(s));
    return LBM3D_OK;
}

int32_t lbm3d_get_f(lbm3d_t h, void* host, size_t bytes)
{
    if (!h || !host) return LBM3D_E_INVAL;
    if (!h->initialised) return LBM3D_E_STATE;
    const size_t need = (size_t)NV * h->n * elem_size(h->mode);
    if (bytes != need) return LBM3D_E_INVAL;
    void* dense = nullptr;
    HIPCHK(hipMalloc(&dense, need));
    hipStream_t s = h->stream;
    hipError_t e = launch_pack(h->mode, h->g, h->f[h->cur], dense, true, s);
    if (e == hipSuccess) e = hipMemcpyAsync(host, dense, need, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(dense);
    return dev_err(e);
}

int32_t lbm3d_set_f(lbm3d_t h, const void* host, size_t bytes)
{
    if (!h || !host) return LBM3D_E_INVAL;
    if (!h->initialised) return LBM3D_E_STATE;
    const size_t need = (size_t)NV * h->n * elem_size(h->mode);
    if (bytes != need) return LBM3D_E_INVAL;
    void* dense = nullptr;
    HIPCHK(hipMalloc(&dense, need));
    hipStream_t s = h->stream;
    hipError_t e = hipMemcpyAsync(dense, host, need, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_pack(h->mode, h->g, h->f[h->cur], dense, false, s);
    if (e == hipSuccess)
        e = launch_ghosts(h->mode, h->g, h->bc, h->md, h->p.inflow, true, h->f[h->cur], s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(dense);
    return dev_err(e);
}

}  // extern "C"
