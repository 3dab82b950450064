// Autotuner of the launch shapes: the fused step's tile (64 x BY x TZ) of a
// single solve and the tile depth of the batched step.  Each candidate is
// timed with HIP events on the solve's own data, launching the step from
// the current buffer into the other one again and again (the current level
// is never overwritten, so the state of the solves is unchanged), in three
// interleaved rounds; the shape with the fastest round is kept and
// remembered for later solves of the same shape.
#include "lbm3d_api_impl.h"
#include "lbm3d_batch.h"

#include <algorithm>
#include <array>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <vector>

namespace lbm3d {
namespace {

constexpr int TUNE_ROUNDS = 3;  // interleaved timing rounds per candidate

struct ShapeKey {
    std::array<int, 10> v;  // precision, nx, ny, nz, six boundary kinds
    bool operator<(const ShapeKey& o) const { return v < o.v; }
};

ShapeKey key_of(int mode, const Grid& g, const FaceBC& bc)
{
    ShapeKey k;
    k.v = {mode, g.nx, g.ny, g.nz, bc.kind[0], bc.kind[1], bc.kind[2], bc.kind[3], bc.kind[4], bc.kind[5]};
    return k;
}

std::mutex g_mu;
std::map<ShapeKey, TileCfg> g_tiles;  // tuned tile per solve shape
int g_batch_tz[3] = {0, 0, 0};        // tuned batch tile depth per precision (0: not tuned)

std::vector<TileCfg> tile_candidates(int mode, const Grid& g)
{
    std::vector<TileCfg> c;
    TileCfg u;
    u.by = 0;
    u.tz = 1;
    c.push_back(u);
    const int bys[3] = {2, 4, 8};
    const int tzs[5] = {8, 16, 32, 64, 128};
    for (int by : bys)
        for (int tz : tzs)
            for (bool stream : {true, false}) {
                TileCfg t;
                t.by = by;
                t.tz = tz;
                t.stream = stream;
                if (tz > 2 * std::max(g.nz, 1) && tz != tzs[0]) continue;  // deeper than the grid adds nothing
                if (tile_supported(mode, g, t)) c.push_back(t);
            }
    return c;
}

// ---- on-disk cache of the results ----
// Text file: a header "lbm3d-tune 2 <arch>" naming the device architecture
// the shapes were measured on, then one line per result:
//   tile <precision> <nx> <ny> <nz> <bc -x> <bc +x> <bc -y> <bc +y> <bc -z> <bc +z> <by> <tz> <stream>
//   batch <precision> <tz>
// (<stream>: 1 for non-temporal stores of the new level, 0 for plain ones.)

std::string device_arch()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "none";
    std::string a = prop.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

int32_t save_locked(const char* path)
{
    const std::string tmp = std::string(path) + ".tmp";
    FILE* fp = std::fopen(tmp.c_str(), "w");
    if (!fp) return LBM3D_E_INVAL;
    bool ok = std::fprintf(fp, "lbm3d-tune 2 %s\n", device_arch().c_str()) > 0;
    for (const auto& kv : g_tiles) {
        const auto& v = kv.first.v;
        ok = ok && std::fprintf(fp, "tile %d %d %d %d %d %d %d %d %d %d %d %d %d\n", v[0], v[1], v[2], v[3], v[4],
                                v[5], v[6], v[7], v[8], v[9], kv.second.by, kv.second.tz, kv.second.stream ? 1 : 0) > 0;
    }
    for (int m = 0; m < 3; m++)
        if (g_batch_tz[m] > 0) ok = ok && std::fprintf(fp, "batch %d %d\n", m, g_batch_tz[m]) > 0;
    ok = (std::fclose(fp) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return LBM3D_E_INVAL;
    }
    return LBM3D_OK;
}

int32_t load_locked(const char* path)
{
    FILE* fp = std::fopen(path, "r");
    if (!fp) return LBM3D_E_NOTFOUND;
    std::map<ShapeKey, TileCfg> tiles;
    int batch[3] = {0, 0, 0};
    char line[512], kind[16], arch[128];
    int version = 0;
    bool ok = std::fgets(line, sizeof line, fp) && std::sscanf(line, "lbm3d-tune %d %127s", &version, arch) == 2 &&
              version == 2 && device_arch() == arch;
    while (ok && std::fgets(line, sizeof line, fp)) {
        if (std::sscanf(line, "%15s", kind) != 1) continue;  // blank line
        if (!std::strcmp(kind, "tile")) {
            ShapeKey k;
            TileCfg t;
            int stream = -1;
            ok = std::sscanf(line, "tile %d %d %d %d %d %d %d %d %d %d %d %d %d", &k.v[0], &k.v[1], &k.v[2], &k.v[3],
                             &k.v[4], &k.v[5], &k.v[6], &k.v[7], &k.v[8], &k.v[9], &t.by, &t.tz, &stream) == 13;
            ok = ok && (stream == 0 || stream == 1);
            t.stream = stream == 1;
            ok = ok && k.v[0] >= 0 && k.v[0] <= 2 && k.v[1] >= 1 && k.v[2] >= 1 && k.v[3] >= 1;
            for (int f = 4; ok && f < 10; f++) ok = k.v[f] >= LBM3D_PERIODIC && k.v[f] <= LBM3D_REFLECT;
            ok = ok && (t.by == 0 || t.by == 2 || t.by == 4 || (t.by == 8 && k.v[0] != 0)) && t.tz >= 1 && t.tz <= 65535;
            if (ok) tiles[k] = t;
        } else if (!std::strcmp(kind, "batch")) {
            int m = -1, tz = 0;
            ok = std::sscanf(line, "batch %d %d", &m, &tz) == 2 && m >= 0 && m <= 2 && tz >= 1 && tz <= 65535;
            if (ok) batch[m] = tz;
        } else {
            ok = false;
        }
    }
    std::fclose(fp);
    if (!ok) return LBM3D_E_INVAL;  // nothing merged from a bad file
    for (const auto& kv : tiles) g_tiles[kv.first] = kv.second;
    for (int m = 0; m < 3; m++)
        if (batch[m] > 0) g_batch_tz[m] = batch[m];
    return LBM3D_OK;
}

// LBM3D_TUNE_CACHE: loaded once per process before the first lookup, saved
// after every tuning.
bool g_env_loaded = false;
const char* env_cache() { return std::getenv("LBM3D_TUNE_CACHE"); }
void env_load_locked()
{
    if (g_env_loaded) return;
    g_env_loaded = true;
    if (const char* p = env_cache()) (void)load_locked(p);
}

}  // namespace

bool cached_tile(int mode, const Grid& g, const FaceBC& bc, TileCfg* out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    env_load_locked();
    auto it = g_tiles.find(key_of(mode, g, bc));
    if (it == g_tiles.end()) return false;
    *out = it->second;
    return true;
}

int batch_tile_depth(int mode)
{
    std::lock_guard<std::mutex> lk(g_mu);
    env_load_locked();
    return (mode >= 0 && mode < 3) ? g_batch_tz[mode] : 0;
}

}  // namespace lbm3d

using namespace lbm3d;

static int32_t herr2(hipError_t e)
{
    return e == hipSuccess ? LBM3D_OK : (e == hipErrorOutOfMemory ? LBM3D_E_NOMEM : LBM3D_E_DEVICE);
}

extern "C" int32_t lbm3d_tune(lbm3d_t h, int32_t launches, int32_t* by, int32_t* tz)
{
    if (!h) return LBM3D_E_INVAL;
    if (!h->initialised) return LBM3D_E_STATE;
    if (launches <= 0) launches = 10;
    hipStream_t s = h->stream;
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return herr2(e);
    std::vector<TileCfg> cands;
    for (const TileCfg& t : tile_candidates(h->mode, h->g))
        if (!(h->upwind2 && t.by != 0)) cands.push_back(t);  // the variant runs untiled only
    // Trials are real steps: they alternate the two buffers and write the
    // candidate's boundary layers, as stepping does, so that each step reads
    // what the one before wrote (from HBM: the step's stores stream past the
    // caches).  Recomputing one level again and again would read it from the
    // memory-side cache and rate some shapes far too fast (64 x 4 x 32 at
    // 127 us against 200 us when stepping, on the 256x128x128 workload).  The
    // current level (its whole buffer) and the health word are saved first
    // and restored afterwards, so the solve's state is unchanged.  Without
    // device memory for the copy the trials recompute the current level.
    const size_t fb = f_bytes(h->g, h->mode);
    void* backup = nullptr;
    if (hipMalloc(&backup, fb) != hipSuccess) {
        (void)hipGetLastError();
        backup = nullptr;
    }
    uint32_t health0 = 0;
    if (backup) e = hipMemcpyAsync(backup, h->f[h->cur], fb, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&health0, h->health, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    int c = h->cur;  // buffer holding the trials' current level
    auto trial_step = [&](const TileCfg& t) {
        hipError_t r = launch_step(h->mode, h->g, h->bc, t, h->md, h->mf, h->p.inflow, h->f[c], h->f[c ^ 1],
                                   h->health, s, h->upwind2);
        if (!backup) return r;
        const uint32_t rest = ghost_faces(h->g, h->bc, t.by != 0);
        if (r == hipSuccess && rest)
            r = launch_ghosts(h->mode, h->g, h->bc, h->md, h->p.inflow, false, h->f[c ^ 1], s, rest);
        c ^= 1;
        return r;
    };
    // every candidate is timed in each of TUNE_ROUNDS interleaved rounds and
    // keeps its fastest round, so a slow moment of the device does not
    // decide between two close candidates
    std::vector<float> ms_best(cands.size(), -1.0f);
    for (int r = 0; r < TUNE_ROUNDS && e == hipSuccess; r++) {
        for (size_t k = 0; k < cands.size() && e == hipSuccess; k++) {
            // every layer of the trials' level in memory: the previous
            // candidate may have formed some in its tiles only
            e = launch_ghosts(h->mode, h->g, h->bc, h->md, h->p.inflow, true, h->f[c], s);
            for (int w = 0; w < (r == 0 ? 2 : 1) && e == hipSuccess; w++) e = trial_step(cands[k]);
            if (e == hipSuccess) e = hipEventRecord(h->ev0, s);
            for (int n = 0; n < launches && e == hipSuccess; n++) e = trial_step(cands[k]);
            if (e == hipSuccess) e = hipEventRecord(h->ev1, s);
            if (e == hipSuccess) e = hipEventSynchronize(h->ev1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, h->ev0, h->ev1);
            if (e == hipSuccess && (ms_best[k] < 0.0f || ms < ms_best[k])) ms_best[k] = ms;
        }
    }
    // restore the current level and the health word (also after an error)
    hipError_t e2 = hipSuccess;
    if (backup) e2 = hipMemcpyAsync(h->f[h->cur], backup, fb, hipMemcpyDeviceToDevice, s);
    if (e2 == hipSuccess) e2 = hipMemcpyAsync(h->health, &health0, sizeof(uint32_t), hipMemcpyHostToDevice, s);
    if (e2 == hipSuccess) e2 = hipStreamSynchronize(s);
    if (backup) (void)hipFree(backup);
    if (e != hipSuccess) return herr2(e);
    if (e2 != hipSuccess) return herr2(e2);
    TileCfg best = h->tile;
    float best_ms = -1.0f;
    for (size_t c = 0; c < cands.size(); c++)
        if (best_ms < 0.0f || ms_best[c] < best_ms) {
            best_ms = ms_best[c];
            best = cands[c];
        }
    int32_t rc = lbm3d_set_tile(h, best.by, best.tz);
    if (rc == LBM3D_OK) rc = lbm3d_set_streaming(h, best.stream ? 1 : 0);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        env_load_locked();
        g_tiles[key_of(h->mode, h->g, h->bc)] = best;
        if (const char* p = env_cache()) (void)save_locked(p);
    }
    if (by) *by = best.by;
    if (tz) *tz = best.tz;
    return LBM3D_OK;
}

extern "C" int32_t lbm3d_tune_save(const char* path)
{
    if (!path || !*path) return LBM3D_E_INVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    env_load_locked();
    return save_locked(path);
}

extern "C" int32_t lbm3d_tune_load(const char* path)
{
    if (!path || !*path) return LBM3D_E_INVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    env_load_locked();
    return load_locked(path);
}

extern "C" int32_t lbm3d_batch_set_depth(int32_t precision, int32_t tz)
{
    if (precision < LBM3D_FP64 || precision > LBM3D_FP32_T64 || tz < 0 || tz > 65535) return LBM3D_E_INVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    env_load_locked();
    g_batch_tz[precision] = tz;
    return LBM3D_OK;
}

extern "C" int32_t lbm3d_batch_tune(lbm3d_t* hs, int32_t count, int32_t launches, int32_t* tz)
{
    int32_t rc = check_batch(hs, count);
    if (rc) return rc;
    if (launches <= 0) launches = 5;
    hipStream_t s = hs[0]->stream;
    for (int32_t k = 0; k < count; k++)
        if (hipStreamSynchronize(hs[k]->stream) != hipSuccess) return LBM3D_E_DEVICE;
    std::vector<lbm3d_solver*> members(hs, hs + count);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    // chunk depths; a depth at or beyond a member's nz gives whole columns
    constexpr int NT = 4;
    const int tzs[NT] = {16, 32, 64, 128};
    BatchPlan plans[NT];
    for (int c = 0; c < NT; c++) {
        rc = plans[c].build(members, s, tzs[c]);
        if (rc) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return rc;
        }
    }
    // Trials are real steps over alternating buffers (see lbm3d_tune): the
    // members' current buffers and health words are saved first and
    // restored afterwards.  Without device memory for the copies the trials
    // recompute the current level.
    std::vector<size_t> off(count + 1, 0);
    for (int32_t k = 0; k < count; k++) off[k + 1] = off[k] + f_bytes(hs[k]->g, hs[k]->mode);
    char* backup = nullptr;
    if (e == hipSuccess && hipMalloc((void**)&backup, off[count]) != hipSuccess) {
        (void)hipGetLastError();
        backup = nullptr;
    }
    std::vector<uint32_t> health0(count, 0u);
    for (int32_t k = 0; k < count && e == hipSuccess; k++) {
        if (backup)
            e = hipMemcpyAsync(backup + off[k], hs[k]->f[hs[k]->cur], off[k + 1] - off[k], hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&health0[k], hs[k]->health, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    // interleaved rounds, each depth keeping its fastest (as for the tiles)
    float ms_best[NT] = {-1.0f, -1.0f, -1.0f, -1.0f};
    int parity = 0;  // buffers holding the trials' current level (the same for every plan)
    auto trial = [&](BatchPlan& p) {
        hipError_t r = p.launch_at(parity, s);
        if (backup) parity ^= 1;
        return r;
    };
    for (int r = 0; r < TUNE_ROUNDS && e == hipSuccess; r++) {
        for (int c = 0; c < NT && e == hipSuccess; c++) {
            for (int w = 0; w < (r == 0 ? 2 : 1) && e == hipSuccess; w++) e = trial(plans[c]);
            if (e == hipSuccess) e = hipEventRecord(e0, s);
            for (int k = 0; k < launches && e == hipSuccess; k++) e = trial(plans[c]);
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess && (ms_best[c] < 0.0f || ms < ms_best[c])) ms_best[c] = ms;
        }
    }
    // restore the members' current levels and health words (also after an error)
    hipError_t e2 = hipSuccess;
    for (int32_t k = 0; k < count && e2 == hipSuccess; k++) {
        if (backup)
            e2 = hipMemcpyAsync(hs[k]->f[hs[k]->cur], backup + off[k], off[k + 1] - off[k], hipMemcpyDeviceToDevice, s);
        if (e2 == hipSuccess)
            e2 = hipMemcpyAsync(hs[k]->health, &health0[k], sizeof(uint32_t), hipMemcpyHostToDevice, s);
    }
    if (e2 == hipSuccess) e2 = hipStreamSynchronize(s);
    if (backup) (void)hipFree(backup);
    if (e == hipSuccess) e = e2;
    int best_tz = 0;
    float best_ms = -1.0f;
    for (int c = 0; c < NT; c++)
        if (ms_best[c] >= 0.0f && (best_ms < 0.0f || ms_best[c] < best_ms)) {
            best_ms = ms_best[c];
            best_tz = tzs[c];
        }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return herr2(e);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        env_load_locked();
        g_batch_tz[hs[0]->mode] = best_tz;
        if (const char* p = env_cache()) (void)save_locked(p);
    }
    if (tz) *tz = best_tz;
    return LBM3D_OK;
}
