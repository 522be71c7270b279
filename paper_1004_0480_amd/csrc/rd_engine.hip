// rd_engine.hip -- grids, models, plans, hipGraphs, batches and the C ABI.
//
// The host loop of the paper's Table 3 (allocate two arrays per species, load
// initial values, step with swaps, export, free) behind plain C calls; each
// step is one fused kernel (two for the Cahn-Hilliard model, section 4.1).
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "rd.h"
#define RD_DEFINE_ENGINE_KERNELS
#include "rd_fch_cfg.hpp"
#include "rd_tring_cfg.hpp"
#include "rd_batch_cfg.hpp"
#include "rd_internal.hpp"

using namespace rdk;

// ------------------------------------------------------------------ errors

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define RD_HIP(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(RD_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));     \
    } while (0)

size_t elem_size(int storage) { return storage == RD_F32 ? 4 : 2; }
int pitch_of(int64_t nx) { return int((nx + 63) / 64 * 64); }
size_t field_elems(int64_t nx, int64_t ny, int64_t nz) {
    return size_t(pitch_of(nx)) * size_t(ny) * size_t(nz) + SLACK;
}
bool is_finite(double v) { return std::isfinite(v); }

// Species of a single-field-group model split into passes that share no
// term, so that each pass carries few fields: the pollutant's coupled pair
// (transfer from the first to the second) is one pass, the remaining species
// another.  Every pass reads the old state only, so their order is free.
struct PassGroups {
    int n = 0;
    int first[2] = {0, 0}, count[2] = {0, 0}, pm[2] = {-1, -1};
};

PassGroups pass_groups(int model, int ns) {
    PassGroups p;
    auto add = [&](int first, int count, int pm) {
        p.first[p.n] = first;
        p.count[p.n] = count;
        p.pm[p.n] = pm;
        ++p.n;
    };
    switch (model) {
    case RD_MODEL_DIFFUSION: add(0, ns, PM_DIFF1 + (ns - 1)); break;
    case RD_MODEL_BRUSSELATOR: add(0, 2, PM_BRUSS); break;
    case RD_MODEL_POLLUTANT:
        add(0, ns >= 2 ? 2 : 1, ns >= 2 ? PM_POLL2 : PM_POLL1);
        if (ns >= 3) add(2, ns - 2, ns == 3 ? PM_POLL1 : PM_POLL2U);
        break;
    case RD_MODEL_TURING: add(0, 2, PM_TURING); break;
    case RD_MODEL_ATMOS:   // independent species, at most two per pass
        add(0, ns >= 2 ? 2 : 1, ns >= 2 ? PM_ATMOS2 : PM_ATMOS1);
        if (ns >= 3) add(2, ns - 2, ns == 3 ? PM_ATMOS1 : PM_ATMOS2);
        break;
    default: break;
    }
    return p;
}

// compute units of the current device (the first query is cached; the
// library runs on one device model at a time)
int num_cus() {
    static const int cus = [] {
        int dev = 0, n = 0;
        hipDeviceProp_t p;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess)
            n = p.multiProcessorCount;
        return n > 0 ? n : 256;
    }();
    return cus;
}

}  // namespace

namespace rdk {

int block_cfg_index(int vx, int ry, int w, int cz) {
    for (int i = 0; i < kNumBlockCfgs; ++i)
        if (kBlockCfgs[i].vx == vx && kBlockCfgs[i].ry == ry && kBlockCfgs[i].w == w && kBlockCfgs[i].cz == cz)
            return i;
    return -1;
}

int tile_cfg_index(int vx, int ry, int w, int pf) {
    for (int i = 0; i < kNumTileCfgs; ++i)
        if (kTileCfgs[i].vx == vx && kTileCfgs[i].ry == ry && kTileCfgs[i].w == w && kTileCfgs[i].pf == pf)
            return i;
    return -1;
}

int lds_cfg_index(int nch, int by, int wc, int d) {
    for (int i = 0; i < kNumLdsCfgs; ++i)
        if (kLdsCfgs[i].nch == nch && kLdsCfgs[i].by == by && kLdsCfgs[i].wc == wc && kLdsCfgs[i].d == d)
            return i;
    return -1;
}

int fch_cfg_index(int by, int wu, int wm, int d) {
    for (int i = 0; i < kNumFchCfgs; ++i)
        if (kFchCfgs[i].by == by && kFchCfgs[i].wu == wu && kFchCfgs[i].wm == wm && kFchCfgs[i].d == d) return i;
    return -1;
}

hipError_t launch_fch(int storage, int cfg, const StepArgs&, const StepArgs* d, long long blocks, hipStream_t s) {
    switch (storage) {
    case ST_F32: return launch_fch_f32(cfg, d, blocks, s);
    case ST_BF16: return launch_fch_bf16(cfg, d, blocks, s);
    case ST_F16: return launch_fch_f16(cfg, d, blocks, s);
    default: return hipErrorInvalidValue;
    }
}

int tr_cfg_index(int by, int wc, int d) {
    for (int i = 0; i < kNumTrCfgs; ++i)
        if (kTrCfgs[i].by == by && kTrCfgs[i].wc == wc && kTrCfgs[i].d == d) return i;
    return -1;
}

int lds2_cfg_index(int nch, int by, int wc, int d) {
    for (int i = 0; i < kNumLds2Cfgs; ++i)
        if (kLds2Cfgs[i].nch == nch && kLds2Cfgs[i].by == by && kLds2Cfgs[i].wc == wc && kLds2Cfgs[i].d == d)
            return i;
    return -1;
}

hipError_t launch_pass(int storage, int pm, int kernel, int cfg, const StepArgs& h, const StepArgs* d,
                       long long blocks, hipStream_t s) {
    // the model groups, one translation unit each per storage type
    const int grp = pm <= PM_DIFF4                       ? 0
                    : pm == PM_BRUSS || pm == PM_TURING  ? 1
                    : pm == PM_CHMU || pm == PM_FRONT    ? 2
                    : pm == PM_ATMOS1 || pm == PM_ATMOS2 ? 4
                                                         : 3;
#define RD_GROUPS(st)                                                        \
    switch (grp) {                                                           \
    case 0: return launch_pass_##st##_diff(pm, kernel, cfg, h, d, blocks, s);  \
    case 1: return launch_pass_##st##_react(pm, kernel, cfg, h, d, blocks, s); \
    case 2: return launch_pass_##st##_front(pm, kernel, cfg, h, d, blocks, s); \
    case 4: return launch_pass_##st##_atmos(pm, kernel, cfg, h, d, blocks, s); \
    default: return launch_pass_##st##_poll(pm, kernel, cfg, h, d, blocks, s); \
    }
    switch (storage) {
    case ST_F32: RD_GROUPS(f32)
    case ST_BF16: RD_GROUPS(bf16)
    case ST_F16: RD_GROUPS(f16)
    default: return hipErrorInvalidValue;
    }
#undef RD_GROUPS
}

hipError_t launch_batched(int storage, int* meta, const BatchEntry* ents, int step, int blocks,
                          hipStream_t s) {
    switch (storage) {
    case ST_F32: return launch_batched_f32(meta, ents, step, blocks, s);
    case ST_BF16: return launch_batched_bf16(meta, ents, step, blocks, s);
    case ST_F16: return launch_batched_f16(meta, ents, step, blocks, s);
    default: return hipErrorInvalidValue;
    }
}

int batched_blocks_per_cu(int storage) {
    switch (storage) {
    case ST_F32: return batched_blocks_per_cu_f32();
    case ST_BF16: return batched_blocks_per_cu_bf16();
    default: return batched_blocks_per_cu_f16();
    }
}

}  // namespace rdk

// ------------------------------------------------------------------- grids

struct rd_grid {
    int64_t nx = 0, ny = 0, nz = 0;
    int ns = 0;
    double h = 1.0;
    int storage = RD_F32;
    hipStream_t stream = nullptr;
    int pitch = 0;
    long long plane = 0;
    size_t elems = 0;
    void* buf[2][RD_MAX_SPECIES] = {};
    float* aux = nullptr;              // Cahn-Hilliard mu (FP32)
    int cur = 0;                       // buffer parity holding the current state
    bool has_model = false;
    int model = -1;
    float* d_wind = nullptr;
    int* d_src_row = nullptr;
    int* d_src_x = nullptr;
    int* d_src_sp = nullptr;
    float* d_src_rate = nullptr;
    StepClock* d_clock = nullptr;      // [parity]: step index and wind of that state
    int npass = 0;
    int pass_pm[2] = {-1, -1};
    StepArgs args[2][2];               // [input parity][pass], host copy
    StepArgs rk_args[2][2];            // Runge-Kutta stage 2 (see launch_rk_step)
    StepArgs rk3_args[2][2];           // Runge-Kutta stage 3 (order 3 only)
    StepArgs* d_args = nullptr;        // args, rk_args, rk3_args, in device memory
    int integrator = RD_EULER;
    int sr_mode = RD_ROUND_NEAREST;    // rounding of BF16 stores
    uint32_t sr_seed = 0;
    void* stage[RD_MAX_SPECIES] = {};  // order-3 Runge-Kutta stage buffers (allocated on demand)
    rd_plan plan{};                    // requested plan (kernel 0 = auto)
    rd_plan eff{};                     // plan in use
    int cfg = -1;
    long long blocks[2] = {0, 0};
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int gchunk = 0;
    double* d_part = nullptr;
    double* d_red = nullptr;
    rd_batch* batch = nullptr;
};

namespace {

constexpr int kRedBlocks = 1024;

void drop_graphs(rd_grid* g) {
    for (auto& e : g->gexec)
        if (e) {
            (void)hipGraphExecDestroy(e);
            e = nullptr;
        }
    g->gchunk = 0;
}

void free_model_arrays(rd_grid* g) {
    (void)hipFree(g->d_wind);
    (void)hipFree(g->d_src_row);
    (void)hipFree(g->d_src_x);
    (void)hipFree(g->d_src_sp);
    (void)hipFree(g->d_src_rate);
    g->d_wind = nullptr;
    g->d_src_row = g->d_src_x = g->d_src_sp = nullptr;
    g->d_src_rate = nullptr;
}

void fill_bc(StepArgs& a, int f, const rd_model_desc* m, int s) {
    int held = 0;
    for (int k = 0; k < 6; ++k) {
        a.bck[f][k] = m->bc_kind[s][k];
        a.bcv[f][k] = float(m->bc_value[s][k]);
        if (m->bc_kind[s][k] == RD_BC_HELD) held |= 1 << k;
    }
    a.held[f] = held;
}

void fill_mirror(StepArgs& a, int f) {
    for (int k = 0; k < 6; ++k) {
        a.bck[f][k] = BC_MIRROR;
        a.bcv[f][k] = 0.f;
    }
    a.held[f] = 0;
}

// Decomposition of a tiled plan: fills tiles_* / cz, returns workgroups.
long long set_tiling(StepArgs& a, const rd_plan& p) {
    // LDS ring: whole rows (vx cells per lane), ry rows per workgroup; the
    // one-pass front kernel: 128-cell x tiles, ry rows per workgroup
    const bool fch = p.kernel == RD_KERNEL_FUSED, tr = p.kernel == RD_KERNEL_TRING;
    const bool ring = p.kernel == RD_KERNEL_LDS || p.kernel == RD_KERNEL_LDS2 || fch || tr;
    const int tx = fch ? kFchTile : tr ? kTrTile : 64 * p.vx, by = ring ? p.ry : p.ry * p.waves;
    const int cz = (p.cz <= 0 || p.cz > a.nz) ? a.nz : p.cz;
    a.tiles_x = (a.nx + tx - 1) / tx;
    a.tiles_y = (a.ny + by - 1) / by;
    a.cz = cz;
    a.chunks_z = (a.nz + cz - 1) / cz;
    a.zfast = (p.kernel == RD_KERNEL_BLOCK || ring) && p.order == 1;
    return (long long)a.tiles_x * a.tiles_y * a.chunks_z;
}

// The single-step LDS ring takes rows of 256*(nch-1) < nx <= 256*nch cells,
// whole 16-byte lane loads: nx a multiple of 4 (FP32) or 8 (2-byte cells).
bool ring_row_fits(const rd_grid* g, int nch) {
    return g->nx <= 256 * nch && g->nx > 256 * (nch - 1) && g->nx % (g->storage == RD_F32 ? 4 : 8) == 0;
}

// Default plan: the plane-block kernel with the compiled slab shape that
// wastes the fewest lanes and rows (ties: wider rows, one row per wave,
// four-plane slabs, multi-wave workgroups).
int check_plan(const rd_grid* g, const rd_plan& p, int* cfg_out);

// z chunk length of a ring plan with `tiles` xy tiles and one workgroup per
// CU: the length that minimises whole rounds of workgroups times the planes a
// workgroup streams (its chunk plus about three halo planes).
int balanced_cz(const rd_grid* g, long long tiles) {
    int best = 0;
    double best_t = 1e300;
    for (int cz : {8, 16, 24, 32, 48, 64, 96, 128, 0}) {
        const int c = (cz <= 0 || cz >= g->nz) ? int(g->nz) : cz;
        const long long wg = tiles * ((g->nz + c - 1) / c);
        const double t = double((wg + num_cus() - 1) / num_cus()) * (c + 3);
        if (t < best_t) {
            best_t = t;
            best = c >= g->nz ? 0 : c;
        }
    }
    return best;
}

// z chunk length for k resident workgroups per CU: every chunk count n from
// 1 to 64 (chunks of ceil(nz/n) planes), scored by rounds x (planes + 3)
// where a round is k workgroups on every CU.  A workgroup count just below a
// multiple of k*CUs leaves no last round mostly idle.
int balanced_cz_k(const rd_grid* g, long long tiles, int k) {
    int best = 0;
    double best_t = 1e300;
    const long long slots = (long long)k * num_cus();
    for (int n = 1; n <= 64 && n <= g->nz; ++n) {
        const int c = int((g->nz + n - 1) / n);
        const long long wg = tiles * ((g->nz + c - 1) / c);
        const double t = double((wg + slots - 1) / slots) * (c + 3);
        if (t < best_t) {
            best_t = t;
            best = c >= g->nz ? 0 : c;
        }
    }
    return best;
}

rd_plan heuristic_plan(const rd_grid* g) {
    rd_plan best{};
    best.kernel = RD_KERNEL_DIRECT;
    if (g->model == RD_MODEL_FRONT_CH && !g->args[0][0].s19) {
        // the one-pass front kernel, its largest shape for this storage
        for (int i = 0; i < kNumFchCfgs; ++i) {
            if (!fch_ok(g->storage, i)) continue;
            rd_plan p{};
            p.kernel = RD_KERNEL_FUSED;
            p.vx = kFchCfgs[i].wm;
            p.ry = kFchCfgs[i].by;
            p.waves = kFchCfgs[i].wu;
            p.prefetch = kFchCfgs[i].d;
            const long long tiles = ((g->nx + kFchTile - 1) / kFchTile) * ((g->ny + p.ry - 1) / p.ry);
            p.cz = balanced_cz(g, tiles);
            int cfg = -1;
            if (check_plan(g, p, &cfg) == RD_OK) return p;
        }
    }
    if (g->args[0][0].s19) {
        // 19-point: the first LDS-ring shape this grid and model take, with
        // z chunks that give about two workgroups per CU; else direct
        for (int i = 0; i < kNumLdsCfgs; ++i) {
            const LdsCfg c = kLdsCfgs[i];
            bool ok = ring_row_fits(g, c.nch);
            for (int k = 0; k < g->npass; ++k) ok = ok && lds_ok(g->storage, g->pass_pm[k], i);
            if (!ok) continue;
            best.kernel = RD_KERNEL_LDS;
            best.vx = 4 * c.nch;
            best.ry = c.by;
            best.waves = c.wc;
            best.prefetch = c.d;
            const int yblocks = (g->ny + c.by - 1) / c.by;
            const int chunks = std::max(1, 2 * num_cus() / yblocks);
            const int cz = (g->nz + chunks - 1) / chunks;
            best.cz = cz < g->nz ? cz : 0;
            break;
        }
        return best;
    }
    double best_score = 1e30;
    unsigned mask = ~0u;
    for (int k = 0; k < g->npass; ++k) mask &= block_mask(g->storage, g->pass_pm[k]);
    for (int i = 0; i < kNumBlockCfgs; ++i) {
        if (!((mask >> i) & 1u)) continue;
        const BlockCfg c = kBlockCfgs[i];
        const int tx = 64 * c.vx, by = c.ry * c.w;
        const double wx = double((g->nx + tx - 1) / tx * tx) / double(g->nx);
        const double wy = double((g->ny + by - 1) / by * by) / double(g->ny);
        const double wz = double((g->nz + c.cz - 1) / c.cz * c.cz) / double(g->nz);
        double score = wx * wy * wz;
        score -= 1e-3 * c.vx;
        score += 1e-4 * std::abs(c.ry - 1);
        score += 1e-5 * std::abs(c.cz - 4);
        score += c.w == 1 ? 1e-2 : 0.0;
        if (score < best_score) {
            best_score = score;
            best.kernel = RD_KERNEL_BLOCK;
            best.vx = c.vx;
            best.ry = c.ry;
            best.waves = c.w;
            best.cz = c.cz;
            best.prefetch = 0;
        }
    }
    best.graph_chunk = 0;
    return best;
}

std::mutex g_tune_mu;
// autotuned plans by (nx, ny, nz, species, model, stencil and integrator, storage)
std::map<std::tuple<int64_t, int64_t, int64_t, int, int, int>, rd_plan> g_tune_cache;
int tune_model_key(const rd_grid* g) {
    return (g->model * 2 + (g->args[0][0].s19 ? 1 : 0)) * 4 + g->integrator;
}

int check_plan(const rd_grid* g, const rd_plan& p, int* cfg_out) {
    if (p.graph_chunk != 0 && (p.graph_chunk < 2 || (p.graph_chunk & 1)))
        return fail(RD_EINVAL, "graph_chunk must be 0 or an even number >= 2");
    if (g->integrator >= RD_RK2 && p.kernel == RD_KERNEL_LDS2)
        return fail(RD_EINVAL, "two-step plans take forward Euler only");
    if (g->args[0][0].s19 && p.kernel != RD_KERNEL_DIRECT && p.kernel != RD_KERNEL_LDS)
        return fail(RD_EINVAL, "the 19-point Laplacian runs on the direct and LDS-ring plans only");
    if (p.kernel == RD_KERNEL_DIRECT) {
        if (g->nz > 65535 || (g->ny + 3) / 4 > 65535)
            return fail(RD_EINVAL, "grid too large for the direct kernel's launch shape");
        *cfg_out = -1;
        return RD_OK;
    }
    if (p.order < 0 || p.order > 1) return fail(RD_EINVAL, "order must be 0 or 1");
    if (p.kernel == RD_KERNEL_BLOCK) {
        const int cfg = block_cfg_index(p.vx, p.ry, p.waves, p.cz);
        if (cfg < 0) return fail(RD_EINVAL, "slab shape not available");
        for (int k = 0; k < g->npass; ++k)
            if (!((block_mask(g->storage, g->pass_pm[k]) >> cfg) & 1u))
                return fail(RD_EINVAL, "slab shape not compiled for this model and storage");
        *cfg_out = cfg;
        return RD_OK;
    }
    if (p.kernel == RD_KERNEL_LDS) {
        const int cfg = (p.vx == 4 || p.vx == 8) ? lds_cfg_index(p.vx / 4, p.ry, p.waves, p.prefetch) : -1;
        if (cfg < 0) return fail(RD_EINVAL, "LDS ring shape not available");
        if (!ring_row_fits(g, p.vx / 4))
            return fail(RD_EINVAL,
                        "the LDS ring kernel needs 64*vx - 256 < nx <= 64*vx, nx a multiple of 4 (FP32) or 8 (BF16)");
        for (int k = 0; k < g->npass; ++k)
            if (!lds_ok(g->storage, g->pass_pm[k], cfg))
                return fail(RD_EINVAL, "LDS ring shape not compiled for this model and storage");
        if (p.cz < 0) return fail(RD_EINVAL, "cz must be >= 0");
        *cfg_out = cfg;
        return RD_OK;
    }
    if (p.kernel == RD_KERNEL_FUSED) {
        const int cfg = fch_cfg_index(p.ry, p.waves, p.vx, p.prefetch);
        if (cfg < 0) return fail(RD_EINVAL, "one-pass front shape not available");
        if (g->model != RD_MODEL_FRONT_CH || g->args[0][0].s19)
            return fail(RD_EINVAL, "the one-pass plan takes the 7-point front model only");
        if (!fch_ok(g->storage, cfg)) return fail(RD_EINVAL, "one-pass front shape not compiled for this storage");
        // the chemical potential one column beyond a 128-cell tile needs C
        // two columns on: a periodic x axis ending one cell into a tile would
        // wrap there
        if (g->args[0][1].bck[2][0] == BC_PERIODIC && g->nx > kFchTile && g->nx % kFchTile != 0)
            return fail(RD_EINVAL, "the one-pass plan needs nx <= 128 or a multiple of 128 for a periodic x axis of C");
        if (p.cz < 0) return fail(RD_EINVAL, "cz must be >= 0");
        *cfg_out = cfg;
        return RD_OK;
    }
    if (p.kernel == RD_KERNEL_TRING) {
        const int cfg = p.vx == 2 ? tr_cfg_index(p.ry, p.waves, p.prefetch) : -1;
        if (cfg < 0) return fail(RD_EINVAL, "tiled LDS ring shape not available (vx must be 2)");
        for (int k = 0; k < g->npass; ++k)
            if (!tr_ok(g->storage, g->pass_pm[k], cfg))
                return fail(RD_EINVAL, "tiled LDS ring shape not compiled for this model and storage");
        if (p.cz < 0) return fail(RD_EINVAL, "cz must be >= 0");
        *cfg_out = cfg;
        return RD_OK;
    }
    if (p.kernel == RD_KERNEL_LDS2) {
        const int cfg = (p.vx == 4 || p.vx == 8) ? lds2_cfg_index(p.vx / 4, p.ry, p.waves, p.prefetch) : -1;
        if (cfg < 0) return fail(RD_EINVAL, "two-step LDS ring shape not available");
        if (g->nx != 64 * p.vx) return fail(RD_EINVAL, "the LDS ring kernel needs rows of exactly 64*vx cells");
        if (g->npass != 1 || !lds2_ok(g->storage, g->pass_pm[0], cfg))
            return fail(RD_EINVAL, "two-step LDS ring shape not compiled for this model and storage");
        if (p.cz < 0) return fail(RD_EINVAL, "cz must be >= 0");
        *cfg_out = cfg;
        return RD_OK;
    }
    if (p.kernel != RD_KERNEL_TILED) return fail(RD_EINVAL, "unknown kernel kind");
    const int cfg = tile_cfg_index(p.vx, p.ry, p.waves, p.prefetch);
    if (cfg < 0) return fail(RD_EINVAL, "tile shape not available");
    for (int k = 0; k < g->npass; ++k)
        if (!((cfg_mask(g->storage, g->pass_pm[k]) >> cfg) & 1u))
            return fail(RD_EINVAL, "tile shape not compiled for this model and storage");
    if (p.cz < 0) return fail(RD_EINVAL, "cz must be >= 0");
    *cfg_out = cfg;
    return RD_OK;
}

// Resolve the plan in use, fill tiling into the argument copies, upload them.
int apply_plan(rd_grid* g) {
    rd_plan p = g->plan;
    int cfg = -1;
    if (p.kernel == RD_KERNEL_AUTO) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find({g->nx, g->ny, g->nz, g->ns, tune_model_key(g), g->storage});
        const int gc = p.graph_chunk;
        p = it != g_tune_cache.end() ? it->second : heuristic_plan(g);
        p.graph_chunk = gc;
        // a cached plan this grid cannot take (other settings since it was
        // tuned) gives way to the heuristic one
        if (check_plan(g, p, &cfg) != RD_OK) {
            p = heuristic_plan(g);
            p.graph_chunk = gc;
        }
    }
    int rc = check_plan(g, p, &cfg);
    if (rc) return rc;
    for (int par = 0; par < 2; ++par)
        for (int k = 0; k < g->npass; ++k) {
            StepArgs& a = g->args[par][k];
            if (p.kernel == RD_KERNEL_TILED || p.kernel == RD_KERNEL_BLOCK || p.kernel == RD_KERNEL_LDS ||
                p.kernel == RD_KERNEL_LDS2 || p.kernel == RD_KERNEL_FUSED || p.kernel == RD_KERNEL_TRING) {
                g->blocks[k] = set_tiling(a, p);
                (void)set_tiling(g->rk_args[par][k], p);
                (void)set_tiling(g->rk3_args[par][k], p);
            } else {
                g->blocks[k] = 0;
            }
        }
    for (int k = 0; k < g->npass; ++k)
        if (g->blocks[k] > 0x7fffffffLL)
            return fail(RD_EINVAL, "too many workgroups for this plan");
    g->eff = p;
    g->cfg = cfg;
    // the step's first launch advances the step clock: the chemical-potential
    // pass of the two-pass front step, or the one-pass kernel
    if (g->model == RD_MODEL_FRONT_CH)
        for (int par = 0; par < 2; ++par)
            for (auto* set : {&g->args, &g->rk_args, &g->rk3_args}) {
                (*set)[par][0].clk_pass = p.kernel == RD_KERNEL_FUSED ? 0 : 1;
                (*set)[par][1].clk_pass = p.kernel == RD_KERNEL_FUSED ? 1 : 0;
            }
    drop_graphs(g);
    RD_HIP(hipMemcpy(g->d_args, g->args, sizeof(g->args), hipMemcpyHostToDevice));
    RD_HIP(hipMemcpy(g->d_args + 4, g->rk_args, sizeof(g->rk_args), hipMemcpyHostToDevice));
    RD_HIP(hipMemcpy(g->d_args + 8, g->rk3_args, sizeof(g->rk3_args), hipMemcpyHostToDevice));
    return RD_OK;
}

// The one-pass front step: the update pass's arguments, one launch.
bool one_pass(const rd_grid* g) { return g->eff.kernel == RD_KERNEL_FUSED; }

int launch_one_step(rd_grid* g, int parity) {
    if (one_pass(g)) {
        const hipError_t e = launch_fch(g->storage, g->cfg, g->args[parity][1], g->d_args + parity * 2 + 1,
                                        g->blocks[1], g->stream);
        if (e != hipSuccess) return fail(RD_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
        return RD_OK;
    }
    for (int k = 0; k < g->npass; ++k) {
        const hipError_t e = launch_pass(g->storage, g->pass_pm[k], g->eff.kernel, g->cfg,
                                         g->args[parity][k], g->d_args + parity * 2 + k,
                                         g->blocks[k], g->stream);
        if (e != hipSuccess) return fail(RD_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    }
    return RD_OK;
}

// One set of step arguments (`set` 1: rk_args, 2: rk3_args) for the grid's
// passes.
int launch_set(rd_grid* g, int set, int parity) {
    const StepArgs(&h)[2][2] = set == 1 ? g->rk_args : g->rk3_args;
    if (one_pass(g)) {
        const hipError_t e = launch_fch(g->storage, g->cfg, h[parity][1], g->d_args + 4 * set + parity * 2 + 1,
                                        g->blocks[1], g->stream);
        if (e != hipSuccess) return fail(RD_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
        return RD_OK;
    }
    for (int k = 0; k < g->npass; ++k) {
        const hipError_t e = launch_pass(g->storage, g->pass_pm[k], g->eff.kernel, g->cfg, h[parity][k],
                                         g->d_args + 4 * set + parity * 2 + k, g->blocks[k], g->stream);
        if (e != hipSuccess) return fail(RD_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    }
    return RD_OK;
}

// One strong-stability-preserving Runge-Kutta step from Euler steps E, the
// combinations fused into the stages' stores (each stored value v becomes
// A + w (v - A), A the state at the same element).  The state stays in the
// current parity's buffers A; B is the other parity, C the stage buffers.
//   order 2:  B = E(A);  A = A + (E(B) - A)/2
//   order 3:  B = E(A);  C = A + (E(B) - A)/4;  A = A + 2 (E(C) - A)/3
int launch_rk_step(rd_grid* g) {
    const int p = g->cur;
    int rc = launch_one_step(g, p);
    if (!rc) rc = launch_set(g, 1, p);
    if (!rc && g->integrator == RD_RK3) rc = launch_set(g, 2, p);
    return rc;
}

int build_graph(rd_grid* g, int parity, int launches, hipGraphExec_t* out) {
    RD_HIP(hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal));
    int rc = RD_OK;
    for (int i = 0; i < launches && rc == RD_OK; ++i)
        rc = g->integrator >= RD_RK2 ? launch_rk_step(g) : launch_one_step(g, (parity + i) & 1);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(g->stream, &graph);
    if (rc != RD_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return fail(RD_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    const hipError_t ei = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return fail(RD_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
    return RD_OK;
}

// Time steps one launch of the plan advances.
int steps_per_launch(const rd_grid* g) { return g->eff.kernel == RD_KERNEL_LDS2 ? 2 : 1; }

// One step with the direct kernel (the odd step left over by a two-step plan).
int launch_direct_step(rd_grid* g, int parity) {
    for (int k = 0; k < g->npass; ++k) {
        const hipError_t e = launch_pass(g->storage, g->pass_pm[k], RD_KERNEL_DIRECT, -1, g->args[parity][k],
                                         g->d_args + parity * 2 + k, 0, g->stream);
        if (e != hipSuccess) return fail(RD_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    }
    return RD_OK;
}

int step_grid(rd_grid* g, int64_t n) {
    if (g->integrator >= RD_RK2) {
        // the state stays in the current parity: one graph of `chunk` steps
        const int chunk = g->eff.graph_chunk;
        if (chunk >= 2 && g->stream != nullptr && n >= chunk) {
            if (g->gchunk != chunk) {
                drop_graphs(g);
                const int rc = build_graph(g, g->cur, chunk, &g->gexec[g->cur]);
                if (rc) {
                    drop_graphs(g);
                    return rc;
                }
                g->gchunk = chunk;
            }
            for (; n >= chunk; n -= chunk) RD_HIP(hipGraphLaunch(g->gexec[g->cur], g->stream));
        }
        for (; n > 0; --n) {
            const int rc = launch_rk_step(g);
            if (rc) return rc;
        }
        return RD_OK;
    }
    const int chunk = g->eff.graph_chunk;          // steps per graph (even)
    const int sp = steps_per_launch(g);
    const int launches = chunk / sp;               // launches per graph
    if (chunk >= 2 && g->stream != nullptr && n >= chunk) {
        if (g->gchunk != chunk) {
            drop_graphs(g);
            for (int par = 0; par < 2; ++par) {
                const int rc = build_graph(g, par, launches, &g->gexec[par]);
                if (rc) {
                    drop_graphs(g);
                    return rc;
                }
            }
            g->gchunk = chunk;
        }
        while (n >= chunk) {
            RD_HIP(hipGraphLaunch(g->gexec[g->cur], g->stream));
            g->cur ^= launches & 1;
            n -= chunk;
        }
    }
    for (; n >= sp; n -= sp) {
        const int rc = launch_one_step(g, g->cur);
        if (rc) return rc;
        g->cur ^= 1;
    }
    if (n > 0) {
        const int rc = launch_direct_step(g, g->cur);
        if (rc) return rc;
        g->cur ^= 1;
    }
    return RD_OK;
}

}  // namespace

// ----------------------------------------------------------- validation

extern "C" size_t rd_grid_bytes(int64_t nx, int64_t ny, int64_t nz, int32_t nspecies,
                                int32_t storage_dtype, int32_t with_aux) {
    if (nx < 1 || ny < 1 || nz < 1 || nspecies < 1 || nspecies > RD_MAX_SPECIES) return 0;
    if (storage_dtype != RD_F32 && storage_dtype != RD_BF16 && storage_dtype != RD_F16) return 0;
    const size_t e = field_elems(nx, ny, nz);
    size_t b = 2 * size_t(nspecies) * e * elem_size(storage_dtype);
    if (with_aux) b += e * sizeof(float);
    b += 12 * sizeof(StepArgs) + 2 * sizeof(StepClock) + 2 * kRedBlocks * sizeof(double) + 2 * sizeof(double);
    return b;
}

extern "C" int rd_validate_model(int64_t nx, int64_t ny, int64_t nz, int32_t ns, double h,
                                 const rd_model_desc* m) {
    if (!m) return fail(RD_EINVAL, "model descriptor is NULL");
    if (nx < 1 || ny < 1 || nz < 1) return fail(RD_EINVAL, "grid extents must be >= 1");
    if (!(h > 0.0) || !is_finite(h)) return fail(RD_EINVAL, "h must be a positive finite number");
    if (m->nspecies != ns) return fail(RD_EINVAL, "model nspecies differs from the grid's");
    switch (m->model) {
    case RD_MODEL_DIFFUSION:
    case RD_MODEL_POLLUTANT:
        if (ns < 1 || ns > RD_MAX_SPECIES) return fail(RD_EINVAL, "nspecies must be 1..4");
        break;
    case RD_MODEL_BRUSSELATOR:
        if (ns != 2) return fail(RD_EINVAL, "the Brusselator has 2 species");
        break;
    case RD_MODEL_FRONT_CH:
        if (ns != 3) return fail(RD_EINVAL, "the front model has 3 species");
        break;
    case RD_MODEL_TURING:
        if (ns != 2) return fail(RD_EINVAL, "the Turing model has 2 species");
        break;
    case RD_MODEL_ATMOS:
        if (ns < 1 || ns > RD_MAX_SPECIES) return fail(RD_EINVAL, "nspecies must be 1..4");
        break;
    default: return fail(RD_EINVAL, "unknown model");
    }
    if (!(m->dt > 0.0) || !is_finite(m->dt)) return fail(RD_EINVAL, "dt must be a positive finite number");
    for (double p : m->param)
        if (!is_finite(p)) return fail(RD_EINVAL, "model parameters must be finite");
    for (int s = 0; s < ns; ++s) {
        for (int d = 0; d < 3; ++d)
            if (!(m->diff[s][d] >= 0.0) || !is_finite(m->diff[s][d]))
                return fail(RD_EINVAL, "diffusion coefficients must be finite and >= 0");
        for (int f = 0; f < 6; ++f) {
            if (m->bc_kind[s][f] < RD_BC_MIRROR || m->bc_kind[s][f] > RD_BC_HELD)
                return fail(RD_EINVAL, "unknown boundary kind");
            if (!is_finite(m->bc_value[s][f])) return fail(RD_EINVAL, "boundary values must be finite");
        }
        for (int a = 0; a < 3; ++a)
            if ((m->bc_kind[s][2 * a] == RD_BC_PERIODIC) != (m->bc_kind[s][2 * a + 1] == RD_BC_PERIODIC))
                return fail(RD_EINVAL, "a periodic axis needs periodic on both faces");
    }
    double umax = 0.0;   // largest sum over axes of |u_d|
    if (m->model == RD_MODEL_ATMOS) {
        if (m->param[3] < 0.0) return fail(RD_EINVAL, "the period of the vertical wind must be >= 0");
        umax = std::fabs(m->param[0]) + std::fabs(m->param[1]) + std::fabs(m->param[2]);
    }
    if (m->model == RD_MODEL_POLLUTANT) {
        if (!m->wind || m->nwind != nz) return fail(RD_EINVAL, "pollutant model needs nz wind values");
        for (int64_t k = 0; k < nz; ++k) {
            if (!(m->wind[k] >= 0.0) || !is_finite(m->wind[k]))
                return fail(RD_EINVAL, "wind speeds must be finite and >= 0 (upwind along +x)");
            umax = std::max(umax, m->wind[k]);
        }
        if (m->param[0] < 0.0 || m->param[1] < 0.0) return fail(RD_EINVAL, "decay and k_AB must be >= 0");
    }
    if (m->model == RD_MODEL_POLLUTANT || m->model == RD_MODEL_ATMOS) {
        if (m->nsrc < 0 || (m->nsrc > 0 && (!m->src_cell || !m->src_species || !m->src_rate)))
            return fail(RD_EINVAL, "bad source arrays");
        const int64_t N = nx * ny * nz;
        for (int64_t q = 0; q < m->nsrc; ++q) {
            if (m->src_cell[q] < 0 || m->src_cell[q] >= N) return fail(RD_EINVAL, "source cell out of range");
            if (m->src_species[q] < 0 || m->src_species[q] >= ns)
                return fail(RD_EINVAL, "source species out of range");
            if (!is_finite(m->src_rate[q])) return fail(RD_EINVAL, "source rates must be finite");
        }
    } else if (m->nsrc != 0) {
        return fail(RD_EINVAL, "point sources need the pollutant or atmospheric model");
    }
    if (m->stencil != 0 && m->stencil != 7 && m->stencil != 19) return fail(RD_EINVAL, "stencil must be 7 or 19");
    if (m->integrator < 0 || m->integrator > RD_RK3) return fail(RD_EINVAL, "unknown integrator");
    if (m->integrator >= RD_RK2 && m->model == RD_MODEL_ATMOS)
        return fail(RD_EINVAL, "Runge-Kutta steps take models without a time-dependent term");
    const bool s19 = m->stencil == 19;
    if (s19)
        for (int s = 0; s < ns; ++s)
            if (m->diff[s][1] != m->diff[s][0] || m->diff[s][2] != m->diff[s][0])
                return fail(RD_EINVAL, "the 19-point Laplacian needs isotropic diffusion coefficients");
    // Explicit stability: monotone bound (non-negative centre weight) of the
    // stencil plus upwind; 19-point centre weight 24/(6h^2) = 4/h^2.
    const double h2 = h * h;
    for (int s = 0; s < ns; ++s) {
        const double k = (s19 ? 4.0 * m->diff[s][0] : 2.0 * (m->diff[s][0] + m->diff[s][1] + m->diff[s][2])) / h2 +
                         umax / h;
        if (m->dt * k > 1.0 + 1e-12)
            return fail(RD_EUNSTABLE, s19 ? "dt exceeds the explicit bound dt*(4*D/h^2 + umax/h) <= 1"
                                          : "dt exceeds the explicit bound dt*(2*sum(K)/h^2 + umax/h) <= 1");
    }
    if (m->model == RD_MODEL_FRONT_CH) {
        const double M = m->param[1], kappa = m->param[2], eps = m->param[3];
        if (M < 0.0 || kappa < 0.0) return fail(RD_EINVAL, "M and kappa must be >= 0");
        if (m->param[5] < 0.0) return fail(RD_EINVAL, "k2 must be >= 0");
        // largest magnitude of the discrete Laplacian: 7-point 12/h^2, 19-point 32/(6h^2)
        const double lam = s19 ? 16.0 / (3.0 * h2) : 12.0 / h2;
        if (m->dt * M * (kappa * lam * lam + std::fabs(eps) * lam) > 1.0 + 1e-12)
            return fail(RD_EUNSTABLE, "dt exceeds the Cahn-Hilliard bound dt*M*(kappa*L^2 + |eps|*L) <= 1");
    }
    return RD_OK;
}

// ------------------------------------------------------------------ C ABI

extern "C" const char* rd_last_error(void) { return g_err.c_str(); }
extern "C" int rd_abi_version(void) { return RD_ABI_VERSION; }

#ifndef RD_SOURCE_DIGEST
#define RD_SOURCE_DIGEST "unknown"
#endif
extern "C" const char* rd_source_digest(void) { return RD_SOURCE_DIGEST; }

extern "C" int rd_create_grid(int64_t nx, int64_t ny, int64_t nz, int32_t nspecies, double h,
                              int32_t storage_dtype, void* hip_stream, rd_grid** out) {
    if (!out) return fail(RD_EINVAL, "out is NULL");
    *out = nullptr;
    if (nx < 1 || ny < 1 || nz < 1) return fail(RD_EINVAL, "grid extents must be >= 1");
    if (nx > (1 << 24) || ny > (1 << 24) || nz > (1 << 24)) return fail(RD_EINVAL, "grid extent too large");
    if ((__int128)pitch_of(nx) * ny * nz > (__int128)1 << 40) return fail(RD_EINVAL, "grid too large");
    if (nspecies < 1 || nspecies > RD_MAX_SPECIES) return fail(RD_EINVAL, "nspecies must be 1..4");
    if (!(h > 0.0) || !is_finite(h)) return fail(RD_EINVAL, "h must be a positive finite number");
    if (storage_dtype != RD_F32 && storage_dtype != RD_BF16 && storage_dtype != RD_F16)
        return fail(RD_EINVAL, "storage dtype must be RD_F32, RD_BF16 or RD_F16");
    rd_grid* g = new rd_grid();
    g->nx = nx;
    g->ny = ny;
    g->nz = nz;
    g->ns = nspecies;
    g->h = h;
    g->storage = storage_dtype;
    g->stream = static_cast<hipStream_t>(hip_stream);
    g->pitch = pitch_of(nx);
    g->plane = (long long)g->pitch * ny;
    g->elems = field_elems(nx, ny, nz);
    const size_t bytes = g->elems * elem_size(storage_dtype);
    auto cleanup = [&](int code, const std::string& msg) {
        rd_destroy_grid(g);
        return fail(code, msg);
    };
    for (int p = 0; p < 2; ++p)
        for (int s = 0; s < nspecies; ++s) {
            const hipError_t e = hipMalloc(&g->buf[p][s], bytes);
            if (e != hipSuccess) {
                g->buf[p][s] = nullptr;
                return cleanup(e == hipErrorOutOfMemory ? RD_ENOMEM : RD_EDEVICE,
                               std::string("hipMalloc: ") + hipGetErrorString(e));
            }
            if (hipMemsetAsync(g->buf[p][s], 0, bytes, g->stream) != hipSuccess)
                return cleanup(RD_EDEVICE, "hipMemsetAsync failed");
        }
    if (hipMalloc(&g->d_args, sizeof(g->args) + sizeof(g->rk_args) + sizeof(g->rk3_args)) != hipSuccess ||
        hipMalloc(&g->d_clock, 2 * sizeof(StepClock)) != hipSuccess ||
        hipMalloc(&g->d_part, 2 * kRedBlocks * sizeof(double)) != hipSuccess ||
        hipMalloc(&g->d_red, 2 * sizeof(double)) != hipSuccess)
        return cleanup(RD_ENOMEM, "hipMalloc of grid work buffers failed");
    if (hipStreamSynchronize(g->stream) != hipSuccess) return cleanup(RD_EDEVICE, "stream sync failed");
    std::memset(g->args, 0, sizeof(g->args));
    *out = g;
    return RD_OK;
}

extern "C" int rd_destroy_grid(rd_grid* g) {
    if (!g) return fail(RD_EINVAL, "grid is NULL");
    if (g->batch) rd_batch_remove(g->batch, g);
    (void)hipStreamSynchronize(g->stream);
    drop_graphs(g);
    for (auto& row : g->buf)
        for (auto& b : row) (void)hipFree(b);
    for (auto& b : g->stage) (void)hipFree(b);
    (void)hipFree(g->aux);
    (void)hipFree(g->d_args);
    (void)hipFree(g->d_clock);
    (void)hipFree(g->d_part);
    (void)hipFree(g->d_red);
    free_model_arrays(g);
    delete g;
    return RD_OK;
}

extern "C" int rd_set_model(rd_grid* g, const rd_model_desc* m) {
    if (!g) return fail(RD_EINVAL, "grid is NULL");
    if (g->batch) return fail(RD_ESTATE, "grid is in a batch");
    int rc = rd_validate_model(g->nx, g->ny, g->nz, g->ns, g->h, m);
    if (rc) return rc;
    if (g->sr_mode == RD_ROUND_STOCHASTIC && m->integrator >= RD_RK2)
        return fail(RD_EINVAL, "stochastic rounding takes forward Euler steps");
    RD_HIP(hipStreamSynchronize(g->stream));
    drop_graphs(g);
    free_model_arrays(g);
    g->has_model = false;
    const double ih2 = 1.0 / (g->h * g->h);
    const int ns = g->ns;

    // Pollutant wind and the sources of both source models (sorted by row,
    // duplicates merged in FP64).
    if (m->model == RD_MODEL_POLLUTANT || m->model == RD_MODEL_ATMOS) {
        std::vector<float> wh(g->nz, 0.f);
        if (m->model == RD_MODEL_POLLUTANT)
            for (int64_t k = 0; k < g->nz; ++k) wh[k] = float(m->wind[k] / g->h);
        std::map<std::tuple<int64_t, int64_t, int>, double> merged;   // (row, x, species)
        for (int64_t q = 0; q < m->nsrc; ++q) {
            const int64_t c = m->src_cell[q];
            merged[{c / g->nx, c % g->nx, m->src_species[q]}] += m->src_rate[q];
        }
        const int64_t rows = g->ny * g->nz;
        std::vector<int> row_start(rows + 1, 0), xs, sps;
        std::vector<float> rates;
        for (auto& kv : merged) row_start[std::get<0>(kv.first) + 1]++;
        for (int64_t r = 0; r < rows; ++r) row_start[r + 1] += row_start[r];
        for (auto& kv : merged) {
            xs.push_back(int(std::get<1>(kv.first)));
            sps.push_back(std::get<2>(kv.first));
            rates.push_back(float(kv.second));
        }
        const size_t n = std::max<size_t>(xs.size(), 1);
        xs.resize(n, -1);
        sps.resize(n, 0);
        rates.resize(n, 0.f);
        RD_HIP(hipMalloc(&g->d_wind, wh.size() * sizeof(float)));
        RD_HIP(hipMalloc(&g->d_src_row, row_start.size() * sizeof(int)));
        RD_HIP(hipMalloc(&g->d_src_x, n * sizeof(int)));
        RD_HIP(hipMalloc(&g->d_src_sp, n * sizeof(int)));
        RD_HIP(hipMalloc(&g->d_src_rate, n * sizeof(float)));
        RD_HIP(hipMemcpy(g->d_wind, wh.data(), wh.size() * sizeof(float), hipMemcpyHostToDevice));
        RD_HIP(hipMemcpy(g->d_src_row, row_start.data(), row_start.size() * sizeof(int), hipMemcpyHostToDevice));
        RD_HIP(hipMemcpy(g->d_src_x, xs.data(), n * sizeof(int), hipMemcpyHostToDevice));
        RD_HIP(hipMemcpy(g->d_src_sp, sps.data(), n * sizeof(int), hipMemcpyHostToDevice));
        RD_HIP(hipMemcpy(g->d_src_rate, rates.data(), n * sizeof(float), hipMemcpyHostToDevice));
    }
    if (m->model == RD_MODEL_FRONT_CH && !g->aux) {
        RD_HIP(hipMalloc(&g->aux, g->elems * sizeof(float)));
        RD_HIP(hipMemset(g->aux, 0, g->elems * sizeof(float)));
    }
    // The clock starts at step 0 in both parities (the state now held is
    // step 0 whichever buffer holds it).
    {
        StepClock c0[2] = {};
        if (m->model == RD_MODEL_ATMOS) {
            const double t0 = m->param[4];
            const double u = m->param[3] != 0.0 ? m->param[2] * std::sin(t0 / m->param[3]) : m->param[2];
            c0[0].uzh = c0[1].uzh = float(u * (1.0 / g->h));
        }
        RD_HIP(hipMemcpy(g->d_clock, c0, sizeof(c0), hipMemcpyHostToDevice));
    }

    const PassGroups groups = pass_groups(m->model, ns);
    // 19-point form: the kernels take K/(6h^2) as their coefficient
    const bool s19 = m->stencil == 19;
    const double lap_scale = s19 ? 1.0 / 6.0 : 1.0;
    for (int par = 0; par < 2; ++par) {
        for (int k = 0; k < 2; ++k) {
            StepArgs& a = g->args[par][k];
            std::memset(&a, 0, sizeof(a));
            a.s19 = s19 ? 1 : 0;
            a.nx = int(g->nx);
            a.ny = int(g->ny);
            a.nz = int(g->nz);
            a.pitch = g->pitch;
            a.plane = g->plane;
            a.dt = float(m->dt);
            a.wind_h = g->d_wind;
            a.src_row = g->d_src_row;
            a.src_x = g->d_src_x;
            a.src_sp = g->d_src_sp;
            a.src_rate = g->d_src_rate;
            a.clk_in = g->d_clock + par;
            a.clk_out = g->d_clock + (par ^ 1);
            a.clk_pass = k == 0 ? 1 : 0;
            if (m->model == RD_MODEL_ATMOS) {
                a.t0 = m->param[4];
                a.dt64 = m->dt;
                a.wamp = m->param[2];
                a.wper = m->param[3];
                a.inv_h = 1.0 / g->h;
            }
        }
        if (m->model == RD_MODEL_FRONT_CH) {
            // pass 0: mu of C with C's faces; pass 1: update A, B, C.
            StepArgs& a0 = g->args[par][0];
            a0.in[0] = g->buf[par][2];
            a0.out[0] = g->aux;
            a0.kx[0] = a0.ky[0] = a0.kz[0] = float(ih2 * lap_scale);
            fill_bc(a0, 0, m, 2);
            a0.out_held[0] = 0;
            StepArgs& a1 = g->args[par][1];
            for (int s = 0; s < 3; ++s) {
                a1.in[s] = g->buf[par][s];
                a1.out[s] = g->buf[par ^ 1][s];
                a1.kx[s] = float(m->diff[s][0] * ih2 * lap_scale);
                a1.ky[s] = float(m->diff[s][1] * ih2 * lap_scale);
                a1.kz[s] = float(m->diff[s][2] * ih2 * lap_scale);
                fill_bc(a1, s, m, s);
                a1.out_held[s] = a1.held[s];
            }
            a1.in[3] = g->aux;
            a1.kx[3] = a1.ky[3] = a1.kz[3] = float(ih2 * lap_scale);
            fill_mirror(a1, 3);
            for (int k = 0; k < 2; ++k) {
                StepArgs& a = g->args[par][k];
                a.p[0] = float(m->param[0]);   // k
                a.p[1] = float(m->param[1]);   // M
                a.p[2] = float(m->param[2]);   // kappa
                a.p[3] = float(m->param[3]);   // eps
                a.p[4] = float(m->param[4]);   // gamma
                a.p[5] = float(m->param[5]);   // k2
            }
        } else {
            // one pass per group of species that share a term (see pass_groups)
            for (int k = 0; k < groups.n; ++k) {
                StepArgs& a = g->args[par][k];
                const int s0 = groups.first[k];
                for (int f = 0; f < groups.count[k]; ++f) {
                    const int s = s0 + f;
                    a.in[f] = g->buf[par][s];
                    a.out[f] = g->buf[par ^ 1][s];
                    a.kx[f] = float(m->diff[s][0] * ih2 * lap_scale);
                    a.ky[f] = float(m->diff[s][1] * ih2 * lap_scale);
                    a.kz[f] = float(m->diff[s][2] * ih2 * lap_scale);
                    fill_bc(a, f, m, s);
                    a.out_held[f] = a.held[f];
                }
                a.sp0 = s0;
                if (m->model == RD_MODEL_BRUSSELATOR) {
                    a.p[0] = float(m->param[0]);
                    a.p[1] = float(m->param[1]);
                    a.p[2] = float(-(m->param[1] + 1.0));
                } else if (m->model == RD_MODEL_POLLUTANT) {
                    a.p[0] = float(m->param[0]);
                    a.p[1] = float(m->param[1]);
                } else if (m->model == RD_MODEL_TURING) {
                    a.p[0] = float(m->param[0]);   // alpha
                    a.p[1] = float(m->param[1]);   // beta
                    a.p[2] = float(m->param[2]);   // gamma
                } else if (m->model == RD_MODEL_ATMOS) {
                    a.p[0] = float(m->param[0] / g->h);   // u_x / h
                    a.p[1] = float(m->param[1] / g->h);   // u_y / h
                }
            }
        }
    }
    for (auto& row : g->args)
        for (StepArgs& a : row) {
            a.sr = g->sr_mode == RD_ROUND_STOCHASTIC ? 1 : 0;
            a.sr_key = g->sr_seed;
            // the centre weight of the front model's Laplacian form, one FP32
            // value shared by every kernel
            for (int f = 0; f < MAXF; ++f) a.kc[f] = 2.f * ((a.kx[f] + a.ky[f]) + a.kz[f]);
        }
    // Runge-Kutta stages: the same step with other buffers, its stored state
    // blended with the current state A (see launch_rk_step).  The chemical
    // potential pass of the front model is no state update and is not blended.
    g->integrator = m->integrator >= RD_RK2 ? m->integrator : RD_EULER;
    if (g->integrator == RD_RK3) {
        const size_t bytes = g->elems * elem_size(g->storage);
        for (int s = 0; s < ns; ++s)
            if (!g->stage[s]) {
                RD_HIP(hipMalloc(&g->stage[s], bytes));
                RD_HIP(hipMemset(g->stage[s], 0, bytes));
            }
    }
    for (int par = 0; par < 2; ++par)
        for (int k = 0; k < 2; ++k) {
            const bool chmu = m->model == RD_MODEL_FRONT_CH && k == 0;
            StepArgs r2 = g->args[par][k];     // stage 2: B in; A (order 2) or C out
            StepArgs r3 = g->args[par][k];     // stage 3 (order 3): C in, A out
            for (int f = 0; f < MAXF; ++f)
                for (int s = 0; s < ns; ++s) {
                    if (g->args[par][k].in[f] == g->buf[par][s]) {
                        r2.in[f] = g->buf[par ^ 1][s];
                        r3.in[f] = g->stage[s];
                    }
                    if (g->args[par][k].out[f] == g->buf[par ^ 1][s]) {
                        r2.out[f] = g->integrator == RD_RK3 ? g->stage[s] : g->buf[par][s];
                        r3.out[f] = g->buf[par][s];
                        r2.rk_base[f] = r3.rk_base[f] = g->buf[par][s];
                    }
                }
            r2.rk_w = chmu ? 0.f : (g->integrator == RD_RK3 ? 0.25f : 0.5f);
            r3.rk_w = chmu ? 0.f : float(2.0 / 3.0);
            g->rk_args[par][k] = r2;
            g->rk3_args[par][k] = r3;
        }
    g->model = m->model;
    if (m->model == RD_MODEL_FRONT_CH) {
        g->npass = 2;
        g->pass_pm[0] = PM_CHMU;
        g->pass_pm[1] = PM_FRONT;
    } else {
        g->npass = groups.n;
        for (int k = 0; k < groups.n; ++k) g->pass_pm[k] = groups.pm[k];
    }
    rc = apply_plan(g);
    if (rc) return rc;
    g->has_model = true;
    return RD_OK;
}

extern "C" int rd_set_plan(rd_grid* g, const rd_plan* p) {
    if (!g || !p) return fail(RD_EINVAL, "NULL argument");
    if (!g->has_model) return fail(RD_ESTATE, "set a model before a plan");
    if (g->batch) return fail(RD_ESTATE, "grid is in a batch");
    RD_HIP(hipStreamSynchronize(g->stream));
    const rd_plan old = g->plan;
    g->plan = *p;
    const int rc = apply_plan(g);
    if (rc) {
        g->plan = old;
        (void)apply_plan(g);
        return rc;
    }
    return RD_OK;
}

extern "C" int rd_get_plan(const rd_grid* g, rd_plan* p) {
    if (!g || !p) return fail(RD_EINVAL, "NULL argument");
    if (!g->has_model) return fail(RD_ESTATE, "no model set");
    *p = g->eff;
    return RD_OK;
}

extern "C" int rd_get_passes(const rd_grid* g, int32_t* out) {
    if (!g || !out) return fail(RD_EINVAL, "NULL argument");
    if (!g->has_model) return fail(RD_ESTATE, "no model set");
    *out = one_pass(g) ? 1 : g->npass;
    return RD_OK;
}

extern "C" int rd_set_rounding(rd_grid* g, int32_t mode, uint64_t seed) {
    if (!g) return fail(RD_EINVAL, "grid is NULL");
    if (g->batch) return fail(RD_ESTATE, "grid is in a batch");
    if (mode != RD_ROUND_NEAREST && mode != RD_ROUND_STOCHASTIC) return fail(RD_EINVAL, "unknown rounding mode");
    if (mode == RD_ROUND_STOCHASTIC && g->storage != RD_BF16)
        return fail(RD_EINVAL, "stochastic rounding needs BF16 storage");
    if (mode == RD_ROUND_STOCHASTIC && g->has_model && g->integrator >= RD_RK2)
        return fail(RD_EINVAL, "stochastic rounding takes forward Euler steps");
    RD_HIP(hipStreamSynchronize(g->stream));
    g->sr_mode = mode;
    g->sr_seed = uint32_t(seed);
    if (!g->has_model) return RD_OK;
    for (int par = 0; par < 2; ++par)
        for (int k = 0; k < 2; ++k) {
            for (StepArgs* a : {&g->args[par][k], &g->rk_args[par][k], &g->rk3_args[par][k]}) {
                a->sr = mode == RD_ROUND_STOCHASTIC ? 1 : 0;
                a->sr_key = g->sr_seed;
            }
        }
    drop_graphs(g);
    RD_HIP(hipMemcpy(g->d_args, g->args, sizeof(g->args), hipMemcpyHostToDevice));
    RD_HIP(hipMemcpy(g->d_args + 4, g->rk_args, sizeof(g->rk_args), hipMemcpyHostToDevice));
    RD_HIP(hipMemcpy(g->d_args + 8, g->rk3_args, sizeof(g->rk3_args), hipMemcpyHostToDevice));
    return RD_OK;
}

extern "C" int rd_write_field(rd_grid* g, int32_t species, const void* src, int32_t src_dtype,
                              int32_t src_on_device) {
    if (!g || !src) return fail(RD_EINVAL, "NULL argument");
    if (species < 0 || species >= g->ns) return fail(RD_EINVAL, "species out of range");
    if (src_dtype < RD_F32 || src_dtype > RD_F64) return fail(RD_EINVAL, "unknown source dtype");
    if (src_on_device < 0 || src_on_device > 2) return fail(RD_EINVAL, "src_on_device must be 0, 1 or 2");
    if (g->batch) return fail(RD_ESTATE, "grid is in a batch");
    const size_t n = size_t(g->nx) * g->ny * g->nz;
    const size_t es = src_dtype == RD_F64 ? 8 : src_dtype == RD_F32 ? 4 : 2;
    const bool enqueue_only = src_on_device == 2;
    if (!enqueue_only) RD_HIP(hipStreamSynchronize(g->stream));
    const void* dsrc = src;
    void* stage = nullptr;
    if (!src_on_device) {
        RD_HIP(hipMalloc(&stage, n * es));
        const hipError_t e = hipMemcpy(stage, src, n * es, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(stage);
            return fail(RD_EDEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
        }
        dsrc = stage;
    }
    void* dst = g->buf[g->cur][species];
    const unsigned blocks = unsigned(std::min<size_t>((n + 255) / 256, 8192));
    const int nx = int(g->nx), ny = int(g->ny), nz = int(g->nz);
#define RD_PACK(S, SRC) hipLaunchKernelGGL((pack_kernel<S, SRC>), dim3(blocks), dim3(256), 0, g->stream, \
                                           dsrc, dst, nx, ny, nz, g->pitch, g->plane)
#define RD_PACK_SRC(S)                                   \
    switch (src_dtype) {                                 \
    case RD_F32: RD_PACK(S, StF32); break;               \
    case RD_F64: RD_PACK(S, StF64); break;               \
    case RD_BF16: RD_PACK(S, StBF16); break;             \
    default: RD_PACK(S, StF16); break;                   \
    }
    switch (g->storage) {
    case RD_F32: RD_PACK_SRC(StF32) break;
    case RD_BF16: RD_PACK_SRC(StBF16) break;
    default: RD_PACK_SRC(StF16) break;
    }
#undef RD_PACK_SRC
#undef RD_PACK
    const hipError_t e1 = hipGetLastError();
    if (enqueue_only) {
        if (e1 != hipSuccess) return fail(RD_EDEVICE, std::string("pack: ") + hipGetErrorString(e1));
        return RD_OK;
    }
    const hipError_t e2 = hipStreamSynchronize(g->stream);
    (void)hipFree(stage);
    if (e1 != hipSuccess || e2 != hipSuccess)
        return fail(RD_EDEVICE, std::string("pack: ") + hipGetErrorString(e1 != hipSuccess ? e1 : e2));
    return RD_OK;
}

extern "C" int rd_read_field(rd_grid* g, int32_t species, void* dst, int32_t dst_dtype,
                             int32_t dst_on_device) {
    if (!g || !dst) return fail(RD_EINVAL, "NULL argument");
    if (species < 0 || species >= g->ns) return fail(RD_EINVAL, "species out of range");
    if (dst_dtype != RD_F32 && dst_dtype != RD_F64) return fail(RD_EINVAL, "dst dtype must be RD_F32 or RD_F64");
    if (dst_on_device && dst_dtype != RD_F32) return fail(RD_EINVAL, "device destinations take RD_F32");
    const size_t n = size_t(g->nx) * g->ny * g->nz;
    const size_t es = dst_dtype == RD_F64 ? 8 : 4;
    RD_HIP(hipStreamSynchronize(g->stream));
    void* ddst = dst;
    void* stage = nullptr;
    if (!dst_on_device) {
        RD_HIP(hipMalloc(&stage, n * es));
        ddst = stage;
    }
    const void* src = g->buf[g->cur][species];
    const unsigned blocks = unsigned(std::min<size_t>((n + 255) / 256, 8192));
    const int nx = int(g->nx), ny = int(g->ny), nz = int(g->nz);
#define RD_UNPACK(S)                                                                                    \
    if (dst_dtype == RD_F64)                                                                            \
        hipLaunchKernelGGL((unpack_kernel<S, double>), dim3(blocks), dim3(256), 0, g->stream, src,       \
                           static_cast<double*>(ddst), nx, ny, nz, g->pitch, g->plane);                 \
    else                                                                                                \
        hipLaunchKernelGGL((unpack_kernel<S, float>), dim3(blocks), dim3(256), 0, g->stream, src,        \
                           static_cast<float*>(ddst), nx, ny, nz, g->pitch, g->plane);
    switch (g->storage) {
    case RD_F32: RD_UNPACK(StF32) break;
    case RD_BF16: RD_UNPACK(StBF16) break;
    default: RD_UNPACK(StF16) break;
    }
#undef RD_UNPACK
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e == hipSuccess && stage) e = hipMemcpy(dst, stage, n * es, hipMemcpyDeviceToHost);
    (void)hipFree(stage);
    if (e != hipSuccess) return fail(RD_EDEVICE, std::string("read_field: ") + hipGetErrorString(e));
    return RD_OK;
}

extern "C" int rd_step(rd_grid* g, int64_t n) {
    if (!g) return fail(RD_EINVAL, "grid is NULL");
    if (n < 0) return fail(RD_EINVAL, "n must be >= 0");
    if (!g->has_model) return fail(RD_ESTATE, "rd_set_model must come before rd_step");
    if (g->batch) return fail(RD_ESTATE, "grid is in a batch");
    return step_grid(g, n);
}

extern "C" int rd_sync(rd_grid* g) {
    if (!g) return fail(RD_EINVAL, "grid is NULL");
    RD_HIP(hipStreamSynchronize(g->stream));
    return RD_OK;
}

extern "C" int rd_reduce(rd_grid* g, int32_t species, double out[2]) {
    if (!g || !out) return fail(RD_EINVAL, "NULL argument");
    if (species < 0 || species >= g->ns) return fail(RD_EINVAL, "species out of range");
    const long long rows = g->ny * g->nz;
    const int blocks = int(std::min<long long>(rows, kRedBlocks));
    const void* f = g->buf[g->cur][species];
    const int nx = int(g->nx), ny = int(g->ny), nz = int(g->nz);
    switch (g->storage) {
    case RD_F32:
        hipLaunchKernelGGL((reduce_partial<StF32>), dim3(blocks), dim3(256), 0, g->stream, f, nx, ny, nz,
                           g->pitch, g->plane, g->d_part);
        break;
    case RD_BF16:
        hipLaunchKernelGGL((reduce_partial<StBF16>), dim3(blocks), dim3(256), 0, g->stream, f, nx, ny, nz,
                           g->pitch, g->plane, g->d_part);
        break;
    default:
        hipLaunchKernelGGL((reduce_partial<StF16>), dim3(blocks), dim3(256), 0, g->stream, f, nx, ny, nz,
                           g->pitch, g->plane, g->d_part);
        break;
    }
    const double h3 = g->h * g->h * g->h;
    hipLaunchKernelGGL(reduce_final, dim3(1), dim3(256), 0, g->stream, g->d_part, blocks, h3, g->d_red);
    RD_HIP(hipGetLastError());
    RD_HIP(hipMemcpyAsync(out, g->d_red, 2 * sizeof(double), hipMemcpyDeviceToHost, g->stream));
    RD_HIP(hipStreamSynchronize(g->stream));
    if (!is_finite(out[0]) || !is_finite(out[1])) return fail(RD_ENONFINITE, "field holds NaN or Inf");
    return RD_OK;
}

extern "C" int rd_chemical_potential(rd_grid* g, float* dst_host) {
    if (!g || !dst_host) return fail(RD_EINVAL, "NULL argument");
    if (!g->has_model || g->model != RD_MODEL_FRONT_CH) return fail(RD_ESTATE, "needs the front model");
    // the one-pass plan keeps no mu array: the direct kernel's first pass fills it
    const hipError_t e = one_pass(g) ? launch_pass(g->storage, PM_CHMU, RD_KERNEL_DIRECT, -1, g->args[g->cur][0],
                                                   g->d_args + g->cur * 2, 0, g->stream)
                                     : launch_pass(g->storage, PM_CHMU, g->eff.kernel, g->cfg, g->args[g->cur][0],
                                                   g->d_args + g->cur * 2, g->blocks[0], g->stream);
    if (e != hipSuccess) return fail(RD_EDEVICE, std::string("mu pass: ") + hipGetErrorString(e));
    const size_t n = size_t(g->nx) * g->ny * g->nz;
    float* stage = nullptr;
    RD_HIP(hipMalloc(&stage, n * sizeof(float)));
    const unsigned blocks = unsigned(std::min<size_t>((n + 255) / 256, 8192));
    hipLaunchKernelGGL((unpack_kernel<StF32, float>), dim3(blocks), dim3(256), 0, g->stream, g->aux, stage,
                       int(g->nx), int(g->ny), int(g->nz), g->pitch, g->plane);
    hipError_t e2 = hipGetLastError();
    if (e2 == hipSuccess) e2 = hipStreamSynchronize(g->stream);
    if (e2 == hipSuccess) e2 = hipMemcpy(dst_host, stage, n * sizeof(float), hipMemcpyDeviceToHost);
    (void)hipFree(stage);
    if (e2 != hipSuccess) return fail(RD_EDEVICE, std::string("mu read: ") + hipGetErrorString(e2));
    return RD_OK;
}

// ------------------------------------------------ allocation-free reduction

namespace {

// The partial sums of one allocation-free reduction: one (sum, sum of
// squares) pair per block of the first kernel, at most kRedBlocks blocks
// (16 KiB).  Each GPU the library runs on holds its own copy until the
// process ends.  Host code never uses this name as an address (it only
// stands for the symbol); kernels get the device address resolved below.
__device__ __align__(256) double scratch[2 * kRedBlocks];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};   // device address of `scratch`, per device

// The address of the current device's scratch, resolved once per device.
int scratch_on_current_device(double** out) {
    int dev = 0;
    RD_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(RD_EDEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(RD_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return RD_OK;
}

}  // namespace

extern "C" int rd_reduce_noalloc(const void* field, int32_t dtype, int64_t nx, int64_t ny, int64_t nz, double h,
                                 double* out_dev, void* hip_stream) {
    if (!field || !out_dev) return fail(RD_EINVAL, "NULL argument");
    if (dtype != RD_F32 && dtype != RD_BF16 && dtype != RD_F16)
        return fail(RD_EINVAL, "dtype must be RD_F32, RD_BF16 or RD_F16");
    if (nx < 1 || ny < 1 || nz < 1) return fail(RD_EINVAL, "extents must be >= 1");
    if (nx > (1 << 24) || ny > (1 << 24) || nz > (1 << 24) || (__int128)nx * ny * nz > (__int128)1 << 40)
        return fail(RD_EINVAL, "field larger than the largest grid (extents <= 2^24, 2^40 cells)");
    if (!(h > 0.0) || !is_finite(h)) return fail(RD_EINVAL, "h must be a positive finite number");
    double* part = nullptr;
    const int rc = scratch_on_current_device(&part);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    // one block per row, at most kRedBlocks of them: the scratch holds every
    // partial pair the first kernel writes, so nothing needs clearing
    const long long rows = ny * nz;
    const int blocks = int(std::min<long long>(rows, kRedBlocks));
    const int ix = int(nx), iy = int(ny), iz = int(nz);
    const long long plane = nx * ny;
    switch (dtype) {
    case RD_F32:
        hipLaunchKernelGGL((reduce_partial<StF32>), dim3(blocks), dim3(256), 0, st, field, ix, iy, iz, ix, plane, part);
        break;
    case RD_BF16:
        hipLaunchKernelGGL((reduce_partial<StBF16>), dim3(blocks), dim3(256), 0, st, field, ix, iy, iz, ix, plane,
                           part);
        break;
    default:
        hipLaunchKernelGGL((reduce_partial<StF16>), dim3(blocks), dim3(256), 0, st, field, ix, iy, iz, ix, plane, part);
        break;
    }
    hipLaunchKernelGGL(reduce_final, dim3(1), dim3(256), 0, st, part, blocks, h * h * h, out_dev);
    RD_HIP(hipGetLastError());
    return RD_OK;
}

// --------------------------------------------------------------- autotune

extern "C" int rd_autotune(rd_grid* g, int32_t trial_steps, rd_plan* best) {
    if (!g || !best) return fail(RD_EINVAL, "NULL argument");
    if (trial_steps < 1) return fail(RD_EINVAL, "trial_steps must be >= 1");
    if (!g->has_model) return fail(RD_ESTATE, "set a model first");
    if (g->batch) return fail(RD_ESTATE, "grid is in a batch");
    RD_HIP(hipStreamSynchronize(g->stream));
    // Save the state (all species at the current parity).
    const size_t bytes = g->elems * elem_size(g->storage);
    std::vector<void*> snap(g->ns, nullptr);
    auto release = [&]() {
        for (void* p : snap) (void)hipFree(p);
    };
    for (int s = 0; s < g->ns; ++s) {
        if (hipMalloc(&snap[s], bytes) != hipSuccess) {
            release();
            return fail(RD_ENOMEM, "no memory for the autotune snapshot");
        }
        if (hipMemcpy(snap[s], g->buf[g->cur][s], bytes, hipMemcpyDeviceToDevice) != hipSuccess) {
            release();
            return fail(RD_EDEVICE, "snapshot copy failed");
        }
    }
    const int cur0 = g->cur;
    const rd_plan user = g->plan;
    StepClock clk0[2];
    if (hipMemcpy(clk0, g->d_clock, sizeof(clk0), hipMemcpyDeviceToHost) != hipSuccess) {
        release();
        return fail(RD_EDEVICE, "clock copy failed");
    }

    std::vector<rd_plan> cands;
    rd_plan d{};
    d.kernel = RD_KERNEL_DIRECT;
    cands.push_back(d);
    unsigned mask = ~0u;
    for (int k = 0; k < g->npass; ++k) mask &= cfg_mask(g->storage, g->pass_pm[k]);
    for (int i = 0; i < kNumTileCfgs; ++i) {
        if (!((mask >> i) & 1u)) continue;
        const TileCfg c = kTileCfgs[i];
        for (int cz : {0, 64, 32, 16, 8, 4}) {
            if (cz != 0 && cz >= g->nz) continue;
            rd_plan p{};
            p.kernel = RD_KERNEL_TILED;
            p.vx = c.vx;
            p.ry = c.ry;
            p.waves = c.w;
            p.prefetch = c.pf;
            p.cz = cz;
            cands.push_back(p);
        }
    }
    unsigned bmask = ~0u;
    for (int k = 0; k < g->npass; ++k) bmask &= block_mask(g->storage, g->pass_pm[k]);
    for (int i = 0; i < kNumBlockCfgs; ++i) {
        if (!((bmask >> i) & 1u)) continue;
        const BlockCfg c = kBlockCfgs[i];
        rd_plan p{};
        p.kernel = RD_KERNEL_BLOCK;
        p.vx = c.vx;
        p.ry = c.ry;
        p.waves = c.w;
        p.cz = c.cz;
        cands.push_back(p);
        p.order = 1;
        cands.push_back(p);
    }
    for (int i = 0; i < kNumFchCfgs && g->model == RD_MODEL_FRONT_CH && !g->args[0][0].s19; ++i) {
        if (!fch_ok(g->storage, i)) continue;
        const FchCfg c = kFchCfgs[i];
        const long long tiles = ((g->nx + kFchTile - 1) / kFchTile) * ((g->ny + c.by - 1) / c.by);
        std::vector<int> czs = {0, 64, 32, 16};
        // chunk lengths balanced for one, two or three resident workgroups per CU
        for (int bal : {balanced_cz(g, tiles), balanced_cz_k(g, tiles, 2), balanced_cz_k(g, tiles, 3)})
            if (std::find(czs.begin(), czs.end(), bal) == czs.end()) czs.push_back(bal);
        for (int cz : czs) {
            if (cz != 0 && cz >= g->nz) continue;
            for (int order : {0, 1}) {
                rd_plan p{};
                p.kernel = RD_KERNEL_FUSED;
                p.vx = c.wm;
                p.ry = c.by;
                p.waves = c.wu;
                p.prefetch = c.d;
                p.cz = cz;
                p.order = order;
                cands.push_back(p);
            }
        }
    }
    for (int i = 0; i < kNumTrCfgs && !g->args[0][0].s19; ++i) {
        bool ok = true;
        for (int k = 0; k < g->npass; ++k) ok = ok && tr_ok(g->storage, g->pass_pm[k], i);
        if (!ok) continue;
        const TrCfg c = kTrCfgs[i];
        const long long tiles = ((g->nx + kTrTile - 1) / kTrTile) * ((g->ny + c.by - 1) / c.by);
        std::vector<int> czs = {0, 64, 32, 16};
        const int bal = balanced_cz(g, tiles);
        if (std::find(czs.begin(), czs.end(), bal) == czs.end()) czs.push_back(bal);
        for (int cz : czs) {
            if (cz != 0 && cz >= g->nz) continue;
            for (int order : {0, 1}) {
                rd_plan p{};
                p.kernel = RD_KERNEL_TRING;
                p.vx = 2;
                p.ry = c.by;
                p.waves = c.wc;
                p.prefetch = c.d;
                p.cz = cz;
                p.order = order;
                cands.push_back(p);
            }
        }
    }
    for (int i = 0; i < kNumLds2Cfgs && g->npass == 1; ++i) {
        const LdsCfg c = kLds2Cfgs[i];
        if (g->nx != 256 * c.nch || !lds2_ok(g->storage, g->pass_pm[0], i)) continue;
        for (int cz : {0, 64, 32, 16}) {
            if (cz != 0 && cz >= g->nz) continue;
            rd_plan p{};
            p.kernel = RD_KERNEL_LDS2;
            p.vx = 4 * c.nch;
            p.ry = c.by;
            p.waves = c.wc;
            p.prefetch = c.d;
            p.cz = cz;
            cands.push_back(p);
        }
    }
    for (int i = 0; i < kNumLdsCfgs; ++i) {
        const LdsCfg c = kLdsCfgs[i];
        if (!ring_row_fits(g, c.nch)) continue;
        bool ok = true;
        for (int k = 0; k < g->npass; ++k) ok = ok && lds_ok(g->storage, g->pass_pm[k], i);
        if (!ok) continue;
        // One or two workgroups per CU: small grids need short z chunks to
        // fill the chip.  Besides the fixed lengths, try the chunk lengths
        // that give at most 1, 2, 3 or 4 workgroups per CU, so that no
        // launch ends with a partial round of workgroups.
        std::vector<int> czs = {0, 64, 32, 16, 8, 4};
        const int yblocks = (g->ny + c.by - 1) / c.by;
        for (int per_cu = 1; per_cu <= 4; ++per_cu) {
            const int chunks = per_cu * num_cus() / yblocks;
            if (chunks < 1) continue;
            const int cz = (g->nz + chunks - 1) / chunks;
            if (std::find(czs.begin(), czs.end(), cz) == czs.end()) czs.push_back(cz);
        }
        for (int cz : czs) {
            if (cz != 0 && cz >= g->nz) continue;
            rd_plan p{};
            p.kernel = RD_KERNEL_LDS;
            p.vx = 4 * c.nch;
            p.ry = c.by;
            p.waves = c.wc;
            p.prefetch = c.d;
            p.cz = cz;
            cands.push_back(p);
        }
    }
    hipEvent_t e0, e1;
    RD_HIP(hipEventCreate(&e0));
    RD_HIP(hipEventCreate(&e1));
    rd_plan best_plan = heuristic_plan(g);
    int rc = RD_OK;
    // time one plan over `steps` steps from the saved state and restore it;
    // negative if the plan does not apply, rc set on a device error
    auto time_plan = [&](const rd_plan& p, int steps) -> float {
        g->plan = p;
        if (apply_plan(g) != RD_OK) return -1.f;
        float ms = -1.f;
        if ((rc = step_grid(g, 2)) != RD_OK) return -1.f;
        if (hipEventRecord(e0, g->stream) != hipSuccess) { rc = fail(RD_EDEVICE, "event"); return -1.f; }
        if ((rc = step_grid(g, steps + (steps & 1))) != RD_OK) return -1.f;
        if (hipEventRecord(e1, g->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
            rc = fail(RD_EDEVICE, "event sync failed");
            return -1.f;
        }
        (void)hipEventElapsedTime(&ms, e0, e1);
        // restore the state for the next candidate
        for (int s = 0; s < g->ns; ++s)
            if (hipMemcpy(g->buf[cur0][s], snap[s], bytes, hipMemcpyDeviceToDevice) != hipSuccess) {
                rc = fail(RD_EDEVICE, "restore failed");
                return -1.f;
            }
        if (hipMemcpy(g->d_clock, clk0, sizeof(clk0), hipMemcpyHostToDevice) != hipSuccess) {
            rc = fail(RD_EDEVICE, "clock restore failed");
            return -1.f;
        }
        g->cur = cur0;
        return ms;
    };
    // every candidate once; then the four fastest twice more, over twice the
    // steps and in turn, so that near ties are settled by the longer runs
    std::vector<std::pair<float, rd_plan>> timed;
    for (const rd_plan& p : cands) {
        const float ms = time_plan(p, trial_steps);
        if (rc) break;
        if (ms >= 0.f) timed.push_back({ms, p});
    }
    if (rc == RD_OK && !timed.empty()) {
        std::stable_sort(timed.begin(), timed.end(),
                         [](const std::pair<float, rd_plan>& x, const std::pair<float, rd_plan>& y) {
                             return x.first < y.first;
                         });
        const size_t top = std::min<size_t>(4, timed.size());
        std::vector<float> acc(top, 0.f);
        for (int rep = 0; rep < 2 && rc == RD_OK; ++rep)
            for (size_t i = 0; i < top && rc == RD_OK; ++i) {
                const float ms = time_plan(timed[i].second, 2 * trial_steps);
                acc[i] += ms >= 0.f ? ms : 1e30f;
            }
        size_t bi = 0;
        for (size_t i = 1; i < top; ++i)
            if (acc[i] < acc[bi]) bi = i;
        if (rc == RD_OK) best_plan = timed[bi].second;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (int s = 0; s < g->ns && rc == RD_OK; ++s)
        if (hipMemcpy(g->buf[cur0][s], snap[s], bytes, hipMemcpyDeviceToDevice) != hipSuccess)
            rc = fail(RD_EDEVICE, "restore failed");
    if (rc == RD_OK && hipMemcpy(g->d_clock, clk0, sizeof(clk0), hipMemcpyHostToDevice) != hipSuccess)
        rc = fail(RD_EDEVICE, "clock restore failed");
    g->cur = cur0;
    release();
    if (rc == RD_OK) {
        best_plan.graph_chunk = 0;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[{g->nx, g->ny, g->nz, g->ns, tune_model_key(g), g->storage}] = best_plan;
    }
    g->plan = user;
    const int rc2 = apply_plan(g);
    if (rc) return rc;
    if (rc2) return rc2;
    *best = best_plan;
    best->graph_chunk = user.graph_chunk;
    return RD_OK;
}

// ------------------------------------------------------------------ batches

namespace {
struct Member {
    rd_grid* g;
    int64_t steps_left;
    size_t bytes;
};
}  // namespace

struct rd_batch {
    int max_grids = 0;
    size_t budget = 0;
    int storage = RD_F32;
    hipStream_t stream = nullptr;
    std::vector<Member> members;
    size_t bytes = 0;
    char* d_tab = nullptr;         // meta ints, then entries (at entries_off)
    // pinned staging of the table, two alternating copies: a tick's table is
    // written while the previous tick's upload may still wait behind the tick
    // before it (the device copy is one: stream order protects it)
    char* h_tab2[2] = {nullptr, nullptr};
    int next_tab = 0;
    size_t tab_bytes = 0;
    hipEvent_t tab_done[2] = {nullptr, nullptr};
    bool tab_pending[2] = {false, false};
    std::map<int64_t, hipGraphExec_t> graphs;   // by chunk
    int blocks = 0;
};

namespace {
// device table: {ngrids, total_items, ticket, finished, first_item[max_grids
// + 1]} padded to 256 bytes, then max_grids entries
size_t meta_bytes(int max_grids) { return (size_t(max_grids + 5) * sizeof(int) + 255) / 256 * 256; }
size_t table_bytes(int max_grids, int n) { return meta_bytes(max_grids) + size_t(std::max(n, 1)) * sizeof(BatchEntry); }
}

extern "C" int rd_batch_create(int32_t max_grids, size_t hbm_budget_bytes, int32_t storage_dtype,
                               void* hip_stream, rd_batch** out) {
    if (!out) return fail(RD_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_grids < 1 || max_grids > 65536) return fail(RD_EINVAL, "max_grids must be 1..65536");
    if (storage_dtype != RD_F32 && storage_dtype != RD_BF16 && storage_dtype != RD_F16)
        return fail(RD_EINVAL, "bad storage dtype");
    rd_batch* b = new rd_batch();
    b->max_grids = max_grids;
    b->budget = hbm_budget_bytes;
    b->storage = storage_dtype;
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->tab_bytes = table_bytes(max_grids, max_grids);
    if (hipMalloc(reinterpret_cast<void**>(&b->d_tab), b->tab_bytes) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&b->h_tab2[0]), b->tab_bytes, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&b->h_tab2[1]), b->tab_bytes, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&b->tab_done[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->tab_done[1], hipEventDisableTiming) != hipSuccess) {
        rd_batch_destroy(b);
        return fail(RD_ENOMEM, "batch table allocation failed");
    }
    b->blocks = batched_blocks_per_cu(storage_dtype) * num_cus();
    *out = b;
    return RD_OK;
}

extern "C" int rd_batch_destroy(rd_batch* b) {
    if (!b) return fail(RD_EINVAL, "batch is NULL");
    (void)hipStreamSynchronize(b->stream);
    for (auto& m : b->members) m.g->batch = nullptr;
    for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
    (void)hipFree(b->d_tab);
    for (int i = 0; i < 2; ++i) {
        if (b->h_tab2[i]) (void)hipHostFree(b->h_tab2[i]);
        if (b->tab_done[i]) (void)hipEventDestroy(b->tab_done[i]);
    }
    delete b;
    return RD_OK;
}

extern "C" int rd_batch_add(rd_batch* b, rd_grid* g, int64_t steps) {
    if (!b || !g) return fail(RD_EINVAL, "NULL argument");
    if (steps < 0) return fail(RD_EINVAL, "steps must be >= 0");
    if (g->batch) return fail(RD_ESTATE, "grid already in a batch");
    if (!g->has_model) return fail(RD_ESTATE, "grid has no model");
    if (!(g->model == RD_MODEL_BRUSSELATOR || (g->model == RD_MODEL_DIFFUSION && g->ns == 1)))
        return fail(RD_EINVAL, "batches take 1-species diffusion or Brusselator grids");
    if (g->args[0][0].s19) return fail(RD_EINVAL, "batches take 7-point grids");
    if (g->integrator >= RD_RK2) return fail(RD_EINVAL, "batches take forward Euler grids");
    if (g->sr_mode != RD_ROUND_NEAREST) return fail(RD_EINVAL, "batches take round-to-nearest grids");
    if (g->storage != b->storage) return fail(RD_EINVAL, "grid storage differs from the batch's");
    if (g->stream != b->stream) return fail(RD_EINVAL, "grid and batch must use the same stream");
    if (int(b->members.size()) >= b->max_grids) return fail(RD_EINVAL, "batch is full");
    const size_t gb = rd_grid_bytes(g->nx, g->ny, g->nz, g->ns, g->storage, 0);
    if (b->bytes + gb > b->budget) return fail(RD_ENOMEM, "grid would exceed the batch's HBM budget");
    RD_HIP(hipStreamSynchronize(g->stream));
    b->members.push_back({g, steps, gb});
    b->bytes += gb;
    g->batch = b;
    return RD_OK;
}

extern "C" int rd_batch_remove(rd_batch* b, rd_grid* g) {
    if (!b || !g) return fail(RD_EINVAL, "NULL argument");
    for (size_t i = 0; i < b->members.size(); ++i)
        if (b->members[i].g == g) {
            RD_HIP(hipStreamSynchronize(b->stream));
            b->bytes -= b->members[i].bytes;
            b->members.erase(b->members.begin() + i);
            g->batch = nullptr;
            return RD_OK;
        }
    return fail(RD_EINVAL, "grid is not in this batch");
}

extern "C" int rd_batch_info(const rd_batch* b, int32_t* n_members, size_t* bytes_in_use,
                             int64_t* steps_left_total) {
    if (!b) return fail(RD_EINVAL, "batch is NULL");
    int64_t tot = 0;
    for (auto& m : b->members) tot += m.steps_left;
    if (n_members) *n_members = int32_t(b->members.size());
    if (bytes_in_use) *bytes_in_use = b->bytes;
    if (steps_left_total) *steps_left_total = tot;
    return RD_OK;
}

extern "C" int rd_batch_step(rd_batch* b, int64_t chunk, rd_grid** finished, int32_t* n_finished) {
    if (!b || !finished || !n_finished) return fail(RD_EINVAL, "NULL argument");
    if (chunk < 1 || chunk > 100000) return fail(RD_EINVAL, "chunk must be 1..100000");
    *n_finished = 0;
    if (b->members.empty()) return RD_OK;
    // this tick's staging copy: its last upload (two ticks ago) must have run
    const int tb = b->next_tab;
    if (b->tab_pending[tb]) {
        RD_HIP(hipEventSynchronize(b->tab_done[tb]));
        b->tab_pending[tb] = false;
    }
    char* h_tab = b->h_tab2[tb];
    // Work list: every member's tiles, with its arguments for both parities,
    // the grids with the largest tiles first (the kernel's workgroups claim
    // items in list order, so the small ones fill in at the end of a step).
    const int ng = int(b->members.size());
    const size_t moff = meta_bytes(b->max_grids);
    int* meta = reinterpret_cast<int*>(h_tab);
    BatchEntry* ents = reinterpret_cast<BatchEntry*>(h_tab + moff);
    std::memset(h_tab, 0, table_bytes(b->max_grids, ng));
    std::vector<int> order(static_cast<size_t>(ng));
    for (int i = 0; i < ng; ++i) order[size_t(i)] = i;
    auto tile_cost = [&](int i) {
        const rd_grid* g = b->members[size_t(i)].g;
        const long long fields = g->model == RD_MODEL_BRUSSELATOR ? 2 : 1;
        return fields * std::min<long long>(g->nx, kTrTile) * std::min<long long>(g->ny, kBatchTr.by) *
               std::min<long long>(g->nz, kBatchTr.cz);
    };
    std::stable_sort(order.begin(), order.end(), [&](int p, int q) { return tile_cost(p) > tile_cost(q); });
    long long items = 0;
    int64_t max_steps = 0;
    for (int i = 0; i < ng; ++i) {
        const Member& m = b->members[size_t(order[size_t(i)])];
        BatchEntry& e = ents[i];
        // tiles of the tiled LDS ring, each marching a z chunk (short enough
        // that one grid's march does not set the length of a step)
        rd_plan tile{};
        tile.kernel = RD_KERNEL_TRING;
        tile.vx = 2;
        tile.ry = kBatchTr.by;
        tile.waves = kBatchTr.wc;
        tile.prefetch = kBatchTr.d;
        tile.cz = kBatchTr.cz;
        for (int par = 0; par < 2; ++par) {
            e.args[par] = m.g->args[par][0];
            e.ntiles = int(set_tiling(e.args[par], tile));
        }
        e.model = m.g->model == RD_MODEL_BRUSSELATOR ? 1 : 0;
        e.first_item = int(items);
        meta[4 + i] = int(items);
        e.parity = m.g->cur;
        e.steps_left = m.steps_left;
        items += e.ntiles;
        max_steps = std::max(max_steps, m.steps_left);
    }
    if (items > 0x7fffffffLL) return fail(RD_EINVAL, "batch work list too long");
    meta[0] = ng;
    meta[1] = int(items);
    meta[4 + ng] = int(items);
    RD_HIP(hipMemcpyAsync(b->d_tab, h_tab, moff, hipMemcpyHostToDevice, b->stream));
    RD_HIP(hipMemcpyAsync(b->d_tab + moff, h_tab + moff, size_t(ng) * sizeof(BatchEntry),
                          hipMemcpyHostToDevice, b->stream));
    RD_HIP(hipEventRecord(b->tab_done[tb], b->stream));
    b->tab_pending[tb] = true;
    b->next_tab = tb ^ 1;
    const int64_t run = std::min(chunk, max_steps);
    if (b->stream != nullptr) {
        auto it = b->graphs.find(run);
        if (it == b->graphs.end()) {
            RD_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            hipError_t le = hipSuccess;
            for (int64_t i = 0; i < run && le == hipSuccess; ++i)
                le = launch_batched(b->storage, reinterpret_cast<int*>(b->d_tab),
                                    reinterpret_cast<const BatchEntry*>(b->d_tab + meta_bytes(b->max_grids)),
                                    int(i), b->blocks, b->stream);
            hipGraph_t graph = nullptr;
            const hipError_t ce = hipStreamEndCapture(b->stream, &graph);
            if (le != hipSuccess || ce != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return fail(RD_EDEVICE, std::string("batch capture: ") + hipGetErrorString(le != hipSuccess ? le : ce));
            }
            hipGraphExec_t ex = nullptr;
            const hipError_t ie = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ie != hipSuccess) return fail(RD_EDEVICE, std::string("batch instantiate: ") + hipGetErrorString(ie));
            it = b->graphs.emplace(run, ex).first;
        }
        RD_HIP(hipGraphLaunch(it->second, b->stream));
    } else {
        for (int64_t i = 0; i < run; ++i) {
            const hipError_t le = launch_batched(b->storage, reinterpret_cast<int*>(b->d_tab),
                                                 reinterpret_cast<const BatchEntry*>(b->d_tab + meta_bytes(b->max_grids)),
                                                 int(i), b->blocks, b->stream);
            if (le != hipSuccess) return fail(RD_EDEVICE, std::string("batch launch: ") + hipGetErrorString(le));
        }
    }
    // Book-keeping: parity and steps left per member; finished ones leave.
    std::vector<Member> keep;
    for (auto& m : b->members) {
        const int64_t done = std::min(run, m.steps_left);
        m.g->cur ^= int(done & 1);
        m.steps_left -= done;
        if (m.steps_left == 0) {
            finished[(*n_finished)++] = m.g;
            m.g->batch = nullptr;
            b->bytes -= m.bytes;
        } else {
            keep.push_back(m);
        }
    }
    b->members.swap(keep);
    return RD_OK;
}

// -------------------------------------------------------------- measurement

extern "C" int rd_copy_probe(void* dst, const void* src, size_t bytes, void* hip_stream) {
    if (!dst || !src) return fail(RD_EINVAL, "NULL argument");
    if (bytes == 0 || (bytes & 15)) return fail(RD_EINVAL, "bytes must be a positive multiple of 16");
    const long long n4 = (long long)(bytes / 16);
    const long long blocks = (n4 + 255) / 256;
    if (blocks > 0x7fffffffLL) return fail(RD_EINVAL, "copy too large");
    hipLaunchKernelGGL(copy_kernel, dim3(unsigned(blocks)), dim3(256), 0, static_cast<hipStream_t>(hip_stream),
                       static_cast<const float4*>(src), static_cast<float4*>(dst), n4);
    RD_HIP(hipGetLastError());
    return RD_OK;
}
