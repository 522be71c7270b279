// rd_internal.hpp -- host-side glue between the engine and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <initializer_list>

#include "rd_device.hpp"

namespace rdk {

// Kernel families a pass can run.
enum PassModel {
    PM_DIFF1 = 0, PM_DIFF2, PM_DIFF3, PM_DIFF4,
    PM_BRUSS,
    PM_CHMU,        // Cahn-Hilliard chemical potential (first Laplacian pass)
    PM_FRONT,       // front + Cahn-Hilliard update (second pass)
    PM_POLL1,       // one pollutant
    PM_POLL2,       // the coupled pair (transfer from the first to the second)
    PM_POLL2U,      // two uncoupled pollutants
    PM_TURING,      // activator-inhibitor (Table 1, second row)
    PM_ATMOS1,      // one species under the atmospheric wind
    PM_ATMOS2,      // two species under the atmospheric wind
    PM_COUNT
};

enum Storage { ST_F32 = 0, ST_BF16 = 1, ST_F16 = 2, ST_COUNT };

// Tile shapes of the tiled (z-march) kernel: cells per lane along x, rows per
// wave, waves per workgroup, planes kept in flight ahead of the z window.
struct TileCfg { int vx, ry, w, pf; };
constexpr TileCfg kTileCfgs[] = {
    {4, 1, 4, 1}, {4, 1, 4, 2}, {2, 2, 4, 2}, {2, 1, 4, 2}, {4, 2, 4, 1}, {1, 4, 4, 2}, {2, 1, 4, 1},
};
constexpr int kNumTileCfgs = sizeof(kTileCfgs) / sizeof(kTileCfgs[0]);

// Slab shapes of the plane-block kernel: cells per lane along x, rows per
// wave, waves per workgroup, planes per slab.
struct BlockCfg { int vx, ry, w, cz; };
constexpr BlockCfg kBlockCfgs[] = {
    {4, 1, 4, 2}, {4, 1, 4, 4}, {4, 2, 4, 2}, {4, 2, 4, 4},
    {4, 1, 4, 8}, {2, 2, 4, 4}, {2, 1, 4, 4}, {4, 2, 1, 2},
    {4, 1, 1, 2}, {4, 2, 1, 4}, {4, 4, 1, 2}, {4, 2, 2, 2}, {4, 3, 1, 2},
};
constexpr int kNumBlockCfgs = sizeof(kBlockCfgs) / sizeof(kBlockCfgs[0]);

// Ring shapes of the LDS-ring z-march (FP32, rows of 256*nch cells): 256-cell
// chunks per row, rows per workgroup, consumer waves, ring slots.
struct LdsCfg { int nch, by, wc, d; };
constexpr LdsCfg kLdsCfgs[] = {
    {1, 8, 4, 7}, {1, 8, 8, 7}, {2, 8, 4, 6}, {2, 4, 4, 6}, {2, 8, 8, 6}, {2, 4, 4, 7},
    {2, 8, 8, 7}, {1, 12, 6, 5}, {2, 12, 6, 5}, {2, 6, 6, 5},
    // four-field shapes (the front model's update pass reads A, B, C and mu)
    {1, 4, 4, 6}, {2, 2, 2, 5},
};
constexpr int kFirstLds4Cfg = 10;
constexpr int kNumLdsCfgs = sizeof(kLdsCfgs) / sizeof(kLdsCfgs[0]);

// Ring shapes of the two-steps-per-launch LDS kernel (same fields).
constexpr LdsCfg kLds2Cfgs[] = {
    {1, 4, 8, 6}, {2, 4, 8, 6}, {1, 8, 8, 5}, {2, 6, 6, 4}, {1, 6, 12, 4}, {2, 6, 12, 4}, {2, 4, 12, 6}, {1, 4, 12, 6},
};
constexpr int kNumLds2Cfgs = sizeof(kLds2Cfgs) / sizeof(kLds2Cfgs[0]);

constexpr unsigned bits(std::initializer_list<int> l) {
    unsigned m = 0;
    for (int i : l) m |= 1u << i;
    return m;
}

// Which shapes are compiled for each storage and pass model (bit i = index
// into the table).  Models with more fields skip the largest register
// footprints.  The chemical-potential pass covers every shape of the front
// update so both passes of a step share one plan.
constexpr unsigned cfg_mask(int storage, int pm) {
    const bool light = pm == PM_DIFF1 || pm == PM_CHMU || pm == PM_BRUSS || pm == PM_TURING;
    const bool medium = pm == PM_DIFF2 || pm == PM_POLL1 || pm == PM_POLL2 || pm == PM_POLL2U ||
                        pm == PM_ATMOS1 || pm == PM_ATMOS2;
    if (storage == ST_F32)
        return light ? bits({0, 1, 2, 3, 4, 5, 6}) : medium ? bits({0, 1, 2, 3, 5, 6}) : bits({3, 6});
    if (storage == ST_BF16) return light ? bits({0, 1, 2, 3, 6}) : bits({3, 6});
    return light ? bits({1, 2, 3, 6}) : bits({3, 6});
}
constexpr unsigned block_mask(int storage, int pm) {
    const bool light = pm == PM_DIFF1 || pm == PM_CHMU || pm == PM_BRUSS || pm == PM_TURING;
    const bool medium = pm == PM_DIFF2 || pm == PM_POLL1 || pm == PM_POLL2 || pm == PM_POLL2U ||
                        pm == PM_ATMOS1 || pm == PM_ATMOS2;
    if (storage == ST_F32) {
        if (light) return bits({0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12});
        if (medium) return bits({0, 1, 2, 5, 6, 7, 8, 11});
        return bits({0, 2, 5, 6, 7, 8, 11});
    }
    if (storage == ST_BF16) {
        if (pm == PM_DIFF1 || pm == PM_BRUSS || pm == PM_TURING) return bits({0, 1, 2, 3, 5});
        if (pm == PM_CHMU || pm == PM_FRONT) return bits({0, 2, 5, 6});
        return bits({0, 5});
    }
    if (pm == PM_DIFF1 || pm == PM_BRUSS || pm == PM_TURING) return bits({0, 1, 5});
    return bits({0, 5});
}

// Stencil fields a pass model reads.
constexpr int pm_fields(int pm) {
    return pm == PM_DIFF1 || pm == PM_CHMU || pm == PM_POLL1 || pm == PM_ATMOS1 ? 1
         : pm == PM_DIFF2 || pm == PM_BRUSS || pm == PM_POLL2 || pm == PM_POLL2U || pm == PM_TURING ||
                   pm == PM_ATMOS2
             ? 2
         : pm == PM_DIFF3 ? 3 : 4;
}

// LDS-ring shape i is compiled for this storage and pass model: FP32 fields,
// a ring that fits the LDS and the vmcnt range; models of one or two fields
// take the first shapes and the first four-field one (1·4·4, D 6: two
// workgroups per CU for two fields), the two passes of the front model the
// four-field ones (both passes of a step share one plan).
// BF16 storage takes the ring with 2-byte cells for models of one or two
// fields, on the four shapes that serve those best in FP32.
constexpr bool lds_ok(int storage, int pm, int i) {
    if (i < 0 || i >= kNumLdsCfgs) return false;
    const bool front = pm == PM_CHMU || pm == PM_FRONT;
    if (storage == ST_BF16) {
        if (front || pm_fields(pm) > 2 || !(i == 1 || i == 4 || i == 7 || i == 9)) return false;
    } else if (storage != ST_F32 || (front ? i < kFirstLds4Cfg : i > kFirstLds4Cfg) ||
               (!front && pm_fields(pm) > 2)) {
        return false;
    }
    const LdsCfg c = kLdsCfgs[i];
    const int es = storage == ST_F32 ? 4 : 2, nf = pm_fields(pm), rows = c.by + 2;
    const int nq = (256 * c.nch * es + 1023) / 1024;            // 16-byte-per-lane loads per row
    const long long bytes = 1LL * es * c.d * nf * rows * 256 * c.nch;
    return bytes <= 160 * 1024 && (c.d - 4) * nf * rows * nq <= 63 && c.d >= 4 && c.by % c.wc == 0;
}

// Two-steps-per-launch shape i: FP32, diffusion or Brusselator (no point
// sources), input ring of by+4 rows and four intermediate planes of by+2
// rows within the LDS and the vmcnt range.
constexpr bool lds2_ok(int storage, int pm, int i) {
    if (storage != ST_F32 || !(pm == PM_DIFF1 || pm == PM_DIFF2 || pm == PM_BRUSS) || i < 0 || i >= kNumLds2Cfgs)
        return false;
    const LdsCfg c = kLds2Cfgs[i];
    const int nf = pm_fields(pm);
    const long long bytes = 4LL * 256 * c.nch * nf * (c.d * (c.by + 4) + 4 * (c.by + 2));
    return bytes <= 160 * 1024 && (c.d - 4) * nf * (c.by + 4) * c.nch <= 63 && c.d >= 4 && c.wc <= 15;
}

int tile_cfg_index(int vx, int ry, int w, int pf);   // -1 if no such shape
int lds_cfg_index(int nch, int by, int wc, int d);   // -1 if no such shape
int lds2_cfg_index(int nch, int by, int wc, int d);  // -1 if no such shape
int block_cfg_index(int vx, int ry, int w, int cz);  // -1 if no such shape

// Launch one pass.  kernel: 1 direct, 2 tiled (cfg = kTileCfgs index),
// 3 plane block (cfg = kBlockCfgs index), 4 LDS ring (cfg = kLdsCfgs index),
// 5 LDS ring with two steps per launch (cfg = kLds2Cfgs index).
// `h` is the host copy of the arguments (for the launch shape), `d` the same
// arguments in device memory (what the kernel reads).
hipError_t launch_pass(int storage, int pm, int kernel, int cfg, const StepArgs& h,
                       const StepArgs* d, long long blocks, hipStream_t s);

// Batched persistent kernel (shape: rd_batch_cfg.hpp): one step of every
// table entry whose steps_left > step.
hipError_t launch_batched(int storage, int* meta, const BatchEntry* ents, int step, int blocks,
                          hipStream_t s);
int batched_blocks_per_cu(int storage);

// Per storage and model group (one translation unit each); return
// hipErrorNotSupported for models outside the group.
#define RD_DECLARE_GROUP(sfx)                                                                  \
    hipError_t launch_pass_##sfx(int pm, int kernel, int cfg, const StepArgs& h,                \
                                 const StepArgs* d, long long blocks, hipStream_t s);
RD_DECLARE_GROUP(f32_diff)
RD_DECLARE_GROUP(f32_react)
RD_DECLARE_GROUP(f32_front)
RD_DECLARE_GROUP(f32_poll)
RD_DECLARE_GROUP(f32_atmos)
RD_DECLARE_GROUP(bf16_diff)
RD_DECLARE_GROUP(bf16_react)
RD_DECLARE_GROUP(bf16_front)
RD_DECLARE_GROUP(bf16_poll)
RD_DECLARE_GROUP(bf16_atmos)
RD_DECLARE_GROUP(f16_diff)
RD_DECLARE_GROUP(f16_react)
RD_DECLARE_GROUP(f16_front)
RD_DECLARE_GROUP(f16_poll)
RD_DECLARE_GROUP(f16_atmos)
#undef RD_DECLARE_GROUP

hipError_t launch_batched_f32(int* meta, const BatchEntry* ents, int step, int blocks, hipStream_t s);
hipError_t launch_batched_bf16(int* meta, const BatchEntry* ents, int step, int blocks, hipStream_t s);
hipError_t launch_batched_f16(int* meta, const BatchEntry* ents, int step, int blocks, hipStream_t s);
int batched_blocks_per_cu_f32();
int batched_blocks_per_cu_bf16();
int batched_blocks_per_cu_f16();

}  // namespace rdk
