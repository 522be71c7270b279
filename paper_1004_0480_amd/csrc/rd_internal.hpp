// rd_internal.hpp -- host-side glue between the engine and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include "rd_device.hpp"

namespace rdk {

// Kernel families a pass can run.
enum PassModel {
    PM_DIFF1 = 0, PM_DIFF2, PM_DIFF3, PM_DIFF4,
    PM_BRUSS,
    PM_CHMU,        // Cahn-Hilliard chemical potential (first Laplacian pass)
    PM_FRONT,       // front + Cahn-Hilliard update (second pass)
    PM_POLL1, PM_POLL2, PM_POLL3, PM_POLL4,
    PM_COUNT
};

enum Storage { ST_F32 = 0, ST_BF16 = 1, ST_F16 = 2, ST_COUNT };

// Tile shapes of the tiled kernel: cells per lane along x, rows per wave,
// waves per workgroup.
struct TileCfg { int vx, ry, w; };
constexpr TileCfg kTileCfgs[] = {
    {4, 4, 4}, {4, 2, 4}, {4, 1, 4}, {2, 4, 4}, {2, 2, 4}, {2, 1, 4}, {1, 4, 4}, {4, 4, 1},
};
constexpr int kNumTileCfgs = sizeof(kTileCfgs) / sizeof(kTileCfgs[0]);

// Which tile shapes are compiled for each storage and pass model (bit i =
// kTileCfgs[i]).  Models with more fields keep fewer rows per wave so that
// their register window fits without spilling.
constexpr unsigned cfg_mask(int storage, int pm) {
    const bool light = pm == PM_DIFF1 || pm == PM_CHMU;
    const bool medium = pm == PM_BRUSS || pm == PM_DIFF2 || pm == PM_POLL1 || pm == PM_POLL2;
    if (storage == ST_F32) {
        if (pm == PM_DIFF1) return 0b11001011u;            // 444 424 244 144 441
        if (pm == PM_CHMU) return 0b00011011u;             // 444 424 244 224
        if (medium) return 0b01011011u;                    // 444 424 244 224 144
        return 0b01110110u;                                // 424 414 224 214 144
    }
    if (storage == ST_BF16) {
        if (pm == PM_DIFF1 || pm == PM_BRUSS) return 0b01001011u;   // 444 424 244 144
        if (light) return 0b00001001u;                              // 444 244
        if (pm == PM_FRONT) return 0b00010110u;                     // 424 414 224
        return 0b00010010u;                                         // 424 224
    }
    if (pm == PM_DIFF1 || pm == PM_BRUSS) return 0b01001010u;       // 424 244 144
    if (light) return 0b00000001u;                                  // 444
    return 0b00010100u;                                             // 414 224
}

int tile_cfg_index(int vx, int ry, int w);   // -1 if no such shape

// Launch one pass.  kernel: 1 direct, 2 tiled (cfg = kTileCfgs index).
// `h` is the host copy of the arguments (for the launch shape), `d` the same
// arguments in device memory (what the kernel reads).
hipError_t launch_pass(int storage, int pm, int kernel, int cfg, const StepArgs& h,
                       const StepArgs* d, long long blocks, hipStream_t s);

// Batched persistent kernel (tile shape kBatchTile): one step of every table
// entry whose steps_left > step.
constexpr TileCfg kBatchTile = {1, 4, 4};
hipError_t launch_batched(int storage, const BatchTable* tab, int step, int blocks, hipStream_t s);
int batched_blocks_per_cu(int storage);

// Per storage and model group (one translation unit each); return
// hipErrorNotSupported for models outside the group.
#define RD_DECLARE_GROUP(sfx)                                                                  \
    hipError_t launch_pass_##sfx(int pm, int kernel, int cfg, const StepArgs& h,                \
                                 const StepArgs* d, long long blocks, hipStream_t s);
RD_DECLARE_GROUP(f32_diff)
RD_DECLARE_GROUP(f32_react)
RD_DECLARE_GROUP(f32_poll)
RD_DECLARE_GROUP(bf16_diff)
RD_DECLARE_GROUP(bf16_react)
RD_DECLARE_GROUP(bf16_poll)
RD_DECLARE_GROUP(f16_diff)
RD_DECLARE_GROUP(f16_react)
RD_DECLARE_GROUP(f16_poll)
#undef RD_DECLARE_GROUP

hipError_t launch_batched_f32(const BatchTable* tab, int step, int blocks, hipStream_t s);
hipError_t launch_batched_bf16(const BatchTable* tab, int step, int blocks, hipStream_t s);
hipError_t launch_batched_f16(const BatchTable* tab, int step, int blocks, hipStream_t s);
int batched_blocks_per_cu_f32();
int batched_blocks_per_cu_bf16();
int batched_blocks_per_cu_f16();

}  // namespace rdk
