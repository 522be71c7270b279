// rd_fch_cfg.hpp -- shapes of the one-pass Cahn-Hilliard front kernel and
// its launchers (shared by the engine and the kernel's translation units).
#pragma once

#include "rd_internal.hpp"

namespace rdk {

// x tiles of 128 cells (2 per lane); rows per workgroup, waves updating A, B
// and C (one or two rows each), waves computing the chemical potential, slots
// of the C ring (the A/B ring has two fewer).
struct FchCfg { int by, wu, wm, d; };
constexpr FchCfg kFchCfgs[] = {
    {8, 8, 5, 7}, {4, 4, 3, 7}, {4, 4, 3, 6}, {2, 2, 2, 7}, {4, 4, 2, 7}, {8, 8, 4, 8}, {16, 8, 6, 7},
    {4, 4, 3, 9}, {8, 8, 5, 6}, {4, 4, 3, 5}, {4, 4, 2, 5}, {8, 8, 5, 5},
};
constexpr int kNumFchCfgs = sizeof(kFchCfgs) / sizeof(kFchCfgs[0]);
constexpr int kFchTile = 128;            // cells of a row per workgroup column

// LDS bytes of shape i for cells of es bytes: d slots of C (rows with a halo
// of two), d-2 slots of A and B (halo of one), each row the tile plus one
// 16-byte unit on each side, and four FP32 chemical-potential planes of by + 2
// rows of 132 cells.
constexpr long long fch_lds_bytes(int es, int i) {
    const FchCfg c = kFchCfgs[i];
    const long long row = 1LL * (kFchTile + 2 * (16 / es)) * es;
    return row * (1LL * c.d * (c.by + 4) + 2LL * (c.d - 2) * (c.by + 2)) + 4LL * (c.by + 2) * (kFchTile + 4) * 4;
}

// Shape i is compiled for this storage: it fits the LDS and a workgroup of
// at most 16 waves, and the shapes are chosen per cell size (one, two or
// three workgroups per CU).
constexpr bool fch_ok(int storage, int i) {
    if (i < 0 || i >= kNumFchCfgs || storage < 0 || storage >= 3) return false;
    const FchCfg c = kFchCfgs[i];
    if (c.by % c.wu != 0 || 1 + c.wu + c.wm > 16 || c.d < 5 || c.wm < 1 || 2 * (c.by + 2) > 64) return false;
    const bool f32 = storage == 0;
    if (f32 ? !(i <= 5 || i == 8 || i == 9 || i == 10) : !(i == 0 || i == 1 || i == 6 || i == 7 || i == 8 || i == 11))
        return false;
    if (storage == 2 && !(i == 0 || i == 1)) return false;
    return fch_lds_bytes(f32 ? 4 : 2, i) <= 160 * 1024;
}

int fch_cfg_index(int by, int wu, int wm, int d);   // -1 if no such shape

// One-pass front step (shape cfg) with the front update-pass arguments; one
// translation unit per storage type.
hipError_t launch_fch(int storage, int cfg, const StepArgs& h, const StepArgs* d, long long blocks, hipStream_t s);
hipError_t launch_fch_f32(int cfg, const StepArgs* d, long long blocks, hipStream_t s);
hipError_t launch_fch_bf16(int cfg, const StepArgs* d, long long blocks, hipStream_t s);
hipError_t launch_fch_f16(int cfg, const StepArgs* d, long long blocks, hipStream_t s);

}  // namespace rdk
