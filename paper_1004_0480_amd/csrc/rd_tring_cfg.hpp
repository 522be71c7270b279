// rd_tring_cfg.hpp -- shapes of the tiled LDS-ring kernel (rd_tring.hpp) and
// the models and storage types it is compiled for.
#pragma once

#include "rd_internal.hpp"

namespace rdk {

// x tiles of 128 cells (2 per lane); rows per workgroup, computing waves (one
// or two rows each), ring slots.
struct TrCfg { int by, wc, d; };
constexpr TrCfg kTrCfgs[] = {
    {8, 8, 6}, {4, 4, 7}, {8, 4, 6}, {4, 4, 6}, {8, 8, 5}, {16, 8, 5}, {8, 8, 4}, {6, 6, 5},
    {16, 8, 6}, {16, 8, 7},
};
constexpr int kNumTrCfgs = sizeof(kTrCfgs) / sizeof(kTrCfgs[0]);
constexpr int kTrTile = 128;

// LDS bytes of shape i for nf fields of es-byte cells: d slots of by + 2 rows
// per field, each row the tile plus one 16-byte unit on each side.
constexpr long long tr_lds_bytes(int nf, int es, int i) {
    return 1LL * (kTrTile + 2 * (16 / es)) * es * nf * (kTrCfgs[i].by + 2) * kTrCfgs[i].d;
}

// Fields of a pass model the kernel takes (every field read and written in
// the storage type), 0 for the others.
constexpr int tr_fields(int pm) {
    switch (pm) {
    case PM_DIFF1: return 1;
    case PM_DIFF2: return 2;
    case PM_BRUSS: return 2;
    case PM_POLL1: return 1;
    case PM_POLL2: return 2;
    case PM_POLL2U: return 2;
    default: return 0;
    }
}

// Loading waves of a shape for nf fields: two when one wave could not keep
// the d-3 steps it should have in flight (nf*(by+2) row loads each) within
// the 63 loads its wait counter can express.
constexpr int tr_np(int nf, int by, int d) { return nf * (by + 2) * (d - 3) > 63 ? 2 : 1; }

// Shape i is compiled for this storage (FP32 or BF16) and pass model.
constexpr bool tr_ok(int storage, int pm, int i) {
    if (i < 0 || i >= kNumTrCfgs || (storage != ST_F32 && storage != ST_BF16)) return false;
    const int nf = tr_fields(pm);
    const TrCfg c = kTrCfgs[i];
    if (nf == 0 || c.by % c.wc != 0 || c.wc + tr_np(nf, c.by, c.d) > 16 || c.d < 4 || (c.by / c.wc) > 2)
        return false;
    return tr_lds_bytes(nf, storage == ST_F32 ? 4 : 2, i) <= 160 * 1024;
}

int tr_cfg_index(int by, int wc, int d);   // -1 if no such shape

}  // namespace rdk
