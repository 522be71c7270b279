// rd_batch_cfg.hpp -- the tile shape of the batched persistent launch
// (rd_tring.hpp, batched_tr_kernel), shared by the engine, which tiles every
// grid of a batch with it, and the translation units that compile the kernel.
#pragma once

namespace rdk {

// Every grid of a batch is tiled for the tiled LDS ring with this shape: rows
// per workgroup, computing waves, ring slots, z planes per tile, producer
// waves.  Two rows per computing wave: the per-plane chain of loads, barrier
// and arithmetic is what bounds the ring on these small grids, and it is
// shared by twice the cells (16-row tiles also re-read fewer halo rows), at
// one workgroup per CU (8-row tiles at two per CU stepped the same 256-grid
// batch 1.5x slower).  Two producer waves share each plane's 36 row loads
// (4.6 % faster on that batch than one; more ring slots gained nothing).
struct BatchTrCfg { int by, wc, d, cz, np; };
constexpr BatchTrCfg kBatchTr = {16, 8, 5, 32, 2};

}  // namespace rdk
