// rd_launch_f32_diff.hip -- f32 storage, diff model group: tiled and direct kernels.
#define RD_STORAGE rdk::StF32
#define RD_STORAGE_ID rdk::ST_F32
#define RD_GROUP_DIFF
#define RD_FN(name) name##_f32_diff
#define RD_WITH_BATCH
#define RD_BATCH_FN(name) name##_f32
#include "rd_batch_cfg.hpp"
#include "rd_launch_impl.hpp"
