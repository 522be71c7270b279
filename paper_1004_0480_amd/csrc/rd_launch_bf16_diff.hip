// rd_launch_bf16_diff.hip -- bf16 storage, diff model group: tiled and direct kernels.
#define RD_STORAGE rdk::StBF16
#define RD_STORAGE_ID rdk::ST_BF16
#define RD_GROUP_DIFF
#define RD_FN(name) name##_bf16_diff
#define RD_WITH_BATCH
#define RD_BATCH_FN(name) name##_bf16
#include "rd_batch_cfg.hpp"
#include "rd_launch_impl.hpp"
