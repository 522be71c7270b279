// rd_launch_f16_diff.hip -- f16 storage, diff model group: tiled and direct kernels.
#define RD_STORAGE rdk::StF16
#define RD_STORAGE_ID rdk::ST_F16
#define RD_GROUP_DIFF
#define RD_FN(name) name##_f16_diff
#define RD_WITH_BATCH
#define RD_BATCH_FN(name) name##_f16
#include "rd_batch_cfg.hpp"
#include "rd_launch_impl.hpp"
