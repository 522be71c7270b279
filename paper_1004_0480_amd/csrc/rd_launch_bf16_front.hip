// rd_launch_bf16_front.hip -- bf16 storage, front model group: tiled and direct kernels.
#define RD_STORAGE rdk::StBF16
#define RD_STORAGE_ID rdk::ST_BF16
#define RD_GROUP_FRONT
#define RD_FN(name) name##_bf16_front
#include "rd_launch_impl.hpp"
