// rd_launch_bf16_atmos.hip -- bf16 storage, atmos model group: tiled and direct kernels.
#define RD_STORAGE rdk::StBF16
#define RD_STORAGE_ID rdk::ST_BF16
#define RD_GROUP_ATMOS
#define RD_FN(name) name##_bf16_atmos
#include "rd_launch_impl.hpp"
