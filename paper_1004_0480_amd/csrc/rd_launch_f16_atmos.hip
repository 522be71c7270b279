// rd_launch_f16_atmos.hip -- f16 storage, atmos model group: tiled and direct kernels.
#define RD_STORAGE rdk::StF16
#define RD_STORAGE_ID rdk::ST_F16
#define RD_GROUP_ATMOS
#define RD_FN(name) name##_f16_atmos
#include "rd_launch_impl.hpp"
