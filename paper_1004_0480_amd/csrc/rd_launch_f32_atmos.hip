// rd_launch_f32_atmos.hip -- f32 storage, atmos model group: tiled and direct kernels.
#define RD_STORAGE rdk::StF32
#define RD_STORAGE_ID rdk::ST_F32
#define RD_GROUP_ATMOS
#define RD_FN(name) name##_f32_atmos
#include "rd_launch_impl.hpp"
