// rd_launch_f32_front.hip -- f32 storage, front model group: tiled and direct kernels.
#define RD_STORAGE rdk::StF32
#define RD_STORAGE_ID rdk::ST_F32
#define RD_GROUP_FRONT
#define RD_FN(name) name##_f32_front
#include "rd_launch_impl.hpp"
