// rd_launch_f16_front.hip -- f16 storage, front model group: tiled and direct kernels.
#define RD_STORAGE rdk::StF16
#define RD_STORAGE_ID rdk::ST_F16
#define RD_GROUP_FRONT
#define RD_FN(name) name##_f16_front
#include "rd_launch_impl.hpp"
