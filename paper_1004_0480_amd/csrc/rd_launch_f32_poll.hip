// rd_launch_f32_poll.hip -- f32 storage, poll model group: tiled and direct kernels.
#define RD_STORAGE rdk::StF32
#define RD_STORAGE_ID rdk::ST_F32
#define RD_GROUP_POLL
#define RD_FN(name) name##_f32_poll
#include "rd_launch_impl.hpp"
