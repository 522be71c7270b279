// rd_launch_f16_poll.hip -- f16 storage, poll model group: tiled and direct kernels.
#define RD_STORAGE rdk::StF16
#define RD_STORAGE_ID rdk::ST_F16
#define RD_GROUP_POLL
#define RD_FN(name) name##_f16_poll
#include "rd_launch_impl.hpp"
