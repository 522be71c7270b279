// rd_launch_bf16_poll.hip -- bf16 storage, poll model group: tiled and direct kernels.
#define RD_STORAGE rdk::StBF16
#define RD_STORAGE_ID rdk::ST_BF16
#define RD_GROUP_POLL
#define RD_FN(name) name##_bf16_poll
#include "rd_launch_impl.hpp"
