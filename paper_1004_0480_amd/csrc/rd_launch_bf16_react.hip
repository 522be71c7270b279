// rd_launch_bf16_react.hip -- bf16 storage, react model group: tiled and direct kernels.
#define RD_STORAGE rdk::StBF16
#define RD_STORAGE_ID rdk::ST_BF16
#define RD_GROUP_REACT
#define RD_FN(name) name##_bf16_react
#include "rd_launch_impl.hpp"
