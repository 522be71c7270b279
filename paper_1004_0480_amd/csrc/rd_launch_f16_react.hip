// rd_launch_f16_react.hip -- f16 storage, react model group: tiled and direct kernels.
#define RD_STORAGE rdk::StF16
#define RD_STORAGE_ID rdk::ST_F16
#define RD_GROUP_REACT
#define RD_FN(name) name##_f16_react
#include "rd_launch_impl.hpp"
