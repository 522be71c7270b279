// rd_launch_f32_react.hip -- f32 storage, react model group: tiled and direct kernels.
#define RD_STORAGE rdk::StF32
#define RD_STORAGE_ID rdk::ST_F32
#define RD_GROUP_REACT
#define RD_FN(name) name##_f32_react
#include "rd_launch_impl.hpp"
