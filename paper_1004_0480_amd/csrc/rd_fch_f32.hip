// rd_fch_f32.hip -- f32 storage: the one-pass Cahn-Hilliard front kernel.
#define RD_FCH_STORAGE rdk::StF32
#define RD_FCH_STORAGE_ID rdk::ST_F32
#define RD_FCH_FN launch_fch_f32
#include "rd_fused_impl.hpp"
