// rd_fch_f16.hip -- f16 storage: the one-pass Cahn-Hilliard front kernel.
#define RD_FCH_STORAGE rdk::StF16
#define RD_FCH_STORAGE_ID rdk::ST_F16
#define RD_FCH_FN launch_fch_f16
#include "rd_fused_impl.hpp"
