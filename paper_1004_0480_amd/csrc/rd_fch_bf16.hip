// rd_fch_bf16.hip -- bf16 storage: the one-pass Cahn-Hilliard front kernel.
#define RD_FCH_STORAGE rdk::StBF16
#define RD_FCH_STORAGE_ID rdk::ST_BF16
#define RD_FCH_FN launch_fch_bf16
#include "rd_fused_impl.hpp"
