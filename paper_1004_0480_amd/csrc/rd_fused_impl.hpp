// rd_fused_impl.hpp -- instantiation and dispatch of the one-pass front
// kernel for one storage type.  Included by rd_fch_<storage>.hip with
//   RD_FCH_STORAGE     the storage struct (rdk::StF32, ...)
//   RD_FCH_STORAGE_ID  its rdk::Storage value
//   RD_FCH_FN          the launcher's name
#pragma once

#include <utility>

#include "rd_fused.hpp"

namespace rdk {
namespace {

template <int I>
hipError_t run_fch(const StepArgs* d, long long blocks, hipStream_t s) {
    if constexpr (fch_ok(RD_FCH_STORAGE_ID, I)) {
        constexpr FchCfg c = kFchCfgs[I];
        hipLaunchKernelGGL((fch_kernel<RD_FCH_STORAGE, c.by, c.wu, c.wm, c.d>), dim3((unsigned)blocks),
                           dim3(64 * (1 + c.wu + c.wm)), 0, s, d);
        return hipGetLastError();
    } else {
        return hipErrorNotSupported;
    }
}

template <int... I>
hipError_t run_fch_index(int cfg, const StepArgs* d, long long blocks, hipStream_t s,
                         std::integer_sequence<int, I...>) {
    hipError_t r = hipErrorInvalidValue;
    ((void)(cfg == I && ((r = run_fch<I>(d, blocks, s)), true)), ...);
    return r;
}

}  // namespace

hipError_t RD_FCH_FN(int cfg, const StepArgs* d, long long blocks, hipStream_t s) {
    return run_fch_index(cfg, d, blocks, s, std::make_integer_sequence<int, kNumFchCfgs>{});
}

}  // namespace rdk
