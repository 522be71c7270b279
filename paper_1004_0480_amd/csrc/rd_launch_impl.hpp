// rd_launch_impl.hpp -- kernel instantiation and dispatch for one storage type
// and one group of models.  Included by rd_launch_<storage>_<group>.hip with
//   RD_STORAGE      the storage struct (rdk::StF32, ...)
//   RD_STORAGE_ID   its rdk::Storage value
//   RD_GROUP_DIFF / _REACT / _FRONT / _POLL / _ATMOS   which models to build
//   RD_FN(name)     the group's function-name suffixing
//   RD_WITH_BATCH   also build the batched kernel (once per storage)
#pragma once

#include "rd_internal.hpp"
#include "rd_tring.hpp"

#include <utility>

namespace rdk {
namespace {

using S = RD_STORAGE;
constexpr int kStorage = RD_STORAGE_ID;

template <class M> struct PmOf;
template <> struct PmOf<Diffusion<1>> { static constexpr int v = PM_DIFF1; };
template <> struct PmOf<Diffusion<2>> { static constexpr int v = PM_DIFF2; };
template <> struct PmOf<Diffusion<3>> { static constexpr int v = PM_DIFF3; };
template <> struct PmOf<Diffusion<4>> { static constexpr int v = PM_DIFF4; };
template <> struct PmOf<Brusselator> { static constexpr int v = PM_BRUSS; };
template <> struct PmOf<ChemPotential> { static constexpr int v = PM_CHMU; };
template <> struct PmOf<FrontCH> { static constexpr int v = PM_FRONT; };
template <> struct PmOf<Pollutant<1, false>> { static constexpr int v = PM_POLL1; };
template <> struct PmOf<Pollutant<2, true>> { static constexpr int v = PM_POLL2; };
template <> struct PmOf<Pollutant<2, false>> { static constexpr int v = PM_POLL2U; };
template <> struct PmOf<Turing> { static constexpr int v = PM_TURING; };
template <> struct PmOf<Atmos<1>> { static constexpr int v = PM_ATMOS1; };
template <> struct PmOf<Atmos<2>> { static constexpr int v = PM_ATMOS2; };

template <class M, bool S19>
hipError_t run_direct(const StepArgs& h, const StepArgs* d, hipStream_t s) {
    dim3 grid((h.nx + 63) / 64, (h.ny + 3) / 4, h.nz);
    hipLaunchKernelGGL((direct_kernel<M, S, S19>), grid, dim3(256), 0, s, d);
    return hipGetLastError();
}

template <class M, int I>
hipError_t run_cfg(const StepArgs* d, long long blocks, hipStream_t s) {
    if constexpr (((cfg_mask(kStorage, PmOf<M>::v) >> I) & 1u) != 0u) {
        constexpr TileCfg c = kTileCfgs[I];
        hipLaunchKernelGGL((tiled_kernel<M, S, c.vx, c.ry, c.w, c.pf>), dim3((unsigned)blocks),
                           dim3(64 * c.w), 0, s, d);
        return hipGetLastError();
    } else {
        return hipErrorNotSupported;
    }
}

template <class M, int I>
hipError_t run_block(const StepArgs* d, long long blocks, hipStream_t s) {
    if constexpr (((block_mask(kStorage, PmOf<M>::v) >> I) & 1u) != 0u) {
        constexpr BlockCfg c = kBlockCfgs[I];
        hipLaunchKernelGGL((block_kernel<M, S, c.vx, c.ry, c.w, c.cz>), dim3((unsigned)blocks),
                           dim3(64 * c.w), 0, s, d);
        return hipGetLastError();
    } else {
        return hipErrorNotSupported;
    }
}

template <class M, int I, bool S19>
hipError_t run_lds(const StepArgs* d, long long blocks, hipStream_t s) {
    if constexpr (lds_ok(kStorage, PmOf<M>::v, I)) {
        constexpr LdsCfg c = kLdsCfgs[I];
        hipLaunchKernelGGL((lds_kernel<M, S, c.nch, c.by, c.wc, c.d, S19>), dim3((unsigned)blocks),
                           dim3(64 * (c.wc + 1)), 0, s, d);
        return hipGetLastError();
    } else {
        return hipErrorNotSupported;
    }
}

template <class M, int I>
hipError_t run_lds2(const StepArgs* d, long long blocks, hipStream_t s) {
    if constexpr (lds2_ok(kStorage, PmOf<M>::v, I)) {
        constexpr LdsCfg c = kLds2Cfgs[I];
        hipLaunchKernelGGL((lds2_kernel<M, c.nch, c.by, c.wc, c.d>), dim3((unsigned)blocks), dim3(64 * (c.wc + 1)),
                           0, s, d);
        return hipGetLastError();
    } else {
        return hipErrorNotSupported;
    }
}

template <class M, int I>
hipError_t run_tr(bool plain, const StepArgs* d, long long blocks, hipStream_t s) {
    if constexpr (tr_ok(kStorage, PmOf<M>::v, I)) {
        constexpr TrCfg c = kTrCfgs[I];
        constexpr int threads = 64 * (c.wc + tr_np(M::NF, c.by, c.d));
        if (plain)
            hipLaunchKernelGGL((tr_kernel<M, S, c.by, c.wc, c.d, true>), dim3((unsigned)blocks), dim3(threads), 0, s,
                               d);
        else
            hipLaunchKernelGGL((tr_kernel<M, S, c.by, c.wc, c.d, false>), dim3((unsigned)blocks), dim3(threads), 0,
                               s, d);
        return hipGetLastError();
    } else {
        return hipErrorNotSupported;
    }
}

// Launch table index `cfg` of a shape table: one branch per compiled entry.
template <class M, int... I>
hipError_t run_tiled_index(int cfg, const StepArgs* d, long long blocks, hipStream_t s,
                           std::integer_sequence<int, I...>) {
    hipError_t r = hipErrorInvalidValue;
    ((void)(cfg == I && ((r = run_cfg<M, I>(d, blocks, s)), true)), ...);
    return r;
}

template <class M, int... I>
hipError_t run_block_index(int cfg, const StepArgs* d, long long blocks, hipStream_t s,
                           std::integer_sequence<int, I...>) {
    hipError_t r = hipErrorInvalidValue;
    ((void)(cfg == I && ((r = run_block<M, I>(d, blocks, s)), true)), ...);
    return r;
}

template <class M, bool S19, int... I>
hipError_t run_lds_index(int cfg, const StepArgs* d, long long blocks, hipStream_t s,
                         std::integer_sequence<int, I...>) {
    hipError_t r = hipErrorInvalidValue;
    ((void)(cfg == I && ((r = run_lds<M, I, S19>(d, blocks, s)), true)), ...);
    return r;
}

template <class M, int... I>
hipError_t run_lds2_index(int cfg, const StepArgs* d, long long blocks, hipStream_t s,
                          std::integer_sequence<int, I...>) {
    hipError_t r = hipErrorInvalidValue;
    ((void)(cfg == I && ((r = run_lds2<M, I>(d, blocks, s)), true)), ...);
    return r;
}

template <class M, int... I>
hipError_t run_tr_index(int cfg, bool plain, const StepArgs* d, long long blocks, hipStream_t s,
                        std::integer_sequence<int, I...>) {
    hipError_t r = hipErrorInvalidValue;
    ((void)(cfg == I && ((r = run_tr<M, I>(plain, d, blocks, s)), true)), ...);
    return r;
}

template <class M>
hipError_t run_model(int kernel, int cfg, const StepArgs& h, const StepArgs* d, long long blocks,
                     hipStream_t s) {
    // the 19-point Laplacian runs on the direct and LDS-ring kernels only
    if (kernel == 1) return h.s19 ? run_direct<M, true>(h, d, s) : run_direct<M, false>(h, d, s);
    if (kernel == 4)
        return h.s19 ? run_lds_index<M, true>(cfg, d, blocks, s, std::make_integer_sequence<int, kNumLdsCfgs>{})
                     : run_lds_index<M, false>(cfg, d, blocks, s, std::make_integer_sequence<int, kNumLdsCfgs>{});
    if (h.s19) return hipErrorNotSupported;
    if (kernel == 5) return run_lds2_index<M>(cfg, d, blocks, s, std::make_integer_sequence<int, kNumLds2Cfgs>{});
    if (kernel == 7)
        return run_tr_index<M>(cfg, h.rk_w == 0.f && !h.sr, d, blocks, s,
                               std::make_integer_sequence<int, kNumTrCfgs>{});
    if (kernel == 3) return run_block_index<M>(cfg, d, blocks, s, std::make_integer_sequence<int, kNumBlockCfgs>{});
    return run_tiled_index<M>(cfg, d, blocks, s, std::make_integer_sequence<int, kNumTileCfgs>{});
}

}  // namespace

hipError_t RD_FN(launch_pass)(int pm, int kernel, int cfg, const StepArgs& h, const StepArgs* d,
                              long long blocks, hipStream_t s) {
    switch (pm) {
#ifdef RD_GROUP_DIFF
    case PM_DIFF1: return run_model<Diffusion<1>>(kernel, cfg, h, d, blocks, s);
    case PM_DIFF2: return run_model<Diffusion<2>>(kernel, cfg, h, d, blocks, s);
    case PM_DIFF3: return run_model<Diffusion<3>>(kernel, cfg, h, d, blocks, s);
    case PM_DIFF4: return run_model<Diffusion<4>>(kernel, cfg, h, d, blocks, s);
#endif
#ifdef RD_GROUP_REACT
    case PM_BRUSS: return run_model<Brusselator>(kernel, cfg, h, d, blocks, s);
    case PM_TURING: return run_model<Turing>(kernel, cfg, h, d, blocks, s);
#endif
#ifdef RD_GROUP_FRONT
    case PM_CHMU: return run_model<ChemPotential>(kernel, cfg, h, d, blocks, s);
    case PM_FRONT: return run_model<FrontCH>(kernel, cfg, h, d, blocks, s);
#endif
#ifdef RD_GROUP_POLL
    case PM_POLL1: return run_model<Pollutant<1, false>>(kernel, cfg, h, d, blocks, s);
    case PM_POLL2: return run_model<Pollutant<2, true>>(kernel, cfg, h, d, blocks, s);
    case PM_POLL2U: return run_model<Pollutant<2, false>>(kernel, cfg, h, d, blocks, s);
#endif
#ifdef RD_GROUP_ATMOS
    case PM_ATMOS1: return run_model<Atmos<1>>(kernel, cfg, h, d, blocks, s);
    case PM_ATMOS2: return run_model<Atmos<2>>(kernel, cfg, h, d, blocks, s);
#endif
    default: return hipErrorNotSupported;
    }
}

#ifdef RD_WITH_BATCH
#define RD_BATCH_KERNEL batched_tr_kernel<S, kBatchTr.by, kBatchTr.wc, kBatchTr.d, kBatchTr.np>
hipError_t RD_BATCH_FN(launch_batched)(int* meta, const BatchEntry* ents, int step, int blocks,
                                       hipStream_t s) {
    hipLaunchKernelGGL((RD_BATCH_KERNEL), dim3(blocks), dim3(64 * (kBatchTr.np + kBatchTr.wc)), 0, s, meta, ents, step);
    return hipGetLastError();
}

int RD_BATCH_FN(batched_blocks_per_cu)() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(&RD_BATCH_KERNEL),
                                                     64 * (kBatchTr.np + kBatchTr.wc), 0) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}
#undef RD_BATCH_KERNEL
#endif

}  // namespace rdk
