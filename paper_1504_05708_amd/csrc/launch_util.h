// Launch of a kernel given by address, with its dynamic LDS size.
#pragma once
#include <hip/hip_runtime.h>

#include "launch.h"

namespace duq {

inline hipError_t launch_fn(const void* kernel, const LaunchCfg& cfg, void** args) {
    hipError_t e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)cfg.shmem);
    if (e != hipSuccess) return e;
    if (cfg.cooperative)
        return hipLaunchCooperativeKernel(kernel, dim3(cfg.nblocks), dim3(cfg.nthreads), args, cfg.shmem, cfg.stream);
    return hipLaunchKernel(kernel, dim3(cfg.nblocks), dim3(cfg.nthreads), args, cfg.shmem, cfg.stream);
}

}  // namespace duq
