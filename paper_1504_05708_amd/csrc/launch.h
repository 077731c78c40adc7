// Host-side launch interface between the runtime (duq_api.cpp) and kernels.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "internal.h"

namespace duq {

struct LaunchCfg {
    int nblocks;
    int nthreads;
    size_t shmem;
    bool cooperative;
    hipStream_t stream;
};

// Problem with type-erased matrix pointers (dtype selects float/double).
struct GenericProblem {
    int n, p;
    const void* Q;
    const void* G;
    const double* q;
    const double* g;
    const double* lb;
    const double* ub;
};

struct LanczosWork;

size_t dfom_lds_bytes(int n, int p, int nblocks);
size_t lanczos_lds_bytes(int n, int p, int nblocks, int k);
hipError_t dfom_occupancy(int dtype, int acc, int nthreads, size_t shmem, int* blocks_per_cu);
hipError_t launch_dfom(int dtype, int acc, const LaunchCfg& cfg, const GenericProblem& gp,
                       const DevParams& par, const DevWork& W);
hipError_t launch_lanczos(int dtype, const LaunchCfg& cfg, const GenericProblem& gp, const LanczosWork& L,
                          int k, int use_gtg);
hipError_t launch_count_nonfinite(int dtype, const void* a, long len, unsigned* out, hipStream_t s);

}  // namespace duq
