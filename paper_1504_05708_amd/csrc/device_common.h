// Device helpers shared by the DFOM kernels: wave/block reductions, the
// team barrier, vector loads.  gfx950 (CDNA4): 64-wide wavefronts.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace duq {

constexpr int kWave = 64;
constexpr int kMaxWaves = 16;            // blocks of at most 1024 threads

__device__ __forceinline__ double wave_sum(double v) {
    // xor butterfly: every lane ends with the bitwise-identical total
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Sum K values over the block in a fixed order; every thread receives the
// totals.  `scratch` holds kMaxWaves*K doubles of LDS.
template <int K>
__device__ __forceinline__ void block_allreduce(double (&v)[K], double* scratch) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) scratch[wid * K + k] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += scratch[w * K + k];
        v[k] = s;
    }
    __syncthreads();
}

// A team is either one workgroup (size 1) or every workgroup of a
// cooperative launch.  The grid barrier spins with a bounded count so that
// every wave exits even if a peer never arrives; the failure is flagged in
// bar[2] and reported by the host.
struct Team {
    int rank;
    int size;
    unsigned* bar;

    // Returns true when the team must abort (barrier timeout seen).
    __device__ __forceinline__ bool sync() const {
        if (size == 1) {
            __syncthreads();
            return false;
        }
        __shared__ int s_abort;
        __syncthreads();
        if (threadIdx.x == 0) {
            int abort = 0;
            __threadfence();  // release this block's writes at device scope
            const unsigned gen0 =
                __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned arrived =
                __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            if (arrived == (unsigned)size - 1u) {
                __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&bar[1], gen0 + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                unsigned spins = 0;
                while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen0) {
                    __builtin_amdgcn_s_sleep(2);
                    ++spins;
                    if ((spins & 1023u) == 0u &&
                        __hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                        abort = 1;   // another block gave up
                        break;
                    }
                    if (spins > (1u << 23)) {  // far beyond any phase: a peer is gone
                        __hip_atomic_store(&bar[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        abort = 1;
                        break;
                    }
                }
            }
            __threadfence();  // acquire: see every block's writes
            if (!abort)
                abort = __hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
            s_abort = abort;
        }
        __syncthreads();
        return s_abort != 0;
    }
};

// Contiguous share [lo, hi) of `len` items for member `rank` of `size`.
__device__ __forceinline__ void share(int len, int rank, int size, int& lo, int& hi) {
    lo = (int)(((long long)len * rank) / size);
    hi = (int)(((long long)len * (rank + 1)) / size);
}

template <typename T> struct Vec16;
template <> struct Vec16<double> {
    typedef double __attribute__((ext_vector_type(2))) type;
    static constexpr int N = 2;
};
template <> struct Vec16<float> {
    typedef float __attribute__((ext_vector_type(4))) type;
    static constexpr int N = 4;
};

}  // namespace duq
