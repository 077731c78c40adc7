// Device helpers shared by the DFOM kernels: wave/block reductions, the
// team barrier, vector loads.  gfx950 (CDNA4): 64-wide wavefronts.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace duq {

constexpr int kWave = 64;
constexpr int kMaxWaves = 16;            // blocks of at most 1024 threads
constexpr int kTlDoubles = 512 * 4;      // short-row G^T v scratch: blockDim (<= 512) x 4

// Lane exchanges of the xor butterfly in VALU registers (no LDS round trip):
// lanes l and l ^ 32 (l ^ 16) by the row swaps of gfx950, which leave each
// lane with its own value and its partner's; l ^ 8 by DPP row_ror:8, l ^ 4
// by row_half_mirror then quad_perm [3,2,1,0], l ^ 2 and l ^ 1 by quad_perm.
template <int CTRL>
__device__ __forceinline__ int dpp_lane(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_lane(double v) {
    const int lo = dpp_lane<CTRL>((int)__double2loint(v)), hi = dpp_lane<CTRL>((int)__double2hiint(v));
    return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_lane(float v) {
    return __int_as_float(dpp_lane<CTRL>(__float_as_int(v)));
}
__device__ __forceinline__ double swap_sum32(double v) {
    const unsigned lo = __double2loint(v), hi = __double2hiint(v);
    const auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    return __hiloint2double(b[0], a[0]) + __hiloint2double(b[1], a[1]);
}
__device__ __forceinline__ double swap_sum16(double v) {
    const unsigned lo = __double2loint(v), hi = __double2hiint(v);
    const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    return __hiloint2double(b[0], a[0]) + __hiloint2double(b[1], a[1]);
}
__device__ __forceinline__ float swap_sum32(float v) {
    const unsigned u = __float_as_uint(v);
    const auto a = __builtin_amdgcn_permlane32_swap(u, u, false, false);
    return __uint_as_float(a[0]) + __uint_as_float(a[1]);
}
__device__ __forceinline__ float swap_sum16(float v) {
    const unsigned u = __float_as_uint(v);
    const auto a = __builtin_amdgcn_permlane16_swap(u, u, false, false);
    return __uint_as_float(a[0]) + __uint_as_float(a[1]);
}

// xor butterfly (offsets 32, 16, ..., 1): every lane ends with the
// bitwise-identical total, each step adding a lane's value and its
// partner's.
template <typename F>
__device__ __forceinline__ F wave_sum_t(F v) {
    v = swap_sum32(v);
    v = swap_sum16(v);
    v += dpp_lane<0x128>(v);                    // l ^ 8
    v += dpp_lane<0x1B>(dpp_lane<0x141>(v));    // l ^ 4
    v += dpp_lane<0x4E>(v);                     // l ^ 2
    v += dpp_lane<0xB1>(v);                     // l ^ 1
    return v;
}
__device__ __forceinline__ double wave_sum(double v) { return wave_sum_t(v); }
__device__ __forceinline__ float wave_sum(float v) { return wave_sum_t(v); }

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

// Data that crosses workgroups of a cooperative grid is written and read only
// with device-scope relaxed atomics.  On this chip family those write through
// and read around the per-XCD L2, so no device-scope fence (which writes back
// and invalidates the whole L2) is needed at a barrier: a thread drains its own
// stores with s_waitcnt before the workgroup announces its arrival.
__device__ __forceinline__ void xstore(double* p, double v) {
    __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), __double_as_longlong(v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double xload(const double* p) {
    return __longlong_as_double(__hip_atomic_load(reinterpret_cast<const unsigned long long*>(p), __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT));
}

// sum over b = first, first + step, ... < nb of xload(base + b * stride), added
// in that order (the same bits as a plain loop); four loads are in flight at
// once instead of one round trip per term.
__device__ __forceinline__ double xsum_strided(const double* base, long stride, int first, int step, int nb) {
    double s = 0.0;
    int b = first;
    for (; b + 3 * step < nb; b += 4 * step) {
        const double v0 = xload(base + (long)b * stride);
        const double v1 = xload(base + (long)(b + step) * stride);
        const double v2 = xload(base + (long)(b + 2 * step) * stride);
        const double v3 = xload(base + (long)(b + 3 * step) * stride);
        s += v0;
        s += v1;
        s += v2;
        s += v3;
    }
    for (; b < nb; b += step) s += xload(base + (long)b * stride);
    return s;
}

// A team is either one workgroup (size 1) or every workgroup of a
// cooperative launch.  Grid barrier: each workgroup publishes its arrival
// epoch in its own 128-byte line, workgroup 0 polls all of them in parallel
// and publishes the generation.  Every spin is bounded, so each wave exits
// even if a peer never arrives; the failure is flagged in bar[kBarErr] and
// reported by the host.
struct Team {
    int rank;
    int size;
    unsigned* bar;
    unsigned epoch;

    __device__ __forceinline__ bool spin_until(unsigned* a) const {
        unsigned spins = 0;
        while ((int)(__hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - epoch) < 0) {
            __builtin_amdgcn_s_sleep(1);
            ++spins;
            if ((spins & 1023u) == 0u &&
                __hip_atomic_load(&bar[kBarErr], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
                return false;   // another workgroup gave up
            if (spins > (1u << 23)) {   // far beyond any phase: a peer is gone
                __hip_atomic_store(&bar[kBarErr], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return false;
            }
        }
        return true;
    }

    // Returns true when the team must abort (barrier timeout seen).
    __device__ __forceinline__ bool sync() {
        if (size == 1) {
            __syncthreads();
            return false;
        }
        __shared__ int s_abort;
        __builtin_amdgcn_s_waitcnt(0);   // this thread's device-scope stores are complete
        __syncthreads();
        ++epoch;
        if (threadIdx.x == 0)
            __hip_atomic_store(&bar[kBarFlag + 32 * rank], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (rank == 0) {
            for (int b = threadIdx.x; b < size; b += blockDim.x) spin_until(&bar[kBarFlag + 32 * b]);
            __syncthreads();
            if (threadIdx.x == 0) __hip_atomic_store(&bar[0], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else if (threadIdx.x == 0) {
            spin_until(&bar[0]);
        }
        if (threadIdx.x == 0)
            s_abort = __hip_atomic_load(&bar[kBarErr], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
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
