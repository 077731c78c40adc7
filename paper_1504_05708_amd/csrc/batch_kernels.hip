// Kernel entry points of the batched forms: one workgroup per instance
// (batches and the serving loop) and MFMA tiles of 16 shared-Hessian
// instances.  Built for gfx950 only.
#include <hip/hip_runtime.h>

#include "batch.h"
#include "launch.h"
#include "launch_util.h"
#include "shared_tile.h"

namespace duq {

template <typename T, typename Acc, bool SHORT, bool SERVE>
__global__ void __launch_bounds__(256, 3) dfom_batch_kernel(BatchArgs<T> a) {
    extern __shared__ __align__(16) double lds[];
    batch_solve<T, Acc, SHORT, SERVE>(a, lds);
}

size_t batch_lds_bytes(int n_max, int p_max, int k) {
    return ((size_t)n_max + p_max + 1 + (size_t)(k + 2) + (size_t)kMaxWaves * kNP + 16 + kTlDoubles) *
           sizeof(double);
}

long long batch_slot_bytes_host(int n_max, int p_max, int k) { return batch_slot_bytes(n_max, p_max, k); }

template <bool SERVE>
static const void* batch_fn_t(int dtype, bool sh) {
    if (dtype == 0)
        return sh ? reinterpret_cast<const void*>(&dfom_batch_kernel<double, double, true, SERVE>)
                  : reinterpret_cast<const void*>(&dfom_batch_kernel<double, double, false, SERVE>);
    return sh ? reinterpret_cast<const void*>(&dfom_batch_kernel<float, double, true, SERVE>)
              : reinterpret_cast<const void*>(&dfom_batch_kernel<float, double, false, SERVE>);
}

static const void* batch_fn(int dtype, bool short_class, bool serve) {
    return serve ? batch_fn_t<true>(dtype, short_class) : batch_fn_t<false>(dtype, short_class);
}

bool batch_short_class(int dtype, int n) { return dtype == 0 ? short_rows<double>(n) : short_rows<float>(n); }

hipError_t batch_occupancy(int dtype, bool short_class, bool serve, size_t shmem, int* blocks_per_cu) {
    const void* f = batch_fn(dtype, short_class, serve);
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, f, 256, shmem);
}

// Count of non-finite entries of a device array (validation of borrowed data).
// Shared-Hessian tiles: eight waves, one workgroup per CU (Q fills the LDS).
template <typename T>
__global__ void __launch_bounds__(64 * kTileWaves, 1) dfom_tile_kernel(TileArgs<T> a) {
    extern __shared__ __align__(16) double lds[];
    tile_solve<T>(a, lds);
}

size_t tile_lds_bytes(int n) { return (size_t)tile_lds_doubles(n) * sizeof(double); }

static const void* tile_fn(int dtype) {
    return dtype == 0 ? reinterpret_cast<const void*>(&dfom_tile_kernel<double>)
                      : reinterpret_cast<const void*>(&dfom_tile_kernel<float>);
}

hipError_t tile_occupancy(int dtype, size_t shmem, int* blocks_per_cu) {
    const void* f = tile_fn(dtype);
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, f, 64 * kTileWaves, shmem);
}

hipError_t launch_tile(int dtype, int nblocks, size_t shmem, hipStream_t stream, const TileLaunch& t) {
    LaunchCfg cfg{nblocks, 64 * kTileWaves, shmem, false, stream};
    const void* f = tile_fn(dtype);
    if (dtype == 0) {
        TileArgs<double> a;
        fill_tile_args(a, t);
        void* args[] = {&a};
        return launch_fn(f, cfg, args);
    }
    TileArgs<float> a;
    fill_tile_args(a, t);
    void* args[] = {&a};
    return launch_fn(f, cfg, args);
}

hipError_t launch_batch(int dtype, bool short_class, int nblocks, size_t shmem, hipStream_t stream,
                        const BatchLaunch& b) {
    LaunchCfg cfg{nblocks, 256, shmem, false, stream};
    const void* f = batch_fn(dtype, short_class, b.inst != nullptr);
    if (dtype == 0) {
        BatchArgs<double> a;
        fill_batch_args(a, b);
        void* args[] = {&a};
        return launch_fn(f, cfg, args);
    }
    BatchArgs<float> a;
    fill_batch_args(a, b);
    void* args[] = {&a};
    return launch_fn(f, cfg, args);
}

}  // namespace duq
