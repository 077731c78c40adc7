// Kernel entry points and launch helpers for the DFOM solver and the
// Lanczos constant estimate.  Built for gfx950 only.
#include <hip/hip_runtime.h>

#include "batch.h"
#include "dfom_solver.h"
#include "shared_tile.h"
#include "lanczos.h"
#include "launch.h"

namespace duq {

// LDS layout of the solver: [x staged (n)] [owned p rows (pmax)] [reduction scratch].
static size_t solver_lds_doubles(int n, int p, int nblocks) {
    const int pmax = (p + nblocks - 1) / nblocks + 1;
    return (size_t)n + (size_t)pmax + (size_t)kMaxWaves * kNP + 2 + kTlDoubles;
}

static size_t lanczos_lds_doubles(int n, int p, int nblocks, int k) {
    const int pmax = (p + nblocks - 1) / nblocks + 1;
    return (size_t)n + (size_t)pmax + (size_t)(k + 2) + (size_t)kMaxWaves * 2 + 2 + kTlDoubles;
}

template <typename T, typename Acc, bool SHORT>
__global__ void __launch_bounds__(512) dfom_kernel(DevProblem<T> P, DevParams par, DevWork W) {
    extern __shared__ __align__(16) double lds[];
    Dfom<T, Acc, SHORT> s;
    s.P = P;
    s.par = par;
    s.W = W;
    s.tm.rank = blockIdx.x;
    s.tm.size = gridDim.x;
    s.tm.bar = W.bar;
    s.tm.epoch = 0;
    share(P.n, blockIdx.x, gridDim.x, s.nlo, s.nhi);
    share(P.p, blockIdx.x, gridDim.x, s.plo, s.phi);
    const int pmax = (P.p + gridDim.x - 1) / gridDim.x + 1;
    s.xl = lds;
    s.vl = lds + P.n;
    s.red = lds + P.n + pmax;
    s.tl = s.red + kMaxWaves * kNP + 2;
    s.run();
}

template <typename T, bool SHORT>
__global__ void __launch_bounds__(512) lanczos_kernel(DevProblem<T> P, LanczosWork L, int k, int use_gtg) {
    extern __shared__ __align__(16) double lds[];
    Lanczos<T, SHORT> s;
    s.P = P;
    s.L = L;
    s.k = k;
    s.use_gtg = use_gtg;
    s.tm.rank = blockIdx.x;
    s.tm.size = gridDim.x;
    s.tm.bar = L.bar;
    s.tm.epoch = 0;
    share(P.n, blockIdx.x, gridDim.x, s.nlo, s.nhi);
    share(P.p, blockIdx.x, gridDim.x, s.plo, s.phi);
    const int pmax = (P.p + gridDim.x - 1) / gridDim.x + 1;
    s.xl = lds;
    s.vl = lds + P.n;
    s.hl = lds + P.n + pmax;
    s.red = s.hl + (k + 2);
    s.tl = s.red + kMaxWaves * 2 + 2;
    s.run();
}

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
template <typename T>
__global__ void count_nonfinite_kernel(const T* a, long len, unsigned* out) {
    unsigned c = 0;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < len; i += (long)gridDim.x * blockDim.x) {
        const double v = (double)a[i];
        c += !(v - v == 0.0);
    }
    for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off, kWave);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, c);
}

static hipError_t launch_fn(const void* kernel, const LaunchCfg& cfg, void** args) {
    const size_t shmem = cfg.shmem;
    hipError_t e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (e != hipSuccess) return e;
    if (cfg.cooperative)
        return hipLaunchCooperativeKernel(kernel, dim3(cfg.nblocks), dim3(cfg.nthreads), args, shmem, cfg.stream);
    return hipLaunchKernel(kernel, dim3(cfg.nblocks), dim3(cfg.nthreads), args, shmem, cfg.stream);
}


// Shared-Hessian tiles: four waves, one workgroup per CU (Q fills the LDS).
template <typename T>
__global__ void __launch_bounds__(256, 1) dfom_tile_kernel(TileArgs<T> a) {
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
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, f, 256, shmem);
}

hipError_t launch_tile(int dtype, int nblocks, size_t shmem, hipStream_t stream, const TileLaunch& t) {
    LaunchCfg cfg{nblocks, 256, shmem, false, stream};
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

size_t dfom_lds_bytes(int n, int p, int nblocks) { return solver_lds_doubles(n, p, nblocks) * sizeof(double); }
size_t lanczos_lds_bytes(int n, int p, int nblocks, int k) {
    return lanczos_lds_doubles(n, p, nblocks, k) * sizeof(double);
}

template <bool SHORT>
static const void* dfom_fn_t(int dtype, int acc) {
    if (dtype == 0) return reinterpret_cast<const void*>(&dfom_kernel<double, double, SHORT>);
    if (acc == 0) return reinterpret_cast<const void*>(&dfom_kernel<float, double, SHORT>);
    return reinterpret_cast<const void*>(&dfom_kernel<float, float, SHORT>);
}

static const void* dfom_fn(int dtype, int acc, int n) {
    const bool sh = dtype == 0 ? short_rows<double>(n) : short_rows<float>(n);
    return sh ? dfom_fn_t<true>(dtype, acc) : dfom_fn_t<false>(dtype, acc);
}

hipError_t dfom_occupancy(int dtype, int acc, int n, int nthreads, size_t shmem, int* blocks_per_cu) {
    const void* f = dfom_fn(dtype, acc, n);
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, f, nthreads, shmem);
}

hipError_t launch_dfom(int dtype, int acc, const LaunchCfg& cfg, const GenericProblem& gp,
                       const DevParams& par, const DevWork& W) {
    DevParams pr = par;
    DevWork w = W;
    const void* f = dfom_fn(dtype, acc, gp.n);
    if (dtype == 0) {
        DevProblem<double> P{gp.n, gp.p, (const double*)gp.Q, (const double*)gp.G, gp.q, gp.g, gp.lb, gp.ub};
        void* args[] = {&P, &pr, &w};
        return launch_fn(f, cfg, args);
    }
    DevProblem<float> P{gp.n, gp.p, (const float*)gp.Q, (const float*)gp.G, gp.q, gp.g, gp.lb, gp.ub};
    void* args[] = {&P, &pr, &w};
    return launch_fn(f, cfg, args);
}

hipError_t launch_lanczos(int dtype, const LaunchCfg& cfg, const GenericProblem& gp, const LanczosWork& L,
                          int k, int use_gtg) {
    LanczosWork l = L;
    int kk = k, ug = use_gtg;
    if (dtype == 0) {
        DevProblem<double> P{gp.n, gp.p, (const double*)gp.Q, (const double*)gp.G, gp.q, gp.g, gp.lb, gp.ub};
        void* args[] = {&P, &l, &kk, &ug};
        const void* f = short_rows<double>(gp.n) ? reinterpret_cast<const void*>(&lanczos_kernel<double, true>)
                                                 : reinterpret_cast<const void*>(&lanczos_kernel<double, false>);
        return launch_fn(f, cfg, args);
    }
    DevProblem<float> P{gp.n, gp.p, (const float*)gp.Q, (const float*)gp.G, gp.q, gp.g, gp.lb, gp.ub};
    void* args[] = {&P, &l, &kk, &ug};
    const void* f = short_rows<float>(gp.n) ? reinterpret_cast<const void*>(&lanczos_kernel<float, true>)
                                            : reinterpret_cast<const void*>(&lanczos_kernel<float, false>);
    return launch_fn(f, cfg, args);
}

hipError_t launch_count_nonfinite(int dtype, const void* a, long len, unsigned* out, hipStream_t s) {
    const int nb = (int)std::min<long>(1024, (len + 255) / 256 + 1);
    if (dtype == 0)
        hipLaunchKernelGGL(count_nonfinite_kernel<double>, dim3(nb), dim3(256), 0, s, (const double*)a, len, out);
    else
        hipLaunchKernelGGL(count_nonfinite_kernel<float>, dim3(nb), dim3(256), 0, s, (const float*)a, len, out);
    return hipGetLastError();
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
