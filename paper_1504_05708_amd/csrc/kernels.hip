// Kernel entry points and launch helpers of the single-QP DFOM solver, the
// Lanczos constant estimate and data validation.  Built for gfx950 only.
#include <hip/hip_runtime.h>

#include "dfom_solver.h"
#include "lanczos.h"
#include "launch.h"
#include "launch_util.h"

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

template <typename T, typename Acc, bool SHORT, bool ROWS, bool SPARSE = false>
__global__ void __launch_bounds__(512) dfom_kernel(DevProblem<T> P, DevParams par, DevWork W) {
    extern __shared__ __align__(16) double lds[];
    Dfom<T, Acc, SHORT, ROWS, SPARSE> s;
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
    const int xn = (SPARSE && par.x_global) ? 0 : P.n;   // x read in place: no LDS copy
    s.xl = lds;
    s.xsrc = nullptr;
    s.vl = lds + xn;
    s.red = lds + xn + pmax;
    s.tl = s.red + kMaxWaves * kNP + 2;
    s.run();
}

template <typename T, bool SHORT, bool SPARSE = false>
__global__ void __launch_bounds__(512) lanczos_kernel(DevProblem<T> P, LanczosWork L, int k, int use_gtg) {
    extern __shared__ __align__(16) double lds[];
    Lanczos<T, SHORT, SPARSE> s;
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
    const int xn = (SPARSE && L.x_global) ? 0 : P.n;
    s.xl = lds;
    s.vl = lds + xn;
    s.hl = lds + xn + pmax;
    s.red = s.hl + (k + 2);
    s.tl = s.red + kMaxWaves * 2 + 2;
    s.run();
}

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

// H = Q + rho G^T G, 64 x 64 output tiles per workgroup of 256 threads (4 x 4
// outputs per thread), G staged in LDS 16 rows at a time; each entry sums
// over the rows of G in ascending order in FP64, so the result does not depend
// on the launch.
template <typename T>
__global__ void __launch_bounds__(256) form_hessian_kernel(int n, int p, const T* __restrict__ Q,
                                                           const T* __restrict__ G, double rho, T* __restrict__ H) {
    constexpr int TB = 64, KB = 16;
    __shared__ double gi[KB][TB + 1];
    __shared__ double gj[KB][TB + 1];
    const int i0 = blockIdx.y * TB, j0 = blockIdx.x * TB;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    for (int k0 = 0; k0 < p; k0 += KB) {
        for (int e = threadIdx.x; e < KB * TB; e += blockDim.x) {
            const int kr = e / TB, c = e % TB;
            const int k = k0 + kr;
            gi[kr][c] = (k < p && i0 + c < n) ? (double)G[(long)k * n + i0 + c] : 0.0;
            gj[kr][c] = (k < p && j0 + c < n) ? (double)G[(long)k * n + j0 + c] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int kr = 0; kr < KB; ++kr) {
            double a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = gi[kr][ty * 4 + u];
                b[u] = gj[kr][tx * 4 + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int i = i0 + ty * 4 + u;
        if (i >= n) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int j = j0 + tx * 4 + v;
            if (j < n) H[(long)i * n + j] = (T)((double)Q[(long)i * n + j] + rho * acc[u][v]);
        }
    }
}

hipError_t launch_form_hessian(int dtype, int n, int p, const void* Q, const void* G, double rho, void* H,
                               hipStream_t s) {
    const dim3 grid((n + 63) / 64, (n + 63) / 64);
    if (dtype == 0)
        hipLaunchKernelGGL(form_hessian_kernel<double>, grid, dim3(256), 0, s, n, p, (const double*)Q,
                           (const double*)G, rho, (double*)H);
    else
        hipLaunchKernelGGL(form_hessian_kernel<float>, grid, dim3(256), 0, s, n, p, (const float*)Q,
                           (const float*)G, rho, (float*)H);
    return hipGetLastError();
}

// x_global: sparse data whose x is read in place (no n-vector in LDS).
size_t dfom_lds_bytes(int n, int p, int nblocks, bool x_global) {
    return solver_lds_doubles(x_global ? 0 : n, p, nblocks) * sizeof(double);
}
size_t lanczos_lds_bytes(int n, int p, int nblocks, int k, bool x_global) {
    return lanczos_lds_doubles(x_global ? 0 : n, p, nblocks, k) * sizeof(double);
}

template <bool SHORT>
static const void* dfom_fn_t(int dtype, int acc, bool rows = false) {
    // row bounds: FP64 accumulation only (the precision switch is not offered)
    if (rows)
        return dtype == 0 ? reinterpret_cast<const void*>(&dfom_kernel<double, double, SHORT, true>)
                          : reinterpret_cast<const void*>(&dfom_kernel<float, double, SHORT, true>);
    if (dtype == 0) return reinterpret_cast<const void*>(&dfom_kernel<double, double, SHORT, false>);
    if (acc == 0) return reinterpret_cast<const void*>(&dfom_kernel<float, double, SHORT, false>);
    return reinterpret_cast<const void*>(&dfom_kernel<float, float, SHORT, false>);
}

// Compressed-row Q and G: one variant per storage type, row form and
// accumulation (the row length does not select a product shape).
static const void* dfom_fn_sparse(int dtype, int acc, bool rows) {
    if (rows)
        return dtype == 0 ? reinterpret_cast<const void*>(&dfom_kernel<double, double, false, true, true>)
                          : reinterpret_cast<const void*>(&dfom_kernel<float, double, false, true, true>);
    if (dtype == 0) return reinterpret_cast<const void*>(&dfom_kernel<double, double, false, false, true>);
    if (acc == 0) return reinterpret_cast<const void*>(&dfom_kernel<float, double, false, false, true>);
    return reinterpret_cast<const void*>(&dfom_kernel<float, float, false, false, true>);
}

static const void* dfom_fn(int dtype, int acc, int n, bool rows = false, bool sparse = false) {
    if (sparse) return dfom_fn_sparse(dtype, acc, rows);
    const bool sh = dtype == 0 ? short_rows<double>(n) : short_rows<float>(n);
    return sh ? dfom_fn_t<true>(dtype, acc, rows) : dfom_fn_t<false>(dtype, acc, rows);
}

size_t dfom_static_lds_bytes() {
    static size_t bytes = [] {
        const void* fns[] = {dfom_fn_t<true>(0, 0), dfom_fn_t<true>(1, 0), dfom_fn_t<true>(1, 1),
                             dfom_fn_t<false>(0, 0), dfom_fn_t<false>(1, 0), dfom_fn_t<false>(1, 1),
                             dfom_fn_t<true>(0, 0, true), dfom_fn_t<true>(1, 0, true),
                             dfom_fn_t<false>(0, 0, true), dfom_fn_t<false>(1, 0, true),
                             reinterpret_cast<const void*>(&lanczos_kernel<double, true>),
                             reinterpret_cast<const void*>(&lanczos_kernel<double, false>),
                             reinterpret_cast<const void*>(&lanczos_kernel<float, true>),
                             reinterpret_cast<const void*>(&lanczos_kernel<float, false>),
                             dfom_fn_sparse(0, 0, false), dfom_fn_sparse(1, 0, false), dfom_fn_sparse(1, 1, false),
                             dfom_fn_sparse(0, 0, true), dfom_fn_sparse(1, 0, true),
                             reinterpret_cast<const void*>(&lanczos_kernel<double, false, true>),
                             reinterpret_cast<const void*>(&lanczos_kernel<float, false, true>)};
        size_t m = 0;
        for (const void* f : fns) {
            hipFuncAttributes a;
            // unknown: reserve a small margin rather than none
            m = std::max(m, hipFuncGetAttributes(&a, f) == hipSuccess ? (size_t)a.sharedSizeBytes : (size_t)256);
        }
        return m;
    }();
    return bytes;
}

hipError_t dfom_occupancy(int dtype, int acc, int n, int nthreads, size_t shmem, int* blocks_per_cu, bool rows,
                          bool sparse) {
    const void* f = dfom_fn(dtype, acc, n, rows, sparse);
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, f, nthreads, shmem);
}

template <typename T>
static void set_sparse(DevProblem<T>& P, const SparseRefs& s) {
    P.Qrp = s.Qrp;
    P.Qci = s.Qci;
    P.Qv = static_cast<const T*>(s.Qv);
    P.Grp = s.Grp;
    P.Gci = s.Gci;
    P.Gv = static_cast<const T*>(s.Gv);
    P.Trp = s.Trp;
    P.Tci = s.Tci;
    P.Tv = static_cast<const T*>(s.Tv);
    P.Qlg = s.Qlg;
    P.Glg = s.Glg;
    P.Tlg = s.Tlg;
}

hipError_t launch_dfom(int dtype, int acc, const LaunchCfg& cfg, const GenericProblem& gp,
                       const DevParams& par, const DevWork& W) {
    DevParams pr = par;
    DevWork w = W;
    const bool rows = gp.rlo != nullptr;
    const void* f = dfom_fn(dtype, acc, gp.n, rows, gp.sp.Qrp != nullptr);
    if (dtype == 0) {
        DevProblem<double> P{gp.n, gp.p, (const double*)gp.Q, (const double*)gp.G, gp.q, gp.g, gp.lb, gp.ub,
                             gp.rlo, gp.rhi};
        set_sparse(P, gp.sp);
        void* args[] = {&P, &pr, &w};
        return launch_fn(f, cfg, args);
    }
    DevProblem<float> P{gp.n, gp.p, (const float*)gp.Q, (const float*)gp.G, gp.q, gp.g, gp.lb, gp.ub,
                        gp.rlo, gp.rhi};
    set_sparse(P, gp.sp);
    void* args[] = {&P, &pr, &w};
    return launch_fn(f, cfg, args);
}

hipError_t launch_lanczos(int dtype, const LaunchCfg& cfg, const GenericProblem& gp, const LanczosWork& L,
                          int k, int use_gtg) {
    LanczosWork l = L;
    int kk = k, ug = use_gtg;
    if (dtype == 0) {
        DevProblem<double> P{gp.n, gp.p, (const double*)gp.Q, (const double*)gp.G, gp.q, gp.g, gp.lb, gp.ub,
                             gp.rlo, gp.rhi};
        set_sparse(P, gp.sp);
        void* args[] = {&P, &l, &kk, &ug};
        const void* f = gp.sp.Qrp ? reinterpret_cast<const void*>(&lanczos_kernel<double, false, true>)
                        : short_rows<double>(gp.n) ? reinterpret_cast<const void*>(&lanczos_kernel<double, true>)
                                                   : reinterpret_cast<const void*>(&lanczos_kernel<double, false>);
        return launch_fn(f, cfg, args);
    }
    DevProblem<float> P{gp.n, gp.p, (const float*)gp.Q, (const float*)gp.G, gp.q, gp.g, gp.lb, gp.ub,
                        gp.rlo, gp.rhi};
    set_sparse(P, gp.sp);
    void* args[] = {&P, &l, &kk, &ug};
    const void* f = gp.sp.Qrp ? reinterpret_cast<const void*>(&lanczos_kernel<float, false, true>)
                    : short_rows<float>(gp.n) ? reinterpret_cast<const void*>(&lanczos_kernel<float, true>)
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

}  // namespace duq
