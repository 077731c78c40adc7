// Serving through the MFMA tiles: gather of the requests' linear terms into
// the tile kernel's contiguous arrays and scatter of its outputs.  Built for
// gfx950 only.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "launch.h"

namespace duq {

// Serving through the tiles: the q, g of B requests against one shared
// system into contiguous B x n and B x p arrays (one workgroup per request),
// and the tile outputs back to each request's x and lambda.
__global__ void __launch_bounds__(256) serve_gather_kernel(const ServeInst* inst, int n, int p, double* q,
                                                           double* g) {
    const ServeInst& si = inst[blockIdx.x];
    for (int i = threadIdx.x; i < n; i += blockDim.x) q[(long)blockIdx.x * n + i] = si.q[i];
    for (int i = threadIdx.x; i < p; i += blockDim.x) g[(long)blockIdx.x * p + i] = si.g[i];
}

__global__ void __launch_bounds__(256) serve_scatter_kernel(const ServeInst* inst, int n, int p, const double* X,
                                                            const double* Lam) {
    const ServeInst& si = inst[blockIdx.x];
    for (int i = threadIdx.x; i < n; i += blockDim.x) si.x[i] = X[(long)blockIdx.x * n + i];
    for (int i = threadIdx.x; i < p; i += blockDim.x) si.lam[i] = Lam[(long)blockIdx.x * p + i];
}

hipError_t launch_serve_gather(const ServeInst* inst, int B, int n, int p, double* q, double* g, hipStream_t s) {
    if (B <= 0) return hipSuccess;
    hipLaunchKernelGGL(serve_gather_kernel, dim3(B), dim3(256), 0, s, inst, n, p, q, g);
    return hipGetLastError();
}

hipError_t launch_serve_scatter(const ServeInst* inst, int B, int n, int p, const double* X, const double* Lam,
                                hipStream_t s) {
    if (B <= 0) return hipSuccess;
    hipLaunchKernelGGL(serve_scatter_kernel, dim3(B), dim3(256), 0, s, inst, n, p, X, Lam);
    return hipGetLastError();
}

}  // namespace duq
