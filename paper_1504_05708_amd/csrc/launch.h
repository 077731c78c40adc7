// Host-side launch interface between the runtime (duq_api.cpp) and kernels.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include <type_traits>

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
    const double* rlo = nullptr;   // row bounds (both or neither)
    const double* rhi = nullptr;
    SparseRefs sp;                 // compressed-row Q, G, G^T (sp.Qrp null: dense)
};

struct LanczosWork;

// Type-erased batch description filled by the host runtime.
struct BatchLaunch {
    int B, shared;
    const int* order;
    const int* n;
    const int* p;
    const long long *qoff, *goff, *voff, *coff;
    int n_shared, p_shared;
    const void* Q;
    const void* G;
    const double *q, *g, *lb, *ub;
    const double *lam_min, *lam_max, *g2;
    double* X;
    double* Lam;
    void* res;
    const ServeInst* inst;
    int slice;
    DevParams base;
    int max_inner, lanczos_k, lanczos_alloc;
    double safety;
    char* slots;
    long long slot_bytes;
    int n_max, p_max;
    unsigned* queue;
};

template <typename A>
inline void fill_batch_args(A& a, const BatchLaunch& b) {
    typedef typename std::remove_const<typename std::remove_pointer<decltype(a.Q)>::type>::type T;
    a.B = b.B; a.shared = b.shared; a.order = b.order; a.n = b.n; a.p = b.p;
    a.qoff = b.qoff; a.goff = b.goff; a.voff = b.voff; a.coff = b.coff;
    a.n_shared = b.n_shared; a.p_shared = b.p_shared;
    a.Q = (const T*)b.Q; a.G = (const T*)b.G;
    a.q = b.q; a.g = b.g; a.lb = b.lb; a.ub = b.ub;
    a.lam_min = b.lam_min; a.lam_max = b.lam_max; a.g2 = b.g2;
    a.X = b.X; a.Lam = b.Lam; a.res = (decltype(a.res))b.res;
    a.inst = b.inst; a.slice = b.slice;
    a.base = b.base; a.max_inner = b.max_inner; a.lanczos_k = b.lanczos_k; a.lanczos_alloc = b.lanczos_alloc; a.safety = b.safety;
    a.slots = b.slots; a.slot_bytes = b.slot_bytes; a.n_max = b.n_max; a.p_max = b.p_max; a.queue = b.queue;
}

size_t batch_lds_bytes(int n_max, int p_max, int k);
long long batch_slot_bytes_host(int n_max, int p_max, int k);
// Instances with short_rows(n) run in the short-row kernel, the others in the
// long-row kernel; `serve` selects the serving instantiation (b.inst set).
bool batch_short_class(int dtype, int n);
hipError_t batch_occupancy(int dtype, bool short_class, bool serve, size_t shmem, int* blocks_per_cu);
hipError_t launch_batch(int dtype, bool short_class, int nblocks, size_t shmem, hipStream_t stream,
                        const BatchLaunch& b);

// Shared-Hessian batch on FP64 MFMA tiles of 16 instances (type-erased TileArgs).
struct TileLaunch {
    int B, n, p;
    const void* Q;
    const void* G;
    const double *q, *g, *lb, *ub;
    double* X;
    double* Lam;
    void* res;
    double* dual;
    double* prim;
    DevParams par;
    double lam_min, lam_max, g2;
    unsigned* queue;
};

template <typename A>
inline void fill_tile_args(A& a, const TileLaunch& t) {
    typedef typename std::remove_const<typename std::remove_pointer<decltype(a.Q)>::type>::type T;
    a.B = t.B; a.n = t.n; a.p = t.p;
    a.Q = (const T*)t.Q; a.G = (const T*)t.G;
    a.q = t.q; a.g = t.g; a.lb = t.lb; a.ub = t.ub;
    a.X = t.X; a.Lam = t.Lam; a.res = (decltype(a.res))t.res;
    a.dual = t.dual; a.prim = t.prim; a.par = t.par;
    a.lam_min = t.lam_min; a.lam_max = t.lam_max; a.g2 = t.g2; a.queue = t.queue;
}

constexpr int kTileMaxN = 128;   // two row tiles of 16 per wave
size_t tile_lds_bytes(int n);
// Serving: q, g of the requests in `inst` (device table) gathered into B x n
// and B x p arrays; X, Lam (B x n, B x p) scattered to the requests' x, lambda.
hipError_t launch_serve_gather(const ServeInst* inst, int B, int n, int p, double* q, double* g, hipStream_t s);
hipError_t launch_serve_scatter(const ServeInst* inst, int B, int n, int p, const double* X, const double* Lam,
                                hipStream_t s);
hipError_t tile_occupancy(int dtype, size_t shmem, int* blocks_per_cu);
hipError_t launch_tile(int dtype, int nblocks, size_t shmem, hipStream_t stream, const TileLaunch& t);

size_t dfom_lds_bytes(int n, int p, int nblocks, bool x_global = false);
// Static LDS of the solver and Lanczos kernels (largest instantiation); the
// dynamic LDS of a launch may use what is left of the workgroup's LDS.
size_t dfom_static_lds_bytes();
size_t lanczos_lds_bytes(int n, int p, int nblocks, int k, bool x_global = false);
hipError_t dfom_occupancy(int dtype, int acc, int n, int nthreads, size_t shmem, int* blocks_per_cu,
                          bool rows = false, bool sparse = false);
hipError_t launch_dfom(int dtype, int acc, const LaunchCfg& cfg, const GenericProblem& gp,
                       const DevParams& par, const DevWork& W);
hipError_t launch_lanczos(int dtype, const LaunchCfg& cfg, const GenericProblem& gp, const LanczosWork& L,
                          int k, int use_gtg);
hipError_t launch_count_nonfinite(int dtype, const void* a, long len, unsigned* out, hipStream_t s);
// H = Q + rho G^T G (n x n, dtype of Q and G, FP64 accumulation): the constant
// inner Hessian of a problem whose rows are all equalities (Sec. 5.1).
hipError_t launch_form_hessian(int dtype, int n, int p, const void* Q, const void* G, double rho, void* H,
                               hipStream_t s);

}  // namespace duq
