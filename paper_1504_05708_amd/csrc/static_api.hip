// duq_solve_static: one DFOM solve of a device-resident QP whose workspace
// lives in a static device array instead of memory the library allocates.
// It is for callers that cannot call hipMalloc (code under HIP graph capture,
// tight serving loops, harnesses that forbid allocation).  The kernels are the
// ones duq_solve launches; only where their workspace lives differs.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "../../include/duq.h"
#include "device_common.h"
#include "internal.h"
#include "launch.h"
#include "workspace.h"

namespace duq {
int set_error(int code, const std::string& msg);
int device_shape(int* cus, size_t* lds_max);
int validate_problem(const duq_problem* pr, const duq_options* o);
int derive_params(int p, double lam_min, double lam_max, double g2, double D_U, const duq_options& o,
                  DevParams* par, double sigma);

// The scratch array, one copy per GPU for the life of the process.  Host code
// never passes its name to a kernel: it takes the device address of this
// GPU's copy from hipGetSymbolAddress (scratch_base) and uses that.
constexpr size_t kScratchHeader = 256;   // validation results
static __device__ __align__(256) char scratch[DUQ_STATIC_SCRATCH_BYTES];

// Zero `nwords` 32-bit words (a fill kernel rather than a memset node, so the
// call can be captured into a graph).
__global__ void zero_words_kernel(unsigned* p, long nwords) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < nwords; i += (long)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// One workgroup: the squared box diameter D_U^2 (fixed-order block sum) and
// the count of box entries that are non-finite or have lb > ub, plus
// non-finite q and g entries.  Results: hdr[0] (double) and hdr[1] (count).
__global__ void __launch_bounds__(256) check_vectors_kernel(const double* q, const double* g, const double* lb,
                                                            const double* ub, int n, int p, double* hdr) {
    __shared__ double red[kMaxWaves * 2];
    double v[2] = {0.0, 0.0};
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double lo = lb[i], hi = ub[i], qi = q[i];
        const bool ok = (lo - lo == 0.0) && (hi - hi == 0.0) && (qi - qi == 0.0) && lo <= hi;
        v[0] += ok ? (hi - lo) * (hi - lo) : 0.0;
        v[1] += ok ? 0.0 : 1.0;
    }
    for (int i = threadIdx.x; i < p; i += blockDim.x) v[1] += (g[i] - g[i] == 0.0) ? 0.0 : 1.0;
    block_allreduce<2>(v, red);
    if (threadIdx.x == 0) {
        hdr[0] = v[0];
        hdr[1] = v[1];
    }
}

namespace {

std::mutex g_scratch_mu;
char* g_scratch_ptr[64];

// Device address of this GPU's copy of `scratch`, looked up once per device
// with that device current.
int scratch_base(char** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(DUQ_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= 64) return set_error(DUQ_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(DUQ_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<char*>(p);
    }
    *out = g_scratch_ptr[dev];
    return DUQ_OK;
}

hipError_t zero_words(unsigned* p, long nwords, hipStream_t s) {
    const int nb = (int)std::min<long>(1024, (nwords + 255) / 256 + 1);
    hipLaunchKernelGGL(zero_words_kernel, dim3(nb), dim3(256), 0, s, p, nwords);
    return hipGetLastError();
}

}  // namespace
}  // namespace duq

using namespace duq;

#define HIP_OK(expr, what)                                                                      \
    do {                                                                                        \
        hipError_t _e = (expr);                                                                 \
        if (_e != hipSuccess) return set_error(DUQ_EDEVICE, std::string(what) + ": " + hipGetErrorString(_e)); \
    } while (0)

extern "C" int duq_solve_static(const duq_problem* pr, const duq_options* o, void* stream, double* x_out,
                                double* lam_out, duq_result* res) {
    if (int rc = validate_problem(pr, o)) return rc;
    if (pr->memspace != DUQ_DEVICE) return set_error(DUQ_EINVAL, "duq_solve_static: the problem must be DEVICE data");
    if (pr->rlo || pr->rhi) return set_error(DUQ_EINVAL, "duq_solve_static: row bounds are not available here");
    if (!x_out || (pr->p > 0 && !lam_out)) return set_error(DUQ_EINVAL, "duq_solve_static: null x_out or lam_out");
    if (o->trace_outer != 0 || o->accumulate != DUQ_ACC_F64)
        return set_error(DUQ_EINVAL, "duq_solve_static: tracing and the precision switch are not available");
    const int n = pr->n, p = pr->p, dtype = pr->dtype;
    if (!(o->lam_min > 0.0 || (o->rho > 0.0 && o->lam_min == 0.0)) || !(o->lam_max > 0.0) ||
        (p > 0 && !(o->G_norm2 > 0.0)) || !std::isfinite(o->lam_min) || !std::isfinite(o->lam_max) ||
        !std::isfinite(o->G_norm2))
        return set_error(DUQ_EINVAL, "duq_solve_static: lam_min, lam_max and G_norm2 must be given (finite, > 0)");
    hipStream_t s = (hipStream_t)stream;

    // launch shape, as duq_setup chooses it
    int cus = 1;
    size_t lds_max = 0;
    if (int rc = device_shape(&cus, &lds_max)) return rc;
    int engine = o->engine;
    if (engine == DUQ_ENGINE_AUTO) engine = (n <= 1536) ? DUQ_ENGINE_BLOCK : DUQ_ENGINE_GRID;
    if (engine != DUQ_ENGINE_BLOCK && engine != DUQ_ENGINE_GRID)
        return set_error(DUQ_EINVAL, "duq_solve_static: engine must be AUTO, BLOCK or GRID");
    LaunchCfg cfg{};
    cfg.nblocks = engine == DUQ_ENGINE_BLOCK ? 1 : std::max(1, std::min(cus, n));
    cfg.nthreads = engine == DUQ_ENGINE_BLOCK ? (n <= 128 ? 256 : 512) : 512;
    cfg.cooperative = engine == DUQ_ENGINE_GRID;
    cfg.stream = s;
    cfg.shmem = dfom_lds_bytes(n, p, cfg.nblocks);
    if (cfg.shmem > lds_max)
        return set_error(DUQ_EINVAL, "duq_solve_static: n = " + std::to_string(n) +
                                         " too large for the LDS-staged products (see duq_max_n)");
    if (cfg.cooperative) {
        int bpc = 0;
        if (dfom_occupancy(dtype, 0, n, cfg.nthreads, cfg.shmem, &bpc) != hipSuccess || bpc < 1)
            return set_error(DUQ_EDEVICE, "cooperative launch does not fit one block per CU");
    }

    // workspace inside the scratch array
    Carve measure;
    DevWork W{};
    double *xstage = nullptr, *lstage = nullptr;
    carve_solver(measure, n, p, cfg.nblocks, 0, &W, &xstage, &lstage);
    if (kScratchHeader + measure.off > (size_t)DUQ_STATIC_SCRATCH_BYTES)
        return set_error(DUQ_EINVAL, "duq_solve_static: the workspace (" + std::to_string(measure.off) +
                                         " bytes for n = " + std::to_string(n) + ", p = " + std::to_string(p) +
                                         ") exceeds the static scratch of " +
                                         std::to_string((size_t)DUQ_STATIC_SCRATCH_BYTES) + " bytes");
    char* base = nullptr;
    if (int rc = scratch_base(&base)) return rc;
    double* hdr = reinterpret_cast<double*>(base);
    Carve c;
    c.base = base + kScratchHeader;
    carve_solver(c, n, p, cfg.nblocks, 0, &W, &xstage, &lstage);

    // what must start at zero: the header, the solver state and the barrier words
    HIP_OK(zero_words(reinterpret_cast<unsigned*>(base), kScratchHeader / 4, s), "clear");
    HIP_OK(zero_words(reinterpret_cast<unsigned*>(W.st), sizeof(DevState) / 4, s), "clear");
    HIP_OK(zero_words(W.bar, bar_words(cfg.nblocks), s), "clear");

    // borrowed data: box diameter and validity on the device; non-finite Q, G
    // entries counted into the header's third word
    hipLaunchKernelGGL(check_vectors_kernel, dim3(1), dim3(256), 0, s, pr->q, p ? pr->g : pr->q, pr->lb, pr->ub, n,
                       p, hdr);
    HIP_OK(hipGetLastError(), "validation");
    unsigned* cnt = reinterpret_cast<unsigned*>(base + 2 * sizeof(double));
    HIP_OK(launch_count_nonfinite(dtype, pr->Q, (long)n * n, cnt, s), "validation");
    if (p > 0) HIP_OK(launch_count_nonfinite(dtype, pr->G, (long)p * n, cnt, s), "validation");
    struct {
        double du2, bad;
        unsigned cnt, pad;
    } chk{};
    HIP_OK(hipMemcpyAsync(&chk, base, sizeof(chk), hipMemcpyDeviceToHost, s), "validation copy");
    HIP_OK(hipStreamSynchronize(s), "validation");
    if (chk.bad != 0.0 || chk.cnt != 0)
        return set_error(DUQ_EINVAL, "duq_solve_static: non-finite data or lb > ub");

    DevParams par{};
    if (int rc = derive_params(p, o->lam_min, o->lam_max, p > 0 ? o->G_norm2 : 0.0, std::sqrt(chk.du2), *o, &par,
                               o->sigma_in))
        return rc;
    par.trace_iters = 0;
    par.has_x0 = 0;
    par.has_lam0 = 0;
    par.resume = 0;
    W.xout = x_out;
    W.x0 = xstage;
    W.lam0 = lstage;
    GenericProblem gp{n, p, pr->Q, pr->G, pr->q, pr->g, pr->lb, pr->ub};
    HIP_OK(launch_dfom(dtype, 0, cfg, gp, par, W), "solver launch");
    if (p > 0) HIP_OK(hipMemcpyAsync(lam_out, W.lamp, p * sizeof(double), hipMemcpyDeviceToDevice, s), "lam copy");
    DevState st{};
    unsigned bar_err = 0;
    HIP_OK(hipMemcpyAsync(&st, W.st, sizeof(DevState), hipMemcpyDeviceToHost, s), "state copy");
    HIP_OK(hipMemcpyAsync(&bar_err, W.bar + kBarErr, sizeof(unsigned), hipMemcpyDeviceToHost, s), "state copy");
    HIP_OK(hipStreamSynchronize(s), "solve");
    if (bar_err) return set_error(DUQ_EDEVICE, "grid barrier timeout (a workgroup did not arrive)");
    const int code = st.status == 0                ? DUQ_OK
                     : st.status == 2             ? DUQ_ENUMERIC
                     : st.status == kStInfeasible ? DUQ_EINFEASIBLE
                                                  : DUQ_EMAXITER;
    if (res) {
        std::memset(res, 0, sizeof(*res));
        res->status = code;
        res->outer_iters = st.k;
        res->inner_iters = st.inner;
        res->gt_rows = st.gt_rows;
        res->f = st.F;
        res->lb_dual = st.LB;
        res->gap = st.F - st.LB;
        res->feas = st.feas;
        res->time_ms = 0.0;
        res->f64_outer_iters = st.k;
        res->engine = engine;
        res->lam_min = o->lam_min;
        res->lam_max = o->lam_max;
        res->G_norm2 = p > 0 ? o->G_norm2 : 0.0;
    }
    if (code == DUQ_ENUMERIC) set_error(code, "non-finite value during the iteration");
    if (code == DUQ_EMAXITER) set_error(code, "max_outer reached");
    if (code == DUQ_EINFEASIBLE) set_error(code, "the constraints have no solution in the box");
    return code;
}
