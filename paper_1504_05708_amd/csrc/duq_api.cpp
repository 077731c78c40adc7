// Host runtime behind the C ABI of include/duq.h: validation, device
// memory, constants, engine choice, launches and result transfer.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/duq.h"
#include "internal.h"
#include "launch.h"
#include "workspace.h"

using namespace duq;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t _e = (expr);                                                          \
        if (_e != hipSuccess)                                                            \
            return fail(_e == hipErrorOutOfMemory ? DUQ_ENOMEM : DUQ_EDEVICE,            \
                        std::string(#expr) + ": " + hipGetErrorString(_e));              \
    } while (0)

struct DeviceInfo {
    int cus = 0;
    size_t lds_max = 0;   // dynamic LDS one workgroup may use (static LDS taken off)
};

int device_info(DeviceInfo* di) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    di->cus = prop.multiProcessorCount;
    di->lds_max = prop.sharedMemPerBlock;
#if HIP_VERSION_MAJOR >= 6
    if (prop.maxSharedMemoryPerMultiProcessor > di->lds_max && prop.maxSharedMemoryPerMultiProcessor <= 160 * 1024)
        di->lds_max = prop.maxSharedMemoryPerMultiProcessor;
#endif
    const size_t st = dfom_static_lds_bytes();
    di->lds_max = di->lds_max > st ? di->lds_max - st : 0;
    return DUQ_OK;
}

size_t esize(int dtype) { return dtype == DUQ_F64 ? 8 : 4; }

// Launch shape of the single-QP solver: one workgroup (BLOCK) or one per CU
// (GRID, at most one per variable).
int solver_blocks(const DeviceInfo& di, int n, int engine) {
    return engine == DUQ_ENGINE_BLOCK ? 1 : std::max(1, std::min(di.cus, n));
}

// Largest n whose LDS-staged iterate fits one workgroup for p rows of G (the
// LDS use grows by one double per variable).  GRID assumes n >= CUs, which
// holds near the bound.
long solver_max_n(const DeviceInfo& di, int p, int engine) {
    const size_t base = dfom_lds_bytes(0, p, engine == DUQ_ENGINE_BLOCK ? 1 : di.cus);
    return base < di.lds_max ? (long)((di.lds_max - base) / sizeof(double)) : 0;
}

int too_large(const DeviceInfo& di, int n, int p, int engine) {
    return fail(DUQ_EINVAL, "n = " + std::to_string(n) + " too large for the LDS-staged products: n <= " +
                                std::to_string(solver_max_n(di, p, engine)) + " for p = " + std::to_string(p) +
                                " on this engine (" + std::to_string(di.lds_max) + " bytes of dynamic LDS per workgroup)");
}

bool finite_all(const double* a, long len) {
    for (long i = 0; i < len; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

template <typename T>
bool finite_all_t(const T* a, long len) {
    for (long i = 0; i < len; ++i)
        if (!std::isfinite((double)a[i])) return false;
    return true;
}

}  // namespace

namespace duq {
int set_error(int code, const std::string& msg) { return fail(code, msg); }
int device_cus() {
    DeviceInfo di;
    if (device_info(&di) != DUQ_OK) return 1;
    return std::max(1, di.cus);
}
int device_shape(int* cus, size_t* lds_max) {
    DeviceInfo di;
    if (int rc = device_info(&di)) return rc;
    *cus = di.cus;
    *lds_max = di.lds_max;
    return DUQ_OK;
}
}  // namespace duq

struct duq_handle {
    int n = 0, p = 0, dtype = 0;
    hipStream_t stream = nullptr;
    duq_options opts;
    // device data
    void* dQ = nullptr;
    void* dG = nullptr;
    double *dq = nullptr, *dg = nullptr, *dlb = nullptr, *dub = nullptr;
    void* owned_data = nullptr;   // allocation holding copied data (HOST memspace)
    // row bounds (user form of Sec. 2) and the equality form
    bool rows = false;
    bool eqform = false;
    double *drlo = nullptr, *drhi = nullptr;
    void* dH = nullptr;            // Q + rho G^T G (equality form), owned
    // compressed-row Q, G and G^T (inside owned_data) when set up from CSR
    bool sparse = false;
    bool x_global = false;         // sparse: x read in place (it does not fit in LDS)
    SparseRefs sp{};
    long long nnzQ = 0, nnzG = 0;
    // constants
    double lam_min = 0, lam_max = 0, G2 = 0;
    double Ld = 0, alpha = 0, L_in = 0, sigma = 0, beta_in = 0, D_U = 0;
    int k_in = 1, Kd_nonneg = 1, variant = 3;
    // engine
    int engine = DUQ_ENGINE_BLOCK;
    LaunchCfg cfg{};
    // workspace
    void* ws = nullptr;
    DevWork W{};
    double* xstage = nullptr;
    double* lstage = nullptr;
    bool ws_borrowed = false;      // ws lent by the caller (not freed here)
    int trace_cap = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int last_records = 0;
};

extern "C" {

void duq_default_options(duq_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->method = DUQ_DFGM;
    o->output = DUQ_LAST;
    o->inner_rule = DUQ_CERT;
    o->inner_variant = DUQ_INNER_AUTO;
    o->accumulate = DUQ_ACC_F64;
    o->engine = DUQ_ENGINE_AUTO;
    o->max_outer = 100000;
    o->max_inner = 0;
    o->lanczos_steps = 0;
    o->trace_outer = 0;
    o->eps_out = 1e-4;
    o->eps_in = 1e-6;
    o->rho = 0.0;
    o->lam_min = 0.0;
    o->lam_max = 0.0;
    o->G_norm2 = 0.0;
    o->safety = 1.02;
    o->switch_factor = 10.0;
    o->switch_stall = 20;
    o->serve_slice = 16;
}

const char* duq_last_error(void) { return g_err.c_str(); }

const char* duq_strerror(int code) {
    switch (code) {
        case DUQ_OK: return "ok";
        case DUQ_EINVAL: return "invalid argument";
        case DUQ_ENOMEM: return "out of memory";
        case DUQ_EDEVICE: return "device error";
        case DUQ_EMAXITER: return "iteration limit reached";
        case DUQ_ENUMERIC: return "non-finite value in the iteration";
        case DUQ_EAGAIN: return "not ready";
        case DUQ_ENOTFOUND: return "not found";
        case DUQ_EINFEASIBLE: return "infeasible constraints (certificate returned)";
        default: return "unknown";
    }
}

void duq_destroy(duq_handle* h) {
    if (!h) return;
    if (h->ws && !h->ws_borrowed) (void)hipFree(h->ws);
    if (h->dH) (void)hipFree(h->dH);
    if (h->owned_data) (void)hipFree(h->owned_data);
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    delete h;
}

}  // extern "C"

namespace duq {

int validate_common(const duq_problem* pr, const duq_options* o, bool sparse) {
    if (!pr || !o) return fail(DUQ_EINVAL, "null problem or options");
    if (pr->n <= 0) return fail(DUQ_EINVAL, "n must be positive");
    if (pr->p < 0) return fail(DUQ_EINVAL, "p must be non-negative");
    if (pr->dtype != DUQ_F64 && pr->dtype != DUQ_F32) return fail(DUQ_EINVAL, "dtype must be F64 or F32");
    if (pr->memspace != DUQ_HOST && pr->memspace != DUQ_DEVICE) return fail(DUQ_EINVAL, "bad memspace");
    if ((!sparse && !pr->Q) || !pr->q || !pr->lb || !pr->ub) return fail(DUQ_EINVAL, "null Q, q, lb or ub");
    if (pr->p > 0 && ((!sparse && !pr->G) || !pr->g)) return fail(DUQ_EINVAL, "null G or g with p > 0");
    if ((pr->rlo == nullptr) != (pr->rhi == nullptr)) return fail(DUQ_EINVAL, "give both rlo and rhi, or neither");
    if (pr->rlo && o->accumulate != DUQ_ACC_F64)
        return fail(DUQ_EINVAL, "row bounds need FP64 accumulation (no precision switch)");
    if (o->method != DUQ_DGM && o->method != DUQ_DFGM) return fail(DUQ_EINVAL, "bad method");
    if (o->output != DUQ_LAST && o->output != DUQ_AVG) return fail(DUQ_EINVAL, "bad output");
    if (o->inner_rule != DUQ_CERT && o->inner_rule != DUQ_FIXED) return fail(DUQ_EINVAL, "bad inner_rule");
    if (o->inner_variant < 0 || o->inner_variant > 3) return fail(DUQ_EINVAL, "bad inner_variant");
    if (o->accumulate != DUQ_ACC_F64 && o->accumulate != DUQ_ACC_F32) return fail(DUQ_EINVAL, "bad accumulate");
    if (o->accumulate == DUQ_ACC_F32 && pr->dtype != DUQ_F32)
        return fail(DUQ_EINVAL, "FP32 accumulation needs FP32 storage");
    if (!(o->eps_out > 0.0) || !(o->eps_in > 0.0)) return fail(DUQ_EINVAL, "eps_out and eps_in must be > 0");
    if (!(o->rho >= 0.0) || !std::isfinite(o->rho)) return fail(DUQ_EINVAL, "rho must be >= 0");
    if (o->max_outer < 1) return fail(DUQ_EINVAL, "max_outer must be >= 1");
    if (o->max_inner < 0 || o->trace_outer < 0 || o->lanczos_steps < 0)
        return fail(DUQ_EINVAL, "negative count");
    if (!(o->safety >= 1.0)) return fail(DUQ_EINVAL, "safety must be >= 1");
    if (o->sparse_x < DUQ_SPX_AUTO || o->sparse_x > DUQ_SPX_IN_PLACE) return fail(DUQ_EINVAL, "bad sparse_x");
    if (o->lb_cert < DUQ_LB_AUTO || o->lb_cert > DUQ_LB_SIGMA_FREE) return fail(DUQ_EINVAL, "bad lb_cert");
    return DUQ_OK;
}

int validate_problem(const duq_problem* pr, const duq_options* o) { return validate_common(pr, o, false); }

// A compressed-row matrix of shape rows x cols (Sec. 5.1 sparse data): offsets
// from 0 and nondecreasing, indices in range, finite values.
int check_csr(const duq_csr* M, int rows, int cols, int dtype, const char* name) {
    const std::string nm(name);
    if (!M) return fail(DUQ_EINVAL, "null " + nm);
    if (M->rows != rows || M->cols != cols)
        return fail(DUQ_EINVAL, nm + " has shape " + std::to_string(M->rows) + " x " + std::to_string(M->cols) +
                                    ", expected " + std::to_string(rows) + " x " + std::to_string(cols));
    if (!M->rowptr) return fail(DUQ_EINVAL, "null " + nm + " row offsets");
    if (M->rowptr[0] != 0) return fail(DUQ_EINVAL, nm + " row offsets must start at 0");
    for (int i = 0; i < rows; ++i)
        if (M->rowptr[i + 1] < M->rowptr[i])
            return fail(DUQ_EINVAL, nm + " row offsets decrease at row " + std::to_string(i));
    const long long nnz = M->rowptr[rows];
    if (nnz > 0 && (!M->col || !M->val)) return fail(DUQ_EINVAL, "null " + nm + " indices or values");
    for (long long k = 0; k < nnz; ++k)
        if (M->col[k] < 0 || M->col[k] >= cols)
            return fail(DUQ_EINVAL, nm + " column index out of range at entry " + std::to_string(k));
    const bool ok =
        dtype == DUQ_F64 ? finite_all_t((const double*)M->val, nnz) : finite_all_t((const float*)M->val, nnz);
    if (!ok) return fail(DUQ_EINVAL, "non-finite value in " + nm);
    return DUQ_OK;
}

int upload_sparse(duq_handle* h, const duq_problem* pr, const duq_csr* Qs, const duq_csr* Gs,
                  const std::vector<double>& lb, const std::vector<double>& ub, const std::vector<double>& rlo,
                  const std::vector<double>& rhi);

}  // namespace duq

namespace duq {
int estimate_constants(duq_handle* h, const DeviceInfo& di);

// Kernel parameters from the spectral constants, the box diameter D_U and
// the options: L_d = ||G||^2/(lam_min + rho ||G||^2) (Sec. 2 eq. Ld), step
// 1/(2 L_d); L_in = lam_max + rho ||G||^2, sigma_in = lam_min (Sec. 3 Step 1);
// the inner cap k_in of Sec. 5 (natural log, rounded up) unless max_inner > 0.
// The inner gap entering LB (options.lb_cert): AUTO is the sigma form, the
// one the stopping test uses.  It is a valid bound when sigma is at most the
// strong convexity of the inner problem; an estimated lambda_min (a Lanczos
// Ritz value, which lies above lambda_min, divided by the safety factor) is a
// margin, not a bound, and SIGMA_FREE (the FW gap, linear rather than
// quadratic in the gradient, so LB converges more slowly) is valid for any
// sigma.
int resolve_lb_cert(int opt) { return opt == DUQ_LB_AUTO ? DUQ_LB_SIGMA : opt; }

int derive_params(int p, double lam_min, double lam_max, double g2, double D_U, const duq_options& o,
                  DevParams* par, double sigma) {
    const double rho = o.rho;
    const double denom = lam_min + rho * g2;
    if (p > 0 && !(denom > 0.0)) return fail(DUQ_EINVAL, "lambda_min(Q) = 0 needs rho > 0 (Sec. 2, Case 2)");
    *par = DevParams{};
    const double Ld = p > 0 ? g2 / denom : 0.0;
    par->alpha = Ld > 0.0 ? 1.0 / (2.0 * Ld) : 0.0;
    par->L = lam_max + rho * g2;
    // sigma > 0: the strong convexity of the inner problem (with equality
    // rows and rho > 0, lambda_min(Q + rho G_eq^T G_eq), Sec. 3 Step 1)
    par->sigma = std::max(sigma > 0.0 ? sigma : lam_min, 0.0);
    const double sqL = std::sqrt(par->L), sqs = std::sqrt(par->sigma);
    par->beta_in = (sqL - sqs) / (sqL + sqs);
    int k_in;
    if (o.max_inner > 0) k_in = o.max_inner;
    else if (par->sigma > 0.0) {
        const double arg = par->L * D_U * D_U / o.eps_in;
        k_in = arg > 1.0 ? (int)std::ceil(std::sqrt(par->L / par->sigma) * std::log(arg)) + 1 : 1;
    } else {
        k_in = (int)std::ceil(std::sqrt(2.0 * par->L * D_U * D_U / o.eps_in));
    }
    par->k_in_max = std::max(k_in, 1);
    par->Kd_nonneg = lam_min > 0.0 ? 1 : 0;
    int v = o.inner_variant;
    if (v == DUQ_INNER_AUTO) v = par->sigma > 0.0 ? DUQ_INNER_FGM_SIGMA : DUQ_INNER_FGM;
    par->inner_variant = v;
    par->method = o.method;
    par->output = o.output;
    par->inner_rule = o.inner_rule;
    par->max_outer = o.max_outer;
    par->eps_out = o.eps_out;
    par->eps_in = o.eps_in;
    par->rho = o.rho;
    par->lb_cert = resolve_lb_cert(o.lb_cert);
    return DUQ_OK;
}
}

extern "C" int duq_max_n(int32_t p, int32_t engine, int32_t* n_max) {
    if (!n_max) return fail(DUQ_EINVAL, "null n_max");
    *n_max = 0;
    if (p < 0) return fail(DUQ_EINVAL, "p < 0");
    if (engine == DUQ_ENGINE_AUTO) engine = DUQ_ENGINE_GRID;
    if (engine != DUQ_ENGINE_BLOCK && engine != DUQ_ENGINE_GRID)
        return fail(DUQ_EINVAL, "duq_max_n: engine must be AUTO, BLOCK or GRID");
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc) return rc;
    *n_max = (int32_t)std::min<long>(solver_max_n(di, p, engine), INT32_MAX);
    return DUQ_OK;
}

// duq_setup (Qs null: dense Q and G in `pr`) and duq_setup_csr (compressed-row
// Q and G, already checked).
static int setup_impl(const duq_problem* pr, const duq_csr* Qs, const duq_csr* Gs, const duq_options* opts,
                      void* stream, duq_handle** out, void* lent_ws = nullptr, size_t lent_bytes = 0) {
    if (!out) return fail(DUQ_EINVAL, "null output handle");
    *out = nullptr;
    const bool sparse = Qs != nullptr;
    int rc = validate_common(pr, opts, sparse);
    if (rc) return rc;
    const int n = pr->n, p = pr->p, dtype = pr->dtype;
    const long nn = (long)n * n, pn = (long)p * n;
    DeviceInfo di;
    if ((rc = device_info(&di))) return rc;
    int engine = opts->engine;
    if (engine == DUQ_ENGINE_AUTO) engine = (n <= 1536) ? DUQ_ENGINE_BLOCK : DUQ_ENGINE_GRID;
    // compressed-row data reads x in place when asked, and by default on the
    // grid engine (a product reads a few entries of x per row, where staging
    // all of x would read n entries per workgroup) or when x does not fit in LDS
    const bool x_global =
        sparse && (opts->sparse_x == DUQ_SPX_IN_PLACE ||
                   (opts->sparse_x == DUQ_SPX_AUTO &&
                    (engine == DUQ_ENGINE_GRID || dfom_lds_bytes(n, p, solver_blocks(di, n, engine)) > di.lds_max)));
    if (dfom_lds_bytes(n, p, solver_blocks(di, n, engine), x_global) > di.lds_max)
        return too_large(di, n, p, engine);

    duq_handle* h = new (std::nothrow) duq_handle();
    if (!h) return fail(DUQ_ENOMEM, "host allocation");
    h->n = n;
    h->p = p;
    h->dtype = dtype;
    h->opts = *opts;
    h->stream = (hipStream_t)stream;

    // lb, ub on the host for validation and the box diameter D_U
    std::vector<double> lb(n), ub(n);
    if (pr->memspace == DUQ_HOST) {
        std::memcpy(lb.data(), pr->lb, n * sizeof(double));
        std::memcpy(ub.data(), pr->ub, n * sizeof(double));
    } else {
        // stream-ordered: the caller may have queued the upload of lb/ub on `stream`
        if (hipMemcpyAsync(lb.data(), pr->lb, n * sizeof(double), hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
            hipMemcpyAsync(ub.data(), pr->ub, n * sizeof(double), hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
            hipStreamSynchronize(h->stream) != hipSuccess) {
            duq_destroy(h);
            return fail(DUQ_EINVAL, "lb/ub are not readable device pointers");
        }
    }
    double du2 = 0.0;
    for (int i = 0; i < n; ++i) {
        if (!std::isfinite(lb[i]) || !std::isfinite(ub[i]) || lb[i] > ub[i]) {
            duq_destroy(h);
            return fail(DUQ_EINVAL, "box must be finite with lb <= ub (U compact, Sec. 2)");
        }
        du2 += (ub[i] - lb[i]) * (ub[i] - lb[i]);
    }
    h->D_U = std::sqrt(du2);

    // row bounds: rlo <= G u + g <= rhi (Sec. 2), each row an equality or up to
    // two inequalities
    std::vector<double> rlo, rhi;
    if (pr->rlo) {
        rlo.resize(std::max(p, 1));
        rhi.resize(std::max(p, 1));
        if (p > 0) {
            if (pr->memspace == DUQ_HOST) {
                std::memcpy(rlo.data(), pr->rlo, p * sizeof(double));
                std::memcpy(rhi.data(), pr->rhi, p * sizeof(double));
            } else if (hipMemcpyAsync(rlo.data(), pr->rlo, p * sizeof(double), hipMemcpyDeviceToHost, h->stream) !=
                           hipSuccess ||
                       hipMemcpyAsync(rhi.data(), pr->rhi, p * sizeof(double), hipMemcpyDeviceToHost, h->stream) !=
                           hipSuccess ||
                       hipStreamSynchronize(h->stream) != hipSuccess) {
                duq_destroy(h);
                return fail(DUQ_EINVAL, "rlo/rhi are not readable device pointers");
            }
        }
        bool all_eq = p > 0;
        for (int i = 0; i < p; ++i) {
            const double lo = rlo[i], hi = rhi[i];
            if (std::isnan(lo) || std::isnan(hi) || lo > hi || lo == INFINITY || hi == -INFINITY ||
                (lo == hi && std::isinf(lo))) {
                duq_destroy(h);
                return fail(DUQ_EINVAL, "row bounds need rlo <= rhi, rlo < +inf, rhi > -inf (row " +
                                            std::to_string(i) + ")");
            }
            all_eq = all_eq && lo == hi;
        }
        h->rows = true;
        h->eqform = all_eq && opts->rho > 0.0 && !sparse;
    }

    if (sparse) {
        if ((rc = upload_sparse(h, pr, Qs, Gs, lb, ub, rlo, rhi))) {
            duq_destroy(h);
            return rc;
        }
    } else if (pr->memspace == DUQ_HOST) {
        bool ok = finite_all(pr->q, n) && (p == 0 || finite_all(pr->g, p));
        ok = ok && (dtype == DUQ_F64 ? finite_all_t((const double*)pr->Q, nn) : finite_all_t((const float*)pr->Q, nn));
        if (p > 0)
            ok = ok && (dtype == DUQ_F64 ? finite_all_t((const double*)pr->G, pn) : finite_all_t((const float*)pr->G, pn));
        if (!ok) {
            duq_destroy(h);
            return fail(DUQ_EINVAL, "non-finite problem data");
        }
        Carve c;
        c.take<char>(nn * esize(dtype));
        c.take<char>(std::max<long>(pn, 1) * esize(dtype));
        c.take<double>(n);
        c.take<double>(std::max(p, 1));
        c.take<double>(n);
        c.take<double>(n);
        c.take<double>(std::max(p, 1));
        c.take<double>(std::max(p, 1));
        if (hipMalloc(&h->owned_data, c.off) != hipSuccess) {
            duq_destroy(h);
            return fail(DUQ_ENOMEM, "device allocation of problem data");
        }
        c.base = (char*)h->owned_data;
        c.off = 0;
        h->dQ = c.take<char>(nn * esize(dtype));
        h->dG = c.take<char>(std::max<long>(pn, 1) * esize(dtype));
        h->dq = c.take<double>(n);
        h->dg = c.take<double>(std::max(p, 1));
        h->dlb = c.take<double>(n);
        h->dub = c.take<double>(n);
        double* rl = c.take<double>(std::max(p, 1));
        double* rh = c.take<double>(std::max(p, 1));
        if (h->rows) {
            h->drlo = rl;
            h->drhi = rh;
        }
        hipError_t e = hipSuccess;
        e = e ? e : hipMemcpy(h->dQ, pr->Q, nn * esize(dtype), hipMemcpyHostToDevice);
        if (p > 0) e = e ? e : hipMemcpy(h->dG, pr->G, pn * esize(dtype), hipMemcpyHostToDevice);
        e = e ? e : hipMemcpy(h->dq, pr->q, n * sizeof(double), hipMemcpyHostToDevice);
        if (p > 0) e = e ? e : hipMemcpy(h->dg, pr->g, p * sizeof(double), hipMemcpyHostToDevice);
        e = e ? e : hipMemcpy(h->dlb, lb.data(), n * sizeof(double), hipMemcpyHostToDevice);
        e = e ? e : hipMemcpy(h->dub, ub.data(), n * sizeof(double), hipMemcpyHostToDevice);
        if (h->rows && p > 0) {
            e = e ? e : hipMemcpy(h->drlo, rlo.data(), p * sizeof(double), hipMemcpyHostToDevice);
            e = e ? e : hipMemcpy(h->drhi, rhi.data(), p * sizeof(double), hipMemcpyHostToDevice);
        }
        if (e != hipSuccess) {
            duq_destroy(h);
            return fail(DUQ_EDEVICE, std::string("copy of problem data: ") + hipGetErrorString(e));
        }
    } else {
        h->dQ = const_cast<void*>(pr->Q);
        h->dG = const_cast<void*>(pr->G);
        h->dq = const_cast<double*>(pr->q);
        h->dg = const_cast<double*>(pr->g);
        h->dlb = const_cast<double*>(pr->lb);
        h->dub = const_cast<double*>(pr->ub);
        if (h->rows) {
            h->drlo = const_cast<double*>(pr->rlo);
            h->drhi = const_cast<double*>(pr->rhi);
        }
        // borrowed data: count non-finite entries on the device
        unsigned* cnt = nullptr;
        if (hipMalloc(&cnt, sizeof(unsigned)) != hipSuccess) {
            duq_destroy(h);
            return fail(DUQ_ENOMEM, "device allocation");
        }
        unsigned hc = 0;
        hipError_t e = hipMemsetAsync(cnt, 0, sizeof(unsigned), h->stream);
        e = e ? e : launch_count_nonfinite(dtype, h->dQ, nn, cnt, h->stream);
        if (p > 0) e = e ? e : launch_count_nonfinite(dtype, h->dG, pn, cnt, h->stream);
        e = e ? e : launch_count_nonfinite(DUQ_F64, h->dq, n, cnt, h->stream);
        if (p > 0) e = e ? e : launch_count_nonfinite(DUQ_F64, h->dg, p, cnt, h->stream);
        e = e ? e : hipMemcpyAsync(&hc, cnt, sizeof(unsigned), hipMemcpyDeviceToHost, h->stream);
        e = e ? e : hipStreamSynchronize(h->stream);
        (void)hipFree(cnt);
        if (e != hipSuccess) {
            duq_destroy(h);
            return fail(DUQ_EDEVICE, std::string("validation of device data: ") + hipGetErrorString(e));
        }
        if (hc) {
            duq_destroy(h);
            return fail(DUQ_EINVAL, "non-finite problem data");
        }
    }

    // engine and launch shape
    h->engine = engine;
    const int acc_first = opts->accumulate;
    if (engine == DUQ_ENGINE_BLOCK) {
        h->cfg.nblocks = 1;
        h->cfg.nthreads = n <= 128 ? 256 : 512;
        h->cfg.cooperative = false;
    } else {
        h->cfg.nthreads = 512;
        int nb = di.cus;
        nb = std::max(1, std::min(nb, n));
        h->cfg.nblocks = nb;
        h->cfg.cooperative = true;
    }
    h->cfg.stream = h->stream;
    h->x_global = x_global;
    h->cfg.shmem = dfom_lds_bytes(n, p, h->cfg.nblocks, x_global);
    if (h->cfg.shmem > di.lds_max) {   // checked before any data moved; kept as a guard
        duq_destroy(h);
        return too_large(di, n, p, engine);
    }
    if (h->cfg.cooperative) {
        for (int acc = 0; acc <= (dtype == DUQ_F32 ? 1 : 0); ++acc) {
            int bpc = 0;
            if (dfom_occupancy(dtype, acc, n, h->cfg.nthreads, h->cfg.shmem, &bpc, h->rows, sparse) != hipSuccess ||
                bpc < 1) {
                duq_destroy(h);
                return fail(DUQ_EDEVICE, "cooperative launch does not fit one block per CU");
            }
        }
    }
    (void)acc_first;

    // workspace
    const int nb = h->cfg.nblocks;
    const int trace = opts->trace_outer;
    auto carve = [&](Carve& c) { carve_solver(c, n, p, nb, trace, &h->W, &h->xstage, &h->lstage, sparse); };
    Carve c0;
    carve(c0);
    if (lent_ws) {
        if (lent_bytes < c0.off) {
            duq_destroy(h);
            return fail(DUQ_ENOMEM, "lent workspace of " + std::to_string(lent_bytes) + " bytes, " +
                                        std::to_string(c0.off) + " needed");
        }
        h->ws = lent_ws;
        h->ws_borrowed = true;
    } else if (hipMalloc(&h->ws, c0.off) != hipSuccess) {
        duq_destroy(h);
        return fail(DUQ_ENOMEM, "device workspace (" + std::to_string(c0.off) + " bytes)");
    }
    Carve c1;
    c1.base = (char*)h->ws;
    carve(c1);
    h->trace_cap = trace;
    if (hipMemset(h->ws, 0, c0.off) != hipSuccess) {
        duq_destroy(h);
        return fail(DUQ_EDEVICE, "workspace clear");
    }
    if (hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess) {
        duq_destroy(h);
        return fail(DUQ_EDEVICE, "event creation");
    }

    // equality form: every row an equality and rho > 0, the inner Hessian
    // Q + rho G^T G is constant (Sec. 5.1) and formed once here
    if (h->eqform) {
        if (hipMalloc(&h->dH, nn * esize(dtype)) != hipSuccess) {
            duq_destroy(h);
            return fail(DUQ_ENOMEM, "device allocation of Q + rho G^T G");
        }
        hipError_t e = launch_form_hessian(dtype, n, p, h->dQ, h->dG, opts->rho, h->dH, h->stream);
        if (e != hipSuccess) {
            duq_destroy(h);
            return fail(DUQ_EDEVICE, std::string("forming Q + rho G^T G: ") + hipGetErrorString(e));
        }
    }

    // constants (a1): caller-supplied or estimated
    h->lam_min = opts->lam_min;
    h->lam_max = opts->lam_max;
    h->G2 = p > 0 ? opts->G_norm2 : 0.0;
    h->sigma = opts->sigma_in > 0.0 ? opts->sigma_in : 0.0;
    if (h->lam_min <= 0.0 || h->lam_max <= 0.0 || (p > 0 && h->G2 <= 0.0) || (h->eqform && h->sigma <= 0.0)) {
        rc = estimate_constants(h, di);
        if (rc) {
            duq_destroy(h);
            return rc;
        }
    }
    DevParams dp;
    rc = derive_params(p, h->lam_min, h->lam_max, h->G2, h->D_U, *opts, &dp, h->sigma);
    if (rc) {
        duq_destroy(h);
        return rc;
    }
    h->Ld = p > 0 ? h->G2 / (h->lam_min + opts->rho * h->G2) : 0.0;
    h->alpha = dp.alpha;
    h->L_in = dp.L;
    h->sigma = dp.sigma;
    h->beta_in = dp.beta_in;
    h->k_in = dp.k_in_max;
    h->Kd_nonneg = dp.Kd_nonneg;
    h->variant = dp.inner_variant;
    *out = h;
    return DUQ_OK;
}

extern "C" int duq_setup(const duq_problem* pr, const duq_options* opts, void* stream, duq_handle** out) {
    return setup_impl(pr, nullptr, nullptr, opts, stream, out);
}

// Internal (serving): bytes of the solver workspace of a dense QP with
// tracing off on `nblocks` workgroups, and duq_setup on a workspace the
// caller lends (a block of its arena, at least that many bytes, 256-byte
// aligned, not freed by duq_destroy).  The constant estimate's Krylov basis
// is still a temporary allocation of the setup.
size_t solver_workspace_bytes(int n, int p, int nblocks) {
    DevWork W;
    double* xs = nullptr;
    double* ls = nullptr;
    Carve c;
    carve_solver(c, n, p, nblocks, 0, &W, &xs, &ls, false);
    return c.off;
}

int setup_lent(const duq_problem* pr, const duq_options* opts, void* stream, void* ws, size_t ws_bytes,
               duq_handle** out) {
    return setup_impl(pr, nullptr, nullptr, opts, stream, out, ws, ws_bytes);
}

extern "C" int duq_setup_csr(const duq_problem* pr, const duq_csr* Q, const duq_csr* G, const duq_options* opts,
                             void* stream, duq_handle** out) {
    if (!out) return fail(DUQ_EINVAL, "null output handle");
    *out = nullptr;
    if (!pr || !opts) return fail(DUQ_EINVAL, "null problem or options");
    if (pr->memspace != DUQ_HOST) return fail(DUQ_EINVAL, "compressed-row data is read from host memory (DUQ_HOST)");
    if (pr->n <= 0 || pr->p < 0) return fail(DUQ_EINVAL, "n must be positive and p non-negative");
    if (pr->dtype != DUQ_F64 && pr->dtype != DUQ_F32) return fail(DUQ_EINVAL, "dtype must be F64 or F32");
    int rc = check_csr(Q, pr->n, pr->n, pr->dtype, "Q");
    if (!rc && pr->p > 0) rc = check_csr(G, pr->p, pr->n, pr->dtype, "G");
    if (rc) return rc;
    return setup_impl(pr, Q, G, opts, stream, out);
}

namespace duq {

// Copy compressed-row Q, G, the vectors and the row bounds to one device
// allocation, and form G^T (a counting sort of the entries of G by column,
// stable in the row index) so the transposed product gathers along rows.
int upload_sparse(duq_handle* h, const duq_problem* pr, const duq_csr* Qs, const duq_csr* Gs,
                  const std::vector<double>& lb, const std::vector<double>& ub, const std::vector<double>& rlo,
                  const std::vector<double>& rhi) {
    const int n = h->n, p = h->p;
    const size_t es = esize(h->dtype);
    const long long nq = Qs->rowptr[n];
    const long long ng = p > 0 ? Gs->rowptr[p] : 0;
    if (!finite_all(pr->q, n) || (p > 0 && !finite_all(pr->g, p))) return fail(DUQ_EINVAL, "non-finite problem data");
    std::vector<long long> trp((size_t)n + 1, 0);
    std::vector<int> tci((size_t)std::max<long long>(ng, 1));
    std::vector<char> tv((size_t)std::max<long long>(ng, 1) * es);
    for (long long k = 0; k < ng; ++k) ++trp[(size_t)Gs->col[k] + 1];
    for (int j = 0; j < n; ++j) trp[j + 1] += trp[j];
    {
        std::vector<long long> pos(trp.begin(), trp.end() - 1);
        const char* gv = (const char*)Gs->val;
        for (int r = 0; r < p; ++r)
            for (long long k = Gs->rowptr[r]; k < Gs->rowptr[r + 1]; ++k) {
                const long long d = pos[Gs->col[k]]++;
                tci[d] = r;
                std::memcpy(tv.data() + d * es, gv + k * es, es);
            }
    }
    auto layout = [&](Carve& c, SparseRefs* s, double** vec) {
        s->Qrp = c.take<long long>((size_t)n + 1);
        s->Qci = c.take<int>(std::max<long long>(nq, 1));
        s->Qv = c.take<char>(std::max<long long>(nq, 1) * es);
        s->Grp = c.take<long long>((size_t)p + 1);
        s->Gci = c.take<int>(std::max<long long>(ng, 1));
        s->Gv = c.take<char>(std::max<long long>(ng, 1) * es);
        s->Trp = c.take<long long>((size_t)n + 1);
        s->Tci = c.take<int>(std::max<long long>(ng, 1));
        s->Tv = c.take<char>(std::max<long long>(ng, 1) * es);
        vec[0] = c.take<double>(n);
        vec[1] = c.take<double>(std::max(p, 1));
        vec[2] = c.take<double>(n);
        vec[3] = c.take<double>(n);
        vec[4] = c.take<double>(std::max(p, 1));
        vec[5] = c.take<double>(std::max(p, 1));
    };
    SparseRefs sp{};
    double* vec[6];
    Carve c0;
    layout(c0, &sp, vec);
    if (hipMalloc(&h->owned_data, c0.off) != hipSuccess)
        return fail(DUQ_ENOMEM, "device allocation of sparse problem data (" + std::to_string(c0.off) + " bytes)");
    Carve c1;
    c1.base = (char*)h->owned_data;
    layout(c1, &sp, vec);
    hipError_t e = hipSuccess;
    auto put = [&](const void* dst, const void* src, size_t bytes) {
        if (bytes && e == hipSuccess) e = hipMemcpy(const_cast<void*>(dst), src, bytes, hipMemcpyHostToDevice);
    };
    std::vector<long long> zeros((size_t)p + 1, 0);
    put(sp.Qrp, Qs->rowptr, ((size_t)n + 1) * sizeof(long long));
    put(sp.Qci, Qs->col, (size_t)nq * sizeof(int));
    put(sp.Qv, Qs->val, (size_t)nq * es);
    put(sp.Grp, p > 0 ? (const void*)Gs->rowptr : (const void*)zeros.data(), ((size_t)p + 1) * sizeof(long long));
    if (p > 0) {
        put(sp.Gci, Gs->col, (size_t)ng * sizeof(int));
        put(sp.Gv, Gs->val, (size_t)ng * es);
    }
    put(sp.Trp, trp.data(), trp.size() * sizeof(long long));
    put(sp.Tci, tci.data(), (size_t)ng * sizeof(int));
    put(sp.Tv, tv.data(), (size_t)ng * es);
    put(vec[0], pr->q, (size_t)n * sizeof(double));
    if (p > 0) put(vec[1], pr->g, (size_t)p * sizeof(double));
    put(vec[2], lb.data(), (size_t)n * sizeof(double));
    put(vec[3], ub.data(), (size_t)n * sizeof(double));
    if (h->rows && p > 0) {
        put(vec[4], rlo.data(), (size_t)p * sizeof(double));
        put(vec[5], rhi.data(), (size_t)p * sizeof(double));
    }
    if (e != hipSuccess)
        return fail(DUQ_EDEVICE, std::string("copy of sparse problem data: ") + hipGetErrorString(e));
    // lanes per row: the power of two that leaves a lane about four nonzeros
    // of a mean row (1..64)
    auto lanes_lg = [](long long nnz, int rows) {
        const double avg = rows > 0 ? (double)nnz / rows : 0.0;
        int lg = 0;
        while (lg < 6 && 4.0 * (double)(2 << lg) <= avg) ++lg;
        return lg;
    };
    sp.Qlg = lanes_lg(nq, n);
    sp.Glg = lanes_lg(ng, p);
    sp.Tlg = lanes_lg(ng, n);
    h->sparse = true;
    h->sp = sp;
    h->nnzQ = nq;
    h->nnzG = ng;
    h->dq = vec[0];
    h->dg = vec[1];
    h->dlb = vec[2];
    h->dub = vec[3];
    if (h->rows) {
        h->drlo = vec[4];
        h->drhi = vec[5];
    }
    return DUQ_OK;
}

int estimate_constants(duq_handle* h, const DeviceInfo& di) {
    const int n = h->n, p = h->p;
    int k = h->opts.lanczos_steps > 0 ? h->opts.lanczos_steps : 96;
    k = std::min(k, n);
    const int nb = h->cfg.nblocks;
    LanczosWork L{};
    Carve c0;
    auto carve = [&](Carve& c) {
        L.V = c.take<double>((size_t)(k + 1) * n);
        L.w = c.take<double>(n);
        L.r = c.take<double>(std::max(p, 1));
        L.part = c.take<double>((size_t)nb * (k + 2));
        L.gtp = c.take<double>(nb > 1 && !h->sparse ? (size_t)nb * n : 1);
        L.ab = c.take<double>(2 * (size_t)k + 2);
        L.out = c.take<double>(4);
        L.bar = c.take<unsigned>(bar_words(nb));
        L.rsh = c.take<double>(std::max(p, 1));
    };
    carve(c0);
    void* buf = nullptr;
    HIP_TRY(hipMalloc(&buf, c0.off));
    Carve c1;
    c1.base = (char*)buf;
    carve(c1);
    L.x_global = h->x_global ? 1 : 0;
    LaunchCfg cfg = h->cfg;
    cfg.shmem = lanczos_lds_bytes(n, p, nb, k, h->x_global);
    if (cfg.shmem > di.lds_max) {
        (void)hipFree(buf);
        return fail(DUQ_EINVAL, "problem too large for the Lanczos estimate; pass the constants");
    }
    GenericProblem gp{n, p, h->dQ, h->dG, h->dq, h->dg, h->dlb, h->dub, h->drlo, h->drhi};
    gp.sp = h->sp;
    double outQ[4] = {0, 0, 0, 0}, outG[4] = {0, 0, 0, 0}, outH[4] = {0, 0, 0, 0};
    unsigned flag = 0;
    auto run = [&](int use_gtg, double* out, const void* Qop) -> int {
        GenericProblem g2 = gp;
        g2.Q = Qop;
        hipError_t e = hipMemsetAsync(buf, 0, c0.off, h->stream);
        e = e ? e : launch_lanczos(h->dtype, cfg, g2, L, k, use_gtg);
        e = e ? e : hipMemcpyAsync(out, L.out, 4 * sizeof(double), hipMemcpyDeviceToHost, h->stream);
        e = e ? e : hipMemcpyAsync(&flag, L.bar + kBarErr, sizeof(unsigned), hipMemcpyDeviceToHost, h->stream);
        e = e ? e : hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return fail(DUQ_EDEVICE, std::string("Lanczos: ") + hipGetErrorString(e));
        if (flag) return fail(DUQ_EDEVICE, "Lanczos: grid barrier timeout");
        return DUQ_OK;
    };
    int rc = DUQ_OK;
    if (h->lam_min <= 0.0 || h->lam_max <= 0.0) rc = run(0, outQ, h->dQ);
    if (!rc && h->p > 0 && h->G2 <= 0.0) rc = run(1, outG, h->dQ);
    if (!rc && h->eqform && h->sigma <= 0.0) rc = run(0, outH, h->dH);   // lambda_min(Q + rho G^T G)
    (void)hipFree(buf);
    if (rc) return rc;
    const double sf = h->opts.safety;
    if (h->lam_min <= 0.0) h->lam_min = outQ[0] / sf;
    if (h->lam_max <= 0.0) h->lam_max = outQ[1] * sf;
    if (h->p > 0 && h->G2 <= 0.0) h->G2 = outG[1] * sf;
    if (h->eqform && h->sigma <= 0.0) h->sigma = outH[0] / sf;
    if (!(h->lam_max > 0.0)) return fail(DUQ_EINVAL, "Q appears to be zero");
    return DUQ_OK;
}

}  // namespace duq

extern "C" int duq_get_constants(duq_handle* h, double* lam_min, double* lam_max, double* G_norm2, double* Ld,
                                 double* L_in, double* sigma_in) {
    if (!h) return fail(DUQ_EINVAL, "null handle");
    if (lam_min) *lam_min = h->lam_min;
    if (lam_max) *lam_max = h->lam_max;
    if (G_norm2) *G_norm2 = h->G2;
    if (Ld) *Ld = h->Ld;
    if (L_in) *L_in = h->L_in;
    if (sigma_in) *sigma_in = h->sigma;
    return DUQ_OK;
}

extern "C" int duq_solve(duq_handle* h, const double* x0, const double* lam0, double* x_out, double* lam_out,
                         duq_result* res) {
    if (!h) return fail(DUQ_EINVAL, "null handle");
    const int n = h->n, p = h->p;
    const duq_options& o = h->opts;
    if (x0) {
        for (int i = 0; i < n; ++i)
            if (!std::isfinite(x0[i])) return fail(DUQ_EINVAL, "non-finite x0");
        HIP_TRY(hipMemcpyAsync(h->xstage, x0, n * sizeof(double), hipMemcpyHostToDevice, h->stream));
    }
    if (lam0 && p > 0 && h->rows) return fail(DUQ_EINVAL, "lam0 is not available with row bounds");
    if (lam0 && p > 0) {
        for (int i = 0; i < p; ++i)
            if (!std::isfinite(lam0[i])) return fail(DUQ_EINVAL, "non-finite lam0");
        HIP_TRY(hipMemcpyAsync(h->lstage, lam0, p * sizeof(double), hipMemcpyHostToDevice, h->stream));
    }
    HIP_TRY(hipMemsetAsync(h->W.st, 0, sizeof(DevState), h->stream));
    HIP_TRY(hipMemsetAsync(h->W.bar, 0, bar_words(h->cfg.nblocks) * sizeof(unsigned), h->stream));
    DevWork W = h->W;
    W.x0 = h->xstage;
    W.lam0 = h->lstage;
    DevParams par{};
    par.method = o.method;
    par.output = o.output;
    par.inner_rule = o.inner_rule;
    par.inner_variant = h->variant;
    par.max_outer = o.max_outer;
    par.k_in_max = h->k_in;
    par.trace_iters = std::min(o.trace_outer, h->trace_cap);
    par.Kd_nonneg = h->Kd_nonneg;
    par.has_x0 = x0 ? 1 : 0;
    par.has_lam0 = (lam0 && p > 0) ? 1 : 0;
    par.resume = 0;
    par.eps_out = o.eps_out;
    par.eps_in = o.eps_in;
    par.rho = o.rho;
    par.alpha = h->alpha;
    par.L = h->L_in;
    par.sigma = h->sigma;
    par.beta_in = h->beta_in;
    par.eqform = h->eqform ? 1 : 0;
    par.x_global = h->x_global ? 1 : 0;
    par.lb_cert = resolve_lb_cert(o.lb_cert);
    GenericProblem gp{n, p, h->eqform ? h->dH : h->dQ, h->dG, h->dq, h->dg, h->dlb, h->dub, h->drlo, h->drhi};
    gp.sp = h->sp;
    DevState st;
    unsigned bar_err = 0;
    int k_phase1 = 0;
    const bool two_phase = h->dtype == DUQ_F32 && o.accumulate == DUQ_ACC_F32;
    HIP_TRY(hipEventRecord(h->ev0, h->stream));
    if (two_phase) {
        // a8: FP32-accumulated products until the outer test passes at
        // switch_factor * eps_out or stalls, then FP64 accumulation from the
        // same device state (a warm start) to eps_out.
        DevParams p1 = par;
        p1.phase1 = 1;
        p1.stall_iters = o.switch_stall;
        p1.eps_out = o.eps_out * std::max(1.0, o.switch_factor);
        HIP_TRY(launch_dfom(h->dtype, DUQ_ACC_F32, h->cfg, gp, p1, W));
        HIP_TRY(hipMemcpyAsync(&st, h->W.st, sizeof(DevState), hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipMemcpyAsync(&bar_err, h->W.bar + kBarErr, sizeof(unsigned), hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        if (bar_err) return fail(DUQ_EDEVICE, "grid barrier timeout (a workgroup did not arrive)");
        k_phase1 = st.k;
        if (st.status != 2 && st.status != kStInfeasible && st.k < o.max_outer) {
            DevParams p2 = par;
            p2.resume = 1;
            HIP_TRY(hipMemsetAsync(h->W.bar, 0, bar_words(h->cfg.nblocks) * sizeof(unsigned), h->stream));
            HIP_TRY(launch_dfom(h->dtype, DUQ_ACC_F64, h->cfg, gp, p2, W));
        }
    } else {
        HIP_TRY(launch_dfom(h->dtype, 0, h->cfg, gp, par, W));
    }
    HIP_TRY(hipEventRecord(h->ev1, h->stream));
    HIP_TRY(hipMemcpyAsync(&st, h->W.st, sizeof(DevState), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipMemcpyAsync(&bar_err, h->W.bar + kBarErr, sizeof(unsigned), hipMemcpyDeviceToHost, h->stream));
    if (x_out) HIP_TRY(hipMemcpyAsync(x_out, h->W.xout, n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    if (lam_out && p > 0)
        HIP_TRY(hipMemcpyAsync(lam_out, h->rows ? h->W.nu : h->W.lamp, p * sizeof(double), hipMemcpyDeviceToHost,
                               h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, h->ev0, h->ev1));
    if (bar_err) return fail(DUQ_EDEVICE, "grid barrier timeout (a workgroup did not arrive)");
    h->last_records = st.n_trace;
    int code = st.status == 0                ? DUQ_OK
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
        res->time_ms = ms;
        res->f64_outer_iters = two_phase ? st.k - k_phase1 : st.k;
        res->engine = h->engine;
        res->lam_min = h->lam_min;
        res->lam_max = h->lam_max;
        res->G_norm2 = h->G2;
    }
    if (code == DUQ_ENUMERIC) g_err = "non-finite value during the iteration";
    if (code == DUQ_EMAXITER) g_err = "max_outer reached";
    if (code == DUQ_EINFEASIBLE) g_err = "the constraints have no solution in the box (certificate returned as the multipliers)";
    return code;
}

namespace duq {

// Serving loop: run at most `slice` more outer iterations of a handle's solve
// (from the projection of 0 when `first`, else from the state the previous
// slice left), with FP64 accumulation, and queue the copy of the scalar state
// to `st_host`.  Nothing waits: the caller synchronises the stream.
int handle_slice(duq_handle* h, bool first, int slice, int k_done, DevState* st_host) {
    const duq_options& o = h->opts;
    if (first) HIP_TRY(hipMemsetAsync(h->W.st, 0, sizeof(DevState), h->stream));
    HIP_TRY(hipMemsetAsync(h->W.bar, 0, bar_words(h->cfg.nblocks) * sizeof(unsigned), h->stream));
    DevParams par{};
    par.method = o.method;
    par.output = o.output;
    par.inner_rule = o.inner_rule;
    par.inner_variant = h->variant;
    par.max_outer = std::min(o.max_outer, k_done + slice);
    par.k_in_max = h->k_in;
    par.Kd_nonneg = h->Kd_nonneg;
    par.resume = first ? 0 : 2;
    par.eps_out = o.eps_out;
    par.eps_in = o.eps_in;
    par.rho = o.rho;
    par.alpha = h->alpha;
    par.L = h->L_in;
    par.sigma = h->sigma;
    par.beta_in = h->beta_in;
    par.lb_cert = resolve_lb_cert(o.lb_cert);
    GenericProblem gp{h->n, h->p, h->dQ, h->dG, h->dq, h->dg, h->dlb, h->dub};
    gp.sp = h->sp;
    HIP_TRY(launch_dfom(h->dtype, DUQ_ACC_F64, h->cfg, gp, par, h->W));
    HIP_TRY(hipMemcpyAsync(st_host, h->W.st, sizeof(DevState), hipMemcpyDeviceToHost, h->stream));
    return DUQ_OK;
}

// Grid-barrier error flag of the last slice (read after the stream is idle).
int handle_barrier_error(duq_handle* h, unsigned* flag) {
    HIP_TRY(hipMemcpy(flag, h->W.bar + kBarErr, sizeof(unsigned), hipMemcpyDeviceToHost));
    return DUQ_OK;
}

// Copy the returned primal point and multipliers of the last slice.
int handle_outputs(duq_handle* h, double* x, double* lam) {
    if (x) HIP_TRY(hipMemcpy(x, h->W.xout, h->n * sizeof(double), hipMemcpyDeviceToHost));
    if (lam && h->p > 0) HIP_TRY(hipMemcpy(lam, h->W.lamp, h->p * sizeof(double), hipMemcpyDeviceToHost));
    return DUQ_OK;
}

// Derived solver parameters of a handle (what duq_solve passes its kernel).
void handle_params(duq_handle* h, DevParams* par) {
    const duq_options& o = h->opts;
    *par = DevParams{};
    par->method = o.method;
    par->output = o.output;
    par->inner_rule = o.inner_rule;
    par->inner_variant = h->variant;
    par->max_outer = o.max_outer;
    par->k_in_max = h->k_in;
    par->Kd_nonneg = h->Kd_nonneg;
    par->eps_out = o.eps_out;
    par->eps_in = o.eps_in;
    par->rho = o.rho;
    par->alpha = h->alpha;
    par->L = h->L_in;
    par->sigma = h->sigma;
    par->beta_in = h->beta_in;
    par->lb_cert = resolve_lb_cert(o.lb_cert);
}

// Constants and engine of a handle, for reporting.
void handle_info(duq_handle* h, double* lam_min, double* lam_max, double* g2, int* engine) {
    *lam_min = h->lam_min;
    *lam_max = h->lam_max;
    *g2 = h->G2;
    *engine = h->engine;
}

}  // namespace duq

extern "C" int duq_get_trace(duq_handle* h, double* out, int32_t max_records, int32_t* n_records) {
    if (!h || !out || max_records < 0) return fail(DUQ_EINVAL, "bad trace arguments");
    const int rec = std::min(std::min(h->last_records, h->trace_cap), (int)max_records);
    const size_t per = (size_t)(kTraceScalars + (h->rows ? 4 : 2) * h->p + h->n);
    if (rec > 0)
        HIP_TRY(hipMemcpy(out, h->W.trace, rec * per * sizeof(double), hipMemcpyDeviceToHost));
    if (n_records) *n_records = rec;
    return DUQ_OK;
}

// ---- parameter planning (Sec. 3.1 eq. choose_ein, Sec. 5) -----------------

extern "C" int duq_plan_params(int32_t method, double eps, double Ld, double Rd, double L_in, double sigma_in,
                               double D_U, duq_plan* out) {
    if (!out) return fail(DUQ_EINVAL, "null plan");
    if (method != DUQ_DGM && method != DUQ_DFGM) return fail(DUQ_EINVAL, "bad method");
    if (!(eps > 0.0) || !(Ld > 0.0) || !(Rd > 0.0) || !std::isfinite(eps) || !std::isfinite(Ld) ||
        !std::isfinite(Rd))
        return fail(DUQ_EINVAL, "eps, L_d and R_d must be finite and > 0");
    std::memset(out, 0, sizeof(*out));
    const double a = 8.0 * Ld * Rd * Rd / eps;
    double kout;
    if (method == DUQ_DGM) {
        out->eps_in = eps / 4.0;
        kout = std::ceil(a);
    } else {
        out->eps_in = eps * std::sqrt(eps) / (8.0 * Rd * std::sqrt(2.0 * Ld));
        kout = std::ceil(std::sqrt(a));
    }
    out->k_out = (int64_t)std::min(std::max(kout, 1.0), 9.0e18);
    out->rho_star = 8.0 * Rd * Rd / eps;
    if (L_in > 0.0 && D_U > 0.0) {
        double kin;
        if (sigma_in > 0.0) {
            const double arg = L_in * D_U * D_U / out->eps_in;
            kin = arg > 1.0 ? std::ceil(std::sqrt(L_in / sigma_in) * std::log(arg)) + 1.0 : 1.0;
        } else {
            kin = std::ceil(std::sqrt(2.0 * L_in * D_U * D_U / out->eps_in));
        }
        out->k_in = (int64_t)std::min(std::max(kin, 1.0), 9.0e18);
        out->k_total = out->k_in * out->k_out;
    }
    return DUQ_OK;
}

extern "C" int duq_solve_planned(duq_handle* h, double eps, double R0, int32_t max_rounds, double* x_out,
                                 double* lam_out, duq_result* res, double* R_out, int32_t* rounds_out) {
    if (!h || !x_out || (h->p > 0 && !lam_out)) return fail(DUQ_EINVAL, "null handle or output");
    if (!(eps > 0.0) || !(R0 > 0.0) || max_rounds < 1) return fail(DUQ_EINVAL, "eps, R0 > 0 and max_rounds >= 1");
    if (!(h->Ld > 0.0)) return fail(DUQ_EINVAL, "planning needs constraint rows (L_d > 0)");
    const duq_options saved = h->opts;
    const int saved_kin = h->k_in;
    double R = R0;
    int rounds = 0, code = DUQ_EMAXITER;
    long long outer = 0, inner = 0, gt_rows = 0;
    double ms = 0.0;
    duq_result r{};
    for (int rnd = 0; rnd < max_rounds; ++rnd) {
        duq_plan pl;
        int rc = duq_plan_params(saved.method, eps, h->Ld, R, 0.0, 0.0, 0.0, &pl);
        if (rc) break;
        h->opts.eps_out = eps;
        h->opts.eps_in = pl.eps_in;
        h->opts.max_outer = (int32_t)std::min<int64_t>(pl.k_out, INT32_MAX);
        DevParams dp;
        rc = derive_params(h->p, h->lam_min, h->lam_max, h->G2, h->D_U, h->opts, &dp, h->sigma);
        if (rc) {
            code = rc;
            break;
        }
        h->k_in = dp.k_in_max;
        const bool warm = rnd > 0;
        code = duq_solve(h, warm ? x_out : nullptr, (warm && !h->rows) ? lam_out : nullptr, x_out, lam_out, &r);
        ++rounds;
        if (code != DUQ_OK && code != DUQ_EMAXITER) break;
        outer += r.outer_iters;
        inner += r.inner_iters;
        gt_rows += r.gt_rows;
        ms += r.time_ms;
        if (code == DUQ_OK) break;
        R *= 2.0;
    }
    h->opts = saved;
    h->k_in = saved_kin;
    if (res) {
        *res = r;
        res->outer_iters = (int32_t)std::min<long long>(outer, INT32_MAX);
        res->inner_iters = inner;
        res->gt_rows = gt_rows;
        res->time_ms = ms;
        res->f64_outer_iters = res->outer_iters;
        res->status = code;
    }
    if (R_out) *R_out = R;
    if (rounds_out) *rounds_out = rounds;
    return code;
}
