// Host side of duq_solve_batch: validation, packing, work order, slots,
// one persistent launch, result transfer.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/duq.h"
#include "internal.h"
#include "launch.h"

using namespace duq;

namespace duq {
int set_error(int code, const std::string& msg);
int device_cus();
void handle_params(duq_handle* h, DevParams* par);
int resolve_lb_cert(int opt);
int derive_params(int p, double lam_min, double lam_max, double g2, double D_U, const duq_options& o,
                  DevParams* par, double sigma);
}

namespace {

// Launch shapes chosen by duq_tune_batch: (dtype, short-row class, largest n
// rounded up to 64) -> workgroups per CU.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, int> g_tune;

int tuned_wpc(int dtype, bool sh, int n_max) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(std::make_tuple(dtype, sh ? 1 : 0, (n_max + 63) / 64));
    return it == g_tune.end() ? 0 : it->second;
}

// Device workspace of the batched solves, kept per device between calls: a
// call takes the kept block when it is free and large enough (a larger
// request replaces it), a call that finds it in use allocates its own.  The
// block goes back only after the call's stream has drained, so the next call
// never sees it in use.  It is held until the process ends.
struct KeptWs {
    void* p = nullptr;
    size_t bytes = 0;
    bool busy = false;
};
std::mutex g_ws_mu;
std::map<int, KeptWs> g_ws;

struct DevBuf {
    void* p = nullptr;
    int dev = -1;                 // >= 0: the kept block of this device
    hipStream_t stream = nullptr;
    hipError_t alloc(size_t bytes, hipStream_t s) {
        stream = s;
        int d = 0;
        hipError_t e = hipGetDevice(&d);
        if (e != hipSuccess) return e;
        {
            std::lock_guard<std::mutex> lk(g_ws_mu);
            KeptWs& k = g_ws[d];
            if (!k.busy) {
                if (k.bytes < bytes) {
                    if (k.p) (void)hipFree(k.p);
                    k.p = nullptr;
                    k.bytes = 0;
                    if ((e = hipMalloc(&k.p, bytes)) != hipSuccess) {
                        k.p = nullptr;
                        return e;
                    }
                    k.bytes = bytes;
                }
                k.busy = true;
                p = k.p;
                dev = d;
                return hipSuccess;
            }
        }
        return hipMalloc(&p, bytes);
    }
    ~DevBuf() {
        if (!p) return;
        if (dev >= 0) {
            (void)hipStreamSynchronize(stream);
            std::lock_guard<std::mutex> lk(g_ws_mu);
            g_ws[dev].busy = false;
        } else {
            (void)hipFree(p);
        }
    }
};

// Events and streams released on every return path.
struct EventH {
    hipEvent_t e = nullptr;
    ~EventH() {
        if (e) (void)hipEventDestroy(e);
    }
};
struct StreamH {
    hipStream_t s = nullptr;
    ~StreamH() {
        if (s) {
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
        }
    }
};

#define BTRY(expr)                                                                                 \
    do {                                                                                           \
        hipError_t _e = (expr);                                                                    \
        if (_e != hipSuccess)                                                                      \
            return set_error(_e == hipErrorOutOfMemory ? DUQ_ENOMEM : DUQ_EDEVICE,                 \
                             std::string(#expr) + ": " + hipGetErrorString(_e));                   \
    } while (0)

template <typename T>
bool all_finite(const T* a, long long len) {
    for (long long i = 0; i < len; ++i)
        if (!std::isfinite((double)a[i])) return false;
    return true;
}

}  // namespace

namespace {

int to_status(int s) {
    return s == 0 ? DUQ_OK : s == 2 ? DUQ_ENUMERIC : s == 4 ? DUQ_EINVAL : s == kStInfeasible ? DUQ_EINFEASIBLE
                                                                                               : DUQ_EMAXITER;
}

// Shared-Hessian batch on the MFMA tile kernel: constants and derived
// parameters from the single-QP setup of the shared data (Lanczos estimate
// unless given), one persistent launch over tiles of 16 instances.
int solve_shared_tiles(const duq_batch* b, const duq_options* o, hipStream_t s, const void* dQ, const void* dG,
                       const double* dq, const double* dg, const double* dlb, const double* dub, int bpc,
                       double* X_out, double* Lam_out, duq_result* res) {
    const int B = b->B, n = b->n_shared, p = b->p_shared;
    duq_problem pr{n, p, b->dtype, DUQ_DEVICE, dQ, p ? dG : nullptr, dq, p ? dg : nullptr, dlb, dub};
    duq_options oo = *o;
    oo.trace_outer = 0;
    oo.engine = DUQ_ENGINE_BLOCK;
    const bool have_c = b->lam_min && b->lam_max && b->G_norm2;
    oo.lam_min = have_c ? b->lam_min[0] : 0.0;
    oo.lam_max = have_c ? b->lam_max[0] : 0.0;
    oo.G_norm2 = have_c ? b->G_norm2[0] : 0.0;
    TileLaunch t{};
    if (have_c && oo.lam_min > 0.0 && oo.lam_max > 0.0 && (p == 0 || oo.G_norm2 > 0.0)) {
        // given constants: derive the parameters here (D_U from the box)
        std::vector<double> lo(n), hi(n);
        BTRY(hipMemcpyAsync(lo.data(), dlb, 8 * (size_t)n, hipMemcpyDeviceToHost, s));
        BTRY(hipMemcpyAsync(hi.data(), dub, 8 * (size_t)n, hipMemcpyDeviceToHost, s));
        BTRY(hipStreamSynchronize(s));
        double du2 = 0.0;
        for (int i = 0; i < n; ++i) {
            if (!std::isfinite(lo[i]) || !std::isfinite(hi[i]) || lo[i] > hi[i])
                return set_error(DUQ_EINVAL, "box must be finite with lb <= ub");
            du2 += (hi[i] - lo[i]) * (hi[i] - lo[i]);
        }
        int rc = derive_params(p, oo.lam_min, oo.lam_max, p ? oo.G_norm2 : 0.0, std::sqrt(du2), oo, &t.par, 0.0);
        if (rc) return rc;
        t.lam_min = oo.lam_min;
        t.lam_max = oo.lam_max;
        t.g2 = p ? oo.G_norm2 : 0.0;
    } else {
        // Lanczos estimate and derivation through the single-QP setup
        duq_handle* h = nullptr;
        int rc = duq_setup(&pr, &oo, s, &h);
        if (rc) return rc;
        handle_params(h, &t.par);
        duq_get_constants(h, &t.lam_min, &t.lam_max, &t.g2, nullptr, nullptr, nullptr);
        duq_destroy(h);
    }
    const int pp = std::max(p, 1);
    DevBuf ws;
    size_t off = 0;
    auto plan = [&](size_t bytes) { size_t r = off; off += ((bytes + 255) / 256) * 256; return r; };
    const bool dev_out = o->out_memspace == DUQ_DEVICE;
    const size_t o_X = plan(dev_out ? 0 : 8 * (size_t)B * n);
    const size_t o_L = plan(dev_out ? 0 : 8 * (size_t)B * pp);
    const size_t o_res = plan(sizeof(BatchResultDev) * (size_t)B);
    const size_t o_dual = plan(8 * 3 * (size_t)B * pp);
    const size_t o_prim = plan(8 * 4 * (size_t)B * n);
    const size_t o_q = plan(256);
    BTRY(ws.alloc(off, s));
    char* w = (char*)ws.p;
    BTRY(hipMemsetAsync(w + o_q, 0, 256, s));
    t.B = B;
    t.n = n;
    t.p = p;
    t.Q = dQ;
    t.G = dG;
    t.q = dq;
    t.g = dg;
    t.lb = dlb;
    t.ub = dub;
    t.X = dev_out ? X_out : (double*)(w + o_X);
    t.Lam = dev_out ? Lam_out : (double*)(w + o_L);
    t.res = w + o_res;
    t.dual = (double*)(w + o_dual);
    t.prim = (double*)(w + o_prim);
    t.queue = (unsigned*)(w + o_q);
    const int tiles = (B + 15) / 16;
    const int nblocks = std::max(1, std::min(tiles, device_cus() * bpc));
    EventH e0, e1;
    BTRY(hipEventCreate(&e0.e));
    BTRY(hipEventCreate(&e1.e));
    BTRY(hipEventRecord(e0.e, s));
    hipError_t le = launch_tile(b->dtype, nblocks, tile_lds_bytes(n), s, t);
    BTRY(hipEventRecord(e1.e, s));
    std::vector<BatchResultDev> rd(B);
    if (le == hipSuccess) {
        BTRY(hipMemcpyAsync(rd.data(), w + o_res, sizeof(BatchResultDev) * B, hipMemcpyDeviceToHost, s));
        if (X_out && !dev_out) BTRY(hipMemcpyAsync(X_out, w + o_X, 8 * (size_t)B * n, hipMemcpyDeviceToHost, s));
        if (Lam_out && p > 0 && !dev_out)
            BTRY(hipMemcpyAsync(Lam_out, w + o_L, 8 * (size_t)B * p, hipMemcpyDeviceToHost, s));
    }
    hipError_t se = hipStreamSynchronize(s);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0.e, e1.e);
    BTRY(le);
    BTRY(se);
    int code = DUQ_OK;
    for (int i = 0; i < B; ++i) {
        const BatchResultDev& r = rd[i];
        const int st = to_status(r.status);
        if (st != DUQ_OK && code == DUQ_OK) code = st;
        if (res) {
            duq_result& q = res[i];
            std::memset(&q, 0, sizeof(q));
            q.status = st;
            q.outer_iters = r.outer;
            q.inner_iters = r.inner;
            q.gt_rows = r.gt_rows;
            q.f = r.F;
            q.lb_dual = r.LB;
            q.gap = r.F - r.LB;
            q.feas = r.feas;
            q.time_ms = ms;
            q.f64_outer_iters = r.outer;
            q.engine = DUQ_ENGINE_TILE;
            q.lam_min = r.lam_min;
            q.lam_max = r.lam_max;
            q.G_norm2 = r.G2;
        }
    }
    if (code != DUQ_OK) set_error(code, "at least one instance did not pass its outer test");
    return code;
}

}  // namespace

extern "C" int duq_solve_batch(const duq_batch* b, const duq_options* o, void* stream, double* X_out,
                               double* Lam_out, duq_result* res) {
    if (!b || !o) return set_error(DUQ_EINVAL, "null batch or options");
    const int B = b->B;
    if (B < 1) return set_error(DUQ_EINVAL, "B must be >= 1");
    if (b->kind != DUQ_BATCH_UNEVEN && b->kind != DUQ_BATCH_SHARED) return set_error(DUQ_EINVAL, "bad kind");
    if (b->dtype != DUQ_F64 && b->dtype != DUQ_F32) return set_error(DUQ_EINVAL, "dtype must be F64 or F32");
    if (b->memspace != DUQ_HOST && b->memspace != DUQ_DEVICE) return set_error(DUQ_EINVAL, "bad memspace");
    if (!(o->eps_out > 0.0) || !(o->eps_in > 0.0) || !(o->rho >= 0.0) || o->max_outer < 1 || o->max_inner < 0)
        return set_error(DUQ_EINVAL, "bad options");
    if (o->method != DUQ_DGM && o->method != DUQ_DFGM) return set_error(DUQ_EINVAL, "bad method");
    if (o->output != DUQ_LAST && o->output != DUQ_AVG) return set_error(DUQ_EINVAL, "bad output");
    if (o->inner_variant < 0 || o->inner_variant > 3) return set_error(DUQ_EINVAL, "bad inner_variant");
    if (o->accumulate != DUQ_ACC_F64) return set_error(DUQ_EINVAL, "batches accumulate in FP64");
    if (o->out_memspace != DUQ_HOST && o->out_memspace != DUQ_DEVICE) return set_error(DUQ_EINVAL, "bad out_memspace");
    if (o->out_memspace == DUQ_DEVICE && (!X_out || !Lam_out))
        return set_error(DUQ_EINVAL, "device outputs need X_out and Lam_out");
    if (!b->Q || !b->q || !b->lb || !b->ub) return set_error(DUQ_EINVAL, "null data pointer");
    const bool shared = b->kind == DUQ_BATCH_SHARED;
    const size_t es = b->dtype == DUQ_F64 ? 8 : 4;
    hipStream_t s = (hipStream_t)stream;

    // sizes and offsets (host metadata)
    std::vector<int> ns(B), ps(B);
    std::vector<long long> qo(B), go(B), vo(B), co(B);
    long long qtot = 0, gtot = 0, vtot = 0, ctot = 0;
    int n_max = 0, p_max = 0;
    if (shared) {
        if (b->n_shared < 1 || b->p_shared < 0) return set_error(DUQ_EINVAL, "bad shared sizes");
        if (b->p_shared > 0 && (!b->G || !b->g)) return set_error(DUQ_EINVAL, "null G or g");
        n_max = b->n_shared;
        p_max = b->p_shared;
        for (int i = 0; i < B; ++i) {
            ns[i] = n_max;
            ps[i] = p_max;
            vo[i] = (long long)i * n_max;
            co[i] = (long long)i * p_max;
        }
        qtot = (long long)n_max * n_max;
        gtot = (long long)p_max * n_max;
        vtot = (long long)B * n_max;
        ctot = (long long)B * p_max;
    } else {
        if (!b->n || !b->p || !b->qoff || !b->goff || !b->voff || !b->coff)
            return set_error(DUQ_EINVAL, "null size/offset arrays");
        for (int i = 0; i < B; ++i) {
            ns[i] = b->n[i];
            ps[i] = b->p[i];
            qo[i] = b->qoff[i];
            go[i] = b->goff[i];
            vo[i] = b->voff[i];
            co[i] = b->coff[i];
            if (ns[i] < 1 || ps[i] < 0 || qo[i] < 0 || go[i] < 0 || vo[i] < 0 || co[i] < 0)
                return set_error(DUQ_EINVAL, "bad size or offset of instance " + std::to_string(i));
            n_max = std::max(n_max, ns[i]);
            p_max = std::max(p_max, ps[i]);
            qtot = std::max(qtot, qo[i] + (long long)ns[i] * ns[i]);
            gtot = std::max(gtot, go[i] + (long long)ps[i] * ns[i]);
            vtot = std::max(vtot, vo[i] + ns[i]);
            ctot = std::max(ctot, co[i] + ps[i]);
        }
        if (gtot > 0 && (!b->G || !b->g)) return set_error(DUQ_EINVAL, "null G or g");
    }
    const long long lbn = shared ? n_max : vtot;

    // device data: copy (HOST) or borrow (DEVICE)
    DevBuf data;
    const void *dQ = b->Q, *dG = b->G;
    const double *dq = b->q, *dg = b->g, *dlb = b->lb, *dub = b->ub;
    if (b->memspace == DUQ_HOST) {
        bool ok = (b->dtype == DUQ_F64 ? all_finite((const double*)b->Q, qtot) : all_finite((const float*)b->Q, qtot));
        if (gtot > 0)
            ok = ok && (b->dtype == DUQ_F64 ? all_finite((const double*)b->G, gtot)
                                            : all_finite((const float*)b->G, gtot));
        ok = ok && all_finite(b->q, vtot) && (ctot == 0 || all_finite(b->g, ctot));
        if (!ok) return set_error(DUQ_EINVAL, "non-finite batch data");
        for (long long j = 0; j < lbn; ++j)
            if (!std::isfinite(b->lb[j]) || !std::isfinite(b->ub[j]) || b->lb[j] > b->ub[j])
                return set_error(DUQ_EINVAL, "box must be finite with lb <= ub");
        const size_t bytes = qtot * es + std::max<long long>(gtot, 1) * es + 8 * (vtot + std::max<long long>(ctot, 1) + 2 * lbn) + 6 * 256;
        BTRY(hipMalloc(&data.p, bytes));
        char* c = (char*)data.p;
        auto take = [&](size_t n) { char* r = c; c += ((n + 255) / 256) * 256; return r; };
        char* Qd = take(qtot * es);
        char* Gd = take(std::max<long long>(gtot, 1) * es);
        double* qd = (double*)take(8 * vtot);
        double* gd = (double*)take(8 * std::max<long long>(ctot, 1));
        double* lbd = (double*)take(8 * lbn);
        double* ubd = (double*)take(8 * lbn);
        BTRY(hipMemcpyAsync(Qd, b->Q, qtot * es, hipMemcpyHostToDevice, s));
        if (gtot > 0) BTRY(hipMemcpyAsync(Gd, b->G, gtot * es, hipMemcpyHostToDevice, s));
        BTRY(hipMemcpyAsync(qd, b->q, 8 * vtot, hipMemcpyHostToDevice, s));
        if (ctot > 0) BTRY(hipMemcpyAsync(gd, b->g, 8 * ctot, hipMemcpyHostToDevice, s));
        BTRY(hipMemcpyAsync(lbd, b->lb, 8 * lbn, hipMemcpyHostToDevice, s));
        BTRY(hipMemcpyAsync(ubd, b->ub, 8 * lbn, hipMemcpyHostToDevice, s));
        dQ = Qd; dG = Gd; dq = qd; dg = gd; dlb = lbd; dub = ubd;
    }

    // shared-Hessian batches on MFMA tiles (rho = 0, n small enough for Q in LDS)
    if (shared && o->engine != DUQ_ENGINE_BLOCK && o->engine != DUQ_ENGINE_GRID) {
        int bpc = 0;
        const bool fits = o->rho == 0.0 && n_max <= kTileMaxN &&
                          tile_occupancy(b->dtype, tile_lds_bytes(n_max), &bpc) == hipSuccess && bpc >= 1;
        if (fits) return solve_shared_tiles(b, o, s, dQ, dG, dq, dg, dlb, dub, bpc, X_out, Lam_out, res);
        if (o->engine == DUQ_ENGINE_TILE)
            return set_error(DUQ_EINVAL, "the MFMA tile engine needs rho = 0 and n <= 128");
        (void)hipGetLastError();
    }
    if (o->engine == DUQ_ENGINE_TILE) return set_error(DUQ_EINVAL, "the MFMA tile engine serves shared batches");

    // constants: per instance from the caller, or one estimate for a shared batch
    const bool have_c = b->lam_min && b->lam_max && b->G_norm2;
    const int nc = shared ? 1 : B;
    std::vector<double> cmin(nc), cmax(nc), cg2(nc);
    bool dev_consts = have_c;
    if (have_c) {
        for (int i = 0; i < nc; ++i) {
            cmin[i] = b->lam_min[i];
            cmax[i] = b->lam_max[i];
            cg2[i] = b->G_norm2[i];
        }
    } else if (shared) {
        duq_problem pr{n_max, p_max, b->dtype, DUQ_DEVICE, dQ, p_max ? dG : nullptr, dq, p_max ? dg : nullptr, dlb, dub};
        duq_options oo = *o;
        oo.lam_min = oo.lam_max = oo.G_norm2 = 0.0;
        oo.trace_outer = 0;
        duq_handle* h = nullptr;
        int rc = duq_setup(&pr, &oo, stream, &h);
        if (rc) return rc;
        duq_get_constants(h, &cmin[0], &cmax[0], &cg2[0], nullptr, nullptr, nullptr);
        duq_destroy(h);
        dev_consts = true;
    }

    // processing order: largest work first, long-row instances and
    // short-row instances (separate kernels) each in that order
    std::vector<int> order(B);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
        const long long wa = (long long)ns[a] * ns[a] + (long long)ps[a] * ns[a];
        const long long wc = (long long)ns[c] * ns[c] + (long long)ps[c] * ns[c];
        return wa > wc;
    });
    std::stable_partition(order.begin(), order.end(), [&](int i) { return !batch_short_class(b->dtype, ns[i]); });

    const int k_req = o->lanczos_steps > 0 ? o->lanczos_steps : 96;
    struct Cls {
        bool sh;
        int first = 0, count = 0, n_max = 1, p_max = 0, k = 0, nblocks = 0;
        size_t shmem = 0;
        long long slot = 0;
        size_t o_slots = 0;
    } cls[2];
    cls[0].sh = false;
    cls[1].sh = true;
    for (int q = 0; q < B; ++q) {
        Cls& c = cls[batch_short_class(b->dtype, ns[order[q]]) ? 1 : 0];
        if (c.count == 0) c.first = q;
        ++c.count;
        c.n_max = std::max(c.n_max, ns[order[q]]);
        c.p_max = std::max(c.p_max, ps[order[q]]);
    }
    for (Cls& c : cls) {
        if (!c.count) continue;
        c.k = std::min(k_req, c.n_max);
        c.shmem = batch_lds_bytes(c.n_max, c.p_max, c.k);
        int bpc = 0;
        BTRY(batch_occupancy(b->dtype, c.sh, false, c.shmem, &bpc));
        if (bpc < 1) return set_error(DUQ_EINVAL, "batch instance too large for one workgroup's LDS");
        // workgroups per CU: the caller's, else the tuned one, else all that fit
        int wpc = o->batch_wpc > 0 ? o->batch_wpc : tuned_wpc(b->dtype, c.sh, c.n_max);
        wpc = wpc > 0 ? std::min(wpc, bpc) : bpc;
        c.nblocks = std::max(1, std::min(c.count, device_cus() * wpc));
        c.slot = batch_slot_bytes_host(c.n_max, c.p_max, c.k);
    }

    // device workspace
    DevBuf ws;
    size_t off = 0;
    auto plan = [&](size_t n) { size_t r = off; off += ((n + 255) / 256) * 256; return r; };
    for (Cls& c : cls) c.o_slots = plan((size_t)c.slot * c.nblocks);
    const bool dev_out = o->out_memspace == DUQ_DEVICE;
    const size_t o_X = plan(dev_out ? 0 : 8 * vtot);
    const size_t o_L = plan(dev_out ? 0 : 8 * std::max<long long>(ctot, 1));
    const size_t o_res = plan(sizeof(BatchResultDev) * B);
    const size_t o_meta = plan((sizeof(int) * 3 + sizeof(long long) * 4) * B);
    const size_t o_c = plan(8 * 3 * nc);
    const size_t o_q = plan(256);
    BTRY(ws.alloc(off, s));
    char* w = (char*)ws.p;
    int* d_order = (int*)(w + o_meta);
    int* d_n = d_order + B;
    int* d_p = d_n + B;
    long long* d_off = (long long*)(w + o_meta + ((sizeof(int) * 3 * B + 7) / 8) * 8);
    std::vector<char> meta(o_c - o_meta, 0);
    std::memcpy(meta.data(), order.data(), sizeof(int) * B);
    std::memcpy(meta.data() + sizeof(int) * B, ns.data(), sizeof(int) * B);
    std::memcpy(meta.data() + 2 * sizeof(int) * B, ps.data(), sizeof(int) * B);
    char* mo = meta.data() + ((sizeof(int) * 3 * B + 7) / 8) * 8;
    std::memcpy(mo, qo.data(), 8 * B);
    std::memcpy(mo + 8 * B, go.data(), 8 * B);
    std::memcpy(mo + 16 * B, vo.data(), 8 * B);
    std::memcpy(mo + 24 * B, co.data(), 8 * B);
    BTRY(hipMemcpyAsync(w + o_meta, meta.data(), meta.size(), hipMemcpyHostToDevice, s));
    double* d_c = (double*)(w + o_c);
    if (dev_consts) {
        std::vector<double> cc(3 * nc);
        std::copy(cmin.begin(), cmin.end(), cc.begin());
        std::copy(cmax.begin(), cmax.end(), cc.begin() + nc);
        std::copy(cg2.begin(), cg2.end(), cc.begin() + 2 * nc);
        BTRY(hipMemcpyAsync(d_c, cc.data(), 8 * 3 * nc, hipMemcpyHostToDevice, s));
    }
    BTRY(hipMemsetAsync(w + o_q, 0, 256, s));

    BatchLaunch L{};
    L.shared = shared ? 1 : 0;
    L.n = d_n;
    L.p = d_p;
    L.qoff = d_off;
    L.goff = d_off + B;
    L.voff = d_off + 2 * B;
    L.coff = d_off + 3 * B;
    L.n_shared = n_max;
    L.p_shared = p_max;
    L.Q = dQ;
    L.G = dG;
    L.q = dq;
    L.g = dg;
    L.lb = dlb;
    L.ub = dub;
    L.lam_min = dev_consts ? d_c : nullptr;
    L.lam_max = dev_consts ? d_c + nc : nullptr;
    L.g2 = dev_consts ? d_c + 2 * nc : nullptr;
    L.X = dev_out ? X_out : (double*)(w + o_X);
    L.Lam = dev_out ? Lam_out : (double*)(w + o_L);
    L.res = w + o_res;
    DevParams par{};
    par.method = o->method;
    par.output = o->output;
    par.inner_rule = o->inner_rule;
    par.inner_variant = o->inner_variant;
    par.max_outer = o->max_outer;
    par.eps_out = o->eps_out;
    par.eps_in = o->eps_in;
    par.rho = o->rho;
    par.lb_cert = resolve_lb_cert(o->lb_cert);
    L.base = par;
    L.max_inner = o->max_inner;
    L.lanczos_k = k_req;
    L.safety = o->safety;

    // the two classes run concurrently: long rows on `s`, short rows on a
    // second stream joined back to `s`
    const bool both = cls[0].count > 0 && cls[1].count > 0;
    StreamH side;
    EventH fork, join, e0, e1;
    BTRY(hipEventCreate(&e0.e));
    BTRY(hipEventCreate(&e1.e));
    BTRY(hipEventRecord(e0.e, s));
    if (both) {
        BTRY(hipStreamCreateWithFlags(&side.s, hipStreamNonBlocking));
        BTRY(hipEventCreateWithFlags(&fork.e, hipEventDisableTiming));
        BTRY(hipEventCreateWithFlags(&join.e, hipEventDisableTiming));
        BTRY(hipEventRecord(fork.e, s));
        BTRY(hipStreamWaitEvent(side.s, fork.e, 0));
    }
    hipStream_t s2 = both ? side.s : s;
    hipError_t le = hipSuccess;
    for (int ci = 0; ci < 2 && le == hipSuccess; ++ci) {
        const Cls& c = cls[ci];
        if (!c.count) continue;
        BatchLaunch Lc = L;
        Lc.B = c.count;
        Lc.order = d_order + c.first;
        Lc.lanczos_alloc = c.k;
        Lc.slots = w + c.o_slots;
        Lc.slot_bytes = c.slot;
        Lc.n_max = c.n_max;
        Lc.p_max = c.p_max;
        Lc.queue = (unsigned*)(w + o_q) + ci;
        le = launch_batch(b->dtype, c.sh, c.nblocks, c.shmem, ci == 1 ? s2 : s, Lc);
    }
    if (both) {
        hipError_t je = hipEventRecord(join.e, s2);
        if (je == hipSuccess) je = hipStreamWaitEvent(s, join.e, 0);
        if (le == hipSuccess) le = je;
    }
    BTRY(hipEventRecord(e1.e, s));
    std::vector<BatchResultDev> rd(B);
    if (le == hipSuccess) {
        BTRY(hipMemcpyAsync(rd.data(), w + o_res, sizeof(BatchResultDev) * B, hipMemcpyDeviceToHost, s));
        if (X_out && !dev_out) BTRY(hipMemcpyAsync(X_out, w + o_X, 8 * vtot, hipMemcpyDeviceToHost, s));
        if (Lam_out && ctot > 0 && !dev_out)
            BTRY(hipMemcpyAsync(Lam_out, w + o_L, 8 * ctot, hipMemcpyDeviceToHost, s));
    }
    hipError_t se = hipStreamSynchronize(s);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0.e, e1.e);
    BTRY(le);
    BTRY(se);
    int code = DUQ_OK;
    for (int i = 0; i < B; ++i) {
        const BatchResultDev& r = rd[i];
        const int st = to_status(r.status);
        if (st != DUQ_OK && code == DUQ_OK) code = st;
        if (res) {
            duq_result& q = res[i];
            std::memset(&q, 0, sizeof(q));
            q.status = st;
            q.outer_iters = r.outer;
            q.inner_iters = r.inner;
            q.gt_rows = r.gt_rows;
            q.f = r.F;
            q.lb_dual = r.LB;
            q.gap = r.F - r.LB;
            q.feas = r.feas;
            q.time_ms = ms;
            q.f64_outer_iters = r.outer;
            q.engine = DUQ_ENGINE_BLOCK;
            q.lam_min = r.lam_min;
            q.lam_max = r.lam_max;
            q.G_norm2 = r.G2;
        }
    }
    if (code != DUQ_OK) set_error(code, "at least one instance did not pass its outer test");
    return code;
}

// ---- launch-shape tuning ------------------------------------------------------

extern "C" int duq_tune_batch(const duq_batch* b, const duq_options* o, void* stream, int32_t* best_wpc,
                              double* ms_out) {
    if (!b || !o || !best_wpc) return set_error(DUQ_EINVAL, "null argument");
    if (b->kind != DUQ_BATCH_UNEVEN) return set_error(DUQ_EINVAL, "tuning takes an uneven batch");
    if (b->B < 1 || !b->n || !b->p) return set_error(DUQ_EINVAL, "empty batch");
    if (ms_out)
        for (int i = 0; i < 3; ++i) ms_out[i] = 0.0;
    long long vtot = 0, ctot = 0;
    for (int i = 0; i < b->B; ++i) {
        vtot = std::max<long long>(vtot, b->voff[i] + b->n[i]);
        ctot = std::max<long long>(ctot, b->coff[i] + b->p[i]);
    }
    std::vector<double> X0, L0, X1, L1;
    std::vector<duq_result> r0(b->B), r1(b->B);
    double best_ms = 0.0;
    int best = 0;
    for (int wpc = 1; wpc <= 3; ++wpc) {
        duq_options oo = *o;
        oo.batch_wpc = wpc;
        oo.out_memspace = DUQ_HOST;
        oo.engine = DUQ_ENGINE_BLOCK;
        std::vector<double>& X = best ? X1 : X0;
        std::vector<double>& L = best ? L1 : L0;
        std::vector<duq_result>& r = best ? r1 : r0;
        X.assign(std::max<long long>(vtot, 1), 0.0);
        L.assign(std::max<long long>(ctot, 1), 0.0);
        const int rc = duq_solve_batch(b, &oo, stream, X.data(), L.data(), r.data());
        if (rc != DUQ_OK && rc != DUQ_EMAXITER && rc != DUQ_ENUMERIC && rc != DUQ_EINFEASIBLE) return rc;
        const double ms = r[0].time_ms;
        if (ms_out) ms_out[wpc - 1] = ms;
        if (best) {
            // the shape must not change any result
            const bool same = std::memcmp(X0.data(), X1.data(), 8 * X0.size()) == 0 &&
                              std::memcmp(L0.data(), L1.data(), 8 * L0.size()) == 0;
            bool cnt = true;
            for (int i = 0; i < b->B; ++i)
                cnt = cnt && r0[i].outer_iters == r1[i].outer_iters && r0[i].inner_iters == r1[i].inner_iters;
            if (!same || !cnt)
                return set_error(DUQ_EDEVICE, "tuning: results differ between launch shapes");
        }
        if (!best || ms < best_ms) {
            best_ms = ms;
            best = wpc;
        }
    }
    // record the choice for both row classes present in the batch
    std::lock_guard<std::mutex> lk(g_tune_mu);
    int nmax[2] = {0, 0};
    for (int i = 0; i < b->B; ++i) {
        const int sh = batch_short_class(b->dtype, b->n[i]) ? 1 : 0;
        nmax[sh] = std::max(nmax[sh], b->n[i]);
    }
    for (int sh = 0; sh < 2; ++sh)
        if (nmax[sh] > 0) g_tune[std::make_tuple(b->dtype, sh, (nmax[sh] + 63) / 64)] = best;
    *best_wpc = best;
    return DUQ_OK;
}

extern "C" int duq_tune_save(const char* path) {
    if (!path) return set_error(DUQ_EINVAL, "null path");
    FILE* f = std::fopen(path, "w");
    if (!f) return set_error(DUQ_EINVAL, std::string("cannot write ") + path);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto& kv : g_tune)
        std::fprintf(f, "%d %d %d %d\n", std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), kv.second);
    std::fclose(f);
    return DUQ_OK;
}

extern "C" int duq_tune_load(const char* path) {
    if (!path) return set_error(DUQ_EINVAL, "null path");
    FILE* f = std::fopen(path, "r");
    if (!f) return set_error(DUQ_EINVAL, std::string("cannot read ") + path);
    int dt, sh, nb, w;
    std::map<std::tuple<int, int, int>, int> t;
    int got;
    while ((got = std::fscanf(f, "%d %d %d %d", &dt, &sh, &nb, &w)) == 4) {
        if ((dt != DUQ_F64 && dt != DUQ_F32) || (sh != 0 && sh != 1) || nb < 1 || w < 1 || w > 3) {
            std::fclose(f);
            return set_error(DUQ_EINVAL, "bad tuning record");
        }
        t[std::make_tuple(dt, sh, nb)] = w;
    }
    const bool eof = got == EOF;
    std::fclose(f);
    if (!eof) return set_error(DUQ_EINVAL, "bad tuning file");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto& kv : t) g_tune[kv.first] = kv.second;
    return DUQ_OK;
}
