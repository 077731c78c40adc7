// Serving loop behind duq_server_create / duq_register_shared / duq_submit /
// duq_poll: a host thread that admits requests into a device arena by
// footprint, runs time-sliced rounds of the batch kernel (and of the
// single-QP engine for large requests), retires finished requests and
// backfills.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/duq.h"
#include "batch.h"
#include "internal.h"
#include "launch.h"

using namespace duq;

namespace duq {
int set_error(int code, const std::string& msg);
int device_cus();
int handle_slice(duq_handle* h, bool first, int slice, int k_done, DevState* st_host);
int handle_barrier_error(duq_handle* h, unsigned* flag);
int handle_outputs(duq_handle* h, double* x, double* lam);
int resolve_lb_cert(int opt);
void handle_info(duq_handle* h, double* lam_min, double* lam_max, double* g2, int* engine);
void handle_params(duq_handle* h, DevParams* par);
}  // namespace duq
size_t solver_workspace_bytes(int n, int p, int nblocks);
int setup_lent(const duq_problem* pr, const duq_options* opts, void* stream, void* ws, size_t ws_bytes,
               duq_handle** out);

namespace {

using Clock = std::chrono::steady_clock;

constexpr size_t kAlign = 256;
size_t up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over one device allocation; free blocks are merged
// with their neighbours.  Host bookkeeping only.
class Arena {
public:
    void init(char* base, size_t bytes) {
        base_ = base;
        size_ = bytes;
        free_.clear();
        free_[0] = bytes;
    }
    char* alloc(size_t bytes) {
        bytes = up(std::max<size_t>(bytes, 1));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > bytes) free_[off + bytes] = len - bytes;
            return base_ + off;
        }
        return nullptr;
    }
    void release(char* p, size_t bytes) {
        bytes = up(std::max<size_t>(bytes, 1));
        size_t off = (size_t)(p - base_);
        auto nx = free_.lower_bound(off);
        if (nx != free_.end() && off + bytes == nx->first) {
            bytes += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == off) {
                pv->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }
    size_t size() const { return size_; }

private:
    char* base_ = nullptr;
    size_t size_ = 0;
    std::map<size_t, size_t> free_;
};

struct Shared {
    int n, p, dtype;
    char* mem;
    size_t bytes;
    const void* Q;
    const void* G;
    const double *lb, *ub;
    double lam_min, lam_max, g2;
    DevParams par{};   // derived once at registration
    bool tile = false; // its requests run on the MFMA tiles (rho = 0, n <= kTileMaxN)
};

enum { ST_PENDING = 0, ST_ACTIVE = 1, ST_DONE = 2 };

struct Req {
    uint64_t ticket = 0;
    int shared_id = -1;
    int n = 0, p = 0, dtype = 0;
    bool large = false;
    int state = ST_PENDING;
    // host copies of the request data (released once uploaded)
    std::vector<char> Q, G;
    std::vector<double> q, g, lb, ub;
    // device placement
    char* mem = nullptr;
    size_t bytes = 0;
    ServeInst inst{};
    duq_handle* h = nullptr;
    DevState* st = nullptr;   // pinned copy of the large path's state
    int k_done = 0;
    // result
    duq_result res{};
    int code = DUQ_OK;
    std::string err;
    std::vector<double> x, lam;
    Clock::time_point t_submit, t_done;
};

int to_code(int status) {
    return status == 0 ? DUQ_OK
           : status == 2 ? DUQ_ENUMERIC
           : status == 4 ? DUQ_EINVAL
           : status == kStInfeasible ? DUQ_EINFEASIBLE
                                     : DUQ_EMAXITER;
}

template <typename T>
bool finite_all(const T* a, long long len) {
    for (long long i = 0; i < len; ++i)
        if (!std::isfinite((double)a[i])) return false;
    return true;
}

}  // namespace

struct duq_server {
    duq_options opts{};
    int device = 0;
    int cus = 1;
    int slice = 16;
    int k_req = 96;
    hipStream_t stream = nullptr;
    hipStream_t reg_stream = nullptr;
    char* arena_mem = nullptr;
    Arena arena;
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    int fatal = DUQ_OK;
    std::string fatal_msg;
    uint64_t next_ticket = 1;
    std::deque<Req*> pending;        // requests for the batch kernel
    std::deque<Req*> pending_large;  // requests for the single-QP engine
    std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
    std::vector<Shared> shared;
    std::thread th;
    // server-thread state
    std::vector<Req*> active;
    void* meta = nullptr;       // device: inst table, order, results, queue
    size_t meta_cap = 0;
    void* tile_ws = nullptr;    // device: gathered q, g, tile outputs and state
    size_t tile_ws_cap = 0;
    char* hmeta = nullptr;      // pinned host mirror
    size_t hmeta_cap = 0;
};

namespace {

size_t footprint(const duq_server* s, int n, int p, int dtype, bool own, bool large, int* k_out) {
    const size_t es = dtype == DUQ_F64 ? 8 : 4;
    const int pp = std::max(p, 1);
    size_t b = 0;
    if (own) b += up((size_t)n * n * es) + up((size_t)pp * n * es) + 2 * up(8 * (size_t)n);   // Q G lb ub
    b += up(8 * (size_t)n) + up(8 * (size_t)pp);                                                // q g
    const bool given = s->opts.lam_min > 0 && s->opts.lam_max > 0 && (p == 0 || s->opts.G_norm2 > 0);
    const int k = (!own || given) ? 0 : std::min(s->k_req, n);
    if (k_out) *k_out = k;
    if (large) {
        // the single-QP engine's workspace, lent to its setup from this block
        // (grid engine above DUQ_SERVE_BATCH_NMAX: one workgroup per CU)
        const int nb = n > DUQ_SERVE_BATCH_NMAX ? std::min(s->cus, n) : 1;
        b += up(solver_workspace_bytes(n, p, nb));
    } else {
        b += up(8 * (size_t)n) + up(8 * (size_t)pp);                                            // x lam
        b += up((size_t)batch_slot_bytes(n, p, k));
    }
    return b;
}

void finish(duq_server* s, Req* r, int code, const std::string& err) {
    if (r->mem) s->arena.release(r->mem, r->bytes);
    r->mem = nullptr;
    if (r->h) duq_destroy(r->h);
    r->h = nullptr;
    if (r->st) (void)hipHostFree(r->st);
    r->st = nullptr;
    r->code = code;
    r->err = err;
    r->t_done = Clock::now();
    r->res.status = code;
    r->res.time_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
    r->state = ST_DONE;
}

// Place an admitted request in its arena block and queue the uploads.
int place(duq_server* s, Req* r) {
    char* c = r->mem;
    auto take = [&](size_t b) { char* o = c; c += up(b); return o; };
    const size_t es = r->dtype == DUQ_F64 ? 8 : 4;
    const int n = r->n, p = r->p, pp = std::max(p, 1);
    hipError_t e = hipSuccess;
    ServeInst& in = r->inst;
    if (r->shared_id < 0) {
        char* Q = take((size_t)n * n * es);
        char* G = take((size_t)pp * n * es);
        double* lb = (double*)take(8 * (size_t)n);
        double* ub = (double*)take(8 * (size_t)n);
        e = e ? e : hipMemcpyAsync(Q, r->Q.data(), r->Q.size(), hipMemcpyHostToDevice, s->stream);
        if (p > 0) e = e ? e : hipMemcpyAsync(G, r->G.data(), r->G.size(), hipMemcpyHostToDevice, s->stream);
        e = e ? e : hipMemcpyAsync(lb, r->lb.data(), 8 * n, hipMemcpyHostToDevice, s->stream);
        e = e ? e : hipMemcpyAsync(ub, r->ub.data(), 8 * n, hipMemcpyHostToDevice, s->stream);
        in.Q = Q;
        in.G = G;
        in.lb = lb;
        in.ub = ub;
    } else {
        const Shared& sh = s->shared[r->shared_id];
        in.Q = sh.Q;
        in.G = sh.G;
        in.lb = sh.lb;
        in.ub = sh.ub;
    }
    double* q = (double*)take(8 * (size_t)n);
    double* g = (double*)take(8 * (size_t)pp);
    e = e ? e : hipMemcpyAsync(q, r->q.data(), 8 * n, hipMemcpyHostToDevice, s->stream);
    if (p > 0) e = e ? e : hipMemcpyAsync(g, r->g.data(), 8 * p, hipMemcpyHostToDevice, s->stream);
    in.q = q;
    in.g = g;
    in.n = n;
    in.p = p;
    if (e != hipSuccess) return set_error(DUQ_EDEVICE, std::string("upload: ") + hipGetErrorString(e));
    if (r->large) {
        // the uploads above must have landed before duq_setup reads lb, ub and
        // scans the data
        if ((e = hipStreamSynchronize(s->stream)) != hipSuccess)
            return set_error(DUQ_EDEVICE, std::string("upload: ") + hipGetErrorString(e));
        duq_problem pr{n, p, r->dtype, DUQ_DEVICE, in.Q, p ? in.G : nullptr, q, p ? g : nullptr, in.lb, in.ub};
        duq_options o = s->opts;
        o.trace_outer = 0;
        o.engine = DUQ_ENGINE_AUTO;
        // the solver workspace is the rest of the request's block
        int rc = setup_lent(&pr, &o, s->stream, c, r->bytes - (size_t)(c - r->mem), &r->h);
        if (rc) return rc;
        if (hipHostMalloc((void**)&r->st, sizeof(DevState), hipHostMallocDefault) != hipSuccess)
            return set_error(DUQ_ENOMEM, "pinned state");
        return DUQ_OK;
    }
    in.x = (double*)take(8 * (size_t)n);
    in.lam = (double*)take(8 * (size_t)pp);
    in.slot = c;
    in.resume = 0;
    if (r->shared_id >= 0) {
        const Shared& sh = s->shared[r->shared_id];
        in.given = 1;
        in.k = 0;
        in.lam_min = sh.lam_min;
        in.lam_max = sh.lam_max;
        in.g2 = sh.g2;
    } else {
        const duq_options& o = s->opts;
        in.given = (o.lam_min > 0 && o.lam_max > 0 && (p == 0 || o.G_norm2 > 0)) ? 1 : 0;
        in.k = in.given ? 0 : std::min(s->k_req, n);
        in.lam_min = o.lam_min;
        in.lam_max = o.lam_max;
        in.g2 = o.G_norm2;
    }
    return DUQ_OK;
}

// Admit pending requests in arrival order while they fit (called with the
// lock held).  Large requests use the whole device in their slices, so one is
// active at a time; they queue apart and do not hold back small ones.
void admit(duq_server* s) {
    int large_active = 0;
    for (Req* r : s->active) large_active += r->large ? 1 : 0;
    for (int q = 0; q < 2; ++q) {
        std::deque<Req*>& dq = q == 0 ? s->pending : s->pending_large;
        while (!dq.empty() && (q == 0 || large_active == 0)) {
            Req* r = dq.front();
            char* m = s->arena.alloc(r->bytes);
            if (!m) {
                if (!s->active.empty()) break;   // wait for retirements
                // nothing will be freed: it cannot fit now
                dq.pop_front();
                finish(s, r, DUQ_ENOMEM, "request does not fit the arena");
                continue;
            }
            dq.pop_front();
            r->mem = m;
            const int rc = place(s, r);
            if (rc) {
                finish(s, r, rc, std::string("admission failed: ") + duq_last_error());
                continue;
            }
            r->state = ST_ACTIVE;
            s->active.push_back(r);
            large_active += r->large ? 1 : 0;
        }
    }
}

// Every constant a request carries into a slice must be finite and positive
// (lambda_min may be 0 only with rho > 0, Sec. 2 Case 2; ||G||^2 is 0 only
// without rows).
bool constants_ok(const ServeInst& in, double rho) {
    const bool lmin_ok = std::isfinite(in.lam_min) && (in.lam_min > 0.0 || (rho > 0.0 && in.lam_min >= 0.0));
    const bool lmax_ok = std::isfinite(in.lam_max) && in.lam_max > 0.0;
    const bool g2_ok = std::isfinite(in.g2) && (in.p == 0 || in.g2 > 0.0);
    return lmin_ok && lmax_ok && g2_ok;
}

int ensure_meta(duq_server* s, size_t bytes) {
    if (bytes > s->meta_cap) {
        if (s->meta) (void)hipFree(s->meta);
        s->meta = nullptr;
        const size_t cap = std::max(bytes, 2 * s->meta_cap);
        if (hipMalloc(&s->meta, cap) != hipSuccess) return DUQ_ENOMEM;
        s->meta_cap = cap;
    }
    if (bytes > s->hmeta_cap) {
        if (s->hmeta) (void)hipHostFree(s->hmeta);
        s->hmeta = nullptr;
        const size_t cap = std::max(bytes, 2 * s->hmeta_cap);
        if (hipHostMalloc((void**)&s->hmeta, cap, hipHostMallocDefault) != hipSuccess) return DUQ_ENOMEM;
        s->hmeta_cap = cap;
    }
    return DUQ_OK;
}

// One batch-kernel launch over the admitted small requests of one dtype and
// one row class (short-row or long-row kernel).
struct Group {
    int dtype;
    bool sh;
    std::vector<Req*> r;
    size_t o_inst, o_order, o_res, o_queue;
};

// Requests against one shared system on the MFMA tiles.
struct TileGroup {
    int sid;
    std::vector<Req*> r;
    size_t o_inst, o_res, o_queue;                  // metadata (and its host mirror)
    size_t w_q, w_g, w_x, w_l, w_dual, w_prim;       // tile workspace
};

// One round: launches, state copies, one synchronisation, retirement.
int round(duq_server* s) {
    std::vector<Req*> act;
    std::vector<Shared> shs;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        act = s->active;
        shs = s->shared;
    }
    Group grp[4] = {{DUQ_F64, false, {}, 0, 0, 0, 0}, {DUQ_F64, true, {}, 0, 0, 0, 0},
                    {DUQ_F32, false, {}, 0, 0, 0, 0}, {DUQ_F32, true, {}, 0, 0, 0, 0}};
    std::vector<Req*> large;
    std::map<int, std::vector<Req*>> by_sys;   // shared system -> its requests for the tiles
    for (Req* r : act) {
        if (r->large) large.push_back(r);
        else if (r->shared_id >= 0 && shs[r->shared_id].tile && !r->inst.resume) by_sys[r->shared_id].push_back(r);
        else grp[(r->dtype == DUQ_F64 ? 0 : 2) + (batch_short_class(r->dtype, r->n) ? 1 : 0)].r.push_back(r);
    }
    size_t off = 0;
    auto plan = [&](size_t b) { size_t o = off; off += up(b); return o; };
    for (Group& gr : grp) {
        if (gr.r.empty()) continue;
        // largest work first; ties in arrival order
        std::stable_sort(gr.r.begin(), gr.r.end(), [](const Req* a, const Req* b) {
            const long long wa = (long long)a->n * a->n + (long long)a->p * a->n;
            const long long wb = (long long)b->n * b->n + (long long)b->p * b->n;
            return wa > wb;
        });
        const size_t B = gr.r.size();
        gr.o_inst = plan(sizeof(ServeInst) * B);
        gr.o_order = plan(sizeof(int) * B);
        gr.o_res = plan(sizeof(BatchResultDev) * B);
        gr.o_queue = plan(sizeof(unsigned));
    }
    // tile groups: the request table, results and queue with the metadata;
    // gathered q, g, the outputs and the tile state in the tile workspace
    std::vector<TileGroup> tgs;
    size_t woff = 0;
    auto wplan = [&](size_t b) { size_t o = woff; woff += up(b); return o; };
    for (auto& kv : by_sys) {
        TileGroup tg;
        tg.sid = kv.first;
        tg.r = kv.second;
        const Shared& sh = shs[tg.sid];
        const size_t B = tg.r.size(), n = (size_t)sh.n, pp = (size_t)std::max(sh.p, 1);
        tg.o_inst = plan(sizeof(ServeInst) * B);
        tg.o_res = plan(sizeof(BatchResultDev) * B);
        tg.o_queue = plan(sizeof(unsigned));
        tg.w_q = wplan(8 * B * n);
        tg.w_g = wplan(8 * B * pp);
        tg.w_x = wplan(8 * B * n);
        tg.w_l = wplan(8 * B * pp);
        tg.w_dual = wplan(8 * 3 * B * pp);
        tg.w_prim = wplan(8 * 4 * B * n);
        tgs.push_back(tg);
    }
    if (int rc = ensure_meta(s, std::max<size_t>(off, kAlign))) return set_error(rc, "serving metadata");
    if (woff > s->tile_ws_cap) {
        if (s->tile_ws) (void)hipFree(s->tile_ws);
        s->tile_ws = nullptr;
        s->tile_ws_cap = 0;
        const size_t cap = std::max(woff, 2 * s->tile_ws_cap);
        if (hipMalloc(&s->tile_ws, cap) != hipSuccess) return set_error(DUQ_ENOMEM, "serving tile workspace");
        s->tile_ws_cap = cap;
    }
    hipError_t e = hipSuccess;
    DevParams par{};
    par.method = s->opts.method;
    par.output = s->opts.output;
    par.inner_rule = s->opts.inner_rule;
    par.inner_variant = s->opts.inner_variant;
    par.max_outer = s->opts.max_outer;
    par.eps_out = s->opts.eps_out;
    par.eps_in = s->opts.eps_in;
    par.rho = s->opts.rho;
    par.lb_cert = resolve_lb_cert(s->opts.lb_cert);
    for (Group& gr : grp) {
        if (gr.r.empty()) continue;
        const int B = (int)gr.r.size();
        ServeInst* hi = (ServeInst*)(s->hmeta + gr.o_inst);
        int* ho = (int*)(s->hmeta + gr.o_order);
        int n_max = 1, p_max = 0;
        for (int j = 0; j < B; ++j) {
            hi[j] = gr.r[j]->inst;
            ho[j] = j;
            n_max = std::max(n_max, gr.r[j]->n);
            p_max = std::max(p_max, gr.r[j]->p);
        }
        std::memset(s->hmeta + gr.o_queue, 0, sizeof(unsigned));
        char* d = (char*)s->meta;
        e = e ? e : hipMemcpyAsync(d + gr.o_inst, hi, sizeof(ServeInst) * B, hipMemcpyHostToDevice, s->stream);
        e = e ? e : hipMemcpyAsync(d + gr.o_order, ho, sizeof(int) * B, hipMemcpyHostToDevice, s->stream);
        e = e ? e : hipMemcpyAsync(d + gr.o_queue, s->hmeta + gr.o_queue, sizeof(unsigned), hipMemcpyHostToDevice,
                                   s->stream);
        const int k_alloc = std::min(s->k_req, n_max);
        const size_t shmem = batch_lds_bytes(n_max, p_max, k_alloc);
        int bpc = 0;
        e = e ? e : batch_occupancy(gr.dtype, gr.sh, true, shmem, &bpc);
        if (e == hipSuccess && bpc < 1) return set_error(DUQ_EDEVICE, "serving batch does not fit a workgroup's LDS");
        BatchLaunch L{};
        L.B = B;
        L.order = (const int*)(d + gr.o_order);
        L.res = d + gr.o_res;
        L.inst = (const ServeInst*)(d + gr.o_inst);
        L.slice = s->slice;
        L.base = par;
        L.max_inner = s->opts.max_inner;
        L.lanczos_k = s->k_req;
        L.lanczos_alloc = k_alloc;
        L.safety = s->opts.safety;
        L.n_max = n_max;
        L.p_max = p_max;
        L.queue = (unsigned*)(d + gr.o_queue);
        const int nblocks = std::max(1, std::min(B, s->cus * std::max(bpc, 1)));
        e = e ? e : launch_batch(gr.dtype, gr.sh, nblocks, shmem, s->stream, L);
        e = e ? e : hipMemcpyAsync(s->hmeta + gr.o_res, d + gr.o_res, sizeof(BatchResultDev) * B,
                                   hipMemcpyDeviceToHost, s->stream);
    }
    for (TileGroup& tg : tgs) {
        const Shared& sh = shs[tg.sid];
        const int B = (int)tg.r.size();
        ServeInst* hi = (ServeInst*)(s->hmeta + tg.o_inst);
        for (int j = 0; j < B; ++j) hi[j] = tg.r[j]->inst;
        std::memset(s->hmeta + tg.o_queue, 0, sizeof(unsigned));
        char* d = (char*)s->meta;
        char* w = (char*)s->tile_ws;
        const ServeInst* di = (const ServeInst*)(d + tg.o_inst);
        e = e ? e : hipMemcpyAsync(d + tg.o_inst, hi, sizeof(ServeInst) * B, hipMemcpyHostToDevice, s->stream);
        e = e ? e : hipMemcpyAsync(d + tg.o_queue, s->hmeta + tg.o_queue, sizeof(unsigned), hipMemcpyHostToDevice,
                                   s->stream);
        e = e ? e : launch_serve_gather(di, B, sh.n, sh.p, (double*)(w + tg.w_q), (double*)(w + tg.w_g), s->stream);
        TileLaunch t{};
        t.B = B;
        t.n = sh.n;
        t.p = sh.p;
        t.Q = sh.Q;
        t.G = sh.G;
        t.q = (const double*)(w + tg.w_q);
        t.g = (const double*)(w + tg.w_g);
        t.lb = sh.lb;
        t.ub = sh.ub;
        t.X = (double*)(w + tg.w_x);
        t.Lam = (double*)(w + tg.w_l);
        t.res = d + tg.o_res;
        t.dual = (double*)(w + tg.w_dual);
        t.prim = (double*)(w + tg.w_prim);
        t.par = sh.par;
        t.lam_min = sh.lam_min;
        t.lam_max = sh.lam_max;
        t.g2 = sh.p ? sh.g2 : 0.0;
        t.queue = (unsigned*)(d + tg.o_queue);
        int bpc = 0;
        e = e ? e : tile_occupancy(sh.dtype, tile_lds_bytes(sh.n), &bpc);
        const int nblocks = std::max(1, std::min((B + 15) / 16, s->cus * std::max(bpc, 1)));
        e = e ? e : launch_tile(sh.dtype, nblocks, tile_lds_bytes(sh.n), s->stream, t);
        e = e ? e : launch_serve_scatter(di, B, sh.n, sh.p, t.X, t.Lam, s->stream);
        e = e ? e : hipMemcpyAsync(s->hmeta + tg.o_res, d + tg.o_res, sizeof(BatchResultDev) * B,
                                   hipMemcpyDeviceToHost, s->stream);
    }
    if (e != hipSuccess) return set_error(DUQ_EDEVICE, std::string("serving launch: ") + hipGetErrorString(e));
    for (Req* r : large) {
        const int rc = handle_slice(r->h, r->k_done == 0 && !r->inst.resume, s->slice, r->k_done, r->st);
        if (rc) return rc;
        r->inst.resume = 1;
    }
    e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return set_error(DUQ_EDEVICE, std::string("serving round: ") + hipGetErrorString(e));
    for (Req* r : act) {   // uploads are complete: drop the host copies
        std::vector<char>().swap(r->Q);
        std::vector<char>().swap(r->G);
        std::vector<double>().swap(r->q);
        std::vector<double>().swap(r->g);
        std::vector<double>().swap(r->lb);
        std::vector<double>().swap(r->ub);
    }

    // retire
    std::vector<Req*> done;
    std::vector<Req*> bad;
    for (Group& gr : grp) {
        const BatchResultDev* rr = (const BatchResultDev*)(s->hmeta + gr.o_res);
        for (size_t j = 0; j < gr.r.size(); ++j) {
            Req* r = gr.r[j];
            const BatchResultDev& x = rr[j];
            r->res.outer_iters = x.outer;
            r->res.inner_iters = x.inner;
            r->res.gt_rows = x.gt_rows;
            r->res.f = x.F;
            r->res.lb_dual = x.LB;
            r->res.gap = x.F - x.LB;
            r->res.feas = x.feas;
            r->res.f64_outer_iters = x.outer;
            r->res.engine = DUQ_ENGINE_BLOCK;
            r->res.lam_min = x.lam_min;
            r->res.lam_max = x.lam_max;
            r->res.G_norm2 = x.G2;
            const bool more = x.status == 1 && x.outer < s->opts.max_outer;
            if (more) {
                r->inst.resume = 1;
                r->inst.lam_min = x.lam_min;
                r->inst.lam_max = x.lam_max;
                r->inst.g2 = x.G2;
                if (!constants_ok(r->inst, s->opts.rho)) {
                    // the next slice would run with these constants: end the
                    // request instead (its state is not resumed)
                    r->code = DUQ_EDEVICE;
                    r->err = "invalid constants carried from the first slice";
                    bad.push_back(r);
                }
                continue;
            }
            r->x.resize(r->n);
            r->lam.resize(r->p);
            e = hipMemcpy(r->x.data(), r->inst.x, 8 * r->n, hipMemcpyDeviceToHost);
            if (r->p > 0 && e == hipSuccess) e = hipMemcpy(r->lam.data(), r->inst.lam, 8 * r->p, hipMemcpyDeviceToHost);
            if (e != hipSuccess) return set_error(DUQ_EDEVICE, "result copy");
            done.push_back(r);
            r->code = to_code(x.status);
            if (x.status == 4)
                r->err = "the constants of the request (estimated or given) are not finite and positive";
        }
    }
    for (TileGroup& tg : tgs) {   // tile requests end in their round
        const BatchResultDev* rr = (const BatchResultDev*)(s->hmeta + tg.o_res);
        for (size_t j = 0; j < tg.r.size(); ++j) {
            Req* r = tg.r[j];
            const BatchResultDev& x = rr[j];
            r->res.outer_iters = x.outer;
            r->res.inner_iters = x.inner;
            r->res.gt_rows = x.gt_rows;
            r->res.f = x.F;
            r->res.lb_dual = x.LB;
            r->res.gap = x.F - x.LB;
            r->res.feas = x.feas;
            r->res.f64_outer_iters = x.outer;
            r->res.engine = DUQ_ENGINE_TILE;
            r->res.lam_min = x.lam_min;
            r->res.lam_max = x.lam_max;
            r->res.G_norm2 = x.G2;
            r->x.resize(r->n);
            r->lam.resize(r->p);
            e = hipMemcpy(r->x.data(), r->inst.x, 8 * r->n, hipMemcpyDeviceToHost);
            if (r->p > 0 && e == hipSuccess) e = hipMemcpy(r->lam.data(), r->inst.lam, 8 * r->p, hipMemcpyDeviceToHost);
            if (e != hipSuccess) return set_error(DUQ_EDEVICE, "result copy");
            r->code = to_code(x.status);
            done.push_back(r);
        }
    }
    for (Req* r : large) {
        const DevState& st = *r->st;
        unsigned flag = 0;
        if (handle_barrier_error(r->h, &flag) != DUQ_OK || flag)
            return set_error(DUQ_EDEVICE, "grid barrier timeout in a large request");
        r->k_done = st.k;
        double lmin, lmax, g2;
        int eng;
        handle_info(r->h, &lmin, &lmax, &g2, &eng);
        r->res.outer_iters = st.k;
        r->res.inner_iters = st.inner;
        r->res.gt_rows = st.gt_rows;
        r->res.f = st.F;
        r->res.lb_dual = st.LB;
        r->res.gap = st.F - st.LB;
        r->res.feas = st.feas;
        r->res.f64_outer_iters = st.k;
        r->res.engine = eng;
        r->res.lam_min = lmin;
        r->res.lam_max = lmax;
        r->res.G_norm2 = g2;
        if (st.status == 1 && st.k < s->opts.max_outer) continue;
        r->x.resize(r->n);
        r->lam.resize(r->p);
        if (handle_outputs(r->h, r->x.data(), r->lam.data()) != DUQ_OK) return DUQ_EDEVICE;
        r->code = to_code(st.status);
        done.push_back(r);
    }
    if (!done.empty() || !bad.empty()) {
        std::lock_guard<std::mutex> lk(s->mu);
        for (Req* r : done) {
            finish(s, r, r->code, !r->err.empty() ? r->err : r->code ? "request did not pass its outer test" : "");
            s->active.erase(std::find(s->active.begin(), s->active.end(), r));
        }
        for (Req* r : bad) {
            finish(s, r, r->code, r->err);
            s->active.erase(std::find(s->active.begin(), s->active.end(), r));
        }
    }
    return DUQ_OK;
}

void serve_loop(duq_server* s) {
    (void)hipSetDevice(s->device);
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv.wait(lk, [&] {
                return s->stop || !s->pending.empty() || !s->pending_large.empty() || !s->active.empty();
            });
            if (s->stop) return;
            admit(s);
            if (s->active.empty()) continue;
        }
        const int rc = round(s);
        if (rc) {
            // a device error ends the service: fail everything outstanding
            std::lock_guard<std::mutex> lk(s->mu);
            s->fatal = rc;
            s->fatal_msg = duq_last_error();
            for (Req* r : s->active) finish(s, r, rc, s->fatal_msg);
            s->active.clear();
            for (Req* r : s->pending) finish(s, r, rc, s->fatal_msg);
            for (Req* r : s->pending_large) finish(s, r, rc, s->fatal_msg);
            s->pending.clear();
            s->pending_large.clear();
            return;
        }
    }
}

int validate_opts(const duq_options* o) {
    if (!o) return set_error(DUQ_EINVAL, "null options");
    if (!(o->eps_out > 0.0) || !(o->eps_in > 0.0) || !(o->rho >= 0.0) || !std::isfinite(o->rho) ||
        o->max_outer < 1 || o->max_inner < 0 || o->lanczos_steps < 0 || o->serve_slice < 0)
        return set_error(DUQ_EINVAL, "bad options");
    if (o->method != DUQ_DGM && o->method != DUQ_DFGM) return set_error(DUQ_EINVAL, "bad method");
    if (o->output != DUQ_LAST && o->output != DUQ_AVG) return set_error(DUQ_EINVAL, "bad output");
    if (o->inner_rule != DUQ_CERT && o->inner_rule != DUQ_FIXED) return set_error(DUQ_EINVAL, "bad inner_rule");
    if (o->inner_variant < 0 || o->inner_variant > 3) return set_error(DUQ_EINVAL, "bad inner_variant");
    if (o->accumulate != DUQ_ACC_F64) return set_error(DUQ_EINVAL, "the serving loop accumulates in FP64");
    if (!(o->safety >= 1.0)) return set_error(DUQ_EINVAL, "safety must be >= 1");
    return DUQ_OK;
}

}  // namespace

extern "C" {

int duq_server_create(size_t hbm_budget_bytes, const duq_options* opts, duq_server** out) {
    if (!out) return set_error(DUQ_EINVAL, "null output");
    *out = nullptr;
    if (int rc = validate_opts(opts)) return rc;
    std::unique_ptr<duq_server> s(new (std::nothrow) duq_server());
    if (!s) return set_error(DUQ_ENOMEM, "host allocation");
    s->opts = *opts;
    s->slice = opts->serve_slice > 0 ? opts->serve_slice : 16;
    s->k_req = opts->lanczos_steps > 0 ? opts->lanczos_steps : 96;
    if (hipGetDevice(&s->device) != hipSuccess) return set_error(DUQ_EDEVICE, "no device");
    s->cus = device_cus();
    const size_t budget = hbm_budget_bytes ? up(hbm_budget_bytes) : ((size_t)4 << 30);
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return set_error(DUQ_EDEVICE, "hipMemGetInfo");
    if (budget > fr) return set_error(DUQ_ENOMEM, "HBM budget exceeds the free device memory");
    if (hipMalloc((void**)&s->arena_mem, budget) != hipSuccess) return set_error(DUQ_ENOMEM, "arena allocation");
    s->arena.init(s->arena_mem, budget);
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->reg_stream, hipStreamNonBlocking) != hipSuccess) {
        duq_server_destroy(s.release());
        return set_error(DUQ_EDEVICE, "stream creation");
    }
    duq_server* raw = s.release();
    raw->th = std::thread(serve_loop, raw);
    *out = raw;
    return DUQ_OK;
}

int duq_register_shared(duq_server* s, const duq_problem* pr, int32_t* id) {
    if (!s || !pr || !id) return set_error(DUQ_EINVAL, "null argument");
    if (pr->rlo || pr->rhi) return set_error(DUQ_EINVAL, "row bounds are available on duq_setup / duq_solve only");
    const int n = pr->n, p = pr->p;
    if (n < 1 || n > DUQ_SERVE_BATCH_NMAX || p < 0)
        return set_error(DUQ_EINVAL, "shared systems need 1 <= n <= DUQ_SERVE_BATCH_NMAX and p >= 0");
    if (pr->dtype != DUQ_F64 && pr->dtype != DUQ_F32) return set_error(DUQ_EINVAL, "dtype must be F64 or F32");
    if (pr->memspace != DUQ_HOST && pr->memspace != DUQ_DEVICE) return set_error(DUQ_EINVAL, "bad memspace");
    if (!pr->Q || !pr->lb || !pr->ub || (p > 0 && !pr->G)) return set_error(DUQ_EINVAL, "null Q, G, lb or ub");
    const size_t es = pr->dtype == DUQ_F64 ? 8 : 4;
    const int pp = std::max(p, 1);
    const size_t bytes = up((size_t)n * n * es) + up((size_t)pp * n * es) + 2 * up(8 * (size_t)n) + 2 * up(8 * (size_t)pp);
    char* mem;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        mem = s->arena.alloc(bytes);
    }
    if (!mem) return set_error(DUQ_ENOMEM, "arena full");
    char* c = mem;
    auto take = [&](size_t b) { char* o = c; c += up(b); return o; };
    char* Q = take((size_t)n * n * es);
    char* G = take((size_t)pp * n * es);
    double* lb = (double*)take(8 * (size_t)n);
    double* ub = (double*)take(8 * (size_t)n);
    double* zq = (double*)take(8 * (size_t)n);
    double* zg = (double*)take(8 * (size_t)pp);
    const hipMemcpyKind kind = pr->memspace == DUQ_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    hipError_t e = hipMemcpyAsync(Q, pr->Q, (size_t)n * n * es, kind, s->reg_stream);
    if (p > 0) e = e ? e : hipMemcpyAsync(G, pr->G, (size_t)p * n * es, kind, s->reg_stream);
    e = e ? e : hipMemcpyAsync(lb, pr->lb, 8 * (size_t)n, kind, s->reg_stream);
    e = e ? e : hipMemcpyAsync(ub, pr->ub, 8 * (size_t)n, kind, s->reg_stream);
    e = e ? e : hipMemsetAsync(zq, 0, 8 * (size_t)n, s->reg_stream);
    e = e ? e : hipMemsetAsync(zg, 0, 8 * (size_t)pp, s->reg_stream);
    e = e ? e : hipStreamSynchronize(s->reg_stream);
    auto undo = [&](int code, const std::string& msg) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->arena.release(mem, bytes);
        return set_error(code, msg);
    };
    if (e != hipSuccess) return undo(DUQ_EDEVICE, std::string("copy of the shared system: ") + hipGetErrorString(e));
    // validation (finite data, box) and constants through the single-QP setup
    duq_problem dp{n, p, pr->dtype, DUQ_DEVICE, Q, p ? G : nullptr, zq, p ? zg : nullptr, lb, ub};
    duq_options o = s->opts;
    o.trace_outer = 0;
    o.engine = DUQ_ENGINE_BLOCK;
    duq_handle* h = nullptr;
    int rc = duq_setup(&dp, &o, s->reg_stream, &h);
    if (rc) {
        const std::string m = duq_last_error();
        return undo(rc, m);
    }
    Shared sh{n, p, pr->dtype, mem, bytes, Q, G, lb, ub, 0, 0, 0};
    int eng;
    handle_info(h, &sh.lam_min, &sh.lam_max, &sh.g2, &eng);
    handle_params(h, &sh.par);
    duq_destroy(h);
    // requests against a system the tile kernel can hold run there, 16 to a
    // tile, each to completion within one round
    int bpc = 0;
    sh.tile = s->opts.rho == 0.0 && n <= kTileMaxN &&
              tile_occupancy(pr->dtype, tile_lds_bytes(n), &bpc) == hipSuccess && bpc >= 1;
    std::lock_guard<std::mutex> lk(s->mu);
    s->shared.push_back(sh);
    *id = (int32_t)s->shared.size() - 1;
    return DUQ_OK;
}

int duq_submit(duq_server* s, const duq_request* rq, uint64_t* ticket) {
    if (!s || !rq || !ticket) return set_error(DUQ_EINVAL, "null argument");
    const duq_problem& pr = rq->prob;
    if (pr.rlo || pr.rhi) return set_error(DUQ_EINVAL, "row bounds are available on duq_setup / duq_solve only");
    std::unique_ptr<Req> r(new (std::nothrow) Req());
    if (!r) return set_error(DUQ_ENOMEM, "host allocation");
    r->shared_id = rq->shared_id;
    if (rq->shared_id >= 0) {
        std::lock_guard<std::mutex> lk(s->mu);
        if (rq->shared_id >= (int)s->shared.size()) return set_error(DUQ_EINVAL, "unknown shared_id");
        const Shared& sh = s->shared[rq->shared_id];
        r->n = sh.n;
        r->p = sh.p;
        r->dtype = sh.dtype;
    } else if (rq->shared_id == -1) {
        if (pr.memspace != DUQ_HOST) return set_error(DUQ_EINVAL, "requests are host data");
        if (pr.n < 1 || pr.p < 0) return set_error(DUQ_EINVAL, "bad sizes");
        if (pr.dtype != DUQ_F64 && pr.dtype != DUQ_F32) return set_error(DUQ_EINVAL, "dtype must be F64 or F32");
        if (!pr.Q || !pr.lb || !pr.ub || (pr.p > 0 && !pr.G)) return set_error(DUQ_EINVAL, "null Q, G, lb or ub");
        r->n = pr.n;
        r->p = pr.p;
        r->dtype = pr.dtype;
    } else {
        return set_error(DUQ_EINVAL, "bad shared_id");
    }
    const int n = r->n, p = r->p;
    if (!pr.q || (p > 0 && !pr.g)) return set_error(DUQ_EINVAL, "null q or g");
    if (!finite_all(pr.q, n) || (p > 0 && !finite_all(pr.g, p))) return set_error(DUQ_EINVAL, "non-finite q or g");
    r->q.assign(pr.q, pr.q + n);
    if (p > 0) r->g.assign(pr.g, pr.g + p);
    if (rq->shared_id < 0) {
        const size_t es = r->dtype == DUQ_F64 ? 8 : 4;
        const long long nn = (long long)n * n, pn = (long long)p * n;
        const bool ok = r->dtype == DUQ_F64
                            ? finite_all((const double*)pr.Q, nn) && (p == 0 || finite_all((const double*)pr.G, pn))
                            : finite_all((const float*)pr.Q, nn) && (p == 0 || finite_all((const float*)pr.G, pn));
        if (!ok) return set_error(DUQ_EINVAL, "non-finite Q or G");
        for (int i = 0; i < n; ++i)
            if (!std::isfinite(pr.lb[i]) || !std::isfinite(pr.ub[i]) || pr.lb[i] > pr.ub[i])
                return set_error(DUQ_EINVAL, "box must be finite with lb <= ub");
        r->Q.assign((const char*)pr.Q, (const char*)pr.Q + nn * es);
        if (p > 0) r->G.assign((const char*)pr.G, (const char*)pr.G + pn * es);
        r->lb.assign(pr.lb, pr.lb + n);
        r->ub.assign(pr.ub, pr.ub + n);
        r->large = n > DUQ_SERVE_BATCH_NMAX;
    }
    r->bytes = footprint(s, n, p, r->dtype, rq->shared_id < 0, r->large, nullptr);
    if (r->bytes > s->arena.size()) return set_error(DUQ_ENOMEM, "request footprint exceeds the HBM budget");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->fatal) return set_error(s->fatal, "server stopped: " + s->fatal_msg);
    r->ticket = s->next_ticket++;
    r->t_submit = Clock::now();
    *ticket = r->ticket;
    (r->large ? s->pending_large : s->pending).push_back(r.get());
    s->reqs[r->ticket] = std::move(r);
    s->cv.notify_one();
    return DUQ_OK;
}

int duq_poll(duq_server* s, uint64_t ticket, double* x_out, double* lam_out, duq_result* res) {
    if (!s) return set_error(DUQ_EINVAL, "null server");
    std::unique_ptr<Req> r;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return set_error(DUQ_ENOTFOUND, "unknown ticket");
        if (it->second->state != ST_DONE) return DUQ_EAGAIN;
        r = std::move(it->second);
        s->reqs.erase(it);
    }
    if (x_out && !r->x.empty()) std::memcpy(x_out, r->x.data(), 8 * r->x.size());
    if (lam_out && !r->lam.empty()) std::memcpy(lam_out, r->lam.data(), 8 * r->lam.size());
    if (res) *res = r->res;
    if (r->code != DUQ_OK) set_error(r->code, r->err);
    return r->code;
}

void duq_server_destroy(duq_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->th.joinable()) s->th.join();
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (auto& kv : s->reqs)
        if (kv.second->h) duq_destroy(kv.second->h);
    for (auto& kv : s->reqs)
        if (kv.second->st) (void)hipHostFree(kv.second->st);
    if (s->meta) (void)hipFree(s->meta);
    if (s->tile_ws) (void)hipFree(s->tile_ws);
    if (s->hmeta) (void)hipHostFree(s->hmeta);
    if (s->arena_mem) (void)hipFree(s->arena_mem);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    if (s->reg_stream) (void)hipStreamDestroy(s->reg_stream);
    delete s;
}

}  // extern "C"
