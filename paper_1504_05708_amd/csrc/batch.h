// Batched DFOM: many independent QPs in one persistent launch.  Each
// workgroup takes the next instance from a device work queue (instances are
// ordered largest first), derives its constants (Sec. 2 eq. Ld, Sec. 3 Step 1,
// Sec. 5 k_in) and runs Algorithm DFOM with the workgroup as the team.
//
// The same kernel serves the time-sliced serving loop: there each instance is
// described by a ServeInst (its own pointers and workspace), runs at most
// `slice` outer iterations per launch and resumes from its saved state in the
// next launch (a separate instantiation, so the batch kernel carries none of
// this).  The host launches short-row and long-row instances
// (short_rows(n)) as separate kernels, so an instance runs the same code and
// computes the same bits whatever else is in the batch.
#pragma once
#include "lanczos.h"

namespace duq {

template <typename T>
struct BatchArgs {
    int B;
    int shared;                  // 1: every instance uses Q, G, lb, ub of instance 0
    const int* order;            // B instance indices, processing order
    const int* n;                // B sizes (uneven) -- unused when shared
    const int* p;
    const long long* qoff;
    const long long* goff;
    const long long* voff;
    const long long* coff;
    int n_shared, p_shared;
    const T* Q;
    const T* G;
    const double* q;
    const double* g;
    const double* lb;
    const double* ub;
    const double* lam_min;       // per instance or null (estimate)
    const double* lam_max;
    const double* g2;
    double* X;
    double* Lam;
    BatchResultDev* res;
    const ServeInst* inst;       // serving kernel: per-instance records (replace the fields above)
    int slice;                   // serving: outer iterations per launch at n = 256 (scaled by work)
    DevParams base;              // options shared by every instance
    int max_inner;               // 0: k_in of Sec. 5
    int lanczos_k;               // requested Krylov steps (per instance: min(lanczos_k, n))
    int lanczos_alloc;           // min(lanczos_k, n_max): sizes the slot and LDS
    double safety;
    char* slots;                 // per-workgroup workspace (batch mode)
    long long slot_bytes;
    int n_max, p_max;
    unsigned* queue;             // [0]: next queue position
};

// Workspace of one slot, carved in a fixed order (mirrored on the host).
__host__ __device__ inline long long slot_take(long long& off, long long bytes) {
    const long long o = off;
    off += ((bytes + 255) / 256) * 256;
    return o;
}

__host__ __device__ inline long long batch_slot_bytes(int n, int p, int k) {
    long long off = 0;
    const int pp = p > 0 ? p : 1;
    for (int i = 0; i < 3; ++i) slot_take(off, 8LL * n);        // xb
    for (int i = 0; i < 3; ++i) slot_take(off, 8LL * n);        // qb
    for (int i = 0; i < 6; ++i) slot_take(off, 8LL * n);        // c us qus usave qusave (spare)
    for (int i = 0; i < 6; ++i) slot_take(off, 8LL * pp);       // r rs lamp mu wv gsave
    for (int i = 0; i < 3; ++i) slot_take(off, 8LL * pp);       // gx
    slot_take(off, sizeof(DevState));
    slot_take(off, 8LL * (k + 1) * n);                          // Lanczos V
    slot_take(off, 8LL * n);                                    // w
    slot_take(off, 8LL * pp);                                   // r
    slot_take(off, 8LL * (2 * k + 2));                          // ab
    slot_take(off, 8LL * 4);                                    // out
    return off;
}

__device__ inline void batch_carve(char* base, int n, int p, int k, DevWork& W, LanczosWork& L) {
    long long off = 0;
    const int pp = p > 0 ? p : 1;
    auto d = [&](long long bytes) { return reinterpret_cast<double*>(base + slot_take(off, bytes)); };
    for (int i = 0; i < 3; ++i) W.xb[i] = d(8LL * n);
    for (int i = 0; i < 3; ++i) W.qb[i] = d(8LL * n);
    W.c = d(8LL * n);
    W.us = d(8LL * n);
    W.qus = d(8LL * n);
    W.usave = d(8LL * n);
    W.qusave = d(8LL * n);
    (void)d(8LL * n);
    W.r = d(8LL * pp);
    W.rs = d(8LL * pp);
    W.lamp = d(8LL * pp);
    W.mu = d(8LL * pp);
    W.wv = d(8LL * pp);
    W.gsave = d(8LL * pp);
    for (int i = 0; i < 3; ++i) W.gx[i] = d(8LL * pp);
    W.st = reinterpret_cast<DevState*>(base + slot_take(off, sizeof(DevState)));
    L.V = d(8LL * (k + 1) * n);
    L.w = d(8LL * n);
    L.r = d(8LL * pp);
    L.ab = d(8LL * (2 * k + 2));
    L.out = d(8LL * 4);
    L.part = nullptr;
    L.gtp = nullptr;
    L.bar = nullptr;
    W.lamm = nullptr;
    W.mum = nullptr;
    W.nu = nullptr;
    W.wsh = nullptr;
    W.part = nullptr;
    W.gtp = nullptr;
    W.trace = nullptr;
    W.bar = nullptr;
    W.x0 = nullptr;
    W.lam0 = nullptr;
}

template <typename T, typename Acc, bool SHORT, bool SERVE>
__device__ __forceinline__ void batch_solve(const BatchArgs<T>& a, double* lds) {
    __shared__ int s_idx;
    DevWork W;
    LanczosWork LW;
    if constexpr (!SERVE) batch_carve(a.slots + (long long)blockIdx.x * a.slot_bytes, a.n_max, a.p_max, a.lanczos_alloc, W, LW);
    double* const red = lds + a.n_max + a.p_max + 1;
    double* const tl = lds + a.n_max + a.p_max + 1 + a.lanczos_alloc + 2 + kMaxWaves * kNP + 16;
    for (;;) {
        if (threadIdx.x == 0) s_idx = (int)atomicAdd(a.queue, 1u);
        __syncthreads();
        const int qpos = s_idx;
        __syncthreads();
        if (qpos >= a.B) break;
        const int i = a.order[qpos];
        DevProblem<T> P;
        double* xo;
        double* lo;
        int kk;
        bool given, resume;
        double lmin, lmax, g2;
        if constexpr (SERVE) {
            const ServeInst& si = a.inst[i];
            P.n = si.n;
            P.p = si.p;
            P.Q = static_cast<const T*>(si.Q);
            P.G = static_cast<const T*>(si.G);
            P.q = si.q;
            P.g = si.g;
            P.lb = si.lb;
            P.ub = si.ub;
            xo = si.x;
            lo = si.lam;
            kk = si.k;
            batch_carve(si.slot, si.n, si.p, si.k, W, LW);
            resume = si.resume != 0;
            given = si.given != 0 || resume;
            lmin = si.lam_min;
            lmax = si.lam_max;
            g2 = si.g2;
        } else {
            P.n = a.shared ? a.n_shared : a.n[i];
            P.p = a.shared ? a.p_shared : a.p[i];
            P.Q = a.shared ? a.Q : a.Q + a.qoff[i];
            P.G = a.shared ? a.G : a.G + a.goff[i];
            const long long vo = a.shared ? (long long)i * P.n : a.voff[i];
            const long long co = a.shared ? (long long)i * P.p : a.coff[i];
            P.q = a.q + vo;
            P.g = a.g + co;
            P.lb = a.shared ? a.lb : a.lb + vo;
            P.ub = a.shared ? a.ub : a.ub + vo;
            xo = a.X + vo;
            lo = a.Lam + co;
            kk = min(a.lanczos_k, P.n);
            resume = false;
            given = a.lam_min && a.lam_max && a.g2;
            const int ci = a.shared ? 0 : i;
            lmin = given ? a.lam_min[ci] : 0.0;
            lmax = given ? a.lam_max[ci] : 0.0;
            g2 = given ? a.g2[ci] : 0.0;
        }
        const int n = P.n, p = P.p;
        if (p == 0) g2 = 0.0;

        // constants: supplied (or found in an earlier slice), else Lanczos on
        // Q and on G^T G in this workgroup
        if (!given) {
            Lanczos<T, SHORT> lz;
            lz.P = P;
            lz.L = LW;
            lz.k = kk;
            lz.tm.rank = 0;
            lz.tm.size = 1;
            lz.tm.bar = nullptr;
            lz.tm.epoch = 0;
            lz.nlo = 0;
            lz.nhi = n;
            lz.plo = 0;
            lz.phi = p;
            lz.xl = lds;
            lz.vl = lds + a.n_max;
            lz.hl = red;
            lz.red = red + a.lanczos_alloc + 2;
            lz.tl = tl;
            lz.use_gtg = 0;
            lz.run();
            __syncthreads();
            lmin = LW.out[0] / a.safety;
            lmax = LW.out[1] * a.safety;
            __syncthreads();
            g2 = 0.0;
            if (p > 0) {
                lz.use_gtg = 1;
                lz.run();
                __syncthreads();
                g2 = LW.out[1] * a.safety;
                __syncthreads();
            }
        }
        // derived constants, same formulas as the single-QP setup
        DevParams par = a.base;
        const double rho = par.rho;
        double du[1] = {0.0};
        for (int j = threadIdx.x; j < n; j += blockDim.x) {
            const double d = P.ub[j] - P.lb[j];
            du[0] += d * d;
        }
        block_allreduce<1>(du, red);
        const double D_U = sqrt(du[0]);
        const double denom = lmin + rho * g2;
        const int bad = (p > 0 && !(denom > 0.0)) || !(lmax > 0.0);
        const double Ld = p > 0 ? g2 / denom : 0.0;
        par.alpha = Ld > 0.0 ? 1.0 / (2.0 * Ld) : 0.0;
        par.L = lmax + rho * g2;
        par.sigma = fmax(lmin, 0.0);
        const double sqL = sqrt(par.L), sqs = sqrt(par.sigma);
        par.beta_in = (sqL - sqs) / (sqL + sqs);
        double kin;
        if (a.max_inner > 0) kin = a.max_inner;
        else if (par.sigma > 0.0) {
            const double arg = par.L * D_U * D_U / par.eps_in;
            kin = arg > 1.0 ? ceil(sqrt(par.L / par.sigma) * log(arg)) + 1.0 : 1.0;
        } else {
            kin = ceil(sqrt(2.0 * par.L * D_U * D_U / par.eps_in));
        }
        par.k_in_max = (int)fmin(fmax(kin, 1.0), 1.0e9);
        par.Kd_nonneg = lmin > 0.0 ? 1 : 0;
        if (par.inner_variant == 0) par.inner_variant = par.sigma > 0.0 ? 3 : 2;
        par.trace_iters = 0;
        par.has_x0 = 0;
        par.has_lam0 = 0;
        par.resume = resume ? 2 : 0;
        if constexpr (SERVE) {
            // outer iterations in this launch: about the work of `slice`
            // iterations at n = 256, from the instance's own n only
            const double w = (256.0 * 256.0 + 128.0 * 128.0) / ((double)n * n + 128.0 * 128.0);
            const int k_slice = max(1, (int)(a.slice * w + 0.5));
            par.max_outer = min(par.max_outer, (resume ? W.st->k : 0) + k_slice);
        }

        if (!bad) {
            Dfom<T, Acc, SHORT> s;
            s.P = P;
            s.par = par;
            s.W = W;
            s.W.xout = xo;
            s.tm.rank = 0;
            s.tm.size = 1;
            s.tm.bar = nullptr;
            s.tm.epoch = 0;
            s.nlo = 0;
            s.nhi = n;
            s.plo = 0;
            s.phi = p;
            s.xl = lds;
            s.vl = lds + a.n_max;
            s.red = red;
            s.tl = tl;
            if (threadIdx.x == 0 && !resume) W.st->gt_rows = 0;
            __syncthreads();
            s.run();
            __syncthreads();
            for (int j = threadIdx.x; j < p; j += blockDim.x) lo[j] = W.lamp[j];
        }
        if (threadIdx.x == 0) {
            BatchResultDev r;
            r.status = bad ? 4 : W.st->status;
            r.outer = bad ? 0 : W.st->k;
            r.inner = bad ? 0 : W.st->inner;
            r.gt_rows = bad ? 0 : W.st->gt_rows;
            r.F = bad ? 0.0 : W.st->F;
            r.LB = bad ? 0.0 : W.st->LB;
            r.feas = bad ? 0.0 : W.st->feas;
            r.lam_min = lmin;
            r.lam_max = lmax;
            r.G2 = g2;
            a.res[i] = r;
        }
        __syncthreads();
    }
}

}  // namespace duq
