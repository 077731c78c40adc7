// Shared-Hessian batches on the matrix cores.
//
// A workgroup of four waves (one per SIMD) advances a tile of 16 instances
// that share Q (n x n), G (p x n) and the box, in lockstep.  The products of
// the tile are dense GEMMs on FP64 MFMA (16x16x4):
//   Q X      (n x 16)  once per inner step       (Sec. 5.1, inner gradient)
//   G U      (p x 16)  once per outer iteration  (residual of Sec. 3 Step 2)
//   G^T M    (n x 16)  once per outer iteration  (linear term q + G^T mu)
// Wave w owns row tiles w and w + 4 of the n rows (two independent MFMA
// chains): lane l holds rows 16 t + l/16 + 4 i (i < 4) of column l % 16 --
// the FP64 MFMA result layout -- and keeps its rows of its instance's primal
// vectors in registers.  Q never moves during the launch, so each lane keeps
// its own A-operand entries of Q (its row, every fourth column) in registers
// for the whole launch; only the B operand X goes through LDS.  G is read
// through the caches.  The multipliers (p per instance) live in device
// memory and are updated in the epilogue of the G U product.
//
// Per column the arithmetic is Algorithm DFOM with inner FOM (rho = 0) as in
// the single-instance solver: an instance whose inner or outer loop has ended
// is masked while the others continue, and the MFMA computes every column
// from that column's data only, so an instance's iterates do not depend on
// which instances share its tile.
#pragma once
#include "device_common.h"
#include "internal.h"

namespace duq {

constexpr int kTile = 16;       // instances per workgroup
constexpr int kTileWaves = 4;   // waves per workgroup, one per SIMD (512 registers each)
constexpr int kTileRT = 2;      // row tiles of 16 per wave: n <= 16 * kTileWaves * kTileRT
constexpr int kTileQS = 32;     // k-steps of 4 columns of Q held per lane: n <= 4 * kTileQS
constexpr int kTileK = 6;       // slots of the outer reduction buffer (longer records go in chunks)

typedef double tile_v4d __attribute__((ext_vector_type(4)));

template <typename T>
struct TileArgs {
    int B, n, p;
    const T* Q;          // n x n, shared
    const T* G;          // p x n, shared
    const double* q;     // B x n
    const double* g;     // B x p
    const double* lb;    // n, shared
    const double* ub;
    double* X;           // B x n
    double* Lam;         // B x p
    BatchResultDev* res; // B
    double* dual;        // B x 3p: mu, lambda (last step), running sum of theta_j r^j
    double* prim;        // B x 4n: running sums of theta_j ubar^j and theta_j Q ubar^j,
                         // ubar^k and Q ubar^k kept across the last-iterate solve
    DevParams par;       // derived constants (shared by all instances)
    double lam_min, lam_max, g2;
    unsigned* queue;
};

// LDS layout, in doubles: two buffers of the B operand X (kp x 16), the
// inner reduction (two buffers), the outer one, the box (lb then ub).
__host__ __device__ inline int tile_kp(int n) { return (n + 3) & ~3; }
__host__ __device__ inline long tile_lds_doubles(int n) {
    return 2L * tile_kp(n) * kTile + 2L * kTileWaves * kTile * 2 + (long)kTileWaves * kTile * kTileK + 2L * n;
}

template <typename T>
struct Tile {
    TileArgs<T> a;
    double* Xs0;
    double* Xs1;
    double* red2;
    double* redK;
    double* box;     // LDS: lb (n) then ub (n)
    int lane, w, col, grp, b;
    bool valid;
    // this lane's rows of its column
    double x[kTileRT][4], xp[kTileRT][4], qx[kTileRT][4], qxp[kTileRT][4], c[kTileRT][4];
    // this lane's A-operand entries of Q: row 16 (w + kTileWaves j) + lane % 16,
    // columns 4 s + lane / 16 (zero outside the matrix)
    double qa[kTileRT][kTileQS];
    double invL;   // 1 / L_in of the inner step

    __device__ __forceinline__ void load_q() {
        const int n = a.n;
#pragma unroll
        for (int j = 0; j < kTileRT; ++j) {
            const int r = 16 * (w + kTileWaves * j) + (lane & 15);
#pragma unroll
            for (int s = 0; s < kTileQS; ++s) {
                const int k = 4 * s + grp;
                qa[j][s] = (r < n && k < n) ? (double)a.Q[(long)r * n + k] : 0.0;
            }
        }
    }

    __device__ __forceinline__ int row(int j, int i) const { return 16 * (w + kTileWaves * j) + grp + 4 * i; }

    // Sum K per-lane values over each column (the lanes of a column across
    // the waves), in a fixed order; every lane gets its column's sums.  One
    // workgroup barrier; `buf` holds kTileWaves x 16 x K doubles.
    template <int K>
    __device__ __forceinline__ void colsum(double (&v)[K], double* buf) const {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            v[k] += __shfl_xor(v[k], 16, 64);
            v[k] += __shfl_xor(v[k], 32, 64);
        }
        if (grp == 0) {
#pragma unroll
            for (int k = 0; k < K; ++k) buf[(w * kTile + col) * K + k] = v[k];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double t = buf[col * K + k];
#pragma unroll
            for (int ww = 1; ww < kTileWaves; ++ww) t += buf[(ww * kTile + col) * K + k];
            v[k] = t;
        }
    }

    // colsum in two halves: publish (wave partials to LDS, then the barrier)
    // and finish (every lane sums its column), so that independent work can
    // be issued between the barrier and the reads.
    template <int K>
    __device__ __forceinline__ void colsum_publish(double (&v)[K], double* buf) const {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            v[k] += __shfl_xor(v[k], 16, 64);
            v[k] += __shfl_xor(v[k], 32, 64);
        }
        if (grp == 0) {
#pragma unroll
            for (int k = 0; k < K; ++k) buf[(w * kTile + col) * K + k] = v[k];
        }
        __syncthreads();
    }
    template <int K>
    __device__ __forceinline__ void colsum_finish(double (&v)[K], const double* buf) const {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double t = buf[col * K + k];
#pragma unroll
            for (int ww = 1; ww < kTileWaves; ++ww) t += buf[(ww * kTile + col) * K + k];
            v[k] = t;
        }
    }

    // colsum for records longer than the outer buffer: chunks of kTileK with
    // a barrier after each read, so the buffer can be reused at once.
    template <int K>
    __device__ __forceinline__ void colsum_long(double (&v)[K], double* buf) const {
#pragma unroll
        for (int k0 = 0; k0 < K; k0 += kTileK) {
            constexpr int C = kTileK;
            double part[C];
#pragma unroll
            for (int k = 0; k < C; ++k) part[k] = k0 + k < K ? v[k0 + k] : 0.0;
            colsum<C>(part, buf);
            __syncthreads();
#pragma unroll
            for (int k = 0; k < C; ++k)
                if (k0 + k < K) v[k0 + k] = part[k];
        }
    }

    // The products run in batches of kB k-steps: every operand load of a
    // batch is issued before its MFMA chain, so loads overlap instead of
    // each MFMA waiting for its own.
    static constexpr int kB = 8;

    // acc[j] = Q Xs for this wave's row tiles: A from the registers of Q, B
    // from LDS in batches of kB k-steps (loads issued before their MFMAs).
    __device__ __forceinline__ void prodQ(const double* Xs, tile_v4d (&acc)[kTileRT]) const {
        const int ks = tile_kp(a.n) / 4;
#pragma unroll
        for (int j = 0; j < kTileRT; ++j) acc[j] = tile_v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s0 = 0; s0 < kTileQS; s0 += kB) {
            if (s0 < ks) {   // uniform
                double bv[kB];
#pragma unroll
                for (int u = 0; u < kB; ++u) {
                    // rows of Xs from n up to kp are zero; steps past ks add zeros
                    const int k = 4 * (s0 + u) + grp;
                    bv[u] = s0 + u < ks ? Xs[k * kTile + col] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < kB; ++u)
#pragma unroll
                    for (int j = 0; j < kTileRT; ++j)
                        acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[j][s0 + u], bv[u], acc[j], 0, 0, 0);
            }
        }
    }

    // acc[j] = G^T v over this wave's row tiles of n; v is the p-vector at
    // offset `voff` of this lane's instance record in `dual`.
    __device__ __forceinline__ void prodGT(int voff, tile_v4d (&acc)[kTileRT]) const {
        const int n = a.n, p = a.p, ks = tile_kp(p) / 4;
        int cidx[kTileRT];
        bool v[kTileRT];
#pragma unroll
        for (int j = 0; j < kTileRT; ++j) {
            const int r = 16 * (w + kTileWaves * j) + (lane & 15);
            v[j] = r < n;
            cidx[j] = v[j] ? r : 0;
            acc[j] = tile_v4d{0.0, 0.0, 0.0, 0.0};
        }
        const double* vb = a.dual + (long)(valid ? b : 0) * 3 * p + voff;
        for (int s0 = 0; s0 < ks; s0 += kB) {
            double av[kTileRT][kB], bv[kB];
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                const int k = 4 * (s0 + u) + grp;
                const bool kv = s0 + u < ks && k < p;
                const long gk = (long)(kv ? k : 0) * n;
                bv[u] = (kv && valid) ? vb[kv ? k : 0] : 0.0;
#pragma unroll
                for (int j = 0; j < kTileRT; ++j) av[j][u] = (v[j] && kv) ? (double)a.G[gk + cidx[j]] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kB; ++u)
#pragma unroll
                for (int j = 0; j < kTileRT; ++j)
                    acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[j][u], bv[u], acc[j], 0, 0, 0);
        }
    }

    // acc0 = G Xs for row tile rt of p and acc1 for row tile rt + kTileWaves
    // (when `two`): two independent chains share the B operand.
    __device__ __forceinline__ void prodG(const double* Xs, int rt, bool two, tile_v4d& acc0,
                                          tile_v4d& acc1) const {
        const int n = a.n, p = a.p, ks = tile_kp(n) / 4;
        const int ra = 16 * rt + (lane & 15), rb = 16 * (rt + kTileWaves) + (lane & 15);
        const bool va = ra < p, vb2 = two && rb < p;
        const T* ga = a.G + (long)(va ? ra : 0) * n;
        const T* gb2 = a.G + (long)(vb2 ? rb : 0) * n;
        acc0 = tile_v4d{0.0, 0.0, 0.0, 0.0};
        acc1 = tile_v4d{0.0, 0.0, 0.0, 0.0};
        for (int s0 = 0; s0 < ks; s0 += kB) {
            double x0[kB], x1[kB], bv[kB];
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                const int k = 4 * (s0 + u) + grp;
                const bool kv = s0 + u < ks && k < n;
                const int kk = kv ? k : 0;
                bv[u] = kv ? Xs[kk * kTile + col] : 0.0;
                x0[u] = (va && kv) ? (double)ga[kk] : 0.0;
                x1[u] = (vb2 && kv) ? (double)gb2[kk] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(x0[u], bv[u], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(x1[u], bv[u], acc1, 0, 0, 0);
            }
        }
    }

    __device__ __forceinline__ void put_x(double* Xs, const double (&v)[kTileRT][4]) const {
#pragma unroll
        for (int j = 0; j < kTileRT; ++j)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (row(j, i) < a.n) Xs[row(j, i) * kTile + col] = v[j][i];
    }

    __device__ __forceinline__ double gap_from(double fw, double pi2) const {
        return a.par.sigma > 0.0 ? fmin(fw, pi2 / (2.0 * a.par.sigma)) : fw;
    }

    // c = q + G^T v for this lane's rows.
    __device__ __forceinline__ void linear_term(int voff) {
        tile_v4d acc[kTileRT];
        prodGT(voff, acc);
#pragma unroll
        for (int j = 0; j < kTileRT; ++j)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = row(j, i);
                c[j][i] = (valid && r < a.n) ? a.q[(long)b * a.n + r] + acc[j][i] : 0.0;
            }
    }

    // Algorithm FOM (rho = 0) on the tile from x (Q x in qx) with the linear
    // term c, for the lanes with `on`; the others keep their state.  On
    // return x / qx hold ubar and Q ubar; t_out, gap_out the inner count and
    // certificate; nan_out a non-finite certificate.
    __device__ __forceinline__ void inner(bool on, int& sel, int& t_out, double& gap_out, bool& nan_out) {
        const DevParams& par = a.par;
#pragma unroll
        for (int j = 0; j < kTileRT; ++j)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                xp[j][i] = x[j][i];
                qxp[j][i] = qx[j][i];
            }
        bool run = on;
        int t = 0;
        double th = 1.0;
        t_out = 0;
        gap_out = 0.0;
        nan_out = false;
        for (;;) {
            double beta = 0.0;
            if (t > 0) {
                if (par.inner_variant == 3) beta = par.beta_in;
                else if (par.inner_variant == 2) {
                    const double thn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * th * th));
                    beta = (th - 1.0) / thn;
                }
            }
            double acc[2] = {0.0, 0.0};
            double xn[kTileRT][4];
#pragma unroll
            for (int j = 0; j < kTileRT; ++j)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    xn[j][i] = 0.0;
                    if (row(j, i) < a.n) {
                        const double xi = x[j][i], gr = qx[j][i] + c[j][i];
                        const double l = box[row(j, i)], h = box[a.n + row(j, i)];
                        // exact-gradient certificate terms at x (fw, pi^2)
                        acc[0] += fmax(gr * (xi - l), gr * (xi - h));
                        const bool atl = xi <= l, atu = xi >= h;
                        double pi = gr;
                        if (atl && atu) pi = 0.0;
                        else if (atl) pi = fmin(gr, 0.0);
                        else if (atu) pi = fmax(gr, 0.0);
                        acc[1] += pi * pi;
                        const double yi = xi + beta * (xi - xp[j][i]);
                        const double qyi = qx[j][i] + beta * (qx[j][i] - qxp[j][i]);
                        xn[j][i] = fmin(fmax(yi - (qyi + c[j][i]) * invL, l), h);
                    }
                }
            double* Xs = sel ? Xs1 : Xs0;
            double* rbuf = red2 + sel * (kTileWaves * kTile * 2);
            put_x(Xs, xn);
            colsum_publish<2>(acc, rbuf);   // barrier: Xs and the partial sums
            // Q x^{t+1} is issued before the stop decision is read back: the
            // product overlaps the column sums, and is dropped when every
            // column has stopped
            tile_v4d qn[kTileRT];
            prodQ(Xs, qn);
            colsum_finish<2>(acc, rbuf);
            const double gap = gap_from(acc[0], acc[1]);
            if (run) {
                if (!(gap == gap)) {
                    nan_out = true;
                    run = false;
                    t_out = t;
                    gap_out = gap;
                } else if ((par.inner_rule == 0 && gap <= par.eps_in) || t >= par.k_in_max) {
                    run = false;
                    t_out = t;
                    // the gap that enters LB: the stopping certificate, or its
                    // sigma-free part (FW gap) when sigma is an estimate
                    gap_out = par.lb_cert == 2 ? acc[0] : gap;
                }
            }
            if (!__any(run)) break;   // every wave holds all 16 columns: same decision
            if (t > 0 && par.inner_variant == 2) th = 0.5 * (1.0 + sqrt(1.0 + 4.0 * th * th));
            if (run) {
#pragma unroll
                for (int j = 0; j < kTileRT; ++j)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        xp[j][i] = x[j][i];
                        qxp[j][i] = qx[j][i];
                        x[j][i] = xn[j][i];
                        qx[j][i] = qn[j][i];
                    }
            }
            sel ^= 1;
            ++t;
        }
        sel ^= 1;
    }

    __device__ __forceinline__ bool outer_ok(double F, double feas, double lnorm, double LB, double gnorm) const {
        const double sc = fmax(1.0, fabs(F));
        return feas <= a.par.eps_out * fmax(1.0, gnorm) && F - LB <= a.par.eps_out * sc &&
               lnorm * feas <= a.par.eps_out * sc;
    }

    __device__ __forceinline__ void solve_tile(int tile) {
        const DevParams& par = a.par;
        const int n = a.n, p = a.p;
        const int PT = (p + 15) / 16;
        b = tile * kTile + col;
        valid = b < a.B;
        double* mu = a.dual + (long)(valid ? b : 0) * 3 * p;
        double* lamp = mu + p;
        double* rs = mu + 2 * p;
        double* us = a.prim + (long)(valid ? b : 0) * 4 * n;
        double* qus = us + n;
        double* usave = us + 2 * n;
        double* qusave = us + 3 * n;
        const double* qb = a.q + (long)(valid ? b : 0) * n;
        const double* gb = a.g + (long)(valid ? b : 0) * p;

        // x^0 = projection of 0 on the box, lambda^0 = mu^1 = 0 (Sec. 4)
#pragma unroll
        for (int j = 0; j < kTileRT; ++j)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = row(j, i);
                x[j][i] = r < n ? fmin(fmax(0.0, box[r]), box[n + r]) : 0.0;
                if (valid && r < n) {
                    us[r] = 0.0;
                    qus[r] = 0.0;
                }
            }
        double gg[1] = {0.0};
        for (int rt = w; rt < PT; rt += kTileWaves)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 16 * rt + grp + 4 * i;
                if (valid && r < p) {
                    mu[r] = 0.0;
                    lamp[r] = 0.0;
                    rs[r] = 0.0;
                    gg[0] += gb[r] * gb[r];
                }
            }
        int sel = 0;
        put_x(Xs0, x);
        colsum<1>(gg, redK);
        __syncthreads();
        const double gnorm = sqrt(gg[0]);
        {
            tile_v4d acc[kTileRT];
            prodQ(Xs0, acc);
#pragma unroll
            for (int j = 0; j < kTileRT; ++j)
#pragma unroll
                for (int i = 0; i < 4; ++i) qx[j][i] = acc[j][i];
        }
        sel = 1;
        double theta = 1.0, S = 0.0, LB = -INFINITY;
        double Fc = 0.0, feasc = 0.0, lnc = 0.0;
        long long inner_total = 0;
        int k = 0, status = 1, gt = 0;
        int it = 0;             // loop trips (uniform); equals k of every active lane
        bool infeas = false;    // mu^k certified infeasibility: it is the output
        bool act = valid;
        const bool last_extra = par.output == 0 && par.method == 1;

        while (__any(act)) {
            if (act) ++k;
            ++it;
            // Step 1: inner solve at mu^k, warm-started from ubar^{k-1}
            linear_term(0);
            ++gt;
            if (p > 0 && it > 1 && it % kInfeasEvery == 1) {
                // certificate of infeasibility at mu^k (as in the per-instance
                // solver): v = mu^T g + sum_j min(lb_j w_j, ub_j w_j), w = c - q.
                // k = 1 is skipped: mu^1 = lambda^0 = 0 here, where v = 0 cannot
                // certify, so the outcome is that of testing it.
                double e[3] = {0.0, 0.0, 0.0};   // v, scale, #(mu < 0)
#pragma unroll
                for (int j = 0; j < kTileRT; ++j)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int r = row(j, i);
                        if (act && r < n) {
                            const double wv = c[j][i] - qb[r], lo = box[r], hi = box[n + r];
                            e[0] += fmin(lo * wv, hi * wv);
                            e[1] += fabs(wv) * fmax(fabs(lo), fabs(hi));
                        }
                    }
                for (int rt = w; rt < PT; rt += kTileWaves)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int r = 16 * rt + grp + 4 * i;
                        if (act && r < p) {
                            const double m = mu[r], mg = m * gb[r];
                            e[0] += mg;
                            e[1] += fabs(mg);
                            e[2] += m < 0.0 ? 1.0 : 0.0;
                        }
                    }
                colsum_long<3>(e, redK);
                if (act && e[2] == 0.0 && e[0] > kInfeasMargin * e[1]) {
                    status = kStInfeasible;
                    infeas = true;
                    act = false;
                }
            }
            int t;
            double gap;
            bool bad;
            inner(act, sel, t, gap, bad);
            if (act) inner_total += t;
            if (act && bad) {
                status = 2;
                act = false;
            }
            // Steps 2-3 fused into the epilogue of G ubar, and the averages
            const double thk = theta;
            const double thn = par.method == 1 ? 0.5 * (1.0 + sqrt(1.0 + 4.0 * thk * thk)) : 1.0;
            const double beta = (thk - 1.0) / thn;
            const double Sn = S + thk;
            double s[11];
#pragma unroll
            for (int z = 0; z < 11; ++z) s[z] = 0.0;
            double* Xs = sel ? Xs1 : Xs0;
            put_x(Xs, x);
            __syncthreads();
            for (int rt0 = w; rt0 < PT; rt0 += 2 * kTileWaves) {
                const bool two = rt0 + kTileWaves < PT;   // wave-uniform
                tile_v4d accs[2];
                prodG(Xs, rt0, two, accs[0], accs[1]);
#pragma unroll
                for (int hh = 0; hh < 2; ++hh)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const tile_v4d& acc = accs[hh];
                    const int r = 16 * (rt0 + hh * kTileWaves) + grp + 4 * i;
                    if (act && (hh == 0 || two) && r < p) {
                        const double ri = acc[i] + gb[r], mui = mu[r];
                        s[2] += mui * ri;
                        const double rp = fmax(ri, 0.0);
                        s[4] += rp * rp;
                        double lk = mui + par.alpha * ri;
                        if (par.Kd_nonneg) lk = fmax(lk, 0.0);
                        s[5] += lk * lk;
                        const double rsn = rs[r] + thk * ri;
                        rs[r] = rsn;
                        const double hp = fmax(rsn / Sn, 0.0);
                        s[6] += hp * hp;
                        s[7] += (mui < 0.0) ? 1.0 : 0.0;
                        s[10] += (lk < 0.0) ? 1.0 : 0.0;
                        mu[r] = lk + beta * (lk - lamp[r]);
                        lamp[r] = lk;
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < kTileRT; ++j)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = row(j, i);
                    if (act && r < n) {
                        const double ui = x[j][i], qui = qx[j][i], qi = qb[r];
                        s[0] += ui * qui;
                        s[1] += qi * ui;
                        const double usn = us[r] + thk * ui, qusn = qus[r] + thk * qui;
                        us[r] = usn;
                        qus[r] = qusn;
                        s[8] += usn * qusn;
                        s[9] += qi * usn;
                    }
                }
            colsum_long<11>(s, redK);
            bool ok = false, extra = false;
            double lnorm = 0.0;
            if (act) {
                const double Fu = 0.5 * s[0] + s[1];
                const double dbar = Fu + s[2];
                if (s[7] == 0.0) LB = fmax(LB, dbar - gap);
                S = Sn;
                double F, feas;
                if (par.output == 0) {
                    F = Fu;
                    feas = sqrt(s[4]);
                } else {
                    F = 0.5 * s[8] / (S * S) + s[9] / S;
                    feas = sqrt(s[6]);
                }
                lnorm = sqrt(s[5]);
                if (!(F == F) || !(LB == LB && dbar == dbar)) {
                    status = 2;
                    act = false;
                } else {
                    ok = outer_ok(F, feas, lnorm, LB, gnorm);
                    Fc = F;
                    feasc = feas;
                    lnc = lnorm;
                    extra = ok && last_extra;
                }
            }
            if (__any(extra)) {
                // Last iterate of DFGM: ubar(lambda^k), eq. last_primal, warm-started
#pragma unroll
                for (int j = 0; j < kTileRT; ++j)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (extra && row(j, i) < n) {
                            usave[row(j, i)] = x[j][i];
                            qusave[row(j, i)] = qx[j][i];
                        }
                linear_term(p);   // c = q + G^T lambda^k
                ++gt;
                int t2;
                double gap2;
                bool bad2;
                inner(extra, sel, t2, gap2, bad2);
                if (extra) inner_total += t2;
                double s2[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                double* Xs2 = sel ? Xs1 : Xs0;
                put_x(Xs2, x);
                __syncthreads();
                for (int rt0 = w; rt0 < PT; rt0 += 2 * kTileWaves) {
                    const bool two = rt0 + kTileWaves < PT;
                    tile_v4d accs[2];
                    prodG(Xs2, rt0, two, accs[0], accs[1]);
#pragma unroll
                    for (int hh = 0; hh < 2; ++hh)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const tile_v4d& acc = accs[hh];
                        const int r = 16 * (rt0 + hh * kTileWaves) + grp + 4 * i;
                        if (extra && (hh == 0 || two) && r < p) {
                            const double ri = acc[i] + gb[r];
                            s2[2] += lamp[r] * ri;
                            const double rp = fmax(ri, 0.0);
                            s2[4] += rp * rp;
                        }
                    }
                }
#pragma unroll
                for (int j = 0; j < kTileRT; ++j)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int r = row(j, i);
                        if (extra && r < n) {
                            s2[0] += x[j][i] * qx[j][i];
                            s2[1] += qb[r] * x[j][i];
                        }
                    }
                colsum_long<6>(s2, redK);
                if (extra) {
                    if (bad2) {
                        status = 2;
                        act = false;
                        ok = false;
                    } else {
                        const double F2 = 0.5 * s2[0] + s2[1];
                        const double d2 = F2 + s2[2];
                        if (s[10] == 0.0) LB = fmax(LB, d2 - gap2);
                        const double feas2 = sqrt(s2[4]);
                        const bool ok2 = outer_ok(F2, feas2, lnorm, LB, gnorm);
                        if (ok2) {
                            Fc = F2;
                            feasc = feas2;
                        } else {
                            ok = false;
                            // continue from ubar^k unchanged
#pragma unroll
                            for (int j = 0; j < kTileRT; ++j)
#pragma unroll
                                for (int i = 0; i < 4; ++i)
                                    if (row(j, i) < n) {
                                        x[j][i] = usave[row(j, i)];
                                        qx[j][i] = qusave[row(j, i)];
                                    }
                        }
                    }
                }
            }
            if (act) {
                theta = thn;
                if (ok) {
                    status = 0;
                    act = false;
                } else if (k >= par.max_outer) {
                    act = false;
                }
            }
        }
        (void)lnc;
        // outputs of this lane's column
        if (valid) {
#pragma unroll
            for (int j = 0; j < kTileRT; ++j)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = row(j, i);
                    if (r < n) a.X[(long)b * n + r] = (par.output == 1 && !infeas) ? us[r] / S : x[j][i];
                }
            for (int rt = w; rt < PT; rt += kTileWaves)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = 16 * rt + grp + 4 * i;
                    if (r < p) a.Lam[(long)b * p + r] = infeas ? mu[r] : lamp[r];
                }
            if (w == 0 && grp == 0) {
                BatchResultDev rr;
                rr.status = status;
                rr.outer = k;
                rr.inner = inner_total;
                rr.gt_rows = (long long)gt * p;
                rr.F = Fc;
                rr.LB = LB;
                rr.feas = feasc;
                rr.lam_min = a.lam_min;
                rr.lam_max = a.lam_max;
                rr.G2 = a.g2;
                a.res[b] = rr;
            }
        }
        __syncthreads();
    }
};

template <typename T>
__device__ __forceinline__ void tile_solve(const TileArgs<T>& args, double* lds) {
    __shared__ int s_tile;
    Tile<T> s;
    s.a = args;
    const int n = args.n;
    s.Xs0 = lds;
    s.Xs1 = s.Xs0 + tile_kp(n) * kTile;
    s.red2 = s.Xs1 + tile_kp(n) * kTile;
    s.redK = s.red2 + 2 * kTileWaves * kTile * 2;
    s.box = s.redK + kTileWaves * kTile * kTileK;
    s.lane = threadIdx.x & 63;
    s.w = threadIdx.x >> 6;
    s.col = s.lane & 15;
    s.grp = s.lane >> 4;
    s.invL = 1.0 / args.par.L;
    // this lane's entries of Q into registers once; both X buffers cleared:
    // their rows >= n stay zero
    s.load_q();
    for (int e = threadIdx.x; e < 2 * tile_kp(n) * kTile; e += blockDim.x) s.Xs0[e] = 0.0;
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        s.box[e] = args.lb[e];
        s.box[n + e] = args.ub[e];
    }
    __syncthreads();
    for (;;) {
        if (threadIdx.x == 0) s_tile = (int)atomicAdd(args.queue, 1u);
        __syncthreads();
        const int tile = s_tile;
        __syncthreads();
        if ((long)tile * kTile >= args.B) break;
        s.solve_tile(tile);
    }
}

}  // namespace duq
