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
#include <type_traits>

#include "device_common.h"
#include "internal.h"

namespace duq {

constexpr int kTile = 16;       // instances per workgroup
constexpr int kTileWaves = 4;   // waves per workgroup, one per SIMD (512 registers each)
constexpr int kTileRT = 2;      // row tiles of 16 per wave: n <= 16 * kTileWaves * kTileRT
constexpr int kTileQS = 32;     // k-steps of 4 columns of Q held per lane: n <= 4 * kTileQS
constexpr int kTileK = 7;       // slots of the outer reduction buffer (longer records go in chunks)
constexpr int kTileRows = 16 * kTileWaves * kTileRT;   // rows the waves hold (n and zero padding)

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

// LDS layout, in doubles: two buffers of the B operand X (kTileRows x 16;
// rows from n on stay zero), the inner reduction (two buffers), the outer
// one, the box (lb then ub, kTileRows each; rows from n on are [0, 0]).
__host__ __device__ inline int tile_kp(int n) { return (n + 3) & ~3; }
__host__ __device__ inline long tile_lds_doubles(int n) {
    (void)n;
    return 2L * kTileRows * kTile + 2L * kTileWaves * kTile * 2 + (long)kTileWaves * kTile * kTileK + 2L * kTileRows;
}

template <typename T>
struct Tile {
    TileArgs<T> a;
    double* Xs0;
    double* Xs1;
    double* red2;
    double* redK;
    double* box;     // LDS: lb then ub (kTileRows each, [0, 0] on padding rows)
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

    // k-steps per batch of the G products: every load of a batch is issued
    // before its MFMAs (one round trip to memory per batch), from clamped
    // addresses, and out-of-range terms are zeroed after the load.
    static constexpr int kBo = 16;

    // acc[j] = G^T v over this wave's row tiles of n; v (p entries) is this
    // lane's multiplier vector.  The
    // multipliers of a batch are read first; a batch in which every
    // multiplier of the tile is zero adds nothing and is skipped.  Returns
    // the number of this lane's nonzero multipliers.
    __device__ __forceinline__ int prodGT(const double* vb, tile_v4d (&acc)[kTileRT]) const {
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
        int nz = 0;
        for (int s0 = 0; s0 < ks; s0 += kBo) {
            double bv[kBo];
            bool any = false;
#pragma unroll
            for (int u = 0; u < kBo; ++u) {
                const int k = 4 * (s0 + u) + grp;
                const bool kv = s0 + u < ks && k < p;
                const double m = vb[kv ? k : 0];
                bv[u] = (kv && valid) ? m : 0.0;
                nz += bv[u] != 0.0;
                any = any || bv[u] != 0.0;
            }
            if (!__any(any)) continue;   // every wave holds the same 16 columns: same decision
            double av[kTileRT][kBo];
#pragma unroll
            for (int u = 0; u < kBo; ++u) {
                const int k = 4 * (s0 + u) + grp;
                const bool kv = s0 + u < ks && k < p;
                const long gk = (long)(kv ? k : 0) * n;
#pragma unroll
                for (int j = 0; j < kTileRT; ++j) {
                    const double gv = (double)a.G[gk + cidx[j]];
                    av[j][u] = (v[j] && kv) ? gv : 0.0;
                }
            }
#pragma unroll
            for (int u = 0; u < kBo; ++u)
#pragma unroll
                for (int j = 0; j < kTileRT; ++j)
                    acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[j][u], bv[u], acc[j], 0, 0, 0);
        }
        return nz;
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
        for (int s0 = 0; s0 < ks; s0 += kBo) {
            double x0[kBo], x1[kBo], bv[kBo];
#pragma unroll
            for (int u = 0; u < kBo; ++u) {
                const int k = 4 * (s0 + u) + grp;
                const bool kv = s0 + u < ks && k < n;
                const int kk = kv ? k : 0;
                // Xs rows from n on are zero; its kTileRows rows cover every k
                bv[u] = s0 + u < kTileQS ? Xs[(4 * (s0 + u) + grp) * kTile + col] : 0.0;
                const double g0 = (double)ga[kk], g1 = (double)gb2[kk];
                x0[u] = (va && kv) ? g0 : 0.0;
                x1[u] = (vb2 && kv) ? g1 : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kBo; ++u) {
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

    // The quotient is formed whatever sigma is (with sigma = 0 it is
    // discarded), so the inner step has no branch here.
    __device__ __forceinline__ double gap_from(double fw, double pi2) const {
        const double m = fmin(fw, pi2 / (2.0 * a.par.sigma));
        const bool use = a.par.sigma > 0.0;
        return use ? m : fw;
    }

    // c = q + G^T v for this lane's rows; returns the number of nonzero
    // multipliers of this lane's instance (the rows of G^T the product needs).
    __device__ __forceinline__ long long linear_term(const double* v, bool zero) {
        tile_v4d acc[kTileRT];
        int nz = 0;
        if (zero) {   // uniform: every multiplier of the tile is zero
#pragma unroll
            for (int j = 0; j < kTileRT; ++j) acc[j] = tile_v4d{0.0, 0.0, 0.0, 0.0};
        } else {
            nz = prodGT(v, acc);
        }
#pragma unroll
        for (int j = 0; j < kTileRT; ++j)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = row(j, i);
                c[j][i] = (valid && r < a.n) ? a.q[(long)b * a.n + r] + acc[j][i] : 0.0;
            }
        return (long long)grpsum((double)nz);
    }

    // Sum of v over the four lane groups of each column (lanes l, l ^ 16,
    // l ^ 32, l ^ 48), as (v_g0 + v_g1) + (v_g2 + v_g3) in every lane: the
    // row swaps of gfx950 (permlane16/32 swap) exchange the halves in VALU
    // registers, without a round trip through LDS.
    __device__ __forceinline__ static double grpsum(double v) {
        const unsigned lo = __double2loint(v), hi = __double2hiint(v);
        const auto a16 = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        const auto b16 = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        const double s = __hiloint2double(b16[0], a16[0]) + __hiloint2double(b16[1], a16[1]);
        const unsigned lo2 = __double2loint(s), hi2 = __double2hiint(s);
        const auto a32 = __builtin_amdgcn_permlane32_swap(lo2, lo2, false, false);
        const auto b32 = __builtin_amdgcn_permlane32_swap(hi2, hi2, false, false);
        return __hiloint2double(b32[0], a32[0]) + __hiloint2double(b32[1], a32[1]);
    }

    // acc[j] = Q Xs as prodQ, over all kTileQS k-steps in straight-line code
    // (Xs rows from n on are zero).  After the two MFMAs of k-step S comes
    // work(S), a piece of work independent of the product: it issues while
    // those MFMAs run.  Only LDS reads may be moved across the pieces.
    template <int S, typename F>
    __device__ __forceinline__ void prodQ_with(const double* Xs, tile_v4d (&acc)[kTileRT], F& work) const {
        if constexpr (S == 0) {
#pragma unroll
            for (int j = 0; j < kTileRT; ++j) acc[j] = tile_v4d{0.0, 0.0, 0.0, 0.0};
        }
        if constexpr (S < kTileQS) {
            const double bv = Xs[(4 * S + grp) * kTile + col];
#pragma unroll
            for (int j = 0; j < kTileRT; ++j)
                acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[j][S], bv, acc[j], 0, 0, 0);
            work(std::integral_constant<int, S>{});
            __builtin_amdgcn_sched_barrier(0x100);
            prodQ_with<S + 1>(Xs, acc, work);
        }
    }

    // Algorithm FOM (rho = 0) on the tile from x (Q x in qx) with the linear
    // term c, for the lanes with `on`; the others keep their state.  On
    // return x / qx hold ubar and Q ubar; t_out, gap_out the inner count and
    // certificate; nan_out a non-finite certificate.
    //
    // Step t: with Q x^t at hand, the certificate terms at x^t and
    // x^{t+1} = P(y^t - (Q y^t + c) / L) (Q y^t by linearity) are formed and
    // published with one workgroup barrier; the product Q x^{t+1} is then
    // issued, and while it runs the certificate of x^t is summed and tested,
    // the next momentum coefficient formed and y^{t+1} computed.  A column
    // that stops keeps x^t, Q x^t; its later iterates only feed its own
    // MFMA column and are dropped.
    __device__ __forceinline__ void inner(bool on, int& sel, int& t_out, double& gap_out, bool& nan_out) {
        const DevParams& par = a.par;
        double bl[kTileRT][4], bh[kTileRT][4], y[kTileRT][4], qp[kTileRT][4];
#pragma unroll
        for (int j = 0; j < kTileRT; ++j)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                bl[j][i] = box[row(j, i)];
                bh[j][i] = box[kTileRows + row(j, i)];
                y[j][i] = x[j][i];     // y^0 = x^0 (beta_0 = 0)
                qp[j][i] = qx[j][i];
            }
        bool run = on;
        int t = 0;
        double th = 1.0;   // theta_t of the FGM rule (inner_variant 2)
        double fth = 1.0;  // theta_{t+1}
        double beta = 0.0; // momentum coefficient of step t
        t_out = 0;
        gap_out = 0.0;
        nan_out = false;
        for (;;) {
            double acc[2] = {0.0, 0.0};
            double xn[kTileRT][4];
#pragma unroll
            for (int j = 0; j < kTileRT; ++j)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    // rows from n on: box [0, 0], c = 0, Q rows 0: every term 0
                    const double xi = x[j][i], gr = qx[j][i] + c[j][i];
                    const double l = bl[j][i], h = bh[j][i];
                    // exact-gradient certificate terms at x (fw, pi^2)
                    acc[0] += fmax(gr * (xi - l), gr * (xi - h));
                    const bool atl = xi <= l, atu = xi >= h;
                    const double glo = fmin(gr, 0.0), ghi = fmax(gr, 0.0);
                    const double pu = atu ? ghi : gr, pl = atl ? glo : pu;
                    const double pi = (atl && atu) ? 0.0 : pl;
                    acc[1] += pi * pi;
                    const double qyi = qx[j][i] + beta * (qx[j][i] - qp[j][i]);
                    xn[j][i] = fmin(fmax(y[j][i] - (qyi + c[j][i]) * invL, l), h);
                }
            double* Xs = sel ? Xs1 : Xs0;
            double* rbuf = red2 + sel * (kTileWaves * kTile * 2);
#pragma unroll
            for (int j = 0; j < kTileRT; ++j)
#pragma unroll
                for (int i = 0; i < 4; ++i) Xs[row(j, i) * kTile + col] = xn[j][i];
            acc[0] = grpsum(acc[0]);
            acc[1] = grpsum(acc[1]);
            if (grp == 0) {
                rbuf[(w * kTile + col) * 2] = acc[0];
                rbuf[(w * kTile + col) * 2 + 1] = acc[1];
            }
            __syncthreads();   // Xs and the partial sums
            tile_v4d qn[kTileRT];
            double s0 = 0.0, s1 = 0.0, gap = 0.0, thn = 1.0, fthn = 1.0, bn = 0.0;
            auto work = [&](auto P) {
                constexpr int ph = decltype(P)::value;
                if constexpr (ph == 1) {
                    s0 = rbuf[col * 2];
                    s1 = rbuf[col * 2 + 1];
#pragma unroll
                    for (int ww = 1; ww < kTileWaves; ++ww) {
                        s0 += rbuf[(ww * kTile + col) * 2];
                        s1 += rbuf[(ww * kTile + col) * 2 + 1];
                    }
                } else if constexpr (ph == 2) {
                    gap = gap_from(s0, s1);
                } else if constexpr (ph == 3) {
                    const bool isnan = !(gap == gap);
                    const bool stop =
                        run && (isnan || (par.inner_rule == 0 && gap <= par.eps_in) || t >= par.k_in_max);
                    // the gap that enters LB: the stopping certificate, or its
                    // sigma-free part (FW gap) when sigma is an estimate
                    const double gl = (isnan || par.lb_cert != 2) ? gap : s0;
                    gap_out = stop ? gl : gap_out;
                    t_out = stop ? t : t_out;
                    nan_out = nan_out || (stop && isnan);
                    run = run && !stop;
                } else if constexpr (ph == 4) {
                    // momentum coefficient of step t + 1 (FGM: theta_{t+1} is
                    // theta_t for t = 0 and the theta rule applied to it after)
                    thn = t > 0 ? fth : th;
                    fthn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * thn * thn));
                } else if constexpr (ph == 5) {
                    const double bfgm = (thn - 1.0) / fthn;
                    const double b3 = par.beta_in, b0 = 0.0;
                    const bool v2 = par.inner_variant == 2, v3 = par.inner_variant == 3;
                    const double b2 = v2 ? bfgm : b0;
                    bn = v3 ? b3 : b2;
                    th = thn;
                    fth = fthn;
                    beta = bn;
                } else if constexpr (ph >= 6 && ph < 6 + 2 * kTileRT) {
                    // next state, two rows per piece; a stopped column keeps
                    // x (and Q x, below)
                    constexpr int j = (ph - 6) / 2, i0 = 2 * ((ph - 6) % 2);
#pragma unroll
                    for (int i = i0; i < i0 + 2; ++i) {
                        y[j][i] = xn[j][i] + bn * (xn[j][i] - x[j][i]);
                        qp[j][i] = qx[j][i];
                        x[j][i] = run ? xn[j][i] : x[j][i];
                    }
                }
            };
            prodQ_with<0>(Xs, qn, work);
#pragma unroll
            for (int j = 0; j < kTileRT; ++j)
#pragma unroll
                for (int i = 0; i < 4; ++i) qx[j][i] = run ? qn[j][i] : qx[j][i];
            if (!__any(run)) break;   // every wave holds all 16 columns: same decision
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
        // lambda^k is kept in the output array itself (the last one written
        // is the result); a lane past the batch points at a record it never
        // writes
        double* lamp = valid ? a.Lam + (long)b * p : mu + p;
        double* rs = mu + 2 * p;
        // the averages (sums of theta_j ubar^j, theta_j Q ubar^j, theta_j r^j)
        // are formed only when the averaged primal point is the output
        const bool avg = par.output == 1;
        double* us = a.prim + (long)(valid ? b : 0) * 4 * n;
        double* qus = us + n;
        double* usave = us + 2 * n;
        double* qusave = us + 3 * n;
        const double* qb = a.q + (long)(valid ? b : 0) * n;
        const double* gb = a.g + (long)(valid ? b : 0) * p;

        // x^0 = projection of 0 on the box, lambda^0 = mu^1 = 0 (Sec. 4): the
        // multipliers and the sums start at zero, which the first outer
        // iteration uses without reading them (nothing is stored before)
#pragma unroll
        for (int j = 0; j < kTileRT; ++j)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = row(j, i);
                x[j][i] = r < n ? fmin(fmax(0.0, box[r]), box[kTileRows + r]) : 0.0;
            }
        double gg[1] = {0.0};
        // rows of p in chunks of four row tiles: the loads of a chunk are
        // issued together (clamped addresses), then used in row order
        for (int rt0 = w; rt0 < PT; rt0 += 4 * kTileWaves) {
            double gv[4][4];
#pragma unroll
            for (int c4 = 0; c4 < 4; ++c4)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = 16 * (rt0 + c4 * kTileWaves) + grp + 4 * i;
                    gv[c4][i] = gb[r < p ? r : 0];
                }
#pragma unroll
            for (int c4 = 0; c4 < 4; ++c4)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = 16 * (rt0 + c4 * kTileWaves) + grp + 4 * i;
                    if (valid && r < p) gg[0] += gv[c4][i] * gv[c4][i];
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
        int k = 0, status = 1;
        long long gt = 0;   // nonzero multipliers of the G^T products (rows of G^T read)
        int it = 0;             // loop trips (uniform); equals k of every active lane
        bool infeas = false;    // mu^k certified infeasibility: it is the output
        bool act = valid;
        bool mu_zero = true;    // mu^1 = 0 in every column of the tile
        const bool last_extra = par.output == 0 && par.method == 1;

        bool dual_ok = false;   // this lane's multipliers have been written
        while (__any(act)) {
            if (act) ++k;
            ++it;
            const bool first = it == 1;   // mu = lambda = 0 and the sums are 0
            // Step 1: inner solve at mu^k, warm-started from ubar^{k-1}
            {
                const long long g1 = linear_term(mu, mu_zero);
                if (act) gt += g1;
            }
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
                            const double wv = c[j][i] - qb[r], lo = box[r], hi = box[kTileRows + r];
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
            double s[13];
#pragma unroll
            for (int z = 0; z < 13; ++z) s[z] = 0.0;
            double* Xs = sel ? Xs1 : Xs0;
            put_x(Xs, x);
            __syncthreads();
            for (int rt0 = w; rt0 < PT; rt0 += 2 * kTileWaves) {
                const bool two = rt0 + kTileWaves < PT;   // wave-uniform
                // this lane's entries of g, mu, the sum of theta r and lambda
                // for the rows of the pair, read before the product
                double pg[2][4], pm[2][4], prs[2][4], pl[2][4];
#pragma unroll
                for (int hh = 0; hh < 2; ++hh)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int r = 16 * (rt0 + hh * kTileWaves) + grp + 4 * i, rr = r < p ? r : 0;
                        pg[hh][i] = gb[rr];
                        pm[hh][i] = first ? 0.0 : mu[rr];
                        prs[hh][i] = (first || !avg) ? 0.0 : rs[rr];
                        pl[hh][i] = first ? 0.0 : lamp[rr];
                    }
                tile_v4d accs[2];
                prodG(Xs, rt0, two, accs[0], accs[1]);
#pragma unroll
                for (int hh = 0; hh < 2; ++hh)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const tile_v4d& acc = accs[hh];
                    const int r = 16 * (rt0 + hh * kTileWaves) + grp + 4 * i;
                    if (act && (hh == 0 || two) && r < p) {
                        const double ri = acc[i] + pg[hh][i], mui = pm[hh][i];
                        s[2] += mui * ri;
                        const double rp = fmax(ri, 0.0);
                        s[4] += rp * rp;
                        double lk = mui + par.alpha * ri;
                        if (par.Kd_nonneg) lk = fmax(lk, 0.0);
                        s[5] += lk * lk;
                        if (avg) {
                            const double rsn = prs[hh][i] + thk * ri;
                            rs[r] = rsn;
                            const double hp = fmax(rsn / Sn, 0.0);
                            s[6] += hp * hp;
                        }
                        s[7] += (mui < 0.0) ? 1.0 : 0.0;
                        s[10] += (lk < 0.0) ? 1.0 : 0.0;
                        const double mun = lk + beta * (lk - pl[hh][i]);
                        s[11] += (lk != 0.0) ? 1.0 : 0.0;
                        s[12] += (mun != 0.0) ? 1.0 : 0.0;
                        mu[r] = mun;
                        lamp[r] = lk;
                    }
                }
            }
            if (act) dual_ok = true;
#pragma unroll
            for (int j = 0; j < kTileRT; ++j)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = row(j, i);
                    if (act && r < n) {
                        const double ui = x[j][i], qui = qx[j][i], qi = qb[r];
                        s[0] += ui * qui;
                        s[1] += qi * ui;
                        if (avg) {
                            const double us0 = first ? 0.0 : us[r], qus0 = first ? 0.0 : qus[r];
                            const double usn = us0 + thk * ui, qusn = qus0 + thk * qui;
                            us[r] = usn;
                            qus[r] = qusn;
                            s[8] += usn * qusn;
                            s[9] += qi * usn;
                        }
                    }
                }
            colsum_long<13>(s, redK);
            // a G^T product whose multipliers are zero in every column of
            // the tile adds nothing: lambda^k feeds the last-iterate solve,
            // mu^{k+1} the next outer iteration
            const bool lam_zero = !__any(s[11] != 0.0);
            mu_zero = !__any(s[12] != 0.0);
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
                const long long g2n = linear_term(lamp, lam_zero);   // c = q + G^T lambda^k
                if (extra) gt += g2n;
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
                    double pg[2][4], pl[2][4];
#pragma unroll
                    for (int hh = 0; hh < 2; ++hh)
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int r = 16 * (rt0 + hh * kTileWaves) + grp + 4 * i, rr = r < p ? r : 0;
                            pg[hh][i] = gb[rr];
                            pl[hh][i] = lamp[rr];
                        }
                    tile_v4d accs[2];
                    prodG(Xs2, rt0, two, accs[0], accs[1]);
#pragma unroll
                    for (int hh = 0; hh < 2; ++hh)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const tile_v4d& acc = accs[hh];
                        const int r = 16 * (rt0 + hh * kTileWaves) + grp + 4 * i;
                        if (extra && (hh == 0 || two) && r < p) {
                            const double ri = acc[i] + pg[hh][i];
                            s2[2] += pl[hh][i] * ri;
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
                    if (r < n) a.X[(long)b * n + r] = (avg && !infeas && dual_ok) ? us[r] / S : x[j][i];
                }
            // lambda^k is already in place; an infeasible instance outputs its
            // certificate mu^k, one whose multipliers were never formed zeros
            if (infeas || !dual_ok) {
                for (int rt0 = w; rt0 < PT; rt0 += 4 * kTileWaves) {
                    double lv[4][4];
#pragma unroll
                    for (int c4 = 0; c4 < 4; ++c4)
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int r = 16 * (rt0 + c4 * kTileWaves) + grp + 4 * i;
                            lv[c4][i] = infeas ? mu[r < p ? r : 0] : 0.0;
                        }
#pragma unroll
                    for (int c4 = 0; c4 < 4; ++c4)
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int r = 16 * (rt0 + c4 * kTileWaves) + grp + 4 * i;
                            if (r < p) lamp[r] = lv[c4][i];
                        }
                }
            }
            if (w == 0 && grp == 0) {
                BatchResultDev rr;
                rr.status = status;
                rr.outer = k;
                rr.inner = inner_total;
                rr.gt_rows = gt;
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
    s.Xs1 = s.Xs0 + kTileRows * kTile;
    s.red2 = s.Xs1 + kTileRows * kTile;
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
    for (int e = threadIdx.x; e < 2 * kTileRows * kTile; e += blockDim.x) s.Xs0[e] = 0.0;
    for (int e = threadIdx.x; e < kTileRows; e += blockDim.x) {
        s.box[e] = e < n ? args.lb[e] : 0.0;
        s.box[kTileRows + e] = e < n ? args.ub[e] : 0.0;
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
