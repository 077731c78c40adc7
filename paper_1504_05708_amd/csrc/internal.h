// Internal structures shared by the host runtime and the HIP kernels.
#pragma once
#include <stdint.h>

namespace duq {

// Scalars reduced per block: count of slots in one partial record.
constexpr int kNP = 12;
// Grid-barrier words: generation at 0, error flag at kBarErr, arrival epoch
// of workgroup b at kBarFlag + 32 b (one 128-byte line each).
constexpr int kBarErr = 32;
constexpr int kBarFlag = 64;
constexpr long bar_words(int nblocks) { return (long)kBarFlag + 32L * (nblocks + 1); }

// Solver status of a run that found a certificate of infeasibility, the
// relative margin that certificate must clear and the outer iterations at
// which it is tested, k = 1, 1 + kInfeasEvery, ... (see Dfom::inner_rho0).
constexpr int kStInfeasible = 5;
constexpr double kInfeasMargin = 1e-6;
constexpr int kInfeasEvery = 8;

// Scalars of one trace record.
constexpr int kTraceScalars = 16;

// Problem as seen by a kernel (device pointers).  Q is n x n, G is p x n,
// both row-major with leading dimension n.
template <typename T>
struct DevProblem {
    int n, p;
    const T* Q;
    const T* G;
    const double* q;
    const double* g;
    const double* lb;
    const double* ub;
    // Row bounds of the user form rlo <= G u + g <= rhi (Sec. 2), or null for
    // G u + g <= 0.  rlo = rhi: an equality; +-inf: an absent side.
    const double* rlo = nullptr;
    const double* rhi = nullptr;
    // Sparse Q and G (compressed rows; Qrp null for dense data): Q (n rows),
    // G (p rows) and G^T (n rows, for the transposed product).
    const long long* Qrp = nullptr;
    const int* Qci = nullptr;
    const T* Qv = nullptr;
    const long long* Grp = nullptr;
    const int* Gci = nullptr;
    const T* Gv = nullptr;
    const long long* Trp = nullptr;
    const int* Tci = nullptr;
    const T* Tv = nullptr;
    int Qlg = 0, Glg = 0, Tlg = 0;   // log2 of the lanes per row of each product
};

// Type-erased compressed-row arrays of a sparse problem (host runtime).
struct SparseRefs {
    const long long* Qrp = nullptr;
    const int* Qci = nullptr;
    const void* Qv = nullptr;
    const long long* Grp = nullptr;
    const int* Gci = nullptr;
    const void* Gv = nullptr;
    const long long* Trp = nullptr;
    const int* Tci = nullptr;
    const void* Tv = nullptr;
    int Qlg = 0, Glg = 0, Tlg = 0;
};

// Per-solve parameters derived on the host from the options and constants.
struct DevParams {
    int method;        // 0 DGM, 1 DFGM
    int output;        // 0 LAST, 1 AVG
    int inner_rule;    // 0 CERT, 1 FIXED
    int inner_variant; // resolved: 1 GM, 2 FGM, 3 FGM_sigma
    int max_outer;
    int k_in_max;
    int trace_iters;
    int Kd_nonneg;     // project multipliers onto R^p_+
    int has_x0;
    int has_lam0;
    int resume;        // continue from the state left by a previous launch:
                       // 1 recomputing the warm start's products (precision
                       // switch), 2 keeping the stored ones (time slicing)
    int phase1;        // first precision phase: no last-iterate solve, stall exit
    int stall_iters;   // phase 1 ends after this many iterations without progress
    int eqform;        // every row an equality and rho > 0: Q holds Q + rho G^T G
                       // (Sec. 5.1), the inner loop is the rho = 0 one
    int x_global;      // sparse data: x read in place from its buffer, not staged in LDS
    int lb_cert;       // inner gap entering LB: 1 sigma form, 2 sigma-free
    double eps_out;    // outer tolerance used by this launch
    double eps_in;
    double rho;
    double alpha;      // 1/(2 L_d)
    double L;          // L_in
    double sigma;      // sigma_in
    double beta_in;    // FGM_sigma momentum
};

// Scalar solver state kept in device memory between launches and the
// final result of a solve.
struct DevState {
    int status;        // 0 ok, 1 max outer, 2 numeric, 3 phase-1 stall, 5 infeasible
    int done;          // outer test passed
    int k;             // outer iterations completed
    int cur;           // index of the warm-start buffer
    long long inner;   // total inner steps
    long long gt_rows; // G rows touched by transposed products
    double theta;
    double S;
    double LB;
    double F;
    double feas;
    double lnorm;
    double gnorm;
    double best_metric; // used by the precision switch (stall detection)
    int stall;
    int n_trace;
};

// Device workspace of one instance.  All pointers refer to one allocation.
struct DevWork {
    double* xb[3];     // rotating inner iterates x^{t-1}, x^t, x^{t+1}
    double* qb[3];     // matching products Q x
    double* c;         // q + G^T mu (rho = 0)
    double* us;        // sum_j theta_j ubar^j
    double* qus;       // sum_j theta_j Q ubar^j
    double* usave;     // ubar^k kept across the extra DFGM-last solve
    double* qusave;
    double* xout;      // returned primal point
    double* r;         // G u + g for the owned rows
    double* rs;        // sum_j theta_j (G ubar^j + g)
    double* lamp;      // lambda^{k} (after the step) = lambda^{k-1} before it
    double* mu;        // mu^k
    double* lamm;      // row bounds: multipliers of the lower sides (lambda-)
    double* mum;       //   and their extrapolation (mu-)
    double* nu;        // row bounds: returned multiplier per row, lambda+ - lambda-
    double* wsh;       // sparse G on a grid team: the weights of G^T w, written
                       // by their owners and read by every workgroup
    double* wv;        // rho > 0: [mu + rho (G y + g)]_+
    double* gsave;     // rho > 0: G ubar^k kept across the extra DFGM-last solve
    double* gx[3];     // rho > 0: G x for the rotating iterates
    double* part;      // 2 x nblocks x kNP partial sums (ping-pong)
    double* gtp;       // nblocks x n partial columns of G^T v
    double* trace;     // trace records
    const double* x0;  // optional warm start (device)
    const double* lam0;
    DevState* st;
    unsigned* bar;     // grid-barrier words (kBarErr: error flag)
};

// Per-instance result of a batched solve.
struct BatchResultDev {
    int status;          // 0 ok, 1 max outer, 2 numeric, 4 invalid constants, 5 infeasible
    int outer;
    long long inner;
    long long gt_rows;
    double F, LB, feas;
    double lam_min, lam_max, G2;
};

// One active request of the serving loop: where its data, outputs and
// persistent workspace live, and the constants found in its first slice.
struct ServeInst {
    const void* Q;
    const void* G;
    const double* q;
    const double* g;
    const double* lb;
    const double* ub;
    double* x;
    double* lam;
    char* slot;          // workspace carved by batch_carve(n, p, k)
    int n, p, k;         // k: Krylov steps (0 when the constants are given)
    int resume;          // 1: continue from the state in `slot`
    int given;           // 1: lam_min, lam_max, g2 below are to be used
    int pad;
    double lam_min, lam_max, g2;
};

// Workspace of the Lanczos constant estimate.
struct LanczosWork {
    double* V;       // (k+1) x n basis
    double* w;       // n
    double* r;       // p (G v for the G^T G operator)
    double* part;    // nblocks x (k+2) partial sums
    double* gtp;     // nblocks x n partial columns (G^T r)
    double* ab;      // alpha[0..k), beta[0..k]
    double* out;     // [theta_min, theta_max, steps]
    unsigned* bar;
    double* rsh = nullptr;   // sparse G on a grid team: G v shared by every workgroup
    int x_global = 0;        // sparse data: Krylov vectors read in place, not staged in LDS
};

}  // namespace duq
