// FP64 Lanczos estimate of extreme eigenvalues on the device (setup step of
// the method: the constants lambda_min(Q), lambda_max(Q) and ||G||^2 that
// define L_d (Sec. 2 eq. Ld) and the inner L, sigma (Sec. 3, Step 1)).
//
// Operator A is either Q (n x n) or G^T G (through G and G^T).  Full
// reorthogonalisation (two classical Gram-Schmidt passes) keeps the Krylov
// basis orthogonal in FP64; the extreme eigenvalues of the k x k tridiagonal
// matrix are found by Sturm-sequence bisection.
#pragma once
#include "dfom_solver.h"

namespace duq {

// xsum_strided for C columns at once: column c (c < nc) sums
// base + c * cstep + b * stride over the same b sequence, each column in
// exactly the order of xsum_strided, with 4 C loads in flight.
template <int C>
__device__ __forceinline__ void xsum_strided_cols(const double* base, long stride, long cstep, int nc, int first,
                                                  int step, int nb, double (&s)[C]) {
#pragma unroll
    for (int c = 0; c < C; ++c) s[c] = 0.0;
    int b = first;
    for (; b + 3 * step < nb; b += 4 * step) {
        double v[C][4];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            if (c < nc) {
#pragma unroll
                for (int u = 0; u < 4; ++u) v[c][u] = xload(base + c * cstep + (long)(b + u * step) * stride);
            }
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            if (c < nc) {
#pragma unroll
                for (int u = 0; u < 4; ++u) s[c] += v[c][u];
            }
        }
    }
    for (; b < nb; b += step) {
#pragma unroll
        for (int c = 0; c < C; ++c)
            if (c < nc) s[c] += xload(base + c * cstep + (long)b * stride);
    }
}

template <typename T, bool SHORT, bool SPARSE = false>
struct Lanczos {
    DevProblem<T> P;
    LanczosWork L;
    Team tm;
    int k;
    int use_gtg;
    int nlo, nhi, plo, phi;
    double* xl;
    double* vl;
    double* hl;      // LDS: k+2 reduced values
    double* red;
    double* tl;      // LDS: blockDim*4 doubles for short-row G^T v

    // The Krylov basis V is staged by every workgroup: device-scope accesses
    // on a grid team.  w is private to its owner rows.
    __device__ __forceinline__ void vput(double* p, double v) const {
        if (tm.size > 1) xstore(p, v); else *p = v;
    }
    __device__ __forceinline__ double vget(const double* p) const { return tm.size > 1 ? xload(p) : *p; }
    __device__ __forceinline__ double wget(const double* w, int i) const {
        return (w == L.V) ? vget(w + i) : w[i];
    }

    // h[j] = sum_i V[j][i] w[i] for j < m over the team; result in hl.
    __device__ __forceinline__ bool dots(const double* w, int m) {
        const int n = P.n;
        const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
        const int ncol = k + 2;
        // Wave wid owns the columns j = wid (mod nw) and takes C of them per
        // trip, so C loads per lane are in flight; each column is summed in the
        // same order whatever C is.
        constexpr int C = 4;
        for (int j0 = wid; j0 < m; j0 += C * nw) {
            double s[C];
#pragma unroll
            for (int c = 0; c < C; ++c) s[c] = 0.0;
            // opaque lane index: keeps the column addresses from being hoisted
            // out of the Lanczos loop (they would stay live and spill)
            int ln = lane;
            asm volatile("" : "+v"(ln));
            for (int i = nlo + ln; i < nhi; i += kWave) {
                const double wi = wget(w, i);
                double v[C];
#pragma unroll
                for (int c = 0; c < C; ++c)
                    if (j0 + c * nw < m) v[c] = vget(L.V + (long)(j0 + c * nw) * n + i);
#pragma unroll
                for (int c = 0; c < C; ++c)
                    if (j0 + c * nw < m) s[c] += v[c] * wi;
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int j = j0 + c * nw;
                if (j < m) {
                    const double t = wave_sum(s[c]);
                    if (lane == 0) {
                        if (tm.size == 1) hl[j] = t;
                        else xstore(L.part + (long)tm.rank * ncol + j, t);
                    }
                }
            }
        }
        if (tm.size == 1) { __syncthreads(); return true; }
        if (tm.sync()) return false;
        for (int j0 = wid; j0 < m; j0 += C * nw) {
            const int nc = min(C, (m - 1 - j0) / nw + 1);
            double s[C];
            xsum_strided_cols<C>(L.part + j0, ncol, (long)nw, nc, lane, kWave, tm.size, s);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                if (c < nc) {
                    const double t = wave_sum(s[c]);
                    if (lane == 0) hl[j0 + c * nw] = t;
                }
            }
        }
        __syncthreads();
        // the next writer of part must not overtake readers: barrier
        if (tm.sync()) return false;
        return true;
    }

    __device__ __forceinline__ bool apply(const double* v, double* w) {
        const int n = P.n;
        if constexpr (SPARSE) {
            if (L.x_global) __syncthreads();   // v read in place (device-scope on a grid team)
            else if (tm.size > 1) stage_shared(v, n, xl);
            else stage(v, n, xl);
            return apply_sparse(v, w);
        }
        if (tm.size > 1) stage_shared(v, n, xl); else stage(v, n, xl);
        if (!use_gtg) {
            if (tm.size > 1) gemv_rows<T, double, 16, true, SHORT>(P.Q, n, nlo, nhi, n, xl, w, nullptr);
            else gemv_rows<T, double, 16, false, SHORT>(P.Q, n, nlo, nhi, n, xl, w, nullptr);
            __syncthreads();
            return true;
        }
        if (tm.size > 1) gemv_rows<T, double, 8, true, SHORT>(P.G, n, plo, phi, n, xl, L.r, nullptr);
        else gemv_rows<T, double, 8, false, SHORT>(P.G, n, plo, phi, n, xl, L.r, nullptr);
        __syncthreads();
        // G^T W G with W_ii = the number of sides of row i in cone form (row
        // bounds: an equality or one-sided row counts once, a two-sided row twice)
        for (int i = plo + (int)threadIdx.x; i < phi; i += blockDim.x) {
            double r = L.r[i];
            if (P.rlo) {
                const RowSides sd = row_sides(P.rlo, P.rhi, i);
                r *= (sd.up ? 1.0 : 0.0) + (sd.dn ? 1.0 : 0.0);
            }
            vl[i - plo] = r;
        }
        __syncthreads();
        if (tm.size == 1) {
            gemvT_rows<T, double, false>(P.G, n, plo, phi, n, vl, w, nullptr, false, tl);
            __syncthreads();
            return true;
        }
        gemvT_rows<T, double, true>(P.G, n, plo, phi, n, vl, L.gtp + (long)tm.rank * n, nullptr, true, tl);
        if (tm.sync()) return false;
        const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
        constexpr int C = 4;
        for (int j0 = nlo + wid; j0 < nhi; j0 += C * nw) {
            const int nc = min(C, (nhi - 1 - j0) / nw + 1);
            double s[C];
            xsum_strided_cols<C>(L.gtp + j0, n, (long)nw, nc, lane, kWave, tm.size, s);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                if (c < nc) {
                    const double t = wave_sum(s[c]);
                    if (lane == 0) w[j0 + c * nw] = t;
                }
            }
        }
        __syncthreads();
        return true;
    }

    // Compressed-row Q, G: w = Q v, or w = G^T W (G v) gathered along the rows
    // of G^T (v staged in xl, or read in place when it does not fit).
    __device__ __forceinline__ void sp_rows(const long long* rp, const int* ci, const T* val, int lo, int hi, int lg,
                                            const double* v, double* out) const {
        if (!L.x_global) spmv_rows<T, double>(rp, ci, val, lo, hi, lg, [&](int j) { return xl[j]; }, out, nullptr);
        else if (tm.size > 1)
            spmv_rows<T, double>(rp, ci, val, lo, hi, lg, [&](int j) { return xload(v + j); }, out, nullptr);
        else spmv_rows<T, double>(rp, ci, val, lo, hi, lg, [&](int j) { return v[j]; }, out, nullptr);
    }
    __device__ __forceinline__ bool apply_sparse(const double* v, double* w) {
        if (!use_gtg) {
            sp_rows(P.Qrp, P.Qci, P.Qv, nlo, nhi, P.Qlg, v, w);
            __syncthreads();
            return true;
        }
        sp_rows(P.Grp, P.Gci, P.Gv, plo, phi, P.Glg, v, L.r);
        __syncthreads();
        auto weight = [&](int i) {
            double r = L.r[i];
            if (P.rlo) {
                const RowSides sd = row_sides(P.rlo, P.rhi, i);
                r *= (sd.up ? 1.0 : 0.0) + (sd.dn ? 1.0 : 0.0);
            }
            return r;
        };
        if (tm.size == 1) {
            for (int i = plo + (int)threadIdx.x; i < phi; i += blockDim.x) vl[i - plo] = weight(i);
            __syncthreads();
            spmvT_cols<T>(P.Trp, P.Tci, P.Tv, nlo, nhi, P.Tlg, [&](int k) { return vl[k - plo]; }, nullptr, w);
        } else {
            for (int i = plo + (int)threadIdx.x; i < phi; i += blockDim.x) xstore(L.rsh + i, weight(i));
            if (tm.sync()) return false;
            spmvT_cols<T>(P.Trp, P.Tci, P.Tv, nlo, nhi, P.Tlg, [&](int k) { return xload(L.rsh + k); }, nullptr, w);
        }
        __syncthreads();
        return true;
    }

    // Number of eigenvalues of the tridiagonal (a, b) below x (Sturm count).
    __device__ static int sturm(const double* a, const double* b, int m, double x) {
        int cnt = 0;
        double d = 1.0;
        for (int i = 0; i < m; ++i) {
            const double bb = i > 0 ? b[i] * b[i] : 0.0;
            d = (a[i] - x) - (i > 0 ? bb / d : 0.0);
            if (d == 0.0) d = -1e-300;
            if (d < 0.0) ++cnt;
        }
        return cnt;
    }

    // Residual of the Ritz pair at x (an extreme eigenvalue of the m x m
    // tridiagonal a, b[1..m-1]): |b_m s_m| + ||(T - x) s|| for s the unit
    // eigenvector of T, found by two steps of inverse iteration with the
    // shift x - d (below the smallest eigenvalue: T - shift I is positive
    // definite, so the tridiagonal elimination needs no pivoting) or x + d
    // (above the largest: negative definite).  A Ritz pair (x, V s) with
    // residual r has an eigenvalue of the operator in [x - r, x + r].
    __device__ static double ritz_residual(const double* a, const double* b, int m, double x, double shift,
                                           double* y, double* cp) {
        for (int i = 0; i < m; ++i) y[i] = 1.0;
        for (int it = 0; it < 2; ++it) {
            // (T - shift I) y_new = y: elimination in place (y holds the
            // modified right-hand side), then back substitution
            double den = a[0] - shift;
            cp[0] = m > 1 ? b[1] / den : 0.0;
            y[0] = y[0] / den;
            for (int i = 1; i < m; ++i) {
                den = (a[i] - shift) - b[i] * cp[i - 1];
                cp[i] = i + 1 < m ? b[i + 1] / den : 0.0;
                y[i] = (y[i] - b[i] * y[i - 1]) / den;
            }
            for (int i = m - 2; i >= 0; --i) y[i] -= cp[i] * y[i + 1];
            double nrm = 0.0;
            for (int i = 0; i < m; ++i) nrm += y[i] * y[i];
            nrm = sqrt(nrm);
            for (int i = 0; i < m; ++i) y[i] /= nrm;
        }
        double res2 = 0.0;
        for (int i = 0; i < m; ++i) {
            const double ti = (a[i] - x) * y[i] + (i > 0 ? b[i] * y[i - 1] : 0.0) + (i + 1 < m ? b[i + 1] * y[i + 1] : 0.0);
            res2 += ti * ti;
        }
        return fabs(b[m] * y[m - 1]) + sqrt(res2);
    }

    __device__ __forceinline__ void run() {
        const int n = P.n;
        double* a = L.ab;        // written by rank 0 only, read back by it
        double* b = L.ab + k;
        // v_1: deterministic start vector with no special structure
        for (int i = nlo + (int)threadIdx.x; i < nhi; i += blockDim.x)
            vput(L.V + i, 1.0 + 0.5 * sin(0.7 * i + 0.3) + 0.25 * cos(1.9 * i));
        __syncthreads();
        if (!dots(L.V, 1)) return;
        {
            const double s = 1.0 / sqrt(hl[0]);
            for (int i = nlo + (int)threadIdx.x; i < nhi; i += blockDim.x) vput(L.V + i, vget(L.V + i) * s);
        }
        double alpha0 = 0.0;
        int m = 0;
        for (int j = 0; j < k; ++j) {
            if (tm.size > 1 && tm.sync()) return;   // V[j] complete before it is staged
            if (!apply(L.V + (long)j * n, L.w)) return;
            // w <- w - V (V^T w), two classical Gram-Schmidt passes; the
            // coefficient of v_j accumulates alpha_j = <A v_j, v_j>
            double aj = 0.0;
            for (int pass = 0; pass < 2; ++pass) {
                if (!dots(L.w, j + 1)) return;
                aj += hl[j];
                for (int i = nlo + (int)threadIdx.x; i < nhi; i += blockDim.x) {
                    double s = L.w[i];
                    int q = 0;
                    for (; q + 8 <= j + 1; q += 8) {   // 8 basis entries in flight
                        double v[8];
#pragma unroll
                        for (int u = 0; u < 8; ++u) v[u] = vget(L.V + (long)(q + u) * n + i);
#pragma unroll
                        for (int u = 0; u < 8; ++u) s -= hl[q + u] * v[u];
                    }
                    for (; q <= j; ++q) s -= hl[q] * vget(L.V + (long)q * n + i);
                    L.w[i] = s;
                }
                __syncthreads();
            }
            if (j == 0) alpha0 = aj;
            if (!dots_self()) return;
            const double beta = sqrt(hl[0]);
            if (tm.rank == 0 && threadIdx.x == 0) {
                a[j] = aj;
                b[j + 1] = beta;
            }
            m = j + 1;
            if (!(beta > 1e-13 * fabs(alpha0) + 1e-300)) break;   // invariant subspace
            const double inv = 1.0 / beta;
            for (int i = nlo + (int)threadIdx.x; i < nhi; i += blockDim.x)
                vput(L.V + (long)(j + 1) * n + i, L.w[i] * inv);
        }
        if (tm.rank == 0 && threadIdx.x == 0) {
            // extreme eigenvalues of the m x m tridiagonal (a, b[1..m-1]) by bisection
            double lo = INFINITY, hi = -INFINITY;
            for (int i = 0; i < m; ++i) {
                const double r = (i > 0 ? fabs(b[i]) : 0.0) + (i + 1 < m ? fabs(b[i + 1]) : 0.0);
                lo = fmin(lo, a[i] - r);
                hi = fmax(hi, a[i] + r);
            }
            double x0 = lo, x1 = hi;
            for (int it = 0; it < 200; ++it) {
                const double mid = 0.5 * (x0 + x1);
                if (sturm(a, b, m, mid) >= 1) x1 = mid; else x0 = mid;
            }
            L.out[0] = 0.5 * (x0 + x1);
            x0 = lo;
            x1 = hi;
            for (int it = 0; it < 200; ++it) {
                const double mid = 0.5 * (x0 + x1);
                if (sturm(a, b, m, mid) >= m) x1 = mid; else x0 = mid;
            }
            L.out[1] = 0.5 * (x0 + x1);
            L.out[2] = m;
            // bounds from the Ritz residuals: lambda_min >= theta_min - r_min
            // (the eigenvalue within r of theta_min, the smallest one once the
            // start vector has a component along it; floored at a tenth of
            // theta_min), lambda_max <= theta_max + r_max
            const double d = 1e-10 * fmax(fabs(lo), fabs(hi)) + 1e-300;
            const double rlo = ritz_residual(a, b, m, L.out[0], L.out[0] - d, hl, tl);
            const double rhi = ritz_residual(a, b, m, L.out[1], L.out[1] + d, hl, tl);
            L.out[3] = rlo;
            L.out[0] = fmax(L.out[0] - rlo, 0.1 * L.out[0]);
            L.out[1] = L.out[1] + rhi;
        }
    }

    // hl[0] = ||w||^2 over the team.
    __device__ __forceinline__ bool dots_self() {
        const int n = P.n;
        (void)n;
        const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x >> 6;
        const int ncol = k + 2;
        double s = 0.0;
        for (int i = nlo + (int)threadIdx.x; i < nhi; i += blockDim.x) s += L.w[i] * L.w[i];
        double v[1] = {s};
        block_allreduce<1>(v, red);
        if (tm.size == 1) {
            if (threadIdx.x == 0) hl[0] = v[0];
            __syncthreads();
            return true;
        }
        if (threadIdx.x == 0) xstore(L.part + (long)tm.rank * ncol + k + 1, v[0]);
        if (tm.sync()) return false;
        if (wid == 0) {
            double t = xsum_strided(L.part + k + 1, ncol, lane, kWave, tm.size);
            t = wave_sum(t);
            if (lane == 0) hl[0] = t;
        }
        __syncthreads();
        if (tm.sync()) return false;
        return true;
    }
};

}  // namespace duq
