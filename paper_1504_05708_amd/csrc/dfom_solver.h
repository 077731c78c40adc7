// Device-side Algorithm DFOM (Sec. 3) with the inner Algorithm FOM
// (Sec. 2.1) on the (augmented) Lagrangian over the box, last / averaged
// primal output (Sec. 4) and the on-device outer test.
//
// One body serves three launch shapes:
//   * the cooperative grid (team = every workgroup; one large QP),
//   * one workgroup per QP (small QPs, batches),
// A team member ("rank") owns a contiguous share of the n variables (rows of
// Q) and of the p constraint rows (rows of G).  Elementwise work touches only
// owned entries; products read the full input vector staged in LDS; every
// reduction is done in a fixed order, so every member holds bitwise the same
// scalars and takes the same branch.
//
// Per inner step with rho = 0 the only product is Q x^{t+1}: the gradient at
// the extrapolated point follows by linearity, Q y = (1+beta) Q x^t - beta Q x^{t-1}
// (Sec. 5.1 counts one matrix-vector product per inner iteration).
#pragma once
#include "device_common.h"

namespace duq {

// ---------------------------------------------------------------------------
// Products
// ---------------------------------------------------------------------------

// out[r] = sum_j A[r, j] x[j] + add[r] for the rows [rlo, rhi), one wavefront
// per row, x staged in LDS.  Lanes stream the row with 16-byte non-temporal
// loads (the matrix is read once per product and must not evict the vectors
// from the caches; on this chip the streaming hint also raises the achieved
// HBM rate from ~6.2 to ~7.3 TB/s for this access pattern).
template <typename T, bool NT>
__device__ __forceinline__ typename Vec16<T>::type vload(const typename Vec16<T>::type* p) {
    if (NT) return __builtin_nontemporal_load(p);
    return *p;
}

template <typename T, bool NT>
__device__ __forceinline__ T sload(const T* p) {
    if (NT) return __builtin_nontemporal_load(p);
    return *p;
}

// NT: stream the matrix with non-temporal loads.  Used when the matrix is far
// larger than the caches and read once per product (one large QP on the whole
// grid); per-instance matrices that are re-read every inner step (one
// workgroup per QP) use ordinary loads so that they stay cached.
template <typename T, typename Acc, int U = 8, bool NT = true, bool SHORT = false>
__device__ __forceinline__ void gemv_rows(const T* A, long ld, int rlo, int rhi, int ncols,
                                          const double* xl, double* out, const double* add) {
    typedef typename Vec16<T>::type VT;
    constexpr int V = Vec16<T>::N;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    const bool vec = ((ld * (long)sizeof(T)) % 16 == 0) && ((((uintptr_t)A) & 15) == 0);
    if constexpr (SHORT) {
        // Short rows (at most two 16-byte vectors per lane; the caller
        // guarantees ncols <= 2*64*V): R rows in flight per wavefront.  Every
        // row is summed in exactly the order of the long-row path below, so
        // the choice of path never changes a result.
        constexpr int R = 8;
        const int nv = ncols / V;
        for (int r0 = rlo + wid * R; r0 < rhi; r0 += nw * R) {
            Acc s[R];
#pragma unroll
            for (int q = 0; q < R; ++q) s[q] = 0;
#pragma unroll
            for (int kk = 0; kk < 2; ++kk) {
                const int v = lane + kk * kWave;
                if (v < nv) {
                    const double* xv = xl + (long)v * V;
                    // element loads whatever the alignment: in the batch
                    // kernels they measured faster than 16-byte loads (the
                    // eight rows' quads constrain register allocation), and
                    // the same entries are summed in the same order
                    VT a[R];
#pragma unroll
                    for (int q = 0; q < R; ++q) {
                        if (r0 + q < rhi) {
                            const T* row = A + (long)(r0 + q) * ld;
#pragma unroll
                            for (int e = 0; e < V; ++e) a[q][e] = row[(long)v * V + e];
                        }
                    }
#pragma unroll
                    for (int q = 0; q < R; ++q) {
                        if (r0 + q < rhi) {
#pragma unroll
                            for (int e = 0; e < V; ++e) s[q] += (Acc)a[q][e] * (Acc)xv[e];
                        }
                    }
                }
            }
            for (int j = nv * V + lane; j < ncols; j += kWave) {
#pragma unroll
                for (int q = 0; q < R; ++q)
                    if (r0 + q < rhi) s[q] += (Acc)A[(long)(r0 + q) * ld + j] * (Acc)xl[j];
            }
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const Acc t = wave_sum(s[q]);
                if (lane == 0 && r0 + q < rhi) out[r0 + q] = (double)t + (add ? add[r0 + q] : 0.0);
            }
        }
        return;
    } else {
    for (int r = rlo + wid; r < rhi; r += nw) {
        const T* row = A + (long)r * ld;
        Acc s = 0;
        int j0 = 0;
        if (vec) {
            const VT* rv = reinterpret_cast<const VT*>(row);
            const int nv = ncols / V;
            int v = lane;
            for (; v + kWave * (U - 1) < nv; v += kWave * U) {
                VT a[U];
#pragma unroll
                for (int u = 0; u < U; ++u) a[u] = vload<T, NT>(rv + v + kWave * u);
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const double* xv = xl + (long)(v + kWave * u) * V;
#pragma unroll
                    for (int e = 0; e < V; ++e) s += (Acc)a[u][e] * (Acc)xv[e];
                }
            }
            for (; v < nv; v += kWave) {
                VT a = vload<T, NT>(rv + v);
                const double* xv = xl + (long)v * V;
#pragma unroll
                for (int e = 0; e < V; ++e) s += (Acc)a[e] * (Acc)xv[e];
            }
            j0 = nv * V;
        } else {
            // rows not 16-byte aligned: element loads, but each lane accumulates
            // the same elements in the same order as the vector path, so the
            // result does not depend on where the matrix sits in memory
            const int nv = ncols / V;
            for (int v = lane; v < nv; v += kWave) {
                const T* pv = row + (long)v * V;
                const double* xv = xl + (long)v * V;
#pragma unroll
                for (int e = 0; e < V; ++e) s += (Acc)pv[e] * (Acc)xv[e];
            }
            j0 = nv * V;
        }
        for (int j = j0 + lane; j < ncols; j += kWave) s += (Acc)row[j] * (Acc)xl[j];
        s = wave_sum(s);
        if (lane == 0) out[r] = (double)s + (add ? add[r] : 0.0);
    }
    }
}

// Phase 1 of z = A^T v over the rows [rlo, rhi) of A: dst[j] = sum_r A[r,j] v[r]
// (+ add[j] when add != null).  Threads run over columns; rows with v[r] = 0
// are skipped (exactly: they add +0).  vl holds v[rlo..rhi) in LDS.
// Returns the number of rows with v != 0.
template <typename T, typename Acc, bool NT = true>
__device__ __forceinline__ int gemvT_rows(const T* A, long ld, int rlo, int rhi, int ncols,
                                          const double* vl, double* dst, const double* add, bool shared_dst,
                                          double* tl = nullptr) {
    typedef typename Vec16<T>::type VT;
    constexpr int V = Vec16<T>::N;
    const bool vec = ((ld * (long)sizeof(T)) % 16 == 0) && ((((uintptr_t)A) & 15) == 0);
    {
        // Short rows: split the rows over G thread groups.  Unit u is a
        // 16-byte column vector (u < nvec) or one tail column; group g sums rows
        // rlo+g, rlo+g+G, ... in order, and the G partials of a column are added
        // in group order.  The order depends only on the shape, not on the
        // alignment of A.  tl: LDS scratch of blockDim*V doubles.
        const int nvec = ncols / V;
        const int nunit = nvec + (ncols - nvec * V);
        const int G = nunit > 0 ? (int)blockDim.x / nunit : 1;
        if (tl != nullptr && G > 1) {
            const int t = threadIdx.x;
            const int u = t % nunit, grp = t / nunit;
            if (grp < G) {
                const bool isvec = u < nvec;
                const int c0 = isvec ? u * V : nvec * V + (u - nvec);
                Acc acc[V];
#pragma unroll
                for (int e = 0; e < V; ++e) acc[e] = 0;
                for (int r = rlo + grp; r < rhi; r += G) {
                    const double vr = vl[r - rlo];
                    if (vr == 0.0) continue;
                    const T* row = A + (long)r * ld;
                    if (isvec) {
                        VT a;
                        if (vec) a = vload<T, NT>(reinterpret_cast<const VT*>(row) + u);
                        else {
#pragma unroll
                            for (int e = 0; e < V; ++e) a[e] = row[c0 + e];
                        }
#pragma unroll
                        for (int e = 0; e < V; ++e) acc[e] += (Acc)a[e] * (Acc)vr;
                    } else {
                        acc[0] += (Acc)row[c0] * (Acc)vr;
                    }
                }
                const int ne = isvec ? V : 1;
                for (int e = 0; e < ne; ++e) tl[(long)grp * ncols + c0 + e] = (double)acc[e];
            }
            __syncthreads();
            for (int j = threadIdx.x; j < ncols; j += blockDim.x) {
                double sum = 0.0;
                for (int g2 = 0; g2 < G; ++g2) sum += tl[(long)g2 * ncols + j];
                const double val = sum + (add ? add[j] : 0.0);
                if (shared_dst) xstore(dst + j, val); else dst[j] = val;
            }
            __syncthreads();
            int nz = 0;
            for (int r = rlo; r < rhi; ++r) nz += (vl[r - rlo] != 0.0);
            return nz;
        }
    }
    // Long rows: threads over 16-byte column vectors; thread t owns the vectors
    // t + k * blockDim.x.  On a grid team (streamed, NT) a thread takes KC of
    // them (16 columns) per pass, two rows per trip, so 2 KC loads are in
    // flight instead of 2.  Every column is summed over the rows in ascending
    // order, skipping zero weights, whatever KC is.
    constexpr int KC = NT ? 16 / V : 1;
    const int nv = vec ? ncols / V : 0;
    const int bd = blockDim.x;
    for (int c0 = threadIdx.x; c0 < nv; c0 += KC * bd) {
        // opaque copy: keeps the KC column offsets from being hoisted out of
        // the solver's loops (they would stay live and spill)
        int cb = c0;
        asm volatile("" : "+v"(cb));
        const bool full = cb + (KC - 1) * bd < nv;
        Acc acc[KC][V];
#pragma unroll
        for (int k = 0; k < KC; ++k)
#pragma unroll
            for (int e = 0; e < V; ++e) acc[k][e] = 0;
        auto rows = [&](int r, int nr) {   // rows r .. r + nr - 1 (nr = 1 or 2)
            VT a[2][KC];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                if (q < nr && vl[r + q - rlo] != 0.0) {
                    const VT* row = reinterpret_cast<const VT*>(A + (long)(r + q) * ld) + cb;
#pragma unroll
                    for (int k = 0; k < KC; ++k)
                        if (full || cb + k * bd < nv) a[q][k] = vload<T, NT>(row + k * bd);
                }
            }
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const double vq = q < nr ? vl[r + q - rlo] : 0.0;
                if (q < nr && vq != 0.0) {
#pragma unroll
                    for (int k = 0; k < KC; ++k)
                        if (full || cb + k * bd < nv) {
#pragma unroll
                            for (int e = 0; e < V; ++e) acc[k][e] += (Acc)a[q][k][e] * (Acc)vq;
                        }
                }
            }
        };
        int r = rlo;
        for (; r + 1 < rhi; r += 2) rows(r, 2);
        if (r < rhi) rows(r, 1);
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            const int cv = cb + k * bd;
            if (cv < nv) {
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    const int j = cv * V + e;
                    const double val = (double)acc[k][e] + (add ? add[j] : 0.0);
                    if (shared_dst) xstore(dst + j, val); else dst[j] = val;
                }
            }
        }
    }
    for (int j = nv * V + threadIdx.x; j < ncols; j += blockDim.x) {
        Acc acc = 0;
        for (int r = rlo; r < rhi; ++r) {
            const double v0 = vl[r - rlo];
            if (v0 != 0.0) acc += (Acc)A[(long)r * ld + j] * (Acc)v0;
        }
        const double val = (double)acc + (add ? add[j] : 0.0);
        if (shared_dst) xstore(dst + j, val); else dst[j] = val;
    }
    int nz = 0;
    for (int r = rlo; r < rhi; ++r) nz += (vl[r - rlo] != 0.0);
    return nz;
}

// Phase 2: out[j] = add[j] + sum_{b < nb} part[b*n + j] for owned columns,
// one wavefront per column, lanes over b in a fixed order.
__device__ __forceinline__ void gemvT_reduce(const double* part, int nb, int n, int clo, int chi,
                                             const double* add, double* out) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    for (int j = clo + wid; j < chi; j += nw) {
        double s = 0.0;
        for (int b = lane; b < nb; b += kWave) s += xload(part + (long)b * n + j);
        s = wave_sum(s);
        if (lane == 0) out[j] = add[j] + s;
    }
}

// Sparse rows (Sec. 5.1: with sparse Q and G the products cost their
// nonzeros): out[r] = sum_k val[k] x[col[k]] + add[r] for rows [rlo, rhi) of
// a compressed-row matrix, x read through `xa` (LDS, or device memory when x
// does not fit).  2^lg lanes per row (chosen per matrix from its mean row
// length so a lane takes about four nonzeros), 64 / 2^lg rows per wavefront
// per trip.  A lane takes its row's nonzeros at stride 2^lg, four loads in
// flight at a time, adding them in index order; the lanes of a row then
// reduce by a butterfly.  The sum order depends on the row and lg only.
template <typename T, typename Acc, typename X>
__device__ __forceinline__ void spmv_rows(const long long* rp, const int* ci, const T* val, int rlo, int rhi,
                                          int lg, X xa, double* out, const double* add) {
    const int L = 1 << lg;
    const int rpw = kWave >> lg;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    const int sub = lane >> lg, sl = lane & (L - 1);
    for (int r0 = rlo + wid * rpw; r0 < rhi; r0 += nw * rpw) {
        const int r = r0 + sub;
        Acc s = 0;
        if (r < rhi) {
            const long long e = rp[r + 1];
            long long k = rp[r] + sl;
            for (; k + 3 * L < e; k += 4 * L) {
                const int c0 = ci[k], c1 = ci[k + L], c2 = ci[k + 2 * L], c3 = ci[k + 3 * L];
                const Acc v0 = (Acc)val[k], v1 = (Acc)val[k + L], v2 = (Acc)val[k + 2 * L], v3 = (Acc)val[k + 3 * L];
                const Acc x0 = (Acc)xa(c0), x1 = (Acc)xa(c1), x2 = (Acc)xa(c2), x3 = (Acc)xa(c3);
                s += v0 * x0;
                s += v1 * x1;
                s += v2 * x2;
                s += v3 * x3;
            }
            for (; k < e; k += L) s += (Acc)val[k] * (Acc)xa(ci[k]);
        }
        for (int off = L >> 1; off >= 1; off >>= 1) s += __shfl_xor(s, off, kWave);
        if (sl == 0 && r < rhi) out[r] = (double)s + (add ? add[r] : 0.0);
    }
}

// Sparse transposed product for the owned columns [clo, chi): z[j] = add[j] +
// sum over the nonzeros of row j of G^T (= column j of G) of val[k] w[col[k]],
// with the weights w read through `wt` (LDS or the team-visible buffer).
template <typename T, typename W>
__device__ __forceinline__ void spmvT_cols(const long long* rp, const int* ci, const T* val, int clo, int chi,
                                           int lg, W wt, const double* add, double* z) {
    spmv_rows<T, double>(rp, ci, val, clo, chi, lg, wt, z, add);
}

__device__ __forceinline__ void stage(const double* src, int len, double* dst) {
    for (int i = threadIdx.x; i < len; i += blockDim.x) dst[i] = src[i];
    __syncthreads();
}

// Staging of a vector written by other workgroups of the grid.  Each thread
// issues up to 8 loads before it waits, so the copy costs a couple of round
// trips to memory rather than one per element.
__device__ __forceinline__ void stage_shared(const double* src, int len, double* dst) {
    constexpr int B = 8;
    const int step = blockDim.x;
    int i = threadIdx.x;
    for (; i + (B - 1) * step < len; i += B * step) {
        double v[B];
#pragma unroll
        for (int u = 0; u < B; ++u) v[u] = xload(src + i + u * step);
#pragma unroll
        for (int u = 0; u < B; ++u) dst[i + u * step] = v[u];
    }
    for (; i + 3 * step < len; i += 4 * step) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = xload(src + i + u * step);
#pragma unroll
        for (int u = 0; u < 4; ++u) dst[i + u * step] = v[u];
    }
    for (; i < len; i += step) dst[i] = xload(src + i);
    __syncthreads();
}

// ---------------------------------------------------------------------------
// The solver
// ---------------------------------------------------------------------------

// Rows of at most 2*64 16-byte vectors take the short-row product.
template <typename T>
__host__ __device__ constexpr bool short_rows(int n) { return n <= 2 * kWave * (int)(16 / sizeof(T)); }

// A row of the user form rlo <= G_i u + g_i <= rhi (Sec. 2) in the cone form
// G u + g in K: an equality G_i u + g_i - rhi = 0 (K_i = {0}, free
// multiplier) when rlo = rhi; otherwise an upper side G_i u + g_i - rhi <= 0
// when rhi is finite and a lower side rlo - G_i u - g_i <= 0 when rlo is
// finite (K_i = R_-, one multiplier each: lambda+ and lambda-).
struct RowSides {
    double lo, hi;
    bool up, dn, eq;
};
__device__ __forceinline__ RowSides row_sides(const double* rlo, const double* rhi, int i) {
    RowSides s;
    s.lo = rlo[i];
    s.hi = rhi[i];
    s.eq = s.lo == s.hi;
    s.up = s.hi < INFINITY;
    s.dn = !s.eq && s.lo > -INFINITY;
    return s;
}

template <typename T, typename Acc, bool SHORT, bool ROWS = false, bool SPARSE = false>
struct Dfom {
    DevProblem<T> P;
    DevParams par;
    DevWork W;
    Team tm;
    int nlo, nhi, plo, phi;  // owned variable / row ranges
    double* xl;              // LDS: staged n-vector
    const double* xsrc;      // sparse data with x read in place (par.x_global)
    double* vl;              // LDS: staged owned rows of a p-vector
    double* red;             // LDS: reduction scratch
    double* tl;              // LDS: blockDim*4 doubles for short-row G^T v
    int pp;                  // ping-pong index of the partial buffer
    long long gt_rows;       // rows of G touched by transposed products
    double glb;              // sigma-free certificate of the last inner answer (enters LB
                             // when par.lb_cert == 2)

    // Rotating buffers selected without runtime-indexed arrays (which would
    // force the pointer tables into scratch memory).
    double *xb0, *xb1, *xb2, *qb0, *qb1, *qb2, *gx0, *gx1, *gx2;

    // The rotating x buffers are read by every workgroup of a grid team:
    // device-scope accesses there, plain ones inside a single workgroup.
    __device__ __forceinline__ void put(double* p, double v) const {
        if (tm.size > 1) xstore(p, v); else *p = v;
    }
    __device__ __forceinline__ double get(const double* p) const { return tm.size > 1 ? xload(p) : *p; }
    __device__ __forceinline__ void stage_x(const double* src) {
        if constexpr (SPARSE) {
            if (par.x_global) {
                // read in place: device-scope loads on a grid team.  (Plain
                // loads after an agent-scope acquire, which would let the
                // gathers share the XCD's L2, measured slower: the acquire
                // invalidates L1 and L2 for every wave.)
                xsrc = src;
                __syncthreads();
                return;
            }
        }
        if (tm.size > 1) stage_shared(src, P.n, xl); else stage(src, P.n, xl);
    }
    // Compressed-row product over rows [lo, hi) with x from LDS or, when it
    // does not fit there, from the rotating buffer itself (device-scope loads
    // on a grid team: other workgroups wrote it).
    __device__ __forceinline__ void sp_rows(const long long* rp, const int* ci, const T* v, int lo, int hi, int lg,
                                            double* out, const double* add) const {
        if (!par.x_global) spmv_rows<T, Acc>(rp, ci, v, lo, hi, lg, [&](int j) { return xl[j]; }, out, add);
        else if (tm.size > 1)
            spmv_rows<T, Acc>(rp, ci, v, lo, hi, lg, [&](int j) { return xload(xsrc + j); }, out, add);
        else spmv_rows<T, Acc>(rp, ci, v, lo, hi, lg, [&](int j) { return xsrc[j]; }, out, add);
    }

    // Products over owned rows: streamed (non-temporal) on a grid team,
    // cached inside a single workgroup.
    __device__ __forceinline__ void prodQ(double* out) const {
        if constexpr (SPARSE) sp_rows(P.Qrp, P.Qci, P.Qv, nlo, nhi, P.Qlg, out, nullptr);
        else if (tm.size > 1) gemv_rows<T, Acc, 16, true, SHORT>(P.Q, P.n, nlo, nhi, P.n, xl, out, nullptr);
        else gemv_rows<T, Acc, 16, false, SHORT>(P.Q, P.n, nlo, nhi, P.n, xl, out, nullptr);
    }
    __device__ __forceinline__ void prodG(double* out, const double* add) const {
        if constexpr (SPARSE) sp_rows(P.Grp, P.Gci, P.Gv, plo, phi, P.Glg, out, add);
        else if (tm.size > 1) gemv_rows<T, Acc, 8, true, SHORT>(P.G, P.n, plo, phi, P.n, xl, out, add);
        else gemv_rows<T, Acc, 8, false, SHORT>(P.G, P.n, plo, phi, P.n, xl, out, add);
    }
    __device__ __forceinline__ void bind_rings() {
        xb0 = W.xb[0]; xb1 = W.xb[1]; xb2 = W.xb[2];
        qb0 = W.qb[0]; qb1 = W.qb[1]; qb2 = W.qb[2];
        gx0 = W.gx[0]; gx1 = W.gx[1]; gx2 = W.gx[2];
    }
    __device__ __forceinline__ static double* pick(int i, double* a, double* b, double* c) {
        double* r = c;
        if (i == 0) r = a;
        if (i == 1) r = b;
        return r;
    }
    __device__ __forceinline__ double* X(int i) const { return pick(i, xb0, xb1, xb2); }
    __device__ __forceinline__ double* QX(int i) const { return pick(i, qb0, qb1, qb2); }
    __device__ __forceinline__ double* GX(int i) const { return pick(i, gx0, gx1, gx2); }

    // ---- team reductions -------------------------------------------------
    // Reduce K per-thread values over the team; every thread gets the sums.
    // Contains a team barrier; returns false on abort.
    template <int K>
    __device__ __forceinline__ bool allreduce(double (&v)[K]) {
        block_allreduce<K>(v, red);
        if (tm.size == 1) return true;
        double* part = W.part + (long)pp * tm.size * kNP;
        if (threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < K; ++k) xstore(part + (long)tm.rank * kNP + k, v[k]);
        }
        if (tm.sync()) return false;
        double s[K];
#pragma unroll
        for (int k = 0; k < K; ++k) s[k] = 0.0;
        for (int b = threadIdx.x; b < tm.size; b += blockDim.x) {
#pragma unroll
            for (int k = 0; k < K; ++k) s[k] += xload(part + (long)b * kNP + k);
        }
        block_allreduce<K>(s, red);
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = s[k];
        pp ^= 1;
        return true;
    }

    // z = add + A^T v restricted to owned columns (full v on the team).
    __device__ __forceinline__ bool gemvT(const double* v, const double* add, double* z) {
        return gemvT_w([&](int i) { return v[i]; }, add, z);
    }
    // z = add + A^T w with w_i = wt(i) for the owned rows.
    template <typename F>
    __device__ __forceinline__ bool gemvT_w(F wt, const double* add, double* z) {
        const int n = P.n;
        if constexpr (SPARSE) {
            // sparse: gather along the rows of G^T; the weights of every row are
            // needed, so they are published (LDS inside one workgroup, the
            // team-visible buffer on a grid team)
            if (tm.size == 1) {
                for (int i = plo + (int)threadIdx.x; i < phi; i += blockDim.x) vl[i - plo] = wt(i);
                __syncthreads();
                spmvT_cols<T>(P.Trp, P.Tci, P.Tv, nlo, nhi, P.Tlg, [&](int k) { return vl[k - plo]; }, add, z);
            } else {
                for (int i = plo + (int)threadIdx.x; i < phi; i += blockDim.x) xstore(W.wsh + i, wt(i));
                if (tm.sync()) return false;
                spmvT_cols<T>(P.Trp, P.Tci, P.Tv, nlo, nhi, P.Tlg, [&](int k) { return xload(W.wsh + k); }, add, z);
            }
            __syncthreads();
            return true;
        } else {
            for (int i = plo + (int)threadIdx.x; i < phi; i += blockDim.x) vl[i - plo] = wt(i);
            __syncthreads();
            if (tm.size == 1) {
                gt_rows += gemvT_rows<T, Acc, false>(P.G, n, plo, phi, n, vl, z, add, false, tl);
                __syncthreads();
                return true;
            }
            gt_rows +=
                gemvT_rows<T, Acc, true>(P.G, n, plo, phi, n, vl, W.gtp + (long)tm.rank * n, nullptr, true, tl);
            if (tm.sync()) return false;
            gemvT_reduce(W.gtp, tm.size, n, nlo, nhi, add, z);
            __syncthreads();
            return true;
        }
    }

    __device__ __forceinline__ double clip(double v, int i) const {
        return fmin(fmax(v, P.lb[i]), P.ub[i]);
    }

    // Exact-gradient certificate terms at a box point (fw, pi^2).
    __device__ __forceinline__ void cert_terms(double x, double gr, int i, double& fw, double& pi2) const {
        const double lo = P.lb[i], hi = P.ub[i];
        fw += fmax(gr * (x - lo), gr * (x - hi));
        const bool atl = x <= lo, atu = x >= hi;
        double pi = gr;
        if (atl && atu) pi = 0.0;
        else if (atl) pi = fmin(gr, 0.0);
        else if (atu) pi = fmax(gr, 0.0);
        pi2 += pi * pi;
    }

    __device__ __forceinline__ double gap_from(double fw, double pi2) const {
        return par.sigma > 0.0 ? fmin(fw, pi2 / (2.0 * par.sigma)) : fw;
    }

    __device__ __forceinline__ int third(int a, int b) const {
        int c = (a + 1) % 3;
        if (c == b) c = (a + 2) % 3;
        return c;
    }

    // ---- inner solve, rho = 0 --------------------------------------------
    // From x^0 = xb[cur] (with Q x^0 in qb[cur]) and c = q + G^T mu.
    // On return xb[cur] / qb[cur] hold ubar and Q ubar.  Returns -1 on abort.
    __device__ __forceinline__ int inner_rho0(int& cur, const double* c, double& gap) {
        const int n = P.n;
        int prv = cur;
        int t = 0;
        double th = 1.0;
        for (;;) {
            const int nxt = third(cur, prv);
            double beta = 0.0;
            if (t > 0) {
                if (par.inner_variant == 3) beta = par.beta_in;
                else if (par.inner_variant == 2) {
                    const double thn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * th * th));
                    beta = (th - 1.0) / thn;
                }
            }
            const double* x = X(cur);
            const double* xp = X(prv);
            const double* qx = QX(cur);
            const double* qxp = QX(prv);
            double* xn = X(nxt);
            double acc[2] = {0.0, 0.0};
            for (int i = nlo + (int)threadIdx.x; i < nhi; i += blockDim.x) {
                const double xi = get(x + i), qi = qx[i], ci = c[i];
                cert_terms(xi, qi + ci, i, acc[0], acc[1]);
                const double yi = xi + beta * (xi - get(xp + i));
                const double qyi = qi + beta * (qi - qxp[i]);
                put(xn + i, clip(yi - (qyi + ci) / par.L, i));
            }
            if (!allreduce<2>(acc)) return -1;
            gap = gap_from(acc[0], acc[1]);
            glb = acc[0];
            if (!(gap == gap)) return -2;
            if ((par.inner_rule == 0 && gap <= par.eps_in) || t >= par.k_in_max) return t;
            if (t > 0 && par.inner_variant == 2) th = 0.5 * (1.0 + sqrt(1.0 + 4.0 * th * th));
            // Q x^{t+1}; the barrier inside allreduce published every x^{t+1} entry
            stage_x(xn);
            prodQ(QX(nxt));
            __syncthreads();
            prv = cur;
            cur = nxt;
            ++t;
        }
    }

    // ---- inner solve, rho > 0 --------------------------------------------
    // Gradient Q y + q + G^T [mu + rho (G y + g)]_+ at the extrapolated point
    // only; G y and Q y follow by linearity from G x, Q x.  Certificate: exact
    // at x^0, gradient-mapping bound after each projected step.
    __device__ __forceinline__ int inner_rhop(int& cur, const double* mu, const double* mum, double& gap) {
        const int n = P.n;
        int prv = cur;
        int t = 0;
        double th = 1.0, beta = 0.0;
        for (;;) {
            const int nxt = third(cur, prv);
            const double* x = X(cur);
            const double* xp = X(prv);
            // w = [mu + rho (G y + g)]_+ on owned rows, G y by linearity; with
            // row bounds w = mu + rho (G y + g - s) per side (s the projection
            // onto K_i), the lower side entering with a minus sign
            for (int i = plo + (int)threadIdx.x; i < phi; i += blockDim.x) {
                const double gxi = GX(cur)[i];
                const double gyi = gxi + beta * (gxi - GX(prv)[i]);
                if constexpr (ROWS) {
                    const RowSides sd = row_sides(P.rlo, P.rhi, i);
                    const double ry = gyi + P.g[i];
                    double w = 0.0;
                    if (sd.up) {
                        const double v = mu[i] + par.rho * (ry - sd.hi);
                        w += sd.eq ? v : fmax(v, 0.0);
                    }
                    if (sd.dn) w -= fmax(mum[i] + par.rho * (sd.lo - ry), 0.0);
                    W.wv[i] = w;
                } else {
                    W.wv[i] = fmax(mu[i] + par.rho * (gyi + P.g[i]), 0.0);
                }
            }
            __syncthreads();
            // h = q + G^T w into W.c (owned columns)
            if (!gemvT(W.wv, P.q, W.c)) return -1;
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            double* xn = X(nxt);
            for (int i = nlo + (int)threadIdx.x; i < nhi; i += blockDim.x) {
                const double xi = get(x + i), qi = QX(cur)[i];
                const double yi = xi + beta * (xi - get(xp + i));
                const double qyi = qi + beta * (qi - QX(prv)[i]);
                const double gy = qyi + W.c[i];
                if (t == 0) cert_terms(xi, gy, i, acc[0], acc[1]);
                const double xnew = clip(yi - gy / par.L, i);
                put(xn + i, xnew);
                const double gm = par.L * (yi - xnew);
                acc[2] += fmax(gm * (yi - P.lb[i]), gm * (yi - P.ub[i]));
                acc[3] += gm * gm;
            }
            if (!allreduce<4>(acc)) return -1;
            if (t == 0) {
                gap = gap_from(acc[0], acc[1]);
                glb = acc[0];
                if (!(gap == gap)) return -2;
                if (par.inner_rule == 0 && gap <= par.eps_in) return 0;
            }
            double g2 = acc[2] - acc[3] / (2.0 * par.L);
            glb = g2;
            if (par.sigma > 0.0) g2 = fmin(g2, 0.5 * acc[3] * (1.0 / par.sigma - 1.0 / par.L));
            gap = g2;
            if (!(gap == gap)) return -2;
            // products of x^{t+1} (published by the barrier inside allreduce)
            stage_x(xn);
            prodQ(QX(nxt));
            prodG(GX(nxt), nullptr);
            __syncthreads();
            ++t;
            prv = cur;
            cur = nxt;
            if ((par.inner_rule == 0 && gap <= par.eps_in) || t >= par.k_in_max) return t;
            // momentum for y^{t+1}
            if (par.inner_variant == 3) beta = par.beta_in;
            else if (par.inner_variant == 2) {
                const double thn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * th * th));
                beta = (th - 1.0) / thn;
                th = thn;
            } else beta = 0.0;
        }
    }

    // Inner solve at mu.  farkas (rho = 0): first test mu as a certificate of
    // infeasibility and return -3 if it is one.  The method assumes a finite
    // optimal multiplier exists (Sec. 2); a mu >= 0 with
    //   v = min over the box of mu^T (G u + g) = mu^T g + sum_j min(lb_j w_j, ub_j w_j),
    // w = G^T mu = c - q, above kInfeasMargin times the sum of the magnitudes
    // of its terms proves that no u in the box has G u + g <= 0.  The test
    // takes one team reduction; it runs at every kInfeasEvery-th outer
    // iteration, outside the inner loop.
    __device__ __forceinline__ int inner(int& cur, const double* mu, const double* mum, double& gap, bool farkas) {
        if (par.rho > 0.0 && !par.eqform) return inner_rhop(cur, mu, mum, gap);
        if constexpr (ROWS) {
            // c = q + G^T (lambda+ - lambda-); in the equality form (all rows
            // equalities, Q + rho G^T G held in Q) c = q + G^T (mu + rho (g - rhi))
            // (Sec. 5.1: the constant part rho G^T g folded into the weights)
            if (par.eqform) {
                if (!gemvT_w([&](int i) { return mu[i] + par.rho * (P.g[i] - P.rhi[i]); }, P.q, W.c)) return -1;
            } else {
                if (!gemvT_w([&](int i) { return mu[i] - mum[i]; }, P.q, W.c)) return -1;
            }
        } else {
            if (!gemvT(mu, P.q, W.c)) return -1;   // c = q + G^T mu (Sec. 5.1)
        }
        if (farkas && P.p > 0 && par.rho == 0.0) {
            double e[3] = {0.0, 0.0, 0.0};   // v, scale, #(mu < 0)
            for (int i = nlo + (int)threadIdx.x; i < nhi; i += blockDim.x) {
                const double w = W.c[i] - P.q[i], lo = P.lb[i], hi = P.ub[i];
                e[0] += fmin(lo * w, hi * w);
                e[1] += fabs(w) * fmax(fabs(lo), fabs(hi));
            }
            for (int i = plo + (int)threadIdx.x; i < phi; i += blockDim.x) {
                if constexpr (ROWS) {
                    // mu^T (G u + g - shifts) over the sides; equality multipliers
                    // may take either sign
                    const RowSides sd = row_sides(P.rlo, P.rhi, i);
                    if (sd.up) {
                        const double m = mu[i], mg = m * (P.g[i] - sd.hi);
                        e[0] += mg;
                        e[1] += fabs(mg);
                        e[2] += (!sd.eq && m < 0.0) ? 1.0 : 0.0;
                    }
                    if (sd.dn) {
                        const double m = mum[i], mg = m * (sd.lo - P.g[i]);
                        e[0] += mg;
                        e[1] += fabs(mg);
                        e[2] += m < 0.0 ? 1.0 : 0.0;
                    }
                } else {
                    const double m = mu[i], mg = m * P.g[i];
                    e[0] += mg;
                    e[1] += fabs(mg);
                    e[2] += m < 0.0 ? 1.0 : 0.0;
                }
            }
            if (!allreduce<3>(e)) return -1;
            if (e[2] == 0.0 && e[0] > kInfeasMargin * e[1]) return -3;
        }
        return inner_rho0(cur, W.c, gap);
    }

    // After an inner solve ending in xb[cur]: r = G u + g on owned rows (for
    // rho > 0 G u is already in gx[cur]).
    __device__ __forceinline__ void residual(int cur) {
        if (par.rho > 0.0 && !par.eqform) {
            for (int i = plo + (int)threadIdx.x; i < phi; i += blockDim.x) W.r[i] = GX(cur)[i] + P.g[i];
            __syncthreads();
            return;
        }
        stage_x(X(cur));
        prodG(W.r, P.g);
        __syncthreads();
    }

    __device__ __forceinline__ bool outer_ok(double F, double feas, double lnorm, double LB, double gnorm) const {
        const double sc = fmax(1.0, fabs(F));
        return feas <= par.eps_out * fmax(1.0, gnorm) && F - LB <= par.eps_out * sc &&
               lnorm * feas <= par.eps_out * sc;
    }

    // Copy owned entries of the primal answer and multipliers to the outputs.
    __device__ __forceinline__ void write_outputs(const double* x, double scale, bool shared) {
        for (int i = nlo + (int)threadIdx.x; i < nhi; i += blockDim.x)
            W.xout[i] = (shared ? get(x + i) : x[i]) * scale;
    }

    // ---- dual step with row bounds (Algorithm DFOM steps 2-3) ---------------
    // The rows of the user form, each side an inequality of K = R_- or the row
    // an equality of K = {0}, updated on owned rows: the partial sums of the
    // outer test (same slots as the one-sided form) and lambda, mu of each side.
    // Equality form: the rho ||G u||^2 parts of u^T (Q + rho G^T G) u are taken
    // off a[0] (last iterate) and a[8] (theta-weighted sum, scaled by S^2).
    __device__ __forceinline__ void dual_rows(double (&a)[11], double thk, double beta, double Sn, double* trec) {
        const int n = P.n, p = P.p;
        const double rho = par.rho;
        for (int i = plo + (int)threadIdx.x; i < phi; i += blockDim.x) {
            const RowSides sd = row_sides(P.rlo, P.rhi, i);
            const double ri = W.r[i];
            const double rs = W.rs[i] + thk * ri;
            W.rs[i] = rs;
            const double ravg = rs / Sn;
            auto side = [&](double e, double ea, double* mu, double* lam, bool eq, double* tlam, double* tmu) {
                const double mui = mu[i];
                double dg;
                if (rho > 0.0) {
                    const double v = e + mui / rho;
                    const double vk = eq ? v : fmax(v, 0.0);
                    a[2] += vk * vk;
                    a[3] += mui * mui;
                    dg = eq ? e : e - fmin(v, 0.0);
                } else {
                    a[2] += mui * e;
                    dg = e;
                }
                const double ep = eq ? e : fmax(e, 0.0);
                a[4] += ep * ep;
                double lk = mui + par.alpha * dg;
                if (par.Kd_nonneg && !eq) lk = fmax(lk, 0.0);
                a[5] += lk * lk;
                const double hp = eq ? ea : fmax(ea, 0.0);
                a[6] += hp * hp;
                a[7] += (!eq && mui < 0.0) ? 1.0 : 0.0;
                a[10] += (!eq && lk < 0.0) ? 1.0 : 0.0;
                if (trec) {
                    tlam[i] = lk;
                    tmu[i] = mui;
                }
                mu[i] = lk + beta * (lk - lam[i]);
                lam[i] = lk;
            };
            double* t0 = trec ? trec + kTraceScalars : nullptr;
            double* t1 = trec ? trec + kTraceScalars + p : nullptr;
            double* t2 = trec ? trec + kTraceScalars + 2 * p + n : nullptr;
            double* t3 = trec ? trec + kTraceScalars + 3 * p + n : nullptr;
            if (sd.up) side(ri - sd.hi, ravg - sd.hi, W.mu, W.lamp, sd.eq, t0, t1);
            else if (trec) { t0[i] = 0.0; t1[i] = 0.0; }
            if (sd.dn) side(sd.lo - ri, sd.lo - ravg, W.mum, W.lamm, false, t2, t3);
            else if (trec) { t2[i] = 0.0; t3[i] = 0.0; }
            if (par.eqform) {
                const double gu = ri - P.g[i], ga = ravg - P.g[i];
                a[0] -= rho * gu * gu;
                a[8] -= rho * ga * ga * Sn * Sn;
            }
        }
    }

    // Partial sums of the last-iterate test at lambda^k with row bounds.
    __device__ __forceinline__ void extra_rows(double (&b)[6]) {
        const double rho = par.rho;
        for (int i = plo + (int)threadIdx.x; i < phi; i += blockDim.x) {
            const RowSides sd = row_sides(P.rlo, P.rhi, i);
            const double ri = W.r[i];
            auto side = [&](double e, double li, bool eq) {
                if (rho > 0.0) {
                    const double v = e + li / rho;
                    const double vk = eq ? v : fmax(v, 0.0);
                    b[2] += vk * vk;
                    b[3] += li * li;
                } else {
                    b[2] += li * e;
                }
                const double ep = eq ? e : fmax(e, 0.0);
                b[4] += ep * ep;
            };
            if (sd.up) side(ri - sd.hi, W.lamp[i], sd.eq);
            if (sd.dn) side(sd.lo - ri, W.lamm[i], false);
            if (par.eqform) {
                const double gu = ri - P.g[i];
                b[0] -= rho * gu * gu;
            }
        }
    }

    // ---- Algorithm DFOM ---------------------------------------------------
    __device__ __forceinline__ void run() {
        const int n = P.n, p = P.p;
        DevState* st = W.st;
        bind_rings();
        pp = 0;
        gt_rows = 0;
        int cur;
        double theta, S, LB, gnorm;
        int k0;
        long long inner_total;
        if (!par.resume) {
            cur = 0;
            // x^0 = warm start or the projection of 0; lambda^0 = lam0 or 0
            for (int i = nlo + (int)threadIdx.x; i < nhi; i += blockDim.x) {
                const double v = par.has_x0 ? W.x0[i] : 0.0;
                put(xb0 + i, clip(v, i));
                W.us[i] = 0.0;
                W.qus[i] = 0.0;
            }
            double gg[1] = {0.0};
            for (int i = plo + (int)threadIdx.x; i < phi; i += blockDim.x) {
                double l = par.has_lam0 ? W.lam0[i] : 0.0;
                if (par.Kd_nonneg) l = fmax(l, 0.0);
                W.lamp[i] = l;   // lambda^{-1} = lambda^0
                W.mu[i] = l;     // mu^1 = lambda^0
                W.rs[i] = 0.0;
                if constexpr (ROWS) {
                    // lambda^0 = 0 for both sides; ||g|| is the norm of the
                    // constant terms of the sides
                    W.lamm[i] = 0.0;
                    W.mum[i] = 0.0;
                    const RowSides sd = row_sides(P.rlo, P.rhi, i);
                    const double gu = sd.up ? P.g[i] - sd.hi : 0.0, gd = sd.dn ? sd.lo - P.g[i] : 0.0;
                    gg[0] += gu * gu + gd * gd;
                } else {
                    gg[0] += P.g[i] * P.g[i];
                }
            }
            if (!allreduce<1>(gg)) return;
            gnorm = sqrt(gg[0]);
            if (tm.size > 1 && tm.sync()) return;
            stage_x(xb0);
            prodQ(qb0);
            if (par.rho > 0.0 && !par.eqform) prodG(gx0, nullptr);
            __syncthreads();
            theta = 1.0;
            S = 0.0;
            LB = -INFINITY;
            k0 = 0;
            inner_total = 0;
        } else {
            cur = st->cur;
            theta = st->theta;
            S = st->S;
            LB = st->LB;
            gnorm = st->gnorm;
            k0 = st->k;
            inner_total = st->inner;
            gt_rows = 0;
            if (par.resume == 1) {
                // products of the warm start in this launch's accumulation precision
                stage_x(X(cur));
                prodQ(QX(cur));
                if (par.rho > 0.0 && !par.eqform) prodG(GX(cur), nullptr);
                __syncthreads();
            }   // resume == 2: the stored products are this precision's; keep them
        }
        double best = par.resume ? st->best_metric : INFINITY;
        int stall = par.resume ? st->stall : 0;
        int status = 1;  // max outer unless the test passes
        double Fc = 0.0, feasc = 0.0, lnc = 0.0;
        int ans_cur = cur;   // buffer of the answer (LAST)
        bool ans_avg = false;
        int k = k0;
        while (k < par.max_outer) {
            ++k;
            // Step 1: inner solve at mu^k, warm-started from ubar^{k-1}
            double gap = 0.0;
            const int t = inner(cur, W.mu, W.mum, gap, k % kInfeasEvery == 1);
            if (t == -1) return;
            if (t == -2) { status = 2; break; }
            if (t == -3) {
                // mu^k certifies infeasibility: it is returned as the multiplier,
                // the warm start ubar^{k-1} as the iterate
                for (int i = plo + (int)threadIdx.x; i < phi; i += blockDim.x) {
                    W.lamp[i] = W.mu[i];
                    if constexpr (ROWS) W.lamm[i] = W.mum[i];
                }
                __syncthreads();
                status = kStInfeasible;
                ans_cur = cur;
                ans_avg = false;
                break;
            }
            inner_total += t;
            residual(cur);
            // Steps 2-3 and averaging on owned rows / variables
            const double thk = theta;
            const double thn = par.method == 1 ? 0.5 * (1.0 + sqrt(1.0 + 4.0 * thk * thk)) : 1.0;
            const double beta = (thk - 1.0) / thn;
            const double Sn = S + thk;
            double a[11];
#pragma unroll
            for (int z = 0; z < 11; ++z) a[z] = 0.0;
            const bool tr = k <= par.trace_iters;
            const long rec = ROWS ? kTraceScalars + 4L * p + n : kTraceScalars + 2L * p + n;
            double* trec = tr ? W.trace + (long)(k - 1) * rec : nullptr;
            for (int i = nlo + (int)threadIdx.x; i < nhi; i += blockDim.x) {
                const double ui = get(X(cur) + i), qui = QX(cur)[i];
                a[0] += ui * qui;
                a[1] += P.q[i] * ui;
                const double us = W.us[i] + thk * ui, qus = W.qus[i] + thk * qui;
                W.us[i] = us;
                W.qus[i] = qus;
                a[8] += us * qus;
                a[9] += P.q[i] * us;
                if (tr) trec[kTraceScalars + 2 * p + i] = ui;
            }
            if constexpr (ROWS) dual_rows(a, thk, beta, Sn, trec);
            else
            for (int i = plo + (int)threadIdx.x; i < phi; i += blockDim.x) {
                const double ri = W.r[i], mui = W.mu[i];
                double dg;
                if (par.rho > 0.0) {
                    const double v = fmax(ri + mui / par.rho, 0.0);
                    a[2] += v * v;
                    a[3] += mui * mui;
                    dg = ri - fmin(ri + mui / par.rho, 0.0);
                } else {
                    a[2] += mui * ri;
                    dg = ri;
                }
                const double rp = fmax(ri, 0.0);
                a[4] += rp * rp;
                double lk = mui + par.alpha * dg;
                if (par.Kd_nonneg) lk = fmax(lk, 0.0);
                a[5] += lk * lk;
                const double rs = W.rs[i] + thk * ri;
                W.rs[i] = rs;
                const double hp = fmax(rs / Sn, 0.0);
                a[6] += hp * hp;
                a[7] += (mui < 0.0) ? 1.0 : 0.0;
                a[10] += (lk < 0.0) ? 1.0 : 0.0;
                if (tr) {
                    trec[kTraceScalars + i] = lk;
                    trec[kTraceScalars + p + i] = mui;
                }
                W.mu[i] = lk + beta * (lk - W.lamp[i]);
                W.lamp[i] = lk;
            }
            if (!allreduce<11>(a)) return;
            // equality form: a[0] and a[8] hold u^T (Q + rho G^T G) u terms with
            // the rho ||G u||^2 parts already taken off (dual_rows)
            const double Fu = 0.5 * a[0] + a[1];
            const double dbar = par.rho > 0.0 ? Fu + 0.5 * par.rho * a[2] - a[3] / (2.0 * par.rho)
                                              : Fu + a[2];
            if (par.rho > 0.0 || a[7] == 0.0) LB = fmax(LB, dbar - (par.lb_cert == 2 ? glb : gap));
            S = Sn;
            double F, feas;
            if (par.output == 0) {
                F = Fu;
                feas = sqrt(a[4]);
            } else {
                F = 0.5 * a[8] / (S * S) + a[9] / S;
                feas = sqrt(a[6]);
            }
            const double lnorm = sqrt(a[5]);
            if (!(F == F) || !(LB == LB && dbar == dbar)) { status = 2; break; }
            const bool ok1 = outer_ok(F, feas, lnorm, LB, gnorm);
            bool ok = ok1;
            Fc = F; feasc = feas; lnc = lnorm;
            ans_cur = cur;
            ans_avg = par.output == 1;
            double ex[5] = {0.0, 0.0, 0.0, 0.0, 0.0};   // extra_t, extra_gap, F2, feas2, passed2
            if (ok1 && par.output == 0 && par.method == 1 && !par.phase1) {
                // Last iterate of DFGM: ubar(lambda^k), eq. last_primal.
                for (int i = nlo + (int)threadIdx.x; i < nhi; i += blockDim.x) {
                    W.usave[i] = get(X(cur) + i);
                    W.qusave[i] = QX(cur)[i];
                }
                if (par.rho > 0.0)
                    for (int i = plo + (int)threadIdx.x; i < phi; i += blockDim.x) W.gsave[i] = GX(cur)[i];
                __syncthreads();
                int c2 = cur;
                double gap2 = 0.0;
                const int t2 = inner(c2, W.lamp, W.lamm, gap2, false);
                if (t2 == -1) return;
                if (t2 == -2) { status = 2; break; }
                inner_total += t2;
                residual(c2);
                double b[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                for (int i = nlo + (int)threadIdx.x; i < nhi; i += blockDim.x) {
                    const double ui = get(X(c2) + i);
                    b[0] += ui * QX(c2)[i];
                    b[1] += P.q[i] * ui;
                }
                if constexpr (ROWS) extra_rows(b);
                else
                for (int i = plo + (int)threadIdx.x; i < phi; i += blockDim.x) {
                    const double ri = W.r[i], li = W.lamp[i];
                    if (par.rho > 0.0) {
                        const double v = fmax(ri + li / par.rho, 0.0);
                        b[2] += v * v;
                        b[3] += li * li;
                    } else {
                        b[2] += li * ri;
                    }
                    const double rp = fmax(ri, 0.0);
                    b[4] += rp * rp;
                }
                if (!allreduce<6>(b)) return;
                const double F2 = 0.5 * b[0] + b[1];
                const double d2 = par.rho > 0.0 ? F2 + 0.5 * par.rho * b[2] - b[3] / (2.0 * par.rho)
                                                : F2 + b[2];
                if (par.rho > 0.0 || a[10] == 0.0) LB = fmax(LB, d2 - (par.lb_cert == 2 ? glb : gap2));
                const double feas2 = sqrt(b[4]);
                const bool ok2 = outer_ok(F2, feas2, lnorm, LB, gnorm);
                ex[0] = t2; ex[1] = gap2; ex[2] = F2; ex[3] = feas2; ex[4] = ok2 ? 1.0 : 0.0;
                if (ok2) {
                    Fc = F2; feasc = feas2;
                    ans_cur = c2;
                } else {
                    ok = false;
                    // continue from ubar^k unchanged
                    for (int i = nlo + (int)threadIdx.x; i < nhi; i += blockDim.x) {
                        put(X(cur) + i, W.usave[i]);
                        QX(cur)[i] = W.qusave[i];
                    }
                    if (par.rho > 0.0)
                        for (int i = plo + (int)threadIdx.x; i < phi; i += blockDim.x) GX(cur)[i] = W.gsave[i];
                    __syncthreads();
                }
            }
            if (tr && tm.rank == 0 && threadIdx.x == 0) {
                trec[0] = k; trec[1] = t; trec[2] = gap; trec[3] = dbar; trec[4] = LB;
                trec[5] = thk; trec[6] = S; trec[7] = F; trec[8] = feas; trec[9] = lnorm;
                trec[10] = ok1 ? 1.0 : 0.0;
                trec[11] = ex[0]; trec[12] = ex[1]; trec[13] = ex[2]; trec[14] = ex[3]; trec[15] = ex[4];
                st->n_trace = k;
            }
            theta = thn;
            if (ok) { status = 0; break; }
            if (par.phase1 && par.stall_iters > 0) {
                // progress measure of the outer test; the phase ends when it has not
                // improved by 1% for stall_iters iterations
                const double sc = fmax(1.0, fabs(F));
                const double m = fmax(fmax(feas / fmax(1.0, gnorm), (F - LB) / sc), lnorm * feas / sc);
                if (m < 0.99 * best) { best = m; stall = 0; }
                else if (++stall >= par.stall_iters) { status = 3; break; }
            }
        }
        // outputs
        if (ans_avg) write_outputs(W.us, 1.0 / S, false);
        else write_outputs(X(ans_cur), 1.0, true);
        if constexpr (ROWS) {
            // one multiplier per row: lambda+ - lambda- (an equality's own sign)
            for (int i = plo + (int)threadIdx.x; i < phi; i += blockDim.x) W.nu[i] = W.lamp[i] - W.lamm[i];
        }
        if (tm.rank == 0 && threadIdx.x == 0) {
            st->status = status;
            st->done = status == 0;
            st->k = k;
            st->cur = cur;
            st->inner = inner_total;
            st->theta = theta;
            st->S = S;
            st->LB = LB;
            st->F = Fc;
            st->feas = feasc;
            st->lnorm = lnc;
            st->gnorm = gnorm;
            st->best_metric = best;
            st->stall = stall;
        }
        // rows of G touched, summed over the team (for reporting)
        if (threadIdx.x == 0 && gt_rows > 0)
            atomicAdd((unsigned long long*)&st->gt_rows, (unsigned long long)gt_rows);
    }
};

}  // namespace duq
