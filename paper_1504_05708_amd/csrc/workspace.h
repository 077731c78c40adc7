// Host-side layout of the single-QP solver workspace (one device block),
// shared by the allocating setup and the allocation-free entry point.
#pragma once
#include <stddef.h>

#include <algorithm>

#include "internal.h"

namespace duq {

// Bump allocator over one device block (256-byte aligned slices).  With a
// null base it only measures: `off` is then the size the layout needs.
struct Carve {
    char* base = nullptr;
    size_t off = 0;
    template <typename T>
    T* take(size_t count) {
        const size_t bytes = ((count * sizeof(T) + 255) / 256) * 256 + 256;
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += bytes;
        return p;
    }
};

// Vectors, partial sums, barrier words and trace of one solve on `nb`
// workgroups (n variables, p rows, `trace` recorded outer iterations), plus
// two staging vectors for the warm start.  Compressed-row data (`sparse`)
// gathers G^T w along rows and needs no per-workgroup partial columns.
inline void carve_solver(Carve& c, int n, int p, int nb, int trace, DevWork* W, double** xstage,
                         double** lstage, bool sparse = false) {
    for (int i = 0; i < 3; ++i) W->xb[i] = c.take<double>(n);
    for (int i = 0; i < 3; ++i) W->qb[i] = c.take<double>(n);
    W->c = c.take<double>(n);
    W->us = c.take<double>(n);
    W->qus = c.take<double>(n);
    W->usave = c.take<double>(n);
    W->qusave = c.take<double>(n);
    W->xout = c.take<double>(n);
    const int pp = std::max(p, 1);
    W->r = c.take<double>(pp);
    W->rs = c.take<double>(pp);
    W->lamp = c.take<double>(pp);
    W->mu = c.take<double>(pp);
    W->wv = c.take<double>(pp);
    W->gsave = c.take<double>(pp);
    for (int i = 0; i < 3; ++i) W->gx[i] = c.take<double>(pp);
    W->lamm = c.take<double>(pp);
    W->mum = c.take<double>(pp);
    W->nu = c.take<double>(pp);
    W->wsh = c.take<double>(pp);
    W->part = c.take<double>((size_t)2 * nb * kNP);
    W->gtp = c.take<double>(nb > 1 && !sparse ? (size_t)nb * n : 1);
    // a record holds lambda+, mu+, ubar and, with row bounds, lambda-, mu-
    W->trace = c.take<double>(trace > 0 ? (size_t)trace * (kTraceScalars + 4 * p + n) : 1);
    W->st = c.take<DevState>(1);
    W->bar = c.take<unsigned>(bar_words(nb));
    *xstage = c.take<double>(n);
    *lstage = c.take<double>(pp);
}

}  // namespace duq
