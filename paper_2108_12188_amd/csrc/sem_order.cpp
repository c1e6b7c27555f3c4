// sem_order.cpp -- element orders that give the gather-scatter spatial
// locality on unstructured meshes.
//
// On an unstructured mesh the element numbering carries no spatial order, so
// the copies of a shared point may sit anywhere in the local vectors (the
// paper's Sec. 4.3 names these unaligned accesses as the cost of the
// gather-scatter; Sec. 8.2 proposes partitioning or sorting the elements to
// recover locality).  Sorting the elements along a space-filling curve
// through their centroids puts face, edge and vertex neighbours close in the
// element-major layout.  Host code only.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <vector>

#include "sem_internal.h"

namespace sem {
namespace {

constexpr int kBits = 21;   // per axis; 3 x 21 bits fit one 64-bit key

// Hilbert index of a point of the 2^kBits grid in 3-D, following J. Skilling,
// "Programming the Hilbert curve" (AIP Conf. Proc. 707, 2004): the axes are
// brought into the curve's "transposed" form (undo the inversions and
// exchanges level by level, then Gray-code), and the key interleaves the
// transposed axes bit by bit, most significant level first.
uint64_t hilbert_key(uint32_t x, uint32_t y, uint32_t z) {
    uint32_t X[3] = {x, y, z};
    const uint32_t top = 1u << (kBits - 1);
    for (uint32_t q = top; q > 1; q >>= 1) {
        const uint32_t low = q - 1;
        for (int i = 0; i < 3; ++i) {
            if (X[i] & q) {
                X[0] ^= low;                       // invert the lower bits of axis 0
            } else {
                const uint32_t t = (X[0] ^ X[i]) & low;   // exchange lower bits
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    for (int i = 1; i < 3; ++i) X[i] ^= X[i - 1];
    uint32_t t = 0;
    for (uint32_t q = top; q > 1; q >>= 1)
        if (X[2] & q) t ^= q - 1;
    for (int i = 0; i < 3; ++i) X[i] ^= t;
    uint64_t key = 0;
    for (int b = kBits - 1; b >= 0; --b)
        for (int i = 0; i < 3; ++i) key = (key << 1) | ((X[i] >> b) & 1u);
    return key;
}

// Morton (Z-order) index: the three coordinates' bits interleaved.
uint64_t morton_key(uint32_t x, uint32_t y, uint32_t z) {
    uint64_t key = 0;
    for (int b = kBits - 1; b >= 0; --b) {
        key = (key << 1) | ((x >> b) & 1u);
        key = (key << 1) | ((y >> b) & 1u);
        key = (key << 1) | ((z >> b) & 1u);
    }
    return key;
}

}  // namespace

namespace {

// Row order: centroids quantized, axis by axis, to the median span of the
// elements' vertices along that axis, then sorted lexicographically with
// the axis that holds the most cells slowest and the one that holds the
// fewest fastest, which keeps the largest distance between neighbours in
// memory as small as a row-major numbering can.  On a quasi-uniform mesh
// this recovers the row-major order of a structured grid.
void row_keys(int64_t E, const double *vert, const std::vector<double> &c,
              const double *lo, std::vector<uint64_t> &key) {
    double h[3];
    std::vector<double> span((size_t)E);
    for (int d = 0; d < 3; ++d) {
        for (int64_t e = 0; e < E; ++e) {
            double mn = INFINITY, mx = -INFINITY;
            for (int v = 0; v < 8; ++v) {
                mn = std::min(mn, vert[(e * 8 + v) * 3 + d]);
                mx = std::max(mx, vert[(e * 8 + v) * 3 + d]);
            }
            span[e] = mx - mn;
        }
        std::nth_element(span.begin(), span.begin() + E / 2, span.end());
        h[d] = span[(size_t)E / 2];
        if (!(h[d] > 0.0)) fail(SEM_EINVAL, "row order: elements of zero extent");
    }
    std::vector<int64_t> q(3 * (size_t)E);
    int64_t cells[3] = {0, 0, 0};
    for (int64_t e = 0; e < E; ++e)
        for (int d = 0; d < 3; ++d) {
            const int64_t v = (int64_t)std::floor((c[3 * e + d] - lo[d]) / h[d] + 0.5);
            if (v < 0 || v >= (int64_t(1) << 21))
                fail(SEM_EINVAL, "row order: more than 2^21 cells along an axis");
            q[3 * e + d] = v;
            cells[d] = std::max(cells[d], v + 1);
        }
    // axes by cell count, most cells first (ties: z before y before x)
    int ax[3] = {2, 1, 0};
    std::stable_sort(ax, ax + 3, [&](int a, int b) { return cells[a] > cells[b]; });
    for (int64_t e = 0; e < E; ++e)
        key[e] = ((uint64_t)q[3 * e + ax[0]] << 42) | ((uint64_t)q[3 * e + ax[1]] << 21) |
                 (uint64_t)q[3 * e + ax[2]];
}

}  // namespace

void element_order(int64_t E, const double *vert, int kind, int64_t *perm) {
    if (E <= 0) fail(SEM_EINVAL, "n_elem must be positive");
    if (!vert || !perm) fail(SEM_EINVAL, "vert_xyz and perm must not be NULL");
    if (kind != SEM_ORDER_HILBERT && kind != SEM_ORDER_MORTON && kind != SEM_ORDER_ROWS)
        fail(SEM_EINVAL, "unknown element order");
    std::vector<double> c(3 * (size_t)E);
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t e = 0; e < E; ++e) {
        for (int d = 0; d < 3; ++d) {
            double s = 0.0;
            for (int v = 0; v < 8; ++v) s += vert[(e * 8 + v) * 3 + d];
            s *= 0.125;
            if (!std::isfinite(s)) fail(SEM_EINVAL, "non-finite vertex coordinate");
            c[3 * e + d] = s;
            lo[d] = std::min(lo[d], s);
            hi[d] = std::max(hi[d], s);
        }
    }
    // one scale for all axes keeps the curve's cells cubes
    double ext = 0.0;
    for (int d = 0; d < 3; ++d) ext = std::max(ext, hi[d] - lo[d]);
    const double cells = (double)((1u << kBits) - 1);
    const double sc = ext > 0 ? cells / ext : 0.0;
    std::vector<uint64_t> key((size_t)E);
    if (kind == SEM_ORDER_ROWS) row_keys(E, vert, c, lo, key);
    else for (int64_t e = 0; e < E; ++e) {
        uint32_t q[3];
        for (int d = 0; d < 3; ++d) {
            double v = std::floor((c[3 * e + d] - lo[d]) * sc + 0.5);
            v = std::min(std::max(v, 0.0), cells);
            q[d] = (uint32_t)v;
        }
        key[e] = kind == SEM_ORDER_HILBERT ? hilbert_key(q[0], q[1], q[2])
                                           : morton_key(q[0], q[1], q[2]);
    }
    std::vector<int64_t> idx((size_t)E);
    std::iota(idx.begin(), idx.end(), int64_t(0));
    // ties (elements with one centroid cell) keep their input order
    std::stable_sort(idx.begin(), idx.end(),
                     [&](int64_t a, int64_t b) { return key[a] < key[b]; });
    std::copy(idx.begin(), idx.end(), perm);
}

}  // namespace sem
