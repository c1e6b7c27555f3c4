// sem_tables.cpp -- host construction of the gather-scatter tables.
//
// The scatter map Q of Sec. 3.1 arrives as one global id per local point.
// Local points sharing an id are the copies summed by the gather-scatter
// (Sec. 4.3: points with equal position).  They are grouped here, once per
// mesh: groups of m > 1 copies are bucketed by m, each group's local
// indices ascending, and groups inside a bucket in ascending order of their
// first local index.  No device call is made in this file.
#include <algorithm>
#include <climits>
#include <numeric>

#include "sem_gs_body.h"
#include "sem_internal.h"

namespace sem {

void gs_classes_finish(GsClasses &c) {
    int64_t blk = 0;
    for (int q = 0; q < c.ncls; ++q) {
        c.blk0[q] = blk;
        blk += (c.ng[q] + gsb::gs_per_block(c.M[q]) - 1) / gsb::gs_per_block(c.M[q]);
    }
}

int64_t gs_total_blocks(const GsClasses &c) {
    const int q = c.ncls - 1;
    return q >= 0 ? c.blk0[q] + (c.ng[q] + gsb::gs_per_block(c.M[q]) - 1) / gsb::gs_per_block(c.M[q])
                  : 0;
}

namespace {

// Local position of face point (a, b) of face f = 2 d + s (d: normal
// direction, s: coordinate N on that side) in an element of order N.
int face_position(int N, int f, int a, int b) {
    const int P = N + 1, d = f >> 1, c = (f & 1) ? N : 0;
    const int i = d == 0 ? c : a;
    const int j = d == 0 ? a : (d == 1 ? c : b);
    const int k = d == 2 ? c : b;
    return i + P * (j + P * k);
}

// Tables of the table-free gather inside the CG update (Mesh::gs_struct).
// Applies to odd N (P^3 a multiple of 4: a pack of 4 points never straddles
// two elements) on meshes where every face-interior point is shared with
// exactly one face point of one neighbour by an affine map of the face
// coordinates, interior points are unshared and free, and every group of
// two or more copies at an edge or corner node consists of edge or corner
// nodes only.  Each condition is checked point by point; any failure keeps
// the per-point table form.
bool build_struct_tables(int64_t E, int N, const std::vector<uint8_t> &mcode,
                         const std::vector<int32_t> &plink, const std::vector<int32_t> &cnt,
                         const std::vector<int64_t> &start, const std::vector<int32_t> &byid,
                         HostTables &t) {
    const int P = N + 1, P3 = P * P * P, MS = edge_slots(N), NR = 6 + MS;
    const int64_t n = E * P3;
    if (N % 2 == 0 || P > 32 || NR > 511) return false;
    // position table
    t.pos_tab.assign(P3, 0);
    for (int k = 0; k < P; ++k)
        for (int j = 0; j < P; ++j)
            for (int i = 0; i < P; ++i) {
                const int loc = i + P * (j + P * k);
                const bool ei = i == 0 || i == N, ej = j == 0 || j == N, ek = k == 0 || k == N;
                const int on = (int)ei + (int)ej + (int)ek;
                if (on == 0) {
                    t.pos_tab[loc] = pos_entry(0, 0, 0, 0);
                } else if (on == 1) {
                    const int d = ei ? 0 : (ej ? 1 : 2);
                    const int f = 2 * d + ((d == 0 ? i : (d == 1 ? j : k)) == N);
                    const int a = d == 0 ? j : i, b = d == 2 ? j : k;
                    t.pos_tab[loc] = pos_entry(1, a, b, f);
                } else {
                    const int es = edge_slot(N, i, j, k);
                    if (es < 0 || es >= MS) return false;
                    t.pos_tab[loc] = pos_entry(2, 0, 0, 6 + es);
                }
            }
    // division by P^3 as a multiply-shift, exact for every l < 2^31
    int lg = 0;
    while ((1 << lg) < P3) ++lg;
    t.p3_shift = 31 + lg;
    t.p3_magic = (uint32_t)(((uint64_t)1 << t.p3_shift) / (uint64_t)P3 + 1);
    // interior points: unshared and free
    for (int64_t l = 0; l < n; ++l) {
        const uint32_t pe = t.pos_tab[l % P3];
        if ((pe & 3) == 0 && mcode[l] != 1) return false;
    }
    const auto fits32 = [](int64_t v) { return v >= INT32_MIN && v <= INT32_MAX; };
    t.erec.assign((size_t)E * NR, ElemRec{0, 0});
    // faces
    for (int64_t e = 0; e < E; ++e)
        for (int f = 0; f < 6; ++f) {
            ElemRec rc{(int32_t)(e * P3), 0};
            if (N >= 3) {
                const int64_t l11 = e * P3 + face_position(N, f, 1, 1);
                const uint8_t code = mcode[l11];
                const int m = code & kMultMask;
                if (m > 2) return false;
                int64_t sa = 0, sb = 0;
                if (m == 2 && !(code & kDirichletBit)) {
                    const int64_t q11 = plink[l11];
                    sa = plink[e * P3 + face_position(N, f, 2, 1)] - q11;
                    sb = plink[e * P3 + face_position(N, f, 1, 2)] - q11;
                    rc.lo = (int32_t)(q11 - sa - sb);
                }
                if (sa < -2048 || sa > 2047 || sb < -2048 || sb > 2047) return false;
                rc.hi = (int32_t)((uint32_t)code | ((uint32_t)(sa & 0xFFF) << 8) |
                                  ((uint32_t)(sb & 0xFFF) << 20));
                for (int b = 1; b < N; ++b)
                    for (int a = 1; a < N; ++a) {
                        const int64_t l = e * P3 + face_position(N, f, a, b);
                        if (mcode[l] != code) return false;
                        // the device forms lo + sa a, then + sb b, in 32 bits
                        if (!fits32((int64_t)rc.lo + sa * a)) return false;
                        const int64_t q = (int64_t)rc.lo + sa * a + sb * b;
                        if (q < 0 || q >= n) return false;
                        if (m == 2 && !(code & kDirichletBit) && q != plink[l]) return false;
                    }
            }
            t.erec[(size_t)e * NR + f] = rc;
        }
    // edge and corner nodes: codes, and their groups of two or more copies
    for (int64_t l = 0; l < n; ++l) {
        const uint32_t pe = t.pos_tab[l % P3];
        if ((pe & 3) == 2) t.erec[(size_t)(l / P3) * NR + (pe >> 12)] = ElemRec{0, mcode[l]};
    }
    const int64_t G = (int64_t)cnt.size();
    auto edge_pos = [&](int64_t l) -> int64_t {
        const uint32_t pe = t.pos_tab[l % P3];
        return (pe & 3) == 2 ? (l / P3) * MS + ((pe >> 12) - 6) : -1;
    };
    GsClasses ec{};
    std::vector<int32_t> &ew = t.ewedge_idx;
    ew.clear();
    t.n_egroups = 0;
    int sizes_seen[256] = {0};
    for (int64_t g = 0; g < G; ++g) {
        if (cnt[g] < 2) continue;
        const int32_t l0 = byid[start[g]];
        if (mcode[l0] & kDirichletBit) continue;      // masked: the update never reads the sum
        const bool first_edge = edge_pos(l0) >= 0;
        for (int64_t o = start[g]; o < start[g + 1]; ++o)
            if ((edge_pos(byid[o]) >= 0) != first_edge) return false;
        if (first_edge) sizes_seen[cnt[g]] = 1;
    }
    for (int msz = 2; msz <= kMaxMultiplicity; ++msz) {
        if (!sizes_seen[msz]) continue;
        if (ec.ncls == kMaxGsClasses) return false;
        const int c = ec.ncls++;
        ec.M[c] = msz;
        while (ew.size() % 8) ew.push_back(0);
        ec.io[c] = (int64_t)ew.size();
        int64_t ng = 0;
        // compact ids are numbered by first appearance: ascending first local
        // index; a group's rank is its position in class order
        for (int64_t g = 0; g < G; ++g) {
            if (cnt[g] != msz) continue;
            const int32_t l0 = byid[start[g]];
            if ((mcode[l0] & kDirichletBit) || edge_pos(l0) < 0) continue;
            const int64_t rank = t.n_egroups + ng;
            if (rank >= (int64_t(1) << 31) - n) return false;
            for (int64_t o = start[g]; o < start[g + 1]; ++o) {
                const int32_t lm = byid[o];
                ew.push_back((int32_t)edge_pos(lm));
                t.erec[(size_t)(lm / P3) * NR + (t.pos_tab[lm % P3] >> 12)].lo = (int32_t)rank;
            }
            ++ng;
        }
        ec.ng[c] = ng;
        t.n_egroups += ng;
    }
    while (ew.size() % 8) ew.push_back(0);
    gs_classes_finish(ec);
    t.ecls = ec;
    // every local index: the division, and the decoded code against mcode
    for (int64_t l = 0; l < n; ++l) {
        const int64_t e = (int64_t)(((uint64_t)l * t.p3_magic) >> t.p3_shift);
        if (e != l / P3) return false;
        const uint32_t pe = t.pos_tab[l - e * P3];
        const int code = (pe & 3) == 0 ? 1 : (t.erec[(size_t)e * NR + (pe >> 12)].hi & 255);
        if (code != mcode[l]) return false;
    }
    return true;
}

}  // namespace

void build_tables(int64_t E, int N, const int64_t *gid, const uint8_t *dir, HostTables &t) {
    const int P = N + 1, P3 = P * P * P;
    const int64_t n = E * P3;
    // ---- global ids: validate, count copies -------------------------------
    int64_t maxid = -1;
    for (int64_t l = 0; l < n; ++l) {
        if (gid[l] < 0) fail(SEM_EINVAL, "glob_id has a negative entry at " + std::to_string(l));
        maxid = std::max(maxid, gid[l]);
    }
    // compact ids to 0..n_glob-1 in order of first appearance
    std::vector<int32_t> cid(n);
    {
        const bool dense = maxid < 4 * n + 16;
        if (dense) {
            std::vector<int32_t> map(maxid + 1, -1);
            int32_t next = 0;
            for (int64_t l = 0; l < n; ++l) {
                int32_t &c = map[gid[l]];
                if (c < 0) c = next++;
                cid[l] = c;
            }
            t.n_glob = next;
        } else {
            std::vector<int64_t> order(n);
            std::iota(order.begin(), order.end(), 0);
            std::stable_sort(order.begin(), order.end(),
                             [&](int64_t a, int64_t b) { return gid[a] < gid[b]; });
            // first-appearance numbering: smallest l of each id
            std::vector<std::pair<int64_t, int64_t>> first;   // (first l, rank in sorted ids)
            int32_t rank = -1;
            std::vector<int32_t> rank_of(n);
            for (int64_t t = 0; t < n; ++t) {
                if (t == 0 || gid[order[t]] != gid[order[t - 1]]) {
                    ++rank;
                    first.push_back({order[t], rank});
                }
                rank_of[order[t]] = rank;
            }
            std::vector<int32_t> renum(first.size());
            std::sort(first.begin(), first.end());
            for (size_t q = 0; q < first.size(); ++q) renum[first[q].second] = (int32_t)q;
            for (int64_t l = 0; l < n; ++l) cid[l] = renum[rank_of[l]];
            t.n_glob = (int64_t)first.size();
        }
    }
    const int64_t G = t.n_glob;
    std::vector<int32_t> cnt(G, 0);
    for (int64_t l = 0; l < n; ++l) ++cnt[cid[l]];
    std::vector<int8_t> dflag(G, -1);
    for (int64_t l = 0; l < n; ++l) {
        const int8_t d = dir ? (dir[l] ? 1 : 0) : 0;
        int8_t &f = dflag[cid[l]];
        if (f < 0) f = d;
        else if (f != d)
            fail(SEM_EINVAL, "dirichlet flags differ between copies of a global point (local " +
                                 std::to_string(l) + ")");
    }
    std::vector<uint8_t> &mcode = t.mcode;
    mcode.assign(n, 0);
    int64_t n_dir = 0;
    for (int64_t l = 0; l < n; ++l) {
        const int32_t c = cnt[cid[l]];
        if (c > kMaxMultiplicity)
            fail(SEM_EINVAL, "more than 127 local copies of one global point");
        const bool d = dflag[cid[l]] == 1;
        mcode[l] = (uint8_t)((d ? kDirichletBit : 0) | c);
        n_dir += d;
    }

    // ---- groups by size class ----------------------------------------------
    // CSR of local points by compact id (ascending l inside each id)
    std::vector<int64_t> start(G + 1, 0);
    for (int64_t g = 0; g < G; ++g) start[g + 1] = start[g] + cnt[g];
    std::vector<int32_t> byid(n);
    {
        std::vector<int64_t> fill(start.begin(), start.end() - 1);
        for (int64_t l = 0; l < n; ++l) byid[fill[cid[l]]++] = (int32_t)l;
    }
    // compact ids are numbered by first appearance, so ascending id order is
    // ascending first-local-index order
    int sizes_seen[256] = {0};
    for (int64_t g = 0; g < G; ++g)
        if (cnt[g] > 1) sizes_seen[cnt[g]] = 1;
    GsClasses cls{};
    int64_t n_shared = 0, n_groups = 0;
    std::vector<int32_t> &gs_idx = t.gs_idx;
    gs_idx.clear();
    // per local point: the other copy of a pair (m = 2), or the rank of its
    // group among the groups of more than two copies (class order)
    std::vector<int32_t> plink(n, 0);
    int64_t n_multi = 0;
    for (int msz = 2; msz <= kMaxMultiplicity; ++msz) {
        if (!sizes_seen[msz]) continue;
        if (cls.ncls == kMaxGsClasses)
            fail(SEM_EUNSUPPORTED, "more than 32 distinct multiplicities");
        const int c = cls.ncls++;
        cls.M[c] = msz;
        // every class starts on a 32-byte boundary (vector index loads)
        while (gs_idx.size() % 8) gs_idx.push_back(0);
        cls.io[c] = (int64_t)gs_idx.size();
        int64_t ng = 0;
        for (int64_t g = 0; g < G; ++g) {
            if (cnt[g] != msz) continue;
            for (int64_t o = start[g]; o < start[g + 1]; ++o) gs_idx.push_back(byid[o]);
            if (msz == 2) {
                plink[byid[start[g]]] = byid[start[g] + 1];
                plink[byid[start[g] + 1]] = byid[start[g]];
            } else {
                for (int64_t o = start[g]; o < start[g + 1]; ++o) plink[byid[o]] = (int32_t)n_multi;
                ++n_multi;
            }
            ++ng;
        }
        cls.ng[c] = ng;
        n_groups += ng;
        n_shared += ng * msz;
    }
    while (gs_idx.size() % 8) gs_idx.push_back(0);
    gs_classes_finish(cls);
    t.gs = cls;
    // order of the gather-scatter's logical blocks: by the first local index
    // of each block's first group (ties: class-major order), so that one
    // launch position range, which one XCD runs, covers every class of one
    // region of the mesh instead of each class sweeping the whole mesh
    {
        const int64_t nblk = gs_total_blocks(cls);
        std::vector<int64_t> key((size_t)nblk);
        for (int c = 0; c < cls.ncls; ++c) {
            const int64_t gpb = gsb::gs_per_block(cls.M[c]);
            const int64_t nb = (cls.ng[c] + gpb - 1) / gpb;
            for (int64_t k = 0; k < nb; ++k)
                key[(size_t)(cls.blk0[c] + k)] = gs_idx[(size_t)(cls.io[c] + k * gpb * cls.M[c])];
        }
        t.gs_lb_order.resize((size_t)nblk);
        std::iota(t.gs_lb_order.begin(), t.gs_lb_order.end(), 0);
        std::stable_sort(t.gs_lb_order.begin(), t.gs_lb_order.end(),
                         [&](int32_t a, int32_t b) { return key[a] < key[b]; });
    }
    // classes are in ascending m: the groups of more than two copies are the
    // gather-scatter blocks from the first class with M > 2 on
    t.n_groups_multi = n_multi;
    t.gs_blk_multi = gs_total_blocks(cls);
    for (int c = 0; c < cls.ncls; ++c)
        if (cls.M[c] > 2) {
            t.gs_blk_multi = cls.blk0[c];
            break;
        }
    t.n_groups = n_groups;
    t.n_shared = n_shared;
    t.n_dir = n_dir;
    std::vector<int32_t> &dir_idx = t.dir_idx;
    dir_idx.clear();
    dir_idx.reserve(n_dir);
    for (int64_t l = 0; l < n; ++l)
        if (mcode[l] & kDirichletBit) dir_idx.push_back((int32_t)l);

    // Table of the gather inside the CG update, used when every shared
    // point lies on its element's surface (true of every conforming mesh:
    // shared nodes are face, edge and vertex nodes; a mesh tying interior
    // nodes takes the separate gather-scatter pass).  The entry of a pair
    // point is its partner's local index; that of a point in a larger group
    // is the group's rank among the groups with m > 2, in class order (the
    // order of the group-sum kernel's output); any other point holds its own
    // index.  One entry per point: the update loads 4 at once.
    bool ok = true;
    for (int64_t l = 0; l < n && ok; ++l) {
        if ((mcode[l] & kMultMask) <= 1) continue;
        const int loc = (int)(l % P3), i = loc % P, j = (loc / P) % P, k = loc / (P * P);
        if (!(i == 0 || i == N || j == 0 || j == N || k == 0 || k == N)) ok = false;
    }
    t.gsrc.clear();
    if (ok) {
        t.gsrc.resize((size_t)n);
        for (int64_t l = 0; l < n; ++l)
            t.gsrc[l] = (mcode[l] & kMultMask) > 1 ? plink[l] : (int32_t)l;
    }
    t.gs_in_update = ok;

    // compact edge-array positions of the copies of the groups with m > 2
    t.gsum_wedge = false;
    t.wedge_idx.clear();
    t.wedge_io0 = 0;
    int c0 = -1;
    for (int c = 0; c < cls.ncls; ++c)
        if (cls.M[c] > 2) {
            c0 = c;
            break;
        }
    if (ok && c0 >= 0) {
        t.wedge_io0 = cls.io[c0];
        const int MS = edge_slots(N);
        bool all_edge = true;
        t.wedge_idx.assign(gs_idx.size() - (size_t)t.wedge_io0, 0);
        for (int c = c0; c < cls.ncls && all_edge; ++c)
            for (int64_t q = 0; q < cls.ng[c] * cls.M[c]; ++q) {
                const int64_t o = cls.io[c] + q;
                const int64_t l = gs_idx[o], e = l / P3, loc = l % P3;
                const int i = (int)(loc % P), j = (int)((loc / P) % P), k = (int)(loc / (P * P));
                const int es = edge_slot(N, i, j, k);
                if (es < 0) {
                    all_edge = false;
                    break;
                }
                t.wedge_idx[o - t.wedge_io0] = (int32_t)(e * MS + es);
            }
        t.gsum_wedge = all_edge;
        if (!all_edge) t.wedge_idx.clear();
    }

    t.gs_struct = ok && build_struct_tables(E, N, mcode, plink, cnt, start, byid, t);
}

}  // namespace sem
