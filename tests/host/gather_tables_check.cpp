// Host check of the gather-scatter tables and of the gather that the CG
// update does with them (the same __host__ __device__ functions the kernel
// calls, run here on the CPU over every local point): the sums of the groups
// of more than two copies, then the update's gather, must give every point
// the ascending-order sum of all its copies, bitwise.
//
// usage: gather_tables_check E N glob_id.bin dirichlet.bin seed
//   glob_id.bin: int64 [E][(N+1)^3], dirichlet.bin: uint8 [E][(N+1)^3]
// Prints "gs_in_update=<0|1> checked=<points> odd_m=<points with m other
// than 1, 2, 4, 8> gsum_wedge=<0|1> table_free=<0|1> checked_tf=<points>"
// and exits 0, or names the first failing point and exits 1.  The
// table-free form (odd N) is checked the same way: every point's decoded
// code and value against its copies' ascending-order sum, bitwise.  The
// gather-scatter's block order must be a permutation of its logical blocks
// sorted by each block's first local index ("gs_blocks=<blocks>").
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <random>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../paper_2108_12188_amd/csrc/sem_gs_body.h"
#include "../../paper_2108_12188_amd/csrc/sem_vec_body.h"

namespace sem {
void set_error(const std::string &) {}
[[noreturn]] void fail(sem_status code, const std::string &msg) {
    throw std::runtime_error("status " + std::to_string((int)code) + ": " + msg);
}
void check_hip(hipError_t, const char *) {}
}  // namespace sem

template <typename T>
static std::vector<T> read_all(const char *path, size_t count) {
    std::vector<T> v(count);
    FILE *f = std::fopen(path, "rb");
    if (!f || std::fread(v.data(), sizeof(T), count, f) != count) {
        std::fprintf(stderr, "cannot read %s\n", path);
        std::exit(2);
    }
    std::fclose(f);
    return v;
}

#define CHECK(cond, ...)                                   \
    do {                                                   \
        if (!(cond)) {                                     \
            std::printf("FAIL l=%lld: ", (long long)l);    \
            std::printf(__VA_ARGS__);                      \
            std::printf("\n");                             \
            return 1;                                      \
        }                                                  \
    } while (0)

int main(int argc, char **argv) {
    if (argc != 6) {
        std::fprintf(stderr, "usage: %s E N glob_id.bin dirichlet.bin seed\n", argv[0]);
        return 2;
    }
    const int64_t E = std::atoll(argv[1]);
    const int N = std::atoi(argv[2]);
    const int P = N + 1, P3 = P * P * P;
    const int64_t n = E * P3;
    const std::vector<int64_t> gid = read_all<int64_t>(argv[3], (size_t)n);
    const std::vector<uint8_t> dir = read_all<uint8_t>(argv[4], (size_t)n);
    sem::HostTables t;
    sem::build_tables(E, N, gid.data(), dir.data(), t);
    int64_t l = -1;

    // reference: copies of every global id in ascending local index
    std::map<int64_t, std::vector<int64_t>> copies;
    for (l = 0; l < n; ++l) copies[gid[l]].push_back(l);

    std::mt19937_64 rng(std::strtoull(argv[5], nullptr, 10));
    std::uniform_real_distribution<float> U(-1.f, 1.f);
    std::vector<float> w32(n);
    std::vector<double> w64(n);
    // the operator leaves w unmasked: Dirichlet points hold values too
    for (l = 0; l < n; ++l) {
        w32[l] = U(rng);
        w64[l] = (double)U(rng) + 1e-9 * (double)U(rng);
    }

    // the gather-scatter's block order: a permutation of all logical blocks,
    // whose blocks' first local indices never decrease along it
    const int64_t nblk = sem::gs_total_blocks(t.gs);
    {
        l = -1;
        CHECK((int64_t)t.gs_lb_order.size() == nblk, "block order holds %lld of %lld blocks",
              (long long)t.gs_lb_order.size(), (long long)nblk);
        std::vector<int64_t> first((size_t)nblk, -1);
        for (int c = 0; c < t.gs.ncls; ++c) {
            const int64_t gpb = sem::gsb::gs_per_block(t.gs.M[c]);
            for (int64_t g = 0; g < t.gs.ng[c]; g += gpb)
                first[(size_t)(t.gs.blk0[c] + g / gpb)] = t.gs_idx[t.gs.io[c] + g * t.gs.M[c]];
        }
        std::vector<char> seen((size_t)nblk, 0);
        int64_t prev = -1;
        for (int64_t b = 0; b < nblk; ++b) {
            const int32_t lb = t.gs_lb_order[(size_t)b];
            CHECK(lb >= 0 && lb < nblk && !seen[(size_t)lb], "block order entry %lld = %d",
                  (long long)b, lb);
            seen[(size_t)lb] = 1;
            CHECK(first[(size_t)lb] >= prev, "block order not by first index at %lld",
                  (long long)b);
            prev = first[(size_t)lb];
        }
    }

    int64_t checked = 0, odd_m = 0;
    if (t.gs_in_update) {
        // the group-sum pass covers exactly the groups of more than two
        // copies: gather-scatter blocks gs_blk_multi onwards
        int64_t n_multi = 0;
        for (int c = 0; c < t.gs.ncls; ++c) {
            CHECK((t.gs.blk0[c] >= t.gs_blk_multi) == (t.gs.M[c] > 2),
                  "class %d (M = %d) on the wrong side of block %lld", c, t.gs.M[c],
                  (long long)t.gs_blk_multi);
            if (t.gs.M[c] > 2) n_multi += t.gs.ng[c];
        }
        CHECK(n_multi == t.n_groups_multi, "%lld groups with m > 2, tables say %lld",
              (long long)n_multi, (long long)t.n_groups_multi);
        // that pass on the host: ascending-order sums, class by class
        std::vector<float> gs32;
        std::vector<double> gs64;
        for (int c = 0; c < t.gs.ncls; ++c) {
            const int M = t.gs.M[c];
            if (M <= 2) continue;
            for (int64_t g = 0; g < t.gs.ng[c]; ++g) {
                const int32_t *ix = t.gs_idx.data() + t.gs.io[c] + g * M;
                float s32 = w32[ix[0]];
                double s64 = w64[ix[0]];
                for (int q = 1; q < M; ++q) {
                    s32 += w32[ix[q]];
                    s64 += w64[ix[q]];
                }
                gs32.push_back(s32);
                gs64.push_back(s64);
            }
        }
        // the same sums from the operator's compact copy of the edge and
        // corner nodes, when the tables allow it
        if (t.gsum_wedge) {
            const int MS = sem::edge_slots(N);
            std::vector<float> we32((size_t)E * MS, 0.f);
            std::vector<double> we64((size_t)E * MS, 0.0);
            for (l = 0; l < n; ++l) {
                const int64_t e = l / P3, loc = l % P3;
                const int es = sem::edge_slot(N, (int)(loc % P), (int)((loc / P) % P),
                                              (int)(loc / (P * P)));
                CHECK(es < MS, "edge slot %d of %d", es, MS);
                if (es >= 0) {
                    we32[e * MS + es] = w32[l];
                    we64[e * MS + es] = w64[l];
                }
            }
            size_t k = 0;
            for (int c = 0; c < t.gs.ncls; ++c) {
                const int M = t.gs.M[c];
                if (M <= 2) continue;
                for (int64_t g = 0; g < t.gs.ng[c]; ++g, ++k) {
                    const int64_t o = t.gs.io[c] + g * M - t.wedge_io0;
                    l = t.gs_idx[t.gs.io[c] + g * M];
                    CHECK(o >= 0 && (size_t)(o + M) <= t.wedge_idx.size(), "edge list offset");
                    float s32 = we32[t.wedge_idx[o]];
                    double s64 = we64[t.wedge_idx[o]];
                    for (int q = 1; q < M; ++q) {
                        CHECK(t.wedge_idx[o + q] >= 0 && t.wedge_idx[o + q] < E * MS, "position");
                        s32 += we32[t.wedge_idx[o + q]];
                        s64 += we64[t.wedge_idx[o + q]];
                    }
                    CHECK(std::memcmp(&s32, &gs32[k], 4) == 0 && std::memcmp(&s64, &gs64[k], 8) == 0,
                          "group sum from the edge array differs");
                }
            }
        }
        const sem::vecb::GatherMap gm{t.gsrc.data()};
        CHECK(t.gsrc.size() == (size_t)n, "gather table size %zu", t.gsrc.size());
        for (l = 0; l < n; ++l) {
            const int loc = (int)(l % P3), li = loc % P, lj = (loc / P) % P, lk_ = loc / (P * P);
            const bool surface = li == 0 || li == N || lj == 0 || lj == N || lk_ == 0 || lk_ == N;
            const int32_t lk = gm.gsrc[l];
            CHECK(lk >= 0 && lk < n, "gather table entry %d", lk);
            const uint8_t code = t.mcode[l];
            const int m = code & sem::kMultMask;
            const std::vector<int64_t> &cp = copies[gid[l]];
            CHECK((int)cp.size() == m, "multiplicity %d, copies %zu", m, cp.size());
            if (m != 1 && m != 2 && m != 4 && m != 8) ++odd_m;
            if (m >= 2) CHECK(surface, "shared point not on the element surface");
            if (m <= 1) CHECK(lk == l, "own entry %d for point %lld", lk, (long long)l);
            if (m == 2) {
                const int64_t other = cp[0] == l ? cp[1] : cp[0];
                CHECK(lk == other, "partner %d, expected %lld", lk, (long long)other);
            }
            if (m > 2) CHECK(lk >= 0 && lk < n_multi, "group rank %d", lk);
            // the gathered value against the ascending-order sum of the copies
            float s32 = w32[cp[0]];
            double s64 = w64[cp[0]];
            for (size_t q = 1; q < cp.size(); ++q) {
                s32 += w32[cp[q]];
                s64 += w64[cp[q]];
            }
            if (code & sem::kDirichletBit) {
                s32 = 0.f;
                s64 = 0.0;
            }
            const float *src32 = sem::vecb::gather_source<float>(w32.data(), gs32.data(), code,
                                                                 lk, l);
            const double *src64 = sem::vecb::gather_source<double>(w64.data(), gs64.data(), code,
                                                                   lk, l);
            const float g32 = sem::vecb::copies_sum<float>(w32[l], code, *src32);
            const double g64 = sem::vecb::copies_sum<double>(w64[l], code, *src64);
            CHECK(std::memcmp(&g32, &s32, 4) == 0, "fp32 gather %a, expected %a", g32, s32);
            CHECK(std::memcmp(&g64, &s64, 8) == 0, "fp64 gather %a, expected %a", g64, s64);
            ++checked;
        }
    }
    // the table-free form: the operator's compact edge copy, the sums of the
    // edge-node groups in class order (the group-sum kernel's order: members
    // as listed), then the update's decode of every point, bitwise against
    // the same ascending-order sums
    int64_t checked_tf = 0;
    if (t.gs_struct) {
        const int MS = sem::edge_slots(N);
        CHECK(N % 2 == 1 && (int)t.pos_tab.size() == P3, "table-free form at N = %d", N);
        std::vector<float> we32((size_t)E * MS, 0.f);
        std::vector<double> we64((size_t)E * MS, 0.0);
        for (l = 0; l < n; ++l) {
            const int loc = (int)(l % P3);
            const int es = sem::edge_slot(N, loc % P, (loc / P) % P, loc / (P * P));
            if (es >= 0) {
                we32[(size_t)(l / P3) * MS + es] = w32[l];
                we64[(size_t)(l / P3) * MS + es] = w64[l];
            }
        }
        std::vector<float> es32;
        std::vector<double> es64;
        for (int c = 0; c < t.ecls.ncls; ++c) {
            const int M = t.ecls.M[c];
            CHECK(M >= 2, "edge class of %d copies", M);
            for (int64_t g = 0; g < t.ecls.ng[c]; ++g) {
                const int32_t *ix = t.ewedge_idx.data() + t.ecls.io[c] + g * M;
                float s32 = we32[ix[0]];
                double s64 = we64[ix[0]];
                for (int q = 1; q < M; ++q) {
                    CHECK(ix[q] >= 0 && ix[q] < E * MS, "edge position %d", ix[q]);
                    s32 += we32[ix[q]];
                    s64 += we64[ix[q]];
                }
                es32.push_back(s32);
                es64.push_back(s64);
            }
        }
        CHECK((int64_t)es32.size() == t.n_egroups, "%zu edge groups, tables say %lld",
              es32.size(), (long long)t.n_egroups);
        const sem::vecb::StructMap sm{t.erec.data(), t.pos_tab.data(), P3, 6 + MS, t.p3_magic,
                                      t.p3_shift};
        // the update's wg: w followed by the edge-group sums
        std::vector<float> wg32(w32);
        std::vector<double> wg64(w64);
        wg32.insert(wg32.end(), es32.begin(), es32.end());
        wg64.insert(wg64.end(), es64.begin(), es64.end());
        for (l = 0; l < n; ++l) {
            const int64_t l0 = l & ~(int64_t)3;
            const int64_t e = sem::vecb::struct_elem(sm, l0);
            CHECK(e == l / P3, "element %lld of a pack", (long long)e);
            const uint32_t pe = t.pos_tab[l - e * P3];
            const sem::ElemRec rc = sem::vecb::struct_record(sm, e, pe);
            const sem::vecb::StructSrc ss = sem::vecb::struct_source(sm, n, l, pe, rc);
            CHECK(ss.code == t.mcode[l], "decoded code %d, expected %d", ss.code, t.mcode[l]);
            CHECK(ss.idx >= 0 && ss.idx < (int64_t)wg32.size(), "source index %lld out of bounds",
                  (long long)ss.idx);
            const std::vector<int64_t> &cp = copies[gid[l]];
            float s32 = w32[cp[0]];
            double s64 = w64[cp[0]];
            for (size_t q = 1; q < cp.size(); ++q) {
                s32 += w32[cp[q]];
                s64 += w64[cp[q]];
            }
            if (t.mcode[l] & sem::kDirichletBit) {
                s32 = 0.f;
                s64 = 0.0;
            }
            const float g32 = sem::vecb::struct_sum<float>(w32[l], ss.code, ss.edge, wg32[ss.idx]);
            const double g64 = sem::vecb::struct_sum<double>(w64[l], ss.code, ss.edge, wg64[ss.idx]);
            CHECK(std::memcmp(&g32, &s32, 4) == 0, "table-free fp32 gather %a, expected %a", g32,
                  s32);
            CHECK(std::memcmp(&g64, &s64, 8) == 0, "table-free fp64 gather %a, expected %a", g64,
                  s64);
            ++checked_tf;
        }
    }
    std::printf("gs_in_update=%d checked=%lld odd_m=%lld gsum_wedge=%d table_free=%d "
                "checked_tf=%lld gs_blocks=%lld\n",
                t.gs_in_update ? 1 : 0, (long long)checked, (long long)odd_m,
                t.gsum_wedge ? 1 : 0, t.gs_struct ? 1 : 0, (long long)checked_tf,
                (long long)nblk);
    return 0;
}
