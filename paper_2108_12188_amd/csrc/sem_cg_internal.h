// sem_cg_internal.h -- CG work vectors of a mesh, shared by the
// single-mesh and the batched drivers.
#pragma once

#include <map>
#include <vector>

#include "sem_internal.h"

namespace sem {

// A captured iteration graph is valid for one geometric-factor form, one
// chunk length and one generation of the tile-shape table.
struct GraphKey {
    bool otf;
    int chunk;
    int shape_gen;
    bool pc = false;
    bool operator<(const GraphKey &o) const {
        if (pc != o.pc) return pc < o.pc;
        if (otf != o.otf) return otf < o.otf;
        if (chunk != o.chunk) return chunk < o.chunk;
        return shape_gen < o.shape_gen;
    }
};

struct Workspace {
    bool fp64 = false;
    int64_t n = 0;
    int device = 0;
    void *x = nullptr, *r = nullptr, *p = nullptr, *w = nullptr, *b = nullptr;
    void *gsum = nullptr;           // sums of the groups with m > 2 (gather in the update)
    void *wedge = nullptr;          // operator's copy of the edge and corner nodes
    double *part_ax = nullptr, *part_vec = nullptr;
    void *z = nullptr;              // preconditioned residual (allocated on first use)
    double *part_vec2 = nullptr;    // second partial set of the preconditioned update
    int64_t cap_ax = 0;
    int cap_vec = 0;
    CgState *st = nullptr;          // device state of this workspace's solves
    CgState *h_st = nullptr;        // pinned mirror
    double *hist = nullptr;         // device histories: rho [cap], alpha [cap]
    int hist_cap = 0;
    double *dval = nullptr;         // device scalars
    double *h_val = nullptr;        // pinned mirror (8 doubles)
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    std::vector<hipEvent_t> tev;    // per-kernel timing events (4 per iteration)
    std::map<GraphKey, hipGraphExec_t> graphs;
    size_t bytes = 0;
};

// the mesh's workspace of one precision (created on first use)
Workspace &cg_workspace(Mesh &m, bool fp64);
int cg_auto_chunk(int64_t n, int fixed);
// w = mask(QQ^T A_L u) in FP64 (precomputed G64 if present, else on the fly)
void api_apply_A64(const Mesh &m, const double *u, double *w, hipStream_t s);

}  // namespace sem
