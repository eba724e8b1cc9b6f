// Host-side problem object of libpcg.
#pragma once

#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "internal.h"

namespace pcg {

// Key of a graph of iteration chunks: every pointer and size baked into it.
struct GraphKey {
    int dtype;
    int kind;             // 0: fused iteration chunk, 1: unfused iteration chunk
    int iters;
    int L;
    int red_mode;
    int64_t bpr;
    int64_t nrhs;
    const void* ptrs[8];
    bool operator<(const GraphKey& o) const
    {
        return std::tie(dtype, kind, iters, L, red_mode, bpr, nrhs, ptrs[0], ptrs[1], ptrs[2],
                        ptrs[3], ptrs[4], ptrs[5], ptrs[6], ptrs[7]) <
               std::tie(o.dtype, o.kind, o.iters, o.L, o.red_mode, o.bpr, o.nrhs, o.ptrs[0],
                        o.ptrs[1], o.ptrs[2], o.ptrs[3], o.ptrs[4], o.ptrs[5], o.ptrs[6],
                        o.ptrs[7]);
    }
};

}  // namespace pcg

struct pcg_problem {
    pcg_problem_desc desc{};
    pcg::Geom geom{};
    int device = 0;
    std::vector<double> vert64, lu64;      // host copies of the tables
    void* dev_tables = nullptr;            // vert64 | lu64 | vert32 | lu32
    const double* d_vert64 = nullptr;
    const double* d_lu64 = nullptr;
    const float* d_vert32 = nullptr;
    const float* d_lu32 = nullptr;
    pcg::Tuning tune[2];                   // launch parameters per dtype
    int last_iters[2] = {0, 0};            // adaptive chunk length per precision
    pcg::SolverState* pinned_states = nullptr;  // host-pinned staging of solver states
    int64_t pinned_cap = 0;
    std::map<pcg::GraphKey, hipGraphExec_t> graphs;
    std::vector<hipEvent_t> events;
};
