// Host-side problem object of libpcg.
#pragma once

#include <map>
#include <string>
#include <mutex>
#include <tuple>
#include <vector>

#include "internal.h"

namespace pcg {

// Key of a graph of iteration chunks: the profiled flag, then for every
// kernel node its function, launch dimensions and every field of its
// argument block (pointers, sizes, flags), so a replay never runs a graph
// built for other vectors or launch parameters.
using GraphKey = std::vector<uint64_t>;

// A cached executable graph and when it was last replayed (the problem's
// graph clock); the cache keeps at most kMaxGraphs, evicting the least
// recently used.
struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    uint64_t last_use = 0;
};
constexpr size_t kMaxGraphs = 16;

}  // namespace pcg

struct pcg_problem;

namespace pcg {

// A coarse level of the multigrid hierarchy (level 1, 2, ...; level 0 is the
// problem itself): its geometry and device tables (the vertical tables are
// the same on every level).
struct MgLevel {
    Geom g{};
    std::vector<double> lu64, hgeo;
    const double* d_lu64 = nullptr;
    const float* d_lu32 = nullptr;
    const double* d_hgeo = nullptr;   // stretched grids only
};

// Tuning cache (tuning_cache.cpp).
bool tuning_lookup(const pcg_problem* P, int dtype, int64_t nrhs, Tuning* out);
void tuning_store(const pcg_problem* P, int dtype, int64_t nrhs, const Tuning& t);
Tuning effective_tuning(const pcg_problem* P, int dtype, int64_t nrhs);

}  // namespace pcg

struct pcg_problem {
    pcg_problem_desc desc{};
    pcg::Geom geom{};
    int device = 0;
    std::vector<double> vert64, lu64;      // host copies of the tables
    std::vector<double> hgeo;              // stretched grids: per-index geometry (else empty)
    std::vector<pcg::MgLevel> mg;          // coarse multigrid levels
    void* mg_tables = nullptr;             // their device tables
    void* dev_tables = nullptr;            // vert64 | lu64 | vert32 | lu32 | hgeo
    const double* d_hgeo = nullptr;        // null for uniform grids
    const double* d_vert64 = nullptr;
    const double* d_lu64 = nullptr;
    const float* d_vert32 = nullptr;
    const float* d_lu32 = nullptr;
    std::string arch;                      // e.g. "gfx950" (tuning-cache key)
    pcg::Tuning tune[2];                   // launch parameters per dtype
    bool tune_explicit[2] = {false, false};  // set by pcg_set_tuning / pcg_autotune
    int last_iters[2] = {0, 0};            // adaptive chunk length per precision
    pcg::SolverState* pinned_states = nullptr;  // host-pinned staging of solver states
    int64_t pinned_cap = 0;
    std::map<pcg::GraphKey, pcg::GraphEntry> graphs;
    uint64_t graph_clock = 0;
    std::vector<hipEvent_t> events;
    std::vector<hipEvent_t> gevents;       // event nodes of profiled graph chunks
};

namespace pcg {

// Workgroups per right-hand side of the kernels of one precision with the
// problem's current tuning: the line-solve kernels (b) and all others.
int64_t blocks_per_rhs(const pcg_problem* P, int dtype);
int64_t blocks_per_rhs_b(const pcg_problem* P, int dtype);

// Launch shapes and reduction mode of one precision in a kernel argument block.
inline void set_launch(ColArgs& a, const pcg_problem* P, int dtype)
{
    a.L = P->tune[dtype].shape.L;
    a.blocks_per_rhs = blocks_per_rhs(P, dtype);
    a.L_b = P->tune[dtype].shape_b.L;
    a.bpr_b = blocks_per_rhs_b(P, dtype);
    a.red_mode = P->tune[dtype].red_mode;
}

// Table pointers of one precision in a kernel argument block.
inline void set_tables(ColArgs& a, const pcg_problem* P, int dtype)
{
    a.vert = dtype == PCG_F64 ? (const void*)P->d_vert64 : (const void*)P->d_vert32;
    a.lu = dtype == PCG_F64 ? (const void*)P->d_lu64 : (const void*)P->d_lu32;
    a.hgeo = P->d_hgeo;
}

// For the duration of one call, the problem's tunings are the effective ones
// for nrhs right-hand sides (explicit setting, else the tuning cache, else
// the defaults).
class TuneScope {
public:
    TuneScope(pcg_problem* P, int64_t nrhs) : P_(P)
    {
        for (int d = 0; d < 2; ++d) {
            saved_[d] = P->tune[d];
            P->tune[d] = effective_tuning(P, d, nrhs);
        }
    }
    ~TuneScope()
    {
        for (int d = 0; d < 2; ++d) P_->tune[d] = saved_[d];
    }

private:
    pcg_problem* P_;
    Tuning saved_[2];
};

// HBM probe (probe.hip): n_read vectors streamed in, n_write out.
hipError_t stream_probe(int n_read, int n_write, void* const* vectors, size_t bytes, int nt,
                        int64_t blocks, hipStream_t s);

}  // namespace pcg
