// Persistent autotuning results: a process-wide table of launch parameters
// keyed by (GPU architecture, horizontal geometry kind, grid n_x n_y n_z,
// precision, right-hand sides),
// loaded from a text file next to libpcg.so (or the file named by the
// PCG_TUNING_CACHE environment variable; an empty value disables it) and
// extended by pcg_autotune.  A problem uses a table entry for a solve unless
// its tuning was set explicitly (pcg_set_tuning / pcg_autotune).
//
// File format, one entry per line ('#' starts a comment):
//   arch geom nx ny nz dtype nrhs lanes_per_column block_cap reduction
//        lanes_per_column_prec block_cap_prec
// with geom "uniform" or "stretched" (the stretched kernels also factorise
// the column blocks, so their best launch shape differs); without the last
// two fields the line-solve kernels take the same shape as the others.
#include <dlfcn.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>

#include "problem.h"

namespace pcg {

namespace {

using Key = std::tuple<std::string, std::string, int32_t, int32_t, int32_t, int32_t, int64_t>;

struct Cache {
    std::mutex mu;
    bool loaded = false;
    std::string path;
    std::map<Key, Tuning> table;
};

Cache& cache()
{
    static Cache c;
    return c;
}

std::string default_path()
{
    if (const char* env = std::getenv("PCG_TUNING_CACHE")) return env;
    Dl_info info;
    if (dladdr(reinterpret_cast<void*>(&default_path), &info) && info.dli_fname) {
        std::string lib = info.dli_fname;
        const size_t slash = lib.rfind('/');
        return (slash == std::string::npos ? std::string(".") : lib.substr(0, slash)) +
               "/tuning_cache.txt";
    }
    return "";
}

bool parse_into(const std::string& path, std::map<Key, Tuning>& table)
{
    std::ifstream in(path);
    if (!in) return false;
    std::string line;
    while (std::getline(in, line)) {
        const size_t hash = line.find('#');
        if (hash != std::string::npos) line.resize(hash);
        std::istringstream ls(line);
        std::string arch, geom;
        int32_t nx, ny, nz, dtype, L, mode;
        int64_t nrhs, cap;
        if (!(ls >> arch >> geom >> nx >> ny >> nz >> dtype >> nrhs >> L >> cap >> mode)) continue;
        int32_t L_b = L;
        int64_t cap_b = cap;
        if (ls >> L_b) {
            if (!(ls >> cap_b)) continue;
        } else {
            L_b = L;
        }
        if (geom != "uniform" && geom != "stretched") continue;
        Shape sh, sh_b;
        sh.L = L;
        sh_b.L = L_b;
        if (dtype < 0 || dtype > 1 || !shape_supported(nz, sh) || !shape_supported(nz, sh_b) ||
            cap < 1 || cap > kMaxBlocks || cap_b < 1 || cap_b > kMaxBlocks ||
            (mode != 0 && mode != 1))
            continue;   // ignore malformed entries
        sh.M = 1;
        while (sh.M * L < nz) sh.M <<= 1;
        sh_b.M = 1;
        while (sh_b.M * L_b < nz) sh_b.M <<= 1;
        Tuning t;
        t.shape = sh;
        t.block_cap = cap;
        t.red_mode = mode;
        t.shape_b = sh_b;
        t.block_cap_b = cap_b;
        table[Key(arch, geom, nx, ny, nz, dtype, nrhs)] = t;
    }
    return true;
}

void ensure_loaded(Cache& c)
{
    if (c.loaded) return;
    c.loaded = true;
    c.path = default_path();
    if (!c.path.empty()) parse_into(c.path, c.table);
}

Key key_of(const pcg_problem* P, int dtype, int64_t nrhs)
{
    return Key(P->arch, P->d_hgeo ? "stretched" : "uniform", P->geom.nx, P->geom.ny, P->geom.nz,
               dtype, nrhs);
}

}  // namespace

bool tuning_lookup(const pcg_problem* P, int dtype, int64_t nrhs, Tuning* out)
{
    Cache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    ensure_loaded(c);
    auto it = c.table.find(key_of(P, dtype, nrhs));
    if (it == c.table.end()) return false;
    *out = it->second;
    return true;
}

void tuning_store(const pcg_problem* P, int dtype, int64_t nrhs, const Tuning& t)
{
    Cache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    ensure_loaded(c);
    c.table[key_of(P, dtype, nrhs)] = t;
}

Tuning effective_tuning(const pcg_problem* P, int dtype, int64_t nrhs)
{
    if (P->tune_explicit[dtype]) return P->tune[dtype];
    Tuning t;
    if (tuning_lookup(P, dtype, nrhs, &t)) return t;
    return P->tune[dtype];
}

}  // namespace pcg

using namespace pcg;

extern "C" {

pcg_status pcg_tuning_cache_load(const char* path)
{
    Cache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    ensure_loaded(c);
    const std::string p = path ? path : c.path;
    if (p.empty() || !parse_into(p, c.table)) {
        set_error("pcg_tuning_cache_load: cannot read '" + p + "'");
        return PCG_E_INVALID;
    }
    return PCG_OK;
}

pcg_status pcg_tuning_cache_save(const char* path)
{
    Cache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    ensure_loaded(c);
    const std::string p = path ? path : c.path;
    std::ofstream out(p);
    if (p.empty() || !out) {
        set_error("pcg_tuning_cache_save: cannot write '" + p + "'");
        return PCG_E_INVALID;
    }
    out << "# libpcg launch parameters found by pcg_autotune\n"
        << "# arch geom nx ny nz dtype nrhs lanes_per_column block_cap reduction "
           "lanes_per_column_prec block_cap_prec\n";
    for (const auto& kv : c.table) {
        const Key& k = kv.first;
        const Tuning& t = kv.second;
        out << std::get<0>(k) << ' ' << std::get<1>(k) << ' ' << std::get<2>(k) << ' '
            << std::get<3>(k) << ' ' << std::get<4>(k) << ' ' << std::get<5>(k) << ' '
            << std::get<6>(k) << ' ' << t.shape.L << ' ' << t.block_cap << ' ' << t.red_mode
            << ' ' << t.shape_b.L << ' ' << t.block_cap_b << '\n';
    }
    return out ? PCG_OK : PCG_E_INVALID;
}

}  // extern "C"
