// tune_table.hip -- the autotuners' table of measured best surface
// configurations (host code): one entry per (kind, device architecture, CU
// count, shape class), kind "single" for sweep_autotune and "batch" for
// sweep_autotune_batched.  When the environment variable SWEEP_TUNE_CACHE
// names a file, the table is read from it on first use and rewritten (to a
// temporary file, then renamed) after each tuning; one entry per line:
//   kind arch cus a0 a1 a2 a3 a4 config ms
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "abi_internal.hpp"

namespace sweep {

namespace {

struct Key {
    std::string kind, arch;
    int cus;
    int a[kTuneClassInts];
    bool operator<(const Key& o) const
    {
        return std::tie(kind, arch, cus, a[0], a[1], a[2], a[3], a[4]) <
               std::tie(o.kind, o.arch, o.cus, o.a[0], o.a[1], o.a[2], o.a[3], o.a[4]);
    }
};
struct Val {
    int config;
    float ms;
};

std::mutex g_mu;
std::map<Key, Val> g_table;
bool g_loaded = false;
std::string g_arch;
int g_cus = -1;

void device_identity()
{
    if (g_cus >= 0) return;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        g_arch = prop.gcnArchName;
        const size_t colon = g_arch.find(':');
        if (colon != std::string::npos) g_arch.resize(colon);
        g_cus = prop.multiProcessorCount;
    } else {
        (void)hipGetLastError();
        g_arch = "unknown";
        g_cus = 0;
    }
}

Key make_key(const char* kind, const int* a)
{
    device_identity();
    Key k{kind, g_arch, g_cus, {}};
    std::memcpy(k.a, a, sizeof k.a);
    return k;
}

void load_locked()
{
    if (g_loaded) return;
    g_loaded = true;
    const char* path = std::getenv("SWEEP_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '#') continue;
        char kind[16], arch[64];
        Key k;
        Val v;
        if (std::sscanf(line, "%15s %63s %d %d %d %d %d %d %d %f", kind, arch, &k.cus, &k.a[0], &k.a[1], &k.a[2],
                        &k.a[3], &k.a[4], &v.config, &v.ms) == 10 &&
            v.config >= 0 && v.config < tile_config_count()) {
            k.kind = kind;
            k.arch = arch;
            g_table[k] = v;
        }
    }
    std::fclose(f);
}

void save_locked()
{
    const char* path = std::getenv("SWEEP_TUNE_CACHE");
    if (!path || !*path) return;
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "# sweep surface tuning: kind arch cus class[5] config ms\n");
    for (const auto& e : g_table)
        std::fprintf(f, "%s %s %d %d %d %d %d %d %d %.6f\n", e.first.kind.c_str(), e.first.arch.c_str(), e.first.cus,
                     e.first.a[0], e.first.a[1], e.first.a[2], e.first.a[3], e.first.a[4], e.second.config,
                     e.second.ms);
    std::fclose(f);
    std::rename(tmp.c_str(), path);
}

}  // namespace

int tune_lookup(const char* kind, const int* cls)
{
    std::lock_guard<std::mutex> lock(g_mu);
    load_locked();
    const auto it = g_table.find(make_key(kind, cls));
    return it == g_table.end() ? -1 : it->second.config;
}

void tune_record(const char* kind, const int* cls, int config, float ms)
{
    std::lock_guard<std::mutex> lock(g_mu);
    load_locked();
    g_table[make_key(kind, cls)] = Val{config, ms};
    save_locked();
}

int ilog2_ll(long long v)
{
    int l = 0;
    while (v > 1) { v >>= 1; ++l; }
    return l;
}

}  // namespace sweep
