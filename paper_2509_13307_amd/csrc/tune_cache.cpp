// On-disk cache of the autotuner's launch-shape choices (the BF16 GEMM tiles
// and the one-kernel emulator shapes), so that a new model on the same kind
// of GPU skips the timing runs for keys measured before.
//
// One line per choice: `<arch> <table signature> <kind> <M> <N> <K> <networks>
// <candidate>`.  The architecture is the device's gcnArchName; the table
// signature is a 64-bit FNV-1a hash of the build's source hash (NSMI_SRC_ID,
// set by the build script) and the names of the candidates of that kind, so
// that entries written by another build (other kernels, another candidate
// list) are ignored rather than read as timings of this one.  Choices never
// change a result (every candidate gives identical outputs), only the speed.
//
// The file is NSMI_TUNE_CACHE if that is set (empty or "off": no cache),
// else $XDG_CACHE_HOME/nsmi/tune.txt, else $HOME/.cache/nsmi/tune.txt.  It is
// read once per model creation and appended to (one short write per new
// choice); a missing or unwritable file only means tuning runs again.
#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <sys/stat.h>

#include "nsmi.h"

namespace nsmi {

static uint64_t fnv1a(const char* s, uint64_t h) {
    for (; *s; ++s) {
        h ^= (unsigned char)*s;
        h *= 1099511628211ull;
    }
    return h;
}

#ifndef NSMI_SRC_ID
#define NSMI_SRC_ID "unversioned"
#endif

static uint64_t tune_table_sig(int kind) {
    uint64_t h = fnv1a(NSMI_SRC_ID, 1469598103934665603ull);
    const int n = tune_ncfg(kind);
    for (int c = 0; c < n; ++c) h = fnv1a(tune_cfg_name(kind, c), fnv1a("|", h));
    return h;
}

static std::string cache_path() {
    const char* p = getenv("NSMI_TUNE_CACHE");
    if (p) return (std::strcmp(p, "off") == 0) ? std::string() : std::string(p);
    const char* x = getenv("XDG_CACHE_HOME");
    if (x && *x) return std::string(x) + "/nsmi/tune.txt";
    const char* h = getenv("HOME");
    if (h && *h) return std::string(h) + "/.cache/nsmi/tune.txt";
    return std::string();
}

static void make_parent_dirs(const std::string& path) {
    for (size_t i = 1; i < path.size(); ++i)
        if (path[i] == '/') {
            const std::string d = path.substr(0, i);
            if (mkdir(d.c_str(), 0755) != 0 && errno != EEXIST) return;
        }
}

void tune_cache_load(ns_model* m) {
    hipDeviceProp_t prop;
    NS_HIP(hipGetDeviceProperties(&prop, m->device));
    m->arch = prop.gcnArchName;
    for (char& c : m->arch)
        if (c == ' ') c = '_';
    m->tune_path = cache_path();
    if (m->tune_path.empty()) return;
    FILE* f = std::fopen(m->tune_path.c_str(), "r");
    if (!f) return;
    char arch[256];
    unsigned long long sig;
    int kind, N, K, G, cfg;
    long long M;
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        if (std::sscanf(line, "%255s %llx %d %lld %d %d %d %d", arch, &sig, &kind, &M, &N, &K, &G, &cfg) != 8)
            continue;
        if (m->arch != arch || kind < 0 || kind > 17 || sig != tune_table_sig(kind)) continue;
        if (cfg < 0 || cfg >= tune_ncfg(kind)) continue;
        m->tune[std::make_tuple(kind, (int64_t)M, N, K, G)] = cfg;
    }
    std::fclose(f);
}

void tune_cache_store(ns_model* m, const std::tuple<int, int64_t, int, int, int>& key, int cfg) {
    m->tune[key] = cfg;
    if (m->tune_path.empty()) return;
    make_parent_dirs(m->tune_path);
    FILE* f = std::fopen(m->tune_path.c_str(), "a");
    if (!f) return;
    const int kind = std::get<0>(key);
    std::fprintf(f, "%s %llx %d %lld %d %d %d %d\n", m->arch.c_str(), (unsigned long long)tune_table_sig(kind), kind,
                 (long long)std::get<1>(key), std::get<2>(key), std::get<3>(key), std::get<4>(key), cfg);
    std::fclose(f);
}

}  // namespace nsmi
