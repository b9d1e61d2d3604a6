// Persistent autotuner choices: see tune_cache.h.
#include "tune_cache.h"

#include <hip/hip_runtime.h>
#include <sys/stat.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <sstream>

namespace sgm {

static std::mutex g_cache_mu;

std::string tune_cache_path() {
    const char* e = std::getenv("SGM_TUNE_CACHE");
    if (e) return std::strcmp(e, "off") == 0 ? std::string() : std::string(e);
    const char* x = std::getenv("XDG_CACHE_HOME");
    if (x && *x) return std::string(x) + "/libsgm/tune.txt";
    const char* h = std::getenv("HOME");
    if (h && *h) return std::string(h) + "/.cache/libsgm/tune.txt";
    return std::string();
}

std::string tune_device_tag() {
    int dev = 0;
    hipDeviceProp_t pr;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&pr, dev) != hipSuccess) return "unknown";
    std::string arch = pr.gcnArchName;
    for (char& c : arch)
        if (c == ' ' || c == '=') c = '_';
    return arch + "/" + std::to_string(pr.multiProcessorCount);
}

bool tune_cache_get(const std::string& key, std::vector<int>& vals) {
    const std::string path = tune_cache_path();
    if (path.empty()) return false;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    FILE* f = std::fopen(path.c_str(), "r");
    if (!f) return false;
    char line[1024];
    bool found = false;
    const std::string head = key + " =";
    while (std::fgets(line, sizeof(line), f)) {
        if (std::strncmp(line, head.c_str(), head.size()) != 0) continue;
        std::istringstream in(line + head.size());
        std::vector<int> v;
        int x;
        while (in >> x) v.push_back(x);
        vals = v;  // the last line for a key wins
        found = true;
    }
    std::fclose(f);
    return found;
}

void tune_cache_put(const std::string& key, const std::vector<int>& vals) {
    const std::string path = tune_cache_path();
    if (path.empty()) return;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    // create the parent directories (one level of libsgm/ under the cache root)
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos && slash > 0) {
        const std::string dir = path.substr(0, slash);
        const size_t up = dir.rfind('/');
        if (up != std::string::npos && up > 0) mkdir(dir.substr(0, up).c_str(), 0755);
        mkdir(dir.c_str(), 0755);
    }
    FILE* f = std::fopen(path.c_str(), "a");
    if (!f) return;
    std::string s = key + " =";
    for (int v : vals) s += " " + std::to_string(v);
    s += "\n";
    std::fputs(s.c_str(), f);
    std::fclose(f);
}

}  // namespace sgm
