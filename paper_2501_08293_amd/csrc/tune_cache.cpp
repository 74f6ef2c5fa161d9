// Persistent cache of autotuner decisions: one line per problem shape,
// "key<TAB>v0 v1 ...", in the file named by the environment variable
// OPF_ADMM_TUNE_CACHE, else $XDG_CACHE_HOME/opf_admm/tune.txt, else
// $HOME/.cache/opf_admm/tune.txt.  A later line for a key overrides earlier
// ones, so storing only appends.  Failures to read or write the file only
// disable the cache; decisions are also kept in memory for the process (per
// file, so pointing the variable at another file starts afresh).
#include "tune_cache.h"

#include <sys/stat.h>

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>

namespace opf {
namespace {

std::mutex g_mu;
std::map<std::string, std::vector<int>> g_mem;

std::string cache_path() {
    if (const char* p = std::getenv("OPF_ADMM_TUNE_CACHE")) return p;
    std::string dir;
    if (const char* x = std::getenv("XDG_CACHE_HOME")) dir = x;
    else if (const char* h = std::getenv("HOME")) dir = std::string(h) + "/.cache";
    else return std::string();
    return dir + "/opf_admm/tune.txt";
}

void make_parent_dirs(const std::string& path) {
    for (size_t i = 1; i < path.size(); ++i)
        if (path[i] == '/') (void)mkdir(path.substr(0, i).c_str(), 0755);
}

}  // namespace

bool tune_cache_get(const std::string& key, std::vector<int>& vals) {
    std::lock_guard<std::mutex> lk(g_mu);
    const std::string path = cache_path();
    auto it = g_mem.find(path + '\n' + key);
    if (it != g_mem.end()) {
        vals = it->second;
        return true;
    }
    if (path.empty()) return false;
    std::ifstream f(path);
    if (!f) return false;
    bool found = false;
    std::string line;
    while (std::getline(f, line)) {
        const size_t tab = line.find('\t');
        if (tab == std::string::npos || line.compare(0, tab, key) != 0 || tab != key.size()) continue;
        std::istringstream is(line.substr(tab + 1));
        std::vector<int> v;
        int x;
        while (is >> x) v.push_back(x);
        if (!v.empty()) {
            vals = v;
            found = true;
        }
    }
    if (found) g_mem[path + '\n' + key] = vals;
    return found;
}

void tune_cache_put(const std::string& key, const std::vector<int>& vals) {
    std::lock_guard<std::mutex> lk(g_mu);
    const std::string path = cache_path();
    g_mem[path + '\n' + key] = vals;
    if (path.empty()) return;
    make_parent_dirs(path);
    std::ofstream f(path, std::ios::app);
    if (!f) return;
    f << key << '\t';
    for (size_t i = 0; i < vals.size(); ++i) f << (i ? " " : "") << vals[i];
    f << '\n';
}

}  // namespace opf
