// On-disk cache of the autotuner's choices (see tune.h).  Lines of the file:
//   <key> <choice> <ms of candidate 0> <ms of candidate 1> ...
// The file is read once per process and path; a store rewrites it through a
// temporary file and a rename, so a reader never sees half a file.
#include "tune.h"

#include <sys/stat.h>
#include <unistd.h>

#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>

namespace hsb {

namespace {

std::mutex g_mu;
std::string g_path;                          // the file the map below was read from
std::map<std::string, std::string> g_lines;  // key -> the rest of its line
bool g_loaded = false;

void load_locked(const std::string &path) {
    if (g_loaded && path == g_path) return;
    g_lines.clear();
    g_path = path;
    g_loaded = true;
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
        std::istringstream ls(line);
        std::string key;
        if (!(ls >> key)) continue;
        std::string rest;
        std::getline(ls, rest);
        g_lines[key] = rest;
    }
}

bool mkdirs(const std::string &dir) {
    if (dir.empty()) return true;
    struct stat st;
    if (stat(dir.c_str(), &st) == 0) return S_ISDIR(st.st_mode);
    const size_t cut = dir.find_last_of('/');
    if (cut != std::string::npos && cut > 0 && !mkdirs(dir.substr(0, cut))) return false;
    return mkdir(dir.c_str(), 0755) == 0 || errno == EEXIST;
}

}  // namespace

std::string tune_cache_path() {
    if (const char *p = std::getenv("HSB_TUNE_CACHE"); p && *p) return p;
    if (const char *x = std::getenv("XDG_CACHE_HOME"); x && *x) return std::string(x) + "/hsb/tune.txt";
    if (const char *h = std::getenv("HOME"); h && *h) return std::string(h) + "/.cache/hsb/tune.txt";
    return "hsb_tune.txt";
}

bool tune_lookup(const std::string &key, int *choice) {
    std::lock_guard<std::mutex> lock(g_mu);
    load_locked(tune_cache_path());
    const auto it = g_lines.find(key);
    if (it == g_lines.end()) return false;
    std::istringstream ls(it->second);
    int c = -1;
    if (!(ls >> c) || c < 0) return false;
    *choice = c;
    return true;
}

bool tune_store(const std::string &key, int choice, const std::vector<double> &ms) {
    std::lock_guard<std::mutex> lock(g_mu);
    const std::string path = tune_cache_path();
    load_locked(path);
    std::ostringstream rest;
    rest << ' ' << choice;
    for (double t : ms) rest << ' ' << t;
    g_lines[key] = rest.str();
    const size_t cut = path.find_last_of('/');
    if (cut != std::string::npos && !mkdirs(path.substr(0, cut))) return false;
    const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
    {
        std::ofstream out(tmp, std::ios::trunc);
        if (!out) return false;
        for (const auto &kv : g_lines) out << kv.first << kv.second << '\n';
        if (!out) return false;
    }
    return std::rename(tmp.c_str(), path.c_str()) == 0;
}

}  // namespace hsb
