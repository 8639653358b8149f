// The library's tuning cache: key -> tokens (choices recorded by the plan
// tuner and the dense split-BF16 tuner).  Kept in memory for the process and,
// when the environment variable ROT_TUNE_CACHE names a file, in that text
// file: one line "key token token ..." per entry, '#' lines are comments.
// The file is read on first use; every new entry rewrites it (through a
// temporary file renamed into place).  Entries whose tokens a user cannot
// parse are treated as absent by that user.
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "rot_internal.h"

namespace rot {
namespace {

std::mutex g_mu;
std::map<std::string, std::vector<std::string>> g_entries;
bool g_loaded = false;

void load_locked() {
    if (g_loaded) return;
    g_loaded = true;
    const char* path = getenv("ROT_TUNE_CACHE");
    if (!path || !*path) return;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        if (line.empty() || line[0] == '#') continue;
        std::istringstream is(line);
        std::string key, tok;
        if (!(is >> key)) continue;
        std::vector<std::string> toks;
        while (is >> tok) toks.push_back(tok);
        if (!toks.empty()) g_entries[key] = toks;
    }
}

void store_locked() {
    const char* path = getenv("ROT_TUNE_CACHE");
    if (!path || !*path) return;
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp);
        f << "# librot tuning cache: key, then the tuner's choices\n";
        for (auto& kv : g_entries) {
            f << kv.first;
            for (auto& t : kv.second) f << ' ' << t;
            f << '\n';
        }
    }
    std::rename(tmp.c_str(), path);
}

}  // namespace

bool tune_get(const std::string& key, std::vector<std::string>* tokens) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    auto it = g_entries.find(key);
    if (it == g_entries.end()) return false;
    *tokens = it->second;
    return true;
}

void tune_put(const std::string& key, const std::vector<std::string>& tokens) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    g_entries[key] = tokens;
    store_locked();
}

}  // namespace rot
