// Tuning classes and the tuning cache file of libperm3.
//
// The cache is plain text, one line per (device, class):
//     <arch> <compute units> <class> key=value ...
// where the keys are the fields of perm_tuning.  Lines for other devices are
// kept untouched when the file is rewritten, so one file can serve several
// kinds of device.
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "perm3.h"
#include "perm3_runtime.h"

namespace perm3 {

const char *const TUNE_CLASS_NAMES[PERM_TUNE_CLASSES] = {"small", "mid", "large", "batch"};

namespace {

struct Field {
    const char *name;
    int32_t perm_tuning::*member;
};

const Field FIELDS[] = {
    {"waves_per_simd", &perm_tuning::waves_per_simd}, {"body_log", &perm_tuning::body_log},
    {"chunk_log_max", &perm_tuning::chunk_log_max},   {"tasks_per_wave", &perm_tuning::tasks_per_wave},
    {"direct_max_n", &perm_tuning::direct_max_n},     {"use_graphs", &perm_tuning::use_graphs},
    {"states_per_lane", &perm_tuning::states_per_lane}, {"body_log_mid", &perm_tuning::body_log_mid},
    {"mid_max_n", &perm_tuning::mid_max_n},           {"max_tasks_log", &perm_tuning::max_tasks_log},
    {"min_task_log", &perm_tuning::min_task_log},     {"queue_task_log", &perm_tuning::queue_task_log},
};

int class_of_name(const std::string &s)
{
    for (int k = 0; k < PERM_TUNE_CLASSES; ++k)
        if (s == TUNE_CLASS_NAMES[k]) return k;
    return -1;
}

// One parsed line: device key, class and tuning (fields not named keep the
// defaults).  False for comments, blank and malformed lines.
bool parse_line(const std::string &line, std::string &arch, int &cus, int &cls, perm_tuning &t)
{
    const std::string body = line.substr(0, line.find('#'));
    std::istringstream in(body);
    std::string cname;
    if (!(in >> arch >> cus >> cname)) return false;
    cls = class_of_name(cname);
    if (cls < 0) return false;
    t = default_tuning();
    std::string kv;
    while (in >> kv) {
        const size_t eq = kv.find('=');
        if (eq == std::string::npos) continue;
        const std::string key = kv.substr(0, eq);
        char *end = nullptr;
        const long v = strtol(kv.c_str() + eq + 1, &end, 10);
        if (!end || *end != '\0' || v < -(1L << 30) || v > (1L << 30)) continue;
        for (const Field &f : FIELDS)
            if (key == f.name) t.*(f.member) = (int32_t)v;
    }
    return true;
}

std::string format_line(const Context &c, int cls)
{
    std::ostringstream o;
    o << c.arch << ' ' << c.cus << ' ' << TUNE_CLASS_NAMES[cls];
    for (const Field &f : FIELDS) o << ' ' << f.name << '=' << c.tunings[cls].*(f.member);
    return o.str();
}

}  // namespace

int cache_apply(Context &c, const char *path)
{
    std::ifstream f(path);
    if (!f) return -1;
    int applied = 0;
    std::string line;
    while (std::getline(f, line)) {
        std::string arch;
        int cus = 0, cls = -1;
        perm_tuning t;
        if (!parse_line(line, arch, cus, cls, t)) continue;
        if (arch != c.arch || cus != c.cus || !tuning_valid(t)) continue;
        c.set_tuning(cls, t, PERM_TUNE_SRC_CACHE);
        ++applied;
    }
    return applied;
}

void load_default_cache(Context &c)
{
    const char *env = getenv("PERM3_TUNING_CACHE");
    if (env) {
        if (*env) (void)cache_apply(c, env);
        return;
    }
    Dl_info info;
    if (!dladdr((void *)&perm_tuning_cache_load, &info) || !info.dli_fname) return;
    std::string dir(info.dli_fname);
    const size_t slash = dir.rfind('/');
    dir = slash == std::string::npos ? std::string(".") : dir.substr(0, slash);
    (void)cache_apply(c, (dir + "/perm3_tuning.txt").c_str());
}

}  // namespace perm3

using namespace perm3;

extern "C" {

int32_t perm_tuning_cache_load(const char *path, int32_t *loaded)
{
    if (!path) return set_error(PERM_EINVAL, "null path");
    Context *c = nullptr;
    int32_t rc = get_context(&c);
    if (rc) return rc;
    std::lock_guard<std::mutex> g(c->mu);
    const int n = cache_apply(*c, path);
    if (n < 0) return set_error(PERM_EINVAL, "cannot read tuning cache %s", path);
    if (loaded) *loaded = n;
    return PERM_OK;
}

int32_t perm_tuning_cache_save(const char *path)
{
    if (!path) return set_error(PERM_EINVAL, "null path");
    Context *c = nullptr;
    int32_t rc = get_context(&c);
    if (rc) return rc;
    std::lock_guard<std::mutex> g(c->mu);
    // keep the lines of other devices and of this device's classes left at the defaults
    std::vector<std::string> keep;
    {
        std::ifstream f(path);
        std::string line;
        while (f && std::getline(f, line)) {
            std::string arch;
            int cus = 0, cls = -1;
            perm_tuning t;
            if (parse_line(line, arch, cus, cls, t) && arch == c->arch && cus == c->cus &&
                c->tune_src[cls] != PERM_TUNE_SRC_DEFAULT)
                continue;
            keep.push_back(line);
        }
    }
    if (keep.empty()) keep.push_back("# perm3 tuning cache: <arch> <compute units> <class> key=value ...");
    for (int k = 0; k < PERM_TUNE_CLASSES; ++k)
        if (c->tune_src[k] != PERM_TUNE_SRC_DEFAULT) keep.push_back(format_line(*c, k));
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream o(tmp, std::ios::trunc);
        if (!o) return set_error(PERM_EINVAL, "cannot write %s", tmp.c_str());
        for (const std::string &l : keep) o << l << '\n';
        if (!o) return set_error(PERM_EINVAL, "cannot write %s", tmp.c_str());
    }
    if (rename(tmp.c_str(), path) != 0) return set_error(PERM_EINVAL, "cannot replace %s", path);
    return PERM_OK;
}

}  // extern "C"
