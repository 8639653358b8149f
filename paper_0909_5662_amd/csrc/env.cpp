// Run-time switches read from the environment (looked up on every use, so a
// process can change them between calls):
//   ROT_LOG_LEVEL    0 (default) silent; 1 failures are also written to
//                    stderr; 2 also plan and execution-path decisions
//   ROT_TRACE        1: every entry point is bracketed by a roctx range named
//                    after it (the roctx library is loaded on first use; a
//                    profiler such as rocprofv3 --marker-trace records them)
//   ROT_DISABLE_GRAPH  1: plans issue their launches directly instead of
//                    capturing a hipGraph (as with ROT_PLAN_NO_GRAPH)
//   ROT_SCHEDULE     static | dynamic: every plan size class uses that
//                    schedule whatever the tuner or its cache chose
#include <dlfcn.h>

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "rot_internal.h"

namespace rot {

int log_level() {
    const char* e = getenv("ROT_LOG_LEVEL");
    return e ? atoi(e) : 0;
}

void log_msg(int level, const char* fmt, ...) {
    if (log_level() < level) return;
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    fprintf(stderr, "[librot] %s\n", buf);
}

bool graphs_disabled() {
    const char* e = getenv("ROT_DISABLE_GRAPH");
    return e && *e && strcmp(e, "0") != 0;
}

int forced_schedule() {
    const char* e = getenv("ROT_SCHEDULE");
    if (!e) return -1;
    if (!strcmp(e, "static")) return 0;
    if (!strcmp(e, "dynamic")) return 1;
    return -1;
}

namespace {

typedef int (*push_fn)(const char*);
typedef int (*pop_fn)();
std::once_flag g_roctx_once;
push_fn g_push = nullptr;
pop_fn g_pop = nullptr;

void load_roctx() {
    for (const char* name : {"librocprofiler-sdk-roctx.so.1", "librocprofiler-sdk-roctx.so", "libroctx64.so.4",
                             "libroctx64.so"}) {
        void* h = dlopen(name, RTLD_NOW | RTLD_LOCAL);
        if (!h) continue;
        push_fn p = reinterpret_cast<push_fn>(dlsym(h, "roctxRangePushA"));
        pop_fn q = reinterpret_cast<pop_fn>(dlsym(h, "roctxRangePop"));
        if (p && q) {
            g_push = p;
            g_pop = q;
            return;
        }
        dlclose(h);
    }
    log_msg(1, "ROT_TRACE: no roctx library found; ranges are not recorded");
}

}  // namespace

TraceRange::TraceRange(const char* name) {
    const char* e = getenv("ROT_TRACE");
    if (!e || !*e || !strcmp(e, "0")) return;
    std::call_once(g_roctx_once, load_roctx);
    if (g_push && g_pop) {
        g_push(name);
        active_ = true;
    }
}

TraceRange::~TraceRange() {
    if (active_) g_pop();
}

}  // namespace rot
