// Error state and small C-ABI entry points.
#include <cstdarg>
#include <cstdio>

#include "common.h"

namespace {
thread_local char g_err[1024] = "";
}

namespace qsd {

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_err[0] = '\0'; }

}  // namespace qsd

extern "C" const char *qsd_last_error(void) { return g_err; }

extern "C" int qsd_version(void) { return 100; }

extern "C" int32_t qsd_max_qubits(void) { return qsd::kMaxWords * 64; }
