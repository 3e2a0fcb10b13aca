// Error state and small C-ABI entry points.
#include <cstdarg>
#include <cstdio>

#include "common.h"

namespace {
thread_local char g_err[1024] = "";
// allocator of the current entry point (NULL: hipMalloc / hipFree) and the stream it is given
thread_local const qsd_allocator *g_alloc = nullptr;
thread_local void *g_alloc_stream = nullptr;
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

AllocScope::AllocScope(const qsd_allocator *a, void *stream) : prev_a(g_alloc), prev_s(g_alloc_stream) {
    g_alloc = (a && a->alloc && a->free) ? a : nullptr;
    g_alloc_stream = stream;
}

AllocScope::~AllocScope() {
    g_alloc = prev_a;
    g_alloc_stream = prev_s;
}

bool custom_allocator() { return g_alloc != nullptr; }

void *raw_alloc(size_t bytes) {
    if (bytes == 0) bytes = 1;
    if (g_alloc) return g_alloc->alloc(g_alloc->ctx, bytes, g_alloc_stream);
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

void raw_free(void *p) {
    if (!p) return;
    if (g_alloc)
        g_alloc->free(g_alloc->ctx, p, g_alloc_stream);
    else
        (void)hipFree(p);
}

}  // namespace qsd

extern "C" const char *qsd_last_error(void) { return g_err; }

extern "C" int qsd_version(void) { return 100; }

extern "C" int32_t qsd_max_qubits(void) { return qsd::kMaxWords * 64; }
