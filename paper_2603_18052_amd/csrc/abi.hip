// C-ABI entry points of liblindblad.so: validation, workspace, dispatch.
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "lb_internal.hpp"
#include "chain.hpp"

namespace lb {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int status, const std::string &msg) {
    g_last_error = msg;
    return status;
}

int check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(LB_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    return LB_OK;
}

// ------------------------------------------------------------ workspace
void ws_begin(Workspace *ws) { ws->used = 0; }

int ws_ensure(Workspace *ws, size_t bytes) {
    bytes = align256(bytes);
    if (ws->used + bytes <= ws->size) return LB_OK;
    if (ws->used != 0)
        return fail(LB_ENOMEM, "workspace: nested request of " + std::to_string(bytes) +
                                   " bytes exceeds the reservation");
    if (bytes > ws->cap)
        return fail(LB_ENOMEM, "workspace: need " + std::to_string(bytes) + " bytes, cap is " +
                                   std::to_string(ws->cap));
    if (ws->base) {
        LB_HIP(hipDeviceSynchronize());
        LB_HIP(hipFree(ws->base));
        ws->base = nullptr;
        ws->size = 0;
    }
    size_t grow = bytes + bytes / 4;
    if (grow > ws->cap) grow = ws->cap;
    void *p = nullptr;
    if (hipMalloc(&p, grow) != hipSuccess) {
        (void)hipGetLastError();
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return fail(LB_ENOMEM, "workspace: hipMalloc of " + std::to_string(bytes) + " bytes failed");
        }
        grow = bytes;
    }
    ws->base = static_cast<char *>(p);
    ws->size = grow;
    return LB_OK;
}

void *ws_take(Workspace *ws, size_t bytes) {
    size_t b = align256(bytes);
    void *p = ws->base + ws->used;
    ws->used += b;
    return p;
}

static std::mutex g_ws_mutex;
static std::map<int, Workspace *> g_default_ws;

Workspace *ws_resolve(lb_workspace *ws) {
    if (ws) return reinterpret_cast<Workspace *>(ws);
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lock(g_ws_mutex);
    Workspace *&w = g_default_ws[dev];
    if (!w) {
        w = new Workspace();
        w->cap = size_t(64) << 30;
        w->device = dev;
    }
    return w;
}

}  // namespace lb

using namespace lb;

extern "C" {

const char *lindblad_last_error(void) { return g_last_error.c_str(); }

int lb_workspace_create(size_t max_bytes, lb_workspace **ws) {
    if (!ws) return fail(LB_EINVAL, "lb_workspace_create: ws is NULL");
    Workspace *w = new Workspace();
    w->cap = max_bytes;
    (void)hipGetDevice(&w->device);
    *ws = reinterpret_cast<lb_workspace *>(w);
    return LB_OK;
}

int lb_workspace_destroy(lb_workspace *ws) {
    if (!ws) return LB_OK;
    Workspace *w = reinterpret_cast<Workspace *>(ws);
    if (w->base) {
        LB_HIP(hipDeviceSynchronize());
        LB_HIP(hipFree(w->base));
    }
    delete w;
    return LB_OK;
}

size_t lb_workspace_bytes(const lb_workspace *ws) {
    return ws ? reinterpret_cast<const Workspace *>(ws)->size : 0;
}

}  // extern "C"
