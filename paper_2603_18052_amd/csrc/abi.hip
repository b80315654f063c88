// C-ABI entry points of liblindblad.so: validation, workspace, dispatch.
#include <cmath>
#include <cstring>
#include <functional>
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

int set_max_lds(const void *kernel, size_t bytes) {
    int dev = 0;
    LB_HIP(hipGetDevice(&dev));
    static std::mutex mu;
    static std::map<std::pair<int, const void *>, size_t> done;
    std::lock_guard<std::mutex> lock(mu);
    size_t &have = done[{dev, kernel}];
    if (have >= bytes) return LB_OK;
    LB_HIP(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    have = bytes;
    return LB_OK;
}

// ------------------------------------------------------------ workspace
void ws_begin(Workspace *ws, hipStream_t s) {
    ws->used = 0;
    ws->stream = s;
}

int ws_ensure(Workspace *ws, size_t bytes) {
    bytes = align256(bytes);
    if (ws->used + bytes <= ws->size) return LB_OK;
    if (ws->fixed)
        return fail(LB_ENOMEM, "workspace: need " + std::to_string(ws->used + bytes) +
                                   " bytes of the fixed scratch of " + std::to_string(ws->size));
    if (ws->used != 0)
        return fail(LB_ENOMEM, "workspace: nested request of " + std::to_string(bytes) +
                                   " bytes exceeds the reservation");
    if (bytes > ws->cap)
        return fail(LB_ENOMEM, "workspace: need " + std::to_string(bytes) + " bytes, cap is " +
                                   std::to_string(ws->cap));
    // stream-ordered: the old buffer is released after the work already
    // enqueued on this call's stream, the new one is valid from here on it
    if (ws->base) {
        LB_HIP(hipFreeAsync(ws->base, ws->stream));
        ws->base = nullptr;
        ws->size = 0;
    }
    size_t grow = bytes + bytes / 4;
    if (grow > ws->cap) grow = ws->cap;
    void *p = nullptr;
    if (hipMallocAsync(&p, grow, ws->stream) != hipSuccess) {
        (void)hipGetLastError();
        if (hipMallocAsync(&p, bytes, ws->stream) != hipSuccess) {
            (void)hipGetLastError();
            return fail(LB_ENOMEM, "workspace: hipMallocAsync of " + std::to_string(bytes) + " bytes failed");
        }
        grow = bytes;
    }
    ws->base = static_cast<char *>(p);
    ws->size = grow;
    ws->alloc_stream = ws->stream;
    return LB_OK;
}

void *ws_take(Workspace *ws, size_t bytes) {
    size_t b = align256(bytes);
    void *p = ws->base + ws->used;
    ws->used += b;
    return p;
}

// ------------------------------------------------------- graph replay
// Steps [0, kGraphSteps) are captured once per call on a private stream of the
// current device (created on first use, default priority) and the executable
// graph is replayed on the caller's stream.  An executable graph is destroyed
// only once an event recorded after its last replay has completed (checked on
// later calls), so nothing in flight is ever freed.
namespace {
struct Retired {
    hipGraphExec_t exec;
    hipGraph_t graph;
    hipEvent_t done;
};
std::mutex g_graph_mu;
std::map<int, hipStream_t> g_capture_stream;
std::vector<Retired> g_retired;

void reap_graphs() {  // caller holds g_graph_mu
    for (size_t i = 0; i < g_retired.size();) {
        if (hipEventQuery(g_retired[i].done) == hipSuccess) {
            (void)hipGraphExecDestroy(g_retired[i].exec);
            (void)hipGraphDestroy(g_retired[i].graph);
            (void)hipEventDestroy(g_retired[i].done);
            g_retired[i] = g_retired.back();
            g_retired.pop_back();
        } else {
            (void)hipGetLastError();  // hipErrorNotReady is not an error here
            ++i;
        }
    }
}
}  // namespace

int run_steps(long long nsteps, bool graph, const std::function<int(long long, hipStream_t)> &step, hipStream_t s) {
    // the last step is always launched directly (it may differ, e.g. write the result)
    const long long reps = graph && nsteps > 0 ? (nsteps - 1) / kGraphSteps : 0;
    long long t = 0;
    if (reps >= 2) {
        std::lock_guard<std::mutex> lock(g_graph_mu);
        reap_graphs();
        int dev = 0;
        LB_HIP(hipGetDevice(&dev));
        hipStream_t &cs = g_capture_stream[dev];
        if (!cs) LB_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        LB_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        int st = LB_OK;
        for (long long k = 0; k < kGraphSteps && st == LB_OK; ++k) st = step(k, cs);
        const hipError_t ce = hipStreamEndCapture(cs, &g);
        if (st != LB_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (ce != hipSuccess) return fail(LB_EHIP, std::string("graph capture: ") + hipGetErrorString(ce));
        if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(g);
            return fail(LB_EHIP, "graph instantiation failed");
        }
        hipEvent_t done = nullptr;
        st = hipEventCreateWithFlags(&done, hipEventDisableTiming) == hipSuccess ? LB_OK
                                                                                : fail(LB_EHIP, "hipEventCreate failed");
        for (long long r = 0; r < reps && st == LB_OK; ++r)
            if (hipGraphLaunch(ge, s) != hipSuccess) st = fail(LB_EHIP, "hipGraphLaunch failed");
        if (st == LB_OK && hipEventRecord(done, s) != hipSuccess) st = fail(LB_EHIP, "hipEventRecord failed");
        if (st != LB_OK) {  // nothing safe to free without waiting
            (void)hipStreamSynchronize(s);
            (void)hipGraphExecDestroy(ge);
            (void)hipGraphDestroy(g);
            if (done) (void)hipEventDestroy(done);
            return st;
        }
        g_retired.push_back({ge, g, done});
        t = reps * kGraphSteps;
    }
    for (; t < nsteps; ++t) LB_TRY(step(t, s));
    return LB_OK;
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
        LB_HIP(hipFreeAsync(w->base, w->alloc_stream));
        LB_HIP(hipDeviceSynchronize());
    }
    delete w;
    return LB_OK;
}

size_t lb_workspace_bytes(const lb_workspace *ws) {
    return ws ? reinterpret_cast<const Workspace *>(ws)->size : 0;
}

}  // extern "C"
