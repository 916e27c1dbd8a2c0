// Launch-sequence graphs: a sequence of kernel launches is captured once per
// exact argument set on a private capture stream, instantiated, and replayed
// on the caller's stream with one hipGraphLaunch (small LRU cache).
#pragma once

#include <initializer_list>
#include <string>

#include "internal.hpp"

namespace gdgs {

class KeyBuilder {
   public:
    template <typename T>
    KeyBuilder& add(const T& v) {
        s_.append(reinterpret_cast<const char*>(&v), sizeof(T));
        return *this;
    }
    KeyBuilder& tag(const char* t) {
        s_.append(t);
        s_.push_back('\0');
        return *this;
    }
    void s_append(const char* t) { tag(t); }
    const std::string& str() const { return s_; }

   private:
    std::string s_;
};

// Defined in api.hip.
hipGraphExec_t graph_find(const std::string& key);
void graph_put(const std::string& key, hipGraphExec_t exec);
int& graphs_flag();
// gdgs_set_channel_streams: 0 runs every Poisson launch over all three
// channels on the caller's stream
int& channel_streams_flag();
hipStream_t capture_stream(int dev);
bool timer_active(const char* name);

// Two helper streams and fork/join events bound to a caller stream (created
// on first use, per thread; kept until the process ends).  false when they
// cannot be created or the environment sets GDGS_CHANNEL_STREAMS=0 (then the
// solve runs all channels in each launch on the caller's stream).
struct ChannelStreams {
    hipStream_t aux[2];
    hipEvent_t fork;
    hipEvent_t join[2];
};
bool channel_streams(hipStream_t st, ChannelStreams* out);

// Key parts shared by the entry points (defined in api.hip).
void add_plan(KeyBuilder& kb, const MgPlan& p);
void add_proj(KeyBuilder& kb, const gdgs_proj& p);
void add_bins(KeyBuilder& kb, const gdgs_bins& b);

// Enqueue `enqueue(stream)` through the graph cache.  Direct launches instead
// when graphs are off, when the stream is itself being captured, or when one
// of the `timed` kernels has an active timer (events recorded as graph nodes
// do not reliably bracket the kernel they surround).
template <typename F>
gdgs_status with_graph(KeyBuilder& kb, hipStream_t st, F&& enqueue,
                       std::initializer_list<const char*> timed = {}) {
    for (const char* n : timed)
        if (timer_active(n)) return enqueue(st);
    if (!graphs_flag()) return enqueue(st);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) {
        (void)hipGetLastError();
        return enqueue(st);
    }
    if (cs != hipStreamCaptureStatusNone) return enqueue(st);
    int dev = 0;
    GDGS_HIP_TRY(hipGetDevice(&dev));
    kb.add(dev);
    hipGraphExec_t exec = graph_find(kb.str());
    if (!exec) {
        hipStream_t cap = capture_stream(dev);
        if (!cap) return enqueue(st);
        GDGS_HIP_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
        const gdgs_status s = enqueue(cap);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(cap, &g);
        if (s != GDGS_OK) {
            if (g) (void)hipGraphDestroy(g);
            return s;
        }
        if (e != hipSuccess || g == nullptr) {
            set_error("graph capture failed: %s", hipGetErrorString(e));
            return GDGS_ERR_HIP;
        }
        if (log_level() >= 2) {
            size_t nodes = 0;
            (void)hipGraphGetNodes(g, nullptr, &nodes);
            log_msg(2, "captured graph \"%s\": %zu nodes", kb.str().c_str(), nodes);
        }
        const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            set_error("graph instantiation failed: %s", hipGetErrorString(ei));
            return GDGS_ERR_HIP;
        }
        graph_put(kb.str(), exec);
    }
    GDGS_HIP_TRY(hipGraphLaunch(exec, st));
    return GDGS_OK;
}

}  // namespace gdgs
