// A CPU stand-in for the HIP runtime calls the library's host layer
// (pf_api.cpp) makes, so that its handle logic (streams of the filter
// groups, event fork and join, graph capture, replay and destruction,
// tuning changes, timing events, host copies) runs under AddressSanitizer
// without a GPU.  Device memory is host memory; work runs when issued, or is
// recorded as a node while its stream is captured.  The stream-capture rules
// are checked strictly; a violation prints a line starting with
// "FAKEHIP VIOLATION" and aborts.  Besides the capture rules it tracks
// lifetimes: every op issued on a stream counts as unfinished until the
// host has waited for it (a stream or event synchronisation, followed
// through the event waits that ordered one stream after another), and a
// graph exec may only be destroyed, and a stream only destroyed, once every
// launch on it or op issued to it is finished.  Events are never recorded
// inside a capture (the library keeps its captured graphs free of events).
// Kernel launches come from stub launchers that call fake_kernel(stream).
#include <hip/hip_runtime_api.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <set>
#include <vector>

#define CHECK(c, ...)                                 \
  do {                                                \
    if (!(c)) {                                       \
      fprintf(stderr, "FAKEHIP VIOLATION: " __VA_ARGS__); \
      fprintf(stderr, "\n");                          \
      abort();                                        \
    }                                                 \
  } while (0)

namespace {

struct FGraph;
struct FStream;
// a wait issued as op `at` of its stream on an event recorded after `src_ops`
// ops of stream `src`
struct FWait {
  long at;
  FStream* src;
  long src_ops;
};
struct FStream {
  bool blocking = true;
  bool destroyed = false;
  FGraph* cap = nullptr;  // capture the stream takes part in
  bool origin = false;    // the stream that began that capture
  bool joined = true;     // the origin has waited for this stream's last op
  long ops = 0;           // ops issued (kernels, copies, waits, graph launches)
  long done = 0;          // ops [0, done) known finished by the host
  std::vector<FWait> waits;
};
struct FEvent {
  bool recorded = false, destroyed = false;
  unsigned flags = 0;
  FGraph* cap = nullptr;  // recorded while this capture was open
  FStream* rec_stream = nullptr;
  long rec_ops = -1;      // ops of the recording stream at the record
  double t = 0;
};
struct FGraph {
  bool capturing = true, destroyed = false;
  std::vector<FStream*> streams;
  std::vector<std::function<void()>> nodes;
};
struct FExec {
  bool destroyed = false;
  std::vector<std::function<void()>> nodes;
  std::vector<std::pair<FStream*, long>> launches;  // (stream, op index)
};

// objects are never freed, so a use after destruction is caught
std::set<void*> g_streams, g_events, g_graphs, g_execs;
FStream g_null;
double g_clock = 0;

FStream* S(hipStream_t s) {
  if (!s) return &g_null;
  CHECK(g_streams.count((void*)s), "unknown stream %p", (void*)s);
  FStream* f = (FStream*)s;
  CHECK(!f->destroyed, "use of a destroyed stream");
  return f;
}
FEvent* E(hipEvent_t e) {
  CHECK(g_events.count((void*)e), "unknown event %p", (void*)e);
  FEvent* f = (FEvent*)e;
  CHECK(!f->destroyed, "use of a destroyed event");
  return f;
}
// The host knows ops [0, upto) of f finished; so did whatever those ops
// waited for.
void complete(FStream* f, long upto) {
  if (upto <= f->done) return;
  f->done = upto;
  for (const FWait& w : f->waits)
    if (w.at < upto) complete(w.src, w.src_ops);
}
bool capture_open() {
  for (void* p : g_graphs)
    if (((FGraph*)p)->capturing) return true;
  return false;
}
// one op on stream s: run it now, or record it into the open capture
void op(hipStream_t s, std::function<void()> fn) {
  FStream* f = S(s);
  // the null stream synchronises with every blocking stream: no use while
  // any capture is open
  if (!s) CHECK(!capture_open(), "null-stream work while a capture is open");
  if (f->cap) {
    f->cap->nodes.push_back(std::move(fn));
    if (!f->origin) f->joined = false;
  } else {
    fn();
  }
  f->ops++;
  g_clock += 1;
}

}  // namespace

extern "C" void fake_kernel(hipStream_t s) {
  op(s, [] {});
}

extern "C" {

hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipGetDevicePropertiesR0600(hipDeviceProp_tR0600* p, int) {
  memset(p, 0, sizeof(*p));
  strcpy(p->gcnArchName, "gfx950:sramecc+:xnack-");
  p->multiProcessorCount = 256;
  return hipSuccess;
}
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "error"; }
hipError_t hipGetLastError(void) { return hipSuccess; }

hipError_t hipStreamCreate(hipStream_t* s) {
  FStream* f = new FStream();
  g_streams.insert(f);
  *s = (hipStream_t)f;
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags) {
  FStream* f = new FStream();
  f->blocking = !(flags & hipStreamNonBlocking);
  g_streams.insert(f);
  *s = (hipStream_t)f;
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  CHECK(s, "destroy of the null stream");
  FStream* f = S(s);
  CHECK(!f->cap, "destroy of a stream taking part in a capture");
  CHECK(f->done == f->ops, "destroy of a stream with unfinished work");
  f->destroyed = true;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  FStream* f = S(s);
  CHECK(!f->cap, "synchronize of a capturing stream");
  if (!s) CHECK(!capture_open(), "null-stream synchronize while a capture is open");
  complete(f, f->ops);
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) {
  FEvent* f = new FEvent();
  g_events.insert(f);
  *e = (hipEvent_t)f;
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags) {
  FEvent* f = new FEvent();
  f->flags = flags;
  g_events.insert(f);
  *e = (hipEvent_t)f;
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  E(e)->destroyed = true;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  FEvent* f = E(e);
  FStream* st = S(s);
  if (!s) CHECK(!capture_open(), "event record on the null stream while a capture is open");
  CHECK(!st->cap, "event recorded inside a capture");
  f->recorded = true;
  f->cap = st->cap;
  f->rec_stream = st;
  f->rec_ops = st->ops;
  f->t = g_clock;
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int) {
  FEvent* f = E(e);
  FStream* st = S(s);
  CHECK(f->recorded, "wait on an event never recorded");
  if (f->cap && f->cap->capturing) {
    if (!st->cap) {  // fork: s joins the capture
      CHECK(s, "the null stream joins a capture");
      st->cap = f->cap;
      st->origin = false;
      st->joined = true;
      f->cap->streams.push_back(st);
    } else {
      CHECK(st->cap == f->cap, "wait across two open captures");
      if (st->origin && f->rec_stream != st && f->rec_ops == f->rec_stream->ops)
        f->rec_stream->joined = true;  // join: the origin waits for a side stream's last op
    }
  } else {
    CHECK(!st->cap, "capturing stream waits on an event recorded outside its capture");
    CHECK(!f->cap, "wait on an event recorded inside a capture");
    st->waits.push_back({st->ops, f->rec_stream, f->rec_ops});
    st->ops++;
  }
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
  FEvent* f = E(e);
  CHECK(f->recorded, "synchronize on an event never recorded");
  CHECK(!f->cap, "synchronize on an event recorded inside a capture");
  complete(f->rec_stream, f->rec_ops);
  return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  FEvent* fa = E(a);
  FEvent* fb = E(b);
  CHECK(fa->recorded && fb->recorded, "elapsed time of events never recorded");
  CHECK(!(fa->flags & hipEventDisableTiming) && !(fb->flags & hipEventDisableTiming),
        "elapsed time of an event created without timing");
  CHECK(!fa->cap && !fb->cap, "elapsed time of events recorded inside a capture");
  CHECK(fa->rec_stream->done >= fa->rec_ops && fb->rec_stream->done >= fb->rec_ops,
        "elapsed time of events the host has not waited for");
  *ms = (float)(fb->t - fa->t) * 1e-3f + 1e-3f;
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t s) {
  CHECK(!S(s)->cap, "host copy recorded into a capture");
  op(s, [=] { memcpy(dst, src, n); });
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* dst, int v, size_t n, hipStream_t s) {
  CHECK(!S(s)->cap, "memset recorded into a capture");
  op(s, [=] { memset(dst, v, n); });
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  CHECK(s, "capture on the null stream");
  FStream* f = S(s);
  CHECK(!f->cap, "begin capture on a stream already capturing");
  FGraph* g = new FGraph();
  g_graphs.insert(g);
  f->cap = g;
  f->origin = true;
  f->joined = true;
  g->streams.push_back(f);
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* out) {
  FStream* f = S(s);
  CHECK(f->cap && f->origin, "end capture on a stream that did not begin one");
  FGraph* g = f->cap;
  for (FStream* st : g->streams) CHECK(st->joined, "capture ends with a stream not joined back");
  for (FStream* st : g->streams) {
    st->cap = nullptr;
    st->origin = false;
    st->joined = true;
  }
  g->capturing = false;
  *out = (hipGraph_t)g;
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* ex, hipGraph_t graph, hipGraphNode_t*, char*,
                               size_t) {
  CHECK(g_graphs.count((void*)graph), "instantiate of an unknown graph");
  FGraph* g = (FGraph*)graph;
  CHECK(!g->destroyed && !g->capturing, "instantiate of a destroyed or open graph");
  FExec* x = new FExec();
  x->nodes = g->nodes;
  g_execs.insert(x);
  *ex = (hipGraphExec_t)x;
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t ex, hipStream_t s) {
  CHECK(g_execs.count((void*)ex), "launch of an unknown graph");
  FExec* x = (FExec*)ex;
  CHECK(!x->destroyed, "launch of a destroyed graph");
  FStream* f = S(s);
  CHECK(!f->cap, "graph launch inside a capture");
  if (!s) CHECK(!capture_open(), "graph launch on the null stream while a capture is open");
  for (auto& n : x->nodes) n();
  x->launches.push_back({f, f->ops});
  f->ops++;
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t ex) {
  CHECK(g_execs.count((void*)ex), "destroy of an unknown graph");
  FExec* x = (FExec*)ex;
  CHECK(!x->destroyed, "graph destroyed twice");
  for (auto& l : x->launches)
    CHECK(l.first->done > l.second, "graph exec destroyed while a launch of it may still run");
  x->destroyed = true;
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t graph) {
  CHECK(g_graphs.count((void*)graph), "destroy of an unknown graph");
  FGraph* g = (FGraph*)graph;
  CHECK(!g->destroyed, "graph destroyed twice");
  CHECK(!g->capturing, "destroy of a graph still being captured");
  g->destroyed = true;
  return hipSuccess;
}

}  // extern "C"
