// A CPU stand-in for the HIP runtime functions libmppi calls, for testing the library's host
// logic (contexts, layouts, the serving runtime's batching, admission and graph bookkeeping)
// without a GPU.  Device allocations are addresses in a PROT_NONE region, so any host
// dereference of device memory faults at once; their contents live in a shadow mapping that
// the copy and memset functions use, and every copy is checked against the live allocation it
// touches.  Kernels do not run.  Streams and events are bookkeeping (work is complete when
// enqueued), graphs record their memcpy nodes and execute them at launch, and node updates
// check that the node exists and has the right kind.  Test infrastructure only.
#include <hip/hip_runtime_api.h>
#include <sys/mman.h>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>
#include <map>

static const size_t kSpan = size_t(64) << 30;
static char *g_dev = nullptr, *g_shadow = nullptr;
static size_t g_top = 0;
static std::mutex g_mu;
static std::map<uintptr_t, size_t> g_live;

static void init_regions() {
  if (g_dev) return;
  g_dev = (char *)mmap(nullptr, kSpan, PROT_NONE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
  g_shadow = (char *)mmap(nullptr, kSpan, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
  if (g_dev == MAP_FAILED || g_shadow == MAP_FAILED) { fprintf(stderr, "mock: mmap failed\n"); abort(); }
}
static bool is_dev(const void *p) { return g_dev && (const char *)p >= g_dev && (const char *)p < g_dev + kSpan; }
static void *shadow(const void *p) { return g_shadow + ((const char *)p - g_dev); }
static void *host_view(const void *p) { return is_dev(p) ? shadow(p) : (void *)p; }
static void check_dev_range(const void *p, size_t n, const char *what) {
  if (!is_dev(p)) return;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_live.upper_bound((uintptr_t)p);
  if (it == g_live.begin()) { fprintf(stderr, "mock: %s of %zu B at unallocated device address %p\n", what, n, p); abort(); }
  --it;
  if ((uintptr_t)p + n > it->first + it->second) {
    fprintf(stderr, "mock: %s of %zu B at %p overruns the allocation [%p, +%zu)\n", what, n, p, (void *)it->first, it->second);
    abort();
  }
}
static void mcopy(void *dst, const void *src, size_t n) {
  check_dev_range(dst, n, "copy to");
  check_dev_range(src, n, "copy from");
  std::memmove(host_view(dst), host_view(src), n);
}

struct MockGraph {
  struct Node { int kind; void *dst; const void *src; size_t n; };   // kind 0 kernel, 1 memcpy
  std::vector<Node> nodes;
};
static MockGraph g_capture;          // stream capture: nothing recorded (kernels only)

extern "C" {
void **__hipRegisterFatBinary(const void *) { static void *h[4]; return h; }
void __hipRegisterFunction(void **, const void *, char *, const char *, unsigned, void *, void *, void *, void *, int *) {}
void __hipRegisterVar(void **, void *, char *, char *, int, size_t, int, int) {}
void __hipUnregisterFatBinary(void **) {}
}
static dim3 g_cg, g_cb; static size_t g_cs; static hipStream_t g_cst;
hipError_t __hipPushCallConfiguration(dim3 g, dim3 b, size_t s, hipStream_t st) { g_cg = g; g_cb = b; g_cs = s; g_cst = st; return hipSuccess; }
hipError_t __hipPopCallConfiguration(dim3 *g, dim3 *b, size_t *s, hipStream_t *st) { *g = g_cg; *b = g_cb; *s = g_cs; *st = g_cst; return hipSuccess; }
hipError_t hipLaunchKernel(const void *, dim3, dim3, void **, size_t, hipStream_t) { return hipSuccess; }
hipError_t hipExtLaunchKernel(const void *, dim3, dim3, void **, size_t, hipStream_t, hipEvent_t, hipEvent_t, int) { return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t *e) { *e = (hipEvent_t)malloc(16); return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { *e = (hipEvent_t)malloc(16); return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) { free(e); return hipSuccess; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) { *ms = 0.f; return hipSuccess; }
hipError_t hipEventQuery(hipEvent_t) { return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipMalloc(void **p, size_t n) {
  init_regions();
  std::lock_guard<std::mutex> lk(g_mu);
  size_t a = (g_top + 255) & ~size_t(255);
  if (a + n > kSpan) return hipErrorOutOfMemory;
  g_top = a + (n ? n : 1);
  *p = g_dev + a;
  g_live[(uintptr_t)*p] = n;
  return hipSuccess;
}
hipError_t hipFree(void *p) {
  if (!p) return hipSuccess;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_live.find((uintptr_t)p);
  if (it == g_live.end()) { fprintf(stderr, "mock: hipFree of %p, not a live allocation\n", p); abort(); }
  g_live.erase(it);
  return hipSuccess;
}
hipError_t hipHostMalloc(void **p, size_t n, unsigned) { *p = malloc(n); return *p ? hipSuccess : hipErrorOutOfMemory; }
hipError_t hipHostFree(void *p) { free(p); return hipSuccess; }
hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) { mcopy(d, s, n); return hipSuccess; }
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind, hipStream_t) { mcopy(d, s, n); return hipSuccess; }
hipError_t hipMemsetAsync(void *d, int v, size_t n, hipStream_t) { check_dev_range(d, n, "memset"); memset(host_view(d), v, n); return hipSuccess; }
hipError_t hipFuncSetAttribute(const void *, hipFuncAttribute, int) { return hipSuccess; }
hipError_t hipGetDeviceCount(int *n) { *n = 1; return hipSuccess; }
hipError_t hipSetDevice(int) { return hipSuccess; }
const char *hipGetErrorString(hipError_t) { return "mock error"; }
hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipGetSymbolAddress(void **p, const void *) { return hipMalloc(p, size_t(8) << 20); }
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) { *s = (hipStream_t)malloc(16); return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t s) { free(s); return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipSuccess; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g) { *g = (hipGraph_t) new MockGraph(); return hipSuccess; }
hipError_t hipGraphCreate(hipGraph_t *g, unsigned) { *g = (hipGraph_t) new MockGraph(); return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t g) { delete (MockGraph *)g; return hipSuccess; }
static hipGraphNode_t add_node(hipGraph_t g, MockGraph::Node nd) {
  auto *G = (MockGraph *)g;
  G->nodes.push_back(nd);
  return (hipGraphNode_t)(uintptr_t)G->nodes.size();      // 1-based index
}
hipError_t hipGraphAddKernelNode(hipGraphNode_t *n, hipGraph_t g, const hipGraphNode_t *, size_t, const hipKernelNodeParams *p) {
  if (!p || !p->func || !p->kernelParams) { fprintf(stderr, "mock: kernel node without function or args\n"); abort(); }
  *n = add_node(g, {0, nullptr, nullptr, 0});
  return hipSuccess;
}
hipError_t hipGraphAddMemcpyNode1D(hipGraphNode_t *n, hipGraph_t g, const hipGraphNode_t *, size_t, void *d, const void *s, size_t c, hipMemcpyKind) {
  *n = add_node(g, {1, d, s, c});
  return hipSuccess;
}
struct MockExec { MockGraph *g; std::vector<MockGraph::Node> nodes; };
hipError_t hipGraphInstantiate(hipGraphExec_t *e, hipGraph_t g, hipGraphNode_t *, char *, size_t) {
  auto *x = new MockExec{(MockGraph *)g, ((MockGraph *)g)->nodes};
  *e = (hipGraphExec_t)x;
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t e) { delete (MockExec *)e; return hipSuccess; }
hipError_t hipGraphExecKernelNodeSetParams(hipGraphExec_t e, hipGraphNode_t n, const hipKernelNodeParams *p) {
  auto *x = (MockExec *)e;
  const size_t i = (size_t)(uintptr_t)n;
  if (i == 0 || i > x->nodes.size() || x->nodes[i - 1].kind != 0) { fprintf(stderr, "mock: bad kernel node\n"); abort(); }
  if (!p || !p->func || !p->kernelParams || p->gridDim.x == 0) { fprintf(stderr, "mock: bad kernel params\n"); abort(); }
  return hipSuccess;
}
hipError_t hipGraphExecMemcpyNodeSetParams1D(hipGraphExec_t e, hipGraphNode_t n, void *d, const void *s, size_t c, hipMemcpyKind) {
  auto *x = (MockExec *)e;
  const size_t i = (size_t)(uintptr_t)n;
  if (i == 0 || i > x->nodes.size() || x->nodes[i - 1].kind != 1) { fprintf(stderr, "mock: bad memcpy node\n"); abort(); }
  x->nodes[i - 1].dst = d; x->nodes[i - 1].src = s; x->nodes[i - 1].n = c;
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t) {
  for (auto &nd : ((MockExec *)e)->nodes)
    if (nd.kind == 1) mcopy(nd.dst, nd.src, nd.n);
  return hipSuccess;
}
