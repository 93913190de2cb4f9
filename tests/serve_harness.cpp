// serve_harness.cpp -- host-only check of the batch bookkeeping of
// csrc/serve.cpp (lbm_step_many's cache of run tables, block maps and
// graphs; lbm_step_many_noalloc's fixed array), built with AddressSanitizer
// against a stub HIP runtime and stub kernel launchers that run on the CPU.
//
// The stubs keep "device memory" in host allocations and track every
// allocation, event, stream, graph and graph executable; each call checks
// that what it is handed is alive (an event, stream or graph used after
// destruction aborts, as does a copy or launch that touches freed memory),
// and every launch checks its run table and block map: each block names a
// run of the table, a block of that run's grid, and a run whose buffers are
// still allocated.  The driver creates, steps, re-seeds and destroys fake
// runs in a seeded random order, with the caller's stream or a run's own,
// and runs the graph replays and LRU evictions of the cache.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <random>
#include <set>
#include <string>
#include <vector>

#include "sim.h"

using namespace ptlbm;

#define CHECK(c, ...)                                                   \
    do {                                                                \
        if (!(c)) {                                                     \
            std::fprintf(stderr, "harness: " __VA_ARGS__);              \
            std::fprintf(stderr, " (%s:%d)\n", __FILE__, __LINE__);     \
            std::abort();                                               \
        }                                                               \
    } while (0)

namespace {

struct Obj { int kind; };   // fake runtime objects (never dereferenced by the library)
std::set<void*> g_streams, g_events, g_graphs, g_execs;
std::map<char*, size_t> g_mem;      // live "device" allocations
std::set<const lbm_sim*> g_live;    // live runs
char* g_symbol_dev = nullptr;       // the device copy of serve.cpp's fixed array
const void* g_symbol_host = nullptr;
size_t g_symbol_size = 0;
long g_launches = 0, g_blocks_checked = 0;

struct Launch {   // one recorded kernel launch
    bool batch;
    int k;
    RunStep one;
    BatchLaunch b;
};
std::map<void*, std::vector<Launch>> g_capture;   // stream -> launches being captured
std::map<void*, std::vector<Launch>> g_graph_body, g_exec_body;

bool in_memory(const void* p, size_t n) {
    const char* c = (const char*)p;
    if (g_symbol_dev && c >= g_symbol_dev && c + n <= g_symbol_dev + g_symbol_size) return true;
    auto it = g_mem.upper_bound((char*)c);
    if (it == g_mem.begin()) return false;
    --it;
    return c >= it->first && c + n <= it->first + it->second;
}

const lbm_sim* owner_of(const void* base) {
    for (const lbm_sim* h : g_live)
        if (h->base == base) return h;
    return nullptr;
}

void check_runstep(const RunStep& R) {
    const lbm_sim* h = owner_of(R.A[0]);
    CHECK(h != nullptr, "launch on the buffers of a destroyed run");
    CHECK(in_memory(R.A[0], 64), "run buffers freed");
}

void execute(const Launch& L) {
    ++g_launches;
    if (!L.batch) {
        check_runstep(L.one);
        return;
    }
    const int c = grid_class(L.k);
    const BatchLaunch& b = L.b;
    const RunStep* tab = L.k == SK_COLLECT ? b.tab_next : b.tab;
    CHECK(b.nblk[c] > 0, "empty batched grid launched");
    CHECK(in_memory(b.bmap[c], (size_t)b.nblk[c] * sizeof(uint2)), "block map not in live memory");
    for (unsigned m = 0; m < b.nblk[c]; ++m) {
        const uint2 e = b.bmap[c][m];
        CHECK(in_memory(tab + e.x, sizeof(RunStep)), "run table entry %u not in live memory", e.x);
        const RunStep& R = tab[e.x];
        CHECK(e.y < run_blocks(c, R.lp), "block %u beyond run %u's grid", e.y, e.x);
        check_runstep(R);
        ++g_blocks_checked;
    }
}

void record(void* s, const Launch& L) {
    CHECK(g_streams.count(s), "launch on a destroyed stream");
    auto it = g_capture.find(s);
    if (it != g_capture.end()) it->second.push_back(L);
    else execute(L);   // the stub runs work at once, in stream order
}

}  // namespace

// ------------------------------------------------------- stub HIP runtime ----
extern "C" {
void** __hipRegisterFatBinary(const void*) {
    static void* m = nullptr;
    return &m;
}
void __hipUnregisterFatBinary(void**) {}
void __hipRegisterVar(void**, void* var, char*, char*, int, size_t size, int, int) {
    g_symbol_host = var;
    g_symbol_size = size;
}
char harness_fatbin_placeholder[16];
}

hipError_t hipGetDevice(int* d) {
    *d = 0;
    return hipSuccess;
}
const char* hipGetErrorString(hipError_t) { return "stub error"; }
hipError_t hipGetSymbolAddress(void** p, const void* sym) {
    CHECK(sym == g_symbol_host && g_symbol_size > 0, "unknown symbol");
    if (!g_symbol_dev) g_symbol_dev = (char*)std::calloc(1, g_symbol_size);
    *p = g_symbol_dev;
    return hipSuccess;
}
hipError_t hipMalloc(void** p, size_t n) {
    char* c = (char*)std::malloc(n ? n : 1);
    g_mem[c] = n;
    *p = c;
    return hipSuccess;
}
hipError_t hipFree(void* p) {
    if (!p) return hipSuccess;
    CHECK(g_mem.erase((char*)p) == 1, "hipFree of memory not allocated");
    std::free(p);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t s) {
    CHECK(g_streams.count(s), "copy on a destroyed stream");
    CHECK(in_memory(dst, n), "copy into memory that is not allocated");
    std::memcpy(dst, src, n);
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
    CHECK(g_streams.count(s), "synchronize of a destroyed stream");
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) {
    void* o = new Obj{1};
    g_events.insert(o);
    *e = (hipEvent_t)o;
    return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
    CHECK(g_events.erase(e) == 1, "destroy of a destroyed event");
    delete (Obj*)e;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
    CHECK(g_events.count(e), "record of a destroyed event");
    CHECK(g_streams.count(s), "record on a destroyed stream");
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
    CHECK(g_events.count(e), "wait for a destroyed event");
    return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
    CHECK(g_events.count(e), "stream wait on a destroyed event");
    CHECK(g_streams.count(s), "wait on a destroyed stream");
    return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
    CHECK(g_streams.count(s), "capture on a destroyed stream");
    CHECK(!g_capture.count(s), "nested capture");
    g_capture[s] = {};
    return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
    CHECK(g_capture.count(s), "end of a capture that did not begin");
    void* o = new Obj{2};
    g_graphs.insert(o);
    g_graph_body[o] = g_capture[s];
    g_capture.erase(s);
    *g = (hipGraph_t)o;
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
    CHECK(g_graphs.count(g), "instantiate of a destroyed graph");
    void* o = new Obj{3};
    g_execs.insert(o);
    g_exec_body[o] = g_graph_body[g];
    *x = (hipGraphExec_t)o;
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
    CHECK(g_graphs.erase(g) == 1, "destroy of a destroyed graph");
    g_graph_body.erase(g);
    delete (Obj*)g;
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
    CHECK(g_execs.erase(x) == 1, "destroy of a destroyed graph executable");
    g_exec_body.erase(x);
    delete (Obj*)x;
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s) {
    CHECK(g_execs.count(x), "launch of a destroyed graph executable");
    CHECK(g_streams.count(s), "graph launch on a destroyed stream");
    for (const Launch& L : g_exec_body[x]) execute(L);
    return hipSuccess;
}

// ---------------------------------------------- stub library internals ----
namespace ptlbm {
int fail(lbm_sim* h, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (h) h->err = buf;
    return code;
}
int hip_fail(lbm_sim* h, hipError_t, const char* what) { return fail(h, LBM_EDEVICE, "%s", what); }
RunStep make_runstep(const lbm_sim* h, int c, int r, int bp) {
    CHECK(g_live.count(h), "run table of a destroyed run");
    RunStep R{};
    R.lp = h->d.lp;
    R.parity = c;
    for (int i = 0; i < 14; ++i) R.A[i] = R.B[i] = h->base;
    R.status = (unsigned*)(h->base + r * 8 + bp);
    return R;
}
unsigned run_blocks(int c, const LP& lp) {
    if (c == GC_LAT) return (unsigned)(((size_t)lp.pitch * lp.ny + 255) / 256);
    if (c == GC_PASS) return (unsigned)lp.np;
    return (unsigned)((lp.np + 3) / 4);
}
size_t links_block_lds(const LP&) { return 4096; }
hipError_t launch_step(int k, const RunStep& R, int, hipStream_t st) {
    Launch L{};
    L.batch = false;
    L.k = k;
    L.one = R;
    record(st, L);
    return hipSuccess;
}
hipError_t launch_step_batch(int k, const BatchLaunch& b, hipStream_t st) {
    if (b.nblk[grid_class(k)] == 0) return hipSuccess;
    Launch L{};
    L.batch = true;
    L.k = k;
    L.b = b;
    record(st, L);
    return hipSuccess;
}
}  // namespace ptlbm

// ------------------------------------------------------------- driver ----
namespace {

hipStream_t new_stream() {
    void* o = new Obj{0};
    g_streams.insert(o);
    return (hipStream_t)o;
}
void destroy_stream(hipStream_t s) {
    CHECK(g_streams.erase(s) == 1, "destroy of a destroyed stream");
    delete (Obj*)s;
}

lbm_sim* new_run(std::mt19937_64& rng) {
    lbm_sim* h = new lbm_sim();
    h->p.nx = 16 + (int)(rng() % 200);
    h->p.ny = 16 + (int)(rng() % 200);
    h->d.mode = 0;
    h->d.lp.nx = h->p.nx;
    h->d.lp.ny = h->p.ny;
    h->d.lp.pitch = (h->p.nx + 63) / 64 * 64;
    h->d.lp.np = (int)(rng() % 9);
    h->np = h->d.lp.np;
    h->stream = new_stream();
    (void)hipEventCreateWithFlags(&h->ev_order, 0);
    (void)hipMalloc((void**)&h->base, 4096);
    g_live.insert(h);
    return h;
}

void destroy_run(lbm_sim* h) {   // the order of lbm_destroy
    forget_batches(h);
    g_live.erase(h);
    (void)hipFree(h->base);
    (void)hipEventDestroy(h->ev_order);
    destroy_stream(h->stream);
    delete h;
}

}  // namespace

int main(int argc, char** argv) {
    const unsigned long long seed = argc > 1 ? std::strtoull(argv[1], nullptr, 10) : 1;
    const int iters = argc > 2 ? std::atoi(argv[2]) : 4000;
    std::mt19937_64 rng(seed);
    std::vector<lbm_sim*> runs;
    hipStream_t server = new_stream();
    long calls = 0, noalloc_calls = 0;
    for (int it = 0; it < iters; ++it) {
        const int op = (int)(rng() % 100);
        if (runs.size() < 3 || (op < 12 && runs.size() < 40)) {
            runs.push_back(new_run(rng));
        } else if (op < 22) {   // a run ends
            const size_t i = rng() % runs.size();
            destroy_run(runs[i]);
            runs.erase(runs.begin() + (long)i);
        } else if (op < 27) {   // new particles: the handle drops its batches
            lbm_sim* h = runs[rng() % runs.size()];
            forget_batches(h);
            h->generation += 1;
            h->d.lp.np = h->np = (int)(rng() % 9);
        } else {   // step a random subset, random counts (zeros included)
            std::vector<lbm_sim*> pick = runs;
            std::shuffle(pick.begin(), pick.end(), rng);
            pick.resize(1 + rng() % std::min<size_t>(pick.size(), 12));
            std::vector<int32_t> n(pick.size());
            for (auto& v : n) v = (int32_t)(rng() % 4 == 0 ? 0 : rng() % 40);
            std::vector<int64_t> before;
            for (lbm_sim* h : pick) before.push_back(h->steps);
            void* stream = rng() % 2 ? (void*)server : nullptr;
            int rc;
            if (op < 45) {
                rc = lbm_step_many_noalloc(pick.data(), (int32_t)pick.size(), n.data(), stream);
                ++noalloc_calls;
            } else {
                rc = lbm_step_many(pick.data(), (int32_t)pick.size(), n.data(), stream);
                ++calls;
            }
            CHECK(rc == LBM_OK, "step call failed: %d %s", rc, pick[0]->err.c_str());
            for (size_t i = 0; i < pick.size(); ++i)
                CHECK(pick[i]->steps == before[i] + n[i], "run %zu advanced by %lld, not %d", i,
                      (long long)(pick[i]->steps - before[i]), n[i]);
        }
    }
    for (lbm_sim* h : runs) destroy_run(h);
    destroy_stream(server);
    std::printf("harness ok: seed %llu, %d operations, %ld cached and %ld fixed-array calls, %ld launches, "
                "%ld batched blocks checked; %zu events, %zu graphs, %zu executables, %zu allocations left\n",
                seed, iters, calls, noalloc_calls, g_launches, g_blocks_checked, g_events.size(),
                g_graphs.size(), g_execs.size(), g_mem.size());
    return 0;
}
