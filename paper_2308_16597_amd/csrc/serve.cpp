// serve.cpp -- several runs advanced together: each step kernel is one grid
// over every run of a batch (a run table in device memory, see RunStep /
// BatchLaunch).
//
// lbm_step_many keeps the device image of a batch (its run tables and block
// maps) in memory of its own and captures one 6-step cycle of the batch as a
// HIP graph, both cached per batch composition.  lbm_step_many_noalloc
// enqueues the same kernels launch by launch from an image it writes into a
// fixed device array, for callers that cannot allocate.
//
// The step state of a run -- time level, particle ring slot and cell-grid
// parity -- repeats every 6 steps, so a batch is fully described by its
// runs, their particle counts and their states at the start of a cycle.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <mutex>
#include <vector>

#include "sim.h"

using namespace ptlbm;

namespace {

constexpr int kCycle = 6;
constexpr size_t kMaxBatches = 16;
constexpr size_t kAlign = 256;

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int state_of(const lbm_sim* h) { return state_index(h->cur, h->ring, h->bin_parity); }

// The RunStep of h at cycle position j, counted from state s.
RunStep runstep_at(const lbm_sim* h, int s, int j) {
    const int cur = s / 6, ring = (s % 6) / 2, bp = s % 2;
    return make_runstep(h, cur ^ (j & 1), (ring + j) % 3, bp ^ (j & 1));
}

// The kernels of one batch at each cycle position: a single run takes its
// RunStep by value, several runs a device image of kCycle run tables (one
// RunStep per run, at that position) followed by one block map per grid
// class ({run, block of the run} per block).
struct Launches {
    bool single = false;
    int mode = 0;
    RunStep one[kCycle] = {};
    BatchLaunch bl[kCycle] = {};
};

struct ImageLayout {
    size_t tab_bytes = 0, off_bm[GC_COUNT] = {}, nblk[GC_COUNT] = {}, total = 0;
};

int image_layout(lbm_sim* const* runs, int n, ImageLayout& L, lbm_sim* herr) {
    L.tab_bytes = round_up((size_t)n * sizeof(RunStep), kAlign);
    L.total = kCycle * L.tab_bytes;
    for (int c = 0; c < GC_COUNT; ++c) {
        size_t tot = 0;
        for (int i = 0; i < n; ++i) tot += run_blocks(c, runs[i]->d.lp);
        if (tot > 0x7fffffffu) return fail(herr, LBM_EINVAL, "batch grid too large");
        L.nblk[c] = tot;
        L.off_bm[c] = L.total;
        L.total += round_up(std::max<size_t>(tot, 1) * sizeof(uint2), kAlign);
    }
    return LBM_OK;
}

// The image of runs at states[i] into host (L.total bytes).
void write_image(lbm_sim* const* runs, int n, const int* states, const ImageLayout& L, char* host) {
    for (int j = 0; j < kCycle; ++j)
        for (int i = 0; i < n; ++i) {
            const RunStep R = runstep_at(runs[i], states[i], j);
            std::memcpy(host + j * L.tab_bytes + (size_t)i * sizeof(RunStep), &R, sizeof R);
        }
    for (int c = 0; c < GC_COUNT; ++c) {
        uint2* bm = (uint2*)(host + L.off_bm[c]);
        size_t at = 0;
        for (int i = 0; i < n; ++i) {
            const unsigned nb = run_blocks(c, runs[i]->d.lp);
            for (unsigned k = 0; k < nb; ++k) bm[at++] = make_uint2((unsigned)i, k);
        }
    }
}

// Launch descriptors of runs at states[i], the image (if any) at dev.
void set_launches(lbm_sim* const* runs, int n, const int* states, const ImageLayout& L, char* dev,
                  Launches& out) {
    out.mode = runs[0]->d.mode;
    out.single = n == 1;
    if (out.single) {
        for (int j = 0; j < kCycle; ++j) out.one[j] = runstep_at(runs[0], states[0], j);
        return;
    }
    size_t lds = 0;
    for (int i = 0; i < n; ++i) lds = std::max(lds, links_block_lds(runs[i]->d.lp));
    for (int j = 0; j < kCycle; ++j) {
        BatchLaunch& B = out.bl[j];
        B.tab = (const RunStep*)(dev + j * L.tab_bytes);
        B.tab_next = (const RunStep*)(dev + ((j + 1) % kCycle) * L.tab_bytes);
        for (int c = 0; c < GC_COUNT; ++c) {
            B.bmap[c] = (const uint2*)(dev + L.off_bm[c]);
            B.nblk[c] = (unsigned)L.nblk[c];
        }
        B.lds = lds;
        B.mode = out.mode;
        B.aa = runs[0]->d.lp.aa != 0;
    }
}

// Kernel k of the step at cycle position j (the link collection takes the
// RunStep of the step after it).
hipError_t launch_pos(const Launches& b, int j, int k, hipStream_t S) {
    if (!b.single) return launch_step_batch(k, b.bl[j], S);
    return launch_step(k, b.one[k == SK_COLLECT ? (j + 1) % kCycle : j], b.mode, S);
}

// L steps launch by launch from cycle position 0.
int launch_steps(const Launches& b, int64_t L, hipStream_t S, lbm_sim* herr) {
    for (int64_t s = 0; s < L; ++s)
        for (int k = 0; k < SK_COUNT; ++k) HIPCHK(herr, launch_pos(b, (int)(s % kCycle), k, S));
    return LBM_OK;
}

void advance_by(lbm_sim* h, int64_t L) {
    h->cur ^= (int)(L & 1);
    h->bin_parity ^= (int)(L & 1);
    h->ring = (int)((h->ring + L) % 3);
    h->steps += L;
}

// Orders stream `to` after the work enqueued so far on h's stream, with h's
// own event (the wait takes the event's state at the time of the call).
int order_after_handle(hipStream_t to, lbm_sim* h, lbm_sim* herr) {
    if (to == h->stream) return LBM_OK;
    HIPCHK(herr, hipEventRecord(h->ev_order, h->stream));
    HIPCHK(herr, hipStreamWaitEvent(to, h->ev_order, 0));
    return LBM_OK;
}

// Checks shared by both entry points: count distinct handles of one storage
// mode and streaming layout, indirect link addressing, counts >= 0.  (The
// pairwise test allocates nothing; calls carry tens of runs.)
int check_runs(lbm_handle* hs, int32_t count, const int32_t* nsteps, const char* who) {
    if (!hs || !nsteps || count <= 0) return fail(nullptr, LBM_EINVAL, "%s: empty or null run list", who);
    for (int32_t i = 0; i < count; ++i)
        if (!hs[i]) return fail(nullptr, LBM_EINVAL, "%s: null handle at %d", who, i);
    lbm_sim* h0 = hs[0];
    for (int32_t i = 0; i < count; ++i)
        for (int32_t j = i + 1; j < count; ++j)
            if (hs[i] == hs[j]) return fail(h0, LBM_EINVAL, "%s: a handle appears twice", who);
    for (int32_t i = 0; i < count; ++i) {
        if (nsteps[i] < 0) return fail(h0, LBM_EINVAL, "%s: negative step count at %d", who, i);
        if (hs[i]->d.mode != h0->d.mode)
            return fail(h0, LBM_EINVAL, "%s: runs of one call must share the storage mode", who);
        if (hs[i]->d.lp.aa != h0->d.lp.aa)
            return fail(h0, LBM_EINVAL, "%s: runs of one call must share the streaming layout", who);
        if (hs[i]->d.lp.direct)
            return fail(h0, LBM_EINVAL, "%s: direct link addressing is for single runs only", who);
    }
    return LBM_OK;
}

// ------------------------------------------------- lbm_step_many (cached) ----

struct RunKey {
    const lbm_sim* h;
    uint64_t generation;
    int state;
    bool operator==(const RunKey& o) const {
        return h == o.h && generation == o.generation && state == o.state;
    }
};

struct Batch {
    std::vector<lbm_sim*> runs;
    std::vector<RunKey> key;
    Launches launch;
    char* dev = nullptr;            // batched: the device image
    std::vector<char> host;         // its host image (kept until the batch is dropped)
    hipGraphExec_t exec = nullptr;  // one captured cycle
    hipEvent_t done = nullptr;      // recorded after each use of the batch
    uint64_t last_use = 0, uses = 0;
};

std::mutex g_mu;
std::vector<std::unique_ptr<Batch>> g_batches;
uint64_t g_clock = 0;

// Waits for the batch's last use (its own event: the streams it ran on may
// be gone by now), then frees what it holds.
void release(Batch& b) {
    if (b.done) {
        (void)hipEventSynchronize(b.done);
        (void)hipEventDestroy(b.done);
    }
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    if (b.dev) (void)hipFree(b.dev);
    b.done = nullptr;
    b.exec = nullptr;
    b.dev = nullptr;
}

int build(Batch& b, lbm_sim* const* runs, int n, lbm_sim* herr) {
    b.runs.assign(runs, runs + n);
    std::vector<int> states((size_t)n);
    for (int i = 0; i < n; ++i) {
        states[i] = state_of(runs[i]);
        b.key.push_back(RunKey{runs[i], runs[i]->generation, states[i]});
    }
    HIPCHK(herr, hipEventCreateWithFlags(&b.done, hipEventDisableTiming));
    ImageLayout L;
    if (n > 1) {
        int rc = image_layout(runs, n, L, herr);
        if (rc != LBM_OK) return rc;
        b.host.assign(L.total, 0);
        write_image(runs, n, states.data(), L, b.host.data());
        HIPCHK(herr, hipMalloc((void**)&b.dev, L.total));
    }
    set_launches(runs, n, states.data(), L, b.dev, b.launch);
    return LBM_OK;
}

int upload(Batch& b, hipStream_t S, lbm_sim* herr) {
    if (b.launch.single || b.host.empty()) return LBM_OK;
    HIPCHK(herr, hipMemcpyAsync(b.dev, b.host.data(), b.host.size(), hipMemcpyHostToDevice, S));
    return LBM_OK;
}

int capture(Batch& b, hipStream_t S, lbm_sim* herr) {
    HIPCHK(herr, hipStreamBeginCapture(S, hipStreamCaptureModeRelaxed));
    hipError_t e = hipSuccess;
    for (int j = 0; j < kCycle && e == hipSuccess; ++j)
        for (int k = 0; k < SK_COUNT && e == hipSuccess; ++k) e = launch_pos(b.launch, j, k, S);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(S, &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&b.exec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        b.exec = nullptr;
        return hip_fail(herr, e, "capture of the step cycle");
    }
    return LBM_OK;
}

// The cached batch for these runs in their current states, or a new one.
int get_batch(lbm_sim* const* runs, int n, hipStream_t S, Batch** out) {
    std::vector<RunKey> key;
    key.reserve(n);
    for (int i = 0; i < n; ++i) key.push_back(RunKey{runs[i], runs[i]->generation, state_of(runs[i])});
    for (auto& b : g_batches)
        if (b->key == key) {
            b->last_use = ++g_clock;
            *out = b.get();
            return LBM_OK;
        }
    if (g_batches.size() >= kMaxBatches) {
        auto lru = std::min_element(g_batches.begin(), g_batches.end(),
                                    [](const auto& a, const auto& c) { return a->last_use < c->last_use; });
        release(**lru);
        g_batches.erase(lru);
    }
    auto b = std::make_unique<Batch>();
    int rc = build(*b, runs, n, runs[0]);
    if (rc == LBM_OK) rc = upload(*b, S, runs[0]);
    if (rc != LBM_OK) {
        release(*b);
        return rc;
    }
    b->last_use = ++g_clock;
    *out = b.get();
    g_batches.push_back(std::move(b));
    return LBM_OK;
}

// Enqueue L steps of the batch on S: whole cycles by graph replay (captured
// on first use once the batch is worth it), the rest launch by launch.
int run_segment(Batch& b, int64_t L, hipStream_t S, lbm_sim* herr) {
    const int64_t full = L / kCycle;
    const int rem = (int)(L % kCycle);
    if (full > 0 && !b.exec && (full >= 2 || b.uses > 0)) {
        int rc = capture(b, S, herr);
        if (rc != LBM_OK) return rc;
    }
    if (b.exec) {
        for (int64_t f = 0; f < full; ++f) HIPCHK(herr, hipGraphLaunch(b.exec, S));
    } else {
        int rc = launch_steps(b.launch, full * kCycle, S, herr);
        if (rc != LBM_OK) return rc;
    }
    int rc = launch_steps(b.launch, rem, S, herr);
    if (rc != LBM_OK) return rc;
    HIPCHK(herr, hipEventRecord(b.done, S));
    b.uses += 1;
    return LBM_OK;
}

// ----------------------------------------- lbm_step_many_noalloc (fixed) ----

constexpr size_t kScratchBytes = (size_t)8 << 20;
constexpr int kMaxNoAllocRuns = 64;
constexpr int kMaxDevices = 64;

}  // namespace

// Device image of lbm_step_many_noalloc: the run tables and block maps of
// the batch segment being stepped.  Each GPU the library runs on holds its
// own copy until the process ends; every call on a GPU overwrites it.
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

struct NoAllocDevice {
    char* scratch = nullptr;         // device address of `scratch` on this GPU
    hipEvent_t copied = nullptr;     // the last upload has read the host image
    hipEvent_t done = nullptr;       // the last call's work on its stream
};
NoAllocDevice g_noalloc[kMaxDevices];
// host image of one segment, rewritten only after its last upload completed
alignas(256) char g_host_image[kScratchBytes];

// Set-up on the current device (its first call there): the device address
// of `scratch` (in host code the array's name is no device address), and
// two events.
int noalloc_device(NoAllocDevice** out, lbm_sim* herr) {
    int dev = 0;
    HIPCHK(herr, hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(herr, LBM_EDEVICE, "device index %d out of range", dev);
    NoAllocDevice& d = g_noalloc[dev];
    if (!d.scratch) {
        void* p = nullptr;
        HIPCHK(herr, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(herr, LBM_EDEVICE, "no device address for the step tables");
        if (!d.copied) HIPCHK(herr, hipEventCreateWithFlags(&d.copied, hipEventDisableTiming));
        if (!d.done) HIPCHK(herr, hipEventCreateWithFlags(&d.done, hipEventDisableTiming));
        d.scratch = (char*)p;
    }
    *out = &d;
    return LBM_OK;
}

}  // namespace

namespace ptlbm {

void forget_batches(const lbm_sim* h) {
    std::lock_guard<std::mutex> lock(g_mu);
    for (size_t i = 0; i < g_batches.size();) {
        Batch& b = *g_batches[i];
        if (std::find(b.runs.begin(), b.runs.end(), h) != b.runs.end()) {
            release(b);
            g_batches.erase(g_batches.begin() + (long)i);
        } else {
            ++i;
        }
    }
}

}  // namespace ptlbm

extern "C" int lbm_step_many(lbm_handle* hs, int32_t count, const int32_t* nsteps, void* hip_stream) {
    int rc = check_runs(hs, count, nsteps, "lbm_step_many");
    if (rc != LBM_OK) return rc;
    lbm_sim* h0 = hs[0];
    hipStream_t S = hip_stream ? (hipStream_t)hip_stream : h0->stream;
    std::lock_guard<std::mutex> lock(g_mu);
    for (int32_t i = 0; i < count; ++i) {
        rc = order_after_handle(S, hs[i], h0);
        if (rc != LBM_OK) return rc;
    }
    std::vector<int64_t> left(nsteps, nsteps + count);
    std::vector<lbm_sim*> active;
    for (;;) {
        active.clear();
        int64_t L = 0;
        for (int32_t i = 0; i < count; ++i)
            if (left[i] > 0) {
                active.push_back(hs[i]);
                L = L == 0 ? left[i] : std::min(L, left[i]);
            }
        if (active.empty()) break;
        Batch* b = nullptr;
        rc = get_batch(active.data(), (int)active.size(), S, &b);
        if (rc == LBM_OK) rc = run_segment(*b, L, S, h0);
        if (rc != LBM_OK) return rc;
        for (lbm_sim* h : active) advance_by(h, L);
        for (int32_t i = 0; i < count; ++i)
            if (left[i] > 0) left[i] -= L;
    }
    // each handle's stream after the batched work on S
    if (count > 1 || S != h0->stream) {
        HIPCHK(h0, hipEventRecord(h0->ev_order, S));
        for (int32_t i = 0; i < count; ++i)
            if (hs[i]->stream != S) HIPCHK(h0, hipStreamWaitEvent(hs[i]->stream, h0->ev_order, 0));
    }
    return LBM_OK;
}

extern "C" int lbm_step_many_noalloc(lbm_handle* hs, int32_t count, const int32_t* nsteps, void* hip_stream) {
    int rc = check_runs(hs, count, nsteps, "lbm_step_many_noalloc");
    if (rc != LBM_OK) return rc;
    lbm_sim* h0 = hs[0];
    if (count > kMaxNoAllocRuns)
        return fail(h0, LBM_EINVAL, "lbm_step_many_noalloc: %d runs, at most %d", count, kMaxNoAllocRuns);
    hipStream_t S = hip_stream ? (hipStream_t)hip_stream : h0->stream;
    std::lock_guard<std::mutex> lock(g_mu);
    // every segment's image is at most that of all runs with steps left
    lbm_sim* act[kMaxNoAllocRuns];
    int n = 0;
    for (int32_t i = 0; i < count; ++i)
        if (nsteps[i] > 0) act[n++] = hs[i];
    if (n == 0) return LBM_OK;
    if (n > 1) {
        ImageLayout L;
        rc = image_layout(act, n, L, h0);
        if (rc != LBM_OK) return rc;
        if (L.total > kScratchBytes)
            return fail(h0, LBM_EINVAL,
                        "lbm_step_many_noalloc: the run tables and block maps of these runs need %zu bytes, "
                        "the fixed array holds %zu",
                        L.total, kScratchBytes);
    }
    NoAllocDevice* dev = nullptr;
    rc = noalloc_device(&dev, h0);
    if (rc != LBM_OK) return rc;
    for (int32_t i = 0; i < count; ++i) {
        rc = order_after_handle(S, hs[i], h0);
        if (rc != LBM_OK) return rc;
    }
    int64_t left[kMaxNoAllocRuns];
    for (int32_t i = 0; i < count; ++i) left[i] = nsteps[i];
    for (;;) {
        int states[kMaxNoAllocRuns];
        int64_t L = 0;
        n = 0;
        for (int32_t i = 0; i < count; ++i)
            if (left[i] > 0) {
                act[n] = hs[i];
                states[n] = state_of(hs[i]);
                ++n;
                L = L == 0 ? left[i] : std::min(L, left[i]);
            }
        if (n == 0) break;
        ImageLayout IL;
        Launches lau;
        if (n > 1) {
            rc = image_layout(act, n, IL, h0);
            if (rc != LBM_OK) return rc;
            // the host image is rewritten once the previous upload has read it
            HIPCHK(h0, hipEventSynchronize(dev->copied));
            write_image(act, n, states, IL, g_host_image);
            HIPCHK(h0, hipMemcpyAsync(dev->scratch, g_host_image, IL.total, hipMemcpyHostToDevice, S));
            HIPCHK(h0, hipEventRecord(dev->copied, S));
        }
        set_launches(act, n, states, IL, dev->scratch, lau);
        rc = launch_steps(lau, L, S, h0);
        if (rc != LBM_OK) return rc;
        for (int k = 0; k < n; ++k) advance_by(act[k], L);
        for (int32_t i = 0; i < count; ++i)
            if (left[i] > 0) left[i] -= L;
    }
    // each handle's stream after the work on S
    HIPCHK(h0, hipEventRecord(dev->done, S));
    for (int32_t i = 0; i < count; ++i)
        if (hs[i]->stream != S) HIPCHK(h0, hipStreamWaitEvent(hs[i]->stream, dev->done, 0));
    return LBM_OK;
}
