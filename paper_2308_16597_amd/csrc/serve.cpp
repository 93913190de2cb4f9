// serve.cpp -- several runs advanced together (lbm_step_many): each step
// kernel is one grid over every run of a batch (a run table in device
// memory, see RunStep / BatchLaunch), and one 6-step cycle of a batch is
// captured once as a HIP graph and replayed.
//
// The step state of a run -- time level, particle ring slot and cell-grid
// parity -- repeats every 6 steps, so a batch is fully described by its
// runs, their particle counts and their states at the start of a cycle; it
// is cached under that key and reused while the composition is unchanged.
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
    int mode = 0;
    bool single = false;            // one run: kernels take its RunStep by value
    RunStep one[kCycle] = {};       // single run: its RunStep at each cycle position
    char* dev = nullptr;            // batched: run tables and block maps
    std::vector<char> host;         // their host image (kept until the batch is dropped)
    BatchLaunch bl[kCycle] = {};
    hipGraphExec_t exec = nullptr;  // one captured cycle
    hipStream_t last_stream = nullptr;
    uint64_t last_use = 0, uses = 0;
};

std::mutex g_mu;
std::vector<std::unique_ptr<Batch>> g_batches;
uint64_t g_clock = 0;

void release(Batch& b) {
    if (b.last_stream) (void)hipStreamSynchronize(b.last_stream);
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    if (b.dev) (void)hipFree(b.dev);
    b.exec = nullptr;
    b.dev = nullptr;
}

int state_of(const lbm_sim* h) { return state_index(h->cur, h->ring, h->bin_parity); }

// The RunStep of h at cycle position j, counted from state s.
RunStep runstep_at(const lbm_sim* h, int s, int j) {
    const int cur = s / 6, ring = (s % 6) / 2, bp = s % 2;
    return make_runstep(h, cur ^ (j & 1), (ring + j) % 3, bp ^ (j & 1));
}

int build(Batch& b, lbm_sim* const* runs, int n, lbm_sim* herr) {
    b.runs.assign(runs, runs + n);
    b.mode = runs[0]->d.mode;
    for (int i = 0; i < n; ++i) b.key.push_back(RunKey{runs[i], runs[i]->generation, state_of(runs[i])});
    if (n == 1) {
        b.single = true;
        for (int j = 0; j < kCycle; ++j) b.one[j] = runstep_at(runs[0], b.key[0].state, j);
        return LBM_OK;
    }
    size_t lds = 0;
    for (int i = 0; i < n; ++i) lds = std::max(lds, links_block_lds(runs[i]->d.lp));
    std::vector<uint2> bm[GC_COUNT];
    for (int c = 0; c < GC_COUNT; ++c) {
        size_t tot = 0;
        for (int i = 0; i < n; ++i) tot += run_blocks(c, runs[i]->d.lp);
        if (tot > 0x7fffffffu) return fail(herr, LBM_EINVAL, "batch grid too large");
        bm[c].reserve(tot);
        for (int i = 0; i < n; ++i) {
            const unsigned nb = run_blocks(c, runs[i]->d.lp);
            for (unsigned k = 0; k < nb; ++k) bm[c].push_back(make_uint2((unsigned)i, k));
        }
    }
    const size_t tab_bytes = round_up((size_t)n * sizeof(RunStep), kAlign);
    size_t off_bm[GC_COUNT], total = kCycle * tab_bytes;
    for (int c = 0; c < GC_COUNT; ++c) {
        off_bm[c] = total;
        total += round_up(std::max<size_t>(bm[c].size(), 1) * sizeof(uint2), kAlign);
    }
    b.host.assign(total, 0);
    for (int j = 0; j < kCycle; ++j)
        for (int i = 0; i < n; ++i) {
            const RunStep R = runstep_at(runs[i], b.key[i].state, j);
            std::memcpy(b.host.data() + j * tab_bytes + (size_t)i * sizeof(RunStep), &R, sizeof R);
        }
    for (int c = 0; c < GC_COUNT; ++c)
        if (!bm[c].empty()) std::memcpy(b.host.data() + off_bm[c], bm[c].data(), bm[c].size() * sizeof(uint2));
    HIPCHK(herr, hipMalloc((void**)&b.dev, total));
    for (int j = 0; j < kCycle; ++j) {
        BatchLaunch& L = b.bl[j];
        L.tab = (const RunStep*)(b.dev + j * tab_bytes);
        L.tab_next = (const RunStep*)(b.dev + ((j + 1) % kCycle) * tab_bytes);
        for (int c = 0; c < GC_COUNT; ++c) {
            L.bmap[c] = (const uint2*)(b.dev + off_bm[c]);
            L.nblk[c] = (unsigned)bm[c].size();
        }
        L.lds = lds;
        L.mode = b.mode;
        L.aa = runs[0]->d.lp.aa != 0;
    }
    return LBM_OK;
}

int upload(Batch& b, hipStream_t S, lbm_sim* herr) {
    if (b.single || b.host.empty()) return LBM_OK;
    HIPCHK(herr, hipMemcpyAsync(b.dev, b.host.data(), b.host.size(), hipMemcpyHostToDevice, S));
    return LBM_OK;
}

// Kernel k of the step at cycle position j (the link collection takes the
// RunStep of the step after it).
hipError_t launch_pos(const Batch& b, int j, int k, hipStream_t S) {
    if (!b.single) return launch_step_batch(k, b.bl[j], S);
    return launch_step(k, b.one[k == SK_COLLECT ? (j + 1) % kCycle : j], b.mode, S);
}

int capture(Batch& b, hipStream_t S, lbm_sim* herr) {
    HIPCHK(herr, hipStreamBeginCapture(S, hipStreamCaptureModeRelaxed));
    hipError_t e = hipSuccess;
    for (int j = 0; j < kCycle && e == hipSuccess; ++j)
        for (int k = 0; k < SK_COUNT && e == hipSuccess; ++k) e = launch_pos(b, j, k, S);
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

void advance_by(lbm_sim* h, int64_t L) {
    h->cur ^= (int)(L & 1);
    h->bin_parity ^= (int)(L & 1);
    h->ring = (int)((h->ring + L) % 3);
    h->steps += L;
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
        for (int64_t f = 0; f < full; ++f)
            for (int j = 0; j < kCycle; ++j)
                for (int k = 0; k < SK_COUNT; ++k) HIPCHK(herr, launch_pos(b, j, k, S));
    }
    for (int j = 0; j < rem; ++j)
        for (int k = 0; k < SK_COUNT; ++k) HIPCHK(herr, launch_pos(b, j, k, S));
    b.last_stream = S;
    b.uses += 1;
    return LBM_OK;
}

// Orders stream `to` after the work enqueued so far on `from`.
int order_after(hipStream_t to, hipStream_t from, lbm_sim* herr) {
    if (to == from) return LBM_OK;
    hipEvent_t ev;
    HIPCHK(herr, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    hipError_t e = hipEventRecord(ev, from);
    if (e == hipSuccess) e = hipStreamWaitEvent(to, ev, 0);
    (void)hipEventDestroy(ev);
    if (e != hipSuccess) return hip_fail(herr, e, "stream ordering");
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
    if (!hs || !nsteps || count <= 0) return fail(nullptr, LBM_EINVAL, "lbm_step_many: empty or null run list");
    for (int32_t i = 0; i < count; ++i)
        if (!hs[i]) return fail(nullptr, LBM_EINVAL, "lbm_step_many: null handle at %d", i);
    lbm_sim* h0 = hs[0];
    std::vector<lbm_sim*> sorted(hs, hs + count);
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
        return fail(h0, LBM_EINVAL, "lbm_step_many: a handle appears twice");
    for (int32_t i = 0; i < count; ++i) {
        if (nsteps[i] < 0) return fail(h0, LBM_EINVAL, "lbm_step_many: negative step count at %d", i);
        if (hs[i]->d.mode != h0->d.mode)
            return fail(h0, LBM_EINVAL, "lbm_step_many: runs of one call must share the storage mode");
        if (hs[i]->d.lp.aa != h0->d.lp.aa)
            return fail(h0, LBM_EINVAL, "lbm_step_many: runs of one call must share the streaming layout");
        if (hs[i]->d.lp.direct)
            return fail(h0, LBM_EINVAL, "lbm_step_many: direct link addressing is for single runs only");
    }
    hipStream_t S = hip_stream ? (hipStream_t)hip_stream : h0->stream;
    std::lock_guard<std::mutex> lock(g_mu);
    for (int32_t i = 0; i < count; ++i) {
        int rc = order_after(S, hs[i]->stream, h0);
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
        int rc = get_batch(active.data(), (int)active.size(), S, &b);
        if (rc == LBM_OK) rc = run_segment(*b, L, S, h0);
        if (rc != LBM_OK) return rc;
        for (lbm_sim* h : active) advance_by(h, L);
        for (int32_t i = 0; i < count; ++i)
            if (left[i] > 0) left[i] -= L;
    }
    for (int32_t i = 0; i < count; ++i) {
        int rc = order_after(hs[i]->stream, S, h0);
        if (rc != LBM_OK) return rc;
    }
    return LBM_OK;
}
