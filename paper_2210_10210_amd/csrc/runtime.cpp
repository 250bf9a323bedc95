// Process-wide caches behind the plans: device memory, pinned host memory,
// streams, events and instantiated CG graphs.
//
// A serving loop builds and destroys a plan per request; hipMalloc, hipFree,
// hipHostMalloc, stream creation and graph instantiation cost tens to
// hundreds of microseconds each, more than the small kernels they feed.
// Destroyed plans therefore hand their buffers, stream and events back to
// per-device free lists (exact-size reuse: a repeated problem gets the same
// buffers back), and instantiated CG graphs are cached under a key that lists
// every argument they captured, so a plan that receives identical buffers
// and sizes replays the existing graph.  efgp_release_workspace empties
// every cache that no live plan uses.  The spread tuning table (measured
// fastest spreader per problem shape) lives here too.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "efgp_internal.h"

namespace efgp {
namespace {

constexpr size_t kDevCap = (size_t)2 << 30;    // cached device bytes per device
constexpr size_t kPinnedCap = (size_t)64 << 20;
constexpr size_t kMaxGraphs = 64;

struct DevPool {
    std::multimap<size_t, void*> free;
    size_t cached = 0;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> sync_events;    // timing disabled
    std::vector<hipEvent_t> timing_events;
};

struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    int refs = 0;
    uint64_t stamp = 0;
};

std::mutex g_mu;
std::map<int, DevPool> g_dev;
std::multimap<size_t, void*> g_pinned;
size_t g_pinned_cached = 0;
std::map<std::pair<int, std::string>, GraphEntry> g_graphs;
uint64_t g_clock = 0;

size_t round_up(size_t b) { return (std::max<size_t>(b, 1) + 255) / 256 * 256; }

struct DeviceGuard {
    int prev = 0;
    explicit DeviceGuard(int dev) {
        (void)hipGetDevice(&prev);
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = 0;
        (void)hipGetDevice(&cur);
        if (cur != prev) (void)hipSetDevice(prev);
    }
};

}  // namespace

int current_device() {
    int d = 0;
    (void)hipGetDevice(&d);
    return d;
}

void* pool_alloc(size_t bytes) {
    bytes = round_up(bytes);
    const int dev = current_device();
    {
        std::lock_guard<std::mutex> g(g_mu);
        DevPool& P = g_dev[dev];
        auto it = P.free.find(bytes);
        if (it != P.free.end()) {
            void* p = it->second;
            P.free.erase(it);
            P.cached -= bytes;
            return p;
        }
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        // give the cached buffers of this device back to the runtime and retry
        std::vector<void*> drop;
        {
            std::lock_guard<std::mutex> g(g_mu);
            DevPool& P = g_dev[dev];
            for (auto& kv : P.free) drop.push_back(kv.second);
            P.free.clear();
            P.cached = 0;
        }
        for (void* q : drop) (void)hipFree(q);
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            throw StatusError{EFGP_ENOMEM, "device allocation failed"};
        }
    }
    return p;
}

void pool_free(int dev, void* p, size_t bytes) {
    if (!p) return;
    bytes = round_up(bytes);
    {
        std::lock_guard<std::mutex> g(g_mu);
        DevPool& P = g_dev[dev];
        if (P.cached + bytes <= kDevCap) {
            P.free.emplace(bytes, p);
            P.cached += bytes;
            return;
        }
    }
    DeviceGuard dg(dev);
    (void)hipFree(p);
}

void* pinned_alloc(size_t bytes) {
    bytes = round_up(bytes);
    {
        std::lock_guard<std::mutex> g(g_mu);
        auto it = g_pinned.find(bytes);
        if (it != g_pinned.end()) {
            void* p = it->second;
            g_pinned.erase(it);
            g_pinned_cached -= bytes;
            return p;
        }
    }
    void* p = nullptr;
    if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        throw StatusError{EFGP_ENOMEM, "pinned host allocation failed"};
    }
    return p;
}

void pinned_free(void* p, size_t bytes) {
    if (!p) return;
    bytes = round_up(bytes);
    {
        std::lock_guard<std::mutex> g(g_mu);
        if (g_pinned_cached + bytes <= kPinnedCap) {
            g_pinned.emplace(bytes, p);
            g_pinned_cached += bytes;
            return;
        }
    }
    (void)hipHostFree(p);
}

hipStream_t acquire_stream() {
    const int dev = current_device();
    {
        std::lock_guard<std::mutex> g(g_mu);
        DevPool& P = g_dev[dev];
        if (!P.streams.empty()) {
            hipStream_t s = P.streams.back();
            P.streams.pop_back();
            return s;
        }
    }
    hipStream_t s = nullptr;
    EFGP_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    return s;
}

void release_stream(int dev, hipStream_t s) {
    if (!s) return;
    std::lock_guard<std::mutex> g(g_mu);
    g_dev[dev].streams.push_back(s);
}

hipEvent_t acquire_event(bool timing) {
    const int dev = current_device();
    {
        std::lock_guard<std::mutex> g(g_mu);
        DevPool& P = g_dev[dev];
        auto& v = timing ? P.timing_events : P.sync_events;
        if (!v.empty()) {
            hipEvent_t e = v.back();
            v.pop_back();
            return e;
        }
    }
    hipEvent_t e = nullptr;
    EFGP_HIP(hipEventCreateWithFlags(&e, timing ? hipEventDefault : hipEventDisableTiming));
    return e;
}

void release_event(int dev, hipEvent_t e, bool timing) {
    if (!e) return;
    std::lock_guard<std::mutex> g(g_mu);
    DevPool& P = g_dev[dev];
    (timing ? P.timing_events : P.sync_events).push_back(e);
}

hipGraphExec_t graph_acquire(int dev, const std::string& key) {
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_graphs.find({dev, key});
    if (it == g_graphs.end()) return nullptr;
    it->second.refs++;
    it->second.stamp = ++g_clock;
    return it->second.exec;
}

void graph_insert(int dev, const std::string& key, hipGraphExec_t exec) {
    std::vector<hipGraphExec_t> drop;
    {
        std::lock_guard<std::mutex> g(g_mu);
        GraphEntry& e = g_graphs[{dev, key}];
        if (e.exec && e.exec != exec) drop.push_back(e.exec);
        e.exec = exec;
        e.refs += 1;
        e.stamp = ++g_clock;
        // evict the least recently used graphs no live plan holds
        while (g_graphs.size() > kMaxGraphs) {
            auto victim = g_graphs.end();
            for (auto it = g_graphs.begin(); it != g_graphs.end(); ++it)
                if (it->second.refs == 0 && (victim == g_graphs.end() || it->second.stamp < victim->second.stamp))
                    victim = it;
            if (victim == g_graphs.end()) break;
            drop.push_back(victim->second.exec);
            g_graphs.erase(victim);
        }
    }
    for (hipGraphExec_t x : drop) (void)hipGraphExecDestroy(x);
}

void graph_release(int dev, const std::string& key) {
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_graphs.find({dev, key});
    if (it != g_graphs.end() && it->second.refs > 0) it->second.refs--;
}

void release_pools() {
    std::vector<std::pair<int, void*>> dev_free;
    std::vector<std::pair<int, hipStream_t>> streams;
    std::vector<std::pair<int, hipEvent_t>> events;
    std::vector<std::pair<int, hipGraphExec_t>> graphs;
    std::vector<void*> pinned;
    {
        std::lock_guard<std::mutex> g(g_mu);
        for (auto& kv : g_dev) {
            for (auto& f : kv.second.free) dev_free.push_back({kv.first, f.second});
            kv.second.free.clear();
            kv.second.cached = 0;
            for (hipStream_t s : kv.second.streams) streams.push_back({kv.first, s});
            kv.second.streams.clear();
            for (hipEvent_t e : kv.second.sync_events) events.push_back({kv.first, e});
            for (hipEvent_t e : kv.second.timing_events) events.push_back({kv.first, e});
            kv.second.sync_events.clear();
            kv.second.timing_events.clear();
        }
        for (auto it = g_graphs.begin(); it != g_graphs.end();) {
            if (it->second.refs == 0) {
                graphs.push_back({it->first.first, it->second.exec});
                it = g_graphs.erase(it);
            } else {
                ++it;
            }
        }
        for (auto& kv : g_pinned) pinned.push_back(kv.second);
        g_pinned.clear();
        g_pinned_cached = 0;
    }
    for (auto& x : graphs) { DeviceGuard dg(x.first); (void)hipGraphExecDestroy(x.second); }
    for (auto& x : streams) { DeviceGuard dg(x.first); (void)hipStreamDestroy(x.second); }
    for (auto& x : events) { DeviceGuard dg(x.first); (void)hipEventDestroy(x.second); }
    for (auto& x : dev_free) { DeviceGuard dg(x.first); (void)hipFree(x.second); }
    for (void* p : pinned) (void)hipHostFree(p);
}

// ------------------------------------------------------------ spread tuning
namespace {
std::mutex g_tune_mu;
std::map<TuneKey, TuneChoice> g_tune;
}  // namespace

bool TuneKey::operator<(const TuneKey& o) const {
    const int a[] = {dev, dim, precision, nrhs, nf, w, nbucket};
    const int b[] = {o.dev, o.dim, o.precision, o.nrhs, o.nf, o.w, o.nbucket};
    return std::lexicographical_compare(a, a + 7, b, b + 7);
}

int n_bucket(int64_t n) {
    int b = 0;
    while (b < 62 && ((int64_t)1 << (b + 1)) <= n) b++;
    return b;   // floor(log2 n)
}

bool tune_lookup(const TuneKey& k, TuneChoice* c) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune.find(k);
    if (it == g_tune.end()) return false;
    *c = it->second;
    return true;
}

void tune_insert(const TuneKey& k, const TuneChoice& c) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[k] = c;
}

void tune_clear() {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune.clear();
}

// Text file: a header line, then one entry per line:
//   dev dim precision nrhs nf w log2n method tile ms
bool tune_save(const char* path) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    FILE* f = std::fopen(path, "w");
    if (!f) return false;
    std::fprintf(f, "efgp-spread-tune 1\n");
    for (const auto& kv : g_tune) {
        const TuneKey& k = kv.first;
        const TuneChoice& c = kv.second;
        std::fprintf(f, "%d %d %d %d %d %d %d %d %d %.6f\n", k.dev, k.dim, k.precision, k.nrhs, k.nf, k.w,
                     k.nbucket, c.method, c.tile, c.ms);
    }
    const bool ok = std::fflush(f) == 0;
    return std::fclose(f) == 0 && ok;
}

// Returns the number of entries read, or -1 for an unreadable or malformed
// file (then nothing is inserted).
int tune_load(const char* path) {
    FILE* f = std::fopen(path, "r");
    if (!f) return -1;
    char head[64] = {0};
    if (!std::fgets(head, sizeof(head), f) || std::strncmp(head, "efgp-spread-tune 1", 18) != 0) {
        std::fclose(f);
        return -1;
    }
    std::vector<std::pair<TuneKey, TuneChoice>> got;
    for (;;) {
        TuneKey k{};
        TuneChoice c{};
        const int r = std::fscanf(f, "%d %d %d %d %d %d %d %d %d %lf", &k.dev, &k.dim, &k.precision, &k.nrhs, &k.nf,
                                  &k.w, &k.nbucket, &c.method, &c.tile, &c.ms);
        if (r == EOF) break;
        const bool valid = r == 10 && k.dim >= 1 && k.dim <= 3 && (k.precision == 32 || k.precision == 64) &&
                           k.nrhs >= 1 && k.nrhs <= 64 && k.nf > 0 && k.w > 0 && k.nbucket >= 0 &&
                           (c.method == EFGP_SPREAD_TILES || c.method == EFGP_SPREAD_GRID_LDS ||
                            c.method == EFGP_SPREAD_REGIONS) && c.tile >= 0 &&
                           c.tile <= 4096;
        if (!valid) {
            std::fclose(f);
            return -1;
        }
        got.push_back({k, c});
    }
    std::fclose(f);
    std::lock_guard<std::mutex> g(g_tune_mu);
    for (const auto& e : got) g_tune[e.first] = e.second;
    return (int)got.size();
}

}  // namespace efgp
