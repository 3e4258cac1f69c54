// C-ABI entry points: validation, error reporting, kernel timing, and the
// host-side orchestration of index build and query answering.
//
// Build (Sec. II iSAX Representation / ADS+ Index; Sec. III ParIS Stage 2,
// MESSI Stages 1-2): summarise every series, sort the words by their
// interleaved key, cut the order into leaves with symbol envelopes.
// Query (Sec. III, query answering): approximate answer -> best-so-far, leaf
// and series lower bounds with pruning, refinement, final ordering.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <optional>

#include "build_kernels.h"
#include "query_kernels.h"

namespace isax {

// ------------------------------------------------------------------ errors
static thread_local std::string g_err_msg;

void set_error(int code, const std::string& msg) {
    (void)code;
    g_err_msg = msg;
}
void clear_error() { g_err_msg.clear(); }

// ------------------------------------------------------------------ profiling
namespace {
struct ProfStat {
    int64_t launches = 0;
    double ms = 0.0;
    double bytes = 0.0;
};
struct PendingPair {
    std::string name;
    hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::map<std::string, ProfStat> g_prof;
std::vector<PendingPair> g_pending;

void drain_pending_locked() {
    for (auto& p : g_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            auto& st = g_prof[p.name];
            st.launches += 1;
            st.ms += ms;
        }
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    g_pending.clear();
}
}  // namespace

bool profiling_on() { return g_prof_on; }

ProfScope::ProfScope(const char* n, hipStream_t s) : name(n), stream(s) {
    if (!g_prof_on) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        a = b = nullptr;
        return;
    }
    (void)hipEventRecord(a, stream);
}
ProfScope::~ProfScope() {
    if (!a) return;
    (void)hipEventRecord(b, stream);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_pending.push_back({name, a, b});
    if (g_pending.size() > 4096) drain_pending_locked();
}
void profile_add_bytes(const char* name, double bytes) {
    if (!g_prof_on) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof[name].bytes += bytes;
}

// ------------------------------------------------------------------ memory
// Block cache for query scratch.  A query call allocates and releases several
// blocks of tens to hundreds of MB (candidate lists, leaf lists, filter
// candidates); through the stream-ordered allocator each such allocation or
// release costs tens to hundreds of microseconds, about a millisecond per call.
// Released blocks therefore stay allocated and are handed out again: on the
// stream that released a block, stream order protects its reuse; another
// stream first waits for the event recorded at the release.  Idle blocks above
// kCacheIdleMax bytes per device are freed, least recently used first.
namespace {
constexpr size_t kCacheMin = size_t(1) << 20, kCacheMax = size_t(1) << 30, kCacheIdleMax = size_t(4) << 30;
constexpr size_t kCacheGranule = size_t(2) << 20;
struct CacheBlock {
    void* p;
    size_t bytes;
    int device;
    hipStream_t stream;  // stream of the last release
    hipEvent_t ready;    // recorded on that stream at the release
    bool in_use;
    uint64_t last_use;
};
std::mutex g_cache_mu;
std::vector<CacheBlock> g_cache;
uint64_t g_cache_tick = 0;

// Free idle blocks of `dev` (least recently used first) until at most `keep`
// idle bytes remain.  Caller holds g_cache_mu.
void cache_trim_locked(int dev, size_t keep) {
    for (;;) {
        size_t idle = 0;
        int lru = -1;
        for (int i = 0; i < (int)g_cache.size(); ++i) {
            const CacheBlock& b = g_cache[i];
            if (b.in_use || b.device != dev) continue;
            idle += b.bytes;
            if (lru < 0 || b.last_use < g_cache[lru].last_use) lru = i;
        }
        if (idle <= keep || lru < 0) return;
        CacheBlock b = g_cache[lru];
        g_cache.erase(g_cache.begin() + lru);
        (void)hipEventSynchronize(b.ready);
        (void)hipEventDestroy(b.ready);
        (void)hipFree(b.p);
    }
}

void* cache_alloc(size_t n, hipStream_t s) {
    int dev = 0;
    ISAX_HIP(hipGetDevice(&dev));
    const size_t want = (n + kCacheGranule - 1) / kCacheGranule * kCacheGranule;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    int best = -1;
    for (int i = 0; i < (int)g_cache.size(); ++i) {
        const CacheBlock& b = g_cache[i];
        if (!b.in_use && b.device == dev && b.bytes >= want && b.bytes <= 2 * want &&
            (best < 0 || b.bytes < g_cache[best].bytes))
            best = i;
    }
    if (best >= 0) {
        CacheBlock& b = g_cache[best];
        if (b.stream != s) ISAX_HIP(hipStreamWaitEvent(s, b.ready, 0));
        b.in_use = true;
        b.stream = s;
        b.last_use = ++g_cache_tick;
        return b.p;
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        cache_trim_locked(dev, 0);
        e = hipMalloc(&p, want);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error{ISAX_ENOMEM, "device allocation of " + std::to_string(n) + " bytes failed: " + hipGetErrorString(e)};
    }
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipFree(p);
        throw Error{ISAX_EDEVICE, "event creation failed"};
    }
    g_cache.push_back({p, want, dev, s, ev, true, ++g_cache_tick});
    return p;
}

void cache_free(void* p, hipStream_t s) noexcept {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    for (CacheBlock& b : g_cache)
        if (b.p == p) {
            (void)hipEventRecord(b.ready, s);
            b.stream = s;
            b.in_use = false;
            b.last_use = ++g_cache_tick;
            cache_trim_locked(b.device, kCacheIdleMax);
            return;
        }
}

// Frees every idle cached block of the current device (before an allocation
// that failed is tried again).
void cache_release_idle() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    cache_trim_locked(dev, 0);
}
}  // namespace

// Fault injection (isax_debug_fail_allocation): the countdown-th allocation fails.
static std::atomic<int64_t> g_fail_countdown{0};
void injected_failure(size_t n) {
    if (g_fail_countdown.load(std::memory_order_relaxed) <= 0) return;
    if (g_fail_countdown.fetch_sub(1) == 1)
        throw Error{ISAX_ENOMEM, "device allocation of " + std::to_string(n) + " bytes failed (injected)"};
}

// ------------------------------------------------------------------ fixed scratch
// The memory of isax_query_noalloc.  Each device that loads the library holds
// its own copy of this array until the process ends; host code reaches it only
// through the address hipGetSymbolAddress returns for the current device (the
// array's name in host code is a host-side stand-in, not a device address).
constexpr size_t kNoAllocBytes = size_t(256) << 20;
constexpr int kNoAllocDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
thread_local FixedScratch* t_fixed = nullptr;
std::mutex g_noalloc_init_mu;
void* g_noalloc_ptr[kNoAllocDevices] = {};
std::mutex g_noalloc_call_mu[kNoAllocDevices];  // one no-allocation call per device at a time

// Device address of `scratch` on device `dev` (current), looked up once per device.
char* noalloc_base(int dev) {
    std::lock_guard<std::mutex> lk(g_noalloc_init_mu);
    if (!g_noalloc_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            throw Error{ISAX_EDEVICE, std::string("hipGetSymbolAddress of the fixed scratch failed: ") +
                                          hipGetErrorString(e)};
        }
        g_noalloc_ptr[dev] = ptr;
    }
    return static_cast<char*>(g_noalloc_ptr[dev]);
}

// Makes the device's fixed scratch the source of every DevBuf of this thread
// for the scope's lifetime (and holds the device's call lock).
// On the way out it waits for the call's stream, so that work of a call that
// failed half-way never overlaps the next call's use of the array.
struct FixedScratchScope {
    std::unique_lock<std::mutex> lk;
    FixedScratch fx;
    hipStream_t stream;
    FixedScratchScope(int dev, hipStream_t s) : lk(g_noalloc_call_mu[dev]), stream(s) {
        fx.base = noalloc_base(dev);
        fx.size = kNoAllocBytes;
        t_fixed = &fx;
    }
    ~FixedScratchScope() {
        t_fixed = nullptr;
        (void)hipStreamSynchronize(stream);
    }
};
}  // namespace

FixedScratch* fixed_scratch() { return t_fixed; }

void* FixedScratch::carve(size_t n) {
    const size_t at = (off + 255) / 256 * 256;
    if (at > size || n > size - at)
        throw Error{ISAX_ENOMEM, "the fixed scratch of isax_query_noalloc (" + std::to_string(size >> 20) +
                                     " MiB) is exhausted: " + std::to_string(n) + " more bytes were needed at offset " +
                                     std::to_string(at) + "; use a smaller batch or isax_query_ex"};
    off = at + n;
    return base + at;
}

DevBuf::DevBuf(size_t n, hipStream_t s) : bytes(n), stream(s) {
    if (n == 0) return;
    if (t_fixed) {
        p = t_fixed->carve(n);
        fixed = true;
        return;
    }
    injected_failure(n);
    if (n >= kCacheMin && n <= kCacheMax) {
        p = cache_alloc(n, s);
        cached = true;
        return;
    }
    hipError_t e = hipMallocAsync(&p, n, s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        cache_release_idle();
        e = hipMallocAsync(&p, n, s);
    }
    if (e != hipSuccess) {
        p = nullptr;
        throw Error{ISAX_ENOMEM, "device allocation of " + std::to_string(n) + " bytes failed: " + hipGetErrorString(e)};
    }
}
static void devbuf_release(void* p, hipStream_t stream, bool cached) noexcept {
    if (cached) cache_free(p, stream);
    else (void)hipFreeAsync(p, stream);
}
DevBuf::~DevBuf() {
    if (p && !fixed) devbuf_release(p, stream, cached);
}
DevBuf& DevBuf::operator=(DevBuf&& o) noexcept {
    if (this != &o) {
        if (p && !fixed) devbuf_release(p, stream, cached);
        p = o.p;
        bytes = o.bytes;
        stream = o.stream;
        cached = o.cached;
        fixed = o.fixed;
        o.p = nullptr;
        o.bytes = 0;
        o.cached = false;
        o.fixed = false;
    }
    return *this;
}

void* dev_alloc(size_t bytes) {
    injected_failure(bytes);
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, std::max<size_t>(bytes, 16));
    if (e != hipSuccess) {
        // idle query scratch kept by the block cache may be what is missing
        (void)hipGetLastError();
        cache_release_idle();
        e = hipMalloc(&p, std::max<size_t>(bytes, 16));
    }
    if (e != hipSuccess)
        throw Error{ISAX_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e)};
    return p;
}

template <class T>
static T* own(isax_index* idx, size_t count) {
    T* p = static_cast<T*>(dev_alloc(count * sizeof(T)));
    idx->owned.push_back(p);
    idx->device_bytes += (int64_t)(count * sizeof(T));
    return p;
}

// Carves aligned sub-arrays out of one stream-ordered allocation.
struct Arena {
    size_t off = 0;
    std::vector<std::pair<void**, size_t>> reqs;
    template <class T>
    void add(T** p, size_t count) {
        reqs.push_back({reinterpret_cast<void**>(p), off});
        off += (count * sizeof(T) + 255) / 256 * 256;
    }
    DevBuf commit(hipStream_t s) {
        DevBuf b(std::max<size_t>(off, 256), s);
        for (auto& r : reqs) *r.first = static_cast<char*>(b.p) + r.second;
        return b;
    }
};

}  // namespace isax

isax_index::~isax_index() {
    for (void* p : owned) (void)hipFree(p);
}

using namespace isax;

// =============================================================================================
// Build
namespace {

// A pointer the kernels dereference must be device memory or pinned host
// memory mapped at the same address; anything else (pageable host memory, a
// stale pointer) is rejected before any device work.
bool is_host_memory(const void* p) {
    hipPointerAttribute_t attr;
    std::memset(&attr, 0, sizeof(attr));
    const hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) (void)hipGetLastError();
    return e == hipSuccess && attr.type == hipMemoryTypeHost;
}

void require_device_accessible(const void* p, const char* name) {
    hipPointerAttribute_t attr;
    std::memset(&attr, 0, sizeof(attr));
    const hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) (void)hipGetLastError();
    if (e != hipSuccess || attr.devicePointer == nullptr)
        throw Error{ISAX_EINVAL, std::string(name) + " is not device memory or pinned host memory"};
    if (attr.devicePointer != p)
        throw Error{ISAX_EINVAL, std::string(name) + " is not mapped at the same address on the device"};
}

int default_key_bits(int w, int c) {
    int b = std::min(64, w * c);
    return (b + 7) / 8 * 8 > 64 ? 64 : (b + 7) / 8 * 8;
}

void validate_series_shape(const float* data, int64_t n, int32_t len, int32_t w, int32_t c) {
    ISAX_REQUIRE(data != nullptr, "data is NULL");
    ISAX_REQUIRE(n >= 1, "n must be >= 1");
    ISAX_REQUIRE(n < (int64_t(1) << 31), "n must be < 2^31");
    ISAX_REQUIRE(len >= 1 && len <= ISAX_MAX_LEN, "len must be in 1..4096");
    ISAX_REQUIRE(w >= 1 && w <= ISAX_MAX_SEGMENTS, "segments must be in 1..64");
    ISAX_REQUIRE(len % w == 0, "segments must divide len (segments of equal length)");
    ISAX_REQUIRE(c >= 1 && c <= 8, "card_bits must be in 1..8");
    ISAX_REQUIRE((reinterpret_cast<uintptr_t>(data) & 3) == 0, "data must be 4-byte aligned");
}

// Empirical region edges (isax_build_options.edges): the FP32 PAA of every
// segment of S = ceil(kEdgeSample / w) evenly spaced series (at most n), and
// edge j = the ceil(j V / 2^c)-th smallest of those V = S w values (the
// inverted-CDF quantile at j / 2^c).  Nested across c like the normal ones.
constexpr int kEdgeSample = 65536;
std::vector<float> empirical_edges(const float* data, int64_t n, int len, int w, int c, hipStream_t s) {
    const int S = (int)std::min<int64_t>(n, (kEdgeSample + w - 1) / w);
    DevBuf buf((size_t)S * w * sizeof(float), s);
    launch_paa_sample(data, n, len, w, S, buf.as<float>(), s);
    std::vector<float> v((size_t)S * w);
    ISAX_HIP(hipMemcpyAsync(v.data(), buf.p, v.size() * sizeof(float), hipMemcpyDeviceToHost, s));
    ISAX_HIP(hipStreamSynchronize(s));
    // a non-finite value is rejected by the summarise pass; keep it out of the sort
    v.erase(std::remove_if(v.begin(), v.end(), [](float x) { return !(std::fabs(x) <= 3.4028235e38f); }), v.end());
    std::sort(v.begin(), v.end());
    const int64_t V = (int64_t)v.size();
    std::vector<float> b((size_t)(1 << c) - 1, 0.f);
    for (int j = 1; j < (1 << c) && V > 0; ++j) {
        const int64_t r = (j * V + (1 << c) - 1) / (1 << c) - 1;  // ceil(j V / 2^c) - 1
        b[j - 1] = v[(size_t)std::max<int64_t>(0, r)];
    }
    return b;
}

float* upload_beta(int c, hipStream_t s, DevBuf* tmp, isax_index* idx, const std::vector<float>* edges = nullptr) {
    const std::vector<float> b = edges ? *edges : breakpoints_f32(c);
    if (idx) idx->beta_host = b;
    float* d = idx ? own<float>(idx, b.size()) : nullptr;
    if (!idx) {
        *tmp = DevBuf(b.size() * sizeof(float), s);
        d = tmp->as<float>();
    }
    ISAX_HIP(hipMemcpyAsync(d, b.data(), b.size() * sizeof(float), hipMemcpyHostToDevice, s));
    return d;
}

// The spectral copy's transform, transposed: entry (j, i) = T_ij of the
// orthonormal DCT-II of length len, T_ij = sqrt((i ? 2 : 1) / len)
// cos(pi i (2j + 1) / (2 len)), for coefficients i < D - 1; column D - 1 (the
// slot of the tail norm) is zero.  The angle is reduced modulo its period
// 4 len (in units of pi / (2 len)) before the cosine.
std::vector<double> spectral_table(int len, int D) {
    std::vector<double> t((size_t)len * D, 0.0);
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < D - 1; ++i) {
        const double c = std::sqrt((i == 0 ? 1.0 : 2.0) / len);
        for (int j = 0; j < len; ++j) {
            const int64_t k = (int64_t)i * (2 * j + 1) % (4 * len);
            t[(size_t)j * D + i] = c * std::cos(pi * (double)k / (2.0 * len));
        }
    }
    return t;
}

// D of the spectral copy for an option value (0: three quarters of the padded
// length rounded down to a multiple of 64, within 64..256).  At 100M x 256
// random walks, D = 128 left 27K candidates per far query (sigma = 1) and
// its filter pass was slower than the full rows'; D = 192 left 3.6K and
// took 0.88 of the full pass.
int spectral_dim_for(int len, int opt) {
    return opt ? opt : std::min(256, std::max(64, filter_len_pad(len) * 3 / 4 / 64 * 64));
}

isax_index* build_impl(const float* data, int64_t n, int32_t len, int32_t w, int32_t c, const isax_build_options* opt) {
    validate_series_shape(data, n, len, w, c);
    isax_build_options o{};
    if (opt) o = *opt;
    const int leaf = o.leaf_size ? o.leaf_size : 256;
    ISAX_REQUIRE(leaf >= 16 && leaf <= kMaxLeaf, "leaf_size must be in 16..1024");
    const int key_bits = o.key_bits ? o.key_bits : default_key_bits(w, c);
    ISAX_REQUIRE(key_bits >= 8 && key_bits <= 64 && key_bits % 8 == 0, "key_bits must be a multiple of 8 in 8..64");
    ISAX_REQUIRE(o.precision >= 0 && o.precision <= 15,
                 "precision must be a bitmask of 1 (BF16), 2 (FP8), 4 (FP32 rows in leaf order) and 8 (spectral)");
    ISAX_REQUIRE(o.reserved == 0, "reserved must be 0");
    const int spec_dim = (o.precision & 8) ? spectral_dim_for(len, o.spectral_dim) : 0;
    ISAX_REQUIRE(!(o.precision & 8) || (len <= 512 && spec_dim % 64 == 0 && spec_dim >= 64 && spec_dim <= 256 &&
                                        spec_dim < len),
                 "the spectral copy needs len <= 512 and spectral_dim a multiple of 64 in 64..256, below len");
    ISAX_REQUIRE((o.precision & 8) || o.spectral_dim == 0, "spectral_dim needs precision bit 8");
    ISAX_REQUIRE(o.edges == ISAX_EDGES_NORMAL || o.edges == ISAX_EDGES_EMPIRICAL, "edges must be 0 or 1");
    require_device_accessible(data, "data");
    hipStream_t s = static_cast<hipStream_t>(o.stream);

    std::unique_ptr<isax_index> idx(new isax_index());
    ISAX_HIP(hipGetDevice(&idx->device));
    idx->stream = s;
    idx->data = data;
    idx->data_on_host = is_host_memory(data);
    idx->n = n;
    idx->len = len;
    idx->w = w;
    idx->c = c;
    idx->m_seg = len / w;
    idx->ws = word_stride(w);
    idx->ns = 1 << c;
    idx->leaf_size = leaf;
    idx->key_bits = key_bits;
    idx->n_leaves = (n + leaf - 1) / leaf;
    idx->edges = o.edges;
    if (o.edges == ISAX_EDGES_EMPIRICAL) {
        const std::vector<float> e = empirical_edges(data, n, len, w, c, s);
        idx->beta = upload_beta(c, s, nullptr, idx.get(), &e);
    } else {
        idx->beta = upload_beta(c, s, nullptr, idx.get());
    }

    const int ws = idx->ws;
    DevBuf words(n * ws, s), flags(16, s);
    ISAX_HIP(hipMemsetAsync(words.p, 0, n * ws, s));
    ISAX_HIP(hipMemsetAsync(flags.p, 0, 16, s));
    unsigned* d_max = flags.as<unsigned>();
    int* d_bad = reinterpret_cast<int*>(d_max + 1);
    launch_summarise(data, n, len, w, ws, idx->beta, c, words.as<uint8_t>(), d_max, d_bad, s);
    unsigned hflags[2];
    ISAX_HIP(hipMemcpyAsync(hflags, flags.p, 8, hipMemcpyDeviceToHost, s));
    ISAX_HIP(hipStreamSynchronize(s));
    ISAX_REQUIRE(hflags[1] == 0, "data holds a non-finite value");
    std::memcpy(&idx->max_abs, &hflags[0], 4);
    // |FP32 PAA - exact PAA| <= m 2^-24 max|x| for any summation order; use twice that.
    idx->delta = (float)((double)idx->m_seg * std::ldexp(1.0, -23) * idx->max_abs * (1.0 + 1e-6));

    DevBuf keys(n * sizeof(uint64_t), s);
    idx->ids_sorted = own<int32_t>(idx.get(), n);
    launch_make_keys(words.as<uint8_t>(), n, ws, w, c, key_bits, keys.as<uint64_t>(), idx->ids_sorted, s);
    sort_keys(keys.as<uint64_t>(), idx->ids_sorted, n, key_bits, s);
    idx->words_sorted = own<uint8_t>(idx.get(), (size_t)n * ws);
    launch_gather_words(words.as<uint8_t>(), idx->ids_sorted, n, ws, idx->words_sorted, s);
    idx->leaf_key = own<uint64_t>(idx.get(), idx->n_leaves);
    idx->env_lo = own<uint8_t>(idx.get(), (size_t)idx->n_leaves * ws);
    idx->env_hi = own<uint8_t>(idx.get(), (size_t)idx->n_leaves * ws);
    idx->n_nodes = (idx->n_leaves + kNodeLeaves - 1) / kNodeLeaves;
    idx->node_lo = own<uint8_t>(idx.get(), (size_t)idx->n_nodes * ws);
    idx->node_hi = own<uint8_t>(idx.get(), (size_t)idx->n_nodes * ws);
    launch_leaf_layout(keys.as<uint64_t>(), idx->words_sorted, n, ws, leaf, idx->n_leaves, idx->leaf_key, idx->env_lo,
                       idx->env_hi, idx->node_lo, idx->node_hi, s);
    ISAX_REQUIRE((o.precision & 3) == 0 || len <= 512, "the reduced-precision copies support len <= 512");
    if (o.precision & 4) {
        idx->xs = own<float>(idx.get(), (size_t)n * len);
        launch_gather_rows(data, idx->ids_sorted, n, len, idx->xs, s);
    }
    const int lp = filter_len_pad(len);
    if (o.precision & 1) {
        idx->x_bf16 = own<uint16_t>(idx.get(), (size_t)n * lp);
        idx->meta_bf16 = own<float4>(idx.get(), n);
        launch_quantise(data, idx->ids_sorted, n, len, lp, 0, idx->x_bf16, nullptr, idx->meta_bf16, s);
    }
    if (o.precision & 2) {
        idx->x_fp8 = own<uint8_t>(idx.get(), (size_t)n * lp);
        idx->meta_fp8 = own<float4>(idx.get(), n);
        launch_quantise(data, idx->ids_sorted, n, len, lp, 1, nullptr, idx->x_fp8, idx->meta_fp8, s);
    }
    if (o.precision & 8) {
        const std::vector<double> t = spectral_table(len, spec_dim);
        idx->spec_dim = spec_dim;
        idx->spec_t = own<double>(idx.get(), t.size());
        ISAX_HIP(hipMemcpyAsync(idx->spec_t, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice, s));
        idx->x_spec = own<uint16_t>(idx.get(), (size_t)n * spec_dim);
        idx->meta_spec = own<float4>(idx.get(), n);
        launch_spectral(data, idx->ids_sorted, n, len, spec_dim, idx->spec_t, idx->x_spec, idx->meta_spec, s);
        ISAX_HIP(hipStreamSynchronize(s));  // t is read by the copy above
    }
    words = DevBuf();
    keys = DevBuf();
    flags = DevBuf();
    ISAX_HIP(hipStreamSynchronize(s));
    ISAX_HIP(hipGetLastError());
    return idx.release();
}

// =============================================================================================
// Query
struct Batch {
    DevBuf mem;
    QueryArgs a;
    int fcap0 = 0;              // initial filter-candidate capacity (0: default)
    int mode = ISAX_MODE_INDEX; // the mode the batch ran in
    bool hist_valid = false;    // leaf_count / leaf_list hold the leaf pass of every query
    DevBuf list_mem;            // leaf lists of the best-first rounds
    DevBuf cand_mem;            // candidate lists grown for a re-run
    // hybrid batches: positions handed to the filter, the per-query skip flags
    // (1 = filter), and the filter's sub-batch with its gathered rows
    std::vector<int32_t> far;
    std::vector<int> skip;
    std::unique_ptr<Batch> sub;
    DevBuf sub_mem;
    // the per-query state holds an approximate answer already (qprep and the
    // approximate answer are not run again)
    bool prepared = false;
    const int32_t* kq_host = nullptr;  // k per query (host), where the caller knows it
    // hybrid batches: leaves within the first bound per query, -1 where the
    // leaf pass did not run (used by the statistics instead of leaf_count)
    std::vector<int64_t> li;
};

// Slack of comparisons with a DTW best-so-far: the FP32 recurrence sums at
// most 2 len - 1 cells of 3 roundings each along its path, so a value is
// within (2 len + 3) 2^-24 relative of the exact one; the ratio of two such
// values stays below 1 + 8 len 2^-24 (power of two, at least 2^-13).
float dtw_tau_eps(int len) {
    double e = 8.0 * len * std::ldexp(1.0, -24);
    double p = std::ldexp(1.0, -13);
    while (p < e) p *= 2;
    return (float)p;
}

Arena batch_arena(QueryArgs& a, const isax_index* idx, int mq, int kmax, int cap, int metric);

void setup_batch(Batch& b, const isax_index* idx, const float* Q, int mq, const int32_t* kq_dev, int kmax, int cap,
                 int flags, int64_t* out_ids, float* out_dists, hipStream_t s, int metric = ISAX_METRIC_ED,
                 int window = 0) {
    QueryArgs& a = b.a;
    std::memset(&a, 0, sizeof(a));
    a.data = idx->data;
    a.xs = idx->xs;
    a.n = idx->n;
    a.len = idx->len;
    a.w = idx->w;
    a.c = idx->c;
    a.m_seg = idx->m_seg;
    a.ws = idx->ws;
    a.ns = idx->ns;
    a.leaf_size = idx->leaf_size;
    a.n_leaves = idx->n_leaves;
    a.words_sorted = idx->words_sorted;
    a.ids_sorted = idx->ids_sorted;
    a.env_lo = idx->env_lo;
    a.env_hi = idx->env_hi;
    a.node_lo = idx->node_lo;
    a.node_hi = idx->node_hi;
    a.n_nodes = idx->n_nodes;
    a.leaf_key = idx->leaf_key;
    a.beta = idx->beta;
    a.delta_x = idx->delta;
    a.mq = mq;
    a.Q = Q;
    a.kq = kq_dev;
    a.kmax = kmax;
    a.cap = cap;
    a.tau_scale = 1.0f + tau_eps(idx->len);
    a.lb_scale = 1.0f - 1.52587890625e-05f;
    a.flags = flags;
    a.rerun = 0;
    a.out_ids = out_ids;
    a.out_dists = out_dists;
    a.metric = metric;
    a.window = window;
    if (metric == ISAX_METRIC_DTW) {
        // LB_Keogh: FP32 sums of at most len / 16 + 4 terms per lane, then 4 adds
        a.tau_scale = 1.0f + dtw_tau_eps(idx->len);
        a.lbk_scale = 1.0f - dtw_tau_eps(idx->len);
    }
    if (metric == ISAX_METRIC_ED && idx->x_bf16 && !(flags & ISAX_QF_NO_PRECHECK)) {
        // refinement precheck with the full-row BF16 copy (100M x 256, index mode: 888 ->
        // 1,142-1,192 queries/s, rows read per query 5.4M -> 5); the approximate answer
        // prechecks only rows in host memory (on the device it cost 0.13 ms per 1000 queries
        // more than reading the rows).  gamma bounds the FP32 dot of len terms (each product
        // and sum rounded once, any order: 2u per term, with room); kappa as the filter's
        // (FP32 norms and the final sum, at least 2^-14)
        a.pc_home = idx->data_on_host ? 1 : 0;
        a.pc_x = idx->x_bf16;
        a.pc_meta = idx->meta_bf16;
        a.pc_stride = filter_len_pad(idx->len);
        a.pc_gamma = (float)((idx->len + 8) * std::ldexp(1.0, -23));
        double kap = std::ldexp(1.0, -14);
        while (kap < 8.0 * idx->len * std::ldexp(1.0, -24)) kap *= 2;
        a.pc_kappa = (float)kap;
    }
    b.mem = batch_arena(a, idx, mq, kmax, cap, metric).commit(s);
}

// The per-query arrays of a batch, laid out in one block (setup_batch; also
// sizes a batch before it runs).
Arena batch_arena(QueryArgs& a, const isax_index* idx, int mq, int kmax, int cap, int metric) {
    Arena ar;
    ar.add(&a.paa, (size_t)mq * idx->w);
    ar.add(&a.sym, (size_t)mq * idx->ws);
    ar.add(&a.qkey, mq);
    ar.add(&a.qinfo, mq);
    ar.add(&a.edges, (size_t)mq * 2 * idx->ns);
    ar.add(&a.T, (size_t)mq * idx->w * idx->ns);
    ar.add(&a.tau0, mq);
    ar.add(&a.bestk, (size_t)mq * kmax);
    ar.add(&a.cand, (size_t)mq * cap);
    ar.add(&a.cand_count, mq);
    ar.add(&a.home, (size_t)mq * 2);
    ar.add(&a.stats, (size_t)mq * ST_N);
    ar.add(&a.done, mq);
    ar.add(&a.status, mq);
    ar.add(&a.theta, mq);
    ar.add(&a.leaf_hist, (size_t)mq * kLeafBins);
    ar.add(&a.leaf_count, mq);
    ar.add(&a.list_rest, mq);
    ar.add(&a.env_paa, (size_t)mq * 2 * idx->w);
    if (metric == ISAX_METRIC_DTW) ar.add(&a.qenv, (size_t)mq * 2 * idx->len);
    return ar;
}

constexpr int kDefaultCap = 16384;
constexpr int kFilterCap = 1 << 18;  // initial filter candidates kept per query and pass
constexpr int64_t kCandBytesMax = int64_t(16) << 30;  // candidate lists of one batch after growth

std::vector<int64_t> leaves_initial(const Batch& b, hipStream_t s) {
    const int mq = b.a.mq;
    std::vector<unsigned> h(mq);
    ISAX_HIP(hipMemcpyAsync(h.data(), b.a.leaf_count, mq * sizeof(unsigned), hipMemcpyDeviceToHost, s));
    ISAX_HIP(hipStreamSynchronize(s));
    return std::vector<int64_t>(h.begin(), h.end());
}

// Leaf lists kept per query by the leaf pass: every leaf within the first
// bound when there are at most this many, else the rounds bound all leaves.
constexpr int64_t kLeafListMax = 32768;

// The leaf pass of the best-first rounds (histogram, theta, leaf lists).
void leaf_pass(Batch& b, int64_t cap, hipStream_t s) {
    QueryArgs& a = b.a;
    a.leaf_cap = std::max<int64_t>(1, std::min<int64_t>(cap, std::min<int64_t>(a.n_leaves, kLeafListMax)));
    b.list_mem = DevBuf((size_t)a.mq * a.leaf_cap * sizeof(uint2), s);
    a.leaf_list = b.list_mem.as<uint2>();
    launch_leaf_order(a, s);
    b.hist_valid = true;
    // leaf envelopes once per block of queries
    if (profiling_on())
        profile_add_bytes("leaf_order",
                          2.0 * a.ws * a.n_leaves * (((a.qsel ? a.nsel : a.mq) + kHistQueries - 1) / kHistQueries));
}

void fill_stats(const Batch& b, isax_query_stats* out, hipStream_t s) {
    const int mq = b.a.mq;
    std::vector<unsigned long long> st((size_t)mq * ST_N);
    std::vector<float4> qi(mq);
    ISAX_HIP(hipMemcpyAsync(st.data(), b.a.stats, st.size() * 8, hipMemcpyDeviceToHost, s));
    ISAX_HIP(hipMemcpyAsync(qi.data(), b.a.qinfo, qi.size() * sizeof(float4), hipMemcpyDeviceToHost, s));
    ISAX_HIP(hipStreamSynchronize(s));
    const std::vector<int64_t> li = !b.li.empty() ? b.li : b.hist_valid ? leaves_initial(b, s) : std::vector<int64_t>(mq, -1);
    for (int i = 0; i < mq; ++i) {
        const unsigned long long* r = &st[(size_t)i * ST_N];
        out[i].leaves_scanned = (int64_t)r[ST_LEAVES];
        out[i].leaves_kept = (int64_t)r[ST_LEAVES_KEPT];
        out[i].series_bounded = (int64_t)r[ST_SERIES_LB];
        out[i].series_refined = (int64_t)r[ST_REFINED];
        out[i].refine_bytes = (int64_t)r[ST_REFINE_BYTES];
        out[i].candidates = (int64_t)r[ST_CANDS];
        out[i].tau_initial = qi[i].w;
        out[i].tau_final = qi[i].y;
        out[i].dtw_series = (int64_t)r[ST_DTW];
        out[i].dtw_cells = (int64_t)r[ST_DTW_CELLS];
        out[i].leaves_initial = li[i];
        out[i].path = b.mode == ISAX_MODE_HYBRID ? ISAX_MODE_INDEX : b.mode;
        out[i].candidate_capacity = b.a.cap;
    }
    if (b.sub) {
        // queries answered by the filter: its statistics, the first histogram's count
        std::vector<isax_query_stats> fs(b.far.size());
        fill_stats(*b.sub, fs.data(), s);
        for (size_t j = 0; j < b.far.size(); ++j) {
            isax_query_stats& o = out[b.far[j]];
            const int64_t keep = o.leaves_initial;
            o = fs[j];
            o.leaves_initial = keep;
            o.path = ISAX_MODE_BF16;
        }
    }
}

// Algorithmic bytes of the iSAX scan for one batch: per leaf, its envelope
// (2 * word stride) for every pass that bounds it, or its list entry (8 bytes)
// for each of the two rounds; word stride per series bounded; refinement
// bytes read.  `cnt` holds the leaf pass's counts (empty: one pass, no lists).
double scan_bytes(const Batch& b, const isax_index* idx, hipStream_t s, const std::vector<int64_t>& cnt,
                  const std::vector<int>& skip) {
    const int mq = b.a.mq;
    std::vector<unsigned long long> st((size_t)mq * ST_N);
    ISAX_HIP(hipMemcpyAsync(st.data(), b.a.stats, st.size() * 8, hipMemcpyDeviceToHost, s));
    ISAX_HIP(hipStreamSynchronize(s));
    double tot = 0;
    for (int i = 0; i < mq; ++i) {
        if (!skip.empty() && skip[i]) continue;
        const unsigned long long* r = &st[(size_t)i * ST_N];
        double leaf_bytes = 2.0 * idx->ws * r[ST_LEAVES];
        if (!cnt.empty()) leaf_bytes = cnt[i] <= b.a.leaf_cap ? 16.0 * cnt[i] : 2.0 * leaf_bytes;
        // the refinement precheck reads a BF16 row and its metadata per series
        tot += leaf_bytes + (double)idx->ws * r[ST_SERIES_LB] + (double)r[ST_REFINE_BYTES] +
               (2.0 * b.a.pc_stride + 16.0) * r[ST_PRECHECKED];
    }
    return tot;
}

void run_filter_batch(isax_index* idx, Batch& b, int mode, hipStream_t s);  // defined below
void finish_batch(isax_index* idx, Batch& b, int mode, hipStream_t s);
void run_batch(isax_index* idx, Batch& b, int mode, hipStream_t s, int64_t hybrid_limit = 0);

// The iSAX scan after qprep and homeleaf (and the leaf pass, for the
// best-first rounds): one pass in layout order, or round 1 then round 2 over
// the leaf lists.  `cnt` holds the leaf pass's counts; queries with skip set
// are not scanned.
void index_rounds(isax_index* idx, Batch& b, hipStream_t s, const std::vector<int64_t>& cnt,
                  const std::vector<int>& skip) {
    QueryArgs& a = b.a;
    if (a.flags & ISAX_QF_NO_BEST_FIRST) {
        a.round = 0;
        launch_index_scan(a, s);
    } else {
        // blocks per query: enough for the longest list, or every leaf for a
        // query whose list did not fit
        const int64_t full = (a.n_leaves + 255) / 256;
        int64_t g = 0;
        for (int q = 0; q < a.mq; ++q)
            if (skip.empty() || !skip[q]) g = std::max(g, cnt[q] <= a.leaf_cap ? (cnt[q] + 255) / 256 : full);
        a.grid_leaves = g;
        if (g > 0) {
            a.round = 1;
            launch_index_scan(a, s);
            a.round = 2;
            launch_index_scan(a, s);
        }
    }
    if (profiling_on())
        profile_add_bytes(a.metric == ISAX_METRIC_DTW ? "dtw_scan" : "index_scan", scan_bytes(b, idx, s, cnt, skip));
}

// Cost model of the hybrid planner, in seconds (fitted on one MI355X at
// 100M x 256).  The iSAX path reads, for every leaf it still has to bound, the
// words of its series (their bounds) at about kIdxBps, and refines the share
// of them that survives, each at len * 4 bytes at the same rate; the share is
// the one round 1 saw for that query.  Before round 1 (and for a query whose
// list did not fit, which has no round 1 to learn from) a query is priced
// optimistically: its round-1 leaves (the histogram's bins up to theta) at
// kFarShare, the others at kNearShare; a query too dear even then goes to the
// filter without round 1.
// The BF16 filter streams its whole copy once per batch at about
// kFilterStreamBps, computes its padded query rows at about kFilterFlopsWide
// (blocks of 512 rows), kFilterFlopsMid (256 rows) or kFilterFlopsNarrow (the
// smaller block classes), and spends kFilterPerQuery per query on refinement
// and ordering (fitted to 100M x 256: 9.7 ms for 1-64 queries, 10.7 for 128,
// 15.0 for 256, 24.1 for 512, 43.2 for 1000).
constexpr double kIdxBps = 4e12;
constexpr double kFarShare = 0.25;
constexpr double kNearShare = 0.01;  // before round 1: the share of a query close to its answer
constexpr double kFilterStreamBps = 5.5e12;
constexpr double kFilterFlopsWide = 1.4e15;
constexpr double kFilterFlopsMid = 1.05e15;
constexpr double kFilterFlopsNarrow = 0.8e15;
constexpr double kFilterPerQuery = 10e-6;
// The spectral copy (fewer coefficients than the padded length) streams at
// about kSpectralStreamBps and computes at kSpectralRate of the rates above
// (fitted to 100M x 256 with 192 coefficients: 7.4 ms for 1-64 queries, 8.1
// for 100, 9.3 for 128, 14.1 for 256, 19.4 for 512, 35.8 for 1000).
constexpr double kSpectralStreamBps = 5.4e12;
constexpr double kSpectralRate = 0.74;
// The hybrid's own work before and around the split (leaf pass, round 1, a
// second approximate answer for the filter's queries, more synchronisation):
// about 1.5 ms per call at 10M x 256; a batch the filter answers in less than
// kHybridFixed takes the BF16 path at once.
constexpr double kHybridFixed = 3e-3;
// Index work per leaf grows with k beyond the words and refinement the model
// counts (longer best-k lists, wider windows): measured about 1.7x at k = 10.
inline double k_prior(int k) { return 1.0 + 0.7 * std::log10((double)std::max(k, 1)); }
// The pre-screen bounds every kPreStride-th node (64 leaves) of the leaf pass.
constexpr int kPreStride = 16;
// Near queries measured at 1.7-2x their optimistic pre-screen price (100M x 256,
// sigma 0.01 and 0.1, k = 10): the pre-screen scales it by this much for k > 1.
// At k = 1 the bound of a near query tightens at once in round 1 (sigma = 0.1:
// about 11 us per query against pre-screen prices of 50-120 us for those whose
// approximate answer was loose), so its price is left as it is.
constexpr double kPreFactor = 1.5;
inline double pre_factor(int k) { return k > 1 ? kPreFactor : 1.0; }

// Codes per row the BF16 filter reads: D of the spectral copy when the index
// holds one (unless the query asks for the full rows), else the padded length.
int bf16_dim(const isax_index* idx, int flags) {
    return idx->x_spec && !(flags & ISAX_QF_FULL_ROWS) ? idx->spec_dim : filter_len_pad(idx->len);
}

// The planner: `fixed` queries go to the filter; of the others, the j of
// largest cost join them, j minimising filter_cost(all of them) + the cost of
// the queries left on the iSAX path.  Returns the filter's set.
double filter_cost(const isax_index* idx, int f, int dim);
double filter_pass_cost(const isax_index* idx, int f, int dim);
// Keeping any query on the index path also costs its own passes and
// synchronisations (leaf pass, rounds, the second plan): about this much.
constexpr double kIndexFixed = 1.5e-3;
std::vector<char> plan_far(const isax_index* idx, const std::vector<double>& cost, const std::vector<char>& fixed,
                           double fscale, int dim) {
    const int mq = (int)cost.size();
    std::vector<int> order;
    int n0 = 0;
    double rest = 0.0;
    for (int q = 0; q < mq; ++q) {
        if (fixed[q]) {
            ++n0;
        } else {
            order.push_back(q);
            rest += cost[q];
        }
    }
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    const int n = (int)order.size();
    double best = fscale * filter_cost(idx, n0, dim) + rest + (n > 0 ? kIndexFixed : 0.0);
    int bj = 0;
    for (int j = 1; j <= n; ++j) {
        rest -= cost[order[j - 1]];
        const double c = fscale * filter_cost(idx, n0 + j, dim) + rest + (j < n ? kIndexFixed : 0.0);
        if (c < best) {
            best = c;
            bj = j;
        }
    }
    std::vector<char> far = fixed;
    for (int j = 0; j < bj; ++j) far[order[j]] = 1;
    return far;
}

// The pass over the copy (streaming or matrix work, whichever binds) ...
double filter_pass_cost(const isax_index* idx, int f, int dim) {
    if (f == 0) return 0.0;
    const bool spec = dim < filter_len_pad(idx->len);
    const double stream = (double)idx->n * (dim * 2 + 16) / (spec ? kSpectralStreamBps : kFilterStreamBps);
    const int rows = filter_rows_bf16(dim, f);
    const double rate = (rows % 512 == 0 ? kFilterFlopsWide : rows == 256 ? kFilterFlopsMid : kFilterFlopsNarrow) *
                        (spec ? kSpectralRate : 1.0);
    const double mfma = 2.0 * dim * (double)idx->n * rows / rate;
    return std::max(stream, mfma);
}
// ... and the refinement and ordering of its queries.
double filter_cost(const isax_index* idx, int f, int dim) {
    return f == 0 ? 0.0 : filter_pass_cost(idx, f, dim) + f * kFilterPerQuery;
}

// The rows of a hybrid batch's filter sub-batch: positions, gathered queries
// and k, and its answers before they are scattered back.
Arena sub_arena(int32_t** pos, float** Qf, int32_t** kqf, int64_t** oid, float** od, int mf, int len, int kmax) {
    Arena ar;
    ar.add(pos, mf);
    ar.add(Qf, (size_t)mf * len);
    ar.add(kqf, mf);
    ar.add(oid, (size_t)mf * kmax);
    ar.add(od, (size_t)mf * kmax);
    return ar;
}

// Hybrid batch.  The leaf pass of the iSAX path lists, for every query, the
// leaves whose bound is within the approximate answer's best-so-far.  Round 1
// (the listed leaves of smallest bound) lowers the best-so-far of every query
// whose list fit, and the list is counted again: est[q] = the leaves round 2
// would still bound (for a query whose list did not fit, the first count).
// With a limit, the queries with est above it go to the BF16 filter; without,
// the planner prices each query's remaining iSAX work (cost[q], model above)
// and sends the j costliest to the filter, j minimising filter_cost(j) + the
// cost of the others.  The filter's queries are gathered into a sub-batch and
// their answers written back to their rows; the others finish on the iSAX
// path (round 2 over their lists, or both rounds over every leaf for a query
// whose list did not fit).
void run_hybrid_batch(isax_index* idx, Batch& b, hipStream_t s, int64_t limit) {
    QueryArgs& a = b.a;
    const int mq = a.mq;
    const double fscale = (a.flags & ISAX_QF_FILTER_CHEAP) ? 1e-3 : (a.flags & ISAX_QF_FILTER_DEAR) ? 1e3 : 1.0;
    const int fdim = bf16_dim(idx, a.flags);
    if (limit == 0 && !(a.flags & ISAX_QF_NO_SHORTCUT) && fscale * filter_cost(idx, mq, fdim) < kHybridFixed) {
        run_batch(idx, b, ISAX_MODE_BF16, s);
        return;
    }
    launch_qprep(a, s);
    launch_homeleaf(a, s);
    const bool best_first = !(a.flags & ISAX_QF_NO_BEST_FIRST);
    const double leaf_words = (double)a.leaf_size * a.ws / kIdxBps;
    // (with the precheck a refined series reads its BF16 row; its FP32 row only rarely)
    const double leaf_refine = (double)a.leaf_size * (a.pc_x ? a.pc_stride * 2.0 : a.len * 4.0) / kIdxBps;
    std::vector<double> cost(mq), kp(mq);
    for (int q = 0; q < mq; ++q) kp[q] = k_prior(b.kq_host ? b.kq_host[q] : a.kmax);
    std::vector<char> pre(mq, 0);  // sent to the filter before the leaf pass
    std::vector<int> flags_a(mq), flags_b(mq);  // done flags of the launches below (kept alive until a sync)
    if (limit == 0 && best_first) {
        // Pre-screen on a sample of the leaves (every kPreStride-th node of 64
        // leaves, no lists): each query's count within its first bound,
        // scaled up, priced optimistically (its first kFirstLeaves leaves at
        // kFarShare, the others at kNearShare).  Queries too dear for the index
        // even then go to the filter without the full leaf pass.
        a.leaf_stride = kPreStride;
        a.leaf_cap = 0;
        launch_leaf_order(a, s);
        a.leaf_stride = 1;
        int64_t sampled = 0;
        for (int64_t nd = 0; nd * kNodeLeaves < a.n_leaves; nd += kPreStride)
            sampled += std::min<int64_t>(kNodeLeaves, a.n_leaves - nd * kNodeLeaves);
        const double scale = (double)a.n_leaves / (double)std::max<int64_t>(sampled, 1);
        std::vector<unsigned> c(mq);
        ISAX_HIP(hipMemcpyAsync(c.data(), a.leaf_count, mq * sizeof(unsigned), hipMemcpyDeviceToHost, s));
        ISAX_HIP(hipStreamSynchronize(s));
        for (int q = 0; q < mq; ++q) {
            const double est = c[q] * scale, n1 = std::min<double>(est, kFirstLeaves);
            cost[q] = pre_factor(b.kq_host ? b.kq_host[q] : a.kmax) * kp[q] *
                      ((leaf_words + kFarShare * leaf_refine) * n1 + (leaf_words + kNearShare * leaf_refine) * (est - n1));
        }
        pre = plan_far(idx, cost, pre, fscale, fdim);
        double total = 0.0;
        int n_pre = 0;
        for (int q = 0; q < mq; ++q) {
            n_pre += pre[q];
            total += pre[q] ? 0.0 : cost[q];
        }
        if (n_pre == mq) {
            // every query to the filter: the batch itself runs the BF16 path from its approximate answer
            b.li.assign(mq, -1);
            b.prepared = true;
            run_batch(idx, b, ISAX_MODE_BF16, s);
            return;
        }
        if (n_pre == 0 && total < 0.5 * fscale * filter_cost(idx, mq, fdim)) {
            // the index is far cheaper than any filter pass: the plain index path
            leaf_pass(b, kLeafListMax, s);
            const std::vector<int64_t> cnt = leaves_initial(b, s);
            b.li = cnt;
            index_rounds(idx, b, s, cnt, {});
            finish_batch(idx, b, ISAX_MODE_INDEX, s);
            return;
        }
    }
    // the approximate answer of every query (the leaf pass changes no per-query
    // state), kept for the filter's sub-batch: its rows take it instead of
    // computing it again
    Batch shadow;
    setup_batch(shadow, idx, a.Q, mq, a.kq, a.kmax, a.cap, a.flags, nullptr, nullptr, s);
    DevBuf maps((size_t)mq * 2 * sizeof(int2) + (size_t)mq * sizeof(int32_t), s);
    int2* ident = maps.as<int2>();
    int2* fmap = ident + mq;
    int32_t* qsel = reinterpret_cast<int32_t*>(fmap + mq);
    // host sources of the copies below stay alive until the batch's last sync
    std::vector<int2> id(mq), fm;
    std::vector<int32_t> sel;
    for (int q = 0; q < mq; ++q) {
        id[q] = make_int2(q, q);
        if (!pre[q]) sel.push_back(q);
    }
    ISAX_HIP(hipMemcpyAsync(ident, id.data(), mq * sizeof(int2), hipMemcpyHostToDevice, s));
    if ((int)sel.size() < mq)
        ISAX_HIP(hipMemcpyAsync(qsel, sel.data(), sel.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    {
        const FilterArgs none{};
        launch_copy_rows(a, none, shadow.a, none, ident, mq, false, s, false);
    }
    // the leaf pass for the queries that stay (the others keep empty lists)
    if ((int)sel.size() < mq) {
        a.qsel = qsel;
        a.nsel = (int)sel.size();
    }
    leaf_pass(b, kLeafListMax, s);
    a.qsel = nullptr;
    a.nsel = 0;
    std::vector<int64_t> cnt = leaves_initial(b, s);
    b.li = cnt;
    for (int q = 0; q < mq; ++q)
        if (pre[q]) b.li[q] = -1;
    std::vector<char> listed(mq);
    for (int q = 0; q < mq; ++q) listed[q] = best_first && cnt[q] <= a.leaf_cap;
    std::vector<int64_t> est = cnt;
    int64_t g1 = 0;
    for (int q = 0; q < mq; ++q) {
        flags_a[q] = !listed[q] || pre[q];
        if (!flags_a[q]) g1 = std::max(g1, (cnt[q] + 255) / 256);
    }
    if (limit == 0)
        for (int q = 0; q < mq; ++q)
            if (!pre[q]) {
                // not listed: priced from its count at the far share until it is known better
                const int64_t n1 = std::min<int64_t>(cnt[q], kFirstLeaves);
                cost[q] = kp[q] * ((leaf_words + kFarShare * leaf_refine) * (double)n1 +
                                   (leaf_words + kNearShare * leaf_refine) * (double)(cnt[q] - n1));
            }
    if (g1 > 0) {
        // round 1 over the lists
        ISAX_HIP(hipMemcpyAsync(a.done, flags_a.data(), mq * sizeof(int), hipMemcpyHostToDevice, s));
        a.grid_leaves = g1;
        a.round = 1;
        launch_index_scan(a, s);
        launch_list_recount(a, g1, s);
        std::vector<unsigned> r(mq);
        std::vector<unsigned long long> st((size_t)mq * ST_N);
        ISAX_HIP(hipMemcpyAsync(r.data(), a.list_rest, mq * sizeof(unsigned), hipMemcpyDeviceToHost, s));
        ISAX_HIP(hipMemcpyAsync(st.data(), a.stats, st.size() * 8, hipMemcpyDeviceToHost, s));
        ISAX_HIP(hipStreamSynchronize(s));
        for (int q = 0; q < mq; ++q)
            if (!flags_a[q]) {
                est[q] = r[q];
                const unsigned long long* sq = &st[(size_t)q * ST_N];
                const double share = (double)sq[ST_REFINED] / (double)std::max<unsigned long long>(sq[ST_SERIES_LB], 1);
                cost[q] = kp[q] * (leaf_words + std::min(1.0, share) * leaf_refine) * (double)est[q];
            }
    }
    b.skip.assign(mq, 0);
    if (limit > 0) {
        for (int q = 0; q < mq; ++q) b.skip[q] = est[q] > limit;
    } else {
        const std::vector<char> far = plan_far(idx, cost, pre, fscale, fdim);
        for (int q = 0; q < mq; ++q) b.skip[q] = far[q];
    }
    for (int q = 0; q < mq; ++q)
        if (b.skip[q]) b.far.push_back(q);
    const int mf = (int)b.far.size();
    if (mf == mq) {
        // every query to the filter: the batch itself runs the BF16 path from its
        // approximate answer (round 1's results dropped, its bound kept)
        b.far.clear();
        b.skip.clear();
        const FilterArgs none{};
        launch_carry_bound(a, shadow.a, ident, mq, s);  // round 1's bound, before the state is restored
        launch_copy_rows(shadow.a, none, a, none, ident, mq, false, s, false);
        b.prepared = true;
        run_batch(idx, b, ISAX_MODE_BF16, s);
        return;
    }
    int32_t* pos = nullptr;
    int64_t* oid = nullptr;
    float* od = nullptr;
    if (mf > 0) {
        // the filter's sub-batch: the rows' approximate answers, with the bound the
        // index path has found for them since
        float* Qf = nullptr;
        int32_t* kqf = nullptr;
        b.sub_mem = sub_arena(&pos, &Qf, &kqf, &oid, &od, mf, a.len, a.kmax).commit(s);
        fm.resize(mf);
        for (int i = 0; i < mf; ++i) fm[i] = make_int2(b.far[i], i);
        ISAX_HIP(hipMemcpyAsync(pos, b.far.data(), mf * sizeof(int32_t), hipMemcpyHostToDevice, s));
        ISAX_HIP(hipMemcpyAsync(fmap, fm.data(), mf * sizeof(int2), hipMemcpyHostToDevice, s));
        b.sub.reset(new Batch);
        setup_batch(*b.sub, idx, Qf, mf, kqf, a.kmax, a.cap, a.flags, oid, od, s);
        b.sub->fcap0 = b.fcap0;
        const FilterArgs none{};
        launch_copy_rows(shadow.a, none, b.sub->a, none, fmap, mf, false, s, true);
        launch_carry_bound(a, b.sub->a, fmap, mf, s);
        b.sub->prepared = true;
    }
    if (best_first) {
        // round 2 over the lists of the listed queries that stay
        int64_t g2 = 0, n_full = 0;
        for (int q = 0; q < mq; ++q) {
            flags_a[q] = b.skip[q] || !listed[q];
            flags_b[q] = b.skip[q] || listed[q];
            if (!flags_a[q]) g2 = std::max(g2, (cnt[q] + 255) / 256);
            n_full += !flags_b[q];
        }
        if (g2 > 0) {
            ISAX_HIP(hipMemcpyAsync(a.done, flags_a.data(), mq * sizeof(int), hipMemcpyHostToDevice, s));
            a.grid_leaves = g2;
            a.round = 2;
            launch_index_scan(a, s);
        }
        if (n_full > 0) {
            // both rounds over every leaf for the queries whose list did not fit
            ISAX_HIP(hipMemcpyAsync(a.done, flags_b.data(), mq * sizeof(int), hipMemcpyHostToDevice, s));
            a.grid_leaves = (a.n_leaves + 255) / 256;
            a.round = 1;
            launch_index_scan(a, s);
            a.round = 2;
            launch_index_scan(a, s);
        }
        if (profiling_on()) profile_add_bytes("index_scan", scan_bytes(b, idx, s, cnt, b.skip));
    }
    // the iSAX kernels and the final ordering pass over a query whose done flag is set
    ISAX_HIP(hipMemcpyAsync(a.done, b.skip.data(), mq * sizeof(int), hipMemcpyHostToDevice, s));
    if (!best_first) index_rounds(idx, b, s, cnt, b.skip);
    finish_batch(idx, b, ISAX_MODE_INDEX, s);
    if (mf > 0) {
        run_batch(idx, *b.sub, ISAX_MODE_BF16, s);
        launch_scatter_answers(oid, od, pos, mf, a.kmax, a.out_ids, a.out_dists, s);
    }
}

void run_batch(isax_index* idx, Batch& b, int mode, hipStream_t s, int64_t hybrid_limit) {
    QueryArgs& a = b.a;
    b.mode = mode;
    if (mode == ISAX_MODE_HYBRID) {
        run_hybrid_batch(idx, b, s, hybrid_limit);
        return;
    }
    if (!b.prepared) launch_qprep(a, s);  // (prepared batches run the filter path, which clears the flag)
    const bool dtw = a.metric == ISAX_METRIC_DTW;
    if (dtw && mode == ISAX_MODE_SCAN) {
        // the plain scan under DTW: the home leaves seed the bound, then every
        // series gets LB_Keogh and the early-abandoning recurrence
        a.all_leaves = 1;
        launch_homeleaf(a, s);
        launch_index_scan(a, s);
    } else if (mode == ISAX_MODE_INDEX) {
        launch_homeleaf(a, s);
        std::vector<int64_t> cnt;
        if (!(a.flags & ISAX_QF_NO_BEST_FIRST)) {
            leaf_pass(b, kLeafListMax, s);
            cnt = leaves_initial(b, s);
        }
        index_rounds(idx, b, s, cnt, {});
    } else if (mode == ISAX_MODE_SCAN) {
        launch_seed(a, s);
        launch_brute_scan(a, s);
        if (profiling_on()) profile_add_bytes("brute_scan", (double)a.n * a.len * 4.0 * ((a.mq + 63) / 64));
    } else {
        run_filter_batch(idx, b, mode, s);
    }
    finish_batch(idx, b, mode, s);
}

// Final ordering, wide windows, and re-runs of the queries whose candidate
// list overflowed.  A re-run freezes the query's bound at the k-th smallest
// stored value and first grows the lists to hold what the last pass emitted.
void finish_batch(isax_index* idx, Batch& b, int mode, hipStream_t s) {
    QueryArgs& a = b.a;
    const bool dtw = a.metric == ISAX_METRIC_DTW;
    launch_topk(a, s);
    std::vector<int> status(a.mq), wide;
    std::vector<unsigned> counts(a.mq);
    for (int round = 0;; ++round) {
        ISAX_HIP(hipMemcpyAsync(status.data(), a.status, a.mq * sizeof(int), hipMemcpyDeviceToHost, s));
        ISAX_HIP(hipMemcpyAsync(counts.data(), a.cand_count, a.mq * sizeof(unsigned), hipMemcpyDeviceToHost, s));
        ISAX_HIP(hipStreamSynchronize(s));
        bool rerun = false;
        unsigned need = 0;
        wide.clear();
        for (int q = 0; q < a.mq; ++q) {
            if (status[q] == 2) throw Error{ISAX_EDEVICE, "internal error: fewer than k candidates were kept"};
            if (status[q] == 3) wide.push_back(q);
            if (status[q] == 1) {
                rerun = true;
                need = std::max(need, counts[q]);
            }
        }
        if (!wide.empty()) {
            // windows wider than the top-k block's LDS: merged in global memory
            DevBuf wq(wide.size() * sizeof(int), s), vals(wide.size() * (size_t)a.cap * sizeof(double), s);
            ISAX_HIP(hipMemcpyAsync(wq.p, wide.data(), wide.size() * sizeof(int), hipMemcpyHostToDevice, s));
            launch_topk_wide(a, wq.as<int>(), (int)wide.size(), vals.as<double>(), s);
            ISAX_HIP(hipStreamSynchronize(s));
        }
        if (!rerun) break;
        if (round >= 8) throw Error{ISAX_EOVERFLOW, "candidate list overflowed on 8 re-runs"};
        a.rerun = 1;
        if ((int64_t)need > a.cap) {
            const int64_t limit = a.n + 4096;  // every series once, plus the approximate answer's
            const int64_t grow = std::min<int64_t>(std::max<int64_t>(2 * (int64_t)a.cap, need + need / 4), limit);
            ISAX_REQUIRE_CODE(ISAX_ENOMEM, (int64_t)a.mq * grow * 8 <= kCandBytesMax,
                              "candidate lists of this batch would exceed 16 GiB; use a smaller batch");
            b.cand_mem = DevBuf((size_t)a.mq * grow * 8, s);
            a.cand = b.cand_mem.as<unsigned long long>();
            a.cap = (int)grow;
        }
        launch_rerun_reset(a, s);
        if (mode == ISAX_MODE_INDEX || dtw) {
            launch_homeleaf(a, s);
            a.round = 0;  // the bound is frozen: one pass over every leaf
            launch_index_scan(a, s);
        } else if (mode == ISAX_MODE_SCAN) {
            launch_brute_scan(a, s);
        } else {
            run_filter_batch(idx, b, mode, s);
        }
        launch_topk(a, s);
    }
}

size_t batch_scratch_bound(const isax_index* idx, int mq, int kmax, int cap, int64_t fcap, int mode, int metric,
                           int flags);

// `noalloc`: every device buffer of the call comes from the device's fixed
// scratch (isax_query_noalloc); batches of opt->batch queries, or of the
// largest size that fits, and sizes beyond the array are rejected up front.
int query_impl(isax_index* idx, const float* Q, int64_t m, int32_t k, int64_t* out_ids, float* out_dists,
               const isax_query_options* opt, bool noalloc = false) {
    ISAX_REQUIRE(idx != nullptr, "index is NULL");
    ISAX_REQUIRE(m >= 0, "m must be >= 0");
    ISAX_REQUIRE(k >= 1 && k <= ISAX_MAX_K && k <= idx->n, "k must be in 1..min(n, 1024)");
    isax_query_options o{};
    if (opt) o = *opt;
    ISAX_REQUIRE(o.mode >= ISAX_MODE_INDEX && o.mode <= ISAX_MODE_HYBRID, "unknown mode");
    ISAX_REQUIRE(o.hybrid_leaves >= 0, "hybrid_leaves must be >= 0");
    ISAX_REQUIRE(o.candidate_capacity >= 0 && o.batch >= 0, "candidate_capacity and batch must be >= 0");
    ISAX_REQUIRE((o.flags & ~(ISAX_QF_NO_SHARING | ISAX_QF_NO_EARLY_ABANDON | ISAX_QF_NO_BEST_FIRST |
                              ISAX_QF_NO_SHORTCUT | ISAX_QF_FILTER_CHEAP | ISAX_QF_FILTER_DEAR |
                              ISAX_QF_FULL_ROWS | ISAX_QF_NO_PRECHECK)) == 0,
                 "unknown flag");
    ISAX_REQUIRE((o.mode != ISAX_MODE_BF16 && o.mode != ISAX_MODE_HYBRID) || idx->x_bf16 || idx->x_spec,
                 "index was built without a BF16 copy (precision bit 1 or 8)");
    ISAX_REQUIRE(!(o.flags & ISAX_QF_FULL_ROWS) || (o.mode != ISAX_MODE_BF16 && o.mode != ISAX_MODE_HYBRID) ||
                     idx->x_bf16,
                 "ISAX_QF_FULL_ROWS needs the full-length BF16 copy (precision bit 1)");
    ISAX_REQUIRE(o.mode != ISAX_MODE_FP8 || idx->x_fp8, "index was built without the FP8 copy");
    ISAX_REQUIRE(o.metric == ISAX_METRIC_ED || o.metric == ISAX_METRIC_DTW, "unknown metric");
    if (o.metric == ISAX_METRIC_ED) {
        ISAX_REQUIRE(o.window == 0, "window must be 0 for the Euclidean metric");
    } else {
        ISAX_REQUIRE(o.mode == ISAX_MODE_INDEX || o.mode == ISAX_MODE_SCAN,
                     "DTW runs in ISAX_MODE_INDEX or ISAX_MODE_SCAN");
        ISAX_REQUIRE(o.window >= 0 && o.window <= ISAX_MAX_WINDOW && o.window < idx->len,
                     "window must be in 0..min(ISAX_MAX_WINDOW, len - 1)");
        ISAX_REQUIRE(idx->len <= kDtwMaxLen, "DTW takes series of at most 2048 points");
    }
    if (m == 0) return ISAX_OK;
    ISAX_REQUIRE(Q && out_ids && out_dists, "queries and outputs must not be NULL");
    ISAX_REQUIRE((reinterpret_cast<uintptr_t>(Q) & 3) == 0, "queries must be 4-byte aligned");
    require_device_accessible(Q, "queries");
    require_device_accessible(out_ids, "out_ids");
    require_device_accessible(out_dists, "out_dists");
    if (o.k_per_query) require_device_accessible(o.k_per_query, "k_per_query");
    hipStream_t s = static_cast<hipStream_t>(o.stream);
    int cur = 0;
    ISAX_HIP(hipGetDevice(&cur));
    ISAX_REQUIRE(cur == idx->device, "current device differs from the index's device");
    int B = o.batch ? o.batch : 1024;
    const int cap = o.candidate_capacity ? std::max(o.candidate_capacity, k) : kDefaultCap;
    const int64_t fcap = o.candidate_capacity > 0 ? o.candidate_capacity : kFilterCap;
    std::optional<FixedScratchScope> fixed;
    if (noalloc) {
        ISAX_REQUIRE(cur >= 0 && cur < kNoAllocDevices, "device ordinal beyond the no-allocation entry point's table");
        // the call's own blocks (finite check, k per query, staged answers), then one batch at a time
        auto blk = [](size_t n) -> size_t { return (std::max<size_t>(n, 256) + 255) / 256 * 256; };
        const size_t call = blk(4) + (o.k_per_query ? 0 : blk((size_t)m * 4)) + blk((size_t)m * k * 12);
        auto need = [&](int bq) {
            return call + batch_scratch_bound(idx, (int)std::min<int64_t>(bq, m), k, cap, fcap, o.mode, o.metric,
                                              o.flags);
        };
        if (!o.batch) {
            int lo = 1, hi = 1024;  // the largest batch that fits
            while (lo < hi) {
                const int mid = (lo + hi + 1) / 2;
                if (need(mid) <= kNoAllocBytes) lo = mid;
                else hi = mid - 1;
            }
            B = lo;
        }
        ISAX_REQUIRE(need(B) <= kNoAllocBytes,
                     "isax_query_noalloc: " + std::to_string(m) + " queries of length " + std::to_string(idx->len) +
                         " with k = " + std::to_string(k) + " in batches of " + std::to_string(std::min<int64_t>(B, m)) +
                         " need " + std::to_string(need(B)) + " bytes of scratch; its fixed array holds " +
                         std::to_string(kNoAllocBytes) + " (use fewer queries, a smaller batch or k)");
        fixed.emplace(cur, s);
    }

    // validation of values before any output is written
    {
        DevBuf flag(4, s);
        ISAX_HIP(hipMemsetAsync(flag.p, 0, 4, s));
        launch_check_finite(Q, m * idx->len, flag.as<int>(), s);
        int bad = 0;
        ISAX_HIP(hipMemcpyAsync(&bad, flag.p, 4, hipMemcpyDeviceToHost, s));
        ISAX_HIP(hipStreamSynchronize(s));
        ISAX_REQUIRE(bad == 0, "queries hold a non-finite value");
    }
    DevBuf kdev;
    const int32_t* kq = o.k_per_query;
    std::vector<int32_t> hk(m, k);  // k per query on the host too (the hybrid planner prices by k)
    if (kq) {
        ISAX_HIP(hipMemcpyAsync(hk.data(), kq, m * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        ISAX_HIP(hipStreamSynchronize(s));
        for (int32_t v : hk) ISAX_REQUIRE(v >= 1 && v <= k, "k_per_query values must be in 1..k");
    } else {
        kdev = DevBuf(m * sizeof(int32_t), s);
        ISAX_HIP(hipMemcpyAsync(kdev.p, hk.data(), m * sizeof(int32_t), hipMemcpyHostToDevice, s));
        ISAX_HIP(hipStreamSynchronize(s));
        kq = kdev.as<int32_t>();
    }
    const int64_t hybrid_limit = o.hybrid_leaves;  // 0: the planner
    // Answers (and statistics) are staged and copied to the caller's buffers
    // only once every batch has succeeded: an error leaves the outputs untouched.
    DevBuf stage((size_t)m * k * (sizeof(int64_t) + sizeof(float)), s);
    int64_t* st_ids = stage.as<int64_t>();
    float* st_dists = reinterpret_cast<float*>(st_ids + (size_t)m * k);
    std::vector<isax_query_stats> st_host(o.stats ? (size_t)m : 0);
    for (int64_t q0 = 0; q0 < m; q0 += B) {
        const int mq = (int)std::min<int64_t>(B, m - q0);
        // fixed scratch: the next batch reuses this one's blocks (stream order)
        const size_t mark = fixed ? fixed->fx.off : 0;
        {
            Batch b;
            setup_batch(b, idx, Q + q0 * idx->len, mq, kq + q0, k, cap, o.flags, st_ids + q0 * k,
                        st_dists + q0 * k, s, o.metric, o.window);
            b.fcap0 = (int)fcap;
            b.kq_host = hk.data() + q0;
            run_batch(idx, b, o.mode, s, hybrid_limit);
            if (o.stats) fill_stats(b, st_host.data() + q0, s);
        }
        if (fixed) fixed->fx.off = mark;
    }
    ISAX_HIP(hipMemcpyAsync(out_ids, st_ids, (size_t)m * k * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    ISAX_HIP(hipMemcpyAsync(out_dists, st_dists, (size_t)m * k * sizeof(float), hipMemcpyDeviceToDevice, s));
    ISAX_HIP(hipStreamSynchronize(s));
    if (o.stats) std::memcpy(o.stats, st_host.data(), (size_t)m * sizeof(isax_query_stats));
    return ISAX_OK;
}

template <class F>
int guarded(F&& f) {
    clear_error();
    try {
        return f();
    } catch (const Error& e) {
        set_error(e.code, e.msg);
        return e.code;
    } catch (const std::bad_alloc&) {
        set_error(ISAX_ENOMEM, "host allocation failed");
        return ISAX_ENOMEM;
    } catch (const std::exception& e) {
        set_error(ISAX_EDEVICE, e.what());
        return ISAX_EDEVICE;
    }
}

}  // namespace

// =============================================================================================
// Reduced-precision filter batch (kernels in filter_kernels.hip)
namespace {

// gamma: FP32 accumulation error of dim exact products, any order and
// rounding (2u per add).  kappa: relative slack on |q|^2 + |x|^2 covering the
// FP32 norms and the epilogue, never below 2^-14.
void filter_constants(int len, int dim, float* gamma, float* kappa) {
    *gamma = (float)(dim * std::ldexp(1.0, -23));
    double k = std::ldexp(1.0, -14);
    while (k < 8.0 * len * std::ldexp(1.0, -24)) k *= 2;
    *kappa = (float)k;
}

struct FilterScratch {
    DevBuf mem, cand;
    FilterArgs f{};
    unsigned* qmax = nullptr;
    int mq_pad = 0;
};

void alloc_filter_cands(FilterScratch& fs, int mq, int64_t fcap, hipStream_t s) {
    ISAX_REQUIRE((int64_t)mq * fcap * 4 <= (int64_t(32) << 30),
                 "filter candidates of this batch exceed 32 GiB; use a smaller batch");
    fs.cand = DevBuf();
    fs.cand = DevBuf((size_t)mq * fcap * 4, s);
    fs.f.fcand = fs.cand.as<unsigned>();
    fs.f.fcap = (int)fcap;
}

// The filter's per-query arrays (query codes, factors, counts) in one block.
Arena filter_arena(FilterScratch& fs, unsigned char** qq, const isax_index* idx, int mq, int kind, int dim) {
    const int qpb = filter_queries_per_block(idx->len);
    fs.mq_pad = (mq + qpb - 1) / qpb * qpb;
    Arena ar;
    ar.add(qq, (size_t)fs.mq_pad * dim * (kind == 0 ? 2 : 1));
    ar.add(&fs.f.qmeta, fs.mq_pad);
    ar.add(&fs.qmax, 4);
    ar.add(&fs.f.fcount, mq);
    return ar;
}

// `fcap`: filter candidates kept per query before the buffer grows.
void setup_filter(FilterScratch& fs, const isax_index* idx, const QueryArgs& a, int mode, int64_t fcap,
                  hipStream_t s, bool full_rows = false) {
    FilterArgs& f = fs.f;
    f.kind = mode == ISAX_MODE_BF16 ? 0 : 1;
    if (f.kind == 0 && idx->x_spec && !(a.flags & ISAX_QF_FULL_ROWS) && !full_rows) {
        f.dim = idx->spec_dim;
        f.spec = idx->spec_t;
        f.xq = idx->x_spec;
        f.xmeta = idx->meta_spec;
    } else {
        ISAX_REQUIRE(f.kind == 1 || idx->x_bf16, "index was built without the full-length BF16 copy");
        f.dim = filter_len_pad(idx->len);
        f.xq = f.kind == 0 ? static_cast<const void*>(idx->x_bf16) : static_cast<const void*>(idx->x_fp8);
        f.xmeta = f.kind == 0 ? idx->meta_bf16 : idx->meta_fp8;
    }
    filter_constants(idx->len, f.dim, &f.gamma, &f.kappa);
    f.phase = 0;
    unsigned char* qq = nullptr;
    fs.mem = filter_arena(fs, &qq, idx, a.mq, f.kind, f.dim).commit(s);
    f.qq = qq;
    f.mq_pad = fs.mq_pad;
    alloc_filter_cands(fs, a.mq, fcap, s);
    ISAX_HIP(hipMemsetAsync(fs.qmax, 0, 16, s));
    ISAX_HIP(hipMemsetAsync(f.fcount, 0, a.mq * sizeof(unsigned), s));
}

// Filter, then refine its candidates.  On a large collection the filter runs
// in two phases: first one tile in kSub (an even sample of the collection),
// whose refined candidates tighten the best-so-far, then the other tiles.  The
// per-query candidate count is exact even past the buffer, so on overflow the
// buffer grows to fit; in a first pass the stored candidates are refined first,
// which tightens the bound (kept in tau0 while the per-query state restarts),
// and the phases run again.
constexpr int kSub = kFilterSub;

// The spectral copy trades matrix work for candidates: where the dropped
// coefficients matter (queries far from every series, large k) it lets
// through many more series than the full rows do.  When the index also holds
// the full rows, the other units run as a second even sample (phase 4, on the
// spectral copy, after the first sample's candidates have tightened the
// bound) and the rest (phase 5): the second sample's candidate count times the
// units left (kSub - 2 of them per sample unit) is priced at kRefineBps of
// row reads against what the spectral copy saves on the matrix work, and when
// the refinement would cost more the rest (and any re-run) reads the full
// rows.  The saving is taken as half the share of coefficients dropped
// (measured at 100M x 256: 192 of 256 coefficients took 0.88 of the full pass).
constexpr double kRefineBps = 2e12;

void run_filter_batch(isax_index* idx, Batch& b, int mode, hipStream_t s) {
    QueryArgs& a = b.a;
    FilterScratch fs;
    setup_filter(fs, idx, a, mode, b.fcap0 > 0 ? b.fcap0 : kFilterCap, s);
    // a prepared batch holds its approximate answer for this first pass only: every
    // re-run (overflowed lists) computes it again
    if (!b.prepared) launch_homeleaf(a, s);
    b.prepared = false;
    launch_quantise_queries(a, fs.f, fs.mq_pad, fs.qmax, s);
    const int64_t n_tiles = (idx->n + 31) / 32;
    std::vector<int> phases;
    if (n_tiles >= 16 * kSub) phases = {1, 2};
    else phases = {0};
    const int qpb = filter_queries_per_block(idx->len);
    auto bytes_all = [&]() {
        return (double)idx->n * (fs.f.dim * (fs.f.kind == 0 ? 2 : 1) + 16) * ((fs.mq_pad + qpb - 1) / qpb);
    };
    // (not under the no-allocation entry point, whose scratch holds one filter's arrays)
    bool may_switch = fs.f.spec && idx->x_bf16 && phases.size() == 2 && !fixed_scratch();
    if (may_switch) phases = {1, 4, 5};
    std::vector<unsigned> cnt(a.mq);
    for (int attempt = 0;; ++attempt) {
        bool over = false;
        unsigned maxc = 0;
        for (int ph : phases) {
            fs.f.phase = ph;
            ISAX_HIP(hipMemsetAsync(fs.f.fcount, 0, a.mq * sizeof(unsigned), s));
            launch_filter(a, fs.f, fs.qmax, s);
            if (profiling_on())
                profile_add_bytes(fs.f.kind == 0 ? "filter_bf16" : "filter_fp8",
                                  bytes_all() * (ph == 0 ? kSub : ph == 2 ? kSub - 1 : ph == 5 ? kSub - 2 : 1) / kSub);
            ISAX_HIP(hipMemcpyAsync(cnt.data(), fs.f.fcount, a.mq * sizeof(unsigned), hipMemcpyDeviceToHost, s));
            ISAX_HIP(hipStreamSynchronize(s));
            for (unsigned c : cnt) maxc = std::max(maxc, c);
            if (maxc > (unsigned)fs.f.fcap) {
                over = true;
                break;
            }
            launch_refine_filtered(a, fs.f, s);
            if (ph == 4 && may_switch) {
                may_switch = false;
                double est = 0.0;
                for (unsigned c : cnt) est += c;
                const double refine = est * (kSub - 2) * idx->len * 4.0 / kRefineBps;
                const int full = filter_len_pad(idx->len);
                const double save = 0.5 * (1.0 - (double)fs.f.dim / full) * filter_pass_cost(idx, a.mq, full);
                if (refine > save) {
                    FilterScratch fr;
                    setup_filter(fr, idx, a, mode, fs.f.fcap, s, true);
                    launch_quantise_queries(a, fr.f, fr.mq_pad, fr.qmax, s);
                    fs = std::move(fr);
                    if (profiling_on()) profile_add_bytes("filter_full_rows_switch", 1.0);
                }
            }
        }
        if (!over) break;
        if (attempt >= 8) throw Error{ISAX_EOVERFLOW, "filter candidates kept overflowing"};
        if (!a.rerun) {
            launch_refine_filtered(a, fs.f, s);
            launch_filter_tighten(a, fs.f, s);
        } else {
            launch_rerun_reset(a, s);
        }
        int64_t grow = std::max<int64_t>((int64_t)fs.f.fcap * 2, (int64_t)maxc + maxc / 4);
        grow = std::min<int64_t>(grow, idx->n);
        alloc_filter_cands(fs, a.mq, grow, s);
        launch_homeleaf(a, s);
    }
}
}  // namespace

// =============================================================================================
// Serving table of the step-level request loop (serve_sched.cpp).  `slots`
// query rows stay resident (a Batch with the filter's per-row state); a step
// runs the filter over one chunk of the collection for every occupied row and
// refines its candidates, so a row that joined at any chunk has covered the
// whole collection after `chunks` steps (the sweep wraps around).  Rows join
// through an admission batch (approximate answer and query codes, as for a
// batch of their own) whose state is copied into the table; finished rows are
// copied into an ordering batch for the top-k.  An admitted row first runs the
// filter over the sample units of the collection (the batch path's first
// phase), which tightens its bound before it joins; the sweep then covers the
// other units only, so every series is met exactly once.  Free rows carry
// done = 1 and take no part (skip_done).  The filter's bound on the query factors is a
// running maximum over every row admitted so far, an upper bound of each
// row's own.  Two steps may be queued at a time: the host staging is double
// buffered, and a step's answers are read once its event has completed.
namespace isax {
constexpr int kServeCand = 16384;   // candidate slots per row (the query's list)
constexpr int kServeFcap = 65536;   // filter candidates per row and step
constexpr int kServeHomeLeaves = 2; // leaves of an admitted row's approximate answer (1: p50 34.5 ms at 15K queries/s offered, 100M x 256; 2: 27.2 ms; 4: 28.7 ms)

struct StepTable {
    isax_index* idx = nullptr;
    int mode = ISAX_MODE_BF16, slots = 0, chunks = 0, kmax = ISAX_MAX_K;
    int64_t chunk_len = 0;          // series per chunk (a multiple of kFilterAlign)
    hipStream_t s = nullptr;
    Batch tab, adm, fin;            // the table, the admission batch, the ordering batch
    FilterScratch ftab, fadm;
    DevBuf dev;                     // device side of the staging below, the overflow flags
    DevBuf own;                     // query rows and k of the table and the ordering batch, answers
    float* dq = nullptr;            // [slots][len] admitted queries
    int32_t* dk = nullptr;          // [slots] their k
    int2* dmap = nullptr;           // [2 slots] row copies: admission, then final ordering
    int* dovf = nullptr;            // [2 slots] overflow flags: the table's rows, then the admitted rows
    // pinned host staging, one set per queued step
    struct Host {
        float* q = nullptr;
        int32_t* k = nullptr;
        int2* map_adm = nullptr;
        int2* map_fin = nullptr;
        int* ovf = nullptr;
        int* ovf_adm = nullptr;     // [n_adm] the admitted rows' first phase
        int* adm = nullptr;         // [n_adm] their table rows
        int* status = nullptr;
        int64_t* ids = nullptr;
        float* dists = nullptr;
        hipEvent_t done = nullptr;
        int n_fin = 0, hi = 0, n_adm = 0;
    } h[2];
    int64_t launched = 0, collected = 0;
    ~StepTable() {
        for (Host& x : h) {
            (void)hipHostFree(x.q);
            (void)hipHostFree(x.k);
            (void)hipHostFree(x.map_adm);
            (void)hipHostFree(x.map_fin);
            (void)hipHostFree(x.ovf);
            (void)hipHostFree(x.ovf_adm);
            (void)hipHostFree(x.adm);
            (void)hipHostFree(x.status);
            (void)hipHostFree(x.ids);
            (void)hipHostFree(x.dists);
            if (x.done) (void)hipEventDestroy(x.done);
        }
    }
};

namespace {
template <class T>
T* pinned(size_t count) {
    void* p = nullptr;
    if (hipHostMalloc(&p, std::max<size_t>(count, 1) * sizeof(T), 0) != hipSuccess) {
        (void)hipGetLastError();
        throw Error{ISAX_ENOMEM, "pinned host allocation of the serving table failed"};
    }
    return static_cast<T*>(p);
}

// A view of rows [0, m) of a batch's arrays.
QueryArgs rows_view(const QueryArgs& a, int m) {
    QueryArgs v = a;
    v.mq = m;
    return v;
}
}  // namespace

StepTable* step_table_create(isax_index* idx, int mode, int slots, int chunks, hipStream_t s) {
    ISAX_REQUIRE(mode == ISAX_MODE_BF16 || mode == ISAX_MODE_FP8, "step-level serving runs the BF16 or FP8 filter");
    ISAX_REQUIRE(mode != ISAX_MODE_BF16 || idx->x_bf16 || idx->x_spec, "index was built without a BF16 copy");
    ISAX_REQUIRE(mode != ISAX_MODE_FP8 || idx->x_fp8, "index was built without the FP8 copy");
    ISAX_REQUIRE(slots >= 1 && slots <= 4096 && chunks >= 1 && chunks <= 1024, "bad serving table size");
    std::unique_ptr<StepTable> t(new StepTable);
    t->idx = idx;
    t->mode = mode;
    t->slots = slots;
    t->s = s;
    t->chunk_len = std::max<int64_t>(kFilterAlign, (idx->n + chunks - 1) / chunks / kFilterAlign * kFilterAlign);
    t->chunks = (int)((idx->n + t->chunk_len - 1) / t->chunk_len);
    std::vector<int32_t> ones(slots, 1);
    Arena ar;
    ar.add(&t->dq, (size_t)slots * idx->len);
    ar.add(&t->dk, slots);
    ar.add(&t->dmap, 2 * (size_t)slots);
    ar.add(&t->dovf, 2 * (size_t)slots);
    t->dev = ar.commit(s);
    ISAX_HIP(hipMemcpyAsync(t->dk, ones.data(), slots * sizeof(int32_t), hipMemcpyHostToDevice, s));
    setup_batch(t->tab, idx, t->dq, slots, t->dk, t->kmax, kServeCand, 0, nullptr, nullptr, s);
    setup_batch(t->adm, idx, t->dq, slots, t->dk, t->kmax, kServeCand, 0, nullptr, nullptr, s);
    setup_batch(t->fin, idx, t->dq, slots, t->dk, t->kmax, kServeCand, 0, nullptr, nullptr, s);
    t->adm.a.home_leaves = kServeHomeLeaves;
    // the table and the ordering batch hold their own query rows and k (copied with the state)
    {
        t->own = DevBuf((size_t)slots * (idx->len * 4 + 4) * 2 + (size_t)slots * t->kmax * 12, s);
        float* tq = t->own.as<float>();
        int32_t* tk = reinterpret_cast<int32_t*>(tq + (size_t)slots * idx->len);
        float* fq = reinterpret_cast<float*>(tk + slots);
        int32_t* fk = reinterpret_cast<int32_t*>(fq + (size_t)slots * idx->len);
        int64_t* oid = reinterpret_cast<int64_t*>(fk + slots);
        float* od = reinterpret_cast<float*>(oid + (size_t)slots * t->kmax);
        t->tab.a.Q = tq;
        t->tab.a.kq = tk;
        t->fin.a.Q = fq;
        t->fin.a.kq = fk;
        t->fin.a.out_ids = oid;
        t->fin.a.out_dists = od;
        ISAX_HIP(hipMemcpyAsync(tk, ones.data(), slots * sizeof(int32_t), hipMemcpyHostToDevice, s));
    }
    t->tab.a.skip_done = 1;
    setup_filter(t->ftab, idx, t->tab.a, mode, kServeFcap, s);
    setup_filter(t->fadm, idx, t->adm.a, mode, kServeFcap, s);
    // every table row free: done = 1
    ISAX_HIP(hipMemcpyAsync(t->tab.a.done, ones.data(), slots * sizeof(int), hipMemcpyHostToDevice, s));
    for (StepTable::Host& x : t->h) {
        x.q = pinned<float>((size_t)slots * idx->len);
        x.k = pinned<int32_t>(slots);
        x.map_adm = pinned<int2>(slots);
        x.map_fin = pinned<int2>(slots);
        x.ovf = pinned<int>(slots);
        x.ovf_adm = pinned<int>(slots);
        x.adm = pinned<int>(slots);
        x.status = pinned<int>(slots);
        x.ids = pinned<int64_t>((size_t)slots * t->kmax);
        x.dists = pinned<float>((size_t)slots * t->kmax);
        ISAX_HIP(hipEventCreateWithFlags(&x.done, hipEventDisableTiming));
    }
    ISAX_HIP(hipStreamSynchronize(s));
    return t.release();
}

void step_table_destroy(StepTable* t) {
    if (!t) return;
    (void)hipStreamSynchronize(t->s);
    delete t;
}

int step_table_chunks(const StepTable* t) { return t->chunks; }

// Queues one step: queries q [n_adm][len] with k into the free rows adm[]
// (approximate answer and query codes in the admission batch, then the state
// into the rows), chunk `chunk` of the sweep for the occupied rows among
// [0, hi) (filter, refinement, overflow flags), then the final ordering of the
// rows fin[] (their state into the ordering batch, the rows become free, the
// top-k, the answers to the host).
void step_table_launch(StepTable* t, const float* q, const int32_t* k, const int* adm, int n_adm, int chunk, int hi,
                       const int* fin, int n_fin) {
    ISAX_REQUIRE(t->launched - t->collected < 2, "at most two serving steps are queued");
    ISAX_REQUIRE(n_adm >= 0 && n_fin >= 0 && n_adm + n_fin <= t->slots && hi <= t->slots && chunk >= 0 &&
                     chunk < t->chunks,
                 "bad serving step");
    StepTable::Host& x = t->h[t->launched & 1];
    const int len = t->idx->len;
    if (n_adm > 0) {
        std::memcpy(x.q, q, (size_t)n_adm * len * sizeof(float));
        std::memcpy(x.k, k, (size_t)n_adm * sizeof(int32_t));
        for (int i = 0; i < n_adm; ++i) x.map_adm[i] = make_int2(i, adm[i]);
        ISAX_HIP(hipMemcpyAsync(t->dq, x.q, (size_t)n_adm * len * sizeof(float), hipMemcpyHostToDevice, t->s));
        ISAX_HIP(hipMemcpyAsync(t->dk, x.k, (size_t)n_adm * sizeof(int32_t), hipMemcpyHostToDevice, t->s));
        ISAX_HIP(hipMemcpyAsync(t->dmap, x.map_adm, (size_t)n_adm * sizeof(int2), hipMemcpyHostToDevice, t->s));
        const QueryArgs a = rows_view(t->adm.a, n_adm);
        launch_qprep(a, t->s);
        launch_homeleaf(a, t->s);
        launch_quantise_queries(a, t->fadm.f, t->fadm.mq_pad, t->ftab.qmax, t->s);
        // the sample units, refined into the admitted rows' own lists
        FilterArgs f1 = t->fadm.f;
        f1.phase = 1;
        launch_filter(a, f1, t->ftab.qmax, t->s);
        launch_refine_filtered(a, f1, t->s);
        launch_note_overflow(a, f1, t->dovf + t->slots, t->s);
        ISAX_HIP(hipMemcpyAsync(x.ovf_adm, t->dovf + t->slots, (size_t)n_adm * sizeof(int), hipMemcpyDeviceToHost,
                                t->s));
        launch_copy_rows(a, t->fadm.f, t->tab.a, t->ftab.f, t->dmap, n_adm, false, t->s);
    }
    x.n_adm = n_adm;
    std::copy(adm, adm + n_adm, x.adm);
    x.hi = hi;
    if (hi > 0) {
        const QueryArgs a = rows_view(t->tab.a, hi);
        FilterArgs f = t->ftab.f;
        f.phase = 3;
        f.range_lo = (int64_t)chunk * t->chunk_len;
        f.range_hi = std::min<int64_t>(t->idx->n, f.range_lo + t->chunk_len);
        launch_filter(a, f, t->ftab.qmax, t->s);
        launch_refine_filtered(a, f, t->s);
        launch_note_overflow(a, f, t->dovf, t->s);
        ISAX_HIP(hipMemcpyAsync(x.ovf, t->dovf, (size_t)hi * sizeof(int), hipMemcpyDeviceToHost, t->s));
    }
    x.n_fin = n_fin;
    if (n_fin > 0) {
        for (int i = 0; i < n_fin; ++i) x.map_fin[i] = make_int2(fin[i], i);
        int2* dm = t->dmap + t->slots;
        ISAX_HIP(hipMemcpyAsync(dm, x.map_fin, (size_t)n_fin * sizeof(int2), hipMemcpyHostToDevice, t->s));
        const QueryArgs fa = rows_view(t->fin.a, n_fin);
        FilterArgs none{};
        launch_copy_rows(t->tab.a, t->ftab.f, fa, none, dm, n_fin, true, t->s);
        launch_topk(fa, t->s);
        ISAX_HIP(hipMemcpyAsync(x.status, fa.status, (size_t)n_fin * sizeof(int), hipMemcpyDeviceToHost, t->s));
        ISAX_HIP(hipMemcpyAsync(x.ids, fa.out_ids, (size_t)n_fin * t->kmax * sizeof(int64_t), hipMemcpyDeviceToHost,
                                t->s));
        ISAX_HIP(hipMemcpyAsync(x.dists, fa.out_dists, (size_t)n_fin * t->kmax * sizeof(float),
                                hipMemcpyDeviceToHost, t->s));
    }
    ISAX_HIP(hipEventRecord(x.done, t->s));
    ++t->launched;
}

// Waits for the oldest queued step: ovf (host, its hi) <- rows that lost filter
// candidates in its sweep; ids / dists (host, [n_fin][kout]) and status (0,
// else the row must be answered alone) of its final ordering.
void step_table_collect(StepTable* t, int* ovf, int kout, int64_t* ids, float* dists, int* status) {
    ISAX_REQUIRE(t->collected < t->launched, "no serving step is queued");
    StepTable::Host& x = t->h[t->collected & 1];
    ISAX_HIP(hipEventSynchronize(x.done));
    std::memcpy(ovf, x.ovf, (size_t)x.hi * sizeof(int));
    for (int i = 0; i < x.n_adm; ++i)
        if (x.ovf_adm[i]) ovf[x.adm[i]] = 1;
    for (int i = 0; i < x.n_fin; ++i) {
        status[i] = x.status[i];
        std::memcpy(ids + (size_t)i * kout, x.ids + (size_t)i * t->kmax, (size_t)kout * sizeof(int64_t));
        std::memcpy(dists + (size_t)i * kout, x.dists + (size_t)i * t->kmax, (size_t)kout * sizeof(float));
    }
    ++t->collected;
}

// After a failure: nothing is queued any more and every row is free.
void step_table_reset(StepTable* t) {
    (void)hipStreamSynchronize(t->s);
    (void)hipGetLastError();
    t->collected = t->launched;
    std::vector<int> ones(t->slots, 1);
    ISAX_HIP(hipMemcpyAsync(t->tab.a.done, ones.data(), t->slots * sizeof(int), hipMemcpyHostToDevice, t->s));
    ISAX_HIP(hipStreamSynchronize(t->s));
}
}  // namespace isax

namespace {
// Upper bound of the device scratch one batch of mq queries takes through
// DevBuf (every block rounded up to 256 bytes) before its candidate lists grow
// or a wide tie window is merged: the batch's arrays, the leaf lists of the
// best-first rounds, the filter's arrays and candidates, and for a hybrid
// batch the filter's sub-batch with its gathered rows.
size_t batch_scratch_bound(const isax_index* idx, int mq, int kmax, int cap, int64_t fcap, int mode, int metric,
                           int flags) {
    auto blk = [](size_t n) -> size_t { return (std::max<size_t>(n, 256) + 255) / 256 * 256; };
    QueryArgs t;
    std::memset(&t, 0, sizeof(t));
    const size_t batch = blk(batch_arena(t, idx, mq, kmax, cap, metric).off);
    const int64_t leaf_cap = std::max<int64_t>(1, std::min<int64_t>(idx->n_leaves, kLeafListMax));
    const size_t lists = blk((size_t)mq * leaf_cap * sizeof(uint2));
    auto filter = [&](int kind) {
        FilterScratch fs;
        unsigned char* qq = nullptr;
        return blk(filter_arena(fs, &qq, idx, mq, kind, filter_len_pad(idx->len)).off) + blk((size_t)mq * fcap * 4);
    };
    size_t tot = batch;
    if (mode == ISAX_MODE_INDEX && !(flags & ISAX_QF_NO_BEST_FIRST)) tot += lists;
    if (mode == ISAX_MODE_BF16 || mode == ISAX_MODE_FP8) tot += filter(mode == ISAX_MODE_BF16 ? 0 : 1);
    if (mode == ISAX_MODE_HYBRID) {
        // the batch alone on the filter, or the leaf pass and a sub-batch of at most mq queries
        int32_t *pos, *kqf;
        float *Qf, *od;
        int64_t* oid;
        tot += lists + blk(sub_arena(&pos, &Qf, &kqf, &oid, &od, mq, idx->len, kmax).off) + batch + filter(0);
    }
    return tot;
}
}  // namespace

int64_t isax::query_scratch_bytes(const isax_index* idx, int mq, int kmax, int mode) {
    return (int64_t)batch_scratch_bound(idx, mq, kmax, kDefaultCap, kFilterCap, mode, ISAX_METRIC_ED, 0);
}

// =============================================================================================
extern "C" {

const char* isax_last_error(void) { return g_err_msg.c_str(); }

isax_index* isax_build_ex(const float* data, int64_t n, int32_t len, int32_t segments, int32_t card_bits,
                          const isax_build_options* opt) {
    isax_index* out = nullptr;
    guarded([&] {
        out = build_impl(data, n, len, segments, card_bits, opt);
        return ISAX_OK;
    });
    return out;
}

isax_index* isax_build(const float* data, int64_t n, int32_t len, int32_t segments, int32_t card_bits) {
    return isax_build_ex(data, n, len, segments, card_bits, nullptr);
}

void isax_free(isax_index* idx) {
    if (!idx) return;
    (void)hipStreamSynchronize(idx->stream);
    delete idx;
}

int isax_query_ex(isax_index* idx, const float* queries, int64_t m, int32_t k, int64_t* out_ids, float* out_dists,
                  const isax_query_options* opt) {
    return guarded([&] { return query_impl(idx, queries, m, k, out_ids, out_dists, opt); });
}

int isax_query_noalloc(isax_index* idx, const float* queries, int64_t m, int32_t k, int64_t* out_ids,
                       float* out_dists, const isax_query_options* opt) {
    return guarded([&] { return query_impl(idx, queries, m, k, out_ids, out_dists, opt, true); });
}

int isax_query(isax_index* idx, const float* queries, int64_t m, int32_t k, int64_t* out_ids, float* out_dists) {
    return isax_query_ex(idx, queries, m, k, out_ids, out_dists, nullptr);
}

int isax_breakpoints(int32_t card_bits, float* out) {
    return guarded([&] {
        ISAX_REQUIRE(card_bits >= 1 && card_bits <= 8, "card_bits must be in 1..8");
        ISAX_REQUIRE(out != nullptr, "out is NULL");
        const std::vector<float> b = breakpoints_f32(card_bits);
        std::memcpy(out, b.data(), b.size() * sizeof(float));
        return ISAX_OK;
    });
}

int isax_summarize(const float* data, int64_t n, int32_t len, int32_t segments, int32_t card_bits, uint8_t* out_words,
                   float* max_abs, void* stream) {
    return guarded([&] {
        validate_series_shape(data, n, len, segments, card_bits);
        ISAX_REQUIRE(out_words != nullptr, "out_words is NULL");
        require_device_accessible(data, "data");
        require_device_accessible(out_words, "out_words");
        hipStream_t s = static_cast<hipStream_t>(stream);
        DevBuf flags(16, s), bt;
        ISAX_HIP(hipMemsetAsync(flags.p, 0, 16, s));
        launch_check_finite(data, n * len, reinterpret_cast<int*>(flags.as<unsigned>() + 1), s);
        unsigned h[2];
        ISAX_HIP(hipMemcpyAsync(h, flags.p, 8, hipMemcpyDeviceToHost, s));
        ISAX_HIP(hipStreamSynchronize(s));
        ISAX_REQUIRE(h[1] == 0, "data holds a non-finite value");
        const float* beta = upload_beta(card_bits, s, &bt, nullptr);
        launch_summarise(data, n, len, segments, segments, beta, card_bits, out_words, flags.as<unsigned>(),
                         reinterpret_cast<int*>(flags.as<unsigned>() + 1), s);
        ISAX_HIP(hipMemcpyAsync(h, flags.p, 8, hipMemcpyDeviceToHost, s));
        ISAX_HIP(hipStreamSynchronize(s));
        if (max_abs) std::memcpy(max_abs, &h[0], 4);
        return ISAX_OK;
    });
}

int isax_index_breakpoints(const isax_index* idx, float* out) {
    return guarded([&] {
        ISAX_REQUIRE(idx && out, "index and out must not be NULL");
        std::memcpy(out, idx->beta_host.data(), idx->beta_host.size() * sizeof(float));
        return ISAX_OK;
    });
}

void* isax_host_alloc(int64_t bytes) {
    void* p = nullptr;
    const int rc = guarded([&] {
        ISAX_REQUIRE(bytes > 0, "bytes must be > 0");
        const hipError_t e = hipHostMalloc(&p, (size_t)bytes, hipHostMallocDefault);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            throw Error{ISAX_ENOMEM, std::string("hipHostMalloc of ") + std::to_string(bytes) +
                                         " bytes failed: " + hipGetErrorString(e)};
        }
        return ISAX_OK;
    });
    return rc == ISAX_OK ? p : nullptr;
}

void isax_host_free(void* p) {
    if (p) (void)hipHostFree(p);
}

int isax_index_get_info(const isax_index* idx, isax_index_info* out) {
    return guarded([&] {
        ISAX_REQUIRE(idx && out, "index and out must not be NULL");
        out->n = idx->n;
        out->len = idx->len;
        out->segments = idx->w;
        out->card_bits = idx->c;
        out->leaf_size = idx->leaf_size;
        out->key_bits = idx->key_bits;
        out->has_bf16 = idx->x_bf16 != nullptr;
        out->has_fp8 = idx->x_fp8 != nullptr;
        out->has_sorted_rows = idx->xs != nullptr;
        out->edges = idx->edges;
        out->spectral_dim = idx->spec_dim;
        out->reserved = 0;
        out->n_leaves = idx->n_leaves;
        out->max_abs = idx->max_abs;
        out->delta = idx->delta;
        out->device_bytes = idx->device_bytes;
        return ISAX_OK;
    });
}

int isax_index_export(const isax_index* idx, int32_t* ids_sorted, uint8_t* words_sorted, uint8_t* env_lo,
                      uint8_t* env_hi) {
    return guarded([&] {
        ISAX_REQUIRE(idx != nullptr, "index is NULL");
        for (const void* p : {(const void*)ids_sorted, (const void*)words_sorted, (const void*)env_lo, (const void*)env_hi})
            if (p) require_device_accessible(p, "export output");
        hipStream_t s = idx->stream;
        if (ids_sorted)
            ISAX_HIP(hipMemcpyAsync(ids_sorted, idx->ids_sorted, idx->n * 4, hipMemcpyDeviceToDevice, s));
        if (words_sorted)
            ISAX_HIP(hipMemcpy2DAsync(words_sorted, idx->w, idx->words_sorted, idx->ws, idx->w, idx->n,
                                      hipMemcpyDeviceToDevice, s));
        if (env_lo)
            ISAX_HIP(hipMemcpy2DAsync(env_lo, idx->w, idx->env_lo, idx->ws, idx->w, idx->n_leaves,
                                      hipMemcpyDeviceToDevice, s));
        if (env_hi)
            ISAX_HIP(hipMemcpy2DAsync(env_hi, idx->w, idx->env_hi, idx->ws, idx->w, idx->n_leaves,
                                      hipMemcpyDeviceToDevice, s));
        ISAX_HIP(hipStreamSynchronize(s));
        return ISAX_OK;
    });
}

int isax_lower_bounds(isax_index* idx, const float* queries, int64_t m, float* out_lb) {
    return guarded([&] {
        ISAX_REQUIRE(idx != nullptr, "index is NULL");
        ISAX_REQUIRE(m >= 0, "m must be >= 0");
        if (m == 0) return ISAX_OK;
        ISAX_REQUIRE(queries && out_lb, "queries and out_lb must not be NULL");
        require_device_accessible(queries, "queries");
        require_device_accessible(out_lb, "out_lb");
        hipStream_t s = idx->stream;
        std::vector<int32_t> ones(std::min<int64_t>(m, 1024), 1);
        DevBuf kd(ones.size() * 4, s);
        ISAX_HIP(hipMemcpyAsync(kd.p, ones.data(), ones.size() * 4, hipMemcpyHostToDevice, s));
        for (int64_t q0 = 0; q0 < m; q0 += 1024) {
            const int mq = (int)std::min<int64_t>(1024, m - q0);
            Batch b;
            setup_batch(b, idx, queries + q0 * idx->len, mq, kd.as<int32_t>(), 1, 1, 0, nullptr, nullptr, s);
            launch_qprep(b.a, s);
            launch_lower_bounds(b.a, out_lb + q0 * idx->n, s);
        }
        ISAX_HIP(hipStreamSynchronize(s));
        return ISAX_OK;
    });
}

int isax_filter_scores(isax_index* idx, const float* queries, int64_t m, int32_t mode, float* out_approx,
                       float* out_margin) {
    return guarded([&] {
        ISAX_REQUIRE(idx != nullptr, "index is NULL");
        ISAX_REQUIRE(mode == ISAX_MODE_BF16 || mode == ISAX_MODE_FP8, "mode must be ISAX_MODE_BF16 or ISAX_MODE_FP8");
        ISAX_REQUIRE(mode != ISAX_MODE_BF16 || idx->x_bf16 || idx->x_spec, "index was built without a BF16 copy");
        ISAX_REQUIRE(mode != ISAX_MODE_FP8 || idx->x_fp8, "index was built without the FP8 copy");
        ISAX_REQUIRE(m >= 0 && m <= 1024, "m must be in 0..1024");
        if (m == 0) return ISAX_OK;
        ISAX_REQUIRE(queries && out_approx && out_margin, "queries and outputs must not be NULL");
        require_device_accessible(queries, "queries");
        require_device_accessible(out_approx, "out_approx");
        require_device_accessible(out_margin, "out_margin");
        hipStream_t s = idx->stream;
        std::vector<int32_t> ones(m, 1);
        DevBuf kd(m * 4, s);
        ISAX_HIP(hipMemcpyAsync(kd.p, ones.data(), m * 4, hipMemcpyHostToDevice, s));
        Batch b;
        setup_batch(b, idx, queries, (int)m, kd.as<int32_t>(), 1, 1, 0, nullptr, nullptr, s);
        launch_qprep(b.a, s);
        FilterScratch fs;
        setup_filter(fs, idx, b.a, mode, 1, s);
        fs.f.out_approx = out_approx;
        fs.f.out_margin = out_margin;
        launch_quantise_queries(b.a, fs.f, fs.mq_pad, fs.qmax, s);
        launch_filter(b.a, fs.f, fs.qmax, s);
        ISAX_HIP(hipStreamSynchronize(s));
        return ISAX_OK;
    });
}

int isax_profile_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    return ISAX_OK;
}

int isax_profile_reset(void) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    drain_pending_locked();
    g_prof.clear();
    return ISAX_OK;
}

int isax_profile_read(isax_profile_entry* out, int32_t max_entries, int32_t* n_entries) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    drain_pending_locked();
    int i = 0;
    for (auto& kv : g_prof) {
        if (i >= max_entries) break;
        std::memset(&out[i], 0, sizeof(out[i]));
        std::strncpy(out[i].name, kv.first.c_str(), sizeof(out[i].name) - 1);
        out[i].launches = kv.second.launches;
        out[i].total_ms = kv.second.ms;
        out[i].algorithmic_bytes = kv.second.bytes;
        ++i;
    }
    if (n_entries) *n_entries = (int32_t)g_prof.size();
    return ISAX_OK;
}

int isax_debug_fail_allocation(int64_t countdown) {
    g_fail_countdown.store(countdown > 0 ? countdown : 0);
    return ISAX_OK;
}

double isax_clock(void) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // extern "C"
