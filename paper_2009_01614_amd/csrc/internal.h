// Internal declarations shared by the library's translation units.
// Not part of the public ABI (that is include/isax.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/isax.h"

namespace isax {

// ------------------------------------------------------------------ errors
struct Error {
    int code;
    std::string msg;
};

void set_error(int code, const std::string& msg);
void clear_error();

#define ISAX_HIP(call)                                                                       \
    do {                                                                                     \
        hipError_t _e = (call);                                                              \
        if (_e != hipSuccess)                                                                \
            throw ::isax::Error{ISAX_EDEVICE, std::string(#call) + ": " + hipGetErrorString(_e)}; \
    } while (0)

#define ISAX_REQUIRE(cond, text)                                     \
    do {                                                             \
        if (!(cond)) throw ::isax::Error{ISAX_EINVAL, (text)};       \
    } while (0)

#define ISAX_REQUIRE_CODE(code, cond, text)                          \
    do {                                                             \
        if (!(cond)) throw ::isax::Error{(code), (text)};            \
    } while (0)

// ------------------------------------------------------------------ constants
constexpr int kWaveSize = 64;
constexpr int kMaxCandLds = 4096;   // candidates one top-k block sorts in LDS
constexpr int kMaxLeaf = 1024;
constexpr int kNodeLeaves = 64;     // leaves per node of the two-level envelope (one wave of the leaf pass)

inline int word_stride(int w) { return (w + 15) / 16 * 16; }

// Blocks for a grid-stride launch over `items` units of work, `per_block` units
// per block and pass.  Capped so that blocks x threads stays far below 2^32:
// a dispatch counts its work-items in 32 bits, and a larger grid would wrap.
inline unsigned grid_blocks(int64_t items, int64_t per_block, int64_t cap = 1 << 16) {
    int64_t b = (items + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

// Relative slack that covers any-order FP32 rounding of a sum of len squares
// (gamma_len <= len * 2^-24); comparisons against the best-so-far use
// tau * (1 + eps).  Never below 2^-13.
inline float tau_eps(int len) {
    double e = 4.0 * len * std::ldexp(1.0, -24);
    double p = std::ldexp(1.0, -13);
    while (p < e) p *= 2;
    return (float)p;
}

// Region edges Phi^-1(j / 2^c), j = 1..2^c-1, FP32 (breakpoints.cpp).
std::vector<float> breakpoints_f32(int card_bits);

// ------------------------------------------------------------------ profiling
struct ProfScope {
    ProfScope(const char* name, hipStream_t s);
    ~ProfScope();
    const char* name;
    hipStream_t stream;
    hipEvent_t a = nullptr, b = nullptr;
};
bool profiling_on();
void profile_add_bytes(const char* name, double bytes);

// ------------------------------------------------------------------ device scratch
// Fixed scratch of the no-allocation query entry point: a per-device array
// compiled into the library.  While a thread has one active (fixed_scratch()),
// DevBuf carves its memory from it (256-byte aligned, in call order) instead
// of allocating; the owner rewinds `off` to a mark once the work that used
// the memory has been queued, and stream order protects its reuse.
struct FixedScratch {
    char* base = nullptr;
    size_t size = 0;
    size_t off = 0;
    void* carve(size_t n);  // throws ISAX_ENOMEM when the array is exhausted
};
FixedScratch* fixed_scratch();

// Stream-ordered device scratch, released when the object dies.  Blocks of
// 1 MiB to 1 GiB come from the library's block cache (kept after release,
// reused in stream order), others from hipMallocAsync / hipFreeAsync; under
// an active FixedScratch, from that array (nothing to release).
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
    bool cached = false;
    bool fixed = false;
    DevBuf() = default;
    DevBuf(size_t n, hipStream_t s);
    ~DevBuf();
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept { *this = std::move(o); }
    DevBuf& operator=(DevBuf&& o) noexcept;
    template <class T> T* as() const { return static_cast<T*>(p); }
};

// Plain device allocation owned by an index (freed with hipFree).
void* dev_alloc(size_t bytes);
// Throws ISAX_ENOMEM when the allocation countdown of isax_debug_fail_allocation runs out.
void injected_failure(size_t bytes);

}  // namespace isax
struct isax_index;
namespace isax {
// Device scratch one query batch of mq queries (row stride kmax) allocates in `mode`.
int64_t query_scratch_bytes(const isax_index* idx, int mq, int kmax, int mode);

// Serving table of the step-level request loop (runtime.hip): `slots` query
// rows resident on the device, the collection swept in `chunks` steps.  Rows
// are chosen by the caller; every call throws isax::Error on failure.
struct StepTable;
StepTable* step_table_create(isax_index* idx, int mode, int slots, int chunks, hipStream_t s);
void step_table_destroy(StepTable* t);
int step_table_chunks(const StepTable* t);  // steps per sweep (at most the requested chunks)
// Queues one step (at most two queued): queries q [n_adm][len] (host) with k
// into the free rows adm[], chunk `chunk` for the occupied rows among [0, hi),
// then the final ordering of the rows fin[] (which become free).
void step_table_launch(StepTable* t, const float* q, const int32_t* k, const int* adm, int n_adm, int chunk, int hi,
                       const int* fin, int n_fin);
// Waits for the oldest queued step: ovf (host, its hi) <- rows that lost filter
// candidates; ids / dists (host, [n_fin][kout]) and status (0, else the row
// must be answered alone) of its final ordering.
void step_table_collect(StepTable* t, int* ovf, int kout, int64_t* ids, float* dists, int* status);
// After a failure: drains the stream, forgets queued steps, frees every row.
void step_table_reset(StepTable* t);

}  // namespace isax

// ---------------------------------------------------------------------------------------------
// The index.  All device arrays are owned except `data`, which the caller lends.
struct isax_index {
    int device = 0;
    hipStream_t stream = nullptr;
    const float* data = nullptr;  // [n][len], borrowed
    bool data_on_host = false;    // data is pinned host memory (rows cross the bus)
    int64_t n = 0;
    int32_t len = 0, w = 0, c = 0, m_seg = 0, ws = 0, ns = 0;  // ws: word stride bytes, ns = 2^c
    int32_t leaf_size = 256, key_bits = 64;
    int64_t n_leaves = 0;
    float max_abs = 0.f;
    float delta = 0.f;
    float* beta = nullptr;          // [ns-1] region edges
    std::vector<float> beta_host;   // the same on the host
    int edges = ISAX_EDGES_NORMAL;  // how the edges were chosen
    uint8_t* words_sorted = nullptr;// [n][ws]
    int32_t* ids_sorted = nullptr;  // [n]
    uint8_t* env_lo = nullptr;      // [n_leaves][ws]
    uint8_t* env_hi = nullptr;      // [n_leaves][ws]
    uint64_t* leaf_key = nullptr;   // [n_leaves] first key of each leaf
    uint8_t* node_lo = nullptr;     // [n_nodes][ws] envelope of leaves [i * kNodeLeaves, (i + 1) * kNodeLeaves)
    uint8_t* node_hi = nullptr;     // [n_nodes][ws]
    int64_t n_nodes = 0;
    // reduced-precision copies for the dot-product filter
    float* xs = nullptr;            // [n][len] FP32 rows in leaf order (optional copy)
    uint16_t* x_bf16 = nullptr;     // [n][len] BF16 bits
    float4* meta_bf16 = nullptr;    // [n] {|x|^2, |e_x| (up), |x~| (up), 1}
    uint8_t* x_fp8 = nullptr;       // [n][len] E4M3 codes
    float4* meta_fp8 = nullptr;     // [n] {|x|^2, |e_x| (up), |x~| (up), scale}
    // spectral copy: BF16 of ext(x) = (D - 1 leading DCT-II coefficients, norm of the rest)
    int spec_dim = 0;               // D (0: none)
    uint16_t* x_spec = nullptr;     // [n][D] BF16 bits, leaf order
    float4* meta_spec = nullptr;    // [n] {|x|^2, |ext(x) - x~| (up), |x~| (up), 1}
    double* spec_t = nullptr;       // [len][D] the transform, column D - 1 zero (FP64)
    int64_t device_bytes = 0;
    std::vector<void*> owned;
    ~isax_index();
};
