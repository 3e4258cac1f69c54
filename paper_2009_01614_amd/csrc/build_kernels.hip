// Index build kernels for gfx950: PAA + iSAX summarisation, interleaved keys,
// LSD radix sort of (key, id), word gather, leaf envelopes, and the BF16 /
// FP8 copies used by the dot-product filter.
//
// Paper: Sec. II (iSAX Representation: PAA segment means, bit-string symbols
// per region; ADS+ Index: root subtrees by the first bit of every segment,
// leaves refine one segment by one bit) and Sec. III (ParIS Stage 2 and MESSI
// Stage 1 summarise every series; MESSI Stage 2 builds the root subtrees).
// Here the tree is replaced by a flat layout: words sorted by their
// bit-interleaved key and cut into fixed-size leaves, each with a per-segment
// symbol envelope.
#include "build_kernels.h"

namespace isax {
namespace {

constexpr int kTile = 4096;            // radix-sort tile
constexpr int kSortThreads = 256;      // histogram blocks: 16 items per thread
constexpr int kScatterThreads = 256;   // scatter blocks: 4 waves of 1024 items
constexpr int kItemsPerWave = kTile / (kScatterThreads / kWaveSize);

__device__ inline unsigned float_ord(float v) { return __float_as_uint(v); }  // v >= 0

// Symbol = #{ j : beta_j <= p } by binary lifting over the 2^c - 1 sorted edges.
__device__ inline int symbol_of(float p, const float* beta, int c) {
    int s = 0;
    for (int step = 1 << (c - 1); step > 0; step >>= 1)
        if (beta[s + step - 1] <= p) s += step;
    return s;
}

// ---------------------------------------------------------------------------------------------
// Summarise, fast path.  The collection is read as a flat stream of float4;
// one wave consumes 64 float4 (1 KB) per "page" with one coalesced load.  A
// segment of M points (M in 4..64, a power of two) spans M/4 consecutive lanes;
// each lane adds its four values as (x0 + x1) + (x2 + x3) and the segment sum is
// completed by a butterfly over those lanes, i.e. a balanced tree of adjacent
// pairs.  The mean is sum * (1/M) (exact for a power of two).
template <int M>
__global__ void __launch_bounds__(256) k_summarise_fast(const float4* __restrict__ data, int64_t n_f4, int w,
                                                        int out_stride, const float* __restrict__ beta_g, int c,
                                                        uint8_t* __restrict__ words, unsigned* __restrict__ maxabs,
                                                        int* __restrict__ nonfinite) {
    constexpr int LPS = M / 4;  // lanes per segment
    __shared__ float beta[256];
    const int nb = (1 << c) - 1;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) beta[i] = beta_g[i];
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int64_t n_waves = (int64_t)gridDim.x * (blockDim.x / 64);
    const int64_t pages = (n_f4 + 63) / 64;
    float amax = 0.f;
    bool bad = false;
    constexpr int U = 4;
    for (int64_t p0 = wave * U; p0 < pages; p0 += n_waves * U) {
        float4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t g = (p0 + u) * 64 + lane;
            v[u] = (p0 + u < pages && g < n_f4) ? data[g] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t g = (p0 + u) * 64 + lane;
            const float4 x = v[u];
            amax = fmaxf(amax, fmaxf(fmaxf(fabsf(x.x), fabsf(x.y)), fmaxf(fabsf(x.z), fabsf(x.w))));
            bad |= !(fabsf(x.x) <= 3.4028235e38f) | !(fabsf(x.y) <= 3.4028235e38f) |
                   !(fabsf(x.z) <= 3.4028235e38f) | !(fabsf(x.w) <= 3.4028235e38f);
            float s = (x.x + x.y) + (x.z + x.w);
#pragma unroll
            for (int o = 1; o < LPS; o <<= 1) s += __shfl_xor(s, o, 64);
            if (p0 + u < pages && g < n_f4 && (lane % LPS) == 0) {
                const float paa = s * (1.0f / M);
                const int64_t seg = g / LPS;
                const int64_t i = seg / w;
                const int j = (int)(seg - i * w);
                words[i * out_stride + j] = (uint8_t)symbol_of(paa, beta, c);
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
    unsigned long long anybad = __ballot(bad);
    if (lane == 0) {
        atomicMax(maxabs, float_ord(amax));
        if (anybad) atomicOr(nonfinite, 1);
    }
}

// Summarise, generic path (any segment length): one thread per segment.  The
// segment is zero-padded to the next power of two and summed as a balanced
// tree of adjacent pairs (binary-counter order), the same tree as above.
__global__ void k_summarise_generic(const float* __restrict__ data, int64_t n, int len, int w, int m,
                                    int out_stride, const float* __restrict__ beta_g, int c,
                                    uint8_t* __restrict__ words, unsigned* __restrict__ maxabs,
                                    int* __restrict__ nonfinite) {
    __shared__ float beta[256];
    const int nb = (1 << c) - 1;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) beta[i] = beta_g[i];
    __syncthreads();
    int P = 1;
    while (P < m) P <<= 1;
    float amax = 0.f;
    bool bad = false;
    const int64_t nseg = n * w;
    for (int64_t seg = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; seg < nseg;
         seg += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = seg / w;
        const int j = (int)(seg - i * w);
        const float* x = data + i * len + (int64_t)j * m;
        float stack[14];
        int level[14];
        int top = 0;
        for (int t = 0; t < P; ++t) {
            float v = 0.f;
            if (t < m) {
                v = x[t];
                amax = fmaxf(amax, fabsf(v));
                bad |= !(fabsf(v) <= 3.4028235e38f);
            }
            stack[top] = v;
            level[top] = 0;
            ++top;
            while (top >= 2 && level[top - 1] == level[top - 2]) {
                stack[top - 2] = stack[top - 2] + stack[top - 1];
                level[top - 2] += 1;
                --top;
            }
        }
        const float paa = stack[0] / (float)m;
        words[i * out_stride + j] = (uint8_t)symbol_of(paa, beta, c);
    }
    for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
    unsigned long long anybad = __ballot(bad);
    if ((threadIdx.x & 63) == 0) {
        atomicMax(maxabs, float_ord(amax));
        if (anybad) atomicOr(nonfinite, 1);
    }
}

// ---------------------------------------------------------------------------------------------
// FP32 PAA of every segment of n_series evenly spaced series (series
// floor(t n / n_series), t = 0..n_series-1) into out[t][w], in the summation
// order of the summarise kernels (zero-padded to a power of two, a balanced
// tree of adjacent pairs, then / m): the sample the empirical region edges
// are taken from.
__global__ void k_paa_sample(const float* __restrict__ data, int64_t n, int len, int w, int m, int n_series,
                             float* __restrict__ out) {
    int P = 1;
    while (P < m) P <<= 1;
    const int64_t items = (int64_t)n_series * w;
    for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < items;
         it += (int64_t)gridDim.x * blockDim.x) {
        const int t = (int)(it / w), j = (int)(it - (int64_t)t * w);
        const int64_t i = (int64_t)t * n / n_series;
        const float* x = data + i * len + (int64_t)j * m;
        float stack[14];
        int level[14];
        int top = 0;
        for (int q = 0; q < P; ++q) {
            stack[top] = q < m ? x[q] : 0.f;
            level[top] = 0;
            ++top;
            while (top >= 2 && level[top - 1] == level[top - 2]) {
                stack[top - 2] = stack[top - 2] + stack[top - 1];
                level[top - 2] += 1;
                --top;
            }
        }
        out[it] = stack[0] / (float)m;
    }
}

// ---------------------------------------------------------------------------------------------
// Interleaved key: bit (63 - (r*w + j)) holds bit (c-1-r) of segment j; only
// the first key_bits positions are kept.  The first w bits are the root subtree.
// 16 segments: the bit of round r of the four bytes of a word is gathered with
// one multiply ((t & 0x01010101) * 0x01020408 puts byte i's bit at bit 24+i),
// the 16 bits are assembled with segment j at bit j and then bit-reversed.
__device__ inline unsigned gather4(unsigned u, int b) {
    return (((u >> b) & 0x01010101u) * 0x01020408u) >> 24 & 15u;
}

__global__ void k_make_keys16(const uint8_t* __restrict__ words, int64_t n, int c, int key_bits,
                              uint64_t* __restrict__ keys, int32_t* __restrict__ ids) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint4 v = reinterpret_cast<const uint4*>(words + i * 16)[0];
        uint64_t key = 0;
        for (int r = 0; r < c && 16 * r < key_bits; ++r) {
            const int b = c - 1 - r;
            const unsigned g = gather4(v.x, b) | gather4(v.y, b) << 4 | gather4(v.z, b) << 8 | gather4(v.w, b) << 12;
            key |= (uint64_t)(__builtin_bitreverse32(g) >> 16) << (48 - 16 * r);
        }
        if (key_bits < 64) key &= ~0ull << (64 - key_bits);
        keys[i] = key;
        ids[i] = (int32_t)i;
    }
}

__global__ void k_make_keys(const uint8_t* __restrict__ words, int64_t n, int ws, int w, int c, int key_bits,
                            uint64_t* __restrict__ keys, int32_t* __restrict__ ids) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint8_t* s = words + i * ws;
        uint64_t key = 0;
        int pos = 0;
        for (int r = 0; r < c && pos < key_bits; ++r)
            for (int j = 0; j < w && pos < key_bits; ++j, ++pos)
                key |= (uint64_t)((s[j] >> (c - 1 - r)) & 1) << (63 - pos);
        keys[i] = key;
        ids[i] = (int32_t)i;
    }
}

// ---------------------------------------------------------------------------------------------
// LSD radix sort, 8-bit digits.  Pass: per-tile histograms (digit-major),
// exclusive scan, stable scatter.  Within a tile, each wave owns a contiguous
// run of 1024 items processed 64 at a time; lanes holding the same digit are
// found with eight ballots, ranked by popcount, and a per-wave LDS counter per
// digit carries the running count, so the scatter is stable.  The scatter
// first reorders the tile by digit in LDS and then writes it out in that
// order, so each digit's run of the tile (16 items on average) leaves as
// consecutive addresses from consecutive lanes.
__global__ void __launch_bounds__(kSortThreads) k_radix_hist(const uint64_t* __restrict__ keys, int64_t n, int shift,
                                                             int n_tiles, uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int t = threadIdx.x; t < kTile; t += kSortThreads) {
        const int64_t i = base + t;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * n_tiles + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of `len` uint32 in place: per-chunk scan, chunk totals in `sums`.
constexpr int kScanChunk = 4096;
__global__ void __launch_bounds__(256) k_scan_chunks(uint32_t* __restrict__ a, int64_t len, uint32_t* __restrict__ sums) {
    __shared__ uint32_t part[256];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + threadIdx.x * 16;
    uint32_t v[16];
    uint32_t tot = 0;
    for (int i = 0; i < 16; ++i) {
        v[i] = (base + i < len) ? a[base + i] : 0u;
        tot += v[i];
    }
    part[threadIdx.x] = tot;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        uint32_t add = threadIdx.x >= o ? part[threadIdx.x - o] : 0u;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - tot;
    for (int i = 0; i < 16; ++i) {
        if (base + i < len) a[base + i] = run;
        run += v[i];
    }
    if (threadIdx.x == 255) sums[blockIdx.x] = part[255];
}

__global__ void __launch_bounds__(1024) k_scan_sums(uint32_t* __restrict__ sums, int nchunks) {
    __shared__ uint32_t part[1024];
    const int per = (nchunks + 1023) / 1024;
    const int base = threadIdx.x * per;
    uint32_t tot = 0;
    for (int i = 0; i < per; ++i)
        if (base + i < nchunks) tot += sums[base + i];
    part[threadIdx.x] = tot;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        uint32_t add = threadIdx.x >= o ? part[threadIdx.x - o] : 0u;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - tot;
    for (int i = 0; i < per; ++i)
        if (base + i < nchunks) {
            uint32_t v = sums[base + i];
            sums[base + i] = run;
            run += v;
        }
}

__global__ void k_scan_add(uint32_t* __restrict__ a, int64_t len, const uint32_t* __restrict__ sums) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) a[i] += sums[i / kScanChunk];
}

__global__ void __launch_bounds__(kScatterThreads) k_radix_scatter(const uint64_t* __restrict__ kin,
                                                                const int32_t* __restrict__ vin, int64_t n, int shift,
                                                                int n_tiles, const uint32_t* __restrict__ offs,
                                                                uint64_t* __restrict__ kout, int32_t* __restrict__ vout) {
    constexpr int R = kItemsPerWave / 64;  // rounds of 64 items per wave
    constexpr int NW = kScatterThreads / 64;
    static_assert(kScatterThreads >= 256, "one thread per digit");
    __shared__ uint32_t cnt[NW][256];
    __shared__ uint32_t delta[256];  // global start of the digit's run minus its start in the tile
    __shared__ uint32_t wsum[4];
    // the tile's keys in digit order, then its values in the same buffer (37 KB of
    // LDS per block in all: four blocks per CU)
    __shared__ uint64_t stage[kTile];
    int32_t* sval = reinterpret_cast<int32_t*>(stage);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = threadIdx.x; i < NW * 256; i += kScatterThreads) cnt[i >> 8][i & 255] = 0;
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint64_t key[R];
    int32_t val[R];
    uint32_t rd[R];  // rank within the wave's items of the digit (low 16 bits), digit + 1 (high; 0 = none)
    const int64_t start = (int64_t)blockIdx.x * kTile + (int64_t)wave * kItemsPerWave;
    // all loads first: the wave barriers of the ranking below also stop the
    // compiler from moving loads, which would leave one memory latency per round
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = start + r * 64 + lane;
        key[r] = i < n ? kin[i] : 0ull;
        val[r] = i < n ? vin[i] : 0;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const bool valid = start + r * 64 + lane < n;
        const int d = (int)((key[r] >> shift) & 255);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t bm = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? bm : ~bm;
        }
        uint32_t prior = 0;
        if (valid) prior = cnt[wave][d];
        rd[r] = valid ? ((uint32_t)(d + 1) << 16) | (prior + (uint32_t)__popcll(peers & lt)) : 0u;
        const int leader = valid ? (int)(__ffsll((long long)peers) - 1) : -1;
        __builtin_amdgcn_wave_barrier();
        if (valid && leader == lane) cnt[wave][d] = prior + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // digit d = threadIdx.x < 256: prefix over the waves, then the digit's start in
    // the tile (exclusive scan of the tile's digit totals: within the wave by
    // shuffles, then over the first four waves)
    const int dd = threadIdx.x;
    uint32_t tot = 0, incl = 0;
    if (dd < 256) {
        for (int wv = 0; wv < NW; ++wv) {
            const uint32_t c0 = cnt[wv][dd];
            cnt[wv][dd] = tot;
            tot += c0;
        }
        incl = tot;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = __shfl_up(incl, o);
            if (lane >= o) incl += t;
        }
        if (lane == 63) wsum[wave] = incl;
    }
    __syncthreads();
    if (dd < 256) {
        uint32_t tstart = incl - tot;
        for (int wv = 0; wv < wave; ++wv) tstart += wsum[wv];
        // unsigned wrap-around: delta + (tile position) is the global position (< 2^31)
        delta[dd] = offs[(int64_t)dd * n_tiles + blockIdx.x] - tstart;
        for (int wv = 0; wv < NW; ++wv) cnt[wv][dd] += tstart;
    }
    __syncthreads();
    // the tile in digit order in LDS (stable: waves in order, ranks within a wave) ...
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (rd[r]) {
            rd[r] = cnt[wave][(rd[r] >> 16) - 1] + (rd[r] & 0xFFFFu);  // now the position in the tile
            stage[rd[r]] = key[r];
        } else {
            rd[r] = ~0u;
        }
    }
    __syncthreads();
    // ... then written out in that order: consecutive lanes write consecutive
    // positions of one digit's run.  Keys first; the global positions are kept for
    // the values, which then take the buffer.
    constexpr int PT = kTile / kScatterThreads;
    const int64_t left = n - (int64_t)blockIdx.x * kTile;
    const int cnt_tile = left < kTile ? (int)left : kTile;
    uint32_t dst[PT];
#pragma unroll
    for (int j = 0; j < PT; ++j) {
        const int i = threadIdx.x + j * kScatterThreads;
        dst[j] = ~0u;
        if (i < cnt_tile) {
            const uint64_t k = stage[i];
            dst[j] = delta[(int)((k >> shift) & 255)] + (uint32_t)i;
            kout[dst[j]] = k;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (rd[r] != ~0u) sval[rd[r]] = val[r];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PT; ++j)
        if (dst[j] != ~0u) vout[dst[j]] = sval[threadIdx.x + j * kScatterThreads];
}

// ---------------------------------------------------------------------------------------------
__global__ void k_gather_words(const uint8_t* __restrict__ words, const int32_t* __restrict__ ids, int64_t n, int ws,
                               uint8_t* __restrict__ out) {
    const int q16 = ws / 16;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n * q16; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = t / q16;
        const int q = (int)(t - p * q16);
        reinterpret_cast<uint4*>(out + p * ws)[q] = reinterpret_cast<const uint4*>(words + (int64_t)ids[p] * ws)[q];
    }
}

// Rows of the collection in leaf order: out[p] = data[ids[p]], 16 bytes per
// thread when rows are 16-byte aligned.
template <bool VEC>
__global__ void k_gather_rows(const float* __restrict__ data, const int32_t* __restrict__ ids, int64_t n, int len,
                              float* __restrict__ out) {
    const int per = VEC ? len / 4 : len;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n * per; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = t / per;
        const int e = (int)(t - p * per);
        if (VEC)
            reinterpret_cast<float4*>(out + p * len)[e] = reinterpret_cast<const float4*>(data + (int64_t)ids[p] * len)[e];
        else
            out[p * len + e] = data[(int64_t)ids[p] * len + e];
    }
}

__global__ void k_leaf_keys(const uint64_t* __restrict__ keys_sorted, int64_t n_leaves, int leaf,
                            uint64_t* __restrict__ leaf_key) {
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l < n_leaves) leaf_key[l] = keys_sorted[l * leaf];
}

// Envelopes of nodes of kNodeLeaves consecutive leaves: per word byte the
// minimum of the leaves' lower and the maximum of their upper symbols, one
// thread per (node, byte).
__global__ void k_node_envelopes(const uint8_t* __restrict__ lo, const uint8_t* __restrict__ hi, int64_t n_leaves,
                                 int ws, int64_t n_nodes, uint8_t* __restrict__ node_lo,
                                 uint8_t* __restrict__ node_hi) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_nodes * ws;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t node = t / ws;
        const int j = (int)(t - node * ws);
        const int64_t l0 = node * kNodeLeaves, l1 = min(n_leaves, l0 + kNodeLeaves);
        int mn = 255, mx = 0;
        for (int64_t l = l0; l < l1; ++l) {
            mn = min(mn, (int)lo[l * ws + j]);
            mx = max(mx, (int)hi[l * ws + j]);
        }
        node_lo[t] = (uint8_t)mn;
        node_hi[t] = (uint8_t)mx;
    }
}

// One wave per leaf: per-segment min and max symbol of the leaf's words.
__global__ void __launch_bounds__(256) k_envelopes(const uint8_t* __restrict__ ws_words, int64_t n, int ws, int leaf,
                                                   int64_t n_leaves, uint8_t* __restrict__ lo,
                                                   uint8_t* __restrict__ hi) {
    const int lane = threadIdx.x & 63;
    for (int64_t l = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); l < n_leaves;
         l += (int64_t)gridDim.x * (blockDim.x / 64)) {
    const int64_t a = l * leaf;
    const int64_t b = min(n, a + leaf);
    for (int q = 0; q < ws / 16; ++q) {
        int mn[16], mx[16];
        for (int j = 0; j < 16; ++j) {
            mn[j] = 255;
            mx[j] = 0;
        }
        for (int64_t p = a + lane; p < b; p += 64) {
            const uint4 v = reinterpret_cast<const uint4*>(ws_words + p * ws)[q];
            const unsigned u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int s = (u[j >> 2] >> (8 * (j & 3))) & 255;
                mn[j] = min(mn[j], s);
                mx[j] = max(mx[j], s);
            }
        }
#pragma unroll
        for (int j = 0; j < 16; ++j)
            for (int o = 32; o > 0; o >>= 1) {
                mn[j] = min(mn[j], __shfl_xor(mn[j], o, 64));
                mx[j] = max(mx[j], __shfl_xor(mx[j], o, 64));
            }
        if (lane < 16) {
            int vmn = 0, vmx = 0;
#pragma unroll
            for (int j = 0; j < 16; ++j)
                if (j == lane) {
                    vmn = mn[j];
                    vmx = mx[j];
                }
            lo[l * ws + q * 16 + lane] = (uint8_t)vmn;
            hi[l * ws + q * 16 + lane] = (uint8_t)vmx;
        }
    }
    }
}

// ---------------------------------------------------------------------------------------------
// Reduced-precision copies.  BF16: round to nearest even.  FP8 E4M3 (OCP, max
// 448): the row is divided by the smallest power of two s with max|x|/s <= 448
// and rounded to nearest even; x~ = s * code value is exact in FP32, and so is
// e_x = x - x~.  Per row: |x|^2 (FP32), |e_x| and |x~| rounded up.
__device__ inline uint16_t bf16_rne(float x) {
    unsigned u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf16_val(uint16_t b) { return __uint_as_float((unsigned)b << 16); }

// E4M3 code of y, |y| <= 448, round to nearest even (exp bias 7, 3 mantissa bits,
// subnormal quantum 2^-9).
__device__ inline uint8_t e4m3_rne(float y) {
    const unsigned sign = (__float_as_uint(y) >> 24) & 0x80u;
    const float a = fabsf(y);
    if (a == 0.f) return (uint8_t)sign;
    int e = ((int)((__float_as_uint(a) >> 23) & 255)) - 127;  // floor(log2 a) for normal FP32
    if (e < -6) {
        const float q = rintf(a * 512.f);  // subnormal grid 2^-9; q == 8 is the smallest normal
        return (uint8_t)(sign | (unsigned)q);
    }
    float q = rintf(ldexpf(a, 3 - e));  // in [8, 16]
    if (q >= 16.f) {
        q = 8.f;
        ++e;
    }
    return (uint8_t)(sign | (unsigned)((e + 7) << 3) | ((unsigned)q - 8u));
}
__device__ inline float e4m3_val(uint8_t b) {
    const int ex = (b >> 3) & 15, mn = b & 7;
    const float v = ex == 0 ? ldexpf((float)mn, -9) : ldexpf((float)(8 + mn), ex - 10);
    return (b & 0x80) ? -v : v;
}

// Round-up for norms: multiply by (1 + 2^-10), which exceeds the relative
// rounding error of an FP32 sum of up to 4096 squares (4096 * 2^-24) plus the sqrt.
__device__ inline float up_norm(float sumsq) { return sqrtf(sumsq * (1.0f + 0.0009765625f)) * (1.0f + 0.0009765625f); }

// Rows are written in leaf order: row p of the copy is series ids_sorted[p].
// One wave per row and pass; float4 loads when the row allows them, packed
// stores (4 BF16 = 8 B or 4 E4M3 = 4 B per lane and step).
template <bool VEC>
__global__ void __launch_bounds__(256) k_quantise(const float* __restrict__ data, const int32_t* __restrict__ ids,
                                                  int64_t n, int len, int len_pad, int kind, uint16_t* __restrict__ xb,
                                                  uint8_t* __restrict__ xf, float4* __restrict__ meta) {
    const int lane = threadIdx.x & 63;
    for (int64_t i = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); i < n;
         i += (int64_t)gridDim.x * (blockDim.x / 64)) {
        const float* x = data + (int64_t)ids[i] * len;
        // rows up to 512 points: every lane holds its (up to) two float4 chunks in registers
        float v[8];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int t = (lane + 64 * c) * 4;
            if (VEC) {
                const float4 q = t < len ? *reinterpret_cast<const float4*>(x + t) : make_float4(0.f, 0.f, 0.f, 0.f);
                v[4 * c] = q.x; v[4 * c + 1] = q.y; v[4 * c + 2] = q.z; v[4 * c + 3] = q.w;
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) v[4 * c + e] = t + e < len ? x[t + e] : 0.f;
            }
        }
        float amax = 0.f;
#pragma unroll
        for (int e = 0; e < 8; ++e) amax = fmaxf(amax, fabsf(v[e]));
        for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
        float scale = 1.f;
        if (kind == 1 && amax > 0.f) {
            int e;
            const float f = frexpf(amax / 448.f, &e);
            scale = ldexpf(1.f, f == 0.5f ? e - 1 : e);
            if (amax / scale > 448.f) scale *= 2.f;
            if (amax / (scale * 0.5f) <= 448.f) scale *= 0.5f;
        }
        float xn = 0.f, en = 0.f, tn = 0.f;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int t = (lane + 64 * c) * 4;
            if (t >= len_pad) continue;
            float vt[4];
            if (kind == 0) {
                uint16_t b[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    b[e] = bf16_rne(v[4 * c + e]);
                    vt[e] = bf16_val(b[e]);
                }
                *reinterpret_cast<uint2*>(xb + i * len_pad + t) =
                    make_uint2((unsigned)b[0] | (unsigned)b[1] << 16, (unsigned)b[2] | (unsigned)b[3] << 16);
            } else {
                unsigned word = 0;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const uint8_t b = e4m3_rne(v[4 * c + e] / scale);
                    word |= (unsigned)b << (8 * e);
                    vt[e] = e4m3_val(b) * scale;
                }
                *reinterpret_cast<unsigned*>(xf + i * len_pad + t) = word;
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float ve = v[4 * c + e];
                const float er = ve - vt[e];
                xn = fmaf(ve, ve, xn);
                en = fmaf(er, er, en);
                tn = fmaf(vt[e], vt[e], tn);
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            xn += __shfl_xor(xn, o, 64);
            en += __shfl_xor(en, o, 64);
            tn += __shfl_xor(tn, o, 64);
        }
        if (lane == 0) meta[i] = make_float4(xn, up_norm(en), up_norm(tn), scale);
    }
}

// ---------------------------------------------------------------------------------------------
// Spectral copy: for the series at sorted position p, y = T x in FP64 (T the
// orthonormal DCT-II, given transposed as tt [len][D] with a zero column D - 1),
// ext(x) = (y_0 .. y_{D-2}, t) with t = sqrt(|x|^2 - |y_head|^2) the norm of the
// dropped coefficients, and its BF16 codes.  A block takes tiles of 64 series,
// staged through LDS kSpecChunk points at a time (rows of kSpecChunk + 1
// floats: lanes read distinct banks) together with the same kSpecChunk rows of
// T; wave g computes coefficients [g DQ, (g + 1) DQ) of every series of the
// tile, one series per lane, reading T from LDS (the same address in every
// lane: one broadcast read per two coefficients).  Each coefficient sums its
// products in point order, as a plain loop over the points would.
// meta[p] = {|x|^2, |ext(x) - x~| (up), |x~| (up), 1}: the FP64 transform (T
// within 2^-50 relative, sums of at most 512 terms) puts the head within
// 1e-12 |x| of the exact one and the tail norm, from a difference of squares,
// within 1.5e-6 |x|; 2^-18 |x| is added to |ext(x) - x~| for both.
constexpr int kSpecChunk = 32;
template <int DQ>
__global__ void __launch_bounds__(256) k_spectral(const float* __restrict__ data, const int32_t* __restrict__ ids,
                                                  int64_t n, int len, const double* __restrict__ tt,
                                                  uint16_t* __restrict__ xs, float4* __restrict__ meta) {
    constexpr int D = 4 * DQ, JC = kSpecChunk;
    __shared__ float sx[64][JC + 1];
    __shared__ __attribute__((aligned(16))) double sT[JC * D];  // rows j0 .. j0 + JC - 1 of T
    __shared__ double s_head[4][64], s_err[4][64], s_code[4][64];
    const int lane = threadIdx.x & 63;
    const int g = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t n_tiles = (n + 63) / 64;
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t p0 = tile * 64;
        double acc[DQ];
#pragma unroll
        for (int r = 0; r < DQ; ++r) acc[r] = 0.0;
        double xn = 0.0;
        for (int j0 = 0; j0 < len; j0 += JC) {
            const int jn = min(JC, len - j0);
            __syncthreads();  // the previous chunk's points and rows of T are no longer read
            for (int e = threadIdx.x; e < 64 * JC; e += 256) {
                const int r = e / JC, j = e % JC;
                const int64_t p = p0 + r;
                sx[r][j] = p < n && j < jn ? data[(int64_t)ids[p] * len + j0 + j] : 0.f;
            }
            {
                const double2* src = reinterpret_cast<const double2*>(tt + (int64_t)j0 * D);
                double2* dst = reinterpret_cast<double2*>(sT);
                for (int e = threadIdx.x; e < jn * D / 2; e += 256) dst[e] = src[e];
            }
            __syncthreads();
            for (int j = 0; j < jn; ++j) {
                const double v = (double)sx[lane][j];
                xn = fma(v, v, xn);
                const double2* tj = reinterpret_cast<const double2*>(sT + j * D + g * DQ);
#pragma unroll
                for (int r = 0; r < DQ / 2; ++r) {
                    const double2 t2 = tj[r];
                    acc[2 * r] = fma(t2.x, v, acc[2 * r]);
                    acc[2 * r + 1] = fma(t2.y, v, acc[2 * r + 1]);
                }
            }
        }
        double hs = 0.0;
#pragma unroll
        for (int r = 0; r < DQ; ++r) hs = fma(acc[r], acc[r], hs);
        s_head[g][lane] = hs;
        __syncthreads();
        const double tail = sqrt(fmax(0.0, xn - (((s_head[0][lane] + s_head[1][lane]) + s_head[2][lane]) + s_head[3][lane])));
        if (g == 3) acc[DQ - 1] = tail;
        const int64_t p = p0 + lane;
        double e2 = 0.0, c2 = 0.0;
        unsigned packed[DQ / 2];
#pragma unroll
        for (int r = 0; r < DQ; ++r) {
            const uint16_t b = bf16_rne((float)acc[r]);
            const double bv = (double)bf16_val(b);
            e2 = fma(acc[r] - bv, acc[r] - bv, e2);
            c2 = fma(bv, bv, c2);
            if (r & 1) packed[r / 2] |= (unsigned)b << 16;
            else packed[r / 2] = b;
        }
        if (p < n) {
            uint4* dst = reinterpret_cast<uint4*>(xs + p * D + g * DQ);
#pragma unroll
            for (int c = 0; c < DQ / 8; ++c)
                dst[c] = make_uint4(packed[4 * c], packed[4 * c + 1], packed[4 * c + 2], packed[4 * c + 3]);
        }
        s_err[g][lane] = e2;
        s_code[g][lane] = c2;
        __syncthreads();
        if (g == 0 && p < n) {
            const double E = ((s_err[0][lane] + s_err[1][lane]) + s_err[2][lane]) + s_err[3][lane];
            const double C = ((s_code[0][lane] + s_code[1][lane]) + s_code[2][lane]) + s_code[3][lane];
            const double nx = sqrt(xn);
            meta[p] = make_float4((float)xn, up_norm((float)(E * (1.0 + 0x1p-40))) + (float)(0x1p-18 * nx) * 1.001f,
                                  up_norm((float)(C * (1.0 + 0x1p-40))), 1.f);
        }
    }
}

}  // namespace

// =============================================================================================
// Host launchers
void launch_summarise(const float* data, int64_t n, int len, int w, int out_stride, const float* beta, int c,
                      uint8_t* words, unsigned* maxabs, int* nonfinite, hipStream_t s) {
    const int m = len / w;
    const bool fast = (len % 4 == 0) && (reinterpret_cast<uintptr_t>(data) & 15) == 0 &&
                      (m == 4 || m == 8 || m == 16 || m == 32 || m == 64);
    ProfScope ps("summarise", s);
    if (fast) {
        const int64_t n_f4 = n * (int64_t)len / 4;
        const int64_t pages = (n_f4 + 63) / 64;
        int64_t blocks = (pages + 15) / 16;  // 4 waves x 4 pages per block iteration
        blocks = std::max<int64_t>(1, std::min<int64_t>(blocks, 256 * 16));
        const float4* d4 = reinterpret_cast<const float4*>(data);
        switch (m) {
            case 4: k_summarise_fast<4><<<blocks, 256, 0, s>>>(d4, n_f4, w, out_stride, beta, c, words, maxabs, nonfinite); break;
            case 8: k_summarise_fast<8><<<blocks, 256, 0, s>>>(d4, n_f4, w, out_stride, beta, c, words, maxabs, nonfinite); break;
            case 16: k_summarise_fast<16><<<blocks, 256, 0, s>>>(d4, n_f4, w, out_stride, beta, c, words, maxabs, nonfinite); break;
            case 32: k_summarise_fast<32><<<blocks, 256, 0, s>>>(d4, n_f4, w, out_stride, beta, c, words, maxabs, nonfinite); break;
            default: k_summarise_fast<64><<<blocks, 256, 0, s>>>(d4, n_f4, w, out_stride, beta, c, words, maxabs, nonfinite); break;
        }
    } else {
        const int64_t nseg = n * w;
        int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((nseg + 255) / 256, 256 * 32));
        k_summarise_generic<<<blocks, 256, 0, s>>>(data, n, len, w, m, out_stride, beta, c, words, maxabs, nonfinite);
    }
    ISAX_HIP(hipGetLastError());
}

void sort_keys(uint64_t* keys, int32_t* ids, int64_t n, int key_bits, hipStream_t s) {
    const int n_tiles = (int)((n + kTile - 1) / kTile);
    const int64_t hlen = (int64_t)256 * n_tiles;
    const int nchunks = (int)((hlen + kScanChunk - 1) / kScanChunk);
    DevBuf k2(n * sizeof(uint64_t), s), v2(n * sizeof(int32_t), s);
    DevBuf hist(hlen * sizeof(uint32_t), s), sums((size_t)nchunks * sizeof(uint32_t), s);
    uint64_t *ka = keys, *kb = k2.as<uint64_t>();
    int32_t *va = ids, *vb = v2.as<int32_t>();
    int passes = 0;
    for (int shift = 64 - key_bits; shift < 64; shift += 8, ++passes) {
        {
            ProfScope ps("radix_hist", s);
            k_radix_hist<<<n_tiles, kSortThreads, 0, s>>>(ka, n, shift, n_tiles, hist.as<uint32_t>());
        }
        {
            ProfScope ps("radix_scan", s);
            k_scan_chunks<<<nchunks, 256, 0, s>>>(hist.as<uint32_t>(), hlen, sums.as<uint32_t>());
            k_scan_sums<<<1, 1024, 0, s>>>(sums.as<uint32_t>(), nchunks);
            k_scan_add<<<(int)((hlen + 255) / 256), 256, 0, s>>>(hist.as<uint32_t>(), hlen, sums.as<uint32_t>());
        }
        {
            ProfScope ps("radix_scatter", s);
            k_radix_scatter<<<n_tiles, kScatterThreads, 0, s>>>(ka, va, n, shift, n_tiles, hist.as<uint32_t>(), kb, vb);
        }
        ISAX_HIP(hipGetLastError());
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != keys) {
        ISAX_HIP(hipMemcpyAsync(keys, ka, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
        ISAX_HIP(hipMemcpyAsync(ids, va, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    }
}

void launch_make_keys(const uint8_t* words, int64_t n, int ws, int w, int c, int key_bits, uint64_t* keys, int32_t* ids,
                      hipStream_t s) {
    ProfScope ps("make_keys", s);
    if (w == 16) k_make_keys16<<<grid_blocks(n, 256), 256, 0, s>>>(words, n, c, key_bits, keys, ids);
    else k_make_keys<<<grid_blocks(n, 256), 256, 0, s>>>(words, n, ws, w, c, key_bits, keys, ids);
    ISAX_HIP(hipGetLastError());
}

void launch_gather_words(const uint8_t* words, const int32_t* ids, int64_t n, int ws, uint8_t* out, hipStream_t s) {
    ProfScope ps("gather_words", s);
    const int64_t t = n * (ws / 16);
    k_gather_words<<<grid_blocks(t, 256), 256, 0, s>>>(words, ids, n, ws, out);
    ISAX_HIP(hipGetLastError());
}

void launch_gather_rows(const float* data, const int32_t* ids, int64_t n, int len, float* out, hipStream_t s) {
    ProfScope ps("gather_rows", s);
    const bool vec = len % 4 == 0 && (reinterpret_cast<uintptr_t>(data) & 15) == 0;
    const int64_t t = n * (vec ? len / 4 : len);
    if (vec) k_gather_rows<true><<<grid_blocks(t, 256), 256, 0, s>>>(data, ids, n, len, out);
    else k_gather_rows<false><<<grid_blocks(t, 256), 256, 0, s>>>(data, ids, n, len, out);
    ISAX_HIP(hipGetLastError());
}

void launch_leaf_layout(const uint64_t* keys_sorted, const uint8_t* words_sorted, int64_t n, int ws, int leaf,
                        int64_t n_leaves, uint64_t* leaf_key, uint8_t* lo, uint8_t* hi, uint8_t* node_lo,
                        uint8_t* node_hi, hipStream_t s) {
    ProfScope ps("envelopes", s);
    k_leaf_keys<<<(int)((n_leaves + 255) / 256), 256, 0, s>>>(keys_sorted, n_leaves, leaf, leaf_key);
    k_envelopes<<<grid_blocks(n_leaves, 4), 256, 0, s>>>(words_sorted, n, ws, leaf, n_leaves, lo, hi);
    const int64_t n_nodes = (n_leaves + kNodeLeaves - 1) / kNodeLeaves;
    k_node_envelopes<<<grid_blocks(n_nodes * ws, 256), 256, 0, s>>>(lo, hi, n_leaves, ws, n_nodes, node_lo, node_hi);
    ISAX_HIP(hipGetLastError());
}

void launch_quantise(const float* data, const int32_t* ids, int64_t n, int len, int len_pad, int kind, uint16_t* xb,
                     uint8_t* xf, float4* meta, hipStream_t s) {
    ProfScope ps("quantise", s);
    if (len_pad > 512) throw Error{ISAX_EINVAL, "the reduced-precision copies support len <= 512"};
    const bool vec = len % 4 == 0 && (reinterpret_cast<uintptr_t>(data) & 15) == 0;
    if (vec) k_quantise<true><<<grid_blocks(n, 4), 256, 0, s>>>(data, ids, n, len, len_pad, kind, xb, xf, meta);
    else k_quantise<false><<<grid_blocks(n, 4), 256, 0, s>>>(data, ids, n, len, len_pad, kind, xb, xf, meta);
    ISAX_HIP(hipGetLastError());
}

void launch_spectral(const float* data, const int32_t* ids, int64_t n, int len, int D, const double* tt, uint16_t* xs,
                     float4* meta, hipStream_t s) {
    ProfScope ps("spectral", s);
    if (len > 512 || D >= len || D < 64 || D > 256 || D % 64)
        throw Error{ISAX_EINVAL, "the spectral copy needs len <= 512 and D in 64..256 (a multiple of 64) below len"};
    const int64_t tiles = (n + 63) / 64;
    const int grid = (int)std::min<int64_t>(tiles, 8192);
    switch (D) {
        case 64: k_spectral<16><<<grid, 256, 0, s>>>(data, ids, n, len, tt, xs, meta); break;
        case 128: k_spectral<32><<<grid, 256, 0, s>>>(data, ids, n, len, tt, xs, meta); break;
        case 192: k_spectral<48><<<grid, 256, 0, s>>>(data, ids, n, len, tt, xs, meta); break;
        default: k_spectral<64><<<grid, 256, 0, s>>>(data, ids, n, len, tt, xs, meta); break;
    }
    ISAX_HIP(hipGetLastError());
}

void launch_paa_sample(const float* data, int64_t n, int len, int w, int n_series, float* out, hipStream_t s) {
    const int64_t items = (int64_t)n_series * w;
    k_paa_sample<<<grid_blocks(items, 256, 4096), 256, 0, s>>>(data, n, len, w, len / w, n_series, out);
    ISAX_HIP(hipGetLastError());
}

}  // namespace isax
