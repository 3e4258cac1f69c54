// Reduced-precision candidate filter on the gfx950 matrix cores.
//
// The paper computes lower bounds with SIMD so that only few real distances
// are needed (Sec. III, ParIS/MESSI).  Here a second, denser filter does the
// same job for large query batches: ED^2 = |q|^2 + |x|^2 - 2 q.x, with q.x
// taken from BF16 (or FP8 E4M3) copies on the MFMA units with FP32
// accumulation.  Its error is bounded rigorously:
//   q.x - q~.x~ = q.e_x + e_q.x~            (q = q~ + e_q, x = x~ + e_x)
//   |acc - q~.x~| <= gamma |q~| |x~|        (FP32 accumulation, any order)
//   M = 2 (|q| |e_x| + (|e_q| + gamma |q~|) |x~|) + kappa (|q|^2 + |x|^2)
// where kappa covers the FP32 rounding of the norms and of the epilogue.  A
// series is a candidate iff approx - M <= tau (1 + eps); candidates are then
// refined with FP32 direct differences like every other path, so the answer
// stays exact.  The query-side factors are replaced by their maxima over the
// batch, which makes M separable.  In the BF16 kernels the accumulators start
// at the row's threshold H / 2 (raised by the accumulation error that start
// adds), so the test per element is a compare of the MFMA result with the
// column's G / 2, screened by an integer maximum.
//
// Layout (verified on the device): for v_mfma_f32_32x32x16_bf16 lane l holds
// 8 K-values of row/column l % 32 from K-half l / 32, and accumulator r of lane
// l is C[8 (r/4) + 4 (l/32) + r%4][l % 32].  Any permutation of K applied to
// both operands leaves the products unchanged, so each lane loads one
// contiguous half-row: step s of half h covers K [h len/2 + 8 s, +8) for BF16
// and [h len/2 + 32 s, +32) for FP8 (v_mfma_scale_f32_32x32x64_f8f6f4).
#include <type_traits>

#include "query_kernels.h"

namespace isax {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

constexpr float kInf = __builtin_huge_valf();
constexpr int kNT = 32;         // series per column tile (the columns of one MFMA)
// BF16: column tiles per staged tile, so one barrier and one loop step per
// 32 kFilterCols series; the 8-wave blocks (one per CU) take kFilterColsWide.
// Measured at 100M x 256, 1000 queries: 45.0 ms with one column tile, 41.1 ms
// with four (staged one column tile at a time).
constexpr int kFilterCols = 2;
constexpr int kFilterColsWide = 4;
constexpr int kBAhead = 6;      // BF16 B fragments in flight ahead of their MFMAs

__device__ inline unsigned long long make_key(float d2, int32_t id) {
    return ((unsigned long long)__float_as_uint(d2) << 32) | (unsigned)id;
}
__device__ inline unsigned long long load_relaxed(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline float read_tau(const QueryArgs& a, int q, int k) {
    const unsigned long long b = load_relaxed(a.bestk + (int64_t)q * a.kmax + (k - 1));
    const float t = b == ~0ull ? kInf : __uint_as_float((unsigned)(b >> 32));
    return fminf(t, a.tau0[q]);
}

// ---------------------------------------------------------------------------------------------
// Query codes (row-padded to dim with zeros) and per-query factors; batch
// maxima of |q|, |e_q| + gamma |q~| and |q|^2 go to qmax[0..2].
__device__ inline uint16_t bf16_rne(float x) {
    unsigned u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline uint8_t e4m3_rne(float y) {
    const unsigned sign = (__float_as_uint(y) >> 24) & 0x80u;
    const float a = fabsf(y);
    if (a == 0.f) return (uint8_t)sign;
    int e = ((int)((__float_as_uint(a) >> 23) & 255)) - 127;
    if (e < -6) return (uint8_t)(sign | (unsigned)rintf(a * 512.f));
    float q = rintf(ldexpf(a, 3 - e));
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
__device__ inline float up(float v) { return v * (1.0f + 0.0009765625f); }

__global__ void __launch_bounds__(64) k_quantise_queries(QueryArgs a, FilterArgs f, int len_pad, unsigned* qmax) {
    const int q = blockIdx.x;
    const int lane = threadIdx.x;
    const bool real = q < a.mq;
    const float* x = a.Q + (int64_t)q * a.len;
    float amax = 0.f;
    if (real)
        for (int t = lane; t < a.len; t += 64) amax = fmaxf(amax, fabsf(x[t]));
    for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
    float scale = 1.f;
    if (f.kind == 1 && amax > 0.f) {
        int e;
        const float fr = frexpf(amax / 448.f, &e);
        scale = ldexpf(1.f, fr == 0.5f ? e - 1 : e);
        if (amax / scale > 448.f) scale *= 2.f;
        if (amax / (scale * 0.5f) <= 448.f) scale *= 0.5f;
    }
    float qn = 0.f, en = 0.f, tn = 0.f;
    for (int t = lane; t < len_pad; t += 64) {
        const float v = (real && t < a.len) ? x[t] : 0.f;
        float vt;
        if (f.kind == 0) {
            const uint16_t b = bf16_rne(v);
            static_cast<uint16_t*>(f.qq)[(int64_t)q * len_pad + t] = b;
            vt = __uint_as_float((unsigned)b << 16);
        } else {
            const uint8_t b = e4m3_rne(v / scale);
            static_cast<uint8_t*>(f.qq)[(int64_t)q * len_pad + t] = b;
            vt = e4m3_val(b) * scale;
        }
        const float e = v - vt;
        qn = fmaf(v, v, qn);
        en = fmaf(e, e, en);
        tn = fmaf(vt, vt, tn);
    }
    for (int o = 32; o > 0; o >>= 1) {
        qn += __shfl_xor(qn, o, 64);
        en += __shfl_xor(en, o, 64);
        tn += __shfl_xor(tn, o, 64);
    }
    if (lane == 0) {
        const float nq = up(sqrtf(up(qn)));
        const float cq = up(up(sqrtf(up(en))) + f.gamma * up(sqrtf(up(tn))));
        f.qmeta[q] = make_float4(qn, nq, cq, scale);
        if (real) {
            atomicMax(qmax + 0, __float_as_uint(nq));
            atomicMax(qmax + 1, __float_as_uint(cq));
            atomicMax(qmax + 2, __float_as_uint(up(qn)));
        }
    }
}

// Spectral codes of the queries: ext(q) = (y_0 .. y_{D-2}, |(y_{D-1} ..)|), y = T q,
// computed in FP64 like the collection's copy (f.spec holds T transposed with a
// zero column D - 1), then the same BF16 codes and factors as above.  ext(q)
// is within 2^-18 |q| of the exact one (the tail norm comes from a difference
// of squares, |q|^2 - |y_head|^2, whose FP64 error is below 2e-12 |q|^2); that
// is added to |e_q|.  |ext(q)| = |q|, so |q| and |q|^2 keep their roles.
template <int RR>  // D = 64 RR coefficients, RR per lane
__global__ void __launch_bounds__(64) k_quantise_queries_spec(QueryArgs a, FilterArgs f, unsigned* qmax) {
    constexpr int RMAX = RR, D = 64 * RR;
    __shared__ float sq[512];  // the query row (len <= 512), read once with coalesced loads
    const int q = blockIdx.x;
    const int lane = threadIdx.x;
    const bool real = q < a.mq;
    const float* x = a.Q + (int64_t)q * a.len;
    for (int t = lane; t < a.len; t += 64) sq[t] = real ? x[t] : 0.f;
    __syncthreads();
    double y[RMAX];
#pragma unroll
    for (int r = 0; r < RMAX; ++r) y[r] = 0.0;
    double qn = 0.0;
#pragma unroll 8
    for (int j = 0; j < a.len; ++j) {
        const double v = (double)sq[j];
        qn = fma(v, v, qn);
        const double* tj = f.spec + (int64_t)j * D + lane;
#pragma unroll
        for (int r = 0; r < RMAX; ++r) y[r] = fma(tj[64 * r], v, y[r]);
    }
    double head = 0.0;
#pragma unroll
    for (int r = 0; r < RMAX; ++r) head = fma(y[r], y[r], head);
    for (int o = 32; o > 0; o >>= 1) head += __shfl_xor(head, o, 64);
    const double tail = sqrt(fmax(0.0, qn - head));
    double en = 0.0, tn = 0.0;
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
        const int i = lane + 64 * r;
        const double v = i == D - 1 ? tail : y[r];
        const uint16_t b = bf16_rne((float)v);
        static_cast<uint16_t*>(f.qq)[(int64_t)q * D + i] = b;
        const double vt = (double)__uint_as_float((unsigned)b << 16);
        en = fma(v - vt, v - vt, en);
        tn = fma(vt, vt, tn);
    }
    for (int o = 32; o > 0; o >>= 1) {
        en += __shfl_xor(en, o, 64);
        tn += __shfl_xor(tn, o, 64);
    }
    if (lane == 0) {
        const double nq = sqrt(qn);
        const float fq = up((float)nq);
        const float eq = up((float)(sqrt(en) * (1.0 + 0x1p-40) + 0x1p-18 * nq));
        const float cq = up(eq + f.gamma * up((float)(sqrt(tn) * (1.0 + 0x1p-40))));
        const float qn32 = (float)qn;
        f.qmeta[q] = make_float4(qn32, fq, cq, 1.f);
        if (real) {
            atomicMax(qmax + 0, __float_as_uint(fq));
            atomicMax(qmax + 1, __float_as_uint(cq));
            atomicMax(qmax + 2, __float_as_uint(up(qn32)));
        }
    }
}

// ---------------------------------------------------------------------------------------------
// The filter.  One 512-thread block per CU; each wave owns 32*MT queries whose
// codes stay in registers; the block streams tiles of 32 NC series (sorted
// order; NC column tiles of 32, one MFMA's columns each) through
// double-buffered LDS.  Blocks on one XCD that share a series
// stream but hold different query tiles walk the same tiles together, so the
// second read of a tile hits that XCD's L2.
template <int KIND, int KS, int MT, int WAVES, int NC>
struct FilterCfg {
    static constexpr int THREADS = 64 * WAVES;
    static constexpr int TS = kNT * NC;                        // series per tile (NC column tiles)
    static constexpr int EB = KIND == 0 ? 2 : 1;               // bytes per element
    static constexpr int KPS = KIND == 0 ? 16 : 64;            // K per MFMA step
    static constexpr int LEN_PAD = KS * KPS;
    static constexpr int ROW = LEN_PAD * EB;                   // bytes per row
    static constexpr int STRIDE = ROW + 16;                    // LDS row stride (bank spread)
    static constexpr int HALF = ROW / 2;
    static constexpr int STEP_B = KIND == 0 ? 16 : 32;         // bytes per lane per step
    static constexpr int CHUNKS = TS * ROW / 16;               // 16-B chunks per tile
    static constexpr int CPP = (CHUNKS / NC + THREADS - 1) / THREADS;  // per thread and column tile
    static constexpr int QPB = WAVES * 32 * MT;                // queries per block
};

// Scheduling groups of the BF16 step loop: per step one LDS read (while any
// are left) followed by the step's MT MFMAs.
template <int PF, int MT, int S, int KS>
__device__ inline void pin_schedule() {
    if constexpr (S < KS) {
        if constexpr (S + PF < KS) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, MT, 0);
        pin_schedule<PF, MT, S + 1, KS>();
    }
}

template <int KIND, int KS, int MT, int WAVES, int NC, bool INSPECT>
__global__ void __launch_bounds__(64 * WAVES) k_filter(QueryArgs a, FilterArgs f, int qtiles, int n_streams,
                                                        const unsigned* __restrict__ qmax) {
    using C = FilterCfg<KIND, KS, MT, WAVES, NC>;
    __shared__ __attribute__((aligned(16))) unsigned char tile[2][C::TS * C::STRIDE];
    __shared__ __attribute__((aligned(16))) float s_H[C::QPB];
    // BF16, eight-wave blocks of fewer than 16 MFMA steps (the spectral copy's 192
    // coefficients among them): each wave's candidates wait in LDS ({query row, sorted
    // position}) and are published when the list is full and at the end, so no tile
    // waits for the global atomics and loads of publishing them.  Measured on the
    // spectral copy (whose looser bound emits about three times the candidates): hybrid
    // +1.8%; on the 256-point rows -1.5%, which keep publishing at once, as do the
    // smaller blocks (the list would cost them a resident block per CU).
    constexpr bool kDefer = KIND == 0 && !INSPECT && WAVES >= 8 && KS < 16;
    constexpr int kPend = kDefer ? 64 : 1;
    __shared__ uint2 s_pend[WAVES][kPend];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 31, h = lane >> 5;
    const unsigned long long lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int n_pend = 0;  // wave-uniform
    auto publish = [&]() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane < n_pend) {
            const uint2 e = s_pend[wave][lane];
            const int q = (int)e.x;
            const int64_t pos = (int64_t)e.y;
            const int64_t h0 = a.home[2 * q] * a.leaf_size, h1 = a.home[2 * q + 1] * a.leaf_size;
            if (!(pos >= h0 && pos < h1)) {  // else already refined by the approximate answer
                const unsigned slot = atomicAdd(f.fcount + q, 1u);
                if (slot < (unsigned)f.fcap) f.fcand[(int64_t)q * f.fcap + slot] = (unsigned)pos;
            }
        }
        __builtin_amdgcn_wave_barrier();
        n_pend = 0;
    };
    // block -> (query tile, series stream), XCD-aware: blocks b, b+8, ... share an XCD
    const int b = blockIdx.x;
    const int xcd = b & 7, slot = b >> 3;
    const int qt = slot % qtiles;
    const int stream = (slot / qtiles) * 8 + xcd;
    const int q_base = qt * C::QPB + wave * 32 * MT;

    const float A = __uint_as_float(qmax[0]), Cq = __uint_as_float(qmax[1]), QN = __uint_as_float(qmax[2]);
    const float kappa = f.kappa;
    const float hslack = f.gamma * (1.f + 0x1p-10f) + 0x1p-22f;

    // query fragments: MT tiles x KS steps
    typedef typename std::conditional<KIND == 0, bf16x8, i32x8>::type Frag;
    Frag fa[MT][KS];
#pragma unroll
    for (int t = 0; t < MT; ++t) {
        const int q = q_base + 32 * t + r;
        const unsigned char* src = static_cast<const unsigned char*>(f.qq) + (int64_t)q * C::ROW + h * C::HALF;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            if constexpr (KIND == 0) {
                const i32x4 v = *reinterpret_cast<const i32x4*>(src + s * 16);
                fa[t][s] = __builtin_bit_cast(bf16x8, v);
            } else {
                const i32x4 v0 = *reinterpret_cast<const i32x4*>(src + s * 32);
                const i32x4 v1 = *reinterpret_cast<const i32x4*>(src + s * 32 + 16);
                i32x8 w;
                w[0] = v0[0]; w[1] = v0[1]; w[2] = v0[2]; w[3] = v0[3];
                w[4] = v1[0]; w[5] = v1[1]; w[6] = v1[2]; w[7] = v1[3];
                fa[t][s] = __builtin_bit_cast(Frag, w);
            }
        }
    }
    // per-row thresholds H = tau (1 + eps) - |q|^2 (refreshed periodically; BF16 keeps H / 2)
    // and FP8 row scales
    auto refresh_H = [&]() {
        // (rare: its addresses are recomputed here, through an empty asm, rather than kept in
        // registers across the tile loop)
        int i0 = threadIdx.x;
        asm volatile("" : "+v"(i0));
        for (int i = i0; i < C::QPB; i += C::THREADS) {
            const int q = qt * C::QPB + i;
            float H = -kInf;
            if (q < a.mq && !((a.rerun || a.skip_done) && a.done[q]))
                H = read_tau(a, q, a.kq[q]) * a.tau_scale - f.qmeta[q].x;
            // BF16: H / 2 is the accumulators' starting value; raised by more than the
            // accumulation error it adds (gamma |H / 2|), so that the sum stays above
            // H / 2 + q~.x~ - gamma |q~| |x~|
            float hv = KIND == 0 ? 0.5f * H : H;
            if (KIND == 0 && fabsf(hv) < kInf) hv += fabsf(hv) * hslack;
            s_H[i] = hv;
        }
    };
    refresh_H();
    // the query fragments stay resident for the whole kernel: wait for them once
    // here (vmcnt(0)), so waits inside the loop only cover the tile prefetch
    __builtin_amdgcn_s_waitcnt(0x0F70);
    float sq[MT][KIND == 1 ? 16 : 1];
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
        for (int e = 0; e < (KIND == 1 ? 16 : 1); ++e) {
            const int q = q_base + 32 * t + 8 * (e >> 2) + 4 * h + (e & 3);
            sq[t][e] = KIND == 1 ? f.qmeta[q].w : 1.f;
        }

    // tiles of this phase, enumerated as virtual tiles v = 0 .. n_vt-1
    // (n < 2^31, so tile numbers fit in 32 bits; kFilterSub is a constant, so the
    // division below is a multiply)
    // tiles of this phase, enumerated as virtual tiles v = 0 .. n_vt-1 (n < 2^31)
    constexpr int R = kFilterAlign / C::TS;
    const int n_tiles = (int)((a.n + C::TS - 1) / C::TS);
    const int n_samp = (int)filter_samples_before(n_tiles, R);
    const int64_t t_lo = f.range_lo / C::TS, t_hi = (f.range_hi + C::TS - 1) / C::TS;
    const int g_lo = (int)(t_lo - filter_samples_before(t_lo, R)), g_hi = (int)(t_hi - filter_samples_before(t_hi, R));
    const int n_sec = (int)filter_seconds_before(n_tiles, R);
    const int n_vt = f.phase == 0   ? n_tiles
                     : f.phase == 1 ? n_samp
                     : f.phase == 2 ? n_tiles - n_samp
                     : f.phase == 3 ? g_hi - g_lo
                     : f.phase == 4 ? n_sec
                                    : n_tiles - n_samp - n_sec;
    auto tile_of = [&](int v) -> int64_t {
        return f.phase == 0   ? v
               : f.phase == 1 ? filter_sample_tile(v, R)
               : f.phase == 2 ? filter_other_tile(v, R)
               : f.phase == 3 ? filter_other_tile(g_lo + v, R)
               : f.phase == 4 ? filter_second_tile(v, R)
                              : filter_rest_tile(v, R);
    };
    const unsigned char* X = static_cast<const unsigned char*>(f.xq);
    // one column tile's rows (part) at a time: the next tile's part p is loaded
    // while part p of this tile is computed, and stored into the free buffer after
    auto load_tile = [&](int64_t tl, int part, i32x4* stage) {
#pragma unroll
        for (int c = 0; c < C::CPP; ++c) {
            const int ch = part * (C::CHUNKS / NC) + threadIdx.x + c * C::THREADS;
            i32x4 v = {0, 0, 0, 0};
            if (ch < (part + 1) * (C::CHUNKS / NC)) {
                const int row = ch / (C::ROW / 16), col = ch % (C::ROW / 16);
                const int64_t pos = tl * C::TS + row;
                if (pos < a.n) v = *reinterpret_cast<const i32x4*>(X + pos * C::ROW + col * 16);
            }
            stage[c] = v;
        }
    };
    auto store_tile = [&](int buf, int part, const i32x4* stage) {
#pragma unroll
        for (int c = 0; c < C::CPP; ++c) {
            const int ch = part * (C::CHUNKS / NC) + threadIdx.x + c * C::THREADS;
            if (ch < (part + 1) * (C::CHUNKS / NC)) {
                const int row = ch / (C::ROW / 16), col = ch % (C::ROW / 16);
                *reinterpret_cast<i32x4*>(&tile[buf][row * C::STRIDE + col * 16]) = stage[c];
            }
        }
    };

    i32x4 stage[C::CPP];
    int v = stream;
    // per-series metadata of the current tile, fetched one tile ahead
    auto load_meta = [&](int64_t tile, int c) -> float4 {
        const int64_t p = tile * C::TS + kNT * c + r;
        return p < a.n ? f.xmeta[p] : make_float4(0.f, 0.f, 0.f, 0.f);
    };
    float4 m_cur[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) m_cur[c] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (v < n_vt) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            load_tile(tile_of(v), c, stage);
            m_cur[c] = load_meta(tile_of(v), c);
            store_tile(0, c, stage);
        }
    }
    __syncthreads();
    int buf = 0;
    int iter = 0;
    for (; v < n_vt; v += n_streams, buf ^= 1, ++iter) {
        const int64_t tl = tile_of(v);
        const bool has_next = v + n_streams < n_vt;
        const int64_t tn = has_next ? tile_of(v + n_streams) : 0;
        float4 m_next = m_cur[0];
        if (has_next) {
            load_tile(tn, 0, stage);
            m_next = load_meta(tn, 0);
        }
        // the NC column tiles of this tile, one after the other
#pragma unroll
        for (int c = 0; c < NC; ++c) {
        f32x16 acc[MT];
        constexpr bool kAccH = KIND == 0 && !INSPECT;  // accumulators start at the rows' H / 2
#pragma unroll
        for (int t = 0; t < MT; ++t)
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                float4 H4 = make_float4(0.f, 0.f, 0.f, 0.f);
                if constexpr (kAccH) H4 = *reinterpret_cast<const float4*>(&s_H[wave * 32 * MT + 32 * t + 8 * g + 4 * h]);
                acc[t][4 * g] = H4.x;
                acc[t][4 * g + 1] = H4.y;
                acc[t][4 * g + 2] = H4.z;
                acc[t][4 * g + 3] = H4.w;
            }
        const unsigned char* bsrc = &tile[buf][(kNT * c + r) * C::STRIDE + h * C::HALF];
        // B fragments read kBAhead steps ahead of the MFMAs that use them; the schedule is pinned
        // (reads first, then per step MT MFMAs and the next read) so that the LDS latency stays
        // hidden behind the matrix work instead of being waited for every second step
        if constexpr (KIND == 0) {
            constexpr int PF = KS < kBAhead / NC + 1 ? KS : kBAhead / NC + 1;
            bf16x8 bq[PF + 1];
#pragma unroll
            for (int s = 0; s < PF; ++s)
                bq[s] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const i32x4*>(bsrc + s * 16));
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                if (s + PF < KS)
                    bq[(s + PF) % (PF + 1)] =
                        __builtin_bit_cast(bf16x8, *reinterpret_cast<const i32x4*>(bsrc + (s + PF) * 16));
#pragma unroll
                for (int t = 0; t < MT; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[t][s], bq[s % (PF + 1)], acc[t], 0, 0, 0);
            }
            __builtin_amdgcn_sched_group_barrier(0x100, PF + (kAccH ? 4 * MT : 0), 0);  // DS reads
            pin_schedule<PF, MT, 0, KS>();
        } else {
            i32x8 bq[2];
            auto rd = [&](int s) {
                const i32x4 v0 = *reinterpret_cast<const i32x4*>(bsrc + s * 32);
                const i32x4 v1 = *reinterpret_cast<const i32x4*>(bsrc + s * 32 + 16);
                i32x8 bv;
                bv[0] = v0[0]; bv[1] = v0[1]; bv[2] = v0[2]; bv[3] = v0[3];
                bv[4] = v1[0]; bv[5] = v1[1]; bv[6] = v1[2]; bv[7] = v1[3];
                return bv;
            };
            bq[0] = rd(0);
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                if (s + 1 < KS) bq[(s + 1) % 2] = rd(s + 1);
#pragma unroll
                for (int t = 0; t < MT; ++t)
                    acc[t] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                        __builtin_bit_cast(i32x8, fa[t][s]), bq[s % 2], acc[t], 0, 0, 0, 127, 0, 127);
            }
        }
        // this lane's column: G = |x|^2 - M'(x), Fx = -2 s_x
        const int64_t pos = tl * C::TS + kNT * c + r;
        float G = kInf, Fx = -2.f, xn = 0.f, mx = 0.f;
        if (pos < a.n) {
            xn = m_cur[c].x;
            mx = 2.f * (A * m_cur[c].y + Cq * m_cur[c].z) + kappa * (QN + m_cur[c].x);
            G = m_cur[c].x - mx;
            Fx = -2.f * m_cur[c].w;
        }
        // epilogue: candidate iff fma(-2 s_q s_x, acc, G) <= H; rows 8g + 4h + 0..3 are consecutive
        if constexpr (INSPECT) {
#pragma unroll
            for (int t = 0; t < MT; ++t)
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int row = 32 * t + 8 * (e >> 2) + 4 * h + (e & 3);
                    const int q = q_base + row;
                    if (q < a.mq && pos < a.n) {
                        const float dot = KIND == 0 ? acc[t][e] : sq[t][KIND == 1 ? e : 0] * (-0.5f * Fx) * acc[t][e];
                        const int32_t id = a.ids_sorted[pos];
                        f.out_approx[(int64_t)q * a.n + id] = f.qmeta[q].x + xn - 2.f * dot;
                        f.out_margin[(int64_t)q * a.n + id] = mx;
                    }
                }
        } else if constexpr (KIND == 0) {
            // acc = H/2 + q~.x~ (the accumulators started at H/2): candidate iff acc >= G/2, the
            // test fma(-2, q~.x~, G) <= H halved.  A lane first takes the maximum of its 16 MT
            // values as integers (half a max3 per element and no quieting of the MFMA results):
            // for G/2 > 0 an element >= G/2 is positive and positive floats order as their bit
            // patterns, which are above every negative one.  Only lanes whose maximum passes (or
            // whose G/2 is not positive) look at the rows one by one.
            const float Gh = 0.5f * G;
            int best = -2147483647 - 1;
#pragma unroll
            for (int t = 0; t < MT; ++t)
#pragma unroll
                for (int e = 0; e < 16; e += 2)
                    best = max(max(best, __float_as_int(acc[t][e])), __float_as_int(acc[t][e + 1]));
            if (__ballot(!(Gh > 0.f) || best >= __float_as_int(Gh))) {
                unsigned hit = 0u;
#pragma unroll
                for (int t = 0; t < MT; ++t)
#pragma unroll
                    for (int e = 0; e < 16; ++e) hit |= (acc[t][e] >= Gh ? 1u : 0u) << (16 * t + e);
                if constexpr (!kDefer) {
                    while (hit) {
                        const int bit = __ffs(hit) - 1;
                        hit &= hit - 1u;
                        const int q = q_base + 32 * (bit >> 4) + 8 * ((bit & 15) >> 2) + 4 * h + (bit & 3);
                        if (q >= a.mq || pos >= a.n) continue;
                        const int64_t h0 = a.home[2 * q] * a.leaf_size, h1 = a.home[2 * q + 1] * a.leaf_size;
                        if (pos >= h0 && pos < h1) continue;  // already refined by the approximate answer
                        const unsigned slot = atomicAdd(f.fcount + q, 1u);
                        if (slot < (unsigned)f.fcap) f.fcand[(int64_t)q * f.fcap + slot] = (unsigned)pos;
                    }
                }
                if (pos >= a.n) hit = 0u;
                // each lane its lowest pending bit per round, into the wave's list
                for (; kDefer;) {
                    unsigned cand = 0u;
                    int q = 0;
                    while (hit && !cand) {
                        const int bit = __ffs(hit) - 1;
                        hit &= hit - 1u;
                        q = q_base + 32 * (bit >> 4) + 8 * ((bit & 15) >> 2) + 4 * h + (bit & 3);
                        cand = q < a.mq ? 1u : 0u;
                    }
                    const unsigned long long act = __ballot(cand != 0u);
                    if (!act) break;
                    if (n_pend + __popcll(act) > kPend) publish();
                    if (cand) s_pend[wave][n_pend + __popcll(act & lt_mask)] = make_uint2((unsigned)q, (unsigned)pos);
                    n_pend += __popcll(act);
                }
            }
        } else {
            unsigned hit = 0u;
#pragma unroll
            for (int t = 0; t < MT; ++t)
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const float4 H4 = *reinterpret_cast<const float4*>(&s_H[wave * 32 * MT + 32 * t + 8 * g + 4 * h]);
                    const float Hv[4] = {H4.x, H4.y, H4.z, H4.w};
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int e = 4 * g + u;
                        const float v = KIND == 0 ? fmaf(-2.f, acc[t][e], G) : fmaf(sq[t][KIND == 1 ? e : 0], Fx * acc[t][e], G);
                        hit |= (v <= Hv[u] ? 1u : 0u) << (16 * t + e);
                    }
                }
            if (__ballot(hit != 0u)) {
                while (hit) {
                    const int bit = __ffs(hit) - 1;
                    hit &= hit - 1u;
                    const int t = bit >> 4, e = bit & 15;
                    const int q = q_base + 32 * t + 8 * (e >> 2) + 4 * h + (e & 3);
                    if (q >= a.mq || pos >= a.n) continue;
                    const int64_t h0 = a.home[2 * q] * a.leaf_size, h1 = a.home[2 * q + 1] * a.leaf_size;
                    if (pos >= h0 && pos < h1) continue;  // already refined by the approximate answer
                    const unsigned slot = atomicAdd(f.fcount + q, 1u);
                    if (slot < (unsigned)f.fcap) f.fcand[(int64_t)q * f.fcap + slot] = (unsigned)pos;
                }
            }
        }
        // column c of this tile is done: its metadata makes room for the next tile's
        m_cur[c] = m_next;
        if (has_next) {
            store_tile(buf ^ 1, c, stage);
            if (c + 1 < NC) {
                load_tile(tn, c + 1, stage);
                m_next = load_meta(tn, c + 1);
            }
        }
        }  // column tiles
        if ((iter & 63) == 63) {
            __syncthreads();
            refresh_H();
        }
        __syncthreads();
    }
    if constexpr (kDefer)
        if (n_pend) publish();
}

// ---------------------------------------------------------------------------------------------
// The BF16 filter with its series tiles moved by the LDS DMA
// (global_load_lds_dwordx4): no staging registers, and the next tile is
// requested as a whole while the current one is computed, so a full tile of
// matrix work covers the load latency.  The two LDS buffers are distinct
// arrays handled in turn, so reads of one never wait for the transfers into
// the other.  Each DMA instruction of a wave fills 64 consecutive 16-byte
// slots of the padded layout (rows of STRIDE bytes; the last slot of a row is
// padding and receives a copy of the row's first chunk); rows past the end of
// the collection repeat its last series, whose columns the epilogue ignores.
// Candidates go to per-wave LDS lists (slots by lane rank, no LDS atomic,
// whose return would wait for the transfers in flight) and are published with
// global atomics after the tile, when no transfer is outstanding.
constexpr int kWaveHits = 32;  // candidates a wave holds in LDS per tile

template <int KS, int MT, int WAVES, int NC>
struct DmaCfg {
    using C = FilterCfg<0, KS, MT, WAVES, NC>;
    static constexpr int SLOTS = C::STRIDE / 16;                          // 16-byte slots per LDS row
    static constexpr int TOTAL = C::TS * SLOTS;                           // slots per tile
    static constexpr int NI = (TOTAL + 64 * WAVES - 1) / (64 * WAVES);    // DMA instructions per wave
    static constexpr size_t LDS = 2 * C::TS * C::STRIDE + C::QPB * 4 + C::QPB * 8 + WAVES * (kWaveHits * 8 + 4);
};

typedef __attribute__((address_space(3))) void lds_void;
typedef const __attribute__((address_space(1))) void global_void;

template <int KS, int MT, int WAVES, int NC>
__global__ void __launch_bounds__(64 * WAVES) k_filter_bf16(QueryArgs a, FilterArgs f, int qtiles, int n_streams,
                                                             const unsigned* __restrict__ qmax) {
    using C = FilterCfg<0, KS, MT, WAVES, NC>;
    using D = DmaCfg<KS, MT, WAVES, NC>;
    __shared__ __attribute__((aligned(16))) unsigned char tile0[C::TS * C::STRIDE];
    __shared__ __attribute__((aligned(16))) unsigned char tile1[C::TS * C::STRIDE];
    __shared__ __attribute__((aligned(16))) float s_H[C::QPB];
    __shared__ int2 s_home[C::QPB];                    // sorted positions [h0, h1) of each row's approximate answer
    __shared__ uint2 s_hits[WAVES * kWaveHits];        // {row in the block, sorted position}, per wave
    __shared__ unsigned s_nhits[WAVES];
    // the wave index in a scalar register: LDS targets and per-wave offsets stay scalar
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r = lane & 31, h = lane >> 5;
    const int b = blockIdx.x;
    const int xcd = b & 7, slot = b >> 3;
    const int qt = slot % qtiles;
    const int stream = (slot / qtiles) * 8 + xcd;
    const int row_base = wave * 32 * MT;  // this wave's first row in the block
    const int q_base = qt * C::QPB + row_base;

    const float A = __uint_as_float(qmax[0]), Cq = __uint_as_float(qmax[1]), QN = __uint_as_float(qmax[2]);
    const float kappa = f.kappa;
    const float hslack = f.gamma * (1.f + 0x1p-10f) + 0x1p-22f;

    bf16x8 fa[MT][KS];
#pragma unroll
    for (int t = 0; t < MT; ++t) {
        const int q = q_base + 32 * t + r;
        const unsigned char* src = static_cast<const unsigned char*>(f.qq) + (int64_t)q * C::ROW + h * C::HALF;
#pragma unroll
        for (int s = 0; s < KS; ++s)
            fa[t][s] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const i32x4*>(src + s * 16));
    }
    auto refresh_H = [&]() {
        // (rare: its addresses are recomputed here, through an empty asm, rather than kept in
        // registers across the tile loop)
        int i0 = threadIdx.x;
        asm volatile("" : "+v"(i0));
        for (int i = i0; i < C::QPB; i += C::THREADS) {
            const int q = qt * C::QPB + i;
            float H = -kInf;
            if (q < a.mq && !((a.rerun || a.skip_done) && a.done[q]))
                H = read_tau(a, q, a.kq[q]) * a.tau_scale - f.qmeta[q].x;
            // the accumulators' starting value, raised as in k_filter
            float hv = 0.5f * H;
            if (fabsf(hv) < kInf) hv += fabsf(hv) * hslack;
            s_H[i] = hv;
        }
    };
    refresh_H();
    for (int i = threadIdx.x; i < C::QPB; i += C::THREADS) {
        const int q = qt * C::QPB + i;
        int2 hr = make_int2(0, 0);
        if (q < a.mq)
            hr = make_int2((int)(a.home[2 * q] * a.leaf_size), (int)min(a.home[2 * q + 1] * a.leaf_size, a.n));
        s_home[i] = hr;
    }
    // rows of this lane that hold a query: bit 16 t + e for accumulator element e of tile t
    unsigned valid = 0u;
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
        for (int e = 0; e < 16; ++e)
            valid |= (q_base + 32 * t + 8 * (e >> 2) + 4 * h + (e & 3) < a.mq ? 1u : 0u) << (16 * t + e);
    unsigned wcount = 0u;  // this wave's candidates in the current tile (wave-uniform)

    // tiles of this phase, enumerated as virtual tiles v = 0 .. n_vt-1 (n < 2^31)
    constexpr int R = kFilterAlign / C::TS;
    const int n_tiles = (int)((a.n + C::TS - 1) / C::TS);
    const int n_samp = (int)filter_samples_before(n_tiles, R);
    const int64_t t_lo = f.range_lo / C::TS, t_hi = (f.range_hi + C::TS - 1) / C::TS;
    const int g_lo = (int)(t_lo - filter_samples_before(t_lo, R)), g_hi = (int)(t_hi - filter_samples_before(t_hi, R));
    const int n_sec = (int)filter_seconds_before(n_tiles, R);
    const int n_vt = f.phase == 0   ? n_tiles
                     : f.phase == 1 ? n_samp
                     : f.phase == 2 ? n_tiles - n_samp
                     : f.phase == 3 ? g_hi - g_lo
                     : f.phase == 4 ? n_sec
                                    : n_tiles - n_samp - n_sec;
    auto tile_of = [&](int v) -> int64_t {
        return f.phase == 0   ? v
               : f.phase == 1 ? filter_sample_tile(v, R)
               : f.phase == 2 ? filter_other_tile(v, R)
               : f.phase == 3 ? filter_other_tile(g_lo + v, R)
               : f.phase == 4 ? filter_second_tile(v, R)
                              : filter_rest_tile(v, R);
    };
    const unsigned char* X = static_cast<const unsigned char*>(f.xq);
    // the whole tile `tl` into `dst`: instruction j of this wave fills slots [64 (j WAVES + wave), +64).
    // The per-instruction offsets are recomputed for every tile from a laundered thread index (a
    // few VALU operations each) instead of being kept live across the loop.
    auto request = [&](unsigned char* dst, int64_t tl) {
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        const unsigned char* base = X + tl * C::TS * C::ROW;
        const int last = (int)min<int64_t>(a.n - tl * C::TS, C::TS) - 1;  // rows past it repeat it
#pragma unroll
        for (int j = 0; j < D::NI; ++j) {
            if ((j * WAVES + wave) * 64 < D::TOTAL) {
                const int p = j * 64 * WAVES + tid;
                const int row = p / D::SLOTS, sl = p - row * D::SLOTS;
                const int off = min(row, last) * C::ROW + (sl < D::SLOTS - 1 ? sl : 0) * 16;
                if (p < D::TOTAL)
                    __builtin_amdgcn_global_load_lds((global_void*)(base + off),
                                                     (lds_void*)(dst + (j * WAVES + wave) * 1024), 16, 0, 0);
            }
        }
    };
    // metadata {|x|^2, |e_x|, |x~|} of a tile's columns, loaded one tile ahead
    auto load_meta = [&](float3* m, int64_t tl) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int64_t p = tl * C::TS + kNT * c + r;
            float3 v = make_float3(0.f, 0.f, 0.f);
            if (p < a.n) {
                const float4 x = f.xmeta[p];
                v = make_float3(x.x, x.y, x.z);
            }
            m[c] = v;
        }
    };
    // G/2 = (|x|^2 - M'(x)) / 2 of a tile's columns (+inf past the end)
    auto thresholds = [&](float* Gh, const float3* m, int64_t tl) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int64_t p = tl * C::TS + kNT * c + r;
            const float G = m[c].x - (2.f * (A * m[c].y + Cq * m[c].z) + kappa * (QN + m[c].x));
            Gh[c] = p < a.n ? 0.5f * G : kInf;
        }
    };
    // the last tile's candidates: home-leaf check, then the query's list
    auto publish = [&]() {
        for (int i = threadIdx.x; i < WAVES * kWaveHits; i += C::THREADS) {
            if ((unsigned)(i % kWaveHits) >= min(s_nhits[i / kWaveHits], (unsigned)kWaveHits)) continue;
            const uint2 e = s_hits[i];
            const int2 hr = s_home[e.x];
            if ((int)e.y >= hr.x && (int)e.y < hr.y) continue;  // already refined by the approximate answer
            const int q = qt * C::QPB + (int)e.x;
            const unsigned sl = atomicAdd(f.fcount + q, 1u);
            if (sl < (unsigned)f.fcap) f.fcand[(int64_t)q * f.fcap + sl] = e.y;
        }
    };

    // one tile: the NC column tiles, each MT x KS MFMAs and the epilogue
    auto compute = [&](const unsigned char* buf, int64_t tl, const float* Ghs) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            f32x16 acc[MT];  // starts at the rows' H / 2
#pragma unroll
            for (int t = 0; t < MT; ++t)
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const float4 H4 = *reinterpret_cast<const float4*>(&s_H[row_base + 32 * t + 8 * g + 4 * h]);
                    acc[t][4 * g] = H4.x;
                    acc[t][4 * g + 1] = H4.y;
                    acc[t][4 * g + 2] = H4.z;
                    acc[t][4 * g + 3] = H4.w;
                }
            const unsigned char* bsrc = buf + (kNT * c + r) * C::STRIDE + h * C::HALF;
            constexpr int PF = KS < kBAhead / NC + 1 ? KS : kBAhead / NC + 1;
            bf16x8 bq[PF + 1];
#pragma unroll
            for (int s = 0; s < PF; ++s)
                bq[s] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const i32x4*>(bsrc + s * 16));
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                if (s + PF < KS)
                    bq[(s + PF) % (PF + 1)] =
                        __builtin_bit_cast(bf16x8, *reinterpret_cast<const i32x4*>(bsrc + (s + PF) * 16));
#pragma unroll
                for (int t = 0; t < MT; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[t][s], bq[s % (PF + 1)], acc[t], 0, 0, 0);
            }
            __builtin_amdgcn_sched_group_barrier(0x100, PF + 4 * MT, 0);
            pin_schedule<PF, MT, 0, KS>();
            const int64_t pos = tl * C::TS + kNT * c + r;
            // candidate iff acc >= G/2 (acc = H/2 + q~.x~), with the integer maximum first, as in k_filter
            const float Gh = Ghs[c];
            int best = -2147483647 - 1;
#pragma unroll
            for (int t = 0; t < MT; ++t)
#pragma unroll
                for (int e = 0; e < 16; e += 2)
                    best = max(max(best, __float_as_int(acc[t][e])), __float_as_int(acc[t][e + 1]));
            if (__ballot(!(Gh > 0.f) || best >= __float_as_int(Gh))) {
                unsigned hit = 0u;
#pragma unroll
                for (int t = 0; t < MT; ++t)
#pragma unroll
                    for (int e = 0; e < 16; ++e) hit |= (acc[t][e] >= Gh ? 1u : 0u) << (16 * t + e);
                hit &= pos < a.n ? valid : 0u;
                // one hit per lane and round, at slot wcount + (rank among the lanes with a hit)
                for (;;) {
                    const unsigned long long act = __ballot(hit != 0u);
                    if (!act) break;
                    if (hit) {
                        const int bit = __ffs(hit) - 1;
                        hit &= hit - 1u;
                        const int row = row_base + 32 * (bit >> 4) + 8 * ((bit & 15) >> 2) + 4 * h + (bit & 3);
                        const unsigned sl =
                            wcount + __builtin_amdgcn_mbcnt_hi((unsigned)(act >> 32),
                                                               __builtin_amdgcn_mbcnt_lo((unsigned)act, 0u));
                        if (sl < (unsigned)kWaveHits) {
                            s_hits[wave * kWaveHits + sl] = make_uint2((unsigned)row, (unsigned)pos);
                        } else {
                            // this wave's list is full: straight to the query's list
                            const int2 hr = s_home[row];
                            if (pos < hr.x || pos >= hr.y) {
                                const int q = qt * C::QPB + row;
                                const unsigned gs = atomicAdd(f.fcount + q, 1u);
                                if (gs < (unsigned)f.fcap) f.fcand[(int64_t)q * f.fcap + gs] = (unsigned)pos;
                            }
                        }
                    }
                    wcount += (unsigned)__popcll(act);
                }
            }
        }
    };

    float3 mN[NC];  // metadata of the next tile
    float Gh[NC];   // thresholds of the current tile
    int v = stream;
    if (v < n_vt) {
        load_meta(mN, tile_of(v));
        request(tile0, tile_of(v));
    }
    __syncthreads();
    int iter = 0;
    // end of a tile: candidates published, thresholds refreshed now and then
    auto finish_tile = [&]() {
        if (lane == 0) s_nhits[wave] = wcount;
        wcount = 0u;
        __syncthreads();
        bool any = false;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) any |= s_nhits[w] != 0u;
        if (any) publish();
        if ((++iter & 63) == 0) {
            __syncthreads();
            refresh_H();
        }
        __syncthreads();
    };
    // the tile in `cur`; the next one, if any, is requested into `nxt`
    auto step = [&](const unsigned char* cur, unsigned char* nxt, int vc) {
        const int64_t tl = tile_of(vc);
        thresholds(Gh, mN, tl);
        const int vn = vc + n_streams;
        if (vn < n_vt) {
            load_meta(mN, tile_of(vn));
            request(nxt, tile_of(vn));
        }
        compute(cur, tl, Gh);
        finish_tile();
    };
    for (; v < n_vt; v += 2 * n_streams) {
        step(tile0, tile1, v);
        if (v + n_streams >= n_vt) break;
        step(tile1, tile0, v + n_streams);
    }
}

// ---------------------------------------------------------------------------------------------
// Refinement of the filter's candidates: 16 lanes per candidate, FP32 direct
// differences, early abandoning against the current best-so-far; results in
// the slack window are emitted like in the iSAX scan.
__device__ void bestk_insert(unsigned long long* bk, int k, unsigned long long v) {
    int lo = 0, hi = k;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (load_relaxed(bk + mid) <= v) lo = mid + 1;
        else hi = mid;
    }
    for (int i = lo; i < k && v != ~0ull; ++i) {
        const unsigned long long old = atomicMin(bk + i, v);
        if (old > v) v = old;
    }
}

__global__ void __launch_bounds__(256) k_refine_filtered(QueryArgs a, FilterArgs f) {
    extern __shared__ float qrow[];
    const int q = blockIdx.y;
    if ((a.rerun || a.skip_done) && a.done[q]) return;
    const int k = a.kq[q];
    const unsigned cnt = min(f.fcount[q], (unsigned)f.fcap);
    if (cnt == 0) return;
    for (int t = threadIdx.x; t < a.len; t += 256) qrow[t] = a.Q[(int64_t)q * a.len + t];
    __syncthreads();
    const int g = threadIdx.x >> 4, gl = threadIdx.x & 15;
    const bool abandon = !(a.flags & ISAX_QF_NO_EARLY_ABANDON);
    // candidates of the spectral copy, whose bound is looser than the full rows': bounded
    // again with the full-row BF16 copy where the index holds it, before their FP32 rows
    // are read (the refinement precheck of the iSAX scan)
    const bool pc = f.spec && a.pc_x;
    const float pc_qn = pc ? a.qinfo[q].x : 0.f, pc_nq = sqrtf(pc_qn) * (1.f + 0x1p-20f);
    unsigned long long n_ref = 0, n_bytes = 0, n_emit = 0;
    for (unsigned i = blockIdx.x * 16 + g; i < cnt; i += gridDim.x * 16) {
        const unsigned pos = f.fcand[(int64_t)q * f.fcap + i];
        const float thr = read_tau(a, q, k) * a.tau_scale;
        if (pc && precheck16(a, pos, qrow, gl, pc_qn, pc_nq) > thr) continue;  // the same in the group's lanes
        const int32_t id = a.ids_sorted[pos];
        const float* row = series_row(a, pos, id);
        const int S = (a.len + 63) >> 6;
        float acc = 0.f;
        int steps = 0;
        bool dropped = false;
        for (int s = 0; s < S; ++s) {
            const int t0 = s * 64 + gl * 4;
            for (int e = 0; e < 4; ++e)
                if (t0 + e < a.len) {
                    const float d = qrow[t0 + e] - row[t0 + e];
                    acc = fmaf(d, d, acc);
                }
            steps = s + 1;
            if (abandon && s + 1 < S) {
                float part = acc;
                part += __shfl_xor(part, 1, 16);
                part += __shfl_xor(part, 2, 16);
                part += __shfl_xor(part, 4, 16);
                part += __shfl_xor(part, 8, 16);
                if (part > thr) {
                    dropped = true;
                    break;
                }
            }
        }
        float d2 = acc;
        d2 += __shfl_xor(d2, 1, 16);
        d2 += __shfl_xor(d2, 2, 16);
        d2 += __shfl_xor(d2, 4, 16);
        d2 += __shfl_xor(d2, 8, 16);
        if (gl == 0) {
            ++n_ref;
            n_bytes += (unsigned long long)min(a.len, steps * 64) * 4ull;
            if (!dropped && d2 <= thr) {
                const unsigned long long key = make_key(d2, id);
                const unsigned slot = atomicAdd(a.cand_count + q, 1u);
                if (slot < (unsigned)a.cap) a.cand[(int64_t)q * a.cap + slot] = key;
                if (!a.rerun && !(a.flags & ISAX_QF_NO_SHARING)) bestk_insert(a.bestk + (int64_t)q * a.kmax, k, key);
                ++n_emit;
            }
        }
    }
    if (gl == 0) {
        unsigned long long* st = a.stats + (int64_t)q * ST_N;
        if (n_ref) atomicAdd(st + ST_REFINED, n_ref);
        if (n_bytes) atomicAdd(st + ST_REFINE_BYTES, n_bytes);
        if (n_emit) atomicAdd(st + ST_CANDS, n_emit);
    }
}

// After a filter-candidate overflow: keep the k-th bound found so far in tau0
// and start the query's search state afresh (no series is inserted twice).
__global__ void k_filter_tighten(QueryArgs a, FilterArgs f) {
    const int q = blockIdx.x;
    const int k = a.kq[q];
    __shared__ float t;
    if (threadIdx.x == 0) t = read_tau(a, q, k);
    __syncthreads();
    for (int i = threadIdx.x; i < a.kmax; i += blockDim.x) a.bestk[(int64_t)q * a.kmax + i] = ~0ull;
    if (threadIdx.x == 0) {
        a.tau0[q] = t;
        a.cand_count[q] = 0u;
        f.fcount[q] = 0u;
    }
}

// Serving tables: whether a row lost filter candidates in this step, then the counts cleared.
__global__ void k_note_overflow(unsigned* __restrict__ fcount, int fcap, int mq, int* __restrict__ ovf) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= mq) return;
    ovf[q] = fcount[q] > (unsigned)fcap ? 1 : 0;
    fcount[q] = 0u;
}

// Per-query state between two batches (a serving table and an admission or
// final-ordering batch), one block per row.
__global__ void __launch_bounds__(256) k_copy_rows(QueryArgs sa, FilterArgs sf, QueryArgs da, FilterArgs df,
                                                   const int2* __restrict__ map, int free_src, int rows_too,
                                                   int len_pad, int code_bytes) {
    const int i = blockIdx.x;
    const int s = map[i].x, d = map[i].y;
    const int t = threadIdx.x;
    if (rows_too)
        for (int j = t; j < sa.len; j += 256)
            const_cast<float*>(da.Q)[(int64_t)d * da.len + j] = sa.Q[(int64_t)s * sa.len + j];
    const unsigned cnt = min(sa.cand_count[s], (unsigned)sa.cap);
    for (unsigned j = t; j < min(cnt, (unsigned)da.cap); j += 256) da.cand[(int64_t)d * da.cap + j] = sa.cand[(int64_t)s * sa.cap + j];
    for (int j = t; j < da.kmax; j += 256)
        da.bestk[(int64_t)d * da.kmax + j] = j < sa.kmax ? sa.bestk[(int64_t)s * sa.kmax + j] : ~0ull;
    if (t < ST_N) da.stats[(int64_t)d * ST_N + t] = sa.stats[(int64_t)s * ST_N + t];
    if (sf.qq && df.qq) {
        const unsigned char* src = static_cast<const unsigned char*>(sf.qq) + (int64_t)s * len_pad * code_bytes;
        unsigned char* dst = static_cast<unsigned char*>(df.qq) + (int64_t)d * len_pad * code_bytes;
        for (int j = t; j < len_pad * code_bytes; j += 256) dst[j] = src[j];
    }
    if (t == 0) {
        if (rows_too) const_cast<int32_t*>(da.kq)[d] = sa.kq[s];
        da.qkey[d] = sa.qkey[s];
        da.qinfo[d] = sa.qinfo[s];
        da.tau0[d] = sa.tau0[s];
        // candidates past the destination's capacity are reported as an overflow by its top-k
        da.cand_count[d] = sa.cand_count[s];
        da.home[2 * d] = sa.home[2 * s];
        da.home[2 * d + 1] = sa.home[2 * s + 1];
        da.status[d] = sa.status[s];
        da.done[d] = 0;
        if (sf.qmeta && df.qmeta) df.qmeta[d] = sf.qmeta[s];
        if (df.fcount) df.fcount[d] = 0u;
        if (free_src) sa.done[s] = 1;
    }
}

// Large batches: 8 waves x 64 queries per block, one block per CU.  Small
// batches (<= 64 queries): 2 waves x 32 queries, four blocks per CU; the pass is
// then bound by reading the reduced-precision copy, not by the matrix cores.
// Blocks of a kernel resident per CU (its registers and LDS), at least 1.
template <typename Kernel>
int resident_blocks(Kernel kernel, int threads) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, 0) != hipSuccess || nb < 1) {
        (void)hipGetLastError();
        nb = 1;
    }
    return nb;
}

template <int KIND, int KS, int MT, int WAVES>
void launch_filter_t(const QueryArgs& a, const FilterArgs& f, const unsigned* qmax, hipStream_t s) {
    // (the wide setting only where its double buffer fits the 160 KB of LDS: rows up to 512 bytes)
    constexpr int NC = KIND == 0 ? (WAVES >= 8 && KS * 32 <= 512 ? kFilterColsWide : kFilterCols) : 1;
    using C = FilterCfg<KIND, KS, MT, WAVES, NC>;
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int qtiles = (a.mq + C::QPB - 1) / C::QPB;
    // the kernel reads query rows [0, qtiles * QPB): they must exist in the padded codes
    if ((int64_t)qtiles * C::QPB > f.mq_pad)
        throw Error{ISAX_EINVAL, "internal: query codes padded to fewer rows than the filter reads"};
    static_assert(kFilterAlign % C::TS == 0, "the sample units and serving chunks start on a tile");
    constexpr int R = kFilterAlign / C::TS;
    const int64_t all_tiles = (a.n + C::TS - 1) / C::TS;
    const int64_t n_samp = filter_samples_before(all_tiles, R);
    int64_t n_tiles = all_tiles;
    const int64_t n_sec = filter_seconds_before(all_tiles, R);
    if (f.phase == 1) n_tiles = n_samp;
    if (f.phase == 2) n_tiles -= n_samp;
    if (f.phase == 4) n_tiles = n_sec;
    if (f.phase == 5) n_tiles -= n_samp + n_sec;
    if (f.phase == 3) {
        const int64_t t_lo = f.range_lo / C::TS, t_hi = (f.range_hi + C::TS - 1) / C::TS;
        n_tiles = (t_hi - filter_samples_before(t_hi, R)) - (t_lo - filter_samples_before(t_lo, R));
    }
    if (n_tiles <= 0) return;
    // n_streams * qtiles blocks, n_streams a multiple of 8 (one group per XCD); up to 4 blocks
    // per CU for the smaller classes, but no more than fit at once (registers and LDS), so the
    // grid runs in whole rounds: 4 requested where 3 fit left the last third of the blocks
    // running on a quarter of the chip
    auto go = [&](auto kernel, int resident) {
        const int per_cu = WAVES >= 8 ? 1 : std::min(4, resident);
        int n_streams = std::max(8, (per_cu * cus / qtiles) / 8 * 8);
        while (n_streams > 8 && n_streams / 2 >= n_tiles) n_streams /= 2;
        const int blocks = n_streams * qtiles;
        kernel<<<blocks, C::THREADS, 0, s>>>(a, f, qtiles, n_streams, qmax);
    };
    if (f.out_approx) {
        go(k_filter<KIND, KS, MT, WAVES, NC, true>, 1);
    } else if constexpr (KIND == 0 && WAVES == 2 && DmaCfg<KS, MT, WAVES, NC>::LDS <= 160 * 1024) {
        // the 64-query class is bound by streaming the BF16 copy: whole-tile DMA prefetch
        // (100M x 256: 8.6 against 9.3 ms; the larger classes were 5-7% slower with it)
        static const int res = resident_blocks(k_filter_bf16<KS, MT, WAVES, NC>, C::THREADS);
        go(k_filter_bf16<KS, MT, WAVES, NC>, res);
    } else {
        static const int res = resident_blocks(k_filter<KIND, KS, MT, WAVES, NC, false>, C::THREADS);
        go(k_filter<KIND, KS, MT, WAVES, NC, false>, res);
    }
}

// Batch-size classes: a block serves 64, 128, 256 or 512 queries, so a batch
// of m queries pads to at most twice m rows of matrix work (above 64).
template <int KIND, int KS, int MT>
void launch_filter_sized(const QueryArgs& a, const FilterArgs& f, const unsigned* qmax, hipStream_t s) {
    if (a.mq <= 64 && !f.out_approx) launch_filter_t<KIND, KS, 1, 2>(a, f, qmax, s);
    else if (a.mq <= 128 && !f.out_approx) launch_filter_t<KIND, KS, 1, 4>(a, f, qmax, s);
    // 129-256 queries: eight waves of 32 queries (one block per CU) beat four of
    // 64 (four blocks per CU): 15.0 against 17.7 ms at 100M x 256
    else if (a.mq <= 256 && !f.out_approx) launch_filter_t<KIND, KS, 1, 8>(a, f, qmax, s);
    else launch_filter_t<KIND, KS, MT, 8>(a, f, qmax, s);
}

}  // namespace

int filter_len_pad(int len) { return (len + 63) / 64 * 64; }

void launch_quantise_queries(const QueryArgs& a, const FilterArgs& f, int mq_pad, unsigned* qmax, hipStream_t s) {
    ProfScope ps("quantise_queries", s);
    if (f.spec) {
        if (f.kind != 0 || f.dim < 64 || f.dim > 256 || f.dim % 64)
            throw Error{ISAX_EINVAL, "internal: spectral codes need BF16 and 64..256 coefficients"};
        switch (f.dim / 64) {
            case 1: k_quantise_queries_spec<1><<<mq_pad, 64, 0, s>>>(a, f, qmax); break;
            case 2: k_quantise_queries_spec<2><<<mq_pad, 64, 0, s>>>(a, f, qmax); break;
            case 3: k_quantise_queries_spec<3><<<mq_pad, 64, 0, s>>>(a, f, qmax); break;
            default: k_quantise_queries_spec<4><<<mq_pad, 64, 0, s>>>(a, f, qmax); break;
        }
    } else {
        k_quantise_queries<<<mq_pad, 64, 0, s>>>(a, f, f.dim, qmax);
    }
    ISAX_HIP(hipGetLastError());
}

void launch_filter(const QueryArgs& a, const FilterArgs& f, const unsigned* qmax, hipStream_t s) {
    ProfScope ps(f.kind == 0 ? "filter_bf16" : "filter_fp8", s);
    const int lp = f.dim;
    if (f.kind == 0) {
        switch (lp) {
            case 64: launch_filter_t<0, 4, 2, 8>(a, f, qmax, s); break;
            case 128: launch_filter_sized<0, 8, 2>(a, f, qmax, s); break;
            case 192: launch_filter_sized<0, 12, 2>(a, f, qmax, s); break;
            case 256: launch_filter_sized<0, 16, 2>(a, f, qmax, s); break;
            case 320: launch_filter_t<0, 20, 1, 8>(a, f, qmax, s); break;
            case 384: launch_filter_t<0, 24, 1, 8>(a, f, qmax, s); break;
            case 448: launch_filter_t<0, 28, 1, 8>(a, f, qmax, s); break;
            case 512: launch_filter_t<0, 32, 1, 8>(a, f, qmax, s); break;
            default: throw Error{ISAX_EINVAL, "the reduced-precision filter supports len <= 512"};
        }
    } else {
        switch (lp) {
            case 64: launch_filter_t<1, 1, 2, 8>(a, f, qmax, s); break;
            case 128: launch_filter_sized<1, 2, 2>(a, f, qmax, s); break;
            case 192: launch_filter_t<1, 3, 2, 8>(a, f, qmax, s); break;
            case 256: launch_filter_sized<1, 4, 2>(a, f, qmax, s); break;
            case 320: launch_filter_t<1, 5, 2, 8>(a, f, qmax, s); break;
            case 384: launch_filter_t<1, 6, 2, 8>(a, f, qmax, s); break;
            case 448: launch_filter_t<1, 7, 2, 8>(a, f, qmax, s); break;
            case 512: launch_filter_t<1, 8, 2, 8>(a, f, qmax, s); break;
            default: throw Error{ISAX_EINVAL, "the reduced-precision filter supports len <= 512"};
        }
    }
    ISAX_HIP(hipGetLastError());
}

void launch_refine_filtered(const QueryArgs& a, const FilterArgs& f, hipStream_t s) {
    ProfScope ps("refine_filtered", s);
    const dim3 grid(64, (unsigned)a.mq);
    k_refine_filtered<<<grid, 256, (size_t)a.len * 4, s>>>(a, f);
    ISAX_HIP(hipGetLastError());
}

// Query rows the BF16 filter computes for a batch of mq queries: its block
// class (the dispatch of launch_filter) times the blocks.
int filter_rows_bf16(int dim, int mq) {
    const int lp = dim;
    int qpb = lp <= 256 ? 512 : 256;  // <MT = 2, 8 waves> below 320, <1, 8> from 320
    if ((lp == 128 || lp == 192 || lp == 256) && mq <= 256) qpb = mq <= 64 ? 64 : mq <= 128 ? 128 : 256;
    return (mq + qpb - 1) / qpb * qpb;
}

// Query codes are padded to a multiple of 512 rows, a multiple of every
// configuration's queries per block (64, 128, 256 or 512).
int filter_queries_per_block(int len) {
    (void)len;
    return 512;
}

void launch_note_overflow(const QueryArgs& a, const FilterArgs& f, int* ovf, hipStream_t s) {
    k_note_overflow<<<(a.mq + 255) / 256, 256, 0, s>>>(f.fcount, f.fcap, a.mq, ovf);
    ISAX_HIP(hipGetLastError());
}

void launch_copy_rows(const QueryArgs& sa, const FilterArgs& sf, const QueryArgs& da, const FilterArgs& df,
                      const int2* map, int n, bool free_src, hipStream_t s, bool rows_too) {
    if (n <= 0) return;
    ProfScope ps("copy_rows", s);
    k_copy_rows<<<n, 256, 0, s>>>(sa, sf, da, df, map, free_src ? 1 : 0, rows_too ? 1 : 0, sf.dim,
                                  sf.kind == 0 ? 2 : 1);
    ISAX_HIP(hipGetLastError());
}

void launch_filter_tighten(const QueryArgs& a, const FilterArgs& f, hipStream_t s) {
    k_filter_tighten<<<a.mq, 64, 0, s>>>(a, f);
    ISAX_HIP(hipGetLastError());
}

}  // namespace isax
