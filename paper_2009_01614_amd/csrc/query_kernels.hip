// Query kernels for gfx950: query preparation, approximate answer, the fused
// leaf-bound / series-bound / refinement scan, the plain FP32 scan, and the
// final top-k with a compensated-arithmetic tie guard.
//
// Paper, Sec. III (ParIS/ParIS+ and MESSI query answering): an approximate
// answer gives the best-so-far (BSF) distance; lower bounds between the query
// and leaves / iSAX summaries prune everything above the BSF; survivors get
// real distances, which may lower the BSF; the BSF at the end is the answer.
// Here the BSF is generalised to the k-th smallest distance (k-NN), kept per
// query in device memory as the k smallest (distance, id) keys, and every
// comparison carries a rounding slack so that FP32 arithmetic never prunes a
// true answer.
#include "query_kernels.h"

namespace isax {
namespace {

constexpr float kInf = __builtin_huge_valf();
constexpr unsigned long long kEmpty = ~0ull;

__device__ inline unsigned long long make_key(float d2, int32_t id) {
    return ((unsigned long long)__float_as_uint(d2) << 32) | (unsigned)id;
}
__device__ inline float key_d2(unsigned long long k) {
    return k == kEmpty ? kInf : __uint_as_float((unsigned)(k >> 32));
}
__device__ inline int32_t key_id(unsigned long long k) { return (int32_t)(unsigned)(k & 0xffffffffu); }

__device__ inline unsigned long long load_relaxed(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Current upper bound on the k-th smallest squared distance of query q.
__device__ inline float read_tau(const QueryArgs& a, int q, int k) {
    const float t = key_d2(load_relaxed(a.bestk + (int64_t)q * a.kmax + (k - 1)));
    return fminf(t, a.tau0[q]);
}

// Insert a key into the query's ascending list of the k smallest keys.  Every
// slot only ever decreases (atomic min), the displaced key moves on to the
// next slot, and the list stays sorted; slot k-1 therefore always bounds the
// k-th smallest key inserted so far.  The start slot is found by binary search:
// a slot observed <= v stays <= v.
__device__ void bestk_insert(unsigned long long* bk, int k, unsigned long long v) {
    int lo = 0, hi = k;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (load_relaxed(bk + mid) <= v) lo = mid + 1;
        else hi = mid;
    }
    for (int i = lo; i < k && v != kEmpty; ++i) {
        const unsigned long long old = atomicMin(bk + i, v);
        if (old > v) v = old;
    }
}

__device__ inline void emit(const QueryArgs& a, int q, int k, float d2, int32_t id) {
    const unsigned long long key = make_key(d2, id);
    const unsigned slot = atomicAdd(a.cand_count + q, 1u);
    if (slot < (unsigned)a.cap) a.cand[(int64_t)q * a.cap + slot] = key;
    if (!a.rerun && !(a.flags & ISAX_QF_NO_SHARING)) bestk_insert(a.bestk + (int64_t)q * a.kmax, k, key);
}

__device__ inline float sum64(float v) {
    for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Squared distance of the query (LDS) to one row, by a group of 16 lanes;
// a step covers 64 consecutive points (16 lanes x 4).  With `abandon`, the
// partial sum is compared with thr after every step but the last and the
// row is dropped (returns +inf) once it exceeds thr.  `steps` = steps read.
template <bool VEC>
__device__ float refine16(const float* __restrict__ row, const float* qrow, int len, int gl, float thr, bool abandon,
                          int& steps) {
    const int S = (len + 63) >> 6;
    float acc = 0.f;
    for (int s = 0; s < S; ++s) {
        const int t = s * 64 + gl * 4;
        if (VEC) {
            if (t < len) {
                const float4 x = *reinterpret_cast<const float4*>(row + t);
                const float4 qv = *reinterpret_cast<const float4*>(qrow + t);
                const float d0 = qv.x - x.x, d1 = qv.y - x.y, d2 = qv.z - x.z, d3 = qv.w - x.w;
                acc = fmaf(d0, d0, acc);
                acc = fmaf(d1, d1, acc);
                acc = fmaf(d2, d2, acc);
                acc = fmaf(d3, d3, acc);
            }
        } else {
            for (int e = 0; e < 4; ++e)
                if (t + e < len) {
                    const float d = qrow[t + e] - row[t + e];
                    acc = fmaf(d, d, acc);
                }
        }
        steps = s + 1;
        if (abandon && s + 1 < S) {
            const float part = sum16(acc);
            if (part > thr) return kInf;
        }
    }
    return sum16(acc);
}


// ---------------------------------------------------------------------------------------------
// DTW pieces.  The grid is D(i, j), i = query index, j = series index, band
// |i - j| <= r.  Filled column by column (j), column j is held as band cells
// D[d] = D(j - r + d, j), d = 0..2r; from column j-1 to j:
//   D(i-1, j-1) = old D[d],  D(i, j-1) = old D[d+1],  D(i-1, j) = new D[d-1].
// Cells beyond the band or the grid are +inf; D(-1, -1) = 0 is old D[r]
// before column 0.
constexpr int kDtwPad = 64;  // +inf entries on each side of the query row in LDS

// LDS copy of the query padded with +inf: qpad[kDtwPad + i] = q_i.
__device__ inline void load_qpad(float* qpad, const float* __restrict__ qg, int len) {
    for (int t = threadIdx.x; t < len + 2 * kDtwPad; t += blockDim.x) {
        const int i = t - kDtwPad;
        qpad[t] = (i >= 0 && i < len) ? qg[i] : kInf;
    }
}

// FP32 DTW^2 of one series per lane, RB >= 2r+1 band cells in registers.
// The query values come from LDS (the same address in every lane); cells
// d >= 2r+1 take +inf as query value and so stay +inf.  With `abandon` the
// lane stops once a whole column exceeds thr and returns +inf: every warping
// path crosses every column and D does not decrease along a path (in FP32
// too: fl(c + m) >= m for c >= 0).  `cols` = columns computed.
template <int RB, bool VEC>
__device__ float dtw_lane(const float* qpad, const float* __restrict__ row, int len, int r, float thr, bool abandon,
                          int& cols) {
    float D[RB];
#pragma unroll
    for (int d = 0; d < RB; ++d) D[d] = d == r ? 0.f : kInf;
    const int B = 2 * r + 1;
    const float* qw0 = qpad + kDtwPad - r;
    cols = 0;
    for (int j0 = 0; j0 < len; j0 += 4) {
        float xv[4];
        if (VEC) {
            const float4 v = *reinterpret_cast<const float4*>(row + j0);
            xv[0] = v.x;
            xv[1] = v.y;
            xv[2] = v.z;
            xv[3] = v.w;
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) xv[e] = j0 + e < len ? row[j0 + e] : 0.f;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (j0 + e < len) {
                const float* qw = qw0 + j0 + e;
                float left = kInf;
#pragma unroll
                for (int d = 0; d < RB; ++d) {
                    const float qv = d < B ? qw[d] : kInf;
                    const float df = qv - xv[e];
                    const float up = d + 1 < RB ? D[d + 1] : kInf;
                    const float m = fminf(fminf(D[d], up), left);
                    D[d] = fmaf(df, df, m);
                    left = D[d];
                }
            }
        }
        cols = min(len, j0 + 4);
        if (abandon && j0 + 4 < len) {
            float mn = D[0];
#pragma unroll
            for (int d = 1; d < RB; ++d) mn = fminf(mn, D[d]);
            if (mn > thr) return kInf;
        }
    }
    float res = kInf;
#pragma unroll
    for (int d = 0; d < RB; ++d)
        if (d == r) res = D[d];
    return res;
}

// DTW of the queued series dq[0..dn) by one wave, one series per lane, with
// refill: a lane that finishes or abandons takes the next queued series, so
// lanes do not idle while the longest series of a batch runs to the end.  The
// grid is walked row by row here (i = query index), band cells D[d] =
// D(i, i - r + d), d < B = 2r + 1 (a compile-time width); from row i-1 to i:
//   D(i-1, j-1) = old D[d],  D(i-1, j) = old D[d+1],  D(i, j-1) = new D[d-1].
// Rows go in groups of four: at a group's first row i0 the registers W[t] hold
// x_{i0-r+t}, t < B + 3 (+inf outside the series), and row i0 + e takes cell
// d's series value from W[d + e], so the window moves by four cells once per
// group instead of one cell per row.  A lane abandons once a whole row exceeds
// the bound (every warping path crosses every row).  Results within the bound
// are emitted.
struct DrainCounts {
    unsigned long long dtw, cells, emit;
};
template <int B, bool VEC>
__device__ DrainCounts dtw_drain(const QueryArgs& a, int q, int k, const float* qpad,
                                                           const int* dq, int dn, bool abandon, int lane,
                                                           unsigned long long lt) {
    unsigned long long n_dtw = 0, n_cells = 0, n_emit = 0;
    constexpr int r = (B - 1) / 2;
    const int len = a.len;
    float D[B], W[B + 3];
#pragma unroll
    for (int d = 0; d < B; ++d) D[d] = kInf;
#pragma unroll
    for (int t = 0; t < B + 3; ++t) W[t] = kInf;
    int row = len;  // >= len: no series
    int32_t id = 0;
    const float* x = a.data;
    int head = 0;
    float thr = read_tau(a, q, k) * a.tau_scale;
    float xn[4];  // the values entering the window at the end of the next group, loaded a group ahead
    auto load_xn = [&]() {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int jn = row + 4 + r + e;
            xn[e] = jn < len ? x[jn] : kInf;
        }
    };
    for (int it = 0;; ++it) {
        const bool idle = row >= len;
        const unsigned long long im = __ballot(idle);
        const int avail = dn - head;
        if (avail <= 0 && im == ~0ull) break;
        if (idle) {
            const int rank = __popcll(im & lt);
            if (rank < avail) {
                const int32_t pos = dq[head + rank];
                id = a.ids_sorted[pos];
                x = series_row(a, pos, id);
                row = 0;
#pragma unroll
                for (int d = 0; d < B; ++d) D[d] = d == r ? 0.f : kInf;
#pragma unroll
                for (int t = 0; t < B + 3; ++t) {
                    const int j = t - r;
                    W[t] = (j >= 0 && j < len) ? x[j] : kInf;
                }
                load_xn();
                ++n_dtw;
            }
        }
        if (avail > 0) head += min(avail, __popcll(im));
        if ((it & 7) == 7) thr = read_tau(a, q, k) * a.tau_scale;
        // the step runs in every lane (an idle lane computes on its stale state and discards it):
        // no per-lane branch around it, so the band is not held twice
        const bool active = row < len;
        {
            float qv[4];
            if (VEC) {
                const float4 q4 = *reinterpret_cast<const float4*>(qpad + kDtwPad + row);
                qv[0] = q4.x;
                qv[1] = q4.y;
                qv[2] = q4.z;
                qv[3] = q4.w;
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) qv[e] = qpad[kDtwPad + row + e];
            }
            float xc[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) xc[e] = xn[e];
            row += 4;
            load_xn();  // the group after this one (+inf past the end), in flight during this group
            row -= 4;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                // with len % 4 == 0 (VEC) every row of the group exists: no per-lane branch, so
                // the band is not held twice across it
                if (VEC || row + e < len) {
                    float left = kInf;
#pragma unroll
                    for (int d = 0; d < B; ++d) {
                        const float df = qv[e] - W[d + e];
                        const float up = d + 1 < B ? D[d + 1] : kInf;
                        const float m = fminf(fminf(D[d], up), left);
                        D[d] = fmaf(df, df, m);
                        left = D[d];
                    }
                }
            }
#pragma unroll
            for (int t = 0; t < B + 3; ++t) W[t] = t + 4 < B + 3 ? W[t + 4] : xc[t - (B - 1)];
        }
        if (active) {
            const int done_rows = min(4, len - row);
            n_cells += (unsigned long long)done_rows * B;
            row += 4;
            if (row >= len) {
                if (D[r] <= thr) {
                    emit(a, q, k, D[r], id);
                    ++n_emit;
                }
            } else if (abandon) {
                float mn = D[0];
#pragma unroll
                for (int d = 1; d < B; ++d) mn = fminf(mn, D[d]);
                if (mn > thr) row = len;
            }
        }
    }
    return DrainCounts{n_dtw, n_cells, n_emit};
}

// The drain for the bands of register class RB (the kernel's template), with
// the band width as a compile-time constant.
template <int RB, bool VEC>
__device__ void dtw_drain_for(const QueryArgs& a, int q, int k, const float* qpad, const int* dq, int dn,
                              bool abandon, int lane, unsigned long long lt, unsigned long long& n_dtw,
                              unsigned long long& n_cells, unsigned long long& n_emit) {
    DrainCounts c{0, 0, 0};
#define ISAX_DRAIN(BW) c = dtw_drain<BW, VEC>(a, q, k, qpad, dq, dn, abandon, lane, lt)
    if constexpr (RB == 64) {
        switch (a.window) {
            case 28: ISAX_DRAIN(57); break;
            case 29: ISAX_DRAIN(59); break;
            case 30: ISAX_DRAIN(61); break;
            default: ISAX_DRAIN(63); break;
        }
    } else if constexpr (RB == 56) {
        switch (a.window) {
            case 24: ISAX_DRAIN(49); break;
            case 25: ISAX_DRAIN(51); break;
            case 26: ISAX_DRAIN(53); break;
            default: ISAX_DRAIN(55); break;
        }
    } else if constexpr (RB == 48) {
        switch (a.window) {
            case 20: ISAX_DRAIN(41); break;
            case 21: ISAX_DRAIN(43); break;
            case 22: ISAX_DRAIN(45); break;
            default: ISAX_DRAIN(47); break;
        }
    } else if constexpr (RB == 40) {
        switch (a.window) {
            case 16: ISAX_DRAIN(33); break;
            case 17: ISAX_DRAIN(35); break;
            case 18: ISAX_DRAIN(37); break;
            default: ISAX_DRAIN(39); break;
        }
    } else {
        ISAX_DRAIN(RB - 1);
    }
#undef ISAX_DRAIN
    n_dtw += c.dtw;
    n_cells += c.cells;
    n_emit += c.emit;
}

// LB_Keogh^2 of one row against the query envelope (U, L in LDS) by a group of
// 16 lanes, 64 points per step, with the same early abandoning as refine16.
template <bool VEC>
__device__ float lbk16(const float* __restrict__ row, const float* U, const float* L, int len, int gl, float thr,
                       bool abandon, int& steps) {
    const int S = (len + 63) >> 6;
    float acc = 0.f;
    for (int s = 0; s < S; ++s) {
        const int t = s * 64 + gl * 4;
        if (VEC) {
            if (t < len) {
                const float4 x = *reinterpret_cast<const float4*>(row + t);
                const float4 u = *reinterpret_cast<const float4*>(U + t);
                const float4 l = *reinterpret_cast<const float4*>(L + t);
                const float d0 = fmaxf(0.f, fmaxf(x.x - u.x, l.x - x.x));
                const float d1 = fmaxf(0.f, fmaxf(x.y - u.y, l.y - x.y));
                const float d2 = fmaxf(0.f, fmaxf(x.z - u.z, l.z - x.z));
                const float d3 = fmaxf(0.f, fmaxf(x.w - u.w, l.w - x.w));
                acc = fmaf(d0, d0, acc);
                acc = fmaf(d1, d1, acc);
                acc = fmaf(d2, d2, acc);
                acc = fmaf(d3, d3, acc);
            }
        } else {
            for (int e = 0; e < 4; ++e)
                if (t + e < len) {
                    const float x = row[t + e];
                    const float d = fmaxf(0.f, fmaxf(x - U[t + e], L[t + e] - x));
                    acc = fmaf(d, d, acc);
                }
        }
        steps = s + 1;
        if (abandon && s + 1 < S) {
            const float part = sum16(acc);
            if (part > thr) return kInf;
        }
    }
    return sum16(acc);
}

// FP64 DTW^2 by one wave, lane d = band cell d (2r+1 <= 64): cell (column j,
// cell d) depends on (j-1, d), (j-1, d+1) and (j, d-1), so all cells with the
// same 2j + d are independent; step t computes them, taking the neighbours'
// values of step t-1 by lane shuffles.  Every cell is d = q_i - x_j in FP64,
// d * d rounded, + min rounded: the same value as any other order of filling
// the grid with these operations.
__device__ double dtw_exact_wave(const float* __restrict__ q, const float* __restrict__ x, int len, int r, int lane) {
    const double inf = __builtin_huge_val();
    const int B = 2 * r + 1;
    double own = inf;
    const int steps = 2 * (len - 1) + B;
    for (int t = 0; t < steps; ++t) {
        const double up = __shfl_down(own, 1, 64);
        const double left = __shfl_up(own, 1, 64);
        const int tj = t - lane;
        if (lane < B && tj >= 0 && (tj & 1) == 0 && (tj >> 1) < len) {
            const int j = tj >> 1, i = j - r + lane;
            double v = inf;
            if (i >= 0 && i < len) {
                const double u = lane + 1 < B ? up : inf;
                const double l = lane > 0 ? left : inf;
                const double m = (i == 0 && j == 0) ? 0.0 : fmin(fmin(own, u), l);
                const double df = (double)q[i] - (double)x[j];
                v = __dadd_rn(__dmul_rn(df, df), m);
            }
            own = v;
        }
    }
    return __shfl(own, r, 64);
}

// ---------------------------------------------------------------------------------------------
// Compensated squared distance (Ogita, Rump, Oishi, "Accurate sum and dot
// product", SIAM J. Sci. Comput. 2005: TwoSum / TwoProduct, Dot2).  The
// difference q - x is split exactly into dh + dl, dh^2 is split exactly with an
// FMA, and the running sum keeps its error term; lanes combine (sum, error)
// pairs by TwoSum in a butterfly, so every lane ends with the same pair.  The
// result (hi, lo) is normalised: hi = fl(hi + lo).  Relative error about
// len * 2^-48, far below the FP32 rounding of the sum.
__device__ inline void two_sum(float a, float b, float& s, float& e) {
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ float2 dist2_dot2(const float* __restrict__ q, const float* __restrict__ x, int len, int lane) {
    float S = 0.f, C = 0.f;
    for (int t = lane; t < len; t += 64) {
        float dh, dl;
        two_sum(q[t], -x[t], dh, dl);
        const float p = dh * dh;
        float pe = fmaf(dh, dh, -p);
        pe = fmaf(2.f * dh, dl, pe);
        pe = fmaf(dl, dl, pe);
        float s, e;
        two_sum(S, p, s, e);
        S = s;
        C = C + (e + pe);
    }
    for (int o = 1; o < 64; o <<= 1) {
        const float S2 = __shfl_xor(S, o, 64), C2 = __shfl_xor(C, o, 64);
        float s, e;
        two_sum(S, S2, s, e);
        S = s;
        C = (C + C2) + e;
    }
    const float hi = S + C;
    const float lo = C - (hi - S);
    return make_float2(hi, lo);
}

// ---------------------------------------------------------------------------------------------
__global__ void k_check_finite(const float* __restrict__ x, int64_t count, int* __restrict__ flag) {
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        bad |= !(fabsf(x[i]) <= 3.4028235e38f);
    if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

// FP32 mean of m consecutive values in a fixed order: a balanced tree of
// adjacent pairs over the values zero-padded to a power of two, then one
// division by m (the collection's PAA uses the same order).
__device__ inline float paa_tree(const float* src, int m) {
    int P = 1;
    while (P < m) P <<= 1;
    float stack[14];
    int level[14];
    int top = 0;
    for (int t = 0; t < P; ++t) {
        stack[top] = t < m ? src[t] : 0.f;
        level[top] = 0;
        ++top;
        while (top >= 2 && level[top - 1] == level[top - 2]) {
            stack[top - 2] = stack[top - 2] + stack[top - 1];
            level[top - 2] += 1;
            --top;
        }
    }
    return stack[0] / (float)m;
}

// Query preparation, one 64-lane block per query: FP32 PAA in the same fixed
// order as the collection's, the symbols and key, |q|^2 and max|q|, the
// widened region edges and the per-segment table T[j][s] = m * dist(query
// segment j, region s widened by delta)^2.  Under ED the query segment is the
// point p_j (its PAA); under DTW it is the interval [PAA(L)_j, PAA(U)_j] of
// the query's envelope (U, L: running max / min over i - r .. i + r), whose
// distance to a region bounds LB_Keogh and so DTW from below.
// delta = delta_x + m 2^-23 max|q| bounds the FP32 PAA error of both sides
// (envelope values are query values, so max|q| bounds them too); edges are
// moved one further ulp outwards after widening.
__global__ void __launch_bounds__(64) k_qprep(QueryArgs a) {
    extern __shared__ float s_env[];  // DTW: [2][len] upper then lower envelope
    const int q = blockIdx.x;
    const int lane = threadIdx.x;
    const float* row = a.Q + (int64_t)q * a.len;
    __shared__ float s_pu[64], s_pl[64];
    __shared__ int s_sym[64];
    const bool dtw = a.metric == ISAX_METRIC_DTW;
    // |q|^2 and max|q|
    float qn = 0.f, amax = 0.f;
    for (int t = lane; t < a.len; t += 64) {
        const float v = row[t];
        qn = fmaf(v, v, qn);
        amax = fmaxf(amax, fabsf(v));
    }
    qn = sum64(qn);
    for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
    if (dtw) {
        float* gu = a.qenv + (int64_t)q * 2 * a.len;
        for (int t = lane; t < a.len; t += 64) {
            float u = -kInf, l = kInf;
            for (int i = max(0, t - a.window); i <= min(a.len - 1, t + a.window); ++i) {
                u = fmaxf(u, row[i]);
                l = fminf(l, row[i]);
            }
            s_env[t] = u;
            s_env[a.len + t] = l;
            gu[t] = u;
            gu[a.len + t] = l;
        }
        __syncthreads();
    }
    // PAA, one lane per segment
    if (lane < a.w) {
        const int m = a.m_seg;
        const float p = paa_tree(row + lane * m, m);
        int s = 0;
        for (int step = 1 << (a.c - 1); step > 0; step >>= 1)
            if (a.beta[s + step - 1] <= p) s += step;
        s_sym[lane] = s;
        a.paa[(int64_t)q * a.w + lane] = p;
        const float pu = dtw ? paa_tree(s_env + lane * m, m) : p;
        const float pl = dtw ? paa_tree(s_env + a.len + lane * m, m) : p;
        s_pu[lane] = pu;
        s_pl[lane] = pl;
        a.env_paa[(int64_t)q * 2 * a.w + lane] = pu;
        a.env_paa[(int64_t)q * 2 * a.w + a.w + lane] = pl;
    }
    __syncthreads();
    if (lane < a.ws) a.sym[(int64_t)q * a.ws + lane] = lane < a.w ? (uint8_t)s_sym[lane] : 0;
    if (lane == 0) {
        unsigned long long key = 0;
        int pos = 0;
        for (int r = 0; r < a.c && pos < 64; ++r)
            for (int j = 0; j < a.w && pos < 64; ++j, ++pos)
                key |= (unsigned long long)((s_sym[j] >> (a.c - 1 - r)) & 1) << (63 - pos);
        a.qkey[q] = key;
    }
    const float delta = (a.delta_x + (float)a.m_seg * 1.1920929e-07f * amax) * 1.0001f;
    if (lane == 0) a.qinfo[q] = make_float4(qn, amax, delta, kInf);
    float* lo_e = a.edges + (int64_t)q * 2 * a.ns;
    float* hi_e = lo_e + a.ns;
    for (int s = lane; s < a.ns; s += 64) {
        lo_e[s] = s == 0 ? -kInf : nextafterf(a.beta[s - 1] - delta, -kInf);
        hi_e[s] = s == a.ns - 1 ? kInf : nextafterf(a.beta[s] + delta, kInf);
    }
    const float mf = (float)a.m_seg;
    float* T = a.T + (int64_t)q * a.w * a.ns;
    for (int idx = lane; idx < a.w * a.ns; idx += 64) {
        const int j = idx / a.ns, s = idx - j * a.ns;
        const float lo = s == 0 ? -kInf : nextafterf(a.beta[s - 1] - delta, -kInf);
        const float hi = s == a.ns - 1 ? kInf : nextafterf(a.beta[s] + delta, kInf);
        const float d = fmaxf(0.f, fmaxf(lo - s_pu[j], s_pl[j] - hi));
        T[idx] = mf * (d * d);
    }
    // per-query search state
    for (int i = lane; i < a.kmax; i += 64) a.bestk[(int64_t)q * a.kmax + i] = kEmpty;
    if (lane < ST_N) a.stats[(int64_t)q * ST_N + lane] = 0ull;
    if (lane == 0) {
        a.cand_count[q] = 0u;
        a.tau0[q] = kInf;
        a.done[q] = 0;
        a.status[q] = 0;
        a.home[2 * q] = 0;
        a.home[2 * q + 1] = 0;
    }
}

// ---------------------------------------------------------------------------------------------
// Bitonic sort of n (power of two) 64-bit keys in LDS by the whole block.
__device__ void bitonic_sort_u64(unsigned long long* v, int n) {
    for (int size = 2; size <= n; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            __syncthreads();
            for (int i = threadIdx.x; i < n / 2; i += blockDim.x) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const unsigned long long x = v[lo], y = v[hi];
                if ((x > y) == up) {
                    v[lo] = y;
                    v[hi] = x;
                }
            }
        }
    __syncthreads();
}

constexpr int kHomeMax = 4096;  // keys the approximate-answer block can sort
constexpr int kHomeLeaves = 4;  // the approximate answer covers at least this many leaves

// Approximate answer (MESSI: descend to the leaf of the query's iSAX summary
// and take the real distances of its series).  The home leaf is the last leaf
// whose first key is <= the query key; it is widened by neighbouring leaves
// (alternately after and before it) until it holds at least max(k, 4 leaves)
// series.  All its series are refined here (under DTW: the FP32 recurrence
// in full, one series per lane), the k smallest keys seed the best-so-far
// list, and those within the slack of the k-th are appended to the candidate
// list.  The scan skips these leaves.
template <int RB>
__global__ void __launch_bounds__(256) k_homeleaf(QueryArgs a) {
    extern __shared__ unsigned char smem_raw[];
    unsigned long long* keys = reinterpret_cast<unsigned long long*>(smem_raw);
    float* qrow = reinterpret_cast<float*>(keys + kHomeMax);
    __shared__ int64_t s_range[2];
    const int q = blockIdx.x;
    if (a.rerun && a.done[q]) return;
    const int k = a.kq[q];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) {
        const unsigned long long key = a.qkey[q];
        int64_t lo = 0, hi = a.n_leaves - 1;
        while (lo < hi) {  // last leaf with leaf_key <= key (leaf 0 if none)
            const int64_t mid = (lo + hi + 1) >> 1;
            if (a.leaf_key[mid] <= key) lo = mid;
            else hi = mid - 1;
        }
        int64_t l0 = lo, l1 = lo + 1;
        auto count = [&](int64_t x0, int64_t x1) { return min(a.n, x1 * a.leaf_size) - x0 * a.leaf_size; };
        const int64_t leaves = a.home_leaves > 0 ? a.home_leaves : kHomeLeaves;
        const int64_t want = max((int64_t)k, min(leaves * a.leaf_size, (int64_t)kHomeMax - 2 * 1024));
        while (count(l0, l1) < want && count(l0, l1) < a.n) {
            // grow alternately after and before the home leaf
            if ((l1 - l0) % 2 == 1 ? l1 < a.n_leaves : l0 == 0) {
                if (l1 < a.n_leaves) ++l1;
                else --l0;
            } else {
                --l0;
            }
        }
        s_range[0] = l0;
        s_range[1] = l1;
    }
    if constexpr (RB > 0) load_qpad(qrow, a.Q + (int64_t)q * a.len, a.len);
    else
        for (int t = threadIdx.x; t < a.len; t += blockDim.x) qrow[t] = a.Q[(int64_t)q * a.len + t];
    __syncthreads();
    const int64_t p0 = s_range[0] * a.leaf_size, p1 = min(a.n, s_range[1] * a.leaf_size);
    const int cnt = (int)(p1 - p0);
    int P = 1;
    while (P < cnt) P <<= 1;
    for (int i = cnt + threadIdx.x; i < P; i += blockDim.x) keys[i] = kEmpty;
    if constexpr (RB > 0) {
        const bool vec = a.len % 4 == 0 && (reinterpret_cast<uintptr_t>(a.data) & 15) == 0;
        for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
            const int32_t id = a.ids_sorted[p0 + i];
            const float* row = series_row(a, p0 + i, id);
            int cols = 0;
            const float v = vec ? dtw_lane<RB, true>(qrow, row, a.len, a.window, kInf, false, cols)
                                : dtw_lane<RB, false>(qrow, row, a.len, a.window, kInf, false, cols);
            keys[i] = make_key(v, id);
        }
    } else {
        // 16 lanes per series, four series per wave at a time (no early abandoning: these
        // values seed the bound)
        const bool vec = a.len % 4 == 0 && (reinterpret_cast<uintptr_t>(a.data) & 15) == 0;
        const int g = lane >> 4, gl = lane & 15;
        float* lbs = qrow + a.len + 2 * kDtwPad;  // [kHomeMax] precheck bounds
        if (a.pc_x && a.pc_home) {
            // the BF16 copy first: the k-th smallest upper bound approx + M over these series
            // bounds the k-th distance of the whole collection from above, and only the series
            // whose lower bound approx - M is within it can be answers (their rows are read)
            const float qn = a.qinfo[q].x, nq = sqrtf(qn) * (1.f + 0x1p-20f);
            for (int i = wave * 4 + g; i < cnt; i += (int)(blockDim.x / 64) * 4) {
                const float lb = precheck16(a, p0 + i, qrow, gl, qn, nq);
                const float4 m = a.pc_meta[p0 + i];
                const float M = (2.f * (nq * m.y + a.pc_gamma * nq * m.z) + a.pc_kappa * (qn + m.x)) * (1.f + 0x1p-20f);
                // ub = lb + 2 M, rounded up (ub >= ED^2 >= 0)
                const float ub = fmaxf(0.f, (lb + 2.f * M) * (1.f + 0x1p-20f) + 0x1p-100f);
                if (gl == 0) {
                    keys[i] = make_key(ub, i);
                    lbs[i] = lb;
                }
            }
            __syncthreads();
            bitonic_sort_u64(keys, P);
            const float tau = key_d2(keys[k - 1]);
            __syncthreads();
            for (int i = threadIdx.x; i < P; i += blockDim.x) keys[i] = kEmpty;
            __syncthreads();
            for (int i = wave * 4 + g; i < cnt; i += (int)(blockDim.x / 64) * 4) {
                if (!(lbs[i] <= tau)) continue;  // the same in the group's 16 lanes
                const int32_t id = a.ids_sorted[p0 + i];
                const float* row = series_row(a, p0 + i, id);
                int steps = 0;
                const float acc = vec ? refine16<true>(row, qrow, a.len, gl, kInf, false, steps)
                                      : refine16<false>(row, qrow, a.len, gl, kInf, false, steps);
                if (gl == 0) keys[i] = make_key(acc, id);
            }
        } else {
            for (int i = wave * 4 + g; i < cnt; i += (int)(blockDim.x / 64) * 4) {
                const int32_t id = a.ids_sorted[p0 + i];
                const float* row = series_row(a, p0 + i, id);
                int steps = 0;
                const float acc = vec ? refine16<true>(row, qrow, a.len, gl, kInf, false, steps)
                                      : refine16<false>(row, qrow, a.len, gl, kInf, false, steps);
                if (gl == 0) keys[i] = make_key(acc, id);
            }
        }
    }
    __syncthreads();
    bitonic_sort_u64(keys, P);
    const float thr = a.rerun ? read_tau(a, q, k) * a.tau_scale : key_d2(keys[k - 1]) * a.tau_scale;
    if (!a.rerun)
        for (int i = threadIdx.x; i < k; i += blockDim.x) a.bestk[(int64_t)q * a.kmax + i] = keys[i];
    // entries <= thr form a prefix of the sorted keys
    __shared__ int s_nc, s_read;
    if (threadIdx.x == 0) {
        s_nc = 0;
        s_read = 0;
    }
    __syncthreads();
    if (RB == 0 && a.pc_x && a.pc_home)
        for (int i = threadIdx.x; i < cnt; i += blockDim.x)
            if (keys[i] != kEmpty) atomicAdd(&s_read, 1);
    for (int i = threadIdx.x; i < cnt; i += blockDim.x)
        if (key_d2(keys[i]) <= thr) {
            atomicMax(&s_nc, i + 1);
            if (i < a.cap) a.cand[(int64_t)q * a.cap + i] = keys[i];
        }
    __syncthreads();
    if (threadIdx.x == 0) {
        a.cand_count[q] = (unsigned)s_nc;
        a.home[2 * q] = s_range[0];
        a.home[2 * q + 1] = s_range[1];
        if (!a.rerun) {
            float4 qi = a.qinfo[q];
            qi.w = key_d2(keys[k - 1]);
            a.qinfo[q] = qi;
            unsigned long long* st = a.stats + (int64_t)q * ST_N;
            const int n_read = RB == 0 && a.pc_x && a.pc_home ? s_read : cnt;  // rows read (the precheck skips the others)
            st[ST_REFINED] += (unsigned long long)n_read;
            st[ST_REFINE_BYTES] += (unsigned long long)n_read * a.len * 4ull;
            st[ST_CANDS] += (unsigned long long)s_nc;
            if (RB > 0) {
                st[ST_DTW] += (unsigned long long)cnt;
                st[ST_DTW_CELLS] += (unsigned long long)cnt * a.len * (2 * a.window + 1);
            }
        }
    }
}

// Squared lower bound of a query against a leaf's envelope: per segment the
// distance from the query segment [pl_j, pu_j] (ED: the PAA point) to
// [widened lower edge of lo, widened upper edge of hi] (the iSAX MINDIST of
// the union of the leaf's regions).
__device__ inline float env_bound(const QueryArgs& a, const uint8_t* el, const uint8_t* eh, const float* pu,
                                  const float* pl, const float* lo_e, const float* hi_e) {
    float lb = 0.f;
    for (int qc = 0; qc < a.ws / 16; ++qc) {
        const uint4 vl = reinterpret_cast<const uint4*>(el)[qc];
        const uint4 vh = reinterpret_cast<const uint4*>(eh)[qc];
        const unsigned ul[4] = {vl.x, vl.y, vl.z, vl.w};
        const unsigned uh[4] = {vh.x, vh.y, vh.z, vh.w};
#pragma unroll
        for (int b = 0; b < 16; ++b) {
            const int j = qc * 16 + b;
            if (j < a.w) {
                const int slo = (ul[b >> 2] >> (8 * (b & 3))) & 255;
                const int shi = (uh[b >> 2] >> (8 * (b & 3))) & 255;
                const float d = fmaxf(0.f, fmaxf(lo_e[slo] - pu[j], pl[j] - hi_e[shi]));
                lb = fmaf(d, d, lb);
            }
        }
    }
    return lb * (float)a.m_seg;
}
__device__ inline float leaf_bound(const QueryArgs& a, int64_t leaf, const float* pu, const float* pl,
                                   const float* lo_e, const float* hi_e) {
    return env_bound(a, a.env_lo + leaf * a.ws, a.env_hi + leaf * a.ws, pu, pl, lo_e, hi_e);
}

// The same bound for 16 segments with the envelope already in registers (the
// same operations in the same order as env_bound, so the same FP32 value).
__device__ inline float env_bound16(const QueryArgs& a, const uint4& vl, const uint4& vh, const float* pu,
                                    const float* pl, const float* lo_e, const float* hi_e) {
    const unsigned ul[4] = {vl.x, vl.y, vl.z, vl.w};
    const unsigned uh[4] = {vh.x, vh.y, vh.z, vh.w};
    float lb = 0.f;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int slo = (ul[j >> 2] >> (8 * (j & 3))) & 255;
        const int shi = (uh[j >> 2] >> (8 * (j & 3))) & 255;
        const float d = fmaxf(0.f, fmaxf(lo_e[slo] - pu[j], pl[j] - hi_e[shi]));
        lb = fmaf(d, d, lb);
    }
    return lb * (float)a.m_seg;
}

// Best-first order (MESSI's priority queues, by rounds): the bound of every
// leaf against the best-so-far of the approximate answer.  Per query: a
// histogram of the bounds over [0, bsf] in kLeafBins equal bins, the count of
// leaves within the bound, and the list of those leaves with their bounds (the
// first leaf_cap of them).  theta[q] = the lowest bin edge below which at least
// kFirstLeaves leaves lie; round 1 refines the listed leaves below theta, which
// lowers the best-so-far before round 2 takes the rest of the list.  A block
// takes 256 kHistLeafRounds leaves of kHistQueries queries: the queries'
// tables are loaded once for all those leaves.  The block first bounds its
// nodes (the envelope of 64 leaves, an inner node of the tree; one wave's
// leaves): the bound of a leaf is at least that of its node in FP32 too (every
// step is monotone in the envelope), so a node above the best-so-far rules
// out its leaves without bounding them.
// W16: 16 segments in 16-byte words; a thread's leaf envelope is then read
// once into registers for all the block's queries.
static_assert(kNodeLeaves == 64, "a node of the leaf pass is the 64 leaves of one wave");
template <bool W16>
__global__ void __launch_bounds__(256) k_leaf_hist(QueryArgs a) {
    constexpr int QB = kHistQueries, R = kHistLeafRounds;
    __shared__ float lo_e[QB][256], hi_e[QB][256], pu[QB][64], pl[QB][64];
    __shared__ unsigned hist[QB][kLeafBins];
    __shared__ float s_thr[QB];
    __shared__ int64_t s_home[QB][2];
    __shared__ unsigned s_valid[QB], s_kept[QB], s_base[QB];
    __shared__ unsigned char s_node_in[QB][4 * R];
    __shared__ int s_q[QB];
    // the block's queries: QB consecutive rows, or QB consecutive entries of the selection
    const int q0 = blockIdx.y * QB;
    const int nq = min(QB, (a.qsel ? a.nsel : a.mq) - q0);
    if (threadIdx.x < nq) s_q[threadIdx.x] = a.qsel ? a.qsel[q0 + threadIdx.x] : q0 + threadIdx.x;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    // nodes of 64 leaves: node nd of this block (nd = 4 r + wave) is node (16 blockIdx.x + nd) * stride;
    // with stride 1 the block takes 1024 consecutive leaves, with a larger one an even sample of nodes
    const int64_t stride = a.leaf_stride > 1 ? a.leaf_stride : 1;
    const int64_t base_leaf = (int64_t)blockIdx.x * 256 * R;  // (stride 1: the first leaf of the block)
    auto node_of = [&](int nd) -> int64_t { return ((int64_t)blockIdx.x * 4 * R + nd) * stride; };
    for (int i = 0; i < nq; ++i) {
        const int q = s_q[i];
        for (int s = threadIdx.x; s < a.ns; s += 256) {
            lo_e[i][s] = a.edges[(int64_t)q * 2 * a.ns + s];
            hi_e[i][s] = a.edges[(int64_t)q * 2 * a.ns + a.ns + s];
        }
        if (threadIdx.x < a.w) {
            pu[i][threadIdx.x] = a.env_paa[(int64_t)q * 2 * a.w + threadIdx.x];
            pl[i][threadIdx.x] = a.env_paa[(int64_t)q * 2 * a.w + a.w + threadIdx.x];
        }
        if (threadIdx.x < kLeafBins) hist[i][threadIdx.x] = 0u;
    }
    if (threadIdx.x < nq) {
        const int q = s_q[threadIdx.x];
        // a query set aside (skip_done) keeps no node and no leaf
        s_thr[threadIdx.x] = a.skip_done && a.done[q] ? -1.f : read_tau(a, q, a.kq[q]) * a.tau_scale;
        s_home[threadIdx.x][0] = a.home[2 * q];
        s_home[threadIdx.x][1] = a.home[2 * q + 1];
        s_valid[threadIdx.x] = 0u;
        s_kept[threadIdx.x] = 0u;
    }
    __syncthreads();
    // node bounds, one (query, node) pair per thread
    if (threadIdx.x < QB * 4 * R) {
        const int i = threadIdx.x / (4 * R), nd = threadIdx.x % (4 * R);
        const int64_t node = node_of(nd);
        bool in = false;
        if (i < nq && node < a.n_nodes)
            in = env_bound(a, a.node_lo + node * a.ws, a.node_hi + node * a.ws, pu[i], pl[i], lo_e[i], hi_e[i]) *
                     a.lb_scale <= s_thr[i];
        s_node_in[i][nd] = in;
    }
    __syncthreads();
    // per (query, leaf of this thread): the bound, and the slot of a kept leaf
    // among the block's kept leaves of that query
    float lbs[QB][R];
    int slot[QB][R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t leaf = node_of(r * 4 + (threadIdx.x >> 6)) * kNodeLeaves + lane;
        uint4 vl = make_uint4(0u, 0u, 0u, 0u), vh = vl;
        if constexpr (W16) {
            bool any_in = false;  // the same in every lane of the wave
#pragma unroll
            for (int i = 0; i < QB; ++i) any_in |= i < nq && s_node_in[i][r * 4 + (threadIdx.x >> 6)];
            if (any_in && leaf < a.n_leaves) {
                vl = *reinterpret_cast<const uint4*>(a.env_lo + leaf * 16);
                vh = *reinterpret_cast<const uint4*>(a.env_hi + leaf * 16);
            }
        }
#pragma unroll
        for (int i = 0; i < QB; ++i) {
            slot[i][r] = -1;
            lbs[i][r] = 0.f;
            if (i >= nq) continue;
            const float thr = s_thr[i];
            const bool valid = leaf < a.n_leaves && !(leaf >= s_home[i][0] && leaf < s_home[i][1]);
            const bool node_in = s_node_in[i][r * 4 + (threadIdx.x >> 6)];  // the same in every lane of the wave
            bool keep = false;
            float lb = 0.f;
            if (valid && node_in) {
                lb = W16 ? env_bound16(a, vl, vh, pu[i], pl[i], lo_e[i], hi_e[i])
                         : leaf_bound(a, leaf, pu[i], pl[i], lo_e[i], hi_e[i]);
                keep = lb * a.lb_scale <= thr;
            }
            if (keep) {
                // thr may be 0 (an exact duplicate) or +inf: keep the bin index in range
                const float f = thr > 0.f ? lb / thr * (float)kLeafBins : 0.f;
                const int bin = f < (float)(kLeafBins - 1) ? (int)f : kLeafBins - 1;
                atomicAdd(&hist[i][bin], 1u);
            }
            const unsigned long long km = __ballot(keep), vm = __ballot(valid);
            if (km) {
                int b = 0;
                if (lane == 0) b = (int)atomicAdd(&s_kept[i], (unsigned)__popcll(km));
                b = __shfl(b, 0, 64);
                if (keep) slot[i][r] = b + __popcll(km & lt);
            }
            lbs[i][r] = lb;
            if (lane == 0 && vm) atomicAdd(&s_valid[i], (unsigned)__popcll(vm));
        }
    }
    __syncthreads();
    // one atomic per query and block for the list position, then the entries
    if (threadIdx.x < nq && s_kept[threadIdx.x])
        s_base[threadIdx.x] = atomicAdd(a.leaf_count + s_q[threadIdx.x], s_kept[threadIdx.x]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < QB; ++i) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (slot[i][r] < 0) continue;
            const int64_t p = (int64_t)s_base[i] + slot[i][r];
            if (p < a.leaf_cap)
                a.leaf_list[(int64_t)s_q[i] * a.leaf_cap + p] =
                    make_uint2((unsigned)(node_of(r * 4 + (threadIdx.x >> 6)) * kNodeLeaves + lane),
                               __float_as_uint(lbs[i][r]));
        }
    }
    for (int i = 0; i < nq; ++i) {
        const int q = s_q[i];
        if (threadIdx.x < kLeafBins && hist[i][threadIdx.x])
            atomicAdd(a.leaf_hist + (int64_t)q * kLeafBins + threadIdx.x, hist[i][threadIdx.x]);
    }
    if (threadIdx.x < nq && s_valid[threadIdx.x])
        atomicAdd(a.stats + (int64_t)s_q[threadIdx.x] * ST_N + ST_LEAVES, (unsigned long long)s_valid[threadIdx.x]);
}

// After round 1: the leaves that round 2 would still take, counted from the
// list against the lowered best-so-far.
__global__ void __launch_bounds__(256) k_list_recount(QueryArgs a) {
    const int q = blockIdx.y;
    if (a.done[q]) return;
    const unsigned n = a.leaf_count[q];
    if ((int64_t)n > a.leaf_cap) return;
    const float thr = read_tau(a, q, a.kq[q]) * a.tau_scale;
    const float theta = a.theta[q];
    unsigned c = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < (int64_t)n; i += (int64_t)gridDim.x * 256) {
        const float lb = __uint_as_float(a.leaf_list[(int64_t)q * a.leaf_cap + i].y);
        c += (lb * a.lb_scale <= thr && !(lb < theta)) ? 1u : 0u;
    }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(a.list_rest + q, c);
}

__global__ void k_leaf_theta(QueryArgs a) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.mq) return;
    const float thr = read_tau(a, q, a.kq[q]) * a.tau_scale;
    unsigned cum = 0;
    float theta = kInf;
    for (int b = 0; b < kLeafBins; ++b) {
        cum += a.leaf_hist[(int64_t)q * kLeafBins + b];
        if (cum >= (unsigned)kFirstLeaves) {
            theta = (float)(b + 1) / kLeafBins * thr;
            break;
        }
    }
    a.theta[q] = theta;
}

// ---------------------------------------------------------------------------------------------
// The iSAX scan, one block per (query, tile of 256 leaves).
//  1. leaf lower bound from the widened region edges of the leaf's envelope
//     (Sec. III, MESSI: prune subtrees / leaves whose bound exceeds the BSF);
//  2. for every surviving leaf, one wave computes the lower bound of each
//     series from its word with the per-segment LDS table (ParIS / MESSI
//     lower-bound calculation on the iSAX summaries);
//  3. ED (RB = 0): each surviving series is refined by 16 lanes with early
//     abandoning, and results within the slack of the current BSF are
//     emitted (candidate list + best-so-far update).
//     DTW (RB = band registers): 16 lanes compute LB_Keogh with early
//     abandoning; the survivors queue up per wave and, 64 at a time, get the
//     FP32 DTW recurrence, one series per lane, with early abandoning.
// With all_leaves (the plain scan under DTW) steps 1 and 2 keep everything.
struct ScanSmem {
    int off_lo, off_hi, off_paa, off_q, off_env, off_T, off_list, off_wl, off_dq, total;
};
// The series-bound table sits in LDS when it is at most 32 KB and the whole
// plan fits in 64 KB, else it is read from global memory (L2-resident: one
// table per query).
constexpr int kTableLdsMax = 32 * 1024;
constexpr int kDtwQueue = 512;   // per-wave queue of series waiting for DTW
constexpr int kDtwDrainAt = 448; // queue length that starts a drain (at most 3 more arrive per step)
__host__ __device__ inline ScanSmem scan_smem(int ns, int w, int len, bool dtw, bool table_in_lds) {
    ScanSmem s;
    int o = 0;
    s.off_lo = o; o += ns * 4;
    s.off_hi = o; o += ns * 4;
    s.off_paa = o; o += 128 * 4;
    s.off_q = o; o += (dtw ? len + 2 * kDtwPad : (len + 3) / 4 * 4) * 4;
    o = (o + 15) / 16 * 16;
    s.off_env = o; o += dtw ? 2 * ((len + 3) / 4 * 4) * 4 : 0;
    s.off_T = o; o += table_in_lds ? w * ns * 4 : 0;
    s.off_list = o; o += 257 * 4;
    o = (o + 15) / 16 * 16;
    s.off_wl = o; o += 4 * 64 * 4;
    s.off_dq = o; o += dtw ? 4 * kDtwQueue * 4 : 0;
    s.total = o;
    return s;
}

template <bool VEC, bool T_LDS, int RB>
__global__ void __launch_bounds__(256) k_index_scan(QueryArgs a) {
    constexpr bool DTW = RB > 0;
    // queue drained with lane refill (dtw_drain) for the bands where it measured faster
    constexpr bool REFILL = RB >= 40;
    extern __shared__ unsigned char smem[];
    const ScanSmem L = scan_smem(a.ns, a.w, a.len, DTW, T_LDS);
    float* lo_e = reinterpret_cast<float*>(smem + L.off_lo);
    float* hi_e = reinterpret_cast<float*>(smem + L.off_hi);
    float* pu = reinterpret_cast<float*>(smem + L.off_paa);
    float* pl = pu + 64;
    float* qrow = reinterpret_cast<float*>(smem + L.off_q);  // DTW: padded query
    float* envU = reinterpret_cast<float*>(smem + L.off_env);
    float* envL = envU + (a.len + 3) / 4 * 4;
    const float* T = T_LDS ? reinterpret_cast<const float*>(smem + L.off_T) : a.T + (int64_t)blockIdx.y * a.w * a.ns;
    int* list = reinterpret_cast<int*>(smem + L.off_list);
    int* wl = reinterpret_cast<int*>(smem + L.off_wl);
    __shared__ int s_nk;
    __shared__ unsigned long long s_st[ST_N];

    const int q = blockIdx.y;
    // finished queries (re-runs), and queries that a hybrid batch hands to the filter
    if (a.done[q]) return;
    const int k = a.kq[q];
    // (the refinement precheck's query norms)
    const float pc_qn = a.pc_x ? a.qinfo[q].x : 0.f, pc_nq = sqrtf(pc_qn) * (1.f + 0x1p-20f);
    // The precheck reads a BF16 row and its metadata; it pays where early abandoning
    // reads more FP32 bytes than that per series.  A wave refines the candidates of its
    // first step (4 per step, one per group of 16 lanes) and then of every 64th step
    // without it, and prechecks the others while the FP32 bytes of those samples
    // average above the BF16 row's (rows in host memory: always, an FP32 read crosses
    // the bus there).  The choice is the same in the whole wave, so its groups do not
    // take both paths in one step.  Either way a series whose FP32 distance can be
    // within the bound is refined, so the answer is the same.
    const float pc_row = 2.f * a.pc_stride + 16.f;
    unsigned pc_it = 0;
    float pc_n = 0.f, pc_b = 0.f;  // wave-uniform
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t leaf_id = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t h0 = a.home[2 * q], h1 = a.home[2 * q + 1];

    for (int s = threadIdx.x; s < a.ns; s += 256) {
        lo_e[s] = a.edges[(int64_t)q * 2 * a.ns + s];
        hi_e[s] = a.edges[(int64_t)q * 2 * a.ns + a.ns + s];
    }
    if (threadIdx.x < a.w) {
        pu[threadIdx.x] = a.env_paa[(int64_t)q * 2 * a.w + threadIdx.x];
        pl[threadIdx.x] = a.env_paa[(int64_t)q * 2 * a.w + a.w + threadIdx.x];
    }
    if (threadIdx.x < ST_N) s_st[threadIdx.x] = 0ull;
    if (threadIdx.x == 0) s_nk = 0;
    __syncthreads();

    float thr = read_tau(a, q, k) * a.tau_scale;
    // rounds 1 and 2 take the query's leaf list when it holds every leaf within
    // the first bound (block x = a tile of list entries), else all leaves again
    const unsigned n_list = a.round != 0 ? a.leaf_count[q] : 0u;
    const bool from_list = a.round != 0 && n_list <= (uint64_t)a.leaf_cap;
    bool valid_leaf = false, keep = false;
    int64_t leaf = leaf_id;
    if (from_list) {
        if (leaf_id < (int64_t)n_list) {
            const uint2 e = a.leaf_list[(int64_t)q * a.leaf_cap + leaf_id];
            leaf = e.x;
            const float lb = __uint_as_float(e.y);
            valid_leaf = true;
            keep = lb * a.lb_scale <= thr && (a.round == 1 ? lb < a.theta[q] : !(lb < a.theta[q]));
        }
    } else if (leaf_id < a.n_leaves && !(leaf_id >= h0 && leaf_id < h1)) {
        valid_leaf = true;
        if (DTW && a.all_leaves) {
            keep = true;
        } else {
            const float lb = leaf_bound(a, leaf_id, pu, pl, lo_e, hi_e);
            keep = lb * a.lb_scale <= thr;
            if (a.round == 1) keep = keep && lb < a.theta[q];
            if (a.round == 2) keep = keep && !(lb < a.theta[q]);
        }
    }
    {
        const unsigned long long vm = __ballot(valid_leaf), km = __ballot(keep);
        const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
        int base = 0;
        if (lane == 0) base = atomicAdd(&s_nk, __popcll(km));
        base = __shfl(base, 0, 64);
        if (keep) list[base + __popcll(km & lt)] = (int)leaf;
        if (lane == 0) {
            // the leaf pass before the rounds counted every leaf bound
            if (a.round == 0) atomicAdd(&s_st[ST_LEAVES], (unsigned long long)__popcll(vm));
            atomicAdd(&s_st[ST_LEAVES_KEPT], (unsigned long long)__popcll(km));
        }
    }
    __syncthreads();
    const int nk = s_nk;
    if (nk > 0) {
        if (T_LDS) {
            float* Tw = reinterpret_cast<float*>(smem + L.off_T);
            for (int i = threadIdx.x; i < a.w * a.ns; i += 256) Tw[i] = a.T[(int64_t)q * a.w * a.ns + i];
        }
        if constexpr (DTW) {
            load_qpad(qrow, a.Q + (int64_t)q * a.len, a.len);
            const float* ge = a.qenv + (int64_t)q * 2 * a.len;
            for (int t = threadIdx.x; t < a.len; t += 256) {
                envU[t] = ge[t];
                envL[t] = ge[a.len + t];
            }
        } else {
            for (int t = threadIdx.x; t < a.len; t += 256) qrow[t] = a.Q[(int64_t)q * a.len + t];
        }
        __syncthreads();
        const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
        const bool abandon = !(a.flags & ISAX_QF_NO_EARLY_ABANDON);
        const bool series_lb = !(DTW && a.all_leaves);
        unsigned long long n_lb = 0, n_ref = 0, n_bytes = 0, n_emit = 0, n_dtw = 0, n_cells = 0, n_pc = 0;
        int* my_wl = wl + wave * 64;
        int* dq = reinterpret_cast<int*>(smem + L.off_dq) + wave * kDtwQueue;
        int dn = 0;  // queued series of this wave (the same in every lane)
        // narrow bands (where three or more waves per SIMD fit this way) and the widest (no room
        // for the refill state at two waves per SIMD): batches of 64, one series per lane, column by
        // column with the query values broadcast from LDS
        auto dtw_batch = [&](int cnt) {
            thr = read_tau(a, q, k) * a.tau_scale;
            if (lane < cnt) {
                const int32_t pos = dq[lane];
                const int32_t id = a.ids_sorted[pos];
                int cols = 0;
                const float d2 = dtw_lane<DTW ? RB : 8, VEC>(qrow, series_row(a, pos, id), a.len, a.window, thr,
                                                             abandon, cols);
                ++n_dtw;
                n_cells += (unsigned long long)cols * (2 * a.window + 1);
                if (d2 <= thr) {
                    emit(a, q, k, d2, id);
                    ++n_emit;
                }
            }
            thr = read_tau(a, q, k) * a.tau_scale;
        };
        for (int li = wave; li < nk; li += 4) {
            const int64_t lf = list[li];
            const int64_t pa = lf * a.leaf_size, pb = min(a.n, pa + a.leaf_size);
            thr = read_tau(a, q, k) * a.tau_scale;
            for (int64_t base = pa; base < pb; base += 64) {
                const int64_t pos = base + lane;
                const bool v = pos < pb;
                float lb = 0.f;
                if (v && series_lb) {
                    const uint4* wp = reinterpret_cast<const uint4*>(a.words_sorted + pos * a.ws);
                    for (int qc = 0; qc < a.ws / 16; ++qc) {
                        const uint4 vw = wp[qc];
                        const unsigned u[4] = {vw.x, vw.y, vw.z, vw.w};
#pragma unroll
                        for (int b = 0; b < 16; ++b) {
                            const int j = qc * 16 + b;
                            if (j < a.w) lb += T[j * a.ns + ((u[b >> 2] >> (8 * (b & 3))) & 255)];
                        }
                    }
                }
                const bool pass = v && lb * a.lb_scale <= thr;
                const unsigned long long pm = __ballot(pass);
                if (series_lb) n_lb += (unsigned long long)__popcll(__ballot(v));
                if (pm == 0ull) continue;
                if (pass) my_wl[__popcll(pm & lt)] = (int)(pos - pa);
                __builtin_amdgcn_wave_barrier();
                const int nc = __popcll(pm);
                const int g = lane >> 4, gl = lane & 15;
                for (int ci = 0; ci < nc; ci += 4) {
                    const int my = ci + g;
                    if constexpr (DTW) {
                        bool surv = false;
                        int32_t p2 = 0;  // sorted position; the queue holds positions
                        if (my < nc) {
                            p2 = (int32_t)(pa + my_wl[my]);
                            int steps = 0;
                            const float lk = lbk16<VEC>(series_row(a, p2, a.ids_sorted[p2]), envU, envL, a.len, gl,
                                                        thr, abandon, steps);
                            surv = lk * a.lbk_scale <= thr;
                            if (gl == 0) {
                                ++n_ref;
                                n_bytes += (unsigned long long)min(a.len, steps * 64) * 4ull;
                            }
                        }
                        const unsigned long long sm = __ballot(surv && gl == 0);
                        if (surv && gl == 0) dq[dn + __popcll(sm & lt)] = p2;
                        dn += __popcll(sm);
                        __builtin_amdgcn_wave_barrier();
                        if (REFILL && dn >= kDtwDrainAt) {
                            dtw_drain_for<REFILL ? RB : 8, VEC>(a, q, k, qrow, dq, dn, abandon, lane, lt, n_dtw, n_cells,
                                                            n_emit);
                            __builtin_amdgcn_wave_barrier();
                            dn = 0;
                            thr = read_tau(a, q, k) * a.tau_scale;
                        } else if (!REFILL && dn >= 64) {
                            // widest bands: a batch of 64 as soon as there is one, the rest moves down
                            dtw_batch(64);
                            __builtin_amdgcn_wave_barrier();
                            const int rest = dn - 64;
                            const int moved = lane < rest ? dq[64 + lane] : 0;
                            __builtin_amdgcn_wave_barrier();
                            if (lane < rest) dq[lane] = moved;
                            __builtin_amdgcn_wave_barrier();
                            dn = rest;
                        }
                    } else {
                        // (uniform across the wave)
                        const bool sample = a.pc_x && !a.pc_home && (pc_it & 63) == 0;
                        const bool use_pc = a.pc_x && !sample && (a.pc_home || pc_b > pc_row * pc_n);
                        ++pc_it;
                        float sb = 0.f;  // this group's sampled FP32 bytes (its first lane)
                        if (my < nc && use_pc && gl == 0) ++n_pc;
                        if (my < nc && !(use_pc && precheck16(a, pa + my_wl[my], qrow, gl, pc_qn, pc_nq) > thr)) {
                            const int64_t p2 = pa + my_wl[my];
                            const int32_t id = a.ids_sorted[p2];
                            const float* row = series_row(a, p2, id);
                            int steps = 0;
                            const float d2 = refine16<VEC>(row, qrow, a.len, gl, thr, abandon, steps);
                            if (sample && gl == 0) sb = (float)(min(a.len, steps * 64) * 4);
                            if (gl == 0) {
                                ++n_ref;
                                n_bytes += (unsigned long long)min(a.len, steps * 64) * 4ull;
                                if (d2 <= thr) {
                                    emit(a, q, k, d2, id);
                                    ++n_emit;
                                }
                            }
                        }
                        if (sample) {
                            // the wave's sums over its groups' first lanes (0, 16, 32, 48)
                            sb += __shfl_xor(sb, 16, 64);
                            sb += __shfl_xor(sb, 32, 64);
                            pc_b += __shfl(sb, 0, 64);
                            pc_n += (float)__popcll(__ballot(my < nc && gl == 0));
                        }
                        thr = read_tau(a, q, k) * a.tau_scale;
                    }
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
        if (DTW && dn > 0) {
            if (REFILL) dtw_drain_for<REFILL ? RB : 8, VEC>(a, q, k, qrow, dq, dn, abandon, lane, lt, n_dtw, n_cells, n_emit);
            else dtw_batch(dn);
        }
        atomicAdd(&s_st[ST_SERIES_LB], lane == 0 ? n_lb : 0ull);
        if ((lane & 15) == 0) {
            atomicAdd(&s_st[ST_REFINED], n_ref);
            atomicAdd(&s_st[ST_REFINE_BYTES], n_bytes);
            if (n_pc) atomicAdd(&s_st[ST_PRECHECKED], n_pc);
        }
        if (DTW) {
            atomicAdd(&s_st[ST_CANDS], n_emit);
            atomicAdd(&s_st[ST_DTW], n_dtw);
            atomicAdd(&s_st[ST_DTW_CELLS], n_cells);
        } else if ((lane & 15) == 0) {
            atomicAdd(&s_st[ST_CANDS], n_emit);
        }
    }
    __syncthreads();
    if (threadIdx.x < ST_N && s_st[threadIdx.x])
        atomicAdd(a.stats + (int64_t)q * ST_N + threadIdx.x, s_st[threadIdx.x]);
}

// ---------------------------------------------------------------------------------------------
// Initial bound for the plain scan: the k-th smallest squared distance over
// an evenly spaced sample of series (real distances, so a valid upper bound).
constexpr int kSeedMax = 4096;
__global__ void __launch_bounds__(256) k_seed(QueryArgs a) {
    __shared__ unsigned long long keys[kSeedMax];
    const int q = blockIdx.x;
    const int k = a.kq[q];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int S = (int)min<int64_t>(a.n, (int64_t)min(kSeedMax, max(1024, 32 * k)));
    int P = 1;
    while (P < S) P <<= 1;
    for (int i = S + threadIdx.x; i < P; i += 256) keys[i] = kEmpty;
    const float* qrow = a.Q + (int64_t)q * a.len;
    for (int i = wave; i < S; i += 4) {
        const int64_t id = (int64_t)i * a.n / S;
        const float* row = a.data + id * a.len;
        float acc = 0.f;
        for (int t = lane; t < a.len; t += 64) {
            const float d = qrow[t] - row[t];
            acc = fmaf(d, d, acc);
        }
        acc = sum64(acc);
        if (lane == 0) keys[i] = make_key(acc, (int32_t)id);
    }
    __syncthreads();
    bitonic_sort_u64(keys, P);
    if (threadIdx.x == 0) {
        a.tau0[q] = key_d2(keys[k - 1]);
        float4 qi = a.qinfo[q];
        qi.w = key_d2(keys[k - 1]);
        a.qinfo[q] = qi;
    }
}

// Plain FP32 scan: every (query, series) pair by direct differences.  Block =
// 64 queries x 64 series, thread = 4 x 4 pairs, points staged through LDS in
// chunks of 32; pairs within the slack of the query's bound are emitted.
constexpr int kBT = 64, kBK = 32;
__global__ void __launch_bounds__(256) k_brute_scan(QueryArgs a) {
    __shared__ float Qs[kBK][kBT + 1];
    __shared__ float Xs[kBK][kBT + 1];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int q0 = blockIdx.y * kBT;
    for (int64_t x0 = (int64_t)blockIdx.x * kBT; x0 < a.n; x0 += (int64_t)gridDim.x * kBT) {
    float acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.f;
    for (int t0 = 0; t0 < a.len; t0 += kBK) {
        for (int e = threadIdx.x; e < kBT * kBK; e += 256) {
            const int r = e / kBK, t = e - r * kBK;
            const int qi = q0 + r;
            const int64_t xi = x0 + r;
            Qs[t][r] = (qi < a.mq && t0 + t < a.len) ? a.Q[(int64_t)qi * a.len + t0 + t] : 0.f;
            Xs[t][r] = (xi < a.n && t0 + t < a.len) ? a.data[xi * a.len + t0 + t] : 0.f;
        }
        __syncthreads();
#pragma unroll 8
        for (int t = 0; t < kBK; ++t) {
            float qv[4], xv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) qv[i] = Qs[t][ty + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j) xv[j] = Xs[t][tx + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float d = qv[i] - xv[j];
                    acc[i][j] = fmaf(d, d, acc[i][j]);
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int qi = q0 + ty + 16 * i;
        if (qi >= a.mq || (a.rerun && a.done[qi])) continue;
        const int k = a.kq[qi];
        const float thr = read_tau(a, qi, k) * a.tau_scale;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t xi = x0 + tx + 16 * j;
            if (xi < a.n && acc[i][j] <= thr) emit(a, qi, k, acc[i][j], (int32_t)xi);
        }
    }
    }
}

// ---------------------------------------------------------------------------------------------
// Final answer, one block per query.  The candidate list holds every series
// whose FP32 squared distance came within the slack of the best-so-far at the
// time, hence every true answer.  v_k = the k-th smallest FP32 value in the
// list (radix select on its bits); the window = entries <= v_k * (1 + eps)
// contains every true top-k series.  Window entries are recomputed with
// compensated arithmetic and ordered by (value, id); the first k are written,
// distance = sqrt(hi).  If the list overflowed, the k-th smallest stored value
// tightens tau0 and the query is marked for a re-run with the bound frozen.
// A window of more than kWindowMax entries (many series at one distance) is
// marked wide (status 3, v_k kept in qinfo.y) and finished by k_window_values
// and k_topk_wide, which have no size limit.
constexpr int kWindowMax = 2048;
static_assert(ISAX_MAX_K <= kWindowMax / 2, "the wide merge keeps k entries beside a chunk of kWindowMax / 2");

// k-th smallest (1-based) of the high 32 bits of list[0..cnt), by 8-bit digits.
__device__ unsigned radix_select_hi32(const unsigned long long* list, int cnt, int k, unsigned* hist) {
    __shared__ unsigned s_prefix;
    __shared__ int s_k;
    if (threadIdx.x == 0) {
        s_prefix = 0u;
        s_k = k;
    }
    for (int shift = 24; shift >= 0; shift -= 8) {
        __syncthreads();
        hist[threadIdx.x] = 0u;
        __syncthreads();
        const unsigned prefix = s_prefix;
        for (int i = threadIdx.x; i < cnt; i += 256) {
            const unsigned b = (unsigned)(list[i] >> 32);
            const bool match = shift == 24 || (b >> (shift + 8)) == prefix;
            if (match) atomicAdd(hist + ((b >> shift) & 255u), 1u);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int kk = s_k;
            unsigned d = 0;
            for (; d < 255u; ++d) {
                if ((int)hist[d] >= kk) break;
                kk -= (int)hist[d];
            }
            s_k = kk;
            s_prefix = (prefix << 8) | d;
        }
    }
    __syncthreads();
    return s_prefix;
}

// The recomputed value of a window entry in 8 bytes: the compensated FP32 pair
// (hi, lo) for ED, the FP64 recurrence for DTW.  Order: value, then id.
__device__ inline double window_value(const QueryArgs& a, const float* qrow, int32_t id, int lane) {
    if (a.metric == ISAX_METRIC_DTW) return dtw_exact_wave(qrow, a.data + (int64_t)id * a.len, a.len, a.window, lane);
    const float2 r = dist2_dot2(qrow, a.data + (int64_t)id * a.len, a.len, lane);
    return __builtin_bit_cast(double, r);
}
__device__ inline double window_none(bool dtw) {
    return dtw ? __builtin_huge_val() : __builtin_bit_cast(double, make_float2(kInf, kInf));
}
__device__ inline bool window_in(double v, bool dtw) {
    return dtw ? v < __builtin_huge_val() : __builtin_bit_cast(float2, v).x < kInf;
}
__device__ inline bool window_gt(double x, double y, unsigned ix, unsigned iy, bool dtw) {
    if (dtw) return x > y || (x == y && ix > iy);
    const float2 u = __builtin_bit_cast(float2, x), v = __builtin_bit_cast(float2, y);
    return u.x > v.x || (u.x == v.x && (u.y > v.y || (u.y == v.y && ix > iy)));
}

// Bitonic sort of PW (power of two) window entries in LDS by (value, id).
__device__ void sort_window(unsigned long long* wkeys, double* wv, int PW, bool dtw) {
    for (int size = 2; size <= PW; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            __syncthreads();
            for (int i = threadIdx.x; i < PW / 2; i += blockDim.x) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const double x = wv[lo], y = wv[hi];
                const unsigned ix = (unsigned)(wkeys[lo] & 0xffffffffu), iy = (unsigned)(wkeys[hi] & 0xffffffffu);
                if (window_gt(x, y, ix, iy, dtw) == up) {
                    wv[lo] = y;
                    wv[hi] = x;
                    const unsigned long long t = wkeys[lo];
                    wkeys[lo] = wkeys[hi];
                    wkeys[hi] = t;
                }
            }
        }
    __syncthreads();
}

// Writes the first k sorted window entries as the query's answer row.
__device__ void write_answer(const QueryArgs& a, int q, int k, const unsigned long long* wkeys, const double* wv,
                             float vk) {
    const bool dtw = a.metric == ISAX_METRIC_DTW;
    for (int i = threadIdx.x; i < a.kmax; i += blockDim.x) {
        const int64_t o = (int64_t)q * a.kmax + i;
        if (i < k) {
            a.out_ids[o] = (int64_t)key_id(wkeys[i]);
            a.out_dists[o] = dtw ? (float)sqrt(wv[i]) : sqrtf(fmaxf(__builtin_bit_cast(float2, wv[i]).x, 0.f));
        } else {
            a.out_ids[o] = -1;
            a.out_dists[o] = kInf;
        }
    }
    if (threadIdx.x == 0) {
        a.done[q] = 1;
        a.status[q] = 0;
        float4 qi = a.qinfo[q];
        qi.y = vk;  // from here on: FP32 k-th squared distance
        a.qinfo[q] = qi;
    }
}

__global__ void __launch_bounds__(256) k_topk(QueryArgs a) {
    __shared__ unsigned long long wkeys[kWindowMax];
    __shared__ double wv[kWindowMax];
    __shared__ unsigned hist[256];
    __shared__ int s_W;
    const int q = blockIdx.x;
    if (a.done[q]) return;
    const int k = a.kq[q];
    const unsigned cnt_all = a.cand_count[q];
    const int cnt = (int)min<unsigned>(cnt_all, (unsigned)a.cap);
    const unsigned long long* list = a.cand + (int64_t)q * a.cap;
    if (cnt < k) {  // cannot happen for k <= n unless candidates were lost
        if (threadIdx.x == 0) a.status[q] = cnt_all > (unsigned)a.cap ? 1 : 2;
        return;
    }
    const float vk = __uint_as_float(radix_select_hi32(list, cnt, k, hist));
    if (cnt_all > (unsigned)a.cap) {
        if (threadIdx.x == 0) {
            a.tau0[q] = fminf(a.tau0[q], vk);
            a.status[q] = 1;
        }
        return;
    }
    const float thr = vk * a.tau_scale;
    if (threadIdx.x == 0) s_W = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < cnt; i += 256) {
        const unsigned long long key = list[i];
        if (key_d2(key) <= thr) {
            const int slot = atomicAdd(&s_W, 1);
            if (slot < kWindowMax) wkeys[slot] = key;
        }
    }
    __syncthreads();
    const int W = s_W;
    if (W > kWindowMax) {
        if (threadIdx.x == 0) {
            float4 qi = a.qinfo[q];
            qi.y = vk;
            a.qinfo[q] = qi;
            a.status[q] = 3;
        }
        return;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const float* qrow = a.Q + (int64_t)q * a.len;
    const bool dtw = a.metric == ISAX_METRIC_DTW;
    for (int i = wave; i < W; i += 4) {
        const double v = window_value(a, qrow, key_id(wkeys[i]), lane);
        if (lane == 0) wv[i] = v;
    }
    int PW = 1;
    while (PW < W) PW <<= 1;
    for (int i = W + threadIdx.x; i < PW; i += 256) {
        wkeys[i] = kEmpty;
        wv[i] = window_none(dtw);
    }
    sort_window(wkeys, wv, PW, dtw);
    write_answer(a, q, k, wkeys, wv, vk);
}

// Wide windows (status 3): the recomputed value of every candidate of query
// wq[y] within the window, +inf for the others, into vals[y][cap]; one wave
// per entry, many blocks per query.
__global__ void __launch_bounds__(256) k_window_values(QueryArgs a, const int* __restrict__ wq,
                                                       double* __restrict__ vals) {
    const int q = wq[blockIdx.y];
    const int cnt = (int)min<unsigned>(a.cand_count[q], (unsigned)a.cap);
    const float thr = a.qinfo[q].y * a.tau_scale;
    const unsigned long long* list = a.cand + (int64_t)q * a.cap;
    double* out = vals + (int64_t)blockIdx.y * a.cap;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const float* qrow = a.Q + (int64_t)q * a.len;
    const bool dtw = a.metric == ISAX_METRIC_DTW;
    for (int i = blockIdx.x * 4 + wave; i < cnt; i += gridDim.x * 4) {
        const unsigned long long key = list[i];
        const double v = key_d2(key) <= thr ? window_value(a, qrow, key_id(key), lane) : window_none(dtw);
        if (lane == 0) out[i] = v;
    }
}

// Wide windows: the k smallest (value, id) of the window, merged chunk by
// chunk: the best k so far plus up to kWindowMax / 2 new entries are sorted in
// LDS and the first k kept (k <= ISAX_MAX_K = kWindowMax / 2).
__global__ void __launch_bounds__(256) k_topk_wide(QueryArgs a, const int* __restrict__ wq,
                                                   const double* __restrict__ vals) {
    __shared__ unsigned long long wkeys[kWindowMax];
    __shared__ double wv[kWindowMax];
    __shared__ int s_n;
    constexpr int kChunk = kWindowMax / 2;
    const int q = wq[blockIdx.x];
    const int k = a.kq[q];
    const int cnt = (int)min<unsigned>(a.cand_count[q], (unsigned)a.cap);
    const unsigned long long* list = a.cand + (int64_t)q * a.cap;
    const double* v = vals + (int64_t)blockIdx.x * a.cap;
    const bool dtw = a.metric == ISAX_METRIC_DTW;
    int kept = 0;
    for (int c0 = 0; c0 < cnt; c0 += kChunk) {
        __syncthreads();
        if (threadIdx.x == 0) s_n = kept;
        __syncthreads();
        for (int i = c0 + threadIdx.x; i < min(cnt, c0 + kChunk); i += 256) {
            const double x = v[i];
            if (window_in(x, dtw)) {
                const int slot = atomicAdd(&s_n, 1);
                wkeys[slot] = list[i];
                wv[slot] = x;
            }
        }
        __syncthreads();
        const int W = s_n;
        int PW = 1;
        while (PW < W) PW <<= 1;
        for (int i = W + threadIdx.x; i < PW; i += 256) {
            wkeys[i] = kEmpty;
            wv[i] = window_none(dtw);
        }
        sort_window(wkeys, wv, PW, dtw);
        kept = min(k, W);
    }
    write_answer(a, q, k, wkeys, wv, a.qinfo[q].y);
}

// Sub-batch of a hybrid batch: query rows and k by position in the batch, and
// the answers written back to those positions.
__global__ void k_gather_queries(const float* __restrict__ Q, const int32_t* __restrict__ kq,
                                 const int32_t* __restrict__ pos, int len, float* __restrict__ Qf,
                                 int32_t* __restrict__ kqf) {
    const int i = blockIdx.x;
    const int64_t src = pos[i];
    for (int t = threadIdx.x; t < len; t += blockDim.x) Qf[(int64_t)i * len + t] = Q[src * len + t];
    if (threadIdx.x == 0) kqf[i] = kq[src];
}

__global__ void k_scatter_answers(const int64_t* __restrict__ ids, const float* __restrict__ dists,
                                  const int32_t* __restrict__ pos, int kmax, int64_t* __restrict__ out_ids,
                                  float* __restrict__ out_dists) {
    const int i = blockIdx.x;
    const int64_t dst = pos[i];
    for (int t = threadIdx.x; t < kmax; t += blockDim.x) {
        out_ids[dst * kmax + t] = ids[(int64_t)i * kmax + t];
        out_dists[dst * kmax + t] = dists[(int64_t)i * kmax + t];
    }
}

// Before a re-run: empty the candidate lists of the unfinished queries.
__global__ void k_rerun_reset(QueryArgs a) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < a.mq && !a.done[q]) {
        a.cand_count[q] = 0u;
        a.status[q] = 0;
    }
}

// Squared lower bound of every (query, series) pair, column = original id.
__global__ void __launch_bounds__(256) k_lower_bounds(QueryArgs a, float* __restrict__ out) {
    const int q = blockIdx.y;
    const float* Ts = a.T + (int64_t)q * a.w * a.ns;
    for (int64_t pos = (int64_t)blockIdx.x * 256 + threadIdx.x; pos < a.n; pos += (int64_t)gridDim.x * 256) {
        const uint8_t* wd = a.words_sorted + pos * a.ws;
        float lb = 0.f;
        for (int j = 0; j < a.w; ++j) lb += Ts[j * a.ns + wd[j]];
        out[(int64_t)q * a.n + a.ids_sorted[pos]] = lb * a.lb_scale;
    }
}

}  // namespace

// =============================================================================================
void launch_check_finite(const float* x, int64_t count, int* flag, hipStream_t s) {
    if (count <= 0) return;
    ProfScope ps("check_finite", s);
    const int64_t blocks = std::min<int64_t>((count + 255) / 256, 4096);
    k_check_finite<<<(int)blocks, 256, 0, s>>>(x, count, flag);
    ISAX_HIP(hipGetLastError());
}

void launch_qprep(const QueryArgs& a, hipStream_t s) {
    ProfScope ps("qprep", s);
    const size_t lds = a.metric == ISAX_METRIC_DTW ? (size_t)a.len * 2 * sizeof(float) : 0;
    k_qprep<<<a.mq, 64, lds, s>>>(a);
    ISAX_HIP(hipGetLastError());
}

// Band cells held in registers for a DTW band of half-width r.
int dtw_band_regs(int r) {
    const int B = 2 * r + 1;
    return B <= 8 ? 8 : B <= 16 ? 16 : B <= 32 ? 32 : B <= 40 ? 40 : B <= 48 ? 48 : B <= 56 ? 56 : 64;
}

void launch_homeleaf(const QueryArgs& a, hipStream_t s) {
    ProfScope ps("homeleaf", s);
    const size_t lds = kHomeMax * sizeof(unsigned long long) + (size_t)(a.len + 2 * kDtwPad) * 4 +
                       (a.pc_x && a.pc_home ? kHomeMax * sizeof(float) : 0);
    if (a.metric != ISAX_METRIC_DTW) {
        k_homeleaf<0><<<a.mq, 256, lds, s>>>(a);
    } else {
        switch (dtw_band_regs(a.window)) {
            case 8: k_homeleaf<8><<<a.mq, 256, lds, s>>>(a); break;
            case 16: k_homeleaf<16><<<a.mq, 256, lds, s>>>(a); break;
            case 32: k_homeleaf<32><<<a.mq, 256, lds, s>>>(a); break;
            case 40: k_homeleaf<40><<<a.mq, 256, lds, s>>>(a); break;
            case 48: k_homeleaf<48><<<a.mq, 256, lds, s>>>(a); break;
            case 56: k_homeleaf<56><<<a.mq, 256, lds, s>>>(a); break;
            default: k_homeleaf<64><<<a.mq, 256, lds, s>>>(a); break;
        }
    }
    ISAX_HIP(hipGetLastError());
}

void launch_gather_queries(const float* Q, const int32_t* kq, const int32_t* pos, int mf, int len, float* Qf,
                           int32_t* kqf, hipStream_t s) {
    if (mf <= 0) return;
    k_gather_queries<<<mf, 256, 0, s>>>(Q, kq, pos, len, Qf, kqf);
    ISAX_HIP(hipGetLastError());
}

void launch_scatter_answers(const int64_t* ids, const float* dists, const int32_t* pos, int mf, int kmax,
                            int64_t* out_ids, float* out_dists, hipStream_t s) {
    if (mf <= 0) return;
    k_scatter_answers<<<mf, 256, 0, s>>>(ids, dists, pos, kmax, out_ids, out_dists);
    ISAX_HIP(hipGetLastError());
}

void launch_list_recount(const QueryArgs& a, int64_t grid_x, hipStream_t s) {
    ProfScope ps("list_recount", s);
    ISAX_HIP(hipMemsetAsync(a.list_rest, 0, (size_t)a.mq * sizeof(unsigned), s));
    const dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>(grid_x, 64)), (unsigned)a.mq);
    k_list_recount<<<grid, 256, 0, s>>>(a);
    ISAX_HIP(hipGetLastError());
}

__global__ void k_carry_bound(QueryArgs src, QueryArgs dst, const int2* __restrict__ map, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int s = map[i].x, d = map[i].y;
    dst.tau0[d] = fminf(dst.tau0[d], read_tau(src, s, src.kq[s]));
}

void launch_carry_bound(const QueryArgs& src, const QueryArgs& dst, const int2* map, int n, hipStream_t s) {
    if (n <= 0) return;
    k_carry_bound<<<(n + 255) / 256, 256, 0, s>>>(src, dst, map, n);
    ISAX_HIP(hipGetLastError());
}

void launch_leaf_order(const QueryArgs& a, hipStream_t s) {
    ProfScope ps("leaf_order", s);
    ISAX_HIP(hipMemsetAsync(a.leaf_hist, 0, (size_t)a.mq * kLeafBins * sizeof(unsigned), s));
    ISAX_HIP(hipMemsetAsync(a.leaf_count, 0, (size_t)a.mq * sizeof(unsigned), s));
    const int64_t per_block = 256 * kHistLeafRounds * std::max(1, a.leaf_stride);
    const int nq = a.qsel ? a.nsel : a.mq;
    if (nq > 0) {
        const dim3 grid((unsigned)((a.n_leaves + per_block - 1) / per_block), (unsigned)((nq + kHistQueries - 1) / kHistQueries));
        if (a.w == 16 && a.ws == 16) k_leaf_hist<true><<<grid, 256, 0, s>>>(a);
        else k_leaf_hist<false><<<grid, 256, 0, s>>>(a);
    }
    k_leaf_theta<<<(a.mq + 255) / 256, 256, 0, s>>>(a);
    ISAX_HIP(hipGetLastError());
}

template <bool VEC, bool TL>
void launch_index_scan_t(const QueryArgs& a, const dim3& grid, hipStream_t s) {
    if (a.metric != ISAX_METRIC_DTW) {
        const ScanSmem L = scan_smem(a.ns, a.w, a.len, false, TL);
        k_index_scan<VEC, TL, 0><<<grid, 256, L.total, s>>>(a);
        return;
    }
    const ScanSmem L = scan_smem(a.ns, a.w, a.len, true, TL);
    switch (dtw_band_regs(a.window)) {
        case 8: k_index_scan<VEC, TL, 8><<<grid, 256, L.total, s>>>(a); break;
        case 16: k_index_scan<VEC, TL, 16><<<grid, 256, L.total, s>>>(a); break;
        case 32: k_index_scan<VEC, TL, 32><<<grid, 256, L.total, s>>>(a); break;
        case 40: k_index_scan<VEC, TL, 40><<<grid, 256, L.total, s>>>(a); break;
        case 48: k_index_scan<VEC, TL, 48><<<grid, 256, L.total, s>>>(a); break;
        case 56: k_index_scan<VEC, TL, 56><<<grid, 256, L.total, s>>>(a); break;
        default: k_index_scan<VEC, TL, 64><<<grid, 256, L.total, s>>>(a); break;
    }
}

void launch_index_scan(const QueryArgs& a, hipStream_t s) {
    ProfScope ps(a.metric == ISAX_METRIC_DTW ? "dtw_scan" : "index_scan", s);
    const bool dtw = a.metric == ISAX_METRIC_DTW;
    const int64_t gx = a.round != 0 && a.grid_leaves > 0 ? a.grid_leaves : (a.n_leaves + 255) / 256;
    const dim3 grid((unsigned)gx, (unsigned)a.mq);
    const bool vec = a.len % 4 == 0 && (reinterpret_cast<uintptr_t>(a.data) & 15) == 0;
    const bool tl = a.w * a.ns * 4 <= kTableLdsMax && scan_smem(a.ns, a.w, a.len, dtw, true).total <= 64 * 1024;
    ISAX_REQUIRE(scan_smem(a.ns, a.w, a.len, dtw, tl).total <= 64 * 1024, "series too long for the scan's LDS plan");
    if (vec && tl) launch_index_scan_t<true, true>(a, grid, s);
    else if (vec) launch_index_scan_t<true, false>(a, grid, s);
    else if (tl) launch_index_scan_t<false, true>(a, grid, s);
    else launch_index_scan_t<false, false>(a, grid, s);
    ISAX_HIP(hipGetLastError());
}

void launch_seed(const QueryArgs& a, hipStream_t s) {
    ProfScope ps("seed", s);
    k_seed<<<a.mq, 256, 0, s>>>(a);
    ISAX_HIP(hipGetLastError());
}

void launch_brute_scan(const QueryArgs& a, hipStream_t s) {
    ProfScope ps("brute_scan", s);
    const dim3 grid(grid_blocks(a.n, kBT, 1 << 15), (unsigned)((a.mq + kBT - 1) / kBT));
    k_brute_scan<<<grid, 256, 0, s>>>(a);
    ISAX_HIP(hipGetLastError());
}

void launch_topk(const QueryArgs& a, hipStream_t s) {
    ProfScope ps("topk", s);
    k_topk<<<a.mq, 256, 0, s>>>(a);
    ISAX_HIP(hipGetLastError());
}

void launch_topk_wide(const QueryArgs& a, const int* wq, int n_wide, double* vals, hipStream_t s) {
    if (n_wide <= 0) return;
    ProfScope ps("topk_wide", s);
    const dim3 grid(grid_blocks(a.cap, 4, 1024), (unsigned)n_wide);
    k_window_values<<<grid, 256, 0, s>>>(a, wq, vals);
    k_topk_wide<<<n_wide, 256, 0, s>>>(a, wq, vals);
    ISAX_HIP(hipGetLastError());
}

void launch_rerun_reset(const QueryArgs& a, hipStream_t s) {
    k_rerun_reset<<<(a.mq + 255) / 256, 256, 0, s>>>(a);
    ISAX_HIP(hipGetLastError());
}

void launch_lower_bounds(const QueryArgs& a, float* out, hipStream_t s) {
    const dim3 grid(grid_blocks(a.n, 256, 4096), (unsigned)a.mq);
    k_lower_bounds<<<grid, 256, 0, s>>>(a, out);
    ISAX_HIP(hipGetLastError());
}

}  // namespace isax
