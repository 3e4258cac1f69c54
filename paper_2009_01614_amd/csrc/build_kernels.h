// Host launchers of the index-build kernels (build_kernels.hip).
#pragma once
#include "internal.h"

namespace isax {
void launch_summarise(const float* data, int64_t n, int len, int w, int out_stride, const float* beta, int c,
                      uint8_t* words, unsigned* maxabs, int* nonfinite, hipStream_t s);
void launch_make_keys(const uint8_t* words, int64_t n, int ws, int w, int c, int key_bits, uint64_t* keys,
                      int32_t* ids, hipStream_t s);
void sort_keys(uint64_t* keys, int32_t* ids, int64_t n, int key_bits, hipStream_t s);
void launch_gather_rows(const float* data, const int32_t* ids, int64_t n, int len, float* out, hipStream_t s);
void launch_gather_words(const uint8_t* words, const int32_t* ids, int64_t n, int ws, uint8_t* out, hipStream_t s);
// Leaf keys and envelopes, and the envelopes of nodes of kNodeLeaves leaves.
void launch_leaf_layout(const uint64_t* keys_sorted, const uint8_t* words_sorted, int64_t n, int ws, int leaf,
                        int64_t n_leaves, uint64_t* leaf_key, uint8_t* lo, uint8_t* hi, uint8_t* node_lo,
                        uint8_t* node_hi, hipStream_t s);
// kind 0: BF16 copy into xb; kind 1: FP8 E4M3 copy into xf; row p (len_pad wide, zero-padded)
// holds series ids[p].
// meta[p] = {|x|^2, |e_x|, |x~|, scale}.
void launch_quantise(const float* data, const int32_t* ids, int64_t n, int len, int len_pad, int kind, uint16_t* xb,
                     uint8_t* xf, float4* meta, hipStream_t s);
// Spectral copy (D coefficients per series, row p = series ids[p]) from the
// transform tt [len][D] (FP64, column D - 1 zero); meta[p] = {|x|^2, |e|, |x~|, 1}.
void launch_spectral(const float* data, const int32_t* ids, int64_t n, int len, int D, const double* tt, uint16_t* xs,
                     float4* meta, hipStream_t s);
// FP32 PAA (the summarise kernels' order) of every segment of n_series evenly
// spaced series into out [n_series][w].
void launch_paa_sample(const float* data, int64_t n, int len, int w, int n_series, float* out, hipStream_t s);
}  // namespace isax
