// SELL-64 rows on the device: slices of 64 rows (one wavefront), each stored
// column-major with the slice's longest row, so lane l of a wavefront reads
// entry k of row 64 s + l at sptr[s] + 64 k + l (unit stride across lanes).
// Column ids are either absolute (col, 32-bit) or, when every stored entry
// lies within 32767 of offset_base(row), 16-bit offsets from it (d16): 6
// instead of 8 bytes per FP32 entry, 10 instead of 12 per FP64 entry.
// Padding entries carry value 0 and an in-range column.
#pragma once

#include <hip/hip_runtime.h>

#include "eqs_internal.h"

namespace eqs {

template <typename T>
struct SellView {
    const int32_t* __restrict__ sptr;
    const int32_t* __restrict__ col;
    const int16_t* __restrict__ d16;
    const T* __restrict__ val;
    int32_t n_rows, n_slices, n_cols;
};

template <typename T>
static inline SellView<T> view(const Sell<T>& A) {
    return SellView<T>{A.sptr, A.col, A.d16, A.val, A.n_rows, A.n_slices, A.n_cols};
}

// sum_k a_{row,k} f(col_k) over the stored entries of `row` (rows past n_rows
// but inside the last slice see padding only). Entries are taken in groups of
// 8 whose loads carry no branch: positions past the row's width re-read its
// last entry (a cache hit) and their terms are dropped by a select, so all
// loads and gathers of a group are in flight together. The sum runs in k order.
template <typename T, typename F>
__device__ __forceinline__ T sell_accum(const SellView<T>& A, int32_t row, F f) {
    const int32_t s = row >> 6, l = row & 63;
    const int32_t beg = A.sptr[s];
    const int32_t w = (A.sptr[s + 1] - beg) >> 6;  // uniform across the wavefront
    const T* vp = A.val + beg + l;
    T acc = T(0);
    for (int32_t k0 = 0; k0 < w; k0 += 8) {
        T v[8];
        int32_t j[8];
        if (A.d16) {
            const int16_t* dp = A.d16 + beg + l;
            const int32_t base = offset_base(row, A.n_rows, A.n_cols);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t kk = (int64_t)min(k0 + u, w - 1) * 64;
                v[u] = vp[kk];
                j[u] = base + (int32_t)dp[kk];
            }
        } else {
            const int32_t* cp = A.col + beg + l;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t kk = (int64_t)min(k0 + u, w - 1) * 64;
                v[u] = vp[kk];
                j[u] = cp[kk];
            }
        }
        T t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = v[u] * f(j[u]);
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += (k0 + u < w) ? t[u] : T(0);
    }
    return acc;
}

template <typename T, typename TX>
__device__ __forceinline__ T sell_row(const SellView<T>& A, int32_t row, const TX* __restrict__ x) {
    return sell_accum(A, row, [&](int32_t j) { return (T)x[j]; });
}

}  // namespace eqs
