// SELL rows on the device: slices of one wavefront (64 lanes) each, stored
// column-major with the slice's longest row, so lane l of a wavefront reads
// its entry k at sptr[s] + 64 k + l (unit stride across lanes). With L lanes
// per row a slice holds 64 / L rows: lane l serves row 64 s / L + l / L and
// takes the row's entries l % L, l % L + L, ... (long rows of coarse AMG
// operators then need 1/L as many sequential loads); the L partial sums are
// combined by cross-lane shuffles.
// Column ids are either absolute (col, 32-bit) or, when every stored entry
// lies within 32767 of offset_base(row), 16-bit offsets from it (d16): 6
// instead of 8 bytes per FP32 entry, 10 instead of 12 per FP64 entry.
// Padding entries carry value 0 and an in-range column.
#pragma once

#include <hip/hip_runtime.h>

#include "eqs_internal.h"

namespace eqs {

// Sum over the L lanes of an aligned lane group (result in every lane).
template <int L, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, L);
    return v;
}

// Row blocks of the sparse kernels. The hardware deals the workgroups of a
// launch to its 8 XCDs round-robin (workgroup i to XCD i mod 8). In the XCD
// order (an operator's `xcd` flag) workgroup i takes row block
// xcd_block(i, nb), so each XCD walks one contiguous range of row blocks and
// the vector entries its rows gather meet in that XCD's L2 instead of being
// fetched by several L2s. On the 2.1M-DOF workload this cut the counted
// traffic of the finest level's kernels (CG SpMV 267 -> 232 MB per launch,
// pre-smoother 168 -> 133 MB, post-smoother 177 -> 158 MB) and their times
// (post-smoother 26.7 -> 25.1 us), while the transfer products between the
// finest two levels and the level-1 smoother became slower (the restriction
// 22.9 -> 24.3 us), so M and the finest level's operator take the XCD order
// and the others the natural one. Partial sums are indexed by row block
// either way.
__device__ __forceinline__ int64_t xcd_block(int64_t i, int64_t nb) {
    const int64_t q = nb >> 3, r = nb & 7, x = i & 7;
    return x * q + (x < r ? x : r) + (i >> 3);
}
__device__ __forceinline__ int64_t row_block(int32_t xcd) {
    return xcd ? xcd_block(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
}

// The row served by global thread g of a SELL kernel with L lanes per row.
template <int L>
__device__ __forceinline__ int32_t sell_row_of(int64_t g) {
    return (int32_t)((g >> 6) * (64 / L) + ((g & 63) / L));
}

template <typename T>
struct SellView {
    const int32_t* __restrict__ sptr;
    const int32_t* __restrict__ col;
    const int16_t* __restrict__ d16;
    const T* __restrict__ val;
    int32_t n_rows, n_slices, n_cols;
    const uint8_t* __restrict__ perm;  // row order within each 256-thread window, or NULL (see sell_perm_row)
    int32_t xcd;                       // block order of its products (see row_block)
};

template <typename T>
static inline SellView<T> view(const Sell<T>& A) {
    return SellView<T>{A.sptr, A.col, A.d16, A.val, A.n_rows, A.n_slices, A.n_cols, A.perm, A.xcd};
}

// With a row order (perm), the rows served by one 256-thread window (4
// slices, 256 / L rows) are stored longest first, so the slices of the window
// pad less; position k of the window serves row window_base + perm[k]. The
// kernels that use it write only rows of their own window (products y = A x,
// the CG SpMV and residual, the finest smoothers), so the rows of a workgroup,
// and with them its partial sums, are the same with and without it.
template <int L>
__device__ __forceinline__ int32_t sell_perm_row(const uint8_t* __restrict__ perm, int64_t g) {
    const int32_t pos = sell_row_of<L>(g);
    if (!perm) return pos;
    const int32_t base = (int32_t)((g >> 8) * (256 / L));
    return base + (int32_t)perm[pos];
}

// sum_k a_{row,k} f(col_k) over the stored entries of `row` served by global
// thread g (rows past n_rows but inside the last slice see padding only).
// Entries are taken in groups of U whose loads carry no branch: positions
// past the slice's width re-read its last entry (a cache hit) and their terms
// are dropped by a select, so all loads and gathers of a group are in flight
// together (a row of w stored entries costs ceil(w / U) dependent rounds of
// loads, then gathers; short rows want a small U, long ones a large U). The
// operator's values and column data are read once per product and carry the
// nontemporal hint, which leaves the caches to the gathered vector. Each lane
// sums in k order; with L > 1 the lane sums are then combined by group_sum
// (every lane of the group gets the row's sum).
template <int L, int U = 8, typename T, typename F>
__device__ __forceinline__ T sell_accum(const SellView<T>& A, int64_t g, int32_t row, F f) {
    const int32_t s = (int32_t)(g >> 6), l = (int32_t)(g & 63);
    const int32_t beg = A.sptr[s];
    const int32_t w = (A.sptr[s + 1] - beg) >> 6;  // uniform across the wavefront
    const T* vp = A.val + beg + l;
    T acc = T(0);
    for (int32_t k0 = 0; k0 < w; k0 += U) {
        T v[U];
        int32_t j[U];
        if (A.d16) {
            const int16_t* dp = A.d16 + beg + l;
            const int32_t base = offset_base(row, A.n_rows, A.n_cols);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t kk = (int64_t)min(k0 + u, w - 1) * 64;
                v[u] = __builtin_nontemporal_load(vp + kk);
                j[u] = base + (int32_t)__builtin_nontemporal_load(dp + kk);
            }
        } else {
            const int32_t* cp = A.col + beg + l;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t kk = (int64_t)min(k0 + u, w - 1) * 64;
                v[u] = __builtin_nontemporal_load(vp + kk);
                j[u] = __builtin_nontemporal_load(cp + kk);
            }
        }
        T t[U];
#pragma unroll
        for (int u = 0; u < U; ++u) t[u] = v[u] * f(j[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) acc += (k0 + u < w) ? t[u] : T(0);
    }
    return group_sum<L>(acc);
}

template <int L, int U = 8, typename T, typename TX>
__device__ __forceinline__ T sell_row(const SellView<T>& A, int64_t g, int32_t row, const TX* __restrict__ x) {
    return sell_accum<L, U>(A, g, row, [&](int32_t j) { return (T)x[j]; });
}

// One lane per row (thread index = row).
template <typename T, typename TX>
__device__ __forceinline__ T sell_row(const SellView<T>& A, int32_t row, const TX* __restrict__ x) {
    return sell_row<1>(A, row, row, x);
}

}  // namespace eqs
