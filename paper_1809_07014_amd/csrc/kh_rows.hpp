// Device helpers over exported rows (keys of W words, most significant
// first, the k-mer right-aligned in 2k bits, rows in ascending key order):
// one-base shifts of a k-mer and binary search over sorted rows.  Used by
// the traversal, merge and pruning kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kh {

// S[1..k) + b, in the export layout (W words, most significant first, the
// k-mer right-aligned in 2k bits; `top` bits live in word 0).
template <int W>
__device__ __forceinline__ void push_right(const uint64_t (&s)[W], int b, int top,
                                           uint64_t (&t)[W]) {
#pragma unroll
  for (int j = 0; j < W - 1; ++j) t[j] = (s[j] << 2) | (s[j + 1] >> 62);
  t[W - 1] = (s[W - 1] << 2) | (uint64_t)b;
  if (top < 64) t[0] &= (1ull << top) - 1;
}

// b + S[0..k-1).
template <int W>
__device__ __forceinline__ void push_left(const uint64_t (&s)[W], int b, int top,
                                          uint64_t (&t)[W]) {
#pragma unroll
  for (int j = W - 1; j > 0; --j) t[j] = (s[j] >> 2) | (s[j - 1] << 62);
  t[0] = (s[0] >> 2) | ((uint64_t)b << (top - 2));
}

template <int W>
__device__ __forceinline__ int cmp_rows(const uint64_t* a, const uint64_t* b) {
#pragma unroll
  for (int j = 0; j < W; ++j)
    if (a[j] != b[j]) return a[j] < b[j] ? -1 : 1;
  return 0;
}

// First row of keys[0..n) not less than q.
template <int W>
__device__ __forceinline__ int64_t lower_bound_rows(const uint64_t* keys, int64_t n,
                                                    const uint64_t* q) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (cmp_rows<W>(keys + mid * W, q) < 0)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

}  // namespace kh
