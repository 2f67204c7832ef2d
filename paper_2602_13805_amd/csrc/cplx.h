// Complex arithmetic on interleaved (re, im) pairs, host and device.
#pragma once

#include <hip/hip_runtime.h>

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T x, y;
};

template <typename T>
__host__ __device__ __forceinline__ cx<T> mk(T a, T b) { return cx<T>{a, b}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.x, s * a.y}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.x, -a.y}; }
template <typename T>
__host__ __device__ __forceinline__ T norm2(cx<T> a) { return a.x * a.x + a.y * a.y; }
// a * conj(b)
template <typename T>
__host__ __device__ __forceinline__ cx<T> mulc(cx<T> a, cx<T> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
// conj(a) * b
template <typename T>
__host__ __device__ __forceinline__ cx<T> cmul_conj_a(cx<T> a, cx<T> b) {
  return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> cdiv(cx<T> a, cx<T> b) {
  T d = b.x * b.x + b.y * b.y;
  return {(a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d};
}

// Workgroups are dispatched to the 8 XCDs round-robin (workgroup x to XCD
// x mod 8), and each XCD has its own L2.  This maps the hardware order x of an
// n-workgroup grid to a logical order in which every XCD takes one contiguous
// range of logical workgroups (a bijection of [0, n)), so that neighbouring
// logical workgroups, which share inputs, share an L2.
__device__ __forceinline__ int xcd_remap(int x, int n) {
  constexpr int X = 8;
  const int q = n / X, r = n % X, c = x % X, slot = x / X;
  return c * q + (c < r ? c : r) + slot;
}

// Grouped launches: one launch serves several argument sets, set g taking the
// workgroups [start[g], start[g+1]).  Returns g for workgroup bx (the search
// is uniform over the workgroup).
__device__ __forceinline__ int group_of(const int* start, int n, int bx) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= bx)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}
