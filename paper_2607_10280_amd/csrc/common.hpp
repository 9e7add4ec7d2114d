// Shared device/host helpers of the anomps HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace anomps {

constexpr int kMaxBond = 16;     // largest slot dimension S compiled in
constexpr int kMaxSites = 1024;

// Bond dimension between sites `bond` and `bond`+1 after `layers` layers of the CNOT-ladder
// circuit when every two-site split keeps min(chi, rows, cols) singular values:
//   D = min(chi, 2^layers, 2^(bond+1), 2^(n-bond-1));  bonds -1 and n-1 are the dummy ends (1).
__host__ __device__ inline int bond_dim(int n, int chi, int layers, int bond) {
  if (bond < 0 || bond >= n - 1) return 1;
  long long d = chi;
  auto cap = [&](int e) {
    if (e < 30) d = d < (1LL << e) ? d : (1LL << e);
  };
  cap(layers);
  cap(bond + 1);
  cap(n - bond - 1);
  return static_cast<int>(d < 1 ? 1 : d);
}

__host__ __device__ inline int slot_dim(int n, int chi, int layers) {
  int s = 1;
  for (int k = 0; k < n - 1; ++k) {
    int d = bond_dim(n, chi, layers, k);
    s = d > s ? d : s;
  }
  return s;
}

// Wave-uniform copies (SGPRs) of values every lane loaded from the same address, so that the
// control flow they steer compiles to scalar branches.
__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }
template <typename P>
__device__ __forceinline__ P* uniform_ptr(P* p) {
  const unsigned long long v = (unsigned long long)p;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return (P*)(((unsigned long long)hi << 32) | lo);
}

// Minimal complex arithmetic on (re, im) pairs.
template <typename R>
struct cx {
  R re, im;
};
using cd = cx<double>;

template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// conj(a) * b
template <typename R>
__device__ __forceinline__ cx<R> cmulc(cx<R> a, cx<R> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// acc += a * b
template <typename R>
__device__ __forceinline__ void cfma(cx<R>& acc, cx<R> a, cx<R> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}
// acc += conj(a) * b
template <typename R>
__device__ __forceinline__ void cfmac(cx<R>& acc, cx<R> a, cx<R> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(-a.im, b.re, acc.im);
}
template <typename R>
__device__ __forceinline__ cx<R> cconj(cx<R> a) {
  return {a.re, -a.im};
}
template <typename R>
__device__ __forceinline__ cx<R> cscale(cx<R> a, R s) {
  return {a.re * s, a.im * s};
}
template <typename R>
__device__ __forceinline__ cx<R> cadd(cx<R> a, cx<R> b) {
  return {a.re + b.re, a.im + b.im};
}

// Global (storage type T) <-> compute type conversion of one complex element.
template <typename T, typename R>
__device__ __forceinline__ cx<R> load_c(const T* p, size_t idx) {
  return {static_cast<R>(p[2 * idx]), static_cast<R>(p[2 * idx + 1])};
}
template <typename T, typename R>
__device__ __forceinline__ void store_c(T* p, size_t idx, cx<R> v) {
  p[2 * idx] = static_cast<T>(v.re);
  p[2 * idx + 1] = static_cast<T>(v.im);
}

// Per-image status flags (mirror of the public enum).
constexpr int kImgNonfinite = 1;
constexpr int kImgNoConvergence = 2;

}  // namespace anomps
