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

// Cross-lane move of an FP64 value inside a DPP row (CTRL = row_mirror, row_half_mirror or a
// quad permutation, which always read a lane of the same row): two 32-bit moves that write every
// lane, so no old value has to be set up first.
template <int CTRL>
__device__ __forceinline__ double dpp_mov_d(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

// One-sided (Hestenes) Jacobi rotation of a column pair with |x|^2 = a, |y|^2 = b and
// x^H y = g (|g|^2 = ag2):
//   x' = c x - sig y,   y' = conj(sig) x + c y,   sig = c tau conj(g),
// with tau = sign(d) / (|d| + sqrt(d^2 + |g|^2)), d = (b - a)/2, the root of
// tau^2 |g|^2 + 2 d tau - 1 = 0 of smaller magnitude (the rotation by less than pi/4), which
// makes x'^H y' = 0; c = 1/sqrt(1 + tau^2 |g|^2).  The update is unitary whenever
// c^2 + |sig|^2 = 1, whatever tau is, so tau comes from the hardware estimates of 1/sqrt and
// 1/x (relative error ~2^-22: the pair is then orthogonal to that fraction of |g|, which the
// next sweep removes) and only c is refined by NR Newton steps: two reach full precision; one
// leaves c^2 + |sig|^2 = 1 to ~1e-13, which only rescales the pair's columns (an update that
// is a scalar multiple of a unitary one keeps their orthogonality), enough where the factors
// are stored in FP32.
struct JacobiRot {
  double c, sr, si;  // sig = sr + i si
};
template <int NR = 2>
__device__ __forceinline__ JacobiRot jacobi_rot(double a, double b, double gr, double gi,
                                                double ag2) {
  const double d = 0.5 * (b - a);
  const double w = fma(d, d, ag2);
  const double q = w * __builtin_amdgcn_rsq(w);
  const double tau = copysign(__builtin_amdgcn_rcp(fabs(d) + q), d);
  const double u = fma(tau * tau, ag2, 1.0);
  const double h = 0.5 * u;
  double c = __builtin_amdgcn_rsq(u);
#pragma unroll
  for (int i = 0; i < NR; ++i) c = c * fma(-h * c, c, 1.5);
  const double ct = c * tau;
  return {c, ct * gr, -ct * gi};
}
// 1/x for finite x != 0: hardware estimate and two Newton steps (within an ulp or so).
__device__ __forceinline__ double rcp_full(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

// The rotated pair of one row.
__device__ __forceinline__ void jacobi_apply(const JacobiRot& j, cd& x, cd& y) {
  const cd x0 = x;
  x.re = fma(j.c, x0.re, fma(-j.sr, y.re, j.si * y.im));
  x.im = fma(j.c, x0.im, fma(-j.sr, y.im, -j.si * y.re));
  const double yr = fma(j.sr, x0.re, fma(j.si, x0.im, j.c * y.re));
  y.im = fma(j.sr, x0.im, fma(-j.si, x0.re, j.c * y.im));
  y.re = yr;
}

// Per-image status flags (mirror of the public enum).
constexpr int kImgNonfinite = 1;
constexpr int kImgNoConvergence = 2;

}  // namespace anomps
