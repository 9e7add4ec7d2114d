// Matrix-core versions of the environment sweeps and pair expectations for 16-wide bonds
// (§II-C, Eq. (4)-(5)).  Every contraction is a 16x16x16 complex product.  FP32: three real
// products (Gauss: Ar Br, Ai Bi, (Ar + Ai)(Br + Bi)), each four v_mfma_f32_16x16x4f32 (one per
// k-chunk).  Split-BF16: four real products (re*re, -im*im, re*im, im*re).  Split-BF16: each FP32 operand x is written as
// x_hi + x_lo with x_hi = bf16(x) and x_lo = bf16(x - x_hi), and each real product as
// a_hi b_hi + a_hi b_lo + a_lo b_hi in three v_mfma_f32_16x16x16_bf16 (FP32 accumulation); the
// dropped a_lo b_lo term and the two roundings leave a relative error of at most ~3 * 2^-18
// per product term.
//
// Operand convention (one wave, lane l, g = l/16): for k-chunk kc the lane supplies
//   A-operand value  A[l%16][4g+kc],   B-operand value  B[4g+kc][l%16],
// and owns accumulator entries D[4g+r][l%16], r = 0..3 (FP64: see kidx).  Because the accumulator layout equals
// the B-operand layout (chunk kc <-> entry r), a product can feed the right factor of the next
// product directly from registers; an accumulator holding M^T is the A-operand of M, so
// environments and carried blocks are kept transposed and no product goes through LDS.  Site
// tiles are read from memory straight into operand registers, one step ahead.  Tiles are zero
// padded to 16 when a bond is narrower.
//
// Work mapping is XCD-aware: workgroup w runs on XCD w % 8, so all workgroups of image b are
// placed on XCD b % 8 (the same XCD that ran the layer kernels of image b), keeping its tensors
// and environments in one L2.
#include "common.hpp"
#include "kernels.hpp"

namespace anomps {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int W = 64;        // one wavefront per workgroup
constexpr int NXCD = 8;
constexpr int kMaxTargets16 = 256;

// How a 16x16x16 complex product runs on the matrix cores:
//  kMmaGauss     FP32, three real products (v_mfma_f32_16x16x4f32),
//  kMmaSplitBf16 FP32 operands split into two bf16 parts (v_mfma_f32_16x16x16bf16_1k),
//  kMmaF64       FP64, four real products (v_mfma_f64_16x16x4f64; its accumulator rows are
//                interleaved differently, see kidx).
enum : int { kMmaGauss = 0, kMmaSplitBf16 = 1, kMmaF64 = 2 };
template <int MODE>
struct MmaReal {
  using type = float;
  using v4 = f4;
};
template <>
struct MmaReal<kMmaF64> {
  using type = double;
  using v4 = d4;
};

template <typename V>
struct AccT {
  V re, im;
};
template <int MODE>
using Acc = AccT<typename MmaReal<MODE>::v4>;

template <int MODE>
__device__ __forceinline__ Acc<MODE> acc_zero() {
  using R = typename MmaReal<MODE>::type;
  Acc<MODE> a;
  a.re = typename MmaReal<MODE>::v4{R(0), R(0), R(0), R(0)};
  a.im = a.re;
  return a;
}

__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

typedef short s4 __attribute__((ext_vector_type(4)));

// FP32 -> bf16 bit pattern, round to nearest even (operands here are finite).
__device__ __forceinline__ unsigned bf16_bits(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}

// hi/lo bf16 parts of four FP32 values (the lane's four k entries); `neg` negates both parts.
struct Split4 {
  s4 hi, lo;
};
__device__ __forceinline__ Split4 split4(float x0, float x1, float x2, float x3, bool neg) {
  const float x[4] = {x0, x1, x2, x3};
  const unsigned sg = neg ? 0x8000u : 0u;
  Split4 r;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const unsigned h = bf16_bits(x[j]);
    const unsigned l = bf16_bits(x[j] - __uint_as_float(h << 16));
    r.hi[j] = (short)(h ^ sg);
    r.lo[j] = (short)(l ^ sg);
  }
  return r;
}

__device__ __forceinline__ f4 mfma_split(const Split4& a, const Split4& b, f4 c) {
  c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.lo, b.hi, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.hi, b.lo, c, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.hi, b.hi, c, 0, 0, 0);
}

// C += A B with per-lane operand values for the four k-chunks (entry kc of the lane holds
// k = 4g + kc, which is also the element order of a 16x16x16 bf16 operand).
template <int MODE, typename C>
__device__ __forceinline__ void cgemm(Acc<MODE>& c, const C (&a)[4], const C (&b)[4]) {
  if constexpr (MODE == kMmaGauss) {
    // Three real products (Gauss): re = Ar Br - Ai Bi, im = (Ar + Ai)(Br + Bi) - Ar Br - Ai Bi,
    // as three independent chains of four MFMAs.
    f4 t1 = f4{0.f, 0.f, 0.f, 0.f}, t2 = t1, t3 = t1;
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      t1 = mfma(a[kc].re, b[kc].re, t1);
      t2 = mfma(a[kc].im, b[kc].im, t2);
      t3 = mfma(a[kc].re + a[kc].im, b[kc].re + b[kc].im, t3);
    }
    c.re += t1 - t2;
    c.im += t3 - t1 - t2;
  } else if constexpr (MODE == kMmaF64) {
    // Four real products accumulated in place: no combination step and no cancellation.
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      c.re = mfma(a[kc].re, b[kc].re, c.re);
      c.re = mfma(-a[kc].im, b[kc].im, c.re);
      c.im = mfma(a[kc].re, b[kc].im, c.im);
      c.im = mfma(a[kc].im, b[kc].re, c.im);
    }
  } else {
    const Split4 ar = split4(a[0].re, a[1].re, a[2].re, a[3].re, false);
    const Split4 ai = split4(a[0].im, a[1].im, a[2].im, a[3].im, false);
    const Split4 nai = split4(a[0].im, a[1].im, a[2].im, a[3].im, true);
    const Split4 br = split4(b[0].re, b[1].re, b[2].re, b[3].re, false);
    const Split4 bi = split4(b[0].im, b[1].im, b[2].im, b[3].im, false);
    c.re = mfma_split(ar, br, c.re);
    c.re = mfma_split(nai, bi, c.re);
    c.im = mfma_split(ar, bi, c.im);
    c.im = mfma_split(ai, br, c.im);
  }
}

// Accumulator -> B-operand values (chunk kc <-> entry r).
template <typename V, typename C>
__device__ __forceinline__ void acc_as_b(const AccT<V>& c, C (&b)[4]) {
#pragma unroll
  for (int r = 0; r < 4; ++r) b[r] = C{c.re[r], c.im[r]};
}

// Sums over the 64 lanes of 16 values at once, in 17 exchanges instead of 16 x 6: at the step
// with lane offset o the lane keeps the half of its values whose index bit matches its own lane
// bit and adds its partner's copy of that half, so after the offsets 32, 16, 8, 4 lane l holds
// value (l >> 2) & 15 summed over the lanes that differ from it in bits 2..5, and the offsets
// 2 and 1 finish the sum.  Total of value e: read it from lane 4e.
template <typename R>
__device__ __forceinline__ R sum16_lanes(const R (&v)[16]) {
  const int l = threadIdx.x;
  R a8[8], a4[4], a2[2];
  bool hi = (l >> 5) & 1;
#pragma unroll
  for (int i = 0; i < 8; ++i) a8[i] = (hi ? v[i + 8] : v[i]) + __shfl_xor(hi ? v[i] : v[i + 8], 32);
  hi = (l >> 4) & 1;
#pragma unroll
  for (int i = 0; i < 4; ++i) a4[i] = (hi ? a8[i + 4] : a8[i]) + __shfl_xor(hi ? a8[i] : a8[i + 4], 16);
  hi = (l >> 3) & 1;
#pragma unroll
  for (int i = 0; i < 2; ++i) a2[i] = (hi ? a4[i + 2] : a4[i]) + __shfl_xor(hi ? a4[i] : a4[i + 2], 8);
  hi = (l >> 2) & 1;
  R s = (hi ? a2[1] : a2[0]) + __shfl_xor(hi ? a2[0] : a2[1], 4);
  s += __shfl_xor(s, 2);
  s += __shfl_xor(s, 1);
  return s;
}

// The k index that lane group g (= l/16) covers in the product's k-chunk kc.  The FP32 and bf16
// instructions leave accumulator entry r of lane l at row 4g + r, so chunk kc takes k = 4g + kc;
// the FP64 instruction leaves it at row g + 4r, so there chunk kc takes k = g + 4kc.  Either way
// accumulator entry r of lane l is the B-operand value of chunk r, and every load and store
// below uses the same map.
template <typename R>
__device__ __forceinline__ int kidx(int kc, int g) {
  if constexpr (sizeof(R) == 8) return g + 4 * kc;
  return 4 * g + kc;
}

// Operand registers of the two physical slices of a site tensor (Dl x 2 x Dr, slot stride 16),
// zero outside the Dl x Dr corner:
//   column form a[u][kc] = A_u[k][l%16]  (B-operand of A_u, A-operand of A_u^T)
//   row form    a[u][kc] = A_u[l%16][k]  (A-operand of A_u, B-operand of A_u^T),  k = kidx(kc, g)
// load() reads all 16 x 16 entries of both slices (always inside the slot) and only notes which
// lie in the corner; settle() zeroes the others and must run before the operands are used.  A
// select on the loaded values at load time would make the wavefront wait for the loads right
// there, and the fetch ahead of use would hide nothing.
template <typename R>
struct SiteOps {
  cx<R> a[2][4];
  unsigned keep;  // bit kc: entry kc of this lane lies in the corner (for both slices)
  __device__ __forceinline__ void load(const R* slot, int Dl, int Dr, bool row) {
    const int l = threadIdx.x, i16 = l & 15, g = l >> 4;
    keep = 0;
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      const int kk = kidx<R>(kc, g), c = row ? i16 : kk, e = row ? kk : i16;
      keep |= (unsigned)(c < Dl && e < Dr) << kc;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int idx = (c * 2 + u) * 16 + e;
        a[u][kc] = cx<R>{slot[2 * idx], slot[2 * idx + 1]};
      }
    }
  }
  __device__ __forceinline__ void settle() {
#pragma unroll
    for (int kc = 0; kc < 4; ++kc)
#pragma unroll
      for (int u = 0; u < 2; ++u)
        if (!((keep >> kc) & 1u)) a[u][kc] = cx<R>{R(0), R(0)};
  }
};

// Row form (A-operand) of a 16x16 environment tile E[x][y] stored at x*16 + y.
template <typename R>
__device__ __forceinline__ void ld_env_row(const R* t, cx<R> (&v)[4]) {
  const int l = threadIdx.x, i16 = l & 15, g = l >> 4;
#pragma unroll
  for (int kc = 0; kc < 4; ++kc) {
    const int idx = i16 * 16 + kidx<R>(kc, g);
    v[kc] = cx<R>{t[2 * idx], t[2 * idx + 1]};
  }
}

template <typename C>
__device__ __forceinline__ void conj4(const C (&a)[4], C (&b)[4]) {
#pragma unroll
  for (int kc = 0; kc < 4; ++kc) b[kc] = C{a[kc].re, -a[kc].im};
}

// A matrix M is carried transposed in the accumulator: the lane then holds M^T[k][l%16] =
// M[l%16][k] (k = kidx(r, g)), which is the A-operand of M, so a chain of products never
// leaves registers.
//
// Left transfer E' = sum_u A_u^T E conj(A_u) with E given as its A-operand (row form):
// X_u = E conj(A_u), then E'^T = sum_u X_u^T A_u (the accumulator of X_u is the A-operand of
// X_u^T).  a = column forms of A_0, A_1.  Returns E'^T.
// Gauss's three partial products of a sum of complex products, kept apart until the sum is
// complete: t1 = sum Ar Br, t2 = sum Ai Bi, t3 = sum (Ar + Ai)(Br +- Bi).  For B (sign +):
// re = t1 - t2, im = t3 - t1 - t2; for conj(B) (sign -): re = t1 + t2, im = t3 - t1 + t2.  The
// conjugate never has to be formed, and several products into one output are combined once.
struct Gauss3 {
  f4 t1, t2, t3;
};
__device__ __forceinline__ Gauss3 gauss_zero() {
  const f4 z = f4{0.f, 0.f, 0.f, 0.f};
  return Gauss3{z, z, z};
}
// bs[kc] = Br + Bi (or Br - Bi for conj(B)), computed once per B operand.
__device__ __forceinline__ void gauss_acc(Gauss3& g, const cx<float> (&a)[4], const cx<float> (&b)[4],
                                          const float (&bs)[4]) {
#pragma unroll
  for (int kc = 0; kc < 4; ++kc) {
    g.t1 = mfma(a[kc].re, b[kc].re, g.t1);
    g.t2 = mfma(a[kc].im, b[kc].im, g.t2);
    g.t3 = mfma(a[kc].re + a[kc].im, bs[kc], g.t3);
  }
}
template <bool CONJ>
__device__ __forceinline__ Acc<kMmaGauss> gauss_done(const Gauss3& g) {
  Acc<kMmaGauss> c;
  c.re = CONJ ? g.t1 + g.t2 : g.t1 - g.t2;
  c.im = CONJ ? g.t3 - g.t1 + g.t2 : g.t3 - g.t1 - g.t2;
  return c;
}

template <int MODE, typename C>
__device__ __forceinline__ Acc<MODE> left_transfer_t(const C (&e)[4], const C (&a)[2][4]) {
  if constexpr (MODE == kMmaGauss) {
    float bsum[2][4], bdif[2][4];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) {
        bsum[u][kc] = a[u][kc].re + a[u][kc].im;
        bdif[u][kc] = a[u][kc].re - a[u][kc].im;
      }
    Gauss3 go = gauss_zero();
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      Gauss3 gx = gauss_zero();
      gauss_acc(gx, e, a[u], bdif[u]);  // X_u = E conj(A_u)
      C xa[4];
      acc_as_b(gauss_done<true>(gx), xa);
      gauss_acc(go, xa, a[u], bsum[u]);  // + X_u^T A_u
    }
    return gauss_done<false>(go);
  } else {
    Acc<MODE> out = acc_zero<MODE>();
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      C ac[4], xa[4];
      conj4(a[u], ac);
      Acc<MODE> x = acc_zero<MODE>();
      cgemm<MODE>(x, e, ac);
      acc_as_b(x, xa);
      cgemm<MODE>(out, xa, a[u]);
    }
    return out;
  }
}

}  // namespace

// ------------------------------------------------------------------------- environments
// One image: st = its n slots, ev = its environment block of this side ([n+1][16][16]).  The
// environment is carried transposed in registers; tiles E[x][y] are stored at x*16 + y.
template <int MODE>
__device__ __forceinline__ void env16_image(const typename MmaReal<MODE>::type* st,
                                            typename MmaReal<MODE>::type* ev, int n, int chi,
                                            int layers, int side) {
  using R = typename MmaReal<MODE>::type;
  using C = cx<R>;
  constexpr size_t SLOT = (size_t)2 * 16 * 16 * 2;
  constexpr size_t ETILE = (size_t)16 * 16 * 2;
  const int l = threadIdx.x, i16 = l & 15, g = l >> 4;
  auto dim = [&](int k) { return bond_dim(n, chi, layers, k); };
  Acc<MODE> e = acc_zero<MODE>();  // the 1 x 1 identity
  if (l == 0) e.re[0] = R(1);
  auto store_env = [&](int k) {
    R* dst = ev + (size_t)k * ETILE;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int idx = i16 * 16 + kidx<R>(r, g);
      dst[2 * idx] = e.re[r];
      dst[2 * idx + 1] = e.im[r];
    }
  };
  // The chain has one wavefront per (image, side), two per SIMD at a batch of 1024, so nothing
  // hides a site's load latency but the chain's own lead: the operands of the next kEnvAhead
  // sites are in flight while a site is transferred (a ring of registers, indexed statically by
  // unrolling the loop kEnvAhead steps at a time).
  constexpr int kEnvAhead = 3;
  SiteOps<R> ring[kEnvAhead];
  const bool right = side != 0;
  auto fetch = [&](int t, SiteOps<R>& o) {
    const int k = right ? n - 1 - t : t;
    o.load(st + (size_t)k * SLOT, dim(k - 1), dim(k), right);
  };
  store_env(right ? n : 0);
#pragma unroll
  for (int j = 0; j < kEnvAhead; ++j)
    if (j < n) fetch(j, ring[j]);
  for (int t0 = 0; t0 < n; t0 += kEnvAhead) {
#pragma unroll
    for (int j = 0; j < kEnvAhead; ++j) {
      const int t = t0 + j;
      if (t < n) {
        C eo[4];
        acc_as_b(e, eo);
        // Left: L_{k+1} = sum_u A_u^T L_k conj(A_u) from the column forms.  Right:
        // R_k = sum_s A_s R_{k+1} A_s^H, i.e. Y_s = R conj(A_s^T) and R_k^T = sum_s Y_s^T A_s^T:
        // the same two products with the row forms (the row form of A_s is the column form of
        // A_s^T).
        ring[j].settle();
        e = left_transfer_t<MODE>(eo, ring[j].a);
        store_env(right ? n - 1 - t : t + 1);
        if (t + kEnvAhead < n) fetch(t + kEnvAhead, ring[j]);
      }
    }
  }
}

// ------------------------------------------------------------------------- pairs
template <typename C>
__device__ __forceinline__ C cmul_c(C a, C b) { return C{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }

// Operands fetched one step ahead: the site (column form to carry through it and to open,
// row form to close) and, at the open, L_i.  R_{j+1} and L_j are read at the close itself:
// prefetching them too made the pair kernel slower (more registers, fewer waves in flight).
template <typename R>
struct PairStep {
  SiteOps<R> s;
  cx<R> li[4];
};

// One image and one start site i: st = its n slots, evL = its environments ([2][n+1][16][16]),
// out = its [m][15] outputs.
//  open at i:   X_s' = L_i conj(A_s'),  F^{0s'} = A_0^T X_s'   (s' = 0, 1)
//  carry k:     F <- sum_u A_u^T F conj(A_u) for F^00 and F^01
//  close at j:  Y_t' = R_{j+1} A_t'^H,  G^{tt'} = A_t Y_t',  F^11 = L_j - F^00
//               rho[(s,t),(s',t')] = sum_{d,d'} F^{ss'}[d][d'] G^{tt'}[d][d']
// F^{ss'} and G^{tt'} are held transposed (lane: entry (x, y) = (l%16, kidx(r, g))), G^01 also
// untransposed (entry (y, x)), so every upper-triangle entry of the Hermitian rho is a sum of
// lane-local products: only F^{ss'} with s <= s' appear there, and G^10[x][y] = conj(G^01[y][x]).
template <int MODE>
__device__ __forceinline__ void pairs16_image(const typename MmaReal<MODE>::type* st,
                                              const typename MmaReal<MODE>::type* evL,
                                              const int* pairs, int m, int n, int chi, int layers,
                                              int i, typename MmaReal<MODE>::type* out) {
  using R = typename MmaReal<MODE>::type;
  using C = cx<R>;
  __shared__ int tq[kMaxTargets16], tj[kMaxTargets16];
  __shared__ int cnt;
  constexpr size_t SLOT = (size_t)2 * 16 * 16 * 2;
  constexpr size_t ETILE = (size_t)16 * 16 * 2;
  const int l = threadIdx.x;
  const R* evR = evL + (size_t)(n + 1) * ETILE;
  auto dim = [&](int k) { return bond_dim(n, chi, layers, k); };
  const R qnan = R(__builtin_nan(""));

  if (l == 0) cnt = 0;
  __syncthreads();
  for (int q = l; q < m; q += W) {
    const int pi = pairs[2 * q], pj = pairs[2 * q + 1];
    const bool valid = pi >= 0 && pi < n - 1 && pj > pi && pj < n;
    if (valid && pi == i) {
      const int slot = atomicAdd(&cnt, 1);
      if (slot < kMaxTargets16) {
        tq[slot] = q;
        tj[slot] = pj;
      } else {
        for (int al = 0; al < 15; ++al) out[(size_t)q * 15 + al] = qnan;
      }
    } else if (!valid && i == 0) {
      for (int al = 0; al < 15; ++al) out[(size_t)q * 15 + al] = qnan;
    }
  }
  __syncthreads();
  const int nt = uniform_int(min(cnt, kMaxTargets16));
  if (nt == 0) return;
  if (l == 0) {
    for (int x = 1; x < nt; ++x) {
      const int kj = tj[x], kq = tq[x];
      int y = x - 1;
      while (y >= 0 && tj[y] > kj) {
        tj[y + 1] = tj[y];
        tq[y + 1] = tq[y];
        --y;
      }
      tj[y + 1] = kj;
      tq[y + 1] = kq;
    }
  }
  __syncthreads();

  // Steps: 2 = open at i, 0 = carry through site `site`, 1 = close at the next target.
  int x = 0, cur = i + 1;
  auto successor = [&](int kind, int site, int& nk, int& ns) {
    int xx = x, cc = cur;
    if (kind == 1) ++xx;
    else if (kind == 0) cc = site + 1;
    if (xx >= nt) {
      nk = -1;
      ns = 0;
      return;
    }
    const int j = uniform_int(tj[xx]);
    nk = cc < j ? 0 : 1;
    ns = cc < j ? cc : j;
  };
  auto fetch = [&](int kind, int site, PairStep<R>& p) {
    p.s.load(st + (size_t)site * SLOT, dim(site - 1), dim(site), kind == 1);
    if (kind == 2) ld_env_row(evL + (size_t)site * ETILE, p.li);
  };
  PairStep<R> pa, pb;
  int kind = 2, site = i;
  fetch(kind, site, pa);
  Acc<MODE> F0 = acc_zero<MODE>(), F1 = acc_zero<MODE>();  // F^00, F^01, transposed
  while (kind >= 0) {
    int nk, ns;
    successor(kind, site, nk, ns);
    if (nk >= 0) fetch(nk, ns, pb);
    pa.s.settle();
    if (kind == 2) {
      C ac[4], xa[4];
      conj4(pa.s.a[0], ac);
      Acc<MODE> x0 = acc_zero<MODE>();
      cgemm<MODE>(x0, pa.li, ac);
      acc_as_b(x0, xa);
      F0 = acc_zero<MODE>();
      cgemm<MODE>(F0, xa, pa.s.a[0]);
      conj4(pa.s.a[1], ac);
      Acc<MODE> x1 = acc_zero<MODE>();
      cgemm<MODE>(x1, pa.li, ac);
      acc_as_b(x1, xa);
      F1 = acc_zero<MODE>();
      cgemm<MODE>(F1, xa, pa.s.a[0]);
    } else if (kind == 0) {
      C fo[4];
      acc_as_b(F0, fo);
      const Acc<MODE> n0 = left_transfer_t<MODE>(fo, pa.s.a);
      acc_as_b(F1, fo);
      F1 = left_transfer_t<MODE>(fo, pa.s.a);
      F0 = n0;
    } else {
      C rj[4], lj[4];
      ld_env_row(evR + (size_t)(site + 1) * ETILE, rj);
      ld_env_row(evL + (size_t)site * ETILE, lj);
      // Y_t' = R A_t'^H (B-operand conj of the row form); G^{tt'T} = Y_t'^T A_t^T; G^01 = A_0 Y_1
      C ah[4], y0a[4], y1a[4];
      conj4(pa.s.a[0], ah);
      Acc<MODE> y = acc_zero<MODE>();
      cgemm<MODE>(y, rj, ah);
      acc_as_b(y, y0a);
      conj4(pa.s.a[1], ah);
      y = acc_zero<MODE>();
      cgemm<MODE>(y, rj, ah);
      acc_as_b(y, y1a);
      Acc<MODE> g00 = acc_zero<MODE>(), g01 = acc_zero<MODE>(), g11 = acc_zero<MODE>(),
                h01 = acc_zero<MODE>();
      cgemm<MODE>(g00, y0a, pa.s.a[0]);
      cgemm<MODE>(g01, y1a, pa.s.a[0]);
      cgemm<MODE>(g11, y1a, pa.s.a[1]);
      cgemm<MODE>(h01, pa.s.a[0], y1a);
      // upper triangle of rho, entry (row, col) with row = s*2+t, col = s'*2+t'
      R d00 = 0, d11 = 0, d22 = 0, d33 = 0;
      C e01{0, 0}, e02{0, 0}, e03{0, 0}, e12{0, 0}, e13{0, 0}, e23{0, 0};
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const C f00{F0.re[r], F0.im[r]}, f01{F1.re[r], F1.im[r]};
        const C f11{lj[r].re - f00.re, lj[r].im - f00.im};
        const C G00{g00.re[r], g00.im[r]}, G01{g01.re[r], g01.im[r]}, G11{g11.re[r], g11.im[r]};
        const C G10{h01.re[r], -h01.im[r]};
        d00 += f00.re * G00.re - f00.im * G00.im;
        d11 += f00.re * G11.re - f00.im * G11.im;
        d22 += f11.re * G00.re - f11.im * G00.im;
        d33 += f11.re * G11.re - f11.im * G11.im;
        const C p01 = cmul_c(f00, G01), p02 = cmul_c(f01, G00), p03 = cmul_c(f01, G01);
        const C p12 = cmul_c(f01, G10), p13 = cmul_c(f01, G11), p23 = cmul_c(f11, G01);
        e01 = C{e01.re + p01.re, e01.im + p01.im};
        e02 = C{e02.re + p02.re, e02.im + p02.im};
        e03 = C{e03.re + p03.re, e03.im + p03.im};
        e12 = C{e12.re + p12.re, e12.im + p12.im};
        e13 = C{e13.re + p13.re, e13.im + p13.im};
        e23 = C{e23.re + p23.re, e23.im + p23.im};
      }
      {
        const R part[16] = {d00,    d11,    d22,    d33,    e01.re, e01.im, e02.re, e02.im,
                            e03.re, e03.im, e12.re, e12.im, e13.re, e13.im, e23.re, e23.im};
        const R s = sum16_lanes(part);
        auto total = [&](int e) { return __shfl(s, 4 * e); };
        d00 = total(0);
        d11 = total(1);
        d22 = total(2);
        d33 = total(3);
        e01 = C{total(4), total(5)};
        e02 = C{total(6), total(7)};
        e03 = C{total(8), total(9)};
        e12 = C{total(10), total(11)};
        e13 = C{total(12), total(13)};
        e23 = C{total(14), total(15)};
      }
      // full rho (row-major 4x4): lower triangle = conjugate transpose
      const C rho[16] = {C{d00, 0}, e01, e02, e03,
                         C{e01.re, -e01.im}, C{d11, 0}, e12, e13,
                         C{e02.re, -e02.im}, C{e12.re, -e12.im}, C{d22, 0}, e23,
                         C{e03.re, -e03.im}, C{e13.re, -e13.im}, C{e23.re, -e23.im}, C{d33, 0}};
      // <P_a (x) P_c> = sum_{s,t,s',t'} rho[(s,t),(s',t')] P_a[s'][s] P_c[t'][t].  A Pauli
      // matrix has one entry per column: P[s'][s] = phi(s) for s' = s XOR x (x = 1 for X and Y),
      // phi = 1 (I, X), i (-1)^s (Y), (-1)^s (Z); so each expectation is four entries of rho
      // times a phase in {1, i, -1, -i}, fixed at compile time.  Every lane evaluates all 15
      // (the entries are the same in all lanes) and lane l keeps number l.
      R val = 0;
#pragma unroll
      for (int o = 0; o < 15; ++o) {
        const int pa_ = (o + 1) >> 2, pc = (o + 1) & 3;
        const int xa = (pa_ == 1 || pa_ == 2), xc = (pc == 1 || pc == 2);
        R acc = 0;
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          const int s = st >> 1, t = st & 1;
          const C z = rho[(s * 2 + t) * 4 + (s ^ xa) * 2 + (t ^ xc)];
          const int ipow = (pa_ == 2) + (pc == 2);
          const bool neg = (((pa_ >= 2) && s) != ((pc >= 2) && t)) != (ipow == 2);
          const R v = (ipow == 1) ? -z.im : z.re;  // Re(z i^ipow) up to the sign
          acc += neg ? -v : v;
        }
        val = (l == o) ? acc : val;
      }
      if (l < 15) out[(size_t)uniform_int(tq[x]) * 15 + l] = val;
    }
    if (kind == 1) ++x;
    else if (kind == 0) cur = site + 1;
    kind = nk;
    site = ns;
    pa = pb;
  }
}

// Workgroup w runs on XCD w % 8; all workgroups of one image sit on the same XCD so that its
// state and environments are shared through that XCD's L2.
template <int MODE>
__global__ __launch_bounds__(W) void k_env16(const typename MmaReal<MODE>::type* state,
                                              typename MmaReal<MODE>::type* env, int n, int chi,
                                              int layers, int batch) {
  constexpr size_t SLOT = (size_t)2 * 16 * 16 * 2;
  constexpr size_t ETILE = (size_t)16 * 16 * 2;
  const int w = blockIdx.x, xcd = w % NXCD, j = w / NXCD;
  const int b = NXCD * (j >> 1) + xcd, side = j & 1;
  if (b >= batch) return;
  env16_image<MODE>(state + (size_t)b * n * SLOT, env + ((size_t)b * 2 + side) * (n + 1) * ETILE,
                    n, chi, layers, side);
}

template <int MODE>
__device__ __forceinline__ void pairs16_block(const typename MmaReal<MODE>::type* state,
                                              const typename MmaReal<MODE>::type* env,
                                              const int* pairs, int m, int n, int chi, int layers,
                                              int batch, typename MmaReal<MODE>::type* out,
                                              int block_groups) {
  constexpr size_t SLOT = (size_t)2 * 16 * 16 * 2;
  constexpr size_t ETILE = (size_t)16 * 16 * 2;
  // Launch order: the images are taken in blocks of `block_groups` groups of NXCD images, and
  // inside a block start site major (every image's start site 0 first, the last sites -- for
  // neighbour pairs those with only short partners and no carry -- last).  A block small
  // enough for its images' tiles to stay in the XCDs' L2 caches reads each tile from HBM once;
  // the last block still ends the launch on short workgroups.  block_groups >= the number of
  // groups is one block: start site major over the whole batch.  Image b runs on XCD b % NXCD.
  const int w = blockIdx.x, xcd = w % NXCD, jw = w / NXCD, groups = (batch + NXCD - 1) / NXCD;
  const int bg = (block_groups > 0 && block_groups < groups) ? block_groups : groups;
  const int per = bg * (n - 1), blk = jw / per, r = jw - blk * per;
  const int g0 = blk * bg, gc = (groups - g0) < bg ? (groups - g0) : bg;
  const int b = NXCD * (g0 + r % gc) + xcd, i = r / gc;
  if (b >= batch) return;
  pairs16_image<MODE>(state + (size_t)b * n * SLOT, env + (size_t)b * 2 * (n + 1) * ETILE, pairs,
                      m, n, chi, layers, i, out + (size_t)b * m * 15);
}

// FP32 modes: three waves per SIMD (168 registers, no spill), measured faster than two or four,
// the extra wave hiding MFMA and load latency.
template <int MODE>
__global__ __launch_bounds__(W) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_pairs16(
    const float* state, const float* env, const int* pairs, int m, int n, int chi, int layers,
    int batch, float* out, int block_groups) {
  pairs16_block<MODE>(state, env, pairs, m, n, chi, layers, batch, out, block_groups);
}

// FP64: every operand and accumulator takes twice the registers.
__global__ __launch_bounds__(W) void k_pairs16_f64(const double* state, const double* env,
                                                   const int* pairs, int m, int n, int chi,
                                                   int layers, int batch, double* out,
                                                   int block_groups) {
  pairs16_block<kMmaF64>(state, env, pairs, m, n, chi, layers, batch, out, block_groups);
}

// Mixed request tables (one bucket: S = 16, FP32 or FP64), with the same XCD grouping by request.
template <int MODE>
__global__ __launch_bounds__(W) void k_env16_mixed(const mps_request* reqs, int begin, int count) {
  using R = typename MmaReal<MODE>::type;
  constexpr size_t ETILE = (size_t)16 * 16 * 2;
  const int w = blockIdx.x, xcd = w % NXCD, j = w / NXCD;
  const int r = NXCD * (j >> 1) + xcd, side = j & 1;
  if (r >= count) return;
  const mps_request* q = reqs + begin + r;
  const int n = uniform_int(q->n_sites), layers = uniform_int(uniform_ptr(q->ctrl)[0]);
  env16_image<MODE>(uniform_ptr((const R*)q->state),
                    uniform_ptr((R*)q->env) + (size_t)side * (n + 1) * ETILE, n,
                    uniform_int(q->chi), layers, side);
}

template <int MODE>
__global__ __launch_bounds__(W) void k_pairs16_mixed(const mps_request* reqs, int begin, int count,
                                                      int max_sites) {
  using R = typename MmaReal<MODE>::type;
  const int w = blockIdx.x, xcd = w % NXCD, jw = w / NXCD;
  const int r = NXCD * (jw / (max_sites - 1)) + xcd, i = jw % (max_sites - 1);
  if (r >= count) return;
  const mps_request* q = reqs + begin + r;
  const int n = uniform_int(q->n_sites), m = uniform_int(q->n_pairs);
  if (i >= n - 1 || m == 0) return;
  const int layers = uniform_int(uniform_ptr(q->ctrl)[0]);
  pairs16_image<MODE>(uniform_ptr((const R*)q->state), uniform_ptr((const R*)q->env),
                      uniform_ptr(q->pairs), m, n, uniform_int(q->chi), layers, i,
                      uniform_ptr((R*)q->out));
}

hipError_t launch_measure16_mixed(const mps_request* reqs, int begin, int count, int max_sites,
                                  bool fp64, hipStream_t stream) {
  if (count == 0) return hipSuccess;
  const int groups = (count + NXCD - 1) / NXCD;
  const dim3 genv((unsigned)(NXCD * groups * 2));
  const dim3 gpair((unsigned)((size_t)NXCD * groups * (max_sites - 1)));
  if (fp64) {
    hipLaunchKernelGGL((k_env16_mixed<kMmaF64>), genv, dim3(W), 0, stream, reqs, begin, count);
    hipLaunchKernelGGL((k_pairs16_mixed<kMmaF64>), gpair, dim3(W), 0, stream, reqs, begin, count,
                       max_sites);
  } else {
    hipLaunchKernelGGL((k_env16_mixed<kMmaGauss>), genv, dim3(W), 0, stream, reqs, begin, count);
    hipLaunchKernelGGL((k_pairs16_mixed<kMmaGauss>), gpair, dim3(W), 0, stream, reqs, begin,
                       count, max_sites);
  }
  return hipGetLastError();
}

// Dynamic LDS that caps the pair kernel at `waves_per_cu` resident workgroups per compute unit
// (160 KiB of LDS per CU on gfx950; 0 = no cap): an occupancy setting that leaves the
// arithmetic of every workgroup unchanged.
template <typename K>
size_t pair_lds_cap(K kernel, int waves_per_cu) {
  if (waves_per_cu <= 0) return 0;
  hipFuncAttributes attr{};
  if (hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(kernel)) != hipSuccess) return 0;
  const size_t per = ((size_t)160 * 1024 / (size_t)waves_per_cu) / 512 * 512;
  return per > attr.sharedSizeBytes ? per - attr.sharedSizeBytes : 0;
}

hipError_t launch_measure16(const void* state, void* env, const int* pairs, int m, int n, int chi,
                            int layers, int batch, void* out, int precision, int block_groups,
                            int waves_per_cu, hipStream_t stream) {
  const int groups = (batch + NXCD - 1) / NXCD;
  const dim3 genv((unsigned)(NXCD * groups * 2)), gpair((unsigned)((size_t)NXCD * groups * (n - 1)));
  hipError_t e;
  if (precision == MPS_PREC_FP64) {
    hipLaunchKernelGGL((k_env16<kMmaF64>), genv, dim3(W), 0, stream, (const double*)state,
                       (double*)env, n, chi, layers, batch);
    if ((e = hipGetLastError()) != hipSuccess || m == 0) return e;
    hipLaunchKernelGGL(k_pairs16_f64, gpair, dim3(W), pair_lds_cap(k_pairs16_f64, waves_per_cu),
                       stream, (const double*)state,
                       (const double*)env, pairs, m, n, chi, layers, batch, (double*)out, block_groups);
  } else if (precision == MPS_PREC_SPLIT_BF16) {
    hipLaunchKernelGGL((k_env16<kMmaSplitBf16>), genv, dim3(W), 0, stream, (const float*)state,
                       (float*)env, n, chi, layers, batch);
    if ((e = hipGetLastError()) != hipSuccess || m == 0) return e;
    hipLaunchKernelGGL((k_pairs16<kMmaSplitBf16>), gpair, dim3(W),
                       pair_lds_cap(k_pairs16<kMmaSplitBf16>, waves_per_cu), stream, (const float*)state,
                       (const float*)env, pairs, m, n, chi, layers, batch, (float*)out, block_groups);
  } else {
    hipLaunchKernelGGL((k_env16<kMmaGauss>), genv, dim3(W), 0, stream, (const float*)state,
                       (float*)env, n, chi, layers, batch);
    if ((e = hipGetLastError()) != hipSuccess || m == 0) return e;
    hipLaunchKernelGGL((k_pairs16<kMmaGauss>), gpair, dim3(W),
                       pair_lds_cap(k_pairs16<kMmaGauss>, waves_per_cu), stream, (const float*)state,
                       (const float*)env, pairs, m, n, chi, layers, batch, (float*)out, block_groups);
  }
  return hipGetLastError();
}

}  // namespace anomps
