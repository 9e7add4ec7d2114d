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
// and owns accumulator entries D[4g+r][l%16], r = 0..3.  Because the accumulator layout equals
// the B-operand layout (chunk kc <-> entry r), a product can feed the right factor of the next
// product directly from registers.  Tiles are zero padded to 16 when a bond is narrower.
//
// Work mapping is XCD-aware: workgroup w runs on XCD w % 8, so all workgroups of image b are
// placed on XCD b % 8 (the same XCD that ran the layer kernels of image b), keeping its tensors
// and environments in one L2.
#include "common.hpp"
#include "kernels.hpp"

namespace anomps {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
using cf = cx<float>;
constexpr int W = 64;        // one wavefront per workgroup
constexpr int TS = 17;       // LDS row stride of a 16x16 complex tile (bank-conflict padding)
constexpr int NXCD = 8;
constexpr int kMaxTargets16 = 256;

struct Acc {
  f4 re, im;
};

__device__ __forceinline__ Acc acc_zero() {
  Acc a;
  a.re = f4{0.f, 0.f, 0.f, 0.f};
  a.im = f4{0.f, 0.f, 0.f, 0.f};
  return a;
}

__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
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
template <bool SPLIT>
__device__ __forceinline__ void cgemm(Acc& c, const cf (&a)[4], const cf (&b)[4]) {
  if constexpr (!SPLIT) {
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
__device__ __forceinline__ void acc_as_b(const Acc& c, cf (&b)[4]) {
#pragma unroll
  for (int r = 0; r < 4; ++r) b[r] = cf{c.re[r], c.im[r]};
}

// Operand loads from a 16x16 LDS tile (row stride TS).
__device__ __forceinline__ void ld_rowop(const cf* t, cf (&v)[4], bool conj_) {  // t[l%16][4g+kc]
  const int l = threadIdx.x, i = l & 15, g = l >> 4;
#pragma unroll
  for (int kc = 0; kc < 4; ++kc) {
    cf x = t[i * TS + 4 * g + kc];
    v[kc] = conj_ ? cf{x.re, -x.im} : x;
  }
}
__device__ __forceinline__ void ld_colop(const cf* t, cf (&v)[4], bool conj_) {  // t[4g+kc][l%16]
  const int l = threadIdx.x, j = l & 15, g = l >> 4;
#pragma unroll
  for (int kc = 0; kc < 4; ++kc) {
    cf x = t[(4 * g + kc) * TS + j];
    v[kc] = conj_ ? cf{x.re, -x.im} : x;
  }
}
__device__ __forceinline__ void st_acc(cf* t, const Acc& c) {  // t[4g+r][l%16] = acc
  const int l = threadIdx.x, j = l & 15, g = l >> 4;
#pragma unroll
  for (int r = 0; r < 4; ++r) t[(4 * g + r) * TS + j] = cf{c.re[r], c.im[r]};
}

// Site tensor (Dl x 2 x Dr, slot stride 16) -> two zero-padded 16x16 tiles at[u][c][e].
struct SiteRegs {
  cf v[8];
  __device__ void load(const float* slot, int Dl, int Dr) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int idx = threadIdx.x + i * W;  // idx = (c*2+u)*16 + e
      const int c = idx >> 5, e = idx & 15;
      v[i] = (c < Dl && e < Dr) ? cf{slot[2 * idx], slot[2 * idx + 1]} : cf{0.f, 0.f};
    }
  }
  __device__ void commit(cf* at) const {  // at[u*16*TS + c*TS + e]
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int idx = threadIdx.x + i * W;
      const int c = idx >> 5, u = (idx >> 4) & 1, e = idx & 15;
      at[u * 16 * TS + c * TS + e] = v[i];
    }
  }
};

// Env tile (16x16, stride 16 in HBM) <-> LDS tile.
__device__ __forceinline__ void env_to_lds(cf* t, const float* src) {
  for (int idx = threadIdx.x; idx < 256; idx += W) t[(idx >> 4) * TS + (idx & 15)] = cf{src[2 * idx], src[2 * idx + 1]};
}

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// X_u = E conj(A_u); E' = sum_u A_u^T X_u   (left transfer of one block E held as A-operand)
template <bool SPLIT>
__device__ __forceinline__ Acc left_transfer(const cf (&e)[4], const cf (&a0)[4], const cf (&a1)[4]) {
  Acc out = acc_zero();
  cf ac[4], xb[4];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const cf (&au)[4] = u ? a1 : a0;
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) ac[kc] = cf{au[kc].re, -au[kc].im};
    Acc x = acc_zero();
    cgemm<SPLIT>(x, e, ac);
    acc_as_b(x, xb);
    cgemm<SPLIT>(out, au, xb);
  }
  return out;
}

}  // namespace

// ------------------------------------------------------------------------- environments
// One image: st = its n slots, ev = its environment block of this side ([n+1][16][16]).
template <bool SPLIT>
__device__ __forceinline__ void env16_image(const float* st, float* ev, int n, int chi, int layers, int side) {
  __shared__ cf at[2 * 16 * TS];
  __shared__ cf E[16 * TS];
  constexpr size_t SLOT = (size_t)2 * 16 * 16 * 2;
  constexpr size_t ETILE = (size_t)16 * 16 * 2;
  const int l = threadIdx.x;
  auto dim = [&](int k) { return bond_dim(n, chi, layers, k); };
  for (int idx = l; idx < 16 * TS; idx += W) E[idx] = cf{0.f, 0.f};
  if (l == 0) E[0] = cf{1.f, 0.f};
  __syncthreads();
  auto store_env = [&](int k) {
    float* dst = ev + (size_t)k * ETILE;
    for (int idx = l; idx < 256; idx += W) {
      const cf v = E[(idx >> 4) * TS + (idx & 15)];
      dst[2 * idx] = v.re;
      dst[2 * idx + 1] = v.im;
    }
  };
  SiteRegs pf;
  if (side == 0) {
    store_env(0);
    pf.load(st, dim(-1), dim(0));
    for (int k = 0; k < n; ++k) {
      pf.commit(at);
      __syncthreads();
      if (k + 1 < n) pf.load(st + (size_t)(k + 1) * SLOT, dim(k), dim(k + 1));
      cf e[4], a0[4], a1[4];
      ld_rowop(E, e, false);
      ld_colop(at, a0, false);
      ld_colop(at + 16 * TS, a1, false);
      const Acc out = left_transfer<SPLIT>(e, a0, a1);
      __syncthreads();
      st_acc(E, out);
      __syncthreads();
      store_env(k + 1);
    }
  } else {
    store_env(n);
    pf.load(st + (size_t)(n - 1) * SLOT, dim(n - 2), dim(n - 1));
    for (int k = n - 1; k >= 0; --k) {
      pf.commit(at);
      __syncthreads();
      if (k > 0) pf.load(st + (size_t)(k - 1) * SLOT, dim(k - 2), dim(k - 1));
      // Y_s = R A_s^H ; R' = sum_s A_s Y_s
      cf r[4], ah[4], as_[4], yb[4];
      ld_rowop(E, r, false);
      Acc out = acc_zero();
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        ld_rowop(at + s * 16 * TS, ah, true);   // B-operand of R A_s^H: conj(A_s[l%16][4g+kc])
        Acc y = acc_zero();
        cgemm<SPLIT>(y, r, ah);
        acc_as_b(y, yb);
        ld_rowop(at + s * 16 * TS, as_, false);  // A-operand A_s[l%16][4g+kc]
        cgemm<SPLIT>(out, as_, yb);
      }
      __syncthreads();
      st_acc(E, out);
      __syncthreads();
      store_env(k);
    }
  }
}

// ------------------------------------------------------------------------- pairs
__device__ __forceinline__ float pauli_re(int a, int r, int c, bool want_im) {
  // (P_a)[r][c] real or imaginary part
  switch (a) {
    case 0: return want_im ? 0.f : (float)(r == c);
    case 1: return want_im ? 0.f : (float)(r != c);
    case 2: return want_im ? ((r == c) ? 0.f : (r == 0 ? -1.f : 1.f)) : 0.f;
    default: return want_im ? 0.f : ((r == c) ? (r == 0 ? 1.f : -1.f) : 0.f);
  }
}

// One image and one start site i: st = its n slots, evL = its environments ([2][n+1][16][16]),
// out = its [m][15] outputs.
template <bool SPLIT>
__device__ __forceinline__ void pairs16_image(const float* st, const float* evL, const int* pairs, int m, int n,
                              int chi, int layers, int i, float* out) {
  __shared__ cf F[3][16 * TS];
  __shared__ cf at[2 * 16 * TS];
  __shared__ cf Ev[16 * TS];
  __shared__ int tq[kMaxTargets16], tj[kMaxTargets16];
  __shared__ int cnt;
  __shared__ float rho[32];
  constexpr size_t SLOT = (size_t)2 * 16 * 16 * 2;
  constexpr size_t ETILE = (size_t)16 * 16 * 2;
  const int l = threadIdx.x, g = l >> 4, lj = l & 15;
  const float* evR = evL + (size_t)(n + 1) * ETILE;
  auto dim = [&](int k) { return bond_dim(n, chi, layers, k); };
  const float qnan = __builtin_nanf("");

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
  const int nt = min(cnt, kMaxTargets16);
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
  // Sites are visited in order i, i+1, ..., j_last; `at` holds the tile of site at_site and
  // the registers of `pf` hold the next site, loaded while the current one is contracted.
  const int jlast = tj[nt - 1];
  SiteRegs pf;
  int at_site = -1;
  pf.load(st + (size_t)i * SLOT, dim(i - 1), dim(i));
  auto need = [&](int s_) {
    if (at_site == s_) return;
    __syncthreads();
    pf.commit(at);
    at_site = s_;
    if (s_ + 1 <= jlast) pf.load(st + (size_t)(s_ + 1) * SLOT, dim(s_), dim(s_ + 1));
    __syncthreads();
  };
  env_to_lds(Ev, evL + (size_t)i * ETILE);
  need(i);
  // ---- open: X_s' = L conj(A_s'); F^{ss'} = A_s^T X_s'
  {
    cf lo[4], a0[4], a1[4], ac[4], x0[4], x1[4];
    ld_rowop(Ev, lo, false);
    ld_colop(at, a0, false);
    ld_colop(at + 16 * TS, a1, false);
    Acc x = acc_zero();
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) ac[kc] = cf{a0[kc].re, -a0[kc].im};
    cgemm<SPLIT>(x, lo, ac);
    acc_as_b(x, x0);
    x = acc_zero();
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) ac[kc] = cf{a1[kc].re, -a1[kc].im};
    cgemm<SPLIT>(x, lo, ac);
    acc_as_b(x, x1);
    Acc f00 = acc_zero(), f01 = acc_zero();
    cgemm<SPLIT>(f00, a0, x0);
    cgemm<SPLIT>(f01, a0, x1);
    st_acc(F[0], f00);
    st_acc(F[1], f01);
  }
  __syncthreads();
  int cur = i + 1;
  for (int x = 0; x < nt; ++x) {
    const int j = tj[x], q = tq[x];
    // ---- propagate through sites cur .. j-1
    for (; cur < j; ++cur) {
      need(cur);
      cf a0[4], a1[4], e[4];
      ld_colop(at, a0, false);
      ld_colop(at + 16 * TS, a1, false);
      Acc nf[2];
#pragma unroll
      for (int blk = 0; blk < 2; ++blk) {
        ld_rowop(F[blk], e, false);
        nf[blk] = left_transfer<SPLIT>(e, a0, a1);
      }
      __syncthreads();
#pragma unroll
      for (int blk = 0; blk < 2; ++blk) st_acc(F[blk], nf[blk]);
      __syncthreads();
    }
    // ---- close at j: Y_t' = R A_t'^H ; G^{tt'} = A_t Y_t'
    env_to_lds(Ev, evR + (size_t)(j + 1) * ETILE);
    // F^{11} = L_j - F^{00}: the two diagonal blocks of the open index sum to the left
    // environment of site j, so only F^{00} and F^{01} are carried through the sites between.
    {
      const float* lj = evL + (size_t)j * ETILE;
      for (int idx = l; idx < 256; idx += W) {
        const int r = idx >> 4, c = idx & 15;
        const cf f0 = F[0][r * TS + c];
        F[2][r * TS + c] = cf{lj[2 * idx] - f0.re, lj[2 * idx + 1] - f0.im};
      }
    }
    need(j);
    __syncthreads();
    Acc G[3];
    {
      cf r[4], ah[4], y0[4], y1[4], as_[4];
      ld_rowop(Ev, r, false);
      ld_rowop(at, ah, true);
      Acc y = acc_zero();
      cgemm<SPLIT>(y, r, ah);
      acc_as_b(y, y0);
      ld_rowop(at + 16 * TS, ah, true);
      y = acc_zero();
      cgemm<SPLIT>(y, r, ah);
      acc_as_b(y, y1);
      G[0] = acc_zero();
      G[1] = acc_zero();
      G[2] = acc_zero();
      ld_rowop(at, as_, false);
      cgemm<SPLIT>(G[0], as_, y0);
      cgemm<SPLIT>(G[1], as_, y1);
      ld_rowop(at + 16 * TS, as_, false);
      cgemm<SPLIT>(G[2], as_, y1);
    }
    // rho[(s,t),(s',t')] = sum_{d,d'} F^{ss'}[d][d'] G^{tt'}[d][d'];  entry e = ((s*2+t)*2+s')*2+t'
    float part[32];
#pragma unroll
    for (int e = 0; e < 32; ++e) part[e] = 0.f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int d = 4 * g + r, dp = lj;
      // F blocks at (d, dp) and at (dp, d)
      cf fa[3], fb[3];
#pragma unroll
      for (int blk = 0; blk < 3; ++blk) {
        fa[blk] = F[blk][d * TS + dp];
        fb[blk] = F[blk][dp * TS + d];
      }
      const cf g00{G[0].re[r], G[0].im[r]}, g01{G[1].re[r], G[1].im[r]}, g11{G[2].re[r], G[2].im[r]};
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int s = e >> 3, t = (e >> 2) & 1, sp = (e >> 1) & 1, tp = e & 1;
        // G^{tt'} at (d,dp); for (t,t')=(1,0) use conj(G01) paired with the transposed position.
        const bool gt = (t == 1 && tp == 0);
        const cf gv = gt ? cf{g01.re, -g01.im} : (t + tp == 0 ? g00 : (t + tp == 1 ? g01 : g11));
        // F^{ss'} at (d,dp) [or at (dp,d) when G was transposed]
        cf fv;
        if (s == 1 && sp == 0) {
          // F^{10}[x][y] = conj(F01[y][x])
          const cf src = gt ? fa[1] : fb[1];
          fv = cf{src.re, -src.im};
        } else {
          fv = gt ? fb[s + sp] : fa[s + sp];
        }
        // rho is Hermitian (row (s,t) = e >> 2, column (s',t') = e & 3): only the upper
        // triangle is accumulated, and only the real part on the diagonal.
        if ((e >> 2) <= (e & 3)) {
          part[2 * e] += fv.re * gv.re - fv.im * gv.im;
          if ((e >> 2) < (e & 3)) part[2 * e + 1] += fv.re * gv.im + fv.im * gv.re;
        }
      }
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      if ((e >> 2) <= (e & 3)) part[2 * e] = wave_sum_f(part[2 * e]);
      if ((e >> 2) < (e & 3)) part[2 * e + 1] = wave_sum_f(part[2 * e + 1]);
    }
    if (l < 32) {
      // entry e = l/2; a lower-triangle entry is the conjugate of its transpose e' = col*4 + row
      const int e = l >> 1, row = e >> 2, col = e & 3;
      const int src = row <= col ? e : col * 4 + row;
      const bool im = l & 1;
      float v = 0.f;
#pragma unroll
      for (int x = 0; x < 32; ++x) v = (x == 2 * src + (im ? 1 : 0)) ? part[x] : v;
      if (im && row > col) v = -v;
      if (im && row == col) v = 0.f;
      rho[l] = v;
    }
    __syncthreads();
    if (l < 15) {
      const int al = l + 1, pa = al >> 2, pc = al & 3;
      float acc = 0.f;
      for (int e = 0; e < 16; ++e) {
        const int s = e >> 3, t = (e >> 2) & 1, sp = (e >> 1) & 1, tp = e & 1;
        // w = P_a[s'][s] * P_c[t'][t]
        const float ar = pauli_re(pa, sp, s, false), ai = pauli_re(pa, sp, s, true);
        const float cr = pauli_re(pc, tp, t, false), ci = pauli_re(pc, tp, t, true);
        const float wr = ar * cr - ai * ci, wi = ar * ci + ai * cr;
        acc += rho[2 * e] * wr - rho[2 * e + 1] * wi;
      }
      out[(size_t)q * 15 + l] = acc;
    }
    __syncthreads();
  }
}

// Workgroup w runs on XCD w % 8; all workgroups of one image sit on the same XCD so that its
// state and environments are shared through that XCD's L2.
template <bool SPLIT>
__global__ __launch_bounds__(W) void k_env16(const float* state, float* env, int n, int chi,
                                              int layers, int batch) {
  constexpr size_t SLOT = (size_t)2 * 16 * 16 * 2;
  constexpr size_t ETILE = (size_t)16 * 16 * 2;
  const int w = blockIdx.x, xcd = w % NXCD, j = w / NXCD;
  const int b = NXCD * (j >> 1) + xcd, side = j & 1;
  if (b >= batch) return;
  env16_image<SPLIT>(state + (size_t)b * n * SLOT, env + ((size_t)b * 2 + side) * (n + 1) * ETILE, n, chi,
              layers, side);
}

// Three waves per SIMD instead of the two its 246 registers allow: the compiler spills ~100
// bytes per lane, and the launch is ~4 % faster with the extra wave hiding MFMA and LDS latency.
template <bool SPLIT>
__global__ __launch_bounds__(W) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_pairs16(const float* state, const float* env,
                                                const int* pairs, int m, int n, int chi,
                                                int layers, int batch, float* out) {
  constexpr size_t SLOT = (size_t)2 * 16 * 16 * 2;
  constexpr size_t ETILE = (size_t)16 * 16 * 2;
  const int w = blockIdx.x, xcd = w % NXCD, jw = w / NXCD;
  const int b = NXCD * (jw / (n - 1)) + xcd, i = jw % (n - 1);
  if (b >= batch) return;
  pairs16_image<SPLIT>(state + (size_t)b * n * SLOT, env + (size_t)b * 2 * (n + 1) * ETILE, pairs, m, n,
                chi, layers, i, out + (size_t)b * m * 15);
}

// Mixed request tables (one bucket: S = 16, FP32), with the same XCD grouping by request.
__global__ __launch_bounds__(W) void k_env16_mixed(const mps_request* reqs, int begin, int count) {
  constexpr size_t ETILE = (size_t)16 * 16 * 2;
  const int w = blockIdx.x, xcd = w % NXCD, j = w / NXCD;
  const int r = NXCD * (j >> 1) + xcd, side = j & 1;
  if (r >= count) return;
  const mps_request* q = reqs + begin + r;
  const int n = uniform_int(q->n_sites), layers = uniform_int(uniform_ptr(q->ctrl)[0]);
  env16_image<false>(uniform_ptr((const float*)q->state),
              uniform_ptr((float*)q->env) + (size_t)side * (n + 1) * ETILE, n, uniform_int(q->chi),
              layers, side);
}

__global__ __launch_bounds__(W) void k_pairs16_mixed(const mps_request* reqs, int begin, int count,
                                                      int max_sites) {
  const int w = blockIdx.x, xcd = w % NXCD, jw = w / NXCD;
  const int r = NXCD * (jw / (max_sites - 1)) + xcd, i = jw % (max_sites - 1);
  if (r >= count) return;
  const mps_request* q = reqs + begin + r;
  const int n = uniform_int(q->n_sites), m = uniform_int(q->n_pairs);
  if (i >= n - 1 || m == 0) return;
  const int layers = uniform_int(uniform_ptr(q->ctrl)[0]);
  pairs16_image<false>(uniform_ptr((const float*)q->state), uniform_ptr((const float*)q->env),
                uniform_ptr(q->pairs), m, n, uniform_int(q->chi), layers, i,
                uniform_ptr((float*)q->out));
}

hipError_t launch_measure16_mixed(const mps_request* reqs, int begin, int count, int max_sites,
                                  hipStream_t stream) {
  if (count == 0) return hipSuccess;
  const int groups = (count + NXCD - 1) / NXCD;
  hipLaunchKernelGGL(k_env16_mixed, dim3((unsigned)(NXCD * groups * 2)), dim3(W), 0, stream, reqs,
                     begin, count);
  hipLaunchKernelGGL(k_pairs16_mixed, dim3((unsigned)((size_t)NXCD * groups * (max_sites - 1))),
                     dim3(W), 0, stream, reqs, begin, count, max_sites);
  return hipGetLastError();
}

template <bool SPLIT>
static hipError_t launch_measure16_t(const float* state, float* env, const int* pairs, int m, int n,
                                     int chi, int layers, int batch, float* out, hipStream_t stream) {
  const int groups = (batch + NXCD - 1) / NXCD;
  hipLaunchKernelGGL((k_env16<SPLIT>), dim3((unsigned)(NXCD * groups * 2)), dim3(W), 0, stream,
                     state, env, n, chi, layers, batch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || m == 0) return e;
  hipLaunchKernelGGL((k_pairs16<SPLIT>), dim3((unsigned)((size_t)NXCD * groups * (n - 1))), dim3(W),
                     0, stream, state, (const float*)env, pairs, m, n, chi, layers, batch, out);
  return hipGetLastError();
}

hipError_t launch_measure16(const float* state, float* env, const int* pairs, int m, int n,
                            int chi, int layers, int batch, float* out, bool split_bf16,
                            hipStream_t stream) {
  return split_bf16
      ? launch_measure16_t<true>(state, env, pairs, m, n, chi, layers, batch, out, stream)
      : launch_measure16_t<false>(state, env, pairs, m, n, chi, layers, batch, out, stream);
}

}  // namespace anomps
