// Encoding and layer kernels: the one-qubit updates, the right-to-left canonical sweep and the
// CNOT ladder with FP64 one-sided Jacobi SVD truncation (§II-B).
//
// One workgroup (a single 64-lane wavefront) owns one image and walks its chain; images are
// independent, so a batch fills the machine with one wavefront per image.  Site tensors live
// in HBM in the slot layout [site][S][2][S] (storage type T: double or float); the tensors of
// the current bond are staged in LDS in FP64 and every factorisation runs in FP64.
#include <algorithm>
#include <mutex>
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace anomps {

// One wavefront per image: every phase is latency-bound at these sizes, and splitting an image
// over more waves costs more in barriers than the extra lanes save (measured at 128 and 256).
constexpr int kLayerThreads = 64;
constexpr int kMaxSweeps = 30;

// Orders LDS accesses across the lanes of a one-wavefront workgroup.  The LDS executes one
// wavefront's instructions in issue order (a read issued after a write sees the write, from
// any lane), so the only ordering the lanes need among themselves is the program order of the
// LDS instructions: this keeps the compiler from moving memory accesses across and waits for
// nothing (the compiler waits for a read's data where it is used).  Global loads stay in flight
// (a __syncthreads waits for every outstanding load and store, which would undo the prefetches
// of the next site tensor).
__device__ __forceinline__ void wave_sync() {
  static_assert(kLayerThreads == 64, "one wavefront per workgroup");
  asm volatile("" ::: "memory");
}

// ------------------------------------------------------------------------------- encode
// One workgroup per image: writes A[k] = (cos(pi x_k/2), sin(pi x_k/2)) as a 1x2x1 tensor (|0>
// for every site when pixels is null) and (re)sets the image's status word (NaN/Inf pixels ->
// non-finite).
template <typename T>
__global__ void k_encode(T* state, const double* pixels, int n, int S, int* status) {
  const int b = blockIdx.x;
  int bad = 0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const double x = pixels ? pixels[(size_t)b * n + k] : 0.0;  // no pixels: |0>
    double s, c;
    sincos(0.5 * M_PI * x, &s, &c);
    T* slot = state + ((size_t)b * n + k) * (size_t)(2 * S * S) * 2;
    store_c<T, double>(slot, 0, cd{c, 0.0});  // (a=0, s=0, b=0)
    store_c<T, double>(slot, S, cd{s, 0.0});  // (a=0, s=1, b=0)
    bad |= !isfinite(x);
  }
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0) status[b] = bad ? kImgNonfinite : 0;
}

// ------------------------------------------------------------------------------- layer
// LDS of one image.  `mat` holds the matrix being factorised column-major with leading
// dimension LD (>= 16 so that a team of 16 lanes can always address padded rows); the
// neighbour tensor `tb` keeps the storage type (it arrives from HBM in that type).
template <int S, typename T>
struct LayerShared {
  // Row strides are padded by one element so that lanes reading different rows of a tile do
  // not fall on the same LDS banks (a power-of-two stride maps every row to bank 0).
  static constexpr int LD = ((2 * S > 16) ? 2 * S : 16) + 1;
  static constexpr int SP = S + 1;
  cd mat[LD * 2 * S];
  cd ta[2 * S * SP];          // centre tensor [a][s][c] at (a*2+s)*SP + c
  cx<T> tb[2 * S * SP];       // neighbour tensor [c][t][b] at (c*2+t)*SP + b
  cd uq[2 * S * SP];          // U [r][j] at r*SP + j (ladder) or V*Sigma [j][a] at j*SP + a (sweep)
  double sig2[2 * S];
  double isig[2 * S];         // 1/|w_c| of the column of rank j (0 for a negligible column)
  int rank[2 * S];            // columns in descending singular-value order
  double red[kLayerThreads / 64];
  double tiny2;               // negligible-column threshold of the last decomposition
};


// Sum over an aligned team of T lanes (T <= 16); every lane gets the bitwise-same result
// (each step adds a lane's value to its mirror image, so all lanes add the same operands).
template <int T>
__device__ __forceinline__ double team_sum(double v) {
  if constexpr (T >= 16) v += dpp_mov_d<0x140>(v);  // row_mirror
  if constexpr (T >= 8) v += dpp_mov_d<0x141>(v);   // row_half_mirror
  if constexpr (T >= 4) v += dpp_mov_d<0x4E>(v);    // quad_perm [2,3,0,1]
  if constexpr (T >= 2) v += dpp_mov_d<0xB1>(v);    // quad_perm [1,0,3,2]
  return v;
}

template <int CTRL>
__device__ __forceinline__ float dpp_mov_f(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
// team_sum in FP32.
template <int T>
__device__ __forceinline__ float team_sum_f(float v) {
  if constexpr (T >= 16) v += dpp_mov_f<0x140>(v);  // row_mirror
  if constexpr (T >= 8) v += dpp_mov_f<0x141>(v);   // row_half_mirror
  if constexpr (T >= 4) v += dpp_mov_f<0x4E>(v);    // quad_perm [2,3,0,1]
  if constexpr (T >= 2) v += dpp_mov_f<0xB1>(v);    // quad_perm [1,0,3,2]
  return v;
}

// Sum over the wavefront, the same value in every lane: the four DPP rows are summed inside
// (team_sum), and their sums are read as scalars and added in a fixed order.
__device__ __forceinline__ double wave_sum(double v) {
  v = team_sum<16>(v);
  auto row = [&](int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
  };
  return (row(0) + row(16)) + (row(32) + row(48));
}

// Sum over the workgroup (kLayerThreads lanes); every lane gets the same value.
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  if constexpr (kLayerThreads == 64) return v;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < kLayerThreads / 64; ++w) t += red[w];
  return t;
}

// 1/sqrt(x) for x > 0: hardware estimate (relative error ~2^-22) refined by NR Newton steps;
// two reach full FP64 precision, one ~1e-13.
template <int NR = 2>
__device__ __forceinline__ double rsqrt_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
#pragma unroll
  for (int i = 0; i < NR; ++i) r = r * fma(-h * r, r, 1.5);
  return r;
}
__device__ __forceinline__ double rsqrt_full(double x) { return rsqrt_nr<2>(x); }
// 1/x likewise.
template <int NR = 2>
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
#pragma unroll
  for (int i = 0; i < NR; ++i) r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

// Division by a runtime divisor that is usually a power of two (bond dimensions of the
// CNOT-ladder circuit are): shifts on the fast path, integer division otherwise.
struct FastDiv {
  int d, sh;
  bool p2;
  __device__ explicit FastDiv(int d_) : d(d_), sh(__ffs(d_) - 1), p2((d_ & (d_ - 1)) == 0) {}
  __device__ __forceinline__ int q(int x) const { return p2 ? (x >> sh) : x / d; }
  __device__ __forceinline__ int r(int x) const { return p2 ? (x & (d - 1)) : x % d; }
};

// Small complex products staged in LDS, on the FP64 matrix cores: out(b, i, j) = sum_{k < K}
// a(b, i, k) bm(b, k, j) for NB independent products of M x N outputs.  The wavefront takes
// one 16 x 16 output tile at a time and accumulates it over 4-deep slices of k with
// v_mfma_f64_16x16x4f64 (lane l supplies A[l % 16][k0 + l / 16] and B[k0 + l / 16][l % 16]
// and holds D[l / 16 + 4r][l % 16], r < 4); the complex product is four real ones, the real
// and imaginary parts in two accumulators.  Entries outside M, N or K enter as zeros; the
// accessors are only called with indices inside their ranges.  At the bond sizes of a chain
// (M, N, K <= 32) the products are bound by the latency of their operand reads and of the
// multiply-add chains, which the matrix cores take in a few dozen instructions.
typedef double dbl4 __attribute__((ext_vector_type(4)));

template <typename FA, typename FB, typename FO>
__device__ __forceinline__ void mfma_cgemm(int NB, int M, int N, int K, FA a, FB bm, FO out) {
  const int l = threadIdx.x, lr = l & 15, lq = l >> 4;
  const int tm = (M + 15) >> 4, tn = (N + 15) >> 4;
  for (int b = 0; b < NB; ++b)
    for (int ti = 0; ti < tm; ++ti)
      for (int tj = 0; tj < tn; ++tj) {
        const int i = ti * 16 + lr, j = tj * 16 + lr;
        const bool iok = i < M, jok = j < N;
        const int ic = iok ? i : M - 1, jc = jok ? j : N - 1;
        dbl4 cr = {0.0, 0.0, 0.0, 0.0}, ci = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
        for (int k0 = 0; k0 < K; k0 += 4) {
          const int k = k0 + lq;
          const bool kok = k < K;
          const int kc = kok ? k : K - 1;
          cd av = a(b, ic, kc), bv = bm(b, kc, jc);
          if (!(iok && kok)) av = cd{0.0, 0.0};
          if (!kok) bv = cd{0.0, 0.0};
          cr = __builtin_amdgcn_mfma_f64_16x16x4f64(av.re, bv.re, cr, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f64_16x16x4f64(av.re, bv.im, ci, 0, 0, 0);
          cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-av.im, bv.im, cr, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f64_16x16x4f64(av.im, bv.re, ci, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ii = ti * 16 + lq + 4 * r;
          if (ii < M && jok) out(b, ii, j, cd{cr[r], ci[r]});
        }
      }
}

// The same products on the vector units, one output per lane and step: cheaper than a padded
// matrix-core tile for fewer than 128 outputs per product (measured at the bond sizes of a
// 16-wide slot).
template <typename FA, typename FB, typename FO>
__device__ __forceinline__ void valu_cgemm(int NB, int M, int N, int K, FA a, FB bm, FO out) {
  const int mn = M * N;
  const FastDiv fmn(mn), fn(N);
  for (int idx = threadIdx.x; idx < NB * mn; idx += kLayerThreads) {
    const int b = fmn.q(idx), rem = fmn.r(idx);
    const int i = fn.q(rem), j = fn.r(rem);
    // even and odd k in two accumulators: half the dependent chain
    cd acc0{0.0, 0.0}, acc1{0.0, 0.0};
    int k = 0;
    for (; k + 2 <= K; k += 2) {
      cfma(acc0, a(b, i, k), bm(b, k, j));
      cfma(acc1, a(b, i, k + 1), bm(b, k + 1, j));
    }
    if (k < K) cfma(acc0, a(b, i, k), bm(b, k, j));
    out(b, i, j, cd{acc0.re + acc1.re, acc0.im + acc1.im});
  }
}

template <typename FA, typename FB, typename FO>
__device__ __forceinline__ void cgemm(int NB, int M, int N, int K, FA a, FB bm, FO out) {
  if (NB <= 0 || M <= 0 || N <= 0) return;
  if (M * N >= 128)
    mfma_cgemm(NB, M, N, K, a, bm, out);
  else
    valu_cgemm(NB, M, N, K, a, bm, out);
}

__host__ __device__ inline int pow2ceil(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

// Tile shape of the Jacobi sweep for an M x N matrix: NP = padded column count (power of 2),
// NP/2 column pairs per round, T lanes per pair (<= 16), R rows per lane, MP = R*T rows.
struct JShape {
  int NP, T, R, MP;
};
__host__ __device__ inline JShape jacobi_shape(int M, int N) {
  JShape j;
  j.NP = pow2ceil(N < 2 ? 2 : N);
  const int P = j.NP / 2;
  j.T = (kLayerThreads / P) < 16 ? kLayerThreads / P : 16;
  j.R = pow2ceil((M + j.T - 1) / j.T);
  j.MP = j.R * j.T;
  return j;
}

// One-sided (Hestenes) Jacobi on the N columns of `mat` (rows [M, MP) must be zero; columns
// [N, NP) are overwritten with zeros) in FP64.
// Column pairs follow the round-robin tournament: NP-1 rounds of NP/2 disjoint pairs per
// sweep.  A team of T lanes owns a pair; each lane holds R rows of both columns in registers,
// the team reduces |x|^2, |y|^2 and x^H y with DPP row moves, and every lane of the team
// evaluates the same rotation.  A pair is rotated when |x^H y|^2 > tol^2 |x|^2 |y|^2 with
// tol = M eps (at least 1e-7 for FP32 storage); columns with |x|^2 <= tiny2 = 1e-30 |A|_F^2
// count as numerically zero.
// On return sig2[c] = |w_c|^2 for c < N.  Returns kImgNoConvergence if the sweep limit hit.
template <int S, typename T, int NP, int R>
__device__ __forceinline__ int jacobi_tile(LayerShared<S, T>& sh, int M, int N) {
  constexpr int LD = LayerShared<S, T>::LD;
  constexpr int P = NP / 2;
  constexpr int TM = (kLayerThreads / P) < 16 ? kLayerThreads / P : 16;
  constexpr int MP = R * TM;
  static_assert(MP <= LD, "tile rows exceed the LDS column");
  const int tid = threadIdx.x;
  const int q = tid / TM, lt = tid % TM;
  const bool active = q < P;
  double f = 0.0;
  for (int idx = tid; idx < N * MP; idx += kLayerThreads) {
    const cd v = sh.mat[(idx / MP) * LD + (idx % MP)];
    f = fma(v.re, v.re, fma(v.im, v.im, f));
  }
  // Padding columns [N, NP) are set to zero: a pair with one of them never passes the
  // negligible-column test, so the rounds need no column-range test.
  for (int idx = tid; idx < (NP - N) * MP; idx += kLayerThreads)
    sh.mat[(N + idx / MP) * LD + (idx % MP)] = cd{0.0, 0.0};
  f = block_sum(f, sh.red);
  const double tiny2 = 1e-30 * f;
  if (tid == 0) sh.tiny2 = tiny2;
  // Factors stored in FP32 (rounding 6e-8) gain nothing from rotating pairs closer than 1e-7
  // to orthogonal: the sweep that confirms convergence then rotates no pair at all.
  const double tol = std::is_same<T, float>::value ? fmax((double)M * 2.220446049250313e-16, 1e-7)
                                                   : (double)M * 2.220446049250313e-16;
  const double tol2 = tol * tol;
  constexpr double kBig = std::is_same<T, float>::value ? 1e-7 : 1e-16;
  // byte offsets into mat: kRow per row, kCol per column
  constexpr int kRow = (int)sizeof(cd), kCol = LD * kRow;
  char* const base = reinterpret_cast<char*>(sh.mat);
  const int inc_i = (active && q > 0) ? kCol : 0, inc_j = active ? kCol : 0;
  const int wrap = NP * kCol + lt * kRow, first = kCol + lt * kRow;
  // lanes without a pair never pass the negligible-column test
  const double tiny2_l = active ? tiny2 : __builtin_huge_val();
  bool converged = (N < 2);
  int sweep = 0;
  for (; !converged && sweep < kMaxSweeps; ++sweep) {
    int big = 0;
    // Round-robin positions: pair q = (pos(q), pos(NP-1-q)), pos(0) = 0 and pos(i) =
    // 1 + ((i - 1 + r) mod (NP - 1)), advanced from round to round as byte offsets oi, oj of
    // the lane's first rows of the two columns: + one column, from column NP back to column 1
    // (column 0 stays; lanes without a pair stay on column 0 and never store).  The next
    // offsets are computed early in each round, off the path from the last store to the next
    // round's loads.
    int oi = ((q == 0 || !active) ? 0 : q) * kCol + lt * kRow;
    int oj = (active ? NP - 1 - q : 0) * kCol + lt * kRow;
    for (int r = 0; r < NP - 1; ++r) {
      cd x[R], y[R];
      double gr = 0.0, gi = 0.0;
      double a = 0.0, bb = 0.0;
#pragma unroll
      for (int t = 0; t < R; ++t) {
        x[t] = *reinterpret_cast<const cd*>(base + oi + t * TM * kRow);
        y[t] = *reinterpret_cast<const cd*>(base + oj + t * TM * kRow);
        gr = fma(x[t].re, y[t].re, fma(x[t].im, y[t].im, gr));
        gi = fma(x[t].re, y[t].im, fma(-x[t].im, y[t].re, gi));
        a = fma(x[t].re, x[t].re, fma(x[t].im, x[t].im, a));
        bb = fma(y[t].re, y[t].re, fma(y[t].im, y[t].im, bb));
      }
      int oi_n = oi + inc_i, oj_n = oj + inc_j;
      oi_n = (oi_n == wrap) ? first : oi_n;
      oj_n = (oj_n == wrap) ? first : oj_n;
      if constexpr (std::is_same<T, float>::value) {
        // FP32 storage: the team sums in FP32, each step one DPP-modified add instead of two
        // lane moves and an FP64 add.  The rotation stays exactly unitary (c and sigma come
        // from the same sums) and the columns are rotated in FP64; only the angle is known to
        // ~1e-7, the rotation floor.
        a = team_sum_f<TM>((float)a);
        bb = team_sum_f<TM>((float)bb);
        gr = team_sum_f<TM>((float)gr);
        gi = team_sum_f<TM>((float)gi);
      } else {
        a = team_sum<TM>(a);
        bb = team_sum<TM>(bb);
        gr = team_sum<TM>(gr);
        gi = team_sum<TM>(gi);
      }
      const double ag2 = fma(gr, gr, gi * gi);
      const double ab = a * bb;
      // the next offsets are computed here, ahead of the test
      asm volatile("" ::"v"(oi_n), "v"(oj_n));
      if (fmin(a, bb) > tiny2_l && ag2 > tol2 * ab) {
        if (ag2 > kBig * ab) big = 1;
        const JacobiRot jr = jacobi_rot<std::is_same<T, float>::value ? 1 : 2>(a, bb, gr, gi, ag2);
#pragma unroll
        for (int tt = 0; tt < R; ++tt) {
          jacobi_apply(jr, x[tt], y[tt]);
          *reinterpret_cast<cd*>(base + oi + tt * TM * kRow) = x[tt];
          *reinterpret_cast<cd*>(base + oj + tt * TM * kRow) = y[tt];
        }
      }
      wave_sync();
      oi = oi_n;
      oj = oj_n;
    }
    // Converged when nothing was rotated, or when every rotated pair of this sweep was already
    // close to orthogonal: one-sided Jacobi converges quadratically, so a sweep whose pairs
    // were all within delta of orthogonal leaves them within ~delta^2.  delta = 1e-8 (columns
    // orthogonal to ~1e-16) for FP64 storage; 3.2e-4 for FP32 storage (~1e-7, the floor below
    // which pairs are not rotated, about the 2^-24 rounding of the stored tensors).  A lane
    // sets big only for a pair it rotates.
    converged = __ballot(big) == 0;
  }
  // sig2[c] = |w_c|^2: each team reduces one column at a time
#pragma unroll
  for (int c0 = 0; c0 < NP; c0 += P) {
    const int col = c0 + q;
    const bool own = active && col < N;
    double s2 = 0.0;
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const cd v = own ? sh.mat[col * LD + lt + t * TM] : cd{0.0, 0.0};
      s2 = fma(v.re, v.re, fma(v.im, v.im, s2));
    }
    s2 = team_sum<TM>(s2);
    if (own && lt == 0) sh.sig2[col] = s2;
  }
  wave_sync();
  return converged ? 0 : kImgNoConvergence;
}

template <int S, typename T>
__device__ __forceinline__ int jacobi_columns(LayerShared<S, T>& sh, int M, int N) {
  const JShape js = jacobi_shape(M, N);
#define ANOMPS_JT(NPV, RV)                                                           \
  if (js.NP == NPV && js.R == RV) {                                                  \
    if constexpr (NPV <= 2 * S && RV * ((kLayerThreads / (NPV / 2)) < 16 ? kLayerThreads / (NPV / 2) : 16) <= \
                                       LayerShared<S, T>::LD)                        \
      return jacobi_tile<S, T, NPV, RV>(sh, M, N);                                  \
  }
#define ANOMPS_JN(NPV) ANOMPS_JT(NPV, 1) ANOMPS_JT(NPV, 2) ANOMPS_JT(NPV, 4) ANOMPS_JT(NPV, 8)
  ANOMPS_JN(2) ANOMPS_JN(4) ANOMPS_JN(8) ANOMPS_JN(16) ANOMPS_JN(32)
#undef ANOMPS_JN
#undef ANOMPS_JT
  return kImgNoConvergence;  // unreachable for shapes within the slot
}

// Householder QR in FP64 of the columns in `mat` (column-major, leading dimension LD, rows
// [0, M) read), in independent blocks of ncb consecutive columns (N = total columns, a multiple
// of ncb, ncb <= M): each block B = Q R with Q (M x ncb) orthonormal columns and R upper
// triangular.  A team of TM lanes owns column c; lane lt holds rows lt + t*TM (R per lane) in
// registers.  Step j reflects rows [j, M) of each block's column j onto beta_j e_j with
// H_j = I - coef_j v_j v_j^H (beta_j = -e^{i arg a_jj} |a_j|, the sign that avoids
// cancellation), publishes v_j in its column of mat and coef_j in sig2, and the later columns of
// the same block take the reflection.  A column whose remaining part has |.|^2 <= 1e-30
// |A|_F^2 is left as it is (H_j = I).  Q is formed by applying H_{ncb-1}, ..., H_0 to the
// first ncb unit vectors.  Out: uq[c*SP + a] = conj(R[a][c]) (block-local row a, global column
// c), and Q into the site slot:
//  kHhCanon  (one block; canonical sweep, A = t^H, t = L Q^H with L = R^H): rows of Q^H as
//            [a][s][b], row index r = s*Dr + b;
//  kHhLadder (one block; Theta = Q R or the centre alone split as Q R): Q as [(a,s)][c], row
//            index r = a*2 + s;
//  kHhBlock2 (two blocks u = 0, 1 holding the s = u rows of the centre): A[(a,s)][c] =
//            Q_u[a][c - u*ncb] if s = u, else 0.
//  kHhBlockLds (blocks as kHhBlock2): Q kept in LDS instead, ta[r*SP + c] = Q_blk[r][c - blk*ncb]
//            for the global column c.
enum : int { kHhCanon = 0, kHhLadder = 1, kHhBlock2 = 2, kHhBlockLds = 3 };

template <int S, typename T, int NC, int R, int MODE>
__device__ __forceinline__ void householder_lq(LayerShared<S, T>& sh, int M, int N, int ncb, int Dr, T* slot) {
  constexpr int LD = LayerShared<S, T>::LD;
  constexpr int SP = LayerShared<S, T>::SP;
  constexpr int TM = (kLayerThreads / NC) < 16 ? kLayerThreads / NC : 16;
  static_assert(R * TM <= LD, "tile rows exceed the LDS column");
  const int tid = threadIdx.x;
  const int c = tid / TM, lt = tid % TM;
  const bool own = c < N;
  const int blk = own ? c / ncb : 0, lc = c - blk * ncb, base = blk * ncb;
  cd x[R];
  double f = 0.0;
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int rr = lt + t * TM;
    x[t] = (own && rr < M) ? sh.mat[c * LD + rr] : cd{0.0, 0.0};
    f = fma(x[t].re, x[t].re, fma(x[t].im, x[t].im, f));
  }
  const double tiny2 = 1e-30 * block_sum(f, sh.red);
  for (int j = 0; j < ncb; ++j) {
    // |rows >= j|^2 and the diagonal entry of this team's column (used by the pivot teams).
    double a2 = 0.0, dr = 0.0, di = 0.0;
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int rr = lt + t * TM;
      if (rr >= j) a2 = fma(x[t].re, x[t].re, fma(x[t].im, x[t].im, a2));
      if (rr == j) { dr = x[t].re; di = x[t].im; }
    }
    a2 = team_sum<TM>(a2);
    dr = team_sum<TM>(dr);
    di = team_sum<TM>(di);
    if (own && lc == j) {
      cd beta{dr, di}, v0{dr, di};
      double coef = 0.0;
      if (a2 > tiny2) {
        // One Newton step where the factors are stored in FP32: the reflector is then unitary
        // and the zeroed entries vanish to ~1e-13 relative, far below the storage rounding.
        constexpr int NR = std::is_same<T, float>::value ? 1 : 2;
        const double alpha = a2 * rsqrt_nr<NR>(a2);
        const double d2 = fma(dr, dr, di * di);
        const double rd = d2 > 0.0 ? rsqrt_nr<NR>(d2) : 0.0;
        const double ad = d2 * rd;                          // |a_jj|
        const cd u = d2 > 0.0 ? cd{dr * rd, di * rd} : cd{1.0, 0.0};
        beta = cd{-u.re * alpha, -u.im * alpha};
        v0 = cd{u.re * (ad + alpha), u.im * (ad + alpha)};
        coef = rcp_nr<NR>(alpha * (alpha + ad));            // 2 / |v|^2
      }
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const int rr = lt + t * TM;
        cd v = x[t];
        if (rr < j) v = cd{0.0, 0.0};
        if (rr == j) v = v0;
        if (rr < LD) sh.mat[c * LD + rr] = v;
        // Column j of the block's R: entries above the diagonal, beta on it.
        if (rr < ncb) sh.uq[c * SP + rr] = rr < j ? cconj(x[t]) : (rr == j ? cconj(beta) : cd{0.0, 0.0});
      }
      if (lt == 0) sh.sig2[c] = coef;
    }
    wave_sync();
    if (own && lc > j) {
      const int pc = base + j;
      const double coef = sh.sig2[pc];
      cd v[R];
      double gr = 0.0, gi = 0.0;
#pragma unroll
      for (int t = 0; t < R; ++t) {
        v[t] = sh.mat[pc * LD + lt + t * TM];
        gr = fma(v[t].re, x[t].re, fma(v[t].im, x[t].im, gr));     // v^H x
        gi = fma(v[t].re, x[t].im, fma(-v[t].im, x[t].re, gi));
      }
      gr = team_sum<TM>(gr) * coef;
      gi = team_sum<TM>(gi) * coef;
#pragma unroll
      for (int t = 0; t < R; ++t) {
        x[t].re -= gr * v[t].re - gi * v[t].im;
        x[t].im -= gr * v[t].im + gi * v[t].re;
      }
    }
  }
  // Q columns: e_lc through H_{ncb-1}, ..., H_0 of the block (column lc only meets H_j, j <= lc).
#pragma unroll
  for (int t = 0; t < R; ++t) x[t] = cd{(lt + t * TM == lc) ? 1.0 : 0.0, 0.0};
  for (int j = ncb - 1; j >= 0; --j) {
    const int pc = base + j;
    const double coef = own ? sh.sig2[pc] : 0.0;
    cd v[R];
    double gr = 0.0, gi = 0.0;
#pragma unroll
    for (int t = 0; t < R; ++t) {
      v[t] = sh.mat[pc * LD + lt + t * TM];
      gr = fma(v[t].re, x[t].re, fma(v[t].im, x[t].im, gr));
      gi = fma(v[t].re, x[t].im, fma(-v[t].im, x[t].re, gi));
    }
    gr = team_sum<TM>(gr) * coef;
    gi = team_sum<TM>(gi) * coef;
#pragma unroll
    for (int t = 0; t < R; ++t) {
      x[t].re -= gr * v[t].re - gi * v[t].im;
      x[t].im -= gr * v[t].im + gi * v[t].re;
    }
  }
  if (own) {
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int rr = lt + t * TM;
      if (rr < M) {
        if constexpr (MODE == kHhLadder) {
          store_c<T, double>(slot, (size_t)rr * S + c, x[t]);  // Q[rr][c]
        } else if constexpr (MODE == kHhBlock2) {
          store_c<T, double>(slot, (size_t)(rr * 2 + blk) * S + c, x[t]);
          store_c<T, double>(slot, (size_t)(rr * 2 + 1 - blk) * S + c, cd{0.0, 0.0});
        } else if constexpr (MODE == kHhBlockLds) {
          sh.ta[rr * SP + c] = x[t];
        } else {
          // row c of Q^H = conj(column c of Q)
          const int s_ = rr >= Dr, b = rr - (s_ ? Dr : 0);
          store_c<T, double>(slot, (size_t)(c * 2 + s_) * S + b, cconj(x[t]));
        }
      }
    }
  }
  wave_sync();
}

__host__ __device__ inline int lq_rows_per_lane(int M, int N) {
  const int nc = pow2ceil(N < 1 ? 1 : N);
  const int tm = (kLayerThreads / nc) < 16 ? kLayerThreads / nc : 16;
  return pow2ceil((M + tm - 1) / tm);
}

template <int S, typename T, int MODE>
__device__ __forceinline__ int lq_columns(LayerShared<S, T>& sh, int M, int N, int ncb, int Dr, T* slot) {
  const int nc = pow2ceil(N < 1 ? 1 : N), r = lq_rows_per_lane(M, N);
#define ANOMPS_LQ(NCV, RV)                                                                  \
  if (nc == NCV && r == RV) {                                                              \
    if constexpr (NCV <= 2 * S && RV * ((kLayerThreads / NCV) < 16 ? kLayerThreads / NCV : 16) <= \
                                      LayerShared<S, T>::LD) {                             \
      householder_lq<S, T, NCV, RV, MODE>(sh, M, N, ncb, Dr, slot);                        \
      return 0;                                                                            \
    }                                                                                      \
  }
#define ANOMPS_LQN(NCV) ANOMPS_LQ(NCV, 1) ANOMPS_LQ(NCV, 2) ANOMPS_LQ(NCV, 4) ANOMPS_LQ(NCV, 8)
  ANOMPS_LQN(1) ANOMPS_LQN(2) ANOMPS_LQN(4) ANOMPS_LQN(8) ANOMPS_LQN(16) ANOMPS_LQN(32)
#undef ANOMPS_LQN
#undef ANOMPS_LQ
  return kImgNoConvergence;  // unreachable for shapes within the slot
}

// One-qubit gates of a layer program, per site k.
enum : int { kGateNone = 0, kGateRyRz = 1, kGateHRy = 2 };
struct Gate2 {
  cd u00, u01, u10, u11;
};
// kGateRyRz: U = R_Y(theta_k) R_Z(phi_k).  kGateHRy: U = R_Y(2 pi x_k - pi) H (§II-B, Eq. (2):
// Hadamard first, then the pixel rotation), i.e. (1/sqrt 2)[[c-s, c+s], [s+c, s-c]] with
// c = cos(phi/2), s = sin(phi/2).
__device__ __forceinline__ Gate2 site_gate(int mode, int k, const double* theta,
                                           const double* phi, const double* pix) {
  Gate2 g;
  if (mode == kGateHRy) {
    double s, c;
    sincos(0.5 * (2.0 * M_PI * pix[k] - M_PI), &s, &c);
    const double r = 0.70710678118654752440;
    g.u00 = cd{(c - s) * r, 0.0};
    g.u01 = cd{(c + s) * r, 0.0};
    g.u10 = cd{(s + c) * r, 0.0};
    g.u11 = cd{(s - c) * r, 0.0};
  } else {
    double st, ct, sp, cp;
    sincos(0.5 * theta[k], &st, &ct);
    sincos(0.5 * phi[k], &sp, &cp);
    const cd em{cp, -sp}, ep{cp, sp};  // e^{-i phi/2}, e^{+i phi/2}
    g.u00 = cscale(em, ct);
    g.u01 = cscale(ep, -st);
    g.u10 = cscale(em, st);
    g.u11 = cscale(ep, ct);
  }
  return g;
}

// Apply a one-qubit gate to the physical index of the (Dl x 2 x Dr) tensor in ta.
template <int S, typename T>
__device__ __forceinline__ void apply_gate(LayerShared<S, T>& sh, int Dl, int Dr, const Gate2& g) {
  constexpr int SP = LayerShared<S, T>::SP;
  const FastDiv fd(Dr);
  for (int idx = threadIdx.x; idx < Dl * Dr; idx += kLayerThreads) {
    const int a = fd.q(idx), b = fd.r(idx);
    const cd v0 = sh.ta[(a * 2 + 0) * SP + b];
    const cd v1 = sh.ta[(a * 2 + 1) * SP + b];
    cd w0 = cmul(g.u00, v0), w1 = cmul(g.u10, v0);
    cfma(w0, g.u01, v1);
    cfma(w1, g.u11, v1);
    sh.ta[(a * 2 + 0) * SP + b] = w0;
    sh.ta[(a * 2 + 1) * SP + b] = w1;
  }
  wave_sync();
}

// FP64 value of lane `lane` in every lane (two scalar reads).
__device__ __forceinline__ double read_lane(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ cd read_lane(cd v, int lane) {
  return cd{read_lane(v.re, lane), read_lane(v.im, lane)};
}

// One-qubit gates of a sweep, computed 64 sites at a time: lane l holds the gate of site
// 64*chunk + l, all lanes evaluate theirs together (one pass of the angle loads and sincos)
// when the sweep enters a chunk, and a site's gate is then read from its lane as scalars.
struct LaneGates {
  Gate2 g{};
  int chunk = -1;
  __device__ __forceinline__ Gate2 get(int mode, int k, int n, const double* theta,
                                       const double* phi, const double* pix) {
    const int ch = k >> 6;
    if (ch != chunk) {
      const int kk = (ch << 6) + (int)threadIdx.x;
      if (kk < n) g = site_gate(mode, kk, theta, phi, pix);
      chunk = ch;
    }
    const int l = k & 63;
    return Gate2{read_lane(g.u00, l), read_lane(g.u01, l), read_lane(g.u10, l),
                 read_lane(g.u11, l)};
  }
};

// Register prefetch of one site tensor (Dl x 2 x Dr, storage type) so that its HBM/L2
// latency overlaps the factorisation of the current bond.
template <int S, typename T>
struct SitePrefetch {
  static constexpr int PF = (2 * S * S + kLayerThreads - 1) / kLayerThreads;
  static constexpr int SP = LayerShared<S, T>::SP;
  cx<T> v[PF];
  int Dl = 0, Dr = 0;
  __device__ __forceinline__ void load(const T* slot, int dl, int dr) {
    Dl = dl;
    Dr = dr;
    const FastDiv fd(Dr);
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int idx = threadIdx.x + i * kLayerThreads;
      if (idx < Dl * 2 * Dr) {
        const int row = fd.q(idx), b = fd.r(idx);
        v[i] = cx<T>{slot[2 * ((size_t)row * S + b)], slot[2 * ((size_t)row * S + b) + 1]};
      }
    }
  }
  __device__ __forceinline__ void commit(cx<T>* dst) const {
    const FastDiv fd(Dr);
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int idx = threadIdx.x + i * kLayerThreads;
      if (idx < Dl * 2 * Dr) dst[fd.q(idx) * SP + fd.r(idx)] = v[i];
    }
  }
};

template <int S, typename T>
__device__ __forceinline__ void store_tensor(T* slot, const cd* src, int Dl, int Dr) {
  constexpr int SP = LayerShared<S, T>::SP;
  const FastDiv fd(Dr);
  for (int idx = threadIdx.x; idx < Dl * 2 * Dr; idx += kLayerThreads) {
    const int row = fd.q(idx), b = fd.r(idx);
    store_c<T, double>(slot, (size_t)row * S + b, src[row * SP + b]);
  }
}

template <typename T>
__device__ __forceinline__ cd to_cd(cx<T> v) {
  return cd{(double)v.re, (double)v.im};
}

// Right-to-left sweep: apply the one-qubit gates (mode != kGateNone) and bring sites n-1..1
// to right-canonical form; the centre ends in ta as site 0.  dims(k) = bond k's dimension.
// With from_lds the tensor of site n-1 is already in ta (the end of a preceding CNOT sweep).
template <int S, typename T, typename Dims>
__device__ __forceinline__ int canon_sweep(LayerShared<S, T>& sh, T* st, int n, Dims dims, int mode,
                                           const double* theta, const double* phi,
                                           const double* pix, bool from_lds,
                                           SitePrefetch<S, T>& pf) {
  constexpr int LD = LayerShared<S, T>::LD;
  constexpr int SP = LayerShared<S, T>::SP;
  constexpr size_t SLOT = (size_t)2 * S * S * 2;  // T values per site slot
  const int tid = threadIdx.x;
  int flags = 0;
  if (!from_lds) {
    pf.load(st + (size_t)(n - 1) * SLOT, dims(n - 2), 1);
    pf.commit(sh.tb);
    wave_sync();
    for (int idx = tid; idx < dims(n - 2) * 2; idx += kLayerThreads) sh.ta[idx * SP] = to_cd(sh.tb[idx * SP]);
    wave_sync();
  }
  LaneGates lg;
  for (int k = n - 1; k >= 1; --k) {
    const int Dl = dims(k - 1), Dr = dims(k), Dll = dims(k - 2);
    pf.load(st + (size_t)(k - 1) * SLOT, Dll, Dl);
    if (mode != kGateNone) apply_gate<S, T>(sh, Dl, Dr, lg.get(mode, k, n, theta, phi, pix));
    // mat = t^H: rows (s, b) -> s*Dr + b, columns a.
    const int M = 2 * Dr, N = Dl;
    const FastDiv fm(M);
    for (int idx = tid; idx < N * M; idx += kLayerThreads) {
      const int a = fm.q(idx), rr = fm.r(idx);
      const int s_ = rr >= Dr, b = rr - (s_ ? Dr : 0);
      sh.mat[a * LD + rr] = cconj(sh.ta[(a * 2 + s_) * SP + b]);
    }
    wave_sync();
    // t = L Q: Q (right-canonical rows) goes to site k, L to uq.
    flags |= lq_columns<S, T, kHhCanon>(sh, M, N, N, Dr, st + (size_t)k * SLOT);
    pf.commit(sh.tb);
    wave_sync();
    // left neighbour times L: ta[row][a] = sum_j tb[row][j] uq[j][a]
    cgemm(
        1, Dll * 2, Dl, Dl, [&](int, int i, int j) { return to_cd(sh.tb[i * SP + j]); },
        [&](int, int j, int a) { return sh.uq[j * SP + a]; },
        [&](int, int i, int a, cd v) { sh.ta[i * SP + a] = v; });
    wave_sync();
  }
  if (mode != kGateNone) apply_gate<S, T>(sh, 1, dims(0), lg.get(mode, 0, n, theta, phi, pix));
  return flags;
}

// Jacobi SVD split of a CNOT bond whose left bond has grown (Dl > Dc), through the block
// factorisation of the two-site matrix: Theta'[(a,s),(t,b)] = sum_c C[a,s,c] B[c, t XOR s, b]
// = blockdiag(C_0, C_1) M with C_u = C[:, u, :] (Dl x Dc, the centre in ta) and
// M[(u,c),(t,b)] = B[c, t XOR u, b] (the neighbour in tb).  With C_u = Q_u R_u (two Householder
// blocks, FP64), Theta' = blockdiag(Q_0, Q_1) K, K = blockdiag(R_0, R_1) M (2Dc x 2Dr), and
// blockdiag(Q) has orthonormal columns, so Theta' and K have the same singular values and right
// singular vectors, and U_Theta = blockdiag(Q) U_K: the one-sided Jacobi runs on K, which has
// 2Dc instead of 2Dl rows.  The truncation, renormalisation and discarded weight are those of
// the SVD of Theta'.  Out: A[k] = blockdiag(Q) U_K in uq as [(a*2 + s)][j] (stored by the
// caller), the new centre U_K^H K / |sigma_kept| in ta as [j][t][b]; *terr (if not null) gets
// the discarded weight.  Needs 2Dr <= S (the products X_s below go to mat's columns >= 2Dr).
template <int S, typename T>
__device__ __forceinline__ int svd_split_block(LayerShared<S, T>& sh, int Dl, int Dc, int Dr, int D,
                                               double* terr) {
  constexpr int LD = LayerShared<S, T>::LD;
  constexpr int SP = LayerShared<S, T>::SP;
  const int tid = threadIdx.x;
  // C_u into mat's columns u*Dc + c (rows a), then C_u = Q_u R_u: Q_u -> ta, conj(R_u) -> uq.
  {
    const FastDiv fdl(Dl);
    for (int idx = tid; idx < 2 * Dc * Dl; idx += kLayerThreads) {
      const int col = fdl.q(idx), a = fdl.r(idx);
      const int u = col >= Dc, c = col - (u ? Dc : 0);
      sh.mat[col * LD + a] = sh.ta[(a * 2 + u) * SP + c];
    }
  }
  wave_sync();
  int flags = lq_columns<S, T, kHhBlockLds>(sh, Dl, 2 * Dc, Dc, 0, nullptr);
  // K[(u,c')][(t,b)] = sum_{c >= c'} R_u[c'][c] B[c][t XOR u][b] -> mat (column-major, rows
  // padded with zeros to the Jacobi tile's height).
  const int Mk = 2 * Dc, N = 2 * Dr;
  const int MP = jacobi_shape(Mk, N).MP;
  // One product per u; uq holds zeros below each R_u's diagonal, so the sum runs over all c.
  cgemm(
      2, Dc, N, Dc, [&](int u, int cp, int c) { return cconj(sh.uq[(u * Dc + c) * SP + cp]); },
      [&](int u, int c, int col) {
        const int t = col >= Dr, b = col - (t ? Dr : 0);
        return to_cd(sh.tb[(c * 2 + (t ^ u)) * SP + b]);
      },
      [&](int u, int cp, int col, cd v) { sh.mat[col * LD + u * Dc + cp] = v; });
  if (MP > Mk) {
    const int pad = MP - Mk;
    for (int idx = tid; idx < N * pad; idx += kLayerThreads)
      sh.mat[(idx / pad) * LD + Mk + idx % pad] = cd{0.0, 0.0};
  }
  wave_sync();
  flags |= jacobi_columns<S, T>(sh, Mk, N);
  const double tiny2 = sh.tiny2;
  // rank, column scales, kept and discarded weights (as in the direct split)
  double vk = 0.0, vd = 0.0;
  if (tid < N) {
    double v = sh.sig2[tid];
    if (!(v >= 0.0)) v = 0.0;
    int rk = 0;
    for (int i = 0; i < N; ++i) {
      double w = sh.sig2[i];
      if (!(w >= 0.0)) w = 0.0;
      rk += (w > v) || (w == v && i < tid);
    }
    sh.rank[rk] = tid;
    sh.isig[rk] = v > tiny2 ? rsqrt_full(v) : 0.0;
    if (rk < D) vk = v; else vd = v;
  }
  const double kept = wave_sum(vk), disc = wave_sum(vd);
  wave_sync();
  if (!isfinite(kept) || !isfinite(disc) || !(kept > 0.0)) flags |= kImgNonfinite;
  const double inv_norm = (kept > 0.0) ? rsqrt_full(kept) : 0.0;
  if (tid == 0 && terr) *terr = (kept + disc > 0.0) ? disc / (kept + disc) : 0.0;
  // X_s[j][c] = sum_{c' <= c} conj(U_K[(s,c')][j]) R_s[c'][c] -> xs[(s*D + j)*Dc + c]
  cd* xs = sh.mat + N * LD;
  cgemm(
      2, D, Dc, Dc, [&](int s_, int j, int cp) { return cconj(sh.mat[sh.rank[j] * LD + s_ * Dc + cp]); },
      [&](int s_, int cp, int c) { return cconj(sh.uq[(s_ * Dc + c) * SP + cp]); },
      [&](int s_, int j, int c, cd v) { xs[(s_ * D + j) * Dc + c] = cscale(v, sh.isig[j]); });
  wave_sync();
  // A[k][(a,s)][j] = sum_c' Q_s[a][c'] U_K[(s,c')][j] -> uq
  cgemm(
      2, Dl, D, Dc, [&](int s_, int a, int cp) { return sh.ta[a * SP + s_ * Dc + cp]; },
      [&](int s_, int cp, int j) { return sh.mat[sh.rank[j] * LD + s_ * Dc + cp]; },
      [&](int s_, int a, int j, cd v) { sh.uq[(a * 2 + s_) * SP + j] = cscale(v, sh.isig[j]); });
  wave_sync();
  // centre[j][(t,b)] = sum_s sum_c X_s[j][c] B[c][t XOR s][b] / |sigma_kept| -> ta, summation
  // index k = 2c + s
  cgemm(
      1, D, 2 * Dr, 2 * Dc, [&](int, int j, int k) { return xs[((k & 1) * D + j) * Dc + (k >> 1)]; },
      [&](int, int k, int o) {
        const int t = o >= Dr, b = o - (t ? Dr : 0);
        return to_cd(sh.tb[((k >> 1) * 2 + (t ^ (k & 1))) * SP + b]);
      },
      [&](int, int j, int o, cd v) {
        const int t = o >= Dr, b = o - (t ? Dr : 0);
        sh.ta[(j * 2 + t) * SP + b] = cscale(v, inv_norm);
      });
  wave_sync();
  return flags;
}

// Left-to-right two-site sweep starting from the centre (site 0) in ta.  Bond k gets a CNOT
// (control k) when parity < 0 or k % 2 == parity, else the update only moves the centre.
// before(k)/after(k) = bond dimensions before/after this sweep; bond k keeps after(k) singular
// triplets (for a CNOT bond min(chi, rows, cols, 2 before(k)), for a plain move before(k)).
// trunc_err[k] receives the discarded weight of every CNOT bond.
template <int S, typename T, typename Before, typename After>
__device__ __forceinline__ int cnot_sweep(LayerShared<S, T>& sh, T* st, int n, Before before,
                                          After after, int parity, double* trunc_err,
                                          SitePrefetch<S, T>& pf, int exact_qr) {
  constexpr int LD = LayerShared<S, T>::LD;
  constexpr int SP = LayerShared<S, T>::SP;
  constexpr size_t SLOT = (size_t)2 * S * S * 2;
  const int tid = threadIdx.x;
  int flags = 0;
  pf.load(st + (size_t)1 * SLOT, before(0), before(1));
  // A truncated bond's U stays in uq and is stored at the start of the next bond, after that
  // bond's wait for its prefetched neighbour: the wait for a load also waits for every store
  // issued before it, so the store is issued a whole bond before the next such wait.
  int pend_k = -1, pend_dl = 0, pend_d = 0;
  for (int k = 0; k <= n - 2; ++k) {
    const int Dl = after(k - 1), Dc = before(k), Dr = before(k + 1), D = after(k);
    const int cx = (parity < 0 || (k & 1) == parity) ? 1 : 0;
    pf.commit(sh.tb);
    wave_sync();
    if (pend_k >= 0) {
      store_tensor<S, T>(st + (size_t)pend_k * SLOT, sh.uq, pend_dl, pend_d);
      wave_sync();
      pend_k = -1;
    }
    if (k + 2 <= n - 1) pf.load(st + (size_t)(k + 2) * SLOT, before(k + 1), before(k + 2));
    if (exact_qr && ((cx && D == 2 * Dc && Dl >= Dc) || (!cx && D == Dc && 2 * Dl >= Dc))) {
      // The bond keeps every singular value of a factorisation with inner dimension D: split
      // it without the two-site matrix.  The centre is in canonical position, so the kept
      // weight is |centre|_F^2 (the CNOT is unitary, A[k+1] right-orthonormal).
      const double f = centre_norm2<S, T>(sh, Dl, Dc);
      if (!isfinite(f) || !(f > 0.0)) flags |= kImgNonfinite;
      const double scale = f > 0.0 ? rsqrt_full(f) : 0.0;
      if (cx) {
        const Gate2 none{};
        flags |= block_split<S, T>(sh, st + (size_t)k * SLOT, Dl, Dc, Dr, none, false, scale);
        if (tid == 0 && trunc_err) trunc_err[k] = 0.0;
      } else {
        flags |= plain_split<S, T>(sh, st + (size_t)k * SLOT, Dl, Dc, Dr, scale);
      }
      continue;
    }
    // The block route pays only where it shortens the Jacobi tile (fewer rows per lane); for
    // smaller matrices the direct split is cheaper than the extra factorisation and products.
    if (cx && Dl > Dc && 2 * Dr <= S &&
        jacobi_shape(2 * Dc, 2 * Dr).R < jacobi_shape(2 * Dl, 2 * Dr).R) {
      flags |= svd_split_block<S, T>(sh, Dl, Dc, Dr, D, trunc_err ? trunc_err + k : nullptr);
      pend_k = k;
      pend_dl = Dl;
      pend_d = D;
      continue;
    }
    const int M = 2 * Dl, N = 2 * Dr;
    const int MP = jacobi_shape(M, N).MP;
    // Theta'[(a,s),(t,b)] = sum_c A[k][a,s,c] A[k+1][c, t XOR (cx s), b]   (CNOT control k).
    // One product per s (rows (a, s) of Theta' = a*2 + s); the tile's padding rows are zero.
    cgemm(
        2, Dl, N, Dc, [&](int s_, int a, int c) { return sh.ta[(a * 2 + s_) * SP + c]; },
        [&](int s_, int c, int col) {
          const int t = col >= Dr, b = col - (t ? Dr : 0);
          return to_cd(sh.tb[(c * 2 + (t ^ (s_ & cx))) * SP + b]);
        },
        [&](int s_, int a, int col, cd v) { sh.mat[col * LD + a * 2 + s_] = v; });
    if (MP > M) {
      const int pad = MP - M;
      for (int idx = tid; idx < N * pad; idx += kLayerThreads)
        sh.mat[(idx / pad) * LD + M + idx % pad] = cd{0.0, 0.0};
    }
    wave_sync();
    if (exact_qr && D == (M < N ? M : N)) {
      // The bond keeps every singular value: the split needs no SVD (the centre is in canonical
      // position, so the kept weight is |Theta'|_F^2 and the discarded weight is 0).
      double f = 0.0;
      const FastDiv fm(M);
      for (int idx = tid; idx < N * M; idx += kLayerThreads) {
        const cd v = sh.mat[fm.q(idx) * LD + fm.r(idx)];
        f = fma(v.re, v.re, fma(v.im, v.im, f));
      }
      f = block_sum(f, sh.red);
      if (!isfinite(f) || !(f > 0.0)) flags |= kImgNonfinite;
      if (cx && tid == 0 && trunc_err) trunc_err[k] = 0.0;
      flags |= exact_split<S, T>(sh, st + (size_t)k * SLOT, M, N, D, Dr, f > 0.0 ? rsqrt_full(f) : 0.0);
      wave_sync();
      continue;
    }
    flags |= jacobi_columns<S, T>(sh, M, N);
    const double tiny2 = sh.tiny2;
    // Rank columns by singular value (descending, ties by index; NaN counts as zero); lane c
    // owns column c (N <= 2S <= 64), records the scale 1/|w_c| of its U column (0 for a
    // numerically zero column) under its rank, and the kept and discarded weights are wave sums.
    double vk = 0.0, vd = 0.0;
    if (tid < N) {
      double v = sh.sig2[tid];
      if (!(v >= 0.0)) v = 0.0;
      int rk = 0;
      for (int i = 0; i < N; ++i) {
        double w = sh.sig2[i];
        if (!(w >= 0.0)) w = 0.0;
        rk += (w > v) || (w == v && i < tid);
      }
      sh.rank[rk] = tid;
      sh.isig[rk] = v > tiny2 ? rsqrt_full(v) : 0.0;
      if (rk < D) vk = v; else vd = v;
    }
    const double kept = wave_sum(vk), disc = wave_sum(vd);
    wave_sync();
    if (!isfinite(kept) || !isfinite(disc) || !(kept > 0.0)) flags |= kImgNonfinite;
    const double inv_norm = (kept > 0.0) ? rsqrt_full(kept) : 0.0;
    if (cx && tid == 0 && trunc_err) trunc_err[k] = (kept + disc > 0.0) ? disc / (kept + disc) : 0.0;
    // U columns = normalised kept columns of W (numerically zero columns become zero).
    {
      const FastDiv fd(D);
      for (int idx = tid; idx < M * D; idx += kLayerThreads) {
        const int r = fd.q(idx), j = fd.r(idx);
        sh.uq[r * SP + j] = cscale(sh.mat[sh.rank[j] * LD + r], sh.isig[j]);
      }
    }
    wave_sync();
    pend_k = k;
    pend_dl = Dl;
    pend_d = D;
    // X_s = U_s^H A_s  ->  mat[(s*S + j)*SP + c]
    cgemm(
        2, D, Dc, Dl, [&](int s_, int j, int a) { return cconj(sh.uq[(a * 2 + s_) * SP + j]); },
        [&](int s_, int a, int c) { return sh.ta[(a * 2 + s_) * SP + c]; },
        [&](int s_, int j, int c, cd v) { sh.mat[(s_ * S + j) * SP + c] = v; });
    wave_sync();
    // New centre S V^H = U^H Theta' / |sigma_kept|  ->  ta[(j*2+t)*SP + b]; summation index
    // k = 2c + s over both X_s.
    cgemm(
        1, D, 2 * Dr, 2 * Dc, [&](int, int j, int k) { return sh.mat[((k & 1) * S + j) * SP + (k >> 1)]; },
        [&](int, int k, int o) {
          const int t = o >= Dr, b = o - (t ? Dr : 0);
          return to_cd(sh.tb[((k >> 1) * 2 + (t ^ ((k & 1) & cx))) * SP + b]);
        },
        [&](int, int j, int o, cd v) {
          const int t = o >= Dr, b = o - (t ? Dr : 0);
          sh.ta[(j * 2 + t) * SP + b] = cscale(v, inv_norm);
        });
    wave_sync();
  }
  if (pend_k >= 0) store_tensor<S, T>(st + (size_t)pend_k * SLOT, sh.uq, pend_dl, pend_d);
  store_tensor<S, T>(st + (size_t)(n - 1) * SLOT, sh.ta, after(n - 2), 1);
  return flags;
}

// Exact split of a two-site matrix Theta' (mat, M x N, column index t*Dr + b) that keeps all its
// D = min(M, N) singular values: when D = M, A[k] <- the identity and the centre <- Theta';
// otherwise (D = N < M) Theta' = Q R by Householder, A[k] <- Q and the centre <- R.  The
// centre (ta, [j][t][b]) is multiplied by `scale`.
template <int S, typename T>
__device__ __forceinline__ int exact_split(LayerShared<S, T>& sh, T* slot, int M, int N, int D,
                                           int Dr, double scale) {
  constexpr int LD = LayerShared<S, T>::LD;
  constexpr int SP = LayerShared<S, T>::SP;
  const int tid = threadIdx.x;
  int flags = 0;
  const FastDiv fn(N);
  if (D == M) {
    const FastDiv fmm(M);
    for (int idx = tid; idx < M * M; idx += kLayerThreads) {
      const int row = fmm.q(idx), j = fmm.r(idx);
      store_c<T, double>(slot, (size_t)row * S + j, cd{row == j ? 1.0 : 0.0, 0.0});
    }
    for (int idx = tid; idx < D * N; idx += kLayerThreads) {
      const int j = fn.q(idx), col = fn.r(idx);
      const int t = col >= Dr, b = col - (t ? Dr : 0);
      sh.ta[(j * 2 + t) * SP + b] = cscale(sh.mat[col * LD + j], scale);
    }
  } else {
    flags |= lq_columns<S, T, kHhLadder>(sh, M, N, N, Dr, slot);
    for (int idx = tid; idx < D * N; idx += kLayerThreads) {
      const int j = fn.q(idx), col = fn.r(idx);
      const int t = col >= Dr, b = col - (t ? Dr : 0);
      sh.ta[(j * 2 + t) * SP + b] = j <= col ? cscale(cconj(sh.uq[col * SP + j]), scale) : cd{0.0, 0.0};
    }
  }
  return flags;
}

// Split of a CNOT bond through its rank-2Dc factorisation, exact when the bond keeps D = 2 Dc
// values and Dl >= Dc: Theta'[(a,s),(t,b)] = sum_c ta[a,s,c] (U B)[c, t XOR s, b] factors as
// blockdiag(ta_0, ta_1) times [(U B)[c, t XOR u, b]] with ta_u = ta[:, u, :] (Dl x Dc), so
// ta_u = Q_u R_u (two independent Householder blocks) gives A[k][(a,s)][(u,c')] = Q_s[a][c']
// (zero for s != u) and centre[(u,c')][(t,b)] = sum_c R_u[c'][c] (U B)[c][t XOR u][b] -- no
// two-site matrix and half the Householder steps.  U = the one-qubit gate of site k+1 when
// `gate` (else the identity); the centre is multiplied by `scale`.
template <int S, typename T>
__device__ __forceinline__ int block_split(LayerShared<S, T>& sh, T* slot, int Dl, int Dc, int Dr,
                                           const Gate2& g, bool gate, double scale) {
  constexpr int LD = LayerShared<S, T>::LD;
  constexpr int SP = LayerShared<S, T>::SP;
  const int tid = threadIdx.x;
  // 2 Dc = D <= S, so mat's columns [S, 2S) are free during the QR: the neighbour (gated in
  // FP64 when `gate`) goes there as gb[(c*2 + t)*SP + b].
  cd* gb = sh.mat + S * LD;
  {
    const FastDiv fdl(Dl);
    for (int idx = tid; idx < 2 * Dc * Dl; idx += kLayerThreads) {
      const int col = fdl.q(idx), a = fdl.r(idx);
      const int u = col >= Dc, c = col - (u ? Dc : 0);
      sh.mat[col * LD + a] = sh.ta[(a * 2 + u) * SP + c];
    }
    const FastDiv fdr(Dr);
    for (int idx = tid; idx < Dc * Dr; idx += kLayerThreads) {
      const int c = fdr.q(idx), b = fdr.r(idx);
      const cd b0 = to_cd(sh.tb[(c * 2) * SP + b]), b1 = to_cd(sh.tb[(c * 2 + 1) * SP + b]);
      if (gate) {
        cd w0 = cmul(g.u00, b0), w1 = cmul(g.u10, b0);
        cfma(w0, g.u01, b1);
        cfma(w1, g.u11, b1);
        gb[(c * 2) * SP + b] = w0;
        gb[(c * 2 + 1) * SP + b] = w1;
      } else {
        gb[(c * 2) * SP + b] = b0;
        gb[(c * 2 + 1) * SP + b] = b1;
      }
    }
  }
  wave_sync();
  int flags = lq_columns<S, T, kHhBlock2>(sh, Dl, 2 * Dc, Dc, 0, slot);
  const FastDiv f2r(2 * Dr);
  for (int idx = tid; idx < 2 * Dc * 2 * Dr; idx += kLayerThreads) {
    const int j = f2r.q(idx), o = f2r.r(idx);
    const int t = o >= Dr, b = o - (t ? Dr : 0);
    const int u = j >= Dc, cp = j - (u ? Dc : 0), tt = t ^ u;
    cd acc{0.0, 0.0};
    for (int c = cp; c < Dc; ++c) cfma(acc, cconj(sh.uq[(u * Dc + c) * SP + cp]), gb[(c * 2 + tt) * SP + b]);
    sh.ta[(j * 2 + t) * SP + b] = cscale(acc, scale);
  }
  wave_sync();
  return flags;
}

// Centre move without a gate, exact when the bond keeps D = Dc values and 2 Dl >= Dc: the
// centre (2Dl x Dc) = Q R, A[k] <- Q, centre <- R A[k+1] (times `scale`).
template <int S, typename T>
__device__ __forceinline__ int plain_split(LayerShared<S, T>& sh, T* slot, int Dl, int Dc, int Dr,
                                           double scale) {
  constexpr int LD = LayerShared<S, T>::LD;
  constexpr int SP = LayerShared<S, T>::SP;
  const int tid = threadIdx.x;
  const int M = 2 * Dl;
  {
    const FastDiv fm(M);
    for (int idx = tid; idx < Dc * M; idx += kLayerThreads) {
      const int c = fm.q(idx), row = fm.r(idx);
      sh.mat[c * LD + row] = sh.ta[row * SP + c];
    }
  }
  wave_sync();
  int flags = lq_columns<S, T, kHhLadder>(sh, M, Dc, Dc, 0, slot);
  const FastDiv f2r(2 * Dr);
  for (int idx = tid; idx < Dc * 2 * Dr; idx += kLayerThreads) {
    const int j = f2r.q(idx), o = f2r.r(idx);
    const int t = o >= Dr, b = o - (t ? Dr : 0);
    cd acc{0.0, 0.0};
    for (int c = j; c < Dc; ++c) cfma(acc, cconj(sh.uq[c * SP + j]), to_cd(sh.tb[(c * 2 + t) * SP + b]));
    sh.ta[(j * 2 + t) * SP + b] = cscale(acc, scale);
  }
  wave_sync();
  return flags;
}

// |ta|_F^2 of a (Dl x 2 x Dc) centre.
template <int S, typename T>
__device__ __forceinline__ double centre_norm2(LayerShared<S, T>& sh, int Dl, int Dc) {
  constexpr int SP = LayerShared<S, T>::SP;
  double f = 0.0;
  const FastDiv fdc(Dc);
  for (int idx = threadIdx.x; idx < 2 * Dl * Dc; idx += kLayerThreads) {
    const cd v = sh.ta[fdc.q(idx) * SP + fdc.r(idx)];
    f = fma(v.re, v.re, fma(v.im, v.im, f));
  }
  return block_sum(f, sh.red);
}

// True when layer `layer` of the CNOT-ladder circuit keeps every singular value at every bond:
// the bond rule gives D_k = min(rows, cols) of each two-site matrix, so no weight can be
// discarded and the split of each bond is exact whatever factorisation is used.
__host__ __device__ inline bool layer_keeps_all(int n, int chi, int layer) {
  for (int k = 0; k <= n - 2; ++k) {
    const int M = 2 * bond_dim(n, chi, layer + 1, k - 1), N = 2 * bond_dim(n, chi, layer, k + 1);
    if (bond_dim(n, chi, layer + 1, k) != (M < N ? M : N)) return false;
  }
  return true;
}

// True when the layer after `layer` truncates (within the batch's n_layers).  The last exact
// layer before it then takes the QR sweep rather than the parity-operator contraction: the
// truncating layer's Jacobi SVDs converge in fewer sweeps from the canonical gauge the QR sweep
// leaves (measured: 7x7, L = 4, chi = 8, and the chi = 64 sweep cell at L = 7).
__host__ __device__ inline bool next_truncates(int n, int chi, int layer, int n_layers) {
  return layer + 1 < n_layers && !layer_keeps_all(n, chi, layer + 1);
}

// A ladder layer without truncation (layer_keeps_all): one left-to-right sweep.  Site 0 takes
// its gate in FP64, then for each bond k the gated neighbour U_{k+1} A[k+1] (the gate commutes
// with the CNOTs on the bonds to its left) is contracted with the centre into
// Theta'[(a,s),(t,b)] = sum_c A[k][a,s,c] (U A[k+1])[c, t XOR s, b] and split exactly: when
// D = rows, A[k] <- the identity and the centre <- Theta'; when D = cols (< rows),
// Theta' = Q R by Householder, A[k] <- Q and the centre <- R.  Every A[k] is left-orthonormal,
// no canonical sweep is needed, the discarded weight of each bond is 0, and the last centre is
// scaled to unit norm.  The state equals the one the canonical sweep + SVD ladder produces,
// up to rounding and the gauge of each bond.
template <int S, typename T, typename Before, typename After>
__device__ __forceinline__ int qr_sweep(LayerShared<S, T>& sh, T* st, int n, Before before,
                                        After after, const double* theta, const double* phi,
                                        double* trunc_err, SitePrefetch<S, T>& pf) {
  constexpr int LD = LayerShared<S, T>::LD;
  constexpr int SP = LayerShared<S, T>::SP;
  constexpr size_t SLOT = (size_t)2 * S * S * 2;
  const int tid = threadIdx.x;
  int flags = 0;
  pf.load(st, 1, before(0));
  pf.commit(sh.tb);
  wave_sync();
  pf.load(st + SLOT, before(0), before(1));
  for (int idx = tid; idx < 2 * before(0); idx += kLayerThreads) {
    const int s_ = idx / before(0), c = idx - s_ * before(0);
    sh.ta[s_ * SP + c] = to_cd(sh.tb[s_ * SP + c]);
  }
  wave_sync();
  apply_gate<S, T>(sh, 1, before(0), site_gate(kGateRyRz, 0, theta, phi, nullptr));
  for (int k = 0; k <= n - 2; ++k) {
    const int Dl = after(k - 1), Dc = before(k), Dr = before(k + 1), D = after(k);
    pf.commit(sh.tb);
    wave_sync();
    if (k + 2 <= n - 1) pf.load(st + (size_t)(k + 2) * SLOT, before(k + 1), before(k + 2));
    if (D == 2 * Dc && Dl >= Dc) {
      flags |= block_split<S, T>(sh, st + (size_t)k * SLOT, Dl, Dc, Dr,
                                 site_gate(kGateRyRz, k + 1, theta, phi, nullptr), true, 1.0);
      if (tid == 0 && trunc_err) trunc_err[k] = 0.0;
      continue;
    }
    // gated neighbour in FP64: uq[(c*2 + t)*SP + b]
    {
      const Gate2 g = site_gate(kGateRyRz, k + 1, theta, phi, nullptr);
      const FastDiv fdr(Dr);
      for (int idx = tid; idx < Dc * Dr; idx += kLayerThreads) {
        const int c = fdr.q(idx), b = fdr.r(idx);
        const cd v0 = to_cd(sh.tb[(c * 2) * SP + b]), v1 = to_cd(sh.tb[(c * 2 + 1) * SP + b]);
        cd w0 = cmul(g.u00, v0), w1 = cmul(g.u10, v0);
        cfma(w0, g.u01, v1);
        cfma(w1, g.u11, v1);
        sh.uq[(c * 2) * SP + b] = w0;
        sh.uq[(c * 2 + 1) * SP + b] = w1;
      }
    }
    wave_sync();
    const int M = 2 * Dl, N = 2 * Dr;
    {
      const FastDiv fm(M), fdr(Dr);
      for (int idx = tid; idx < N * M; idx += kLayerThreads) {
        const int col = fm.q(idx), row = fm.r(idx);
        const int t = col >= Dr, b = col - (t ? Dr : 0), s_ = row & 1;
        cd acc{0.0, 0.0};
        for (int c = 0; c < Dc; ++c) cfma(acc, sh.ta[row * SP + c], sh.uq[(c * 2 + (t ^ s_)) * SP + b]);
        sh.mat[col * LD + row] = acc;
      }
    }
    wave_sync();
    flags |= exact_split<S, T>(sh, st + (size_t)k * SLOT, M, N, D, Dr, 1.0);
    if (tid == 0 && trunc_err) trunc_err[k] = 0.0;
    wave_sync();
  }
  const int Dn = after(n - 2);
  double f = 0.0;
  for (int idx = tid; idx < 2 * Dn; idx += kLayerThreads) {
    const cd v = sh.ta[idx * SP];
    f = fma(v.re, v.re, fma(v.im, v.im, f));
  }
  f = block_sum(f, sh.red);
  if (!isfinite(f) || !(f > 0.0)) flags |= kImgNonfinite;
  const double scale = f > 0.0 ? rsqrt_full(f) : 0.0;
  for (int idx = tid; idx < 2 * Dn; idx += kLayerThreads) sh.ta[idx * SP] = cscale(sh.ta[idx * SP], scale);
  wave_sync();
  store_tensor<S, T>(st + (size_t)(n - 1) * SLOT, sh.ta, Dn, 1);
  return flags;
}

// ----------------------------------------------------------------- exact layers as one contraction
// The CNOT ladder CNOT(n-2, n-1) ... CNOT(0, 1) maps |x_0 x_1 ...> to |y_0 y_1 ...> with
// y_k = x_0 XOR ... XOR x_k, a matrix product operator of bond dimension 2 whose bond carries
// the running parity: site k reads the parity p of its left bond, emits y = x XOR p and passes
// q = y on.  With the one-qubit gate U_k in front, the exact layer on the MPS is, site by site,
//   B[k][(p,a), y, (q,b)] = (U_k A[k])[a, y XOR p, b] * delta(q, y)
// (no p at site 0, no q at site n-1), a tensor of bonds 2 D^old: nothing couples two sites.
// Where the bond rule keeps D_k < 2 D_k^old the doubled bond is reduced exactly at the chain
// ends: on a prefix of bonds with D_k = 2 D_{k-1} the sites become identities
// (A[k][a, s, 2a+s] = 1) and the product of the B's is carried into the next site; on a suffix
// with D_k = 2 D_{k+1} the sites become identities A[k][s D_k + b, s, b] = 1 and the product is
// carried left.  Every bond between keeps D_k = 2 D_k^old.
constexpr int kXcds = 8;

struct MpoPlan {
  int kl, kr;  // bonds 0..kl reduced from the left, kr..n-2 from the right
};

// True when the bond rule of the layer has that shape (which holds exactly when the layer
// keeps every singular value); fills the two ends.
template <typename Before, typename After>
__host__ __device__ inline bool mpo_plan(int n, Before dold, After dnew, MpoPlan& p) {
  int kl = -1;
  while (kl + 1 <= n - 2 && dnew(kl + 1) < 2 * dold(kl + 1) && dnew(kl + 1) == 2 * dnew(kl)) ++kl;
  int kr = n - 1;
  while (kr - 1 > kl && dnew(kr - 1) < 2 * dold(kr - 1) && dnew(kr - 1) == 2 * dnew(kr)) --kr;
  for (int k = kl + 1; k < kr; ++k)
    if (dnew(k) != 2 * dold(k)) return false;
  p.kl = kl;
  p.kr = kr;
  return true;
}

// (U A)[a, t, b] of an old site tensor read through at(a, s, b).
template <typename At>
__device__ __forceinline__ cd gated_at(const At& at, const Gate2& g, int a, int t, int b) {
  const cd v0 = at(a, 0, b), v1 = at(a, 1, b);
  cd w = cmul(t ? g.u10 : g.u00, v0);
  cfma(w, t ? g.u11 : g.u01, v1);
  return w;
}

__device__ __forceinline__ bool finite_c(cd v) { return isfinite(v.re) && isfinite(v.im); }

// LDS ordering of the one-wavefront workgroups (see wave_sync).
__device__ __forceinline__ void lds_sync() { wave_sync(); }

// The bit a site passes to its right bond.  Ladder: its output y.  The paper's brickwork layer
// (§II-B, Eq. (2); CNOTs on the even bonds, then on the odd ones), written the same way with
// one bit per bond: an odd site k is the target of CNOT(k-1, k) and the control of
// CNOT(k, k+1), so it outputs y = x XOR p and passes y; an even site is the control of
// CNOT(k, k+1) (passing its input x) and then the target of CNOT(k-1, k), so it outputs
// y = x XOR p and passes x = y XOR p.  The gates U_k are applied first in both programs.
__device__ __forceinline__ int mpo_bit(int k, int y, int p, bool brick) {
  return (brick && !(k & 1)) ? (y ^ p) : y;
}

// A site between the reduced ends: A[k] <- B[k] (bonds 2 Dp x 2 x 2 Do), written to `slot` by
// `nthreads` lanes; the old tensor is read through `at` from a staged copy, so the slot may be
// overwritten.  Returns true if a value is not finite.
template <int S, typename T, typename At>
__device__ __forceinline__ bool mpo_plain_site(const At& at, const Gate2& g, int Dp, int Do, T* slot,
                                               int lane, int nthreads, int k = 1,
                                               bool brick = false) {
  bool bad = false;
  const int R = 2 * Do;
  const FastDiv fr(R), fdp(Dp), fdo(Do);
  for (int idx = lane; idx < 4 * Dp * R; idx += nthreads) {
    const int row = fr.q(idx), m = fr.r(idx), i = row >> 1, y = row & 1;
    const int p = fdp.q(i), a = fdp.r(i), q = fdo.q(m), b = fdo.r(m);
    const cd v = (q == mpo_bit(k, y, p, brick)) ? gated_at(at, g, a, y ^ p, b) : cd{0.0, 0.0};
    bad |= !finite_c(v);
    store_c<T, double>(slot, (size_t)row * S + m, v);
  }
  return bad;
}

// The reduced ends and the sites that receive their carries (FP64 carries in LDS):
//  part 0: the left end, and the right end too when both carries land on one site;
//  part 1: the right end (nothing when both carries land on one site);
//  part 2: both ends.
// The next site's load overlaps each carry step, and the identity tensors are stored after the
// last load, so that no step waits for earlier stores.  Returns true if a value is not finite.
// LDS of the end carries: left carry ping-pong c[2] (S x 2S each, the free one also holds the
// carry site's product), right carry ping-pong r[2] (2S x S each), the staged old tensor tb.
// A part that does not take an end may leave its two pointers null.
template <typename T>
struct MpoBufs {
  cd* c[2];
  cd* r[2];
  cx<T>* tb;
};

template <int S, typename T>
__device__ __forceinline__ MpoBufs<T> mpo_bufs(LayerShared<S, T>& sh) {
  return MpoBufs<T>{{sh.mat, sh.mat + S * 2 * S}, {sh.uq, sh.ta}, sh.tb};
}

// Stage: how the old site tensor reaches tb (SitePrefetch: registers, loaded ahead; for slots
// wider than 16, WideStage: a direct copy).  GLOBAL_BUFS: the carries and tb live in global
// memory (the wide slots' workspace), so steps are ordered with a full barrier, whose fence
// makes the lanes' global stores visible, instead of an LDS-only wait.
template <int S, typename T, typename Before, typename After, typename Stage = SitePrefetch<S, T>,
          bool GLOBAL_BUFS = false>
__device__ bool mpo_ends(const MpoBufs<T>& bufs, T* st, int n, Before dold, After dnew,
                         const MpoPlan& plan, const double* theta, const double* phi,
                         Stage& pf, int part, int gmode = kGateRyRz,
                         const double* pix = nullptr, bool brick = false, int extra_lo = 0,
                         int extra_hi = -1) {
  constexpr size_t SLOT = (size_t)2 * S * S * 2;
  constexpr int CS = 2 * S;  // row stride of the left carry (columns <= 2 S)
  constexpr int SP = LayerShared<S, T>::SP;
  const int tid = threadIdx.x, kl = plan.kl, kr = plan.kr;
  auto step_sync = [] {
    if constexpr (GLOBAL_BUFS) {
      __syncthreads();
    } else {
      lds_sync();
    }
  };
  const bool meet = kl + 1 == kr;
  if (part == 1 && meet) return false;
  const bool do_left = part != 1, do_right = part != 0 || meet;
  // MPO bond size on the left of site k: 2 D_{k-1}^old (1 at site 0).
  auto lm = [&](int k) { return k == 0 ? 1 : 2 * dold(k - 1); };
  cx<T>* tb = bufs.tb;
  auto at = [&](int a, int s_, int b) { return to_cd(tb[(a * 2 + s_) * SP + b]); };
  // Visiting order: left chain 0..kl, right chain n-1..kr+1, the carry sites, then the plain
  // sites extra_lo..extra_hi (sites between the ends that the caller hands to this part).
  const int nl = do_left ? kl + 1 : 0, nr = do_right ? n - 1 - kr : 0;
  const bool two = do_left && do_right && !meet;
  const int ncarry = nl + nr + (two ? 2 : 1);
  const int total = ncarry + (extra_hi >= extra_lo ? extra_hi - extra_lo + 1 : 0);
  auto site_at = [&](int t) {
    if (t < nl) return t;
    if (t < nl + nr) return n - 1 - (t - nl);
    if (t >= ncarry) return extra_lo + (t - ncarry);
    return (t == nl + nr && do_left) ? kl + 1 : kr;
  };
  cd* const c0 = bufs.c[0];
  cd* const c1 = bufs.c[1];
  cd* const r0 = bufs.r[0];
  cd* const r1 = bufs.r[1];
  auto cbuf = [&](int i) { return i ? c1 : c0; };
  auto rbuf = [&](int i) { return i ? r1 : r0; };
  int cur = 0, rcur = 0;
  if (tid == 0) {
    if (do_left) c0[0] = cd{1.0, 0.0};
    if (do_right) r0[0] = cd{1.0, 0.0};
  }
  bool bad = false;
  // Sites are loaded two steps ahead (pf: the next step's site, pf2: the one after), and the next
  // site's gate is computed while this step runs: each step is short next to a load's latency.
  Stage pf2 = pf;
  pf.load(st + (size_t)site_at(0) * SLOT, dold(site_at(0) - 1), dold(site_at(0)));
  if (total > 1) pf2.load(st + (size_t)site_at(1) * SLOT, dold(site_at(1) - 1), dold(site_at(1)));
  Gate2 gnext = site_gate(gmode, site_at(0), theta, phi, pix);
  for (int t = 0; t < total; ++t) {
    const int k = site_at(t);
    pf.commit(tb);
    step_sync();
    const Gate2 g = gnext;
    pf = pf2;
    if (t + 2 < total) {
      const int kn = site_at(t + 2);
      pf2.load(st + (size_t)kn * SLOT, dold(kn - 1), dold(kn));
    }
    if (t + 1 < total) gnext = site_gate(gmode, site_at(t + 1), theta, phi, pix);
    const int Dp = dold(k - 1), Do = dold(k), L = lm(k);
    const FastDiv fdp(Dp), fdo(Do);
    if (t < nl) {
      // C_k[2a+s][(q,b)] = sum_i C_{k-1}[a][i] B[k][i, s, (q,b)]
      const int rows = dnew(k - 1), R = 2 * Do;
      const FastDiv fr(R);
      const cd* C = cbuf(cur);
      cd* Cn = cbuf(cur ^ 1);
      for (int idx = tid; idx < rows * 2 * R; idx += kLayerThreads) {
        const int row = fr.q(idx), m = fr.r(idx), a = row >> 1, s_ = row & 1;
        const int q = fdo.q(m), b = fdo.r(m);
        cd acc{0.0, 0.0};
        for (int i = 0; i < L; ++i) {
          const int p = fdp.q(i);
          if (q == mpo_bit(k, s_, p, brick)) cfma(acc, C[a * CS + i], gated_at(at, g, fdp.r(i), s_ ^ p, b));
        }
        Cn[row * CS + m] = acc;
      }
      cur ^= 1;
    } else if (t < nl + nr) {
      // R_k[i][s D_k + b] = sum_b' B[k][i, s, (q,b')] R_{k+1}[(q,b')][b], q = the site's bit
      const int Dn = dnew(k), cols = 2 * Dn;
      const FastDiv fc(cols), fdn(Dn);
      const cd* Rk = rbuf(rcur);
      cd* Rn = rbuf(rcur ^ 1);
      for (int idx = tid; idx < L * cols; idx += kLayerThreads) {
        const int i = fc.q(idx), f = fc.r(idx), s_ = fdn.q(f), b = fdn.r(f);
        const int p = fdp.q(i), a = fdp.r(i);
        cd acc{0.0, 0.0};
        const int q = mpo_bit(k, s_, p, brick);
        for (int bp = 0; bp < Do; ++bp) {
          const int mrow = (k == n - 1) ? bp : q * Do + bp;
          cfma(acc, gated_at(at, g, a, s_ ^ p, bp), Rk[mrow * S + b]);
        }
        Rn[i * S + f] = acc;
      }
      rcur ^= 1;
    } else if (t >= ncarry) {
      bad |= mpo_plain_site<S, T>(at, g, Dp, Do, st + (size_t)k * SLOT, tid, kLayerThreads, k,
                                  brick);
    } else {
      // a carry site: C B[k] when k = kl+1 (left end), B[k] R when k = kr (right end)
      const bool lc = do_left && k == kl + 1, rc = do_right && k == kr;
      const cd* C = cbuf(cur);
      const cd* Rc = rbuf(rcur);
      T* slot = st + (size_t)k * SLOT;
      const int R = (k == n - 1) ? 1 : 2 * Do;
      // B[k][i, y, m], zero off its bit's delta
      auto bel = [&](int i, int y, int m) -> cd {
        const int p = fdp.q(i), a = fdp.r(i);
        if (k == n - 1) return gated_at(at, g, a, y ^ p, m);
        return fdo.q(m) == mpo_bit(k, y, p, brick) ? gated_at(at, g, a, y ^ p, fdo.r(m))
                                                    : cd{0.0, 0.0};
      };
      if (lc && rc) {
        // both carries land here (short chains of the ladder): V = C B[k] in the free left
        // buffer ([D_kl][2][D_k^old]; its bit is y), then V R
        cd* V = cbuf(cur ^ 1);
        const int rows = dnew(kl), cols = dnew(kr);
        const FastDiv f2o(2 * Do), fc(cols);
        for (int idx = tid; idx < rows * 2 * Do; idx += kLayerThreads) {
          const int an = f2o.q(idx), r2 = f2o.r(idx), y = fdo.q(r2), bp = fdo.r(r2);
          cd acc{0.0, 0.0};
          for (int i = 0; i < L; ++i) cfma(acc, C[an * CS + i], gated_at(at, g, fdp.r(i), y ^ fdp.q(i), bp));
          V[idx] = acc;
        }
        step_sync();
        for (int idx = tid; idx < rows * 2 * cols; idx += kLayerThreads) {
          const int row = fc.q(idx), j = fc.r(idx), r = row >> 1, y = row & 1;
          cd acc{0.0, 0.0};
          for (int bp = 0; bp < Do; ++bp) {
            const int mrow = (k == n - 1) ? bp : y * Do + bp;
            cfma(acc, V[(r * 2 + y) * Do + bp], Rc[mrow * S + j]);
          }
          bad |= !finite_c(acc);
          store_c<T, double>(slot, (size_t)row * S + j, acc);
        }
      } else if (lc) {
        const int rows = dnew(kl);
        const FastDiv fr(R);
        for (int idx = tid; idx < rows * 2 * R; idx += kLayerThreads) {
          const int row = fr.q(idx), m = fr.r(idx), r = row >> 1, y = row & 1;
          cd acc{0.0, 0.0};
          for (int i = 0; i < L; ++i) cfma(acc, C[r * CS + i], bel(i, y, m));
          bad |= !finite_c(acc);
          store_c<T, double>(slot, (size_t)row * S + m, acc);
        }
      } else {
        // rows are B's left index i = (p, a)
        const int cols = dnew(kr);
        const FastDiv fc(cols);
        for (int idx = tid; idx < L * 2 * cols; idx += kLayerThreads) {
          const int row = fc.q(idx), j = fc.r(idx), i = row >> 1, y = row & 1;
          const int p = fdp.q(i), a = fdp.r(i), q = mpo_bit(k, y, p, brick);
          cd acc{0.0, 0.0};
          for (int bp = 0; bp < Do; ++bp) {
            const int mrow = (k == n - 1) ? bp : q * Do + bp;
            cfma(acc, gated_at(at, g, a, y ^ p, bp), Rc[mrow * S + j]);
          }
          bad |= !finite_c(acc);
          store_c<T, double>(slot, (size_t)row * S + j, acc);
        }
      }
    }
    step_sync();
  }
  // identity tensors of the reduced sites
  for (int k = 0; k < nl; ++k) {
    const int D = dnew(k);
    for (int idx = tid; idx < D * D; idx += kLayerThreads) {
      const int row = idx / D, col = idx - row * D;
      store_c<T, double>(st + (size_t)k * SLOT, (size_t)row * S + col, cd{row == col ? 1.0 : 0.0, 0.0});
    }
  }
  for (int k = n - 1; k > n - 1 - nr; --k) {
    const int Dn = dnew(k), rows = 4 * Dn;
    for (int idx = tid; idx < rows * Dn; idx += kLayerThreads) {
      const int row = idx / Dn, b = idx - row * Dn, j = row >> 1, s_ = row & 1;
      store_c<T, double>(st + (size_t)k * SLOT, (size_t)row * S + b, cd{j == s_ * Dn + b ? 1.0 : 0.0, 0.0});
    }
  }
  return bad;
}

// One wavefront applies a whole exact layer: both ends, then the sites between.  The result is
// the exact state (up to rounding) in the gauge of the contraction: no site is orthonormalised
// and the norm is the input's (the layer is unitary); trunc_err is 0.
template <int S, typename T, typename Before, typename After>
__device__ int mpo_layer(LayerShared<S, T>& sh, T* st, int n, Before dold, After dnew,
                         const MpoPlan& plan, const double* theta, const double* phi,
                         double* trunc_err, SitePrefetch<S, T>& pf) {
  constexpr size_t SLOT = (size_t)2 * S * S * 2;
  constexpr int SP = LayerShared<S, T>::SP;
  const int tid = threadIdx.x;
  if (trunc_err)
    for (int k = tid; k < n - 1; k += kLayerThreads) trunc_err[k] = 0.0;
  bool bad = mpo_ends<S, T>(mpo_bufs(sh), st, n, dold, dnew, plan, theta, phi, pf, 2);
  auto at = [&](int a, int s_, int b) { return to_cd(sh.tb[(a * 2 + s_) * SP + b]); };
  const int k0 = plan.kl + 2, k1 = plan.kr - 1;
  if (k0 <= k1) pf.load(st + (size_t)k0 * SLOT, dold(k0 - 1), dold(k0));
  for (int k = k0; k <= k1; ++k) {
    pf.commit(sh.tb);
    lds_sync();
    if (k + 1 <= k1) pf.load(st + (size_t)(k + 1) * SLOT, dold(k), dold(k + 1));
    bad |= mpo_plain_site<S, T>(at, site_gate(kGateRyRz, k, theta, phi, nullptr), dold(k - 1),
                                dold(k), st + (size_t)k * SLOT, tid, kLayerThreads);
    lds_sync();
  }
  return __any(bad) ? kImgNonfinite : 0;
}

// Applies layer `layer` (0-based) to one image whose n slots start at `st`.
//  program kLayerRyRzLadder: R_Y(theta_k) R_Z(phi_k) on every site, then CNOT(k, k+1) for
//    k = 0..n-2 in order: one canonical sweep and one CNOT sweep.
//  program kLayerHRyBrickwork (§II-B, Eq. (2)): R_Y(2 pi x_k - pi) H on every site from the
//    image's pixels, then CNOTs on the even bonds, then on the odd bonds: canonical sweep (with
//    gates), even sweep, canonical sweep, odd sweep.  Between the two halves the even bonds are
//    at the new dimensions and the odd ones at the old.
enum : int { kLayerRyRzLadder = 0, kLayerHRyBrickwork = 1 };

// WITH_MPO: the one-wavefront form of a layer applied as the parity product operator.  The
// batched kernel leaves it out (the host sends such layers to k_mpo_ends / k_mpo_sites), which
// keeps its register allocation that of the SVD and QR paths.
template <int S, typename T, bool WITH_MPO>
__device__ __forceinline__ void layer_chain(LayerShared<S, T>& sh, T* st, int n, int chi, int layer,
                                            int program, const double* theta, const double* phi,
                                            const double* pix, double* trunc_err, int* status,
                                            int exact_qr, int n_layers) {
  auto dold = [&](int k) { return bond_dim(n, chi, layer, k); };
  auto dnew = [&](int k) { return bond_dim(n, chi, layer + 1, k); };
  SitePrefetch<S, T> pf;
  int flags = 0;
  if (program == kLayerHRyBrickwork) {
    auto dmid = [&](int k) { return bond_dim(n, chi, (k & 1) ? layer : layer + 1, k); };
    flags |= canon_sweep<S, T>(sh, st, n, dold, kGateHRy, theta, phi, pix, false, pf);
    __syncthreads();  // each sweep's global stores are read back by the next sweep
    flags |= cnot_sweep<S, T>(sh, st, n, dold, dmid, 0, trunc_err, pf, exact_qr);
    __syncthreads();
    flags |= canon_sweep<S, T>(sh, st, n, dmid, kGateNone, theta, phi, pix, true, pf);
    __syncthreads();
    flags |= cnot_sweep<S, T>(sh, st, n, dmid, dnew, 1, trunc_err, pf, exact_qr);
  } else if (exact_qr && layer_keeps_all(n, chi, layer)) {
    MpoPlan plan;
    if (WITH_MPO && exact_qr == kExactMpo && !next_truncates(n, chi, layer, n_layers) &&
        mpo_plan(n, dold, dnew, plan))
      flags |= mpo_layer<S, T>(sh, st, n, dold, dnew, plan, theta, phi, trunc_err, pf);
    else
      flags |= qr_sweep<S, T>(sh, st, n, dold, dnew, theta, phi, trunc_err, pf);
  } else {
    flags |= canon_sweep<S, T>(sh, st, n, dold, kGateRyRz, theta, phi, pix, false, pf);
    __syncthreads();  // the sweep's stores of sites 1..n-1 are read back by the ladder
    flags |= cnot_sweep<S, T>(sh, st, n, dold, dnew, -1, trunc_err, pf, exact_qr);
  }
  if (threadIdx.x == 0 && flags) status[0] |= flags;
}

// One kernel per layer program (PROG), so that each holds only its own sweeps.
template <int S, typename T, int PROG>
__global__ __launch_bounds__(kLayerThreads) void k_layer(T* state, int n, int chi, int layer,
                                                         const double* theta, const double* phi,
                                                         const double* pixels, double* trunc_err,
                                                         int* status, int exact_qr) {
  __shared__ LayerShared<S, T> sh;
  const int b = blockIdx.x;
  T* st = state + (size_t)b * n * ((size_t)2 * S * S * 2);
  layer_chain<S, T, false>(sh, st, n, chi, layer, PROG, theta, phi,
                    pixels ? pixels + (size_t)b * n : nullptr,
                    trunc_err ? trunc_err + (size_t)b * (n - 1) : nullptr, status + b, exact_qr,
                    0);
}

// A layer that keeps every singular value, batched: the ends (two workgroups per image, the
// left and the right end) and the sites between (one workgroup per site) run as two launches
// over disjoint sites.  All workgroups of image b sit on XCD b % 8, like the other kernels.
template <int S, typename T>
__global__ __launch_bounds__(kLayerThreads) void k_mpo_ends(T* state, int n, int chi, int layer,
                                                            MpoPlan plan, const double* theta,
                                                            const double* phi,
                                                            const double* pixels, int brick,
                                                            double* trunc_err, int* status,
                                                            int batch) {
  __shared__ LayerShared<S, T> sh;
  const int w = blockIdx.x, xcd = w % kXcds, j = w / kXcds;
  const int b = kXcds * (j >> 1) + xcd, part = j & 1;
  if (b >= batch) return;
  auto dold = [&](int k) { return bond_dim(n, chi, layer, k); };
  auto dnew = [&](int k) { return bond_dim(n, chi, layer + 1, k); };
  if (part == 0 && trunc_err)
    for (int k = threadIdx.x; k < n - 1; k += kLayerThreads) trunc_err[(size_t)b * (n - 1) + k] = 0.0;
  SitePrefetch<S, T> pf;
  const bool bad = mpo_ends<S, T>(mpo_bufs(sh), state + (size_t)b * n * ((size_t)2 * S * S * 2), n, dold,
                                  dnew, plan, theta, phi, pf, part, brick ? kGateHRy : kGateRyRz,
                                  pixels ? pixels + (size_t)b * n : nullptr, brick != 0);
  if (__any(bad) && threadIdx.x == 0) atomicOr(status + b, kImgNonfinite);
}

template <int S, typename T>
__global__ __launch_bounds__(kLayerThreads) void k_mpo_sites(T* state, int n, int chi, int layer,
                                                             MpoPlan plan, const double* theta,
                                                             const double* phi,
                                                             const double* pixels, int brick,
                                                             int* status, int batch) {
  // a site between the ends has old bonds D^old = D / 2 <= S / 2
  constexpr int H = S / 2 > 0 ? S / 2 : 1;
  constexpr size_t SLOT = (size_t)2 * S * S * 2;
  __shared__ cx<T> old[H * 2 * H];
  const int nmid = plan.kr - plan.kl - 2;
  const int w = blockIdx.x, xcd = w % kXcds, j = w / kXcds;
  const int b = kXcds * (j / nmid) + xcd, k = plan.kl + 2 + j % nmid;
  if (b >= batch) return;
  const int Dp = bond_dim(n, chi, layer, k - 1), Do = bond_dim(n, chi, layer, k);
  T* slot = state + ((size_t)b * n + k) * SLOT;
  const FastDiv fdo(Do);
  for (int idx = threadIdx.x; idx < Dp * 2 * Do; idx += kLayerThreads) {
    const int row = fdo.q(idx), c = fdo.r(idx);
    old[idx] = cx<T>{slot[2 * ((size_t)row * S + c)], slot[2 * ((size_t)row * S + c) + 1]};
  }
  lds_sync();
  auto at = [&](int a, int s_, int c) { return to_cd(old[(a * 2 + s_) * Do + c]); };
  const Gate2 g = site_gate(brick ? kGateHRy : kGateRyRz, k, theta, phi,
                            pixels ? pixels + (size_t)b * n : nullptr);
  const bool bad = mpo_plain_site<S, T>(at, g, Dp, Do, slot, threadIdx.x, kLayerThreads, k,
                                        brick != 0);
  if (__any(bad) && threadIdx.x == 0) atomicOr(status + b, kImgNonfinite);
}

// Host-side policy for bonds and layers that keep every singular value (kExactMpo: whole
// ladder layers as one contraction, other such bonds split exactly; kExactQr: such layers by
// the QR sweep; kExactSvd: canonical sweep + Jacobi SVD ladder like every other layer), read
// at each launch.
int g_exact_qr = kExactMpo;

void set_exact_qr(int mode) { g_exact_qr = mode; }
int exact_qr() { return g_exact_qr; }

// ------------------------------------------------------------------------------- mixed requests
// Encode: one workgroup per request of the bucket (same arithmetic as k_encode).
template <typename T>
__global__ void k_encode_mixed(const mps_request* reqs, int begin, int S) {
  const mps_request* r = reqs + begin + blockIdx.x;
  const int n = uniform_int(r->n_sites);
  T* state = uniform_ptr((T*)r->state);
  const double* pixels = uniform_ptr(r->pixels);
  int32_t* ctrl = uniform_ptr(r->ctrl);
  int bad = 0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const double x = pixels[k];
    double s, c;
    sincos(0.5 * M_PI * x, &s, &c);
    T* slot = state + (size_t)k * (size_t)(2 * S * S) * 2;
    store_c<T, double>(slot, 0, cd{c, 0.0});
    store_c<T, double>(slot, S, cd{s, 0.0});
    bad |= !isfinite(x);
  }
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0) {
    ctrl[0] = 0;
    ctrl[1] = bad ? kImgNonfinite : 0;
  }
}

// One layer for every request of the bucket that still needs one.  Persistent: each workgroup
// (one wavefront) takes the next table entry from the bucket's queue counter until the table
// is exhausted, so every wave leaves the loop once the counter passes the bucket size.
// Every value that steers control flow is made wave-uniform with readfirstlane, so the loop
// and everything in layer_chain compile to scalar branches as in k_layer.  The ticket is taken
// without a lane-dependent branch (all lanes issue the add, only lane 0 adds 1): with a branch
// around the atomic, the compiler may specialise the loop for the lanes that skip it and fold
// their readfirstlane to a constant, after which those lanes never see the queue advance.
template <int S, typename T>
__global__ __launch_bounds__(kLayerThreads) void k_layer_mixed(const mps_request* reqs, int begin,
                                                               int count, int* queue,
                                                               int exact_qr) {
  __shared__ LayerShared<S, T> sh;
  for (;;) {
    const int ticket = atomicAdd(queue, threadIdx.x == 0 ? 1 : 0);
    const int t = __builtin_amdgcn_readfirstlane(ticket);
    if (t >= count) break;
    const mps_request* r = reqs + begin + t;
    int32_t* ctrl = uniform_ptr(r->ctrl);
    const int n = uniform_int(r->n_sites), chi = uniform_int(r->chi);
    const int n_layers = uniform_int(r->n_layers), layer = uniform_int(ctrl[0]);
    if (layer < 0 || layer >= n_layers) continue;
    const double* theta = uniform_ptr(r->theta) + (size_t)layer * n;
    const double* phi = uniform_ptr(r->phi) + (size_t)layer * n;
    double* te = uniform_ptr(r->trunc_err);
    layer_chain<S, T, true>(sh, uniform_ptr((T*)r->state), n, chi, layer, kLayerRyRzLadder, theta, phi,
                      nullptr, te ? te + (size_t)layer * (n - 1) : nullptr, ctrl + 1, exact_qr,
                      n_layers);
    __syncthreads();
    if (threadIdx.x == 0) ctrl[0] = layer + 1;
  }
}

__global__ void k_zero_ints(int* p, int count) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) p[i] = 0;
}

hipError_t launch_zero_ints(int* p, int count, hipStream_t stream) {
  hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, stream, p, count);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_encode_mixed(const mps_request* reqs, int begin, int count, int S,
                               hipStream_t stream) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_encode_mixed<T>, dim3(count), dim3(64), 0, stream, reqs, begin, S);
  return hipGetLastError();
}

namespace {
// Workgroups per CU that fit (LDS and registers) for a layer kernel, cached per kernel.
template <int S, typename T>
int layer_mixed_fit() {
  static int fit = 0;
  if (fit == 0) {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_layer_mixed<S, T>, kLayerThreads, 0) !=
            hipSuccess || blocks < 1)
      blocks = 1;
    fit = blocks;
  }
  return fit;
}

int device_cus() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 1;
  }
  return cus;
}

template <int S, typename T>
hipError_t launch_layer_mixed_s(const mps_request* reqs, int begin, int count, int* queue,
                                int blocks_per_cu, hipStream_t stream) {
  const int fit = layer_mixed_fit<S, T>();
  const int per_cu = (blocks_per_cu > 0 && blocks_per_cu < fit) ? blocks_per_cu : fit;
  long long grid = (long long)per_cu * device_cus();
  if (grid > count) grid = count;
  hipLaunchKernelGGL((k_layer_mixed<S, T>), dim3((unsigned)grid), dim3(kLayerThreads), 0, stream,
                     reqs, begin, count, queue, g_exact_qr);
  return hipGetLastError();
}
}  // namespace

template <typename T>
hipError_t launch_layer_mixed(const mps_request* reqs, int begin, int count, int S, int* queue,
                              int blocks_per_cu, hipStream_t stream) {
  if (count == 0) return hipSuccess;
  switch (S) {
    case 2: return launch_layer_mixed_s<2, T>(reqs, begin, count, queue, blocks_per_cu, stream);
    case 4: return launch_layer_mixed_s<4, T>(reqs, begin, count, queue, blocks_per_cu, stream);
    case 8: return launch_layer_mixed_s<8, T>(reqs, begin, count, queue, blocks_per_cu, stream);
    case 16: return launch_layer_mixed_s<16, T>(reqs, begin, count, queue, blocks_per_cu, stream);
    default: return hipErrorInvalidValue;
  }
}

// ------------------------------------------------------------------------------- launchers
template <typename T>
hipError_t launch_encode(T* state, const double* pixels, int n, int S, int batch, int* status,
                         hipStream_t stream) {
  hipLaunchKernelGGL(k_encode<T>, dim3(batch), dim3(64), 0, stream, state, pixels, n, S, status);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_layer(T* state, int n, int chi, int S, int layer, int batch, int program,
                        const double* theta, const double* phi, const double* pixels,
                        double* trunc_err, int* status, int n_layers, hipStream_t stream) {
  const dim3 grid(batch), block(kLayerThreads);
  MpoPlan plan;
  // the brickwork program takes the site-local form when its two end carries land on two
  // different sites (its even-site bit rule is not in the meeting-carries step)
  if (g_exact_qr == kExactMpo && layer_keeps_all(n, chi, layer) &&
      !next_truncates(n, chi, layer, n_layers) &&
      mpo_plan(n, [&](int k) { return bond_dim(n, chi, layer, k); },
               [&](int k) { return bond_dim(n, chi, layer + 1, k); }, plan) &&
      (program == kLayerRyRzLadder || (program == kLayerHRyBrickwork && plan.kl + 1 < plan.kr))) {
    const int brick = program == kLayerHRyBrickwork;
    const unsigned groups = (unsigned)((batch + kXcds - 1) / kXcds);
    const int nmid = plan.kr - plan.kl - 2;
    switch (S) {
#define ANOMPS_KM(SV)                                                                              \
  case SV:                                                                                         \
    hipLaunchKernelGGL((k_mpo_ends<SV, T>), dim3(kXcds * groups * 2), block, 0, stream, state, n,  \
                       chi, layer, plan, theta, phi, pixels, brick, trunc_err, status, batch);     \
    if (nmid > 0)                                                                                  \
      hipLaunchKernelGGL((k_mpo_sites<SV, T>), dim3(kXcds * groups * (unsigned)nmid), block, 0,    \
                         stream, state, n, chi, layer, plan, theta, phi, pixels, brick, status,    \
                         batch);                                                                   \
    break;
      ANOMPS_KM(2) ANOMPS_KM(4) ANOMPS_KM(8) ANOMPS_KM(16)
#undef ANOMPS_KM
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  switch (S) {
#define ANOMPS_KL(SV)                                                                              \
  case SV:                                                                                         \
    if (program == kLayerHRyBrickwork)                                                             \
      hipLaunchKernelGGL((k_layer<SV, T, kLayerHRyBrickwork>), grid, block, 0, stream, state, n,   \
                         chi, layer, theta, phi, pixels, trunc_err, status, g_exact_qr);           \
    else                                                                                           \
      hipLaunchKernelGGL((k_layer<SV, T, kLayerRyRzLadder>), grid, block, 0, stream, state, n,     \
                         chi, layer, theta, phi, pixels, trunc_err, status, g_exact_qr);           \
    break;
    ANOMPS_KL(2) ANOMPS_KL(4) ANOMPS_KL(8) ANOMPS_KL(16)
#undef ANOMPS_KL
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ----------------------------------------------------------------- several exact layers per call
// A run of consecutive layers that all keep every singular value.  The sites between the
// reduced ends in every layer of the run (core_lo..core_hi) are local to the whole run: each
// takes all of its layers in LDS (FP64) and is written once.  The ends take the layers one
// after the other, each layer's ends plus the sites of that layer between its ends and the core.
constexpr int kMaxRun = 16;

struct MpoRun {
  int layer0, count, core_lo, core_hi;
  int carry_elems;  // complex128 elements of one carry buffer (the larger end's need)
  MpoPlan plan[kMaxRun];
};

template <int S, typename T>
__global__ __launch_bounds__(kLayerThreads) void k_mpo_run_ends(T* state, int n, int chi, MpoRun run,
                                                                const double* theta,
                                                                const double* phi,
                                                                double* trunc_err, int* status,
                                                                int batch) {
  // One end per workgroup (a run never has the two carries meeting in one site), so the carry
  // LDS holds one ping-pong pair, sized on the host for this run's bond dimensions (8 KiB at
  // 7x7, L = 4, chi = 16, against 16 KiB for the slot's worst case): all of a batch's end
  // workgroups then fit on the chip at once.
  constexpr size_t SLOT = (size_t)2 * S * S * 2;
  constexpr int SP = LayerShared<S, T>::SP;
  extern __shared__ cd dyn_lds[];
  cd* pool = dyn_lds;
  cx<T>* tbuf = reinterpret_cast<cx<T>*>(pool + 2 * run.carry_elems);
  const int w = blockIdx.x, xcd = w % kXcds, j = w / kXcds;
  const int b = kXcds * (j >> 1) + xcd, part = j & 1;
  if (b >= batch) return;
  // This chain of short dependent steps runs beside the core launch and bounds the call: its
  // waves take issue priority over the core's on a shared SIMD.
  __builtin_amdgcn_s_setprio(2);
  const int tid = threadIdx.x;
  T* st = state + (size_t)b * n * SLOT;
  SitePrefetch<S, T> pf;
  const MpoBufs<T> bufs =
      part == 0 ? MpoBufs<T>{{pool, pool + run.carry_elems}, {nullptr, nullptr}, tbuf}
                : MpoBufs<T>{{nullptr, nullptr}, {pool, pool + run.carry_elems}, tbuf};
  auto at = [&](int a, int s_, int c) { return to_cd(tbuf[(a * 2 + s_) * SP + c]); };
  bool bad = false;
  for (int r = 0; r < run.count; ++r) {
    const int layer = run.layer0 + r;
    auto dold = [&](int k) { return bond_dim(n, chi, layer, k); };
    auto dnew = [&](int k) { return bond_dim(n, chi, layer + 1, k); };
    const double* th = theta + (size_t)r * n;
    const double* ph = phi + (size_t)r * n;
    if (part == 0 && trunc_err)
      for (int k = tid; k < n - 1; k += kLayerThreads)
        trunc_err[((size_t)r * batch + b) * (n - 1) + k] = 0.0;
    const MpoPlan plan = run.plan[r];
    // with this layer's sites between its own ends and the core, on this side
    const int k0 = part == 0 ? plan.kl + 2 : run.core_hi + 1;
    const int k1 = part == 0 ? run.core_lo - 1 : plan.kr - 1;
    bad |= mpo_ends<S, T>(bufs, st, n, dold, dnew, plan, th, ph, pf, part, kGateRyRz, nullptr,
                          false, k0, k1);
    // the next layer reads what this one stored: the barrier's fence makes it visible
    __syncthreads();
  }
  if (__any(bad) && tid == 0) atomicOr(status + b, kImgNonfinite);
}

template <int S, typename T>
__global__ __launch_bounds__(kLayerThreads) void k_mpo_run_core(T* state, int n, int chi, MpoRun run,
                                                                const double* theta,
                                                                const double* phi, int* status,
                                                                int batch) {
  // every layer but the last stays in LDS: at most (S/2) x 2 x (S/2) entries before the last
  constexpr int H = S / 2 > 0 ? S / 2 : 1;
  constexpr size_t SLOT = (size_t)2 * S * S * 2;
  __shared__ cd buf[2][H * 2 * H];
  __shared__ Gate2 gates[kMaxRun];
  const int ncore = run.core_hi - run.core_lo + 1;
  const int w = blockIdx.x, xcd = w % kXcds, j = w / kXcds;
  const int b = kXcds * (j / ncore) + xcd, k = run.core_lo + j % ncore;
  if (b >= batch) return;
  const int tid = threadIdx.x;
  T* slot = state + ((size_t)b * n + k) * SLOT;
  int Dp = bond_dim(n, chi, run.layer0, k - 1), Do = bond_dim(n, chi, run.layer0, k);
  if (tid < run.count)  // one lane per layer: the gates' trigonometry runs side by side
    gates[tid] = site_gate(kGateRyRz, k, theta + (size_t)tid * n, phi + (size_t)tid * n, nullptr);
  {
    const FastDiv fdo(Do);
    for (int idx = tid; idx < Dp * 2 * Do; idx += kLayerThreads) {
      const int row = fdo.q(idx), c = fdo.r(idx);
      buf[0][idx] = to_cd(cx<T>{slot[2 * ((size_t)row * S + c)], slot[2 * ((size_t)row * S + c) + 1]});
    }
  }
  lds_sync();
  int cur = 0;
  bool bad = false;
  for (int r = 0; r < run.count; ++r) {
    const Gate2 g = gates[r];
    const cd* src = buf[cur];
    const int D = Do;
    auto at = [&](int a, int s_, int c) { return src[(a * 2 + s_) * D + c]; };
    if (r + 1 == run.count) {
      bad = mpo_plain_site<S, T>(at, g, Dp, Do, slot, tid, kLayerThreads);
    } else {
      cd* dst = buf[cur ^ 1];
      const int R = 2 * Do;
      const FastDiv fr(R), fdp(Dp), fdo(Do);
      for (int idx = tid; idx < 4 * Dp * R; idx += kLayerThreads) {
        const int row = fr.q(idx), m = fr.r(idx), i = row >> 1, y = row & 1;
        const int p = fdp.q(i), a = fdp.r(i), q = fdo.q(m), c = fdo.r(m);
        dst[idx] = (q == y) ? gated_at(at, g, a, y ^ p, c) : cd{0.0, 0.0};
      }
      lds_sync();
      cur ^= 1;
      Dp *= 2;
      Do *= 2;
    }
  }
  if (__any(bad) && tid == 0) atomicOr(status + b, kImgNonfinite);
}

// Length of the run of layers from `layer` (at most max_count) that can go through the two run
// kernels: every layer keeps all its singular values, and some sites lie between the reduced
// ends in all of them.  Fills `run`.  0 when the layer at `layer` cannot start such a run.
int mpo_run(int n, int chi, int S, int layer, int max_count, int n_layers, MpoRun& run) {
  if (g_exact_qr != kExactMpo || S > kMaxBond) return 0;
  run.layer0 = layer;
  run.core_lo = 0;
  run.core_hi = n - 1;
  int count = 0;
  while (count < max_count && count < kMaxRun) {
    const int l = layer + count;
    MpoPlan p;
    if (!layer_keeps_all(n, chi, l) || next_truncates(n, chi, l, n_layers) ||
        !mpo_plan(n, [&](int k) { return bond_dim(n, chi, l, k); },
                  [&](int k) { return bond_dim(n, chi, l + 1, k); }, p))
      break;
    const int lo = std::max(run.core_lo, p.kl + 2), hi = std::min(run.core_hi, p.kr - 1);
    if (lo > hi) break;
    run.plan[count] = p;
    run.core_lo = lo;
    run.core_hi = hi;
    ++count;
  }
  run.count = count;
  // One carry buffer: the left carry C_k (D_k rows, row stride 2S), the carry site's product
  // (D_kl x 2 x D_{kl+1}^old) and the right carry R_k (2 D_{k-1}^old rows, row stride S).
  int need = 1;
  for (int r = 0; r < count; ++r) {
    const int l = layer + r, kl = run.plan[r].kl, kr = run.plan[r].kr;
    const int dl = bond_dim(n, chi, l + 1, kl);
    need = std::max(need, dl * 2 * S);
    need = std::max(need, dl * 2 * bond_dim(n, chi, l, kl + 1));
    if (kr <= n - 2) need = std::max(need, 2 * bond_dim(n, chi, l, kr) * S);
  }
  run.carry_elems = (need + 15) & ~15;
  return count;
}

// A second stream per device (default priority) so that the ends of a run, a chain of small
// dependent steps, overlap the core launch: the caller's stream forks to it through an event
// and joins it again before returning, so the caller sees one ordered step.  Created on first
// use and kept until the process ends; the fork and join are serialised by a mutex.
struct SideStream {
  hipStream_t stream = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
constexpr int kMaxDevices = 64;
std::mutex g_side_mu;
SideStream g_side[kMaxDevices];

hipError_t side_stream(SideStream*& out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  SideStream& sd = g_side[dev];
  if (!sd.stream) {
    if ((e = hipStreamCreateWithFlags(&sd.stream, hipStreamNonBlocking)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&sd.fork, hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&sd.join, hipEventDisableTiming)) != hipSuccess) return e;
  }
  out = &sd;
  return hipSuccess;
}

template <typename T>
hipError_t launch_mpo_run(T* state, int n, int chi, int S, const MpoRun& run, int batch,
                          const double* theta, const double* phi, double* trunc_err, int* status,
                          hipStream_t stream) {
  const unsigned groups = (unsigned)((batch + kXcds - 1) / kXcds);
  const unsigned ncore = (unsigned)(run.core_hi - run.core_lo + 1);
  const dim3 block(kLayerThreads);
  std::lock_guard<std::mutex> lock(g_side_mu);
  SideStream* sd = nullptr;
  hipError_t e = side_stream(sd);
  if (e != hipSuccess) return e;
  if ((e = hipEventRecord(sd->fork, stream)) != hipSuccess) return e;
  if ((e = hipStreamWaitEvent(sd->stream, sd->fork, 0)) != hipSuccess) return e;
  switch (S) {
#define ANOMPS_KR(SV)                                                                              \
  case SV:                                                                                         \
    hipLaunchKernelGGL((k_mpo_run_ends<SV, T>), dim3(kXcds * groups * 2), block,                   \
                       (unsigned)(2 * run.carry_elems * sizeof(cd) +                               \
                                  2 * SV * LayerShared<SV, T>::SP * sizeof(cx<T>)),                \
                       sd->stream, state, n, chi, run, theta, phi, trunc_err, status, batch);      \
    if ((e = hipGetLastError()) != hipSuccess) break;                                              \
    hipLaunchKernelGGL((k_mpo_run_core<SV, T>), dim3(kXcds * groups * ncore), block, 0, stream,    \
                       state, n, chi, run, theta, phi, status, batch);                             \
    e = hipGetLastError();                                                                         \
    break;
    ANOMPS_KR(2) ANOMPS_KR(4) ANOMPS_KR(8) ANOMPS_KR(16)
#undef ANOMPS_KR
    default: e = hipErrorInvalidValue;
  }
  // join even after a failed launch, so that the caller's stream never runs ahead of the side
  const hipError_t e2 = hipEventRecord(sd->join, sd->stream);
  const hipError_t e3 = e2 == hipSuccess ? hipStreamWaitEvent(stream, sd->join, 0) : e2;
  return e != hipSuccess ? e : e3;
}

// Applies `count` ladder layers: runs of exact layers through the run kernels, the others one
// call of launch_layer each.  theta, phi: [count][n]; trunc_err: [count][batch][n-1] or null.
template <typename T>
hipError_t launch_layers(T* state, int n, int chi, int S, int layer, int count, int batch,
                         const double* theta, const double* phi, double* trunc_err, int* status,
                         int n_layers, hipStream_t stream) {
  int r = 0;
  while (r < count) {
    const double* th = theta + (size_t)r * n;
    const double* ph = phi + (size_t)r * n;
    double* te = trunc_err ? trunc_err + (size_t)r * batch * (n - 1) : nullptr;
    MpoRun run;
    const int len = mpo_run(n, chi, S, layer + r, count - r, n_layers, run);
    hipError_t e;
    if (len >= 2) {
      e = launch_mpo_run<T>(state, n, chi, S, run, batch, th, ph, te, status, stream);
    } else {
      e = launch_layer<T>(state, n, chi, S, layer + r, batch, kLayerRyRzLadder, th, ph, nullptr,
                          te, status, n_layers, stream);
    }
    if (e != hipSuccess) return e;
    r += len >= 2 ? len : 1;
  }
  return hipSuccess;
}

// ----------------------------------------------------------------- exact layers, slots above 16
// The same contraction for slots of 32..128.  A site tensor of up to 128 x 2 x 128 cannot be
// prefetched into registers, so the ends copy each old tensor into a buffer (WideStage) and keep
// their carries in the image's FP64 workspace (the wide kernels' HBM/L2 workspace); the sites
// between stage their old tensor in dynamic LDS with 256 lanes each.
template <int S, typename T>
struct WideStage {
  static constexpr int SP = S + 1;
  const T* src = nullptr;
  int Dl = 0, Dr = 0;
  __device__ void load(const T* slot, int dl, int dr) {
    src = slot;
    Dl = dl;
    Dr = dr;
  }
  __device__ void commit(cx<T>* dst) const {
    for (int idx = threadIdx.x; idx < Dl * 2 * Dr; idx += kLayerThreads) {
      const int row = idx / Dr, b = idx - row * Dr;
      dst[row * SP + b] = cx<T>{src[2 * ((size_t)row * S + b)], src[2 * ((size_t)row * S + b) + 1]};
    }
  }
};

// Two workgroups per image (left end, right end; one when the carries meet), one wavefront
// each.  Workspace of an image: left carries, right carries (2 S^2 complex128 each, two of
// each), then the two parts' staged tensors.
template <int S, typename T>
__global__ __launch_bounds__(kLayerThreads) void k_mpo_ends_wide(
    T* state, cd* ws, size_t ws_stride, int n, int chi, int layer, MpoPlan plan,
    const double* theta, const double* phi, const double* pixels, int brick, double* trunc_err,
    int* status, int batch) {
  const int b = blockIdx.x >> 1, part = blockIdx.x & 1;
  if (b >= batch) return;
  cd* wsb = ws + (size_t)b * ws_stride;
  cd* c0 = wsb;
  cd* r0 = wsb + 4 * S * S;
  cx<T>* tb = reinterpret_cast<cx<T>*>(wsb + 8 * S * S) + (size_t)part * 2 * S * (S + 1);
  const MpoBufs<T> bufs{{c0, c0 + 2 * S * S}, {r0, r0 + 2 * S * S}, tb};
  auto dold = [&](int k) { return bond_dim(n, chi, layer, k); };
  auto dnew = [&](int k) { return bond_dim(n, chi, layer + 1, k); };
  if (part == 0 && trunc_err)
    for (int k = threadIdx.x; k < n - 1; k += kLayerThreads) trunc_err[(size_t)b * (n - 1) + k] = 0.0;
  WideStage<S, T> pf;
  const bool bad = mpo_ends<S, T, decltype(dold), decltype(dnew), WideStage<S, T>, true>(
      bufs, state + (size_t)b * n * ((size_t)2 * S * S * 2), n, dold, dnew, plan, theta, phi, pf,
      part, brick ? kGateHRy : kGateRyRz, pixels ? pixels + (size_t)b * n : nullptr, brick != 0);
  if (__any(bad) && threadIdx.x == 0) atomicOr(status + b, kImgNonfinite);
}

constexpr int kWideSiteThreads = 256;

template <int S, typename T>
__global__ __launch_bounds__(kWideSiteThreads) void k_mpo_sites_wide(
    T* state, int n, int chi, int layer, MpoPlan plan, const double* theta, const double* phi,
    const double* pixels, int brick, int* status, int batch) {
  constexpr size_t SLOT = (size_t)2 * S * S * 2;
  extern __shared__ unsigned char wide_lds[];
  cx<T>* old = reinterpret_cast<cx<T>*>(wide_lds);
  const int nmid = plan.kr - plan.kl - 2;
  const int b = blockIdx.x / nmid, k = plan.kl + 2 + blockIdx.x % nmid;
  if (b >= batch) return;
  const int tid = threadIdx.x;
  const int Dp = bond_dim(n, chi, layer, k - 1), Do = bond_dim(n, chi, layer, k);
  T* slot = state + ((size_t)b * n + k) * SLOT;
  for (int idx = tid; idx < Dp * 2 * Do; idx += kWideSiteThreads) {
    const int row = idx / Do, c = idx - row * Do;
    old[idx] = cx<T>{slot[2 * ((size_t)row * S + c)], slot[2 * ((size_t)row * S + c) + 1]};
  }
  __syncthreads();
  auto at = [&](int a, int s_, int c) { return to_cd(old[(a * 2 + s_) * Do + c]); };
  const Gate2 g = site_gate(brick ? kGateHRy : kGateRyRz, k, theta, phi,
                            pixels ? pixels + (size_t)b * n : nullptr);
  const bool bad = mpo_plain_site<S, T>(at, g, Dp, Do, slot, tid, kWideSiteThreads, k, brick != 0);
  if (__any(bad) && (tid & 63) == 0) atomicOr(status + b, kImgNonfinite);
}

// Launches the contraction for a wide-slot layer that keeps every singular value; false (and
// nothing launched) when the layer takes the canonical sweep path instead.
template <typename T>
bool launch_mpo_wide(T* state, double* ws, size_t ws_stride, int n, int chi, int S, int layer,
                     int batch, int program, const double* theta, const double* phi,
                     const double* pixels, double* trunc_err, int* status, int n_layers,
                     hipStream_t stream, hipError_t& err) {
  MpoPlan plan;
  if (g_exact_qr != kExactMpo || !layer_keeps_all(n, chi, layer) ||
      next_truncates(n, chi, layer, n_layers) ||
      !mpo_plan(n, [&](int k) { return bond_dim(n, chi, layer, k); },
                [&](int k) { return bond_dim(n, chi, layer + 1, k); }, plan))
    return false;
  if (program != kLayerRyRzLadder && !(program == kLayerHRyBrickwork && plan.kl + 1 < plan.kr))
    return false;
  const int brick = program == kLayerHRyBrickwork;
  const int nmid = plan.kr - plan.kl - 2;
  const size_t lds = (size_t)(S / 2) * 2 * (S / 2) * sizeof(cx<T>);
  switch (S) {
#define ANOMPS_KW(SV)                                                                              \
  case SV:                                                                                         \
    hipLaunchKernelGGL((k_mpo_ends_wide<SV, T>), dim3(2 * batch), dim3(kLayerThreads), 0, stream,  \
                       state, (cd*)ws, ws_stride, n, chi, layer, plan, theta, phi, pixels, brick,  \
                       trunc_err, status, batch);                                                  \
    if (nmid > 0)                                                                                  \
      hipLaunchKernelGGL((k_mpo_sites_wide<SV, T>), dim3((unsigned)(batch * nmid)),               \
                         dim3(kWideSiteThreads), lds, stream, state, n, chi, layer, plan, theta,   \
                         phi, pixels, brick, status, batch);                                       \
    break;
    ANOMPS_KW(32) ANOMPS_KW(64) ANOMPS_KW(128)
#undef ANOMPS_KW
    default: return false;
  }
  err = hipGetLastError();
  return true;
}

template bool launch_mpo_wide<double>(double*, double*, size_t, int, int, int, int, int, int,
                                      const double*, const double*, const double*, double*, int*,
                                      int, hipStream_t, hipError_t&);
template bool launch_mpo_wide<float>(float*, double*, size_t, int, int, int, int, int, int,
                                     const double*, const double*, const double*, double*, int*,
                                     int, hipStream_t, hipError_t&);

template hipError_t launch_encode<double>(double*, const double*, int, int, int, int*, hipStream_t);
template hipError_t launch_encode<float>(float*, const double*, int, int, int, int*, hipStream_t);
template hipError_t launch_layer<double>(double*, int, int, int, int, int, int, const double*,
                                         const double*, const double*, double*, int*, int,
                                         hipStream_t);
template hipError_t launch_layer<float>(float*, int, int, int, int, int, int, const double*,
                                        const double*, const double*, double*, int*, int,
                                        hipStream_t);
template hipError_t launch_layers<double>(double*, int, int, int, int, int, int, const double*,
                                          const double*, double*, int*, int, hipStream_t);
template hipError_t launch_layers<float>(float*, int, int, int, int, int, int, const double*,
                                         const double*, double*, int*, int, hipStream_t);
template hipError_t launch_encode_mixed<double>(const mps_request*, int, int, int, hipStream_t);
template hipError_t launch_encode_mixed<float>(const mps_request*, int, int, int, hipStream_t);
template hipError_t launch_layer_mixed<double>(const mps_request*, int, int, int, int*, int, hipStream_t);
template hipError_t launch_layer_mixed<float>(const mps_request*, int, int, int, int*, int, hipStream_t);

}  // namespace anomps
