// Wide slots (S = 32, 64, 128): the layer (canonical sweep + CNOT ladder with FP64 SVD
// truncation, §II-B) and the measurement (environments and pair density matrices, §II-C,
// Eq. (4)-(5)) for bond dimensions whose two-site matrices (up to 256 x 256 complex128, 1 MiB)
// do not fit one workgroup's LDS.
//
// One workgroup of 256 lanes (four wavefronts) per image.  The centre and neighbour tensors,
// the matrix being factorised and the products of a bond live in a per-image FP64 workspace in
// HBM that stays hot in L2; LDS holds only reductions, singular values and the column ranking.
// The arithmetic and the truncation rule are those of the LDS kernels: Householder LQ for the
// canonical sweep, one-sided Jacobi (round-robin, FP64) for the ladder, the same convergence
// test, ranking, renormalisation and status flags.  The measurement computes in FP64 and
// stores environments and outputs in the batch's storage type.
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace anomps {
namespace {

constexpr int kWT = 256;                 // lanes per workgroup
constexpr int kTeam = 16;                // lanes per Jacobi column pair / Householder column
constexpr int kTeams = kWT / kTeam;
constexpr int kWideSweeps = 40;
constexpr int kWideTargets = 256;        // pairs per start site (host-validated)
constexpr int kWideGroups = 4;           // pair workgroups per image
constexpr size_t kSlotAlign = 64;        // complex128 elements (1 KiB)

// Workspace per image in complex128 elements: the larger of the layer's (ta, tb [2S^2] each,
// mat [4S^2], uq [2S^2], xb [2S^2]), the environments' (E [S^2] + Tm [2S^2] per side) and the
// pairs' (kWideGroups workgroups of F [3S^2] + Tm [6S^2] + G [3S^2]; F^{00}, F^{01} and four
// Tm blocks in use).
__host__ __device__ size_t ws_elems(int S) {
  const size_t s2 = (size_t)S * S;
  size_t e = 12 * s2;
  if (2 * 3 * s2 > e) e = 2 * 3 * s2;
  if ((size_t)kWideGroups * 12 * s2 > e) e = (size_t)kWideGroups * 12 * s2;
  return (e + kSlotAlign - 1) / kSlotAlign * kSlotAlign;
}

__device__ __forceinline__ double wv_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Sum over the 16 lanes of a DPP row (mirror, half-mirror and two quad swaps); every lane of
// the row ends with the same value.
__device__ __forceinline__ double team_sum16(double v) {
  v += dpp_mov_d<0x140>(v);
  v += dpp_mov_d<0x141>(v);
  v += dpp_mov_d<0x4E>(v);
  v += dpp_mov_d<0xB1>(v);
  return v;
}

// Sum over each half (8 lanes) of a DPP row: half-mirror, then the two quad swaps.
__device__ __forceinline__ double team_sum8(double v) {
  v += dpp_mov_d<0x141>(v);
  v += dpp_mov_d<0x4E>(v);
  v += dpp_mov_d<0xB1>(v);
  return v;
}

template <int TEAM>
__device__ __forceinline__ double team_sum(double v) {
  static_assert(TEAM == 8 || TEAM == 16, "team of 8 or 16 lanes");
  if constexpr (TEAM == 8) return team_sum8(v);
  return team_sum16(v);
}

// 1/sqrt(x), x > 0: hardware estimate and two Newton steps.
__device__ __forceinline__ double w_rsqrt(double x) {
  double r = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  r = r * fma(-h * r, r, 1.5);
  r = r * fma(-h * r, r, 1.5);
  return r;
}

struct WideShared {
  double sig2[256];     // squared singular values / Householder coefficients
  int rank[256];        // columns in descending singular-value order
  double red[kWT / 64];
  double part[kWT / 64][32];
  double rho[32];
  double tiny2;
  int tq[kWideTargets], tj[kWideTargets];
  int cnt;
};

__device__ double wblock_sum(double v, WideShared& sh) {
  v = wv_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh.red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < kWT / 64; ++w) t += sh.red[w];
  __syncthreads();
  return t;
}

struct WideWs {
  cd *ta, *tb, *mat, *uq, *xb;
};

__device__ WideWs layer_ws(cd* base, int S) {
  const size_t s2 = (size_t)S * S;
  WideWs w;
  w.ta = base;
  w.tb = w.ta + 2 * s2;
  w.mat = w.tb + 2 * s2;
  w.uq = w.mat + 4 * s2;
  w.xb = w.uq + 2 * s2;
  return w;
}

// Site tensor (Dl x 2 x Dr) of a slot (element (a, s, b) at (a*2 + s)*S + b) <-> workspace
// copy with the same indexing.
template <typename T>
__device__ void wload_site(cd* dst, const T* slot, int S, int Dl, int Dr) {
  for (int idx = threadIdx.x; idx < Dl * 2 * Dr; idx += kWT) {
    const int row = idx / Dr, b = idx % Dr;
    dst[(size_t)row * S + b] = load_c<T, double>(slot, (size_t)row * S + b);
  }
}

template <typename T>
__device__ void wstore_site(T* slot, const cd* src, int S, int Dl, int Dr) {
  for (int idx = threadIdx.x; idx < Dl * 2 * Dr; idx += kWT) {
    const int row = idx / Dr, b = idx % Dr;
    store_c<T, double>(slot, (size_t)row * S + b, src[(size_t)row * S + b]);
  }
}

enum : int { kWGateNone = 0, kWGateRyRz = 1, kWGateHRy = 2 };

// One-qubit gate U of site k: R_Y(theta_k) R_Z(phi_k), or R_Y(2 pi x_k - pi) H (§II-B, Eq. (2)).
__device__ void wapply_gate(cd* ta, int S, int Dl, int Dr, int mode, int k, const double* theta,
                            const double* phi, const double* pix) {
  cd u00, u01, u10, u11;
  if (mode == kWGateHRy) {
    double s, c;
    sincos(0.5 * (2.0 * M_PI * pix[k] - M_PI), &s, &c);
    const double r = 0.70710678118654752440;
    u00 = cd{(c - s) * r, 0.0};
    u01 = cd{(c + s) * r, 0.0};
    u10 = cd{(s + c) * r, 0.0};
    u11 = cd{(s - c) * r, 0.0};
  } else {
    double st, ct, sp, cp;
    sincos(0.5 * theta[k], &st, &ct);
    sincos(0.5 * phi[k], &sp, &cp);
    const cd em{cp, -sp}, ep{cp, sp};
    u00 = cscale(em, ct);
    u01 = cscale(ep, -st);
    u10 = cscale(em, st);
    u11 = cscale(ep, ct);
  }
  for (int idx = threadIdx.x; idx < Dl * Dr; idx += kWT) {
    const int a = idx / Dr, b = idx % Dr;
    const cd v0 = ta[(size_t)(a * 2) * S + b], v1 = ta[(size_t)(a * 2 + 1) * S + b];
    cd w0 = cmul(u00, v0), w1 = cmul(u10, v0);
    cfma(w0, u01, v1);
    cfma(w1, u11, v1);
    ta[(size_t)(a * 2) * S + b] = w0;
    ta[(size_t)(a * 2 + 1) * S + b] = w1;
  }
  __syncthreads();
}

// Householder QR of A = t^H (M rows, N <= M columns, column-major in w.mat with leading
// dimension 2S): t = L Q with L = R^H.  Step j reflects rows [j, M) of column j onto beta_j e_j
// (beta_j = -e^{i arg a_jj}|a_j|), keeps v_j in column j (rows >= j) and coef_j = 2/|v_j|^2 in
// sig2[j]; a column whose remaining part has |.|^2 <= 1e-30 |A|_F^2 is not reflected.  Q's
// columns (H_0 ... H_{N-1} applied to e_c) are formed in w.xb; Q's rows, conjugated, go to the
// site slot, and L to w.uq[j*S + a].
template <typename T>
__device__ void wide_lq(WideShared& sh, const WideWs& w, int S, int M, int N, int Dr, T* slot,
                        bool ladder = false) {
  const int ld = 2 * S;
  const int tid = threadIdx.x, team = tid / kTeam, lt = tid % kTeam;
  double f = 0.0;
  for (int idx = tid; idx < N * M; idx += kWT) {
    const cd v = w.mat[(size_t)(idx / M) * ld + idx % M];
    f = fma(v.re, v.re, fma(v.im, v.im, f));
  }
  const double tiny2 = 1e-30 * wblock_sum(f, sh);
  for (int j = 0; j < N; ++j) {
    cd* vj = w.mat + (size_t)j * ld;
    double a2 = 0.0;
    for (int r = j + tid; r < M; r += kWT) a2 = fma(vj[r].re, vj[r].re, fma(vj[r].im, vj[r].im, a2));
    a2 = wblock_sum(a2, sh);
    const double dr = vj[j].re, di = vj[j].im;
    cd beta{dr, di}, v0{dr, di};
    double coef = 0.0;
    if (a2 > tiny2) {
      const double alpha = a2 * w_rsqrt(a2);
      const double d2 = fma(dr, dr, di * di);
      const double rd = d2 > 0.0 ? w_rsqrt(d2) : 0.0;
      const double ad = d2 * rd;
      const cd u = d2 > 0.0 ? cd{dr * rd, di * rd} : cd{1.0, 0.0};
      beta = cd{-u.re * alpha, -u.im * alpha};
      v0 = cd{u.re * (ad + alpha), u.im * (ad + alpha)};
      coef = rcp_full(alpha * (alpha + ad));
    }
    for (int a = tid; a < N; a += kWT)
      w.uq[(size_t)j * S + a] = a < j ? cconj(vj[a]) : (a == j ? cconj(beta) : cd{0.0, 0.0});
    __syncthreads();
    if (tid == 0) {
      vj[j] = v0;
      sh.sig2[j] = coef;
    }
    __syncthreads();
    if (coef != 0.0) {
      for (int c = j + 1 + team; c < N; c += kTeams) {
        cd* col = w.mat + (size_t)c * ld;
        double gr = 0.0, gi = 0.0;
        for (int r = j + lt; r < M; r += kTeam) {
          const cd v = vj[r], x = col[r];
          gr = fma(v.re, x.re, fma(v.im, x.im, gr));
          gi = fma(v.re, x.im, fma(-v.im, x.re, gi));
        }
        gr = team_sum16(gr) * coef;
        gi = team_sum16(gi) * coef;
        for (int r = j + lt; r < M; r += kTeam) {
          const cd v = vj[r];
          col[r].re -= gr * v.re - gi * v.im;
          col[r].im -= gr * v.im + gi * v.re;
        }
      }
    }
    __syncthreads();
  }
  // Q columns in xb[c*ld + r].
  for (int idx = tid; idx < N * M; idx += kWT) {
    const int c = idx / M, r = idx % M;
    w.xb[(size_t)c * ld + r] = cd{r == c ? 1.0 : 0.0, 0.0};
  }
  __syncthreads();
  for (int j = N - 1; j >= 0; --j) {
    const double coef = sh.sig2[j];
    if (coef == 0.0) continue;
    const cd* vj = w.mat + (size_t)j * ld;
    for (int c = j + team; c < N; c += kTeams) {
      cd* col = w.xb + (size_t)c * ld;
      double gr = 0.0, gi = 0.0;
      for (int r = j + lt; r < M; r += kTeam) {
        const cd v = vj[r], x = col[r];
        gr = fma(v.re, x.re, fma(v.im, x.im, gr));
        gi = fma(v.re, x.im, fma(-v.im, x.re, gi));
      }
      gr = team_sum16(gr) * coef;
      gi = team_sum16(gi) * coef;
      for (int r = j + lt; r < M; r += kTeam) {
        const cd v = vj[r];
        col[r].re -= gr * v.re - gi * v.im;
        col[r].im -= gr * v.im + gi * v.re;
      }
    }
    __syncthreads();
  }
  if (ladder) {  // Theta' = Q R: Q itself into the slot as [(a,s)][j], row r = a*2 + s
    for (int idx = tid; idx < N * M; idx += kWT) {
      const int r = idx / N, c = idx % N;
      store_c<T, double>(slot, (size_t)r * S + c, w.xb[(size_t)c * ld + r]);
    }
  } else {
    for (int idx = tid; idx < N * M; idx += kWT) {
      const int c = idx / M, r = idx % M;
      const int s_ = r >= Dr, b = r - (s_ ? Dr : 0);
      store_c<T, double>(slot, (size_t)(c * 2 + s_) * S + b, cconj(w.xb[(size_t)c * ld + r]));
    }
  }
  __syncthreads();
}

// Column position of round-robin slot i in round r (slot 0 fixed, the others rotate).
__device__ __forceinline__ int rr_pos(int i, int r, int NP) {
  return i == 0 ? 0 : 1 + (i - 1 + r) % (NP - 1);
}

// One-sided Jacobi on the N columns (rows [0, M)) of mat (leading dimension ld), FP64: per
// round the NP/2 disjoint pairs of the round-robin tournament are spread over the teams of TEAM
// lanes; a team holds R rows per lane of both columns in registers, reduces |x|^2, |y|^2 and
// x^H y with DPP, rotates when |x^H y|^2 > (M eps)^2 |x|^2 |y|^2 and writes both columns back.
// Stops after a sweep whose rotated pairs all had |x^H y|^2 <= big_tol |x|^2 |y|^2 (1e-16 for
// FP64 storage, 1e-8 for FP32 storage: quadratic convergence leaves the columns orthogonal to
// ~1e-16 and ~1e-8, the latter below the storage rounding).  On return
// sig2[c] = |w_c|^2 and sh.tiny2 = 1e-30 |A|_F^2 (columns at or below it count as zero).
template <int R, int TEAM>
__device__ int wide_jacobi_r(WideShared& sh, cd* mat, int ld, int M, int N, double big_tol) {
  constexpr int TEAMS = kWT / TEAM;
  const int tid = threadIdx.x, team = tid / TEAM, lt = tid % TEAM;
  double f = 0.0;
  for (int idx = tid; idx < N * M; idx += kWT) {
    const cd v = mat[(size_t)(idx / M) * ld + idx % M];
    f = fma(v.re, v.re, fma(v.im, v.im, f));
  }
  const double tiny2 = 1e-30 * wblock_sum(f, sh);
  const double tol = (double)M * 2.220446049250313e-16;
  const double tol2 = tol * tol;
  const int NP = N + (N & 1), P = NP / 2;
  bool converged = N < 2;
  for (int sweep = 0; !converged && sweep < kWideSweeps; ++sweep) {
    int rotated = 0, big = 0;
    for (int r = 0; r < NP - 1; ++r) {
      for (int q = team; q < P; q += TEAMS) {
        const int ci = rr_pos(q, r, NP), cj = rr_pos(NP - 1 - q, r, NP);
        if (ci >= N || cj >= N) continue;
        cd* xc = mat + (size_t)ci * ld;
        cd* yc = mat + (size_t)cj * ld;
        cd x[R], y[R];
        double gr = 0.0, gi = 0.0, a = 0.0, bb = 0.0;
#pragma unroll
        for (int t = 0; t < R; ++t) {
          const int row = lt + t * TEAM;
          x[t] = row < M ? xc[row] : cd{0.0, 0.0};
          y[t] = row < M ? yc[row] : cd{0.0, 0.0};
          gr = fma(x[t].re, y[t].re, fma(x[t].im, y[t].im, gr));
          gi = fma(x[t].re, y[t].im, fma(-x[t].im, y[t].re, gi));
          a = fma(x[t].re, x[t].re, fma(x[t].im, x[t].im, a));
          bb = fma(y[t].re, y[t].re, fma(y[t].im, y[t].im, bb));
        }
        a = team_sum<TEAM>(a);
        bb = team_sum<TEAM>(bb);
        gr = team_sum<TEAM>(gr);
        gi = team_sum<TEAM>(gi);
        const double ag2 = fma(gr, gr, gi * gi);
        const double ab = a * bb;
        if (a > tiny2 && bb > tiny2 && ag2 > tol2 * ab) {
          rotated = 1;
          big |= ag2 > big_tol * ab;
          const JacobiRot jr = jacobi_rot(a, bb, gr, gi, ag2);
#pragma unroll
          for (int t = 0; t < R; ++t) {
            const int row = lt + t * TEAM;
            jacobi_apply(jr, x[t], y[t]);
            if (row < M) {
              xc[row] = x[t];
              yc[row] = y[t];
            }
          }
        }
      }
      __syncthreads();
    }
    converged = !__syncthreads_or(rotated & big);
  }
  for (int c = team; c < N; c += TEAMS) {
    const cd* col = mat + (size_t)c * ld;
    double s2 = 0.0;
    for (int row = lt; row < M; row += TEAM) s2 = fma(col[row].re, col[row].re, fma(col[row].im, col[row].im, s2));
    s2 = team_sum<TEAM>(s2);
    if (lt == 0) sh.sig2[c] = s2;
  }
  if (tid == 0) sh.tiny2 = tiny2;
  __syncthreads();
  return converged ? 0 : kImgNoConvergence;
}

// Teams of 8 lanes (32 column pairs at a time) up to 128 rows, of 16 lanes above: the sweep's
// rounds are short chains of dependent steps, and more pairs in flight per image shorten them.
__device__ int wide_jacobi(WideShared& sh, cd* mat, int ld, int M, int N, double big_tol) {
  if (M <= 128) {
    const int rows = (M + 7) / 8;
    if (rows <= 1) return wide_jacobi_r<1, 8>(sh, mat, ld, M, N, big_tol);
    if (rows <= 2) return wide_jacobi_r<2, 8>(sh, mat, ld, M, N, big_tol);
    if (rows <= 4) return wide_jacobi_r<4, 8>(sh, mat, ld, M, N, big_tol);
    if (rows <= 8) return wide_jacobi_r<8, 8>(sh, mat, ld, M, N, big_tol);
    return wide_jacobi_r<16, 8>(sh, mat, ld, M, N, big_tol);
  }
  return wide_jacobi_r<(256 + kTeam - 1) / kTeam, kTeam>(sh, mat, ld, M, N, big_tol);
}

// Right-to-left sweep: gates (mode != none) and right-canonical sites n-1..1 by Householder LQ;
// the centre ends in w.ta as site 0.  With from_ws the tensor of site n-1 is already in w.ta.
template <typename T, typename Dims>
__device__ int wide_canon(WideShared& sh, const WideWs& w, T* st, int S, int n, Dims dims, int mode,
                          const double* theta, const double* phi, const double* pix, bool from_ws) {
  const size_t SLOT = (size_t)2 * S * S * 2;
  const int ld = 2 * S, tid = threadIdx.x;
  if (!from_ws) {
    wload_site(w.ta, st + (size_t)(n - 1) * SLOT, S, dims(n - 2), 1);
    __syncthreads();
  }
  for (int k = n - 1; k >= 1; --k) {
    const int Dl = dims(k - 1), Dr = dims(k), Dll = dims(k - 2);
    if (mode != kWGateNone) wapply_gate(w.ta, S, Dl, Dr, mode, k, theta, phi, pix);
    const int M = 2 * Dr, N = Dl;
    for (int idx = tid; idx < N * M; idx += kWT) {
      const int a = idx / M, rr = idx % M;
      const int s_ = rr >= Dr, b = rr - (s_ ? Dr : 0);
      w.mat[(size_t)a * ld + rr] = cconj(w.ta[(size_t)(a * 2 + s_) * S + b]);
    }
    __syncthreads();
    wide_lq(sh, w, S, M, N, Dr, st + (size_t)k * SLOT);
    wload_site(w.tb, st + (size_t)(k - 1) * SLOT, S, Dll, Dl);
    __syncthreads();
    for (int idx = tid; idx < Dll * 2 * Dl; idx += kWT) {
      const int row = idx / Dl, a = idx % Dl;
      cd acc{0.0, 0.0};
      for (int j = 0; j < Dl; ++j) cfma(acc, w.tb[(size_t)row * S + j], w.uq[(size_t)j * S + a]);
      w.ta[(size_t)row * S + a] = acc;
    }
    __syncthreads();
  }
  if (mode != kWGateNone) wapply_gate(w.ta, S, 1, dims(0), mode, 0, theta, phi, pix);
  return 0;
}

// Left-to-right two-site sweep from the centre (site 0) in w.ta; CNOT(k, k+1) on bond k when
// parity < 0 or k % 2 == parity.  Keeps after(k) singular triplets, renormalises the kept
// weight to one, records the discarded weight of CNOT bonds in trunc_err[k].
template <typename T, typename Before, typename After>
__device__ int wide_cnot(WideShared& sh, const WideWs& w, T* st, int S, int n, Before before,
                         After after, int parity, double* trunc_err, int exact_qr) {
  const size_t SLOT = (size_t)2 * S * S * 2;
  const int ld = 2 * S, tid = threadIdx.x;
  int flags = 0;
  for (int k = 0; k <= n - 2; ++k) {
    const int Dl = after(k - 1), Dc = before(k), Dr = before(k + 1), D = after(k);
    const int cx = (parity < 0 || (k & 1) == parity) ? 1 : 0;
    wload_site(w.tb, st + (size_t)(k + 1) * SLOT, S, Dc, Dr);
    __syncthreads();
    const int M = 2 * Dl, N = 2 * Dr;
    // Theta'[(a,s),(t,b)] = sum_c A[k][a,s,c] A[k+1][c, t XOR (cx s), b]
    for (int idx = tid; idx < N * M; idx += kWT) {
      const int col = idx / M, row = idx % M;
      const int t = col >= Dr, b = col - (t ? Dr : 0), s_ = row & 1;
      cd acc{0.0, 0.0};
      for (int c = 0; c < Dc; ++c)
        cfma(acc, w.ta[(size_t)row * S + c], w.tb[(size_t)(c * 2 + (t ^ (s_ & cx))) * S + b]);
      w.mat[(size_t)col * ld + row] = acc;
    }
    __syncthreads();
    if (exact_qr && D == (M < N ? M : N)) {
      // The bond keeps every singular value: split exactly (identity when D = M, else
      // Householder QR), centre scaled by 1/|Theta'|_F, discarded weight 0.
      double f = 0.0;
      for (int idx = tid; idx < N * M; idx += kWT) {
        const cd v = w.mat[(size_t)(idx / M) * ld + idx % M];
        f = fma(v.re, v.re, fma(v.im, v.im, f));
      }
      f = wblock_sum(f, sh);
      if (!isfinite(f) || !(f > 0.0)) flags |= kImgNonfinite;
      const double scale = f > 0.0 ? w_rsqrt(f) : 0.0;
      if (cx && tid == 0 && trunc_err) trunc_err[k] = 0.0;
      T* slot = st + (size_t)k * SLOT;
      if (D == M) {
        for (int idx = tid; idx < M * M; idx += kWT) {
          const int r = idx / M, j = idx % M;
          store_c<T, double>(slot, (size_t)r * S + j, cd{r == j ? 1.0 : 0.0, 0.0});
        }
        for (int idx = tid; idx < D * N; idx += kWT) {
          const int j = idx / N, col = idx % N;
          const int t = col >= Dr, b = col - (t ? Dr : 0);
          w.ta[(size_t)(j * 2 + t) * S + b] = cscale(w.mat[(size_t)col * ld + j], scale);
        }
      } else {
        wide_lq(sh, w, S, M, N, Dr, slot, true);
        for (int idx = tid; idx < D * N; idx += kWT) {
          const int j = idx / N, col = idx % N;
          const int t = col >= Dr, b = col - (t ? Dr : 0);
          w.ta[(size_t)(j * 2 + t) * S + b] =
              j <= col ? cscale(cconj(w.uq[(size_t)col * S + j]), scale) : cd{0.0, 0.0};
        }
      }
      __syncthreads();
      continue;
    }
    flags |= wide_jacobi(sh, w.mat, ld, M, N, std::is_same<T, float>::value ? 1e-8 : 1e-16);
    const double tiny2 = sh.tiny2;
    for (int c = tid; c < N; c += kWT) {
      double v = sh.sig2[c];
      if (!(v >= 0.0)) v = 0.0;
      int rk = 0;
      for (int i = 0; i < N; ++i) {
        double u = sh.sig2[i];
        if (!(u >= 0.0)) u = 0.0;
        rk += (u > v) || (u == v && i < c);
      }
      sh.rank[rk] = c;
    }
    __syncthreads();
    double kept = 0.0, disc = 0.0;
    for (int r = 0; r < N; ++r) {
      double v = sh.sig2[sh.rank[r]];
      if (!(v >= 0.0)) v = 0.0;
      if (r < D) kept += v; else disc += v;
    }
    if (!isfinite(kept) || !isfinite(disc) || !(kept > 0.0)) flags |= kImgNonfinite;
    const double inv_norm = (kept > 0.0) ? w_rsqrt(kept) : 0.0;
    if (cx && tid == 0 && trunc_err) trunc_err[k] = (kept + disc > 0.0) ? disc / (kept + disc) : 0.0;
    for (int idx = tid; idx < M * D; idx += kWT) {
      const int r = idx / D, j = idx % D;
      const int c = sh.rank[j];
      const double s2 = sh.sig2[c];
      cd v{0.0, 0.0};
      if (s2 > tiny2) v = cscale(w.mat[(size_t)c * ld + r], w_rsqrt(s2));
      w.uq[(size_t)r * S + j] = v;
    }
    __syncthreads();
    wstore_site(st + (size_t)k * SLOT, w.uq, S, Dl, D);
    // X_s = U_s^H A_s -> xb[(s*S + j)*S + c]
    for (int idx = tid; idx < 2 * D * Dc; idx += kWT) {
      const int sj = idx / Dc, c = idx % Dc;
      const int s_ = sj >= D, j = sj - (s_ ? D : 0);
      cd acc{0.0, 0.0};
      for (int a = 0; a < Dl; ++a)
        cfmac(acc, w.uq[(size_t)(a * 2 + s_) * S + j], w.ta[(size_t)(a * 2 + s_) * S + c]);
      w.xb[(size_t)(s_ * S + j) * S + c] = acc;
    }
    __syncthreads();
    // New centre S V^H = U^H Theta' / |sigma_kept| -> ta[(j*2 + t)*S + b]
    for (int idx = tid; idx < D * 2 * Dr; idx += kWT) {
      const int j = idx / (2 * Dr), o = idx % (2 * Dr);
      const int t = o >= Dr, b = o - (t ? Dr : 0);
      cd acc{0.0, 0.0};
      for (int c = 0; c < Dc; ++c) {
        cfma(acc, w.xb[(size_t)j * S + c], w.tb[(size_t)(c * 2 + t) * S + b]);
        cfma(acc, w.xb[(size_t)(S + j) * S + c], w.tb[(size_t)(c * 2 + (t ^ cx)) * S + b]);
      }
      w.ta[(size_t)(j * 2 + t) * S + b] = cscale(acc, inv_norm);
    }
    __syncthreads();
  }
  wstore_site(st + (size_t)(n - 1) * SLOT, w.ta, S, after(n - 2), 1);
  __syncthreads();
  return flags;
}

template <typename T, int PROG>
__global__ __launch_bounds__(kWT) void k_layer_wide(T* state, cd* ws, int n, int chi, int S,
                                                    int layer, const double* theta,
                                                    const double* phi, const double* pixels,
                                                    double* trunc_err, int* status, int exact_qr) {
  __shared__ WideShared sh;
  const int b = blockIdx.x;
  T* st = state + (size_t)b * n * ((size_t)2 * S * S * 2);
  const WideWs w = layer_ws(ws + (size_t)b * ws_elems(S), S);
  const double* pix = pixels ? pixels + (size_t)b * n : nullptr;
  double* te = trunc_err ? trunc_err + (size_t)b * (n - 1) : nullptr;
  auto dold = [&](int k) { return bond_dim(n, chi, layer, k); };
  auto dnew = [&](int k) { return bond_dim(n, chi, layer + 1, k); };
  int flags = 0;
  if (PROG == 1) {
    auto dmid = [&](int k) { return bond_dim(n, chi, (k & 1) ? layer : layer + 1, k); };
    flags |= wide_canon(sh, w, st, S, n, dold, kWGateHRy, theta, phi, pix, false);
    flags |= wide_cnot(sh, w, st, S, n, dold, dmid, 0, te, exact_qr);
    flags |= wide_canon(sh, w, st, S, n, dmid, kWGateNone, theta, phi, pix, true);
    flags |= wide_cnot(sh, w, st, S, n, dmid, dnew, 1, te, exact_qr);
  } else {
    flags |= wide_canon(sh, w, st, S, n, dold, kWGateRyRz, theta, phi, pix, false);
    flags |= wide_cnot(sh, w, st, S, n, dold, dnew, -1, te, exact_qr);
  }
  if (threadIdx.x == 0 && flags) status[b] |= flags;
}

// ------------------------------------------------------------------------ measurement
// C = sum_k A(i, k) B(k, j) over an Mr x Nc output, K terms, in FP64: each lane computes TI x TJ
// output tiles (consecutive lanes take consecutive column tiles), so each k step loads TI + TJ
// operands for TI*TJ complex multiply-adds.  `a`, `b` return operands (conjugation and storage
// type inside), `out(i, j, v)` stores or accumulates.
template <int TI, int TJ, typename FA, typename FB, typename FC>
__device__ __forceinline__ void tile_cgemm_t(int Mr, int Nc, int K, FA a, FB b, FC out) {
  const int ti = (Mr + TI - 1) / TI, tj = (Nc + TJ - 1) / TJ;
  for (int tile = threadIdx.x; tile < ti * tj; tile += kWT) {
    const int i0 = (tile / tj) * TI, j0 = (tile % tj) * TJ;
    cd acc[TI][TJ];
#pragma unroll
    for (int ii = 0; ii < TI; ++ii)
#pragma unroll
      for (int jj = 0; jj < TJ; ++jj) acc[ii][jj] = cd{0.0, 0.0};
    for (int k = 0; k < K; ++k) {
      cd av[TI], bv[TJ];
#pragma unroll
      for (int ii = 0; ii < TI; ++ii) av[ii] = (i0 + ii < Mr) ? a(i0 + ii, k) : cd{0.0, 0.0};
#pragma unroll
      for (int jj = 0; jj < TJ; ++jj) bv[jj] = (j0 + jj < Nc) ? b(k, j0 + jj) : cd{0.0, 0.0};
#pragma unroll
      for (int ii = 0; ii < TI; ++ii)
#pragma unroll
        for (int jj = 0; jj < TJ; ++jj) cfma(acc[ii][jj], av[ii], bv[jj]);
    }
#pragma unroll
    for (int ii = 0; ii < TI; ++ii)
#pragma unroll
      for (int jj = 0; jj < TJ; ++jj)
        if (i0 + ii < Mr && j0 + jj < Nc) out(i0 + ii, j0 + jj, acc[ii][jj]);
  }
}

// LDS-staged form for outputs of 64 x 64 entries or more: the workgroup walks 64 x 64 output
// blocks; per chunk of 16 k it stages the 64 x 16 slice of the left operand and the 16 x 64
// slice of the right one in LDS (each operand entry read once per block instead of once per
// lane tile), then each lane accumulates a 4 x 4 tile, rows tr + 16 ii and columns tc + 16 jj
// (tr = lane / 16, tc = lane % 16), so that the 16 lanes of a row group read consecutive LDS
// entries and store consecutive columns.  The k order of every sum is the plain 0..K-1, as in
// tile_cgemm_t.  Every lane of the workgroup must call it (it holds barriers).
constexpr int kGB = 64, kGK = 16, kGAS = kGB + 1;  // block, k chunk, padded row of the A slice
struct GemmLds {
  cd a[kGK * kGAS];  // a[kk][row], rows padded to 65 so that the staging stores miss no bank
  cd b[kGK * kGB];   // b[kk][col]
};

template <typename FA, typename FB, typename FC>
__device__ void lds_cgemm(GemmLds& g, int Mr, int Nc, int K, FA a, FB b, FC out) {
  const int t = threadIdx.x, tr = t >> 4, tc = t & 15;
  const int bn = (Nc + kGB - 1) / kGB, nblk = ((Mr + kGB - 1) / kGB) * bn;
  for (int blk = 0; blk < nblk; ++blk) {
    const int i0 = (blk / bn) * kGB, j0 = (blk % bn) * kGB;
    cd acc[4][4];
#pragma unroll
    for (int ii = 0; ii < 4; ++ii)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) acc[ii][jj] = cd{0.0, 0.0};
    for (int k0 = 0; k0 < K; k0 += kGK) {
#pragma unroll
      for (int r = 0; r < kGB * kGK / kWT; ++r) {
        const int idx = t + r * kWT;
        const int ka = idx & (kGK - 1), row = idx >> 4;
        g.a[ka * kGAS + row] =
            (i0 + row < Mr && k0 + ka < K) ? a(i0 + row, k0 + ka) : cd{0.0, 0.0};
        const int kb = idx >> 6, col = idx & (kGB - 1);
        g.b[kb * kGB + col] =
            (k0 + kb < K && j0 + col < Nc) ? b(k0 + kb, j0 + col) : cd{0.0, 0.0};
      }
      __syncthreads();
#pragma unroll 4
      for (int kk = 0; kk < kGK; ++kk) {
        cd av[4], bv[4];
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) av[ii] = g.a[kk * kGAS + tr + 16 * ii];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) bv[jj] = g.b[kk * kGB + tc + 16 * jj];
#pragma unroll
        for (int ii = 0; ii < 4; ++ii)
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) cfma(acc[ii][jj], av[ii], bv[jj]);
      }
      __syncthreads();
    }
#pragma unroll
    for (int ii = 0; ii < 4; ++ii)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int i = i0 + tr + 16 * ii, j = j0 + tc + 16 * jj;
        if (i < Mr && j < Nc) out(i, j, acc[ii][jj]);
      }
  }
}

// LDS-staged blocks when the output has 64 x 64 entries or more, 2 x 2 lane tiles otherwise.
// Called by every lane of the workgroup.
template <typename FA, typename FB, typename FC>
__device__ __forceinline__ void tile_cgemm(GemmLds& g, int Mr, int Nc, int K, FA a, FB b, FC out) {
  if (Mr * Nc >= kGB * kGB)
    lds_cgemm(g, Mr, Nc, K, a, b, out);
  else
    tile_cgemm_t<2, 2>(Mr, Nc, K, a, b, out);
}

// Left (side 0) or right (side 1) environments of one image, stored as T in env
// ([2][n+1][S][S], ket index first), computed in FP64 with E and Tm in the workspace.
template <typename T>
__global__ __launch_bounds__(kWT) void k_env_wide(const T* state, T* env, cd* ws, int n, int chi,
                                                  int S, int layers) {
  const int b = blockIdx.x >> 1, side = blockIdx.x & 1;
  const size_t SLOT = (size_t)2 * S * S * 2, s2 = (size_t)S * S;
  const T* st = state + (size_t)b * n * SLOT;
  T* ev = env + ((size_t)b * 2 + side) * (n + 1) * s2 * 2;
  __shared__ GemmLds gl;
  cd* E = ws + (size_t)b * ws_elems(S) + (size_t)side * 3 * s2;
  cd* Tm = E + s2;
  const int tid = threadIdx.x;
  auto dim = [&](int k) { return bond_dim(n, chi, layers, k); };
  auto store_env = [&](int k, int D) {
    for (int idx = tid; idx < D * D; idx += kWT) {
      const int r = idx / D, c = idx % D;
      store_c<T, double>(ev + (size_t)k * s2 * 2, (size_t)r * S + c, E[(size_t)r * S + c]);
    }
  };
  if (tid == 0) E[0] = cd{1.0, 0.0};
  __syncthreads();
  if (side == 0) {
    store_env(0, 1);
    for (int k = 0; k < n; ++k) {
      const int Dl = dim(k - 1), Dr = dim(k);
      const T* A = st + (size_t)k * SLOT;
      // Tm[s][a][b'] = sum_a' E[a][a'] conj(A[a'][s][b'])
      for (int s = 0; s < 2; ++s)
        tile_cgemm(gl, Dl, Dr, Dl, [&](int a, int ap) { return E[(size_t)a * S + ap]; },
                   [&](int ap, int bp) { return cconj(load_c<T, double>(A, (size_t)(ap * 2 + s) * S + bp)); },
                   [&](int a, int bp, cd v) { Tm[(size_t)(s * S + a) * S + bp] = v; });
      __syncthreads();
      // L_{k+1}[b][b'] = sum_s sum_a A[a][s][b] Tm[s][a][b']  (k runs over (s, a))
      tile_cgemm(gl, Dr, Dr, 2 * Dl,
                 [&](int bb, int k) { const int s = k >= Dl, a = k - (s ? Dl : 0);
                                      return load_c<T, double>(A, (size_t)(a * 2 + s) * S + bb); },
                 [&](int k, int bp) { const int s = k >= Dl, a = k - (s ? Dl : 0);
                                      return Tm[(size_t)(s * S + a) * S + bp]; },
                 [&](int bb, int bp, cd v) { E[(size_t)bb * S + bp] = v; });
      __syncthreads();
      store_env(k + 1, Dr);
    }
  } else {
    store_env(n, 1);
    for (int k = n - 1; k >= 0; --k) {
      const int Dl = dim(k - 1), Dr = dim(k);
      const T* A = st + (size_t)k * SLOT;
      // Tm[s][c][a'] = sum_c' E[c][c'] conj(A[a'][s][c'])
      for (int s = 0; s < 2; ++s)
        tile_cgemm(gl, Dr, Dl, Dr, [&](int c, int cp) { return E[(size_t)c * S + cp]; },
                   [&](int cp, int ap) { return cconj(load_c<T, double>(A, (size_t)(ap * 2 + s) * S + cp)); },
                   [&](int c, int ap, cd v) { Tm[(size_t)(s * S + c) * S + ap] = v; });
      __syncthreads();
      // R_k[a][a'] = sum_s sum_c A[a][s][c] Tm[s][c][a']  (k runs over (s, c))
      tile_cgemm(gl, Dl, Dl, 2 * Dr,
                 [&](int a, int k) { const int s = k >= Dr, c = k - (s ? Dr : 0);
                                     return load_c<T, double>(A, (size_t)(a * 2 + s) * S + c); },
                 [&](int k, int ap) { const int s = k >= Dr, c = k - (s ? Dr : 0);
                                      return Tm[(size_t)(s * S + c) * S + ap]; },
                 [&](int a, int ap, cd v) { E[(size_t)a * S + ap] = v; });
      __syncthreads();
      store_env(k, Dl);
    }
  }
}

__device__ __forceinline__ cd pauli_w(int a, int r, int c) {
  switch (a) {
    case 0: return cd{(double)(r == c), 0.0};
    case 1: return cd{(double)(r != c), 0.0};
    case 2: return (r == c) ? cd{0.0, 0.0} : cd{0.0, r == 0 ? -1.0 : 1.0};
    default: return (r == c) ? cd{r == 0 ? 1.0 : -1.0, 0.0} : cd{0.0, 0.0};
  }
}

// Pair expectations: workgroup (image, g) takes the start sites i = g, g + G, ...; for each it
// opens the blocks F^{00} and F^{01} (F^{10} = F^{01 H}) from L_i and A[i], carries them through
// the transfer maps of the sites up to each listed partner j, closes with A[j] and R_{j+1} into
// rho_ij and writes Re Tr(rho_ij P_a (x) P_c).  F^{11} is not carried: the two diagonal blocks
// sum to the left environment at every step (the open and the transfer maps are linear and
// take L_i to L_{i+1}, L_{i+2}, ...), so at the close F^{11} = L_j - F^{00}.
template <typename T>
__global__ __launch_bounds__(kWT) void k_pairs_wide(const T* state, const T* env, cd* ws,
                                                    const int* pairs, int m, int n, int chi, int S,
                                                    int layers, T* out) {
  __shared__ WideShared sh;
  __shared__ GemmLds gl;
  const int b = blockIdx.x / kWideGroups, g = blockIdx.x % kWideGroups;
  const size_t SLOT = (size_t)2 * S * S * 2, s2 = (size_t)S * S;
  const T* st = state + (size_t)b * n * SLOT;
  const T* evl = env + (size_t)b * 2 * (n + 1) * s2 * 2;
  const T* evr = evl + (size_t)(n + 1) * s2 * 2;
  cd* F = ws + (size_t)b * ws_elems(S) + (size_t)g * 12 * s2;
  cd* Tm = F + 3 * s2;
  cd* G = Tm + 6 * s2;
  T* o = out + (size_t)b * m * 15;
  const int tid = threadIdx.x;
  auto dim = [&](int k) { return bond_dim(n, chi, layers, k); };
  const T qnan = (T)__builtin_nan("");
  for (int i = g; i < n - 1; i += kWideGroups) {
    if (tid == 0) sh.cnt = 0;
    __syncthreads();
    for (int q = tid; q < m; q += kWT) {
      const int pi = pairs[2 * q], pj = pairs[2 * q + 1];
      const bool valid = pi >= 0 && pi < n - 1 && pj > pi && pj < n;
      if (valid && pi == i) {
        const int slot = atomicAdd(&sh.cnt, 1);
        if (slot < kWideTargets) {
          sh.tq[slot] = q;
          sh.tj[slot] = pj;
        } else {
          for (int al = 0; al < 15; ++al) o[(size_t)q * 15 + al] = qnan;
        }
      } else if (!valid && i == 0) {
        for (int al = 0; al < 15; ++al) o[(size_t)q * 15 + al] = qnan;
      }
    }
    __syncthreads();
    const int nt = min(sh.cnt, kWideTargets);
    if (nt == 0) continue;
    if (tid == 0) {
      for (int x = 1; x < nt; ++x) {  // insertion sort by partner site
        const int kj = sh.tj[x], kq = sh.tq[x];
        int y = x - 1;
        while (y >= 0 && sh.tj[y] > kj) {
          sh.tj[y + 1] = sh.tj[y];
          sh.tq[y + 1] = sh.tq[y];
          --y;
        }
        sh.tj[y + 1] = kj;
        sh.tq[y + 1] = kq;
      }
    }
    __syncthreads();
    // open at site i: F^{ss'} = A^{sT} L_i conj(A^{s'})
    {
      const int Dl = dim(i - 1), Dc = dim(i);
      const T* A = st + (size_t)i * SLOT;
      const T* Ev = evl + (size_t)i * s2 * 2;
      for (int sp = 0; sp < 2; ++sp)
        tile_cgemm(gl, Dl, Dc, Dl, [&](int a, int ap) { return load_c<T, double>(Ev, (size_t)a * S + ap); },
                   [&](int ap, int cp) { return cconj(load_c<T, double>(A, (size_t)(ap * 2 + sp) * S + cp)); },
                   [&](int a, int cp, cd v) { Tm[(size_t)(sp * S + a) * S + cp] = v; });
      __syncthreads();
      for (int blk = 0; blk < 2; ++blk) {
        const int s = 0, sp = blk;
        tile_cgemm(gl, Dc, Dc, Dl, [&](int c, int a) { return load_c<T, double>(A, (size_t)(a * 2 + s) * S + c); },
                   [&](int a, int cp) { return Tm[(size_t)(sp * S + a) * S + cp]; },
                   [&](int c, int cp, cd v) { F[(size_t)(blk * S + c) * S + cp] = v; });
      }
      __syncthreads();
    }
    int cur = i + 1;
    for (int x = 0; x < nt; ++x) {
      const int j = sh.tj[x], q = sh.tq[x];
      for (; cur < j; ++cur) {
        const int Dc = dim(cur - 1), Dn = dim(cur);
        const T* A = st + (size_t)cur * SLOT;
        for (int bu = 0; bu < 4; ++bu) {
          const int blk = bu >> 1, u = bu & 1;
          tile_cgemm(gl, Dc, Dn, Dc, [&](int c, int cp) { return F[(size_t)(blk * S + c) * S + cp]; },
                     [&](int cp, int ep) { return cconj(load_c<T, double>(A, (size_t)(cp * 2 + u) * S + ep)); },
                     [&](int c, int ep, cd v) { Tm[(size_t)(bu * S + c) * S + ep] = v; });
        }
        __syncthreads();
        for (int blk = 0; blk < 2; ++blk)  // k runs over (u, c)
          tile_cgemm(gl, Dn, Dn, 2 * Dc,
                     [&](int e, int k) { const int u = k >= Dc, c = k - (u ? Dc : 0);
                                         return load_c<T, double>(A, (size_t)(c * 2 + u) * S + e); },
                     [&](int k, int ep) { const int u = k >= Dc, c = k - (u ? Dc : 0);
                                          return Tm[(size_t)((blk * 2 + u) * S + c) * S + ep]; },
                     [&](int e, int ep, cd v) { F[(size_t)(blk * S + e) * S + ep] = v; });
        __syncthreads();
      }
      // close at j: G^{tt'} = A^t R_{j+1} A^{t'H}; rho = sum F^{ss'} (.) G^{tt'}
      const int Dd = dim(j - 1), Dj = dim(j);
      const T* A = st + (size_t)j * SLOT;
      const T* Ev = evr + (size_t)(j + 1) * s2 * 2;
      for (int tp = 0; tp < 2; ++tp)
        tile_cgemm(gl, Dj, Dd, Dj, [&](int bb, int bp) { return load_c<T, double>(Ev, (size_t)bb * S + bp); },
                   [&](int bp, int dp) { return cconj(load_c<T, double>(A, (size_t)(dp * 2 + tp) * S + bp)); },
                   [&](int bb, int dp, cd v) { Tm[(size_t)(tp * S + bb) * S + dp] = v; });
      __syncthreads();
      for (int blk = 0; blk < 3; ++blk) {
        const int t = blk == 2 ? 1 : 0, tp = blk == 0 ? 0 : 1;
        tile_cgemm(gl, Dd, Dd, Dj, [&](int d, int bb) { return load_c<T, double>(A, (size_t)(d * 2 + t) * S + bb); },
                   [&](int bb, int dp) { return Tm[(size_t)(tp * S + bb) * S + dp]; },
                   [&](int d, int dp, cd v) { G[(size_t)(blk * S + d) * S + dp] = v; });
      }
      __syncthreads();
      // rho[(s,t),(s',t')], entry e = ((s*2+t)*2+s')*2+t'
      double part[32];
#pragma unroll
      for (int e = 0; e < 32; ++e) part[e] = 0.0;
      const T* Lj = evl + (size_t)j * s2 * 2;
      for (int idx = tid; idx < Dd * Dd; idx += kWT) {
        const int d = idx / Dd, dp = idx % Dd;
        const cd f00 = F[(size_t)d * S + dp], lj = load_c<T, double>(Lj, (size_t)d * S + dp);
        const cd f11{lj.re - f00.re, lj.im - f00.im};
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int s = e >> 3, t = (e >> 2) & 1, sp = (e >> 1) & 1, tp = e & 1;
          const cd f = (s == 1 && sp == 0) ? cconj(F[(size_t)(1 * S + dp) * S + d])
                       : (s == 1)          ? f11
                       : (sp == 1)         ? F[(size_t)(1 * S + d) * S + dp]
                                           : f00;
          const cd gg = (t == 1 && tp == 0) ? cconj(G[(size_t)(1 * S + dp) * S + d])
                                            : G[(size_t)((t + tp) * S + d) * S + dp];
          const cd fg = cmul(f, gg);
          part[2 * e] += fg.re;
          part[2 * e + 1] += fg.im;
        }
      }
#pragma unroll
      for (int e = 0; e < 32; ++e) {
        const double v = wv_sum(part[e]);
        if ((tid & 63) == 0) sh.part[tid >> 6][e] = v;
      }
      __syncthreads();
      if (tid < 32) {
        double v = 0.0;
        for (int wv = 0; wv < kWT / 64; ++wv) v += sh.part[wv][tid];
        sh.rho[tid] = v;
      }
      __syncthreads();
      if (tid < 15) {
        const int al = tid + 1, pa = al >> 2, pc = al & 3;
        double acc = 0.0;
        for (int e = 0; e < 16; ++e) {
          const int s = e >> 3, t = (e >> 2) & 1, sp = (e >> 1) & 1, tp = e & 1;
          const cd r{sh.rho[2 * e], sh.rho[2 * e + 1]};
          const cd wgt = cmul(pauli_w(pa, sp, s), pauli_w(pc, tp, t));
          acc += r.re * wgt.re - r.im * wgt.im;
        }
        o[(size_t)q * 15 + tid] = (T)acc;
      }
      __syncthreads();
    }
  }
}

}  // namespace

size_t wide_workspace_bytes(int S) { return ws_elems(S) * sizeof(cd); }

template <typename T>
hipError_t launch_layer_wide(T* state, double* ws, int n, int chi, int S, int layer, int batch,
                             int program, const double* theta, const double* phi,
                             const double* pixels, double* trunc_err, int* status, int n_layers,
                             hipStream_t stream) {
  if (S <= kMaxBond || S > 128) return hipErrorInvalidValue;
  hipError_t err = hipSuccess;
  if (launch_mpo_wide<T>(state, ws, ws_elems(S), n, chi, S, layer, batch, program, theta, phi,
                         pixels, trunc_err, status, n_layers, stream, err))
    return err;
  if (program == 1)
    hipLaunchKernelGGL((k_layer_wide<T, 1>), dim3(batch), dim3(kWT), 0, stream, state, (cd*)ws, n,
                       chi, S, layer, theta, phi, pixels, trunc_err, status, exact_qr());
  else
    hipLaunchKernelGGL((k_layer_wide<T, 0>), dim3(batch), dim3(kWT), 0, stream, state, (cd*)ws, n,
                       chi, S, layer, theta, phi, pixels, trunc_err, status, exact_qr());
  return hipGetLastError();
}

template <typename T>
hipError_t launch_measure_wide(const T* state, T* env, double* ws, const int* pairs, int m, int n,
                               int chi, int S, int layers, int batch, T* out, hipStream_t stream) {
  if (S <= kMaxBond || S > 128) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_env_wide<T>), dim3(2 * batch), dim3(kWT), 0, stream, state, env, (cd*)ws,
                     n, chi, S, layers);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || m == 0) return e;
  hipLaunchKernelGGL((k_pairs_wide<T>), dim3(batch * kWideGroups), dim3(kWT), 0, stream, state,
                     (const T*)env, (cd*)ws, pairs, m, n, chi, S, layers, out);
  return hipGetLastError();
}

template hipError_t launch_layer_wide<double>(double*, double*, int, int, int, int, int, int,
                                              const double*, const double*, const double*, double*,
                                              int*, int, hipStream_t);
template hipError_t launch_layer_wide<float>(float*, double*, int, int, int, int, int, int,
                                             const double*, const double*, const double*, double*,
                                             int*, int, hipStream_t);
template hipError_t launch_measure_wide<double>(const double*, double*, double*, const int*, int,
                                                int, int, int, int, int, double*, hipStream_t);
template hipError_t launch_measure_wide<float>(const float*, float*, double*, const int*, int, int,
                                               int, int, int, int, float*, hipStream_t);

}  // namespace anomps
