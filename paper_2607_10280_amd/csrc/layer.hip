// Encoding and layer kernels: the one-qubit updates, the right-to-left canonical sweep and the
// CNOT ladder with FP64 one-sided Jacobi SVD truncation (§II-B).
//
// One workgroup (a single 64-lane wavefront) owns one image and walks its chain; images are
// independent, so a batch fills the machine with one wavefront per image.  Site tensors live
// in HBM in the slot layout [site][S][2][S] (storage type T: double or float); the tensors of
// the current bond are staged in LDS in FP64 and every factorisation runs in FP64.
#include "common.hpp"
#include "kernels.hpp"

namespace anomps {

constexpr int kLayerThreads = 64;
constexpr int kMaxSweeps = 30;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// ------------------------------------------------------------------------------- encode
// One workgroup per image: writes A[k] = (cos(pi x_k/2), sin(pi x_k/2)) as a 1x2x1 tensor and
// (re)sets the image's status word (NaN/Inf pixels -> non-finite).
template <typename T>
__global__ void k_encode(T* state, const double* pixels, int n, int S, int* status) {
  const int b = blockIdx.x;
  int bad = 0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const double x = pixels[(size_t)b * n + k];
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
template <int S>
struct LayerShared {
  cd mat[(2 * S) * (2 * S)];  // column-major working matrix, leading dimension 2S
  cd ta[2 * S * S];           // centre tensor [a][s][c] at (a*2+s)*S + c
  cd tb[2 * S * S];           // neighbour tensor [c][t][b] at (c*2+t)*S + b
  cd uq[2 * S * S];           // U [r][j] at r*S + j  (ladder) or V*Sigma [j][a] at j*S + a (sweep)
  double sig2[2 * S];
  int order[2 * S];
};

// One-sided (Hestenes) Jacobi on the N columns (length M) of `mat` in FP64.  Column pairs are
// scheduled by the round-robin tournament (N-1 rounds of disjoint pairs per sweep); a team of
// T lanes owns one pair per round and reduces its three inner products with lane shuffles.
// A pair is rotated when |x^H y| > tol sqrt(|x|^2 |y|^2); columns whose squared norm is below
// tiny2 = 1e-30 |A|_F^2 are treated as numerically zero.  On return sig2[c] = |w_c|^2.
template <int S>
__device__ int jacobi_columns(LayerShared<S>& sh, int M, int N, double* tiny2_out) {
  constexpr int LD = 2 * S;
  constexpr int RMAX = (2 * S * S + kLayerThreads - 1) / kLayerThreads > 0
                           ? (2 * S * S + kLayerThreads - 1) / kLayerThreads
                           : 1;
  const int tid = threadIdx.x;
  double f = 0.0;
  for (int idx = tid; idx < M * N; idx += kLayerThreads) {
    const cd v = sh.mat[(idx / M) * LD + (idx % M)];
    f += v.re * v.re + v.im * v.im;
  }
  f = wave_sum(f);
  const double tiny2 = 1e-30 * f;
  *tiny2_out = tiny2;
  const double tol = (double)M * 2.220446049250313e-16;
  const int Nr = N + (N & 1);
  const int P = Nr / 2;
  int T = 64;
  while (T * P > kLayerThreads) T >>= 1;
  const int q = tid / T;
  const int lt = tid % T;
  const bool active = q < P;
  int sweep = 0;
  bool converged = (N < 2);
  for (; !converged && sweep < kMaxSweeps; ++sweep) {
    int rotated = 0;
    for (int r = 0; r < Nr - 1; ++r) {
      int ci = 0, cj = 0;
      if (active) {
        ci = (q == 0) ? 0 : 1 + (q - 1 + r) % (Nr - 1);
        const int p2 = Nr - 1 - q;
        cj = 1 + (p2 - 1 + r) % (Nr - 1);
      }
      const bool valid = active && ci < N && cj < N;
      cd x[RMAX], y[RMAX];
      double a = 0.0, bb = 0.0, gr = 0.0, gi = 0.0;
#pragma unroll
      for (int t = 0; t < RMAX; ++t) {
        const int rr = lt + t * T;
        if (valid && rr < M) {
          x[t] = sh.mat[ci * LD + rr];
          y[t] = sh.mat[cj * LD + rr];
          a = fma(x[t].re, x[t].re, fma(x[t].im, x[t].im, a));
          bb = fma(y[t].re, y[t].re, fma(y[t].im, y[t].im, bb));
          gr = fma(x[t].re, y[t].re, fma(x[t].im, y[t].im, gr));
          gi = fma(x[t].re, y[t].im, fma(-x[t].im, y[t].re, gi));
        }
      }
      for (int off = T >> 1; off >= 1; off >>= 1) {
        a += __shfl_xor(a, off);
        bb += __shfl_xor(bb, off);
        gr += __shfl_xor(gr, off);
        gi += __shfl_xor(gi, off);
      }
      if (valid) {
        const double ag = hypot(gr, gi);
        if (a > tiny2 && bb > tiny2 && ag > tol * sqrt(a * bb)) {
          rotated = 1;
          const double zeta = (bb - a) / (2.0 * ag);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
          const double c = 1.0 / sqrt(1.0 + t * t);
          const double s = c * t;
          const cd e{gr / ag, -gi / ag};  // conj(g)/|g|
#pragma unroll
          for (int tt = 0; tt < RMAX; ++tt) {
            const int rr = lt + tt * T;
            if (rr < M) {
              const cd ye = cmul(e, y[tt]);
              sh.mat[ci * LD + rr] = cd{c * x[tt].re - s * ye.re, c * x[tt].im - s * ye.im};
              sh.mat[cj * LD + rr] = cd{s * x[tt].re + c * ye.re, s * x[tt].im + c * ye.im};
            }
          }
        }
      }
      __syncthreads();
    }
    converged = !__syncthreads_or(rotated);
  }
  for (int col = tid; col < N; col += kLayerThreads) {
    double s2 = 0.0;
    for (int r = 0; r < M; ++r) {
      const cd v = sh.mat[col * LD + r];
      s2 = fma(v.re, v.re, fma(v.im, v.im, s2));
    }
    sh.sig2[col] = s2;
  }
  __syncthreads();
  return converged ? 0 : kImgNoConvergence;
}

// Apply U = R_Y(theta) R_Z(phi) to the physical index of the (Dl x 2 x Dr) tensor in ta.
template <int S>
__device__ void apply_gate(LayerShared<S>& sh, int Dl, int Dr, double theta, double phi) {
  double st, ct, sp, cp;
  sincos(0.5 * theta, &st, &ct);
  sincos(0.5 * phi, &sp, &cp);
  const cd em{cp, -sp}, ep{cp, sp};  // e^{-i phi/2}, e^{+i phi/2}
  const cd u00 = cscale(em, ct), u01 = cscale(ep, -st);
  const cd u10 = cscale(em, st), u11 = cscale(ep, ct);
  for (int idx = threadIdx.x; idx < Dl * Dr; idx += kLayerThreads) {
    const int a = idx / Dr, b = idx % Dr;
    const cd v0 = sh.ta[(a * 2 + 0) * S + b];
    const cd v1 = sh.ta[(a * 2 + 1) * S + b];
    cd w0 = cmul(u00, v0), w1 = cmul(u10, v0);
    cfma(w0, u01, v1);
    cfma(w1, u11, v1);
    sh.ta[(a * 2 + 0) * S + b] = w0;
    sh.ta[(a * 2 + 1) * S + b] = w1;
  }
  __syncthreads();
}

template <int S, typename T>
__device__ void load_tensor(cd* dst, const T* slot, int Dl, int Dr) {
  for (int idx = threadIdx.x; idx < Dl * 2 * Dr; idx += kLayerThreads) {
    const int row = idx / Dr, b = idx % Dr;  // row = a*2 + s
    dst[row * S + b] = load_c<T, double>(slot, (size_t)row * S + b);
  }
}

template <int S, typename T>
__device__ void store_tensor(T* slot, const cd* src, int Dl, int Dr) {
  for (int idx = threadIdx.x; idx < Dl * 2 * Dr; idx += kLayerThreads) {
    const int row = idx / Dr, b = idx % Dr;
    store_c<T, double>(slot, (size_t)row * S + b, src[row * S + b]);
  }
}

// Applies layer `layer` (0-based) to one image whose n slots start at `st`.
template <int S, typename T>
__device__ void layer_chain(LayerShared<S>& sh, T* st, int n, int chi, int layer,
                            const double* theta, const double* phi, double* trunc_err,
                            int* status) {
  constexpr int LD = 2 * S;
  constexpr size_t SLOT = (size_t)2 * S * S * 2;  // T values per site slot
  const int tid = threadIdx.x;
  int flags = 0;
  auto dold = [&](int k) { return bond_dim(n, chi, layer, k); };
  auto dnew = [&](int k) { return bond_dim(n, chi, layer + 1, k); };

  // ---- right-to-left sweep: gate every site, make sites n-1..1 right-canonical.
  load_tensor<S, T>(sh.ta, st + (size_t)(n - 1) * SLOT, dold(n - 2), 1);
  __syncthreads();
  for (int k = n - 1; k >= 1; --k) {
    const int Dl = dold(k - 1), Dr = dold(k);
    apply_gate<S>(sh, Dl, Dr, theta[k], phi[k]);
    // mat = t^H: rows (s, b) -> s*Dr + b, columns a.
    const int M = 2 * Dr, N = Dl;
    for (int idx = tid; idx < N * M; idx += kLayerThreads) {
      const int a = idx / M, rr = idx % M;
      const int s = rr / Dr, b = rr % Dr;
      sh.mat[a * LD + rr] = cconj(sh.ta[(a * 2 + s) * S + b]);
    }
    __syncthreads();
    double tiny2;
    flags |= jacobi_columns<S>(sh, M, N, &tiny2);
    // Right-canonical rows q_a^H and V*Sigma = t Q.
    T* slot = st + (size_t)k * SLOT;
    for (int idx = tid; idx < N * M; idx += kLayerThreads) {
      const int a = idx / M, rr = idx % M;
      const int s = rr / Dr, b = rr % Dr;
      const double s2 = sh.sig2[a];
      cd v{0.0, 0.0};
      if (s2 > tiny2) v = cscale(cconj(sh.mat[a * LD + rr]), 1.0 / sqrt(s2));
      store_c<T, double>(slot, (size_t)(a * 2 + s) * S + b, v);
    }
    for (int idx = tid; idx < N * N; idx += kLayerThreads) {
      const int j = idx / N, a = idx % N;
      const double s2 = sh.sig2[a];
      cd acc{0.0, 0.0};
      if (s2 > tiny2) {
        for (int rr = 0; rr < M; ++rr) {
          const int s = rr / Dr, b = rr % Dr;
          cfma(acc, sh.ta[(j * 2 + s) * S + b], sh.mat[a * LD + rr]);
        }
        acc = cscale(acc, 1.0 / sqrt(s2));
      }
      sh.uq[j * S + a] = acc;
    }
    const int Dll = dold(k - 2);
    load_tensor<S, T>(sh.tb, st + (size_t)(k - 1) * SLOT, Dll, Dl);
    __syncthreads();
    for (int idx = tid; idx < Dll * 2 * Dl; idx += kLayerThreads) {
      const int row = idx / Dl, a = idx % Dl;
      cd acc{0.0, 0.0};
      for (int j = 0; j < Dl; ++j) cfma(acc, sh.tb[row * S + j], sh.uq[j * S + a]);
      sh.ta[row * S + a] = acc;
    }
    __syncthreads();
  }
  apply_gate<S>(sh, 1, dold(0), theta[0], phi[0]);

  // ---- left-to-right CNOT ladder with SVD truncation.
  for (int k = 0; k <= n - 2; ++k) {
    const int Dl = dnew(k - 1), Dc = dold(k), Dr = dold(k + 1);
    load_tensor<S, T>(sh.tb, st + (size_t)(k + 1) * SLOT, Dc, Dr);
    __syncthreads();
    const int M = 2 * Dl, N = 2 * Dr;
    // Theta'[(a,s),(t,b)] = sum_c A[k][a,s,c] A[k+1][c, t XOR s, b]   (CNOT control k)
    for (int idx = tid; idx < M * N; idx += kLayerThreads) {
      const int col = idx / M, row = idx % M;
      const int t = col / Dr, b = col % Dr, s = row & 1;
      cd acc{0.0, 0.0};
      for (int c = 0; c < Dc; ++c) cfma(acc, sh.ta[row * S + c], sh.tb[(c * 2 + (t ^ s)) * S + b]);
      sh.mat[col * LD + row] = acc;
    }
    __syncthreads();
    double tiny2;
    flags |= jacobi_columns<S>(sh, M, N, &tiny2);
    const int D = min(chi, min(M, N));
    // Sort singular values (descending, ties by column index); NaN counts as zero.
    for (int c = tid; c < N; c += kLayerThreads) {
      double v = sh.sig2[c];
      if (!(v >= 0.0)) v = 0.0;
      int rank = 0;
      for (int i = 0; i < N; ++i) {
        double w = sh.sig2[i];
        if (!(w >= 0.0)) w = 0.0;
        rank += (w > v) || (w == v && i < c);
      }
      sh.order[rank] = c;
    }
    __syncthreads();
    double kept = 0.0, disc = 0.0;
    for (int r = 0; r < N; ++r) {
      const double v = sh.sig2[sh.order[r]];
      if (r < D) kept += v; else disc += v;
    }
    if (!isfinite(kept) || !isfinite(disc) || !(kept > 0.0)) flags |= kImgNonfinite;
    const double inv_norm = (kept > 0.0) ? 1.0 / sqrt(kept) : 0.0;
    if (tid == 0 && trunc_err) trunc_err[k] = (kept + disc > 0.0) ? disc / (kept + disc) : 0.0;
    // U columns = normalised kept columns of W (numerically zero columns become zero).
    for (int idx = tid; idx < M * D; idx += kLayerThreads) {
      const int r = idx / D, j = idx % D;
      const int c = sh.order[j];
      const double s2 = sh.sig2[c];
      cd v{0.0, 0.0};
      if (s2 > tiny2) v = cscale(sh.mat[c * LD + r], 1.0 / sqrt(s2));
      sh.uq[r * S + j] = v;
    }
    __syncthreads();
    store_tensor<S, T>(st + (size_t)k * SLOT, sh.uq, Dl, D);
    // X_s = U_s^H A_s  ->  mat[(s*S + j)*S + c]
    for (int idx = tid; idx < 2 * D * Dc; idx += kLayerThreads) {
      const int s = idx / (D * Dc), j = (idx / Dc) % D, c = idx % Dc;
      cd acc{0.0, 0.0};
      for (int a = 0; a < Dl; ++a) cfmac(acc, sh.uq[(a * 2 + s) * S + j], sh.ta[(a * 2 + s) * S + c]);
      sh.mat[(s * S + j) * S + c] = acc;
    }
    __syncthreads();
    // New centre S V^H = U^H Theta' / |sigma_kept|  ->  ta[(j*2+t)*S + b]
    for (int idx = tid; idx < D * 2 * Dr; idx += kLayerThreads) {
      const int j = idx / (2 * Dr), t = (idx / Dr) & 1, b = idx % Dr;
      cd acc{0.0, 0.0};
      for (int s = 0; s < 2; ++s)
        for (int c = 0; c < Dc; ++c)
          cfma(acc, sh.mat[(s * S + j) * S + c], sh.tb[(c * 2 + (t ^ s)) * S + b]);
      sh.ta[(j * 2 + t) * S + b] = cscale(acc, inv_norm);
    }
    __syncthreads();
  }
  store_tensor<S, T>(st + (size_t)(n - 1) * SLOT, sh.ta, dnew(n - 2), 1);
  if (tid == 0 && flags) status[0] |= flags;
}

template <int S, typename T>
__global__ __launch_bounds__(kLayerThreads) void k_layer(T* state, int n, int chi, int layer,
                                                         const double* theta, const double* phi,
                                                         double* trunc_err, int* status) {
  __shared__ LayerShared<S> sh;
  const int b = blockIdx.x;
  T* st = state + (size_t)b * n * ((size_t)2 * S * S * 2);
  layer_chain<S, T>(sh, st, n, chi, layer, theta, phi,
                    trunc_err ? trunc_err + (size_t)b * (n - 1) : nullptr, status + b);
}

// ------------------------------------------------------------------------------- launchers
template <typename T>
hipError_t launch_encode(T* state, const double* pixels, int n, int S, int batch, int* status,
                         hipStream_t stream) {
  hipLaunchKernelGGL(k_encode<T>, dim3(batch), dim3(64), 0, stream, state, pixels, n, S, status);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_layer(T* state, int n, int chi, int S, int layer, int batch,
                        const double* theta, const double* phi, double* trunc_err, int* status,
                        hipStream_t stream) {
  const dim3 grid(batch), block(kLayerThreads);
  switch (S) {
    case 2: hipLaunchKernelGGL((k_layer<2, T>), grid, block, 0, stream, state, n, chi, layer, theta, phi, trunc_err, status); break;
    case 4: hipLaunchKernelGGL((k_layer<4, T>), grid, block, 0, stream, state, n, chi, layer, theta, phi, trunc_err, status); break;
    case 8: hipLaunchKernelGGL((k_layer<8, T>), grid, block, 0, stream, state, n, chi, layer, theta, phi, trunc_err, status); break;
    case 16: hipLaunchKernelGGL((k_layer<16, T>), grid, block, 0, stream, state, n, chi, layer, theta, phi, trunc_err, status); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template hipError_t launch_encode<double>(double*, const double*, int, int, int, int*, hipStream_t);
template hipError_t launch_encode<float>(float*, const double*, int, int, int, int*, hipStream_t);
template hipError_t launch_layer<double>(double*, int, int, int, int, int, const double*,
                                         const double*, double*, int*, hipStream_t);
template hipError_t launch_layer<float>(float*, int, int, int, int, int, const double*,
                                        const double*, double*, int*, hipStream_t);

}  // namespace anomps
