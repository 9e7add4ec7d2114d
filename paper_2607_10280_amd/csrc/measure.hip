// Measurement kernels: left/right environment sweeps and two-site reduced density matrices /
// Pauli-pair expectations on image-local pairs (§II-C, Eq. (4)-(5)).
//
// Environments: one wavefront per (image, side) walks the chain and stores every L_k / R_k.
// Pairs: one wavefront per (image, start site i) opens the two-layer block at i, carries it
// through the transfer matrices of the sites between i and each listed partner j (all
// partners of i share one pass), and closes it against A[j] and R_{j+1}.
#include "common.hpp"
#include "kernels.hpp"

namespace anomps {

constexpr int kMeasThreads = 64;
constexpr int kMaxTargets = 256;

template <typename C>
__device__ __forceinline__ C wsum(C v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

template <int S, typename T, typename C>
__device__ void load_site(cx<C>* dst, const T* slot, int Dl, int Dr) {
  for (int idx = threadIdx.x; idx < Dl * 2 * Dr; idx += kMeasThreads) {
    const int row = idx / Dr, b = idx % Dr;
    dst[row * S + b] = load_c<T, C>(slot, (size_t)row * S + b);
  }
}

// ------------------------------------------------------------------------- environments
// One image: st = its n slots, ev = its environment block of this side ([n+1][S][S]).
template <int S, typename T, typename C>
__device__ __forceinline__ void env_image(const T* st, C* ev, int n, int chi, int layers, int side) {
  using cc = cx<C>;
  __shared__ cc E[S * S];
  __shared__ cc A[2 * S * S];
  __shared__ cc Tm[2 * S * S];
  constexpr size_t SLOT = (size_t)2 * S * S * 2;
  const int tid = threadIdx.x;
  auto dim = [&](int k) { return bond_dim(n, chi, layers, k); };
  auto store_env = [&](int k, int D) {
    for (int idx = tid; idx < D * D; idx += kMeasThreads) {
      const int r = idx / D, c = idx % D;
      store_c<C, C>(ev + (size_t)k * S * S * 2, (size_t)r * S + c, E[r * S + c]);
    }
  };
  if (tid == 0) E[0] = cc{(C)1, (C)0};
  __syncthreads();
  if (side == 0) {
    store_env(0, 1);
    for (int k = 0; k < n; ++k) {
      const int Dl = dim(k - 1), Dr = dim(k);
      load_site<S, T, C>(A, st + (size_t)k * SLOT, Dl, Dr);
      __syncthreads();
      // Tm[s][a][b'] = sum_a' E[a][a'] conj(A[a'][s][b'])
      for (int idx = tid; idx < 2 * Dl * Dr; idx += kMeasThreads) {
        const int s = idx / (Dl * Dr), a = (idx / Dr) % Dl, bp = idx % Dr;
        cc acc{(C)0, (C)0};
        for (int ap = 0; ap < Dl; ++ap) cfma(acc, E[a * S + ap], cconj(A[(ap * 2 + s) * S + bp]));
        Tm[(s * S + a) * S + bp] = acc;
      }
      __syncthreads();
      // L_{k+1}[b][b'] = sum_s sum_a A[a][s][b] Tm[s][a][b']
      for (int idx = tid; idx < Dr * Dr; idx += kMeasThreads) {
        const int bb = idx / Dr, bp = idx % Dr;
        cc acc{(C)0, (C)0};
        for (int s = 0; s < 2; ++s)
          for (int a = 0; a < Dl; ++a) cfma(acc, A[(a * 2 + s) * S + bb], Tm[(s * S + a) * S + bp]);
        E[bb * S + bp] = acc;
      }
      __syncthreads();
      store_env(k + 1, Dr);
    }
  } else {
    store_env(n, 1);
    for (int k = n - 1; k >= 0; --k) {
      const int Dl = dim(k - 1), Dr = dim(k);
      load_site<S, T, C>(A, st + (size_t)k * SLOT, Dl, Dr);
      __syncthreads();
      // Tm[s][c][a'] = sum_c' E[c][c'] conj(A[a'][s][c'])
      for (int idx = tid; idx < 2 * Dr * Dl; idx += kMeasThreads) {
        const int s = idx / (Dr * Dl), c = (idx / Dl) % Dr, ap = idx % Dl;
        cc acc{(C)0, (C)0};
        for (int cp = 0; cp < Dr; ++cp) cfma(acc, E[c * S + cp], cconj(A[(ap * 2 + s) * S + cp]));
        Tm[(s * S + c) * S + ap] = acc;
      }
      __syncthreads();
      // R_k[a][a'] = sum_s sum_c A[a][s][c] Tm[s][c][a']
      for (int idx = tid; idx < Dl * Dl; idx += kMeasThreads) {
        const int a = idx / Dl, ap = idx % Dl;
        cc acc{(C)0, (C)0};
        for (int s = 0; s < 2; ++s)
          for (int c = 0; c < Dr; ++c) cfma(acc, A[(a * 2 + s) * S + c], Tm[(s * S + c) * S + ap]);
        E[a * S + ap] = acc;
      }
      __syncthreads();
      store_env(k, Dl);
    }
  }
}

template <int S, typename T, typename C>
__global__ __launch_bounds__(kMeasThreads) void k_env(const T* state, C* env, int n, int chi,
                                                      int layers) {
  constexpr size_t SLOT = (size_t)2 * S * S * 2;
  const int b = blockIdx.x >> 1, side = blockIdx.x & 1;
  env_image<S, T, C>(state + (size_t)b * n * SLOT,
                     env + ((size_t)b * 2 + side) * (n + 1) * S * S * 2, n, chi, layers, side);
}

// ------------------------------------------------------------------------- pairs
// Pauli matrix entry (P_a)[r][c], a in I,X,Y,Z.
template <typename C>
__device__ __forceinline__ cx<C> pauli_entry(int a, int r, int c) {
  switch (a) {
    case 0: return cx<C>{(C)(r == c), (C)0};
    case 1: return cx<C>{(C)(r != c), (C)0};
    case 2: return (r == c) ? cx<C>{(C)0, (C)0} : cx<C>{(C)0, (C)(r == 0 ? -1 : 1)};
    default: return (r == c) ? cx<C>{(C)(r == 0 ? 1 : -1), (C)0} : cx<C>{(C)0, (C)0};
  }
}

// blocks of a Hermitian-structured 2x2 block family stored as 00, 01, 11 (10 = 01^H)
__device__ __forceinline__ int blk_of(int s, int sp) { return s + sp; }  // 00->0, 01->1, 11->2

// One image and one start site i: st = its n slots, ev = its environments ([2][n+1][S][S]),
// out = its [m][15] outputs.
template <int S, typename T, typename C>
__device__ __forceinline__ void pairs_image(const T* st, const C* ev, const int* pairs, int m, int n, int chi,
                            int layers, int i, C* out) {
  using cc = cx<C>;
  __shared__ cc F[3 * S * S];
  __shared__ cc A[2 * S * S];
  __shared__ cc Tm[6 * S * S];
  __shared__ cc G[3 * S * S];
  __shared__ cc Ev[S * S];
  __shared__ int tq[kMaxTargets], tj[kMaxTargets];
  __shared__ int cnt;
  __shared__ C rho[32];
  constexpr size_t SLOT = (size_t)2 * S * S * 2;
  const int tid = threadIdx.x;
  auto dim = [&](int k) { return bond_dim(n, chi, layers, k); };
  const C qnan = (C)__builtin_nan("");
  auto nan_out = [&](int q) {
    for (int al = 0; al < 15; ++al) out[(size_t)q * 15 + al] = qnan;
  };

  if (tid == 0) cnt = 0;
  __syncthreads();
  for (int q = tid; q < m; q += kMeasThreads) {
    const int pi = pairs[2 * q], pj = pairs[2 * q + 1];
    const bool valid = pi >= 0 && pi < n - 1 && pj > pi && pj < n;
    if (valid && pi == i) {
      const int slot = atomicAdd(&cnt, 1);
      if (slot < kMaxTargets) {
        tq[slot] = q;
        tj[slot] = pj;
      } else {
        nan_out(q);
      }
    } else if (!valid && i == 0) {
      nan_out(q);
    }
  }
  __syncthreads();
  const int nt = min(cnt, kMaxTargets);
  if (nt == 0) return;
  if (tid == 0) {
    for (int x = 1; x < nt; ++x) {  // insertion sort by partner site
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
  // ---- open at site i: F^{ss'} = A^{sT} L_i conj(A^{s'})
  {
    const int Dl = dim(i - 1), Dc = dim(i);
    load_site<S, T, C>(A, st + (size_t)i * SLOT, Dl, Dc);
    for (int idx = tid; idx < Dl * Dl; idx += kMeasThreads)
      Ev[(idx / Dl) * S + idx % Dl] = load_c<C, C>(ev + (size_t)i * S * S * 2, (size_t)(idx / Dl) * S + idx % Dl);
    __syncthreads();
    for (int idx = tid; idx < 2 * Dl * Dc; idx += kMeasThreads) {
      const int sp = idx / (Dl * Dc), a = (idx / Dc) % Dl, cp = idx % Dc;
      cc acc{(C)0, (C)0};
      for (int ap = 0; ap < Dl; ++ap) cfma(acc, Ev[a * S + ap], cconj(A[(ap * 2 + sp) * S + cp]));
      Tm[(sp * S + a) * S + cp] = acc;
    }
    __syncthreads();
    for (int idx = tid; idx < 3 * Dc * Dc; idx += kMeasThreads) {
      const int blk = idx / (Dc * Dc), c = (idx / Dc) % Dc, cp = idx % Dc;
      const int s = blk == 2 ? 1 : 0, sp = blk == 0 ? 0 : 1;
      cc acc{(C)0, (C)0};
      for (int a = 0; a < Dl; ++a) cfma(acc, A[(a * 2 + s) * S + c], Tm[(sp * S + a) * S + cp]);
      F[(blk * S + c) * S + cp] = acc;
    }
    __syncthreads();
  }
  int cur = i + 1;
  for (int x = 0; x < nt; ++x) {
    const int j = tj[x], q = tq[x];
    // ---- propagate through sites cur .. j-1
    for (; cur < j; ++cur) {
      const int Dc = dim(cur - 1), Dn = dim(cur);
      load_site<S, T, C>(A, st + (size_t)cur * SLOT, Dc, Dn);
      __syncthreads();
      for (int idx = tid; idx < 6 * Dc * Dn; idx += kMeasThreads) {
        const int bu = idx / (Dc * Dn), c = (idx / Dn) % Dc, ep = idx % Dn;
        const int blk = bu >> 1, u = bu & 1;
        cc acc{(C)0, (C)0};
        for (int cp = 0; cp < Dc; ++cp)
          cfma(acc, F[(blk * S + c) * S + cp], cconj(A[(cp * 2 + u) * S + ep]));
        Tm[(bu * S + c) * S + ep] = acc;
      }
      __syncthreads();
      for (int idx = tid; idx < 3 * Dn * Dn; idx += kMeasThreads) {
        const int blk = idx / (Dn * Dn), e = (idx / Dn) % Dn, ep = idx % Dn;
        cc acc{(C)0, (C)0};
        for (int u = 0; u < 2; ++u)
          for (int c = 0; c < Dc; ++c)
            cfma(acc, A[(c * 2 + u) * S + e], Tm[((blk * 2 + u) * S + c) * S + ep]);
        F[(blk * S + e) * S + ep] = acc;
      }
      __syncthreads();
    }
    // ---- close at j: G^{tt'} = A^t R_{j+1} A^{t'H}; rho = sum F^{ss'} (.) G^{tt'}
    const int Dd = dim(j - 1), Dj = dim(j);
    load_site<S, T, C>(A, st + (size_t)j * SLOT, Dd, Dj);
    for (int idx = tid; idx < Dj * Dj; idx += kMeasThreads)
      Ev[(idx / Dj) * S + idx % Dj] = load_c<C, C>(ev + ((size_t)(n + 1) + j + 1) * S * S * 2, (size_t)(idx / Dj) * S + idx % Dj);
    __syncthreads();
    for (int idx = tid; idx < 2 * Dj * Dd; idx += kMeasThreads) {
      const int tp = idx / (Dj * Dd), bb = (idx / Dd) % Dj, dp = idx % Dd;
      cc acc{(C)0, (C)0};
      for (int bp = 0; bp < Dj; ++bp) cfma(acc, Ev[bb * S + bp], cconj(A[(dp * 2 + tp) * S + bp]));
      Tm[(tp * S + bb) * S + dp] = acc;
    }
    __syncthreads();
    for (int idx = tid; idx < 3 * Dd * Dd; idx += kMeasThreads) {
      const int blk = idx / (Dd * Dd), d = (idx / Dd) % Dd, dp = idx % Dd;
      const int t = blk == 2 ? 1 : 0, tp = blk == 0 ? 0 : 1;
      cc acc{(C)0, (C)0};
      for (int bb = 0; bb < Dj; ++bb) cfma(acc, A[(d * 2 + t) * S + bb], Tm[(tp * S + bb) * S + dp]);
      G[(blk * S + d) * S + dp] = acc;
    }
    __syncthreads();
    // rho[(s,t),(s',t')], entry e = ((s*2+t)*2+s')*2+t'
    C part[32];
#pragma unroll
    for (int e = 0; e < 32; ++e) part[e] = (C)0;
    for (int idx = tid; idx < Dd * Dd; idx += kMeasThreads) {
      const int d = idx / Dd, dp = idx % Dd;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int s = e >> 3, t = (e >> 2) & 1, sp = (e >> 1) & 1, tp = e & 1;
        const cc f = (s == 1 && sp == 0) ? cconj(F[(1 * S + dp) * S + d]) : F[(blk_of(s, sp) * S + d) * S + dp];
        const cc g = (t == 1 && tp == 0) ? cconj(G[(1 * S + dp) * S + d]) : G[(blk_of(t, tp) * S + d) * S + dp];
        const cc fg = cmul(f, g);
        part[2 * e] += fg.re;
        part[2 * e + 1] += fg.im;
      }
    }
#pragma unroll
    for (int e = 0; e < 32; ++e) part[e] = wsum<C>(part[e]);
    if (tid < 32) {
      C v = (C)0;
#pragma unroll
      for (int e = 0; e < 32; ++e) v = (tid == e) ? part[e] : v;
      rho[tid] = v;
    }
    __syncthreads();
    if (tid < 15) {
      const int al = tid + 1, pa = al >> 2, pc = al & 3;
      C acc = (C)0;
      for (int e = 0; e < 16; ++e) {
        const int s = e >> 3, t = (e >> 2) & 1, sp = (e >> 1) & 1, tp = e & 1;
        const cc r{rho[2 * e], rho[2 * e + 1]};
        const cc w = cmul(pauli_entry<C>(pa, sp, s), pauli_entry<C>(pc, tp, t));
        acc += r.re * w.re - r.im * w.im;
      }
      out[(size_t)q * 15 + tid] = acc;
    }
    __syncthreads();
  }
}

template <int S, typename T, typename C>
__global__ __launch_bounds__(kMeasThreads) void k_pairs(const T* state, const C* env,
                                                        const int* pairs, int m, int n, int chi,
                                                        int layers, C* out) {
  constexpr size_t SLOT = (size_t)2 * S * S * 2;
  const int i = blockIdx.x % (n - 1), b = blockIdx.x / (n - 1);
  pairs_image<S, T, C>(state + (size_t)b * n * SLOT, env + (size_t)b * 2 * (n + 1) * S * S * 2,
                       pairs, m, n, chi, layers, i, out + (size_t)b * m * 15);
}

// ------------------------------------------------------------------------- mixed requests
// Table entries [begin, begin + count) share the slot size S and the precision.  Environments:
// one workgroup per (request, side); pairs: one per (request, start site), the grid sized for
// the bucket's largest chain (workgroups past a request's last start site exit at once).
template <int S, typename T, typename C>
__global__ __launch_bounds__(kMeasThreads) void k_env_mixed(const mps_request* reqs, int begin) {
  const mps_request* r = reqs + begin + (blockIdx.x >> 1);
  const int side = blockIdx.x & 1, n = uniform_int(r->n_sites);
  const int layers = uniform_int(uniform_ptr(r->ctrl)[0]);
  env_image<S, T, C>(uniform_ptr((const T*)r->state),
                     uniform_ptr((C*)r->env) + (size_t)side * (n + 1) * S * S * 2, n,
                     uniform_int(r->chi), layers, side);
}

template <int S, typename T, typename C>
__global__ __launch_bounds__(kMeasThreads) void k_pairs_mixed(const mps_request* reqs, int begin,
                                                              int max_sites) {
  const mps_request* r = reqs + begin + blockIdx.x / (max_sites - 1);
  const int i = blockIdx.x % (max_sites - 1), n = uniform_int(r->n_sites);
  const int m = uniform_int(r->n_pairs);
  if (i >= n - 1 || m == 0) return;
  const int layers = uniform_int(uniform_ptr(r->ctrl)[0]);
  pairs_image<S, T, C>(uniform_ptr((const T*)r->state), uniform_ptr((const C*)r->env),
                       uniform_ptr(r->pairs), m, n, uniform_int(r->chi), layers, i,
                       uniform_ptr((C*)r->out));
}

template <typename T, typename C>
hipError_t launch_measure_mixed(const mps_request* reqs, int begin, int count, int max_sites,
                                int S, hipStream_t stream) {
  if (count == 0) return hipSuccess;
  const dim3 ge(2 * count), gp((unsigned)((size_t)count * (max_sites - 1))), block(kMeasThreads);
  switch (S) {
#define ANOMPS_MM(SV)                                                                          \
  case SV:                                                                                     \
    hipLaunchKernelGGL((k_env_mixed<SV, T, C>), ge, block, 0, stream, reqs, begin);           \
    hipLaunchKernelGGL((k_pairs_mixed<SV, T, C>), gp, block, 0, stream, reqs, begin, max_sites); \
    break;
    ANOMPS_MM(2) ANOMPS_MM(4) ANOMPS_MM(8) ANOMPS_MM(16)
#undef ANOMPS_MM
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------------- launchers
template <typename T, typename C>
hipError_t launch_envs(const T* state, C* env, int n, int chi, int S, int layers, int batch,
                       hipStream_t stream) {
  const dim3 grid(2 * batch), block(kMeasThreads);
  switch (S) {
    case 2: hipLaunchKernelGGL((k_env<2, T, C>), grid, block, 0, stream, state, env, n, chi, layers); break;
    case 4: hipLaunchKernelGGL((k_env<4, T, C>), grid, block, 0, stream, state, env, n, chi, layers); break;
    case 8: hipLaunchKernelGGL((k_env<8, T, C>), grid, block, 0, stream, state, env, n, chi, layers); break;
    case 16: hipLaunchKernelGGL((k_env<16, T, C>), grid, block, 0, stream, state, env, n, chi, layers); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, typename C>
hipError_t launch_pairs(const T* state, const C* env, const int* pairs, int m, int n, int chi,
                        int S, int layers, int batch, C* out, hipStream_t stream) {
  if (m == 0) return hipSuccess;
  const dim3 grid((unsigned)((size_t)(n - 1) * batch)), block(kMeasThreads);
  switch (S) {
    case 2: hipLaunchKernelGGL((k_pairs<2, T, C>), grid, block, 0, stream, state, env, pairs, m, n, chi, layers, out); break;
    case 4: hipLaunchKernelGGL((k_pairs<4, T, C>), grid, block, 0, stream, state, env, pairs, m, n, chi, layers, out); break;
    case 8: hipLaunchKernelGGL((k_pairs<8, T, C>), grid, block, 0, stream, state, env, pairs, m, n, chi, layers, out); break;
    case 16: hipLaunchKernelGGL((k_pairs<16, T, C>), grid, block, 0, stream, state, env, pairs, m, n, chi, layers, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template hipError_t launch_envs<double, double>(const double*, double*, int, int, int, int, int, hipStream_t);
template hipError_t launch_envs<float, float>(const float*, float*, int, int, int, int, int, hipStream_t);
template hipError_t launch_pairs<double, double>(const double*, const double*, const int*, int, int, int, int, int, int, double*, hipStream_t);
template hipError_t launch_pairs<float, float>(const float*, const float*, const int*, int, int, int, int, int, int, float*, hipStream_t);
template hipError_t launch_measure_mixed<double, double>(const mps_request*, int, int, int, int, hipStream_t);
template hipError_t launch_measure_mixed<float, float>(const mps_request*, int, int, int, int, hipStream_t);

}  // namespace anomps
