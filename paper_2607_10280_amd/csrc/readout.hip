// Adaptive-observable readout: Pauli-basis coefficients of H_q (Eq. (4)), features by linearity
// (Eq. (5)) and the linear reconstruction y = W q + b (Eq. (6)).
#include "common.hpp"
#include "kernels.hpp"

namespace anomps {

template <typename R>
__device__ __forceinline__ cx<R> pauli_e(int a, int r, int c) {
  switch (a) {
    case 0: return cx<R>{(R)(r == c), (R)0};
    case 1: return cx<R>{(R)(r != c), (R)0};
    case 2: return (r == c) ? cx<R>{(R)0, (R)0} : cx<R>{(R)0, (R)(r == 0 ? -1 : 1)};
    default: return (r == c) ? cx<R>{(R)(r == 0 ? 1 : -1), (R)0} : cx<R>{(R)0, (R)0};
  }
}

// One thread per (observable, alpha): coeff[q][alpha] = Re Tr(H_q (P_a (x) P_c)) / 4.
template <typename R>
__global__ void k_coeffs(const R* A, const R* B, const R* D, int m, R* coeff) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= m * 16) return;
  const int q = gid / 16, al = gid % 16, pa = al >> 2, pc = al & 3;
  // H[j][k]: diagonal D, upper (0,1),(0,2),(0,3),(1,2),(1,3),(2,3) = A + iB, lower = conj.
  auto h = [&](int j, int k) -> cx<R> {
    if (j == k) return cx<R>{D[q * 4 + j], (R)0};
    const int lo = j < k ? j : k, hi = j < k ? k : j;
    const int idx = lo == 0 ? hi - 1 : (lo == 1 ? hi + 1 : 5);
    const R im = B[q * 6 + idx];
    return cx<R>{A[q * 6 + idx], j < k ? im : -im};
  };
  R acc = (R)0;
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) {
      // (P_a (x) P_c)[c][r] with row/col index s_i*2 + s_j
      const cx<R> p = cmul(pauli_e<R>(pa, c >> 1, r >> 1), pauli_e<R>(pc, c & 1, r & 1));
      const cx<R> hv = h(r, c);
      acc += hv.re * p.re - hv.im * p.im;
    }
  coeff[gid] = (R)0.25 * acc;
}

// y[b][o] = sum_j W[o][j] q_b[j] + bias[o], q_b[j] = c_j0 + sum_alpha c_j,alpha <P_alpha>_bj.
// One workgroup per (block of kRoOut outputs, block of kRoImg images): the block's rows of W
// (contiguous in memory) and the images' q vectors are staged in LDS, so W is read once per
// image block instead of once per image, and every global read is coalesced.  LDS rows are
// padded to an odd stride so that lanes on consecutive rows fall on different banks.
constexpr int kRoOut = 128, kRoImg = 16, kRoThreads = 256;
constexpr size_t kRoLds = 64 * 1024;  // LDS budget of one block

__host__ __device__ inline int ro_stride(int m) { return m | 1; }

template <typename R>
__global__ __launch_bounds__(kRoThreads) void k_readout(const R* pauli, const R* coeff, const R* W,
                                                        const R* bias, int batch, int m,
                                                        int out_dim, int ob, int ib, R* y) {
  extern __shared__ unsigned char smem[];
  const int mp = ro_stride(m);
  R* ws = reinterpret_cast<R*>(smem);  // [ob][mp]
  R* qs = ws + (size_t)ob * mp;         // [ib][mp]
  const int o0 = blockIdx.x * ob, b0 = blockIdx.y * ib, tid = threadIdx.x;
  const int no = min(ob, out_dim - o0), nb = min(ib, batch - b0);
  for (int idx = tid; idx < no * m; idx += kRoThreads) {
    const int oo = idx / m, jj = idx - oo * m;
    ws[oo * mp + jj] = W[(size_t)o0 * m + idx];
  }
  for (int idx = tid; idx < nb * m; idx += kRoThreads) {
    const int bi = idx / m, jj = idx - bi * m;
    const R* pb = pauli + ((size_t)(b0 + bi) * m + jj) * 15;
    R acc = coeff[jj * 16];
    for (int al = 0; al < 15; ++al) acc += coeff[jj * 16 + al + 1] * pb[al];
    qs[bi * mp + jj] = acc;
  }
  __syncthreads();
  // Each lane: images 2 ip, 2 ip + 1 and outputs oq + 32 u (u < 4), so that a step of the sum
  // reads 4 + 2 LDS values for 8 products; rows past the block's images or outputs are clamped
  // to the last one (in bounds) and not stored.  Each sum runs over j in order, as a plain dot.
  for (int item = tid; item < ((nb + 1) / 2) * 32; item += kRoThreads) {
    const int ip = item / 32, oq = item % 32;
    const R* wr[4];
    const R* qv[2];
    R acc[2][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) wr[u] = ws + min(oq + 32 * u, no - 1) * mp;
#pragma unroll
    for (int v = 0; v < 2; ++v) qv[v] = qs + min(2 * ip + v, nb - 1) * mp;
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int o = min(oq + 32 * u, no - 1);
        acc[v][u] = bias ? bias[o0 + o] : (R)0;
      }
    for (int jj = 0; jj < m; ++jj) {
      const R q0 = qv[0][jj], q1 = qv[1][jj];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const R w = wr[u][jj];
        acc[0][u] += w * q0;
        acc[1][u] += w * q1;
      }
    }
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int bi = 2 * ip + v, o = oq + 32 * u;
        if (bi < nb && o < no) y[(size_t)(b0 + bi) * out_dim + o0 + o] = acc[v][u];
      }
  }
}

// Feature vectors too long for two LDS rows of the blocked kernel: one workgroup per image.
template <typename R>
__global__ void k_readout_image(const R* pauli, const R* coeff, const R* W, const R* bias, int m,
                                int out_dim, R* y) {
  extern __shared__ unsigned char smem[];
  R* qv = reinterpret_cast<R*>(smem);
  const int b = blockIdx.x;
  const R* pb = pauli + (size_t)b * m * 15;
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    R acc = coeff[j * 16];
    for (int al = 0; al < 15; ++al) acc += coeff[j * 16 + al + 1] * pb[j * 15 + al];
    qv[j] = acc;
  }
  __syncthreads();
  for (int o = threadIdx.x; o < out_dim; o += blockDim.x) {
    R acc = bias ? bias[o] : (R)0;
    const R* wr = W + (size_t)o * m;
    for (int j = 0; j < m; ++j) acc += wr[j] * qv[j];
    y[(size_t)b * out_dim + o] = acc;
  }
}

template <typename R>
hipError_t launch_coeffs(const R* A, const R* B, const R* D, int m, R* coeff, hipStream_t stream) {
  if (m == 0) return hipSuccess;
  const int threads = 256;
  hipLaunchKernelGGL(k_coeffs<R>, dim3((m * 16 + threads - 1) / threads), dim3(threads), 0, stream,
                     A, B, D, m, coeff);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_readout(const R* pauli, const R* coeff, const R* W, const R* bias, int batch,
                          int m, int out_dim, R* y, hipStream_t stream) {
  if (batch == 0 || out_dim == 0) return hipSuccess;
  const size_t row = (size_t)ro_stride(m) * sizeof(R);
  int ob = out_dim < kRoOut ? out_dim : kRoOut, ib = batch < kRoImg ? batch : kRoImg;
  while ((size_t)(ob + ib) * row > kRoLds && ob > 1) ob = (ob + 1) / 2;
  while ((size_t)(ob + ib) * row > kRoLds && ib > 1) ib = (ib + 1) / 2;
  if ((size_t)(ob + ib) * row > kRoLds) {
    hipLaunchKernelGGL(k_readout_image<R>, dim3(batch), dim3(256), (size_t)m * sizeof(R), stream,
                       pauli, coeff, W, bias, m, out_dim, y);
    return hipGetLastError();
  }
  const dim3 grid((unsigned)((out_dim + ob - 1) / ob), (unsigned)((batch + ib - 1) / ib));
  hipLaunchKernelGGL(k_readout<R>, grid, dim3(kRoThreads), (size_t)(ob + ib) * row, stream, pauli,
                     coeff, W, bias, batch, m, out_dim, ob, ib, y);
  return hipGetLastError();
}

template hipError_t launch_coeffs<double>(const double*, const double*, const double*, int, double*, hipStream_t);
template hipError_t launch_coeffs<float>(const float*, const float*, const float*, int, float*, hipStream_t);
template hipError_t launch_readout<double>(const double*, const double*, const double*, const double*, int, int, int, double*, hipStream_t);
template hipError_t launch_readout<float>(const float*, const float*, const float*, const float*, int, int, int, float*, hipStream_t);

}  // namespace anomps
