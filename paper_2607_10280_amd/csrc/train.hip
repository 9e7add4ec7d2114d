// One training step of the adaptive observables (A, B, D) and the linear reconstruction (W, b)
// on cached Pauli features (§II-C: the expectations are computed once; §II-D: two Adam
// optimizers).  Loss: the MSE term of Eq. (7), L = mean_{b,o} (y_hat[b][o] - y[b][o])^2 with
// y_hat = W q + b (Eq. (6)), q_q = sum_alpha c_{q,alpha} <P_alpha> (Eq. (5)) and
// c = Tr(H P) / 4 (Eq. (4)).
//
// Workspace (caller-owned, R = float or double), in this order:
//   coeff [m][16] | q [B][m] | gy [B][out] | gq [B][m] | grad [16m + out*m + out] | lossp [B]
// grad holds dA [m][6], dB [m][6], dD [m][4], dW [out][m], db [out] back to back, the same
// packing as the Adam moment arrays.
#include "common.hpp"
#include "kernels.hpp"

namespace anomps {

namespace {

template <typename R>
__device__ __forceinline__ cx<R> pauli_m(int a, int r, int c) {
  switch (a) {
    case 0: return cx<R>{(R)(r == c), (R)0};
    case 1: return cx<R>{(R)(r != c), (R)0};
    case 2: return (r == c) ? cx<R>{(R)0, (R)0} : cx<R>{(R)0, (R)(r == 0 ? -1 : 1)};
    default: return (r == c) ? cx<R>{(R)(r == 0 ? 1 : -1), (R)0} : cx<R>{(R)0, (R)0};
  }
}

// (P_a (x) P_c)[r][c], rows/columns indexed s_i*2 + s_j.
template <typename R>
__device__ __forceinline__ cx<R> pair_pauli(int alpha16, int r, int c) {
  return cmul(pauli_m<R>(alpha16 >> 2, r >> 1, c >> 1), pauli_m<R>(alpha16 & 3, r & 1, c & 1));
}

// Forward for one image per workgroup: q (kept for the backward pass), y_hat, dL/dy_hat and the
// image's squared error.
template <typename R>
__global__ void k_train_fwd(const R* pauli, const R* target, const R* coeff, const R* W,
                            const R* bias, int batch, int m, int out_dim, R* q, R* gy, R* lossp) {
  extern __shared__ unsigned char smem[];
  R* qv = reinterpret_cast<R*>(smem);
  R* red = qv + m;
  const int b = blockIdx.x;
  const R* pb = pauli + (size_t)b * m * 15;
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    R acc = coeff[j * 16];
    for (int al = 0; al < 15; ++al) acc += coeff[j * 16 + al + 1] * pb[j * 15 + al];
    qv[j] = acc;
    q[(size_t)b * m + j] = acc;
  }
  __syncthreads();
  const R scale = (R)2 / ((R)batch * (R)out_dim);
  R part = (R)0;
  for (int o = threadIdx.x; o < out_dim; o += blockDim.x) {
    R acc = bias[o];
    const R* wr = W + (size_t)o * m;
    for (int j = 0; j < m; ++j) acc += wr[j] * qv[j];
    const R r = acc - target[(size_t)b * out_dim + o];
    gy[(size_t)b * out_dim + o] = scale * r;
    part += r * r;
  }
  red[threadIdx.x] = part;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) lossp[b] = red[0];
}

// dW[o][j] = sum_b gy[b][o] q[b][j]; db[o] = sum_b gy[b][o].  One workgroup per output o.
template <typename R>
__global__ void k_train_gw(const R* gy, const R* q, int batch, int m, int out_dim, R* dW, R* db) {
  const int o = blockIdx.x;
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    R acc = (R)0;
    for (int b = 0; b < batch; ++b) acc += gy[(size_t)b * out_dim + o] * q[(size_t)b * m + j];
    dW[(size_t)o * m + j] = acc;
  }
  if (threadIdx.x == 0) {
    R acc = (R)0;
    for (int b = 0; b < batch; ++b) acc += gy[(size_t)b * out_dim + o];
    db[o] = acc;
  }
}

// gq[b][j] = sum_o gy[b][o] W[o][j].  One workgroup per image.
template <typename R>
__global__ void k_train_gq(const R* gy, const R* W, int m, int out_dim, R* gq) {
  const int b = blockIdx.x;
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    R acc = (R)0;
    for (int o = 0; o < out_dim; ++o) acc += gy[(size_t)b * out_dim + o] * W[(size_t)o * m + j];
    gq[(size_t)b * m + j] = acc;
  }
}

// dc[j][alpha] = sum_b gq[b][j] <P_alpha>[b][j] (alpha = 0: 1), then the observable gradients
// dD[j] = sum_alpha dc_alpha Re P_alpha[j][j] / 4, and for each upper position (lo, hi):
// dA = sum_alpha dc_alpha Re(P[hi][lo] + P[lo][hi]) / 4,
// dB = sum_alpha dc_alpha (Im P[lo][hi] - Im P[hi][lo]) / 4.  One workgroup of 256 per pair j.
template <typename R>
__global__ void k_train_gobs(const R* pauli, const R* gq, int batch, int m, R* dA, R* dB, R* dD) {
  __shared__ R part[256];
  __shared__ R dc[16];
  const int j = blockIdx.x, al = threadIdx.x & 15, g = threadIdx.x >> 4;
  R acc = (R)0;
  for (int b = g; b < batch; b += 16) {
    const R pv = al == 0 ? (R)1 : pauli[((size_t)b * m + j) * 15 + al - 1];
    acc += gq[(size_t)b * m + j] * pv;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x < 16) {
    R s = (R)0;
    for (int k = 0; k < 16; ++k) s += part[k * 16 + threadIdx.x];
    dc[threadIdx.x] = s;
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < 4) {
    R s = (R)0;
    for (int a = 0; a < 16; ++a) s += dc[a] * pair_pauli<R>(a, t, t).re;
    dD[j * 4 + t] = (R)0.25 * s;
  } else if (t < 10) {
    const int idx = t - 4;
    const int lo = idx < 3 ? 0 : (idx < 5 ? 1 : 2), hi = idx < 3 ? idx + 1 : (idx < 5 ? idx - 1 : 3);
    R sa = (R)0, sb = (R)0;
    for (int a = 0; a < 16; ++a) {
      const cx<R> phl = pair_pauli<R>(a, hi, lo), plh = pair_pauli<R>(a, lo, hi);
      sa += dc[a] * (phl.re + plh.re);
      sb += dc[a] * (plh.im - phl.im);
    }
    dA[j * 6 + idx] = (R)0.25 * sa;
    dB[j * 6 + idx] = (R)0.25 * sb;
  }
}

// Adam (Kingma & Ba) on a packed parameter range with learning rate lr.
template <typename R>
__global__ void k_adam(R* param, const R* grad, R* mom, R* vel, int count, R lr, R beta1, R beta2,
                       R eps, R corr1, R corr2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const R g = grad[i];
  const R mi = beta1 * mom[i] + ((R)1 - beta1) * g;
  const R vi = beta2 * vel[i] + ((R)1 - beta2) * g * g;
  mom[i] = mi;
  vel[i] = vi;
  param[i] -= lr * (mi / corr1) / (sqrt(vi / corr2) + eps);
}

template <typename R>
__global__ void k_loss_sum(const R* lossp, int batch, int out_dim, R* loss) {
  __shared__ R red[256];
  R s = (R)0;
  for (int b = threadIdx.x; b < batch; b += blockDim.x) s += lossp[b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = red[0] / ((R)batch * (R)out_dim);
}

template <typename R>
hipError_t adam_range(R* p, const R* g, R* mo, R* ve, int count, double lr, double b1, double b2,
                      double eps, int step, hipStream_t stream) {
  if (count == 0) return hipSuccess;
  const R corr1 = (R)(1.0 - pow(b1, step)), corr2 = (R)(1.0 - pow(b2, step));
  hipLaunchKernelGGL(k_adam<R>, dim3((count + 255) / 256), dim3(256), 0, stream, p, g, mo, ve,
                     count, (R)lr, (R)b1, (R)b2, (R)eps, corr1, corr2);
  return hipGetLastError();
}

}  // namespace

size_t train_workspace_elems(int batch, int m, int out_dim) {
  return (size_t)m * 16 + (size_t)batch * m * 2 + (size_t)batch * out_dim +
         (size_t)16 * m + (size_t)out_dim * m + out_dim + batch;
}

template <typename R>
hipError_t launch_train_step(const R* pauli, const R* target, R* A, R* B, R* D, R* W, R* bias,
                             R* mom, R* vel, int batch, int m, int out_dim, int step, double lr_obs,
                             double lr_lin, double beta1, double beta2, double eps, R* loss,
                             R* ws, hipStream_t stream) {
  R* coeff = ws;
  R* q = coeff + (size_t)m * 16;
  R* gy = q + (size_t)batch * m;
  R* gq = gy + (size_t)batch * out_dim;
  R* grad = gq + (size_t)batch * m;
  R* lossp = grad + (size_t)16 * m + (size_t)out_dim * m + out_dim;
  R* dA = grad;
  R* dB = dA + (size_t)m * 6;
  R* dD = dB + (size_t)m * 6;
  R* dW = dD + (size_t)m * 4;
  R* db = dW + (size_t)out_dim * m;
  hipError_t e = launch_coeffs<R>(A, B, D, m, coeff, stream);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_train_fwd<R>, dim3(batch), dim3(256), (size_t)(m + 256) * sizeof(R), stream,
                     pauli, target, coeff, W, bias, batch, m, out_dim, q, gy, lossp);
  hipLaunchKernelGGL(k_loss_sum<R>, dim3(1), dim3(256), 0, stream, lossp, batch, out_dim, loss);
  hipLaunchKernelGGL(k_train_gw<R>, dim3(out_dim), dim3(128), 0, stream, gy, q, batch, m, out_dim,
                     dW, db);
  hipLaunchKernelGGL(k_train_gq<R>, dim3(batch), dim3(128), 0, stream, gy, W, m, out_dim, gq);
  hipLaunchKernelGGL(k_train_gobs<R>, dim3(m), dim3(256), 0, stream, pauli, gq, batch, m, dA, dB, dD);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // observable parameters (A, B, D: 16 m values) and the linear layer (W, b) are packed
  // separately in the caller's buffers but contiguously in the moment arrays
  const size_t nobs[3] = {(size_t)m * 6, (size_t)m * 6, (size_t)m * 4};
  R* obs[3] = {A, B, D};
  size_t off = 0;
  for (int k = 0; k < 3; ++k) {
    e = adam_range<R>(obs[k], grad + off, mom + off, vel + off, (int)nobs[k], lr_obs, beta1, beta2,
                      eps, step, stream);
    if (e != hipSuccess) return e;
    off += nobs[k];
  }
  e = adam_range<R>(W, grad + off, mom + off, vel + off, out_dim * m, lr_lin, beta1, beta2, eps,
                    step, stream);
  if (e != hipSuccess) return e;
  off += (size_t)out_dim * m;
  return adam_range<R>(bias, grad + off, mom + off, vel + off, out_dim, lr_lin, beta1, beta2, eps,
                       step, stream);
}

template hipError_t launch_train_step<double>(const double*, const double*, double*, double*,
                                              double*, double*, double*, double*, double*, int, int,
                                              int, int, double, double, double, double, double,
                                              double*, double*, hipStream_t);
template hipError_t launch_train_step<float>(const float*, const float*, float*, float*, float*,
                                             float*, float*, float*, float*, int, int, int, int,
                                             double, double, double, double, double, float*,
                                             float*, hipStream_t);

}  // namespace anomps
