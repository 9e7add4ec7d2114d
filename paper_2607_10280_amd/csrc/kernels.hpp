// Host-side launchers of the anomps kernels (internal; the public interface is anomps.h).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/anomps.h"

namespace anomps {

template <typename T>
hipError_t launch_encode(T* state, const double* pixels, int n, int S, int batch, int* status,
                         hipStream_t stream);

// program 0: R_Y R_Z gates + CNOT ladder (theta, phi); program 1: the paper's H, R_Y(2 pi x - pi)
// gates from pixels + brickwork CNOTs.
// `count` ladder layers from `layer` (theta, phi [count][n]; trunc_err [count][batch][n-1]).
template <typename T>
hipError_t launch_layers(T* state, int n, int chi, int S, int layer, int count, int batch,
                         const double* theta, const double* phi, double* trunc_err, int* status,
                         int n_layers, hipStream_t stream);
template <typename T>
hipError_t launch_layer(T* state, int n, int chi, int S, int layer, int batch, int program,
                        const double* theta, const double* phi, const double* pixels,
                        double* trunc_err, int* status, int n_layers, hipStream_t stream);

// Bonds and ladder layers that keep all their singular values: kExactMpo (default) applies such
// a layer as one site-local contraction and splits other such bonds exactly; kExactQr splits
// every bond of such a layer by Householder QR in one sweep; kExactSvd runs the canonical sweep
// + Jacobi SVD ladder everywhere.  Kernels test the mode for non-zero to enable the exact splits.
enum : int { kExactSvd = 0, kExactQr = 1, kExactMpo = 2 };
void set_exact_qr(int mode);
int exact_qr();

// Environment sweeps (left and right) and pair expectations.  T = storage type of the state,
// C = compute/output type of the measurement (double for FP64 batches, float otherwise).
template <typename T, typename C>
hipError_t launch_envs(const T* state, C* env, int n, int chi, int S, int layers, int batch,
                       hipStream_t stream);

template <typename T, typename C>
hipError_t launch_pairs(const T* state, const C* env, const int* pairs, int m, int n, int chi,
                        int S, int layers, int batch, C* out, hipStream_t stream);

// Matrix-core measurement for 16-wide slots (environments + pairs), by the batch's precision:
// FP64 products (state, environments and outputs FP64), FP32 products, or split-BF16 products
// with FP32 accumulation.
hipError_t launch_measure16(const void* state, void* env, const int* pairs, int m, int n, int chi,
                            int layers, int batch, void* out, int precision, int block_groups,
                            int waves_per_cu, hipStream_t stream);

// Wide slots (S = 32, 64, 128; wide.hip): the same layer and measurement with one 256-lane
// workgroup per image and the per-bond matrices in an FP64 workspace of
// wide_workspace_bytes(S) bytes per image (placed by the library after the environments).
size_t wide_workspace_bytes(int S);
// A wide-slot layer that keeps every singular value as the parity product operator (ws: the
// batch's FP64 workspace, ws_stride complex128 elements per image); false when not applicable.
template <typename T>
bool launch_mpo_wide(T* state, double* ws, size_t ws_stride, int n, int chi, int S, int layer,
                     int batch, int program, const double* theta, const double* phi,
                     const double* pixels, double* trunc_err, int* status, int n_layers,
                     hipStream_t stream, hipError_t& err);
template <typename T>
hipError_t launch_layer_wide(T* state, double* ws, int n, int chi, int S, int layer, int batch,
                             int program, const double* theta, const double* phi,
                             const double* pixels, double* trunc_err, int* status, int n_layers,
                             hipStream_t stream);
template <typename T>
hipError_t launch_measure_wide(const T* state, T* env, double* ws, const int* pairs, int m, int n,
                               int chi, int S, int layers, int batch, T* out, hipStream_t stream);

// Mixed request tables: entries [begin, begin + count) form one bucket (slot S, precision T).
template <typename T>
hipError_t launch_encode_mixed(const mps_request* reqs, int begin, int count, int S,
                               hipStream_t stream);
template <typename T>
hipError_t launch_layer_mixed(const mps_request* reqs, int begin, int count, int S, int* queue,
                              int blocks_per_cu, hipStream_t stream);
template <typename T, typename C>
hipError_t launch_measure_mixed(const mps_request* reqs, int begin, int count, int max_sites,
                                int S, hipStream_t stream);
hipError_t launch_measure16_mixed(const mps_request* reqs, int begin, int count, int max_sites,
                                  bool fp64, hipStream_t stream);
hipError_t launch_zero_ints(int* p, int count, hipStream_t stream);

template <typename R>
hipError_t launch_coeffs(const R* A, const R* B, const R* D, int m, R* coeff, hipStream_t stream);

template <typename R>
hipError_t launch_readout(const R* pauli, const R* coeff, const R* W, const R* bias, int batch,
                          int m, int out_dim, R* y, hipStream_t stream);

// One training step on cached features (train.hip); workspace in elements of the real type.
size_t train_workspace_elems(int batch, int m, int out_dim);
template <typename R>
hipError_t launch_train_step(const R* pauli, const R* target, R* A, R* B, R* D, R* W, R* bias,
                             R* mom, R* vel, int batch, int m, int out_dim, int step, double lr_obs,
                             double lr_lin, double beta1, double beta2, double eps, R* loss,
                             R* ws, hipStream_t stream);

}  // namespace anomps
