// C-ABI entry points of libanomps (declared in include/anomps.h): host-side validation, size
// arithmetic and dispatch to the typed kernel launchers.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "../../include/anomps.h"
#include "common.hpp"
#include "kernels.hpp"

using namespace anomps;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int ok() {
  g_last_error.clear();
  return MPS_OK;
}

int check_hip(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(MPS_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
  return ok();
}

// Slot bucket: smallest compiled S (2, 4, 8, 16) >= the largest bond the batch reaches.
int slot_bucket(int n, int chi, int layers) {
  const int d = slot_dim(n, chi, layers);
  int s = 2;
  while (s < d) s <<= 1;
  return s;
}

bool valid_prec(int p) { return p == MPS_PREC_FP64 || p == MPS_PREC_FP32 || p == MPS_PREC_SPLIT_BF16; }

int check_shape(int n, int chi, int layers, int batch, int prec) {
  if (n < 2 || n > MPS_MAX_SITES) return fail(MPS_ERR_INVALID_ARG, "n_sites=%d outside [2, %d]", n, MPS_MAX_SITES);
  if (chi < 1) return fail(MPS_ERR_INVALID_ARG, "chi=%d must be >= 1", chi);
  if (layers < 0) return fail(MPS_ERR_INVALID_ARG, "n_layers=%d must be >= 0", layers);
  if (batch < 1) return fail(MPS_ERR_INVALID_ARG, "batch=%d must be >= 1", batch);
  if (!valid_prec(prec)) return fail(MPS_ERR_INVALID_ARG, "precision=%d unknown", prec);
  if (slot_dim(n, chi, layers) > MPS_MAX_BOND)
    return fail(MPS_ERR_CAPACITY, "bond dimension %d exceeds MPS_MAX_BOND=%d", slot_dim(n, chi, layers), MPS_MAX_BOND);
  return MPS_OK;
}

size_t real_size(int prec) { return prec == MPS_PREC_FP64 ? sizeof(double) : sizeof(float); }

int check_batch(const mps_batch* b) {
  if (!b) return fail(MPS_ERR_INVALID_ARG, "batch descriptor is NULL");
  int rc = check_shape(b->n_sites, b->chi, b->n_layers, b->batch, b->precision);
  if (rc) return rc;
  if (!b->state || !b->status) return fail(MPS_ERR_INVALID_ARG, "state/status pointer is NULL");
  return MPS_OK;
}

}  // namespace

extern "C" {

int32_t mps_bond_dim(int32_t n_sites, int32_t chi, int32_t layers, int32_t bond) {
  if (n_sites < 2 || chi < 1 || layers < 0 || bond < -1 || bond > n_sites - 1) return 0;
  return bond_dim(n_sites, chi, layers, bond);
}

int32_t mps_slot_dim(int32_t n_sites, int32_t chi, int32_t n_layers) {
  if (n_sites < 2 || chi < 1 || n_layers < 0) return 0;
  return slot_bucket(n_sites, chi, n_layers);
}

size_t mps_state_bytes(int32_t n, int32_t chi, int32_t layers, int32_t batch, int32_t prec) {
  if (check_shape(n, chi, layers, batch, prec)) return 0;
  const size_t S = slot_bucket(n, chi, layers);
  return (size_t)batch * n * 2 * S * S * 2 * real_size(prec);
}

size_t mps_env_bytes(int32_t n, int32_t chi, int32_t layers, int32_t batch, int32_t prec) {
  if (check_shape(n, chi, layers, batch, prec)) return 0;
  const size_t S = slot_bucket(n, chi, layers);
  return (size_t)batch * 2 * (n + 1) * S * S * 2 * real_size(prec);
}

int mps_init_batch(mps_batch* b, const double* pixels, hipStream_t stream) {
  int rc = check_batch(b);
  if (rc) return rc;
  if (!pixels) return fail(MPS_ERR_INVALID_ARG, "pixels is NULL");
  const int S = slot_bucket(b->n_sites, b->chi, b->n_layers);
  hipError_t e;
  if (b->precision == MPS_PREC_FP64)
    e = launch_encode<double>((double*)b->state, pixels, b->n_sites, S, b->batch, b->status, stream);
  else
    e = launch_encode<float>((float*)b->state, pixels, b->n_sites, S, b->batch, b->status, stream);
  if (e != hipSuccess) return check_hip(e, "encode launch");
  b->layers_done = 0;
  return ok();
}

int mps_apply_layer(mps_batch* b, const double* theta, const double* phi, double* trunc_err,
                    hipStream_t stream) {
  int rc = check_batch(b);
  if (rc) return rc;
  if (!theta || !phi) return fail(MPS_ERR_INVALID_ARG, "theta/phi is NULL");
  if (b->layers_done < 0 || b->layers_done >= b->n_layers)
    return fail(MPS_ERR_INVALID_ARG, "layers_done=%d: batch sized for %d layers", b->layers_done, b->n_layers);
  const int S = slot_bucket(b->n_sites, b->chi, b->n_layers);
  hipError_t e;
  if (b->precision == MPS_PREC_FP64)
    e = launch_layer<double>((double*)b->state, b->n_sites, b->chi, S, b->layers_done, b->batch,
                             theta, phi, trunc_err, b->status, stream);
  else
    e = launch_layer<float>((float*)b->state, b->n_sites, b->chi, S, b->layers_done, b->batch,
                            theta, phi, trunc_err, b->status, stream);
  if (e != hipSuccess) return check_hip(e, "layer launch");
  b->layers_done += 1;
  return ok();
}

int mps_validate_pairs(const int32_t* pairs_host, int32_t m, int32_t n_sites) {
  if (m < 0) return fail(MPS_ERR_INVALID_ARG, "m=%d < 0", m);
  if (m > 0 && !pairs_host) return fail(MPS_ERR_INVALID_ARG, "pairs is NULL");
  if (n_sites < 2 || n_sites > MPS_MAX_SITES) return fail(MPS_ERR_INVALID_ARG, "n_sites=%d", n_sites);
  std::vector<int> per_site(n_sites, 0);
  for (int q = 0; q < m; ++q) {
    const int i = pairs_host[2 * q], j = pairs_host[2 * q + 1];
    if (i < 0 || j <= i || j >= n_sites)
      return fail(MPS_ERR_INVALID_ARG, "pair %d = (%d, %d): need 0 <= i < j < %d", q, i, j, n_sites);
    if (++per_site[i] > 256)
      return fail(MPS_ERR_CAPACITY, "more than 256 pairs start at site %d", i);
  }
  return ok();
}

int mps_pauli_pair_expect(mps_batch* b, const int32_t* pairs, int32_t m, void* out,
                          hipStream_t stream) {
  int rc = check_batch(b);
  if (rc) return rc;
  if (!b->env) return fail(MPS_ERR_INVALID_ARG, "env is NULL");
  if (m < 0) return fail(MPS_ERR_INVALID_ARG, "m=%d < 0", m);
  if (m > 0 && (!pairs || !out)) return fail(MPS_ERR_INVALID_ARG, "pairs/out is NULL");
  if (b->precision == MPS_PREC_SPLIT_BF16)
    return fail(MPS_ERR_UNSUPPORTED, "split-bf16 pair contractions are not built in this library");
  const int S = slot_bucket(b->n_sites, b->chi, b->n_layers);
  const int L = b->layers_done;
  hipError_t e;
  if (b->precision == MPS_PREC_FP64) {
    e = launch_envs<double, double>((const double*)b->state, (double*)b->env, b->n_sites, b->chi, S, L, b->batch, stream);
    if (e == hipSuccess)
      e = launch_pairs<double, double>((const double*)b->state, (const double*)b->env, pairs, m, b->n_sites, b->chi, S, L, b->batch, (double*)out, stream);
  } else if (S == 16) {
    e = launch_measure16((const float*)b->state, (float*)b->env, pairs, m, b->n_sites, b->chi, L,
                         b->batch, (float*)out, stream);
  } else {
    e = launch_envs<float, float>((const float*)b->state, (float*)b->env, b->n_sites, b->chi, S, L, b->batch, stream);
    if (e == hipSuccess)
      e = launch_pairs<float, float>((const float*)b->state, (const float*)b->env, pairs, m, b->n_sites, b->chi, S, L, b->batch, (float*)out, stream);
  }
  if (e != hipSuccess) return check_hip(e, "measurement launch");
  return ok();
}

int mps_ano_coeffs(const void* A, const void* B, const void* D, int32_t m, void* coeff,
                   int32_t is_f64, hipStream_t stream) {
  if (m < 0) return fail(MPS_ERR_INVALID_ARG, "m=%d < 0", m);
  if (m > 0 && (!A || !B || !D || !coeff)) return fail(MPS_ERR_INVALID_ARG, "NULL argument");
  hipError_t e = is_f64 ? launch_coeffs<double>((const double*)A, (const double*)B, (const double*)D, m, (double*)coeff, stream)
                        : launch_coeffs<float>((const float*)A, (const float*)B, (const float*)D, m, (float*)coeff, stream);
  if (e != hipSuccess) return check_hip(e, "coeff launch");
  return ok();
}

int mps_ano_readout(const void* pauli, const void* coeff, const void* W, const void* bias,
                    int32_t batch, int32_t m, int32_t out_dim, void* y, int32_t is_f64,
                    hipStream_t stream) {
  if (batch < 0 || m < 0 || out_dim < 0) return fail(MPS_ERR_INVALID_ARG, "negative size");
  if (m > 4096) return fail(MPS_ERR_CAPACITY, "m=%d exceeds 4096", m);
  if (batch > 0 && out_dim > 0 && (!pauli || !coeff || !W || !y))
    return fail(MPS_ERR_INVALID_ARG, "NULL argument");
  hipError_t e = is_f64
      ? launch_readout<double>((const double*)pauli, (const double*)coeff, (const double*)W, (const double*)bias, batch, m, out_dim, (double*)y, stream)
      : launch_readout<float>((const float*)pauli, (const float*)coeff, (const float*)W, (const float*)bias, batch, m, out_dim, (float*)y, stream);
  if (e != hipSuccess) return check_hip(e, "readout launch");
  return ok();
}

const char* mps_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
