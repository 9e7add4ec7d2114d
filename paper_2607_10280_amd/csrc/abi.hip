// C-ABI entry points of libanomps (declared in include/anomps.h): host-side validation, size
// arithmetic and dispatch to the typed kernel launchers.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
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

// ---- mixed request tables
int g_mixed_blocks_per_cu[MPS_MIXED_BUCKETS] = {0};

// Image blocking of the 16-wide pair launch, in groups of 8 images (0 = the whole batch), and
// its cap on resident workgroups per compute unit (0 = none).  Default: blocks of 64 images,
// which read each image's tiles from HBM about once (counters: half the traffic of one block)
// at the same speed.
int g_pair_block_groups = 8;
int g_pair_waves_per_cu = 0;

int bucket_of(int S, int prec) {
  int lg = 0;
  while ((2 << lg) < S) ++lg;  // S = 2, 4, 8, 16 -> 0..3
  return 4 * (prec == MPS_PREC_FP32 ? 1 : 0) + lg;
}
int bucket_slot(int bucket) { return 2 << (bucket & 3); }
bool bucket_fp64(int bucket) { return bucket < 4; }

int check_request(const mps_request& r, int idx) {
  int rc = check_shape(r.n_sites, r.chi, r.n_layers, 1, r.precision);
  if (rc) return fail(rc, "request %d: %s", idx, g_last_error.c_str());
  if (r.precision == MPS_PREC_SPLIT_BF16)
    return fail(MPS_ERR_UNSUPPORTED, "request %d: split-bf16 requests are not built in this library", idx);
  if (slot_bucket(r.n_sites, r.chi, r.n_layers) > kMaxBond)
    return fail(MPS_ERR_CAPACITY, "request %d: slot %d exceeds the mixed-table limit %d", idx,
                slot_bucket(r.n_sites, r.chi, r.n_layers), kMaxBond);
  if (r.n_pairs < 0 || r.reserved != 0)
    return fail(MPS_ERR_INVALID_ARG, "request %d: n_pairs=%d reserved=%d", idx, r.n_pairs, r.reserved);
  if (!r.pixels || !r.state || !r.env || !r.ctrl)
    return fail(MPS_ERR_INVALID_ARG, "request %d: pixels/state/env/ctrl is NULL", idx);
  if (r.n_layers > 0 && (!r.theta || !r.phi))
    return fail(MPS_ERR_INVALID_ARG, "request %d: theta/phi is NULL", idx);
  if (r.n_pairs > 0 && (!r.pairs || !r.out))
    return fail(MPS_ERR_INVALID_ARG, "request %d: pairs/out is NULL", idx);
  return MPS_OK;
}

int check_plan(const mps_request* reqs, const mps_mixed_plan* plan) {
  if (!plan) return fail(MPS_ERR_INVALID_ARG, "plan is NULL");
  if (plan->n_req < 0) return fail(MPS_ERR_INVALID_ARG, "plan n_req=%d", plan->n_req);
  int expect = 0;
  for (int k = 0; k < MPS_MIXED_BUCKETS; ++k) {
    if (plan->count[k] < 0 || plan->begin[k] != expect ||
        (plan->count[k] > 0 && (plan->max_sites[k] < 2 || plan->max_sites[k] > MPS_MAX_SITES)))
      return fail(MPS_ERR_INVALID_ARG, "plan bucket %d is inconsistent", k);
    expect += plan->count[k];
  }
  if (expect != plan->n_req) return fail(MPS_ERR_INVALID_ARG, "plan counts do not sum to n_req");
  if (plan->n_req > 0 && !reqs) return fail(MPS_ERR_INVALID_ARG, "request table is NULL");
  return MPS_OK;
}

// Environments [batch][2][n+1][S][S]; wide slots (S > kMaxBond) append a 256-byte aligned FP64
// workspace of wide_workspace_bytes(S) per image, used by the layer and measurement kernels.
size_t env_part_bytes(int n, int S, int batch, int prec) {
  const size_t e = (size_t)batch * 2 * (n + 1) * S * S * 2 * real_size(prec);
  return S > kMaxBond ? (e + 255) / 256 * 256 : e;
}

double* wide_ws(const mps_batch* b, int S) {
  return (double*)((char*)b->env + env_part_bytes(b->n_sites, S, b->batch, b->precision));
}

// ---- scratch of the allocation-free measurement (mps_pauli_pair_expect_noalloc)
// A fixed device array that holds the environments of one call.  Every device the library runs
// on gets its own copy (at its own address) when the code object is loaded there, kept until
// the process ends.  In host code `scratch` only names the symbol: its device address comes
// from hipGetSymbolAddress, taken once per device with that device current.
__device__ __align__(256) unsigned char scratch[MPS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {nullptr};

int noalloc_scratch(void** ptr) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return check_hip(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(MPS_ERR_UNSUPPORTED, "device %d outside the %d devices this build tracks", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return check_hip(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(MPS_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return MPS_OK;
}

// Environments and pair expectations of a batch into `env` (the caller's buffer, or the
// allocation-free entry point's scratch).
int measure(mps_batch* b, void* env, const int32_t* pairs, int32_t m, void* out,
            hipStream_t stream) {
  if (m < 0) return fail(MPS_ERR_INVALID_ARG, "m=%d < 0", m);
  if (m > 0 && (!pairs || !out)) return fail(MPS_ERR_INVALID_ARG, "pairs/out is NULL");
  const int S = slot_bucket(b->n_sites, b->chi, b->n_layers);
  const int L = b->layers_done;
  hipError_t e;
  if (S > kMaxBond) {
    double* ws = (double*)((char*)env + env_part_bytes(b->n_sites, S, b->batch, b->precision));
    if (b->precision == MPS_PREC_FP64)
      e = launch_measure_wide<double>((const double*)b->state, (double*)env, ws, pairs, m,
                                      b->n_sites, b->chi, S, L, b->batch, (double*)out, stream);
    else
      e = launch_measure_wide<float>((const float*)b->state, (float*)env, ws, pairs, m,
                                     b->n_sites, b->chi, S, L, b->batch, (float*)out, stream);
  } else if (S == 16) {
    e = launch_measure16(b->state, env, pairs, m, b->n_sites, b->chi, L, b->batch, out,
                         b->precision, g_pair_block_groups, g_pair_waves_per_cu, stream);
  } else if (b->precision == MPS_PREC_FP64) {
    e = launch_envs<double, double>((const double*)b->state, (double*)env, b->n_sites, b->chi, S, L, b->batch, stream);
    if (e == hipSuccess)
      e = launch_pairs<double, double>((const double*)b->state, (const double*)env, pairs, m, b->n_sites, b->chi, S, L, b->batch, (double*)out, stream);
  } else {
    e = launch_envs<float, float>((const float*)b->state, (float*)env, b->n_sites, b->chi, S, L, b->batch, stream);
    if (e == hipSuccess)
      e = launch_pairs<float, float>((const float*)b->state, (const float*)env, pairs, m, b->n_sites, b->chi, S, L, b->batch, (float*)out, stream);
  }
  if (e != hipSuccess) return check_hip(e, "measurement launch");
  return ok();
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
  const int S = slot_bucket(n, chi, layers);
  size_t e = env_part_bytes(n, S, batch, prec);
  if (S > kMaxBond) e += (size_t)batch * wide_workspace_bytes(S);
  return e;
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

int mps_apply_layer_program(mps_batch* b, int32_t program, const double* theta,
                            const double* phi, const double* pixels, double* trunc_err,
                            hipStream_t stream) {
  int rc = check_batch(b);
  if (rc) return rc;
  if (program == MPS_LAYER_RYRZ_LADDER) {
    if (!theta || !phi) return fail(MPS_ERR_INVALID_ARG, "theta/phi is NULL");
  } else if (program == MPS_LAYER_H_RY_BRICKWORK) {
    if (!pixels) return fail(MPS_ERR_INVALID_ARG, "pixels is NULL");
  } else {
    return fail(MPS_ERR_INVALID_ARG, "layer program %d unknown", program);
  }
  if (b->layers_done < 0 || b->layers_done >= b->n_layers)
    return fail(MPS_ERR_INVALID_ARG, "layers_done=%d: batch sized for %d layers", b->layers_done, b->n_layers);
  const int S = slot_bucket(b->n_sites, b->chi, b->n_layers);
  hipError_t e;
  if (S > kMaxBond) {
    if (!b->env) return fail(MPS_ERR_INVALID_ARG, "env is NULL (slot %d layers use it as workspace)", S);
    if (b->precision == MPS_PREC_FP64)
      e = launch_layer_wide<double>((double*)b->state, wide_ws(b, S), b->n_sites, b->chi, S,
                                    b->layers_done, b->batch, program, theta, phi, pixels,
                                    trunc_err, b->status, b->n_layers, stream);
    else
      e = launch_layer_wide<float>((float*)b->state, wide_ws(b, S), b->n_sites, b->chi, S,
                                   b->layers_done, b->batch, program, theta, phi, pixels,
                                   trunc_err, b->status, b->n_layers, stream);
  } else if (b->precision == MPS_PREC_FP64) {
    e = launch_layer<double>((double*)b->state, b->n_sites, b->chi, S, b->layers_done, b->batch,
                             program, theta, phi, pixels, trunc_err, b->status, b->n_layers,
                             stream);
  } else {
    e = launch_layer<float>((float*)b->state, b->n_sites, b->chi, S, b->layers_done, b->batch,
                            program, theta, phi, pixels, trunc_err, b->status, b->n_layers,
                            stream);
  }
  if (e != hipSuccess) return check_hip(e, "layer launch");
  b->layers_done += 1;
  return ok();
}

int mps_apply_layer(mps_batch* b, const double* theta, const double* phi, double* trunc_err,
                    hipStream_t stream) {
  return mps_apply_layer_program(b, MPS_LAYER_RYRZ_LADDER, theta, phi, nullptr, trunc_err, stream);
}

int mps_apply_layers(mps_batch* b, int32_t count, const double* theta, const double* phi,
                     double* trunc_err, hipStream_t stream) {
  int rc = check_batch(b);
  if (rc) return rc;
  if (!theta || !phi) return fail(MPS_ERR_INVALID_ARG, "theta/phi is NULL");
  if (count < 1) return fail(MPS_ERR_INVALID_ARG, "count=%d < 1", count);
  if (b->layers_done < 0 || b->layers_done + count > b->n_layers)
    return fail(MPS_ERR_INVALID_ARG, "layers_done=%d + count=%d: batch sized for %d layers",
                b->layers_done, count, b->n_layers);
  const int S = slot_bucket(b->n_sites, b->chi, b->n_layers);
  if (S > kMaxBond) {
    // wide slots: one layer call after the other
    const size_t n = (size_t)b->n_sites, te = (size_t)b->batch * (n - 1);
    for (int r = 0; r < count; ++r) {
      rc = mps_apply_layer(b, theta + r * n, phi + r * n, trunc_err ? trunc_err + r * te : nullptr,
                           stream);
      if (rc) return rc;
    }
    return ok();
  }
  hipError_t e;
  if (b->precision == MPS_PREC_FP64)
    e = launch_layers<double>((double*)b->state, b->n_sites, b->chi, S, b->layers_done, count,
                              b->batch, theta, phi, trunc_err, b->status, b->n_layers, stream);
  else
    e = launch_layers<float>((float*)b->state, b->n_sites, b->chi, S, b->layers_done, count,
                             b->batch, theta, phi, trunc_err, b->status, b->n_layers, stream);
  if (e != hipSuccess) return check_hip(e, "layer launch");
  b->layers_done += count;
  return ok();
}

int mps_init_zero(mps_batch* b, hipStream_t stream) {
  int rc = check_batch(b);
  if (rc) return rc;
  const int S = slot_bucket(b->n_sites, b->chi, b->n_layers);
  hipError_t e;
  if (b->precision == MPS_PREC_FP64)
    e = launch_encode<double>((double*)b->state, nullptr, b->n_sites, S, b->batch, b->status, stream);
  else
    e = launch_encode<float>((float*)b->state, nullptr, b->n_sites, S, b->batch, b->status, stream);
  if (e != hipSuccess) return check_hip(e, "encode launch");
  b->layers_done = 0;
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
  return measure(b, b->env, pairs, m, out, stream);
}

int mps_pauli_pair_expect_noalloc(mps_batch* b, const int32_t* pairs, int32_t m, void* out,
                                  hipStream_t stream) {
  int rc = check_batch(b);
  if (rc) return rc;
  const int S = slot_bucket(b->n_sites, b->chi, b->n_layers);
  if (S > kMaxBond)
    return fail(MPS_ERR_UNSUPPORTED, "slot %d: the allocation-free measurement takes slots up to %d",
                S, kMaxBond);
  const size_t need = env_part_bytes(b->n_sites, S, b->batch, b->precision);
  if (need > MPS_NOALLOC_SCRATCH_BYTES)
    return fail(MPS_ERR_CAPACITY, "environments need %zu bytes, more than the %zu-byte scratch",
                need, (size_t)MPS_NOALLOC_SCRATCH_BYTES);
  void* env = nullptr;
  rc = noalloc_scratch(&env);
  if (rc) return rc;
  return measure(b, env, pairs, m, out, stream);
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

int mps_plan_mixed(const mps_request* reqs_host, int32_t n_req, int32_t* order,
                   mps_mixed_plan* plan) {
  if (n_req < 0) return fail(MPS_ERR_INVALID_ARG, "n_req=%d < 0", n_req);
  if (!plan || (n_req > 0 && (!reqs_host || !order)))
    return fail(MPS_ERR_INVALID_ARG, "NULL argument");
  std::vector<int> bucket(n_req);
  std::vector<double> cost(n_req);
  for (int i = 0; i < n_req; ++i) {
    const mps_request& r = reqs_host[i];
    int rc = check_request(r, i);
    if (rc) return rc;
    const int S = slot_bucket(r.n_sites, r.chi, r.n_layers);
    bucket[i] = bucket_of(S, r.precision);
    // Work estimate: each layer runs ~n SVDs of (2D)x(2D) matrices, D = min(chi, 2^layers).
    const double d = (double)slot_dim(r.n_sites, r.chi, r.n_layers);
    cost[i] = (double)r.n_layers * r.n_sites * d * d * d + r.n_sites * d * d;
  }
  for (int i = 0; i < n_req; ++i) order[i] = i;
  std::stable_sort(order, order + n_req, [&](int a, int b) {
    if (bucket[a] != bucket[b]) return bucket[a] < bucket[b];
    return cost[a] > cost[b];
  });
  memset(plan, 0, sizeof(*plan));
  plan->n_req = n_req;
  for (int t = 0; t < n_req; ++t) {
    const int k = bucket[order[t]];
    if (plan->count[k]++ == 0) plan->begin[k] = t;
    const int n = reqs_host[order[t]].n_sites;
    if (n > plan->max_sites[k]) plan->max_sites[k] = n;
  }
  int at = 0;  // empty buckets start where the next one would
  for (int k = 0; k < MPS_MIXED_BUCKETS; ++k) {
    plan->begin[k] = at;
    at += plan->count[k];
  }
  return ok();
}

int mps_init_mixed(const mps_request* reqs, const mps_mixed_plan* plan, hipStream_t stream) {
  int rc = check_plan(reqs, plan);
  if (rc) return rc;
  for (int k = 0; k < MPS_MIXED_BUCKETS; ++k) {
    if (!plan->count[k]) continue;
    const hipError_t e = bucket_fp64(k)
        ? launch_encode_mixed<double>(reqs, plan->begin[k], plan->count[k], bucket_slot(k), stream)
        : launch_encode_mixed<float>(reqs, plan->begin[k], plan->count[k], bucket_slot(k), stream);
    if (e != hipSuccess) return check_hip(e, "mixed encode launch");
  }
  return ok();
}

int mps_apply_layer_mixed(const mps_request* reqs, const mps_mixed_plan* plan, int32_t* queue,
                          hipStream_t stream) {
  int rc = check_plan(reqs, plan);
  if (rc) return rc;
  if (plan->n_req == 0) return ok();
  if (!queue) return fail(MPS_ERR_INVALID_ARG, "queue is NULL");
  hipError_t e = launch_zero_ints(queue, MPS_MIXED_BUCKETS, stream);
  if (e != hipSuccess) return check_hip(e, "queue reset launch");
  for (int k = 0; k < MPS_MIXED_BUCKETS; ++k) {
    if (!plan->count[k]) continue;
    e = bucket_fp64(k)
        ? launch_layer_mixed<double>(reqs, plan->begin[k], plan->count[k], bucket_slot(k), queue + k,
                                     g_mixed_blocks_per_cu[k], stream)
        : launch_layer_mixed<float>(reqs, plan->begin[k], plan->count[k], bucket_slot(k), queue + k,
                                    g_mixed_blocks_per_cu[k], stream);
    if (e != hipSuccess) return check_hip(e, "mixed layer launch");
  }
  return ok();
}

int mps_pauli_pair_expect_mixed(const mps_request* reqs, const mps_mixed_plan* plan,
                                hipStream_t stream) {
  int rc = check_plan(reqs, plan);
  if (rc) return rc;
  for (int k = 0; k < MPS_MIXED_BUCKETS; ++k) {
    if (!plan->count[k]) continue;
    const int S = bucket_slot(k), b0 = plan->begin[k], c = plan->count[k], ns = plan->max_sites[k];
    hipError_t e;
    if (S == 16)
      e = launch_measure16_mixed(reqs, b0, c, ns, bucket_fp64(k), stream);
    else if (bucket_fp64(k))
      e = launch_measure_mixed<double, double>(reqs, b0, c, ns, S, stream);
    else
      e = launch_measure_mixed<float, float>(reqs, b0, c, ns, S, stream);
    if (e != hipSuccess) return check_hip(e, "mixed measurement launch");
  }
  return ok();
}

int mps_set_exact_layers(int32_t mode) {
  switch (mode) {
    case MPS_EXACT_MPO: set_exact_qr(kExactMpo); break;
    case MPS_EXACT_QR: set_exact_qr(kExactQr); break;
    case MPS_EXACT_SVD: set_exact_qr(kExactSvd); break;
    default: return fail(MPS_ERR_INVALID_ARG, "mode=%d", mode);
  }
  return ok();
}

int mps_set_measure_tuning(int32_t pair_block_images, int32_t pair_waves_per_cu) {
  if (pair_block_images < 0 || pair_waves_per_cu < 0 || (pair_waves_per_cu > 0 && pair_waves_per_cu < 4))
    return fail(MPS_ERR_INVALID_ARG, "pair_block_images=%d pair_waves_per_cu=%d", pair_block_images,
                pair_waves_per_cu);
  g_pair_block_groups = (pair_block_images + 7) / 8;
  g_pair_waves_per_cu = pair_waves_per_cu;
  return ok();
}

int mps_set_mixed_tuning(int32_t bucket, int32_t blocks_per_cu) {
  if (bucket < 0 || bucket >= MPS_MIXED_BUCKETS || blocks_per_cu < 0)
    return fail(MPS_ERR_INVALID_ARG, "bucket=%d blocks_per_cu=%d", bucket, blocks_per_cu);
  g_mixed_blocks_per_cu[bucket] = blocks_per_cu;
  return ok();
}

size_t mps_ano_train_workspace_bytes(int32_t batch, int32_t m, int32_t out_dim, int32_t is_f64) {
  if (batch < 1 || m < 1 || m > 4096 || out_dim < 1) return 0;
  return train_workspace_elems(batch, m, out_dim) * (is_f64 ? sizeof(double) : sizeof(float));
}

int mps_ano_train_step(const void* pauli, const void* target, void* A, void* B, void* D, void* W,
                       void* bias, void* adam_m, void* adam_v, int32_t batch, int32_t m,
                       int32_t out_dim, int32_t step, double lr_obs, double lr_lin, double beta1,
                       double beta2, double eps, void* loss, void* workspace, int32_t is_f64,
                       hipStream_t stream) {
  if (batch < 1 || m < 1 || out_dim < 1) return fail(MPS_ERR_INVALID_ARG, "batch, m and out_dim must be >= 1");
  if (m > 4096) return fail(MPS_ERR_CAPACITY, "m=%d exceeds 4096", m);
  if (step < 1) return fail(MPS_ERR_INVALID_ARG, "step=%d: Adam steps count from 1", step);
  if (!(beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0 && eps > 0.0))
    return fail(MPS_ERR_INVALID_ARG, "Adam needs 0 <= beta1, beta2 < 1 and eps > 0");
  if (!pauli || !target || !A || !B || !D || !W || !bias || !adam_m || !adam_v || !loss || !workspace)
    return fail(MPS_ERR_INVALID_ARG, "NULL argument");
  hipError_t e = is_f64
      ? launch_train_step<double>((const double*)pauli, (const double*)target, (double*)A, (double*)B,
                                  (double*)D, (double*)W, (double*)bias, (double*)adam_m,
                                  (double*)adam_v, batch, m, out_dim, step, lr_obs, lr_lin, beta1,
                                  beta2, eps, (double*)loss, (double*)workspace, stream)
      : launch_train_step<float>((const float*)pauli, (const float*)target, (float*)A, (float*)B,
                                 (float*)D, (float*)W, (float*)bias, (float*)adam_m, (float*)adam_v,
                                 batch, m, out_dim, step, lr_obs, lr_lin, beta1, beta2, eps,
                                 (float*)loss, (float*)workspace, stream);
  if (e != hipSuccess) return check_hip(e, "training step launch");
  return ok();
}

const char* mps_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
