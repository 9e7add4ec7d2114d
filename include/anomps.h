/*
 * anomps.h -- C-ABI of the MI355X (gfx950) library for MPS Pauli-pair feature extraction.
 *
 * The library simulates the feature-extraction circuit of an adaptive non-local observable
 * VQC on a matrix product state (§II of the paper) for a batch of images and returns the
 * fixed two-qubit Pauli expectations that the trainable observables are built from:
 *
 *   image x (p x p pixels, x in [0,1], row-major site k = r*p + c)
 *     -> product state, qubit k in R_Y(pi x_k)|0>                              (mps_init_batch)
 *     -> L layers: R_Y(theta_k) R_Z(phi_k) on every qubit, then CNOT(k,k+1) for
 *        k = 0..n-2, each two-site update split by an SVD that keeps at most chi
 *        singular values (§II-B, Eq. (3))                                     (mps_apply_layer)
 *     -> <P_a (x) P_b> on each listed pair (i, j)   (§II-C, Eq. (4)-(5))      (mps_pauli_pair_expect)
 *     -> q_q = sum_alpha c_{q,alpha} <P_alpha>, y = W q + b   (Eq. (4)-(6))   (mps_ano_coeffs, mps_ano_readout)
 *
 * Conventions shared by every call:
 *  - Ownership: every pointer argument is caller-owned.  Unless a parameter says "host", it
 *    points to DEVICE memory of the current HIP device.  The library never allocates device
 *    memory in these calls; it keeps only host-side tables, the message of the last error and,
 *    per device, one stream of its own with two events (default priority, created by the first
 *    mps_apply_layers call that runs a run of exact layers, kept until the process ends).
 *  - Streams: every call only enqueues work on `stream` (0 = the null stream) and returns
 *    without synchronising.  Independent batches may run on different streams.
 *  - Errors: argument and capacity errors are detected on the host and returned before any
 *    launch (the batch is left unchanged).  A failed launch returns MPS_ERR_HIP.  Numerical
 *    trouble inside a kernel is reported per image in `status` (read after the stream is
 *    synchronised).  mps_last_error() gives a message for the last non-OK return of the
 *    calling thread.
 *  - Pauli index: alpha = 4a + b - 1 with I,X,Y,Z = 0,1,2,3, P_a acting on the lower site i,
 *    P_b on site j; the identity-identity term (a = b = 0) is omitted (its value is 1).
 *  - Gates: R_Y(t) = [[cos t/2, -sin t/2], [sin t/2, cos t/2]], R_Z(t) = diag(e^{-it/2}, e^{it/2}),
 *    CNOT(c,t) |c,t> = |c, t XOR c>.
 *  - Complex numbers are stored as interleaved (re, im) pairs of the precision's real type.
 */
#ifndef ANOMPS_H
#define ANOMPS_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return value of every int-returning call. */
typedef enum {
  MPS_OK = 0,
  MPS_ERR_INVALID_ARG = -1, /* bad pointer, size, pair, precision or order of calls */
  MPS_ERR_CAPACITY = -2,    /* request exceeds a documented limit (e.g. bond dimension) */
  MPS_ERR_HIP = -3,         /* a HIP runtime call or kernel launch failed */
  MPS_ERR_UNSUPPORTED = -4  /* valid request outside what this build implements */
} mps_status;

/* Arithmetic of a batch.  FP64: complex128 state, FP64 everywhere.  FP32: complex64 state,
 * environments, pair contractions and outputs in FP32; the SVD, the orthogonalisation of the
 * canonical sweep and the singular-value renormalisation in FP64.  SPLIT_BF16: as FP32 but,
 * for batches whose slot is 16 wide, the environment and pair contractions run on bf16 matrix
 * cores: each FP32 operand x = x_hi + x_lo (x_hi = bf16(x), x_lo = bf16(x - x_hi)) and each
 * product a*b = a_hi b_hi + a_hi b_lo + a_lo b_hi, accumulated in FP32 (relative error of a
 * product term <= ~3 * 2^-18).  Narrower slots use the FP32 vector contractions.  Not accepted
 * in mixed request tables. */
typedef enum { MPS_PREC_FP64 = 0, MPS_PREC_FP32 = 1, MPS_PREC_SPLIT_BF16 = 2 } mps_precision;

/* Per-image status word (bit flags, 0 = fine). */
enum {
  MPS_IMG_OK = 0,
  MPS_IMG_NONFINITE = 1,      /* a pixel or an intermediate value was NaN/Inf */
  MPS_IMG_NO_CONVERGENCE = 2  /* a Jacobi SVD hit its sweep limit (result still written) */
};

/* Largest bond dimension this build keeps (after the min with 2^layers and the chain ends).
 * Slots up to 16 run one wavefront per image with the bond's matrices in LDS; slots 32, 64 and
 * 128 run one 256-lane workgroup per image with the bond's matrices (up to 256 x 256
 * complex128) in an FP64 workspace that the library places in the env buffer (see
 * mps_env_bytes).  Both use the same arithmetic and truncation rule.  Mixed request tables
 * take slots up to MPS_MIXED_MAX_SLOT. */
#define MPS_MAX_BOND 128
#define MPS_MIXED_MAX_SLOT 16
/* Largest number of sites. */
#define MPS_MAX_SITES 1024

/*
 * Bond dimension after `layers` layers, between sites `bond` and `bond`+1:
 *   D = min(chi, 2^layers, 2^(bond+1), 2^(n_sites-bond-1)).
 * chi is the maximum virtual dimension of §II-B; each two-site update keeps
 * min(chi, rows, cols) singular values of its (2 D_left) x (2 D_right) matrix, which gives this
 * closed form for the CNOT-ladder circuit.  Returns 0 for out-of-range arguments.
 */
int32_t mps_bond_dim(int32_t n_sites, int32_t chi, int32_t layers, int32_t bond);

/* Slot dimension of a batch that will receive `n_layers` layers: the largest bond dimension it
 * will reach, max_k mps_bond_dim(n_sites, chi, n_layers, k) (at least 1). */
int32_t mps_slot_dim(int32_t n_sites, int32_t chi, int32_t n_layers);

/*
 * Sizes in bytes of the caller-owned buffers of a batch (0 for invalid arguments).
 *  state : [batch][n_sites][S][2][S] complex, S = mps_slot_dim(...).  Site k's tensor
 *          A[k] (D_{k-1} x 2 x D_k) occupies the leading corner: element (a, s, b) at
 *          ((a*2 + s)*S + b).  Entries outside the corner are never read.
 *  env   : [batch][2][n_sites+1][S][S] complex: left environments L_0..L_n then right
 *          environments R_0..R_n (ket index first).  Filled by mps_pauli_pair_expect.
 *          For S > 16 the buffer continues (at the next 256-byte boundary) with an FP64
 *          workspace of 48 S^2 complex128 elements (rounded up to 64) per image, which
 *          mps_apply_layer and mps_pauli_pair_expect overwrite; env is then also required by
 *          the layer calls.
 */
size_t mps_state_bytes(int32_t n_sites, int32_t chi, int32_t n_layers, int32_t batch, int32_t precision);
size_t mps_env_bytes(int32_t n_sites, int32_t chi, int32_t n_layers, int32_t batch, int32_t precision);

/* A batch of images that share n_sites, chi, the number of layers and the layer angles.
 * Plain descriptor: the caller fills every field except layers_done, which the library
 * maintains (set to 0 by mps_init_batch, incremented by mps_apply_layer). */
typedef struct {
  int32_t n_sites;    /* n = p*p qubits, 2 <= n <= MPS_MAX_SITES */
  int32_t chi;        /* maximum bond dimension, >= 1 */
  int32_t n_layers;   /* layers this batch will receive (sizes the slots), >= 0 */
  int32_t batch;      /* images, >= 1 */
  int32_t precision;  /* mps_precision */
  int32_t layers_done;
  void* state;        /* device, >= mps_state_bytes(...) */
  void* env;          /* device, >= mps_env_bytes(...) */
  int32_t* status;    /* device [batch], per-image MPS_IMG_* flags (OR-ed) */
} mps_batch;

/*
 * Angle-encode the pixels into the product state (§II-B: one pixel per qubit, row-major):
 * A[k] = (cos(pi x_k / 2), sin(pi x_k / 2)) as a 1 x 2 x 1 tensor.  Clears `status` and sets
 * layers_done = 0.  pixels: device [batch][n_sites] float64 (values outside [0,1] are
 * accepted; NaN/Inf set MPS_IMG_NONFINITE).
 */
int mps_init_batch(mps_batch* b, const double* pixels, hipStream_t stream);

/*
 * Apply the next layer (§II-B): the one-qubit gates R_Y(theta_k) R_Z(phi_k) (updating single
 * site tensors), then CNOT(k, k+1) for k = 0..n-2 in order, each as a two-site update: contract
 * A[k] A[k+1], apply the CNOT, split with a one-sided Jacobi SVD in FP64, keep the
 * min(chi, rows, cols) largest singular triplets, rescale the kept singular values to unit
 * 2-norm, A[k] <- U (left-orthonormal), A[k+1] <- S V^dag.  Before the ladder the chain is
 * swept right to left into right-canonical form (the one-qubit gates are applied during that
 * sweep), so every truncation acts on Schmidt values.
 *  theta, phi : device [n_sites] float64, this layer's angles (shared by the batch).
 *  trunc_err  : device [batch][n_sites-1] float64 or NULL; receives the discarded weight
 *               sum_discarded sigma^2 / sum sigma^2 of every bond of this layer.
 * Errors: MPS_ERR_INVALID_ARG if layers_done == n_layers, the batch was not initialised, or
 *   env is NULL for a slot wider than 16.
 */
int mps_apply_layer(mps_batch* b, const double* theta, const double* phi, double* trunc_err,
                    hipStream_t stream);

/*
 * Apply the next `count` ladder layers (§II-B) in one call: the same result as `count` calls of
 * mps_apply_layer with theta + r*n_sites, phi + r*n_sites and trunc_err + r*batch*(n_sites-1),
 * r = 0..count-1.  Under MPS_EXACT_MPO (slots <= 16) a run of two or more consecutive layers that
 * keep every singular value is applied by two launches: the sites that lie between the reduced
 * chain ends in every layer of the run take all of the run's layers in on-chip memory and are
 * written once; the ends take the layers one after the other.  The state is the one the
 * separate calls produce up to rounding: in complex64 the run's intermediate tensors stay in
 * FP64 instead of being rounded to FP32 after each layer.
 *  theta, phi : device [count][n_sites] float64.
 *  trunc_err  : device [count][batch][n_sites-1] float64 or NULL.
 * Errors: MPS_ERR_INVALID_ARG if count < 1 or layers_done + count > n_layers, and as
 *   mps_apply_layer.
 */
int mps_apply_layers(mps_batch* b, int32_t count, const double* theta, const double* phi,
                     double* trunc_err, hipStream_t stream);

/*
 * How mps_apply_layer (and the mixed layer step) handle a layer in which the bond rule keeps
 * every singular value, i.e. D_k = min(2 D_{k-1}, 2 D_{k+1}^old) at every bond k (always the
 * case when chi >= 2^n_layers, the exact regime of §II-B).  Nothing can be discarded in such a
 * layer, so every mode below produces the state the SVD ladder produces (up to rounding and
 * the gauge of each bond), the features agree to rounding, and trunc_err is 0.
 *  MPS_EXACT_MPO (default): the CNOT ladder is the product operator that maps each bit to the
 *    parity of the bits up to it (bond dimension 2), so the layer is applied site by site:
 *    B[k][(p,a), y, (q,b)] = (U_k A[k])[a, y XOR p, b] delta(q, y), U_k = R_Y R_Z of site k.
 *    Where the rule keeps D_k < 2 D_k^old (the chain ends) the doubled bond is reduced exactly:
 *    those sites become identity tensors and the product of their B's is carried into the
 *    first site with a full bond.  No site is orthonormalised (the norm is the input's, the
 *    layer being unitary); the measurement contracts both environments and needs no gauge.
 *    The brickwork program of mps_apply_layer_program takes the same form (one bit per bond:
 *    an even site passes its input bit, an odd site its output bit) unless its two end carries
 *    land on one site.  Slots wider than 16 take the same contraction (the carries in the
 *    batch's FP64 workspace).  A layer that keeps every singular value but is followed, in the
 *    batch's n_layers, by a truncating layer takes the MPS_EXACT_QR path instead: the
 *    truncating layer's SVDs converge faster from the canonical gauge that path leaves.
 *  MPS_EXACT_QR: one left-to-right sweep; each two-site matrix Theta' is split exactly, by
 *    Householder QR in FP64 (A[k] <- Q, centre <- R) or, when D_k equals its row count, as
 *    A[k] <- identity, centre <- Theta'; the one-qubit gates are applied as each site is
 *    reached and the last centre is scaled to unit norm.
 *  MPS_EXACT_SVD: the canonical sweep + Jacobi SVD ladder, as for every other layer.
 * Layers with any truncating bond keep the canonical sweep (so do slots wider than 16 under
 * MPS_EXACT_QR); under MPS_EXACT_MPO and MPS_EXACT_QR their ladder still splits each bond that
 * keeps all min(rows, cols) singular values exactly (identity or QR, centre renormalised by
 * |Theta'|) and runs the Jacobi SVD only where weight can be discarded.  Process-wide
 * setting, read at each launch.  Returns MPS_ERR_INVALID_ARG for another mode.
 */
enum { MPS_EXACT_QR = 0, MPS_EXACT_SVD = 1, MPS_EXACT_MPO = 2 };
int mps_set_exact_layers(int32_t mode);

/* Layer programs of mps_apply_layer_program. */
enum {
  MPS_LAYER_RYRZ_LADDER = 0,    /* R_Y(theta_k) R_Z(phi_k), then the CNOT ladder (mps_apply_layer) */
  MPS_LAYER_H_RY_BRICKWORK = 1  /* the paper's encoding-entangling layer, see below */
};

/*
 * Apply the next layer of a given program.
 *  MPS_LAYER_RYRZ_LADDER: exactly mps_apply_layer (pixels ignored, may be NULL).
 *  MPS_LAYER_H_RY_BRICKWORK (§II-B, Eq. (2)): on every qubit a Hadamard gate followed by
 *    R_Y(phi_k), phi_k = 2 pi x_k - pi from the image's own pixel, then CNOT(k, k+1) on every
 *    even bond k, then on every odd bond (staggered nearest-neighbour CNOTs).  Implemented as a
 *    right-canonical sweep (gates applied), a left-to-right sweep over the even bonds, a second
 *    right-canonical sweep and a sweep over the odd bonds; bonds without a CNOT in a sweep only
 *    move the orthogonality centre.  Bond dimensions after the layer follow mps_bond_dim; start
 *    the batch from |0...0> with mps_init_zero.  pixels: device [batch][n_sites] float64
 *    (theta, phi ignored, may be NULL).
 *  trunc_err as in mps_apply_layer (each bond once per layer).
 * Errors: MPS_ERR_INVALID_ARG for an unknown program or a NULL argument it needs, and as
 * mps_apply_layer.
 */
int mps_apply_layer_program(mps_batch* b, int32_t program, const double* theta,
                            const double* phi, const double* pixels, double* trunc_err,
                            hipStream_t stream);

/* Product state |0...0> for every image (the start of the paper's encoding circuit); clears
 * status and sets layers_done = 0. */
int mps_init_zero(mps_batch* b, hipStream_t stream);

/*
 * Host-side check of a pair list (host pointer): 0 <= i < j < n_sites for every pair.
 * Returns MPS_OK or MPS_ERR_INVALID_ARG (with the first offending pair in mps_last_error()).
 */
int mps_validate_pairs(const int32_t* pairs_host, int32_t m, int32_t n_sites);

/*
 * Two-qubit Pauli expectations on the listed pairs (§II-C, Eq. (4)-(5)):
 *   out[b][q][4a + c - 1] = Re Tr(rho_{i_q j_q} (P_a (x) P_c)).
 * Computes the left and right environment sweeps into b->env, then for every start site i the
 * reduced density matrices of all pairs (i, j) by carrying the open two-layer block from i
 * through the transfer matrices of sites i+1..j-1.  pairs: device [m][2] int32 with i < j
 * (check the list with mps_validate_pairs; an invalid pair yields NaN outputs).  out: device
 * [batch][m][15], float64 for MPS_PREC_FP64, float32 otherwise.  m may be 0.
 */
int mps_pauli_pair_expect(mps_batch* b, const int32_t* pairs, int32_t m, void* out,
                          hipStream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): mps_pauli_pair_expect with the environments kept in
 * a fixed scratch array of the library instead of b->env (which is ignored and may be NULL).
 * The array holds MPS_NOALLOC_SCRATCH_BYTES on every device the library runs on (its own copy
 * per device, held until the process ends); the call allocates nothing and calls no allocating
 * routine.  Results are those of mps_pauli_pair_expect on the same batch.
 * Errors: as mps_pauli_pair_expect; MPS_ERR_CAPACITY when the environments
 *   (2 (n_sites+1) S^2 complex values per image, S = mps_slot_dim) exceed the scratch;
 *   MPS_ERR_UNSUPPORTED for slots wider than 16.
 * Every call on a device shares that device's scratch and it keeps the last call's contents
 * (nothing in it needs to start at zero: each call writes every environment before reading
 * it).  Calls that overlap on one device -- on different streams, or from different threads --
 * race on the scratch: serialise them.
 */
#define MPS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int mps_pauli_pair_expect_noalloc(mps_batch* b, const int32_t* pairs, int32_t m, void* out,
                                  hipStream_t stream);

/*
 * Schedule of the measurement's pair kernel for 16-wide slots (host-side settings of the calling
 * process, read at each launch):
 *  pair_block_images : launch order -- the batch is taken in blocks of this many images (rounded
 *                      up to a multiple of 8), every start site of a block's images before the
 *                      next block, start site major inside a block; 0 = the whole batch as one
 *                      block.  Default 64.
 *  pair_waves_per_cu : at most this many resident workgroups (one wavefront each) per compute
 *                      unit, enforced through the launch's LDS allocation; 0 (the default) = as
 *                      many as the registers allow; otherwise >= 4.
 * Results do not depend on either: each (image, start site) runs the same arithmetic.  The
 * autotuner of the Python package chooses them by measurement.  MPS_ERR_INVALID_ARG for values
 * out of range.
 */
int mps_set_measure_tuning(int32_t pair_block_images, int32_t pair_waves_per_cu);

/*
 * Pauli-basis coefficients of the adaptive observables (§II-A, Eq. (4)):
 *   H_q[j][j] = D[q][j]; for the upper positions (0,1),(0,2),(0,3),(1,2),(1,3),(2,3), in this
 *   order, H_q[j][k] = A[q][idx] + i B[q][idx] and H_q[k][j] = conj; basis |s_i s_j>.
 *   coeff[q][4a + c] = Tr(H_q (P_a (x) P_c)) / 4, alpha = 0 the identity term.
 * A, B: device [m][6]; D: device [m][4]; coeff: device [m][16].  Real type float64 if is_f64,
 * float32 otherwise.
 */
int mps_ano_coeffs(const void* A, const void* B, const void* D, int32_t m, void* coeff,
                   int32_t is_f64, hipStream_t stream);

/*
 * Observable-weighted linear readout (Eq. (5)-(6)):
 *   q[b][q] = coeff[q][0] + sum_{alpha=0..14} coeff[q][alpha+1] * pauli[b][q][alpha]
 *   y[b][o] = sum_q W[o][q] q[b][q] + bias[o]
 * pauli: device [batch][m][15]; coeff: [m][16]; W: [out_dim][m]; bias: [out_dim] or NULL;
 * y: [batch][out_dim].  All float64 if is_f64, else float32.  m <= 4096 (MPS_ERR_CAPACITY).
 */
int mps_ano_readout(const void* pauli, const void* coeff, const void* W, const void* bias,
                    int32_t batch, int32_t m, int32_t out_dim, void* y, int32_t is_f64,
                    hipStream_t stream);

/*
 * One training step of the observables and the linear layer on cached features (§II-C: the
 * expectations are computed once and cached; §II-D: separate Adam optimizers for (A, B, D) and
 * (W, b)).  Loss: the MSE term of Eq. (7) only (the LPIPS term needs a trained network),
 *   L = mean_{b,o} (y_hat[b][o] - target[b][o])^2,  y_hat from (A, B, D, W, bias) as in
 *   mps_ano_coeffs / mps_ano_readout.
 * Gradients by the chain rule through Eq. (6), (5), (4); then Adam with bias correction
 * (Kingma & Ba): m = beta1 m + (1-beta1) g, v = beta2 v + (1-beta2) g^2,
 * p -= lr m/(1-beta1^step) / (sqrt(v/(1-beta2^step)) + eps), lr = lr_obs for A, B, D and lr_lin
 * for W, bias.
 *  pauli [batch][m][15], target [batch][out_dim]: device, read only.
 *  A [m][6], B [m][6], D [m][4], W [out_dim][m], bias [out_dim]: device, updated in place.
 *  adam_m, adam_v: device [16 m + out_dim m + out_dim], the moments of A, B, D, W, bias packed in
 *    that order; zero before step 1, caller-owned between steps.
 *  loss: device [1], receives L before the update.  workspace: device, >=
 *    mps_ano_train_workspace_bytes(batch, m, out_dim, is_f64).  Real type float64 if is_f64.
 * Errors: MPS_ERR_INVALID_ARG (sizes, step < 1, Adam constants, NULL), MPS_ERR_CAPACITY (m > 4096).
 */
size_t mps_ano_train_workspace_bytes(int32_t batch, int32_t m, int32_t out_dim, int32_t is_f64);
int mps_ano_train_step(const void* pauli, const void* target, void* A, void* B, void* D, void* W,
                       void* bias, void* adam_m, void* adam_v, int32_t batch, int32_t m,
                       int32_t out_dim, int32_t step, double lr_obs, double lr_lin, double beta1,
                       double beta2, double eps, void* loss, void* workspace, int32_t is_f64,
                       hipStream_t stream);

/* ---------------------------------------------------------------------------------------
 * Mixed requests (continuous batching).  A request is one image with its own n_sites, chi,
 * layer count, precision, angles, pair list and buffers; a table of requests runs through one
 * persistent launch per (slot size, precision) bucket and layer step.  The arithmetic per
 * image is exactly that of the batch calls above (the same device code runs), so a request's
 * results do not depend on the other requests of the table.
 * --------------------------------------------------------------------------------------- */
typedef struct {
  int32_t n_sites;        /* 2 <= n <= MPS_MAX_SITES */
  int32_t chi;            /* maximum bond dimension, >= 1 */
  int32_t n_layers;       /* layers this request receives, >= 0 */
  int32_t precision;      /* MPS_PREC_FP64 or MPS_PREC_FP32 */
  int32_t n_pairs;        /* m of this request's pair list, >= 0 */
  int32_t reserved;       /* set to 0 */
  const double* pixels;   /* device [n_sites] float64 */
  void* state;            /* device, >= mps_state_bytes(n_sites, chi, n_layers, 1, precision) */
  void* env;              /* device, >= mps_env_bytes(n_sites, chi, n_layers, 1, precision) */
  const double* theta;    /* device [n_layers][n_sites] float64 */
  const double* phi;      /* device [n_layers][n_sites] float64 */
  double* trunc_err;      /* device [n_layers][n_sites-1] float64, or NULL */
  const int32_t* pairs;   /* device [n_pairs][2], checked like mps_validate_pairs */
  void* out;              /* device [n_pairs][15]: float64 for FP64, float32 for FP32 */
  int32_t* ctrl;          /* device [2]: ctrl[0] = layers applied so far, ctrl[1] = MPS_IMG_* flags */
} mps_request;

/* Requests are grouped by bucket = 4*(precision == FP32) + log2(S) - 1, S = mps_slot_dim(...);
 * S must not exceed MPS_MIXED_MAX_SLOT (MPS_ERR_CAPACITY from mps_plan_mixed otherwise). */
#define MPS_MIXED_BUCKETS 8
typedef struct {
  int32_t n_req;
  int32_t begin[MPS_MIXED_BUCKETS];      /* first table index of each bucket */
  int32_t count[MPS_MIXED_BUCKETS];      /* requests in each bucket */
  int32_t max_sites[MPS_MIXED_BUCKETS];  /* largest n_sites in each bucket */
} mps_mixed_plan;

/*
 * Host-side planning of a request table (host pointer reqs_host; the device pointers inside
 * are only checked for NULL).  Validates every request like the batch calls would, then writes
 * order[t] = the index in reqs_host of the request that belongs at table position t: requests
 * grouped by bucket, and within a bucket by decreasing estimated work (largest first, so the
 * persistent launches finish evenly).  The caller uploads the table in that order and passes
 * it with `plan` to the calls below.  Errors: MPS_ERR_INVALID_ARG / MPS_ERR_CAPACITY naming
 * the first bad request; MPS_ERR_UNSUPPORTED for SPLIT_BF16 requests.
 */
int mps_plan_mixed(const mps_request* reqs_host, int32_t n_req, int32_t* order,
                   mps_mixed_plan* plan);

/* Encode every request of the table (mps_init_batch per request); sets ctrl = {0, flags}.
 * reqs: device table ordered as `plan` says. */
int mps_init_mixed(const mps_request* reqs, const mps_mixed_plan* plan, hipStream_t stream);

/*
 * Apply one more layer (mps_apply_layer) to every request of the table with
 * ctrl[0] < n_layers, and increment its ctrl[0]; requests already done are skipped.  One
 * persistent launch per non-empty bucket: each workgroup takes the next request from a queue
 * counter in `queue` (device [MPS_MIXED_BUCKETS] int32, caller-owned, reset by this call with
 * a kernel, so the call can be captured in a HIP graph).  Concurrent calls must not share
 * `queue`.  The grid of each bucket is set by mps_set_mixed_tuning (default: what fits).
 */
int mps_apply_layer_mixed(const mps_request* reqs, const mps_mixed_plan* plan, int32_t* queue,
                          hipStream_t stream);

/* Environments and Pauli-pair expectations (mps_pauli_pair_expect) of every request of the
 * table, at the layers applied so far. */
int mps_pauli_pair_expect_mixed(const mps_request* reqs, const mps_mixed_plan* plan,
                                hipStream_t stream);

/* Persistent-grid size of a bucket's layer launch, in workgroups per compute unit
 * (0 = the occupancy limit, the default).  Host-side setting of the calling process; the
 * autotuner in the Python package chooses it by measurement.  MPS_ERR_INVALID_ARG for a bad
 * bucket or a negative value. */
int mps_set_mixed_tuning(int32_t bucket, int32_t blocks_per_cu);

/* Message for the last non-OK return on the calling thread ("" if none).  The pointer stays
 * valid until the next call on that thread. */
const char* mps_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ANOMPS_H */
