"""Thin Python binding of libanomps (include/anomps.h): argument marshalling only.

Every computation happens in the HIP kernels of the shared library; this module only turns
torch device tensors into pointers, the current torch stream into a hipStream_t, and non-OK
return codes into exceptions.  There is no CPU fallback: if the library is missing, loading
fails with an error.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libanomps.so")

MPS_OK = 0
PREC_FP64, PREC_FP32, PREC_SPLIT_BF16 = 0, 1, 2
PRECISIONS = {"fp64": PREC_FP64, "fp32": PREC_FP32, "split_bf16": PREC_SPLIT_BF16}
LAYER_RYRZ_LADDER, LAYER_H_RY_BRICKWORK = 0, 1
IMG_NONFINITE, IMG_NO_CONVERGENCE = 1, 2
MAX_BOND = 128
MIXED_MAX_SLOT = 16

_lib = None


class MpsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"anomps error {code}: {msg}")
        self.code = code


class MpsBatch(ctypes.Structure):
    _fields_ = [
        ("n_sites", ctypes.c_int32),
        ("chi", ctypes.c_int32),
        ("n_layers", ctypes.c_int32),
        ("batch", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("layers_done", ctypes.c_int32),
        ("state", ctypes.c_void_p),
        ("env", ctypes.c_void_p),
        ("status", ctypes.c_void_p),
    ]


class MpsRequest(ctypes.Structure):
    _fields_ = [
        ("n_sites", ctypes.c_int32),
        ("chi", ctypes.c_int32),
        ("n_layers", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("n_pairs", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("pixels", ctypes.c_void_p),
        ("state", ctypes.c_void_p),
        ("env", ctypes.c_void_p),
        ("theta", ctypes.c_void_p),
        ("phi", ctypes.c_void_p),
        ("trunc_err", ctypes.c_void_p),
        ("pairs", ctypes.c_void_p),
        ("out", ctypes.c_void_p),
        ("ctrl", ctypes.c_void_p),
    ]


MIXED_BUCKETS = 8


class MixedPlan(ctypes.Structure):
    _fields_ = [
        ("n_req", ctypes.c_int32),
        ("begin", ctypes.c_int32 * MIXED_BUCKETS),
        ("count", ctypes.c_int32 * MIXED_BUCKETS),
        ("max_sites", ctypes.c_int32 * MIXED_BUCKETS),
    ]


EXPORTS = {
    "mps_bond_dim": (ctypes.c_int32, [ctypes.c_int32] * 4),
    "mps_slot_dim": (ctypes.c_int32, [ctypes.c_int32] * 3),
    "mps_state_bytes": (ctypes.c_size_t, [ctypes.c_int32] * 5),
    "mps_env_bytes": (ctypes.c_size_t, [ctypes.c_int32] * 5),
    "mps_init_batch": (ctypes.c_int, [ctypes.POINTER(MpsBatch), ctypes.c_void_p, ctypes.c_void_p]),
    "mps_apply_layer": (ctypes.c_int, [ctypes.POINTER(MpsBatch), ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p]),
    "mps_apply_layers": (ctypes.c_int, [ctypes.POINTER(MpsBatch), ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "mps_apply_layer_program": (ctypes.c_int, [ctypes.POINTER(MpsBatch), ctypes.c_int32,
                                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_void_p, ctypes.c_void_p]),
    "mps_init_zero": (ctypes.c_int, [ctypes.POINTER(MpsBatch), ctypes.c_void_p]),
    "mps_validate_pairs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]),
    "mps_pauli_pair_expect": (ctypes.c_int, [ctypes.POINTER(MpsBatch), ctypes.c_void_p,
                                             ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "mps_pauli_pair_expect_noalloc": (ctypes.c_int, [ctypes.POINTER(MpsBatch), ctypes.c_void_p,
                                                     ctypes.c_int32, ctypes.c_void_p,
                                                     ctypes.c_void_p]),
    "mps_ano_coeffs": (ctypes.c_int, [ctypes.c_void_p] * 3 + [ctypes.c_int32, ctypes.c_void_p,
                                                             ctypes.c_int32, ctypes.c_void_p]),
    "mps_ano_readout": (ctypes.c_int, [ctypes.c_void_p] * 4 + [ctypes.c_int32] * 3 +
                        [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "mps_plan_mixed": (ctypes.c_int, [ctypes.POINTER(MpsRequest), ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.POINTER(MixedPlan)]),
    "mps_init_mixed": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(MixedPlan), ctypes.c_void_p]),
    "mps_apply_layer_mixed": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(MixedPlan),
                                             ctypes.c_void_p, ctypes.c_void_p]),
    "mps_pauli_pair_expect_mixed": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(MixedPlan),
                                                   ctypes.c_void_p]),
    "mps_set_mixed_tuning": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32]),
    "mps_set_measure_tuning": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32]),
    "mps_set_exact_layers": (ctypes.c_int, [ctypes.c_int32]),
    "mps_ano_train_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32] * 4),
    "mps_ano_train_step": (ctypes.c_int, [ctypes.c_void_p] * 9 + [ctypes.c_int32] * 4 +
                           [ctypes.c_double] * 5 + [ctypes.c_void_p, ctypes.c_void_p,
                                                    ctypes.c_int32, ctypes.c_void_p]),
    "mps_last_error": (ctypes.c_char_p, []),
}


def lib():
    """Load libanomps.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} not found: build it with "
                               "`python -m paper_2607_10280_amd.build`")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def _check(rc: int):
    if rc != MPS_OK:
        raise MpsError(rc, lib().mps_last_error().decode())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def bond_dim(n, chi, layers, bond) -> int:
    return int(lib().mps_bond_dim(n, chi, layers, bond))


def slot_dim(n, chi, layers) -> int:
    return int(lib().mps_slot_dim(n, chi, layers))


def state_bytes(n, chi, layers, batch, precision) -> int:
    return int(lib().mps_state_bytes(n, chi, layers, batch, precision))


def env_bytes(n, chi, layers, batch, precision) -> int:
    return int(lib().mps_env_bytes(n, chi, layers, batch, precision))


def validate_pairs(pairs: np.ndarray, n_sites: int) -> None:
    p = np.ascontiguousarray(pairs, dtype=np.int32)
    _check(lib().mps_validate_pairs(p.ctypes.data_as(ctypes.c_void_p), len(p), n_sites))


def footprint_bytes(n, chi, layers, batch, precision, m) -> int:
    """HBM bytes one batch holds: state + environments + status + Pauli outputs."""
    real = 8 if precision == PREC_FP64 else 4
    return (state_bytes(n, chi, layers, batch, precision) +
            env_bytes(n, chi, layers, batch, precision) + 4 * batch + batch * m * 15 * real)


@dataclass
class Batch:
    """A device-resident batch: the descriptor plus the torch tensors that own its memory."""
    desc: MpsBatch
    state: object
    env: object
    status: object

    @property
    def real_dtype(self):
        import torch
        return torch.float64 if self.desc.precision == PREC_FP64 else torch.float32


def new_batch(n_sites: int, chi: int, n_layers: int, batch: int, precision: int = PREC_FP32,
              device="cuda") -> Batch:
    import torch
    sb = state_bytes(n_sites, chi, n_layers, batch, precision)
    eb = env_bytes(n_sites, chi, n_layers, batch, precision)
    if sb == 0 or eb == 0:
        raise MpsError(-1, lib().mps_last_error().decode())
    state = torch.empty(sb, dtype=torch.uint8, device=device)
    env = torch.empty(eb, dtype=torch.uint8, device=device)
    status = torch.zeros(batch, dtype=torch.int32, device=device)
    desc = MpsBatch(n_sites, chi, n_layers, batch, precision, 0,
                    state.data_ptr(), env.data_ptr(), status.data_ptr())
    return Batch(desc, state, env, status)


def init_batch(b: Batch, pixels, stream=None) -> None:
    assert pixels.dtype.is_floating_point and pixels.is_cuda and pixels.is_contiguous()
    assert pixels.numel() == b.desc.batch * b.desc.n_sites
    _check(lib().mps_init_batch(ctypes.byref(b.desc), _ptr(pixels), _stream(stream)))


def apply_layer(b: Batch, theta, phi, trunc_err=None, stream=None) -> None:
    for t in (theta, phi):
        assert t.is_cuda and t.is_contiguous() and t.numel() == b.desc.n_sites
    _check(lib().mps_apply_layer(ctypes.byref(b.desc), _ptr(theta), _ptr(phi), _ptr(trunc_err),
                                 _stream(stream)))


def apply_layers(b: Batch, theta, phi, trunc_err=None, stream=None) -> None:
    """The next theta.shape[0] ladder layers in one call; theta, phi: device [count][n_sites]
    float64, trunc_err: device [count][batch][n_sites-1] float64 or None."""
    for t in (theta, phi):
        assert t.is_cuda and t.is_contiguous() and t.dim() == 2 and t.shape[1] == b.desc.n_sites
    assert theta.shape == phi.shape
    _check(lib().mps_apply_layers(ctypes.byref(b.desc), int(theta.shape[0]), _ptr(theta), _ptr(phi),
                                  _ptr(trunc_err), _stream(stream)))


def apply_layer_program(b: Batch, program: int, theta=None, phi=None, pixels=None,
                        trunc_err=None, stream=None) -> None:
    _check(lib().mps_apply_layer_program(ctypes.byref(b.desc), program, _ptr(theta), _ptr(phi),
                                         _ptr(pixels), _ptr(trunc_err), _stream(stream)))


def init_zero(b: Batch, stream=None) -> None:
    _check(lib().mps_init_zero(ctypes.byref(b.desc), _stream(stream)))


def pauli_pair_expect(b: Batch, pairs_dev, out, stream=None) -> None:
    m = 0 if pairs_dev is None else pairs_dev.shape[0]
    _check(lib().mps_pauli_pair_expect(ctypes.byref(b.desc), _ptr(pairs_dev), m, _ptr(out),
                                       _stream(stream)))


NOALLOC_SCRATCH_BYTES = 64 << 20


def pauli_pair_expect_noalloc(b: Batch, pairs_dev, out, stream=None) -> None:
    """mps_pauli_pair_expect with the environments in the library's fixed scratch array (no
    allocation; b.env is not used).  Calls that overlap on one device race on the scratch."""
    m = 0 if pairs_dev is None else pairs_dev.shape[0]
    _check(lib().mps_pauli_pair_expect_noalloc(ctypes.byref(b.desc), _ptr(pairs_dev), m, _ptr(out),
                                               _stream(stream)))


def ano_coeffs(A, B, D, coeff, stream=None) -> None:
    is_f64 = int(coeff.dtype.itemsize == 8)
    _check(lib().mps_ano_coeffs(_ptr(A), _ptr(B), _ptr(D), A.shape[0], _ptr(coeff), is_f64,
                                _stream(stream)))


def ano_readout(pauli, coeff, W, bias, y, stream=None) -> None:
    batch, m = pauli.shape[0], pauli.shape[1]
    out_dim = W.shape[0]
    is_f64 = int(y.dtype.itemsize == 8)
    _check(lib().mps_ano_readout(_ptr(pauli), _ptr(coeff), _ptr(W), _ptr(bias), batch, m,
                                 out_dim, _ptr(y), is_f64, _stream(stream)))


class AnoTrainer:
    """Device state of the observable/readout training on cached features: parameters, Adam
    moments and workspace (all torch tensors); `step` calls mps_ano_train_step."""

    def __init__(self, A, B, D, W, bias, batch: int, lr_obs=1e-2, lr_lin=1e-2, beta1=0.9,
                 beta2=0.999, eps=1e-8):
        import torch
        self.params = [A, B, D, W, bias]
        dt, dev = W.dtype, W.device
        m, out_dim = A.shape[0], W.shape[0]
        n = 16 * m + out_dim * m + out_dim
        self.mom = torch.zeros(n, dtype=dt, device=dev)
        self.vel = torch.zeros(n, dtype=dt, device=dev)
        self.loss = torch.zeros(1, dtype=dt, device=dev)
        self.is_f64 = int(dt == torch.float64)
        nb = int(lib().mps_ano_train_workspace_bytes(batch, m, out_dim, self.is_f64))
        if nb == 0:
            raise MpsError(-1, "invalid training sizes")
        self.ws = torch.empty(nb, dtype=torch.uint8, device=dev)
        self.batch, self.m, self.out_dim = batch, m, out_dim
        self.hyper = (lr_obs, lr_lin, beta1, beta2, eps)
        self.t = 0

    def step(self, pauli, target, stream=None):
        self.t += 1
        _check(lib().mps_ano_train_step(_ptr(pauli), _ptr(target), *[_ptr(p) for p in self.params],
                                        _ptr(self.mom), _ptr(self.vel), self.batch, self.m,
                                        self.out_dim, self.t, *self.hyper, _ptr(self.loss),
                                        _ptr(self.ws), self.is_f64, _stream(stream)))
        return self.loss


def extract_features(pixels, theta, phi, pairs, chi: int, precision: int = PREC_FP32,
                     stream=None, return_trunc_err: bool = False, per_layer: bool = False):
    """Whole path for one batch: encode, all layers (one mps_apply_layers call, or one
    mps_apply_layer call per layer with per_layer=True), Pauli-pair expectations.

    pixels [B][n] (host numpy or device tensor), theta/phi [L][n], pairs [m][2] (numpy, validated
    on the host).  Returns device tensors (features [B][m][15], status [B][, trunc_err [B][L][n-1]]).
    """
    import torch
    dev = torch.device("cuda")
    pairs_np = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    pix = torch.as_tensor(pixels, dtype=torch.float64, device=dev).contiguous()
    B, n = pix.shape
    validate_pairs(pairs_np, n)
    th = torch.as_tensor(np.asarray(theta), dtype=torch.float64, device=dev).contiguous()
    ph = torch.as_tensor(np.asarray(phi), dtype=torch.float64, device=dev).contiguous()
    L = th.shape[0]
    b = new_batch(n, chi, L, B, precision)
    init_batch(b, pix, stream)
    te = torch.zeros((B, max(L, 1), n - 1), dtype=torch.float64, device=dev) if return_trunc_err else None
    if per_layer:
        for layer in range(L):
            tl = torch.empty((B, n - 1), dtype=torch.float64, device=dev) if return_trunc_err else None
            apply_layer(b, th[layer], ph[layer], tl, stream)
            if return_trunc_err:
                te[:, layer] = tl
    elif L > 0:
        tl = torch.empty((L, B, n - 1), dtype=torch.float64, device=dev) if return_trunc_err else None
        apply_layers(b, th, ph, tl, stream)
        if return_trunc_err:
            te[:, :L] = tl.permute(1, 0, 2)
    pd = torch.as_tensor(pairs_np, device=dev)
    out = torch.empty((B, len(pairs_np), 15), dtype=b.real_dtype, device=dev)
    pauli_pair_expect(b, pd, out, stream)
    if return_trunc_err:
        return out, b.status, te
    return out, b.status


def paper_features(pixels, layers: int, pairs, chi: int, precision: int = PREC_FP32,
                   stream=None, return_trunc_err: bool = False):
    """The paper's own encoding circuit (§II-B, Eq. (2)) for a batch: |0...0>, then `layers`
    layers of H, R_Y(2 pi x - pi) and brickwork CNOTs, then the Pauli-pair expectations.
    pixels [B][n]; returns device tensors (features [B][m][15], status [B][, trunc_err])."""
    import torch
    dev = torch.device("cuda")
    pairs_np = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    pix = torch.as_tensor(pixels, dtype=torch.float64, device=dev).contiguous()
    B, n = pix.shape
    validate_pairs(pairs_np, n)
    b = new_batch(n, chi, layers, B, precision)
    init_zero(b, stream)
    te = torch.zeros((B, max(layers, 1), n - 1), dtype=torch.float64, device=dev) if return_trunc_err else None
    for layer in range(layers):
        tl = torch.empty((B, n - 1), dtype=torch.float64, device=dev) if return_trunc_err else None
        apply_layer_program(b, LAYER_H_RY_BRICKWORK, None, None, pix, tl, stream)
        if return_trunc_err:
            te[:, layer] = tl
    pd = torch.as_tensor(pairs_np, device=dev)
    out = torch.empty((B, len(pairs_np), 15), dtype=b.real_dtype, device=dev)
    pauli_pair_expect(b, pd, out, stream)
    if return_trunc_err:
        return out, b.status, te
    return out, b.status


# ----------------------------------------------------------------------------- mixed requests
def plan_mixed(reqs):
    """Host planning of a list of MpsRequest: returns (order, MixedPlan); the device table must
    hold reqs[order[0]], reqs[order[1]], ..."""
    n = len(reqs)
    arr = (MpsRequest * max(n, 1))(*reqs)
    order = np.zeros(max(n, 1), dtype=np.int32)
    plan = MixedPlan()
    _check(lib().mps_plan_mixed(arr, n, order.ctypes.data_as(ctypes.c_void_p), ctypes.byref(plan)))
    return order[:n], plan


def request_table(reqs, order, device="cuda"):
    """Device copy of the request table in plan order (a uint8 tensor holding the structs)."""
    import torch
    n = len(order)
    arr = (MpsRequest * max(n, 1))(*[reqs[i] for i in order])
    raw = np.frombuffer(bytes(arr), dtype=np.uint8)[: n * ctypes.sizeof(MpsRequest)].copy()
    return torch.as_tensor(raw, device=device)


def init_mixed(table, plan: MixedPlan, stream=None) -> None:
    _check(lib().mps_init_mixed(_ptr(table), ctypes.byref(plan), _stream(stream)))


def apply_layer_mixed(table, plan: MixedPlan, queue, stream=None) -> None:
    assert queue.is_cuda and queue.numel() >= MIXED_BUCKETS
    _check(lib().mps_apply_layer_mixed(_ptr(table), ctypes.byref(plan), _ptr(queue),
                                       _stream(stream)))


def pauli_pair_expect_mixed(table, plan: MixedPlan, stream=None) -> None:
    _check(lib().mps_pauli_pair_expect_mixed(_ptr(table), ctypes.byref(plan), _stream(stream)))


EXACT_QR, EXACT_SVD, EXACT_MPO = 0, 1, 2


def set_exact_layers(mode: int) -> None:
    """Ladder layers that keep every singular value: EXACT_MPO (default) applies them site by
    site as the parity product operator with exact reduction at the chain ends; EXACT_QR splits
    them by QR in one sweep; EXACT_SVD runs the canonical sweep + Jacobi SVD for every layer."""
    _check(lib().mps_set_exact_layers(mode))


# the library's pair-kernel schedule until set_measure_tuning changes it
DEFAULT_MEASURE_SCHEDULE = (64, 0)


def set_measure_tuning(pair_block_images: int = DEFAULT_MEASURE_SCHEDULE[0],
                       pair_waves_per_cu: int = DEFAULT_MEASURE_SCHEDULE[1]) -> None:
    """Schedule of the 16-wide pair launch: image blocking (0 = the whole batch as one block) and
    a cap on resident workgroups per compute unit (0 = none)."""
    _check(lib().mps_set_measure_tuning(pair_block_images, pair_waves_per_cu))


def set_mixed_tuning(bucket: int, blocks_per_cu: int) -> None:
    _check(lib().mps_set_mixed_tuning(bucket, blocks_per_cu))
