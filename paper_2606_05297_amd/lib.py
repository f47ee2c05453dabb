"""ctypes binding of libfock (argument marshalling only; all work runs in the
HIP library).  Names mirror the C ABI declared in include/fock.h.

Device buffers are torch tensors on the current HIP device (states are
complex64, workspaces uint8); streams are torch's current stream unless given.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfock.so")

TYPES = {"HR": 0, "HI": 1, "DH": 2, "PR": 3, "PI": 4, "KERR": 5, "ROT": 6, "CK": 7, "SR": 8, "SI": 9,
         "BS": 10, "TMS": 11, "SQ": 12}
TYPE_NAMES = {v: k for k, v in TYPES.items()}

FOCK_OK = 0
ERRORS = {-1: "FOCK_ERR_ARG", -2: "FOCK_ERR_SIZE", -3: "FOCK_ERR_UNSUPPORTED", -4: "FOCK_ERR_NONFINITE",
          -5: "FOCK_ERR_HIP", -6: "FOCK_ERR_LINESEARCH", -7: "FOCK_ERR_STATE"}
K_APPLY_H, K_POOL, K_GATE, K_ADJ, K_DIAG, K_REDUCE = range(6)
K_SCORE = 9


class Ham(C.Structure):
    _fields_ = [("L", C.c_int32), ("d", C.c_int32), ("periodic", C.c_int32), ("layout", C.c_int32),
                ("J", C.c_double), ("U", C.c_double), ("mu", C.c_double), ("Delta", C.c_double),
                ("K", C.c_double)]


class Op(C.Structure):
    _fields_ = [("type", C.c_int32), ("i", C.c_int32), ("j", C.c_int32)]


class AdaptOpts(C.Structure):
    _fields_ = [("max_iters", C.c_int32), ("bfgs_maxiter", C.c_int32), ("grad_tol", C.c_double),
                ("tie_tau", C.c_double), ("gtol_floor_rel", C.c_double), ("warm_gtol", C.c_double),
                ("n_warm", C.c_int32), ("grad_mode", C.c_int32), ("warm_ops", C.POINTER(Op)),
                ("warm_theta0", C.POINTER(C.c_double)), ("fd_step", C.c_double),
                ("recycle_hessian", C.c_int32), ("warm_fixed", C.c_int32), ("noise_rel", C.c_double)]


class AdaptReport(C.Structure):
    _fields_ = [("iter", C.c_int32), ("k_sel", C.c_int32), ("converged", C.c_int32), ("status", C.c_int32),
                ("bfgs_iters", C.c_int32), ("bfgs_evals", C.c_int32), ("n_params", C.c_int32),
                ("capped", C.c_int32), ("g_sel", C.c_double), ("g_norm2", C.c_double), ("g_inf", C.c_double),
                ("E", C.c_double), ("norm2", C.c_double), ("E_init", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class SweepPoint(C.Structure):
    _fields_ = [("ham", Ham), ("pool", C.POINTER(Op)), ("P", C.c_int32), ("n_warm", C.c_int32),
                ("warm_ops", C.POINTER(Op)), ("warm_theta0", C.POINTER(C.c_double)), ("psi0", C.c_void_p)]


OBJECTIVE = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double),
                        C.POINTER(C.c_double))

_lib = None


class FockError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def load(path: str = LIB_PATH):
    """Load libfock.so (fails loudly when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libfock.so not found at {path}; build it with `python -m paper_2606_05297_amd.build`")
    L = C.CDLL(path)
    vp, sz, dp, ip = C.c_void_p, C.c_size_t, C.POINTER(C.c_double), C.POINTER(C.c_int)
    L.fock_last_error.restype = C.c_char_p
    L.fock_version.restype = C.c_int
    L.fock_workspace_bytes.argtypes = [C.POINTER(Ham), C.c_int, C.c_int, C.POINTER(C.c_size_t)]
    L.fock_set_stencil_schedule.argtypes = [C.c_int]
    L.fock_set_stencil_variant.argtypes = [C.c_int]
    fp = C.POINTER(C.c_float)
    L.fock_mlp_create.argtypes = [C.c_int, C.POINTER(C.c_void_p)]
    L.fock_mlp_set_params.argtypes = [vp, fp, C.c_int, vp]
    L.fock_mlp_get_params.argtypes = [vp, fp, C.c_int, vp]
    L.fock_mlp_forward.argtypes = [vp, vp, C.c_int, vp, vp]
    L.fock_mlp_loss_grad.argtypes = [vp, vp, vp, vp, C.c_int, dp, fp, vp]
    L.fock_mlp_adam_step.argtypes = [vp, vp, vp, vp, C.c_int, C.c_float, dp, vp]
    L.fock_mlp_destroy.argtypes = [vp]
    L.fock_autotune_stencil.argtypes = [C.POINTER(Ham), vp, vp, vp, sz, vp, C.c_char_p, C.POINTER(C.c_int)]
    L.fock_stencil_schedule_table.argtypes = [C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int), C.c_int]
    L.fock_apply_H.argtypes = [C.POINTER(Ham), vp, vp, dp, dp, vp, sz, vp]
    L.fock_apply_gate2.argtypes = [C.c_int, C.c_int, Op, C.c_double, C.c_int, vp, vp, sz, vp]
    L.fock_pool_grads.argtypes = [C.POINTER(Ham), C.POINTER(Op), C.c_int, vp, vp, dp, vp, sz, vp]
    L.fock_energy_grad_adjoint.argtypes = [C.POINTER(Ham), C.POINTER(Op), dp, C.c_int, vp, vp, vp, dp, dp, dp, vp,
                                           sz, vp]
    L.fock_apply_H_noalloc.argtypes = [C.POINTER(Ham), vp, vp, vp, vp]
    L.fock_stream_probe.argtypes = [C.c_int, vp, vp, sz, C.c_int, C.c_int, dp, vp]
    L.fock_score.argtypes = [C.POINTER(Ham), C.POINTER(Op), C.c_int, vp, vp, dp, dp, dp, vp, sz, vp]
    L.fock_adjoint_sweep.argtypes = [C.POINTER(Ham), C.POINTER(Op), dp, C.c_int, vp, vp, C.c_double, dp, vp, sz, vp]
    L.adapt_default_opts.argtypes = [C.POINTER(AdaptOpts)]
    L.adapt_default_opts.restype = None
    L.adapt_create.argtypes = [C.POINTER(Ham), C.POINTER(Op), C.c_int, vp, C.POINTER(AdaptOpts), vp,
                               C.POINTER(vp)]
    L.adapt_step.argtypes = [vp, C.POINTER(AdaptReport)]
    L.adapt_step_select.argtypes = [vp, C.POINTER(AdaptReport)]
    L.adapt_state_store.argtypes = [vp, ip]
    L.fock_set_state_store.argtypes = [C.c_int]
    L.fock_prepare.argtypes = [C.c_int, C.c_int]
    L.fock_set_sector_layout.argtypes = [C.c_int]
    L.fock_set_real_states.argtypes = [C.c_int]
    L.fock_set_real_fusion.argtypes = [C.c_int]
    L.fock_real_fusion_plan.argtypes = [C.POINTER(Ham), C.POINTER(Op), C.c_int, ip, ip, ip]
    L.adapt_real.argtypes = [vp, ip]
    L.fock_sector_pack.argtypes = [C.c_int, C.c_int, C.c_int, vp, vp, vp]
    L.fock_sector_unpack.argtypes = [C.c_int, C.c_int, C.c_int, vp, vp, vp]
    L.adapt_layout.argtypes = [vp, ip]
    L.adapt_step_finish.argtypes = [vp, C.POINTER(AdaptReport)]
    L.adapt_warm_report.argtypes = [vp, C.POINTER(AdaptReport)]
    L.adapt_get_ansatz.argtypes = [vp, C.POINTER(Op), dp, C.c_int, ip]
    L.adapt_propose.argtypes = [vp, dp, C.c_int]
    L.adapt_last_proposal.argtypes = [vp, ip, dp, dp]
    L.adapt_destroy.argtypes = [vp]
    L.adapt64_create.argtypes = [C.POINTER(Ham), C.POINTER(Op), C.c_int, vp, C.POINTER(AdaptOpts), vp,
                                 C.POINTER(vp)]
    L.adapt64_step.argtypes = [vp, C.POINTER(AdaptReport)]
    L.adapt64_warm_report.argtypes = [vp, C.POINTER(AdaptReport)]
    L.adapt64_get_ansatz.argtypes = [vp, C.POINTER(Op), dp, C.c_int, ip]
    L.adapt64_energy_grad.argtypes = [vp, C.POINTER(Op), dp, C.c_int, dp, dp]
    L.adapt64_destroy.argtypes = [vp]
    L.hva_create.argtypes = [C.POINTER(Ham), C.POINTER(Op), C.c_int, C.c_int, vp, C.POINTER(AdaptOpts), C.c_double,
                             vp, C.POINTER(vp)]
    L.hva_add_layer.argtypes = [vp, dp, C.POINTER(AdaptReport)]
    L.hva_initial_report.argtypes = [vp, C.POINTER(AdaptReport)]
    L.hva_get_ansatz.argtypes = [vp, C.POINTER(Op), dp, C.c_int, ip]
    L.hva_destroy.argtypes = [vp]
    L.fock_sweep_create.argtypes = [C.POINTER(SweepPoint), C.c_int, C.POINTER(AdaptOpts), vp, C.POINTER(vp)]
    L.fock_sweep_step.argtypes = [vp, C.POINTER(AdaptReport), C.POINTER(C.c_int)]
    L.fock_sweep_warm_reports.argtypes = [vp, C.POINTER(AdaptReport)]
    L.fock_sweep_get_ansatz.argtypes = [vp, C.c_int, C.POINTER(Op), dp, C.c_int, ip]
    L.fock_sweep_set_grid.argtypes = [vp, C.c_int]
    L.fock_sweep_destroy.argtypes = [vp]
    L.fock_sweep_autotune.argtypes = [vp, C.c_char_p, ip]
    L.fock_sweep_propose.argtypes = [vp, C.c_int, dp, C.c_int]
    L.fock_sweep_last_proposal.argtypes = [vp, C.c_int, ip, dp, dp]
    L.fock_bfgs_minimize.argtypes = [C.c_int, dp, OBJECTIVE, vp, C.c_double, C.c_int, dp, ip, ip, dp, ip]
    L.fock_prof_enable.argtypes = [C.c_int]
    L.fock_prof_query.argtypes = [C.c_int, C.POINTER(C.c_int64), dp, dp]
    L.fock_prof_reset.argtypes = []
    L.fock_prof_set_sample.argtypes = [C.c_int]
    _lib = L
    return L


def _check(rc):
    if rc != FOCK_OK:
        raise FockError(rc, _lib.fock_last_error().decode())


def last_error() -> str:
    return load().fock_last_error().decode()


# ---------------------------------------------------------------- marshalling helpers

LAYOUT_FULL, LAYOUT_EVEN, LAYOUT_ODD, LAYOUT_REAL = 0, 1, 2, 4


def ham(L, d, periodic=False, J=1.0, U=0.0, mu=0.0, Delta=0.0, K=0.0, layout=LAYOUT_FULL) -> Ham:
    """Hamiltonian record; layout says how the state buffers of a call hold psi
    (LAYOUT_FULL: d^L amplitudes; LAYOUT_EVEN / LAYOUT_ODD: the parity-halved
    layout of a state of that total parity, d^L / 2 amplitudes; plus
    LAYOUT_REAL: float32 amplitudes instead of complex64)."""
    return Ham(int(L), int(d), int(bool(periodic)), int(layout), float(J), float(U), float(mu), float(Delta),
               float(K))


def n_amplitudes(h: Ham) -> int:
    """Amplitudes of one state buffer of a call on h."""
    n = int(h.d) ** int(h.L)
    return n // 2 if (int(h.layout) & 3) != LAYOUT_FULL else n


def ham_from(cfg: dict, layout: int = 0) -> Ham:
    return ham(cfg["L"], cfg["d"], cfg["periodic"], cfg["J"], cfg["U"], cfg["mu"], cfg["Delta"], cfg["K"],
               layout=layout)


def op(t, i, j=-1) -> Op:
    return Op(TYPES[t] if isinstance(t, str) else int(t), int(i), int(j))


def ops_array(ops):
    arr = (Op * max(1, len(ops)))()
    for k, o in enumerate(ops):
        arr[k] = op(*o)
    return arr


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def workspace_bytes(h: Ham, n_pool: int = 0, n_ops: int = 0) -> int:
    L = load()
    b = C.c_size_t(0)
    _check(L.fock_workspace_bytes(C.byref(h), int(n_pool), int(n_ops), C.byref(b)))
    return int(b.value)


def workspace(h: Ham, n_pool: int = 0, n_ops: int = 0, device="cuda"):
    import torch
    return torch.empty(workspace_bytes(h, n_pool, n_ops), dtype=torch.uint8, device=device)


def _state_arg(t, L_, d, name, dtype="c64", layout=LAYOUT_FULL):
    """Reject a state tensor the kernels cannot take: not a contiguous complex64
    (complex128 for the FP64 driver) tensor on the current GPU, or not holding
    exactly d^L amplitudes (d^L / 2 in the parity-halved layouts).  Raised before
    any launch, so a wrong buffer never reaches a kernel that would read or
    write past it."""
    import torch
    want = torch.complex64 if dtype == "c64" else torch.complex128
    if int(layout) & LAYOUT_REAL:
        want = torch.float32
    if not isinstance(t, torch.Tensor):
        raise FockError(-1, f"{name} must be a torch tensor, got {type(t).__name__}")
    if t.dtype != want or not t.is_contiguous():
        raise FockError(-1, f"{name} must be a contiguous {want} tensor (got {t.dtype}, "
                            f"contiguous={t.is_contiguous()})")
    n = int(d) ** int(L_)
    if (int(layout) & 3) != LAYOUT_FULL:
        n //= 2
        if t.numel() != n:
            raise FockError(-2, f"{name} must hold d^L / 2 = {n} amplitudes (parity-halved layout), got {t.numel()}")
    if t.numel() != n:
        raise FockError(-2, f"{name} must hold d^L = {d}^{L_} = {n} amplitudes, got {t.numel()}")
    if not t.is_cuda:
        raise FockError(-1, f"{name} must live on the GPU, got {t.device}")
    if t.device.index != torch.cuda.current_device():
        raise FockError(-1, f"{name} lives on {t.device}, not on the current device cuda:{torch.cuda.current_device()}")


def _ws_arg(ws, name="ws"):
    import torch
    if not isinstance(ws, torch.Tensor) or not ws.is_cuda or ws.dtype != torch.uint8 or not ws.is_contiguous():
        raise FockError(-1, f"{name} must be a contiguous CUDA uint8 tensor")


def _disjoint(a, b, na, nb):
    pa, pb = a.data_ptr(), b.data_ptr()
    ea, eb = pa + a.numel() * a.element_size(), pb + b.numel() * b.element_size()
    if pa < eb and pb < ea:
        raise FockError(-1, f"{na} and {nb} must not overlap")


# ---------------------------------------------------------------- entry points

def apply_H(h: Ham, psi, hpsi, ws, energy=True, stream=None):
    """hpsi = H psi; returns (<psi|H|psi>, <psi|psi>) when energy is True."""
    L = load()
    _state_arg(psi, h.L, h.d, "psi", layout=h.layout)
    _state_arg(hpsi, h.L, h.d, "hpsi", layout=h.layout)
    _disjoint(psi, hpsi, "psi", "hpsi")
    _ws_arg(ws)
    E, n2 = C.c_double(0), C.c_double(0)
    _check(L.fock_apply_H(C.byref(h), _ptr(psi), _ptr(hpsi), C.byref(E) if energy else None,
                          C.byref(n2) if energy else None, _ptr(ws), ws.numel(), _stream(stream)))
    return (E.value, n2.value) if energy else None


def apply_H_noalloc(h: Ham, psi, hpsi, res=None, stream=None):
    """hpsi = H psi through the allocation-free entry point; res (optional): a
    CUDA float64 tensor of 2 entries receiving (<psi|H|psi>, <psi|psi>) on the
    device, without a host synchronisation."""
    L = load()
    _state_arg(psi, h.L, h.d, "psi", layout=h.layout)
    _state_arg(hpsi, h.L, h.d, "hpsi", layout=h.layout)
    _disjoint(psi, hpsi, "psi", "hpsi")
    if res is not None:
        import torch
        if not (isinstance(res, torch.Tensor) and res.is_cuda and res.dtype == torch.float64 and res.numel() >= 2
                and res.is_contiguous()):
            raise FockError(-1, "res must be a contiguous CUDA float64 tensor of at least 2 entries")
    _check(L.fock_apply_H_noalloc(C.byref(h), _ptr(psi), _ptr(hpsi), _ptr(res) if res is not None else None,
                                  _stream(stream)))


STORE_OFF, STORE_ON, STORE_AUTO = 0, 1, 2
SECTOR_OFF, SECTOR_AUTO = 0, 1


def prepare(L_, d):
    """Build the per-device tables of (L, d) and this thread's pinned staging
    ahead of time (fock_prepare), so later calls on them allocate nothing."""
    _check(load().fock_prepare(int(L_), int(d)))


REAL_OFF, REAL_AUTO = 0, 1


def set_real_states(mode: int):
    """Real states in ADAPT drivers created afterwards (fock_set_real_states):
    REAL_OFF or REAL_AUTO (the default)."""
    _check(load().fock_set_real_states(int(mode)))


def get_real_states() -> int:
    return int(load().fock_get_real_states())


RFUSE_OFF, RFUSE_ON = 0, 1


def set_real_fusion(mode: int):
    """Fused runs of real gates (fock_set_real_fusion): RFUSE_ON (the
    default) or RFUSE_OFF (gate by gate)."""
    _check(load().fock_set_real_fusion(int(mode)))


def get_real_fusion() -> int:
    return int(load().fock_get_real_fusion())


def real_fusion_plan(h: Ham, ops):
    """[(first gate, lowest tile mode or -1), ...]: the runs an evaluation of
    ops on real states launches (fock_real_fusion_plan; host only)."""
    n = len(ops)
    k0 = (C.c_int * max(n, 1))()
    a = (C.c_int * max(n, 1))()
    nr = C.c_int(0)
    _check(load().fock_real_fusion_plan(C.byref(h), ops_array(ops), n, k0, a, C.byref(nr)))
    return [(k0[r], a[r]) for r in range(nr.value)]


def set_sector_layout(mode: int):
    """Parity-halved states in ADAPT drivers created afterwards
    (fock_set_sector_layout): SECTOR_OFF or SECTOR_AUTO (the default)."""
    _check(load().fock_set_sector_layout(int(mode)))


def get_sector_layout() -> int:
    return int(load().fock_get_sector_layout())


def _sector_bufs(L_, d, layout, full, half):
    if int(layout) not in (LAYOUT_EVEN, LAYOUT_ODD):
        raise FockError(-1, f"layout must be LAYOUT_EVEN or LAYOUT_ODD, got {layout}")
    _state_arg(full, L_, d, "full")
    _state_arg(half, L_, d, "half", layout=layout)
    _disjoint(full, half, "full", "half")


def sector_pack(L_, d, layout, full, half, stream=None):
    """half = the stored amplitudes of the full state in the parity-halved
    layout (fock_sector_pack)."""
    _sector_bufs(L_, d, layout, full, half)
    _check(load().fock_sector_pack(int(L_), int(d), int(layout), _ptr(full), _ptr(half), _stream(stream)))


def sector_unpack(L_, d, layout, half, full, stream=None):
    """full = the d^L state of a parity-halved one, zero outside its sector
    (fock_sector_unpack)."""
    _sector_bufs(L_, d, layout, full, half)
    _check(load().fock_sector_unpack(int(L_), int(d), int(layout), _ptr(half), _ptr(full), _stream(stream)))



def set_state_store(mode: int):
    """Forward-state store of drivers created afterwards (fock_set_state_store):
    STORE_OFF, STORE_ON or STORE_AUTO (the default)."""
    _check(load().fock_set_state_store(int(mode)))


def get_state_store() -> int:
    return int(load().fock_get_state_store())


def stream_probe(kind, a, b, grid=4096, iters=10, stream=None):
    """Mean duration (ms) of the streaming probe: kind 0 copies a into b, 1
    reads a, 2 updates b in place (fock_stream_probe).  a and b: contiguous
    CUDA tensors of the same byte size (a unused for kind 2)."""
    import torch
    L = load()
    if not (isinstance(b, torch.Tensor) and b.is_cuda and b.is_contiguous()):
        raise FockError(-1, "b must be a contiguous CUDA tensor")
    nbytes = b.numel() * b.element_size()
    if kind != 2 and not (isinstance(a, torch.Tensor) and a.is_cuda and a.is_contiguous()
                          and a.numel() * a.element_size() == nbytes):
        raise FockError(-1, "a must be a contiguous CUDA tensor of b's byte size")
    ms = C.c_double(0.0)
    _check(L.fock_stream_probe(int(kind), _ptr(a) if kind != 2 else None, _ptr(b), nbytes, int(grid), int(iters),
                               C.byref(ms), _stream(stream)))
    return ms.value


def apply_gate2(L_, d, o, theta, psi, ws, adjoint=False, stream=None):
    L = load()
    _state_arg(psi, L_, d, "psi")
    _ws_arg(ws)
    _check(L.fock_apply_gate2(int(L_), int(d), op(*o), float(theta), int(bool(adjoint)), _ptr(psi), _ptr(ws),
                              ws.numel(), _stream(stream)))


def pool_grads(h: Ham, pool, psi, hpsi, ws, stream=None) -> np.ndarray:
    L = load()
    _state_arg(psi, h.L, h.d, "psi", layout=h.layout)
    _state_arg(hpsi, h.L, h.d, "hpsi", layout=h.layout)
    _ws_arg(ws)
    P = len(pool)
    out = np.zeros(P, dtype=np.float64)
    _check(L.fock_pool_grads(C.byref(h), ops_array(pool), P, _ptr(psi), _ptr(hpsi),
                             out.ctypes.data_as(C.POINTER(C.c_double)), _ptr(ws), ws.numel(), _stream(stream)))
    return out


def energy_grad_adjoint(h: Ham, ops, theta, psi0, psi_work, lam_work, ws, grad=True, stream=None):
    """Returns (E, norm2, dE/dtheta or None) for the ansatz ops/theta on psi0."""
    L = load()
    n = len(ops)
    for t, nm in ((psi0, "psi0"), (psi_work, "psi_work"), (lam_work, "lam_work")):
        _state_arg(t, h.L, h.d, nm, layout=h.layout)
    _disjoint(psi0, psi_work, "psi0", "psi_work")
    _disjoint(psi0, lam_work, "psi0", "lam_work")
    _disjoint(psi_work, lam_work, "psi_work", "lam_work")
    _ws_arg(ws)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    if th.shape != (n,):
        raise FockError(-1, f"theta must have shape ({n},), got {th.shape}")
    E, n2 = C.c_double(0), C.c_double(0)
    g = np.zeros(max(n, 1), dtype=np.float64)
    _check(L.fock_energy_grad_adjoint(C.byref(h), ops_array(ops), th.ctypes.data_as(C.POINTER(C.c_double)), n,
                                      _ptr(psi0), _ptr(psi_work), _ptr(lam_work), C.byref(E), C.byref(n2),
                                      g.ctypes.data_as(C.POINTER(C.c_double)) if grad else None, _ptr(ws),
                                      ws.numel(), _stream(stream)))
    return E.value, n2.value, (g[:n].copy() if grad else None)


def score(h: Ham, pool, psi, hpsi, ws, stream=None):
    """hpsi = H psi and the pool gradients in one call (fock_score, fused where
    the pool allows it); returns (grads, <psi|H|psi>, <psi|psi>)."""
    L = load()
    _state_arg(psi, h.L, h.d, "psi", layout=h.layout)
    _state_arg(hpsi, h.L, h.d, "hpsi", layout=h.layout)
    _disjoint(psi, hpsi, "psi", "hpsi")
    _ws_arg(ws)
    P = len(pool)
    out = np.zeros(P, dtype=np.float64)
    E, n2 = C.c_double(0), C.c_double(0)
    _check(L.fock_score(C.byref(h), ops_array(pool), P, _ptr(psi), _ptr(hpsi), C.byref(E), C.byref(n2),
                        out.ctypes.data_as(C.POINTER(C.c_double)), _ptr(ws), ws.numel(), _stream(stream)))
    return out, E.value, n2.value


def adjoint_sweep(h: Ham, ops, theta, psi_work, lam_work, norm2, ws, stream=None) -> np.ndarray:
    """dE/dtheta by the reverse sweep alone, from psi_work = psi_n and
    lam_work = H psi_n left by energy_grad_adjoint(..., grad=False) on the same
    ops/theta (both buffers are overwritten); norm2 is that call's <psi|psi>."""
    L = load()
    n = len(ops)
    _state_arg(psi_work, h.L, h.d, "psi_work", layout=h.layout)
    _state_arg(lam_work, h.L, h.d, "lam_work", layout=h.layout)
    _disjoint(psi_work, lam_work, "psi_work", "lam_work")
    _ws_arg(ws)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    if th.shape != (n,):
        raise FockError(-1, f"theta must have shape ({n},), got {th.shape}")
    g = np.zeros(max(n, 1), dtype=np.float64)
    _check(L.fock_adjoint_sweep(C.byref(h), ops_array(ops), th.ctypes.data_as(C.POINTER(C.c_double)), n,
                                _ptr(psi_work), _ptr(lam_work), float(norm2), g.ctypes.data_as(C.POINTER(C.c_double)),
                                _ptr(ws), ws.numel(), _stream(stream)))
    return g[:n].copy()


def bfgs_minimize(fun, x0, gtol=1e-8, maxiter=1000, hinv=None):
    """fun(x) -> (f, g) on the host; returns dict(x, f, iters, evals, status, hinv)."""
    L = load()
    n = len(x0)
    x = np.ascontiguousarray(x0, dtype=np.float64).copy()

    def cb(ctx, n_, xp, fp, gp):
        try:
            xv = np.ctypeslib.as_array(xp, shape=(n_,)).copy()
            f, g = fun(xv)
            fp[0] = float(f)
            gv = np.ctypeslib.as_array(gp, shape=(n_,))
            gv[:] = g
            return 0
        except Exception:  # abort the minimisation; reported as FOCK_ERR_ARG
            return -1

    cfun = OBJECTIVE(cb)
    H = np.zeros(n * n) if hinv is None else np.ascontiguousarray(hinv, dtype=np.float64).reshape(-1).copy()
    it, ev, st = C.c_int(0), C.c_int(0), C.c_int(0)
    fmin = C.c_double(0)
    dp = C.POINTER(C.c_double)
    _check(L.fock_bfgs_minimize(n, x.ctypes.data_as(dp), cfun, None, float(gtol), int(maxiter), H.ctypes.data_as(dp),
                                C.byref(it), C.byref(ev), C.byref(fmin), C.byref(st)))
    return dict(x=x, f=fmin.value, iters=it.value, evals=ev.value, status=st.value, hinv=H.reshape(n, n))


class Adapt:
    """One CV-ADAPT-VQE run on the device (adapt_create / adapt_step)."""

    def __init__(self, h: Ham, pool, psi0, max_iters=60, grad_tol=1e-3, warm_ops=(), warm_theta0=(),
                 grad_mode=0, fd_step=1e-3, recycle_hessian=False, bfgs_maxiter=1000, tie_tau=1e-4,
                 gtol_floor_rel=1e-5, warm_gtol=1e-6, noise_rel=1e-7, stream=None):
        L = load()
        self._L = L
        _state_arg(psi0, h.L, h.d, "psi0")
        o = AdaptOpts()
        L.adapt_default_opts(C.byref(o))
        o.max_iters = int(max_iters)
        o.grad_tol = float(grad_tol)
        o.grad_mode = int(grad_mode)
        o.fd_step = float(fd_step)
        o.recycle_hessian = int(bool(recycle_hessian))
        o.bfgs_maxiter = int(bfgs_maxiter)
        o.tie_tau = float(tie_tau)
        o.gtol_floor_rel = float(gtol_floor_rel)
        o.warm_gtol = float(warm_gtol)
        o.noise_rel = float(noise_rel)
        self._warm = ops_array(list(warm_ops))
        self._warm_th = np.ascontiguousarray(warm_theta0, dtype=np.float64)
        if len(self._warm_th) != len(warm_ops):
            raise ValueError("warm_theta0 needs one angle per warm-up op")
        o.n_warm = len(warm_ops)
        if len(warm_ops):
            o.warm_ops = C.cast(self._warm, C.POINTER(Op))
            o.warm_theta0 = self._warm_th.ctypes.data_as(C.POINTER(C.c_double))
        self.pool = list(pool)
        self._pool = ops_array(self.pool)
        self.h = h
        self._st = C.c_void_p()
        _check(L.adapt_create(C.byref(h), self._pool, len(self.pool), _ptr(psi0), C.byref(o), _stream(stream),
                              C.byref(self._st)))

    def warm_report(self) -> dict:
        r = AdaptReport()
        _check(self._L.adapt_warm_report(self._st, C.byref(r)))
        return r.as_dict()

    def step(self) -> dict:
        r = AdaptReport()
        _check(self._L.adapt_step(self._st, C.byref(r)))
        return r.as_dict()

    def select(self) -> dict:
        """First half of a step: score, test, select and append (adapt_step_select)."""
        r = AdaptReport()
        _check(self._L.adapt_step_select(self._st, C.byref(r)))
        return r.as_dict()

    def finish(self) -> dict:
        """Second half: BFGS from the plain start or a pending proposal (adapt_step_finish)."""
        r = AdaptReport()
        _check(self._L.adapt_step_finish(self._st, C.byref(r)))
        return r.as_dict()

    def real(self) -> bool:
        """Whether the run keeps float32 states for evaluations whose gates are all HR or PR."""
        n = C.c_int(0)
        _check(self._L.adapt_real(self._st, C.byref(n)))
        return bool(n.value)

    def layout(self) -> int:
        """Layout the run keeps its states in (LAYOUT_FULL, LAYOUT_EVEN or LAYOUT_ODD)."""
        n = C.c_int(0)
        _check(self._L.adapt_layout(self._st, C.byref(n)))
        return n.value

    def state_store(self) -> int:
        """Forward states this run keeps for its gradient evaluations (0: none)."""
        n = C.c_int(0)
        _check(self._L.adapt_state_store(self._st, C.byref(n)))
        return n.value

    def ansatz(self):
        n = C.c_int(0)
        _check(self._L.adapt_get_ansatz(self._st, None, None, 0, C.byref(n)))
        m = n.value
        ops = (Op * max(1, m))()
        th = np.zeros(max(1, m))
        _check(self._L.adapt_get_ansatz(self._st, ops, th.ctypes.data_as(C.POINTER(C.c_double)), m, C.byref(n)))
        return [(TYPE_NAMES[ops[k].type], ops[k].i, ops[k].j) for k in range(m)], th[:m].copy()

    def propose(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        _check(self._L.adapt_propose(self._st, th.ctypes.data_as(C.POINTER(C.c_double)), len(th)))

    def last_proposal(self):
        a, ep, el = C.c_int(0), C.c_double(0), C.c_double(0)
        _check(self._L.adapt_last_proposal(self._st, C.byref(a), C.byref(ep), C.byref(el)))
        return dict(accepted=bool(a.value), E_prop=ep.value, E_plain=el.value)

    def close(self):
        if self._st:
            self._L.adapt_destroy(self._st)
            self._st = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Adapt64:
    """CV-ADAPT-VQE on complex128 states (adapt64_create / adapt64_step): psi0
    is a device complex128 tensor; optional warm-up layer of one-parameter ops
    (optimised, or with warm_fixed kept at warm_theta0), adjoint gradients, no
    noise-floor stop.  The BFGS tolerance floor defaults
    to 1e-11 |E| (FP64 gradients), not the complex64 path's 1e-5 |E|."""

    def __init__(self, h: Ham, pool, psi0, max_iters=60, grad_tol=1e-3, recycle_hessian=False, bfgs_maxiter=1000,
                 tie_tau=1e-4, gtol_floor_rel=1e-11, warm_ops=(), warm_theta0=(), warm_gtol=1e-6, warm_fixed=False,
                 stream=None):
        L = load()
        self._L = L
        _state_arg(psi0, h.L, h.d, "psi0", dtype="c128")
        o = AdaptOpts()
        L.adapt_default_opts(C.byref(o))
        o.max_iters = int(max_iters)
        o.grad_tol = float(grad_tol)
        o.recycle_hessian = int(bool(recycle_hessian))
        o.bfgs_maxiter = int(bfgs_maxiter)
        o.tie_tau = float(tie_tau)
        o.gtol_floor_rel = float(gtol_floor_rel)
        o.warm_gtol = float(warm_gtol)
        o.warm_fixed = int(bool(warm_fixed))
        self._warm = ops_array(list(warm_ops))
        self._warm_th = np.ascontiguousarray(warm_theta0, dtype=np.float64)
        if len(self._warm_th) != len(warm_ops):
            raise ValueError("warm_theta0 needs one angle per warm-up op")
        o.n_warm = len(warm_ops)
        if len(warm_ops):
            o.warm_ops = C.cast(self._warm, C.POINTER(Op))
            o.warm_theta0 = self._warm_th.ctypes.data_as(C.POINTER(C.c_double))
        self.pool = list(pool)
        self._pool = ops_array(self.pool)
        self.h = h
        self._st = C.c_void_p()
        _check(L.adapt64_create(C.byref(h), self._pool, len(self.pool), _ptr(psi0), C.byref(o), _stream(stream),
                                C.byref(self._st)))

    def warm_report(self) -> dict:
        r = AdaptReport()
        _check(self._L.adapt64_warm_report(self._st, C.byref(r)))
        return r.as_dict()

    def step(self) -> dict:
        r = AdaptReport()
        _check(self._L.adapt64_step(self._st, C.byref(r)))
        return r.as_dict()

    def ansatz(self):
        n = C.c_int(0)
        _check(self._L.adapt64_get_ansatz(self._st, None, None, 0, C.byref(n)))
        m = n.value
        ops = (Op * max(1, m))()
        th = np.zeros(max(1, m))
        _check(self._L.adapt64_get_ansatz(self._st, ops, th.ctypes.data_as(C.POINTER(C.c_double)), m, C.byref(n)))
        return [(TYPE_NAMES[ops[k].type], ops[k].i, ops[k].j) for k in range(m)], th[:m].copy()

    def energy_grad(self, ops, theta, grad=True):
        """(E, dE/dtheta or None) of an ansatz on this run's psi0, in FP64."""
        n = len(ops)
        th = np.ascontiguousarray(theta, dtype=np.float64)
        E = C.c_double(0)
        g = np.zeros(max(n, 1))
        _check(self._L.adapt64_energy_grad(self._st, ops_array(list(ops)), th.ctypes.data_as(C.POINTER(C.c_double)), n,
                                           C.byref(E), g.ctypes.data_as(C.POINTER(C.c_double)) if grad else None))
        return E.value, (g[:n].copy() if grad else None)

    def close(self):
        if self._st:
            self._L.adapt64_destroy(self._st)
            self._st = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Hva:
    """HVA-CV-VQE on the device (hva_create / hva_add_layer): the layer of
    gates `layer` repeated up to max_layers times, grown one layer at a time."""

    def __init__(self, h: Ham, layer, psi0, max_layers, gtol=1e-9, bfgs_maxiter=1000, gtol_floor_rel=1e-5,
                 noise_rel=1e-7, stream=None):
        L = load()
        self._L = L
        _state_arg(psi0, h.L, h.d, "psi0")
        o = AdaptOpts()
        L.adapt_default_opts(C.byref(o))
        o.bfgs_maxiter, o.gtol_floor_rel, o.noise_rel = int(bfgs_maxiter), float(gtol_floor_rel), float(noise_rel)
        self.layer = list(layer)
        self._layer = ops_array(self.layer)
        self._st = C.c_void_p()
        _check(L.hva_create(C.byref(h), self._layer, len(self.layer), int(max_layers), _ptr(psi0), C.byref(o),
                            float(gtol), _stream(stream), C.byref(self._st)))

    def initial_report(self) -> dict:
        r = AdaptReport()
        _check(self._L.hva_initial_report(self._st, C.byref(r)))
        return r.as_dict()

    def add_layer(self, theta_new) -> dict:
        th = np.ascontiguousarray(theta_new, dtype=np.float64)
        if th.shape != (len(self.layer),):
            raise FockError(-1, f"theta_new must have shape ({len(self.layer)},), got {th.shape}")
        r = AdaptReport()
        _check(self._L.hva_add_layer(self._st, th.ctypes.data_as(C.POINTER(C.c_double)), C.byref(r)))
        return r.as_dict()

    def ansatz(self):
        n = C.c_int(0)
        _check(self._L.hva_get_ansatz(self._st, None, None, 0, C.byref(n)))
        m = n.value
        ops = (Op * max(1, m))()
        th = np.zeros(max(1, m))
        _check(self._L.hva_get_ansatz(self._st, ops, th.ctypes.data_as(C.POINTER(C.c_double)), m, C.byref(n)))
        return [(TYPE_NAMES[ops[k].type], ops[k].i, ops[k].j) for k in range(m)], th[:m].copy()

    def close(self):
        if self._st:
            self._L.hva_destroy(self._st)
            self._st = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _opts(max_iters=60, grad_tol=1e-3, bfgs_maxiter=1000, tie_tau=1e-4, gtol_floor_rel=1e-5, warm_gtol=1e-6,
          noise_rel=1e-7, grad_mode=0, fd_step=1e-3, recycle_hessian=False):
    o = AdaptOpts()
    load().adapt_default_opts(C.byref(o))
    o.max_iters, o.grad_tol, o.bfgs_maxiter, o.tie_tau = int(max_iters), float(grad_tol), int(bfgs_maxiter), float(tie_tau)
    o.gtol_floor_rel, o.warm_gtol, o.noise_rel = float(gtol_floor_rel), float(warm_gtol), float(noise_rel)
    o.grad_mode, o.fd_step, o.recycle_hessian = int(grad_mode), float(fd_step), int(bool(recycle_hessian))
    return o


class Sweep:
    """CV-ADAPT-VQE on many points in lockstep (fock_sweep_*).

    points: list of dicts with keys ham (Ham), pool (list of ops), psi0 (device
    complex64 tensor), and optionally warm_ops / warm_theta0."""

    def __init__(self, points, stream=None, **opts):
        L = load()
        self._L = L
        self.n = len(points)
        self._keep = []
        arr = (SweepPoint * self.n)()
        for k, p in enumerate(points):
            _state_arg(p["psi0"], p["ham"].L, p["ham"].d, f"points[{k}].psi0")
            pool = ops_array(p["pool"])
            wo = p.get("warm_ops", ())
            wops = ops_array(list(wo))
            wth = np.ascontiguousarray(p.get("warm_theta0", ()), dtype=np.float64)
            self._keep += [pool, wops, wth, p["psi0"]]
            arr[k].ham = p["ham"]
            arr[k].pool = C.cast(pool, C.POINTER(Op))
            arr[k].P = len(p["pool"])
            arr[k].n_warm = len(wo)
            arr[k].warm_ops = C.cast(wops, C.POINTER(Op))
            arr[k].warm_theta0 = wth.ctypes.data_as(C.POINTER(C.c_double)) if len(wo) else None
            arr[k].psi0 = C.c_void_p(p["psi0"].data_ptr())
        o = _opts(**opts)
        self._st = C.c_void_p()
        _check(L.fock_sweep_create(arr, self.n, C.byref(o), _stream(stream), C.byref(self._st)))

    def step(self):
        reps = (AdaptReport * self.n)()
        na = C.c_int(0)
        _check(self._L.fock_sweep_step(self._st, reps, C.byref(na)))
        return [reps[k].as_dict() for k in range(self.n)], na.value

    def warm_reports(self):
        reps = (AdaptReport * self.n)()
        _check(self._L.fock_sweep_warm_reports(self._st, reps))
        return [reps[k].as_dict() for k in range(self.n)]

    def ansatz(self, point):
        n = C.c_int(0)
        _check(self._L.fock_sweep_get_ansatz(self._st, int(point), None, None, 0, C.byref(n)))
        m = n.value
        ops = (Op * max(1, m))()
        th = np.zeros(max(1, m))
        _check(self._L.fock_sweep_get_ansatz(self._st, int(point), ops, th.ctypes.data_as(C.POINTER(C.c_double)), m,
                                             C.byref(n)))
        return [(TYPE_NAMES[ops[k].type], ops[k].i, ops[k].j) for k in range(m)], th[:m].copy()

    def set_grid(self, grid):
        _check(self._L.fock_sweep_set_grid(self._st, int(grid)))

    def propose(self, point, theta):
        t = np.ascontiguousarray(theta, dtype=np.float64)
        _check(self._L.fock_sweep_propose(self._st, int(point), t.ctypes.data_as(C.POINTER(C.c_double)), len(t)))

    def last_proposal(self, point):
        acc, ep, e0 = C.c_int(0), C.c_double(0), C.c_double(0)
        _check(self._L.fock_sweep_last_proposal(self._st, int(point), C.byref(acc), C.byref(ep), C.byref(e0)))
        return {"accepted": bool(acc.value), "E_prop": ep.value, "E_plain": e0.value}

    def autotune(self, cache_path=None):
        g = C.c_int(0)
        _check(self._L.fock_sweep_autotune(self._st, cache_path.encode() if cache_path else None, C.byref(g)))
        return g.value

    def close(self):
        if self._st:
            self._L.fock_sweep_destroy(self._st)
            self._st = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- warm-start network

MLP_NPARAMS = 25408


def _mlp_arg(t, cols, dtype, name):
    import torch
    want = torch.float32 if dtype == "f32" else torch.int32
    if not (t.is_cuda and t.dtype == want and t.is_contiguous()):
        raise FockError(-1, f"{name} must be a contiguous CUDA {want} tensor")
    if cols is not None and (t.dim() != 2 or t.shape[1] != cols):
        raise FockError(-1, f"{name} must have shape [B, {cols}], got {tuple(t.shape)}")
    if cols is None and t.dim() != 1:
        raise FockError(-1, f"{name} must be one-dimensional")


class Mlp:
    """Warm-start network 4 -> 128 -> 128 -> 64 (fock_mlp_*).  X, T, Y are
    float32 CUDA tensors, nvalid an int32 CUDA tensor; parameters and
    gradients are numpy float32 arrays."""

    def __init__(self, max_batch, params=None, stream=None):
        self._L = load()
        self._st = C.c_void_p()
        self.max_batch = int(max_batch)
        self._s = stream
        _check(self._L.fock_mlp_create(self.max_batch, C.byref(self._st)))
        if params is not None:
            self.set_params(params)

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        _check(self._L.fock_mlp_set_params(self._st, p.ctypes.data_as(C.POINTER(C.c_float)), len(p),
                                           _stream(self._s)))

    def params(self):
        p = np.zeros(MLP_NPARAMS, dtype=np.float32)
        _check(self._L.fock_mlp_get_params(self._st, p.ctypes.data_as(C.POINTER(C.c_float)), len(p),
                                           _stream(self._s)))
        return p

    def _batch(self, X, T=None, nvalid=None):
        _mlp_arg(X, 4, "f32", "X")
        B = X.shape[0]
        if T is not None:
            _mlp_arg(T, 64, "f32", "T")
            _mlp_arg(nvalid, None, "i32", "nvalid")
            if T.shape[0] != B or nvalid.shape[0] != B:
                raise FockError(-1, "X, T and nvalid must have the same number of rows")
        return B

    def forward(self, X, Y=None):
        import torch
        self._batch(X)
        if Y is None:
            Y = torch.empty((X.shape[0], 64), dtype=torch.float32, device=X.device)
        _mlp_arg(Y, 64, "f32", "Y")
        if Y.shape[0] != X.shape[0]:
            raise FockError(-1, "Y must have as many rows as X")
        _check(self._L.fock_mlp_forward(self._st, _ptr(X), int(X.shape[0]), _ptr(Y), _stream(self._s)))
        return Y

    def loss_grad(self, X, T, nvalid, grad=True):
        self._batch(X, T, nvalid)
        loss = C.c_double(0)
        g = np.zeros(MLP_NPARAMS, dtype=np.float32) if grad else None
        _check(self._L.fock_mlp_loss_grad(self._st, _ptr(X), _ptr(T), _ptr(nvalid), int(X.shape[0]), C.byref(loss),
                                          g.ctypes.data_as(C.POINTER(C.c_float)) if grad else None,
                                          _stream(self._s)))
        return loss.value, g

    def adam_step(self, X, T, nvalid, lr, want_loss=False):
        self._batch(X, T, nvalid)
        loss = C.c_double(0)
        _check(self._L.fock_mlp_adam_step(self._st, _ptr(X), _ptr(T), _ptr(nvalid), int(X.shape[0]), float(lr),
                                          C.byref(loss) if want_loss else None, _stream(self._s)))
        return loss.value if want_loss else None

    def close(self):
        if self._st:
            self._L.fock_mlp_destroy(self._st)
            self._st = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- stencil schedules

def set_stencil_schedule(scheme: int):
    _check(load().fock_set_stencil_schedule(int(scheme)))


def autotune_stencil(h: Ham, psi, hpsi, ws, cache_path=None, stream=None) -> int:
    """Time fock_apply_H under every tile schedule, keep the fastest."""
    L = load()
    best = C.c_int(0)
    _check(L.fock_autotune_stencil(C.byref(h), _ptr(psi), _ptr(hpsi), _ptr(ws), ws.numel(), _stream(stream),
                                   cache_path.encode() if cache_path else None, C.byref(best)))
    return best.value


GATE_BLOCK, GATE_DENSE_MFMA = 0, 1


def set_gate_variant(variant: int):
    """0: block-sparse gate kernels (default); 1: dense d^2 x d^2 gates on FP32 matrix cores (d in {4, 6, 8})."""
    _check(load().fock_set_gate_variant(int(variant)))


def get_gate_variant() -> int:
    return int(load().fock_get_gate_variant())


FUSE_OFF, FUSE_FORWARD, FUSE_ALL = 0, 1, 2


def set_gate_fusion(mode: int):
    """0: per-gate passes (default); 1: fused forward circuit; 2: fused forward and adjoint sweep."""
    _check(load().fock_set_gate_fusion(int(mode)))


def get_gate_fusion() -> int:
    return int(load().fock_get_gate_fusion())


def get_stencil_schedule() -> int:
    return int(load().fock_get_stencil_schedule())


STENCIL_ROWS, STENCIL_LANES, STENCIL_SLAB = 0, 1, 2


def set_stencil_variant(variant: int):
    """Work split of the H psi kernel: 0 = one thread per row, 1 = four lanes per
    row (d = 8, 4 <= L <= 10, open chains), 2 = two-pass slab stencil (the
    default; L = 8, d = 8); elsewhere the row split runs."""
    _check(load().fock_set_stencil_variant(int(variant)))


def get_stencil_variant() -> int:
    return int(load().fock_get_stencil_variant())


def stencil_schedule_table(L: int, d: int, scheme: int, n: int):
    out = np.zeros(n, dtype=np.int32)
    _check(load().fock_stencil_schedule_table(int(L), int(d), int(scheme),
                                              out.ctypes.data_as(C.POINTER(C.c_int)), int(n)))
    return out


# ---------------------------------------------------------------- profiling

def prof_enable(on=True):
    _check(load().fock_prof_enable(int(bool(on))))


def prof_reset():
    _check(load().fock_prof_reset())


def prof_set_sample(every: int):
    """Time one launch in `every` per kernel id (1: every launch)."""
    _check(load().fock_prof_set_sample(int(every)))


def prof_query(kid: int) -> dict:
    n = C.c_int64(0)
    ms, b = C.c_double(0), C.c_double(0)
    _check(load().fock_prof_query(int(kid), C.byref(n), C.byref(ms), C.byref(b)))
    return dict(launches=n.value, ms=ms.value, bytes=b.value)
