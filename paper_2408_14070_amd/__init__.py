"""Reinforced-Dynamics neural-bias hot path on MI355X (gfx950).

Thin Python binding of the C ABI in include/rid.h: argument marshalling
only.  Every step of the path runs in the HIP kernels of librid.so; tensors
are torch CUDA (ROCm) tensors used for device memory and streams.  There is
no CPU fallback: importing works without a GPU (the library loads and its
symbols resolve), but every compute call needs the device.

Paper: "RiD-kit: Software package designed to do enhanced sampling using
reinforced dynamics" (arXiv 2408.14070).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librid.so")

RID_OK, RID_EINVAL, RID_ENOMEM, RID_EDEVICE, RID_EDEGENERATE, RID_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
RID_FP32, RID_BF16, RID_FP16, RID_BF16_ALL = 0, 1, 2, 3
_STATUS = {0: "RID_OK", -1: "RID_EINVAL", -2: "RID_ENOMEM", -3: "RID_EDEVICE",
           -4: "RID_EDEGENERATE", -5: "RID_EUNSUPPORTED"}

# Every symbol include/rid.h declares.
EXPORTS = (
    "rid_last_error", "rid_version", "rid_system_create", "rid_system_destroy",
    "rid_packed_param_count", "rid_ensemble_create", "rid_ensemble_get_params",
    "rid_ensemble_set_params", "rid_ensemble_load_params", "rid_ensemble_step", "rid_ensemble_set_dropout",
    "rid_ensemble_set_resnet", "rid_ensemble_set_angular_mask", "rid_ensemble_set_cv_bounds",
    "rid_ensemble_set_train_budget",
    "rid_ensemble_destroy",
    "rid_cv_eval", "rid_model_dev", "rid_cluster_frames", "rid_select",
    "rid_ensemble_set_cv_weights", "rid_adjust_trust_levels", "rid_bias_force",
    "rid_bias_force_conservative", "rid_bias_force_noalloc", "rid_noalloc_scratch_floats",
    "rid_mcmc_run",
    "rid_cv_apply_force",
    "rid_mf_train_step", "rid_lr_exponential", "rid_mf_label",
    "rid_profile_enable", "rid_profile_read", "rid_mf_loss_grad", "rid_mf_grad",
    "rid_server_create", "rid_server_register", "rid_server_submit", "rid_server_submit_device",
    "rid_server_wait", "rid_server_replay",
    "rid_server_stats", "rid_server_reset_stats", "rid_server_destroy",
)
RID_SERVE_FIFO = 1


class ServerStats(ctypes.Structure):
    _fields_ = [("requests_done", ctypes.c_int64), ("walkers_done", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("admission_waits", ctypes.c_int64),
                ("max_inflight_batches", ctypes.c_int64),
                ("mean_batch_walkers", ctypes.c_double), ("p50_us", ctypes.c_double),
                ("p99_us", ctypes.c_double), ("mean_us", ctypes.c_double),
                ("max_us", ctypes.c_double), ("walker_steps_per_s", ctypes.c_double)]
class ReplayRequest(ctypes.Structure):
    _fields_ = [("model_id", ctypes.c_int), ("n_walkers", ctypes.c_int),
                ("arrival_s", ctypes.c_double), ("pos", ctypes.c_void_p),
                ("device", ctypes.c_int), ("force", ctypes.c_void_p),
                ("energy", ctypes.c_void_p), ("eps", ctypes.c_void_p),
                ("sigma", ctypes.c_void_p)]


PROF_CV, PROF_MLP, PROF_SCATTER, PROF_REDUCE, PROF_EMBED, PROF_TRAIN, PROF_LABEL, PROF_HVP = range(8)


class RidError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load librid.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} missing: build it first "
                          "(python -m paper_2408_14070_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i, f, d, sz, i64 = (ctypes.c_void_p, ctypes.c_int, ctypes.c_float,
                           ctypes.c_double, ctypes.c_size_t, ctypes.c_int64)
    P = ctypes.POINTER
    sig = {
        "rid_last_error": (ctypes.c_char_p, []),
        "rid_version": (ctypes.c_char_p, []),
        "rid_system_create": (i, [i, i, vp, vp, P(vp)]),
        "rid_system_destroy": (None, [vp]),
        "rid_packed_param_count": (sz, [i, i, i, vp]),
        "rid_ensemble_create": (i, [i, i, i, vp, i, vp, P(vp)]),
        "rid_ensemble_get_params": (i, [vp, vp]),
        "rid_ensemble_set_params": (i, [vp, vp]),
        "rid_ensemble_load_params": (i, [vp, vp, vp]),
        "rid_ensemble_step": (i64, [vp]),
        "rid_ensemble_set_dropout": (i, [vp, f, ctypes.c_uint64]),
        "rid_ensemble_set_resnet": (i, [vp, i]),
        "rid_ensemble_set_angular_mask": (i, [vp, vp]),
        "rid_ensemble_set_cv_bounds": (i, [vp, vp, vp]),
        "rid_ensemble_set_train_budget": (i, [vp, ctypes.c_size_t]),
        "rid_ensemble_destroy": (None, [vp]),
        "rid_cv_eval": (i, [vp, vp, i, vp, vp, vp]),
        "rid_model_dev": (i, [vp, vp, i, vp, vp, vp, vp, vp]),
        "rid_cluster_frames": (i, [vp, i, i, vp, f, f, i, i, i, i, vp, vp, P(i), P(f), vp]),
        "rid_select": (i, [vp, vp, i, f, f, i, i, i, i, vp, vp, vp, P(i), P(i), P(f), vp]),
        "rid_ensemble_set_cv_weights": (i, [vp, vp]),
        "rid_adjust_trust_levels": (i, [i, i, f, P(f), P(f)]),
        "rid_bias_force": (i, [vp, vp, vp, i, f, f, vp, vp, vp, vp, vp, vp]),
        "rid_bias_force_conservative": (i, [vp, vp, vp, i, f, f, vp, vp, vp, vp, vp, vp]),
        "rid_bias_force_noalloc": (i, [vp, vp, vp, i, f, f, vp, vp, vp, vp, vp, vp]),
        "rid_noalloc_scratch_floats": (sz, []),
        "rid_mcmc_run": (i, [vp, vp, i, i64, i64, ctypes.c_double, f, ctypes.c_uint64, i, i, i,
                             vp, vp, vp, vp]),
        "rid_cv_apply_force": (i, [vp, vp, vp, i, vp, vp]),
        "rid_mf_train_step": (i, [vp, vp, vp, i, f, vp, vp]),
        "rid_lr_exponential": (d, [i64, d, i, d]),
        "rid_mf_label": (i, [vp, vp, vp, vp, i, i, i, f, vp, vp, vp, vp]),
        "rid_profile_enable": (None, [i]),
        "rid_profile_read": (i, [i, P(d), P(i64)]),
        "rid_mf_loss_grad": (i, [vp, vp, vp, i, vp, vp, vp]),
        "rid_mf_grad": (i, [vp, vp, vp, i, vp, vp]),
        "rid_server_create": (i, [sz, i, i, i, P(vp)]),
        "rid_server_register": (i, [vp, vp, vp, f, f, P(i)]),
        "rid_server_submit": (i, [vp, i, vp, i, P(i64)]),
        "rid_server_submit_device": (i, [vp, i, vp, i, vp, vp, vp, vp, P(i64)]),
        "rid_server_replay": (i, [vp, P(ReplayRequest), i, vp, vp, P(d)]),
        "rid_server_wait": (i, [vp, i64, vp, vp, vp, vp, P(d)]),
        "rid_server_stats": (i, [vp, P(ServerStats)]),
        "rid_server_reset_stats": (None, [vp]),
        "rid_server_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(status):
    if status != RID_OK:
        msg = lib().rid_last_error()
        raise RidError(status, msg.decode() if msg else "")


def _torch():
    import torch
    return torch


def _ptr(t):
    """Device pointer of a contiguous CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device (CUDA/ROCm) tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _f32(t, shape, name):
    if t.dtype != _torch().float32:
        raise TypeError(f"{name} must be float32")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


class System:
    """Atoms and CVs (rid_system_create): torsion rows (a, b, c, d) and,
    where angular_mask is 0, distance rows (a, b, -1, -1)."""

    def __init__(self, n_atoms: int, quads, angular_mask=None):
        q = np.ascontiguousarray(np.asarray(quads, dtype=np.int32))
        if q.ndim != 2 or q.shape[1] != 4:
            raise ValueError("quads must be [n_cv][4]")
        m = None
        if angular_mask is not None:
            m = np.ascontiguousarray(np.asarray(angular_mask, dtype=np.uint8))
        h = ctypes.c_void_p()
        _check(lib().rid_system_create(int(n_atoms), int(q.shape[0]),
                                       q.ctypes.data_as(ctypes.c_void_p),
                                       None if m is None else m.ctypes.data_as(ctypes.c_void_p),
                                       ctypes.byref(h)))
        self.handle = h
        self.n_atoms = int(n_atoms)
        self.n_cv = int(q.shape[0])

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.rid_system_destroy(self.handle)
        self.handle = None

    __del__ = close


class Ensemble:
    """Ensemble of MLP free-energy models (rid_ensemble_create)."""

    def __init__(self, n_cv: int, widths, n_models: int, params, precision=RID_FP32):
        w = np.ascontiguousarray(np.asarray(widths, dtype=np.int32))
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        need = lib().rid_packed_param_count(int(n_cv), int(n_models), int(w.size),
                                            w.ctypes.data_as(ctypes.c_void_p))
        if p.size != need:
            raise ValueError(f"params has {p.size} values, expected {need}")
        h = ctypes.c_void_p()
        _check(lib().rid_ensemble_create(int(n_cv), int(n_models), int(w.size),
                                         w.ctypes.data_as(ctypes.c_void_p), int(precision),
                                         p.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h)))
        self.handle = h
        self.n_cv, self.K, self.widths = int(n_cv), int(n_models), [int(v) for v in w]
        self.precision = int(precision)
        self.n_params = int(need)
        self.dropout_rate = 0.0

    def get_params(self) -> np.ndarray:
        out = np.empty(self.n_params, dtype=np.float32)
        _check(lib().rid_ensemble_get_params(self.handle, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def set_params(self, params):
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        if p.size != self.n_params:
            raise ValueError("wrong parameter count")
        _check(lib().rid_ensemble_set_params(self.handle, p.ctypes.data_as(ctypes.c_void_p)))

    @property
    def step(self) -> int:
        return int(lib().rid_ensemble_step(self.handle))

    def set_dropout(self, rate: float, seed: int = 0):
        """rid_ensemble_set_dropout: training-time dropout rate and mask seed."""
        _check(lib().rid_ensemble_set_dropout(self.handle, float(rate), int(seed)))
        self.dropout_rate = float(rate)

    def set_resnet(self, enable: bool = True):
        """rid_ensemble_set_resnet: residual connections between the hidden
        layers after the first (hidden widths must be equal; FP32 only)."""
        _check(lib().rid_ensemble_set_resnet(self.handle, 1 if enable else 0))

    def set_angular_mask(self, angular_mask=None):
        """rid_ensemble_set_angular_mask: CVs whose entry is 0 enter the
        networks raw, as (s, 0); None makes every CV angular again."""
        if angular_mask is None:
            _check(lib().rid_ensemble_set_angular_mask(self.handle, None))
            return
        m = np.ascontiguousarray(np.asarray(angular_mask, dtype=np.uint8))
        if m.shape != (self.n_cv,):
            raise ValueError("angular_mask must be [n_cv]")
        _check(lib().rid_ensemble_set_angular_mask(self.handle, m.ctypes.data_as(ctypes.c_void_p)))

    def set_cv_weights(self, weights=None):
        """rid_ensemble_set_cv_weights: per-CV weights of the selection
        phase's clustering distance; None makes every weight 1 again."""
        if weights is None:
            _check(lib().rid_ensemble_set_cv_weights(self.handle, None))
            return
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.float32))
        if w.shape != (self.n_cv,):
            raise ValueError("weights must be [n_cv]")
        _check(lib().rid_ensemble_set_cv_weights(self.handle, w.ctypes.data_as(ctypes.c_void_p)))

    def set_train_budget(self, nbytes: int = 0):
        """rid_ensemble_set_train_budget: device bytes of stored activations
        one training pass may hold (0: the default); larger batches run in
        chunks of rows."""
        _check(lib().rid_ensemble_set_train_budget(self.handle, int(nbytes)))

    def set_cv_bounds(self, lower=None, upper=None):
        """rid_ensemble_set_cv_bounds: the MCMC box of the raw CVs (host
        arrays [n_cv]); None clears."""
        if lower is None and upper is None:
            _check(lib().rid_ensemble_set_cv_bounds(self.handle, None, None))
            return
        lo = np.ascontiguousarray(np.asarray(lower, dtype=np.float32))
        hi = np.ascontiguousarray(np.asarray(upper, dtype=np.float32))
        if lo.shape != (self.n_cv,) or hi.shape != (self.n_cv,):
            raise ValueError("bounds must be [n_cv]")
        _check(lib().rid_ensemble_set_cv_bounds(self.handle, lo.ctypes.data_as(ctypes.c_void_p),
                                                hi.ctypes.data_as(ctypes.c_void_p)))

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.rid_ensemble_destroy(self.handle)
        self.handle = None

    __del__ = close


def cv_eval(system: System, pos, stream=None, with_x=True):
    """rid_cv_eval: pos [B][n_atoms][3] -> (s [B][n], x [B][2n] or None)."""
    torch = _torch()
    B = pos.shape[0]
    _f32(pos, (B, system.n_atoms, 3), "pos")
    s = torch.empty((B, system.n_cv), dtype=torch.float32, device=pos.device)
    x = torch.empty((B, 2 * system.n_cv), dtype=torch.float32, device=pos.device) if with_x else None
    _check(lib().rid_cv_eval(system.handle, _ptr(pos), B, _ptr(s), _ptr(x), _stream(stream)))
    return s, x


def model_dev(ens: Ensemble, s, stream=None, want_g=True):
    """rid_model_dev: s [B][n] -> (eps [B], gbar [B][n], A [B][K], g [B][K][n])."""
    torch = _torch()
    B = s.shape[0]
    _f32(s, (B, ens.n_cv), "s")
    dev = s.device
    eps = torch.empty(B, dtype=torch.float32, device=dev)
    gbar = torch.empty((B, ens.n_cv), dtype=torch.float32, device=dev)
    A = torch.empty((B, ens.K), dtype=torch.float32, device=dev) if want_g else None
    g = torch.empty((B, ens.K, ens.n_cv), dtype=torch.float32, device=dev) if want_g else None
    _check(lib().rid_model_dev(ens.handle, _ptr(s), B, _ptr(eps), _ptr(gbar), _ptr(A),
                               _ptr(g), _stream(stream)))
    return eps, gbar, A, g


def cluster_frames(s, threshold: float, eps=None, eps0: float = 0.0, max_clusters: int = 4096,
                   adapt: bool = False, lower: int = 1, upper: int = 1, stream=None):
    """rid_cluster_frames: s [B][n] (cuda float32) -> dict(labels [B] int32,
    leaders [n] int32 frame indices, n_clusters, threshold)."""
    torch = _torch()
    B, n = s.shape
    _f32(s, (B, n), "s")
    if eps is not None:
        _f32(eps, (B,), "eps")
    labels = torch.empty(B, dtype=torch.int32, device=s.device)
    leaders = torch.empty(max_clusters, dtype=torch.int32, device=s.device)
    nc = ctypes.c_int()
    tu = ctypes.c_float()
    _check(lib().rid_cluster_frames(_ptr(s), B, n, _ptr(eps), float(eps0), float(threshold),
                                    int(bool(adapt)), int(lower), int(upper), int(max_clusters),
                                    _ptr(labels), _ptr(leaders), ctypes.byref(nc),
                                    ctypes.byref(tu), _stream(stream)))
    nl = min(nc.value, max_clusters)
    return dict(labels=labels, leaders=leaders[:nl], n_clusters=nc.value, threshold=tu.value)


def select(ens: Ensemble, s, eps0: float, threshold: float, lower: int, upper: int,
           max_selection: int, adapt: bool = True, stream=None):
    """rid_select: the selection phase on CV frames s [B][n] -> dict(eps [B],
    labels [B], selected [<= max_selection] frame indices, n_clusters,
    threshold)."""
    torch = _torch()
    B = s.shape[0]
    _f32(s, (B, ens.n_cv), "s")
    eps = torch.empty(B, dtype=torch.float32, device=s.device)
    labels = torch.empty(B, dtype=torch.int32, device=s.device)
    sel = torch.empty(max_selection, dtype=torch.int32, device=s.device)
    ns, nc = ctypes.c_int(), ctypes.c_int()
    tu = ctypes.c_float()
    _check(lib().rid_select(ens.handle, _ptr(s), B, float(eps0), float(threshold),
                            int(bool(adapt)), int(lower), int(upper), int(max_selection),
                            _ptr(eps), _ptr(labels), _ptr(sel), ctypes.byref(ns),
                            ctypes.byref(nc), ctypes.byref(tu), _stream(stream)))
    return dict(eps=eps, labels=labels, selected=sel[:ns.value], n_clusters=nc.value,
                threshold=tu.value)


def adjust_trust_levels(n_clusters: int, numb_cluster_threshold: int, trust_lvl_1: float,
                        trust_lvl_2: float, scale: float):
    """rid_adjust_trust_levels: the trust levels of the next iteration
    (raised by `scale` when n_clusters < numb_cluster_threshold)."""
    l1, l2 = ctypes.c_float(trust_lvl_1), ctypes.c_float(trust_lvl_2)
    _check(lib().rid_adjust_trust_levels(int(n_clusters), int(numb_cluster_threshold),
                                         float(scale), ctypes.byref(l1), ctypes.byref(l2)))
    return l1.value, l2.value


def bias_force(system: System, ens: Ensemble, pos, eps0: float, eps1: float,
               stream=None, out=None, conservative=False, noalloc=False):
    """rid_bias_force (rid_bias_force_conservative when ``conservative``,
    rid_bias_force_noalloc when ``noalloc``):
    pos [B][n_atoms][3] -> dict(F, E, eps, sigma, flags)."""
    torch = _torch()
    B = pos.shape[0]
    _f32(pos, (B, system.n_atoms, 3), "pos")
    dev = pos.device
    if out is None:
        out = dict(
            F=torch.empty((B, system.n_atoms, 3), dtype=torch.float32, device=dev),
            E=torch.empty(B, dtype=torch.float32, device=dev),
            eps=torch.empty(B, dtype=torch.float32, device=dev),
            sigma=torch.empty(B, dtype=torch.float32, device=dev),
            flags=torch.empty(B, dtype=torch.uint8, device=dev),
        )
    if conservative and noalloc:
        raise ValueError("the no-allocation entry point is the frozen-switch bias force")
    fn = (lib().rid_bias_force_conservative if conservative else
          lib().rid_bias_force_noalloc if noalloc else lib().rid_bias_force)
    _check(fn(system.handle, ens.handle, _ptr(pos), B, float(eps0), float(eps1),
              _ptr(out["F"]), _ptr(out.get("E")), _ptr(out.get("eps")),
              _ptr(out.get("sigma")), _ptr(out.get("flags")), _stream(stream)))
    return out


def mcmc_run(ens: Ensemble, s, n_steps: int, kT: float, step_size: float, seed: int,
             step0: int = 0, proj=(0, 1), nbins: int = 101, hist1=None, hist2=None,
             accepted=None, stream=None):
    """rid_mcmc_run: Metropolis MCMC of W walkers in CV space; s [W][n] float32
    on the device is updated in place.  The uint32 counts are held in int32
    tensors (hist1 [n][nbins], hist2 [nbins][nbins]), accepted in an int64
    tensor; pass them back in to accumulate.  Returns dict(hist1, hist2,
    accepted)."""
    torch = _torch()
    W = s.shape[0]
    _f32(s, (W, ens.n_cv), "s")
    dev = s.device
    if hist1 is None:
        hist1 = torch.zeros((ens.n_cv, nbins), dtype=torch.int32, device=dev)
    if hist2 is None:
        hist2 = torch.zeros((nbins, nbins), dtype=torch.int32, device=dev)
    if accepted is None:
        accepted = torch.zeros(1, dtype=torch.int64, device=dev)
    _check(lib().rid_mcmc_run(ens.handle, _ptr(s), W, int(n_steps), int(step0), float(kT),
                              float(step_size), int(seed) & 0xFFFFFFFFFFFFFFFF, int(proj[0]),
                              int(proj[1]), int(nbins), _ptr(hist1), _ptr(hist2),
                              _ptr(accepted), _stream(stream)))
    return dict(hist1=hist1, hist2=hist2, accepted=accepted)


def cv_apply_force(system: System, pos, fcv, stream=None):
    """rid_cv_apply_force: F_a = sum_i f_i ds_i/dr_a."""
    torch = _torch()
    B = pos.shape[0]
    _f32(pos, (B, system.n_atoms, 3), "pos")
    _f32(fcv, (B, system.n_cv), "fcv")
    F = torch.empty((B, system.n_atoms, 3), dtype=torch.float32, device=pos.device)
    _check(lib().rid_cv_apply_force(system.handle, _ptr(pos), _ptr(fcv), B, _ptr(F),
                                    _stream(stream)))
    return F


def mf_train_step(ens: Ensemble, s, F, lr: float, stream=None):
    """rid_mf_train_step: one double-backward + Adam step; returns loss [K]."""
    torch = _torch()
    B = s.shape[0]
    _f32(s, (B, ens.n_cv), "s")
    _f32(F, (B, ens.n_cv), "F")
    loss = torch.empty(ens.K, dtype=torch.float32, device=s.device)
    _check(lib().rid_mf_train_step(ens.handle, _ptr(s), _ptr(F), B, float(lr), _ptr(loss),
                                   _stream(stream)))
    return loss


def mf_loss_grad(ens: Ensemble, s, F, stream=None):
    """rid_mf_loss_grad: (loss [K], grad [n_params] packed) without update."""
    torch = _torch()
    B = s.shape[0]
    _f32(s, (B, ens.n_cv), "s")
    _f32(F, (B, ens.n_cv), "F")
    loss = torch.empty(ens.K, dtype=torch.float32, device=s.device)
    grad = torch.empty(ens.n_params, dtype=torch.float32, device=s.device)
    _check(lib().rid_mf_loss_grad(ens.handle, _ptr(s), _ptr(F), B, _ptr(loss), _ptr(grad),
                                  _stream(stream)))
    return loss, grad


def mf_grad(ens: Ensemble, s, rho, stream=None):
    """rid_mf_grad: d/dtheta sum rho . g for rho [B][K][n] -> grad [n_params]."""
    torch = _torch()
    B = s.shape[0]
    _f32(s, (B, ens.n_cv), "s")
    _f32(rho, (B, ens.K, ens.n_cv), "rho")
    grad = torch.empty(ens.n_params, dtype=torch.float32, device=s.device)
    _check(lib().rid_mf_grad(ens.handle, _ptr(s), _ptr(rho), B, _ptr(grad), _stream(stream)))
    return grad


def _make_mean_force_fn():
    torch = _torch()

    class MeanForce(torch.autograd.Function):
        """g = grad_s A_k(s) of every member as a differentiable function of
        the ensemble's packed parameters.  forward loads ``params`` (FP32,
        packed layout, on the device) into the ensemble
        (rid_ensemble_load_params, stream-ordered) and calls rid_model_dev;
        backward calls the double-backward kernels (rid_mf_grad) at those
        parameters.  ``params`` is therefore the source of truth: the
        ensemble's masters follow it at every forward call.  Ensembles with a
        dropout rate are refused: rid_model_dev evaluates the full network
        while the training sweeps apply the masks, so the backward would
        belong to another function."""

        @staticmethod
        def forward(ctx, s, params, ens):
            if ens.dropout_rate > 0.0:
                raise ValueError("mean_force: the ensemble has a dropout rate; the "
                                 "autograd form is defined for the full network only")
            _f32(params, (ens.n_params,), "params")
            _check(lib().rid_ensemble_load_params(ens.handle, _ptr(params), _stream(None)))
            ctx.ens = ens
            ctx.save_for_backward(s)
            _, _, _, g = model_dev(ens, s.contiguous())
            return g

        @staticmethod
        def backward(ctx, gout):
            (s,) = ctx.saved_tensors
            grad = mf_grad(ctx.ens, s.contiguous(), gout.contiguous())
            return None, grad, None

    return MeanForce


_MEAN_FORCE = None


def mean_force(s, params, ens: Ensemble):
    """Differentiable per-member mean forces g [B][K][n] (see MeanForce)."""
    global _MEAN_FORCE
    if _MEAN_FORCE is None:
        _MEAN_FORCE = _make_mean_force_fn()
    return _MEAN_FORCE.apply(s, params, ens)


class Server:
    """Continuous-batching bias-force server (rid_server_*).  submit(): host
    arrays in, host arrays out; submit_device(): device tensors in and out
    (walker state resident); submit() and wait() may be called from several
    threads (the C calls release the GIL); replay() drives a whole trace from
    native threads."""

    def __init__(self, hbm_budget_bytes: int, n_streams: int = 4,
                 max_batch_walkers: int = 4096, fifo: bool = False):
        h = ctypes.c_void_p()
        _check(lib().rid_server_create(int(hbm_budget_bytes), int(n_streams),
                                       int(max_batch_walkers),
                                       RID_SERVE_FIFO if fifo else 0, ctypes.byref(h)))
        self.handle = h
        self._models = []        # keep registered handles alive
        self._tickets = {}

    def register(self, system: System, ensemble: Ensemble, eps0: float, eps1: float) -> int:
        mid = ctypes.c_int()
        _check(lib().rid_server_register(self.handle, system.handle, ensemble.handle,
                                         float(eps0), float(eps1), ctypes.byref(mid)))
        self._models.append((system, ensemble))
        return mid.value

    def submit(self, model_id: int, pos) -> int:
        p = np.ascontiguousarray(np.asarray(pos, dtype=np.float32))
        system = self._models[model_id][0]
        if p.ndim != 3 or p.shape[1:] != (system.n_atoms, 3):
            raise ValueError("pos must be [n_walkers][n_atoms][3]")
        t = ctypes.c_int64()
        _check(lib().rid_server_submit(self.handle, int(model_id),
                                       p.ctypes.data_as(ctypes.c_void_p), int(p.shape[0]),
                                       ctypes.byref(t)))
        self._tickets[t.value] = (p.shape[0], system.n_atoms)
        return t.value

    def submit_device(self, model_id: int, pos, out: dict) -> int:
        """rid_server_submit_device: pos [w][N][3] float32 on the device;
        out: dict of device tensors F [w][N][3] and (optional) E, eps, sigma
        [w], written by the request's batch.  Keep them alive and pos
        unchanged until wait()."""
        system = self._models[model_id][0]
        w = pos.shape[0]
        _f32(pos, (w, system.n_atoms, 3), "pos")
        _f32(out["F"], (w, system.n_atoms, 3), "F")
        t = ctypes.c_int64()
        _check(lib().rid_server_submit_device(
            self.handle, int(model_id), _ptr(pos), int(w), _ptr(out["F"]), _ptr(out.get("E")),
            _ptr(out.get("eps")), _ptr(out.get("sigma")), ctypes.byref(t)))
        self._tickets[t.value] = None
        return t.value

    def wait(self, ticket: int):
        dims = self._tickets.pop(ticket)
        lat = ctypes.c_double()
        if dims is None:            # device request: results are in its tensors
            _check(lib().rid_server_wait(self.handle, ctypes.c_int64(ticket), None, None, None,
                                         None, ctypes.byref(lat)))
            return dict(latency_us=lat.value)
        w, N = dims
        F = np.empty((w, N, 3), np.float32)
        E = np.empty(w, np.float32)
        eps = np.empty(w, np.float32)
        sig = np.empty(w, np.float32)
        vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        _check(lib().rid_server_wait(self.handle, ctypes.c_int64(ticket), vp(F), vp(E),
                                     vp(eps), vp(sig), ctypes.byref(lat)))
        return dict(F=F, E=E, eps=eps, sigma=sig, latency_us=lat.value)

    def replay(self, reqs):
        """rid_server_replay over a list of dicts (model, arrival_s, pos and,
        for device requests, F / E / eps / sigma device tensors; host
        requests give host numpy positions and get no host results).
        Returns (latency_us, submit_lag_us, wall_s)."""
        n = len(reqs)
        arr = (ReplayRequest * n)()
        keep = []
        for i, q in enumerate(reqs):
            pos = q["pos"]
            dev = not isinstance(pos, np.ndarray)
            if dev:
                p = _ptr(pos)
                out = q.get("out", {})
                arr[i] = ReplayRequest(int(q["model"]), int(pos.shape[0]), float(q["arrival_s"]),
                                       p, 1, _ptr(out.get("F")), _ptr(out.get("E")),
                                       _ptr(out.get("eps")), _ptr(out.get("sigma")))
            else:
                a = np.ascontiguousarray(pos, dtype=np.float32)
                keep.append(a)
                arr[i] = ReplayRequest(int(q["model"]), int(a.shape[0]), float(q["arrival_s"]),
                                       a.ctypes.data_as(ctypes.c_void_p), 0, None, None, None, None)
        lat = np.zeros(n, np.float64)
        lag = np.zeros(n, np.float64)
        wall = ctypes.c_double()
        _check(lib().rid_server_replay(self.handle, arr, n, lat.ctypes.data_as(ctypes.c_void_p),
                                       lag.ctypes.data_as(ctypes.c_void_p), ctypes.byref(wall)))
        return lat, lag, wall.value

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().rid_server_stats(self.handle, ctypes.byref(st)))
        return {name: getattr(st, name) for name, _ in ServerStats._fields_}

    def reset_stats(self):
        lib().rid_server_reset_stats(self.handle)

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.rid_server_destroy(self.handle)
        self.handle = None

    __del__ = close


def profile_enable(on: bool = True, keep: bool = False):
    """Per-kernel HIP-event timing inside the library: on=True clears and
    starts (keep=True resumes without clearing); on=False pauses and keeps
    what was collected."""
    lib().rid_profile_enable((2 if keep else 1) if on else 0)


def profile_read(kind: int):
    """(total_ms, launches) of a kernel family since the last clear."""
    tot = ctypes.c_double()
    cnt = ctypes.c_int64()
    _check(lib().rid_profile_read(int(kind), ctypes.byref(tot), ctypes.byref(cnt)))
    return tot.value, cnt.value


def lr_exponential(step: int, init_lr=8e-4, decay_steps=120, decay_rate=0.96) -> float:
    return float(lib().rid_lr_exponential(int(step), float(init_lr), int(decay_steps),
                                          float(decay_rate)))


def mf_label(traj, s0, kappa, angular_mask=None, std_threshold=5.0, stream=None):
    """rid_mf_label: traj [M][T][n], s0 [M][n] -> (F [M][n] f64, SE, keep)."""
    torch = _torch()
    M, T, n = traj.shape
    _f32(traj, (M, T, n), "traj")
    _f32(s0, (M, n), "s0")
    k = np.ascontiguousarray(np.broadcast_to(np.asarray(kappa, np.float32), (n,)))
    m = None if angular_mask is None else np.ascontiguousarray(np.asarray(angular_mask, np.uint8))
    dev = traj.device
    F = torch.empty((M, n), dtype=torch.float64, device=dev)
    se = torch.empty((M, n), dtype=torch.float64, device=dev)
    keep = torch.empty(M, dtype=torch.uint8, device=dev)
    _check(lib().rid_mf_label(_ptr(traj), _ptr(s0), k.ctypes.data_as(ctypes.c_void_p),
                              None if m is None else m.ctypes.data_as(ctypes.c_void_p),
                              M, T, n, float(std_threshold), _ptr(F), _ptr(se), _ptr(keep),
                              _stream(stream)))
    return F, se, keep
