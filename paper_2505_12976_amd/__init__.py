"""Python binding of the MI355X Schulze library (``libschulze.so``).

Argument marshalling only: every step runs in the library's HIP kernels.
Tensors are torch tensors on the GPU; the library receives their device
pointers and torch's current stream.  The entry points carry the C ABI's
names (``include/schulze.h``):

    pairwise(ballots, m, voter_weight=None, dtype="u16"|"i32") -> d
    closure(d, mode="winning_votes"|"margin")                  -> p
    winners(p)                                                  -> (is_winner, n_winners)
    ranking(p)                                                  -> (order, beaten_by)

A missing or unloadable library raises; nothing falls back to the CPU.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libschulze.so")

OK, EINVAL, ERANGE, ENOMEM, EDEVICE, EBALLOT, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
U16, I32 = 1, 2
WINNING_VOTES, MARGIN = 0, 1

EXPORTS = (
    "schulze_create", "schulze_destroy", "schulze_strerror", "schulze_get_device_error",
    "schulze_pairwise", "schulze_closure", "schulze_winners", "schulze_ranking",
    "schulze_set_timing", "schulze_kernel_time", "schulze_reset_timing", "schulze_set_closure_schedule",
    "schulze_set_value_ranking", "schulze_set_closure_tile", "schulze_set_sparse_count", "schulze_set_sweep_limits",
    "schulze_weights", "schulze_widest_from", "schulze_verify", "schulze_features",
    "schulze_mlp_param_count", "schulze_mlp_forward", "schulze_mlp_loss", "schulze_mlp_backward", "schulze_mlp_adam",
    "schulze_mlp_train_step",
    "schulze_winners_learned",
    "schulze_batch_plan", "schulze_batch_destroy", "schulze_batch_run", "schulze_batch_set_closure",
    "schulze_batch_get_closure", "schulze_batch_autotune", "schulze_winners_propagate",
    "schulze_topk_propagate", "schulze_valu_probe", "schulze_closure_value_bits", "schulze_set_proposer", "schulze_verify_noalloc",
    "schulze_verify_counts",
)


class PropagateStats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("sweeps", ctypes.c_int32), ("n_winners", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class TopkStats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("ranked", ctypes.c_int32), ("rounds", ctypes.c_int32),
                ("sweeps", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class LearnedStats(ctypes.Structure):
    _fields_ = [("proposal", ctypes.c_int32), ("first_hit", ctypes.c_int32), ("verify_calls", ctypes.c_int32),
                ("climbs", ctypes.c_int32), ("fallback", ctypes.c_int32), ("n_winners", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}
class MlpState(ctypes.Structure):
    """schulze_mlp: parameters, Adam moments, gradient, device step counter, hyperparameters."""
    _fields_ = [("params", ctypes.c_void_p), ("adam_m", ctypes.c_void_p), ("adam_v", ctypes.c_void_p),
                ("grad", ctypes.c_void_p), ("step", ctypes.c_void_p), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float)]


class TrainBatch(ctypes.Structure):
    """schulze_train_batch: feature rows, election offsets, winner marks."""
    _fields_ = [("feat", ctypes.c_void_p), ("offsets", ctypes.c_void_p), ("winner", ctypes.c_void_p),
                ("M", ctypes.c_int64), ("E", ctypes.c_int32)]


SCHEDULE_AUTO, SCHEDULE_PHASED = 0, 1
PROPOSERS = {"network": 0, "borda": 1, "copeland": 2, "filter+borda": 3}

_lib = None


BATCH_MAX_M = 1024
BATCH_GRAPH = 1
CLOSURE_VARIANTS = {"auto": -1, "registers": 0, "tiled32": 1, "tiled64": 2, "tiled128": 3}


class Election(ctypes.Structure):
    """One election of a batch (offsets in elements)."""
    _fields_ = [("ballot_off", ctypes.c_int64), ("n", ctypes.c_int64), ("L", ctypes.c_int32),
                ("m", ctypes.c_int32), ("mat_off", ctypes.c_int64), ("vec_off", ctypes.c_int64)]


class BatchOptions(ctypes.Structure):
    _fields_ = [("max_range_pairs", ctypes.c_int32), ("closure_only", ctypes.c_int32), ("topk", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 5)]


class SchulzeError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


def build() -> str:
    from . import _build
    return _build.build()


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libschulze.so (building it first only if it does not exist)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        build()
    lib = ctypes.CDLL(path)
    c_int, c_i32, c_i64, vp = ctypes.c_int, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    lib.schulze_create.argtypes = [ctypes.POINTER(vp), c_int]
    lib.schulze_destroy.argtypes = [vp]
    lib.schulze_destroy.restype = None
    lib.schulze_strerror.argtypes = [c_int]
    lib.schulze_strerror.restype = ctypes.c_char_p
    lib.schulze_get_device_error.argtypes = [vp, vp, ctypes.POINTER(c_i32)]
    lib.schulze_pairwise.argtypes = [vp, vp, vp, c_int, c_i64, c_i32, c_i32, vp, c_int, vp, c_i64]
    lib.schulze_closure.argtypes = [vp, vp, vp, c_i64, c_i32, c_int, c_int, vp, c_i64]
    lib.schulze_winners.argtypes = [vp, vp, vp, c_i64, c_i32, c_int, vp, vp]
    lib.schulze_ranking.argtypes = [vp, vp, vp, c_i64, c_i32, c_int, vp, vp]
    lib.schulze_set_timing.argtypes = [vp, c_int]
    lib.schulze_kernel_time.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(c_i64), ctypes.POINTER(ctypes.c_double)]
    lib.schulze_reset_timing.argtypes = [vp]
    lib.schulze_set_closure_schedule.argtypes = [vp, c_int]
    lib.schulze_set_value_ranking.argtypes = [vp, c_int]
    lib.schulze_set_sweep_limits.argtypes = [vp, c_i64, c_i32]
    lib.schulze_closure_value_bits.argtypes = [vp, vp, ctypes.POINTER(c_i32)]
    lib.schulze_set_proposer.argtypes = [vp, c_int]
    lib.schulze_set_closure_tile.argtypes = [vp, c_int]
    lib.schulze_set_sparse_count.argtypes = [vp, c_int]
    lib.schulze_valu_probe.argtypes = [vp, vp, c_i32, c_i64, vp, ctypes.POINTER(c_i64)]
    lib.schulze_weights.argtypes = [vp, vp, vp, c_i64, c_i32, c_int, c_int, vp, c_i64, vp, c_i64]
    lib.schulze_widest_from.argtypes = [vp, vp, vp, c_i64, c_i32, c_int, c_i32, vp]
    lib.schulze_verify.argtypes = [vp, vp, vp, c_i64, vp, c_i64, c_i32, c_int, c_i32, vp, vp, vp, vp, vp]
    lib.schulze_verify_noalloc.argtypes = [vp, vp, vp, c_i64, vp, c_i64, c_i32, c_int, c_i32, vp, vp, vp, vp, vp]
    lib.schulze_verify_counts.argtypes = [vp, vp, vp, c_i64, c_i32, c_int, c_int, c_i32, vp, vp, vp, vp, vp]
    lib.schulze_features.argtypes = [vp, vp, vp, c_i64, c_i32, c_int, c_int, ctypes.c_float, vp]
    lib.schulze_mlp_param_count.argtypes = []
    lib.schulze_winners_learned.argtypes = [vp, vp, vp, c_i64, c_i32, c_int, c_int, ctypes.c_float, vp, c_i32, c_i32,
                                            vp, vp, ctypes.POINTER(LearnedStats)]
    lib.schulze_mlp_forward.argtypes = [vp, vp, vp, vp, c_i64, vp]
    lib.schulze_mlp_loss.argtypes = [vp, vp, vp, vp, vp, c_i32, vp, vp]
    lib.schulze_mlp_backward.argtypes = [vp, vp, vp, vp, c_i64, vp, vp]
    lib.schulze_mlp_adam.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                     ctypes.c_float, c_i32]
    lib.schulze_mlp_train_step.argtypes = [vp, vp, ctypes.POINTER(MlpState), ctypes.POINTER(TrainBatch), vp]
    lib.schulze_batch_plan.argtypes = [vp, ctypes.POINTER(Election), c_i32, c_int, c_int,
                                       ctypes.POINTER(BatchOptions), ctypes.POINTER(vp)]
    lib.schulze_winners_propagate.argtypes = [vp, vp, vp, c_i64, c_i32, c_int, c_int, c_int, vp, vp,
                                              ctypes.POINTER(PropagateStats)]
    lib.schulze_topk_propagate.argtypes = [vp, vp, vp, c_i64, c_i32, c_int, c_int, c_int, c_i32, vp,
                                           ctypes.POINTER(TopkStats)]
    lib.schulze_batch_destroy.argtypes = [vp]
    lib.schulze_batch_destroy.restype = None
    lib.schulze_batch_run.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, c_int]
    lib.schulze_batch_set_closure.argtypes = [vp, c_i32, c_i32, c_i32, c_i32]
    lib.schulze_batch_get_closure.argtypes = [vp, c_i32, c_i32, ctypes.POINTER(c_i32)]
    lib.schulze_batch_autotune.argtypes = [vp, vp, c_i32, c_i32, ctypes.POINTER(ctypes.c_float)]
    for name in EXPORTS:
        if name not in ("schulze_destroy", "schulze_strerror", "schulze_batch_destroy"):
            getattr(lib, name).restype = c_int
    _lib = lib
    return lib


def mlp_param_count() -> int:
    return int(load_library().schulze_mlp_param_count())


def strerror(code: int) -> str:
    return load_library().schulze_strerror(code).decode()


def _check(rc: int, where: str) -> None:
    if rc != OK:
        raise SchulzeError(rc, where)


def _dtype_code(dtype) -> int:
    import torch
    if dtype in ("u16", U16, torch.uint16):
        return U16
    if dtype in ("i32", I32, torch.int32):
        return I32
    raise ValueError(f"unknown counter dtype {dtype!r}")


def _torch_dtype(code: int):
    import torch
    return torch.uint16 if code == U16 else torch.int32


def _mode_code(mode) -> int:
    if mode in ("winning_votes", WINNING_VOTES):
        return WINNING_VOTES
    if mode in ("margin", MARGIN):
        return MARGIN
    raise ValueError(f"unknown weight mode {mode!r}")


class Context:
    """One library context bound to a GPU (one per host thread)."""

    def __init__(self, device: int = 0):
        import torch
        self.device = device
        self._torch_device = torch.device("cuda", device)
        lib = load_library()
        h = ctypes.c_void_p()
        _check(lib.schulze_create(ctypes.byref(h), device), "schulze_create")
        self._h = h
        self._lib = lib

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.schulze_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- helpers
    def _stream(self):
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream(self._torch_device).cuda_stream)

    def _dev(self, t, what):
        if t.device != self._torch_device:
            raise ValueError(f"{what} must live on {self._torch_device}")
        return ctypes.c_void_p(t.data_ptr())

    def device_error(self) -> int:
        v = ctypes.c_int32(0)
        _check(self._lib.schulze_get_device_error(self._h, self._stream(), ctypes.byref(v)),
               "schulze_get_device_error")
        return v.value

    def raise_device_error(self) -> None:
        code = self.device_error()
        if code != OK:
            raise SchulzeError(code, "device")

    # -------------------------------------------------------------- entry points
    def pairwise(self, ballots, m: int, voter_weight=None, dtype="i32", out=None):
        """d[x][y] = weight of voters preferring x to y.  ballots: (n, L)
        uint16 (0xFFFF pads) or int32 (negative pads) on the GPU."""
        import torch
        if ballots.dim() != 2 or not ballots.is_contiguous():
            raise ValueError("ballots must be a contiguous (n, L) tensor")
        if ballots.dtype == torch.uint16:
            bcode = U16
        elif ballots.dtype == torch.int32:
            bcode = I32
        else:
            raise ValueError("ballots must be uint16 or int32")
        n, L = ballots.shape
        dcode = _dtype_code(dtype)
        d = out if out is not None else torch.empty((m, m), dtype=_torch_dtype(dcode), device=self._torch_device)
        wp = None
        if voter_weight is not None:
            if voter_weight.dtype != torch.uint32 or voter_weight.shape != (n,) or not voter_weight.is_contiguous():
                raise ValueError("voter_weight must be a contiguous uint32 tensor of shape (n,)")
            wp = self._dev(voter_weight, "voter_weight")
        rc = self._lib.schulze_pairwise(self._h, self._stream(), self._dev(ballots, "ballots"), bcode, n, L, m,
                                        wp, dcode, self._dev(d, "d"), d.stride(0))
        _check(rc, "schulze_pairwise")
        return d

    def closure(self, d, mode="winning_votes", out=None):
        """p[x][y] = width of a widest x->y path (zero diagonal)."""
        import torch
        m = d.shape[0]
        dcode = _dtype_code(d.dtype)
        p = out if out is not None else torch.empty_like(d)
        rc = self._lib.schulze_closure(self._h, self._stream(), self._dev(d, "d"), d.stride(0), m, dcode,
                                       _mode_code(mode), self._dev(p, "p"), p.stride(0))
        _check(rc, "schulze_closure")
        return p

    def winners(self, p):
        """(is_winner uint8[m], n_winners int32[1]) on the GPU."""
        import torch
        m = p.shape[0]
        w = torch.empty(m, dtype=torch.uint8, device=self._torch_device)
        nw = torch.empty(1, dtype=torch.int32, device=self._torch_device)
        rc = self._lib.schulze_winners(self._h, self._stream(), self._dev(p, "p"), p.stride(0), m,
                                       _dtype_code(p.dtype), self._dev(w, "is_winner"), self._dev(nw, "n_winners"))
        _check(rc, "schulze_winners")
        return w, nw

    def ranking(self, p):
        """(order int32[m], beaten_by int32[m]) on the GPU."""
        import torch
        m = p.shape[0]
        order = torch.empty(m, dtype=torch.int32, device=self._torch_device)
        beaten = torch.empty(m, dtype=torch.int32, device=self._torch_device)
        rc = self._lib.schulze_ranking(self._h, self._stream(), self._dev(p, "p"), p.stride(0), m,
                                       _dtype_code(p.dtype), self._dev(order, "order"), self._dev(beaten, "beaten_by"))
        _check(rc, "schulze_ranking")
        return order, beaten

    def weights(self, d, mode="winning_votes", transposed=True, direct=True):
        """(w, wt): edge weights and their transpose (either may be skipped)."""
        import torch
        m = d.shape[0]
        w = torch.empty_like(d) if direct else None
        wt = torch.empty_like(d) if transposed else None
        rc = self._lib.schulze_weights(self._h, self._stream(), self._dev(d, "d"), d.stride(0), m,
                                       _dtype_code(d.dtype), _mode_code(mode),
                                       None if w is None else self._dev(w, "w"), 0 if w is None else w.stride(0),
                                       None if wt is None else self._dev(wt, "wt"),
                                       0 if wt is None else wt.stride(0))
        _check(rc, "schulze_weights")
        return w, wt

    def widest_from(self, w, source: int, out=None):
        """out[v] = p(source, v) (with transposed weights: p(v, source))."""
        import torch
        m = w.shape[0]
        out = out if out is not None else torch.empty(m, dtype=w.dtype, device=self._torch_device)
        rc = self._lib.schulze_widest_from(self._h, self._stream(), self._dev(w, "w"), w.stride(0), m,
                                           _dtype_code(w.dtype), source, self._dev(out, "out"))
        _check(rc, "schulze_widest_from")
        return out

    def verify(self, w, wt, cand: int, score=None, want_tied=False, noalloc=False, out=None):
        """(verdict int32[4], p_from, p_to, tied or None); see schulze_verify.
        noalloc: call schulze_verify_noalloc (sweep state in the library's
        static device scratch).  out: optional (verdict, p_from, p_to, tied)
        tensors to write into."""
        import torch
        if out is not None:
            verdict, p_from, p_to, tied = out
            fn = self._lib.schulze_verify_noalloc if noalloc else self._lib.schulze_verify
            m = w.shape[0]
            sp = None if score is None else self._dev(score, "score")
            rc = fn(self._h, self._stream(), self._dev(w, "w"), w.stride(0), self._dev(wt, "wt"), wt.stride(0), m,
                    _dtype_code(w.dtype), cand, sp, self._dev(p_from, "p_from"), self._dev(p_to, "p_to"),
                    self._dev(verdict, "verdict"), None if tied is None else self._dev(tied, "tied"))
            _check(rc, "schulze_verify_noalloc" if noalloc else "schulze_verify")
            return verdict, p_from, p_to, tied
        m = w.shape[0]
        p_from = torch.empty(m, dtype=w.dtype, device=self._torch_device)
        p_to = torch.empty(m, dtype=w.dtype, device=self._torch_device)
        verdict = torch.empty(4, dtype=torch.int32, device=self._torch_device)
        tied = torch.empty(m, dtype=torch.int32, device=self._torch_device) if want_tied else None
        sp = None
        if score is not None:
            if score.dtype != torch.float32 or score.shape != (m,):
                raise ValueError("score must be a float32 tensor of shape (m,)")
            sp = self._dev(score, "score")
        fn = self._lib.schulze_verify_noalloc if noalloc else self._lib.schulze_verify
        rc = fn(self._h, self._stream(), self._dev(w, "w"), w.stride(0),
                self._dev(wt, "wt"), wt.stride(0), m, _dtype_code(w.dtype), cand, sp,
                self._dev(p_from, "p_from"), self._dev(p_to, "p_to"),
                self._dev(verdict, "verdict"), None if tied is None else self._dev(tied, "tied"))
        _check(rc, "schulze_verify_noalloc" if noalloc else "schulze_verify")
        return verdict, p_from, p_to, tied

    def verify_counts(self, d, cand: int, mode="winning_votes", score=None, want_tied=False):
        """(verdict int32[4], p_from, p_to, tied or None) of cand straight
        from the counts d; see schulze_verify_counts."""
        import torch
        m = d.shape[0]
        p_from = torch.empty(m, dtype=d.dtype, device=self._torch_device)
        p_to = torch.empty(m, dtype=d.dtype, device=self._torch_device)
        verdict = torch.empty(4, dtype=torch.int32, device=self._torch_device)
        tied = torch.empty(m, dtype=torch.int32, device=self._torch_device) if want_tied else None
        sp = None
        if score is not None:
            if score.dtype != torch.float32 or score.shape != (m,):
                raise ValueError("score must be a float32 tensor of shape (m,)")
            sp = self._dev(score, "score")
        rc = self._lib.schulze_verify_counts(self._h, self._stream(), self._dev(d, "d"), d.stride(0), m,
                                             _dtype_code(d.dtype), _mode_code(mode), cand, sp,
                                             self._dev(p_from, "p_from"), self._dev(p_to, "p_to"),
                                             self._dev(verdict, "verdict"),
                                             None if tied is None else self._dev(tied, "tied"))
        _check(rc, "schulze_verify_counts")
        return verdict, p_from, p_to, tied

    def features(self, d, n_voters: float, mode="winning_votes", out=None):
        """m x 16 float32 per-candidate features of d."""
        import torch
        m = d.shape[0]
        out = out if out is not None else torch.empty((m, 16), dtype=torch.float32, device=self._torch_device)
        rc = self._lib.schulze_features(self._h, self._stream(), self._dev(d, "d"), d.stride(0), m,
                                        _dtype_code(d.dtype), _mode_code(mode), float(n_voters),
                                        self._dev(out, "feat"))
        _check(rc, "schulze_features")
        return out

    def mlp_forward(self, params, feat, out=None):
        import torch
        M = feat.shape[0]
        out = out if out is not None else torch.empty(M, dtype=torch.float32, device=self._torch_device)
        rc = self._lib.schulze_mlp_forward(self._h, self._stream(), self._dev(params, "params"),
                                           self._dev(feat, "feat"), M, self._dev(out, "score"))
        _check(rc, "schulze_mlp_forward")
        return out

    def mlp_loss(self, score, offsets, winner):
        """(dscore, loss per election)."""
        import torch
        E = offsets.shape[0] - 1
        ds = torch.empty_like(score)
        loss = torch.empty(E, dtype=torch.float32, device=self._torch_device)
        rc = self._lib.schulze_mlp_loss(self._h, self._stream(), self._dev(score, "score"),
                                        self._dev(offsets, "offsets"), self._dev(winner, "winner"), E,
                                        self._dev(ds, "dscore"), self._dev(loss, "loss"))
        _check(rc, "schulze_mlp_loss")
        return ds, loss

    def mlp_backward(self, params, feat, dscore, out=None):
        import torch
        out = out if out is not None else torch.empty_like(params)
        rc = self._lib.schulze_mlp_backward(self._h, self._stream(), self._dev(params, "params"),
                                            self._dev(feat, "feat"), feat.shape[0], self._dev(dscore, "dscore"),
                                            self._dev(out, "grad"))
        _check(rc, "schulze_mlp_backward")
        return out

    def mlp_adam(self, params, grad, m1, m2, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
        rc = self._lib.schulze_mlp_adam(self._h, self._stream(), self._dev(params, "params"), self._dev(grad, "grad"),
                                        self._dev(m1, "adam_m"), self._dev(m2, "adam_v"), float(lr), float(beta1),
                                        float(beta2), float(eps), int(step))
        _check(rc, "schulze_mlp_adam")

    def mlp_train_step(self, params, adam_m, adam_v, grad, step, feat, offsets, winner, lr=1e-3, beta1=0.9,
                       beta2=0.999, eps=1e-8, loss=None):
        """One step (forward, segmented loss, backward, Adam); step: one
        int32 CUDA tensor that counts Adam steps (advanced on the device).
        Returns the per-election losses (a CUDA tensor)."""
        import torch
        E = offsets.shape[0] - 1
        if offsets.dtype != torch.int64 or winner.dtype != torch.uint8 or step.dtype != torch.int32:
            raise ValueError("offsets must be int64, winner uint8, step int32")
        if feat.dim() != 2 or feat.shape[1] != 16 or winner.shape != (feat.shape[0],):
            raise ValueError("feat must be (M, 16) and winner (M,)")
        loss = loss if loss is not None else torch.empty(E, dtype=torch.float32, device=self._torch_device)
        net = MlpState(self._dev(params, "params").value, self._dev(adam_m, "adam_m").value,
                       self._dev(adam_v, "adam_v").value, self._dev(grad, "grad").value,
                       self._dev(step, "step").value, float(lr), float(beta1), float(beta2), float(eps))
        b = TrainBatch(self._dev(feat, "feat").value, self._dev(offsets, "offsets").value,
                       self._dev(winner, "winner").value, int(feat.shape[0]), int(E))
        rc = self._lib.schulze_mlp_train_step(self._h, self._stream(), ctypes.byref(net), ctypes.byref(b),
                                              self._dev(loss, "loss"))
        _check(rc, "schulze_mlp_train_step")
        return loss

    def winners_learned(self, d, n_voters: float, params, mode="winning_votes", max_climb=8, max_tied=64):
        """(is_winner uint8[m], n_winners int32[1], stats dict): exact winners
        found through the proposer network (synchronises)."""
        import torch
        m = d.shape[0]
        w = torch.empty(m, dtype=torch.uint8, device=self._torch_device)
        nw = torch.empty(1, dtype=torch.int32, device=self._torch_device)
        st = LearnedStats()
        rc = self._lib.schulze_winners_learned(self._h, self._stream(), self._dev(d, "d"), d.stride(0), m,
                                               _dtype_code(d.dtype), _mode_code(mode), float(n_voters),
                                               None if params is None else self._dev(params, "params"),
                                               int(max_climb), int(max_tied),
                                               self._dev(w, "is_winner"), self._dev(nw, "n_winners"),
                                               ctypes.byref(st))
        _check(rc, "schulze_winners_learned")
        return w, nw, st.as_dict()

    def winners_propagate(self, d, mode="winning_votes", borda_order=True):
        """(is_winner uint8[m], n_winners int32[1], stats dict): winners by
        the paper's label-propagation algorithm (synchronises)."""
        import torch
        m = d.shape[0]
        w = torch.empty(m, dtype=torch.uint8, device=self._torch_device)
        nw = torch.empty(1, dtype=torch.int32, device=self._torch_device)
        st = PropagateStats()
        rc = self._lib.schulze_winners_propagate(self._h, self._stream(), self._dev(d, "d"), d.stride(0), m,
                                                 _dtype_code(d.dtype), _mode_code(mode), int(bool(borda_order)),
                                                 self._dev(w, "is_winner"), self._dev(nw, "n_winners"),
                                                 ctypes.byref(st))
        _check(rc, "schulze_winners_propagate")
        return w, nw, st.as_dict()

    def topk_propagate(self, d, k, mode="winning_votes", borda_order=True):
        """(level int32[m], stats dict): top-k by iterated winner removal,
        each level by the label-propagation algorithm (synchronises)."""
        import torch
        m = d.shape[0]
        level = torch.empty(m, dtype=torch.int32, device=self._torch_device)
        st = TopkStats()
        rc = self._lib.schulze_topk_propagate(self._h, self._stream(), self._dev(d, "d"), d.stride(0), m,
                                              _dtype_code(d.dtype), _mode_code(mode), int(bool(borda_order)),
                                              int(k), self._dev(level, "level"), ctypes.byref(st))
        _check(rc, "schulze_topk_propagate")
        return level, st.as_dict()

    # -------------------------------------------------------------- batches
    def batch_plan(self, elections, ballot_dtype="u16", mode="winning_votes", max_range_pairs=0,
                   closure_only=False, topk=0):
        """Plan a batch.  elections: sequence of (ballot_off, n, L, m, mat_off,
        vec_off) tuples (element offsets) or of Election structs.  topk > 0:
        runs given a level array compute top-k levels by winner removal."""
        import torch
        bcode = U16 if ballot_dtype in ("u16", U16, torch.uint16) else (
            I32 if ballot_dtype in ("i32", I32, torch.int32) else None)
        if bcode is None:
            raise ValueError("ballot dtype must be uint16 or int32")
        E = len(elections)
        arr = (Election * max(E, 1))()
        for i, el in enumerate(elections):
            arr[i] = el if isinstance(el, Election) else Election(*[int(v) for v in el])
        opt = BatchOptions(int(max_range_pairs), int(bool(closure_only)), int(topk))
        h = ctypes.c_void_p()
        rc = self._lib.schulze_batch_plan(self._h, arr, E, bcode, _mode_code(mode), ctypes.byref(opt), ctypes.byref(h))
        _check(rc, "schulze_batch_plan")
        d_elems = max((arr[i].mat_off + arr[i].m * arr[i].m for i in range(E)), default=0)
        vec_elems = max((arr[i].vec_off + arr[i].m for i in range(E)), default=0)
        return BatchPlan(self, h, E, bcode, d_elems, vec_elems)

    def batch_run(self, plan, ballots, d, is_winner, p=None, n_winners=None, beaten_by=None, order=None,
                  graph=False, level=None):
        """Run a planned batch (ballots None: d is the input counts)."""
        import torch

        def ptr(t, what, dtype, elems):
            if t is None:
                return None
            if t.dtype != dtype or not t.is_contiguous() or t.numel() < elems:
                raise ValueError(f"{what} must be a contiguous {dtype} tensor of at least {elems} elements")
            return self._dev(t, what)

        if ballots is not None and ballots.dtype != _torch_dtype(plan.ballot_dtype):
            raise ValueError("ballots dtype differs from the plan's")
        bp = None if ballots is None else self._dev(ballots, "ballots")
        rc = self._lib.schulze_batch_run(
            self._h, self._stream(), plan._h, bp, ptr(d, "d", torch.int32, plan.d_elems),
            ptr(p, "p", torch.int32, plan.d_elems), ptr(is_winner, "is_winner", torch.uint8, plan.vec_elems),
            ptr(n_winners, "n_winners", torch.int32, plan.E), ptr(beaten_by, "beaten_by", torch.int32, plan.vec_elems),
            ptr(order, "order", torch.int32, plan.vec_elems), ptr(level, "level", torch.int32, plan.vec_elems),
            BATCH_GRAPH if graph else 0)
        _check(rc, "schulze_batch_run")

    def batch_set_closure(self, value_bits: int, m_lo: int, m_hi: int, variant) -> None:
        v = CLOSURE_VARIANTS[variant] if isinstance(variant, str) else int(variant)
        _check(self._lib.schulze_batch_set_closure(self._h, value_bits, m_lo, m_hi, v), "schulze_batch_set_closure")

    def batch_get_closure(self, value_bits: int, m: int) -> str:
        v = ctypes.c_int32(0)
        _check(self._lib.schulze_batch_get_closure(self._h, value_bits, m, ctypes.byref(v)),
               "schulze_batch_get_closure")
        return {c: k for k, c in CLOSURE_VARIANTS.items()}[v.value]

    def batch_autotune(self, value_bits: int, m_max: int):
        """Time every closure schedule per bucket of 32 candidates up to m_max
        and keep the fastest; returns the (buckets, 4) millisecond table."""
        import numpy as np
        nb = (m_max + 31) // 32
        ms = (ctypes.c_float * (nb * 4))()
        _check(self._lib.schulze_batch_autotune(self._h, self._stream(), value_bits, m_max, ms),
               "schulze_batch_autotune")
        return np.array(ms[:], dtype=np.float32).reshape(nb, 4)

    def set_closure_schedule(self, schedule: str) -> None:
        """"auto" (one persistent launch) or "phased" (three launches per round)."""
        code = {"auto": SCHEDULE_AUTO, "phased": SCHEDULE_PHASED}[schedule]
        _check(self._lib.schulze_set_closure_schedule(self._h, code), "schulze_set_closure_schedule")

    def set_closure_tile(self, tile: int) -> None:
        """Closure tile size: 0 (by value width and m), 64 or 128."""
        _check(self._lib.schulze_set_closure_tile(self._h, int(tile)), "schulze_set_closure_tile")

    def set_sparse_count(self, mode: str) -> None:
        """Truncated ballots over many candidates: "bucketed" (default) or "atomic"."""
        code = {"bucketed": 0, "atomic": 1}[mode]
        _check(self._lib.schulze_set_sparse_count(self._h, code), "schulze_set_sparse_count")

    def set_value_ranking(self, enable: bool) -> None:
        """Run int32 closures of m >= 1024 on value ranks in uint16 when the values fit (default on)."""
        _check(self._lib.schulze_set_value_ranking(self._h, int(bool(enable))), "schulze_set_value_ranking")

    def set_sweep_limits(self, spin_limit: int = 0, max_sweeps: int = 0) -> None:
        """Limits of the frontier sweeps' bounded waits (0: defaults); for tests of the failure paths."""
        _check(self._lib.schulze_set_sweep_limits(self._h, int(spin_limit), int(max_sweeps)),
               "schulze_set_sweep_limits")

    def set_proposer(self, proposer: str) -> None:
        """First proposal of winners_learned: "network" (default), "borda", "copeland" or "filter+borda"."""
        code = PROPOSERS[proposer]
        _check(self._lib.schulze_set_proposer(self._h, code), "schulze_set_proposer")

    def closure_value_bits(self) -> int:
        """Value width (16 or 32) the last closure ran its recurrence in; 0 if none ran (synchronises)."""
        v = ctypes.c_int32(0)
        _check(self._lib.schulze_closure_value_bits(self._h, self._stream(), ctypes.byref(v)),
               "schulze_closure_value_bits")
        return v.value

    # -------------------------------------------------------------- timing
    def valu_probe(self, workgroups: int, trips: int) -> int:
        """Launch the integer VALU throughput probe on the current stream;
        returns the lane operations it issues (time it with events)."""
        import torch
        out = torch.zeros(1, dtype=torch.int32, device=self._torch_device)
        n = ctypes.c_int64(0)
        _check(self._lib.schulze_valu_probe(self._h, self._stream(), int(workgroups), int(trips),
                                            self._dev(out, "out"), ctypes.byref(n)), "schulze_valu_probe")
        return n.value

    def set_timing(self, enable: bool) -> None:
        _check(self._lib.schulze_set_timing(self._h, int(bool(enable))), "schulze_set_timing")

    def reset_timing(self) -> None:
        _check(self._lib.schulze_reset_timing(self._h), "schulze_reset_timing")

    def kernel_time(self, name: str):
        """(launches, total milliseconds) for a kernel since the last reset."""
        n = ctypes.c_int64(0)
        ms = ctypes.c_double(0.0)
        _check(self._lib.schulze_kernel_time(self._h, name.encode(), ctypes.byref(n), ctypes.byref(ms)),
               "schulze_kernel_time")
        return n.value, ms.value


class BatchPlan:
    """A planned batch (owns the plan's device memory until destroyed)."""

    def __init__(self, ctx, handle, E, ballot_dtype, d_elems, vec_elems):
        self._ctx = ctx
        self._h = handle
        self.E = E
        self.ballot_dtype = ballot_dtype
        self.d_elems = d_elems
        self.vec_elems = vec_elems

    def destroy(self) -> None:
        if getattr(self, "_h", None):
            self._ctx._lib.schulze_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
