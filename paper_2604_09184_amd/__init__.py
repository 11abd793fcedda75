"""Python binding of libnbody.so, the MI355X library for the hot path of the hybrid symplectic
planetesimal integrator (changeover-weighted all-pairs kick, close-encounter detection, Kepler
drift and momentum jump in democratic heliocentric coordinates).

Argument marshalling only: every step runs in the library's HIP kernels. Tensors are float64
CUDA (HIP) tensors of shape (n, 4), contiguous: xm = [x, y, z, m], v = [vx, vy, vz, pad],
thr = [rc, H, V, T]. Work goes to torch's current stream. The binding raises if the library is
not built; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import warnings

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnbody.so")

PREC_F64 = 0
PREC_SPLIT = 1

RESERVE_KICK = 1
RESERVE_LIST = 2
RESERVE_CE = 4


class NBodyError(RuntimeError):
    pass


class NBodyWarning(RuntimeWarning):
    """A call finished, but part of its result is not the method's: a close-encounter group too
    large for the direct integrator (moved on Kepler orbits only), an integration that did not
    finish, or an encounter list longer than the hybrid step's internal capacity."""


class _Params(ctypes.Structure):
    _fields_ = [("G", ctypes.c_double), ("m0", ctypes.c_double), ("dt", ctypes.c_double),
                ("n1", ctypes.c_double), ("n2", ctypes.c_double), ("f_in", ctypes.c_double),
                ("precision", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Collisions(ctypes.Structure):
    """nbody_collisions: collisions as perfect mergers in the close-encounter drift."""
    _fields_ = [("radius", ctypes.c_void_p), ("f", ctypes.c_double), ("merges", ctypes.c_void_p),
                ("time", ctypes.c_void_p), ("cap", ctypes.c_int64), ("count", ctypes.c_void_p)]


class Levels(ctypes.Structure):
    """nbody_levels: intermediate changeover levels of the hybrid step."""
    _fields_ = [("levels", ctypes.c_int32), ("substeps", ctypes.c_int32), ("margin", ctypes.c_double)]


@dataclasses.dataclass
class Params:
    G: float = 1.0
    m0: float = 1.0
    dt: float = 6.0 * 0.01720209895
    n1: float = 3.0
    n2: float = 0.4
    f_in: float = 0.1
    precision: int = PREC_F64

    def c(self):
        return _Params(self.G, self.m0, self.dt, self.n1, self.n2, self.f_in, self.precision, 0)


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_D = ctypes.c_double
_I32 = ctypes.c_int32

# name -> argument types after the context pointer
EXPORTS = {
    "nbody_reserve": [_I64, ctypes.c_uint32, _P],
    "nbody_rcrit": [_I64, _P, _P, _P, _P],
    "nbody_kick": [_I64, _P, _P, _P, _D, _P, _P, _P],
    "nbody_kick_noalloc": [_I64, _P, _P, _P, _D, _P, _P, _P],
    "nbody_encounters": [_I64, _P, _P, _P, _I64, _P, _P],
    "nbody_jump": [_I64, _P, _P, _D, _P],
    "nbody_drift": [_I64, _P, _P, _D, _P, _P],
    "nbody_step": [_I64, _P, _P, _P, _I32, _P, _I64, _P, _P, _P],
    "nbody_validate": [_I64, _P, _P, _P, _P],
    "nbody_encounter_groups": [_I64, _P, _I64, _P, _P, _P, _P],
    "nbody_drift_groups": [_I64, _P, _P, _P, _P, _D, _P, _P, _P],
    "nbody_step_hybrid": [_I64, _P, _P, _P, _I32, _P, _P, _P, _P],
    "nbody_energy": [_I64, _P, _P, _P, _P, _P],
    "nbody_bench_pairs": [_I64, _P, _P, _I32, _P, _P],
    "nbody_kick_vjp": [_I64, _P, _P, _D, _P, _P, _P],
    "nbody_jump_vjp": [_I64, _P, _P, _D, _P, _P, _P],
    "nbody_drift_vjp": [_I64, _P, _P, _D, _P, _P, _P],
    "nbody_step_vjp": [_I64, _P, _P, _P, _I32, _P, _P, _P],
    "nbody_step_batched": [_I32, _P, _P, _P, _I32, _P, _P],
    "nbody_autotune_batched": [_I32, _P, _P, _P, _I32, _P],
    "nbody_autotune_step": [_I64, _P, _P, _I32, _P, _P],
    "nbody_step_auto": [_I64, _P, _P, _I32, _P],
    "nbody_get_batched_tiles": [_P, _I32],
    "nbody_set_batched_tiles": [_P, _I32],
}
OTHER_EXPORTS = ["nbody_create", "nbody_destroy", "nbody_set_params", "nbody_last_error",
                 "nbody_version", "nbody_tune"]

_lib = None


def lib():
    """Loads libnbody.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise NBodyError(f"{LIB_PATH} is missing: build it with paper_2604_09184_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    L.nbody_create.restype = ctypes.c_int
    L.nbody_create.argtypes = [ctypes.POINTER(_P), ctypes.POINTER(_Params)]
    L.nbody_destroy.argtypes = [_P]
    L.nbody_set_params.argtypes = [_P, ctypes.POINTER(_Params)]
    L.nbody_last_error.restype = ctypes.c_char_p
    L.nbody_last_error.argtypes = [_P]
    L.nbody_version.restype = ctypes.c_char_p
    L.nbody_tune.restype = ctypes.c_int
    L.nbody_tune.argtypes = [_P, ctypes.c_char_p, _I64]
    for name, args in EXPORTS.items():
        f = getattr(L, name)
        f.restype = ctypes.c_int
        f.argtypes = [_P] + args
    _lib = L
    return L


def _ptr(t):
    return None if t is None else t.data_ptr()


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _body(t, name):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float64 and t.dim() == 2 and t.shape[1] == 4
            and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor of shape (n, 4)")
    return t


class Context:
    """Owns an nbody_ctx (parameters, workspace). Calls on one context must not overlap."""

    def __init__(self, params: Params | None = None):
        self.params = params or Params()
        self._h = _P()
        rc = lib().nbody_create(ctypes.byref(self._h), ctypes.byref(self.params.c()))
        if rc != 0:
            raise NBodyError(f"nbody_create failed ({rc})")

    def close(self):
        if self._h:
            lib().nbody_destroy(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params: Params):
        self.params = params
        self._check(lib().nbody_set_params(self._h, ctypes.byref(params.c())), "nbody_set_params")

    def tune(self, name, value):
        """Launch-shape knobs: locality_min_n, locality_every, emit_slots, target_waves."""
        self._check(lib().nbody_tune(self._h, name.encode(), int(value)), "nbody_tune")

    def _check(self, rc, name):
        if rc != 0:
            msg = lib().nbody_last_error(self._h)
            raise NBodyError(f"{name} failed ({rc}): {msg.decode() if msg else ''}")

    # ------------------------------------------------------------ entry points
    def reserve(self, n, what=RESERVE_KICK | RESERVE_LIST):
        """Sizes the context's workspace for n bodies in advance (synchronizes the stream)."""
        self._check(lib().nbody_reserve(self._h, int(n), int(what), _stream()), "nbody_reserve")

    def rcrit(self, xm, v, thr=None):
        _body(xm, "xm"); _body(v, "v")
        if thr is None:
            thr = torch.empty_like(xm)
        _body(thr, "thr")
        self._check(lib().nbody_rcrit(self._h, xm.shape[0], _ptr(xm), _ptr(v), _ptr(thr), _stream()),
                    "nbody_rcrit")
        return thr

    def kick(self, xm, thr, v=None, h=0.0, acc=None, acc_ce=None):
        for t, nm in ((xm, "xm"), (thr, "thr"), (v, "v"), (acc, "acc"), (acc_ce, "acc_ce")):
            _body(t, nm)
        self._check(lib().nbody_kick(self._h, xm.shape[0], _ptr(xm), _ptr(thr), _ptr(v), float(h),
                                     _ptr(acc), _ptr(acc_ce), _stream()), "nbody_kick")
        return acc

    def kick_noalloc(self, xm, thr, v=None, h=0.0, acc=None, acc_ce=None):
        """nbody_kick with the workspace in the library's per-device array (no allocation)."""
        for t, nm in ((xm, "xm"), (thr, "thr"), (v, "v"), (acc, "acc"), (acc_ce, "acc_ce")):
            _body(t, nm)
        self._check(lib().nbody_kick_noalloc(self._h, xm.shape[0], _ptr(xm), _ptr(thr), _ptr(v), float(h),
                                             _ptr(acc), _ptr(acc_ce), _stream()), "nbody_kick_noalloc")
        return acc

    def accelerations(self, xm, thr, with_ce=False):
        acc = torch.empty_like(xm)
        ce = torch.empty_like(xm) if with_ce else None
        self.kick(xm, thr, None, 0.0, acc, ce)
        return (acc, ce) if with_ce else acc

    def encounters(self, xm, thr, cap=None):
        """Returns (pairs (k, 2) int32 on the device, true count)."""
        _body(xm, "xm"); _body(thr, "thr")
        n = xm.shape[0]
        count = torch.zeros(1, dtype=torch.int64, device=xm.device)
        if cap is None:
            self._check(lib().nbody_encounters(self._h, n, _ptr(xm), _ptr(thr), None, 0, _ptr(count),
                                               _stream()), "nbody_encounters")
            cap = int(count.item())
        pairs = torch.empty((max(cap, 1), 2), dtype=torch.int32, device=xm.device)
        self._check(lib().nbody_encounters(self._h, n, _ptr(xm), _ptr(thr), _ptr(pairs), cap,
                                           _ptr(count), _stream()), "nbody_encounters")
        c = int(count.item())
        return pairs[:min(c, cap)], c

    def jump(self, xm, v, h):
        _body(xm, "xm"); _body(v, "v")
        self._check(lib().nbody_jump(self._h, xm.shape[0], _ptr(xm), _ptr(v), float(h), _stream()),
                    "nbody_jump")

    def drift(self, xm, v, h, status=None):
        _body(xm, "xm"); _body(v, "v")
        self._check(lib().nbody_drift(self._h, xm.shape[0], _ptr(xm), _ptr(v), float(h), _ptr(status),
                                      _stream()), "nbody_drift")
        return status

    def step(self, xm, v, nsteps, thr=None, pairs_cap=None, step_counts=False, out=None):
        """nsteps steps in place. With pairs_cap, also returns the final encounter list (pairs, count).
        With step_counts, also returns the int64 tensor of close-pair counts at the nsteps + 1 force
        evaluations. Returns None, (pairs, count), counts or ((pairs, count), counts).
        out = (pairs int32 (cap, 2), count int64 (1,)) device tensors to write the list into, in place
        of pairs_cap: the call then enqueues its work without creating tensors or waiting, and
        returns None (read count when the stream has finished)."""
        _body(xm, "xm"); _body(v, "v"); _body(thr, "thr")
        n = xm.shape[0]
        if out is not None:
            pairs, count = out
            if pairs.dtype != torch.int32 or pairs.dim() != 2 or pairs.shape[1] != 2 or not pairs.is_contiguous():
                raise NBodyError("out pairs must be a contiguous int32 (cap, 2) tensor")
            if count.dtype != torch.int64 or count.numel() < 1:
                raise NBodyError("out count must be an int64 tensor")
            self._check(lib().nbody_step(self._h, n, _ptr(xm), _ptr(v), _ptr(thr), int(nsteps), _ptr(pairs),
                                         pairs.shape[0], _ptr(count), None, _stream()), "nbody_step")
            return None
        sc = torch.zeros(int(nsteps) + 1, dtype=torch.int64, device=xm.device) if step_counts else None
        if pairs_cap is None:
            self._check(lib().nbody_step(self._h, n, _ptr(xm), _ptr(v), _ptr(thr), int(nsteps), None, 0,
                                         None, _ptr(sc), _stream()), "nbody_step")
            return sc
        count = torch.zeros(1, dtype=torch.int64, device=xm.device)
        pairs = torch.empty((max(pairs_cap, 1), 2), dtype=torch.int32, device=xm.device)
        self._check(lib().nbody_step(self._h, n, _ptr(xm), _ptr(v), _ptr(thr), int(nsteps), _ptr(pairs),
                                     pairs_cap, _ptr(count), _ptr(sc), _stream()), "nbody_step")
        c = int(count.item())
        res = (pairs[:min(c, pairs_cap)], c)
        return (res, sc) if step_counts else res

    def encounter_groups(self, n, pairs, count):
        """Close-encounter groups of an encounter list: (labels int32 [n] on the device, number
        of groups with at least two bodies, number of ignored pairs). pairs: int32 (cap, 2) device
        tensor; count: the true pair count, a device int64 tensor (or a host int)."""
        if pairs.dtype != torch.int32 or pairs.dim() != 2 or pairs.shape[1] != 2 or not pairs.is_contiguous():
            raise NBodyError("pairs must be a contiguous int32 (cap, 2) tensor")
        if not torch.is_tensor(count):
            count = torch.tensor([int(count)], dtype=torch.int64, device=pairs.device)
        labels = torch.empty(int(n), dtype=torch.int32, device=pairs.device)
        out = torch.empty(2, dtype=torch.int64, device=pairs.device)
        self._check(lib().nbody_encounter_groups(self._h, int(n), _ptr(pairs), pairs.shape[0], _ptr(count),
                                                 _ptr(labels), _ptr(out), _stream()), "nbody_encounter_groups")
        o = out.cpu().tolist()
        return labels, int(o[0]), int(o[1])

    _CE_STATS = ("groups", "largest", "bodies", "too_large", "unfinished", "list_overflows")

    @staticmethod
    def _collisions(radius, f, cap, device):
        """The nbody_collisions block for radius (or None) and its log buffers."""
        if radius is None:
            return None, None
        if radius.dtype != torch.float64 or not radius.is_contiguous():
            raise NBodyError("radius must be a contiguous float64 tensor")
        log = {"merges": torch.zeros((max(cap, 1), 3), dtype=torch.int32, device=device),
               "time": torch.zeros(max(cap, 1), dtype=torch.float64, device=device),
               "count": torch.zeros(1, dtype=torch.int64, device=device), "cap": int(cap)}
        col = Collisions(_ptr(radius), float(f), _ptr(log["merges"]), _ptr(log["time"]), int(cap),
                         _ptr(log["count"]))
        return col, log

    def _ce_result(self, stats, log):
        out = dict(zip(self._CE_STATS, stats.cpu().tolist()))
        if out["too_large"]:
            warnings.warn(f"{out['too_large']} close-encounter group(s) above 64 bodies moved on Kepler orbits "
                          f"only (largest {out['largest']}); intermediate changeover levels (levels > 0) "
                          f"split such groups", NBodyWarning, stacklevel=3)
        if out["unfinished"]:
            warnings.warn(f"{out['unfinished']} close-encounter integration(s) did not finish", NBodyWarning,
                          stacklevel=3)
        if out["list_overflows"]:
            warnings.warn(f"{out['list_overflows']} encounter list(s) exceeded the hybrid step's capacity of "
                          f"max(16 n, 65536) pairs: groups were built from a truncated list", NBodyWarning,
                          stacklevel=3)
        if log is not None:
            cnt = int(log["count"].item())
            k = min(cnt, log["cap"])
            out["mergers"] = cnt
            out["merges"] = log["merges"][:k].cpu().numpy()
            out["merge_times"] = log["time"][:k].cpu().numpy()
        return out

    def drift_groups(self, xm, v, thr, labels, h, radius=None, f=1.0, cap=4096):
        """Close-encounter drift (H_A in full) over h with the given group labels; with radius
        (float64 [n], in/out), bodies of a group closer than f (R_i + R_j) merge. Returns the
        statistics as a dict (with the merger log when colliding)."""
        _body(xm, "xm"); _body(v, "v"); _body(thr, "thr")
        stats = torch.zeros(6, dtype=torch.int64, device=xm.device)
        col, log = self._collisions(radius, f, cap, xm.device)
        self._check(lib().nbody_drift_groups(self._h, xm.shape[0], _ptr(xm), _ptr(v), _ptr(thr),
                                             _ptr(labels.contiguous()), float(h),
                                             ctypes.byref(col) if col else None, _ptr(stats), _stream()),
                    "nbody_drift_groups")
        return self._ce_result(stats, log)

    def step_hybrid(self, xm, v, nsteps, thr=None, radius=None, f=1.0, cap=4096, levels=0, substeps=8,
                    margin=0.5):
        """nsteps hybrid steps in place (close-encounter groups integrated in the drift); with
        levels > 0, the drift of the bodies with close partners runs through that many
        intermediate changeover levels (time steps dt / substeps^l), the close pairs listed at
        (1 + margin) rc; with radius (float64 [n],
        in/out), collisions merge bodies. Returns the statistics as a dict (with the merger log
        when colliding)."""
        _body(xm, "xm"); _body(v, "v"); _body(thr, "thr")
        stats = torch.zeros(6, dtype=torch.int64, device=xm.device)
        col, log = self._collisions(radius, f, cap, xm.device)
        lv = Levels(int(levels), int(substeps), float(margin))
        self._check(lib().nbody_step_hybrid(self._h, xm.shape[0], _ptr(xm), _ptr(v), _ptr(thr), int(nsteps),
                                            ctypes.byref(lv), ctypes.byref(col) if col else None, _ptr(stats),
                                            _stream()), "nbody_step_hybrid")
        return self._ce_result(stats, log)

    def validate(self, xm, v):
        """(index, reason) of the first invalid body, or (-1, 0); reasons: 1 non-finite value,
        2 negative mass, 3 at the central mass, 4 same position as a later body."""
        _body(xm, "xm"); _body(v, "v")
        out = torch.empty(2, dtype=torch.int64, device=xm.device)
        self._check(lib().nbody_validate(self._h, xm.shape[0], _ptr(xm), _ptr(v), _ptr(out), _stream()),
                    "nbody_validate")
        o = out.cpu().tolist()
        return int(o[0]), int(o[1])

    def energy(self, xm, v, thr):
        out = torch.empty(8, dtype=torch.float64, device=xm.device)
        self._check(lib().nbody_energy(self._h, xm.shape[0], _ptr(xm), _ptr(v), _ptr(thr), _ptr(out),
                                       _stream()), "nbody_energy")
        o = out.cpu().numpy()
        return {"E": o[0], "Eprime": o[1], "L": o[2:5].copy(), "P": o[5:8].copy()}


    def bench_pairs(self, xm, thr, reps=10):
        """Mean duration (ms) of one pair-kernel launch, timed with HIP events on the stream."""
        _body(xm, "xm"); _body(thr, "thr")
        ms = ctypes.c_double()
        self._check(lib().nbody_bench_pairs(self._h, xm.shape[0], _ptr(xm), _ptr(thr), int(reps),
                                            ctypes.byref(ms), _stream()), "nbody_bench_pairs")
        return ms.value


    # ------------------------------------------------------------ reverse mode
    def kick_vjp(self, xm, thr, h, lam_v, lam_x):
        for t, nm in ((xm, "xm"), (thr, "thr"), (lam_v, "lam_v"), (lam_x, "lam_x")):
            _body(t, nm)
        self._check(lib().nbody_kick_vjp(self._h, xm.shape[0], _ptr(xm), _ptr(thr), float(h), _ptr(lam_v),
                                         _ptr(lam_x), _stream()), "nbody_kick_vjp")

    def jump_vjp(self, xm, v, h, lam_x, lam_v):
        for t, nm in ((xm, "xm"), (v, "v"), (lam_x, "lam_x"), (lam_v, "lam_v")):
            _body(t, nm)
        self._check(lib().nbody_jump_vjp(self._h, xm.shape[0], _ptr(xm), _ptr(v), float(h), _ptr(lam_x),
                                         _ptr(lam_v), _stream()), "nbody_jump_vjp")

    def drift_vjp(self, xm, v, h, lam_x, lam_v):
        for t, nm in ((xm, "xm"), (v, "v"), (lam_x, "lam_x"), (lam_v, "lam_v")):
            _body(t, nm)
        self._check(lib().nbody_drift_vjp(self._h, xm.shape[0], _ptr(xm), _ptr(v), float(h), _ptr(lam_x),
                                          _ptr(lam_v), _stream()), "nbody_drift_vjp")

    def step_vjp(self, xm0, v0, thr, nsteps, lam_x, lam_v):
        for t, nm in ((xm0, "xm0"), (v0, "v0"), (thr, "thr"), (lam_x, "lam_x"), (lam_v, "lam_v")):
            _body(t, nm)
        self._check(lib().nbody_step_vjp(self._h, xm0.shape[0], _ptr(xm0), _ptr(v0), _ptr(thr), int(nsteps),
                                         _ptr(lam_x), _ptr(lam_v), _stream()), "nbody_step_vjp")


    # ------------------------------------------------------------ batched ensembles
    @staticmethod
    def _offs(offs):
        import numpy as np
        o = np.ascontiguousarray(offs, dtype=np.int64)
        return o, o.ctypes.data

    def step_batched(self, offs, xm, v, nsteps, count_pairs=False):
        """Advances every system in place; offs is a host int64 sequence of length nsys + 1."""
        _body(xm, "xm"); _body(v, "v")
        o, op = self._offs(offs)
        nsys = len(o) - 1
        npairs = torch.zeros(nsys, dtype=torch.int64, device=xm.device) if count_pairs else None
        self._check(lib().nbody_step_batched(self._h, nsys, op, _ptr(xm), _ptr(v), int(nsteps), _ptr(npairs),
                                             _stream()), "nbody_step_batched")
        return npairs

    def autotune_batched(self, offs, xm, v, nsteps=10):
        _body(xm, "xm"); _body(v, "v")
        o, op = self._offs(offs)
        self._check(lib().nbody_autotune_batched(self._h, len(o) - 1, op, _ptr(xm), _ptr(v), int(nsteps),
                                                 _stream()), "nbody_autotune_batched")
        return self.batched_tiles()

    def autotune_step(self, xm, v, ntrial=20):
        """Times nbody_step's per-step launches against one persistent launch for this system size
        (on copies) and records the faster; returns the path (0 per-step, 1/2 persistent)."""
        _body(xm, "xm"); _body(v, "v")
        ch = ctypes.c_int32(-1)
        self._check(lib().nbody_autotune_step(self._h, xm.shape[0], _ptr(xm), _ptr(v), int(ntrial),
                                              ctypes.byref(ch), _stream()), "nbody_autotune_step")
        return ch.value

    def step_auto(self, xm, v, nsteps):
        """nsteps steps in place with the path recorded by autotune_step for this size."""
        _body(xm, "xm"); _body(v, "v")
        self._check(lib().nbody_step_auto(self._h, xm.shape[0], _ptr(xm), _ptr(v), int(nsteps), _stream()),
                    "nbody_step_auto")

    def batched_tiles(self):
        t = (ctypes.c_int32 * 6)()
        n = lib().nbody_get_batched_tiles(self._h, t, 6)
        if n < 0:
            raise NBodyError("nbody_get_batched_tiles failed")
        return list(t)[:n]

    def set_batched_tiles(self, tiles):
        t = (ctypes.c_int32 * len(tiles))(*tiles)
        self._check(lib().nbody_set_batched_tiles(self._h, t, len(tiles)), "nbody_set_batched_tiles")


def version():
    return lib().nbody_version().decode()
