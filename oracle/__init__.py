"""Python access to the CPU oracle (oracle.cpp).

TEST INFRASTRUCTURE ONLY: the plain, slow reference of the hybrid-symplectic step that the HIP
library is checked against. Only tests, the smoke check and the benchmark's CPU baseline use it;
the library never imports it. Arrays are float64 numpy arrays with positions/velocities as
(n, 3) and masses as (n,); parameters are a dict with G, m0, dt, n1, n2, f_in.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.cpp")

BUILD_CMD = ["g++", "-O2", "-mfma", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
             "-o", _SO, _SRC, "-lquadmath"]


def build():
    subprocess.run(BUILD_CMD, check=True)


def _lib():
    global _L
    try:
        return _L
    except NameError:
        pass
    if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        build()
    L = ctypes.CDLL(_SO)
    P = ctypes.c_void_p
    I = ctypes.c_int64
    D = ctypes.c_double
    sig = {
        "or_thresholds": (None, [I, P, P, P, P, P, P, P]),
        "or_changeover": (None, [D, P, P]),
        "or_changeover_q": (None, [D, P, P]),
        "or_kick_acc": (None, [I, P, P, P, P, P, P, P, P, P]),
        "or_kick_acc_ld": (None, [I, P, P, P, P, P, P, P]),
        "or_kick_acc_q": (None, [I, P, P, P, P, P, P, P]),
        "or_kick_acc_rows": (None, [I, P, P, P, P, P, P, I, P, P, P]),
        "or_encounters": (I, [I, P, P, P, I, P]),
        "or_groups": (I, [I, P, I, P, P]),
        "or_ce_drift_group": (ctypes.c_int, [P, ctypes.c_int, P, P, P, P, P, D, D]),
        "or_step_hybrid": (ctypes.c_int, [I, P, P, P, P, ctypes.c_int, P, P, P, D, P]),
        "or_drift_groups": (ctypes.c_int, [I, P, P, P, P, P, P, D, D, P]),
        "or_drift_groups_merge": (ctypes.c_int, [I, P, P, P, P, P, P, D, D, P, P, D, ctypes.c_int, P, P, I, P]),
        "or_step_merge": (ctypes.c_int, [I, P, P, P, P, ctypes.c_int, P, P, P, D, P, P, D, P, P, I, P]),
        "or_level_kick_acc": (None, [I, P, P, P, I, P, ctypes.c_int, P, P]),
        "or_ce_drift_group_levels": (ctypes.c_int, [P, ctypes.c_int, P, P, P, P, ctypes.c_int, P, D, D]),
        "or_drift_levels": (ctypes.c_int, [I, P, P, P, P, I, P, P, P, ctypes.c_int, ctypes.c_int, P, D, D]),
        "or_step_levels": (ctypes.c_int, [I, P, P, P, P, ctypes.c_int, P, P, P, D, P, ctypes.c_int, ctypes.c_int,
                                          P, D, P, P, I, P, D]),
        "or_jump": (None, [I, P, P, P, P, D]),
        "or_drift": (ctypes.c_int, [I, P, P, P, D, P]),
        "or_drift_q": (ctypes.c_int, [I, P, P, P, D]),
        "or_step": (ctypes.c_int, [I, P, P, P, P, ctypes.c_int, P, P, P]),
        "or_step_jvp": (ctypes.c_int, [I, P, P, P, P, P, P, P, ctypes.c_int, P, P, P, P]),
        "or_energy": (None, [I, P, P, P, P, P, P, P, P]),
        "or_num_threads": (ctypes.c_int, []),
        "or_set_threads": (None, [ctypes.c_int]),
        "or_kick_jvp": (None, [I, P, P, P, P, P, P, P, P, P]),
        "or_drift_jvp": (None, [I, P, P, P, P, P, D, P, P]),
        "or_jump_jvp": (None, [I, P, P, P, P, P, P, P, D, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _L = L
    return L


def _p(a):
    return None if a is None else a.ctypes.data


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _prm(p):
    return np.array([p["G"], p["m0"], p["dt"], p["n1"], p["n2"], p["f_in"]], dtype=np.float64)


def num_threads():
    return _lib().or_num_threads()


def set_threads(k):
    """Number of OpenMP threads of the following oracle calls."""
    _lib().or_set_threads(int(k))


def thresholds(x, v, m, p):
    """rc, H, V per body (critical radius and exact-predicate thresholds)."""
    x = _f64(x); v = _f64(v); m = _f64(m)
    n = m.shape[0]
    rc, H, V = np.empty(n), np.empty(n), np.empty(n)
    _lib().or_thresholds(n, _p(x), _p(v), _p(m), _p(_prm(p)), _p(rc), _p(H), _p(V))
    return rc, H, V


def changeover(y, quad=False):
    K, d = ctypes.c_double(), ctypes.c_double()
    f = _lib().or_changeover_q if quad else _lib().or_changeover
    f(float(y), ctypes.byref(K), ctypes.byref(d))
    return K.value, d.value


def kick_acc(x, m, thr, p, precision="f64"):
    """H_B accelerations. Returns (acc, acc_ce, l1) for f64; acc only for 'ld' / 'quad'."""
    x = _f64(x); m = _f64(m)
    rc, H, V = (_f64(t) for t in thr)
    n = m.shape[0]
    acc = np.empty((n, 3))
    if precision == "f64":
        ce = np.empty((n, 3)); l1 = np.empty(n)
        _lib().or_kick_acc(n, _p(x), _p(m), _p(rc), _p(H), _p(V), _p(_prm(p)), _p(acc), _p(ce), _p(l1))
        return acc, ce, l1
    f = {"ld": _lib().or_kick_acc_ld, "quad": _lib().or_kick_acc_q}[precision]
    f(n, _p(x), _p(m), _p(rc), _p(H), _p(V), _p(_prm(p)), _p(acc))
    return acc


def kick_acc_rows(x, m, thr, p, rows):
    """Accelerations (and l1 scale) of the listed bodies only."""
    x = _f64(x); m = _f64(m)
    rc, H, V = (_f64(t) for t in thr)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    k = rows.shape[0]
    acc = np.empty((k, 3)); l1 = np.empty(k)
    _lib().or_kick_acc_rows(m.shape[0], _p(x), _p(m), _p(rc), _p(H), _p(V), _p(_prm(p)), k,
                            _p(rows), _p(acc), _p(l1))
    return acc, l1


def encounters(x, thr, cap=None):
    """Close pairs (i<j) sorted by (i, j) as an (count, 2) int32 array."""
    x = _f64(x)
    rc, H, V = (_f64(t) for t in thr)
    n = x.shape[0]
    if cap is None:
        cnt = _lib().or_encounters(n, _p(x), _p(H), _p(V), 0, None)
        cap = cnt
    pairs = np.empty((max(cap, 1), 2), dtype=np.int32)
    cnt = _lib().or_encounters(n, _p(x), _p(H), _p(V), cap, _p(pairs))
    return pairs[:min(cnt, cap)].copy()


def groups(n, pairs):
    """Close-encounter groups: (labels, ngroups, ignored); labels[i] = smallest index in i's
    connected component of the close-pair graph (breadth-first search, ascending start)."""
    pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
    lab = np.empty(n, dtype=np.int32)
    ign = ctypes.c_int64(0)
    g = _lib().or_groups(n, _p(pr), pr.shape[0], _p(lab), ctypes.byref(ign))
    return lab, int(g), int(ign.value)


def ce_drift_group(x, v, m, rc, p, idx, h, tol=1e-18):
    """Close-encounter drift of the group idx (H_A in full, Gragg-Bulirsch-Stoer in long double; at
    the default tolerance the result is within about 2e-15 of the exact flow on the 2048 disk);
    returns new copies of x, v and the status."""
    x = _f64(x).copy(); v = _f64(v).copy()
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    st = _lib().or_ce_drift_group(_p(idx), len(idx), _p(x), _p(v), _p(_f64(m)), _p(_f64(rc)), _p(_prm(p)),
                                  float(h), float(tol))
    return x, v, st


def drift_groups(x, v, m, rc, labels, p, h, tol=1e-18):
    """Drift of all bodies over h: close-encounter groups (labels) integrated in full, the other
    bodies on Kepler orbits; returns x, v, status, stats (groups, largest, bodies)."""
    x = _f64(x).copy(); v = _f64(v).copy()
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    stats = np.zeros(3, dtype=np.int64)
    st = _lib().or_drift_groups(len(lab), _p(x), _p(v), _p(_f64(m)), _p(_f64(rc)), _p(lab), _p(_prm(p)),
                                float(h), float(tol), _p(stats))
    return x, v, st, tuple(int(s) for s in stats)


def step_hybrid(x, v, m, p, nsteps, thr=None, tol=1e-18):
    """nsteps hybrid steps: the drift integrates every close-encounter group in full (H_A with its
    [1 - K] part); returns x, v, status, stats = (groups integrated, largest group, bodies)."""
    x = _f64(x).copy(); v = _f64(v).copy(); m = _f64(m)
    rc, H, V = (None, None, None) if thr is None else (_f64(t) for t in thr)
    stats = np.zeros(3, dtype=np.int64)
    st = _lib().or_step_hybrid(len(m), _p(x), _p(v), _p(m), _p(_prm(p)), int(nsteps), _p(rc), _p(H), _p(V),
                               float(tol), _p(stats))
    return x, v, st, tuple(int(s) for s in stats)


def _merge_log(merges, mtime, cnt):
    k = min(int(cnt), merges.shape[0])
    return merges[:k].copy(), mtime[:k].copy()


def drift_groups_merge(x, v, m, rc, R, f, labels, p, h, tol=1e-18, step=0, cap=4096):
    """drift_groups with collisions as perfect mergers: two bodies of a group merge when their
    distance falls below f (R_i + R_j), at the first contact time. Returns x, v, m, R, status,
    stats, merges {step, survivor, removed} and their times within the drift."""
    x = _f64(x).copy(); v = _f64(v).copy(); m = _f64(m).copy(); R = _f64(R).copy()
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    stats = np.zeros(3, dtype=np.int64)
    merges = np.zeros((cap, 3), dtype=np.int32); mtime = np.zeros(cap)
    cnt = ctypes.c_int64(0)
    st = _lib().or_drift_groups_merge(len(lab), _p(x), _p(v), _p(m), _p(_f64(rc)), _p(lab), _p(_prm(p)),
                                      float(h), float(tol), _p(stats), _p(R), float(f), int(step),
                                      _p(merges), _p(mtime), cap, ctypes.byref(cnt))
    mg, mt = _merge_log(merges, mtime, cnt.value)
    return x, v, m, R, st, tuple(int(s) for s in stats), mg, mt


def step_merge(x, v, m, R, f, p, nsteps, thr=None, tol=1e-18, cap=4096):
    """nsteps hybrid steps with collisions as perfect mergers (radius factor f). Returns x, v, m, R,
    status, stats, merges {step, survivor, removed} and their times within the step's drift."""
    x = _f64(x).copy(); v = _f64(v).copy(); m = _f64(m).copy(); R = _f64(R).copy()
    rc, H, V = (None, None, None) if thr is None else (_f64(t) for t in thr)
    stats = np.zeros(3, dtype=np.int64)
    merges = np.zeros((cap, 3), dtype=np.int32); mtime = np.zeros(cap)
    cnt = ctypes.c_int64(0)
    st = _lib().or_step_merge(len(m), _p(x), _p(v), _p(m), _p(_prm(p)), int(nsteps), _p(rc), _p(H), _p(V),
                              float(tol), _p(stats), _p(R), float(f), _p(merges), _p(mtime), cap,
                              ctypes.byref(cnt))
    mg, mt = _merge_log(merges, mtime, cnt.value)
    return x, v, m, R, st, tuple(int(s) for s in stats), mg, mt


def level_kick_acc(x, m, pairs, rc_levels, level, p):
    """Acceleration of the level-`level` kick over the listed pairs (rc_levels: [level + 1][n])."""
    x = _f64(x); m = _f64(m)
    pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
    rcl = np.ascontiguousarray(rc_levels, dtype=np.float64)
    acc = np.empty((len(m), 3))
    _lib().or_level_kick_acc(len(m), _p(x), _p(m), _p(pr), pr.shape[0], _p(rcl), int(level), _p(_prm(p)), _p(acc))
    return acc


def ce_drift_group_levels(x, v, m, rc_levels, p, idx, h, tol=1e-18):
    """Close-encounter drift of the group idx with the pair term weighted by prod_l [1 - K_l]
    (rc_levels: [nl][n]); returns new copies of x, v and the status."""
    x = _f64(x).copy(); v = _f64(v).copy()
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    rcl = np.ascontiguousarray(np.asarray(rc_levels, dtype=np.float64)[:, idx])
    st = _lib().or_ce_drift_group_levels(_p(idx), len(idx), _p(x), _p(v), _p(_f64(m)), _p(rcl), rcl.shape[0],
                                         _p(_prm(p)), float(h), float(tol))
    return x, v, st


def drift_levels(x, v, m, pairs, thr_levels, p, levels, substeps, h, tol=1e-18):
    """The drift A(h) alone through `levels` intermediate levels; thr_levels = (rc, H, V), each
    [levels + 1][n]; pairs: the step's close pairs. Returns x, v, status."""
    x = _f64(x).copy(); v = _f64(v).copy()
    pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
    rc, H, V = (np.ascontiguousarray(t, dtype=np.float64) for t in thr_levels)
    st = _lib().or_drift_levels(len(m), _p(x), _p(v), _p(_f64(m)), _p(pr), pr.shape[0], _p(rc), _p(H), _p(V),
                                int(levels), int(substeps), _p(_prm(p)), float(h), float(tol))
    return x, v, st


def step_levels(x, v, m, p, nsteps, levels, substeps, thr=None, tol=1e-18, R=None, f=0.0, cap=4096, margin=0.0):
    """nsteps hybrid steps whose close-encounter drift runs through `levels` intermediate changeover
    levels (time steps dt / substeps^l), the step's close pairs listed at (1 + margin) rc; with R,
    collisions merge bodies. Returns x, v, m, R, status, stats, merges and their times."""
    x = _f64(x).copy(); v = _f64(v).copy(); m = _f64(m).copy()
    R = None if R is None else _f64(R).copy()
    rc, H, V = (None, None, None) if thr is None else (_f64(t) for t in thr)
    stats = np.zeros(3, dtype=np.int64)
    merges = np.zeros((cap, 3), dtype=np.int32); mtime = np.zeros(cap)
    cnt = ctypes.c_int64(0)
    st = _lib().or_step_levels(len(m), _p(x), _p(v), _p(m), _p(_prm(p)), int(nsteps), _p(rc), _p(H), _p(V),
                               float(tol), _p(stats), int(levels), int(substeps), _p(R), float(f), _p(merges),
                               _p(mtime), cap, ctypes.byref(cnt), float(margin))
    if st < 0:
        raise ValueError("levels must be 0..4 and substeps >= 1")
    mg, mt = _merge_log(merges, mtime, cnt.value)
    return x, v, m, R, st, tuple(int(s) for s in stats), mg, mt


def jump(x, v, m, p, h):
    x = _f64(x).copy(); v = _f64(v); m = _f64(m)
    _lib().or_jump(m.shape[0], _p(x), _p(v), _p(m), _p(_prm(p)), h)
    return x


def drift(x, v, p, h, quad=False):
    x = _f64(x).copy(); v = _f64(v).copy()
    n = x.shape[0]
    if quad:
        st = _lib().or_drift_q(n, _p(x), _p(v), _p(_prm(p)), h)
        return x, v, st
    status = np.zeros(n, dtype=np.uint32)
    _lib().or_drift(n, _p(x), _p(v), _p(_prm(p)), h, _p(status))
    return x, v, status


def step(x, v, m, p, nsteps, thr=None):
    """nsteps full steps; thresholds from the initial state unless given."""
    x = _f64(x).copy(); v = _f64(v).copy(); m = _f64(m)
    if thr is None:
        rc = H = V = None
    else:
        rc, H, V = (_f64(t) for t in thr)
    st = _lib().or_step(m.shape[0], _p(x), _p(v), _p(m), _p(_prm(p)), nsteps, _p(rc), _p(H), _p(V))
    return x, v, st


def step_jvp(x, v, m, p, nsteps, dx=None, dv=None, dm=None):
    x = _f64(x); v = _f64(v); m = _f64(m)
    n = m.shape[0]
    xo, vo, dxo, dvo = (np.empty((n, 3)) for _ in range(4))
    dx = None if dx is None else _f64(dx)
    dv = None if dv is None else _f64(dv)
    dm = None if dm is None else _f64(dm)
    st = _lib().or_step_jvp(n, _p(x), _p(v), _p(m), _p(dx), _p(dv), _p(dm), _p(_prm(p)), nsteps,
                            _p(xo), _p(vo), _p(dxo), _p(dvo))
    return xo, vo, dxo, dvo, st


def kick_jvp(x, m, thr, p, dx, dm):
    """Directional derivative of the H_B accelerations (thresholds fixed)."""
    x = _f64(x); m = _f64(m); dx = _f64(dx); dm = _f64(dm)
    rc, H, V = (_f64(t) for t in thr)
    n = m.shape[0]
    out = np.empty((n, 3))
    _lib().or_kick_jvp(n, _p(x), _p(m), _p(dx), _p(dm), _p(rc), _p(H), _p(V), _p(_prm(p)), _p(out))
    return out


def drift_jvp(x, v, p, h, dx, dv):
    x = _f64(x); v = _f64(v); dx = _f64(dx); dv = _f64(dv)
    n = x.shape[0]
    ox, ov = np.empty((n, 3)), np.empty((n, 3))
    _lib().or_drift_jvp(n, _p(x), _p(v), _p(dx), _p(dv), _p(_prm(p)), h, _p(ox), _p(ov))
    return ox, ov


def jump_jvp(x, v, m, p, h, dx, dv, dm):
    x = _f64(x); v = _f64(v); m = _f64(m); dx = _f64(dx); dv = _f64(dv); dm = _f64(dm)
    n = m.shape[0]
    out = np.empty((n, 3))
    _lib().or_jump_jvp(n, _p(x), _p(v), _p(m), _p(dx), _p(dv), _p(dm), _p(_prm(p)), h, _p(out))
    return out


def energy(x, v, m, p, thr):
    """dict E, Eprime, L (3,), P (3,)."""
    x = _f64(x); v = _f64(v); m = _f64(m)
    rc, H, V = (_f64(t) for t in thr)
    out = np.empty(8)
    _lib().or_energy(m.shape[0], _p(x), _p(v), _p(m), _p(_prm(p)), _p(rc), _p(H), _p(V), _p(out))
    return {"E": out[0], "Eprime": out[1], "L": out[2:5].copy(), "P": out[5:8].copy()}


def grad_loss_jvp(x, v, m, p, nsteps, target):
    """Gradient of L = sum |x(T) - target|^2 w.r.t. (x0, v0, m) by one JVP per input direction."""
    n = m.shape[0]
    gx = np.zeros((n, 3)); gv = np.zeros((n, 3)); gm = np.zeros(n)
    zero3 = np.zeros((n, 3)); zero1 = np.zeros(n)
    for kind in ("x", "v", "m"):
        for i in range(n):
            for c in (range(3) if kind != "m" else [0]):
                d3 = zero3.copy(); d1 = zero1.copy()
                if kind == "m":
                    d1[i] = 1.0
                else:
                    d3[i, c] = 1.0
                xo, vo, dxo, dvo, _ = step_jvp(x, v, m, p, nsteps,
                                               dx=d3 if kind == "x" else None,
                                               dv=d3 if kind == "v" else None,
                                               dm=d1 if kind == "m" else None)
                g = float(2.0 * ((xo - target) * dxo).sum())
                if kind == "x":
                    gx[i, c] = g
                elif kind == "v":
                    gv[i, c] = g
                else:
                    gm[i] = g
    return gx, gv, gm
