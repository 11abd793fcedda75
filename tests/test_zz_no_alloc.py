"""The allocation-free kick (nbody_kick_noalloc, workspace in the library's per-device array)
against nbody_kick, through the C ABI, on two calls in a row with the second smaller (the array
keeps the first call's contents), on equal and unequal masses, with the close-encounter part,
and the host-side rejection of a size beyond the array.

Bar (eq. Hb kick, binary64): every body's acceleration within 1e-12 of max(|a|, l1), l1 the
conditioning norm sum_j G m_j |w_ij| r_ij from the oracle; the two entry points may split the
j-range into different chunk counts, so their sums may differ in the last bits.
"""
import numpy as np
import pytest

import diskgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DEV = "cuda:0"


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def nb():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2604_09184_amd as nb
    nb.lib()
    return nb


@pytest.fixture(scope="module")
def ctx(nb):
    return nb.Context(nb.Params(**diskgen.PARAMS))


def case(nb, ctx, d, with_ce):
    p = diskgen.PARAMS
    xm, v4 = diskgen.pack4(d["x"], d["v"], d["m"])
    X = torch.tensor(xm, device=DEV)
    V0 = torch.tensor(v4, device=DEV)
    thr = ctx.rcrit(X, V0)
    n = X.shape[0]
    h = 0.5 * p["dt"]
    # the library's own kick, then the allocation-free one on fresh copies
    Va, Vb = V0.clone(), V0.clone()
    Aa, Ab = torch.empty_like(X), torch.empty_like(X)
    Ca = torch.empty_like(X) if with_ce else None
    Cb = torch.empty_like(X) if with_ce else None
    ctx.kick(X, thr, Va, h, Aa, Ca)
    ctx.kick_noalloc(X, thr, Vb, h, Ab, Cb)
    torch.cuda.synchronize()
    othr = oracle.thresholds(d["x"], d["v"], d["m"], p)
    _, _, l1 = oracle.kick_acc(d["x"], d["m"], othr, p)
    a, b = Aa.cpu().numpy()[:, :3], Ab.cpu().numpy()[:, :3]
    err = (np.abs(a - b).max(1) / np.maximum(np.abs(a).max(1), l1)).max()
    va, vb = Va.cpu().numpy()[:, :3], Vb.cpu().numpy()[:, :3]
    ev = (np.abs(va - vb).max(1) / np.linalg.norm(va, axis=1)).max()
    out = {"n": n, "acc": float(err), "v": float(ev)}
    if with_ce:
        ca, cb = Ca.cpu().numpy()[:, :3], Cb.cpu().numpy()[:, :3]
        out["ce"] = float((np.abs(ca - cb).max(1) / np.maximum(np.abs(a + ca).max(1), l1)).max())
    say(f"  {out}")
    assert err < 1e-12 and ev < 1e-14
    if with_ce:
        assert out["ce"] < 1e-12
    return out


def test_noalloc_kick_matches_the_kick_twice_second_smaller(nb, ctx):
    say("kick_noalloc: 32768 disk, then 2048 disk")
    case(nb, ctx, diskgen.workload("disk32768"), with_ce=False)
    case(nb, ctx, diskgen.workload("disk2048"), with_ce=False)


def test_noalloc_kick_unequal_masses_with_close_part(nb, ctx):
    say("kick_noalloc: power-law masses 4096 with acc_ce, then 1000 with acc_ce")
    for n, seed in ((4096, 1011), (1000, 1012)):
        d = diskgen.make_disk(diskgen.Disk(n, 0.5, 4.0, 0.01, 0.005, None, (2.5, 1e-4, 1e-2), seed=seed))
        case(nb, ctx, d, with_ce=True)


def test_noalloc_kick_rejects_sizes_beyond_its_workspace(nb, ctx):
    say("kick_noalloc: size beyond the array")
    n = 1200000
    X = torch.zeros((n, 4), dtype=torch.float64, device=DEV)
    with pytest.raises(nb.NBodyError, match="workspace"):
        ctx.kick_noalloc(X, X, None, 0.0, X, X)
