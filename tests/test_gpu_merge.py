"""GPU parity of collisions as perfect mergers inside the close-encounter drift, against the
oracle's long-double integration with the same merger rule (contact below f (R_i + R_j), first
contact time by bisection, merged at that time; the removed body parked massless far away).

Bars: the merger logs equal as sets of {step, survivor, removed}; merger times to the accuracy of
the states divided by the contact speed (stated per test); masses bit-exact (both sides add the same two binary64 masses); radii 1e-15
relative; states as for the hybrid step without collisions.
"""
import math

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


def dev_state(x, v, m):
    xm, v4 = diskgen.pack4(x, v, m)
    return torch.tensor(xm, device=DEV), torch.tensor(v4, device=DEV)


def sorted_log(mg):
    mg = np.asarray(mg).reshape(-1, 3)
    return mg[np.lexsort((mg[:, 2], mg[:, 1], mg[:, 0]))]


def test_merge_radial_infall_matches_oracle_and_closed_form(nb):
    """Two bodies falling radially onto each other (negligible central mass): the GPU merges them
    at the closed-form contact time, as the oracle does, into the centre-of-mass body."""
    say("merge radial infall")
    p = dict(diskgen.PARAMS, m0=1e-30)
    ctx = nb.Context(nb.Params(**p))
    m = np.array([3e-6, 1e-6]); R = np.array([6e-5, 4e-5]); f = 1.5
    r0 = 2e-3
    x = np.array([[1.0, 0.0, 0.0], [1.0 + r0, 0.0, 0.0]])
    v = np.array([[0.01, 0.02, 0.0], [0.01, 0.02, 0.0]])
    rc = np.array([5e-2, 5e-2])
    h = 0.1
    X, V = dev_state(x, v, m)
    thr = torch.zeros((2, 4), dtype=torch.float64, device=DEV)
    thr[:, 0] = torch.tensor(rc)
    Rd = torch.tensor(R, device=DEV)
    lab = torch.zeros(2, dtype=torch.int32, device=DEV)
    out = ctx.drift_groups(X, V, thr, lab, h, radius=Rd, f=f)
    ox, ov, om, oR, st, ostats, omg, omt = oracle.drift_groups_merge(x, v, m, rc, R, f, np.array([0, 0]), p, h)
    mu = p["G"] * m.sum()
    E = math.acos(1 - 2 * f * R.sum() / r0)
    tc = math.sqrt(r0 ** 3 / (8 * mu)) * (math.pi - E + math.sin(E))
    say(f"  {out}; closed form {tc}")
    assert out["mergers"] == 1 and out["unfinished"] == 0
    np.testing.assert_array_equal(out["merges"], [[0, 0, 1]])
    np.testing.assert_array_equal(out["merges"], omg)
    # the binary64 integration holds positions to ~1e-13 of the 1 AU scale, so the contact time is
    # known to that distance over the contact speed: bar |dt| v_contact < 1e-12
    v_contact = math.sqrt(2 * mu * (1 / (f * R.sum()) - 1 / r0))
    say(f"  contact time error {out['merge_times'][0] - tc:.2e} (x v_contact {abs(out['merge_times'][0] - tc) * v_contact:.2e})")
    assert abs(out["merge_times"][0] - tc) * v_contact < 1e-12
    xm = X.cpu().numpy(); vv = V.cpu().numpy()
    assert xm[0, 3] == m.sum() and xm[1, 3] == 0.0
    np.testing.assert_allclose(xm[:, :3], ox, rtol=0, atol=1e-13 * 1e6)   # the parked body sits at 1e6
    np.testing.assert_allclose(xm[0, :3], ox[0], rtol=0, atol=1e-14)
    # the merged velocity is the centre-of-mass velocity of the two integrated velocities, each held
    # to the integrator's tolerance, 1e-14 of the group's velocity scale (0.022) per accepted macro
    # step: ten steps' worth is 2e-15 (the oracle integrates to 1e-18)
    np.testing.assert_allclose(vv[0, :3], ov[0], rtol=0, atol=2e-15)
    np.testing.assert_allclose(Rd.cpu().numpy(), oR, rtol=1e-15, atol=0)


def test_step_hybrid_merges_match_oracle(nb):
    """10 hybrid steps of the 2048 disk with f = 300 (five mergers, one of a pair already in contact
    at the start of a drift): the same mergers as the oracle, at the same times, with the same
    masses and radii, and the same states."""
    say("step_hybrid merges disk2048 f=300 x10")
    p = diskgen.PARAMS
    ctx = nb.Context(nb.Params(**p))
    d = diskgen.workload("disk2048")
    X, V = dev_state(d["x"], d["v"], d["m"])
    thr = ctx.rcrit(X, V)
    Rd = torch.tensor(d["radius"], device=DEV)
    out = ctx.step_hybrid(X, V, 10, thr=thr, radius=Rd, f=300.0)
    othr = oracle.thresholds(d["x"], d["v"], d["m"], p)
    ox, ov, om, oR, st, ostats, omg, omt = oracle.step_merge(d["x"], d["v"], d["m"], d["radius"], 300.0, p, 10,
                                                             thr=othr)
    say(f"  gpu {out['mergers']} mergers {sorted_log(out['merges']).tolist()}; oracle {sorted_log(omg).tolist()}")
    assert st == 0 and out["unfinished"] == 0 and out["too_large"] == 0
    assert out["mergers"] == len(omg) >= 3
    np.testing.assert_array_equal(sorted_log(out["merges"]), sorted_log(omg))
    key = lambda mg: [tuple(r) for r in np.asarray(mg)]
    gt = dict(zip(key(out["merges"]), out["merge_times"]))
    ot = dict(zip(key(omg), omt))
    # contact times follow from states that agree to ~1e-11 of the AU scale after several chaotic
    # steps; divided by the slowest contact speeds here (~1e-2) that is ~1e-9 of dt, so the bar on
    # the times is 1e-8 dt (the merged states themselves are held to the state bar below)
    dts = [abs(t - ot[e]) for e, t in gt.items()]
    say(f"  largest merger-time difference {max(dts):.2e} ({max(dts) / p['dt']:.2e} dt)")
    assert max(dts) < 1e-8 * p["dt"]
    xm = X.cpu().numpy(); vv = V.cpu().numpy()
    np.testing.assert_array_equal(xm[:, 3], om)
    np.testing.assert_allclose(Rd.cpu().numpy(), oR, rtol=1e-15, atol=0)
    live = om > 0
    ex = (np.abs(xm[live, :3] - ox[live]).max(1) / np.linalg.norm(ox[live], axis=1)).max()
    ev = (np.abs(vv[live, :3] - ov[live]).max(1) / np.linalg.norm(ov[live], axis=1)).max()
    say(f"  state rel err x {ex:.2e} v {ev:.2e}")
    assert ex < 1e-10 and ev < 1e-10
    gone = ~live
    np.testing.assert_allclose(np.linalg.norm(xm[gone, :3], axis=1), 1e6, rtol=1e-12)
    assert (Rd.cpu().numpy()[gone] == 0).all()


def test_merge_without_contact_is_the_hybrid_step(nb):
    """f = 0: the contact tests never fire, and the state is the hybrid step's bit for bit."""
    say("step_hybrid merges f=0")
    p = diskgen.PARAMS
    ctx = nb.Context(nb.Params(**p))
    d = diskgen.workload("disk2048")
    X1, V1 = dev_state(d["x"], d["v"], d["m"])
    X2, V2 = X1.clone(), V1.clone()
    thr = ctx.rcrit(X1, V1)
    Rd = torch.tensor(d["radius"], device=DEV)
    out = ctx.step_hybrid(X1, V1, 3, thr=thr, radius=Rd, f=0.0)
    ctx.step_hybrid(X2, V2, 3, thr=thr)
    assert out["mergers"] == 0
    assert torch.equal(X1, X2) and torch.equal(V1, V2)


def test_merge_arguments_checked(nb):
    say("merge argument checks")
    ctx = nb.Context(nb.Params(**diskgen.PARAMS))
    d = diskgen.workload("disk2048", n=64)
    X, V = dev_state(d["x"], d["v"], d["m"])
    Rd = torch.tensor(d["radius"], device=DEV)
    with pytest.raises(nb.NBodyError):
        ctx.step_hybrid(X, V, 1, radius=Rd, f=-1.0)
    with pytest.raises(nb.NBodyError):
        ctx.step_hybrid(X, V, 1, radius=Rd, f=float("nan"))
    with pytest.raises(nb.NBodyError):
        ctx.step_hybrid(X, V, 1, radius=Rd.float(), f=1.0)


def test_merge_log_truncated_at_capacity(nb):
    """With room for two entries the log keeps two of the five mergers (any two of the oracle's) and
    the count still says five; cap = 0 needs no log buffers."""
    say("merge log capacity")
    p = diskgen.PARAMS
    ctx = nb.Context(nb.Params(**p))
    d = diskgen.workload("disk2048")
    othr = oracle.thresholds(d["x"], d["v"], d["m"], p)
    omg = oracle.step_merge(d["x"], d["v"], d["m"], d["radius"], 300.0, p, 10, thr=othr)[6]
    for cap in (2, 0):
        X, V = dev_state(d["x"], d["v"], d["m"])
        thr = ctx.rcrit(X, V)
        Rd = torch.tensor(d["radius"], device=DEV)
        out = ctx.step_hybrid(X, V, 10, thr=thr, radius=Rd, f=300.0, cap=cap)
        say(f"  cap {cap}: count {out['mergers']}, logged {len(out['merges'])}")
        assert out["mergers"] == len(omg)
        assert len(out["merges"]) == min(cap, len(omg))
        logged = {tuple(r) for r in np.asarray(out["merges"]).tolist()}
        assert logged <= {tuple(r) for r in np.asarray(omg).tolist()}
