"""GPU parity: the HIP library against the CPU oracle on the same seeded inputs.

Tolerances (binary64 path):
  accelerations: |a - a_ref|_inf <= 1e-12 * max(|a_ref|_inf, l1) per body, l1 = G sum_j m_j |w_ij| r_ij
                 (the conditioning of the sum; both sides sum in different orders);
  encounter lists: bit-exact (the predicate is evaluated exactly in binary64 on both sides);
  thresholds H, V: bit-exact; rc: 4 ulp (cube root of two libraries);
  drift: 1e-14 relative per step; states after k steps: 1e-11 relative (chaotic growth over 10
  steps of roundoff differences in the Kepler solve and summation order).
"""
import math

import numpy as np
import pytest

import diskgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


DEV = "cuda:0"


def to_dev(d):
    xm, v4 = diskgen.pack4(d["x"], d["v"], d["m"])
    return torch.tensor(xm, device=DEV), torch.tensor(v4, device=DEV)


def acc_err(acc, oacc, l1):
    return (np.abs(acc - oacc).max(1) / np.maximum(np.abs(oacc).max(1), l1)).max()


def cluster_disk(n, ncl, seed=11):
    """Disk with ncl consecutive bodies packed into a tight clump (many close pairs per row)."""
    d = diskgen.workload("disk2048", n=n)
    rng = np.random.default_rng(seed)
    c0 = d["x"][0].copy()
    d["x"][:ncl] = c0 + 0.004 * rng.standard_normal((ncl, 3))
    d["v"][:ncl] = d["v"][0] + 1e-3 * rng.standard_normal((ncl, 3))
    return d


# ------------------------------------------------------------------ thresholds
def test_rcrit_matches_oracle(ctx):
    p = diskgen.PARAMS
    for n in (1, 77, 2048):
        say(f"rcrit n={n}")
        d = diskgen.workload("disk2048", n=n)
        X, V = to_dev(d)
        thr = ctx.rcrit(X, V).cpu().numpy()
        rc, H, V_ = oracle.thresholds(d["x"], d["v"], d["m"], p)
        np.testing.assert_array_equal(thr[:, 1], H)
        np.testing.assert_array_equal(thr[:, 2], V_)
        np.testing.assert_allclose(thr[:, 0], rc, rtol=1e-15, atol=0)
        assert np.all(thr[:, 3] >= np.maximum(V_, np.cbrt(H)))


# ------------------------------------------------------------------ kick
@pytest.mark.parametrize("n", [2, 3, 63, 64, 65, 255, 257, 1000, 2048])
def test_kick_matches_oracle_ragged(ctx, n):
    say(f"kick n={n}")
    p = diskgen.PARAMS
    d = diskgen.workload("disk2048", n=n)
    X, V = to_dev(d)
    othr = oracle.thresholds(d["x"], d["v"], d["m"], p)
    thr = ctx.rcrit(X, V)
    acc, ce = ctx.accelerations(X, thr, with_ce=True)
    oacc, oce, l1 = oracle.kick_acc(d["x"], d["m"], othr, p)
    a = acc.cpu().numpy()[:, :3]
    assert acc_err(a, oacc, l1) < 1e-12
    c = ce.cpu().numpy()[:, :3]
    assert (np.abs(c - oce).max(1) / np.maximum(l1, 1e-300)).max() < 1e-12


def test_kick_single_body_is_zero(ctx):
    say("kick n=1")
    d = diskgen.workload("disk2048", n=1)
    X, V = to_dev(d)
    thr = ctx.rcrit(X, V)
    acc = ctx.accelerations(X, thr)
    assert torch.all(acc == 0)


def test_kick_close_cluster_and_velocity_update(ctx):
    say("kick cluster n=1500 ncl=300")
    p = diskgen.PARAMS
    d = cluster_disk(1500, 300)
    X, V = to_dev(d)
    othr = oracle.thresholds(d["x"], d["v"], d["m"], p)
    thr = ctx.rcrit(X, V)
    oacc, oce, l1 = oracle.kick_acc(d["x"], d["m"], othr, p)
    assert np.abs(oce).max() > 0
    acc, ce = ctx.accelerations(X, thr, with_ce=True)
    assert acc_err(acc.cpu().numpy()[:, :3], oacc, l1) < 1e-12
    v0 = V.clone()
    h = 0.05
    ctx.kick(X, thr, V, h)
    ref = d["v"] + h * oacc
    got = V.cpu().numpy()
    assert np.abs(got[:, :3] - ref).max() <= 1e-12 * h * np.maximum(np.abs(oacc).max(1), l1).max() + 4e-16
    assert torch.equal(V[:, 3], v0[:, 3])


def test_kick_split_precision_error_bound(nb):
    say("kick split n=2048")
    p = diskgen.PARAMS
    ctx_s = nb.Context(nb.Params(**p, precision=nb.PREC_SPLIT))
    d = diskgen.workload("disk2048")
    X, V = to_dev(d)
    othr = oracle.thresholds(d["x"], d["v"], d["m"], p)
    thr = ctx_s.rcrit(X, V)
    acc = ctx_s.accelerations(X, thr).cpu().numpy()[:, :3]
    oacc, _, l1 = oracle.kick_acc(d["x"], d["m"], othr, p)
    err = acc_err(acc, oacc, l1)
    # binary32 r^-3: each term carries ~1e-7 relative error
    assert err < 1e-6
    assert err > 1e-12       # really the split path


# ------------------------------------------------------------------ encounters
def test_encounters_bit_exact_disk(ctx):
    say("encounters disk2048")
    p = diskgen.PARAMS
    d = diskgen.workload("disk2048")
    X, V = to_dev(d)
    othr = oracle.thresholds(d["x"], d["v"], d["m"], p)
    thr = ctx.rcrit(X, V)
    pairs, count = ctx.encounters(X, thr)
    ref = oracle.encounters(d["x"], othr)
    assert count == len(ref) > 100
    np.testing.assert_array_equal(pairs.cpu().numpy(), ref)


def test_encounters_dense_rows_and_truncation(ctx):
    say("encounters cluster n=16384 ncl=400")
    p = diskgen.PARAMS
    d = cluster_disk(16384, 400)
    X, V = to_dev(d)
    othr = oracle.thresholds(d["x"], d["v"], d["m"], p)
    thr = ctx.rcrit(X, V)
    ref = oracle.encounters(d["x"], othr)
    rows = np.bincount(ref[:, 0], minlength=16384)
    assert rows.max() > 200          # rows beyond the per-chunk buffer take the rescan path
    pairs, count = ctx.encounters(X, thr)
    assert count == len(ref)
    np.testing.assert_array_equal(pairs.cpu().numpy(), ref)
    cap = len(ref) // 3
    pairs_t, count_t = ctx.encounters(X, thr, cap=cap)
    assert count_t == len(ref)
    np.testing.assert_array_equal(pairs_t.cpu().numpy(), ref[:cap])


def test_encounters_none_and_empty_capacity(ctx):
    say("encounters far bodies")
    x = np.array([[1.0, 0, 0], [-1.0, 0, 0], [0, 2.0, 0]])
    v = np.array([[0, 1.0, 0], [0, -1.0, 0], [-0.7, 0, 0]])
    m = np.full(3, 1e-9)
    X, V = to_dev({"x": x, "v": v, "m": m})
    thr = ctx.rcrit(X, V)
    pairs, count = ctx.encounters(X, thr, cap=0)
    assert count == 0


# ------------------------------------------------------------------ jump and drift
def test_jump_matches_oracle(ctx):
    say("jump n=1000")
    p = diskgen.PARAMS
    d = diskgen.workload("disk2048", n=1000)
    X, V = to_dev(d)
    ctx.jump(X, V, 0.05)
    ox = oracle.jump(d["x"], d["v"], d["m"], p, 0.05)
    np.testing.assert_allclose(X.cpu().numpy()[:, :3], ox, rtol=0, atol=1e-15)


def test_drift_matches_oracle(ctx):
    say("drift disk n=2048")
    p = diskgen.PARAMS
    d = diskgen.workload("disk2048")
    st = torch.zeros(2048, dtype=torch.int32, device=DEV)
    for h in (p["dt"], -0.3 * p["dt"], 7.5):
        X, V = to_dev(d)
        ctx.drift(X, V, h, status=st)
        ox, ov, ost = oracle.drift(d["x"], d["v"], p, h)
        x = X.cpu().numpy()[:, :3]; v = V.cpu().numpy()[:, :3]
        assert int(st.abs().max()) == 0
        tol = 2e-14 if abs(h) < 1 else 2e-13      # phase error grows with the angle swept
        assert (np.abs(x - ox).max(1) / np.linalg.norm(ox, axis=1)).max() < tol
        assert (np.abs(v - ov).max(1) / np.linalg.norm(ov, axis=1)).max() < tol
        np.testing.assert_array_equal(X[:, 3].cpu().numpy(), d["m"])


def test_drift_hyperbolic_and_closed_form(ctx):
    say("drift special orbits")
    p = diskgen.PARAMS
    r, mu = 1.3, 1.0
    n = math.sqrt(mu / r ** 3)
    x = np.array([[r, 0.0, 0.0], [0.8, 0.1, -0.05], [0.3, 0.0, 0.0]])
    v = np.array([[0.0, r * n, 0.0], [0.3, 1.9, 0.2], [0.0, 2.5, 0.1]])
    X, V = to_dev({"x": x, "v": v, "m": np.zeros(3)})
    t = 0.731
    ctx.drift(X, V, t)
    got = X.cpu().numpy()[:, :3]
    np.testing.assert_allclose(got[0], r * np.array([math.cos(n * t), math.sin(n * t), 0.0]), atol=2e-15)
    ox, ov, _ = oracle.drift(x, v, p, t)
    np.testing.assert_allclose(got, ox, rtol=0, atol=1e-14)
    np.testing.assert_allclose(V.cpu().numpy()[:, :3], ov, rtol=0, atol=1e-14)


# ------------------------------------------------------------------ full step
def test_step_matches_oracle_disk2048(ctx):
    """The small workload: N = 2048, 10 steps at dt = 6 days; state and final encounter list."""
    say("step disk2048 x10")
    p = diskgen.PARAMS
    d = diskgen.workload("disk2048")
    X, V = to_dev(d)
    thr = ctx.rcrit(X, V)
    pairs, count = ctx.step(X, V, 10, thr=thr, pairs_cap=100000)
    othr = oracle.thresholds(d["x"], d["v"], d["m"], p)
    ox, ov, st = oracle.step(d["x"], d["v"], d["m"], p, 10, thr=othr)
    x = X.cpu().numpy()[:, :3]; v = V.cpu().numpy()[:, :3]
    ex = (np.abs(x - ox).max(1) / np.linalg.norm(ox, axis=1)).max()
    ev = (np.abs(v - ov).max(1) / np.linalg.norm(ov, axis=1)).max()
    say(f"  state rel err x {ex:.2e} v {ev:.2e}")
    assert ex < 1e-11 and ev < 1e-11
    ref = oracle.encounters(ox, othr)
    assert count == len(ref)
    np.testing.assert_array_equal(pairs.cpu().numpy(), ref)


def test_step_composition_and_determinism(ctx):
    say("step composition n=700")
    d = diskgen.workload("disk2048", n=700)
    X, V = to_dev(d)
    thr = ctx.rcrit(X, V)
    X1, V1 = X.clone(), V.clone()
    ctx.step(X1, V1, 6, thr=thr)
    X2, V2 = X.clone(), V.clone()
    ctx.step(X2, V2, 2, thr=thr)
    ctx.step(X2, V2, 4, thr=thr)
    X3, V3 = X.clone(), V.clone()
    ctx.step(X3, V3, 6, thr=thr)
    torch.cuda.synchronize()
    assert torch.equal(X1, X2) and torch.equal(V1, V2)
    assert torch.equal(X1, X3) and torch.equal(V1, V3)


def test_step_zero_steps_lists_pairs(ctx):
    say("step nsteps=0")
    p = diskgen.PARAMS
    d = diskgen.workload("disk2048")
    X, V = to_dev(d)
    X0 = X.clone()
    pairs, count = ctx.step(X, V, 0, pairs_cap=10000)
    assert torch.equal(X, X0)
    ref = oracle.encounters(d["x"], oracle.thresholds(d["x"], d["v"], d["m"], p))
    np.testing.assert_array_equal(pairs.cpu().numpy(), ref)


@pytest.mark.parametrize("case", ["disk2048", "cluster4096"])
def test_step_counts_match_oracle(ctx, case):
    """Close-pair counts at each of the nsteps + 1 force evaluations equal the oracle's list
    lengths at the oracle's states; counting changes no bit of the state."""
    say(f"step counts {case}")
    p = diskgen.PARAMS
    d = diskgen.workload("disk2048") if case == "disk2048" else cluster_disk(4096, 300)
    k = 5 if case == "disk2048" else 2
    X, V = to_dev(d)
    thr = ctx.rcrit(X, V)
    Xa, Va = X.clone(), V.clone()
    (pairs, count), sc = ctx.step(Xa, Va, k, thr=thr, pairs_cap=200000, step_counts=True)
    Xb, Vb = X.clone(), V.clone()
    ctx.step(Xb, Vb, k, thr=thr)
    Xc, Vc = X.clone(), V.clone()
    sc_only = ctx.step(Xc, Vc, k, thr=thr, step_counts=True)
    torch.cuda.synchronize()
    assert torch.equal(Xa, Xb) and torch.equal(Va, Vb)
    assert torch.equal(Xa, Xc) and torch.equal(Va, Vc)
    sc = sc.cpu().numpy()
    np.testing.assert_array_equal(sc, sc_only.cpu().numpy())
    assert sc[-1] == count
    othr = oracle.thresholds(d["x"], d["v"], d["m"], p)
    ox, ov = d["x"].copy(), d["v"].copy()
    ref = [len(oracle.encounters(ox, othr))]
    for s in range(k):
        ox, ov, _ = oracle.step(ox, ov, d["m"], p, 1, thr=othr)
        ref.append(len(oracle.encounters(ox, othr)))
    say(f"  counts {sc.tolist()}")
    np.testing.assert_array_equal(sc, np.array(ref))
    # no steps: the count at the given positions
    sc0 = ctx.step(X.clone(), V.clone(), 0, thr=thr, step_counts=True).cpu().numpy()
    np.testing.assert_array_equal(sc0, ref[:1])


def test_encounter_groups_from_lists(ctx):
    """Groups of real encounter lists (the 2048 disk, a 400-body clump in N = 16384) equal the
    oracle's breadth-first components of the same list, label for label."""
    for name, d in (("disk2048", diskgen.workload("disk2048")), ("clump16384", cluster_disk(16384, 400))):
        say(f"groups {name}")
        X, V = to_dev(d)
        thr = ctx.rcrit(X, V)
        pairs, count = ctx.encounters(X, thr, cap=1 << 20)
        lab, g, ign = ctx.encounter_groups(X.shape[0], pairs.contiguous(), count)
        olab, og, oign = oracle.groups(X.shape[0], pairs.cpu().numpy())
        np.testing.assert_array_equal(lab.cpu().numpy(), olab)
        assert (g, ign) == (og, oign) and og > 0


@pytest.mark.parametrize("n", [1, 2, 1000, 70000])
def test_encounter_groups_synthetic_edges(ctx, n):
    """Random edges with repeats, self-pairs and out-of-range indices; a shuffled chain (the
    deepest union-find trees); truncation by cap; an empty list."""
    say(f"groups synthetic n={n}")
    rng = np.random.default_rng(n)
    cases = []
    e = rng.integers(-2, n + 2, size=(max(1, n // 2), 2)).astype(np.int32)
    cases.append(("random", e, len(e)))
    if n > 1:
        ch = np.stack([np.arange(n - 1), np.arange(1, n)], axis=1).astype(np.int32)
        cases.append(("chain", ch[rng.permutation(n - 1)], n - 1))
        cases.append(("truncated", ch[rng.permutation(n - 1)], (n - 1) // 3))
    cases.append(("empty", np.zeros((4, 2), dtype=np.int32), 0))
    for label, edges, cap in cases:
        P = torch.tensor(edges, device=DEV)
        count = torch.tensor([len(edges)], dtype=torch.int64, device=DEV)
        lab, g, ign = ctx.encounter_groups(n, P[:max(cap, 1)].contiguous() if cap else P[:0].contiguous(), count)
        olab, og, oign = oracle.groups(n, edges[:cap])
        np.testing.assert_array_equal(lab.cpu().numpy(), olab, err_msg=label)
        assert (g, ign) == (og, oign), label


def test_validate_reports_first_problem(ctx):
    say("validate")
    d = diskgen.workload("disk2048", n=1000)
    xm, v4 = diskgen.pack4(d["x"], d["v"], d["m"])

    def run(mod):
        a, b = xm.copy(), v4.copy()
        mod(a, b)
        return ctx.validate(torch.tensor(a, device=DEV), torch.tensor(b, device=DEV))

    assert run(lambda a, b: None) == (-1, 0)
    assert run(lambda a, b: a.__setitem__((500, 1), np.nan)) == (500, 1)
    assert run(lambda a, b: b.__setitem__((42, 2), np.inf)) == (42, 1)

    def two(a, b):
        a[300, 3] = -1e-9
        a[700, 0] = np.nan
    assert run(two) == (300, 2)
    assert run(lambda a, b: a.__setitem__((600, slice(0, 3)), 0.0)) == (600, 3)

    def dup(a, b):
        a[789, :3] = a[123, :3]
    assert run(dup) == (123, 4)

    def both(a, b):          # index 5 has a duplicate later and a negative mass: smallest reason
        a[900, :3] = a[5, :3]
        a[5, 3] = -1.0
    assert run(both) == (5, 2)
    assert ctx.validate(torch.tensor(xm[:1], device=DEV), torch.tensor(v4[:1], device=DEV)) == (-1, 0)


def test_energy_matches_oracle(ctx):
    say("energy n=2048")
    p = diskgen.PARAMS
    d = diskgen.workload("disk2048")
    X, V = to_dev(d)
    thr = ctx.rcrit(X, V)
    e = ctx.energy(X, V, thr)
    oe = oracle.energy(d["x"], d["v"], d["m"], p, oracle.thresholds(d["x"], d["v"], d["m"], p))
    assert abs(e["E"] - oe["E"]) < 1e-13 * abs(oe["E"])
    assert abs(e["Eprime"] - oe["Eprime"]) < 1e-13 * abs(oe["Eprime"])
    np.testing.assert_allclose(e["L"], oe["L"], rtol=1e-13)
    scale = (d["m"][:, None] * np.abs(d["v"])).sum()
    np.testing.assert_allclose(e["P"], oe["P"], rtol=0, atol=1e-14 * scale)


# ------------------------------------------------------------------ full size (N = 32768)
@pytest.fixture(scope="module")
def big():
    d = diskgen.workload("disk32768")
    p = diskgen.PARAMS
    return d, oracle.thresholds(d["x"], d["v"], d["m"], p)


def test_full_size_kick_sampled_rows(ctx, big):
    say("kick disk32768 sampled rows")
    d, othr = big
    p = diskgen.PARAMS
    X, V = to_dev(d)
    thr = ctx.rcrit(X, V)
    acc = ctx.accelerations(X, thr).cpu().numpy()[:, :3]
    rows = np.random.default_rng(5).choice(len(d["m"]), 96, replace=False)
    rows = np.concatenate([rows, [0, 1, 32767, 16384]])
    oacc, l1 = oracle.kick_acc_rows(d["x"], d["m"], othr, p, rows)
    err = (np.abs(acc[rows] - oacc).max(1) / np.maximum(np.abs(oacc).max(1), l1)).max()
    say(f"  max rel err {err:.2e}")
    assert err < 1e-12
    mom = (d["m"][:, None] * acc).sum(0)
    assert np.abs(mom).max() < 1e-13 * (d["m"][:, None] * np.abs(acc)).sum()


def test_full_size_encounters(ctx, big):
    say("encounters disk32768")
    d, othr = big
    X, V = to_dev(d)
    thr = ctx.rcrit(X, V)
    pairs, count = ctx.encounters(X, thr)
    ref = oracle.encounters(d["x"], othr)
    say(f"  {count} pairs")
    assert count == len(ref)
    np.testing.assert_array_equal(pairs.cpu().numpy(), ref)


def test_full_size_long_run_invariants(ctx, big):
    """1000 steps at N = 32768: angular momentum to roundoff, K-weighted energy bounded."""
    say("step disk32768 x1000 invariants")
    d, othr = big
    X, V = to_dev(d)
    thr = ctx.rcrit(X, V)
    e0 = ctx.energy(X, V, thr)
    ctx.step(X, V, 1000, thr=thr)
    e1 = ctx.energy(X, V, thr)
    dL = np.abs(e1["L"] - e0["L"]).max() / np.abs(e0["L"]).max()
    dE = abs(e1["Eprime"] - e0["Eprime"]) / abs(e0["Eprime"])
    say(f"  dL/L {dL:.2e}  dE'/E' {dE:.2e}")
    assert dL < 1e-11
    assert dE < 1e-7


def test_locality_permutation_changes_no_bit(nb):
    """Grouping bodies into waves by position (n >= locality_min_n) must not change a bit of the
    accelerations, the encounter list or a multi-step state."""
    say("locality permutation on/off n=9000")
    p = diskgen.PARAMS
    d = cluster_disk(9000, 300)
    res = []
    for min_n in (1, 1 << 30):
        ctx = nb.Context(nb.Params(**p))
        ctx.tune("locality_min_n", min_n)
        ctx.tune("locality_every", 3)
        X, V = to_dev(d)
        thr = ctx.rcrit(X, V)
        acc, ce = ctx.accelerations(X, thr, with_ce=True)
        pairs, count = ctx.encounters(X, thr)
        spairs, scount = ctx.step(X, V, 7, thr=thr, pairs_cap=1 << 20)
        res.append((acc, ce, pairs, X, V, spairs))
    for a, b in zip(res[0], res[1]):
        assert torch.equal(a, b)


def test_tuning_knobs_validate(nb):
    ctx = nb.Context(nb.Params(**diskgen.PARAMS))
    with pytest.raises(nb.NBodyError):
        ctx.tune("no_such_knob", 3)
    with pytest.raises(nb.NBodyError):
        ctx.tune("emit_slots", 0)


def test_encounter_groups_full_size(ctx, big):
    """The N = 32768 disk's list at its initial positions."""
    say("groups disk32768")
    d, _ = big
    X, V = to_dev(d)
    thr = ctx.rcrit(X, V)
    pairs, count = ctx.encounters(X, thr, cap=1 << 20)
    lab, g, ign = ctx.encounter_groups(X.shape[0], pairs.contiguous(), count)
    olab, og, oign = oracle.groups(X.shape[0], pairs.cpu().numpy())
    np.testing.assert_array_equal(lab.cpu().numpy(), olab)
    assert (g, ign) == (og, oign)
    say(f"  {count} pairs, {g} groups, largest {np.bincount(olab).max()}")


# ------------------------------------------------------------------ full size ring (N = 131072)
def test_full_size_ring_f64_and_split(nb):
    """The 131072-body ring in the launch configuration the benchmark times: binary64 and split
    kicks on 48 sampled rows against the oracle; the full encounter list at the initial
    positions bit-exact."""
    say("ring131072 kick f64/split sampled rows + list")
    p = diskgen.PARAMS
    d = diskgen.workload("ring131072")
    n = len(d["m"])
    othr = oracle.thresholds(d["x"], d["v"], d["m"], p)
    rows = np.concatenate([np.random.default_rng(21).choice(n, 44, replace=False), [0, 1, n // 2, n - 1]])
    oacc, l1 = oracle.kick_acc_rows(d["x"], d["m"], othr, p, rows)
    X, V = to_dev(d)
    for prec, bound in ((nb.PREC_F64, 1e-12), (nb.PREC_SPLIT, 1e-6)):
        ctx = nb.Context(nb.Params(**p, precision=prec))
        thr = ctx.rcrit(X, V)
        acc = ctx.accelerations(X, thr).cpu().numpy()[:, :3]
        err = (np.abs(acc[rows] - oacc).max(1) / np.maximum(np.abs(oacc).max(1), l1)).max()
        say(f"  precision {prec}: max rel err {err:.2e}")
        assert err < bound
        if prec == nb.PREC_SPLIT:
            assert err > 1e-12           # really the binary32 core
    ctx = nb.Context(nb.Params(**p))
    thr = ctx.rcrit(X, V)
    pairs, count = ctx.encounters(X, thr, cap=1 << 25)
    ref = oracle.encounters(d["x"], othr)
    say(f"  {count} pairs")
    assert count == len(ref)
    np.testing.assert_array_equal(pairs.cpu().numpy(), ref)


# ------------------------------------------------------------------ close-encounter drift, hybrid step
def test_drift_groups_matches_oracle(ctx):
    """H_A in full over one step: the groups of the 2048 disk's list (the GPU's own groups, equal to
    the oracle's) integrated by the GPU's Bulirsch-Stoer kernel (binary64, tolerance 1e-14) against
    the oracle's (long double, tolerance 1e-18, within ~2e-15 of the exact flow); the bodies in no
    group on Kepler orbits. Measured on the CPU: the same method at tolerance 1e-14 stays within
    ~2e-12 of the exact flow in velocity, so the bar is 1e-11."""
    say("drift_groups disk2048")
    p = diskgen.PARAMS
    d = diskgen.workload("disk2048")
    X, V = to_dev(d)
    thr = ctx.rcrit(X, V)
    pairs, count = ctx.encounters(X, thr, cap=1 << 20)
    lab, g, _ = ctx.encounter_groups(X.shape[0], pairs.contiguous(), count)
    othr = oracle.thresholds(d["x"], d["v"], d["m"], p)
    olab, og, _ = oracle.groups(X.shape[0], oracle.encounters(d["x"], othr))
    np.testing.assert_array_equal(lab.cpu().numpy(), olab)
    stats = ctx.drift_groups(X, V, thr, lab, p["dt"])
    ox, ov, st, ostats = oracle.drift_groups(d["x"], d["v"], d["m"], othr[0], olab, p, p["dt"])
    x = X.cpu().numpy()[:, :3]; v = V.cpu().numpy()[:, :3]
    ex = (np.abs(x - ox).max(1) / np.linalg.norm(ox, axis=1)).max()
    ev = (np.abs(v - ov).max(1) / np.linalg.norm(ov, axis=1)).max()
    say(f"  {stats}; state rel err x {ex:.2e} v {ev:.2e}")
    assert st == 0 and stats["unfinished"] == 0 and stats["too_large"] == 0
    assert (stats["groups"], stats["largest"], stats["bodies"]) == ostats
    assert ex < 1e-11 and ev < 1e-11


def test_step_hybrid_matches_oracle_and_conserves_energy(ctx):
    """10 hybrid steps of the 2048 disk against the oracle's hybrid step (state, group statistics),
    and the full energy E conserved as the oracle conserves it."""
    say("step_hybrid disk2048 x10")
    p = diskgen.PARAMS
    d = diskgen.workload("disk2048")
    X, V = to_dev(d)
    thr = ctx.rcrit(X, V)
    e0 = ctx.energy(X, V, thr)
    stats = ctx.step_hybrid(X, V, 10, thr=thr)
    e1 = ctx.energy(X, V, thr)
    othr = oracle.thresholds(d["x"], d["v"], d["m"], p)
    ox, ov, st, ostats = oracle.step_hybrid(d["x"], d["v"], d["m"], p, 10, thr=othr)
    x = X.cpu().numpy()[:, :3]; v = V.cpu().numpy()[:, :3]
    ex = (np.abs(x - ox).max(1) / np.linalg.norm(ox, axis=1)).max()
    ev = (np.abs(v - ov).max(1) / np.linalg.norm(ov, axis=1)).max()
    dE = abs(e1["E"] - e0["E"]) / abs(e0["E"])
    say(f"  {stats}; state rel err x {ex:.2e} v {ev:.2e}; dE/E {dE:.2e}")
    assert st == 0 and stats["unfinished"] == 0 and stats["too_large"] == 0 and stats["list_overflows"] == 0
    assert (stats["groups"], stats["largest"], stats["bodies"]) == ostats
    assert ex < 1e-10 and ev < 1e-10
    assert dE < 3e-10


def test_step_hybrid_reports_oversized_groups(nb, ctx):
    """A clump of 300 bodies forms one group above the 64 a wave integrates: reported in the
    statistics and as a warning of the binding."""
    say("step_hybrid clump")
    d = cluster_disk(4096, 300)
    X, V = to_dev(d)
    with pytest.warns(nb.NBodyWarning, match="Kepler orbits only"):
        stats = ctx.step_hybrid(X, V, 1)
    assert stats["too_large"] >= 1 and stats["largest"] >= 0
