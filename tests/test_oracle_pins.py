"""Pins of the CPU oracle against closed forms, invariants and independent references.

Each test names the passage of the paper it follows (Grimm & Stadel, section "The hybrid
symplectic integrator": equations Ha, Hb, Hc and rcrit) and pins the oracle to something other
than itself: hand-derived closed forms, a textbook Newtonian sum, Kepler's equation solved from
orbital elements, finite differences of the oracle's own potential, and conservation laws.
"""
import math

import numpy as np
import pytest

import diskgen
import oracle


def P(**kw):
    p = dict(diskgen.PARAMS)
    p.update(kw)
    return p


def newtonian(x, m, G=1.0):
    """Textbook pairwise Newtonian accelerations (brute force, numpy)."""
    d = x[None, :, :] - x[:, None, :]           # d[i, j] = x_j - x_i
    r2 = (d * d).sum(-1)
    np.fill_diagonal(r2, np.inf)
    return G * (m[None, :, None] * d / r2[..., None] ** 1.5).sum(1)


def no_close(x, v, m, p):
    """Thresholds with every pair far (n1 = n2 = 0): the K = 1 regime."""
    return oracle.thresholds(x, v, m, P(n1=0.0, n2=0.0))


# ------------------------------------------------------------------ changeover K (eq. Hb)
def test_changeover_endpoints_and_symmetry():
    for y, K in [(0.0, 0.0), (1.0, 1.0), (0.5, 0.5), (-3.0, 0.0), (7.0, 1.0)]:
        assert oracle.changeover(y)[0] == K
    assert oracle.changeover(0.0)[1] == 0.0 and oracle.changeover(1.0)[1] == 0.0
    for y in np.linspace(0.01, 0.99, 37):
        K, d = oracle.changeover(y)
        K2, _ = oracle.changeover(1.0 - y)
        assert abs(K + K2 - 1.0) < 4e-16
        h = 1e-6
        fd = (oracle.changeover(y + h)[0] - oracle.changeover(y - h)[0]) / (2 * h)
        assert abs(fd - d) < 1e-9
        assert d > 0


def test_changeover_interior_values():
    """Hand values of the changeover of reading 1 (Chambers' K = y^2/(2y^2 - 2y + 1)): at y = 1/4,
    D = 1/8 - 1/2 + 1 = 5/8, so K = (1/16)/(5/8) = 1/10 and dK/dy = 2y(1-y)/D^2 = (3/8)(64/25) = 24/25;
    at y = 3/4, K = (9/16)/(10/16) = 9/10 with the same slope; at y = 1/2, D = 1/2 and the slope is
    (1/2)/(1/4) = 2. Any other symmetric C1 step (for instance 3y^2 - 2y^3, which gives 5/32 and 9/8
    at y = 1/4 and slope 3/2 at 1/2) fails these."""
    for y, K, dK in ((0.25, 0.1, 0.96), (0.75, 0.9, 0.96), (0.5, 0.5, 2.0)):
        k, d = oracle.changeover(y)
        assert abs(k - K) <= 2e-17 and abs(d - dK) <= 4e-16, (y, k, d)


def test_kick_in_changeover_span_closed_form(params):
    """Two bodies inside the changeover span, with hand-made thresholds (H = 0, V = rc^2, so the
    pair is close exactly when r < rc = 1) and f_in = 1/2: at r = 0.625, y = (0.625 - 0.5)/0.5 = 1/4,
    K = 1/10, dK/dr = (24/25)/0.5, and the kick weight is w = K/r^3 - (dK/dr)/r^2
    = 0.1/0.244140625 - 1.92/0.390625 = 0.4096 - 4.9152 = -4.5056 (the changeover's slope pushes the
    pair apart); the close-encounter part is 1/r^3 - w = 4.096 + 4.5056 = 8.6016. This pins the
    kick's interior form (the gradient of K/r, eq. Hb) to numbers worked out by hand."""
    p = P(f_in=0.5)
    x = np.array([[1.0, 0.0, 0.0], [1.0, 0.375, 0.5]])      # |d| = 0.625
    m = np.array([2e-3, 5e-3])
    thr = (np.array([1.0, 1.0]), np.zeros(2), np.array([1.0, 1.0]))
    acc, ce, _ = oracle.kick_acc(x, m, thr, p)
    d = np.array([0.0, 0.375, 0.5])
    np.testing.assert_allclose(acc[0], 5e-3 * -4.5056 * d, rtol=1e-14)
    np.testing.assert_allclose(acc[1], -2e-3 * -4.5056 * d, rtol=1e-14)
    np.testing.assert_allclose(ce[0], 5e-3 * 8.6016 * d, rtol=1e-14)
    np.testing.assert_allclose(acc[0] + ce[0], 5e-3 * d / 0.625 ** 3, rtol=1e-15)


def test_changeover_quad_agrees():
    for y in np.linspace(0.0, 1.0, 21):
        assert abs(oracle.changeover(y)[0] - oracle.changeover(y, quad=True)[0]) < 4e-16


# ------------------------------------------------------------------ kick, K = 1 regime
def test_two_body_closed_form(params):
    x = np.array([[1.0, 0.0, 0.0], [1.0, 3.0, 4.0]])
    m = np.array([2e-3, 5e-3])
    v = np.zeros((2, 3))
    acc, ce, _ = oracle.kick_acc(x, m, no_close(x, v, m, params), params)
    np.testing.assert_allclose(acc[0], 5e-3 * np.array([0.0, 3.0, 4.0]) / 125.0, rtol=1e-15)
    np.testing.assert_allclose(acc[1], -2e-3 * np.array([0.0, 3.0, 4.0]) / 125.0, rtol=1e-15)
    assert np.all(ce == 0)


def test_triangle_and_square_closed_form(params):
    s, m0 = 0.7, 1e-3
    c = np.array([2.0, -1.0, 0.5])
    tri = np.array([[0, 0, 0], [s, 0, 0], [s / 2, s * math.sqrt(3) / 2, 0]], float) + c
    m = np.full(3, m0)
    acc, _, _ = oracle.kick_acc(tri, m, no_close(tri, 0 * tri, m, params), params)
    cen = tri.mean(0)
    for i in range(3):
        u = (cen - tri[i]) / np.linalg.norm(cen - tri[i])
        np.testing.assert_allclose(acc[i], math.sqrt(3) * m0 / s ** 2 * u, rtol=2e-15, atol=1e-20)
    sq = np.array([[0, 0, 0], [s, 0, 0], [s, s, 0], [0, s, 0]], float) + c
    m = np.full(4, m0)
    acc, _, _ = oracle.kick_acc(sq, m, no_close(sq, 0 * sq, m, params), params)
    cen = sq.mean(0)
    for i in range(4):
        u = (cen - sq[i]) / np.linalg.norm(cen - sq[i])
        np.testing.assert_allclose(acc[i], (math.sqrt(2) + 0.5) * m0 / s ** 2 * u, rtol=2e-15, atol=1e-20)


def test_far_field_equals_textbook_newton(params):
    d = diskgen.workload("disk2048", n=256)
    thr = no_close(d["x"], d["v"], d["m"], params)
    acc, ce, l1 = oracle.kick_acc(d["x"], d["m"], thr, params)
    ref = newtonian(d["x"], d["m"])
    err = np.abs(acc - ref).max(1) / l1
    assert err.max() < 1e-14
    assert np.all(ce == 0)


# ------------------------------------------------------------------ kick with changeover
def _cluster(params, seed=3):
    """Five bodies with separations spread over [0, rc]: every pair in the changeover zone."""
    rng = np.random.default_rng(seed)
    x = np.array([1.0, 0.0, 0.0]) + 0.02 * rng.standard_normal((5, 3))
    v = np.array([0.0, 1.0, 0.0]) + 0.05 * rng.standard_normal((5, 3))
    m = rng.uniform(1e-4, 1e-3, 5)
    return x, v, m


def test_kick_is_gradient_of_changeover_potential(params):
    """m_i a_i = -dU_B/dx_i with U_B = -sum G m_i m_j K/r (eq. Hb), by central differences of the
    oracle's K-weighted energy E' minus the star term."""
    x, v, m = _cluster(params)
    thr = oracle.thresholds(x, v, m, params)
    rc = thr[0]
    acc, ce, _ = oracle.kick_acc(x, m, thr, params)
    r = np.linalg.norm(x[:, None] - x[None], axis=-1)
    rcij = np.maximum(rc[:, None], rc[None])
    iu = np.triu_indices(5, 1)
    y = (r[iu] - 0.1 * rcij[iu]) / (0.9 * rcij[iu])
    assert np.any((y > 0) & (y < 1)), "fixture must exercise the changeover"
    h = 1e-7
    for i in range(5):
        for c in range(3):
            xp = x.copy(); xp[i, c] += h
            xn = x.copy(); xn[i, c] -= h
            Ep = oracle.energy(xp, v, m, params, thr)["Eprime"]
            En = oracle.energy(xn, v, m, params, thr)["Eprime"]
            dE = (Ep - En) / (2 * h)
            star = params["G"] * params["m0"] * m[i] * x[i, c] / np.linalg.norm(x[i]) ** 3
            force = -(dE - star)
            assert abs(force - m[i] * acc[i, c]) < 1e-6 * abs(m[i] * np.abs(acc[i]).max())


def test_split_sums_to_newton(params):
    """a^B + a^CE equals the plain Newtonian pull."""
    x, v, m = _cluster(params)
    thr = oracle.thresholds(x, v, m, params)
    acc, ce, l1 = oracle.kick_acc(x, m, thr, params)
    ref = newtonian(x, m)
    assert np.abs(acc + ce - ref).max() <= 1e-14 * np.abs(ref).max()
    assert np.abs(ce).max() > 0


def test_newton_third_law_and_permutation(params):
    d = diskgen.workload("disk2048", n=512)
    thr = oracle.thresholds(d["x"], d["v"], d["m"], params)
    acc, ce, l1 = oracle.kick_acc(d["x"], d["m"], thr, params)
    mom = (d["m"][:, None] * acc).sum(0)
    assert np.abs(mom).max() <= 1e-14 * (d["m"][:, None] * np.abs(acc)).sum()
    perm = np.random.default_rng(0).permutation(512)
    thr_p = tuple(t[perm] for t in thr)
    acc_p, _, _ = oracle.kick_acc(d["x"][perm], d["m"][perm], thr_p, params)
    err = np.abs(acc_p - acc[perm]).max(1) / l1[perm]
    assert err.max() < 1e-15


def test_f64_within_bound_of_quad(params):
    d = diskgen.workload("disk2048", n=512)
    thr = oracle.thresholds(d["x"], d["v"], d["m"], params)
    acc, _, l1 = oracle.kick_acc(d["x"], d["m"], thr, params)
    aq = oracle.kick_acc(d["x"], d["m"], thr, params, "quad")
    al = oracle.kick_acc(d["x"], d["m"], thr, params, "ld")
    assert (np.abs(acc - aq).max(1) / l1).max() < 1e-15
    assert (np.abs(al - aq).max(1) / l1).max() < 2.3e-16   # both rounded once to binary64


# ------------------------------------------------------------------ critical radius (eq. rcrit)
def test_rcrit_definition(params):
    d = diskgen.workload("disk2048", n=64)
    rc, H, V = oracle.thresholds(d["x"], d["v"], d["m"], params)
    r = np.linalg.norm(d["x"], axis=1)
    rhill = r * np.cbrt(d["m"] / (3 * params["m0"]))
    vel = np.linalg.norm(d["v"], axis=1)
    ref = np.maximum(3 * rhill, 0.4 * params["dt"] * vel)
    np.testing.assert_allclose(rc, ref, rtol=1e-15)
    np.testing.assert_allclose(H, (3 * rhill) ** 6, rtol=1e-14)
    np.testing.assert_allclose(V, (0.4 * params["dt"] * vel) ** 2, rtol=1e-15)


# ------------------------------------------------------------------ encounter list
def test_encounters_match_real_arithmetic_definition(params):
    d = diskgen.workload("disk2048")
    thr = oracle.thresholds(d["x"], d["v"], d["m"], params)
    pairs = oracle.encounters(d["x"], thr)
    x = d["x"]
    r = np.sqrt(((x[:, None] - x[None]) ** 2).sum(-1))
    rcij = np.maximum(thr[0][:, None], thr[0][None])
    iu = np.triu_indices(len(x), 1)
    ratio = r[iu] / rcij[iu]
    assert np.all(np.abs(ratio - 1) > 1e-9), "no pair sits on the threshold"
    ref = np.stack([iu[0][ratio < 1], iu[1][ratio < 1]], 1)
    assert len(pairs) > 50
    np.testing.assert_array_equal(pairs, ref)


def test_encounters_hand_placed(params):
    """Pairs at rc (1 +- 1e-9): inside flagged, outside not; m = 0 leaves only the velocity term."""
    base = np.array([1.0, 0.0, 0.0])
    vel = np.array([0.0, 1.0, 0.0])
    pts, vs = [], []
    for k in range(4):
        pts.append(base + np.array([0, 0, 10.0 * k]))
        vs.append(vel)
    x = np.array(pts)
    v = np.array(vs)
    m = np.zeros(4)
    rc, H, V = oracle.thresholds(x, v, m, params)
    assert np.all(H == 0)
    rcv = 0.4 * params["dt"]
    np.testing.assert_allclose(rc, rcv, rtol=1e-15)
    # partner bodies along y at distances rc(1-1e-9) and rc(1+1e-9)
    x2 = np.concatenate([x, x + np.array([[0, rcv * (1 - 1e-9), 0]] * 2 + [[0, rcv * (1 + 1e-9), 0]] * 2)])
    v2 = np.concatenate([v, v])
    m2 = np.zeros(8)
    thr2 = oracle.thresholds(x2, v2, m2, params)
    pairs = oracle.encounters(x2, thr2)
    np.testing.assert_array_equal(pairs, np.array([[0, 4], [1, 5]]))


# ------------------------------------------------------------------ jump (eq. Hc)
def test_jump_hand_values(params):
    x = np.array([[1.0, 2.0, 3.0], [-1.0, 0.5, 0.0]])
    v = np.array([[0.1, 0.0, -0.2], [0.3, 0.4, 0.0]])
    m = np.array([0.5, 0.25])
    h = 0.125
    Ptot = np.array([0.5 * 0.1 + 0.25 * 0.3, 0.25 * 0.4, 0.5 * -0.2])
    xo = oracle.jump(x, v, m, P(m0=2.0), h)
    np.testing.assert_allclose(xo, x + h * Ptot / 2.0, rtol=0, atol=1e-16)


# ------------------------------------------------------------------ Kepler drift (eq. Ha)
def _orbit_state(a, e, inc, node, argp, M, mu):
    x, v = diskgen.elements_to_cartesian(np.atleast_1d(a), np.atleast_1d(e), np.atleast_1d(inc),
                                         np.atleast_1d(node), np.atleast_1d(argp), np.atleast_1d(M),
                                         np.atleast_1d(mu))
    return x, v


def test_drift_circular_rotation(params):
    r, mu = 1.3, params["G"] * params["m0"]
    n = math.sqrt(mu / r ** 3)
    x = np.array([[r, 0.0, 0.0]])
    v = np.array([[0.0, r * n, 0.0]])
    t = 0.731
    xo, vo, st = oracle.drift(x, v, params, t)
    ref = r * np.array([math.cos(n * t), math.sin(n * t), 0.0])
    np.testing.assert_allclose(xo[0], ref, atol=2e-15)
    np.testing.assert_allclose(vo[0], r * n * np.array([-math.sin(n * t), math.cos(n * t), 0.0]), atol=2e-15)
    assert st[0] == 0


@pytest.mark.parametrize("e", [0.0, 0.05, 0.3, 0.7, 0.95])
def test_drift_matches_kepler_equation_from_elements(params, e):
    mu = params["G"] * params["m0"]
    a, inc, node, argp, M0 = 1.7, 0.3, 1.1, 2.2, 0.4
    n = math.sqrt(mu / a ** 3)
    x0, v0 = _orbit_state(a, e, inc, node, argp, M0, mu)
    for t in (0.1032, -0.77, 3.0, 25.0):
        xt, vt = _orbit_state(a, e, inc, node, argp, M0 + n * t, mu)
        xo, vo, st = oracle.drift(x0, v0, params, t)
        assert st[0] == 0
        np.testing.assert_allclose(xo, xt, rtol=0, atol=2e-13 * a / (1 - e))
        np.testing.assert_allclose(vo, vt, rtol=0, atol=2e-13 * math.sqrt(mu / a) / (1 - e))


def test_drift_hyperbolic_and_invariants(params):
    mu = params["G"] * params["m0"]
    x = np.array([[0.8, 0.1, -0.05]])
    v = np.array([[0.3, 1.9, 0.2]])           # v^2 > 2 mu / r: unbound
    assert (v ** 2).sum() > 2 * mu / np.linalg.norm(x)

    def inv(x, v):
        r = np.linalg.norm(x)
        L = np.cross(x, v)
        E = 0.5 * (v * v).sum() - mu / r
        A = np.cross(v, L) - mu * x / r       # Laplace-Runge-Lenz
        return E, L, A

    E0, L0, A0 = inv(x[0], v[0])
    for t in (0.05, 0.5, 3.0, -0.4):
        xo, vo, st = oracle.drift(x, v, params, t)
        assert st[0] == 0
        E1, L1, A1 = inv(xo[0], vo[0])
        assert abs(E1 - E0) < 1e-14 * abs(E0) + 1e-15
        np.testing.assert_allclose(L1, L0, atol=1e-14)
        np.testing.assert_allclose(A1, A0, atol=1e-13)
        xb, vb, _ = oracle.drift(xo, vo, params, -t)
        np.testing.assert_allclose(xb, x, atol=1e-13)
        np.testing.assert_allclose(vb, v, atol=1e-13)


def test_drift_one_period_and_quad(params):
    mu = params["G"] * params["m0"]
    d = diskgen.workload("disk2048", n=64)
    xo, vo, st = oracle.drift(d["x"], d["v"], params, 0.1032)
    xq, vq, stq = oracle.drift(d["x"], d["v"], params, 0.1032, quad=True)
    assert stq == 0 and np.all(st == 0)
    assert np.abs(xo - xq).max() < 4e-16 * 4 and np.abs(vo - vq).max() < 4e-16 * 2
    x, v = d["x"][:1], d["v"][:1]
    r = np.linalg.norm(x); a = 1 / (2 / r - (v ** 2).sum() / mu)
    T = 2 * math.pi * math.sqrt(a ** 3 / mu)
    xp, vp, _ = oracle.drift(x, v, params, T)
    np.testing.assert_allclose(xp, x, atol=1e-13)
    np.testing.assert_allclose(vp, v, atol=1e-13)


# ------------------------------------------------------------------ full step
def test_step_massless_is_pure_kepler(params):
    """All masses zero: kicks and jumps vanish and the step is the exact Kepler flow."""
    mu = params["G"] * params["m0"]
    a = np.array([0.6, 1.0, 2.5]); e = np.array([0.0, 0.1, 0.4]); inc = np.array([0.0, 0.2, 0.05])
    node = np.array([0.3, 1.0, 2.0]); argp = np.array([0.1, 0.5, 4.0]); M0 = np.array([0.0, 1.0, 2.0])
    x0, v0 = diskgen.elements_to_cartesian(a, e, inc, node, argp, M0, np.full(3, mu))
    m = np.zeros(3)
    k = 7
    xo, vo, st = oracle.step(x0, v0, m, params, k)
    n = np.sqrt(mu / a ** 3)
    xt, vt = diskgen.elements_to_cartesian(a, e, inc, node, argp, M0 + n * k * params["dt"], np.full(3, mu))
    np.testing.assert_allclose(xo, xt, atol=1e-13)
    np.testing.assert_allclose(vo, vt, atol=1e-13)


def test_step_conserves_angular_momentum_and_Eprime(params):
    d = diskgen.workload("disk2048", n=256)
    thr = oracle.thresholds(d["x"], d["v"], d["m"], params)
    e0 = oracle.energy(d["x"], d["v"], d["m"], params, thr)
    x, v, st = oracle.step(d["x"], d["v"], d["m"], params, 20, thr=thr)
    e1 = oracle.energy(x, v, d["m"], params, thr)
    assert np.abs(e1["L"] - e0["L"]).max() < 1e-13 * np.abs(e0["L"]).max()
    assert abs(e1["Eprime"] - e0["Eprime"]) < 1e-9 * abs(e0["Eprime"])


def test_step_energy_error_scales_as_dt_squared(params):
    """Second-order splitting: the K-weighted energy error drops about 4x when dt halves."""
    x, v, m = _cluster(params, seed=5)
    x = x + np.array([0.0, 0.0, 0.0]); m = m * 0.1
    thr = oracle.thresholds(x, v, m, params)
    e0 = oracle.energy(x, v, m, params, thr)["Eprime"]
    errs = []
    for div in (1, 2):
        p = P(dt=params["dt"] / div)
        xs, vs = x.copy(), v.copy()
        worst = 0.0
        for _ in range(8 * div):
            xs, vs, _ = oracle.step(xs, vs, m, p, 1, thr=thr)
            worst = max(worst, abs(oracle.energy(xs, vs, m, p, thr)["Eprime"] - e0))
        errs.append(worst)
    ratio = errs[0] / errs[1]
    assert 3.0 < ratio < 5.5, (errs, ratio)


def test_step_time_reversible(params):
    d = diskgen.workload("disk2048", n=128)
    thr = oracle.thresholds(d["x"], d["v"], d["m"], params)
    x, v, _ = oracle.step(d["x"], d["v"], d["m"], params, 5, thr=thr)
    xb, vb, _ = oracle.step(x, v, d["m"], P(dt=-params["dt"]), 5, thr=thr)
    np.testing.assert_allclose(xb, d["x"], atol=2e-14)
    np.testing.assert_allclose(vb, d["v"], atol=2e-14)


# ------------------------------------------------------------------ derivatives (gradient reference)
def test_jvp_matches_central_differences(params):
    d = diskgen.workload("disk2048", n=24)
    x, v, m = d["x"], d["v"], d["m"]
    rng = np.random.default_rng(1)
    dx = rng.standard_normal(x.shape); dv = rng.standard_normal(v.shape); dm = rng.standard_normal(m.shape) * m
    thr = oracle.thresholds(x, v, m, params)
    xo, vo, jx, jv, st = oracle.step_jvp(x, v, m, params, 6, dx, dv, dm)
    eps = 1e-6
    xp, vp, _ = oracle.step(x + eps * dx, v + eps * dv, m + eps * dm, params, 6, thr=thr)
    xn, vn, _ = oracle.step(x - eps * dx, v - eps * dv, m - eps * dm, params, 6, thr=thr)
    np.testing.assert_allclose(jx, (xp - xn) / (2 * eps), rtol=0, atol=1e-7 * np.abs(jx).max())
    np.testing.assert_allclose(jv, (vp - vn) / (2 * eps), rtol=0, atol=1e-7 * np.abs(jv).max())
    x1, v1, _ = oracle.step(x, v, m, params, 6, thr=thr)
    np.testing.assert_allclose(xo, x1, rtol=0, atol=1e-13)   # dual path rounds differently


def test_step_is_symplectic(params):
    """The step's Jacobian in canonical (x, p = m v) coordinates preserves the symplectic form."""
    x, v, m = _cluster(params, seed=7)
    x, v, m = x[:3], v[:3], m[:3]
    n = 3
    J = np.zeros((6 * n, 6 * n))
    for k in range(6 * n):
        dx = np.zeros((n, 3)); dv = np.zeros((n, 3))
        if k < 3 * n:
            dx.reshape(-1)[k] = 1.0
        else:
            dv.reshape(-1)[k - 3 * n] = 1.0 / np.repeat(m, 3)[k - 3 * n]   # unit change of p
        _, _, jx, jv, _ = oracle.step_jvp(x, v, m, params, 3, dx, dv, None)
        J[:3 * n, k] = jx.reshape(-1)
        J[3 * n:, k] = (jv * m[:, None]).reshape(-1)
    Om = np.block([[np.zeros((3 * n, 3 * n)), np.eye(3 * n)], [-np.eye(3 * n), np.zeros((3 * n, 3 * n))]])
    S = J.T @ Om @ J
    assert np.abs(S - Om).max() < 1e-9 * np.abs(J).max() ** 2


# ------------------------------------------------------------------ close-encounter groups
def test_groups_hand_cases():
    """Connected components of the close-pair graph, labelled by the smallest index."""
    lab, g, ign = oracle.groups(6, [[0, 1], [1, 2], [4, 5]])            # chain and a pair
    assert lab.tolist() == [0, 0, 0, 3, 4, 4] and g == 2 and ign == 0
    lab, g, ign = oracle.groups(5, [[4, 0], [4, 1], [4, 2], [4, 3]])    # star, edges given (j, i)
    assert lab.tolist() == [0] * 5 and g == 1
    lab, g, ign = oracle.groups(4, [[2, 3], [3, 2], [2, 3]])            # repeated edges
    assert lab.tolist() == [0, 1, 2, 2] and g == 1
    lab, g, ign = oracle.groups(3, [])                                  # no pairs: singletons
    assert lab.tolist() == [0, 1, 2] and g == 0
    lab, g, ign = oracle.groups(4, [[1, 1], [0, 7], [-1, 2], [3, 0]])   # not edges: ignored
    assert lab.tolist() == [0, 1, 2, 0] and g == 1 and ign == 3


def _closure_labels(n, edges):
    """Brute force: reachability by repeated boolean squaring, label = smallest reachable index."""
    A = np.eye(n, dtype=bool)
    for i, j in edges:
        A[i, j] = A[j, i] = True
    while True:
        B = (A.astype(np.int64) @ A.astype(np.int64)) > 0
        if (B == A).all():
            break
        A = B
    return np.array([np.flatnonzero(A[i])[0] for i in range(n)])


def test_groups_against_brute_force_and_library():
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    rng = np.random.default_rng(3)
    for n, ne in ((1, 0), (2, 1), (9, 5), (40, 30), (200, 150), (500, 700)):
        e = rng.integers(0, n, size=(ne, 2)) if ne else np.zeros((0, 2), dtype=np.int64)
        e = e[e[:, 0] != e[:, 1]]
        lab, g, ign = oracle.groups(n, e)
        assert ign == 0
        if n <= 200:
            np.testing.assert_array_equal(lab, _closure_labels(n, e.tolist()))
        ncomp, comp = connected_components(coo_matrix((np.ones(len(e)), (e[:, 0], e[:, 1])), shape=(n, n)),
                                           directed=False)
        # same partition: equal labels exactly when the library puts bodies in one component
        np.testing.assert_array_equal(lab[:, None] == lab[None, :], comp[:, None] == comp[None, :])
        sizes = np.bincount(comp, minlength=ncomp)
        assert g == int((sizes >= 2).sum())
        assert (lab <= np.arange(n)).all() and (lab[lab] == lab).all()


# ------------------------------------------------------------------ close-encounter drift (full H_A)
@pytest.fixture(scope="module")
def disk2048_groups(params):
    d = diskgen.workload("disk2048")
    thr = oracle.thresholds(d["x"], d["v"], d["m"], params)
    lab, g, _ = oracle.groups(len(d["m"]), oracle.encounters(d["x"], thr))
    return d, thr, lab


def test_ce_drift_far_group_is_kepler(params, disk2048_groups):
    """Two bodies far outside each other's critical radius: the [1 - K] term is zero and the group
    integration must reproduce two independent Kepler drifts (closed-form f and g functions)."""
    d, (rc, H, V), _ = disk2048_groups
    idx = np.array([3, 1700])
    assert np.linalg.norm(d["x"][3] - d["x"][1700]) > 10 * max(rc[3], rc[1700])
    xa, va, st = oracle.ce_drift_group(d["x"], d["v"], d["m"], rc, params, idx, params["dt"])
    xk, vk, _ = oracle.drift(d["x"][idx], d["v"][idx], params, params["dt"])
    assert st == 0
    np.testing.assert_allclose(xa[idx], xk, rtol=0, atol=1e-15 * np.abs(xk).max())
    np.testing.assert_allclose(va[idx], vk, rtol=0, atol=1e-15 * np.abs(vk).max())


def _energy_A(x, v, m, rc, idx, p):
    """H_A of the group idx from its definition: Kepler energies minus the [1 - K] pair part."""
    E = 0.0
    for a in idx:
        E += 0.5 * m[a] * (v[a] ** 2).sum() - p["G"] * p["m0"] * m[a] / np.linalg.norm(x[a])
    for k, a in enumerate(idx):
        for b in idx[k + 1:]:
            q = np.linalg.norm(x[b] - x[a])
            rcij = max(rc[a], rc[b])
            y = (q - p["f_in"] * rcij) / ((1 - p["f_in"]) * rcij)
            K, _ = oracle.changeover(min(max(y, 0.0), 1.0))
            E -= p["G"] * m[a] * m[b] * (1 - K) / q
    return E


def test_ce_drift_conserves_HA_and_reverses(params, disk2048_groups):
    """The largest group of the 2048 disk (10 bodies): H_A and the group's angular momentum are
    conserved, the integration is time-reversible, and the [1 - K] term does act."""
    d, (rc, H, V), lab = disk2048_groups
    idx = np.flatnonzero(lab == np.argmax(np.bincount(lab)))
    assert len(idx) == 10
    x, v, m = d["x"], d["v"], d["m"]
    xa, va, st = oracle.ce_drift_group(x, v, m, rc, params, idx, params["dt"])
    assert st == 0
    e0, e1 = _energy_A(x, v, m, rc, idx, params), _energy_A(xa, va, m, rc, idx, params)
    assert abs(e1 - e0) < 1e-14 * abs(e0)
    L0 = (m[idx, None] * np.cross(x[idx], v[idx])).sum(0)
    L1 = (m[idx, None] * np.cross(xa[idx], va[idx])).sum(0)
    assert np.abs(L1 - L0).max() < 1e-15 * np.abs(L0).max()
    xb, vb, _ = oracle.ce_drift_group(xa, va, m, rc, params, idx, -params["dt"])
    assert np.abs(xb[idx] - x[idx]).max() < 1e-14 * np.abs(x[idx]).max()
    assert np.abs(vb[idx] - v[idx]).max() < 1e-14 * np.abs(v[idx]).max()
    xk, vk, _ = oracle.drift(x[idx], v[idx], params, params["dt"])
    assert np.abs(xa[idx] - xk).max() > 1e-9                        # the pair term is not zero


def test_ce_drift_tight_binary_is_two_body_kepler(params):
    """A bound binary well inside f_in rc (K = 0: full Newtonian pull) with a negligible central
    mass: the relative orbit is the two-body Kepler orbit with mu = G (m1 + m2) and the centre of
    mass moves uniformly (closed forms)."""
    p = dict(params, m0=1e-30)
    m = np.array([3e-6, 1e-6])
    sep = 2e-3
    x = np.array([[1.0, 0.0, 0.0], [1.0 + sep, 5e-5, 0.0]])
    vrel = np.sqrt(p["G"] * m.sum() / sep) * 0.8
    v = np.array([[0.01, 0.02, 0.0], [0.01, 0.02 + vrel, 1e-3 * vrel]])
    rc = np.array([5e-2, 5e-2])
    h = 1.0                                   # about 3.5 orbits of the binary
    xa, va, st = oracle.ce_drift_group(x, v, m, rc, p, np.array([0, 1]), h)
    assert st == 0
    assert np.linalg.norm(xa[1] - xa[0]) < 0.1 * rc[0]              # stayed where K = 0
    M = m.sum()
    xc0, vc0 = (m[:, None] * x).sum(0) / M, (m[:, None] * v).sum(0) / M
    xr, vr, _ = oracle.drift((x[1] - x[0])[None], (v[1] - v[0])[None], dict(p, m0=M), h)
    xc1, vc1 = (m[:, None] * xa).sum(0) / M, (m[:, None] * va).sum(0) / M
    np.testing.assert_allclose(xc1, xc0 + h * vc0, rtol=0, atol=1e-15)
    np.testing.assert_allclose(vc1, vc0, rtol=0, atol=1e-15 * vrel)   # rounding of velocities of size vrel
    # the integration error is relative to the heliocentric scale (1 AU), so against the
    # separation it is looser by 1/sep
    np.testing.assert_allclose(xa[1] - xa[0], xr[0], rtol=0, atol=1e-11 * sep)
    np.testing.assert_allclose(va[1] - va[0], vr[0], rtol=0, atol=1e-11 * vrel)


def test_hybrid_step_conserves_full_energy(params, disk2048_groups):
    """The hybrid step integrates H_A in full, so it conserves the full energy E (the plain step
    conserves the K-weighted E' instead): over 20 steps of the 2048 disk, E drifts at ~1e-10 in
    the hybrid step and ~1e-9 in the plain one; with no close pairs the two steps coincide."""
    d, thr, _ = disk2048_groups
    x, v, m = d["x"], d["v"], d["m"]
    E0 = oracle.energy(x, v, m, params, thr)
    xh, vh, st, stats = oracle.step_hybrid(x, v, m, params, 20, thr=thr)
    xp, vp, _ = oracle.step(x, v, m, params, 20, thr=thr)
    Eh, Ep = oracle.energy(xh, vh, m, params, thr), oracle.energy(xp, vp, m, params, thr)
    dEh = abs(Eh["E"] - E0["E"]) / abs(E0["E"])
    dEp = abs(Ep["E"] - E0["E"]) / abs(E0["E"])
    assert st == 0 and stats[0] > 0
    assert dEh < 3e-10 and dEp > 10 * dEh
    assert abs(Ep["Eprime"] - E0["Eprime"]) / abs(E0["Eprime"]) < 1e-10
    # far-apart bodies only: identical to the plain step
    far = diskgen.workload("disk2048", n=40)
    fthr = oracle.thresholds(far["x"], far["v"], far["m"], params)
    assert len(oracle.encounters(far["x"], fthr)) == 0
    a = oracle.step_hybrid(far["x"], far["v"], far["m"], params, 3, thr=fthr)
    b = oracle.step(far["x"], far["v"], far["m"], params, 3, thr=fthr)
    if a[3][0] == 0:
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_array_equal(a[1], b[1])


# ------------------------------------------------------------------ collisions as perfect mergers
def test_merge_radial_infall_contact_time_closed_form(params):
    """Two bodies released at rest with a negligible central mass fall radially onto each other: the
    relative orbit is the degenerate Kepler ellipse of mu = G (m1 + m2), so the separation reaches
    f (R1 + R2) at t = sqrt(r0^3 / (8 mu)) (pi - E + sin E), cos E = 1 - 2 f (R1 + R2)/r0 (closed
    form). The merged body has the summed mass and volume and moves with the centre of mass; the
    removed body is parked far away, massless."""
    p = dict(params, m0=1e-30)
    m = np.array([3e-6, 1e-6]); R = np.array([6e-5, 4e-5]); f = 1.5
    r0 = 2e-3
    x = np.array([[1.0, 0.0, 0.0], [1.0 + r0, 0.0, 0.0]])
    v = np.array([[0.01, 0.02, 0.0], [0.01, 0.02, 0.0]])
    rc = np.array([5e-2, 5e-2])                  # r0 < f_in rc: full Newtonian pull
    h = 0.1
    X, V, M, RR, st, stats, mg, mt = oracle.drift_groups_merge(x, v, m, rc, R, f, np.array([0, 0]), p, h)
    assert st == 0
    np.testing.assert_array_equal(mg, [[0, 0, 1]])
    mu = p["G"] * m.sum()
    E = math.acos(1 - 2 * f * R.sum() / r0)
    tc = math.sqrt(r0 ** 3 / (8 * mu)) * (math.pi - E + math.sin(E))
    assert abs(mt[0] - tc) < 1e-14 * tc
    assert M[0] == m[0] + m[1] and M[1] == 0.0
    assert abs(RR[0] ** 3 - (R ** 3).sum()) < 1e-15 * (R ** 3).sum() and RR[1] == 0.0
    xcm = (m[:, None] * x).sum(0) / m.sum(); vcm = (m[:, None] * v).sum(0) / m.sum()
    np.testing.assert_allclose(X[0], xcm + vcm * h, rtol=0, atol=1e-15)
    np.testing.assert_allclose(V[0], vcm, rtol=0, atol=1e-17)
    assert abs(np.linalg.norm(X[1]) - 1e6) < 1e-6


def test_merge_conserves_mass_momentum_volume_in_a_cluster(params):
    """Six bodies on crossing paths with a negligible central mass: every merger conserves mass,
    momentum and volume, so over the whole drift the totals stay fixed, the centre of mass moves
    uniformly, and the log names each removed body once, always a higher index than its
    survivor."""
    p = dict(params, m0=1e-30)
    rng = np.random.default_rng(7)
    k = 6
    x = 1.0 + 2e-3 * rng.standard_normal((k, 3))
    v = 0.02 * rng.standard_normal((k, 3))
    v -= v.mean(0)
    v += x.mean(0) - x                           # converging flow: several contacts
    m = rng.uniform(1e-6, 4e-6, k)
    R = rng.uniform(2e-4, 4e-4, k)
    rc = np.full(k, 0.2)
    h = 0.05
    X, V, M, RR, st, stats, mg, mt = oracle.drift_groups_merge(x, v, m, rc, R, 1.0, np.zeros(k), p, h)
    assert st == 0 and len(mg) >= 2
    assert (mg[:, 1] < mg[:, 2]).all() and len(set(mg[:, 2])) == len(mg)
    assert (np.diff(mt) >= 0).all() and mt[-1] <= h
    alive = M > 0
    assert alive.sum() == k - len(mg)
    assert abs(M.sum() - m.sum()) < 1e-15 * m.sum()
    assert abs((RR ** 3).sum() - (R ** 3).sum()) < 1e-14 * (R ** 3).sum()
    P0 = (m[:, None] * v).sum(0); P1 = (M[:, None] * V).sum(0)
    np.testing.assert_allclose(P1, P0, rtol=0, atol=1e-15 * np.abs(m[:, None] * v).sum())
    xcm0 = (m[:, None] * x).sum(0) / m.sum(); xcm1 = (M[alive, None] * X[alive]).sum(0) / M.sum()
    np.testing.assert_allclose(xcm1, xcm0 + P0 / m.sum() * h, rtol=0, atol=1e-14)
    assert np.all(np.abs(np.linalg.norm(X[~alive], axis=1) - 1e6) < 1e-6)


def test_merge_step_without_contacts_equals_hybrid_step(params, disk2048_groups):
    """With f = 0 nothing can touch: the merging step is the hybrid step bit for bit."""
    d, thr, _ = disk2048_groups
    R = d["radius"]
    a = oracle.step_merge(d["x"], d["v"], d["m"], R, 0.0, params, 3, thr=thr)
    b = oracle.step_hybrid(d["x"], d["v"], d["m"], params, 3, thr=thr)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_array_equal(a[2], d["m"])
    assert len(a[6]) == 0


# ------------------------------------------------------------------ multi-level changeover
def _level_rc(d, p, L, s):
    """Critical radii of the levels 0..L (eq. rcrit at the time steps dt / s^l), [L + 1][n]."""
    return np.array([oracle.thresholds(d["x"], d["v"], d["m"], dict(p, dt=p["dt"] / s ** l))[0]
                     for l in range(L + 1)])


def _K(q, rc, f_in):
    return oracle.changeover((q - f_in * rc) / ((1 - f_in) * rc))[0]


def test_levels_zero_is_the_hybrid_step(params, disk2048_groups):
    """Without intermediate levels the step is the hybrid step, bit for bit."""
    d, thr, _ = disk2048_groups
    a = oracle.step_levels(d["x"], d["v"], d["m"], params, 3, 0, 8, thr=thr)
    b = oracle.step_hybrid(d["x"], d["v"], d["m"], params, 3, thr=thr)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


def test_level_kick_is_the_gradient_of_its_potential(params, disk2048_groups):
    """The level-1 kick over the close pairs is minus the gradient of
    U_1 = -sum G m_i m_j [1 - K_0] K_1 / r (central differences), for the bodies it moves most."""
    d, thr, _ = disk2048_groups
    p = params
    rcl = _level_rc(d, p, 1, 8)
    pairs = oracle.encounters(d["x"], thr)
    x, m = d["x"], d["m"]
    acc = oracle.level_kick_acc(x, m, pairs, rcl, 1, p)

    def U(xx, body):
        tot = 0.0
        for i, j in pairs:
            if body not in (i, j):
                continue
            q = np.linalg.norm(xx[j] - xx[i])
            r0, r1 = max(rcl[0, i], rcl[0, j]), max(rcl[1, i], rcl[1, j])
            tot -= p["G"] * m[i] * m[j] * (1 - _K(q, r0, p["f_in"])) * _K(q, r1, p["f_in"]) / q
        return tot

    top = np.argsort(-np.abs(acc).max(1))[:4]
    assert np.abs(acc[top]).max() > 0
    eps = 1e-8
    for b in top:
        for k in range(3):
            xp = x.copy(); xp[b, k] += eps
            xq = x.copy(); xq[b, k] -= eps
            g = (U(xp, b) - U(xq, b)) / (2 * eps)
            assert abs(m[b] * acc[b, k] + g) < 1e-6 * np.abs(m[b] * acc[b]).max()


def test_deepest_level_conserves_its_HA(params, disk2048_groups):
    """The group integrator with the pair term weighted by [1 - K_0][1 - K_1] conserves
    Kepler + (-sum G m_i m_j [1 - K_0][1 - K_1]/r), and the second factor does act."""
    d, thr, lab = disk2048_groups
    p = params
    rcl = _level_rc(d, p, 1, 2)
    idx = np.flatnonzero(lab == np.argmax(np.bincount(lab)))
    x, v, m = d["x"], d["v"], d["m"]

    def HA(xx, vv):
        E = 0.0
        for a in idx:
            E += 0.5 * m[a] * (vv[a] ** 2).sum() - p["G"] * p["m0"] * m[a] / np.linalg.norm(xx[a])
        for k, a in enumerate(idx):
            for b in idx[k + 1:]:
                q = np.linalg.norm(xx[b] - xx[a])
                W = (1 - _K(q, max(rcl[0, a], rcl[0, b]), p["f_in"])) * (1 - _K(q, max(rcl[1, a], rcl[1, b]), p["f_in"]))
                E -= p["G"] * m[a] * m[b] * W / q
        return E

    x2, v2, st = oracle.ce_drift_group_levels(x, v, m, rcl, p, idx, p["dt"])
    assert st == 0
    assert abs(HA(x2, v2) - HA(x, v)) < 1e-14 * abs(HA(x, v))
    x1, v1, _ = oracle.ce_drift_group_levels(x, v, m, rcl[:1], p, idx, p["dt"])
    assert np.abs(x2[idx] - x1[idx]).max() > 1e-12


def test_levels_step_conserves_full_energy(params, disk2048_groups):
    """One and two intermediate levels keep the hybrid step's conservation of the full energy E
    (2048 disk, 20 steps: ~1.5e-10, against ~2e-9 for the plain step) and hand only small groups to
    the direct integrator."""
    d, thr, _ = disk2048_groups
    E0 = oracle.energy(d["x"], d["v"], d["m"], params, thr)
    for L, s in ((1, 8), (2, 4)):
        x, v, m, R, st, stats, mg, mt = oracle.step_levels(d["x"], d["v"], d["m"], params, 20, L, s, thr=thr)
        E1 = oracle.energy(x, v, m, params, thr)
        assert st == 0 and stats[1] <= 3
        assert abs(E1["E"] - E0["E"]) < 3e-10 * abs(E0["E"])


def test_level_drift_converges_to_the_HA_flow(params, disk2048_groups):
    """The drift through one intermediate level is a Strang splitting of H_A = Kepler + [1 - K_0] U
    over the close pairs: H_A is conserved up to the splitting error, which falls as the substep
    factor grows (measured 2e-11 at s = 2, 3e-14 at s = 32)."""
    d, thr, _ = disk2048_groups
    p = params
    x, v, m = d["x"], d["v"], d["m"]
    pairs = oracle.encounters(x, thr)
    S0 = np.unique(pairs.ravel())

    def HA(xx, vv, rc0):
        E = (0.5 * m[S0] * (vv[S0] ** 2).sum(1) - p["G"] * p["m0"] * m[S0] / np.linalg.norm(xx[S0], axis=1)).sum()
        for i, j in pairs:
            q = np.linalg.norm(xx[j] - xx[i])
            E -= p["G"] * m[i] * m[j] * (1 - _K(q, max(rc0[i], rc0[j]), p["f_in"])) / q
        return E

    errs = {}
    for s in (2, 32):
        th = [oracle.thresholds(x, v, m, dict(p, dt=p["dt"] / s ** l)) for l in range(2)]
        lv = tuple(np.array([t[k] for t in th]) for k in range(3))
        x1, v1, st = oracle.drift_levels(x, v, m, pairs, lv, p, 1, s, p["dt"])
        assert st == 0
        errs[s] = abs(HA(x1, v1, lv[0][0]) - HA(x, v, lv[0][0])) / abs(HA(x, v, lv[0][0]))
    assert errs[32] < 1e-12 and errs[32] < errs[2] / 50


def test_list_margin_changes_only_the_list(params, disk2048_groups):
    """Listing close pairs at (1 + margin) rc (thresholds H (1+margin)^6, V (1+margin)^2) leaves the
    kick bit for bit (beyond rc the changeover weight is K/r^3 - K'/r^2 = 1/r^3, the far-pair
    weight) and gives a list that contains the list at rc."""
    d, (rc, H, V), _ = disk2048_groups
    g = 1.5
    g2 = g * g
    H2, V2 = H * ((g2 * g2) * g2), V * g2
    a0 = oracle.kick_acc(d["x"], d["m"], (rc, H, V), params)[0]
    a1 = oracle.kick_acc(d["x"], d["m"], (rc, H2, V2), params)[0]
    np.testing.assert_array_equal(a0, a1)
    p0 = {tuple(r) for r in oracle.encounters(d["x"], (rc, H, V)).tolist()}
    p1 = {tuple(r) for r in oracle.encounters(d["x"], (rc, H2, V2)).tolist()}
    assert p0 < p1 and len(p1) > 2 * len(p0)
