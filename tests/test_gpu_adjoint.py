"""GPU parity of the reverse-mode kernels against the oracle's forward-mode (dual-number)
derivatives: for every map M and random directions, <VJP_gpu(lam), delta> = <lam, JVP_oracle(delta)>
(dot-product test), plus the checkpointed gradient of the adjoint workload.

Tolerances: single maps 1e-11 relative to sum |lam_i| |Jdelta_i|; several steps 1e-9 (the two
trajectories differ by roundoff, which the step Jacobian amplifies).
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


def dev4(a3, col3=None):
    n = a3.shape[0]
    out = np.zeros((n, 4))
    out[:, :3] = a3
    if col3 is not None:
        out[:, 3] = col3
    return torch.tensor(out, device=DEV)


def cluster(n, ncl, seed=2):
    d = diskgen.workload("disk2048", n=n)
    rng = np.random.default_rng(seed)
    d["x"][:ncl] = d["x"][0] + 0.01 * rng.standard_normal((ncl, 3))
    d["v"][:ncl] = d["v"][0] + 1e-3 * rng.standard_normal((ncl, 3))
    return d


def directions(n, m, seed=9):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((n, 3)), rng.standard_normal((n, 3)), rng.standard_normal(n) * m,
            rng.standard_normal((n, 3)), rng.standard_normal((n, 3)), rng.standard_normal(n))


def rel(a, b, scale):
    return abs(a - b) / scale


def test_kick_vjp_dot_test(ctx):
    p = diskgen.PARAMS
    for name, d in (("disk n=700", diskgen.workload("disk2048", n=700)), ("cluster n=400", cluster(400, 60))):
        say(f"kick vjp {name}")
        x, v, m = d["x"], d["v"], d["m"]
        n = len(m)
        dx, _, dm, lv, _, _ = directions(n, m)
        thr_o = oracle.thresholds(x, v, m, p)
        jv = oracle.kick_jvp(x, m, thr_o, p, dx, dm)
        h = 0.37
        X = dev4(x, m)
        thr = ctx.rcrit(X, dev4(v))
        LX = torch.zeros_like(X)
        ctx.kick_vjp(X, thr, h, dev4(lv), LX)
        g = LX.cpu().numpy()
        lhs = (g[:, :3] * dx).sum() + (g[:, 3] * dm).sum()
        rhs = h * (lv * jv).sum()
        scale = h * np.abs(lv * jv).sum()
        assert rel(lhs, rhs, scale) < 1e-11, (lhs, rhs)


def test_jump_vjp_dot_test(ctx):
    say("jump vjp n=500")
    p = diskgen.PARAMS
    d = diskgen.workload("disk2048", n=500)
    x, v, m = d["x"], d["v"], d["m"]
    dx, dv, dm, lx, lv, _ = directions(500, m)
    h = 0.05
    jx = oracle.jump_jvp(x, v, m, p, h, dx, dv, dm)
    LX = dev4(lx)
    LV = dev4(lv)
    ctx.jump_vjp(dev4(x, m), dev4(v), h, LX, LV)
    gx, gv = LX.cpu().numpy(), LV.cpu().numpy()
    # the map (x, v, m) -> (x + h P/m0, v, m): v passes through, so <lam_v, dv> is on both sides
    lhs = (gx[:, :3] * dx).sum() + (gv[:, :3] * dv).sum() + (gx[:, 3] * dm).sum()
    rhs = (lx * jx).sum() + (lv * dv).sum()
    assert rel(lhs, rhs, np.abs(lx * jx).sum() + np.abs(lv * dv).sum()) < 1e-12
    assert np.array_equal(gx[:, :3], lx)       # positions' adjoint passes through


def test_drift_vjp_dot_test(ctx):
    p = diskgen.PARAMS
    d = diskgen.workload("disk2048", n=600)
    x, v, m = d["x"].copy(), d["v"].copy(), d["m"]
    # a few unbound and eccentric bodies as well
    v[:20] *= 1.5
    v[20:40] *= 1.25
    dx, dv, _, lx, lv, _ = directions(600, m)
    for h in (p["dt"], -0.4, 3.0):
        say(f"drift vjp h={h}")
        jx, jvv = oracle.drift_jvp(x, v, p, h, dx, dv)
        LX, LV = dev4(lx), dev4(lv)
        ctx.drift_vjp(dev4(x, m), dev4(v), h, LX, LV)
        gx, gv = LX.cpu().numpy()[:, :3], LV.cpu().numpy()[:, :3]
        per_body_lhs = (gx * dx).sum(1) + (gv * dv).sum(1)
        per_body_rhs = (lx * jx).sum(1) + (lv * jvv).sum(1)
        scale = np.abs(lx * jx).sum(1) + np.abs(lv * jvv).sum(1)
        assert (np.abs(per_body_lhs - per_body_rhs) / scale).max() < 1e-10


def test_step_vjp_dot_test(ctx):
    say("step vjp n=300 x5")
    p = diskgen.PARAMS
    d = cluster(300, 40, seed=4)
    x, v, m = d["x"], d["v"], d["m"]
    dx, dv, dm, lx, lv, _ = directions(300, m, seed=5)
    k = 5
    xo, vo, jx, jv, st = oracle.step_jvp(x, v, m, p, k, dx, dv, dm)
    X, V = dev4(x, m), dev4(v)
    thr = ctx.rcrit(X, V)
    LX, LV = dev4(lx), dev4(lv)
    ctx.step_vjp(X, V, thr, k, LX, LV)
    gx, gv = LX.cpu().numpy(), LV.cpu().numpy()
    lhs = (gx[:, :3] * dx).sum() + (gv[:, :3] * dv).sum() + (gx[:, 3] * dm).sum()
    rhs = (lx * jx).sum() + (lv * jv).sum()
    scale = np.abs(lx * jx).sum() + np.abs(lv * jv).sum()
    say(f"  rel {rel(lhs, rhs, scale):.2e}")
    assert rel(lhs, rhs, scale) < 1e-9


def test_checkpointed_equals_single_segment_bitwise(nb, ctx):
    say("checkpointing n=256 x12")
    from paper_2604_09184_amd.autograd import trajectory
    d = diskgen.workload("disk2048", n=256)
    grads = []
    for every in (3, 12, 5):
        X = dev4(d["x"], d["m"]).requires_grad_(True)
        V = dev4(d["v"]).requires_grad_(True)
        xT, vT = trajectory(ctx, X, V, 12, every=every)
        loss = (xT[:, :3] ** 2).sum() + (vT[:, :3] ** 2).sum()
        loss.backward()
        grads.append((X.grad.clone(), V.grad.clone(), xT.detach().clone()))
    for g in grads[1:]:
        assert torch.equal(g[2], grads[0][2])
        assert torch.equal(g[0], grads[0][0]) and torch.equal(g[1], grads[0][1])


def _loss_setup(n, nsteps):
    d = diskgen.workload("adjoint8192") if n is None else diskgen.workload("adjoint8192", n=n)
    p = diskgen.PARAMS
    xT, _, _ = oracle.step(d["x"], d["v"], d["m"], p, nsteps)
    target = diskgen.loss_target(xT)
    return d, target


def test_adjoint_subset_n64_against_oracle_gradient(ctx):
    """Bodies 0..63 of the adjoint workload as a standalone system, 100 steps: the full gradient
    of L = sum |x(T) - target|^2 against one oracle JVP per input coordinate."""
    say("adjoint n=64 x100 full gradient")
    from paper_2604_09184_amd.autograd import trajectory
    p = diskgen.PARAMS
    d, target = _loss_setup(64, 100)
    gx_o, gv_o, gm_o = oracle.grad_loss_jvp(d["x"], d["v"], d["m"], p, 100, target)
    X = dev4(d["x"], d["m"]).requires_grad_(True)
    V = dev4(d["v"]).requires_grad_(True)
    xT, vT = trajectory(ctx, X, V, 100, every=10)
    T = torch.tensor(target, device=DEV)
    loss = ((xT[:, :3] - T) ** 2).sum()
    loss.backward()
    gx = X.grad.cpu().numpy()
    gv = V.grad.cpu().numpy()
    for got, ref in ((gx[:, :3], gx_o), (gv[:, :3], gv_o), (gx[:, 3], gm_o)):
        err = np.abs(got - ref).max() / np.abs(ref).max()
        say(f"  rel err {err:.2e}")
        assert err < 1e-8
    # central differences of the oracle loss for a few coordinates
    thr = oracle.thresholds(d["x"], d["v"], d["m"], p)
    for (i, c) in ((0, 0), (17, 2), (63, 1)):
        eps = 1e-7
        xp = d["x"].copy(); xp[i, c] += eps
        xn = d["x"].copy(); xn[i, c] -= eps
        Lp = ((oracle.step(xp, d["v"], d["m"], p, 100, thr=thr)[0] - target) ** 2).sum()
        Ln = ((oracle.step(xn, d["v"], d["m"], p, 100, thr=thr)[0] - target) ** 2).sum()
        fd = (Lp - Ln) / (2 * eps)
        assert abs(fd - gx[i, c]) < 1e-5 * np.abs(gx[:, :3]).max()


def test_adjoint_full_size_n8192(ctx):
    """The adjoint workload at full size (N = 8192, 100 steps, checkpoint every 10): gradient
    along a random direction against central differences of the GPU loss, and one oracle JVP over
    the first 10 steps (dot-product test)."""
    say("adjoint n=8192 x100")
    from paper_2604_09184_amd.autograd import trajectory
    p = diskgen.PARAMS
    d = diskgen.workload("adjoint8192")
    X0 = dev4(d["x"], d["m"])
    V0 = dev4(d["v"])
    thr = ctx.rcrit(X0, V0)
    xT = X0.clone(); vT = V0.clone()
    ctx.step(xT, vT, 100, thr=thr)
    target = xT[:, :3] + 1e-4 * torch.randn(xT[:, :3].shape, generator=torch.Generator(device=DEV).manual_seed(3),
                                             device=DEV, dtype=torch.float64)
    X = X0.clone().requires_grad_(True)
    V = V0.clone().requires_grad_(True)
    xs, vs = trajectory(ctx, X, V, 100, every=10, thr=thr)
    loss = ((xs[:, :3] - target) ** 2).sum()
    loss.backward()
    rng = np.random.default_rng(21)
    dxn = rng.standard_normal((8192, 3)); dvn = rng.standard_normal((8192, 3)) * 0.1
    dX = dev4(dxn); dV = dev4(dvn)
    dirderiv = float((X.grad * dX).sum() + (V.grad * dV).sum())

    def L_at(eps):
        x = X0 + eps * dX; v = V0 + eps * dV
        ctx.step(x, v, 100, thr=thr)
        return float(((x[:, :3] - target) ** 2).sum())
    eps = 1e-8
    fd = (L_at(eps) - L_at(-eps)) / (2 * eps)
    say(f"  directional derivative {dirderiv:.6e} fd {fd:.6e}")
    assert abs(fd - dirderiv) < 1e-5 * abs(dirderiv)
    # oracle dot test over the first 10 steps
    k = 10
    xo, vo, jx, jv, _ = oracle.step_jvp(d["x"], d["v"], d["m"], p, k, dxn, dvn, None)
    rngl = np.random.default_rng(5)
    lx = rngl.standard_normal((8192, 3)); lv = rngl.standard_normal((8192, 3))
    LX, LV = dev4(lx), dev4(lv)
    ctx.step_vjp(X0, V0, thr, k, LX, LV)
    gx, gv = LX.cpu().numpy(), LV.cpu().numpy()
    lhs = (gx[:, :3] * dxn).sum() + (gv[:, :3] * dvn).sum()
    rhs = (lx * jx).sum() + (lv * jv).sum()
    scale = np.abs(lx * jx).sum() + np.abs(lv * jv).sum()
    say(f"  10-step dot test rel {abs(lhs - rhs) / scale:.2e}")
    assert abs(lhs - rhs) / scale < 1e-9
