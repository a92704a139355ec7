"""The learned initial guess on the GPU: network forward and gradients against
the oracle's bfloat16 emulation, training, feature construction and the
learned guess inside the projection.

Tolerances: the GPU stores activations and activation gradients in bfloat16
(relative rounding 2^-9) and sums in FP32, the oracle rounds the same
activations but keeps gradients in FP64, so outputs agree to about 1e-2 and
weight gradients to a few 1e-2 (relative L2)."""
import numpy as np
import pytest

from oracle import net_oracle as N
from paper_2206_07732_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _ns():
    from paper_2206_07732_amd import ns
    return ns


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, dtype=np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def random_beta(nx, ny, nz, seed):
    """Positive face coefficients with zero walls (x, y, bottom) as FP32 device tensors."""
    rng = np.random.default_rng(seed)
    bx = np.exp(rng.standard_normal((nz, ny, nx + 1)))
    by = np.exp(rng.standard_normal((nz, ny + 1, nx)))
    bz = np.exp(rng.standard_normal((nz + 1, ny, nx)))
    bx[:, :, 0] = bx[:, :, -1] = 0
    by[:, 0] = by[:, -1] = 0
    bz[0] = 0
    b32 = [a.astype(np.float32) for a in (bx, by, bz)]
    return b32, tuple(torch.from_numpy(a).cuda() for a in b32)


def test_param_count_matches_oracle():
    assert _ns().net_param_count() == N.param_count()


@pytest.mark.parametrize("dims", [(16, 8, 8), (24, 12, 8)])
def test_forward_matches_oracle_bf16(dims):
    ns = _ns()
    nx, ny, nz = dims
    rng = np.random.default_rng(sum(dims))
    theta = N.he_init(7)
    theta[-161:] = rng.standard_normal(161) * 0.05
    feat = rng.standard_normal((4, nz, ny, nx)).astype(np.float32)
    net = ns.Net(nx, ny, nz)
    net.set_params(theta)
    assert np.array_equal(net.get_params(), theta.astype(np.float32))
    out = net.forward(torch.from_numpy(feat).cuda()).cpu().numpy()
    ref, _ = N.forward(N.unflatten(theta.astype(np.float32).astype(np.float64)), feat.astype(np.float64), bf16=True)
    r = rel(out, ref)
    print(f"[net fwd] dims={dims} rel={r:.2e}", flush=True)
    assert r < 1e-2


def test_gradients_match_oracle(orc):
    ns = _ns()
    nx, ny, nz = 16, 8, 8
    rng = np.random.default_rng(3)
    theta = N.he_init(11)
    theta[-161:] = rng.standard_normal(161) * 0.05
    th32 = theta.astype(np.float32).astype(np.float64)
    feat = rng.standard_normal((4, nz, ny, nx)).astype(np.float32)
    target = (rng.standard_normal((nz, ny, nx)) * 0.3).astype(np.float32)
    (bx, by, bz), beta = random_beta(nx, ny, nz, 4)
    net = ns.Net(nx, ny, nz, training=True)
    net.set_params(theta)
    loss = net.train_step(torch.from_numpy(feat).cuda(), torch.from_numpy(target).cuda(), beta, 1e-3, update=False)
    g = net.get_grads()
    out, cache = N.forward(N.unflatten(th32), feat.astype(np.float64), bf16=True)
    op = lambda x: orc.apply_A(nx, ny, nz, 1.0, bx.astype(np.float64), by.astype(np.float64),
                               bz.astype(np.float64), x)
    L, dout = N.energy_loss_and_grad(out, target.astype(np.float64), op)
    gr = N.backward(cache, dout)
    print(f"[net grad] loss gpu={loss:.6f} oracle={L:.6f}", flush=True)
    assert abs(loss - L) < 1e-2 * L
    G = N.unflatten(g.astype(np.float64))
    for k in gr:
        r = rel(G[k], gr[k])
        print(f"[net grad] {k} rel={r:.2e}", flush=True)
        assert r < 5e-2, k


def test_training_reduces_loss():
    ns = _ns()
    nx, ny, nz = 16, 16, 8
    rng = np.random.default_rng(5)
    teacher = N.he_init(21)
    _, beta = random_beta(nx, ny, nz, 6)
    samples = []
    for s in range(4):
        feat = rng.standard_normal((4, nz, ny, nx))
        t, _ = N.forward(N.unflatten(teacher), feat)
        samples.append((torch.from_numpy(feat.astype(np.float32)).cuda(),
                        torch.from_numpy(t.astype(np.float32)).cuda()))
    net = ns.Net(nx, ny, nz, training=True)
    net.set_params(N.he_init(22, zero_head=True))
    first = np.mean([net.train_step(f, t, beta, 1e-3, update=False) for f, t in samples])
    assert abs(first - 1.0) < 1e-6            # zero head: the guess is p_prev
    for epoch in range(40):
        for f, t in samples:
            net.train_step(f, t, beta, 2e-3)
    last = np.mean([net.train_step(f, t, beta, 1e-3, update=False) for f, t in samples])
    print(f"[net train] loss {first:.4f} -> {last:.4f}", flush=True)
    assert last < 0.5 * first


def test_features_match_oracle(orc):
    ns = _ns()
    wl = I.workload("tiny3d")
    f = I.make_fields(wl)
    dt = I.cfl_dt(wl, f)
    dev = ns.device_fields(f)
    S = ns.Solver(ns.params(wl), dev)
    S.levelset_advect_reinit(dt)
    S.momentum_step(dt, dt)
    pprev = torch.from_numpy(np.random.default_rng(1).standard_normal(f["p"].shape) * 1e3).cuda()
    feat = torch.empty((4,) + f["p"].shape, dtype=torch.float32, device="cuda")
    S.features(dt, pprev, feat)
    torch.cuda.synchronize()
    Po = orc.params(wl)
    us, vs, ws = (S.buffer(k).cpu().numpy() for k in ("us", "vs", "ws"))
    bx, by, bz = (S.buffer(k).cpu().numpy() for k in ("bx", "by", "bz"))
    b = orc.rhs(Po, us, vs, ws, dt)
    rho = S.buffer("rho").cpu().numpy()
    pp = pprev.cpu().numpy()
    r0 = b - orc.apply_A(wl.nx, wl.ny, wl.nz, wl.h, bx, by, bz, pp)
    P0 = wl.rho_w * wl.g * wl.depth
    ref = N.features(b, rho, pp, r0, wl.h, wl.rho_w, wl.rho_a, P0)
    got = feat.cpu().numpy()
    for c in range(4):
        assert rel(got[c], ref[c]) < 1e-6, c


def test_learned_guess_in_projection():
    ns = _ns()
    wl = I.workload("tiny3d")
    f = I.make_fields(wl)
    dt = I.cfl_dt(wl, f)
    net = ns.Net(wl.nx, wl.ny, wl.nz)
    net.set_params(N.he_init(3) * 0.1)
    dev = ns.device_fields(f)
    S = ns.Solver(ns.params(wl, x0=ns.X0_LEARNED), dev)
    S.attach_net(net)
    t = 0.0
    for s in range(3):
        st = S.step(dt, t)
        t += dt
        assert st["converged"] == 1 and st["true_rel_resid"] <= 1e-10 and st["x0_fallback"] == 0
    # a non-finite network output falls back to the previous pressure
    bad = N.he_init(3)
    bad[-1] = np.nan            # head bias: every delta is NaN (a ReLU would swallow an inner NaN)
    net.set_params(bad)
    st = S.step(dt, t)
    assert st["x0_fallback"] == 1 and st["converged"] == 1
    # without an attached network the learned guess is refused
    S2 = ns.Solver(ns.params(wl, x0=ns.X0_LEARNED), ns.device_fields(f))
    S2.levelset_advect_reinit(dt)
    S2.momentum_step(dt, dt)
    with pytest.raises(ns.NSError):
        S2.projection_solve(dt)
