"""Conservative predictor with consistent mass/momentum transport (Sec.
"Multiphase incompressible Navier-Stokes solution"), computed by the gfx950
library through its C ABI, against the FP64 CPU oracle.  The predictor is
elementwise (1e-13 relative; beta 1e-14); a whole step with the CG count
forced to the oracle's agrees to 1e-10 relative per field."""
import numpy as np
import pytest

from paper_2206_07732_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = ["tiny2d", "tiny3d"]


def _ns():
    from paper_2206_07732_amd import ns
    return ns


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(np.asarray(a) - b) / (nb if nb > 0 else 1.0))


def workload(name):
    wl = I.workload(name)
    wl.consistent = 1
    return wl


def make_solver(wl, fields, **opts):
    ns = _ns()
    dev = ns.device_fields(fields)
    return ns.Solver(ns.params(wl, **opts), dev), dev


@pytest.mark.parametrize("name", CASES)
def test_consistent_predictor_and_beta(orc, name):
    wl = workload(name)
    f = I.make_fields(wl)
    dt = I.cfl_dt(wl, f)
    P = orc.params(wl)
    S, dev = make_solver(wl, f)
    S.momentum_step(dt, dt)          # rho^n from the fields as they are (t = 0)
    torch.cuda.synchronize()
    rho_n = orc.properties(P, f["sigma"], 0.0)[0]
    (us, vs, ws), rb = orc.momentum_cons(P, f["u"], f["v"], f["w"], f["sigma"], dt, dt, rho_n)
    for k, r in (("us", us), ("vs", vs), ("ws", ws)):
        g = host(S.buffer(k))
        print(f"[consistent predictor] {name} {k} rel={rel(g, r):.2e}", flush=True)
        if np.linalg.norm(r) > 0:
            assert rel(g, r) < 1e-13, k
    for k, r in zip(("bx", "by", "bz"), orc.face_beta_rho(P, rb, f["sigma"], dt, dt)):
        if np.linalg.norm(r) > 0:
            assert rel(host(S.buffer(k)), r) < 1e-14, k
    S.close()


@pytest.mark.parametrize("name", CASES)
def test_consistent_step_parity_forced_iterations(orc, name):
    wl = workload(name)
    f = I.make_fields(wl)
    dt = I.cfl_dt(wl, f)
    _, st, rc = orc.step(orc.params(wl), f, dt, 0.0)
    assert rc == 0
    k = st["iters"]
    ref, _, _ = orc.step(orc.params(wl, max_iters=k, rtol=0.0), f, dt, 0.0)
    S, dev = make_solver(wl, f, max_iters=k, rtol=0.0)
    sg = S.step(dt, 0.0, allow_noconv=True)
    torch.cuda.synchronize()
    assert sg["iters"] == k
    for key in ("sigma", "u", "v", "w", "p"):
        r = rel(host(dev[key]), ref[key])
        print(f"[consistent step parity] case={name} field={key} rel={r:.2e}", flush=True)
        if np.linalg.norm(ref[key]) > 0:
            assert r < 1e-10, key
    S.close()


def test_consistent_free_running_steps(orc):
    """Four free-running 2-D steps stay with the oracle's (the density at
    t^n of each later step is the one the previous step's properties left)."""
    wl = workload("tiny2d")
    f = I.make_fields(wl)
    dt = I.cfl_dt(wl, f)
    P = orc.params(wl)
    S, dev = make_solver(wl, f)
    ref = f
    t = 0.0
    for s in range(4):
        ref, _, rc = orc.step(P, ref, dt, t)
        assert rc == 0
        S.step(dt, t)
        t += dt
    torch.cuda.synchronize()
    for key in ("sigma", "u", "w", "p"):
        r = rel(host(dev[key]), ref[key])
        print(f"[consistent free run] field={key} rel={r:.2e}", flush=True)
        assert r < 1e-8, key
    S.close()


@pytest.mark.parametrize("name", ["fsi2d", "fsi3d"])
def test_consistent_free_heave_coupled_step_parity(orc, name):
    """A free body with consistent transport: the density the step starts
    from is that of the body before its heave update (the state at t^n);
    one coupled step with the CG count forced to the oracle's."""
    wl = workload(name)
    f = I.make_fields(wl)
    dt = I.cfl_dt(wl, f)
    _, st, rc, _ = orc.step_fsi(orc.params(wl), f, dt, 0.0)
    assert rc == 0
    k = st["iters"]
    Pk = orc.params(wl, max_iters=k, rtol=0.0)
    ref, _, _, _ = orc.step_fsi(Pk, f, dt, 0.0)
    S, dev = make_solver(wl, f, max_iters=k, rtol=0.0)
    sg = S.step(dt, 0.0, allow_noconv=True)
    torch.cuda.synchronize()
    assert sg["iters"] == k
    b = S.body_state(0)
    assert abs(b["zeta"] - Pk.body[0].zeta) <= 1e-12 * abs(Pk.body[0].zeta) + 1e-15
    for key in ("sigma", "u", "v", "w", "p"):
        r = rel(host(dev[key]), ref[key])
        print(f"[consistent fsi step parity] case={name} field={key} rel={r:.2e}", flush=True)
        if np.linalg.norm(ref[key]) > 0:
            assert r < 1e-10, key
    S.close()


def test_all_options_free_running_fsi2d(orc):
    """Free heave, consistent transport and the Crank-Nicolson viscous term
    together: three free-running coupled steps of the 2-D spar."""
    wl = I.workload("fsi2d", consistent=1, cn_sweeps=3)
    f = I.make_fields(wl)
    dt = I.cfl_dt(wl, f)
    P = orc.params(wl)
    S, dev = make_solver(wl, f)
    ref = f
    t = 0.0
    for s in range(3):
        ref, _, rc, _ = orc.step_fsi(P, ref, dt, t)
        assert rc == 0
        S.step(dt, t)
        t += dt
    torch.cuda.synchronize()
    b = S.body_state(0)
    print(f"[all options fsi2d] zeta {b['zeta']:+.3e} oracle {P.body[0].zeta:+.3e}", flush=True)
    assert abs(b["zeta"] - P.body[0].zeta) <= 1e-9 * abs(P.body[0].zeta) + 1e-15
    for key in ("sigma", "u", "w", "p"):
        r = rel(host(dev[key]), ref[key])
        print(f"[all options fsi2d] field={key} rel={r:.2e}", flush=True)
        assert r < 1e-8, key
    S.close()
