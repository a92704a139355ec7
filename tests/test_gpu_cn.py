"""Crank-Nicolson viscous term (Sec. "Time stepping scheme") computed by the
gfx950 library through its C ABI against the FP64 CPU oracle.

The oracle solves the Crank-Nicolson system to convergence (Gauss-Seidel to
round-off); the library runs batches of point-Jacobi sweeps until the last
sweep of a batch changes no face by more than cn_tol of the largest |u*|.
Each sweep contracts the error by roughly nu dt/h^2, so at the default
cn_tol = 1e-10 the predictor is within 1e-10 of the system's solution and
at cn_tol = 1e-14 within 1e-12: the tests gate those, relative L2 and
elementwise on the flow's velocity scale (tests/gates.py).  A whole step
with the CG count forced to the oracle's agrees to 1e-10.  Batches of one
and of two sweeps cover both ends of the iterate ping-pong and the copy
back after an odd number of extra batches; the viscous variant (nu = 0.01
in both phases) needs several batches.  A viscosity far past the Jacobi
bound is refused with an error instead of an unconverged predictor."""
import numpy as np
import pytest

from gates import Scales, gate, gate_fields, gate_velocity, host, velocity_norm
from paper_2206_07732_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _ns():
    from paper_2206_07732_amd import ns
    return ns


def workload(name, sweeps, viscous=False, consistent=0, nu=0.01):
    over = dict(cn_sweeps=sweeps, consistent=consistent)
    if viscous:
        wl0 = I.workload(name)
        over.update(mu_w=nu * wl0.rho_w, mu_a=nu * wl0.rho_a)
    return I.workload(name, **over)


def cfl_dt(orc, wl, f):
    return orc.cfl_dt(orc.params(wl), f, wl.cfl, wl.dt_max)


def make_solver(wl, fields, **opts):
    ns = _ns()
    dev = ns.device_fields(fields)
    return ns.Solver(ns.params(wl, **opts), dev), dev


def oracle_predictor(orc, wl, f, dt):
    """The oracle's Crank-Nicolson predictor (converged) and its status."""
    P = orc.params(wl)
    if wl.consistent:
        rho_n = orc.properties(P, f["sigma"], 0.0)[0]
        ref = orc.momentum_cons(P, f["u"], f["v"], f["w"], f["sigma"], dt, dt, rho_n)[0]
    else:
        ref = orc.momentum(P, f["u"], f["v"], f["w"], f["sigma"], dt, dt)
    assert orc.last_flags() == 0
    return ref


PRED = [("tiny2d", 3, False, 0), ("tiny3d", 2, False, 0), ("tiny3d", 1, True, 0), ("tiny3d", 3, True, 0),
        ("tiny2d", 4, True, 1), ("tiny2d", 1, True, 1), ("c1nwt", 3, False, 0)]


@pytest.mark.parametrize("name,sweeps,viscous,consistent", PRED)
@pytest.mark.parametrize("cn_tol,tol", [(1e-10, 1e-10), (1e-14, 1e-12)])
def test_cn_predictor_solves_the_system(orc, name, sweeps, viscous, consistent, cn_tol, tol):
    wl = workload(name, sweeps, viscous, consistent)
    f = I.make_fields(wl)
    dt = cfl_dt(orc, wl, f)
    ref = oracle_predictor(orc, wl, f, dt)
    ex = orc.momentum(orc.params(workload(name, 0, viscous, 0)), f["u"], f["v"], f["w"], f["sigma"], dt, dt)
    S, dev = make_solver(wl, f, cn_tol=cn_tol)
    S.momentum_step(dt, dt)
    torch.cuda.synchronize()
    got = [host(S.buffer(k)).copy() for k in ("us", "vs", "ws")]
    st = S.projection_solve(dt)
    print(f"[cn predictor] {name} batch={sweeps} viscous={viscous} cons={consistent} cn_tol={cn_tol:.0e}: "
          f"{st['cn_sweeps']} sweeps", flush=True)
    assert st["cn_sweeps"] >= sweeps and st["cn_sweeps"] % sweeps == 0
    sc = Scales(wl, f, dt)
    gate_velocity(f"cn predictor {name}", got, ref, ("us", "vs", "ws"), tol, sc)
    vn = velocity_norm(ref)
    print(f"[cn predictor] Crank-Nicolson vs explicit: "
          f"{velocity_norm([r - e for r, e in zip(ref, ex)]) / vn:.2e}", flush=True)
    S.close()


def test_cn_batches_until_converged(orc):
    """With one sweep per batch the viscous tank needs several batches; the
    count the stats report is the library's own, and a tighter tolerance
    takes more of them."""
    wl = workload("tiny3d", 1, viscous=True)
    f = I.make_fields(wl)
    dt = cfl_dt(orc, wl, f)
    counts = []
    for cn_tol in (1e-6, 1e-10, 1e-14):
        S, dev = make_solver(wl, f, cn_tol=cn_tol)
        st = S.step(dt, 0.0)
        counts.append(st["cn_sweeps"])
        S.close()
    print(f"[cn batches] sweeps for cn_tol 1e-6, 1e-10, 1e-14: {counts}", flush=True)
    assert counts[0] >= 2 and counts[0] < counts[1] < counts[2] <= 64


def test_cn_refuses_a_viscosity_past_the_jacobi_bound(orc):
    """nu dt/h^2 = 2, far past the bound (1/4) under which the sweeps contract:
    the iterate grows instead of converging, and the library returns an
    error (NS_ENOCONV after 64 sweeps, or NS_ENAN if it overflows) rather
    than a predictor that does not solve the system."""
    ns = _ns()
    base = I.workload("tiny3d")
    f = I.make_fields(base)
    dt = cfl_dt(orc, base, f)
    nu = 2.0 * base.h ** 2 / dt
    wl = workload("tiny3d", 4, viscous=True, nu=nu)
    S, dev = make_solver(wl, f)
    with pytest.raises(ns.NSError) as e:
        S.step(dt, 0.0)
    print(f"[cn bound] nu dt/h^2 = 2: {e.value}", flush=True)
    assert e.value.status in (ns.NS_ENOCONV, ns.NS_ENAN)
    S.close()


@pytest.mark.parametrize("name,sweeps,viscous", [("tiny2d", 3, True), ("tiny3d", 2, False)])
def test_cn_step_parity_forced_iterations(orc, name, sweeps, viscous):
    wl = workload(name, sweeps, viscous)
    f = I.make_fields(wl)
    dt = cfl_dt(orc, wl, f)
    _, st, rc = orc.step(orc.params(wl), f, dt, 0.0)
    assert rc == 0
    k = st["iters"]
    ref, _, _ = orc.step(orc.params(wl, max_iters=k, rtol=0.0), f, dt, 0.0)
    S, dev = make_solver(wl, f, max_iters=k, rtol=0.0)
    sg = S.step(dt, 0.0, allow_noconv=True)
    torch.cuda.synchronize()
    assert sg["iters"] == k
    gate_fields(f"cn step {name}", dev, ref, ("sigma", "u", "v", "w", "p"), 1e-10, Scales(wl, f, dt))
    S.close()


def test_cn_free_running_steps(orc):
    wl = workload("tiny2d", 3, viscous=True)
    f = I.make_fields(wl)
    dt = cfl_dt(orc, wl, f)
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
    gate_fields("cn free run", dev, ref, ("sigma", "u", "w", "p"), 1e-8, Scales(wl, f, dt))
    S.close()


def test_cn_c2_predictor_solves_the_system(orc):
    """The benchmark tank (128x64x64) in the bench's configuration: batches of
    3 sweeps at cn_tol = 1e-10 against the oracle's converged solve.  nu
    dt/h^2 = 2.4e-4 here: each sweep contracts the error by ~2e-3 from a start
    ~1e-5 away (the explicit value), so one or two batches converge."""
    wl = workload("c2", 3)
    f = I.make_fields(wl)
    dt = cfl_dt(orc, wl, f)
    S, dev = make_solver(wl, f)
    S.momentum_step(dt, dt)
    torch.cuda.synchronize()
    g3 = [host(S.buffer(k)).copy() for k in ("us", "vs", "ws")]
    st = S.projection_solve(dt)
    S.close()
    # the first step starts from a velocity that jumps at the interface, so
    # it may take a second batch
    print(f"[cn c2] {st['cn_sweeps']} sweeps", flush=True)
    assert st["cn_sweeps"] in (3, 6)
    ref = oracle_predictor(orc, wl, f, dt)
    gate_velocity("cn c2 predictor", g3, ref, ("us", "vs", "ws"), 1e-10, Scales(wl, f, dt))


SHAPES = [("ragged3d", 3, 1), ("odd1level", 2, 0), ("odd1level", 3, 1)]


@pytest.mark.parametrize("name,sweeps,consistent", SHAPES)
def test_options_on_ragged_and_single_level_grids(orc, name, sweeps, consistent):
    """70x6x22 (not a multiple of the tiles, two MG levels) and 129x8x8 (odd
    nx: one level solved by the multi-block sweeps) with the Crank-Nicolson
    term, alone or with consistent transport: the predictor, then a step with
    the CG count forced to the oracle's."""
    from test_gpu_parity import case
    wl = case(name)
    wl.cn_sweeps, wl.consistent = sweeps, consistent
    f = I.make_fields(wl)
    dt = cfl_dt(orc, wl, f)
    P = orc.params(wl)
    sc = Scales(wl, f, dt)
    S, dev = make_solver(wl, f)
    S.momentum_step(dt, dt)
    torch.cuda.synchronize()
    ref = oracle_predictor(orc, wl, f, dt)
    gate_velocity(f"options {name} cons={consistent}", [S.buffer(k) for k in ("us", "vs", "ws")], ref,
                  ("us", "vs", "ws"), 1e-10, sc)
    S.close()
    _, st, rc = orc.step(P, f, dt, 0.0)
    assert rc == 0
    it = st["iters"]
    ref, _, _ = orc.step(orc.params(wl, max_iters=it, rtol=0.0), f, dt, 0.0)
    S, dev = make_solver(wl, f, max_iters=it, rtol=0.0)
    sg = S.step(dt, 0.0, allow_noconv=True)
    torch.cuda.synchronize()
    assert sg["iters"] == it
    gate_fields(f"options step {name}", dev, ref, ("sigma", "u", "v", "w", "p"), 1e-10, sc)
    S.close()


def test_wave_tank_with_both_options_step_parity(orc):
    """The 2-D wave tank (inlet, relaxation zones, vorticity damping) with
    consistent transport and the Crank-Nicolson term: a step with the CG
    count forced to the oracle's, then two free-running steps."""
    wl = workload("c1nwt", 3, consistent=1)
    f = I.make_fields(wl)
    dt = cfl_dt(orc, wl, f)
    P = orc.params(wl)
    sc = Scales(wl, f, dt)
    _, st, rc = orc.step(P, f, dt, 0.0)
    assert rc == 0
    it = st["iters"]
    ref, _, _ = orc.step(orc.params(wl, max_iters=it, rtol=0.0), f, dt, 0.0)
    S, dev = make_solver(wl, f, max_iters=it, rtol=0.0)
    sg = S.step(dt, 0.0, allow_noconv=True)
    torch.cuda.synchronize()
    assert sg["iters"] == it
    gate_fields("nwt options step", dev, ref, ("sigma", "u", "w", "p"), 1e-10, sc)
    S.close()
    S, dev = make_solver(wl, f)
    ref, t = f, 0.0
    for s in range(3):
        ref, _, rc = orc.step(P, ref, dt, t)
        assert rc == 0
        S.step(dt, t)
        t += dt
    torch.cuda.synchronize()
    gate_fields("nwt options free run", dev, ref, ("sigma", "u", "w", "p"), 1e-8, sc)
    S.close()


def test_long_free_run_wave_tank_with_both_options(orc):
    """60 free-running steps of the 2-D wave tank (about two wave periods)
    with consistent transport and the Crank-Nicolson term, checked against
    the oracle every 20 steps: the two stay together to 1e-8."""
    wl = workload("c1nwt", 3, consistent=1)
    f = I.make_fields(wl)
    dt = cfl_dt(orc, wl, f)
    P = orc.params(wl)
    sc = Scales(wl, f, dt)
    S, dev = make_solver(wl, f)
    ref, t = f, 0.0
    for s in range(60):
        ref, _, rc = orc.step(P, ref, dt, t)
        assert rc == 0
        S.step(dt, t)
        t += dt
        if (s + 1) % 20 == 0:
            torch.cuda.synchronize()
            gate_fields(f"nwt long run step {s + 1}", dev, ref, ("sigma", "u", "w", "p"), 1e-8, sc)
    S.close()
