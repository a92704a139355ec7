"""Conservative predictor with consistent mass/momentum transport (Sec.
"Multiphase incompressible Navier-Stokes solution"), computed by the gfx950
library through its C ABI, against the FP64 CPU oracle.  The predictor is
elementwise (1e-13, beta too); a whole step with the CG count forced to
the oracle's agrees to 1e-10 per field (relative L2 and elementwise on the
field's natural scale, tests/gates.py).

The carried face density stays positive only while the outflow Courant
number is at most 1/2.  On the half-resolution C2 tank the flow along the
cylinder's waterline speeds up: with the time step fixed from the initial
field the oracle reports a non-positive density within a dozen steps, and
the library must refuse that step (NS_EUNSTABLE); with the time step of the
CFL rule at every step both run forty steps, and the library matches the
oracle step by step."""
import numpy as np
import pytest

from gates import Scales, gate, gate_fields, gate_velocity, host
from paper_2206_07732_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = ["tiny2d", "tiny3d"]


def _ns():
    from paper_2206_07732_amd import ns
    return ns


def workload(name, **over):
    return I.workload(name, consistent=1, **over)


def cfl_dt(orc, wl, f, cfl=None):
    return orc.cfl_dt(orc.params(wl), f, wl.cfl if cfl is None else cfl, wl.dt_max)


def make_solver(wl, fields, **opts):
    ns = _ns()
    dev = ns.device_fields(fields)
    return ns.Solver(ns.params(wl, **opts), dev), dev


@pytest.mark.parametrize("name", CASES)
def test_consistent_predictor_and_beta(orc, name):
    wl = workload(name)
    f = I.make_fields(wl)
    dt = cfl_dt(orc, wl, f)
    P = orc.params(wl)
    sc = Scales(wl, f, dt)
    S, dev = make_solver(wl, f)
    S.momentum_step(dt, dt)          # rho^n from the fields as they are (t = 0)
    torch.cuda.synchronize()
    rho_n = orc.properties(P, f["sigma"], 0.0)[0]
    (us, vs, ws), rb = orc.momentum_cons(P, f["u"], f["v"], f["w"], f["sigma"], dt, dt, rho_n)
    assert orc.last_flags() == 0
    gate_velocity(f"consistent predictor {name}", [S.buffer(k) for k in ("us", "vs", "ws")], [us, vs, ws],
                  ("us", "vs", "ws"), 1e-13, sc)
    # the carried density of an air face is a small difference of large
    # fluxes: a few ulps of it move beta by up to ~1e-13 of 1/rho_a
    for k, r in zip(("bx", "by", "bz"), orc.face_beta_rho(P, rb, f["sigma"], dt, dt)):
        if np.linalg.norm(r) > 0:
            gate(f"consistent beta {name} {k}", S.buffer(k), r, 1e-13, sc.of(k, r))
    S.close()


@pytest.mark.parametrize("name", CASES)
def test_consistent_step_parity_forced_iterations(orc, name):
    wl = workload(name)
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
    gate_fields(f"consistent step {name}", dev, ref, ("sigma", "u", "v", "w", "p"), 1e-10, Scales(wl, f, dt))
    S.close()


def test_consistent_free_running_steps(orc):
    """Four free-running 2-D steps stay with the oracle's (the density at
    t^n of each later step is the one the previous step's properties left)."""
    wl = workload("tiny2d")
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
    gate_fields("consistent free run", dev, ref, ("sigma", "u", "w", "p"), 1e-8, Scales(wl, f, dt))
    S.close()


@pytest.mark.parametrize("name", ["fsi2d", "fsi3d"])
def test_consistent_free_heave_coupled_step_parity(orc, name):
    """A free body with consistent transport: the density the step starts
    from is that of the body before its heave update (the state at t^n);
    one coupled step with the CG count forced to the oracle's."""
    wl = workload(name)
    f = I.make_fields(wl)
    dt = cfl_dt(orc, wl, f)
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
    gate_fields(f"consistent fsi step {name}", dev, ref, ("sigma", "u", "v", "w", "p"), 1e-10, Scales(wl, f, dt))
    S.close()


def test_all_options_free_running_fsi2d(orc):
    """Free heave, consistent transport and the Crank-Nicolson viscous term
    together: three free-running coupled steps of the 2-D spar."""
    wl = I.workload("fsi2d", consistent=1, cn_sweeps=3)
    f = I.make_fields(wl)
    dt = cfl_dt(orc, wl, f)
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
    gate_fields("all options fsi2d", dev, ref, ("sigma", "u", "w", "p"), 1e-8, Scales(wl, f, dt))
    S.close()


def oracle_run(orc, wl, f0, steps, fixed_dt=None):
    """The oracle's free run: a list of (state, t, dt, rc, iters) before each step."""
    P = orc.params(wl)
    out, f, t = [], f0, 0.0
    for _ in range(steps):
        dt = fixed_dt if fixed_dt is not None else cfl_dt(orc, wl, f)
        nf, st, rc = orc.step(P, f, dt, t)
        out.append((f, t, dt, rc, st["iters"]))
        if rc:
            break
        f, t = nf, t + dt
    return out


def test_c2half_cfl_rule_forty_steps_step_by_step(orc):
    """Every third of the oracle's forty steps under the CFL rule, the library
    starts from the oracle's state: its own ns_cfl_dt gives the oracle's time
    step bit for bit, and one step with the CG count forced to the oracle's
    matches it to 1e-10."""
    wl = workload("c2half")
    f0 = I.make_fields(wl)
    run = oracle_run(orc, wl, f0, 40)
    assert len(run) == 40 and all(r[3] == 0 for r in run)
    assert max(r[4] for r in run) <= 15
    for s in list(range(0, 40, 3)) + [39]:
        f, t, dt, _, k = run[s]
        S, dev = make_solver(wl, f, max_iters=k, rtol=0.0)
        assert S.cfl_dt(wl.cfl, wl.dt_max) == dt, s
        ref, _, rc = orc.step(orc.params(wl, max_iters=k, rtol=0.0), f, dt, t)
        sg = S.step(dt, t, allow_noconv=True)
        torch.cuda.synchronize()
        assert sg["iters"] == k
        print(f"[c2half cfl] step {s}: t {t:.4f} dt {dt:.5f} iters {k}", flush=True)
        gate_fields(f"c2half cfl step {s}", dev, ref, ("sigma", "u", "v", "w", "p"), 1e-10, Scales(wl, f0, dt))
        S.close()


def test_c2half_cfl_rule_forty_steps_free_running(orc):
    """The library alone, forty steps with its own ns_cfl_dt at every step:
    no step is refused, CG stays bounded, and the tank is where the oracle's
    free run is after the same number of steps (the two runs' time steps
    are each side's own rule)."""
    wl = workload("c2half")
    f0 = I.make_fields(wl)
    S, dev = make_solver(wl, f0)
    t, iters = 0.0, []
    for s in range(40):
        dt = S.cfl_dt(wl.cfl, wl.dt_max)
        st = S.step(dt, t)
        iters.append(st["iters"])
        t += dt
    torch.cuda.synchronize()
    run = oracle_run(orc, wl, f0, 40)
    f_last, t_last, dt_last, _, _ = run[-1]
    ref, _, rc = orc.step(orc.params(wl), f_last, dt_last, t_last)
    assert rc == 0
    print(f"[c2half free] t {t:.5f} (oracle {t_last + dt_last:.5f}), iters {iters}", flush=True)
    assert max(iters) <= 15
    assert abs(t - (t_last + dt_last)) <= 1e-9 * t
    gate_fields("c2half free run", dev, ref, ("sigma", "u", "v", "w", "p"), 1e-6, Scales(wl, f0, dt))
    S.close()


def test_c2half_fixed_time_step_is_refused_where_the_oracle_fails(orc):
    """With the time step fixed from the initial field the oracle's carried
    density turns non-positive at some step s (status 2).  From the oracle's
    state before step s the library refuses the step with NS_EUNSTABLE and
    leaves the velocity as it was; from the state before step s - 1 it takes
    the step."""
    ns = _ns()
    wl = workload("c2half")
    f0 = I.make_fields(wl)
    dt0 = cfl_dt(orc, wl, f0)
    run = oracle_run(orc, wl, f0, 16, fixed_dt=dt0)
    f_bad, t_bad, _, rc, _ = run[-1]
    assert rc == 2
    print(f"[c2half fixed] the oracle's density turns non-positive at step {len(run) - 1}", flush=True)
    f_ok, t_ok, _, _, _ = run[-2]
    S, dev = make_solver(wl, f_ok)
    S.step(dt0, t_ok)
    S.close()
    S, dev = make_solver(wl, f_bad)
    u_before = dev["u"].clone()
    with pytest.raises(ns.NSError) as e:
        S.step(dt0, t_bad)
    print(f"[c2half fixed] {e.value}", flush=True)
    assert e.value.status == ns.NS_EUNSTABLE
    assert torch.equal(dev["u"], u_before)
    S.close()
