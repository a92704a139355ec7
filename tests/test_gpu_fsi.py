"""Free heave of a body (Sec. "Fluid-structure coupling"): the hydrodynamic
force of eqn_int_fh and the heave update of eqn_newton_u, computed by the
gfx950 library through its C ABI, against the FP64 CPU oracle.

The force is a sum of a few hundred face terms whose largest parts (the
pressure on the bottom and top of the body) are of the order of the body's
weight m g; both sides form the same terms up to rounding and fused
multiply-adds and sum them in different orders, so they must agree to
1e-11 m g.  The heave update is scalar arithmetic on that force (1e-12 of
g dt).  The coupled step's fields follow the step-parity bar (1e-10
relative with the CG count forced to the oracle's)."""
import numpy as np
import pytest

from gates import Scales, gate, gate_fields
from paper_2206_07732_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = ["fsi2d", "fsi3d"]


def _ns():
    from paper_2206_07732_amd import ns
    return ns


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(np.asarray(a) - b) / (nb if nb > 0 else 1.0))


def make_solver(wl, fields, **opts):
    ns = _ns()
    dev = ns.device_fields(fields)
    return ns.Solver(ns.params(wl, **opts), dev), dev


@pytest.mark.parametrize("name", CASES)
def test_force_and_heave_follow_the_oracle_step_by_step(orc, name):
    wl = I.workload(name)
    B = wl.bodies[0]
    f = I.make_fields(wl)
    dt = orc.cfl_dt(orc.params(wl), f, wl.cfl, wl.dt_max)
    mg = B.mass * wl.g
    S, dev = make_solver(wl, f)
    # the first heave update uses the force of the initial fields
    P = orc.params(wl)
    mu0 = orc.properties(P, f["sigma"], 0.0)[2]
    F = orc.hydro_force(P, 0, f["p"], f["u"], f["v"], f["w"], mu0, 0.0)
    zeta, zdot = orc.heave_update(B.mass, B.pto_damping, wl.g, dt, F[2], B.zeta0, B.zdot0)
    t = 0.0
    for s in range(5):
        S.step(dt, t)
        torch.cuda.synchronize()
        t += dt
        st = S.body_state(0)
        print(f"[fsi] {name} step {s}: zeta {st['zeta']:+.6f} zdot {st['zdot']:+.6f} Fz {st['F'][2]:.4f} "
              f"(oracle heave {zeta:+.6f} {zdot:+.6f})", flush=True)
        assert abs(st["zeta"] - zeta) <= 1e-12 * wl.g * dt * dt * (s + 1) + 1e-15
        assert abs(st["zdot"] - zdot) <= 1e-12 * wl.g * dt
        assert st["f_pto"] == -B.pto_damping * st["zdot"]
        # the force the library computed at the end of the step, against the
        # oracle's from the same state (fields, and the body where the step left it)
        Q = orc.params(wl)
        Q.body[0].zeta, Q.body[0].zdot = st["zeta"], st["zdot"]
        fh = {k: host(v) for k, v in dev.items()}
        mu = orc.properties(Q, fh["sigma"], t)[2]
        Fo = orc.hydro_force(Q, 0, fh["p"], fh["u"], fh["v"], fh["w"], mu, t)
        d = np.max(np.abs(np.asarray(st["F"]) - Fo))
        print(f"[fsi] {name} step {s}: force {st['F']} oracle {tuple(Fo)} max diff {d:.2e}", flush=True)
        assert d <= 1e-11 * mg
        assert abs(Fo[2]) > 0.1 * mg            # the body is afloat: a real buoyant force
        # the heave the next step must produce, from the library's force
        zeta, zdot = orc.heave_update(B.mass, B.pto_damping, wl.g, dt, st["F"][2], st["zeta"], st["zdot"])
    S.close()


@pytest.mark.parametrize("name", CASES)
def test_coupled_step_parity_forced_iterations(orc, name):
    """One coupled step from the initial state (force of the initial fields,
    heave update, then the step with psi and u_b of the new heave), CG count
    forced to the oracle's."""
    wl = I.workload(name)
    f = I.make_fields(wl)
    dt = orc.cfl_dt(orc.params(wl), f, wl.cfl, wl.dt_max)
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
    assert abs(b["zdot"] - Pk.body[0].zdot) <= 1e-12 * wl.g * dt
    gate_fields(f"fsi step {name}", dev, ref, ("sigma", "u", "v", "w", "p"), 1e-10, Scales(wl, f, dt))
    S.close()


def test_prescribed_body_state_and_no_force(orc):
    """A prescribed body reports its analytic heave and no force."""
    import math
    wl = I.workload("tiny3d")
    wl.bodies[0].heave_amp, wl.bodies[0].heave_omega, wl.bodies[0].heave_phase = 0.05, math.pi, 0.3
    f = I.make_fields(wl)
    dt = orc.cfl_dt(orc.params(wl), f, wl.cfl, wl.dt_max)
    S, dev = make_solver(wl, f)
    S.step(dt, 0.0)
    st = S.body_state(0)
    assert abs(st["zeta"] - 0.05 * math.sin(math.pi * dt + 0.3)) < 1e-15
    assert abs(st["zdot"] - 0.05 * math.pi * math.cos(math.pi * dt + 0.3)) < 1e-15
    assert st["F"] == (0.0, 0.0, 0.0) and st["f_pto"] == 0.0
    ns = _ns()
    with pytest.raises(ns.NSError):
        S.body_state(3)
    S.close()
