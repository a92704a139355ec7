"""Numerical wave tank (Sec. "Numerical wave tank"): the inlet face, the
vorticity damping in the predictor and the generation and damping zones,
computed by the gfx950 library through its C ABI, against the FP64 CPU
oracle.  Bars as for the step: the predictor is elementwise (1e-13
relative); a whole step with the CG count forced to the oracle's agrees to
1e-10 relative per field (the relaxation after the correction is
elementwise on top of that)."""
import numpy as np
import pytest

from gates import Scales, gate, gate_fields, gate_velocity
from paper_2206_07732_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = ["c1nwt", "nwt3d"]


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
def test_predictor_with_inlet_and_vorticity_damping(orc, name):
    wl = I.workload(name)
    f = I.make_fields(wl)
    dt = orc.cfl_dt(orc.params(wl), f, wl.cfl, wl.dt_max)
    P = orc.params(wl)
    S, dev = make_solver(wl, f)
    S.momentum_step(dt, dt)
    torch.cuda.synchronize()
    ref = orc.momentum(P, f["u"], f["v"], f["w"], f["sigma"], dt, dt)
    sc = Scales(wl, f, dt)
    gate_velocity(f"nwt predictor {name}", [S.buffer(k) for k in ("us", "vs", "ws")], ref, ("us", "vs", "ws"),
                  1e-13, sc)
    # the inlet face carries the generated wave, and the top rows are damped
    us = host(S.buffer("us"))
    assert np.max(np.abs(us[..., 0])) > 0.1 * wl.wave["a"]
    bx, by, bz = orc.face_beta(P, f["sigma"], dt, dt)
    gate(f"nwt beta {name}", S.buffer("bx"), bx, 1e-13, sc.of("bx", bx))   # see the stage parity
    S.close()


@pytest.mark.parametrize("name", CASES)
def test_step_parity_forced_iterations(orc, name):
    """A whole step (inlet, damping force, projection, relaxation zones)."""
    wl = I.workload(name)
    f = I.make_fields(wl)
    dt = orc.cfl_dt(orc.params(wl), f, wl.cfl, wl.dt_max)
    _, st, rc = orc.step(orc.params(wl), f, dt, 0.0)
    assert rc == 0
    k = st["iters"]
    ref, _, _ = orc.step(orc.params(wl, max_iters=k, rtol=0.0), f, dt, 0.0)
    S, dev = make_solver(wl, f, max_iters=k, rtol=0.0)
    sg = S.step(dt, 0.0, allow_noconv=True)
    torch.cuda.synchronize()
    assert sg["iters"] == k
    gate_fields(f"nwt step {name}", dev, ref, ("sigma", "u", "v", "w", "p"), 1e-10, Scales(wl, f, dt))
    S.close()


def test_c1nwt_free_running_steps(orc):
    """Five free-running steps of the 2-D wave tank stay with the oracle's."""
    wl = I.workload("c1nwt")
    f = I.make_fields(wl)
    dt = orc.cfl_dt(orc.params(wl), f, wl.cfl, wl.dt_max)
    P = orc.params(wl)
    S, dev = make_solver(wl, f)
    ref = f
    t = 0.0
    for s in range(5):
        ref, _, rc = orc.step(P, ref, dt, t)
        assert rc == 0
        S.step(dt, t)
        t += dt
    torch.cuda.synchronize()
    gate_fields("nwt free run", dev, ref, ("sigma", "u", "w", "p"), 1e-8, Scales(wl, f, dt))
    S.close()
