"""Degenerate grids through the C ABI against the FP64 CPU oracle: the
smallest accepted tank (2x1x2: a 1x1x1 coarsest level), odd sizes that stop
coarsening at once (3x1x2, 5x3x7: one level, solved by the coarsest-level
sweeps), a 2x2x2 box and a tall 4x1x64 column whose coarsest level is a
single 1x1x16 column.  A step with the CG count forced to the oracle's agrees
to 1e-10 relative per field; a free-running step converges to the same
1e-10 residual and agrees to 1e-8."""
import numpy as np
import pytest

from gates import Scales, gate, gate_fields
from paper_2206_07732_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SHAPES = [(2, 1, 2), (3, 1, 2), (2, 2, 2), (5, 3, 7), (4, 1, 64)]


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(np.asarray(a) - b) / (nb if nb > 0 else 1.0))


def rel_flow(a, b, fields):
    """Relative error on the flow's velocity scale (v of an x-z wave is zero
    up to round-off and is not divided by its own norm)."""
    U = max(float(np.max(np.abs(fields[k]))) for k in ("u", "v", "w"))
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(np.asarray(a) - b) / max(np.linalg.norm(b), U * np.sqrt(b.size), 1e-300))


def small_tank(nx, ny, nz):
    h = 0.1
    return I.workload("tiny2d", nx=nx, ny=ny, nz=nz, h=h, depth=0.5 * nz * h, bodies=[],
                      wave={"kind": "airy", "a": 0.02 * nz * h, "T": 1.0, "phase": 0.3}, seed=5)


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_degenerate_grid_step_parity(orc, shape):
    from paper_2206_07732_amd import ns
    wl = small_tank(*shape)
    f = I.make_fields(wl)
    dt = orc.cfl_dt(orc.params(wl), f, wl.cfl, wl.dt_max)
    free, st, rc = orc.step(orc.params(wl), f, dt, 0.0)
    assert rc == 0
    k = st["iters"]
    ref, _, _ = orc.step(orc.params(wl, max_iters=k, rtol=0.0), f, dt, 0.0)
    dev = ns.device_fields(f)
    S = ns.Solver(ns.params(wl, max_iters=k, rtol=0.0), dev)
    sg = S.step(dt, 0.0, allow_noconv=True)
    torch.cuda.synchronize()
    assert sg["iters"] == k
    sc = Scales(wl, f, dt)
    gate_fields(f"edge {shape} forced {k} it", dev, ref, ("sigma", "u", "v", "w", "p"), 1e-10, sc)
    S.close()
    dev = ns.device_fields(f)
    S = ns.Solver(ns.params(wl), dev)
    sg = S.step(dt, 0.0)
    torch.cuda.synchronize()
    assert sg["true_rel_resid"] <= 1e-10
    gate_fields(f"edge {shape} free ({sg['iters']} it, oracle {k})", dev, free, ("u", "w", "p"), 1e-8, sc)
    S.close()
