"""The finest level's fused red-black sweep (one launch per sweep, each face
coefficient read once) against the same sweep as two colour passes, through
the C ABI: V-cycles and whole steps must agree bit for bit, in FP64 and
with the FP32 V-cycle.  A block is 64 lanes by 15 rows of cell pairs (13
stored) plus a halo wave that forms the red values just beyond the row
ends, marching up a chunk of planes chosen per grid.  Rows of at most 64
pairs fit one block (C2's 64; a 127-cell row, 64 pairs with a single last
cell; the half-resolution tank's 32; a 63-cell row; a ragged 35 pairs).
Longer rows span several blocks whose end lanes read the halo: 66 pairs
(two blocks) and 150 pairs (three, the middle one with both halos inside
the grid).  Rows and planes are not multiples of the block's 13 rows or
its chunk, and most grids span several row blocks and plane chunks.  The
512x256x256 tank runs the launch the library uses there: 4 x 20 tiles in
3 chunks of 86 planes, one round of 240 blocks."""



import numpy as np
import pytest

from paper_2206_07732_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _ns():
    from paper_2206_07732_amd import ns
    return ns


def case(name):
    from test_gpu_parity import case as parity_case
    if name == "g63":
        return I.workload("tiny3d", nx=63, ny=40, nz=20, h=4.0 / 63, seed=33,
                          bodies=[I.Body(1, (2.0, 0.8, 0.0), (0.3, 0.7, 1.5))])
    if name == "g127":
        return I.workload("tiny3d", nx=127, ny=20, nz=40, h=4.0 / 127, seed=32,
                          bodies=[I.Body(1, (2.0, 0.3, 0.0), (0.3, 0.7, 1.5))])
    if name == "c2half":
        return I.workload("c2half")
    if name == "g300":
        return I.workload("tiny3d", nx=300, ny=30, nz=40, h=4.0 / 300, seed=34, depth=0.3,
                          wave={"kind": "airy", "a": 0.01, "T": 1.2, "phase": 0.0},
                          bodies=[I.Body(1, (2.0, 0.2, 0.0), (0.1, 0.1, 0.45))])
    if name == "g132":
        return I.workload("tiny3d", nx=132, ny=26, nz=100, h=4.0 / 132, seed=31,
                          bodies=[I.Body(1, (2.0, 0.4, 0.0), (0.3, 0.7, 1.5))])
    return parity_case(name)


CASES = ["c2", "g63", "g127", "c2half", "ragged3d", "rbragged", "g132", "g300", "c5"]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("name", CASES)
def test_fused_sweep_vcycle_is_bitwise_the_two_passes(orc, name, prec):
    ns = _ns()
    wl = case(name)
    f = I.make_fields(wl)
    dt = orc.cfl_dt(orc.params(wl), f, wl.cfl, wl.dt_max)
    dev = ns.device_fields(f)
    S = ns.Solver(ns.params(wl, prec=prec), dev)
    S.momentum_step(dt, dt)
    x = torch.from_numpy(np.random.default_rng(3).standard_normal(f["p"].shape)).cuda()
    out = {}
    for fused in (True, False):
        S.set_fine_sweep(fused)
        z = torch.empty_like(x)
        S.vcycle(x, z)
        torch.cuda.synchronize()
        out[fused] = z.clone()
    d = float((out[True] - out[False]).abs().max())
    print(f"[fine sweep] {name} prec={prec}: max |fused - two passes| = {d:.3e}", flush=True)
    assert torch.equal(out[True], out[False])
    S.close()


@pytest.mark.parametrize("name", ["c2", "g63", "g127", "g132", "g300"])
def test_fused_sweep_steps_are_bitwise_the_two_passes(orc, name):
    """Three whole steps (graph-replayed V-cycles inside CG) with the fused
    sweep and three with the two colour passes, from the same state."""
    ns = _ns()
    wl = case(name)
    f = I.make_fields(wl)
    outs = []
    for fused in (True, False):
        dev = ns.device_fields(f)
        S = ns.Solver(ns.params(wl), dev)
        S.set_fine_sweep(fused)
        t, its = 0.0, []
        for _ in range(3):
            dt = S.cfl_dt(wl.cfl, wl.dt_max)
            its.append(S.step(dt, t)["iters"])
            t += dt
        torch.cuda.synchronize()
        outs.append(({k: v.clone() for k, v in dev.items()}, its))
        S.close()
    print(f"[fine sweep steps] {name}: iters {outs[0][1]} / {outs[1][1]}", flush=True)
    assert outs[0][1] == outs[1][1]
    for k in outs[0][0]:
        assert torch.equal(outs[0][0][k], outs[1][0][k]), k


def test_fused_sweep_switch_refuses_grids_it_does_not_fit(orc):
    ns = _ns()
    wl = I.workload("tiny2d")      # a 2-D tank: no fused finest sweep
    S = ns.Solver(ns.params(wl), ns.device_fields(I.make_fields(wl)))
    assert not S.fine_sweep()
    S.set_fine_sweep(False)
    with pytest.raises(ns.NSError) as e:
        S.set_fine_sweep(True)
    assert e.value.status == ns.NS_EINVAL
    S.close()


@pytest.mark.parametrize("name,prec,default", [("c2", 0, False), ("c3", 0, False), ("c5", 0, False),
                                               ("c5", 1, False)])
def test_fused_sweep_default_follows_the_grid_size(orc, name, prec, default):
    """The library starts with the two colour passes (with the line tables
    on, the default, they beat the fused launch also on the 512x256x256
    tank in FP64), and the switch turns the fused launch on and off."""
    ns = _ns()
    wl = case(name)
    S = ns.Solver(ns.params(wl, prec=prec), ns.device_fields(I.make_fields(wl)))
    assert S.fine_sweep() == default
    S.set_fine_sweep(True)
    assert S.fine_sweep()
    S.set_fine_sweep(False)
    assert not S.fine_sweep()
    S.close()
