"""The finest level's line tables of the face coefficients, through the C
ABI.  A solve first records, per x-line of bx, by and bz (and of their FP32
copies in a mixed cycle), whether every face of the line holds one value
(for an x-line: every interior face, its wall faces being zero); the
finest-level kernels then take such a line's faces from the table instead
of loading them.  The tables only spare loads, so every result must be
bitwise the one computed with them switched off: V-cycles in both
precisions on 2-D and 3-D grids with one-block and multi-block rows, ragged
rows and planes and odd extents, and on the 512x256x256 tank, whose first
coarse level (256x128x128) has line tables of its own; whole steps; and caller-written coefficients whose
lines are built to sit on each side of every rule (a line of one value; one
face a unit in the last place away; an interior of one value between
nonzero walls or walls of negative zero; a line of negative zeros)."""

import numpy as np
import pytest

from paper_2206_07732_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _ns():
    from paper_2206_07732_amd import ns
    return ns


def case(name):
    from test_gpu_fine_sweep import case as sweep_case
    return sweep_case(name)


CASES = ["tiny2d", "c1", "rb2d", "tiny3d", "ragged3d", "odd1level", "rbragged", "c2", "g63", "g127", "c2half", "g300", "c5"]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("name", CASES)
def test_vcycle_with_tables_is_bitwise_without(orc, name, prec):
    ns = _ns()
    wl = case(name)
    f = I.make_fields(wl)
    dt = orc.cfl_dt(orc.params(wl), f, wl.cfl, wl.dt_max)
    S = ns.Solver(ns.params(wl, prec=prec), ns.device_fields(f))
    S.momentum_step(dt, dt)
    x = torch.from_numpy(np.random.default_rng(5).standard_normal(f["p"].shape)).cuda()
    out = {}
    for on in (True, False):
        S.set_face_tables(on)
        z = torch.empty_like(x)
        S.vcycle(x, z)
        torch.cuda.synchronize()
        out[on] = z
    d = float((out[True] - out[False]).abs().max())
    print(f"[face tables] {name} prec={prec}: max |with - without| = {d:.3e}", flush=True)
    assert torch.equal(out[True], out[False])
    S.close()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("name", ["c1", "c2", "rbragged", "g127", "g300"])
def test_steps_with_tables_are_bitwise_without(orc, name, prec):
    """Three whole steps (graph-replayed V-cycles inside CG) from the same
    state, with the tables and without."""
    ns = _ns()
    wl = case(name)
    f = I.make_fields(wl)
    outs = []
    for on in (True, False):
        dev = ns.device_fields(f)
        S = ns.Solver(ns.params(wl, prec=prec), dev)
        S.set_face_tables(on)
        t, its = 0.0, []
        for _ in range(3):
            dt = S.cfl_dt(wl.cfl, wl.dt_max)
            its.append(S.step(dt, t)["iters"])
            t += dt
        torch.cuda.synchronize()
        outs.append(({k: v.clone() for k, v in dev.items()}, its))
        S.close()
    print(f"[face tables steps] {name} prec={prec}: iters {outs[0][1]} / {outs[1][1]}", flush=True)
    assert outs[0][1] == outs[1][1]
    for k in outs[0][0]:
        assert torch.equal(outs[0][0][k], outs[1][0][k]), k


def _crafted_faces(shape, rng, xline):
    """A face array (lines along the last axis) whose lines are, by kind:
    0 one value; 1 one value but one face a unit in the last place away; 2
    random; x-lines also 3 one interior value between walls of which one is
    nonzero, 4 one interior value between walls of negative zero, 5 negative
    zeros between zero walls.  Other values lie in [1e-3, 1], so every cell
    keeps faces of positive weight."""
    a = rng.uniform(1e-3, 1.0, size=shape)
    lines = a.reshape(-1, shape[-1])
    kinds = rng.integers(0, 6 if xline else 3, size=lines.shape[0])
    vals = np.array([1.0 / 1025.0, 1.0 / 1.225, 0.3, 1e-3])
    for q, kd in enumerate(kinds):
        c = vals[rng.integers(0, len(vals))]
        if kd in (0, 1, 3, 4):
            lines[q, :] = c
        if kd == 1:
            p = rng.integers(1, shape[-1] - 1) if xline else rng.integers(0, shape[-1])
            lines[q, p] = np.nextafter(c, 2.0)
        if kd == 5:
            lines[q, :] = -0.0
        if xline:
            lines[q, 0] = lines[q, -1] = 0.0
            if kd == 3:
                lines[q, rng.integers(0, 2) * (shape[-1] - 1)] = c
            if kd == 4:
                lines[q, 0] = -0.0
    return a


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("name", ["ragged3d", "c2"])
def test_caller_written_faces_on_each_side_of_the_rules(orc, name, prec):
    """Coefficients written through ns_buffer: a V-cycle and a whole PCG
    solve with the tables agree bit for bit with those without (a line read
    through a table it does not match would change them)."""
    ns = _ns()
    wl = case(name)
    f = I.make_fields(wl)
    dt = orc.cfl_dt(orc.params(wl), f, wl.cfl, wl.dt_max)
    dev = ns.device_fields(f)
    S = ns.Solver(ns.params(wl, prec=prec), dev)
    S.momentum_step(dt, dt)
    rng = np.random.default_rng(17)
    for k in ("bx", "by", "bz"):
        buf = S.buffer(k)
        a = _crafted_faces(tuple(buf.shape), rng, k == "bx")
        if k == "by":   # the y-walls stay walls
            a[:, 0, :] = 0.0
            a[:, -1, :] = 0.0
        if k == "bz":   # the bed stays a wall
            a[0] = 0.0
        buf.copy_(torch.from_numpy(a))
    rhs = S.buffer("rhs")
    rhs.copy_(torch.from_numpy(rng.standard_normal(tuple(rhs.shape))))
    torch.cuda.synchronize()
    x = torch.from_numpy(rng.standard_normal(f["p"].shape)).cuda()
    p0 = dev["p"].clone()
    out = {}
    for on in (True, False):
        S.set_face_tables(on)
        z = torch.empty_like(x)
        S.vcycle(x, z)
        dev["p"].copy_(p0)
        st = S.pcg_solve(allow_noconv=True)
        torch.cuda.synchronize()
        out[on] = (z, dev["p"].clone(), st["iters"])
    print(f"[face tables crafted] {name} prec={prec}: iters {out[True][2]} / {out[False][2]}", flush=True)
    assert torch.equal(out[True][0].view(torch.int64), out[False][0].view(torch.int64))
    assert out[True][2] == out[False][2]
    assert torch.equal(out[True][1].view(torch.int64), out[False][1].view(torch.int64))
    S.close()


@pytest.mark.parametrize("name,default", [("tiny3d", False), ("c2", False), ("c3", True)])
def test_face_table_switch(orc, name, default):
    """On from 2^21 cells (256x128x128 and up), off below; the switch turns
    them on and off and refuses another value."""
    ns = _ns()
    wl = case(name)
    S = ns.Solver(ns.params(wl), ns.device_fields(I.make_fields(wl)))
    assert S.face_tables() == default
    S.set_face_tables(False)
    assert not S.face_tables()
    S.set_face_tables(True)
    assert S.face_tables()
    assert ns.lib().ns_set_face_tables(S.ctx, 2) == ns.NS_EINVAL
    assert S.face_tables()
    S.close()
