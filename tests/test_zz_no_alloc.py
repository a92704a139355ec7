"""The allocation-free CFL rule (ns_cfl_dt_noalloc) against the context's
ns_cfl_dt, through the C ABI: two calls in a row, the second on a smaller
grid (the static scratch keeps the first call's contents), then replays of a
recorded HIP graph holding the call, each checked."""
import math

import pytest

from paper_2206_07732_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _ns():
    from paper_2206_07732_amd import ns
    return ns


def test_noalloc_cfl_matches_the_context_call():
    ns = _ns()
    out = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    for name in ("c3", "tiny3d", "c1"):           # large, then smaller grids
        wl = I.workload(name)
        dev = ns.device_fields(I.make_fields(wl))
        S = ns.Solver(ns.params(wl), dev)
        for cfl, dt_max in ((wl.cfl, wl.dt_max), (0.45, 1.0)):
            ref = S.cfl_dt(cfl, dt_max)
            ns.cfl_dt_noalloc(wl.nx, wl.ny, wl.nz, wl.h, dev["u"], dev["v"], dev["w"], cfl, dt_max, out)
            torch.cuda.synchronize()
            print(f"[noalloc] {name} cfl={cfl}: {out.item()!r} context {ref!r}", flush=True)
            assert out.item() == ref
        S.close()
    # at rest: dt_max; a non-finite velocity: NaN
    wl = I.workload("tiny2d", wave={"kind": "flat"})
    dev = ns.device_fields(I.make_fields(wl))
    ns.cfl_dt_noalloc(wl.nx, wl.ny, wl.nz, wl.h, dev["u"], dev["v"], dev["w"], 0.2, 0.03, out)
    torch.cuda.synchronize()
    assert out.item() == 0.03
    dev["w"][3, 0, 5] = float("inf")
    ns.cfl_dt_noalloc(wl.nx, wl.ny, wl.nz, wl.h, dev["u"], dev["v"], dev["w"], 0.2, 0.03, out)
    torch.cuda.synchronize()
    assert math.isnan(out.item())
    with pytest.raises(ns.NSError) as e:
        ns.cfl_dt_noalloc(1, 1, 4, wl.h, dev["u"], dev["v"], dev["w"], 0.2, 0.03, out)
    assert e.value.status == ns.NS_EINVAL


def test_noalloc_cfl_under_graph_capture():
    """The call recorded into a HIP graph (through torch's capture) and
    replayed after the velocity changes in place, with eager work and host
    waits between the replays: each replay gives the context call's value."""
    ns = _ns()
    wl = I.workload("tiny3d")
    dev = ns.device_fields(I.make_fields(wl))
    S = ns.Solver(ns.params(wl), dev)
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):        # a warm-up launch outside the graph
        ns.cfl_dt_noalloc(wl.nx, wl.ny, wl.nz, wl.h, dev["u"], dev["v"], dev["w"], 0.2, 1.0, out, side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ns.cfl_dt_noalloc(wl.nx, wl.ny, wl.nz, wl.h, dev["u"], dev["v"], dev["w"], 0.2, 1.0, out,
                          torch.cuda.current_stream())
    for rep in range(4):
        dev["u"].mul_(1.5)                   # eager work between the replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        ref = S.cfl_dt(0.2, 1.0)
        print(f"[noalloc graph] replay {rep}: {out.item()!r} context {ref!r}", flush=True)
        assert out.item() == ref
    S.close()
