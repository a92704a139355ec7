"""The C-ABI library loads on the host and exports every declared entry point
(no compute calls: no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ns.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s+\**([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def nslib():
    from paper_2206_07732_amd import ns
    if not os.path.exists(ns.LIB_PATH):
        from paper_2206_07732_amd import build
        build.build()
    return ns


def test_header_declares_the_five_path_calls():
    names = declared_functions()
    for n in ("ns_init", "levelset_advect_reinit", "momentum_step", "projection_solve", "ns_step"):
        assert n in names


def test_library_exports_every_declared_symbol(nslib):
    L = ctypes.CDLL(nslib.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert sorted(nslib.EXPORTED) == names


def test_workspace_size_and_validation(nslib):
    from paper_2206_07732_amd import inputs as I
    L = nslib.lib()
    wl = I.workload("c2")
    P = nslib.params(wl)
    nb = L.ns_workspace_bytes(ctypes.byref(P))
    ncell = wl.nx * wl.ny * wl.nz
    assert 8 * 20 * ncell < nb < 8 * 40 * ncell
    bad = nslib.params(wl)
    bad.nx = 0
    assert L.ns_workspace_bytes(ctypes.byref(bad)) == 0
    bad = nslib.params(wl)
    bad.h = -1.0
    assert L.ns_workspace_bytes(ctypes.byref(bad)) == 0
    bad = nslib.params(wl)
    bad.n_bodies = 5
    assert L.ns_workspace_bytes(ctypes.byref(bad)) == 0
    bad = nslib.params(wl, prec=7)
    assert L.ns_workspace_bytes(ctypes.byref(bad)) == 0
    # the guess modes: 0..3, and the two that run the network need P0 > 0
    for x0 in (nslib.X0_ZERO, nslib.X0_PREV, nslib.X0_LEARNED, nslib.X0_AUTO):
        assert L.ns_workspace_bytes(ctypes.byref(nslib.params(wl, x0=x0))) == nb
    assert L.ns_workspace_bytes(ctypes.byref(nslib.params(wl, x0=4))) == 0
    for x0 in (nslib.X0_LEARNED, nslib.X0_AUTO):
        assert L.ns_workspace_bytes(ctypes.byref(nslib.params(wl, x0=x0, p_scale=0.0))) == 0
    assert L.ns_workspace_bytes(ctypes.byref(nslib.params(wl, x0=nslib.X0_PREV, p_scale=0.0))) == nb
    # indices are 32-bit: the largest face array must stay under 2e9 entries
    # (here nx (ny+1) nz = 2.002e9 while the cell count is 1.992e9)
    bad = nslib.params(wl)
    bad.nx, bad.ny, bad.nz = 1000, 199, 10010
    assert L.ns_workspace_bytes(ctypes.byref(bad)) == 0
    # a free-heave body needs a positive mass and a non-negative PTO damping
    fsi = I.workload("fsi3d")
    assert L.ns_workspace_bytes(ctypes.byref(nslib.params(fsi))) > 0
    for field, value in (("mass", 0.0), ("pto_damping", -1.0), ("free_heave", 2)):
        bad = nslib.params(fsi)
        setattr(bad.body[0], field, value)
        assert L.ns_workspace_bytes(ctypes.byref(bad)) == 0, field


def test_level_count_matches_oracle(nslib, orc):
    for dims in [(256, 1, 64), (128, 64, 64), (256, 128, 128), (70, 6, 22), (37, 1, 19), (512, 256, 256)]:
        assert nslib.num_levels(*dims) == orc.num_levels(*dims)
    assert nslib.num_levels(256, 1, 64) == 7
    assert nslib.num_levels(128, 64, 64) == 7
    assert nslib.num_levels(512, 256, 256) == 9


def test_workspace_options_consistent_and_cn(nslib):
    """The consistent predictor adds one cell array (the density at t^n),
    Crank-Nicolson nine face arrays (rhs, diagonal, second iterate) and two
    values per block of its convergence check; values out of range are
    refused."""
    from paper_2206_07732_amd import inputs as I
    L = nslib.lib()
    wl = I.workload("c2")
    nb0 = L.ns_workspace_bytes(ctypes.byref(nslib.params(wl)))
    nc = wl.nx * wl.ny * wl.nz
    nf = (wl.nx + 1) * wl.ny * wl.nz + wl.nx * (wl.ny + 1) * wl.nz + wl.nx * wl.ny * (wl.nz + 1)
    nbc = L.ns_workspace_bytes(ctypes.byref(nslib.params(wl, consistent=1)))
    assert 8 * nc <= nbc - nb0 <= 8 * nc + 256
    nbn = L.ns_workspace_bytes(ctypes.byref(nslib.params(wl, cn_sweeps=3)))
    def blocks(mx, my, mz):                        # 64 x 4 x 1 tiles of a face array
        return -(-mx // 64) * -(-my // 4) * mz
    nblk = blocks(wl.nx + 1, wl.ny, wl.nz) + blocks(wl.nx, wl.ny + 1, wl.nz) + blocks(wl.nx, wl.ny, wl.nz + 1)
    checks = 2 * 8 * nblk                          # (largest change, largest |u*|) per block
    assert 3 * 8 * nf <= nbn - nb0 <= 3 * 8 * nf + checks + 10 * 256
    for field, value in (("consistent", 2), ("cn_sweeps", -1), ("cn_sweeps", 65)):
        assert L.ns_workspace_bytes(ctypes.byref(nslib.params(wl, **{field: value}))) == 0, (field, value)
    for tol in (0.0, -1e-10, float("nan")):
        assert L.ns_workspace_bytes(ctypes.byref(nslib.params(wl, cn_sweeps=3, cn_tol=tol))) == 0, tol
