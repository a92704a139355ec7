"""Pins for the seeded input generator (wave initial conditions)."""
import json
import math
import os

import numpy as np
import pytest

from paper_2206_07732_amd import inputs as I

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_dispersion_matches_printed_example():
    # Sec. "Grid convergence study": T = 1.5652 s in d = 2 m gives lambda = 3.8144 m
    g = json.load(open(os.path.join(GOLD, "dispersion_example.json")))
    k = I.wavenumber(2 * math.pi / g["T"], g["depth"], g["g"])
    lam = 2 * math.pi / k
    # the printed value is cut (not rounded) to four decimals: 3.81447 -> 3.8144
    assert 0.0 <= lam - g["wavelength"] < 10 ** (-g["printed_digits"])
    # the root satisfies eq_dispersion_relation to machine precision
    om = 2 * math.pi / g["T"]
    assert abs(g["g"] * k * math.tanh(k * g["depth"]) - om * om) < 1e-12 * om * om


def test_fenton_explicit_approximation_bound():
    # eq_explicit_dispersion_relation is an explicit fit valid at every depth;
    # its largest relative error over Gamma in (0, 20] is about 5e-4
    worst = 0.0
    for gam in np.linspace(1e-3, 20.0, 400):
        om = math.sqrt(gam * 9.81 / 1.0)
        kd_newton = I.wavenumber(om, 1.0) * 1.0
        worst = max(worst, abs(I.fenton_kd(om, 1.0) - kd_newton) / kd_newton)
    assert worst < 6e-4


def test_deep_and_shallow_limits():
    # deep water: omega^2 = g kappa (eq_deep_water_limit); shallow: omega = kappa sqrt(g d)
    om = 2 * math.pi / 0.5
    assert abs(I.wavenumber(om, 50.0) - om * om / 9.81) < 1e-12 * om * om / 9.81
    om = 0.01
    k = I.wavenumber(om, 1.0)
    assert abs(k - om / math.sqrt(9.81)) / k < 1e-4


def test_bretschneider_hs_consistency():
    # eq_Bretshneider_wave_spec: 4 sqrt(m0) recovers H_s (Fig. caption: Hs 0.15, Tp 1.7475)
    w = np.linspace(0.2, 60.0, 400001)
    s = I.bretschneider(w, 0.15, 1.7475)
    m0 = np.trapezoid(s, w)
    assert abs(4 * math.sqrt(m0) - 0.15) < 1e-4


def test_jonswap_components_rescaled_to_hs():
    om, k, a, th = I.jonswap_components(0.1, 1.5, 64, seed=3, depth=1.0)
    assert len(om) == 64
    assert abs(4 * math.sqrt(0.5 * np.sum(a * a)) - 0.1) < 1e-14
    assert np.all((th >= 0) & (th < 2 * math.pi))
    wp = 2 * math.pi / 1.5
    assert om.min() > 0.5 * wp and om.max() < 3 * wp
    # peak component sits at the spectral peak
    assert abs(om[np.argmax(a)] - wp) < 2 * (om[1] - om[0])
    # every component satisfies the dispersion relation
    assert np.allclose(9.81 * k * np.tanh(k), om ** 2, rtol=1e-12)


def test_fields_shapes_and_walls():
    wl = I.workload("tiny3d")
    f = I.make_fields(wl)
    nx, ny, nz = wl.nx, wl.ny, wl.nz
    assert f["sigma"].shape == (nz, ny, nx)
    assert f["u"].shape == (nz, ny, nx + 1)
    assert f["v"].shape == (nz, ny + 1, nx)
    assert f["w"].shape == (nz + 1, ny, nx)
    assert np.all(f["u"][:, :, 0] == 0) and np.all(f["u"][:, :, -1] == 0)
    assert np.all(f["w"][0] == 0)
    # sigma is negative in water below the still level
    assert f["sigma"][0].max() < 0 and f["sigma"][-1].min() > 0


def test_seeded_inputs_are_reproducible():
    a = I.make_fields(I.workload("tiny3d"))
    b = I.make_fields(I.workload("tiny3d"))
    for k in a:
        assert np.array_equal(a[k], b[k])
    c = I.make_fields(I.workload("tiny3d", seed=99))
    assert not np.array_equal(a["sigma"], c["sigma"])


def test_parity_cases_hold_an_interface_and_a_body_crossing_it():
    """Every 3-D stage-parity case has water and air, and each body reaches
    from the water into the air (a case whose body sits outside the water, or
    whose tank is all water, would leave the interface and penalisation terms
    untested)."""
    import sys
    import os
    sys.path.insert(0, os.path.dirname(__file__))
    from test_gpu_parity import STAGE_CASES, case
    for name in STAGE_CASES:
        wl = case(name)
        f = I.make_fields(wl)
        assert f["sigma"].min() < 0.0 < f["sigma"].max(), name
        top = wl.nz * wl.h
        for b in wl.bodies:
            if b.kind == 1:                      # cylinder: half = (R, z_bottom, z_top)
                assert b.half[1] < wl.depth < b.half[2] and b.half[1] < top, name
                assert 0.0 < b.c[0] < wl.nx * wl.h and (wl.ny == 1 or 0.0 < b.c[1] < wl.ny * wl.h), name
