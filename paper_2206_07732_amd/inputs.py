"""Seeded synthetic wave-tank inputs shared by the GPU path and the oracle.

This module produces *inputs* only: grid sizes, fluid constants, body
geometry, the initial level set and the initial face velocities of a wave
tank.  It contains none of the arithmetic of the time step itself (no
advection, properties, momentum or projection), so the GPU library and the
CPU oracle can both consume the same arrays without sharing any code.

Wave theory used for the initial conditions:
  * first-order (Airy) elevation and the linear dispersion relation, Sec.
    "Regular waves" (eq_first_order_wave_elev, eq_dispersion_relation);
    the explicit Fenton approximation (eq_explicit_dispersion_relation) is
    provided as an independent cross-check of the Newton solve;
  * irregular seas as a superposition of first-order components with
    uniform random phases and amplitudes a_i = sqrt(2 S(w_i) dw), Sec.
    "Irregular waves" (eq_irregular_elevation, eq_wave_spectrum_amplitude);
  * the spectrum is JONSWAP (gamma = 3.3), the peak-enhanced relative of the
    paper's Bretschneider spectrum (eq_Bretshneider_wave_spec); the
    Bretschneider formula as printed is also provided;
  * the second-order Stokes elevation/potential is the textbook extension
    of the first-order wave (the paper stops at first order).

Layout: every array is C-ordered with x fastest.  Cell arrays have shape
(nz, ny, nx); face arrays are u (nz, ny, nx+1), v (nz, ny+1, nx) and
w (nz+1, ny, nx).  A 2-D tank in the (x, z) plane has ny == 1.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

G = 9.81
RHO_W, MU_W = 1025.0, 1.0e-3      # water (Sec. "Grid convergence study")
RHO_A, MU_A = 1.225, 1.8e-5       # air


# ----------------------------------------------------------------------------
# dispersion relation
# ----------------------------------------------------------------------------
def wavenumber(omega: float, depth: float, g: float = G) -> float:
    """kappa solving omega^2 = g kappa tanh(kappa d) (eq_dispersion_relation),
    by Newton's method to machine precision."""
    if omega <= 0.0:
        raise ValueError("omega must be positive")
    k = max(omega * omega / g, omega / math.sqrt(g * depth))
    for _ in range(100):
        t = math.tanh(k * depth)
        f = g * k * t - omega * omega
        df = g * t + g * k * depth * (1.0 - t * t)
        dk = f / df
        k -= dk
        if abs(dk) <= 1e-15 * k:
            break
    return k


def fenton_kd(omega: float, depth: float, g: float = G) -> float:
    """Explicit approximation of kappa*d (eq_explicit_dispersion_relation)."""
    gam = omega * omega * depth / g
    b = gam / math.sqrt(math.tanh(gam))
    sech2 = 1.0 / math.cosh(b) ** 2
    return (gam + b * b * sech2) / (math.tanh(b) + b * sech2)


# ----------------------------------------------------------------------------
# spectra
# ----------------------------------------------------------------------------
def bretschneider(omega, hs: float, tp: float):
    """S(omega) exactly as printed in eq_Bretshneider_wave_spec."""
    omega = np.asarray(omega, dtype=np.float64)
    return 173.0 * hs ** 2 / tp ** 4 * omega ** -5 * np.exp(-692.0 / tp ** 4 * omega ** -4)


def jonswap(omega, hs: float, tp: float, gamma: float = 3.3):
    """JONSWAP spectral density with peak omega_p = 2 pi / T_p (unnormalised
    Pierson-Moskowitz shape times the peak-enhancement factor)."""
    omega = np.asarray(omega, dtype=np.float64)
    wp = 2.0 * math.pi / tp
    sig = np.where(omega <= wp, 0.07, 0.09)
    r = np.exp(-((omega - wp) ** 2) / (2.0 * sig ** 2 * wp ** 2))
    return (5.0 / 16.0) * hs ** 2 * wp ** 4 * omega ** -5 * np.exp(-1.25 * (wp / omega) ** 4) * gamma ** r


def jonswap_components(hs: float, tp: float, n: int, seed: int, depth: float, g: float = G):
    """n midpoint components on [0.5 w_p, 3 w_p]; amplitudes from
    eq_wave_spectrum_amplitude, rescaled so that 4 sqrt(sum a_i^2 / 2) = H_s;
    phases uniform on [0, 2 pi) from numpy's default_rng(seed)."""
    wp = 2.0 * math.pi / tp
    lo, hi = 0.5 * wp, 3.0 * wp
    dw = (hi - lo) / n
    om = lo + (np.arange(n) + 0.5) * dw
    a = np.sqrt(2.0 * jonswap(om, hs, tp) * dw)
    a *= hs / (4.0 * math.sqrt(0.5 * float(np.sum(a * a))))
    rng = np.random.default_rng(seed)
    th = 2.0 * math.pi * rng.random(n)
    k = np.array([wavenumber(float(w), depth, g) for w in om])
    return om, k, a, th


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Body:
    kind: int                       # 0: box in the (x, z) plane, 1: vertical cylinder
    c: tuple                        # box (xc, -, zc); cylinder (xc, yc, -)
    half: tuple                     # box (a, -, b) half-widths; cylinder (R, z_bot, z_top)
    heave_amp: float = 0.0          # prescribed heave zeta(t) = A sin(w t + phi)
    heave_omega: float = 0.0
    heave_phase: float = 0.0
    free_heave: int = 0             # 1: heave follows Newton's law under the hydrodynamic force
    mass: float = 0.0               # kg (per metre of depth in 2-D)
    pto_damping: float = 0.0        # linear-damper PTO force F_PTO = -c zdot, N s/m
    zeta0: float = 0.0              # initial heave offset (m) and velocity (m/s) of a free body
    zdot0: float = 0.0


@dataclasses.dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    h: float
    depth: float
    wave: dict
    bodies: List[Body]
    steps: int
    cfl: float = 0.2
    seed: int = 0
    rho_w: float = RHO_W
    mu_w: float = MU_W
    rho_a: float = RHO_A
    mu_a: float = MU_A
    rho_s: float = RHO_W            # solid takes water's values (reading A8)
    mu_s: float = MU_W
    g: float = G
    n_cells: float = 1.0            # Heaviside half-width in cells
    inv_kappa_p: float = 1.0e8      # Brinkman 1/kappa_p
    proj_penalty_weight: float = 1.0
    dt_max: float = 0.05
    p_init: str = "zero"            # initial pressure: "zero", or "hydrostatic" under the initial surface
    nwt: Optional[dict] = None      # numerical wave tank: {"gen": m, "damp": m, "vort": m} zone sizes
    consistent: int = 0             # 1: conservative predictor with consistent mass/momentum transport
    cn_sweeps: int = 0              # > 0: Crank-Nicolson viscous term by this many Jacobi sweeps

    @property
    def dim(self) -> int:
        return 2 if self.ny == 1 else 3

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def lengths(self):
        return self.nx * self.h, self.ny * self.h, self.nz * self.h


def _cyl(xc=2.0, yc=1.0, **kw) -> Body:
    # radius 0.25 m, length 0.8 m, draft 0.3 m in 1 m of water: z in [0.7, 1.5]
    return Body(1, (xc, yc, 0.0), (0.25, 0.7, 1.5), **kw)


# mass of the water the cylinder displaces at rest (floats in equilibrium)
_CYL_MASS = RHO_W * math.pi * 0.25 ** 2 * 0.3


def harvest_draw(seed: int):
    """Wave and buoy of one seeded learned-guess run: amplitude U[0.01, 0.08] m,
    period U[0.8, 2] s, buoy centre (x, y) in U([1.5, 2.5] x [0.75, 1.25]) m,
    phase U[0, 2 pi).  Returns (a, T, phase, x, y)."""
    rng = np.random.default_rng(1000 + seed)
    a = float(rng.uniform(0.01, 0.08))
    T = float(rng.uniform(0.8, 2.0))
    bx, by = float(rng.uniform(1.5, 2.5)), float(rng.uniform(0.75, 1.25))
    phase = float(rng.uniform(0, 2 * math.pi))
    return a, T, phase, bx, by


def workload(name: str, **over) -> Workload:
    """Named synthetic tanks.  'c1'..'c5' are the five measured configurations;
    'tiny2d'/'tiny3d' are small variants for quick parity tests."""
    two_pi = 2.0 * math.pi
    if name == "c1":
        wl = Workload("c1: 2-D tank 256x64 (8 m x 2 m, h=1/32), Airy a=0.02 m T=1 s, fixed box 0.4x0.2 m",
                      256, 1, 64, 8.0 / 256, 1.0, {"kind": "airy", "a": 0.02, "T": 1.0, "phase": 0.0},
                      [Body(0, (4.0, 0.0, 1.0), (0.2, 0.0, 0.1))], steps=10, seed=1)
    elif name == "c2":
        wl = Workload("c2: 3-D tank 128x64x64 (4x2x2 m, h=1/32), Stokes-2 a=0.05 m T=1.2 s, fixed cylinder",
                      128, 64, 64, 4.0 / 128, 1.0, {"kind": "stokes2", "a": 0.05, "T": 1.2}, [_cyl()],
                      steps=20, seed=2)
    elif name == "c2half":
        # C2's tank and wave at half the resolution: the smallest tank on which
        # the cylinder's waterline drives the local Courant number past 0.5
        # within a dozen steps of the fixed initial-field time step
        wl = Workload("c2half: 3-D tank 64x32x32 (4x2x2 m, h=1/16), Stokes-2 a=0.05 m T=1.2 s, fixed cylinder",
                      64, 32, 32, 4.0 / 64, 1.0, {"kind": "stokes2", "a": 0.05, "T": 1.2}, [_cyl()],
                      steps=40, seed=2)
    elif name == "c3":
        wl = Workload("c3: 3-D tank 256x128x128 (4x2x2 m, h=1/64), JONSWAP Hs=0.1 m Tp=1.5 s 64 comps, fixed cylinder",
                      256, 128, 128, 4.0 / 256, 1.0, {"kind": "jonswap", "hs": 0.1, "tp": 1.5, "n": 64},
                      [_cyl()], steps=10, seed=3)
    elif name == "c4train":
        wl = Workload("c4-train: 3-D tank 128x64x64, seeded Airy wave and buoy position",
                      128, 64, 64, 4.0 / 128, 1.0, {"kind": "airy", "a": 0.04, "T": 1.2, "phase": 0.0},
                      [_cyl()], steps=50, seed=4)
    elif name == "c4eval":
        a, T, phase, bx, by = harvest_draw(40)
        wl = Workload("c4-eval: 3-D tank 256x128x128 (h=1/64), held-out seeded Airy wave and buoy (draw 40)",
                      256, 128, 128, 4.0 / 256, 1.0, {"kind": "airy", "a": a, "T": T, "phase": phase},
                      [_cyl(bx, by)], steps=20, seed=40)
    elif name == "c5":
        wl = Workload("c5: 3-D tank 512x256x256 (4x2x2 m, h=1/128), JONSWAP Hs=0.2 m Tp=2 s, two heaving cylinders",
                      512, 256, 256, 4.0 / 512, 1.0, {"kind": "jonswap", "hs": 0.2, "tp": 2.0, "n": 64},
                      [_cyl(4.0 / 3.0, 1.0, heave_amp=0.05, heave_omega=two_pi / 2.0, heave_phase=0.0),
                       _cyl(8.0 / 3.0, 1.0, heave_amp=0.05, heave_omega=two_pi / 2.0, heave_phase=0.5 * math.pi)],
                      steps=50, seed=5)
    elif name == "tiny2d":
        wl = Workload("tiny2d: 2-D tank 64x16 (8x2 m), Airy a=0.05 T=1.5, fixed box",
                      64, 1, 16, 8.0 / 64, 1.0, {"kind": "airy", "a": 0.05, "T": 1.5, "phase": 0.3},
                      [Body(0, (4.0, 0.0, 1.0), (0.4, 0.0, 0.25))], steps=3, seed=11)
    elif name == "tiny3d":
        wl = Workload("tiny3d: 3-D tank 32x16x16 (4x2x2 m), Stokes-2 a=0.08 T=1.2, fixed cylinder",
                      32, 16, 16, 4.0 / 32, 1.0, {"kind": "stokes2", "a": 0.08, "T": 1.2}, [_cyl()],
                      steps=3, seed=12)
    elif name == "c1nwt":
        # C1's tank as a numerical wave tank: generation zone of one
        # wavelength at the inlet, damping zone of 1.5 wavelengths at the far
        # end, vorticity damping over the top four cells
        lam = 2.0 * math.pi / wavenumber(2.0 * math.pi / 1.0, 1.0, G)
        wl = Workload("c1nwt: 2-D wave tank 256x64 (8x2 m, h=1/32), Airy a=0.02 m T=1 s generated at x=0, "
                      "zones 1 and 1.5 wavelengths, fixed box 0.4x0.2 m",
                      256, 1, 64, 8.0 / 256, 1.0, {"kind": "airy", "a": 0.02, "T": 1.0, "phase": 0.0},
                      [Body(0, (4.0, 0.0, 1.0), (0.2, 0.0, 0.1))], steps=10, seed=1,
                      nwt={"gen": lam, "damp": 1.5 * lam, "vort": 4 * 8.0 / 256})
    elif name == "c2nwt":
        # the C2 tank as a wave tank: Airy waves generated at x = 0 (the tank is
        # 1.8 wavelengths long, so the zones are 0.8 and 1.2 m)
        wl = Workload("c2nwt: 3-D wave tank 128x64x64 (4x2x2 m, h=1/32), Airy a=0.05 m T=1.2 s generated at x=0, "
                      "zones 0.8 and 1.2 m, vorticity damping 4 cells, fixed cylinder",
                      128, 64, 64, 4.0 / 128, 1.0, {"kind": "airy", "a": 0.05, "T": 1.2, "phase": 0.0}, [_cyl()],
                      steps=20, seed=2, nwt={"gen": 0.8, "damp": 1.2, "vort": 4 * 4.0 / 128})
    elif name == "nwt3d":
        lam = 2.0 * math.pi / wavenumber(2.0 * math.pi / 1.2, 1.0, G)
        wl = Workload("nwt3d: 3-D wave tank 32x16x16 (4x2x2 m), Airy a=0.05 T=1.2 s generated at x=0, "
                      "zones 1 and 1.5 m, fixed cylinder",
                      32, 16, 16, 4.0 / 32, 1.0, {"kind": "airy", "a": 0.05, "T": 1.2, "phase": 0.4}, [_cyl()],
                      steps=3, seed=15, nwt={"gen": 1.0, "damp": 1.5, "vort": 4 * 4.0 / 32})
    elif name == "fsi2d":
        # a spar-like box 0.25 m wide and 0.75 m tall floating at a 0.5 m draft
        # (mass of the displaced water, per metre of depth), released 2 cm
        # above its rest position
        wl = Workload("fsi2d: 2-D tank 128x32 (8x2 m, h=1/16), Airy a=0.03 T=1.5, free-heave box 0.25x0.75 m, "
                      "PTO 20 N s/m",
                      128, 1, 32, 8.0 / 128, 1.0, {"kind": "airy", "a": 0.03, "T": 1.5, "phase": 0.3},
                      [Body(0, (4.0, 0.0, 0.875), (0.125, 0.0, 0.375), free_heave=1, mass=RHO_W * 0.25 * 0.5,
                            pto_damping=20.0, zeta0=0.02)], steps=5, seed=13, p_init="hydrostatic")
    elif name == "fsi3d":
        wl = Workload("fsi3d: 3-D tank 32x16x16 (4x2x2 m), Stokes-2 a=0.08 T=1.2, free-heave cylinder, PTO 50 N s/m",
                      32, 16, 16, 4.0 / 32, 1.0, {"kind": "stokes2", "a": 0.08, "T": 1.2},
                      [_cyl(free_heave=1, mass=_CYL_MASS, pto_damping=50.0)], steps=5, seed=14,
                      p_init="hydrostatic")
    elif name == "c2fsi":
        wl = Workload("c2fsi: 3-D tank 128x64x64 (4x2x2 m, h=1/32), Stokes-2 a=0.05 m T=1.2 s, "
                      "free-heave cylinder, PTO 200 N s/m",
                      128, 64, 64, 4.0 / 128, 1.0, {"kind": "stokes2", "a": 0.05, "T": 1.2},
                      [_cyl(free_heave=1, mass=_CYL_MASS, pto_damping=200.0)], steps=20, seed=2,
                      p_init="hydrostatic")
    else:
        raise KeyError(name)
    for k, v in over.items():
        if not hasattr(wl, k):
            raise KeyError(k)
        setattr(wl, k, v)
    return wl


# ----------------------------------------------------------------------------
# initial fields
# ----------------------------------------------------------------------------
def _wave_terms(wl: Workload):
    """Return a list of (a, omega, kappa, phase, order) linear components and,
    for Stokes-2, the second-order amplitude terms."""
    wv = wl.wave
    kind = wv["kind"]
    rng = np.random.default_rng(wl.seed)
    if kind in ("airy", "standing"):
        om = 2.0 * math.pi / wv["T"] if "T" in wv else None
        k = wv.get("kappa")
        if k is None:
            k = wavenumber(om, wl.depth, wl.g)
        elif om is None:
            om = math.sqrt(wl.g * k * math.tanh(k * wl.depth))
        return kind, [(wv["a"], om, k, wv.get("phase", 0.0))]
    if kind == "stokes2":
        om = 2.0 * math.pi / wv["T"]
        k = wavenumber(om, wl.depth, wl.g)
        th0 = 2.0 * math.pi * float(rng.random())
        return kind, [(wv["a"], om, k, th0)]
    if kind == "jonswap":
        om, k, a, th = jonswap_components(wv["hs"], wv["tp"], wv["n"], wl.seed, wl.depth, wl.g)
        return kind, list(zip(a.tolist(), om.tolist(), k.tolist(), th.tolist()))
    if kind == "flat":
        return kind, []
    raise KeyError(kind)


def wave_components(wl: Workload):
    """The linear components (a, kappa, omega, phase) of the workload's wave,
    as arrays: the waves a numerical wave tank generates, a cos(kappa x -
    omega t + phase).  Only linear kinds (Airy, JONSWAP, flat) qualify."""
    kind, comps = _wave_terms(wl)
    if kind not in ("airy", "jonswap", "flat"):
        raise ValueError(f"a wave tank generates linear waves only, not {kind}")
    if len(comps) > 64:
        raise ValueError("at most 64 components")
    a = np.array([c[0] for c in comps], dtype=np.float64)
    om = np.array([c[1] for c in comps], dtype=np.float64)
    k = np.array([c[2] for c in comps], dtype=np.float64)
    ph = np.array([c[3] for c in comps], dtype=np.float64)
    return a, k, om, ph


def elevation(wl: Workload, x):
    """Free-surface elevation eta(x) at t = 0 (relative to still water)."""
    kind, comps = _wave_terms(wl)
    x = np.asarray(x, dtype=np.float64)
    eta = np.zeros_like(x)
    for a, om, k, th in comps:
        eta += a * np.cos(k * x + th)
        if kind == "stokes2":
            d = wl.depth
            a2 = 0.25 * k * a * a * math.cosh(k * d) * (2.0 + math.cosh(2 * k * d)) / math.sinh(k * d) ** 3
            eta += a2 * np.cos(2.0 * (k * x + th))
    return eta


def _velocity(wl: Workload, x, z):
    """Potential-flow (u, w) under the wave at t = 0; z measured from the bed."""
    kind, comps = _wave_terms(wl)
    u = np.zeros(np.broadcast(x, z).shape)
    w = np.zeros_like(u)
    if kind in ("standing", "flat"):
        return u, w                   # standing waves start from rest
    d = wl.depth
    for a, om, k, th in comps:
        ph = k * x + th
        u += a * om * np.cosh(k * z) / math.sinh(k * d) * np.cos(ph)
        w += a * om * np.sinh(k * z) / math.sinh(k * d) * np.sin(ph)
        if kind == "stokes2":
            c2 = 0.75 * a * a * om * k / math.sinh(k * d) ** 4
            u += c2 * np.cosh(2 * k * z) * np.cos(2 * ph)
            w += c2 * np.sinh(2 * k * z) * np.sin(2 * ph)
    return u, w


def make_fields(wl: Workload):
    """Initial sigma (cells), u/v/w (faces) and p: 0, or with p_init =
    "hydrostatic" rho_w g (d + eta(x) - z) under the initial surface and 0
    above it.

    sigma = z - (d + eta(x)): negative in water, not an exact signed distance.
    Faces below the initial surface carry the potential-flow velocity, faces
    above it are at rest.  Wall-normal faces (x = 0, x = Lx, y = 0, y = Ly,
    z = 0) are zero."""
    nx, ny, nz, h = wl.nx, wl.ny, wl.nz, wl.h
    xc = (np.arange(nx) + 0.5) * h
    zc = (np.arange(nz) + 0.5) * h
    xf = np.arange(nx + 1) * h
    zf = np.arange(nz + 1) * h
    eta_c = elevation(wl, xc)
    sigma = np.empty((nz, ny, nx))
    sigma[:] = (zc[:, None, None] - (wl.depth + eta_c[None, None, :]))

    eta_xf = elevation(wl, xf)
    uu, _ = _velocity(wl, xf[None, :], zc[:, None])              # (nz, nx+1)
    wet = zc[:, None] < wl.depth + eta_xf[None, :]
    uu = np.where(wet, uu, 0.0)
    uu[:, 0] = 0.0
    uu[:, -1] = 0.0
    u = np.repeat(uu[:, None, :], ny, axis=1).copy()

    v = np.zeros((nz, ny + 1, nx))

    _, ww = _velocity(wl, xc[None, :], zf[:, None])              # (nz+1, nx)
    wet = zf[:, None] < wl.depth + eta_c[None, :]
    ww = np.where(wet, ww, 0.0)
    ww[0, :] = 0.0
    w = np.repeat(ww[:, None, :], ny, axis=1).copy()
    p = np.zeros((nz, ny, nx))
    if wl.p_init == "hydrostatic":
        p[:] = np.maximum(-sigma, 0.0) * wl.rho_w * wl.g
    elif wl.p_init != "zero":
        raise ValueError(wl.p_init)
    return {"sigma": np.ascontiguousarray(sigma), "u": u, "v": v, "w": w, "p": p}


def random_fields(nx: int, ny: int, nz: int, seed: int, scale: float = 1.0):
    """Random cell/face arrays (for operator-level parity tests)."""
    rng = np.random.default_rng(seed)
    return {
        "c": rng.standard_normal((nz, ny, nx)) * scale,
        "u": rng.standard_normal((nz, ny, nx + 1)) * scale,
        "v": rng.standard_normal((nz, ny + 1, nx)) * scale,
        "w": rng.standard_normal((nz + 1, ny, nx)) * scale,
    }
