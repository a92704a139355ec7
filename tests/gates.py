"""Parity gates of the GPU tests.

Every comparison of a GPU field with the oracle's is judged twice at the
same tolerance: by the relative L2 norm of the difference over the whole
field, and elementwise, by the largest absolute difference over the field's
natural scale (a velocity by the flow's speed, a pressure by rho_w g d, a
level set by the tank height, a property by its largest value).  The
elementwise bound is never looser than the L2 one for an error at a single
point, so a local defect that a whole-field norm would dilute still fails;
and it gives the fields whose reference is zero (a transverse velocity of a
2-D flow) an absolute bound on the flow's scale.
"""
from __future__ import annotations

import numpy as np


def host(t):
    """A torch tensor (or array) as a float64 numpy array."""
    if hasattr(t, "detach"):
        t = t.detach().cpu().numpy()
    return np.asarray(t, dtype=np.float64)


def rel(a, b) -> float:
    a, b = host(a), host(b)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def flow_speed(fields) -> float:
    """The largest face speed of a state (its velocity scale)."""
    return max(float(np.max(np.abs(host(fields[k])))) for k in ("u", "v", "w"))


class Scales:
    """Natural scales of the fields of a workload: U the initial flow's
    largest speed (at least g dt when the tank starts at rest), P = rho_w g d,
    L the tank height."""

    def __init__(self, wl, fields0, dt: float = 0.0):
        self.U = max(flow_speed(fields0), wl.g * dt, 1e-12)
        self.P = wl.rho_w * wl.g * wl.depth
        self.L = wl.nz * wl.h
        self.wl = wl

    def of(self, key: str, ref) -> float:
        """Scale of field `key` (never below the reference's own largest value)."""
        m = float(np.max(np.abs(host(ref)))) if np.size(ref) else 0.0
        base = {"sigma": self.L, "p": self.P, "rho": self.wl.rho_w, "rho_flow": self.wl.rho_w,
                "mu": self.wl.mu_w, "chi": 1.0, "bx": 1.0 / self.wl.rho_a, "by": 1.0 / self.wl.rho_a,
                "bz": 1.0 / self.wl.rho_a}.get(key)
        if key in ("u", "v", "w", "us", "vs", "ws"):
            base = self.U
        if base is None:
            base = m
        return max(base, m, 1e-300)


def gate(label: str, got, ref, tol: float, scale: float, l2: bool = True, l2_norm: float = None):
    """Assert ||got - ref|| <= tol ||ref|| and max|got - ref| <= tol scale;
    print both figures first.  l2_norm replaces ||ref|| as the L2 yardstick
    (a velocity component is judged against the norm of the whole velocity
    field: a transverse component a thousandth of the flow is computed to
    the flow's accuracy, not to its own).  The L2 bound is skipped (l2
    False, or a reference that is zero up to round-off on its scale): the
    elementwise bound on the scale then judges the field alone."""
    g, r = host(got), host(ref)
    assert g.shape == r.shape, (label, g.shape, r.shape)
    d = g - r
    nr = float(np.linalg.norm(r)) if l2_norm is None else float(l2_norm)
    rl = float(np.linalg.norm(d)) / nr if nr > 0 else 0.0
    ma = float(np.max(np.abs(d))) / scale if d.size else 0.0
    print(f"[{label}] rel_l2={rl:.2e} maxabs/scale={ma:.2e} (scale {scale:.3e}, tol {tol:.0e})", flush=True)
    if l2 and nr > 1e-6 * scale * np.sqrt(r.size):
        assert rl <= tol, (label, "rel L2", rl, tol)
    assert ma <= tol, (label, "max abs", ma, tol)
    return rl, ma


def velocity_norm(refs) -> float:
    """The L2 norm of a whole velocity field given as its components."""
    return float(np.sqrt(sum(np.linalg.norm(host(r)) ** 2 for r in refs)))


def gate_velocity(label: str, gots, refs, names, tol: float, sc: Scales):
    """gate() for the three components of a face velocity field, each on the
    flow's speed elementwise and against the whole field's norm in L2."""
    vn = velocity_norm(refs)
    for n, g, r in zip(names, gots, refs):
        gate(f"{label} {n}", g, r, tol, sc.of(n, r), l2_norm=vn)


def gate_fields(label: str, got: dict, ref: dict, keys, tol: float, sc: Scales, l2: bool = True):
    """gate() for each named field of two states, on the fields' natural
    scales; velocity components against the whole velocity field's norm."""
    vel = [k for k in ("u", "v", "w") if k in ref]
    vn = velocity_norm([ref[k] for k in vel]) if len(vel) == 3 else None
    for k in keys:
        gate(f"{label} {k}", got[k], ref[k], tol, sc.of(k, ref[k]), l2=l2,
             l2_norm=vn if k in ("u", "v", "w") else None)
