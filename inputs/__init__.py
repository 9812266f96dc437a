"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module draws phase-space points and uniforms; it holds none of the
matrix-element arithmetic.  Both sides of every parity test read the momenta
produced here, so nothing here may call into ``oracle/`` or the HIP package.

Random numbers come from numpy's Philox counter-based generator
(Salmon et al., SC'11) keyed by the integer seed, so a seed names one fixed
stream on every machine.

Phase space is RAMBO (Kleiss, Stirling, Ellis, Comput. Phys. Commun. 40
(1986) 359): flat n-body momenta at fixed partonic energy, massless points
rescaled to the final-state masses.  The paper's event generator draws random
numbers, maps them to momenta and then evaluates the matrix element (Sec. 2);
this module is the first two steps, reduced to flat phase space.

Layout of every momentum array: ``[nevt][npart][4]`` float64, components
``(E, px, py, pz)`` in GeV.  Particles 0 and 1 are the incoming partons along
+z and -z with energy sqrt(s)/2 each; the final state follows in process order.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["rng", "rambo", "process_masses", "PROCESS_KINEMATICS", "uniforms"]


def rng(seed: int) -> np.random.Generator:
    """Philox stream for ``seed``."""
    return np.random.Generator(np.random.Philox(key=int(seed)))


def uniforms(n: int, k: int, seed: int) -> np.ndarray:
    """``[n][k]`` float64 uniforms in (0, 1) for the method's random draws."""
    u = rng(seed).random((n, k))
    return np.where(u == 0.0, 0.5 * np.finfo(np.float64).tiny, u)


LD = np.longdouble


def _massless(n_evt: int, n_fin: int, roots: float, g: np.random.Generator, LD=LD) -> np.ndarray:
    """Flat massless n-body momenta at energy ``roots`` (RAMBO, Sec. 2 of KSE).

    Computed in x87 extended precision by default so that, once rounded to
    float64, the points are on shell and balance momentum to float64 rounding."""
    r = g.random((n_evt, n_fin, 4)).astype(LD)
    c = 2.0 * r[..., 0] - 1.0
    phi = 2.0 * LD(math.pi) * r[..., 1]
    # 1 - u lies in (0, 1], so the logarithm stays finite.
    q0 = -np.log((1.0 - r[..., 2]) * (1.0 - r[..., 3]))
    st = np.sqrt(np.maximum(0.0, 1.0 - c * c))
    q = np.empty((n_evt, n_fin, 4), dtype=LD)
    q[..., 0] = q0
    q[..., 1] = q0 * st * np.cos(phi)
    q[..., 2] = q0 * st * np.sin(phi)
    q[..., 3] = q0 * c
    Q = q.sum(axis=1)  # [n_evt][4]
    M = np.sqrt(Q[:, 0] ** 2 - (Q[:, 1:] ** 2).sum(axis=1))
    b = -Q[:, 1:] / M[:, None]
    x = LD(roots) / M
    gam = Q[:, 0] / M
    a = 1.0 / (1.0 + gam)
    bq = (b[:, None, :] * q[..., 1:]).sum(axis=2)  # [n_evt][n_fin]
    p = np.empty_like(q)
    p[..., 0] = x[:, None] * (gam[:, None] * q[..., 0] + bq)
    p[..., 1:] = x[:, None, None] * (
        q[..., 1:] + b[:, None, :] * q[..., 0:1] + a[:, None, None] * bq[..., None] * b[:, None, :]
    )
    return p


def massless_volume(n_fin: int, s: float) -> float:
    """Volume of massless n-body phase space, (2pi)^(4-3n) convention."""
    return ((2.0 * math.pi) ** (4 - 3 * n_fin) * (math.pi / 2.0) ** (n_fin - 1)
            * s ** (n_fin - 2) / (math.factorial(n_fin - 1) * math.factorial(n_fin - 2)))


def rambo(n_evt: int, roots: float, masses, seed: int, return_weight: bool = False, precise: bool = True):
    """``n_evt`` RAMBO points for 2 -> len(masses) at energy ``roots``.

    Returns momenta ``[n_evt][2 + n_fin][4]`` (and, if asked, the phase-space
    weight per point in the (2pi)^(4-3n) convention, so that the mean weight
    estimates the phase-space volume).  ``precise=False`` works in float64
    (about 5x faster; points then balance momentum to ~1e-13 relative only),
    for large samples that feed training and unweighting.
    """
    LD = np.longdouble if precise else np.float64
    masses = np.asarray(masses, dtype=np.float64)
    n_fin = masses.size
    g = rng(seed)
    p = _massless(n_evt, n_fin, roots, g, LD)
    w0 = massless_volume(n_fin, roots * roots)
    if np.any(masses > 0.0):
        if masses.sum() >= roots:
            raise ValueError("final-state masses exceed the collision energy")
        # Rescale 3-momenta by xi so that energies with masses add up to roots.
        E0 = p[..., 0]
        xi = np.full(n_evt, math.sqrt(1.0 - (masses.sum() / roots) ** 2), dtype=LD)
        m2 = masses.astype(LD)[None, :] ** 2
        for _ in range(60):
            e = np.sqrt(m2 + (xi[:, None] * E0) ** 2)
            f = e.sum(axis=1) - roots
            df = (xi[:, None] * E0 * E0 / e).sum(axis=1)
            step = f / df
            xi = xi - step
            if np.all(np.abs(step) <= 4 * np.finfo(LD).eps * np.abs(xi)):
                break
        k = np.empty_like(p)
        k[..., 1:] = xi[:, None, None] * p[..., 1:]
        k[..., 0] = np.sqrt(m2 + (xi[:, None] * E0) ** 2)
        kabs = np.sqrt((k[..., 1:] ** 2).sum(axis=2))
        kE = k[..., 0]
        w = (w0 * (kabs.sum(axis=1) / roots) ** (2 * n_fin - 3)
             * np.prod(kabs / kE, axis=1) * roots / (kabs ** 2 / kE).sum(axis=1)).astype(np.float64)
        p = k
    else:
        w = np.full(n_evt, w0)
    # Energies are recomputed from the rounded 3-momenta so that every
    # final-state momentum is on its mass shell to float64 rounding (massive
    # spinors amplify an E^2 - |p|^2 defect); balance then holds to rounding too.
    p = p.astype(np.float64)
    p[..., 0] = (np.sqrt(masses.astype(LD)[None, :] ** 2 + (p[..., 1:].astype(LD) ** 2).sum(axis=2))).astype(np.float64)
    out = np.empty((n_evt, 2 + n_fin, 4))
    half = 0.5 * roots
    out[:, 0] = (half, 0.0, 0.0, half)
    out[:, 1] = (half, 0.0, 0.0, -half)
    out[:, 2:] = p
    if return_weight:
        return out, w
    return out


# Final-state masses and energies of the workloads (GeV).  The top width is a
# matrix-element parameter and does not enter the kinematics.
MT = 173.0
PROCESS_KINEMATICS = {
    "ee_mumu": dict(roots=500.0, masses=(0.0, 0.0)),
    "gg_tt": dict(roots=13000.0, masses=(MT, MT)),
    "gg_ttg": dict(roots=13000.0, masses=(MT, MT, 0.0)),
    "gg_ttgg": dict(roots=13000.0, masses=(MT, MT, 0.0, 0.0)),
    "gg_ttggg": dict(roots=13000.0, masses=(MT, MT, 0.0, 0.0, 0.0)),
    # quark line + lepton pair (particles g, ubar, tau+, tau-, then gluons, ubar),
    # all massless; the gluon cuts apply to every final-state parton
    "gux_taptamux": dict(roots=13000.0, masses=(0.0, 0.0, 0.0)),
    "gux_taptamgux": dict(roots=13000.0, masses=(0.0, 0.0, 0.0, 0.0)),
    "gux_taptamggux": dict(roots=13000.0, masses=(0.0, 0.0, 0.0, 0.0, 0.0)),
}


def process_masses(process: str):
    return PROCESS_KINEMATICS[process]["masses"]


def process_points(process: str, n_evt: int, seed: int, return_weight: bool = False, precise: bool = True):
    """Seeded RAMBO points for one of the named workloads."""
    k = PROCESS_KINEMATICS[process]
    return rambo(n_evt, k["roots"], k["masses"], seed, return_weight=return_weight, precise=precise)


def gluon_cuts(mom, pt_min: float = 20.0, eta_max: float = 5.0, dr_min: float = 0.4) -> np.ndarray:
    """Generator-level cuts on the final-state gluons (particles 4, 5, ...):
    p_T > pt_min, |eta| < eta_max, and Delta R > dr_min between gluon pairs.
    Without them |M|^2 diverges in soft and collinear regions and unweighting is
    ill-posed; points that fail get phase-space weight 0."""
    g = np.asarray(mom)[:, 4:, :]
    pt = np.hypot(g[..., 1], g[..., 2])
    pabs = np.sqrt(pt ** 2 + g[..., 3] ** 2)
    eta = np.arctanh(np.clip(g[..., 3] / np.maximum(pabs, 1e-300), -1 + 1e-15, 1 - 1e-15))
    phi = np.arctan2(g[..., 2], g[..., 1])
    ok = np.all((pt > pt_min) & (np.abs(eta) < eta_max), axis=1)
    ng = g.shape[1]
    for i in range(ng):
        for j in range(i + 1, ng):
            dphi = np.abs(phi[:, i] - phi[:, j])
            dphi = np.minimum(dphi, 2 * np.pi - dphi)
            ok &= np.hypot(eta[:, i] - eta[:, j], dphi) > dr_min
    return ok
