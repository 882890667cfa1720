"""Problem definitions for the synthetic workloads (data only).

Material kinds: ``NH_COMP`` (compressible neo-Hookean with the Gibbs
volumetric energy of the block-compression example), ``NH_INCOMP`` (same
isochoric part, fully incompressible volumetric part) and ``HGO_INCOMP``
(neo-Hookean matrix plus two exponential fibre families, fully
incompressible).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .mesh import cube_mesh, strip_dims, strip_mesh, tube_mesh

NH_COMP, NH_INCOMP, HGO_INCOMP = 0, 1, 2


@dataclass
class Material:
    kind: int = NH_COMP
    rho0: float = 1000.0
    mu: float = 1.0e5
    kappa: float = 1.0e6
    k1: float = 0.0
    k2: float = 0.0
    kd: float = 0.0
    c_m: float = 1.0e-3


@dataclass
class TimeInt:
    dt: float = 1.0e-3
    rho_inf: float = 0.5
    n_steps: int = 1          # the dead load ramps linearly to full over n_steps * dt


def material_from_nu(mu: float, nu: float, rho0: float = 1000.0) -> Material:
    """Shear modulus + Poisson ratio -> bulk modulus (nu = 0.5: incompressible)."""
    if nu >= 0.5:
        return Material(kind=NH_INCOMP, rho0=rho0, mu=mu, kappa=np.inf)
    kappa = 2.0 * mu * (1.0 + nu) / (3.0 * (1.0 - 2.0 * nu))
    return Material(kind=NH_COMP, rho0=rho0, mu=mu, kappa=kappa)


def cube_case(N: int, nu: float | None = None, kappa: float = 1.0e6, seed: int = 0,
              dt: float = 1.0e-3, n_steps: int = 1):
    """Unit-cube compression: mu = 1e5, rho0 = 1000, top traction -1e4."""
    mesh = cube_mesh(N, seed=seed)
    if nu is None:
        mat = Material(kind=NH_COMP, rho0=1000.0, mu=1.0e5, kappa=kappa)
    else:
        mat = material_from_nu(1.0e5, nu)
    return mesh, mat, TimeInt(dt=dt, rho_inf=0.5, n_steps=n_steps)


def tube_case(nr: int = 2, nt: int = 16, nz: int = 8, dt: float = 0.05, n_steps: int = 20,
              stretch: float = 1.5):
    """Fully incompressible HGO tube under axial stretch."""
    mesh = tube_mesh(nr, nt, nz, t_end=dt * n_steps, stretch=stretch)
    mat = Material(kind=HGO_INCOMP, rho0=1000.0, mu=3.0e4, kappa=np.inf,
                   k1=2.36e5, k2=0.84, kd=0.0)
    return mesh, mat, TimeInt(dt=dt, rho_inf=0.5, n_steps=n_steps)


def strip_case(n: int = 200, kd: float = 0.226, fibre_deg: float = 49.98, dt: float = 1.0e-5,
               t_ramp: float = 100.0, seed: int = 0, dims: tuple | None = None):
    """Tensile test of the adventitial strip (section 5.2): fully incompressible
    HGO, mu = 7.64 kPa, k1 = 996.6 kPa, k2 = 524.6, density 1 g/cm^3; the
    tensile force ramps linearly to 2 N over t_ramp seconds.  n = 1/dx sets the
    mesh (strip_dims); fibre_deg = 49.98 is the circumferential specimen,
    40.02 the axial one.  dims = (nx, ny, nz) overrides the hex counts."""
    mesh = strip_mesh(*(dims or strip_dims(n)), fibre_deg=fibre_deg, seed=seed)
    mat = Material(kind=HGO_INCOMP, rho0=1000.0, mu=7.64e3, kappa=np.inf,
                   k1=996.6e3, k2=524.6, kd=kd)
    return mesh, mat, TimeInt(dt=dt, rho_inf=0.5, n_steps=int(round(t_ramp / dt)))


def random_vector(n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """Standard-normal test vector."""
    return np.random.default_rng(seed).standard_normal(n).astype(dtype)


def random_state(n_nodes: int, seed: int, scale: dict | None = None) -> dict:
    """A seeded, physically small nodal state (for tangent / parity tests)."""
    s = {"u": 1e-2, "p": 1e3, "v": 1e-1, "du": 1e-1, "dp": 1e5, "dv": 1e1}
    if scale:
        s.update(scale)
    rng = np.random.default_rng(seed)
    out = {}
    for key, shape in (("u", (n_nodes, 3)), ("p", (n_nodes,)), ("v", (n_nodes, 3)),
                       ("du", (n_nodes, 3)), ("dp", (n_nodes,)), ("dv", (n_nodes, 3))):
        out[key] = s[key] * rng.uniform(-1.0, 1.0, size=shape)
    return out
