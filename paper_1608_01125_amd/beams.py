"""Seeded synthetic photon beams shaped like the paper's workloads.

This module only draws inputs: positions, directions, energies and the
macro-particle weight of every photon. It contains none of the collision
method's arithmetic (no cross-section, no threshold, no distance test), so the
GPU path and the CPU oracle can both be fed from it without sharing any part of
the computation.

Beam shapes follow the set-ups of Sec. 3.1 and Sec. 3.2 of the paper: two beams
approaching each other under a crossing angle Phi_B (180 deg = head-on), a total
opening angle (divergence) per beam, mono-energetic or spread photon energies,
and a per-macro-particle weight (number of physical photons, Sec. 2.2).

Units: micrometres for lengths, micrometres/c for times (c = 1), MeV for
energies, MeV/c for momenta.

Conventions used for every workload (the paper leaves them open):
  * beam A moves along +z; beam B moves along (sin Phi, 0, cos Phi);
  * each beam's centre starts a distance ``z0`` behind the origin on its own
    axis, so both centres reach the origin at the same time;
  * a Gaussian beam is an ellipsoid with rms ``sigma_r`` on both transverse axes
    and ``sigma_z`` along its own axis; a cylinder beam has radius ``R`` and
    length ``L`` (radius drawn as R*sqrt(u), so the density is uniform);
  * directions are uniform in solid angle inside a cone whose *full* opening is
    ``opening`` radians (the paper's "total opening angle");
  * Gaussian energies that come out <= 0 are drawn again; the E^-2 power law is
    drawn by inverting its cumulative distribution.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass, field, replace
from typing import Dict, List, Optional, Tuple

import numpy as np

FIELDS = ("x", "y", "z", "px", "py", "pz", "E", "w")

_HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS_FILE = os.path.join(_HERE, "workload_weights.json")


@dataclass(frozen=True)
class BeamSpec:
    n: int
    profile: str            # "cylinder" or "gauss"
    size_r: float           # cylinder radius R, or Gaussian transverse rms sigma_r
    size_z: float           # cylinder length L, or Gaussian longitudinal rms sigma_z
    z0: float               # start distance of the centre behind the origin
    phi_deg: float          # axis angle from +z in the x-z plane (0 for beam A)
    energy: str             # "mono", "gauss" or "powerlaw"
    e_par: Tuple[float, ...]  # (E,) | (mean, rms) | (E_min, E_max)
    opening: float          # full opening angle in radians
    w: float                # macro-particle weight (physical photons per photon record)
    advance: float = 0.0    # every photon moved this far [um] along its own direction after
                            # the draw (a later time origin for beams that start far away)


@dataclass(frozen=True)
class Workload:
    name: str
    a: BeamSpec
    b: BeamSpec
    dt: float
    n_steps: int
    seed: int


def _axis_frame(phi_deg: float):
    """Orthonormal frame (ex, ey, ez) with ez = (sin phi, 0, cos phi).

    Multiples of 90 degrees use exact sines/cosines so that e.g. a head-on beam
    moves exactly along -z.
    """
    exact = {0.0: (0.0, 1.0), 90.0: (1.0, 0.0), 180.0: (0.0, -1.0), 270.0: (-1.0, 0.0)}
    key = float(phi_deg) % 360.0
    if key in exact:
        sp, cp = exact[key]
    else:
        ph = math.radians(phi_deg)
        sp, cp = math.sin(ph), math.cos(ph)
    ez = np.array([sp, 0.0, cp])
    ey = np.array([0.0, 1.0, 0.0])
    ex = np.array([cp, 0.0, -sp])
    return ex, ey, ez


def draw_beam(spec: BeamSpec, rng: np.random.Generator) -> Dict[str, np.ndarray]:
    """Draw one beam as a dict of float64 arrays (SoA): x y z px py pz E w."""
    n = int(spec.n)
    ex, ey, ez = _axis_frame(spec.phi_deg)
    # positions in the beam's own frame
    if spec.profile == "cylinder":
        rad = spec.size_r * np.sqrt(rng.random(n))
        ang = 2.0 * np.pi * rng.random(n)
        lx = rad * np.cos(ang)
        ly = rad * np.sin(ang)
        lz = (rng.random(n) - 0.5) * spec.size_z
    elif spec.profile == "gauss":
        lx = rng.normal(0.0, spec.size_r, n)
        ly = rng.normal(0.0, spec.size_r, n)
        lz = rng.normal(0.0, spec.size_z, n)
    else:
        raise ValueError(f"unknown profile {spec.profile!r}")
    centre = -spec.z0 * ez
    pos = centre[None, :] + lx[:, None] * ex + ly[:, None] * ey + lz[:, None] * ez

    # directions: uniform in solid angle inside a cone of half-angle opening/2
    if spec.opening > 0.0:
        half = 0.5 * spec.opening
        cos_t = 1.0 - rng.random(n) * (1.0 - math.cos(half))
        sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t * cos_t))
        az = 2.0 * np.pi * rng.random(n)
        dirs = ((sin_t * np.cos(az))[:, None] * ex + (sin_t * np.sin(az))[:, None] * ey
                + cos_t[:, None] * ez)
    else:
        dirs = np.repeat(ez[None, :], n, axis=0)
    if spec.advance != 0.0:
        pos = pos + spec.advance * dirs

    # energies
    if spec.energy == "mono":
        E = np.full(n, float(spec.e_par[0]))
    elif spec.energy == "gauss":
        mean, rms = spec.e_par
        E = rng.normal(mean, rms, n)
        bad = E <= 0.0
        while bad.any():
            E[bad] = rng.normal(mean, rms, int(bad.sum()))
            bad = E <= 0.0
    elif spec.energy == "powerlaw":
        lo, hi = spec.e_par
        u = rng.random(n)
        E = 1.0 / (1.0 / lo - u * (1.0 / lo - 1.0 / hi))
    else:
        raise ValueError(f"unknown energy law {spec.energy!r}")

    out = {
        "x": np.ascontiguousarray(pos[:, 0]),
        "y": np.ascontiguousarray(pos[:, 1]),
        "z": np.ascontiguousarray(pos[:, 2]),
        "px": np.ascontiguousarray(E * dirs[:, 0]),
        "py": np.ascontiguousarray(E * dirs[:, 1]),
        "pz": np.ascontiguousarray(E * dirs[:, 2]),
        "E": np.ascontiguousarray(E),
        "w": np.full(n, float(spec.w)),
    }
    return out


def draw_pair(wl: Workload):
    """Both beams of a workload from per-beam streams of one seed."""
    ss = np.random.SeedSequence(wl.seed)
    sa, sb = ss.spawn(2)
    A = draw_beam(wl.a, np.random.Generator(np.random.PCG64(sa)))
    B = draw_beam(wl.b, np.random.Generator(np.random.PCG64(sb)))
    return A, B


def head(beam: Dict[str, np.ndarray], n: int) -> Dict[str, np.ndarray]:
    """First ``n`` photons of a beam (photons are i.i.d., so a prefix is a uniform sample)."""
    return {k: np.ascontiguousarray(v[:n]) for k, v in beam.items()}


def concat(beams: List[Dict[str, np.ndarray]]):
    """Concatenate beams into one SoA plus CSR instance offsets."""
    off = np.zeros(len(beams) + 1, dtype=np.int64)
    for m, b in enumerate(beams):
        off[m + 1] = off[m] + len(b["E"])
    out = {k: np.ascontiguousarray(np.concatenate([b[k] for b in beams])) for k in FIELDS}
    return out, off


# --------------------------------------------------------------------------------------
# The workloads. Weights that no workload fixes are calibrated so that about 2% of
# the smaller beam's photons collide; the calibrated values are stored beside this file.
# --------------------------------------------------------------------------------------

def _frozen_weights() -> dict:
    if os.path.exists(WEIGHTS_FILE):
        with open(WEIGHTS_FILE) as f:
            return json.load(f)
    return {}


def _w(key: str, default: float) -> float:
    return float(_frozen_weights().get(key, default))


def mono_headon_2k(seed: int = 0, w: Optional[float] = None, n: int = 2000) -> Workload:
    """Two head-on mono-energetic (1 MeV) cylinder beams, R = 1 um, L = 10 um,
    directions exactly +-z, 200 steps of 0.1 um/c. Centres start 10 um from the
    origin, so every pair crosses inside the run."""
    w = _w("mono_headon_2k", 2.3e12) if w is None else w
    a = BeamSpec(n, "cylinder", 1.0, 10.0, 10.0, 0.0, "mono", (1.0,), 0.0, w)
    b = replace(a, phi_deg=180.0)
    return Workload("mono_headon_2k", a, b, 0.1, 200, seed)


def uniform_headon_1m(seed: int = 0, w: Optional[float] = None, n: int = 1_000_000) -> Workload:
    """The 2k cylinder set-up at 1e6 photons per beam: uniform density (R = 1 um, L = 10 um),
    mono-energetic 1 MeV, directions exactly +-z, 200 steps of 0.1 um/c; the case most
    favourable to a uniform grid."""
    w = _w("uniform_headon_1m", 1e7) if w is None else w
    a = BeamSpec(n, "cylinder", 1.0, 10.0, 10.0, 0.0, "mono", (1.0,), 0.0, w)
    b = replace(a, phi_deg=180.0)
    return Workload("uniform_headon_1m", a, b, 0.1, 200, seed)


def gauss_headon_1m(seed: int = 0, w: Optional[float] = None, n: int = 1_000_000) -> Workload:
    """1e6 photons per beam, Gaussian sigma_r = 2 um, sigma_z = 5 um, energies
    N(2 MeV, 0.2 MeV), 10 mrad full opening, head-on, 400 steps of 0.1 um/c
    (centres start 4 sigma_z = 20 um from the origin)."""
    w = _w("gauss_headon_1m", 1.8e11) if w is None else w
    a = BeamSpec(n, "gauss", 2.0, 5.0, 20.0, 0.0, "gauss", (2.0, 0.2), 0.010, w)
    b = replace(a, phi_deg=180.0)
    return Workload("gauss_headon_1m", a, b, 0.1, 400, seed)


def batch64_instance(m: int, w: Optional[float] = None) -> Workload:
    """Instance m of the batched workload: photons per beam log-uniform in
    [1e4, 1e6] (drawn independently per beam), crossing angle uniform in
    [90, 180] deg, mean energy log-uniform in [0.6, 10] MeV with 10% rms,
    Gaussian profiles as the 1e6 head-on workload, 10 mrad opening, 400 steps of 0.1 um/c."""
    seed = 1000 + m
    prng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 7])))
    na = int(round(10.0 ** prng.uniform(4.0, 6.0)))
    nb = int(round(10.0 ** prng.uniform(4.0, 6.0)))
    phi = float(prng.uniform(90.0, 180.0))
    mu = float(10.0 ** prng.uniform(math.log10(0.6), 1.0))
    w = _w(f"batch64/{m}", 1e11) if w is None else w
    a = BeamSpec(na, "gauss", 2.0, 5.0, 20.0, 0.0, "gauss", (mu, 0.1 * mu), 0.010, w)
    b = replace(a, n=nb, phi_deg=phi)
    return Workload(f"batch64/{m}", a, b, 0.1, 400, seed)


BATCH64_INSTANCES = 64


def broadband_16m(seed: int = 0, w: Optional[float] = None, n: int = 16_000_000) -> Workload:
    """1.6e7 photons per beam, dN/dE ~ E^-2 on [0.1, 10] MeV, 30 mrad opening,
    crossing angle 150 deg, 1000 steps of 0.04 um/c."""
    w = _w("broadband_16m", 1e11) if w is None else w
    a = BeamSpec(n, "gauss", 2.0, 5.0, 20.0, 0.0, "powerlaw", (0.1, 10.0), 0.030, w)
    b = replace(a, phi_deg=150.0)
    return Workload("broadband_16m", a, b, 0.04, 1000, seed)


ME = 0.51099895  # electron rest energy [MeV]


def positron_spectra_1m(g1: float = 5.0, g2: float = 5.0, seed: int = 0, w: Optional[float] = None,
                        n: int = 1_000_000) -> Workload:
    """Positron-spectrum set-up: two head-on mono-energetic cylinder beams of 4 um length and
    diameter (R = 2 um, L = 4 um), photon energies g1 m_e and g2 m_e (5/5 or 7/3), 20 deg full
    opening, sources 1 mm apart. Every photon is moved 480 um along its own direction after
    the draw (time origin 480 um/c after the start), so that 400 steps of 0.1 um/c cover the
    crossing at t = 20 um/c without the empty approach; by then each beam is a disc of about
    85 um radius."""
    key = f"positron_spectra_1m/{g1:g}_{g2:g}"
    w = _w(key, 1e14) if w is None else w
    a = BeamSpec(n, "cylinder", 2.0, 4.0, 500.0, 0.0, "mono", (g1 * ME,), math.radians(20.0), w,
                 advance=480.0)
    b = replace(a, phi_deg=180.0, e_par=(g2 * ME,))
    return Workload(key, a, b, 0.1, 400, seed)


def crossing_angle_1e4(phi_b: float = 180.0, seed: int = 0, w: Optional[float] = None,
                       n: int = 10_000) -> Workload:
    """Crossing-angle study: two beams of 1e4 photon records with gamma = 4 photons
    (E = 4 m_e), each a cylinder of 1 um^3 (L = 1 um, R = 1/sqrt(pi) um), collimated, the
    second beam's axis at phi_b degrees to the first; centres start 3 um from the origin,
    120 steps of 0.05 um/c."""
    key = f"crossing_angle_1e4/{phi_b:g}"
    w = _w(key, 1e11) if w is None else w
    a = BeamSpec(n, "cylinder", 1.0 / math.sqrt(math.pi), 1.0, 3.0, 0.0, "mono", (4.0 * ME,),
                 0.0, w)
    b = replace(a, phi_deg=float(phi_b))
    return Workload(key, a, b, 0.05, 120, seed)


def st_headon(n_mp: int = 10_000_000, physical: float = 1e9, seed: int = 0) -> Workload:
    """Statistical regime: beams shaped like the 1e6 head-on workload (Gaussian sigma_r =
    2 um, sigma_z = 5 um, N(2, 0.2) MeV, 10 mrad), ``physical`` photons per beam carried by
    ``n_mp`` macro-particles of equal weight, 400 steps of 0.1 um/c."""
    base = gauss_headon_1m()
    a = replace(base.a, n=n_mp, w=physical / n_mp)
    b = replace(base.b, n=n_mp, w=physical / n_mp)
    return Workload(f"st_headon_{n_mp}", a, b, base.dt, base.n_steps, seed)


def st_train_instance(m: int, n_mp: int, physical: float = 1e9) -> Workload:
    """Training instance m of the statistical-regime surrogate (seed 2000 + m), drawn from
    the batched workload's parameter ranges: crossing angle uniform in [90, 180] deg, mean
    energy log-uniform in [0.6, 10] MeV with 10% rms; Gaussian profiles as the 1e6 head-on
    workload; ``physical`` photons per beam on ``n_mp`` macro-particles; 400 steps."""
    seed = 2000 + m
    prng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 11])))
    phi = float(prng.uniform(90.0, 180.0))
    mu = float(10.0 ** prng.uniform(math.log10(0.6), 1.0))
    a = BeamSpec(n_mp, "gauss", 2.0, 5.0, 20.0, 0.0, "gauss", (mu, 0.1 * mu), 0.010, physical / n_mp)
    b = replace(a, phi_deg=phi)
    return Workload(f"st_train_{m}", a, b, 0.1, 400, seed)


@dataclass(frozen=True)
class StGridSpec:
    """Binning grid of one beam in the statistical regime (field meanings as in
    tril_st_grid): lab box, cells per axis, energy range and bins, polar-angle range and
    bins about the beam axis, time at which positions are binned."""
    lo: Tuple[float, float, float]
    hi: Tuple[float, float, float]
    n_pos: Tuple[int, int, int]
    n_e: int
    e_lo: float
    e_hi: float
    n_th: int
    th_max: float
    axis: Tuple[float, float, float]
    t_bin: float

    @property
    def n_bins(self) -> int:
        return int(np.prod(self.n_pos)) * self.n_e * self.n_th

    @property
    def cell(self) -> Tuple[float, float, float]:
        return tuple((self.hi[a] - self.lo[a]) / self.n_pos[a] for a in range(3))


def st_grid(wl: Workload, which: str, beam: Dict[str, np.ndarray], n_pos: int = 32,
            n_e: int = 16, n_th: int = 8) -> StGridSpec:
    """Grid of beam ``which`` ("a" or "b"): the lab box [+-4 sigma_r]^2 x [+-4 sigma_z]
    about the origin (where both centres meet at mid-run, the time at which positions are
    binned), n_e log-spaced energy bins over the beam's sampled energy range (widened by
    1e-6 of itself at both ends, so no photon sits on an edge), n_th
    polar-angle bins over [0, opening/2] about the beam's own axis."""
    spec = wl.a if which == "a" else wl.b
    phi = math.radians(spec.phi_deg)
    axis = (math.sin(phi), 0.0, math.cos(phi))
    r, zz = 4.0 * spec.size_r, 4.0 * spec.size_z
    e = beam["E"]
    return StGridSpec((-r, -r, -zz), (r, r, zz), (n_pos, n_pos, n_pos), n_e,
                      float(e.min()) * (1.0 - 1e-6), float(e.max()) * (1.0 + 1e-6), n_th,
                      0.5 * spec.opening, axis, 0.5 * wl.n_steps * wl.dt)


def spectrum_edges(lo: float = 0.0, hi: float = 25.0, n_bins: int = 50) -> np.ndarray:
    """Default pair-energy (E_i + E_j) histogram edges in MeV, strictly increasing."""
    return np.linspace(lo, hi, n_bins + 1)
