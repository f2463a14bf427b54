"""Seeded synthetic workloads: initial particle states and field/run parameters.

This module only *describes inputs* -- seeds, sizes, unit conversions and initial
conditions shaped like the setups of Gonoskov et al. (arXiv:1412.6426, Sec. VII and the
generator comparison of Sec. IV.G).  It contains none of the QED step's arithmetic, and
both the HIP path and the CPU oracle consume the same arrays it produces.

Units: time 1/w_r, length c/w_r, momentum m c, fields m c w_r / e, with
eps_r = hbar w_r / (m c^2) (so E_S = 1/eps_r).  Species 0 electron, 1 positron, 2 photon.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

#: Compton wavelength h/(m c) in metres, CODATA 2018.
LAMBDA_COMPTON_M = 2.42631023867e-12
NO_PARENT = np.uint64(0xFFFFFFFFFFFFFFFF)

FIELD_UNIFORM, FIELD_ROTATING_E, FIELD_CP_STANDING, FIELD_YEE = 0, 1, 2, 3
FIELD_LP_STANDING = 4


def eps_r_for_wavelength(lam_m: float) -> float:
    """hbar w / (m c^2) for a wave of vacuum wavelength lam_m (= lambda_C / lambda)."""
    return LAMBDA_COMPTON_M / lam_m


@dataclass
class FieldSpec:
    kind: int
    e0: tuple = (0.0, 0.0, 0.0)
    b0: tuple = (0.0, 0.0, 0.0)
    amp: float = 0.0
    omega: float = 1.0
    phase: float = 0.0
    # Yee grid (kind == FIELD_YEE): cells per dimension, cell size, node-0 position
    grid_n: tuple = (0, 0, 0)
    grid_dx: tuple = (1.0, 1.0, 1.0)
    grid_origin: tuple = (0.0, 0.0, 0.0)
    # analytic wave sampled onto the grid at every step (stands in for a field solver)
    grid_wave_amp: float = 0.0


@dataclass
class Workload:
    name: str
    eps_r: float
    dt: float
    n_steps: int
    field: FieldSpec
    capacity: tuple            # per species store (electron, positron, photon)
    seed: int = 0
    emission: int = 1
    pairs: int = 1
    push_photons: int = 1
    adaptive: int = 1
    kappa: float = 1.0
    t0: float = 0.0
    precision: str = "f64"     # "f64" or "mixed"
    n_seed: int = 0
    instances: int = 1
    instance_amp: Optional[List[float]] = None
    instance_n: Optional[List[int]] = None
    instance_capacity: Optional[tuple] = None
    description: str = ""


def _seed_columns(x, y, z, px, py, pz, first_id: int = 0) -> Dict[str, np.ndarray]:
    n = len(x)
    return {
        "x": np.ascontiguousarray(x, dtype=np.float64),
        "y": np.ascontiguousarray(y, dtype=np.float64),
        "z": np.ascontiguousarray(z, dtype=np.float64),
        "px": np.ascontiguousarray(px, dtype=np.float64),
        "py": np.ascontiguousarray(py, dtype=np.float64),
        "pz": np.ascontiguousarray(pz, dtype=np.float64),
        "w": np.ones(n, dtype=np.float64),
        "id": np.arange(first_id, first_id + n, dtype=np.uint64),
        "parent": np.full(n, NO_PARENT, dtype=np.uint64),
        "birth": np.zeros(n, dtype=np.uint32),
        "n_events": np.zeros(n, dtype=np.uint32),
    }


def empty_columns() -> Dict[str, np.ndarray]:
    z = np.zeros(0)
    return _seed_columns(z, z, z, z, z, z)


# ---------------------------------------------------------------------------------------
# Uniform B: FP64 plain method, single instance, static uniform B (chi = 1 at gamma = 1000)
# ---------------------------------------------------------------------------------------
def uniform_b(n: int = 10_000, gamma: float = 1000.0, steps: int = 100, seed: int = 0,
              dt_frac: float = 0.01, photon_capacity: Optional[int] = None) -> Workload:
    """Electrons of Lorentz factor gamma with momenta isotropic in the plane perpendicular
    to a static uniform B whose strength makes chi = 1 (time unit hbar/(m c^2), eps_r = 1,
    so fields are in units of E_S); dt = dt_frac of the gyro period.  Emission only;
    emitted photons are recorded but not pushed."""
    pabs = math.sqrt(gamma * gamma - 1.0)
    bz = 1.0 / pabs                      # |p x B| / E_S = 1
    t_gyro = 2.0 * math.pi * gamma / bz  # 2 pi gamma m c / (e B)
    cap = photon_capacity if photon_capacity is not None else max(1024, int(1.0 * n * steps))
    return Workload(
        name="uniform_b_chi1", eps_r=1.0, dt=dt_frac * t_gyro, n_steps=steps,
        field=FieldSpec(kind=FIELD_UNIFORM, b0=(0.0, 0.0, bz)),
        capacity=(n, 1, cap), seed=seed, emission=1, pairs=0, push_photons=0, n_seed=n,
        description=f"{n} e-, gamma={gamma:g}, chi=1 in uniform static B, dt={dt_frac:g} T_gyro, "
                    f"{steps} steps, emission only")


def uniform_b_initial(w: Workload, gamma: float = 1000.0) -> List[Dict[str, np.ndarray]]:
    rng = np.random.default_rng(w.seed)
    n = w.n_seed
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    pabs = math.sqrt(gamma * gamma - 1.0)
    zero = np.zeros(n)
    e = _seed_columns(zero, zero, zero, pabs * np.cos(phi), pabs * np.sin(phi), zero)
    return [e, empty_columns(), empty_columns()]


# ---------------------------------------------------------------------------------------
# Rotating-electric-field cascade (FP64 and mixed precision)
# ---------------------------------------------------------------------------------------
def rotating_e(n: int = 100_000, a0: float = 1000.0, periods: float = 3.0, seed: int = 0,
               capacity: int = 100_000_000, lepton_capacity: Optional[int] = None,
               precision: str = "f64", lam_m: float = 0.8e-6,
               steps_per_period: int = 200) -> Workload:
    """E = a0 (cos t, sin t, 0), B = 0 (units of the laser frequency), seed electrons at
    rest uniformly in a 1 um^3 box, dt = T/steps_per_period, emission plus pairs."""
    eps_r = eps_r_for_wavelength(lam_m)
    dt = 2.0 * math.pi / steps_per_period
    lcap = lepton_capacity if lepton_capacity is not None else capacity
    return Workload(
        name="rotating_e_a%g" % a0, eps_r=eps_r, dt=dt,
        n_steps=int(round(periods * steps_per_period)),
        field=FieldSpec(kind=FIELD_ROTATING_E, amp=a0, omega=1.0),
        capacity=(max(lcap, n), lcap, capacity), seed=seed, precision=precision, n_seed=n,
        description=f"rotating E a0={a0:g}, lambda={lam_m*1e6:g} um, {n} e- at rest in 1 um^3, "
                    f"dt=T/{steps_per_period}, {periods:g} periods, capacity {capacity:.3g}")


def box_side(lam_m: float = 0.8e-6, side_m: float = 1e-6) -> float:
    """A side of side_m metres in units of c/w for wavelength lam_m."""
    return 2.0 * math.pi * side_m / lam_m


def rotating_e_initial(n: int, seed: int, lam_m: float = 0.8e-6,
                       first_id: int = 0) -> List[Dict[str, np.ndarray]]:
    rng = np.random.default_rng(seed)
    L = box_side(lam_m)
    pos = rng.uniform(-0.5 * L, 0.5 * L, size=(3, n))
    zero = np.zeros(n)
    e = _seed_columns(pos[0], pos[1], pos[2], zero, zero, zero, first_id=first_id)
    return [e, empty_columns(), empty_columns()]


# ---------------------------------------------------------------------------------------
# Standing-wave cascade with Yee-grid fields
# ---------------------------------------------------------------------------------------
def standing_wave_grid(n: int = 1_000_000, a0: float = 2000.0, cells: int = 256,
                       cells_per_lambda: int = 32, capacity: int = 200_000_000,
                       lepton_capacity: Optional[int] = None, steps: int = 100,
                       seed: int = 0, lam_m: float = 0.8e-6,
                       steps_per_period: int = 100, precision: str = "f64") -> Workload:
    """Two counter-propagating circularly polarised waves of amplitude a0 each, i.e.
    E = 2 a0 cos(x) (0, cos t, sin t), B = 2 a0 sin(x) (0, cos t, sin t), sampled at every
    step on a periodic Yee grid of cells^3 FP32 cells of lambda/cells_per_lambda; seed
    electrons at rest, Gaussian (sigma = 0.1 lambda) about x = 0 (E antinode, B node)."""
    eps_r = eps_r_for_wavelength(lam_m)
    dx = 2.0 * math.pi / cells_per_lambda
    half = 0.5 * cells * dx
    lcap = lepton_capacity if lepton_capacity is not None else max(n, capacity // 8)
    return Workload(
        name="standing_wave_yee", eps_r=eps_r, dt=2.0 * math.pi / steps_per_period,
        n_steps=steps,
        field=FieldSpec(kind=FIELD_YEE, grid_n=(cells, cells, cells), grid_dx=(dx, dx, dx),
                        grid_origin=(-half, -half, -half), grid_wave_amp=a0, omega=1.0),
        capacity=(max(lcap, n), lcap, capacity), seed=seed, n_seed=n, precision=precision,
        description=f"CP standing wave a0={a0:g} on a {cells}^3 Yee grid (dx=lambda/"
                    f"{cells_per_lambda}), {n} e- Gaussian sigma=0.1 lambda, dt=T/{steps_per_period}")


def standing_wave_initial(n: int, seed: int, sigma: float = 0.2 * math.pi
                          ) -> List[Dict[str, np.ndarray]]:
    rng = np.random.default_rng(seed)
    pos = rng.normal(0.0, sigma, size=(3, n))
    zero = np.zeros(n)
    return [_seed_columns(pos[0], pos[1], pos[2], zero, zero, zero), empty_columns(),
            empty_columns()]


def yee_offsets() -> List[tuple]:
    """Node offsets (in cells) of Ex, Ey, Ez, Bx, By, Bz on the Yee mesh."""
    return [(0.5, 0.0, 0.0), (0.0, 0.5, 0.0), (0.0, 0.0, 0.5),
            (0.0, 0.5, 0.5), (0.5, 0.0, 0.5), (0.5, 0.5, 0.0)]


def standing_wave_grid_values(fs: FieldSpec, t: float) -> List[np.ndarray]:
    """The analytic standing wave sampled (FP64, rounded to FP32) at each component's Yee
    nodes at time t: six arrays of shape (nz, ny, nx)."""
    nx, ny, nz = fs.grid_n
    out = []
    a = fs.grid_wave_amp
    ph = fs.omega * t + fs.phase
    for c, off in enumerate(yee_offsets()):
        xs = fs.grid_origin[0] + (np.arange(nx) + off[0]) * fs.grid_dx[0]
        if c == 0 or c == 3:
            prof = np.zeros(nx)
        elif c in (1, 2):
            prof = 2.0 * a * np.cos(fs.omega * xs) * (math.cos(ph) if c == 1 else math.sin(ph))
        else:
            prof = 2.0 * a * np.sin(fs.omega * xs) * (math.cos(ph) if c == 4 else math.sin(ph))
        g = np.broadcast_to(prof.astype(np.float32)[None, None, :], (nz, ny, nx))
        out.append(np.ascontiguousarray(g))
    return out


# ---------------------------------------------------------------------------------------
# Batched ensemble of rotating-field cascades
# ---------------------------------------------------------------------------------------
def batched_rotating(instances: int = 64, a_lo: float = 500.0, a_hi: float = 3000.0,
                     n_lo: int = 1000, n_hi: int = 100_000, periods: float = 2.0,
                     total_capacity: int = 200_000_000, precision: str = "mixed",
                     lam_m: float = 0.8e-6, steps_per_period: int = 200,
                     n_override: Optional[List[int]] = None) -> Workload:
    """Independent rotating-field cascades: a0 log-spaced over [a_lo, a_hi], seed-electron
    count drawn uniformly in [n_lo, n_hi] with numpy default_rng(i), instance seed i."""
    amps = [a_lo * (a_hi / a_lo) ** (i / max(1, instances - 1)) for i in range(instances)]
    if n_override is not None:
        ns = list(n_override)
    else:
        ns = [int(np.random.default_rng(i).integers(n_lo, n_hi + 1)) for i in range(instances)]
    per = total_capacity // instances
    return Workload(
        name="batched_rotating_e", eps_r=eps_r_for_wavelength(lam_m),
        dt=2.0 * math.pi / steps_per_period, n_steps=int(round(periods * steps_per_period)),
        field=FieldSpec(kind=FIELD_ROTATING_E, amp=1.0, omega=1.0), capacity=(0, 0, 0),
        precision=precision, instances=instances, instance_amp=amps, instance_n=ns,
        instance_capacity=(max(per, max(ns)), per, per), n_seed=sum(ns),
        description=f"{instances} rotating-E cascades, a0 in [{a_lo:g},{a_hi:g}] log-spaced, "
                    f"{n_lo}-{n_hi} seeds each, {periods:g} periods, dt=T/{steps_per_period}")


def batched_initial(w: Workload, lam_m: float = 0.8e-6) -> List[List[Dict[str, np.ndarray]]]:
    """Per instance i: seed electrons at rest, uniform in 1 um^3, from default_rng(i)."""
    return [rotating_e_initial(n, seed=i, lam_m=lam_m) for i, n in enumerate(w.instance_n)]


# ---------------------------------------------------------------------------------------
# Sec. VII cascade development (shower): electrons of gamma_0 = 2e5 moving across a static
# uniform B of 0.2 E_S; time unit hbar / (m c^2), fields in units of E_S (eps_r = 1)
# ---------------------------------------------------------------------------------------
SHOWER_GAMMA0 = 2e5
SHOWER_B = 0.2
FINE_STRUCTURE = 7.2973525693e-3


def shower_t_rad(gamma0: float = SHOWER_GAMMA0, b: float = SHOWER_B) -> float:
    """The shower's radiation time 3.85 gamma_0^(1/3) (E_S / H_0)^(2/3) hbar^2 / (m c e^2),
    in units of hbar / (m c^2) (hbar^2 / (m c e^2) = (hbar / m c^2) / alpha)."""
    return 3.85 * gamma0 ** (1.0 / 3.0) * (1.0 / b) ** (2.0 / 3.0) / FINE_STRUCTURE


def shower(n: int = 1000, dt: float = 25_000.0, steps: int = 3, kappa: float = 0.25,
           seed: int = 0, capacity: Optional[tuple] = None,
           precision: str = "f64") -> Workload:
    """n seed electrons at the origin with p = sqrt(gamma_0^2 - 1) along x, B along z.
    At dt = 25000 (0.28 t_rad) and kappa = 0.25 the seeds take about 400 sub-steps a step;
    the children of a step need about 16 generations of same-step processing."""
    cap = capacity if capacity is not None else (2000 * n, 2000 * n, 40_000 * n)
    return Workload(
        name="shower", eps_r=1.0, dt=dt, n_steps=steps,
        field=FieldSpec(kind=FIELD_UNIFORM, b0=(0.0, 0.0, SHOWER_B)),
        capacity=tuple(cap), seed=seed, kappa=kappa, n_seed=n, precision=precision,
        description=f"{n} e-, gamma0={SHOWER_GAMMA0:g} across B={SHOWER_B} E_S, dt={dt:g} "
                    f"hbar/mc^2 ({dt / shower_t_rad():.3f} t_rad), kappa={kappa}, "
                    f"{steps} steps")


def shower_initial(w: Workload) -> List[Dict[str, np.ndarray]]:
    n = w.n_seed
    zero = np.zeros(n)
    pabs = np.full(n, math.sqrt(SHOWER_GAMMA0 * SHOWER_GAMMA0 - 1.0))
    return [_seed_columns(zero, zero, zero, pabs, zero, zero), empty_columns(), empty_columns()]


# ---------------------------------------------------------------------------------------
# Sec. VII avalanche-type cascade: a plane standing wave E_y(t = 0) = 1e-2 E_S sin(2 pi x /
# lambda), lambda = 1 um, seeded by electrons at x = lambda / 8 with p_y = 1000 m c; time
# unit 1 / omega, lengths c / omega, fields as a = e E / (m c omega)
# ---------------------------------------------------------------------------------------
AVALANCHE_LAMBDA_M = 1e-6
AVALANCHE_E0 = 1e-2  # in units of E_S
AVALANCHE_P0 = 1000.0


def avalanche_t_rad(lam_m: float = AVALANCHE_LAMBDA_M, e0: float = AVALANCHE_E0) -> float:
    """t_rad = 14 (E_S / H_0)^(2/3) lambda_C / c with H_0 = e0 E_S, in units of 1 / omega
    (omega lambda_C / c = 2 pi eps_r)."""
    eps_r = eps_r_for_wavelength(lam_m)
    return 14.0 * (1.0 / e0) ** (2.0 / 3.0) * 2.0 * math.pi * eps_r


def avalanche(n: int = 100, dt_over_t_rad: float = 173.0, periods: float = 3.0,
              kappa: float = 0.25, seed: int = 0, capacity: Optional[tuple] = None,
              precision: str = "f64") -> Workload:
    """n seed electrons (independent runs) in the standing wave; dt in units of t_rad
    (0.17 and 173 in the paper's comparison, the latter about T / 8)."""
    eps_r = eps_r_for_wavelength(AVALANCHE_LAMBDA_M)
    dt = dt_over_t_rad * avalanche_t_rad()
    steps = int(math.ceil(periods * 2.0 * math.pi / dt))
    cap = capacity if capacity is not None else (20_000 * n, 20_000 * n, 200_000 * n)
    return Workload(
        name="avalanche", eps_r=eps_r, dt=dt, n_steps=steps,
        field=FieldSpec(kind=FIELD_LP_STANDING, amp=AVALANCHE_E0 / eps_r, omega=1.0),
        capacity=tuple(cap), seed=seed, kappa=kappa, n_seed=n, precision=precision,
        description=f"{n} e- at x = lambda/8 with p_y = {AVALANCHE_P0:g} m c in a standing "
                    f"wave E_y(0) = {AVALANCHE_E0:g} E_S sin(kx), lambda = 1 um; "
                    f"dt = {dt_over_t_rad:g} t_rad, {steps} steps ({periods:g} periods), "
                    f"kappa = {kappa}")


def avalanche_initial(w: Workload) -> List[Dict[str, np.ndarray]]:
    n = w.n_seed
    zero = np.zeros(n)
    x = np.full(n, math.pi / 4.0)  # lambda / 8 in units of c / omega
    py = np.full(n, AVALANCHE_P0)
    return [_seed_columns(x, zero, zero, zero, py, zero), empty_columns(), empty_columns()]


# ---------------------------------------------------------------------------------------
# Photon-energy binning used for spectra (130 log bins of eps/mc^2 in [1e-8, 1e5])
# ---------------------------------------------------------------------------------------
SPECTRUM_BINS = 130
SPECTRUM_LO, SPECTRUM_HI = 1e-8, 1e5
