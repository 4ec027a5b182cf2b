"""Seeded synthetic inputs for the particle-by-particle VMC hot path.

This module only *builds inputs*: cell sizes, orbital coefficient tables, ion
positions, Jastrow control points and run lengths.  It performs none of the
method's arithmetic (no orbital evaluation, no determinant, no Jastrow, no
energy) and imports neither the GPU package nor the oracle; both of those take
a ``Workload`` from here and translate it into their own argument structures.

Workloads follow the paper's periodic-solid setting (section "B-spline basis
sets": orbitals tabulated on a regular 3D grid; section "Jastrow factors":
one- and two-body B-spline radial functions; section "Hamiltonian": ions with
bare Coulomb charges in periodic boundary conditions).  The paper's material
systems need DFT orbitals that are not available, so seeded synthetic stand-ins
are used:

* ``heg`` -- the homogeneous electron gas: real plane waves of a closed shell,
  tabulated as interpolating periodic cubic B-spline coefficients.
* ``solid`` -- "solid-like" random smooth orbitals: periodic Gaussian-filtered
  white noise, scaled to unit RMS and rounded to FP32, used directly as
  B-spline coefficients, with randomly placed ions of charge 4.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = [
    "Workload", "cell_side", "heg_shell", "heg_coefficients", "heg",
    "solid_table", "request_table", "bspline_jastrow_params", "solid", "heg14", "solid128",
    "mixed384", "batched_systems", "served_trace", "WORKLOADS",
]


@dataclasses.dataclass
class Workload:
    """Everything one VMC run needs, as plain numbers and numpy arrays."""

    name: str
    n_up: int
    n_dn: int
    L: float                      # cubic cell side (bohr)
    n_orb: int
    grid: tuple                   # (gx, gy, gz)
    coefs: Optional[np.ndarray]   # [gx][gy][gz][n_orb], float64 or float32
    ion_pos: np.ndarray           # [n_ions][3] (bohr)
    ion_Z: np.ndarray             # [n_ions]
    j2: Optional[dict]            # {'kind':'pade','a','b'} or {'kind':'bspline','M','rc','p','cusp_same','cusp_opp'}
    j1: Optional[dict]            # {'kind':'bspline','M','rc','p','cusp'}
    hamiltonian: str              # 'coulomb' (kinetic + Ewald Coulomb) or 'kinetic'
    sigma: float                  # Gaussian proposal width (bohr)
    seed: int                     # key of the counter-based random streams
    n_walkers: int
    n_sweeps: int
    precision: str = "fp64"       # 'fp64' or 'mixed'
    delay_rank: int = 1           # 1 = Sherman-Morrison, k > 1 = rank-k delayed update
    recompute_period: int = 0     # sweeps between full FP64 inverse recomputes (0 = never)
    pw_k: Optional[np.ndarray] = None     # [n_orb][3] wave vectors of the analytic plane-wave orbitals
    pw_kind: Optional[np.ndarray] = None  # [n_orb] 0 = cos(k.r), 1 = sin(k.r)
    all_electron: bool = False    # moves: False = particle-by-particle sweeps, True = all-electron moves
    drift: bool = False           # moves drawn from the drift-diffusion distribution (all-electron
                                  # or particle-by-particle)
    j3: Optional[dict] = None     # three-body e-e-I term: {"m_ei", "m_ee", "rc", "gamma" [2][m_ei+1][m_ei+1][m_ee+1]}

    @property
    def n_elec(self) -> int:
        return self.n_up + self.n_dn

    @property
    def n_ions(self) -> int:
        return int(self.ion_pos.shape[0])

    def table_bytes(self) -> int:
        return 0 if self.coefs is None else int(self.coefs.nbytes)


def cell_side(n_elec: int, rs: float = 1.0) -> float:
    """Side of the cubic cell holding ``n_elec`` electrons at density parameter rs."""
    return (4.0 * math.pi * n_elec / 3.0) ** (1.0 / 3.0) * rs


# --------------------------------------------------------------------------
# Homogeneous electron gas
# --------------------------------------------------------------------------

def heg_shell(n_max_sq: int):
    """Integer wave vectors n with |n|^2 <= n_max_sq as real orbitals.

    Returns (n_vectors [n_orb][3] int, kind [n_orb] with 0 = cos, 1 = sin).
    The n = 0 orbital (a constant) comes first; every other +-n pair gives a
    cos and a sin orbital.  Closed shells of the simple-cubic reciprocal
    lattice hold 1, 7, 19, 27, 33, ... orbitals.
    """
    r = int(math.isqrt(n_max_sq)) + 1
    half = []
    for nx in range(-r, r + 1):
        for ny in range(-r, r + 1):
            for nz in range(-r, r + 1):
                n = (nx, ny, nz)
                if 0 < nx * nx + ny * ny + nz * nz <= n_max_sq and n > (0, 0, 0):
                    half.append(n)
    half.sort(key=lambda n: (n[0] ** 2 + n[1] ** 2 + n[2] ** 2, tuple(-c for c in n)))
    vecs, kind = [(0, 0, 0)], [0]
    for n in half:
        vecs += [n, n]
        kind += [0, 1]
    return np.array(vecs, dtype=np.int64), np.array(kind, dtype=np.int32)


def heg_coefficients(n_vec: np.ndarray, kind: np.ndarray, L: float, grid: int) -> np.ndarray:
    """Periodic cubic B-spline coefficients that interpolate cos/sin(k.r) on the grid.

    Interpolation of a plane wave e^{i k x} on a periodic uniform grid with the
    cubic B-spline basis has coefficients e^{i k x_j} * 3 / (2 + cos(theta)),
    theta = k L / G, per axis (the spline value at a knot is
    (c_{j-1} + 4 c_j + c_{j+1}) / 6).  This is input preparation, the same
    role a plane-wave-to-spline converter plays.
    """
    G = grid
    x = np.arange(G) * (L / G)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    out = np.empty((G, G, G, len(kind)), dtype=np.float64)
    for j, (n, kd) in enumerate(zip(n_vec, kind)):
        k = 2.0 * math.pi * n / L
        scale = 1.0
        for a in range(3):
            th = k[a] * L / G
            scale *= 3.0 / (2.0 + math.cos(th))
        phase = k[0] * X + k[1] * Y + k[2] * Z
        out[..., j] = scale * (np.cos(phase) if kd == 0 else np.sin(phase))
    return out


def heg(n_per_spin: int = 7, grid: int = 16, rs: float = 1.0, jastrow: bool = True,
        hamiltonian: str = "coulomb", n_walkers: int = 8, n_sweeps: int = 100,
        sigma: float = 0.3, seed: int = 0) -> Workload:
    """Closed-shell electron gas: n_per_spin orbitals per spin, Pade two-body Jastrow."""
    shells = {1: 0, 7: 1, 19: 2, 27: 3, 33: 4}
    if n_per_spin not in shells:
        raise ValueError("n_per_spin must fill a closed shell (1, 7, 19, 27 or 33)")
    n_vec, kind = heg_shell(shells[n_per_spin])
    N = 2 * n_per_spin
    L = cell_side(N, rs)
    coefs = heg_coefficients(n_vec, kind, L, grid)
    j2 = {"kind": "pade", "a": 0.5, "b": 1.0} if jastrow else None
    return Workload(
        name=f"heg{N}_g{grid}" + ("" if jastrow else "_noJ"), n_up=n_per_spin, n_dn=n_per_spin,
        L=L, n_orb=n_per_spin, grid=(grid, grid, grid), coefs=coefs,
        ion_pos=np.zeros((0, 3)), ion_Z=np.zeros(0), j2=j2, j1=None,
        hamiltonian=hamiltonian, sigma=sigma, seed=seed, n_walkers=n_walkers,
        n_sweeps=n_sweeps, pw_k=2.0 * math.pi * n_vec.astype(np.float64) / L, pw_kind=kind)


# --------------------------------------------------------------------------
# Solid-like synthetic system
# --------------------------------------------------------------------------

def solid_table(n_orb: int, grid: int, seed: int, width_cells: float = 4.0,
                dtype=np.float32) -> np.ndarray:
    """Random smooth periodic orbitals: N(0,1) noise, periodic Gaussian filter, unit RMS, FP32.

    The filter is a periodic Gaussian with standard deviation ``width_cells``
    grid cells per axis, applied in Fourier space.  Every value is rounded to
    FP32 (and then widened again if ``dtype`` is float64), so the same table
    is exactly representable in both precisions.  Layout [gx][gy][gz][n_orb].
    """
    G = grid
    rng = np.random.default_rng([seed, 0x5011D])
    f = np.fft.fftfreq(G)  # cycles per grid cell
    h = np.exp(-2.0 * (math.pi * width_cells * f) ** 2)
    H = h[:, None, None] * h[None, :, None] * h[None, None, :]
    out = np.empty((G, G, G, n_orb), dtype=dtype)
    for j in range(n_orb):
        noise = rng.standard_normal((G, G, G))
        sm = np.fft.ifftn(np.fft.fftn(noise) * H).real
        sm /= math.sqrt(float(np.mean(sm * sm)))
        out[..., j] = sm.astype(np.float32)
    return out


def request_table(bank: np.ndarray, n_orb: int, seed: int) -> np.ndarray:
    """A request's own table from an orbital bank [G][G][G][M] of ``solid_table``: the cyclic
    window of n_orb orbitals starting at a seeded offset, translated on the periodic grid by a
    seeded shift per axis, each orbital with a seeded sign.  Translation, selection and sign
    keep the orbitals draws of the same stationary filtered field."""
    rng = np.random.default_rng([seed, 0x7AB1E])
    G, M = bank.shape[0], bank.shape[3]
    if n_orb > M:
        raise ValueError("the bank holds fewer orbitals than requested")
    start = int(rng.integers(0, M))
    idx = (start + np.arange(n_orb)) % M
    shift = rng.integers(0, G, size=3)
    sign = np.where(rng.random(n_orb) < 0.5, -1.0, 1.0).astype(bank.dtype)
    # out[x, y, z, j] = sign_j bank[x - sx, y - sy, z - sz, idx_j] (periodic), one gather
    ax = [(np.arange(G) - int(sh)) % G for sh in shift]
    out = bank[np.ix_(ax[0], ax[1], ax[2], idx)]
    out *= sign
    return out


def bspline_jastrow_params(M: int, A: float) -> np.ndarray:
    """Synthetic control points p_1..p_M = -A (1 - (m-1)/(M-1))^3 (p_M = 0)."""
    m = np.arange(1, M + 1, dtype=np.float64)
    return -A * (1.0 - (m - 1.0) / (M - 1.0)) ** 3


def j3_params(m_ei: int, m_ee: int, rc: float, seed: int, A: float = 0.05) -> dict:
    """Seeded coefficients of the three-body term: gamma_lmn = A z_lmn / (h^(6+l+m) (2h)^n),
    h = rc/2, z uniform in (-1, 1) and symmetric in (l, m), one set per spin relation (same,
    opposite), so that no single term exceeds A in size inside the cutoff."""
    rng = np.random.default_rng([seed, 0x3B0D])
    h = rc / 2.0
    g = np.zeros((2, m_ei + 1, m_ei + 1, m_ee + 1))
    for sp in range(2):
        z = rng.uniform(-1.0, 1.0, size=(m_ei + 1, m_ei + 1, m_ee + 1))
        z = 0.5 * (z + z.transpose(1, 0, 2))
        for l in range(m_ei + 1):
            for m in range(m_ei + 1):
                for n in range(m_ee + 1):
                    g[sp, l, m, n] = A * z[l, m, n] / (h ** (6 + l + m) * (2 * h) ** n)
    return {"m_ei": m_ei, "m_ee": m_ee, "rc": rc, "gamma": g}


def solid(n_elec: int, grid: int, n_walkers: int, n_sweeps: int, precision: str = "fp64",
          table_dtype=None, delay_rank: int = 1, recompute_period: int = 0, seed: int = 0,
          sigma: float = 0.3, M: int = 8, A_ee: float = 0.4, A_eI: float = 0.3,
          ions_per_elec: float = 0.25, Z: float = 4.0, name: Optional[str] = None,
          j3: bool = False, j3_strength: float = 0.05) -> Workload:
    """Spin-balanced solid-like system at rs = 1 with one- and two-body B-spline Jastrows
    (and, with j3, a three-body e-e-I term of orders 2, 2 and cutoff L/2)."""
    if n_elec % 2:
        raise ValueError("solid-like systems are spin balanced: n_elec must be even")
    ns = n_elec // 2
    L = cell_side(n_elec)
    if table_dtype is None:
        table_dtype = np.float64 if precision == "fp64" else np.float32
    coefs = solid_table(ns, grid, seed, dtype=table_dtype)
    n_ions = max(1, int(round(n_elec * ions_per_elec)))
    irng = np.random.default_rng([seed, 0x10A5])
    ion_pos = irng.uniform(0.0, L, size=(n_ions, 3))
    ion_Z = np.full(n_ions, n_elec / n_ions if Z is None else Z)
    rc = L / 2.0
    j2 = {"kind": "bspline", "M": M, "rc": rc, "p": bspline_jastrow_params(M, A_ee),
          "cusp_same": 0.25, "cusp_opp": 0.5}
    j1 = {"kind": "bspline", "M": M, "rc": rc, "p": bspline_jastrow_params(M, A_eI), "cusp": 0.0}
    return Workload(
        name=name or f"solid{n_elec}_g{grid}_{precision}", n_up=ns, n_dn=ns, L=L, n_orb=ns,
        grid=(grid, grid, grid), coefs=coefs, ion_pos=ion_pos, ion_Z=ion_Z, j2=j2, j1=j1,
        hamiltonian="coulomb", sigma=sigma, seed=seed, n_walkers=n_walkers, n_sweeps=n_sweeps,
        precision=precision, delay_rank=delay_rank, recompute_period=recompute_period,
        j3=j3_params(2, 2, rc, seed, A=j3_strength) if j3 else None)


# --------------------------------------------------------------------------
# The named workloads
# --------------------------------------------------------------------------

def heg14(jastrow: bool = True, grid: int = 16, hamiltonian: str = "coulomb") -> Workload:
    """14-electron gas, 16^3 table, Pade J2 (a=0.5, b=1), 8 walkers, 100 sweeps, seed 0."""
    return heg(7, grid=grid, jastrow=jastrow, hamiltonian=hamiltonian)


def solid128() -> Workload:
    """128 electrons, 64 orbitals on 48^3 (FP32-exact values stored FP64), 32 ions, 512 walkers."""
    return solid(128, 48, n_walkers=512, n_sweeps=200, precision="fp64", name="solid128_fp64")


def mixed384(precision: str = "mixed") -> Workload:
    """384 electrons, 192 orbitals on 64^3 in FP32, 96 ions, rank-32 delay, LU every 64 sweeps."""
    return solid(384, 64, n_walkers=1024, n_sweeps=500, precision=precision,
                 table_dtype=np.float32 if precision == "mixed" else np.float64,
                 delay_rank=32 if precision == "mixed" else 1,
                 recompute_period=64 if precision == "mixed" else 0, name=f"solid384_{precision}")


def batched_systems(n_walkers: int = 256, n_sweeps: int = 100):
    """Four uneven solid-like FP32 systems for one batched launch."""
    spec = [(32, 24), (96, 32), (192, 48), (512, 64)]
    return [solid(n, g, n_walkers=n_walkers, n_sweeps=n_sweeps, precision="mixed",
                  table_dtype=np.float32, delay_rank=16, recompute_period=64, seed=i,
                  name=f"batched{n}_g{g}") for i, (n, g) in enumerate(spec)]


def served_trace(n_requests: int = 200, rate_per_s: float = 20.0, seed: int = 0):
    """Poisson request stream: electron counts log-uniform in [32, 1024] (even), grids 32..64,
    64..1024 walkers (multiples of 64), 100..1000 sweeps.  Returns a list of dicts."""
    rng = np.random.default_rng([seed, 0x5E7E])
    t = 0.0
    out = []
    for rid in range(n_requests):
        t += rng.exponential(1.0 / rate_per_s)
        n = 2 * int(round(math.exp(rng.uniform(math.log(32), math.log(1024))) / 2))
        out.append({
            "id": rid, "arrival_s": t, "n_elec": n,
            "grid": int(rng.choice([32, 40, 48, 56, 64])),
            "n_walkers": 64 * int(rng.integers(1, 17)),
            "n_sweeps": int(rng.integers(100, 1001)), "seed": rid,
        })
    return out


WORKLOADS = {
    "heg14": heg14,
    "solid128": solid128,
    "mixed384": mixed384,
}
