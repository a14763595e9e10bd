"""Seeded synthetic workloads for the coupled Yee-FDTD / quantum-emitter step.

This module only draws inputs: grid sizes, permittivity maps, emitter
positions, frequencies, dipoles, initial states and source parameters.  It
holds none of the method's arithmetic (no kernel weights, no propagation), so
both the CPU oracle and the HIP library can be fed from it.

Units are natural (c = eps0 = mu0 = hbar = 1, dx = 1 cell, dt = 0.5 dx: the
paper's runs all use c dt / dx ~ 0.50, App. B Table III).  Kernels are
Gaussians of width sigma = dx (App. B).  Random draws use numpy PCG64
``default_rng(seed)``; the draw order below is fixed.

Workloads (sizes are arguments so tests can shrink them):
  * ``single_emitter``   -- 32^3 PEC box, one TLS at the centre (omega0 0.25,
    d = 0.01 z), probe E_z 8 cells away, 1000 steps, FP64.
  * ``slab``             -- 128^3, 10-cell CPML, eps 2.25 slab 16 cells thick,
    1000 TLS in the slab, y-polarised Gaussian-pulse plane wave, 5000 steps.
  * ``bragg``            -- 64x64x1024, periodic x/y, CPML z, 20 quarter-wave
    pairs with a half-wave defect holding 10,000 multilevel (2-6) emitters
    with random Hamiltonians and dephasing 1e-3, 20,000 steps.
  * ``batch``            -- 64 independent cubic domains 32^3..96^3, CPML 8,
    random eps per 8^3 block, 1-256 TLS each, 2000 steps.
  * ``radiating_cube``   -- 256^3, 10-cell CPML, 100,000 TLS in the central
    128^3, flux plane at z index 200, design box [96,160)^3, 4000 steps.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

SQRT_HALF = float(np.sqrt(0.5))


@dataclass
class TLSSet:
    pos: np.ndarray      # (M,3) cell units, domain [0, N] per axis
    sigma: np.ndarray    # (M,)
    gamma: np.ndarray    # (M,)
    omega0: np.ndarray   # (M,)
    dipole: np.ndarray   # (M,3)
    rho0: np.ndarray     # (M,3): rho11, Re rho01, Im rho01

    def __len__(self):
        return int(self.pos.shape[0])

    def subset(self, idx):
        idx = np.asarray(idx)
        return TLSSet(self.pos[idx], self.sigma[idx], self.gamma[idx], self.omega0[idx],
                      self.dipole[idx], self.rho0[idx])


@dataclass
class MultilevelSet:
    nlev: np.ndarray           # (M,) int
    energies: List[np.ndarray]  # H0 eigenvalues per emitter
    mop: List[np.ndarray]      # real symmetric dipole matrix per emitter
    dipole: np.ndarray         # (M,3)
    gphi: np.ndarray           # (M,)
    rho0: List[np.ndarray]     # complex (L,L)
    pos: np.ndarray
    sigma: np.ndarray
    gamma: np.ndarray

    def __len__(self):
        return int(len(self.nlev))

    def subset(self, idx):
        idx = [int(q) for q in np.asarray(idx)]
        return MultilevelSet(self.nlev[idx], [self.energies[q] for q in idx],
                             [self.mop[q] for q in idx], self.dipole[idx], self.gphi[idx],
                             [self.rho0[q] for q in idx], self.pos[idx], self.sigma[idx],
                             self.gamma[idx])


@dataclass
class PlaneSource:
    axis: int
    index: int
    comp: int
    amp: float
    omega: float
    tau: float
    t0: float


@dataclass
class PointSource:
    comp: int
    ijk: Tuple[int, int, int]
    amp: float
    omega: float
    tau: float
    t0: float


@dataclass
class Workload:
    name: str
    shape: Tuple[int, int, int]          # (nx, ny, nz)
    bc: Tuple[str, ...] = ("pec",) * 6   # x-, x+, y-, y+, z-, z+
    cpml: Tuple[int, ...] = (0,) * 6
    dx: float = 1.0
    courant: float = 0.5
    eps: Optional[np.ndarray] = None     # (nz, ny, nx) relative permittivity, None = vacuum
    tls: Optional[TLSSet] = None
    multilevel: Optional[MultilevelSet] = None
    plane_sources: List[PlaneSource] = field(default_factory=list)
    point_sources: List[PointSource] = field(default_factory=list)
    probes: List[Tuple[int, Tuple[int, int, int]]] = field(default_factory=list)
    flux: Optional[Tuple[int, int]] = None
    pop_every: int = 0
    steps: int = 1000
    precision: str = "fp64"              # "fp64" or "fp32" (FP32 fields, FP64 emitters)
    design_box: Optional[Tuple[int, int, int, int, int, int]] = None  # x0,x1,y0,y1,z0,z1

    @property
    def ncell(self):
        return int(np.prod(self.shape))

    @property
    def n_emitters(self):
        return (len(self.tls) if self.tls is not None else 0) + \
            (len(self.multilevel) if self.multilevel is not None else 0)


def _unit_vectors(rng, n):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _tls_state(kind, n):
    """rho0 rows (rho11, Re rho01, Im rho01) for a pure state c_g|0> + c_e|1>."""
    if kind == "ground":
        cg, ce = 1.0, 0.0
    elif kind == "excited":
        cg, ce = 0.0, 1.0
    elif kind == "superposition":
        cg, ce = SQRT_HALF, SQRT_HALF
    elif kind == "weak":
        cg, ce = float(np.sqrt(0.9999)), 0.01
    else:
        raise ValueError(kind)
    row = np.array([ce * ce, cg * ce, 0.0])   # rho01 = c_g c_e^* (real amplitudes)
    return np.tile(row, (n, 1))


def gaussian_pulse_params(omega_c=0.25, rel_width=0.3 / 3.5):
    """Centre frequency, tau and t0 of the plane-wave pulse: the relative width of the
    paper's pulse (3.5 um^-1 centre, 0.3 um^-1 width, App. B) at centre omega_c."""
    dw = omega_c * rel_width
    tau = 1.0 / dw
    return omega_c, tau, 5.0 * tau


def single_emitter(state="excited", n=32, steps=1000, precision="fp64"):
    tls = TLSSet(pos=np.array([[n / 2, n / 2, n / 2]], dtype=np.float64),
                 sigma=np.ones(1), gamma=np.ones(1), omega0=np.array([0.25]),
                 dipole=np.array([[0.0, 0.0, 0.01]]), rho0=_tls_state(state, 1))
    return Workload(name=f"single_emitter_{state}_{n}^3", shape=(n, n, n), tls=tls,
                    probes=[(2, (3 * n // 4, n // 2, n // 2))], pop_every=1, steps=steps,
                    precision=precision)


def tls_ensemble(rng, n, lo, hi, state):
    pos = rng.uniform(lo, hi, size=(n, 3))
    omega0 = rng.uniform(0.24, 0.26, size=n)
    dip = 0.01 * _unit_vectors(rng, n)
    return TLSSet(pos=pos, sigma=np.ones(n), gamma=np.ones(n), omega0=omega0, dipole=dip,
                  rho0=_tls_state(state, n))


def slab(n=128, n_emit=1000, steps=5000, cpml=10, thick=16, precision="fp32", seed=2):
    """Dielectric slab (eps 2.25) with TLS inside, excited by a y-polarised pulse."""
    rng = np.random.default_rng(seed)
    z0 = n // 2 - thick // 2
    eps = np.ones((n, n, n))
    eps[z0:z0 + thick] = 2.25
    lo = np.array([cpml + 4, cpml + 4, z0], dtype=np.float64)
    hi = np.array([n - cpml - 4, n - cpml - 4, z0 + thick], dtype=np.float64)
    # keep windows inside the slab's reach but clear of the PML interface
    lo[2] = max(lo[2], cpml + 4)
    hi[2] = min(hi[2], n - cpml - 4)
    tls = tls_ensemble(rng, n_emit, lo, hi, "ground")
    w, tau, t0 = gaussian_pulse_params()
    src = PlaneSource(axis=2, index=cpml + 2, comp=1, amp=1.0, omega=w, tau=tau, t0=t0)
    return Workload(name=f"slab_{n}^3_cpml{cpml}_{n_emit}tls", shape=(n, n, n),
                    bc=("cpml",) * 6, cpml=(cpml,) * 6, eps=eps, tls=tls, plane_sources=[src],
                    probes=[(1, (n // 2, n // 2, n - cpml - 6)), (1, (n // 2, n // 2, cpml + 4))],
                    pop_every=max(1, steps // 50), steps=steps, precision=precision)


def random_multilevel(rng, n_emit, pos, levels=(2, 6), gphi=1e-3, dmag=0.01, w01=0.25):
    """Random model Hamiltonians: H0 from the spectrum of a random Hermitian matrix
    shifted to E0 = 0 and scaled to E1 - E0 = w01; dipole matrix M real symmetric with
    zero diagonal and max |M_ij| = 1; initial state (|0> + |1>)/sqrt 2."""
    nlev = rng.integers(levels[0], levels[1] + 1, size=n_emit)
    energies, mops, rhos = [], [], []
    for q in range(n_emit):
        L = int(nlev[q])
        A = rng.standard_normal((L, L)) + 1j * rng.standard_normal((L, L))
        Hh = 0.5 * (A + A.conj().T)
        ev = np.sort(np.linalg.eigvalsh(Hh))
        ev = ev - ev[0]
        ev = ev * (w01 / ev[1])
        energies.append(ev)
        Mm = rng.standard_normal((L, L))
        Mm = 0.5 * (Mm + Mm.T)
        np.fill_diagonal(Mm, 0.0)
        Mm = Mm / np.max(np.abs(Mm))
        mops.append(Mm)
        psi = np.zeros(L, dtype=np.complex128)
        psi[0] = psi[1] = SQRT_HALF
        rhos.append(np.outer(psi, psi.conj()))
    dip = dmag * _unit_vectors(rng, n_emit)
    return MultilevelSet(nlev=nlev.astype(np.int32), energies=energies, mop=mops, dipole=dip,
                         gphi=np.full(n_emit, gphi), rho0=rhos, pos=pos,
                         sigma=np.ones(n_emit), gamma=np.ones(n_emit))


def bragg(nx=64, ny=64, nz=1024, n_emit=10000, steps=20000, pairs_per_mirror=10, cpml=10,
          precision="fp32", seed=3):
    """Bragg resonator: quarter-wave layers (6 cells eps 1, 4 cells eps 2.25 at design
    frequency 0.25), pairs_per_mirror pairs per mirror, a 12-cell half-wave defect in the
    middle holding the multilevel emitters; periodic in x/y, CPML in z."""
    rng = np.random.default_rng(seed)
    eps_z = []
    for _ in range(pairs_per_mirror):
        eps_z += [1.0] * 6 + [2.25] * 4
    defect0 = len(eps_z)
    eps_z += [1.0] * 12
    for _ in range(pairs_per_mirror):
        eps_z += [2.25] * 4 + [1.0] * 6
    stack = np.array(eps_z)
    if stack.size + 2 * (cpml + 4) > nz:
        raise ValueError("stack does not fit")
    z_start = (nz - stack.size) // 2
    prof = np.ones(nz)
    prof[z_start:z_start + stack.size] = stack
    eps = np.broadcast_to(prof[:, None, None], (nz, ny, nx)).copy()
    zd0 = z_start + defect0
    pos = np.column_stack([rng.uniform(0, nx, n_emit), rng.uniform(0, ny, n_emit),
                           rng.uniform(zd0, zd0 + 12, n_emit)])
    ml = random_multilevel(rng, n_emit, pos)
    return Workload(name=f"bragg_{nx}x{ny}x{nz}_{n_emit}ml", shape=(nx, ny, nz),
                    bc=("periodic", "periodic", "periodic", "periodic", "cpml", "cpml"),
                    cpml=(0, 0, 0, 0, cpml, cpml), eps=eps, multilevel=ml,
                    probes=[(0, (nx // 2, ny // 2, zd0 + 6))], pop_every=max(1, steps // 50),
                    steps=steps, precision=precision)


def batch_domain(rng, n, cpml=8, max_emit=256, steps=2000, precision="fp32"):
    nb = n // 8
    blk = rng.choice(np.array([1.0, 2.25, 4.0]), size=(nb, nb, nb))
    nbp = cpml // 8
    if nbp:
        blk[:nbp], blk[-nbp:] = 1.0, 1.0
        blk[:, :nbp], blk[:, -nbp:] = 1.0, 1.0
        blk[:, :, :nbp], blk[:, :, -nbp:] = 1.0, 1.0
    eps = np.kron(blk, np.ones((8, 8, 8)))
    ne = int(rng.integers(1, max_emit + 1))
    tls = tls_ensemble(rng, ne, cpml + 4, n - cpml - 4, "superposition")
    return Workload(name=f"domain_{n}^3_{ne}tls", shape=(n, n, n), bc=("cpml",) * 6,
                    cpml=(cpml,) * 6, eps=eps, tls=tls, probes=[(2, (n // 2, n // 2, n // 2))],
                    steps=steps, precision=precision)


def batch(n_domains=64, sizes=(4, 12), steps=2000, cpml=8, max_emit=256, precision="fp32",
          seed=4):
    """Independent cubic domains of edge 8*U{sizes}, each with its own RNG stream."""
    out = []
    for child in np.random.SeedSequence(seed).spawn(n_domains):
        rng = np.random.default_rng(child)
        n = 8 * int(rng.integers(sizes[0], sizes[1] + 1))
        out.append(batch_domain(rng, n, cpml=cpml, max_emit=max_emit, steps=steps,
                                precision=precision))
    return out


def radiating_cube(n=256, n_emit=100000, steps=4000, cpml=10, emit_box=None, design_box=None,
                   flux_index=None, precision="fp32", seed=5):
    """Vacuum cube with TLS in superposition states filling the central half; the
    objective plane sits at z index 200 of 256 (scaled with n)."""
    rng = np.random.default_rng(seed)
    if emit_box is None:
        emit_box = (max(n // 4, cpml + 4), min(3 * n // 4, n - cpml - 4))
    if design_box is None:
        a = 3 * n // 8
        design_box = (a, n - a) * 3
    if flux_index is None:
        flux_index = int(round(200 * n / 256))
    tls = tls_ensemble(rng, n_emit, emit_box[0], emit_box[1], "superposition")
    return Workload(name=f"radiating_cube_{n}^3_cpml{cpml}_{n_emit}tls", shape=(n, n, n),
                    bc=("cpml",) * 6, cpml=(cpml,) * 6, eps=None, tls=tls,
                    probes=[(0, (n // 2, n // 2, flux_index))], flux=(2, flux_index),
                    steps=steps, precision=precision, design_box=design_box)
