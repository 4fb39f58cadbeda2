"""Seeded synthetic systems (no method arithmetic here).

Every workload of the build is described by a :class:`SystemSpec`: the mesh, the
atoms, the atom-centred enrichment list, the occupations, the propagation
parameters and the random draws of the initial-state recipe.  The oracle and the
GPU library both receive exactly these numbers and derive everything else
(basis, Hamiltonian, initial orbitals) independently.

Physical choices follow the paper's sodium-cluster study (Sec. 3.3, Table 2) at
the sizes of the benchmark configurations, with the readings stated in the
design notes: Gaussian-smeared nuclei of width 0.2 bohr, Slater-type enrichment
radial functions r^l exp(-zeta r) with the smooth cutoff (1-(r/r_c)^2)^3 and
r_c = 6 bohr, zetas from Slater's rules for sodium.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Tuple

import numpy as np

# (m_x, m_y, m_z) of the low-frequency sine modes of the initial-state noise,
# lexicographic with m_x slowest.
NOISE_MODES: List[Tuple[int, int, int]] = [
    (mx, my, mz) for mx in (1, 2, 3) for my in (1, 2, 3) for mz in (1, 2, 3)]

# Slater's-rules exponents for Na: 1s, 2s/2p, 3s (bohr^-1).
NA_ZETA_1S = 10.70
NA_ZETA_2SP = 3.425
NA_ZETA_3S = 0.733


@dataclasses.dataclass
class SystemSpec:
    name: str
    ncell: Tuple[int, int, int]
    lo: Tuple[float, float, float]
    hi: Tuple[float, float, float]
    degree: int
    R: np.ndarray                 # (natom, 3) bohr
    Z: np.ndarray                 # (natom,)
    nuc_sigma: float
    enr_atom: np.ndarray          # (nenr,) int
    enr_l: np.ndarray             # (nenr,) int, 0 or 1
    enr_m: np.ndarray             # (nenr,) int, -1 (y), 0 (z), +1 (x) for l = 1
    enr_zeta: np.ndarray          # (nenr,)
    r_cut: float
    occ: np.ndarray               # (norb,) occupation f_alpha
    xc: str                       # "none" | "slater" | "slater_pw92"
    trap_omega: float = 0.0       # > 0: add 1/2 w^2 |x|^2 (test systems only)
    quad_cell: int = 0            # Gauss points per direction, 0 -> degree + 1
    quad_enr: int = 0             # Gauss points per direction, 0 -> 2 degree + 2
    enr_drop_tol: float = 1e-8    # canonical-orthogonalisation threshold
    # graded tensor-product mesh: per axis the ncell[d] + 1 cell boundaries from lo[d] to hi[d]
    # (None: uniform cells)
    bounds: Optional[Tuple[np.ndarray, np.ndarray, np.ndarray]] = None
    # propagation
    dt: float = 0.05
    nsteps: int = 1
    krylov_tol: float = 1e-10
    kmax: int = 64
    kick: float = 0.0
    kick_dir: int = 2             # 0 x, 1 y, 2 z
    # initial state
    init: str = "scf"             # "scf" | "enr_noise"
    init_enr: Optional[np.ndarray] = None   # (norb,) enrichment index per orbital
    noise_amp: float = 0.1
    noise_seed0: int = 1000

    @property
    def natom(self) -> int:
        return int(len(self.Z))

    @property
    def nenr(self) -> int:
        return int(len(self.enr_zeta))

    @property
    def norb(self) -> int:
        return int(len(self.occ))

    @property
    def n_electrons(self) -> float:
        return float(np.sum(self.occ))

    @property
    def qcell(self) -> int:
        return self.quad_cell if self.quad_cell > 0 else self.degree + 1

    @property
    def qenr(self) -> int:
        return self.quad_enr if self.quad_enr > 0 else 2 * self.degree + 2

    def noise(self) -> np.ndarray:
        """(norb, 27) N(0,1) draws, orbital alpha drawn from seed noise_seed0+alpha."""
        return noise_coefficients(self.norb, self.noise_seed0)


def noise_coefficients(norb: int, seed0: int = 1000) -> np.ndarray:
    g = np.empty((norb, len(NOISE_MODES)))
    for a in range(norb):
        g[a] = np.random.default_rng(seed0 + a).standard_normal(len(NOISE_MODES))
    return g


def cluster_positions(natom: int, radius: float, min_sep: float = 5.5,
                      seed: int = 0, restart_after: int = 2000) -> np.ndarray:
    """Uniform rejection sampling in a ball, with a minimum separation.

    Candidates are drawn uniformly in the cube [-radius, radius]^3 and kept if
    they fall inside the ball and at least ``min_sep`` from every accepted atom.
    After ``restart_after`` consecutive rejections the sampler restarts from an
    empty set (it can otherwise jam).
    """
    rng = np.random.default_rng(seed)
    pos: List[np.ndarray] = []
    rejects = 0
    while len(pos) < natom:
        x = rng.uniform(-radius, radius, size=3)
        ok = float(np.dot(x, x)) <= radius * radius and all(
            float(np.linalg.norm(x - y)) >= min_sep for y in pos)
        if ok:
            pos.append(x)
            rejects = 0
        else:
            rejects += 1
            if rejects >= restart_after:
                pos = []
                rejects = 0
    return np.array(pos, dtype=np.float64)


def tiny() -> SystemSpec:
    """One Li-like atom (Z = 3) at the origin, 4^3 cells of degree 4 on [-8, 8]^3."""
    return SystemSpec(
        name="tiny", ncell=(4, 4, 4), lo=(-8.0,) * 3, hi=(8.0,) * 3, degree=4,
        R=np.zeros((1, 3)), Z=np.array([3.0]), nuc_sigma=0.2,
        enr_atom=np.zeros(5, dtype=np.int32),
        enr_l=np.array([0, 0, 1, 1, 1], dtype=np.int32),
        enr_m=np.array([0, 0, -1, 0, 1], dtype=np.int32),
        enr_zeta=np.array([3.0, 1.2, 1.0, 1.0, 1.0]),
        r_cut=6.0, occ=np.array([2.0, 1.0]), xc="slater",
        dt=0.05, nsteps=200, krylov_tol=1e-10, kmax=64, kick=1e-3, kick_dir=2,
        init="scf")


def na_cluster(natom: int, seed: int, ncell: Optional[int] = None,
               kick: float = 1e-3, kick_dir: int = 2) -> SystemSpec:
    """Na_n cluster: ball radius 6 (n/8)^(1/3), cells of 40/24 bohr, degree 5.

    Orbitals: the 1s, 2s, 2p enrichment functions of every atom (core) plus the
    3s of atoms 0 .. n/2-1 (valence); each doubly occupied, 11 n electrons.
    """
    radius = 6.0 * (natom / 8.0) ** (1.0 / 3.0)
    if ncell is None:
        ncell = {2: 12, 4: 16, 6: 20, 8: 24}[natom]
    half = 20.0 * ncell / 24.0
    R = cluster_positions(natom, radius, 5.5, seed)
    enr_atom, enr_l, enr_m, enr_zeta = [], [], [], []
    for a in range(natom):
        for (l, m, z) in ((0, 0, NA_ZETA_1S), (0, 0, NA_ZETA_2SP),
                          (1, -1, NA_ZETA_2SP), (1, 0, NA_ZETA_2SP),
                          (1, 1, NA_ZETA_2SP), (0, 0, NA_ZETA_3S)):
            enr_atom.append(a); enr_l.append(l); enr_m.append(m); enr_zeta.append(z)
    core = [6 * a + j for a in range(natom) for j in range(5)]
    valence = [6 * a + 5 for a in range(natom // 2)]
    init_enr = np.array(core + valence, dtype=np.int32)
    norb = len(init_enr)
    return SystemSpec(
        name=f"Na{natom}", ncell=(ncell,) * 3, lo=(-half,) * 3, hi=(half,) * 3,
        degree=5, R=R, Z=np.full(natom, 11.0), nuc_sigma=0.2,
        enr_atom=np.array(enr_atom, dtype=np.int32),
        enr_l=np.array(enr_l, dtype=np.int32),
        enr_m=np.array(enr_m, dtype=np.int32),
        enr_zeta=np.array(enr_zeta), r_cut=6.0,
        occ=np.full(norb, 2.0), xc="slater_pw92",
        dt=0.02, nsteps=100, krylov_tol=1e-10, kmax=64,
        kick=kick, kick_dir=kick_dir, init="enr_noise", init_enr=init_enr)


def na8() -> SystemSpec:
    """8 Na atoms, 24^3 cells of degree 5 on [-20, 20]^3 (1,771,561 nodes), 44 orbitals."""
    return na_cluster(8, seed=0)


def hhg_field(kappa: float = 0.01, omega: float = 0.03, ncycles: int = 5, direction: int = 0) -> dict:
    """The sinusoidal pulse of the high-harmonic study, kappa sin(pi t / T) sin(omega t) on
    [0, T], T = ncycles 2 pi / omega, in the sum-of-sines form the field interface takes
    (sum_k A_k sin(w_k t + phi_k) with a flat envelope, s = inf), using
    sin(a) sin(b) = (cos(a - b) - cos(a + b)) / 2 and cos(x) = sin(x + pi/2)."""
    T = ncycles * 2.0 * np.pi / omega
    return dict(direction=direction, A=np.array([0.5 * kappa, -0.5 * kappa]),
                w=np.array([omega - np.pi / T, omega + np.pi / T]), phi=np.array([0.5 * np.pi, 0.5 * np.pi]),
                t0=0.0, s=float("inf"), T=T)


def graded_bounds(lo: float, hi: float, ncell: int, beta: float) -> np.ndarray:
    """ncell + 1 cell boundaries on [lo, hi] from x = c + a sinh(beta xi) / sinh(beta),
    xi uniform on [-1, 1] (c, a the box centre and half-length; beta = 0: uniform).
    Cells are finest at the centre and grow smoothly toward both faces."""
    xi = np.linspace(-1.0, 1.0, ncell + 1)
    c, a = 0.5 * (lo + hi), 0.5 * (hi - lo)
    b = c + a * (xi if beta == 0.0 else np.sinh(beta * xi) / np.sinh(beta))
    b[0], b[-1] = lo, hi
    return b


def lattice13() -> SystemSpec:
    """Thirteen Z = 1 atoms on a 2.5-bohr lattice (the centre, the 8 cube corners
    and 4 face points) in the tiny box, each with a 1s (zeta 2.5) and three 2p
    (zeta 1.8) enrichment functions: 52 functions, all nonzero on the central
    cells, so more than 48 meet on one T-cell and more than 48 are kept."""
    base = tiny()
    pos = [(0.0, 0.0, 0.0)] + [(a, b, c) for a in (-2.5, 2.5) for b in (-2.5, 2.5) for c in (-2.5, 2.5)] + \
          [(2.5, 0.0, 0.0), (-2.5, 0.0, 0.0), (0.0, 2.5, 0.0), (0.0, -2.5, 0.0)]
    R = np.array(pos)
    na = len(R)
    return dataclasses.replace(
        base, name="lattice13", R=R, Z=np.full(na, 1.0),
        enr_atom=np.repeat(np.arange(na), 4).astype(np.int32),
        enr_l=np.tile([0, 1, 1, 1], na).astype(np.int32),
        enr_m=np.tile([0, -1, 0, 1], na).astype(np.int32),
        enr_zeta=np.tile([2.5, 1.8, 1.8, 1.8], na).astype(float))


def tiny_graded() -> SystemSpec:
    """The tiny system on a graded, axis-dependent 4^3 mesh of [-8, 8]^3."""
    s = tiny()
    s.name = "tiny_graded"
    s.bounds = (np.array([-8.0, -2.5, 0.0, 3.0, 8.0]),
                np.array([-8.0, -3.5, -0.5, 2.5, 8.0]),
                np.array([-8.0, -4.0, 0.5, 4.0, 8.0]))
    return s


def na8_graded() -> SystemSpec:
    """Na8 in a 70-bohr box (the domain length of the paper's Na_3 / Na_11 runs) with
    the node count of na8(): 24^3 cells of degree 5, sinh-graded with beta = 1.93, so the
    central cells keep about the 40/24 bohr of the uniform mesh and the outer ones reach 5.5."""
    s = na_cluster(8, seed=0)
    s.name = "Na8_graded"
    s.lo, s.hi = (-35.0,) * 3, (35.0,) * 3
    s.bounds = tuple(graded_bounds(-35.0, 35.0, 24, 1.93) for _ in range(3))
    return s


def trap(omega: float = 0.5, ncell: int = 6, half: float = 9.0, degree: int = 4,
         xc: str = "slater") -> SystemSpec:
    """Two electrons in a harmonic trap: no atoms, no enrichment (test system)."""
    return SystemSpec(
        name="trap", ncell=(ncell,) * 3, lo=(-half,) * 3, hi=(half,) * 3,
        degree=degree, R=np.zeros((0, 3)), Z=np.zeros(0), nuc_sigma=0.2,
        enr_atom=np.zeros(0, dtype=np.int32), enr_l=np.zeros(0, dtype=np.int32),
        enr_m=np.zeros(0, dtype=np.int32), enr_zeta=np.zeros(0), r_cut=6.0,
        occ=np.array([2.0]), xc=xc, trap_omega=omega,
        dt=0.05, nsteps=1, krylov_tol=1e-10, kmax=64, kick=1e-3, kick_dir=2,
        init="scf")


def gaussian_box(ncell: int, half: float, degree: int) -> SystemSpec:
    """Empty box (no atoms, no enrichment, no electrons): mesh-only test system."""
    return SystemSpec(
        name="box", ncell=(ncell,) * 3, lo=(-half,) * 3, hi=(half,) * 3,
        degree=degree, R=np.zeros((0, 3)), Z=np.zeros(0), nuc_sigma=0.2,
        enr_atom=np.zeros(0, dtype=np.int32), enr_l=np.zeros(0, dtype=np.int32),
        enr_m=np.zeros(0, dtype=np.int32), enr_zeta=np.zeros(0), r_cut=6.0,
        occ=np.zeros(0), xc="none", init="scf")


def adjoint_field_params(seed, ncomp=3, a_range=(1e-3, 1e-2), w_range=(0.5, 5.0)):
    """Seeded field parameters theta = (A_1..A_m, w_1..w_m, phi_1..phi_m) of a
    sum-of-sines pulse: A ~ U(a_range), w ~ U(w_range), phi ~ U[0, 2 pi)."""
    rng = np.random.default_rng(seed)
    A = rng.uniform(a_range[0], a_range[1], ncomp)
    w = rng.uniform(w_range[0], w_range[1], ncomp)
    phi = rng.uniform(0.0, 2.0 * np.pi, ncomp)
    return np.concatenate([A, w, phi])


# The field-gradient workload on the tiny system: no kick, 20 steps of 0.05 au,
# envelope centre 0.5 and width 0.4, theta from seed 7, target trace from seed 8.
ADJOINT_TINY = dict(nsteps=20, dt=0.05, t0=0.5, s=0.4, seed=7, seed_target=8, ncomp=3)
