"""Seeded synthetic workloads for Langevin Speculative Dynamics.

This module only generates inputs: positions, momenta, boxes, species and
run parameters.  It holds none of the method's arithmetic (no forces, no
integrator, no transport map), so both the HIP path and the CPU oracle can be
fed from it.  Every floating-point value it returns is exactly representable
in binary32, so the FP32 device state and the FP64 oracle start from
bit-identical numbers.

The paper's own workloads (FCC copper, bulk water, LGPS, alanine peptides
with pretrained interatomic potentials) are not available; these seeded
systems stand in for them:

* ``lj_fluid``: Lennard-Jones fluid in reduced units (epsilon = sigma = m =
  k_B = 1) on a jittered simple-cubic lattice with Maxwell-Boltzmann momenta.
* ``triatomic_liquid``: rigid-geometry bent triatomics (three species) on a
  jittered lattice with random orientations, in Angstrom / amu / fs / eV.
"""
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

# 1 eV/Angstrom expressed in amu * Angstrom / fs^2 (CODATA 2018 eV and amu)
EV_PER_A_IN_AMU_A_PER_FS2 = 9.648533212331e-3
BOLTZMANN_EV_PER_K = 8.617333262e-5


def f32(a):
    """Round to the nearest binary32 value, returned as float64."""
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


@dataclass
class Workload:
    """One system (or a batch of replicas) with its run parameters."""
    name: str
    positions: np.ndarray          # [N, 3] float64, binary32-representable, in [0, L_r)
    momenta: np.ndarray            # [N, 3] float64, binary32-representable
    species: np.ndarray            # [N] int32
    species_mass: np.ndarray       # [S] float64
    atom_offsets: np.ndarray       # [R + 1] int32
    box: np.ndarray                # [R] float64 (binary32-representable edges)
    dt: float
    gamma: float
    kT: float
    force_unit: float
    K: int
    n_steps: int
    seed: int
    target: Dict = field(default_factory=dict)
    draft: Dict = field(default_factory=dict)
    skin: float = 0.3

    @property
    def n_atoms(self) -> int:
        return int(self.positions.shape[0])

    @property
    def n_replicas(self) -> int:
        return int(self.box.shape[0])

    def masses(self) -> np.ndarray:
        return self.species_mass[self.species]

    def replica_slice(self, r: int) -> slice:
        return slice(int(self.atom_offsets[r]), int(self.atom_offsets[r + 1]))


def maxwell_boltzmann(rng: np.random.Generator, masses: np.ndarray, kT: float,
                      force_unit: float = 1.0) -> np.ndarray:
    """Momenta p ~ N(0, m kT) per component (kT converted by force_unit)."""
    sd = np.sqrt(masses * kT * force_unit)
    return f32(rng.standard_normal((masses.shape[0], 3)) * sd[:, None])


def _wrap_f32(x: np.ndarray, L: float) -> np.ndarray:
    x = np.mod(x, L)
    x = f32(x)
    x[x >= L] = 0.0
    return x


def lj_fluid(n_side: int, rho: float = 0.8, kT: float = 1.0, jitter: float = 0.05,
             seed: int = 1, dt: float = 0.005, gamma: float = 1.0, K: int = 8,
             n_steps: int = 2000, rc_target: float = 2.5, rc_draft: float = 1.5,
             skin: float = 0.3, name: Optional[str] = None) -> Workload:
    """n_side^3 LJ atoms at reduced density rho on a jittered simple-cubic
    lattice; box edge L = (N / rho)^(1/3) rounded to binary32."""
    rng = np.random.default_rng(seed)
    n = n_side ** 3
    L = float(f32((n / rho) ** (1.0 / 3.0)))
    a = L / n_side
    idx = np.arange(n)
    # atom index i = x + n_side * (y + n_side * z): lattice order
    lat = np.stack([idx % n_side, (idx // n_side) % n_side, idx // (n_side * n_side)],
                   axis=1).astype(np.float64)
    pos = (lat + 0.5) * a + rng.uniform(-jitter, jitter, size=(n, 3))
    pos = _wrap_f32(pos, L)
    masses = np.ones(n)
    p = maxwell_boltzmann(rng, masses, kT)
    return Workload(
        name=name or f"lj{n}", positions=pos, momenta=p, species=np.zeros(n, np.int32),
        species_mass=np.array([1.0]), atom_offsets=np.array([0, n], np.int32),
        box=np.array([L]), dt=dt, gamma=gamma, kT=kT, force_unit=1.0, K=K,
        n_steps=n_steps, seed=seed,
        target=dict(kind="lj", rc=rc_target, eps=1.0, sig=1.0),
        draft=dict(kind="lj", rc=rc_draft, eps=1.0, sig=1.0), skin=skin)


def lj_replicas(sides, rho: float = 0.8, seed: int = 100, K: int = 8, **kw) -> Workload:
    """Independent Lennard-Jones systems of side^3 atoms each (one box per
    replica, same density), concatenated as one batch of replicas."""
    parts = [lj_fluid(int(n), rho=rho, seed=seed + r, K=K, **kw) for r, n in enumerate(sides)]
    offs = np.cumsum([0] + [w.n_atoms for w in parts]).astype(np.int32)
    w0 = parts[0]
    return Workload(
        name=f"lj_replicas{len(parts)}", positions=np.concatenate([w.positions for w in parts]),
        momenta=np.concatenate([w.momenta for w in parts]),
        species=np.zeros(int(offs[-1]), np.int32), species_mass=np.array([1.0]), atom_offsets=offs,
        box=np.array([w.box[0] for w in parts]), dt=w0.dt, gamma=w0.gamma, kT=w0.kT,
        force_unit=1.0, K=K, n_steps=w0.n_steps, seed=seed, target=dict(w0.target),
        draft=dict(w0.draft), skin=w0.skin)


def tether_replicas(n_replicas: int, k: float = 2.0, m: float = 1.0, dt: float = 0.2,
                    gamma: float = 2.0, kT: float = 1.0, L: float = 1000.0, K: int = 4,
                    seed: int = 7) -> Workload:
    """Independent one-atom systems on harmonic tethers at the box centre,
    starting at rest on their anchors."""
    n = n_replicas
    pos = np.full((n, 3), L / 2)
    return Workload(
        name=f"tether{n}", positions=pos, momenta=np.zeros((n, 3)), species=np.zeros(n, np.int32),
        species_mass=np.array([m]), atom_offsets=np.arange(n + 1, dtype=np.int32),
        box=np.full(n, L), dt=dt, gamma=gamma, kT=kT, force_unit=1.0, K=K, n_steps=100,
        seed=seed, target=dict(kind="harmonic", k=k, anchor=pos.copy()),
        draft=dict(kind="harmonic", k=k, anchor=pos.copy()), skin=0.3)


# --- triatomic liquid (molecular units: Angstrom, amu, fs, eV) -------------
TRIATOMIC_MASSES = np.array([1.008, 12.011, 15.999])   # H-like, C-like, O-like
TRIATOMIC_BONDS = (1.1, 1.2)                            # A-B, B-C in Angstrom
TRIATOMIC_ANGLE_DEG = 120.0


def _molecule_template() -> np.ndarray:
    b1, b2 = TRIATOMIC_BONDS
    th = np.deg2rad(TRIATOMIC_ANGLE_DEG)
    centre = np.zeros(3)
    a = np.array([b1, 0.0, 0.0])
    c = np.array([b2 * np.cos(th), b2 * np.sin(th), 0.0])
    xyz = np.stack([a, centre, c])
    return xyz - xyz.mean(axis=0)


def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def triatomic_box_edge(n_mol: int, density_g_cm3: float = 1.0) -> float:
    mass_amu = n_mol * TRIATOMIC_MASSES.sum()
    grams = mass_amu * 1.66053906660e-24
    vol_a3 = grams / density_g_cm3 * 1e24
    return float(f32(vol_a3 ** (1.0 / 3.0)))


def _triatomic_positions(rng, n_mol, L, jitter=0.1):
    n_side = int(np.ceil(n_mol ** (1.0 / 3.0) - 1e-9))
    a = L / n_side
    sites = np.array([(i, j, k) for k in range(n_side) for j in range(n_side)
                      for i in range(n_side)], dtype=np.float64)
    choose = np.sort(rng.choice(len(sites), size=n_mol, replace=False))
    tmpl = _molecule_template()
    out = []
    for s in sites[choose]:
        centre = (s + 0.5) * a + rng.uniform(-jitter, jitter, size=3)
        out.append(centre + tmpl @ _random_rotation(rng).T)
    return _wrap_f32(np.concatenate(out, axis=0), L)


def triatomic_liquid(n_mol: int = 512, T_kelvin: float = 300.0, seed: int = 3,
                     dt: float = 0.5, gamma: float = 0.01, K: int = 8, n_steps: int = 1000,
                     rc_target: float = 5.0, rc_draft: float = 4.0, skin: float = 0.5,
                     name: Optional[str] = None) -> Workload:
    """n_mol rigid-geometry bent triatomics (species 0, 1, 2 per molecule) at
    about 1 g/cm^3 with Maxwell-Boltzmann momenta at T_kelvin."""
    rng = np.random.default_rng(seed)
    L = triatomic_box_edge(n_mol)
    pos = _triatomic_positions(rng, n_mol, L)
    species = np.tile(np.arange(3, dtype=np.int32), n_mol)
    kT = BOLTZMANN_EV_PER_K * T_kelvin
    p = maxwell_boltzmann(rng, TRIATOMIC_MASSES[species], kT, EV_PER_A_IN_AMU_A_PER_FS2)
    n = pos.shape[0]
    return Workload(
        name=name or f"tri{n_mol}", positions=pos, momenta=p, species=species,
        species_mass=TRIATOMIC_MASSES.copy(), atom_offsets=np.array([0, n], np.int32),
        box=np.array([L]), dt=dt, gamma=gamma, kT=kT, force_unit=EV_PER_A_IN_AMU_A_PER_FS2,
        K=K, n_steps=n_steps, seed=seed, target=dict(kind="mpnn", rc=rc_target),
        draft=dict(kind="pair", rc=rc_draft), skin=skin)


def triatomic_replicas(n_replicas: int = 256, n_mol_lo: int = 8, n_mol_hi: int = 64,
                       seed: int = 4, **kw) -> Workload:
    """Independent triatomic systems with molecule counts drawn uniformly
    from [n_mol_lo, n_mol_hi]; each box is sized for the same density."""
    rng = np.random.default_rng(seed)
    counts = rng.integers(n_mol_lo, n_mol_hi + 1, size=n_replicas)
    pos, sp, mom, boxes, offs = [], [], [], [], [0]
    kT = BOLTZMANN_EV_PER_K * kw.get("T_kelvin", 300.0)
    for c in counts:
        L = triatomic_box_edge(int(c))
        pos.append(_triatomic_positions(rng, int(c), L))
        s = np.tile(np.arange(3, dtype=np.int32), int(c))
        sp.append(s)
        mom.append(maxwell_boltzmann(rng, TRIATOMIC_MASSES[s], kT, EV_PER_A_IN_AMU_A_PER_FS2))
        boxes.append(L)
        offs.append(offs[-1] + 3 * int(c))
    return Workload(
        name=f"tri_replicas{n_replicas}", positions=np.concatenate(pos), momenta=np.concatenate(mom),
        species=np.concatenate(sp), species_mass=TRIATOMIC_MASSES.copy(),
        atom_offsets=np.array(offs, np.int32), box=np.array(boxes), dt=kw.get("dt", 0.5),
        gamma=kw.get("gamma", 0.01), kT=kT, force_unit=EV_PER_A_IN_AMU_A_PER_FS2,
        K=kw.get("K", 8), n_steps=kw.get("n_steps", 5000), seed=seed,
        target=dict(kind="mpnn", rc=5.0), draft=dict(kind="pair", rc=4.0), skin=kw.get("skin", 0.5))


# --- random-init message-passing potential (weights are data) --------------
MPNN_HIDDEN = 128
MPNN_RBF = 16
MPNN_LAYERS = 3
MPNN_READOUT = 64


def mpnn_weight_shapes(n_species: int, H: int = MPNN_HIDDEN, R: int = MPNN_RBF,
                       T: int = MPNN_LAYERS, RH: int = MPNN_READOUT):
    """Names and shapes of the flat weight vector, in storage order.  Matrices
    are stored [out][in]."""
    shapes = [("W_emb", (n_species, H))]
    for t in range(T):
        shapes += [(f"A1_{t}", (H, R)), (f"a1_{t}", (H,)), (f"A2_{t}", (H, H)), (f"a2_{t}", (H,)),
                   (f"B_{t}", (H, H)), (f"C1_{t}", (H, H)), (f"c1_{t}", (H,)),
                   (f"C2_{t}", (H, H)), (f"c2_{t}", (H,))]
    shapes += [("W1", (RH, H)), ("b1", (RH,)), ("w2", (RH,)), ("b2", (1,))]
    return shapes


# Energy scale s_E of the seeded network (weights mpnn_weights(3, seed=17)):
# the RMS force component on the seeded 1536-atom liquid of config("c3") is
# then 1 eV/Angstrom.  Computed once by the FP64 evaluation of the network
# (tests/golden/make_mpnn_scale.py) and fixed before any draft work.
MPNN_WEIGHT_SEED = 17
MPNN_C3_SCALE = 115.52612798524363


def mpnn_target(n_species: int = 3, rc: float = 5.0) -> dict:
    """The message-passing target of the triatomic configurations."""
    return dict(kind="mpnn", rc=rc, weights=mpnn_weights(n_species, seed=MPNN_WEIGHT_SEED),
                n_model_species=n_species, scale=MPNN_C3_SCALE)


def mpnn_weights(n_species: int = 3, seed: int = 17) -> np.ndarray:
    """Seeded random-init weights: U(+-1/sqrt(fan_in)) for every matrix and
    the readout vector, zero biases, N(0, 1) species embeddings; rounded to
    binary32 and returned as one flat float64 vector."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shp in mpnn_weight_shapes(n_species):
        if name == "W_emb":
            v = rng.standard_normal(shp)
        elif name.split("_")[0] in ("a1", "a2", "c1", "c2", "b1", "b2"):
            v = np.zeros(shp)  # biases
        else:
            fan_in = shp[-1] if len(shp) == 2 else shp[0]
            v = rng.uniform(-1.0, 1.0, shp) / np.sqrt(fan_in)
        parts.append(f32(v).ravel())
    return np.concatenate(parts)


def random_box_positions(n: int, L: float, seed: int) -> np.ndarray:
    """Uniform positions in [0, L)^3 (binary32-representable)."""
    rng = np.random.default_rng(seed)
    return _wrap_f32(rng.uniform(0.0, L, size=(n, 3)), L)


# --- the five named configurations ----------------------------------------
def config(name: str) -> Workload:
    """c1: LJ-64, K=8, 2000 steps.  c2: LJ-32768, K=16, 10 000 steps.
    c3: triatomic liquid 1536 atoms, K=8.  c4: 256 triatomic replicas (24-192
    atoms), K=8.  c5: triatomic liquid 24 576 atoms, K=32."""
    if name == "c1":
        return lj_fluid(4, seed=1, K=8, n_steps=2000, name="c1_lj64")
    if name == "c2":
        return lj_fluid(32, seed=2, K=16, n_steps=10000, name="c2_lj32768")
    if name == "c3":
        return triatomic_liquid(512, seed=3, K=8, n_steps=1000, name="c3_tri1536")
    if name == "c4":
        return triatomic_replicas(256, seed=4, K=8, n_steps=5000)
    if name == "c5":
        return triatomic_liquid(8192, seed=5, K=32, n_steps=2000, name="c5_tri24576")
    raise KeyError(name)


CONFIG_NAMES: List[str] = ["c1", "c2", "c3", "c4", "c5"]

# List skins of the benchmark's LSD and plain runs, per configuration (the
# fastest measured on MI355X for each mode; the workload's own skin serves
# the tests and the other configurations).  LSD verifies every frame that
# the skin admits but commits only a few per window (~1.2 on the
# 32768-atom fluid, ~1.3-3 on the triatomic liquids), so a short skin
# pays; a plain window commits every valid frame, so a long one does.
BENCH_SKINS: Dict[str, tuple] = {"c2": (0.125, 0.6), "c3": (0.15, 1.0), "c4": (0.15, 1.0),
                                 "c5": (0.15, 2.0)}
