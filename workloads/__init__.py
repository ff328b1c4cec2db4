"""Seeded synthetic particle configurations for the neighbor-search workloads.

These generators stand in for the molecular-dynamics snapshots the paper
benchmarks (Section 4: Lennard-Jones fluid at fixed density in a cubic periodic
box; the size-asymmetric colloid/solvent mixtures of the authors' earlier BVH
work; liquid/vapor inhomogeneity as in the spinodal benchmark).  No snapshot
data is available, so every configuration is drawn from a seeded NumPy
generator with the same box shape, density and particle count.

This module holds inputs only: no neighbor-search arithmetic lives here, and it
imports neither the HIP library nor the oracle.  Every generator returns
positions as C-contiguous float32 ``[N, 3]`` arrays inside the half-open box
``[0, L_d)`` on each axis, together with the box as float32 ``[3]``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Config",
    "wrap_f32",
    "lj_lattice",
    "uniform",
    "sc_lattice",
    "lj_fluid",
    "colloid_solvent",
    "ensemble",
    "slab",
    "SEEDS",
]

# Seeds fixed per workload so every consumer sees the same particles.
SEEDS = {
    "lj4000": 19010881,
    "lj1m": 19010882,
    "lj8m": 19010883,
    "colloid": 19010884,
    "ensemble": 19010885,
    "served": 19010886,
    "wca": 19010887,
    "spinodal": 19010888,
}


@dataclass
class Config:
    """One particle configuration plus the cutoff table it is searched with."""

    pos: np.ndarray  # float32 [N, 3] (float64 for fp64 data, see as_f64)
    box: np.ndarray  # float32 [3] (float64 for fp64 data)
    rcut: np.ndarray  # float32 [ntypes, ntypes]
    skin: float
    types: np.ndarray | None = None  # int32 [N] or None for one type
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    @property
    def ntypes(self) -> int:
        return int(self.rcut.shape[0])


def wrap_f32(x64: np.ndarray, box32: np.ndarray) -> np.ndarray:
    """Wrap fp64 coordinates into [0, L) and round them to fp32.

    The wrap is done in fp64 against the exact fp32 box edge; a value that
    rounds up to L after conversion is mapped onto 0 so the result lies in the
    half-open box.
    """
    L = box32.astype(np.float64)
    w = np.mod(x64, L)
    w = np.where(w < 0.0, w + L, w)
    out = w.astype(np.float32)
    out = np.where(out >= box32, np.float32(0.0), out)
    out = np.where(out < 0, np.float32(0.0), out)
    return np.ascontiguousarray(out, dtype=np.float32)


def _lattice_n(n_particles: int) -> int:
    n = int(round(n_particles ** (1.0 / 3.0)))
    while n ** 3 < n_particles:
        n += 1
    while n > 1 and (n - 1) ** 3 >= n_particles:
        n -= 1
    return n


def lj_lattice(n_particles: int, rho: float, seed, jitter: float = 0.3,
               box: np.ndarray | None = None) -> tuple[np.ndarray, np.ndarray]:
    """Jittered simple-cubic lattice at number density ``rho`` in a cubic box.

    L = (N / rho)^(1/3); the lattice has n = ceil(N^(1/3)) sites per axis with
    spacing a = L / n, N sites are picked by a seeded permutation (so particle
    order is random, as in an unsorted snapshot) and each coordinate gets a
    uniform displacement in [-jitter, +jitter].
    """
    rng = np.random.default_rng(seed)
    if box is None:
        L = (n_particles / rho) ** (1.0 / 3.0)
        box32 = np.full(3, L, dtype=np.float32)
    else:
        box32 = np.asarray(box, dtype=np.float32)
    n = _lattice_n(n_particles)
    a = box32.astype(np.float64) / n
    sites = rng.permutation(n ** 3)[:n_particles]
    iz, rem = np.divmod(sites, n * n)
    iy, ix = np.divmod(rem, n)
    m = np.stack([ix, iy, iz], axis=1).astype(np.float64)
    x = (m + 0.5) * a + rng.uniform(-jitter, jitter, size=(n_particles, 3))
    return wrap_f32(x, box32), box32


def uniform(n_particles: int, box, seed) -> tuple[np.ndarray, np.ndarray]:
    """Independent uniform (ideal-gas) positions in an orthorhombic box."""
    rng = np.random.default_rng(seed)
    box32 = np.asarray(box, dtype=np.float32).reshape(3)
    x = rng.uniform(0.0, 1.0, size=(n_particles, 3)) * box32.astype(np.float64)
    return wrap_f32(x, box32), box32


def sc_lattice(n: int, a: float = 1.0) -> tuple[np.ndarray, np.ndarray]:
    """Perfect simple-cubic lattice with n sites per axis, spacing a, at m*a."""
    g = np.arange(n, dtype=np.float64) * a
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    box32 = np.full(3, n * a, dtype=np.float32)
    return wrap_f32(pos, box32), box32


def lj_fluid(n_particles: int, seed=None, rho: float = 0.85, rc: float = 3.0,
             skin: float = 0.4) -> Config:
    """Single-type Lennard-Jones-fluid stand-in (jittered lattice), rc and skin in sigma."""
    if seed is None:
        seed = {4000: SEEDS["lj4000"], 1_000_000: SEEDS["lj1m"],
                8_000_000: SEEDS["lj8m"]}.get(n_particles, SEEDS["lj4000"])
    pos, box = lj_lattice(n_particles, rho, seed)
    return Config(pos=pos, box=box, rcut=np.array([[rc]], dtype=np.float32), skin=skin,
                  name=f"lj_fluid_N{n_particles}_rho{rho}",
                  meta={"rho": rho, "seed": seed})


class _CellGrid:
    """Points binned into cells of edge >= ``cell`` in a periodic box (sorted by cell)."""

    def __init__(self, pts, box64, cell):
        self.box = box64
        self.nc = np.maximum((box64 // cell).astype(np.int64), 1)
        self.width = box64 / self.nc
        self.pts = pts
        c = self.cells(pts)
        self.order = np.argsort(c, kind="stable")
        self.starts = np.searchsorted(c[self.order], np.arange(int(self.nc.prod()) + 1))

    def cells(self, x):
        c = np.minimum((x // self.width).astype(np.int64), self.nc - 1)
        return (c[:, 0] * self.nc[1] + c[:, 1]) * self.nc[2] + c[:, 2]

    def clashes(self, trial, dmin, trial_index=None):
        """True where a trial point lies closer than dmin to a grid point.

        With ``trial_index`` (the grid holds the trials themselves), only grid
        points with a smaller index count.
        """
        bad = np.zeros(trial.shape[0], dtype=bool)
        if self.pts.shape[0] == 0 or trial.shape[0] == 0:
            return bad
        c = np.minimum((trial // self.width).astype(np.int64), self.nc - 1)
        for off in _OFFSETS:
            cc = np.mod(c + off, self.nc)
            lin = (cc[:, 0] * self.nc[1] + cc[:, 1]) * self.nc[2] + cc[:, 2]
            lo, hi = self.starts[lin], self.starts[lin + 1]
            cnt = hi - lo
            for slot in range(int(cnt.max()) if cnt.size else 0):
                has = np.nonzero(cnt > slot)[0]
                j = self.order[lo[has] + slot]
                d = self.pts[j] - trial[has]
                d -= self.box * np.round(d / self.box)
                close = np.einsum("ij,ij->i", d, d) < dmin * dmin
                if trial_index is not None:
                    close &= j < trial_index[has]
                bad[has[close]] = True
        return bad


_OFFSETS = np.array([[i, j, k] for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)])


def _rsa_insert(rng, box64, n_target, existing, self_min, batch=131072, max_rounds=20000):
    """Random sequential addition: uniform trial points, each kept unless it comes
    closer than ``self_min`` to a kept point of this species, or closer than the
    given distance to a point of an ``existing`` species ((points, min distance)).

    Trials are drawn in seeded batches; inside a batch a trial is also dropped
    when it clashes with an earlier trial of the same batch, so the outcome is
    a deterministic function of the seed.
    """
    placed = np.empty((0, 3), dtype=np.float64)
    grids = [(_CellGrid(p, box64, d), d) for p, d in existing]
    rounds = 0
    while placed.shape[0] < n_target:
        rounds += 1
        if rounds > max_rounds:
            raise RuntimeError("random sequential addition did not converge")
        m = int(min(batch, max(1024, 8 * (n_target - placed.shape[0]))))
        trial = rng.uniform(0.0, 1.0, size=(m, 3)) * box64
        ok = np.ones(m, dtype=bool)
        for g, d in grids:
            ok &= ~g.clashes(trial, d)
        if placed.shape[0]:
            ok &= ~_CellGrid(placed, box64, self_min).clashes(trial, self_min)
        idx = np.nonzero(ok)[0]
        cand = trial[idx]
        own = _CellGrid(cand, box64, self_min)
        keep = ~own.clashes(cand, self_min, trial_index=np.arange(cand.shape[0]))
        placed = np.concatenate([placed, cand[keep][: n_target - placed.shape[0]]], axis=0)
    return placed


def colloid_solvent(n_total: int = 1_000_000, seed=SEEDS["colloid"], frac_colloid: float = 0.02,
                    d_colloid: float = 5.0, rho_solvent_accessible: float = 0.5,
                    skin: float = 0.4) -> Config:
    """Binary colloid/solvent mixture placed by random sequential addition.

    Type 0 = solvent (diameter 1), type 1 = colloid (diameter ``d_colloid``).
    The solvent density is read as the number density in the volume that
    solvent centers can reach (box minus the colloid exclusion shells of radius
    (1 + d_colloid) / 2): any reading against the total box volume would need a
    colloid volume fraction above the random-sequential-addition jamming limit.
    Cutoffs are rc_ij = (sigma_i + sigma_j) / 2 and the list radius adds ``skin``.
    """
    rng = np.random.default_rng(seed)
    n_c = int(round(frac_colloid * n_total))
    n_s = n_total - n_c
    r_excl = 0.5 * (1.0 + d_colloid)
    v_excl = n_c * (4.0 / 3.0) * math.pi * r_excl ** 3
    volume = n_s / rho_solvent_accessible + v_excl
    L = volume ** (1.0 / 3.0)
    box32 = np.full(3, L, dtype=np.float32)
    box64 = box32.astype(np.float64)
    col = _rsa_insert(rng, box64, n_c, [], d_colloid)
    sol = _rsa_insert(rng, box64, n_s, [(col, r_excl)], 1.0)
    pos64 = np.concatenate([sol, col], axis=0)
    types = np.concatenate([np.zeros(n_s, np.int32), np.ones(n_c, np.int32)])
    perm = rng.permutation(n_total)
    pos = wrap_f32(pos64[perm], box32)
    types = types[perm]
    sig = np.array([1.0, d_colloid])
    rcut = (0.5 * (sig[:, None] + sig[None, :])).astype(np.float32)
    return Config(pos=pos, box=box32, rcut=rcut, skin=skin, types=np.ascontiguousarray(types),
                  name=f"colloid_solvent_N{n_total}",
                  meta={"seed": seed, "n_colloid": n_c, "n_solvent": n_s, "L": float(L),
                        "colloid_volume_fraction": n_c * (math.pi / 6) * d_colloid ** 3 / volume})


def ensemble(n_systems: int = 256, seed=SEEDS["ensemble"], n_min: int = 2000, n_max: int = 200_000,
             rho_lo: float = 0.3, rho_hi: float = 0.9, rc_lo: float = 2.5, rc_hi: float = 3.0,
             skin: float = 0.4, scale: float = 1.0) -> list[Config]:
    """Independent Lennard-Jones replicas with log-uniform N and uniform density and cutoff.

    ``scale`` shrinks every N (for CPU-sized tests) without changing the draws.
    """
    children = np.random.SeedSequence(seed).spawn(n_systems)
    out = []
    for k, ss in enumerate(children):
        rng = np.random.default_rng(ss)
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        rho = float(rng.uniform(rho_lo, rho_hi))
        rc = float(rng.uniform(rc_lo, rc_hi))
        n = max(2, int(round(n * scale)))
        pos_seed = int(rng.integers(0, 2 ** 63 - 1))
        pos, box = lj_lattice(n, rho, pos_seed)
        out.append(Config(pos=pos, box=box, rcut=np.array([[rc]], dtype=np.float32), skin=skin,
                          name=f"replica{k}_N{n}", meta={"rho": rho, "rc": rc, "index": k}))
    return out


def as_f64(cfg: Config, seed, scale: float = 1e-3) -> Config:
    """fp64 particle data from a configuration: every coordinate moved by a
    seeded uniform offset of up to ``scale`` sigma in fp64 and wrapped into
    [0, L) in fp64 (so almost no coordinate is an fp32 value); the box is the
    same, held as fp64."""
    rng = np.random.default_rng(seed)
    box64 = np.asarray(cfg.box, dtype=np.float32).astype(np.float64)
    x = cfg.pos.astype(np.float64) + rng.uniform(-scale, scale, size=cfg.pos.shape)
    x = np.mod(x, box64)
    x = np.where(x >= box64, 0.0, x)  # mod can return L for tiny negative inputs
    return Config(pos=np.ascontiguousarray(x), box=box64, rcut=cfg.rcut, skin=cfg.skin, types=cfg.types,
                  name=cfg.name + "_f64", meta=dict(cfg.meta, f64_seed=seed))


def near_cutoff_pairs_f64(n_base: int, n_pairs: int, box: float, r_list: float, seed,
                          rel: tuple[float, float] = (1e-13, 1e-8)) -> Config:
    """fp64 stress case for the exact decision: ``n_base`` uniform points and,
    for ``n_pairs`` of them, a partner at distance r_list (1 +- e) in a random
    direction with e log-uniform in ``rel`` (fp32 cannot resolve these)."""
    rng = np.random.default_rng(seed)
    L = float(box)
    base = rng.uniform(0.0, L, size=(n_base, 3))
    who = rng.choice(n_base, size=n_pairs, replace=False)
    u = rng.normal(size=(n_pairs, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    e = np.exp(rng.uniform(np.log(rel[0]), np.log(rel[1]), size=n_pairs)) * rng.choice([-1.0, 1.0], size=n_pairs)
    partner = base[who] + u * (r_list * (1.0 + e))[:, None]
    x = np.mod(np.concatenate([base, partner]), L)
    x = np.where(x >= L, 0.0, x)
    x = x[rng.permutation(x.shape[0])]
    return Config(pos=np.ascontiguousarray(x), box=np.full(3, L), rcut=np.array([[np.float32(r_list)]], np.float32),
                  skin=0.0, name=f"near_cutoff_f64_N{x.shape[0]}", meta={"seed": seed})


def compact_type_f64(n_bulk: int = 3000, n_compact: int = 40, n_pairs: int = 400, box: float = 100.0,
                     spread: float = 0.1, rc01: float = 2.5, seed=19010890,
                     rel: tuple[float, float] = (1e-9, 1e-6)) -> Config:
    """fp64 two-type case with a compact second type: ``n_bulk`` uniform type-0
    points in a cubic box of edge ``box`` and ``n_compact`` type-1 points within
    ``spread`` sigma of a centre near the far corner (large coordinates round
    to fp32 by the most).  For ``n_pairs`` type-1 points a type-0 partner sits
    at rc01 (1 +- e) in a random direction, e log-uniform in ``rel``.
    rcut = [[1.0, rc01], [rc01, 0.5]], skin 0."""
    rng = np.random.default_rng(seed)
    L = float(box)
    bulk = rng.uniform(0.0, L, size=(n_bulk, 3))
    centre = np.array([0.97, 0.96, 0.98]) * L
    comp = centre + rng.uniform(-spread / 2, spread / 2, size=(n_compact, 3))
    who = rng.integers(0, n_compact, size=n_pairs)
    u = rng.normal(size=(n_pairs, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    e = np.exp(rng.uniform(np.log(rel[0]), np.log(rel[1]), size=n_pairs)) * rng.choice([-1.0, 1.0], size=n_pairs)
    r = float(np.float32(rc01))
    partner = comp[who] + u * (r * (1.0 + e))[:, None]
    x = np.concatenate([bulk, partner, comp])
    t = np.concatenate([np.zeros(n_bulk + n_pairs, np.int32), np.ones(n_compact, np.int32)])
    x = np.mod(x, L)
    x = np.where(x >= L, 0.0, x)
    order = rng.permutation(x.shape[0])
    rcut = np.array([[1.0, rc01], [rc01, 0.5]], np.float32)
    return Config(pos=np.ascontiguousarray(x[order]), box=np.full(3, L), rcut=rcut, skin=0.0,
                  types=np.ascontiguousarray(t[order]), name=f"compact_type_f64_N{x.shape[0]}",
                  meta={"seed": seed})


WCA_RC = 2.0 ** (1.0 / 6.0)


def wca_fluid(n_particles: int, seed=SEEDS["wca"], rho: float = 0.85, skin: float = 0.4) -> Config:
    """Purely repulsive (WCA) fluid stand-in: the LJ lattice generator with the
    short cutoff rc = 2^(1/6) sigma, so each particle has only ~12 list
    neighbors (the low-occupancy case the paper names as hard for grids)."""
    pos, box = lj_lattice(n_particles, rho, seed)
    return Config(pos=pos, box=box, rcut=np.array([[WCA_RC]], dtype=np.float32), skin=skin,
                  name=f"wca_fluid_N{n_particles}_rho{rho}", meta={"rho": rho, "seed": seed})


def _bicontinuous_field(rng, box64: np.ndarray, n_modes: int, wavelength: float):
    """A smooth random field on the periodic box: a sum of plane waves whose
    wavevectors are lattice vectors of the box with length near 2 pi / wavelength."""
    m_max = np.maximum(1, np.round(box64 / wavelength * 1.5)).astype(int)
    cand = np.stack(np.meshgrid(*[np.arange(-m, m + 1) for m in m_max], indexing="ij"), -1).reshape(-1, 3)
    k = 2.0 * np.pi * cand / box64
    kn = np.linalg.norm(k, axis=1)
    k0 = 2.0 * np.pi / wavelength
    pool = np.nonzero(np.abs(kn - k0) <= 0.35 * k0)[0]
    pick = rng.choice(pool, size=min(n_modes, pool.size), replace=False)
    kv, phase = k[pick], rng.uniform(0.0, 2.0 * np.pi, size=pick.size)

    def field(x):
        return np.cos(x @ kv.T + phase).sum(axis=1)
    return field


def spinodal(n_target: int = 1_000_000, seed=SEEDS["spinodal"], rho_liquid: float = 0.75,
             rho_vapor: float = 0.05, wavelength: float = 30.0, rc: float = 3.0, skin: float = 0.4) -> Config:
    """Spinodal-like liquid-vapor configuration: a bicontinuous structure in
    which half of the box (where a smooth random field of domain size
    ``wavelength`` is positive) holds liquid at ``rho_liquid`` (jittered cubic
    lattice, kept where the field is positive) and the other half holds vapor
    at ``rho_vapor`` (uniform points, kept where it is negative).  This is the
    strong density variation the paper's spinodal benchmarks show; the box is
    cubic with L chosen so that about ``n_target`` particles result."""
    rng = np.random.default_rng(seed)
    L = (n_target / (0.5 * (rho_liquid + rho_vapor))) ** (1.0 / 3.0)
    box32 = np.full(3, L, dtype=np.float32)
    box64 = box32.astype(np.float64)
    field = _bicontinuous_field(rng, box64, 24, wavelength)
    n = int(np.ceil((rho_liquid * box64.prod()) ** (1.0 / 3.0)))
    a = box64 / n
    g = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"), -1).reshape(-1, 3)
    liq = (g + 0.5) * a + rng.uniform(-0.3, 0.3, size=g.shape) * a
    liq = liq[field(liq) > 0.0]
    n_vap = int(round(rho_vapor * box64.prod()))
    vap = rng.uniform(0.0, 1.0, size=(4 * n_vap + 64, 3)) * box64
    vap = vap[field(vap) <= 0.0][: n_vap // 2]
    pos64 = np.concatenate([liq, vap], axis=0)
    pos64 = pos64[rng.permutation(pos64.shape[0])]
    return Config(pos=wrap_f32(pos64, box32), box=box32, rcut=np.array([[rc]], dtype=np.float32), skin=skin,
                  name=f"spinodal_N{pos64.shape[0]}",
                  meta={"seed": seed, "n_liquid": int(liq.shape[0]), "n_vapor": int(vap.shape[0]),
                        "L": float(L), "wavelength": wavelength})


def slab(n_target_liquid_thickness: float = 80.0, seed=SEEDS["served"], box=(60.0, 60.0, 240.0),
         rho_liquid: float = 0.8, rho_vapor: float = 0.02, min_vapor_gap: float = 0.8,
         rc: float = 3.0, skin: float = 0.4) -> Config:
    """Liquid slab (jittered lattice at ``rho_liquid``) in a dilute uniform vapor.

    The liquid fills |z - Lz/2| < t/2; vapor points are uniform elsewhere and
    are rejected closer than ``min_vapor_gap`` to any liquid particle.
    """
    rng = np.random.default_rng(seed)
    box32 = np.asarray(box, dtype=np.float32)
    box64 = box32.astype(np.float64)
    t = float(n_target_liquid_thickness)
    a = rho_liquid ** (-1.0 / 3.0)
    nx, ny = int(round(box64[0] / a)), int(round(box64[1] / a))
    nz = max(1, int(round(t / a)))
    ax, ay, az = box64[0] / nx, box64[1] / ny, t / nz
    g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"),
                 axis=-1).reshape(-1, 3).astype(np.float64)
    liq = (g + 0.5) * np.array([ax, ay, az])
    liq[:, 2] += box64[2] / 2 - t / 2
    liq += rng.uniform(-0.3, 0.3, size=liq.shape) * np.array([ax, ay, az]) / a
    v_vap = box64[0] * box64[1] * (box64[2] - t)
    n_vap = int(round(rho_vapor * v_vap))
    vap = np.empty((0, 3))
    while vap.shape[0] < n_vap:
        trial = rng.uniform(0.0, 1.0, size=(2 * n_vap + 16, 3)) * box64
        dz = np.abs(trial[:, 2] - box64[2] / 2)
        trial = trial[dz >= t / 2 + min_vapor_gap]
        vap = np.concatenate([vap, trial[: n_vap - vap.shape[0]]], axis=0)
    pos64 = np.concatenate([liq, vap], axis=0)
    pos64 = pos64[rng.permutation(pos64.shape[0])]
    pos = wrap_f32(pos64, box32)
    return Config(pos=pos, box=box32, rcut=np.array([[rc]], dtype=np.float32), skin=skin,
                  name=f"slab_t{t:g}_N{pos.shape[0]}",
                  meta={"seed": seed, "n_liquid": liq.shape[0], "n_vapor": n_vap})


def served_sims(n_sims: int = 64, n_slabs: int = 16, seed=SEEDS["served"], n_min: int = 10_000,
                n_max: int = 2_000_000, scale: float = 1.0) -> list[Config]:
    """The simulations behind the served stream: ``n_slabs`` liquid-vapor slabs
    (box 60 x 60 x 240, liquid thickness chosen so N is log-uniform in
    [n_min, n_max] within what the box allows) and Lennard-Jones fluids
    (density 0.85, N log-uniform in [n_min, n_max]); rc 3.0 + skin 0.4.

    ``scale`` shrinks every N (and the slab box edges by its cube root) for
    test-sized streams without changing the draws.
    """
    children = np.random.SeedSequence(seed).spawn(n_sims)
    out = []
    for k, ss in enumerate(children):
        rng = np.random.default_rng(ss)
        n = float(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))) * scale
        sub = int(rng.integers(0, 2 ** 63 - 1))
        if k < n_slabs:
            f = scale ** (1.0 / 3.0)
            box = (60.0 * f, 60.0 * f, 240.0 * f)
            area = box[0] * box[1]
            # N = area (0.8 t + 0.02 (Lz - t))  =>  t
            t = (n / area - 0.02 * box[2]) / 0.78
            t = float(min(max(t, 4.0), box[2] - 2.0))
            c = slab(t, seed=sub, box=box)
            c.name = f"sim{k}_{c.name}"
        else:
            # at least 400 particles, so the box edge exceeds twice the list radius
            n_i = max(400, int(round(n)))
            c = lj_fluid(n_i, seed=sub)
            c.name = f"sim{k}_lj_N{n_i}"
        c.meta = dict(c.meta, sim=k)
        out.append(c)
    return out

