"""Seeded initial-state generators.

Every state is a plain container of NumPy arrays:

* ``pos``   float32 (N, 3), inside the periodic box [-L/2, L/2) per axis;
* ``vel``   float32 (N, 3), read as the half-step velocity v(-dt/2);
* ``types`` int32 (N,);
* ``box``   float64 (3,), each side exactly representable in float32
  (the GPU keeps the box in float32, so the oracle is handed the same value);
* ``mass``  float64 (ntypes,).

Workload shapes follow the benchmark systems of the paper's benchmark section
(melting FCC Lennard-Jones crystal, NVE) and the Kob-Andersen 80:20 binary
mixture; the exact recipes (density, temperature, composition rounding,
placement rule) are listed with each generator.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Kob-Andersen 80:20 parameters (type 0 = A, type 1 = B).
KA_SIGMA = np.array([[1.0, 0.8], [0.8, 0.88]])
KA_EPSILON = np.array([[1.0, 1.5], [1.5, 0.5]])


@dataclasses.dataclass
class State:
    pos: np.ndarray
    vel: np.ndarray
    types: np.ndarray
    box: np.ndarray
    mass: np.ndarray
    ntypes: int
    seed: int
    recipe: str

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    def copy(self) -> "State":
        return dataclasses.replace(self, pos=self.pos.copy(), vel=self.vel.copy(),
                                   types=self.types.copy(), box=self.box.copy(),
                                   mass=self.mass.copy())


def _f32_side(length: float) -> float:
    """Box side rounded once to float32 (the value both sides then use)."""
    return float(np.float32(length))


def _wrap_f32(pos: np.ndarray, box: np.ndarray) -> np.ndarray:
    """Map float positions into [-L/2, L/2) per axis, in float32."""
    p = pos.astype(np.float64)
    p = p - box * np.floor(p / box + 0.5)
    p32 = p.astype(np.float32)
    half = (box / 2).astype(np.float32)
    box32 = box.astype(np.float32)
    # float32 rounding can land exactly on +L/2; move those to -L/2.
    for k in range(3):
        col = p32[:, k]
        col[col >= half[k]] -= box32[k]
        col[col < -half[k]] += box32[k]
    return p32


def fcc_lattice(m: int, a: float) -> np.ndarray:
    """4*m^3 sites of an FCC lattice with cubic cell side ``a``, centred on the origin.

    The cube of side L = m*a spans [-L/2, L/2); the basis is (0,0,0), (0,1/2,1/2),
    (1/2,0,1/2), (1/2,1/2,0) in units of a, offset by a/4 so no site sits on a face.
    """
    basis = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]], dtype=np.float64)
    idx = np.arange(m)
    cells = np.stack(np.meshgrid(idx, idx, idx, indexing="ij"), axis=-1).reshape(-1, 3)
    sites = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3)
    L = m * a
    return (sites + 0.25) * a - L / 2


def maxwell_boltzmann(n: int, T: float, mass_per_particle: np.ndarray, seed: int) -> np.ndarray:
    """Gaussian velocities with variance T/m, zero total momentum, 2KE/(3N-3) = T exactly (FP64).

    Returned in float64; callers round to float32 when building a State.
    """
    rng = np.random.default_rng(seed)
    m = np.asarray(mass_per_particle, dtype=np.float64)
    v = rng.standard_normal((n, 3)) * np.sqrt(T / m)[:, None]
    p_mean = (m[:, None] * v).sum(axis=0) / m.sum()
    v -= p_mean
    ke = 0.5 * float((m[:, None] * v * v).sum())
    g = 3 * n - 3
    if ke > 0 and T > 0:
        v *= math.sqrt(T * g / (2.0 * ke))
    elif T == 0:
        v[:] = 0.0
    return v


def jitter_positions(state: State, amplitude: float, seed: int) -> State:
    """Displace every particle uniformly in a cube of half-width ``amplitude`` (then wrap)."""
    rng = np.random.default_rng(seed)
    s = state.copy()
    d = rng.uniform(-amplitude, amplitude, size=s.pos.shape)
    s.pos = _wrap_f32(s.pos.astype(np.float64) + d, s.box)
    s.recipe += f"+jitter({amplitude},{seed})"
    return s


def lj_params(rc: float = 2.5):
    """Single-component LJ: sigma = epsilon = 1, absolute cutoff rc."""
    return (np.array([[1.0]]), np.array([[1.0]]), np.array([[rc]]))


def ka_params(rc_factor: float = 2.5):
    """Kob-Andersen: cutoff rc_factor * sigma_ab per type pair."""
    return (KA_SIGMA.copy(), KA_EPSILON.copy(), rc_factor * KA_SIGMA)


def lj_fcc_state(n: int, rho: float, T: float, seed: int) -> State:
    """Single-component LJ state on an FCC lattice.

    m = ceil((N/4)^(1/3)) cubic cells on a side of L = (N/rho)^(1/3); if 4m^3 > N a
    seeded random subset of N sites is kept (vacancies).  Velocities from
    ``maxwell_boltzmann`` at T with the same seed.
    """
    m = int(math.ceil((n / 4.0) ** (1.0 / 3.0) - 1e-9))
    L = _f32_side((n / rho) ** (1.0 / 3.0))
    box = np.array([L, L, L])
    sites = fcc_lattice(m, L / m)
    rng = np.random.default_rng(seed)
    if sites.shape[0] > n:
        keep = np.sort(rng.choice(sites.shape[0], size=n, replace=False))
        sites = sites[keep]
    pos = _wrap_f32(sites, box)
    mass = np.array([1.0])
    vel = maxwell_boltzmann(n, T, np.ones(n), seed + 7919).astype(np.float32)
    return State(pos=pos, vel=vel, types=np.zeros(n, dtype=np.int32), box=box, mass=mass,
                 ntypes=1, seed=seed, recipe=f"lj_fcc(N={n},rho={rho},T={T},seed={seed})")


def _random_insertion(n, L, types, dmin, rng, batch=256):
    """Random sequential insertion in a periodic cube of side L.

    Candidates are drawn uniformly; candidate k is accepted when it is at least
    dmin[t_k, t_j] from every particle j placed before it, where t_k = types[number
    placed so far].  Candidates are drawn and tested against the particles already
    placed in vectorised batches (through a cell grid), and then accepted one by one
    in draw order, so the result is that of the one-at-a-time rule.
    """
    dmin2 = dmin * dmin
    dmax = float(dmin.max())
    nc = max(3, int(L // dmax))
    cl = L / nc
    cap = 24
    grid = -np.ones((nc, nc, nc, cap), dtype=np.int64)
    cnt = np.zeros((nc, nc, nc), dtype=np.int64)
    offs = np.array([(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)])
    pos = np.empty((n, 3))
    placed = 0
    draws = 0
    while placed < n:
        B = batch
        cand = rng.uniform(-L / 2, L / 2, size=(B, 3))
        draws += B
        if draws > 400 * n + 10000:
            raise RuntimeError("random insertion did not converge")
        cc = np.floor((cand + L / 2) / cl).astype(np.int64) % nc
        nb = (cc[:, None, :] + offs[None, :, :]) % nc
        idx = grid[nb[..., 0], nb[..., 1], nb[..., 2]].reshape(B, -1)
        valid = idx >= 0
        j = np.where(valid, idx, 0)
        d = pos[j] - cand[:, None, :]
        d -= L * np.round(d / L)
        r2 = (d * d).sum(-1)
        tj = types[j]
        bad_placed = [(valid & (r2 < dmin2[t][tj])).any(1).tolist() for t in (0, 1)]
        # earlier candidates of this batch that could conflict with candidate k
        dd = cand[:, None, :] - cand[None, :, :]
        dd -= L * np.round(dd / L)
        rr = (dd * dd).sum(-1)
        ks, ms = np.nonzero(np.tril(rr < dmax * dmax, -1))
        earlier = {}
        for k, m in zip(ks.tolist(), ms.tolist()):
            earlier.setdefault(k, []).append(m)
        acc_type = {}
        for k in range(B):
            if placed >= n:
                break
            t = int(types[placed])
            if bad_placed[t][k]:
                continue
            if k in earlier and any(m in acc_type and rr[k, m] < dmin2[t, acc_type[m]] for m in earlier[k]):
                continue
            acc_type[k] = t
            pos[placed] = cand[k]
            c0, c1, c2 = cc[k]
            if cnt[c0, c1, c2] >= cap:
                raise RuntimeError("insertion grid cell overflow")
            grid[c0, c1, c2, cnt[c0, c1, c2]] = placed
            cnt[c0, c1, c2] += 1
            placed += 1
    return pos


def ka_random_state(n: int, rho: float, T: float, seed: int, min_dist_factor: float = 0.75) -> State:
    """Kob-Andersen 80:20 mixture by random sequential insertion.

    N_A = round(0.8 N), N_B = N - N_A, types assigned by a seeded permutation.
    Particles are inserted at uniform random points, a candidate being rejected if it
    is closer than ``min_dist_factor`` * sigma_ab to any particle already placed.
    Velocities from ``maxwell_boltzmann`` at T.
    """
    rng = np.random.default_rng(seed)
    n_a = int(round(0.8 * n))
    types = np.zeros(n, dtype=np.int32)
    types[n_a:] = 1
    types = types[rng.permutation(n)]
    L = _f32_side((n / rho) ** (1.0 / 3.0))
    box = np.array([L, L, L])
    pos = _random_insertion(n, L, types, min_dist_factor * KA_SIGMA, rng)
    mass = np.array([1.0, 1.0])
    vel = maxwell_boltzmann(n, T, np.ones(n), seed + 7919).astype(np.float32)
    return State(pos=_wrap_f32(pos, box), vel=vel, types=types, box=box, mass=mass, ntypes=2,
                 seed=seed, recipe=f"ka_random(N={n},rho={rho},T={T},seed={seed},dmin={min_dist_factor})")


def _ka_replica(args):
    n, rho, T, seed = args
    return ka_random_state(n, rho, T, seed)


def ka_replica_states(count: int = 256, master_seed: int = 2026, n_lo: int = 500, n_hi: int = 8000, rho=1.2,
                      workers: int = 1):
    """The batched-replica workload: KA systems with N_r ~ U{n_lo..n_hi}, T_r ~ U[0.4, 1.0],
    replica r seeded 1000 + r.  ``workers`` > 1 generates replicas in worker processes
    (the result does not depend on it)."""
    jobs = [(n, rho, T, seed) for (n, T, seed) in config3_states(count, master_seed, n_lo, n_hi)]
    if workers <= 1:
        return [_ka_replica(j) for j in jobs]
    from concurrent.futures import ProcessPoolExecutor

    with ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(_ka_replica, jobs, chunksize=4))


# ---- the benchmark configurations ------------------------------------------------------

LJ_RHO = 0.8442
LJ_T = 0.722
KA_RHO = 1.2


def config0_state(seed: int = 0) -> State:
    """LJ, N = 864 (6x6x6 FCC cells), rho 0.8442, T 0.722; SP cutoff 2.5, skin 0.3."""
    return lj_fcc_state(864, LJ_RHO, LJ_T, seed)


def config1_state(seed: int = 1) -> State:
    """KA 80:20, N = 4096, rho 1.2, T 0.45; SF cutoff 2.5 sigma_ab, skin 0.3."""
    return ka_random_state(4096, KA_RHO, 0.45, seed)


def config2_state(n: int) -> State:
    """LJ fluid start for the size sweep, N in {1000, 4000, 16000, 64000, 256000, 1024000}; seed = N."""
    return lj_fcc_state(n, LJ_RHO, LJ_T, n)


def config3_states(count: int = 256, master_seed: int = 2026, n_lo: int = 500, n_hi: int = 8000):
    """Replica set: N_r ~ U{n_lo..n_hi}, T_r ~ U[0.4, 1.0]; replica r uses seed 1000 + r."""
    rng = np.random.default_rng(master_seed)
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    ts = rng.uniform(0.4, 1.0, size=count)
    return [(int(ns[r]), float(ts[r]), 1000 + r) for r in range(count)]


def config4_state() -> State:
    """LJ fluid, N = 32768, config 0 parameters, seed 4."""
    return lj_fcc_state(32768, LJ_RHO, LJ_T, 4)


# ---- the molten salt of the Coulomb benchmark (paper section 9) ------------------------

SALT_RHO = 0.3677
SALT_T = 2.0
SALT_RC_COUL = 6.0


def salt_params(rc_lj: float = 2.5):
    """Molten salt: identical Lennard-Jones parameters (sigma = epsilon = 1, cutoff rc_lj)
    for both species; charges +1 and -1 (reduced units); Coulomb cutoff 6.0.
    Returns (sigma, epsilon, rc, charges, rc_coulomb)."""
    one = np.ones((2, 2))
    return one.copy(), one.copy(), rc_lj * one, np.array([1.0, -1.0]), SALT_RC_COUL


def molten_salt_state(n: int, seed: int, rho: float = SALT_RHO, T: float = SALT_T, min_dist: float = 0.8) -> State:
    """Half cations (type 0), half anions (type 1), assigned by a seeded permutation
    (n even: neutral), placed by random sequential insertion at least ``min_dist``
    apart, unit masses, Maxwell-Boltzmann velocities at T."""
    if n % 2:
        raise ValueError("the salt needs an even particle count")
    rng = np.random.default_rng(seed)
    types = np.zeros(n, dtype=np.int32)
    types[n // 2:] = 1
    types = types[rng.permutation(n)]
    L = _f32_side((n / rho) ** (1.0 / 3.0))
    box = np.array([L, L, L])
    pos = _random_insertion(n, L, types, np.full((2, 2), min_dist), rng)
    vel = maxwell_boltzmann(n, T, np.ones(n), seed + 7919).astype(np.float32)
    return State(pos=_wrap_f32(pos, box), vel=vel, types=types, box=box, mass=np.array([1.0, 1.0]), ntypes=2,
                 seed=seed, recipe=f"molten_salt(N={n},rho={rho},T={T},seed={seed},dmin={min_dist})")
