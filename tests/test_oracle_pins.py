"""Pins of the CPU oracle against facts fixed by the mathematics and the paper.

None of these re-types the oracle's formulas: each checks a property the correct
result must have (closed forms of the 12-6 potential, derivative relations, lattice
sums enumerated independently, library routines, exact time-reversal, analytic
solutions), chosen so that a dropped term, a wrong sign, a wrong factor or a
transposed operand anywhere in the oracle fails at least one of them.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.spatial import cKDTree

import oracle
from workloads import generators as gen

RM = 2.0 ** (1.0 / 6.0)


# ---------------------------------------------------------------- pair function

@pytest.mark.parametrize("sig,eps", [(1.0, 1.0), (0.8, 1.5), (0.88, 0.5)])
def test_lj_closed_forms(oracle_lib, sig, eps):
    rc = 2.5 * sig
    u, f = oracle.pair(RM * sig, sig, eps, 1e9, "trunc")
    assert u == pytest.approx(-eps, rel=1e-14)          # depth of the well
    assert abs(f) < 1e-12 * eps / sig                      # force zero at the minimum
    u, f = oracle.pair(sig, sig, eps, 1e9, "trunc")
    assert abs(u) < 1e-14                                  # U(sigma) = 0
    assert f == pytest.approx(24.0 * eps / sig, rel=1e-14)  # -U'(sigma) = 24 eps / sigma
    # long range: U -> -4 eps (sigma/r)^6 ; short range: U -> 4 eps (sigma/r)^12
    r = 50.0 * sig
    u, _ = oracle.pair(r, sig, eps, 1e9, "trunc")
    assert u == pytest.approx(-4.0 * eps * (sig / r) ** 6, rel=1e-9)
    r = 0.2 * sig
    u, _ = oracle.pair(r, sig, eps, 1e9, "trunc")
    assert u == pytest.approx(4.0 * eps * (sig / r) ** 12, rel=1e-4)
    # scaling: U(r; sig, eps) = eps U(r / sig; 1, 1)
    for r in (0.9, 1.3, 2.2):
        u1, f1 = oracle.pair(r * sig, sig, eps, rc, "sf")
        u0, f0 = oracle.pair(r, 1.0, 1.0, 2.5, "sf")
        assert u1 == pytest.approx(eps * u0, rel=1e-12)
        assert f1 == pytest.approx(eps * f0 / sig, rel=1e-12)


@pytest.mark.parametrize("method", ["trunc", "sp", "sf"])
def test_force_is_minus_derivative_of_pair_energy(oracle_lib, method):
    h = 1e-6
    for r in np.linspace(0.85, 2.45, 17):
        up, _ = oracle.pair(r + h, 1.0, 1.0, 2.5, method)
        um, _ = oracle.pair(r - h, 1.0, 1.0, 2.5, method)
        _, f = oracle.pair(r, 1.0, 1.0, 2.5, method)
        assert -(up - um) / (2 * h) == pytest.approx(f, rel=1e-7, abs=1e-8)


def test_cutoff_methods_at_the_cutoff(oracle_lib):
    rc = 2.5
    ut, ft = oracle.pair(rc, 1.0, 1.0, rc, "trunc")
    us, fs = oracle.pair(rc, 1.0, 1.0, rc, "sp")
    uf, ff = oracle.pair(rc, 1.0, 1.0, rc, "sf")
    assert ut < 0 and ft < 0                  # attractive tail is cut, not shifted
    assert abs(us) < 1e-15 and fs == ft       # SP: energy continuous, force untouched
    assert abs(uf) < 1e-15 and abs(ff) < 1e-15  # SF: energy and force continuous
    # SP shifts the energy by a constant; SF additionally by a linear term in r
    for r in (1.0, 1.7, 2.2):
        u0, f0 = oracle.pair(r, 1.0, 1.0, rc, "trunc")
        u1, f1 = oracle.pair(r, 1.0, 1.0, rc, "sp")
        u2, f2 = oracle.pair(r, 1.0, 1.0, rc, "sf")
        assert u1 - u0 == pytest.approx(-ut, rel=1e-12)
        assert f1 == f0
        assert f2 == pytest.approx(f0 - ft, rel=1e-12)
        assert u2 - u0 == pytest.approx(-ut + (r - rc) * ft, rel=1e-10)


# ---------------------------------------------------------------- whole-system forces

def _small_ka(n=80, seed=3):
    s = gen.ka_random_state(n, 1.2, 0.5, seed)
    sig, eps, rc = gen.ka_params()
    return s, sig, eps, rc


def _min_gap_to_cutoff(pos, box, types, rc):
    d = pos[:, None, :].astype(np.float64) - pos[None, :, :].astype(np.float64)
    d -= box * np.rint(d / box)
    r = np.sqrt((d * d).sum(-1))
    np.fill_diagonal(r, 1e9)
    return np.abs(r - rc[types[:, None], types[None, :]]).min()


@pytest.mark.parametrize("method", ["trunc", "sp", "sf"])
def test_force_is_minus_energy_gradient(oracle_lib, method):
    s, sig, eps, rc = _small_ka()
    pos = s.pos.astype(np.float64)
    assert _min_gap_to_cutoff(pos, s.box, s.types, rc) > 1e-4  # FD never crosses a cutoff
    F, _, _, _, _ = oracle.forces_f64(pos, s.types, s.box, sig, eps, rc, method)
    h = 1e-6
    rng = np.random.default_rng(0)
    for i in rng.choice(s.n, 10, replace=False):
        for c in range(3):
            p1 = pos.copy(); p1[i, c] += h
            p2 = pos.copy(); p2[i, c] -= h
            e1 = oracle.forces_f64(p1, s.types, s.box, sig, eps, rc, method)[3]
            e2 = oracle.forces_f64(p2, s.types, s.box, sig, eps, rc, method)[3]
            assert -(e1 - e2) / (2 * h) == pytest.approx(F[i, c], rel=1e-6, abs=1e-6 * np.abs(F).max())


def test_virial_is_minus_third_of_scaling_derivative(oracle_lib):
    # Under r -> lambda r (box scaled too), dU/dlambda at 1 = sum_pairs r u'(r) = -3 W.
    s, sig, eps, rc = _small_ka()
    pos = s.pos.astype(np.float64)
    _, _, _, U0, W = oracle.forces_f64(pos, s.types, s.box, sig, eps, rc, "sf")
    h = 1e-7
    up = oracle.forces_f64(pos * (1 + h), s.types, s.box * (1 + h), sig, eps, rc, "sf")[3]
    um = oracle.forces_f64(pos * (1 - h), s.types, s.box * (1 - h), sig, eps, rc, "sf")[3]
    assert -(up - um) / (2 * h) / 3.0 == pytest.approx(W, rel=1e-6)


@pytest.mark.parametrize("method", ["sp", "sf"])
def test_newton_third_law(oracle_lib, method):
    s, sig, eps, rc = _small_ka(200, 5)
    F, _, _, _, _ = oracle.forces_f32(s.pos, s.types, s.box, sig, eps, rc, method)
    assert np.abs(F.sum(0)).max() <= 1e-12 * s.n * np.abs(F).max()


def test_f32_and_f64_force_paths_agree_away_from_cutoff(oracle_lib):
    for seed in range(7, 60):  # first seeded state with no pair within 1e-4 of a cutoff
        s, sig, eps, rc = _small_ka(200, seed)
        if _min_gap_to_cutoff(s.pos, s.box, s.types, rc) > 1e-4:
            break
    assert _min_gap_to_cutoff(s.pos, s.box, s.types, rc) > 1e-4
    F1, pe1, w1, U1, W1 = oracle.forces_f32(s.pos, s.types, s.box, sig, eps, rc, "sp")
    F2, pe2, w2, U2, W2 = oracle.forces_f64(s.pos.astype(np.float64), s.types, s.box, sig, eps, rc, "sp")
    np.testing.assert_allclose(F1, F2, rtol=0, atol=1e-12 * np.abs(F2).max())
    assert U1 == pytest.approx(U2, rel=1e-13)
    assert W1 == pytest.approx(W2, rel=1e-13)
    sel = np.array([3, 17, 150], np.int32)
    F3, pe3, w3, _, _ = oracle.forces_f32(s.pos, s.types, s.box, sig, eps, rc, "sp", sel=sel)
    np.testing.assert_array_equal(F3, F1[sel])
    np.testing.assert_array_equal(pe3, pe1[sel])


def _fcc_shells(a, rmax):
    """Distances to all FCC lattice points within rmax of the origin (independent enumeration)."""
    prim = np.array([[0, .5, .5], [.5, 0, .5], [.5, .5, 0]]) * a
    k = int(math.ceil(2 * rmax / a)) + 2
    rng_ = np.arange(-k, k + 1)
    n = np.stack(np.meshgrid(rng_, rng_, rng_, indexing="ij"), -1).reshape(-1, 3)
    v = n @ prim
    r = np.sqrt((v * v).sum(1))
    return r[(r > 0) & (r < rmax)]


@pytest.mark.parametrize("method,pe_survey,w_survey", [
    ("sp", -6.332812, -7.386066), ("sf", -5.693278, -6.721756), ("trunc", -6.773368, None)])
def test_fcc_lattice_sums(oracle_lib, method, pe_survey, w_survey):
    s = gen.config0_state()
    sig, eps, rc = gen.lj_params()
    a = s.box[0] / 6
    shells = _fcc_shells(a, 2.5)
    u_sum = 0.0
    w_sum = 0.0
    for r in shells:
        u, f = oracle.pair(r, 1.0, 1.0, 2.5, method)
        u_sum += u
        w_sum += r * f
    pe_lat = 0.5 * u_sum
    w_lat = w_sum / 6.0
    F, pe, w, U, W = oracle.forces_f32(s.pos, s.types, s.box, sig, eps, rc, method)
    # float32 rounding of the lattice sites perturbs the sums at the 1e-7 level
    assert U / s.n == pytest.approx(pe_lat, rel=2e-6)
    assert W / s.n == pytest.approx(w_lat, rel=2e-6)
    assert np.abs(F).max() < 1e-4                   # zero force by symmetry
    assert np.ptp(pe) < 1e-5                        # every site equivalent
    assert U / s.n == pytest.approx(pe_survey, abs=3e-6)
    if w_survey is not None:
        assert W / s.n == pytest.approx(w_survey, abs=3e-6)
    assert len(shells) == 54


# ---------------------------------------------------------------- pressure and thermo record

def test_pressure_of_an_ideal_gas(oracle_lib):
    # No pair inside the cutoff: the virial vanishes and the pressure is the ideal-gas
    # value N k T_kin / V with the kinetic temperature m <v^2> / (3 k) of equipartition
    # (every particle, no momentum constraint).  Free flight keeps v(n) = v(n +- 1/2).
    rng = np.random.default_rng(12)
    n = 8
    box = np.array([30.0, 24.0, 18.0])
    pos = rng.uniform(-9.0, 9.0, (n, 3)) * np.array([1.0, 0.8, 0.6])
    vel = rng.normal(0.0, 1.3, (n, 3))
    types = np.array([0, 1] * 4, np.int32)
    mass = np.array([1.0, 2.5])
    one = np.ones((2, 2))
    out = oracle.integrate(pos, vel, types, mass, box, one, one, one * 1e-3, "sp", 1e-3, 3)
    m = mass[types][:, None]
    t_kin = (m * vel * vel).sum() / (3 * n)
    p_ideal = n * t_kin / np.prod(box)
    np.testing.assert_allclose(out["thermo"][:, 4], p_ideal, rtol=1e-13)
    np.testing.assert_array_equal(out["thermo"][:, 2], 0.0)
    # the thermodynamic temperature counts 3N - 3 degrees of freedom (momentum fixed)
    np.testing.assert_allclose(out["thermo"][:, 3], t_kin * 3 * n / (3 * n - 3), rtol=1e-13)


@pytest.mark.parametrize("method", ["sp", "sf"])
def test_static_pressure_is_minus_energy_volume_derivative(oracle_lib, method):
    # At rest (T = 0) the pressure is -dU/dV under a uniform dilation of the
    # configuration.  For the perfect config-0 FCC lattice the derivative is taken from
    # independently enumerated lattice sums (U/N as a function of the lattice constant).
    s = gen.config0_state()
    sig, eps, rc = gen.lj_params()
    a = s.box[0] / 6

    def u_per_particle(lat):
        return 0.5 * sum(oracle.pair(r, 1.0, 1.0, 2.5, method)[0] for r in _fcc_shells(lat, 2.5))

    h = 1e-6
    # V/N = a^3 / 4, so dV/da per particle = 3 a^2 / 4
    dudv = (u_per_particle(a * (1 + h)) - u_per_particle(a * (1 - h))) / (2 * h * a) / (0.75 * a * a)
    out = oracle.integrate(s.pos, np.zeros_like(s.pos, dtype=np.float64), s.types, s.mass, s.box, sig, eps,
                           rc, method, 0.005, 1)
    assert out["thermo"][0, 4] == pytest.approx(-dudv, rel=1e-5)
    if method == "sp":
        assert out["thermo"][0, 4] == pytest.approx(-6.235317, abs=5e-6)  # shell-sum value of the survey


def test_pressure_adds_kinetic_and_virial_terms(oracle_lib):
    # Lattice with velocities: P(T) - P(T = 0) is the kinetic part 2 KE / (3V) of the
    # same record (the lattice does not move in the first step's force evaluation).
    s = gen.config0_state()
    sig, eps, rc = gen.lj_params()
    v = gen.maxwell_boltzmann(s.n, 0.722, np.ones(s.n), 6)
    hot = oracle.integrate(s.pos, v, s.types, s.mass, s.box, sig, eps, rc, "sp", 0.005, 1)
    cold = oracle.integrate(s.pos, np.zeros_like(v), s.types, s.mass, s.box, sig, eps, rc, "sp", 0.005, 1)
    ke = hot["thermo"][0, 1]
    assert hot["thermo"][0, 2] == cold["thermo"][0, 2]  # same positions, same virial
    assert hot["thermo"][0, 4] - cold["thermo"][0, 4] == pytest.approx(2 * ke / (3 * np.prod(s.box)), rel=1e-10)
    # the record's KE is that of v(0) = (v(-1/2) + v(1/2)) / 2; on the lattice F = 0, so v(0) = v(-1/2)
    assert ke == pytest.approx(0.5 * (v * v).sum(), rel=1e-9)


def test_conserved_energy_record(oracle_lib):
    # NVE: H is KE + PE of the record; under Nose-Hoover it adds the thermostat's
    # g T0 (tau^2 xi^2 / 2 + integral of xi) and stays constant along the run
    s = gen.lj_fcc_state(108, 0.8442, 1.5, 23)
    sig, eps, rc = gen.lj_params()
    pos, vel = s.pos.astype(np.float64), s.vel.astype(np.float64)
    nve = oracle.integrate(pos, vel, s.types, s.mass, s.box, sig, eps, rc, "sf", 0.002, 5)["thermo"]
    np.testing.assert_array_equal(nve[:, 7], nve[:, 1] + nve[:, 0])
    nvt = oracle.integrate(pos, vel, s.types, s.mass, s.box, sig, eps, rc, "sf", 0.002, 600, thermostat=True,
                           T0=0.5, tau=0.1)["thermo"]
    e = nvt[:, 0] + nvt[:, 1]
    assert np.ptp(e) > 0.2 * s.n                              # the thermostat removes energy
    assert np.ptp(nvt[:, 7]) < 1e-3 * np.ptp(e)               # but H stays put


# ---------------------------------------------------------------- pair sets

def test_fcc_pair_counts(oracle_lib):
    s = gen.config0_state()
    _, _, rc = gen.lj_params()
    cs2, rc2 = oracle.cut_tables(rc, 0.3)
    P = oracle.pair_set(s.pos, s.types, s.box, cs2)
    assert len(P) == 78 * s.n
    assert np.all(np.bincount(P[:, 0], minlength=s.n) == 78)
    cs2, _ = oracle.cut_tables(rc, 0.0)
    P0 = oracle.pair_set(s.pos, s.types, s.box, cs2)
    assert len(P0) == 54 * s.n


def test_pair_set_sorted_symmetric_and_matches_kdtree(oracle_lib):
    s = gen.jitter_positions(gen.config1_state(), 0.05, 11)
    sig, eps, rc = gen.ka_params()
    skin = 0.3
    cs2, _ = oracle.cut_tables(rc, skin)
    P = oracle.pair_set(s.pos, s.types, s.box, cs2)
    key = P[:, 0].astype(np.int64) * s.n + P[:, 1]
    assert np.all(np.diff(key) > 0)                               # sorted, no duplicates
    assert np.all(P[:, 0] != P[:, 1])
    rev = np.sort(P[:, 1].astype(np.int64) * s.n + P[:, 0])
    np.testing.assert_array_equal(rev, key)                       # both directions present
    # compare with scipy's periodic kd-tree in FP64: agreement except within 1e-5 of the radius
    pos = s.pos.astype(np.float64) + s.box / 2
    pos = np.mod(pos, s.box)
    tree = cKDTree(pos, boxsize=s.box)
    rmax = float(np.max(rc)) + skin
    pairs = tree.query_pairs(rmax + 1e-4, output_type="ndarray")
    d = pos[pairs[:, 0]] - pos[pairs[:, 1]]
    d -= s.box * np.rint(d / s.box)
    r = np.sqrt((d * d).sum(1))
    lim = rc[s.types[pairs[:, 0]], s.types[pairs[:, 1]]] + skin
    both = np.concatenate([pairs, pairs[:, ::-1]])
    rb = np.concatenate([r, r])
    lb = np.concatenate([lim, lim])
    inside = both[rb < lb - 1e-5]
    maybe = both[np.abs(rb - lb) <= 1e-5]
    kin = inside[:, 0].astype(np.int64) * s.n + inside[:, 1]
    kmaybe = maybe[:, 0].astype(np.int64) * s.n + maybe[:, 1]
    assert np.isin(kin, key).all()
    extra = np.setdiff1d(key, kin)
    assert np.isin(extra, kmaybe).all()


def test_pair_set_periodic_and_strict(oracle_lib):
    box = np.array([10.0, 10.0, 10.0])
    types = np.zeros(2, np.int32)
    rc = np.array([[2.5]])
    cs2, _ = oracle.cut_tables(rc, 0.5)                 # (2.5 + 0.5)^2 = 9 exactly
    assert cs2[0, 0] == 9.0
    pos = np.array([[-4.9, 0, 0], [4.9, 0, 0]], np.float32)  # 0.2 apart through the boundary
    P = oracle.pair_set(pos, types, box, cs2)
    assert P.tolist() == [[0, 1], [1, 0]]
    pos = np.array([[0, 0, 0], [3.0, 0, 0]], np.float32)     # exactly on the radius: excluded
    assert len(oracle.pair_set(pos, types, box, cs2)) == 0
    pos[1, 0] = np.nextafter(np.float32(3.0), np.float32(0))  # one ulp inside: included
    assert len(oracle.pair_set(pos, types, box, cs2)) == 2
    pos = np.array([[0, 0, 0], [0, 0, -3.0]], np.float32)    # same along z
    assert len(oracle.pair_set(pos, types, box, cs2)) == 0
    nb = oracle.neighbors_of(np.array([[0, 0, 0], [0, 2.0, 0], [0, 0, 1.0]], np.float32),
                             np.zeros(3, np.int32), box, cs2, 0)
    assert nb.tolist() == [1, 2]


def test_pair_set_uses_type_pair_radius(oracle_lib):
    box = np.array([10.0, 10.0, 10.0])
    sig, eps, rc = gen.ka_params()
    cs2, _ = oracle.cut_tables(rc, 0.3)
    # A-B radius 2.0 + 0.3, B-B radius 2.2 + 0.3, A-A 2.5 + 0.3
    pos = np.array([[0, 0, 0], [2.4, 0, 0]], np.float32)
    for ta, tb, expect in [(0, 0, 2), (0, 1, 0), (1, 0, 0), (1, 1, 2)]:
        P = oracle.pair_set(pos, np.array([ta, tb], np.int32), box, cs2)
        assert len(P) == expect, (ta, tb)


# ---------------------------------------------------------------- displacement criterion

def test_rebuild_criterion_half_skin_boundary(oracle_lib):
    box = np.array([8.0, 8.0, 8.0])
    pos0 = np.zeros((4, 3), np.float32)
    pos0[:, 0] = [-3.0, -1.0, 1.0, 3.9375]
    skin = 0.25                        # s/2 = 0.125 exactly representable
    pos = pos0.copy()
    pos[1, 1] += np.float32(0.125)
    assert oracle.max_disp2(pos, pos0, box) == 0.015625
    assert not oracle.rebuild_needed(pos, pos0, box, skin)     # "more than" half the skin
    pos[1, 1] = np.nextafter(pos[1, 1], np.float32(1))
    assert oracle.rebuild_needed(pos, pos0, box, skin)
    # moving through the periodic boundary counts the short way round
    pos = pos0.copy()
    pos[3, 0] = np.float32(-3.9375)    # 3.9375 -> -3.9375 is a displacement of 0.125
    assert oracle.max_disp2(pos, pos0, box) == pytest.approx(0.015625, abs=0)
    assert not oracle.rebuild_needed(pos, pos0, box, skin)


# ---------------------------------------------------------------- integrator

def test_free_flight_and_wrap(oracle_lib):
    box = np.array([5.0, 5.0, 5.0])
    pos = np.array([[2.4, 0.0, 0.0], [-2.0, 1.0, 0.5]])
    vel = np.array([[1.0, 0.0, 0.0], [0.0, -3.0, 0.25]])
    types = np.zeros(2, np.int32)
    sig, eps, rc = np.array([[1.0]]), np.array([[1.0]]), np.array([[0.01]])  # no pair in range
    out = oracle.integrate(pos, vel, types, np.array([1.0]), box, sig, eps, rc, "sp", 0.01, 100)
    exp = pos + vel * 1.0
    img = np.floor((exp + box / 2) / box).astype(int)
    np.testing.assert_allclose(out["pos"], exp - img * box, atol=1e-12)
    np.testing.assert_array_equal(out["image"], img)
    np.testing.assert_array_equal(out["vel"], vel)


def test_dimer_small_oscillation_period(oracle_lib):
    # Two unit masses at the LJ minimum: omega^2 = U''(r_m) / mu with U''(r_m) = 72 eps / r_m^2, mu = 1/2
    box = np.array([20.0, 20.0, 20.0])
    amp = 1e-3
    pos = np.array([[-(RM + amp) / 2, 0, 0], [(RM + amp) / 2, 0, 0]])
    vel = np.zeros((2, 3))
    types = np.zeros(2, np.int32)
    dt = 1e-3
    out = oracle.integrate(pos, vel, types, np.array([1.0]), box, np.array([[1.0]]), np.array([[1.0]]),
                           np.array([[2.5]]), "trunc", dt, 2000)
    pe = out["thermo"][:, 0]
    # PE oscillates at twice the bond frequency; find its period from minima (bond at r_m)
    k = np.where((pe[1:-1] < pe[:-2]) & (pe[1:-1] <= pe[2:]))[0] + 1
    period = 2 * np.mean(np.diff(k)) * dt
    omega = math.sqrt(72.0 / RM ** 2 / 0.5)
    assert period == pytest.approx(2 * math.pi / omega, rel=5e-3)
    # momentum stays zero, bond stays along x
    assert np.abs(out["vel"].sum(0)).max() < 1e-12


def test_leapfrog_time_reversal(oracle_lib):
    s, sig, eps, rc = _small_ka(64, 9)
    pos = s.pos.astype(np.float64)
    vel = s.vel.astype(np.float64)
    K = 40
    fw = oracle.integrate(pos, vel, s.types, s.mass, s.box, sig, eps, rc, "sf", 0.002, K)
    fw1 = oracle.integrate(pos, vel, s.types, s.mass, s.box, sig, eps, rc, "sf", 0.002, K + 1)
    back = oracle.integrate(fw["pos"], -fw1["vel"], s.types, s.mass, s.box, sig, eps, rc, "sf", 0.002, K,
                            image=fw["image"])
    d = back["pos"] - pos
    d -= s.box * np.rint(d / s.box)
    assert np.abs(d).max() < 1e-9
    np.testing.assert_array_equal(back["image"], 0)


def test_nve_energy_conservation_and_lattice_at_rest(oracle_lib):
    m = 3
    L = (4 * m ** 3 / 0.8442) ** (1 / 3)
    sites = gen.fcc_lattice(m, L / m)
    box = np.array([L, L, L])
    types = np.zeros(len(sites), np.int32)
    sig, eps, rc = np.array([[1.0]]), np.array([[1.0]]), np.array([[2.5]])
    rest = oracle.integrate(sites, np.zeros_like(sites), types, np.array([1.0]), box, sig, eps, rc, "sp",
                            0.005, 20)
    assert np.abs(rest["pos"] - sites).max() < 1e-12                     # perfect lattice at T = 0
    v = gen.maxwell_boltzmann(len(sites), 0.722, np.ones(len(sites)), 3)
    out = oracle.integrate(sites, v, types, np.array([1.0]), box, sig, eps, rc, "sf", 0.002, 400)
    E = out["thermo"][:, 0] + out["thermo"][:, 1]
    assert np.ptp(E) / len(sites) < 2e-4
    # halving dt cuts the energy fluctuation about fourfold (second-order scheme)
    out2 = oracle.integrate(sites, v, types, np.array([1.0]), box, sig, eps, rc, "sf", 0.004, 200)
    E2 = out2["thermo"][:, 0] + out2["thermo"][:, 1]
    assert 2.5 < np.std(E2[20:]) / np.std(E[40:]) < 6.0


def test_nose_hoover_free_particles_matches_ode(oracle_lib):
    # With no interactions, K and xi obey dK/dt = -2 xi K, dxi/dt = (2K/(g T0) - 1)/tau^2.
    rng = np.random.default_rng(4)
    n = 50
    box = np.array([30.0, 30.0, 30.0])
    pos = rng.uniform(-15, 15, (n, 3))
    vel = gen.maxwell_boltzmann(n, 2.0, np.ones(n), 5)
    types = np.zeros(n, np.int32)
    g = 3 * n - 3
    T0, tau, dt, steps = 1.0, 0.5, 1e-3, 1000
    out = oracle.integrate(pos, vel, types, np.array([1.0]), box, np.array([[1.0]]), np.array([[1.0]]),
                           np.array([[1e-3]]), "sp", dt, steps, thermostat=True, T0=T0, tau=tau)
    K0 = 0.5 * (vel * vel).sum()

    def rhs(t, y):
        K, xi = y
        return [-2 * xi * K, (2 * K / (g * T0) - 1) / tau ** 2]
    sol = solve_ivp(rhs, (0, steps * dt), [K0, 0.0], rtol=1e-11, atol=1e-12, dense_output=True)
    # integer-step xi of the scheme vs the ODE at the same times
    t = np.arange(steps) * dt
    xi_ode = sol.sol(t)[1]
    assert np.abs(out["thermo"][:, 5] - xi_ode).max() < 2e-3 * np.abs(xi_ode).max()
    # conserved extended energy (no potential energy here)
    H = out["thermo"][:, 7]
    assert np.ptp(H) < 1e-4 * abs(H[0])


def test_nose_hoover_infinite_tau_is_nve_bitwise(oracle_lib):
    s, sig, eps, rc = _small_ka(64, 2)
    pos = s.pos.astype(np.float64)
    vel = s.vel.astype(np.float64)
    a = oracle.integrate(pos, vel, s.types, s.mass, s.box, sig, eps, rc, "sf", 0.003, 30)
    b = oracle.integrate(pos, vel, s.types, s.mass, s.box, sig, eps, rc, "sf", 0.003, 30, thermostat=True,
                         T0=0.5, tau=np.inf)
    np.testing.assert_array_equal(a["pos"], b["pos"])
    np.testing.assert_array_equal(a["vel"], b["vel"])


def test_nose_hoover_reaches_target_temperature(oracle_lib):
    s = gen.lj_fcc_state(108, 0.8442, 1.5, 21)
    sig, eps, rc = gen.lj_params()
    out = oracle.integrate(s.pos.astype(np.float64), s.vel.astype(np.float64), s.types, s.mass, s.box, sig,
                           eps, rc, "sp", 0.005, 3000, thermostat=True, T0=0.8, tau=0.2)
    T = out["thermo"][1000:, 3]
    assert np.mean(T) == pytest.approx(0.8, rel=0.05)
    H = out["thermo"][:, 7]
    assert np.ptp(H[200:]) / s.n < 5e-3


# ---------------------------------------------------------------- initial states

def test_initial_states(oracle_lib):
    s = gen.config1_state()
    v = gen.maxwell_boltzmann(s.n, 0.45, np.ones(s.n), 99)
    assert np.abs(v.sum(0)).max() < 1e-12
    assert 2 * oracle.kinetic(v, s.types, s.mass) / (3 * s.n - 3) == pytest.approx(0.45, rel=1e-13)
    assert np.bincount(s.types).tolist() == [3277, 819]
    pos = np.mod(s.pos.astype(np.float64) + s.box / 2, s.box)
    tree = cKDTree(pos, boxsize=s.box)
    pairs = tree.query_pairs(0.75, output_type="ndarray")
    d = pos[pairs[:, 0]] - pos[pairs[:, 1]]
    d -= s.box * np.rint(d / s.box)
    r = np.sqrt((d * d).sum(1))
    dmin = 0.75 * gen.KA_SIGMA[s.types[pairs[:, 0]], s.types[pairs[:, 1]]]
    assert np.all(r >= dmin * (1 - 1e-6))
    assert np.all(np.abs(s.pos) <= s.box[0] / 2)
    c0 = gen.config0_state()
    assert c0.n == 864 and c0.box[0] == pytest.approx(10.0776, abs=1e-4)


def _paper_values():
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")) as f:
        return json.load(f)


def test_pair_count_matches_paper_molten_salt_neighbour_count(oracle_lib):
    """Section 9 prints ~330 neighbours per particle at density 0.3677 within 6.0 sigma.
    The oracle's list (r^2 < (r_c + s)^2, skin 0) on a uniform random configuration at
    that density must count about that many; a dropped square, a wrong minimum image or
    a wrong radius would miss it by far more than the 3 % allowed for the paper's
    rounding (the ideal-gas mean is 4/3 pi 6^3 0.3677 = 332.7)."""
    v = _paper_values()["molten_salt_neighbours"]
    n = 2000
    L = (n / v["density"]) ** (1.0 / 3.0)
    rng = np.random.default_rng(9)
    pos = rng.uniform(-L / 2, L / 2, size=(n, 3)).astype(np.float32)
    types = np.zeros(n, np.int32)
    cs2, _ = oracle.cut_tables(np.array([[v["cutoff"]]]), 0.0)
    pairs = oracle.pair_set(pos, types, np.array([L, L, L]), cs2)
    per_particle = len(pairs) / n
    assert abs(per_particle - v["neighbours_per_particle"]) <= 0.03 * v["neighbours_per_particle"], per_particle

