"""Pins of the oracle's shifted-force Coulomb term (paper section 9), each chosen so
that a plausible mistake fails it: a dropped shift (the term must vanish with its
force at the cutoff), a sign error in the linear term (the energy must be the
integral of the force), a wrong power or sign of the plain part (Coulomb's law in
the limit of a large cutoff), a charge taken from the wrong particle (Newton's
third law with unequal charges), a wrong virial factor (the virial is minus a third
of the derivative of the energy under uniform scaling), and a wrong combination
with the Lennard-Jones term (the two add)."""
import numpy as np
import pytest
from scipy.integrate import quad

import oracle

pytestmark = pytest.mark.filterwarnings("ignore")


@pytest.fixture(scope="module", autouse=True)
def _lib():
    oracle.load()


@pytest.mark.parametrize("qq", [1.0, -1.0, 2.0, -0.5])
def test_vanishes_with_its_force_at_the_cutoff(qq):
    rcc = 6.0
    u, f = oracle.coulomb_sf(rcc * (1 - 1e-9), qq, rcc)
    assert abs(u) < 1e-12 and abs(f) < 1e-9
    u, f = oracle.coulomb_sf(1.0, qq, rcc)
    assert abs(u) > 0.5 * abs(qq) and abs(f) > 0.9 * abs(qq)


@pytest.mark.parametrize("r", [0.8, 1.3, 2.9, 5.5])
def test_energy_is_the_integral_of_the_force_from_the_cutoff(r):
    rcc, qq = 6.0, -1.0
    integral, err = quad(lambda s: oracle.coulomb_sf(s, qq, rcc)[1], r, rcc, epsabs=1e-13, epsrel=1e-13)
    u, _ = oracle.coulomb_sf(r, qq, rcc)
    assert abs(u - integral) <= 1e-10 * max(1.0, abs(u))


@pytest.mark.parametrize("qq", [1.0, -1.0, 3.0])
def test_coulombs_law_for_a_large_cutoff(qq):
    for r in (0.7, 1.0, 2.5):
        u, f = oracle.coulomb_sf(r, qq, 1e7)
        assert abs(f - qq / r ** 2) <= 1e-9 * abs(qq / r ** 2)
        assert abs(u - qq / r) <= 1e-6 * abs(qq / r)


def _two_ion_forces(q0, q1, r, rcc=6.0):
    box = np.array([20.0, 20.0, 20.0])
    pos = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]], np.float32)
    types = np.array([0, 1], np.int32)
    zero = np.zeros((2, 2))
    F, pe, w, U, W = oracle.forces_f32(pos, types, box, np.ones((2, 2)), zero, np.full((2, 2), 1.0), "sf",
                                       charges=[q0, q1], rc_coul=rcc)
    return F, U


def test_unlike_charges_attract_and_like_charges_repel():
    F, U = _two_ion_forces(1.0, -1.0, 1.5)
    assert F[0, 0] > 0 and F[1, 0] < 0 and U < 0  # the ion at the origin is pulled towards +x
    F, U = _two_ion_forces(1.0, 1.0, 1.5)
    assert F[0, 0] < 0 and F[1, 0] > 0 and U > 0
    assert np.abs(F[:, 1:]).max() == 0.0


def _salt(n, L, charges, seed, dmin=0.9):
    rng = np.random.default_rng(seed)
    pos = []
    while len(pos) < n:
        p = rng.uniform(-L / 2, L / 2, 3)
        if pos:
            d = np.array(pos) - p
            d -= L * np.rint(d / L)
            if (d * d).sum(1).min() < dmin * dmin:
                continue
        pos.append(p)
    pos = np.array(pos)
    nt = len(charges)
    types = np.arange(n, dtype=np.int32) % nt
    return pos, types


def test_newtons_third_law_with_unequal_charges():
    """Charges +2 and -1 (types 0 and 1, one to two): a charge product taken from one
    particle only, or a per-type table read with swapped indices, breaks sum F = 0."""
    q = [2.0, -1.0, -1.0]
    L = 10.0
    pos, types = _salt(150, L, q, 3)
    box = np.array([L, L, L])
    sig = np.full((3, 3), 1.0)
    eps = np.full((3, 3), 0.5)
    rc = np.full((3, 3), 2.5)
    F, pe, w, U, W = oracle.forces_f64(pos, types, box, sig, eps, rc, "sf", charges=q, rc_coul=4.5)
    assert np.abs(F.sum(0)).max() <= 1e-11 * np.abs(F).max()
    # and the float32-decision form agrees with it on these positions (no pair at a cutoff)
    F32, _, _, U32, W32 = oracle.forces_f32(pos.astype(np.float32), types, box, sig, eps, rc, "sf", charges=q,
                                            rc_coul=4.5)
    F64b, _, _, U64b, W64b = oracle.forces_f64(pos.astype(np.float32).astype(np.float64), types, box, sig, eps, rc,
                                               "sf", charges=q, rc_coul=4.5)
    assert np.abs(F32 - F64b).max() <= 1e-12 * np.abs(F64b).max()
    assert abs(U32 - U64b) <= 1e-12 * abs(U64b)


def test_virial_is_the_scaling_derivative_of_the_energy():
    """W = (1/3) sum r f = -(1/3) dU(lambda)/dlambda at lambda = 1 when every position
    and the box are scaled by lambda (cutoffs fixed)."""
    q = [1.0, -1.0]
    L = 9.0
    pos, types = _salt(120, L, q, 5)
    box = np.array([L, L, L])
    sig, eps, rc = np.ones((2, 2)), np.full((2, 2), 0.7), np.full((2, 2), 2.5)
    _, _, _, U0, W = oracle.forces_f64(pos, types, box, sig, eps, rc, "sf", charges=q, rc_coul=4.0)
    h = 1e-6
    Up = oracle.forces_f64(pos * (1 + h), types, box * (1 + h), sig, eps, rc, "sf", charges=q, rc_coul=4.0)[3]
    Um = oracle.forces_f64(pos * (1 - h), types, box * (1 - h), sig, eps, rc, "sf", charges=q, rc_coul=4.0)[3]
    dU = (Up - Um) / (2 * h)
    assert abs(W - (-dU / 3.0)) <= 1e-6 * max(abs(W), 1.0)


def test_lennard_jones_and_coulomb_terms_add():
    q = [1.0, -1.0]
    L = 9.0
    pos, types = _salt(120, L, q, 8)
    box = np.array([L, L, L])
    sig, eps, rc = np.ones((2, 2)), np.full((2, 2), 0.7), np.full((2, 2), 2.5)
    F, _, _, U, W = oracle.forces_f32(pos, types, box, sig, eps, rc, "sf", charges=q, rc_coul=4.0)
    Fl, _, _, Ul, Wl = oracle.forces_f32(pos, types, box, sig, eps, rc, "sf")
    Fc, _, _, Uc, Wc = oracle.forces_f32(pos, types, box, sig, np.zeros((2, 2)), rc, "sf", charges=q, rc_coul=4.0)
    assert np.abs(F - (Fl + Fc)).max() <= 1e-12 * np.abs(F).max()
    assert abs(U - (Ul + Uc)) <= 1e-12 * abs(U) and abs(W - (Wl + Wc)) <= 1e-12 * abs(W)
    # charges scaled by 2: the Coulomb part scales by 4
    Fc2, _, _, Uc2, _ = oracle.forces_f32(pos, types, box, sig, np.zeros((2, 2)), rc, "sf", charges=[2.0, -2.0],
                                          rc_coul=4.0)
    assert abs(Uc2 - 4 * Uc) <= 1e-12 * abs(Uc2)


def test_integrator_conserves_energy_with_coulomb():
    """Leapfrog NVE of a small melt with the Coulomb term: the energy drift over 400
    steps stays at the level of the time step error (a force inconsistent with the
    energy would drift linearly)."""
    q = [1.0, -1.0]
    L = 9.0
    pos, types = _salt(100, L, q, 12, dmin=1.0)
    rng = np.random.default_rng(1)
    vel = rng.standard_normal(pos.shape) * np.sqrt(0.5)
    vel -= vel.mean(0)
    box = np.array([L, L, L])
    sig, eps, rc = np.ones((2, 2)), np.ones((2, 2)), np.full((2, 2), 2.5)
    out = oracle.integrate(pos, vel, types, np.ones(2), box, sig, eps, rc, "sf", 0.002, 400, charges=q, rc_coul=4.0)
    h = out["thermo"][:, 7]
    assert np.abs(h - h[0]).max() <= 2e-4 * len(pos)
