"""Pins of the oracle's further pair potentials (paper section 2 names Yukawa,
Buckingham, Gaussian core, Dzugutov and Girifalco potentials among its pair
potentials; the forms are the textbook ones).  None re-types the oracle's
formulas: each pin is a derivative relation, a special case that reduces to a
known function, a limit or an asymptote, or a scaling law."""
import math

import numpy as np
import pytest

import oracle
from workloads import generators as gen

KINDS = {
    "yukawa": ([1.3, 2.0, 0.0, 0.0], 0.9, 3.0),
    "buckingham": ([600.0, 0.25, 1.7, 0.0], 1.0, 3.0),
    "gaussian": ([2.0, 0.0, 0.0, 0.0], 1.0, 2.6),
    "dzugutov": ([1.0, 0.0, 0.0, 0.0], 1.0, 1.94),
    "girifalco": ([0.7, 0.05, 0.0, 0.0], 1.0, 2.5),
}


@pytest.mark.parametrize("kind", list(KINDS))
@pytest.mark.parametrize("method", ["trunc", "sp", "sf"])
def test_force_is_minus_derivative(oracle_lib, kind, method):
    p, sig, rc = KINDS[kind]
    h = 1e-6
    lo = 1.3 if kind == "girifalco" else 0.75
    for r in np.linspace(lo * sig, rc - 0.05, 19):
        up, _ = oracle.pair_potential(kind, r + h, p, sig, rc, method)
        um, _ = oracle.pair_potential(kind, r - h, p, sig, rc, method)
        _, f = oracle.pair_potential(kind, r, p, sig, rc, method)
        assert -(up - um) / (2 * h) == pytest.approx(f, rel=1e-6, abs=1e-8)


@pytest.mark.parametrize("kind", list(KINDS))
def test_cutoff_methods(oracle_lib, kind):
    p, sig, rc = KINDS[kind]
    ut, ft = oracle.pair_potential(kind, rc, p, sig, rc, "trunc")
    us, fs = oracle.pair_potential(kind, rc, p, sig, rc, "sp")
    uf, ff = oracle.pair_potential(kind, rc, p, sig, rc, "sf")
    assert abs(us) < 1e-14 and fs == ft
    assert abs(uf) < 1e-14 and abs(ff) < 1e-14
    for r in (0.8 * rc, 0.9 * rc):
        u0, f0 = oracle.pair_potential(kind, r, p, sig, rc, "trunc")
        u2, f2 = oracle.pair_potential(kind, r, p, sig, rc, "sf")
        assert u2 - u0 == pytest.approx(-ut + (r - rc) * ft, rel=1e-9, abs=1e-13)
        assert f2 == pytest.approx(f0 - ft, rel=1e-12, abs=1e-14)


def test_yukawa_special_cases(oracle_lib):
    # U(sigma) = eps; kappa = 0 is a bare Coulomb eps sigma / r; screening multiplies by
    # exp(-kappa (r - sigma))
    for r in (0.7, 1.0, 2.2):
        u, f = oracle.pair_potential("yukawa", r, [1.5, 0.0, 0, 0], 0.8, 1e9, "trunc")
        assert u == pytest.approx(1.5 * 0.8 / r, rel=1e-14) and f == pytest.approx(1.5 * 0.8 / r ** 2, rel=1e-14)
        u2, _ = oracle.pair_potential("yukawa", r, [1.5, 2.0, 0, 0], 0.8, 1e9, "trunc")
        assert u2 / u == pytest.approx(math.exp(-2.0 * (r - 0.8)), rel=1e-13)
    u, _ = oracle.pair_potential("yukawa", 0.8, [1.5, 3.0, 0, 0], 0.8, 1e9, "trunc")
    assert u == pytest.approx(1.5, rel=1e-14)


def test_buckingham_special_cases(oracle_lib):
    # C = 0: a pure exponential with decay length rho; A = 0: the -C / r^6 dispersion tail
    u, f = oracle.pair_potential("buckingham", 0.3, [5.0, 0.3, 0.0, 0], 1.0, 1e9, "trunc")
    assert u == pytest.approx(5.0 / math.e, rel=1e-14) and f == pytest.approx(5.0 / math.e / 0.3, rel=1e-14)
    u, f = oracle.pair_potential("buckingham", 2.0, [0.0, 0.3, 3.0, 0], 1.0, 1e9, "trunc")
    assert u == pytest.approx(-3.0 / 64, rel=1e-14) and f == pytest.approx(-18.0 / 128, rel=1e-14)


def test_gaussian_core_special_cases(oracle_lib):
    u0, f0 = oracle.pair_potential("gaussian", 1e-9, [2.0, 0, 0, 0], 1.3, 1e9, "trunc")
    assert u0 == pytest.approx(2.0, rel=1e-12) and abs(f0) < 1e-8       # soft core: finite at r = 0
    u, _ = oracle.pair_potential("gaussian", 1.3, [2.0, 0, 0, 0], 1.3, 1e9, "trunc")
    assert u == pytest.approx(2.0 / math.e, rel=1e-14)
    # the force peaks at r = sigma / sqrt(2)
    rs = np.linspace(0.5, 1.3, 801)
    fs = [oracle.pair_potential("gaussian", r, [2.0, 0, 0, 0], 1.3, 1e9, "trunc")[1] for r in rs]
    assert rs[int(np.argmax(fs))] == pytest.approx(1.3 / math.sqrt(2), abs=1e-3)


def test_dzugutov_structure(oracle_lib):
    # both terms and all their derivatives vanish at their ends (x = 1.87 and 1.94): the
    # potential is smooth and zero from 1.94 sigma on, without any cutoff shift
    for sig in (1.0, 1.2):
        for x in (1.94, 1.95, 2.5):
            u, f = oracle.pair_potential("dzugutov", x * sig, [1.0, 0, 0, 0], sig, 1e9, "trunc")
            assert u == 0.0 and f == 0.0
        u, f = oracle.pair_potential("dzugutov", (1.94 - 1e-3) * sig, [1.0, 0, 0, 0], sig, 1e9, "trunc")
        assert abs(u) < 1e-100 and abs(f) < 1e-100
        # just below 1.87 only the second term is left, to within exp(-1100)
        x = 1.87 - 1e-3
        u, _ = oracle.pair_potential("dzugutov", x * sig, [1.0, 0, 0, 0], sig, 1e9, "trunc")
        assert u == pytest.approx(1.28 * math.exp(0.27 / (x - 1.94)), rel=1e-12)
    # eps and sigma scale energy and length
    u1, f1 = oracle.pair_potential("dzugutov", 1.3, [2.5, 0, 0, 0], 1.2, 1e9, "trunc")
    u0, f0 = oracle.pair_potential("dzugutov", 1.3 / 1.2, [1.0, 0, 0, 0], 1.0, 1e9, "trunc")
    assert u1 == pytest.approx(2.5 * u0, rel=1e-13) and f1 == pytest.approx(2.5 * f0 / 1.2, rel=1e-13)
    # a repulsive core and one attractive well inside 1.87 sigma
    rs = np.linspace(0.9, 1.93, 2000)
    us = np.array([oracle.pair_potential("dzugutov", r, [1.0, 0, 0, 0], 1.0, 1e9, "trunc")[0] for r in rs])
    assert us[0] > 0 and us.min() < 0


def test_girifalco_asymptote(oracle_lib):
    # far from contact the sphere-sphere form becomes -12 alpha / s^6 + 90 beta / s^12, s = r/d
    a, b, d = 0.7, 0.05, 1.1
    for s in (30.0, 60.0):
        u, _ = oracle.pair_potential("girifalco", s * d, [a, b, 0, 0], d, 1e9, "trunc")
        assert u == pytest.approx(-12 * a / s ** 6 + 90 * b / s ** 12, rel=20.0 / s ** 2)
    # alpha and beta enter linearly
    u1, _ = oracle.pair_potential("girifalco", 1.6 * d, [a, 0.0, 0, 0], d, 1e9, "trunc")
    u2, _ = oracle.pair_potential("girifalco", 1.6 * d, [0.0, b, 0, 0], d, 1e9, "trunc")
    u3, _ = oracle.pair_potential("girifalco", 1.6 * d, [a, b, 0, 0], d, 1e9, "trunc")
    assert u3 == pytest.approx(u1 + u2, rel=1e-13)


@pytest.mark.parametrize("kind", list(KINDS))
def test_whole_system_gradient_and_newton(oracle_lib, kind):
    p, sig, rc = KINDS[kind]
    s = gen.lj_fcc_state(108, 0.5 if kind != "girifalco" else 0.15, 1.0, 5)
    s = gen.jitter_positions(s, 0.05, 6)
    one = np.ones((1, 1))
    pot = (kind, np.array(p).reshape(1, 1, 4))
    pos = s.pos.astype(np.float64)
    F, _, _, U, W = oracle.forces_f64(pos, s.types, s.box, sig * one, one, rc * one, "sf", pot=pot)
    assert np.abs(F.sum(0)).max() <= 1e-12 * s.n * np.abs(F).max()
    h = 1e-6
    for i in (3, 40, 99):
        for c in range(3):
            p1 = pos.copy(); p1[i, c] += h
            p2 = pos.copy(); p2[i, c] -= h
            e1 = oracle.forces_f64(p1, s.types, s.box, sig * one, one, rc * one, "sf", pot=pot)[3]
            e2 = oracle.forces_f64(p2, s.types, s.box, sig * one, one, rc * one, "sf", pot=pot)[3]
            assert -(e1 - e2) / (2 * h) == pytest.approx(F[i, c], rel=1e-5, abs=1e-6 * np.abs(F).max())
