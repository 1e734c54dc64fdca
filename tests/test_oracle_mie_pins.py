"""Pins of the oracle's two-power pair potential U(r) = A (sigma/r)^m - B (sigma/r)^n
(paper section 2 lists generalised Lennard-Jones and inverse power laws among the
pair potentials).  Each pin would fail for a plausible mistake: the 12-6 special
case must be the (separately pinned) Lennard-Jones oracle; the generalised
Lennard-Jones form eps/(m-n) [n s^m - m s^n] has its minimum -eps at r = sigma for
any exponents; a homogeneous inverse power law has r F = m U pair by pair, so the
virial is m/3 times the energy; the force is minus the derivative of the energy; the
shifted-force variant vanishes with its force at the cutoff."""
import numpy as np
import pytest

import oracle


@pytest.fixture(scope="module", autouse=True)
def _lib():
    oracle.load()


@pytest.mark.parametrize("method", ["trunc", "sp", "sf"])
def test_twelve_six_is_lennard_jones(method):
    for r in (0.95, 1.12, 1.7, 2.4):
        u, f = oracle.pair_mie(r, 4 * 0.8, 4 * 0.8, 12, 6, 1.1, 2.6, method)
        ul, fl = oracle.pair(r, 1.1, 0.8, 2.6, method)
        assert abs(u - ul) <= 1e-13 * max(1.0, abs(ul)) and abs(f - fl) <= 1e-13 * max(1.0, abs(fl))


def test_twelve_six_forces_match_lennard_jones_oracle():
    rng = np.random.default_rng(3)
    L = 7.0
    pos = rng.uniform(-L / 2, L / 2, (120, 3)).astype(np.float32)
    types = (np.arange(120) % 2).astype(np.int32)
    box = np.array([L, L, L])
    sig = np.array([[1.0, 0.8], [0.8, 0.88]])
    eps = np.array([[1.0, 1.5], [1.5, 0.5]])
    rc = 2.5 * sig
    mie = (4 * eps, 4 * eps, np.full((2, 2), 12), np.full((2, 2), 6))
    F, _, _, U, W = oracle.forces_f32(pos, types, box, sig, np.zeros((2, 2)), rc, "sf", mie=mie)
    Fl, _, _, Ul, Wl = oracle.forces_f32(pos, types, box, sig, eps, rc, "sf")
    assert np.abs(F - Fl).max() <= 1e-12 * np.abs(Fl).max()
    assert abs(U - Ul) <= 1e-12 * abs(Ul) and abs(W - Wl) <= 1e-12 * abs(Wl)


@pytest.mark.parametrize("m,n", [(12, 6), (18, 6), (24, 12), (36, 18), (8, 4)])
def test_generalised_lennard_jones_minimum(m, n):
    eps, sig = 1.3, 0.9
    A, B = eps * n / (m - n), eps * m / (m - n)
    u, f = oracle.pair_mie(sig, A, B, m, n, sig, 10.0, "trunc")
    assert abs(u + eps) <= 1e-13 and abs(f) <= 1e-12
    u2, _ = oracle.pair_mie(sig * 1.01, A, B, m, n, sig, 10.0, "trunc")
    u3, _ = oracle.pair_mie(sig * 0.99, A, B, m, n, sig, 10.0, "trunc")
    assert u2 > u and u3 > u


@pytest.mark.parametrize("m", [6, 12, 18])
def test_inverse_power_law_virial_is_m_thirds_of_energy(m):
    """B = 0: U = A (sigma/r)^m, r F = m U for every pair, so W = (m/3) U (plain truncation)."""
    rng = np.random.default_rng(m)
    L = 8.0
    pos = rng.uniform(-L / 2, L / 2, (150, 3)).astype(np.float32)
    types = np.zeros(150, np.int32)
    box = np.array([L, L, L])
    one = np.ones((1, 1))
    mie = (0.7 * one, 0 * one, np.full((1, 1), m), np.full((1, 1), 6))
    _, _, _, U, W = oracle.forces_f32(pos, types, box, one, 0 * one, 3.5 * one, "trunc", mie=mie)
    assert abs(W - m / 3.0 * U) <= 1e-12 * abs(W)
    assert abs(oracle.pair_mie(1.0, 0.7, 0.0, m, 6, 1.0, 3.5, "trunc")[0] - 0.7) <= 1e-15


@pytest.mark.parametrize("m,n,method", [(18, 6, "sf"), (36, 18, "sp"), (12, 4, "trunc")])
def test_force_is_minus_energy_derivative(m, n, method):
    A, B, sig, rc = 1.7, 2.2, 1.0, 2.7
    for r in (0.9, 1.15, 1.6, 2.3):
        h = 1e-6
        up = oracle.pair_mie(r + h, A, B, m, n, sig, rc, method)[0]
        um = oracle.pair_mie(r - h, A, B, m, n, sig, rc, method)[0]
        f = oracle.pair_mie(r, A, B, m, n, sig, rc, method)[1]
        assert abs(-(up - um) / (2 * h) - f) <= 1e-6 * max(1.0, abs(f))


def test_shifted_force_vanishes_at_cutoff():
    u, f = oracle.pair_mie(2.5 * (1 - 1e-10), 1.7, 2.2, 18, 6, 1.0, 2.5, "sf")
    assert abs(u) < 1e-12 and abs(f) < 1e-9
    u, f = oracle.pair_mie(2.5 * (1 - 1e-10), 1.7, 2.2, 18, 6, 1.0, 2.5, "sp")
    assert abs(u) < 1e-10 and abs(f) > 1e-4
