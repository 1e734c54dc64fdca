"""The two-power pair potential A (sigma/r)^m - B (sigma/r)^n (kernel method 4) on the
GPU against the oracle: generalised Lennard-Jones 18-6 under the three cutoff methods,
an inverse power law (B = 0) in a two-type mixture, a short trajectory, and the
chain and persistent forms bitwise equal.  Forces within 1e-5 of the max-norm,
energies within 1e-6, positions within 1e-4."""
import numpy as np
import pytest

import oracle
from workloads import generators as gen

from gpu_common import ENERGY_TOL, FORCE_TOL, force_error, min_image, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1506_05094_amd import srmd
    srmd.load()
    oracle.load()


def _system(state, mie, sigma, rc, method, launch=None, skin=0.3):
    import torch
    from paper_1506_05094_amd import srmd
    s = srmd.System(state.pos, state.types, state.box, vel=state.vel, mass=state.mass, ntypes=state.ntypes,
                    stream=torch.cuda.current_stream().cuda_stream)
    s.set_skin(skin)
    s.set_pairs_mie(*mie, sigma, rc, method)
    if launch is not None:
        s.set_launch(*launch)
    return s


def _glj(m, n, eps=1.0):
    one = np.ones((1, 1))
    return (eps * n / (m - n) * one, eps * m / (m - n) * one, m * one, n * one)


@pytest.fixture(scope="module")
def lj2000():
    return gen.jitter_positions(gen.config2_state(2000), 0.05, 9)


@pytest.mark.parametrize("method,tp", [("trunc", 1), ("sp", 8), ("sf", 32)])
def test_generalised_lj_forces(lj2000, method, tp):
    print(f"two-power 18-6 {method} tp={tp}", flush=True)
    st = lj2000
    mie = _glj(18, 6)
    sig, rc = np.ones((1, 1)), np.full((1, 1), 2.5)
    with _system(st, mie, sig, rc, method, launch=(tp, max(1, 256 // tp))) as s:
        th = s.compute_forces()
        F = s.get_state()["force"]
    Fr, _, _, U, W = oracle.forces_f32(st.pos, st.types, st.box, sig, np.zeros((1, 1)), rc, method, mie=mie)
    assert force_error(F, Fr) <= FORCE_TOL
    assert rel(th["pe"], U) <= ENERGY_TOL and rel(th["virial"], W) <= ENERGY_TOL


def test_inverse_power_law_mixture():
    """B = 0, m = 12 with Kob-Andersen sigmas and amplitudes (a soft-sphere mixture)."""
    print("IPL-12 mixture", flush=True)
    st = gen.jitter_positions(gen.config1_state(), 0.02, 4)
    sig, eps, rc = gen.ka_params()
    mie = (4 * eps, np.zeros((2, 2)), np.full((2, 2), 12), np.full((2, 2), 6))
    with _system(st, mie, sig, rc, "sp", launch=(8, 32)) as s:
        th = s.compute_forces()
        F = s.get_state()["force"]
    Fr, _, _, U, W = oracle.forces_f32(st.pos, st.types, st.box, sig, np.zeros((2, 2)), rc, "sp", mie=mie)
    assert force_error(F, Fr) <= FORCE_TOL
    assert rel(th["pe"], U) <= ENERGY_TOL and rel(th["virial"], W) <= ENERGY_TOL


def test_trajectory_and_forms_equal(lj2000):
    print("two-power trajectory", flush=True)
    st = lj2000
    mie = _glj(24, 12)
    sig, rc = np.ones((1, 1)), np.full((1, 1), 2.2)
    out = []
    for mode in (0, -1):
        with _system(st, mie, sig, rc, "sf", launch=(8, 32)) as s:
            s.set_integrator_nve(0.004)
            s.set_persistent(mode)
            s.step(20)
            out.append(s.get_state()["pos"])
    np.testing.assert_array_equal(out[0], out[1])
    ref = oracle.integrate(st.pos, st.vel, st.types, st.mass, st.box, sig, np.zeros((1, 1)), rc, "sf", 0.004, 20,
                           mie=mie)
    d = min_image(out[0].astype(np.float64) - ref["pos"], st.box)
    assert np.abs(d).max() <= 1e-4


def test_mixing_potentials_is_rejected(lj2000):
    from paper_1506_05094_amd import srmd
    st = gen.config1_state()
    sig, eps, rc = gen.ka_params()
    with _system(st, (4 * eps, 4 * eps, np.full((2, 2), 12), np.full((2, 2), 6)), sig, rc, "sf") as s:
        with pytest.raises(srmd.SrmdError) as e:
            s.set_pairs(sig, eps, rc, "sf")
        assert e.value.status == srmd.SRMD_EINVAL
        s.set_coulomb_sf([1.0, -1.0], 3.0)
        s.set_integrator_nve(0.004)
        with pytest.raises(srmd.SrmdError) as e:
            s.step(1)
        assert e.value.status == srmd.SRMD_EUNSUPPORTED
