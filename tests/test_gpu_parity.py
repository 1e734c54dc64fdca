"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle on the same
seeded inputs.  Pair sets bit-exact; forces within 1e-5 of the max-norm; potential
energy and virial within 1e-6 relative."""
import numpy as np
import pytest

import oracle
from workloads import generators as gen

from gpu_common import ENERGY_TOL, FORCE_TOL, force_error, make_system, min_image, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1506_05094_amd import srmd
    srmd.load()
    oracle.load()


def _cases():
    c0 = gen.config0_state()
    c0j = gen.jitter_positions(c0, 0.1, 3)
    c1 = gen.config1_state()
    return {
        "lj864_fcc": (c0, gen.lj_params(), "sp"),
        "lj864_jitter": (c0j, gen.lj_params(), "sp"),
        "ka4096_random": (c1, gen.ka_params(), "sf"),
    }


CASES = _cases()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("tp", [1, 4, 16])
def test_pair_set_bit_exact(name, tp):
    state, (sig, eps, rc), method = CASES[name]
    print(f"case {name} tp={tp}", flush=True)
    with make_system(state, sig, eps, rc, method, launch=(tp, 256 // tp)) as s:
        s.build_neighbor_list()
        got = s.neighbor_pairs()
    cs2, _ = oracle.cut_tables(rc, 0.3)
    ref = oracle.pair_set(state.pos, state.types, state.box, cs2)
    assert got.shape == ref.shape
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("tp", [1, 2, 8, 32])
def test_forces_energy_virial(name, tp):
    state, (sig, eps, rc), method = CASES[name]
    print(f"case {name} tp={tp}", flush=True)
    with make_system(state, sig, eps, rc, method, launch=(tp, 256 // tp)) as s:
        th = s.compute_forces()
        F = s.get_state()["force"]
    Fr, pe, w, U, W = oracle.forces_f32(state.pos, state.types, state.box, sig, eps, rc, method)
    if name == "lj864_fcc":  # forces vanish by symmetry: absolute check
        assert np.abs(F).max() < 1e-3
    else:
        assert force_error(F, Fr) <= FORCE_TOL
    assert rel(th["pe"], U) <= ENERGY_TOL
    assert rel(th["virial"], W) <= ENERGY_TOL


@pytest.mark.parametrize("method", ["trunc", "sp", "sf"])
def test_cutoff_methods(method):
    state = gen.jitter_positions(gen.config0_state(), 0.1, 8)
    sig, eps, rc = gen.lj_params()
    with make_system(state, sig, eps, rc, method) as s:
        th = s.compute_forces()
        F = s.get_state()["force"]
    Fr, _, _, U, W = oracle.forces_f32(state.pos, state.types, state.box, sig, eps, rc, method)
    assert force_error(F, Fr) <= FORCE_TOL
    assert rel(th["pe"], U) <= ENERGY_TOL
    assert rel(th["virial"], W) <= ENERGY_TOL


def test_state_roundtrip_original_order():
    state = gen.config1_state()
    sig, eps, rc = gen.ka_params()
    with make_system(state, sig, eps, rc, "sf") as s:
        s.build_neighbor_list()          # reorders particles on the device
        st = s.get_state()
    np.testing.assert_array_equal(st["pos"], state.pos)
    np.testing.assert_array_equal(st["vel"], state.vel)
    np.testing.assert_array_equal(st["image"], 0)


def test_short_trajectory_nve():
    state = gen.config0_state()
    sig, eps, rc = gen.lj_params()
    steps = 10
    with make_system(state, sig, eps, rc, "sp") as s:
        s.set_integrator_nve(0.005)
        tr = s.step(steps, thermo_every=1)
        st = s.get_state()
    ref = oracle.integrate(state.pos, state.vel, state.types, state.mass, state.box, sig, eps, rc, "sp", 0.005,
                           steps)
    d = min_image(st["pos"].astype(np.float64) - ref["pos"], state.box)
    assert np.abs(d).max() <= 1e-4
    np.testing.assert_allclose(tr["pe"], ref["thermo"][:, 0], rtol=1e-5)
    np.testing.assert_allclose(tr["ke"], ref["thermo"][:, 1], rtol=1e-5)


def test_short_trajectory_nvt():
    state = gen.config1_state()
    sig, eps, rc = gen.ka_params()
    steps = 10
    with make_system(state, sig, eps, rc, "sf") as s:
        s.set_integrator_nvt(0.005, 0.45, 0.2)
        tr = s.step(steps, thermo_every=1)
        st = s.get_state()
    ref = oracle.integrate(state.pos, state.vel, state.types, state.mass, state.box, sig, eps, rc, "sf", 0.005,
                           steps, thermostat=True, T0=0.45, tau=0.2)
    d = min_image(st["pos"].astype(np.float64) - ref["pos"], state.box)
    assert np.abs(d).max() <= 1e-4
    np.testing.assert_allclose(tr["xi"], ref["thermo"][:, 5], rtol=1e-4, atol=1e-6)
    np.testing.assert_allclose(tr["pe"], ref["thermo"][:, 0], rtol=1e-5)


@pytest.mark.parametrize("name", ["lj864_jitter", "ka4096_random"])
def test_thermo_record_against_oracle(name):
    """Every field of the thermodynamic record (paper section 2: energy, pressure)
    against the oracle.  Kinetic energies of identical velocities agree to 1e-12
    (float64 on both sides, only the summation order differs); the fields that
    depend on the first step's forces (through v(1/2)) to the force tolerance."""
    state, (sig, eps, rc), method = CASES[name]
    nvt = name.startswith("ka")
    print(f"case {name}", flush=True)
    with make_system(state, sig, eps, rc, method) as s:
        th = s.compute_forces()
        if nvt:
            s.set_integrator_nvt(0.005, 0.45, 0.2)
        else:
            s.set_integrator_nve(0.005)
        tr = s.step(1, thermo_every=1)
        v_half = s.get_state()["vel"].astype(np.float64)
    kw = dict(thermostat=True, T0=0.45, tau=0.2) if nvt else {}
    ref = oracle.integrate(state.pos, state.vel, state.types, state.mass, state.box, sig, eps, rc, method, 0.005,
                           1, **kw)["thermo"][0]
    pe, ke, w, T, P, xi, xi_int, h, ke_half = ref
    v0 = state.vel.astype(np.float64)
    # force-only record: the kinetic energy of the stored velocities v(-1/2)
    assert rel(th["ke"], oracle.kinetic(v0, state.types, state.mass)) <= 1e-12
    assert rel(th["pe"], pe) <= ENERGY_TOL and rel(th["virial"], w) <= ENERGY_TOL
    r = tr[0]
    # identical velocities: v(1/2) as the device holds it, v(0) = (v(-1/2) + v(1/2)) / 2
    assert rel(r["ke_half"], oracle.kinetic(v_half, state.types, state.mass)) <= 1e-12
    assert rel(r["ke"], oracle.kinetic(0.5 * (v0 + v_half), state.types, state.mass)) <= 1e-12
    # the record against the oracle's own step (its v(1/2) from float64 forces)
    assert rel(r["pe"], pe) <= ENERGY_TOL and rel(r["virial"], w) <= ENERGY_TOL
    assert rel(r["ke"], ke) <= 1e-5 and rel(r["ke_half"], ke_half) <= 1e-5
    assert rel(r["temperature"], T) <= 1e-5
    assert rel(r["pressure"], P) <= 1e-5
    assert rel(r["h_conserved"], h) <= 1e-5
    assert r["xi"] == xi == 0.0 and r["xi_integral"] == xi_int == 0.0
    assert r["step"] == 0
