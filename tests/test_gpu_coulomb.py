"""The molten salt of the paper's Coulomb benchmark (section 9) on the GPU against the
oracle: shifted-force Lennard-Jones plus shifted-force Coulomb with cutoff 6.0, charges
+1 / -1.  Pair sets bit-exact (listed within max(r_c, r_cc) + skin), forces within
1e-5 of the max-norm, energies within 1e-6, short trajectories within 1e-4, and the
step forms (chains, persistent kernel, batched replicas) bitwise equal at one layout."""
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


SKIN = 0.3


def _salt_system(state, launch=None, skin=SKIN):
    sig, eps, rc, q, rcc = gen.salt_params()
    s = make_system(state, sig, eps, rc, "sf", skin=skin, launch=launch)
    s.set_coulomb_sf(q, rcc)
    return s


def _oracle_forces(pos, state, sel=None):
    sig, eps, rc, q, rcc = gen.salt_params()
    return oracle.forces_f32(pos, state.types, state.box, sig, eps, rc, "sf", sel=sel, charges=q, rc_coul=rcc)


def _list_cut(skin=SKIN):
    _, _, rc, _, rcc = gen.salt_params()
    cs2, _ = oracle.cut_tables(np.maximum(rc, rcc), skin)
    return cs2


@pytest.fixture(scope="module")
def salt2000():
    return gen.jitter_positions(gen.molten_salt_state(2000, 11), 0.02, 3)


@pytest.mark.parametrize("paths", [(0, 0), (2, 2), (2, 3), (1, 4)])
def test_pair_set_bit_exact(salt2000, paths):
    print(f"salt 2000 pair set paths={paths}", flush=True)
    st = salt2000
    with _salt_system(st) as s:
        s.set_rebuild_path(*paths)
        s.build_neighbor_list()
        got = s.neighbor_pairs()
    ref = oracle.pair_set(st.pos, st.types, st.box, _list_cut())
    assert got.shape == ref.shape and len(ref) > 2000 * 300
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("tp", [1, 4, 16, 64])
def test_forces_energy_virial(salt2000, tp):
    print(f"salt 2000 forces tp={tp}", flush=True)
    st = salt2000
    with _salt_system(st, launch=(tp, max(1, 256 // tp))) as s:
        th = s.compute_forces()
        F = s.get_state()["force"]
    Fr, _, _, U, W = _oracle_forces(st.pos, st)
    assert force_error(F, Fr) <= FORCE_TOL
    assert rel(th["pe"], U) <= ENERGY_TOL
    assert rel(th["virial"], W) <= ENERGY_TOL


def test_coulomb_term_is_present_and_removable(salt2000):
    """Without the Coulomb term the library matches the Lennard-Jones-only oracle, and
    the two differ by far more than the tolerance (so the term is really added)."""
    st = salt2000
    sig, eps, rc, q, rcc = gen.salt_params()
    with _salt_system(st) as s:
        th_c = s.compute_forces()
        s.set_coulomb_sf(None, 0.0)
        th_lj = s.compute_forces()
        F_lj = s.get_state()["force"]
    Fl, _, _, Ul, Wl = oracle.forces_f32(st.pos, st.types, st.box, sig, eps, rc, "sf")
    assert force_error(F_lj, Fl) <= FORCE_TOL and rel(th_lj["pe"], Ul) <= ENERGY_TOL
    assert abs(th_c["pe"] - th_lj["pe"]) > 100 * ENERGY_TOL * abs(th_c["pe"])


def test_shifted_potential_lj_with_charges_is_rejected(salt2000):
    from paper_1506_05094_amd import srmd
    sig, eps, rc, q, rcc = gen.salt_params()
    with make_system(salt2000, sig, eps, rc, "sp", skin=SKIN) as s:
        s.set_coulomb_sf(q, rcc)
        s.set_integrator_nve(0.004)
        with pytest.raises(srmd.SrmdError) as e:
            s.step(1)
        assert e.value.status == srmd.SRMD_EUNSUPPORTED


def test_trajectory_vs_oracle_and_forms_equal(salt2000):
    """20 Nose-Hoover steps at the benchmark's dt and T against the FP64 oracle; the
    launch chains and the persistent kernel agree bit for bit."""
    print("salt 2000 trajectory", flush=True)
    st = salt2000
    sig, eps, rc, q, rcc = gen.salt_params()
    out = []
    for mode in (0, -1):
        with _salt_system(st, launch=(16, 16)) as s:
            s.set_integrator_nvt(0.004, gen.SALT_T, 0.2)
            s.set_persistent(mode)
            s.step(20)
            out.append(s.get_state()["pos"])
    np.testing.assert_array_equal(out[0], out[1])
    ref = oracle.integrate(st.pos, st.vel, st.types, st.mass, st.box, sig, eps, rc, "sf", 0.004, 20, thermostat=True,
                           T0=gen.SALT_T, tau=0.2, charges=q, rc_coul=rcc)
    d = min_image(out[0].astype(np.float64) - ref["pos"], st.box)
    assert np.abs(d).max() <= 1e-4


def test_batched_salt_replicas_equal_single_runs():
    from paper_1506_05094_amd import srmd
    # at density 0.3677, N >= 1000 keeps half the box side above r_cc + skin = 6.3
    states = [gen.molten_salt_state(n, 40 + n) for n in (1000, 1500, 2400)]
    print("salt batch", flush=True)
    singles = []
    for st in states:
        with _salt_system(st, launch=(1, 256)) as s:
            s.set_integrator_nvt(0.002, gen.SALT_T, 0.2)
            s.set_persistent(-1)
            s.step(40)
            singles.append(s.get_state()["pos"])
    systems = [_salt_system(st, launch=(1, 256)) for st in states]
    try:
        for s in systems:
            s.set_integrator_nvt(0.002, gen.SALT_T, 0.2)
        with srmd.Batch(systems) as b:
            b.step(40)
        for s, ref in zip(systems, singles):
            np.testing.assert_array_equal(s.get_state()["pos"], ref)
    finally:
        for s in systems:
            s.close()


def test_large_salt_sampled_forces():
    """N = 20 000 (the paper's middle size): forces on 256 sampled particles against the
    oracle's per-particle sums, and PE/W of the whole system."""
    print("salt 20000 sampled forces", flush=True)
    st = gen.molten_salt_state(20000, 21)
    sel = np.random.default_rng(2).choice(st.n, 256, replace=False).astype(np.int32)
    with _salt_system(st) as s:
        th = s.compute_forces()
        F = s.get_state()["force"]
    Fr, _, _, _, _ = _oracle_forces(st.pos, st, sel=sel)
    assert force_error(F[sel], Fr) <= FORCE_TOL
    _, _, _, U, W = _oracle_forces(st.pos, st)
    assert rel(th["pe"], U) <= ENERGY_TOL and rel(th["virial"], W) <= ENERGY_TOL


def test_large_salt_persistent_equals_chain():
    """N = 20 000 runs the large-system persistent kernel (four-phase sort, lists in
    device memory) with the Coulomb method: bitwise equal to the launch chains."""
    print("salt 20000 persistent vs chain", flush=True)
    st = gen.molten_salt_state(20000, 23)
    out = []
    for mode in (0, -1):
        with _salt_system(st, launch=(8, 32)) as s:
            s.set_integrator_nvt(0.004, gen.SALT_T, 0.2)
            s.set_persistent(mode)
            s.step(60)
            assert (s.stats()["persistent_groups"] > 0) == (mode == -1)
            out.append(s.get_state()["pos"])
    np.testing.assert_array_equal(out[0], out[1])


@pytest.mark.parametrize("precision", ["f32_kahan", "f64pos"])
def test_salt_trajectory_other_position_precisions(salt2000, precision):
    """The Coulomb method in the compensated and float64-master position variants:
    20 NVT steps within 1e-4 of the FP64 oracle."""
    print(f"salt 2000 trajectory {precision}", flush=True)
    st = salt2000
    sig, eps, rc, q, rcc = gen.salt_params()
    with make_system(st, sig, eps, rc, "sf", skin=SKIN, precision=precision) as s:
        s.set_coulomb_sf(q, rcc)
        s.set_integrator_nvt(0.004, gen.SALT_T, 0.2)
        s.step(20)
        got = s.get_state()["pos"]
    ref = oracle.integrate(st.pos, st.vel, st.types, st.mass, st.box, sig, eps, rc, "sf", 0.004, 20, thermostat=True,
                           T0=gen.SALT_T, tau=0.2, charges=q, rc_coul=rcc)
    d = min_image(got.astype(np.float64) - ref["pos"], st.box)
    assert np.abs(d).max() <= 1e-4
