"""The autotuner of the paper's appendix with its skin optimisation and its
tuned-parameter file, on the GPU: the state is restored bitwise, the chosen skin
is the one the list is built with (pair set bit-exact against the oracle at that
skin), forces keep parity, a second system with the same user parameters takes
the record without timing anything, and other user parameters tune again."""
import numpy as np
import pytest

import oracle
from workloads import generators as gen

from gpu_common import ENERGY_TOL, FORCE_TOL, force_error, make_system, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1506_05094_amd import srmd
    srmd.load()
    oracle.load()


def _pairs_at(pos, types, box, rc, skin):
    cs2, _ = oracle.cut_tables(rc, skin)
    return oracle.pair_set(pos, types, box, cs2)


def _check_choice(t):
    assert t["tp"] in (1, 2, 4, 8, 16, 32, 64) and (t["tp"] * t["ppb"]) % 64 == 0 and t["tp"] * t["ppb"] <= 1024
    assert t["list_mode"] in (1, 2, 3, 4) and t["persistent"] in (0, -1)
    assert 0.0 < t["skin"]


def test_full_autotune_skin_cache_and_reuse(tmp_path):
    state = gen.config1_state()
    sig, eps, rc = gen.ka_params()
    cache = str(tmp_path / "tuned.txt")
    print("KA 4096 NVT: full autotune", flush=True)
    with make_system(state, sig, eps, rc, "sf") as s:
        s.set_integrator_nvt(0.002, 0.45, 0.2)
        s.step(50)
        before = s.get_state()
        key = s.tuning_key()
        t = s.autotune_full(40, cache)
        print(f"tuned {t}", flush=True)
        _check_choice(t)
        assert t["from_cache"] == 0 and t["trials"] > 10
        assert t["baseline_ms_per_step"] > 0 and t["tuned_ms_per_step"] > 0
        assert s.get_launch() == (t["tp"], t["ppb"])
        assert (s.stats()["persistent_groups"] > 0) == (t["persistent"] == -1)
        after = s.get_state()
        np.testing.assert_array_equal(before["pos"], after["pos"])
        np.testing.assert_array_equal(before["vel"], after["vel"])
        s.build_neighbor_list()
        got = s.neighbor_pairs()
        th = s.compute_forces()
        F = s.get_state()["force"]
    assert key["gpu"] and key["compute_units"] > 0 and key["thermostat"] == 1
    assert key["count"] == [int((state.types == 0).sum()), int((state.types == 1).sum())]
    assert key["temperature"] == 0.45 and key["dt"] == 0.002
    assert rel(key["density"], 4096 / np.prod(state.box.astype(np.float32).astype(np.float64))) < 1e-12
    np.testing.assert_array_equal(key["rcut"], rc)
    np.testing.assert_array_equal(got, _pairs_at(after["pos"], state.types, state.box, rc, t["skin"]))
    Fr, _, _, U, W = oracle.forces_f32(after["pos"], state.types, state.box, sig, eps, rc, "sf")
    assert force_error(F, Fr) <= FORCE_TOL
    assert rel(th["pe"], U) <= ENERGY_TOL and rel(th["virial"], W) <= ENERGY_TOL
    assert len(open(cache).read().splitlines()) == 1

    # same user parameters, another configuration: the record applies, nothing is timed
    print("same parameters: cached", flush=True)
    state2 = gen.jitter_positions(state, 0.02, 7)
    with make_system(state2, sig, eps, rc, "sf") as s2:
        s2.set_integrator_nvt(0.002, 0.45, 0.2)
        t2 = s2.autotune_full(40, cache)
        assert t2["from_cache"] == 1 and t2["trials"] == 0
        assert [t2[k] for k in ("tp", "ppb", "list_mode", "persistent", "skin")] == \
            [t[k] for k in ("tp", "ppb", "list_mode", "persistent", "skin")]
        assert s2.get_launch() == (t["tp"], t["ppb"])
        s2.build_neighbor_list()
        got2 = s2.neighbor_pairs()
        pos2 = s2.get_state()["pos"]
    np.testing.assert_array_equal(got2, _pairs_at(pos2, state2.types, state2.box, rc, t["skin"]))

    # another time step: tuned again, a second record
    print("other dt: tuned again", flush=True)
    with make_system(state, sig, eps, rc, "sf") as s3:
        s3.set_integrator_nvt(0.004, 0.45, 0.2)
        t3 = s3.autotune_full(40, cache)
        _check_choice(t3)
        assert t3["from_cache"] == 0 and t3["trials"] > 10
    assert len(open(cache).read().splitlines()) == 2


def test_full_autotune_without_cache_nve_key_temperature():
    """NVE: the key's temperature is the kinetic temperature of the state; without a
    cache path the tuner still runs and the list follows the tuned skin."""
    state = gen.config2_state(2000)
    sig, eps, rc = gen.lj_params()
    print("LJ 2000 NVE: full autotune, no cache", flush=True)
    with make_system(state, sig, eps, rc, "sp") as s:
        s.set_integrator_nve(0.005)
        key = s.tuning_key()
        v = state.vel.astype(np.float64)
        m = np.asarray(state.mass, np.float64)[state.types]
        T = (m[:, None] * v * v).sum() / (3 * len(v) - 3)
        assert rel(key["temperature"], T) < 1e-12
        assert key["thermostat"] == 0 and key["count"] == [2000]
        before = s.get_state()
        t = s.autotune_full(30)
        _check_choice(t)
        assert t["from_cache"] == 0
        after = s.get_state()
        np.testing.assert_array_equal(before["pos"], after["pos"])
        np.testing.assert_array_equal(before["vel"], after["vel"])
        s.build_neighbor_list()
        got = s.neighbor_pairs()
    np.testing.assert_array_equal(got, _pairs_at(after["pos"], state.types, state.box, rc, t["skin"]))


def test_full_autotune_salt_key_separates_charged_system(tmp_path):
    """The molten salt tunes with its Coulomb method in the key; the same particles
    without charges do not reuse that record."""
    st = gen.molten_salt_state(2000, 31)
    sig, eps, rc, q, rcc = gen.salt_params()
    cache = str(tmp_path / "tuned.txt")
    print("salt 2000: full autotune", flush=True)
    with make_system(st, sig, eps, rc, "sf") as s:
        s.set_coulomb_sf(q, rcc)
        s.set_integrator_nvt(0.004, gen.SALT_T, 0.2)
        key = s.tuning_key()
        t = s.autotune_full(20, cache)
        _check_choice(t)
        assert key["cutoff_method"] == 3 and t["from_cache"] == 0
        s.build_neighbor_list()
        got = s.neighbor_pairs()
        pos = s.get_state()["pos"]
    cs2, _ = oracle.cut_tables(np.maximum(rc, rcc), t["skin"])
    np.testing.assert_array_equal(got, oracle.pair_set(pos, st.types, st.box, cs2))
    with make_system(st, sig, eps, rc, "sf") as s2:
        s2.set_integrator_nvt(0.004, gen.SALT_T, 0.2)
        assert s2.tuning_key()["cutoff_method"] == 2
        t2 = s2.autotune_full(20, cache)
        assert t2["from_cache"] == 0
    assert len(open(cache).read().splitlines()) == 2
