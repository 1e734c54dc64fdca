"""The further pair potentials of paper section 2 (kernel method 5: Yukawa,
Buckingham, Gaussian core, Dzugutov, Girifalco) on the GPU against the oracle, each
in a liquid-like configuration: forces within 1e-5 of the max-norm and energies
within 1e-6 under the three cutoff methods and several thread layouts, the list's
pair set bit-exact, a short NVE trajectory within 1e-4, and the launch chain and the
persistent kernel bitwise equal."""
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


# kind: (params, sigma, rcut, number density, jitter) of a dense, non-overlapping start
CASES = {
    "yukawa": ([1.3, 2.0, 0.0, 0.0], 0.9, 3.0, 0.5, 0.06),
    "buckingham": ([600.0, 0.25, 1.7, 0.0], 1.0, 3.0, 0.6, 0.05),
    "gaussian": ([2.0, 0.0, 0.0, 0.0], 1.0, 2.6, 0.5, 0.1),
    "dzugutov": ([1.0, 0.0, 0.0, 0.0], 1.0, 1.94, 0.85, 0.05),
    "girifalco": ([0.7, 0.05, 0.0, 0.0], 1.0, 2.5, 0.15, 0.05),
}


def _state(kind, n=2048, seed=3):
    _, _, _, rho, jit = CASES[kind]
    return gen.jitter_positions(gen.lj_fcc_state(n, rho, 1.0, seed), jit, seed + 1)


def _tables(kind, nt=1):
    p, sig, rc, _, _ = CASES[kind]
    params = np.tile(np.asarray(p, np.float64), (nt, nt, 1))
    return params, np.full((nt, nt), sig), np.full((nt, nt), rc)


def _system(state, kind, method, launch=None, skin=0.3):
    import torch
    from paper_1506_05094_amd import srmd
    params, sig, rc = _tables(kind, state.ntypes)
    s = srmd.System(state.pos, state.types, state.box, vel=state.vel, mass=state.mass, ntypes=state.ntypes,
                    stream=torch.cuda.current_stream().cuda_stream)
    s.set_skin(skin)
    s.set_pairs_potential(kind, params, sig, rc, method)
    if launch is not None:
        s.set_launch(*launch)
    return s


def _ref(state, kind, method):
    params, sig, rc = _tables(kind, state.ntypes)
    one = np.ones_like(sig)
    return oracle.forces_f32(state.pos, state.types, state.box, sig, one, rc, method, pot=(kind, params))


@pytest.mark.parametrize("kind", list(CASES))
@pytest.mark.parametrize("method,tp", [("trunc", 1), ("sp", 4), ("sf", 16)])
def test_forces_energy_virial(kind, method, tp):
    st = _state(kind)
    print(f"{kind} {method} tp={tp}", flush=True)
    with _system(st, kind, method, launch=(tp, 256 // tp)) as s:
        th = s.compute_forces()
        F = s.get_state()["force"]
        pairs = s.neighbor_pairs()
    Fr, _, _, U, W = _ref(st, kind, method)
    assert force_error(F, Fr) <= FORCE_TOL
    assert rel(th["pe"], U) <= ENERGY_TOL and rel(th["virial"], W) <= ENERGY_TOL
    _, _, rc = _tables(kind)
    cs2, _ = oracle.cut_tables(rc, 0.3)
    np.testing.assert_array_equal(pairs, oracle.pair_set(st.pos, st.types, st.box, cs2))


@pytest.mark.parametrize("kind", list(CASES))
def test_short_trajectory_and_forms_agree(kind):
    st = _state(kind, n=1000, seed=8)
    params, sig, rc = _tables(kind)
    one = np.ones_like(sig)
    with _system(st, kind, "sf", launch=(8, 32)) as a, _system(st, kind, "sf", launch=(8, 32)) as b:
        a.set_integrator_nve(0.002)
        b.set_integrator_nve(0.002)
        b.set_persistent(-1)
        tr = a.step(10, thermo_every=1)
        b.step(10)
        sa, sb = a.get_state(), b.get_state()
    np.testing.assert_array_equal(sa["pos"], sb["pos"])
    ref = oracle.integrate(st.pos, st.vel, st.types, st.mass, st.box, sig, one, rc, "sf", 0.002, 10,
                           pot=(kind, params))
    assert np.abs(min_image(sa["pos"].astype(np.float64) - ref["pos"], st.box)).max() <= 1e-4
    # the float32 pair energies carry ~1e-6 relative error each; where attractive and
    # repulsive pairs cancel in the total (the Dzugutov start: the total is a quarter
    # of the sum of per-particle magnitudes), the bound is relative to that sum
    _, pe_i, _, _, _ = oracle.forces_f32(st.pos, st.types, st.box, sig, one, rc, "sf", pot=(kind, params))
    assert np.abs(tr["pe"] - ref["thermo"][:, 0]).max() <= 1e-5 * np.abs(pe_i).sum()


def test_two_types_mixed_parameters():
    # a 50:50 Yukawa mixture with its own prefactor and screening per type pair
    st = _state("yukawa")
    rng = np.random.default_rng(5)
    st.types[:] = (rng.random(st.n) < 0.5).astype(np.int32)
    st.ntypes = 2
    st.mass = np.array([1.0, 2.0])
    params = np.zeros((2, 2, 4))
    params[..., 0] = [[1.0, 1.5], [1.5, 0.7]]
    params[..., 1] = [[2.0, 1.5], [1.5, 1.0]]
    sig = np.array([[0.9, 0.95], [0.95, 1.0]])
    rc = np.array([[3.0, 2.8], [2.8, 2.6]])
    import torch
    from paper_1506_05094_amd import srmd
    with srmd.System(st.pos, st.types, st.box, vel=st.vel, mass=st.mass, ntypes=2,
                     stream=torch.cuda.current_stream().cuda_stream) as s:
        s.set_pairs_potential("yukawa", params, sig, rc, "sp")
        th = s.compute_forces()
        F = s.get_state()["force"]
    Fr, _, _, U, W = oracle.forces_f32(st.pos, st.types, st.box, sig, np.ones((2, 2)), rc, "sp",
                                       pot=("yukawa", params))
    assert force_error(F, Fr) <= FORCE_TOL
    assert rel(th["pe"], U) <= ENERGY_TOL and rel(th["virial"], W) <= ENERGY_TOL


def test_rejected_arguments():
    from paper_1506_05094_amd import srmd
    st = _state("yukawa", n=500)
    params, sig, rc = _tables("yukawa")
    with _system(st, "yukawa", "sp") as s:
        with pytest.raises(srmd.SrmdError):
            s.set_pairs_potential("gaussian", params, sig, rc, "sp")   # one kind per system
        with pytest.raises(srmd.SrmdError):
            s.set_pair_lj(0, 0, 1.0, 1.0, 2.5, "sp")                   # nor Lennard-Jones beside it
        bad = params.copy()
        bad[..., 1] = 100.0                                            # kappa sigma > 60
        with pytest.raises(srmd.SrmdError):
            s.set_pairs_potential("yukawa", bad, sig, rc, "sp")
