"""GPU edge cases against the oracle: the smallest system (two particles, also with
the pair across the periodic boundary), a system with no pair in range, four
particle types with their own masses, sizes that leave ragged last blocks at the
extreme thread layouts, and a box with fewer than five cells along every axis.
Pair sets bit-exact; forces within 1e-5 of the max-norm; energies within 1e-6."""
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


def _state(pos, types, L, vel, mass, recipe):
    box = np.array([L, L, L], np.float64)
    p = np.asarray(pos, np.float64)
    p = p - box * np.floor((p + box / 2) / box)  # into [-L/2, L/2)
    p = p.astype(np.float32)
    p[p >= np.float32(L / 2)] = np.float32(-L / 2)
    return gen.State(pos=p, vel=np.asarray(vel, np.float32), types=np.asarray(types, np.int32), box=box,
                     mass=np.asarray(mass, np.float64), ntypes=len(mass), seed=0, recipe=recipe)


def _against_oracle(state, params, method, launch=None, paths=None, skin=0.3):
    sig, eps, rc = params
    with make_system(state, sig, eps, rc, method, skin=skin, launch=launch) as s:
        if paths is not None:
            s.set_rebuild_path(*paths)
        s.build_neighbor_list()
        got = s.neighbor_pairs()
        th = s.compute_forces()
        F = s.get_state()["force"]
    cs2, _ = oracle.cut_tables(rc, skin)
    ref = oracle.pair_set(state.pos, state.types, state.box, cs2)
    assert got.shape == ref.shape
    np.testing.assert_array_equal(got, ref)
    Fr, _, _, U, W = oracle.forces_f32(state.pos, state.types, state.box, sig, eps, rc, method)
    if np.abs(Fr).max() > 0:
        assert force_error(F, Fr) <= FORCE_TOL
        assert rel(th["pe"], U) <= ENERGY_TOL
        assert rel(th["virial"], W) <= ENERGY_TOL
    else:
        assert np.abs(F).max() == 0.0 and th["pe"] == 0.0 and th["virial"] == 0.0
    return got


def _trajectory_vs_oracle(state, params, method, steps, launch=None, persistent=0, nvt=None, tol=1e-4):
    sig, eps, rc = params
    with make_system(state, sig, eps, rc, method, launch=launch) as s:
        if nvt is None:
            s.set_integrator_nve(0.004)
        else:
            s.set_integrator_nvt(0.004, *nvt)
        s.set_persistent(persistent)
        s.step(steps)
        got = s.get_state()["pos"]
    kw = {} if nvt is None else dict(thermostat=True, T0=nvt[0], tau=nvt[1])
    ref = oracle.integrate(state.pos, state.vel, state.types, state.mass, state.box, sig, eps, rc, method, 0.004,
                           steps, **kw)
    d = min_image(got.astype(np.float64) - ref["pos"], state.box)
    assert np.abs(d).max() <= tol
    return got


TWO = {
    "inside": [[0.3, -0.2, 0.1], [1.5, 0.1, -0.3]],
    "across_boundary": [[-3.55, 0.05, 0.0], [3.45, 0.25, 0.1]],  # 1.02 apart through the face x = +-4
}


@pytest.mark.parametrize("where", list(TWO))
@pytest.mark.parametrize("paths", [(1, 1), (2, 2), (2, 3), (1, 4)])
def test_two_particles(where, paths):
    print(f"two particles {where} paths={paths}", flush=True)
    st = _state(TWO[where], [0, 0], 8.0, [[0.1, 0.0, -0.05], [-0.1, 0.02, 0.05]], [1.0], f"two {where}")
    got = _against_oracle(st, gen.lj_params(), "sf", paths=paths)
    np.testing.assert_array_equal(got, [[0, 1], [1, 0]])


@pytest.mark.parametrize("persistent", [0, -1])
def test_two_particles_trajectory(persistent):
    st = _state(TWO["across_boundary"], [0, 0], 8.0, [[0.3, 0.0, -0.05], [-0.3, 0.02, 0.05]], [1.0], "two")
    _trajectory_vs_oracle(st, gen.lj_params(), "sf", 200, persistent=persistent)


def test_no_pair_in_range():
    """A simple cubic lattice of spacing 3.0 > r_c + s = 2.8: every list is empty and
    the particles move ballistically."""
    print("no pair in range", flush=True)
    g = (np.arange(4) - 1.5) * 3.0
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    vel = np.random.default_rng(4).uniform(-0.5, 0.5, pos.shape)
    st = _state(pos, np.zeros(len(pos)), 12.0, vel, [1.0], "sc lattice spacing 3")
    got = _against_oracle(st, gen.lj_params(), "sp")
    assert got.shape == (0, 2)
    for persistent in (0, -1):
        _trajectory_vs_oracle(st, gen.lj_params(), "sp", 20, persistent=persistent, tol=1e-5)


def _four_types():
    # density 0.8: the per-particle virials all have one sign (at 0.9 with these sigmas
    # the total is 1/20 of the sum of their magnitudes, and a relative check of the
    # total would measure the cancellation, not the kernel)
    rng = np.random.default_rng(11)
    m = 7
    L = (4 * m ** 3 / 0.8) ** (1.0 / 3.0)
    pos = gen.fcc_lattice(m, L / m) + rng.uniform(-0.05, 0.05, (4 * m ** 3, 3))
    types = rng.integers(0, 4, 4 * m ** 3)
    mass = np.array([1.0, 0.5, 2.0, 1.5])
    vel = rng.standard_normal(pos.shape) * np.sqrt(0.8 / mass[types])[:, None]
    vel -= (mass[types][:, None] * vel).sum(0) / mass[types].sum()
    sig = np.array([[1.0, 0.9, 1.1, 0.8], [0.9, 0.95, 1.0, 0.85], [1.1, 1.0, 1.05, 0.9], [0.8, 0.85, 0.9, 0.9]])
    eps = np.array([[1.0, 1.5, 0.8, 1.2], [1.5, 0.5, 1.0, 0.7], [0.8, 1.0, 1.3, 0.9], [1.2, 0.7, 0.9, 0.6]])
    return _state(pos, types, L, vel, mass, "fcc 1372, four types"), (sig, eps, 2.5 * sig)


@pytest.mark.parametrize("tp", [1, 8, 64])
def test_four_types(tp):
    print(f"four types tp={tp}", flush=True)
    st, params = _four_types()
    _against_oracle(st, params, "sf", launch=(tp, max(1, 256 // tp)))


def test_four_types_nvt_trajectory_and_persistent_equal():
    st, params = _four_types()
    a = _trajectory_vs_oracle(st, params, "sf", 20, launch=(8, 32), nvt=(0.8, 0.2))
    b = _trajectory_vs_oracle(st, params, "sf", 20, launch=(8, 32), nvt=(0.8, 0.2), persistent=-1)
    np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("n", [1001, 4097])
@pytest.mark.parametrize("launch", [(64, 4), (1, 64), (2, 512)])
def test_ragged_sizes_extreme_layouts(n, launch):
    """N not a multiple of any block: the last block, wave and lane group are partial;
    t_p = 64 (a whole wave per particle), t_p = 1 and 1024-thread blocks."""
    print(f"ragged N={n} launch={launch}", flush=True)
    st = gen.jitter_positions(gen.config2_state(n), 0.05, n)
    _against_oracle(st, gen.lj_params(), "sp", launch=launch)


@pytest.mark.parametrize("launch", [(64, 4), (2, 512)])
def test_ragged_size_persistent_equals_chain(launch):
    st = gen.jitter_positions(gen.config2_state(1001), 0.05, 5)
    sig, eps, rc = gen.lj_params()
    out = []
    for mode in (0, -1):
        with make_system(st, sig, eps, rc, "sp", launch=launch) as s:
            s.set_integrator_nve(0.004)
            s.set_persistent(mode)
            s.step(150)
            out.append(s.get_state()["pos"])
    np.testing.assert_array_equal(out[0], out[1])


def test_fewer_than_five_cells_per_axis():
    """N = 200 at density 0.8442: L = 6.19 holds 4 cells of side >= 1.4 per axis, so
    the stencil takes every cell of each axis once."""
    print("small box", flush=True)
    st = gen.jitter_positions(gen.lj_fcc_state(200, 0.8442, 0.722, 6), 0.05, 6)
    for paths in [(1, 1), (2, 2), (2, 3), (1, 4)]:
        _against_oracle(st, gen.lj_params(), "sp", paths=paths)
    a = _trajectory_vs_oracle(st, gen.lj_params(), "sp", 30, launch=(8, 32))
    b = _trajectory_vs_oracle(st, gen.lj_params(), "sp", 30, launch=(8, 32), persistent=-1)
    np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("form", ["chain", "persistent", "force_only"])
def test_non_finite_force_reports_estate(form):
    """Two particles on one site (r = 0): the first force evaluation is not finite,
    and the call returns SRMD_ESTATE.  Only these two particles turn non-finite
    (NVE); the cell coordinate of a non-finite position is clamped into the grid, so
    the later steps of the call index nothing outside the arrays."""
    from paper_1506_05094_amd import srmd
    state = gen.config0_state().copy()
    state.pos[7] = state.pos[3]
    sig, eps, rc = gen.lj_params()
    print(f"form={form}", flush=True)
    with make_system(state, sig, eps, rc, "sp") as s:
        s.set_integrator_nve(0.005)
        if form == "persistent":
            s.set_persistent(-1)
        with pytest.raises(srmd.SrmdError) as e:
            if form == "force_only":
                s.compute_forces()
            else:
                s.step(30)
        assert e.value.status == srmd.SRMD_ESTATE
        # the system stays usable: a finite state set from the host steps again
        s.set_state(pos=gen.config0_state().pos, vel=gen.config0_state().vel)
        if form == "persistent":
            s.set_persistent(0)
        s.step(5)
        assert np.isfinite(s.get_state()["pos"]).all()
