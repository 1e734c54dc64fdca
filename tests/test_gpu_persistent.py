"""Persistent mode: every step of a call in one cooperative launch.  The trajectory
must be the launch chain's bit for bit at the same launch shape, for any workgroup
count, across mode switches in the middle of a run and through list-overflow
replays, for small systems (positions in LDS) and large ones (positions in device
memory, four-phase sort); systems the kernel cannot run are rejected."""
import numpy as np
import pytest

import oracle
from workloads import generators as gen

from gpu_common import make_system, min_image

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1506_05094_amd import srmd
    srmd.load()
    oracle.load()


CASES = [(500, 0.4, 21), (2600, 0.8, 22), (4100, 0.45, 23)]


def _ka(n, T, seed, launch, persistent, dt=0.002):
    sig, eps, rc = gen.ka_params()
    st = gen.ka_random_state(n, 1.2, T, seed)
    s = make_system(st, sig, eps, rc, "sf", launch=launch)
    s.set_integrator_nvt(dt, T, 0.2)
    s.set_persistent(persistent)
    return s


def _same(a, b, tra=None, trb=None, label=""):
    sa, sb = a.get_state(), b.get_state()
    np.testing.assert_array_equal(sa["pos"], sb["pos"], err_msg=label)
    np.testing.assert_array_equal(sa["vel"], sb["vel"], err_msg=label)
    np.testing.assert_array_equal(sa["image"], sb["image"], err_msg=label)
    ta, tb = a.thermo(), b.thermo()
    for f in ("pe", "ke", "virial", "xi", "xi_integral", "h_conserved", "step", "n_rebuilds", "max_nbrs"):
        assert ta[f] == tb[f], (label, f, ta[f], tb[f])
    if tra is not None:
        for f in ("pe", "ke", "virial", "xi", "h_conserved"):
            np.testing.assert_array_equal(tra[f], trb[f], err_msg=f"{label} {f}")


@pytest.mark.parametrize("launch", [(8, 32), (1, 256), (16, 16), (4, 64)])
@pytest.mark.parametrize("case", CASES)
def test_persistent_bitwise_equals_chain(case, launch):
    n, T, seed = case
    print(f"persistent vs chain N={n} launch={launch}", flush=True)
    a = _ka(n, T, seed, launch, 0)
    b = _ka(n, T, seed, launch, -1)
    assert a.stats()["persistent_groups"] == 0
    assert b.stats()["persistent_groups"] > 0
    steps = 300
    tra = a.step(steps, thermo_every=10)
    trb = b.step(steps, thermo_every=10)
    assert a.thermo()["n_rebuilds"] > 2  # the run crosses several list rebuilds
    _same(a, b, tra, trb, f"N={n} {launch}")
    a.close()
    b.close()


@pytest.mark.parametrize("groups", [1, 6, 13, 64, 200])
def test_group_count_does_not_change_result(groups):
    # N = 2600 at (8, 32): 82 blocks of 4 waves; one workgroup runs them all in rounds
    n, T, seed = CASES[1]
    print(f"persistent groups={groups}", flush=True)
    a = _ka(n, T, seed, (8, 32), 0)
    b = _ka(n, T, seed, (8, 32), groups)
    assert b.stats()["persistent_groups"] == groups
    a.step(200)
    b.step(200)
    _same(a, b, label=f"groups={groups}")
    a.close()
    b.close()


@pytest.mark.parametrize("launch", [(8, 32), (2, 128)])
def test_largest_system_lists_built_from_device_memory(launch):
    """N = 8192, the largest the persistent kernel takes: its positions fill the LDS, so
    the list build reads the sorted arrays from device memory instead of LDS copies."""
    print(f"persistent N=8192 launch={launch}", flush=True)
    a = _ka(8192, 0.6, 31, launch, 0)
    b = _ka(8192, 0.6, 31, launch, -1)
    tra = a.step(120, thermo_every=10)
    trb = b.step(120, thermo_every=10)
    assert a.thermo()["n_rebuilds"] > 2
    _same(a, b, tra, trb, f"N=8192 {launch}")
    a.close()
    b.close()


@pytest.mark.parametrize("case", [CASES[0], (7000, 0.6, 25)])
def test_mode_switches_mid_run_and_odd_chunks(case):
    """Chunks of odd length in both modes, for a system on few and on many workgroups."""
    n, T, seed = case
    print(f"mode switches N={n}", flush=True)
    a = _ka(n, T, seed, (8, 32), 0)
    b = _ka(n, T, seed, (8, 32), 0)
    a.step(331)
    for k, (mode, cnt) in enumerate([(0, 57), (-1, 101), (0, 1), (-1, 63), (-1, 1), (0, 108)]):
        b.set_persistent(mode)
        b.step(cnt)
    _same(a, b, label="switches")
    a.close()
    b.close()


def test_nve_lj_matches_chain_and_oracle():
    print("persistent NVE LJ 864", flush=True)
    st = gen.jitter_positions(gen.config0_state(), 0.05, 5)
    sig, eps, rc = gen.lj_params()
    a = make_system(st, sig, eps, rc, "sp", launch=(8, 32))
    b = make_system(st, sig, eps, rc, "sp", launch=(8, 32))
    for s in (a, b):
        s.set_integrator_nve(0.004)
    b.set_persistent(-1)
    steps = 10
    a.step(steps)
    b.step(steps)
    _same(a, b, label="nve")
    ref = oracle.integrate(st.pos, st.vel, st.types, st.mass, st.box, sig, eps, rc, "sp", 0.004, steps)
    d = min_image(b.get_state()["pos"].astype(np.float64) - ref["pos"], st.box)
    assert np.abs(d).max() <= 1e-4
    a.close()
    b.close()


def test_list_overflow_replays_like_chain():
    from paper_1506_05094_amd import srmd
    import torch
    print("persistent overflow replay", flush=True)
    rng = np.random.default_rng(7)
    L = 12.0
    g = (np.arange(9) - 4) * (L / 9)
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    pos = (pos + rng.uniform(-0.1, 0.1, pos.shape)).astype(np.float32)
    vel = (-0.5 * pos).astype(np.float32)
    stream = torch.cuda.current_stream().cuda_stream

    def contracting(mode):
        s = srmd.System(pos, np.zeros(len(pos), np.int32), [L, L, L], vel=vel, stream=stream)
        s.set_skin(0.4)
        s.set_pair_lj(0, 0, 1.0, 0.05, 2.5, "sp")
        s.set_integrator_nve(0.002)
        s.set_launch(8, 32)
        s.set_persistent(mode)
        return s

    a, b = contracting(0), contracting(-1)
    n0 = b.stats()["n_max"]
    a.step(400)
    b.step(400)
    assert b.stats()["n_max"] > n0
    _same(a, b, label="overflow")
    a.close()
    b.close()


def test_profile_reports_one_launch():
    n, T, seed = CASES[2]
    s = _ka(n, T, seed, (8, 32), -1)
    s.step(20)
    ms, dev, launches = s.profile_step_kernel(500)
    assert launches == 1 and ms > 0  # 500 steps: one launch
    assert s.thermo()["step"] == 519
    s.close()


@pytest.mark.parametrize("launch,groups", [((16, 16), -1), ((8, 32), 13), ((2, 128), 1)])
def test_all_pairs_lists_persistent_equals_chain(launch, groups):
    """List mode 4 (all pairs in index order, no sort): the persistent kernel builds
    from its LDS copy of the positions, the chain from device memory; same lists, same
    trajectory bit for bit, through rebuilds and a mode switch."""
    n, T, seed = CASES[2]
    print(f"all pairs N={n} launch={launch} groups={groups}", flush=True)
    a = _ka(n, T, seed, launch, 0)
    b = _ka(n, T, seed, launch, groups)
    for s in (a, b):
        s.set_rebuild_path(0, 4)
    tra = a.step(300, thermo_every=10)
    trb = b.step(300, thermo_every=10)
    assert a.thermo()["n_rebuilds"] > 2
    _same(a, b, tra, trb, f"all pairs {launch}")
    np.testing.assert_array_equal(a.neighbor_pairs(), b.neighbor_pairs())
    a.step(57)
    b.set_persistent(0)
    b.step(20)
    b.set_persistent(groups)
    b.step(37)
    _same(a, b, label="all pairs after switches")
    a.close()
    b.close()


def test_all_pairs_overflow_and_rejection():
    from paper_1506_05094_amd import srmd
    import torch
    rng = np.random.default_rng(7)
    L = 12.0
    g = (np.arange(9) - 4) * (L / 9)
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    pos = (pos + rng.uniform(-0.1, 0.1, pos.shape)).astype(np.float32)
    vel = (-0.5 * pos).astype(np.float32)
    stream = torch.cuda.current_stream().cuda_stream

    def contracting(mode):
        s = srmd.System(pos, np.zeros(len(pos), np.int32), [L, L, L], vel=vel, stream=stream)
        s.set_skin(0.4)
        s.set_pair_lj(0, 0, 1.0, 0.05, 2.5, "sp")
        s.set_integrator_nve(0.002)
        s.set_launch(8, 32)
        s.set_rebuild_path(0, 4)
        s.set_persistent(mode)
        return s

    a, b = contracting(0), contracting(-1)
    n0 = b.stats()["n_max"]
    a.step(400)
    b.step(400)
    assert b.stats()["n_max"] > n0
    _same(a, b, label="all pairs overflow")
    a.close()
    b.close()
    sig, eps, rc = gen.ka_params()
    big = make_system(gen.ka_random_state(9000, 1.2, 0.5, 3), sig, eps, rc, "sf")
    big.set_integrator_nve(0.002)
    big.set_rebuild_path(0, 4)
    with pytest.raises(srmd.SrmdError) as e:
        big.step(1)
    assert e.value.status == srmd.SRMD_EINVAL
    big.close()


@pytest.fixture(scope="module")
def ka12000():
    return gen.ka_random_state(12000, 1.2, 0.6, 24)


@pytest.mark.parametrize("launch,groups", [((2, 128), -1), ((8, 32), 37), ((1, 256), 256), ((4, 64), 1)])
def test_large_system_bitwise_equals_chain(ka12000, launch, groups):
    """N = 12000 (more than 8192 particles): positions from device memory and the
    four-phase sort with grid barriers, for several workgroup counts (one workgroup
    runs every phase alone)."""
    from paper_1506_05094_amd import srmd
    print(f"large persistent N=12000 launch={launch} groups={groups}", flush=True)
    sig, eps, rc = gen.ka_params()
    a = make_system(ka12000, sig, eps, rc, "sf", launch=launch)
    b = make_system(ka12000, sig, eps, rc, "sf", launch=launch)
    for s in (a, b):
        s.set_integrator_nvt(0.003, 0.6, 0.2)
    b.set_persistent(groups)
    try:
        b.step(1)
    except srmd.SrmdError as e:  # fewer workgroups fit on this device
        assert e.status == srmd.SRMD_EUNSUPPORTED and groups > 1
        pytest.skip("workgroup count does not fit")
    a.step(1)
    assert b.stats()["persistent_groups"] > 0
    tra = a.step(300, thermo_every=10)
    trb = b.step(300, thermo_every=10)
    assert a.thermo()["n_rebuilds"] > 3
    _same(a, b, tra, trb, f"N=12000 {launch} groups={groups}")
    a.close()
    b.close()


def test_large_lj_sweep_size_and_mode_switches():
    """LJ N = 64000 at t_p = 1: persistent and chain in turns, against the chain alone."""
    print("large persistent LJ 64000 switches", flush=True)
    st = gen.config2_state(64000)
    sig, eps, rc = gen.lj_params()
    a = make_system(st, sig, eps, rc, "sp", launch=(1, 256))
    b = make_system(st, sig, eps, rc, "sp", launch=(1, 256))
    for s in (a, b):
        s.set_integrator_nve(0.005)
    a.step(260)
    for mode, cnt in [(-1, 101), (0, 37), (-1, 1), (0, 1), (-1, 120)]:
        b.set_persistent(mode)
        b.step(cnt)
    assert a.thermo()["n_rebuilds"] > 3
    _same(a, b, label="LJ 64000 switches")
    a.close()
    b.close()


def test_large_system_overflow_replays_like_chain():
    from paper_1506_05094_amd import srmd
    import torch
    print("large persistent overflow replay", flush=True)
    rng = np.random.default_rng(8)
    m = 21
    L = 12.0 * m / 9
    g = (np.arange(m) - m // 2) * (L / m)
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    pos = (pos + rng.uniform(-0.1, 0.1, pos.shape)).astype(np.float32)
    vel = (-0.5 * pos).astype(np.float32)  # the same contraction rate as the small lattice
    stream = torch.cuda.current_stream().cuda_stream

    def contracting(mode):
        s = srmd.System(pos, np.zeros(len(pos), np.int32), [L, L, L], vel=vel, stream=stream)
        s.set_skin(0.4)
        s.set_pair_lj(0, 0, 1.0, 0.05, 2.5, "sp")
        s.set_integrator_nve(0.002)
        s.set_launch(4, 64)
        s.set_persistent(mode)
        return s

    a, b = contracting(0), contracting(-1)
    n0 = b.stats()["n_max"]
    a.step(400)
    b.step(400)
    assert b.stats()["n_max"] > n0
    _same(a, b, label="large overflow")
    a.close()
    b.close()


def test_rejections():
    from paper_1506_05094_amd import srmd
    sig, eps, rc = gen.ka_params()
    big = gen.ka_random_state(9000, 1.2, 0.5, 3)
    s_big = make_system(big, sig, eps, rc, "sf", launch=(16, 16))  # t_p > 8 above 8192 particles
    s_big.set_integrator_nve(0.002)
    s_big.set_persistent(-1)
    with pytest.raises(srmd.SrmdError) as e:
        s_big.step(2)
    assert e.value.status == srmd.SRMD_EUNSUPPORTED
    s_big.set_persistent(0)
    s_big.step(2)  # the launch chain still runs it
    st = gen.ka_random_state(1000, 1.2, 0.5, 4)
    p64 = make_system(st, sig, eps, rc, "sf", precision="f64pos")
    p64.set_integrator_nve(0.002)
    p64.set_persistent(-1)
    with pytest.raises(srmd.SrmdError) as e:
        p64.step(2)
    assert e.value.status == srmd.SRMD_EUNSUPPORTED
    too_many = make_system(st, sig, eps, rc, "sf")
    too_many.set_integrator_nve(0.002)
    too_many.set_persistent(4096)
    with pytest.raises(srmd.SrmdError) as e:
        too_many.step(2)
    assert e.value.status == srmd.SRMD_EUNSUPPORTED
    with pytest.raises(srmd.SrmdError) as e:
        too_many.set_persistent(-2)
    assert e.value.status == srmd.SRMD_EINVAL
    for s in (s_big, p64, too_many):
        s.close()
