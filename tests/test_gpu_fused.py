"""Launch chains with the step ended inside the step kernel (its last workgroup runs
the fixed-order reduction, thermostat, record, rebuild decision and a small system's
spatial sort) against the separate one-workgroup end-of-step kernel: the same
trajectory, records and neighbour lists bit for bit (paper sections 5-7: one time
step; the reduction order is fixed, so the form of the launch must not show)."""
import numpy as np
import pytest

import oracle
from workloads import generators as gen

from gpu_common import make_system

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1506_05094_amd import srmd
    srmd.load()
    oracle.load()


def _ka(n, seed):
    return gen.ka_random_state(n, 1.2, 0.6, seed), gen.ka_params(), "sf"


def _lj(n, seed):
    return gen.lj_fcc_state(n, 0.8442, 0.722, seed), gen.lj_params(), "sp"


def _pair_runs(state, params, method, launch, precision="f32", list_mode=0, sort_every=0, steps=200, nvt=True):
    sig, eps, rc = params
    out = []
    for fused in (2, 1, 0):  # lists built in the step kernel too; end of step only; separate kernels
        s = make_system(state, sig, eps, rc, method, precision=precision, launch=launch)
        s.set_fused_reduction(fused)
        if list_mode:
            s.set_rebuild_path(0, list_mode)
        if sort_every:
            s.set_sort_interval(sort_every)
        if nvt:
            s.set_integrator_nvt(0.002, 0.6, 0.2)
        else:
            s.set_integrator_nve(0.004)
        tr = s.step(steps, thermo_every=10)
        tr2 = s.step(37, thermo_every=1)  # a chunk that is not a whole graph
        out.append((s, np.concatenate([tr, tr2]), s.get_state()))
    return out


def _assert_same(runs, label):
    sb, tb, xb = runs[-1]  # separate kernels
    pb = sb.neighbor_pairs()
    for form, (sa, ta, xa) in zip((2, 1), runs[:-1]):
        for k in ("pos", "vel", "image", "pos64"):
            np.testing.assert_array_equal(xa[k], xb[k], err_msg=f"{label} form {form}: {k}")
        for f in ta.dtype.names:
            np.testing.assert_array_equal(ta[f], tb[f], err_msg=f"{label} form {form}: record field {f}")
        np.testing.assert_array_equal(sa.neighbor_pairs(), pb, err_msg=f"{label} form {form}: neighbour pairs")
    assert tb["n_rebuilds"][-1] > tb["n_rebuilds"][0], f"{label}: no rebuild in the run"
    for s, _, _ in runs:
        s.close()


@pytest.mark.parametrize("launch", [(16, 16), (8, 32), (32, 8), (1, 256), (4, 64), (64, 16)])
def test_fused_equals_separate_small_ka(launch):
    """KA N = 1500 NVT (small system: the sort runs in the last workgroup; the lists
    are built in the step kernel at (16, 16), (8, 32) and (32, 8); the other layouts
    have more particles per wave or more LDS than that form takes and fall back)."""
    print(f"fused vs separate: KA 1500 launch={launch}", flush=True)
    st, params, method = _ka(1500, 31)
    _assert_same(_pair_runs(st, params, method, launch), f"KA 1500 {launch}")


@pytest.mark.parametrize("precision", ["f32_kahan", "f64pos"])
def test_fused_equals_separate_precisions(precision):
    print(f"fused vs separate: LJ 2048 {precision}", flush=True)
    st, params, method = _lj(2048, 32)
    _assert_same(_pair_runs(st, params, method, (8, 32), precision=precision, nvt=False), f"LJ {precision}")


@pytest.mark.parametrize("launch", [(16, 16), (32, 8)])
@pytest.mark.parametrize("sort_every", [0, 3])
def test_fused_equals_separate_all_pairs(sort_every, launch):
    """All-pairs lists: the tail re-sorts only when the periodic re-sort is due; at
    (32, 8) the lists are built in the step kernel (two particles per wave), at
    (16, 16) form 2 falls back to form 1."""
    print(f"fused vs separate: KA 1000 all pairs {launch}, re-sort every {sort_every}", flush=True)
    st, params, method = _ka(1000, 33)
    _assert_same(_pair_runs(st, params, method, launch, list_mode=4, sort_every=sort_every),
                 f"all pairs {launch} re-sort {sort_every}")


def test_step_form_reported():
    """The stats report the form each request resolves to."""
    st, (sig, eps, rc), method = _ka(1500, 39)
    s = make_system(st, sig, eps, rc, method, launch=(16, 16))
    got = []
    for flag in (0, 1, 2, None):
        s.set_fused_reduction(flag)
        got.append(s.stats()["step_form"])
    s.set_launch(1, 256)  # 64 particles per wave to build: form 2 falls back to 1
    s.set_fused_reduction(2)
    got.append(s.stats()["step_form"])
    assert got == [0, 1, 2, 2, 1], got
    assert s.stats()["list_mode"] == 1
    s.close()


@pytest.mark.parametrize("launch,list_mode", [((1, 256), 0), ((4, 16), 0), ((1, 256), 1), ((2, 128), 2),
                                              ((1, 256), 5)])
def test_fused_equals_separate_large_system(launch, list_mode):
    """LJ N = 20 000 (multi-kernel sort, no sort in the tail; form 2 falls back to 1)
    with each list builder of large systems (wave per cell by default at this size,
    wave per particle, thread per particle, row-staged threads); at (4, 16) the grid
    has 1250 blocks, so each stand-in thread of the tail folds two partials."""
    print(f"fused vs separate: LJ 20000 launch={launch} list mode {list_mode}", flush=True)
    st, params, method = _lj(20000, 34)
    _assert_same(_pair_runs(st, params, method, launch, list_mode=list_mode, steps=120, nvt=False),
                 f"LJ 20000 {launch} list mode {list_mode}")


def test_sort_arrays_past_the_lds_limit_fall_back():
    """A dilute LJ fluid of N = 8000 at density 0.34 in 20^3 cells (a cell side is at
    least half of r_c + skin): the sort's LDS arrays (4 (8001 + 8000) bytes) exceed the
    tail's 60 KiB, so the separate kernel ends the steps, with the same results."""
    print("fused vs separate: LJ 8000 at density 0.34 in 8000 cells", flush=True)
    st = gen.lj_fcc_state(8000, 0.34, 0.722, 35)
    runs = _pair_runs(st, gen.lj_params(), "sp", (8, 32), steps=160, nvt=False)
    assert runs[0][0].stats()["ncell"] == 8000
    _assert_same(runs, "LJ gas 8000")


def test_fused_chain_equals_persistent():
    """The one-launch chain (lists built in the step kernel) follows the persistent
    kernel's trajectory bit for bit."""
    print("fused chain vs persistent: KA 3000 (16, 16)", flush=True)
    st, (sig, eps, rc), method = _ka(3000, 36)
    runs = []
    for mode in (0, -1):
        s = make_system(st, sig, eps, rc, method, launch=(16, 16))
        s.set_fused_reduction(2)
        s.set_persistent(mode)
        s.set_integrator_nvt(0.002, 0.6, 0.2)
        tr = s.step(600, thermo_every=20)
        runs.append((s, tr, s.get_state()))
    (sa, ta, xa), (sb, tb, xb) = runs
    np.testing.assert_array_equal(xa["pos"], xb["pos"])
    np.testing.assert_array_equal(xa["vel"], xb["vel"])
    for f in ("pe", "ke", "virial", "h_conserved", "xi", "n_rebuilds"):
        np.testing.assert_array_equal(ta[f], tb[f], err_msg=f)
    sa.close()
    sb.close()


def test_automatic_choice_matches_both_forms():
    """The default (the library's choice) gives the same trajectory as either form,
    for a grid the automatic rule keeps separate (KA 4096 at t_p = 32: 512 blocks)."""
    print("fused: automatic choice, KA 4096 (32, 8)", flush=True)
    st, (sig, eps, rc), method = _ka(4096, 38)
    finals = []
    for flag in (None, 2, 1, 0):
        s = make_system(st, sig, eps, rc, method, launch=(32, 8))
        s.set_fused_reduction(flag)
        s.set_integrator_nvt(0.002, 0.6, 0.2)
        s.step(150)
        finals.append(s.get_state()["pos"])
        s.close()
    for f in finals[1:]:
        np.testing.assert_array_equal(finals[0], f)


def test_rejects_bad_flag():
    from paper_1506_05094_amd import srmd

    st, (sig, eps, rc), method = _ka(500, 37)
    s = make_system(st, sig, eps, rc, method)
    with pytest.raises(srmd.SrmdError):
        srmd._check(srmd.load().srmd_set_fused_reduction(s._h, 3), s._h)
    s.close()
