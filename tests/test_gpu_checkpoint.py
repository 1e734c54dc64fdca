"""Full-state checkpoint at the C-ABI (srmd_save_state / srmd_load_state): 2n steps
equal n steps + save + load + n steps bit for bit, in the launch chain, the
persistent kernel, the precision variants, a batch and a large system; a state
loaded into another list layout continues with a rebuilt list and stays at parity
with the oracle."""
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


KA = gen.config1_state()
KA_P = gen.ka_params()


def _ka(mode="chain", precision="f32", launch=(8, 32)):
    s = make_system(KA, *KA_P, "sf", precision=precision, launch=launch)
    s.set_integrator_nvt(0.005, 0.45, 0.2)
    if mode == "persistent":
        s.set_persistent(-1)
    return s


def _same(a, b):
    sa, sb = a.get_state(), b.get_state()
    for k in ("pos", "vel", "image", "force", "pos64"):
        np.testing.assert_array_equal(sa[k], sb[k], err_msg=k)
    ta, tb = a.thermo(), b.thermo()
    for k in ("pe", "ke", "virial", "xi", "xi_integral", "h_conserved", "step", "n_rebuilds"):
        assert ta[k] == tb[k], k


def _pending_rebuild_step():
    """A step count after which a list rebuild is pending (its sort already done)."""
    with _ka() as s:
        tr = s.step(300, thermo_every=1)
    k = np.nonzero(np.diff(tr["n_rebuilds"]) > 0)[0]
    assert len(k) > 0
    return int(k[len(k) // 2] + 1)


@pytest.mark.parametrize("mode", ["chain", "persistent"])
@pytest.mark.parametrize("where", ["odd", "pending_rebuild"])
def test_save_load_continues_bitwise(mode, where):
    n = 137 if where == "odd" else _pending_rebuild_step()
    print(f"mode={mode} n={n}", flush=True)
    with _ka(mode) as ref, _ka(mode) as a, _ka(mode) as b:
        ref.step(2 * n)
        a.step(n)
        blob = a.save_state()
        a.step(n)
        b.load_state(blob)
        b.step(n)
        _same(ref, a)
        _same(ref, b)
        # the saved system itself rewinds to the checkpoint
        a.load_state(blob)
        a.step(n)
        _same(ref, a)


@pytest.mark.parametrize("precision", ["f32_kahan", "f64pos"])
def test_save_load_precision_variants(precision):
    with _ka(precision=precision) as ref, _ka(precision=precision) as a, _ka(precision=precision) as b:
        ref.step(240)
        a.step(120)
        b.load_state(a.save_state())
        b.step(120)
        _same(ref, b)


def test_save_load_across_modes_and_batch():
    from paper_1506_05094_amd import srmd
    small = gen.ka_random_state(1200, 1.2, 0.6, 31)
    sig, eps, rc = KA_P

    def mk():
        s = make_system(small, sig, eps, rc, "sf", launch=(4, 64))
        s.set_integrator_nvt(0.005, 0.6, 0.2)
        return s

    with mk() as ref, mk() as a, mk() as b, mk() as c:
        ref.step(300)
        with srmd.Batch([a, c]) as bt:
            bt.step(150)
        blob = a.save_state()
        # continued in the persistent kernel of a fresh system, and in a batch
        b.set_persistent(-1)
        b.load_state(blob)
        b.step(150)
        _same(ref, b)
        c.load_state(blob)
        with srmd.Batch([c]) as bt:
            bt.step(150)
        _same(ref, c)


def test_save_load_large_system_chain():
    state = gen.config2_state(16000)
    sig, eps, rc = gen.lj_params()

    def mk():
        s = make_system(state, sig, eps, rc, "sp", launch=(2, 128))
        s.set_integrator_nve(0.005)
        return s

    with mk() as ref, mk() as a, mk() as b:
        ref.step(90)
        a.step(45)
        b.load_state(a.save_state())
        b.step(45)
        _same(ref, b)


def test_load_into_other_layout_rebuilds_and_keeps_parity():
    with _ka(launch=(8, 32)) as a, _ka(launch=(2, 128)) as b:
        a.step(77)
        saved = a.get_state()
        b.load_state(a.save_state())
        got = b.get_state()
        np.testing.assert_array_equal(got["pos"], saved["pos"])
        np.testing.assert_array_equal(got["vel"], saved["vel"])
        np.testing.assert_array_equal(got["image"], saved["image"])
        assert b.thermo()["step"] == a.thermo()["step"]
        th = b.compute_forces()
        F = b.get_state()["force"]
    sig, eps, rc = KA_P
    Fr, _, _, U, W = oracle.forces_f32(saved["pos"], KA.types, KA.box, sig, eps, rc, "sf")
    assert force_error(F, Fr) <= FORCE_TOL
    assert rel(th["pe"], U) <= ENERGY_TOL and rel(th["virial"], W) <= ENERGY_TOL


def test_load_rejects_foreign_or_damaged_blobs():
    from paper_1506_05094_amd import srmd
    with _ka() as a:
        a.step(10)
        blob = a.save_state()
        before = a.get_state()
        with make_system(gen.config0_state(), *gen.lj_params(), "sp") as other:
            with pytest.raises(srmd.SrmdError) as e:
                other.load_state(blob)          # another particle count
            assert e.value.status == srmd.SRMD_EINVAL
        with pytest.raises(srmd.SrmdError):
            a.load_state(blob[:-4])              # truncated
        bad = bytearray(blob)
        bad[0] ^= 0xFF
        with pytest.raises(srmd.SrmdError):
            a.load_state(bytes(bad))             # not a saved state
        np.testing.assert_array_equal(a.get_state()["pos"], before["pos"])
