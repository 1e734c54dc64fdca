"""The allocation-free force entry point (srmd_compute_forces_noalloc) against the
existing one (srmd_compute_forces on a system of the same configuration), through
the C-ABI: two calls in a row on one GPU, the second with a smaller system, each
equal to the allocating path (bit for bit at the same default launch shape) and at
parity with the oracle."""
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


def _noalloc(state, sig, eps, rc, method, skin):
    import torch
    from paper_1506_05094_amd import srmd
    n = state.n
    dev = torch.device("cuda")
    pos = torch.from_numpy(np.ascontiguousarray(state.pos, np.float32)).to(dev)
    typ = torch.from_numpy(np.ascontiguousarray(state.types, np.int32)).to(dev)
    force = torch.full((n, 3), np.nan, dtype=torch.float32, device=dev)
    energy = torch.full((2,), np.nan, dtype=torch.float64, device=dev)
    status = torch.full((1,), -1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    cfg = srmd.lj_config(n, state.box, sig, eps, rc, method, skin)
    srmd.compute_forces_noalloc(cfg, pos.data_ptr(), typ.data_ptr(), force.data_ptr(), energy.data_ptr(),
                                status.data_ptr(), stream.cuda_stream)
    stream.synchronize()
    return force.cpu().numpy(), energy.cpu().numpy(), int(status.cpu().item())


def _allocating(state, sig, eps, rc, method, skin):
    with make_system(state, sig, eps, rc, method, skin=skin) as s:
        th = s.compute_forces()
        return s.get_state()["force"], np.array([th["pe"], th["virial"]])


def test_noalloc_matches_allocating_path_twice_shrinking():
    cases = [
        (gen.jitter_positions(gen.config1_state(), 0.05, 17), gen.ka_params(), "sf"),  # N = 4096, 2 types
        (gen.jitter_positions(gen.config0_state(), 0.1, 18), gen.lj_params(), "sp"),   # N = 864, smaller
    ]
    for state, (sig, eps, rc), method in cases:
        print(f"N={state.n} method={method}", flush=True)
        F, E, status = _noalloc(state, sig, eps, rc, method, 0.3)
        assert status == 0
        Fa, Ea = _allocating(state, sig, eps, rc, method, 0.3)
        np.testing.assert_array_equal(F, Fa)
        np.testing.assert_array_equal(E, Ea)
        Fr, _, _, U, W = oracle.forces_f32(state.pos, state.types, state.box, sig, eps, rc, method)
        assert force_error(F, Fr) <= FORCE_TOL
        assert rel(E[0], U) <= ENERGY_TOL and rel(E[1], W) <= ENERGY_TOL


def test_noalloc_rejects_what_it_cannot_hold():
    from paper_1506_05094_amd import srmd
    state = gen.config2_state(16000)
    sig, eps, rc = gen.lj_params()
    cfg = srmd.lj_config(state.n, state.box, sig, eps, rc, "sp", 0.3)
    with pytest.raises(srmd.SrmdError) as e:
        srmd.compute_forces_noalloc(cfg, 1, 1, 1, 1, 1)  # rejected on the host before any device access
    assert e.value.status == srmd.SRMD_EUNSUPPORTED
