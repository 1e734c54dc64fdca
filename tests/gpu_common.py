"""Helpers shared by the GPU tests: building systems from seeded states and the
tolerance checks of the parity contract."""
import numpy as np

FORCE_TOL = 1e-5   # max-norm error / max-norm of the reference
ENERGY_TOL = 1e-6  # relative, potential energy and virial


def force_error(F_gpu, F_ref):
    return float(np.abs(np.asarray(F_gpu, np.float64) - F_ref).max() / np.abs(F_ref).max())


def rel(a, b):
    return abs(a - b) / abs(b)


def make_system(state, sig, eps, rc, method, skin=0.3, precision="f32", launch=None):
    import torch
    from paper_1506_05094_amd import srmd

    stream = torch.cuda.current_stream().cuda_stream
    s = srmd.system_from_state(state, sig, eps, rc, method, skin=skin, precision=precision, stream=stream)
    if launch is not None:
        s.set_launch(*launch)
    return s


def min_image(d, box):
    return d - box * np.rint(d / box)
