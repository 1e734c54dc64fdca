"""Thin ctypes binding of libsrmd (the C-ABI declared in include/srmd.h).

Argument marshalling only: every step of the computation runs in the HIP kernels
of libsrmd.so.  The module-level functions carry the C names; ``System`` is a small
convenience wrapper over them.  PyTorch is used for device memory (the allocator
hook) and for the HIP stream the library enqueues on.
"""
from __future__ import annotations

import ctypes
import os
import sys

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsrmd.so")

SRMD_OK, SRMD_EINVAL, SRMD_ENOMEM, SRMD_EHIP, SRMD_ESTATE, SRMD_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
SRMD_CUT_TRUNC, SRMD_CUT_SP, SRMD_CUT_SF = 0, 1, 2
SRMD_PREC_F32, SRMD_PREC_F32_KAHAN, SRMD_PREC_F64POS = 0, 1, 2
CUTOFF = {"trunc": SRMD_CUT_TRUNC, "sp": SRMD_CUT_SP, "sf": SRMD_CUT_SF}
POTENTIALS = {"yukawa": 2, "buckingham": 3, "gaussian": 4, "dzugutov": 5, "girifalco": 6}
PRECISION = {"f32": SRMD_PREC_F32, "f32_kahan": SRMD_PREC_F32_KAHAN, "f64pos": SRMD_PREC_F64POS}


class srmd_thermo(ctypes.Structure):
    _fields_ = [(name, ctypes.c_double) for name in
                ("pe", "ke", "virial", "temperature", "pressure", "xi", "xi_integral", "h_conserved", "ke_half")] + [
        ("step", ctypes.c_int64), ("n_rebuilds", ctypes.c_int64), ("max_nbrs", ctypes.c_int32),
        ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


class srmd_stats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("n_rebuilds", ctypes.c_int64), ("list_entries", ctypes.c_int64),
                ("max_nbrs", ctypes.c_int32), ("n_max", ctypes.c_int32), ("tp", ctypes.c_int32),
                ("ppb", ctypes.c_int32), ("blocks", ctypes.c_int32), ("ncell", ctypes.c_int32),
                ("persistent_groups", ctypes.c_int32), ("list_mode", ctypes.c_int32), ("step_form", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class srmd_tuning_key(ctypes.Structure):
    _fields_ = [("gpu", ctypes.c_char * 64), ("compute_units", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("cutoff_method", ctypes.c_int32), ("thermostat", ctypes.c_int32), ("ntypes", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("count", ctypes.c_int64 * 4), ("density", ctypes.c_double),
                ("temperature", ctypes.c_double), ("dt", ctypes.c_double), ("sigma", ctypes.c_double * 16),
                ("epsilon", ctypes.c_double * 16), ("rcut", ctypes.c_double * 16), ("potential", ctypes.c_int32),
                ("reserved2", ctypes.c_int32), ("pot_param", ctypes.c_double * 64), ("charge", ctypes.c_double * 4),
                ("rc_coulomb", ctypes.c_double)]

    def as_dict(self):
        k = self.ntypes
        d = {name: getattr(self, name) for name in ("compute_units", "precision", "cutoff_method", "thermostat",
                                                    "ntypes", "density", "temperature", "dt", "potential",
                                                    "rc_coulomb")}
        d["gpu"] = self.gpu.decode()
        d["count"] = list(self.count[:k])
        for name in ("sigma", "epsilon", "rcut"):
            d[name] = np.array(getattr(self, name)[:k * k]).reshape(k, k)
        d["pot_param"] = np.array(self.pot_param[:4 * k * k]).reshape(k, k, 4)
        d["charge"] = list(self.charge[:k])
        return d

    @classmethod
    def from_dict(cls, d):
        k = cls()
        k.gpu = d["gpu"].encode()
        for name in ("compute_units", "precision", "cutoff_method", "thermostat", "ntypes", "density",
                     "temperature", "dt"):
            setattr(k, name, d[name])
        nt = int(d["ntypes"])
        for q, c in enumerate(d["count"]):
            k.count[q] = int(c)
        for name in ("sigma", "epsilon", "rcut"):
            a = np.asarray(d[name], np.float64).reshape(-1)
            assert a.size == nt * nt
            for q, v in enumerate(a):
                getattr(k, name)[q] = float(v)
        k.potential = int(d.get("potential", 0))
        k.rc_coulomb = float(d.get("rc_coulomb", 0.0))
        if "pot_param" in d:
            a = np.asarray(d["pot_param"], np.float64).reshape(-1)
            assert a.size == 4 * nt * nt
            for q, v in enumerate(a):
                k.pot_param[q] = float(v)
        for q, v in enumerate(d.get("charge", [])):
            k.charge[q] = float(v)
        return k


class srmd_lj_config(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("ntypes", ctypes.c_int32), ("method", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("box", ctypes.c_double * 3), ("skin", ctypes.c_double),
                ("sigma", ctypes.c_double * 16), ("epsilon", ctypes.c_double * 16), ("rcut", ctypes.c_double * 16)]


class srmd_tuning(ctypes.Structure):
    _fields_ = [("tp", ctypes.c_int32), ("ppb", ctypes.c_int32), ("list_mode", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("skin", ctypes.c_double),
                ("baseline_ms_per_step", ctypes.c_double), ("tuned_ms_per_step", ctypes.c_double),
                ("trials", ctypes.c_int32), ("from_cache", ctypes.c_int32), ("sort_every", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}

    @classmethod
    def from_dict(cls, d):
        t = cls()
        for name, _ in cls._fields_:
            if name in d:
                setattr(t, name, d[name])
        return t


THERMO_DTYPE = np.dtype([(name, np.float64) for name in
                         ("pe", "ke", "virial", "temperature", "pressure", "xi", "xi_integral", "h_conserved",
                          "ke_half")] + [("step", np.int64), ("n_rebuilds", np.int64), ("max_nbrs", np.int32),
                                         ("reserved", np.int32)])
assert THERMO_DTYPE.itemsize == ctypes.sizeof(srmd_thermo)


class SrmdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"srmd status {status}: {msg}")
        self.status = status


_lib = None
_ALLOC_T = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_T = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_alloc_keepalive = []

_vp = ctypes.c_void_p
_fp = ctypes.POINTER(ctypes.c_float)
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


def library_path() -> str:
    return LIB_PATH


def load():
    """Load libsrmd.so; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libsrmd.so not built at {LIB_PATH}; run paper_1506_05094_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    st = ctypes.c_int
    sysp = ctypes.c_void_p
    sig = {
        "srmd_create": (st, [ctypes.POINTER(sysp), ctypes.c_int32, ctypes.c_int32, _dp, _fp, _ip, _fp, _dp,
                             ctypes.c_int, _vp]),
        "srmd_destroy": (st, [sysp]),
        "srmd_set_allocator": (st, [_ALLOC_T, _FREE_T, _vp]),
        "srmd_set_pair_lj": (st, [sysp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_int]),
        "srmd_set_skin": (st, [sysp, ctypes.c_double]),
        "srmd_set_coulomb_sf": (st, [sysp, _dp, ctypes.c_double]),
        "srmd_set_pair_mie": (st, [sysp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_int]),
        "srmd_set_pair_potential": (st, [sysp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int, _dp, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_int]),
        "srmd_set_integrator_nve": (st, [sysp, ctypes.c_double]),
        "srmd_set_integrator_nvt": (st, [sysp, ctypes.c_double, ctypes.c_double, ctypes.c_double]),
        "srmd_set_launch": (st, [sysp, ctypes.c_int32, ctypes.c_int32]),
        "srmd_get_launch": (st, [sysp, _ip, _ip]),
        "srmd_set_rebuild_path": (st, [sysp, ctypes.c_int32, ctypes.c_int32]),
        "srmd_set_persistent": (st, [sysp, ctypes.c_int32]),
        "srmd_set_sort_interval": (st, [sysp, ctypes.c_int32]),
        "srmd_set_fused_reduction": (st, [sysp, ctypes.c_int32]),
        "srmd_batch_create": (st, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32]),
        "srmd_batch_create_limited": (st, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                           ctypes.c_int32, ctypes.c_int32]),
        "srmd_batch_step": (st, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, _vp, ctypes.c_int64]),
        "srmd_batch_destroy": (st, [ctypes.c_void_p]),
        "srmd_batch_autotune": (st, [ctypes.c_void_p, ctypes.c_int32, _ip, _ip]),
        "srmd_batch_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
        "srmd_autotune": (st, [sysp, ctypes.c_int32, _ip, _ip]),
        "srmd_tuning_key_of": (st, [sysp, ctypes.POINTER(srmd_tuning_key)]),
        "srmd_tuning_cache_find": (st, [ctypes.c_char_p, ctypes.POINTER(srmd_tuning_key),
                                        ctypes.POINTER(srmd_tuning), _ip]),
        "srmd_tuning_cache_store": (st, [ctypes.c_char_p, ctypes.POINTER(srmd_tuning_key),
                                         ctypes.POINTER(srmd_tuning)]),
        "srmd_autotune_full": (st, [sysp, ctypes.c_int32, ctypes.c_char_p, ctypes.POINTER(srmd_tuning)]),
        "srmd_build_neighbor_list": (st, [sysp]),
        "srmd_compute_forces": (st, [sysp, ctypes.POINTER(srmd_thermo)]),
        "srmd_step": (st, [sysp, ctypes.c_int64, ctypes.c_int32, _vp, ctypes.c_int64]),
        "srmd_get_state": (st, [sysp, _fp, _fp, _ip, _fp, _dp]),
        "srmd_get_particle_terms": (st, [sysp, _fp, _fp]),
        "srmd_compute_forces_noalloc": (st, [ctypes.POINTER(srmd_lj_config), _vp, _vp, _vp, _vp, _vp, _vp]),
        "srmd_save_state": (st, [sysp, _vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]),
        "srmd_load_state": (st, [sysp, _vp, ctypes.c_size_t]),
        "srmd_set_state": (st, [sysp, _fp, _fp]),
        "srmd_get_neighbor_pairs": (st, [sysp, _ip, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
        "srmd_get_thermo": (st, [sysp, ctypes.POINTER(srmd_thermo)]),
        "srmd_get_box": (st, [sysp, _dp]),
        "srmd_last_error": (ctypes.c_char_p, [sysp]),
        "srmd_get_stats": (st, [sysp, ctypes.POINTER(srmd_stats)]),
        "srmd_profile_step_kernel": (st, [sysp, ctypes.c_int64, _dp, _dp, ctypes.POINTER(ctypes.c_int64)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status, sysp=None):
    if status != SRMD_OK:
        msg = load().srmd_last_error(sysp)
        raise SrmdError(status, msg.decode() if msg else "")


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _ptr(a, t):
    return None if a is None else a.ctypes.data_as(t)


def install_torch_allocator():
    """Route every later device allocation of libsrmd through torch's caching allocator."""
    import torch

    lib = load()

    def _alloc(nbytes, ctx):
        try:
            dev = torch.cuda.current_device()
            return int(torch.cuda.caching_allocator_alloc(int(nbytes), dev))
        except Exception:  # reported to the library as an allocation failure
            return None

    def _free(ptr, ctx):
        torch.cuda.caching_allocator_delete(int(ptr))

    a = _ALLOC_T(_alloc)
    f = _FREE_T(_free)
    _alloc_keepalive[:] = [a, f]
    _check(lib.srmd_set_allocator(a, f, None))


def uninstall_allocator():
    lib = load()
    _check(lib.srmd_set_allocator(_ALLOC_T(), _FREE_T(), None))


class System:
    """One simulated system on the GPU (a handle to srmd_system)."""

    def __init__(self, pos, types, box, vel=None, mass=None, ntypes=None, precision="f32", stream=None):
        lib = load()
        pos = _f32(pos).reshape(-1, 3)
        n = pos.shape[0]
        types = np.ascontiguousarray(types, dtype=np.int32)
        box = np.ascontiguousarray(box, dtype=np.float64)
        vel = None if vel is None else _f32(vel).reshape(-1, 3)
        nt = int(ntypes if ntypes is not None else types.max() + 1)
        mass = None if mass is None else np.ascontiguousarray(mass, dtype=np.float64)
        prec = PRECISION[precision] if isinstance(precision, str) else int(precision)
        if stream is None:
            stream_ptr = None
        else:
            stream_ptr = ctypes.c_void_p(int(stream))
        h = ctypes.c_void_p()
        _check(lib.srmd_create(ctypes.byref(h), n, nt, _ptr(box, _dp), _ptr(pos, _fp), _ptr(types, _ip),
                               _ptr(vel, _fp), _ptr(mass, _dp), prec, stream_ptr))
        self._h = h
        self.n = n
        self.ntypes = nt

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None):
            load().srmd_destroy(self._h)
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter shutdown the HIP runtime may already be gone: leave the
        # memory to the process exit instead of calling into the library (the
        # check is bound at definition: module globals such as sys may already
        # be cleared when a late finaliser runs)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- setup
    def set_pair_lj(self, ti, tj, sigma, epsilon, rcut, method):
        m = CUTOFF[method] if isinstance(method, str) else int(method)
        _check(load().srmd_set_pair_lj(self._h, ti, tj, sigma, epsilon, rcut, m), self._h)

    def set_pairs(self, sigma, eps, rc, method):
        sigma = np.asarray(sigma)
        for a in range(sigma.shape[0]):
            for b in range(a, sigma.shape[0]):
                self.set_pair_lj(a, b, float(sigma[a, b]), float(eps[a, b]), float(rc[a, b]), method)

    def set_skin(self, skin):
        _check(load().srmd_set_skin(self._h, float(skin)), self._h)

    def set_pairs_mie(self, A, B, m, n, sigma, rc, method):
        """Two-power potential A (sigma/r)^m - B (sigma/r)^n for every type pair (arrays
        ntypes x ntypes, symmetric) with one cutoff method."""
        lib = load()
        mth = CUTOFF[method] if isinstance(method, str) else int(method)
        A, B, m, n, sigma, rc = (np.asarray(x).reshape(self.ntypes, self.ntypes) for x in (A, B, m, n, sigma, rc))
        for a in range(self.ntypes):
            for b in range(a, self.ntypes):
                _check(lib.srmd_set_pair_mie(self._h, a, b, float(A[a, b]), float(B[a, b]), int(m[a, b]),
                                             int(n[a, b]), float(sigma[a, b]), float(rc[a, b]), mth), self._h)

    def set_pairs_potential(self, kind, params, sigma, rc, method):
        """A further potential (srmd_set_pair_potential) for every type pair: kind a name
        of POTENTIALS, params ntypes x ntypes x 4, sigma and rc ntypes x ntypes."""
        lib = load()
        k = POTENTIALS[kind] if isinstance(kind, str) else int(kind)
        mth = CUTOFF[method] if isinstance(method, str) else int(method)
        nt = self.ntypes
        params = np.asarray(params, np.float64).reshape(nt, nt, 4)
        sigma, rc = (np.asarray(x, np.float64).reshape(nt, nt) for x in (sigma, rc))
        for a in range(nt):
            for b in range(a, nt):
                p = np.ascontiguousarray(params[a, b])
                _check(lib.srmd_set_pair_potential(self._h, a, b, k, _ptr(p, _dp), float(sigma[a, b]),
                                                   float(rc[a, b]), mth), self._h)

    def set_coulomb_sf(self, charges, rcut):
        """Shifted-force Coulomb term (paper section 9): one charge per type, one cutoff;
        charges=None removes it."""
        if charges is None:
            _check(load().srmd_set_coulomb_sf(self._h, None, 0.0), self._h)
            return
        q = np.ascontiguousarray(charges, dtype=np.float64)
        if q.shape != (self.ntypes,):
            raise ValueError("one charge per type")
        _check(load().srmd_set_coulomb_sf(self._h, _ptr(q, _dp), float(rcut)), self._h)

    def set_integrator_nve(self, dt):
        _check(load().srmd_set_integrator_nve(self._h, float(dt)), self._h)

    def set_integrator_nvt(self, dt, T0, tau):
        _check(load().srmd_set_integrator_nvt(self._h, float(dt), float(T0), float(tau)), self._h)

    def set_launch(self, tp, ppb):
        _check(load().srmd_set_launch(self._h, int(tp), int(ppb)), self._h)

    def set_rebuild_path(self, sort_mode=0, list_mode=0):
        """sort_mode 0 auto, 1 one-workgroup sort, 2 multi-kernel sort; list_mode 0 auto,
        1 wave per particle, 2 thread per particle, 3 wave per cell, 4 all pairs (small
        systems, no sort).  Every mode gives the same pair set."""
        _check(load().srmd_set_rebuild_path(self._h, int(sort_mode), int(list_mode)), self._h)

    def set_sort_interval(self, builds):
        """All-pairs lists: spatial re-sort before every builds-th list build (0: never)."""
        _check(load().srmd_set_sort_interval(self._h, int(builds)), self._h)

    def set_fused_reduction(self, enable=True):
        """Launch chains: the step kernel's last workgroup ends each step (True or 1),
        and also builds a small system's lists at the start of the step (2); separate
        kernels (False or 0); the library's choice (None, the default).  Bitwise the
        same results in every form."""
        v = -1 if enable is None else int(enable)
        _check(load().srmd_set_fused_reduction(self._h, v), self._h)

    def set_persistent(self, groups=-1):
        """Run steps as persistent launches of 500 steps each (groups > 0 workgroups,
        or -1 for the library's choice); 0 returns to graph-captured launch chains."""
        _check(load().srmd_set_persistent(self._h, int(groups)), self._h)

    def get_launch(self):
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check(load().srmd_get_launch(self._h, ctypes.byref(a), ctypes.byref(b)), self._h)
        return a.value, b.value

    def autotune(self, steps_per_trial=200):
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check(load().srmd_autotune(self._h, int(steps_per_trial), ctypes.byref(a), ctypes.byref(b)), self._h)
        return a.value, b.value

    def autotune_full(self, steps_per_trial=200, cache_path=None):
        """The appendix's autotuner with skin optimisation; with cache_path, its
        tuned-parameter file is read first and written after tuning.  Returns the
        chosen parameters as a dict (srmd_tuning)."""
        t = srmd_tuning()
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(load().srmd_autotune_full(self._h, int(steps_per_trial), path, ctypes.byref(t)), self._h)
        return t.as_dict()

    def tuning_key(self):
        k = srmd_tuning_key()
        _check(load().srmd_tuning_key_of(self._h, ctypes.byref(k)), self._h)
        return k.as_dict()

    # -- compute
    def build_neighbor_list(self):
        _check(load().srmd_build_neighbor_list(self._h), self._h)

    def compute_forces(self):
        t = srmd_thermo()
        _check(load().srmd_compute_forces(self._h, ctypes.byref(t)), self._h)
        return t.as_dict()

    def step(self, nsteps, thermo_every=0, trace_cap=None):
        if thermo_every > 0:
            cap = int(trace_cap if trace_cap is not None else (nsteps + thermo_every - 1) // thermo_every)
            trace = np.zeros(cap, dtype=THERMO_DTYPE)
            _check(load().srmd_step(self._h, int(nsteps), int(thermo_every), trace.ctypes.data_as(_vp), cap),
                   self._h)
            return trace
        _check(load().srmd_step(self._h, int(nsteps), 0, None, 0), self._h)
        return None

    # -- state
    def get_state(self):
        n = self.n
        pos = np.zeros((n, 3), np.float32)
        vel = np.zeros((n, 3), np.float32)
        img = np.zeros((n, 3), np.int32)
        frc = np.zeros((n, 3), np.float32)
        p64 = np.zeros((n, 3), np.float64)
        _check(load().srmd_get_state(self._h, _ptr(pos, _fp), _ptr(vel, _fp), _ptr(img, _ip), _ptr(frc, _fp),
                                     _ptr(p64, _dp)), self._h)
        return dict(pos=pos, vel=vel, image=img, force=frc, pos64=p64)

    def particle_terms(self):
        """Per-particle potential energy (half the pair energies) and virial (1/6 sum of
        r_ij . F_ij, from the last compute_forces call), original order."""
        pe = np.zeros(self.n, np.float32)
        w = np.zeros(self.n, np.float32)
        _check(load().srmd_get_particle_terms(self._h, _ptr(pe, _fp), _ptr(w, _fp)), self._h)
        return pe, w

    def save_state(self):
        """The full dynamic state as bytes (srmd_save_state)."""
        lib = load()
        need = ctypes.c_size_t()
        _check(lib.srmd_save_state(self._h, None, 0, ctypes.byref(need)), self._h)
        buf = ctypes.create_string_buffer(need.value)
        _check(lib.srmd_save_state(self._h, buf, need.value, ctypes.byref(need)), self._h)
        return buf.raw[:need.value]

    def load_state(self, blob):
        """Load bytes written by save_state (srmd_load_state)."""
        buf = ctypes.create_string_buffer(bytes(blob), len(blob))
        _check(load().srmd_load_state(self._h, buf, len(blob)), self._h)

    def set_state(self, pos=None, vel=None):
        pos = None if pos is None else _f32(pos).reshape(-1, 3)
        vel = None if vel is None else _f32(vel).reshape(-1, 3)
        _check(load().srmd_set_state(self._h, _ptr(pos, _fp), _ptr(vel, _fp)), self._h)

    def neighbor_pairs(self):
        lib = load()
        cnt = ctypes.c_int64()
        _check(lib.srmd_get_neighbor_pairs(self._h, None, 0, ctypes.byref(cnt)), self._h)
        pairs = np.zeros((max(cnt.value, 1), 2), np.int32)
        _check(lib.srmd_get_neighbor_pairs(self._h, _ptr(pairs, _ip), cnt.value, ctypes.byref(cnt)), self._h)
        return pairs[:cnt.value]

    def thermo(self):
        t = srmd_thermo()
        _check(load().srmd_get_thermo(self._h, ctypes.byref(t)), self._h)
        return t.as_dict()

    def stats(self):
        t = srmd_stats()
        _check(load().srmd_get_stats(self._h, ctypes.byref(t)), self._h)
        return t.as_dict()

    def profile_step_kernel(self, nsteps):
        """(sum of HIP-event intervals around the step kernel [ms], device-clock sum [ms], launches)."""
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
        _check(load().srmd_profile_step_kernel(self._h, int(nsteps), ctypes.byref(a), ctypes.byref(b),
                                               ctypes.byref(c)), self._h)
        return a.value, b.value, c.value

    def box(self):
        b = np.zeros(3)
        _check(load().srmd_get_box(self._h, _ptr(b, _dp)), self._h)
        return b


def _bcheck(status, bp=None):
    if status != SRMD_OK:
        msg = load().srmd_batch_last_error(bp)
        raise SrmdError(status, msg.decode() if msg else "")


class Batch:
    """Many systems advanced together by persistent launches (handle to srmd_batch).

    max_workgroups > 0 caps the workgroups the batch uses.  The systems stay usable on
    their own; they must outlive the batch."""

    def __init__(self, systems, max_workgroups=0):
        lib = load()
        self.systems = list(systems)
        arr = (ctypes.c_void_p * len(self.systems))(*[s._h.value for s in self.systems])
        h = ctypes.c_void_p()
        _bcheck(lib.srmd_batch_create_limited(ctypes.byref(h), arr, len(self.systems), int(max_workgroups)))
        self._h = h

    def step(self, nsteps, thermo_every=0, trace_cap=None):
        lib = load()
        if thermo_every > 0:
            cap = int(trace_cap if trace_cap is not None else (nsteps + thermo_every - 1) // thermo_every)
            trace = np.zeros((len(self.systems), cap), dtype=THERMO_DTYPE)
            _bcheck(lib.srmd_batch_step(self._h, int(nsteps), int(thermo_every), trace.ctypes.data_as(_vp), cap),
                    self._h)
            return trace
        _bcheck(lib.srmd_batch_step(self._h, int(nsteps), 0, None, 0), self._h)
        return None

    def autotune(self, steps_per_trial=200):
        """srmd_batch_autotune: returns (tp, particles per block of each replica)."""
        tp = ctypes.c_int32()
        ppb = np.zeros(len(self.systems), np.int32)
        _bcheck(load().srmd_batch_autotune(self._h, int(steps_per_trial), ctypes.byref(tp), _ptr(ppb, _ip)),
                self._h)
        return tp.value, ppb

    def close(self):
        if getattr(self, "_h", None):
            load().srmd_batch_destroy(self._h)
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter shutdown the HIP runtime may already be gone: leave the
        # memory to the process exit instead of calling into the library (the
        # check is bound at definition: module globals such as sys may already
        # be cleared when a late finaliser runs)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


EXPORTED = ["srmd_autotune", "srmd_autotune_full", "srmd_batch_autotune", "srmd_batch_create",
            "srmd_batch_create_limited", "srmd_batch_destroy", "srmd_batch_last_error", "srmd_batch_step",
            "srmd_build_neighbor_list", "srmd_compute_forces", "srmd_compute_forces_noalloc", "srmd_create",
            "srmd_destroy", "srmd_get_box", "srmd_get_launch", "srmd_get_neighbor_pairs",
            "srmd_get_particle_terms", "srmd_get_state", "srmd_get_stats", "srmd_get_thermo", "srmd_last_error",
            "srmd_load_state", "srmd_profile_step_kernel", "srmd_save_state", "srmd_set_allocator",
            "srmd_set_coulomb_sf", "srmd_set_fused_reduction", "srmd_set_integrator_nve", "srmd_set_integrator_nvt", "srmd_set_launch",
            "srmd_set_pair_lj", "srmd_set_pair_mie", "srmd_set_pair_potential", "srmd_set_persistent",
            "srmd_set_rebuild_path", "srmd_set_skin", "srmd_set_sort_interval", "srmd_set_state", "srmd_step",
            "srmd_tuning_cache_find", "srmd_tuning_cache_store", "srmd_tuning_key_of"]


def _export_c_names():
    """Module-level functions with the C names (thin pass-through to the loaded library)."""
    def make(name):
        def fn(*args):
            return getattr(load(), name)(*args)
        fn.__name__ = name
        fn.__doc__ = f"Direct call of {name} from libsrmd (see include/srmd.h)."
        return fn
    g = globals()
    for name in EXPORTED:
        g[name] = make(name)


_export_c_names()


def tuning_cache_find(path, key):
    """Look a key (dict of srmd_tuning_key fields) up in a tuned-parameter file;
    returns the stored parameters as a dict, or None."""
    k = srmd_tuning_key.from_dict(key)
    t = srmd_tuning()
    found = ctypes.c_int32()
    _check(load().srmd_tuning_cache_find(os.fsencode(path), ctypes.byref(k), ctypes.byref(t), ctypes.byref(found)))
    return t.as_dict() if found.value else None


def tuning_cache_store(path, key, tuning):
    """Append a record (key and tuned parameters, both dicts) to a tuned-parameter file."""
    k = srmd_tuning_key.from_dict(key)
    t = srmd_tuning.from_dict(tuning)
    _check(load().srmd_tuning_cache_store(os.fsencode(path), ctypes.byref(k), ctypes.byref(t)))


def lj_config(n, box, sigma, eps, rc, method, skin=0.3):
    """srmd_lj_config of a Lennard-Jones configuration (pair arrays ntypes x ntypes)."""
    sigma, eps, rc = (np.asarray(x, np.float64) for x in (sigma, eps, rc))
    nt = sigma.shape[0]
    cfg = srmd_lj_config()
    cfg.n, cfg.ntypes = int(n), nt
    cfg.method = CUTOFF[method] if isinstance(method, str) else int(method)
    for k in range(3):
        cfg.box[k] = float(box[k])
    cfg.skin = float(skin)
    for q, (a, b, c) in enumerate(zip(sigma.reshape(-1), eps.reshape(-1), rc.reshape(-1))):
        cfg.sigma[q], cfg.epsilon[q], cfg.rcut[q] = float(a), float(b), float(c)
    return cfg


def compute_forces_noalloc(cfg, d_pos, d_type, d_force, d_energy, d_status, stream=None):
    """srmd_compute_forces_noalloc on device pointers (ints); enqueued only, no sync."""
    _check(load().srmd_compute_forces_noalloc(ctypes.byref(cfg), _vp(d_pos), _vp(d_type), _vp(d_force),
                                              _vp(d_energy), _vp(d_status), None if stream is None else _vp(stream)))


def system_from_state(state, sigma, eps, rc, method, skin=0.3, precision="f32", stream=None):
    """Create a System from a workloads.State and set its pair potential and skin."""
    s = System(state.pos, state.types, state.box, vel=state.vel, mass=state.mass, ntypes=state.ntypes,
               precision=precision, stream=stream)
    s.set_skin(skin)
    s.set_pairs(sigma, eps, rc, method)
    return s
