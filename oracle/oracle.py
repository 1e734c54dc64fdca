"""ctypes wrapper over oracle.c (plain FP64 O(N^2) reference).

TEST INFRASTRUCTURE ONLY.  See oracle.c for what each routine computes and which
passage of the paper it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "oracle.c")

TRUNC, SP, SF = 0, 1, 2
METHODS = {"trunc": TRUNC, "sp": SP, "sf": SF}

__all__ = [
    "build", "load", "TRUNC", "SP", "SF", "METHODS", "cut_tables", "pair_set", "neighbors_of",
    "forces_f32", "forces_f64", "pair", "kinetic", "max_disp2", "rebuild_needed", "integrate", "num_threads",
    "coulomb_sf", "pair_mie", "set_num_threads", "pair_potential", "POTENTIAL_KINDS",
]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, OpenMP, no FP contraction, no fast-math)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-o", tmp, SRC_PATH, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_ip = ctypes.POINTER(ctypes.c_int)


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    lib = ctypes.CDLL(LIB_PATH)
    lib.oracle_cut_tables.argtypes = [ctypes.c_int, _dp, ctypes.c_double, _fp, _fp]
    lib.oracle_cut_tables.restype = None
    lib.oracle_neighbors_of.argtypes = [ctypes.c_int, _fp, _ip, _dp, ctypes.c_int, _fp, ctypes.c_int, _ip,
                                        ctypes.c_longlong]
    lib.oracle_neighbors_of.restype = ctypes.c_longlong
    lib.oracle_pair_set.argtypes = [ctypes.c_int, _fp, _ip, _dp, ctypes.c_int, _fp, _ip, ctypes.c_longlong]
    lib.oracle_pair_set.restype = ctypes.c_longlong
    lib.oracle_pair.argtypes = [ctypes.c_double] * 4 + [ctypes.c_int, _dp, _dp]
    lib.oracle_pair.restype = None
    lib.oracle_forces_f32.argtypes = [ctypes.c_int, _fp, _ip, _dp, ctypes.c_int, _dp, _dp, _dp, ctypes.c_int,
                                      ctypes.c_int, _ip, _dp, _dp, _dp, _dp]
    lib.oracle_forces_f32.restype = None
    lib.oracle_forces_f64.argtypes = [ctypes.c_int, _dp, _ip, _dp, ctypes.c_int, _dp, _dp, _dp, ctypes.c_int,
                                      _dp, _dp, _dp, _dp]
    lib.oracle_forces_f64.restype = None
    lib.oracle_coulomb_sf.argtypes = [ctypes.c_double] * 3 + [_dp, _dp]
    lib.oracle_coulomb_sf.restype = None
    lib.oracle_pair_mie.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_int, _dp, _dp]
    lib.oracle_pair_mie.restype = None
    lib.oracle_pair_further.argtypes = [ctypes.c_double, ctypes.c_int, _dp, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_int, _dp, _dp]
    lib.oracle_pair_further.restype = None
    lib.oracle_forces_f32_g.argtypes = [ctypes.c_int, _fp, _ip, _dp, ctypes.c_int, _dp, _dp, _dp, ctypes.c_int,
                                        _dp, _dp, ctypes.c_double, ctypes.c_int, _ip, _dp, _dp, _dp, _dp]
    lib.oracle_forces_f32_g.restype = None
    lib.oracle_forces_f64_g.argtypes = [ctypes.c_int, _dp, _ip, _dp, ctypes.c_int, _dp, _dp, _dp, ctypes.c_int,
                                        _dp, _dp, ctypes.c_double, _dp, _dp, _dp, _dp]
    lib.oracle_forces_f64_g.restype = None
    lib.oracle_integrate_g.argtypes = [ctypes.c_int, _dp, _dp, _ip, _ip, _dp, _dp, ctypes.c_int, _dp, _dp, _dp,
                                       ctypes.c_int, _dp, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                       ctypes.c_double, ctypes.c_double, _dp, _dp, ctypes.c_int, _dp]
    lib.oracle_integrate_g.restype = ctypes.c_int
    lib.oracle_kinetic.argtypes = [ctypes.c_int, _dp, _ip, _dp]
    lib.oracle_kinetic.restype = ctypes.c_double
    lib.oracle_max_disp2.argtypes = [ctypes.c_int, _fp, _fp, _dp]
    lib.oracle_max_disp2.restype = ctypes.c_double
    lib.oracle_rebuild_needed.argtypes = [ctypes.c_int, _fp, _fp, _dp, ctypes.c_double]
    lib.oracle_rebuild_needed.restype = ctypes.c_int
    lib.oracle_integrate.argtypes = [ctypes.c_int, _dp, _dp, _ip, _ip, _dp, _dp, ctypes.c_int, _dp, _dp, _dp,
                                     ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_double, _dp, _dp, ctypes.c_int, _dp]
    lib.oracle_integrate.restype = ctypes.c_int
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_num_threads.restype = None
    _lib = lib
    return lib


def _c(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a


def _p(a):
    if a.dtype == np.float64:
        return a.ctypes.data_as(_dp)
    if a.dtype == np.float32:
        return a.ctypes.data_as(_fp)
    if a.dtype == np.int32:
        return a.ctypes.data_as(_ip)
    raise TypeError(a.dtype)


def _method(m):
    return METHODS[m] if isinstance(m, str) else int(m)


def cut_tables(rc, skin):
    """(cs2, rc2) float32 tables: fl32((rc_ab + s)^2) and fl32(rc_ab^2)."""
    rc = _c(rc, np.float64)
    nt = rc.shape[0]
    cs2 = np.zeros((nt, nt), np.float32)
    rc2 = np.zeros((nt, nt), np.float32)
    load().oracle_cut_tables(nt, _p(rc), float(skin), _p(cs2), _p(rc2))
    return cs2, rc2


def neighbors_of(pos, types, box, cs2, i):
    pos = _c(pos, np.float32)
    types = _c(types, np.int32)
    box = _c(box, np.float64)
    cs2 = _c(cs2, np.float32)
    n = pos.shape[0]
    lib = load()
    cnt = lib.oracle_neighbors_of(n, _p(pos), _p(types), _p(box), cs2.shape[0], _p(cs2), int(i), None, 0)
    out = np.zeros(max(cnt, 1), np.int32)
    lib.oracle_neighbors_of(n, _p(pos), _p(types), _p(box), cs2.shape[0], _p(cs2), int(i), _p(out), cnt)
    return out[:cnt]


def pair_set(pos, types, box, cs2):
    """All ordered pairs (i, j) of the list, lexicographically sorted, as an (M, 2) int32 array."""
    pos = _c(pos, np.float32)
    types = _c(types, np.int32)
    box = _c(box, np.float64)
    cs2 = _c(cs2, np.float32)
    n = pos.shape[0]
    lib = load()
    total = lib.oracle_pair_set(n, _p(pos), _p(types), _p(box), cs2.shape[0], _p(cs2), None, 0)
    pairs = np.zeros((max(total, 1), 2), np.int32)
    got = lib.oracle_pair_set(n, _p(pos), _p(types), _p(box), cs2.shape[0], _p(cs2), _p(pairs), total)
    assert got == total
    return pairs[:total]


def pair(r, sigma, eps, rc, method):
    """(u, f) of one pair at distance r; f is the radial force magnitude (positive = repulsive)."""
    u = ctypes.c_double()
    f = ctypes.c_double()
    load().oracle_pair(float(r), float(sigma), float(eps), float(rc), _method(method), ctypes.byref(u),
                       ctypes.byref(f))
    return u.value, f.value


def coulomb_sf(r, qq, rcc):
    """(u, f) of the shifted-force Coulomb term of one pair (paper section 9)."""
    u = ctypes.c_double()
    f = ctypes.c_double()
    load().oracle_coulomb_sf(float(r), float(qq), float(rcc), ctypes.byref(u), ctypes.byref(f))
    return u.value, f.value


def pair_mie(r, A, B, m, n, sigma, rc, method):
    """(u, f) of one pair of the two-power potential A (sigma/r)^m - B (sigma/r)^n."""
    u = ctypes.c_double()
    f = ctypes.c_double()
    load().oracle_pair_mie(float(r), float(A), float(B), int(m), int(n), float(sigma), float(rc), _method(method),
                           ctypes.byref(u), ctypes.byref(f))
    return u.value, f.value


# kinds of the potential block (1 the two-power potential; 2..6 the further potentials)
POTENTIAL_KINDS = {"yukawa": 2, "buckingham": 3, "gaussian": 4, "dzugutov": 5, "girifalco": 6}


def pair_potential(kind, r, params, sigma, rc, method):
    """(u, f) of one pair of a further potential (yukawa, buckingham, gaussian,
    dzugutov, girifalco) with 4 parameters (see oracle.c), f positive = repulsive."""
    u = ctypes.c_double()
    f = ctypes.c_double()
    p = np.zeros(4)
    p[:len(params)] = params
    load().oracle_pair_further(float(r), POTENTIAL_KINDS[kind], _p(p), float(sigma), float(rc), _method(method),
                               ctypes.byref(u), ctypes.byref(f))
    return u.value, f.value


def _mie(mie, ntypes, pot=None):
    """The potential block: kind, then 4 doubles per type pair.  mie = (A, B, m, n),
    each ntypes x ntypes, gives kind 1; pot = (kind name, ntypes x ntypes x 4 array)
    a further potential."""
    if pot is not None:
        kind, params = pot
        p = np.asarray(params, np.float64).reshape(ntypes * ntypes * 4)
        return np.ascontiguousarray(np.concatenate([[float(POTENTIAL_KINDS[kind])], p]))
    if mie is None:
        return None
    parts = [np.asarray(x, np.float64).reshape(ntypes, ntypes) for x in mie]
    return np.ascontiguousarray(np.concatenate([[1.0], np.stack(parts, -1).reshape(-1)]))


def _charges(charges, ntypes):
    if charges is None:
        return None
    q = _c(charges, np.float64)
    if q.shape != (ntypes,):
        raise ValueError("one charge per type")
    return q


def forces_f32(pos, types, box, sigma, eps, rc, method, sel=None, charges=None, rc_coul=0.0, mie=None, pot=None):
    """Forces (k, 3), per-particle PE (k,), per-particle virial (k,), total PE, total W on float32 positions.
    With charges (one per type), the shifted-force Coulomb term with cutoff rc_coul is added.
    With mie = (A, B, m, n) (each ntypes x ntypes), the two-power potential replaces
    Lennard-Jones (eps is then unused); with pot = (kind, ntypes x ntypes x 4 params)
    one of the further potentials does (see pair_potential)."""
    pos = _c(pos, np.float32)
    types = _c(types, np.int32)
    box = _c(box, np.float64)
    sigma = _c(sigma, np.float64)
    eps = _c(eps, np.float64)
    rc = _c(rc, np.float64)
    n = pos.shape[0]
    if sel is None:
        k = n
        selp = None
    else:
        sel = _c(sel, np.int32)
        k = sel.shape[0]
        selp = _p(sel)
    F = np.zeros((k, 3))
    pe = np.zeros(k)
    w = np.zeros(k)
    tot = np.zeros(2)
    q = _charges(charges, sigma.shape[0])
    g = _mie(mie, sigma.shape[0], pot)
    load().oracle_forces_f32_g(n, _p(pos), _p(types), _p(box), sigma.shape[0], _p(sigma), _p(eps), _p(rc),
                               _method(method), None if g is None else _p(g), None if q is None else _p(q),
                               float(rc_coul), k, selp, _p(F), _p(pe), _p(w), _p(tot))
    return F, pe, w, float(tot[0]), float(tot[1])


def forces_f64(pos, types, box, sigma, eps, rc, method, charges=None, rc_coul=0.0, mie=None, pot=None):
    pos = _c(pos, np.float64)
    types = _c(types, np.int32)
    box = _c(box, np.float64)
    sigma = _c(sigma, np.float64)
    eps = _c(eps, np.float64)
    rc = _c(rc, np.float64)
    n = pos.shape[0]
    F = np.zeros((n, 3))
    pe = np.zeros(n)
    w = np.zeros(n)
    tot = np.zeros(2)
    q = _charges(charges, sigma.shape[0])
    g = _mie(mie, sigma.shape[0], pot)
    load().oracle_forces_f64_g(n, _p(pos), _p(types), _p(box), sigma.shape[0], _p(sigma), _p(eps), _p(rc),
                               _method(method), None if g is None else _p(g), None if q is None else _p(q),
                               float(rc_coul), _p(F), _p(pe), _p(w), _p(tot))
    return F, pe, w, float(tot[0]), float(tot[1])


def kinetic(vel, types, mass):
    vel = _c(vel, np.float64)
    types = _c(types, np.int32)
    mass = _c(mass, np.float64)
    return float(load().oracle_kinetic(vel.shape[0], _p(vel), _p(types), _p(mass)))


def max_disp2(pos, pos0, box):
    pos = _c(pos, np.float32)
    pos0 = _c(pos0, np.float32)
    box = _c(box, np.float64)
    return float(load().oracle_max_disp2(pos.shape[0], _p(pos), _p(pos0), _p(box)))


def rebuild_needed(pos, pos0, box, skin):
    pos = _c(pos, np.float32)
    pos0 = _c(pos0, np.float32)
    box = _c(box, np.float64)
    return bool(load().oracle_rebuild_needed(pos.shape[0], _p(pos), _p(pos0), _p(box), float(skin)))


THERMO_FIELDS = ("pe", "ke", "virial", "temperature", "pressure", "xi", "xi_integral", "h", "ke_half")


def integrate(pos, vel, types, mass, box, sigma, eps, rc, method, dt, nsteps, thermostat=False, T0=1.0,
              tau=None, xi=0.0, xi_int=0.0, image=None, charges=None, rc_coul=0.0, mie=None, pot=None):
    """Run nsteps of leapfrog (NVE) or Nose-Hoover leapfrog (NVT) in FP64.

    Returns dict(pos, vel, image, xi, xi_int, thermo) with thermo an (nsteps, 9) array whose
    columns are THERMO_FIELDS (row n = integer step n, before the step's position update).
    """
    pos = np.array(pos, dtype=np.float64, order="C")
    vel = np.array(vel, dtype=np.float64, order="C")
    n = pos.shape[0]
    image = np.zeros((n, 3), np.int32) if image is None else np.array(image, dtype=np.int32, order="C")
    types = _c(types, np.int32)
    mass = _c(mass, np.float64)
    box = _c(box, np.float64)
    sigma = _c(sigma, np.float64)
    eps = _c(eps, np.float64)
    rc = _c(rc, np.float64)
    inv_tau2 = 0.0 if (tau is None or not np.isfinite(tau)) else 1.0 / (tau * tau)
    xi_c = ctypes.c_double(xi)
    xi_i = ctypes.c_double(xi_int)
    thermo = np.zeros((nsteps, 9))
    q = _charges(charges, sigma.shape[0])
    g = _mie(mie, sigma.shape[0], pot)
    rc_ = load().oracle_integrate_g(n, _p(pos), _p(vel), _p(image), _p(types), _p(mass), _p(box), sigma.shape[0],
                                    _p(sigma), _p(eps), _p(rc), _method(method), None if g is None else _p(g),
                                    None if q is None else _p(q), float(rc_coul), float(dt), int(bool(thermostat)), float(T0), float(inv_tau2),
                                    ctypes.byref(xi_c), ctypes.byref(xi_i), int(nsteps), _p(thermo))
    if rc_ != 0:
        raise MemoryError("oracle_integrate failed")
    return dict(pos=pos, vel=vel, image=image, xi=xi_c.value, xi_int=xi_i.value, thermo=thermo)


def num_threads():
    """Threads the oracle's OpenMP loops use."""
    return int(load().oracle_num_threads())


def set_num_threads(k):
    """Threads of the oracle's later OpenMP loops (results do not depend on it)."""
    load().oracle_set_num_threads(int(k))
