"""Plain FP64 CPU oracle for the Wilson-fermion HMC hot path.

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product
library never loads it and shares no code with it.

Thin ctypes wrappers over ``oracle.c`` (plain C99, FP64, canonical layout):

* gauge / momentum fields: complex128 arrays of shape ``(V, 4, 3, 3)``,
* spinors: complex128 arrays of shape ``(V, 4, 3)``,

with the lexicographic site index ``i = x + Lx*(y + Ly*(z + Lz*t))``.  The
operations follow the HMC step list of the paper's introduction (Sec. 1);
the paper gives no formulas, so each C function documents the textbook
definition it implements.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# ORACLE_SANITIZE=1: build and load an AddressSanitizer + UBSan build of the
# oracle (the process must preload libasan; see tests/test_oracle_sanitized.py)
_SANITIZE = os.environ.get("ORACLE_SANITIZE") == "1"
_SAN_LIB = os.path.join(_HERE, "liboracle_san.so")
_SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]

GAUSSIAN, Z2, POINT = 0, 1, 2
ST_WEAKFIELD, ST_MOMENTA, ST_ETA, ST_ACCEPT, ST_SOURCE = 0, 1, 2, 3, 4


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile ``oracle.c`` with gcc into ``liboracle.so`` (in-tree); with
    sanitize, an AddressSanitizer + UBSan build ``liboracle_san.so``."""
    lib = _SAN_LIB if sanitize else _LIB
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fcx-limited-range", "-fPIC", "-shared",
               "-Wall", *(_SAN_FLAGS if sanitize else []), "-o", lib + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(lib + ".tmp", lib)
    return lib


class CgStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("rel_res", C.c_double), ("true_rel_res", C.c_double)]


class Action(C.Structure):
    _fields_ = [("beta", C.c_double), ("kappa", C.c_double), ("tol", C.c_double), ("maxiter", C.c_int)]


class MtsAction(C.Structure):
    _fields_ = [("beta", C.c_double), ("kappa", C.c_double), ("kappa_h", C.c_double), ("tol", C.c_double),
                ("maxiter", C.c_int), ("n_ratio", C.c_int), ("n_heavy", C.c_int), ("n_gauge", C.c_int)]


class MtsStats(C.Structure):
    _fields_ = [("S1_old", C.c_double), ("S2_old", C.c_double), ("S1_new", C.c_double), ("S2_new", C.c_double),
                ("solves_ratio", C.c_int), ("solves_heavy", C.c_int), ("gauge_forces", C.c_int),
                ("link_updates", C.c_int)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class MdStats(C.Structure):
    _fields_ = [("solves", C.c_int), ("iters_total", C.c_int), ("iters_max", C.c_int),
                ("nonconverged", C.c_int)]


class TrajResult(C.Structure):
    _fields_ = [(n, C.c_double) for n in
                ("H_old", "H_new", "dH", "S_g_old", "S_g_new", "S_f_old", "S_f_new", "KE_old", "KE_new",
                 "plaquette", "u")] + \
               [(n, C.c_int) for n in ("accepted", "cg_iters_total", "cg_iters_max", "nonconverged")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


_lib = None
_P = C.c_void_p
_I = C.POINTER(C.c_int)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    lib = _SAN_LIB if _SANITIZE else _LIB
    if not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
        build(force=True, sanitize=_SANITIZE)
    _lib = bind(lib)
    return _lib


def bind(path):
    """Load a compiled oracle library and declare its signatures."""
    lib = C.CDLL(path)
    sig = {
        "or_set_threads": (C.c_int, [C.c_int]),
        "or_lex_index": (C.c_long, [_I, C.c_int, C.c_int, C.c_int, C.c_int]),
        "or_site_parity": (C.c_int, [_I, C.c_long]),
        "or_neighbor_table": (None, [_I, _P]),
        "or_gamma_matrices": (None, [_P]),
        "or_dslash": (None, [_I, _P, _P, _P, C.c_int, C.c_int]),
        "or_dslash_sites": (None, [_I, _P, _P, _P, C.c_long, C.c_int, _P]),
        "or_weak_field_sites": (None, [_I, C.c_uint64, C.c_double, _P, C.c_long, _P]),
        "or_gauss_source_sites": (None, [C.c_uint64, C.c_uint64, _P, C.c_long, _P]),
        "or_wilson_m": (None, [_I, _P, C.c_double, _P, _P, C.c_int]),
        "or_mhat": (None, [_I, _P, C.c_double, _P, _P, C.c_int]),
        "or_norm2": (C.c_double, [C.c_long, _P]),
        "or_inner": (None, [C.c_long, _P, _P, _P]),
        "or_sum_multi": (None, [C.c_long, C.c_int, _P, _P, C.c_int, _P]),
        "or_plaquette": (C.c_double, [_I, _P]),
        "or_gauge_action": (C.c_double, [_I, _P, C.c_double]),
        "or_gauge_force": (None, [_I, _P, C.c_double, _P]),
        "or_eta2": (None, [_I, C.c_uint64, C.c_uint64, C.c_int, _P]),
        "or_cg_mhat_x0": (C.c_int, [_I, _P, C.c_double, _P, _P, C.c_double, C.c_int, _P]),
        "or_chrono_guess": (C.c_int, [_I, _P, C.c_double, _P, _P, C.c_int, _P]),
        "or_hmc_trajectory_chrono": (C.c_int, [_I, _P, _P, C.c_uint64, C.c_uint64, C.c_double, C.c_int, C.c_int,
                                               _P]),
        "or_mts_force": (C.c_int, [_I, _P, _P, C.c_int, _P, _P, _P]),
        "or_mts_schedule": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_double, _P, _P, C.c_int]),
        "or_mts_integrate": (C.c_int, [_I, _P, _P, _P, _P, _P, C.c_double, _P, _P, _P, _P]),
        "or_hmc_trajectory_mts": (C.c_int, [_I, _P, _P, C.c_uint64, C.c_uint64, C.c_double, _P, _P]),
        "or_ratio_action": (C.c_double, [_I, _P, _P, _P]),
        "or_gauge_force_sites": (None, [_I, _P, C.c_double, _P, C.c_long, _P]),
        "or_fermion_force_sites": (None, [_I, _P, C.c_double, _P, _P, _P, C.c_long, _P]),
        "or_fermion_force": (None, [_I, _P, C.c_double, _P, _P, _P]),
        "or_mat_exp": (None, [_P, _P]),
        "or_reunit": (None, [_P]),
        "or_update_links": (None, [_I, _P, _P, C.c_double]),
        "or_momentum_update": (None, [_I, _P, _P, C.c_double]),
        "or_kinetic": (C.c_double, [_I, _P]),
        "or_philox4x64_10": (None, [_P, _P, _P]),
        "or_u53": (C.c_double, [C.c_uint64]),
        "or_site_words": (None, [C.c_uint64, C.c_long, C.c_uint64, C.c_uint64, C.c_int, _P]),
        "or_site_gaussians": (None, [C.c_uint64, C.c_long, C.c_uint64, C.c_uint64, C.c_int, _P]),
        "or_algebra_matrix": (None, [_P, _P]),
        "or_refresh_momenta": (None, [_I, C.c_uint64, C.c_uint64, _P]),
        "or_weak_field": (None, [_I, C.c_uint64, C.c_double, _P]),
        "or_eta": (None, [_I, C.c_uint64, C.c_uint64, C.c_int, _P]),
        "or_source": (None, [_I, C.c_int, C.c_uint64, C.c_uint64, _P]),
        "or_accept_uniform": (C.c_double, [C.c_uint64, C.c_uint64]),
        "or_cg_mhat": (C.c_int, [_I, _P, C.c_double, _P, _P, C.c_double, C.c_int, C.c_int,
                                 C.POINTER(CgStats)]),
        "or_wilson_solve": (C.c_int, [_I, _P, C.c_double, _P, _P, C.c_double, C.c_int, C.POINTER(CgStats)]),
        "or_leapfrog": (C.c_int, [_I, _P, _P, _P, C.POINTER(Action), C.c_double, C.c_int, _P,
                                  C.POINTER(MdStats)]),
        "or_hmc_trajectory": (C.c_int, [_I, _P, C.POINTER(Action), C.c_uint64, C.c_uint64, C.c_double,
                                        C.c_int, C.POINTER(TrajResult)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


def compile_variant(src_text: str, path: str) -> str:
    """Compile an edited copy of oracle.c (used to check that the pins
    detect planted mistakes)."""
    src = path + ".c"
    with open(src, "w") as f:
        f.write(src_text)
    subprocess.run(["gcc", "-O1", "-std=gnu11", "-fopenmp", "-fcx-limited-range", "-fPIC", "-shared", "-w",
                    "-o", path, src, "-lm"], check=True)
    return path


def _dims(L):
    L = [int(v) for v in L]
    if len(L) != 4 or any(v < 2 or v % 2 for v in L):
        raise ValueError(f"lattice extents must be four even numbers >= 2, got {L}")
    return (C.c_int * 4)(*L)


def _ptr(a: np.ndarray):
    assert a.flags.c_contiguous
    return a.ctypes.data_as(C.c_void_p)


def set_threads(n: int) -> int:
    """Threads of the oracle's site loops; returns the previous count
    (n <= 0 only queries)."""
    return _load().or_set_threads(int(n))


def volume(L):
    return int(np.prod(L))


def gauge_zeros(L):
    return np.zeros((volume(L), 4, 3, 3), np.complex128)


def spinor_zeros(L):
    return np.zeros((volume(L), 4, 3), np.complex128)


def unit_gauge(L):
    U = gauge_zeros(L)
    U[:, :, 0, 0] = U[:, :, 1, 1] = U[:, :, 2, 2] = 1.0
    return U


def _c128(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if shape is not None and a.shape != shape:
        a = a.reshape(shape)
    return a


def parity_mask(L):
    """Boolean array over lexicographic sites: True on odd sites."""
    lib = _load()
    d = _dims(L)
    return np.array([lib.or_site_parity(d, i) for i in range(volume(L))], dtype=bool)


def lex_index(L, x, y, z, t):
    return _load().or_lex_index(_dims(L), x, y, z, t)


def neighbor_table(L):
    nb = np.zeros((volume(L), 4, 2), np.int64)
    _load().or_neighbor_table(_dims(L), _ptr(nb))
    return nb


def gamma_matrices():
    g = np.zeros((4, 4, 4), np.complex128)
    _load().or_gamma_matrices(_ptr(g))
    return g


def dslash(L, U, psi, out_parity=-1, dagger=False):
    U = _c128(U); psi = _c128(psi)
    out = spinor_zeros(L)
    _load().or_dslash(_dims(L), _ptr(U), _ptr(psi), _ptr(out), int(out_parity), int(bool(dagger)))
    return out


def dslash_sites(L, U, psi, sites, dagger=False):
    """Hopping term at the listed lexicographic sites only -> (n, 4, 3)."""
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.zeros((sites.size, 4, 3), np.complex128)
    _load().or_dslash_sites(_dims(L), _ptr(U), _ptr(psi), _ptr(sites), sites.size, int(bool(dagger)), _ptr(out))
    return out


def weak_field_sites(L, seed, eps, sites, U):
    """Fill the links of the listed sites of the full-size array U in place."""
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    assert U.flags.c_contiguous and U.dtype == np.complex128
    _load().or_weak_field_sites(_dims(L), seed, float(eps), _ptr(sites), sites.size, _ptr(U))


def gauss_source_sites(seed, epoch, sites, b):
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    assert b.flags.c_contiguous and b.dtype == np.complex128
    _load().or_gauss_source_sites(seed, epoch, _ptr(sites), sites.size, _ptr(b))


def wilson_m(L, U, kappa, psi, dagger=False):
    U = _c128(U); psi = _c128(psi)
    out = spinor_zeros(L)
    _load().or_wilson_m(_dims(L), _ptr(U), float(kappa), _ptr(psi), _ptr(out), int(bool(dagger)))
    return out


def mhat(L, U, kappa, psi, dagger=False):
    U = _c128(U); psi = _c128(psi)
    out = spinor_zeros(L)
    _load().or_mhat(_dims(L), _ptr(U), float(kappa), _ptr(psi), _ptr(out), int(bool(dagger)))
    return out


def norm2(a):
    a = _c128(a)
    return _load().or_norm2(a.size, _ptr(a))


def inner(a, b):
    a = _c128(a); b = _c128(b)
    assert a.size == b.size
    out = np.zeros(2)
    _load().or_inner(a.size, _ptr(a), _ptr(b), _ptr(out))
    return complex(out[0], out[1])


def sum_multi(f, subset, nsub):
    """f: real array (nsites, per_site); subset: int array (nsites,) in [0, nsub)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    if f.ndim == 1:
        f = f.reshape(-1, 1)
    subset = np.ascontiguousarray(subset, dtype=np.int32)
    out = np.zeros(nsub)
    _load().or_sum_multi(f.shape[0], f.shape[1], _ptr(f), _ptr(subset), int(nsub), _ptr(out))
    return out


def plaquette(L, U):
    return _load().or_plaquette(_dims(L), _ptr(_c128(U)))


def gauge_action(L, U, beta):
    return _load().or_gauge_action(_dims(L), _ptr(_c128(U)), float(beta))


def gauge_force(L, U, beta):
    F = gauge_zeros(L)
    _load().or_gauge_force(_dims(L), _ptr(_c128(U)), float(beta), _ptr(F))
    return F


def gauge_force_sites(L, U, beta, sites):
    """Gauge force at the listed lexicographic sites only -> (n, 4, 3, 3)."""
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    assert U.flags.c_contiguous and U.dtype == np.complex128
    F = np.zeros((sites.size, 4, 3, 3), np.complex128)
    _load().or_gauge_force_sites(_dims(L), _ptr(U), float(beta), _ptr(sites), sites.size, _ptr(F))
    return F


def fermion_force(L, U, coef, X, Y):
    F = gauge_zeros(L)
    _load().or_fermion_force(_dims(L), _ptr(_c128(U)), float(coef), _ptr(_c128(X)), _ptr(_c128(Y)), _ptr(F))
    return F


def fermion_force_sites(L, U, coef, X, Y, sites):
    """Fermion force at the listed lexicographic sites only -> (n, 4, 3, 3);
    X and Y full-size arrays, read at those sites and their +mu neighbours."""
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    for a in (U, X, Y):
        assert a.flags.c_contiguous and a.dtype == np.complex128
    out = np.zeros((sites.size, 4, 3, 3), np.complex128)
    _load().or_fermion_force_sites(_dims(L), _ptr(U), float(coef), _ptr(X), _ptr(Y), _ptr(sites), sites.size,
                                   _ptr(out))
    return out


def mat_exp(A):
    A = _c128(A, (3, 3))
    E = np.zeros((3, 3), np.complex128)
    _load().or_mat_exp(_ptr(A), _ptr(E))
    return E


def reunit(u):
    u = _c128(u, (3, 3)).copy()
    _load().or_reunit(_ptr(u))
    return u


def update_links(L, U, P, eps):
    U = _c128(U).copy()
    _load().or_update_links(_dims(L), _ptr(U), _ptr(_c128(P)), float(eps))
    return U


def kinetic(L, P):
    return _load().or_kinetic(_dims(L), _ptr(_c128(P)))


def philox(counter, key):
    ctr = np.array(counter, dtype=np.uint64)
    k = np.array(key, dtype=np.uint64)
    out = np.zeros(4, np.uint64)
    _load().or_philox4x64_10(_ptr(ctr), _ptr(k), _ptr(out))
    return out


def u53(w):
    return _load().or_u53(int(w))


def site_words(seed, site, stream, epoch, nblocks):
    out = np.zeros(4 * nblocks, np.uint64)
    _load().or_site_words(seed, site, stream, epoch, nblocks, _ptr(out))
    return out


def site_gaussians(seed, site, stream, epoch, n):
    out = np.zeros(n)
    _load().or_site_gaussians(seed, site, stream, epoch, n, _ptr(out))
    return out


def algebra_matrix(omega):
    om = np.ascontiguousarray(omega, dtype=np.float64)
    H = np.zeros((3, 3), np.complex128)
    _load().or_algebra_matrix(_ptr(om), _ptr(H))
    return H


def refresh_momenta(L, seed, traj):
    P = gauge_zeros(L)
    _load().or_refresh_momenta(_dims(L), seed, traj, _ptr(P))
    return P


def weak_field(L, seed, eps):
    U = gauge_zeros(L)
    _load().or_weak_field(_dims(L), seed, float(eps), _ptr(U))
    return U


def eta(L, seed, traj, parity=0):
    e = spinor_zeros(L)
    _load().or_eta(_dims(L), seed, traj, parity, _ptr(e))
    return e


def source(L, kind, seed, epoch):
    b = spinor_zeros(L)
    _load().or_source(_dims(L), int(kind), seed, epoch, _ptr(b))
    return b


def accept_uniform(seed, traj):
    return _load().or_accept_uniform(seed, traj)


def cg_mhat(L, U, kappa, b, tol=1e-10, maxiter=10000, fixed_iters=0):
    x = spinor_zeros(L)
    st = CgStats()
    status = _load().or_cg_mhat(_dims(L), _ptr(_c128(U)), float(kappa), _ptr(_c128(b)), _ptr(x), float(tol),
                                int(maxiter), int(fixed_iters), C.byref(st))
    return x, {"status": status, "iters": st.iters, "rel_res": st.rel_res, "true_rel_res": st.true_rel_res}


def wilson_solve(L, U, kappa, b, tol=1e-10, maxiter=10000):
    x = spinor_zeros(L)
    st = CgStats()
    status = _load().or_wilson_solve(_dims(L), _ptr(_c128(U)), float(kappa), _ptr(_c128(b)), _ptr(x),
                                     float(tol), int(maxiter), C.byref(st))
    return x, {"status": status, "iters": st.iters, "rel_res": st.rel_res, "true_rel_res": st.true_rel_res}


def leapfrog(L, U, P, phi, beta, kappa, tau, nsteps, tol=1e-10, maxiter=10000):
    """Returns (U, P, X_e, stats) after the PQP integration; inputs untouched."""
    U = _c128(U).copy(); P = _c128(P).copy()
    Xe = spinor_zeros(L)
    a = Action(beta, kappa, tol, maxiter)
    ms = MdStats()
    status = _load().or_leapfrog(_dims(L), _ptr(U), _ptr(P), _ptr(_c128(phi)), C.byref(a), float(tau),
                                 int(nsteps), _ptr(Xe), C.byref(ms))
    return U, P, Xe, {"status": status, "solves": ms.solves, "iters_total": ms.iters_total,
                      "iters_max": ms.iters_max, "nonconverged": ms.nonconverged}


def hmc_trajectory(L, U, beta, kappa, seed, traj, tau, nsteps, tol=1e-10, maxiter=10000):
    """One trajectory; returns (U_after, result dict).  Input U untouched."""
    U = _c128(U).copy()
    a = Action(beta, kappa, tol, maxiter)
    r = TrajResult()
    status = _load().or_hmc_trajectory(_dims(L), _ptr(U), C.byref(a), seed, traj, float(tau), int(nsteps),
                                       C.byref(r))
    d = r.as_dict()
    d["status"] = status
    return U, d


# ------------------------------------------------ mass preconditioning


def mts_action(beta, kappa, kappa_h, n_ratio, n_heavy, n_gauge, tol=1e-10, maxiter=10000):
    return MtsAction(beta, kappa, kappa_h, tol, maxiter, n_ratio, n_heavy, n_gauge)


def eta2(L, seed, traj, parity=0):
    e = spinor_zeros(L)
    _load().or_eta2(_dims(L), seed, traj, parity, _ptr(e))
    return e


def mts_force(L, U, a: MtsAction, level, phi=None):
    """Force of one monomial (0 ratio, 1 heavy, 2 gauge) -> (F, X, status)."""
    F = gauge_zeros(L)
    X = spinor_zeros(L)
    ph = _c128(phi) if phi is not None else spinor_zeros(L)
    s = _load().or_mts_force(_dims(L), _ptr(_c128(U)), C.byref(a), int(level), _ptr(ph), _ptr(X), _ptr(F))
    return F, X, s


def mts_schedule(n_ratio, n_heavy, n_gauge, tau):
    """Coalesced nested-leapfrog schedule -> (coef[s, 3], eps[s])."""
    m = n_ratio * n_heavy * n_gauge + 1
    coef = np.zeros((m, 3))
    eps = np.zeros(m)
    ns = _load().or_mts_schedule(n_ratio, n_heavy, n_gauge, float(tau), _ptr(coef), _ptr(eps), m)
    assert ns == m
    return coef, eps


def mts_integrate(L, U, P, phi1, phi2, a: MtsAction, tau):
    """Returns (U, P, X1, X2, chi, stats, status); inputs untouched."""
    U = _c128(U).copy(); P = _c128(P).copy()
    X1, X2, chi = spinor_zeros(L), spinor_zeros(L), spinor_zeros(L)
    ms = MtsStats()
    s = _load().or_mts_integrate(_dims(L), _ptr(U), _ptr(P), _ptr(_c128(phi1)), _ptr(_c128(phi2)), C.byref(a),
                                 float(tau), _ptr(X1), _ptr(X2), _ptr(chi), C.byref(ms))
    return U, P, X1, X2, chi, ms.as_dict(), s


def hmc_trajectory_mts(L, U, a: MtsAction, seed, traj, tau):
    """One mass-preconditioned trajectory -> (U_after, result dict incl. the per-monomial actions)."""
    U = _c128(U).copy()
    r = TrajResult()
    ms = MtsStats()
    status = _load().or_hmc_trajectory_mts(_dims(L), _ptr(U), C.byref(a), seed, traj, float(tau), C.byref(r),
                                           C.byref(ms))
    d = r.as_dict()
    d.update(ms.as_dict())
    d["status"] = status
    return U, d


def ratio_action(L, U, a: MtsAction, phi2):
    return _load().or_ratio_action(_dims(L), _ptr(_c128(U)), C.byref(a), _ptr(_c128(phi2)))


# ------------------------------------------------ chronological guess


def cg_mhat_x0(L, U, kappa, b, x0, tol=1e-10, maxiter=10000):
    """CG on Mhat^dag Mhat started from x0 -> (x, stats)."""
    x = _c128(x0).copy()
    st = CgStats()
    status = _load().or_cg_mhat_x0(_dims(L), _ptr(_c128(U)), float(kappa), _ptr(_c128(b)), _ptr(x), float(tol),
                                   int(maxiter), C.byref(st))
    return x, {"status": status, "iters": st.iters, "rel_res": st.rel_res, "true_rel_res": st.true_rel_res}


def chrono_guess(L, U, kappa, b, history):
    """Minimal-residual extrapolation over the solutions in `history` (oldest first)."""
    m = len(history)
    Y = np.ascontiguousarray(np.stack([_c128(h) for h in history]))
    x0 = spinor_zeros(L)
    s = _load().or_chrono_guess(_dims(L), _ptr(_c128(U)), float(kappa), _ptr(_c128(b)), _ptr(Y), m, _ptr(x0))
    return x0, s


def hmc_trajectory_chrono(L, U, beta, kappa, seed, traj, tau, nsteps, n_chrono, tol=1e-10, maxiter=10000):
    U = _c128(U).copy()
    a = Action(beta, kappa, tol, maxiter)
    r = TrajResult()
    status = _load().or_hmc_trajectory_chrono(_dims(L), _ptr(U), C.byref(a), seed, traj, float(tau), int(nsteps),
                                              int(n_chrono), C.byref(r))
    d = r.as_dict()
    d["status"] = status
    return U, d
