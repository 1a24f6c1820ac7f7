"""ctypes binding of libhmc (include/hmc.h): argument marshalling only.

Every ``hmc_*`` function here calls the C entry point of the same name;
all work runs in the library's HIP kernels.  Device memory comes from
PyTorch tensors (passed as raw pointers) and streams from
``torch.cuda.current_stream()``.  The module refuses to run without the
built library: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhmc.so")

HMC_OK, HMC_E_ARG, HMC_E_OOM, HMC_E_HIP, HMC_E_NOCONV, HMC_E_BUSY, HMC_E_NAN = 0, -1, -2, -3, -4, -5, -6
F64, F32, F16, BF16 = 0, 1, 2, 3
KIND_HALF_SPINOR, KIND_FULL_SPINOR, KIND_GAUGE, KIND_MOMENTA = 0, 1, 2, 3
FIELDS_LOWPREC = 1
FIELD_GAUGE, FIELD_MOMENTA, FIELD_ETA, FIELD_PHI, FIELD_XE = 0, 1, 2, 3, 4
REFRESH_MOM, REFRESH_PF = 1, 2
SOURCE_GAUSS, SOURCE_Z2, SOURCE_POINT = 0, 1, 2
CG_NORMAL_MHAT, CG_WILSON_SOLVE = 0, 1

PREC_NAMES = {"f64": F64, "f32": F32, "f16": F16, "bf16": BF16}


class HmcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libhmc status {status}: {msg}")
        self.status = status


class Geom(C.Structure):
    _fields_ = [("L", C.c_int32 * 4)]


class Action(C.Structure):
    _fields_ = [("beta", C.c_double), ("kappa", C.c_double)]


class CgParams(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxiter", C.c_int32), ("mode", C.c_int32), ("prec", C.c_int32),
                ("fixed_iters", C.c_int32), ("reliable_delta", C.c_double), ("initial_guess", C.c_int32),
                ("pad", C.c_int32)]


class CgStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("reliable_updates", C.c_int32), ("rel_res", C.c_double),
                ("true_rel_res", C.c_double), ("seconds", C.c_double)]


class MdStats(C.Structure):
    _fields_ = [("solves", C.c_int32), ("iters_total", C.c_int32), ("iters_max", C.c_int32),
                ("nonconverged", C.c_int32), ("nonfinite", C.c_int32)]


class TrajParams(C.Structure):
    _fields_ = [("tau", C.c_double), ("nsteps", C.c_int32), ("n_chrono", C.c_int32), ("cg", CgParams)]


class MtsParams(C.Structure):
    _fields_ = [("tau", C.c_double), ("kappa_h", C.c_double), ("n_ratio", C.c_int32), ("n_heavy", C.c_int32),
                ("n_gauge", C.c_int32), ("pad", C.c_int32), ("cg", CgParams)]


class MtsStats(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("S1_old", "S2_old", "S1_new", "S2_new")] + \
        [(n, C.c_int32) for n in ("solves_ratio", "solves_heavy", "gauge_forces", "link_updates", "iters_ratio",
                                  "iters_heavy", "nonconverged", "nonfinite")]


class TrajResult(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("H_old", "H_new", "dH", "S_g_old", "S_g_new", "S_f_old", "S_f_new",
                                          "KE_old", "KE_new", "plaquette", "u")] + \
               [(n, C.c_int32) for n in ("accepted", "cg_iters_total", "cg_iters_max", "nonconverged")] + \
               [("seconds", C.c_double)]


class ServiceParams(C.Structure):
    _fields_ = [("arena", C.c_void_p), ("arena_bytes", C.c_size_t), ("max_batch", C.c_int32),
                ("inner_prec", C.c_int32), ("tol", C.c_double), ("maxiter", C.c_int32), ("manual", C.c_int32),
                ("chunk", C.c_int32), ("n_streams", C.c_int32), ("streams", C.c_void_p * 8),
                ("reliable_delta", C.c_double)]


class SolveRequest(C.Structure):
    _fields_ = [("L", C.c_int32 * 4), ("kappa", C.c_double), ("gauge_seed", C.c_uint64), ("gauge_eps", C.c_double),
                ("source_kind", C.c_int32), ("pad", C.c_int32), ("source_seed", C.c_uint64),
                ("source_epoch", C.c_uint64), ("out", C.c_void_p)]


class SolveResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("reliable_updates", C.c_int32),
                ("max_group", C.c_int32), ("true_rel_res", C.c_double), ("t_submit", C.c_double),
                ("t_start", C.c_double), ("t_done", C.c_double)]


class TimingEntry(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64), ("total_ms", C.c_double), ("bytes", C.c_double),
                ("calls", C.c_int64), ("bytes_moved", C.c_double)]


def struct_dict(s) -> dict:
    out = {}
    for name, _ in s._fields_:
        v = getattr(s, name)
        out[name] = struct_dict(v) if isinstance(v, C.Structure) else v
    return out


_lib = None
_P, _I32, _U32, _U64, _D = C.c_void_p, C.c_int32, C.c_uint32, C.c_uint64, C.c_double

_SIGNATURES = {
    "hmc_last_error": (C.c_char_p, []),
    "hmc_get_version": (_I32, [C.POINTER(_I32), C.POINTER(_I32)]),
    "hmc_field_bytes": (_I32, [C.POINTER(Geom), _I32, _I32, C.POINTER(C.c_size_t)]),
    "hmc_fields_bytes": (_I32, [C.POINTER(Geom), _U32, C.POINTER(C.c_size_t)]),
    "hmc_alloc_fields": (_I32, [C.POINTER(Geom), C.POINTER(Action), _U32, _P, C.c_size_t, C.POINTER(_P)]),
    "hmc_free_fields": (_I32, [_P]),
    "hmc_set_action": (_I32, [_P, C.POINTER(Action)]),
    "hmc_field_pointer": (_I32, [_P, _I32, C.POINTER(_P)]),
    "hmc_import_gauge": (_I32, [_P, _P, _P]),
    "hmc_export_gauge": (_I32, [_P, _P, _P]),
    "hmc_import_momenta": (_I32, [_P, _P, _P]),
    "hmc_export_momenta": (_I32, [_P, _P, _P]),
    "hmc_import_spinor": (_I32, [_P, _P, _P, _I32, _P]),
    "hmc_export_spinor": (_I32, [_P, _P, _P, _I32, _P]),
    "hmc_convert_spinor": (_I32, [_P, _P, _I32, _P, _I32, _P]),
    "hmc_sync_lowprec": (_I32, [_P, _P]),
    "hmc_links_two_row": (_I32, [_P, _P]),
    "hmc_stream_triad": (_I32, [_P, _P, _P, C.c_double, C.c_uint64, C.c_int32, _P]),
    "hmc_wilson_dslash": (_I32, [_P, _P, _P, _I32, _I32, _I32, _P]),
    "hmc_mhat": (_I32, [_P, _P, _P, _I32, _I32, _P]),
    "hmc_wilson_m": (_I32, [_P, _P, _P, _I32, _P]),
    "hmc_norm2": (_I32, [_P, _P, _I32, _I32, C.POINTER(_D), _P]),
    "hmc_inner": (_I32, [_P, _P, _P, _I32, C.POINTER(_D), _P]),
    "hmc_norm2_static": (_I32, [C.POINTER(Geom), _P, _I32, _I32, _P, _P]),
    "hmc_sum_multi": (_I32, [_P, _P, _I32, _P, _I32, C.POINTER(_D), _P]),
    "hmc_plaquette": (_I32, [_P, C.POINTER(_D), _P]),
    "hmc_gauge_action": (_I32, [_P, C.POINTER(_D), _P]),
    "hmc_kinetic_energy": (_I32, [_P, C.POINTER(_D), _P]),
    "hmc_gauge_force": (_I32, [_P, _D, _P]),
    "hmc_fermion_force": (_I32, [_P, _P, _D, _P]),
    "hmc_exp_update_reunit": (_I32, [_P, _D, _P]),
    "hmc_refresh": (_I32, [_P, _U64, _U64, _U32, _P]),
    "hmc_weak_field_start": (_I32, [_P, _U64, _D, _P]),
    "hmc_make_source": (_I32, [_P, _P, _I32, _U64, _U64, _P]),
    "hmc_random_words": (_I32, [_U64, _U64, _U64, _P, _I32, _I32, _P, _P]),
    "hmc_random_gaussians": (_I32, [_U64, _U64, _U64, _P, _I32, _I32, _P, _P]),
    "hmc_cg_solve": (_I32, [_P, _P, _P, C.POINTER(CgParams), C.POINTER(CgStats), _P]),
    "hmc_md_leapfrog": (_I32, [_P, _D, _I32, C.POINTER(CgParams), C.POINTER(MdStats), _P]),
    "hmc_trajectory": (_I32, [_P, _U64, _U64, C.POINTER(TrajParams), C.POINTER(TrajResult), _P]),
    "hmc_fermion_force_bilinear": (_I32, [_P, _P, _P, C.c_double, C.c_double, _P]),
    "hmc_autotune": (_I32, [_P, C.c_char_p, _P]),
    "hmc_tune_load": (_I32, [C.c_char_p, C.POINTER(C.c_int32)]),
    "hmc_tune_save": (_I32, [C.c_char_p, C.POINTER(C.c_int32)]),
    "hmc_tune_query": (_I32, [C.POINTER(C.c_int32), C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                              C.POINTER(C.c_int32)]),
    "hmc_md_mts": (_I32, [_P, _P, C.POINTER(MtsParams), C.POINTER(MtsStats), _P]),
    "hmc_trajectory_mts": (_I32, [_P, _U64, _U64, C.POINTER(MtsParams), C.POINTER(TrajResult), C.POINTER(MtsStats),
                                  _P]),
    "hmc_request_bytes": (_I32, [C.POINTER(SolveRequest), _I32, C.POINTER(C.c_size_t)]),
    "hmc_service_create": (_I32, [C.POINTER(ServiceParams), C.POINTER(_P)]),
    "hmc_service_submit": (_I32, [_P, C.POINTER(SolveRequest), C.POINTER(_U64)]),
    "hmc_service_poll": (_I32, [_P, _U64, C.POINTER(SolveResult)]),
    "hmc_service_wait": (_I32, [_P, _U64, C.POINTER(SolveResult)]),
    "hmc_service_step": (_I32, [_P, C.POINTER(_I32)]),
    "hmc_service_destroy": (_I32, [_P]),
    "hmc_timing_enable": (_I32, [_I32]),
    "hmc_timing_reset": (_I32, []),
    "hmc_timing_probe": (_I32, [_I32, _P]),
    "hmc_timing_read": (_I32, [C.POINTER(TimingEntry), _I32, C.POINTER(_I32)]),
}


# The launch-shape table measured on MI355X, loaded by lib() unless
# HMC_TUNE_DB is set (the library then reads that file; "none" loads none).
TUNE_TABLE = os.path.join(_HERE, "tune", "mi355x.txt")


def lib():
    """Load libhmc.so (raises if it has not been built) and, unless
    HMC_TUNE_DB is set, the MI355X tuning table TUNE_TABLE."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(there is no fallback implementation)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
        if os.environ.get("HMC_TUNE_DB") is None and os.path.exists(TUNE_TABLE):
            n = C.c_int32()
            check(L.hmc_tune_load(TUNE_TABLE.encode(), C.byref(n)))
    return _lib


def last_error() -> str:
    return lib().hmc_last_error().decode()


def check(status: int, allow=()) -> int:
    if status != HMC_OK and status not in allow:
        raise HmcError(status, last_error())
    return status


def _ptr(t) -> int | None:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream) -> int | None:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def geom(L) -> Geom:
    g = Geom()
    for k in range(4):
        g.L[k] = int(L[k])
    return g


# ------------------------------------------------------------------ sizes


def hmc_field_bytes(L, prec: int, kind: int) -> int:
    n = C.c_size_t()
    check(lib().hmc_field_bytes(C.byref(geom(L)), prec, kind, C.byref(n)))
    return n.value


def hmc_fields_bytes(L, flags: int = 0) -> int:
    n = C.c_size_t()
    check(lib().hmc_fields_bytes(C.byref(geom(L)), flags, C.byref(n)))
    return n.value


# ------------------------------------------------------------- fields


class Fields:
    """A fields object in a torch-allocated device arena."""

    def __init__(self, L, beta: float, kappa: float, flags: int = 0, device="cuda"):
        self.L = tuple(int(v) for v in L)
        self.V = 1
        for v in self.L:
            self.V *= v
        self.flags = flags
        self.beta, self.kappa = float(beta), float(kappa)
        nbytes = hmc_fields_bytes(self.L, flags)
        self.arena = torch.empty(nbytes, dtype=torch.uint8, device=device)
        h = C.c_void_p()
        a = Action(beta, kappa)
        check(lib().hmc_alloc_fields(C.byref(geom(self.L)), C.byref(a), flags, self.arena.data_ptr(), nbytes,
                                     C.byref(h)))
        self.handle = h

    def close(self):
        if self.handle:
            lib().hmc_free_fields(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # device buffers in the library's layouts
    def spinor(self, prec=F64, full=False, device="cuda"):
        n = hmc_field_bytes(self.L, prec, KIND_FULL_SPINOR if full else KIND_HALF_SPINOR)
        return torch.zeros(n, dtype=torch.uint8, device=device)

    def pointer(self, which: int) -> int:
        p = C.c_void_p()
        check(lib().hmc_field_pointer(self.handle, which, C.byref(p)))
        return p.value


def _h(f):
    return f.handle if isinstance(f, Fields) else f


def hmc_set_action(f, beta, kappa):
    a = Action(beta, kappa)
    check(lib().hmc_set_action(_h(f), C.byref(a)))
    if isinstance(f, Fields):
        f.beta, f.kappa = float(beta), float(kappa)


def hmc_import_gauge(f, canon, stream=None):
    check(lib().hmc_import_gauge(_h(f), _ptr(canon), _stream(stream)))


def hmc_export_gauge(f, canon, stream=None):
    check(lib().hmc_export_gauge(_h(f), _ptr(canon), _stream(stream)))


def hmc_import_momenta(f, canon, stream=None):
    check(lib().hmc_import_momenta(_h(f), _ptr(canon), _stream(stream)))


def hmc_export_momenta(f, canon, stream=None):
    check(lib().hmc_export_momenta(_h(f), _ptr(canon), _stream(stream)))


def hmc_import_spinor(f, dst, canon, parity, stream=None):
    check(lib().hmc_import_spinor(_h(f), _ptr(dst), _ptr(canon), parity, _stream(stream)))


def hmc_export_spinor(f, canon, src, parity, stream=None):
    check(lib().hmc_export_spinor(_h(f), _ptr(canon), _ptr(src), parity, _stream(stream)))


def hmc_convert_spinor(f, dst, dst_prec, src, src_prec, stream=None):
    check(lib().hmc_convert_spinor(_h(f), _ptr(dst), dst_prec, _ptr(src), src_prec, _stream(stream)))


def hmc_sync_lowprec(f, stream=None):
    check(lib().hmc_sync_lowprec(_h(f), _stream(stream)))


def hmc_stream_triad(a, b, c, s, nontemporal=False, stream=None):
    """a = b + s c over float64 device tensors of one size."""
    n = a.numel()
    assert b.numel() == n and c.numel() == n
    check(lib().hmc_stream_triad(_ptr(a), _ptr(b), _ptr(c), float(s), int(n), int(bool(nontemporal)),
                                 _stream(stream)))


def hmc_links_two_row(f) -> bool:
    on = C.c_int32()
    check(lib().hmc_links_two_row(_h(f), C.byref(on)))
    return bool(on.value)


def hmc_wilson_dslash(f, out, inp, out_parity, dagger=0, prec=F64, stream=None):
    check(lib().hmc_wilson_dslash(_h(f), _ptr(out), _ptr(inp), out_parity, int(dagger), prec, _stream(stream)))


def hmc_mhat(f, out, inp, dagger=0, prec=F64, stream=None):
    check(lib().hmc_mhat(_h(f), _ptr(out), _ptr(inp), int(dagger), prec, _stream(stream)))


def hmc_wilson_m(f, out, inp, dagger=0, stream=None):
    check(lib().hmc_wilson_m(_h(f), _ptr(out), _ptr(inp), int(dagger), _stream(stream)))


def hmc_norm2(f, x, nhalves=1, prec=F64, stream=None) -> float:
    out = C.c_double()
    check(lib().hmc_norm2(_h(f), _ptr(x), nhalves, prec, C.byref(out), _stream(stream)))
    return out.value


def hmc_norm2_static(L, x, nhalves, prec, out_dev, stream=None):
    """Asynchronous: the sum lands in the device double out_dev."""
    check(lib().hmc_norm2_static(C.byref(geom(L)), _ptr(x), nhalves, prec, _ptr(out_dev), _stream(stream)))


def hmc_inner(f, a, b, nhalves=1, stream=None) -> complex:
    out = (C.c_double * 2)()
    check(lib().hmc_inner(_h(f), _ptr(a), _ptr(b), nhalves, out, _stream(stream)))
    return complex(out[0], out[1])


def hmc_sum_multi(f, x, nhalves, subset, nsub, stream=None):
    out = (C.c_double * nsub)()
    check(lib().hmc_sum_multi(_h(f), _ptr(x), nhalves, _ptr(subset), nsub, out, _stream(stream)))
    return list(out)


def hmc_plaquette(f, stream=None) -> float:
    out = C.c_double()
    check(lib().hmc_plaquette(_h(f), C.byref(out), _stream(stream)))
    return out.value


def hmc_gauge_action(f, stream=None) -> float:
    out = C.c_double()
    check(lib().hmc_gauge_action(_h(f), C.byref(out), _stream(stream)))
    return out.value


def hmc_kinetic_energy(f, stream=None) -> float:
    out = C.c_double()
    check(lib().hmc_kinetic_energy(_h(f), C.byref(out), _stream(stream)))
    return out.value


def hmc_gauge_force(f, coef, stream=None):
    check(lib().hmc_gauge_force(_h(f), float(coef), _stream(stream)))


(TUNE_DSLASH, TUNE_GAUGE_FORCE, TUNE_DSLASH_LINKS, TUNE_GAUGE_FORCE_LINKS, TUNE_DSLASH_STREAM, TUNE_DSLASH_ORDER,
 TUNE_DSLASH_OCC) = 0, 1, 2, 3, 4, 5, 6
LINK_FULL, LINK_ROWS2, LINK_ROWCOL = 18, 12, 10


def hmc_autotune(f, db_path=None, stream=None):
    check(lib().hmc_autotune(_h(f), db_path.encode() if db_path else None, _stream(stream)))


def hmc_tune_load(path) -> int:
    n = C.c_int32()
    check(lib().hmc_tune_load(path.encode(), C.byref(n)))
    return n.value


def hmc_tune_save(path) -> int:
    n = C.c_int32()
    check(lib().hmc_tune_save(path.encode(), C.byref(n)))
    return n.value


def hmc_tune_query(L, kind, prec=F64):
    """-> (choice, tuned): the active launch shape for lattice L."""
    arr = (C.c_int32 * 4)(*[int(v) for v in L])
    ch, tu = C.c_int32(), C.c_int32()
    check(lib().hmc_tune_query(arr, int(kind), int(prec), C.byref(ch), C.byref(tu)))
    return ch.value, bool(tu.value)


def mts_params(tau, kappa_h, n_ratio, n_heavy, n_gauge, cg: CgParams):
    return MtsParams(float(tau), float(kappa_h), int(n_ratio), int(n_heavy), int(n_gauge), 0, cg)


def hmc_fermion_force_bilinear(f, X_e, Y_e, kappa_c, coef, stream=None):
    check(lib().hmc_fermion_force_bilinear(_h(f), _ptr(X_e), _ptr(Y_e), float(kappa_c), float(coef),
                                           _stream(stream)))


def hmc_md_mts(f, phi2, p: MtsParams, stream=None, allow_noconv=False):
    ms = MtsStats()
    status = lib().hmc_md_mts(_h(f), _ptr(phi2), C.byref(p), C.byref(ms), _stream(stream))
    check(status, allow=(HMC_E_NOCONV, HMC_E_NAN) if allow_noconv else ())
    d = struct_dict(ms)
    d["status"] = status
    return d


def hmc_trajectory_mts(f, seed, traj, p: MtsParams, stream=None):
    r = TrajResult()
    ms = MtsStats()
    status = lib().hmc_trajectory_mts(_h(f), seed, traj, C.byref(p), C.byref(r), C.byref(ms), _stream(stream))
    check(status, allow=(HMC_E_NOCONV, HMC_E_NAN))
    d = struct_dict(r)
    d.update(struct_dict(ms))
    d["status"] = status
    return d


def hmc_fermion_force(f, X_e, coef, stream=None):
    check(lib().hmc_fermion_force(_h(f), _ptr(X_e), float(coef), _stream(stream)))


def hmc_exp_update_reunit(f, eps, stream=None):
    check(lib().hmc_exp_update_reunit(_h(f), float(eps), _stream(stream)))


def hmc_refresh(f, seed, traj, what=REFRESH_MOM | REFRESH_PF, stream=None):
    check(lib().hmc_refresh(_h(f), seed, traj, what, _stream(stream)))


def hmc_weak_field_start(f, seed, eps, stream=None):
    check(lib().hmc_weak_field_start(_h(f), seed, float(eps), _stream(stream)))


def hmc_make_source(f, b, kind, seed, epoch, stream=None):
    check(lib().hmc_make_source(_h(f), _ptr(b), kind, seed, epoch, _stream(stream)))


def hmc_random_words(seed, rng_stream, epoch, sites, nblocks, stream=None):
    """sites: int64 cuda tensor of lexicographic sites -> uint64 words (as int64 tensor)."""
    out = torch.empty((sites.numel(), nblocks * 4), dtype=torch.int64, device=sites.device)
    check(lib().hmc_random_words(seed, rng_stream, epoch, _ptr(sites), sites.numel(), nblocks, _ptr(out),
                                 _stream(stream)))
    return out


def hmc_random_gaussians(seed, rng_stream, epoch, sites, n, stream=None):
    out = torch.empty((sites.numel(), n), dtype=torch.float64, device=sites.device)
    check(lib().hmc_random_gaussians(seed, rng_stream, epoch, _ptr(sites), sites.numel(), n, _ptr(out),
                                     _stream(stream)))
    return out


def cg_params(tol=1e-10, maxiter=10000, mode=CG_NORMAL_MHAT, prec=F64, fixed_iters=0, reliable_delta=0.0,
              initial_guess=0):
    return CgParams(tol, maxiter, mode, prec, fixed_iters, reliable_delta, initial_guess, 0)


def hmc_cg_solve(f, x, b, params: CgParams, stream=None, allow_noconv=False):
    st = CgStats()
    status = lib().hmc_cg_solve(_h(f), _ptr(x), _ptr(b), C.byref(params), C.byref(st), _stream(stream))
    check(status, allow=(HMC_E_NOCONV, HMC_E_NAN) if allow_noconv else ())
    d = struct_dict(st)
    d["status"] = status
    return d


def hmc_md_leapfrog(f, tau, nsteps, params: CgParams, stream=None, allow_noconv=False):
    st = MdStats()
    status = lib().hmc_md_leapfrog(_h(f), float(tau), int(nsteps), C.byref(params), C.byref(st), _stream(stream))
    check(status, allow=(HMC_E_NOCONV, HMC_E_NAN) if allow_noconv else ())
    d = struct_dict(st)
    d["status"] = status
    return d


def hmc_trajectory(f, seed, traj, tau, nsteps, params: CgParams, stream=None, n_chrono=0):
    tp = TrajParams(float(tau), int(nsteps), int(n_chrono), params)
    r = TrajResult()
    status = lib().hmc_trajectory(_h(f), seed, traj, C.byref(tp), C.byref(r), _stream(stream))
    check(status, allow=(HMC_E_NOCONV, HMC_E_NAN))
    d = struct_dict(r)
    d["status"] = status
    return d


def hmc_timing_enable(sample_every: int):
    check(lib().hmc_timing_enable(int(sample_every)))


def hmc_timing_probe(n: int, stream=None):
    check(lib().hmc_timing_probe(int(n), _stream(stream)))


def hmc_timing_reset():
    check(lib().hmc_timing_reset())


def hmc_timing_read() -> dict:
    n = C.c_int32()
    buf = (TimingEntry * 16)()
    check(lib().hmc_timing_read(buf, 16, C.byref(n)))
    return {buf[k].name.decode(): {"launches": buf[k].launches, "total_ms": buf[k].total_ms,
                                   "bytes": buf[k].bytes, "calls": buf[k].calls, "bytes_moved": buf[k].bytes_moved}
            for k in range(min(n.value, 16))}


# ------------------------------------------------------- solve service


def solve_request(L, kappa, gauge_seed, gauge_eps, source_kind=SOURCE_Z2, source_seed=0, source_epoch=0, out=None):
    r = SolveRequest()
    for k in range(4):
        r.L[k] = int(L[k])
    r.kappa, r.gauge_seed, r.gauge_eps = float(kappa), int(gauge_seed), float(gauge_eps)
    r.source_kind, r.source_seed, r.source_epoch = int(source_kind), int(source_seed), int(source_epoch)
    r.out = _ptr(out)
    return r


def hmc_request_bytes(req: SolveRequest, inner_prec: int) -> int:
    n = C.c_size_t()
    check(lib().hmc_request_bytes(C.byref(req), inner_prec, C.byref(n)))
    return n.value


class Service:
    """A solve service over a torch-allocated device arena, on torch streams
    (``streams``: torch.cuda.Stream objects, default n_streams new ones)."""

    def __init__(self, arena_bytes, inner_prec=F32, max_batch=64, tol=1e-10, maxiter=50000, manual=False,
                 chunk=16, device="cuda", streams=None, n_streams=8, reliable_delta=0.0):
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
        # default priority on purpose: streams of mixed priorities are not used
        self.streams = list(streams) if streams is not None else [torch.cuda.Stream(device=device)
                                                                  for _ in range(n_streams)]
        p = ServiceParams(self.arena.data_ptr(), int(arena_bytes), int(max_batch), int(inner_prec), float(tol),
                          int(maxiter), int(bool(manual)), int(chunk), len(self.streams))
        for k, s in enumerate(self.streams):
            p.streams[k] = _stream(s)
        p.reliable_delta = float(reliable_delta)
        h = C.c_void_p()
        check(lib().hmc_service_create(C.byref(p), C.byref(h)))
        self.handle = h
        self.inner_prec = inner_prec

    def submit(self, req: SolveRequest) -> int:
        t = C.c_uint64()
        check(lib().hmc_service_submit(self.handle, C.byref(req), C.byref(t)))
        return t.value

    def poll(self, ticket):
        r = SolveResult()
        st = lib().hmc_service_poll(self.handle, ticket, C.byref(r))
        if st == HMC_E_BUSY:
            return None
        check(st, allow=(HMC_E_NOCONV,))
        return struct_dict(r)

    def wait(self, ticket):
        r = SolveResult()
        check(lib().hmc_service_wait(self.handle, ticket, C.byref(r)), allow=(HMC_E_NOCONV,))
        return struct_dict(r)

    def step(self) -> int:
        n = C.c_int32()
        check(lib().hmc_service_step(self.handle, C.byref(n)))
        return n.value

    def close(self):
        if self.handle:
            lib().hmc_service_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hmc_service_create(params: ServiceParams):
    h = C.c_void_p()
    check(lib().hmc_service_create(C.byref(params), C.byref(h)))
    return h


def hmc_service_submit(svc, req):
    t = C.c_uint64()
    check(lib().hmc_service_submit(_h(svc), C.byref(req), C.byref(t)))
    return t.value


def hmc_service_poll(svc, ticket):
    r = SolveResult()
    return lib().hmc_service_poll(_h(svc), ticket, C.byref(r)), struct_dict(r)


def hmc_service_wait(svc, ticket):
    r = SolveResult()
    return lib().hmc_service_wait(_h(svc), ticket, C.byref(r)), struct_dict(r)


def hmc_service_step(svc):
    n = C.c_int32()
    check(lib().hmc_service_step(_h(svc), C.byref(n)))
    return n.value


def hmc_service_destroy(svc):
    check(lib().hmc_service_destroy(_h(svc)))


# --------------------------------------------------- canonical helpers


def to_device_c128(a, device="cuda"):
    """numpy complex128 array -> contiguous complex128 cuda tensor."""
    return torch.from_numpy(a).to(device).contiguous()


def canon_gauge_zeros(L, device="cuda"):
    V = L[0] * L[1] * L[2] * L[3]
    return torch.zeros((V, 4, 3, 3), dtype=torch.complex128, device=device)


def canon_spinor_zeros(L, device="cuda"):
    V = L[0] * L[1] * L[2] * L[3]
    return torch.zeros((V, 4, 3), dtype=torch.complex128, device=device)


# --------------------------------------------------- checkpoints


def save_checkpoint(f: Fields, path, seed: int, next_traj: int, stream=None):
    """Write a chain's state to `path` (numpy .npz, no pickled objects): the
    gauge field in the canonical layout (hmc_export_gauge) and the chain's
    position (lattice, beta, kappa, seed, next trajectory, plaquette).  The
    random numbers of a trajectory come from the counter-based generator
    keyed by (seed, trajectory), so a chain resumed from this file with
    load_checkpoint repeats the uninterrupted chain bit for bit."""
    import json

    import numpy as np
    U = canon_gauge_zeros(f.L)
    hmc_export_gauge(f, U, stream)
    torch.cuda.synchronize()
    meta = {"format": 1, "lattice": list(f.L), "beta": f.beta, "kappa": f.kappa, "seed": int(seed),
            "next_traj": int(next_traj), "plaquette": hmc_plaquette(f, stream)}
    with open(path, "wb") as fh:
        np.savez(fh, gauge=U.cpu().numpy(), meta=np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8))


def load_checkpoint(f: Fields, path, stream=None) -> dict:
    """Resume a chain saved by save_checkpoint into a fields object of the
    same lattice: sets beta and kappa, imports the gauge field and checks
    its plaquette against the saved one; returns the saved position
    (``seed``, ``next_traj``, ...).  Raises ValueError on a lattice or
    plaquette mismatch."""
    import json

    import numpy as np
    with np.load(path, allow_pickle=False) as z:
        meta = json.loads(bytes(z["meta"]).decode())
        U = z["gauge"]
    if meta.get("format") != 1 or tuple(meta["lattice"]) != f.L:
        raise ValueError(f"checkpoint of lattice {meta.get('lattice')} does not fit {f.L}")
    hmc_set_action(f, meta["beta"], meta["kappa"])
    hmc_import_gauge(f, to_device_c128(U), stream)
    p = hmc_plaquette(f, stream)
    if not abs(p - meta["plaquette"]) <= 1e-12:
        raise ValueError(f"plaquette {p!r} of the loaded field differs from the saved {meta['plaquette']!r}")
    return meta
