"""ctypes binding of the HIP library ``libhfx.so`` (see include/hfx.h).

Argument marshalling only: every step of a Fock build or an SCF runs in
the library's HIP kernels.  There is no CPU fallback: importing this module
raises if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhfx.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1708_00033_amd.build` "
                      "(the HIP library is required; there is no CPU fallback)")

# torch's ROCm build carries its own HIP runtime with the same soname as the
# system one; loading torch first makes libhfx.so bind to that runtime so
# that torch tensors' device pointers and torch streams are valid in the
# library (one HIP runtime per process).
try:
    import torch  # noqa: F401
except ImportError:  # the C ABI does not need torch
    torch = None

_lib = C.CDLL(LIB_PATH)

HFX_OK = 0
HFX_ERR_INVALID_ARG = 1
HFX_ERR_OOM = 2
HFX_ERR_DEVICE = 3
HFX_ERR_NOT_CONVERGED = 4
HFX_ERR_NUMERICAL = 5
HFX_ERR_STATE = 6
STATUS_NAMES = {0: "HFX_OK", 1: "HFX_ERR_INVALID_ARG", 2: "HFX_ERR_OOM", 3: "HFX_ERR_DEVICE",
                4: "HFX_ERR_NOT_CONVERGED", 5: "HFX_ERR_NUMERICAL", 6: "HFX_ERR_STATE"}
HFX_PREC_FP64, HFX_PREC_MIXED = 0, 1
HFX_DIGEST_LDS, HFX_DIGEST_GLOBAL, HFX_DIGEST_PRIVATE, HFX_DIGEST_LDS_D = 0, 1, 2, 3
HFX_GUESS_SAD, HFX_GUESS_CORE, HFX_GUESS_LEARNED = 0, 1, 2
GUESS_NFEAT = 164
GUESS_HEAD_OUT = (225, 30, 4)

CLASS_NAMES = [f"({b}|{k})" for bi, b in enumerate(["ss", "ps", "pp", "ds", "dp", "dd"])
               for k in ["ss", "ps", "pp", "ds", "dp", "dd"][:bi + 1]]


HFX_SHELL_SP = -1


class hfx_shell(C.Structure):
    _fields_ = [("atom", C.c_int), ("l", C.c_int), ("nprim", C.c_int),
                ("exps", C.POINTER(C.c_double)), ("coefs", C.POINTER(C.c_double)),
                ("coefs_p", C.POINTER(C.c_double))]


class hfx_options(C.Structure):
    _fields_ = [("device", C.c_int), ("schwarz_tau", C.c_double), ("precision", C.c_int),
                ("fp32_tau", C.c_double), ("digest", C.c_int), ("task_quartets", C.c_int),
                ("log_level", C.c_int)]


class hfx_scf_options(C.Structure):
    _fields_ = [("max_iter", C.c_int), ("e_tol", C.c_double), ("d_rms_tol", C.c_double),
                ("diis_max", C.c_int), ("guess", C.c_int), ("D0", C.POINTER(C.c_double)),
                ("lindep", C.c_double), ("model", C.c_void_p), ("graph", C.c_int)]


class hfx_scf_result(C.Structure):
    _fields_ = [("energy", C.c_double), ("e_nuc", C.c_double), ("iterations", C.c_int),
                ("converged", C.c_int), ("guess_used", C.c_int), ("ndropped", C.c_int),
                ("t_total_s", C.c_double), ("t_fock_s", C.c_double), ("graph_segments", C.c_int)]


class hfx_fock_stats(C.Structure):
    _fields_ = [("quartets_fp64", C.c_longlong), ("quartets_fp32", C.c_longlong),
                ("integrals", C.c_longlong), ("prim_quartets", C.c_longlong), ("t_s", C.c_double)]


_ctx_p = C.c_void_p
_dp = C.POINTER(C.c_double)
_sigs = {
    "hfx_default_options": ([C.POINTER(hfx_options)], C.c_int),
    "hfx_default_scf_options": ([C.POINTER(hfx_scf_options)], C.c_int),
    "hfx_create": ([C.POINTER(hfx_options), C.POINTER(_ctx_p)], C.c_int),
    "hfx_load": ([_ctx_p, C.c_int, C.POINTER(C.c_int), _dp, C.c_int, C.POINTER(hfx_shell), C.c_int], C.c_int),
    "hfx_load_batch": ([_ctx_p, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), _dp, C.POINTER(C.c_int),
                        C.POINTER(hfx_shell), C.POINTER(C.c_int)], C.c_int),
    "hfx_batch_layout": ([_ctx_p, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                          C.POINTER(C.c_longlong), C.POINTER(C.c_longlong)], C.c_int),
    "hfx_graph_capture": ([_ctx_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "hfx_graph_launch": ([_ctx_p, C.c_void_p], C.c_int),
    "hfx_dims": ([_ctx_p, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)], C.c_int),
    "hfx_core": ([_ctx_p, _dp, _dp, _dp], C.c_int),
    "hfx_schwarz": ([_ctx_p, _dp], C.c_int),
    "hfx_build_fock": ([_ctx_p, _dp, _dp, C.POINTER(hfx_fock_stats)], C.c_int),
    "hfx_build_fock_dev": ([_ctx_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(hfx_fock_stats)], C.c_int),
    "hfx_build_2e_dev": ([_ctx_p, C.c_void_p, C.c_double, C.c_double, C.c_void_p, C.c_void_p,
                          C.POINTER(hfx_fock_stats)], C.c_int),
    "hfx_build_2e_shard_dev": ([_ctx_p, C.c_void_p, C.c_double, C.c_double, C.c_int, C.c_int, C.c_void_p,
                                C.c_void_p, C.POINTER(hfx_fock_stats)], C.c_int),
    "hfx_build_2e_noalloc_dev": ([_ctx_p, C.c_void_p, C.c_double, C.c_double, C.c_void_p, C.c_void_p,
                                  C.POINTER(hfx_fock_stats)], C.c_int),
    "hfx_build_jk_multi_dev": ([_ctx_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                C.POINTER(hfx_fock_stats)], C.c_int),
    "hfx_scf": ([_ctx_p, C.POINTER(hfx_scf_options), C.POINTER(hfx_scf_result), _dp, _dp, _dp], C.c_int),
    "hfx_batch_scf": ([_ctx_p, C.POINTER(hfx_scf_options), C.POINTER(hfx_scf_result), _dp], C.c_int),
    "hfx_configure": ([_ctx_p, C.POINTER(hfx_options)], C.c_int),
    "hfx_class_counts": ([_ctx_p, C.POINTER(C.c_longlong)], C.c_int),
    "hfx_set_class_tuning": ([_ctx_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int], C.c_int),
    "hfx_set_class_precision": ([_ctx_p, C.c_int, C.c_int], C.c_int),
    "hfx_kernel_timing": ([_ctx_p, C.c_int], C.c_int),
    "hfx_kernel_times": ([_ctx_p, _dp, C.POINTER(C.c_longlong)], C.c_int),
    "hfx_set_streams": ([_ctx_p, C.c_int], C.c_int),
    "hfx_plan_count": ([_ctx_p, C.POINTER(C.c_int)], C.c_int),
    "hfx_plan_info": ([_ctx_p, C.c_int, C.POINTER(C.c_longlong), _dp], C.c_int),
    "hfx_sad_density": ([_ctx_p, _dp], C.c_int),
    "hfx_guess_setup": ([_ctx_p, C.POINTER(C.c_int)], C.c_int),
    "hfx_guess_features": ([_ctx_p, C.POINTER(C.c_float), C.POINTER(C.c_int), _dp], C.c_int),
    "hfx_guess_features_dev": ([_ctx_p, C.POINTER(C.c_void_p)], C.c_int),
    "hfx_guess_targets_dev": ([_ctx_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "hfx_guess_assemble_dev": ([_ctx_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "hfx_guess_create": ([C.c_int, C.POINTER(C.c_void_p)], C.c_int),
    "hfx_guess_destroy": ([C.c_void_p], None),
    "hfx_guess_param_count": ([], C.c_longlong),
    "hfx_guess_set_params": ([C.c_void_p, C.POINTER(C.c_float)], C.c_int),
    "hfx_guess_get_params": ([C.c_void_p, C.POINTER(C.c_float)], C.c_int),
    "hfx_guess_get_grads": ([C.c_void_p, C.POINTER(C.c_float)], C.c_int),
    "hfx_guess_forward_dev": ([C.c_void_p, C.c_void_p, C.POINTER(C.c_int), C.c_void_p, C.c_void_p], C.c_int),
    "hfx_guess_grad_dev": ([C.c_void_p, C.c_void_p, C.POINTER(C.c_int), C.c_void_p, C.c_void_p,
                            C.POINTER(C.c_double)], C.c_int),
    "hfx_guess_adam": ([C.c_void_p, C.c_double, C.c_void_p], C.c_int),
    "hfx_guess_apply": ([_ctx_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int)], C.c_int),
    "hfx_guess_last_error": ([C.c_void_p], C.c_char_p),
    "hfx_kernel_resources": ([C.c_int, C.POINTER(C.c_longlong)], C.c_int),
    "hfx_last_error": ([_ctx_p], C.c_char_p),
    "hfx_destroy": ([_ctx_p], None),
}
for _name, (_args, _res) in _sigs.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res
    globals()[_name] = _f

EXPORTED = sorted(_sigs)


def kernel_resources(device: int = 0) -> np.ndarray:
    """Per class (21 x 3): largest per-lane scratch bytes, largest register
    count over the class's kernel variants, and the scratch budget."""
    a = np.zeros(21 * 3, dtype=np.int64)
    st = hfx_kernel_resources(device, a.ctypes.data_as(C.POINTER(C.c_longlong)))
    if st != HFX_OK:
        raise HfxError(st, "hfx_kernel_resources failed")
    return a.reshape(21, 3)


class HfxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _d(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _fill_shell(dst: hfx_shell, sh, keep: list) -> None:
    """One hfx_shell from a workloads.Shell (keeps the arrays alive in keep)."""
    ex = np.ascontiguousarray(sh.exps, dtype=np.float64)
    co = np.ascontiguousarray(sh.coefs, dtype=np.float64)
    keep += [ex, co]
    dst.atom, dst.l, dst.nprim = int(sh.atom), int(sh.l), len(ex)
    dst.exps, dst.coefs = _d(ex), _d(co)
    if int(sh.l) == HFX_SHELL_SP:
        cp = np.ascontiguousarray(sh.coefs_p, dtype=np.float64)
        keep.append(cp)
        dst.coefs_p = _d(cp)


def default_options(**kw) -> hfx_options:
    o = hfx_options()
    hfx_default_options(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def default_scf_options(**kw) -> hfx_scf_options:
    o = hfx_scf_options()
    hfx_default_scf_options(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Context:
    """One hfx_ctx (owns its device memory)."""

    def __init__(self, **opts):
        self.opt = default_options(**opts)
        p = _ctx_p()
        st = hfx_create(C.byref(self.opt), C.byref(p))
        if st != HFX_OK:
            raise HfxError(st, "hfx_create failed")
        self.ptr = p
        self.nbf = self.nocc = self.nshell = 0

    def _check(self, st: int):
        if st != HFX_OK:
            raise HfxError(st, hfx_last_error(self.ptr).decode())

    def close(self):
        if getattr(self, "ptr", None):
            hfx_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load(self, mol, charge: int = 0):
        f = mol.flat()
        shells = (hfx_shell * f["nshell"])()
        self._keep = []
        for s, sh in enumerate(mol.shells):
            _fill_shell(shells[s], sh, self._keep)
        Z = np.ascontiguousarray(f["Z"], dtype=np.int32)
        xyz = np.ascontiguousarray(f["xyz"], dtype=np.float64)
        self._check(hfx_load(self.ptr, f["natom"], Z.ctypes.data_as(C.POINTER(C.c_int)), _d(xyz), f["nshell"],
                             shells, charge))
        self.layout = None
        nbf, nocc, nsh = C.c_int(), C.c_int(), C.c_int()
        self._check(hfx_dims(self.ptr, C.byref(nbf), C.byref(nocc), C.byref(nsh)))
        self.nbf, self.nocc, self.nshell = nbf.value, nocc.value, nsh.value
        return self

    def load_batch(self, mols):
        """Load independent molecules as one batch; returns self.  Layout in
        self.layout = (nbf[], nocc[], offset[], total)."""
        nat = np.array([m.natom for m in mols], dtype=np.int32)
        nsh = np.array([m.nshell for m in mols], dtype=np.int32)
        Z = np.ascontiguousarray(np.concatenate([m.Z for m in mols]).astype(np.int32))
        xyz = np.ascontiguousarray(np.concatenate([m.xyz for m in mols]), dtype=np.float64)
        shells = (hfx_shell * int(nsh.sum()))()
        self._keep = []
        i = 0
        for m in mols:
            for sh in m.shells:
                _fill_shell(shells[i], sh, self._keep)
                i += 1
        ip = C.POINTER(C.c_int)
        self._check(hfx_load_batch(self.ptr, len(mols), nat.ctypes.data_as(ip), Z.ctypes.data_as(ip), _d(xyz),
                                   nsh.ctypes.data_as(ip), shells, None))
        nm = C.c_int()
        nbf = np.zeros(len(mols), dtype=np.int32)
        nocc = np.zeros(len(mols), dtype=np.int32)
        off = np.zeros(len(mols), dtype=np.int64)
        tot = C.c_longlong()
        self._check(hfx_batch_layout(self.ptr, C.byref(nm), nbf.ctypes.data_as(ip), nocc.ctypes.data_as(ip),
                                     off.ctypes.data_as(C.POINTER(C.c_longlong)), C.byref(tot)))
        self.layout = (nbf, nocc, off, tot.value)
        n1, n2, n3 = C.c_int(), C.c_int(), C.c_int()
        self._check(hfx_dims(self.ptr, C.byref(n1), C.byref(n2), C.byref(n3)))
        self.nbf, self.nocc, self.nshell = n1.value, n2.value, n3.value
        return self

    def graph_capture(self, dD_ptr: int, dF_ptr: int, stream: int):
        self._check(hfx_graph_capture(self.ptr, C.c_void_p(dD_ptr), C.c_void_p(dF_ptr), C.c_void_p(stream)))

    def graph_launch(self, stream: int):
        self._check(hfx_graph_launch(self.ptr, C.c_void_p(stream)))

    def configure(self, **kw):
        for k, v in kw.items():
            setattr(self.opt, k, v)
        self._check(hfx_configure(self.ptr, C.byref(self.opt)))

    def core(self):
        """S, H (n x n for one molecule; ragged 1-D for a batch) and E_nuc."""
        if getattr(self, "layout", None) is not None:
            tot = self.layout[3]
            S, H = np.zeros(tot), np.zeros(tot)
        else:
            n = self.nbf
            S, H = np.zeros((n, n)), np.zeros((n, n))
        e = C.c_double()
        self._check(hfx_core(self.ptr, _d(S), _d(H), C.byref(e)))
        return S, H, e.value

    def schwarz(self):
        Q = np.zeros((self.nshell, self.nshell))
        self._check(hfx_schwarz(self.ptr, _d(Q)))
        return Q

    def build_fock(self, D: np.ndarray):
        """F from a host D (n x n, or the ragged 1-D layout for a batch)."""
        D = np.ascontiguousarray(D, dtype=np.float64)
        F = np.zeros_like(D)
        st = hfx_fock_stats()
        self._check(hfx_build_fock(self.ptr, _d(D), _d(F), C.byref(st)))
        return F, st

    def build_fock_dev(self, dD_ptr: int, dF_ptr: int, stream: int = 0, stats: bool = False):
        st = hfx_fock_stats() if stats else None
        self._check(hfx_build_fock_dev(self.ptr, C.c_void_p(dD_ptr), C.c_void_p(dF_ptr), C.c_void_p(stream),
                                       C.byref(st) if stats else None))
        return st

    def build_2e_dev(self, dD_ptr: int, cj: float, ck: float, dG_ptr: int, stream: int = 0, stats: bool = False):
        st = hfx_fock_stats() if stats else None
        self._check(hfx_build_2e_dev(self.ptr, C.c_void_p(dD_ptr), cj, ck, C.c_void_p(dG_ptr), C.c_void_p(stream),
                                     C.byref(st) if stats else None))
        return st

    def build_2e_shard_dev(self, dD_ptr: int, cj: float, ck: float, shard: int, nshards: int, dG_ptr: int,
                           stream: int = 0, stats: bool = False):
        st = hfx_fock_stats() if stats else None
        self._check(hfx_build_2e_shard_dev(self.ptr, C.c_void_p(dD_ptr), cj, ck, shard, nshards, C.c_void_p(dG_ptr),
                                           C.c_void_p(stream), C.byref(st) if stats else None))
        return st

    def build_jk_multi_dev(self, ndens: int, dD_ptr: int, dJ_ptr: int, dK_ptr: int, stream: int = 0,
                           stats: bool = False):
        """hfx_build_jk_multi_dev: J and K of ndens consecutive densities from one pass over the integrals
        (dJ_ptr / dK_ptr may be 0)."""
        st = hfx_fock_stats() if stats else None
        self._check(hfx_build_jk_multi_dev(self.ptr, int(ndens), C.c_void_p(dD_ptr), C.c_void_p(dJ_ptr or None),
                                           C.c_void_p(dK_ptr or None), C.c_void_p(stream),
                                           C.byref(st) if stats else None))
        return st

    def build_2e_noalloc_dev(self, dD_ptr: int, cj: float, ck: float, dG_ptr: int, stream: int = 0,
                             stats: bool = False):
        """hfx_build_2e_noalloc_dev: per-build scratch in the library's fixed device array."""
        st = hfx_fock_stats() if stats else None
        self._check(hfx_build_2e_noalloc_dev(self.ptr, C.c_void_p(dD_ptr), cj, ck, C.c_void_p(dG_ptr),
                                             C.c_void_p(stream), C.byref(st) if stats else None))
        return st

    def scf(self, D0: Optional[np.ndarray] = None, want_c: bool = False, model: "GuessNet" = None, **kw):
        o = default_scf_options(**kw)
        if model is not None:
            o.model = model.ptr
            if "guess" not in kw:
                o.guess = HFX_GUESS_LEARNED
        keep = None
        if D0 is not None:
            keep = np.ascontiguousarray(D0, dtype=np.float64)
            o.D0 = _d(keep)
        n = self.nbf
        res = hfx_scf_result()
        D = np.zeros((n, n))
        Cm = np.zeros((n, n)) if want_c else None
        eps = np.zeros(n)
        st = hfx_scf(self.ptr, C.byref(o), C.byref(res), _d(D), _d(Cm) if want_c else None, _d(eps))
        if st not in (HFX_OK, HFX_ERR_NOT_CONVERGED):
            self._check(st)
        nmo = n - res.ndropped
        out = dict(energy=res.energy, e_nuc=res.e_nuc, iterations=res.iterations, converged=bool(res.converged),
                   guess_used=res.guess_used, ndropped=res.ndropped, t_total_s=res.t_total_s,
                   t_fock_s=res.t_fock_s, D=D, eps=eps[:nmo], status=st)
        if want_c:
            out["C"] = Cm.reshape(-1)[: n * nmo].reshape(n, nmo)
        return out

    # ---- learned initial guess ----
    def sad_density(self) -> np.ndarray:
        D = np.zeros((self.nbf, self.nbf))
        self._check(hfx_sad_density(self.ptr, _d(D)))
        return D

    def guess_setup(self):
        """Pair list, frames and features on the device; returns counts per
        pair type (O-O, O-H, H-H)."""
        c = (C.c_int * 3)()
        self._check(hfx_guess_setup(self.ptr, c))
        self.guess_counts = tuple(int(x) for x in c)
        return self.guess_counts

    def guess_features(self):
        """Host copies: X (npair, 164) float32, pairs (npair, 2), frames (npair, 3, 3)."""
        n = sum(self.guess_counts)
        X = np.zeros((n, GUESS_NFEAT), dtype=np.float32)
        P = np.zeros((n, 2), dtype=np.int32)
        R = np.zeros((n, 3, 3))
        self._check(hfx_guess_features(self.ptr, X.ctypes.data_as(C.POINTER(C.c_float)),
                                       P.ctypes.data_as(C.POINTER(C.c_int)), _d(R)))
        return X, P, R

    def guess_features_dev(self) -> int:
        p = C.c_void_p()
        self._check(hfx_guess_features_dev(self.ptr, C.byref(p)))
        return p.value

    def guess_packed_size(self) -> int:
        return sum(c * n for c, n in zip(self.guess_counts, GUESS_HEAD_OUT))

    def guess_targets_dev(self, dD_ptr: int, dDbase_ptr: int, dT_ptr: int, stream: int = 0):
        self._check(hfx_guess_targets_dev(self.ptr, C.c_void_p(dD_ptr), C.c_void_p(dDbase_ptr or None),
                                          C.c_void_p(dT_ptr), C.c_void_p(stream)))

    def guess_assemble_dev(self, dT_ptr: int, dDbase_ptr: int, dD_ptr: int, stream: int = 0):
        self._check(hfx_guess_assemble_dev(self.ptr, C.c_void_p(dT_ptr), C.c_void_p(dDbase_ptr or None),
                                           C.c_void_p(dD_ptr), C.c_void_p(stream)))

    def guess_apply(self, model: "GuessNet", dD_ptr: int, stream: int = 0) -> bool:
        used = C.c_int()
        self._check(hfx_guess_apply(self.ptr, model.ptr, C.c_void_p(dD_ptr), C.c_void_p(stream), C.byref(used)))
        return bool(used.value)

    def batch_scf(self, D0: Optional[np.ndarray] = None, **kw):
        """Lockstep SCF of a loaded batch: list of per-molecule dicts and the
        ragged converged densities."""
        o = default_scf_options(**kw)
        keep = None
        if D0 is not None:
            keep = np.ascontiguousarray(D0, dtype=np.float64)
            o.D0 = _d(keep)
        if self.layout is None:     # a single molecule is a batch of one
            nbf, off, tot = [self.nbf], [0], self.nbf * self.nbf
        else:
            nbf, _, off, tot = self.layout
        nmol = len(nbf)
        res = (hfx_scf_result * nmol)()
        D = np.zeros(int(tot))
        st = hfx_batch_scf(self.ptr, C.byref(o), res, _d(D))
        if st not in (HFX_OK, HFX_ERR_NOT_CONVERGED):
            self._check(st)
        out = [dict(energy=r.energy, e_nuc=r.e_nuc, iterations=r.iterations, converged=bool(r.converged),
                    guess_used=r.guess_used, ndropped=r.ndropped, t_total_s=r.t_total_s, t_fock_s=r.t_fock_s,
                    graph_segments=r.graph_segments)
               for r in res]
        return out, D

    def set_class_tuning(self, cls: int, task_quartets: int = 0, xcd_stripe: int = -1, persistent: int = 0,
                         digest: int = -1):
        """hfx_set_class_tuning: persistent 0 = one workgroup per task, 1 = resident grid with per-XCD
        queues, 2 = resident grid with one task per wave, 3 = resident grid, register-tiled (FP64)."""
        self._check(hfx_set_class_tuning(self.ptr, cls, task_quartets, xcd_stripe, persistent, digest))

    def set_class_precision(self, cls: int, fp32: int):
        self._check(hfx_set_class_precision(self.ptr, cls, fp32))

    def apply_tuning(self, table: dict):
        """table: {class index or name: {"task_quartets", "xcd_stripe", "persistent", "digest"}}"""
        for k, v in table.items():
            cid = CLASS_NAMES.index(k) if isinstance(k, str) and not k.isdigit() else int(k)
            self.set_class_tuning(cid, int(v.get("task_quartets", 0)), int(v.get("xcd_stripe", -1)),
                                  int(v.get("persistent", 0)), int(v.get("digest", -1)))

    def class_counts(self) -> np.ndarray:
        a = np.zeros(21 * 4, dtype=np.int64)
        self._check(hfx_class_counts(self.ptr, a.ctypes.data_as(C.POINTER(C.c_longlong))))
        return a.reshape(21, 4)

    def kernel_timing(self, enable: bool = True):
        self._check(hfx_kernel_timing(self.ptr, int(enable)))

    def set_streams(self, n: int):
        self._check(hfx_set_streams(self.ptr, int(n)))

    def plans(self):
        """Per launch: dict(cls, ket_nprim, tasks, quartets, prim, integrals, launches, mode, wgs,
        persistent, blocks, bras_per_task, dstage, ms)."""
        n = C.c_int()
        self._check(hfx_plan_count(self.ptr, C.byref(n)))
        out = []
        for i in range(n.value):
            info = (C.c_longlong * 13)()
            ms = C.c_double()
            self._check(hfx_plan_info(self.ptr, i, info, C.byref(ms)))
            out.append(dict(cls=int(info[0]), ket_nprim=int(info[1]), tasks=int(info[2]), quartets=int(info[3]),
                            prim=int(info[4]), integrals=int(info[5]), launches=int(info[6]), mode=int(info[7]),
                            wgs=int(info[8]), persistent=int(info[9]), blocks=int(info[10]),
                            bras_per_task=int(info[11]), dstage=int(info[12]), ms=ms.value))
        return out

    def kernel_times(self):
        ms = np.zeros(21)
        n = np.zeros(21, dtype=np.int64)
        self._check(hfx_kernel_times(self.ptr, _d(ms), n.ctypes.data_as(C.POINTER(C.c_longlong))))
        return ms, n


class GuessNet:
    """The learned-guess network (hfx_guess): parameters, BF16 MFMA forward
    and gradient, Adam.  Parameters are a packed float32 vector of
    ``param_count()`` entries (layout in include/hfx.h)."""

    def __init__(self, device: int = 0, params: Optional[np.ndarray] = None):
        self.ptr = C.c_void_p()
        st = hfx_guess_create(device, C.byref(self.ptr))
        if st != HFX_OK:
            raise HfxError(st, "hfx_guess_create failed")
        if params is not None:
            self.set_params(params)

    @staticmethod
    def param_count() -> int:
        return int(hfx_guess_param_count())

    # packed layout of include/hfx.h: (name, rows, cols)
    LAYOUT = (("W1", 256, GUESS_NFEAT), ("b1", 256, 1), ("W2", 256, 256), ("b2", 256, 1), ("W3", 256, 256),
              ("b3", 256, 1), ("H0", 225, 256), ("c0", 225, 1), ("H1", 30, 256), ("c1", 30, 1), ("H2", 4, 256),
              ("c2", 4, 1), ("fmean", GUESS_NFEAT, 1), ("fscale", GUESS_NFEAT, 1), ("tscale", 3, 1))

    @classmethod
    def init_params(cls, seed: int, fmean, fscale, tscale) -> np.ndarray:
        """Seeded start: uniform(+-sqrt(6 / fan_in)) hidden weights, heads ten
        times smaller, zero biases, and the given input / target scalers."""
        rng = np.random.default_rng(seed)
        parts = []
        for name, r, c in cls.LAYOUT:
            if name[0] in "WH":
                lim = np.sqrt(6.0 / c) * (0.1 if name[0] == "H" else 1.0)
                parts.append(rng.uniform(-lim, lim, size=r * c))
            elif name == "fmean":
                parts.append(np.asarray(fmean, float).ravel())
            elif name == "fscale":
                parts.append(np.asarray(fscale, float).ravel())
            elif name == "tscale":
                parts.append(np.asarray(tscale, float).ravel())
            else:
                parts.append(np.zeros(r * c))
        out = np.concatenate(parts).astype(np.float32)
        assert out.size == cls.param_count()
        return out

    def _check(self, st: int):
        if st != HFX_OK:
            raise HfxError(st, hfx_guess_last_error(self.ptr).decode())

    def close(self):
        if self.ptr:
            hfx_guess_destroy(self.ptr)
            self.ptr = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params: np.ndarray):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != self.param_count():
            raise ValueError(f"expected {self.param_count()} parameters, got {p.size}")
        self._check(hfx_guess_set_params(self.ptr, p.ctypes.data_as(C.POINTER(C.c_float))))

    def get_params(self) -> np.ndarray:
        p = np.zeros(self.param_count(), dtype=np.float32)
        self._check(hfx_guess_get_params(self.ptr, p.ctypes.data_as(C.POINTER(C.c_float))))
        return p

    def get_grads(self) -> np.ndarray:
        p = np.zeros(self.param_count(), dtype=np.float32)
        self._check(hfx_guess_get_grads(self.ptr, p.ctypes.data_as(C.POINTER(C.c_float))))
        return p

    def forward_dev(self, dX_ptr: int, counts, dT_ptr: int, stream: int = 0):
        c = (C.c_int * 3)(*[int(x) for x in counts])
        self._check(hfx_guess_forward_dev(self.ptr, C.c_void_p(dX_ptr), c, C.c_void_p(dT_ptr), C.c_void_p(stream)))

    def grad_dev(self, dX_ptr: int, counts, dT_ptr: int, stream: int = 0, want_loss: bool = True):
        c = (C.c_int * 3)(*[int(x) for x in counts])
        loss = C.c_double()
        self._check(hfx_guess_grad_dev(self.ptr, C.c_void_p(dX_ptr), c, C.c_void_p(dT_ptr), C.c_void_p(stream),
                                       C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def adam(self, lr: float, stream: int = 0):
        self._check(hfx_guess_adam(self.ptr, float(lr), C.c_void_p(stream)))
