"""CPU oracle for the closed-shell Hartree-Fock Fock build.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  The product path never imports this
package.  The oracle shares no code with the HIP library (see
``hfx_oracle.c``: McMurchie-Davidson integrals in plain FP64 loops) and the
SCF driver in ``scf.py`` is plain numpy.

Parity status of each function is documented in ``scf.py`` / ``hfx_oracle.c``
and pinned by ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "hfx_oracle.c")

_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle (gcc, OpenMP)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp,
                               SRC_PATH, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        L.orc_basis_new.restype = C.c_void_p
        L.orc_basis_new.argtypes = [C.c_int, ip, dp, C.c_int, ip, ip, ip, ip, dp, dp]
        L.orc_basis_free.argtypes = [C.c_void_p]
        L.orc_nbf.argtypes = [C.c_void_p]
        L.orc_nbf.restype = C.c_int
        L.orc_shell_bf.argtypes = [C.c_void_p, ip]
        L.orc_boys.argtypes = [C.c_int, C.c_double, dp]
        L.orc_one_electron.argtypes = [C.c_void_p, dp, dp, dp, dp]
        L.orc_eri_shell.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, dp]
        L.orc_eri_full.argtypes = [C.c_void_p, dp]
        L.orc_schwarz.argtypes = [C.c_void_p, dp]
        L.orc_jk_brute.argtypes = [C.c_void_p, dp, C.c_double, dp, dp, dp]
        L.orc_jk_8fold.argtypes = [C.c_void_p, dp, C.c_double, dp, C.c_long, C.c_long, dp, dp,
                                   C.POINTER(C.c_longlong)]
        L.orc_jk_block.argtypes = [C.c_void_p, C.c_int, C.c_int, dp, C.c_double, dp, dp, dp]
        L.orc_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def boys(mmax: int, T: float) -> np.ndarray:
    out = np.zeros(mmax + 1)
    lib().orc_boys(mmax, float(T), _d(out))
    return out


def num_threads() -> int:
    return lib().orc_num_threads()


def _expand_sp(f):
    """An SP (L) shell (l = -1) is an s shell and a p shell on the same atom
    sharing its exponents, with the s and the p coefficients: written out as
    those two shells, s first (so its functions come as s, x, y, z)."""
    if not (f["sh_l"] == -1).any():
        return f
    atom, l, np_, off, exps, coefs = [], [], [], [], [], []
    pos = 0
    for sh in range(f["nshell"]):
        o, n = int(f["sh_off"][sh]), int(f["sh_np"][sh])
        ex = f["exps"][o:o + n]
        parts = [(0, f["coefs"][o:o + n]), (1, f["coefs_p"][o:o + n])] if f["sh_l"][sh] == -1 else \
            [(int(f["sh_l"][sh]), f["coefs"][o:o + n])]
        for (ll, co) in parts:
            atom.append(int(f["sh_atom"][sh]))
            l.append(ll)
            np_.append(n)
            off.append(pos)
            exps.append(ex)
            coefs.append(co)
            pos += n
    g = dict(f)
    g.update(nshell=len(l), sh_atom=np.array(atom, dtype=np.int32), sh_l=np.array(l, dtype=np.int32),
             sh_np=np.array(np_, dtype=np.int32), sh_off=np.array(off, dtype=np.int32),
             exps=np.ascontiguousarray(np.concatenate(exps)), coefs=np.ascontiguousarray(np.concatenate(coefs)))
    return g


class Basis:
    """A molecule's basis as the oracle sees it (owns a C-side copy).  SP
    shells are written out as an s and a p shell, so shell indices count the
    expanded shells."""

    def __init__(self, mol):
        f = _expand_sp(mol.flat())
        self._keep = f
        self.mol = mol
        self.ptr = lib().orc_basis_new(f["natom"], _i(f["Z"]), _d(f["xyz"]), f["nshell"],
                                       _i(f["sh_atom"]), _i(f["sh_l"]), _i(f["sh_np"]),
                                       _i(f["sh_off"]), _d(f["exps"]), _d(f["coefs"]))
        if not self.ptr:
            raise ValueError("oracle rejected the basis")
        self.nbf = lib().orc_nbf(self.ptr)
        self.nshell = f["nshell"]
        self.shell_bf = np.zeros(self.nshell, dtype=np.int32)
        if self.nshell:
            lib().orc_shell_bf(self.ptr, _i(self.shell_bf))
        self.shell_l = f["sh_l"].copy()
        self.shell_np = f["sh_np"].copy()
        self._Q = None

    def __del__(self):
        try:
            if self.ptr:
                lib().orc_basis_free(self.ptr)
        except Exception:
            pass

    def one_electron(self):
        n = self.nbf
        S, T, V = np.zeros((n, n)), np.zeros((n, n)), np.zeros((n, n))
        e = np.zeros(1)
        lib().orc_one_electron(self.ptr, _d(S), _d(T), _d(V), _d(e))
        return S, T, V, float(e[0])

    def eri_shell(self, a, b, c, d) -> np.ndarray:
        n = [(int(self.shell_l[s]) + 1) * (int(self.shell_l[s]) + 2) // 2 for s in (a, b, c, d)]
        out = np.zeros(n)
        lib().orc_eri_shell(self.ptr, a, b, c, d, _d(out))
        return out

    def eri_full(self) -> np.ndarray:
        n = self.nbf
        out = np.zeros((n, n, n, n))
        lib().orc_eri_full(self.ptr, _d(out))
        return out

    def schwarz(self) -> np.ndarray:
        if self._Q is None:
            Q = np.zeros((self.nshell, self.nshell))
            lib().orc_schwarz(self.ptr, _d(Q))
            self._Q = Q
        return self._Q

    def jk_brute(self, D, tau: float = 0.0):
        D = np.ascontiguousarray(D, dtype=np.float64)
        n = self.nbf
        J, K = np.zeros((n, n)), np.zeros((n, n))
        Q = self.schwarz() if tau > 0 else np.ones((self.nshell, self.nshell))
        lib().orc_jk_brute(self.ptr, _d(D), float(tau), _d(np.ascontiguousarray(Q)), _d(J), _d(K))
        return J, K

    def jk(self, D, tau: float = 1e-10, stride: int = 1, phase: int = 0):
        """8-fold-symmetric J, K; returns (J, K, stats) with stats =
        (surviving quartets, integrals, primitive quartets)."""
        D = np.ascontiguousarray(D, dtype=np.float64)
        n = self.nbf
        J, K = np.zeros((n, n)), np.zeros((n, n))
        Q = self.schwarz() if tau > 0 else np.ones((self.nshell, self.nshell))
        st = np.zeros(3, dtype=np.int64)
        lib().orc_jk_8fold(self.ptr, _d(D), float(tau), _d(np.ascontiguousarray(Q)), int(stride), int(phase),
                           _d(J), _d(K), st.ctypes.data_as(C.POINTER(C.c_longlong)))
        return J, K, tuple(int(x) for x in st)

    def jk_block(self, a: int, b: int, D, tau: float = 1e-10):
        D = np.ascontiguousarray(D, dtype=np.float64)
        na = (int(self.shell_l[a]) + 1) * (int(self.shell_l[a]) + 2) // 2
        nb = (int(self.shell_l[b]) + 1) * (int(self.shell_l[b]) + 2) // 2
        Jb, Kb = np.zeros((na, nb)), np.zeros((na, nb))
        Q = self.schwarz() if tau > 0 else np.ones((self.nshell, self.nshell))
        lib().orc_jk_block(self.ptr, a, b, _d(D), float(tau), _d(np.ascontiguousarray(Q)), _d(Jb), _d(Kb))
        return Jb, Kb

    def fock_2e(self, D, tau: float = 1e-10):
        """G(D) = 2J - K."""
        J, K, _ = self.jk(D, tau)
        return 2.0 * J - K
