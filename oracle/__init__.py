"""CPU oracle for the J/K build -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may import
this package. The product path (paper_2407_09700_amd) never imports it, and it imports
nothing from the product path. Inputs are plain numpy arrays in the layout documented
in paper_2407_09700_amd/synth.py (which draws inputs and holds no J/K arithmetic).

The C library (jk_oracle.c) computes contracted ERIs with the Obara-Saika vertical and
Head-Gordon-Pople horizontal recurrences over the Boys function, and J/K with explicit
loops. Spherical functions use the numerically fitted matrices of oracle/sph.py.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import sph

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libjk_oracle.so")
_SRC = os.path.join(_HERE, "jk_oracle.c")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP). Returns the library path."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               "-D_DEFAULT_SOURCE", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        basis = [dp, ctypes.c_int, ip, ip, ip, ip, ip, dp, dp, dp]
        L.oracle_boys.argtypes = [ctypes.c_int, ctypes.c_double, dp]
        L.oracle_boys.restype = None
        L.oracle_eri_block.argtypes = basis + [ctypes.c_int] * 4 + [dp]
        L.oracle_schwarz.argtypes = basis + [dp]
        L.oracle_eri_tensor.argtypes = basis + [dp]
        L.oracle_jk.argtypes = basis + [dp, ctypes.c_double, dp, dp, ctypes.c_int]
        L.oracle_jk.restype = ctypes.c_longlong
        L.oracle_jk_want.argtypes = basis + [dp, ctypes.c_double, dp, dp, ctypes.c_int, ctypes.c_int]
        L.oracle_jk_want.restype = ctypes.c_longlong
        L.oracle_jk_block.argtypes = basis + [dp, ctypes.c_double, dp, dp, ctypes.c_int, ctypes.c_int,
                                              dp, dp, ctypes.c_int]
        L.oracle_screen_tables.argtypes = basis + [dp, dp, dp]
        L.oracle_jk_sample.argtypes = basis + [dp, ctypes.c_double, ctypes.c_longlong, ctypes.c_longlong, ctypes.c_int]
        L.oracle_jk_sample.restype = ctypes.c_longlong
        L.oracle_grad.argtypes = [dp, ctypes.c_int, ctypes.c_int, ip, ip, ip, ip, ip, dp, dp, dp, dp, ctypes.c_double,
                                  dp, ctypes.c_int]
        L.oracle_grad.restype = ctypes.c_longlong
        L.oracle_one_electron.argtypes = [dp, ctypes.c_int, ctypes.c_int, ip, ip, ip, ip, ip, dp, dp, dp, dp, dp, dp,
                                          dp, dp]
        L.oracle_count_kept.argtypes = [ctypes.c_int, dp, dp, ctypes.c_double]
        L.oracle_count_kept.restype = ctypes.c_longlong
        L.oracle_count_kept_want.argtypes = [ctypes.c_int, dp, dp, ctypes.c_double, ctypes.c_int]
        L.oracle_count_kept_want.restype = ctypes.c_longlong
        _lib = L
    return _lib


def _p(a, t=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(t))


def boys(mmax: int, T: float) -> np.ndarray:
    out = np.zeros(mmax + 1)
    lib().oracle_boys(int(mmax), float(T), _p(out))
    return out


def ncart(l):
    return (l + 1) * (l + 2) // 2


def nfunc(l, pure):
    return 2 * l + 1 if (pure and l >= 2) else ncart(l)


class Oracle:
    """Oracle bound to one molecule (any object with the synth.Molecule fields)."""

    def __init__(self, mol):
        self.mol = mol
        self.coords = np.ascontiguousarray(mol.coords, np.float64)
        self.sa = np.ascontiguousarray(mol.shell_atom, np.int32)
        self.sl = np.ascontiguousarray(mol.shell_l, np.int32)
        self.sn = np.ascontiguousarray(mol.shell_nprim, np.int32)
        self.so = np.ascontiguousarray(mol.shell_off, np.int32)
        self.sp = np.ascontiguousarray(mol.shell_pure, np.int32)
        self.pe = np.ascontiguousarray(mol.prim_exp, np.float64)
        self.pc = np.ascontiguousarray(mol.prim_coef, np.float64)
        self.ts = np.ascontiguousarray(sph.tsph_packed(), np.float64)
        self.ns = int(self.sl.shape[0])
        sizes = [nfunc(int(l), int(p)) for l, p in zip(self.sl, self.sp)]
        self.off = np.concatenate([[0], np.cumsum(sizes)]).astype(int)
        self.nbf = int(self.off[-1])

    def _b(self):
        i = ctypes.c_int
        return [_p(self.coords), self.ns, _p(self.sa, i), _p(self.sl, i), _p(self.sn, i), _p(self.so, i),
                _p(self.sp, i), _p(self.pe), _p(self.pc), _p(self.ts)]

    def size(self, s):
        return int(self.off[s + 1] - self.off[s])

    def eri_block(self, i, j, k, l):
        out = np.zeros(self.size(i) * self.size(j) * self.size(k) * self.size(l))
        lib().oracle_eri_block(*self._b(), int(i), int(j), int(k), int(l), _p(out))
        return out.reshape(self.size(i), self.size(j), self.size(k), self.size(l))

    def eri_tensor(self):
        n = self.nbf
        t = np.zeros((n, n, n, n))
        lib().oracle_eri_tensor(*self._b(), _p(t))
        return t

    def schwarz(self):
        out = np.zeros((self.ns, self.ns))
        lib().oracle_schwarz(*self._b(), _p(out))
        return out

    def screen_tables(self, D=None):
        D = np.ascontiguousarray(self.mol.D if D is None else D, np.float64)
        I = np.zeros((self.ns, self.ns))
        P = np.zeros((self.ns, self.ns))
        lib().oracle_screen_tables(*self._b(), _p(D), _p(I), _p(P))
        return I, P

    def jk(self, D=None, tau=None, nthreads=0, want="jk"):
        """J and K over the quartets the density-weighted screen keeps for the outputs `want`
        ("jk", "j" or "k": which density blocks enter the screen)."""
        D = np.ascontiguousarray(self.mol.D if D is None else D, np.float64)
        tau = float(self.mol.thresh if tau is None else tau)
        J = np.zeros((self.nbf, self.nbf))
        K = np.zeros((self.nbf, self.nbf))
        w = {"jk": 3, "j": 1, "k": 2}[want]
        kept = lib().oracle_jk_want(*self._b(), _p(D), tau, _p(J), _p(K), int(nthreads), w)
        self.kept = int(kept)
        return J, K

    def jk_block(self, si, sj, D=None, tau=None, I=None, P=None, nthreads=0):
        D = np.ascontiguousarray(self.mol.D if D is None else D, np.float64)
        tau = float(self.mol.thresh if tau is None else tau)
        Jb = np.zeros((self.size(si), self.size(sj)))
        Kb = np.zeros((self.size(si), self.size(sj)))
        Ip = None if I is None else _p(np.ascontiguousarray(I, np.float64))
        Pp = None if P is None else _p(np.ascontiguousarray(P, np.float64))
        lib().oracle_jk_block(*self._b(), _p(D), tau, Ip, Pp, int(si), int(sj), _p(Jb), _p(Kb), int(nthreads))
        return Jb, Kb

    def jk_sample(self, stride, offset=0, D=None, tau=None, nthreads=0):
        """Run the full J/K loop on the unique quartets of every stride-th bra pair;
        returns the number of kept quartets processed (for timing)."""
        D = np.ascontiguousarray(self.mol.D if D is None else D, np.float64)
        tau = float(self.mol.thresh if tau is None else tau)
        return int(lib().oracle_jk_sample(*self._b(), _p(D), tau, int(stride), int(offset), int(nthreads)))

    def grad(self, D=None, tau=None, nthreads=0):
        """d/dR of E = tr(D (J - K/2)) with D held fixed, natom x 3 (shells up to l = 3)."""
        D = np.ascontiguousarray(self.mol.D if D is None else D, np.float64)
        tau = float(self.mol.thresh if tau is None else tau)
        natom = int(self.coords.shape[0])
        g = np.zeros((natom, 3))
        b = self._b()
        kept = lib().oracle_grad(b[0], natom, *b[1:], _p(D), tau, _p(g), int(nthreads))
        if kept < 0:
            raise ValueError("oracle gradient: shells up to l = 3 only")
        self.kept = int(kept)
        return g

    def one_electron(self, charges):
        """Overlap, kinetic and nuclear-attraction matrices and the nuclear repulsion."""
        Z = np.ascontiguousarray(charges, np.float64)
        n = self.nbf
        S, T, V = (np.zeros((n, n)) for _ in range(3))
        e = np.zeros(1)
        b = self._b()
        lib().oracle_one_electron(b[0], int(self.coords.shape[0]), *b[1:], _p(Z), _p(S), _p(T), _p(V), _p(e))
        return S, T, V, float(e[0])

    def count_kept(self, I, P, tau, want="jk"):
        I = np.ascontiguousarray(I, np.float64)
        P = np.ascontiguousarray(P, np.float64)
        w = {"jk": 3, "j": 1, "k": 2}[want]
        return int(lib().oracle_count_kept_want(self.ns, _p(I), _p(P), float(tau), w))
