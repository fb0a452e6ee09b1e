"""Python binding of libjk.so (argument marshalling only; every step runs in the library).

The library must be built (``python -m paper_2407_09700_amd.build``); importing this
module without it raises immediately -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("JK_LIB", os.path.join(_HERE, "libjk.so"))

JK_OK, JK_EINVAL, JK_EUNSUPPORTED, JK_ENOMEM, JK_EDEVICE, JK_ENODEV, JK_EOVERFLOW = 0, -1, -2, -3, -4, -5, -6
JK_FP64, JK_MIXED = 0, 1

# every symbol declared in include/jk.h
EXPORTS = ["jk_plan_create", "jk_plan_execute", "jk_plan_check", "jk_grad", "jk_one_electron", "jk_build",
           "jk_build_static", "jk_plan_destroy", "jk_plan_sizes", "jk_stats",
           "jk_profile", "jk_eri_tensor", "jk_schwarz", "jk_sph_matrix", "jk_rys_closed", "jk_rys_grid", "jk_batch_create",
           "jk_batch_offsets", "jk_batch_execute", "jk_batch_check", "jk_batch_stats", "jk_batch_graph_info", "jk_batch_destroy",
           "jk_last_error"]
JK_FLAG_PROFILE, JK_FLAG_GRAPH, JK_FLAG_TUNE, JK_FLAG_J_ONLY, JK_FLAG_K_ONLY = 1, 2, 4, 8, 16


class JKError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"jk error {code}: {msg}")
        self.code = code


class Basis(ctypes.Structure):
    _fields_ = [("nshell", ctypes.c_int), ("atom", ctypes.POINTER(ctypes.c_int)), ("l", ctypes.POINTER(ctypes.c_int)),
                ("nprim", ctypes.POINTER(ctypes.c_int)), ("prim_off", ctypes.POINTER(ctypes.c_int)),
                ("pure", ctypes.POINTER(ctypes.c_int)), ("nprim_total", ctypes.c_int),
                ("exps", ctypes.POINTER(ctypes.c_double)), ("coefs", ctypes.POINTER(ctypes.c_double))]


class Opts(ctypes.Structure):
    _fields_ = [("thresh", ctypes.c_double), ("precision", ctypes.c_int), ("fp32_cutoff", ctypes.c_double),
                ("flags", ctypes.c_int), ("tune_cache", ctypes.c_char_p), ("dmax", ctypes.c_double)]


class ProfileEntry(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("la", ctypes.c_int), ("lb", ctypes.c_int), ("lc", ctypes.c_int),
                ("ld", ctypes.c_int), ("team", ctypes.c_int), ("nroots", ctypes.c_int),
                ("quartets", ctypes.c_longlong), ("prim_quartets", ctypes.c_longlong), ("ms", ctypes.c_double),
                ("flops", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("kept_quartets", ctypes.c_longlong), ("candidate_quartets", ctypes.c_longlong),
                ("kept_fp32", ctypes.c_longlong), ("prim_quartets", ctypes.c_longlong),
                ("npairs_kept", ctypes.c_int), ("nao", ctypes.c_int), ("nao_cart", ctypes.c_int),
                ("nshell", ctypes.c_int), ("plan_ms", ctypes.c_double), ("overflow", ctypes.c_int),
                ("list_capacity", ctypes.c_longlong)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_2407_09700_amd.build")
        # PyTorch first: the library then binds to the HIP runtime PyTorch loaded (one runtime
        # per process; loaded the other way round, PyTorch found no GPU)
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.jk_plan_create.argtypes = [ctypes.POINTER(Basis), ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                                     ctypes.POINTER(Opts), ctypes.POINTER(vp)]
        L.jk_plan_execute.argtypes = [vp, vp, vp, vp, vp]
        L.jk_plan_check.argtypes = [vp]
        L.jk_grad.argtypes = [vp, vp, vp, vp]
        dpp = ctypes.POINTER(ctypes.c_double)
        L.jk_one_electron.argtypes = [ctypes.POINTER(Basis), dpp, ctypes.c_int, dpp, dpp, dpp, dpp, dpp]
        L.jk_build.argtypes = [ctypes.POINTER(Basis), ctypes.POINTER(ctypes.c_double), ctypes.c_int, vp,
                               ctypes.c_double, vp, vp, ctypes.POINTER(Opts), vp]
        L.jk_build_static.argtypes = L.jk_build.argtypes
        L.jk_plan_destroy.argtypes = [vp]
        L.jk_plan_destroy.restype = None
        L.jk_plan_sizes.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
        L.jk_stats.argtypes = [vp, ctypes.POINTER(Stats)]
        L.jk_profile.argtypes = [vp, ctypes.POINTER(ProfileEntry), ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        L.jk_eri_tensor.argtypes = [vp, vp, vp]
        L.jk_schwarz.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
        L.jk_sph_matrix.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
        L.jk_rys_closed.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]
        L.jk_rys_grid.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double)]
        L.jk_batch_create.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.POINTER(Basis)),
                                      ctypes.POINTER(ctypes.POINTER(ctypes.c_double)), ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(Opts), ctypes.POINTER(vp)]
        L.jk_batch_offsets.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_int)]
        L.jk_batch_execute.argtypes = [vp, vp, vp, vp, vp]
        L.jk_batch_check.argtypes = [vp]
        L.jk_batch_stats.argtypes = [vp, ctypes.POINTER(Stats)]
        L.jk_batch_graph_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_longlong),
                                          ctypes.POINTER(ctypes.c_int)]
        L.jk_batch_destroy.argtypes = [vp]
        L.jk_batch_destroy.restype = None
        L.jk_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def last_error() -> str:
    return lib().jk_last_error().decode()


def check(rc):
    if rc != JK_OK:
        raise JKError(rc, last_error())


def sph_matrix(l: int) -> np.ndarray:
    out = np.zeros((2 * l + 1) * (l + 1) * (l + 2) // 2)
    check(lib().jk_sph_matrix(int(l), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out.reshape(2 * l + 1, (l + 1) * (l + 2) // 2)


def rys_closed(nroots: int, T: float):
    u = np.zeros(nroots)
    w = np.zeros(nroots)
    dp = ctypes.POINTER(ctypes.c_double)
    check(lib().jk_rys_closed(int(nroots), float(T), u.ctypes.data_as(dp), w.ctypes.data_as(dp)))
    return u, w


def rys_grid(nroots: int, T: float):
    u = np.zeros(nroots)
    w = np.zeros(nroots)
    dp = ctypes.POINTER(ctypes.c_double)
    check(lib().jk_rys_grid(int(nroots), float(T), u.ctypes.data_as(dp), w.ctypes.data_as(dp)))
    return u, w


class BasisArrays:
    """Keeps the numpy arrays behind a Basis struct alive."""

    def __init__(self, shell_atom, shell_l, shell_nprim, shell_off, shell_pure, prim_exp, prim_coef):
        ip = ctypes.POINTER(ctypes.c_int)
        dp = ctypes.POINTER(ctypes.c_double)
        self.arrs = [np.ascontiguousarray(a, np.int32) for a in (shell_atom, shell_l, shell_nprim, shell_off, shell_pure)]
        self.exps = np.ascontiguousarray(prim_exp, np.float64)
        self.coefs = np.ascontiguousarray(prim_coef, np.float64)
        a = self.arrs
        self.struct = Basis(len(a[1]), a[0].ctypes.data_as(ip), a[1].ctypes.data_as(ip), a[2].ctypes.data_as(ip),
                            a[3].ctypes.data_as(ip), a[4].ctypes.data_as(ip), len(self.exps),
                            self.exps.ctypes.data_as(dp), self.coefs.ctypes.data_as(dp))

    @classmethod
    def from_molecule(cls, mol):
        return cls(mol.shell_atom, mol.shell_l, mol.shell_nprim, mol.shell_off, mol.shell_pure, mol.prim_exp,
                   mol.prim_coef)


def make_opts(thresh=1e-12, precision=JK_FP64, fp32_cutoff=1e-6, profile=False, graph=False, tune=False,
              tune_cache=None, want="jk", dmax=0.0):
    flags = (JK_FLAG_PROFILE if profile else 0) | (JK_FLAG_GRAPH if graph else 0) | (JK_FLAG_TUNE if tune else 0)
    flags |= {"jk": 0, "j": JK_FLAG_J_ONLY, "k": JK_FLAG_K_ONLY}[want]
    return Opts(float(thresh), int(precision), float(fp32_cutoff), flags,
                None if tune_cache is None else os.fsencode(tune_cache), float(dmax))


def _ptr(t):
    return ctypes.c_void_p(None if t is None else t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(stream)


def one_electron(mol, charges):
    """Overlap, kinetic and nuclear-attraction matrices (host numpy, nao x nao) and the nuclear
    repulsion energy of a molecule with the given nuclear charges (jk_one_electron)."""
    basis = BasisArrays.from_molecule(mol)
    coords = np.ascontiguousarray(mol.coords, np.float64)
    Z = np.ascontiguousarray(charges, np.float64)
    assert Z.shape == (coords.shape[0],)
    n = int(mol.nbf)
    S, T, V = (np.zeros((n, n)) for _ in range(3))
    e = ctypes.c_double()
    dp = ctypes.POINTER(ctypes.c_double)
    check(lib().jk_one_electron(ctypes.byref(basis.struct), coords.ctypes.data_as(dp), int(coords.shape[0]),
                                Z.ctypes.data_as(dp), S.ctypes.data_as(dp), T.ctypes.data_as(dp), V.ctypes.data_as(dp),
                                ctypes.byref(e)))
    return S, T, V, e.value


def build(mol, D, thresh=None, static=False, J=None, K=None, stream=None, **opts):
    """One-shot build (jk_build, or jk_build_static when static: no device allocation by the
    library). D, J, K: torch float64 CUDA tensors, nao x nao. Waits for the build."""
    import torch
    basis = BasisArrays.from_molecule(mol)
    coords = np.ascontiguousarray(mol.coords, np.float64)
    th = mol.thresh if thresh is None else thresh
    o = make_opts(th, **opts)
    if J is None:
        J = torch.empty_like(D)
    if K is None:
        K = torch.empty_like(D)
    fn = lib().jk_build_static if static else lib().jk_build
    check(fn(ctypes.byref(basis.struct), coords.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(coords.shape[0]),
             _ptr(D), float(th), _ptr(J), _ptr(K), ctypes.byref(o), _stream(stream)))
    return J, K


class Plan:
    """A J/K plan for one molecule. D, J, K are torch float64 CUDA tensors (nao x nao)."""

    def __init__(self, coords, basis: BasisArrays, thresh=1e-12, precision=JK_FP64, fp32_cutoff=1e-6, profile=False,
                 graph=False, tune=False, tune_cache=None, want="jk", dmax=0.0):
        self.basis = basis
        self.want = want
        self.coords = np.ascontiguousarray(coords, np.float64)
        self.opts = make_opts(thresh, precision, fp32_cutoff, profile, graph, tune, tune_cache, want, dmax)
        h = ctypes.c_void_p()
        check(lib().jk_plan_create(ctypes.byref(basis.struct),
                                   self.coords.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   int(self.coords.shape[0]), ctypes.byref(self.opts), ctypes.byref(h)))
        self.h = h
        nao, nc = ctypes.c_int(), ctypes.c_int()
        check(lib().jk_plan_sizes(self.h, ctypes.byref(nao), ctypes.byref(nc)))
        self.nao, self.nao_cart = nao.value, nc.value

    @classmethod
    def from_molecule(cls, mol, thresh=None, **kw):
        return cls(mol.coords, BasisArrays.from_molecule(mol), mol.thresh if thresh is None else thresh, **kw)

    def execute(self, D, J=None, K=None, stream=None):
        """Enqueue a build (returns without waiting). A J-only plan returns (J, None), a
        K-only plan (None, K)."""
        import torch
        assert D.dtype == torch.float64 and D.is_cuda and D.is_contiguous() and D.shape == (self.nao, self.nao)
        if J is None and "j" in self.want:
            J = torch.empty_like(D)
        if K is None and "k" in self.want:
            K = torch.empty_like(D)
        for t in (J, K):
            assert t is None or (t.dtype == torch.float64 and t.is_cuda and t.is_contiguous()
                                 and t.shape == (self.nao, self.nao))
        check(lib().jk_plan_execute(self.h, _ptr(D), _ptr(J), _ptr(K), _stream(stream)))
        return J, K

    def check(self):
        """Wait for the last build; raises JKError(JK_EOVERFLOW) if its work lists overflowed
        (the plan has then grown them and a new execute completes)."""
        check(lib().jk_plan_check(self.h))

    def grad(self, D, out=None, stream=None):
        """Enqueue the nuclear gradient of tr(D (J - K/2)) with D fixed; returns the natom x 3
        tensor (valid after the stream synchronises)."""
        import torch
        assert D.dtype == torch.float64 and D.is_cuda and D.is_contiguous() and D.shape == (self.nao, self.nao)
        if out is None:
            out = torch.empty((self.coords.shape[0], 3), dtype=torch.float64, device=D.device)
        assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous() and out.numel() == 3 * self.coords.shape[0]
        check(lib().jk_grad(self.h, _ptr(D), _ptr(out), _stream(stream)))
        return out

    def eri_tensor(self, stream=None):
        import torch
        n = self.nao_cart
        out = torch.empty((n, n, n, n), dtype=torch.float64, device="cuda")
        check(lib().jk_eri_tensor(self.h, _ptr(out), _stream(stream)))
        return out

    def schwarz(self):
        ns = len(self.basis.arrs[1])
        out = np.zeros((ns, ns))
        check(lib().jk_schwarz(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def stats(self):
        s = Stats()
        check(lib().jk_stats(self.h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in Stats._fields_}

    def profile(self):
        buf = (ProfileEntry * 256)()
        n = ctypes.c_int()
        check(lib().jk_profile(self.h, buf, 256, ctypes.byref(n)))
        return [{k: getattr(buf[i], k) for k, _ in ProfileEntry._fields_} for i in range(min(n.value, 256))]

    def close(self):
        if getattr(self, "h", None):
            lib().jk_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """A batched J/K build over many molecules. D, J, K are packed 1-D torch float64 CUDA
    tensors: molecule m's nao[m] x nao[m] block starts at offsets[m]."""

    def __init__(self, mols, thresh=None, precision=JK_FP64, fp32_cutoff=1e-6, profile=False, graph=False,
                 tune=False, tune_cache=None):
        self.bases = [BasisArrays.from_molecule(m) for m in mols]
        self.coords = [np.ascontiguousarray(m.coords, np.float64) for m in mols]
        th = mols[0].thresh if thresh is None else thresh
        self.opts = make_opts(th, precision, fp32_cutoff, profile, graph, tune, tune_cache)
        n = len(mols)
        bp = (ctypes.POINTER(Basis) * n)(*[ctypes.pointer(b.struct) for b in self.bases])
        cp = (ctypes.POINTER(ctypes.c_double) * n)(*[c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
                                                      for c in self.coords])
        na = (ctypes.c_int * n)(*[c.shape[0] for c in self.coords])
        h = ctypes.c_void_p()
        check(lib().jk_batch_create(n, bp, cp, na, ctypes.byref(self.opts), ctypes.byref(h)))
        self.h = h
        off = (ctypes.c_longlong * (n + 1))()
        nao = (ctypes.c_int * n)()
        check(lib().jk_batch_offsets(self.h, off, nao))
        self.offsets = np.array(off[:], dtype=np.int64)
        self.nao = np.array(nao[:], dtype=np.int64)
        self.nmol = n

    def pack(self, mats):
        import torch
        return torch.cat([torch.as_tensor(np.ascontiguousarray(m), dtype=torch.float64).reshape(-1)
                          for m in mats]).cuda()

    def unpack(self, flat):
        return [flat[self.offsets[m]:self.offsets[m + 1]].reshape(int(self.nao[m]), int(self.nao[m]))
                for m in range(self.nmol)]

    def execute(self, D, J=None, K=None, stream=None):
        import torch
        tot = int(self.offsets[-1])
        assert D.dtype == torch.float64 and D.is_cuda and D.is_contiguous() and D.numel() == tot
        if J is None:
            J = torch.empty_like(D)
        if K is None:
            K = torch.empty_like(D)
        for t in (J, K):
            assert t.dtype == torch.float64 and t.is_cuda and t.is_contiguous() and t.numel() == tot
        check(lib().jk_batch_execute(self.h, _ptr(D), _ptr(J), _ptr(K), _stream(stream)))
        return J, K

    def check(self):
        check(lib().jk_batch_check(self.h))

    def stats(self):
        s = Stats()
        check(lib().jk_batch_stats(self.h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in Stats._fields_}

    def graph_info(self):
        rec, rep, rr = ctypes.c_int(), ctypes.c_longlong(), ctypes.c_int()
        check(lib().jk_batch_graph_info(self.h, ctypes.byref(rec), ctypes.byref(rep), ctypes.byref(rr)))
        return {"recorded": bool(rec.value), "replays": rep.value, "rerecords": rr.value}

    def close(self):
        if getattr(self, "h", None):
            lib().jk_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
