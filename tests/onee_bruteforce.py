"""Brute-force one-electron integrals over unnormalised primitive Cartesian Gaussians (no
recurrence, no Boys function): every 3D integral is a product of 1D Gaussian integrals done
by Gauss-Hermite quadrature about the product centre; the Coulomb potential 1/r uses the
Gaussian transform 1/r = (2/sqrt(pi)) int_0^inf exp(-s^2 r^2) ds, the s integral by
Gauss-Legendre after the map s = t / (1 - t)."""
import numpy as np


def _comps(l):
    return [(ax, ay, l - ax - ay) for ax in range(l, -1, -1) for ay in range(l - ax, -1, -1)]


def _gh(n):
    x, w = np.polynomial.hermite.hermgauss(n)
    return x, w


def _overlap_1d(i, j, a, b, A, B, x, w, extra_p=0.0, extra_c=0.0):
    """int (x-A)^i (x-B)^j exp(-a(x-A)^2 - b(x-B)^2 - extra_p (x-extra_c)^2) dx."""
    p = a + b + extra_p
    P = (a * A + b * B + extra_p * extra_c) / p
    pref = np.exp(-(a * b * (A - B) ** 2 + a * extra_p * (A - extra_c) ** 2 + b * extra_p * (B - extra_c) ** 2) / p)
    t = P + x / np.sqrt(p)
    return pref / np.sqrt(p) * np.sum(w * (t - A) ** i * (t - B) ** j)


def primitive_blocks(la, lb, a, b, A, B, nuclei=(), charges=(), ngh=40, ns=200):
    """Cartesian S, T, V blocks of two primitives (coefficient 1)."""
    A = np.asarray(A, float)
    B = np.asarray(B, float)
    x, w = _gh(ngh)
    ca, cb = _comps(la), _comps(lb)
    S = np.zeros((len(ca), len(cb)))
    T = np.zeros_like(S)
    V = np.zeros_like(S)
    tl, wl = np.polynomial.legendre.leggauss(ns)
    tl = 0.5 * (tl + 1.0)
    wl = 0.5 * wl
    s = tl / (1.0 - tl)
    ds = 1.0 / (1.0 - tl) ** 2
    for p, ea in enumerate(ca):
        for q, eb in enumerate(cb):
            sd = [_overlap_1d(ea[d], eb[d], a, b, A[d], B[d], x, w) for d in range(3)]
            S[p, q] = np.prod(sd)
            td = []
            for d in range(3):
                j = eb[d]
                t = -2 * b * (2 * j + 1) * sd[d] + 4 * b * b * _overlap_1d(ea[d], j + 2, a, b, A[d], B[d], x, w)
                if j >= 2:
                    t += j * (j - 1) * _overlap_1d(ea[d], j - 2, a, b, A[d], B[d], x, w)
                td.append(-0.5 * t)
            T[p, q] = td[0] * sd[1] * sd[2] + sd[0] * td[1] * sd[2] + sd[0] * sd[1] * td[2]
            v = 0.0
            for C, Z in zip(nuclei, charges):
                f = np.array([np.prod([_overlap_1d(ea[d], eb[d], a, b, A[d], B[d], x, w, sk * sk, C[d])
                                       for d in range(3)]) for sk in s])
                v -= Z * 2.0 / np.sqrt(np.pi) * np.sum(wl * ds * f)
            V[p, q] = v
    return S, T, V
