"""Brute-force numerical ERIs for primitive Cartesian Gaussians (test pin, no recurrences).

Uses the Gaussian transform 1/r12 = (2/sqrt(pi)) * int_0^inf exp(-u^2 r12^2) du. For a
fixed u the six-dimensional integrand factorises into three two-dimensional integrals,
one per Cartesian direction, each a polynomial times exp(-x^T M x + linear): these are
integrated exactly by a tensor Gauss-Hermite rule in the Cholesky frame of M. The outer
u integral is mapped to t in [0, 1) by u = s t / sqrt(1 - t^2) with s^2 = pq/(p+q) and
integrated by Gauss-Legendre. Nothing here uses the Boys function, Rys roots or any
Obara-Saika / Rys recurrence.
"""
import numpy as np


def _cart(l):
    return [(ax, ay, l - ax - ay) for ax in range(l, -1, -1) for ay in range(l - ax, -1, -1)]


def primitive_block(la, lb, lc, ld, a, b, c, d, A, B, C, D, nu=120, ngh=14):
    A, B, C, D = (np.asarray(v, float) for v in (A, B, C, D))
    p, q = a + b, c + d
    s = np.sqrt(p * q / (p + q))
    t, wt = np.polynomial.legendre.leggauss(nu)
    t = 0.5 * (t + 1.0)
    wt = 0.5 * wt
    u = s * t / np.sqrt(1.0 - t * t)
    du = s / (1.0 - t * t) ** 1.5 * wt
    y, wy = np.polynomial.hermite.hermgauss(ngh)
    Y1, Y2 = np.meshgrid(y, y, indexing="ij")
    W2 = np.outer(wy, wy)
    # per direction, per u: 2D integrals for all exponent tuples (ex<=la, fx<=lb, gx<=lc, hx<=ld)
    Ixyz = []
    for k in range(3):
        out = np.zeros((nu, la + 1, lb + 1, lc + 1, ld + 1))
        for iu in range(nu):
            u2 = u[iu] ** 2
            M = np.array([[p + u2, -u2], [-u2, q + u2]])
            lin = np.array([a * A[k] + b * B[k], c * C[k] + d * D[k]])
            x0 = np.linalg.solve(M, lin)
            const = -(a * A[k] ** 2 + b * B[k] ** 2 + c * C[k] ** 2 + d * D[k] ** 2) + lin @ x0
            L = np.linalg.cholesky(M)
            Linv_T = np.linalg.inv(L).T
            X1 = x0[0] + Linv_T[0, 0] * Y1 + Linv_T[0, 1] * Y2
            X2 = x0[1] + Linv_T[1, 0] * Y1 + Linv_T[1, 1] * Y2
            jac = 1.0 / np.prod(np.diag(L))
            pa = np.stack([(X1 - A[k]) ** e for e in range(la + 1)])
            pb = np.stack([(X1 - B[k]) ** e for e in range(lb + 1)])
            pc = np.stack([(X2 - C[k]) ** e for e in range(lc + 1)])
            pd = np.stack([(X2 - D[k]) ** e for e in range(ld + 1)])
            out[iu] = np.exp(const) * jac * np.einsum("ixy,jxy,kxy,lxy,xy->ijkl", pa, pb, pc, pd, W2)
        Ixyz.append(out)
    ca, cb, cc, cd = _cart(la), _cart(lb), _cart(lc), _cart(ld)
    blk = np.zeros((len(ca), len(cb), len(cc), len(cd)))
    pref = 2.0 / np.sqrt(np.pi)
    for i, ea in enumerate(ca):
        for j, eb in enumerate(cb):
            for kk, ec in enumerate(cc):
                for m, ed in enumerate(cd):
                    v = du.copy()
                    for k in range(3):
                        v = v * Ixyz[k][:, ea[k], eb[k], ec[k], ed[k]]
                    blk[i, j, kk, m] = pref * v.sum()
    return blk
