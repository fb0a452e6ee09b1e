"""Generate rys_table.h: Rys roots and weights for N = 1..9 as piecewise polynomials in T.

The N-point Rys rule for the parameter T is the Gauss rule of the weight
exp(-T u) u^(-1/2) / 2 on u = t^2 in [0, 1]; its moments are the Boys values
F_m(T) = int_0^1 t^(2m) exp(-T t^2) dt, and sum_n w_n u_n^m = F_m(T) for m < 2N
(paper section 2: the ERI is an exact N-point quadrature over the Rys roots).

Method (all in mpmath at 60 significant digits):
  1. F_0..F_17(T) from the lower incomplete gamma function.
  2. Recurrence coefficients of the monic orthogonal polynomials from the ordinary
     moments (Chebyshev's algorithm; ill-conditioned, hence the working precision).
  3. Nodes and weights from the symmetric tridiagonal Jacobi matrix (Golub-Welsch).
For T in [0, TMAX[N]) the interval [k, k+1) carries, for every root, a degree-11
polynomial in s = 2(T-k) - 1 for u_n and one for w_n (Chebyshev interpolation at 12
nodes, converted to monomial coefficients in mpmath, evaluated by Horner). For T >= TMAX[N] the
large-T limit u_n = s_n^2 / T, w_n = W_n / sqrt(T) holds to double precision, where s_n
are the positive roots of the Hermite polynomial H_2N and W_n their Gauss-Hermite
weights.

Usage: python gen_rys_table.py [out.h]   (about a minute on 8 cores)
"""
from __future__ import annotations

import multiprocessing as mproc
import os
import sys

import mpmath as mp
import numpy as np

NMAX = 9
DEG = 11
TMAX = [0, 40, 50, 56, 62, 70, 76, 84, 92, 100]     # index N
DPS = 60


def boys(m, T):
    T = mp.mpf(T)
    if T == 0:
        return mp.mpf(1) / (2 * m + 1)
    h = m + mp.mpf(1) / 2
    return mp.gammainc(h, 0, T) / (2 * T ** h)


def recurrence(T, n):
    """a_k, b_k (k < n) of the monic orthogonal polynomials of the Rys weight."""
    mom = [boys(k, T) for k in range(2 * n)]
    a = [mp.mpf(0)] * n
    b = [mp.mpf(0)] * n
    prev = [mp.mpf(0)] * (2 * n)
    cur = list(mom)
    a[0] = mom[1] / mom[0]
    b[0] = mom[0]
    for k in range(1, n):
        nxt = [mp.mpf(0)] * (2 * n)
        for l in range(k, 2 * n - k):
            nxt[l] = cur[l + 1] - a[k - 1] * cur[l] - b[k - 1] * prev[l]
        a[k] = nxt[k + 1] / nxt[k] - cur[k] / cur[k - 1]
        b[k] = nxt[k] / cur[k - 1]
        prev, cur = cur, nxt
    return a, b


def gauss_from_recurrence(a, b, n):
    J = mp.matrix(n, n)
    for i in range(n):
        J[i, i] = a[i]
        if i + 1 < n:
            J[i, i + 1] = J[i + 1, i] = mp.sqrt(b[i + 1])
    E, Q = mp.eigsy(J)
    pairs = sorted((E[i], b[0] * Q[0, i] ** 2) for i in range(n))
    return [p[0] for p in pairs], [p[1] for p in pairs]


def nodes_and_values(T):
    """u_n, w_n for every N at one T (float lists), sharing one recurrence."""
    mp.mp.dps = DPS
    T = mp.mpf(T)
    a, b = recurrence(T, NMAX)
    out = {}
    for N in range(1, NMAX + 1):
        if T >= TMAX[N]:
            continue
        u, w = gauss_from_recurrence(a, b, N)
        out[N] = ([mp.nstr(x, 40) for x in u], [mp.nstr(x, 40) for x in w])
    return out


def hermite_limit(N):
    """Positive roots s_n of H_2N (ascending) and their Gauss-Hermite weights."""
    mp.mp.dps = DPS
    n = 2 * N
    J = mp.matrix(n, n)
    for i in range(n - 1):
        J[i, i + 1] = J[i + 1, i] = mp.sqrt(mp.mpf(i + 1) / 2)
    E, Q = mp.eigsy(J)
    pairs = sorted((E[i], mp.sqrt(mp.pi) * Q[0, i] ** 2) for i in range(n))
    pos = [p for p in pairs if p[0] > 0]
    return [float(p[0] ** 2) for p in pos], [float(p[1]) for p in pos]


def cheb_nodes():
    mp.mp.dps = DPS
    return [mp.cos(mp.pi * (k + mp.mpf(1) / 2) / (DEG + 1)) for k in range(DEG + 1)]


def monomial_fit(x, y):
    """Interpolate y at the Chebyshev nodes x (all mpmath) and return the ascending
    monomial coefficients of the interpolant, rounded to double at the very end."""
    n = DEG + 1
    cheb = []
    for j in range(n):
        c = mp.fsum(y[k] * mp.cos(j * mp.acos(x[k])) for k in range(n)) * 2 / n
        cheb.append(c / 2 if j == 0 else c)
    # T_j(s) in ascending powers: T_0 = 1, T_1 = s, T_{j+1} = 2 s T_j - T_{j-1}
    tpow = [[mp.mpf(1)], [mp.mpf(0), mp.mpf(1)]]
    for j in range(2, n):
        nxt = [mp.mpf(0)] * (j + 1)
        for i, v in enumerate(tpow[j - 1]):
            nxt[i + 1] += 2 * v
        for i, v in enumerate(tpow[j - 2]):
            nxt[i] -= v
        tpow.append(nxt)
    mono = [mp.mpf(0)] * n
    for j in range(n):
        for i, v in enumerate(tpow[j]):
            mono[i] += cheb[j] * v
    return [float(v) for v in mono]


def build_tables(procs=None):
    x = cheb_nodes()
    kmax = max(TMAX)
    Ts = [mp.nstr(kk + (xx + 1) / 2, 50) for kk in range(kmax) for xx in x]
    with mproc.Pool(procs or min(8, os.cpu_count() or 1)) as pool:
        vals = pool.map(nodes_and_values, Ts, chunksize=8)
    tables = {}
    for N in range(1, NMAX + 1):
        coef = np.zeros((TMAX[N], N, 2, DEG + 1))
        for kk in range(TMAX[N]):
            for n in range(N):
                for q in (0, 1):
                    Y = [mp.mpf(vals[kk * (DEG + 1) + j][N][q][n]) for j in range(DEG + 1)]
                    coef[kk, n, q] = monomial_fit(x, Y)                # ascending powers of s
        tables[N] = coef
    return tables


def write_header(tables, path):
    lines = ["/* Generated by gen_rys_table.py -- do not edit. Rys roots u_n = t_n^2 and weights w_n.",
             " * coef layout per N: [interval k][root n][u|w][power 0..RYS_DEG] in s = 2(T-k)-1. */",
             "#pragma once", f"#define RYS_NMAX {NMAX}", f"#define RYS_DEG {DEG}",
             "static constexpr int RYS_TMAX[RYS_NMAX + 1] = {" + ", ".join(str(t) for t in TMAX) + "};"]
    offs = [0] * (NMAX + 2)
    for N in range(1, NMAX + 1):
        offs[N + 1] = offs[N] + tables[N].size
    lines.append("static constexpr int RYS_OFF[RYS_NMAX + 2] = {" + ", ".join(str(o) for o in offs) + "};")
    lines.append(f"#define RYS_NCOEF {offs[NMAX + 1]}")
    lines.append("RYS_STORAGE double RYS_COEF[RYS_NCOEF] = {")
    for N in range(1, NMAX + 1):
        flat = tables[N].ravel()
        for i in range(0, flat.size, 4):
            lines.append("  " + ", ".join(float(v).hex() for v in flat[i:i + 4]) + ",")
    lines.append("};")
    s2all, wall = [], []
    hoff = [0] * (NMAX + 2)
    for N in range(1, NMAX + 1):
        s2, w = hermite_limit(N)
        s2all += s2
        wall += w
        hoff[N + 1] = hoff[N] + N
    lines.append("static constexpr int RYS_HOFF[RYS_NMAX + 2] = {" + ", ".join(str(o) for o in hoff) + "};")
    lines.append("RYS_STORAGE double RYS_HERM_S2[" + str(len(s2all)) + "] = {" + ", ".join(v.hex() for v in s2all) + "};")
    lines.append("RYS_STORAGE double RYS_HERM_W[" + str(len(wall)) + "] = {" + ", ".join(v.hex() for v in wall) + "};")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def main():
    out = sys.argv[1] if len(sys.argv) > 1 else os.path.join(os.path.dirname(os.path.abspath(__file__)), "rys_table.h")
    write_header(build_tables(), out)
    print("wrote", out)


if __name__ == "__main__":
    main()
