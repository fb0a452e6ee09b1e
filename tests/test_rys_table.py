"""Pins of the generated Rys root/weight table (CPU, no GPU).

The table is evaluated here the way the kernels evaluate it (interval k = floor(T),
Horner in s = 2(T-k)-1; Hermite limit beyond TMAX[N]) and checked against facts that do
not depend on it: the moment identity sum_n w_n u_n^m = F_m(T) for m < 2N with F_m from
scipy's incomplete gamma, Gauss-Legendre at T = 0, and Gauss-Hermite as T grows.
"""
import os
import re

import numpy as np
import pytest
from scipy.special import gamma, gammainc

HDR = os.path.join(os.path.dirname(__file__), "..", "paper_2407_09700_amd", "csrc", "rys_table.h")


def _arr(text, name):
    m = re.search(name + r"\[[^\]]*\]\s*=\s*\{(.*?)\};", text, re.S)
    return [float.fromhex(t) if "0x" in t else float(t) for t in re.split(r"[,\s]+", m.group(1).strip()) if t]


@pytest.fixture(scope="module")
def table():
    text = open(HDR).read()
    deg = int(re.search(r"#define RYS_DEG (\d+)", text).group(1))
    return dict(deg=deg, tmax=[int(v) for v in _arr(text, "RYS_TMAX")], off=[int(v) for v in _arr(text, "RYS_OFF")],
                coef=np.array(_arr(text, "RYS_COEF")), hoff=[int(v) for v in _arr(text, "RYS_HOFF")],
                s2=np.array(_arr(text, "RYS_HERM_S2")), hw=np.array(_arr(text, "RYS_HERM_W")))


def rys_eval(tab, N, T):
    if T >= tab["tmax"][N]:
        o = tab["hoff"][N]
        return tab["s2"][o:o + N] / T, tab["hw"][o:o + N] / np.sqrt(T)
    deg = tab["deg"]
    k = int(np.floor(T))
    s = 2.0 * (T - k) - 1.0
    c = tab["coef"][tab["off"][N]:tab["off"][N + 1]].reshape(tab["tmax"][N], N, 2, deg + 1)[k]
    u = np.zeros(N)
    w = np.zeros(N)
    for n in range(N):
        pu, pw = c[n, 0, deg], c[n, 1, deg]
        for p in range(deg - 1, -1, -1):
            pu = pu * s + c[n, 0, p]
            pw = pw * s + c[n, 1, p]
        u[n], w[n] = pu, pw
    return u, w


def boys(m, T):
    if T == 0:
        return 1.0 / (2 * m + 1)
    return gamma(m + 0.5) * gammainc(m + 0.5, T) / (2.0 * T ** (m + 0.5))


@pytest.mark.parametrize("N", range(1, 10))
def test_moment_identity(table, N):
    rng = np.random.default_rng(N)
    Ts = np.concatenate([[0.0, 1e-9, 0.5, 1.0, 2.0 - 1e-12, table["tmax"][N] - 1e-9, table["tmax"][N],
                          table["tmax"][N] + 0.5, 150.0, 1e4], rng.uniform(0, table["tmax"][N] + 5, 60)])
    worst = 0.0
    for T in Ts:
        u, w = rys_eval(table, N, float(T))
        assert np.all(u > 0) and np.all(u < 1) and np.all(w > 0) and np.all(np.diff(u) > 0)
        for m in range(2 * N):
            ref = boys(m, float(T))
            worst = max(worst, abs(np.sum(w * u ** m) - ref) / ref)
    assert worst < 2e-13, worst


@pytest.mark.parametrize("N", range(1, 10))
def test_zero_T_is_gauss_legendre(table, N):
    x, wl = np.polynomial.legendre.leggauss(2 * N)
    u, w = rys_eval(table, N, 0.0)
    np.testing.assert_allclose(u, x[N:] ** 2, rtol=1e-14)
    np.testing.assert_allclose(w, wl[N:], rtol=0, atol=2e-15)   # numpy's rule itself is good to ~1e-15 absolute


@pytest.mark.parametrize("N", range(1, 10))
def test_large_T_is_gauss_hermite(table, N):
    x, wh = np.polynomial.hermite.hermgauss(2 * N)
    T = 400.0
    u, w = rys_eval(table, N, T)
    np.testing.assert_allclose(u * T, x[N:] ** 2, rtol=1e-13)
    np.testing.assert_allclose(w * np.sqrt(T), wh[N:], rtol=1e-13)


@pytest.mark.parametrize("N", [1, 2])
def test_closed_form_roots_moment_identity(N):
    """The kernels' closed-form rule for one or two roots (compiled for the host) against
    the moment identity with scipy's incomplete gamma."""
    from paper_2407_09700_amd import jk
    rng = np.random.default_rng(40 + N)
    Ts = np.concatenate([[0.0, 1e-12, 1e-6, 0.3, 0.999999, 1.0, 1.000001, 7.0, 35.0, 60.0, 300.0, 1e5],
                         rng.uniform(0, 3, 40), rng.uniform(0, 80, 40)])
    worst = 0.0
    for T in Ts:
        u, w = jk.rys_closed(N, float(T))
        assert np.all(u > 0) and np.all(u < 1) and np.all(w > 0)
        for m in range(2 * N):
            ref = boys(m, float(T))
            worst = max(worst, abs(np.sum(w * u ** m) - ref) / ref)
    assert worst < 2e-14, worst


@pytest.mark.parametrize("N", [1, 2])
def test_closed_form_matches_table(table, N):
    from paper_2407_09700_amd import jk
    for T in np.linspace(0.0, 60.0, 121):
        u, w = jk.rys_closed(N, float(T))
        ut, wt = rys_eval(table, N, float(T))
        np.testing.assert_allclose(u, ut, rtol=2e-13)
        np.testing.assert_allclose(w, wt, rtol=2e-13)


@pytest.mark.parametrize("N", [1, 2])
def test_grid_rule_moment_identity(table, N):
    """The lane bodies' rule for one or two roots (Boys values from a Taylor series about the
    nearest grid point, then the Gauss rule of the moments; compiled for the host) against the
    moment identity with scipy's incomplete gamma, over [0, TMAX[N]) including grid points,
    midpoints between them and the ends."""
    from paper_2407_09700_amd import jk
    rng = np.random.default_rng(70 + N)
    tmax = table["tmax"][N]
    Ts = np.concatenate([[0.0, 1e-12, 1e-6, 0.0625, 0.0625 + 1e-13, 0.125, 0.1875, 1.0, 7.3125, tmax - 1e-9,
                          tmax - 0.0625], rng.uniform(0, 2, 60), rng.uniform(0, tmax, 200)])
    worst = 0.0
    for T in Ts:
        u, w = jk.rys_grid(N, float(T))
        assert np.all(u > 0) and np.all(u < 1) and np.all(w > 0) and np.all(np.diff(u) > 0)
        for m in range(2 * N):
            ref = boys(m, float(T))
            worst = max(worst, abs(np.sum(w * u ** m) - ref) / ref)
    assert worst < 2e-14, worst


@pytest.mark.parametrize("N", [1, 2])
def test_grid_rule_matches_table(table, N):
    """Two independent evaluations of the same rule: the grid rule and the interpolation table
    (which the larger root counts use) agree to 1e-13 relative."""
    from paper_2407_09700_amd import jk
    for T in np.linspace(0.0, table["tmax"][N] - 1e-6, 397):
        u, w = jk.rys_grid(N, float(T))
        ut, wt = rys_eval(table, N, float(T))
        np.testing.assert_allclose(u, ut, rtol=1e-13)
        np.testing.assert_allclose(w, wt, rtol=1e-13)


def test_grid_rule_rejects_out_of_range():
    from paper_2407_09700_amd import jk
    with pytest.raises(jk.JKError):
        jk.rys_grid(1, 40.0)
    with pytest.raises(jk.JKError):
        jk.rys_grid(2, -1.0)
    with pytest.raises(jk.JKError):
        jk.rys_grid(3, 1.0)
