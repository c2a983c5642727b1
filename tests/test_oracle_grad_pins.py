"""Pins of the float64 gradient oracle: its 2F is the numpy oracle's 2F, and
its autograd gradient is the central finite difference of the numpy oracle."""
import numpy as np
import pytest

from oracle import fstat_oracle as O
from oracle import fstat_oracle_grad as G
from paper_2201_00451_amd import synth

COL = {"alpha": 0, "delta": 1, "df": 2, "f1dot": 3, "asini": 5, "porb": 6, "tp": 7}
STEP = {"df": 1e-7, "f1dot": 1e-12, "alpha": 1e-6, "delta": 1e-6, "asini": 1e-5, "porb": 1e-1,
        "tp": 1e-1}


def fd_grad(ds, row, w, name):
    h = STEP[name]
    rp, rm = row.copy(), row.copy()
    rp[COL[name]] += h
    rm[COL[name]] -= h
    return (np.sum(w * O.oracle_twoF(ds, rp[None])[0]) -
            np.sum(w * O.oracle_twoF(ds, rm[None])[0])) / (2 * h)


@pytest.mark.parametrize("binary,asini,f2dot", [(False, None, 0.0), (True, None, 0.0),
                                               (True, 2e-3, 0.0), (False, None, 4e-12)])
def test_gradient_oracle_matches_oracle_and_finite_differences(binary, asini, f2dot):
    """asini = 2e-3 ls: a barely binary template, where the orbit derivatives
    are real and small; f2dot != 0: the held-fixed second spin-down term
    enters the phase the derivatives are taken through."""
    ds = synth.small_case(seed=51, n=3000, n_fft=1 << 13, ndet=2, binary=binary, gaps=True,
                          rho=20, f2dot=f2dot)
    row = ds.templates[0].copy()
    row[0] += 0.002
    if binary:
        row[5] = asini if asini is not None else row[5] * 1.001
    tf_np = O.oracle_twoF(ds, row[None])[0]
    w = np.zeros(ds.n_bins)
    ipk = int(np.argmax(tf_np))
    w[ipk - 3:ipk + 4] = 1.0
    w[100:110] = 0.5
    tf_t, g = G.oracle_grad(ds, row, w)
    np.testing.assert_allclose(tf_t, tf_np, rtol=1e-10, atol=1e-10)
    for i, name in enumerate(G.PARAMS):
        if not binary and name in ("asini", "porb", "tp"):
            assert g[i] == 0.0
            continue
        fd = fd_grad(ds, row, w, name)
        assert abs(g[i] - fd) <= 1e-4 * abs(fd) + 1e-9, (name, g[i], fd)
        if asini is not None and name == "asini":
            assert abs(fd) > 1e-2   # a real, non-vanishing derivative


def test_gradient_oracle_keplerian_orbit():
    """The gradient oracle with a Keplerian orbit (eccentricity and argument
    of periapsis held fixed) against central differences of the numpy oracle."""
    ds = synth.small_case(seed=52, n=3000, n_fft=1 << 13, ndet=2, binary=True, gaps=True,
                          rho=20, ecc=0.3, argp=0.9)
    row = ds.templates[0].copy()
    row[0] += 0.002
    row[5] *= 1.001
    tf_np = O.oracle_twoF(ds, row[None])[0]
    w = np.zeros(ds.n_bins)
    ipk = int(np.argmax(tf_np))
    w[ipk - 3:ipk + 4] = 1.0
    tf_t, g = G.oracle_grad(ds, row, w)
    np.testing.assert_allclose(tf_t, tf_np, rtol=1e-10, atol=1e-10)
    for i, name in enumerate(G.PARAMS):
        fd = fd_grad(ds, row, w, name)
        assert abs(g[i] - fd) <= 1e-4 * abs(fd) + 1e-9, (name, g[i], fd)
