"""Adjoint (gradient) path vs the FP64 gradient oracle, through the C ABI.

The gradient oracle (float64 autograd of the resampled 2F) is pinned to
central finite differences of the numpy oracle on the CPU.  Bar here: every
component within 1e-3 relative of the oracle's (the finite-difference bar of
the refinement workload), on templates displaced from the injection in every
parameter so that no component vanishes by symmetry.
"""
import sys

import numpy as np
import pytest

from oracle import fstat_oracle as O
from oracle import fstat_oracle_grad as G
from paper_2201_00451_amd import synth

pytestmark = pytest.mark.gpu

GRAD_RTOL = 1e-3


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_2201_00451_amd import binding
    binding.load_library()
    return torch


CASES = {
    "isolated_2det_gaps": dict(seed=51, n=3000, n_fft=1 << 13, ndet=2, gaps=True, rho=20),
    "binary_2det_gaps": dict(seed=52, n=3000, n_fft=1 << 13, ndet=2, gaps=True, rho=20,
                             binary=True),
    "binary_d12": dict(seed=53, n=3000, n_fft=1 << 13, ndet=2, binary=True, D=12, rho=25),
    "three_det_d4": dict(seed=54, n=2500, n_fft=1 << 13, ndet=3, D=4, rho=20,
                         noise_vars=[1.0, 0.7, 1.4]),
    "ragged_band": dict(seed=55, n=3000, n_fft=1 << 13, ndet=1, rho=25, bin_lo=1500,
                        n_bins=3001),
    "kepler": dict(seed=52, n=3000, n_fft=1 << 13, ndet=2, gaps=True, rho=20, binary=True,
                   ecc=0.3, argp=0.9),
}


def displaced_row(ds):
    """The first template moved off the injection in every parameter."""
    row = ds.templates[0].copy()
    T = ds.detectors[0].n * ds.dt
    row[0] += 0.002
    row[1] -= 0.0015
    row[2] += 0.3 / T
    row[3] += 0.5 / T ** 2
    if row[5] != 0.0:
        row[5] *= 1.002
        row[6] *= 1.0 + 2e-5
        row[7] += 3.0
    return row


def bin_weights(ds, row):
    """Weights over the band: the peak bins and a stretch of noise bins."""
    tf = O.oracle_twoF(ds, row[None])[0]
    w = np.zeros(ds.n_bins)
    ipk = int(np.argmax(tf))
    w[max(ipk - 3, 0):ipk + 4] = 1.0
    w[100:110] = 0.5
    return w


@pytest.mark.parametrize("case", sorted(CASES))
def test_gradient_matches_oracle(torch_dev, case):
    from paper_2201_00451_amd import binding
    say(f"grad parity {case}")
    ds = synth.small_case(**CASES[case])
    row = displaced_row(ds)
    w = bin_weights(ds, row)
    tf_ref, g_ref = G.oracle_grad(ds, row, w)
    dd = binding.DeviceData(ds)
    g, tf = binding.compute_2f_grad(dd, row[None], w[None], want_twoF=True)
    binding.sync_check()
    g = g.cpu().numpy()[0]
    tf = tf.cpu().numpy()[0]
    # the 2F computed alongside meets the forward bar
    strong = tf_ref >= 10.0
    assert np.max(np.abs(tf[strong] - tf_ref[strong]) / tf_ref[strong]) <= 1e-4
    assert np.max(np.abs(tf[~strong] - tf_ref[~strong])) <= 1e-3
    for i, name in enumerate(G.PARAMS):
        rel = abs(g[i] - g_ref[i]) / max(abs(g_ref[i]), 1e-300)
        say(f"  {name:6s} gpu {g[i]: .9e} oracle {g_ref[i]: .9e} rel {rel:.2e}")
    for i, name in enumerate(G.PARAMS):
        if row[5] == 0.0 and i >= 4:
            assert g[i] == 0.0, name
            continue
        assert abs(g[i] - g_ref[i]) <= GRAD_RTOL * abs(g_ref[i]), (name, g[i], g_ref[i])


def test_gradient_batch_independent_and_2f_bitwise(torch_dev):
    """Several templates per launch give the same gradients as one at a time,
    and the 2F of the adjoint call equals the batched forward path bit for bit."""
    from paper_2201_00451_amd import binding
    ds = synth.small_case(seed=56, n=3000, n_fft=1 << 13, ndet=2, binary=True, gaps=True,
                          ntmpl=6, rho=20)
    rows = np.array([displaced_row(ds) for _ in range(6)])
    rows[:, 0] += 0.001 * np.arange(6)
    rng = np.random.default_rng(0)
    w = rng.uniform(0.0, 1.0, size=(6, ds.n_bins))
    dd = binding.DeviceData(ds, batch=6)
    g1, tf1 = binding.compute_2f_grad(dd, rows, w, want_twoF=True, batch=1)
    g4, tf4 = binding.compute_2f_grad(dd, rows, w, want_twoF=True, batch=4)
    fwd = binding.compute_2f_batched(dd, rows)
    binding.sync_check()
    assert torch_dev.equal(g1, g4)
    assert torch_dev.equal(tf1, tf4)
    assert torch_dev.equal(tf1, fwd)


def test_flagged_and_isolated_rows(torch_dev):
    """A template whose delay exceeds the bound gets NaN gradients and NaN 2F;
    an isolated one reports zero orbit derivatives; neighbours are unaffected."""
    from paper_2201_00451_amd import binding
    ds = synth.small_case(seed=57, n=3000, n_fft=1 << 13, ndet=1, ntmpl=3, rho=20)
    rows = ds.templates.copy()
    rows[1, 5], rows[1, 6], rows[1, 7] = 3000.0, 1e7, 6000.0 + 2.5e6
    w = np.ones((3, ds.n_bins))
    dd = binding.DeviceData(ds)
    g, tf = binding.compute_2f_grad(dd, rows, w, want_twoF=True, batch=3)
    g_solo = binding.compute_2f_grad(dd, rows[[0]], w[[0]], batch=1)
    binding.sync_check()
    g, tf = g.cpu().numpy(), tf.cpu().numpy()
    assert np.all(np.isnan(g[1])) and np.all(np.isnan(tf[1]))
    assert np.all(np.isfinite(g[[0, 2]])) and np.all(np.isfinite(tf[[0, 2]]))
    assert np.all(g[[0, 2], 4:] == 0.0)
    assert np.array_equal(g[0], g_solo.cpu().numpy()[0])


def test_autograd_function(torch_dev):
    """torch.autograd through the adjoint kernels: the forward is the batched
    path and params.grad equals fstat_compute_2f_grad with the same weights."""
    torch = torch_dev
    from paper_2201_00451_amd import binding
    ds = synth.small_case(seed=58, n=3000, n_fft=1 << 13, ndet=2, binary=True, ntmpl=2, rho=20)
    rows = np.array([displaced_row(ds), ds.templates[1]])
    params = torch.tensor(rows[:, list(binding.GRAD_COLUMNS)], dtype=torch.float64,
                          device="cuda:0", requires_grad=True)
    dd = binding.DeviceData(ds, batch=2)
    tf = binding.twoF(dd, params)
    w = torch.linspace(0.0, 1.0, ds.n_bins, device="cuda:0")[None].repeat(2, 1)
    (tf * w).sum().backward()
    g = binding.compute_2f_grad(dd, rows, w)
    ref = binding.compute_2f_batched(dd, rows)
    binding.sync_check()
    assert torch.equal(tf.detach(), ref)
    assert torch.equal(params.grad, g)


def test_refinement_climbs_to_the_injection(torch_dev):
    """Gradient ascent from a displaced start on noiseless data recovers the
    2F of the true parameters (the global maximum there) in the injection's bin."""
    from paper_2201_00451_amd import binding
    ds = synth.small_case(seed=59, n=4000, n_fft=1 << 13, ndet=2, binary=True, rho=20,
                          noise=False, ntmpl=1)
    inj = ds.injections[0]
    N, dt = ds.n_fft, ds.dt
    m = int(round((inj["f"] - ds.f_het) * N * dt)) + N // 2
    df = (inj["f"] - ds.f_het) - (m - N // 2) / (N * dt)
    truth = ds.templates[0].copy()
    truth[2] = df
    T = ds.detectors[0].n * dt
    start = truth.copy()
    start[2] -= 0.5 / T
    start[5] *= 1.005
    start[7] += 20.0
    dd = binding.DeviceData(ds)
    tf_true = binding.compute_2f(dd, truth[None]).cpu().numpy()[0, m]
    tf_start = binding.compute_2f(dd, start[None]).cpu().numpy()[0, m]
    om = 2.0 * np.pi / inj["porb"]
    scales = np.array([1.0 / T, 1.0 / T ** 2, 1e-3, 1e-3, 1.0 / (2 * np.pi * inj["f"]), 1.0,
                       1.0 / (2 * np.pi * inj["f"] * inj["asini"] * om)])
    rows, vals = binding.refine(dd, start[None], [m], scales, steps=30,
                                free=("df", "asini", "tp"))
    binding.sync_check()
    say(f"  refinement: 2F start {tf_start:.3f} -> {vals[0]:.3f} (true parameters {tf_true:.3f})")
    assert tf_start < 0.9 * tf_true
    assert vals[0] >= 0.99 * tf_true


def test_single_bin_path_matches_general_adjoint_and_oracle(torch_dev):
    """The single-bin form (direct one-bin transform, adjoint series in closed
    form) against the general adjoint with one-hot weights and against the FP64
    oracle gradient; a bin outside the band gives NaN for that template only."""
    from paper_2201_00451_amd import binding
    ds = synth.small_case(seed=60, n=3000, n_fft=1 << 13, ndet=2, binary=True, gaps=True,
                          ntmpl=3, rho=25, bin_lo=1000, n_bins=5000)
    rows = np.array([displaced_row(ds) for _ in range(3)])
    rows[1, 0] += 0.004
    tf_ref = O.oracle_twoF(ds, rows)
    bins = np.array([int(np.argmax(tf_ref[0])) + 2, int(np.argmax(tf_ref[1])), 17])
    dd = binding.DeviceData(ds, batch=3)
    g_bin, tf_bin = binding.compute_2f_grad_bin(dd, rows, bins)
    onehot = np.zeros((3, ds.n_bins))
    onehot[np.arange(3), bins] = 1.0
    g_gen, tf_gen = binding.compute_2f_grad(dd, rows, onehot, want_twoF=True)
    bad = bins.copy()
    bad[1] = ds.n_bins
    g_bad, tf_bad = binding.compute_2f_grad_bin(dd, rows, bad)
    binding.sync_check()
    g_bin, tf_bin = g_bin.cpu().numpy(), tf_bin.cpu().numpy()
    g_gen, tf_gen = g_gen.cpu().numpy(), tf_gen.cpu().numpy()
    for m in range(3):
        ref2f = tf_ref[m, bins[m]]
        got = tf_bin[m]
        say(f"  template {m} bin {bins[m]}: 2F single-bin {got:.6f} fft {tf_gen[m, bins[m]]:.6f} "
            f"oracle {ref2f:.6f}")
        if ref2f >= 10.0:
            assert abs(got - ref2f) <= 1e-4 * ref2f
        else:
            assert abs(got - ref2f) <= 1e-3
        _, g_or = G.oracle_grad(ds, rows[m], onehot[m])
        for i, name in enumerate(G.PARAMS):
            say(f"    {name:6s} bin {g_bin[m, i]: .9e} general {g_gen[m, i]: .9e} "
                f"oracle {g_or[i]: .9e}")
            assert abs(g_bin[m, i] - g_or[i]) <= GRAD_RTOL * abs(g_or[i]), (m, name)
            assert abs(g_bin[m, i] - g_gen[m, i]) <= GRAD_RTOL * abs(g_or[i]), (m, name)
    g_bad, tf_bad = g_bad.cpu().numpy(), tf_bad.cpu().numpy()
    assert np.all(np.isnan(g_bad[1])) and np.isnan(tf_bad[1])
    assert np.array_equal(g_bad[[0, 2]], g_bin[[0, 2]])
    assert np.array_equal(tf_bad[[0, 2]], tf_bin[[0, 2]])
