"""Steps (i)-(ii) on the GPU (fstat_sfts_to_series) against the oracle's
literal sum, and the whole pipeline from SFTs to 2F.

Bar: the series within 2e-6 of its peak magnitude sample by sample (FP32
transform of at most 4096 points against the float64 sum), validity equal;
2F from the GPU series within the 2F bar of the oracle's pipeline.
"""
import sys

import numpy as np
import pytest

from oracle import fstat_oracle as O
from paper_2201_00451_amd import synth

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("K", [6, 150, 360, 900, 1800, 3600, 4096, 2 * 3 * 5 * 4 * 9])
def test_series_matches_oracle_sum(torch_dev, K):
    from paper_2201_00451_amd import binding
    rng = np.random.default_rng(K)
    n_sft, t_sft, t0 = 7, 1800.0, 123456.0
    k0 = 7 * K + 3
    S = (rng.standard_normal((n_sft, K)) + 1j * rng.standard_normal((n_sft, K))).astype(
        np.complex64)
    present = np.array([1, 1, 0, 1, 0, 1, 1], dtype=np.uint8)
    x, v, f_h, dt = binding.sfts_to_series(S, present, k0, t_sft, t0)
    binding.sync_check()
    xr, vr, fr, dr = O.sfts_to_series(S, present, k0, t_sft, t0)
    assert f_h == fr and dt == dr
    x = x.cpu().numpy()
    err = np.abs(x - xr).max() / np.abs(xr).max()
    say(f"  K={K}: max error / peak {err:.2e}")
    assert err < 2e-6
    np.testing.assert_array_equal(v.cpu().numpy(), vr)
    assert np.all(x[vr == 0] == 0)


def test_pipeline_from_sfts(torch_dev):
    """SFTs -> series (GPU) -> 2F (GPU), against the same chain in the oracle."""
    from paper_2201_00451_amd import binding
    ds, sfts = synth.sft_case(seed=85, ndet=2, rho=20.0, drop_p=0.15, binary=True)
    sf = ds.sft
    gx, gv, ox, ov = [], [], [], []
    for S, pres in sfts:
        x, v, f_h, dt = binding.sfts_to_series(S, pres, sf["k0"], sf["t_sft"], sf["t_start"])
        assert abs(f_h - ds.f_het) < 1e-12 and dt == ds.dt
        gx.append(x.cpu().numpy())
        gv.append(v.cpu().numpy())
        a, b, _, _ = O.sfts_to_series(S, pres, sf["k0"], sf["t_sft"], sf["t_start"])
        ox.append(a)
        ov.append(b)
    ds.x, ds.valid = gx, gv
    dd = binding.DeviceData(ds)
    tf = binding.compute_2f(dd, ds.templates).cpu().numpy()
    binding.sync_check()
    ds.x, ds.valid = ox, ov
    ref = O.oracle_twoF(ds)
    for i in range(ds.ntmpl):
        strong = ref[i] >= 10.0
        rel = np.abs(tf[i] - ref[i])[strong] / ref[i][strong]
        ab = np.abs(tf[i] - ref[i])[~strong]
        say(f"  template {i}: max rel {rel.max():.2e} ({strong.sum()} bins), max abs {ab.max():.2e}")
        assert rel.max() <= 1e-4 and ab.max() <= 1e-3
    inj = ds.injections[0]
    say(f"  peak 2F {tf[0].max():.2f}, rho^2 {inj['rho2']:.1f}")
    assert tf[0].max() > 0.7 * inj["rho2"]
