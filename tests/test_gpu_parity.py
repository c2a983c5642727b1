"""GPU path vs the FP64 oracle on the same seeded inputs, through the C ABI.

Bar (2F, float32 path vs float64 oracle): relative error <= 1e-4 in bins where
the oracle's 2F >= 10, absolute error <= 1e-3 elsewhere.  Intermediate
results (resampled series, Fa, Fb) are compared with the accuracy metrics of
Sec. 4.2 (r_1, r_2, theta).
"""
import math
import os
import sys

import numpy as np
import pytest

from oracle import fstat_oracle as O
from paper_2201_00451_amd import synth

pytestmark = pytest.mark.gpu

REL_TOL, ABS_TOL, STRONG = 1e-4, 1e-3, 10.0


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


def assert_2f_parity(gpu, ref, label=""):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert gpu.shape == ref.shape
    assert np.all(np.isfinite(gpu)), f"{label}: non-finite GPU output"
    strong = ref >= STRONG
    rel = np.abs(gpu[strong] - ref[strong]) / ref[strong] if strong.any() else np.zeros(1)
    ab = np.abs(gpu[~strong] - ref[~strong])
    say(f"  {label}: max rel (2F>=10, {strong.sum()} bins) {rel.max():.3e}; "
        f"max abs (else) {ab.max():.3e}; r2 {O.rel_err(gpu, ref, 2):.3e}")
    assert rel.max() <= REL_TOL, f"{label}: relative error {rel.max():.3e}"
    assert ab.max() <= ABS_TOL, f"{label}: absolute error {ab.max():.3e}"


def run_gpu(ds, templates=None, fafb=False, batched=False, batch=1):
    from paper_2201_00451_amd import binding
    dd = binding.DeviceData(ds, batch=batch)
    tm = ds.templates if templates is None else templates
    out = binding.compute_2f(dd, tm, fafb=fafb, batched=batched)
    binding.sync_check()
    if fafb:
        return out[0].cpu().numpy(), out[1].cpu().numpy()
    return out.cpu().numpy()


CASES = {
    "one_det": dict(seed=31, n=6000, n_fft=1 << 14, ndet=1),
    "two_det_gaps": dict(seed=32, n=7000, n_fft=1 << 15, ndet=2, gaps=True, noise_vars=[0.8, 1.2]),
    "binary": dict(seed=33, n=7000, n_fft=1 << 14, ndet=2, binary=True, gaps=True),
    "ragged_band": dict(seed=34, n=5000, n_fft=1 << 13, ndet=1, bin_lo=1001, n_bins=3333),
    "d4": dict(seed=35, n=5000, n_fft=1 << 13, ndet=1, D=4),
    "d12": dict(seed=36, n=5000, n_fft=1 << 13, ndet=2, D=12, binary=True),
    "n_fft_2e12": dict(seed=37, n=1200, n_fft=1 << 12, ndet=1, dt=2.0),
    "n_fft_2e16": dict(seed=38, n=20000, n_fft=1 << 16, ndet=2, dt=2.0),
    "three_det": dict(seed=39, n=3000, n_fft=1 << 13, ndet=3, noise_vars=[1.0, 0.7, 1.4]),
    # the other accepted interpolation half-widths
    "d6": dict(seed=61, n=5000, n_fft=1 << 13, ndet=1, D=6),
    "d10": dict(seed=62, n=5000, n_fft=1 << 13, ndet=2, D=10, binary=True, gaps=True),
    "d16": dict(seed=63, n=5000, n_fft=1 << 14, ndet=2, D=16, gaps=True),
    # the second spin-down term: f2dot T^3 / 6 is about 5 cycles over the data
    "f2dot": dict(seed=64, n=7000, n_fft=1 << 14, ndet=2, gaps=True, f2dot=1.1e-11),
    "f2dot_binary": dict(seed=65, n=7000, n_fft=1 << 14, ndet=2, binary=True, f2dot=-1.1e-11),
    # Keplerian orbits (rows of ten: eccentricity and argument of periapsis)
    "kepler": dict(seed=66, n=7000, n_fft=1 << 14, ndet=2, binary=True, gaps=True, ecc=0.3,
                   argp=1.2),
    "kepler_high_e": dict(seed=67, n=6000, n_fft=1 << 14, ndet=1, binary=True, ecc=0.7,
                          argp=-2.4, D=12),
    # grids coarse enough that a 512-point tile spans more than 0.1 rad of
    # sidereal angle: the tiles evaluate the antenna patterns per point (knot
    # spacing 16 and 32, so the knots are still solved ahead)
    "dt10": dict(seed=68, n=6000, n_fft=1 << 14, ndet=2, dt=10.0, gaps=True, eph_spacing=120.0),
    "dt6_binary": dict(seed=69, n=8000, n_fft=1 << 14, ndet=2, dt=6.0, binary=True),
}


def test_antenna_moments_definition(torch_dev):
    """M_n = sum_j v_j exp(i n phi(t_j)), evaluated here by its definition."""
    from paper_2201_00451_amd import binding
    ds = synth.small_case(**CASES["two_det_gaps"])
    dd = binding.DeviceData(ds)
    binding.sync_check()
    got = dd.moments.cpu().numpy()
    m = ds.ephem_model
    for X, det in enumerate(ds.detectors):
        t = det.t0 + ds.dt * np.arange(det.n)
        phi = det.lon + m["sidereal_angle0_rad"] + m["sidereal_rate_rad_s"] * t
        for n in range(5):
            ref = np.sum(ds.valid[X] * np.exp(1j * n * phi))
            assert abs(got[X, 2 * n] + 1j * got[X, 2 * n + 1] - ref) < 1e-9 * det.n


@pytest.mark.parametrize("case", ["two_det_gaps", "binary", "dt10"])
def test_resampled_series_parity(torch_dev, case):
    from paper_2201_00451_amd import binding
    say(f"resample parity {case}")
    ds = synth.small_case(**CASES[case])
    dd = binding.DeviceData(ds)
    y = binding.resample(dd, ds.templates[:2])
    binding.sync_check()
    y = y.cpu().numpy()
    for i in range(2):
        ya, yb = O.resampled_series(ds, O.template_dict(ds.templates[i]))
        for got, ref, nm in ((y[i, 0], ya, "ya"), (y[i, 1], yb, "yb")):
            r2 = O.rel_err(got, ref, 2)
            mx = np.abs(got - ref).max() / np.abs(ref).max()
            say(f"  tmpl {i} {nm}: r2 {r2:.3e} max/peak {mx:.3e}")
            assert r2 < 2e-6 and mx < 5e-6


@pytest.mark.parametrize("case", sorted(CASES))
def test_2f_parity_small(torch_dev, case):
    say(f"2F parity {case}: {CASES[case]}")
    ds = synth.small_case(**CASES[case])
    ref, fab_ref = O.oracle_twoF(ds, return_fafb=True)
    gpu, fab = run_gpu(ds, fafb=True)
    for i in range(ds.ntmpl):
        assert_2f_parity(gpu[i], ref[i], f"{case} tmpl {i}")
        Fa, Fb, _ = fab_ref[i]
        for got, want, nm in ((fab[i, 0], Fa, "Fa"), (fab[i, 1], Fb, "Fb")):
            assert O.rel_err(got, want, 2) < 1e-5, nm
            assert O.rel_err(got, want, 1) < 1e-5, nm
            assert O.angle(got, want) < 1e-5, nm


def test_tiny_config_full_parity(torch_dev):
    """One detector, 1 day at 2 s, 11 spin-down templates, n_fft = 2^17."""
    say("tiny config parity")
    ds = synth.config_tiny()
    ref = O.oracle_twoF(ds)
    gpu = run_gpu(ds)
    for i in range(ds.ntmpl):
        assert_2f_parity(gpu[i], ref[i], f"tiny tmpl {i}")
    # the template at the injected spin-down recovers the injection
    inj = ds.injections[0]
    i5 = int(np.argmin(np.abs(ds.templates[:, 3] - inj["f1dot"])))
    fpk = ds.bin_frequencies()[int(np.argmax(gpu[i5]))]
    assert abs(fpk - inj["f"]) < 2.0 / (ds.n_fft * ds.dt)
    assert gpu[i5].max() > 0.8 * inj["rho2"]


def test_batched_equals_plain_and_deterministic(torch_dev):
    ds = synth.small_case(**dict(CASES["binary"], ntmpl=7))
    plain = run_gpu(ds)
    again = run_gpu(ds)
    batched = run_gpu(ds, batched=True, batch=3)
    np.testing.assert_array_equal(plain, again)
    np.testing.assert_array_equal(plain, batched)


def test_invalid_templates_give_nan_rows(torch_dev):
    ds = synth.small_case(**dict(CASES["one_det"], ntmpl=4))
    tm = ds.templates.copy()
    tm[1, 3] = np.nan                 # non-finite parameter
    tm[2, 5], tm[2, 6] = 0.3, -5.0    # binary with a negative period
    gpu = run_gpu(ds, templates=tm)
    assert np.all(np.isnan(gpu[1])) and np.all(np.isnan(gpu[2]))
    ref = O.oracle_twoF(ds, tm[[0, 3]])
    assert_2f_parity(gpu[0], ref[0], "valid row 0")
    assert_2f_parity(gpu[3], ref[1], "valid row 3")


def test_delay_bound_violation_gives_nan(torch_dev):
    """A binary delay beyond the plan's max_delay breaks the grid coverage the
    plan was sized for: the template is flagged, not silently truncated."""
    ds = synth.small_case(**dict(CASES["one_det"], ntmpl=2))
    tm = ds.templates.copy()
    # a 3000 light-s orbit near its extremum R = -3000 s: the last samples map
    # beyond the grid the plan computes
    porb = 1.0e7
    tm[1, 5], tm[1, 6], tm[1, 7] = 3000.0, porb, 6000.0 + porb / 4
    gpu = run_gpu(ds, templates=tm)
    assert np.all(np.isfinite(gpu[0]))
    assert np.all(np.isnan(gpu[1]))


@pytest.mark.parametrize("tune", [
    dict(tune_col_lines=32),                         # full column line count: same arithmetic
    dict(tune_row_lines=4),                          # half row count: same arithmetic
    dict(tune_col_log_len=10),                       # other split of 2^19
    dict(tune_fft_radix=16),                         # 3-stage plans for 2^9 and 2^10 lines
    dict(tune_fft_radix=16, tune_col_lines=32, tune_row_lines=4),
])
def test_fft_launch_shapes(torch_dev, tune):
    """n_fft = 2^19 (columns 2^9 x rows 2^10 by default: both lengths where the
    radix-32 and radix-16 stage plans differ) in several launch shapes."""
    from paper_2201_00451_amd import binding
    say(f"launch shape {tune}")
    ds = synth.small_case(**dict(CASES["two_det_gaps"], n=3000, n_fft=1 << 19, ntmpl=3))
    base = run_gpu(ds)
    dd = binding.DeviceData(ds, tune=tune, batch=2)
    got = binding.compute_2f_batched(dd, ds.templates).cpu().numpy()
    binding.sync_check()
    if "tune_col_log_len" not in tune and "tune_fft_radix" not in tune:
        np.testing.assert_array_equal(got, base)
    ref = O.oracle_twoF(ds)
    for i in range(ds.ntmpl):
        assert_2f_parity(got[i], ref[i], f"{tune} tmpl {i}")


def grouped_bank(ds, nsky=3, nf1=5, binary_rows=2):
    """Sky x spin-down bank (spin-down fastest) plus a short binary run."""
    base = ds.templates[0]
    rows = []
    for sky in range(nsky):
        for f1 in range(nf1):
            r = base.copy()
            r[0] += 0.03 * sky
            r[3] = base[3] + 1e-10 * (f1 - nf1 // 2)
            r[2] = 2e-6 * f1
            rows.append(r)
    for b in range(binary_rows):
        r = base.copy()
        r[5], r[6], r[7] = 0.2, 0.4 * 86400, 500.0
        r[3] = base[3] + 1e-10 * b
        rows.append(r)
    return np.array(rows)


@pytest.mark.parametrize("slots", [1, 4, 8])
def test_search_grouped_equals_plain(torch_dev, slots):
    """Shared resampling per sky/orbit group gives the per-template result bit
    for bit, also when groups span launch sequences and for a template whose
    own spin-down parameter is invalid (only its row is NaN)."""
    from paper_2201_00451_amd import binding
    ds = synth.small_case(seed=41, n=5000, n_fft=1 << 13, ndet=2, gaps=True, ntmpl=1)
    tm = grouped_bank(ds)
    tm[7, 3] = np.nan
    dd = binding.DeviceData(ds)
    plain = binding.compute_2f(dd, tm).cpu().numpy()
    binding.sync_check()
    sr = binding.Search(dd, tm, slots=slots)
    assert sr.ngroups == 4
    got = sr.run().cpu().numpy()
    binding.sync_check()
    np.testing.assert_array_equal(got, plain)
    assert np.all(np.isnan(got[7])) and np.isfinite(got[6]).all() and np.isfinite(got[8]).all()
    ref = O.oracle_twoF(ds, tm[[0, 16]])
    assert_2f_parity(got[0], ref[0], "grouped sky 0")
    assert_2f_parity(got[16], ref[1], "grouped binary")


def test_search_graph_replays(torch_dev):
    """The captured launch sequence replays correctly several times, with other
    work on the device in between."""
    import torch
    from paper_2201_00451_amd import binding
    ds = synth.small_case(seed=42, n=4000, n_fft=1 << 13, ndet=2, ntmpl=1)
    tm = grouped_bank(ds, nsky=2, nf1=4, binary_rows=1)
    dd = binding.DeviceData(ds)
    eager = binding.compute_2f(dd, tm).cpu().numpy()
    torch.cuda.synchronize()
    sr = binding.Search(dd, tm, slots=4, graph=True)
    s = torch.cuda.Stream()
    out = torch.empty((tm.shape[0], ds.n_bins), dtype=torch.float32, device=dd.device)
    for rep in range(4):
        out.fill_(-1.0)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            sr.run(out=out, stream=s)
        s.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), eager)
        # unrelated eager work between replays
        binding.compute_2f(dd, tm[:2])
        torch.cuda.synchronize()


def nearest_template(ds):
    """Index of the template closest to the first injection, in units of the
    bank's own spacing along each parameter that varies."""
    inj = ds.injections[0]
    tm = ds.templates
    target = np.array([inj["alpha"], inj["delta"], 0.0, inj["f1dot"], 0.0,
                       inj.get("asini", 0.0), inj.get("porb", 1.0), inj.get("tp", 0.0)])
    cost = np.zeros(len(tm))
    for c in (0, 1, 3, 5, 6, 7):
        vals = np.unique(tm[:, c])
        if len(vals) < 2:
            continue
        cost += np.abs(tm[:, c] - target[c]) / np.min(np.diff(vals))
    return int(np.argmin(cost))


def test_full_size_bench_workload_sampled(torch_dev):
    """The benchmark workload at full size (2 detectors x 864 000 samples,
    1000 templates, n_fft 2^21, full band), run as the benchmark runs it
    (grouped search, 32 slots: launch sequences of 30, default launch
    shapes): two whole templates
    (2 097 152 bins each: the first one and the one nearest an injection)
    against the oracle."""
    from paper_2201_00451_amd import binding
    ds = synth.config_sky_spindown()
    dd = binding.DeviceData(ds)
    sr = binding.Search(dd, ds.templates, slots=32)
    tf = sr.run()
    binding.sync_check()
    pick = [0, nearest_template(ds)]
    say(f"  full-size bench workload: templates {pick}")
    ref = O.oracle_twoF(ds, ds.templates[pick])
    for i, t in enumerate(pick):
        assert_2f_parity(tf[t].cpu().numpy(), ref[i], f"bench workload template {t}")
    assert ref[1].max() > 30.0


def test_max_fft_length_2e24(torch_dev):
    """n_fft = 2^24, the largest the plan accepts (columns and rows of 2^12,
    both FFT passes in their half-LDS form), where the oracle's full-grid
    timing takes minutes: checked by a property that holds at any size.  The
    same data zero-padded to 2^24 has the 2^23 spectrum at its even bins
    (bin 2m lies at the frequency of 2^23 bin m); the 2^23 path meets the bar
    against the oracle at full size.  Also: the grouped search equals the
    per-template path bit for bit, and candidate retention equals the
    thresholded band."""
    import torch
    from paper_2201_00451_amd import binding
    kw = dict(seed=41, n=20000, ndet=2, binary=True, gaps=True, ntmpl=2, rho=20.0)
    ds24 = synth.small_case(n_fft=1 << 24, **kw)
    ds23 = synth.small_case(n_fft=1 << 23, **kw)
    dd24 = binding.DeviceData(ds24, batch=2)
    tf24 = binding.compute_2f(dd24, ds24.templates)
    sr = binding.Search(dd24, ds24.templates, slots=2)
    full = sr.run()
    binding.sync_check()
    assert torch.equal(full, tf24)
    thr = float(np.float32(0.5 * float(full.max())))
    res = sr.run_candidates(thr, capacity=1 << 16)
    binding.sync_check()
    want = torch.nonzero(full > thr)
    assert res["count"] == want.shape[0] > 0
    got = set(zip(res["tmpl"].cpu().numpy().tolist(), res["bin"].cpu().numpy().tolist()))
    assert got == set(map(tuple, want.cpu().numpy().tolist()))
    assert torch.equal(res["best_twoF"], torch.max(full, dim=1)[0])
    even = tf24[:, 0::2].cpu().numpy()
    del dd24, sr, full, tf24, res
    torch.cuda.empty_cache()
    dd23 = binding.DeviceData(ds23, batch=2)
    tf23 = binding.compute_2f(dd23, ds23.templates).cpu().numpy()
    binding.sync_check()
    for t in range(2):
        say(f"  2^24 template {t}: peak 2F {even[t].max():.2f}")
        assert_2f_parity(even[t], tf23[t].astype(np.float64), f"2^24 even bins, template {t}")
    assert tf23.max() > 30.0


def test_full_size_binary_workload_sampled(torch_dev):
    """The binary workload at full size (2 detectors x 5 184 000 samples at 70%
    duty, n_fft 2^23, full band): 32 lattice templates around the injection in
    one batched call; the one nearest the injection against the oracle over
    all 8 388 608 bins."""
    from paper_2201_00451_amd import binding
    ds = synth.config_binary()
    t0 = nearest_template(ds)
    lo = max(0, t0 - 16)
    rows = ds.templates[lo:lo + 32]
    dd = binding.DeviceData(ds, batch=8)
    tf = binding.compute_2f_batched(dd, rows)
    binding.sync_check()
    say(f"  full-size binary workload: template {t0}")
    ref = O.oracle_twoF(ds, ds.templates[[t0]])[0]
    assert_2f_parity(tf[t0 - lo].cpu().numpy(), ref, f"binary workload template {t0}")
    assert ref.max() > 30.0
    # as the benchmark runs it: grouped search (32 slots) keeping the bins
    # above a threshold and the loudest bin, equal to the thresholded band bit
    # for bit
    import torch
    thr = float(np.float32(0.5 * float(tf.max())))
    sr = binding.Search(dd, rows, slots=32)
    res = sr.run_candidates(thr, capacity=1 << 16)
    binding.sync_check()
    want = torch.nonzero(tf > thr)
    assert res["count"] == want.shape[0] > 0
    got = set(zip(res["tmpl"].cpu().numpy().tolist(), res["bin"].cpu().numpy().tolist()))
    assert got == set(map(tuple, want.cpu().numpy().tolist()))
    best, arg = torch.max(tf, dim=1)
    assert torch.equal(res["best_twoF"], best)
    np.testing.assert_array_equal(res["twoF"].cpu().numpy(),
                                  tf[res["tmpl"].long(), res["bin"].long()].cpu().numpy())


def test_autotuned_launch_shape(torch_dev):
    """The autotuner returns a launch shape the plan accepts, and 2F computed
    with it meets the bar against the oracle."""
    from paper_2201_00451_amd import binding
    ds = synth.small_case(**dict(CASES["two_det_gaps"], n=3000, n_fft=1 << 13, ntmpl=3))
    tune, ms = binding.autotune(ds, ds.templates, batch=2)
    say(f"  autotuned {tune} in {ms:.3f} ms")
    assert ms > 0.0 and tune["tune_col_log_len"] in (6, 7)
    assert tune["tune_fft_radix"] in (16, 32)
    dd = binding.DeviceData(ds, tune=tune, batch=2)
    got = binding.compute_2f_batched(dd, ds.templates).cpu().numpy()
    binding.sync_check()
    ref = O.oracle_twoF(ds)
    for i in range(ds.ntmpl):
        assert_2f_parity(got[i], ref[i], f"autotuned tmpl {i}")


def test_autotuned_search_shape_and_cache(torch_dev, tmp_path):
    """The search-path autotuner (median of three timed searches per shape)
    returns a shape the plan accepts, writes it to the cache, and a second
    call takes it from there without timing; a search with the shape meets
    the bar against the oracle."""
    from paper_2201_00451_amd import binding
    ds = synth.small_case(**dict(CASES["binary"], n=3000, n_fft=1 << 13, ntmpl=4))
    dd = binding.DeviceData(ds)
    cache = tmp_path / "tune.jsonl"
    tune, ms, hit = binding.autotune_search(dd, ds.templates, slots=2, repeats=3, cache=cache)
    say(f"  search-path autotune {tune}, median {ms:.3f} ms, cached {hit}")
    assert not hit and ms > 0.0
    assert tune["tune_col_log_len"] in (6, 7) and tune["tune_fft_radix"] in (16, 32)
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and '"tune": [' in lines[0]
    tune2, ms2, hit2 = binding.autotune_search(dd, ds.templates, slots=2, repeats=3,
                                               cache=cache)
    assert hit2 and tune2 == tune and abs(ms2 - ms) <= 1e-5 * ms
    assert len(cache.read_text().splitlines()) == 1
    dd2 = binding.DeviceData(ds, tune=tune)
    got = binding.Search(dd2, ds.templates, slots=2).run().cpu().numpy()
    binding.sync_check()
    ref = O.oracle_twoF(ds)
    for i in range(ds.ntmpl):
        assert_2f_parity(got[i], ref[i], f"search-autotuned tmpl {i}")


def test_second_spindown_term_grouped_and_peak(torch_dev):
    """f2dot moving the phase by several cycles over the data: a sky group of
    templates that differ only in f2dot (one shared resampled series, each
    template's cubic spin-down phase applied as the column pass loads it)
    equals the per-template path bit for bit and the oracle to the bar, and
    the template at the injected f2dot recovers the injection."""
    from paper_2201_00451_amd import binding
    ds = synth.small_case(**dict(CASES["f2dot"], ntmpl=1))
    inj = ds.injections[0]
    T = ds.detectors[0].n * ds.dt
    rows = np.repeat(ds.templates[:1], 5, axis=0)
    rows[:, 4] = inj["f2dot"] + (np.arange(5) - 2) * 6.0 / T ** 3
    dd = binding.DeviceData(ds)
    plain = binding.compute_2f(dd, rows).cpu().numpy()
    sr = binding.Search(dd, rows, slots=4)
    assert sr.ngroups == 1
    got = sr.run().cpu().numpy()
    binding.sync_check()
    np.testing.assert_array_equal(got, plain)
    ref = O.oracle_twoF(ds, rows[[0, 2]])
    assert_2f_parity(got[0], ref[0], "f2dot off by -12 cycles T^-3")
    assert_2f_parity(got[2], ref[1], "f2dot at the injection")
    say(f"  peak 2F by f2dot offset: {np.round(got.max(axis=1), 2)}; rho^2 {inj['rho2']:.1f}")
    assert int(np.argmax(got.max(axis=1))) == 2
    assert got[2].max() > 0.8 * inj["rho2"]


def test_keplerian_grouped_equals_plain(torch_dev):
    """Keplerian orbits on the grouped path: templates that share an orbit
    share its resampled series (a different eccentricity or argument of
    periapsis starts a new group), bit for bit as the per-template path."""
    from paper_2201_00451_amd import binding
    ds = synth.small_case(**dict(CASES["kepler"], ntmpl=1))
    base = ds.templates[0]
    rows = np.repeat(base[None], 6, axis=0)
    rows[:, 3] += 1e-10 * np.array([0, 1, 0, 1, 0, 1])
    rows[2:4, 8] += 0.05
    rows[4:6, 9] += 0.1
    dd = binding.DeviceData(ds)
    plain = binding.compute_2f(dd, rows).cpu().numpy()
    sr = binding.Search(dd, rows, slots=4)
    assert sr.ngroups == 3
    got = sr.run().cpu().numpy()
    binding.sync_check()
    np.testing.assert_array_equal(got, plain)
    ref = O.oracle_twoF(ds, rows[[0, 5]])
    assert_2f_parity(got[0], ref[0], "kepler group 0")
    assert_2f_parity(got[5], ref[1], "kepler group 2")
    inj = ds.injections[0]
    say(f"  peak 2F at the injected orbit {got[0].max():.2f}, rho^2 {inj['rho2']:.1f}")
    assert got[0].max() > 0.8 * inj["rho2"]
