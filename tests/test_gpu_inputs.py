"""Inputs, captured graphs and flagged templates, through the C ABI.

* A captured search or batch replays only while every input it baked into
  its kernel arguments is the same: a new detector-1 series or a new
  ephemeris table captures again and gives the eager result on the new data.
* An isolated template (asini = 0) ignores porb and tp whatever they hold,
  also as the leader of a sky group.
* A reference time far from the data (spin-down phase of ~1e9 cycles at the
  grid origin) keeps parity with the oracle.
* fstat_flagged_count reports the templates set to NaN by the last call.
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


def parity(gpu, ref, label):
    gpu = np.asarray(gpu, dtype=np.float64)
    strong = ref >= 10.0
    rel = np.abs(gpu[strong] - ref[strong]) / ref[strong] if strong.any() else np.zeros(1)
    ab = np.abs(gpu[~strong] - ref[~strong])
    say(f"  {label}: max rel {rel.max():.3e}, max abs {ab.max():.3e}")
    assert rel.max() <= 1e-4 and ab.max() <= 1e-3


def bank(ds, nsky=2, nf1=3):
    base = ds.templates[0]
    rows = []
    for s in range(nsky):
        for f in range(nf1):
            r = base.copy()
            r[0] += 0.02 * s
            r[3] += 1e-10 * (f - 1)
            rows.append(r)
    return np.array(rows)


def test_graph_recaptures_on_new_series_and_ephemeris(torch_dev):
    torch = torch_dev
    from paper_2201_00451_amd import binding
    ds = synth.small_case(seed=71, n=4000, n_fft=1 << 13, ndet=2, ntmpl=1)
    other = synth.small_case(seed=71, n=4000, n_fft=1 << 13, ndet=2, ntmpl=1, noise_seed=99)
    rows = bank(ds)
    dd = binding.DeviceData(ds)
    sr = binding.Search(dd, rows, slots=4, graph=True)
    st = torch.cuda.Stream()
    out = torch.empty((rows.shape[0], ds.n_bins), dtype=torch.float32, device=dd.device)

    def graph_run():
        out.fill_(-1.0)
        torch.cuda.synchronize()
        with torch.cuda.stream(st):
            sr.run(out=out, stream=st)
        st.synchronize()
        return out.cpu().numpy()

    first = graph_run()
    np.testing.assert_array_equal(first, binding.compute_2f(dd, rows).cpu().numpy())
    # detector 1's series replaced (the old tensor stays alive)
    old_x1 = dd.x[1]
    new_x1 = torch.from_numpy(np.ascontiguousarray(other.x[1])).to(dd.device)
    dd.inputs.x[1] = new_x1.data_ptr()
    got = graph_run()
    eager = binding.compute_2f(dd, rows).cpu().numpy()
    binding.sync_check()
    np.testing.assert_array_equal(got, eager)
    assert not np.array_equal(got, first)
    # a different ephemeris table for detector 0 (positions moved by 1 ms)
    eph = dd.ephem[0].clone()
    eph[:, 0] += 1e-3
    dd.inputs.ephem[0] = eph.data_ptr()
    got2 = graph_run()
    eager2 = binding.compute_2f(dd, rows).cpu().numpy()
    binding.sync_check()
    np.testing.assert_array_equal(got2, eager2)
    assert not np.array_equal(got2, got)
    del old_x1


def test_batch_recaptures_on_new_series(torch_dev):
    torch = torch_dev
    from paper_2201_00451_amd import binding
    dss = [synth.small_case(seed=72 + i, n=3000, n_fft=1 << 13, ndet=2, ntmpl=1)
           for i in range(2)]
    other = synth.small_case(seed=72, n=3000, n_fft=1 << 13, ndet=2, ntmpl=1, noise_seed=98)
    srs = [binding.Search(binding.DeviceData(d), bank(d), slots=4) for d in dss]
    batch = binding.Batch(srs, lanes=2)
    outs = [torch.empty((s.ntmpl, s.dd.n_bins), dtype=torch.float32, device=s.dd.device)
            for s in srs]
    first = [o.cpu().numpy() for o in batch.run(outs)]
    # only detector 1's series of search 0 changes: the batch captures again
    new_x1 = torch.from_numpy(np.ascontiguousarray(other.x[1])).to(srs[0].dd.device)
    srs[0].dd.inputs.x[1] = new_x1.data_ptr()
    for o in outs:
        o.fill_(-1.0)
    torch.cuda.synchronize()
    again = [o.cpu().numpy() for o in batch.run(outs)]
    eager = binding.compute_2f(srs[0].dd, bank(dss[0])).cpu().numpy()
    binding.sync_check()
    np.testing.assert_array_equal(again[0], eager)
    np.testing.assert_array_equal(again[1], first[1])
    assert not np.array_equal(again[0], first[0])


def test_isolated_leader_ignores_orbit_fields(torch_dev):
    """porb and tp of an isolated template are placeholders: NaN there flags
    nothing, for the plain path and for a sky group it leads."""
    from paper_2201_00451_amd import binding
    ds = synth.small_case(seed=73, n=4000, n_fft=1 << 13, ndet=2, gaps=True, ntmpl=1)
    rows = bank(ds, nsky=1, nf1=3)
    rows[0, 6], rows[0, 7] = np.nan, np.nan
    rows[1, 6] = -3.0
    dd = binding.DeviceData(ds)
    plain = binding.compute_2f(dd, rows).cpu().numpy()
    sr = binding.Search(dd, rows, slots=4)
    assert sr.ngroups == 1
    got = sr.run().cpu().numpy()
    binding.sync_check()
    assert np.all(np.isfinite(plain))
    np.testing.assert_array_equal(got, plain)
    clean = rows.copy()
    clean[:, 6], clean[:, 7] = 1.0, 0.0
    np.testing.assert_array_equal(binding.compute_2f(dd, clean).cpu().numpy(), plain)
    ref = O.oracle_twoF(ds, clean[:1])
    parity(got[0], ref[0], "isolated leader with NaN orbit fields")


def test_distant_reference_time(torch_dev):
    """t_ref 1.3e9 s before the data (a GPS-era epoch against data at t = 0)
    with f1dot 1e-9: the spin-down phase at the grid origin is ~8e8 cycles
    (3.4e9 quarter turns, beyond 32 bits)."""
    from paper_2201_00451_amd import binding
    ds = synth.small_case(seed=74, n=4000, n_fft=1 << 13, ndet=1, ntmpl=2)
    ds.t_ref = -1.3e9
    rows = ds.templates.copy()
    rows[:, 3] = [1e-9, -7e-10]
    rows[:, 2] = [0.0, 3e-6]
    dd = binding.DeviceData(ds)
    got = binding.compute_2f(dd, rows).cpu().numpy()
    sr = binding.Search(dd, rows, slots=2)
    grouped = sr.run().cpu().numpy()
    binding.sync_check()
    np.testing.assert_array_equal(grouped, got)
    ref = O.oracle_twoF(ds, rows)
    for i in range(2):
        parity(got[i], ref[i], f"t_ref -1.3e9 s, template {i}")


def test_flagged_count(torch_dev):
    from paper_2201_00451_amd import binding
    ds = synth.small_case(seed=75, n=3000, n_fft=1 << 13, ndet=1, ntmpl=5)
    rows = ds.templates.copy()
    rows[1, 3] = np.nan                       # spin-down not finite
    rows[3, 5], rows[3, 6] = 0.2, -1.0        # binary with a negative period
    dd = binding.DeviceData(ds, batch=2)
    tf = binding.compute_2f(dd, rows)
    assert binding.flagged_count(dd.ws) == 2
    binding.compute_2f_batched(dd, rows[[0, 2, 4]])
    assert binding.flagged_count(dd.ws) == 0
    sr = binding.Search(dd, rows, slots=4)
    sr.run()
    assert binding.flagged_count(sr.ws) == 2
    sr.run_candidates(1e9, capacity=16)
    assert binding.flagged_count(sr.ws) == 2
    g, tfb = binding.compute_2f_grad_bin(dd, rows, np.full(5, 100))
    assert binding.flagged_count(dd.grad_bin_ws) == 2
    binding.sync_check()
    bad = np.isnan(tf.cpu().numpy()).all(axis=1)
    assert list(np.nonzero(bad)[0]) == [1, 3]
