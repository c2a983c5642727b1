#!/usr/bin/env python3
"""Throughput of the resampling F-statistic on one MI355X.

Workload (the plain method at scale): two detectors, 10 days at 1 s
(864 000 samples each) around 150 Hz with ten 1800 s gaps each, noise
variance U(0.8, 1.2), three injections; 1000 templates (10 x 10 sky patch x
10 spin-downs); n_fft = 2^21, full-band 2F (2 097 152 bins per template).
A step is one pass of the whole hot path (barycentring, resampling,
antenna weighting, FFT, 2F) over all 1000 templates with the inputs already
resident in HBM.

Prints one JSON line.  ``value`` is templates/s of the batched path; the plain
per-template path, per-kernel device times (HIP events on the library's
stream), the HBM roofline of the dominant kernel and the FP64 oracle timed on
the host cores on a bounded sample are reported beside it.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "templates/s (full-band 2F) & % HBM roofline, batched vs plain, rel err ≤1e-4"


# HBM traffic of the two FFT passes per template on this workload, measured
# with rocprofv3 FETCH_SIZE and WRITE_SIZE runs of this benchmark (summary and
# commands in profiles/search_bench_workload_2e21.md; FETCH_SIZE scaled by 2.0
# and WRITE_SIZE by 1.0, the factors a plain 512 MiB device copy gives).  The
# figures hold for the kernel sources, header and build flags with this
# digest; for any other version the roofline reports traffic as null.
MEASURED_TRAFFIC = {
    "sources_sha256": "b3e4756cced3d056b429362ae8adba94261d366587cac560985c818495d5add0",
    "bytes_per_template": {"fft_columns": 13881424 + 33759698,
                           "fft_rows_2f": 33563484 + 8416371},
}


def sources_digest():
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2201_00451_amd", "csrc")
    for fn in sorted(os.listdir(csrc)):
        h.update(fn.encode())
        with open(os.path.join(csrc, fn), "rb") as f:
            h.update(f.read())
    for fn in ("include/fstat.h", "paper_2201_00451_amd/build.py"):
        h.update(fn.encode())
        with open(os.path.join(ROOT, fn), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def step_bytes(ds, k_pad, n_resampled):
    """Algorithmic HBM bytes of one step, per kernel.

    resample: read every input series once (8 B/sample/detector) and write the
      two resampled series on the computed grid (2 x k_pad x 8 B), once per
      resampled series (per sky/orbit group on the grouped path);
    fft_columns: read the two series on the computed grid (2 x k_pad x 8 B) and
      write the full column-transformed arrays (2 x n_fft x 8 B), per template;
    fft_rows_2f: read those (2 x n_fft x 8 B) and write 2F (4 B/bin), per template."""
    n_in = sum(d.n for d in ds.detectors)
    return {
        "prologue": ds.ntmpl * 1024,
        "resample": n_resampled * (8 * n_in + 2 * 8 * k_pad),
        "fft_columns": ds.ntmpl * (2 * 8 * k_pad + 2 * 8 * ds.n_fft),
        "fft_rows_2f": ds.ntmpl * (2 * 8 * ds.n_fft + 4 * ds.n_bins),
    }


def cpu_baseline(ds, ntmpl):
    """The FP64 oracle on the first ntmpl templates, single-threaded."""
    from threadpoolctl import threadpool_limits
    from oracle import fstat_oracle as O
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        O.oracle_twoF(ds, ds.templates[:ntmpl])
        el = time.perf_counter() - t0
    return {"value": ntmpl / el, "unit": "templates/s", "cores": 1, "kind": "oracle",
            "sample": f"{ntmpl} of the {ds.ntmpl} templates, full band, "
                      f"{el:.1f} s on one host core (numpy float64)"}


def refinement_leg(steps, refine_steps):
    """The single-bin adjoint on the refinement workload (2 detectors x 30 d
    at 1 s, 0.2 Hz band at 400 Hz, 64 binary candidates 0.3-1 metric spacing
    from 8 injections): gradient evaluations per second, and a short
    preconditioned ascent with the recovered fraction of the 2F at the true
    parameters."""
    import math
    import numpy as np
    import torch
    from paper_2201_00451_amd import binding, synth
    ds = synth.config_refine()
    dd = binding.DeviceData(ds)
    rows, bins = ds.templates, ds.cand_bins
    n = len(rows)
    binding.compute_2f_grad_bin(dd, rows, bins)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        binding.compute_2f_grad_bin(dd, rows, bins)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    # 2F at the injections' own parameters, in each candidate's bin
    truth = rows.copy()
    T = ds.detectors[0].n * ds.dt
    scales = np.zeros((n, 7))
    for m in range(n):
        inj = ds.injections[ds.cand_inj[m]]
        nat = bins[m] + ds.bin_lo - ds.n_fft // 2
        truth[m, 2] = (inj["f"] - ds.f_het) - nat / (ds.n_fft * ds.dt)
        truth[m, 5], truth[m, 6], truth[m, 7] = inj["asini"], inj["porb"], inj["tp"]
        om = 2 * math.pi / inj["porb"]
        scales[m] = [1.0 / T, 1.0 / T ** 2, 1e-3, 1e-3, 1.0 / (2 * math.pi * inj["f"]),
                     inj["porb"] ** 2 / (2 * math.pi * inj["f"] * inj["asini"] * T),
                     1.0 / (2 * math.pi * inj["f"] * inj["asini"] * om)]
    _, tf_true = binding.compute_2f_grad_bin(dd, truth, bins)
    _, tf_start = binding.compute_2f_grad_bin(dd, rows, bins)
    tf_true = tf_true.cpu().numpy()
    tf_start = tf_start.cpu().numpy()
    t0 = time.perf_counter()
    _, vals = binding.refine(dd, rows, bins, scales, steps=refine_steps,
                             free=("df", "asini", "porb", "tp"))
    el = time.perf_counter() - t0
    return {"workload": "2 detectors x 2592000 samples, n_fft 2^22, 0.2 Hz band at 400 Hz, "
                        "64 binary candidates", "candidates": n,
            "grad_evals_per_s": round(n / (ms / 1e3), 1), "ms_per_call": round(ms, 3),
            "refine_steps": refine_steps, "refine_wall_s": round(el, 2),
            "median_2F_start_over_true": round(float(np.median(tf_start / tf_true)), 4),
            "median_2F_end_over_true": round(float(np.median(vals / tf_true)), 4),
            "min_2F_end_over_true": round(float(np.min(vals / tf_true)), 4)}


def uneven_leg(n_search, steps):
    """Independent searches of uneven span, band, FFT length and detector
    count (spans log-uniform in 1-30 d, dt in {0.5, 1, 2, 5} s, n_fft 2^16 to
    2^22, 8-64 templates each), run one after the other and as one captured
    batch over 4 branches."""
    import torch
    from paper_2201_00451_amd import binding, synth
    dss = synth.config_uneven(seed=4, n_search=n_search)
    srs = [binding.Search(binding.DeviceData(ds), ds.templates, slots=8) for ds in dss]
    outs = [torch.empty((sr.ntmpl, ds.n_bins), dtype=torch.float32, device="cuda")
            for sr, ds in zip(srs, dss)]
    ntmpl = sum(sr.ntmpl for sr in srs)
    nbins = sum(sr.ntmpl * ds.n_bins for sr, ds in zip(srs, dss))
    batch = binding.Batch(srs, lanes=4)
    st = torch.cuda.Stream()

    def run_seq():
        with torch.cuda.stream(st):
            for sr, o in zip(srs, outs):
                sr.run(out=o, stream=st)

    def run_batch():
        batch.run(outs, stream=st)

    res = {}
    for name, fn in (("sequential", run_seq), ("batch", run_batch)):
        fn()
        st.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(steps):
            fn()
        e1.record(st)
        st.synchronize()
        ms = e0.elapsed_time(e1) / steps
        res[name] = {"ms_per_step": round(ms, 3), "templates_per_s": round(ntmpl / (ms / 1e3), 1),
                     "bins_per_s": float(f"{nbins / (ms / 1e3):.4g}")}
    binding.sync_check()
    return {"workload": f"{n_search} searches: spans log-uniform 1-30 d, dt in 0.5-5 s, "
                        "1 or 2 detectors, n_fft 2^16-2^22, full band, 8-64 templates each",
            "searches": n_search, "templates": ntmpl, "n_fft_range": [min(d.n_fft for d in dss),
                                                                      max(d.n_fft for d in dss)],
            "steps": steps, **res,
            "batch_over_sequential": round(res["sequential"]["ms_per_step"] /
                                           res["batch"]["ms_per_step"], 3)}


def workload_leg(name):
    """Other workloads of the grouped search.  tiny: one timed step after an
    untimed one, full-band 2F.  binary: the full bank with candidate
    retention on the device (threshold 70, the paper's pilot search; the
    full band of 10^4 templates at 2^23 bins would take 335 GB), one timed
    step after an untimed one, plus the per-kernel split from a profiled
    full-band run of the first 256 templates."""
    import torch
    from paper_2201_00451_amd import binding, synth
    ds = {"tiny": synth.config_tiny, "binary": synth.config_binary}[name]()
    dd = binding.DeviceData(ds, batch=1)
    slots = min(32, ds.ntmpl)
    sr = binding.Search(dd, ds.templates, slots=slots)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res = {"templates": ds.ntmpl, "n_fft": ds.n_fft, "detectors": ds.ndet,
           "samples_per_detector": ds.detectors[0].n, "sky_orbit_groups": sr.ngroups,
           "slots": slots}
    if name == "binary":
        sr.run_candidates(70.0, capacity=1 << 20)
        torch.cuda.synchronize()
        e0.record(st)
        c = sr.run_candidates(70.0, capacity=1 << 20)
        e1.record(st)
        torch.cuda.synchronize()
        res["output"] = "candidates 2F > 70"
        res["candidates"] = c["count"]
        sub = binding.Search(dd, ds.templates[:256], slots=slots)
        out = torch.empty((256, ds.n_bins), dtype=torch.float32, device=dd.device)
        sub.run_profiled(out=out)
        _, kt = sub.run_profiled(out=out)
        nk = 256
        del out, sub
    else:
        out = torch.empty((ds.ntmpl, ds.n_bins), dtype=torch.float32, device=dd.device)
        sr.run_profiled(out=out)
        torch.cuda.synchronize()
        e0.record(st)
        _, kt = sr.run_profiled(out=out)
        e1.record(st)
        torch.cuda.synchronize()
        res["output"] = "full band"
        nk = ds.ntmpl
    ms = e0.elapsed_time(e1)
    binding.sync_check()
    res.update({"ms_per_step": round(ms, 3), "templates_per_s": round(ds.ntmpl / (ms / 1e3), 1),
                "us_per_template": {k: round(v[0] * 1e3 / nk, 3) for k, v in kt.items()}})
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=32, help="templates in flight per launch")
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--graph-steps", type=int, default=5)
    ap.add_argument("--cand-steps", type=int, default=5,
                    help="timed steps of the candidate-retention epilogue (0: skip)")
    ap.add_argument("--cand-threshold", type=float, default=40.0)
    ap.add_argument("--uneven-searches", type=int, default=64,
                    help="independent searches of uneven shape run as one captured batch "
                         "(0: skip)")
    ap.add_argument("--uneven-steps", type=int, default=3)
    ap.add_argument("--other-workloads", type=int, default=1,
                    help="also time the tiny (1 detector, 1 d, 2^17) and binary (2 detectors, "
                         "120 d, 2^23, 10^4 orbits) workloads, one step each (0: skip)")
    ap.add_argument("--cpu-templates", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--refine-calls", type=int, default=10,
                    help="timed single-bin gradient calls on the refinement workload (0: skip)")
    ap.add_argument("--refine-steps", type=int, default=30)
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="after the measurements, run one plain device copy of this many MiB "
                         "(a reference kernel of known traffic for hardware counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library runs the whole search on a single "
              "MI355X (templates would shard across GPUs with no exchange step); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2201_00451_amd import binding, synth

    print("bench: generating the 10 d, 2-detector, 1000-template workload", file=sys.stderr,
          flush=True)
    ds = synth.config_sky_spindown()
    dd = binding.DeviceData(ds, batch=args.batch)
    tm = torch.from_numpy(ds.templates).to(dd.device)
    out = torch.empty((ds.ntmpl, ds.n_bins), dtype=torch.float32, device=dd.device)
    stream = torch.cuda.current_stream()
    k_pad, _, _ = dd.plan.info()

    sr = binding.Search(dd, ds.templates, slots=args.batch)
    print(f"bench: {ds.ntmpl} templates in {sr.ngroups} sky/orbit groups, "
          f"{sr.nchunks} launch sequences of at most {args.batch} templates (whole groups)",
          file=sys.stderr, flush=True)

    print("bench: warmup", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        sr.run_profiled(out=out)
    torch.cuda.synchronize()

    # timed region: K steps of the grouped batched path, per-kernel HIP events
    # recorded on the library's stream around every launch
    print(f"bench: timing {args.steps} steps", file=sys.stderr, flush=True)
    totals = {k: [0.0, 0] for k in binding.KERNELS}
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    t_wall = time.perf_counter()
    for _ in range(args.steps):
        _, kt = sr.run_profiled(out=out)
        for k, (ms, n) in kt.items():
            totals[k][0] += ms
            totals[k][1] += n
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ms_total = ev0.elapsed_time(ev1)
    ms_step = ms_total / args.steps
    value = ds.ntmpl * args.steps / (ms_total / 1e3)
    binding.sync_check()

    bytes_step = step_bytes(ds, k_pad, sr.ngroups)
    kern = {}
    for k, (ms, n) in totals.items():
        avg = ms / max(n, 1)
        b_launch = bytes_step[k] * args.steps / max(n, 1)
        kern[k] = {"ms_per_step": round(ms / args.steps, 4), "launches_per_step": n // args.steps,
                   "avg_us": round(avg * 1e3, 2), "bytes_per_launch": int(b_launch),
                   "gbs": round(b_launch / (avg / 1e3) / 1e9, 1) if avg > 0 else None}
    dom = max((k for k in kern if k != "prologue"), key=lambda k: totals[k][0])
    achieved = kern[dom]["gbs"]
    traffic = None
    per_t = MEASURED_TRAFFIC["bytes_per_template"].get(dom)
    if per_t is not None and sources_digest() == MEASURED_TRAFFIC["sources_sha256"]:
        traffic = int(per_t * ds.ntmpl / max(kern[dom]["launches_per_step"], 1))
    roof = {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
            "bytes_per_launch": kern[dom]["bytes_per_launch"]}

    def timed(fn, steps):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(torch.cuda.current_stream())
        for _ in range(steps):
            fn()
        e1.record(torch.cuda.current_stream())
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        return {"value": round(ds.ntmpl / (ms / 1e3), 1), "ms_per_step": round(ms, 3),
                "steps": steps}

    # the same grouped path replayed from a captured HIP graph
    graph = None
    if args.graph_steps > 0:
        print("bench: graph replay", file=sys.stderr, flush=True)
        srg = binding.Search(dd, ds.templates, slots=args.batch, graph=True)
        gs = torch.cuda.Stream()
        torch.cuda.synchronize()

        def run_graph():
            with torch.cuda.stream(gs):
                srg.run(out=out, stream=gs)
            gs.synchronize()
        run_graph()
        graph = timed(run_graph, args.graph_steps)
        del srg

    # the same search keeping only bins above a 2F threshold (and the loudest
    # bin per template) instead of writing the full band
    cand = None
    if args.cand_steps > 0:
        print("bench: candidate retention", file=sys.stderr, flush=True)
        cap = 1 << 20
        res = sr.run_candidates(args.cand_threshold, capacity=cap)
        cand = timed(lambda: sr.run_candidates(args.cand_threshold, capacity=cap),
                     args.cand_steps)
        cand.update({"threshold": args.cand_threshold, "candidates": res["count"],
                     "capacity": cap})
        del res

    # every template resampled on its own, several templates per launch
    ungrouped = None
    plain = None
    if args.plain_steps > 0:
        print("bench: ungrouped batched path", file=sys.stderr, flush=True)
        ungrouped = timed(lambda: binding.compute_2f_batched(dd, tm, out=out), args.plain_steps)
        # the plain per-template path (one template in flight, as in the paper)
        print("bench: plain path", file=sys.stderr, flush=True)
        dd1 = binding.DeviceData(ds, batch=1)
        plain = timed(lambda: binding.compute_2f(dd1, tm, out=out), args.plain_steps)
        del dd1
    binding.sync_check()

    calib = None
    if args.calibrate_copy_mib > 0:
        nbytes = args.calibrate_copy_mib << 20
        src = torch.empty(nbytes // 4, dtype=torch.float32, device=dd.device).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        calib = {"copy_bytes_read": nbytes, "copy_bytes_written": nbytes}
        del src, dst

    refine = None
    if args.refine_calls > 0:
        print("bench: single-bin adjoint on the refinement workload", file=sys.stderr, flush=True)
        refine = refinement_leg(args.refine_calls, args.refine_steps)
        binding.sync_check()

    others = None
    if args.other_workloads:
        others = {}
        for name in ("tiny", "binary"):
            print(f"bench: {name} workload", file=sys.stderr, flush=True)
            others[name] = workload_leg(name)
            torch.cuda.empty_cache()

    uneven = None
    if args.uneven_searches > 0:
        print(f"bench: {args.uneven_searches} uneven searches, sequential and batched",
              file=sys.stderr, flush=True)
        uneven = uneven_leg(args.uneven_searches, args.uneven_steps)

    cpu = None
    if not args.no_cpu_baseline:
        print("bench: FP64 oracle on the host", file=sys.stderr, flush=True)
        cpu = cpu_baseline(ds, args.cpu_templates)
        cpu["value"] = round(cpu["value"], 5)

    n_bins_total = ds.ntmpl * ds.n_bins
    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "templates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "two detectors, 10 d at 1 s (864000 samples each), 150 Hz, "
                               "1000 templates (10x10 sky x 10 spin-down), n_fft 2^21, "
                               "full band", "templates": ds.ntmpl, "n_fft": ds.n_fft,
                   "n_bins": ds.n_bins, "detectors": ds.ndet,
                   "samples_per_detector": ds.detectors[0].n,
                   "sinc_halfwidth": ds.sinc_halfwidth, "slots": args.batch,
                   "launch_sequences": sr.nchunks,
                   "timing_dtype": "f64", "path": "grouped: one resampled series per sky "
                   "position, spin-down phase applied in the FFT load",
                   "sky_orbit_groups": sr.ngroups},
        "graph_replay": graph,
        "candidates": cand,
        "batched_ungrouped": ungrouped,
        "plain": plain,
        "batched_over_plain": round(value / plain["value"], 3) if plain else None,
        "tau_eff_s_per_bin_per_det": (ms_step / 1e3) / (n_bins_total * ds.ndet),
        "kernels": kern,
        "roofline": roof,
        "cpu_baseline": cpu,
        "refinement": refine,
        "uneven_batch": uneven,
        "other_workloads": others,
        "wall_s_timed": round(wall, 3),
    }
    if calib:
        line["calibration_copy"] = calib
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
