#!/usr/bin/env python3
"""Throughput of the resampling F-statistic on one MI355X.

Headline workload (a narrowband binary-pulsar batch shaped like the pilot
search of Sec. 5): two detectors, 120 days at 2 s (5 184 000 samples each) at
70 % duty in 1800 s blocks, one band of 0.5 Hz centred in 200-600 Hz, a
circular-binary injection at rho 20, and 10^4 binary templates on a lattice in
(asini, porb, tp) around it; n_fft = 2^23 and 2F written for every one of the
8 388 608 bins of every template.  A step computes all 10^4 full bands with
the inputs already resident in HBM.  The 335 GB the bands add up to do not fit
the GPU, so the bank runs as blocks of `--ring` templates that write one
reused output array (as a search copies each block out or thresholds it);
every band is still computed and stored inside the timed region.

Prints one JSON line.  ``value`` is templates/s of the batched search path
on the headline workload; beside it: the plain per-template path on the same
workload, per-kernel device times (HIP events on the library's stream), the
HBM roofline of the dominant kernel, the error against the FP64 oracle on
sampled templates, the oracle itself timed on the host cores, and the other
workloads (sky/spin-down at 2^21, the tiny case, candidate refinement with
the adjoint, and a batch of uneven searches), each with its error against
the oracle.
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

# HBM traffic of the kernels per template, measured with rocprofv3
# FETCH_SIZE and WRITE_SIZE runs of this benchmark (summaries and commands in
# profiles/; FETCH_SIZE scaled by 2.0 and WRITE_SIZE by 1.0, the factors a
# plain 512 MiB device copy gives).  The figures hold for the kernel sources,
# header and build flags with this digest; for any other version the
# roofline reports traffic as null.
MEASURED_TRAFFIC = {
    "sources_sha256": "86893e7221d92b932e52b8eb5c6a174c272a19769c8573477d2a24167977684c",
    "bytes_per_template": {
        "binary": {"resample": 190059765, "fft_columns": 260420974, "fft_rows_2f": 231387746},
        "sky_spindown": {"resample": 3171116, "fft_columns": 48114543, "fft_rows_2f": 41978569},
    },
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


def say(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def step_bytes(ds, k_pad, n_resampled, ntmpl=None):
    """Algorithmic HBM bytes of one step, per kernel.

    resample: read every input series once (8 B/sample/detector) and write the
      two resampled series on the computed grid (2 x k_pad x 8 B), once per
      resampled series (per sky/orbit group on the grouped path);
    fft_columns: read the two series on the computed grid (2 x k_pad x 8 B) and
      write the full column-transformed arrays (2 x n_fft x 8 B), per template;
    fft_rows_2f: read those (2 x n_fft x 8 B) and write 2F (4 B/bin), per template."""
    nt = ds.ntmpl if ntmpl is None else ntmpl
    n_in = sum(d.n for d in ds.detectors)
    return {
        "prologue": nt * 1024,
        "resample": n_resampled * (8 * n_in + 2 * 8 * k_pad),
        "fft_columns": nt * (2 * 8 * k_pad + 2 * 8 * ds.n_fft),
        "fft_rows_2f": nt * (2 * 8 * ds.n_fft + 4 * ds.n_bins),
    }


def error_stats(gpu, ref):
    """Error of GPU 2F against the oracle over the given bins: the bar's two
    measures (relative where the oracle's 2F >= 10, absolute elsewhere), the
    RMS fractional error, and Sec. 4.2's r_1, r_2 (relative L1 and L2 errors)
    and theta (the angle between the two 2F vectors)."""
    import numpy as np
    from oracle import fstat_oracle as O
    gpu = np.asarray(gpu, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    strong = ref >= 10.0
    rel = np.abs(gpu[strong] - ref[strong]) / ref[strong] if strong.any() else np.zeros(1)
    ab = np.abs(gpu[~strong] - ref[~strong]) if (~strong).any() else np.zeros(1)
    frac = (gpu - ref) / np.maximum(ref, 1.0)
    return {"bins": int(ref.size), "bins_2F_ge_10": int(strong.sum()),
            "max_rel_2F_ge_10": float(f"{rel.max():.3e}"),
            "max_abs_else": float(f"{ab.max():.3e}"),
            "rms_frac": float(f"{np.sqrt(np.mean(frac ** 2)):.3e}"),
            "r1": float(f"{O.rel_err(gpu, ref, 1):.3e}"),
            "r2": float(f"{O.rel_err(gpu, ref, 2):.3e}"),
            "theta": float(f"{O.angle(gpu, ref):.3e}"),
            "within_bar": bool(rel.max() <= 1e-4 and ab.max() <= 1e-3)}


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return model, os.cpu_count(), avail


_POOL_DS = None


def _oracle_one(t, fafb=False):
    from threadpoolctl import threadpool_limits
    from oracle import fstat_oracle as O
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        out = O.oracle_twoF(_POOL_DS, _POOL_DS.templates[[t]], return_fafb=fafb)
        el = time.perf_counter() - t0
        if fafb:
            tf, ff = out
            return t, tf[0], el, ff[0][:2]
        return t, out[0], el


def cpu_baseline(ds, picks, workers):
    """The FP64 oracle (numpy, one thread per process) on sampled templates of
    the headline workload: picks[0] alone on one core, then picks[1:] on
    `workers` forked processes at once (run before the GPU is touched).
    Returns the baseline record, the oracle's 2F of every pick, and
    (picks[0], (Fa, Fb)) of the first."""
    import multiprocessing as mp
    global _POOL_DS
    _POOL_DS = ds
    model, ncpu, avail = host_cpu()
    t, ref0, el1, fafb0 = _oracle_one(picks[0], fafb=True)
    say(f"oracle: template {t} on one core in {el1:.1f} s")
    refs = {t: ref0}
    rest = list(picks[1:])
    elp = None
    if rest and workers > 1:
        ctx = mp.get_context("fork")
        t0 = time.perf_counter()
        with ctx.Pool(processes=workers) as pool:
            for t, out, el in pool.imap_unordered(_oracle_one, rest):
                refs[t] = out
                say(f"oracle: template {t} done ({el:.1f} s in its process, "
                    f"{len(refs) - 1}/{len(rest)})")
        elp = time.perf_counter() - t0
    one = 1.0 / el1
    allc = len(rest) / elp if elp else None
    rec = {"value": round(allc if allc else one, 5), "unit": "templates/s",
           "cores": workers if allc else 1, "kind": "oracle",
           "sample": (f"headline workload, full band ({ds.n_bins} bins): template {picks[0]} on one "
                      f"core in {el1:.1f} s; {len(rest)} more templates on {workers} processes "
                      f"(one thread each) in {elp:.1f} s" if elp else
                      f"headline workload, template {picks[0]}, {el1:.1f} s on one core"),
           "one_core": {"value": round(one, 5), "unit": "templates/s", "seconds": round(el1, 2)},
           "all_cores": ({"value": round(allc, 5), "unit": "templates/s", "processes": workers,
                          "templates": len(rest), "seconds": round(elp, 2)} if elp else None),
           "cpu_model": model, "nproc": ncpu, "cpus_available": avail,
           "tau_eff_s_per_bin_per_det_one_core": el1 / (ds.n_bins * ds.ndet)}
    _POOL_DS = None
    return rec, refs, (picks[0], fafb0)


def kernel_table(totals, bytes_step, steps):
    kern = {}
    for k, (ms, n) in totals.items():
        avg = ms / max(n, 1)
        b_launch = bytes_step[k] * steps / max(n, 1)
        kern[k] = {"ms_per_step": round(ms / steps, 4), "launches_per_step": n // steps,
                   "avg_us": round(avg * 1e3, 2), "bytes_per_launch": int(b_launch),
                   "gbs": round(b_launch / (avg / 1e3) / 1e9, 1) if avg > 0 else None}
    return kern


def roofline(kern, totals, workload, ntmpl):
    dom = max((k for k in kern if k != "prologue"), key=lambda k: totals[k][0])
    achieved = kern[dom]["gbs"]
    traffic = None
    per_t = MEASURED_TRAFFIC["bytes_per_template"].get(workload, {}).get(dom)
    if per_t is not None and sources_digest() == MEASURED_TRAFFIC["sources_sha256"]:
        traffic = int(per_t * ntmpl / max(kern[dom]["launches_per_step"], 1))
    return {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
            "bytes_per_launch": kern[dom]["bytes_per_launch"]}


def headline(args, ds, refs, fafb_ref=None):
    """The binary workload: 10^4 templates, full band, batched search path."""
    import numpy as np
    import torch
    from paper_2201_00451_amd import binding
    tune, tuned = None, None
    if args.autotune > 0:
        # the FFT launch shape from the search-path autotuner (median of three
        # timed searches of a sample per shape; FSTAT_AUTOTUNE_CACHE, if set,
        # keeps the result across runs)
        dd0 = binding.DeviceData(ds, batch=1)
        sample = ds.templates[:args.autotune]
        t0 = time.perf_counter()
        tune, tms, hit = binding.autotune_search(dd0, sample, slots=args.batch, repeats=3)
        tuned = {"tune": tune, "median_ms_sample": round(tms, 3),
                 "sample_templates": len(sample), "from_cache": hit,
                 "seconds": round(time.perf_counter() - t0, 2)}
        say(f"autotune: {tune} ({tms:.2f} ms per {len(sample)}-template search, "
            f"{'cached' if hit else 'timed'})")
        del dd0
        torch.cuda.empty_cache()
    dd = binding.DeviceData(ds, batch=1, tune=tune)
    k_pad, _, _ = dd.plan.info()
    ring = min(args.ring, ds.ntmpl)
    blocks = [(i, min(i + ring, ds.ntmpl)) for i in range(0, ds.ntmpl, ring)]
    ws_bytes = max(binding.search_workspace_size(dd, ds.templates[a:b], args.batch)
                   for a, b in blocks)
    shared = torch.empty(ws_bytes, dtype=torch.uint8, device=dd.device)
    searches = [binding.Search(dd, ds.templates[a:b], slots=args.batch, workspace=shared)
                for a, b in blocks]
    out = torch.empty((ring, ds.n_bins), dtype=torch.float32, device=dd.device)
    nchunks = sum(s.nchunks for s in searches)
    ngroups = sum(s.ngroups for s in searches)
    say(f"{ds.ntmpl} templates ({ngroups} sky/orbit groups) in {len(blocks)} blocks of "
        f"<= {ring}, {nchunks} launch sequences of <= {args.batch}; output ring "
        f"{out.numel() * 4 / 2**30:.1f} GiB, workspace {ws_bytes / 2**30:.1f} GiB")

    def step():
        tot = {k: [0.0, 0] for k in binding.KERNELS}
        for (a, b), s in zip(blocks, searches):
            _, kt = s.run_profiled(out=out[:b - a])
            for k, (ms, n) in kt.items():
                tot[k][0] += ms
                tot[k][1] += n
        return tot

    say("headline warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    say(f"headline: timing {args.steps} steps")
    totals = {k: [0.0, 0] for k in binding.KERNELS}
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    t_wall = time.perf_counter()
    for _ in range(args.steps):
        tot = step()
        for k in totals:
            totals[k][0] += tot[k][0]
            totals[k][1] += tot[k][1]
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ms_step = ev0.elapsed_time(ev1) / args.steps
    value = ds.ntmpl / (ms_step / 1e3)
    binding.sync_check()
    flagged = binding.flagged_count(shared)
    kern = kernel_table(totals, step_bytes(ds, k_pad, ngroups), args.steps)
    roof = roofline(kern, totals, "binary", ds.ntmpl)

    res = {"value": value, "ms_per_step": ms_step, "wall_s_timed": wall, "kernels": kern,
           "roofline": roof, "blocks": len(blocks), "ring": ring, "nchunks": nchunks,
           "ngroups": ngroups, "flagged_templates": flagged, "autotune": tuned}

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

    tm = torch.from_numpy(ds.templates).to(dd.device)
    if args.plain_steps > 0:
        # the plain per-template path (one template in flight, as in the
        # paper), over the whole bank into the same ring
        say("headline: plain per-template path")

        def plain():
            for a, b in blocks:
                binding.compute_2f(dd, tm[a:b], out=out[:b - a])
        res["plain"] = timed(plain, args.plain_steps)
        binding.sync_check()
    if args.graph_steps > 0:
        say("headline: graph replay")
        gsr = [binding.Search(dd, ds.templates[a:b], slots=args.batch, workspace=shared,
                              graph=True) for a, b in blocks]
        gs = torch.cuda.Stream()

        def graph():
            gs.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(gs):
                for (a, b), s in zip(blocks, gsr):
                    s.run(out=out[:b - a], stream=gs)
            torch.cuda.current_stream().wait_stream(gs)
        graph()
        res["graph_replay"] = timed(graph, args.graph_steps)
        binding.sync_check()
        del gsr
    if args.cand_steps > 0:
        # the same bank keeping only the bins above the pilot search's
        # threshold 2F > 70 (Sec. 5.4) and the loudest bin per template
        say("headline: candidate retention")
        csr = binding.Search(dd, ds.templates, slots=args.batch)
        c = csr.run_candidates(70.0, capacity=1 << 20)
        cr = timed(lambda: csr.run_candidates(70.0, capacity=1 << 20), args.cand_steps)
        cr.update({"threshold": 70.0, "candidates": c["count"]})
        res["candidates"] = cr
        del csr, c
        torch.cuda.empty_cache()
    # error against the oracle on the sampled templates
    if refs:
        from oracle import fstat_oracle as O
        picks = sorted(refs)
        rows = []
        dd8 = binding.DeviceData(ds, batch=8, tune=tune)
        for i in range(0, len(picks), 8):
            rows.append(binding.compute_2f_batched(dd8, tm[picks[i:i + 8]]).cpu().numpy())
        got = np.concatenate(rows, axis=0)
        binding.sync_check()
        ref = np.stack([refs[t] for t in picks])
        st = error_stats(got, ref)
        st["templates"] = picks
        if fafb_ref is not None:
            # Sec. 4.2's metrics for Fa and Fb of the template nearest the injection
            t_f, (fa_ref, fb_ref) = fafb_ref
            _, fab = binding.compute_2f(dd8, tm[[t_f]], fafb=True)
            fab = fab[0].cpu().numpy()
            st["fa_fb"] = {"template": t_f}
            for name, g, r in (("Fa", fab[0], fa_ref), ("Fb", fab[1], fb_ref)):
                st["fa_fb"][name] = {"r1": float(f"{O.rel_err(g, r, 1):.3e}"),
                                     "r2": float(f"{O.rel_err(g, r, 2):.3e}"),
                                     "theta": float(f"{O.angle(g, r):.3e}")}
        res["error_vs_oracle"] = st
        del dd8
    del searches, shared, out
    torch.cuda.empty_cache()
    return res


def sky_leg(args):
    """The sky/spin-down workload (2 detectors x 10 d at 1 s, 1000 templates =
    10 x 10 sky x 10 spin-downs, n_fft 2^21, full band): grouped search (one
    resampled series per sky position), plain and ungrouped paths, graph
    replay, candidate retention, error on two templates."""
    import numpy as np
    import torch
    from oracle import fstat_oracle as O
    from paper_2201_00451_amd import binding, synth
    say("sky/spin-down workload")
    ds = synth.config_sky_spindown()
    dd = binding.DeviceData(ds, batch=args.batch)
    tm = torch.from_numpy(ds.templates).to(dd.device)
    out = torch.empty((ds.ntmpl, ds.n_bins), dtype=torch.float32, device=dd.device)
    k_pad, _, _ = dd.plan.info()
    sr = binding.Search(dd, ds.templates, slots=args.batch)
    for _ in range(max(args.warmup, 1)):
        sr.run_profiled(out=out)
    torch.cuda.synchronize()
    steps = args.sky_steps
    totals = {k: [0.0, 0] for k in binding.KERNELS}
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(torch.cuda.current_stream())
    for _ in range(steps):
        _, kt = sr.run_profiled(out=out)
        for k, (ms, n) in kt.items():
            totals[k][0] += ms
            totals[k][1] += n
    ev1.record(torch.cuda.current_stream())
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / steps
    kern = kernel_table(totals, step_bytes(ds, k_pad, sr.ngroups), steps)
    res = {"workload": "two detectors, 10 d at 1 s (864000 samples each), 150 Hz, 1000 templates "
                       "(10x10 sky x 10 spin-down), n_fft 2^21, full band",
           "value": round(ds.ntmpl / (ms_step / 1e3), 1), "ms_per_step": round(ms_step, 3),
           "steps": steps, "sky_orbit_groups": sr.ngroups, "launch_sequences": sr.nchunks,
           "kernels": kern, "roofline": roofline(kern, totals, "sky_spindown", ds.ntmpl)}

    def timed(fn, n):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(torch.cuda.current_stream())
        for _ in range(n):
            fn()
        e1.record(torch.cuda.current_stream())
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / n
        return {"value": round(ds.ntmpl / (ms / 1e3), 1), "ms_per_step": round(ms, 3), "steps": n}

    if args.plain_steps > 0:
        res["batched_ungrouped"] = timed(lambda: binding.compute_2f_batched(dd, tm, out=out), 1)
        dd1 = binding.DeviceData(ds, batch=1)
        res["plain"] = timed(lambda: binding.compute_2f(dd1, tm, out=out), 1)
        res["batched_over_plain"] = round(res["value"] / res["plain"]["value"], 3)
        del dd1
    if args.graph_steps > 0:
        srg = binding.Search(dd, ds.templates, slots=args.batch, graph=True)
        gs = torch.cuda.Stream()

        def run_graph():
            with torch.cuda.stream(gs):
                srg.run(out=out, stream=gs)
            gs.synchronize()
        run_graph()
        res["graph_replay"] = timed(run_graph, 3)
        del srg
    if args.cand_steps > 0:
        cap = 1 << 20
        c = sr.run_candidates(40.0, capacity=cap)
        cr = timed(lambda: sr.run_candidates(40.0, capacity=cap), 3)
        cr.update({"threshold": 40.0, "candidates": c["count"]})
        res["candidates"] = cr
    binding.sync_check()
    if args.errors:
        sr.run(out=out)
        inj = ds.injections[0]
        cost = (np.abs(ds.templates[:, 0] - inj["alpha"]) + np.abs(ds.templates[:, 1] -
                inj["delta"]) + np.abs(ds.templates[:, 3] - inj["f1dot"]) * 1e8)
        picks = [0, int(np.argmin(cost))]
        ref = O.oracle_twoF(ds, ds.templates[picks])
        got = out[picks].cpu().numpy()
        st = error_stats(got, ref)
        st["templates"] = picks
        res["error_vs_oracle"] = st
    del out, sr
    torch.cuda.empty_cache()
    return res


def tiny_leg(args):
    """One detector, 1 d at 2 s, 11 spin-down templates, n_fft 2^17."""
    import torch
    from oracle import fstat_oracle as O
    from paper_2201_00451_amd import binding, synth
    say("tiny workload")
    ds = synth.config_tiny()
    dd = binding.DeviceData(ds, batch=1)
    sr = binding.Search(dd, ds.templates, slots=ds.ntmpl)
    out = torch.empty((ds.ntmpl, ds.n_bins), dtype=torch.float32, device=dd.device)
    sr.run_profiled(out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(torch.cuda.current_stream())
    for _ in range(10):
        sr.run(out=out)
    e1.record(torch.cuda.current_stream())
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    res = {"templates": ds.ntmpl, "n_fft": ds.n_fft, "ms_per_step": round(ms, 4),
           "templates_per_s": round(ds.ntmpl / (ms / 1e3), 1)}
    if args.errors:
        res["error_vs_oracle"] = error_stats(out.cpu().numpy(), O.oracle_twoF(ds))
    binding.sync_check()
    return res


def refinement_leg(args):
    """The adjoint on the refinement workload (2 detectors x 30 d at 1 s,
    0.2 Hz band at 400 Hz, n_fft 2^22, 8 circular-binary injections with
    rho U(10, 40), candidates 0.3-1 metric spacing from their injection):
    single-bin gradient evaluations per second, and preconditioned gradient
    ascent with the recovered 2F against the injected rho^2, against 4 + rho^2
    and against the 2F at the true parameters."""
    import math
    import numpy as np
    import torch
    from oracle import fstat_oracle as O
    from paper_2201_00451_amd import binding, synth
    say(f"refinement workload: {8 * args.refine_per_inj} candidates")
    ds = synth.config_refine(per_inj=args.refine_per_inj)
    dd = binding.DeviceData(ds)
    rows, bins = ds.templates, ds.cand_bins
    n = len(rows)
    binding.compute_2f_grad_bin(dd, rows, bins)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.refine_calls):
        binding.compute_2f_grad_bin(dd, rows, bins)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / max(args.refine_calls, 1)
    truth = rows.copy()
    T = ds.detectors[0].n * ds.dt
    scales = np.zeros((n, 7))
    rho2 = np.zeros(n)
    for m in range(n):
        inj = ds.injections[ds.cand_inj[m]]
        nat = bins[m] + ds.bin_lo - ds.n_fft // 2
        truth[m, 2] = (inj["f"] - ds.f_het) - nat / (ds.n_fft * ds.dt)
        truth[m, 5], truth[m, 6], truth[m, 7] = inj["asini"], inj["porb"], inj["tp"]
        om = 2 * math.pi / inj["porb"]
        scales[m] = [1.0 / T, 1.0 / T ** 2, 1e-3, 1e-3, 1.0 / (2 * math.pi * inj["f"]),
                     inj["porb"] ** 2 / (2 * math.pi * inj["f"] * inj["asini"] * T),
                     1.0 / (2 * math.pi * inj["f"] * inj["asini"] * om)]
        rho2[m] = inj["rho2"]
    _, tf_true = binding.compute_2f_grad_bin(dd, truth, bins)
    _, tf_start = binding.compute_2f_grad_bin(dd, rows, bins)
    tf_true = tf_true.cpu().numpy()
    tf_start = tf_start.cpu().numpy()
    t0 = time.perf_counter()
    _, vals = binding.refine(dd, rows, bins, scales, steps=args.refine_steps,
                             free=("df", "asini", "porb", "tp"))
    el = time.perf_counter() - t0
    evals = n * (args.refine_steps + 1)
    res = {"workload": f"2 detectors x 2592000 samples, n_fft 2^22, 0.2 Hz band at 400 Hz, "
                       f"8 binary injections x {args.refine_per_inj} candidates",
           "candidates": n, "grad_evals_per_s": round(n / (ms / 1e3), 1),
           "ms_per_call": round(ms, 3), "refine_steps": args.refine_steps,
           "refine_wall_s": round(el, 2), "refine_grad_evals_per_s": round(evals / el, 1),
           "median_2F_start_over_true": round(float(np.median(tf_start / tf_true)), 4),
           "median_2F_end_over_true": round(float(np.median(vals / tf_true)), 4),
           "min_2F_end_over_true": round(float(np.min(vals / tf_true)), 4),
           "median_2F_end_over_rho2": round(float(np.median(vals / rho2)), 4),
           "median_2F_end_over_4_plus_rho2": round(float(np.median(vals / (4.0 + rho2))), 4),
           "median_2F_true_over_rho2": round(float(np.median(tf_true / rho2)), 4)}
    if args.errors:
        c0 = 0
        got = binding.compute_2f_batched(dd, rows[[c0]]).cpu().numpy()
        res["error_vs_oracle"] = error_stats(got, O.oracle_twoF(ds, rows[[c0]]))
        res["error_vs_oracle"]["templates"] = [c0]
    binding.sync_check()
    return res


def uneven_leg(args):
    """Independent searches of uneven span, band, FFT length and detector
    count (spans log-uniform in 1-30 d, dt in {0.5, 1, 2, 5} s, n_fft 2^16 to
    2^22, 8-64 templates each), run one after the other and as one captured
    batch over 4 branches; the error of the first template of the first
    searches against the oracle."""
    import torch
    from oracle import fstat_oracle as O
    from paper_2201_00451_amd import binding, synth
    n_search = args.uneven_searches
    say(f"{n_search} uneven searches")
    dss = []
    for i in range(0, n_search, 32):
        pick = set(range(i, min(i + 32, n_search)))
        dss += synth.config_uneven(seed=4, n_search=n_search, pick=pick)
        say(f"uneven: {len(dss)}/{n_search} searches generated")
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
        for _ in range(args.uneven_steps):
            fn()
        e1.record(st)
        st.synchronize()
        ms = e0.elapsed_time(e1) / args.uneven_steps
        res[name] = {"ms_per_step": round(ms, 3), "templates_per_s": round(ntmpl / (ms / 1e3), 1),
                     "bins_per_s": float(f"{nbins / (ms / 1e3):.4g}")}
    binding.sync_check()
    out = {"workload": f"{n_search} searches: spans log-uniform 1-30 d, dt in 0.5-5 s, "
                       "1 or 2 detectors, n_fft 2^16-2^22, full band, 8-64 templates each",
           "searches": n_search, "templates": ntmpl,
           "n_fft_range": [min(d.n_fft for d in dss), max(d.n_fft for d in dss)],
           "steps": args.uneven_steps, **res,
           "batch_over_sequential": round(res["sequential"]["ms_per_step"] /
                                          res["batch"]["ms_per_step"], 3)}
    if args.errors:
        per = []
        for k in range(min(args.uneven_errors, n_search)):
            ds = dss[k]
            st_k = error_stats(outs[k][0].cpu().numpy(), O.oracle_twoF(ds, ds.templates[:1])[0])
            st_k.update({"search": k, "n_fft": ds.n_fft, "detectors": ds.ndet,
                         "kind": "binary" if ds.templates[0, 5] else "spin-down"})
            per.append(st_k)
        out["error_vs_oracle_per_search"] = per
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=32, help="templates in flight per launch")
    ap.add_argument("--ring", type=int, default=1024,
                    help="headline: templates per block (rows of the reused output array)")
    ap.add_argument("--ntmpl", type=int, default=10000, help="headline bank size")
    ap.add_argument("--autotune", type=int, default=64,
                    help="headline: templates of the sample the search-path autotuner times "
                         "each FFT launch shape on (0: the default shape)")
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--graph-steps", type=int, default=1)
    ap.add_argument("--cand-steps", type=int, default=1)
    ap.add_argument("--sky", type=int, default=1, help="the sky/spin-down workload (0: skip)")
    ap.add_argument("--sky-steps", type=int, default=5)
    ap.add_argument("--tiny", type=int, default=1)
    ap.add_argument("--uneven-searches", type=int, default=64,
                    help="independent searches of uneven shape (0: skip)")
    ap.add_argument("--uneven-steps", type=int, default=3)
    ap.add_argument("--uneven-errors", type=int, default=4,
                    help="searches whose first template is checked against the oracle")
    ap.add_argument("--refine-per-inj", type=int, default=64,
                    help="candidates per injection of the refinement workload (8 injections; "
                         "512 gives its full 4096)")
    ap.add_argument("--refine-calls", type=int, default=5,
                    help="timed single-bin gradient calls on the refinement workload (0: skip)")
    ap.add_argument("--refine-steps", type=int, default=50)
    ap.add_argument("--cpu-samples", type=int, default=0,
                    help="templates of the headline workload the oracle runs on all cores "
                         "(default: one per available core, at most 16)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--errors", type=int, default=1,
                    help="error against the FP64 oracle for each workload (0: skip)")
    ap.add_argument("--no-headline", action="store_true",
                    help="run only the other workloads asked for (profiling and the full-scale "
                         "refinement and uneven-batch runs); the line's value is null")
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
    from paper_2201_00451_amd import synth

    if args.no_headline:
        args.no_cpu_baseline = True
        ds = None
    else:
        say("generating the headline workload (2 x 5184000 samples, 10^4 binary templates)")
        ds = synth.config_binary(ntmpl=args.ntmpl)
    # oracle on the host before the GPU is touched (its worker processes are
    # forked): the template nearest the injection, then a seeded sample
    cpu, refs, fafb_ref = None, {}, None
    if not args.no_cpu_baseline:
        _, _, avail = host_cpu()
        workers = min(16, avail) if args.cpu_samples == 0 else args.cpu_samples
        inj = ds.injections[0]
        d = (np.abs(ds.templates[:, 5] - inj["asini"]) / np.ptp(ds.templates[:, 5]) +
             np.abs(ds.templates[:, 6] - inj["porb"]) / np.ptp(ds.templates[:, 6]) +
             np.abs(ds.templates[:, 7] - inj["tp"]) / np.ptp(ds.templates[:, 7]))
        near = int(np.argmin(d))
        rng = np.random.default_rng(12345)
        others = [int(t) for t in rng.choice(ds.ntmpl, size=workers + 4, replace=False)
                  if t != near][:workers]
        say(f"FP64 oracle on the host: template {near} on one core, {len(others)} on "
            f"{workers} processes")
        cpu, refs, fafb_ref = cpu_baseline(ds, [near] + others, workers)

    import torch
    from paper_2201_00451_amd import binding
    hl = headline(args, ds, refs, fafb_ref) if ds is not None else None
    plain = hl.get("plain") if hl else None
    others = {}
    if args.sky:
        others["sky_spindown"] = sky_leg(args)
    if args.tiny:
        others["tiny"] = tiny_leg(args)
    refine = refinement_leg(args) if args.refine_calls > 0 else None
    uneven = uneven_leg(args) if args.uneven_searches > 0 else None

    calib = None
    if args.calibrate_copy_mib > 0:
        nbytes = args.calibrate_copy_mib << 20
        src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        calib = {"copy_bytes_read": nbytes, "copy_bytes_written": nbytes}
        del src, dst
    binding.sync_check()

    if hl is None:
        print(json.dumps({"metric": METRIC, "value": None, "unit": "templates/s", "n_gpus": 1,
                          "headline": "skipped (--no-headline)", "other_workloads": others,
                          "refinement": refine, "uneven_batch": uneven,
                          "calibration_copy": calib}), flush=True)
        return
    value = hl["value"]
    ms_step = hl["ms_per_step"]
    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "templates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "narrowband binary batch shaped like the pilot search: two "
                               "detectors, 120 d at 2 s (5184000 samples each, 70% duty in "
                               "1800 s blocks), 0.5 Hz band in 200-600 Hz, 10^4 circular-binary "
                               "templates on an (asini, porb, tp) lattice, n_fft 2^23, full band "
                               "(8388608 bins per template)",
                   "templates": ds.ntmpl, "n_fft": ds.n_fft, "n_bins": ds.n_bins,
                   "detectors": ds.ndet, "samples_per_detector": ds.detectors[0].n,
                   "sinc_halfwidth": ds.sinc_halfwidth, "slots": args.batch,
                   "launch_sequences": hl["nchunks"], "output_ring_templates": hl["ring"],
                   "timing_dtype": "f64",
                   "path": "grouped search (one resampled series per sky/orbit group; every "
                           "binary template is its own group)",
                   "sky_orbit_groups": hl["ngroups"]},
        "plain": plain,
        "batched_over_plain": round(value / plain["value"], 3) if plain else None,
        "graph_replay": hl.get("graph_replay"),
        "candidates": hl.get("candidates"),
        "tau_eff_s_per_bin_per_det": (ms_step / 1e3) / (ds.ntmpl * ds.n_bins * ds.ndet),
        "kernels": hl["kernels"],
        "roofline": hl["roofline"],
        "autotune": hl["autotune"],
        "error_vs_oracle": hl.get("error_vs_oracle"),
        "flagged_templates": hl["flagged_templates"],
        "cpu_baseline": cpu,
        "other_workloads": others,
        "refinement": refine,
        "uneven_batch": uneven,
        "wall_s_timed": round(hl["wall_s_timed"], 3),
    }
    if calib:
        line["calibration_copy"] = calib
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
