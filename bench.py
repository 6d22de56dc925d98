"""Throughput of the ray-tracing hot path on one MI355X.

One step = one pass of the forward hot path over one batch of synthetic input:
resonance seeding (rt_sample_resonance) -> adaptive FP64 DOPRI5 tracing to r_max
(rt_trace_forward) -> sky/frequency binning (rt_bin_flux), on the full forward
workload: 1e6 rays, Schwarzschild M = 1.4 Msun, oblique rotator theta_m = 0.3,
anisotropic strongly magnetised plasma (LO mode), GJ density, m_a = 2e-5 eV,
64 x 128 x 64 bins, rtol 1e-8.

Prints one JSON line: value = accepted ray-steps per second of the whole step
(whole-job throughput, inputs resident in HBM); rays/s alongside; the roofline of
the dominant kernel (the persistent tracing kernel, FP64 vector ALU bound); and the
CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X, AMD published (256 CU x 128 FLOP/clk x 2.4 GHz)


# HBM traffic of the tracing kernel, measured with hardware counters (FETCH_SIZE and
# WRITE_SIZE per dispatch, each scaled by what it reads for a copy of known size) on this
# workload; valid only while the kernel's sources and build flags are the ones it was
# measured on
COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "trace_fwd_kernel_forward-full-1e6_counters.md")
TRACE_SOURCES = ["csrc/rt_forward.hip", "csrc/rt_common.hpp", "csrc/rt_device.hpp", "csrc/rt_integrator.hpp",
                 "csrc/rt_seed.hpp", "build.py"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in TRACE_SOURCES:
        with open(os.path.join(ROOT, "paper_2309_08655_amd", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_values(n):
    """Counter-measured values per launch of the tracing kernel (HBM bytes, hardware FP64
    flops), or {} when there is no measurement for these sources and this ray count."""
    if not os.path.exists(COUNTER_SUMMARY):
        return {}
    vals = {}
    with open(COUNTER_SUMMARY) as f:
        for line in f:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256") != kernel_source_hash() or int(vals.get("rays", -1)) != n:
        return {}
    return {k: float(v) for k, v in vals.items() if k.endswith("_per_launch")}


def variant_key(star):
    pl = "iso" if star["plasma"] == 0 else "aniso"
    de = ["gj", "magnetar", "spherical", "none"][star["density"]]
    ob = "oblique" if math.sin(star["theta_m"]) != 0.0 else "aligned"
    return f"{pl}_{de}_{ob}"


def flop_table():
    with open(os.path.join(ROOT, "paper_2309_08655_amd", "flops.json")) as f:
        return json.load(f)


def host_threads():
    """(cores this process may run on, threads the oracle uses).  One GPU's share of the
    GPU machine's host is 16 threads, whatever the affinity mask shows there."""
    aff = len(os.sched_getaffinity(0))
    return aff, min(aff, 16)


def _oracle():
    import oracle
    oracle.build(force=False)
    return oracle


def cpu_baseline(cfg, n_sample, threads, n_single=1 << 11):
    """The oracle as it stands, on the first n_sample rays of the same workload (seed, trace,
    bin) on `threads` host threads, and on its first n_single rays on one core."""
    orc = _oracle()

    def run(n, nt):
        t0 = time.perf_counter()
        rays, st = orc.sample(cfg["star"], cfg["seed"], n, nthreads=nt)
        fin, ifin = orc.trace_forward(cfg["star"], cfg["tol"], rays, st, nthreads=nt)
        orc.bin_flux(fin, ifin, rays[8], cfg["bins"])
        dt = time.perf_counter() - t0
        return dt, float(ifin[0].sum()), float((st == 0).sum())

    dt, steps, traced = run(n_sample, threads)
    dt1, steps1, traced1 = run(n_single, 1)
    aff, _ = host_threads()
    return dict(value=steps / dt, unit="ray-steps/s", cores=threads, kind="oracle",
                sample=f"first {n_sample} rays of the same workload (seed, trace, bin), {dt:.2f} s",
                rays_per_s=traced / dt, affinity_cores=aff,
                single_core=dict(ray_steps_per_s=steps1 / dt1, rays_per_s=traced1 / dt1, cores=1,
                                 sample=f"first {n_single} rays, {dt1:.2f} s"))


def cpu_baseline_batched(W, threads, n_per=1000, stride=17):
    """The oracle on the batched scan's bounded sample: the first n_per rays of every
    stride-th instance (16 instances along the grid's diagonal: every axion mass and every
    inclination once), seeded, traced and binned per instance."""
    orc = _oracle()
    stars, counts = W.batched_instances(W.CFG4["n_inst"], seed=W.CFG4["seed"])
    ks = list(range(0, len(stars), stride))
    t0 = time.perf_counter()
    steps = traced = 0.0
    for k in ks:
        m = min(n_per, int(counts[k]))
        rays, st = orc.sample(stars[k], W.CFG4["seed"], m, instance=k, nthreads=threads)
        fin, ifin = orc.trace_forward(stars[k], W.tol(), rays, st, nthreads=threads)
        orc.bin_flux(fin, ifin, rays[8], W.CFG4["bins"])
        steps += float(ifin[0].sum())
        traced += float((st == 0).sum())
    dt = time.perf_counter() - t0
    return dict(value=steps / dt, unit="ray-steps/s", rays_per_s=traced / dt, cores=threads, kind="oracle",
                sample=f"first {n_per} rays of {len(ks)} instances (every {stride}th), seed + trace + bin, "
                       f"{dt:.2f} s")


def cpu_baseline_adjoint(W, threads, n=1000):
    """The oracle's forward-mode gradient of the smoothed flux (6 tangents through seeding,
    every step and the r_max crossing) on the adjoint workload's first n rays; ray-steps/s
    counts the accepted steps of those rays' traces."""
    orc = _oracle()
    cfg = W.CFG5
    obs = W.observers(cfg["n_obs"])
    t0 = time.perf_counter()
    orc.flux_fwdmode(cfg["star"], cfg["tol"], cfg["seed"], n, obs, cfg["sigma"], nthreads=threads)
    dt = time.perf_counter() - t0
    rays, st = orc.sample(cfg["star"], cfg["seed"], n, nthreads=threads)
    fin, ifin = orc.trace_forward(cfg["star"], cfg["tol"], rays, st, nthreads=threads)
    return dict(value=float(ifin[0].sum()) / dt, unit="ray-steps/s", rays_per_s=float((st == 0).sum()) / dt,
                cores=threads, kind="oracle",
                sample=f"first {n} rays, flux and its 6-parameter gradient by forward mode, {dt:.2f} s")


def cpu_baseline_backward(W, threads, stride=8):
    """The oracle's backward tracer on a strided sub-grid of the image (every stride-th pixel
    in each direction: 128^2 of the 1024^2 pixels)."""
    orc = _oracle()
    cfg = W.CFG3
    im = cfg["image"]
    ni, nj = im["nx"] // stride, im["ny"] // stride
    t0 = time.perf_counter()
    ev, nev, fin, ifin = orc.trace_backward(cfg["star"], cfg["tol"], im, cfg["K"], 0, 0, stride, ni, nj,
                                            nthreads=threads)
    dt = time.perf_counter() - t0
    return dict(value=float(ifin[0].sum()) / dt, unit="ray-steps/s", rays_per_s=ni * nj / dt, cores=threads,
                kind="oracle", sample=f"{ni}x{nj} pixels (every {stride}th in each direction), {dt:.2f} s")


def bench_batched(args, rt, W, np, torch):
    """Batched persistent launch over the 256-instance scan (16 axion masses x 16
    inclinations, 1e4-2e5 rays each): autotuned schedule, captured into one hipGraph;
    compared with one launch of each entry point per instance."""
    from paper_2309_08655_amd import autotune
    stars, counts = W.batched_instances(W.CFG4["n_inst"], seed=W.CFG4["seed"])
    tol, bins = W.tol(), W.CFG4["bins"]
    print(f"bench: batched {len(stars)} instances, {int(counts.sum())} rays", file=sys.stderr, flush=True)
    b = rt.Batch(stars, counts, W.CFG4["seed"], tol, bins)
    best, times = (None, None)
    if not args.no_tune:
        def run_sc(sc):
            b.set_schedule(sc)
            b.run()
        best, times = autotune.tune(run_sc, key=f"batched|{len(stars)}|{int(counts.sum())}", reps=3,
                                    candidates=autotune.BATCHED_CANDIDATES)
    b.set_schedule(best)
    g = b.capture()
    for _ in range(max(1, args.warmup)):
        g.replay()
    torch.cuda.synchronize()
    reps = max(2, min(args.steps, 5))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    ifn = b.ifin.cpu().numpy()
    acc = float(ifn[0].astype(np.float64).sum())
    rej = float(ifn[1].astype(np.float64).sum())
    traced = float((b.status.cpu().numpy() == 0).sum())
    # the tracing kernel alone (eager runs: events are not recorded inside a captured graph),
    # against its algorithmic work, and its lane efficiency (third word of the work counter)
    rt.timing(True)
    for _ in range(2):
        b.run()
    torch.cuda.synchronize()
    rt.timing(False)
    kt = [t for name, t in rt.kernel_times() if name == "trace_fwd_kernel(batched)"]
    kernel_ms = float(np.mean(kt))
    wave_iters = int(b.ws[16:24].cpu().numpy().view(np.uint64)[0])
    ft = flop_table()["iso_gj_oblique"]  # the batch takes the rotating-axis formula throughout
    ktf = (acc + rej) * ft["attempt"] / (kernel_ms * 1e-3) / 1e12
    # one launch of each entry point per instance, on buffers sized for the largest instance
    nmax = int(counts.max())
    dev = torch.device("cuda")
    rays = torch.empty((10, nmax), dtype=torch.float64, device=dev)
    st = torch.empty(nmax, dtype=torch.int32, device=dev)
    fin = torch.empty((rt.RT_NFIN, nmax), dtype=torch.float64, device=dev)
    ifin = torch.empty((rt.RT_NIFIN, nmax), dtype=torch.int32, device=dev)
    ws = rt.workspace(rt.OP_TRACE_FORWARD, nmax)
    wsb = rt.workspace(rt.OP_BIN, nmax)
    hist = torch.empty((1, bins["n_theta"], bins["n_psi"], bins["n_omega"]), dtype=torch.float64, device=dev)
    cnt = torch.empty_like(hist)
    over = torch.empty(2, dtype=torch.float64, device=dev)

    def per_instance():
        for k, s in enumerate(stars):
            m = int(counts[k])
            t_ = st[:m]
            # contiguous [F][m] views over the front of the max-size buffers
            rr = rays.view(-1)[:10 * m].view(10, m)
            ff = fin.view(-1)[:rt.RT_NFIN * m].view(rt.RT_NFIN, m)
            ii = ifin.view(-1)[:rt.RT_NIFIN * m].view(rt.RT_NIFIN, m)
            rt.rt_sample_resonance(s, W.CFG4["seed"], m, instance=k, rays=rr, status=t_)
            rt.rt_trace_forward(s, tol, rr, t_, schedule=best, ws=ws, fin=ff, ifin=ii)
            rt.rt_bin_flux(ff, ii, rr[8], bins, ws=wsb, hist=hist, cnt=cnt, over=over)

    # the plain (single-star) tracing kernel on the same physics: the scan's largest oblique
    # instance alone, against the same per-attempt count, for the batched kernel's rate
    kbig = max((k for k in range(len(stars)) if stars[k]["theta_m"] > 0 and stars[k]["m_a_eV"] < 9e-5),
               key=lambda k: counts[k])
    mb = int(counts[kbig])
    rrb = rays.view(-1)[:10 * mb].view(10, mb)
    ffb = fin.view(-1)[:rt.RT_NFIN * mb].view(rt.RT_NFIN, mb)
    iib = ifin.view(-1)[:rt.RT_NIFIN * mb].view(rt.RT_NIFIN, mb)
    rt.rt_sample_resonance(stars[kbig], W.CFG4["seed"], mb, instance=kbig, rays=rrb, status=st[:mb])
    rt.rt_trace_forward(stars[kbig], tol, rrb, st[:mb], ws=ws, fin=ffb, ifin=iib)
    torch.cuda.synchronize()
    rt.timing(True)
    for _ in range(3):
        rt.rt_trace_forward(stars[kbig], tol, rrb, st[:mb], ws=ws, fin=ffb, ifin=iib)
    torch.cuda.synchronize()
    rt.timing(False)
    kp = float(np.mean([t for name, t in rt.kernel_times() if name == "trace_fwd_kernel"]))
    ib = iib.cpu().numpy().astype(np.float64)
    plain_same = dict(instance=kbig, m_a_eV=stars[kbig]["m_a_eV"], theta_m=stars[kbig]["theta_m"], rays=mb,
                      kernel_ms=kp, kernel_frac=(ib[0].sum() + ib[1].sum()) * ft["attempt"] / (kp * 1e-3) / 1e12
                      / FP64_VECTOR_PEAK_TFLOPS)

    # kernels and buffers are already warm from the batched runs: time a single pass
    torch.cuda.synchronize()
    e0.record()
    per_instance()
    e1.record()
    torch.cuda.synchronize()
    ms_loop = e0.elapsed_time(e1)
    return dict(workload=W.CFG4["name"], instances=len(stars), rays=int(counts.sum()), traced_rays=traced,
                ms_per_launch=ms, ray_steps_per_s=acc / (ms * 1e-3), rays_per_s=traced / (ms * 1e-3),
                accepted_steps=acc, rejected_steps=rej, schedule=best, graph="one hipGraph replay per launch",
                kernel_ms=kernel_ms, kernel_tflops=ktf, kernel_frac=ktf / FP64_VECTOR_PEAK_TFLOPS,
                flop_per_attempt=ft["attempt"], lane_efficiency=(acc + rej) / max(1, 64 * wave_iters),
                per_instance_ms=ms_loop, speedup_vs_per_instance=ms_loop / ms, tune_ms=times,
                plain_kernel_same_physics=plain_same)


def bench_backward(args, rt, W, np, torch):
    """Backward image: 1024^2 pixels at 1e5 km traced inward through the magnetar-like star,
    recording up to 8 production events per ray."""
    cfg = W.CFG3
    star, tol, image, K = cfg["star"], cfg["tol"], cfg["image"], cfg["K"]
    n = image["nx"] * image["ny"]
    print(f"bench: backward {cfg['name']} n={n}", file=sys.stderr, flush=True)
    ws = rt.workspace(rt.OP_TRACE_BACKWARD, n)
    rt.rt_trace_backward(star, tol, image, K, ws=ws)
    torch.cuda.synchronize()
    reps = max(2, min(args.steps, 3))
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rt.timing(True)
    e0.record(stream)
    for _ in range(reps):
        ev, nev, fin, ifin = rt.rt_trace_backward(star, tol, image, K, ws=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    rt.timing(False)
    ms_call = e0.elapsed_time(e1) / reps
    kt = [ms for name, ms in rt.kernel_times() if name == "trace_bwd_kernel"]
    kernel_ms = float(np.mean(kt))
    inf = ifin.cpu().numpy().astype(np.int64)
    nv = nev.cpu().numpy().astype(np.int64)
    acc, rej = float(inf[0].sum()), float(inf[1].sum())
    ft = flop_table()[variant_key(star)]
    # per attempt one DOPRI5 attempt; per accepted step three probes of G on the continuous
    # extension and one at the step's end point (no dense output there); per recorded event
    # 60 bisection probes
    flops = ((acc + rej) * ft["attempt"] + acc * (3 * ft["event_probe"] + ft["event_g"])
             + float(nv.sum()) * 60 * ft["event_probe"])
    tf = flops / (kernel_ms * 1e-3) / 1e12
    st = {str(k): int(v) for k, v in zip(*np.unique(inf[2], return_counts=True))}
    out = dict(workload=cfg["name"], pixels=n, events=int(nv.sum()), rays_with_events=int((nv > 0).sum()),
               statuses=st, accepted_steps=acc, rejected_steps=rej, ms_per_image=ms_call, kernel_ms=kernel_ms,
               rays_per_s=n / (ms_call * 1e-3), ray_steps_per_s=acc / (ms_call * 1e-3), kernel_tflops=tf,
               kernel_frac=tf / FP64_VECTOR_PEAK_TFLOPS, flop_per_attempt=ft["attempt"],
               flop_per_event_probe=ft["event_probe"], flop_per_end_point_probe=ft["event_g"])
    out["power"] = bench_backward_power(args, rt, W, np, torch, cfg, ev, nev)
    return out


def bench_backward_power(args, rt, W, np, torch, cfg, ev, nev):
    """rt_backward_power over the image's recorded events: dP/dOmega of the image (1 km
    conversion-length cutoff, as in the paper) and the event-weight kernel's time against
    its algorithmic bytes: per pixel the event count (4 B) and the weight sum (8 B), per
    stored event its 8 state doubles (64 B)."""
    image, K = cfg["image"], cfg["K"]
    n = image["nx"] * image["ny"]
    area = (2 * image["half_width_km"] / image["nx"]) ** 2
    ws = rt.workspace(rt.OP_BACKWARD_POWER, n)
    rt.rt_backward_power(cfg["star"], ev, nev, 1.0, pixel_area_km2=area, ws=ws)
    torch.cuda.synchronize()
    reps = max(3, min(args.steps, 10))
    rt.timing(True)
    for _ in range(reps):
        wsum, total = rt.rt_backward_power(cfg["star"], ev, nev, 1.0, pixel_area_km2=area, ws=ws)
    torch.cuda.synchronize()
    rt.timing(False)
    kt = [ms for name, ms in rt.kernel_times() if name == "event_power_kernel"]
    kernel_ms = float(np.mean(kt))
    stored = float(torch.clamp(nev.to(torch.int64), max=K).sum().item())
    nbytes = n * (4 + 8) + stored * 64
    _, total_nocut = rt.rt_backward_power(cfg["star"], ev, nev, 0.0, pixel_area_km2=area, ws=ws)
    return dict(dP_dOmega_eV2=total.item(), dP_dOmega_no_cutoff_eV2=total_nocut.item(), Lc_max_km=1.0,
                kernel_ms=kernel_ms, stored_events=stored, algorithmic_bytes=nbytes,
                achieved_GBps=nbytes / (kernel_ms * 1e-3) / 1e9,
                hbm_frac=nbytes / (kernel_ms * 1e-3) / 8e12)


def forward_vs_backward_total(rt, W, np, torch, n_mu=24, n_phi=8, npx=1024, half_width=70.0):
    """Total power of the magnetar workload star two ways (Sec. 2.4 reports agreement within
    a few percent): forward, the escaped seed weight over N = 2e6 seeds; backward, the image
    sum dP/dOmega over n_mu Gauss-Legendre polar nodes x n_phi azimuths of npx^2 pixels at
    1e5 km, integrated over the sky (the rotating star's total is time independent).  The
    azimuth-averaged dP/dOmega at each polar node is also set against the forward escaped
    weight per unit solid angle in the cell of cos(theta) around the node (Fig. 4's
    comparison); polar_shape_distance is half the L1 distance of the two normalised polar
    distributions."""
    star = W.CFG3["star"]
    tol = W.tol(r_max_km=1e5)
    N = 2_000_000
    print("bench: forward vs backward total power", file=sys.stderr, flush=True)
    t0 = time.time()
    rays, st = rt.rt_sample_resonance(star, 7, N)
    fin, ifin = rt.rt_trace_forward(star, tol, rays, st)
    esc = ifin[2] == 1
    P_fwd = rays[8][esc].sum().item() / N
    xg, wg = np.polynomial.legendre.leggauss(n_mu)
    image = dict(D_km=1e5, half_width_km=half_width, nx=npx, ny=npx)
    area = (2 * half_width / npx) ** 2
    ws = rt.workspace(rt.OP_TRACE_BACKWARD, npx * npx)
    wsp = rt.workspace(rt.OP_BACKWARD_POWER, npx * npx)
    acc = {0.0: 0.0, 1.0: 0.0, 2.0: 0.0}
    dpdo_b = {0.0: np.zeros(n_mu), 1.0: np.zeros(n_mu)}  # azimuth-averaged dP/dOmega per polar node
    for a in range(n_mu):
        for b in range(n_phi):
            image["incl"] = math.acos(xg[a])
            image["phi_o"] = 2 * math.pi * (b + 0.5) / n_phi
            ev, nev, _, _ = rt.rt_trace_backward(star, tol, image, K=8, ws=ws)
            for Lc in acc:
                _, tot = rt.rt_backward_power(star, ev, nev, Lc, pixel_area_km2=area, ws=wsp)
                acc[Lc] += tot.item() * wg[a] * 2 * math.pi / n_phi
                if Lc in dpdo_b:
                    dpdo_b[Lc][a] += tot.item() / n_phi
    # the forward side on the same polar nodes: escaped weight in the cell of cos(theta) around
    # each node (bounded by the midpoints between nodes), per unit solid angle
    mu = torch.cos(fin[8][esc]).cpu().numpy()
    wf = rays[8][esc].cpu().numpy() / N
    edges = np.concatenate([[-1.0], 0.5 * (xg[1:] + xg[:-1]), [1.0]])
    cell, _ = np.histogram(mu, bins=edges, weights=wf)
    dpdo_f = cell / (2 * math.pi * np.diff(edges))
    pf = cell / cell.sum()
    shape = {}
    node_ratio = {}
    for Lc, d in dpdo_b.items():
        key = f"Lc_max_{Lc:g}km" if Lc else "no_cutoff"
        pb = d * wg / (d * wg).sum()
        shape[key] = float(0.5 * np.abs(pf - pb).sum())
        node_ratio[key] = [float(x) for x in d / dpdo_f]
    return dict(workload=f"{W.CFG3['name']} star, {n_mu}x{n_phi} directions x {npx}^2 pixels, {N} forward seeds",
                P_forward_eV2=P_fwd, P_backward_eV2={f"Lc_max_{k:g}km" if k else "no_cutoff": v
                                                     for k, v in acc.items()},
                ratio={f"Lc_max_{k:g}km" if k else "no_cutoff": v / P_fwd for k, v in acc.items()},
                polar_nodes_cos_theta=[float(x) for x in xg],
                dP_dOmega_ratio_backward_over_forward=node_ratio,
                polar_shape_distance=shape,
                seconds=time.time() - t0)


def bench_maxwell(args, rt, W, np, torch):
    """The plain step on the full forward workload with Maxwellian axion momenta at infinity
    (Sec. 4.3 eq. (GaussianDist)) beside the monochromatic one: time per step, total escaped
    power and the spread of the photons' energies at infinity (the line width)."""
    cfg = W.CFG2
    n = cfg["n"]
    out = {}
    for label, speeds in (("monochromatic", W.SPEEDS_MONO), ("maxwellian", W.SPEEDS_MAXWELL)):
        star = dict(cfg["star"], speeds=speeds)
        print(f"bench: maxwell form, {label}", file=sys.stderr, flush=True)
        ws = rt.workspace(rt.OP_TRACE_FORWARD, n)
        rays, st = rt.rt_sample_resonance(star, cfg["seed"], n)
        fin, ifin = rt.rt_trace_forward(star, cfg["tol"], rays, st, ws=ws)
        torch.cuda.synchronize()
        reps = max(2, min(args.steps, 5))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(torch.cuda.current_stream())
        for _ in range(reps):
            rays, st = rt.rt_sample_resonance(star, cfg["seed"], n)
            fin, ifin = rt.rt_trace_forward(star, cfg["tol"], rays, st, ws=ws)
        e1.record(torch.cuda.current_stream())
        torch.cuda.synchronize()
        esc = ifin[2] == 1
        om = fin[11][esc]
        wt = rays[8][esc]
        mean = float((om * wt).sum() / wt.sum())
        sd = float(torch.sqrt(((om - mean) ** 2 * wt).sum() / wt.sum()))
        out[label] = dict(ms_per_step=e0.elapsed_time(e1) / reps,
                          ray_steps_per_s=float(ifin[0].double().sum()) / (e0.elapsed_time(e1) / reps * 1e-3),
                          escaped_power_eV2=float(wt.sum()) / n, omega_mean=mean, omega_sd=sd)
    out["power_ratio"] = out["maxwellian"]["escaped_power_eV2"] / out["monochromatic"]["escaped_power_eV2"]
    out["workload"] = cfg["name"] + " with Maxwellian |k_inf| (dispersion k0 = m_a v0)"
    return out


def bench_magnetar(args, rt, W, np, torch):
    """The four magnetar models of Sec. 6 (M1-M4: lambda in {1, 20}, B0 in {1.6e14, 4e14} G,
    twisted-magnetosphere density, m_a = 1e-4 eV, conversion on open field lines removed):
    1e6 seeds each through seeding, tracing, resonant cyclotron depth and binning; time per
    pass, escaped power before and after absorption, excised fraction."""
    t = W.tol()
    bins = dict(n_theta=64, n_psi=128, n_omega=1, d_omega=1.0)
    n = 1_000_000
    out = {}
    for name, s in W.MAGNETAR_MODELS.items():
        print(f"bench: magnetar {name}", file=sys.stderr, flush=True)
        ws = rt.workspace(rt.OP_TRACE_FORWARD, n)

        def one():
            rays, st = rt.rt_sample_resonance(s, 0, n)
            fin, ifin = rt.rt_trace_forward(s, t, rays, st, ws=ws)
            tau, rcyc, w_out = rt.rt_cyclotron_depth(s, rays, fin, ifin)
            hist, cnt, over = rt.rt_bin_flux(fin, ifin, w_out, bins)
            return rays, st, fin, ifin, tau, w_out, hist

        one()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = max(2, min(args.steps, 3))
        e0.record(torch.cuda.current_stream())
        for _ in range(reps):
            rays, st, fin, ifin, tau, w_out, hist = one()
        e1.record(torch.cuda.current_stream())
        torch.cuda.synchronize()
        esc = ifin[2] == 1
        ok = st == 0
        out[name] = dict(ms_per_pass=e0.elapsed_time(e1) / reps, multiplicity=s["multiplicity"], B0_G=s["B0_G"],
                         excised_fraction=float((st == 7).double().mean()),
                         no_resonance_fraction=float((st == 3).double().mean()),
                         median_r_c_km=float(rays[9][ok].median()) if bool(ok.any()) else None,
                         escaped_power_eV2=float(rays[8][esc].sum()) / n,
                         absorbed_power_eV2=float(w_out[esc].sum()) / n,
                         median_tau=float(tau[esc].median()) if bool(esc.any()) else None,
                         accepted_steps=float(ifin[0].double().sum()))
    return out


def bench_variants(args, rt, W, np, torch):
    """The approximation variants of App. B and Sec. 6, and the Schwarzschild vacuum dipole
    field, beside the full method on the full forward workload (1e6 seeds): time of seeding + tracing, escaped power relative to the
    full method, and the change of the sky distribution: half the L1 distance between the
    normalised escaped-power histograms over cos(theta) (64 bins) of the variant and of the
    full method (0 = same shape, 1 = disjoint)."""
    cfg = W.CFG2
    n = cfg["n"]
    out = {}
    ref = None
    for label, flag in (("full", 0), ("flat_propagation", W.FLAG_FLAT_PROPAGATION),
                        ("thin_surface", W.FLAG_THIN_SURFACE), ("renormalised", W.FLAG_RENORM_WEIGHTS),
                        ("gr_dipole", W.FLAG_GR_DIPOLE)):
        star = dict(cfg["star"], flags=flag)
        print(f"bench: variant {label}", file=sys.stderr, flush=True)
        ws = rt.workspace(rt.OP_TRACE_FORWARD, n)
        rays, st = rt.rt_sample_resonance(star, cfg["seed"], n)
        fin, ifin = rt.rt_trace_forward(star, cfg["tol"], rays, st, ws=ws)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = max(2, min(args.steps, 3))
        e0.record(torch.cuda.current_stream())
        for _ in range(reps):
            rays, st = rt.rt_sample_resonance(star, cfg["seed"], n)
            fin, ifin = rt.rt_trace_forward(star, cfg["tol"], rays, st, ws=ws)
        e1.record(torch.cuda.current_stream())
        torch.cuda.synchronize()
        esc = (ifin[2] == 1).cpu().numpy()
        w = rays[8].cpu().numpy()[esc]
        ct = np.cos(fin[8].cpu().numpy()[esc])
        h, _ = np.histogram(ct, bins=64, range=(-1.0, 1.0), weights=w)
        h = h / h.sum()
        if ref is None:
            ref = (h, w.sum())
        out[label] = dict(ms_per_step=e0.elapsed_time(e1) / reps, escaped_power_eV2=float(w.sum()) / n,
                          power_vs_full=float(w.sum() / ref[1]),
                          sky_shape_change=float(0.5 * np.abs(h - ref[0]).sum()))
    out["workload"] = cfg["name"] + " (renormalised weights: P_ag = 1, arbitrary normalisation)"
    return out


def bench_adjoint(args, rt, W, np, torch):
    """Smoothed flux at 32 observers and its gradient with respect to the six star parameters
    (flat metric, aligned rotator, isotropic plasma, GJ density; 1e6 rays, a checkpoint every
    64 accepted steps):
    forward phase (trace with checkpoints) and reverse phase (recompute + stage adjoints)
    timed separately.  The checkpoint pool is grown to what the rays ask for before timing."""
    cfg = W.CFG5
    star, tol, n, C = cfg["star"], cfg["tol"], cfg["n"], cfg["ckpt_every"]
    obs = W.observers(cfg["n_obs"])
    print(f"bench: adjoint {cfg['name']} n={n}", file=sys.stderr, flush=True)
    fg = rt.FluxGrad(star, tol, cfg["seed"], n, obs, cfg["sigma"], C, 64)
    gbar = torch.linspace(-1.0, 1.0, cfg["n_obs"], dtype=torch.float64, device="cuda")
    _, info = fg.forward(ray_info=True)
    fg.backward(gbar)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    reps = max(2, min(args.steps, 5))
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(reps)]
    for r in range(reps):
        ev[r][0].record(stream)
        fg.forward()
        ev[r][1].record(stream)
        fg.backward(gbar)
        ev[r][2].record(stream)
    torch.cuda.synchronize()
    fwd_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    rev_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
    inf = info.cpu().numpy().astype(np.int64)
    acc, rej, st = inf[0], inf[1], inf[2]
    traced = st != W.STATUS_NO_RESONANCE
    esc = st == W.STATUS_ESCAPED
    # the star's own counts: the right-hand sides take the aligned axis where sin theta_m = 0,
    # and the stage products' counts include their rotating-axis pass
    ft = flop_table()[variant_key(cfg["star"])]
    flops_fwd = float((acc + rej)[traced].sum()) * ft["attempt"] + float(traced.sum()) * 3 * ft["rhs"]
    nseg = (acc[esc] + C - 1) // C
    # reverse, per escaped ray: recompute every attempt of its segments, then per accepted step
    # one FSAL derivative + the step's stages again (no error estimate) + the six stage
    # adjoints + the b-weights
    flops_rev = (float((acc + rej)[esc].sum()) * ft["attempt"] + float(nseg.sum()) * ft["rhs"]
                 + float(acc[esc].sum()) * (ft["rhs"] + ft["stages"] + ft["stages_adjoint"] + 80))
    tot_ms = fwd_ms + rev_ms
    return dict(workload=cfg["name"], rays=n, traced_rays=int(traced.sum()), escaped_rays=int(esc.sum()),
                observers=cfg["n_obs"], ckpt_every=C, forward_ms=fwd_ms, reverse_ms=rev_ms,
                ms_per_gradient=tot_ms, accepted_steps=float(acc[traced].sum()),
                ray_steps_per_s=float(acc[traced].sum()) / (tot_ms * 1e-3),
                rays_per_s=float(traced.sum()) / (tot_ms * 1e-3),
                forward_tflops=flops_fwd / (fwd_ms * 1e-3) / 1e12, reverse_tflops=flops_rev / (rev_ms * 1e-3) / 1e12,
                flop_per_vjp=ft["vjp"], flop_per_stage_adjoint=ft["stages_adjoint"],
                checkpoints=int(fg.ckpt_used.item()), checkpoint_pool=int(fg.ckpt_pool),
                checkpoint_bytes=int(fg.ckpt_used.item()) * 96, workspace_bytes=int(fg.ws.numel()))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=None, help="rays per step (default: the workload's 1e6)")
    ap.add_argument("--cpu-sample", type=int, default=1 << 19,
                    help="rays of the CPU oracle sample (about 15 s on 16 host threads)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--schedule", type=str, default=None, help="JSON rt_schedule override")
    ap.add_argument("--forms", type=str, default="plain,batched,adjoint,backward,maxwell,magnetar,variants,fbtotal",
                    help="comma list of forms to time beside plain (the headline value): batched, adjoint, "
                         "backward, maxwell (Maxwellian axion speeds), magnetar (models M1-M4 with excision "
                         "and cyclotron absorption), variants (flat propagation, thin surface, renormalised "
                         "weights), fbtotal (forward against backward total power of the magnetar star)")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the plain form's schedule too (default: the library's default schedule)")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner in the batched form")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 5 times (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps(dict(copy_probe_bytes=src.numel() * 8, repeats=5)))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the tracer shards rays across GPUs by index with no "
              "communication until one histogram all-reduce, which this build does not run; use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2309_08655_amd as rt
    import workloads as W

    cfg = dict(W.CFG2)
    n = args.n or cfg["n"]
    sched = json.loads(args.schedule) if args.schedule else None
    forms = set(args.forms.split(","))
    dev = torch.device("cuda")
    rays = torch.empty((10, n), dtype=torch.float64, device=dev)
    status = torch.empty(n, dtype=torch.int32, device=dev)
    fin = torch.empty((rt.RT_NFIN, n), dtype=torch.float64, device=dev)
    ifin = torch.empty((rt.RT_NIFIN, n), dtype=torch.int32, device=dev)
    ws = rt.workspace(rt.OP_TRACE_FORWARD, n)
    wsb = rt.workspace(rt.OP_BIN, n)
    b = cfg["bins"]
    hist = torch.empty((1, b["n_theta"], b["n_psi"], b["n_omega"]), dtype=torch.float64, device=dev)
    cnt = torch.empty_like(hist)
    over = torch.empty(2, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        rt.rt_sample_resonance(cfg["star"], cfg["seed"], n, rays=rays, status=status)
        rt.rt_trace_forward(cfg["star"], cfg["tol"], rays, status, schedule=sched, ws=ws, fin=fin, ifin=ifin)
        rt.rt_bin_flux(fin, ifin, rays[8], b, ws=wsb, hist=hist, cnt=cnt, over=over)

    tune_times = None
    if sched is None and args.tune:
        from paper_2309_08655_amd import autotune
        rt.rt_sample_resonance(cfg["star"], cfg["seed"], n, rays=rays, status=status)
        sched, tune_times = autotune.tune(
            lambda sc: rt.rt_trace_forward(cfg["star"], cfg["tol"], rays, status, schedule=sc, ws=ws, fin=fin,
                                           ifin=ifin), key=f"{cfg['name']}|{n}")
        print(f"bench: autotuned schedule {sched}", file=sys.stderr, flush=True)

    print(f"bench: {cfg['name']} n={n} warmup={args.warmup} steps={args.steps}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    # HIP events around every launch of the persistent tracing kernel, on its stream
    rt.timing(True)
    t_start.record(stream)
    for k in range(args.steps):
        step()
    t_end.record(stream)
    torch.cuda.synchronize()
    rt.timing(False)
    total_ms = t_start.elapsed_time(t_end)
    ms_step = total_ms / args.steps
    ktimes = [ms for name, ms in rt.kernel_times() if name == "trace_fwd_kernel"]
    assert len(ktimes) == args.steps, ktimes
    trace_ms = float(np.mean(ktimes))

    ifn = ifin.cpu().numpy()
    stn = status.cpu().numpy()
    # wave-iterations of the persistent loop (third 64-bit word of the work counter)
    wave_iters = int(ws[16:24].cpu().numpy().view(np.uint64)[0])
    restarts = int(ws[32:40].cpu().numpy().view(np.uint64)[0])  # work counter pad[1]
    att = (ifn[0].astype(np.int64) + ifn[1])[stn == 0]
    acc = float(ifn[0].astype(np.float64).sum())
    rej = float(ifn[1].astype(np.float64).sum())
    n_traced = float((stn == 0).sum())
    steps_per_s = acc / (ms_step * 1e-3)
    rays_per_s = n_traced / (ms_step * 1e-3)

    ft = flop_table()[variant_key(cfg["star"])]
    # algorithmic work of one launch of the persistent tracing kernel: one DOPRI5 attempt per
    # attempted step (the FSAL derivative and starting step come from the init kernel)
    flops = (acc + rej) * ft["attempt"]
    achieved_tflops = flops / (trace_ms * 1e-3) / 1e12
    cv = counter_values(n)
    roofline = dict(bound="alu", achieved=achieved_tflops, peak=FP64_VECTOR_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=achieved_tflops / FP64_VECTOR_PEAK_TFLOPS, traffic=cv.get("hbm_bytes_per_launch"),
                    kernel="trace_fwd_kernel", kernel_ms=trace_ms, flop_per_attempt=ft["attempt"],
                    attempted_steps=acc + rej, flop_per_launch=flops)
    if "hw_fp64_flops_per_launch" in cv:
        # the hardware's own FP64 operation count (every lane of every issued FP64
        # instruction: library expansions, Newton refinements, idle lanes included)
        hw = cv["hw_fp64_flops_per_launch"] / (trace_ms * 1e-3) / 1e12
        roofline.update(hw_fp64_tflops=hw, hw_fp64_frac=hw / FP64_VECTOR_PEAK_TFLOPS)
    out = dict(metric="ray-steps/s and rays/s at rtol 1e-8 (FP64), plain vs batched vs adjoint",
               value=steps_per_s, unit="ray-steps/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
               ms_per_step=ms_step, higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f64",
               data="synthetic",
               config=dict(workload=cfg["name"], rays_per_step=n, form="plain",
                           rays_per_s=rays_per_s, accepted_steps=acc, rejected_steps=rej,
                           statuses={str(k): int(v) for k, v in zip(*np.unique(ifn[2], return_counts=True))},
                           lane_efficiency=(acc + rej) / max(1, 64 * wave_iters),
                           null_surface_restarts=restarts,
                           attempts_per_ray=dict(mean=float(att.mean()), p99=float(np.percentile(att, 99)),
                                                 p9999=float(np.percentile(att, 99.99)), max=int(att.max())),
                           schedule=sched, autotune_ms=tune_times),
               roofline=roofline)
    out["forms"] = {}
    if "batched" in forms:
        out["forms"]["batched"] = bench_batched(args, rt, W, np, torch)
    if "adjoint" in forms:
        out["forms"]["adjoint"] = bench_adjoint(args, rt, W, np, torch)
    if "backward" in forms:
        out["forms"]["backward"] = bench_backward(args, rt, W, np, torch)
    if "magnetar" in forms:
        out["forms"]["magnetar"] = bench_magnetar(args, rt, W, np, torch)
    if "variants" in forms:
        out["forms"]["variants"] = bench_variants(args, rt, W, np, torch)
    if "maxwell" in forms:
        out["forms"]["maxwell"] = bench_maxwell(args, rt, W, np, torch)
    if "fbtotal" in forms:
        out["forms"]["forward_vs_backward"] = forward_vs_backward_total(rt, W, np, torch)
    if not args.no_cpu:
        aff, threads = host_threads()
        print(f"bench: cpu baseline on {args.cpu_sample} rays, {threads} threads ({aff} cores in the affinity "
              f"mask)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_sample, threads)
        # the oracle beside each form, on the bounded samples of the same workloads
        for form, fn in (("batched", cpu_baseline_batched), ("adjoint", cpu_baseline_adjoint),
                         ("backward", cpu_baseline_backward)):
            if form in out["forms"]:
                print(f"bench: cpu baseline of the {form} form", file=sys.stderr, flush=True)
                out["forms"][form]["cpu_baseline"] = fn(W, threads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
