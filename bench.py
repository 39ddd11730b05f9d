#!/usr/bin/env python3
"""Benchmark of the TACAW hot path on one MI355X.

Workload (one "step"): the 512 x 512 grid class of the batched uneven configuration - 8 rocksalt
specimens of 160 x 160 Angstrom with 10, 20, ..., 80 slices of 2 Angstrom, a 100 keV probe
(30 mrad, Cs = 0) scanned over 8 x 8 positions, 256 snapshots at 5 fs.  One step runs the whole
path from atom positions resident in HBM: slice potentials of every snapshot, batched multislice of
all 8 x 64 x 256 waves (8 position chunks of 8 positions, every chunk one uneven batched call),
periodograms accumulated over positions, Kubo correction and normalisation of the 256-bin
S(q, omega) of every specimen.

Metric: snapshot-slice steps per second = (probe positions x snapshots x sum of slices) / step time.
The timed steps replay the captured slice-loop graphs (no instrumentation).  After them: one exit
wave of the last timed step is recomputed by the FP64 oracle (rel-L2 <= 1e-4, else exit status 3),
and one instrumented step brackets every kernel with HIP events on its stream for the per-kernel
durations, algorithmic bandwidths and the roofline of the dominant slice-step pass.
Side legs (outside the timed region): the plain one-snapshot-per-launch path on a labelled subset
(batched vs plain), the whole 24-specimen batched-uneven configuration (128^2/256^2/512^2 classes;
plain, batched and persistent modes), the adjoint/forward time ratio on the differentiation
configuration, a plane-wave 512^2 batch with the analysis outputs, the 560^2 and 1000^2 grids and
the large 1024^2 configuration; then the CPU baselines (FP64 oracle, scipy.fft) on the host cores.

Prints ONE JSON line.  Progress goes to stderr.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=1)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--snapshots", type=int, default=256, help="trajectory length per specimen")
    p.add_argument("--specimens", type=int, default=8, help="specimens of the 512^2 class (<= 8)")
    p.add_argument("--pos-chunk", type=int, default=8, help="probe positions per batched call")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--no-legs", action="store_true", help="skip the side legs")
    p.add_argument("--no-full", action="store_true",
                   help="skip the whole 24-specimen batched-uneven leg")
    p.add_argument("--no-check", action="store_true",
                   help="skip the oracle check of one exit wave of the timed work")
    p.add_argument("--cpu-budget-s", type=float, default=20.0)
    p.add_argument("--calibrate", action="store_true",
                   help="run a 1 GiB device-to-device copy first (HBM counter calibration)")
    p.add_argument("--profile-slice-step", action="store_true",
                   help="short run for counter collection: one batched 512^2 multislice call of "
                        "the workload (8 snapshots) and a 1 GiB device copy as HBM calibration")
    p.add_argument("--odd-grids-only", action="store_true",
                   help="run only the 560^2 and 1000^2 lines (for kernel traces of their passes)")
    p.add_argument("--large-only", action="store_true",
                   help="run only the large configuration at full size (1024^2, 2048 snapshots)")
    p.add_argument("--adjoint-only", action="store_true",
                   help="run only the adjoint line (256^2 differentiation workload)")
    p.add_argument("--summarize-traffic", nargs=4,
                   metavar=("FETCH_CSV", "WRITE_CSV", "FETCH_RUN_JSON", "OUT_JSON"),
                   help="turn two rocprofv3 counter files (FETCH_SIZE, WRITE_SIZE) of a --calibrate "
                        "run (and the JSON line that run printed) into the HBM traffic record of the "
                        "512^2 slice-step passes")
    return p.parse_args()


# ------------------------------------------------------------------------------------------------
def make_specimens(n_spec, T, device, grids=(512,)):
    import torch
    from workloads.configs import c3_specimens, make_workload
    specs = []
    for n in grids:
        specs += [c for c in c3_specimens() if c["n"] == (n, n)][:n_spec]
    out = []
    for cfg in specs:
        w = make_workload(cfg, n_snap=T, generate=False, name=f"c3-{cfg['n'][0]}-S{cfg['n_slices']}")
        from workloads.trajectory import harmonic_trajectory
        w.positions = harmonic_trajectory(w.extra["structure"], T, cfg["dt"], cfg["seed"],
                                          device=device)
        w.species_dev = torch.from_numpy(w.species).to(device)
        out.append(w)
    return out


def run_step(tw, ctx, ws, Vs, exits, Ps, Ss, pos_chunk, mode=None, ms_events=None):
    """One pass of the whole hot path over the batch.  With ms_events (a list), a pair of CUDA
    events on the caller's stream brackets every multislice call (the library joins its side
    streams back into that stream before the call returns)."""
    import torch
    mode = tw.MODE_BATCHED if mode is None else mode
    spec_objs = [tw.specimen_from(w) for w in ws]
    for w, sp, V in zip(ws, spec_objs, Vs):
        tw.tacaw_build_potentials(ctx, sp, w.positions, w.species_dev, w.ff, V)
    P = ws[0].n_pos
    for c0 in range(0, P, pos_chunk):
        jobs = []
        for w, sp, V, ex in zip(ws, spec_objs, Vs, exits):
            b = tw.Beam(w.energy_ev, True, w.alpha_rad, 0.0, 0.0, w.probe_xy[c0:c0 + pos_chunk])
            jobs.append(tw.MsJob(sp, b, V, ex))
        if ms_events is not None:
            ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            ev[0].record()
        tw.tacaw_multislice(ctx, jobs, mode=mode)
        if ms_events is not None:
            ev[1].record()
            ms_events.append(ev)
        for w, ex, Pacc in zip(ws, exits, Ps):
            tw.tacaw_periodogram(ctx, ex, w.n_e, w.hop, Pacc, accumulate=c0 > 0)
    for w, Pacc, S in zip(ws, Ps, Ss):
        opts = tw.SpectrumOpts(w.dt_fs, w.temperature_k, w.n_e, w.hop, w.nx, w.ny)
        tw.tacaw_spectrum_finalize(ctx, Pacc, opts, S)


def plain_leg(tw, ctx, ws, Vs):
    """Plain one-snapshot-per-launch path vs batched on the same labelled subset:
    the 40-slice specimen, 4 probe positions, 32 snapshots."""
    import torch
    w = [x for x in ws if x.n_slices == 40][0] if any(x.n_slices == 40 for x in ws) else ws[-1]
    nt = min(32, Vs[ws.index(w)].shape[0])
    V = Vs[ws.index(w)][:nt].contiguous()
    ex = torch.empty((nt, 4, w.ny, w.nx), dtype=torch.complex64, device="cuda:0")
    sp = tw.specimen_from(w)
    b = tw.Beam(w.energy_ev, True, w.alpha_rad, 0.0, 0.0, w.probe_xy[:4])
    steps = nt * 4 * w.n_slices
    out = {}
    for name, mode in (("plain", tw.MODE_PLAIN), ("batched", tw.MODE_BATCHED)):
        tw.tacaw_multislice(ctx, [tw.MsJob(sp, b, V, ex)], mode=mode)
        torch.cuda.synchronize()
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            tw.tacaw_multislice(ctx, [tw.MsJob(sp, b, V, ex)], mode=mode)
        torch.cuda.synchronize()
        out[name] = steps * reps / (time.perf_counter() - t0)
    return dict(subset=f"{w.name}: 4 positions x {nt} snapshots x {w.n_slices} slices, 512^2",
                plain_slice_steps_per_s=out["plain"], batched_slice_steps_per_s=out["batched"],
                batched_over_plain=out["batched"] / out["plain"])


def adjoint_leg(tw):
    """Adjoint/forward time ratio on the differentiation configuration (256^2, 20 slices,
    128 snapshots, B/N-like layers): checkpointed forward vs checkpointed adjoint."""
    import torch
    from workloads import make_workload
    ctx = tw.context(0)
    w = make_workload("c4", device="cuda:0")
    sp, bm = tw.specimen_from(w), tw.beam_from(w)
    T, S = w.n_snap, w.n_slices
    k = math.ceil(math.sqrt(S))
    nck = (S + k - 1) // k
    xyz = w.positions
    spc = torch.from_numpy(w.species).to("cuda:0")
    V = torch.empty((T, S, w.ny, w.nx), dtype=torch.float32, device="cuda:0")
    tw.tacaw_build_potentials(ctx, sp, xyz, spc, w.ff, V)
    ex = torch.empty((T, 1, w.ny, w.nx), dtype=torch.complex64, device="cuda:0")
    ck = torch.empty((T, 1, nck, w.ny, w.nx), dtype=torch.complex64, device="cuda:0")
    gex = torch.randn((T, 1, w.ny, w.nx), dtype=torch.complex64, device="cuda:0")
    gV = torch.empty_like(V)
    gxy = torch.empty((T, xyz.shape[1], 2), dtype=torch.float32, device="cuda:0")

    def fwd():
        tw.tacaw_multislice(ctx, [tw.MsJob(sp, bm, V, ex, ck)], ckpt_stride=k, mode=tw.MODE_BATCHED)

    def adj():
        tw.tacaw_multislice_adjoint(ctx, [tw.MsJob(sp, bm, V, None, ck)], k, [gex], [gV])

    def adj_xy():
        adj()
        tw.tacaw_build_potentials_backward(ctx, sp, xyz, spc, w.ff, gV, gxy)

    def timeit(f, reps=3):
        f()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            f()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    def fwd_pot():
        tw.tacaw_build_potentials(ctx, sp, xyz, spc, w.ff, V)
        fwd()

    tf, ta, tax, tfp = timeit(fwd), timeit(adj), timeit(adj_xy), timeit(fwd_pot)
    return dict(config="B/N-like 16x9x10 cells, 256^2, 20 slices, 128 snapshots, ckpt stride 5",
                forward_ms=tf * 1e3, adjoint_ms=ta * 1e3, adjoint_plus_positions_ms=tax * 1e3,
                forward_with_potentials_ms=tfp * 1e3,
                adjoint_over_forward=ta / tf, adjoint_with_positions_over_forward=tax / tf,
                adjoint_with_positions_over_forward_with_potentials=tax / tfp)


def plane_wave_leg(tw):
    """Secondary line: a homogeneous plane-wave 512^2 batch (rocksalt 40 x 40 x 20 cells,
    0.3125 A pixels, 40 slices, 256 snapshots, trajectory seed 6001); multislice only, median of
    5 timed calls after one warm-up call."""
    import torch
    from workloads.configs import make_workload
    from workloads.trajectory import harmonic_trajectory
    ctx = tw.context(0)
    cfg = dict(kind="rocksalt", a=4.0, reps=(40, 40, 20), n=(512, 512), n_slices=40, dz=2.0,
               energy=100e3, T=256, dt=5.0, n_e=256, hop=256, seed=6001, probe=False, alpha=0.0)
    w = make_workload(cfg, generate=False, name="plane-wave-512-S40")
    T = cfg["T"]
    xyz = harmonic_trajectory(w.extra["structure"], T, cfg["dt"], cfg["seed"], device="cuda:0")
    sp, bm = tw.specimen_from(w), tw.Beam(w.energy_ev)
    V = torch.empty((T, w.n_slices, w.ny, w.nx), dtype=torch.float32, device="cuda:0")
    tw.tacaw_build_potentials(ctx, sp, xyz, torch.from_numpy(w.species).to("cuda:0"), w.ff, V)
    del xyz
    ex = torch.empty((T, 1, w.ny, w.nx), dtype=torch.complex64, device="cuda:0")
    job = [tw.MsJob(sp, bm, V, ex)]
    tw.tacaw_multislice(ctx, job, mode=tw.MODE_BATCHED)
    torch.cuda.synchronize()
    times = []
    for _ in range(5):
        t0 = time.perf_counter()
        tw.tacaw_multislice(ctx, job, mode=tw.MODE_BATCHED)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    med = sorted(times)[len(times) // 2]
    steps = T * w.n_slices
    # analysis outputs of the same exit waves: spectrum, energy-integrated patterns, QEP patterns
    # (all snapshots and every 16th), the q_y = 0 relative-difference profile and a Gamma-X-M-Gamma
    # dispersion cut; the c~ pattern must equal the all-snapshot QEP pattern (one segment)
    n_e = 256
    opts = tw.SpectrumOpts(w.dt_fs, 300.0, n_e, n_e, w.nx, w.ny)
    P = torch.empty((n_e, w.ny, w.nx), dtype=torch.float32, device="cuda:0")
    S = torch.empty_like(P)
    ct, c, q_all, q16 = (torch.empty((w.ny, w.nx), dtype=torch.float32, device="cuda:0") for _ in range(4))
    prof = torch.empty(w.nx, dtype=torch.float32, device="cuda:0")
    a = 4.0
    verts = [(0.0, 0.0), (1.0 / a, 0.0), (1.0 / a, 1.0 / a), (0.0, 0.0)]
    cut = torch.empty((n_e, 3 * 64 + 1), dtype=torch.float32, device="cuda:0")
    steps_an = [
        ("periodogram", lambda: tw.tacaw_periodogram(ctx, ex, n_e, n_e, P)),
        ("finalize", lambda: tw.tacaw_spectrum_finalize(ctx, P, opts, S)),
        ("energy_integrals", lambda: tw.tacaw_energy_integrals(ctx, P, opts, ct, c)),
        ("qep_all", lambda: tw.tacaw_qep_pattern(ctx, ex, 0, 1, T, q_all)),
        ("qep_every_16th", lambda: tw.tacaw_qep_pattern(ctx, ex, 0, 16, T // 16, q16)),
        ("relative_difference", lambda: tw.tacaw_relative_difference(ctx, c, q16, prof)),
        ("path_cut", lambda: tw.tacaw_path_cut(ctx, w.lx, w.ly, S, verts, 64, cut)),
    ]
    an_ms = {}
    for name, f in steps_an:
        f()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f()
        torch.cuda.synchronize()
        an_ms[name] = (time.perf_counter() - t0) * 1e3
    parseval = float(((ct - q_all).abs().max() / q_all.abs().max()).item())
    return dict(workload="plane wave, rocksalt 40x40x20 cells, 512^2, 40 slices, 256 snapshots",
                slice_steps=steps, median_ms=med * 1e3, slice_steps_per_s=steps / med,
                analysis_ms=an_ms, parseval_max_rel_diff=parseval)


def odd_grid_leg(tw):
    """Secondary lines on the grids of the paper's own runs, whose lengths are not powers of two
    (synthetic stand-ins, multislice only, median of 3 timed calls after one warm-up call):
      * 560^2: silicon-like diamond crystal, 7 x 7 x 23 cubic cells (a = 5.4773 A; a quarter of
        the paper's 92-cell thickness), 184 slices of a/8, 60 keV plane wave, 64 snapshots at
        25 fs (trajectory seed 7001);
      * 1000^2: iron-like bcc crystal, 20 x 20 x 4 cells (a = 2.87 A), 120 slices of a/30,
        200 keV probe of 1 mrad at one position, 32 snapshots at 4 fs (seed 7002).
    Per-pass rates are the algorithmic bytes of the x and y passes over their kernel time."""
    import torch
    from workloads.configs import make_workload
    from workloads.trajectory import harmonic_trajectory
    out = {}
    legs = [
        ("si_560", dict(kind="diamond", a=5.4773, reps=(7, 7, 23), n=(560, 560), n_slices=184,
                        dz=5.4773 / 8, energy=60e3, T=64, dt=25.0, n_e=64, hop=64, seed=7001,
                        probe=False, alpha=0.0),
         "plane wave 60 keV, silicon-like 7x7x23 cells, 560^2, 184 slices, 64 snapshots"),
        ("fe_1000", dict(kind="bcc", a=2.87, reps=(20, 20, 4), n=(1000, 1000), n_slices=120,
                         dz=2.87 / 30, energy=200e3, T=32, dt=4.0, n_e=32, hop=32, seed=7002,
                         probe=True, alpha=1e-3),
         "probe 200 keV 1 mrad, iron-like bcc 20x20x4 cells, 1000^2, 120 slices, 32 snapshots"),
    ]
    for key, cfg, desc in legs:
        ctx = tw.Context(0)
        w = make_workload(cfg, generate=False, name=key)
        if w.probe:
            w.probe_xy = w.probe_xy[:1]
        T = cfg["T"]
        xyz = harmonic_trajectory(w.extra["structure"], T, cfg["dt"], cfg["seed"], device="cuda:0")
        sp = tw.specimen_from(w)
        V = torch.empty((T, w.n_slices, w.ny, w.nx), dtype=torch.float32, device="cuda:0")
        tw.tacaw_build_potentials(ctx, sp, xyz, torch.from_numpy(w.species).to("cuda:0"), w.ff, V)
        del xyz
        n_pos = len(w.probe_xy) if w.probe else 1
        ex = torch.empty((T, n_pos, w.ny, w.nx), dtype=torch.complex64, device="cuda:0")
        job = [tw.MsJob(sp, tw.beam_from(w), V, ex)]
        tw.tacaw_multislice(ctx, job, mode=tw.MODE_BATCHED)
        torch.cuda.synchronize()
        times = []
        for _ in range(3):
            t0 = time.perf_counter()
            tw.tacaw_multislice(ctx, job, mode=tw.MODE_BATCHED)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        tw.tacaw_set_slice_blocking(ctx, tw.SLICE_BLOCK_BYTES, 1)   # one stream: no overlap
        tw.tacaw_set_timing(ctx, True)
        tw.tacaw_multislice(ctx, job, mode=tw.MODE_BATCHED)
        torch.cuda.synchronize()
        kinds = {k: tw.tacaw_get_timing(ctx, k) for k in ("row", "col")}
        tw.tacaw_set_timing(ctx, False)
        tw.tacaw_set_slice_blocking(ctx, tw.SLICE_BLOCK_BYTES, tw.SLICE_BLOCK_STREAMS)
        med = sorted(times)[len(times) // 2]
        steps = T * n_pos * w.n_slices
        out[key] = dict(
            workload=desc, slice_steps=steps, median_ms=med * 1e3, slice_steps_per_s=steps / med,
            pixel_slice_steps_per_s=steps * w.nx * w.ny / med,
            pass_GBps={k: (v["algo_bytes"] / (v["total_ms"] * 1e-3) / 1e9) if v["total_ms"] else None
                       for k, v in kinds.items()},
            pass_ms={k: v["total_ms"] for k, v in kinds.items()},
            schedule=tw.tacaw_describe_schedule(ctx, w.nx))
        del V, ex, job, ctx
        torch.cuda.empty_cache()
    return out


def inrun_oracle_check(ws, exits, pos_chunk):
    """One exit wave of the benchmark's own timed work against the FP64 oracle: the 80-slice
    specimen, the last snapshot, the first probe position of the last position chunk (the
    buffers hold that chunk after the timed steps).  The oracle rebuilds the slice potentials of
    that snapshot from the same float32 positions and propagates the wave by dense DFTs."""
    from types import SimpleNamespace
    from oracle import multislice as o_ms
    from oracle import potential as o_pot
    k = max(range(len(ws)), key=lambda i: ws[i].n_slices)
    w = ws[k]
    t = w.n_snap - 1
    p0 = ((w.n_pos - 1) // pos_chunk) * pos_chunk
    t0 = time.perf_counter()
    pos = w.positions[t:t + 1].float().cpu().numpy()
    V, _ = o_pot.potentials(pos, w.species, w.ff, w)
    beam = SimpleNamespace(probe=True, energy_ev=w.energy_ev, alpha_rad=w.alpha_rad,
                           defocus_a=w.defocus_a, cs_a=w.cs_a, probe_xy=w.probe_xy[p0:p0 + 1])
    ref = o_ms.exit_waves(V, w, beam)[0, 0]
    got = exits[k][t, 0].cpu().numpy().astype(np.complex128)
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    return dict(wave=f"{w.name}: snapshot {t}, probe position {p0}, {w.n_slices} slices, {w.nx}^2",
                rel_l2=err, tolerance=1e-4, passed=bool(err <= 1e-4),
                oracle_s=time.perf_counter() - t0)


def full_uneven_leg(tw, T=256, pos_chunk=8):
    """The whole batched-uneven configuration: 24 rocksalt specimens (8 each on 128^2, 256^2 and
    512^2 grids, 10..80 slices), the 100 keV 30 mrad probe at 8 x 8 positions, T snapshots.  The
    multislice of all 24 specimens runs as one call per chunk of probe positions; timed once over
    all 64 positions in the batched mode (one graph of per-slice launches) and in the persistent
    mode (classes as concurrent graph branches, the 128^2 class in one resident launch), and in
    the plain mode on a labelled subset (one specimen per class, 4 positions, 16 snapshots)."""
    import torch
    ctx = tw.context(0)
    ws = make_specimens(8, T, "cuda:0", grids=(128, 256, 512))
    Vs = [torch.empty((T, w.n_slices, w.ny, w.nx), dtype=torch.float32, device="cuda:0") for w in ws]
    for w, V in zip(ws, Vs):
        tw.tacaw_build_potentials(ctx, tw.specimen_from(w), w.positions, w.species_dev, w.ff, V)
    for w in ws:
        w.positions = None
    torch.cuda.synchronize()
    exits = [torch.empty((T, pos_chunk, w.ny, w.nx), dtype=torch.complex64, device="cuda:0") for w in ws]
    specs = [tw.specimen_from(w) for w in ws]
    P = ws[0].n_pos

    def jobs_for(c0, npos=pos_chunk, subset=None, nt=None):
        out = []
        for i, (w, sp, V, ex) in enumerate(zip(ws, specs, Vs, exits)):
            if subset is not None and i not in subset:
                continue
            b = tw.Beam(w.energy_ev, True, w.alpha_rad, 0.0, 0.0, w.probe_xy[c0:c0 + npos])
            out.append(tw.MsJob(sp, b, V if nt is None else V[:nt], ex if nt is None else ex[:nt, :npos]))
        return out

    steps = sum(w.n_slices for w in ws) * P * T
    res = {}
    for name, mode in (("batched", tw.MODE_BATCHED), ("persistent", tw.MODE_PERSISTENT)):
        tw.tacaw_multislice(ctx, jobs_for(0), mode=mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for c0 in range(0, P, pos_chunk):
            tw.tacaw_multislice(ctx, jobs_for(c0), mode=mode)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res[name] = dict(seconds=dt, slice_steps_per_s=steps / dt)
        log(f"[full] {name}: {dt:.2f} s, {steps / dt / 1e6:.3f} M snapshot-slice steps/s")
    # plain vs batched vs persistent on the subset (exit buffers sliced to 4 positions x 16 snapshots)
    sub = [i for i, w in enumerate(ws) if w.n_slices == 40]
    nt = 16
    sub_steps = sum(ws[i].n_slices for i in sub) * 4 * nt
    for name, mode in (("plain", tw.MODE_PLAIN), ("batched", tw.MODE_BATCHED),
                       ("persistent", tw.MODE_PERSISTENT)):
        j = jobs_for(0, npos=4, subset=sub, nt=nt)
        j = [tw.MsJob(x.spec, x.beam, x.V.contiguous(), torch.empty((nt, 4, x.spec.ny, x.spec.nx),
                      dtype=torch.complex64, device="cuda:0")) for x in j]
        tw.tacaw_multislice(ctx, j, mode=mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            tw.tacaw_multislice(ctx, j, mode=mode)
        torch.cuda.synchronize()
        res[f"subset_{name}_slice_steps_per_s"] = sub_steps * 3 / (time.perf_counter() - t0)
    res["subset"] = "the 40-slice specimen of each class, 4 probe positions x 16 snapshots"
    res["persistent_over_batched"] = res["persistent"]["slice_steps_per_s"] / res["batched"]["slice_steps_per_s"]
    res["subset_batched_over_plain"] = res["subset_batched_slice_steps_per_s"] / res["subset_plain_slice_steps_per_s"]
    res["workload"] = ("24 rocksalt specimens (8 x 128^2, 8 x 256^2, 8 x 512^2; 10..80 slices), "
                       f"30 mrad probe at 8x8 positions, {T} snapshots; multislice only")
    res["slice_steps"] = steps
    del Vs, exits
    torch.cuda.empty_cache()
    return res


def large_run(tw, chunk=64, keep=False):
    """The large configuration at full size: B/N-like hexagonal crystal of 40 x 40 x 50 cells
    (640,000 atoms), 1024^2 grid, 100 slices of 3.33 A, 60 keV plane wave, 2048 snapshots at 2 fs
    (trajectory seed 5001), S(q, w) with 1024 energy bins and hop 512 (3 segments).  Its potentials
    (819 GB) cannot all be resident, so the snapshots stream through in chunks: potentials of a
    chunk, then the chunk's batched multislice into the resident exit stack (17 GB); the spectrum
    follows from the whole stack.  Returns timings (and, with keep, the device buffers)."""
    import torch
    from workloads.configs import CONFIGS, make_workload
    from workloads.trajectory import harmonic_trajectory
    cfg = CONFIGS["c5"]
    ctx = tw.Context(0)
    w = make_workload(cfg, generate=False, name="large-1024")
    T, S = w.n_snap, w.n_slices
    t_gen = time.perf_counter()
    xyz = harmonic_trajectory(w.extra["structure"], T, w.dt_fs, w.seed, omega_a_mev=cfg["omega_a"],
                              omega_o_mev=cfg["omega_o"], device="cuda:0")
    species = torch.from_numpy(w.species).to("cuda:0")
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    sp, bm = tw.specimen_from(w), tw.beam_from(w)
    ex = torch.empty((T, 1, w.ny, w.nx), dtype=torch.complex64, device="cuda:0")
    V = torch.empty((chunk, S, w.ny, w.nx), dtype=torch.float32, device="cuda:0")
    t_pot = t_ms = 0.0
    for t0 in range(0, T, chunk):
        n = min(chunk, T - t0)
        a = time.perf_counter()
        tw.tacaw_build_potentials(ctx, sp, xyz[t0:t0 + n], species, w.ff, V[:n])
        torch.cuda.synchronize()
        b = time.perf_counter()
        tw.tacaw_multislice(ctx, [tw.MsJob(sp, bm, V[:n], ex[t0:t0 + n])], mode=tw.MODE_BATCHED)
        torch.cuda.synchronize()
        t_pot += b - a
        t_ms += time.perf_counter() - b
        if (t0 // chunk) % 8 == 7:
            log(f"[large] {t0 + n}/{T} snapshots: potentials {t_pot:.1f} s, multislice {t_ms:.1f} s")
    # per-pass bandwidth: the last chunk's multislice again, launches isolated on one stream and
    # bracketed by HIP events (algorithmic bytes of the band-limited columns)
    t0 = ((T - 1) // chunk) * chunk
    n = T - t0
    tw.tacaw_set_slice_blocking(ctx, tw.SLICE_BLOCK_BYTES, 1)
    tw.tacaw_set_timing(ctx, True)
    tw.tacaw_multislice(ctx, [tw.MsJob(sp, bm, V[:n], ex[t0:t0 + n])], mode=tw.MODE_BATCHED)
    torch.cuda.synchronize()
    kinds = {k: tw.tacaw_get_timing(ctx, k) for k in ("row", "col")}
    tw.tacaw_set_timing(ctx, False)
    tw.tacaw_set_slice_blocking(ctx, tw.SLICE_BLOCK_BYTES, tw.SLICE_BLOCK_STREAMS)
    pass_GBps = {k: (v["algo_bytes"] / (v["total_ms"] * 1e-3) / 1e9) if v["total_ms"] else None
                 for k, v in kinds.items()}
    opts = tw.SpectrumOpts(w.dt_fs, w.temperature_k, w.n_e, w.hop, w.nx, w.ny)
    Pacc = torch.empty((w.n_e, w.ny, w.nx), dtype=torch.float32, device="cuda:0")
    Sq = torch.empty_like(Pacc)
    norm = torch.empty((1,), dtype=torch.float64, device="cuda:0")
    a = time.perf_counter()
    tw.tacaw_periodogram(ctx, ex, w.n_e, w.hop, Pacc)
    tw.tacaw_spectrum_finalize(ctx, Pacc, opts, Sq, norm)
    torch.cuda.synchronize()
    t_sp = time.perf_counter() - a
    steps = T * S
    out = dict(workload="B/N-like 40x40x50 cells (640,000 atoms), 1024^2, 100 slices, 60 keV plane "
                        "wave, 2048 snapshots streamed in chunks of %d, S(q,w) 1024 bins hop 512" % chunk,
               trajectory_s=t_gen, potentials_s=t_pot, multislice_s=t_ms, spectrum_s=t_sp,
               slice_steps=steps, multislice_slice_steps_per_s=steps / t_ms,
               total_s=t_gen + t_pot + t_ms + t_sp,
               exit_stack_GB=ex.numel() * 8 / 1e9, pass_GBps=pass_GBps)
    if keep:
        out["tensors"] = dict(xyz=xyz, V=V, exit=ex, P=Pacc, S=Sq, norm=norm, w=w, ctx=ctx,
                              last_t0=((T - 1) // chunk) * chunk)
    return out


def structure_factor_work(ws):
    """Complex multiply-adds the structure-factor contraction needs per step: for every map, the
    band-limited k points of the computed half plane (ky >= 0, the rest is the conjugate
    reflection) times the atoms of the slice."""
    total = 0.0
    for w in ws:
        kx = np.fft.fftfreq(w.nx) * w.nx / w.lx
        ky = np.fft.fftfreq(w.ny) * w.ny / w.ly
        kn = min(w.nx / (2 * w.lx), w.ny / (2 * w.ly))
        kept = (ky[:, None] ** 2 + kx[None, :] ** 2) < (w.bandlimit * kn) ** 2
        half = int(np.count_nonzero(kept[: w.ny // 2]))
        total += w.n_snap * w.n_slices * half * (w.species.shape[0] / w.n_slices)
    return total


# ------------------------------------------------------------------------------------------------
def host_info():
    """Host cores and CPU model of the machine the baselines run on."""
    model = None
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
    return dict(nproc=avail, cpu_count=os.cpu_count(), model=model)


def cpu_baseline(budget_s):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload: one 512^2
    specimen slab of 10 slices, 2 snapshots x 2 probe positions (40 slice steps, 20 potential
    maps), timed on the host cores; scaled to the workload's mix of one potential map per 64
    probe positions."""
    from threadpoolctl import threadpool_info
    from oracle import multislice as o_ms
    from oracle import potential as o_pot
    from workloads.configs import c3_specimens, make_workload
    cfg = [c for c in c3_specimens() if c["n"] == (512, 512)][0]
    w = make_workload(cfg, n_snap=2, name="cpu-sample")
    w.probe_xy = w.probe_xy[:2]
    t0 = time.perf_counter()
    V, _ = o_pot.potentials(w.positions, w.species, w.ff, w)
    t_pot = time.perf_counter() - t0
    n_maps = V.shape[0] * V.shape[1]
    t0 = time.perf_counter()
    ex = o_ms.exit_waves(V, w, w)
    t_ms = time.perf_counter() - t0
    n_steps = V.shape[0] * w.probe_xy.shape[0] * w.n_slices
    per_step = t_ms / n_steps + (t_pot / n_maps) / 64.0
    threads = sum(i.get("num_threads", 0) for i in threadpool_info() if i.get("user_api") == "blas")
    hi = host_info()
    out = {"value": 1.0 / per_step, "unit": "snapshot-slice steps/s", "cores": threads or hi["nproc"],
           "kind": "oracle",
           "sample": f"512^2 rocksalt slab, 10 slices, 2 snapshots x 2 probe positions: {n_maps} "
                     f"potential maps in {t_pot:.1f} s, {n_steps} dense-DFT slice steps in "
                     f"{t_ms:.1f} s; scaled to 1 map per 64 positions",
           "nproc": hi["nproc"], "cpu_model": hi["model"], "blas_threads": threads,
           "multislice_only_slice_steps_per_s": n_steps / t_ms,
           "wall_s": t_pot + t_ms}
    out["fft_lines"] = cpu_fft_baseline(V, w, ex)
    return out


def cpu_fft_baseline(V, w, ref):
    """A fairer CPU line than the dense-DFT oracle: the same multislice with scipy.fft (complex128
    and complex64, workers = the host's cores) on the oracle's slab (same V, probe and
    propagators), slice steps per second of the multislice alone; checked against the oracle's
    exit waves."""
    import scipy.fft as sfft
    from oracle import multislice as o_ms
    from oracle.physics import interaction_parameter
    workers = host_info()["nproc"]
    psi0 = o_ms.initial_waves(w, w)
    sigma = interaction_parameter(w.energy_ev)
    n = w.nx * w.ny
    out = {"workers": workers, "sample": "the oracle's slab: 10 slices, 2 snapshots x 2 positions, "
                                         "repeated for at least 2 s"}
    for name, cdt, rdt in (("complex128", np.complex128, np.float64), ("complex64", np.complex64, np.float32)):
        props = [o_ms.propagator(w, w.energy_ev, dz).astype(cdt) for dz in w.dz]
        trans = np.exp(1j * sigma * V).astype(cdt)
        steps, t0, exits = 0, time.perf_counter(), None
        while True:
            exits = np.empty((V.shape[0], psi0.shape[0], w.ny, w.nx), dtype=cdt)
            for t in range(V.shape[0]):
                for p in range(psi0.shape[0]):
                    psi = psi0[p].astype(cdt)
                    for s in range(V.shape[1]):
                        k = sfft.fft2(trans[t, s] * psi, workers=workers)
                        if s < V.shape[1] - 1:
                            psi = sfft.ifft2(props[s] * k, workers=workers)
                        else:
                            exits[t, p] = props[s] * k / np.sqrt(n).astype(rdt)
                    steps += V.shape[1]
            if time.perf_counter() - t0 >= 2.0:
                break
        dt = time.perf_counter() - t0
        err = float(np.linalg.norm(exits - ref) / np.linalg.norm(ref))
        out[name] = {"slice_steps_per_s": steps / dt, "rel_l2_vs_oracle": err}
    return out


def summarize_traffic(fetch_csv, write_csv, bench_json, out_json):
    """HBM traffic of the 512^2 slice-step passes from FETCH_SIZE and WRITE_SIZE counter runs (KiB
    per dispatch), each scaled by what the counter reads for the 1 GiB device-to-device copy of the
    same run (the calibration copy moves 2^30 bytes each way), per launch and as a ratio to the
    algorithmic bytes per launch that the run's own instrumented step reports (its JSON line).  The
    counter run has the benchmark's kernels, block size and streams but fewer snapshots: the
    profiler's counter collection does not survive the ~10^5 dispatches of a full-size run."""
    import csv

    def load(path, counter):
        per = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            key = (r["Dispatch_Id"], r["Kernel_Name"])
            per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
        return per

    import paper_2401_15599_amd as tw
    line = json.loads(open(bench_json).read().strip().splitlines()[-1])
    kinds = line["extra"]["kernel_ms_per_step"]
    fetch, write = load(fetch_csv, "FETCH_SIZE"), load(write_csv, "WRITE_SIZE")
    copy_f = max(v for (d, k), v in fetch.items() if "copybuffer" in k.lower())
    copy_w = max(v for (d, k), v in write.items() if "copybuffer" in k.lower())
    fs, ws = (1 << 30) / (copy_f * 1024.0), (1 << 30) / (copy_w * 1024.0)
    rec = {"kernel": "slice step passes at 512^2 (batched-uneven workload)",
           "source_sha256_16": hashlib.sha256(open(os.path.join(
               ROOT, "paper_2401_15599_amd", "csrc", "ms_kernels.hip"), "rb").read()).hexdigest()[:16],
           "slice_block_bytes": tw.SLICE_BLOCK_BYTES,
           "counter_run": line["config"]["workload"],
           "calibration": {"copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30,
                           "FETCH_SIZE_KiB": copy_f, "WRITE_SIZE_KiB": copy_w,
                           "fetch_scale": fs, "write_scale": ws}}
    for name, tag in (("row", "k_row<tacaw::Plan<512, 64"), ("col", "k_colb<tacaw::Plan<512, 64")):
        rd = [v for (d, k), v in fetch.items() if tag in k]
        wr = [v for (d, k), v in write.items() if tag in k]
        rec[f"{name}_launches"] = len(rd)
        rec[f"{name}_read_bytes_per_launch_scaled"] = sum(rd) / max(1, len(rd)) * 1024.0 * fs
        rec[f"{name}_write_bytes_per_launch_scaled"] = sum(wr) / max(1, len(wr)) * 1024.0 * ws
        rec[f"{name}_bytes_per_launch_scaled"] = (rec[f"{name}_read_bytes_per_launch_scaled"] +
                                                  rec[f"{name}_write_bytes_per_launch_scaled"])
        algo = kinds[name]["algo_bytes"] / max(1, kinds[name]["launches"])
        rec[f"{name}_algo_bytes_per_launch"] = algo
        rec[f"{name}_traffic_over_algorithmic"] = rec[f"{name}_bytes_per_launch_scaled"] / algo
    rec["commands"] = [
        "rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir> -o run -- python3 bench.py --steps 1 "
        "--warmup 0 --snapshots 32 --no-legs --no-cpu --no-check --calibrate  (> <fetch json>)",
        "rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir> -o run -- python3 bench.py --steps 1 "
        "--warmup 0 --snapshots 32 --no-legs --no-cpu --no-check --calibrate",
        "python3 bench.py --summarize-traffic <fetch csv> <write csv> <fetch json> "
        "profiles/traffic_slice_step_512.json"]
    json.dump(rec, open(out_json, "w"), indent=1)
    return rec


def traffic_record():
    """HBM traffic of the dominant kernel from the committed counter summary, if it was taken on
    the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic_slice_step_512.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = os.path.join(ROOT, "paper_2401_15599_amd", "csrc", "ms_kernels.hip")
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if rec.get("source_sha256_16") != h:
        return None
    import paper_2401_15599_amd as tw
    if rec.get("slice_block_bytes") != tw.SLICE_BLOCK_BYTES:
        return None
    return rec


# ------------------------------------------------------------------------------------------------
def profile_slice_step(args):
    """Counter-collection run: the calibration copy, then two batched multislice calls of the
    benchmark workload at 8 snapshots (512 waves of 512^2, 2 GiB per pass, well above the 256 MB
    last-level cache), with the per-launch algorithmic bytes printed for comparison."""
    import torch
    import paper_2401_15599_amd as tw
    ctx = tw.context(0)
    src = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0").fill_(1.0)   # 1 GiB
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    T = 8
    ws = make_specimens(args.specimens, T, "cuda:0")
    Vs = [torch.empty((T, w.n_slices, w.ny, w.nx), dtype=torch.float32, device="cuda:0") for w in ws]
    exits = [torch.empty((T, args.pos_chunk, w.ny, w.nx), dtype=torch.complex64, device="cuda:0")
             for w in ws]
    for w, V in zip(ws, Vs):
        tw.tacaw_build_potentials(ctx, tw.specimen_from(w), w.positions, w.species_dev, w.ff, V)
    jobs = []
    for w, V, ex in zip(ws, Vs, exits):
        b = tw.Beam(w.energy_ev, True, w.alpha_rad, 0.0, 0.0, w.probe_xy[:args.pos_chunk])
        jobs.append(tw.MsJob(tw.specimen_from(w), b, V, ex))
    tw.tacaw_multislice(ctx, jobs, mode=tw.MODE_BATCHED)
    torch.cuda.synchronize()
    tw.tacaw_set_slice_blocking(ctx, tw.SLICE_BLOCK_BYTES, 1)   # one stream: no overlap
    tw.tacaw_set_timing(ctx, True)
    tw.tacaw_multislice(ctx, jobs, mode=tw.MODE_BATCHED)
    torch.cuda.synchronize()
    out = {k: tw.tacaw_get_timing(ctx, k) for k in ("row", "col")}
    tw.tacaw_set_timing(ctx, False)
    for k, v in out.items():
        v["algo_bytes_per_launch"] = v["algo_bytes"] / max(1, v["launches"])
        v["avg_ms"] = v["total_ms"] / max(1, v["launches"])
        v["algo_GBps"] = v["algo_bytes"] / (v["total_ms"] * 1e-3) / 1e9
    print(json.dumps({"calibration_copy_bytes": 2 * (1 << 30), "slice_step": out}))


def main():
    args = parse()
    if args.summarize_traffic:
        print(json.dumps(summarize_traffic(*args.summarize_traffic), indent=1))
        return
    if args.profile_slice_step:
        profile_slice_step(args)
        return
    if args.odd_grids_only:
        import paper_2401_15599_amd as tw
        print(json.dumps({"odd_grids": odd_grid_leg(tw)}))
        return
    if args.large_only:
        import paper_2401_15599_amd as tw
        print(json.dumps({"large": large_run(tw)}))
        return
    if args.adjoint_only:
        import paper_2401_15599_amd as tw
        print(json.dumps({"adjoint": adjoint_leg(tw)}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding is a design note only)"}))
        sys.exit(2)
    import torch
    import paper_2401_15599_amd as tw

    ctx = tw.context(0)
    if args.calibrate:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0").fill_(1.0)   # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    tune = os.path.join(ROOT, "profiles", "tuning_gfx950.jsonl")
    if os.path.exists(tune):
        tw.tacaw_load_tuning(ctx, tune)
    log(f"[bench] generating {args.specimens} specimens x {args.snapshots} snapshots on the GPU")
    ws = make_specimens(args.specimens, args.snapshots, "cuda:0")
    T = args.snapshots
    for w in ws:
        w.n_e = min(256, T)
        w.hop = w.n_e
    Vs = [torch.empty((T, w.n_slices, w.ny, w.nx), dtype=torch.float32, device="cuda:0") for w in ws]
    exits = [torch.empty((T, args.pos_chunk, w.ny, w.nx), dtype=torch.complex64, device="cuda:0")
             for w in ws]
    Ps = [torch.empty((w.n_e, w.ny, w.nx), dtype=torch.float32, device="cuda:0") for w in ws]
    Ss = [torch.empty((w.n_e, w.ny, w.nx), dtype=torch.float32, device="cuda:0") for w in ws]
    slice_steps = sum(w.n_pos * T * w.n_slices for w in ws)
    log(f"[bench] {slice_steps / 1e6:.2f} M snapshot-slice steps per step; "
        f"HBM in use {torch.cuda.memory_allocated() / 2**30:.1f} GiB")
    for i in range(args.warmup):
        run_step(tw, ctx, ws, Vs, exits, Ps, Ss, args.pos_chunk)
        torch.cuda.synchronize()
        log(f"[bench] warmup {i + 1}/{args.warmup} done")
    # timed steps: the batched multislice calls replay their captured graphs
    torch.cuda.synchronize()
    ms_events = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        run_step(tw, ctx, ws, Vs, exits, Ps, Ss, args.pos_chunk, ms_events=ms_events)
        torch.cuda.synchronize()
        log(f"[bench] step {i + 1}/{args.steps} done")
    dt = time.perf_counter() - t0
    ms_graph_s = sum(a.elapsed_time(b) for a, b in ms_events) * 1e-3 / args.steps
    torch.cuda.synchronize()
    ms_step = dt / args.steps * 1e3
    value = slice_steps * args.steps / dt
    # correctness of the timed work: one wave of the last timed step against the FP64 oracle
    check = None
    if not args.no_check:
        log("[bench] oracle check of one exit wave of the timed work")
        check = inrun_oracle_check(ws, exits, args.pos_chunk)
        log(f"[bench] oracle check: rel-L2 {check['rel_l2']:.2e} ({check['oracle_s']:.1f} s)")
    # one instrumented step: every kernel bracketed by HIP events on its stream (eager launches of
    # the same kernels, grids and snapshot blocks, all on one stream so that no two launches
    # overlap), for the per-kernel durations and bandwidths
    tw.tacaw_set_slice_blocking(ctx, tw.SLICE_BLOCK_BYTES, 1)
    tw.tacaw_set_timing(ctx, True)
    torch.cuda.synchronize()
    ti = time.perf_counter()
    run_step(tw, ctx, ws, Vs, exits, Ps, Ss, args.pos_chunk)
    torch.cuda.synchronize()
    ti = time.perf_counter() - ti
    kinds = {k: tw.tacaw_get_timing(ctx, k) for k in ("row", "col", "sf", "pot_ifft", "pgram")}
    tw.tacaw_set_timing(ctx, False)
    tw.tacaw_set_slice_blocking(ctx, tw.SLICE_BLOCK_BYTES, tw.SLICE_BLOCK_STREAMS)
    # dominant kernel among the slice-step passes
    dom = max(("row", "col"), key=lambda k: kinds[k]["total_ms"])
    kd = kinds[dom]
    achieved = kd["algo_bytes"] / (kd["total_ms"] * 1e-3) / 1e9 if kd["total_ms"] > 0 else 0.0
    rec = traffic_record()
    roofline = {"bound": "hbm", "kernel": f"slice step, {dom} pass (512^2)",
                "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS,
                # counter bytes per launch: this launch's algorithmic bytes times the counter /
                # algorithmic ratio measured on the same kernels and blocks (smaller batch)
                "traffic": (rec[f"{dom}_traffic_over_algorithmic"] * kd["algo_bytes"] /
                            max(1, kd["launches"])) if rec else None,
                "traffic_note": ("FETCH_SIZE x 2 + WRITE_SIZE counter bytes over algorithmic bytes "
                                 "of this pass in a 32-snapshot run of the same kernels and blocks "
                                 "(profiles/traffic_slice_step_512.json), times this run's "
                                 "algorithmic bytes per launch") if rec else None,
                "algo_bytes_per_launch": kd["algo_bytes"] / max(1, kd["launches"]),
                "avg_launch_ms": kd["total_ms"] / max(1, kd["launches"]),
                "timing": "HIP events on the launch stream, one instrumented step after the timed "
                          "steps (eager launches of the same kernels, grids and snapshot blocks "
                          "on one stream)"}
    # the whole slice loop as timed: both passes' algorithmic bytes over the multislice calls of
    # the timed steps (graph replays, blocks overlapping on two streams)
    loop_bytes = kinds["row"]["algo_bytes"] + kinds["col"]["algo_bytes"]
    roofline["slice_loop"] = {
        "achieved": loop_bytes / ms_graph_s / 1e9 if ms_graph_s else None,
        "frac": loop_bytes / ms_graph_s / 1e9 / PEAK_HBM_GBS if ms_graph_s else None,
        "seconds_per_step": ms_graph_s, "algo_bytes_per_step": loop_bytes,
        "timing": "CUDA events on the caller's stream around every multislice call of the timed "
                  "steps"}
    breakdown = {k: {"launches": v["launches"], "ms": v["total_ms"], "algo_bytes": v["algo_bytes"],
                     "algo_GBps": (v["algo_bytes"] / (v["total_ms"] * 1e-3) / 1e9) if v["total_ms"] else None}
                 for k, v in kinds.items()}
    ms_time = kinds["row"]["total_ms"] + kinds["col"]["total_ms"]
    extra = {"multislice_only_slice_steps_per_s": slice_steps / (ms_time * 1e-3) if ms_time else None,
             "kernel_ms_per_step": breakdown,
             "instrumented_step_ms": ti * 1e3,
             "graph_replay_step_ms": ms_step,
             "inrun_oracle_check": check}
    cmacs = structure_factor_work(ws)
    if kinds["sf"]["total_ms"]:
        extra["structure_factor"] = {
            "complex_mac_per_step": cmacs,
            "fp32_equivalent_tflops": 8.0 * cmacs / (kinds["sf"]["total_ms"] * 1e-3) / 1e12,
            "note": "8 flops per complex multiply-add of the contraction over the half plane "
                    "ky >= 0 (the kernel forms them from four real sums over the quarter kx, ky >= 0 "
                    "that serve both kx signs, each product as 3 fp16 matrix-core products of "
                    "split operands)"}
    if not args.no_legs:
        log("[bench] plain vs batched leg")
        extra["plain_vs_batched"] = plain_leg(tw, ctx, ws, Vs)
        del exits, Ss, Vs, Ps, ws
        torch.cuda.empty_cache()
        if not args.no_full:
            log("[bench] the whole batched-uneven configuration (24 specimens, 3 grid classes)")
            extra["full_uneven_24"] = full_uneven_leg(tw, T=T, pos_chunk=args.pos_chunk)
            torch.cuda.empty_cache()
        log("[bench] adjoint/forward leg")
        extra["adjoint"] = adjoint_leg(tw)
        torch.cuda.empty_cache()
        log("[bench] homogeneous plane-wave leg")
        extra["plane_wave_512"] = plane_wave_leg(tw)
        extra["plane_wave_512"]["pixel_slice_steps_per_s"] = (
            extra["plane_wave_512"]["slice_steps_per_s"] * 512 * 512)
        torch.cuda.empty_cache()
        log("[bench] odd-length grid legs (560^2, 1000^2)")
        extra["odd_grids"] = odd_grid_leg(tw)
        torch.cuda.empty_cache()
        log("[bench] large configuration at full size (1024^2, 2048 snapshots, streamed)")
        extra["large_1024"] = large_run(tw)
    cpu = None
    if not args.no_cpu:
        log("[bench] CPU baselines on the host cores (FP64 oracle, scipy.fft)")
        cpu = cpu_baseline(args.cpu_budget_s)
    line = {
        "metric": "snapshot-slice steps/sec at 512^2 (batched vs plain) + adjoint/forward time ratio",
        "value": value, "unit": "snapshot-slice steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64/f32 (structure factor: fp16 x3 split operands on the matrix cores)",
        "data": "synthetic (seeded harmonic trajectories)",
        "config": {"workload": "batched-uneven 512^2 class: 8 rocksalt specimens 160x160 A, "
                               "10..80 slices, 100 keV 30 mrad probe at 8x8 positions, "
                               f"{T} snapshots at 5 fs, S(q,w) with {min(256, T)} bins",
                   "grid": 512, "specimens": args.specimens, "probe_positions": 64,
                   "snapshots": T, "slice_steps_per_step": slice_steps, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line))
    if check is not None and not check["passed"]:
        log(f"[bench] oracle check FAILED: rel-L2 {check['rel_l2']:.3e} > 1e-4")
        sys.exit(3)


if __name__ == "__main__":
    main()
