"""Throughput benchmark of the posterior-sampling sweep on one MI355X.

Workload: a 2048 x 2048 sCMOS frame, Airy PSF (NA 1.4, 0.6 um, 65 nm pixels)
sampled 31 x 31, 5000 beads + 2000 filaments on a 1..10 photon/px gradient,
per-pixel gain/offset/read-noise maps, 4 independent chains, plain sampler
(the block-series scan that the library picks by itself).  One step = one full
sweep over every pixel of every chain (mu refresh + proposals, 4 block phases,
moments and log-posterior trace).  The first --settle sweeps (default 60) are
the burn-in: they adapt the per-pixel steps toward acceptance 0.44, the
regime in which a 1000-sweep run spends nearly all of its time.  The warm-up
and the --steps timed sweeps follow, so every timed sweep runs the whole
post-burn-in path (moments included), replayed from the captured HIP graph
with profiling off; the kernel split and the roofline come from a separate
profiled pass of a few sweeps after the timed region.

Prints one JSON line: pixel-updates/s, the roofline of the dominant kernel
(the block pass, VALU-bound: its updates priced by the cost model of direct
evaluation, 18 + 4 K lane-slots per footprint term, with the work the kernel
actually executes beside it) and the FP64 CPU oracle timed on a bounded sample
of the same workload.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import re
import time
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 3.93e13 VALU lane-ops/s
# (one non-packed FP32 or FP64 add/mul/fma per lane per cycle), HBM3E 8 TB/s.
PEAK_VALU_OPS = 256 * 4 * 16 * 2.4e9
PEAK_HBM = 8.0e12
PEAK_BF16_MFMA = 2.5e15     # dense BF16 matrix-core peak
OPS_PER_TERM = 5            # per phi term: 2 multiplies, 2 FMAs, 1 tilt multiply (FP64)
OPS_PER_SERIES_EVAL = 9     # series evaluation: 7 FMAs (two-point Horner), 1 multiply, 1 add
OPS_PER_ANCHOR_TERM = 12    # per phi term of a series anchor: 2 multiplies, 5 adds, 5 multiplies (FP64)
SETUP_SLOTS, SLOTS_PER_TERM = 18, 4   # cost model of one direct footprint evaluation: 18 + 4 K slots
BYTES_PER_UPDATE = 44       # rho r/w, mu r/w, (c, a), step, (mean, M2) r/w


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = ["bdc_kernels.hip", "bdc_device.h", "bdc_kernels.h", "bdc_consts.h"]


def counter_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary of this workload (already scaled by the copy-kernel
    calibration), or None when the kernel sources changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "%s_%s.md" % (kernel, workload))
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2411_00991_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    vals = {}
    with open(path) as fh:
        for line in fh:
            m = re.match(r"^(traffic_bytes_per_launch|traffic_source_sha256):\s*(\S+)", line)
            if m:
                vals[m.group(1)] = m.group(2)
    if vals.get("traffic_source_sha256") != h.hexdigest() or "traffic_bytes_per_launch" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch"])


def cpu_baseline(fr, rho, ls, t, B, C, seed, burn_in, budget_s=15.0, threads=0, nine=False):
    """The FP64 oracle on a bounded sample: successive colour groups of block
    phase 0 (of the four- or the nine-phase scan) from the GPU's state, until
    ~budget_s of wall time, on `threads` OpenMP threads (0: all host threads)."""
    import numpy as np
    import oracle
    full = oracle.max_threads()
    oracle.set_threads(threads if threads > 0 else full)
    try:
        return _cpu_baseline(fr, rho, ls, t, B, C, seed, burn_in, budget_s, oracle, np, nine)
    finally:
        oracle.set_threads(full)


def _cpu_baseline(fr, rho, ls, t, B, C, seed, burn_in, budget_s, oracle, np, nine=False):
    g, o, s = fr.camera.maps(*fr.image.shape)
    f64 = lambda a: np.asarray(np.asarray(a, np.float32), np.float64)
    O = oracle.OracleSampler(f64(fr.image), f64(fr.psf), f64(g), f64(o), f64(s), n_chains=C, seed=seed,
                             burn_in=burn_in, schedule=oracle.SCHED_BLOCK9 if nine else oracle.SCHED_BLOCK,
                             block=B)
    O.init()
    O.set_state(rho.astype(np.float64), ls.astype(np.float64), t)
    O.run_groups(t, 0, 0, refresh=True)          # mu refresh (not timed)
    done, gi = 0, 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s and gi < O.n_groups():
        _, _, acc = O.run_groups(t, gi, gi + 1, refresh=False)
        done += int((acc != 255).sum())
        gi += 1
    el = time.perf_counter() - t0
    return {"value": done / el, "unit": "pixel-updates/s", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": "%d pixel-updates (%d colour groups of block phase 0, all %d chains) of the same "
                      "%dx%d frame from the GPU's state, %.1f s" % (done, gi, C, fr.image.shape[0],
                                                                    fr.image.shape[1], el)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--settle", type=int, default=60,
                    help="burn-in sweeps before the warm-up (step adaptation toward acceptance 0.44, no "
                         "moments); the warm-up and timed sweeps follow it, as in the post-burn-in half of a run")
    ap.add_argument("--size", type=int, default=2048)
    ap.add_argument("--chains", type=int, default=4)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--schedule", default="auto", choices=["auto", "series", "series9", "block", "chromatic"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--workload", default="dense", choices=["dense", "tiles256", "race", "unet", "rl", "prior", "lattice", "emccd"],
                    help="dense: the 2048^2 4-chain frame (default); tiles256: 256 heterogeneous tiles batched; "
                         "race: train the network on sampler-generated 256^2 crops, then plain vs learned start "
                         "on a fresh frame (--race-side) until R-hat < 1.01")
    ap.add_argument("--no-unet", action="store_true", help="skip the network throughput figures")
    ap.add_argument("--race-sweeps", type=int, default=12000, help="race: most sweeps per arm")
    ap.add_argument("--race-side", type=int, default=2048, help="race: side of the fresh frame")
    ap.add_argument("--race-check", type=int, default=250, help="race: sweeps between R-hat checks")
    ap.add_argument("--race-rhat-block", type=int, default=50, help="race: sweeps per R-hat batch")
    ap.add_argument("--race-arms", default="plain,learned",
                    help="race: plain (photon-image start), learned (network start + a block move after every "
                         "sweep), warm (network start, no block moves), rl (Richardson-Lucy start, "
                         "--race-rl-iters iterations), walk (plain start + a block walk along what the blur "
                         "removes after every sweep), dirichlet (plain start, Dirichlet-OTF prior per block)")
    ap.add_argument("--race-rl-iters", type=int, default=20, help="race: RL iterations of the rl arm's start")
    ap.add_argument("--race-walk-step", type=float, default=0.3,
                    help="race: step of the walk arm's block moves along what the blur removes")
    ap.add_argument("--race-crops", type=int, default=64, help="race: sampler-labelled training crops")
    ap.add_argument("--race-crop", type=int, default=256, help="race: side of the training crops")
    ap.add_argument("--race-psf", default="airy31", choices=["airy31", "gauss11"], help="race: PSF of frames and crops")
    ap.add_argument("--race-train-steps", type=int, default=1500, help="race: Adam steps of the network")
    ap.add_argument("--no-race", action="store_true",
                    help="dense: skip the compact plain-vs-learned race (--no-unet skips it too: it trains a network)")
    ap.add_argument("--race-seeds", default="100", help="race: comma-separated seeds of the fresh frames")
    ap.add_argument("--race-net", default="", help="race: network parameters (.npy) to load, or to save after training")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one plain device copy of this size first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the sampler shards by chain, tile or strip across GPUs, "
              "but this program runs and reports a single MI355X (use --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2411_00991_amd as bdc
    from paper_2411_00991_amd import synth

    torch.cuda.set_device(0)
    if args.calib_copy_mib:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d bytes read, %d bytes written" % (4 * n, 4 * n))
        del src, dst
    if args.workload == "tiles256":
        return bench_tiles(args, bdc, synth, np, torch)
    if args.workload == "race":
        return bench_race(args, bdc, synth, np, torch)
    if args.workload == "rl":
        return bench_rl(args, bdc, synth, np, torch)
    if args.workload == "prior":
        return bench_prior(args, bdc, synth, np, torch)
    if args.workload == "lattice":
        return bench_lattice(args, bdc, synth, np, torch)
    if args.workload == "emccd":
        return bench_emccd(args, bdc, synth, np, torch)
    if args.workload == "unet":
        u = bench_unet(bdc, np, torch)
        print(json.dumps({"metric": "U-Net BF16 TFLOP/s", "value": u["forward_2048"]["tflops"], "unit": "TFLOP/s",
                          "n_gpus": 1, "higher_is_better": True, "data": "synthetic", "dtype": "bf16",
                          "config": {"workload": "unet_l4_c32_forward2048_train8x256"}, "unet": u}), flush=True)
        return
    log("building the %dx%d frame" % (args.size, args.size))
    fr = synth.frame_dense(args.size, seed=2, n_chains=args.chains)
    H, W = fr.image.shape
    g, o, s = [np.asarray(a, np.float32) for a in fr.camera.maps(H, W)]
    C = args.chains
    burn_in, timed_from = sweep_plan(args)
    n_prof = 4
    sched = {"auto": bdc.BDC_SCHED_AUTO, "series": bdc.BDC_SCHED_BLOCK_SERIES, "block": bdc.BDC_SCHED_BLOCK,
             "series9": bdc.BDC_SCHED_BLOCK9_SERIES, "chromatic": bdc.BDC_SCHED_CHROMATIC}[args.schedule]
    S = bdc.Sampler(np.asarray(fr.psf, np.float32), g, o, s, height=H, width=W, n_chains=C, seed=2,
                    burn_in=burn_in, schedule=sched, block_size=args.block,
                    max_sweeps=timed_from + args.steps + n_prof)
    n_groups, sched_used, B = S.schedule_info()
    S.init(np.asarray(fr.image, np.float32))
    if args.settle:
        log("settling %d sweeps (the burn-in: step adaptation, no moments)" % args.settle)
        S.sweep(args.settle)
    log("warmup %d sweeps" % args.warmup)
    S.sweep(args.warmup)
    torch.cuda.synchronize()
    acc0, prop0 = S.accept_stats()
    # Timed region: exactly --steps post-burn-in sweeps replayed from the
    # captured graph (profiling off), in five segments whose rates give the
    # median beside the whole-region rate.
    segs = [args.steps // 5 + (1 if i < args.steps % 5 else 0) for i in range(5)]
    segs = [k for k in segs if k > 0]
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(len(segs) + 1)]
    log("timing %d sweeps (graph replay, %d segments)" % (args.steps, len(segs)))
    torch.cuda.synchronize()
    evs[0].record()
    for k, n in enumerate(segs):
        S.sweep(n)
        evs[k + 1].record()
    torch.cuda.synchronize()
    ms = evs[0].elapsed_time(evs[-1])
    seg_ms = [evs[k].elapsed_time(evs[k + 1]) for k in range(len(segs))]
    seg_rate = [H * W * C * n / (t / 1e3) for n, t in zip(segs, seg_ms)]
    updates = float(H * W * C * args.steps)
    value = updates / (ms / 1e3)
    acc, prop = S.accept_stats()
    acc, prop = acc - acc0, prop - prop0      # the timed sweeps

    # Separate profiled pass (kernel by kernel, HIP events on the library's
    # stream around every launch): the kernel split and the dominant kernel's
    # average launch duration for the roofline.
    log("profiled pass: %d sweeps" % n_prof)
    S.profile_read()                      # reset counters
    S.profile(True)
    S.sweep(n_prof)
    torch.cuda.synchronize()
    kms, launches, work = S.profile_read()
    S.profile(False)
    prof_updates = float(H * W * C * n_prof)
    nl = max(int(launches[1]), 1)
    pass_ms = kms[1] / nl
    terms, evals, direct, anchors, aterms, fused = [float(x) for x in work]
    series = sched_used in (bdc.BDC_SCHED_BLOCK_SERIES, bdc.BDC_SCHED_BLOCK9_SERIES)
    if series:
        # executed algorithmic work: series evaluations, direct evaluations' phi
        # terms (5 operations each; those of an accepted move's PSF-core entries,
        # a share fused / direct of them, also build the series at the new mean:
        # 12 more) and the anchors' phi terms
        ops = (OPS_PER_SERIES_EVAL * (evals - direct) + OPS_PER_TERM * terms
               + OPS_PER_ANCHOR_TERM * terms * (fused / max(direct, 1.0)) + OPS_PER_ANCHOR_TERM * aterms)
        kbar = aterms / max(anchors, 1.0)      # window length at the current state
    else:
        ops = OPS_PER_TERM * terms
        kbar = terms / max(evals, 1.0)
    executed = ops / nl / (pass_ms / 1e3)
    # algorithmic work of the updates, per the cost model of direct evaluation:
    # every footprint term with its own phi window of K terms, 18 + 4 K VALU
    # lane-slots (K = the mean window length at the current state)
    alg_ops = evals * (SETUP_SLOTS + SLOTS_PER_TERM * kbar)
    achieved = alg_ops / nl / (pass_ms / 1e3)
    kname = {bdc.BDC_SCHED_BLOCK: "k_block_phase", bdc.BDC_SCHED_BLOCK_SERIES: "k_block_series",
             bdc.BDC_SCHED_BLOCK9_SERIES: "k_wave_series"}.get(sched_used, "k_colour_pass")
    workload = "dense%d_airy%d_%dchains" % (H, int(fr.psf.shape[0]), C)
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_VALU_OPS / 1e12, "unit": "TOP/s",
            "frac": achieved / PEAK_VALU_OPS, "traffic": counter_traffic(kname, workload),
            "traffic_unit": "bytes/launch", "kernel": kname,
            "kernel_ms_avg": pass_ms, "launches": nl, "profiled_sweeps": n_prof, "phi_terms_mean": kbar,
            "footprint_evals_per_update": evals / prof_updates,
            "slots_per_update": alg_ops / prof_updates,
            "direct_evals_per_update": direct / prof_updates if series else evals / prof_updates,
            "anchors_per_update": (anchors + fused) / prof_updates,
            "executed": {"ops_per_update": ops / prof_updates, "achieved": executed / 1e12,
                         "frac": executed / PEAK_VALU_OPS},
            "hbm_alg_frac": (BYTES_PER_UPDATE * updates / (ms / 1e3)) / PEAK_HBM,
            "time_split_ms_per_sweep": {"forward_propose": kms[0] / n_prof, "passes": kms[1] / n_prof,
                                        "moments": kms[2] / n_prof}}
    rho, ls, t = S.rho()
    S.close()
    unet = None if args.no_unet else bench_unet(bdc, np, torch)
    race = None
    if not (args.no_race or args.no_unet):
        log("compact race: plain vs learned start, 128^2, Gaussian 11x11")
        race = compact_race(args, bdc, synth, np, torch)
    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle) for ~%.0f s on all host threads, then ~%.0f s on one" % (
            args.cpu_budget, args.cpu_budget / 2))
        nine = sched_used == bdc.BDC_SCHED_BLOCK9_SERIES
        cpu = cpu_baseline(fr, rho, ls, t, B, C, 2, burn_in, args.cpu_budget, nine=nine)
        one = cpu_baseline(fr, rho, ls, t, B, C, 2, burn_in, args.cpu_budget / 2, threads=1, nine=nine)
        cpu["single_thread"] = {k: one[k] for k in ("value", "cores", "sample")}
        cpu["cpu_model"] = cpu_model()
    out = {"metric": "pixel-updates/s (MCMC) at 2048^2", "value": value, "unit": "pixel-updates/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
           "data": "synthetic",
           "config": {"workload": "dense_%d_airy31_%dchains" % (H, C), "height": H, "width": W,
                      "psf_side": int(fr.psf.shape[0]), "chains": C, "burn_in": burn_in,
                      "timed_from_sweep": timed_from, "timing": "graph replay, profiling off",
                      "segments": segs, "segment_rates_median": float(np.median(seg_rate)),
                      "schedule": {bdc.BDC_SCHED_BLOCK: "block", bdc.BDC_SCHED_BLOCK_SERIES: "block_series",
                                   bdc.BDC_SCHED_BLOCK9_SERIES: "block9_series"}.get(sched_used, "chromatic"),
                      "block": B, "acceptance": float(acc.sum() / max(prop.sum(), 1))},
           "roofline": roof, "cpu_baseline": cpu, "unet": unet, "race": race}
    print(json.dumps(out), flush=True)


def sweep_plan(args):
    """(burn_in, first timed sweep index).  The settling sweeps are the burn-in
    (step adaptation toward acceptance 0.44, no moments), so every warm-up and
    timed sweep is a post-burn-in sweep of the product path: proposals, the
    block passes, the Welford and batch moments and the log-posterior trace."""
    burn_in = args.settle
    return burn_in, args.settle + args.warmup


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _timed(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def bench_unet(bdc, np, torch):
    """Matrix-core throughput of the learned network (4 levels, 32 base channels,
    random weights): inference on one 2048^2 frame and one training step
    (forward + backward + Adam) on a batch of 8 crops of 256^2."""
    from paper_2411_00991_amd import learned
    log("network throughput")
    p = learned.he_init(4, 32, seed=0)
    inf = bdc.UNet(4, 32, max_pixels=2048 * 2048)
    inf.set_params(p)
    x = torch.rand((1, 2048, 2048), device="cuda")
    out = torch.empty((1, 2048, 2048, 2), device="cuda")
    ms_f = _timed(torch, lambda: bdc.bdc_unet_forward(inf.handle, x, out), 5)
    f_f = inf.flops(1, 2048, 2048)
    inf.close()
    tr = bdc.UNet(4, 32, max_pixels=8 * 256 * 256, training=True)
    tr.set_params(p)
    xb = torch.rand((8, 256, 256), device="cuda")
    tb = torch.randn((8, 256, 256, 2), device="cuda")
    ms_t = _timed(torch, lambda: tr.train_step(xb, tb, 1e-4, want_loss=False), 10)
    f_t = 3.0 * tr.flops(8, 256, 256)          # forward + data gradient + weight gradient
    tr.close()
    return {"params": int(learned.param_count(4, 32)), "bound": "mfma", "peak_tflops": PEAK_BF16_MFMA / 1e12,
            "forward_2048": {"ms": ms_f, "tflop": f_f / 1e12, "tflops": f_f / ms_f / 1e9,
                             "frac": f_f / (ms_f / 1e3) / PEAK_BF16_MFMA},
            "train_step_8x256": {"ms": ms_t, "tflop": f_t / 1e12, "tflops": f_t / ms_t / 1e9,
                                 "frac": f_t / (ms_t / 1e3) / PEAK_BF16_MFMA}}


def bench_race(args, bdc, synth, np, torch):
    print(json.dumps(race_result(args, bdc, synth, np, torch)), flush=True)


def compact_race(args, bdc, synth, np, torch):
    """The race at a size the default run affords (about a minute): plain against
    learned start on one fresh 128^2 mixed frame with the 64^2 configuration's
    Gaussian PSF (sigma 1.5 px, 11 x 11), the network trained on 32 sampler-
    labelled 128^2 crops of the same statistics.  The full-size race is
    --workload race."""
    a = argparse.Namespace(**vars(args))
    a.race_side, a.race_crop, a.race_crops, a.race_psf = 128, 128, 32, "gauss11"
    a.race_train_steps, a.race_check, a.race_rhat_block, a.race_sweeps = 600, 50, 25, 8000
    a.race_arms, a.race_seeds, a.race_net = "plain,learned", "100", ""
    r = race_result(a, bdc, synth, np, torch)
    return {"config": r["config"], "summary": r["summary"],
            "arms": {m: {k: v for k, v in arm.items() if k != "trajectory"} for m, arm in r["race"][100].items()}}


def race_result(args, bdc, synth, np, torch):
    """Plain against learned start on fresh dense frames (4 chains, one frame per
    seed in --race-seeds, paired differences over them), each run until the
    split-R-hat criterion (99th percentile of the per-pixel map and the
    log-posterior R-hat both below 1.01) or --race-sweeps.  The network
    (4 levels, 32 base channels) is trained first on 256^2 crops with the dense
    frame's statistics, posterior moments from the batched sampler, or loaded
    from --race-net.  The learned arm starts from the network's log-normal and
    runs one block move (beta = 0.1) after every sweep; the warm arm starts
    there and runs plain sweeps; their clocks include the network's forward pass.  Reports sweeps and wall seconds to the criterion
    and the error of the window posterior mean against the ground truth."""
    from paper_2411_00991_amd import learned
    side = args.race_side
    n_crop, crop = args.race_crops, args.race_crop
    psf = synth.gaussian_psf(1.5, 11) if args.race_psf == "gauss11" else None      # None: Airy 31 x 31
    psf_name = "gauss11" if psf is not None else "airy31"
    info, t_train, loss, params, net_src = None, None, None, None, None
    arms = args.race_arms.split(",")
    uses_net = "learned" in arms or "warm" in arms
    if uses_net and args.race_net and os.path.exists(args.race_net):
        params = np.load(args.race_net)
        net_src = "loaded"
        log("network parameters from %s" % args.race_net)
    elif uses_net:
        log("training data: %d crops %d^2, 300 sweeps each" % (n_crop, crop))
        crops = [synth.frame_mixed(crop, 2000 + i, psf=psf) for i in range(n_crop)]
        X, T, info = learned.generate(crops, sweeps=300, burn_in=150, log=log)
        log("training")
        net = bdc.UNet(4, 32, max_pixels=8 * crop * crop, training=True)
        net.set_params(learned.he_init(4, 32, seed=0))
        t0 = time.perf_counter()
        losses = learned.train(net, X, T, steps=args.race_train_steps, batch=8, lr=1e-3, log=log, log_every=250)
        torch.cuda.synchronize()
        t_train, loss = time.perf_counter() - t0, losses[-1]
        params = net.get_params()
        net_src = "trained"
        net.close()
        del X, T
        if args.race_net:
            np.save(args.race_net, params)
    infer = None
    if params is not None:
        infer = bdc.UNet(4, 32, max_pixels=side * side)
        infer.set_params(params)
    rb, check = args.race_rhat_block, args.race_check

    def run_arm(fr, mode, seed):
        kw = dict(prior_kind=bdc.BDC_PRIOR_DIRICHLET, schedule=bdc.BDC_SCHED_BLOCK) if mode == "dirichlet" else {}
        sp = learned.make_sampler(fr, 4, seed, burn_in=10 ** 6, max_sweeps=args.race_sweeps + check, rhat_block=rb,
                                  **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if mode in ("learned", "warm"):
            sp.init_learned(infer)
            sp.set_block_beta(0.1)
        if mode == "rl":
            sp.init_rl(args.race_rl_iters)
        if mode == "walk":
            sp.set_block_walk(args.race_walk_step)
        pts = []
        done, hit = 0, None
        while done < args.race_sweeps and hit is None:
            if mode in ("learned", "walk"):
                for _ in range(check):
                    sp.sweep(1)
                    sp.block_move(1)
            else:
                sp.sweep(check)
            done += check
            if done < 4 * rb:
                continue
            p99, rlp = sp.rhat()
            wm = sp.window_mean()
            sec = time.perf_counter() - t0
            err = float(np.sqrt(np.mean((wm - fr.truth) ** 2)))
            pt = {"sweeps": done, "seconds": sec, "rhat_p99": float(p99), "rhat_logpost": float(rlp),
                  "rmse_vs_truth": err}
            if p99 < 1.01 and rlp < 1.01:
                hit = pt
            if hit is not None or done % 500 == 0:
                pts.append(pt)
                log("  seed %d %s %d sweeps %.1f s: R-hat p99 %.4f logpost %.4f rmse %.3f" % (
                    seed, mode, done, sec, p99, rlp, err))
        arm = {"converged": hit is not None, "trajectory": pts}
        if hit is not None:
            arm.update({"seconds_to_rhat": hit["seconds"], "sweeps_to_rhat": hit["sweeps"],
                        "rmse_at_rhat": hit["rmse_vs_truth"]})
        if mode in ("learned", "walk"):
            a, pr = sp.block_stats()
            arm["block_acceptance"] = a / max(pr, 1)
        sp.close()
        return arm

    seeds = [int(v) for v in args.race_seeds.split(",")]
    frames = {}
    for seed in seeds:
        fr = (synth.frame_dense(2048, seed=seed, n_chains=4) if side == 2048 and psf is None
              else synth.frame_mixed(side, seed, psf=psf, n_chains=4))
        frames[seed] = {}
        for mode in arms:
            log("race: frame seed %d, %s start" % (seed, mode))
            frames[seed][mode] = run_arm(fr, mode, seed)
    if infer is not None:
        infer.close()
    # paired comparison with the plain arm over the frames where both reached the criterion
    summary = {}
    for key in ("seconds_to_rhat", "sweeps_to_rhat", "rmse_at_rhat"):
        for m in arms:
            v = [frames[k][m][key] for k in seeds if frames[k][m].get("converged")]
            if v:
                summary["%s_%s_mean" % (m, key)] = float(np.mean(v))
        for m in arms:
            both = [k for k in seeds if m != "plain" and "plain" in frames[k]
                    and frames[k]["plain"].get("converged") and frames[k][m].get("converged")]
            if len(both) >= 2:
                d = np.array([frames[k][m][key] - frames[k]["plain"][key] for k in both])
                summary["%s_minus_plain_%s" % (m, key)] = {"mean": float(d.mean()),
                                                           "se": float(d.std(ddof=1) / np.sqrt(len(d))), "n": len(d)}
    main = next((a for a in ("learned", "walk", "rl", "warm", "dirichlet") if a in arms), None)
    lrn = [frames[k][main]["seconds_to_rhat"] for k in seeds if main and frames[k][main].get("converged")]
    kind = "dense" if side == 2048 else "mixed"
    out = {"metric": "time to R-hat < 1.01, plain vs learned start",
           "value": float(np.mean(lrn)) if lrn and len(lrn) == len(seeds) else None,
           "unit": "s", "n_gpus": 1, "higher_is_better": False, "data": "synthetic", "dtype": "f32",
           "vs_baseline": None,
           "config": {"workload": "race_%s_%d_%s_4chains_seeds%s" % (kind, side, psf_name,
                                                                    "-".join(map(str, seeds))),
                      "rhat_block": rb, "check_every": check, "max_sweeps": args.race_sweeps,
                      "network": net_src, "train_crops": n_crop, "crop": crop, "train_steps": args.race_train_steps,
                      "train_data_s": info["seconds"] if info else None, "train_s": t_train, "train_loss": loss},
           "summary": summary, "race": frames}
    return out


def _psnr(est, truth):
    import numpy as np
    mse = float(np.mean((est - truth) ** 2))
    return 10.0 * math.log10(float(truth.max()) ** 2 / mse), math.sqrt(mse)


def bench_rl(args, bdc, synth, np, torch):
    """Richardson-Lucy against the sampler on a spoke target (the analogue of
    the paper's simulated comparison): RMSE and PSNR of RL after k iterations,
    and of the posterior mean after N post-burn-in sweeps (4 chains pooled),
    with the flat prior and with the Dirichlet-OTF prior per chunk."""
    fr = synth.frame_spokes(128, seed=10)
    H, W = fr.image.shape
    one = np.float32

    def sampler(**kw):
        sp = bdc.Sampler(np.asarray(fr.psf, np.float32), one(1.0), one(0.0), one(0.25), height=H, width=W,
                         n_chains=4, seed=10, burn_in=500, max_sweeps=4096, **kw)
        sp.init(np.asarray(fr.image, np.float32))
        return sp

    def mc_curve_of(sp):
        sp.sweep(500)
        curve, done = [], 0
        t0 = time.perf_counter()
        for n in (2, 10, 100, 1000, 3000):
            sp.sweep(n - done)
            done = n
            m, _, _ = sp.moments()
            p, e = _psnr(m.astype(np.float64), fr.truth)
            a, pr = sp.accept_stats()
            curve.append({"sweeps": n, "psnr_db": p, "rmse": e, "seconds": time.perf_counter() - t0,
                          "acceptance": float(a.sum() / max(pr.sum(), 1))})
        return curve

    S = sampler()
    rl_curve = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in (1, 2, 5, 10, 20, 50, 100, 200, 500):
        p, e = _psnr(S.richardson_lucy(k).astype(np.float64), fr.truth)
        rl_curve.append({"iterations": k, "psnr_db": p, "rmse": e})
    t_rl = time.perf_counter() - t0
    mc_curve = mc_curve_of(S)
    S.close()
    # the same with the paper's Dirichlet-OTF prior, read per PSF-sized chunk
    log("sampler with the Dirichlet-OTF prior")
    S = sampler(prior_kind=bdc.BDC_PRIOR_DIRICHLET, schedule=bdc.BDC_SCHED_BLOCK, block_size=int(fr.psf.shape[0]))
    dir_curve = mc_curve_of(S)
    S.close()
    best = max(rl_curve, key=lambda r: r["psnr_db"])
    out = {"metric": "posterior-mean PSNR vs Richardson-Lucy, spoke target", "value": mc_curve[-1]["psnr_db"],
           "unit": "dB", "n_gpus": 1, "higher_is_better": True, "data": "synthetic", "dtype": "f32+f64",
           "vs_baseline": None,
           "config": {"workload": "spokes128_gauss_na1.3_510nm_4chains", "rl_best_iterations": best["iterations"],
                      "rl_best_psnr_db": best["psnr_db"], "rl_seconds": t_rl},
           "rl": rl_curve, "sampler": mc_curve, "sampler_dirichlet": dir_curve}
    print(json.dumps(out), flush=True)


def bench_prior(args, bdc, synth, np, torch):
    """Sweep throughput on the 2048^2 frame with the Dirichlet-OTF prior per
    31 x 31 chunk (block-phase scan), beside the same scan with the flat prior."""
    fr = synth.frame_dense(args.size, seed=2, n_chains=args.chains)
    H, W = fr.image.shape
    g, o, s = [np.asarray(a, np.float32) for a in fr.camera.maps(H, W)]
    res = {}
    for name, kind in (("flat", bdc.BDC_PRIOR_FLAT), ("dirichlet", bdc.BDC_PRIOR_DIRICHLET)):
        S = bdc.Sampler(np.asarray(fr.psf, np.float32), g, o, s, height=H, width=W, n_chains=args.chains, seed=2,
                        burn_in=args.settle, schedule=bdc.BDC_SCHED_BLOCK, block_size=int(fr.psf.shape[0]),
                        prior_kind=kind, max_sweeps=args.settle + args.warmup + args.steps + 4)
        S.init(np.asarray(fr.image, np.float32))
        S.sweep(args.settle + args.warmup)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        S.sweep(args.steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        a, p = S.accept_stats()
        res[name] = {"ms_per_sweep": ms / args.steps, "pixel_updates_per_s": H * W * args.chains * args.steps / (ms / 1e3),
                     "acceptance": float(a.sum() / max(p.sum(), 1))}
        log("%s prior: %.1f ms per sweep" % (name, ms / args.steps))
        S.close()
    out = {"metric": "pixel-updates/s with the Dirichlet-OTF prior (block-phase scan)",
           "value": res["dirichlet"]["pixel_updates_per_s"], "unit": "pixel-updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "data": "synthetic",
           "dtype": "f32+f64", "vs_baseline": None,
           "config": {"workload": "dense_%d_airy31_%dchains_dirichlet_chunks31" % (H, args.chains)}, "runs": res}
    print(json.dumps(out), flush=True)


def bench_lattice(args, bdc, synth, np, torch):
    """Sweep throughput with the object on a lattice twice as fine as the camera:
    the dense 2048^2 object (photons per cell a quarter of the pixel-lattice
    frame's, so the pixel fluxes match) imaged onto 1024^2 pixels through the
    same Airy PSF sampled at 32.5 nm (63 x 63 cells, pixel footprints 33 x 33),
    per-pixel camera maps, block-phase scan over cell phases."""
    from scipy import signal
    k = 2
    n_obj = args.size
    H = W = n_obj // k
    fr = synth.frame_dense(n_obj, seed=2, n_chains=args.chains)
    psf = synth.airy_psf(1.4, 0.6, 0.0325, 63)
    truth = np.asarray(fr.truth, np.float64) / (k * k)
    mu = signal.fftconvolve(truth, psf / psf.sum(), mode="same").reshape(H, k, W, k).sum(axis=(1, 3))
    rng = np.random.default_rng(5)
    cam = synth.scmos_maps(rng, H, W)
    g, o, s = [np.asarray(a, np.float32) for a in cam.maps(H, W)]
    img = (g * rng.poisson(np.clip(mu, 0.0, None)) + o + s * rng.standard_normal((H, W))).astype(np.float32)
    settle = min(args.settle, 10)
    S = bdc.Sampler(np.asarray(psf, np.float32), g, o, s, height=H, width=W, n_chains=args.chains, seed=2,
                    burn_in=settle, object_sub=k, schedule=bdc.BDC_SCHED_BLOCK,
                    max_sweeps=settle + args.warmup + args.steps + 4)
    n_groups, _, B = S.schedule_info()
    S.init(img)
    log("object lattice %dx%d on %dx%d pixels: %d sweeps to settle" % (n_obj, n_obj, H, W, settle))
    S.sweep(settle + args.warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    S.sweep(args.steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    a, p = S.accept_stats()
    S.close()
    cells = n_obj * n_obj * args.chains
    out = {"metric": "cell-updates/s on an object lattice twice as fine as the camera (block-phase scan)",
           "value": cells * args.steps / (ms / 1e3), "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms / args.steps, "higher_is_better": True, "data": "synthetic",
           "dtype": "f32+f64", "vs_baseline": None,
           "config": {"workload": "dense_obj%d_px%d_airy63_k2_%dchains" % (n_obj, H, args.chains), "object_sub": k,
                      "block": B, "groups_per_sweep": n_groups, "burn_in": settle,
                      "acceptance": float(a.sum() / max(p.sum(), 1))}}
    print(json.dumps(out), flush=True)


def bench_emccd(args, bdc, synth, np, torch):
    """Sweep throughput with the EMCCD reading: the dense 2048^2 object and Airy
    31 x 31 PSF imaged through Poisson photoelectrons, the Gamma multiplication
    stage and read noise on the zero-photon reading (per-pixel maps), block-phase
    scan (the closed-form footprint term with log I_1)."""
    fr = synth.frame_dense(args.size, seed=2, n_chains=args.chains)
    H, W = fr.image.shape
    rng = np.random.default_rng(6)
    img = np.asarray(synth.simulate_frame_emccd(fr.truth, fr.psf, fr.camera, rng), np.float32)
    g, o, s = [np.asarray(a, np.float32) for a in fr.camera.maps(H, W)]
    settle = min(args.settle, 20)
    S = bdc.Sampler(np.asarray(fr.psf, np.float32), g, o, s, height=H, width=W, n_chains=args.chains, seed=2,
                    burn_in=settle, camera=bdc.BDC_CAMERA_EMCCD, max_sweeps=settle + args.warmup + args.steps + 4)
    _, sched, B = S.schedule_info()
    S.init(img)
    log("EMCCD frame %dx%d: %d sweeps to settle" % (H, W, settle))
    S.sweep(settle + args.warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    S.sweep(args.steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    a, p = S.accept_stats()
    S.close()
    out = {"metric": "pixel-updates/s with the EMCCD reading (block-phase scan)",
           "value": H * W * args.chains * args.steps / (ms / 1e3), "unit": "pixel-updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms / args.steps, "higher_is_better": True,
           "data": "synthetic", "dtype": "f32+f64", "vs_baseline": None,
           "config": {"workload": "dense_%d_airy31_%dchains_emccd" % (H, args.chains), "schedule": int(sched),
                      "block": B, "burn_in": settle, "acceptance": float(a.sum() / max(p.sum(), 1))}}
    print(json.dumps(out), flush=True)


def bench_tiles(args, bdc, synth, np, torch):
    """256 tiles, sides U{64..512}, Gaussian/Airy PSFs 9x9..31x31, per-tile photon
    budgets 10..1000, sCMOS maps; one batch, scans chosen by the cached autotuner."""
    from paper_2411_00991_amd import autotune
    log("building 256 tiles")
    tiles = synth.tile_batch(256, seed=3)
    samplers, sides = [], []
    for i, fr in enumerate(tiles):
        H, W = fr.image.shape
        g, o, s = [np.asarray(a, np.float32) for a in fr.camera.maps(H, W)]
        sp = bdc.Sampler(np.asarray(fr.psf, np.float32), g, o, s, height=H, width=W, n_chains=1,
                         seed=fr.seed, burn_in=100, max_sweeps=8)
        sp.init(np.asarray(fr.image, np.float32))
        samplers.append(sp)
        sides.append(int(fr.psf.shape[0]))
    log("autotuning the scan per tile class")
    chosen = autotune.tune_tiles(samplers, sides, sweeps=1)
    batch = bdc.Batch(samplers)
    n_items, grid, lds = batch.info()
    log("warmup %d batched sweeps (%d items/sweep)" % (args.warmup, n_items))
    batch.sweep(args.warmup)
    batch.check()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    batch.sweep(args.steps)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    area = float(sum(sp.H * sp.W for sp in samplers))
    value = area * args.steps / (ms / 1e3)
    out = {"metric": "pixel-updates/s (MCMC), 256-tile batch", "value": value, "unit": "pixel-updates/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
           "data": "synthetic",
           "config": {"workload": "tiles256_side64-512_psf9-31", "tiles": len(samplers), "pixels": int(area),
                      "items_per_sweep": n_items, "classes": len(chosen)},
           "roofline": None, "cpu_baseline": None}
    batch.close()
    for sp in samplers:
        sp.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
