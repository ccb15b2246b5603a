"""Benchmark: multislice forward + adjoint (one gradient evaluation) on one MI355X.

One step = the whole hot path over the 512 x 512 x 2048 bars-on-substrate
workload (5 nm slices, 0.1 nm wavelength): slice pack (every slice's
transmission T - 1, tiled), forward sweep with checkpoints every 32 slices,
far-field intensity, amplitude loss and its derivative, far-field adjoint,
and the checkpointed adjoint sweep producing dL/d delta, dL/d beta and
dL/d probe.  Inputs are resident in HBM before timing starts.

Prints one JSON line.  `value` is voxel-slice-steps per second of the
forward + adjoint step (Ny * Nz * Ns / step time).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3  # MI355X FP32 vector
# VALU issue ceiling without packed FP32: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# lane-instructions per second (a wave64 instruction is 64 lane-instructions, 4 cycles)
VALU_PEAK_TLANES = 256 * 4 * 16 * 2.4e9 / 1e12
FWD_BYTES = 24.0          # per voxel-slice: delta + beta (8 B) + field read and write (16 B)


def fwd_flops_per_voxel_slice(n):
    # one line pass: four n-point complex FFTs (5 n log2 n flops each), two
    # propagator multiplies and the transmission multiply (6 flops each); the
    # transmission's exponential is not counted
    return 4 * 5 * math.log2(n) + 3 * 6


def grad_bytes_per_voxel_slice(k):
    # forward 24 + 8/k (checkpoint stores) ; segment recompute 24 + 8 (store psi_s) ;
    # reverse 8 (delta, beta) + 8 (psi_s) + 16 (cotangent read + write) + 8 (two gradients)
    return 24.0 + 8.0 / k + 32.0 + 40.0


KERNEL_SOURCES = ("paper_2212_01253_amd/csrc/msl_device.hpp", "paper_2212_01253_amd/csrc/msl_passes.hpp",
                  "paper_2212_01253_amd/csrc/msl.hip")
TRAFFIC_PROFILE = "profiles/k_pass_512_bars_512x512x2048.md"


def profile_figures():
    """Figures of the forward middle pass from the committed rocprofv3 summary, or {} when the
    kernel sources changed since it was taken: HBM bytes per launch (FETCH_SIZE + WRITE_SIZE,
    calibrated), kernel microseconds per launch, executed VALU instructions per wavefront
    (SQ_INSTS_VALU / SQ_WAVES) of the row and the column pass, wavefronts per launch."""
    import hashlib
    import re
    try:
        text = open(os.path.join(ROOT, TRAFFIC_PROFILE)).read()
        h = hashlib.sha256()
        for p in KERNEL_SOURCES:
            h.update(open(os.path.join(ROOT, p), "rb").read())
    except OSError:
        return {}
    sha = re.search(r"sources_sha256: ([0-9a-f]+)", text)
    if not sha or sha.group(1) != h.hexdigest():
        return {}
    out = {}
    for key, conv in (("traffic_bytes_per_launch", int), ("kernel_us_per_launch", float),
                      ("valu_per_wave_row", float), ("valu_per_wave_column", float), ("waves_per_launch", int)):
        m = re.search(key + r": ([0-9.]+)", text)
        if m:
            out[key] = conv(m.group(1))
    return out


def cpu_baseline(w, meas):
    """The FP64 oracle (forward, far field, loss, adjoint with every field kept) timed on this
    host: the full throughput workload (all slices) is the reported value; beside it the parity
    workload in full, one gradient of the gradient workload, and single-thread runs."""
    import numpy as np
    from oracle import msl_oracle as O
    from paper_2212_01253_amd import synth

    def timed(g, d, b, m):
        t0 = time.perf_counter()
        O.loss_and_gradient(g, d, b, m)
        dt = time.perf_counter() - t0
        vs = g.ny * g.nz * g.n_slices
        return {"voxel_slices": vs, "seconds": dt, "value": vs / dt, "threads": O.WORKERS}

    legs = {}
    g = w.geom
    legs["throughput_full"] = timed(g, w.delta, w.beta, meas)
    p1 = synth.parity_small(0)
    m1 = synth.random_measured_amplitude(p1.geom.ny, p1.geom.nz, 78, 1.0)
    legs["parity_full"] = timed(p1.geom, p1.delta, p1.beta, m1)
    r4 = synth.recon_256()
    m4 = synth.random_measured_amplitude(r4.geom.ny, r4.geom.nz, 79, 1.0)
    legs["gradient_workload_one_gradient"] = timed(r4.geom, r4.delta, r4.beta, m4)
    keep = O.WORKERS
    try:
        O.WORKERS = 1
        legs["parity_full_1_thread"] = timed(p1.geom, p1.delta, p1.beta, m1)
        g64 = synth.Geometry(**{**g.as_dict(), "n_slices": 64})
        legs["throughput_64_slices_1_thread"] = timed(g64, w.delta[:64], w.beta[:64], meas)
    finally:
        O.WORKERS = keep
    full = legs["throughput_full"]
    return {"value": full["value"], "unit": "voxel-slice-steps/s", "cores": O.WORKERS, "kind": "oracle",
            "sample": f"FP64 oracle forward + far field + loss + adjoint (all fields kept) on the whole "
                      f"{g.ny}x{g.nz}x{g.n_slices} workload: {full['seconds']:.2f} s; SciPy FFTs on "
                      f"{O.WORKERS} threads, NumPy elementwise work on one",
            "cpu": _cpu_model(), "legs": legs}


def recon_leg():
    """Seconds from data on the GPU to the first ADAM iterate at or below 1.1 x the loss of the
    ground truth, on the 256x256x1024 gradient workload, from the plain random initialisation."""
    from paper_2212_01253_amd import recon, synth
    p = recon.make_problem()
    init = synth.random_init(p.region, 4244)
    adam = recon.Adam()
    L_truth, res = recon.seconds_to_threshold(p, init, adam=adam)
    n_it = len(res.losses) - 1
    g, r = p.geom, p.region
    return {"secs_to_threshold": res.secs_to_threshold, "iterations": res.iters_to_threshold,
            "ms_per_iteration": 1e3 * res.times[-1] / max(1, n_it), "loss_truth": L_truth,
            "threshold": res.threshold, "loss_init": res.losses[0], "loss_final": res.losses[-1],
            "init": "plain: delta ~ U[0, 3e-5) on the box", "adam_lr": adam.lr,
            "workload": f"recon_{g.ny}x{g.nz}x{g.n_slices}: box {r['ns']}x{r['ny']}x{r['nz']} "
                        f"(slices x rows x columns), beta = delta/20, 1e6 photons, checkpoints every 32"}


def batch_leg(n_inst, steps=3, autotune=True):
    """Batched forward (msl_forward_batch) over the batched workload: instances seeded 1000 + i,
    grids 128..1024, 256..4096 slices, per-instance wavelength and incidence; far field included.
    As the workload is specified: the launch shape picked by msl_autotune_batch first (untimed;
    the previous tuning is restored afterwards), and the call captured once in a HIP graph whose
    replays are timed (every replay's output is the eager call's, bit for bit; checked here on the
    last replay)."""
    import numpy as np
    import torch
    from paper_2212_01253_amd import msl, synth
    stacks = synth.batch_workload(n_inst)
    items = []
    for cs in stacks:
        g = cs.geom
        items.append({"geom": g, "pool_delta": torch.from_numpy(cs.pool_delta).cuda(),
                      "pool_beta": torch.from_numpy(cs.pool_beta).cuda(),
                      "slice_index": torch.from_numpy(cs.index.astype(np.int32)).cuda(),
                      "field": torch.empty((g.ny, g.nz), dtype=torch.complex64, device="cuda"),
                      "intensity": torch.empty((g.ny, g.nz), dtype=torch.float32, device="cuda")})
    ws = msl.batch_workspace(items)
    before = msl.get_tuning()
    tuning = None
    if autotune:
        tuning, _ = msl.autotune_batch(items, ws, reps=1)
    msl.forward_batch(items, ws)
    torch.cuda.synchronize()
    eager = [it["intensity"].cpu().numpy().copy() for it in items]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            msl.forward_batch(items, ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    same = all(np.array_equal(it["intensity"].cpu().numpy(), r) for it, r in zip(items, eager))
    del graph
    used = tuning or msl.get_tuning()
    msl.restore_tuning(before)
    vs = sum(cs.geom.ny * cs.geom.nz * cs.geom.n_slices for cs in stacks)
    grids = {}
    for cs in stacks:
        grids[cs.geom.ny] = grids.get(cs.geom.ny, 0) + 1
    return {"value": vs / (ms / 1e3), "unit": "voxel-slice-steps/s", "ms": ms, "instances": n_inst,
            "voxel_slices": vs, "achieved_GBs": vs * FWD_BYTES / (ms / 1e3) / 1e9,
            "frac": vs * FWD_BYTES / (ms / 1e3) / 1e9 / HBM_PEAK_GBS,
            "pool_slices": int(sum(cs.pool_delta.shape[0] for cs in stacks)),
            "instances_per_grid": grids, "tuning": used, "autotuned": bool(autotune),
            "hip_graph": True, "graph_replay_equals_eager": bool(same),
            "workload": "batched forward + far field: instances seeded 1000+i, grids {128,256,512,1024}^2, "
                        "256..4096 slices of 5 nm, wavelength U[0.08, 0.15] nm, incidence U[0.05, 0.5] deg"}


def learned_leg():
    """Learned initialiser (U-Net, bfloat16 matrix cores): trained for one epoch over its 50,000
    model samples (not timed), then the reconstruction of the same workload as recon_leg from its
    start, timed from data on the GPU: inference in a batch of 64 images (this one and 63 held-out
    ones), the error judge, refinement watched for stalls with the plain start as fallback.  The
    learned arm is reported at its own refinement step and at the plain arm's step."""
    from paper_2212_01253_amd import learned, recon, synth
    net, info = learned.train_initialiser()
    comp = info.pop("companions")
    p = recon.make_problem()
    init = synth.random_init(p.region, 4244)
    out = dict(info)
    for key, lr in (("", recon.REFINE_LR), ("at_plain_lr_", None)):
        run = recon.seconds_to_threshold_learned(p, net, init, refine_lr=lr, companions=comp, batch=64)
        out.update({key + "secs_to_threshold": run.result.secs_to_threshold,
                    key + "iterations": run.result.iters_to_threshold,
                    key + "start": run.start, key + "learned_iters": run.learned_iters})
        if not key:
            out.update({"adam_lr_refine": recon.REFINE_LR, "loss_learned_start": run.loss_learned_start,
                        "loss_plain_start": run.loss_plain_start, "inference_batch": 64})
    out["adam_lr_plain"] = recon.Adam().lr
    return out


def roofline(pass_bytes, launch_s, traffic, prof, ny, nz, pass_gbs, pass_tflops, prof_us):
    """Roofline of the forward middle pass against both of its ceilings: HBM bandwidth (its
    algorithmic bytes at 8 TB/s) and VALU issue (its executed lane-instructions at the unpacked
    FP32 rate).  `bound` names the ceiling that allows less, i.e. whose floor time is longer."""
    hbm = {"achieved": pass_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": pass_gbs / HBM_PEAK_GBS,
           "floor_us": pass_bytes / (HBM_PEAK_GBS * 1e9) * 1e6}
    roof = {"bound": "hbm", "achieved": pass_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": pass_gbs / HBM_PEAK_GBS, "traffic": (traffic / launch_s / 1e9) if traffic else None,
            "kernel": "k_pass<512,*,1> forward line pass (propagate, transmit, propagate)",
            "bytes_per_launch": pass_bytes, "us_per_launch": launch_s * 1e6, "traffic_bytes_per_launch": traffic,
            "rocprof_kernel_us": prof_us, "hbm": hbm,
            "flops_per_launch": fwd_flops_per_voxel_slice(nz) * ny * nz, "achieved_TFLOPs": pass_tflops,
            "fp32_frac": pass_tflops / FP32_PEAK_TFLOPS, "valu": None}
    vr, vc, waves = prof.get("valu_per_wave_row"), prof.get("valu_per_wave_column"), prof.get("waves_per_launch")
    if vr and vc and waves:
        per_wave = 0.5 * (vr + vc)   # the sweep alternates row and column passes
        lanes = per_wave * waves * 64
        achieved = lanes / launch_s / 1e12
        roof["valu"] = {"instr_per_wave_row": vr, "instr_per_wave_column": vc, "waves_per_launch": waves,
                        "lane_instr_per_launch": lanes, "achieved": achieved, "peak": VALU_PEAK_TLANES,
                        "unit": "Tlane-instr/s", "frac": achieved / VALU_PEAK_TLANES,
                        "floor_us": lanes / (VALU_PEAK_TLANES * 1e12) * 1e6}
        if roof["valu"]["floor_us"] > hbm["floor_us"]:
            roof.update({"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TLANES, "unit": "Tlane-instr/s",
                         "frac": achieved / VALU_PEAK_TLANES})
    return roof


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--ckpt-every", type=int, default=32)
    ap.add_argument("--schedule", type=int, default=0, help="0 auto, 1 per-pass launches, 2 persistent")
    ap.add_argument("--slices", type=int, default=2048)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-recon", action="store_true", help="skip the reconstruction seconds-to-loss leg")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-initialiser leg")
    ap.add_argument("--no-every-slice", action="store_true",
                    help="skip the extra timing with a checkpoint at every slice (no recompute)")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the single-instance launch shape with the library's autotuner before the timed "
                         "runs (the batched leg autotunes unless --no-batch-autotune)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run eight plain 2 MiB device-to-device copies (the reference kernel that "
                         "calibrates the FETCH_SIZE / WRITE_SIZE counters of a profile)")
    ap.add_argument("--no-batch-autotune", action="store_true",
                    help="time the batched forward at the default launch shape instead of the autotuner's")
    ap.add_argument("--batch", type=int, default=96, metavar="N",
                    help="also time the batched forward over N instances of the batched workload (96 = full, 0 = skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the multislice recurrence is sequential over slices and "
              f"the library has no multi-GPU path); got --gpus {args.gpus}", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2212_01253_amd import msl, synth

    w = synth.throughput_512(n_slices=args.slices)
    g = w.geom
    ny, nz, ns = g.ny, g.nz, g.n_slices
    k = args.ckpt_every
    meas = synth.random_measured_amplitude(ny, nz, 77, 1.0)
    print(f"# workload {w.name}: alpha {math.degrees(g.alpha_i_rad):.4f} deg", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        src = torch.ones(1 << 18, dtype=torch.float64, device=dev)   # 2 MiB
        dst = torch.empty_like(src)
        for _ in range(8):
            dst.copy_(src)
        torch.cuda.synchronize()
    msl.set_schedule(args.schedule)
    D = torch.from_numpy(w.delta).to(dev)
    B = torch.from_numpy(w.beta).to(dev)
    Mm = torch.from_numpy(meas).to(dev)
    ws = msl.workspace(g, k, dev)
    if args.autotune:
        print("# autotuning the launch shape ...", file=sys.stderr, flush=True)
        msl.autotune_forward(g, D, B, ws=ws, reps=3)
    field = torch.empty((ny, nz), dtype=torch.complex64, device=dev)
    ck = torch.empty((msl.checkpoint_count(g, k), ny, nz), dtype=torch.complex64, device=dev)
    gd = torch.empty_like(D)
    gb = torch.empty_like(B)
    I = torch.empty((ny, nz), dtype=torch.float32, device=dev)
    gpsi = torch.empty((ny, nz), dtype=torch.complex64, device=dev)

    def step(ev=None):
        if ev:
            ev[0].record()
        msl.pack_slices(g, D, B, ws)
        if ev:
            ev[1].record()
        msl.forward(g, D, B, None, k, ws=ws, out=field, ckpt=ck, reuse_pack=True)
        if ev:
            ev[2].record()
        msl.far_field(g, field, ws=ws, out=I)
        _, gI = msl.amp_loss(g, I, Mm, ws=ws)
        msl.far_field_adjoint(g, field, gI, ws=ws, out=gpsi)
        if ev:
            ev[3].record()
        msl.adjoint(g, D, B, ck, k, gpsi, ws=ws, gd=gd, gb=gb, want_probe=True, reuse_pack=True)
        if ev:
            ev[4].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"# warmup done", file=sys.stderr, flush=True)

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(args.steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record()
    for i in range(args.steps):
        step(evs[i])
    t_end.record()
    torch.cuda.synchronize()
    total_ms = t_start.elapsed_time(t_end)
    ms = total_ms / args.steps
    pack_ms = [e[0].elapsed_time(e[1]) for e in evs]
    fwd_ms = [e[1].elapsed_time(e[2]) for e in evs]
    mid_ms = [e[2].elapsed_time(e[3]) for e in evs]
    adj_ms = [e[3].elapsed_time(e[4]) for e in evs]
    step_ms = [e[0].elapsed_time(e[4]) for e in evs]
    vs = ny * nz * ns
    value = vs / (ms / 1e3)
    bpv = grad_bytes_per_voxel_slice(k)
    achieved = vs * bpv / (ms / 1e3) / 1e9
    fwd_med = float(np.median(fwd_ms))
    # the forward region holds the line passes only (plus three table kernels
    # and the probe, a few microseconds): Ns + 1 launches back to back, so the
    # per-launch time is kernel duration plus the dispatch gap between launches
    pass_bytes = (FWD_BYTES + 8.0 / k) * ny * nz
    launch_s = fwd_med / 1e3 / (ns + 1)
    pass_gbs = pass_bytes / launch_s / 1e9
    pass_tflops = fwd_flops_per_voxel_slice(nz) * ny * nz / launch_s / 1e12
    prof = profile_figures()
    traffic, prof_us = prof.get("traffic_bytes_per_launch"), prof.get("kernel_us_per_launch")
    fwd_path_ms = float(np.median([a + b + c for a, b, c in zip(pack_ms, fwd_ms, mid_ms)]))
    print(f"# step {ms:.3f} ms: pack {np.median(pack_ms):.3f} ms, forward {fwd_med:.3f} ms, "
          f"far field+loss+seed {np.median(mid_ms):.3f} ms, adjoint {np.median(adj_ms):.3f} ms",
          file=sys.stderr, flush=True)

    out = {
        "metric": "multislice voxel-slice-steps/s fwd+adj (c64)",
        "value": value,
        "unit": "voxel-slice-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": w.name, "grid": [ny, nz], "n_slices": ns, "dx_nm": g.dx_nm,
                   "wavelength_nm": g.wavelength_nm, "alpha_deg": math.degrees(g.alpha_i_rad),
                   "propagator": "paraxial", "ckpt_every": k, "seed": w.seed,
                   "schedule": ["auto", "per_pass", "persistent"][args.schedule]},
        # dominant kernel: the forward middle line pass (also the recompute's);
        # per launch = forward time / launches, i.e. kernel plus dispatch gap
        "roofline": roofline(pass_bytes, launch_s, traffic, prof, ny, nz, pass_gbs, pass_tflops, prof_us),
        "step": {"bytes_per_voxel_slice": bpv, "achieved_GBs": achieved, "frac": achieved / HBM_PEAK_GBS,
                 "ms_p10": float(np.percentile(step_ms, 10)), "ms_p50": float(np.median(step_ms)),
                 "ms_p90": float(np.percentile(step_ms, 90)),
                 "pack_ms": float(np.median(pack_ms)), "forward_ms": fwd_med, "adjoint_ms": float(np.median(adj_ms)),
                 "far_field_loss_seed_ms": float(np.median(mid_ms)), "tuning": msl.get_tuning()},
        # forward path alone (pack, forward sweep, far field, loss): Ny Nz Ns / time
        "forward_throughput": {"value": vs / (fwd_path_ms / 1e3), "unit": "voxel-slice-steps/s",
                               "ms": fwd_path_ms},
    }
    if not args.no_every_slice and k != 1:
        # the same step with a checkpoint at every slice: the adjoint reads the stored
        # fields and skips the recompute, at Ns Ny Nz complex values of checkpoint memory
        del ck
        torch.cuda.empty_cache()
        ws1 = msl.workspace(g, 1, dev)
        ck1 = torch.empty((msl.checkpoint_count(g, 1), ny, nz), dtype=torch.complex64, device=dev)

        def step1():
            msl.pack_slices(g, D, B, ws1)
            msl.forward(g, D, B, None, 1, ws=ws1, out=field, ckpt=ck1, reuse_pack=True)
            msl.far_field(g, field, ws=ws1, out=I)
            _, gI1 = msl.amp_loss(g, I, Mm, ws=ws1)
            msl.far_field_adjoint(g, field, gI1, ws=ws1, out=gpsi)
            msl.adjoint(g, D, B, ck1, 1, gpsi, ws=ws1, gd=gd, gb=gb, want_probe=True, reuse_pack=True)

        for _ in range(args.warmup):
            step1()
        torch.cuda.synchronize()
        t_start.record()
        for _ in range(args.steps):
            step1()
        t_end.record()
        torch.cuda.synchronize()
        ms1 = t_start.elapsed_time(t_end) / args.steps
        out["every_slice_checkpointed"] = {"ckpt_every": 1, "ms_per_step": ms1, "value": vs / (ms1 / 1e3),
                                           "checkpoint_bytes": ck1.numel() * 8}
        print(f"# checkpoint at every slice: {ms1:.3f} ms/step", file=sys.stderr, flush=True)
        del ck1, ws1
        torch.cuda.empty_cache()
    if args.batch:
        print(f"# batched forward ({args.batch} instances) ...", file=sys.stderr, flush=True)
        out["batch"] = batch_leg(args.batch, autotune=not args.no_batch_autotune)
    if not args.no_recon:
        print("# reconstruction (plain init) ...", file=sys.stderr, flush=True)
        out["recon"] = recon_leg()
        if not args.no_learned:
            print("# learned initialiser: training, then reconstruction from its start ...", file=sys.stderr,
                  flush=True)
            try:
                out["recon"]["learned"] = learned_leg()
            except Exception as e:   # report, keep the line
                out["recon"]["learned"] = {"error": repr(e)}
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, meas)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
