"""Throughput of the COLA PM step on one MI355X.

Workload: 256^3 particles, 768^3 PM mesh (3x the particle grid), 600 Mpc/h
box, flat LCDM Omega_m = 0.27, BBKS P(k) with sigma_8 = 0.8, Gaussian
white-noise initial conditions (GPU Philox, seed 2) displaced by 2LPT,
10 COLA steps uniform in a from 0.02 to 1.  A "step" is one cola_step: tile
sort, deterministic CIC deposit, r2c FFT, Green's function x ik and the
inverse FFTs of the three force components, CIC readout fused with the
kick/drift.

Timed region: K consecutive steps of the 10-step schedule (K <= 10) after a
fresh initial condition, inputs resident in HBM, bracketed by
torch.cuda.synchronize().  Then, each in its own pass: the adjoint of the
same K steps (fwd_adjoint: each adjoint step recomputes its forces;
fwd_adjoint_kept: the forward steps store them, one force slot per step,
where the slots fit in HBM), the 96-mock ensemble batched and one by one
(batched), and the library's per-stage HIP event timers, which give the
dominant kernel's achieved bandwidth against the 8 TB/s HBM peak (roofline;
`traffic` comes from the committed counter summary while its kernel source
is unchanged), followed by the particle velocities at the final position
time with their redshift-space displacement (velocity: whole call with its
force pipeline, and the velocity kernel against its algorithmic bytes), the
snapshot and velocity-spectra calls, and the friends-of-friends groups (fof).  The FP64 CPU oracle is timed on one step of the same
workload on the host cores (cpu_baseline).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def stage_bytes(np_side: int, nm: int) -> dict:
    """Algorithmic HBM bytes per launch of each stage (what the method must move)."""
    n_p = np_side ** 3
    M = nm ** 3
    R = 4 * M                               # real float32 mesh
    C = 8 * nm * nm * (nm // 2 + 1)         # complex half mesh
    return {
        "sort": 32 * n_p,                   # read d (12), write+read key/rank (16), write perm (4)
        "deposit": 16 * n_p + R,            # read perm + d, write delta
        "fft_z": R + C,                     # real in, half spectrum out
        "fft_y": 2 * C,
        "fft_x_green": 3 * C,               # 1 read, 2 writes (IDFT_x of i k_x phi and of phi)
        "ifft_y": 2 * C,                    # g_x: read + write
        "ifft_y_grad": 3 * C,               # IDFT_x[phi]: 1 read, 2 writes (g_y, g_z)
        "ifft_z": 3 * (C + R),              # three meshes, half spectrum in, real out
        "kick_drift": 72 * n_p + 3 * 4 * min(M, 8 * n_p),  # state r/w + CIC gathers
    }


# Counter-measured HBM bytes per launch (rocprofv3 FETCH_SIZE / WRITE_SIZE,
# scaled by a plain copy of known size) for the production workload, with the
# sha256 of the kernel sources they were taken on.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_256p_768m.txt")
STAGE_SOURCES = {
    "sort": ["k_sort.hip"], "deposit": ["k_deposit.hip"], "fft_z": ["k_fft.hip"],
    "fft_y": ["k_fft.hip"], "fft_x_green": ["k_fft.hip"], "ifft_y": ["k_fft.hip"],
    "ifft_z": ["k_fft.hip"], "ifft_y_grad": ["k_fft.hip"], "kick_drift": ["k_particles.hip"],
}


def velocity_leg(sim, cfg, reps=3):
    """cola_velocity at the final state (a_v != a_x, so the call runs the force
    pipeline, then the velocity kernel with a redshift-space output): whole-call
    time and the kernel's own time from the stage timers (HIP events on the
    library's stream) against its algorithmic bytes."""
    import torch
    vel, sdisp = sim.particles(), sim.particles()
    sim.velocity(vel, rsd_axis=2, sdisp=sdisp)
    torch.cuda.synchronize()
    sim.stage_times()
    t0 = time.perf_counter()
    for _ in range(reps):
        sim.velocity(vel, rsd_axis=2, sdisp=sdisp)
    torch.cuda.synchronize()
    ms_call = (time.perf_counter() - t0) / reps * 1e3
    ms, cnt = sim.stage_times()["velocity"]
    ms_k = ms / max(cnt, 1)
    n_p, M = cfg.np_side ** 3, cfg.nmesh ** 3
    nbytes = 72 * n_p + 12 * min(M, 8 * n_p)   # state reads 48, outputs 24, CIC gathers
    # a snapshot half way through a following step, and the velocity spectra
    st = sim.get_state(which=())
    a1 = st["a_x"] + 0.098
    sim.snapshot(a1, st["a_x"] + 0.049)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sim.snapshot(a1, st["a_x"] + 0.049)
    torch.cuda.synchronize()
    ms_snap = (time.perf_counter() - t0) / reps * 1e3
    import numpy as np
    edges = np.linspace(2 * np.pi / cfg.box, np.pi * cfg.nmesh / cfg.box, 41)
    sim.pk_velocity(edges, axis=2)
    t0 = time.perf_counter()
    for _ in range(reps):
        sim.pk_velocity(edges, axis=2)
    ms_pkv = (time.perf_counter() - t0) / reps * 1e3
    return {"ms_call": round(ms_call, 3), "ms_kernel": round(ms_k, 4), "bytes_alg": nbytes,
            "GB/s": round(nbytes / (ms_k * 1e-3) / 1e9, 1),
            "ms_snapshot_call": round(ms_snap, 3), "ms_pk_velocity_call": round(ms_pkv, 3),
            "note": "velocity at the position time plus the redshift-space displacement (axis 2); "
                    "each call includes the force pipeline at the current positions; pk_velocity "
                    "adds the weighted deposit, 2 FFTs and 40-bin spectra (synchronous)"}


def fof_leg(sim, reps=3):
    """cola_fof (b = 0.2 of the mean separation) at the final positions: time per
    call (the call synchronises) and the groups of at least 32 particles."""
    import torch
    lab = sim.fof(0.2)
    t0 = time.perf_counter()
    for _ in range(reps):
        sim.fof(0.2, out=lab)
    ms = (time.perf_counter() - t0) / reps * 1e3
    sizes = torch.bincount(lab.long())
    big = sizes >= 32
    vel = sim.velocity()
    sim.fof_halos(lab, vel, min_members=32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        cat = sim.fof_halos(lab, vel, min_members=32)
    ms_cat = (time.perf_counter() - t0) / reps * 1e3
    return {"ms_call": round(ms, 3), "ms_catalogue_call": round(ms_cat, 3), "halos": int(cat["root"].numel()),
            "b_frac": 0.2, "groups_ge_32": int(big.sum()),
            "frac_in_groups_ge_32": round(float(sizes[big].sum()) / lab.numel(), 4),
            "largest": int(sizes.max())}


def measured_traffic(stage, workload):
    """HBM bytes per launch of a stage from the committed counter summary, or
    None when there is none for this workload or the kernel source changed."""
    import hashlib
    if workload != "production" or not os.path.exists(TRAFFIC_FILE):
        return None
    sha, traffic = {}, {}
    for line in open(TRAFFIC_FILE):
        f = line.split()
        if len(f) == 3 and f[0] == "sha256":
            sha[f[1]] = f[2]
        elif len(f) >= 3 and f[0] == "traffic":
            traffic[f[1]] = int(f[2])
    if stage not in traffic:
        return None
    csrc = os.path.join(ROOT, "paper_1507_05329_amd", "csrc")
    for name in STAGE_SOURCES.get(stage, []) + ["cola_device.h"]:
        h = hashlib.sha256(open(os.path.join(csrc, name), "rb").read()).hexdigest()
        if sha.get(name) != h:
            return None
    return traffic[stage]


def batch_leg(steps, table, dev):
    """The 96-mock uneven ensemble (32 x 48^3/96^3, 32 x 64^3/128^3,
    32 x 96^3/192^3 particles/mesh, boxes 150/200/300 Mpc/h, distinct seeds):
    K batched steps (one graph per step) against the same mocks stepped one
    by one with plain contexts."""
    import torch
    from paper_1507_05329_amd.inputs import batch_configs, step_edges
    from paper_1507_05329_amd.sim import ColaBatch, ColaSim
    cfgs = batch_configs()
    e = step_edges()
    n_part = sum(c.n_particles for c in cfgs)
    b = ColaBatch([dict(np=c.np_side, nmesh=c.nmesh, box=c.box) for c in cfgs], device=dev)
    for m, c in zip(b.mocks, cfgs):
        m.init_2lpt(c.seed, *table)
    b.step(e[0], e[1])                      # warm-up; captures the graph
    for m, c in zip(b.mocks, cfgs):
        m.init_2lpt(c.seed, *table)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        b.step(e[i], e[i + 1])
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    b.close()
    del b
    sims = {}
    t_seq = 0.0
    for c in cfgs:
        key = (c.np_side, c.nmesh, c.box)
        if key not in sims:
            sims[key] = ColaSim(c.np_side, c.nmesh, c.box, device=dev)
            sims[key].init_2lpt(c.seed, *table)
            sims[key].step(e[0], e[1])      # warm-up of this size
        s = sims[key]
        s.init_2lpt(c.seed, *table)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            s.step(e[i], e[i + 1])
        torch.cuda.synchronize()
        t_seq += time.perf_counter() - t0
    for s in sims.values():
        s.close()
    return {"workload": "96 mocks: 32 x 48^3/96^3 (150 Mpc/h), 32 x 64^3/128^3 (200), "
                        "32 x 96^3/192^3 (300), distinct seeds",
            "mocks": len(cfgs), "particles": n_part, "steps": steps,
            "value": n_part * steps / t_batch, "unit": "particle-updates/s",
            "ms_per_step": t_batch / steps * 1e3,
            "sequential_value": n_part * steps / t_seq,
            "sequential_ms_per_step": t_seq / steps * 1e3,
            "speedup": t_seq / t_batch}


def adjoint_leg(sim, cfg, table, e, steps):
    """Average adjoint step (ms): reverse the K steps from their stored starts."""
    import torch
    sim.init_2lpt(cfg.seed, *table)
    starts = []
    for i in range(steps):
        st = sim.get_state()
        starts.append((st["disp"], st["a_v"]))
        sim.step(e[i], e[i + 1])
    dbar = torch.randn_like(starts[0][0])
    vbar = torch.zeros_like(dbar)
    p1b, p2b = torch.zeros_like(dbar), torch.zeros_like(dbar)
    sim.step_adjoint(e[steps - 1], e[steps], starts[-1][1], starts[-1][0], dbar, vbar, p1b, p2b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in reversed(range(steps)):
        sim.step_adjoint(e[i], e[i + 1], starts[i][1], starts[i][0], dbar, vbar, p1b, p2b)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3


def kept_leg(sim, cfg, table, e, steps):
    """Store instead of recompute: the K forward steps keep their force
    meshes (cola_step_keep, one slot per step) and the adjoint reads them
    (cola_step_adjoint_kept).  Returns (ms per forward step, ms per adjoint
    step, GB of slots), or None when the slots do not fit in free HBM."""
    import torch
    slots = [sim.force_slot()]
    per = slots[0].numel() * 4
    free, _ = torch.cuda.mem_get_info()
    if (steps - 1) * per > 0.8 * free:
        return None
    slots += [sim.force_slot() for _ in range(steps - 1)]
    sim.init_2lpt(cfg.seed, *table)
    starts = []
    torch.cuda.synchronize()
    t_fwd = 0.0
    for i in range(steps):
        st = sim.get_state()
        starts.append((st["disp"], st["a_v"]))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step_keep(e[i], e[i + 1], slots[i])
        torch.cuda.synchronize()
        t_fwd += time.perf_counter() - t0
    dbar = torch.randn_like(starts[0][0])
    vbar = torch.zeros_like(dbar)
    p1b, p2b = torch.zeros_like(dbar), torch.zeros_like(dbar)
    sim.step_adjoint(e[steps - 1], e[steps], starts[-1][1], starts[-1][0], dbar, vbar, p1b, p2b,
                     slot=slots[-1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in reversed(range(steps)):
        sim.step_adjoint(e[i], e[i + 1], starts[i][1], starts[i][0], dbar, vbar, p1b, p2b, slot=slots[i])
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    gb = steps * per / 1e9
    del slots
    torch.cuda.empty_cache()
    return t_fwd / steps * 1e3, t_adj / steps * 1e3, gb


def cpu_baseline(cfg, table, seed):
    """One oracle step of the same workload on the host (FP64, NumPy/SciPy)."""
    from oracle import cola
    from paper_1507_05329_amd.inputs import white_noise, step_edges
    cores = len(os.sched_getaffinity(0))
    w = white_noise(seed, cfg.np_side)
    st = cola.init_state(w, cfg.box, cfg.nmesh, *table)
    e = step_edges()
    t0 = time.perf_counter()
    cola.step(st, e[1])
    dt = time.perf_counter() - t0
    return {"value": cfg.n_particles / dt, "unit": "particle-updates/s", "cores": cores,
            "kind": "oracle",
            "sample": f"one FP64 oracle COLA step (a {e[0]:.3f}->{e[1]:.3f}) of the full "
                      f"{cfg.np_side}^3/{cfg.nmesh}^3 workload, {dt:.1f} s, scipy.fft workers={cores}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="production")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-ensemble leg")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint leg")
    ap.add_argument("--no-velocity", action="store_true", help="skip the velocity / redshift-space leg")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a device-to-device copy of this many MiB (for HBM counter "
                         "calibration under rocprofv3) and exit")
    args = ap.parse_args()
    if args.copy_calibration_mib:
        import torch
        n = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_mib": args.copy_calibration_mib, "launches": 3}))
        return
    if args.gpus != 1:
        print("bench.py: the library runs one context per GPU and this benchmark measures one GPU; "
              "multi-GPU runs are not supported (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    if not (1 <= args.steps <= 10) or not (0 <= args.warmup <= 10):
        print("bench.py: --steps and --warmup must lie in [1, 10] and [0, 10] "
              "(the workload is a 10-step run)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1507_05329_amd import _lib
    from paper_1507_05329_amd.inputs import CONFIGS, bbks_table, step_edges
    from paper_1507_05329_amd.sim import ColaSim

    cfg = CONFIGS[args.config]
    table = bbks_table(cfg.omega_m, cfg.h, cfg.n_s, cfg.sigma8)
    e = step_edges(cfg.a_init, cfg.a_final, cfg.nstep)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    sim = ColaSim(cfg.np_side, cfg.nmesh, cfg.box, omega_m=cfg.omega_m, n_lpt=cfg.n_lpt,
                  a_init=cfg.a_init, device=dev)
    # warm-up (also first-touch of the workspace and code objects)
    sim.init_2lpt(cfg.seed, *table)
    for i in range(args.warmup):
        sim.step(e[i], e[i + 1])
    sim.init_2lpt(cfg.seed, *table)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        sim.step(e[i], e[i + 1])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = dt / args.steps * 1e3
    value = cfg.n_particles * args.steps / dt

    # adjoint: reverse the same K steps from their stored start positions
    ms_adj = kept = None
    if not args.no_adjoint:
        ms_adj = adjoint_leg(sim, cfg, table, e, args.steps)
        kept = kept_leg(sim, cfg, table, e, args.steps)
    sim.close()
    del sim

    # per-stage timing pass (HIP events on the library's stream)
    simt = ColaSim(cfg.np_side, cfg.nmesh, cfg.box, omega_m=cfg.omega_m, n_lpt=cfg.n_lpt,
                   a_init=cfg.a_init, device=dev, flags=_lib.COLA_F_STAGE_TIMERS)
    simt.init_2lpt(cfg.seed, *table)
    simt.step(e[0], e[1])
    simt.stage_times()
    for i in range(1, args.steps if args.steps > 1 else 2):
        simt.step(e[i], e[i + 1])
    st = simt.stage_times()
    snapshot = None if args.no_velocity else velocity_leg(simt, cfg)
    halos = None if args.no_velocity else fof_leg(simt)
    simt.close()
    sb = stage_bytes(cfg.np_side, cfg.nmesh)
    stages = {}
    for name, (ms, cnt) in st.items():
        if cnt == 0:
            continue
        avg = ms / cnt
        stages[name] = {"ms": round(avg, 4), "GB/s": round(sb[name] / (avg * 1e-3) / 1e9, 1)}
    dom = max(stages, key=lambda n: stages[n]["ms"])
    dom_gbs = sb[dom] / (stages[dom]["ms"] * 1e-3) / 1e9
    step_bytes = sum(sb.values())
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(dom_gbs, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(dom_gbs / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(dom, args.config),
                "bytes_alg": sb[dom],
                "step_bytes_alg": step_bytes,
                "step_frac": round(step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

    batched = None
    if not args.no_batch:
        batched = batch_leg(args.steps, bbks_table(), dev)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(cfg, table, cfg.seed)

    out = {
        "metric": "particle-updates/s per COLA PM step (fwd; fwd+adjoint in fwd_adjoint)",
        "value": value,
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (BBKS Gaussian random field, GPU Philox seed %d)" % cfg.seed,
        "config": {"workload": cfg.name, "np": cfg.np_side, "nmesh": cfg.nmesh, "box": cfg.box,
                   "nstep": cfg.nstep, "a": [cfg.a_init, cfg.a_final]},
        "fwd_adjoint": None if ms_adj is None else {
            "value": cfg.n_particles / ((ms_step + ms_adj) * 1e-3), "unit": "particle-updates/s",
            "ms_adjoint_step": ms_adj, "adjoint_over_forward": ms_adj / ms_step},
        "fwd_adjoint_kept": None if kept is None else {
            "value": cfg.n_particles / ((kept[0] + kept[1]) * 1e-3), "unit": "particle-updates/s",
            "ms_forward_step": kept[0], "ms_adjoint_step": kept[1], "slots_GB": kept[2],
            "note": "forward steps keep their force meshes (one slot per step); the adjoint reads them"},
        "batched": batched,
        "velocity": snapshot,
        "fof": halos,
        "stages": stages,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
